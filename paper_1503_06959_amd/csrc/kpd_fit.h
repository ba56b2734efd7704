// The exact least-squares quadratic fit of a 3 x 3 score patch shared by
// the refinement passes (Sec. 2's sub-pixel interpolation).
#pragma once

#include <hip/hip_runtime.h>

namespace kpd {

struct Fit {
    double u, v, m;
};

// S[3(i+1) + (j+1)] is the score at x offset i, y offset j. With exact
// integer sums A, B (first differences), Cx, Cy (second differences), E
// (cross term) and K0 (centre stencil), the maximum is at (U/D, V/D),
// clamped to a pixel, when D = 16 Cx Cy - 9 E^2 > 0 and Cx < 0, else at the
// centre; m is the fit's value there, in IEEE double steps in a fixed
// order with no fused multiply-add.
__device__ inline Fit fit_patch(const int* S)
{
#pragma clang fp contract(off)
    long long sx[3], sy[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        sx[k] = (long long)S[3 * k] + S[3 * k + 1] + S[3 * k + 2];
        sy[k] = (long long)S[k] + S[3 + k] + S[6 + k];
    }
    auto P = [&](int i, int j) -> long long { return S[3 * (i + 1) + (j + 1)]; };
    const long long A = sx[2] - sx[0], B = sy[2] - sy[0];
    const long long Cx = sx[2] + sx[0] - 2 * sx[1], Cy = sy[2] + sy[0] - 2 * sy[1];
    const long long E = P(1, 1) - P(1, -1) - P(-1, 1) + P(-1, -1);
    const long long K0 = 5 * P(0, 0) + 2 * (P(0, -1) + P(-1, 0) + P(1, 0) + P(0, 1)) -
                         (P(-1, -1) + P(1, -1) + P(-1, 1) + P(1, 1));
    const long long D = 16 * Cx * Cy - 9 * E * E;
    long long U = 0, V = 0, Dn = 1;
    if (D > 0 && Cx < 0) {
        U = min(max(6 * E * B - 8 * Cy * A, -D), D);
        V = min(max(6 * E * A - 8 * Cx * B, -D), D);
        Dn = D;
    }
    Fit r;
    r.u = (double)U / (double)Dn;
    r.v = (double)V / (double)Dn;
    double f = (double)K0 / 9.0;
    f = f + ((double)A / 6.0) * r.u;
    f = f + ((double)B / 6.0) * r.v;
    f = f + (((double)Cx / 6.0) * r.u) * r.u;
    f = f + (((double)E / 4.0) * r.u) * r.v;
    f = f + (((double)Cy / 6.0) * r.v) * r.v;
    r.m = f;
    return r;
}

}  // namespace kpd
