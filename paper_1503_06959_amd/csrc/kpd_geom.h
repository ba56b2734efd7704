// Cell and octave geometry shared by the host library and the kernels.
//
// Coordinates follow the paper's frame I_n of size N_x x N_y (Sec. 3) and its
// N_r x N_c bin grid (Sec. 3.2): level-0 column X lies in cell column
// floor(X * N_c / W), so cell column j spans [ceil(j*W/N_c), ceil((j+1)*W/N_c)).
// A level-o pixel x belongs to the cell of its footprint start x << o, so the
// level-o columns of cell column j are [ceil(X0 / 2^o), ceil(X1 / 2^o)).
#pragma once

#include <stdint.h>

#include "../../include/kpd.h"

#if defined(__HIPCC__)
#define KPD_HD __host__ __device__ inline
#else
#define KPD_HD inline
#endif

namespace kpd {

// Detection keeps 3 pixels away from every level border (the ring radius).
constexpr int kRingR = 3;

struct Box {
    int x0, x1, y0, y1;  // half-open
};

KPD_HD bool box_empty(const Box& b) { return b.x0 >= b.x1 || b.y0 >= b.y1; }
KPD_HD int box_w(const Box& b) { return b.x1 - b.x0; }
KPD_HD int box_h(const Box& b) { return b.y1 - b.y0; }
KPD_HD int imin(int a, int b) { return a < b ? a : b; }
KPD_HD int imax(int a, int b) { return a > b ? a : b; }

KPD_HD int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
KPD_HD int shr_ceil(int a, int o) { return (a + (1 << o) - 1) >> o; }

// Level-0 span [a, b) of cell index j of n along an axis of length len.
KPD_HD void cell_span(int j, int n, int len, int* a, int* b)
{
    *a = ceil_div((int64_t)j * len, n);
    *b = ceil_div((int64_t)(j + 1) * len, n);
}

// Level-0 rectangle of cell c (row-major over grid_cols x grid_rows).
KPD_HD Box cell_rect(int c, int W, int H, int nc, int nr)
{
    Box r;
    cell_span(c % nc, nc, W, &r.x0, &r.x1);
    cell_span(c / nc, nr, H, &r.y0, &r.y1);
    return r;
}

// Pixels of level o (size w_o x h_o) whose keypoint decision belongs to the
// cell with level-0 rectangle r: the cell's level-o columns and rows clipped
// to the detectable interior [3, w_o - 3) x [3, h_o - 3).
KPD_HD Box decision_box(const Box& r, int o, int wo, int ho)
{
    Box d;
    d.x0 = imax(shr_ceil(r.x0, o), kRingR);
    d.x1 = imin(shr_ceil(r.x1, o), wo - kRingR);
    d.y0 = imax(shr_ceil(r.y0, o), kRingR);
    d.y1 = imin(shr_ceil(r.y1, o), ho - kRingR);
    return d;
}

KPD_HD void box_union(Box* acc, bool* have, const Box& b)
{
    if (box_empty(b)) return;
    if (!*have) { *acc = b; *have = true; return; }
    acc->x0 = imin(acc->x0, b.x0); acc->x1 = imax(acc->x1, b.x1);
    acc->y0 = imin(acc->y0, b.y0); acc->y1 = imax(acc->y1, b.y1);
}

// Score region of level o for one cell: every level-o pixel whose score the
// scale-space suppression of the cell's decisions can read. Decisions at
// level o read their 8 in-plane neighbours; decisions at level o+1 read the
// finer 4x4 block [2X-1, 2X+2]; decisions at level o-1 read the coarser
// pixels X with 2X-1 <= x <= 2X+2, i.e. [(x-1)>>1, (x+1)>>1]. The result is
// clipped to the detectable interior, outside which every score is 0.
KPD_HD Box score_box(const Box* dec, int o, int O, int wo, int ho)
{
    Box acc = {0, 0, 0, 0};
    bool have = false;
    const Box& d = dec[o];
    if (!box_empty(d)) box_union(&acc, &have, Box{d.x0 - 1, d.x1 + 1, d.y0 - 1, d.y1 + 1});
    if (o + 1 < O && !box_empty(dec[o + 1])) {
        const Box& u = dec[o + 1];
        box_union(&acc, &have, Box{2 * u.x0 - 1, 2 * u.x1 + 1, 2 * u.y0 - 1, 2 * u.y1 + 1});
    }
    if (o > 0 && !box_empty(dec[o - 1])) {
        const Box& f = dec[o - 1];
        box_union(&acc, &have, Box{(f.x0 - 1) >> 1, ((f.x1 - 1 + 1) >> 1) + 1,
                                   (f.y0 - 1) >> 1, ((f.y1 - 1 + 1) >> 1) + 1});
    }
    if (!have) return Box{0, 0, 0, 0};
    acc.x0 = imax(acc.x0, kRingR); acc.x1 = imin(acc.x1, wo - kRingR);
    acc.y0 = imax(acc.y0, kRingR); acc.y1 = imin(acc.y1, ho - kRingR);
    if (box_empty(acc)) return Box{0, 0, 0, 0};
    return acc;
}

// Largest number of keypoints a cell can hold: two keypoints of one level are
// never 8-neighbours, so each 2x2 block of a decision box holds at most one.
KPD_HD int decision_capacity(const Box& d)
{
    if (box_empty(d)) return 0;
    return ((box_w(d) + 1) >> 1) * ((box_h(d) + 1) >> 1);
}

KPD_HD int round_up(int v, int a) { return (v + a - 1) / a * a; }

// Bytes of LDS the detection kernel needs for one cell: one uint16 score map
// per level over its score box (each padded to 4 bytes), plus one uint8
// pixel tile reused across levels covering the largest score box plus the
// 3-pixel ring apron.
KPD_HD int cell_lds_bytes(const Box* sbox, int O)
{
    int scores = 0, tile = 0;
    for (int o = 0; o < O; ++o) {
        if (box_empty(sbox[o])) continue;
        scores += round_up(box_w(sbox[o]) * box_h(sbox[o]) * 2, 4);
        int t = (box_w(sbox[o]) + 2 * kRingR) * (box_h(sbox[o]) + 2 * kRingR);
        tile = imax(tile, t);
    }
    return scores + round_up(tile, 4);
}

}  // namespace kpd
