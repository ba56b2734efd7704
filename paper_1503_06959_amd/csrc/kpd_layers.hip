// Detection over octaves and intra-octaves (Sec. 2's scale space with the
// layers between the octaves) for one frame: the layers, the FAST score of
// every layer pixel, suppression among same-layer and adjacent-layer
// pixels whose level-0 footprints meet, and the keypoints in (layer, y, x)
// order by a block-count / scan / write pass over the flattened layers.
#include <hip/hip_runtime.h>

#include "kpd_fit.h"
#include "kpd_layers.h"

namespace kpd {
namespace {

__constant__ int8_t kLayRingDx[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
__constant__ int8_t kLayRingDy[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};

// Two levels of a chain per launch. k_lay_quad: a thread per 2x2 quad of
// level d1 (each pixel the 2x2 mean of src, round half up, for the quad
// pixels inside d1) and, when the quad lies inside d2's reach, the d2 pixel
// that is the mean of the quad; d2 may be absent (w2 = 0). Frame z of a
// chunk (blockIdx.z) reads src + z * sstep and writes d1, d2 + z * dstep;
// with a slot table, slot z's (skipped when inactive), whose frame is the
// source when from_frame is set.
__device__ __forceinline__ int mean4(int a, int b, int c, int d) { return (a + b + c + d + 2) >> 2; }

__global__ __launch_bounds__(256) void k_lay_quad(const uint8_t* src, int spitch, uint8_t* d1, int w1, int h1,
                                                  uint8_t* d2, int w2, int h2, size_t sstep, size_t dstep,
                                                  const LbSlot* slots, int from_frame)
{
    const int qx = blockIdx.x * 16 + (threadIdx.x & 15), qy = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (2 * qx >= w1 || 2 * qy >= h1) return;
    if (slots && !slots[blockIdx.z].active) return;
    if (slots && from_frame) {
        src = slots[blockIdx.z].cur;
        spitch = slots[blockIdx.z].cur_pitch;
    } else {
        src += blockIdx.z * sstep;
    }
    d1 += blockIdx.z * dstep;
    if (w2 > 0) d2 += blockIdx.z * dstep;
    int v[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int x = 2 * qx + i, y = 2 * qy + j;
            if (x < w1 && y < h1) {
                const uint8_t* p = src + (size_t)(2 * y) * spitch + 2 * x;
                v[j][i] = mean4(p[0], p[1], p[spitch], p[spitch + 1]);
                d1[(size_t)y * w1 + x] = (uint8_t)v[j][i];
            }
        }
    if (qx < w2 && qy < h2) d2[(size_t)qy * w2 + qx] = (uint8_t)mean4(v[0][0], v[0][1], v[1][0], v[1][1]);
}

// The 1.5x downsampling and the halving after it: a thread per whole 3x3
// block (a, b) of the frame writes the block's 2x2 outputs of d_0 (output
// (2a+p, 2b+q) = the rounded mean over the 1.5 x 1.5 area it covers,
// weights (2, 1, 0) or (0, 1, 2) along each axis, over 9) and, when d_1 is
// built here, their mean (d_1 has exactly one pixel per block). Frames of a
// chunk as in k_lay_quad.
__global__ __launch_bounds__(256) void k_lay_third(const uint8_t* src, int spitch, uint8_t* d0, int w0, int h0,
                                                   uint8_t* d1, int w1, int h1, size_t sstep, size_t dstep,
                                                   const LbSlot* slots)
{
    const int a = blockIdx.x * 16 + (threadIdx.x & 15), b = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (2 * a >= w0 || 2 * b >= h0) return;
    if (slots) {
        if (!slots[blockIdx.z].active) return;
        src = slots[blockIdx.z].cur;
        spitch = slots[blockIdx.z].cur_pitch;
    } else {
        src += blockIdx.z * sstep;
    }
    d0 += blockIdx.z * dstep;
    if (w1 > 0) d1 += blockIdx.z * dstep;
    const uint8_t* s = src + (size_t)(3 * b) * spitch + 3 * a;
    int r[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) r[j][i] = s[(size_t)j * spitch + i];
    int v[2][2];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            int sum = 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int wy = q ? j : 2 - j;
                sum += wy * ((p ? 0 : 2) * r[j][0] + r[j][1] + (p ? 2 : 0) * r[j][2]);
            }
            v[q][p] = (sum + 4) / 9;
            d0[(size_t)(2 * b + q) * w0 + 2 * a + p] = (uint8_t)v[q][p];
        }
    if (a < w1 && b < h1) d1[(size_t)b * w1 + a] = (uint8_t)mean4(v[0][0], v[0][1], v[1][0], v[1][1]);
}

__device__ __forceinline__ bool arc9(unsigned m)
{
    const unsigned d = m | (m << 16);
    unsigned r = d & (d >> 1);
    r &= r >> 2;
    r &= r >> 4;
    r &= d >> 8;
    return (r & 0xFFFFu) != 0;
}

// FAST score of the pixel at P (0 for non-corners).
__device__ int layer_score(const uint8_t* P, int pw, int t)
{
    const int p = P[0], hi = p + t, lo = p - t;
    unsigned bm = 0, dm = 0;
    int sb = 0, sd = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int c = P[kLayRingDy[k] * pw + kLayRingDx[k]];
        if (c > hi) { bm |= 1u << k; sb += c - hi; }
        if (c < lo) { dm |= 1u << k; sd += lo - c; }
    }
    if (!arc9(bm) && !arc9(dm)) return 0;
    return max(sb, sd);
}

__device__ __forceinline__ int layer_of(const LayArgs& a, uint32_t i)
{
    int l = 0;
    while (l + 1 < a.L && i >= a.base[l + 1]) ++l;
    return l;
}

// Cell of layer-l pixel (x, y): the cell of its level-0 footprint start
// (floor(x S / 2), floor(y S / 2)).
__device__ __forceinline__ int pixel_cell(const LayArgs& a, int l, int x, int y)
{
    const int X = (int)(((long long)x * a.S[l]) >> 1), Y = (int)(((long long)y * a.S[l]) >> 1);
    return (int)(((long long)Y * a.nr) / a.H) * a.nc + (int)(((long long)X * a.nc) / a.W);
}

// Frame j (blockIdx.y) of a chunk: its level 0 frame_step bytes past
// frame 0's, its other layers, scores, flags and block counts ws_step bytes
// past, its per-cell arrays cells_step entries past.
__device__ __forceinline__ const uint8_t* frame_plane(const LayArgs& a, int l, int j)
{
    if (l == 0 && a.slots) return a.slots[j].cur;
    return a.plane[l] + (size_t)j * (l == 0 ? a.frame_step : a.ws_step);
}

__device__ __forceinline__ int frame_pitch(const LayArgs& a, int l, int j)
{
    return l == 0 && a.slots ? a.slots[j].cur_pitch : a.pitch[l];
}

__global__ __launch_bounds__(kLayBlock) void k_lay_score(LayArgs a)
{
    const uint32_t i = blockIdx.x * kLayBlock + threadIdx.x;
    if (i >= a.N) return;
    const int j = blockIdx.y;
    if (a.slots && !a.slots[j].active) return;
    const int l = layer_of(a, i);
    const uint32_t r = i - a.base[l];
    const int w = a.w[l], h = a.h[l], y = (int)(r / (uint32_t)w), x = (int)(r - (uint32_t)y * w);
    int v = 0;
    const bool need = !a.need_score || a.need_score[(size_t)j * a.cells_step + pixel_cell(a, l, x, y)];
    if (need && x >= 3 && y >= 3 && x < w - 3 && y < h - 3)
        v = layer_score(frame_plane(a, l, j) + (size_t)y * frame_pitch(a, l, j) + x, frame_pitch(a, l, j), a.t);
    a.score[(size_t)j * (a.ws_step >> 1) + i] = (uint16_t)v;
}

// A pixel with V > 0 is kept when no pixel of its own layer or an adjacent
// one whose closed footprint meets its own ranks above it: higher V, then
// the lower layer, then the smaller (y, x). The range of pixels x' of a
// layer of pixel size S2 meeting pixel x of pixel size S1 is
// ceil(x S1 / S2) - 1 .. floor((x + 1) S1 / S2).
__global__ __launch_bounds__(kLayBlock) void k_lay_nms(LayArgs a)
{
    __shared__ uint32_t s_cnt[kLayBlock / 64];
    const uint32_t i = blockIdx.x * kLayBlock + threadIdx.x;
    const int j = blockIdx.y;
    if (a.slots && !a.slots[j].active) return;   // the whole workgroup: one slot
    const uint16_t* score = a.score + (size_t)j * (a.ws_step >> 1);
    const size_t cj = (size_t)j * a.cells_step;
    bool keep = false;
    if (i < a.N) {
        const int v = score[i];
        if (v > 0) {
            const int l = layer_of(a, i);
            const uint32_t r = i - a.base[l];
            const int w = a.w[l], y = (int)(r / (uint32_t)w), x = (int)(r - (uint32_t)y * w);
            const int cell = a.need_flag ? pixel_cell(a, l, x, y) : 0;
            keep = !a.need_flag || a.need_flag[cj + cell];
            // Between adjacent layers the size ratio is 1.5 or 4/3, so a
            // range holds at most floor(ratio + 2) = 3 pixels a side: the
            // reads of a 3 x 3 window per layer are issued together, with
            // no early exit; a wider range (none arises) takes the loop.
            bool above = false;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int m = l - 1 + k;
                if (!keep || m < 0 || m >= a.L) continue;
                const int S1 = a.S[l], S2 = a.S[m], wm = a.w[m], hm = a.h[m];
                const int x0 = max((x * S1 + S2 - 1) / S2 - 1, 0), x1 = min(((x + 1) * S1) / S2, wm - 1);
                const int y0 = max((y * S1 + S2 - 1) / S2 - 1, 0), y1 = min(((y + 1) * S1) / S2, hm - 1);
                const uint16_t* sc = score + a.base[m];
                auto ranks_above = [&](int qx, int qy) {
                    const int vq = sc[(size_t)qy * wm + qx];
                    return vq > v || (vq == v && (m < l || (m == l && (qy < y || (qy == y && qx < x)))));
                };
                if (x1 - x0 < 3 && y1 - y0 < 3) {
#pragma unroll
                    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                        for (int dx = 0; dx < 3; ++dx) {
                            const int qx = x0 + dx, qy = y0 + dy;
                            if (qx <= x1 && qy <= y1) above |= ranks_above(qx, qy);
                        }
                } else {
                    for (int qy = y0; qy <= y1; ++qy)
                        for (int qx = x0; qx <= x1; ++qx) above |= ranks_above(qx, qy);
                }
            }
            keep = keep && !above;
            if (keep && a.cell_new) atomicAdd(&a.cell_new[cj + cell], 1u);
        }
        a.flag[(size_t)j * a.ws_step + i] = keep ? 1 : 0;
    }
    const uint64_t b = __ballot(keep);
    if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = (uint32_t)__popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t c = 0;
        for (int k = 0; k < kLayBlock / 64; ++k) c += s_cnt[k];
        a.bcount[(size_t)j * (a.ws_step >> 2) + blockIdx.x] = c;
    }
}

// Exclusive prefix of the block counts (one workgroup) and the total.
constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(kScanBlock) void k_lay_scan(LayArgs a)
{
    __shared__ uint32_t s_wave[kScanBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < a.nblocks; base += kScanBlock) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t c = i < a.nblocks ? a.bcount[i] : 0;
        uint32_t incl = c;   // inclusive prefix within the wave
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(incl, off);
            if (lane >= off) incl += o;
        }
        if (lane == 63) s_wave[wave] = incl;
        __syncthreads();
        uint32_t before = 0, round = 0;
        for (int k = 0; k < kScanBlock / 64; ++k) {
            before += k < wave ? s_wave[k] : 0;
            round += s_wave[k];
        }
        if (i < a.nblocks) a.boff[i] = carry + before + incl - c;
        carry += round;
        __syncthreads();
    }
    if (threadIdx.x == 0) *a.count = carry;
}

__global__ __launch_bounds__(kLayBlock) void k_lay_write(LayArgs a)
{
    __shared__ uint32_t s_cnt[kLayBlock / 64];
    const uint32_t i = blockIdx.x * kLayBlock + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool f = i < a.N && a.flag[i] != 0;
    const uint64_t b = __ballot(f);
    if (lane == 0) s_cnt[wave] = (uint32_t)__popcll(b);
    __syncthreads();
    if (!f) return;
    uint32_t pos = a.boff[blockIdx.x] + (uint32_t)__popcll(b & ((1ull << lane) - 1));
    for (int k = 0; k < wave; ++k) pos += s_cnt[k];
    if (pos >= a.cap) return;
    const int l = layer_of(a, i);
    const uint32_t r = i - a.base[l];
    const int w = a.w[l], y = (int)(r / (uint32_t)w), x = (int)(r - (uint32_t)y * w);
    kpd_keypoint k;
    k.x = (uint16_t)x;
    k.y = (uint16_t)y;
    k.octave = (uint8_t)l;
    k.pad = 0;
    k.score = a.score[i];
    a.out[pos] = k;
}

// Refinement of the keypoints on these layers: for a keypoint (x, y) of
// layer l, the fits at the pixel holding its footprint centre on layers
// l-1, l, l+1 (scores from the maps of the last detection; 0 outside a
// layer), a parabola through the fit values at the layers' log2 scales in
// Newton form with its vertex clamped between the outer two, the position
// moved towards the coarser or finer layer's maximum by the fraction of the
// way in log2 scale. One thread per keypoint; IEEE double steps in a fixed
// order, none fused.
constexpr double kLog2OneHalf = 0.58496250072115618;   // log2(1.5), the nearest double

__device__ __forceinline__ double layer_sigma(int m)
{
    return m % 2 == 0 ? (double)(m / 2) : (double)((m - 1) / 2) + kLog2OneHalf;
}

__global__ __launch_bounds__(kLayBlock) void k_lay_refine(LayArgs a, const kpd_keypoint* list,
                                                          const uint32_t* count, uint32_t cap, kpd_refined* out)
{
#pragma clang fp contract(off)
    const uint32_t i = blockIdx.x * kLayBlock + threadIdx.x;
    if (i >= min(*count, cap)) return;
    const kpd_keypoint kp = list[i];
    const int x = kp.x, y = kp.y, l = kp.octave;
    if (l >= a.L) {   // not a keypoint of these layers
        out[i] = kpd_refined{0.0f, 0.0f, 0.0f, 0.0f};
        return;
    }
    double m[3] = {0.0, 0.0, 0.0}, X[3] = {0.0, 0.0, 0.0}, Y[3] = {0.0, 0.0, 0.0}, sg[3];
    for (int k = 0; k < 3; ++k) {
        const int ll = l - 1 + k;
        sg[k] = layer_sigma(ll);
        if (ll < 0 || ll >= a.L) continue;
        const int cx = (int)(((long long)(2 * x + 1) * a.S[l]) / (2LL * a.S[ll]));
        const int cy = (int)(((long long)(2 * y + 1) * a.S[l]) / (2LL * a.S[ll]));
        const int w = a.w[ll], h = a.h[ll];
        const uint16_t* sc = a.score + a.base[ll];
        int P[9];
        for (int di = -1; di <= 1; ++di)
            for (int dj = -1; dj <= 1; ++dj) {
                const int px = cx + di, py = cy + dj;
                P[3 * (di + 1) + (dj + 1)] = (px >= 0 && py >= 0 && px < w && py < h) ? sc[(size_t)py * w + px] : 0;
            }
        const Fit f = fit_patch(P);
        m[k] = f.m;
        X[k] = (((double)cx + 0.5) + f.u) * ((double)a.S[ll] / 2.0);
        Y[k] = (((double)cy + 0.5) + f.v) * ((double)a.S[ll] / 2.0);
    }
    if (l == 0) { X[0] = X[1]; Y[0] = Y[1]; }
    if (l + 1 >= a.L) { X[2] = X[1]; Y[2] = Y[1]; }
    const double d1 = (m[1] - m[0]) / (sg[1] - sg[0]);
    const double d2 = (m[2] - m[1]) / (sg[2] - sg[1]);
    const double c2 = (d2 - d1) / (sg[2] - sg[0]);
    double sig = sg[1];
    if (c2 < 0.0) {
        sig = (sg[0] + sg[1]) / 2.0 - d1 / (2.0 * c2);
        if (sig > sg[2]) sig = sg[2];
        if (sig < sg[0]) sig = sg[0];
    }
    const double score = (m[0] + d1 * (sig - sg[0])) + (c2 * (sig - sg[0])) * (sig - sg[1]);
    double px, py;
    if (sig >= sg[1]) {
        const double f = (sig - sg[1]) / (sg[2] - sg[1]);
        px = X[1] + f * (X[2] - X[1]);
        py = Y[1] + f * (Y[2] - Y[1]);
    } else {
        const double f = (sg[1] - sig) / (sg[1] - sg[0]);
        px = X[1] + f * (X[0] - X[1]);
        py = Y[1] + f * (Y[0] - Y[1]);
    }
    kpd_refined r;
    r.x = (float)px;
    r.y = (float)py;
    r.log2_scale = (float)sig;
    r.score = (float)score;
    out[i] = r;
}

// ---------------------------------------------------- the masked stream

// Mask of one frame, one workgroup per cell: every cell on a forced frame;
// otherwise the cell's summed |I_n - I_{n-1}| over its level-0 box against
// T_I times its area, or its count in D_{n-1} against T_H.
__global__ __launch_bounds__(256) void k_ls_mask(LsArgs a)
{
    __shared__ unsigned long long s_sum[4];
    const int c = blockIdx.x, cc = c % a.nc, rr = c / a.nc;
    if (threadIdx.x == 0) a.cell_new[c] = 0;   // counted by this frame's suppression
    if (a.force) {
        if (threadIdx.x == 0) a.mask[c] = 1;
        return;
    }
    const int x0 = (int)a.xs[cc], x1 = (int)a.xs[cc + 1], y0 = (int)a.ys[rr], y1 = (int)a.ys[rr + 1];
    const int bw = x1 - x0, n = bw * (y1 - y0);
    unsigned long long sum = 0;
    for (int q = threadIdx.x; q < n; q += 256) {
        const int y = y0 + q / bw, x = x0 + q % bw;
        sum += (unsigned)abs((int)a.cur[(size_t)y * a.cur_pitch + x] - (int)a.prev[(size_t)y * a.prev_pitch + x]);
    }
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
        const bool id = (long long)t > (long long)a.id_thresh * (long long)n;
        const bool kb = a.cnt_prev[c] >= a.kb_thresh;
        a.mask[c] = (id || kb) ? 1 : 0;
    }
}

// The cells whose pixels are scored: those within rx columns and ry rows
// of a marked cell, which holds every neighbour that a marked cell's
// suppression reads (one workgroup).
__global__ __launch_bounds__(256) void k_ls_dilate(LsArgs a)
{
    for (int c = threadIdx.x; c < a.ncell; c += 256) {
        const int cc = c % a.nc, rr = c / a.nc;
        uint8_t need = 0;
        for (int r2 = max(rr - a.ry, 0); r2 <= min(rr + a.ry, a.nr - 1) && !need; ++r2)
            for (int c2 = max(cc - a.rx, 0); c2 <= min(cc + a.rx, a.nc - 1); ++c2)
                if (a.mask[r2 * a.nc + c2]) {
                    need = 1;
                    break;
                }
        a.need_score[c] = need;
    }
}

// D_n's per-cell counts (a marked cell's keypoints, as the suppression
// counted them; an unmarked cell's count in D_{n-1}), their exclusive prefix
// and D_n's size (one workgroup).
__global__ __launch_bounds__(kScanBlock) void k_ls_scan(LsArgs a)
{
    __shared__ uint32_t s_wave[kScanBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int base = 0; base < a.ncell; base += kScanBlock) {
        const int i = base + threadIdx.x;
        uint32_t c = 0;
        if (i < a.ncell) {
            c = a.mask[i] ? a.cell_new[i] : a.cnt_prev[i];
            a.cnt_cur[i] = c;
        }
        uint32_t incl = c;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(incl, off);
            if (lane >= off) incl += o;
        }
        if (lane == 63) s_wave[wave] = incl;
        __syncthreads();
        uint32_t before = 0, round = 0;
        for (int k = 0; k < kScanBlock / 64; ++k) {
            before += k < wave ? s_wave[k] : 0;
            round += s_wave[k];
        }
        if (i < a.ncell) a.off_cur[i] = carry + before + incl - c;
        carry += round;
        __syncthreads();
    }
    if (threadIdx.x == 0) *a.total_cur = carry;
}

// D_n, one workgroup per cell: a marked cell emits the flagged pixels of
// its boxes layer by layer in row-major order (ballot ranks, wave counts in
// LDS, 1024 pixels a round) and stops once it has emitted the count the
// suppression found; an unmarked cell copies its entries of D_{n-1}.
constexpr int kLsWrite = 1024;

__global__ __launch_bounds__(kLsWrite) void k_ls_write(LsArgs a, LayArgs l)
{
    __shared__ uint32_t s_cnt[kLsWrite / 64];
    const int c = blockIdx.x, cc = c % a.nc, rr = c / a.nc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t dst = a.off_cur[c];
    if (!a.mask[c]) {
        const uint32_t src = a.off_prev[c], n = a.cnt_prev[c];
        for (uint32_t i = threadIdx.x; i < n; i += kLsWrite)
            if (src + i < a.cap && dst + i < a.cap) a.list_cur[dst + i] = a.list_prev[src + i];
        return;
    }
    const uint32_t want = a.cnt_cur[c];
    uint32_t run = 0;
    for (int m = 0; m < l.L && run < want; ++m) {
        const int x0 = (int)a.xs[m * (a.nc + 1) + cc], x1 = (int)a.xs[m * (a.nc + 1) + cc + 1];
        const int y0 = (int)a.ys[m * (a.nr + 1) + rr], y1 = (int)a.ys[m * (a.nr + 1) + rr + 1];
        const int bw = x1 - x0, n = bw * (y1 - y0);
        const size_t fb = l.base[m];
        for (int base = 0; base < n && run < want; base += kLsWrite) {
            const int q = base + threadIdx.x;
            int x = 0, y = 0;
            bool f = false;
            if (q < n) {
                y = y0 + q / bw;
                x = x0 + q % bw;
                f = l.flag[fb + (size_t)y * l.w[m] + x] != 0;
            }
            const uint64_t b = __ballot(f);
            if (lane == 0) s_cnt[wave] = (uint32_t)__popcll(b);
            __syncthreads();
            uint32_t pos = run + (uint32_t)__popcll(b & ((1ull << lane) - 1)), total = 0;
            for (int k = 0; k < kLsWrite / 64; ++k) {
                pos += k < wave ? s_cnt[k] : 0;
                total += s_cnt[k];
            }
            if (f && dst + pos < a.cap) {
                kpd_keypoint kp;
                kp.x = (uint16_t)x;
                kp.y = (uint16_t)y;
                kp.octave = (uint8_t)m;
                kp.pad = 0;
                kp.score = l.score[fb + (size_t)y * l.w[m] + x];
                a.list_cur[dst + pos] = kp;
            }
            run += total;
            __syncthreads();   // s_cnt is rewritten by the next round
        }
    }
}

// ------------------------------------------- chunks of the masked stream

// Marks of a chunk, a workgroup per (cell, frame): every cell of a forced
// frame 0 or when the parameters mark every cell, otherwise the cell's
// summed |I_j - I_{j-1}| over its level-0 box against T_I times its area
// (I_{-1}: the frame before the chunk).
__global__ __launch_bounds__(256) void k_ls_mask_chunk(LsChunkArgs a)
{
    __shared__ unsigned long long s_sum[4];
    const int c = blockIdx.x, j = blockIdx.y, cc = c % a.nc, rr = c / a.nc;
    const size_t jc = (size_t)j * a.ncell;
    if (threadIdx.x == 0) a.cell_new[jc + c] = 0;   // counted by frame j's suppression
    bool mark = a.all_marked || (a.force0 && j == 0);
    if (!mark) {
        const uint8_t* cur = a.frames + (size_t)j * a.stride;
        const uint8_t* prev = j ? a.frames + (size_t)(j - 1) * a.stride : a.prev0;
        const int pp = j ? a.pitch : a.prev0_pitch;
        const int x0 = (int)a.xs[cc], x1 = (int)a.xs[cc + 1], y0 = (int)a.ys[rr], y1 = (int)a.ys[rr + 1];
        const int bw = x1 - x0, n = bw * (y1 - y0);
        unsigned long long sum = 0;
        for (int q = threadIdx.x; q < n; q += 256) {
            const int y = y0 + q / bw, x = x0 + q % bw;
            sum += (unsigned)abs((int)cur[(size_t)y * a.pitch + x] - (int)prev[(size_t)y * pp + x]);
        }
        for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
        if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = sum;
        __syncthreads();
        const unsigned long long t = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
        mark = (long long)t > (long long)a.id_thresh * (long long)n;
    }
    if (threadIdx.x == 0) {
        a.mask[jc + c] = mark ? 1 : 0;
        if (j == a.n_frames - 1) a.last_mask[c] = mark ? 1 : 0;
    }
}

// Per frame (a workgroup each): the cells scored, those within rx columns
// and ry rows of a marked cell; per (cell, 64 frames) (the same grid's
// threads): the cell's mark word.
__global__ __launch_bounds__(256) void k_ls_dilate_chunk(LsChunkArgs a)
{
    const int j = blockIdx.x;
    if (j < a.n_frames) {
        const uint8_t* m = a.mask + (size_t)j * a.ncell;
        for (int c = threadIdx.x; c < a.ncell; c += 256) {
            const int cc = c % a.nc, rr = c / a.nc;
            uint8_t need = 0;
            for (int r2 = max(rr - a.ry, 0); r2 <= min(rr + a.ry, a.nr - 1) && !need; ++r2)
                for (int c2 = max(cc - a.rx, 0); c2 <= min(cc + a.rx, a.nc - 1); ++c2)
                    if (m[r2 * a.nc + c2]) {
                        need = 1;
                        break;
                    }
            a.need[(size_t)j * a.ncell + c] = need;
        }
    }
    const int nw = (a.n_frames + 63) >> 6;
    for (int g = blockIdx.x * 256 + threadIdx.x; g < a.ncell * nw; g += gridDim.x * 256) {
        const int c = g / nw, w = g - c * nw;
        unsigned long long bits = 0;
        for (int k = 0; k < 64 && w * 64 + k < a.n_frames; ++k)
            if (a.mask[(size_t)(w * 64 + k) * a.ncell + c]) bits |= 1ull << k;
        a.marks[(size_t)c * a.Kw + w] = bits;
    }
}

// A marked (cell, frame)'s keypoints at the cell's base of the frame's
// sparse list: the flagged pixels of its boxes layer by layer in row-major
// order (as k_ls_write), as many as the suppression counted.
__global__ __launch_bounds__(kLsWrite) void k_ls_write_chunk(LsChunkArgs a, LayArgs l)
{
    __shared__ uint32_t s_cnt[kLsWrite / 64];
    const int c = blockIdx.x, j = blockIdx.y, cc = c % a.nc, rr = c / a.nc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const size_t jc = (size_t)j * a.ncell;
    if (!a.mask[jc + c]) return;
    const uint8_t* flag = l.flag + (size_t)j * l.ws_step;
    const uint16_t* score = l.score + (size_t)j * (l.ws_step >> 1);
    kpd_keypoint* list = a.sparse + (size_t)j * a.list_stride;
    const uint32_t dst = a.cbase[c], want = a.cell_new[jc + c];
    uint32_t run = 0;
    for (int m = 0; m < l.L && run < want; ++m) {
        const int x0 = (int)a.xs[m * (a.nc + 1) + cc], x1 = (int)a.xs[m * (a.nc + 1) + cc + 1];
        const int y0 = (int)a.ys[m * (a.nr + 1) + rr], y1 = (int)a.ys[m * (a.nr + 1) + rr + 1];
        const int bw = x1 - x0, n = bw * (y1 - y0);
        const size_t fb = l.base[m];
        for (int base = 0; base < n && run < want; base += kLsWrite) {
            const int q = base + threadIdx.x;
            int x = 0, y = 0;
            bool f = false;
            if (q < n) {
                y = y0 + q / bw;
                x = x0 + q % bw;
                f = flag[fb + (size_t)y * l.w[m] + x] != 0;
            }
            const uint64_t b = __ballot(f);
            if (lane == 0) s_cnt[wave] = (uint32_t)__popcll(b);
            __syncthreads();
            uint32_t pos = run + (uint32_t)__popcll(b & ((1ull << lane) - 1)), total = 0;
            for (int k = 0; k < kLsWrite / 64; ++k) {
                pos += k < wave ? s_cnt[k] : 0;
                total += s_cnt[k];
            }
            if (f && dst + pos < a.cap) {
                kpd_keypoint kp;
                kp.x = (uint16_t)x;
                kp.y = (uint16_t)y;
                kp.octave = (uint8_t)m;
                kp.pad = 0;
                kp.score = score[fb + (size_t)y * l.w[m] + x];
                list[dst + pos] = kp;
            }
            run += total;
            __syncthreads();   // s_cnt is rewritten by the next round
        }
    }
}

// ------------------------------------- batches of layered streams (ticks)

// Slot s's mask, a workgroup per (cell, slot): every cell of a forced
// slot, otherwise the cell's summed |I_n - I_{n-1}| over its level-0 box
// against T_I times its area, or its count in the slot's D_{n-1} against T_H.
__global__ __launch_bounds__(256) void k_lb_mask(LbArgs a)
{
    __shared__ unsigned long long s_sum[4];
    const int c = blockIdx.x, sl = blockIdx.y, cc = c % a.nc, rr = c / a.nc;
    const LbSlot& S = a.slots[sl];
    if (!S.active) return;
    const size_t sc = (size_t)sl * a.ncell;
    if (threadIdx.x == 0) a.cell_new[sc + c] = 0;
    if (S.force) {
        if (threadIdx.x == 0) a.mask[sc + c] = 1;
        return;
    }
    const int x0 = (int)a.xs[cc], x1 = (int)a.xs[cc + 1], y0 = (int)a.ys[rr], y1 = (int)a.ys[rr + 1];
    const int bw = x1 - x0, n = bw * (y1 - y0);
    unsigned long long sum = 0;
    for (int q = threadIdx.x; q < n; q += 256) {
        const int y = y0 + q / bw, x = x0 + q % bw;
        sum += (unsigned)abs((int)S.cur[(size_t)y * S.cur_pitch + x] - (int)S.prev[(size_t)y * S.prev_pitch + x]);
    }
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
        const bool id = (long long)t > (long long)a.id_thresh * (long long)n;
        const bool kb = a.cnt[1 - S.fb][sc + c] >= a.kb_thresh;
        a.mask[sc + c] = (id || kb) ? 1 : 0;
    }
}

// Slot s's scored cells (a workgroup per slot).
__global__ __launch_bounds__(256) void k_lb_dilate(LbArgs a)
{
    const int sl = blockIdx.x;
    if (!a.slots[sl].active) return;
    const uint8_t* m = a.mask + (size_t)sl * a.ncell;
    for (int c = threadIdx.x; c < a.ncell; c += 256) {
        const int cc = c % a.nc, rr = c / a.nc;
        uint8_t need = 0;
        for (int r2 = max(rr - a.ry, 0); r2 <= min(rr + a.ry, a.nr - 1) && !need; ++r2)
            for (int c2 = max(cc - a.rx, 0); c2 <= min(cc + a.rx, a.nc - 1); ++c2)
                if (m[r2 * a.nc + c2]) {
                    need = 1;
                    break;
                }
        a.need[(size_t)sl * a.ncell + c] = need;
    }
}

// Slot s's D_n counts, offsets and size (a workgroup per slot), as k_ls_scan.
__global__ __launch_bounds__(kScanBlock) void k_lb_scan(LbArgs a)
{
    __shared__ uint32_t s_wave[kScanBlock / 64];
    const int sl = blockIdx.x;
    const LbSlot& S = a.slots[sl];
    if (!S.active) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const size_t sc = (size_t)sl * a.ncell;
    const uint32_t* cnt_prev = a.cnt[1 - S.fb] + sc;
    uint32_t* cnt_cur = a.cnt[S.fb] + sc;
    uint32_t* off_cur = a.off[S.fb] + sc;
    uint32_t carry = 0;
    for (int base = 0; base < a.ncell; base += kScanBlock) {
        const int i = base + threadIdx.x;
        uint32_t c = 0;
        if (i < a.ncell) {
            c = a.mask[sc + i] ? a.cell_new[sc + i] : cnt_prev[i];
            cnt_cur[i] = c;
        }
        uint32_t incl = c;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(incl, off);
            if (lane >= off) incl += o;
        }
        if (lane == 63) s_wave[wave] = incl;
        __syncthreads();
        uint32_t before = 0, round = 0;
        for (int k = 0; k < kScanBlock / 64; ++k) {
            before += k < wave ? s_wave[k] : 0;
            round += s_wave[k];
        }
        if (i < a.ncell) off_cur[i] = carry + before + incl - c;
        carry += round;
        __syncthreads();
    }
    if (threadIdx.x == 0) a.total[S.fb][sl] = carry;
}

// Slot s's D_n, a workgroup per (cell, slot), as k_ls_write.
__global__ __launch_bounds__(kLsWrite) void k_lb_write(LbArgs a, LayArgs l)
{
    __shared__ uint32_t s_cnt[kLsWrite / 64];
    const int c = blockIdx.x, sl = blockIdx.y, cc = c % a.nc, rr = c / a.nc;
    const LbSlot& S = a.slots[sl];
    if (!S.active) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const size_t sc = (size_t)sl * a.ncell;
    kpd_keypoint* list_cur = a.list[S.fb] + (size_t)sl * a.list_stride;
    const uint32_t dst = a.off[S.fb][sc + c];
    if (!a.mask[sc + c]) {
        const kpd_keypoint* list_prev = a.list[1 - S.fb] + (size_t)sl * a.list_stride;
        const uint32_t src = a.off[1 - S.fb][sc + c], n = a.cnt[1 - S.fb][sc + c];
        for (uint32_t i = threadIdx.x; i < n; i += kLsWrite)
            if (src + i < a.cap && dst + i < a.cap) list_cur[dst + i] = list_prev[src + i];
        return;
    }
    const uint8_t* flag = l.flag + (size_t)sl * l.ws_step;
    const uint16_t* score = l.score + (size_t)sl * (l.ws_step >> 1);
    const uint32_t want = a.cnt[S.fb][sc + c];
    uint32_t run = 0;
    for (int m = 0; m < l.L && run < want; ++m) {
        const int x0 = (int)a.xs[m * (a.nc + 1) + cc], x1 = (int)a.xs[m * (a.nc + 1) + cc + 1];
        const int y0 = (int)a.ys[m * (a.nr + 1) + rr], y1 = (int)a.ys[m * (a.nr + 1) + rr + 1];
        const int bw = x1 - x0, n = bw * (y1 - y0);
        const size_t fb = l.base[m];
        for (int base = 0; base < n && run < want; base += kLsWrite) {
            const int q = base + threadIdx.x;
            int x = 0, y = 0;
            bool f = false;
            if (q < n) {
                y = y0 + q / bw;
                x = x0 + q % bw;
                f = flag[fb + (size_t)y * l.w[m] + x] != 0;
            }
            const uint64_t b = __ballot(f);
            if (lane == 0) s_cnt[wave] = (uint32_t)__popcll(b);
            __syncthreads();
            uint32_t pos = run + (uint32_t)__popcll(b & ((1ull << lane) - 1)), total = 0;
            for (int k = 0; k < kLsWrite / 64; ++k) {
                pos += k < wave ? s_cnt[k] : 0;
                total += s_cnt[k];
            }
            if (f && dst + pos < a.cap) {
                kpd_keypoint kp;
                kp.x = (uint16_t)x;
                kp.y = (uint16_t)y;
                kp.octave = (uint8_t)m;
                kp.pad = 0;
                kp.score = score[fb + (size_t)y * l.w[m] + x];
                list_cur[dst + pos] = kp;
            }
            run += total;
            __syncthreads();   // s_cnt is rewritten by the next round
        }
    }
}

}  // namespace

hipError_t launch_lb_mask(const LbArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_lb_mask, dim3(a.ncell, a.nslots), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_lb_dilate, dim3(a.nslots), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_lb_emit(const LbArgs& a, const LayArgs& l, hipStream_t s)
{
    hipLaunchKernelGGL(k_lb_scan, dim3(a.nslots), dim3(kScanBlock), 0, s, a);
    hipLaunchKernelGGL(k_lb_write, dim3(a.ncell, a.nslots), dim3(kLsWrite), 0, s, a, l);
    return hipGetLastError();
}

hipError_t launch_ls_mask_chunk(const LsChunkArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_ls_mask_chunk, dim3(a.ncell, a.n_frames), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_ls_dilate_chunk, dim3(a.n_frames), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ls_write_chunk(const LsChunkArgs& a, const LayArgs& l, hipStream_t s)
{
    hipLaunchKernelGGL(k_ls_write_chunk, dim3(a.ncell, a.n_frames), dim3(kLsWrite), 0, s, a, l);
    return hipGetLastError();
}

hipError_t launch_ls_mask(const LsArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_ls_mask, dim3(a.ncell), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_ls_dilate, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ls_emit(const LsArgs& a, const LayArgs& l, hipStream_t s)
{
    hipLaunchKernelGGL(k_ls_scan, dim3(1), dim3(kScanBlock), 0, s, a);
    hipLaunchKernelGGL(k_ls_write, dim3(a.ncell), dim3(kLsWrite), 0, s, a, l);
    return hipGetLastError();
}

hipError_t launch_lay_score_nms(const LayArgs& a, hipStream_t s, int frames)
{
    if (a.nblocks > 0 && frames > 0) {
        hipLaunchKernelGGL(k_lay_score, dim3(a.nblocks, frames), dim3(kLayBlock), 0, s, a);
        hipLaunchKernelGGL(k_lay_nms, dim3(a.nblocks, frames), dim3(kLayBlock), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_lay_refine(const LayArgs& a, const kpd_keypoint* list, const uint32_t* count, uint32_t cap,
                             kpd_refined* out, hipStream_t s)
{
    if (cap == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lay_refine, dim3((cap + kLayBlock - 1) / kLayBlock), dim3(kLayBlock), 0, s, a, list, count,
                       cap, out);
    return hipGetLastError();
}

hipError_t launch_lay_quad(const uint8_t* src, int spitch, uint8_t* d1, int w1, int h1, uint8_t* d2, int w2, int h2,
                           hipStream_t s, int frames, size_t sstep, size_t dstep, const LbSlot* slots, int from_frame)
{
    if (w1 <= 0 || h1 <= 0 || frames < 1) return hipSuccess;
    const int qx = (w1 + 1) / 2, qy = (h1 + 1) / 2;
    hipLaunchKernelGGL(k_lay_quad, dim3((qx + 15) / 16, (qy + 15) / 16, frames), dim3(256), 0, s, src, spitch, d1, w1,
                       h1, d2, w2, h2, sstep, dstep, slots, from_frame);
    return hipGetLastError();
}

hipError_t launch_lay_third(const uint8_t* src, int spitch, uint8_t* d0, int w0, int h0, uint8_t* d1, int w1, int h1,
                            hipStream_t s, int frames, size_t sstep, size_t dstep, const LbSlot* slots)
{
    if (w0 <= 0 || h0 <= 0 || frames < 1) return hipSuccess;
    const int bx = w0 / 2, by = h0 / 2;
    hipLaunchKernelGGL(k_lay_third, dim3((bx + 15) / 16, (by + 15) / 16, frames), dim3(256), 0, s, src, spitch, d0, w0,
                       h0, d1, w1, h1, sstep, dstep, slots);
    return hipGetLastError();
}

hipError_t launch_lay_detect(const LayArgs& a, hipStream_t s)
{
    if (a.nblocks > 0) {
        hipLaunchKernelGGL(k_lay_score, dim3(a.nblocks), dim3(kLayBlock), 0, s, a);
        hipLaunchKernelGGL(k_lay_nms, dim3(a.nblocks), dim3(kLayBlock), 0, s, a);
    }
    hipLaunchKernelGGL(k_lay_scan, dim3(1), dim3(kScanBlock), 0, s, a);
    if (a.nblocks > 0) hipLaunchKernelGGL(k_lay_write, dim3(a.nblocks), dim3(kLayBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace kpd
