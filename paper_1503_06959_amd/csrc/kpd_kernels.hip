// gfx950 kernels of the masked multi-scale FAST detector.
//
// Per frame, on the caller's stream:
//   k_cell_mask   per-cell SAD of I_n vs I_{n-1} and the mark decision
//                 (Sec. 3.1 Eq. 2 as a per-cell mean absolute difference;
//                 Sec. 3.2 Eqs. 3-4 from the per-cell counts of D_{n-1});
//   k_pyramid     octave pyramid by 2x2 box average, round half up (Sec. 2,
//                 Sec. 3.1), all levels of one level-0 tile per workgroup;
//   k_detect      one workgroup per marked cell: AST segment test + FAST
//                 score on every level over the cell's score boxes (LDS),
//                 3x3 scale-space suppression (Sec. 2), ordered compaction
//                 of the survivors into the cell's slot; the last workgroup
//                 scans the per-cell counts into list offsets;
//   k_gather      Eq. (1): concatenates every cell's slot (new keypoints in
//                 marked cells, untouched carried ones elsewhere) into D_n.
#include <hip/hip_runtime.h>

#include "kpd_geom.h"
#include "kpd_kernels.h"

namespace kpd {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// floor(i / d) for i < 2^24 and 0 < d < 2^16 with magic = ceil(2^32 / d)
// (kept in 64 bits so that d = 1 works): the rounding error
// i * (magic - 2^32/d) / 2^32 stays below 1/d, so the floor is exact.
__device__ __forceinline__ unsigned fast_div(unsigned i, uint64_t magic)
{
    return (unsigned)(((uint64_t)i * magic) >> 32);
}
__device__ __forceinline__ uint64_t div_magic_dev(unsigned d) { return (0x100000000ull + d - 1) / d; }

// ------------------------------------------------------------------ mask

__global__ __launch_bounds__(kBlock) void k_cell_mask(MaskArgs a)
{
    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    const Box r = cell_rect(c, a.W, a.H, a.nc, a.nr);
    const int cw = box_w(r), ch = box_h(r);
    const uint64_t magic = div_magic_dev(cw);
    unsigned sad = 0;
    if (a.id_on) {
        const int n = cw * ch;
        for (int i = tid; i < n; i += kBlock) {
            const int ry = fast_div(i, magic);
            const int rx = i - ry * cw;
            const int cur = a.cur[(size_t)(r.y0 + ry) * a.cur_pitch + r.x0 + rx];
            const int prv = a.prev[(size_t)(r.y0 + ry) * a.prev_pitch + r.x0 + rx];
            sad += (unsigned)abs(cur - prv);
        }
    }
    // wave reduction, then across the 4 waves
    for (int off = 32; off > 0; off >>= 1) sad += __shfl_xor(sad, off);
    __shared__ unsigned part[kWaves];
    if ((tid & 63) == 0) part[tid >> 6] = sad;
    __syncthreads();
    if (tid == 0) {
        unsigned s = 0;
        for (int w = 0; w < kWaves; ++w) s += part[w];
        a.sad[c] = s;
        const bool id = a.id_on && (int64_t)s > (int64_t)a.id_thresh * (int64_t)(cw * ch);
        const bool kb = a.count[c] >= a.kb_thresh;
        a.mask[c] = (uint8_t)(id || kb);
    }
}

// --------------------------------------------------------------- pyramid

__global__ __launch_bounds__(kBlock) void k_pyramid(PyrArgs a)
{
    extern __shared__ uint8_t smem[];
    const int T = a.tile;           // level-0 tile side, a power of two >= 2^(O-1)
    uint8_t* buf0 = smem;
    uint8_t* buf1 = smem + (T / 2) * (T / 2);
    const int tid = threadIdx.x;
    uint8_t* prev = nullptr;
    uint8_t* cur = buf0;
    for (int o = 1; o < a.O; ++o) {
        const int ts = T >> o;
        const int lg = __builtin_ctz(ts);
        const int wo = a.w[o], ho = a.h[o];
        uint8_t* dst = a.lvl[o];
        const int pitch = a.pitch[o];
        for (int i = tid; i < ts * ts; i += kBlock) {
            const int yy = i >> lg, xx = i & (ts - 1);
            const int gx = blockIdx.x * ts + xx, gy = blockIdx.y * ts + yy;
            int v = 0;
            if (o == 1) {
                if (gx < wo && gy < ho) {
                    const uint8_t* s0 = a.lvl0 + (size_t)(2 * gy) * a.pitch0 + 2 * gx;
                    const uint8_t* s1 = s0 + a.pitch0;
                    v = (s0[0] + s0[1] + s1[0] + s1[1] + 2) >> 2;
                }
            } else {
                const int ps = ts * 2;
                const uint8_t* s0 = prev + (2 * yy) * ps + 2 * xx;
                v = (s0[0] + s0[1] + s0[ps] + s0[ps + 1] + 2) >> 2;
            }
            cur[i] = (uint8_t)v;
            if (gx < wo && gy < ho) dst[(size_t)gy * pitch + gx] = (uint8_t)v;
        }
        __syncthreads();
        prev = cur;
        cur = (cur == buf0) ? buf1 : buf0;
    }
}

// ---------------------------------------------------------------- detect

// Radius-3 Bresenham circle, clockwise from straight up (Sec. 2).
__constant__ int8_t kRingDx[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
__constant__ int8_t kRingDy[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};

// True when the 16-bit circular mask has 9 contiguous set bits.
__device__ __forceinline__ bool has_arc9(unsigned m)
{
    unsigned d = m | (m << 16);
    unsigned r = d & (d >> 1);  // runs of 2
    r &= r >> 2;                // runs of 4
    r &= r >> 4;                // runs of 8
    r &= d >> 8;                // runs of 9
    return (r & 0xFFFFu) != 0;
}

// Segment test and FAST score of the pixel at P (row pitch pw) for
// threshold t; 0 for pixels that are not corners.
__device__ __forceinline__ int fast_score(const uint8_t* P, int pw, int t)
{
    const int p = P[0];
    const int hi = p + t, lo = p - t;
    const int n = P[-3 * pw], s = P[3 * pw], e = P[3], w = P[-3];
    // Any 9-arc of 16 holds ring position k or k+8 for every k, so a
    // bright arc needs one of {up, down} and one of {right, left} brighter.
    const bool maybe_b = max(n, s) > hi && max(e, w) > hi;
    const bool maybe_d = min(n, s) < lo && min(e, w) < lo;
    if (!(maybe_b || maybe_d)) return 0;
    unsigned bm = 0, dm = 0;
    int sb = 0, sd = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int c = P[kRingDy[k] * pw + kRingDx[k]];
        const int db = c - hi, dd = lo - c;
        if (db > 0) { bm |= 1u << k; sb += db; }
        if (dd > 0) { dm |= 1u << k; sd += dd; }
    }
    if (!has_arc9(bm) && !has_arc9(dm)) return 0;
    return max(sb, sd);
}

// Score maps of one workgroup: level o covers box sb[o] at LDS offset voff[o].
struct ScoreMaps {
    const uint8_t* smem;
    const Box* sb;
    const int* voff;
};

__device__ __forceinline__ int vget(const ScoreMaps& M, int o, int x, int y)
{
    const Box b = M.sb[o];
    if (x < b.x0 || x >= b.x1 || y < b.y0 || y >= b.y1) return 0;
    const uint16_t* v = reinterpret_cast<const uint16_t*>(M.smem + M.voff[o]);
    return v[(y - b.y0) * (b.x1 - b.x0) + (x - b.x0)];
}

// p = (o, x, y) with score v > 0 is a keypoint when no scale-space neighbour
// ranks above it: higher score, or equal score and a finer octave, or equal
// score and octave and an earlier (y, x).
__device__ bool is_local_max(const ScoreMaps& M, int o, int O, int x, int y, int v)
{
    // in-plane: the three pixels above and the one to the left precede p
    if (vget(M, o, x - 1, y - 1) >= v || vget(M, o, x, y - 1) >= v || vget(M, o, x + 1, y - 1) >= v ||
        vget(M, o, x - 1, y) >= v)
        return false;
    if (vget(M, o, x + 1, y) > v || vget(M, o, x - 1, y + 1) > v || vget(M, o, x, y + 1) > v ||
        vget(M, o, x + 1, y + 1) > v)
        return false;
    if (o > 0) {
        for (int yy = 2 * y - 1; yy <= 2 * y + 2; ++yy)
            for (int xx = 2 * x - 1; xx <= 2 * x + 2; ++xx)
                if (vget(M, o - 1, xx, yy) >= v) return false;
    }
    if (o + 1 < O) {
        for (int yy = (y - 1) >> 1; yy <= (y + 1) >> 1; ++yy)
            for (int xx = (x - 1) >> 1; xx <= (x + 1) >> 1; ++xx)
                if (vget(M, o + 1, xx, yy) > v) return false;
    }
    return true;
}

__global__ __launch_bounds__(kBlock) void k_detect(DetectArgs a)
{
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ Box s_dec[KPD_MAX_OCTAVES];
    __shared__ Box s_sb[KPD_MAX_OCTAVES];
    __shared__ int s_voff[KPD_MAX_OCTAVES];
    __shared__ int s_tile_off;
    __shared__ unsigned s_wcount[kWaves];
    __shared__ int s_last;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int c = blockIdx.x;
    const int O = a.O;

    bool active = a.all_marked || a.mask[c];
    if (active) {
        if (tid == 0) {
            if (a.all_marked) a.mask[c] = 1;
            const Box r = cell_rect(c, a.W, a.H, a.nc, a.nr);
            for (int o = 0; o < O; ++o) s_dec[o] = decision_box(r, o, a.w[o], a.h[o]);
            int off = 0;
            for (int o = 0; o < O; ++o) {
                s_sb[o] = score_box(s_dec, o, O, a.w[o], a.h[o]);
                s_voff[o] = off;
                if (!box_empty(s_sb[o])) off += round_up(box_w(s_sb[o]) * box_h(s_sb[o]) * 2, 4);
            }
            s_tile_off = off;
        }
        __syncthreads();

        uint8_t* tile = smem + s_tile_off;
        // 1) scores of every level over its score box
        for (int o = 0; o < O; ++o) {
            const Box sb = s_sb[o];
            if (box_empty(sb)) continue;
            const int vw = box_w(sb), vh = box_h(sb);
            const int tw = vw + 6, th = vh + 6;
            const uint8_t* src = a.lvl[o];
            const int pitch = a.pitch[o];
            const uint64_t mt = div_magic_dev(tw);
            for (int i = tid; i < tw * th; i += kBlock) {
                const int ry = fast_div(i, mt), rx = i - ry * tw;
                tile[i] = src[(size_t)(sb.y0 - 3 + ry) * pitch + (sb.x0 - 3 + rx)];
            }
            __syncthreads();
            uint16_t* V = reinterpret_cast<uint16_t*>(smem + s_voff[o]);
            const uint64_t mv = div_magic_dev(vw);
            for (int i = tid; i < vw * vh; i += kBlock) {
                const int ry = fast_div(i, mv), rx = i - ry * vw;
                V[i] = (uint16_t)fast_score(tile + (ry + 3) * tw + (rx + 3), tw, a.t);
            }
            __syncthreads();
        }

        // 2) suppression and ordered compaction, octave by octave, raster order
        const ScoreMaps M{smem, s_sb, s_voff};
        kpd_keypoint* slot = a.store + a.store_base[c];
        const unsigned slot_cap = a.store_base[c + 1] - a.store_base[c];
        unsigned base = 0;
        for (int o = 0; o < O; ++o) {
            const Box d = s_dec[o];
            if (box_empty(d)) continue;
            const int dw = box_w(d);
            const int n = dw * box_h(d);
            const uint64_t md = div_magic_dev(dw);
            for (int chunk = 0; chunk < n; chunk += kBlock) {
                const int i = chunk + tid;
                bool keep = false;
                int x = 0, y = 0, v = 0;
                if (i < n) {
                    const int ry = fast_div(i, md);
                    y = d.y0 + ry;
                    x = d.x0 + (i - ry * dw);
                    v = vget(M, o, x, y);
                    if (v > 0) keep = is_local_max(M, o, O, x, y, v);
                }
                const unsigned long long bal = __ballot(keep);
                const unsigned below = __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
                if (lane == 0) s_wcount[wave] = (unsigned)__popcll(bal);
                __syncthreads();
                unsigned woff = 0, tot = 0;
                for (int w2 = 0; w2 < kWaves; ++w2) {
                    const unsigned cnt = s_wcount[w2];
                    woff += (w2 < wave) ? cnt : 0u;
                    tot += cnt;
                }
                // a cell never holds more than its slot (one keypoint per 2x2
                // block of each decision box); the bound only guards the store
                if (keep && base + woff + below < slot_cap) {
                    kpd_keypoint k;
                    k.x = (uint16_t)x; k.y = (uint16_t)y; k.octave = (uint8_t)o; k.pad = 0;
                    k.score = (uint16_t)v;
                    slot[base + woff + below] = k;
                }
                base += tot;
                __syncthreads();
            }
        }
        if (tid == 0) a.count[c] = base;
    }

    // 3) the last workgroup to finish scans the per-cell counts into offsets
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        const unsigned ticket = atomicAdd(&a.hdr[1], 1u);
        s_last = (ticket == gridDim.x - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    const int ncell = a.nc * a.nr;
    const int per = (ncell + kBlock - 1) / kBlock;
    const int c0 = tid * per, c1 = min(c0 + per, ncell);
    unsigned sum = 0;
    for (int cc = c0; cc < c1; ++cc) sum += __hip_atomic_load(&a.count[cc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned* scan = reinterpret_cast<unsigned*>(smem);
    scan[tid] = sum;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const unsigned add = tid >= off ? scan[tid - off] : 0u;
        __syncthreads();
        scan[tid] += add;
        __syncthreads();
    }
    unsigned run = scan[tid] - sum;  // exclusive prefix
    for (int cc = c0; cc < c1; ++cc) {
        a.offsets[cc] = run;
        run += __hip_atomic_load(&a.count[cc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid == kBlock - 1) {
        a.hdr[0] = scan[kBlock - 1];
        a.hdr[1] = 0;  // reset the ticket for the next frame
    }
}

// ---------------------------------------------------------------- gather

__global__ __launch_bounds__(64) void k_gather(GatherArgs a)
{
    const int c = blockIdx.x;
    const unsigned n = a.count[c];
    const unsigned off = a.offsets[c];
    const kpd_keypoint* src = a.store + a.store_base[c];
    for (unsigned i = threadIdx.x; i < n; i += 64) a.out[off + i] = src[i];
}

// ------------------------------------------------------------- launchers

// The last workgroup's count scan reuses the dynamic LDS: at least one word
// per thread.
int detect_lds_bytes(int lds_bytes) { return lds_bytes < kBlock * 4 ? kBlock * 4 : lds_bytes; }

hipError_t launch_cell_mask(const MaskArgs& a, int ncell, hipStream_t s)
{
    hipLaunchKernelGGL(k_cell_mask, dim3(ncell), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pyramid(const PyrArgs& a, hipStream_t s)
{
    const int T = a.tile;
    dim3 grid((a.W + T - 1) / T, (a.H + T - 1) / T);
    const size_t lds = 2 * (size_t)(T / 2) * (T / 2);
    hipLaunchKernelGGL(k_pyramid, grid, dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_detect(const DetectArgs& a, int ncell, int lds_bytes, hipStream_t s)
{
    const int lds = detect_lds_bytes(lds_bytes);
    hipLaunchKernelGGL(k_detect, dim3(ncell), dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs& a, int ncell, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather, dim3(ncell), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace kpd
