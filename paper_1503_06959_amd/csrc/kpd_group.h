// Device body of the gfx950 group detector: one workgroup detects a
// rectangle of cells of one frame over every octave (Sec. 2: AST segment
// test on the radius-3 circle, FAST score, 3x3 scale-space suppression) and
// writes each cell's keypoints in the cell's (octave, y, x) order at the
// cell's base of a list. The cells of a group share one score map per
// octave, so the suppression apron is scored once per group instead of
// once per cell; how many cells a group holds is a tuning knob that never
// changes results.
//
// Steps of one workgroup:
//   1. clear the bitmaps and score maps (pixels are read from the levels in
//      place, through the caches);
//   2. compass pre-test on 8-pixel groups in packed 16-bit lanes (a 9-arc of
//      the 16 ring pixels holds one of north/south and one of east/west);
//      groups with a survivor are queued per wave, expanded 64 at a time to
//      their survivors, and the full segment test and score run 64 queued
//      pixels at a time;
//   3. suppression of the candidates in the decision boxes;
//   4. per cell, the kept maxima of each (octave, row) run counted, scanned
//      and written in order.
//
// Included by the HIP sources whose kernels run it (chunks, single frames,
// the single-launch batch tick).
#pragma once

#include <hip/hip_runtime.h>

#include "kpd_geom.h"
#include "kpd_kernels.h"

namespace kpd {

namespace {

constexpr int kXcdsG = 8;

__device__ __forceinline__ unsigned gdiv(unsigned i, uint64_t magic)
{
    return (unsigned)(((uint64_t)i * magic) >> 32);
}

// Frames and levels are device global memory, but their pointers reach the
// detector through LDS, where the compiler loses that and would emit flat
// loads (which also count against the LDS counter, so LDS waits wait for
// them). These read through global loads.
template <typename T>
__device__ __forceinline__ T gld(const uint8_t* p)
{
    // through scalar types: the compiler keeps the address space of those
    if constexpr (sizeof(T) == 8) {
        const unsigned long long v = *(const __attribute__((address_space(1))) unsigned long long*)p;
        return T{(uint32_t)v, (uint32_t)(v >> 32)};
    } else {
        return *(const __attribute__((address_space(1))) T*)p;
    }
}

// A global store of a scalar type (the output lists are device global
// memory whose pointers also come through LDS or a table).
template <typename T>
__device__ __forceinline__ void gst(void* p, T v)
{
    *(__attribute__((address_space(1))) T*)p = v;
}

// A value every lane of the wave holds, moved to a scalar register.
__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t rfl64(uint64_t v)
{
    return ((uint64_t)(uint32_t)rfl((int)(v >> 32)) << 32) | (uint32_t)rfl((int)(uint32_t)v);
}

// 8 bytes of a level row at column gx of a level of width w, for rows that
// cannot be read 8 bytes at a time: dwords when mode = 1 (4-byte aligned
// rows), else bytes; columns outside [0, w) read as 0.
__device__ __noinline__ uint2 load8_slow(const uint8_t* src, int gx, int w, int mode)
{
    uint32_t wv[2] = {0u, 0u};
    for (int d = 0; d < 2; ++d) {
        const int g = gx + 4 * d;
        if (mode == 1 && g >= 0 && g + 4 <= w) {
            wv[d] = gld<uint32_t>(src + 4 * d);
        } else {
            for (int k = 0; k < 4; ++k)
                if (g + k >= 0 && g + k < w) wv[d] |= (uint32_t)gld<uint8_t>(src + 4 * d + k) << (8 * k);
        }
    }
    return make_uint2(wv[0], wv[1]);
}

__device__ __forceinline__ int glevel(const int* start, int O, int i)
{
    int o = 0;
    while (o + 1 < O && i >= start[o + 1]) ++o;
    return o;
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as_v(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t as_u(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }

// Compass pre-test of two pixels held in the 16-bit halves of P, with their
// north, south, east and west ring points likewise: a half of the result is
// nonzero when a bright arc (min(max(N,S), max(E,W)) > p + t) or a dark arc
// (max(min(N,S), min(E,W)) < p - t) is still possible.
__device__ __forceinline__ uint32_t compass2(uint32_t P, uint32_t N, uint32_t S, uint32_t E, uint32_t W, u16x2 T2)
{
    const u16x2 p = as_v(P);
    const u16x2 hi = p + T2;
    const u16x2 lo = __builtin_elementwise_sub_sat(p, T2);
    const u16x2 n = as_v(N), s = as_v(S), e = as_v(E), w = as_v(W);
    const u16x2 b = __builtin_elementwise_min(__builtin_elementwise_max(n, s), __builtin_elementwise_max(e, w));
    const u16x2 d = __builtin_elementwise_max(__builtin_elementwise_min(n, s), __builtin_elementwise_min(e, w));
    return as_u(__builtin_elementwise_sub_sat(b, hi)) | as_u(__builtin_elementwise_sub_sat(lo, d));
}

// Two bytes of the 8-byte value {hi, lo} (selectors a, b: byte a to the low
// half, byte b to the high half, each zero-extended to 16 bits).
__device__ __forceinline__ uint32_t pick2(uint32_t hi, uint32_t lo, unsigned a, unsigned b)
{
    return __builtin_amdgcn_perm(hi, lo, 0x0C000C00u | (b << 16) | a);
}

// True when the 16-bit circular mask has 9 contiguous set bits.
__device__ __forceinline__ bool arc9(unsigned m)
{
    const unsigned d = m | (m << 16);
    unsigned r = d & (d >> 1);
    r &= r >> 2;
    r &= r >> 4;
    r &= d >> 8;
    return (r & 0xFFFFu) != 0;
}

// Radius-3 Bresenham circle, clockwise from straight up (Sec. 2), as
// offsets into the 7 x 7 window whose top-left is (x - 3, y - 3).
__device__ __forceinline__ int ring_row(int k)
{
    constexpr int r[16] = {0, 0, 1, 2, 3, 4, 5, 6, 6, 6, 5, 4, 3, 2, 1, 0};
    return r[k];
}
__device__ __forceinline__ int ring_col(int k)
{
    constexpr int c[16] = {3, 4, 5, 6, 6, 6, 5, 4, 3, 2, 1, 0, 0, 0, 1, 2};
    return c[k];
}

// Segment test and FAST score of the pixel whose 7 x 7 window starts at B
// (row pitch tp) for threshold t: 0 unless 9 contiguous ring pixels are all
// brighter than p + t or all darker than p - t; then the larger of the
// bright sum of (c - p - t) and the dark sum of (p - t - c) over the ring.
// The ring masks are collected through the sign of (p + t - c) for bright
// and (c - p + t) for dark, one funnel shift per point (the bit order is
// reversed, which keeps contiguity).
__device__ __forceinline__ int group_score(const uint8_t* B, int tp, int t)
{
    int c[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) c[k] = gld<uint8_t>(B + ring_row(k) * tp + ring_col(k));
    const int p = gld<uint8_t>(B + 3 * tp + 3);
    const int hi = p + t, lo = p - t;
    unsigned bm = 0, dm = 0;
    int smax = 0, smin = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        bm = __builtin_amdgcn_alignbit(bm, (unsigned)(hi - c[k]), 31);
        dm = __builtin_amdgcn_alignbit(dm, (unsigned)(c[k] - lo), 31);
        smax += max(c[k], hi);
        smin += min(c[k], lo);
    }
    if (!arc9(bm & 0xFFFFu) && !arc9(dm & 0xFFFFu)) return 0;
    // sum of (c - hi) over bright points = sum of max(c, hi) - 16 hi; dark alike
    return max(smax - 16 * hi, 16 * lo - smin);
}

}  // namespace

// Score of level-o pixel (x, y) in the group's map.
__device__ __forceinline__ int gv(const uint8_t* sm, const GroupLayout& G, int o, int x, int y)
{
    const uint16_t* v = reinterpret_cast<const uint16_t*>(sm + G.voff[o]);
    return v[(y - G.my0[o]) * G.vpitch[o] + (x - G.mx0[o])];
}

// p = (o, x, y) with score v > 0 is a keypoint when no scale-space
// neighbour ranks above it (higher score; equal score and a finer octave;
// equal score and octave and an earlier (y, x)).
__device__ bool group_local_max(const uint8_t* sm, const GroupLayout& G, int o, int O, int x, int y, int v)
{
    const uint16_t* V = reinterpret_cast<const uint16_t*>(sm + G.voff[o]);
    const int pv = G.vpitch[o];
    const uint16_t* c = V + (y - G.my0[o]) * pv + (x - G.mx0[o]);
    const int before = max(max((int)c[-pv - 1], (int)c[-pv]), max((int)c[-pv + 1], (int)c[-1]));
    const int after = max(max((int)c[1], (int)c[pv - 1]), max((int)c[pv], (int)c[pv + 1]));
    bool keep = before < v && after <= v;
    if (o > 0) {
        const uint16_t* F = reinterpret_cast<const uint16_t*>(sm + G.voff[o - 1]);
        const int pf = G.vpitch[o - 1];
        const uint16_t* f = F + (2 * y - 1 - G.my0[o - 1]) * pf + (2 * x - 1 - G.mx0[o - 1]);
        int m = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int k = 0; k < 4; ++k) m = max(m, (int)f[r * pf + k]);
        keep = keep && m < v;
    }
    if (o + 1 < O) {
        const uint16_t* C = reinterpret_cast<const uint16_t*>(sm + G.voff[o + 1]);
        const int pc = G.vpitch[o + 1];
        const uint16_t* q = C + (((y - 1) >> 1) - G.my0[o + 1]) * pc + (((x - 1) >> 1) - G.mx0[o + 1]);
        const int m = max(max((int)q[0], (int)q[1]), max((int)q[pc], (int)q[pc + 1]));
        keep = keep && m <= v;
    }
    return keep;
}

// Where a group writes: cell c's keypoints start at list[base] (the base
// its layout names), its count goes to own_count[c].
struct GroupOut {
    kpd_keypoint* list;
    uint32_t* own_count;
    uint32_t list_cap;
};

// Detection of one group. lvl/pitch: the frame's levels (level 0 may be
// any pointer and pitch; al8 / al4 say whether its rows can be read 8 / 4
// bytes at a time).
template <int NT>
__device__ void detect_group(const GroupLayout* glob, const uint8_t* const* lvl, const int* pitch, int al8, int al4,
                             int t, const GroupOut& out, uint8_t* sm)
{
    __shared__ GroupLayout G;
    __shared__ const uint8_t* s_lvl[KPD_MAX_OCTAVES];
    __shared__ int s_pitch[KPD_MAX_OCTAVES];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(glob);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&G);
        for (int i = tid; i < (int)(sizeof(GroupLayout) / 4); i += NT) dst[i] = src[i];
        if (tid < KPD_MAX_OCTAVES) {
            s_lvl[tid] = lvl[tid];
            s_pitch[tid] = pitch[tid];
        }
    }
    __syncthreads();
    const int O = G.O;

    // 1) clear bitmaps and score maps (pixels are read from the levels in
    //    place, through the caches)
    uint32_t* s_ncand = reinterpret_cast<uint32_t*>(sm + G.queue_off + (NT / 64) * 2 * kGroupQueue * 4);
    uint32_t* clist = s_ncand + 4;
    {
        uint4* z = reinterpret_cast<uint4*>(sm);
        for (int i = tid; i < G.zero_bytes / 16; i += NT) z[i] = make_uint4(0u, 0u, 0u, 0u);
        if (tid == 0) *s_ncand = 0u;
    }
    __syncthreads();

    uint64_t* keepw = reinterpret_cast<uint64_t*>(sm);
    uint64_t* candw = reinterpret_cast<uint64_t*>(sm + G.cand_off);
    // each wave's two queues: eight-pixel groups with a compass survivor,
    // then single pixels awaiting the full test
    uint32_t* gqueue = reinterpret_cast<uint32_t*>(sm + G.queue_off) + wave * 2 * kGroupQueue;
    uint32_t* queue = gqueue + kGroupQueue;

    // 2) the compass pre-test on the wave's chunks of 64 eight-pixel groups
    //    (chunk k of the group goes to wave k % waves, octave by octave,
    //    with the octave's layout in scalar registers); a group with a
    //    survivor is queued once with its octave and 8-bit survivor mask;
    //    64 queued groups at a time are expanded to their survivors in the
    //    pixel queue, where the full test runs 64 pixels at a time. Both
    //    queues run across octaves, so only the last batch of each is part
    //    full. Candidates inside the decision box are listed for the
    //    suppression (and marked in the candidate bitmap, which the
    //    suppression scans instead if the list overflows).
    {
        constexpr int NW = NT / 64;
        const u16x2 T2 = {(unsigned short)t, (unsigned short)t};
        const u16x2 ONE = {(unsigned short)1, (unsigned short)1};
        uint32_t g_head = 0, g_tail = 0, q_head = 0, q_tail = 0;
        auto full_test = [&](int count) {
            if (lane < count) {
                const uint32_t e = queue[(q_head + lane) & (kGroupQueue - 1)];
                const int o = (int)(e >> 24), row = (int)((e >> 12) & 0xFFFu), col = (int)(e & 0xFFFu);
                const int x = G.tx0[o] + col, y = G.ty0[o] + row;
                if (x >= kRingR && x < G.w[o] - kRingR) {
                    const int pt = s_pitch[o];
                    const int v = group_score(s_lvl[o] + (size_t)(y - kRingR) * pt + (x - kRingR), pt, t);
                    if (v > 0) {
                        reinterpret_cast<uint16_t*>(sm + G.voff[o])[(y - G.my0[o]) * G.vpitch[o] + (x - G.mx0[o])] =
                            (uint16_t)v;
                        const Box d = G.dec[o];
                        if (x >= d.x0 && x < d.x1 && y >= d.y0 && y < d.y1) {
                            const int wd = G.cwoff[o] + (y - d.y0) * G.wpr[o] + ((x - d.x0) >> 6);
                            const int bit = (x - d.x0) & 63;
                            atomicOr(&candw[wd], 1ull << bit);
                            const uint32_t at = atomicAdd(s_ncand, 1u);
                            if (at < (uint32_t)kGroupCands) clist[at] = ((uint32_t)wd << 6) | (uint32_t)bit;
                        }
                    }
                }
            }
            q_head += count;
        };
        // expand up to 64 queued groups into pixel entries, in windows of
        // 64 so the pixel queue never overflows
        auto expand = [&](int ng) {
            uint32_t ge = 0, c = 0;
            if (lane < ng) {
                ge = gqueue[(g_head + lane) & (kGroupQueue - 1)];
                c = (uint32_t)__popc(ge & 0xFFu);
            }
            g_head += ng;
            uint32_t pfx = 0, total = 0;   // exclusive prefix of c over the lanes, by bit planes (c <= 8)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const uint64_t bal = __ballot((c >> b) & 1u);
                pfx += __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u))
                       << b;
                total += (uint32_t)__popcll(bal) << b;
            }
            // pixel entry of pixel 0: octave << 24 | row << 12 | col
            const uint32_t pbase = ((ge >> 29) << 24) | (((ge >> 19) & 0x3FFu) << 12) | ((ge >> 8) & 0x7FFu);
            for (uint32_t win = 0; win < total; win += 64) {
                const uint32_t wend = min(win + 64, total);
                if (c && pfx < wend && pfx + c > win) {
                    uint32_t m = ge & 0xFFu, pos = pfx;
                    while (m) {
                        const int k = __builtin_ctz(m);
                        m &= m - 1;
                        if (pos >= win && pos < wend) queue[(q_tail + pos - win) & (kGroupQueue - 1)] = pbase + k;
                        ++pos;
                    }
                }
                q_tail += wend - win;
                __builtin_amdgcn_wave_barrier();
                while (q_tail - q_head >= 64) {
                    full_test(64);
                    __builtin_amdgcn_wave_barrier();
                }
            }
        };
        int ck0 = 0;
        for (int o = 0; o < O; ++o) {
            const int ngx = rfl(G.ngx[o]), nsr = rfl(G.nsr[o]);
            const int ngroups = ngx * nsr;
            const int nck = (ngroups + 63) >> 6;
            if (nck == 0) continue;
            const int tx0 = rfl(G.tx0[o]), gx0 = rfl(G.gx0[o]), sy0 = rfl(G.sy0[o]), wo = rfl(G.w[o]);
            const uint64_t gcm = rfl64(G.gcm[o]);
            const int pt = rfl(s_pitch[o]);
            const uint8_t* lvo = reinterpret_cast<const uint8_t*>(rfl64(reinterpret_cast<uint64_t>(s_lvl[o])));
            // level 0 may be caller memory whose last row ends the buffer:
            // its south rows are read only up to the frame's width, and its
            // rows are read a dword or a byte at a time when not 8-byte
            // aligned; levels 1.. are 8-byte aligned arena rows
            const int mode = o > 0 ? 2 : (al8 ? 2 : (al4 ? 1 : 0));
            const bool guard = o == 0;
            const uint32_t obits = (uint32_t)o << 29;
            int first = (wave - ck0) % NW;
            if (first < 0) first += NW;
            for (int lc = first; lc < nck; lc += NW) {
                const int g = lc * 64 + lane;
                uint32_t pass = 0u, gent = 0u;
                if (g < ngroups) {
                    const int ry = gdiv(g, gcm);
                    const int gx = gx0 + 8 * (g - ry * ngx), y = sy0 + ry;
                    const int row = ry + kRingR, col = gx - tx0;
                    // the group's row and the rows 3 above and below; the
                    // centre row is never a level's last, so its dword
                    // right of the group stays inside the level, and its
                    // dword left of the group (read from the row above when
                    // gx = 0) only feeds pixels outside the interior
                    const uint8_t* T = lvo + (size_t)y * pt + gx;
                    uint2 c, n, s;
                    uint32_t cm, cp;
                    if (mode == 2) {
                        c = gld<uint2>(T);
                        n = gld<uint2>(T - 3 * pt);
                        cm = gld<uint32_t>(T - 4);
                        cp = gld<uint32_t>(T + 8);
                        if (!guard || gx + 8 <= wo) {
                            s = gld<uint2>(T + 3 * pt);
                        } else {   // bytes past the width feed no interior pixel
                            s.x = gx + 4 <= wo ? gld<uint32_t>(T + 3 * pt) : 0u;
                            s.y = 0u;
                        }
                    } else {
                        c = load8_slow(T, gx, wo, mode);
                        n = load8_slow(T - 3 * pt, gx, wo, mode);
                        s = load8_slow(T + 3 * pt, gx, wo, mode);
                        cm = load8_slow(T - 4, gx - 4, wo, mode).x;
                        cp = load8_slow(T + 8, gx + 8, wo, mode).x;
                    }
                    // pixel i of the group is byte i of {c.y, c.x}; its east
                    // point is byte i + 3, its west point byte i - 3
                    const uint32_t r0 = compass2(pick2(c.y, c.x, 0, 1), pick2(n.y, n.x, 0, 1),
                                                 pick2(s.y, s.x, 0, 1), pick2(c.y, c.x, 3, 4),
                                                 pick2(c.x, cm, 1, 2), T2);
                    const uint32_t r1 = compass2(pick2(c.y, c.x, 2, 3), pick2(n.y, n.x, 2, 3),
                                                 pick2(s.y, s.x, 2, 3), pick2(c.y, c.x, 5, 6),
                                                 pick2(c.x, cm, 3, 4), T2);
                    const uint32_t r2 = compass2(pick2(c.y, c.x, 4, 5), pick2(n.y, n.x, 4, 5),
                                                 pick2(s.y, s.x, 4, 5), pick2(cp, c.y, 3, 4),
                                                 pick2(c.y, c.x, 1, 2), T2);
                    const uint32_t r3 = compass2(pick2(c.y, c.x, 6, 7), pick2(n.y, n.x, 6, 7),
                                                 pick2(s.y, s.x, 6, 7), pick2(cp, c.y, 5, 6),
                                                 pick2(c.y, c.x, 3, 4), T2);
                    // survivor bits: each 16-bit half to 0 or 1, pixel 2j at
                    // bit 2j and pixel 2j+1 at bit 16 + 2j, then folded to 8 bits
                    const uint32_t m = as_u(__builtin_elementwise_min(as_v(r0), ONE)) |
                                       (as_u(__builtin_elementwise_min(as_v(r1), ONE)) << 2) |
                                       (as_u(__builtin_elementwise_min(as_v(r2), ONE)) << 4) |
                                       (as_u(__builtin_elementwise_min(as_v(r3), ONE)) << 6);
                    pass = (m | (m >> 15)) & 0xFFu;
                    gent = obits | ((uint32_t)row << 19) | ((uint32_t)col << 8) | pass;
                }
                const uint64_t bal = __ballot(pass != 0u);
                if (bal) {
                    if (pass) {
                        const unsigned below = __builtin_amdgcn_mbcnt_hi(
                            (unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
                        gqueue[(g_tail + below) & (kGroupQueue - 1)] = gent;
                    }
                    g_tail += (uint32_t)__popcll(bal);
                    if (g_tail - g_head >= 64) {
                        __builtin_amdgcn_wave_barrier();
                        expand(64);
                        __builtin_amdgcn_wave_barrier();
                    }
                }
            }
            ck0 += nck;
        }
        __builtin_amdgcn_wave_barrier();
        if (g_tail != g_head) expand((int)(g_tail - g_head));
        __builtin_amdgcn_wave_barrier();
        if (q_tail != q_head) full_test((int)(q_tail - q_head));
    }
    __syncthreads();

    // 3) suppression of the listed candidates, a thread each; when the list
    //    overflowed, each wave scans 64 candidate words at a time (one per
    //    lane), queues the candidates and tests 64 queued ones at a time
    const uint32_t ncand = *s_ncand;
    auto suppress = [&](uint32_t e) {
        const int wd = (int)(e >> 6), b = (int)(e & 63);
        const int o = glevel(G.cwoff, O, wd);
        const unsigned jw = wd - G.cwoff[o];
        const int ry = gdiv(jw, G.wpm[o]);
        const int x = G.dec[o].x0 + 64 * (int)(jw - ry * G.wpr[o]) + b, y = G.dec[o].y0 + ry;
        if (group_local_max(sm, G, o, O, x, y, gv(sm, G, o, x, y))) atomicOr(&keepw[wd], 1ull << b);
    };
    if (ncand <= (uint32_t)kGroupCands) {
        for (uint32_t i = tid; i < ncand; i += NT) suppress(clist[i]);
    } else {
        uint32_t q_head = 0, q_tail = 0;
        auto nms = [&](int count) {
            if (lane < count) suppress(queue[(q_head + lane) & (kGroupQueue - 1)]);
            q_head += count;
        };
        constexpr uint32_t kWindow = kGroupQueue - 64;
        const int nw = G.nwords;
        for (int w0 = wave * 64; w0 < nw; w0 += (NT / 64) * 64) {
            const int w = w0 + lane;
            const uint64_t word = w < nw ? candw[w] : 0ull;
            const uint32_t cnt = (uint32_t)__popcll(word);
            uint32_t incl = cnt;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t up = __shfl_up(incl, off, 64);
                if (lane >= off) incl += up;
            }
            const uint32_t total = __shfl(incl, 63, 64);
            const uint32_t excl = incl - cnt;
            for (uint32_t win = 0; win < total; win += kWindow) {
                const uint32_t wend = min(win + kWindow, total);
                if (excl < wend && excl + cnt > win) {
                    uint64_t bits = word;
                    uint32_t e = excl;
                    while (bits) {
                        const int k = __builtin_ctzll(bits);
                        bits &= bits - 1;
                        if (e >= win && e < wend) queue[(q_tail + e - win) & (kGroupQueue - 1)] = (uint32_t)(w * 64 + k);
                        ++e;
                    }
                }
                q_tail += wend - win;
                __builtin_amdgcn_wave_barrier();
                while (q_tail - q_head >= 64) {
                    nms(64);
                    __builtin_amdgcn_wave_barrier();
                }
            }
        }
        if (q_tail != q_head) nms((int)(q_tail - q_head));
    }
    __syncthreads();

    // 4) per cell: its decision box on each octave, the kept maxima of each
    //    (octave, row) run counted, scanned and written in order
    {
        for (int k = wave; k < G.ncells; k += NT / 64) {
            const int c = G.cell_c[k];
            const int X0 = G.cell_rect[k].x0, X1 = G.cell_rect[k].x1, Y0 = G.cell_rect[k].y0, Y1 = G.cell_rect[k].y1;
            int dx0[KPD_MAX_OCTAVES], dx1[KPD_MAX_OCTAVES], dy0[KPD_MAX_OCTAVES], start[KPD_MAX_OCTAVES + 1];
            int nseg = 0;
#pragma unroll
            for (int o = 0; o < KPD_MAX_OCTAVES; ++o) {
                start[o] = nseg;
                dx0[o] = dx1[o] = dy0[o] = 0;
                if (o < O) {
                    const int wo = G.w[o], ho = G.h[o];
                    const int x0 = max(shr_ceil(X0, o), kRingR), x1 = min(shr_ceil(X1, o), wo - kRingR);
                    const int y0 = max(shr_ceil(Y0, o), kRingR), y1 = min(shr_ceil(Y1, o), ho - kRingR);
                    if (x0 < x1 && y0 < y1) {
                        dx0[o] = x0;
                        dx1[o] = x1;
                        dy0[o] = y0;
                        nseg += y1 - y0;
                    }
                }
            }
            start[KPD_MAX_OCTAVES] = nseg;
            const uint32_t base = G.cell_base[k];
            uint32_t run = 0;
            for (int s0 = 0; s0 < nseg; s0 += 64) {
                const int s = s0 + lane;
                int o = 0;
#pragma unroll
                for (int q = 1; q < KPD_MAX_OCTAVES; ++q) o += (q < O && s >= start[q]) ? 1 : 0;
                uint32_t cnt = 0;
                int wb = 0, b0 = 0, b1 = 0, y = 0;
                if (s < nseg) {
                    const Box d = G.dec[o];
                    y = dy0[o] + (s - start[o]);
                    wb = G.cwoff[o] + (y - d.y0) * G.wpr[o];
                    b0 = dx0[o] - d.x0;
                    b1 = dx1[o] - d.x0;
                    for (int wi = b0 >> 6; wi <= (b1 - 1) >> 6; ++wi) {
                        uint64_t word = keepw[wb + wi];
                        const int lo = max(b0 - 64 * wi, 0), hi = min(b1 - 64 * wi, 64);
                        word &= (hi == 64 ? ~0ull : ((1ull << hi) - 1)) & (~0ull << lo);
                        cnt += (uint32_t)__popcll(word);
                    }
                }
                // exclusive prefix of the counts over the lanes, by bit planes
                // (a row run holds at most 64 keypoints)
                uint32_t excl = 0, total = 0;
#pragma unroll
                for (int b = 0; b < 7; ++b) {
                    const uint64_t bal = __ballot((cnt >> b) & 1u);
                    excl += __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u)) << b;
                    total += (uint32_t)__popcll(bal) << b;
                }
                if (cnt) {
                    uint32_t pos = base + run + excl;
                    const int x0 = G.dec[o].x0;
                    for (int wi = b0 >> 6; wi <= (b1 - 1) >> 6; ++wi) {
                        uint64_t word = keepw[wb + wi];
                        const int lo = max(b0 - 64 * wi, 0), hi = min(b1 - 64 * wi, 64);
                        word &= (hi == 64 ? ~0ull : ((1ull << hi) - 1)) & (~0ull << lo);
                        while (word) {
                            const int b = __builtin_ctzll(word);
                            word &= word - 1;
                            const int x = x0 + 64 * wi + b;
                            const uint32_t v = (uint32_t)gv(sm, G, o, x, y);
                            // one keypoint per 2x2 block keeps pos below the cell's capacity
                            if (pos < out.list_cap)
                                gst<unsigned long long>(out.list + pos,
                                                        (unsigned long long)((uint32_t)x | ((uint32_t)y << 16)) |
                                                            ((unsigned long long)((uint32_t)o | (v << 16)) << 32));
                            ++pos;
                        }
                    }
                }
                run += total;
            }
            if (lane == 0) gst<uint32_t>(out.own_count + c, run);
        }
    }
}

}  // namespace kpd
