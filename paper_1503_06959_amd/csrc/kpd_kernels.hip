// gfx950 kernels of the masked multi-scale FAST detector, beside the group
// detector (kpd_group.h, kpd_group.hip). Three launches per frame of one
// stream (k_frame1, then k_det1_groups and k_compact1; k_detect1 for the
// per-pixel masks); four per batch tick over many streams (k_frame_batch,
// k_mark_batch, k_detect_list_batch_groups, k_compact_batch) or one
// persistent k_tick; three to six per chunk of consecutive frames of one
// stream (k_frame_chunk_seq or k_frame_chunk, then k_mark_chunk and
// k_detect_list_groups, the speculation passes, or k_detect_chunk_groups,
// then k_compact_chunk). The bodies here:
//
//   frame_tile   one workgroup per level-0 tile, aligned to the coarsest
//                octave: loads the tile of I_n (dwords, or 16-byte row
//                segments for 128-px tiles), builds every coarser octave of
//                it (from registers for 128-px tiles, else in LDS) by 2x2
//                box average with round-half-up (Sec. 2, Sec. 3.1) and
//                writes them out; when the intensity-difference mask is
//                active it also sums |I_n - I_{n-1}| per cell (v_sad_u8 per
//                dword, register and LDS partials, one atomic per tile and
//                cell) for the per-cell mean-difference test (Sec. 3.1
//                Eq. 2, read per cell).
//   k_frame_chunk_seq  the tile pass of a chunk whose frames test
//                differences, each workgroup walking a run of frames of its
//                tile in order so that every frame is read once.
//   detect_marked / detect_cell  the per-cell detector of the per-pixel
//                mask modes: stages the cell's octave tiles in LDS, runs the
//                compass pre-test and the segment test and FAST score, keeps
//                the scale-space maxima (Sec. 2) as a bitmask; the counts of
//                earlier cells give the cell's offset in D_n (Eq. 1).
//   compact_frame  builds a frame's D_n in cell order from the marked
//                cells' sparse lists and D_{n-1} (Eq. 1).
//
// The kernel boundary between passes publishes the pyramid and the SAD to
// every XCD at once. In the per-pixel mask modes a cell only waits for the
// counts of lower-numbered cells of its stream (relaxed agent-scope count
// words, no fences); each XCD dispatches its workgroups in index order, so
// the lowest unfinished cell can always run, and every wait is bounded and
// sets an error flag instead of hanging. In a chunk, only T_H marking
// waits, on the same cell's count word of the previous frame.
#include <hip/hip_runtime.h>

#include <atomic>
#include <type_traits>

#include "kpd_fit.h"
#include "kpd_geom.h"
#include "kpd_group.h"
#include "kpd_kernels.h"

namespace kpd {

constexpr int kFrameBlock = 256;
// Workgroup size of the cell-layout detector (the per-pixel mask modes of
// single frames), where one cell's latency decides.
constexpr int kDetLatency = kDetectBlock;
constexpr int kRegOctaves = 6;   // 128-px tiles build up to this many levels in registers

// floor(i / d) with magic = div_magic(d) (see kpd_geom.h)
__device__ __forceinline__ unsigned fast_div(unsigned i, uint64_t magic)
{
    return (unsigned)(((uint64_t)i * magic) >> 32);
}

// ------------------------------------------------------------------ k_frame

// 2x2 mean with round-half-up ((a+b+c+d+2)>>2) of two rows of eight
// pixels, rows a and b as two dwords each (pixel k in byte k % 4 of dword
// k / 4): the four outputs, packed. Pair sums are formed in 16-bit lanes, so
// no lane carries into the next.
__device__ __forceinline__ uint32_t mean2x2(uint32_t a0, uint32_t a1, uint32_t b0, uint32_t b1)
{
    constexpr uint32_t m = 0x00FF00FFu;
    const uint32_t s0 = (((a0 & m) + ((a0 >> 8) & m) + (b0 & m) + ((b0 >> 8) & m) + 0x00020002u) >> 2) & m;
    const uint32_t s1 = (((a1 & m) + ((a1 >> 8) & m) + (b1 & m) + ((b1 >> 8) & m) + 0x00020002u) >> 2) & m;
    return ((s0 | (s0 >> 8)) & 0xFFFFu) | ((s1 | (s1 >> 8)) << 16);
}

// Store the first n bytes of packed pixels at level position (gx, gy) of
// `out`, clipped to the level's w x h; one wide store when the run is whole.
template <int N>
__device__ __forceinline__ void store_px(uint8_t* out, int pitch, int w, int h, int gx, int gy, uint32_t lo,
                                         uint32_t hi)
{
    if (gy >= h || gx >= w) return;
    uint8_t* p = out + (size_t)gy * pitch + gx;
    if (gx + N - 1 < w) {
        if constexpr (N == 8) *reinterpret_cast<uint2*>(p) = make_uint2(lo, hi);
        else if constexpr (N == 4) *reinterpret_cast<uint32_t*>(p) = lo;
        else if constexpr (N == 2) *reinterpret_cast<uint16_t*>(p) = (uint16_t)lo;
        else *p = (uint8_t)lo;
        return;
    }
    for (int k = 0; k < N && gx + k < w; ++k) p[k] = (uint8_t)((k < 4 ? lo : hi) >> (8 * (k & 3)));
}

// Octaves 1..O-1 (O <= 6) of a 128-px tile from registers: thread (rb, seg)
// holds level-0 rows 4rb..4rb+3, columns 16seg..16seg+15 (rows[u], one
// uint4 each), so its level-1 block (2 x 8) and level-2 block (1 x 4) are
// its own; level 3 pairs it with the thread one row block down (8 lanes
// on), level 4 with the threads 16 and 24 lanes on, and level 5 with the
// thread 32 lanes on and the next segment. Outputs go straight to the
// level buffers through st.put<N>(octave, x, y, low dword, high dword, on):
// N pixels, stored by the threads with `on` set.
template <class Store>
__device__ __forceinline__ void pyramid_regs(const Store& st, int O, const uint4* rows, int x0, int y0, int rb,
                                             int seg)
{
    if (O <= 1) return;
    const uint32_t r[4][4] = {{rows[0].x, rows[0].y, rows[0].z, rows[0].w},
                              {rows[1].x, rows[1].y, rows[1].z, rows[1].w},
                              {rows[2].x, rows[2].y, rows[2].z, rows[2].w},
                              {rows[3].x, rows[3].y, rows[3].z, rows[3].w}};
    uint32_t l1[2][2];
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int k = 0; k < 2; ++k) l1[y][k] = mean2x2(r[2 * y][2 * k], r[2 * y][2 * k + 1], r[2 * y + 1][2 * k],
                                                       r[2 * y + 1][2 * k + 1]);
#pragma unroll
    for (int y = 0; y < 2; ++y) st.template put<8>(1, (x0 >> 1) + 8 * seg, (y0 >> 1) + 2 * rb + y, l1[y][0], l1[y][1], true);
    if (O <= 2) return;
    const uint32_t l2 = mean2x2(l1[0][0], l1[0][1], l1[1][0], l1[1][1]);
    st.template put<4>(2, (x0 >> 2) + 4 * seg, (y0 >> 2) + rb, l2, 0u, true);
    if (O <= 3) return;
    // level 3: rows rb (even) and rb + 1, four pixels each -> two pixels
    const uint32_t l2d = (uint32_t)__shfl_down((int)l2, 8);
    const uint32_t l3 = mean2x2(l2, 0u, l2d, 0u) & 0xFFFFu;
    st.template put<2>(3, (x0 >> 3) + 2 * seg, (y0 >> 3) + rb / 2, l3, 0u, (rb & 1) == 0);
    if (O <= 4) return;
    // level 4: level-3 rows rb/2 and rb/2 + 1 (threads rb and rb + 2) -> one pixel
    const uint32_t l3d = (uint32_t)__shfl_down((int)l3, 16);
    const uint32_t l4 = mean2x2(l3, 0u, l3d, 0u) & 0xFFu;
    st.template put<1>(4, (x0 >> 4) + seg, (y0 >> 4) + rb / 4, l4, 0u, (rb & 3) == 0);
    if (O <= 5) return;
    // level 5: level-4 pixels of (rb, seg), (rb, seg + 1), (rb + 4, seg), (rb + 4, seg + 1)
    const uint32_t l4r = (uint32_t)__shfl_down((int)l4, 1);
    const uint32_t l4d = (uint32_t)__shfl_down((int)l4, 32);
    const uint32_t l4dr = (uint32_t)__shfl_down((int)l4, 33);
    const uint32_t l5 = (l4 + l4r + l4d + l4dr + 2) >> 2;
    st.template put<1>(5, (x0 >> 5) + seg / 2, (y0 >> 5) + rb / 8, l5, 0u, (rb & 7) == 0 && (seg & 1) == 0);
}

// Octave stores of the tile pass: level o at a.lvl[o] + lvl_off, clipped to
// the level's size.
struct PxStore {
    const FrameArgs& a;
    size_t lvl_off;
    template <int N>
    __device__ __forceinline__ void put(int o, int gx, int gy, uint32_t lo, uint32_t hi, bool on) const
    {
        if (on) store_px<N>(a.lvl[o] + lvl_off, a.pitch[o], a.w[o], a.h[o], gx, gy, lo, hi);
    }
};

// Raw buffer access (gfx9 resource word 3 for untyped dword data): loads
// past num_records return zeros and stores past it are dropped, so edge
// rows need no branches.
typedef unsigned int v2u __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
constexpr int kRawBufferWord3 = 0x00020000;
constexpr int kNonTemporal = 2;   // cache-policy operand of buffer loads: nt

__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kRawBufferWord3);
}

// Octave stores through buffer resources of the levels' rows (pitch x h
// bytes each): rows below a level, and threads without `on` (sent past the
// range), are dropped by the range check; columns must lie inside the level.
struct BufStore {
    __amdgpu_buffer_rsrc_t r[KPD_MAX_OCTAVES];
    int pitch[KPD_MAX_OCTAVES];
    template <int N>
    __device__ __forceinline__ void put(int o, int gx, int gy, uint32_t lo, uint32_t hi, bool on) const
    {
        const int off = on ? gy * pitch[o] + gx : 0x7FFFFFF0;
        if constexpr (N == 8) __builtin_amdgcn_raw_buffer_store_b64(v2u{lo, hi}, r[o], off, 0, 0);
        else if constexpr (N == 4) __builtin_amdgcn_raw_buffer_store_b32(lo, r[o], off, 0, 0);
        else if constexpr (N == 2) __builtin_amdgcn_raw_buffer_store_b16((unsigned short)lo, r[o], off, 0, 0);
        else __builtin_amdgcn_raw_buffer_store_b8((unsigned char)lo, r[o], off, 0, 0);
    }
};

template <int B>
__device__ void frame_tile_b(const FrameArgs& a, const FrameSrc& f, int bx, int by, uint8_t* sm)
{
    const int T = a.tile;
    const int tid = threadIdx.x;
    const int x0 = bx * T, y0 = by * T;
    const int lgq = __builtin_ctz(T / 4);

    // 1) level-0 loads (and I_{n-1}'s for the SAD), issued first: nothing
    //    they need comes from memory, so their latency overlaps the table
    //    set-up below. 128-px tiles (B = 0): thread (rb, seg) holds rows
    //    4rb..4rb+3, columns 16seg..16seg+15, so eight lanes read a whole
    //    128-byte row; a row segment inside the frame and 16-byte aligned is
    //    one 16-byte load. Smaller tiles: each thread holds one dword column
    //    of the tile, B rows kFrameBlock*4/T apart (T*T/4 <= B*kFrameBlock).
    constexpr int NV = B == 0 ? 4 : B;
    using Word = typename std::conditional<B == 0, uint4, uint32_t>::type;
    Word v[NV], pv[NV];
    const int rb = tid >> 3, seg = tid & 7;   // B = 0
    const int cx = 16 * seg, gxs = x0 + cx;
    const int cq = tid & (T / 4 - 1), gx = x0 + 4 * cq;   // B > 0
    const int ry0 = tid >> lgq, rstep = kFrameBlock >> lgq;
    if constexpr (B == 0) {
        auto load = [&](const uint8_t* row, bool al) -> uint4 {
            const uint8_t* src = row + gxs;
            if (al && gxs + 15 < a.W && (reinterpret_cast<uintptr_t>(src) & 15) == 0)
                return *reinterpret_cast<const uint4*>(src);
            uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int g = gxs + 4 * d;
                if (al && g + 3 < a.W) {
                    w[d] = *reinterpret_cast<const uint32_t*>(src + 4 * d);
                } else {
                    for (int k = 0; k < 4; ++k)
                        if (g + k < a.W) w[d] |= (uint32_t)src[4 * d + k] << (8 * k);
                }
            }
            return make_uint4(w[0], w[1], w[2], w[3]);
        };
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int gy = y0 + 4 * rb + u;
            v[u] = make_uint4(0u, 0u, 0u, 0u);
            pv[u] = v[u];
            if (gy < a.H && gxs < a.W) {
                v[u] = load(f.cur + (size_t)gy * f.cur_pitch, f.cur_aligned);
                if (f.sad_on) pv[u] = load(f.prev + (size_t)gy * f.prev_pitch, f.prev_aligned);
            }
        }
        if (a.O <= kRegOctaves) pyramid_regs(PxStore{a, f.lvl_off}, a.O, v, x0, y0, rb, seg);
    } else {
        auto load = [&](const uint8_t* src, bool al) -> uint32_t {
            if (al) return *reinterpret_cast<const uint32_t*>(src);
            uint32_t w = 0;
            for (int k = 0; k < 4; ++k)
                if (gx + k < a.W) w |= (uint32_t)src[k] << (8 * k);
            return w;
        };
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int ry = ry0 + u * rstep;
            const int gy = y0 + ry;
            v[u] = 0;
            pv[u] = 0;
            if (ry < T && gy < a.H && gx < a.W) {
                v[u] = load(f.cur + (size_t)gy * f.cur_pitch + gx, f.cur_aligned);
                if (f.sad_on) pv[u] = load(f.prev + (size_t)gy * f.prev_pitch + gx, f.prev_aligned);
            }
        }
    }

    // 2) per-level output pointers and sizes (static indices only), and the
    //    tile's column/row -> local cell tables from the stream's maps
    //    (column X is in cell column floor(X * Nc / W)). LDS: level buffers
    //    (T^2, (T/2)^2, ...), then the per-cell SAD partials and the tables.
    __shared__ uint8_t* s_out[KPD_MAX_OCTAVES];
    __shared__ int s_pitch[KPD_MAX_OCTAVES], s_w[KPD_MAX_OCTAVES], s_h[KPD_MAX_OCTAVES];
    if (tid == 0) {
#pragma unroll
        for (int o = 0; o < KPD_MAX_OCTAVES; ++o) {
            s_out[o] = a.lvl[o] + f.lvl_off;
            s_pitch[o] = a.pitch[o];
            s_w[o] = a.w[o];
            s_h[o] = a.h[o];
        }
    }
    uint32_t* sadl = reinterpret_cast<uint32_t*>(sm + a.sad_lds_off);
    uint16_t* colcell = reinterpret_cast<uint16_t*>(sm + a.sad_lds_off + 4 * a.sad_slots);
    uint16_t* rowcell = colcell + T;
    const int xe = min(x0 + T, a.W), ye = min(y0 + T, a.H);
    int cx0 = 0, cy0 = 0, ncx = 1, ncy = 1;
    if (f.sad_on) {
        cx0 = a.colmap[x0];
        cy0 = a.rowmap[y0];
        ncx = a.colmap[xe - 1] - cx0 + 1;
        ncy = a.rowmap[ye - 1] - cy0 + 1;
        for (int i = tid; i < a.sad_slots; i += kFrameBlock) sadl[i] = 0;
        for (int i = tid; i < T; i += kFrameBlock) {
            colcell[i] = (uint16_t)(x0 + i < a.W ? a.colmap[x0 + i] - cx0 : 0);
            rowcell[i] = (uint16_t)(y0 + i < a.H ? a.rowmap[y0 + i] - cy0 : 0);
        }
    }
    __syncthreads();

    // 3) the level-0 tile into LDS, and the SAD against I_{n-1}: the SAD of
    //    consecutive dwords of one cell is summed in a register and added to
    //    the cell's LDS slot when the cell changes; dwords straddling a cell
    //    column border go byte by byte.
    uint8_t* L0 = sm;
    uint32_t acc = 0;
    int acc_slot = -1;
    if constexpr (B == 0) {
        if (a.O > kRegOctaves) {
#pragma unroll
            for (int u = 0; u < 4; ++u) *reinterpret_cast<uint4*>(L0 + (4 * rb + u) * T + cx) = v[u];
        }
        if (f.sad_on) {
            // The thread's 4 x 16 block usually lies in at most two cell
            // columns (its first dword's and its last dword's, each dword in
            // one of them) and two cell rows (its first row's and its last
            // row's): then four register sums, without branches, one LDS
            // atomic each. Pixels outside the frame are zero in both frames
            // and add nothing. Other blocks go pixel by pixel.
            int cc[4];
#pragma unroll
            for (int d = 0; d < 4; ++d) cc[d] = colcell[cx + 4 * d];
            bool two = true;
#pragma unroll
            for (int d = 0; d < 4; ++d) two = two && colcell[cx + 4 * d + 3] == cc[d];
            two = two && (cc[1] == cc[0] || cc[1] == cc[3]) && (cc[2] == cc[0] || cc[2] == cc[3]);
            int rr[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) rr[u] = rowcell[4 * rb + u];
            two = two && (rr[1] == rr[0] || rr[1] == rr[3]) && (rr[2] == rr[0] || rr[2] == rr[3]);
            if (two) {
                uint32_t s00 = 0, s01 = 0, s10 = 0, s11 = 0;   // (first/last row cell, first/last column cell)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t cw[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
                    const uint32_t pw[4] = {pv[u].x, pv[u].y, pv[u].z, pv[u].w};
                    uint32_t sl = 0, sr = 0;
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        const uint32_t sd = __builtin_amdgcn_sad_u8(cw[d], pw[d], 0u);
                        const bool left = cc[d] == cc[0];
                        sl += left ? sd : 0u;
                        sr += left ? 0u : sd;
                    }
                    const bool top = rr[u] == rr[0];
                    s00 += top ? sl : 0u;
                    s01 += top ? sr : 0u;
                    s10 += top ? 0u : sl;
                    s11 += top ? 0u : sr;
                }
                const int t0 = rr[0] * ncx, t1 = rr[3] * ncx;
                if (s00) atomicAdd(&sadl[t0 + cc[0]], s00);
                if (s01) atomicAdd(&sadl[t0 + cc[3]], s01);
                if (s10) atomicAdd(&sadl[t1 + cc[0]], s10);
                if (s11) atomicAdd(&sadl[t1 + cc[3]], s11);
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int rc = rr[u] * ncx;
                    const uint32_t cw[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
                    const uint32_t pw[4] = {pv[u].x, pv[u].y, pv[u].z, pv[u].w};
                    for (int d = 0; d < 4; ++d)
                        for (int k = 0; k < 4; ++k) {
                            const uint32_t m = 0xFFu << (8 * k);
                            const uint32_t sd = __builtin_amdgcn_sad_u8(cw[d] & m, pw[d] & m, 0u);
                            if (sd) atomicAdd(&sadl[rc + colcell[cx + 4 * d + k]], sd);
                        }
                }
            }
        }
    } else {
        const bool straddle = f.sad_on && (gx + 3 >= a.W || colcell[4 * cq] != colcell[4 * cq + 3]);
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int ry = ry0 + u * rstep;
            if (ry >= T) continue;
            *reinterpret_cast<uint32_t*>(L0 + ry * T + 4 * cq) = v[u];
            const int gy = y0 + ry;
            if (!f.sad_on || gy >= a.H || gx >= a.W) continue;
            const int rc = rowcell[ry] * ncx;
            if (!straddle) {
                const int slot = rc + colcell[4 * cq];
                const uint32_t d = __builtin_amdgcn_sad_u8(v[u], pv[u], 0u);
                if (slot != acc_slot) {
                    if (acc_slot >= 0 && acc) atomicAdd(&sadl[acc_slot], acc);
                    acc_slot = slot;
                    acc = 0;
                }
                acc += d;
            } else {
                for (int k = 0; k < 4 && gx + k < a.W; ++k) {
                    const uint32_t m = 0xFFu << (8 * k);
                    atomicAdd(&sadl[rc + colcell[4 * cq + k]], __builtin_amdgcn_sad_u8(v[u] & m, pv[u] & m, 0u));
                }
            }
        }
        if (acc_slot >= 0 && acc) atomicAdd(&sadl[acc_slot], acc);
    }
    __syncthreads();
    if (f.sad_on) {
        for (int i = tid; i < ncx * ncy; i += kFrameBlock) {
            const uint32_t s = sadl[i];
            if (s) atomicAdd(&f.sad[(cy0 + i / ncx) * a.nc + cx0 + i % ncx], s);
        }
    }

    if (B == 0 && a.O <= kRegOctaves) return;   // octaves already written from registers

    // coarser octaves, four outputs per thread while a level row holds >= 4
    int src_off = 0;
    for (int o = 1; o < a.O; ++o) {
        const int ts = T >> o;
        const int dst_off = src_off + 4 * ts * ts;
        const uint8_t* src = sm + src_off;
        uint8_t* dst = sm + dst_off;
        src_off = dst_off;
        const int wo = s_w[o], ho = s_h[o];
        const int gx0 = x0 >> o, gy0 = y0 >> o;
        uint8_t* out = s_out[o];
        const int pitch = s_pitch[o];
        if (ts >= 4) {
            const int q = ts / 4;
            const int lq = __builtin_ctz(q);
            for (int g = tid; g < ts * q; g += kFrameBlock) {
                const int yy = g >> lq, xq = g & (q - 1);
                const uint8_t* r0 = src + (2 * yy) * (2 * ts) + 8 * xq;
                const uint8_t* r1 = r0 + 2 * ts;
                const uint32_t a0 = *reinterpret_cast<const uint32_t*>(r0);
                const uint32_t a1 = *reinterpret_cast<const uint32_t*>(r0 + 4);
                const uint32_t b0 = *reinterpret_cast<const uint32_t*>(r1);
                const uint32_t b1 = *reinterpret_cast<const uint32_t*>(r1 + 4);
                uint32_t packed = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t ra = k < 2 ? a0 : a1, rb = k < 2 ? b0 : b1;
                    const int sh = 16 * (k & 1);
                    const uint32_t s = ((ra >> sh) & 0xFF) + ((ra >> (sh + 8)) & 0xFF) + ((rb >> sh) & 0xFF) +
                                       ((rb >> (sh + 8)) & 0xFF) + 2;
                    packed |= (s >> 2) << (8 * k);
                }
                *reinterpret_cast<uint32_t*>(dst + yy * ts + 4 * xq) = packed;
                const int gy = gy0 + yy, gx = gx0 + 4 * xq;
                if (gy < ho && gx < wo) {
                    uint8_t* p = out + (size_t)gy * pitch + gx;
                    if (gx + 3 < wo) {
                        *reinterpret_cast<uint32_t*>(p) = packed;
                    } else {
                        for (int k = 0; k < 4 && gx + k < wo; ++k) p[k] = (uint8_t)(packed >> (8 * k));
                    }
                }
            }
        } else {
            for (int g = tid; g < ts * ts; g += kFrameBlock) {
                const int yy = g / ts, xx = g % ts;
                const uint8_t* r0 = src + (2 * yy) * (2 * ts) + 2 * xx;
                const uint8_t* r1 = r0 + 2 * ts;
                const uint8_t v = (uint8_t)((r0[0] + r0[1] + r1[0] + r1[1] + 2) >> 2);
                dst[yy * ts + xx] = v;
                const int gy = gy0 + yy, gx = gx0 + xx;
                if (gy < ho && gx < wo) out[(size_t)gy * pitch + gx] = v;
            }
        }
        __syncthreads();
    }
}

// A thread holds T*T/4/kFrameBlock level-0 dwords of its tile: 1, 4 or 16
// for T = 32, 64, 128 (the last as four 16-byte row segments).
__device__ __forceinline__ void frame_tile(const FrameArgs& a, const FrameSrc& f, int bx, int by, uint8_t* sm)
{
    if (a.tile <= 32) frame_tile_b<1>(a, f, bx, by, sm);
    else if (a.tile == 64) frame_tile_b<4>(a, f, bx, by, sm);
    else frame_tile_b<0>(a, f, bx, by, sm);
}

// ----------------------------------------------------------------- k_detect

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

// Necessary condition for a corner at P (row pitch pw): any 9-arc of the 16
// ring pixels holds position k or k+8 for every k, so a bright arc needs one
// of {up, down} and one of {right, left} brighter than p + t (darker than
// p - t for a dark arc).
__device__ __forceinline__ bool compass_pass(const uint8_t* P, int pw, int t)
{
    const int p = P[0];
    const int hi = p + t, lo = p - t;
    const int n = P[-3 * pw], s = P[3 * pw], e = P[3], w = P[-3];
    const bool maybe_b = max(n, s) > hi && max(e, w) > hi;
    const bool maybe_d = min(n, s) < lo && min(e, w) < lo;
    return maybe_b || maybe_d;
}

// Segment test and FAST score of the pixel at P for threshold t (Sec. 2);
// 0 for pixels that are not corners.
__device__ __forceinline__ int full_score(const uint8_t* P, int pw, int t)
{
    const int p = P[0];
    const int hi = p + t, lo = p - t;
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

__device__ __forceinline__ int level_of(const int* start, int O, int i)
{
    int o = 0;
    while (o + 1 < O && i >= start[o + 1]) ++o;
    return o;
}

// Score of level-o pixel (x, y) from the LDS maps. Every pixel the
// suppression reads lies inside its level's map (the query box); pixels
// outside the score box hold 0.
__device__ __forceinline__ int vget(const uint8_t* sm, const CellLayout& L, int o, int x, int y)
{
    const uint16_t* v = reinterpret_cast<const uint16_t*>(sm + L.voff[o]);
    return v[(y - L.qb[o].y0) * L.vpitch[o] + (x - L.qb[o].x0)];
}

// p = (o, x, y) with score v > 0 is a keypoint when no scale-space neighbour
// ranks above it: higher score, or equal score and a finer octave, or equal
// score and octave and an earlier (y, x). All 28 neighbour reads are
// independent, so they are issued together.
__device__ bool is_local_max(const uint8_t* sm, const CellLayout& L, int o, int O, int x, int y, int v)
{
    const uint16_t* V = reinterpret_cast<const uint16_t*>(sm + L.voff[o]);
    const int pv = L.vpitch[o];
    const uint16_t* c = V + (y - L.qb[o].y0) * pv + (x - L.qb[o].x0);
    // in-plane: the three pixels above and the one to the left precede p
    const int before = max(max((int)c[-pv - 1], (int)c[-pv]), max((int)c[-pv + 1], (int)c[-1]));
    const int after = max(max((int)c[1], (int)c[pv - 1]), max((int)c[pv], (int)c[pv + 1]));
    bool keep = before < v && after <= v;
    if (o > 0) {
        const uint16_t* F = reinterpret_cast<const uint16_t*>(sm + L.voff[o - 1]);
        const int pf = L.vpitch[o - 1];
        const uint16_t* f = F + (2 * y - 1 - L.qb[o - 1].y0) * pf + (2 * x - 1 - L.qb[o - 1].x0);
        int m = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int k = 0; k < 4; ++k) m = max(m, (int)f[r * pf + k]);
        keep = keep && m < v;
    }
    if (o + 1 < O) {
        const uint16_t* C = reinterpret_cast<const uint16_t*>(sm + L.voff[o + 1]);
        const int pc = L.vpitch[o + 1];
        const uint16_t* q = C + (((y - 1) >> 1) - L.qb[o + 1].y0) * pc + (((x - 1) >> 1) - L.qb[o + 1].x0);
        const int m = max(max((int)q[0], (int)q[1]), max((int)q[pc], (int)q[pc + 1]));
        keep = keep && m <= v;
    }
    return keep;
}

// Count word of a marked cell: [63:32] frame epoch, [31:0] the cell's number
// of keypoints in D_n. Unmarked cells publish nothing: their count is
// D_{n-1}'s, which every workgroup can read.
constexpr int kSpinLimit = 1 << 20;  // about a second: far beyond any real wait

// Mark decision of cell c (Eq. 2 per cell from the SAD, Eqs. 3-4 from the
// cell's count in D_{n-1}); every workgroup can evaluate it for any cell.
__device__ __forceinline__ bool cell_marked(const DetectArgs& a, int c)
{
    if (a.all_marked) return true;
    const int cx = c % a.nc, cy = c / a.nc;
    const int64_t area = (int64_t)a.col_w[cx] * a.row_h[cy];
    const bool id = a.id_on && (int64_t)a.sad[c] > (int64_t)a.id_thresh * area;
    const bool kb = a.count_prev[c] >= a.kb_thresh;
    return id || kb;
}

// Steps 0-4 for a marked cell c: stage the octave tiles, score, suppress and
// rank. Leaves the keep bitmask and word offsets in LDS and the cell's number
// of keypoints in *s_n (valid after the final barrier).
// Exclusive popcount prefix of nw bitmask words into offs (wave 0 calls it;
// returns the total in lane 63).
__device__ __forceinline__ uint32_t prefix_words(const uint64_t* words, uint32_t* offs, int nw, int lane)
{
    const int per = (nw + 63) / 64;
    const int w0 = lane * per, w1 = min(w0 + per, nw);
    uint32_t sum = 0;
    for (int w = w0; w < w1; ++w) sum += (uint32_t)__popcll(words[w]);
    uint32_t incl = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t up = __shfl_up(incl, off, 64);
        if (lane >= off) incl += up;
    }
    uint32_t run = incl - sum;
    for (int w = w0; w < w1; ++w) {
        offs[w] = run;
        run += (uint32_t)__popcll(words[w]);
    }
    return incl;
}

// Step 4: rank the keep words (word offsets into LDS, the count into *s_n);
// with `carr`, also the word offsets of the carried-entry bits.
__device__ __forceinline__ void rank_words(const CellLayout& L, uint8_t* sm, uint32_t* s_n,
                                           const uint64_t* carr = nullptr, uint32_t* cwoff = nullptr)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (wave == 0) {
        const uint32_t n = prefix_words(reinterpret_cast<const uint64_t*>(sm),
                                        reinterpret_cast<uint32_t*>(sm + L.woff_off), L.nwords, lane);
        if (carr) prefix_words(carr, cwoff, L.nwords, lane);
        if (lane == 63) *s_n = n;
    }
    __syncthreads();
}

template <int NT>
__device__ __forceinline__ void detect_marked(const DetectArgs& a, int t, int lvl0_aligned, int c, uint8_t* sm,
                                              CellLayout& L, const uint8_t* const* s_lvl, const int* s_pitch,
                                              uint32_t* s_n, bool rank = true)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int O = a.O;
    uint64_t* keepw = reinterpret_cast<uint64_t*>(sm);
    // 0) the cell's precomputed layout, one dword per thread
    {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(a.layouts + c);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&L);
        for (int i = tid; i < (int)(sizeof(CellLayout) / 4); i += NT) dst[i] = src[i];
    }
    __syncthreads();
    uint64_t* candw = reinterpret_cast<uint64_t*>(sm + L.cand_off);
    for (int i = tid; i < L.nwords; i += NT) {
        candw[i] = 0;
        keepw[i] = 0;
    }
    {
        uint32_t* v = reinterpret_cast<uint32_t*>(sm + L.voff[0]);
        for (int i = tid; i < L.vbytes / 4; i += NT) v[i] = 0;
    }

    // 1) pixel tiles of every octave, a dword per load, four loads in flight
    const int nld = L.ld_start[O];
    for (int base = tid; base < nld; base += 4 * NT) {
        uint32_t val[4];
        int dst[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = base + u * NT;
            dst[u] = -1;
            val[u] = 0;
            if (i < nld) {
                const int o = level_of(L.ld_start, O, i);
                const unsigned j = i - L.ld_start[o];
                const int q = L.tpitch[o] / 4;
                const int ry = fast_div(j, L.ldm[o]), cq = j - ry * q;
                const int gy = L.ty0[o] + ry, gx = L.tx0[o] + 4 * cq;
                const uint8_t* src = s_lvl[o] + (size_t)gy * s_pitch[o] + gx;
                if (o > 0 || lvl0_aligned) {
                    val[u] = *reinterpret_cast<const uint32_t*>(src);
                } else {
                    uint32_t v = 0;
                    for (int k = 0; k < 4; ++k)
                        if (gx + k < a.W) v |= (uint32_t)src[k] << (8 * k);
                    val[u] = v;
                }
                dst[u] = L.toff[o] + ry * L.tpitch[o] + 4 * cq;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (dst[u] >= 0) *reinterpret_cast<uint32_t*>(sm + dst[u]) = val[u];
    }
    __syncthreads();

    // 2) segment test and score over every octave's score box. A lane takes
    //    a group of four pixels of a score row (one dword of the tile row),
    //    reads the dwords holding their compass points (N and S at rows -3
    //    and +3, E and W shifted out of the neighbouring dwords) and queues
    //    the pixels that pass the four-compass-point test; the full
    //    16-pixel test runs 64 queued pixels at a time, so lanes stay busy.
    {
        uint16_t* queue = reinterpret_cast<uint16_t*>(sm + L.queue_off) + wave * kQueue;
        uint32_t q_tail = 0, q_head = 0;
        auto full_test = [&](int count) {
            if (lane < count) {
                const int i = queue[(q_head + lane) & (kQueue - 1)];
                const int o = level_of(L.sc_start, O, i);
                const unsigned j = i - L.sc_start[o];
                const Box sb = L.sb[o];
                const int ry = fast_div(j, L.scm[o]), rx = j - ry * box_w(sb);
                const uint8_t* P = sm + L.toff[o] + (ry + kRingR) * L.tpitch[o] + (sb.x0 + rx - L.tx0[o]);
                const int v = full_score(P, L.tpitch[o], t);
                const int x = sb.x0 + rx, y = sb.y0 + ry;
                if (v > 0) {
                    reinterpret_cast<uint16_t*>(sm + L.voff[o])[(y - L.qb[o].y0) * L.vpitch[o] + (x - L.qb[o].x0)] =
                        (uint16_t)v;
                    const Box d = L.dec[o];
                    if (x >= d.x0 && x < d.x1 && y >= d.y0 && y < d.y1) {
                        const int bit = L.dc_start[o] + (y - d.y0) * box_w(d) + (x - d.x0);
                        atomicOr(&candw[bit >> 6], 1ull << (bit & 63));
                    }
                }
            }
            q_head += count;
        };
        const int nck = L.ck_start[O];
        for (int ck = wave; ck < nck; ck += (NT / 64)) {
            const int o = level_of(L.ck_start, O, ck);
            const Box sb = L.sb[o];
            const int tp = L.tpitch[o], tx0 = L.tx0[o];
            const int ngx = L.ngx[o], gx0 = L.gx0[o];
            const int wsb = box_w(sb);
            const int lo_col = sb.x0 - tx0, hi_col = sb.x1 - tx0;   // score columns in the tile
            const int sc0 = L.sc_start[o];
            const uint8_t* base = sm + L.toff[o] + kRingR * tp;      // tile row of score row 0
            const int g = (ck - L.ck_start[o]) * 64 + lane;
            uint32_t pass = 0;
            int ry = 0, cx = 0;
            if (g < ngx * box_h(sb)) {
                ry = fast_div(g, L.gcm[o]);
                cx = 4 * (gx0 + g - ry * ngx);
                const uint8_t* P = base + ry * tp + cx;
                const uint32_t c = *reinterpret_cast<const uint32_t*>(P);
                const uint32_t cm = *reinterpret_cast<const uint32_t*>(P - 4);
                const uint32_t cp = *reinterpret_cast<const uint32_t*>(P + 4);
                const uint32_t nw = *reinterpret_cast<const uint32_t*>(P - 3 * tp);
                const uint32_t sw = *reinterpret_cast<const uint32_t*>(P + 3 * tp);
                const uint32_t ew = __builtin_amdgcn_alignbyte(cp, c, 3);   // bytes x+3
                const uint32_t ww = __builtin_amdgcn_alignbyte(c, cm, 1);   // bytes x-3
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int sh = 8 * k;
                    const int p = (c >> sh) & 0xFF;
                    const int n = (nw >> sh) & 0xFF, so = (sw >> sh) & 0xFF;
                    const int e = (ew >> sh) & 0xFF, w = (ww >> sh) & 0xFF;
                    const int hi = p + t, lo = p - t;
                    const bool b = min(max(n, so), max(e, w)) > hi;
                    const bool d = max(min(n, so), min(e, w)) < lo;
                    const bool in = cx + k >= lo_col && cx + k < hi_col;
                    pass |= (uint32_t)((b || d) && in) << k;
                }
            }
            const int idx0 = sc0 + ry * wsb + (cx - lo_col);   // score index of byte 0
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool pk = (pass >> k) & 1;
                const uint64_t bal = __ballot(pk);
                if (pk) {
                    const unsigned below = __builtin_amdgcn_mbcnt_hi(
                        (unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
                    queue[(q_tail + below) & (kQueue - 1)] = (uint16_t)(idx0 + k);
                }
                q_tail += (uint32_t)__popcll(bal);
            }
            __builtin_amdgcn_wave_barrier();
            while (q_tail - q_head >= 64) {
                full_test(64);
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (q_tail != q_head) full_test((int)(q_tail - q_head));
    }
    __syncthreads();

    // 3) scale-space maxima of the candidates. Each wave scans 64 candidate
    //    words at a time (one per lane), queues the candidates' decision
    //    indices in its LDS queue, and runs the neighbourhood test on 64
    //    queued candidates at a time; survivors set their keep bit.
    {
        uint16_t* queue = reinterpret_cast<uint16_t*>(sm + L.queue_off) + wave * kQueue;
        uint32_t q_head = 0, q_tail = 0;
        auto nms = [&](int count) {
            if (lane < count) {
                const int i = queue[(q_head + lane) & (kQueue - 1)];
                const int o = level_of(L.dc_start, O, i);
                const unsigned j = i - L.dc_start[o];
                const Box d = L.dec[o];
                const int ry = fast_div(j, L.dcm[o]);
                const int x = d.x0 + (int)(j - ry * box_w(d)), y = d.y0 + ry;
                if (is_local_max(sm, L, o, O, x, y, vget(sm, L, o, x, y)))
                    atomicOr(&keepw[i >> 6], 1ull << (i & 63));
            }
            q_head += count;
        };
        constexpr uint32_t kWindow = kQueue - 64;   // entries added between drains
        const int nw = L.nwords;
        for (int w0 = wave * 64; w0 < nw; w0 += (NT / 64) * 64) {
            const int w = w0 + lane;
            const uint64_t word = w < nw ? candw[w] : 0ull;
            const uint32_t cnt = (uint32_t)__popcll(word);
            uint32_t incl = cnt;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t up = __shfl_up(incl, off, 64);
                if (lane >= off) incl += up;
            }
            const uint32_t total = __shfl(incl, 63, 64);
            const uint32_t excl = incl - cnt;
            for (uint32_t win = 0; win < total; win += kWindow) {
                const uint32_t wend = min(win + kWindow, total);
                if (excl < wend && excl + cnt > win) {
                    uint64_t b = word;
                    uint32_t e = excl;
                    while (b) {
                        const int k = __builtin_ctzll(b);
                        b &= b - 1;
                        if (e >= win && e < wend) queue[(q_tail + e - win) & (kQueue - 1)] = (uint16_t)(w * 64 + k);
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

    // 4) rank: exclusive popcount prefix over the keep words (wave 0)
    if (rank) rank_words(L, sm, s_n);
}

// Step 6 for a marked cell: write its ranked maxima from position excl on.
template <int NT>
__device__ __forceinline__ void emit_marked(const DetectArgs& a, const CellLayout& L, const uint8_t* sm, uint32_t excl,
                            kpd_keypoint* list, uint32_t cap)
{
    const int tid = threadIdx.x;
    const int O = a.O;
    const uint64_t* keepw = reinterpret_cast<const uint64_t*>(sm);
    const uint32_t* woff = reinterpret_cast<const uint32_t*>(sm + L.woff_off);
    for (int w = tid; w < L.nwords; w += NT) {
        uint64_t bits = keepw[w];
        uint32_t pos = excl + woff[w];
        while (bits) {
            const int b = __builtin_ctzll(bits);
            bits &= bits - 1;
            const int i = w * 64 + b;
            const int o = level_of(L.dc_start, O, i);
            const unsigned j = i - L.dc_start[o];
            const Box d = L.dec[o];
            const int ry = fast_div(j, L.dcm[o]);
            const int x = d.x0 + (int)(j - ry * box_w(d)), y = d.y0 + ry;
            kpd_keypoint k;
            k.x = (uint16_t)x;
            k.y = (uint16_t)y;
            k.octave = (uint8_t)o;
            k.pad = 0;
            k.score = (uint16_t)vget(sm, L, o, x, y);
            // at most one keypoint per 2x2 block keeps pos below the capacity
            if (pos < cap) {
                list[pos] = k;
                if (a.src_cur) a.src_cur[pos] = kNewFeature;
            }
            ++pos;
        }
    }
}

// Step 6 for a cell that keeps some new maxima and carries some D_{n-1}
// entries: the ranked union in decision order, carried entries with their
// previous scores (the k-th carried bit takes cscore[k]).
template <int NT>
__device__ __forceinline__ void emit_merged(const DetectArgs& a, const CellLayout& L, const uint8_t* sm,
                                            uint32_t excl, kpd_keypoint* list, uint32_t cap, const uint64_t* carr,
                                            const uint32_t* cwoff, const uint16_t* cscore, const uint32_t* csrc)
{
    const int O = a.O;
    const uint64_t* keepw = reinterpret_cast<const uint64_t*>(sm);
    const uint32_t* woff = reinterpret_cast<const uint32_t*>(sm + L.woff_off);
    for (int w = threadIdx.x; w < L.nwords; w += NT) {
        uint64_t bits = keepw[w];
        const uint64_t cb = carr[w];
        uint32_t pos = excl + woff[w];
        while (bits) {
            const int b = __builtin_ctzll(bits);
            bits &= bits - 1;
            const int i = w * 64 + b;
            const int o = level_of(L.dc_start, O, i);
            const unsigned j = i - L.dc_start[o];
            const Box d = L.dec[o];
            const int ry = fast_div(j, L.dcm[o]);
            const int x = d.x0 + (int)(j - ry * box_w(d)), y = d.y0 + ry;
            kpd_keypoint k;
            k.x = (uint16_t)x;
            k.y = (uint16_t)y;
            k.octave = (uint8_t)o;
            k.pad = 0;
            const bool carried = ((cb >> b) & 1) != 0;
            const uint32_t r = carried ? cwoff[w] + (uint32_t)__popcll(cb & ((1ull << b) - 1)) : 0u;
            k.score = carried ? cscore[r] : (uint16_t)vget(sm, L, o, x, y);
            if (pos < cap) {
                list[pos] = k;
                if (a.src_cur) a.src_cur[pos] = carried ? csrc[r] : kNewFeature;
            }
            ++pos;
        }
    }
}

// Sum over cells [0, c) of their count words for `epoch`, spinning on each
// until it is published (block-wide; the result is valid in every thread).
template <int NT>
__device__ uint32_t sum_count_words(const unsigned long long* words, int c, uint32_t epoch, uint32_t* err,
                                    uint32_t* s_part)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    uint32_t acc = 0;
    bool ok = true;
    for (int p = tid; p < c; p += NT) {
        int spins = 0;
        while (true) {
            const uint64_t st = __hip_atomic_load(&words[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((uint32_t)(st >> 32) == epoch) {
                acc += (uint32_t)st;
                break;
            }
            if (++spins > kSpinLimit) { ok = false; break; }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    if (!ok) __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    __syncthreads();
    if (lane == 0) s_part[wave] = acc;
    __syncthreads();
    uint32_t sum = 0;
    for (int w = 0; w < (NT / 64); ++w) sum += s_part[w];
    return sum;
}

__device__ void load_level_ptrs(const DetectArgs& a, const uint8_t** s_lvl, int* s_pitch)
{
#pragma unroll
    for (int o = 0; o < KPD_MAX_OCTAVES; ++o) {
        s_lvl[o] = a.lvl[o];
        s_pitch[o] = a.pitch[o];
    }
}

// One frame of one stream with per-pixel masks (Sec. 3.1): one mask on a
// chosen pyramid layer for all octaves (id_mode 1), or one mask per octave on
// its own level (id_mode 2). Cell c compares its pixels of those layers in
// I_n and I_{n-1}. A cell with no changed pixel carries D_{n-1}; a cell
// marked by T_H detects everything; otherwise it keeps the new maxima whose
// mask pixel changed and the D_{n-1} entries whose mask pixel did not (Eq. 1
// per feature), merged in decision order. Every cell publishes its count
// word, and offsets wait on all earlier cells.
template <int NT>
__device__ void detect_cell_layer(const DetectArgs& a, int c, uint8_t* sm)
{
    __shared__ CellLayout L;
    __shared__ int s_touched;
    __shared__ uint32_t s_n, s_base, s_part[(NT / 64)];
    __shared__ const uint8_t* s_lvl[KPD_MAX_OCTAVES];
    __shared__ int s_pitch[KPD_MAX_OCTAVES];
    // per mask layer: the cell's first pixel and width on it, and where its
    // bits start in the bit map (a multiple of 64)
    __shared__ int s_kx0[KPD_MAX_OCTAVES], s_ky0[KPD_MAX_OCTAVES], s_nx[KPD_MAX_OCTAVES], s_npx[KPD_MAX_OCTAVES];
    __shared__ int s_boff[KPD_MAX_OCTAVES];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const bool one = a.id_mode == 1;
    const int l_lo = one ? a.id_layer : 0, l_hi = one ? a.id_layer : a.O - 1;
    uint32_t* bits = reinterpret_cast<uint32_t*>(sm + a.lds_bits);
    if (tid == 0) {
        load_level_ptrs(a, s_lvl, s_pitch);
        s_touched = 0;
        // the layer pixels the cell's level-0 pixels map to (clamped into the layer)
        const Box r = cell_rect(c, a.W, a.H, a.nc, a.nr);
        int boff = 0;
        for (int l = l_lo; l <= l_hi; ++l) {
            const int lw = a.w[l], lh = a.h[l];
            const int kx0 = min(r.x0 >> l, lw - 1), kx1 = min((r.x1 - 1) >> l, lw - 1);
            const int ky0 = min(r.y0 >> l, lh - 1), ky1 = min((r.y1 - 1) >> l, lh - 1);
            s_kx0[l] = kx0;
            s_ky0[l] = ky0;
            s_nx[l] = kx1 - kx0 + 1;
            s_npx[l] = s_nx[l] * (ky1 - ky0 + 1);
            s_boff[l] = boff;
            boff += (s_npx[l] + 63) & ~63;
        }
    }
    __syncthreads();
    const bool kb = a.count_prev[c] >= a.kb_thresh;
    if (!kb) {
        for (int l = l_lo; l <= l_hi; ++l) {
            const int nx = s_nx[l], npx = s_npx[l], kx0 = s_kx0[l], ky0 = s_ky0[l], boff = s_boff[l];
            const uint8_t* cur = s_lvl[l];
            const uint8_t* prv = a.lprev[l];
            const int cp = s_pitch[l], pp = a.lprev_pitch[l];
            for (int base = 0; base < npx; base += NT) {
                const int i = base + tid;
                bool ch = false;
                if (i < npx) {
                    const int ry = i / nx, rx = i - ry * nx;
                    const int vc = cur[(size_t)(ky0 + ry) * cp + kx0 + rx];
                    const int vp = prv[(size_t)(ky0 + ry) * pp + kx0 + rx];
                    ch = abs(vc - vp) > a.id_thresh;
                }
                const uint64_t bal = __ballot(ch);
                if (lane == 0 && base + wave * 64 < npx) {   // the layer's bits are npx rounded up to 64
                    const int w0 = (boff + base + wave * 64) >> 5;
                    bits[w0] = (uint32_t)bal;
                    bits[w0 + 1] = (uint32_t)(bal >> 32);
                    if (bal) s_touched = 1;
                }
            }
        }
    }
    __syncthreads();
    const int state = kb ? 2 : (s_touched ? 1 : 0);   // full, partial, carried
    if (tid == 0) {
        a.mask[c] = (uint8_t)(state != 0);
        a.sad_next[c] = 0;
    }
    if (state) detect_marked<NT>(a, a.t, a.lvl0_aligned, c, sm, L, s_lvl, s_pitch, &s_n, state == 2);
    uint64_t* carr = reinterpret_cast<uint64_t*>(sm + a.lds_carr);
    uint32_t* cwoff = reinterpret_cast<uint32_t*>(sm + a.lds_cwoff);
    uint16_t* cscore = reinterpret_cast<uint16_t*>(sm + a.lds_cscore);
    uint32_t* csrc = reinterpret_cast<uint32_t*>(sm + a.lds_csrc);   // with features: carried entries' sources
    if (state == 1) {
        uint64_t* keepw = reinterpret_cast<uint64_t*>(sm);
        // the mask pixel of the feature at level o, (x,y): on the chosen
        // layer at its level-0 position, or on level o itself
        auto changed_at = [&](int o, int x, int y) -> bool {
            const int l = one ? l_lo : o;
            const int kx = min((x << o) >> l, a.w[l] - 1) - s_kx0[l];
            const int ky = min((y << o) >> l, a.h[l] - 1) - s_ky0[l];
            const int i = s_boff[l] + ky * s_nx[l] + kx;
            return (bits[i >> 5] >> (i & 31)) & 1u;
        };
        // new maxima only where the mask is 1
        for (int w = tid; w < L.nwords; w += NT) {
            uint64_t k = keepw[w], out = k;
            while (k) {
                const int b = __builtin_ctzll(k);
                k &= k - 1;
                const int i = w * 64 + b;
                const int o = level_of(L.dc_start, a.O, i);
                const unsigned j = i - L.dc_start[o];
                const Box d = L.dec[o];
                const int ry = fast_div(j, L.dcm[o]);
                if (!changed_at(o, d.x0 + (int)(j - ry * box_w(d)), d.y0 + ry)) out &= ~(1ull << b);
            }
            keepw[w] = out;
            carr[w] = 0;
        }
        if (tid == 0) s_base = 0;
        __syncthreads();
        // D_{n-1}'s entries of the cell where the mask is 0, in order
        const uint32_t n0 = a.count_prev[c], src0 = a.off_prev[c];
        for (uint32_t b0 = 0; b0 < n0; b0 += NT) {
            const uint32_t jj = b0 + tid;
            bool keep = false;
            kpd_keypoint e{};
            if (jj < n0 && src0 + jj < a.list_cap) {
                e = a.list_prev[src0 + jj];
                const Box d = L.dec[e.octave < a.O ? e.octave : 0];
                keep = e.octave < a.O && e.x >= d.x0 && e.x < d.x1 && e.y >= d.y0 && e.y < d.y1 &&
                       !changed_at(e.octave, e.x, e.y);
            }
            const uint64_t bal = __ballot(keep);
            if (lane == 0) s_part[wave] = (uint32_t)__popcll(bal);
            __syncthreads();
            uint32_t before = s_base, total = 0;
            for (int w = 0; w < (NT / 64); ++w) {
                if (w < wave) before += s_part[w];
                total += s_part[w];
            }
            if (keep) {
                const unsigned below = __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
                cscore[before + below] = e.score;
                if (a.src_cur) csrc[before + below] = src0 + jj;
                const int o = e.octave;
                const Box d = L.dec[o];
                const int i = L.dc_start[o] + (e.y - d.y0) * box_w(d) + (e.x - d.x0);
                atomicOr(&carr[i >> 6], 1ull << (i & 63));
            }
            __syncthreads();
            if (tid == 0) s_base += total;
            __syncthreads();
        }
        for (int w = tid; w < L.nwords; w += NT) keepw[w] |= carr[w];
        __syncthreads();
        rank_words(L, sm, &s_n, carr, cwoff);
    }

    // offsets: every cell publishes its count word
    if (tid == 0) {
        const uint32_t own = state ? s_n : a.count_prev[c];
        s_n = own;
        __hip_atomic_store(&a.status[c], ((uint64_t)a.epoch << 32) | own, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const uint32_t excl = sum_count_words<NT>(a.status, c, a.epoch, a.err, s_part);
    const uint32_t n = s_n;
    if (tid == 0) {
        a.count_cur[c] = n;
        a.off_cur[c] = excl;
        if (c == a.nc * a.nr - 1) *a.total_cur = excl + n;
    }
    if (state == 2) {
        emit_marked<NT>(a, L, sm, excl, a.list_cur, a.list_cap);
    } else if (state == 1) {
        emit_merged<NT>(a, L, sm, excl, a.list_cur, a.list_cap, carr, cwoff, cscore, csrc);
    } else {
        const uint32_t src0 = a.off_prev[c];
        for (uint32_t j = tid; j < n; j += NT)
            if (src0 + j < a.list_cap && excl + j < a.list_cap) a.list_cur[excl + j] = a.list_prev[src0 + j];
    }
}

// One frame of one stream: cell c's mark, detection, offset and output.
template <int NT>
__device__ void detect_cell(const DetectArgs& a, int c, uint8_t* sm)
{
    if (a.id_mode != 0 && !a.all_marked) {
        detect_cell_layer<NT>(a, c, sm);
        return;
    }
    __shared__ CellLayout L;
    __shared__ int s_mark;
    __shared__ uint32_t s_n, s_excl, s_part[(NT / 64)];
    __shared__ const uint8_t* s_lvl[KPD_MAX_OCTAVES];
    __shared__ int s_pitch[KPD_MAX_OCTAVES];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;

    if (tid == 0) {
        load_level_ptrs(a, s_lvl, s_pitch);
        const bool mark = cell_marked(a, c);
        a.mask[c] = (uint8_t)mark;
        a.sad_next[c] = 0;
        s_mark = mark;
    }
    __syncthreads();
    const bool mark = s_mark != 0;
    if (mark) detect_marked<NT>(a, a.t, a.lvl0_aligned, c, sm, L, s_lvl, s_pitch, &s_n);

    // 5) this cell's offset in D_n: the counts of all earlier cells, carried
    //    ones read from D_{n-1}'s counts, marked ones from their count words
    if (tid == 0) {
        const uint32_t own = mark ? s_n : a.count_prev[c];
        s_n = own;
        if (mark)
            __hip_atomic_store(&a.status[c], ((uint64_t)a.epoch << 32) | own, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t acc = 0;
    bool ok = true;
    for (int p = tid; p < c; p += NT) {
        if (!cell_marked(a, p)) {
            acc += a.count_prev[p];
            continue;
        }
        int spins = 0;
        while (true) {
            const uint64_t st = __hip_atomic_load(&a.status[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((uint32_t)(st >> 32) == a.epoch) {
                acc += (uint32_t)st;
                break;
            }
            if (++spins > kSpinLimit) { ok = false; break; }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    if (!ok) __hip_atomic_store(a.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) s_part[wave] = acc;
    __syncthreads();
    if (tid == 0) {
        uint32_t excl = 0;
        for (int w = 0; w < (NT / 64); ++w) excl += s_part[w];
        a.count_cur[c] = s_n;
        a.off_cur[c] = excl;
        if (c == a.nc * a.nr - 1) *a.total_cur = excl + s_n;
        s_excl = excl;
    }
    __syncthreads();
    const uint32_t excl = s_excl, n = s_n;

    // 6) write D_n entries of this cell: the ranked maxima, or D_{n-1}'s
    if (mark) {
        emit_marked<NT>(a, L, sm, excl, a.list_cur, a.list_cap);
    } else {
        const uint32_t src0 = a.off_prev[c];
        for (uint32_t j = tid; j < n; j += NT)
            if (src0 + j < a.list_cap && excl + j < a.list_cap) a.list_cur[excl + j] = a.list_prev[src0 + j];
    }
}

// Frame j of a chunk marks every cell: frame 0 after a first frame, reset or
// new t, or every frame when the parameters say so.
__device__ __forceinline__ bool chunk_all_marked(const ChunkHead& h, int j)
{
    return h.all_marked || (j == 0 && h.force0);
}

// ----------------------------------------------------------------- kernels

// ------------------------------------------------------------ k_describe

// Sub-pixel, sub-scale refinement of one feature (Sec. 2's interpolation on
// the octave layers). S holds the FAST scores of the 3 x 3 patches on the
// finer, own and coarser layers (S[9k + 3(i+1) + (j+1)], x offset i, y
// offset j). Per layer, an exact integer least-squares quadratic gives its
// maximum (clamped to a pixel; the centre when not concave) and the value
// there; a parabola through the three values along log2 scale gives t. The
// floating steps are IEEE double operations in a fixed order, none fused.
__device__ kpd_refined refine_feature(const int* S, int x, int y, int o, int O)
{
#pragma clang fp contract(off)
    double m[3] = {0.0, 0.0, 0.0}, X[3] = {0.0, 0.0, 0.0}, Y[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int l = o - 1 + k;
        if (l < 0 || l >= O) continue;
        const int cx = k == 0 ? 2 * x + 1 : (k == 1 ? x : x >> 1);
        const int cy = k == 0 ? 2 * y + 1 : (k == 1 ? y : y >> 1);
        const Fit f = fit_patch(S + 9 * k);
        m[k] = f.m;
        X[k] = (((double)cx + 0.5) + f.u) * (double)(1 << l);
        Y[k] = (((double)cy + 0.5) + f.v) * (double)(1 << l);
    }
    if (o == 0) { X[0] = X[1]; Y[0] = Y[1]; }
    if (o + 1 >= O) { X[2] = X[1]; Y[2] = Y[1]; }
    const double q = (m[0] - 2.0 * m[1]) + m[2];
    double tt = 0.0;
    if (q < 0.0) tt = fmin(fmax((m[0] - m[2]) / (2.0 * q), -1.0), 1.0);
    const double score = (m[1] + (0.5 * (m[2] - m[0])) * tt) + (0.5 * q) * (tt * tt);
    const int side = tt >= 0.0 ? 2 : 0;
    const double a = tt >= 0.0 ? tt : -tt;
    kpd_refined r;
    r.x = (float)(X[1] + a * (X[side] - X[1]));
    r.y = (float)(Y[1] + a * (Y[side] - Y[1]));
    r.log2_scale = (float)((double)o + tt);
    r.score = (float)score;
    return r;
}

// Features (Sec. 3 feature model; Eq. 1 carries whole features). New
// features are computed by the waves of a workgroup, one feature at a time
// each. Refinement: 27 lanes score one pixel each of the three 3 x 3
// patches and one lane fits them. Descriptor: the wave loads the feature's
// 27 x 27 patch (every point of the pattern, turned any way, with its box)
// into LDS in one round of loads, a lane per pattern point takes the box
// mean around its point, the lanes sum the long pairs' gradient, 32 lanes
// test the sector boundaries, the points are taken again turned to the
// sector, and eight ballots over the short pairs give the bits. Carried
// features keep the records they were computed with, copied in order.
constexpr int kDescBlock = 256;
constexpr int kPatchR = 13;                  // pattern radius 11 plus a box half-size 2
constexpr int kPatch = 2 * kPatchR + 1;      // patch side

// Copies the records of n features from entry src0 of one list to entry
// dst0 of another (a null descriptor or refined destination leaves that
// part out); entries past list_cap on either side are left out.
__device__ void copy_feature_records(const kpd_descriptor* dsrc, kpd_descriptor* ddst, const kpd_refined* rsrc,
                                     kpd_refined* rdst, uint32_t src0, uint32_t dst0, uint32_t n, uint32_t list_cap)
{
    if (ddst) {
        constexpr int kw = sizeof(kpd_descriptor) / 8;
        const uint64_t* src = reinterpret_cast<const uint64_t*>(dsrc);
        uint64_t* dst = reinterpret_cast<uint64_t*>(ddst);
        for (uint32_t i = threadIdx.x; i < n * kw; i += kDescBlock) {
            const uint32_t e = i / kw;
            if (src0 + e < list_cap && dst0 + e < list_cap)
                dst[(size_t)(dst0 + e) * kw + i % kw] = src[(size_t)(src0 + e) * kw + i % kw];
        }
    }
    if (rdst)
        for (uint32_t e = threadIdx.x; e < n; e += kDescBlock)
            if (src0 + e < list_cap && dst0 + e < list_cap) rdst[dst0 + e] = rsrc[src0 + e];
}

// Features of entries [dst0, dst0 + n) of a keypoint list, computed on the
// levels of their frame (lv: ptr, pitch, w and h of octave o) into the same
// entries of desc and ref (either may be null: that part is left out; tab
// is null exactly when desc is). With src, entries whose source is not
// kNewFeature are left to the caller.
template <class Lv>
__device__ void describe_entries(const Lv& lv, const DescTables* tab, int O, int t, const kpd_keypoint* list,
                                 kpd_descriptor* desc, kpd_refined* ref, uint32_t dst0, uint32_t n,
                                 uint32_t list_cap, int (*s_v)[64], uint8_t (*s_patch)[kPatch * kPatch],
                                 const uint32_t* src = nullptr)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int* V = s_v[wave];
    uint8_t* patch = s_patch[wave];
    for (uint32_t k = wave; k < n; k += kDescBlock / 64) {
        if (dst0 + k >= list_cap) break;
        if (src && src[dst0 + k] != kNewFeature) continue;   // a carried feature keeps its records
        const kpd_keypoint kp = list[dst0 + k];
        const int o = kp.octave;
        if (ref) {
            if (lane < 27) {
                const int kl = lane / 9, r = lane - 9 * kl, i = r / 3 - 1, j = r - 3 * (r / 3) - 1;
                const int l = o - 1 + kl;
                int sc = 0;
                if (l >= 0 && l < O) {
                    const int x = kl == 0 ? 2 * (int)kp.x + 1 : (kl == 1 ? (int)kp.x : (int)kp.x >> 1);
                    const int y = kl == 0 ? 2 * (int)kp.y + 1 : (kl == 1 ? (int)kp.y : (int)kp.y >> 1);
                    const int px = x + i, py = y + j;
                    if (px >= 3 && py >= 3 && px < lv.w(l) - 3 && py < lv.h(l) - 3)
                        sc = full_score(lv.ptr(l) + (size_t)py * lv.pitch(l) + px, lv.pitch(l), t);
                }
                V[lane] = sc;
            }
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) ref[dst0 + k] = refine_feature(V, kp.x, kp.y, o, O);
            __builtin_amdgcn_wave_barrier();   // V is reused below
        }
        if (!tab) continue;
        const DescTables& T = *tab;
        const uint8_t* L = lv.ptr(o);
        const int pitch = lv.pitch(o), w = lv.w(o), h = lv.h(o);
        // the patch around the feature, edge pixels repeated
        constexpr int kPer = (kPatch * kPatch + 63) / 64;
        uint8_t px[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int q = u * 64 + lane;
            px[u] = 0;
            if (q < kPatch * kPatch) {
                const int py = q / kPatch, pxx = q - py * kPatch;
                const int yy = min(max((int)kp.y + py - kPatchR, 0), h - 1);
                const int xx = min(max((int)kp.x + pxx - kPatchR, 0), w - 1);
                px[u] = L[(size_t)yy * pitch + xx];
            }
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int q = u * 64 + lane;
            if (q < kPatch * kPatch) patch[q] = px[u];
        }
        __builtin_amdgcn_wave_barrier();
        // box mean of point i turned to sector sct
        auto value = [&](int sct, int i) -> int {
            const int cx = kPatchR + T.pt[sct][i][0], cy = kPatchR + T.pt[sct][i][1], r = T.half[i];
            int sum = 0;
            for (int yy = cy - r; yy <= cy + r; ++yy)
                for (int xx = cx - r; xx <= cx + r; ++xx) sum += patch[yy * kPatch + xx];
            return sum * (225 / ((2 * r + 1) * (2 * r + 1)));
        };
        if (lane < kDescPts) V[lane] = value(0, lane);
        __builtin_amdgcn_wave_barrier();
        long long gx = 0, gy = 0;
        for (int q = lane; q < T.nlong; q += 64) {
            const int dv = V[T.lp[q][1]] - V[T.lp[q][0]];
            gx += (long long)T.ld[q][0] * dv;
            gy += (long long)T.ld[q][1] * dv;
        }
        for (int off = 32; off > 0; off >>= 1) {
            gx += __shfl_xor(gx, off);
            gy += __shfl_xor(gy, off);
        }
        bool in = false;
        if (lane < kDescSectors) {
            const int nx = (lane + 1) & (kDescSectors - 1);
            in = T.ux[lane] * gy - T.uy[lane] * gx >= 0 && T.ux[nx] * gy - T.uy[nx] * gx < 0;
        }
        const uint64_t sec = __ballot(in);
        const int sector = (gx == 0 && gy == 0) || !sec ? 0 : __builtin_ctzll(sec);
        if (lane < kDescPts) V[lane] = value(sector, lane);
        __builtin_amdgcn_wave_barrier();
        uint64_t mine = 0;
#pragma unroll
        for (int r = 0; r < kDescBits / 64; ++r) {
            const int q = r * 64 + lane;
            const uint64_t b = __ballot(V[T.sp[q][0]] > V[T.sp[q][1]]);
            if (lane == r) mine = b;
        }
        kpd_descriptor* D = desc + dst0 + k;
        if (lane < kDescBits / 64) D->bits[lane] = mine;
        if (lane == kDescBits / 64) {
            D->sector = (uint32_t)sector;
            D->pad = 0;
        }
        __builtin_amdgcn_wave_barrier();   // V is reused by the wave's next feature
    }
}

// The levels of one frame as the single-frame arguments give them.
struct DescLevels {
    const DescArgs& a;
    __device__ const uint8_t* ptr(int o) const { return a.lvl[o]; }
    __device__ int pitch(int o) const { return a.pitch[o]; }
    __device__ int w(int o) const { return a.w[o]; }
    __device__ int h(int o) const { return a.h[o]; }
};

// The records of a marked cell's carried entries (per-pixel masks: an
// entry whose source is an index of D_{n-1}'s list).
__device__ void copy_carried_records(const uint32_t* src, const kpd_descriptor* dsrc, kpd_descriptor* ddst,
                                     const kpd_refined* rsrc, kpd_refined* rdst, uint32_t dst0, uint32_t n,
                                     uint32_t list_cap)
{
    constexpr int kw = sizeof(kpd_descriptor) / 8;
    for (uint32_t i = threadIdx.x; i < n * kw; i += kDescBlock) {
        const uint32_t e = i / kw;
        if (dst0 + e >= list_cap) break;
        const uint32_t f = src[dst0 + e];
        if (f == kNewFeature || f >= list_cap) continue;
        if (ddst)
            reinterpret_cast<uint64_t*>(ddst)[(size_t)(dst0 + e) * kw + i % kw] =
                reinterpret_cast<const uint64_t*>(dsrc)[(size_t)f * kw + i % kw];
        if (rdst && i % kw == 0) rdst[dst0 + e] = rsrc[f];
    }
}

// One frame, a workgroup per cell: an unmarked cell's features are
// D_{n-1}'s, copied; a marked cell's are new, or with a per-pixel mask new
// where the mask pixel changed and copied from D_{n-1} elsewhere.
__global__ __launch_bounds__(kDescBlock) void k_describe1(DescArgs a)
{
    __shared__ int s_v[kDescBlock / 64][64];
    __shared__ uint8_t s_patch[kDescBlock / 64][kPatch * kPatch];
    const int c = blockIdx.x;
    const uint32_t n = a.count_cur[c], dst0 = a.off_cur[c];
    if (!a.mask[c]) {
        copy_feature_records(a.desc_prev, a.tab ? a.desc_cur : nullptr, a.ref_prev, a.ref_cur, a.off_prev[c], dst0, n,
                             a.list_cap);
        return;
    }
    if (a.src_cur)
        copy_carried_records(a.src_cur, a.desc_prev, a.tab ? a.desc_cur : nullptr, a.ref_prev, a.ref_cur, dst0, n,
                             a.list_cap);
    describe_entries(DescLevels{a}, a.tab, a.O, a.t, a.list_cur, a.desc_cur, a.ref_cur, dst0, n, a.list_cap, s_v,
                     s_patch, a.src_cur);
}

// The levels of a batch tick's stream, from its detection arguments.
struct TickLevels {
    const DetectArgs& d;
    __device__ const uint8_t* ptr(int o) const { return d.lvl[o]; }
    __device__ int pitch(int o) const { return d.pitch[o]; }
    __device__ int w(int o) const { return d.w[o]; }
    __device__ int h(int o) const { return d.h[o]; }
};

// Features of a batch tick after its compaction: workgroup g takes cell
// g - cell_base of stream map[g], as k_describe1 does for one stream;
// streams without a frame in the tick or without features are skipped.
__global__ __launch_bounds__(kDescBlock) void k_describe_batch(const TickArgs* table, const uint16_t* map)
{
    __shared__ int s_v[kDescBlock / 64][64];
    __shared__ uint8_t s_patch[kDescBlock / 64][kPatch * kPatch];
    const int g = blockIdx.x;
    const TickArgs& t = table[map[g]];
    if (!t.active || (!t.tab && !t.ref_cur)) return;
    const DetectArgs& d = t.d;
    const int c = g - t.cell_base;
    const uint32_t n = d.count_cur[c], dst0 = d.off_cur[c];
    if (!d.mask[c]) {
        copy_feature_records(t.desc_prev, t.tab ? t.desc_cur : nullptr, t.ref_prev, t.ref_cur, d.off_prev[c], dst0, n,
                             d.list_cap);
        return;
    }
    if (d.src_cur)
        copy_carried_records(d.src_cur, t.desc_prev, t.tab ? t.desc_cur : nullptr, t.ref_prev, t.ref_cur, dst0, n,
                             d.list_cap);
    describe_entries(TickLevels{d}, t.tab, d.O, d.t, d.list_cur, t.desc_cur, t.ref_cur, dst0, n, d.list_cap, s_v,
                     s_patch, d.src_cur);
}

// The levels of chunk frame j: level 0 is the frame itself, the others its
// octave copies.
struct ChunkLevels {
    const ChunkArgs& t;
    const uint8_t* f0;
    int p0;
    __device__ const uint8_t* ptr(int o) const { return o == 0 ? f0 : t.d.lvl[o]; }
    __device__ int pitch(int o) const { return o == 0 ? p0 : t.d.pitch[o]; }
    __device__ int w(int o) const { return t.d.w[o]; }
    __device__ int h(int o) const { return t.d.h[o]; }
};

// Features of a chunk's lists after compaction, in two launches of a
// 256-thread workgroup per (cell c, frame j). Frame j's list holds cell c's
// entries of the newest frame f <= j that marked c, or of the list before
// the chunk when none did. The first launch computes, where j marked c,
// the features of those entries on frame j's levels; the second copies,
// where j did not, the records of frame f's entries (or of the list before
// the chunk) to frame j's.
struct ChunkFeatureLists {
    const DescChunkArgs& a;
    int c;
    __device__ const kpd_keypoint* list(int f) const
    {
        return f == a.n_frames - 1 ? a.last_list : a.lists + (size_t)f * a.list_stride;
    }
    __device__ uint32_t count(int f) const
    {
        return f == a.n_frames - 1 ? a.last_count[c] : a.counts[(size_t)f * a.ncell + c];
    }
    __device__ uint32_t off(int f) const
    {
        return f == a.n_frames - 1 ? a.last_offs[c] : a.offs[(size_t)f * a.ncell + c];
    }
    __device__ kpd_descriptor* desc(int f) const
    {
        if (!a.tab) return nullptr;
        return f == a.n_frames - 1 ? a.last_desc : a.descs + (size_t)f * a.list_stride;
    }
    __device__ kpd_refined* ref(int f) const
    {
        if (!a.refs) return nullptr;
        return f == a.n_frames - 1 ? a.last_ref : a.refs + (size_t)f * a.list_stride;
    }
    // the newest frame <= j whose bit is set in the cell's mark words, -1 if none
    __device__ int newest_marked(int j) const
    {
        const unsigned long long* mw = a.marks + (size_t)c * a.Kw;
        for (int q = j >> 6; q >= 0; --q) {
            unsigned long long w = mw[q];
            if (q == (j >> 6) && (j & 63) != 63) w &= (2ull << (j & 63)) - 1ull;
            if (w) return 64 * q + 63 - __clzll(w);
        }
        return -1;
    }
};

__global__ __launch_bounds__(kDescBlock) void k_describe_chunk(DescChunkArgs a)
{
    __shared__ int s_v[kDescBlock / 64][64];
    __shared__ uint8_t s_patch[kDescBlock / 64][kPatch * kPatch];
    const int c = blockIdx.x, j = blockIdx.y;
    if (((a.marks[(size_t)c * a.Kw + (j >> 6)] >> (j & 63)) & 1ull) == 0ull) return;
    const ChunkFeatureLists F{a, c};
    const ChunkArgs& t = a.table[j];
    describe_entries(ChunkLevels{t, a.frames + (size_t)j * a.stride, a.pitch}, a.tab, a.O, a.t, F.list(j), F.desc(j),
                     F.ref(j), F.off(j), F.count(j), a.list_cap, s_v, s_patch);
}

__global__ __launch_bounds__(kDescBlock) void k_carry_chunk_features(DescChunkArgs a)
{
    const int c = blockIdx.x, j = blockIdx.y;
    const ChunkFeatureLists F{a, c};
    const int f = F.newest_marked(j);
    if (f == j) return;   // computed by the first launch
    if (f < 0)
        copy_feature_records(a.prev_desc, F.desc(j), a.prev_ref, F.ref(j), a.prev_offs[c], F.off(j), F.count(j),
                             a.list_cap);
    else
        copy_feature_records(F.desc(f), F.desc(j), F.ref(f), F.ref(j), F.off(f), F.off(j), F.count(j), a.list_cap);
}

// One workgroup copies what get_keypoints reads into its pinned staging
// buffer (host memory the device writes over the bus): one launch and one
// wait instead of a copy per part.
constexpr int kPublishBlock = 1024;

__global__ __launch_bounds__(kPublishBlock) void k_publish(const uint32_t* hdr, int total_word,
                                                           const kpd_keypoint* list, uint32_t pre,
                                                           const uint8_t* mask, int ncell, uint32_t stage_entries,
                                                           uint8_t* stage)
{
    const uint32_t total = hdr[total_word];
    const uint32_t n = min(total, pre);
    if (threadIdx.x < 4) reinterpret_cast<uint32_t*>(stage)[threadIdx.x] = hdr[threadIdx.x];
    uint2* dst = reinterpret_cast<uint2*>(stage + 64);
    const uint2* src = reinterpret_cast<const uint2*>(list);
    for (uint32_t i = threadIdx.x; i < n; i += kPublishBlock) dst[i] = src[i];
    if (mask) {
        uint8_t* m = stage + 64 + (size_t)stage_entries * sizeof(kpd_keypoint);
        for (int c = threadIdx.x; c < ncell; c += kPublishBlock) m[c] = mask[c];
    }
}

// Workgroups are dealt to the 8 XCDs round-robin by index. The tile pass
// runs on a grid rounded up to a multiple of 8 and hands XCD k the k-th
// contiguous band of row-major tiles, so tiles that share cache lines share
// an L2.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_band_tile(int b, int ntiles)
{
    const int per = (ntiles + kXcds - 1) / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

// One frame of one stream.
__global__ __launch_bounds__(kFrameBlock) void k_frame1(FrameArgs a)
{
    extern __shared__ __align__(16) uint8_t sm[];
    const int tile = xcd_band_tile(blockIdx.x, a.ntiles);
    if (tile >= a.ntiles) return;
    const FrameSrc f{a.cur, a.prev, a.cur_pitch, a.prev_pitch, a.cur_aligned, a.prev_aligned, a.sad_on, 0, a.sad};
    frame_tile(a, f, tile % a.tiles_x, tile / a.tiles_x, sm);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_detect1(DetectArgs a)
{
    extern __shared__ __align__(16) uint8_t sm[];
    detect_cell<NT>(a, blockIdx.x, sm);
}

// The streams of a batch tick with a per-pixel mask: workgroup g runs cell
// g - cell_base of stream map[g] as k_detect1 does for one stream (marks,
// detection, Eq. 1 per feature and the cell's place in D_n); the cells of
// other streams return at once. A cell waits only on lower cells of its
// own stream, whose workgroups come earlier in the grid.
template <int NT>
__global__ __launch_bounds__(NT) void k_detect_pixel_batch(const TickArgs* table, const uint16_t* map)
{
    extern __shared__ __align__(16) uint8_t sm[];
    const TickArgs& t = table[map[blockIdx.x]];
    if (!t.active || t.d.id_mode == 0) return;
    detect_cell<NT>(t.d, (int)blockIdx.x - t.cell_base, sm);
}

// Tile pass of a chunk: tiles of all its frames banded over the XCDs;
// frame j's tile source is frame j of the chunk and its predecessor, its
// octaves go pyr_stride * j bytes past frame 0's and its SAD accumulators
// one cell grid past frame j-1's. Every workgroup reads the same arguments.
__global__ __launch_bounds__(kFrameBlock) void k_frame_chunk(FrameArgs a, ChunkHead h, size_t pyr_stride)
{
    extern __shared__ __align__(16) uint8_t sm[];
    const int nblocks = h.n_frames * h.ntiles;
    const int b = xcd_band_tile(blockIdx.x, nblocks);
    if (b >= nblocks) return;
    const int j = b / h.ntiles, local = b - j * h.ntiles;
    const bool sad_on = !chunk_all_marked(h, j) && h.id_thresh < 255;
    if (a.O == 1 && !sad_on) return;
    FrameSrc f;
    f.cur = h.frames + (size_t)j * h.stride;
    f.cur_pitch = h.pitch;
    f.cur_aligned = h.aligned;
    f.prev = j == 0 ? h.prev0 : f.cur - h.stride;
    f.prev_pitch = j == 0 ? h.prev0_pitch : h.pitch;
    f.prev_aligned = j == 0 ? h.prev0_aligned : h.aligned;
    f.sad_on = sad_on ? 1 : 0;
    f.lvl_off = pyr_stride * (size_t)j;
    f.sad = a.sad + (size_t)j * (a.nc * a.nr);
    frame_tile(a, f, local % a.tiles_x, local / a.tiles_x, sm);
}

// Tile pass of a chunk whose frames test intensity differences, frames in
// sequence: workgroup (tile, run) walks frames j0 .. j0 + nf - 1 of its
// level-0 tile (TW x TH: 256 x 64, or 128 x 128) in order. Each frame's
// rows are loaded once (two frames ahead of the one being summed) and serve
// as I_n of their frame and I_{n-1} of the next, so a frame is read once
// instead of twice. Per frame: |I_n - I_{n-1}| summed per cell into an LDS
// slot row of that frame (one global atomic per slot when the run ends) and
// the octaves written from registers.
//
// Thread (rb, seg) holds rows 4rb..4rb+3 and columns 16seg..16seg+15 of
// the tile (SEGS = TW / 16 segments a row block, 64 / SEGS row blocks a
// wave): its level-1 block (2 x 8) and level-2 block (1 x 4) are its own,
// level 3 pairs it with the thread one row block down (SEGS lanes on),
// level 4 with the one two row blocks down, and (128-px tiles) level 5 with
// the thread 32 lanes on and the next segment, so 256-px tiles build
// octaves to level 4 (O <= 5), 128-px tiles to level 5. A level-1 tile row
// of a 256-px tile is one 128-byte line of the level (pitches are multiples
// of 128), which the L2 writes back whole.
//
// The host launches it only when the frame width is a multiple of 16 (a
// segment lies inside the frame or past it), the chunk's frames (and the
// frame before it) have 16-byte aligned rows, and every segment inside the
// frame lies in at most two cell columns (its first dword's and its last
// dword's, each dword in one of them) and every row block in at most two
// cell rows (its first row's and its last row inside the frame's). Loads
// and octave stores go through buffer resources (a frame, a level) whose
// range checks zero the rows below the frame and the segments past it
// (sent past the range), and drop the octave rows below a level and the
// stores of threads that hold no output: the loop takes no branches around
// memory accesses, so the compiler keeps two frames' loads in flight.
template <int SEGS>
__device__ __forceinline__ void pyramid_regs_buf(const BufStore& st, const uint4* rows, int x0, int y0, int rb,
                                                 int seg, bool col_in)
{
    const uint32_t r[4][4] = {{rows[0].x, rows[0].y, rows[0].z, rows[0].w},
                              {rows[1].x, rows[1].y, rows[1].z, rows[1].w},
                              {rows[2].x, rows[2].y, rows[2].z, rows[2].w},
                              {rows[3].x, rows[3].y, rows[3].z, rows[3].w}};
    uint32_t l1[2][2];
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int k = 0; k < 2; ++k) l1[y][k] = mean2x2(r[2 * y][2 * k], r[2 * y][2 * k + 1], r[2 * y + 1][2 * k],
                                                       r[2 * y + 1][2 * k + 1]);
#pragma unroll
    for (int y = 0; y < 2; ++y)
        st.put<8>(1, (x0 >> 1) + 8 * seg, (y0 >> 1) + 2 * rb + y, l1[y][0], l1[y][1], col_in);
    const uint32_t l2 = mean2x2(l1[0][0], l1[0][1], l1[1][0], l1[1][1]);
    st.put<4>(2, (x0 >> 2) + 4 * seg, (y0 >> 2) + rb, l2, 0u, col_in);
    // level 3: rows rb (even) and rb + 1 (SEGS lanes on), four pixels each -> two
    const uint32_t l2d = (uint32_t)__shfl_down((int)l2, SEGS);
    const uint32_t l3 = mean2x2(l2, 0u, l2d, 0u) & 0xFFFFu;
    st.put<2>(3, (x0 >> 3) + 2 * seg, (y0 >> 3) + rb / 2, l3, 0u, col_in && (rb & 1) == 0);
    // level 4: level-3 rows of threads rb and rb + 2 -> one pixel
    const uint32_t l3d = (uint32_t)__shfl_down((int)l3, 2 * SEGS);
    const uint32_t l4 = mean2x2(l3, 0u, l3d, 0u) & 0xFFu;
    st.put<1>(4, (x0 >> 4) + seg, (y0 >> 4) + rb / 4, l4, 0u, col_in && (rb & 3) == 0);
    if constexpr (SEGS == 8) {
        // level 5: level-4 pixels of (rb, seg), (rb, seg + 1), (rb + 4, seg), (rb + 4, seg + 1)
        const uint32_t l4r = (uint32_t)__shfl_down((int)l4, 1);
        const uint32_t l4d = (uint32_t)__shfl_down((int)l4, 32);
        const uint32_t l4dr = (uint32_t)__shfl_down((int)l4, 33);
        const uint32_t l5 = (l4 + l4r + l4d + l4dr + 2) >> 2;
        st.put<1>(5, (x0 >> 5) + seg / 2, (y0 >> 5) + rb / 8, l5, 0u, col_in && (rb & 7) == 0 && (seg & 1) == 0);
    }
}

// NT: the frames are read non-temporally (a chunk larger than the last
// level cache streams through it; marking the reads evict-first keeps the
// L2 lines of the octave rows that neighbouring tiles complete).
template <int TW, bool NT>
__global__ __launch_bounds__(kFrameBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_frame_chunk_seq(
    FrameArgs a, ChunkHead h, size_t pyr_stride, SeqGrid g)
{
    constexpr int SEGS = TW / 16;                       // 16-column segments a row block
    constexpr int TH = 4 * (kFrameBlock / SEGS);        // tile rows
    constexpr int LEVELS = SEGS == 8 ? 6 : 5;           // levels the register pyramid builds
    extern __shared__ __align__(16) uint8_t sm[];
    const int run = g.run;
    const int nruns = (h.n_frames + run - 1) / run;
    const int total = nruns * g.ntiles;
    const int b = xcd_band_tile(blockIdx.x, total);
    if (b >= total) return;
    const int ri = b / g.ntiles, local = b - ri * g.ntiles;
    const int j0 = ri * run, nf = min(run, h.n_frames - j0);
    const int bx = local % g.tiles_x, by = local / g.tiles_x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int seg = lane % SEGS, rb = (tid >> 6) * (64 / SEGS) + lane / SEGS;
    const int x0 = bx * TW, y0 = by * TH, gxs = x0 + 16 * seg;
    const bool col_in = gxs < a.W;
    auto sad_of = [&](int j) { return !chunk_all_marked(h, j) && h.id_thresh < 255; };

    // the tile's cells and the thread's share of them (LDS: a slot row of
    // g.slots per frame of the run, then the column and row tables)
    const int rows4 = (run + 3) / 4 * 4;
    uint32_t* sadl = reinterpret_cast<uint32_t*>(sm);
    uint16_t* colcell = reinterpret_cast<uint16_t*>(sm + 4 * g.slots * rows4);
    uint16_t* rowcell = colcell + TW;
    const int xe = min(x0 + TW, a.W), ye = min(y0 + TH, a.H);
    const int cx0 = a.colmap[x0], cy0 = a.rowmap[y0];
    const int ncx = a.colmap[xe - 1] - cx0 + 1, ncy = a.rowmap[ye - 1] - cy0 + 1;
    for (int i = tid; i < g.slots * nf; i += kFrameBlock) sadl[i] = 0;
    for (int i = tid; i < TW; i += kFrameBlock) colcell[i] = (uint16_t)(x0 + i < a.W ? a.colmap[x0 + i] - cx0 : 0);
    for (int i = tid; i < TH; i += kFrameBlock) rowcell[i] = (uint16_t)(y0 + i < a.H ? a.rowmap[y0 + i] - cy0 : 0);
    __syncthreads();
    // segments past the frame and rows below it load zeros in both frames
    // and add nothing, wherever their sums go
    const int c0 = colcell[16 * seg], c3 = colcell[16 * seg + 12];
    bool left[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) left[d] = colcell[16 * seg + 4 * d] == c0;
    const int r0 = rowcell[4 * rb], r3 = rowcell[max(4 * rb, min(4 * rb + 3, a.H - 1 - y0))];
    bool top[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) top[u] = rowcell[4 * rb + u] == r0;
    const int t0 = r0 * ncx, t1 = r3 * ncx;

    const uint8_t* f0 = h.frames + (size_t)j0 * h.stride;
    // row offsets inside a frame (the same for every frame of the chunk);
    // a frame is a buffer of pitch x H bytes
    int roff[4], poff[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int gy = y0 + 4 * rb + u;
        roff[u] = col_in ? gy * h.pitch + gxs : (int)0x80000000u;
        poff[u] = col_in ? gy * h.prev0_pitch + gxs : (int)0x80000000u;
    }
    auto load4 = [&](uint4* v, const uint8_t* base, int pitch, const int* off) {
        const __amdgpu_buffer_rsrc_t rs = raw_rsrc(base, (uint32_t)pitch * (uint32_t)a.H);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const v4u w = __builtin_amdgcn_raw_buffer_load_b128(rs, off[u], 0, NT ? kNonTemporal : 0);
            v[u] = make_uint4(w.x, w.y, w.z, w.w);
        }
    };
    // frame j0 + k's rows live in set S[k mod 4] (frame j0 - 1's in S[3]);
    // step k loads frame k + 2 while it sums frame k against frame k - 1.
    // Steps run in groups of four past the run's end (to a multiple of
    // four): there the loads re-read the run's last frame, the sums are
    // skipped and the octave stores go to empty buffers, so no step
    // branches around a memory access.
    uint4 S0[4], S1[4], S2[4], S3[4];
    auto step = [&](int k, const uint4* pv, const uint4* cv, uint4* dst) {
        const bool live = k < nf;
        const int j = j0 + min(k, nf - 1);
        load4(dst, f0 + (size_t)min(k + 2, nf - 1) * h.stride, h.pitch, roff);
        if (live && sad_of(j)) {
            uint32_t s00 = 0, s01 = 0, s10 = 0, s11 = 0;   // (first/last row cell, first/last column cell)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t cw[4] = {cv[u].x, cv[u].y, cv[u].z, cv[u].w};
                const uint32_t pw[4] = {pv[u].x, pv[u].y, pv[u].z, pv[u].w};
                uint32_t sa = 0, sb = 0;
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const uint32_t sd = __builtin_amdgcn_sad_u8(cw[d], pw[d], 0u);
                    sa += left[d] ? sd : 0u;
                    sb += left[d] ? 0u : sd;
                }
                s00 += top[u] ? sa : 0u;
                s01 += top[u] ? sb : 0u;
                s10 += top[u] ? 0u : sa;
                s11 += top[u] ? 0u : sb;
            }
            uint32_t* sl = sadl + k * g.slots;
            if (s00) atomicAdd(&sl[t0 + c0], s00);
            if (s01) atomicAdd(&sl[t0 + c3], s01);
            if (s10) atomicAdd(&sl[t1 + c0], s10);
            if (s11) atomicAdd(&sl[t1 + c3], s11);
        }
        // octaves 1..O-1 of frame j; levels from O on (and dead steps) get
        // empty buffers, so the register pyramid runs to its full depth
        BufStore st;
#pragma unroll
        for (int o = 0; o < LEVELS; ++o) {
            const bool on = live && o < a.O;
            st.r[o] = raw_rsrc(on ? a.lvl[o] + pyr_stride * (size_t)j : nullptr,
                               on ? (uint32_t)a.pitch[o] * (uint32_t)a.h[o] : 0u);
            st.pitch[o] = on ? a.pitch[o] : 0;
        }
        pyramid_regs_buf<SEGS>(st, cv, x0, y0, rb, seg, col_in);
    };
#pragma unroll
    for (int u = 0; u < 4; ++u) S3[u] = make_uint4(0u, 0u, 0u, 0u);
    if (sad_of(j0)) {
        if (j0 == 0) load4(S3, h.prev0, h.prev0_pitch, poff);
        else load4(S3, f0 - h.stride, h.pitch, roff);
    }
    load4(S0, f0, h.pitch, roff);
    load4(S1, f0 + (size_t)min(1, nf - 1) * h.stride, h.pitch, roff);
    for (int k = 0; k < nf; k += 4) {
        step(k, S3, S0, S2);
        step(k + 1, S0, S1, S3);
        step(k + 2, S1, S2, S0);
        step(k + 3, S2, S3, S1);
    }
    __syncthreads();
    const int per = ncx * ncy;
    for (int i = tid; i < per * nf; i += kFrameBlock) {
        const int k = i / per, l = i - k * per;
        const uint32_t v = sadl[k * g.slots + l];
        if (v) atomicAdd(&a.sad[(size_t)(j0 + k) * (a.nc * a.nr) + (cy0 + l / ncx) * a.nc + cx0 + l % ncx], v);
    }
}

// Mark pass of a chunk whose marks need no counts: one wave per cell and 64
// consecutive frames, one lane per frame. The wave's ballot is the cell's
// mark word for those frames; marked items are appended to the work list
// (one LDS atomic per wave, one global atomic per workgroup).
constexpr int kMarkBlock = 1024;

__global__ __launch_bounds__(kMarkBlock) void k_mark_chunk(ChunkHead h)
{
    __shared__ uint32_t s_count, s_base;
    const int nw = (h.n_frames + 63) >> 6;
    const int g = blockIdx.x * kMarkBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int cw = g >> 6;               // (cell, word) of this wave
    const int c = cw / nw, w = cw - c * nw;
    const int j = w * 64 + lane;
    if (threadIdx.x == 0) s_count = 0;
    __syncthreads();
    bool mark = false;
    if (c < h.ncell && j < h.n_frames) {
        mark = chunk_all_marked(h, j);
        if (!mark && h.id_thresh < 255) {
            const int cx = c % h.nc, cy = c / h.nc;
            const int64_t area = (int64_t)h.col_w[cx] * h.row_h[cy];
            mark = (int64_t)h.sad0[(size_t)j * h.ncell + c] > (int64_t)h.id_thresh * area;
        }
        if (j == h.n_frames - 1) h.mask[c] = (uint8_t)mark;
    }
    const uint64_t bal = __ballot(mark);
    if (lane == 0 && c < h.ncell) h.marks[(size_t)c * h.Kw + w] = bal;
    // workgroup-local slots first, then one global atomic per workgroup
    uint32_t wbase = 0;
    if (bal && lane == 0) wbase = atomicAdd(&s_count, (uint32_t)__popcll(bal));
    wbase = __shfl(wbase, 0);
    __syncthreads();
    if (threadIdx.x == 0) s_base = s_count ? atomicAdd(h.work_count, s_count) : 0;
    __syncthreads();
    if (mark) {
        const unsigned below =
            __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
        h.work[s_base + wbase + below] = (uint32_t)(j * h.ncell + c);
    }
}

// With T_H active, cell c is marked in frame j when the intensity test or
// a forced frame marks it (a root) or when its count in D_{j-1} reaches T_H
// (Eqs. 3-4); that count is its detection count in the newest marked frame
// before j. Instead of detecting frame after frame, a chunk detects in two
// rounds: first every root, then, speculatively, every other frame of a
// cell that follows a root whose count reaches T_H (or, from frame 0, a
// count before the chunk that does) up to the cell's next root: these are
// all the frames a chain of counts can mark. The resolve pass then walks
// each cell's frames in order and keeps the marks. One wave per cell, 64
// frames per step; both rounds append to the work list, the second after
// the first's items.
constexpr int kWaveCells = 4;   // cells (waves) per workgroup of these passes

__device__ __forceinline__ bool chunk_root(const ChunkHead& h, int j, int c, int64_t thr)
{
    return chunk_all_marked(h, j) || (h.id_thresh < 255 && (int64_t)h.sad0[(size_t)j * h.ncell + c] > thr);
}

__device__ __forceinline__ int64_t chunk_sad_thresh(const ChunkHead& h, int c)
{
    return (int64_t)h.id_thresh * h.col_w[c % h.nc] * h.row_h[c / h.nc];
}

// Append the frames in `bits` (frames w*64 + k) of cell c to the work list
// after *count, at base + the items before them (one atomic per wave).
__device__ __forceinline__ void append_frames(const ChunkHead& h, uint64_t bits, int w, int c, uint32_t base,
                                              uint32_t* count)
{
    if (!bits) return;
    const int lane = threadIdx.x & 63;
    uint32_t at = 0;
    if (lane == 0) at = atomicAdd(count, (uint32_t)__popcll(bits));
    at = base + __shfl(at, 0);
    if ((bits >> lane) & 1) {
        const unsigned below = __builtin_amdgcn_mbcnt_hi((unsigned)(bits >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((unsigned)bits, 0u));
        h.work[at + below] = (uint32_t)((w * 64 + lane) * h.ncell + c);
    }
}

// Round 1: every root of every cell.
__global__ __launch_bounds__(kWaveCells * 64) void k_spec_chunk(ChunkHead h)
{
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * kWaveCells + (int)(threadIdx.x >> 6);
    if (c >= h.ncell) return;   // the whole wave
    const int64_t thr = chunk_sad_thresh(h, c);
    for (int w = 0; w * 64 < h.n_frames; ++w) {
        const int j = w * 64 + lane;
        append_frames(h, __ballot(j < h.n_frames && chunk_root(h, j, c, thr)), w, c, 0u, h.work_count);
    }
}

// Round 2: the non-root frames a chain can reach, after round 1's items.
__global__ __launch_bounds__(kWaveCells * 64) void k_spec2_chunk(ChunkHead h, const uint32_t* own)
{
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * kWaveCells + (int)(threadIdx.x >> 6);
    if (c >= h.ncell) return;   // the whole wave
    const int64_t thr = chunk_sad_thresh(h, c);
    const uint32_t base = *h.work_count;
    bool chain = h.prev_count[c] >= h.kb_thresh;
    for (int w = 0; w * 64 < h.n_frames; ++w) {
        const int j = w * 64 + lane;
        bool root = false, g = false;
        if (j < h.n_frames) {
            root = chunk_root(h, j, c, thr);
            g = root && own[(size_t)j * h.ncell + c] >= h.kb_thresh;
        }
        const uint64_t R = __ballot(root), G = __ballot(g);
        const int nj = min(64, h.n_frames - w * 64);
        uint64_t S = 0;
        for (int k = 0; k < nj; ++k) {
            if ((R >> k) & 1) chain = (G >> k) & 1;
            else if (chain) S |= 1ull << k;
        }
        append_frames(h, S, w, c, base, h.work_count + 1);
    }
}

__global__ __launch_bounds__(kWaveCells * 64) void k_resolve_chunk(ChunkHead h, const uint32_t* own)
{
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * kWaveCells + (int)(threadIdx.x >> 6);
    if (c >= h.ncell) return;   // the whole wave
    const int64_t thr = chunk_sad_thresh(h, c);
    bool pass = h.prev_count[c] >= h.kb_thresh;   // the running count reaches T_H
    bool m = false;
    for (int w = 0; w * 64 < h.n_frames; ++w) {
        const int j = w * 64 + lane;
        bool root = false, g = false;
        if (j < h.n_frames) {
            root = chunk_root(h, j, c, thr);
            g = own[(size_t)j * h.ncell + c] >= h.kb_thresh;   // used only where frame j was detected
        }
        const uint64_t R = __ballot(root), G = __ballot(g);
        const int nj = min(64, h.n_frames - w * 64);
        uint64_t M = 0;
        for (int k = 0; k < nj; ++k) {
            m = ((R >> k) & 1) || pass;
            if (m) {
                M |= 1ull << k;
                pass = (G >> k) & 1;
            }
        }
        if (lane == 0) h.marks[(size_t)c * h.Kw + w] = M;
    }
    if (lane == 0) h.mask[c] = (uint8_t)m;
}

// Compaction of a chunk, one workgroup per frame j, cells in tiles of
// kCompact: each cell's source (the last chunk frame up to j that marked it,
// else the list before the chunk) and count, their exclusive prefix (the
// cell's offset in frame j's list), then a flat copy of the tile's entries.
// The last frame's list goes where the next push reads it. Also clears the
// chunk's SAD accumulators and hands the last frame's SAD to the statistics.
constexpr int kCompact = 512;
constexpr int kMaxChunk = KPD_MAX_CHUNK;

// Compaction core, one workgroup per frame: cells in tiles of kCompact.
// source(c, &n, &src) gives cell c's count and the address of its first
// entry (and may record per-cell side results); the counts' exclusive
// prefix is the cell's offset in D_n, and a flat copy (each entry finds its
// cell by binary search in LDS) writes D_n in cell order. Writes the counts,
// offsets and total of D_n. A source whose entries would leave their list
// has been clamped by source().
template <int NT, class Source>
__device__ void compact_frame(int ncell, uint32_t list_cap, kpd_keypoint* dst, uint32_t* cnt_out,
                              uint32_t* off_out, uint32_t* total_out, Source&& source)
{
    __shared__ uint32_t s_excl[NT], s_wsum[NT / 64];
    __shared__ const kpd_keypoint* s_src[NT];
    __shared__ uint32_t s_base;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_base = 0;
    __syncthreads();
    for (int c0 = 0; c0 < ncell; c0 += NT) {
        const int c = c0 + tid;
        const int ntile = min(NT, ncell - c0);
        const uint32_t base = s_base;
        uint32_t n = 0;
        const kpd_keypoint* src = nullptr;
        if (c < ncell) source(c, &n, &src);
        uint32_t incl = n;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t v = __shfl_up(incl, d);
            if (lane >= d) incl += v;
        }
        if (lane == 63) s_wsum[wave] = incl;
        __syncthreads();
        uint32_t wbase = 0;
        for (int w = 0; w < wave; ++w) wbase += s_wsum[w];
        const uint32_t excl = base + wbase + incl - n;
        s_excl[tid] = excl;
        s_src[tid] = src;
        if (c < ncell) {
            cnt_out[c] = n;
            off_out[c] = excl;
        }
        __syncthreads();
        // every thread needs the tile's end: the last cell's thread publishes it
        if (tid == ntile - 1) s_wsum[0] = excl + n;
        __syncthreads();
        const uint32_t t1 = s_wsum[0];
        for (uint32_t d = base + tid; d < t1; d += NT) {
            int lo = 0, hi = ntile - 1;   // largest cell of the tile starting at or before d
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_excl[mid] <= d) lo = mid;
                else hi = mid - 1;
            }
            if (d < list_cap) dst[d] = s_src[lo][d - s_excl[lo]];
        }
        __syncthreads();
        if (tid == 0) s_base = t1;
        __syncthreads();
    }
    if (tid == 0) *total_out = s_base;
}

// Entries of a cell that stay inside their list of `cap` entries.
__device__ __forceinline__ uint32_t clamp_count(uint32_t off, uint32_t n, uint32_t cap)
{
    return off >= cap ? 0u : min(n, cap - off);
}

__global__ __launch_bounds__(kCompact) void k_compact_chunk(CompactArgs a)
{
    const int j = blockIdx.x;
    const bool last = j == a.last;
    const size_t jc = (size_t)j * a.ncell;
    kpd_keypoint* dst = last ? a.next_list : a.lists + (size_t)j * a.list_stride;
    uint32_t* cnt_out = last ? a.next_count : a.counts + jc;
    uint32_t* off_out = last ? a.next_offs : a.offs + jc;
    compact_frame<kCompact>(a.ncell, a.list_cap, dst, cnt_out, off_out, last ? a.next_total : a.totals + j,
                  [&](int c, uint32_t* n, const kpd_keypoint** src) {
        // the newest frame <= j that marked this cell: its mark words up
        // to frame j, all loads issued before any is used
        const unsigned long long* mw = a.marks + (size_t)c * a.Kw;
        const int qj = j >> 6;
        const unsigned long long upto = (j & 63) == 63 ? ~0ull : (2ull << (j & 63)) - 1ull;   // frames <= j
        unsigned long long m[kMaxChunk / 64];
#pragma unroll
        for (int q = 0; q < kMaxChunk / 64; ++q) m[q] = q <= qj ? mw[q] : 0ull;
        int f = -1;
#pragma unroll
        for (int q = 0; q < kMaxChunk / 64; ++q) {
            const unsigned long long x = q == qj ? m[q] & upto : m[q];
            if (q <= qj && x) f = 64 * q + 63 - __clzll(x);
        }
        if (f >= 0) {
            const uint32_t off = a.cell_base[c];
            *n = clamp_count(off, a.own_count[(size_t)f * a.ncell + c], a.list_cap);
            *src = a.sparse + (size_t)f * a.list_stride + off;
        } else {
            const uint32_t off = a.prev_offs[c];
            *n = clamp_count(off, a.prev_count[c], a.list_cap);
            *src = a.prev_list + off;
        }
        if (last) {
            a.sad_stats[c] = a.sad_chunk[jc + c];
            a.sad_single_next[c] = 0;
        }
        a.sad_chunk[jc + c] = 0;
    });
    if (j == 0 && threadIdx.x == 0) a.work_count[0] = a.work_count[1] = 0;
}

// ------------------------------------------------ per-pixel masks in chunks

// Layer l of chunk frame j (j = -1: the frame before the chunk).
__device__ __forceinline__ const uint8_t* pixel_layer(const PixelChunkArgs& a, int j, int l, int* pitch)
{
    if (j < 0) {
        *pitch = a.prev_pitch[l];
        return a.prev_lvl[l];
    }
    if (l == 0) {
        *pitch = a.pitch;
        return a.frames + (size_t)j * a.stride;
    }
    *pitch = a.table[j].d.pitch[l];
    return a.table[j].d.lvl[l];
}

// The layer pixels cell rectangle r maps to on a layer of lw x lh: its
// level-0 pixels shifted down by l, clamped into the layer.
struct LayerSpan {
    int kx0, ky0, nx, npx;
};

__device__ __forceinline__ LayerSpan layer_span(const Box& r, int l, int lw, int lh)
{
    const int kx0 = min(r.x0 >> l, lw - 1), kx1 = min((r.x1 - 1) >> l, lw - 1);
    const int ky0 = min(r.y0 >> l, lh - 1), ky1 = min((r.y1 - 1) >> l, lh - 1);
    return LayerSpan{kx0, ky0, kx1 - kx0 + 1, (kx1 - kx0 + 1) * (ky1 - ky0 + 1)};
}

// A wave per (frame j, cell c): the changed bits (|I_j - I_{j-1}| > T_I on
// the mask layers) of the layer pixels of the cell, each layer's bits
// starting at a multiple of 64, and whether any is set. A forced frame 0
// marks every cell without reading the frame before.
constexpr int kDiffWaves = 4;

__global__ __launch_bounds__(64 * kDiffWaves) void k_pixel_diff_chunk(PixelChunkArgs a)
{
    const int lane = threadIdx.x & 63;
    const int item = blockIdx.x * kDiffWaves + (threadIdx.x >> 6);
    if (item >= a.n_frames * a.ncell) return;
    const int j = item / a.ncell, c = item - j * a.ncell;
    if (a.force0 && j == 0) {
        if (lane == 0) a.flags[item] = 0u;
        return;
    }
    const DetectArgs& d = a.table[j].d;
    const Box r = cell_rect(c, a.W, a.H, a.nc, a.nr);
    unsigned long long* fp = a.fp + (size_t)item * a.fpw;
    bool any = false;
    int boff = 0;
    for (int l = a.l_lo; l <= a.l_hi; ++l) {
        const LayerSpan sp = layer_span(r, l, d.w[l], d.h[l]);
        int cp, pp;
        const uint8_t* cur = pixel_layer(a, j, l, &cp);
        const uint8_t* prv = pixel_layer(a, j - 1, l, &pp);
        for (int base = 0; base < sp.npx; base += 64) {
            const int i = base + lane;
            bool ch = false;
            if (i < sp.npx) {
                const int ry = i / sp.nx, rx = i - ry * sp.nx;
                const int vc = cur[(size_t)(sp.ky0 + ry) * cp + sp.kx0 + rx];
                const int vp = prv[(size_t)(sp.ky0 + ry) * pp + sp.kx0 + rx];
                ch = abs(vc - vp) > a.id_thresh;
            }
            const uint64_t bal = __ballot(ch);
            if (lane == 0) fp[(boff + base) >> 6] = bal;
            any = any || bal != 0;
        }
        boff += (sp.npx + 63) & ~63;
    }
    if (lane == 0) a.flags[item] = any ? 1u : 0u;
}

// A workgroup per cell walks the cell's listed frames in order, holding
// D_j of the cell as a map over its decision pixels (a presence bit and a
// score each) in LDS: at frame j the entries whose mask pixel changed are
// dropped, F_j's maxima whose mask pixel changed are added (Eq. 1 per
// feature; a forced frame replaces everything), and the map is written in
// decision order, (octave, y, x), at the cell's per-pixel base of frame j's
// merged list. The map starts from the cell's entries before the chunk.
// The listed frames' change bits and maxima are staged in LDS a batch of
// frames at a time (one round of loads per batch), so the walk itself
// waits on no memory; when they fit, tables of every decision pixel's
// position and mask bit (built once per cell) replace the decoding.
constexpr int kMergeBlock = 256;
constexpr int kMergeBatchMax = 32;   // listed frames staged at once

__global__ __launch_bounds__(kMergeBlock) void k_pixel_merge_chunk(PixelChunkArgs a)
{
    extern __shared__ __align__(16) uint8_t sm[];
    __shared__ CellLayout L;
    __shared__ int s_kx0[KPD_MAX_OCTAVES], s_ky0[KPD_MAX_OCTAVES], s_nx[KPD_MAX_OCTAVES], s_boff[KPD_MAX_OCTAVES];
    __shared__ int s_w[KPD_MAX_OCTAVES], s_h[KPD_MAX_OCTAVES];
    __shared__ uint32_t s_part[kMergeBlock / 64];
    __shared__ uint16_t s_frames[KPD_MAX_CHUNK];
    __shared__ uint32_t s_cnt[kMergeBatchMax], s_eoff[kMergeBatchMax + 1];
    __shared__ int s_nl, s_nb;
    const int c = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    unsigned long long* pres = reinterpret_cast<unsigned long long*>(sm + a.lds_pres);
    uint16_t* score = reinterpret_cast<uint16_t*>(sm + a.lds_score);
    unsigned long long* fps = reinterpret_cast<unsigned long long*>(sm + a.lds_fp);
    kpd_keypoint* ents = reinterpret_cast<kpd_keypoint*>(sm + a.lds_ents);
    uint16_t* tgate = reinterpret_cast<uint16_t*>(sm + a.lds_tgate);
    uint32_t* txy = reinterpret_cast<uint32_t*>(sm + a.lds_txy);
    uint8_t* toct = sm + a.lds_toct;
    uint32_t* tsrc = reinterpret_cast<uint32_t*>(sm + a.lds_tsrc);
    {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(a.layouts + c);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&L);
        for (int i = tid; i < (int)(sizeof(CellLayout) / 4); i += kMergeBlock) dst[i] = src[i];
    }
    if (tid == 0) {
        const Box r = cell_rect(c, a.W, a.H, a.nc, a.nr);
        const DetectArgs& d = a.table[0].d;
        int boff = 0;
        for (int l = 0; l < KPD_MAX_OCTAVES; ++l) {
            s_w[l] = d.w[l];
            s_h[l] = d.h[l];
            s_kx0[l] = s_ky0[l] = s_nx[l] = s_boff[l] = 0;
            if (l < a.l_lo || l > a.l_hi) continue;
            const LayerSpan sp = layer_span(r, l, d.w[l], d.h[l]);
            s_kx0[l] = sp.kx0;
            s_ky0[l] = sp.ky0;
            s_nx[l] = sp.nx;
            s_boff[l] = boff;
            boff += (sp.npx + 63) & ~63;
        }
        // the listed frames of this chunk, in order
        const unsigned long long* mw = a.marks + (size_t)c * a.Kw;
        int n = 0;
        for (int q = 0; q <= (a.n_frames - 1) >> 6; ++q) {
            unsigned long long w = mw[q];
            if (q == (a.n_frames - 1) >> 6 && ((a.n_frames - 1) & 63) != 63)
                w &= (2ull << ((a.n_frames - 1) & 63)) - 1ull;
            while (w) {
                s_frames[n++] = (uint16_t)(64 * q + __builtin_ctzll(w));
                w &= w - 1ull;
            }
        }
        s_nl = n;
    }
    __syncthreads();
    const int nw = L.nwords, O = a.O;
    for (int w = tid; w < nw; w += kMergeBlock) pres[w] = 0ull;
    // decision index of (o, x, y), -1 outside the cell's decision box
    auto index_of = [&](int o, int x, int y) -> int {
        if (o >= O) return -1;
        const Box d = L.dec[o];
        if (x < d.x0 || x >= d.x1 || y < d.y0 || y >= d.y1) return -1;
        return L.dc_start[o] + (y - d.y0) * box_w(d) + (x - d.x0);
    };
    // the octave and level position of decision pixel i, computed
    auto decode = [&](int i, int& o, int& x, int& y) {
        o = level_of(L.dc_start, O, i);
        const unsigned r = (unsigned)(i - L.dc_start[o]);
        const Box d = L.dec[o];
        const int ry = (int)fast_div(r, L.dcm[o]);
        x = d.x0 + (int)r - ry * box_w(d);
        y = d.y0 + ry;
    };
    // the mask bit (index into a frame's change bits) of a feature at level o, (x, y)
    auto gate_of = [&](int o, int x, int y) -> int {
        const int l = a.one ? a.l_lo : o;
        const int kx = min((x << o) >> l, s_w[l] - 1) - s_kx0[l];
        const int ky = min((y << o) >> l, s_h[l] - 1) - s_ky0[l];
        return s_boff[l] + ky * s_nx[l] + kx;
    };
    const int ndc = L.dc_start[O];
    if (a.tab_on)
        for (int i = tid; i < ndc; i += kMergeBlock) {
            int o, x, y;
            decode(i, o, x, y);
            tgate[i] = (uint16_t)gate_of(o, x, y);
            txy[i] = (uint32_t)x | ((uint32_t)y << 16);
            toct[i] = (uint8_t)o;
        }
    __syncthreads();
    auto bit_at = [](const unsigned long long* fpb, int g) -> bool { return ((fpb[g >> 6] >> (g & 63)) & 1ull) != 0ull; };
    // decision pixel i's mask pixel changed (change bits fpb)
    auto changed_i = [&](const unsigned long long* fpb, int i) -> bool {
        if (a.tab_on) return bit_at(fpb, tgate[i]);
        int o, x, y;
        decode(i, o, x, y);
        return bit_at(fpb, gate_of(o, x, y));
    };
    if (!a.force0) {
        const uint32_t n0 = a.prev_count[c], src0 = a.prev_offs[c];
        for (uint32_t e = tid; e < n0; e += kMergeBlock) {
            if (src0 + e >= a.prev_cap) break;
            const kpd_keypoint kp = a.prev_list[src0 + e];
            const int i = index_of(kp.octave, kp.x, kp.y);
            if (i < 0) continue;
            atomicOr(&pres[i >> 6], 1ull << (i & 63));
            score[i] = kp.score;
            if (a.msrc) tsrc[i] = kPixelFromPrev | (src0 + e);
        }
    }
    __syncthreads();
    const uint32_t cb = a.cell_base[c], pb = a.pbase[c];
    const int nl = s_nl;
    for (int b0 = 0; b0 < nl;) {
        // the batch: up to a.batch listed frames whose maxima fit the staging
        // area (the first frame always; past the area its maxima stay in
        // global memory)
        const int bm = min(a.batch, nl - b0);
        if (tid < bm) {
            const int j = s_frames[b0 + tid];
            s_cnt[tid] = cb >= a.list_cap ? 0u : min(a.own[(size_t)j * a.ncell + c], a.list_cap - cb);
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t acc = 0;
            int k = 0;
            for (; k < bm; ++k) {
                const uint32_t take = min(s_cnt[k], a.ents_cap);
                if (k > 0 && acc + take > a.ents_cap) break;
                s_eoff[k] = acc;
                acc += take;
            }
            s_eoff[k] = acc;
            s_nb = k;
        }
        __syncthreads();
        const int nb = s_nb;
        for (int i = tid; i < nb * a.fpw; i += kMergeBlock) {
            const int k = i / a.fpw;
            fps[i] = a.fp[((size_t)s_frames[b0 + k] * a.ncell + c) * a.fpw + (i - k * a.fpw)];
        }
        const uint32_t tot = s_eoff[nb];
        for (uint32_t i = tid; i < tot; i += kMergeBlock) {
            int lo = 0, hi = nb - 1;   // the frame whose staged maxima hold entry i
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_eoff[mid] <= i) lo = mid;
                else hi = mid - 1;
            }
            ents[i] = a.sparse[(size_t)s_frames[b0 + lo] * a.list_stride + cb + (i - s_eoff[lo])];
        }
        __syncthreads();
        for (int k = 0; k < nb; ++k) {
            const int j = s_frames[b0 + k];
            const bool forced = a.force0 && j == 0;
            const unsigned long long* fpb = fps + (size_t)k * a.fpw;
            // entries whose mask pixel changed leave (all, when forced)
            for (int w = tid; w < nw; w += kMergeBlock) {
                unsigned long long bits = pres[w], out = forced ? 0ull : bits;
                while (bits && !forced) {
                    const int b = __builtin_ctzll(bits);
                    bits &= bits - 1ull;
                    if (changed_i(fpb, w * 64 + b)) out &= ~(1ull << b);
                }
                pres[w] = out;
            }
            __syncthreads();
            // F_j's maxima whose mask pixel changed come in
            const uint32_t nf = s_cnt[k], staged = s_eoff[k + 1] - s_eoff[k];
            const kpd_keypoint* se = ents + s_eoff[k];
            const kpd_keypoint* ge = a.sparse + (size_t)j * a.list_stride + cb;
            for (uint32_t e = tid; e < nf; e += kMergeBlock) {
                const kpd_keypoint kp = e < staged ? se[e] : ge[e];
                const int i = index_of(kp.octave, kp.x, kp.y);
                if (i < 0 || !(forced || changed_i(fpb, i))) continue;
                atomicOr(&pres[i >> 6], 1ull << (i & 63));
                score[i] = kp.score;
                if (a.msrc) tsrc[i] = ((uint32_t)j << kPixelFrameShift) | (cb + e);
            }
            __syncthreads();
            // D_j of the cell in decision order
            uint32_t total = 0;
            for (int w0 = 0; w0 < nw; w0 += kMergeBlock) {
                const int w = w0 + tid;
                const unsigned long long bits = w < nw ? pres[w] : 0ull;
                const uint32_t cnt = (uint32_t)__popcll(bits);
                uint32_t incl = cnt;
                for (int dd = 1; dd < 64; dd <<= 1) {
                    const uint32_t v = __shfl_up(incl, dd);
                    if (lane >= dd) incl += v;
                }
                if (lane == 63) s_part[wave] = incl;
                __syncthreads();
                uint32_t before = total, sum = 0;
                for (int q = 0; q < kMergeBlock / 64; ++q) {
                    if (q < wave) before += s_part[q];
                    sum += s_part[q];
                }
                kpd_keypoint* dst = a.merged + (size_t)j * a.list_stride + pb;
                unsigned long long m = bits;
                uint32_t at = before + incl - cnt;
                while (m) {
                    const int b = __builtin_ctzll(m);
                    m &= m - 1ull;
                    const int i = w * 64 + b;
                    kpd_keypoint kp;
                    if (a.tab_on) {
                        const uint32_t xy = txy[i];
                        kp.x = (uint16_t)(xy & 0xFFFFu);
                        kp.y = (uint16_t)(xy >> 16);
                        kp.octave = toct[i];
                    } else {
                        int o, x, y;
                        decode(i, o, x, y);
                        kp.x = (uint16_t)x;
                        kp.y = (uint16_t)y;
                        kp.octave = (uint8_t)o;
                    }
                    kp.pad = 0;
                    kp.score = score[i];
                    if (pb + at < a.plist_cap) {
                        dst[at] = kp;
                        if (a.msrc) a.msrc[(size_t)j * a.list_stride + pb + at] = tsrc[i];
                    }
                    ++at;
                }
                total += sum;
                __syncthreads();   // s_part, and the map for the next frame
            }
            if (tid == 0) a.mcount[(size_t)j * a.ncell + c] = total;
        }
        b0 += nb;
    }
}

// Features of the maxima of every listed (frame, cell) of a chunk with a
// per-pixel mask, on that frame's levels, at their places in its F list
// (a 256-thread workgroup per (cell, frame), as k_describe_chunk).
__global__ __launch_bounds__(kDescBlock) void k_pixel_features_chunk(PixelChunkArgs a)
{
    __shared__ int s_v[kDescBlock / 64][64];
    __shared__ uint8_t s_patch[kDescBlock / 64][kPatch * kPatch];
    const int c = blockIdx.x, j = blockIdx.y;
    if (((a.marks[(size_t)c * a.Kw + (j >> 6)] >> (j & 63)) & 1ull) == 0ull) return;
    const uint32_t cb = a.cell_base[c];
    const uint32_t n = cb >= a.list_cap ? 0u : min(a.table[j].own_count[c], a.list_cap - cb);
    const ChunkArgs& t = a.table[j];
    describe_entries(ChunkLevels{t, a.frames + (size_t)j * a.stride, a.pitch}, a.tab, a.O, a.t, t.d.list_cur,
                     a.tab ? a.sdesc + (size_t)j * a.list_cap : nullptr,
                     a.sref ? a.sref + (size_t)j * a.list_cap : nullptr, cb, n, a.list_cap, s_v, s_patch);
}

// Each chunk frame's records after the compaction, a workgroup per (cell,
// frame): frame j's entries of cell c are the merged list of the newest
// listed frame f <= j (in order), so entry k takes the record its source
// names; with no listed frame, the records of the list before the chunk.
__global__ __launch_bounds__(kDescBlock) void k_pixel_gather_chunk(PixelChunkArgs a)
{
    const int c = blockIdx.x, j = blockIdx.y;
    const bool last = j == a.n_frames - 1;
    const uint32_t n = last ? a.last_count[c] : a.counts[(size_t)j * a.ncell + c];
    const uint32_t dst0 = last ? a.last_offs[c] : a.offs[(size_t)j * a.ncell + c];
    kpd_descriptor* ddst = a.tab ? (last ? a.last_desc : a.cdesc + (size_t)j * a.list_stride) : nullptr;
    kpd_refined* rdst = a.sref ? (last ? a.last_ref : a.cref + (size_t)j * a.list_stride) : nullptr;
    // the newest listed frame up to j
    const unsigned long long* mw = a.marks + (size_t)c * a.Kw;
    int f = -1;
    for (int q = j >> 6; q >= 0 && f < 0; --q) {
        unsigned long long w = mw[q];
        if (q == (j >> 6) && (j & 63) != 63) w &= (2ull << (j & 63)) - 1ull;
        if (w) f = 64 * q + 63 - __clzll(w);
    }
    constexpr int kw = sizeof(kpd_descriptor) / 8;
    for (uint32_t i = threadIdx.x; i < n * kw; i += kDescBlock) {
        const uint32_t e = i / kw, q = i % kw;
        if (dst0 + e >= a.dlist_cap) break;
        uint32_t src;
        if (f < 0) {
            src = kPixelFromPrev | (a.prev_offs[c] + e);
        } else {
            src = a.msrc[(size_t)f * a.list_stride + a.pbase[c] + e];
        }
        const bool prev = (src & kPixelFromPrev) != 0u;
        const size_t at = prev ? (size_t)(src & ~kPixelFromPrev)
                               : (size_t)(src >> kPixelFrameShift) * a.list_cap + (src & ((1u << kPixelFrameShift) - 1u));
        if (prev && at >= a.prev_cap) continue;
        if (ddst) {
            const uint64_t* s64 = reinterpret_cast<const uint64_t*>(prev ? a.prev_desc : a.sdesc);
            reinterpret_cast<uint64_t*>(ddst)[(size_t)(dst0 + e) * kw + q] = s64[at * kw + q];
        }
        if (rdst && q == 0) rdst[dst0 + e] = prev ? a.prev_ref[at] : a.sref[at];
    }
}

// One batch tick: workgroup b works for stream map[b] (streams' workgroups
// are contiguous and in stream order); inactive streams' workgroups exit.
// Tiles are banded over the XCDs across the whole grid, as in k_frame1.
__global__ __launch_bounds__(kFrameBlock) void k_frame_batch(const TickArgs* table, const uint16_t* map, int nblocks)
{
    extern __shared__ __align__(16) uint8_t sm[];
    const int b = xcd_band_tile(blockIdx.x, nblocks);
    if (b >= nblocks) return;
    const TickArgs& t = table[map[b]];
    const int local = b - t.tile_base;
    if (!t.active || !t.f_on) return;
    const FrameArgs& a = t.f;
    const FrameSrc f{a.cur, a.prev, a.cur_pitch, a.prev_pitch, a.cur_aligned, a.prev_aligned, a.sad_on, 0, a.sad};
    frame_tile(a, f, local % a.tiles_x, local / a.tiles_x, sm);
}


// A batch tick in four passes after the tile pass's: marks of every cell
// of every active stream with the marked cells listed, detection of the
// listed cells into per-stream sparse lists, and compaction of each
// stream's D_n (Eq. 1). D_{n-1} is final before the tick, so the marks need
// no waits.
__global__ __launch_bounds__(kMarkBlock) void k_mark_batch(const TickArgs* table, const uint16_t* map, int ncells,
                                                           uint32_t* work, uint32_t* work_count)
{
    __shared__ uint32_t s_count, s_base;
    const int g = blockIdx.x * kMarkBlock + threadIdx.x;
    if (threadIdx.x == 0) s_count = 0;
    __syncthreads();
    bool mark = false;
    if (g < ncells) {
        const TickArgs& t = table[map[g]];
        if (t.active && t.d.id_mode == 0) {   // per-pixel streams run their own pass
            const int c = g - t.cell_base;
            mark = cell_marked(t.d, c);
            t.d.mask[c] = (uint8_t)mark;
            t.d.sad_next[c] = 0;
        }
    }
    const uint64_t bal = __ballot(mark);
    const int lane = threadIdx.x & 63;
    const int leader = bal ? __builtin_ctzll(bal) : 0;
    uint32_t wbase = 0;
    if (bal && lane == leader) wbase = atomicAdd(&s_count, (uint32_t)__popcll(bal));
    wbase = __shfl(wbase, leader);
    __syncthreads();
    if (threadIdx.x == 0) s_base = s_count ? atomicAdd(work_count, s_count) : 0;
    __syncthreads();
    if (mark) {
        const unsigned below =
            __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
        work[s_base + wbase + below] = (uint32_t)g;
    }
}

// D_n of one frame of one stream after k_det1_groups (Eq. 1): marked cells
// take their new keypoints from the sparse list, the others D_{n-1}'s. A
// workgroup per run of kCells1 cells: it sums the counts of every earlier
// cell for its base offset, scans its own cells' counts and copies their
// entries, a wave per cell; the last workgroup writes the total.
constexpr int kCells1 = 16;
constexpr int kCompact1Block = 256;

__global__ __launch_bounds__(kCompact1Block) void k_compact1(DetectArgs a, const kpd_keypoint* sparse,
                                                            const uint32_t* cbase, const uint32_t* own)
{
    __shared__ uint32_t s_wsum[kCompact1Block / 64];
    __shared__ uint32_t s_off[kCells1], s_n[kCells1];
    __shared__ const kpd_keypoint* s_src[kCells1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ncell = a.nc * a.nr;
    const int c0 = blockIdx.x * kCells1, c1 = min(c0 + kCells1, ncell);
    // both sources' words are loaded with the mark and one is kept, so a
    // cell's count costs one round trip to memory instead of two
    auto count_of = [&](int c) -> uint32_t {
        const uint8_t m = a.mask[c];
        const uint32_t nb = cbase[c], nn = own[c], pb = a.off_prev[c], pn = a.count_prev[c];
        return clamp_count(m ? nb : pb, m ? nn : pn, a.list_cap);
    };
    uint32_t acc = 0;
#pragma unroll 4
    for (int c = tid; c < c0; c += kCompact1Block) acc += count_of(c);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) s_wsum[wave] = acc;
    if (tid < c1 - c0) {
        const int c = c0 + tid;
        const uint8_t m = a.mask[c];
        const uint32_t nb = cbase[c], nn = own[c], pb = a.off_prev[c], pn = a.count_prev[c];
        s_n[tid] = clamp_count(m ? nb : pb, m ? nn : pn, a.list_cap);
        s_src[tid] = m ? sparse + nb : a.list_prev + pb;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t base = 0;
        for (int w = 0; w < kCompact1Block / 64; ++w) base += s_wsum[w];
        for (int k = 0; k < c1 - c0; ++k) {
            s_off[k] = base;
            a.count_cur[c0 + k] = s_n[k];
            a.off_cur[c0 + k] = base;
            base += s_n[k];
        }
        if (c1 == ncell) *a.total_cur = base;
    }
    __syncthreads();
    for (int k = wave; k < c1 - c0; k += kCompact1Block / 64) {
        const uint32_t n = s_n[k], off = s_off[k];
        const kpd_keypoint* src = s_src[k];
        for (uint32_t e = lane; e < n; e += 64)
            if (off + e < a.list_cap) a.list_cur[off + e] = src[e];
    }
}

hipError_t launch_compact1(const DetectArgs& a, const kpd_keypoint* sparse, const uint32_t* cbase,
                           const uint32_t* own, hipStream_t s)
{
    const int ncell = a.nc * a.nr;
    hipLaunchKernelGGL(k_compact1, dim3((ncell + kCells1 - 1) / kCells1), dim3(kCompact1Block), 0, s, a, sparse,
                       cbase, own);
    return hipGetLastError();
}

__global__ __launch_bounds__(kCompact) void k_compact_batch(const TickArgs* table, uint32_t* work_count)
{
    const TickArgs& t = table[blockIdx.x];
    if (t.active && t.d.id_mode == 0) {
        const DetectArgs& a = t.d;
        compact_frame<kCompact>(a.nc * a.nr, a.list_cap, a.list_cur, a.count_cur, a.off_cur, a.total_cur,
                      [&](int c, uint32_t* n, const kpd_keypoint** src) {
            if (a.mask[c]) {
                const uint32_t off = t.sparse_base[c];
                *n = clamp_count(off, t.own_count[c], a.list_cap);
                *src = t.sparse + off;
            } else {
                const uint32_t off = a.off_prev[c];
                *n = clamp_count(off, a.count_prev[c], a.list_cap);
                *src = a.list_prev + off;
            }
        });
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *work_count = 0;
}

// Concatenate the D_n of every active stream of a tick table (one workgroup
// per stream; offsets from the counts of lower-numbered streams).
__global__ __launch_bounds__(256) void k_gather_batch(const TickArgs* table, int n, kpd_keypoint* out,
                                                      uint32_t out_cap, uint32_t* counts)
{
    const int i = blockIdx.x;
    __shared__ uint32_t s_part[4];
    uint32_t acc = 0;
    for (int j = threadIdx.x; j < i; j += 256)
        if (table[j].active) acc += *table[j].d.total_cur;
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
    __syncthreads();
    const uint32_t base = s_part[0] + s_part[1] + s_part[2] + s_part[3];
    const TickArgs& t = table[i];
    const uint32_t cnt = t.active ? *t.d.total_cur : 0u;
    if (threadIdx.x == 0) counts[i] = cnt;
    for (uint32_t k = threadIdx.x; k < cnt; k += 256)
        if (base + k < out_cap) out[base + k] = t.d.list_cur[k];
}

// ------------------------------------------------------------- launchers

hipError_t launch_gather_batch(const TickArgs* table, int n, kpd_keypoint* out, uint32_t out_cap, uint32_t* counts,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_batch, dim3(n), dim3(256), 0, s, table, n, out, out_cap, counts);
    return hipGetLastError();
}

int frame_sad_lds_off(int tile, int O)
{
    if (tile == 128 && O <= kRegOctaves) return 0;   // no level buffers in LDS
    int lv = 0;
    for (int o = 0; o < O; ++o) lv += (tile >> o) * (tile >> o);
    return round_up(lv, 16);
}

int frame_lds_bytes(int tile, int O, int sad_slots)
{
    return frame_sad_lds_off(tile, O) + 4 * sad_slots + 2 * 2 * tile;
}

hipError_t set_detect_lds_limit(int lds_bytes)
{
    // the limit is a property of the kernels, shared by every stream: only raise it
    static std::atomic<int> g_limit{65536};
    int cur = g_limit.load();
    while (lds_bytes > cur && !g_limit.compare_exchange_weak(cur, lds_bytes)) {
    }
    if (lds_bytes <= cur) return hipSuccess;
    const void* kernels[] = {
        reinterpret_cast<const void*>(k_detect1<kDetLatency>),
        reinterpret_cast<const void*>(k_detect_pixel_batch<kDetLatency>),
    };
    for (const void* k : kernels) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_frame(const FrameArgs& a, hipStream_t s)
{
    const int grid = (a.ntiles + kXcds - 1) / kXcds * kXcds;
    hipLaunchKernelGGL(k_frame1, dim3(grid), dim3(kFrameBlock), frame_lds_bytes(a.tile, a.O, a.sad_slots), s, a);
    return hipGetLastError();
}

hipError_t launch_detect(const DetectArgs& a, int ncell, int lds_bytes, hipStream_t s)
{
    hipLaunchKernelGGL(k_detect1<kDetLatency>, dim3(ncell), dim3(kDetLatency), lds_bytes, s, a);
    return hipGetLastError();
}

hipError_t launch_detect_pixel_batch(const TickArgs* table, const uint16_t* map, int ncells, int lds_bytes,
                                     hipStream_t s)
{
    hipLaunchKernelGGL(k_detect_pixel_batch<kDetLatency>, dim3(ncells), dim3(kDetLatency), lds_bytes, s, table, map);
    return hipGetLastError();
}

hipError_t launch_publish(const uint32_t* hdr, int total_word, const kpd_keypoint* list, uint32_t pre,
                          const uint8_t* mask, int ncell, uint32_t stage_entries, uint8_t* stage, hipStream_t s)
{
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(kPublishBlock), 0, s, hdr, total_word, list, pre, mask, ncell,
                       stage_entries, stage);
    return hipGetLastError();
}

hipError_t launch_describe(const DescArgs& a, int ncell, hipStream_t s)
{
    hipLaunchKernelGGL(k_describe1, dim3(ncell), dim3(kDescBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pixel_diff_chunk(const PixelChunkArgs& a, hipStream_t s)
{
    const int items = a.n_frames * a.ncell;
    hipLaunchKernelGGL(k_pixel_diff_chunk, dim3((items + kDiffWaves - 1) / kDiffWaves), dim3(64 * kDiffWaves), 0, s,
                       a);
    return hipGetLastError();
}

hipError_t launch_pixel_features_chunk(const PixelChunkArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_pixel_features_chunk, dim3(a.ncell, a.n_frames), dim3(kDescBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pixel_gather_chunk(const PixelChunkArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_pixel_gather_chunk, dim3(a.ncell, a.n_frames), dim3(kDescBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pixel_merge_chunk(const PixelChunkArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_pixel_merge_chunk, dim3(a.ncell), dim3(kMergeBlock), a.lds_bytes, s, a);
    return hipGetLastError();
}

hipError_t launch_describe_batch(const TickArgs* table, const uint16_t* map, int ncells, hipStream_t s)
{
    hipLaunchKernelGGL(k_describe_batch, dim3(ncells), dim3(kDescBlock), 0, s, table, map);
    return hipGetLastError();
}

hipError_t launch_describe_chunk(const DescChunkArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_describe_chunk, dim3(a.ncell, a.n_frames), dim3(kDescBlock), 0, s, a);
    hipLaunchKernelGGL(k_carry_chunk_features, dim3(a.ncell, a.n_frames), dim3(kDescBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_frame_chunk(const FrameArgs& a, size_t pyr_stride, const ChunkHead& h, int lds_bytes, hipStream_t s)
{
    const int nblocks = h.n_frames * h.ntiles;
    const int grid = (nblocks + kXcds - 1) / kXcds * kXcds;
    hipLaunchKernelGGL(k_frame_chunk, dim3(grid), dim3(kFrameBlock), lds_bytes, s, a, h, pyr_stride);
    return hipGetLastError();
}

int frame_seq_lds_bytes(int slots, int run) { return 4 * slots * ((run + 3) / 4 * 4) + 2 * (256 + 128); }

hipError_t frame_seq_capacity(int lds_bytes, int* blocks)
{
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(k_frame_chunk_seq<256, false>),
                                                         kFrameBlock, (size_t)lds_bytes);
    *blocks = per * cus;
    return e;
}

hipError_t launch_frame_chunk_seq(const FrameArgs& a, size_t pyr_stride, const ChunkHead& h, const SeqGrid& g,
                                  bool nt, hipStream_t s)
{
    const int total = (h.n_frames + g.run - 1) / g.run * g.ntiles;
    const int grid = (total + kXcds - 1) / kXcds * kXcds;
    const int lds = frame_seq_lds_bytes(g.slots, g.run);
    if (g.tile_w == 256 && nt)
        hipLaunchKernelGGL((k_frame_chunk_seq<256, true>), dim3(grid), dim3(kFrameBlock), lds, s, a, h, pyr_stride, g);
    else if (g.tile_w == 256)
        hipLaunchKernelGGL((k_frame_chunk_seq<256, false>), dim3(grid), dim3(kFrameBlock), lds, s, a, h, pyr_stride, g);
    else if (nt)
        hipLaunchKernelGGL((k_frame_chunk_seq<128, true>), dim3(grid), dim3(kFrameBlock), lds, s, a, h, pyr_stride, g);
    else
        hipLaunchKernelGGL((k_frame_chunk_seq<128, false>), dim3(grid), dim3(kFrameBlock), lds, s, a, h, pyr_stride, g);
    return hipGetLastError();
}

hipError_t launch_spec_chunk(const ChunkHead& h, hipStream_t s)
{
    hipLaunchKernelGGL(k_spec_chunk, dim3((h.ncell + kWaveCells - 1) / kWaveCells), dim3(kWaveCells * 64), 0, s, h);
    return hipGetLastError();
}

hipError_t launch_spec2_chunk(const ChunkHead& h, const uint32_t* own, hipStream_t s)
{
    hipLaunchKernelGGL(k_spec2_chunk, dim3((h.ncell + kWaveCells - 1) / kWaveCells), dim3(kWaveCells * 64), 0, s,
                       h, own);
    return hipGetLastError();
}

hipError_t launch_resolve_chunk(const ChunkHead& h, const uint32_t* own, hipStream_t s)
{
    hipLaunchKernelGGL(k_resolve_chunk, dim3((h.ncell + kWaveCells - 1) / kWaveCells), dim3(kWaveCells * 64), 0, s,
                       h, own);
    return hipGetLastError();
}

hipError_t launch_mark_chunk(const ChunkHead& h, hipStream_t s)
{
    const int n = (h.n_frames + 63) / 64 * 64 * h.ncell;   // a wave per cell and 64 frames
    hipLaunchKernelGGL(k_mark_chunk, dim3((n + kMarkBlock - 1) / kMarkBlock), dim3(kMarkBlock), 0, s, h);
    return hipGetLastError();
}

hipError_t launch_compact_chunk(const CompactArgs& a, int n_frames, hipStream_t s)
{
    hipLaunchKernelGGL(k_compact_chunk, dim3(n_frames), dim3(kCompact), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------ k_tick

// Device-wide barrier of the single-launch tick: every workgroup arrives,
// then waits until all gridDim.x have. The fences publish each
// workgroup's writes (pyramid, SAD sums, sparse lists) to every XCD before
// it arrives and make the others' visible after it leaves. The wait is
// bounded: on time-out it flags every active stream's error word and goes
// on, so the kernel always ends.
__device__ void tick_barrier(uint32_t* ctr, const TickArgs* table, int nstreams)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(ctr, 1u);
        int spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gridDim.x) {
            if (++spins > kSpinLimit) {
                for (int i = 0; i < nstreams; ++i)
                    if (table[i].active) __hip_atomic_store(table[i].d.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
    }
    __syncthreads();
}

// One batch tick in one launch: the tile passes of every active stream
// (banded over the XCDs), a device-wide barrier, the marks of every cell
// (Eq. 2 per cell, Eqs. 3-4) with the marked ones detected by the group
// detector's one-cell layouts into their stream's sparse list, a second
// barrier, and each stream's D_n (Eq. 1). Items are dealt to the
// workgroups in turn; the grid is at most what fits on the device at once,
// so every workgroup reaches every barrier.
__global__ __launch_bounds__(kFrameBlock) void k_tick(const TickArgs* table, const uint16_t* fmap, int nframe,
                                                      const uint16_t* cmap, int ncells, int nstreams, TickSync* sync,
                                                      int parity)
{
    extern __shared__ __align__(16) uint8_t sm[];
    const int G = gridDim.x;   // a multiple of kXcds: item i runs on XCD i % kXcds
    for (int i = blockIdx.x; i < (nframe + kXcds - 1) / kXcds * kXcds; i += G) {
        const int b = xcd_band_tile(i, nframe);
        if (b >= nframe) continue;
        const TickArgs& t = table[fmap[b]];
        if (!t.active || !t.f_on) continue;
        const FrameArgs& a = t.f;
        const FrameSrc f{a.cur, a.prev, a.cur_pitch, a.prev_pitch, a.cur_aligned, a.prev_aligned, a.sad_on, 0, a.sad};
        const int local = b - t.tile_base;
        frame_tile(a, f, local % a.tiles_x, local / a.tiles_x, sm);
        __syncthreads();   // the LDS is reused by the next tile
    }
    tick_barrier(&sync->arrive[parity][0], table, nstreams);
    for (int g = blockIdx.x; g < ncells; g += G) {
        const TickArgs& t = table[cmap[g]];
        if (!t.active || t.d.id_mode != 0) continue;
        const int c = g - t.cell_base;
        const bool mark = cell_marked(t.d, c);
        if (threadIdx.x == 0) {
            t.d.mask[c] = (uint8_t)mark;
            t.d.sad_next[c] = 0;
        }
        if (!mark) continue;
        const GroupOut out{t.sparse, t.own_count, t.d.list_cap};
        detect_group<kFrameBlock>(t.glay1 + c, t.d.lvl, t.d.pitch, t.al8, t.d.lvl0_aligned, t.d.t, out, sm);
        __syncthreads();   // the LDS is reused by the next cell
    }
    tick_barrier(&sync->arrive[parity][1], table, nstreams);
    for (int i = blockIdx.x; i < nstreams; i += G) {
        const TickArgs& t = table[i];
        if (!t.active || t.d.id_mode != 0) continue;
        const DetectArgs& a = t.d;
        compact_frame<kFrameBlock>(a.nc * a.nr, a.list_cap, a.list_cur, a.count_cur, a.off_cur, a.total_cur,
                                   [&](int c, uint32_t* n, const kpd_keypoint** src) {
            if (a.mask[c]) {
                const uint32_t off = t.sparse_base[c];
                *n = clamp_count(off, t.own_count[c], a.list_cap);
                *src = t.sparse + off;
            } else {
                const uint32_t off = a.off_prev[c];
                *n = clamp_count(off, a.count_prev[c], a.list_cap);
                *src = a.list_prev + off;
            }
        });
    }
    // the next tick's counters; no workgroup of this tick reads them
    if (blockIdx.x == 0 && threadIdx.x == 0) sync->arrive[parity ^ 1][0] = sync->arrive[parity ^ 1][1] = 0u;
}

hipError_t tick_capacity(int lds_bytes, int* blocks)
{
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess && lds_bytes > 65536)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_tick), hipFuncAttributeMaxDynamicSharedMemorySize,
                                lds_bytes);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(k_tick), kFrameBlock,
                                                         (size_t)lds_bytes);
    *blocks = per * cus;
    return e;
}

hipError_t launch_tick(const TickArgs* table, const uint16_t* fmap, int nframe, const uint16_t* cmap, int ncells,
                       int nstreams, TickSync* sync, int parity, int grid, int lds_bytes, hipStream_t s)
{
    hipLaunchKernelGGL(k_tick, dim3(grid), dim3(kFrameBlock), lds_bytes, s, table, fmap, nframe, cmap, ncells,
                       nstreams, sync, parity);
    return hipGetLastError();
}

hipError_t launch_frame_batch(const TickArgs* table, const uint16_t* map, int nblocks, int lds_bytes, hipStream_t s)
{
    const int grid = (nblocks + kXcds - 1) / kXcds * kXcds;
    hipLaunchKernelGGL(k_frame_batch, dim3(grid), dim3(kFrameBlock), lds_bytes, s, table, map, nblocks);
    return hipGetLastError();
}

hipError_t launch_mark_batch(const TickArgs* table, const uint16_t* map, int ncells, uint32_t* work,
                             uint32_t* work_count, hipStream_t s)
{
    hipLaunchKernelGGL(k_mark_batch, dim3((ncells + kMarkBlock - 1) / kMarkBlock), dim3(kMarkBlock), 0, s, table, map,
                       ncells, work, work_count);
    return hipGetLastError();
}

hipError_t launch_compact_batch(const TickArgs* table, int n, uint32_t* work_count, hipStream_t s)
{
    hipLaunchKernelGGL(k_compact_batch, dim3(n), dim3(kCompact), 0, s, table, work_count);
    return hipGetLastError();
}


}  // namespace kpd
