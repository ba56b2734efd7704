// Kernels of the gfx950 group detector (kpd_group.h): full-frame chunks,
// one workgroup per (frame, group of cells); single frames with the
// per-cell mask, one workgroup per cell; and the listed marked cells of
// masked chunks and batch ticks, one cell per workgroup at a time.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kpd_group.h"

namespace kpd {

// Every cell of every frame of a chunk, a workgroup per (frame, group):
// items banded over the XCDs so that a frame's neighbouring groups, which
// share apron rows and columns, share an L2. Sets the cells' mark bits.
template <int NT>
__global__ __launch_bounds__(NT) void k_detect_chunk_groups(const ChunkArgs* table, ChunkHead h, GroupArgs g)
{
    extern __shared__ __align__(16) uint8_t sm[];
    const int total = h.n_frames * g.ngroups;
    const int per = (total + kXcdsG - 1) / kXcdsG;
    const int item = (int)(blockIdx.x % kXcdsG) * per + (int)(blockIdx.x / kXcdsG);
    if (item >= total) return;
    const int j = item / g.ngroups, grp = item - j * g.ngroups;
    const ChunkArgs& t = table[j];
    const GroupLayout* gl = g.layouts + grp;
    if (threadIdx.x < 64) {
        // the group's cells are marked in frame j (their words are shared
        // across frames: each frame sets its own bit)
        const int gc0 = gl->gc0, gc1 = gl->gc1, gr0 = gl->gr0, gr1 = gl->gr1;
        const int ncx = gc1 - gc0;
        for (int k = threadIdx.x; k < ncx * (gr1 - gr0); k += 64) {
            const int c = (gr0 + k / ncx) * g.nc + gc0 + k % ncx;
            atomicOr(&t.marks[(size_t)c * t.Kw + (j >> 6)], 1ull << (j & 63));
            if (j == h.n_frames - 1) t.d.mask[c] = 1;
        }
    }
    const uint8_t* lv[KPD_MAX_OCTAVES];
    int pt[KPD_MAX_OCTAVES];
#pragma unroll
    for (int o = 0; o < KPD_MAX_OCTAVES; ++o) {
        lv[o] = t.d.lvl[o];
        pt[o] = t.d.pitch[o];
    }
    lv[0] = h.frames + (size_t)j * h.stride;
    pt[0] = h.pitch;
    const GroupOut out{t.d.list_cur, t.own_count, t.d.list_cap};
    detect_group<NT>(gl, lv, pt, g.al8, h.aligned, h.t, out, sm);
}

// One frame of one stream with the per-cell mask: cell c decides its mark
// (Eq. 2 read per cell from the SAD, Eqs. 3-4 from its count in D_{n-1});
// a marked cell detects with its one-cell layout and writes its keypoints
// at its base of the sparse list. Unmarked cells only record their mark;
// k_compact1 then builds D_n (Eq. 1). No workgroup waits for another.
template <int NT>
__global__ __launch_bounds__(NT) void k_det1_groups(DetectArgs a, GroupArgs g, kpd_keypoint* sparse, uint32_t* own)
{
    extern __shared__ __align__(16) uint8_t sm[];
    const int c = blockIdx.x;
    bool mark = a.all_marked != 0;
    if (!mark) {
        const int64_t area = (int64_t)a.col_w[c % a.nc] * a.row_h[c / a.nc];
        const bool id = a.id_on && (int64_t)a.sad[c] > (int64_t)a.id_thresh * area;
        mark = id || a.count_prev[c] >= a.kb_thresh;
    }
    if (threadIdx.x == 0) {
        a.mask[c] = (uint8_t)mark;
        a.sad_next[c] = 0;
    }
    if (!mark) return;
    const GroupOut out{sparse, own, a.list_cap};
    detect_group<NT>(g.layouts + c, a.lvl, a.pitch, g.al8, a.lvl0_aligned, a.t, out, sm);
}

// Listed (frame, cell) items of a chunk (marks from the SAD, or from the
// counts in rounds): workgroups take items in turn; cell c of frame j
// detects with its one-cell layout on frame j's levels and writes its
// keypoints at its base of frame j's sparse list. Round 0 takes items
// [0, count 0), round 1 [count 0, count 0 + count 1).
template <int NT>
__global__ __launch_bounds__(NT) void k_detect_list_groups(const ChunkArgs* table, ChunkHead h, GroupArgs g, int round)
{
    extern __shared__ __align__(16) uint8_t sm[];
    const uint32_t b = round ? h.work_count[0] : 0u;
    const uint32_t n = b + h.work_count[round];
    for (uint32_t it = b + blockIdx.x; it < n; it += gridDim.x) {
        const uint32_t item = h.work[it];
        const int j = (int)(item / (uint32_t)h.ncell);
        const int c = (int)(item - (uint32_t)j * h.ncell);
        const ChunkArgs& t = table[j];
        const uint8_t* lv[KPD_MAX_OCTAVES];
        int pt[KPD_MAX_OCTAVES];
#pragma unroll
        for (int o = 0; o < KPD_MAX_OCTAVES; ++o) {
            lv[o] = t.d.lvl[o];
            pt[o] = t.d.pitch[o];
        }
        lv[0] = h.frames + (size_t)j * h.stride;
        pt[0] = h.pitch;
        const GroupOut out{t.d.list_cur, t.own_count, t.d.list_cap};
        detect_group<NT>(g.layouts + c, lv, pt, g.al8, h.aligned, h.t, out, sm);
        __syncthreads();   // the layout and the LDS maps are reused by the next item
    }
}

// Listed cells of a batch tick: work item g is cell g - cell_base of stream
// map[g], detected with that stream's one-cell layout on its levels.
template <int NT>
__global__ __launch_bounds__(NT) void k_detect_list_batch_groups(const TickArgs* table, const uint16_t* map,
                                                                 const uint32_t* work, const uint32_t* work_count)
{
    extern __shared__ __align__(16) uint8_t sm[];
    const uint32_t n = *work_count;
    for (uint32_t it = blockIdx.x; it < n; it += gridDim.x) {
        const int gi = (int)work[it];
        const TickArgs& t = table[map[gi]];
        const int c = gi - t.cell_base;
        const GroupOut out{t.sparse, t.own_count, t.d.list_cap};
        detect_group<NT>(t.glay1 + c, t.d.lvl, t.d.pitch, t.al8, t.d.lvl0_aligned, t.d.t, out, sm);
        __syncthreads();
    }
}

hipError_t launch_detect_list_groups(const ChunkArgs* table, const ChunkHead& h, const GroupArgs& g, int lds_bytes,
                                     int threads, int round, hipStream_t s)
{
    const int items = h.n_frames * h.ncell;
    const int cap = threads == 128 ? 4096 : 2048;
    const int grid = items < cap ? items : cap;
    if (threads == 512)
        hipLaunchKernelGGL(k_detect_list_groups<512>, dim3(grid), dim3(512), lds_bytes, s, table, h, g, round);
    else if (threads == 128)
        hipLaunchKernelGGL(k_detect_list_groups<128>, dim3(grid), dim3(128), lds_bytes, s, table, h, g, round);
    else
        hipLaunchKernelGGL(k_detect_list_groups<256>, dim3(grid), dim3(256), lds_bytes, s, table, h, g, round);
    return hipGetLastError();
}

hipError_t launch_detect_list_batch_groups(const TickArgs* table, const uint16_t* map, int ncells,
                                           const uint32_t* work, const uint32_t* work_count, int lds_bytes,
                                           hipStream_t s)
{
    const int grid = ncells < 2048 ? ncells : 2048;
    hipLaunchKernelGGL(k_detect_list_batch_groups<256>, dim3(grid), dim3(256), lds_bytes, s, table, map, work,
                       work_count);
    return hipGetLastError();
}

hipError_t launch_det1_groups(const DetectArgs& a, const GroupArgs& g, kpd_keypoint* sparse, uint32_t* own,
                              int ncell, int lds_bytes, int threads, hipStream_t s)
{
    if (threads == 1024)
        hipLaunchKernelGGL(k_det1_groups<1024>, dim3(ncell), dim3(1024), lds_bytes, s, a, g, sparse, own);
    else if (threads == 512)
        hipLaunchKernelGGL(k_det1_groups<512>, dim3(ncell), dim3(512), lds_bytes, s, a, g, sparse, own);
    else
        hipLaunchKernelGGL(k_det1_groups<256>, dim3(ncell), dim3(256), lds_bytes, s, a, g, sparse, own);
    return hipGetLastError();
}

hipError_t launch_detect_chunk_groups(const ChunkArgs* table, const ChunkHead& h, const GroupArgs& g, int lds_bytes,
                                      int threads, hipStream_t s)
{
    const int total = h.n_frames * g.ngroups;
    const int grid = (total + kXcdsG - 1) / kXcdsG * kXcdsG;
    if (threads == 512)
        hipLaunchKernelGGL(k_detect_chunk_groups<512>, dim3(grid), dim3(512), lds_bytes, s, table, h, g);
    else
        hipLaunchKernelGGL(k_detect_chunk_groups<256>, dim3(grid), dim3(256), lds_bytes, s, table, h, g);
    return hipGetLastError();
}

namespace {
const void* const kGroupKernels[] = {reinterpret_cast<const void*>(k_detect_chunk_groups<512>),
                                     reinterpret_cast<const void*>(k_detect_chunk_groups<256>),
                                     reinterpret_cast<const void*>(k_det1_groups<1024>),
                                     reinterpret_cast<const void*>(k_det1_groups<512>),
                                     reinterpret_cast<const void*>(k_det1_groups<256>),
                                     reinterpret_cast<const void*>(k_detect_list_groups<512>),
                                     reinterpret_cast<const void*>(k_detect_list_groups<256>),
                                     reinterpret_cast<const void*>(k_detect_list_groups<128>),
                                     reinterpret_cast<const void*>(k_detect_list_batch_groups<256>)};
}  // namespace

hipError_t group_static_lds(int* bytes)
{
    *bytes = 0;
    for (const void* k : kGroupKernels) {
        hipFuncAttributes fa{};
        const hipError_t e = hipFuncGetAttributes(&fa, k);
        if (e != hipSuccess) return e;
        *bytes = std::max(*bytes, (int)fa.sharedSizeBytes);
    }
    return hipSuccess;
}

hipError_t set_group_lds_limit(int lds_bytes)
{
    if (lds_bytes <= 65536) return hipSuccess;
    for (const void* k : kGroupKernels) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace kpd
