// Kernels of the temporally coherent detector, the comparison system of
// Sec. 4: keypoints of a group's first frame propagated to the following
// frames by block matching of 16 x 16 patches, a coarse spiral search over
// 2-pixel steps, then a quarter-pixel one, with early termination.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kpd_tcd.h"

namespace kpd {
namespace {

constexpr int kTcdBlock = 256;
constexpr int kTcdWaves = kTcdBlock / 64;
constexpr int kCoarseR = 6, kCoarseScale = 8;   // (2u, 2v) pixels, |u|, |v| <= 6
constexpr int kFineR = 7, kFineScale = 1;       // (u/4, v/4) pixels, |u|, |v| <= 7
// Every sample a track's searches read lies within 22 pixels of the track's
// position in I_{n-1} (displacements up to 12 + 1.75 pixels, the patch's
// 8 pixels, the bilinear neighbour), so each workgroup stages that 45 x 45
// region of I_n in LDS once.
constexpr int kReach = 22;
constexpr int kRegion = 2 * kReach + 1;
constexpr int kRegionPitch = 48;

// Usable position: the patch's samples and their right and lower neighbours
// lie in the frame.
__device__ __forceinline__ bool usable(int W, int H, int X, int Y)
{
    return X >= 32 && Y >= 32 && X + 28 <= 4 * (W - 2) && Y + 28 <= 4 * (H - 2);
}

// The k-th offset of the spiral order: ring r holds indices (2r-1)^2 ..
// (2r+1)^2 - 1 and starts at its top-left corner, walking the top row
// rightwards, the right column down, the bottom row leftwards and the left
// column up (y down).
__device__ __forceinline__ void spiral_uv(int k, int& u, int& v)
{
    u = 0;
    v = 0;
    if (k == 0) return;
    int r = 1;
    while ((2 * r + 1) * (2 * r + 1) <= k) ++r;
    const int e = k - (2 * r - 1) * (2 * r - 1), side = e / (2 * r), pos = e - side * 2 * r;
    switch (side) {
    case 0: u = -r + pos; v = -r; break;
    case 1: u = r; v = -r + pos; break;
    case 2: u = r - pos; v = r; break;
    default: u = -r; v = r - pos; break;
    }
}

// SAD between the reference patch and the bilinear patch whose top-left
// sample has integer part (rx, ry) in the region and fraction (a, b). Each
// lane starts at a different patch row (`rot`), so the lanes of a wave,
// whose candidates sit a few pixels apart, spread their LDS reads over the
// banks.
__device__ int patch_sad(const uint8_t* ref, const uint8_t* reg, int rx, int ry, int a, int b, int rot)
{
    const int w00 = (4 - a) * (4 - b), w10 = a * (4 - b), w01 = (4 - a) * b, w11 = a * b;
    int sad = 0;
    for (int jj = 0; jj < 16; ++jj) {
        const int j = (jj + rot) & 15;
        const uint8_t* r0 = reg + (ry + j) * kRegionPitch + rx;
        const uint8_t* r1 = r0 + kRegionPitch;
        const uint8_t* q = ref + j * 16;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int v = (w00 * r0[i] + w10 * r0[i + 1] + w01 * r1[i] + w11 * r1[i + 1] + 8) >> 4;
            sad += abs((int)q[i] - v);
        }
    }
    return sad;
}

struct Best {
    int x, y, sad;
};

// One search step around (X, Y), by the whole workgroup: thread i takes
// the i-th candidate of the spiral order (256 threads cover both grids). In
// each wave a ballot finds its earliest candidate with a SAD below t_et and
// a min-reduction its lowest (SAD, index) key; the waves' results meet in
// LDS. The earliest candidate below t_et over all waves is the step's
// result when there is one (every earlier candidate had a SAD of at least
// t_et, so a sequential search would have stopped there with it as the
// lowest so far); otherwise the lowest SAD, earliest on ties. sad < 0 when
// no candidate is usable.
__device__ Best search(const uint8_t* ref, const uint8_t* reg, int ox, int oy, int W, int H, int X, int Y, int R,
                       int scale, int t_et, int* s_et, int* s_min)
{
    const int n = (2 * R + 1) * (2 * R + 1);
    const int k = threadIdx.x, lane = k & 63, wave = k >> 6;
    int cx = 0, cy = 0, sad = 0;
    bool ok = k < n;
    if (ok) {
        int u, v;
        spiral_uv(k, u, v);
        cx = X + scale * u;
        cy = Y + scale * v;
        ok = usable(W, H, cx, cy);
    }
    if (ok) sad = patch_sad(ref, reg, (cx >> 2) - 8 - ox, (cy >> 2) - 8 - oy, cx & 3, cy & 3, k);
    const uint64_t et = __ballot(ok && sad < t_et);
    int et_key = 0x7FFFFFFF;   // (index, SAD) of the wave's earliest candidate below t_et
    if (et) {
        const int first = __builtin_ctzll(et);
        et_key = ((wave * 64 + first) << 16) | __shfl(sad, first);   // sad <= 65280 < 2^16
    }
    int key = ok ? (sad << 8) | k : 0x7FFFFFFF;   // sad <= 65280, k < 256
    for (int off = 32; off > 0; off >>= 1) key = min(key, __shfl_xor(key, off));
    if (lane == 0) {
        s_et[wave] = et_key;
        s_min[wave] = key;
    }
    __syncthreads();
    int e = 0x7FFFFFFF, m = 0x7FFFFFFF;
#pragma unroll
    for (int w = 0; w < kTcdWaves; ++w) {
        e = min(e, s_et[w]);
        m = min(m, s_min[w]);
    }
    __syncthreads();   // s_et and s_min are rewritten by the next step
    int idx, bs;
    if (e != 0x7FFFFFFF) {
        idx = e >> 16;
        bs = e & 0xFFFF;
    } else if (m != 0x7FFFFFFF) {
        idx = m & 255;
        bs = m >> 8;
    } else {
        return Best{0, 0, -1};
    }
    int u, v;
    spiral_uv(idx, u, v);
    return Best{X + scale * u, Y + scale * v, bs};
}

// One workgroup per track (grid-stride over the device-side count): the
// patch in I_{n-1} and the region of I_n go to LDS, then the coarse and the
// fine step, each with one candidate per thread.
__global__ __launch_bounds__(kTcdBlock) void k_tcd_track(TcdTrackArgs a)
{
    __shared__ uint8_t s_ref[256];
    __shared__ uint8_t s_reg[kRegion * kRegionPitch];
    __shared__ int s_et[kTcdWaves], s_min[kTcdWaves];
    static_assert(kTcdBlock >= (2 * kFineR + 1) * (2 * kFineR + 1), "one candidate per thread");
    static_assert(kTcdBlock >= (2 * kCoarseR + 1) * (2 * kCoarseR + 1), "one candidate per thread");
    const uint32_t n = min(*a.in_count, a.cap);
    for (uint32_t k = blockIdx.x; k < n; k += gridDim.x) {
        const kpd_track t = a.in[k];
        if (!usable(a.W, a.H, t.x4, t.y4)) {
            if (threadIdx.x == 0) a.keep[k] = 0;
            continue;
        }
        // the reference patch: one bilinear sample per thread, all in the frame
        {
            const int fa = t.x4 & 3, fb = t.y4 & 3;
            const int w00 = (4 - fa) * (4 - fb), w10 = fa * (4 - fb), w01 = (4 - fa) * fb, w11 = fa * fb;
            const int q = threadIdx.x, i = q & 15, j = q >> 4;
            const uint8_t* p = a.prev + (size_t)((t.y4 >> 2) - 8 + j) * a.prev_pitch + ((t.x4 >> 2) - 8 + i);
            s_ref[q] = (uint8_t)((w00 * p[0] + w10 * p[1] + w01 * p[a.prev_pitch] + w11 * p[a.prev_pitch + 1] + 8) >> 4);
        }
        // the region of I_n around the track, coordinates clamped to the
        // frame (clamped pixels are read only by unusable candidates, which
        // are skipped)
        const int ox = (t.x4 >> 2) - kReach, oy = (t.y4 >> 2) - kReach;
        for (int q = threadIdx.x; q < kRegion * kRegion; q += kTcdBlock) {
            const int yy = q / kRegion, xx = q - yy * kRegion;
            const int gx = min(max(ox + xx, 0), a.W - 1), gy = min(max(oy + yy, 0), a.H - 1);
            s_reg[yy * kRegionPitch + xx] = a.cur[(size_t)gy * a.cur_pitch + gx];
        }
        __syncthreads();
        const Best c = search(s_ref, s_reg, ox, oy, a.W, a.H, t.x4, t.y4, kCoarseR, kCoarseScale, a.t_et, s_et, s_min);
        Best f = c;
        if (c.sad >= 0) f = search(s_ref, s_reg, ox, oy, a.W, a.H, c.x, c.y, kFineR, kFineScale, a.t_et, s_et, s_min);
        if (threadIdx.x == 0) {
            const bool kept = c.sad >= 0 && f.sad < a.t_bm;
            a.keep[k] = kept ? 1u : 0u;
            if (kept) {
                kpd_track o = t;
                o.x4 = f.x;
                o.y4 = f.y;
                o.sad = (uint32_t)f.sad;
                a.moved[k] = o;
            }
        }
        __syncthreads();   // the LDS patch and region are reused by the next track
    }
}

// The kept tracks in input order: one workgroup, 1024 items per round, a
// ballot prefix within each wave and the wave totals in LDS.
constexpr int kCompactBlock = 1024;

__global__ __launch_bounds__(kCompactBlock) void k_tcd_compact(TcdCompactArgs a)
{
    __shared__ uint32_t s_wave[kCompactBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t n = min(*a.in_count, a.cap);
    uint32_t total = 0;
    for (uint32_t base = 0; base < n; base += kCompactBlock) {
        const uint32_t i = base + threadIdx.x;
        const bool f = i < n && a.keep[i] != 0;
        const uint64_t m = __ballot(f);
        if (lane == 0) s_wave[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = 0, round = 0;
        for (int w = 0; w < kCompactBlock / 64; ++w) {
            const uint32_t c = s_wave[w];
            before += w < wave ? c : 0;
            round += c;
        }
        if (f) {
            const uint32_t pos = total + before + (uint32_t)__popcll(m & ((1ull << lane) - 1));
            a.out[pos] = a.moved[i];
        }
        total += round;
        __syncthreads();   // s_wave is rewritten by the next round
    }
    if (threadIdx.x == 0) *a.out_count = total;
}

// The group's first frame: D_n's keypoints at their footprint centres.
__global__ __launch_bounds__(256) void k_tcd_seed(TcdSeedArgs a)
{
    const uint32_t n = min(*a.count, a.cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const kpd_keypoint p = a.list[i];
        const int o = p.octave;
        kpd_track t;
        t.x4 = 4 * ((int)p.x << o) + 2 * ((1 << o) - 1);
        t.y4 = 4 * ((int)p.y << o) + 2 * ((1 << o) - 1);
        t.octave = p.octave;
        t.pad = 0;
        t.score = p.score;
        t.sad = 0;
        a.out[i] = t;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.out_count = n;
}

}  // namespace

hipError_t launch_tcd_seed(const TcdSeedArgs& a, hipStream_t s)
{
    const uint32_t blocks = a.cap == 0 ? 1u : std::min<uint32_t>((a.cap + 255) / 256, 256u);
    hipLaunchKernelGGL(k_tcd_seed, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tcd_track(const TcdTrackArgs& a, hipStream_t s)
{
    const uint32_t blocks = a.cap == 0 ? 1u : std::min<uint32_t>(a.cap, 4096u);
    hipLaunchKernelGGL(k_tcd_track, dim3(blocks), dim3(kTcdBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tcd_compact(const TcdCompactArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_tcd_compact, dim3(1), dim3(kCompactBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace kpd
