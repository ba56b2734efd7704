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
// 8 pixels, the bilinear neighbour), so each wave stages that 45 x 45
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
// sample has integer part (rx, ry) in the region and fraction (a, b).
__device__ int patch_sad(const uint8_t* ref, const uint8_t* reg, int rx, int ry, int a, int b)
{
    const int w00 = (4 - a) * (4 - b), w10 = a * (4 - b), w01 = (4 - a) * b, w11 = a * b;
    int sad = 0;
    for (int j = 0; j < 16; ++j) {
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

// One search step around (X, Y): the lanes take 64 spiral candidates at a
// time; the first round with a SAD below t_et ends the step at its earliest
// such candidate (every earlier one had a SAD of at least t_et, so it is
// also the lowest so far), otherwise the lowest SAD, earliest on ties, wins.
// sad < 0 when no candidate is usable.
__device__ Best search(const uint8_t* ref, const uint8_t* reg, int ox, int oy, int W, int H, int X, int Y, int R,
                       int scale, int t_et, int lane)
{
    const int n = (2 * R + 1) * (2 * R + 1);
    int best_key = 0x7FFFFFFF;
    for (int base = 0; base < n; base += 64) {
        const int k = base + lane;
        int cx = 0, cy = 0, sad = 0;
        bool ok = k < n;
        if (ok) {
            int u, v;
            spiral_uv(k, u, v);
            cx = X + scale * u;
            cy = Y + scale * v;
            ok = usable(W, H, cx, cy);
        }
        if (ok) sad = patch_sad(ref, reg, (cx >> 2) - 8 - ox, (cy >> 2) - 8 - oy, cx & 3, cy & 3);
        const uint64_t et = __ballot(ok && sad < t_et);
        if (et) {
            const int first = __builtin_ctzll(et);
            return Best{__shfl(cx, first), __shfl(cy, first), __shfl(sad, first)};
        }
        int key = ok ? (sad << 8) | k : 0x7FFFFFFF;   // sad <= 65280, k < 256
        for (int off = 32; off > 0; off >>= 1) key = min(key, __shfl_xor(key, off));
        best_key = min(best_key, key);
    }
    if (best_key == 0x7FFFFFFF) return Best{0, 0, -1};
    int u, v;
    spiral_uv(best_key & 255, u, v);
    return Best{X + scale * u, Y + scale * v, best_key >> 8};
}

// One wave per track (grid-stride over the device-side count): the patch
// in I_{n-1} and the region of I_n go to LDS, then the coarse and the fine
// step.
__global__ __launch_bounds__(kTcdBlock) void k_tcd_track(TcdTrackArgs a)
{
    __shared__ uint8_t s_ref[kTcdWaves][256];
    __shared__ uint8_t s_reg[kTcdWaves][kRegion * kRegionPitch];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint8_t* ref = s_ref[wave];
    uint8_t* reg = s_reg[wave];
    const uint32_t n = min(*a.in_count, a.cap);
    for (uint32_t k = blockIdx.x * kTcdWaves + wave; k < n; k += gridDim.x * kTcdWaves) {
        const kpd_track t = a.in[k];
        if (!usable(a.W, a.H, t.x4, t.y4)) {
            if (lane == 0) a.keep[k] = 0;
            continue;
        }
        // the reference patch: 4 bilinear samples per lane, all in the frame
        {
            const int fa = t.x4 & 3, fb = t.y4 & 3;
            const int w00 = (4 - fa) * (4 - fb), w10 = fa * (4 - fb), w01 = (4 - fa) * fb, w11 = fa * fb;
            const int x0 = (t.x4 >> 2) - 8, y0 = (t.y4 >> 2) - 8;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int q = m * 64 + lane, i = q & 15, j = q >> 4;
                const uint8_t* p = a.prev + (size_t)(y0 + j) * a.prev_pitch + (x0 + i);
                ref[q] = (uint8_t)((w00 * p[0] + w10 * p[1] + w01 * p[a.prev_pitch] + w11 * p[a.prev_pitch + 1] + 8) >> 4);
            }
        }
        // the region of I_n around the track, coordinates clamped to the
        // frame (clamped pixels are read only by unusable candidates, which
        // are skipped)
        const int ox = (t.x4 >> 2) - kReach, oy = (t.y4 >> 2) - kReach;
        for (int q = lane; q < kRegion * kRegion; q += 64) {
            const int yy = q / kRegion, xx = q - yy * kRegion;
            const int gx = min(max(ox + xx, 0), a.W - 1), gy = min(max(oy + yy, 0), a.H - 1);
            reg[yy * kRegionPitch + xx] = a.cur[(size_t)gy * a.cur_pitch + gx];
        }
        __builtin_amdgcn_wave_barrier();
        const Best c = search(ref, reg, ox, oy, a.W, a.H, t.x4, t.y4, kCoarseR, kCoarseScale, a.t_et, lane);
        Best f = c;
        if (c.sad >= 0) f = search(ref, reg, ox, oy, a.W, a.H, c.x, c.y, kFineR, kFineScale, a.t_et, lane);
        if (lane == 0) {
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
        __builtin_amdgcn_wave_barrier();   // the LDS patch and region are reused by the next track
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
    const uint32_t blocks = a.cap == 0 ? 1u : std::min<uint32_t>((a.cap + kTcdWaves - 1) / kTcdWaves, 2048u);
    hipLaunchKernelGGL(k_tcd_track, dim3(blocks), dim3(kTcdBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tcd_compact(const TcdCompactArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_tcd_compact, dim3(1), dim3(kCompactBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace kpd
