// C ABI of the masked multi-scale FAST detector: arena layout, stream state
// and per-frame launch sequence. The declarations and their contracts are in
// include/kpd.h.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/kpd.h"
#include "kpd_geom.h"
#include "kpd_kernels.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return KPD_EDEVICE;
}

#define KPD_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Byte layout of one stream's device arena.
struct Layout {
    int W = 0, H = 0, O = 0, nc = 0, nr = 0, ncell = 0;
    int w[KPD_MAX_OCTAVES] = {}, h[KPD_MAX_OCTAVES] = {}, pitch[KPD_MAX_OCTAVES] = {};
    int slot_pitch = 0;
    int pyr_tile = 64;
    size_t off_hdr = 0, off_slot[2] = {0, 0}, off_lvl[KPD_MAX_OCTAVES] = {};
    size_t off_sad = 0, off_count = 0, off_offsets = 0, off_base = 0, off_mask = 0;
    size_t off_store = 0, off_out = 0;
    size_t store_cap = 0;
    int lds_bytes = 0;
    size_t total = 0;
    std::vector<uint32_t> base;  // per-cell slot start in the keypoint store, plus the end
};

bool valid_params(int W, int H, const kpd_params* p, std::string* why)
{
    if (!p) { *why = "params is NULL"; return false; }
    if (W < 1 || H < 1 || W > KPD_MAX_DIM || H > KPD_MAX_DIM) { *why = "frame size out of range"; return false; }
    if (p->fast_t < 1 || p->fast_t > 254) { *why = "fast_t must be in 1..254"; return false; }
    if (p->n_octaves < 1 || p->n_octaves > KPD_MAX_OCTAVES) { *why = "n_octaves out of range"; return false; }
    if ((W >> (p->n_octaves - 1)) < 1 || (H >> (p->n_octaves - 1)) < 1) {
        *why = "frame too small for n_octaves";
        return false;
    }
    if (p->grid_cols < 1 || p->grid_rows < 1 || p->grid_cols > W || p->grid_rows > H) {
        *why = "grid out of range";
        return false;
    }
    if (kpd::ceil_div(W, p->grid_cols) > KPD_MAX_CELL || kpd::ceil_div(H, p->grid_rows) > KPD_MAX_CELL) {
        *why = "cells larger than KPD_MAX_CELL pixels";
        return false;
    }
    return true;
}

bool make_layout(int W, int H, const kpd_params* p, Layout* L, std::string* why)
{
    if (!valid_params(W, H, p, why)) return false;
    L->W = W; L->H = H; L->O = p->n_octaves; L->nc = p->grid_cols; L->nr = p->grid_rows;
    L->ncell = L->nc * L->nr;
    for (int o = 0; o < L->O; ++o) {
        L->w[o] = W >> o;
        L->h[o] = H >> o;
        L->pitch[o] = kpd::round_up(L->w[o], 64);
    }
    L->slot_pitch = kpd::round_up(W, 64);
    L->pyr_tile = std::max(64, 1 << (L->O - 1));

    // per-cell keypoint slots and the detection kernel's LDS need
    L->base.assign(L->ncell + 1, 0);
    size_t cap = 0;
    int lds = 0;
    for (int c = 0; c < L->ncell; ++c) {
        const kpd::Box r = kpd::cell_rect(c, W, H, L->nc, L->nr);
        kpd::Box dec[KPD_MAX_OCTAVES], sb[KPD_MAX_OCTAVES];
        for (int o = 0; o < L->O; ++o) dec[o] = kpd::decision_box(r, o, L->w[o], L->h[o]);
        for (int o = 0; o < L->O; ++o) sb[o] = kpd::score_box(dec, o, L->O, L->w[o], L->h[o]);
        L->base[c] = (uint32_t)cap;
        for (int o = 0; o < L->O; ++o) cap += kpd::decision_capacity(dec[o]);
        lds = std::max(lds, kpd::cell_lds_bytes(sb, L->O));
        if (cap > 0xFFFFFFF0ull) { *why = "keypoint store too large"; return false; }
    }
    L->base[L->ncell] = (uint32_t)cap;
    L->store_cap = std::max<size_t>(cap, 1);
    L->lds_bytes = kpd::detect_lds_bytes(lds);

    size_t off = 0;
    L->off_hdr = off; off = align_up(off + 64);
    for (int k = 0; k < 2; ++k) { L->off_slot[k] = off; off = align_up(off + (size_t)L->slot_pitch * H); }
    for (int o = 1; o < L->O; ++o) { L->off_lvl[o] = off; off = align_up(off + (size_t)L->pitch[o] * L->h[o]); }
    const size_t nc4 = (size_t)L->ncell * 4;
    L->off_sad = off; off = align_up(off + nc4);
    L->off_count = off; off = align_up(off + nc4);
    L->off_offsets = off; off = align_up(off + nc4);
    L->off_base = off; off = align_up(off + nc4 + 4);
    L->off_mask = off; off = align_up(off + (size_t)L->ncell);
    L->off_store = off; off = align_up(off + L->store_cap * sizeof(kpd_keypoint));
    L->off_out = off; off = align_up(off + L->store_cap * sizeof(kpd_keypoint));
    L->total = off;
    return true;
}

}  // namespace

struct kpd_stream {
    Layout L;
    kpd_params p{};
    hipStream_t stream = nullptr;
    uint8_t* arena = nullptr;
    int n_pushed = 0;
    bool force_all = true;
    int cur_slot = 0;
    const uint8_t* prev0 = nullptr;
    int prev_pitch = 0;
    bool closed = false;

    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(arena + off); }
};

extern "C" {

const char* kpd_last_error(void) { return g_err.c_str(); }

size_t stream_bytes(int width, int height, const kpd_params* params)
{
    Layout L;
    std::string why;
    if (!make_layout(width, height, params, &L, &why)) {
        g_err = why;
        return 0;
    }
    return L.total;
}

int open_stream(int width, int height, const kpd_params* params, void* dev_arena, size_t arena_bytes,
                void* hip_stream, kpd_stream** out)
{
    if (!out) return fail(KPD_EINVAL, "out is NULL");
    *out = nullptr;
    Layout L;
    std::string why;
    if (!make_layout(width, height, params, &L, &why)) return fail(KPD_EINVAL, why);
    if (!dev_arena) return fail(KPD_EINVAL, "arena is NULL");
    if (reinterpret_cast<uintptr_t>(dev_arena) % kAlign) return fail(KPD_EINVAL, "arena not 256-byte aligned");
    if (arena_bytes < L.total)
        return fail(KPD_ENOMEM, "arena has " + std::to_string(arena_bytes) + " bytes, stream needs " +
                                    std::to_string(L.total));
    // cells of at most KPD_MAX_CELL pixels need < 64 KiB of LDS per workgroup
    if (L.lds_bytes > 65536) return fail(KPD_EINVAL, "cells need more LDS than a workgroup can hold");

    kpd_stream* s = new (std::nothrow) kpd_stream();
    if (!s) return fail(KPD_ENOMEM, "host allocation failed");
    s->L = std::move(L);
    s->p = *params;
    s->stream = reinterpret_cast<hipStream_t>(hip_stream);
    s->arena = reinterpret_cast<uint8_t*>(dev_arena);

    // constant per-cell slot starts, and zeroed counters
    hipError_t e = hipMemcpyAsync(s->at<uint32_t>(s->L.off_base), s->L.base.data(), s->L.base.size() * 4,
                                  hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->arena + s->L.off_hdr, 0, 64, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->arena + s->L.off_count, 0, (size_t)s->L.ncell * 4, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "open_stream initialisation");
    }
    *out = s;
    return KPD_OK;
}

int set_thresholds(kpd_stream* s, int32_t fast_t, int32_t id_thresh, uint32_t kb_thresh)
{
    if (!s || s->closed) return fail(KPD_ESTATE, "stream is closed");
    if (fast_t < 1 || fast_t > 254) return fail(KPD_EINVAL, "fast_t must be in 1..254");
    if (fast_t != s->p.fast_t) s->force_all = true;
    s->p.fast_t = fast_t;
    s->p.id_thresh = id_thresh;
    s->p.kb_thresh = kb_thresh;
    return KPD_OK;
}

int push_frame(kpd_stream* s, const uint8_t* frame, size_t pitch_bytes, int flags)
{
    if (!s || s->closed) return fail(KPD_ESTATE, "stream is closed");
    const Layout& L = s->L;
    if (!frame) return fail(KPD_EINVAL, "frame is NULL");
    if (pitch_bytes < (size_t)L.W || pitch_bytes > (1u << 30)) return fail(KPD_EINVAL, "bad pitch");
    if (flags != KPD_FRAME_HOST && flags != KPD_FRAME_DEVICE && flags != KPD_FRAME_DEVICE_RETAIN)
        return fail(KPD_EINVAL, "bad flags");

    const uint8_t* cur;
    int cur_pitch;
    if (flags == KPD_FRAME_DEVICE_RETAIN) {
        cur = frame;
        cur_pitch = (int)pitch_bytes;
    } else {
        uint8_t* dst = s->at<uint8_t>(L.off_slot[s->cur_slot]);
        KPD_HIP(hipMemcpy2DAsync(dst, L.slot_pitch, frame, pitch_bytes, L.W, L.H,
                                 flags == KPD_FRAME_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                                 s->stream));
        cur = dst;
        cur_pitch = L.slot_pitch;
        s->cur_slot ^= 1;
    }

    const bool all_marked = s->force_all || s->p.id_thresh < 0 || s->p.kb_thresh == 0;
    if (!all_marked) {
        kpd::MaskArgs m{};
        m.cur = cur; m.prev = s->prev0;
        m.cur_pitch = cur_pitch; m.prev_pitch = s->prev_pitch;
        m.W = L.W; m.H = L.H; m.nc = L.nc; m.nr = L.nr;
        m.id_on = s->p.id_thresh < 255;
        m.id_thresh = s->p.id_thresh;
        m.kb_thresh = s->p.kb_thresh;
        m.count = s->at<uint32_t>(L.off_count);
        m.sad = s->at<uint32_t>(L.off_sad);
        m.mask = s->at<uint8_t>(L.off_mask);
        KPD_HIP(kpd::launch_cell_mask(m, L.ncell, s->stream));
    }

    if (L.O > 1) {
        kpd::PyrArgs pa{};
        pa.lvl0 = cur; pa.pitch0 = cur_pitch;
        for (int o = 1; o < L.O; ++o) {
            pa.lvl[o] = s->at<uint8_t>(L.off_lvl[o]);
            pa.pitch[o] = L.pitch[o];
            pa.w[o] = L.w[o];
            pa.h[o] = L.h[o];
        }
        pa.W = L.W; pa.H = L.H; pa.O = L.O; pa.tile = L.pyr_tile;
        KPD_HIP(kpd::launch_pyramid(pa, s->stream));
    }

    kpd::DetectArgs d{};
    d.lvl[0] = cur; d.pitch[0] = cur_pitch; d.w[0] = L.W; d.h[0] = L.H;
    for (int o = 1; o < L.O; ++o) {
        d.lvl[o] = s->at<uint8_t>(L.off_lvl[o]);
        d.pitch[o] = L.pitch[o];
        d.w[o] = L.w[o];
        d.h[o] = L.h[o];
    }
    d.W = L.W; d.H = L.H; d.O = L.O; d.nc = L.nc; d.nr = L.nr;
    d.t = s->p.fast_t;
    d.all_marked = all_marked ? 1 : 0;
    d.mask = s->at<uint8_t>(L.off_mask);
    d.count = s->at<uint32_t>(L.off_count);
    d.offsets = s->at<uint32_t>(L.off_offsets);
    d.store_base = s->at<uint32_t>(L.off_base);
    d.store = s->at<kpd_keypoint>(L.off_store);
    d.hdr = s->at<uint32_t>(L.off_hdr);
    KPD_HIP(kpd::launch_detect(d, L.ncell, L.lds_bytes, s->stream));

    kpd::GatherArgs g{};
    g.count = d.count; g.offsets = d.offsets; g.store_base = d.store_base; g.store = d.store;
    g.out = s->at<kpd_keypoint>(L.off_out);
    KPD_HIP(kpd::launch_gather(g, L.ncell, s->stream));

    s->prev0 = cur;
    s->prev_pitch = cur_pitch;
    s->force_all = false;
    s->n_pushed += 1;
    return KPD_OK;
}

int get_keypoints(kpd_stream* s, kpd_keypoint* out, size_t capacity, size_t* count, uint8_t* cell_mask)
{
    if (!s || s->closed) return fail(KPD_ESTATE, "stream is closed");
    if (!count) return fail(KPD_EINVAL, "count is NULL");
    if (s->n_pushed == 0) return fail(KPD_ESTATE, "no frame pushed yet");
    uint32_t total = 0;
    KPD_HIP(hipMemcpyAsync(&total, s->at<uint32_t>(s->L.off_hdr), 4, hipMemcpyDeviceToHost, s->stream));
    KPD_HIP(hipStreamSynchronize(s->stream));
    *count = total;
    if (total > capacity) return fail(KPD_ETRUNC, "capacity smaller than the keypoint count");
    if (total > 0) {
        if (!out) return fail(KPD_EINVAL, "out is NULL");
        KPD_HIP(hipMemcpyAsync(out, s->at<kpd_keypoint>(s->L.off_out), (size_t)total * sizeof(kpd_keypoint),
                               hipMemcpyDeviceToHost, s->stream));
    }
    if (cell_mask)
        KPD_HIP(hipMemcpyAsync(cell_mask, s->at<uint8_t>(s->L.off_mask), (size_t)s->L.ncell,
                               hipMemcpyDeviceToHost, s->stream));
    KPD_HIP(hipStreamSynchronize(s->stream));
    return KPD_OK;
}

int close_stream(kpd_stream* s)
{
    if (!s || s->closed) return fail(KPD_ESTATE, "stream is closed");
    hipError_t e = hipStreamSynchronize(s->stream);
    s->closed = true;
    delete s;
    if (e != hipSuccess) return hip_fail(e, "close_stream");
    return KPD_OK;
}

int kpd_device_result(kpd_stream* s, const kpd_keypoint** d_list, const uint32_t** d_count)
{
    if (!s || s->closed) return fail(KPD_ESTATE, "stream is closed");
    if (d_list) *d_list = s->at<kpd_keypoint>(s->L.off_out);
    if (d_count) *d_count = s->at<uint32_t>(s->L.off_hdr);
    return KPD_OK;
}

int kpd_cell_stats(kpd_stream* s, uint32_t* sad, uint32_t* counts)
{
    if (!s || s->closed) return fail(KPD_ESTATE, "stream is closed");
    if (s->n_pushed == 0) return fail(KPD_ESTATE, "no frame pushed yet");
    const size_t n = (size_t)s->L.ncell * 4;
    if (sad) KPD_HIP(hipMemcpyAsync(sad, s->at<uint32_t>(s->L.off_sad), n, hipMemcpyDeviceToHost, s->stream));
    if (counts)
        KPD_HIP(hipMemcpyAsync(counts, s->at<uint32_t>(s->L.off_count), n, hipMemcpyDeviceToHost, s->stream));
    KPD_HIP(hipStreamSynchronize(s->stream));
    return KPD_OK;
}

int kpd_pyramid_level(kpd_stream* s, int octave, uint8_t* out)
{
    if (!s || s->closed) return fail(KPD_ESTATE, "stream is closed");
    if (s->n_pushed == 0) return fail(KPD_ESTATE, "no frame pushed yet");
    if (octave < 1 || octave >= s->L.O || !out) return fail(KPD_EINVAL, "bad octave or NULL output");
    const Layout& L = s->L;
    KPD_HIP(hipMemcpy2DAsync(out, L.w[octave], s->at<uint8_t>(L.off_lvl[octave]), L.pitch[octave], L.w[octave],
                             L.h[octave], hipMemcpyDeviceToHost, s->stream));
    KPD_HIP(hipStreamSynchronize(s->stream));
    return KPD_OK;
}

}  // extern "C"
