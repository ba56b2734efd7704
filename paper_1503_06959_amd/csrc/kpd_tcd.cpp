// C ABI of the temporally coherent detector (the comparison system of
// Sec. 4): arena layout, group bookkeeping and the per-frame launches. The
// contracts are in include/kpd.h.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdint>
#include <new>
#include <string>

#include "../../include/kpd.h"
#include "kpd_errors.h"
#include "kpd_tcd.h"
#include "kpd_trace.h"

namespace {

#define TCD_HIP(call)                                            \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return kpd::api_hip_fail(e_, #call); \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct TcdLayout {
    int W = 0, H = 0;
    kpd_params det{};
    kpd_tcd_params tp{};
    size_t inner = 0;               // the inner stream's arena, at offset 0
    int slot_pitch = 0;
    size_t off_slot[2] = {0, 0};    // frames copied in (host or device sources)
    size_t off_tracks[2] = {0, 0};  // tracks of the previous and the current frame
    size_t off_moved = 0, off_keep = 0, off_count = 0;
    uint32_t cap = 0;
    size_t total = 0;
};

// At most one keypoint per 2 x 2 block of every level's interior: no two
// keypoints of a level are 8-neighbours.
uint32_t track_cap(int W, int H, int O)
{
    uint64_t n = 0;
    for (int o = 0; o < O; ++o) n += (uint64_t)(((W >> o) + 1) / 2) * (uint64_t)(((H >> o) + 1) / 2);
    return (uint32_t)std::min<uint64_t>(n + 16, 0xFFFFFFF0ull);
}

bool make_layout(int W, int H, const kpd_params* det, const kpd_tcd_params* tp, TcdLayout* L, std::string* why)
{
    if (!det || !tp) { *why = "params are NULL"; return false; }
    if (tp->gop < 1) { *why = "gop must be >= 1"; return false; }
    if (tp->t_bm < 0 || tp->t_et < 0) { *why = "thresholds must be >= 0"; return false; }
    if (tp->pad != 0) { *why = "pad must be 0"; return false; }
    L->W = W;
    L->H = H;
    L->det = *det;
    L->det.id_thresh = -1;   // the group's first frame is detected whole
    L->det.kb_thresh = 0xFFFFFFFFu;
    L->det.chunk_frames = 0;
    L->det.layer_mask = 0;
    L->det.features = 0;
    L->tp = *tp;
    L->inner = stream_bytes(W, H, &L->det);
    if (L->inner == 0) { *why = kpd_last_error(); return false; }
    size_t off = align_up(L->inner);
    L->slot_pitch = (W + 63) / 64 * 64;
    for (int k = 0; k < 2; ++k) { L->off_slot[k] = off; off = align_up(off + (size_t)L->slot_pitch * H); }
    L->cap = track_cap(W, H, det->n_octaves);
    for (int k = 0; k < 2; ++k) { L->off_tracks[k] = off; off = align_up(off + (size_t)L->cap * sizeof(kpd_track)); }
    L->off_moved = off; off = align_up(off + (size_t)L->cap * sizeof(kpd_track));
    L->off_keep = off;  off = align_up(off + (size_t)L->cap * 4);
    L->off_count = off; off = align_up(off + 64);
    L->total = off;
    return true;
}

}  // namespace

struct kpd_tcd {
    TcdLayout L;
    hipStream_t stream = nullptr;
    uint8_t* arena = nullptr;
    kpd_stream* det = nullptr;
    int n_frames = 0;        // frames since open or reset
    int fb = 0;              // buffer of the current tracks
    int cur_slot = 0;
    const uint8_t* prev = nullptr;
    int prev_pitch = 0;
    template <class T> T* at(size_t off) { return reinterpret_cast<T*>(arena + off); }
};

extern "C" {

size_t tcd_bytes(int width, int height, const kpd_params* det, const kpd_tcd_params* tp)
{
    TcdLayout L;
    std::string why;
    if (!make_layout(width, height, det, tp, &L, &why)) {
        kpd::api_fail(KPD_EINVAL, why);
        return 0;
    }
    return L.total;
}

int tcd_open(int width, int height, const kpd_params* det, const kpd_tcd_params* tp, void* dev_arena,
             size_t arena_bytes, void* hip_stream, kpd_tcd** out)
{
    if (!out) return kpd::api_fail(KPD_EINVAL, "out is NULL");
    *out = nullptr;
    TcdLayout L;
    std::string why;
    if (!make_layout(width, height, det, tp, &L, &why)) return kpd::api_fail(KPD_EINVAL, why);
    if (!dev_arena) return kpd::api_fail(KPD_EINVAL, "arena is NULL");
    if (reinterpret_cast<uintptr_t>(dev_arena) % kAlign) return kpd::api_fail(KPD_EINVAL, "arena not 256-byte aligned");
    if (arena_bytes < L.total)
        return kpd::api_fail(KPD_ENOMEM, "arena has " + std::to_string(arena_bytes) + " bytes, tracker needs " +
                                             std::to_string(L.total));
    kpd_stream* inner = nullptr;
    const int rc = open_stream(width, height, &L.det, dev_arena, L.inner, hip_stream, &inner);
    if (rc != KPD_OK) return rc;
    kpd_tcd* s = new (std::nothrow) kpd_tcd();
    if (!s) {
        close_stream(inner);
        return kpd::api_fail(KPD_ENOMEM, "host allocation failed");
    }
    s->L = L;
    s->stream = reinterpret_cast<hipStream_t>(hip_stream);
    s->arena = reinterpret_cast<uint8_t*>(dev_arena);
    s->det = inner;
    hipError_t e = hipMemsetAsync(s->arena + L.off_count, 0, 64, s->stream);
    if (e != hipSuccess || !kpd::handle_add(s)) {
        close_stream(inner);
        delete s;
        return e != hipSuccess ? kpd::api_hip_fail(e, "tcd_open") : kpd::api_fail(KPD_ENOMEM, "host allocation failed");
    }
    *out = s;
    return KPD_OK;
}

int tcd_push(kpd_tcd* s, const uint8_t* frame, size_t pitch_bytes, int flags)
{
    const kpd::TraceRange trace_range("kpd:tcd_push");
    if (!kpd::handle_live(s)) return kpd::api_fail(KPD_ESTATE, "tracker is closed");
    const TcdLayout& L = s->L;
    if (!frame) return kpd::api_fail(KPD_EINVAL, "frame is NULL");
    if (pitch_bytes < (size_t)L.W || pitch_bytes > (1u << 30)) return kpd::api_fail(KPD_EINVAL, "bad pitch");
    if (flags != KPD_FRAME_HOST && flags != KPD_FRAME_DEVICE && flags != KPD_FRAME_DEVICE_RETAIN)
        return kpd::api_fail(KPD_EINVAL, "bad flags");

    const uint8_t* cur = frame;
    int cur_pitch = (int)pitch_bytes;
    if (flags != KPD_FRAME_DEVICE_RETAIN) {
        uint8_t* dst = s->at<uint8_t>(L.off_slot[s->cur_slot]);
        const hipMemcpyKind kind = flags == KPD_FRAME_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        TCD_HIP(hipMemcpy2DAsync(dst, L.slot_pitch, frame, pitch_bytes, L.W, L.H, kind, s->stream));
        cur = dst;
        cur_pitch = L.slot_pitch;
        s->cur_slot ^= 1;
    }
    const int fb_prev = s->fb, fb_cur = 1 - s->fb;
    uint32_t* counts = s->at<uint32_t>(L.off_count);
    if (s->n_frames % L.tp.gop == 0) {
        // the group's first frame: full-frame detection, then every
        // keypoint becomes a track
        const int rc = push_frame(s->det, cur, (size_t)cur_pitch, KPD_FRAME_DEVICE_RETAIN);
        if (rc != KPD_OK) return rc;
        const kpd_keypoint* list = nullptr;
        const uint32_t* count = nullptr;
        const int rc2 = kpd_device_result(s->det, &list, &count);
        if (rc2 != KPD_OK) return rc2;
        kpd::TcdSeedArgs a{list, count, s->at<kpd_track>(L.off_tracks[fb_cur]), counts + fb_cur, L.cap};
        TCD_HIP(kpd::launch_tcd_seed(a, s->stream));
    } else {
        kpd::TcdTrackArgs a{};
        a.prev = s->prev;
        a.prev_pitch = s->prev_pitch;
        a.cur = cur;
        a.cur_pitch = cur_pitch;
        a.W = L.W;
        a.H = L.H;
        a.t_bm = L.tp.t_bm;
        a.t_et = L.tp.t_et;
        a.in = s->at<kpd_track>(L.off_tracks[fb_prev]);
        a.in_count = counts + fb_prev;
        a.moved = s->at<kpd_track>(L.off_moved);
        a.keep = s->at<uint32_t>(L.off_keep);
        a.cap = L.cap;
        TCD_HIP(kpd::launch_tcd_track(a, s->stream));
        kpd::TcdCompactArgs c{a.moved, a.keep, a.in_count, s->at<kpd_track>(L.off_tracks[fb_cur]), counts + fb_cur,
                              L.cap};
        TCD_HIP(kpd::launch_tcd_compact(c, s->stream));
    }
    s->fb = fb_cur;
    s->prev = cur;
    s->prev_pitch = cur_pitch;
    s->n_frames += 1;
    return KPD_OK;
}

int tcd_device_result(kpd_tcd* s, const kpd_track** d_tracks, const uint32_t** d_count)
{
    if (!kpd::handle_live(s)) return kpd::api_fail(KPD_ESTATE, "tracker is closed");
    if (s->n_frames == 0 && s->prev == nullptr) return kpd::api_fail(KPD_ESTATE, "no frame pushed yet");
    if (d_tracks) *d_tracks = s->at<kpd_track>(s->L.off_tracks[s->fb]);
    if (d_count) *d_count = s->at<uint32_t>(s->L.off_count) + s->fb;
    return KPD_OK;
}

int tcd_get(kpd_tcd* s, kpd_track* out, size_t capacity, size_t* count)
{
    if (!kpd::handle_live(s)) return kpd::api_fail(KPD_ESTATE, "tracker is closed");
    if (!count) return kpd::api_fail(KPD_EINVAL, "count is NULL");
    if (s->n_frames == 0 && s->prev == nullptr) return kpd::api_fail(KPD_ESTATE, "no frame pushed yet");
    const TcdLayout& L = s->L;
    uint32_t n = 0;
    TCD_HIP(hipMemcpyAsync(&n, s->at<uint32_t>(L.off_count) + s->fb, 4, hipMemcpyDeviceToHost, s->stream));
    TCD_HIP(hipStreamSynchronize(s->stream));
    n = std::min(n, L.cap);
    *count = n;
    if (n > capacity) return kpd::api_fail(KPD_ETRUNC, "capacity smaller than the track count");
    if (n > 0) {
        if (!out) return kpd::api_fail(KPD_EINVAL, "out is NULL");
        TCD_HIP(hipMemcpyAsync(out, s->at<kpd_track>(L.off_tracks[s->fb]), (size_t)n * sizeof(kpd_track),
                               hipMemcpyDeviceToHost, s->stream));
        TCD_HIP(hipStreamSynchronize(s->stream));
    }
    return KPD_OK;
}

int tcd_reset(kpd_tcd* s)
{
    if (!kpd::handle_live(s)) return kpd::api_fail(KPD_ESTATE, "tracker is closed");
    s->n_frames = 0;
    return KPD_OK;
}

int tcd_close(kpd_tcd* s)
{
    if (!kpd::handle_live(s)) return kpd::api_fail(KPD_ESTATE, "tracker is closed");
    const int rc = close_stream(s->det);
    kpd::handle_remove(s);
    delete s;
    return rc;
}

}  // extern "C"
