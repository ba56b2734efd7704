// C ABI of detection over octaves and intra-octaves: workspace layout and
// the launch sequence. The contracts are in include/kpd.h.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdint>
#include <new>
#include <string>
#include <vector>

#include "../../include/kpd.h"
#include "kpd_errors.h"
#include "kpd_kernels.h"
#include "kpd_layers.h"
#include "kpd_trace.h"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool layer_geom(int W, int H, int O, kpd::LayerGeom* g, std::string* why)
{
    if (W < 1 || H < 1 || W > 65535 || H > 65535) { *why = "width and height must be 1..65535"; return false; }
    if (O < 1 || O > KPD_MAX_OCTAVES) { *why = "n_octaves must be 1..KPD_MAX_OCTAVES"; return false; }
    g->L = 2 * O;
    uint64_t N = 0;
    size_t off = 0;
    for (int i = 0; i < O; ++i) {
        g->w[2 * i] = W >> i;
        g->h[2 * i] = H >> i;
        g->S[2 * i] = 2 << i;
        g->w[2 * i + 1] = ((W / 3) * 2) >> i;
        g->h[2 * i + 1] = ((H / 3) * 2) >> i;
        g->S[2 * i + 1] = 3 << i;
    }
    for (int l = 0; l < g->L; ++l) {
        g->base[l] = (uint32_t)N;
        N += (uint64_t)g->w[l] * g->h[l];
        if (l > 0) { g->plane_off[l] = off; off = align_up(off + (size_t)g->w[l] * g->h[l]); }
    }
    if (N > 0x7FFFFFFFull) { *why = "frame too large"; return false; }
    g->base[g->L] = (uint32_t)N;
    g->N = (uint32_t)N;
    g->nblocks = (uint32_t)((N + kpd::kLayBlock - 1) / kpd::kLayBlock);
    g->off_score = off;  off = align_up(off + (size_t)N * 2);
    g->off_flag = off;   off = align_up(off + (size_t)N);
    g->off_bcount = off; off = align_up(off + (size_t)g->nblocks * 4 + 4);
    g->off_boff = off;   off = align_up(off + (size_t)g->nblocks * 4 + 4);
    g->total = off;
    return true;
}

kpd::LayArgs layer_args(const kpd::LayerGeom& g, const uint8_t* frame, size_t pitch_bytes, uint8_t* ws)
{
    kpd::LayArgs a{};
    a.L = g.L;
    a.N = g.N;
    for (int l = 0; l < g.L; ++l) {
        a.plane[l] = l == 0 ? frame : ws + g.plane_off[l];
        a.pitch[l] = l == 0 ? (int)pitch_bytes : g.w[l];
        a.w[l] = g.w[l];
        a.h[l] = g.h[l];
        a.S[l] = g.S[l];
        a.base[l] = g.base[l];
    }
    a.base[g.L] = g.base[g.L];
    a.score = reinterpret_cast<uint16_t*>(ws + g.off_score);
    a.flag = ws + g.off_flag;
    a.bcount = reinterpret_cast<uint32_t*>(ws + g.off_bcount);
    a.boff = reinterpret_cast<uint32_t*>(ws + g.off_boff);
    a.nblocks = g.nblocks;
    return a;
}

// Arena of the masked stream over the layers: the layer workspace, two
// frame slots, the cell tables, the mask, and per-cell counts, offsets and
// D lists that alternate between frames.
struct LsLayout {
    kpd::LayerGeom g;
    int W = 0, H = 0, O = 0, nc = 0, nr = 0, ncell = 0;
    int slot_pitch = 0;
    size_t off_ws = 0, off_slot[2] = {0, 0}, off_xs = 0, off_ys = 0, off_mask = 0, off_need = 0, off_new = 0;
    int rx = 0, ry = 0;   // cell radius of the scored neighbourhood of a marked cell
    size_t off_cnt[2] = {0, 0}, off_off[2] = {0, 0}, off_list[2] = {0, 0}, off_total = 0;
    uint32_t cap = 0;
    // chunks (chunk_frames K >= 2): K layer workspaces ws_step apart, per
    // frame and cell the mask, the scored-cell flags and the suppression
    // counts, the mark words, the sparse lists (fixed per-cell bases), the
    // lists of frames 0..K-2 with their counts, offsets and totals, and the
    // compaction's difference accumulators (all zero here) and work words
    int K = 1, Kw = 1;
    size_t ws_step = 0;
    size_t off_cmask = 0, off_cneed = 0, off_cnew = 0, off_marks = 0, off_cbase = 0, off_sparse = 0;
    size_t off_clist = 0, off_ccount = 0, off_coffs = 0, off_ctotal = 0, off_csad = 0, off_sadstat = 0;
    size_t off_sadnext = 0, off_cwork = 0;
    size_t list_stride = 0;   // entries between consecutive frames' lists
    size_t total = 0;
};

void ls_tables(const LsLayout& L, std::vector<uint32_t>* xs, std::vector<uint32_t>* ys);

// Room of cell c in a chunk's sparse list: one keypoint per 2x2 block of
// each of its layer boxes (suppression keeps no two neighbours of a layer).
uint64_t ls_cell_cap(const LsLayout& L, const std::vector<uint32_t>& xs, const std::vector<uint32_t>& ys, int c)
{
    const int cc = c % L.nc, rr = c / L.nc;
    uint64_t n = 0;
    for (int l = 0; l < L.g.L; ++l) {
        const uint64_t bw = xs[(size_t)l * (L.nc + 1) + cc + 1] - xs[(size_t)l * (L.nc + 1) + cc];
        const uint64_t bh = ys[(size_t)l * (L.nr + 1) + rr + 1] - ys[(size_t)l * (L.nr + 1) + rr];
        n += ((bw + 1) / 2) * ((bh + 1) / 2);
    }
    return n;
}

bool ls_layout(int W, int H, const kpd_params* p, LsLayout* L, std::string* why)
{
    if (!p) { *why = "params are NULL"; return false; }
    if (!layer_geom(W, H, p->n_octaves, &L->g, why)) return false;
    if (p->fast_t < 1 || p->fast_t > 254) { *why = "fast_t must be 1..254"; return false; }
    if (p->grid_cols < 1 || p->grid_rows < 1 || p->grid_cols > W || p->grid_rows > H) {
        *why = "grid must be 1..width x 1..height cells";
        return false;
    }
    L->W = W; L->H = H; L->O = p->n_octaves; L->nc = p->grid_cols; L->nr = p->grid_rows;
    L->ncell = L->nc * L->nr;
    uint64_t cap = 16;
    for (int l = 0; l < L->g.L; ++l) cap += (uint64_t)((L->g.w[l] + 1) / 2) * ((L->g.h[l] + 1) / 2);
    // the chunks' sparse lists give each cell room for one keypoint per 2x2
    // block of each layer box; the lists hold their sum too
    std::vector<uint32_t> xs, ys;
    ls_tables(*L, &xs, &ys);
    uint64_t cells_cap = 0;
    for (int c = 0; c < L->ncell; ++c) cells_cap += ls_cell_cap(*L, xs, ys, c);
    cap = std::max(cap, cells_cap);
    if (cap > 0xFFFFFFF0ull) { *why = "frame too large"; return false; }
    L->cap = (uint32_t)cap;
    L->K = std::max(1, (int)p->chunk_frames);
    if (L->K > KPD_MAX_CHUNK) { *why = "chunk_frames must be 0.." + std::to_string(KPD_MAX_CHUNK); return false; }
    L->Kw = (L->K + 63) / 64;
    L->ws_step = align_up(L->g.total);
    size_t off = 0;
    L->off_ws = off; off = align_up(off + L->ws_step * (size_t)L->K);
    L->slot_pitch = (W + 63) / 64 * 64;
    for (int k = 0; k < 2; ++k) { L->off_slot[k] = off; off = align_up(off + (size_t)L->slot_pitch * H); }
    L->off_xs = off; off = align_up(off + (size_t)L->g.L * (L->nc + 1) * 4);
    L->off_ys = off; off = align_up(off + (size_t)L->g.L * (L->nr + 1) * 4);
    L->off_mask = off; off = align_up(off + (size_t)L->ncell);
    L->off_need = off; off = align_up(off + (size_t)L->ncell);
    L->off_new = off;  off = align_up(off + (size_t)L->ncell * 4);
    // A neighbour q (same or adjacent layer, footprints meeting) of a pixel
    // p has its level-0 footprint start within max(S_p, S_q) / 2 + 1 pixels
    // of p's, so within R = S_max / 2 + 1 pixels; points R apart lie at
    // most R / (narrowest cell) + 1 cells apart.
    int smax = 0;
    for (int l = 0; l < L->g.L; ++l) smax = std::max(smax, L->g.S[l]);
    const int R = smax / 2 + 1;
    L->rx = R / (W / L->nc) + 1;
    L->ry = R / (H / L->nr) + 1;
    for (int k = 0; k < 2; ++k) {
        L->off_cnt[k] = off;  off = align_up(off + (size_t)L->ncell * 4);
        L->off_off[k] = off;  off = align_up(off + (size_t)L->ncell * 4);
        L->off_list[k] = off; off = align_up(off + (size_t)L->cap * sizeof(kpd_keypoint));
    }
    L->off_total = off; off = align_up(off + 16);
    if (L->K > 1) {
        const size_t kc = (size_t)L->K * L->ncell;
        L->list_stride = align_up((size_t)L->cap * sizeof(kpd_keypoint)) / sizeof(kpd_keypoint);
        L->off_cmask = off;   off = align_up(off + kc);
        L->off_cneed = off;   off = align_up(off + kc);
        L->off_cnew = off;    off = align_up(off + kc * 4);
        L->off_marks = off;   off = align_up(off + (size_t)L->ncell * L->Kw * 8);
        L->off_cbase = off;   off = align_up(off + (size_t)L->ncell * 4);
        L->off_sparse = off;  off += L->list_stride * sizeof(kpd_keypoint) * (size_t)L->K;
        L->off_clist = off;   off += L->list_stride * sizeof(kpd_keypoint) * (size_t)(L->K - 1);
        L->off_ccount = off;  off = align_up(off + kc * 4);
        L->off_coffs = off;   off = align_up(off + kc * 4);
        L->off_ctotal = off;  off = align_up(off + (size_t)L->K * 4);
        L->off_csad = off;    off = align_up(off + kc * 4);
        L->off_sadstat = off; off = align_up(off + (size_t)L->ncell * 4);
        L->off_sadnext = off; off = align_up(off + (size_t)L->ncell * 4);
        L->off_cwork = off;   off = align_up(off + 16);
    }
    L->total = off;
    return true;
}

// For each layer, the first pixel column whose level-0 footprint start
// floor(x S / 2) lies in cell column c or later, c = 0..nc (the last entry
// is the layer's width); rows likewise. The cell column of level-0 column X
// is floor(X nc / W).
void ls_tables(const LsLayout& L, std::vector<uint32_t>* xs, std::vector<uint32_t>* ys)
{
    auto build = [](int n_layers, const int* len, const int* S, int extent, int cells, std::vector<uint32_t>* out) {
        out->assign((size_t)n_layers * (cells + 1), 0);
        for (int l = 0; l < n_layers; ++l) {
            uint32_t* t = out->data() + (size_t)l * (cells + 1);
            int c = 0;
            for (int x = 0; x < len[l]; ++x) {
                const long X0 = ((long)x * S[l]) / 2;
                const int cx = (int)((X0 * cells) / extent);
                while (c <= cx) t[c++] = (uint32_t)x;
            }
            while (c <= cells) t[c++] = (uint32_t)len[l];
        }
    };
    build(L.g.L, L.g.w, L.g.S, L.W, L.nc, xs);
    build(L.g.L, L.g.h, L.g.S, L.H, L.nr, ys);
}

// The layers past the frame: the octaves two halvings per launch, the
// intra-octaves from the 1.5x downsampling (with d_1) and then two halvings
// per launch. n frames of a chunk: frame j at frame + j * fstep, its
// workspace at ws + j * wstep.
hipError_t build_layers(const kpd::LayerGeom& g, const uint8_t* frame, int pitch, uint8_t* ws, hipStream_t s,
                        int n = 1, size_t fstep = 0, size_t wstep = 0, const kpd::LbSlot* slots = nullptr)
{
    const int O = g.L / 2;
    auto plane = [&](int l) { return ws + g.plane_off[l]; };
    hipError_t e = hipSuccess;
    // octaves: c_i = layer 2i, from c_0 = the frame
    for (int i = 1; i < O && e == hipSuccess; i += 2) {
        const uint8_t* src = i == 1 ? frame : plane(2 * (i - 1));
        const int sp = i == 1 ? pitch : g.w[2 * (i - 1)];
        const int l1 = 2 * i, l2 = 2 * (i + 1);
        const bool two = i + 1 < O;
        e = kpd::launch_lay_quad(src, sp, plane(l1), g.w[l1], g.h[l1], two ? plane(l2) : nullptr, two ? g.w[l2] : 0,
                                 two ? g.h[l2] : 0, s, n, i == 1 ? fstep : wstep, wstep, slots, i == 1 ? 1 : 0);
    }
    // intra-octaves: d_i = layer 2i + 1
    if (e == hipSuccess) {
        const bool d1 = O > 1;
        e = kpd::launch_lay_third(frame, pitch, plane(1), g.w[1], g.h[1], d1 ? plane(3) : nullptr, d1 ? g.w[3] : 0,
                                  d1 ? g.h[3] : 0, s, n, fstep, wstep, slots);
    }
    for (int i = 2; i < O && e == hipSuccess; i += 2) {
        const int ls = 2 * (i - 1) + 1, l1 = 2 * i + 1, l2 = 2 * (i + 1) + 1;
        const bool two = i + 1 < O;
        e = kpd::launch_lay_quad(plane(ls), g.w[ls], plane(l1), g.w[l1], g.h[l1], two ? plane(l2) : nullptr,
                                 two ? g.w[l2] : 0, two ? g.h[l2] : 0, s, n, wstep, wstep, slots, 0);
    }
    return e;
}

}  // namespace

struct kpd_lstream {
    LsLayout L;
    kpd_params p{};
    hipStream_t stream = nullptr;
    uint8_t* arena = nullptr;
    std::vector<uint32_t> xs, ys;
    bool force = true;
    int fb = 0;              // buffer of the current D
    int chunk_n = 0;         // frames of the last kpd_lstream_push_frames (0: a single push since)
    std::vector<uint32_t> cbase;
    int cur_slot = 0;
    uint64_t n_pushed = 0;
    const uint8_t* prev = nullptr;
    int prev_pitch = 0;
    template <class T> T* at(size_t off) { return reinterpret_cast<T*>(arena + off); }
};

extern "C" {

size_t kpd_lstream_bytes(int width, int height, const kpd_params* params)
{
    LsLayout L;
    std::string why;
    if (!ls_layout(width, height, params, &L, &why)) {
        kpd::api_fail(KPD_EINVAL, why);
        return 0;
    }
    return L.total;
}

int kpd_lstream_open(int width, int height, const kpd_params* params, void* dev_arena, size_t arena_bytes,
                     void* hip_stream, kpd_lstream** out)
{
    if (!out) return kpd::api_fail(KPD_EINVAL, "out is NULL");
    *out = nullptr;
    LsLayout L;
    std::string why;
    if (!ls_layout(width, height, params, &L, &why)) return kpd::api_fail(KPD_EINVAL, why);
    if (!dev_arena) return kpd::api_fail(KPD_EINVAL, "arena is NULL");
    if (reinterpret_cast<uintptr_t>(dev_arena) % kAlign) return kpd::api_fail(KPD_EINVAL, "arena not 256-byte aligned");
    if (arena_bytes < L.total)
        return kpd::api_fail(KPD_ENOMEM, "arena has " + std::to_string(arena_bytes) + " bytes, stream needs " +
                                             std::to_string(L.total));
    kpd_lstream* s = new (std::nothrow) kpd_lstream();
    if (!s) return kpd::api_fail(KPD_ENOMEM, "host allocation failed");
    s->L = L;
    s->p = *params;
    s->stream = reinterpret_cast<hipStream_t>(hip_stream);
    s->arena = reinterpret_cast<uint8_t*>(dev_arena);
    ls_tables(L, &s->xs, &s->ys);
    hipError_t e = hipMemcpyAsync(s->at<uint32_t>(L.off_xs), s->xs.data(), s->xs.size() * 4, hipMemcpyHostToDevice,
                                  s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->at<uint32_t>(L.off_ys), s->ys.data(), s->ys.size() * 4, hipMemcpyHostToDevice, s->stream);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipMemsetAsync(s->at<uint32_t>(L.off_cnt[k]), 0, (size_t)L.ncell * 4, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->at<uint32_t>(L.off_total), 0, 16, s->stream);
    if (L.K > 1) {
        s->cbase.resize(L.ncell);
        uint32_t acc = 0;
        for (int c = 0; c < L.ncell; ++c) {
            s->cbase[c] = acc;
            acc += (uint32_t)ls_cell_cap(L, s->xs, s->ys, c);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->at<uint32_t>(L.off_cbase), s->cbase.data(), (size_t)L.ncell * 4,
                               hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = hipMemsetAsync(s->at<uint32_t>(L.off_csad), 0, (size_t)L.K * L.ncell * 4, s->stream);
        if (e == hipSuccess) e = hipMemsetAsync(s->at<uint32_t>(L.off_cwork), 0, 16, s->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);   // the host tables are copied before they go
    if (e != hipSuccess) {
        delete s;
        return kpd::api_hip_fail(e, "kpd_lstream_open");
    }
    if (!kpd::handle_add(s)) {
        delete s;
        return kpd::api_fail(KPD_ENOMEM, "host allocation failed");
    }
    *out = s;
    return KPD_OK;
}

int kpd_lstream_push(kpd_lstream* s, const uint8_t* frame, size_t pitch_bytes, int flags)
{
    const kpd::TraceRange trace_range("kpd:lstream_push");
    if (!kpd::handle_live(s)) return kpd::api_fail(KPD_ESTATE, "stream is closed");
    const LsLayout& L = s->L;
    if (!frame) return kpd::api_fail(KPD_EINVAL, "frame is NULL");
    if (pitch_bytes < (size_t)L.W || pitch_bytes > (1u << 30)) return kpd::api_fail(KPD_EINVAL, "bad pitch");
    if (flags != KPD_FRAME_HOST && flags != KPD_FRAME_DEVICE && flags != KPD_FRAME_DEVICE_RETAIN)
        return kpd::api_fail(KPD_EINVAL, "bad flags");
    const uint8_t* cur = frame;
    int cur_pitch = (int)pitch_bytes;
    if (flags != KPD_FRAME_DEVICE_RETAIN) {
        uint8_t* dst = s->at<uint8_t>(L.off_slot[s->cur_slot]);
        const hipMemcpyKind kind = flags == KPD_FRAME_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        hipError_t e = hipMemcpy2DAsync(dst, L.slot_pitch, frame, pitch_bytes, L.W, L.H, kind, s->stream);
        if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_lstream_push");
        cur = dst;
        cur_pitch = L.slot_pitch;
        s->cur_slot ^= 1;
    }
    const int fp = s->fb, fc = 1 - s->fb;
    uint8_t* ws = s->at<uint8_t>(L.off_ws);
    kpd::LayArgs la = layer_args(L.g, cur, (size_t)cur_pitch, ws);
    la.t = s->p.fast_t;
    kpd::LsArgs a{};
    a.cur = cur;
    a.prev = s->force ? cur : s->prev;
    a.cur_pitch = cur_pitch;
    a.prev_pitch = s->force ? cur_pitch : s->prev_pitch;
    a.nc = L.nc;
    a.nr = L.nr;
    a.ncell = L.ncell;
    a.force = s->force ? 1 : 0;
    a.id_thresh = s->p.id_thresh;
    a.kb_thresh = s->p.kb_thresh;
    a.xs = s->at<uint32_t>(L.off_xs);
    a.ys = s->at<uint32_t>(L.off_ys);
    a.mask = s->at<uint8_t>(L.off_mask);
    a.cnt_prev = s->at<uint32_t>(L.off_cnt[fp]);
    a.off_prev = s->at<uint32_t>(L.off_off[fp]);
    a.list_prev = s->at<kpd_keypoint>(L.off_list[fp]);
    a.cnt_cur = s->at<uint32_t>(L.off_cnt[fc]);
    a.off_cur = s->at<uint32_t>(L.off_off[fc]);
    a.list_cur = s->at<kpd_keypoint>(L.off_list[fc]);
    a.total_cur = s->at<uint32_t>(L.off_total) + fc;
    a.cap = L.cap;
    a.need_score = s->at<uint8_t>(L.off_need);
    a.cell_new = s->at<uint32_t>(L.off_new);
    la.cell_new = a.cell_new;
    a.rx = L.rx;
    a.ry = L.ry;
    la.need_score = a.need_score;
    la.need_flag = a.mask;
    la.nc = L.nc;
    la.nr = L.nr;
    la.W = L.W;
    la.H = L.H;
    hipError_t e = kpd::launch_ls_mask(a, s->stream);
    // the layers of I_n, as kpd_detect_layers builds them
    if (e == hipSuccess) e = build_layers(L.g, cur, cur_pitch, ws, s->stream);
    if (e == hipSuccess) e = kpd::launch_lay_score_nms(la, s->stream);
    if (e == hipSuccess) e = kpd::launch_ls_emit(a, la, s->stream);
    if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_lstream_push");
    s->fb = fc;
    s->prev = cur;
    s->prev_pitch = cur_pitch;
    s->force = false;
    s->n_pushed += 1;
    s->chunk_n = 0;
    return KPD_OK;
}

int kpd_lstream_push_frames(kpd_lstream* s, const uint8_t* frames, size_t frame_stride, size_t pitch_bytes,
                            int n_frames)
{
    const kpd::TraceRange trace_range("kpd:lstream_push_frames");
    if (!kpd::handle_live(s)) return kpd::api_fail(KPD_ESTATE, "stream is closed");
    const LsLayout& L = s->L;
    if (L.K < 2) return kpd::api_fail(KPD_EINVAL, "stream opened without chunk_frames");
    if (!frames) return kpd::api_fail(KPD_EINVAL, "frames is NULL");
    if (n_frames < 1 || n_frames > L.K) return kpd::api_fail(KPD_EINVAL, "n_frames out of range");
    if (pitch_bytes < (size_t)L.W || pitch_bytes > (1u << 30)) return kpd::api_fail(KPD_EINVAL, "bad pitch");
    if (n_frames > 1 && frame_stride < pitch_bytes * (size_t)(L.H - 1) + (size_t)L.W)
        return kpd::api_fail(KPD_EINVAL, "frames overlap");
    // T_H marks a cell from the previous frame's counts, a chain through the
    // chunk's frames that these passes do not follow
    const bool all_marked = s->p.id_thresh < 0 || s->p.kb_thresh == 0;
    if (!all_marked && s->p.kb_thresh != KPD_KB_OFF)
        return kpd::api_fail(KPD_EINVAL, "chunks of the layered stream need kb_thresh off");
    const int fp = s->fb, fc = 1 - s->fb;
    const int pitch = (int)pitch_bytes;
    uint8_t* ws = s->at<uint8_t>(L.off_ws);

    kpd::LsChunkArgs ca{};
    ca.frames = frames;
    ca.stride = frame_stride;
    ca.pitch = pitch;
    ca.prev0 = s->prev ? s->prev : frames;   // read only when frame 0 tests differences
    ca.prev0_pitch = s->prev ? s->prev_pitch : pitch;
    ca.n_frames = n_frames;
    ca.force0 = s->force ? 1 : 0;
    ca.all_marked = all_marked ? 1 : 0;
    ca.nc = L.nc;
    ca.nr = L.nr;
    ca.ncell = L.ncell;
    ca.Kw = L.Kw;
    ca.id_thresh = s->p.id_thresh;
    ca.xs = s->at<uint32_t>(L.off_xs);
    ca.ys = s->at<uint32_t>(L.off_ys);
    ca.mask = s->at<uint8_t>(L.off_cmask);
    ca.need = s->at<uint8_t>(L.off_cneed);
    ca.cell_new = s->at<uint32_t>(L.off_cnew);
    ca.marks = s->at<unsigned long long>(L.off_marks);
    ca.last_mask = s->at<uint8_t>(L.off_mask);
    ca.sparse = s->at<kpd_keypoint>(L.off_sparse);
    ca.cbase = s->at<uint32_t>(L.off_cbase);
    ca.list_stride = L.list_stride;
    ca.cap = L.cap;
    ca.rx = L.rx;
    ca.ry = L.ry;

    kpd::LayArgs la = layer_args(L.g, frames, pitch_bytes, ws);
    la.t = s->p.fast_t;
    la.need_score = ca.need;
    la.need_flag = ca.mask;
    la.cell_new = ca.cell_new;
    la.nc = L.nc;
    la.nr = L.nr;
    la.W = L.W;
    la.H = L.H;
    la.frame_step = frame_stride;
    la.ws_step = L.ws_step;
    la.cells_step = L.ncell;

    kpd::CompactArgs cp{};
    cp.ncell = L.ncell;
    cp.last = n_frames - 1;
    cp.Kw = L.Kw;
    cp.list_cap = L.cap;
    cp.list_stride = L.list_stride;
    cp.sparse = ca.sparse;
    cp.cell_base = ca.cbase;
    cp.marks = ca.marks;
    cp.own_count = ca.cell_new;
    cp.prev_list = s->at<kpd_keypoint>(L.off_list[fp]);
    cp.prev_count = s->at<uint32_t>(L.off_cnt[fp]);
    cp.prev_offs = s->at<uint32_t>(L.off_off[fp]);
    cp.lists = s->at<kpd_keypoint>(L.off_clist);
    cp.counts = s->at<uint32_t>(L.off_ccount);
    cp.offs = s->at<uint32_t>(L.off_coffs);
    cp.totals = s->at<uint32_t>(L.off_ctotal);
    cp.next_list = s->at<kpd_keypoint>(L.off_list[fc]);
    cp.next_count = s->at<uint32_t>(L.off_cnt[fc]);
    cp.next_offs = s->at<uint32_t>(L.off_off[fc]);
    cp.next_total = s->at<uint32_t>(L.off_total) + fc;
    cp.sad_chunk = s->at<uint32_t>(L.off_csad);
    cp.sad_stats = s->at<uint32_t>(L.off_sadstat);
    cp.sad_single_next = s->at<uint32_t>(L.off_sadnext);
    cp.work_count = s->at<uint32_t>(L.off_cwork);

    // marks and scored cells of every frame, the layers of every frame,
    // scores and suppression where needed, the marked cells' keypoints,
    // then each frame's D by Eq. 1 (the newest frame up to it that marked
    // a cell, else the list before the chunk)
    hipError_t e = kpd::launch_ls_mask_chunk(ca, s->stream);
    if (e == hipSuccess) e = build_layers(L.g, frames, pitch, ws, s->stream, n_frames, frame_stride, L.ws_step);
    if (e == hipSuccess) e = kpd::launch_lay_score_nms(la, s->stream, n_frames);
    if (e == hipSuccess) e = kpd::launch_ls_write_chunk(ca, la, s->stream);
    if (e == hipSuccess) e = kpd::launch_compact_chunk(cp, n_frames, s->stream);
    if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_lstream_push_frames");
    s->fb = fc;
    s->prev = frames + (size_t)(n_frames - 1) * frame_stride;
    s->prev_pitch = pitch;
    s->force = false;
    s->n_pushed += (uint64_t)n_frames;
    s->chunk_n = n_frames;
    return KPD_OK;
}

int kpd_lstream_get_chunk(kpd_lstream* s, int i, kpd_keypoint* out, size_t capacity, size_t* count)
{
    if (!kpd::handle_live(s)) return kpd::api_fail(KPD_ESTATE, "stream is closed");
    if (!count) return kpd::api_fail(KPD_EINVAL, "count is NULL");
    if (i < 0 || i >= s->chunk_n) return kpd::api_fail(KPD_EINVAL, "no such frame in the last chunk");
    if (i == s->chunk_n - 1) return kpd_lstream_get(s, out, capacity, count, nullptr);   // D_n itself
    const LsLayout& L = s->L;
    uint32_t total = 0;
    hipError_t e = hipMemcpyAsync(&total, s->at<uint32_t>(L.off_ctotal) + i, 4, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_lstream_get_chunk");
    total = std::min(total, L.cap);
    *count = total;
    if (total > capacity) return kpd::api_fail(KPD_ETRUNC, "capacity smaller than the keypoint count");
    if (total > 0) {
        if (!out) return kpd::api_fail(KPD_EINVAL, "out is NULL");
        e = hipMemcpyAsync(out, s->at<kpd_keypoint>(L.off_clist) + L.list_stride * (size_t)i,
                           (size_t)total * sizeof(kpd_keypoint), hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_lstream_get_chunk");
    }
    return KPD_OK;
}

int kpd_lstream_get(kpd_lstream* s, kpd_keypoint* out, size_t capacity, size_t* count, uint8_t* cell_mask)
{
    if (!kpd::handle_live(s)) return kpd::api_fail(KPD_ESTATE, "stream is closed");
    if (!count) return kpd::api_fail(KPD_EINVAL, "count is NULL");
    if (s->n_pushed == 0) return kpd::api_fail(KPD_ESTATE, "no frame pushed yet");
    const LsLayout& L = s->L;
    uint32_t n = 0;
    hipError_t e = hipMemcpyAsync(&n, s->at<uint32_t>(L.off_total) + s->fb, 4, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && cell_mask)
        e = hipMemcpyAsync(cell_mask, s->at<uint8_t>(L.off_mask), (size_t)L.ncell, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_lstream_get");
    n = std::min(n, L.cap);
    *count = n;
    if (n > capacity) return kpd::api_fail(KPD_ETRUNC, "capacity smaller than the keypoint count");
    if (n > 0) {
        if (!out) return kpd::api_fail(KPD_EINVAL, "out is NULL");
        e = hipMemcpyAsync(out, s->at<kpd_keypoint>(L.off_list[s->fb]), (size_t)n * sizeof(kpd_keypoint),
                           hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_lstream_get");
    }
    return KPD_OK;
}

int kpd_lstream_reset(kpd_lstream* s)
{
    if (!kpd::handle_live(s)) return kpd::api_fail(KPD_ESTATE, "stream is closed");
    s->force = true;
    return KPD_OK;
}

int kpd_lstream_close(kpd_lstream* s)
{
    if (!kpd::handle_live(s)) return kpd::api_fail(KPD_ESTATE, "stream is closed");
    const hipError_t e = hipStreamSynchronize(s->stream);
    kpd::handle_remove(s);
    delete s;
    if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_lstream_close");
    return KPD_OK;
}

}  // extern "C"

namespace {

// Arena of a batch of layered streams: per slot a layer workspace, the mask,
// scored cells, suppression counts and two sets of D counts, offsets, lists
// and sizes; the cell tables and the tick's slot table.
struct LbLayout {
    LsLayout s;   // one slot's geometry, capacity and cell tables
    int nslots = 0;
    size_t off_ws = 0, off_xs = 0, off_ys = 0, off_mask = 0, off_need = 0, off_new = 0, off_table = 0;
    size_t off_cnt[2] = {0, 0}, off_off[2] = {0, 0}, off_list[2] = {0, 0}, off_total[2] = {0, 0};
    size_t list_stride = 0;
    size_t total = 0;
};

bool lb_layout(int W, int H, const kpd_params* p, int nslots, LbLayout* B, std::string* why)
{
    if (nslots < 1 || nslots > 65535) { *why = "max_streams must be 1..65535"; return false; }
    kpd_params q = *p;
    q.chunk_frames = 0;
    if (!ls_layout(W, H, &q, &B->s, why)) return false;
    const LsLayout& L = B->s;
    B->nslots = nslots;
    const size_t sc = (size_t)nslots * L.ncell;
    B->list_stride = align_up((size_t)L.cap * sizeof(kpd_keypoint)) / sizeof(kpd_keypoint);
    size_t off = 0;
    B->off_ws = off;    off = align_up(off + L.ws_step * (size_t)nslots);
    B->off_xs = off;    off = align_up(off + (size_t)L.g.L * (L.nc + 1) * 4);
    B->off_ys = off;    off = align_up(off + (size_t)L.g.L * (L.nr + 1) * 4);
    B->off_mask = off;  off = align_up(off + sc);
    B->off_need = off;  off = align_up(off + sc);
    B->off_new = off;   off = align_up(off + sc * 4);
    B->off_table = off; off = align_up(off + (size_t)nslots * sizeof(kpd::LbSlot));
    for (int k = 0; k < 2; ++k) {
        B->off_cnt[k] = off;   off = align_up(off + sc * 4);
        B->off_off[k] = off;   off = align_up(off + sc * 4);
        B->off_list[k] = off;  off += B->list_stride * sizeof(kpd_keypoint) * (size_t)nslots;
        B->off_total[k] = off; off = align_up(off + (size_t)nslots * 4);
    }
    B->total = off;
    return true;
}

}  // namespace

struct kpd_lbatch {
    LbLayout B;
    kpd_params p{};
    hipStream_t stream = nullptr;
    uint8_t* arena = nullptr;
    std::vector<uint32_t> xs, ys;
    std::vector<kpd::LbSlot> slot;   // host state: previous frame, force, next buffer, staged frame
    std::vector<char> staged, ticked;
    kpd::LbSlot* host_table[2] = {nullptr, nullptr};
    hipEvent_t table_free[2] = {nullptr, nullptr};
    int tk = 0;
    template <class T> T* at(size_t off) { return reinterpret_cast<T*>(arena + off); }
};

extern "C" {

size_t kpd_lbatch_bytes(int width, int height, const kpd_params* params, int max_streams)
{
    LbLayout B;
    std::string why;
    if (!params || !lb_layout(width, height, params, max_streams, &B, &why)) {
        kpd::api_fail(KPD_EINVAL, params ? why : "params are NULL");
        return 0;
    }
    return B.total;
}

int kpd_lbatch_close(kpd_lbatch* b);

int kpd_lbatch_open(int width, int height, const kpd_params* params, int max_streams, void* dev_arena,
                    size_t arena_bytes, void* hip_stream, kpd_lbatch** out)
{
    if (!out) return kpd::api_fail(KPD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!params) return kpd::api_fail(KPD_EINVAL, "params are NULL");
    LbLayout B;
    std::string why;
    if (!lb_layout(width, height, params, max_streams, &B, &why)) return kpd::api_fail(KPD_EINVAL, why);
    if (!dev_arena) return kpd::api_fail(KPD_EINVAL, "arena is NULL");
    if (reinterpret_cast<uintptr_t>(dev_arena) % kAlign) return kpd::api_fail(KPD_EINVAL, "arena not 256-byte aligned");
    if (arena_bytes < B.total)
        return kpd::api_fail(KPD_ENOMEM, "arena has " + std::to_string(arena_bytes) + " bytes, the batch needs " +
                                             std::to_string(B.total));
    kpd_lbatch* b = new (std::nothrow) kpd_lbatch();
    if (!b) return kpd::api_fail(KPD_ENOMEM, "host allocation failed");
    if (!kpd::handle_add(b)) {   // first, so that the error path below can close it
        delete b;
        return kpd::api_fail(KPD_ENOMEM, "host allocation failed");
    }
    b->B = B;
    b->p = *params;
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->arena = reinterpret_cast<uint8_t*>(dev_arena);
    b->slot.assign((size_t)max_streams, kpd::LbSlot{});
    for (auto& sl : b->slot) sl.force = 1;
    b->staged.assign((size_t)max_streams, 0);
    b->ticked.assign((size_t)max_streams, 0);
    ls_tables(B.s, &b->xs, &b->ys);
    hipError_t e = hipMemcpyAsync(b->at<uint32_t>(B.off_xs), b->xs.data(), b->xs.size() * 4, hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->at<uint32_t>(B.off_ys), b->ys.data(), b->ys.size() * 4, hipMemcpyHostToDevice, b->stream);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = hipHostMalloc(reinterpret_cast<void**>(&b->host_table[k]), (size_t)max_streams * sizeof(kpd::LbSlot),
                          hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->table_free[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);   // the host tables are copied before they go
    if (e != hipSuccess) {
        kpd_lbatch_close(b);
        return kpd::api_hip_fail(e, "kpd_lbatch_open");
    }
    *out = b;
    return KPD_OK;
}

int kpd_lbatch_push(kpd_lbatch* b, int slot, const uint8_t* frame, size_t pitch_bytes)
{
    if (!kpd::handle_live(b)) return kpd::api_fail(KPD_ESTATE, "batch is closed");
    if (slot < 0 || slot >= b->B.nslots) return kpd::api_fail(KPD_EINVAL, "no such slot");
    if (!frame) return kpd::api_fail(KPD_EINVAL, "frame is NULL");
    if (pitch_bytes < (size_t)b->B.s.W || pitch_bytes > (1u << 30)) return kpd::api_fail(KPD_EINVAL, "bad pitch");
    if (b->staged[slot]) return kpd::api_fail(KPD_ESTATE, "a frame is already staged for this tick");
    b->slot[slot].cur = frame;
    b->slot[slot].cur_pitch = (int)pitch_bytes;
    b->staged[slot] = 1;
    return KPD_OK;
}

int kpd_lbatch_tick(kpd_lbatch* b)
{
    const kpd::TraceRange trace_range("kpd:lbatch_tick");
    if (!kpd::handle_live(b)) return kpd::api_fail(KPD_ESTATE, "batch is closed");
    const LbLayout& B = b->B;
    const LsLayout& L = B.s;
    const int n = B.nslots;
    // this host table's previous copy has been done before it is rewritten
    hipError_t e = hipEventSynchronize(b->table_free[b->tk]);
    if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_lbatch_tick");
    kpd::LbSlot* t = b->host_table[b->tk];
    for (int i = 0; i < n; ++i) {
        t[i] = b->slot[i];
        t[i].active = b->staged[i] ? 1 : 0;
        if (!t[i].prev) {   // a slot's first frame marks every cell and reads no previous frame
            t[i].prev = t[i].cur;
            t[i].prev_pitch = t[i].cur_pitch;
        }
    }
    kpd::LbSlot* dt = b->at<kpd::LbSlot>(B.off_table);
    e = hipMemcpyAsync(dt, t, (size_t)n * sizeof(kpd::LbSlot), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->table_free[b->tk], b->stream);

    kpd::LbArgs a{};
    a.slots = dt;
    a.nslots = n;
    a.nc = L.nc;
    a.nr = L.nr;
    a.ncell = L.ncell;
    a.id_thresh = b->p.id_thresh;
    a.kb_thresh = b->p.kb_thresh;
    a.xs = b->at<uint32_t>(B.off_xs);
    a.ys = b->at<uint32_t>(B.off_ys);
    a.mask = b->at<uint8_t>(B.off_mask);
    a.need = b->at<uint8_t>(B.off_need);
    a.cell_new = b->at<uint32_t>(B.off_new);
    for (int k = 0; k < 2; ++k) {
        a.cnt[k] = b->at<uint32_t>(B.off_cnt[k]);
        a.off[k] = b->at<uint32_t>(B.off_off[k]);
        a.list[k] = b->at<kpd_keypoint>(B.off_list[k]);
        a.total[k] = b->at<uint32_t>(B.off_total[k]);
    }
    a.list_stride = B.list_stride;
    a.cap = L.cap;
    a.rx = L.rx;
    a.ry = L.ry;

    uint8_t* ws = b->at<uint8_t>(B.off_ws);
    kpd::LayArgs la = layer_args(L.g, nullptr, (size_t)L.W, ws);
    la.t = b->p.fast_t;
    la.need_score = a.need;
    la.need_flag = a.mask;
    la.cell_new = a.cell_new;
    la.nc = L.nc;
    la.nr = L.nr;
    la.W = L.W;
    la.H = L.H;
    la.ws_step = L.ws_step;
    la.cells_step = L.ncell;
    la.slots = dt;
    if (e == hipSuccess) e = kpd::launch_lb_mask(a, b->stream);
    if (e == hipSuccess) e = build_layers(L.g, nullptr, 0, ws, b->stream, n, 0, L.ws_step, dt);
    if (e == hipSuccess) e = kpd::launch_lay_score_nms(la, b->stream, n);
    if (e == hipSuccess) e = kpd::launch_lb_emit(a, la, b->stream);
    if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_lbatch_tick");
    for (int i = 0; i < n; ++i) {
        if (!b->staged[i]) continue;
        kpd::LbSlot& sl = b->slot[i];
        sl.prev = sl.cur;
        sl.prev_pitch = sl.cur_pitch;
        sl.force = 0;
        sl.fb ^= 1;   // D_n went to the old fb; the next frame's goes to the other
        b->staged[i] = 0;
        b->ticked[i] = 1;
    }
    b->tk ^= 1;
    return KPD_OK;
}

int kpd_lbatch_get(kpd_lbatch* b, int slot, kpd_keypoint* out, size_t capacity, size_t* count, uint8_t* cell_mask)
{
    if (!kpd::handle_live(b)) return kpd::api_fail(KPD_ESTATE, "batch is closed");
    if (slot < 0 || slot >= b->B.nslots) return kpd::api_fail(KPD_EINVAL, "no such slot");
    if (!count) return kpd::api_fail(KPD_EINVAL, "count is NULL");
    if (!b->ticked[slot]) return kpd::api_fail(KPD_ESTATE, "the slot has had no frame yet");
    const LbLayout& B = b->B;
    const int k = 1 - b->slot[slot].fb;   // the buffer holding D_n
    uint32_t total = 0;
    hipError_t e = hipMemcpyAsync(&total, b->at<uint32_t>(B.off_total[k]) + slot, 4, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess && cell_mask)
        e = hipMemcpyAsync(cell_mask, b->at<uint8_t>(B.off_mask) + (size_t)slot * B.s.ncell, (size_t)B.s.ncell,
                           hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_lbatch_get");
    total = std::min(total, B.s.cap);
    *count = total;
    if (total > capacity) return kpd::api_fail(KPD_ETRUNC, "capacity smaller than the keypoint count");
    if (total > 0) {
        if (!out) return kpd::api_fail(KPD_EINVAL, "out is NULL");
        e = hipMemcpyAsync(out, b->at<kpd_keypoint>(B.off_list[k]) + B.list_stride * (size_t)slot,
                           (size_t)total * sizeof(kpd_keypoint), hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_lbatch_get");
    }
    return KPD_OK;
}

int kpd_lbatch_reset(kpd_lbatch* b, int slot)
{
    if (!kpd::handle_live(b)) return kpd::api_fail(KPD_ESTATE, "batch is closed");
    if (slot < 0 || slot >= b->B.nslots) return kpd::api_fail(KPD_EINVAL, "no such slot");
    b->slot[slot].force = 1;
    return KPD_OK;
}

int kpd_lbatch_close(kpd_lbatch* b)
{
    if (!kpd::handle_live(b)) return kpd::api_fail(KPD_ESTATE, "batch is closed");
    hipError_t e = hipStreamSynchronize(b->stream);
    for (int k = 0; k < 2; ++k) {
        if (b->host_table[k]) (void)hipHostFree(b->host_table[k]);
        if (b->table_free[k]) (void)hipEventDestroy(b->table_free[k]);
    }
    kpd::handle_remove(b);
    delete b;
    if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_lbatch_close");
    return KPD_OK;
}


size_t kpd_layers_bytes(int width, int height, int n_octaves)
{
    kpd::LayerGeom g;
    std::string why;
    if (!layer_geom(width, height, n_octaves, &g, &why)) {
        kpd::api_fail(KPD_EINVAL, why);
        return 0;
    }
    return g.total;
}

int kpd_layer_plane(int width, int height, int n_octaves, int layer, size_t* offset, int* w, int* h)
{
    kpd::LayerGeom g;
    std::string why;
    if (!layer_geom(width, height, n_octaves, &g, &why)) return kpd::api_fail(KPD_EINVAL, why);
    if (layer < 1 || layer >= g.L) return kpd::api_fail(KPD_EINVAL, "layer must be 1..2 n_octaves - 1");
    if (offset) *offset = g.plane_off[layer];
    if (w) *w = g.w[layer];
    if (h) *h = g.h[layer];
    return KPD_OK;
}

int kpd_detect_layers(const uint8_t* frame, size_t pitch_bytes, int width, int height, int fast_t, int n_octaves,
                      void* workspace, size_t workspace_bytes, kpd_keypoint* out, uint32_t capacity, uint32_t* count,
                      void* hip_stream)
{
    const kpd::TraceRange trace_range("kpd:detect_layers");
    kpd::LayerGeom g;
    std::string why;
    if (!layer_geom(width, height, n_octaves, &g, &why)) return kpd::api_fail(KPD_EINVAL, why);
    if (!frame || !workspace || !count || (capacity > 0 && !out)) return kpd::api_fail(KPD_EINVAL, "NULL pointer");
    if (pitch_bytes < (size_t)width || pitch_bytes > (1u << 30)) return kpd::api_fail(KPD_EINVAL, "bad pitch");
    if (fast_t < 1 || fast_t > 254) return kpd::api_fail(KPD_EINVAL, "fast_t must be 1..254");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return kpd::api_fail(KPD_EINVAL, "workspace not 256-byte aligned");
    if (workspace_bytes < g.total)
        return kpd::api_fail(KPD_ENOMEM, "workspace has " + std::to_string(workspace_bytes) + " bytes, needs " +
                                             std::to_string(g.total));
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    uint8_t* ws = reinterpret_cast<uint8_t*>(workspace);
    kpd::LayArgs a = layer_args(g, frame, pitch_bytes, ws);
    a.t = fast_t;
    a.out = out;
    a.cap = capacity;
    a.count = count;
    // the layers: octaves by halving from the frame, d_0 from the frame,
    // the other intra-octaves by halving d_0
    hipError_t e = build_layers(g, frame, (int)pitch_bytes, ws, s);
    if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_detect_layers");
    e = kpd::launch_lay_detect(a, s);
    if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_detect_layers");
    return KPD_OK;
}

int kpd_refine_layers(int width, int height, int n_octaves, void* workspace, size_t workspace_bytes,
                      const kpd_keypoint* list, const uint32_t* count, uint32_t capacity, kpd_refined* out,
                      void* hip_stream)
{
    kpd::LayerGeom g;
    std::string why;
    if (!layer_geom(width, height, n_octaves, &g, &why)) return kpd::api_fail(KPD_EINVAL, why);
    if (!workspace || !count || (capacity > 0 && (!list || !out))) return kpd::api_fail(KPD_EINVAL, "NULL pointer");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return kpd::api_fail(KPD_EINVAL, "workspace not 256-byte aligned");
    if (workspace_bytes < g.total) return kpd::api_fail(KPD_ENOMEM, "workspace smaller than kpd_layers_bytes()");
    // the frame is not read: the fits take the score maps of the last detection
    const kpd::LayArgs a = layer_args(g, nullptr, (size_t)width, reinterpret_cast<uint8_t*>(workspace));
    const hipError_t e = kpd::launch_lay_refine(a, list, count, capacity, out, reinterpret_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_refine_layers");
    return KPD_OK;
}

}  // extern "C"
