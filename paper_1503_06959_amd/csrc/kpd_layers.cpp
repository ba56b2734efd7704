// C ABI of detection over octaves and intra-octaves: workspace layout and
// the launch sequence. The contracts are in include/kpd.h.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdint>
#include <string>

#include "../../include/kpd.h"
#include "kpd_errors.h"
#include "kpd_layers.h"

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

}  // namespace

extern "C" {

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
    auto plane = [&](int l) { return ws + g.plane_off[l]; };
    for (int i = 1; i < n_octaves; ++i) {
        const int l = 2 * i, src = 2 * i - 2;
        hipError_t e = kpd::launch_lay_half(a.plane[src], a.pitch[src], plane(l), g.w[l], g.h[l], s);
        if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_detect_layers");
    }
    hipError_t e = kpd::launch_lay_twothirds(frame, (int)pitch_bytes, plane(1), g.w[1], g.h[1], s);
    if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_detect_layers");
    for (int i = 1; i < n_octaves; ++i) {
        const int l = 2 * i + 1, src = 2 * i - 1;
        e = kpd::launch_lay_half(plane(src), g.w[src], plane(l), g.w[l], g.h[l], s);
        if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_detect_layers");
    }
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
