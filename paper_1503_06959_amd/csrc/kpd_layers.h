// Geometry, kernel arguments and launchers of detection over octaves and
// intra-octaves (internal to the library).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/kpd.h"

namespace kpd {

constexpr int kMaxLayers = 2 * KPD_MAX_OCTAVES;

// The 2O layers in scale order c_0, d_0, c_1, d_1, ...: sizes, pixel sizes
// in half level-0 pixels, where each plane lives in the workspace (layer 0
// is the caller's frame) and where each layer's pixels start in the
// flattened index space that the score, suppression and output passes
// share.
struct LayerGeom {
    int L = 0;
    int w[kMaxLayers] = {}, h[kMaxLayers] = {}, S[kMaxLayers] = {};
    size_t plane_off[kMaxLayers] = {};
    uint32_t base[kMaxLayers + 1] = {};
    uint32_t N = 0;        // pixels of all layers
    uint32_t nblocks = 0;  // blocks of the flattened passes
    size_t off_score = 0, off_flag = 0, off_bcount = 0, off_boff = 0;
    size_t total = 0;
};

constexpr int kLayBlock = 256;

// A batch of layered streams of one shape and one set of parameters:
// slot s's frame of a tick and its state.
struct LbSlot {
    const uint8_t* cur;    // the frame of this tick (device memory, read in place)
    const uint8_t* prev;   // the slot's previous frame (read when not forced)
    int cur_pitch, prev_pitch;
    int active;            // a frame is staged for this tick
    int force;             // every cell is marked (first frame, reset)
    int fb;                // the list buffer D_n goes to (D_{n-1} is in the other)
};

struct LayArgs {
    const uint8_t* plane[kMaxLayers];
    int pitch[kMaxLayers];
    int w[kMaxLayers], h[kMaxLayers], S[kMaxLayers];
    uint32_t base[kMaxLayers + 1];
    int L, t;
    uint32_t N;
    uint16_t* score;
    uint8_t* flag;
    uint32_t* bcount;
    uint32_t* boff;
    uint32_t nblocks;
    kpd_keypoint* out;
    uint32_t cap;
    uint32_t* count;
    // the masked stream: pixels whose cell (of the level-0 footprint start)
    // has need_score[c] == 0 are not scored, those with need_flag[c] == 0
    // not suppressed; NULL for full-frame detection
    const uint8_t* need_score;
    const uint8_t* need_flag;
    uint32_t* cell_new;   // keypoints found per cell (the masked stream; NULL otherwise)
    int nc, nr, W, H;
    // chunks: frame j's level 0 lies frame_step bytes past plane[0], its
    // other planes and its score, flag and block-count maps ws_step bytes
    // past frame 0's, its need and count arrays cells_step entries past
    size_t frame_step, ws_step;
    int cells_step;
    // a batch of layered streams: frame j is slot j's, from this table
    // (inactive slots are skipped); null otherwise
    const LbSlot* slots;
};

// The masked stream over these layers: per-cell mask, Eq. 1 with cells
// taken from the layers' footprints, D_n in (cell, layer, y, x) order.
// xs[l * (nc + 1) + c] is the first pixel column of layer l whose footprint
// start lies in cell column c or later (xs[.. + nc] = the layer's width);
// ys likewise for rows.
struct LsArgs {
    const uint8_t* cur;
    const uint8_t* prev;
    int cur_pitch, prev_pitch;
    int nc, nr, ncell;
    int force;
    int32_t id_thresh;
    uint32_t kb_thresh;
    const uint32_t* xs;
    const uint32_t* ys;
    uint8_t* mask;
    const uint32_t* cnt_prev;
    const uint32_t* off_prev;
    const kpd_keypoint* list_prev;
    uint32_t* cnt_cur;
    uint32_t* off_cur;
    kpd_keypoint* list_cur;
    uint32_t* total_cur;
    uint32_t cap;
    uint8_t* need_score;   // cells within (rx, ry) cells of a marked one
    uint32_t* cell_new;    // keypoints the suppression keeps per marked cell
    int rx, ry;
};

hipError_t launch_ls_mask(const LsArgs& a, hipStream_t s);
hipError_t launch_ls_emit(const LsArgs& a, const LayArgs& l, hipStream_t s);

// A chunk of the masked stream over these layers (T_H off): frame j at
// frames + j * stride (the frame before the chunk: prev0), its per-cell
// mask, scored-cell flags and suppression counts at j * ncell, mark words
// (cells x Kw, bit j = frame j) for the chunk compaction, and the marked
// cells' keypoints at fixed per-cell bases of frame j's sparse list.
struct LsChunkArgs {
    const uint8_t* frames;
    size_t stride;
    int pitch;
    const uint8_t* prev0;
    int prev0_pitch;
    int n_frames, force0, all_marked;
    int nc, nr, ncell, Kw;
    int32_t id_thresh;
    const uint32_t* xs;
    const uint32_t* ys;
    uint8_t* mask;               // frames x cells
    uint8_t* need;               // frames x cells
    uint32_t* cell_new;          // frames x cells
    unsigned long long* marks;   // cells x Kw
    uint8_t* last_mask;          // the last frame's mask, the stream's reported M_n
    kpd_keypoint* sparse;        // frame j's at sparse + j * list_stride
    const uint32_t* cbase;       // cell c's first entry in a sparse list
    size_t list_stride;
    uint32_t cap;
    int rx, ry;
};

hipError_t launch_ls_mask_chunk(const LsChunkArgs& a, hipStream_t s);
hipError_t launch_ls_write_chunk(const LsChunkArgs& a, const LayArgs& l, hipStream_t s);

// A tick of a batch of layered streams: per slot the mask, scored cells,
// suppression counts and the D lists of the masked stream (two buffers per
// slot, D_n in slots[s].fb), slots x cells arrays and list_stride entries
// between slots' lists.
struct LbArgs {
    const LbSlot* slots;
    int nslots, nc, nr, ncell;
    int32_t id_thresh;
    uint32_t kb_thresh;
    const uint32_t* xs;
    const uint32_t* ys;
    uint8_t* mask;
    uint8_t* need;
    uint32_t* cell_new;
    uint32_t* cnt[2];
    uint32_t* off[2];
    kpd_keypoint* list[2];
    uint32_t* total[2];   // one per slot
    size_t list_stride;
    uint32_t cap;
    int rx, ry;
};

hipError_t launch_lb_mask(const LbArgs& a, hipStream_t s);
hipError_t launch_lb_emit(const LbArgs& a, const LayArgs& l, hipStream_t s);

// Two halvings of a chain (src -> d1 -> d2; d2 absent when w2 = 0), and the
// 1.5x downsampling of the frame with the halving after it (d1 absent when
// w1 = 0). `frames` consecutive frames of a chunk: sources sstep bytes
// apart, destinations dstep bytes apart.
// With a slot table, frame z is slot z's (inactive slots skipped) and a
// step that reads the frame (from_frame) takes it from the table.
hipError_t launch_lay_quad(const uint8_t* src, int spitch, uint8_t* d1, int w1, int h1, uint8_t* d2, int w2, int h2,
                           hipStream_t s, int frames = 1, size_t sstep = 0, size_t dstep = 0,
                           const LbSlot* slots = nullptr, int from_frame = 0);
hipError_t launch_lay_third(const uint8_t* src, int spitch, uint8_t* d0, int w0, int h0, uint8_t* d1, int w1, int h1,
                            hipStream_t s, int frames = 1, size_t sstep = 0, size_t dstep = 0,
                            const LbSlot* slots = nullptr);
hipError_t launch_lay_detect(const LayArgs& a, hipStream_t s);
hipError_t launch_lay_score_nms(const LayArgs& a, hipStream_t s, int frames = 1);
hipError_t launch_lay_refine(const LayArgs& a, const kpd_keypoint* list, const uint32_t* count, uint32_t cap,
                             kpd_refined* out, hipStream_t s);

}  // namespace kpd
