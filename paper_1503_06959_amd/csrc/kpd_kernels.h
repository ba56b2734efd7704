// Kernel argument blocks and launchers (internal to the library).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "../../include/kpd.h"
#include "kpd_geom.h"

namespace kpd {

// k_frame: pyramid of I_n and, optionally, per-cell SAD against I_{n-1}.
struct FrameArgs {
    const uint8_t* cur;   // I_n, level 0
    const uint8_t* prev;  // I_{n-1}, level 0 (read when sad_on)
    int cur_pitch, prev_pitch;
    int cur_aligned, prev_aligned;  // base and pitch 4-byte aligned
    uint8_t* lvl[KPD_MAX_OCTAVES];  // levels 1..O-1
    int pitch[KPD_MAX_OCTAVES];
    int w[KPD_MAX_OCTAVES], h[KPD_MAX_OCTAVES];
    int W, H, O, nc, nr;
    int tile;        // level-0 tile side: power of two, >= 2^(O-1), >= 32
    int tiles_x;     // tiles per row
    int ntiles;      // tiles in the frame
    int sad_on;
    int sad_slots;   // LDS per-cell partial slots (cells a tile can touch)
    int sad_lds_off;
    uint32_t* sad;   // per-cell SAD, accumulated; zero on entry
    const uint16_t* colmap;   // cell column of every level-0 column (W entries)
    const uint16_t* rowmap;   // cell row of every level-0 row (H entries)
};

// The frame-dependent inputs of one tile pass: the frames, and where this
// frame's octaves (FrameArgs::lvl + lvl_off) and SAD accumulators go.
struct FrameSrc {
    const uint8_t* cur;
    const uint8_t* prev;
    int cur_pitch, prev_pitch;
    int cur_aligned, prev_aligned;
    int sad_on;
    size_t lvl_off;
    uint32_t* sad;
};

// Descriptor pattern tables, built on the host at open: the 60 points turned
// to each of the 32 sectors (rounded offsets in level pixels), their box
// half-sizes, the long pairs with the unturned offset difference p_b - p_a,
// the 512 short pairs in bit order, and the sector boundary vectors.
constexpr int kDescPts = 60, kDescSectors = 32, kDescBits = 512, kDescLongMax = kDescPts * (kDescPts - 1) / 2;
struct DescTables {
    int8_t pt[kDescSectors][kDescPts][2];
    uint8_t half[kDescPts];
    int32_t nlong;
    uint8_t lp[kDescLongMax][2];
    int8_t ld[kDescLongMax][2];
    uint8_t sp[kDescBits][2];
    int64_t ux[kDescSectors], uy[kDescSectors];
};

// k_describe: descriptors and refined values of D_n's features, computed for
// the cells marked this frame and carried with the keypoints of the others.
// A null tab (desc_*) or ref_cur leaves that part out.
struct DescArgs {
    const DescTables* tab;
    const uint8_t* lvl[KPD_MAX_OCTAVES];
    int pitch[KPD_MAX_OCTAVES];
    int w[KPD_MAX_OCTAVES], h[KPD_MAX_OCTAVES];
    int O, t;
    const kpd_refined* ref_prev;
    kpd_refined* ref_cur;
    const uint8_t* mask;
    const uint32_t* count_cur;
    const uint32_t* off_cur;
    const uint32_t* off_prev;
    const kpd_keypoint* list_cur;
    const kpd_descriptor* desc_prev;
    kpd_descriptor* desc_cur;
    uint32_t list_cap;
    // per-pixel masks: the entries' sources (DetectArgs::src_cur), null otherwise
    const uint32_t* src_cur;
};

// k_detect: per-cell mark, detection, look-back offsets and output.
struct DetectArgs {
    const uint8_t* lvl[KPD_MAX_OCTAVES];
    int pitch[KPD_MAX_OCTAVES];
    int w[KPD_MAX_OCTAVES], h[KPD_MAX_OCTAVES];
    int lvl0_aligned;
    int W, H, O, nc, nr;
    int t;
    int all_marked;
    int id_on;
    int32_t id_thresh;
    uint32_t kb_thresh;
    const uint32_t* sad;     // this frame's per-cell SAD
    uint32_t* sad_next;      // zeroed here for the next frame
    uint8_t* mask;
    const uint32_t* count_prev;
    const uint32_t* off_prev;
    const kpd_keypoint* list_prev;
    uint32_t* count_cur;
    uint32_t* off_cur;
    kpd_keypoint* list_cur;
    uint32_t* total_cur;
    uint32_t list_cap;           // entries of each keypoint list
    const CellLayout* layouts;   // per-cell detection layout, computed at open
    const uint16_t* col_w;       // cell column widths (level-0 pixels)
    const uint16_t* row_h;       // cell row heights
    unsigned long long* status;  // per-cell count words of marked cells
    uint32_t epoch;              // frame number + 1
    uint32_t* err;               // set when a wait for an earlier cell gives up
    // per-pixel masks (single frames): id_mode 1 builds one mask on layer
    // id_layer, id_mode 2 one per octave on its own level. lprev holds
    // I_{n-1}'s levels that the masks read (I_n's are lvl); the lds_ fields
    // say where the per-cell scratch lives in LDS (changed-pixel bits,
    // carried-entry bits, their word offsets, scores and, with features,
    // sources), past every cell's detection layout
    int id_mode, id_layer;
    const uint8_t* lprev[KPD_MAX_OCTAVES];
    int lprev_pitch[KPD_MAX_OCTAVES];
    int lds_bits, lds_carr, lds_cwoff, lds_cscore, lds_csrc;
    // with features and a per-pixel mask: for every D_n entry of a marked
    // cell, its index in D_{n-1}'s list when carried, else kNewFeature
    uint32_t* src_cur;
};

constexpr uint32_t kNewFeature = 0xFFFFFFFFu;

// Everything one stream needs for one batch tick. tile_base and cell_base
// are the stream's first workgroups in the tick's two launches.
struct TickArgs {
    FrameArgs f;
    DetectArgs d;
    int active;     // the stream has a frame in this tick
    int f_on;       // the tile pass runs (pyramid or SAD needed)
    int tile_base, cell_base;
    // marked cells' keypoints at fixed per-cell bases of a sparse list, and
    // their counts; the tick's compaction pass builds D_n from them
    kpd_keypoint* sparse;
    const uint32_t* sparse_base;
    uint32_t* own_count;
    // the stream's one-cell layouts of the group detector, and whether its
    // level 0 can be read 8 bytes at a time (the single-launch tick)
    const GroupLayout* glay1;
    int al8;
    // features of D_n (null when the stream computes none): as DescArgs's,
    // with the levels, mask, lists, counts and offsets of d
    const DescTables* tab;
    const kpd_descriptor* desc_prev;
    kpd_descriptor* desc_cur;
    const kpd_refined* ref_prev;
    kpd_refined* ref_cur;
};

// Counters of the single-launch tick: arrivals at its two device-wide
// barriers, one set per tick parity (a tick clears the other parity's set,
// which the next tick uses).
struct TickSync {
    uint32_t arrive[2][2];
};

// A chunk of consecutive frames of one stream, in two passes after the
// tile pass. The detection pass writes each marked cell's keypoints at the
// cell's fixed base in its frame's sparse list (no cross-cell offsets, so no
// waits between cells) and records the mark. The compaction pass (one
// workgroup per frame) finds for every cell the last chunk frame up to its
// own where the cell was marked, or the list before the chunk, and copies
// the entries into the frame's list in cell order (Eq. 1).
struct ChunkArgs {
    DetectArgs d;                               // frame j's fixed detection arguments (list_cur = sparse list j)
    int j;                                      // frame index in the chunk
    int Kw;                                     // mark words per cell
    const uint32_t* cell_base;                  // each cell's first index in a sparse list
    unsigned long long* marks;                  // cells x Kw mark words: bit j of a cell = frame j marked
    uint32_t* own_count;                        // frame j's per-cell counts of detected cells
};

// What changes from one chunk to the next, passed by value: the frames, the
// frame before the chunk, thresholds and the buffers that alternate.
struct ChunkHead {
    const uint8_t* frames;      // frame j at frames + j * stride
    const uint8_t* prev0;       // the frame before the chunk
    size_t stride;
    int pitch, prev0_pitch;
    int aligned, prev0_aligned; // rows dword-readable
    int n_frames;
    int force0;                 // frame 0 marks every cell (first frame, reset, new t)
    int all_marked;             // the parameters mark every cell
    int t;
    int32_t id_thresh;
    uint32_t kb_thresh;
    int kb_chain;               // marks depend on the previous frame's counts (T_H active)
    const uint32_t* prev_count; // counts of the frame before the chunk
    int ntiles, ncell;          // tiles and cells per frame
    int nc;                     // cell columns
    // marks decided before detection (no T_H chain): the mark pass lists
    // the marked (frame, cell) items and the detection pass runs only those
    const uint32_t* sad0;       // frame j's SAD at sad0 + j * ncell
    const uint16_t* col_w;
    const uint16_t* row_h;
    unsigned long long* marks;  // cells x Kw mark words (bit j = frame j)
    uint8_t* mask;              // M of the last frame
    int Kw;
    uint32_t* work;             // marked items j * ncell + c
    uint32_t* work_count;       // their number (two: a second round of items follows the first);
                                // cleared by the compaction pass
};

struct CompactArgs {
    int ncell, last, Kw;
    uint32_t list_cap;
    size_t list_stride;              // entries between consecutive chunk lists
    const kpd_keypoint* sparse;      // chunk frames' sparse lists
    const uint32_t* cell_base;
    const unsigned long long* marks; // cells x Kw mark words
    const uint32_t* own_count;       // chunk frames x cells
    const kpd_keypoint* prev_list;   // D before the chunk, its counts and offsets
    const uint32_t* prev_count;
    const uint32_t* prev_offs;
    kpd_keypoint* lists;             // chunk frames' lists (all but the last)
    uint32_t* counts;                // chunk frames x cells
    uint32_t* offs;
    uint32_t* totals;                // one per chunk frame
    kpd_keypoint* next_list;         // the last frame's D, where the next push reads it
    uint32_t* next_count;
    uint32_t* next_offs;
    uint32_t* next_total;
    uint32_t* sad_chunk;             // chunk frames x cells, cleared here
    uint32_t* sad_stats;             // receives the last frame's SAD
    uint32_t* sad_single_next;       // cleared for the next single frame
    uint32_t* work_count;            // both words cleared for the next chunk
};

// k_describe_chunk: features of a chunk's lists after compaction (the
// lists, counts and offsets CompactArgs names). A null tab (descs,
// last_desc) or refs (last_ref) leaves that part out.
struct DescChunkArgs {
    const ChunkArgs* table;            // frame j's octaves 1.. and level sizes
    const uint8_t* frames;             // level 0 of frame j at frames + j * stride
    size_t stride;
    int pitch;
    int n_frames, ncell, Kw, O, t;
    const unsigned long long* marks;   // cells x Kw mark words (bit j = frame j)
    const DescTables* tab;
    uint32_t list_cap;
    size_t list_stride;                // entries between consecutive chunk lists
    const kpd_keypoint* lists;         // frames 0..n_frames-2: lists, counts and offsets
    const uint32_t* counts;            // (chunk frames x cells)
    const uint32_t* offs;
    kpd_descriptor* descs;             // their features, list_stride entries apart
    kpd_refined* refs;
    const kpd_keypoint* last_list;     // the last frame's D_n
    const uint32_t* last_count;
    const uint32_t* last_offs;
    kpd_descriptor* last_desc;
    kpd_refined* last_ref;
    const kpd_descriptor* prev_desc;   // features of the list before the chunk
    const kpd_refined* prev_ref;
    const uint32_t* prev_offs;
};

// Per-pixel masks in chunks (Sec. 3.1, Eq. 2 per pixel): mode 1 reads one
// layer for every octave, mode 2 each octave on its own level. The diff
// pass records, per (frame j, cell c), the changed pixels of the layers the
// cell's level-0 pixels map to and whether any changed; the mark pass lists
// the (frame, cell) items with a change; the listed detection writes F_j of
// those cells; the merge pass walks each cell's listed frames in order and
// applies Eq. 1 per feature, writing the cell's D_j at its per-pixel base.
struct PixelChunkArgs {
    const ChunkArgs* table;                     // frame j: octaves 1.., level sizes, F list and counts
    const uint8_t* frames;                      // level 0 of frame j at frames + j * stride
    size_t stride;
    int pitch;
    const uint8_t* prev_lvl[KPD_MAX_OCTAVES];   // the frame before the chunk (level 0: the frame itself)
    int prev_pitch[KPD_MAX_OCTAVES];
    int n_frames, ncell, nc, nr, W, H, O, Kw;
    int l_lo, l_hi;                             // layers that hold mask pixels
    int one;                                    // 1: layer l_lo masks every octave; 0: octave o on level o
    int id_thresh;
    int force0;                                 // frame 0 detects everything and carries nothing
    uint32_t* flags;                            // frames x cells: a mask pixel of the cell changed
    unsigned long long* fp;                     // frames x cells x fpw: changed bits of the cell's layer pixels
    int fpw;
    const unsigned long long* marks;            // cells x Kw mark words (bit j = frame j)
    const CellLayout* layouts;
    const uint32_t* cell_base;                  // F lists' bases
    uint32_t list_cap;                          // F lists' entries
    const kpd_keypoint* sparse;                 // frame j's F list at sparse + j * list_stride
    const uint32_t* own;                        // F counts, frames x cells
    const uint32_t* pbase;                      // merged lists' bases (decision pixels of the earlier cells)
    kpd_keypoint* merged;                       // frame j's at merged + j * list_stride
    uint32_t* mcount;                           // frames x cells
    size_t list_stride;
    uint32_t plist_cap;                         // merged lists' entries
    const kpd_keypoint* prev_list;              // D before the chunk, its counts and offsets
    const uint32_t* prev_count;
    const uint32_t* prev_offs;
    uint32_t prev_cap;
    // the merge pass's dynamic LDS: map bits, scores, the staged change
    // words of `batch` frames, up to ents_cap staged maxima and, with tab_on,
    // per decision pixel its mask bit (u16), level position (x | y << 16)
    // and octave (u8)
    int lds_pres, lds_score, lds_fp, lds_ents, lds_tgate, lds_txy, lds_toct, lds_bytes;
    int batch, tab_on;
    uint32_t ents_cap;
    // features (msrc non-null): the merge keeps each map entry's source in
    // LDS (lds_tsrc) and writes it beside the entry: kPixelFromPrev | index
    // in the list before the chunk, or (frame << kPixelFrameShift) | index in
    // that frame's F list. Features of every listed (frame, cell)'s maxima
    // go to sdesc / sref at their F list places (list_cap apart by frame);
    // after the compaction each frame's list gathers its records from there
    // or from the list before the chunk.
    int lds_tsrc;
    uint32_t* msrc;                 // frame j's at msrc + j * list_stride
    const DescTables* tab;          // null: no descriptors
    kpd_descriptor* sdesc;
    kpd_refined* sref;
    int t;
    const uint32_t* counts;         // the compaction's lists, frames 0..n-2, and the last frame's
    const uint32_t* offs;
    kpd_descriptor* cdesc;          // their features, list_stride entries apart
    kpd_refined* cref;
    const uint32_t* last_count;
    const uint32_t* last_offs;
    kpd_descriptor* last_desc;
    kpd_refined* last_ref;
    const kpd_descriptor* prev_desc; // features of the list before the chunk
    const kpd_refined* prev_ref;
    uint32_t dlist_cap;             // entries of the compaction's lists
};

constexpr uint32_t kPixelFromPrev = 0x80000000u;
constexpr int kPixelFrameShift = 22;   // F list indices below 2^22

hipError_t launch_pixel_diff_chunk(const PixelChunkArgs& a, hipStream_t s);
hipError_t launch_pixel_merge_chunk(const PixelChunkArgs& a, hipStream_t s);
hipError_t launch_pixel_features_chunk(const PixelChunkArgs& a, hipStream_t s);
hipError_t launch_pixel_gather_chunk(const PixelChunkArgs& a, hipStream_t s);

// The group detector: the groups' layouts (a rectangle of cells each,
// row-major over the group grid; each layout names its cells and their
// list bases) and whether level 0's rows can be read 8 bytes at a time.
struct GroupArgs {
    const GroupLayout* layouts;
    int ngroups, nc;
    int al8;
};

hipError_t launch_detect_list_groups(const ChunkArgs* table, const ChunkHead& h, const GroupArgs& g, int lds_bytes,
                                     int threads, int round, hipStream_t s);
hipError_t launch_detect_list_batch_groups(const TickArgs* table, const uint16_t* map, int ncells,
                                           const uint32_t* work, const uint32_t* work_count, int lds_bytes,
                                           hipStream_t s);
hipError_t launch_detect_chunk_groups(const ChunkArgs* table, const ChunkHead& h, const GroupArgs& g, int lds_bytes,
                                      int threads, hipStream_t s);
hipError_t set_group_lds_limit(int lds_bytes);
// largest static LDS of the group kernels, which their dynamic LDS sits beside
hipError_t group_static_lds(int* bytes);
// one frame with the per-cell mask: marks and detection of the marked cells
// with one-cell layouts (sparse list), then D_n by k_compact1
hipError_t launch_det1_groups(const DetectArgs& a, const GroupArgs& g, kpd_keypoint* sparse, uint32_t* own,
                              int ncell, int lds_bytes, int threads, hipStream_t s);
// Copy a stream's header words (4), the first min(its D_n size, pre)
// entries of D_n and, when mask is not null, the cell mask into pinned host
// memory: words at stage, entries from stage + 64, the mask after kStage
// entries. total_word: the header word that holds D_n's size.
hipError_t launch_publish(const uint32_t* hdr, int total_word, const kpd_keypoint* list, uint32_t pre,
                          const uint8_t* mask, int ncell, uint32_t stage_entries, uint8_t* stage, hipStream_t s);
hipError_t launch_compact1(const DetectArgs& a, const kpd_keypoint* sparse, const uint32_t* cbase,
                           const uint32_t* own, hipStream_t s);

// The sequential tile pass of chunks with intensity differences (tiles of
// 256 x 64 for O <= 5, or 128 x 128 for O <= 6): `run` frames per
// workgroup, each read once; tiles_x and ntiles count its tiles, slots the
// cells one tile can touch.
struct SeqGrid {
    int tile_w, tiles_x, ntiles, slots, run;
};
int frame_seq_lds_bytes(int slots, int run);
// Workgroups of the sequential tile pass the device holds at once.
hipError_t frame_seq_capacity(int lds_bytes, int* blocks);
// nt: read the frames non-temporally (chunks larger than the last level cache).
hipError_t launch_frame_chunk_seq(const FrameArgs& a, size_t pyr_stride, const ChunkHead& h, const SeqGrid& g,
                                  bool nt, hipStream_t s);
hipError_t launch_frame_chunk(const FrameArgs& a, size_t pyr_stride, const ChunkHead& h, int lds_bytes, hipStream_t s);
hipError_t launch_mark_chunk(const ChunkHead& h, hipStream_t s);
hipError_t launch_spec_chunk(const ChunkHead& h, hipStream_t s);
hipError_t launch_spec2_chunk(const ChunkHead& h, const uint32_t* own, hipStream_t s);
hipError_t launch_resolve_chunk(const ChunkHead& h, const uint32_t* own, hipStream_t s);
hipError_t launch_compact_chunk(const CompactArgs& a, int n_frames, hipStream_t s);

int frame_sad_lds_off(int tile, int O);
int frame_lds_bytes(int tile, int O, int sad_slots);
hipError_t set_detect_lds_limit(int lds_bytes);
hipError_t launch_frame(const FrameArgs& a, hipStream_t s);
hipError_t launch_detect(const DetectArgs& a, int ncell, int lds_bytes, hipStream_t s);
hipError_t launch_describe(const DescArgs& a, int ncell, hipStream_t s);
hipError_t launch_describe_chunk(const DescChunkArgs& a, hipStream_t s);
hipError_t launch_describe_batch(const TickArgs* table, const uint16_t* map, int ncells, hipStream_t s);
hipError_t launch_detect_pixel_batch(const TickArgs* table, const uint16_t* map, int ncells, int lds_bytes,
                                     hipStream_t s);
hipError_t launch_frame_batch(const TickArgs* table, const uint16_t* map, int nblocks, int lds_bytes, hipStream_t s);
hipError_t launch_gather_batch(const TickArgs* table, int n, kpd_keypoint* out, uint32_t out_cap, uint32_t* counts,
                               hipStream_t s);
hipError_t launch_mark_batch(const TickArgs* table, const uint16_t* map, int ncells, uint32_t* work,
                             uint32_t* work_count, hipStream_t s);
hipError_t launch_compact_batch(const TickArgs* table, int n, uint32_t* work_count, hipStream_t s);
// One batch tick in one launch of `grid` co-resident workgroups (phases
// separated by device-wide barriers); `parity` selects the counter set.
hipError_t launch_tick(const TickArgs* table, const uint16_t* fmap, int nframe, const uint16_t* cmap, int ncells,
                       int nstreams, TickSync* sync, int parity, int grid, int lds_bytes, hipStream_t s);
// Workgroups of the single-launch tick that fit on the device at once.
hipError_t tick_capacity(int lds_bytes, int* blocks);

}  // namespace kpd
