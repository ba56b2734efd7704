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
};

// Everything one stream needs for one batch tick. tile_base and cell_base
// are the stream's first workgroups in the tick's two launches.
struct TickArgs {
    FrameArgs f;
    DetectArgs d;
    int active;     // the stream has a frame in this tick
    int f_on;       // the tile pass runs (pyramid or SAD needed)
    int tile_base, cell_base;
};

// A chunk of consecutive frames of one stream.
constexpr uint32_t kChunkPrev = 63;  // source id of the list before the chunk

struct CarryDesc {
    uint32_t src_id;   // chunk frame whose list holds the cell's entries, or kChunkPrev
    uint32_t src_off;  // their first index there
    uint32_t count;
    uint32_t dst_off;  // the cell's first index in its own frame's list
    uint32_t carried;  // 1: copy the entries (the cell was not marked)
    uint32_t pad[3];
};

struct ChunkArgs {
    DetectArgs d;                               // frame j's detection arguments
    int j, last;                                // frame index in the chunk, is it the last
    const uint32_t* prev_count;                 // counts of the frame before the chunk
    const uint32_t* prev_offs;                  // and their offsets
    unsigned long long* cnt_words;              // frame j's count words
    const unsigned long long* cnt_words_prev;   // frame j-1's
    unsigned long long* src_words;              // frame j's source words
    const unsigned long long* src_words_prev;   // frame j-1's
    CarryDesc* carry;                           // frame j's copy descriptors
};

struct CarryArgs {
    int ncell, last;
    uint32_t list_cap;
    size_t list_stride;          // entries between consecutive chunk lists
    kpd_keypoint* lists;         // chunk lists
    const kpd_keypoint* prev_list;
    const CarryDesc* carry;      // chunk frames x cells
    kpd_keypoint* next_list;     // buffers the frame after the chunk reads
    uint32_t* next_count;
    uint32_t* next_offs;
    uint32_t* next_total;
    uint32_t* sad_chunk;         // chunk frames x cells, cleared here
    uint32_t* sad_stats;         // receives the last frame's SAD
    uint32_t* sad_single_next;   // cleared for the next single frame
};

hipError_t launch_detect_chunk(const ChunkArgs* table, int n_frames, int ncell, int lds_bytes, hipStream_t s);
hipError_t launch_carry_chunk(const CarryArgs& a, int n_frames, hipStream_t s);

int frame_sad_lds_off(int tile, int O);
int frame_lds_bytes(int tile, int O, int sad_slots);
hipError_t set_detect_lds_limit(int lds_bytes);
hipError_t launch_frame(const FrameArgs& a, hipStream_t s);
hipError_t launch_detect(const DetectArgs& a, int ncell, int lds_bytes, hipStream_t s);
hipError_t launch_frame_batch(const TickArgs* table, const uint16_t* map, int nblocks, int lds_bytes, hipStream_t s);
hipError_t launch_gather_batch(const TickArgs* table, int n, kpd_keypoint* out, uint32_t out_cap, uint32_t* counts,
                               hipStream_t s);
hipError_t launch_detect_batch(const TickArgs* table, const uint16_t* map, int nblocks, int lds_bytes,
                               hipStream_t s);

}  // namespace kpd
