// Kernel argument blocks and launchers (internal to the library).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "../../include/kpd.h"

namespace kpd {

struct MaskArgs {
    const uint8_t* cur;   // I_n, level 0
    const uint8_t* prev;  // I_{n-1}, level 0
    int cur_pitch, prev_pitch;
    int W, H, nc, nr;
    int id_on;            // T_I < 255: the intensity test can fire
    int32_t id_thresh;
    uint32_t kb_thresh;
    const uint32_t* count;  // per-cell counts of D_{n-1}
    uint32_t* sad;
    uint8_t* mask;
};

struct PyrArgs {
    const uint8_t* lvl0;
    int pitch0;
    uint8_t* lvl[KPD_MAX_OCTAVES];
    int pitch[KPD_MAX_OCTAVES];
    int w[KPD_MAX_OCTAVES], h[KPD_MAX_OCTAVES];
    int W, H, O;
    int tile;  // level-0 tile side (power of two, >= 2^(O-1), >= 64)
};

struct DetectArgs {
    const uint8_t* lvl[KPD_MAX_OCTAVES];
    int pitch[KPD_MAX_OCTAVES];
    int w[KPD_MAX_OCTAVES], h[KPD_MAX_OCTAVES];
    int W, H, O, nc, nr;
    int t;
    int all_marked;
    uint8_t* mask;
    uint32_t* count;
    uint32_t* offsets;
    const uint32_t* store_base;  // ncell + 1 entries
    kpd_keypoint* store;
    uint32_t* hdr;  // [0] total keypoints of D_n, [1] workgroup ticket
};

struct GatherArgs {
    const uint32_t* count;
    const uint32_t* offsets;
    const uint32_t* store_base;
    const kpd_keypoint* store;
    kpd_keypoint* out;
};

hipError_t launch_cell_mask(const MaskArgs& a, int ncell, hipStream_t s);
hipError_t launch_pyramid(const PyrArgs& a, hipStream_t s);
hipError_t launch_detect(const DetectArgs& a, int ncell, int lds_bytes, hipStream_t s);
hipError_t launch_gather(const GatherArgs& a, int ncell, hipStream_t s);
int detect_lds_bytes(int lds_bytes);

}  // namespace kpd
