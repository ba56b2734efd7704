// Kernel arguments and launchers of the temporally coherent detector
// (internal to the library).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "../../include/kpd.h"

namespace kpd {

// D_n of the group's first frame (the inner stream's list) into tracks.
struct TcdSeedArgs {
    const kpd_keypoint* list;
    const uint32_t* count;
    kpd_track* out;
    uint32_t* out_count;
    uint32_t cap;
};

// One propagation step: every track of `in` searched in `cur` against its
// patch in `prev`; the result goes to moved[k] with keep[k] = 1 when kept.
struct TcdTrackArgs {
    const uint8_t* prev;
    const uint8_t* cur;
    int prev_pitch, cur_pitch;
    int W, H;
    int t_bm, t_et;
    const kpd_track* in;
    const uint32_t* in_count;
    kpd_track* moved;
    uint32_t* keep;
    uint32_t cap;
};

// The kept tracks, in order, into `out`.
struct TcdCompactArgs {
    const kpd_track* moved;
    const uint32_t* keep;
    const uint32_t* in_count;
    kpd_track* out;
    uint32_t* out_count;
    uint32_t cap;
};

hipError_t launch_tcd_seed(const TcdSeedArgs& a, hipStream_t s);
hipError_t launch_tcd_track(const TcdTrackArgs& a, hipStream_t s);
hipError_t launch_tcd_compact(const TcdCompactArgs& a, hipStream_t s);

}  // namespace kpd
