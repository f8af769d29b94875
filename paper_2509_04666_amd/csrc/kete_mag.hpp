// H-G magnitudes of the pairs: parameters shared by the host layer and
// the kernels.
#pragma once

#include <algorithm>

#include "kete_internal.hpp"

namespace kete {

struct MagParams {
    EphemArgs eph;
    const double* x_epoch;      // [B][N][6]
    int32_t n_obj;
    int32_t n_batch;
    int64_t n_frames;
    const double* t_ref;        // [B]
    const int32_t* batch_off;   // [B+1]
    const int32_t* frame_order; // [F]
    const double* ft;           // [F]
    const double* fobs;         // [F][3]
    const int32_t* pf;          // [n_pairs]
    const int32_t* po;          // [n_pairs]
    int64_t n_pairs;
    const double* h_mag;        // [N]
    const double* g_slope;      // [N]
    double* v_mag;              // [n_pairs]
    double* geom;               // [n_pairs][3] or null
    double smu, c_light, lt_tol;
    int32_t lt_iter;
    int32_t kepler_iter;
    double t_lo, t_hi;          // ephemeris span
};

// Doubles of a frame's record (the quantities every pair of the frame uses).
constexpr int kMagRec = 24;
// Workspace: the frame-to-batch map, then the frame records.
size_t mag_workspace_bytes(int64_t n_frames);

// Frames covered by the static frame-to-batch map (4 bytes per frame).
constexpr int64_t kMagScratchFrames = KETE_MAG_NOALLOC_MAX_FRAMES;
// Device address of that map on the current device, looked up on the
// first call per device and kept.
hipError_t mag_static_scratch(void** ptr);
// ws: the map, and the frame records after it when frame_records (the
// static map of the entry point that allocates nothing has no room for
// them: its pairs compute their frame's quantities themselves).
hipError_t launch_pair_mag(const MagParams& p, void* ws, bool frame_records, hipStream_t s);

}  // namespace kete
