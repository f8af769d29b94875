// Batched uneven propagation jobs: parameters shared by the host layer
// and the persistent kernel.
#pragma once

#include "kete_fov.hpp"
#include "kete_internal.hpp"

// lanes per body of the persistent kernel (7: 9 bodies per wavefront,
// 8: 8 bodies) and bodies per tile, one wavefront each
#define KETE_BATCH_LANES 7
#define KETE_BATCH_TILE (KETE_BATCH_LANES == 7 ? 9 : 8)

namespace kete {

struct BatchParams {
    EphemArgs eph;
    RadauConst rc;
    const kete_job_t* jobs;     // [n_jobs]
    int32_t n_jobs;
    int32_t n_tiles;
    const int2* tiles;          // [n_tiles] (job, tile of KETE_BATCH_TILE bodies), longest first
    unsigned int* tile_counter;
    const double* x0;           // [bodies][6]
    const double* epochs;       // concatenated epochs of all jobs
    double* x_out;              // per-job blocks [n_epoch][n_obj][6]
    int32_t* status;            // [bodies]
    int32_t* perm;              // [bodies] job-local order of each job's bodies
    int32_t n_buckets;
    int32_t max_win_segs;
    int32_t max_iter;
    int32_t max_steps;
    int32_t zero_start;         // corrector starts from zero increments (no extrapolation)
    int32_t land_epochs;        // land on every epoch (else epochs inside a step come off its polynomial)
    double* dense_coef;         // [kDenseCoefDoubles] Ap, Bp of rc, written by the launch
    double eps, h_min, h_max, h_init, safety;
};

size_t batch_lds_bytes(const BatchParams& p);
hipError_t launch_batch(const BatchParams& p, int waves_per_cu, hipStream_t s);

}  // namespace kete
