// Adjoint (sky-residual gradient) stage: parameters shared by the host
// layer and kernels.
#pragma once

#include "kete_internal.hpp"

namespace kete {

// x[3], v[3], wave step, failed flag, force F0[3], F0 valid, the last accepted step's increments
// at nodes 1..7 [7][3], that step (0: none), the checkpoint's time, 1 spare
constexpr int kCkptDoubles = 36;
constexpr int kAdjStateDoubles = 8; // lx[3], lv[3], next observation, overflow flag
constexpr int kAdjLanes = 8;         // lanes per object in the adjoint kernels (8 objects per wavefront)
constexpr int kAdjTabDoubles = 8 * (16 + 18);   // constant rows of the reverse sweep
constexpr int kStepDoubles = 2;      // per stored step and object: start time, step size
constexpr int kJacDoubles = 18;      // per stored step, node and object: Jx (9), Jv (9)
constexpr int kStepRecDoubles = kStepDoubles + 8 * kJacDoubles;   // step store per step and object

struct AdjParams {
    EphemArgs eph;
    RadauConst rc;
    const double* x0;           // [N][6]
    const int32_t* perm;        // [N] object order (bucketed)
    double t0;
    int32_t n_obj;
    int32_t k_obs;
    const double* t_obs;        // [N][K], ascending per object, in [t0, t_end]
    const double* obs_pos;      // [N][K][3]
    const double* dL_dsky;      // [N][K][2] (backward)
    double* sky_out;            // [N][K][2] (forward)
    double* grad;               // [N][6] (backward)
    int32_t* status;            // [N]
    double* h_pref;             // [N]
    double* ckpt;               // [C+1][N][kCkptDoubles]
    double t_end;
    double ckpt_days;           // checkpoint c: the first step start at or after t0 + c ckpt_days
    int32_t n_ckpt;             // C segments
    int32_t pad_;
    double* obs_state;          // [N][K][6] states at the observation times (forward)
    double* obs_grad;           // [N][K][6] dL/d(state) at the observation times (backward)
    double* obs_hop;            // [N][K][2] light time and final universal anomaly (forward)
    double* steps;              // [s_max][kStepDoubles][N] (store 0; store 1 follows the Jacobians)
    double* jac;                // [s_max][kJacDoubles][N][8 nodes]: one object's nodes side by side
    double* adj_state;          // [N][kAdjStateDoubles] carried between backward segments
    int32_t* seg_ns;            // [2][ceil(N / 8)] steps stored per wavefront, per step store
    double* adj_tab;            // [kAdjTabDoubles] constant rows of the reverse sweep
    double* dense_coef;         // [kDenseCoefDoubles] Ap, Bp of rc (written by the forward launch)
    int32_t s_max;
    int32_t max_win_segs;
    int32_t max_iter;
    int32_t max_steps;
    double eps, h_min, h_max, h_init, safety;
    double smu, c_light, lt_tol, cos_eps, sin_eps;
    int32_t lt_iter;
    int32_t kepler_iter;
    int32_t zero_start;         // correctors start from zero increments (no extrapolation)
};

size_t adjoint_lds_bytes(const AdjParams& p);
hipError_t launch_adjoint(const AdjParams& p, int mode, hipStream_t s);

}  // namespace kete
