// Host-side internal interfaces between the C ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "kete_device.hpp"
#include "kete_mi.h"

namespace kete {

// Gauss-Radau collocation constants (8 nodes including 0) for the
// increment form of the step: with D_m = F_m - F_0 (m = 1..7),
//   X(s) = x0 + s h v0 + h^2 (s^2/2 F0 + sum_m A_m(s) D_m)
//   V(s) = v0 + h (s F0 + sum_m B_m(s) D_m)
// and the highest monomial coefficient of the acceleration polynomial
//   b6 = sum_m E6[m] D_m.
// Row n = 0..7 is node s_n, row 8 is s = 1.
struct RadauConst {
    double s[9];
    double A[9][7];
    double B[9][7];
    double E6[7];
    double half_s2[9];
    // dense output at any sig in [0, 1]:
    //   A_m(sig) = sum_k Ap[m][k] sig^(k+2),  B_m(sig) = sum_k Bp[m][k] sig^(k+1)
    double Ap[7][8];
    double Bp[7][8];
    // Lagrange basis l_m on the nodes 0, s_1..s_7 (m = 1..7): 1 / prod_{k != m} (s_m - s_k)
    // and l_m(1), to extrapolate a step's increments into the next step
    double Lden[7];
    double L1[7];
};
// Ap then Bp, as copied next to the output epochs for the dense-output kernels
constexpr int kDenseCoefDoubles = 2 * 7 * 8;

// One staged ephemeris window of the integration: [t_a, t_b] lies within
// Chebyshev segments [seg_lo, seg_hi]; out >= 0 marks an output epoch.
struct Window {
    double t_a, t_b;
    int32_t seg_lo, seg_hi;
    int32_t out, pad;
};

// Segment holding time t (floor rule, clamped to the table).
__host__ __device__ inline int seg_clamped(double t, double t_start, double inv_seg, int n_seg) {
    const double k = floor((t - t_start) * inv_seg);
    return k < 0.0 ? 0 : (k > (double)(n_seg - 1) ? n_seg - 1 : (int)k);
}

// The next integration window from t toward target: it ends at target or
// at the segment joint w segment lengths past the start of t's segment,
// whichever comes first, and reads at most w + 1 consecutive segments
// (seg_lo..seg_hi), the capacity of the staging buffers.  Every path
// (host plans and the persistent kernel) uses this rule, so they window
// identically.  If t sits on a joint that rounding placed in the earlier
// segment, the limit moves one segment on so the window never has zero
// length.
__host__ __device__ inline Window next_window(double t, double target, double t_start, double seg_days,
                                              double inv_seg, int n_seg, int w) {
    const bool fwd = target > t;
    double tb;
    if (fwd) {
        const double kk = floor((t - t_start) * inv_seg);
        double limit = t_start + (kk + w) * seg_days;
        if (!(limit > t)) limit = t_start + (kk + w + 1) * seg_days;
        tb = limit < target ? limit : target;
    } else {
        const double kk = ceil((t - t_start) * inv_seg) - 1.0;
        double limit = t_start + (kk - w + 1) * seg_days;
        if (!(limit < t)) limit = t_start + (kk - w) * seg_days;
        tb = limit > target ? limit : target;
    }
    Window W;
    W.t_a = t;
    W.t_b = tb;
    int lo = seg_clamped(fwd ? t : tb, t_start, inv_seg, n_seg);
    int hi = seg_clamped(fwd ? tb : t, t_start, inv_seg, n_seg);
    if (hi - lo > w) {
        if (fwd) hi = lo + w; else lo = hi - w;
    }
    W.seg_lo = lo;
    W.seg_hi = hi;
    W.out = -1;
    W.pad = 0;
    return W;
}

// The same, forward in time only, with the window ends on a fixed grid:
// multiples of w segments from t_start (or the target).  A run that resumes
// inside a window (from a checkpoint) then ends its windows where the first
// run did, so both cut their steps at the same times.
__host__ __device__ inline Window aligned_window(double t, double target, double t_start, double seg_days,
                                                 double inv_seg, int n_seg, int w) {
    const double kk = floor((t - t_start) * inv_seg);
    double limit = t_start + (floor(kk / w) + 1.0) * w * seg_days;
    if (!(limit > t)) limit += w * seg_days;
    Window W;
    W.t_a = t;
    W.t_b = limit < target ? limit : target;
    const int lo = seg_clamped(t, t_start, inv_seg, n_seg);
    int hi = seg_clamped(W.t_b, t_start, inv_seg, n_seg);
    if (hi - lo > w) hi = lo + w;
    W.seg_lo = lo;
    W.seg_hi = hi;
    W.out = -1;
    W.pad = 0;
    return W;
}

struct NbodyParams {
    EphemArgs eph;
    RadauConst rc;
    double* state;          // [N][6] working state
    double* h_pref;         // [N] preferred step (days, > 0)
    const int32_t* perm;    // [N] object order (bucketed) or null
    int32_t* status;        // [N]
    double* x_out;          // [E][N][6]
    unsigned long long* stats;  // [8] or null
    const Window* win;      // windows of this launch
    const double* t_out;    // [E] output epochs (device)
    const double* dense_coef;   // [2][7][8] the monomial rows Ap, Bp of RadauConst (device)
    int32_t e_first;        // epochs e_first .. e_land - 1 are read off the step polynomials,
    int32_t e_land;         // epoch e_land ends the launch's last window (no dense epochs: e_first = e_land)
    int32_t n_win;
    int32_t n_obj;
    int32_t max_iter;
    int32_t max_steps;
    int32_t max_win_segs;   // LDS capacity in segments
    int32_t first_launch;
    int32_t zero_start;     // corrector starts from zero increments (no extrapolation)
    int32_t pad_;
    double eps, h_min, h_max, h_init, safety;
};

const RadauConst& radau_const();

// lanes_per_body: 1 (one lane per object) or 8 (an 8-lane group per object).
hipError_t launch_nbody(const NbodyParams& p, int block, int lanes_per_body, hipStream_t s);
// LDS of one block of the grouped integrator (dynamic and static).
size_t nbody_g8_lds_bytes(int n_body, int deg1, int max_win_segs, int block);

// Stable counting sort of objects into step-size buckets.
// Buckets per octave of the predicted step (the batched jobs' sort), and
// the most buckets one counting-sort pass takes.
constexpr int kBucketSub = 8;
constexpr int kMaxBuckets = 256;

// Sort keys of the bodies of one integrator launch (k_hpref_init): the high
// 16 bits hold the step class, the low 16 the time class; bodies are
// ordered by class, then by time (two stable counting-sort passes).
//   step class 0: "critical" bodies, whose predicted step count over the
//     launch exceeds kCritSteps: they set the launch's longest wavefronts,
//     so they come first, ordered by the time of their smallest distance
//     alone (kCritTimeBins classes), which lines up their perihelion
//     passages inside a wavefront;
//   step class 1 + k: the others, kClassSub classes per octave of the
//     predicted step above h_ref, then kTimeBins classes of that time.
constexpr double kCritSteps = 100.0;
constexpr int kClassSub = 2;
constexpr int kTimeBins = 64;
constexpr int kCritTimeBins = 256;

// One counting-sort pass over a digit of the keys: item i of the input
// order (in_perm[i], or i when in_perm is null) goes to its digit's
// bucket, stably.
struct BucketParams {
    const uint32_t* keys;   // [N] packed keys
    const int32_t* in_perm; // [N] input order or null
    int32_t* perm;          // [N] out
    int32_t* counts;        // [n_buckets][n_blocks] scratch
    int32_t n_obj;
    int32_t n_buckets;      // digit range (<= kMaxBuckets)
    int32_t shift;          // digit = (key >> shift) & 0xffff
    int32_t pad;
};
hipError_t launch_bucket(const BucketParams& p, hipStream_t s);

// Optional live timing of kernel launches with HIP events (per thread).
// kTimeFov brackets every kernel of a field-of-view call (preparation,
// binning, join, exact test, pair sort); kTimeFovJoin the join alone.
enum TimedKernel {
    kTimeNbody = 0, kTimeFov = 1, kTimeAdjoint = 2, kTimeBatch = 3, kTimeFovJoin = 4, kTimeKinds = 8
};
struct TimedScope {
    TimedScope(int kind, hipStream_t s);
    ~TimedScope();
    int kind;
    hipStream_t stream;
    void* stop;
};

// Exclusive scan of int32 counts (n + 1 outputs); scratch >= scan_scratch(n).
size_t scan_scratch_bytes(int64_t n);
hipError_t exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, void* scratch, hipStream_t s);

}  // namespace kete
