// n-body propagation of massless bodies on gfx950 (App. A force model,
// Gauss-Radau collocation with the predictor removed, App. A.6).
//
// Two layouts share the force, the Chebyshev window staging and the step
// control.  k_nbody_g8 (the default) spreads each object over an 8-lane
// group, one collocation node per lane, so a wavefront integrates 8
// objects; k_nbody keeps one object per lane (64 per wavefront).  The
// objects of a wavefront share the time grid: the step size is the
// smallest one any of them asks for, so the perturber states at the node
// times of a step are evaluated once per wavefront and read from LDS.
// The Chebyshev coefficients of the segments a window needs are staged in
// LDS once per workgroup.  Objects are sorted by predicted step size
// before a launch so that the objects of one wavefront want similar steps.
#include <math.h>

#include "kete_radau.hpp"

namespace kete {
hipError_t launch_bucket(const BucketParams& p, hipStream_t s);

namespace {

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_nbody(const NbodyParams p) {
    extern __shared__ double smem[];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const EphemArgs& E = p.eph;
    const RadauConst& rc = p.rc;
    const int nb = E.n_body, deg1 = E.deg1;
    const int cps = 3 * deg1;                         // doubles per segment
    const int bstride = p.max_win_segs * cps;         // doubles per body in LDS
    double* coefL = smem;
    double* ephW = smem + (size_t)nb * bstride + (size_t)wid * kNodes * nb * 6;

    const long gi = (long)blockIdx.x * BLOCK + tid;
    const bool valid = gi < p.n_obj;
    const int j = valid ? (p.perm ? p.perm[gi] : (int)gi) : 0;
    bool active = valid && p.status[j] == 0;
    int my_status = valid ? p.status[j] : 0;

    double x0[3] = {1.0, 0.0, 0.0}, v0[3] = {0.0, 0.0, 0.0};
    double hin = kInf;
    if (valid) {
#pragma unroll
        for (int i = 0; i < 3; ++i) { x0[i] = p.state[6 * j + i]; v0[i] = p.state[6 * j + 3 + i]; }
        hin = p.h_pref[j];
    }
    double hw = wave_min(active ? hin : kInf);
    if (!(hw < kInf)) hw = p.h_init;
    double hp_new = kInf;

    unsigned long long c_steps = 0, c_iter = 0, c_rej = 0, c_lsteps = 0, c_liter = 0, c_chain = 0;
    double t = p.win[0].t_a;
    double F0[3] = {0.0, 0.0, 0.0};
    bool haveF0 = false;

    for (int w = 0; w < p.n_win; ++w) {
        const Window W = p.win[w];
        __syncthreads();
        stage_window(E, W.seg_lo, W.seg_hi, bstride, tid, BLOCK, coefL);
        __syncthreads();
        const double tb = W.t_b;
        if (__ballot(active) == 0ull) {
            t = tb;
        }
        while (t != tb) {
            const double dir = tb > t ? 1.0 : -1.0;
            double hmag = hw;
            if (p.h_max > 0.0 && hmag > p.h_max) hmag = p.h_max;
            double h = dir * hmag;
            bool landed = false;
            if (fabs(h) >= fabs(tb - t)) { h = tb - t; landed = true; }
            if ((long)c_steps >= p.max_steps) {
                if (active) { my_status = KETE_ST_MAX_STEPS; active = false; }
                t = tb;
                break;
            }
            const double t_end = landed ? tb : t + h;
            const double hh = h * h;

            // perturbers at the 9 node times, one Clenshaw chain per lane
            node_ephemeris(coefL, bstride, E, rc, W.seg_lo, W.seg_hi, t, h, t_end, lane, ephW);
            c_chain += kNodes * nb * 3;

            if (!haveF0) { accel(ephW, E, x0, v0, F0); haveF0 = true; }

            double D[7][3], b6p[3];
            const int it = corrector(rc, E, ephW, x0, v0, F0, h, active, p.max_iter, D, b6p, c_liter);
            c_iter += it;

            // IAS15-style control on |b6| / |a| at the last node
            double fm = 0.0, bm = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) { fm = fmax(fm, fabs(D[6][c] + F0[c])); bm = fmax(bm, fabs(b6p[c])); }
            const double ebl = fm > 0.0 ? bm / fm : 0.0;
            double hl = (ebl > 0.0 && ebl < kInf) ? fabs(h) * step_factor(p.eps / ebl) : fabs(h) / p.safety;
            if (!active) hl = kInf;
            if (active && hl < p.h_min) { my_status = KETE_ST_STEP_UNDERFLOW; active = false; hl = kInf; }
            const double hn = wave_min(hl);
            if (!(hn < kInf)) { t = tb; break; }
            if (hn < p.safety * fabs(h)) {       // reject and retry from the same state
                hw = hn;
                ++c_rej;
                continue;
            }
            // accept: step end from the collocation polynomial
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double ax = rc.half_s2[8] * F0[c], av = F0[c];
#pragma unroll
                for (int m = 0; m < 7; ++m) {
                    ax = fma(rc.A[8][m], D[m][c], ax);
                    av = fma(rc.B[8][m], D[m][c], av);
                }
                x0[c] = fma(hh, ax, fma(h, v0[c], x0[c]));
                v0[c] = fma(h, av, v0[c]);
            }
            t = t_end;
            ++c_steps;
            c_lsteps += __popcll(__ballot(active));
            if (active && !(isfinite(x0[0]) && isfinite(x0[1]) && isfinite(x0[2]) &&
                            isfinite(v0[0]) && isfinite(v0[1]) && isfinite(v0[2]))) {
                my_status = KETE_ST_NONFINITE; active = false;
            }
            accel(ephW + 8 * nb * 6, E, x0, v0, F0);
            if (landed) {
                hw = fmin(hw, hn);
            } else {
                hw = fmin(hn, fabs(h) / p.safety);
                hp_new = fmin(hp_new, fmin(hl, fabs(h) / p.safety));
            }
        }
        if (W.out >= 0 && valid) {
            double* dst = p.x_out + ((size_t)W.out * p.n_obj + j) * 6;
            const bool ok = active && my_status == 0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                dst[i] = ok ? x0[i] : __builtin_nan("");
                dst[3 + i] = ok ? v0[i] : __builtin_nan("");
            }
        }
    }
    if (valid) {
#pragma unroll
        for (int i = 0; i < 3; ++i) { p.state[6 * j + i] = x0[i]; p.state[6 * j + 3 + i] = v0[i]; }
        if (hp_new < kInf) p.h_pref[j] = hp_new;
        p.status[j] = my_status;
    }
    if (p.stats && lane == 0 && __ballot(valid) != 0ull) {
        atomicAdd(p.stats + 0, c_steps);
        atomicAdd(p.stats + 1, c_iter);
        atomicAdd(p.stats + 2, c_rej);
        atomicAdd(p.stats + 3, c_lsteps);
        atomicAdd(p.stats + 4, c_liter);
        atomicAdd(p.stats + 5, c_chain);
    }
}

// G lanes per object (7 or 8, see GroupMap): a wavefront integrates 9 or
// 8 objects, each spread over a group whose lanes own one collocation
// node each.  The objects of a wavefront share the time grid and the
// perturber table as above; each sweep evaluates the force at all 7 nodes
// of an object at once.  Output and counters are per object, as in
// k_nbody.
template <int BLOCK, int G, int NB, int NGR, int DEG1>
__global__ __launch_bounds__(BLOCK, 3) void k_nbody_g8(const NbodyParams p) {
    extern __shared__ double smem[];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const GroupMap<G> M(lane);
    const int gl = M.gl;                              // lane within the object's group
    const int node = gl < 7 ? gl + 1 : 7;
    const EphemArgs& E = p.eph;
    const RadauConst& rc = p.rc;
    const int nb = E.n_body, deg1 = E.deg1;
    const int cps = 3 * deg1;
    const int bstride = p.max_win_segs * cps;
    double* coefL = smem;
    // the table is read with 16-byte loads: start it on a 16-byte boundary
    double* e8 = smem + (((size_t)nb * bstride + 1) & ~(size_t)1) + (size_t)wid * g8_wave_doubles(nb);
    g8_table_init(E, lane, e8);
    // per-node constants of the 8 lanes of a group, read from LDS in the
    // sweeps to keep registers for more wavefronts per SIMD
    __shared__ NodeRow rows[kGroup];
    if (tid < kGroup) {
        NodeRow r;
        load_node_row(rc, tid < 7 ? tid + 1 : 7, r);
        rows[tid] = r;
    }
    // dense-output rows, read from LDS at the epochs inside a step
    __shared__ double dcoef[kDenseCoefDoubles];
    __shared__ double dwts[BLOCK / kWave][16];      // per wavefront: the 14 weights of an epoch
    if (p.e_first < p.e_land)
        for (int i = tid; i < kDenseCoefDoubles; i += BLOCK) dcoef[i] = p.dense_coef[i];
    __syncthreads();
    const NodeRow& R = rows[gl];

    const long gi = ((long)blockIdx.x * (BLOCK / kWave) + wid) * GroupMap<G>::kBodies + M.grp;
    const bool valid = gi < p.n_obj;
    const int j = valid ? (p.perm ? p.perm[gi] : (int)gi) : 0;
    G8State S;
    S.active = valid && p.status[j] == 0;
    S.status = valid ? p.status[j] : 0;
    S.x0[0] = 1.0; S.x0[1] = S.x0[2] = 0.0;
    S.v0[0] = S.v0[1] = S.v0[2] = 0.0;
    S.F0[0] = S.F0[1] = S.F0[2] = 0.0;
    double hin = kInf;
    if (valid) {
#pragma unroll
        for (int i = 0; i < 3; ++i) { S.x0[i] = p.state[6 * j + i]; S.v0[i] = p.state[6 * j + 3 + i]; }
        hin = p.h_pref[j];
    }
    S.hw = groups_min<G>(S.active ? hin : kInf);
    if (!(S.hw < kInf)) S.hw = p.h_init;
    S.hp_new = kInf;
    S.t = p.win[0].t_a;
    S.haveF0 = false;
    G8Count C;

    // Epochs e_first .. e_land - 1 come off the collocation polynomial of
    // the accepted step that spans them (the cursor is wave-uniform: the
    // wavefront's objects share every step).
    double* xg = g8_xch(e8, nb, M.grp);
    int e_next = p.e_first;
    auto put = [&](int e, double v, bool ok) {      // lane gl writes component gl
        if (valid && gl < 6) p.x_out[((size_t)e * p.n_obj + j) * 6 + gl] = ok ? v : __builtin_nan("");
    };
    while (e_next < p.e_land && p.t_out[e_next] == S.t) {       // epochs at the start time
        put(e_next, state_component(S.x0, S.v0, gl < 6 ? gl : 5), S.active && S.status == 0);
        ++e_next;
    }
    auto dense_out = [&](double ts, double h, const double dn[3], const G8State& St) {
        if (e_next >= p.e_land) return;
        const double te = ts + h;
        double tk = p.t_out[e_next];
        if (!(h > 0.0 ? tk <= te : tk >= te)) return;
        wave_lds_sync();                    // earlier reads of the exchange rows are done
        xg[gl] = dn[0];
        xg[8 + gl] = dn[1];
        xg[16 + gl] = dn[2];
        wave_lds_sync();
        for (;;) {
            const double sig = (tk - ts) / h;
            dense_weights_wave(dcoef, sig, lane, dwts[wid]);
            double X[3], V[3];
            dense_state_wave(dwts[wid], xg, St.x0, St.v0, St.F0, h, sig, X, V);
            put(e_next, state_component(X, V, gl < 6 ? gl : 5), St.active && St.status == 0);
            if (++e_next >= p.e_land) break;
            tk = p.t_out[e_next];
            if (!(h > 0.0 ? tk <= te : tk >= te)) break;
        }
    };

    for (int w = 0; w < p.n_win; ++w) {
        const Window W = p.win[w];
        __syncthreads();
        stage_window(E, W.seg_lo, W.seg_hi, bstride, tid, BLOCK, coefL);
        __syncthreads();
        g8_integrate<NB, NGR, DEG1, G, kStartExtrapolate>(p, R, node, gl, M.grp, lane, coefL, bstride, e8, W.seg_lo,
                                                          W.seg_hi, W.t_b, S, C, dense_out);
        if (W.out >= 0 && valid && gl < 6) {
            // lane gl of the group writes component gl of the state
            double* dst = p.x_out + ((size_t)W.out * p.n_obj + j) * 6;
            const bool ok = S.active && S.status == 0;
            dst[gl] = ok ? state_component(S.x0, S.v0, gl) : __builtin_nan("");
        }
    }
    if (valid && gl < 6) p.state[6 * j + gl] = state_component(S.x0, S.v0, gl);
    if (valid && gl == 0) {
        if (S.hp_new < kInf) p.h_pref[j] = S.hp_new;
        p.status[j] = S.status;
    }
    const unsigned long long c_steps = C.steps, c_iter = C.iter, c_rej = C.rej, c_lsteps = C.lsteps,
                             c_liter = C.liter, c_chain = C.chain, c_vchain = C.vchain, c_lpred = C.lpred;
    if (p.stats && lane == 0 && __ballot(valid) != 0ull) {
        atomicAdd(p.stats + 0, c_steps);
        atomicAdd(p.stats + 1, c_iter);
        atomicAdd(p.stats + 2, c_rej);
        atomicAdd(p.stats + 3, c_lsteps);
        atomicAdd(p.stats + 4, c_liter);
        atomicAdd(p.stats + 5, c_chain);
        atomicAdd(p.stats + 6, c_vchain);
        atomicAdd(p.stats + 7, c_lpred);
    }
}

// ---------------------------------------------------------------- buckets
__device__ __forceinline__ int bucket_digit(const BucketParams& p, long i, int& item) {
    item = p.in_perm ? p.in_perm[i] : (int)i;
    const int d = (int)((p.keys[item] >> p.shift) & 0xffffu);
    return d < p.n_buckets ? d : p.n_buckets - 1;
}

__global__ __launch_bounds__(256) void k_bucket_count(const BucketParams p) {
    __shared__ int hist[kMaxBuckets];
    const int tid = threadIdx.x;
    for (int k = tid; k < p.n_buckets; k += 256) hist[k] = 0;
    __syncthreads();
    const long i = (long)blockIdx.x * 256 + tid;
    int item;
    if (i < p.n_obj) atomicAdd(&hist[bucket_digit(p, i, item)], 1);
    __syncthreads();
    for (int k = tid; k < p.n_buckets; k += 256) p.counts[(size_t)k * gridDim.x + blockIdx.x] = hist[k];
}

// Stable scatter: the rank inside a block follows the object index.
__global__ __launch_bounds__(256) void k_bucket_scatter(const BucketParams p, const int32_t* __restrict__ offs) {
    __shared__ int wcount[4][kMaxBuckets];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const long i = (long)blockIdx.x * 256 + tid;
    const bool valid = i < p.n_obj;
    int item = 0;
    const int key = valid ? bucket_digit(p, i, item) : -1;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int rank = 0;
    for (int k = 0; k < p.n_buckets; ++k) {
        const unsigned long long m = __ballot(key == k);
        if (key == k) rank = __popcll(m & lt);
        if (lane == 0) wcount[wid][k] = __popcll(m);
    }
    __syncthreads();
    if (valid) {
        int before = 0;
        for (int w = 0; w < wid; ++w) before += wcount[w][key];
        const int pos = offs[(size_t)key * gridDim.x + blockIdx.x] + before + rank;
        p.perm[pos] = (int32_t)item;
    }
}

__global__ void k_iota(int32_t* __restrict__ perm, int n) {
    const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) perm[j] = (int32_t)j;
}

// Predicted step and sort key (see BucketParams) of every body over the
// launch's time span [dt_lo, dt_hi] from its start state (taken as
// heliocentric: the Sun is within 0.01 au of the barycentre, which only
// blurs the ordering).
__global__ void k_hpref_init(const double* __restrict__ x0, double* __restrict__ h_pref, uint32_t* __restrict__ keys,
                             int n, double mu, double dt_lo, double dt_hi, int n_class, double h_ref) {
    const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double tm = 0.0;
    const double h = predicted_step(x0 + 6 * j, x0 + 6 * j + 3, mu, dt_lo, dt_hi, &tm);
    h_pref[j] = h;
    if (!keys) return;
    const double span = dt_hi - dt_lo;
    const double frac = span > 0.0 ? fmin(fmax((tm - dt_lo) / span, 0.0), 1.0) : 0.0;
    uint32_t hi, lo;
    if (h > 0.0 && span / h > kCritSteps) {
        hi = 0;
        lo = (uint32_t)fmin(frac * kCritTimeBins, kCritTimeBins - 1.0);
    } else {
        const double c = (h > 0.0 && h < kInf) ? floor(kClassSub * log2(h / h_ref)) : (double)(n_class - 2);
        hi = 1u + (uint32_t)fmin(fmax(c, 0.0), (double)(n_class - 2));
        lo = (uint32_t)fmin(frac * kTimeBins, kTimeBins - 1.0);
    }
    keys[j] = hi << 16 | lo;
}

}  // namespace

size_t nbody_g8_lds_bytes(int n_body, int deg1, int max_win_segs, int block) {
    return ((((size_t)n_body * max_win_segs * 3 * deg1 + 1) & ~(size_t)1) +
            (size_t)(block / kWave) * g8_wave_doubles(n_body)) * sizeof(double) +
           sizeof(NodeRow) * kGroup + kDenseCoefDoubles * sizeof(double);
}

hipError_t launch_nbody(const NbodyParams& p, int block, int lanes_per_body, hipStream_t s) {
    const size_t lds = ((size_t)p.eph.n_body * p.max_win_segs * 3 * p.eph.deg1 +
                        (size_t)(block / kWave) * kNodes * p.eph.n_body * 6) * sizeof(double);
    if (lanes_per_body == 7 || lanes_per_body == 8) {
        const size_t lds8 = ((((size_t)p.eph.n_body * p.max_win_segs * 3 * p.eph.deg1 + 1) & ~(size_t)1) +
                             (size_t)(block / kWave) * g8_wave_doubles(p.eph.n_body)) * sizeof(double);
        const long per_wave = lanes_per_body == 7 ? GroupMap<7>::kBodies : GroupMap<8>::kBodies;
        const long waves = ((long)p.n_obj + per_wave - 1) / per_wave;
        const int wpb = block / kWave;
        const int grid = (int)((waves + wpb - 1) / wpb);
        if (grid == 0) return hipSuccess;
        // perturber tables of the common shapes get an unrolled force loop
        const int nb = p.eph.n_body, ngr = p.eph.n_gr, d1 = p.eph.deg1;
#define KETE_G8(B, G)                                                                                           \
    do {                                                                                                        \
        if (nb == 10 && ngr == 3 && d1 == 13)                                                                   \
            hipLaunchKernelGGL((k_nbody_g8<B, G, 10, 3, 13>), dim3(grid), dim3(B), lds8, s, p);                 \
        else if (nb == 3 && ngr == 2 && d1 == 13)                                                               \
            hipLaunchKernelGGL((k_nbody_g8<B, G, 3, 2, 13>), dim3(grid), dim3(B), lds8, s, p);                  \
        else hipLaunchKernelGGL((k_nbody_g8<B, G, 0, 0, 0>), dim3(grid), dim3(B), lds8, s, p);                  \
    } while (0)
        if (lanes_per_body == 7) {
            switch (block) {
                case 64: KETE_G8(64, 7); break;
                case 128: KETE_G8(128, 7); break;
                case 256: KETE_G8(256, 7); break;
                default: return hipErrorInvalidValue;
            }
        } else {
            switch (block) {
                case 64: KETE_G8(64, 8); break;
                case 128: KETE_G8(128, 8); break;
                case 256: KETE_G8(256, 8); break;
                default: return hipErrorInvalidValue;
            }
        }
#undef KETE_G8
        return hipGetLastError();
    }
    if (lanes_per_body != 1) return hipErrorInvalidValue;
    const int grid = (int)((p.n_obj + block - 1) / block);
    if (grid == 0) return hipSuccess;
    switch (block) {
        case 64: hipLaunchKernelGGL(k_nbody<64>, dim3(grid), dim3(64), lds, s, p); break;
        case 128: hipLaunchKernelGGL(k_nbody<128>, dim3(grid), dim3(128), lds, s, p); break;
        case 256: hipLaunchKernelGGL(k_nbody<256>, dim3(grid), dim3(256), lds, s, p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_hpref_init(const double* x0, double* h_pref, uint32_t* keys, int n, double mu, double dt_lo,
                             double dt_hi, int n_class, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hpref_init, dim3((n + 255) / 256), dim3(256), 0, s, x0, h_pref, keys, n, mu, dt_lo, dt_hi,
                       n_class, 1.0 / 64.0);
    return hipGetLastError();
}

// Bodies ordered by their keys: the time class first, then (stably) the
// step class, into perm; tmp [n] holds the first pass's order.
hipError_t launch_body_sort(const uint32_t* keys, int n, int n_class, int32_t* perm, int32_t* tmp, int32_t* counts,
                            hipStream_t s) {
    BucketParams B;
    B.keys = keys;
    B.counts = counts;
    B.n_obj = n;
    B.pad = 0;
    B.in_perm = nullptr;
    B.perm = tmp;
    B.n_buckets = kCritTimeBins;
    B.shift = 0;
    hipError_t e = launch_bucket(B, s);
    if (e != hipSuccess) return e;
    B.in_perm = tmp;
    B.perm = perm;
    B.n_buckets = n_class;
    B.shift = 16;
    return launch_bucket(B, s);
}

hipError_t launch_iota(int32_t* perm, int n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3((n + 255) / 256), dim3(256), 0, s, perm, n);
    return hipGetLastError();
}

hipError_t launch_bucket(const BucketParams& p, hipStream_t s) {
    const int nblk = (p.n_obj + 255) / 256;
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bucket_count, dim3(nblk), dim3(256), 0, s, p);
    // offsets are written after the counts (bucket-major), total at the end
    int32_t* offs = p.counts + (size_t)p.n_buckets * nblk;
    void* scratch = offs + (size_t)p.n_buckets * nblk + 1;
    hipError_t e = exclusive_scan_i32(p.counts, offs, (int64_t)p.n_buckets * nblk, scratch, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bucket_scatter, dim3(nblk), dim3(256), 0, s, p, (const int32_t*)offs);
    return hipGetLastError();
}

size_t bucket_scratch_ints(int64_t n_obj, int n_buckets) {
    const int64_t nblk = (n_obj + 255) / 256;
    return (size_t)(2 * n_buckets * nblk + 1) + scan_scratch_bytes(n_buckets * nblk) / sizeof(int32_t) + 64;
}

}  // namespace kete
