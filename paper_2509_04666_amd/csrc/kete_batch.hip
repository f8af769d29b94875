// Many independent propagation jobs of uneven size in one persistent
// launch.  A job is a set of bodies with a common start epoch and its own
// list of output epochs.  Its bodies are sorted by predicted step size
// (stable, per job) and cut into tiles of 8; a grid sized to the device
// pops tiles from a queue ordered longest-first, one wavefront per tile
// (8 bodies on 8-lane groups, as in the propagation kernel), each with
// its own LDS window of Chebyshev segments.
#include <math.h>

#include "kete_batch.hpp"
#include "kete_radau.hpp"

namespace kete {
namespace {

// Stable per-job bucketing by the initial step estimate 0.05 (r^3/mu)^(1/2):
// one block per job, two passes over the job's bodies in chunks of 256.
__global__ __launch_bounds__(256) void k_job_bucket(const BatchParams p) {
    __shared__ int hist[kMaxBuckets], base[kMaxBuckets], run[kMaxBuckets], wcount[4][kMaxBuckets];
    __shared__ double ext[2][4];
    const int J = blockIdx.x;
    const kete_job_t job = p.jobs[J];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nbk = p.n_buckets;
    for (int b = tid; b < nbk; b += 256) { hist[b] = 0; run[b] = 0; }
    // the job's time extent around its start, for the predicted steps
    double lo = 0.0, hi = 0.0;
    for (int64_t e = tid; e < job.n_epoch; e += 256) {
        const double dt = p.epochs[job.epoch_off + e] - job.t0;
        lo = fmin(lo, dt);
        hi = fmax(hi, dt);
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    if (lane == 0) { ext[0][wid] = lo; ext[1][wid] = hi; }
    __syncthreads();
    lo = fmin(fmin(ext[0][0], ext[0][1]), fmin(ext[0][2], ext[0][3]));
    hi = fmax(fmax(ext[1][0], ext[1][1]), fmax(ext[1][2], ext[1][3]));
    auto key_of = [&](int64_t k) {
        const double* x = p.x0 + 6 * (job.obj_off + k);
        const double h = predicted_step(x, x + 3, p.eph.gm[0], lo, hi);
        if (!(h < kInf)) return nbk - 1;
        int b = (int)floor(kBucketSub * log2(h * 64.0));
        return b < 0 ? 0 : (b >= nbk ? nbk - 1 : b);
    };
    for (int64_t k = tid; k < job.n_obj; k += 256) atomicAdd(&hist[key_of(k)], 1);
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int b = 0; b < nbk; ++b) { base[b] = acc; acc += hist[b]; }
    }
    __syncthreads();
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int64_t c0 = 0; c0 < job.n_obj; c0 += 256) {
        const int64_t k = c0 + tid;
        const int key = k < job.n_obj ? key_of(k) : -1;
        int rank = 0;
        for (int b = 0; b < nbk; ++b) {
            const unsigned long long m = __ballot(key == b);
            if (key == b) rank = __popcll(m & lt);
            if (lane == 0) wcount[wid][b] = __popcll(m);
        }
        __syncthreads();
        if (key >= 0) {
            int before = 0;
            for (int w = 0; w < wid; ++w) before += wcount[w][key];
            p.perm[job.obj_off + base[key] + run[key] + before + rank] = (int32_t)k;
        }
        __syncthreads();
        if (tid < nbk) for (int w = 0; w < 4; ++w) run[tid] += wcount[w][tid];
        __syncthreads();
    }
}


// One wavefront per block; it pops tiles of KETE_BATCH_TILE bodies of one
// job and integrates them as lane groups (one lane per collocation node,
// see GroupMap) through the job's epochs.
template <int NB, int NGR, int DEG1>
__global__ __launch_bounds__(64, 3) void k_batch_g8(const BatchParams p) {
    constexpr int G = KETE_BATCH_LANES;
    static_assert(GroupMap<G>::kBodies == KETE_BATCH_TILE, "tile = bodies per wavefront");
    extern __shared__ double smem[];
    const int lane = threadIdx.x;
    const GroupMap<G> M(lane);
    const int gl = M.gl;
    const int node = gl < 7 ? gl + 1 : 7;
    const EphemArgs& E = p.eph;
    const int bstride = p.max_win_segs * 3 * E.deg1;
    double* coefL = smem;
    double* e8 = smem + (((size_t)E.n_body * bstride + 1) & ~(size_t)1);
    g8_table_init(E, lane, e8);
    NodeRow R;
    load_node_row(p.rc, node, R);
    // dense-output rows and the wavefront's weight slots
    __shared__ double dcoef[kDenseCoefDoubles];
    __shared__ double dwts[16];
    for (int i = lane; i < kDenseCoefDoubles; i += 64) dcoef[i] = p.dense_coef[i];
    __syncthreads();
    const int W = p.max_win_segs - 1;            // segment lengths per window
    int lo = 1, hi = 0;                          // nothing staged yet
    for (;;) {
        int tile = 0;
        if (lane == 0) tile = (int)atomicAdd(p.tile_counter, 1u);
        tile = __shfl(tile, 0, 64);
        if (tile >= p.n_tiles) break;
        const int2 tj = p.tiles[tile];
        const kete_job_t job = p.jobs[tj.x];
        const int64_t k = (int64_t)tj.y * KETE_BATCH_TILE + M.grp;
        const bool valid = k < job.n_obj;
        const int64_t local = valid ? (p.n_buckets > 1 ? p.perm[job.obj_off + k] : k) : 0;
        const int64_t gobj = job.obj_off + local;
        G8State S;
        S.status = 0;
        S.active = valid;
        for (int i = 0; i < 3; ++i) {
            S.x0[i] = valid ? p.x0[6 * gobj + i] : (i == 0 ? 1.0 : 0.0);
            S.v0[i] = valid ? p.x0[6 * gobj + 3 + i] : 0.0;
            S.F0[i] = 0.0;
        }
        double hp = kInf;
        if (valid) {
            const double r = sqrt(dot3(S.x0, S.x0));
            hp = 0.05 * sqrt(r * r * r / E.gm[0]);
        }
        S.hw = groups_min<G>(S.active ? hp : kInf);
        if (!(S.hw < kInf)) S.hw = p.h_init;
        S.hp_new = kInf;
        S.t = job.t0;
        S.haveF0 = false;
        G8Count C;
        const double* ep = p.epochs + job.epoch_off;
        double* xg = g8_xch(e8, E.n_body, M.grp);
        auto put = [&](int e, double v, bool ok) {       // lane gl writes component gl
            if (valid && gl < 6)
                p.x_out[job.xout_off + ((int64_t)e * job.n_obj + local) * 6 + gl] = ok ? v : __builtin_nan("");
        };
        // The epochs run away from t0 (later ones ascending, then earlier
        // ones descending).  Each run of epochs in one direction lands on
        // its last epoch; the others come off the collocation polynomial
        // of the step that spans them (unless every epoch is landed on).
        int e = 0;
        while (e < job.n_epoch) {
            if (ep[e] == S.t) {
                put(e, state_component(S.x0, S.v0, gl < 6 ? gl : 5), S.active && S.status == 0);
                ++e;
                continue;
            }
            const bool fwd = ep[e] > S.t;
            int e_end = e;
            if (!p.land_epochs)
                while (e_end + 1 < job.n_epoch && (fwd ? ep[e_end + 1] > ep[e_end] : ep[e_end + 1] < ep[e_end]))
                    ++e_end;
            const double target = ep[e_end];
            int e_next = e;                              // wave-uniform cursor over e .. e_end - 1
            auto dense_out = [&](double ts, double h, const double dn[3], const G8State& St) {
                if (e_next >= e_end) return;
                const double te = ts + h;
                double tk = ep[e_next];
                if (!(h > 0.0 ? tk <= te : tk >= te)) return;
                wave_lds_sync();                        // earlier reads of the exchange rows are done
                xg[gl] = dn[0];
                xg[8 + gl] = dn[1];
                xg[16 + gl] = dn[2];
                wave_lds_sync();
                for (;;) {
                    const double sig = (tk - ts) / h;
                    dense_weights_wave(dcoef, sig, lane, dwts);
                    double X[3], V[3];
                    dense_state_wave(dwts, xg, St.x0, St.v0, St.F0, h, sig, X, V);
                    put(e_next, state_component(X, V, gl < 6 ? gl : 5), St.active && St.status == 0);
                    if (++e_next >= e_end) break;
                    tk = ep[e_next];
                    if (!(h > 0.0 ? tk <= te : tk >= te)) break;
                }
            };
            while (S.t != target) {
                const Window Wn = next_window(S.t, target, E.t_start, E.seg_days, E.inv_seg, E.n_seg, W);
                ensure_window(E, Wn.seg_lo, Wn.seg_hi, lo, hi, coefL, bstride);
                g8_integrate<NB, NGR, DEG1, G, kStartExtrapolate>(p, R, node, gl, M.grp, lane, coefL, bstride, e8, lo,
                                                                  hi, Wn.t_b, S, C, dense_out);
                S.t = Wn.t_b;
            }
            put(e_end, state_component(S.x0, S.v0, gl < 6 ? gl : 5), S.active && S.status == 0);
            e = e_end + 1;
        }
        if (valid && gl == 0) p.status[gobj] = S.status;
    }
}

}  // namespace

size_t batch_lds_bytes(const BatchParams& p) {
    return ((((size_t)p.eph.n_body * p.max_win_segs * 3 * p.eph.deg1 + 1) & ~(size_t)1) +
            (size_t)g8_wave_doubles(p.eph.n_body)) * sizeof(double);
}

// The dense-output rows of the constants into device memory (a tiny kernel,
// so the copy is part of a captured graph too).
__global__ void k_dense_coef(const BatchParams p) {
    const int i = threadIdx.x;
    if (i < 56) p.dense_coef[i] = p.rc.Ap[i / 8][i % 8];
    else if (i < kDenseCoefDoubles) p.dense_coef[i] = p.rc.Bp[(i - 56) / 8][(i - 56) % 8];
}

hipError_t launch_batch(const BatchParams& p, int waves_per_cu, hipStream_t s) {
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    hipError_t e;
    if ((e = fill_zero(p.tile_counter, sizeof(unsigned int), s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_dense_coef, dim3(1), dim3(128), 0, s, p);
    if (p.n_jobs > 0 && p.n_buckets > 1)
        hipLaunchKernelGGL(k_job_bucket, dim3((unsigned)p.n_jobs), dim3(256), 0, s, p);
    const int grid = std::max(1, std::min(ncu * waves_per_cu, p.n_tiles));
    const size_t lds = batch_lds_bytes(p);
    const int nb = p.eph.n_body, ngr = p.eph.n_gr, d1 = p.eph.deg1;
    if (nb == 10 && ngr == 3 && d1 == 13) hipLaunchKernelGGL((k_batch_g8<10, 3, 13>), dim3(grid), dim3(64), lds, s, p);
    else if (nb == 3 && ngr == 2 && d1 == 13)
        hipLaunchKernelGGL((k_batch_g8<3, 2, 13>), dim3(grid), dim3(64), lds, s, p);
    else hipLaunchKernelGGL((k_batch_g8<0, 0, 0>), dim3(grid), dim3(64), lds, s, p);
    return hipGetLastError();
}

}  // namespace kete
