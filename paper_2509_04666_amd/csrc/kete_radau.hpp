// Device pieces of the Gauss-Radau collocation step shared by the
// propagation and adjoint kernels: perturber chains into LDS, the force
// of Eqs. A.1 + A.3, its Jacobians, and the corrector sweep.
#pragma once

#include "kete_internal.hpp"

namespace kete {

constexpr int kNodes = 9;   // s_0 = 0, s_1..s_7, and s = 1 (step end)
constexpr double kInf = 1e300;

// Eq. A.4 (App. A.3) of J2 body q in vector form.  With d = x - x_m the
// object's offset from the body (Eq. A.4's r is -d, the sign of Eq. A.2's
// Newtonian term), z = d . p along the unit pole p and k = (3/2) J2 mu R^2,
// the componentwise expression in the body's equatorial frame reads
//   a = -k / |d|^5 [(1 - 5 z^2 / |d|^2) d + 2 z p].
// id = 1 / |d|.
__device__ __forceinline__ void j2_add(const EphemArgs& E, int q, const double d[3], double id, double a[3]) {
    const double* p = E.j2p[q];
    const double id2 = id * id;
    const double s = -E.j2k[q] * (id2 * id2 * id);
    const double z = fma(d[0], p[0], fma(d[1], p[1], d[2] * p[2]));
    const double c = s * fma(-5.0 * z * id2, z, 1.0);
    const double e = 2.0 * s * z;
#pragma unroll
    for (int i = 0; i < 3; ++i) a[i] = fma(c, d[i], fma(e, p[i], a[i]));
}

// Its Jacobian da/dx, added to Jx (symmetric, the Hessian of the J2
// potential):
//   -k [A I + B d d^T + C (d p^T + p d^T) + E p p^T],
//   A = |d|^-5 - 5 z^2 |d|^-7, B = 35 z^2 |d|^-9 - 5 |d|^-7,
//   C = -10 z |d|^-7, E = 2 |d|^-5.
__device__ __forceinline__ void j2_jac_add(const EphemArgs& E, int q, const double d[3], double id, double Jx[9]) {
    const double* p = E.j2p[q];
    const double k = E.j2k[q];
    const double id2 = id * id, id5 = id2 * id2 * id, id7 = id5 * id2;
    const double z = fma(d[0], p[0], fma(d[1], p[1], d[2] * p[2]));
    const double A = -k * (id5 - 5.0 * z * z * id7);
    const double B = -k * (35.0 * z * z * id7 * id2 - 5.0 * id7);
    const double C = -k * (-10.0 * z * id7);
    const double Ee = -k * 2.0 * id5;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Jx[3 * i + j] += (i == j ? A : 0.0) + B * d[i] * d[j] + C * (d[i] * p[j] + p[i] * d[j]) + Ee * p[i] * p[j];
}

// Acceleration at one node from the LDS perturber table e[b][6]:
// Eq. A.1 with the attractive sign, plus Eq. A.3 (eps = 0) where kgr != 0
// and Eq. A.4 for the J2 bodies.
__device__ __forceinline__ void accel(const double* __restrict__ e, const EphemArgs& E,
                                      const double X[3], const double V[3], double F[3]) {
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int b = 0; b < E.n_body; ++b) {
        const double* pb = e + 6 * b;
        const double rx = X[0] - pb[0], ry = X[1] - pb[1], rz = X[2] - pb[2];
        const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
        const double ir = rsqrt(r2);
        const double ir3 = ir * ir * ir;
        const double gm = E.gm[b];
        double f = -gm * ir3;
        const double k = E.kgr[b];
        if (k != 0.0) {
            const double wx = V[0] - pb[3], wy = V[1] - pb[4], wz = V[2] - pb[5];
            const double w2 = fma(wx, wx, fma(wy, wy, wz * wz));
            const double rw = fma(rx, wx, fma(ry, wy, rz * wz));
            const double g = k * ir3;
            f = fma(g, 4.0 * gm * ir - w2, f);
            const double q = 4.0 * g * rw;
            ax = fma(q, wx, ax); ay = fma(q, wy, ay); az = fma(q, wz, az);
        }
        ax = fma(f, rx, ax); ay = fma(f, ry, ay); az = fma(f, rz, az);
    }
    F[0] = ax; F[1] = ay; F[2] = az;
    for (int q = 0; q < E.n_j2; ++q) {
        const double* pb = e + 6 * E.j2_body[q];
        const double d[3] = {X[0] - pb[0], X[1] - pb[1], X[2] - pb[2]};
        j2_add(E, q, d, rsqrt(fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2]))), F);
    }
}

// Perturber positions and velocities at the 9 node times of a step
// (t + s_n h, and t_end for s = 1), one Clenshaw chain per lane, from the
// LDS window of segments [seg_lo, seg_hi]; results in ephW[n][b][6].
__device__ __forceinline__ void node_ephemeris(const double* __restrict__ coefL, int bstride, const EphemArgs& E,
                                               const RadauConst& rc, int seg_lo, int seg_hi, double t, double h,
                                               double t_end, int lane, double* __restrict__ ephW) {
    const int nb = E.n_body, deg1 = E.deg1, cps = 3 * deg1;
    const int nchain = kNodes * nb * 3;
    for (int c = lane; c < nchain; c += kWave) {
        const int n = c / (nb * 3);
        const int r = c - n * nb * 3;
        const int b = r / 3, i = r - 3 * b;
        const double tt = (n == kNodes - 1) ? t_end : t + rc.s[n] * h;
        const int k = seg_index(tt, E.t_start, E.inv_seg, seg_lo, seg_hi);
        const double tau = 2.0 * (tt - (E.t_start + (double)k * E.seg_days)) * E.inv_seg - 1.0;
        double pv, dv;
        clenshaw(coefL + b * bstride + (k - seg_lo) * cps + i * deg1, deg1, tau, pv, dv);
        ephW[(n * nb + b) * 6 + i] = pv;
        ephW[(n * nb + b) * 6 + 3 + i] = dv * 2.0 * E.inv_seg;
    }
    wave_lds_sync();
}

// Stage the Chebyshev segments [seg_lo, seg_hi] of every body into LDS
// (cooperatively by `nthreads` threads; the caller synchronizes).
__device__ __forceinline__ void stage_window(const EphemArgs& E, int seg_lo, int seg_hi, int bstride, int tid,
                                             int nthreads, double* __restrict__ coefL) {
    const int cps = 3 * E.deg1;
    const int per_body = (seg_hi - seg_lo + 1) * cps;
    const int total = E.n_body * per_body;
    for (int i = tid; i < total; i += nthreads) {
        const int b = i / per_body, r = i - b * per_body;
        coefL[b * bstride + r] = E.coef[((size_t)b * E.n_seg + seg_lo) * cps + r];
    }
}

// Stage segments a..b into LDS unless they are already there (one
// wavefront per block: lanes 0..63 copy).
__device__ __forceinline__ void ensure_window(const EphemArgs& E, int a, int b, int& lo, int& hi, double* coefL,
                                              int bstride) {
    if (a >= lo && b <= hi) return;
    __syncthreads();
    stage_window(E, a, b, bstride, threadIdx.x, 64, coefL);
    __syncthreads();
    lo = a; hi = b;
}

// The collocation corrector: fixed-point sweeps over the 7 nodes
// (Gauss-Seidel: each node sees the increments already updated) until the
// change of b6 relative to |a| is below 1e-16, stops decreasing after the
// third sweep, or max_iter sweeps ran.  Returns the sweep count; b6 gets
// the final highest coefficient.
__device__ __forceinline__ int corrector(const RadauConst& rc, const EphemArgs& E, const double* __restrict__ ephW,
                                         const double x0[3], const double v0[3], const double F0[3], double h,
                                         bool active, int max_iter, double D[7][3], double b6[3],
                                         unsigned long long& lane_iters) {
    const double hh = h * h;
#pragma unroll
    for (int m = 0; m < 7; ++m) { D[m][0] = D[m][1] = D[m][2] = 0.0; }
    b6[0] = b6[1] = b6[2] = 0.0;
    double pc = 1e300, pcl;
    int it = 0;
    do {
        pcl = pc;
        ++it;
        // An opaque zero row offset keeps the collocation constants in the
        // kernel-argument segment (scalar loads per node) instead of being
        // hoisted into vector registers.
        int z;
        asm volatile("s_mov_b32 %0, 0" : "=s"(z));
#pragma unroll
        for (int n = 1; n <= 7; ++n) {
            const int nz = n + z;
            const double sh = rc.s[nz] * h;
            double X[3], V[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double acc = rc.half_s2[nz] * F0[c];
#pragma unroll
                for (int m = 0; m < 7; ++m) acc = fma(rc.A[nz][m], D[m][c], acc);
                X[c] = fma(hh, acc, fma(sh, v0[c], x0[c]));
            }
            if (E.has_gr) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double av = rc.s[nz] * F0[c];
#pragma unroll
                    for (int m = 0; m < 7; ++m) av = fma(rc.B[nz][m], D[m][c], av);
                    V[c] = fma(h, av, v0[c]);
                }
            } else {
                V[0] = v0[0]; V[1] = v0[1]; V[2] = v0[2];
            }
            double F[3];
            accel(ephW + n * E.n_body * 6, E, X, V, F);
#pragma unroll
            for (int c = 0; c < 3; ++c) D[n - 1][c] = F[c] - F0[c];
        }
        double db = 0.0, fm = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double b = 0.0;
#pragma unroll
            for (int m = 0; m < 7; ++m) b = fma(rc.E6[m + z], D[m][c], b);
            db = fmax(db, fabs(b - b6[c]));
            b6[c] = b;
            fm = fmax(fm, fabs(D[6][c] + F0[c]));
        }
        const double lpc = (active && fm > 0.0) ? db / fm : 0.0;
        pc = wave_max(lpc);
        lane_iters += __popcll(__ballot(active));
    } while (!(pc < 1e-16) && !(it > 2 && pcl <= pc) && it < max_iter);
    return it;
}

// ---------------------------------------------------------------- 8 lanes per body
// A body can be spread over an 8-lane group: lane k of the group owns
// collocation node k + 1 (lane 7 repeats node 7), every lane keeps the
// body's state and all seven increments, and one corrector sweep updates
// all nodes at once from the previous sweep's increments (a Jacobi sweep
// of the same fixed-point map, converging to the same collocation
// solution).
constexpr int kGroup = 8;

// Lanes of a wavefront by body.  With G = 8 a wavefront holds 8 bodies,
// lanes 8g..8g+7 for body g.  With G = 7 it holds 9: lanes 7g..7g+6 for
// body g, and lane 63 joins body 8 as its eighth lane.  In both layouts
// lane gl = 7 of a group repeats node 7, so every node has exactly one
// owning lane and the code below needs no other distinction.
template <int G>
struct GroupMap {
    static_assert(G == 7 || G == 8, "7 or 8 lanes per body");
    static constexpr int kBodies = G == 8 ? 8 : 9;   // bodies per wavefront
    int grp, gl;
    __device__ __forceinline__ explicit GroupMap(int lane) {
        if constexpr (G == 8) {
            grp = lane >> 3;
            gl = lane & 7;
        } else {
            grp = lane < 63 ? lane / 7 : 8;
            gl = lane - 7 * grp;
        }
    }
};
constexpr int kMaxGroups = 9;

// Constants of one node, held in registers by the lane that owns it.
struct NodeRow {
    double s, hs2, A[7], B[7];
    double pad_[2];       // 144-byte rows: the 8 rows start in distinct LDS banks
};

// Row n (lane-varying, 1..7) selected from uniform constants without any
// lane-indexed memory access.
__device__ __forceinline__ void load_node_row(const RadauConst& rc, int n, NodeRow& r) {
    r.s = 0.0; r.hs2 = 0.0;
#pragma unroll
    for (int m = 0; m < 7; ++m) { r.A[m] = 0.0; r.B[m] = 0.0; }
#pragma unroll
    for (int k = 1; k <= 7; ++k) {
        const bool me = (n == k);
        r.s = me ? rc.s[k] : r.s;
        r.hs2 = me ? rc.half_s2[k] : r.hs2;
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            r.A[m] = me ? rc.A[k][m] : r.A[m];
            r.B[m] = me ? rc.B[k][m] : r.B[m];
        }
    }
}

// Wave-wide reductions of values that are equal within each group, as a
// butterfly of lane permutations that stay in the vector unit: DPP quad
// permutes (lanes xor 1, xor 2), the half-row and row mirrors (lane i with
// 7 - i, with 15 - i) and the row-pair and half-wave swaps (xor 16, xor
// 32).  Aligned 8-lane groups need only the last three steps.
struct PermDouble {
    unsigned lo, hi;
};
__device__ __forceinline__ PermDouble split_double(double x) {
    const unsigned long long u = __double_as_longlong(x);
    return PermDouble{(unsigned)u, (unsigned)(u >> 32)};
}
__device__ __forceinline__ double join_double(unsigned lo, unsigned hi) {
    return __longlong_as_double(((long long)hi << 32) | lo);
}
template <int CTRL>
__device__ __forceinline__ double dpp_double(double x) {
    const PermDouble d = split_double(x);
    return join_double((unsigned)__builtin_amdgcn_update_dpp(0, (int)d.lo, CTRL, 0xF, 0xF, false),
                       (unsigned)__builtin_amdgcn_update_dpp(0, (int)d.hi, CTRL, 0xF, 0xF, false));
}
// the other operand of a max/min step across rows (xor 16) and halves (xor 32)
__device__ __forceinline__ double swap16_double(double x) {
    const PermDouble d = split_double(x);
    const auto lo = __builtin_amdgcn_permlane16_swap(d.lo, d.lo, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(d.hi, d.hi, false, false);
    // both results hold each lane's own value in one and its xor-16 partner in the other
    const double a = join_double(lo[0], hi[0]), b = join_double(lo[1], hi[1]);
    return ((threadIdx.x >> 4) & 1) ? a : b;
}
__device__ __forceinline__ double swap32_double(double x) {
    const PermDouble d = split_double(x);
    const auto lo = __builtin_amdgcn_permlane32_swap(d.lo, d.lo, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(d.hi, d.hi, false, false);
    const double a = join_double(lo[0], hi[0]), b = join_double(lo[1], hi[1]);
    return ((threadIdx.x >> 5) & 1) ? a : b;
}
template <int G = kGroup, bool MAX = true>
__device__ __forceinline__ double groups_reduce(double x) {
    auto op = [](double a, double b) { return MAX ? fmax(a, b) : fmin(a, b); };
    if constexpr (G != 8) {
        x = op(x, dpp_double<0xB1>(x));      // lane xor 1
        x = op(x, dpp_double<0x4E>(x));      // lane xor 2
        x = op(x, dpp_double<0x141>(x));     // 7 - lane within 8
    }
    x = op(x, dpp_double<0x140>(x));         // 15 - lane within 16
    x = op(x, swap16_double(x));
    x = op(x, swap32_double(x));
    return uniform(x);
}
template <int G = kGroup>
__device__ __forceinline__ double groups_max(double x) { return groups_reduce<G, true>(x); }
template <int G = kGroup>
__device__ __forceinline__ double groups_min(double x) { return groups_reduce<G, false>(x); }

// Perturber table of the grouped integrator: per node and slot 8 doubles
// (x, y, z, GM, vx, vy, vz, GM/c^2).  GM values are written once per
// launch (g8_table_init); node_ephemeris8 fills positions, and velocities
// only for the slots that carry the Eq. A.3 term.
constexpr int kSlot = 8;
// Doubles per node row: 4 (4 n_body + 1) dwords, so the 8 rows read
// together by an 8-lane group fall in distinct LDS banks.
__host__ __device__ inline int g8_row(int n_body) { return n_body * kSlot + 2; }

// Exchange rows of the grouped corrector, after the wave's node table:
// per group three rows (x, y, z) of 8 doubles, lane gl writing column gl,
// padded to 26 doubles so that the 16-byte reads of the groups of a
// wavefront fall in distinct LDS banks.
constexpr int kXchGroup = 26;
// Doubles of LDS per wavefront: node table plus exchange rows.
__host__ __device__ inline int g8_wave_doubles(int n_body) {
    return kNodes * g8_row(n_body) + kMaxGroups * kXchGroup;
}
__device__ __forceinline__ double* g8_xch(double* e8, int n_body, int grp) {
    return e8 + kNodes * g8_row(n_body) + grp * kXchGroup;
}

// Publish this lane's increment dn (node gl + 1) and read the increments
// D[m] of nodes m + 1 = 1..7 of the group.  Every lane of the wavefront
// takes part.
__device__ __forceinline__ void g8_exchange(double* __restrict__ xg, int gl, const double dn[3], double D[7][3]) {
    wave_lds_sync();                        // earlier reads of the rows are done
    xg[gl] = dn[0];
    xg[8 + gl] = dn[1];
    xg[16 + gl] = dn[2];
    wave_lds_sync();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double2 v = *reinterpret_cast<const double2*>(xg + 8 * c + 2 * k);
            D[2 * k][c] = v.x;
            if (2 * k + 1 < 7) D[2 * k + 1][c] = v.y;
        }
    }
}

__device__ __forceinline__ void g8_table_init(const EphemArgs& E, int lane, double* __restrict__ e8) {
    for (int b = 0; b < E.n_body; ++b) {
        const int sl = body_slot(E, b);
        for (int n = lane; n < kNodes; n += kWave) {
            e8[n * g8_row(E.n_body) + sl * kSlot + 3] = E.gm[b];
            e8[n * g8_row(E.n_body) + sl * kSlot + 7] = E.kgr[b];
        }
    }
}

// Perturber states at the node times of a step.  Lane k of each 8-lane
// group takes node (k & 7) + 1 (node 8 is the step end) and finds that
// node's segment and tau once; the 3 n_body coordinates are spread over
// the 8 groups (group g takes coordinates g, g + 8, ...).  Coordinates of
// the slots with the Eq. A.3 term come first and also get the velocity
// (derivative chain); a pass holding any of them evaluates derivatives in
// every lane so the wavefront does not diverge.  Node 0 (the step start,
// needed before the first step or when the caller asks) takes one more
// pass with coordinate = lane.  The node of a lane here follows lane & 7
// whatever the lane's body group.
template <int NB, int NGR, int DEG1>
__device__ __forceinline__ void node_ephemeris8(const double* __restrict__ coefL, int bstride, const EphemArgs& E,
                                                const RadauConst& rc, int seg_lo, int seg_hi, double t, double h,
                                                double t_end, bool node0, int lane, double* __restrict__ e8) {
    const int nb = NB > 0 ? NB : E.n_body;
    const int ngr = NB > 0 ? NGR : E.n_gr;
    const int deg1 = DEG1 > 0 ? DEG1 : E.deg1;
    const int cps = 3 * deg1, nc = 3 * nb, ngc = 3 * ngr;
    const double sc = 2.0 * E.inv_seg;
    auto chains = [&](int n, double tt, int c0, int cstep, int npass) {
        const int k = seg_index(tt, E.t_start, E.inv_seg, seg_lo, seg_hi);
        const double tau = 2.0 * (tt - (E.t_start + (double)k * E.seg_days)) * E.inv_seg - 1.0;
        const double* cb = coefL + (k - seg_lo) * cps;
        double* row = e8 + n * g8_row(nb);
        // one chain in flight per lane: the coefficient loads of several
        // unrolled passes would crowd out the integrator state
#pragma unroll 1
        for (int j = 0; j < npass; ++j) {
            const int c = c0 + cstep * j;
            if (c >= nc) continue;
            const int sl = c / 3, i = c - 3 * sl;
            const double* cp = cb + slot_body(E, sl) * bstride + i * deg1;
            if (cstep * j < ngc) {                 // wave-uniform: the pass holds derivative chains
                double pv, dv;
                clenshaw_n<DEG1>(cp, deg1, tau, pv, dv);
                row[sl * kSlot + i] = pv;
                if (c < ngc) row[sl * kSlot + 4 + i] = dv * sc;
            } else {
                row[sl * kSlot + i] = clenshaw_value_n<DEG1>(cp, deg1, tau);
            }
        }
    };
    const int nl = lane & (kGroup - 1);
    chains(nl + 1, nl == kGroup - 1 ? t_end : t + rc.s[nl + 1] * h, lane / kGroup, kGroup, (nc + kGroup - 1) / kGroup);
    if (node0) chains(0, t, lane, kWave, 1);
    wave_lds_sync();
}

// 1/sqrt(x) for a positive normal x: the hardware estimate y0 times the
// series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + O(e^3), e = 1 - x y0^2.  The
// truncation leaves a relative error of about 5e^3/16, below an ulp when
// the estimate is good to 2^-19.  No special-value handling: a zero or
// non-finite x gives a non-finite result, reported as a failed body.
__device__ __forceinline__ double rsqrt_pos(double x) {
    const double y0 = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y0, y0, 1.0);
    return fma(y0 * e, fma(e, 0.375, 0.5), y0);
}

// Force of Eqs. A.1 + A.3 + A.4 from the grouped table e8 (one node):
// slots below NGR carry the Eq. A.3 term, the J2 bodies (found by slot)
// the Eq. A.4 term.  NB = 0 takes the counts at run time.
template <int NB, int NGR>
__device__ __forceinline__ void accel8(const double* __restrict__ e8, const EphemArgs& E, const double X[3],
                                       const double V[3], double F[3]) {
    const int nb = NB > 0 ? NB : E.n_body;
    const int ngr = NB > 0 ? NGR : E.n_gr;
    double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
    for (int b = 0; b < (NB > 0 ? NGR : KETE_MAX_BODIES); ++b) {
        if (NB == 0 && b >= ngr) break;
        const double* pb = e8 + kSlot * b;
        const double2 pxy = *reinterpret_cast<const double2*>(pb);
        const double2 pzg = *reinterpret_cast<const double2*>(pb + 2);
        const double2 vxy = *reinterpret_cast<const double2*>(pb + 4);
        const double2 vzk = *reinterpret_cast<const double2*>(pb + 6);
        const double rx = X[0] - pxy.x, ry = X[1] - pxy.y, rz = X[2] - pzg.x;
        const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
        const double ir = rsqrt_pos(r2);
        const double ir3 = ir * ir * ir;
        const double gm = pzg.y;
        const double wx = V[0] - vxy.x, wy = V[1] - vxy.y, wz = V[2] - vzk.x;
        const double w2 = fma(wx, wx, fma(wy, wy, wz * wz));
        const double rw = fma(rx, wx, fma(ry, wy, rz * wz));
        const double g = vzk.y * ir3;
        const double f = fma(g, 4.0 * gm * ir - w2, -gm * ir3);
        const double q = 4.0 * g * rw;
        ax = fma(q, wx, ax); ay = fma(q, wy, ay); az = fma(q, wz, az);
        ax = fma(f, rx, ax); ay = fma(f, ry, ay); az = fma(f, rz, az);
    }
#pragma unroll
    for (int b = (NB > 0 ? NGR : 0); b < (NB > 0 ? NB : KETE_MAX_BODIES); ++b) {
        if (NB == 0 && b >= nb - ngr) break;
        const double* pb = e8 + kSlot * (NB > 0 ? b : b + ngr);
        const double2 pxy = *reinterpret_cast<const double2*>(pb);
        const double2 pzg = *reinterpret_cast<const double2*>(pb + 2);
        const double rx = X[0] - pxy.x, ry = X[1] - pxy.y, rz = X[2] - pzg.x;
        const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
        const double ir = rsqrt_pos(r2);
        const double f = -pzg.y * (ir * ir * ir);
        ax = fma(f, rx, ax); ay = fma(f, ry, ay); az = fma(f, rz, az);
    }
    F[0] = ax; F[1] = ay; F[2] = az;
    for (int q = 0; q < E.n_j2; ++q) {
        const double* pb = e8 + kSlot * E.j2_slot[q];
        const double d[3] = {X[0] - pb[0], X[1] - pb[1], X[2] - pb[2]};
        j2_add(E, q, d, rsqrt_pos(fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2]))), F);
    }
}

// The same force computed by a group together: node lane gl < 7 takes
// slots gl, gl + 7, ...; the partial sums meet in the group's exchange
// rows xg and every lane adds them in the same order, so all lanes of the
// group return the same total.  The whole wavefront takes part.
__device__ __forceinline__ void accel8_group(const double* __restrict__ e8, const EphemArgs& E, const double X[3],
                                             const double V[3], int gl, double* __restrict__ xg, double F[3]) {
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int sl = gl; gl < 7 && sl < E.n_body; sl += 7) {
        const double* pb = e8 + kSlot * sl;
        const double2 pxy = *reinterpret_cast<const double2*>(pb);
        const double2 pzg = *reinterpret_cast<const double2*>(pb + 2);
        const double rx = X[0] - pxy.x, ry = X[1] - pxy.y, rz = X[2] - pzg.x;
        const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
        const double ir = rsqrt_pos(r2);
        const double ir3 = ir * ir * ir;
        const double gm = pzg.y;
        double f = -gm * ir3;
        if (sl < E.n_gr) {
            const double2 vxy = *reinterpret_cast<const double2*>(pb + 4);
            const double2 vzk = *reinterpret_cast<const double2*>(pb + 6);
            const double wx = V[0] - vxy.x, wy = V[1] - vxy.y, wz = V[2] - vzk.x;
            const double w2 = fma(wx, wx, fma(wy, wy, wz * wz));
            const double rw = fma(rx, wx, fma(ry, wy, rz * wz));
            const double g = vzk.y * ir3;
            f = fma(g, 4.0 * gm * ir - w2, f);
            const double q = 4.0 * g * rw;
            ax = fma(q, wx, ax); ay = fma(q, wy, ay); az = fma(q, wz, az);
        }
        ax = fma(f, rx, ax); ay = fma(f, ry, ay); az = fma(f, rz, az);
    }
    double part[3] = {ax, ay, az};
    if (gl < E.n_j2) {                         // node lane q takes J2 body q
        const double* pb = e8 + kSlot * E.j2_slot[gl];
        const double d[3] = {X[0] - pb[0], X[1] - pb[1], X[2] - pb[2]};
        j2_add(E, gl, d, rsqrt_pos(fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2]))), part);
    }
    double D[7][3];
    g8_exchange(xg, gl, part, D);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double f = D[0][c];
#pragma unroll
        for (int m = 1; m < 7; ++m) f += D[m][c];
        F[c] = f;
    }
}

// Jacobians Jx = da/dx, Jv = da/dv (row-major 3x3) from the grouped
// table e8 (one node) of the force of accel8, Eq. A.4 included.  The Newtonian part is
// symmetric and accumulated once per pair (i <= j); the Eq. A.3 part,
// with P = s1 r + 4 (r.w) w and s1 = 4 mu / r - w^2, is
//   Jx += k [(-3 P / r^5 - 4 mu r / r^6) r^T + 4 w w^T / r^3 + s1 I / r^3]
//   Jv += k / r^3 [-2 r w^T + 4 w r^T + 4 (r.w) I].
// NB = 0 takes the counts at run time.
template <int NB, int NGR>
__device__ __forceinline__ void accel_jac8(const double* __restrict__ e8, const EphemArgs& E, const double X[3],
                                           const double V[3], double Jx[9], double Jv[9]) {
    const int nb = NB > 0 ? NB : E.n_body;
    const int ngr = NB > 0 ? NGR : E.n_gr;
    double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // xx xy xz yy yz zz
    double dg = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) { Jx[i] = 0.0; Jv[i] = 0.0; }
#pragma unroll
    for (int sl = 0; sl < (NB > 0 ? NB : KETE_MAX_BODIES); ++sl) {
        if (NB == 0 && sl >= nb) break;
        const double* pb = e8 + kSlot * sl;
        const double2 pxy = *reinterpret_cast<const double2*>(pb);
        const double2 pzg = *reinterpret_cast<const double2*>(pb + 2);
        const double r[3] = {X[0] - pxy.x, X[1] - pxy.y, X[2] - pzg.x};
        const double r2 = fma(r[0], r[0], fma(r[1], r[1], r[2] * r[2]));
        const double ir = rsqrt_pos(r2);
        const double ir2 = ir * ir, ir3 = ir2 * ir, ir5 = ir3 * ir2;
        const double gm = pzg.y;
        const double sN = 3.0 * gm * ir5;
        const double a[3] = {sN * r[0], sN * r[1], sN * r[2]};
        S[0] = fma(a[0], r[0], S[0]); S[1] = fma(a[0], r[1], S[1]); S[2] = fma(a[0], r[2], S[2]);
        S[3] = fma(a[1], r[1], S[3]); S[4] = fma(a[1], r[2], S[4]); S[5] = fma(a[2], r[2], S[5]);
        dg = fma(-gm, ir3, dg);
        if (sl < ngr) {
            const double2 vxy = *reinterpret_cast<const double2*>(pb + 4);
            const double2 vzk = *reinterpret_cast<const double2*>(pb + 6);
            const double k = vzk.y;
            const double w[3] = {V[0] - vxy.x, V[1] - vxy.y, V[2] - vzk.x};
            const double w2 = fma(w[0], w[0], fma(w[1], w[1], w[2] * w[2]));
            const double rw = fma(r[0], w[0], fma(r[1], w[1], r[2] * w[2]));
            const double s1 = 4.0 * gm * ir - w2;
            const double kr3 = k * ir3;
            const double c1 = -3.0 * k * ir5, c2 = -4.0 * k * gm * ir3 * ir3, c4 = 4.0 * kr3;
            double u[3], v[3], pr[3], qw[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double P = fma(s1, r[i], 4.0 * rw * w[i]);
                u[i] = fma(c1, P, c2 * r[i]);
                v[i] = c4 * w[i];
                pr[i] = -2.0 * kr3 * r[i];
                qw[i] = c4 * w[i];
            }
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    Jx[3 * i + j] = fma(u[i], r[j], fma(v[i], w[j], Jx[3 * i + j]));
                    Jv[3 * i + j] = fma(pr[i], w[j], fma(qw[i], r[j], Jv[3 * i + j]));
                }
            const double dx = kr3 * s1, dv = c4 * rw;
            Jx[0] += dx; Jx[4] += dx; Jx[8] += dx;
            Jv[0] += dv; Jv[4] += dv; Jv[8] += dv;
        }
    }
    Jx[0] += S[0] + dg; Jx[1] += S[1]; Jx[2] += S[2];
    Jx[3] += S[1]; Jx[4] += S[3] + dg; Jx[5] += S[4];
    Jx[6] += S[2]; Jx[7] += S[4]; Jx[8] += S[5] + dg;
    for (int q = 0; q < E.n_j2; ++q) {
        const double* pb = e8 + kSlot * E.j2_slot[q];
        const double d[3] = {X[0] - pb[0], X[1] - pb[1], X[2] - pb[2]};
        j2_jac_add(E, q, d, rsqrt_pos(fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2]))), Jx);
    }
}

// Step-size factor (eps / e)^(1/7) of the IAS15 control, in single
// precision: the factor only sets the next trial step.
__device__ __forceinline__ double step_factor(double q) {
    const float qf = (float)fmin(fmax(q, 1e-35), 1e35);
    return (double)exp2f(log2f(qf) * (1.0f / 7.0f));
}

// Starting increment of this lane's node for a step q times the previous
// accepted one: that step's collocation polynomial of the force
// increments (values Dp at its nodes, 0 at its start) evaluated at the new
// node's time sig = 1 + q s_n of the old step, less its value at sig = 1.
// The Lagrange basis of the 8 nodes is formed from prefix and suffix
// products of (sig - s_k).  With RELOAD the constants are read through an
// opaque zero offset, so they are loaded here rather than kept in scalar
// registers across the step loop.
template <bool RELOAD>
__device__ __forceinline__ void extrapolate_increment(const RadauConst& rc, double* __restrict__ xg, int gl,
                                                      const NodeRow& R, const double Dp[3], double q, double dn[3]) {
    int z = 0;
    if constexpr (RELOAD) asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    double D[7][3];
    g8_exchange(xg, gl, Dp, D);
    const double sig = fma(q, R.s, 1.0);
    double dk[8], pre[8];
    dk[0] = sig;
#pragma unroll
    for (int k = 1; k < 8; ++k) dk[k] = sig - rc.s[k + z];
    pre[0] = 1.0;
#pragma unroll
    for (int k = 1; k < 8; ++k) pre[k] = pre[k - 1] * dk[k - 1];
    double suf = 1.0;
    dn[0] = dn[1] = dn[2] = 0.0;
#pragma unroll
    for (int m = 7; m >= 1; --m) {
        const double w = fma(pre[m] * suf, rc.Lden[m - 1 + z], -rc.L1[m - 1 + z]);
#pragma unroll
        for (int c = 0; c < 3; ++c) dn[c] = fma(w, D[m - 1][c], dn[c]);
        suf *= dk[m];
    }
}

// Corrector for a body spread over an 8-lane group (see above), with the
// same stopping rule as corrector().  Each lane keeps only its own node's
// increment dn; the other nodes' increments are read from the group's
// lanes when the predictor sums and b6 are formed.  With q > 0 the
// iteration starts from the previous step's increments Dp extrapolated
// (extrapolate_increment), otherwise from zero.  On return dn holds the
// converged increment of this lane's node, b6 the highest coefficient and
// d6 the increment of node 7 (all lanes).
template <int NB, int NGR, int G, bool RELOAD = true>
__device__ __forceinline__ int corrector_g8(const RadauConst& rc, const EphemArgs& E, const double* __restrict__ e8,
                                            double* __restrict__ xg, int gl, const NodeRow& R, int node,
                                            const double x0[3], const double v0[3],
                                            const double F0[3], double h, bool active, int max_iter, double dn[3],
                                            double b6[3], double d6[3], const double* Dp = nullptr,
                                            double q = 0.0) {
    const double hh = h * h, sh = R.s * h;
    const double* en = e8 + node * g8_row(E.n_body);
    const bool started = q > 0.0;           // wave-uniform
    if (started) extrapolate_increment<RELOAD>(rc, xg, gl, R, Dp, q, dn);
    else dn[0] = dn[1] = dn[2] = 0.0;
    b6[0] = b6[1] = b6[2] = 0.0;
    d6[0] = d6[1] = d6[2] = 0.0;
    double pc = 1e300;
    int it = 0;
    for (;;) {
        double ax[3], av[3], bb[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) { ax[c] = R.hs2 * F0[c]; av[c] = R.s * F0[c]; bb[c] = 0.0; }
        if (it > 0 || started) {
            double D[7][3];
            g8_exchange(xg, gl, dn, D);
#pragma unroll
            for (int m = 0; m < 7; ++m) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double d = D[m][c];
                    ax[c] = fma(R.A[m], d, ax[c]);
                    av[c] = fma(R.B[m], d, av[c]);
                    bb[c] = fma(rc.E6[m], d, bb[c]);
                    if (m == 6) d6[c] = d;
                }
            }
            const double pcl = pc;
            double db = 0.0, fm = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                db = fmax(db, fabs(bb[c] - b6[c]));
                b6[c] = bb[c];
                fm = fmax(fm, fabs(d6[c] + F0[c]));
            }
            // the ratio only steers the stopping rule: the reciprocal estimate suffices
            const double lpc = (active && fm > 0.0) ? db * __builtin_amdgcn_rcp(fm) : 0.0;
            pc = groups_max<G>(lpc);
            if (it > 0 && (pc < 1e-16 || (it > 2 && pcl <= pc) || it >= max_iter)) break;
        }
        ++it;
        double X[3], V[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) X[c] = fma(hh, ax[c], fma(sh, v0[c], x0[c]));
        if (NB > 0 ? NGR > 0 : E.has_gr) {
#pragma unroll
            for (int c = 0; c < 3; ++c) V[c] = fma(h, av[c], v0[c]);
        } else {
            V[0] = v0[0]; V[1] = v0[1]; V[2] = v0[2];
        }
        double F[3];
        accel8<NB, NGR>(en, E, X, V, F);
#pragma unroll
        for (int c = 0; c < 3; ++c) dn[c] = F[c] - F0[c];
    }
    return it;
}

// Step end of a group-integrated body from the converged increments.
__device__ __forceinline__ void step_end_g8(const RadauConst& rc, double* __restrict__ xg, int gl, const double dn[3],
                                            double h, double x0[3], double v0[3], const double F0[3]) {
    double ax[3], av[3];
    double D[7][3];
    g8_exchange(xg, gl, dn, D);
    // opaque zero row offset: the constants are loaded where used instead
    // of being held in (spilled) scalar registers for the whole kernel
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
#pragma unroll
    for (int c = 0; c < 3; ++c) { ax[c] = rc.half_s2[8 + z] * F0[c]; av[c] = F0[c]; }
#pragma unroll
    for (int m = 0; m < 7; ++m) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double d = D[m][c];
            ax[c] = fma(rc.A[8 + z][m], d, ax[c]);
            av[c] = fma(rc.B[8 + z][m], d, av[c]);
        }
    }
    const double hh = h * h;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x0[c] = fma(hh, ax[c], fma(h, v0[c], x0[c]));
        v0[c] = fma(h, av[c], v0[c]);
    }
}

// Stepping state of a group-integrated body (replicated in its 8 lanes).
struct G8State {
    double x0[3], v0[3], F0[3];
    double Dp[3] = {0.0, 0.0, 0.0};   // this lane's increment in the last accepted step
    double hprev = 0.0;               // that step (0: none yet)
    double t, hw, hp_new;
    bool active, haveF0;
    bool row0 = false;          // table row 0 holds the perturbers at t (node 0)
    int status;
};
struct G8Count {
    unsigned long long steps = 0, iter = 0, rej = 0, lsteps = 0, liter = 0, chain = 0, vchain = 0, lpred = 0;
};

// Largest ratio of a step to the previous accepted one for which the
// corrector starts from the extrapolated increments.
constexpr double kPredMaxRatio = 3.0;

// Corrector start of g8_integrate: always from zero, or extrapolated from
// the previous step (constants reloaded at each use, or held in registers
// where the kernel has room).
enum G8Start { kStartZero = 0, kStartExtrapolate = 1, kStartExtrapolateHeld = 2 };

// Integrate one window [S.t, tb] whose Chebyshev segments seg_lo..seg_hi
// are staged at coefL, with wave-shared adaptive steps (the 8 bodies of
// the wavefront take the smallest step any of them asks for).
struct G8NoVisit {
    template <class... A>
    __device__ __forceinline__ void operator()(A&&...) const {}
};

// visit(ts, h, dn, S) is called by every lane after each accepted step,
// before S moves to the step end (dn: this lane's converged increment,
// e8: the step's perturber table).  With need_node0 the table also holds
// node 0 (the step start) on every step.
template <int NB, int NGR, int DEG1, int G, int START = kStartZero, class Params, class Visit = G8NoVisit>
__device__ __forceinline__ void g8_integrate(const Params& p, const NodeRow& R, int node, int gl, int grp, int lane,
                                             const double* __restrict__ coefL, int bstride, double* __restrict__ e8,
                                             int seg_lo, int seg_hi, double tb, G8State& S, G8Count& C,
                                             Visit&& visit = Visit(), bool need_node0 = false,
                                             double t_stop = kInf) {
    const EphemArgs& E = p.eph;
    const RadauConst& rc = p.rc;
    const int nb = E.n_body;
    double* xg = g8_xch(e8, nb, grp);
    if (__ballot(S.active) == 0ull) { S.t = tb; return; }
    while (S.t != tb) {
        if (S.t >= t_stop) return;          // a recompute ends where the recorded run took its checkpoint
        const double dir = tb > S.t ? 1.0 : -1.0;
        double hmag = S.hw;
        if (p.h_max > 0.0 && hmag > p.h_max) hmag = p.h_max;
        double h = dir * hmag;
        bool landed = false;
        if (fabs(h) >= fabs(tb - S.t)) { h = tb - S.t; landed = true; }
        if ((long)C.steps >= p.max_steps) {
            if (S.active) { S.status = KETE_ST_MAX_STEPS; S.active = false; }
            S.t = tb;
            return;
        }
        const double t_end = landed ? tb : S.t + h;
        // node 0 is evaluated before the first step; with need_node0 it is
        // afterwards the previous step's end row, copied when that step is accepted
        const int n0 = (S.haveF0 && (!need_node0 || S.row0)) ? 1 : 0;
        node_ephemeris8<NB, NGR, DEG1>(coefL, bstride, E, rc, seg_lo, seg_hi, S.t, h, t_end, n0 == 0, lane, e8);
        S.row0 = true;
        C.chain += (kNodes - n0) * E.n_gr * 3;
        C.vchain += (kNodes - n0) * (nb - E.n_gr) * 3;
        if (!S.haveF0) { accel8<NB, NGR>(e8, E, S.x0, S.v0, S.F0); S.haveF0 = true; }

        double q = 0.0;                       // wave-uniform, like h and S.hprev
        if constexpr (START != kStartZero) {
            if (!p.zero_start && S.hprev != 0.0) q = h / S.hprev;
            if (!(q <= kPredMaxRatio)) q = 0.0;
        }
        double dn[3], b6p[3], d6[3];
        const int it = corrector_g8<NB, NGR, G, START != kStartExtrapolateHeld>(rc, E, e8, xg, gl, R, node, S.x0, S.v0,
                                                                                S.F0, h, S.active, p.max_iter, dn, b6p,
                                                                                d6, S.Dp, q);
        C.iter += it;
        const unsigned long long n_act = __popcll(__ballot(S.active && gl == 0));
        C.liter += (unsigned long long)it * n_act;
        if (q > 0.0) C.lpred += n_act;

        double fm = 0.0, bm = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) { fm = fmax(fm, fabs(d6[c] + S.F0[c])); bm = fmax(bm, fabs(b6p[c])); }
        const double ebl = fm > 0.0 ? bm / fm : 0.0;
        double hl = (ebl > 0.0 && ebl < kInf) ? fabs(h) * step_factor(p.eps / ebl) : fabs(h) / p.safety;
        if (!S.active) hl = kInf;
        if (S.active && hl < p.h_min) { S.status = KETE_ST_STEP_UNDERFLOW; S.active = false; hl = kInf; }
        const double hn = groups_min<G>(hl);
        if (!(hn < kInf)) { S.t = tb; return; }
        if (hn < p.safety * fabs(h)) {       // reject and retry from the same state
            S.hw = hn;
            ++C.rej;
            continue;
        }
        visit(S.t, h, dn, S);
        if constexpr (START != kStartZero) {
#pragma unroll
            for (int c = 0; c < 3; ++c) S.Dp[c] = dn[c];
            S.hprev = h;
        }
        step_end_g8(rc, xg, gl, dn, h, S.x0, S.v0, S.F0);
        S.t = t_end;
        ++C.steps;
        C.lsteps += n_act;
        if (S.active && !(isfinite(S.x0[0]) && isfinite(S.x0[1]) && isfinite(S.x0[2]) && isfinite(S.v0[0]) &&
                          isfinite(S.v0[1]) && isfinite(S.v0[2]))) {
            S.status = KETE_ST_NONFINITE; S.active = false;
        }
        accel8_group(e8 + 8 * g8_row(nb), E, S.x0, S.v0, gl, xg, S.F0);
        if (need_node0) {
            wave_lds_sync();
            for (int i = lane; i < g8_row(nb); i += kWave) e8[i] = e8[8 * g8_row(nb) + i];
            wave_lds_sync();
        }
        if (landed) {
            S.hw = fmin(S.hw, hn);
        } else {
            S.hw = fmin(hn, fabs(h) / p.safety);
            S.hp_new = fmin(S.hp_new, fmin(hl, fabs(h) / p.safety));
        }
    }
}

// Component gl (0..5) of a state.
__device__ __forceinline__ double state_component(const double x0[3], const double v0[3], int gl) {
    return gl == 0 ? x0[0] : gl == 1 ? x0[1] : gl == 2 ? x0[2] : gl == 3 ? v0[0] : gl == 4 ? v0[1] : v0[2];
}

// Collocation polynomial at fraction sig of the step (sig = 1: step end),
// from the monomial weights alpha_m(sig) = sum_k Ap[m][k] sig^(k+2) and
// beta_m(sig) = sum_k Bp[m][k] sig^(k+1) (m = 1..7, k = 0..7).
__device__ __forceinline__ void dense_weights(const RadauConst& rc, double sig, double al[7], double be[7]) {
    // opaque zero row offset: the 112 constants are loaded where used
    // rather than held in registers across the caller's loops
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        double a = rc.Ap[m + z][7], b = rc.Bp[m + z][7];
#pragma unroll
        for (int k = 6; k >= 0; --k) { a = fma(a, sig, rc.Ap[m + z][k]); b = fma(b, sig, rc.Bp[m + z][k]); }
        al[m] = a * sig * sig;
        be[m] = b * sig;
    }
}

__device__ __forceinline__ void dense_state(const RadauConst& rc, const double x0[3], const double v0[3],
                                            const double F0[3], const double D[7][3], double h, double sig,
                                            double X[3], double V[3]) {
    double al[7], be[7];
    dense_weights(rc, sig, al, be);
    const double hh = h * h;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double ax = 0.5 * sig * sig * F0[c], av = sig * F0[c];
#pragma unroll
        for (int m = 0; m < 7; ++m) { ax = fma(al[m], D[m][c], ax); av = fma(be[m], D[m][c], av); }
        X[c] = fma(hh, ax, fma(sig * h, v0[c], x0[c]));
        V[c] = fma(h, av, v0[c]);
    }
}

// dense_state with the monomial rows read from a copy in LDS (cw: Ap[7][8]
// then Bp[7][8]) rather than from the kernel's argument block, and the
// step's node increments from the group's exchange rows xg (component c of
// node m + 1 at xg[8 c + m]), one node at a time; sig may differ between
// groups.
__device__ __forceinline__ void dense_state_rows(const double* __restrict__ cw, const double* __restrict__ xg,
                                                 const double x0[3], const double v0[3], const double F0[3],
                                                 double h, double sig, double X[3], double V[3]) {
    double ax[3], av[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) { ax[c] = 0.5 * sig * sig * F0[c]; av[c] = sig * F0[c]; }
#pragma unroll 1
    for (int m = 0; m < 7; ++m) {
        const double* am = cw + 8 * m;
        const double* bm = cw + 56 + 8 * m;
        double a = am[7], b = bm[7];
#pragma unroll
        for (int k = 6; k >= 0; --k) { a = fma(a, sig, am[k]); b = fma(b, sig, bm[k]); }
        a *= sig * sig;
        b *= sig;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double d = xg[8 * c + m];
            ax[c] = fma(a, d, ax[c]);
            av[c] = fma(b, d, av[c]);
        }
    }
    const double hh = h * h;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        X[c] = fma(hh, ax[c], fma(sig * h, v0[c], x0[c]));
        V[c] = fma(h, av[c], v0[c]);
    }
}

// Dense output at fraction sig of a step, in two parts.  The 14 weights
// alpha_m(sig) = sum_k Ap[m][k] sig^(k+2) and beta_m(sig) = sum_k Bp[m][k]
// sig^(k+1) are the same for every object of a wavefront (they share the
// step), so lanes 0..13 evaluate one each from the monomial rows in LDS
// (cw: Ap[7][8] then Bp[7][8]) into the wavefront's slots wt[14]; then
// each lane forms its object's state from the weights and the step's node
// increments in the group's exchange rows xg (component c
// of node m + 1 at xg[8 c + m]) in dense_state_wave.  The first call is
// made by the whole wavefront.
__device__ __forceinline__ void dense_weights_wave(const double* __restrict__ cw, double sig, int lane,
                                                   double* __restrict__ wt) {
    wave_lds_sync();                        // earlier reads of wt are done
    if (lane < 14) {
        const double* pm = cw + 8 * lane;
        double w = pm[7];
#pragma unroll
        for (int k = 6; k >= 0; --k) w = fma(w, sig, pm[k]);
        wt[lane] = w * (lane < 7 ? sig * sig : sig);
    }
    wave_lds_sync();
}
__device__ __forceinline__ void dense_state_wave(const double* __restrict__ wt, const double* __restrict__ xg,
                                                 const double x0[3], const double v0[3], const double F0[3],
                                                 double h, double sig, double X[3], double V[3]) {
    double ax[3], av[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) { ax[c] = 0.5 * sig * sig * F0[c]; av[c] = sig * F0[c]; }
#pragma unroll 1
    for (int m = 0; m < 7; ++m) {
        const double a = wt[m], b = wt[7 + m];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double d = xg[8 * c + m];
            ax[c] = fma(a, d, ax[c]);
            av[c] = fma(b, d, av[c]);
        }
    }
    const double hh = h * h;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        X[c] = fma(hh, ax[c], fma(sig * h, v0[c], x0[c]));
        V[c] = fma(h, av[c], v0[c]);
    }
}

// Shared stepping state of one lane.
struct Lane {
    double x0[3], v0[3], F0[3];
    bool active;
    int status;
};

// Integrate one window [t, W.t_b] with wave-shared adaptive steps.  The
// visitor is called after every accepted step with (t_prev, h, D).
template <class Params, class Visit>
__device__ __forceinline__ void integrate_window(const Params& p, const Window& W, double* coefL, int bstride,
                                                 double* ephW, Lane& L, double& t, double& hw, bool& haveF0,
                                                 long& wsteps, Visit&& visit) {
    const EphemArgs& E = p.eph;
    const RadauConst& rc = p.rc;
    const int lane = threadIdx.x & 63;
    const double tb = W.t_b;
    unsigned long long dummy = 0;
    if (__ballot(L.active) == 0ull) { t = tb; return; }
    while (t != tb) {
        const double dir = tb > t ? 1.0 : -1.0;
        double hmag = hw;
        if (p.h_max > 0.0 && hmag > p.h_max) hmag = p.h_max;
        double h = dir * hmag;
        bool landed = false;
        if (fabs(h) >= fabs(tb - t)) { h = tb - t; landed = true; }
        if (wsteps >= p.max_steps) {
            if (L.active) { L.status = KETE_ST_MAX_STEPS; L.active = false; }
            t = tb;
            return;
        }
        const double t_end = landed ? tb : t + h;
        node_ephemeris(coefL, bstride, E, rc, W.seg_lo, W.seg_hi, t, h, t_end, lane, ephW);
        if (!haveF0) { accel(ephW, E, L.x0, L.v0, L.F0); haveF0 = true; }
        double D[7][3], b6[3];
        corrector(rc, E, ephW, L.x0, L.v0, L.F0, h, L.active, p.max_iter, D, b6, dummy);
        double fm = 0.0, bm = 0.0;
        for (int c = 0; c < 3; ++c) { fm = fmax(fm, fabs(D[6][c] + L.F0[c])); bm = fmax(bm, fabs(b6[c])); }
        const double ebl = fm > 0.0 ? bm / fm : 0.0;
        double hl = (ebl > 0.0 && ebl < kInf) ? fabs(h) * step_factor(p.eps / ebl) : fabs(h) / p.safety;
        if (!L.active) hl = kInf;
        if (L.active && hl < p.h_min) { L.status = KETE_ST_STEP_UNDERFLOW; L.active = false; hl = kInf; }
        const double hn = wave_min(hl);
        if (!(hn < kInf)) { t = tb; return; }
        if (hn < p.safety * fabs(h)) { hw = hn; continue; }
        visit(t, h, D, ephW);
        const double hh = h * h;
        for (int c = 0; c < 3; ++c) {
            double ax = rc.half_s2[8] * L.F0[c], av = L.F0[c];
            for (int m = 0; m < 7; ++m) { ax = fma(rc.A[8][m], D[m][c], ax); av = fma(rc.B[8][m], D[m][c], av); }
            L.x0[c] = fma(hh, ax, fma(h, L.v0[c], L.x0[c]));
            L.v0[c] = fma(h, av, L.v0[c]);
        }
        t = t_end;
        ++wsteps;
        if (L.active && !(isfinite(L.x0[0]) && isfinite(L.x0[1]) && isfinite(L.x0[2]) && isfinite(L.v0[0]) &&
                          isfinite(L.v0[1]) && isfinite(L.v0[2]))) {
            L.status = KETE_ST_NONFINITE; L.active = false;
        }
        accel(ephW + 8 * E.n_body * 6, E, L.x0, L.v0, L.F0);
        hw = landed ? fmin(hw, hn) : fmin(hn, fabs(h) / p.safety);
    }
}


}  // namespace kete
