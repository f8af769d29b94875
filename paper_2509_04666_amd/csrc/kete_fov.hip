// Field-of-view membership on gfx950 (Sect. 2 and 3.1).
//
// Per batch, frames are binned by the direction of their bounding cap on
// a uniform 3-D grid over [-1, 1]^3 (unit vectors only touch cells near
// the sphere).  Every (object, batch) gets a rigorous bound on how far the
// object's light-time direction can move inside the batch -- perihelion
// speed of its heliocentric conic, the Sun's speed, the observers' spread
// and the batch half-span.  Objects whose reach stays inside the 3x3x3
// cells around their own direction ("narrow") are binned on the same
// grid, and a persistent join pops work items (one per 64 narrow objects
// of a cell) and scans the frames of the 27 neighbouring cells with
// wave-uniform loops; the remaining ("wide") objects scan the cells their
// cap touches, one wavefront per object.  Pairs that pass the cap test
// and a linear-motion test with a rigorous remainder bound become
// candidates; the exact test (universal-variable hop with light time,
// then n.d > 0 for every normal) decides membership.  Appends are staged
// in LDS per wavefront and flushed to the global lists in chunks; the
// pairs are then ordered by (frame, sub-frame, object) with a counting
// sort by frame and a sort inside each frame's segment.
#include <math.h>

#include <algorithm>

#include "kete_fov.hpp"

namespace kete {
namespace {

constexpr double kNaN = __builtin_nan("");

__device__ __forceinline__ void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Vertex k (0..3) of sub-frame quadrilateral n[4][3] (not normalized): the
// intersection of normal i = k / 2 of the pair (0, 1) with normal 2 + k % 2
// of the pair (2, 3), signed to lie inside the opposite edge.
__device__ __forceinline__ void quad_vertex(const double* __restrict__ n, int k, double v[3]) {
    const int i = k >> 1;
    cross3(n + 3 * i, n + 3 * (2 + (k & 1)), v);
    if (dot3(v, n + 3 * (1 - i)) < 0.0) { v[0] = -v[0]; v[1] = -v[1]; v[2] = -v[2]; }
}

// Sum over the 64 lanes of a wavefront (wave-uniform result).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, kWave);
    return uniform(x);
}

// Cap of every frame: centre the normalized sum of its sub-frames' unit
// vertex directions, radius the widest vertex seen from it (less a
// rounding margin).  One wavefront per frame, a lane per sub-frame (and
// 64 + lane), so that the normals are read in whole lines.
__global__ __launch_bounds__(256) void k_frame_caps(const double* __restrict__ normals, int64_t n_frames, int n_sub,
                                                    double* __restrict__ cap) {
    const int lane = threadIdx.x & 63;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t f = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; f < n_frames; f += n_waves) {
        double u[2][4][3];
        double sum[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int sf = lane + 64 * h;
            if (sf >= n_sub) continue;
            const double* n = normals + (f * n_sub + sf) * 12;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double v[3];
                quad_vertex(n, k, v);
                const double vn = sqrt(dot3(v, v));
                for (int c = 0; c < 3; ++c) {
                    u[h][k][c] = v[c] / vn;
                    sum[c] += u[h][k][c];
                }
            }
        }
        for (int c = 0; c < 3; ++c) sum[c] = wave_sum(sum[c]);
        const double sn = sqrt(dot3(sum, sum));
        double ctr[3] = {sum[0] / sn, sum[1] / sn, sum[2] / sn};
        double cmin = 1.0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (lane + 64 * h >= n_sub) continue;
#pragma unroll
            for (int k = 0; k < 4; ++k) cmin = fmin(cmin, dot3(u[h][k], ctr));
        }
        cmin = wave_min(cmin) - 1e-12;       // rounding margin (radius grows)
        if (!(sn > 0.0) || !(cmin > -1.0)) { ctr[0] = 1.0; ctr[1] = ctr[2] = 0.0; cmin = -1.0; }
        if (lane < 8) {
            const double v = lane < 3 ? ctr[lane] : lane == 3 ? cmin : lane == 4 ? sqrt(fmax(0.0, 1.0 - cmin * cmin))
                                                                             : 0.0;
            cap[8 * f + lane] = v;
        }
    }
}

// The same caps with one lane per frame, for frames of a few sub-frames
// (a wavefront per frame would leave most of its lanes idle).
__global__ void k_frame_caps_lane(const double* __restrict__ normals, int64_t n_frames, int n_sub,
                                  double* __restrict__ cap) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n_frames) return;
    double sum[3] = {0.0, 0.0, 0.0};
    for (int sf = 0; sf < n_sub; ++sf) {
        const double* n = normals + (f * n_sub + sf) * 12;
        for (int k = 0; k < 4; ++k) {
            double v[3];
            quad_vertex(n, k, v);
            const double vn = sqrt(dot3(v, v));
            for (int c = 0; c < 3; ++c) sum[c] += v[c] / vn;
        }
    }
    const double sn = sqrt(dot3(sum, sum));
    double ctr[3] = {sum[0] / sn, sum[1] / sn, sum[2] / sn};
    double cmin = 1.0;
    for (int sf = 0; sf < n_sub; ++sf) {
        const double* n = normals + (f * n_sub + sf) * 12;
        for (int k = 0; k < 4; ++k) {
            double v[3];
            quad_vertex(n, k, v);
            cmin = fmin(cmin, dot3(v, ctr) / sqrt(dot3(v, v)));
        }
    }
    cmin -= 1e-12;                       // rounding margin (radius grows)
    if (!(sn > 0.0) || !(cmin > -1.0)) { ctr[0] = 1.0; ctr[1] = ctr[2] = 0.0; cmin = -1.0; }
    double* o = cap + 8 * f;
    o[0] = ctr[0]; o[1] = ctr[1]; o[2] = ctr[2];
    o[3] = cmin;
    o[4] = sqrt(fmax(0.0, 1.0 - cmin * cmin));
    o[5] = o[6] = o[7] = 0.0;
}

// Sub-frame locator of every frame (see kLocStride), in cell order, one
// wavefront per frame with a lane per sub-frame (and 64 + lane).  The
// gnomonic image of a quadrilateral with great-circle edges inside the
// hemisphere around the centre is the convex quadrilateral of its
// vertices' images, so the box of those four points holds it; of the
// locator cells the box (widened by a rounding pad) overlaps, each lane
// marks those its quadrilateral really meets (bits set with LDS OR
// atomics).  The tangent basis follows the first edge of sub-frame 0, so
// that the cells of a regular mosaic line up with its rows and columns and
// most cells name one sub-frame.  The same pass writes the cell-ordered
// copy of the frame's time, observer and normals the join reads.
__global__ __launch_bounds__(256) void k_frame_locator(const FovParams p) {
    __shared__ unsigned long long s_mask[4][2 * kLocL * kLocL];
    unsigned long long* wm = s_mask[threadIdx.x >> 6];
    const int lane = threadIdx.x & 63;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int S = p.n_sub;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < p.n_frames; r += n_waves) {
        double* L = p.loc + (size_t)kLocStride * r;
        unsigned long long* M = reinterpret_cast<unsigned long long*>(L + kLocHead);
        const double* cp = p.cell_caps + 8 * r;
        const int f = p.cell_frames[r];
        const double c[3] = {cp[0], cp[1], cp[2]};
        const double* src = p.normals + (size_t)f * S * 12;
        float* dst = p.cell_normals + (size_t)r * S * 12;
        // tangent basis: e1 along the first edge of sub-frame 0 (the cells of
        // a regular mosaic then line up with its sub-frames), else from the
        // axis least aligned with c; any orthonormal basis is correct
        double dv[3] = {0.0, 0.0, 0.0};
        if (lane == 0) {
            double va[3], vb[3];
            quad_vertex(src, 0, va);
            quad_vertex(src, 1, vb);
            const double na = sqrt(dot3(va, va)), nb = sqrt(dot3(vb, vb));
            if (na > 0.0 && nb > 0.0)
                for (int k = 0; k < 3; ++k) dv[k] = vb[k] / nb - va[k] / na;
        }
        for (int k = 0; k < 3; ++k) dv[k] = __shfl(dv[k], 0, kWave);
        const double dc = dot3(dv, c);
        double e1[3] = {dv[0] - dc * c[0], dv[1] - dc * c[1], dv[2] - dc * c[2]};
        double n1 = sqrt(dot3(e1, e1));
        if (!(n1 > 1e-9)) {
            int ax = 0;
            if (fabs(c[1]) < fabs(c[ax])) ax = 1;
            if (fabs(c[2]) < fabs(c[ax])) ax = 2;
            for (int k = 0; k < 3; ++k) e1[k] = -c[ax] * c[k];
            e1[ax] += 1.0;
            n1 = sqrt(dot3(e1, e1));
        }
        for (int k = 0; k < 3; ++k) e1[k] /= n1;
        double e2[3];
        cross3(c, e1, e2);
        // gnomonic boxes of sub-frames lane and 64 + lane, whose normals are
        // copied to the cell-ordered table on the way
        double a0[2], a1[2], b0[2], b1[2];
        bool ok = true;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            a0[h] = 1e300; a1[h] = -1e300; b0[h] = 1e300; b1[h] = -1e300;
            const int sf = lane + 64 * h;
            if (sf >= S) continue;
            double nq[12];
            for (int k = 0; k < 12; ++k) nq[k] = src[12 * sf + k];
            for (int k = 0; k < 12; ++k) dst[12 * sf + k] = (float)nq[k];
            for (int k = 0; k < 4; ++k) {
                double v[3];
                quad_vertex(nq, k, v);
                const double vc = dot3(v, c);
                if (!(vc > 1e-6 * sqrt(dot3(v, v)))) { ok = false; continue; }
                const double X = dot3(v, e1) / vc, Y = dot3(v, e2) / vc;
                a0[h] = fmin(a0[h], X); a1[h] = fmax(a1[h], X); b0[h] = fmin(b0[h], Y); b1[h] = fmax(b1[h], Y);
            }
        }
        if (lane < 4) p.cell_obs[4 * r + lane] = lane == 0 ? p.ft[f] : p.fobs[3 * (size_t)f + lane - 1];
        ok = __ballot(!ok) == 0ull;
        double x0 = wave_min(fmin(a0[0], a0[1])), x1 = wave_max(fmax(a1[0], a1[1]));
        double y0 = wave_min(fmin(b0[0], b0[1])), y1 = wave_max(fmax(b1[0], b1[1]));
        const bool usable = ok && x1 >= x0 && y1 >= y0 && x1 - x0 < 1e6 && y1 - y0 < 1e6;
        wm[2 * lane] = 0ull;
        wm[2 * lane + 1] = 0ull;
        wave_lds_sync();
        double pad = 0.0, idx = 0.0, idy = 0.0;
        if (usable) {
            pad = 1e-9 * (1.0 + fmax(fmax(fabs(x0), fabs(x1)), fmax(fabs(y0), fabs(y1))));
            x0 -= pad; x1 += pad; y0 -= pad; y1 += pad;
            idx = kLocL / (x1 - x0);
            idy = kLocL / (y1 - y0);
            const double cw = (x1 - x0) / kLocL, ch = (y1 - y0) / kLocL;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (lane + 64 * h >= S) continue;
                const int i0 = max(0, (int)floor((a0[h] - pad - x0) * idx));
                const int i1 = min(kLocL - 1, (int)floor((a1[h] + pad - x0) * idx));
                const int j0 = max(0, (int)floor((b0[h] - pad - y0) * idy));
                const int j1 = min(kLocL - 1, (int)floor((b1[h] + pad - y0) * idy));
                // a cell in the box is marked unless one edge of the
                // sub-frame has the whole cell outside it: with v = c + X e1 +
                // Y e2 the edge's n . v is linear in (X, Y), so its largest
                // value over the cell is at a corner (an exact separating-axis
                // test of the two convex gnomonic images, the box giving the
                // cell's own axes; cells widened by a rounding pad)
                const unsigned long long bit = 1ull << lane;
                if (i0 == i1 && j0 == j1) {           // a box in one cell: that cell
                    atomicOr(&wm[2 * (i0 * kLocL + j0) + h], bit);
                    continue;
                }
                double A[4], B[4], Cg[4];
                const double* nh = src + 12 * (lane + 64 * h);     // read again (cached)
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const double nk[3] = {nh[3 * k], nh[3 * k + 1], nh[3 * k + 2]};
                    A[k] = dot3(nk, c);
                    B[k] = dot3(nk, e1);
                    Cg[k] = dot3(nk, e2);
                }
                for (int ci = i0; ci <= i1; ++ci) {
                    const double xa = x0 + ci * cw - pad, xb = x0 + (ci + 1) * cw + pad;
                    for (int cj = j0; cj <= j1; ++cj) {
                        const double ya = y0 + cj * ch - pad, yb = y0 + (cj + 1) * ch + pad;
                        const double tol = 1e-9 * (1.0 + fmax(fabs(xa), fabs(xb)) + fmax(fabs(ya), fabs(yb)));
                        bool sep = false;
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const double m = A[k] + fmax(B[k] * xa, B[k] * xb) + fmax(Cg[k] * ya, Cg[k] * yb);
                            sep = sep || m < -tol;
                        }
                        if (!sep) atomicOr(&wm[2 * (ci * kLocL + cj) + h], bit);
                    }
                }
            }
        }
        wave_lds_sync();
        static_assert(kLocL * kLocL == kWave, "one locator cell per lane");
        M[2 * lane] = wm[2 * lane];
        M[2 * lane + 1] = wm[2 * lane + 1];
        wave_lds_sync();
        if (lane < kLocHead) {
            double v = 0.0;
            if (lane < 3) v = c[lane];
            else if (lane < 6) v = e1[lane - 3];
            else if (lane < 9) v = e2[lane - 6];
            else if (usable)
                v = lane == 9 ? x0 : lane == 10 ? y0 : lane == 11 ? idx : lane == 12 ? idy : lane == 13 ? 1.0
                  : lane == 14 ? x0 + kLocL / idx : y0 + kLocL / idy;
            L[lane] = v;
        }
    }
}

// Cell-ordered copies of what the join reads of each frame: one wavefront
// per frame.
__global__ __launch_bounds__(256) void k_frame_gather(const FovParams p) {
    const int lane = threadIdx.x & 63;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int nd = 12 * p.n_sub;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < p.n_frames; r += n_waves) {
        const int f = p.cell_frames[r];
        const double* src = p.normals + (size_t)f * nd;
        float* dst = p.cell_normals + (size_t)r * nd;
        for (int i = lane; i < nd; i += kWave) dst[i] = (float)src[i];
        if (lane < 4) p.cell_obs[4 * r + lane] = lane == 0 ? p.ft[f] : p.fobs[3 * (size_t)f + lane - 1];
    }
}

// Rigorous bounds of the Sun's speed and acceleration over segments
// [lo, hi]: |T_n'| <= n^2 and |T_n''| <= n^2 (n^2 - 1) / 3 on [-1, 1].
__device__ void sun_bounds(const EphemArgs& E, int lo, int hi, double& vmax, double& amax) {
    vmax = 0.0; amax = 0.0;
    const double sc = 2.0 * E.inv_seg;
    for (int k = lo; k <= hi; ++k) {
        double v2 = 0.0, a2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double* cf = E.coef + ((size_t)k * 3 + c) * E.deg1;   // body 0
            double sv = 0.0, sa = 0.0;
            for (int n = 1; n < E.deg1; ++n) {
                const double n2 = (double)n * n;
                sv += n2 * fabs(cf[n]);
                sa += n2 * (n2 - 1.0) / 3.0 * fabs(cf[n]);
            }
            v2 += sv * sv; a2 += sa * sa;
        }
        vmax = fmax(vmax, sqrt(v2) * sc);
        amax = fmax(amax, sqrt(a2) * sc * sc);
    }
}

// One block per batch: Sun state at t_ref, mean observer, observer
// spread, half-span, largest frame radius, Sun speed/acceleration bounds.
__global__ __launch_bounds__(256) void k_batch_prep(const FovParams p) {
    __shared__ double red[256 * 4];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int q0 = p.batch_off[b], q1 = p.batch_off[b + 1];
    const double tr = p.t_ref[b];
    double s[3] = {0.0, 0.0, 0.0};
    for (int q = q0 + tid; q < q1; q += 256) {
        const int f = p.frame_order[q];
        for (int c = 0; c < 3; ++c) s[c] += p.fobs[3 * f + c];
    }
    for (int c = 0; c < 3; ++c) red[c * 256 + tid] = s[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) for (int c = 0; c < 3; ++c) red[c * 256 + tid] += red[c * 256 + tid + w];
        __syncthreads();
    }
    const double inv = 1.0 / (double)(q1 - q0);
    const double ob[3] = {red[0] * inv, red[256] * inv, red[512] * inv};
    __syncthreads();
    double dmax = 0.0, tmax = 0.0, cmin = 1.0;
    for (int q = q0 + tid; q < q1; q += 256) {
        const int f = p.frame_order[q];
        double dd[3] = {p.fobs[3 * f] - ob[0], p.fobs[3 * f + 1] - ob[1], p.fobs[3 * f + 2] - ob[2]};
        dmax = fmax(dmax, sqrt(dot3(dd, dd)));
        tmax = fmax(tmax, fabs(p.ft[f] - tr));
        cmin = fmin(cmin, p.fcap[8 * f + 3]);
    }
    red[tid] = dmax; red[256 + tid] = tmax; red[512 + tid] = -cmin;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) for (int c = 0; c < 3; ++c) red[c * 256 + tid] = fmax(red[c * 256 + tid], red[c * 256 + tid + w]);
        __syncthreads();
    }
    if (tid == 0) {
        double* o = p.btab + kBatchStride * b;
        const EphemArgs& E = p.eph;
        const int hi_all = E.n_seg - 1;
        double S[3], Sd[3];
        cheb_body(E.coef, 0, E.deg1, tr, E.t_start, E.seg_days, E.inv_seg, 0, hi_all, S, Sd);
        const double delta = red[256] * (1.0 + 1e-15) + 1e-12;
        const double span = delta + kMaxLightDays;
        const int lo = seg_index(tr - span, E.t_start, E.inv_seg, 0, hi_all);
        const int hi = seg_index(tr + span, E.t_start, E.inv_seg, 0, hi_all);
        double vs, as;
        sun_bounds(E, lo, hi, vs, as);
        for (int c = 0; c < 3; ++c) { o[c] = S[c]; o[3 + c] = Sd[c]; o[6 + c] = ob[c]; }
        o[9] = red[0] * (1.0 + 1e-12) + 1e-12;    // observer spread
        o[10] = delta;                             // max |t_f - t_ref|
        const double cR = -red[512];
        o[11] = cR;
        o[12] = sqrt(fmax(0.0, 1.0 - cR * cR));
        o[13] = vs * (1.0 + 1e-9) + 1e-15;
        o[14] = as * (1.0 + 1e-9) + 1e-15;
        o[15] = (double)lo;
        o[16] = (double)hi;
        // Large frames: coarsen the grid so that a frame plus a typical
        // motion cap (1.5 deg) fits in one cell, keeping most objects on
        // the per-cell join.
        const double Rm = atan2(o[12], cR) + 1.5 * (3.14159265358979323846 / 180.0);
        const double L = 1.2 * 2.0 * sin(0.5 * fmin(Rm, 3.0));
        const int G = L > 0.0 ? (int)floor(2.0 / L) : 1;
        if (G < p.b_G[b]) p.b_G[b] = G < 1 ? 1 : G;
    }
}

// Cell of coordinate u in [-1, 1] on a grid of G cells per axis.
__device__ __forceinline__ int cell_coord(double u, int G) {
    int i = (int)floor((u + 1.0) * (0.5 * G));
    return i < 0 ? 0 : (i >= G ? G - 1 : i);
}

__device__ __forceinline__ int cell_of(const double u[3], int G) {
    return (cell_coord(u[0], G) * G + cell_coord(u[1], G)) * G + cell_coord(u[2], G);
}

__global__ void k_frame_keys(const FovParams p, int32_t* __restrict__ qkey, int32_t* __restrict__ cnt) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= p.n_frames) return;
    // batch of sorted position q
    int lo = 0, hi = p.n_batch;            // batch_off[lo] <= q < batch_off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (p.batch_off[mid] <= q) lo = mid; else hi = mid;
    }
    const int f = p.frame_order[q];
    const double* c = p.fcap + 8 * f;
    const int key = (int)(p.b_koff[lo] + cell_of(c, p.b_G[lo]));
    qkey[q] = key;
    p.frame_batch[f] = lo;
    atomicAdd(cnt + key, 1);
}

__global__ void k_frame_scatter(const FovParams p, const int32_t* __restrict__ qkey, int32_t* __restrict__ cursor) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= p.n_frames) return;
    const int key = qkey[q];
    const int pos = p.cell_start[key] + atomicAdd(cursor + key, 1);
    const int f = p.frame_order[q];
    p.cell_frames[pos] = f;
    const double* src = p.fcap + 8 * f;
    double* dst = p.cell_caps + 8 * (int64_t)pos;
    for (int i = 0; i < 5; ++i) dst[i] = src[i];
    dst[5] = (double)f;
    dst[6] = dst[7] = 0.0;
}

// Append a key to a bounded list with one atomic per wavefront: the
// active lanes take consecutive slots in lane order (ballot + popcount).
__device__ __forceinline__ void wave_append(unsigned long long* list, unsigned long long* count, int64_t cap,
                                            unsigned long long key) {
    const unsigned long long m = __ballot(1);
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(count, (unsigned long long)__popcll(m));
    base = __shfl(base, leader, 64);
    const unsigned long long idx = base + __popcll(m & lt);
    if (idx < (unsigned long long)cap) list[idx] = key;
}

// Per-wavefront staging of list appends in LDS: appends gather in `buf`
// (kEntries entries) and reach the global list kEntries - 63 or more at a
// time, so the shared counter, one address that every wavefront of the
// chip updates, sees one atomic per flush instead of one per append.  The
// pair list, by far the longest, gets the larger buffer.  Both calls must
// be made by the whole wavefront.
constexpr int kBufEntries = 128;
constexpr int kPairBufEntries = 512;

__device__ __forceinline__ void buf_flush(unsigned long long* __restrict__ buf, int& n,
                                          unsigned long long* __restrict__ list, unsigned long long* count,
                                          int64_t cap) {
    if (n == 0) return;
    const int lane = threadIdx.x & 63;
    wave_lds_sync();
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(count, (unsigned long long)n);
    base = __shfl(base, 0, 64);
    for (int i = lane; i < n; i += 64) {
        const unsigned long long idx = base + (unsigned long long)i;
        if (idx < (unsigned long long)cap) list[idx] = buf[i];
    }
    wave_lds_sync();
    n = 0;
}

template <int kEntries>
__device__ __forceinline__ void buf_append(unsigned long long* __restrict__ buf, int& n, bool pred,
                                           unsigned long long key, unsigned long long* __restrict__ list,
                                           unsigned long long* count, int64_t cap) {
    const unsigned long long m = __ballot(pred);
    if (m == 0ull) return;
    const int lane = threadIdx.x & 63;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (pred) buf[n + __popcll(m & lt)] = key;
    n += __popcll(m);
    if (n > kEntries - kWave) buf_flush(buf, n, list, count, cap);
}

// Everything one (object, batch) needs to skip frames it cannot reach.
struct ObjBounds {
    double x[3], v[3];        // barycentric state at the batch epoch
    double dh[3];             // unit direction from the batch's mean observer
    double sth, cth;          // sin/cos of the cap on the direction's motion
    double taumax;            // light-time bound
    double a2b, vbn;          // heliocentric acceleration bound, |v|
    int lo[3], hi[3];         // grid box of the cap (valid when !overflow)
    int ncell;
    bool lin_ok;              // the linear-motion test is valid
    bool overflow;            // no usable cap: test every frame of the batch
};

// Rigorous motion bounds inside batch b (half-span Delta):
//  - speed on the heliocentric conic <= perihelion speed mu (1 + e) / |r x v|,
//    plus the Sun's speed bound;
//  - light time tau <= (|d| + D_obs + V Delta) / (c - V);
//  - |x_e - o_f - d_ref| <= V (Delta + tau) + D_obs, so the direction
//    moves by at most asin of that over |d_ref|;
//  - between the batch epoch and the emission time the heliocentric
//    acceleration is at most mu / r_min^2 with r_min >= perihelion.
// Returns false for failed or non-finite objects.
__device__ __forceinline__ bool object_bounds(const FovParams& p, int b, int64_t j, ObjBounds& o) {
    if (p.status && p.status[p.b_obj0[b] + j] != 0) return false;
    const double* st = p.x_epoch + p.b_xoff[b] + 6 * j;
    for (int c = 0; c < 3; ++c) { o.x[c] = st[c]; o.v[c] = st[3 + c]; }
    if (!(isfinite(o.x[0]) && isfinite(o.x[1]) && isfinite(o.x[2]) && isfinite(o.v[0]) && isfinite(o.v[1]) &&
          isfinite(o.v[2])))
        return false;
    const double* bt = p.btab + kBatchStride * b;
    const double mu = p.mu, cl = p.c_light;
    const double Dobs = bt[9], Delta = bt[10], cosRm = bt[11], sinRm = bt[12], Vsun = bt[13];
    double r0[3], v0[3];
    for (int c = 0; c < 3; ++c) { r0[c] = o.x[c] - bt[c]; v0[c] = o.v[c] - bt[3 + c]; }
    const double r0n = sqrt(dot3(r0, r0));
    const double v2 = dot3(v0, v0);
    double hv[3];
    cross3(r0, v0, hv);
    const double hn = sqrt(dot3(hv, hv));
    const double rv = dot3(r0, v0);
    double ev[3];
    for (int c = 0; c < 3; ++c) ev[c] = ((v2 - mu / r0n) * r0[c] - rv * v0[c]) / mu;
    const double ecc = sqrt(dot3(ev, ev));
    const double vp = (hn > 0.0) ? mu * (1.0 + ecc) / hn * (1.0 + 1e-12) : 1e300;
    const double q = (hn > 0.0) ? hn * hn / (mu * (1.0 + ecc)) * (1.0 - 1e-12) : 0.0;
    const double V = vp + Vsun;
    double dref[3];
    for (int c = 0; c < 3; ++c) dref[c] = o.x[c] - bt[6 + c];
    const double dn = sqrt(dot3(dref, dref));
    for (int c = 0; c < 3; ++c) o.dh[c] = dref[c] / dn;
    const bool bounded = (V < 0.5 * cl) && (dn > 0.0);
    o.taumax = 0.0; o.sth = 1.0; o.cth = 0.0;
    o.overflow = !bounded;
    if (bounded) {
        o.taumax = (dn + Dobs + V * Delta) / (cl - V) * (1.0 + 1e-12);
        const double delta = V * (Delta + o.taumax) + Dobs + 1e-12;
        o.sth = delta / dn;
        if (!(o.sth < p.sin_overflow)) o.overflow = true;
        else o.cth = sqrt(1.0 - o.sth * o.sth);
    }
    // the linear test also uses the Sun's acceleration bound, which covers
    // light times up to kMaxLightDays
    o.lin_ok = bounded && o.taumax <= kMaxLightDays;
    const double rmin = fmax(q, r0n - vp * (Delta + o.taumax));
    o.a2b = (rmin > 0.0) ? mu / (rmin * rmin) : 1e300;
    o.vbn = sqrt(dot3(o.v, o.v));
    o.ncell = 0;
    if (!o.overflow) {
        const double cosRT = cosRm * o.cth - sinRm * o.sth;      // cos(Rmax + theta)
        if (!(cosRT > 0.0)) {
            o.overflow = true;
        } else {
            const double chord = sqrt(2.0 - 2.0 * cosRT) + 1e-9;
            o.ncell = 1;
            for (int c = 0; c < 3; ++c) {
                o.lo[c] = cell_coord(o.dh[c] - chord, p.b_G[b]);
                o.hi[c] = cell_coord(o.dh[c] + chord, p.b_G[b]);
                o.ncell *= o.hi[c] - o.lo[c] + 1;
            }
            if (o.ncell > p.max_cells) o.overflow = true;
        }
    }
    return true;
}

constexpr int kNarrowCells = 27;

// Narrow: the cap's grid box lies inside the 3x3x3 neighbourhood of the
// cell holding the direction itself, so every frame the object can reach
// is listed in one of those 27 cells.
__device__ __forceinline__ bool is_narrow(const ObjBounds& o, int G) {
    if (o.overflow) return false;
    for (int c = 0; c < 3; ++c) {
        const int home = cell_coord(o.dh[c], G);
        if (o.lo[c] < home - 1 || o.hi[c] > home + 1) return false;
    }
    return true;
}

// Cap test with the frame's own radius, then the linear-motion test with
// its remainder bound; survivors become exact-test candidates.
__device__ __forceinline__ bool frame_cap_hit(const ObjBounds& o, const double* __restrict__ cp) {
    if (o.overflow) return true;
    const double thr = cp[3] * o.cth - cp[4] * o.sth;         // cos(R_f + theta)
    return !(dot3(cp, o.dh) < thr - 1e-12);
}

// Linear prediction of an (object, frame) pair: ul = x + v dt - o for the
// frame's time t and observer o (ob = {t, o}), and the bound e2 on the
// distance from ul to the true line of sight (light time and curvature of
// the path, see classify_emit).
__device__ __forceinline__ double lin_predict(const ObjBounds& o, const double ob[4], double tr, double Asun,
                                              double ul[3]) {
    const double dt = ob[0] - tr;
    for (int c = 0; c < 3; ++c) ul[c] = o.x[c] + o.v[c] * dt - ob[1 + c];
    const double ad = fabs(dt) + o.taumax;
    return 2.0 * (o.vbn * o.taumax + 0.5 * (o.a2b + Asun) * ad * ad + 1e-12);
}

// The same prediction carried back over the light time as well, for the
// sub-frame tests: with u0 = x + v dt - o and tau0 = |u0| / c,
// ul = u0 - v tau0 (the straight line at t - tau0).  The body's position
// at the emission time t - tau is within eps0 = |v| tau_max + a ad^2 / 2
// of x + v dt (a the acceleration bound, ad = |dt| + tau_max), so |tau -
// tau0| <= eps0 / c, and it is within a ad^2 / 2 + |v| eps0 / c of ul: the
// light-time term |v| tau_max, which dominates eps0 for most bodies, is
// scaled down by |v| / c.  Returns the bound, doubled as lin_predict's.
__device__ __forceinline__ double lin_predict_lt(const ObjBounds& o, const double ob[4], double tr, double Asun,
                                                 double c_light, double ul[3]) {
    const double dt = ob[0] - tr;
    double u0[3];
    for (int c = 0; c < 3; ++c) u0[c] = o.x[c] + o.v[c] * dt - ob[1 + c];
    const double tau0 = sqrt(dot3(u0, u0)) / c_light;
    for (int c = 0; c < 3; ++c) ul[c] = u0[c] - o.v[c] * tau0;
    const double ad = fabs(dt) + o.taumax;
    const double acc = 0.5 * (o.a2b + Asun) * ad * ad;
    return 2.0 * (acc + o.vbn * (o.vbn * o.taumax + acc) / c_light + 1e-12);
}

// Can a line of sight within e2 of ul reach the frame's cap (centre cp,
// cos and sin of the radius R)?  Its angle from ul is at most
// asin(e2 / |ul|), so it misses the cap when the angle of ul from the centre
// exceeds R + asin(e2 / |ul|), i.e. when A = ul . c + sin R e2 falls below
// B = cos R sqrt(|ul|^2 - e2^2) (R below 90 degrees).  B >= 0, so the test
// is A >= 0 and A^2 >= B^2, with no square root; A is raised by
// 1e-12 |ul|_1 >= 1e-12 |ul| to cover rounding.  A void bound
// (e2 >= |ul|) or a wider frame passes.
__device__ __forceinline__ bool lin_cap_hit(const double* __restrict__ cp, const double ul[3], double e2) {
    const double u2 = dot3(ul, ul);
    if (!(e2 * e2 < u2) || !(cp[3] > 0.0)) return true;
    const double a = dot3(ul, cp) + cp[4] * e2 + 1e-12 * (fabs(ul[0]) + fabs(ul[1]) + fabs(ul[2]));
    return a >= 0.0 && a * a >= cp[3] * cp[3] * (u2 - e2 * e2);
}

// Locator header of one frame (see kLocStride), read with eight 16-byte
// loads issued together rather than one dependent read after another.
struct LocHead {
    double c[3], e1[3], e2[3];
    double x0, y0, idx, idy, usable, x1, y1;
};
__device__ __forceinline__ LocHead loc_head(const double* __restrict__ L) {
    const double2* q = reinterpret_cast<const double2*>(L);
    const double2 a = q[0], b = q[1], c = q[2], d = q[3], e = q[4], f = q[5], g = q[6], k = q[7];
    LocHead h;
    h.c[0] = a.x; h.c[1] = a.y; h.c[2] = b.x;
    h.e1[0] = b.y; h.e1[1] = c.x; h.e1[2] = c.y;
    h.e2[0] = d.x; h.e2[1] = d.y; h.e2[2] = e.x;
    h.x0 = e.y; h.y0 = f.x; h.idx = f.y; h.idy = g.x; h.usable = g.y;
    h.x1 = k.x; h.y1 = k.y;
    return h;
}

// Can an object's direction cap (o.dh, theta) reach the gnomonic box of
// the sub-frames of the frame at cell rank r?  The same widening of the
// cap's image as in sub_candidates; without a usable locator, yes.
__device__ __forceinline__ bool loc_box_hit(const FovParams& p, const ObjBounds& o, int r) {
    if (!p.loc || o.overflow) return true;
    const LocHead h = loc_head(p.loc + (size_t)kLocStride * (unsigned)r);
    if (!(h.usable > 0.5)) return true;
    const double uc = dot3(o.dh, h.c);
    if (!(uc > 0.0) || !(o.cth > 0.0)) return true;
    const double X = dot3(o.dh, h.e1) / uc, Y = dot3(o.dh, h.e2) / uc;
    const double t = o.sth / o.cth;
    const double ru = sqrt(X * X + Y * Y);
    if (!(ru * t < 0.5)) return true;
    const double T = (ru + t) / (1.0 - ru * t);
    const double mg = t * (1.0 + T * T) * (1.0 + 1e-9) + 1e-12 * (1.0 + ru);
    return !(X + mg < h.x0 || X - mg > h.x1 || Y + mg < h.y0 || Y - mg > h.y1);
}

// Sub-frames of a frame (locator header h, mask words M, or no locator)
// that a direction within angle atan(t) of u can lie in: bit s of
// m[s / 64].  With a locator, u's gnomonic point widened by the image of
// that angle (the map stretches by at most 1 + T^2 at tangent-plane
// radius T) selects the locator cells; without one, or for a wide query,
// every sub-frame.  A query box off the frame's box gives none.  The mask
// words of up to nine cells are read together.
__device__ __forceinline__ void sub_candidates(int S, bool have_loc, const LocHead& h,
                                               const ulonglong2* __restrict__ M, const double u[3], double t,
                                               unsigned long long m[2]) {
    m[0] = S >= 64 ? ~0ull : ((1ull << S) - 1ull);
    m[1] = S > 64 ? (S >= 128 ? ~0ull : ((1ull << (S - 64)) - 1ull)) : 0ull;
    if (!have_loc || !(h.usable > 0.5)) return;
    const double uc = dot3(u, h.c);
    if (!(uc > 0.0)) return;
    // (the product with 1 / uc and the bound 1 / (1 - q) <= 1 + 2q for
    // q <= 1/2 replace two divisions; both errors are far inside the margin)
    const double iuc = 1.0 / uc;
    const double X = dot3(u, h.e1) * iuc, Y = dot3(u, h.e2) * iuc;
    const double ru = sqrt(X * X + Y * Y);
    if (!(ru * t < 0.5)) return;
    const double T = (ru + t) * (1.0 + 2.0 * ru * t);
    const double mg = t * (1.0 + T * T) * (1.0 + 1e-9) + 1e-12 * (1.0 + ru);
    const double fx0 = (X - mg - h.x0) * h.idx, fx1 = (X + mg - h.x0) * h.idx;
    const double fy0 = (Y - mg - h.y0) * h.idy, fy1 = (Y + mg - h.y0) * h.idy;
    if (fx1 < 0.0 || fy1 < 0.0 || fx0 >= kLocL || fy0 >= kLocL) {   // off the frame's box
        m[0] = m[1] = 0ull;
        return;
    }
    if (!(fx0 >= -1e9 && fx1 <= 1e9 && fy0 >= -1e9 && fy1 <= 1e9)) return;
    const int ix0 = (int)floor(fmax(fx0, 0.0)), ix1 = (int)floor(fmin(fx1, kLocL - 1.0));
    const int iy0 = (int)floor(fmax(fy0, 0.0)), iy1 = (int)floor(fmin(fy1, kLocL - 1.0));
    const int ny = iy1 - iy0 + 1, n = (ix1 - ix0 + 1) * ny;
    if (n > 9) return;
    unsigned long long a = 0ull, b = 0ull;
    int dx = 0, dy = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const bool in = k < n;
        const ulonglong2 w = M[in ? (ix0 + dx) * kLocL + iy0 + dy : ix0 * kLocL + iy0];
        if (in) { a |= w.x; b |= w.y; }
        if (++dy == ny) { dy = 0; ++dx; }
    }
    m[0] = a;
    m[1] = b;
}

// The r-th set bit (counted from 0, r < popcount(w)) of a 64-bit word.
__device__ __forceinline__ int nth_set_bit(unsigned long long w, int r) {
    int pos = 0;
#pragma unroll
    for (int width = 32; width >= 1; width >>= 1) {
        const int c = __popcll(w & ((1ull << width) - 1ull));
        if (r >= c) { r -= c; w >>= width; pos += width; }
    }
    return pos;
}

// Linear-motion test of an (object, frame) pair that passed the cap test
// (and, with a linear test, the linear cap test),
// with its remainder bound: the object moves on x + v dt within eps of its
// true emission point, so with unit normals and ul = x + v dt - o a
// sub-frame is out when some n . ul <= -2 eps, surely in when every
// n . ul > 2 eps (the true direction's dot products then keep their
// signs), and undecided otherwise; the test is void when 2 eps reaches
// |ul|.  Every lane with `has` classifies its pair: sure pairs go to the
// pair list, undecided (frame, sub-frame, object) keys, or one
// (frame, kAllSubs, object) key for a void test, to the exact-test
// candidates.  The sub-frames the locator leaves to each pair are pooled
// over the wavefront and tested 64 at a time, one per lane, so a pair with
// many of them does not hold the others up.  Frames are named by their
// cell rank r.  The whole wavefront calls it.
constexpr int kTestList = 256;          // tests a wavefront lists in LDS at once
constexpr int kTestListPer = 8;         // and per pair
__device__ void classify_emit(const FovParams& p, bool has, const ObjBounds& o, int r, double tr, double Asun,
                              unsigned long long gobj, unsigned long long* cbuf, int& nc, unsigned long long* pbuf,
                              int& np, unsigned long long& n_exact) {
    __shared__ unsigned short s_tests[4][kTestList];
    const int lane = threadIdx.x & 63;
    bool all = false;
    unsigned long long m0 = 0ull, m1 = 0ull;
    double ul[3] = {0.0, 0.0, 0.0}, e2 = 0.0;
    int f = 0;
    if (has) {
        // every read of the frame's records is issued before the first use
        f = p.cell_frames[r];
        const double2* q = reinterpret_cast<const double2*>(p.cell_obs + 4 * (size_t)(unsigned)r);
        const double2 ob01 = q[0], ob23 = q[1];
        LocHead h;
        h.usable = 0.0;
        if (p.loc) h = loc_head(p.loc + (size_t)kLocStride * (unsigned)r);
        all = !o.lin_ok;
        if (o.lin_ok) {
            const double ob[4] = {ob01.x, ob01.y, ob23.x, ob23.y};
            e2 = lin_predict_lt(o, ob, tr, Asun, p.c_light, ul);
            const double u2 = dot3(ul, ul);
            if (!(e2 * e2 < u2)) {
                all = true;
            } else {
                unsigned long long m[2];
                const ulonglong2* M = p.loc ? reinterpret_cast<const ulonglong2*>(
                                                  p.loc + (size_t)kLocStride * (unsigned)r + kLocHead)
                                            : nullptr;
                sub_candidates(p.n_sub, p.loc != nullptr, h, M, ul, e2 / sqrt(u2 - e2 * e2), m);
                m0 = m[0];
                m1 = m[1];
            }
        }
    }
    const unsigned long long base = ((unsigned long long)(unsigned)f << 32) | gobj;
    if (all) ++n_exact;
    buf_append<kBufEntries>(cbuf, nc, all, base | kAllSubs, p.cand, p.n_cand, p.cand_cap);
    // test of sub-frame s of pair (ri, bi) with ul = (u0, u1, u2), margin e.
    // The normals are single-precision copies: each component is within
    // 2^-24 of its own magnitude of the double, so n . u moves by at most
    // 2^-24 sum |n_i u_i| (to first order; 2^-23 covers the rest), which
    // widens the margin; the undecided band grows by about 1e-7 rad.
    auto sub_test = [&](bool act, int ri, int s, double u0, double u1, double u2, double e, unsigned long long bi) {
        int res = 0;
        if (act) {
            const float4* n4 = reinterpret_cast<const float4*>(p.cell_normals +
                                                               ((size_t)(unsigned)ri * p.n_sub + s) * 12);
            const float4 q0 = n4[0], q1 = n4[1], q2 = n4[2];
            const double n[12] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
            res = 1;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double a = n[3 * k] * u0, b = n[3 * k + 1] * u1, c = n[3 * k + 2] * u2;
                const double d = a + b + c;
                const double ek = e + 0x1p-23 * (fabs(a) + fabs(b) + fabs(c));
                if (d <= -ek) res = 0;
                else if (!(d > ek) && res == 1) res = 2;
            }
        }
        const unsigned long long key = bi | ((unsigned long long)(act ? s : 0) << 25);
        if (res == 2) ++n_exact;
        buf_append<kPairBufEntries>(pbuf, np, res == 1, key, p.pairs, p.n_pairs, p.cap);
        buf_append<kBufEntries>(cbuf, nc, res == 2, key, p.cand, p.n_cand, p.cand_cap);
    };
    const int cnt = __popcll(m0) + __popcll(m1);
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int t = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += t;
    }
    const int total = __shfl(incl, kWave - 1, kWave);
    if (total == 0) return;
    if (total <= kTestList && __ballot(cnt > kTestListPer) == 0ull) {
        // The usual case, a few tests per pair: each lane lists its tests
        // (lane << 8 | sub-frame) at its exclusive prefix in LDS, one
        // sub-frame per round, and lane t of a pass reads test t back.
        unsigned short* tl = s_tests[(threadIdx.x >> 6) & 3];
        unsigned long long a = m0, b = m1;
        int pos = incl - cnt;
#pragma unroll 1
        for (int k = 0; k < kTestListPer; ++k) {
            const bool more = (a | b) != 0ull;
            if (__ballot(more) == 0ull) break;
            if (more) {
                const int sb = a ? __ffsll((long long)a) - 1 : 64 + __ffsll((long long)b) - 1;
                if (a) a &= a - 1ull; else b &= b - 1ull;
                tl[pos++] = (unsigned short)((lane << 8) | sb);
            }
        }
        wave_lds_sync();
        for (int t0 = 0; t0 < total; t0 += kWave) {
            const int t = t0 + lane;
            const unsigned te = t < total ? tl[t] : 0u;
            const int i = (int)(te >> 8);
            const double u0 = __shfl(ul[0], i, kWave), u1 = __shfl(ul[1], i, kWave), u2 = __shfl(ul[2], i, kWave);
            const double e = __shfl(e2, i, kWave);
            const int ri = __shfl(r, i, kWave);
            const unsigned long long bi = __shfl(base, i, kWave);
            sub_test(t < total, ri, (int)(te & 0xffu), u0, u1, u2, e, bi);
        }
        wave_lds_sync();                      // the list is read before the next call writes it
        return;
    }
    for (int t0 = 0; t0 < total; t0 += kWave) {
        const int t = t0 + lane;
        // the pair holding test t: the first lane whose inclusive count exceeds t
        int i = 0;
#pragma unroll
        for (int step = kWave / 2; step > 0; step >>= 1) {
            const int v = __shfl(incl, i + step - 1, kWave);
            if (v <= t) i += step;
        }
        const int nb = t - (__shfl(incl, i, kWave) - __shfl(cnt, i, kWave));   // its nb-th sub-frame
        const unsigned long long w0 = __shfl(m0, i, kWave), w1 = __shfl(m1, i, kWave);
        const double u0 = __shfl(ul[0], i, kWave), u1 = __shfl(ul[1], i, kWave), u2 = __shfl(ul[2], i, kWave);
        const double e = __shfl(e2, i, kWave);
        const int ri = __shfl(r, i, kWave);
        const unsigned long long bi = __shfl(base, i, kWave);
        int s = 0;
        if (t < total) {
            const int c0 = __popcll(w0);
            s = nb < c0 ? nth_set_bit(w0, nb) : 64 + nth_set_bit(w1, nb - c0);
        }
        sub_test(t < total, ri, s, u0, u1, u2, e, bi);
    }
}

// Narrow objects: one wavefront per (batch, sky cell) of objects.  The
// lanes take the cell's objects 64 at a time and scan the frames of the 27
// neighbouring cells together: the loops are the same for every lane and
// the frame records are broadcast loads.
// batch of a flattened (batch, object) index: b_poff[b] <= i < b_poff[b+1]
__device__ __forceinline__ int batch_of(const int64_t* __restrict__ poff, int n_batch, int64_t i) {
    int lo = 0, hi = n_batch;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (poff[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// batch holding sort key `key` (keys are batch-major)
__device__ __forceinline__ int batch_of_key(const int64_t* __restrict__ koff, int n_batch, int64_t key) {
    int lo = 0, hi = n_batch;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (koff[mid] <= key) lo = mid; else hi = mid;
    }
    return lo;
}

// Read lane m's value (m uniform) into every lane.
__device__ __forceinline__ double lane_value(double v, int m) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), m);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), m);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Work items of the join: one per 64 narrow objects of a (batch, cell).
__global__ void k_item_count(const FovParams p, int32_t* __restrict__ icnt) {
    const int64_t key = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (key >= p.n_keys) return;
    const int b = batch_of_key(p.b_koff, p.n_batch, key);
    const int G = p.b_G[b];
    const bool narrow_cell = key - p.b_koff[b] < (int64_t)G * G * G;
    icnt[key] = narrow_cell ? (p.obj_count[key] + kWave - 1) / kWave : 0;
}

__global__ void k_item_scatter(const FovParams p, const int32_t* __restrict__ icnt) {
    const int64_t key = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (key >= p.n_keys) return;
    const int n = icnt[key], s0 = p.item_start[key];
    for (int c = 0; c < n; ++c) p.items[s0 + c] = ((unsigned long long)key << 32) | (unsigned long long)c;
}

// A frame's record for the per-cell join's broadcast loop: cap (centre,
// cos and sin of the radius), cell rank, time and observer, as five
// 16-byte LDS words.
struct __align__(16) FrameRec {
    double c[3], cosr, sinr, rank, t, o[3];
};

constexpr int kLinQueue = 2 * kWave;
constexpr int kItemChunk = 3;

// Persistent join: every wavefront pops work items until none is left.
// An item is up to 64 narrow objects of one (batch, cell), one per lane;
// the frame records of the 27 neighbouring cells are read 64 at a time,
// one per lane, and broadcast for the cap test.  (object, frame) pairs
// that pass it are queued in LDS and take the linear-motion test 64 at a
// time, one pair per lane, reading their object's data from the lane that
// holds it.  The broadcast loop reads LDS only: after the motion-cap test
// an object with a linear test takes the linear cap test there (the frame
// record carries the frame's time and observer), and only objects without
// one take the locator-box test, a global read.  Items are in (batch, cell) order; the waves of
// one XCD start on their own slice of the list, so that neighbouring cells
// share that XCD's L2, and help the other slices when theirs runs out.
constexpr int kJoinWaves = 3;        // resident waves per SIMD of the join kernels (168 VGPRs, a few spilled)
__global__ __launch_bounds__(256, kJoinWaves) void k_fov_cells(const FovParams p) {
    const int lane = threadIdx.x & 63, wv = (threadIdx.x >> 6) & 3;
    unsigned long long n_cand = 0, n_exact = 0, n_visit = 0;
    const double* __restrict__ caps = p.cell_caps;
    const int n_items = p.item_start[p.n_keys];
    __shared__ unsigned long long bufs[4][kBufEntries], pbufs[4][kPairBufEntries];
    __shared__ unsigned long long queue_all[4][kLinQueue];
    __shared__ FrameRec fcap_all[4][kWave];
    unsigned long long* buf = bufs[wv];
    unsigned long long* pbuf = pbufs[wv];
    int npbuf = 0;
    FrameRec* fcap = fcap_all[wv];
    unsigned long long* queue = queue_all[wv];
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int nbuf = 0;
    int item = 0, item_end = 0;
    const int home = (int)(blockIdx.x % kXcds);
    int tried = 0;                            // slices found empty
    for (;;) {
        // items are taken kItemChunk at a time: one atomic on a slice's
        // cursor per chunk
        if (item >= item_end) {
            while (tried < kXcds) {
                const int x = (home + tried) % kXcds;
                const int lo = (int)((int64_t)n_items * x / kXcds), hi = (int)((int64_t)n_items * (x + 1) / kXcds);
                int first = 0;
                if (lane == 0) first = (int)atomicAdd(p.item_next + kCursorStride * x, (unsigned)kItemChunk);
                first = __shfl(first, 0, kWave);
                if (first < hi - lo) {
                    item = lo + first;
                    item_end = min(item + kItemChunk, hi);
                    break;
                }
                ++tried;
            }
            if (tried >= kXcds) break;
        }
        const unsigned long long it = p.items[item++];
        const int64_t key = (int64_t)(it >> 32);
        const int chunk = (int)(it & 0xffffffffull);
        const int o1 = p.obj_start[key + 1];
        const int o0 = p.obj_start[key] + chunk * kWave;
        const int b = batch_of_key(p.b_koff, p.n_batch, key);
        const int G = p.b_G[b];
        const int64_t base = p.b_koff[b];
        const int cell = (int)(key - base);
        const int ix = cell / (G * G), iy = (cell / G) % G, iz = cell % G;
        const double tr = p.t_ref[b];
        const double Asun = p.btab[kBatchStride * b + 14];
        // frame ranges of the 27 neighbouring cells, one per lane, and their
        // offsets in the concatenated neighbourhood list
        int my_a0 = 0, my_len = 0;
        if (lane < 27) {
            const int cx = ix + lane / 9 - 1, cy = iy + (lane / 3) % 3 - 1, cz = iz + lane % 3 - 1;
            if (cx >= 0 && cx < G && cy >= 0 && cy < G && cz >= 0 && cz < G) {
                const int64_t nk = base + ((int64_t)cx * G + cy) * G + cz;
                my_a0 = p.cell_start[nk];
                my_len = p.cell_start[nk + 1] - my_a0;
            }
        }
        int incl = my_len;
#pragma unroll
        for (int off = 1; off < 32; off <<= 1) {
            const int t = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += t;
        }
        const int excl = incl - my_len;
        const int total = __shfl(incl, 26, kWave);
        if (total == 0) continue;
        const int q = o0 + lane;
        const bool has = q < o1;
        const int64_t j = has ? p.obj_sorted[q] : 0;
        ObjBounds o;
#pragma unroll
        for (int c = 0; c < 3; ++c) { o.x[c] = 0.0; o.v[c] = 0.0; }
        o.taumax = o.vbn = o.a2b = 0.0;
        o.lin_ok = false;
        const bool live = has && object_bounds(p, b, j, o);
        if (__ballot(live) == 0ull) continue;
        // A cap around every live object's motion cap: centre ic the
        // normalized sum of their directions, cos of the radius the least
        // cos(A + theta) over them (A the angle of the object's direction
        // from ic, its sine from the cross product).  A frame whose cap
        // misses it can reach none of the item's objects.  Usable when
        // every A + theta stays below 90 degrees (else every frame is kept).
        double ic[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double v = live ? o.dh[c] : 0.0;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
            ic[c] = v;
        }
        bool item_cap = false;
        double icr = -1.0, isr = 1.0;        // cos and sin of the item cap's radius
        {
            const double in = sqrt(dot3(ic, ic));
            if (in > 0.0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) ic[c] /= in;
                double cA = 2.0;
                if (live) {
                    double cx[3];
                    cross3(ic, o.dh, cx);
                    const double ca = dot3(ic, o.dh), sa = sqrt(dot3(cx, cx));
                    cA = ca > 0.0 ? ca * o.cth - sa * o.sth : -2.0;
                }
                icr = wave_min(cA) - 1e-12;
                item_cap = icr > 0.0;
                isr = sqrt(fmax(0.0, 1.0 - icr * icr));
            }
        }
        // global object index; bit 63 set: no linear test
        const unsigned long long gtag = (unsigned long long)(p.b_obj0[b] + j) | (o.lin_ok ? 0ull : (1ull << 63));
        wave_lds_sync();                      // the previous item's queue is done
        int nq = 0;                           // queued (object, frame) pairs, wave-uniform
        // linear test of the first n queued pairs, one per lane
        auto drain = [&](int n) {
            const bool queued = lane < n;
            const unsigned long long e = queued ? queue[lane] : 0ull;
            const int src = (int)(e & 63);
            const int r = (int)(e >> 8);
            ObjBounds lo;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                lo.x[c] = __shfl(o.x[c], src, kWave);
                lo.v[c] = __shfl(o.v[c], src, kWave);
            }
            lo.taumax = __shfl(o.taumax, src, kWave);
            lo.vbn = __shfl(o.vbn, src, kWave);
            lo.a2b = __shfl(o.a2b, src, kWave);
            const unsigned long long g = __shfl(gtag, src, kWave);
            lo.lin_ok = (g >> 63) == 0ull;
            classify_emit(p, queued, lo, r, tr, Asun, g & ~(1ull << 63), buf, nbuf, pbuf, npbuf, n_exact);
        };
        for (int g0 = 0; g0 < total; g0 += kWave) {
            // lane l holds frame record g0 + l of the neighbourhood list
            const int g = g0 + lane;
            int nc = 0;
            for (int t = 1; t < 27; ++t) nc = (__shfl(excl, t, kWave) <= g) ? t : nc;
            const int rk = __shfl(my_a0, nc, kWave) + (g - __shfl(excl, nc, kWave));
            // the chunk's frame records that can meet the item's cap go to
            // LDS, packed, and are read back as broadcasts
            FrameRec rec = {{0.0, 0.0, 0.0}, 2.0, 0.0, 0.0, 0.0, {0.0, 0.0, 0.0}};
            bool keep = false;
            if (g < total) {
                const double* cp = caps + 8 * (int64_t)rk;
                const double2 c01 = *reinterpret_cast<const double2*>(cp);
                const double2 c23 = *reinterpret_cast<const double2*>(cp + 2);
                const double sr = cp[4];
                // cos of the angle between the caps' centres against
                // cos(R_item + R_f); frames of 90 degrees or more are kept
                keep = !item_cap || !(c23.y > 0.0) ||
                       !(c01.x * ic[0] + c01.y * ic[1] + c23.x * ic[2] < icr * c23.y - isr * sr - 1e-12);
                if (keep) {
                    const double2* ob = reinterpret_cast<const double2*>(p.cell_obs + 4 * (int64_t)rk);
                    const double2 o01 = ob[0], o23 = ob[1];
                    rec = {{c01.x, c01.y, c23.x}, c23.y, sr, (double)rk, o01.x, {o01.y, o23.x, o23.y}};
                }
            }
            const unsigned long long kmask = __ballot(keep);
            wave_lds_sync();                  // the previous chunk's records are read
            if (keep) fcap[__popcll(kmask & lt)] = rec;
            wave_lds_sync();
            const int n = __popcll(kmask);
            n_visit += (unsigned long long)n;
            for (int m = 0; m < n; ++m) {
                const FrameRec cm = fcap[m];
                const double cpm[5] = {cm.c[0], cm.c[1], cm.c[2], cm.cosr, cm.sinr};
                const unsigned long long rq = (unsigned long long)(unsigned int)(int)cm.rank;
                bool hit = live && frame_cap_hit(o, cpm);
                if (hit) {
                    if (o.lin_ok) {
                        const double ob[4] = {cm.t, cm.o[0], cm.o[1], cm.o[2]};
                        double ul[3];
                        const double e2 = lin_predict(o, ob, tr, Asun, ul);
                        hit = lin_cap_hit(cpm, ul, e2);
                    } else {
                        hit = loc_box_hit(p, o, (int)rq);
                    }
                }
                const unsigned long long mask = __ballot(hit);
                if (mask == 0ull) continue;
                if (hit) ++n_cand;
                if (hit) queue[nq + __popcll(mask & lt)] = (rq << 8) | (unsigned long long)lane;
                nq += __popcll(mask);
                if (nq >= kWave) {
                    wave_lds_sync();
                    drain(kWave);
                    // move the overflow to the front (fewer than 64 entries)
                    const unsigned long long rest = lane < nq - kWave ? queue[kWave + lane] : 0ull;
                    wave_lds_sync();
                    if (lane < nq - kWave) queue[lane] = rest;
                    nq -= kWave;
                    wave_lds_sync();
                }
            }
        }
        if (nq > 0) {
            wave_lds_sync();
            drain(nq);
        }
    }
    buf_flush(buf, nbuf, p.cand, p.n_cand, p.cand_cap);
    buf_flush(pbuf, npbuf, p.pairs, p.n_pairs, p.cap);
    if (p.stats) {
        unsigned long long a = n_cand, e = n_exact;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            a += __shfl_xor(a, off, 64);
            e += __shfl_xor(e, off, 64);
        }
        if (lane == 0) {
            atomicAdd(p.stats + 0, a);
            atomicAdd(p.stats + 1, e);
            atomicAdd(p.stats + 3, n_visit);
        }
    }
}

// Frame test of the wide join, one frame per lane: the motion-cap test, and
// for an object with a linear test the much tighter linear cap test (its
// frames are not shared across lanes, so each lane reads its own record);
// without one, the locator-box test.
__device__ __forceinline__ bool wide_frame_hit(const FovParams& p, const ObjBounds& o, int r, double tr, double Asun) {
    const double* cp = p.cell_caps + 8 * (size_t)(unsigned)r;
    if (!frame_cap_hit(o, cp)) return false;
    if (!o.lin_ok) return loc_box_hit(p, o, r);
    const double2* q = reinterpret_cast<const double2*>(p.cell_obs + 4 * (size_t)(unsigned)r);
    const double2 ob01 = q[0], ob23 = q[1];
    const double ob[4] = {ob01.x, ob01.y, ob23.x, ob23.y};
    double ul[3];
    const double e2 = lin_predict(o, ob, tr, Asun, ul);
    return lin_cap_hit(cp, ul, e2);
}

// Work units of wide object w: the cells of its cap box, or the frames of
// its batch when it has no usable cap (0 for a failed or non-finite
// object), and the parts they split into: one per 64 cells or
// kWidePartFrames frames, at most p.wide_max_parts.
__device__ __forceinline__ int wide_units(const FovParams& p, int64_t w, ObjBounds& o, int& b, int64_t& j,
                                          int& parts) {
    const unsigned long long e = p.wide[w];
    b = (int)(e >> 32);
    j = (int64_t)(e & 0xffffffffull);
    parts = 0;
    if (!object_bounds(p, b, j, o)) return 0;
    const int n = o.overflow ? p.cell_start[p.b_koff[b + 1]] - p.cell_start[p.b_koff[b]] : o.ncell;
    const int per = o.overflow ? kWidePartFrames : kWave;
    parts = min((n + per - 1) / per, p.wide_max_parts);
    return n;
}

__global__ void k_wide_parts(const FovParams p) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= p.n_pairs_total) return;
    const unsigned long long nw = *p.n_wide;
    int parts = 0;
    if ((unsigned long long)w < nw) {
        ObjBounds o;
        int b;
        int64_t j;
        wide_units(p, w, o, b, j, parts);
    }
    p.wide_parts[w] = parts;
}

// Wide objects, one part per wavefront at a time: the cap-box cells of a
// part (64 at most) or its frames of the batch for an object without a
// usable cap.  The frame records of a part's cells are dealt out 64 at a
// time across the lanes (a prefix sum of the cell lengths, then a binary
// search per lane), so empty and short cells cost nothing.  Frames that
// pass the cap test are queued in LDS and take the linear test 64 at a
// time, one per lane.  Parts are taken through per-XCD cursors, as in the
// per-cell join; a part's object is found by a 64-way search of the part
// offsets, the lanes probing together.
__global__ __launch_bounds__(256, kJoinWaves) void k_fov_wide(const FovParams p) {
    const int lane = threadIdx.x & 63, wv = (threadIdx.x >> 6) & 3;
    __shared__ int s_incl[4][kWave], s_base[4][kWave], s_queue[4][2 * kWave];
    __shared__ unsigned long long bufs[4][kBufEntries], pbufs[4][kPairBufEntries];
    int* incl_w = s_incl[wv];
    int* base_w = s_base[wv];
    int* queue = s_queue[wv];
    unsigned long long* buf = bufs[wv];
    unsigned long long* pbuf = pbufs[wv];
    const unsigned long long nw = *p.n_wide;
    const int n_obj_w = (int)(nw < (unsigned long long)p.n_pairs_total ? nw : p.n_pairs_total);
    const int n_parts = p.wide_off[p.n_pairs_total];
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int nbuf = 0, npbuf = 0;
    unsigned long long n_cand = 0, n_exact = 0, n_over = 0;
    const int home = (int)(blockIdx.x % kXcds);
    int tried = 0, part = 0, part_end = 0;
    int w = 0;                                   // object of the previous part
    for (;;) {
        if (part >= part_end) {
            while (tried < kXcds) {
                const int x = (home + tried) % kXcds;
                const int lo = (int)((int64_t)n_parts * x / kXcds), hi = (int)((int64_t)n_parts * (x + 1) / kXcds);
                int first = 0;
                if (lane == 0) first = (int)atomicAdd(p.wide_next + kCursorStride * x, 4u);
                first = __shfl(first, 0, kWave);
                if (first < hi - lo) {
                    part = lo + first;
                    part_end = min(part + 4, hi);
                    break;
                }
                ++tried;
            }
            if (tried >= kXcds) break;
        }
        const int pi = part++;
        // object w of part pi: the last w with wide_off[w] <= pi
        if (!(w < n_obj_w && p.wide_off[w] <= pi && pi < p.wide_off[w + 1])) {
            int lo = 0, hi = n_obj_w;               // wide_off[lo] <= pi < wide_off[hi]
            while (hi - lo > 1) {
                const int q = lo + (int)(((int64_t)(hi - lo) * (lane + 1)) >> 6);
                const bool le = lane < kWave - 1 && p.wide_off[q] <= pi;
                const unsigned long long m = __ballot(le);
                const int L = m ? 63 - __clzll((long long)m) : -1;
                const int nlo = L >= 0 ? __shfl(q, L, kWave) : lo;
                const int nhi = L + 1 < kWave - 1 ? __shfl(q, L + 1, kWave) : hi;
                lo = nlo;
                hi = nhi;
            }
            w = lo;
        }
        const int k = pi - p.wide_off[w];
        ObjBounds o;
        int b, parts;
        int64_t j;
        const int n_units = wide_units(p, w, o, b, j, parts);
        if (k >= parts) continue;
        // units [u0, u1) of the object's n_units
        const int u0 = (int)((int64_t)n_units * k / parts), u1 = (int)((int64_t)n_units * (k + 1) / parts);
        const unsigned long long gobj = (unsigned long long)(p.b_obj0[b] + j);
        const double tr = p.t_ref[b];
        const double Asun = p.btab[kBatchStride * b + 14];
        int nq = 0;                              // queued frames, wave-uniform
        // queue the frames (cell ranks) of the lanes with `hit`; run the
        // linear test on every full 64
        auto offer = [&](bool hit, int r) {
            const unsigned long long m = __ballot(hit);
            if (m == 0ull) return;
            if (hit) {
                ++n_cand;
                queue[nq + __popcll(m & lt)] = r;
            }
            nq += __popcll(m);
            if (nq >= kWave) {
                wave_lds_sync();
                const int fq = queue[lane];
                classify_emit(p, true, o, fq, tr, Asun, gobj, buf, nbuf, pbuf, npbuf, n_exact);
                // move the overflow to the front (fewer than 64 entries)
                const int rest = lane < nq - kWave ? queue[kWave + lane] : 0;
                wave_lds_sync();
                if (lane < nq - kWave) queue[lane] = rest;
                nq -= kWave;
                wave_lds_sync();
            }
        };
        if (o.overflow) {
            if (lane == 0 && k == 0) ++n_over;
            // frames u0 .. u1 - 1 of the batch, in cell order
            const int qb = p.cell_start[p.b_koff[b]];
            const int q1 = qb + u1;
            for (int q0 = qb + u0; q0 < q1; q0 += 64) {
                const int q = q0 + lane;
                const bool hit = q < q1 && wide_frame_hit(p, o, q, tr, Asun);
                offer(hit, q);
            }
        } else {
            const int G = p.b_G[b];
            const int ny = o.hi[1] - o.lo[1] + 1, nz = o.hi[2] - o.lo[2] + 1;
            const int64_t base = p.b_koff[b];
            for (int c0 = u0; c0 < u1; c0 += kWave) {
                const int c = c0 + lane;
                int a0 = 0, len = 0;
                if (c < u1) {
                    const int ix = o.lo[0] + c / (ny * nz);
                    const int iy = o.lo[1] + (c / nz) % ny;
                    const int iz = o.lo[2] + c % nz;
                    const int64_t key = base + (ix * G + iy) * G + iz;
                    a0 = p.cell_start[key];
                    len = p.cell_start[key + 1] - a0;
                }
                int incl = len;
#pragma unroll
                for (int off = 1; off < kWave; off <<= 1) {
                    const int t = __shfl_up(incl, off, kWave);
                    if (lane >= off) incl += t;
                }
                const int total = __shfl(incl, kWave - 1, kWave);
                if (total > 0) {
                    wave_lds_sync();                 // the previous chunk's searches are done
                    incl_w[lane] = incl;
                    base_w[lane] = a0 - (incl - len); // record of position t in this cell: base + t
                    wave_lds_sync();
                    for (int t0 = 0; t0 < total; t0 += kWave) {
                        const int t = t0 + lane;
                        // cell of position t: the first lane whose inclusive sum exceeds t
                        int i = 0;
#pragma unroll
                        for (int step = kWave / 2; step > 0; step >>= 1)
                            if (incl_w[i + step - 1] <= t) i += step;
                        int rq = 0;
                        bool hit = false;
                        if (t < total) {
                            rq = base_w[i] + t;
                            hit = wide_frame_hit(p, o, rq, tr, Asun);
                        }
                        offer(hit, rq);
                    }
                }
            }
        }
        if (nq > 0) {
            wave_lds_sync();
            const int fq = lane < nq ? queue[lane] : 0;
            classify_emit(p, lane < nq, o, fq, tr, Asun, gobj, buf, nbuf, pbuf, npbuf, n_exact);
            wave_lds_sync();
        }
    }
    buf_flush(buf, nbuf, p.cand, p.n_cand, p.cand_cap);
    buf_flush(pbuf, npbuf, p.pairs, p.n_pairs, p.cap);
    if (p.stats) {
        unsigned long long a = n_cand, e = n_exact;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            a += __shfl_xor(a, off, 64);
            e += __shfl_xor(e, off, 64);
        }
        if (lane == 0) {
            atomicAdd(p.stats + 0, a);
            atomicAdd(p.stats + 1, e);
            atomicAdd(p.stats + 2, n_over);
        }
    }
}

// Sky cell of every (object, batch): direction from the batch's mean
// observer, on the frame grid; wide and failed objects sort after the
// narrow ones of their batch.  The rank inside the cell comes from a
// block-local count (an LDS hash table of the block's keys) plus one
// global atomic per distinct key of the block, so objects sharing a cell
// do not queue on its global counter one by one.
constexpr int kKeyBlock = 256;
constexpr int kKeySlots = 2 * kKeyBlock;     // at most half full: probing always ends
// Sub-cell key of a narrow object: the Morton code of its direction's
// position on a kSubL^3 grid inside its sky cell, with the objects whose
// motion cap is wider than kFastCapSin after all the others, so that runs
// of the cell's objects in key order cover small patches of sky and share
// similar caps.
constexpr int kSubL = 8;
constexpr int kSubBits = 3;                  // log2(kSubL)
constexpr int kSubKeys = 2 * kSubL * kSubL * kSubL;
constexpr double kFastCapSin = 0.035;        // about 2 degrees
__device__ __forceinline__ int sub_cell_key(const ObjBounds& o, int G) {
    int m = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        int lc = cell_coord(o.dh[c], kSubL * G) - kSubL * cell_coord(o.dh[c], G);
        lc = lc < 0 ? 0 : (lc >= kSubL ? kSubL - 1 : lc);
#pragma unroll
        for (int k = 0; k < kSubBits; ++k) m |= ((lc >> k) & 1) << (3 * k + c);
    }
    return m | (o.sth > kFastCapSin ? kSubL * kSubL * kSubL : 0);
}

__global__ __launch_bounds__(kKeyBlock) void k_obj_keys(const FovParams p, int32_t* __restrict__ okey,
                                                        int32_t* __restrict__ orank, int32_t* __restrict__ cnt,
                                                        int32_t* __restrict__ osub) {
    __shared__ int32_t hkey[kKeySlots], hcnt[kKeySlots], hbase[kKeySlots];
    const int tid = threadIdx.x;
    for (int k = tid; k < kKeySlots; k += kKeyBlock) { hkey[k] = -1; hcnt[k] = 0; }
    __syncthreads();
    // block k takes chunk k / n_batch of batch k % n_batch: the blocks in
    // flight at any time spread over every batch, so that the per-cell
    // counters they update (disjoint between batches) are not all hit at
    // once
    const int b = (int)(blockIdx.x % (unsigned)p.n_batch);
    const int64_t j = (int64_t)(blockIdx.x / (unsigned)p.n_batch) * kKeyBlock + tid;
    const int64_t i = p.b_poff[b] + j;
    const bool valid = i < p.b_poff[b + 1];
    int slot = 0, lrank = 0;
    if (valid) {
        ObjBounds o;
        const int G = p.b_G[b], G3 = G * G * G;
        int key, sk;
        const bool live = object_bounds(p, b, j, o);
        if (live && is_narrow(o, G)) {
            key = (int)(p.b_koff[b] + cell_of(o.dh, G));
            sk = sub_cell_key(o, G);
        } else {
            // the batch's wide slot: wide objects ordered by a coarse sky
            // key (the Morton code of the direction on a kSubL^3 grid of the
            // whole sphere's cube), objects out of the join last
            key = (int)(p.b_koff[b] + G3);
            sk = live ? sub_cell_key(o, 1) : kSubKeys - 1;
        }
        okey[i] = key;
        osub[i] = sk;
        slot = (int)(((unsigned)key * 2654435761u) >> 23) & (kKeySlots - 1);
        for (;;) {
            const int prev = atomicCAS(&hkey[slot], -1, key);
            if (prev == -1 || prev == key) break;
            slot = (slot + 1) & (kKeySlots - 1);
        }
        lrank = atomicAdd(&hcnt[slot], 1);
    }
    __syncthreads();
    for (int k = tid; k < kKeySlots; k += kKeyBlock)
        if (hkey[k] >= 0) hbase[k] = atomicAdd(cnt + hkey[k], hcnt[k]);
    __syncthreads();
    if (valid) orank[i] = hbase[slot] + lrank;
}

// Objects into their cell's slots, at the rank the key pass drew (the order
// inside a cell is arbitrary: the pairs are sorted at the end).
__global__ void k_obj_scatter(const FovParams p, const int32_t* __restrict__ okey, const int32_t* __restrict__ orank,
                              const int32_t* __restrict__ start, int32_t* __restrict__ sorted) {
    // blocks map to (batch, chunk) as in k_obj_keys
    const int b = (int)(blockIdx.x % (unsigned)p.n_batch);
    const int64_t j = (int64_t)(blockIdx.x / (unsigned)p.n_batch) * blockDim.x + threadIdx.x;
    const int64_t i = p.b_poff[b] + j;
    if (i >= p.b_poff[b + 1]) return;
    sorted[start[okey[i]] + orank[i]] = (int32_t)j;
}

// Each sky cell's objects ordered by sub-cell key (counting sort in LDS,
// kCellSortCap objects at a time; longer cells are ordered chunk by chunk).
// The order of equal keys is arbitrary: the join's results do not depend on
// the order of a cell's objects, only its speed does.  Cells of fewer than
// two items' worth of objects are left as they are.  Each batch's wide slot
// is ordered the same way by its coarse sky key.
constexpr int kCellSortCap = 4096;

// One cell's objects sorted[s0, s1) by sub-cell key, by the whole block.
__device__ __forceinline__ void sort_cell(int s0, int s1, int64_t xo, int32_t* __restrict__ sorted,
                                          const int32_t* __restrict__ osub, int32_t* sj, int32_t* sk, int* cnt,
                                          int* wsum) {
    constexpr int kPer = kSubKeys / 256;
    static_assert(kPer * 256 == kSubKeys, "whole keys per thread");
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int c0 = s0; c0 < s1; c0 += kCellSortCap) {
        const int n = min(kCellSortCap, s1 - c0);
        for (int k = tid; k < kSubKeys; k += 256) cnt[k] = 0;
        __syncthreads();
        for (int i = tid; i < n; i += 256) {
            const int j = sorted[c0 + i];
            const int k = osub[xo + j];
            sj[i] = j;
            sk[i] = k;
            atomicAdd(&cnt[k], 1);
        }
        __syncthreads();
        int c[kPer], tot = 0;
#pragma unroll
        for (int q = 0; q < kPer; ++q) { c[q] = cnt[kPer * tid + q]; tot += c[q]; }
        int incl = tot;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int t = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += t;
        }
        if (lane == kWave - 1) wsum[wv] = incl;
        __syncthreads();
        int run = incl - tot;
        for (int w = 0; w < wv; ++w) run += wsum[w];
#pragma unroll
        for (int q = 0; q < kPer; ++q) { cnt[kPer * tid + q] = run; run += c[q]; }
        __syncthreads();
        for (int i = tid; i < n; i += 256) sorted[c0 + atomicAdd(&cnt[sk[i]], 1)] = sj[i];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_obj_cell_sort(const FovParams p, const int32_t* __restrict__ start,
                                                      int32_t* __restrict__ sorted, const int32_t* __restrict__ osub) {
    __shared__ int32_t sj[kCellSortCap], sk[kCellSortCap];
    __shared__ int cnt[kSubKeys];
    __shared__ int wsum[4];
    __shared__ unsigned long long s_need[4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // the block's threads look at 256 keys at once; the keys with more
    // than two items' worth of objects are then sorted one after another
    for (int64_t k0 = (int64_t)blockIdx.x * 256; k0 < p.n_keys; k0 += (int64_t)gridDim.x * 256) {
        const int64_t kt = k0 + tid;
        const bool need = kt < p.n_keys && start[kt + 1] - start[kt] > 2 * kWave;
        const unsigned long long m = __ballot(need);
        if (lane == 0) s_need[wv] = m;
        __syncthreads();
        unsigned long long need_w[4];
        for (int q = 0; q < 4; ++q) need_w[q] = s_need[q];
        __syncthreads();
        for (int q = 0; q < 4; ++q)
            for (unsigned long long mm = need_w[q]; mm != 0ull; mm &= mm - 1ull) {
                const int64_t key = k0 + 64 * q + (__ffsll((long long)mm) - 1);
                const int b = batch_of_key(p.b_koff, p.n_batch, key);
                sort_cell(start[key], start[key + 1], p.b_poff[b], sorted, osub, sj, sk, cnt, wsum);
            }
    }
}

// The wide list, batch-major: batch b's wide objects are its wide slot of
// the cell-sorted objects (sky-ordered, objects out of the join at the end,
// where the wide join gives them no parts).  k_wide_count writes each
// batch's count, a scan their offsets (wpos[B] = the total), k_wide_list
// copies the slots, one wavefront per batch, and sets the list's length.
__global__ void k_wide_count(const FovParams p, int32_t* __restrict__ cnt) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= p.n_batch) return;
    const int G = p.b_G[b];
    const int64_t kw = p.b_koff[b] + (int64_t)G * G * G;
    cnt[b] = p.obj_start[kw + 1] - p.obj_start[kw];
}
__global__ void k_wide_list(const FovParams p, const int32_t* __restrict__ wpos) {
    const int lane = threadIdx.x & 63;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t b = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; b < p.n_batch; b += n_waves) {
        const int G = p.b_G[b];
        const int64_t kw = p.b_koff[b] + (int64_t)G * G * G;
        const int q0 = p.obj_start[kw], n = p.obj_start[kw + 1] - q0, w0 = wpos[b];
        for (int q = lane; q < n; q += kWave)
            p.wide[w0 + q] = ((unsigned long long)b << 32) | (unsigned long long)(unsigned)p.obj_sorted[q0 + q];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *p.n_wide = (unsigned long long)wpos[p.n_batch];
}

// One exact-test record per frame (layout at FovParams::exact_rec), so
// that a candidate reaches everything its frame contributes in one round
// of loads and the light-time loop takes the Sun from a cubic.
__global__ void k_frame_exact_rec(const FovParams p) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= p.n_frames) return;
    double* R = p.exact_rec + (size_t)kExactRec * f;
    const int b = p.frame_batch[f];
    if (b < 0 || b >= p.n_batch) {
        for (int k = 0; k < kExactRec; ++k) R[k] = 0.0;
        return;
    }
    const EphemArgs& E = p.eph;
    const double tf = p.ft[f];
    const double* bt = p.btab + kBatchStride * b;
    const SunCubic S = sun_cubic(E.coef, 0, E.deg1, tf, E.t_start, E.seg_days, E.inv_seg, 0, E.n_seg - 1);
    R[0] = tf;
    R[1] = p.t_ref[b];
    for (int k = 0; k < 3; ++k) {
        R[2 + k] = p.fobs[3 * f + k];
        R[5 + k] = bt[k];
        R[8 + k] = bt[3 + k];
        R[12 + k] = S.s[k];
        R[15 + k] = S.v[k];
        R[18 + k] = S.a[k];
        R[21 + k] = S.j[k];
    }
    R[11] = __longlong_as_double((long long)(p.b_xoff[b] - 6 * (int64_t)p.b_obj0[b]));
}

// Exact test of every candidate (one lane per candidate, grid-stride): the
// candidate's sub-frame, or every sub-frame of its frame for kAllSubs.
// Each wavefront runs the same trips (lanes past the end idle), reads the
// next trip's candidate key ahead, and stages its pairs in LDS so that the
// shared pair counter takes one atomic per kPairBufEntries - 63 or more
// pairs.
__global__ __launch_bounds__(256) void k_fov_exact(const FovParams p) {
    __shared__ unsigned long long s_buf[4][kPairBufEntries];
    unsigned long long* buf = s_buf[threadIdx.x >> 6];
    int nbuf = 0;
    const unsigned long long nc = *p.n_cand;
    const unsigned long long n = nc < (unsigned long long)p.cand_cap ? nc : (unsigned long long)p.cand_cap;
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    const unsigned long long w0 = (unsigned long long)blockIdx.x * blockDim.x + (threadIdx.x & ~63u);
    unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long c_next = i < n ? p.cand[i] : 0ull;
    for (unsigned long long w = w0; w < n; w += stride, i += stride) {
        const bool valid = i < n;
        const unsigned long long c = c_next;
        c_next = i + stride < n ? p.cand[i + stride] : 0ull;
        const int f = (int)((c >> 32) & 0x7fffffffull);
        const int s0 = (int)((c >> 25) & 0x7full);
        const bool all_subs = (c & kAllSubs) != 0ull;
        const int j = (int)(c & 0x1ffffffull);              // global object
        bool ok = false;
        double d[3] = {0.0, 0.0, 0.0};
        if (valid) {
            const double2* R = reinterpret_cast<const double2*>(p.exact_rec + (size_t)kExactRec * f);
            double r[kExactRec];
#pragma unroll
            for (int k = 0; k < kExactRec / 2; ++k) {
                const double2 q = R[k];
                r[2 * k] = q.x;
                r[2 * k + 1] = q.y;
            }
            const double* st = p.x_epoch + __double_as_longlong(r[11]) + 6 * (int64_t)j;
            double r0[3], v0[3];
            for (int k = 0; k < 3; ++k) { r0[k] = st[k] - r[5 + k]; v0[k] = st[3 + k] - r[8 + k]; }
            const EphemArgs& E = p.eph;
            SunCubic sun = sun_table(E.coef, 0, E.deg1, E.t_start, E.seg_days, E.inv_seg, 0, E.n_seg - 1);
            sun.t0 = r[0];
            for (int k = 0; k < 3; ++k) {
                sun.s[k] = r[12 + k];
                sun.v[k] = r[15 + k];
                sun.a[k] = r[18 + k];
                sun.j[k] = r[21 + k];
            }
            const double o[3] = {r[2], r[3], r[4]};
            double tau, ve[3];
            const int kst = lighttime(sun, p.mu, p.smu, p.c_light, p.lt_tol, p.lt_iter, r[1], r0, v0, r[0], o, d,
                                      tau, ve, nullptr, p.kepler_iter);
            if (kst) {
                // the object fails: none of its pairs is kept (the host
                // drops those already appended by other candidates)
                p.fail[j] = 1;
                if (p.status_out) p.status_out[j] = KETE_ST_KEPLER_NOCONV;
                atomicAdd(p.n_fail, 1ull);
            }
            ok = kst == 0;
        }
        // sub-frame tests: one trip for single sub-frames, n_sub when a lane
        // of the wavefront tests a whole frame
        const int trips = __ballot(ok && all_subs) != 0ull ? p.n_sub : (__ballot(ok) != 0ull ? 1 : 0);
        const double* nrm = p.normals + (size_t)f * p.n_sub * 12;
        for (int t = 0; t < trips; ++t) {
            const int s = all_subs ? t : s0;
            bool in = false;
            if (ok && (all_subs || t == 0)) {
                const double* ns = nrm + 12 * s;
                in = dot3(ns, d) > 0.0 && dot3(ns + 3, d) > 0.0 && dot3(ns + 6, d) > 0.0 && dot3(ns + 9, d) > 0.0;
            }
            buf_append<kPairBufEntries>(buf, nbuf, in,
                                        ((unsigned long long)f << 32) | ((unsigned long long)s << 25) |
                                            (unsigned long long)j,
                                        p.pairs, p.n_pairs, p.cap);
        }
    }
    buf_flush(buf, nbuf, p.pairs, p.n_pairs, p.cap);
}

// ---------------------------------------------------------------- sort
// Pairs of objects whose hop failed somewhere in the call are dropped: the
// survivors are copied to `out` (in any order; the sort that follows
// fixes it) and counted in *n_out.
__global__ void k_pair_drop_failed(const unsigned long long* __restrict__ keys, int64_t n,
                                   const int32_t* __restrict__ fail, unsigned long long* __restrict__ out,
                                   unsigned long long* __restrict__ n_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool keep = i < n && fail[(int)(keys[i] & 0x1ffffffull)] == 0;
    const unsigned long long m = __ballot(keep);
    if (m == 0ull) return;
    const int lane = threadIdx.x & 63;
    unsigned long long base = 0;
    if (lane == __ffsll((long long)m) - 1) base = atomicAdd(n_out, (unsigned long long)__popcll(m));
    base = __shfl(base, __ffsll((long long)m) - 1, 64);
    if (keep) out[base + __popcll(m & ((1ull << lane) - 1ull))] = keys[i];
}

// Runs of equal frames among a wavefront's 64 consecutive keys (pairs are
// appended frame by frame, so runs are common): the head lane of each run
// gets the run's length, so the frame counters see one atomic per run.
struct FrameRun {
    int f;          // frame of this lane's key (-1 past the end)
    int head;       // lane heading this lane's run
    int len;        // run length (head lanes)
};
__device__ __forceinline__ FrameRun frame_run(unsigned long long key, bool valid) {
    const int lane = threadIdx.x & 63;
    FrameRun r;
    r.f = valid ? (int)(key >> 32) : -1;
    const int fp = __shfl_up(r.f, 1, 64);
    const bool is_head = valid && (lane == 0 || fp != r.f);
    const unsigned long long heads = __ballot(is_head);
    const int n_valid = __popcll(__ballot(valid));
    const unsigned long long upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    r.head = 63 - __clzll(heads & upto);
    const unsigned long long above = lane == 63 ? 0ull : (heads & ~upto);
    r.len = is_head ? ((above ? __ffsll((long long)above) - 1 : n_valid) - lane) : 0;
    return r;
}

// Each wavefront of the frame counting sort takes kRunChunks chunks of 64
// consecutive keys, all loaded before the first is used.  The runs of a
// block meet in an LDS table keyed by frame (open addressing, one slot per
// key of the block at most, so it never fills), and the frame counters see
// one atomic per frame of the block.
constexpr int kRunChunks = 4;
constexpr int kRunKeysPerBlock = 256 * kRunChunks;       // 256-thread blocks
constexpr int kRunSlots = kRunKeysPerBlock;

__device__ __forceinline__ int run_slot(int* hkey, int f) {
    int slot = (int)(((unsigned)f * 2654435761u) >> 22) & (kRunSlots - 1);
    for (;;) {
        const int prev = atomicCAS(&hkey[slot], -1, f);
        if (prev == -1 || prev == f) return slot;
        slot = (slot + 1) & (kRunSlots - 1);
    }
}

__global__ __launch_bounds__(256) void k_pair_hist(const unsigned long long* __restrict__ keys, int64_t n,
                                                   int32_t* __restrict__ fcnt) {
    __shared__ int hkey[kRunSlots], hcnt[kRunSlots];
    for (int k = threadIdx.x; k < kRunSlots; k += 256) { hkey[k] = -1; hcnt[k] = 0; }
    __syncthreads();
    const int64_t i0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * (kWave * kRunChunks) +
                       (threadIdx.x & 63);
    unsigned long long k[kRunChunks];
#pragma unroll
    for (int c = 0; c < kRunChunks; ++c) k[c] = i0 + kWave * c < n ? keys[i0 + kWave * c] : 0ull;
#pragma unroll
    for (int c = 0; c < kRunChunks; ++c) {
        const FrameRun r = frame_run(k[c], i0 + kWave * c < n);
        if (r.len > 0) atomicAdd(&hcnt[run_slot(hkey, r.f)], r.len);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kRunSlots; q += 256)
        if (hkey[q] >= 0) atomicAdd(fcnt + hkey[q], hcnt[q]);
}

// The keys of one frame differ only in (sub-frame, object): inside a
// frame's segment a key is sub << ob | obj, ob the bits of the object
// index (sub < 128, obj < 2^25, so ob + 7 <= 32 bits suffice).
__device__ __forceinline__ unsigned radix_key(unsigned long long k, int ob) {
    return ((unsigned)((k >> 25) & 0x7f) << ob) | ((unsigned)k & 0x1ffffffu);
}

// Each run takes its place in the block's share of its frame's segment
// from the LDS table, and each frame of the block takes that share with
// one atomic on the frame's cursor.
__global__ __launch_bounds__(256) void k_pair_scatter(const unsigned long long* __restrict__ keys, int64_t n,
                                                      const int32_t* __restrict__ fstart,
                                                      int32_t* __restrict__ fcur, int ob, unsigned* __restrict__ out) {
    __shared__ int hkey[kRunSlots], hcnt[kRunSlots];
    for (int q = threadIdx.x; q < kRunSlots; q += 256) { hkey[q] = -1; hcnt[q] = 0; }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t i0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * (kWave * kRunChunks) + lane;
    unsigned long long k[kRunChunks];
#pragma unroll
    for (int c = 0; c < kRunChunks; ++c) k[c] = i0 + kWave * c < n ? keys[i0 + kWave * c] : 0ull;
    FrameRun r[kRunChunks];
    int slot[kRunChunks], off[kRunChunks];
#pragma unroll
    for (int c = 0; c < kRunChunks; ++c) {
        r[c] = frame_run(k[c], i0 + kWave * c < n);
        slot[c] = 0;
        off[c] = 0;
        if (r[c].len > 0) {
            slot[c] = run_slot(hkey, r[c].f);
            off[c] = atomicAdd(&hcnt[slot[c]], r[c].len);
        }
    }
    __syncthreads();
    // hcnt becomes the block's base in each frame's segment
    for (int q = threadIdx.x; q < kRunSlots; q += 256)
        if (hkey[q] >= 0) hcnt[q] = fstart[hkey[q]] + atomicAdd(fcur + hkey[q], hcnt[q]);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kRunChunks; ++c) {
        const int pos = r[c].len > 0 ? hcnt[slot[c]] + off[c] : 0;
        const int b = __shfl(pos, r[c].head < 0 ? 0 : r[c].head, 64);
        if (i0 + kWave * c < n) out[b + (lane - r[c].head)] = radix_key(k[c], ob);
    }
}

// Pair i of frame f from its segment key k.
__device__ __forceinline__ void unpack_pair(unsigned k, int64_t f, int ob, int i, int32_t* __restrict__ pf,
                                            int32_t* __restrict__ ps, int32_t* __restrict__ po) {
    pf[i] = (int32_t)f;
    ps[i] = (int32_t)(k >> ob);
    po[i] = (int32_t)(ob >= 32 ? k : (k & ((1u << ob) - 1u)));
}

// Ordering inside each frame's segment of the pair keys (keys are unique),
// by segment size: up to kSortSmall by one thread (insertion sort), up to
// kSortWave by one wavefront in LDS (radix sort), up to kSortLds by a
// block in LDS (radix sort), larger ones by a block with bottom-up merge
// passes through global memory (merge-path partitions), ping-ponging with
// `tmp` at the same offsets.
constexpr int kSortSmall = 32;
constexpr int kSortWave = 1024;
constexpr int kSortLds = 8192;

__global__ void k_pair_sort_small(unsigned* __restrict__ keys, const int32_t* __restrict__ fstart,
                                  int64_t n_frames, int ob, int32_t* __restrict__ pf, int32_t* __restrict__ ps,
                                  int32_t* __restrict__ po) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n_frames) return;
    const int a = fstart[f], e = fstart[f + 1];
    if (e - a > kSortSmall) return;
    for (int i = a + 1; i < e; ++i) {
        const unsigned k = keys[i];
        int j = i - 1;
        while (j >= a && keys[j] > k) { keys[j + 1] = keys[j]; --j; }
        keys[j + 1] = k;
    }
    for (int i = a; i < e; ++i) unpack_pair(keys[i], f, ob, i, pf, ps, po);
}

// Stable LSD radix sort of one frame's keys by one wavefront in LDS.  The
// keys of a frame differ only in (sub-frame, object), packed here into
// bits = sb + ob <= 32 bits as sub << ob | obj.  Each pass of rb bits
// (the fewest passes of at most kMaxRadixBits, see radix_digit_bits)
// counts its digits with LDS atomics, scans the counts, then scatters the
// keys 64 at a time in order, a key's rank among the lanes sharing its
// digit coming from that digit's lane mask, so equal digits keep their
// order.
constexpr int kMaxRadixBits = 8;
constexpr int kRadixBuckets = 1 << kMaxRadixBits;

// Scatter of one chunk of up to 64 keys (lane l holds key k of digit d
// when v) to B at the digit cursors cnt, keeping the lanes' order among
// equal digits.  The lanes sharing a digit find each other through mk, a
// per-wavefront array of one 64-bit lane mask per digit that is all zero
// on entry and on exit: each lane ORs its bit into its digit's mask, reads
// the mask and the cursor back, and the lowest lane of each digit advances
// the cursor and clears the mask.  LDS instructions of one wavefront run in
// order, so the reads see every lane's OR and the old cursor; the fences
// only keep the compiler from reordering them.
__device__ __forceinline__ void radix_scatter_chunk(bool v, unsigned k, unsigned d, int* cnt,
                                                    unsigned long long* mk, unsigned* B, unsigned long long lt) {
    const int lane = threadIdx.x & 63;
    if (v) atomicOr(mk + d, 1ull << lane);
    wave_lds_sync();
    unsigned long long m = 0ull;
    int base = 0;
    if (v) {
        m = mk[d];
        base = cnt[d];
    }
    wave_lds_sync();
    if (v && (m & lt) == 0ull) {
        cnt[d] = base + __popcll(m);
        mk[d] = 0ull;
    }
    if (v) B[base + __popcll(m & lt)] = k;
    wave_lds_sync();
}

// Each wavefront sorts segments of up to kCap keys on its own; a lane
// keeps its keys of a pass in registers (key c * 64 + lane in slot c), so
// the pass scatters them back over the one LDS array they came from.
template <int kCap, int kWaves>
__global__ __launch_bounds__(64 * kWaves) void k_pair_sort_radix(const unsigned* __restrict__ keys,
                                                                const int32_t* __restrict__ fstart, int64_t n_frames,
                                                                int lo_n, int ob, int bits, int rb,
                                                                int32_t* __restrict__ pf, int32_t* __restrict__ ps,
                                                                int32_t* __restrict__ po) {
    constexpr int kChunks = kCap / kWave;
    __shared__ unsigned sh_a[kWaves][kCap];
    __shared__ int sh_cnt[kWaves][kRadixBuckets];
    __shared__ unsigned long long sh_mk[kWaves][kRadixBuckets];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const unsigned omask = ob >= 32 ? ~0u : ((1u << ob) - 1u);
    int* cnt = sh_cnt[wv];
    unsigned long long* mk = sh_mk[wv];
    unsigned* A = sh_a[wv];
    for (int d = lane; d < kRadixBuckets; d += kWave) mk[d] = 0ull;
    wave_lds_sync();
    const unsigned dm = (1u << rb) - 1u;
    for (int64_t f = (int64_t)blockIdx.x * kWaves + wv; f < n_frames; f += (int64_t)gridDim.x * kWaves) {
        const int a0 = fstart[f], n = fstart[f + 1] - a0;
        if (n <= lo_n || n > kCap) continue;
        unsigned kr[kChunks];
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            const int i = kWave * c + lane;
            kr[c] = i < n ? keys[a0 + i] : 0u;
        }
        for (int shift = 0; shift < bits; shift += rb) {
            if (shift > 0) {
#pragma unroll
                for (int c = 0; c < kChunks; ++c) {
                    const int i = kWave * c + lane;
                    kr[c] = i < n ? A[i] : 0u;
                }
            }
            for (int d = lane; d < kRadixBuckets; d += kWave) cnt[d] = 0;
            wave_lds_sync();
#pragma unroll
            for (int c = 0; c < kChunks; ++c)
                if (kWave * c + lane < n) atomicAdd(&cnt[(kr[c] >> shift) & dm], 1);
            wave_lds_sync();
            // exclusive scan of the counts, kRadixBuckets / 64 per lane
            constexpr int kPer = kRadixBuckets / kWave;
            int cc[kPer], tot = 0;
#pragma unroll
            for (int q = 0; q < kPer; ++q) { cc[q] = cnt[kPer * lane + q]; tot += cc[q]; }
            int incl = tot;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const int t = __shfl_up(incl, off, kWave);
                if (lane >= off) incl += t;
            }
            int run = incl - tot;
#pragma unroll
            for (int q = 0; q < kPer; ++q) { cnt[kPer * lane + q] = run; run += cc[q]; }
            wave_lds_sync();
#pragma unroll
            for (int c = 0; c < kChunks; ++c)
                if (kWave * c < n)
                    radix_scatter_chunk(kWave * c + lane < n, kr[c], (kr[c] >> shift) & dm, cnt, mk, A, lt);
        }
        for (int i = lane; i < n; i += kWave) {
            const unsigned k = A[i];
            pf[a0 + i] = (int32_t)f;
            ps[a0 + i] = (int32_t)(k >> ob);
            po[a0 + i] = (int32_t)(k & omask);
        }
        wave_lds_sync();
    }
}

// The same radix sort by a block of kSortWaves wavefronts per segment: per
// pass each wavefront counts the digits of its quarter of the keys (whole
// 64-key chunks, in order, held in registers), a block scan turns the
// per-wavefront counts into per-wavefront cursors (digit-major,
// wavefront-minor), and each wavefront scatters its quarter with its own
// cursors, so the order of equal digits is kept across the block.
constexpr int kSortWaves = 4;

template <int kCap>
__global__ __launch_bounds__(64 * kSortWaves) void k_pair_sort_radix_block(
    const unsigned* __restrict__ keys, const int32_t* __restrict__ fstart, int64_t n_frames, int lo_n,
    int ob, int bits, int rb, int32_t* __restrict__ pf, int32_t* __restrict__ ps, int32_t* __restrict__ po) {
    constexpr int kChunks = kCap / (kWave * kSortWaves);          // chunks of one wavefront at most
    __shared__ unsigned A[kCap];
    __shared__ int cnt[kSortWaves][kRadixBuckets];
    __shared__ unsigned long long sh_mk[kSortWaves][kRadixBuckets];
    __shared__ int wsum[kSortWaves];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int d = lane; d < kRadixBuckets; d += kWave) sh_mk[wv][d] = 0ull;
    wave_lds_sync();
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const unsigned omask = ob >= 32 ? ~0u : ((1u << ob) - 1u);
    constexpr int kPerT = kRadixBuckets / (64 * kSortWaves);      // digits per thread in the cursor scan
    static_assert(kPerT * 64 * kSortWaves == kRadixBuckets, "whole digits per thread");
    const unsigned dm = (1u << rb) - 1u;
    for (int64_t f = blockIdx.x; f < n_frames; f += gridDim.x) {
        const int a0 = fstart[f], n = fstart[f + 1] - a0;
        if (n <= lo_n || n > kCap) continue;
        // this wavefront's keys: chunks ca .. cb - 1 of 64 (at most kChunks)
        const int nc = (n + kWave - 1) / kWave;
        const int ca = nc * wv / kSortWaves, cb = nc * (wv + 1) / kSortWaves;
        unsigned kr[kChunks];
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            const int i = kWave * (ca + c) + lane;
            kr[c] = (ca + c < cb && i < n) ? keys[a0 + i] : 0u;
        }
        for (int shift = 0; shift < bits; shift += rb) {
            if (shift > 0) {
#pragma unroll
                for (int c = 0; c < kChunks; ++c) {
                    const int i = kWave * (ca + c) + lane;
                    kr[c] = (ca + c < cb && i < n) ? A[i] : 0u;
                }
            }
            for (int d = lane; d < kRadixBuckets; d += kWave) cnt[wv][d] = 0;
            wave_lds_sync();
#pragma unroll
            for (int c = 0; c < kChunks; ++c)
                if (ca + c < cb && kWave * (ca + c) + lane < n) atomicAdd(&cnt[wv][(kr[c] >> shift) & dm], 1);
            // (every wavefront has read its keys out of A before this barrier)
            __syncthreads();
            // thread tid: digits kPerT tid .. kPerT tid + kPerT - 1, their
            // total, its exclusive scan over the threads, then the cursors of
            // the digits and wavefronts in order
            int cc[kPerT][kSortWaves], tot = 0;
#pragma unroll
            for (int q = 0; q < kPerT; ++q)
#pragma unroll
                for (int w = 0; w < kSortWaves; ++w) { cc[q][w] = cnt[w][kPerT * tid + q]; tot += cc[q][w]; }
            int incl = tot;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const int t = __shfl_up(incl, off, kWave);
                if (lane >= off) incl += t;
            }
            if (lane == kWave - 1) wsum[wv] = incl;
            __syncthreads();
            int run = incl - tot;
            for (int w = 0; w < wv; ++w) run += wsum[w];
#pragma unroll
            for (int q = 0; q < kPerT; ++q)
#pragma unroll
                for (int w = 0; w < kSortWaves; ++w) { cnt[w][kPerT * tid + q] = run; run += cc[q][w]; }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < kChunks; ++c)
                if (ca + c < cb)
                    radix_scatter_chunk(kWave * (ca + c) + lane < n, kr[c], (kr[c] >> shift) & dm, cnt[wv],
                                        sh_mk[wv], A, lt);
            __syncthreads();
        }
        for (int i = tid; i < n; i += 64 * kSortWaves) {
            const unsigned k = A[i];
            pf[a0 + i] = (int32_t)f;
            ps[a0 + i] = (int32_t)(k >> ob);
            po[a0 + i] = (int32_t)(k & omask);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_pair_sort_large(unsigned* __restrict__ keys, unsigned* __restrict__ tmp,
                                                        const int32_t* __restrict__ fstart, int64_t n_frames,
                                                        int ob, int32_t* __restrict__ pf, int32_t* __restrict__ ps,
                                                        int32_t* __restrict__ po) {
    for (int64_t f = blockIdx.x; f < n_frames; f += gridDim.x) {
        const int a = fstart[f], n = fstart[f + 1] - a;
        if (n <= kSortLds) continue;
        unsigned* src = keys + a;
        unsigned* dst = tmp + a;
        for (int w = 1; w < n; w <<= 1) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const int p0 = (i / (2 * w)) * (2 * w);
                const int a1 = min(p0 + w, n), b1 = min(p0 + 2 * w, n);
                const int m = a1 - p0, m2 = b1 - a1, k = i - p0;
                int lo = max(0, k - m2), hi = min(k, m);
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (src[p0 + mid] < src[a1 + k - mid - 1]) lo = mid + 1; else hi = mid;
                }
                const unsigned va = lo < m ? src[p0 + lo] : ~0u;
                const unsigned vb = k - lo < m2 ? src[a1 + k - lo] : ~0u;
                dst[i] = va < vb ? va : vb;
            }
            __syncthreads();
            unsigned* t = src; src = dst; dst = t;
        }
        for (int i = threadIdx.x; i < n; i += blockDim.x) unpack_pair(src[i], f, ob, a + i, pf, ps, po);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- layout
__global__ void k_single_job_layout(int64_t* b_poff, int32_t* b_obj0, int64_t* b_xoff, int32_t* b_G, int64_t* b_koff,
                                    int64_t n_batch, int64_t n_obj, int G) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > n_batch) return;
    b_poff[b] = b * n_obj;
    b_koff[b] = b * ((int64_t)G * G * G + 1);
    if (b < n_batch) { b_obj0[b] = 0; b_xoff[b] = 6 * b * n_obj; b_G[b] = G; }
}

// Zero fill as a kernel (graph-capturable without memset nodes).
__global__ void k_fill_zero(unsigned int* __restrict__ p, size_t n_words) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ---------------------------------------------------------------- checks
__global__ __launch_bounds__(128) void k_directions(const FovParams p, const double* __restrict__ x_ref, double t_ref,
                             const double* __restrict__ t_obs, const double* __restrict__ obs, int64_t n_q,
                             double* __restrict__ d_out, double* __restrict__ tau_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)p.n_obj * n_q) return;
    const int64_t j = i % p.n_obj, qn = i / p.n_obj;
    const EphemArgs& E = p.eph;
    const SunTable sun{E.coef, 0, E.n_seg - 1, E.deg1, E.t_start, E.seg_days, E.inv_seg};
    double S[3], Sd[3];
    sun.eval(t_ref, S, Sd);
    const double* st = x_ref + 6 * j;
    double r0[3] = {st[0] - S[0], st[1] - S[1], st[2] - S[2]};
    double v0[3] = {st[3] - Sd[0], st[4] - Sd[1], st[5] - Sd[2]};
    SunCubic sun_e = sun_cubic(E.coef, 0, E.deg1, t_obs[qn], E.t_start, E.seg_days, E.inv_seg, 0, E.n_seg - 1);
    double d[3], tau, ve[3];
    const int kst = lighttime(sun_e, p.mu, p.smu, p.c_light, p.lt_tol, p.lt_iter, t_ref, r0, v0, t_obs[qn],
                              obs + 3 * qn, d, tau, ve, nullptr, p.kepler_iter);
    // a hop that ended on the Kepler iteration cap gives NaN
    for (int c = 0; c < 3; ++c) d_out[3 * i + c] = kst ? __builtin_nan("") : d[c];
    if (tau_out) tau_out[i] = kst ? __builtin_nan("") : tau;
}

__global__ void k_ephem_eval(EphemArgs E, const double* __restrict__ t, int64_t n_q, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_q * E.n_body) return;
    const int64_t qn = i / E.n_body;
    const int b = (int)(i % E.n_body);
    double pos[3], vel[3];
    cheb_body(E.coef + (size_t)b * E.n_seg * 3 * E.deg1, 0, E.deg1, t[qn], E.t_start, E.seg_days, E.inv_seg,
              0, E.n_seg - 1, pos, vel);
    for (int c = 0; c < 3; ++c) { out[6 * i + c] = pos[c]; out[6 * i + 3 + c] = vel[c]; }
}

}  // namespace

hipError_t fov_prepare(const FovParams& p, int32_t* qkey, int32_t* cnt, int32_t* cursor, void* scan_scratch,
                       hipStream_t s) {
    const int64_t n_keys = p.n_keys;
    const int64_t F = p.n_frames;
    const unsigned gF = (unsigned)((F + 255) / 256);
    hipError_t e;
    // one wavefront per frame, four per block
    const unsigned gw = (unsigned)std::min<int64_t>((F + 3) / 4, 65536);
    if (F > 0 && p.n_sub >= 8)
        hipLaunchKernelGGL(k_frame_caps, dim3(gw), dim3(256), 0, s, p.normals, F, p.n_sub, p.fcap);
    else if (F > 0)
        hipLaunchKernelGGL(k_frame_caps_lane, dim3(gF), dim3(256), 0, s, p.normals, F, p.n_sub, p.fcap);
    if (p.n_batch > 0) hipLaunchKernelGGL(k_batch_prep, dim3((unsigned)p.n_batch), dim3(256), 0, s, p);
    if ((e = fill_zero(cnt, (size_t)(n_keys + 1) * sizeof(int32_t), s)) != hipSuccess) return e;
    if (F > 0) hipLaunchKernelGGL(k_frame_keys, dim3(gF), dim3(256), 0, s, p, qkey, cnt);
    if ((e = exclusive_scan_i32(cnt, (int32_t*)p.cell_start, n_keys, scan_scratch, s)) != hipSuccess) return e;
    if ((e = fill_zero(cursor, (size_t)n_keys * sizeof(int32_t), s)) != hipSuccess) return e;
    if (F > 0) hipLaunchKernelGGL(k_frame_scatter, dim3(gF), dim3(256), 0, s, p, (const int32_t*)qkey, cursor);
    // the locator pass writes the cell-ordered frame copies itself
    if (F > 0 && !p.loc) hipLaunchKernelGGL(k_frame_gather, dim3(gw), dim3(256), 0, s, p);
    if (F > 0 && p.loc) hipLaunchKernelGGL(k_frame_locator, dim3(gw), dim3(256), 0, s, p);
    return hipGetLastError();
}

static int cu_count() {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
        ncu = 256;
    return ncu;
}

hipError_t fov_sort_objects(const FovParams& p, int32_t* okey, int32_t* orank, int32_t* cnt, int32_t* start,
                            int32_t* sorted, int32_t* osub, void* scan_scratch, hipStream_t s) {
    const int64_t n = p.n_pairs_total;
    const int64_t nkeys = p.n_keys;
    if (n == 0) return hipSuccess;
    hipError_t e;
    if ((e = fill_zero(cnt, (size_t)(nkeys + 1) * sizeof(int32_t), s)) != hipSuccess) return e;
    // one block per (batch, chunk of kKeyBlock objects)
    const int64_t chunks = (p.max_batch_obj + kKeyBlock - 1) / kKeyBlock;
    if (p.n_batch <= 0 || chunks <= 0) return hipSuccess;
    const unsigned gk = (unsigned)(p.n_batch * chunks);
    hipLaunchKernelGGL(k_obj_keys, dim3(gk), dim3(kKeyBlock), 0, s, p, okey, orank, cnt, osub);
    if ((e = exclusive_scan_i32(cnt, start, nkeys, scan_scratch, s)) != hipSuccess) return e;
    static_assert(kKeyBlock == 256, "the scatter uses the key pass's chunks");
    hipLaunchKernelGGL(k_obj_scatter, dim3(gk), dim3(256), 0, s, p, (const int32_t*)okey, (const int32_t*)orank,
                       (const int32_t*)start, sorted);
    hipLaunchKernelGGL(k_obj_cell_sort, dim3((unsigned)std::min<int64_t>(nkeys, (int64_t)cu_count() * 8)), dim3(256),
                       0, s, p, (const int32_t*)start, sorted, (const int32_t*)osub);
    return hipGetLastError();
}

hipError_t fov_single_job_layout(int64_t* b_poff, int32_t* b_obj0, int64_t* b_xoff, int32_t* b_G, int64_t* b_koff,
                                 int64_t n_batch, int64_t n_obj, int G, hipStream_t s) {
    hipLaunchKernelGGL(k_single_job_layout, dim3((unsigned)((n_batch + 1 + 255) / 256)), dim3(256), 0, s, b_poff,
                       b_obj0, b_xoff, b_G, b_koff, n_batch, n_obj, G);
    return hipGetLastError();
}

hipError_t fill_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    const size_t words = (bytes + 3) / 4;
    unsigned g = (unsigned)std::min<size_t>((words + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill_zero, dim3(g), dim3(256), 0, s, (unsigned int*)p, words);
    return hipGetLastError();
}

hipError_t fov_candidates(FovParams& p, int32_t* icnt, int32_t* istart, unsigned long long* items,
                          unsigned int* item_next, void* scan_scratch, void* wide_scan_scratch, hipStream_t s) {
    if (p.n_pairs_total == 0 || p.n_batch == 0) return hipSuccess;
    p.items = items;
    p.item_start = istart;
    p.item_next = item_next;
    const unsigned gk = (unsigned)((p.n_keys + 255) / 256);
    hipError_t e;
    hipLaunchKernelGGL(k_item_count, dim3(gk), dim3(256), 0, s, p, icnt);
    if ((e = exclusive_scan_i32(icnt, istart, p.n_keys, scan_scratch, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_item_scatter, dim3(gk), dim3(256), 0, s, p, (const int32_t*)icnt);
    if ((e = fill_zero(item_next, kJoinCursorWords * sizeof(unsigned int), s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_fov_cells, dim3((unsigned)(cu_count() * kJoinWaves)), dim3(256), 0, s, p);
    // the wide list, with the join's item counts as scratch (free now)
    hipLaunchKernelGGL(k_wide_count, dim3((unsigned)((p.n_batch + 255) / 256)), dim3(256), 0, s, p, icnt);
    if ((e = exclusive_scan_i32(icnt, istart, p.n_batch, scan_scratch, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_wide_list, dim3((unsigned)std::min<int64_t>((p.n_batch + 3) / 4, 65536)), dim3(256), 0, s, p,
                       (const int32_t*)istart);
    // parts per wide object: up to 32, fewer when the total could pass 2^31
    p.wide_max_parts = (int)std::max<int64_t>(1, std::min<int64_t>(32, (int64_t)(INT32_MAX - 1) / p.n_pairs_total));
    const unsigned gw = (unsigned)((p.n_pairs_total + 255) / 256);
    hipLaunchKernelGGL(k_wide_parts, dim3(gw), dim3(256), 0, s, p);
    if ((e = exclusive_scan_i32(p.wide_parts, p.wide_off, p.n_pairs_total, wide_scan_scratch, s)) != hipSuccess) return e;
    if ((e = fill_zero(p.wide_next, kJoinCursorWords * sizeof(unsigned int), s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_fov_wide, dim3((unsigned)(cu_count() * kJoinWaves)), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t fov_exact(const FovParams& p, hipStream_t s) {
    if (p.n_frames > 0)
        hipLaunchKernelGGL(k_frame_exact_rec, dim3((unsigned)((p.n_frames + 255) / 256)), dim3(256), 0, s, p);
    hipLaunchKernelGGL(k_fov_exact, dim3((unsigned)(cu_count() * 16)), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t fov_drop_failed(const unsigned long long* keys, int64_t n, const int32_t* fail, unsigned long long* out,
                           unsigned long long* n_out, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_pair_drop_failed, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, keys, n, fail, out,
                           n_out);
    return hipGetLastError();
}

// Bits needed for values 0 .. n - 1.
static int bits_for(int64_t n) {
    int b = 0;
    while (b < 62 && ((int64_t)1 << b) < n) ++b;
    return b;
}

// Digit width of the radix segment sorts for keys of `bits` bits: the
// fewest passes of at most kMaxRadixBits, split evenly (26 bits: 4 x 7).
static int radix_digit_bits(int bits) {
    const int passes = std::max(1, (bits + kMaxRadixBits - 1) / kMaxRadixBits);
    return std::max(1, (bits + passes - 1) / passes);
}

hipError_t fov_sort(unsigned long long* keys, int64_t n, int64_t n_frames, int64_t n_obj, int n_sub, int32_t* fcnt,
                    int32_t* fstart, unsigned long long* sorted, void* scan_scratch, int32_t* pf, int32_t* ps,
                    int32_t* po, hipStream_t s) {
    // the scatter writes 32-bit segment keys into `sorted`; `keys` is free
    // once they are scattered and holds the merge sort's second copy
    unsigned* seg = reinterpret_cast<unsigned*>(sorted);
    unsigned* tmp = reinterpret_cast<unsigned*>(keys);
    const int ob = bits_for(n_obj), bits = ob + bits_for(n_sub), rb = radix_digit_bits(bits);
    hipError_t e;
    if ((e = fill_zero(fcnt, (size_t)(n_frames + 1) * sizeof(int32_t), s)) != hipSuccess) return e;
    const unsigned run_blocks = (unsigned)((n + kRunKeysPerBlock - 1) / kRunKeysPerBlock);
    if (n > 0) hipLaunchKernelGGL(k_pair_hist, dim3(run_blocks), dim3(256), 0, s, keys, n, fcnt);
    if ((e = exclusive_scan_i32(fcnt, fstart, n_frames, scan_scratch, s)) != hipSuccess) return e;
    if ((e = fill_zero(fcnt, (size_t)n_frames * sizeof(int32_t), s)) != hipSuccess) return e;
    if (n > 0) hipLaunchKernelGGL(k_pair_scatter, dim3(run_blocks), dim3(256), 0, s, keys, n,
                                  (const int32_t*)fstart, fcnt, ob, seg);
    if (n_frames > 0) {
        const unsigned gb = (unsigned)std::min<int64_t>(n_frames, (int64_t)cu_count() * 16);
        hipLaunchKernelGGL(k_pair_sort_small, dim3((unsigned)((n_frames + 255) / 256)), dim3(256), 0, s, seg,
                           (const int32_t*)fstart, n_frames, ob, pf, ps, po);
        hipLaunchKernelGGL((k_pair_sort_radix<kSortWave, 4>), dim3(gb), dim3(256), 0, s, (const unsigned*)seg,
                           (const int32_t*)fstart, n_frames, kSortSmall, ob, bits, rb, pf, ps, po);
        hipLaunchKernelGGL((k_pair_sort_radix_block<4096>), dim3(gb), dim3(64 * kSortWaves), 0, s,
                           (const unsigned*)seg, (const int32_t*)fstart, n_frames, kSortWave, ob, bits, rb, pf, ps,
                           po);
        hipLaunchKernelGGL((k_pair_sort_radix_block<kSortLds>), dim3(gb), dim3(64 * kSortWaves), 0, s,
                           (const unsigned*)seg, (const int32_t*)fstart, n_frames, 4096, ob, bits, rb, pf, ps, po);
        hipLaunchKernelGGL(k_pair_sort_large, dim3(gb), dim3(256), 0, s, seg, tmp, (const int32_t*)fstart,
                           n_frames, ob, pf, ps, po);
    }
    return hipGetLastError();
}

hipError_t launch_directions(const FovParams& p, const double* x_ref, double t_ref, const double* t_obs,
                             const double* obs, int64_t n_q, double* d, double* tau, hipStream_t s) {
    const int64_t n = (int64_t)p.n_obj * n_q;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_directions, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, p, x_ref, t_ref, t_obs,
                       obs, n_q, d, tau);
    return hipGetLastError();
}

hipError_t launch_ephem_eval(const EphemArgs& E, const double* t, int64_t n_q, double* out, hipStream_t s) {
    const int64_t n = n_q * E.n_body;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ephem_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, E, t, n_q, out);
    return hipGetLastError();
}

}  // namespace kete
