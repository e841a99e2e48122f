// Batched execution engine (see ma_engine.h).
//
// Device side.  The per-node arithmetic of every phase (sweep update,
// residual, FAS restriction with the tau-corrected coarse right-hand side,
// prolongation, and their FP32 mixed-precision counterparts) is written once
// below as pt_* functions.  Two kernels drive them:
//   k_batched  single-wave blocks walk the work items of a BatchList, one
//              x-row segment of 64 nodes per item.  The items are split into
//              8 contiguous chunks, one per XCD (blocks are dispatched
//              round-robin over XCDs), so rows that read each other as
//              stencil halos are processed on one XCD and share its L2.
//   k_tail     one workgroup per solve runs all of that solve's coarse
//              levels (down, coarsest sweeps, up) with workgroup barriers
//              between phases, replacing dozens of tiny launches.
// Both call the same pt_* code, so a node's update is bitwise the same
// whichever kernel runs it; inside one colour phase the nodes are
// independent, so the order in which they are visited does not matter.
#include "ma_engine.h"
#include "ma_mixed_device.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>

namespace mafas {

namespace {

__device__ __forceinline__ double wave_sum64(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Per-node phases, written once over pointer types (global memory for the
// row kernels, LDS for the coarse-level kernel), so a node's result is
// bitwise the same whichever kernel computes it.  p is the node's linear
// index, (sy, sz) the strides of its grid.
// ---------------------------------------------------------------------------
template <int OP, typename PU>
__device__ __forceinline__ void sweep_node(PU u, double Fv, long p, long sy, long sz, double s,
                                           double hk, int slot,
                                           unsigned long long *__restrict__ ncount)
{
    if (OP == OP_MA) {
        const Hess g = hessian_at(u, p, 1, sy, sz, s, 0.25 * s);
        bool nc = false;
        u[p] = ma_point_update(g, u[p], Fv, hk, nc);
        if (nc)
            atomicAdd(ncount + slot, 1ull);
    } else {
        u[p] = lap_point_update(laplacian_at(u, p, 1, sy, sz, s), u[p], Fv, hk);
    }
}

// r = F - S(u) at node p of u with right-hand side value Fv.
template <int OP, typename PU>
__device__ __forceinline__ double resid_val(PU u, long p, long sy, long sz, double s, double Fv)
{
    if (OP == OP_MA)
        return Fv - det3(hessian_at(u, p, 1, sy, sz, s, 0.25 * s));
    return Fv - laplacian_at(u, p, 1, sy, sz, s);
}

template <int OP, typename PU, typename PF>
__device__ __forceinline__ double resid_node(PU u, PF F, long p, long sy, long sz, double s)
{
    return resid_val<OP>(u, p, sy, sz, s, F[p]);
}

// The same residual from the node's 3x3 neighbourhoods in the planes below,
// at and above it (D, C, U point at the centre; x stride 1, y stride 3),
// e.g. held in registers by a lane walking along z.
template <int OP>
__device__ __forceinline__ double resid_win(const double *D, const double *C, const double *U,
                                            double s, double Fv)
{
    if (OP == OP_MA)
        return Fv - det3(hessian3(D, C, U, 1, -1, 3, s, 0.25 * s));
    return Fv - laplacian3(D, C, U, 1, -1, 3, s);
}

// b_H at a coarse interior node: S_H(w_H) + I_h^H r (Algorithm 1, step 3),
// with w_H the injection of u.  The coarse node sits at fine index fu of uf
// (strides uy, uz) and fr of rf (strides ry, rz); sc = 1/H^2.
template <int OP, int RMODE, typename PU, typename PR>
__device__ __forceinline__ double restrict_b(PU uf, long fu, long uy, long uz, PR rf, long fr,
                                             long ry, long rz, double sc)
{
    double rh;
    if (RMODE == 0) {
        const double w[3] = {0.25, 0.5, 0.25};
        rh = 0.0;
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx)
                    rh += (w[dz + 1] * w[dy + 1] * w[dx + 1]) * rf[fr + dx + ry * dy + rz * dz];
    } else {
        rh = (6.0 * rf[fr] + (rf[fr - 1] + rf[fr + 1]) + (rf[fr - ry] + rf[fr + ry])
              + (rf[fr - rz] + rf[fr + rz])) / 12.0;
    }
    double sh;
    if (OP == OP_MA)
        sh = det3(hessian_at(uf, fu, 2, 2 * uy, 2 * uz, sc, 0.25 * sc));
    else
        sh = laplacian_at(uf, fu, 2, 2 * uy, 2 * uz, sc);
    return sh + rh;
}

// FAS restriction at coarse node (I, J, K) of the fine grid nf: injection
// of u into w_H and u_H, and b_H = S_H(w_H) + I_h^H r at coarse interior
// nodes, 0 on the boundary (Algorithm 1, step 3).
template <int OP, int RMODE, typename PU, typename PR, typename PO>
__device__ __forceinline__ void restrict_node(int nf, int I, int J, int K, PU uf, PR rf, PO wc,
                                              PO uc, PO bc)
{
    const int nc = nf / 2;
    const long fy = nf + 1, fz = fy * fy, cy = nc + 1, cz = cy * cy;
    const long f = 2 * I + fy * (2 * J) + fz * (2 * K);
    const long c = I + cy * J + cz * K;
    const double v = uf[f];
    wc[c] = v;
    uc[c] = v;
    double b = 0.0;
    if (I >= 1 && I <= nc - 1 && J >= 1 && J <= nc - 1 && K >= 1 && K <= nc - 1)
        b = restrict_b<OP, RMODE>(uf, f, fy, fz, rf, f, fy, fz, double(nc) * double(nc));
    bc[c] = b;
}

// Trilinear prolongation of the coarse correction (u_H - w_H) added at
// fine interior node (i, j, k) of the fine grid nf (Algorithm 1, step 5).
// T: double or float.  A node has one or two coarse neighbours along each
// axis (two where its index is odd), added in the order of loops over the
// (k, j, i) offsets.  The j and k parities are the same for a whole row, so
// one of four fixed shapes runs; inside it every load is issued before any
// is used (a lane with even i reads its first x neighbour again for the
// second, and the select drops it), and the sum is that of the plain loops.
template <int NJ, int NK, typename T, typename PC>
__device__ __forceinline__ T prolong_sum(long cy, long cz, int I0, int J0, int K0, int oi, T w,
                                         PC uc, PC wc)
{
    T e[NK * NJ * 2];
#pragma unroll
    for (int c = 0; c < NK; ++c)
#pragma unroll
        for (int b = 0; b < NJ; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const long q = (I0 + (a <= oi ? a : 0)) + cy * (J0 + b) + cz * (K0 + c);
                e[(c * NJ + b) * 2 + a] = uc[q] - wc[q];
            }
    T d = T(0);
#pragma unroll
    for (int c = 0; c < NK; ++c)
#pragma unroll
        for (int b = 0; b < NJ; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a)
                if (a <= oi)
                    d += w * e[(c * NJ + b) * 2 + a];
    return d;
}

template <typename T, typename PF, typename PC>
__device__ __forceinline__ void prolong_node(int nf, int i, int j, int k, PF uf, PC uc, PC wc)
{
    const int nc = nf / 2;
    const long sy = nf + 1, sz = sy * sy, cy = nc + 1, cz = cy * cy;
    const int oi = i & 1, oj = j & 1, ok = k & 1;
    const int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
    const long p = i + sy * j + sz * k;
    const T one = T(1), half = T(0.5);
    const T wi = oi ? half : one, wj = oj ? half : one, wk = ok ? half : one;
    const T w = wk * wj * wi;
    T d;
    if (oj == 0 && ok == 0)
        d = prolong_sum<1, 1, T>(cy, cz, I0, J0, K0, oi, w, uc, wc);
    else if (ok == 0)
        d = prolong_sum<2, 1, T>(cy, cz, I0, J0, K0, oi, w, uc, wc);
    else if (oj == 0)
        d = prolong_sum<1, 2, T>(cy, cz, I0, J0, K0, oi, w, uc, wc);
    else
        d = prolong_sum<2, 2, T>(cy, cz, I0, J0, K0, oi, w, uc, wc);
    uf[p] += d;
}

// The same prolongation for the 64 fine nodes i = 1 + 64 bx + t of one row
// kernel item, every lane of the wave taking part.  Lane t loads the coarse
// column its node starts from (i >> 1); a node with odd i also needs the next
// column, which is the column lane t + 1 starts from, so it takes that
// difference from lane t + 1 instead of loading it.  Half the coarse loads of
// prolong_node, and the same terms summed in the same order.
template <int NJ, int NK, typename T, typename PC>
__device__ __forceinline__ T prolong_sum_row(long cy, long cz, int X, int J0, int K0, int oi, T w,
                                             PC uc, PC wc)
{
    T a[NK * NJ], b[NK * NJ];
#pragma unroll
    for (int c = 0; c < NK; ++c)
#pragma unroll
        for (int m = 0; m < NJ; ++m) {
            const long q = X + cy * (J0 + m) + cz * (K0 + c);
            a[c * NJ + m] = uc[q];
            b[c * NJ + m] = wc[q];
        }
    T d = T(0);
#pragma unroll
    for (int c = 0; c < NK; ++c)
#pragma unroll
        for (int m = 0; m < NJ; ++m) {
            const T e0 = a[c * NJ + m] - b[c * NJ + m];
            const T e1 = __shfl_down(e0, 1, 64);
            d += w * e0;
            if (oi)
                d += w * e1;
        }
    return d;
}

template <typename T>
__device__ __forceinline__ void prolong_row(const GridItem &G, int bx, int t, int j, int k)
{
    const int nf = G.n, nc = nf / 2;
    const long sy = nf + 1, sz = sy * sy, cy = nc + 1, cz = cy * cy;
    const int i = 1 + bx * 64 + t;
    const int oi = i & 1, oj = j & 1, ok = k & 1;
    const int J0 = j >> 1, K0 = k >> 1;
    // i >> 1; clamped only for lanes past the end of the row, whose sums
    // are not used
    const int X = min(bx * 32 + (t >> 1) + (t & 1), nc);
    const T one = T(1), half = T(0.5);
    const T wi = oi ? half : one, wj = oj ? half : one, wk = ok ? half : one;
    const T w = wk * wj * wi;
    const auto uc = gptr<const T>(G.p[1]);
    const auto wc = gptr<const T>(G.p[2]);
    T d;
    if (oj == 0 && ok == 0)
        d = prolong_sum_row<1, 1, T>(cy, cz, X, J0, K0, oi, w, uc, wc);
    else if (ok == 0)
        d = prolong_sum_row<2, 1, T>(cy, cz, X, J0, K0, oi, w, uc, wc);
    else if (oj == 0)
        d = prolong_sum_row<1, 2, T>(cy, cz, X, J0, K0, oi, w, uc, wc);
    else
        d = prolong_sum_row<2, 2, T>(cy, cz, X, J0, K0, oi, w, uc, wc);
    if (i <= nf - 1)
        gptr<T>(G.p[0])[i + sy * j + sz * k] += d;
}

// The same phases on a grid of a device table (global memory).
template <int OP>
__device__ __forceinline__ void pt_sweep(const GridItem &G, long p, long sy, long sz,
                                         unsigned long long *__restrict__ ncount)
{
    sweep_node<OP>(gptr<double>(G.p[0]), gptr<const double>(G.p[1])[p], p, sy, sz, G.s, G.hk,
                   G.slot, ncount);
}

template <int OP>
__device__ __forceinline__ double pt_resid(const GridItem &G, long p, long sy, long sz)
{
    return resid_node<OP>(gptr<const double>(G.p[0]), gptr<const double>(G.p[1]), p, sy, sz,
                          G.s);
}

template <int OP, int RMODE>
__device__ __forceinline__ void pt_restrict(const GridItem &G, int I, int J, int K)
{
    restrict_node<OP, RMODE>(G.n, I, J, K, gptr<const double>(G.p[0]),
                             gptr<const double>(G.p[1]), gptr<double>(G.p[2]),
                             gptr<double>(G.p[3]), gptr<double>(G.p[4]));
}

template <typename T>
__device__ __forceinline__ void pt_prolong(const GridItem &G, int i, int j, int k)
{
    prolong_node<T>(G.n, i, j, k, gptr<T>(G.p[0]), gptr<const T>(G.p[1]), gptr<const T>(G.p[2]));
}

__device__ __forceinline__ void pt_msweep(const GridItem &G, long p, long sy, long sz,
                                          unsigned long long *__restrict__ ncount,
                                          unsigned long long *__restrict__ nfall)
{
    float *d = static_cast<float *>(G.p[0]);
    const float *b = static_cast<const float *>(G.p[1]);
    const double *U = static_cast<const double *>(G.p[2]);
    const LevelConst lc = level_const(G.n);
    bool fb = false, nc = false;
    d[p] = mixed_point(d, U, b[p], p, sy, sz, lc.s, lc.s4, lc.sf, lc.s4f, lc.hkf, fb, nc);
    if (fb)
        atomicAdd(nfall + G.slot, 1ull);
    if (nc)
        atomicAdd(ncount + G.slot, 1ull);
}

__device__ __forceinline__ void pt_mresid(const GridItem &G, long p, long sy, long sz)
{
    const float *d = static_cast<const float *>(G.p[0]);
    const float *b = static_cast<const float *>(G.p[1]);
    const double *U = static_cast<const double *>(G.p[2]);
    const LevelConst lc = level_const(G.n);
    const Sym32 H = to32(hessian_at(U, p, 1, sy, sz, lc.s, lc.s4));
    const Sym32 E = hess32(d, p, 1, sy, sz, lc.sf, lc.s4f);
    static_cast<float *>(G.p[3])[p] = b[p] - t_of(H, adj32(H), E);
}

template <int RMODE>
__device__ __forceinline__ void pt_mrestrict(const GridItem &G, int I, int J, int K)
{
    const int nf = G.n, nc = nf / 2;
    const float *df = static_cast<const float *>(G.p[0]);
    const float *rf = static_cast<const float *>(G.p[1]);
    const double *Uc = static_cast<const double *>(G.p[2]);
    const long fy = nf + 1, fz = fy * fy, cy = nc + 1, cz = cy * cy;
    const long f = 2 * I + fy * (2 * J) + fz * (2 * K);
    const long c = I + cy * J + cz * K;
    const float v = df[f];
    static_cast<float *>(G.p[3])[c] = v;
    static_cast<float *>(G.p[4])[c] = v;
    float bv = 0.0f;
    if (I >= 1 && I <= nc - 1 && J >= 1 && J <= nc - 1 && K >= 1 && K <= nc - 1) {
        float rh;
        if (RMODE == 0) {
            const float w[3] = {0.25f, 0.5f, 0.25f};
            rh = 0.0f;
#pragma unroll
            for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx)
                        rh += (w[dz + 1] * w[dy + 1] * w[dx + 1]) * rf[f + dx + fy * dy + fz * dz];
        } else {
            rh = (6.0f * rf[f] + (rf[f - 1] + rf[f + 1]) + (rf[f - fy] + rf[f + fy])
                  + (rf[f - fz] + rf[f + fz])) * (1.0f / 12.0f);
        }
        const LevelConst lcc = level_const(nc);
        const Sym32 H = to32(hessian_at(Uc, c, 1, cy, cz, lcc.s, lcc.s4));
        const Sym32 E = hess32(df, f, 2, 2 * fy, 2 * fz, lcc.sf, lcc.s4f);
        bv = t_of(H, adj32(H), E) + rh;
    }
    static_cast<float *>(G.p[5])[c] = bv;
}

// ---------------------------------------------------------------------------
// Row kernel: work item (bx, by, bz) of grid G, lane t.
// ---------------------------------------------------------------------------
// Colour rows: (bx, by, bz) -> node (i, j, k) of lane t.
template <int ORDER>
__device__ __forceinline__ void colour_row(int color, int bx, int by, int bz, int t, int &i,
                                           int &j, int &k)
{
    int i0;
    if (ORDER == 0) {
        const int c0 = color & 1, c1 = color >> 1;
        j = 1 + by;
        k = (((c0 + c1 + j) & 1) ? 1 : 2) + 2 * bz;
        i0 = ((c0 + j) & 1) ? 1 : 2;
    } else {
        j = ((color >> 1) & 1 ? 1 : 2) + 2 * by;
        k = ((color >> 2) & 1 ? 1 : 2) + 2 * bz;
        i0 = (color & 1) ? 1 : 2;
    }
    i = i0 + 2 * (bx * 64 + t);
}

template <int KIND, int OP, int ORDER, int RMODE>
__device__ __forceinline__ void run_item(const GridItem &G, int bx, int by, int bz, int color,
                                         int t, unsigned long long *__restrict__ ncount,
                                         unsigned long long *__restrict__ nfall)
{
    const int n = G.n;
    const long sy = n + 1, sz = sy * sy;
    if (KIND == LK_SWEEP || KIND == LK_MSWEEP) {
        int i, j, k;
        colour_row<ORDER>(color, bx, by, bz, t, i, j, k);
        if (i <= n - 1 && j <= n - 1 && k <= n - 1) {
            const long p = i + sy * j + sz * k;
            if (KIND == LK_SWEEP && ORDER == 0 && G.p[2]) {
                // colour-ordered F (ma_solver::fs): this row's values are
                // contiguous, so the phase reads F of its own colour only
                const long q = (long(bz) * G.gy + by) * G.gx + bx;
                const double Fv = gptr<const double>(G.p[2])[long(color) * G.pbase + 64 * q + t];
                sweep_node<OP>(gptr<double>(G.p[0]), Fv, p, sy, sz, G.s, G.hk, G.slot, ncount);
            } else if (KIND == LK_SWEEP) {
                pt_sweep<OP>(G, p, sy, sz, ncount);
            } else {
                pt_msweep(G, p, sy, sz, ncount, nfall);
            }
        }
    } else if (KIND == LK_NORM) {
        // Squared residuals of a 64-node row segment over kNormPlanes planes:
        // each lane walks along z keeping the 3x3 neighbourhoods of three
        // planes in registers, 9 loads per node instead of the 19 of the
        // gathered stencil.
        const int i = 1 + bx * 64 + t, j = 1 + by;
        const int k0 = 1 + bz * kNormPlanes, k1 = min(k0 + kNormPlanes, n);
        const int ic = min(i, n - 1);
        const auto u = gptr<const double>(G.p[0]);
        const auto F = gptr<const double>(G.p[1]);
        double P0[9], P1[9], P2[9];
        auto load = [&](double *P, int kk) {
            const long b0 = ic + sy * j + sz * kk;
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx)
                    P[(dy + 1) * 3 + (dx + 1)] = u[b0 + dx + sy * dy];
        };
        // the next plane's loads are issued before this plane's residual,
        // so each iteration's arithmetic overlaps the loads of the next
        double P3[9];
        load(P0, k0 - 1);
        load(P1, k0);
        load(P2, k0 + 1);   // k0 + 1 <= k1 <= n
        double fc = F[ic + sy * j + sz * k0];
        double acc = 0.0;
        for (int k = k0; k < k1; ++k) {
            double fn = 0.0;
            const bool more = k + 1 < k1;   // uniform across the wavefront
            if (more) {
                load(P3, k + 2);
                fn = F[ic + sy * j + sz * (k + 1)];
            }
            const double rv = resid_win<OP>(P0 + 4, P1 + 4, P2 + 4, G.s, fc);
            if (i <= n - 1)
                acc += rv * rv;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                P0[q] = P1[q];
                P1[q] = P2[q];
                P2[q] = P3[q];
            }
            fc = fn;
        }
        const double sum = wave_sum64(acc);
        if (t == 0)
            static_cast<double *>(G.p[2])[G.pbase + bx + G.gx * (by + G.gy * bz)] = sum;
    } else if (KIND == LK_RESIDUAL || KIND == LK_RES32) {
        const int i = 1 + bx * 64 + t, j = 1 + by, k = 1 + bz;
        double rv = 0.0;
        if (i <= n - 1) {
            const long p = i + sy * j + sz * k;
            rv = pt_resid<OP>(G, p, sy, sz);
            if (KIND == LK_RESIDUAL)
                gptr<double>(G.p[2])[p] = rv;
            if (KIND == LK_RES32)
                static_cast<float *>(G.p[2])[p] = float(rv);
        }
        if (KIND == LK_RES32) {
            const double sum = wave_sum64(rv * rv);
            if (t == 0) {
                const int local = bx + G.gx * (by + G.gy * bz);
                static_cast<double *>(G.p[3])[G.pbase + local] = sum;
            }
        }
    } else if (KIND == LK_RESTRICT || KIND == LK_MRESTRICT || KIND == LK_INJECT) {
        const int nc = n / 2;
        const int I = bx * 64 + t, J = by, K = bz;
        if (I <= nc) {
            if (KIND == LK_RESTRICT)
                pt_restrict<OP, RMODE>(G, I, J, K);
            else if (KIND == LK_MRESTRICT)
                pt_mrestrict<RMODE>(G, I, J, K);
            else {
                const long fy = n + 1, cy = nc + 1;
                static_cast<double *>(G.p[1])[I + cy * J + cy * cy * K] =
                    static_cast<const double *>(G.p[0])[2 * I + fy * (2 * J) + fy * fy * (2 * K)];
            }
        }
    } else if (KIND == LK_PROLONG || KIND == LK_MPROLONG) {
        // every lane takes part (lanes exchange coarse differences)
        if (KIND == LK_PROLONG)
            prolong_row<double>(G, bx, t, 1 + by, 1 + bz);
        else
            prolong_row<float>(G, bx, t, 1 + by, 1 + bz);
    } else if (KIND == LK_MRESIDUAL) {
        const int i = 1 + bx * 64 + t, j = 1 + by, k = 1 + bz;
        if (i <= n - 1)
            pt_mresid(G, i + sy * j + sz * k, sy, sz);
    } else if (KIND == LK_ACCUM) {
        const int i = 1 + bx * 64 + t, j = 1 + by, k = 1 + bz;
        if (i <= n - 1) {
            const long p = i + sy * j + sz * k;
            static_cast<double *>(G.p[0])[p] += double(static_cast<const float *>(G.p[1])[p]);
        }
    } else if (KIND == LK_ZERO) {
        const int i = bx * 64 + t, j = by, k = bz;
        if (i <= n)
            static_cast<float *>(G.p[0])[i + sy * j + sz * k] = 0.0f;
    }
}

// gridDim.x is a multiple of 8: gridDim.x / 8 blocks per XCD chunk.
template <int KIND, int OP, int ORDER, int RMODE>
__global__ __launch_bounds__(64) void k_batched(const BatchList *__restrict__ L, int color,
                                                unsigned long long *__restrict__ ncount,
                                                unsigned long long *__restrict__ nfall)
{
    const int bpx = int(gridDim.x >> 3);
    const int total = L->total;
    const int xcd = blockIdx.x & 7, lb = blockIdx.x >> 3;
    const int per = (total + 7) >> 3;
    const int lo = xcd * per;
    const int hi = min(total, lo + per);
    int it = lo + lb;
    if (it >= hi)
        return;
    const int ng = L->ngrids;
    int g0 = 0, g1 = ng - 1;  // last grid whose start <= it
    while (g0 < g1) {
        const int mid = (g0 + g1 + 1) >> 1;
        if (L->g[mid].start <= it)
            g0 = mid;
        else
            g1 = mid - 1;
    }
    int g = g0;
    const unsigned long long stopped = L->stopped;
    for (; it < hi; it += bpx) {
        while (g + 1 < ng && L->g[g + 1].start <= it)
            ++g;
        const GridItem G = L->g[g];   // the whole descriptor in one set of loads
        const int local = it - G.start;
        const int bx = local % G.gx;
        int rest = local / G.gx;
        const int jj = rest % G.w;
        rest /= G.w;
        const int bz = rest % G.gz;
        const int by = (rest / G.gz) * G.w + jj;
        // the stopped test after the descriptor's other fields, so they load
        // together
        if (by < G.gy && !((stopped >> G.slot) & 1ull))
            run_item<KIND, OP, ORDER, RMODE>(G, bx, by, bz, color, int(threadIdx.x), ncount,
                                             nfall);
    }
}

// fs[c * cs + 64 q + t] = F at the node of lane t of 4-colour row q of
// colour c (0 where the row runs past the grid): the right-hand side in the
// order the finest-level colour sweep reads it.  Block b = row q.
__global__ __launch_bounds__(64) void k_fsplit(int n, const double *__restrict__ F,
                                               double *__restrict__ fs, long cs, int gx, int gy)
{
    const int q = int(blockIdx.x), t = int(threadIdx.x);
    const int bx = q % gx, r = q / gx;
    const int by = r % gy, bz = r / gy;
    const long sy = n + 1, sz = sy * sy;
    const auto Fg = to_global(F);
    const auto out = to_global(fs);
    for (int c = 0; c < 4; ++c) {
        int i, j, k;
        colour_row<0>(c, bx, by, bz, t, i, j, k);
        const bool in = i <= n - 1 && j <= n - 1 && k <= n - 1;
        out[long(c) * cs + 64L * q + t] = in ? Fg[i + sy * j + sz * k] : 0.0;
    }
}

// Fixed-order per-grid sum of the partials of a norm list: thread t adds
// partials t, t + 1024, ... in order, then a fixed shuffle tree per wave and
// the 16 wave sums in order.  The sum of solve `slot` goes to the pinned
// host ring R: the k-th sum of a slot (k = R.seq[slot], counted on the
// device) lands in entry k mod kNormRing with its k stamped beside it.  When the
// slot's threshold is armed (thr >= 0), a sum at or below it, or one that is
// not finite, means the host's stopping test has passed: the slot's bit is
// set in the stopped mask of every list header, and the ticks already
// queued after this one skip the solve.
__global__ __launch_bounds__(1024) void k_batched_reduce(const BatchList *__restrict__ L,
                                                         const double *__restrict__ partials,
                                                         NormRing R)
{
    __shared__ double part[16];
    const int g = blockIdx.x;
    if (g >= L->ngrids)
        return;
    const GridItem &G = L->g[g];
    if ((L->stopped >> G.slot) & 1ull)
        return;
    const int cnt = G.gx * G.gy * G.gz;
    // the same additions in the same order as one add per step, with the
    // loads of eight steps in flight together
    const double *pp = partials + G.pbase;
    double v = 0.0;
    int q = int(threadIdx.x);
    for (; q + 7 * 1024 < cnt; q += 8 * 1024) {
        double a[8];
#pragma unroll
        for (int m = 0; m < 8; ++m)
            a[m] = pp[q + m * 1024];
#pragma unroll
        for (int m = 0; m < 8; ++m)
            v += a[m];
    }
    for (; q < cnt; q += 1024)
        v += pp[q];
    v = wave_sum64(v);
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < 16; ++w)
            s += part[w];
        const int slot = G.slot;
        const unsigned k = R.seq[slot];
        const int e = int(k % unsigned(kNormRing)) * kMaxGrids + slot;
        R.sum[e] = s;
        R.stamp[e] = k;
        R.seq[slot] = k + 1u;
        const double t = R.thr[slot];
        if (t >= 0.0 && (s <= t || !isfinite(s))) {
            const unsigned nh = R.stop[0];
            for (unsigned q = 0; q < nh; ++q)
                atomicOr(reinterpret_cast<unsigned long long *>(R.base + R.stop[1 + q] + 8),
                         1ull << slot);
        }
    }
}

// Arm solves for pipelined ticks: slot a.slot[q] takes threshold a.thr[q]
// (negative: never stop) and its bit cleared in every list header.
__global__ __launch_bounds__(64) void k_arm(ArmSet a, double *__restrict__ thr, char *base,
                                            const unsigned *__restrict__ stop)
{
    const int q = int(threadIdx.x);
    if (q < a.count) {
        thr[a.slot[q]] = a.thr[q];
        if (stop) {
            const unsigned nh = stop[0];
            for (unsigned h = 0; h < nh; ++h)
                atomicAnd(reinterpret_cast<unsigned long long *>(base + stop[1 + h] + 8),
                          ~(1ull << a.slot[q]));
        }
    }
}

// ---------------------------------------------------------------------------
// Coarse-level kernel: one workgroup runs the coarse end of one solve's
// V-cycle.  Nodes are enumerated densely per phase (a colour class has at
// most (n/2)^2 (n-1) or (n/2)^3 candidates), since the rows of a coarse
// grid are far shorter than a wavefront.
// ---------------------------------------------------------------------------
// Candidates of one colour class of an n grid: q < colour_count(n) -> node
// (i, j, k); true when the node is interior.
template <int ORDER>
__device__ __forceinline__ int colour_count(int n)
{
    const int hn = n / 2;
    return ORDER == 0 ? hn * hn * (n - 1) : hn * hn * hn;
}

template <int ORDER>
__device__ __forceinline__ bool colour_node(int n, int color, int q, int &i, int &j, int &k)
{
    const int hn = n / 2;
    const int ii = q % hn, r = q / hn;
    const int jj = r % hn, kk = r / hn;
    if (ORDER == 0) {
        const int c0 = color & 1, c1 = color >> 1;
        k = 1 + kk;
        j = (((c0 + c1 + k) & 1) ? 1 : 2) + 2 * jj;
        i = (((c0 + j) & 1) ? 1 : 2) + 2 * ii;
    } else {
        i = ((color & 1) ? 1 : 2) + 2 * ii;
        j = (((color >> 1) & 1) ? 1 : 2) + 2 * jj;
        k = (((color >> 2) & 1) ? 1 : 2) + 2 * kk;
    }
    return i <= n - 1 && j <= n - 1 && k <= n - 1;
}

template <int OP, bool MIXED, int ORDER>
__device__ __forceinline__ void tail_sweep(const GridItem &G, int color,
                                           unsigned long long *__restrict__ ncount,
                                           unsigned long long *__restrict__ nfall)
{
    const int n = G.n;
    const long sy = n + 1, sz = sy * sy;
    const int cnt = colour_count<ORDER>(n);
    for (int q = threadIdx.x; q < cnt; q += kTailThreads) {
        int i, j, k;
        if (colour_node<ORDER>(n, color, q, i, j, k)) {
            const long p = i + sy * j + sz * k;
            if (MIXED)
                pt_msweep(G, p, sy, sz, ncount, nfall);
            else
                pt_sweep<OP>(G, p, sy, sz, ncount);
        }
    }
}

template <int OP, bool MIXED>
__device__ __forceinline__ void tail_residual(const GridItem &G)
{
    const int n = G.n, m = n - 1;
    const long sy = n + 1, sz = sy * sy;
    const int cnt = m * m * m;
    for (int q = threadIdx.x; q < cnt; q += kTailThreads) {
        const int i = 1 + q % m, r = q / m;
        const int j = 1 + r % m, k = 1 + r / m;
        const long p = i + sy * j + sz * k;
        if (MIXED)
            pt_mresid(G, p, sy, sz);
        else
            static_cast<double *>(G.p[2])[p] = pt_resid<OP>(G, p, sy, sz);
    }
}

template <int OP, bool MIXED, int RMODE>
__device__ __forceinline__ void tail_restrict(const GridItem &G)
{
    const int m = G.n / 2 + 1;
    const int cnt = m * m * m;
    for (int q = threadIdx.x; q < cnt; q += kTailThreads) {
        const int I = q % m, r = q / m;
        const int J = r % m, K = r / m;
        if (MIXED)
            pt_mrestrict<RMODE>(G, I, J, K);
        else
            pt_restrict<OP, RMODE>(G, I, J, K);
    }
}

template <bool MIXED>
__device__ __forceinline__ void tail_prolong(const GridItem &G)
{
    const int m = G.n - 1;
    const int cnt = m * m * m;
    for (int q = threadIdx.x; q < cnt; q += kTailThreads) {
        const int i = 1 + q % m, r = q / m;
        const int j = 1 + r % m, k = 1 + r / m;
        if (MIXED)
            pt_prolong<float>(G, i, j, k);
        else
            pt_prolong<double>(G, i, j, k);
    }
}

// Every thread of the block reaches every barrier below: all loop bounds
// depend only on the block's table entry and the sweep counts.
template <int OP, bool MIXED, int ORDER, int RMODE>
__global__ __launch_bounds__(kTailThreads) void k_tail(const TailList *__restrict__ T, int nu1,
                                                       int nu2, int nu0,
                                                       unsigned long long *__restrict__ ncount,
                                                       unsigned long long *__restrict__ nfall)
{
    if (int(blockIdx.x) >= T->nsolves)
        return;
    const TailEntry &E = T->e[blockIdx.x];
    if ((T->stopped >> E.lv[0].sw.slot) & 1ull)
        return;
    const int L = E.nlev;
    constexpr int colours = ORDER == 0 ? 4 : 8;
    for (int l = 0; l < L; ++l) {
        const int cnt = l < L - 1 ? nu1 : nu0;
        for (int s = 0; s < cnt; ++s)
            for (int c = 0; c < colours; ++c) {
                tail_sweep<OP, MIXED, ORDER>(E.lv[l].sw, c, ncount, nfall);
                __syncthreads();
            }
        if (l < L - 1) {
            tail_residual<OP, MIXED>(E.lv[l].res);
            __syncthreads();
            tail_restrict<OP, MIXED, RMODE>(E.lv[l].rst);
            __syncthreads();
        }
    }
    for (int l = L - 2; l >= 0; --l) {
        tail_prolong<MIXED>(E.lv[l].pro);
        __syncthreads();
        for (int s = 0; s < nu2; ++s)
            for (int c = 0; c < colours; ++c) {
                tail_sweep<OP, MIXED, ORDER>(E.lv[l].sw, c, ncount, nfall);
                __syncthreads();
            }
    }
}

// Fused residual and FAS restriction (FP64 operators): one workgroup per
// TC^3 block of coarse nodes.  It loads the fine u it needs into LDS,
// computes r = F - S(u) once per fine node of the block's footprint into
// LDS, and restricts from LDS: injection into w_H and u_H and b_H =
// S_H(w_H) + I_h^H r.  The fine residual never goes through memory, and the
// arithmetic is that of resid_node and restrict_node, so the coarse arrays
// are bitwise those of the separate residual and restriction launches.
template <int TC>
struct RrShape {
    static constexpr int RU = 2 * TC + 3;    // u footprint per side (fine nodes)
    static constexpr int RR = 2 * TC + 1;    // r footprint per side
    // LDS row strides, padded to 4 mod 8 doubles: the restriction reads the
    // footprints at x stride 2, and rows of 4 mod 8 doubles spread the 4 x 4
    // coarse nodes of a plane over more LDS banks than rows of 11 or 9
    static constexpr int UX = RU + (12 - RU % 8) % 8, RX = RR + (12 - RR % 8) % 8;
    static constexpr int SU = UX * RU * RU, SR = RX * RR * RR;   // LDS doubles
};

template <int OP, int RMODE, int TC, int NT>
__global__ __launch_bounds__(NT) void k_rrestrict(const RrList *__restrict__ Lst)
{
    using R = RrShape<TC>;
    constexpr int RU = R::RU, RR = R::RR, UX = R::UX, RX = R::RX;
    __shared__ double su[R::SU];
    __shared__ double sr[R::SR];
    const int total = Lst->total;
    const int t = tile_of_block(int(blockIdx.x), int(gridDim.x));
    if (t >= total)
        return;
    const int ng = Lst->ngrids;
    int g = 0;
    while (g + 1 < ng && Lst->g[g + 1].start <= t)
        ++g;
    const RrGrid G = Lst->g[g];   // the whole descriptor in one set of loads
    if ((Lst->stopped >> G.slot) & 1ull)
        return;
    const int tile = t - G.start;
    const int nf = G.n, nc = nf / 2;
    const int tx = tile % G.tiles_x, rest = tile / G.tiles_x;
    const int ty = rest % G.tiles_y, tz = rest / G.tiles_y;
    const int I0 = tx * TC, J0 = ty * TC, K0 = tz * TC;
    const int ux0 = 2 * I0 - 2, uy0 = 2 * J0 - 2, uz0 = 2 * K0 - 2;   // u footprint origin
    const long fy = nf + 1, fz = fy * fy;
    const int tid = int(threadIdx.x);
    const auto uf = to_global(G.uf);
    const auto F = to_global(G.F);
    // A thread takes one column (x, y) of a footprint and a run of its
    // planes: the column's offset and bounds are worked out once, and each
    // plane adds a plane stride.  Every global load of a thread is issued
    // before the first is used; outside the grid a load reads node 0 and is
    // discarded.
    constexpr int CU2 = RU * RU, GU = NT / CU2, PU = (RU + GU - 1) / GU;   // u footprint
    constexpr int CR2 = RR * RR, GR = NT / CR2, PR = (RR + GR - 1) / GR;   // r footprint
    static_assert(GU >= 1 && GR >= 1, "a block covers every column of a footprint");
    {
        const int col = tid % CU2, grp = tid / CU2;
        const int lx = col % RU, ly = col / RU, lz0 = grp * PU;
        const int gx = ux0 + lx, gy = uy0 + ly;
        const bool cin = grp < GU && gx >= 0 && gx <= nf && gy >= 0 && gy <= nf;
        const long co = gx + fy * gy;
        double v[PU];
#pragma unroll
        for (int m = 0; m < PU; ++m) {
            const int gz = uz0 + lz0 + m;
            const bool in = cin && lz0 + m < RU && gz >= 0 && gz <= nf;
            const double x = uf[in ? co + fz * gz : 0];
            v[m] = in ? x : 0.0;
        }
#pragma unroll
        for (int m = 0; m < PU; ++m)
            if (grp < GU && lz0 + m < RU)
                su[lx + UX * (ly + RU * (lz0 + m))] = v[m];
    }
    // right-hand side of the fine interior nodes of the footprint (origin
    // ux0 + 1), for the planes of this thread's residual column, loaded while
    // the block waits at the barrier
    const int rcol = tid % CR2, rgrp = tid / CR2;
    const int rx = rcol % RR, ry = rcol / RR, rz0 = rgrp * PR;
    const int hx = ux0 + 1 + rx, hy = uy0 + 1 + ry;
    const bool rcin = rgrp < GR && hx >= 1 && hx <= nf - 1 && hy >= 1 && hy <= nf - 1;
    const long rco = hx + fy * hy;
    double fv[PR];
#pragma unroll
    for (int m = 0; m < PR; ++m) {
        const int gz = uz0 + 1 + rz0 + m;
        const bool in = rcin && rz0 + m < RR && gz >= 1 && gz <= nf - 1;
        fv[m] = F[in ? rco + fz * gz : 0];
    }
    lds_barrier();
    // r on the fine interior nodes of the footprint, walking the column up
    // its planes with the 3 x 3 neighbourhoods of three consecutive planes
    // in registers (the residual's expression is that of resid_val)
    if (rgrp < GR && rz0 < RR) {
        const double *cb = static_cast<const double *>(su) + (rx + 1) + UX * (ry + 1);
        auto win = [&](double *W, int pz) {
            const double *b = cb + UX * RU * pz;
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx)
                    W[(dy + 1) * 3 + (dx + 1)] = b[dx + UX * dy];
        };
        double P0[9], P1[9], P2[9];
        win(P0, rz0);
        win(P1, rz0 + 1);
#pragma unroll
        for (int m = 0; m < PR; ++m) {
            const int lz = rz0 + m;
            if (lz >= RR)
                break;
            win(P2, lz + 2);
            const int gz = uz0 + 1 + lz;
            double rv = 0.0;
            if (rcin && gz >= 1 && gz <= nf - 1)
                rv = resid_win<OP>(P0 + 4, P1 + 4, P2 + 4, G.s, fv[m]);
            sr[rx + RX * (ry + RR * lz)] = rv;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                P0[q] = P1[q];
                P1[q] = P2[q];
            }
        }
    }
    lds_barrier();
    const long cy = nc + 1, cz = cy * cy;
    const auto wc = to_global(G.wc);
    const auto uc = to_global(G.uc);
    const auto bc = to_global(G.bc);
    const double sc = double(nc) * double(nc);
    for (int el = tid; el < TC * TC * TC; el += NT) {
        const int a = el % TC, b2 = el / TC;
        const int I = I0 + a, J = J0 + b2 % TC, K = K0 + b2 / TC;
        if (I > nc || J > nc || K > nc)
            continue;
        const long fu = (2 * I - ux0) + UX * (2 * J - uy0) + long(UX * RU) * (2 * K - uz0);
        const long fr = (2 * I - ux0 - 1) + RX * (2 * J - uy0 - 1) + long(RX * RR) * (2 * K - uz0 - 1);
        const long c = I + cy * J + cz * K;
        const double v = su[fu];
        wc[c] = v;
        uc[c] = v;
        double bv = 0.0;
        if (I >= 1 && I <= nc - 1 && J >= 1 && J <= nc - 1 && K >= 1 && K <= nc - 1)
            bv = restrict_b<OP, RMODE>(static_cast<const double *>(su), fu, UX, UX * RU,
                                       static_cast<const double *>(sr), fr, RX, RX * RR, sc);
        bc[c] = bv;
    }
}

// Threads per tile: 256 when the launch has many tiles (throughput), 512
// when it has few (one tile's residual rounds are the latency).
constexpr int kRrManyTiles = 2048;

template <int OP, int RMODE>
hipError_t launch_rr_t(hipStream_t st, const RrList *L, int blocks)
{
    if (blocks >= kRrManyTiles)
        hipLaunchKernelGGL((k_rrestrict<OP, RMODE, kRrTile, 256>), dim3(blocks), dim3(256), 0, st, L);
    else
        hipLaunchKernelGGL((k_rrestrict<OP, RMODE, kRrTile, 512>), dim3(blocks), dim3(512), 0, st, L);
    return hipGetLastError();
}

// LDS form of the coarse-level kernel (FP64 operators only): the solve's
// coarse levels live in LDS for the whole launch -- the top level's u and
// b are loaded at entry and its u is written back at exit -- so every phase
// reads and writes LDS and the barriers order LDS only.  The phases and the
// per-node arithmetic are those of k_tail, so the results are bitwise the
// same.
template <int OP, int ORDER, int RMODE>
__global__ __launch_bounds__(kTailLdsThreads) void k_tail_lds(
    const TailList *__restrict__ T, int nu1, int nu2, int nu0,
    unsigned long long *__restrict__ ncount)
{
    __shared__ double S[kTailLdsDoubles];
    if (int(blockIdx.x) >= T->nsolves)
        return;
    const TailEntry &E = T->e[blockIdx.x];
    if ((T->stopped >> E.lv[0].sw.slot) & 1ull)
        return;
    const int L = E.nlev;
    const int tid = int(threadIdx.x);
    constexpr int NT = kTailLdsThreads;
    constexpr int colours = ORDER == 0 ? 4 : 8;
    auto npts3 = [](int n) { return (n + 1) * (n + 1) * (n + 1); };
    {
        const int N = npts3(E.lv[0].sw.n);
        const auto gu = gptr<const double>(E.lv[0].sw.p[0]);
        const auto gb = gptr<const double>(E.lv[0].sw.p[1]);
        double *u = S + E.L.u[0], *b = S + E.L.b[0];
        // five elements per thread with their loads in flight together (a
        // 17^3 top level is 4913 nodes)
        constexpr int KQ = 5;
        for (int q0 = 0; q0 < N; q0 += KQ * NT) {
            double vu[KQ], vb[KQ];
#pragma unroll
            for (int m = 0; m < KQ; ++m) {
                const int q = q0 + tid + m * NT;
                vu[m] = gu[q < N ? q : 0];
                vb[m] = gb[q < N ? q : 0];
            }
#pragma unroll
            for (int m = 0; m < KQ; ++m) {
                const int q = q0 + tid + m * NT;
                if (q < N) {
                    u[q] = vu[m];
                    b[q] = vb[m];
                }
            }
        }
    }
    lds_barrier();
    auto sweep = [&](int l) {
        const GridItem &G = E.lv[l].sw;
        const int n = G.n;
        const long sy = n + 1, sz = sy * sy;
        double *u = S + E.L.u[l];
        const double *b = S + E.L.b[l];
        const int cnt = colour_count<ORDER>(n);
        if (cnt <= NT) {
            // at most one candidate per thread: its position in the colour
            // class, the same for every colour, is decomposed once per sweep
            const int hn = n / 2;
            const int ii = tid % hn, r = tid / hn;
            const int jj = r % hn, kk = r / hn;
            for (int c = 0; c < colours; ++c) {
                int i, j, k;
                if (ORDER == 0) {
                    const int c0 = c & 1, c1 = c >> 1;
                    k = 1 + kk;
                    j = (((c0 + c1 + k) & 1) ? 1 : 2) + 2 * jj;
                    i = (((c0 + j) & 1) ? 1 : 2) + 2 * ii;
                } else {
                    i = ((c & 1) ? 1 : 2) + 2 * ii;
                    j = (((c >> 1) & 1) ? 1 : 2) + 2 * jj;
                    k = (((c >> 2) & 1) ? 1 : 2) + 2 * kk;
                }
                if (tid < cnt && i <= n - 1 && j <= n - 1 && k <= n - 1) {
                    const long p = i + sy * j + sz * k;
                    sweep_node<OP>(u, b[p], p, sy, sz, G.s, G.hk, G.slot, ncount);
                }
                lds_barrier();
            }
            return;
        }
        for (int c = 0; c < colours; ++c) {
            for (int q = tid; q < cnt; q += NT) {
                int i, j, k;
                if (colour_node<ORDER>(n, c, q, i, j, k))
                {
                    const long p = i + sy * j + sz * k;
                    sweep_node<OP>(u, b[p], p, sy, sz, G.s, G.hk, G.slot, ncount);
                }
            }
            lds_barrier();
        }
    };
    for (int l = 0; l < L; ++l) {
        const int cnt = l < L - 1 ? nu1 : nu0;
        for (int s = 0; s < cnt; ++s)
            sweep(l);
        if (l < L - 1) {
            const int n = E.lv[l].sw.n, m = n - 1;
            const long sy = n + 1, sz = sy * sy;
            const double *u = S + E.L.u[l], *b = S + E.L.b[l];
            double *r = S + E.L.r[l];
            for (int q = tid; q < m * m * m; q += NT) {
                const int i = 1 + q % m, rr = q / m;
                const int j = 1 + rr % m, k = 1 + rr / m;
                const long p = i + sy * j + sz * k;
                r[p] = resid_node<OP>(u, b, p, sy, sz, E.lv[l].sw.s);
            }
            lds_barrier();
            const int mc = n / 2 + 1;
            for (int q = tid; q < mc * mc * mc; q += NT) {
                const int I = q % mc, rr = q / mc;
                const int J = rr % mc, K = rr / mc;
                restrict_node<OP, RMODE>(n, I, J, K, static_cast<const double *>(u),
                                         static_cast<const double *>(r), S + E.L.w[l + 1],
                                         S + E.L.u[l + 1], S + E.L.b[l + 1]);
            }
            lds_barrier();
        }
    }
    for (int l = L - 2; l >= 0; --l) {
        const int n = E.lv[l].sw.n, m = n - 1;
        double *u = S + E.L.u[l];
        const double *uc = S + E.L.u[l + 1], *wc = S + E.L.w[l + 1];
        for (int q = tid; q < m * m * m; q += NT) {
            const int i = 1 + q % m, rr = q / m;
            const int j = 1 + rr % m, k = 1 + rr / m;
            prolong_node<double>(n, i, j, k, u, uc, wc);
        }
        lds_barrier();
        for (int s = 0; s < nu2; ++s)
            sweep(l);
    }
    {
        const int N = npts3(E.lv[0].sw.n);
        const auto gu = gptr<double>(E.lv[0].sw.p[0]);
        const double *u = S + E.L.u[0];
        for (int q = tid; q < N; q += NT)
            gu[q] = u[q];
    }
}

template <int OP, int ORDER>
hipError_t launch_tail_lds_t(hipStream_t st, int rmode, const TailList *T, int blocks, int nu1,
                             int nu2, int nu0, unsigned long long *nc)
{
    const dim3 grid(blocks), block(kTailLdsThreads);
    if (rmode == 0)
        hipLaunchKernelGGL((k_tail_lds<OP, ORDER, 0>), grid, block, 0, st, T, nu1, nu2, nu0, nc);
    else
        hipLaunchKernelGGL((k_tail_lds<OP, ORDER, 1>), grid, block, 0, st, T, nu1, nu2, nu0, nc);
    return hipGetLastError();
}

template <int KIND, int OP>
hipError_t launch_k(hipStream_t st, int order, int color, int rmode, const BatchList *L,
                    int blocks, unsigned long long *nc, unsigned long long *nf)
{
    const dim3 grid(blocks), block(64);
    if (order == 0) {
        if (rmode == 0)
            hipLaunchKernelGGL((k_batched<KIND, OP, 0, 0>), grid, block, 0, st, L, color, nc, nf);
        else
            hipLaunchKernelGGL((k_batched<KIND, OP, 0, 1>), grid, block, 0, st, L, color, nc, nf);
    } else {
        if (rmode == 0)
            hipLaunchKernelGGL((k_batched<KIND, OP, 1, 0>), grid, block, 0, st, L, color, nc, nf);
        else
            hipLaunchKernelGGL((k_batched<KIND, OP, 1, 1>), grid, block, 0, st, L, color, nc, nf);
    }
    return hipGetLastError();
}

template <int KIND>
hipError_t launch_kind(hipStream_t st, int op, int order, int color, int rmode, const BatchList *L,
                       int blocks, unsigned long long *nc, unsigned long long *nf)
{
    if (op == OP_MA)
        return launch_k<KIND, OP_MA>(st, order, color, rmode, L, blocks, nc, nf);
    return launch_k<KIND, OP_LAP>(st, order, color, rmode, L, blocks, nc, nf);
}

template <int OP, bool MIXED>
hipError_t launch_tail_t(hipStream_t st, int order, int rmode, const TailList *T, int blocks,
                         int nu1, int nu2, int nu0, unsigned long long *nc, unsigned long long *nf)
{
    const dim3 grid(blocks), block(kTailThreads);
    if (order == 0) {
        if (rmode == 0)
            hipLaunchKernelGGL((k_tail<OP, MIXED, 0, 0>), grid, block, 0, st, T, nu1, nu2, nu0, nc,
                               nf);
        else
            hipLaunchKernelGGL((k_tail<OP, MIXED, 0, 1>), grid, block, 0, st, T, nu1, nu2, nu0, nc,
                               nf);
    } else {
        if (rmode == 0)
            hipLaunchKernelGGL((k_tail<OP, MIXED, 1, 0>), grid, block, 0, st, T, nu1, nu2, nu0, nc,
                               nf);
        else
            hipLaunchKernelGGL((k_tail<OP, MIXED, 1, 1>), grid, block, 0, st, T, nu1, nu2, nu0, nc,
                               nf);
    }
    return hipGetLastError();
}

size_t npts_sz(int n) { return npts(n); }

} // namespace

void item_dims(int kind, int order, int n, int *gx, int *gy, int *gz)
{
    switch (kind) {
    case LK_SWEEP:
    case LK_MSWEEP:
        *gx = ((n + 1) / 2 + 63) / 64;
        *gy = order == 0 ? n - 1 : n / 2;
        *gz = n / 2;
        break;
    case LK_RESTRICT:
    case LK_MRESTRICT:
    case LK_INJECT: {
        const int nc = n / 2;
        *gx = (nc + 1 + 63) / 64;
        *gy = nc + 1;
        *gz = nc + 1;
        break;
    }
    case LK_ZERO:
        *gx = (n + 1 + 63) / 64;
        *gy = n + 1;
        *gz = n + 1;
        break;
    case LK_NORM:  // interior rows, planes in chunks of kNormPlanes
        *gx = (n - 1 + 63) / 64;
        *gy = n - 1;
        *gz = (n - 1 + kNormPlanes - 1) / kNormPlanes;
        break;
    default:  // interior rows
        *gx = (n - 1 + 63) / 64;
        *gy = n - 1;
        *gz = n - 1;
        break;
    }
}

hipError_t launch_batched(hipStream_t st, int kind, int op, int order, int color, int rmode,
                          const BatchList *L, int blocks, unsigned long long *nc,
                          unsigned long long *nf)
{
    if (blocks <= 0 || blocks % 8 != 0)
        return hipErrorInvalidValue;
    // kinds whose arithmetic does not depend on op / order / rmode use one
    // instantiation
    switch (kind) {
    case LK_SWEEP:
        return launch_kind<LK_SWEEP>(st, op, order, color, 0, L, blocks, nc, nf);
    case LK_RESIDUAL:
        return launch_kind<LK_RESIDUAL>(st, op, 0, 0, 0, L, blocks, nc, nf);
    case LK_NORM:
        return launch_kind<LK_NORM>(st, op, 0, 0, 0, L, blocks, nc, nf);
    case LK_RESTRICT:
        return launch_kind<LK_RESTRICT>(st, op, 0, 0, rmode, L, blocks, nc, nf);
    case LK_PROLONG:
        return launch_k<LK_PROLONG, OP_MA>(st, 0, 0, 0, L, blocks, nc, nf);
    case LK_MSWEEP:
        return launch_k<LK_MSWEEP, OP_MA>(st, order, color, 0, L, blocks, nc, nf);
    case LK_MRESIDUAL:
        return launch_k<LK_MRESIDUAL, OP_MA>(st, 0, 0, 0, L, blocks, nc, nf);
    case LK_MRESTRICT:
        return launch_k<LK_MRESTRICT, OP_MA>(st, 0, 0, rmode, L, blocks, nc, nf);
    case LK_MPROLONG:
        return launch_k<LK_MPROLONG, OP_MA>(st, 0, 0, 0, L, blocks, nc, nf);
    case LK_INJECT:
        return launch_k<LK_INJECT, OP_MA>(st, 0, 0, 0, L, blocks, nc, nf);
    case LK_ACCUM:
        return launch_k<LK_ACCUM, OP_MA>(st, 0, 0, 0, L, blocks, nc, nf);
    case LK_ZERO:
        return launch_k<LK_ZERO, OP_MA>(st, 0, 0, 0, L, blocks, nc, nf);
    case LK_RES32:
        return launch_k<LK_RES32, OP_MA>(st, 0, 0, 0, L, blocks, nc, nf);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_fsplit(hipStream_t st, int n, const double *F, double *fs, long cs)
{
    int gx, gy, gz;
    item_dims(LK_SWEEP, 0, n, &gx, &gy, &gz);
    if (long(gx) * gy * gz * 64 != cs || n < 2)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fsplit, dim3(gx * gy * gz), dim3(64), 0, st, n, F, fs, cs, gx, gy);
    return hipGetLastError();
}

hipError_t launch_batched_reduce(hipStream_t st, const BatchList *L, int grids,
                                 const double *partials, const NormRing &ring)
{
    if (grids < 1 || grids > kMaxGrids)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batched_reduce, dim3(grids), dim3(1024), 0, st, L, partials, ring);
    return hipGetLastError();
}

hipError_t launch_arm(hipStream_t st, const ArmSet &a, double *thr, char *base,
                      const unsigned *stop)
{
    if (a.count < 0 || a.count > kMaxGrids || (!base) != (!stop))
        return hipErrorInvalidValue;
    for (int q = 0; q < a.count; ++q)
        if (a.slot[q] < 0 || a.slot[q] >= kMaxGrids)
            return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_arm, dim3(1), dim3(64), 0, st, a, thr, base, stop);
    return hipGetLastError();
}

hipError_t launch_tail(hipStream_t st, int mode, int order, int rmode, const TailList *T,
                       int blocks, int nu1, int nu2, int nu0, unsigned long long *nc,
                       unsigned long long *nf)
{
    if (blocks <= 0 || blocks > kMaxGrids)
        return hipErrorInvalidValue;
    switch (mode) {
    case Engine::MODE_MA:
        return launch_tail_t<OP_MA, false>(st, order, rmode, T, blocks, nu1, nu2, nu0, nc, nf);
    case Engine::MODE_LAP:
        return launch_tail_t<OP_LAP, false>(st, order, rmode, T, blocks, nu1, nu2, nu0, nc, nf);
    case Engine::MODE_MIXED:
        return launch_tail_t<OP_MA, true>(st, order, rmode, T, blocks, nu1, nu2, nu0, nc, nf);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_rrestrict(hipStream_t st, int op, int rmode, const RrList *L, int blocks)
{
    if (blocks <= 0)
        return hipErrorInvalidValue;
    if (op == OP_MA)
        return rmode == 0 ? launch_rr_t<OP_MA, 0>(st, L, blocks) : launch_rr_t<OP_MA, 1>(st, L, blocks);
    return rmode == 0 ? launch_rr_t<OP_LAP, 0>(st, L, blocks) : launch_rr_t<OP_LAP, 1>(st, L, blocks);
}

hipError_t launch_tail_lds(hipStream_t st, int mode, int order, int rmode, const TailList *T,
                           int blocks, int nu1, int nu2, int nu0, unsigned long long *nc)
{
    if (blocks <= 0 || blocks > kMaxGrids)
        return hipErrorInvalidValue;
    if (mode != Engine::MODE_MA && mode != Engine::MODE_LAP)
        return hipErrorInvalidValue;
    const bool ma = mode == Engine::MODE_MA;
    if (order == 0)
        return ma ? launch_tail_lds_t<OP_MA, 0>(st, rmode, T, blocks, nu1, nu2, nu0, nc)
                  : launch_tail_lds_t<OP_LAP, 0>(st, rmode, T, blocks, nu1, nu2, nu0, nc);
    return ma ? launch_tail_lds_t<OP_MA, 1>(st, rmode, T, blocks, nu1, nu2, nu0, nc)
              : launch_tail_lds_t<OP_LAP, 1>(st, rmode, T, blocks, nu1, nu2, nu0, nc);
}

// ---------------------------------------------------------------------------
// Engine
// ---------------------------------------------------------------------------
Engine::~Engine()
{
    // ticks queued ahead may still run: drain the stream before freeing
    if (stream_)
        (void)hipStreamSynchronize(stream_);
    drop_graphs();
    for (hipEvent_t e : pev_)
        (void)hipEventDestroy(e);
    for (const Pending &p : fifo_)
        (void)hipEventDestroy(p.ev);
    for (hipEvent_t e : evpool_)
        (void)hipEventDestroy(e);
    if (ev_in_)
        (void)hipEventDestroy(ev_in_);
    if (stream_)
        (void)hipStreamDestroy(stream_);
    if (side_) {
        (void)hipStreamSynchronize(side_);
        (void)hipStreamDestroy(side_);
    }
    (void)hipFree(dl_);
    (void)hipFree(partials_);
    (void)hipFree(dcount_);
    (void)hipFree(dfall_);
    (void)hipFree(dseq_);
    (void)hipFree(dthr_);
    if (hstage_)
        (void)hipHostFree(hstage_);
    if (hnorm_)
        (void)hipHostFree(hnorm_);
    if (hstamp_)
        (void)hipHostFree(hstamp_);
    if (hcount_)
        (void)hipHostFree(hcount_);
}

void Engine::drop_graphs()
{
    for (int m = 0; m < kSlots; ++m) {
        for (hipGraphExec_t x : gseg_[m])
            if (x)
                (void)hipGraphExecDestroy(x);
        gseg_[m].clear();
        graph_shape_[m].clear();
        graph_dl_[m] = nullptr;
    }
}

#define E_HIP(expr)                                                                              \
    do {                                                                                         \
        const hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                                    \
            return fail(MA_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

ma_status Engine::set(const std::vector<SolveRef> &solves, hipStream_t user, bool graphs,
                      bool profile)
{
    if (solves.empty() || solves.size() > size_t(kMaxGrids))
        return fail(MA_ERR_ARG, "a batch holds 1 to 64 solves");
    const ma_params *p0 = nullptr;
    for (const SolveRef &r : solves) {
        if (!r.s)
            continue;
        if (!r.u || !r.f)
            return fail(MA_ERR_ARG, "null u or f in a batch");
        const ma_params &p = r.s->p;
        if (!p0)
            p0 = &p;
        else if (p.nu1 != p0->nu1 || p.nu2 != p0->nu2 || p.nu0 != p0->nu0 || p.order != p0->order ||
                 p.restriction != p0->restriction || p.precision != p0->precision ||
                 p.inner_cycles != p0->inner_cycles || p.coarse_n != p0->coarse_n ||
                 p.max_blocks != p0->max_blocks || p.strip_rows != p0->strip_rows ||
                 p.smoother != p0->smoother || p.tile_config != p0->tile_config ||
                 p.block_n != p0->block_n || p.zsweep_n != p0->zsweep_n ||
                 p.fuse_prolong != p0->fuse_prolong)
            return fail(MA_ERR_ARG,
                        "solvers in one batch must share smoothing counts, ordering, "
                        "restriction, precision, inner cycles, coarse_n, max_blocks, "
                        "strip_rows, smoother, tile_config, block_n, zsweep_n and "
                        "fuse_prolong");
    }
    if (!p0)
        return fail(MA_ERR_ARG, "a batch needs at least one solver");
    // ticks still queued: skipped ones are waited for; a live one is left by
    // a step that failed, and is dropped with the state resynchronised
    if (settle() != MA_OK)
        MA_TRY(abandon());
    // A captured tick reads the grids' operand pointers from the device
    // tables, which every rebuild rewrites; what it holds as a plain kernel
    // argument is the partials buffer, whose reallocation drops the graphs.
    solves_ = solves;
    user_dirty_ = true;
    fs_src_.assign(solves_.size(), nullptr);   // contents of f unknown: rebuild
    user_ = user;
    graphs_ = graphs;
    profile_ = profile;
    nu1_ = p0->nu1;
    nu2_ = p0->nu2;
    nu0_ = p0->nu0;
    order_ = p0->order;
    rmode_ = p0->restriction == MA_RESTRICT_HALF ? 1 : 0;
    inner_ = p0->inner_cycles;
    mixed_ = p0->precision == MA_MIXED;
    coarse_n_ = p0->coarse_n;
    max_blocks_ = p0->max_blocks > 0 ? p0->max_blocks : kDefaultMaxBlocks;
    strip_rows_ = p0->strip_rows;
    smoother_ = p0->smoother;
    tile_config_ = p0->tile_config;
    block_n_ = p0->block_n;
    zsweep_n_ = p0->zsweep_n;
    fuse_prolong_ = p0->fuse_prolong == 0;
    built_ = false;
    if (!stream_) {
        E_HIP(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
        E_HIP(hipEventCreateWithFlags(&ev_in_, hipEventDisableTiming));
        E_HIP(hipMalloc(reinterpret_cast<void **>(&dcount_), kMaxGrids * sizeof(unsigned long long)));
        E_HIP(hipMalloc(reinterpret_cast<void **>(&dfall_), kMaxGrids * sizeof(unsigned long long)));
        E_HIP(hipStreamCreateWithFlags(&side_, hipStreamNonBlocking));
        // The reduction kernel writes each tick's sums straight into these
        // pinned, coherent host buffers: no copy is queued after a tick, and
        // the host reads them once the tick's event has completed.
        E_HIP(hipHostMalloc(reinterpret_cast<void **>(&hnorm_),
                            kNormRing * kMaxGrids * sizeof(double),
                            hipHostMallocMapped | hipHostMallocCoherent));
        E_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&dnorm_), hnorm_, 0));
        E_HIP(hipHostMalloc(reinterpret_cast<void **>(&hstamp_),
                            kNormRing * kMaxGrids * sizeof(unsigned),
                            hipHostMallocMapped | hipHostMallocCoherent));
        E_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&dstamp_), hstamp_, 0));
        for (int e = 0; e < kNormRing * kMaxGrids; ++e)
            hstamp_[e] = ~0u;
        E_HIP(hipMalloc(reinterpret_cast<void **>(&dseq_), kMaxGrids * sizeof(unsigned)));
        E_HIP(hipMalloc(reinterpret_cast<void **>(&dthr_), kMaxGrids * sizeof(double)));
        E_HIP(hipMemsetAsync(dseq_, 0, kMaxGrids * sizeof(unsigned), stream_));
        ArmSet a;
        a.count = kMaxGrids;
        for (int i = 0; i < kMaxGrids; ++i) {
            a.slot[i] = i;
            a.thr[i] = -1.0;
        }
        E_HIP(launch_arm(stream_, a, dthr_, nullptr, nullptr));
        E_HIP(hipHostMalloc(reinterpret_cast<void **>(&hcount_),
                            2 * kMaxGrids * sizeof(unsigned long long)));
    }
    // partial sums: one per work item of the norm list of a tick, whose kind
    // is LK_NORM (FP64 and Poisson ticks) or LK_RES32 (mixed corrections)
    size_t need = 0;
    for (const SolveRef &r : solves_)
        if (r.s) {
            int gx, gy, gz, hx, hy, hz;
            item_dims(LK_NORM, 0, r.s->p.n, &gx, &gy, &gz);
            item_dims(LK_RES32, 0, r.s->p.n, &hx, &hy, &hz);
            need += std::max(size_t(gx) * gy * gz, size_t(hx) * hy * hz);
        }
    if (need > partials_cap_) {
        E_HIP(hipStreamSynchronize(stream_));
        drop_graphs();
        (void)hipFree(partials_);
        partials_ = nullptr;
        E_HIP(hipMalloc(reinterpret_cast<void **>(&partials_), need * sizeof(double)));
        partials_cap_ = need;
    }
    return MA_OK;
}

void Engine::rhs_changed(int i)
{
    if (i >= 0 && size_t(i) < fs_src_.size())
        fs_src_[i] = nullptr;
}

// Rebuild the colour-ordered right-hand side of every active solve whose
// finest-level colour sweeps read it and whose copy is not of the operand
// this mode uses (f for FAS cycles, R for the Poisson start).  Runs on the
// engine stream ahead of the tick, outside any captured graph.
ma_status Engine::refresh_fs(Mode mode, const std::vector<char> &active)
{
    if (mode == MODE_MIXED || order_ != 0)
        return MA_OK;
    for (size_t i = 0; i < solves_.size(); ++i) {
        ma_solver *sv = solves_[i].s;
        if (!sv || !active[i] || !sv->fs || multiblock_levels(int(i)) == 0)
            continue;
        const double *F = level_F(int(i), 0, mode);
        if (fs_src_[i] == F)
            continue;
        E_HIP(launch_fsplit(stream_, sv->lv[0].n, F, sv->fs, sv->fs_cs));
        fs_src_[i] = F;
    }
    return MA_OK;
}

ma_status Engine::reset_counters(int slot)
{
    MA_TRY(settle());
    if (slot < 0) {
        E_HIP(launch_fill_u64(stream_, kMaxGrids, 0ull, dcount_));
        E_HIP(launch_fill_u64(stream_, kMaxGrids, 0ull, dfall_));
    } else {
        E_HIP(launch_fill_u64(stream_, 1, 0ull, dcount_ + slot));
        E_HIP(launch_fill_u64(stream_, 1, 0ull, dfall_ + slot));
    }
    return MA_OK;
}

ma_status Engine::read_counters(std::vector<unsigned long long> &nonconvex,
                                std::vector<unsigned long long> &fallbacks)
{
    // With ticks queued ahead still on the engine stream, every solve in them
    // has stopped, so they leave the counters alone: read them on the side
    // stream instead of waiting for those ticks.  Everything queued before
    // them has completed (the host waited for the last tick it consumed).
    hipStream_t st = stream_;
    if (!fifo_.empty()) {
        for (const Pending &p : fifo_)
            for (size_t i = 0; i < solves_.size(); ++i)
                if (solves_[i].s && p.active[i] && !halted_[i])
                    return fail(MA_ERR_DEVICE, "internal: counters read with a live tick queued");
        st = side_;
    }
    E_HIP(hipMemcpyAsync(hcount_, dcount_, kMaxGrids * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, st));
    E_HIP(hipMemcpyAsync(hcount_ + kMaxGrids, dfall_, kMaxGrids * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, st));
    E_HIP(hipStreamSynchronize(st));
    nonconvex.assign(hcount_, hcount_ + solves_.size());
    fallbacks.assign(hcount_ + kMaxGrids, hcount_ + kMaxGrids + solves_.size());
    return MA_OK;
}

int Engine::levels(int i) const { return int(solves_[i].s->lv.size()); }

// Rows per y-strip: strip_rows when set, else 32 (a strip of 32 rows walked
// along z keeps ~20 planes of it in flight per XCD within the 4 MB L2).
int Engine::strip_width(int gy) const
{
    const int w = strip_rows_ > 0 ? strip_rows_ : 32;
    return std::max(1, std::min(w, gy));
}

// Block sweeps for a multi-block level of n intervals (4-colour FP64 only;
// the caller excludes MODE_MIXED).
bool Engine::block_level(int n, Mode mode) const
{
    if (order_ != MA_COLOR4 || smoother_ == MA_SMOOTHER_COLOR)
        return false;
    if (smoother_ == MA_SMOOTHER_FUSED || zs_level(n, mode))
        return true;
    const int lim = block_n_ == 0 ? 64 : block_n_;
    return n <= lim;
}

// Automatic choice (zsweep_n = 0), from whole-solve timings on MI355X: the
// z-stream sweep moves each node once per sweep but recomputes ~23% of the
// updates and waits on its barriers, and a grid needs enough 32 x 24
// columns to give every compute unit a chunk of planes; with the
// prolongation folded into the first post-smoothing sweep it pays from
// n = 192 (385^3 solve 68.8 -> 66.7 ms with level 192 as z-stream sweeps;
// Monge-Ampere sweeps 169 against 201 us at 257^3 and 564 against 801 us at
// 385^3, Poisson sweeps alike) but not at n = 128 (257^3 solve 22.1 against
// 23.0 ms, 129^3 6.0 against 7.1 ms).
bool Engine::zs_level(int n, Mode mode) const
{
    if (order_ != MA_COLOR4 || smoother_ != MA_SMOOTHER_AUTO)
        return false;
    const int lim = zsweep_n_ != 0 ? zsweep_n_ : (mode == MODE_LAP ? kZsweepAutoLap : kZsweepAuto);
    return lim > 0 && n >= lim;
}

int Engine::multiblock_levels(int i) const
{
    const ma_solver *s = solves_[i].s;
    int m = 0;
    while (m < int(s->lv.size()) && s->lv[m].n > coarse_n_)
        ++m;
    return m;
}

const double *Engine::level_u(int i, int l, Mode mode) const
{
    const ma_solver *s = solves_[i].s;
    if (mode == MODE_MIXED)
        return l == 0 ? solves_[i].u : s->mx[l].U;
    return l == 0 ? solves_[i].u : s->lv[l].u;
}

const double *Engine::level_F(int i, int l, Mode mode) const
{
    const ma_solver *s = solves_[i].s;
    if (l == 0)
        return mode == MODE_LAP ? s->R : solves_[i].f;
    return s->lv[l].b;
}

GridItem Engine::grid(int kind, int i, int l, Mode mode) const
{
    const ma_solver *s = solves_[i].s;
    GridItem G;
    std::memset(&G, 0, sizeof(G));
    const int n = (mode == MODE_MIXED) ? s->mx[l].n : s->lv[l].n;
    G.n = n;
    G.slot = i;
    G.s = double(n) * double(n);
    G.hk = mode == MODE_LAP ? 1.0 / (6.0 * G.s) : 0.5 / G.s;
    auto P = [](const void *q) { return const_cast<void *>(q); };
    switch (kind) {
    case LK_SWEEP:
        G.p[0] = P(level_u(i, l, mode));
        G.p[1] = P(level_F(i, l, mode));
        if (l == 0 && mode != MODE_MIXED && order_ == 0 && s->fs) {
            G.p[2] = s->fs;
            G.pbase = int(s->fs_cs);
        }
        break;
    case LK_RESIDUAL:
        G.p[0] = P(level_u(i, l, mode));
        G.p[1] = P(level_F(i, l, mode));
        G.p[2] = s->lv[l].r;
        break;
    case LK_RESTRICT:
        G.p[0] = P(level_u(i, l, mode));
        G.p[1] = s->lv[l].r;
        G.p[2] = s->lv[l + 1].w;
        G.p[3] = s->lv[l + 1].u;
        G.p[4] = s->lv[l + 1].b;
        break;
    case LK_PROLONG:
        G.p[0] = P(level_u(i, l, mode));
        G.p[1] = s->lv[l + 1].u;
        G.p[2] = s->lv[l + 1].w;
        break;
    case LK_NORM:
        G.p[0] = P(level_u(i, l, mode));
        G.p[1] = P(level_F(i, l, mode));
        G.p[2] = partials_;
        break;
    case LK_MSWEEP:
        G.p[0] = s->mx[l].d;
        G.p[1] = s->mx[l].b;
        G.p[2] = P(level_u(i, l, mode));
        break;
    case LK_MRESIDUAL:
        G.p[0] = s->mx[l].d;
        G.p[1] = s->mx[l].b;
        G.p[2] = P(level_u(i, l, mode));
        G.p[3] = s->mx[l].r;
        break;
    case LK_MRESTRICT:
        G.p[0] = s->mx[l].d;
        G.p[1] = s->mx[l].r;
        G.p[2] = s->mx[l + 1].U;
        G.p[3] = s->mx[l + 1].w;
        G.p[4] = s->mx[l + 1].d;
        G.p[5] = s->mx[l + 1].b;
        break;
    case LK_MPROLONG:
        G.p[0] = s->mx[l].d;
        G.p[1] = s->mx[l + 1].d;
        G.p[2] = s->mx[l + 1].w;
        break;
    case LK_INJECT:
        G.p[0] = P(level_u(i, l, mode));
        G.p[1] = s->mx[l + 1].U;
        break;
    case LK_ACCUM:
        G.p[0] = solves_[i].u;
        G.p[1] = s->mx[0].d;
        break;
    case LK_ZERO:
        G.p[0] = s->mx[0].d;
        break;
    case LK_RES32:
        G.p[0] = solves_[i].u;
        G.p[1] = P(solves_[i].f);
        G.p[2] = s->mx[0].b;
        G.p[3] = partials_;
        break;
    default:
        break;
    }
    return G;
}

// Builds the device tables of one tick of mode over the active solves.  A
// list's launch size comes from ALL solves of the engine (active or not), so
// it does not change when solves pause or finish, and neither does a
// captured graph that replays it.
ma_status Engine::rebuild(Mode mode, const std::vector<char> &active)
{
    hbuf_.clear();
    loff_.clear();
    lng_.clear();
    lgrid_.clear();
    stride_ = list_bytes(int(solves_.size()));
    const int S = int(solves_.size());
    auto on = [&](int i) { return solves_[i].s && active[i]; };
    D_ = Dall_ = 0;
    for (int i = 0; i < S; ++i)
        if (on(i)) {
            D_ = std::max(D_, multiblock_levels(i));
            Dall_ = std::max(Dall_, levels(i));
        }
    const bool mixed = mode == MODE_MIXED;
    bool overflow = false;
    int pnext = 0;
    // A list of kind at depth d over the solves for which pred holds and
    // which have a level d: a multi-block level when mb is set, any level
    // otherwise.
    auto make = [&](int kind, int d, bool mb, auto pred, bool partial) {
        BatchList L;
        L.ngrids = 0;
        L.total = 0;
        L.stopped = 0;
        int start = 0;
        long bound = 0;
        for (int i = 0; i < S; ++i) {
            if (!solves_[i].s || (mb ? multiblock_levels(i) : levels(i)) <= d || !pred(i))
                continue;
            int gx, gy, gz;
            const int n = mixed ? solves_[i].s->mx[d].n : solves_[i].s->lv[d].n;
            item_dims(kind, order_, n, &gx, &gy, &gz);
            const int w = strip_width(gy);
            const int items = padded_items(gx, gy, gz, w);
            bound += items;
            if (!active[i])
                continue;
            if (L.ngrids == kMaxGrids) {
                overflow = true;
                break;
            }
            GridItem G = grid(kind, i, d, mode);
            G.gx = gx;
            G.gy = gy;
            G.gz = gz;
            G.w = w;
            G.start = start;
            if (partial) {
                G.pbase = pnext;
                pnext += gx * gy * gz;
            }
            start += items;
            L.g[L.ngrids++] = G;
        }
        L.total = start;
        // every list sits at index * stride_, so a list's device address
        // depends only on its index
        const size_t off = loff_.size() * stride_;
        loff_.push_back(off);
        lng_.push_back(L.ngrids);
        const long b8 = ((bound + 7) / 8) * 8;
        lgrid_.push_back(bound == 0 ? 0 : int(std::min<long>(b8, max_blocks_)));
        hbuf_.resize(off + stride_, 0);
        std::memcpy(hbuf_.data() + off, &L, list_bytes(L.ngrids));
        return int(loff_.size()) - 1;
    };
    const int ksw = std::max(nu1_, nu0_);
    swd_.assign(D_, std::vector<int>());
    swu_.assign(D_, std::vector<int>());
    res_.assign(D_, -1);
    rst_.assign(D_, -1);
    pro_.assign(D_, -1);
    inj_.assign(std::max(Dall_ - 1, 0), -1);
    const int SW = mixed ? LK_MSWEEP : LK_SWEEP;
    for (int d = 0; d < D_; ++d) {
        for (int k = 0; k < ksw; ++k)
            swd_[d].push_back(make(SW, d, true, [&](int i) {
                const int cnt = d < levels(i) - 1 ? nu1_ : nu0_;
                return cnt > k;
            }, false));
        auto nc = [&](int i) { return d < levels(i) - 1; };
        res_[d] = make(mixed ? LK_MRESIDUAL : LK_RESIDUAL, d, true, nc, false);
        rst_[d] = make(mixed ? LK_MRESTRICT : LK_RESTRICT, d, true, nc, false);
        pro_[d] = make(mixed ? LK_MPROLONG : LK_PROLONG, d, true, nc, false);
        for (int k = 0; k < nu2_; ++k)
            swu_[d].push_back(make(SW, d, true, nc, false));
    }
    if (mixed)
        for (int d = 0; d + 1 < Dall_; ++d)
            inj_[d] = make(LK_INJECT, d, false, [&](int i) { return d < levels(i) - 1; }, false);
    auto all = [](int) { return true; };
    norm_ = make(mixed ? LK_RES32 : LK_NORM, 0, false, all, true);
    accum_ = zero_ = -1;
    if (mixed) {
        accum_ = make(LK_ACCUM, 0, false, all, false);
        zero_ = make(LK_ZERO, 0, false, all, false);
    }
    if (overflow)
        return fail(MA_ERR_ARG, "too many grids in one batched launch");
    if (size_t(pnext) > partials_cap_)
        return fail(MA_ERR_ARG, "partial-sum buffer too small for the batch");

    // coarse-level table, after the lists.  The LDS form of the coarse-level
    // kernel runs when every solve's coarse levels fit its LDS (decided over
    // all solves of the engine, so it does not change when solves pause).
    auto lds_layout = [&](int i, TailLds &Ld) {
        const int m = multiblock_levels(i), L = levels(i);
        int off = 0;
        for (int l = 0; l < kMaxTail; ++l) {
            Ld.u[l] = Ld.b[l] = Ld.w[l] = Ld.r[l] = -1;
            if (l >= L - m)
                continue;
            const int N = int(npts(solves_[i].s->lv[m + l].n));
            Ld.u[l] = off;
            off += N;
            Ld.b[l] = off;
            off += N;
            if (l > 0) {
                Ld.w[l] = off;
                off += N;
            }
            if (l < L - m - 1) {
                Ld.r[l] = off;
                off += N;
            }
        }
        return off <= kTailLdsDoubles;
    };
    tail_lds_ = !mixed;
    for (int i = 0; i < S && tail_lds_; ++i) {
        if (!solves_[i].s || levels(i) - multiblock_levels(i) <= 0)
            continue;
        TailLds Ld;
        tail_lds_ = levels(i) - multiblock_levels(i) <= kMaxTail && lds_layout(i, Ld);
    }
    toff_ = hbuf_.size();
    hbuf_.resize(toff_ + tail_bytes(S), 0);
    {
        TailList *T = reinterpret_cast<TailList *>(hbuf_.data() + toff_);
        int nt = 0, bound = 0;
        for (int i = 0; i < S; ++i) {
            if (!solves_[i].s)
                continue;
            const int m = multiblock_levels(i), L = levels(i);
            if (L - m <= 0)
                continue;
            if (L - m > kMaxTail)
                return fail(MA_ERR_ARG, "too many coarse levels for the coarse-level kernel");
            ++bound;
            if (!active[i])
                continue;
            TailEntry &E = T->e[nt++];
            E.nlev = L - m;
            E.lds = lds_layout(i, E.L) ? 1 : 0;
            for (int l = 0; l < L - m; ++l) {
                const int d = m + l;
                TailLevel &V = E.lv[l];
                V.sw = grid(mixed ? LK_MSWEEP : LK_SWEEP, i, d, mode);
                if (d < L - 1) {
                    V.res = grid(mixed ? LK_MRESIDUAL : LK_RESIDUAL, i, d, mode);
                    V.rst = grid(mixed ? LK_MRESTRICT : LK_RESTRICT, i, d, mode);
                    V.pro = grid(mixed ? LK_MPROLONG : LK_PROLONG, i, d, mode);
                }
            }
        }
        T->nsolves = nt;
        T->stopped = 0;
        tail_blocks_ = bound;
    }

    // Block-sweep lists, after the tail table.  Sweeps 2q and 2q + 1 of a
    // depth run as a block sweep u -> t followed by t -> u when the depth's
    // grids take block sweeps and every solve with that level takes part in
    // both sweeps.  Both decisions cover all solves of the engine, active or
    // not, so they do not change when solves pause or finish.
    fsoff_.clear();
    fsblocks_.clear();
    fscfg_.clear();
    fspro_.clear();
    pro_fused_.assign(D_, 0);
    fs_stride_ = fs_list_bytes(S);
    bsd_.assign(D_, std::vector<int>());
    bsu_.assign(D_, std::vector<int>());
    {
        const int op = mode == MODE_LAP ? OP_LAP : OP_MA;
        for (int d = 0; d < D_; ++d) {
            bool blk = !mixed;
            int nmax = 0;
            long tiles8 = 0;
            for (int i = 0; i < S && blk; ++i) {
                if (!solves_[i].s || multiblock_levels(i) <= d)
                    continue;
                const int n = solves_[i].s->lv[d].n;
                blk = block_level(n, mode);
                nmax = std::max(nmax, n);
                const long t = (n - 1 + 7) / 8;
                tiles8 += t * t * t;
            }
            // z-stream levels take a z-stream shape (tile_config 8..12, else
            // the automatic pick), the others a block shape (tile_config
            // 1..7, else the automatic pick)
            const bool zs = zs_level(nmax, mode) ||
                            (smoother_ == MA_SMOOTHER_FUSED && tile_config_ > kZsFirstConfig);
            int cfg;
            if (zs)
                cfg = tile_config_ >= kZsFirstConfig + 1 ? tile_config_ - 1 : bsweep_zs_pick(nmax);
            else if (tile_config_ > 0 && tile_config_ <= kZsFirstConfig)
                cfg = tile_config_ - 1;
            else
                cfg = bsweep_pick(nmax, tiles8);
            auto has = [&](int i) { return solves_[i].s && multiblock_levels(i) > d; };
            // up: the post-smoothing pairs, whose first z-stream sweep also
            // applies the coarse-grid correction (the solves in it are those
            // of the depth's prolongation list: a coarser level, nu2 > 0)
            auto pairs = [&](int nsw, auto count, std::vector<int> &out, bool up) {
                out.assign(nsw, -1);
                if (!blk)
                    return;
                for (int k = 0; k + 1 < nsw; k += 2) {
                    bool same = true;
                    for (int i = 0; i < S && same; ++i)
                        if (has(i))
                            same = (count(i) > k) == (count(i) > k + 1);
                    if (!same)
                        continue;
                    const bool pro = up && k == 0 && fuse_prolong_ && bsweep_is_zstream(cfg);
                    if (pro)
                        pro_fused_[d] = 1;
                    out[k] = int(fsoff_.size());
                    for (int half = 0; half < 2; ++half) {
                        FsList L;
                        L.ngrids = 0;
                        L.stopped = 0;
                        int start = 0;
                        long bound = 0;
                        for (int i = 0; i < S; ++i) {
                            if (!has(i) || count(i) <= k)
                                continue;
                            const ma_solver *sv = solves_[i].s;
                            double *u = const_cast<double *>(level_u(i, d, mode));
                            double *t = sv->lv[d].t;
                            FsGrid G;
                            bsweep_grid(cfg, sv->lv[d].n, half ? t : u, half ? u : t,
                                        level_F(i, d, mode), op, i, &G);
                            if (pro && half == 0) {
                                G.cu = sv->lv[d + 1].u;
                                G.cw = sv->lv[d + 1].w;
                            }
                            const int tiles = G.tiles_x * G.tiles_y * G.tiles_z;
                            bound += tiles;
                            if (!active[i])
                                continue;
                            G.start = start;
                            start += tiles;
                            L.g[L.ngrids++] = G;
                        }
                        L.total = start;
                        const size_t off = hbuf_.size();
                        fsoff_.push_back(off);
                        fsblocks_.push_back(int(bound));
                        fscfg_.push_back(cfg);
                        fspro_.push_back(pro && half == 0 ? 1 : 0);
                        hbuf_.resize(off + fs_stride_, 0);
                        std::memcpy(hbuf_.data() + off, &L, fs_list_bytes(L.ngrids));
                    }
                }
            };
            pairs(int(swd_[d].size()),
                  [&](int i) { return d < levels(i) - 1 ? nu1_ : nu0_; }, bsd_[d], false);
            pairs(int(swu_[d].size()), [&](int i) { return d < levels(i) - 1 ? nu2_ : 0; },
                  bsu_[d], true);
        }
    }

    // Fused residual-restriction lists, after the block-sweep lists: every
    // depth's residual and restriction in one launch (FP64 operators; the
    // COLOR smoother keeps the separate launches as the reference form).
    rroff_.clear();
    rrblocks_.clear();
    rr_stride_ = rr_list_bytes(S);
    rr_.assign(D_, -1);
    if (!mixed && smoother_ != MA_SMOOTHER_COLOR) {
        for (int d = 0; d < D_; ++d) {
            RrList Lr;
            Lr.ngrids = 0;
            Lr.stopped = 0;
            int start = 0;
            long bound = 0;
            for (int i = 0; i < S; ++i) {
                if (!solves_[i].s || multiblock_levels(i) <= d || d >= levels(i) - 1)
                    continue;
                const ma_solver *sv = solves_[i].s;
                RrGrid G;
                std::memset(&G, 0, sizeof(G));
                G.uf = level_u(i, d, mode);
                G.F = level_F(i, d, mode);
                G.wc = sv->lv[d + 1].w;
                G.uc = sv->lv[d + 1].u;
                G.bc = sv->lv[d + 1].b;
                G.n = sv->lv[d].n;
                G.slot = i;
                const int tc = (G.n / 2 + 1 + kRrTile - 1) / kRrTile;
                G.tiles_x = G.tiles_y = G.tiles_z = tc;
                G.s = double(G.n) * double(G.n);
                bound += long(tc) * tc * tc;
                if (!active[i])
                    continue;
                G.start = start;
                start += tc * tc * tc;
                Lr.g[Lr.ngrids++] = G;
            }
            Lr.total = start;
            if (bound == 0)
                continue;
            rr_[d] = int(rroff_.size());
            const size_t off = hbuf_.size();
            rroff_.push_back(off);
            rrblocks_.push_back(int(bound));
            hbuf_.resize(off + rr_stride_, 0);
            std::memcpy(hbuf_.data() + off, &Lr, rr_list_bytes(Lr.ngrids));
        }
    }

    // Byte offsets of every list header (count first): a solve that stops
    // sets its bit in each header's stopped mask (k_batched_reduce), arming
    // clears it (k_arm).  The upload writes every mask as zero.
    {
        std::vector<unsigned> offs(loff_.begin(), loff_.end());
        offs.push_back(unsigned(toff_));
        offs.insert(offs.end(), fsoff_.begin(), fsoff_.end());
        offs.insert(offs.end(), rroff_.begin(), rroff_.end());
        const unsigned cnt = unsigned(offs.size());
        stoff_ = (hbuf_.size() + 15) / 16 * 16;
        hbuf_.resize(stoff_ + sizeof(unsigned) * (1 + offs.size()), 0);
        std::memcpy(hbuf_.data() + stoff_, &cnt, sizeof(cnt));
        std::memcpy(hbuf_.data() + stoff_ + sizeof(cnt), offs.data(), sizeof(unsigned) * cnt);
    }

    prof_bytes_tick_ = 0.0;
    prof_launches_tick_ = 0;
    for (int i = 0; i < S; ++i)
        if (on(i) && multiblock_levels(i) > 0) {
            const double in = interior(mixed ? solves_[i].s->mx[0].n : solves_[i].s->lv[0].n);
            const bool single = levels(i) == 1;
            const int sweeps = single ? nu0_ : nu1_ + nu2_;
            const int reps = mixed ? inner_ : 1;
            prof_bytes_tick_ += reps * sweeps * (mixed ? 20.0 : 24.0) * in;
            // a sweep that also prolongs reads the coarse u and w
            if (D_ > 0 && pro_fused_[0] && !single)
                prof_bytes_tick_ += 16.0 * double(npts(solves_[i].s->lv[1].n));
        }
    if (D_ > 0) {
        const int reps = mixed ? inner_ : 1;
        const int colours = order_ == 1 ? 8 : 4;
        int launches = 0;
        auto count = [&](const std::vector<int> &lists, const std::vector<int> &pairs) {
            for (size_t k = 0; k < lists.size();) {
                if (k + 1 < lists.size() && pairs[k] >= 0) {
                    launches += (fsblocks_[pairs[k]] > 0 ? 1 : 0) +
                                (fsblocks_[pairs[k] + 1] > 0 ? 1 : 0);
                    k += 2;
                } else {
                    launches += lgrid_[lists[k]] > 0 ? colours : 0;
                    ++k;
                }
            }
        };
        count(swd_[0], bsd_[0]);
        count(swu_[0], bsu_[0]);
        prof_launches_tick_ = reps * launches;
    }
    built_mode_ = mode;
    built_active_ = active;
    built_ = true;
    return upload();
}

ma_status Engine::upload()
{
    const size_t bytes = hbuf_.size();
    if (bytes > dl_cap_) {
        E_HIP(hipStreamSynchronize(stream_));
        drop_graphs();
        (void)hipFree(dl_);
        dl_ = nullptr;
        const size_t cap = std::max<size_t>(bytes, 64 * 1024);
        E_HIP(hipMalloc(reinterpret_cast<void **>(&dl_), cap));
        dl_cap_ = cap;
    }
    if (bytes > hstage_cap_) {
        if (hstage_)
            (void)hipHostFree(hstage_);
        hstage_ = nullptr;
        const size_t cap = std::max<size_t>(bytes, 64 * 1024);
        E_HIP(hipHostMalloc(reinterpret_cast<void **>(&hstage_), cap));
        hstage_cap_ = cap;
    }
    std::memcpy(hstage_, hbuf_.data(), bytes);
    E_HIP(hipMemcpyAsync(dl_, hstage_, bytes, hipMemcpyHostToDevice, stream_));
    return MA_OK;
}

ma_status Engine::prof_mark()
{
    if (seg_capture_) {
        // close the current segment and open the next one
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(stream_, &g);
        if (g)
            seg_tmp_.push_back(g);
        E_HIP(e);
        E_HIP(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
        ++pev_used_;
        return MA_OK;
    }
    if (pev_used_ == pev_.size()) {
        hipEvent_t e;
        E_HIP(hipEventCreate(&e));
        pev_.push_back(e);
    }
    E_HIP(hipEventRecord(pev_[pev_used_++], stream_));
    return MA_OK;
}

ma_status Engine::enqueue(Mode mode, bool cycle)
{
    const bool mixed = mode == MODE_MIXED;
    const int op = mode == MODE_LAP ? OP_LAP : OP_MA;
    const int colours = order_ == 1 ? 8 : 4;
    auto L = [&](int idx) { return reinterpret_cast<const BatchList *>(dl_ + loff_[idx]); };
    auto go = [&](int kind, int idx, int color) -> ma_status {
        if (lgrid_[idx] == 0)
            return MA_OK;
        E_HIP(launch_batched(stream_, kind, op, order_, color, rmode_, L(idx), lgrid_[idx], dcount_,
                             dfall_));
        return MA_OK;
    };
    const int SW = mixed ? LK_MSWEEP : LK_SWEEP;
    auto FL = [&](int f) { return reinterpret_cast<const FsList *>(dl_ + fsoff_[f]); };
    // the sweeps of one depth: paired sweeps as two block sweeps, the others
    // one launch per colour phase
    auto sweeps = [&](const std::vector<int> &lists, const std::vector<int> &pairs) -> ma_status {
        for (size_t k = 0; k < lists.size();) {
            if (k + 1 < lists.size() && pairs[k] >= 0) {
                for (int h = 0; h < 2; ++h) {
                    const int f = pairs[k] + h;
                    if (fsblocks_[f] > 0)
                        E_HIP(launch_bsweep(stream_, op, fscfg_[f], FL(f), fsblocks_[f], dcount_,
                                            fspro_[f] != 0));
                }
                k += 2;
            } else {
                for (int c = 0; c < colours; ++c)
                    MA_TRY(go(SW, lists[k], c));
                ++k;
            }
        }
        return MA_OK;
    };
    auto vcycle = [&]() -> ma_status {
        for (int d = 0; d < D_; ++d) {
            if (profile_ && d == 0)
                MA_TRY(prof_mark());
            MA_TRY(sweeps(swd_[d], bsd_[d]));
            if (profile_ && d == 0)
                MA_TRY(prof_mark());
            if (rr_[d] >= 0) {
                E_HIP(launch_rrestrict(stream_, op, rmode_,
                                       reinterpret_cast<const RrList *>(dl_ + rroff_[rr_[d]]),
                                       rrblocks_[rr_[d]]));
            } else {
                MA_TRY(go(mixed ? LK_MRESIDUAL : LK_RESIDUAL, res_[d], 0));
                MA_TRY(go(mixed ? LK_MRESTRICT : LK_RESTRICT, rst_[d], 0));
            }
        }
        if (tail_blocks_ > 0 && tail_lds_)
            E_HIP(launch_tail_lds(stream_, int(mode), order_, rmode_,
                                  reinterpret_cast<const TailList *>(dl_ + toff_), tail_blocks_,
                                  nu1_, nu2_, nu0_, dcount_));
        else if (tail_blocks_ > 0)
            E_HIP(launch_tail(stream_, int(mode), order_, rmode_,
                              reinterpret_cast<const TailList *>(dl_ + toff_), tail_blocks_, nu1_,
                              nu2_, nu0_, dcount_, dfall_));
        for (int d = D_ - 1; d >= 0; --d) {
            // a fused depth prolongs inside its first post-smoothing sweep
            if (!pro_fused_[d])
                MA_TRY(go(mixed ? LK_MPROLONG : LK_PROLONG, pro_[d], 0));
            if (profile_ && d == 0)
                MA_TRY(prof_mark());
            MA_TRY(sweeps(swu_[d], bsu_[d]));
            if (profile_ && d == 0)
                MA_TRY(prof_mark());
        }
        return MA_OK;
    };
    if (cycle) {
        if (mixed) {
            for (int d = 0; d + 1 < Dall_; ++d)
                MA_TRY(go(LK_INJECT, inj_[d], 0));
            MA_TRY(go(LK_ZERO, zero_, 0));
            for (int it = 0; it < inner_; ++it)
                MA_TRY(vcycle());
            MA_TRY(go(LK_ACCUM, accum_, 0));
        } else {
            MA_TRY(vcycle());
        }
    }
    MA_TRY(go(mixed ? LK_RES32 : LK_NORM, norm_, 0));
    // one block per solve of the engine (blocks past the list's grids
    // return): the launch shape does not change when solves pause or stop
    E_HIP(launch_batched_reduce(stream_, L(norm_), int(solves_.size()), partials_,
                                NormRing{dnorm_, dstamp_, dseq_, dthr_, dl_,
                                         reinterpret_cast<const unsigned *>(dl_ + stoff_)}));
    return MA_OK;
}

// The launch shapes baked into a captured tick.
std::vector<int> Engine::shape() const
{
    std::vector<int> s;
    s.reserve(lgrid_.size() + 8);
    s.push_back(D_);
    s.push_back(Dall_);
    s.push_back(int(stride_));
    s.push_back(int(toff_));
    s.push_back(tail_blocks_);
    s.push_back(tail_lds_ ? 1 : 0);
    s.push_back(strip_rows_);
    s.push_back(int(loff_.size()));
    s.insert(s.end(), lgrid_.begin(), lgrid_.end());
    s.push_back(int(fsoff_.size()));
    s.push_back(fsoff_.empty() ? 0 : int(fsoff_[0]));
    s.push_back(int(fs_stride_));
    s.insert(s.end(), fsblocks_.begin(), fsblocks_.end());
    s.insert(s.end(), fscfg_.begin(), fscfg_.end());
    s.insert(s.end(), fspro_.begin(), fspro_.end());
    s.insert(s.end(), pro_fused_.begin(), pro_fused_.end());
    s.push_back(int(rroff_.size()));
    s.push_back(rroff_.empty() ? 0 : int(rroff_[0]));
    s.insert(s.end(), rrblocks_.begin(), rrblocks_.end());
    s.push_back(int(stoff_));
    s.push_back(int(solves_.size()));
    return s;
}

// Queue one tick (cycle) or one norm evaluation of the active solves on the
// engine stream, followed by an event; the host waits in collect().  ticks =
// 2 queues two cycles as one entry (one graph when graphs are on).
ma_status Engine::launch(Mode mode, bool cycle, const std::vector<char> &active, int ticks)
{
    if (active.size() != solves_.size())
        return fail(MA_ERR_ARG, "active mask size");
    if (ticks < 1 || ticks > 2 || (ticks == 2 && (!cycle || profile_)))
        return fail(MA_ERR_ARG, "internal: ticks per launch");
    if (!built_ || mode != built_mode_ || active != built_active_) {
        if (!fifo_.empty())
            return fail(MA_ERR_DEVICE, "internal: list rebuild with ticks in flight");
        MA_TRY(rebuild(mode, active));
    }
    MA_TRY(flush_arms());
    if (user_dirty_) {
        E_HIP(hipEventRecord(ev_in_, user_));
        E_HIP(hipStreamWaitEvent(stream_, ev_in_, 0));
        user_dirty_ = false;
    }
    if (cycle)
        MA_TRY(refresh_fs(mode, active));
    const int m = int(mode) + (profile_ ? 3 : 0) + (ticks == 2 ? 6 : 0);
    size_t nev = 0;
    if (cycle && graphs_) {
        if (gseg_[m].empty() || graph_dl_[m] != dl_ || graph_shape_[m] != shape())
            MA_TRY(capture(m, mode, ticks));
        // segment k is followed by timing event k (profiled form only)
        const size_t ns = gseg_[m].size();
        while (pev_.size() + 1 < ns) {
            hipEvent_t e;
            E_HIP(hipEventCreate(&e));
            pev_.push_back(e);
        }
        for (size_t k = 0; k < ns; ++k) {
            if (gseg_[m][k])
                E_HIP(hipGraphLaunch(gseg_[m][k], stream_));
            if (k + 1 < ns)
                E_HIP(hipEventRecord(pev_[k], stream_));
        }
        nev = ns - 1;
    } else {
        pev_used_ = 0;
        for (int t = 0; t < ticks; ++t)
            MA_TRY(enqueue(mode, cycle));
        nev = pev_used_;
    }
    hipEvent_t ev = nullptr;
    if (!evpool_.empty()) {
        ev = evpool_.back();
        evpool_.pop_back();
    } else {
        E_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    const hipError_t er = hipEventRecord(ev, stream_);
    if (er != hipSuccess) {
        (void)hipEventDestroy(ev);
        return fail(MA_ERR_DEVICE, std::string("hipEventRecord: ") + hipGetErrorString(er));
    }
    Pending p;
    p.mode = mode;
    p.cycle = cycle;
    p.active = active;
    p.ev = ev;
    p.nev = nev;
    p.ticks = ticks;
    fifo_.push_back(std::move(p));
    return MA_OK;
}

// Wait for the oldest queued entry (unless an earlier call did) and read
// the norms of its next tick for the solves that tick ran (those not halted
// before it).  The sum of a slot is the next entry of its ring; a stamp that
// disagrees with the host's count means the host and the device disagree on
// which ticks ran, and fails.
ma_status Engine::collect(std::vector<double> &norms)
{
    if (fifo_.empty())
        return fail(MA_ERR_DEVICE, "internal: no tick to collect");
    Pending &p = fifo_.front();
    if (!p.synced) {
        const hipError_t er = hipEventSynchronize(p.ev);
        if (er != hipSuccess) {
            evpool_.push_back(p.ev);
            fifo_.pop_front();
            return fail(MA_ERR_DEVICE, std::string("tick: ") + hipGetErrorString(er));
        }
        p.synced = true;
        // the ring entries the entry's ticks may have written, before a
        // later entry can reuse them
        p.sum.assign(size_t(p.ticks) * kMaxGrids, 0.0);
        p.stamp.assign(size_t(p.ticks) * kMaxGrids, ~0u);
        for (size_t i = 0; i < solves_.size(); ++i) {
            if (!solves_[i].s || !p.active[i] || halted_[i])
                continue;
            for (int t = 0; t < p.ticks; ++t) {
                const unsigned k = seq_[i] + unsigned(t);
                const size_t e = size_t(k % unsigned(kNormRing)) * kMaxGrids + i;
                p.sum[size_t(t) * kMaxGrids + i] = hnorm_[e];
                p.stamp[size_t(t) * kMaxGrids + i] = hstamp_[e];
            }
        }
    }
    const int t = p.done;
    norms.resize(solves_.size());
    for (size_t i = 0; i < solves_.size(); ++i) {
        if (!solves_[i].s || !p.active[i] || halted_[i])
            continue;
        const unsigned k = seq_[i];
        const size_t e = size_t(t) * kMaxGrids + i;
        if (p.stamp[e] != k)
            return fail(MA_ERR_DEVICE, "internal: norm ring out of step with the host");
        const double raw = p.sum[e];
        seq_[i] = k + 1u;
        const int n = solves_[i].s->p.n;
        const double h = 1.0 / double(n);
        norms[i] = std::sqrt(raw * h * h * h);
        // the device's decision in k_batched_reduce, on the same values
        const double th = thr_dev_[i];
        if (th >= 0.0 && (raw <= th || !std::isfinite(raw)))
            halted_[i] = 1;
    }
    if (profile_ && p.cycle) {
        for (size_t q = 0; q + 1 < p.nev; q += 2) {
            float ms = 0.f;
            E_HIP(hipEventElapsedTime(&ms, pev_[q], pev_[q + 1]));
            prof_seconds_ += 1e-3 * double(ms);
        }
        prof_bytes_ += prof_bytes_tick_;
        prof_launches_ += prof_launches_tick_;
    }
    if (++p.done == p.ticks) {
        evpool_.push_back(p.ev);
        fifo_.pop_front();
    }
    return MA_OK;
}

// Wait for every tick still queued.  Such ticks were queued ahead of the
// host's stopping test; each solve in them must have stopped before them
// (the device skipped it), else the host would lose a cycle it ran.
ma_status Engine::settle()
{
    while (!fifo_.empty()) {
        Pending p = std::move(fifo_.front());
        fifo_.pop_front();
        hipError_t er = hipSuccess;
        if (!p.synced)
            er = hipEventSynchronize(p.ev);
        evpool_.push_back(p.ev);
        if (er != hipSuccess)
            return fail(MA_ERR_DEVICE, std::string("tick: ") + hipGetErrorString(er));
        for (size_t i = 0; i < solves_.size(); ++i)
            if (solves_[i].s && p.active[i] && !halted_[i])
                return fail(MA_ERR_DEVICE,
                            "internal: a tick queued ahead ran for a solve that had not stopped");
    }
    return MA_OK;
}

// Largest non-negative sum of squares x for which the host's stopping test
// sqrt(x h h h) <= c passes (h = 1/n, the expression collect() evaluates);
// the test is monotone in x, so it passes exactly for x <= the result.
// Bisection over the ordered bit patterns of the non-negative doubles.
double sum_threshold(double c, int n)
{
    if (!(c >= 0.0) || n < 1)
        return -1.0;
    const double h = 1.0 / double(n);
    auto ok = [&](double x) { return std::sqrt(x * h * h * h) <= c; };
    auto val = [](uint64_t b) {
        double x;
        std::memcpy(&x, &b, sizeof(x));
        return x;
    };
    const double top = std::numeric_limits<double>::max();
    if (ok(top))
        return top;
    uint64_t lo = 0, hi;   // ok(val(lo)) holds, ok(val(hi)) does not
    std::memcpy(&hi, &top, sizeof(hi));
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (ok(val(mid)))
            lo = mid;
        else
            hi = mid;
    }
    return val(lo);
}

// Drop every queued tick, whatever it ran: after a failed step the host no
// longer reads them.  The device's per-slot sums counts are read back and
// every slot is re-armed before its next launch (a dropped tick may have
// stopped solves the host did not see stop).
ma_status Engine::abandon()
{
    if (!stream_)
        return MA_OK;
    E_HIP(hipStreamSynchronize(stream_));
    while (!fifo_.empty()) {
        evpool_.push_back(fifo_.front().ev);
        fifo_.pop_front();
    }
    E_HIP(hipMemcpy(seq_.data(), dseq_, kMaxGrids * sizeof(unsigned), hipMemcpyDeviceToHost));
    for (int i = 0; i < kMaxGrids; ++i) {
        thr_dev_[i] = std::numeric_limits<double>::quiet_NaN();   // never equal: re-arm
        halted_[i] = 0;
    }
    return MA_OK;
}

// Queue (slot, thr) for the next launch unless the device already holds
// that threshold with a clear halt flag.
void Engine::arm(int slot, double thr)
{
    if (thr_dev_[slot] == thr && !halted_[slot] && !armq_[slot])
        return;
    armq_[slot] = 1;
    armv_[slot] = thr;
}

ma_status Engine::flush_arms()
{
    ArmSet a;
    a.count = 0;
    for (int i = 0; i < kMaxGrids; ++i)
        if (armq_[i]) {
            a.slot[a.count] = i;
            a.thr[a.count] = armv_[i];
            ++a.count;
        }
    if (a.count == 0)
        return MA_OK;
    if (!fifo_.empty())
        return fail(MA_ERR_DEVICE, "internal: thresholds changed with ticks in flight");
    E_HIP(launch_arm(stream_, a, dthr_, dl_,
                     dl_ ? reinterpret_cast<const unsigned *>(dl_ + stoff_) : nullptr));
    for (int q = 0; q < a.count; ++q) {
        const int i = a.slot[q];
        thr_dev_[i] = armv_[i];
        halted_[i] = 0;
        armq_[i] = 0;
    }
    return MA_OK;
}

ma_status Engine::plain(Mode mode, bool cycle, const std::vector<char> &active,
                        std::vector<double> &norms)
{
    if (active.size() != solves_.size())
        return fail(MA_ERR_ARG, "active mask size");
    MA_TRY(settle());
    for (size_t i = 0; i < active.size(); ++i)
        if (active[i])
            arm(int(i), -1.0);
    MA_TRY(launch(mode, cycle, active));
    return collect(norms);
}

ma_status Engine::tick_ahead(Mode mode, const std::vector<char> &active,
                             const std::vector<double> &thr, bool ahead,
                             std::vector<double> &norms, bool pair)
{
    if (active.size() != solves_.size() || thr.size() != solves_.size())
        return fail(MA_ERR_ARG, "active mask size");
    if (!fifo_.empty()) {
        // the queued tick serves this call when it ran these solves
        const Pending &f = fifo_.front();
        bool same = f.cycle && f.mode == mode;
        for (size_t i = 0; i < active.size() && same; ++i)
            if (active[i] && (!f.active[i] || halted_[i]))
                same = false;
        if (!same)
            MA_TRY(settle());
    }
    for (size_t i = 0; i < active.size(); ++i)
        if (active[i])
            arm(int(i), thr[i]);
    if (fifo_.empty())
        MA_TRY(launch(mode, true, active));
    bool armed = false;
    for (int i = 0; i < kMaxGrids; ++i)
        armed |= armq_[i] != 0;
    if (armed)
        return fail(MA_ERR_DEVICE, "internal: thresholds changed with ticks in flight");
    // Queue ahead so that the device has a tick to run while the host reads
    // this one: when the tick read now is the last one queued, one tick or
    // (pair) two in one graph; when it is the first of two in one graph,
    // one tick behind them, which the pair condition allows (no stop the
    // device does not see at this tick or the next).  At most two entries
    // of at most two ticks each are ever queued, as the ring requires.
    if (!profile_ && fifo_.size() == 1 && built_ && built_mode_ == mode &&
        built_active_ == active) {
        const int rem = fifo_.front().ticks - fifo_.front().done;
        if (rem == 1 && ahead)
            MA_TRY(launch(mode, true, active, pair ? 2 : 1));
        else if (rem == 2 && ahead && pair)
            MA_TRY(launch(mode, true, active, 1));
    }
    return collect(norms);
}

// Capture ticks (1 or 2) ticks of mode into slot m: one graph, or
// (profiled form, one tick) one graph per segment between the finest-level
// sweep boundaries.  A segment with no work is kept as a null entry so the
// event order is unchanged.
ma_status Engine::capture(int m, Mode mode, int ticks)
{
    for (hipGraphExec_t x : gseg_[m])
        if (x)
            (void)hipGraphExecDestroy(x);
    gseg_[m].clear();
    graph_shape_[m].clear();
    graph_dl_[m] = nullptr;
    seg_tmp_.clear();
    pev_used_ = 0;
    seg_capture_ = profile_;
    E_HIP(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
    ma_status st = MA_OK;
    for (int t = 0; t < ticks && st == MA_OK; ++t)
        st = enqueue(mode, true);
    hipGraph_t last = nullptr;
    const hipError_t ec = hipStreamEndCapture(stream_, &last);
    seg_capture_ = false;
    if (last)
        seg_tmp_.push_back(last);
    auto release = [&]() {
        for (hipGraph_t g : seg_tmp_)
            (void)hipGraphDestroy(g);
        seg_tmp_.clear();
    };
    auto drop = [&]() {
        for (hipGraphExec_t x : gseg_[m])
            if (x)
                (void)hipGraphExecDestroy(x);
        gseg_[m].clear();
    };
    if (st != MA_OK || ec != hipSuccess) {
        release();
        drop();
        if (st != MA_OK)
            return st;
        return fail(MA_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    }
    for (hipGraph_t g : seg_tmp_) {
        size_t nodes = 0;
        hipError_t e = hipGraphGetNodes(g, nullptr, &nodes);
        hipGraphExec_t x = nullptr;
        if (e == hipSuccess && nodes > 0)
            e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            release();
            drop();
            return fail(MA_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        gseg_[m].push_back(x);
    }
    release();
    graph_shape_[m] = shape();
    graph_dl_[m] = dl_;
    return MA_OK;
}

ma_status Engine::tick(Mode mode, const std::vector<char> &active, std::vector<double> &norms)
{
    return plain(mode, true, active, norms);
}

ma_status Engine::norms_only(Mode mode, const std::vector<char> &active,
                             std::vector<double> &norms)
{
    return plain(mode, false, active, norms);
}

void Engine::take_profile(double *seconds, int *launches, double *bytes)
{
    *seconds = prof_seconds_;
    *launches = prof_launches_;
    *bytes = prof_bytes_;
    prof_seconds_ = prof_bytes_ = 0.0;
    prof_launches_ = 0;
}

// Algorithmic bytes per kernel (per interior node unless stated):
//   FP64 sweep 24 (read u, F; write u), residual 24 (read u, F; write r),
//   restriction 8 per fine node + 32 per coarse node (inject u, write w, u,
//   b), prolongation 16 per fine node + 16 per coarse node, norm 16;
//   mixed sweep 20 (U 8, delta 4+4, b 4), mixed residual 20, mixed
//   restriction 4 per fine + 24 per coarse node, mixed prolongation 8 per
//   fine + 8 per coarse node, injection 16 per coarse node, accumulation
//   20, FP64 residual into FP32 20, zeroing 4 per node.
void Engine::tick_cost(Mode mode, int i, double *updates, double *bytes) const
{
    const ma_solver *s = solves_[i].s;
    const bool mixed = mode == MODE_MIXED;
    const int L = int(s->lv.size());
    double up = 0.0, by = 0.0;
    const int reps = mixed ? inner_ : 1;
    for (int l = 0; l < L; ++l) {
        const int n = s->lv[l].n;
        const double in = interior(n);
        const int sweeps = l < L - 1 ? nu1_ + nu2_ : nu0_;
        if (mode != MODE_LAP)
            up += reps * sweeps * in;
        by += reps * sweeps * (mixed ? 20.0 : 24.0) * in;
        if (l < L - 1) {
            const double nc = double(npts_sz(s->lv[l + 1].n));
            if (mixed)
                by += reps * (20.0 * in + 4.0 * in + 24.0 * nc + 8.0 * in + 8.0 * nc) + 16.0 * nc;
            else
                by += 24.0 * in + 8.0 * in + 32.0 * nc + 16.0 * in + 16.0 * nc;
        }
    }
    const double in0 = interior(s->lv[0].n);
    by += mixed ? (20.0 * in0 + 20.0 * in0 + 4.0 * double(npts_sz(s->lv[0].n))) : 16.0 * in0;
    *updates = up;
    *bytes = by;
}

} // namespace mafas
