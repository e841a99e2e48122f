// Batched execution engine (see ma_engine.h).  The device side is one kernel
// template: a fixed grid of kPersistBlocks single-wave blocks walks the work
// items of a BatchList; each item is one x-row of 64 nodes of one grid.  The
// items are split into 8 contiguous chunks, one per XCD (blocks are
// dispatched round-robin over XCDs), so the rows a stencil reads as halos
// are processed on the same XCD at about the same time and share its L2.
// The point arithmetic is the same device code as the single-grid kernels.
#include "ma_engine.h"
#include "ma_mixed_device.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace mafas {

namespace {

__device__ __forceinline__ double wave_sum64(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

// Colour rows: (bx, by, bz) -> first node (i, j, k) of the row segment.
template <int ORDER>
__device__ __forceinline__ void colour_row(int color, int bx, int by, int bz, int &i, int &j,
                                           int &k)
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
    i = i0 + 2 * (bx * 64 + int(threadIdx.x));
}

template <int KIND, int OP, int ORDER, int RMODE>
__device__ __forceinline__ void run_item(const GridItem &G, int bx, int by, int bz, int color,
                                         unsigned long long *__restrict__ ncount,
                                         unsigned long long *__restrict__ nfall)
{
    const int n = G.n;
    const long sy = n + 1, sz = sy * sy;
    const int t = threadIdx.x;
    if (KIND == LK_SWEEP) {
        int i, j, k;
        colour_row<ORDER>(color, bx, by, bz, i, j, k);
        if (i <= n - 1 && j <= n - 1 && k <= n - 1) {
            double *u = static_cast<double *>(G.p[0]);
            const double *F = static_cast<const double *>(G.p[1]);
            const long p = i + sy * j + sz * k;
            if (OP == OP_MA) {
                const Hess g = hessian_at(u, p, 1, sy, sz, G.s, 0.25 * G.s);
                bool nc = false;
                u[p] = ma_point_update(g, u[p], F[p], G.hk, nc);
                if (nc)
                    atomicAdd(ncount + G.slot, 1ull);
            } else {
                u[p] = lap_point_update(laplacian_at(u, p, 1, sy, sz, G.s), u[p], F[p], G.hk);
            }
        }
    } else if (KIND == LK_RESIDUAL || KIND == LK_NORM || KIND == LK_RES32) {
        const int i = 1 + bx * 64 + t, j = 1 + by, k = 1 + bz;
        double rv = 0.0;
        if (i <= n - 1) {
            const double *u = static_cast<const double *>(G.p[0]);
            const double *F = static_cast<const double *>(G.p[1]);
            const long p = i + sy * j + sz * k;
            if (OP == OP_MA)
                rv = F[p] - det3(hessian_at(u, p, 1, sy, sz, G.s, 0.25 * G.s));
            else
                rv = F[p] - laplacian_at(u, p, 1, sy, sz, G.s);
            if (KIND == LK_RESIDUAL)
                static_cast<double *>(G.p[2])[p] = rv;
            if (KIND == LK_RES32)
                static_cast<float *>(G.p[2])[p] = float(rv);
        }
        if (KIND != LK_RESIDUAL) {
            const double sum = wave_sum64(rv * rv);
            if (t == 0) {
                const int local = bx + G.gx * (by + G.gy * bz);
                double *part = static_cast<double *>(KIND == LK_NORM ? G.p[2] : G.p[3]);
                part[G.pbase + local] = sum;
            }
        }
    } else if (KIND == LK_RESTRICT) {
        const int nf = n, nc = nf / 2;
        const int I = bx * 64 + t, J = by, K = bz;
        if (I <= nc) {
            const double *uf = static_cast<const double *>(G.p[0]);
            const double *rf = static_cast<const double *>(G.p[1]);
            const long fy = nf + 1, fz = fy * fy, cy = nc + 1, cz = cy * cy;
            const long f = 2 * I + fy * (2 * J) + fz * (2 * K);
            const long c = I + cy * J + cz * K;
            const double v = uf[f];
            static_cast<double *>(G.p[2])[c] = v;
            static_cast<double *>(G.p[3])[c] = v;
            double b = 0.0;
            if (I >= 1 && I <= nc - 1 && J >= 1 && J <= nc - 1 && K >= 1 && K <= nc - 1) {
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
                                rh += (w[dz + 1] * w[dy + 1] * w[dx + 1])
                                      * rf[f + dx + fy * dy + fz * dz];
                } else {
                    rh = (6.0 * rf[f] + (rf[f - 1] + rf[f + 1]) + (rf[f - fy] + rf[f + fy])
                          + (rf[f - fz] + rf[f + fz])) / 12.0;
                }
                const double sc = double(nc) * double(nc);
                double sh;
                if (OP == OP_MA)
                    sh = det3(hessian_at(uf, f, 2, 2 * fy, 2 * fz, sc, 0.25 * sc));
                else
                    sh = laplacian_at(uf, f, 2, 2 * fy, 2 * fz, sc);
                b = sh + rh;
            }
            static_cast<double *>(G.p[4])[c] = b;
        }
    } else if (KIND == LK_PROLONG || KIND == LK_MPROLONG) {
        const int nf = n, nc = nf / 2;
        const int i = 1 + bx * 64 + t, j = 1 + by, k = 1 + bz;
        if (i <= nf - 1) {
            const long cy = nc + 1, cz = cy * cy;
            const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1, nk = (k & 1) ? 2 : 1;
            const int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
            const long p = i + sy * j + sz * k;
            if (KIND == LK_PROLONG) {
                const double *uc = static_cast<const double *>(G.p[1]);
                const double *wc = static_cast<const double *>(G.p[2]);
                const double wi = (i & 1) ? 0.5 : 1.0, wj = (j & 1) ? 0.5 : 1.0,
                             wk = (k & 1) ? 0.5 : 1.0;
                double d = 0.0;
                for (int c = 0; c < nk; ++c)
                    for (int b = 0; b < nj; ++b)
                        for (int a = 0; a < ni; ++a) {
                            const long q = (I0 + a) + cy * (J0 + b) + cz * (K0 + c);
                            d += (wk * wj * wi) * (uc[q] - wc[q]);
                        }
                static_cast<double *>(G.p[0])[p] += d;
            } else {
                const float *dc = static_cast<const float *>(G.p[1]);
                const float *wc = static_cast<const float *>(G.p[2]);
                const float wi = (i & 1) ? 0.5f : 1.0f, wj = (j & 1) ? 0.5f : 1.0f,
                            wk = (k & 1) ? 0.5f : 1.0f;
                float d = 0.0f;
                for (int c = 0; c < nk; ++c)
                    for (int b = 0; b < nj; ++b)
                        for (int a = 0; a < ni; ++a) {
                            const long q = (I0 + a) + cy * (J0 + b) + cz * (K0 + c);
                            d += (wk * wj * wi) * (dc[q] - wc[q]);
                        }
                static_cast<float *>(G.p[0])[p] += d;
            }
        }
    } else if (KIND == LK_MSWEEP) {
        int i, j, k;
        colour_row<ORDER>(color, bx, by, bz, i, j, k);
        if (i <= n - 1 && j <= n - 1 && k <= n - 1) {
            float *d = static_cast<float *>(G.p[0]);
            const float *b = static_cast<const float *>(G.p[1]);
            const double *U = static_cast<const double *>(G.p[2]);
            const long p = i + sy * j + sz * k;
            const LevelConst lc = level_const(n);
            bool fb = false, nc = false;
            d[p] = mixed_point(d, U, b[p], p, sy, sz, lc.s, lc.s4, lc.sf, lc.s4f, lc.hkf, fb, nc);
            if (fb)
                atomicAdd(nfall + G.slot, 1ull);
            if (nc)
                atomicAdd(ncount + G.slot, 1ull);
        }
    } else if (KIND == LK_MRESIDUAL) {
        const int i = 1 + bx * 64 + t, j = 1 + by, k = 1 + bz;
        if (i <= n - 1) {
            const float *d = static_cast<const float *>(G.p[0]);
            const float *b = static_cast<const float *>(G.p[1]);
            const double *U = static_cast<const double *>(G.p[2]);
            const long p = i + sy * j + sz * k;
            const LevelConst lc = level_const(n);
            const Sym32 H = to32(hessian_at(U, p, 1, sy, sz, lc.s, lc.s4));
            const Sym32 E = hess32(d, p, 1, sy, sz, lc.sf, lc.s4f);
            static_cast<float *>(G.p[3])[p] = b[p] - t_of(H, adj32(H), E);
        }
    } else if (KIND == LK_MRESTRICT) {
        const int nf = n, nc = nf / 2;
        const int I = bx * 64 + t, J = by, K = bz;
        if (I <= nc) {
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
                                rh += (w[dz + 1] * w[dy + 1] * w[dx + 1])
                                      * rf[f + dx + fy * dy + fz * dz];
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
    } else if (KIND == LK_INJECT) {
        const int nf = n, nc = nf / 2;
        const int I = bx * 64 + t, J = by, K = bz;
        if (I <= nc) {
            const long fy = nf + 1, cy = nc + 1;
            static_cast<double *>(G.p[1])[I + cy * J + cy * cy * K] =
                static_cast<const double *>(G.p[0])[2 * I + fy * (2 * J) + fy * fy * (2 * K)];
        }
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

template <int KIND, int OP, int ORDER, int RMODE>
__global__ __launch_bounds__(64) void k_batched(const BatchList *__restrict__ L, int color,
                                                unsigned long long *__restrict__ ncount,
                                                unsigned long long *__restrict__ nfall)
{
    constexpr int kBlocksPerXcd = kPersistBlocks / 8;
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
    for (; it < hi; it += kBlocksPerXcd) {
        while (g + 1 < ng && L->g[g + 1].start <= it)
            ++g;
        const GridItem &G = L->g[g];
        const int local = it - G.start;
        const int bx = local % G.gx;
        const int rest = local / G.gx;
        const int by = rest % G.gy;
        const int bz = rest / G.gy;
        run_item<KIND, OP, ORDER, RMODE>(G, bx, by, bz, color, ncount, nfall);
    }
}

// Fixed-order per-grid sum of the partials of a norm list.
__global__ __launch_bounds__(256) void k_batched_reduce(const BatchList *__restrict__ L,
                                                        const double *__restrict__ partials,
                                                        double *__restrict__ out)
{
    __shared__ double part[4];
    const int g = blockIdx.x;
    if (g >= L->ngrids)
        return;
    const GridItem &G = L->g[g];
    const int end = (g + 1 < L->ngrids) ? L->g[g + 1].start : L->total;
    const int cnt = end - G.start;
    double v = 0.0;
    for (int q = threadIdx.x; q < cnt; q += 256)
        v += partials[G.pbase + q];
    v = wave_sum64(v);
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        out[G.slot] = ((part[0] + part[1]) + part[2]) + part[3];
}

template <int KIND, int OP>
hipError_t launch_k(hipStream_t st, int order, int color, int rmode, const BatchList *L,
                    unsigned long long *nc, unsigned long long *nf)
{
    const dim3 grid(kPersistBlocks), block(64);
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
                       unsigned long long *nc, unsigned long long *nf)
{
    if (op == OP_MA)
        return launch_k<KIND, OP_MA>(st, order, color, rmode, L, nc, nf);
    return launch_k<KIND, OP_LAP>(st, order, color, rmode, L, nc, nf);
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
    default:  // interior rows
        *gx = (n - 1 + 63) / 64;
        *gy = n - 1;
        *gz = n - 1;
        break;
    }
}

hipError_t launch_batched(hipStream_t st, int kind, int op, int order, int color, int rmode,
                          const BatchList *L, unsigned long long *nc, unsigned long long *nf)
{
    // kinds whose arithmetic does not depend on op / order / rmode use one
    // instantiation
    switch (kind) {
    case LK_SWEEP:
        return launch_kind<LK_SWEEP>(st, op, order, color, 0, L, nc, nf);
    case LK_RESIDUAL:
        return launch_kind<LK_RESIDUAL>(st, op, 0, 0, 0, L, nc, nf);
    case LK_NORM:
        return launch_kind<LK_NORM>(st, op, 0, 0, 0, L, nc, nf);
    case LK_RESTRICT:
        return launch_kind<LK_RESTRICT>(st, op, 0, 0, rmode, L, nc, nf);
    case LK_PROLONG:
        return launch_k<LK_PROLONG, OP_MA>(st, 0, 0, 0, L, nc, nf);
    case LK_MSWEEP:
        return launch_k<LK_MSWEEP, OP_MA>(st, order, color, 0, L, nc, nf);
    case LK_MRESIDUAL:
        return launch_k<LK_MRESIDUAL, OP_MA>(st, 0, 0, 0, L, nc, nf);
    case LK_MRESTRICT:
        return launch_k<LK_MRESTRICT, OP_MA>(st, 0, 0, rmode, L, nc, nf);
    case LK_MPROLONG:
        return launch_k<LK_MPROLONG, OP_MA>(st, 0, 0, 0, L, nc, nf);
    case LK_INJECT:
        return launch_k<LK_INJECT, OP_MA>(st, 0, 0, 0, L, nc, nf);
    case LK_ACCUM:
        return launch_k<LK_ACCUM, OP_MA>(st, 0, 0, 0, L, nc, nf);
    case LK_ZERO:
        return launch_k<LK_ZERO, OP_MA>(st, 0, 0, 0, L, nc, nf);
    case LK_RES32:
        return launch_k<LK_RES32, OP_MA>(st, 0, 0, 0, L, nc, nf);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_batched_reduce(hipStream_t st, const BatchList *L, const double *partials,
                                 double *out)
{
    hipLaunchKernelGGL(k_batched_reduce, dim3(kMaxGrids), dim3(256), 0, st, L, partials, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Engine
// ---------------------------------------------------------------------------
Engine::~Engine()
{
    drop_graphs();
    for (hipEvent_t e : pev_)
        (void)hipEventDestroy(e);
    if (ev_in_)
        (void)hipEventDestroy(ev_in_);
    if (stream_) {
        (void)hipStreamSynchronize(stream_);
        (void)hipStreamDestroy(stream_);
    }
    (void)hipFree(dl_);
    (void)hipFree(partials_);
    (void)hipFree(dnorm_);
    (void)hipFree(dcount_);
    (void)hipFree(dfall_);
    if (hstage_)
        (void)hipHostFree(hstage_);
    if (hnorm_)
        (void)hipHostFree(hnorm_);
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
        graph_D_[m] = -1;
        graph_dl_[m] = nullptr;
        graph_stride_[m] = 0;
        graph_nl_[m] = 0;
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
                 p.inner_cycles != p0->inner_cycles)
            return fail(MA_ERR_ARG,
                        "solvers in one batch must share smoothing counts, ordering, "
                        "restriction and precision");
    }
    if (!p0)
        return fail(MA_ERR_ARG, "a batch needs at least one solver");
    // A captured tick reads the grids' operand pointers from the device lists,
    // which every rebuild rewrites; what it holds as plain kernel arguments
    // is the partials buffer and, on the fused path, the grids themselves.
    // A change of either invalidates the graphs.
    const bool fused = solves.size() == 1 && p0->smoother == MA_SMOOTHER_FUSED &&
                       p0->order == MA_COLOR4;
    bool same = solves.size() == solves_.size();
    for (size_t i = 0; same && i < solves.size(); ++i)
        same = solves[i].s == solves_[i].s && solves[i].u == solves_[i].u &&
               solves[i].f == solves_[i].f;
    if (fused != fused_ || (fused && !same))
        drop_graphs();
    solves_ = solves;
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
    fused_ = fused;
    built_ = false;
    if (!stream_) {
        E_HIP(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
        E_HIP(hipEventCreateWithFlags(&ev_in_, hipEventDisableTiming));
        E_HIP(hipMalloc(reinterpret_cast<void **>(&dnorm_), kMaxGrids * sizeof(double)));
        E_HIP(hipMalloc(reinterpret_cast<void **>(&dcount_), kMaxGrids * sizeof(unsigned long long)));
        E_HIP(hipMalloc(reinterpret_cast<void **>(&dfall_), kMaxGrids * sizeof(unsigned long long)));
        E_HIP(hipHostMalloc(reinterpret_cast<void **>(&hnorm_), kMaxGrids * sizeof(double)));
        E_HIP(hipHostMalloc(reinterpret_cast<void **>(&hcount_),
                            2 * kMaxGrids * sizeof(unsigned long long)));
    }
    size_t need = 0;
    for (const SolveRef &r : solves_)
        if (r.s) {
            int gx, gy, gz;
            item_dims(LK_NORM, 0, r.s->p.n, &gx, &gy, &gz);
            need += size_t(gx) * gy * gz;
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

ma_status Engine::reset_counters(int slot)
{
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
    E_HIP(hipMemcpyAsync(hcount_, dcount_, kMaxGrids * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, stream_));
    E_HIP(hipMemcpyAsync(hcount_ + kMaxGrids, dfall_, kMaxGrids * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, stream_));
    E_HIP(hipStreamSynchronize(stream_));
    nonconvex.assign(hcount_, hcount_ + solves_.size());
    fallbacks.assign(hcount_ + kMaxGrids, hcount_ + kMaxGrids + solves_.size());
    return MA_OK;
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

ma_status Engine::rebuild(Mode mode, const std::vector<char> &active)
{
    hbuf_.clear();
    loff_.clear();
    lng_.clear();
    stride_ = list_bytes(int(solves_.size()));
    const int S = int(solves_.size());
    auto on = [&](int i) { return solves_[i].s && active[i]; };
    auto levels = [&](int i) { return int(solves_[i].s->lv.size()); };
    D_ = 0;
    for (int i = 0; i < S; ++i)
        if (on(i))
            D_ = std::max(D_, levels(i));
    const bool mixed = mode == MODE_MIXED;
    bool overflow = false;
    int pnext = 0;
    auto make = [&](int kind, int d, auto pred, bool partial) {
        BatchList L;
        L.ngrids = 0;
        L.total = 0;
        L.pad[0] = L.pad[1] = 0;
        int start = 0;
        for (int i = 0; i < S; ++i) {
            if (!on(i) || levels(i) <= d || !pred(i))
                continue;
            if (L.ngrids == kMaxGrids) {
                overflow = true;
                break;
            }
            GridItem G = grid(kind, i, d, mode);
            int gx, gy, gz;
            item_dims(kind, order_, G.n, &gx, &gy, &gz);
            G.gx = gx;
            G.gy = gy;
            G.start = start;
            if (partial) {
                G.pbase = pnext;
                pnext += gx * gy * gz;
            }
            start += gx * gy * gz;
            L.g[L.ngrids++] = G;
        }
        L.total = start;
        // every list sits at index * stride_, so a list's device address
        // depends only on its index: graphs captured for one composition
        // stay valid when solves join or leave (same depth, same slots)
        const size_t off = loff_.size() * stride_;
        loff_.push_back(off);
        lng_.push_back(L.ngrids);
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
    inj_.assign(D_, -1);
    const int SW = mixed ? LK_MSWEEP : LK_SWEEP;
    for (int d = 0; d < D_; ++d) {
        for (int k = 0; k < ksw; ++k)
            swd_[d].push_back(make(SW, d, [&](int i) {
                const int cnt = d < levels(i) - 1 ? nu1_ : nu0_;
                return cnt > k;
            }, false));
        if (d < D_ - 1) {
            auto nc = [&](int i) { return d < levels(i) - 1; };
            res_[d] = make(mixed ? LK_MRESIDUAL : LK_RESIDUAL, d, nc, false);
            rst_[d] = make(mixed ? LK_MRESTRICT : LK_RESTRICT, d, nc, false);
            pro_[d] = make(mixed ? LK_MPROLONG : LK_PROLONG, d, nc, false);
            if (mixed)
                inj_[d] = make(LK_INJECT, d, nc, false);
        }
        for (int k = 0; k < nu2_; ++k)
            swu_[d].push_back(make(SW, d, [&](int i) { return d < levels(i) - 1; }, false));
    }
    auto all = [](int) { return true; };
    norm_ = make(mixed ? LK_RES32 : LK_NORM, 0, all, true);
    accum_ = zero_ = -1;
    if (mixed) {
        accum_ = make(LK_ACCUM, 0, all, false);
        zero_ = make(LK_ZERO, 0, all, false);
    }
    if (overflow)
        return fail(MA_ERR_ARG, "too many grids in one batched launch");
    if (size_t(pnext) > partials_cap_)
        return fail(MA_ERR_ARG, "partial-sum buffer too small for the batch");
    prof_bytes_tick_ = 0.0;
    prof_launches_tick_ = 0;
    for (int i = 0; i < S; ++i)
        if (on(i)) {
            const double in = interior(mixed ? solves_[i].s->mx[0].n : solves_[i].s->lv[0].n);
            const bool single = levels(i) == 1;
            const int sweeps = single ? nu0_ : nu1_ + nu2_;
            const int reps = mixed ? inner_ : 1;
            prof_bytes_tick_ += reps * sweeps * (mixed ? 20.0 : 24.0) * in;
        }
    {
        const int reps = mixed ? inner_ : 1;
        const int colours = order_ == 1 ? 8 : 4;
        prof_launches_tick_ = reps * colours * (ksw + (D_ > 1 ? nu2_ : 0));
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
        E_HIP(launch_batched(stream_, kind, op, order_, color, rmode_, L(idx), dcount_, dfall_));
        return MA_OK;
    };
    const int SW = mixed ? LK_MSWEEP : LK_SWEEP;
    // the explicitly selected fused smoother of a one-solve FP64 engine:
    // sweeps of depth d in out-of-place pairs, a leftover sweep per colour
    auto sweeps = [&](const std::vector<int> &lists, int d) -> ma_status {
        const ma_solver *s0 = solves_[0].s;
        const int nd = s0->lv[d].n;
        if (fused_ && !mixed && nd >= 4) {
            double *u = const_cast<double *>(level_u(0, d, mode));
            const double *F = level_F(0, d, mode);
            double *t = s0->lv[d].t;
            size_t cnt = 0;
            for (int idx : lists)
                cnt += lng_[idx] > 0 ? 1 : 0;
            size_t done = 0;
            if (cnt >= 2) {
                E_HIP(launch_copy_boundary(stream_, nd, u, t));
                for (; done + 2 <= cnt; done += 2) {
                    E_HIP(launch_sweep_fused(stream_, op, nd, u, t, F, dcount_, s0->p.tile_config - 1,
                                             s0->p.zchunk));
                    E_HIP(launch_sweep_fused(stream_, op, nd, t, u, F, dcount_, s0->p.tile_config - 1,
                                             s0->p.zchunk));
                }
            }
            for (size_t q = done; q < lists.size(); ++q)
                for (int c = 0; c < colours; ++c)
                    MA_TRY(go(SW, lists[q], c));
            return MA_OK;
        }
        for (int idx : lists)
            for (int c = 0; c < colours; ++c)
                MA_TRY(go(SW, idx, c));
        return MA_OK;
    };
    auto vcycle = [&]() -> ma_status {
        for (int d = 0; d < D_; ++d) {
            if (profile_ && d == 0)
                MA_TRY(prof_mark());
            MA_TRY(sweeps(swd_[d], d));
            if (profile_ && d == 0)
                MA_TRY(prof_mark());
            if (d < D_ - 1) {
                MA_TRY(go(mixed ? LK_MRESIDUAL : LK_RESIDUAL, res_[d], 0));
                MA_TRY(go(mixed ? LK_MRESTRICT : LK_RESTRICT, rst_[d], 0));
            }
        }
        for (int d = D_ - 2; d >= 0; --d) {
            MA_TRY(go(mixed ? LK_MPROLONG : LK_PROLONG, pro_[d], 0));
            if (profile_ && d == 0)
                MA_TRY(prof_mark());
            MA_TRY(sweeps(swu_[d], d));
            if (profile_ && d == 0)
                MA_TRY(prof_mark());
        }
        return MA_OK;
    };
    if (cycle) {
        if (mixed) {
            for (int d = 0; d + 1 < D_; ++d)
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
    E_HIP(launch_batched_reduce(stream_, L(norm_), partials_, dnorm_));
    return MA_OK;
}

ma_status Engine::run(Mode mode, bool cycle, const std::vector<char> &active,
                      std::vector<double> &norms)
{
    if (active.size() != solves_.size())
        return fail(MA_ERR_ARG, "active mask size");
    if (!built_ || mode != built_mode_ || active != built_active_)
        MA_TRY(rebuild(mode, active));
    E_HIP(hipEventRecord(ev_in_, user_));
    E_HIP(hipStreamWaitEvent(stream_, ev_in_, 0));
    const int m = int(mode) + (profile_ ? 3 : 0);
    size_t nev = 0;
    if (cycle && graphs_) {
        if (gseg_[m].empty() || graph_D_[m] != D_ || graph_dl_[m] != dl_ ||
            graph_stride_[m] != stride_ || graph_nl_[m] != loff_.size())
            MA_TRY(capture(m, mode));
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
        MA_TRY(enqueue(mode, cycle));
        nev = pev_used_;
    }
    E_HIP(hipMemcpyAsync(hnorm_, dnorm_, solves_.size() * sizeof(double), hipMemcpyDeviceToHost,
                         stream_));
    E_HIP(hipStreamSynchronize(stream_));
    norms.resize(solves_.size());
    for (size_t i = 0; i < solves_.size(); ++i)
        if (solves_[i].s && active[i]) {
            const int n = solves_[i].s->p.n;
            const double h = 1.0 / double(n);
            norms[i] = std::sqrt(hnorm_[i] * h * h * h);
        }
    if (profile_ && cycle) {
        for (size_t q = 0; q + 1 < nev; q += 2) {
            float ms = 0.f;
            E_HIP(hipEventElapsedTime(&ms, pev_[q], pev_[q + 1]));
            prof_seconds_ += 1e-3 * double(ms);
        }
        prof_bytes_ += prof_bytes_tick_;
        prof_launches_ += prof_launches_tick_;
    }
    return MA_OK;
}

// Capture one tick of mode into slot m: one graph, or (profiled form) one
// graph per segment between the finest-level sweep boundaries.  A segment
// with no work is kept as a null entry so the event order is unchanged.
ma_status Engine::capture(int m, Mode mode)
{
    for (hipGraphExec_t x : gseg_[m])
        if (x)
            (void)hipGraphExecDestroy(x);
    gseg_[m].clear();
    seg_tmp_.clear();
    pev_used_ = 0;
    seg_capture_ = profile_;
    E_HIP(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
    const ma_status st = enqueue(mode, true);
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
    if (st != MA_OK || ec != hipSuccess) {
        release();
        for (hipGraphExec_t x : gseg_[m])
            if (x)
                (void)hipGraphExecDestroy(x);
        gseg_[m].clear();
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
            for (hipGraphExec_t y : gseg_[m])
                if (y)
                    (void)hipGraphExecDestroy(y);
            gseg_[m].clear();
            return fail(MA_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        gseg_[m].push_back(x);
    }
    release();
    graph_D_[m] = D_;
    graph_dl_[m] = dl_;
    graph_stride_[m] = stride_;
    graph_nl_[m] = loff_.size();
    return MA_OK;
}

ma_status Engine::tick(Mode mode, const std::vector<char> &active, std::vector<double> &norms)
{
    return run(mode, true, active, norms);
}

ma_status Engine::norms_only(Mode mode, const std::vector<char> &active,
                             std::vector<double> &norms)
{
    return run(mode, false, active, norms);
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
