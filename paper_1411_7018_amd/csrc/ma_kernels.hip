// FP64 kernels of the FAS V-cycle (Algorithm 1) for det(D^2 u) = f and of
// the linear 7-point V-cycle used for the initial guess.  All grid functions
// are (n+1)^3 x-fastest arrays; Dirichlet nodes are read, never written.
#include "ma_device.h"
#include "ma_internal.h"
#include "ma_runtime.h"

namespace mafas {

namespace {

constexpr int RES_BX = 64;   // residual / transfer block: 64 x 4 threads
constexpr int RES_BY = 4;

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

// Sum over a block of exactly nwaves full wavefronts, fixed order.
template <int NWAVES>
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double part[NWAVES];
    const int lane = threadIdx.x & 63;
    const int wid = (threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z)) >> 6;
    v = wave_sum(v);
    if (lane == 0)
        part[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (wid == 0 && lane == 0)
        for (int w = 0; w < NWAVES; ++w)
            t += part[w];
    return t;
}

// ---------------------------------------------------------------------------
// Smoother, one launch per colour phase.  Colour of node (i,j,k):
//   4 colours: ((i+j) mod 2) + 2 ((i+k) mod 2)   [i = j + c0, k parity from c1]
//   8 colours: (i mod 2) + 2 (j mod 2) + 4 (k mod 2)
// Nodes of one colour are never stencil neighbours, so the in-place updates
// of a phase do not interact.
// ---------------------------------------------------------------------------
template <int OP, int ORDER>
__global__ __launch_bounds__(64) void k_sweep_color(double *__restrict__ u,
                                                    const double *__restrict__ F, int n,
                                                    int color, int gx, int gy, int nb, double s,
                                                    double s4, double hk,
                                                    unsigned long long *__restrict__ ncount)
{
    // one block = 64 colour nodes of one x-row; rows in XCD-contiguous order
    const int tile = tile_of_block(blockIdx.x, nb);
    const int bx = tile % gx, rest = tile / gx, by = rest % gy, bz = rest / gy;
    int i0, j, k;
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
    const int i = i0 + 2 * (bx * 64 + int(threadIdx.x));
    if (i > n - 1 || j > n - 1 || k > n - 1)
        return;
    const long sy = n + 1, sz = sy * sy;
    const long p = i + sy * j + sz * k;
    if (OP == OP_MA) {
        const Hess g = hessian_at(u, p, 1, sy, sz, s, s4);
        bool nc = false;
        u[p] = ma_point_update(g, u[p], F[p], hk, nc);
        if (nc && ncount)
            atomicAdd(ncount, 1ull);
    } else {
        u[p] = lap_point_update(laplacian_at(u, p, 1, sy, sz, s), u[p], F[p], hk);
    }
}

// ---------------------------------------------------------------------------
// Residual r = F - S(u) and per-block sums of r^2 over interior nodes.
// ---------------------------------------------------------------------------
template <int OP>
__global__ __launch_bounds__(RES_BX *RES_BY) void k_residual(const double *__restrict__ u,
                                                             const double *__restrict__ F,
                                                             double *__restrict__ r,
                                                             double *__restrict__ partials,
                                                             int n, double s, double s4)
{
    const int i = 1 + blockIdx.x * RES_BX + threadIdx.x;
    const int j = 1 + blockIdx.y * RES_BY + threadIdx.y;
    const int k = 1 + blockIdx.z;
    double rv = 0.0;
    if (i <= n - 1 && j <= n - 1) {
        const long sy = n + 1, sz = sy * sy;
        const long p = i + sy * j + sz * k;
        if (OP == OP_MA)
            rv = F[p] - det3(hessian_at(u, p, 1, sy, sz, s, s4));
        else
            rv = F[p] - laplacian_at(u, p, 1, sy, sz, s);
        if (r)
            r[p] = rv;
    }
    const double t = block_sum<RES_BX * RES_BY / 64>(rv * rv);
    if (threadIdx.x == 0 && threadIdx.y == 0)
        partials[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * size_t(blockIdx.z))] = t;
}

// Fixed-order sum of count partials by one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_reduce(const double *__restrict__ partials,
                                                 size_t count, double *__restrict__ out)
{
    double v = 0.0;
    for (size_t q = threadIdx.x; q < count; q += 1024)
        v += partials[q];
    const double t = block_sum<16>(v);
    if (threadIdx.x == 0)
        out[0] = t;
}

// ---------------------------------------------------------------------------
// FAS restriction (Algorithm 1 steps 3-5) for coarse node P = (I,J,K):
//   w_H = u_H = u_h(2P) at every coarse node;
//   b_H = S_H(w_H) + I_h^H r_h at coarse interior nodes, 0 on the boundary.
// S_H reads the fine array at stride 2 (the injected coarse values).
// ---------------------------------------------------------------------------
template <int OP, int RMODE>
__global__ __launch_bounds__(RES_BX *RES_BY) void k_restrict(const double *__restrict__ uf,
                                                             const double *__restrict__ rf,
                                                             int nf, double *__restrict__ wc,
                                                             double *__restrict__ uc,
                                                             double *__restrict__ bc, double sc,
                                                             double s4c)
{
    const int nc = nf / 2;
    const int I = blockIdx.x * RES_BX + threadIdx.x;
    const int J = blockIdx.y * RES_BY + threadIdx.y;
    const int K = blockIdx.z;
    if (I > nc || J > nc)
        return;
    const long fy = nf + 1, fz = fy * fy;
    const long cy = nc + 1, cz = cy * cy;
    const long f = 2 * I + fy * (2 * J) + fz * (2 * K);
    const long c = I + cy * J + cz * K;
    const double v = uf[f];
    wc[c] = v;
    uc[c] = v;
    double b = 0.0;
    if (I >= 1 && I <= nc - 1 && J >= 1 && J <= nc - 1 && K >= 1 && K <= nc - 1) {
        double rh;
        if (RMODE == 0) {
            const double w[3] = {0.25, 0.5, 0.25};
            rh = 0.0;
#pragma unroll
            for (int dc = -1; dc <= 1; ++dc)
#pragma unroll
                for (int db = -1; db <= 1; ++db)
#pragma unroll
                    for (int da = -1; da <= 1; ++da)
                        rh += (w[dc + 1] * w[db + 1] * w[da + 1]) * rf[f + da + fy * db + fz * dc];
        } else {
            rh = (6.0 * rf[f] + (rf[f - 1] + rf[f + 1]) + (rf[f - fy] + rf[f + fy])
                  + (rf[f - fz] + rf[f + fz])) / 12.0;
        }
        double sh;
        if (OP == OP_MA)
            sh = det3(hessian_at(uf, f, 2, 2 * fy, 2 * fz, sc, s4c));
        else
            sh = laplacian_at(uf, f, 2, 2 * fy, 2 * fz, sc);
        b = sh + rh;
    }
    bc[c] = b;
}

// ---------------------------------------------------------------------------
// Coarse-grid correction (Algorithm 1 steps 7-8): u_h += I_H^h (u_H - w_H),
// trilinear; an even fine index takes the coincident coarse index with
// weight 1, an odd one both neighbours with weight 1/2.  Corners are summed
// with k, then j, then i ascending.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RES_BX *RES_BY) void k_prolong(double *__restrict__ uf, int nf,
                                                            const double *__restrict__ uc,
                                                            const double *__restrict__ wc)
{
    const int i = 1 + blockIdx.x * RES_BX + threadIdx.x;
    const int j = 1 + blockIdx.y * RES_BY + threadIdx.y;
    const int k = 1 + blockIdx.z;
    if (i > nf - 1 || j > nf - 1)
        return;
    const int nc = nf / 2;
    const long cy = nc + 1, cz = cy * cy;
    const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1, nk = (k & 1) ? 2 : 1;
    const double wi = (i & 1) ? 0.5 : 1.0, wj = (j & 1) ? 0.5 : 1.0, wk = (k & 1) ? 0.5 : 1.0;
    const int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
    double d = 0.0;
    for (int c = 0; c < nk; ++c)
        for (int b = 0; b < nj; ++b)
            for (int a = 0; a < ni; ++a) {
                const long q = (I0 + a) + cy * (J0 + b) + cz * (K0 + c);
                d += (wk * wj * wi) * (uc[q] - wc[q]);
            }
    const long fy = nf + 1;
    uf[i + fy * j + fy * fy * k] += d;
}

__global__ void k_poisson_rhs(const double *__restrict__ f, double *__restrict__ R, size_t count)
{
    const size_t q = blockIdx.x * size_t(blockDim.x) + threadIdx.x;
    if (q < count)
        R[q] = 3.0 * cbrt(f[q]);
}

__global__ void k_copy(const double *__restrict__ src, double *__restrict__ dst, size_t count)
{
    const size_t q = blockIdx.x * size_t(blockDim.x) + threadIdx.x;
    if (q < count)
        dst[q] = src[q];
}

__global__ void k_copy_boundary(const double *__restrict__ src, double *__restrict__ dst, int n)
{
    const int i = blockIdx.x * RES_BX + threadIdx.x;
    const int j = blockIdx.y * RES_BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i > n || j > n)
        return;
    if (i == 0 || i == n || j == 0 || j == n || k == 0 || k == n) {
        const long q = i + long(n + 1) * (j + long(n + 1) * k);
        dst[q] = src[q];
    }
}

// Injection onto the grid with half the intervals: every coarse node,
// boundary included, takes the fine value at the same point.
__global__ void k_inject_all(const double *__restrict__ vf, double *__restrict__ vc, int nc)
{
    const int I = blockIdx.x * RES_BX + threadIdx.x;
    const int J = blockIdx.y * RES_BY + threadIdx.y;
    const int K = blockIdx.z;
    if (I > nc || J > nc)
        return;
    const long fy = 2L * nc + 1, cy = nc + 1;
    vc[I + cy * (J + cy * K)] = vf[2 * I + fy * (2 * J + fy * 2 * K)];
}

// 1D rule of the FMG interpolation at fine index i (nf = 2 nc intervals):
// a coarse node is copied; a midpoint takes the cubic Lagrange value through
// the four nearest coarse nodes (one-sided next to the boundary), or the
// quadratic value when the coarse grid has only three nodes.
__device__ __forceinline__ int fmg_rule(int nc, int i, int &first, double w[4])
{
    if ((i & 1) == 0) {
        first = i >> 1;
        w[0] = 1.0;
        return 1;
    }
    const int m = i >> 1;  // midpoint between coarse m and m + 1
    if (nc < 3) {
        first = 0;
        w[0] = m == 0 ? 0.375 : -0.125;
        w[1] = 0.75;
        w[2] = m == 0 ? -0.125 : 0.375;
        return 3;
    }
    if (m == 0) {
        first = 0;
        w[0] = 0.3125; w[1] = 0.9375; w[2] = -0.3125; w[3] = 0.0625;
    } else if (m == nc - 1) {
        first = nc - 3;
        w[0] = 0.0625; w[1] = -0.3125; w[2] = 0.9375; w[3] = 0.3125;
    } else {
        first = m - 1;
        w[0] = -0.0625; w[1] = 0.5625; w[2] = 0.5625; w[3] = -0.0625;
    }
    return 4;
}

// FMG interpolation (Algorithm 2, step 4) into the interior of uf: tensor
// product of the 1D rule, accumulated over (k, j, i) offsets in order.
__global__ __launch_bounds__(RES_BX *RES_BY) void k_fmg_interp(const double *__restrict__ uc,
                                                               double *__restrict__ uf, int nc)
{
    const int nf = 2 * nc;
    const int i = 1 + blockIdx.x * RES_BX + threadIdx.x;
    const int j = 1 + blockIdx.y * RES_BY + threadIdx.y;
    const int k = 1 + blockIdx.z;
    if (i > nf - 1 || j > nf - 1)
        return;
    int fi, fj, fk;
    double wi[4], wj[4], wk[4];
    const int ci = fmg_rule(nc, i, fi, wi);
    const int cj = fmg_rule(nc, j, fj, wj);
    const int ck = fmg_rule(nc, k, fk, wk);
    const long cy = nc + 1;
    double v = 0.0;
    for (int c = 0; c < ck; ++c)
        for (int b = 0; b < cj; ++b)
            for (int a = 0; a < ci; ++a)
                v += wk[c] * wj[b] * wi[a] * uc[(fi + a) + cy * ((fj + b) + cy * (fk + c))];
    uf[i + long(nf + 1) * (j + long(nf + 1) * k)] = v;
}

// Zero the interior nodes of an (n+1)^3 grid.
__global__ void k_zero_interior(double *__restrict__ u, int n)
{
    const int i = 1 + blockIdx.x * RES_BX + threadIdx.x;
    const int j = 1 + blockIdx.y * RES_BY + threadIdx.y;
    const int k = 1 + blockIdx.z;
    if (i > n - 1 || j > n - 1)
        return;
    u[i + long(n + 1) * (j + long(n + 1) * k)] = 0.0;
}

inline dim3 res_grid(int cnt_x, int cnt_y, int cnt_z)
{
    return dim3((cnt_x + RES_BX - 1) / RES_BX, (cnt_y + RES_BY - 1) / RES_BY, cnt_z);
}

} // namespace

size_t residual_partials(int n)
{
    const dim3 g = res_grid(n - 1, n - 1, n - 1);
    return size_t(g.x) * g.y * g.z;
}

hipError_t launch_sweep_color(hipStream_t st, int op, int order, int n, double *u,
                              const double *F, unsigned long long *nonconvex)
{
    const double s = double(n) * double(n), s4 = 0.25 * s;
    const double hk = op == OP_MA ? 0.5 / s : 1.0 / (6.0 * s);
    const int ncol = order == 1 ? 8 : 4;
    const int gx = ((n + 1) / 2 + 63) / 64;
    const int gy = order == 0 ? n - 1 : n / 2, gz = n / 2;
    const int nb = gx * gy * gz;
    for (int c = 0; c < ncol; ++c) {
#define MA_COLOR_LAUNCH(OPV, ORD)                                                                \
    hipLaunchKernelGGL((k_sweep_color<OPV, ORD>), dim3(nb), dim3(64), 0, st, u, F, n, c, gx, gy,  \
                       nb, s, s4, hk, nonconvex)
        if (op == OP_MA) {
            if (order == 0)
                MA_COLOR_LAUNCH(OP_MA, 0);
            else
                MA_COLOR_LAUNCH(OP_MA, 1);
        } else {
            if (order == 0)
                MA_COLOR_LAUNCH(OP_LAP, 0);
            else
                MA_COLOR_LAUNCH(OP_LAP, 1);
        }
#undef MA_COLOR_LAUNCH
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_residual(hipStream_t st, int op, int n, const double *u, const double *F,
                           double *r, double *partials)
{
    const double s = double(n) * double(n), s4 = 0.25 * s;
    const dim3 grid = res_grid(n - 1, n - 1, n - 1), block(RES_BX, RES_BY);
    if (op == OP_MA)
        hipLaunchKernelGGL((k_residual<OP_MA>), grid, block, 0, st, u, F, r, partials, n, s, s4);
    else
        hipLaunchKernelGGL((k_residual<OP_LAP>), grid, block, 0, st, u, F, r, partials, n, s, s4);
    return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t st, const double *partials, size_t count, double *out)
{
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, partials, count, out);
    return hipGetLastError();
}

hipError_t launch_restrict(hipStream_t st, int op, int rmode, int nf, const double *uf,
                           const double *rf, double *wc, double *uc, double *bc)
{
    const int nc = nf / 2;
    const double sc = double(nc) * double(nc), s4c = 0.25 * sc;
    const dim3 grid = res_grid(nc + 1, nc + 1, nc + 1), block(RES_BX, RES_BY);
#define MA_RESTRICT_LAUNCH(OPV, RM)                                                              \
    hipLaunchKernelGGL((k_restrict<OPV, RM>), grid, block, 0, st, uf, rf, nf, wc, uc, bc, sc, s4c)
    if (op == OP_MA) {
        if (rmode == 0)
            MA_RESTRICT_LAUNCH(OP_MA, 0);
        else
            MA_RESTRICT_LAUNCH(OP_MA, 1);
    } else {
        if (rmode == 0)
            MA_RESTRICT_LAUNCH(OP_LAP, 0);
        else
            MA_RESTRICT_LAUNCH(OP_LAP, 1);
    }
#undef MA_RESTRICT_LAUNCH
    return hipGetLastError();
}

hipError_t launch_prolong(hipStream_t st, int nf, double *uf, const double *uc, const double *wc)
{
    const dim3 grid = res_grid(nf - 1, nf - 1, nf - 1), block(RES_BX, RES_BY);
    hipLaunchKernelGGL(k_prolong, grid, block, 0, st, uf, nf, uc, wc);
    return hipGetLastError();
}

hipError_t launch_poisson_rhs(hipStream_t st, int n, const double *f, double *R)
{
    const size_t cnt = npts(n);
    hipLaunchKernelGGL(k_poisson_rhs, dim3((cnt + 255) / 256), dim3(256), 0, st, f, R, cnt);
    return hipGetLastError();
}

hipError_t launch_copy(hipStream_t st, size_t count, const double *src, double *dst)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3((count + 255) / 256), dim3(256), 0, st, src, dst, count);
    return hipGetLastError();
}

hipError_t launch_inject_all(hipStream_t st, int nf, const double *vf, double *vc)
{
    const int nc = nf / 2;
    hipLaunchKernelGGL(k_inject_all, res_grid(nc + 1, nc + 1, nc + 1), dim3(RES_BX, RES_BY), 0, st,
                       vf, vc, nc);
    return hipGetLastError();
}

hipError_t launch_fmg_interp(hipStream_t st, int nc, const double *uc, double *uf)
{
    const int nf = 2 * nc;
    hipLaunchKernelGGL(k_fmg_interp, res_grid(nf - 1, nf - 1, nf - 1), dim3(RES_BX, RES_BY), 0, st,
                       uc, uf, nc);
    return hipGetLastError();
}

hipError_t launch_zero_interior(hipStream_t st, int n, double *u)
{
    if (n < 2)
        return hipSuccess;
    hipLaunchKernelGGL(k_zero_interior, res_grid(n - 1, n - 1, n - 1), dim3(RES_BX, RES_BY), 0, st,
                       u, n);
    return hipGetLastError();
}

hipError_t launch_copy_boundary(hipStream_t st, int n, const double *src, double *dst)
{
    const dim3 grid = res_grid(n + 1, n + 1, n + 1), block(RES_BX, RES_BY);
    hipLaunchKernelGGL(k_copy_boundary, grid, block, 0, st, src, dst, n);
    return hipGetLastError();
}

} // namespace mafas

namespace mafas {
namespace {
template <typename T>
__global__ void k_fill(T *__restrict__ dst, size_t count, T v)
{
    const size_t q = blockIdx.x * size_t(blockDim.x) + threadIdx.x;
    if (q < count)
        dst[q] = v;
}
} // namespace

hipError_t launch_fill(hipStream_t st, size_t count, double v, double *dst)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill<double>, dim3((count + 255) / 256), dim3(256), 0, st, dst, count, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(hipStream_t st, size_t count, unsigned long long v,
                           unsigned long long *dst)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3((count + 255) / 256), dim3(256), 0, st, dst,
                       count, v);
    return hipGetLastError();
}

} // namespace mafas
