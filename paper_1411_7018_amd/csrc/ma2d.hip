// Two-dimensional variant (include/ma2d.h): 9-point nonlinear Gauss-Seidel
// smoother, FAS V-cycle and FMG for u_xx u_yy - u_xy^2 = f.  Single-grid
// kernels on 64 x 4 thread blocks (x fastest, coalesced rows) driven from
// the host level by level: a 2D grid of the sizes this variant targets
// (up to 8193^2) fills the chip on its own, so no batching is needed.
#include "ma2d.h"
#include "ma_runtime.h"

#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace {

constexpr int BX = 64, BY = 4;

struct H2 {
    double xx, yy, xy;
};

// Discrete Hessian at linear index p of an (n+1)^2 grid with row stride sy
// and node spacing step (1 for the grid itself, 2 for the coarse operator
// evaluated on the fine array); s = 1/h^2 of the spacing used.
__device__ __forceinline__ H2 hess2(const double *__restrict__ u, long p, long sx, long sy,
                                    double s)
{
    const double c = u[p];
    H2 g;
    g.xx = ((u[p + sx] - c) - (c - u[p - sx])) * s;
    g.yy = ((u[p + sy] - c) - (c - u[p - sy])) * s;
    g.xy = ((u[p + sx + sy] - u[p - sx + sy]) - (u[p + sx - sy] - u[p - sx - sy])) * (0.25 * s);
    return g;
}

__device__ __forceinline__ double det2(const H2 &g) { return g.xx * g.yy - g.xy * g.xy; }

// Smaller root of (xx - sigma)(yy - sigma) - xy^2 = F.  With t = tr G and
// D = (xx - yy)^2 + 4 xy^2 + 4 F the roots are (t -+ sqrt D) / 2; for t > 0
// the smaller one is evaluated as 2 (det G - F) / (t + sqrt D), free of
// cancellation.  D < 0 (no real root, F far below zero): the vertex t / 2.
__device__ __forceinline__ double root2(const H2 &g, double F, bool &nonconvex)
{
    const double t = g.xx + g.yy;
    const double a = g.xx - g.yy;
    const double D = a * a + 4.0 * g.xy * g.xy + 4.0 * F;
    if (!(F > 0.0))
        nonconvex = true;
    if (D < 0.0) {
        nonconvex = true;
        return 0.5 * t;
    }
    const double r = sqrt(D);
    if (t > 0.0)
        return 2.0 * (det2(g) - F) / (t + r);
    return 0.5 * (t - r);
}

// 4-colour sweep phase: colour points (i, j) with i = ip + 2 ii, j = jp + 2 jj.
__global__ __launch_bounds__(BX *BY) void k2_sweep4(double *__restrict__ u,
                                                    const double *__restrict__ F, int n,
                                                    int color, unsigned long long *cnt)
{
    const int i = ((color & 1) ? 1 : 2) + 2 * int(blockIdx.x * BX + threadIdx.x);
    const int j = ((color & 2) ? 1 : 2) + 2 * int(blockIdx.y * BY + threadIdx.y);
    if (i > n - 1 || j > n - 1)
        return;
    const long sy = n + 1, p = i + sy * j;
    const double s = double(n) * double(n);
    bool nc = false;
    const double sig = root2(hess2(u, p, 1, sy, s), F[p], nc);
    u[p] += sig * (0.5 / s);
    if (nc)
        atomicAdd(cnt, 1ull);
}

// Red-black phase, first half: every node with (i + j) mod 2 == color from
// the values before the phase, into t.
__global__ __launch_bounds__(BX *BY) void k2_sweep_rb(const double *__restrict__ u,
                                                      const double *__restrict__ F,
                                                      double *__restrict__ t, int n, int color,
                                                      unsigned long long *cnt)
{
    const int j = 1 + int(blockIdx.y * BY + threadIdx.y);
    const int i = (((color + j) & 1) ? 1 : 2) + 2 * int(blockIdx.x * BX + threadIdx.x);
    if (i > n - 1 || j > n - 1)
        return;
    const long sy = n + 1, p = i + sy * j;
    const double s = double(n) * double(n);
    bool nc = false;
    const double sig = root2(hess2(u, p, 1, sy, s), F[p], nc);
    t[p] = u[p] + sig * (0.5 / s);
    if (nc)
        atomicAdd(cnt, 1ull);
}

// Red-black phase, second half: the colour's new values into u.
__global__ __launch_bounds__(BX *BY) void k2_commit_rb(const double *__restrict__ t,
                                                       double *__restrict__ u, int n, int color)
{
    const int j = 1 + int(blockIdx.y * BY + threadIdx.y);
    const int i = (((color + j) & 1) ? 1 : 2) + 2 * int(blockIdx.x * BX + threadIdx.x);
    if (i > n - 1 || j > n - 1)
        return;
    const long p = i + long(n + 1) * j;
    u[p] = t[p];
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

// r = F - det(D^2 u) at interior nodes (r may be null) and one partial sum
// of r^2 per block, summed in a fixed order.
__global__ __launch_bounds__(BX *BY) void k2_residual(const double *__restrict__ u,
                                                      const double *__restrict__ F,
                                                      double *__restrict__ r,
                                                      double *__restrict__ part, int n)
{
    __shared__ double ws[BY];
    const int i = 1 + int(blockIdx.x * BX + threadIdx.x);
    const int j = 1 + int(blockIdx.y * BY + threadIdx.y);
    double rv = 0.0;
    if (i <= n - 1 && j <= n - 1) {
        const long sy = n + 1, p = i + sy * j;
        rv = F[p] - det2(hess2(u, p, 1, sy, double(n) * double(n)));
        if (r)
            r[p] = rv;
    }
    const double w = wave_sum(rv * rv);
    if (threadIdx.x == 0)
        ws[threadIdx.y] = w;
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0)
        part[blockIdx.x + gridDim.x * blockIdx.y] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

// FAS restriction at coarse node (I, J): w_H = u_H = u_h(2I, 2J); at coarse
// interior nodes b_H = det(D^2_H w_H) + restricted residual.
__global__ __launch_bounds__(BX *BY) void k2_restrict(const double *__restrict__ uf,
                                                      const double *__restrict__ rf,
                                                      double *__restrict__ wc,
                                                      double *__restrict__ uc,
                                                      double *__restrict__ bc, int nf, int half)
{
    const int nc = nf / 2;
    const int I = int(blockIdx.x * BX + threadIdx.x);
    const int J = int(blockIdx.y * BY + threadIdx.y);
    if (I > nc || J > nc)
        return;
    const long fy = nf + 1, f = 2 * I + fy * (2 * J), c = I + long(nc + 1) * J;
    wc[c] = uf[f];
    uc[c] = uf[f];
    double b = 0.0;
    if (I >= 1 && I <= nc - 1 && J >= 1 && J <= nc - 1) {
        double rh;
        if (half) {
            rh = (4.0 * rf[f] + (rf[f - 1] + rf[f + 1]) + (rf[f - fy] + rf[f + fy])) / 8.0;
        } else {
            const double w[3] = {0.25, 0.5, 0.25};
            rh = 0.0;
#pragma unroll
            for (int b2 = -1; b2 <= 1; ++b2)
#pragma unroll
                for (int a2 = -1; a2 <= 1; ++a2)
                    rh += (w[b2 + 1] * w[a2 + 1]) * rf[f + a2 + fy * b2];
        }
        b = det2(hess2(uf, f, 2, 2 * fy, double(nc) * double(nc))) + rh;
    }
    bc[c] = b;
}

// u_f += bilinear interpolation of (u_c - w_c) at fine interior nodes.
__global__ __launch_bounds__(BX *BY) void k2_prolong(double *__restrict__ uf,
                                                     const double *__restrict__ uc,
                                                     const double *__restrict__ wc, int nf)
{
    const int i = 1 + int(blockIdx.x * BX + threadIdx.x);
    const int j = 1 + int(blockIdx.y * BY + threadIdx.y);
    if (i > nf - 1 || j > nf - 1)
        return;
    const long cy = nf / 2 + 1;
    const int I0 = i >> 1, J0 = j >> 1;
    const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1;
    const double wi = (i & 1) ? 0.5 : 1.0, wj = (j & 1) ? 0.5 : 1.0;
    double d = 0.0;
    for (int b = 0; b < nj; ++b)
        for (int a = 0; a < ni; ++a) {
            const long q = (I0 + a) + cy * (J0 + b);
            d += (wj * wi) * (uc[q] - wc[q]);
        }
    uf[i + long(nf + 1) * j] += d;
}

__global__ __launch_bounds__(BX *BY) void k2_inject(const double *__restrict__ vf,
                                                    double *__restrict__ vc, int nf)
{
    const int nc = nf / 2;
    const int I = int(blockIdx.x * BX + threadIdx.x);
    const int J = int(blockIdx.y * BY + threadIdx.y);
    if (I > nc || J > nc)
        return;
    vc[I + long(nc + 1) * J] = vf[2 * I + long(nf + 1) * (2 * J)];
}

// 1D rule of the FMG interpolation (a coarse node is copied; a midpoint
// takes the cubic Lagrange value through the 4 nearest coarse nodes,
// one-sided at the boundary; quadratic on a 3-node grid).
__device__ __forceinline__ int rule2(int nc, int i, int &first, double w[4])
{
    if ((i & 1) == 0) {
        first = i >> 1;
        w[0] = 1.0;
        return 1;
    }
    const int m = i >> 1;
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

__global__ __launch_bounds__(BX *BY) void k2_fmg_interp(const double *__restrict__ uc,
                                                        double *__restrict__ uf, int nc)
{
    const int nf = 2 * nc;
    const int i = 1 + int(blockIdx.x * BX + threadIdx.x);
    const int j = 1 + int(blockIdx.y * BY + threadIdx.y);
    if (i > nf - 1 || j > nf - 1)
        return;
    int fi, fj;
    double wi[4], wj[4];
    const int ci = rule2(nc, i, fi, wi);
    const int cj = rule2(nc, j, fj, wj);
    const long cy = nc + 1;
    double v = 0.0;
    for (int b = 0; b < cj; ++b)
        for (int a = 0; a < ci; ++a)
            v += wj[b] * wi[a] * uc[(fi + a) + cy * (fj + b)];
    uf[i + long(nf + 1) * j] = v;
}

__global__ __launch_bounds__(BX *BY) void k2_zero_interior(double *__restrict__ u, int n)
{
    const int i = 1 + int(blockIdx.x * BX + threadIdx.x);
    const int j = 1 + int(blockIdx.y * BY + threadIdx.y);
    if (i > n - 1 || j > n - 1)
        return;
    u[i + long(n + 1) * j] = 0.0;
}

inline dim3 grid2(int cx, int cy) { return dim3((cx + BX - 1) / BX, (cy + BY - 1) / BY); }

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

thread_local std::string g_err2;

bool valid2(const ma2d_params *p, std::string &why)
{
    if (!p) {
        why = "params is NULL";
        return false;
    }
    if (p->n < 2 || p->n > 65536) {
        why = "n must satisfy 2 <= n <= 65536";
        return false;
    }
    if (p->nu1 < 0 || p->nu2 < 0 || p->nu0 < 1 || p->nu1 > 16 || p->nu2 > 16 || p->nu0 > 16) {
        why = "smoothing counts must satisfy 0 <= nu1, nu2 <= 16 and 1 <= nu0 <= 16";
        return false;
    }
    if (p->order != MA2D_COLOR4 && p->order != MA2D_RED_BLACK) {
        why = "order must be MA2D_COLOR4 or MA2D_RED_BLACK";
        return false;
    }
    if (p->restriction != MA_RESTRICT_FULL && p->restriction != MA_RESTRICT_HALF) {
        why = "restriction must be MA_RESTRICT_FULL or MA_RESTRICT_HALF";
        return false;
    }
    if (p->max_cycles < 0 || !std::isfinite(p->tol)) {
        why = "max_cycles must be >= 0 and tol finite";
        return false;
    }
    return true;
}

int levels2(int n, int *ns, int cap)
{
    int L = 0;
    ns[L++] = n;
    while (n % 2 == 0 && n >= 4 && L < cap) {
        n /= 2;
        ns[L++] = n;
    }
    return L;
}

size_t pts2(int n) { return size_t(n + 1) * size_t(n + 1); }

size_t partials2(int n) { return size_t((n - 1 + BX - 1) / BX) * size_t((n - 1 + BY - 1) / BY); }

} // namespace

struct ma2d_solver {
    ma2d_params p{};
    hipStream_t st = nullptr;
    std::vector<int> ns;
    std::vector<double *> u, b, w, r, t;   // per level (u, b, w unused on level 0)
    double *part = nullptr, *dsum = nullptr, *hpin = nullptr;
    unsigned long long *cnt = nullptr, *hcnt = nullptr;
    std::vector<void *> owned;
    std::string err;

    ~ma2d_solver()
    {
        if (st)
            (void)hipStreamSynchronize(st);
        for (void *q : owned)
            (void)hipFree(q);
        if (hpin)
            (void)hipHostFree(hpin);
        if (hcnt)
            (void)hipHostFree(hcnt);
    }
    ma_status fail(ma_status s, const std::string &m)
    {
        err = m;
        return s;
    }
    ma_status alloc(double **q, size_t count)
    {
        const hipError_t e = hipMalloc(reinterpret_cast<void **>(q), count * sizeof(double));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *q = nullptr;
            return fail(MA_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        owned.push_back(*q);
        return MA_OK;
    }
};

#define H2_HIP(s, expr)                                                                          \
    do {                                                                                         \
        const hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                                    \
            return (s)->fail(MA_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)
#define H2_TRY(expr)                                                                             \
    do {                                                                                         \
        const ma_status s_ = (expr);                                                             \
        if (s_ != MA_OK)                                                                         \
            return s_;                                                                           \
    } while (0)

namespace {

ma_status sweep2(ma2d_solver *s, int l, double *u, const double *F, int count)
{
    const int n = s->ns[l];
    for (int k = 0; k < count; ++k) {
        if (s->p.order == MA2D_COLOR4) {
            for (int c = 0; c < 4; ++c) {
                hipLaunchKernelGGL(k2_sweep4, grid2(n / 2, n / 2), dim3(BX, BY), 0, s->st, u, F,
                                   n, c, s->cnt);
                H2_HIP(s, hipGetLastError());
            }
        } else {
            for (int c = 0; c < 2; ++c) {
                hipLaunchKernelGGL(k2_sweep_rb, grid2(n / 2, n - 1), dim3(BX, BY), 0, s->st, u,
                                   F, s->t[l], n, c, s->cnt);
                H2_HIP(s, hipGetLastError());
                hipLaunchKernelGGL(k2_commit_rb, grid2(n / 2, n - 1), dim3(BX, BY), 0, s->st,
                                   s->t[l], u, n, c);
                H2_HIP(s, hipGetLastError());
            }
        }
    }
    return MA_OK;
}

// residual of level l into r (may be null) and, with l2 set, its norm
ma_status residual2(ma2d_solver *s, int l, const double *u, const double *F, double *r,
                    double *l2)
{
    const int n = s->ns[l];
    const dim3 g = grid2(n - 1, n - 1);
    hipLaunchKernelGGL(k2_residual, g, dim3(BX, BY), 0, s->st, u, F, r, s->part, n);
    H2_HIP(s, hipGetLastError());
    if (l2) {
        H2_HIP(s, mafas::launch_reduce(s->st, s->part, size_t(g.x) * g.y, s->dsum));
        H2_HIP(s, hipMemcpyAsync(s->hpin, s->dsum, sizeof(double), hipMemcpyDeviceToHost, s->st));
        H2_HIP(s, hipStreamSynchronize(s->st));
        *l2 = std::sqrt(s->hpin[0]) / double(n);
    }
    return MA_OK;
}

ma_status vcycle2(ma2d_solver *s, int l, double *u, const double *b)
{
    const int L = int(s->ns.size());
    const int n = s->ns[l];
    if (l == L - 1)
        return sweep2(s, l, u, b, s->p.nu0);
    H2_TRY(sweep2(s, l, u, b, s->p.nu1));
    H2_TRY(residual2(s, l, u, b, s->r[l], nullptr));
    const int nc = s->ns[l + 1];
    hipLaunchKernelGGL(k2_restrict, grid2(nc + 1, nc + 1), dim3(BX, BY), 0, s->st, u, s->r[l],
                       s->w[l + 1], s->u[l + 1], s->b[l + 1], n,
                       s->p.restriction == MA_RESTRICT_HALF ? 1 : 0);
    H2_HIP(s, hipGetLastError());
    H2_TRY(vcycle2(s, l + 1, s->u[l + 1], s->b[l + 1]));
    hipLaunchKernelGGL(k2_prolong, grid2(n - 1, n - 1), dim3(BX, BY), 0, s->st, u, s->u[l + 1],
                       s->w[l + 1], n);
    H2_HIP(s, hipGetLastError());
    return sweep2(s, l, u, b, s->p.nu2);
}

ma_status fmg2(ma2d_solver *s, double *u, const double *f)
{
    const int L = int(s->ns.size());
    auto U = [&](int l) { return l == 0 ? u : s->u[l]; };
    auto B = [&](int l) -> const double * { return l == 0 ? f : s->b[l]; };
    for (int l = 1; l < L; ++l) {
        const int nc = s->ns[l];
        hipLaunchKernelGGL(k2_inject, grid2(nc + 1, nc + 1), dim3(BX, BY), 0, s->st, B(l - 1),
                           s->b[l], s->ns[l - 1]);
        H2_HIP(s, hipGetLastError());
        hipLaunchKernelGGL(k2_inject, grid2(nc + 1, nc + 1), dim3(BX, BY), 0, s->st, U(l - 1),
                           s->u[l], s->ns[l - 1]);
        H2_HIP(s, hipGetLastError());
    }
    // coarsest: zero inside, then an approximate solve (nu0 sweeps solve a
    // one-unknown grid exactly; a 3-interval grid takes 8)
    const int c = L - 1, n0 = s->ns[c];
    hipLaunchKernelGGL(k2_zero_interior, grid2(n0 - 1, n0 - 1), dim3(BX, BY), 0, s->st, U(c), n0);
    H2_HIP(s, hipGetLastError());
    H2_TRY(sweep2(s, c, U(c), B(c), (n0 == 3 && s->p.nu0 < 8) ? 8 : s->p.nu0));
    for (int l = L - 2; l >= 0; --l) {
        const int n = s->ns[l];
        hipLaunchKernelGGL(k2_fmg_interp, grid2(n - 1, n - 1), dim3(BX, BY), 0, s->st, U(l + 1),
                           U(l), s->ns[l + 1]);
        H2_HIP(s, hipGetLastError());
        H2_TRY(vcycle2(s, l, U(l), B(l)));
    }
    return MA_OK;
}

ma_status read_count(ma2d_solver *s, long long *out)
{
    H2_HIP(s, hipMemcpyAsync(s->hcnt, s->cnt, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                             s->st));
    H2_HIP(s, hipStreamSynchronize(s->st));
    *out = (long long)s->hcnt[0];
    return MA_OK;
}

// point updates of one V-cycle and of the FMG start (sweeps on every level)
double vcycle_updates(const ma2d_solver *s)
{
    double up = 0.0;
    const int L = int(s->ns.size());
    for (int l = 0; l < L; ++l) {
        const double in = double(s->ns[l] - 1) * double(s->ns[l] - 1);
        up += (l < L - 1 ? s->p.nu1 + s->p.nu2 : s->p.nu0) * in;
    }
    return up;
}

} // namespace

extern "C" {

void ma2d_params_default(ma2d_params *p, int n)
{
    std::memset(p, 0, sizeof(*p));
    p->n = n;
    p->nu1 = 2;
    p->nu2 = 2;
    p->nu0 = 1;
    p->order = MA2D_RED_BLACK;
    p->restriction = MA_RESTRICT_HALF;
    p->max_cycles = 100;
    p->tol = 1e-6;
}

size_t ma2d_footprint_bytes(const ma2d_params *p)
{
    std::string why;
    if (!valid2(p, why))
        return 0;
    int ns[40];
    const int L = levels2(p->n, ns, 40);
    size_t b = 0;
    for (int l = 0; l < L; ++l)
        b += (l == 0 ? 2 : 5) * pts2(ns[l]) * sizeof(double);
    return b + partials2(p->n) * sizeof(double) + 4096;
}

ma_status ma2d_create(const ma2d_params *p, void *hip_stream, ma2d_solver **out)
{
    std::string why;
    if (!out) {
        g_err2 = "out is NULL";
        return MA_ERR_ARG;
    }
    *out = nullptr;
    if (!valid2(p, why)) {
        g_err2 = why;
        return MA_ERR_ARG;
    }
    ma2d_solver *s = new ma2d_solver();
    s->p = *p;
    s->st = static_cast<hipStream_t>(hip_stream);
    int ns[40];
    const int L = levels2(p->n, ns, 40);
    s->ns.assign(ns, ns + L);
    s->u.assign(L, nullptr);
    s->b.assign(L, nullptr);
    s->w.assign(L, nullptr);
    s->r.assign(L, nullptr);
    s->t.assign(L, nullptr);
    ma_status st = MA_OK;
    for (int l = 0; l < L && st == MA_OK; ++l) {
        const size_t c = pts2(ns[l]);
        if (l > 0) {
            st = s->alloc(&s->u[l], c);
            if (st == MA_OK)
                st = s->alloc(&s->b[l], c);
            if (st == MA_OK)
                st = s->alloc(&s->w[l], c);
        }
        if (st == MA_OK)
            st = s->alloc(&s->r[l], c);
        if (st == MA_OK)
            st = s->alloc(&s->t[l], c);
        if (st == MA_OK) {
            // the boundary layer of every array is never written by the
            // kernels: start them all at zero
            if (hipMemsetAsync(s->r[l], 0, c * sizeof(double), s->st) != hipSuccess ||
                hipMemsetAsync(s->t[l], 0, c * sizeof(double), s->st) != hipSuccess)
                st = s->fail(MA_ERR_DEVICE, "clearing the hierarchy");
        }
    }
    if (st == MA_OK)
        st = s->alloc(&s->part, partials2(p->n));
    if (st == MA_OK)
        st = s->alloc(&s->dsum, 4);
    if (st == MA_OK) {
        void *q = nullptr;
        if (hipMalloc(&q, 64) != hipSuccess)
            st = s->fail(MA_ERR_OOM, "hipMalloc of the counter");
        else {
            s->owned.push_back(q);
            s->cnt = static_cast<unsigned long long *>(q);
        }
    }
    if (st == MA_OK && (hipHostMalloc(reinterpret_cast<void **>(&s->hpin), 4 * sizeof(double)) !=
                            hipSuccess ||
                        hipHostMalloc(reinterpret_cast<void **>(&s->hcnt),
                                      4 * sizeof(unsigned long long)) != hipSuccess))
        st = s->fail(MA_ERR_OOM, "hipHostMalloc failed");
    if (st == MA_OK && hipStreamSynchronize(s->st) != hipSuccess)
        st = s->fail(MA_ERR_DEVICE, "allocation");
    if (st != MA_OK) {
        g_err2 = s->err;
        delete s;
        return st;
    }
    *out = s;
    return MA_OK;
}

void ma2d_destroy(ma2d_solver *s) { delete s; }

const char *ma2d_last_error(const ma2d_solver *s) { return s ? s->err.c_str() : g_err2.c_str(); }

ma_status ma2d_sweep(ma2d_solver *s, double *u, const double *f, int count,
                     long long *nonconvex_host)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f || count < 0)
        return s->fail(MA_ERR_ARG, "u, f must be device pointers and count >= 0");
    H2_HIP(s, mafas::launch_fill_u64(s->st, 1, 0ull, s->cnt));
    H2_TRY(sweep2(s, 0, u, f, count));
    if (nonconvex_host)
        H2_TRY(read_count(s, nonconvex_host));
    return MA_OK;
}

ma_status ma2d_residual(ma2d_solver *s, const double *u, const double *f, double *r_or_null,
                        double *l2_host)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f)
        return s->fail(MA_ERR_ARG, "u and f must be device pointers");
    if (r_or_null)
        H2_HIP(s, hipMemsetAsync(r_or_null, 0, pts2(s->p.n) * sizeof(double), s->st));
    double l2 = 0.0;
    H2_TRY(residual2(s, 0, u, f, r_or_null, l2_host ? &l2 : nullptr));
    if (l2_host)
        *l2_host = l2;
    return MA_OK;
}

ma_status ma2d_vcycle(ma2d_solver *s, double *u, const double *f)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f)
        return s->fail(MA_ERR_ARG, "u and f must be device pointers");
    return vcycle2(s, 0, u, f);
}

ma_status ma2d_fmg(ma2d_solver *s, double *u, const double *f, long long *nonconvex_host)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f)
        return s->fail(MA_ERR_ARG, "u and f must be device pointers");
    H2_HIP(s, mafas::launch_fill_u64(s->st, 1, 0ull, s->cnt));
    H2_TRY(fmg2(s, u, f));
    long long nc = 0;
    H2_TRY(read_count(s, &nc));
    if (nonconvex_host)
        *nonconvex_host = nc;
    return MA_OK;
}

ma_status ma2d_solve(ma2d_solver *s, double *u, const double *f, double tol, unsigned flags,
                     ma_report *rep)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f)
        return s->fail(MA_ERR_ARG, "u and f must be device pointers");
    if (flags & MA_INIT_POISSON)
        return s->fail(MA_ERR_ARG, "the 2D solver starts from u or from MA_INIT_FMG");
    const double t0 = now_s();
    const double target = tol > 0.0 ? tol : s->p.tol;
    const int n = s->p.n;
    ma_report r;
    std::memset(&r, 0, sizeof(r));
    H2_HIP(s, mafas::launch_fill_u64(s->st, 1, 0ull, s->cnt));
    const bool fmg = (flags & MA_INIT_FMG) != 0;
    if (fmg) {
        hipLaunchKernelGGL(k2_zero_interior, grid2(n - 1, n - 1), dim3(BX, BY), 0, s->st, u, n);
        H2_HIP(s, hipGetLastError());
    }
    H2_TRY(residual2(s, 0, u, f, nullptr, &r.res0));
    r.res = r.res0;
    const double vc_up = vcycle_updates(s);
    const double in0 = double(n - 1) * double(n - 1);
    ma_status st = MA_ERR_NOT_CONVERGED;
    if (!std::isfinite(r.res0)) {
        st = MA_ERR_NONFINITE;
    } else {
        if (fmg) {
            H2_TRY(fmg2(s, u, f));
            r.cycles = 1;
            r.point_updates += vc_up * (4.0 / 3.0);
            H2_TRY(residual2(s, 0, u, f, nullptr, &r.res));
            r.history[0] = r.res;
        }
        if (!std::isfinite(r.res))
            st = MA_ERR_NONFINITE;
        else if (r.res <= target * r.res0)
            st = MA_OK;
        while (st == MA_ERR_NOT_CONVERGED && r.cycles < s->p.max_cycles) {
            H2_TRY(vcycle2(s, 0, u, f));
            r.cycles += 1;
            r.point_updates += vc_up;
            H2_TRY(residual2(s, 0, u, f, nullptr, &r.res));
            if (r.cycles <= 64)
                r.history[r.cycles - 1] = r.res;
            if (!std::isfinite(r.res))
                st = MA_ERR_NONFINITE;
            else if (r.res <= target * r.res0)
                st = MA_OK;
        }
    }
    r.rel_res = r.res0 > 0.0 ? r.res / r.res0 : 0.0;
    r.converged = st == MA_OK;
    r.alg_bytes = r.point_updates * 24.0 + double(r.cycles + 1) * 16.0 * in0;
    long long nc = 0;
    H2_TRY(read_count(s, &nc));
    r.nonconvex = nc;
    r.seconds = now_s() - t0;
    if (rep)
        *rep = r;
    if (st == MA_ERR_NOT_CONVERGED)
        return s->fail(st, "max_cycles reached before the tolerance");
    if (st == MA_ERR_NONFINITE)
        return s->fail(st, "residual is not finite");
    return MA_OK;
}

} // extern "C"
