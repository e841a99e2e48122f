// One complete 4-colour Gauss-Seidel sweep in a single launch.
//
// The sweep is the same as four per-colour phases (colour c = ((i+j) mod 2)
// + 2 ((i+k) mod 2), phases 0..3), but each workgroup streams its tile
// through the z direction with the four phases skewed by one plane: at step
// t it applies phase 0 to plane t, phase 1 to plane t-1, phase 2 to t-2 and
// phase 3 to t-3.  Each phase reads its stencil neighbours in planes p-1,
// p, p+1, which at that moment hold exactly the values the globally phased
// sweep would see (nodes of one colour are never stencil neighbours, so
// whether a neighbour plane has already taken the same phase does not
// matter).  Six z-planes of the tile (t-4 .. t+1) live in an LDS ring.
//
// Tiles own a TX x TY x zc block of output nodes.  A colour phase at a node
// needs its neighbours after the previous phase, so the valid region of a
// tile shrinks by one node per phase: the tile loads a halo of 4 nodes in x
// and y, and phase c is computed on the core grown by 3 - c nodes (also in
// z at the ends of a z-chunk).  The sweep reads u_in and writes u_out, so
// halos read from a neighbouring tile are never modified during the launch
// and every tile computes exactly the values of the global 4-phase sweep.
//
// Bytes per interior node (one launch): read u 8, read F 8, write u 8.
#include "ma_device.h"
#include "ma_internal.h"

namespace mafas {

namespace {

constexpr int HALO = 4;
constexpr int NSLOT = 6;

// Colour-c nodes of plane p inside the core grown by 3 - c: rows
// j = c0 + c1 + p (mod 2), columns i = c0 + j (mod 2), stride 2 in both.
struct PhaseGeom {
    int is, js, nr, ncol;  // first node, row and column counts
    int off0;              // LDS offset of node (is, js) within a plane
    int px;                // parity of (is - lx0): which half of an LDS row
};

// LDS planes store each row de-interleaved by x parity: positions
// lx = 0, 2, 4, ... in the first half of the row and 1, 3, 5, ... in the
// second, so the nodes of one colour in a row (all of one parity) are
// contiguous and a wavefront reads them without bank conflicts.
//
// Lane mapping: a wavefront covers RPW = 64 / (W/2) rows, one lane per
// colour node of a row; wave w takes rows w*RPW + NW*RPW*k, k < R.
template <int OP, int TX, int TY, int NW, int R>
__global__ __launch_bounds__(NW * 64) void k_sweep_fused(const double *__restrict__ uin,
                                                         double *__restrict__ uout,
                                                         const double *__restrict__ F, int n,
                                                         int zc, int tiles_x, int tiles_y,
                                                         int nblocks, double s, double s4,
                                                         double hk,
                                                         unsigned long long *__restrict__ ncount)
{
    constexpr int NT = NW * 64;
    constexpr int W = TX + 2 * HALO;
    constexpr int HW = W / 2;
    constexpr int RPW = 64 / HW;
    constexpr int HH = TY + 2 * HALO, PL = W * HH;
    constexpr int KU = (PL + NT - 1) / NT;
    static_assert(W == 64 || W == 128, "row width must be 64 or 128");
    static_assert(TX / 2 + 3 <= HW, "a phase row must fit one lane group");
    static_assert(NW * RPW * R >= TY / 2 + 3, "too few rows per phase covered");
    __shared__ double su[NSLOT * PL];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int col = lane % HW, rbase = wave * RPW + lane / HW;
    const int tile = tile_of_block(blockIdx.x, nblocks);
    const int tx = tile % tiles_x;
    const int rest = tile / tiles_x;
    const int ty = rest % tiles_y;
    const int tz = rest / tiles_y;
    const int x0 = 1 + tx * TX, y0 = 1 + ty * TY, z0 = 1 + tz * zc;
    const int x1 = min(x0 + TX, n), y1 = min(y0 + TY, n), z1 = min(z0 + zc, n);
    const int lx0 = x0 - HALO, ly0 = y0 - HALO;
    const long sy = n + 1, sz = sy * sy;
    const int pfirst = max(1, z0 - 3);
    const int plast = min(n - 1, z1 + 2);
    const int tlast = z1 + 2;

    double ureg[KU];
    auto load_plane = [&](int p) {
#pragma unroll
        for (int q = 0; q < KU; ++q) {
            const int e = tid + q * NT;
            double v = 0.0;
            if (e < PL) {
                const int ly = e / W, lx = e % W;
                const int gx = lx0 + lx, gy = ly0 + ly;
                if (gx >= 0 && gx <= n && gy >= 0 && gy <= n)
                    v = uin[gx + sy * gy + sz * p];
            }
            ureg[q] = v;
        }
    };
    auto store_plane = [&](int p) {
        double *dst = su + (p % NSLOT) * PL;
#pragma unroll
        for (int q = 0; q < KU; ++q) {
            const int e = tid + q * NT;
            if (e < PL) {
                const int ly = e / W, lx = e % W;
                dst[ly * W + (lx & 1) * HW + (lx >> 1)] = ureg[q];
            }
        }
    };
    auto geom = [&](int c, int p) {
        PhaseGeom g;
        g.nr = 0;
        g.ncol = 0;
        g.is = g.js = g.off0 = g.px = 0;
        const int ex = 3 - c;
        if (p < max(1, z0 - ex) || p > min(n - 1, z1 - 1 + ex))
            return g;
        const int xa = max(1, x0 - ex), xb = min(n - 1, x1 - 1 + ex);
        const int ya = max(1, y0 - ex), yb = min(n - 1, y1 - 1 + ex);
        const int c0 = c & 1, c1 = c >> 1;
        const int rp = (c0 + c1 + p) & 1, ip = (c0 + rp) & 1;
        g.js = ya + ((ya ^ rp) & 1);
        g.is = xa + ((xa ^ ip) & 1);
        g.nr = g.js <= yb ? (yb - g.js) / 2 + 1 : 0;
        g.ncol = g.is <= xb ? (xb - g.is) / 2 + 1 : 0;
        const int lxs = g.is - lx0;
        g.px = lxs & 1;
        g.off0 = (g.js - ly0) * W + g.px * HW + (lxs >> 1);
        return g;
    };
    // Right-hand side values of this lane's nodes at step t.
    auto load_F = [&](int t, double (&fb)[4][R]) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const PhaseGeom g = geom(c, t - c);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int r = rbase + k * NW * RPW;
                double v = 0.0;
                if (r < g.nr && col < g.ncol)
                    v = F[(g.is + 2 * col) + sy * (g.js + 2 * r) + sz * (t - c)];
                fb[c][k] = v;
            }
        }
    };

    load_plane(pfirst - 1);
    store_plane(pfirst - 1);
    load_plane(pfirst);
    store_plane(pfirst);
    load_plane(pfirst + 1);
    store_plane(pfirst + 1);
    double Fc[4][R], Fn[4][R];
    load_F(pfirst, Fc);
    __syncthreads();

    for (int t = pfirst; t <= tlast; ++t) {
        const bool more = t + 2 <= plast + 1;
        if (more)
            load_plane(t + 2);
        if (t + 1 <= tlast)
            load_F(t + 1, Fn);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int p = t - c;
            const PhaseGeom g = geom(c, p);
            if (g.nr > 0) {
                double *Cp = su + (p % NSLOT) * PL;
                const double *Dp = su + ((p - 1) % NSLOT) * PL;
                const double *Up = su + ((p + 1) % NSLOT) * PL;
                const int xp = g.px ? 1 - HW : HW;
                const int xm = g.px ? -HW : HW - 1;
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int r = rbase + k * NW * RPW;
                    if (r < g.nr && col < g.ncol) {
                        const int off = g.off0 + 2 * r * W + col;
                        double *C = Cp + off;
                        if (OP == OP_MA) {
                            const Hess h = hessian3(Dp + off, C, Up + off, xp, xm, W, s, s4);
                            bool nc = false;
                            C[0] = ma_point_update(h, C[0], Fc[c][k], hk, nc);
                            // halo recomputations are not counted: only the
                            // tile's own nodes
                            if (nc && ncount) {
                                const int i = g.is + 2 * col, j = g.js + 2 * r;
                                if (i >= x0 && i < x1 && j >= y0 && j < y1 && p >= z0 && p < z1)
                                    atomicAdd(ncount, 1ull);
                            }
                        } else {
                            const double lap = laplacian3(Dp + off, C, Up + off, xp, xm, W, s);
                            C[0] = lap_point_update(lap, C[0], Fc[c][k], hk);
                        }
                    }
                }
            }
            __syncthreads();
        }
        const int pw = t - 3;
        if (pw >= z0 && pw <= z1 - 1) {
            const double *src = su + (pw % NSLOT) * PL;
            for (int e = tid; e < TX * TY; e += NT) {
                const int jj = e / TX, ii = e - jj * TX;
                const int i = x0 + ii, j = y0 + jj;
                const int lx = ii + HALO;
                if (i <= x1 - 1 && j <= y1 - 1)
                    uout[i + sy * j + sz * pw] = src[(jj + HALO) * W + (lx & 1) * HW + (lx >> 1)];
            }
        }
        if (more)
            store_plane(t + 2);
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int k = 0; k < R; ++k)
                Fc[c][k] = Fn[c][k];
    }
}

struct Cfg {
    int tx, ty, nw, r;
};
// Tile shapes the fused sweep is built for (index = tile_config - 1).
constexpr Cfg kCfgs[] = {{120, 14, 10, 1}, {120, 10, 8, 1}, {120, 18, 6, 2},
                         {56, 16, 6, 1},   {56, 8, 4, 1},   {120, 6, 6, 1}};
constexpr int kNumCfgs = int(sizeof(kCfgs) / sizeof(kCfgs[0]));

template <int OP, int TX, int TY, int NW, int R>
hipError_t launch_cfg(hipStream_t st, int n, int zc, const double *uin, double *uout,
                      const double *F, unsigned long long *nc)
{
    const int tiles_x = (n - 1 + TX - 1) / TX, tiles_y = (n - 1 + TY - 1) / TY;
    const int tiles_z = (n - 1 + zc - 1) / zc;
    const int nb = tiles_x * tiles_y * tiles_z;
    const double s = double(n) * double(n), s4 = 0.25 * s;
    const double hk = OP == OP_MA ? 0.5 / s : 1.0 / (6.0 * s);
    hipLaunchKernelGGL((k_sweep_fused<OP, TX, TY, NW, R>), dim3(nb), dim3(NW * 64), 0, st, uin,
                       uout, F, n, zc, tiles_x, tiles_y, nb, s, s4, hk, nc);
    return hipGetLastError();
}

template <int OP>
hipError_t launch_op(int cfg, hipStream_t st, int n, int zc, const double *uin, double *uout,
                     const double *F, unsigned long long *nc)
{
    switch (cfg) {
    case 0:
        return launch_cfg<OP, 120, 14, 10, 1>(st, n, zc, uin, uout, F, nc);
    case 1:
        return launch_cfg<OP, 120, 10, 8, 1>(st, n, zc, uin, uout, F, nc);
    case 2:
        return launch_cfg<OP, 120, 18, 6, 2>(st, n, zc, uin, uout, F, nc);
    case 3:
        return launch_cfg<OP, 56, 16, 6, 1>(st, n, zc, uin, uout, F, nc);
    case 4:
        return launch_cfg<OP, 56, 8, 4, 1>(st, n, zc, uin, uout, F, nc);
    case 5:
        return launch_cfg<OP, 120, 6, 6, 1>(st, n, zc, uin, uout, F, nc);
    default:
        return hipErrorInvalidValue;
    }
}

} // namespace

int fused_num_configs() { return kNumCfgs; }

// Automatic choice: the widest tiles that still give every CU work, and
// z-chunks of at least 16 planes.
void fused_pick(int n, int *cfg, int *zc)
{
    const int c = (n >= 160) ? 0 : 3;
    const int tiles_xy = ((n - 1 + kCfgs[c].tx - 1) / kCfgs[c].tx) *
                         ((n - 1 + kCfgs[c].ty - 1) / kCfgs[c].ty);
    int chunks = (512 + tiles_xy - 1) / tiles_xy;
    const int max_chunks = (n - 1 + 15) / 16;
    if (chunks > max_chunks)
        chunks = max_chunks;
    if (chunks < 1)
        chunks = 1;
    *cfg = c;
    *zc = (n - 1 + chunks - 1) / chunks;
}

// The automatic smoother choice: the per-colour kernel with XCD-contiguous
// rows measured faster than this kernel at every grid size on MI355X (the
// fused sweep spends its time on halo recomputation and idle lanes, not on
// bytes), so it runs only when selected explicitly.
bool fused_supported(int) { return false; }

hipError_t launch_sweep_fused(hipStream_t st, int op, int n, const double *u_in, double *u_out,
                              const double *F, unsigned long long *nonconvex, int cfg, int zc)
{
    if (n < 4)
        return hipErrorInvalidValue;
    if (cfg < 0 || cfg >= kNumCfgs || zc < 1) {
        int c2, z2;
        fused_pick(n, &c2, &z2);
        if (cfg < 0 || cfg >= kNumCfgs)
            cfg = c2;
        if (zc < 1)
            zc = z2;
    }
    if (zc > n - 1)
        zc = n - 1;
    if (op == OP_MA)
        return launch_op<OP_MA>(cfg, st, n, zc, u_in, u_out, F, nonconvex);
    return launch_op<OP_LAP>(cfg, st, n, zc, u_in, u_out, F, nonconvex);
}

} // namespace mafas
