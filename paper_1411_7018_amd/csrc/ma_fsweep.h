// One complete 4-colour nonlinear Gauss-Seidel sweep per launch (Section 2:
// the pointwise update of eqs. 2.7-2.9 applied colour by colour), for many
// grids at once: the block sweep.
//
// Colour c = ((i+j) mod 2) + 2 ((i+k) mod 2).  A colour-c node reads only
// nodes of the three other colours, so a sweep is four phases, each
// updating all nodes of one colour at once.  Launched phase by phase, a
// sweep costs four kernel launches, which on the smaller grids of the
// V-cycle take longer than the work itself.  The block sweep runs all four
// phases in one launch:
//
// * A workgroup owns a TX x TY x TZ block of output nodes.  It loads the
//   block with a halo of 4 nodes into LDS (rows de-interleaved by x parity,
//   so the nodes of one colour in a row are contiguous), and prefetches the
//   right-hand side of every node it will update into registers.
// * It applies phase c = 0..3 to the colour-c nodes of the block grown by
//   3 - c nodes in every direction, with a workgroup barrier after each
//   phase.  A phase-c value one node outside the grown block of phase c + 1
//   is never needed, so the grown blocks shrink by one node per phase; the
//   nodes outside the owned block are recomputed from the same values by
//   the neighbouring workgroups.
// * It writes the owned block (and the Dirichlet layer next to it) to
//   u_out.  The sweep reads u_in and writes u_out (out of place), so halos
//   read from a neighbouring block are never modified during the launch.
//
// The update of a node evaluates the same expressions (hessian3 and the root
// rule of ma_device.h) on the same values as the colour-phase kernels, so
// the results are bitwise identical to four colour phases.
//
// Algorithmic bytes per interior node and sweep: read u 8, read F 8,
// write u 8.  The recomputation costs ALU work, which on the grids this
// kernel is used for is cheaper than three extra launches.
#pragma once

#include "ma_device.h"
#include "ma_internal.h"

namespace mafas {

// One grid of a block-sweep launch.
struct FsGrid {
    const double *uin;
    double *uout;
    const double *F;
    int n;          // intervals per side
    int tiles_x, tiles_y, tiles_z;
    int start;      // first block of this grid in the launch
    int slot;       // counter slot of the solve
    double s, s4;   // 1/h^2, 1/(4h^2)
    double hk;      // h^2/2 (nonlinear update) or 1/(6s) (linear update)
    // z-stream sweeps that also prolong (the first sweep after the coarse
    // correction): the coarse level's u and w, whose difference is
    // interpolated onto u_in as it is read; null otherwise
    const double *cu, *cw;
};

constexpr int kFsMaxGrids = 64;

struct FsList {
    int ngrids;
    int total;      // blocks over all grids
    unsigned long long stopped;  // bit s: solve s has stopped, skip it
    FsGrid g[kFsMaxGrids];
};
constexpr size_t fs_list_bytes(int ngrids) { return 16 + sizeof(FsGrid) * size_t(ngrids); }
static_assert(offsetof(FsList, g) == 16, "list header is 16 bytes");

template <int TX, int TY, int TZ>
struct FsShape {
    static constexpr int H = 4;              // halo loaded around the block
    static constexpr int LX = TX + 2 * H;    // LDS row length
    static constexpr int LY = TY + 2 * H;    // LDS rows per plane
    static constexpr int LZ = TZ + 2 * H;    // LDS planes
    static constexpr int HW = LX / 2;        // one parity half of a row
    static constexpr int PL = LX * LY;       // doubles per plane
    static constexpr int NL = PL * LZ;       // doubles in LDS
    // phase c covers (TX/2 + e) columns, TY + 2e rows and (TZ/2 + e) planes
    // of its colour's sub-lattice, e = 3 - c
    static constexpr int ncol(int c) { return TX / 2 + 3 - c; }
    static constexpr int nrow(int c) { return TY + 2 * (3 - c); }
    static constexpr int npl(int c) { return TZ / 2 + 3 - c; }
    static constexpr int count(int c) { return ncol(c) * nrow(c) * npl(c); }
    static constexpr int SX = TX + 2, SY = TY + 2, SZ = TZ + 2;   // store bound
    static constexpr size_t lds_bytes() { return size_t(NL) * sizeof(double); }
    static_assert(TX % 2 == 0 && TZ % 2 == 0, "TX and TZ must be even");
};

// Workgroup barrier that orders LDS accesses only: global loads issued
// before it (the right-hand side prefetch) stay in flight across it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Block `tile` of grid G by a workgroup of NT threads; su: LDS.  Global
// offsets are 32-bit: grids up to n = 1289.
template <int OP, int TX, int TY, int TZ, int NT>
__device__ __forceinline__ void bsweep_tile(const FsGrid &G, int tile, double *__restrict__ su,
                                            unsigned long long *__restrict__ ncount)
{
    using S = FsShape<TX, TY, TZ>;
    constexpr int LX = S::LX, HW = S::HW, PL = S::PL, H = S::H;
    constexpr int M0 = (S::count(0) + NT - 1) / NT, M1 = (S::count(1) + NT - 1) / NT;
    constexpr int M2 = (S::count(2) + NT - 1) / NT, M3 = (S::count(3) + NT - 1) / NT;
    constexpr int KL = (S::NL + NT - 1) / NT;
    constexpr int KS = (S::SX * S::SY * S::SZ + NT - 1) / NT;

    const int n = G.n;
    const int tid = int(threadIdx.x);
    const int tx = tile % G.tiles_x;
    const int rest = tile / G.tiles_x;
    const int ty = rest % G.tiles_y;
    const int tz = rest / G.tiles_y;
    const int x0 = 1 + tx * TX, y0 = 1 + ty * TY, z0 = 1 + tz * TZ;
    const int x1 = min(x0 + TX, n), y1 = min(y0 + TY, n), z1 = min(z0 + TZ, n);
    const int lx0 = x0 - H, ly0 = y0 - H, lz0 = z0 - H;
    const int sy = n + 1, sz = sy * sy;
    const auto uin = to_global(G.uin);
    const auto uout = to_global(G.uout);
    const auto F = to_global(G.F);

    // Node of item m of phase c: rows j over the grown block, planes k and
    // columns i of the colour's parities (k = j + c0 + c1, i = j + c0 mod 2).
    // Returns false when the item lies outside the grid interior.
    auto node = [&](int c, int item, int &i, int &j, int &k) -> bool {
        const int e = 3 - c, c0 = c & 1, c1 = c >> 1;
        const int nc = TX / 2 + e, np = TZ / 2 + e;
        const int q = item % nc;
        const int r2 = item / nc;
        const int kk = r2 % np;
        const int jj = r2 / np;
        j = y0 - e + jj;
        const int pk = (j + c0 + c1) & 1, pi = (j + c0) & 1;
        k = (z0 - e) + (((z0 - e) ^ pk) & 1) + 2 * kk;
        i = (x0 - e) + (((x0 - e) ^ pi) & 1) + 2 * q;
        return item < S::count(c) && i >= max(1, x0 - e) && i <= min(n - 1, x1 - 1 + e) &&
               j >= max(1, y0 - e) && j <= min(n - 1, y1 - 1 + e) && k >= max(1, z0 - e) &&
               k <= min(n - 1, z1 - 1 + e);
    };
    auto lds_off = [&](int i, int j, int k) {
        const int lx = i - lx0;
        return (k - lz0) * PL + (j - ly0) * LX + (lx & 1) * HW + (lx >> 1);
    };

    // ---- right-hand sides of every item of this lane, in flight during
    // the block load (a lane without a node reads node 0 and discards it)
    double f0[M0], f1[M1], f2[M2], f3[M3];
    auto fetch = [&](int c, int m) {
        int i, j, k;
        const bool ok = node(c, tid + m * NT, i, j, k);
        return F[ok ? i + sy * j + sz * k : 0];
    };
#pragma unroll
    for (int m = 0; m < M0; ++m)
        f0[m] = fetch(0, m);
#pragma unroll
    for (int m = 0; m < M1; ++m)
        f1[m] = fetch(1, m);
#pragma unroll
    for (int m = 0; m < M2; ++m)
        f2[m] = fetch(2, m);
#pragma unroll
    for (int m = 0; m < M3; ++m)
        f3[m] = fetch(3, m);

    // ---- the block and its halo into LDS (0 outside the grid): every load
    // of the lane first, then the LDS writes, so all of them are in flight
    // together
    double lv[KL];
#pragma unroll
    for (int k = 0; k < KL; ++k) {
        const int el = tid + k * NT;
        const int lz = el / PL, rem = el - (el / PL) * PL;
        const int ly = rem / LX, lx = rem - (rem / LX) * LX;
        const int gx = lx0 + lx, gy = ly0 + ly, gz = lz0 + lz;
        const bool in = el < S::NL && gx >= 0 && gx <= n && gy >= 0 && gy <= n && gz >= 0 &&
                        gz <= n;
        const double v = uin[in ? gx + sy * gy + sz * gz : 0];
        lv[k] = in ? v : 0.0;
    }
#pragma unroll
    for (int k = 0; k < KL; ++k) {
        const int el = tid + k * NT;
        const int lz = el / PL, rem = el - (el / PL) * PL;
        const int ly = rem / LX, lx = rem - (rem / LX) * LX;
        if (el < S::NL)
            su[lz * PL + ly * LX + (lx & 1) * HW + (lx >> 1)] = lv[k];
    }
    lds_barrier();

    // ---- the four phases
    auto update = [&](int c, int m, double f) {
        int i, j, k;
        if (!node(c, tid + m * NT, i, j, k))
            return;
        const int off = lds_off(i, j, k);
        double *C = su + off;
        const double *D = C - PL;
        const double *U = C + PL;
        const int odd = (i - lx0) & 1;
        const int xp = odd ? 1 - HW : HW;
        const int xm = odd ? -HW : HW - 1;
        if (OP == OP_MA) {
            const Hess h = hessian3(D, C, U, xp, xm, LX, G.s, G.s4);
            bool nc = false;
            C[0] = ma_point_update(h, C[0], f, G.hk, nc);
            // recomputed halo nodes are counted by their own block
            if (nc && ncount && i >= x0 && i < x1 && j >= y0 && j < y1 && k >= z0 && k < z1)
                atomicAdd(ncount + G.slot, 1ull);
        } else {
            const double lap = laplacian3(D, C, U, xp, xm, LX, G.s);
            C[0] = lap_point_update(lap, C[0], f, G.hk);
        }
    };
#pragma unroll
    for (int m = 0; m < M0; ++m)
        update(0, m, f0[m]);
    lds_barrier();
#pragma unroll
    for (int m = 0; m < M1; ++m)
        update(1, m, f1[m]);
    lds_barrier();
#pragma unroll
    for (int m = 0; m < M2; ++m)
        update(2, m, f2[m]);
    lds_barrier();
#pragma unroll
    for (int m = 0; m < M3; ++m)
        update(3, m, f3[m]);
    lds_barrier();

    // ---- the owned block and the Dirichlet layer next to it to u_out
    const int xs0 = x0 == 1 ? 0 : x0, xs1 = x1 == n ? n + 1 : x1;
    const int ys0 = y0 == 1 ? 0 : y0, ys1 = y1 == n ? n + 1 : y1;
    const int zs0 = z0 == 1 ? 0 : z0, zs1 = z1 == n ? n + 1 : z1;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int el = tid + k * NT;
        const int c2 = el / (S::SX * S::SY), rem = el - c2 * (S::SX * S::SY);
        const int b = rem / S::SX, a = rem - b * S::SX;
        const int gx = xs0 + a, gy = ys0 + b, gz = zs0 + c2;
        if (el < S::SX * S::SY * S::SZ && gx < xs1 && gy < ys1 && gz < zs1)
            uout[gx + sy * gy + sz * gz] = su[lds_off(gx, gy, gz)];
    }
}

// Blocks are dispatched round-robin over the 8 XCDs; tile_of_block gives
// each XCD a contiguous range of tiles, so tiles that share halos share an
// L2.  One tile per workgroup.
template <int OP, int TX, int TY, int TZ, int NT>
__global__ __launch_bounds__(NT) void k_bsweep(const FsList *__restrict__ L,
                                                unsigned long long *__restrict__ ncount)
{
    __shared__ double su[FsShape<TX, TY, TZ>::NL];
    const int total = L->total;
    const int t = tile_of_block(int(blockIdx.x), int(gridDim.x));
    if (t >= total)
        return;
    const int ng = L->ngrids;
    int g = 0;
    while (g + 1 < ng && L->g[g + 1].start <= t)
        ++g;
    const FsGrid G = L->g[g];   // the whole descriptor in one set of loads
    if ((L->stopped >> G.slot) & 1ull)
        return;
    bsweep_tile<OP, TX, TY, TZ, NT>(G, t - G.start, su, ncount);
}

// The same for one grid passed by value (gridDim.x = its tile count).
template <int OP, int TX, int TY, int TZ, int NT>
__global__ __launch_bounds__(NT) void k_bsweep1(FsGrid G, unsigned long long *__restrict__ ncount)
{
    __shared__ double su[FsShape<TX, TY, TZ>::NL];
    const int t = tile_of_block(int(blockIdx.x), int(gridDim.x));
    bsweep_tile<OP, TX, TY, TZ, NT>(G, t, su, ncount);
}

} // namespace mafas
