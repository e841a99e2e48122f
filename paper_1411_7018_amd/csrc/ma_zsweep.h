// One complete 4-colour nonlinear Gauss-Seidel sweep per launch for large
// grids, streamed along z: the z-stream sweep (Section 2: the pointwise
// update of eqs. 2.7-2.9 applied colour by colour).
//
// The colour-phase kernels re-read the whole grid once per colour, since
// the 19-point stencil of a node touches all three other colours; a sweep
// then moves about twice its algorithmic bytes.  Here every node is read
// and written once per sweep:
//
// * A workgroup owns a TX x TY column of output nodes and a chunk of planes
//   [z0, z1).  It walks the chunk plane by plane with the colour phases
//   skewed two planes apart: at step s it applies colour c to plane
//   s - 2c, c = 0..3.  A colour-c node at plane P reads planes P-1..P+1;
//   colour c-1 has finished those planes at earlier steps, colours above c
//   reach them only at later steps, and the four updates of one step are at
//   least two planes apart, so they are independent.  One workgroup
//   barrier per step.
// * The planes live in an LDS ring of 10 planes (9 are read at a step, one
//   is being filled), each with a halo of 4 nodes in x and y, rows
//   de-interleaved by x parity so a colour's nodes in a row are contiguous.
//   The loads of plane s+4 are issued at the start of step s and written to
//   LDS at the end of step s+2; a step is short next to the latency of HBM,
//   and with loads one step ahead the walk waited on memory every step.
// * Neighbouring columns update the same grid at the same time, so colour c
//   is applied to the column grown by 3 - c nodes in x and y, and to the
//   chunk grown by 3 - c planes in z: the recomputed halo needs only old
//   values, which the sweep reads from u_in and never modifies (it writes
//   u_out: out of place).
// * Plane q is final after step q + 6 and is written to u_out at step
//   q + 7 (owned nodes and the Dirichlet layer next to them).
//
// Each node's update is the same expression (hessian3 and the root rule of
// ma_device.h) on the same values as in the colour-phase kernels, so the
// result is bitwise identical to four colour phases.  Algorithmic bytes
// per interior node and sweep: read u 8, read F 8, write u 8.
//
// The first sweep after a coarse-grid correction can also prolong it (PRO):
// u_in then holds u before the correction, and each interior value is
// corrected as it enters the ring by the trilinear interpolation of the
// coarse e = u_H - w_H (Algorithm 1's correction step), summed in the order
// of the prolongation kernels, so u_in + P e is bitwise the prolonged u they
// write.  The coarse e of the column's footprint goes through a second LDS
// ring of four coarse planes: coarse plane K is loaded at step 2K - 6,
// written to the ring at step 2K - 4 and read by the fine planes 2K - 1 ..
// 2K + 1 as they enter the fine ring at steps 2K - 3 .. 2K - 1.  The
// separate prolongation pass (read and write u once more) goes away; the
// fused sweep reads 16 bytes more per coarse node.
#pragma once

#include "ma_fsweep.h"

#include <type_traits>

namespace mafas {

template <int TX, int TY>
struct ZsShape {
    static constexpr int H = 4;              // halo loaded around the column
    static constexpr int LX = TX + 2 * H;    // LDS row length
    static constexpr int LY = TY + 2 * H;    // LDS rows per plane
    static constexpr int HW = LX / 2;        // one parity half of a row
    static constexpr int PL = LX * LY;       // doubles per plane
    static constexpr int R = 10;             // planes in the ring
    static constexpr int NL = PL * R;        // doubles in LDS
    // colour c covers TX/2 + e columns and TY/2 + e rows of its colour's
    // nodes in a plane, e = 3 - c
    static constexpr int ncol(int c) { return TX / 2 + 3 - c; }
    static constexpr int nrow(int c) { return TY / 2 + 3 - c; }
    static constexpr int count(int c) { return ncol(c) * nrow(c); }
    // Update items.  When every colour can start on a whole wavefront
    // within 1024 items (pure), each wavefront updates one colour and the
    // colour is uniform across it; else colours 0 and 1, then colours 2 and
    // 3 from the next whole wavefront on.  A colour-c node at plane P has x
    // parity (c >> 1) + P mod 2 and P has the step's parity, so the x parity
    // -- and with it the LDS offsets of the x neighbours -- is the same
    // across every wavefront either way.
    static constexpr int pad64(int x) { return (x + 63) / 64 * 64; }
    static constexpr bool pure = pad64(count(0)) + pad64(count(1)) + pad64(count(2)) + count(3) <= 1024;
    static constexpr int first(int c)
    {
        return pure ? (c == 0 ? 0
                       : c == 1 ? pad64(count(0))
                       : c == 2 ? pad64(count(0)) + pad64(count(1))
                                : pad64(count(0)) + pad64(count(1)) + pad64(count(2)))
               : c == 0 ? 0
               : c == 1 ? count(0)
               : c == 2 ? pad64(count(0) + count(1))
                        : pad64(count(0) + count(1)) + count(2);
    }
    static constexpr int items = first(3) + count(3);
    static constexpr size_t lds_bytes() { return size_t(NL) * sizeof(double); }
    // coarse-correction ring of a prolonging sweep: the footprint's first
    // x is odd (1 + tx TX - H), so its coarse nodes span LX / 2 + 2 columns
    // and LY / 2 + 2 rows
    static constexpr int CX = LX / 2 + 2, CY = LY / 2 + 2, CPL = CX * CY, CR = 4;
    static constexpr int NLP = NL + CR * CPL;
    static_assert(TX % 2 == 0 && TY % 2 == 0, "TX and TY must be even");
};

// Planes per chunk of an n grid cut into `chunks` chunks.
__host__ __device__ inline int zs_chunk(int n, int chunks)
{
    return (n - 1 + chunks - 1) / chunks;
}

// Column `tile` of grid G by a workgroup of NT threads; su: LDS.  The
// plane loads and stores go through raw buffer accesses (buf_rsrc), one
// resource per plane, byte offsets inside a plane in registers.  Grids up
// to n = 1289 (element offsets of the coarse loads are 32-bit).
template <int OP, int TX, int TY, int NT, bool PRO>
__device__ __forceinline__ void zsweep_tile(const FsGrid &G, int tile, double *__restrict__ su,
                                            unsigned long long *__restrict__ ncount)
{
    using S = ZsShape<TX, TY>;
    constexpr int LX = S::LX, HW = S::HW, PL = S::PL, H = S::H, R = S::R;
    constexpr int KL = (PL + NT - 1) / NT;        // plane elements per thread
    constexpr int MI = (S::items + NT - 1) / NT;  // update items per thread and step
    constexpr int SX = TX + 2, SY = TY + 2;       // store bound (with Dirichlet layer)
    constexpr int KS = (SX * SY + NT - 1) / NT;

    const int n = G.n;
    const int tid = int(threadIdx.x);
    const int tx = tile % G.tiles_x;
    const int rest = tile / G.tiles_x;
    const int ty = rest % G.tiles_y;
    const int tz = rest / G.tiles_y;
    const int zc = zs_chunk(n, G.tiles_z);
    const int x0 = 1 + tx * TX, y0 = 1 + ty * TY, z0 = 1 + tz * zc;
    if (z0 > n - 1)
        return;
    const int x1 = min(x0 + TX, n), y1 = min(y0 + TY, n), z1 = min(z0 + zc, n);
    const int lx0 = x0 - H, ly0 = y0 - H;
    const int sy = n + 1, sz = sy * sy;

    // ---- this thread's share of a plane load: global offset inside the
    // plane (-1: outside the grid, LDS gets 0) and LDS offset inside a slot
    unsigned gofs[KL];
    int lofs[KL];
#pragma unroll
    for (int k = 0; k < KL; ++k) {
        const int el = tid + k * NT;
        const int ly = el / LX, lx = el - (el / LX) * LX;
        const int gx = lx0 + lx, gy = ly0 + ly;
        const bool in = el < PL && gx >= 0 && gx <= n && gy >= 0 && gy <= n;
        gofs[k] = in ? unsigned(gx + sy * gy) * 8u : kBufOob;
        lofs[k] = el < PL ? ly * LX + (lx & 1) * HW + (lx >> 1) : -1;
    }
    const unsigned plane_bytes = unsigned(sz) * 8u;
    auto slot = [&](int p) { return ((p + 2 * R) % R) * PL; };   // p >= -2R
    // planes outside the grid read 0 through an empty resource
    auto fetch_plane = [&](int p, double *v) {
        const bool pin = p >= 0 && p <= n;
        const auto r = buf_rsrc(G.uin + (pin ? size_t(sz) * p : 0), pin ? plane_bytes : 0u);
#pragma unroll
        for (int k = 0; k < KL; ++k)
            v[k] = buf_load(r, gofs[k]);
    };

    // ---- prolongation (PRO): the coarse ring after the fine one.  This
    // thread's share of a coarse plane (coarse offset inside the plane, -1:
    // outside the coarse grid) and, for each of its plane elements, the
    // ring offset of the coarse node below it and its parities (bit 2: the
    // element is an interior node in x and y).
    constexpr int CX = S::CX, CPL = S::CPL, CR = S::CR;
    constexpr int KC = PRO ? (CPL + NT - 1) / NT : 1;
    const int nch = n / 2, ccy = nch + 1, ccz = ccy * ccy;
    const int cxa = (lx0 - 1) / 2, cya = (ly0 - 1) / 2;   // lx0, ly0 are odd
    double *cr = su + S::NL;
    int cgofs[KC], fco[KL], fpar[KL];
    if (PRO) {
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const int el = tid + k * NT;
            const int cyy = el / CX, cxx = el - (el / CX) * CX;
            const int X = cxa + cxx, Y = cya + cyy;
            cgofs[k] = el < CPL && X >= 0 && X <= nch && Y >= 0 && Y <= nch ? X + ccy * Y : -1;
        }
#pragma unroll
        for (int k = 0; k < KL; ++k) {
            const int el = tid + k * NT;
            const int ly = el / LX, lx = el - (el / LX) * LX;
            const int gx = lx0 + lx, gy = ly0 + ly;
            const bool inxy = el < PL && gx >= 1 && gx <= n - 1 && gy >= 1 && gy <= n - 1;
            fco[k] = inxy ? ((gy >> 1) - cya) * CX + ((gx >> 1) - cxa) : 0;
            fpar[k] = inxy ? 4 | (gx & 1) | ((gy & 1) << 1) : 0;
        }
    }
    const auto gcu = to_global(G.cu);
    const auto gcw = to_global(G.cw);
    // The loads land in a and b as they are; put_coarse masks the nodes
    // outside the coarse grid (a select right after the load would make the
    // step wait for every load in flight).
    auto fetch_coarse = [&](int K, double *a, double *b) {
        const bool kin = K >= 0 && K <= nch;
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const int q = kin && cgofs[k] >= 0 ? cgofs[k] + ccz * K : 0;
            a[k] = gcu[q];
            b[k] = gcw[q];
        }
    };
    auto put_coarse = [&](int K, const double *a, const double *b) {
        const bool kin = K >= 0 && K <= nch;
        double *c = cr + (K & (CR - 1)) * CPL;
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const int el = tid + k * NT;
            if (el < CPL)
                c[el] = kin && cgofs[k] >= 0 ? a[k] - b[k] : 0.0;
        }
    };
    // v += P e for the elements of plane p (PRO, interior planes), read
    // straight from the coarse ring: the planes the prologue loads.  Element
    // k's coarse nodes below it are (X, Y), (X + 1, Y), (X, Y + 1),
    // (X + 1, Y + 1) of coarse plane p >> 1 and, for odd p, of the next; a
    // node sums those its parities select (x odd: X + 1 too, y odd: Y + 1
    // too) in the prolongation kernels' order -- coarse plane, row, column
    // -- from d = 0.
    auto correct_flat = [&](int p, double *v) {
        if (!(PRO && p >= 1 && p <= n - 1))
            return;
        const int ok = p & 1;
        const double *E0 = cr + ((p >> 1) & (CR - 1)) * CPL;
        const double *E1 = cr + (((p >> 1) + 1) & (CR - 1)) * CPL;
#pragma unroll
        for (int k = 0; k < KL; ++k) {
            if (!(fpar[k] & 4))
                continue;
            const int oi = fpar[k] & 1, oj = (fpar[k] >> 1) & 1;
            const double wi = oi ? 0.5 : 1.0, wj = oj ? 0.5 : 1.0;
            const double wk = ok ? 0.5 : 1.0;
            const double w = wk * wj * wi;
            double d = 0.0;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (c == 1 && !ok)
                    break;
                const double *a = (c ? E1 : E0) + fco[k];
                d += w * a[0];
                if (oi)
                    d += w * a[1];
                if (oj) {
                    d += w * a[CX];
                    if (oi)
                        d += w * a[CX + 1];
                }
            }
            v[k] += d;
        }
    };
    // The walk's planes from partial sums kept per element.  With
    // B_K = 0 + (wj wi e) over the selected nodes of coarse plane K (in the
    // order above), an even plane 2K is corrected by B_K, and an odd plane
    // 2K + 1 by (B_K + the terms of plane K + 1) / 2: the weights are powers
    // of two, so halving commutes with every rounding of the sum and both
    // equal the prolongation kernels' sums bitwise.  Odd steps read coarse
    // plane K = (s + 3) / 2 once per element for both B_K and the sum.
    double Bp[KL];
    auto bsum = [&](const double *a, int k, double start, double &b, double &sm) {
        const int oi = fpar[k] & 1, oj = (fpar[k] >> 1) & 1;
        const double wi = oi ? 0.5 : 1.0, wj = oj ? 0.5 : 1.0;
        const double w2 = wj * wi;
        const double t0 = a[0], t1 = a[1], t2 = a[CX], t3 = a[CX + 1];
        b = 0.0;
        sm = start;
        b += w2 * t0;
        sm += w2 * t0;
        if (oi) {
            b += w2 * t1;
            sm += w2 * t1;
        }
        if (oj) {
            b += w2 * t2;
            sm += w2 * t2;
            if (oi) {
                b += w2 * t3;
                sm += w2 * t3;
            }
        }
    };
    auto correct_step = [&](int s, double *v) {
        const int p = s + 2;
        const bool pin = p >= 1 && p <= n - 1;
        if (s & 1) {
            const double *E = cr + (((s + 3) >> 1) & (CR - 1)) * CPL;
#pragma unroll
            for (int k = 0; k < KL; ++k) {
                if (!(fpar[k] & 4))
                    continue;
                double b, sm;
                bsum(E + fco[k], k, Bp[k], b, sm);
                if (pin)
                    v[k] += 0.5 * sm;
                Bp[k] = b;
            }
        } else if (pin) {
#pragma unroll
            for (int k = 0; k < KL; ++k)
                if (fpar[k] & 4)
                    v[k] += Bp[k];
        }
    };
    // plane elements into ring slot offset so (a multiple of PL)
    auto put_plane = [&](int so, const double *v) {
        double *b = su + so;
#pragma unroll
        for (int k = 0; k < KL; ++k)
            if (lofs[k] >= 0)
                b[lofs[k]] = v[k];
    };

    // ---- this thread's update items, fixed for the whole walk: colour
    // (-1: none), the planes its colour covers, and for each parity of the
    // step the node's offsets inside a plane (LDS and global), whether it
    // lies in the grid interior and whether this column owns it.
    int ic[MI], plo[MI], phi[MI], lio[MI][2];
    unsigned gio[MI][2];
    bool okxy[MI][2], own[MI][2];
#pragma unroll
    for (int m = 0; m < MI; ++m) {
        const int q = tid + m * NT;
        int c = -1;
        if (q < S::first(0) + S::count(0))
            c = 0;
        else if (q >= S::first(1) && q < S::first(1) + S::count(1))
            c = 1;
        else if (q >= S::first(2) && q < S::first(2) + S::count(2))
            c = 2;
        else if (q >= S::first(3) && q < S::first(3) + S::count(3))
            c = 3;
        const int cc = c < 0 ? 0 : c;
        const int local = q - (cc == 0 ? S::first(0) : cc == 1 ? S::first(1)
                               : cc == 2 ? S::first(2) : S::first(3));
        const int e = 3 - cc, c0 = cc & 1, c1 = cc >> 1;
        const int nc = TX / 2 + e;
        const int r = local / nc, col = local - (local / nc) * nc;
        const int xa = x0 - e, ya = y0 - e;
        ic[m] = c;
        plo[m] = max(1, z0 - e);
        phi[m] = min(n - 1, z1 - 1 + e);
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
            // P = s - 2c has the parity sp of the step
            const int i = xa + ((xa + c1 + sp) & 1) + 2 * col;
            const int j = ya + ((ya + c1 + sp + c0) & 1) + 2 * r;
            const int lx = i - lx0;
            lio[m][sp] = (j - ly0) * LX + (lx & 1) * HW + (lx >> 1);
            // byte offset of the node in plane P = s - 2c from plane s - 6
            gio[m][sp] = unsigned(i + sy * j + (6 - 2 * cc) * sz) * 8u;
            okxy[m][sp] = c >= 0 && i >= max(1, xa) && i <= min(n - 1, x1 - 1 + e) &&
                          j >= max(1, ya) && j <= min(n - 1, y1 - 1 + e);
            own[m][sp] = i >= x0 && i < x1 && j >= y0 && j < y1;
        }
    }
    // nonconvex updates of owned nodes (added to ncount after the walk)
    unsigned nown = 0;
    // item m has a node at step s (sp = s & 1, P = s - 2c)
    auto active = [&](int m, int sp, int P) {
        return okxy[m][sp] && P >= plo[m] && P <= phi[m];
    };
    // right-hand sides of the items at step s: one resource based at plane
    // s - 6 (it may start below the grid; every offset read lands on the
    // item's own plane P = s - 2c >= 1), inactive items read 0
    auto fetch_f = [&](int s, double *f) {
        const int sp = s & 1;
        const auto r = buf_rsrc(reinterpret_cast<const double *>(
                                   reinterpret_cast<uintptr_t>(G.F) + (long(s) - 6) * long(plane_bytes)),
                               7u * plane_bytes);
#pragma unroll
        for (int m = 0; m < MI; ++m) {
            // one colour per wavefront (pure): its plane and range are scalars
            const int c = S::pure ? __builtin_amdgcn_readfirstlane(ic[m]) : ic[m];
            const int P = s - 2 * c;
            const bool ok = S::pure ? okxy[m][sp] && P >= max(1, z0 - 3 + c) &&
                                          P <= min(n - 1, z1 + 2 - c)
                                    : active(m, sp, P);
            f[m] = buf_load(r, ok ? gio[m][sp] : kBufOob);
        }
    };

    // ---- the update of item m at step s, right-hand side f.  The x
    // parity of the node is uniform across the wavefront, so the branch on
    // it is too, and each side reads its neighbours at constant offsets.
    auto update = [&](int m, int s, int rs, double f) {
        const int sp = s & 1;
        // one colour per wavefront (pure): read it from the first lane, so
        // the plane, its range and the ring slots below are scalars (the
        // items past a colour's count, c = -1, are never active)
        const int c = S::pure ? __builtin_amdgcn_readfirstlane(ic[m]) : ic[m];
        const int P = s - 2 * c;
        const bool in_planes = S::pure ? P >= max(1, z0 - 3 + c) && P <= min(n - 1, z1 + 2 - c)
                                       : P >= plo[m] && P <= phi[m];
        if (!(okxy[m][sp] && in_planes))
            return;
        const int io = lio[m][sp];
        // ring slots of planes P, P - 1, P + 1 from the step's slot rs =
        // s mod R: P = s - 2c with 0 <= 2c <= 6 wraps at most once
        int b = rs - 2 * c;
        b += b < 0 ? R : 0;
        const int bm = b == 0 ? R - 1 : b - 1;
        const int bp = b == R - 1 ? 0 : b + 1;
        double *C = su + b * PL + io;
        const double *D = su + bm * PL + io;
        const double *U = su + bp * PL + io;
        auto apply = [&](auto parity) {
            constexpr int odd = decltype(parity)::value;
            constexpr int xp = odd ? 1 - HW : HW;
            constexpr int xm = odd ? -HW : HW - 1;
            if (OP == OP_MA) {
                const Hess h = hessian3(D, C, U, xp, xm, LX, G.s, G.s4);
                bool nc = false;
                C[0] = ma_point_update(h, C[0], f, G.hk, nc);
                // recomputed halo nodes are counted by their own column / chunk
                if (nc)
                    nown += own[m][sp] && P >= z0 && P < z1;
            } else {
                const double lap = laplacian3(D, C, U, xp, xm, LX, G.s);
                C[0] = lap_point_update(lap, C[0], f, G.hk);
            }
        };
        // colours 0 and 1 (2 and 3) share wavefronts and c >> 1, so the
        // parity is the same on every active lane.  For the Monge-Ampere
        // update it is read from the first active lane, which makes the
        // branch a scalar branch instead of two exec-masked paths; the short
        // Poisson update runs faster without the read.
        int odd = ((c >> 1) + sp - lx0) & 1;
        if (OP == OP_MA)
            odd = __builtin_amdgcn_readfirstlane(odd);
        if (odd)
            apply(std::integral_constant<int, 1>{});
        else
            apply(std::integral_constant<int, 0>{});
    };

    // ---- write plane q (owned nodes and the Dirichlet layer beside them)
    const int xs0 = x0 == 1 ? 0 : x0, xs1 = x1 == n ? n + 1 : x1;
    const int ys0 = y0 == 1 ? 0 : y0, ys1 = y1 == n ? n + 1 : y1;
    // this thread's share of a stored plane: byte offset in the grid plane
    // (kBufOob: none) and LDS offset in a slot
    unsigned sofs[KS];
    int sl[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int el = tid + k * NT;
        const int bb = el / SX, a = el - (el / SX) * SX;
        const int gx = xs0 + a, gy = ys0 + bb;
        const bool in = el < SX * SY && gx < xs1 && gy < ys1;
        const int lx = gx - lx0;
        sofs[k] = in ? unsigned(gx + sy * gy) * 8u : kBufOob;
        sl[k] = in ? (gy - ly0) * LX + (lx & 1) * HW + (lx >> 1) : 0;
    }
    auto store_plane = [&](int q, int so) {
        const double *b = su + so;
        const auto r = buf_rsrc(G.uout + size_t(sz) * q, plane_bytes);
#pragma unroll
        for (int k = 0; k < KS; ++k)
            buf_store(r, sofs[k], b[sl[k]]);
    };

    // ---- the walk.  Steps S0..S1 update; plane q is stored at step q + 7.
    // Loads run three steps ahead: the plane written to LDS at the end of
    // step s (s + 2) and the right-hand sides used at step s were issued at
    // step s - 2, so each step's loads have two steps to arrive.
    const int S0 = max(1, z0 - 3);
    const int S1 = min(n - 1, z1 - 1) + 6;
    // Coarse planes (PRO): the even steps s >= sw0 write plane s / 2 + 2
    // (loaded two steps earlier) and load the next one; the planes the
    // prologue's fine planes and the first steps' fine planes read go into
    // the ring here, before them.
    const int sw0 = S0 + (S0 & 1);
    double ca[KC], cb[KC];
    if (PRO) {
        for (int K = (S0 - 1) >> 1; K <= sw0 / 2 + 1; ++K) {
            fetch_coarse(K, ca, cb);
            put_coarse(K, ca, cb);
        }
        lds_barrier();
        fetch_coarse(sw0 / 2 + 2, ca, cb);
        // B of the coarse plane below the first step's even plane
        const double *E = cr + (((S0 + 2) >> 1) & (CR - 1)) * CPL;
#pragma unroll
        for (int k = 0; k < KL; ++k) {
            double sm;
            Bp[k] = 0.0;
            if (fpar[k] & 4)
                bsum(E + fco[k], k, 0.0, Bp[k], sm);
        }
    }
    {
        double v[KL];
        for (int p = S0 - 1; p <= S0 + 1; ++p) {
            fetch_plane(p, v);
            correct_flat(p, v);
            put_plane(slot(p), v);
        }
    }
    double p0[KL], p1[KL], p2[KL];   // plane prefetch buffers (rotate by step)
    double f0[MI], f1[MI], f2[MI];   // right-hand sides of the next steps' items
    fetch_plane(S0 + 2, p1);
    fetch_plane(S0 + 3, p2);
    fetch_f(S0, f0);
    fetch_f(S0 + 1, f1);
    lds_barrier();
    // the Dirichlet planes travel with the chunk next to them
    if (z0 == 1)
        store_plane(0, slot(0));

    // one step: issue the loads of plane s+4 into pn and of the right-hand
    // sides of step s+2 into fn, (PRO) correct plane s+2, store plane s-7,
    // update with fc, then write plane s+2 (loaded two steps earlier into
    // pw) to LDS
    auto step = [&](int s, double *pn, double *pw, double *fc, double *fn) {
        fetch_plane(s + 4, pn);
        fetch_f(s + 2, fn);
        // the correction of plane s + 2 (its coarse planes are in the ring
        // since earlier steps) ahead of the updates, whose work hides the
        // latency of its reads
        if (PRO)
            correct_step(s, pw);
        // ring slot offsets of planes s + d from s mod R (uniform)
        const int rs = s % R;
        auto rslot = [&](int d) {
            int x = rs + d;
            x += x < 0 ? R : 0;
            x -= x >= R ? R : 0;
            return x * PL;
        };
        const int q = s - 7;
        if (q >= z0 && q < z1) {
            store_plane(q, rslot(-7));
            if (q == n - 1)
                store_plane(n, rslot(-6));
        }
        if (s <= S1) {
#pragma unroll
            for (int m = 0; m < MI; ++m)
                update(m, s, rs, fc[m]);
        }
        put_plane(rslot(2), pw);
        if (PRO && !(s & 1)) {
            // plane s / 2 + 2 into a slot this step's fine plane does not read
            put_coarse(s / 2 + 2, ca, cb);
            fetch_coarse(s / 2 + 3, ca, cb);
        }
        lds_barrier();
    };
    for (int s = S0; s <= S1 + 1; s += 3) {
        step(s, p0, p1, f0, f2);
        if (s + 1 > S1 + 1)
            break;
        step(s + 1, p1, p2, f1, f0);
        if (s + 2 > S1 + 1)
            break;
        step(s + 2, p2, p0, f2, f1);
    }
    if (OP == OP_MA && ncount && nown)
        atomicAdd(ncount + G.slot, (unsigned long long)nown);
}

// Blocks are dispatched round-robin over the 8 XCDs; tile_of_block gives
// each XCD a contiguous range of columns (x fastest, then y, then the z
// chunk), so columns that share halos share an L2.
template <int OP, int TX, int TY, int NT, bool PRO>
__global__ __launch_bounds__(NT) void k_zsweep(const FsList *__restrict__ L,
                                               unsigned long long *__restrict__ ncount)
{
    __shared__ double su[PRO ? ZsShape<TX, TY>::NLP : ZsShape<TX, TY>::NL];
    const int total = L->total;
    const int t = tile_of_block(int(blockIdx.x), int(gridDim.x));
    if (t >= total)
        return;
    const int ng = L->ngrids;
    int g = 0;
    while (g + 1 < ng && L->g[g + 1].start <= t)
        ++g;
    const FsGrid G = L->g[g];
    if ((L->stopped >> G.slot) & 1ull)
        return;
    zsweep_tile<OP, TX, TY, NT, PRO>(G, t - G.start, su, ncount);
}

template <int OP, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_zsweep1(FsGrid G, unsigned long long *__restrict__ ncount)
{
    __shared__ double su[ZsShape<TX, TY>::NL];
    const int t = tile_of_block(int(blockIdx.x), int(gridDim.x));
    zsweep_tile<OP, TX, TY, NT, false>(G, t, su, ncount);
}

} // namespace mafas
