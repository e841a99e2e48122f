// Device-side pointwise pieces of the nonlinear Gauss-Seidel smoother:
// discrete Hessian (eqs. 2.1-2.6), its determinant (the explicit operator of
// Section 1) and the smallest-real-root rule for the local cubic (eqs.
// 2.8-2.9, Theorems 2.1-2.2), in FP64.
#pragma once

#include <hip/hip_runtime.h>

namespace mafas {

// A pointer read from a device-side table is generic to the compiler, which
// then accesses it with FLAT instructions; those count against the LDS wait
// counter too, so waiting for an LDS access would also wait for every
// global load in flight.  Casting to the global address space gives
// global_load / global_store instead.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *to_global(T *p)
{
    return (__attribute__((address_space(1))) T *)(p);
}
// An untyped table entry as a global pointer to T.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gptr(void *p)
{
    return (__attribute__((address_space(1))) T *)(p);
}

// Raw buffer accesses.  A buffer resource carries a base address and a size
// in bytes; a byte offset at or beyond the size reads 0 and drops a write.
// Kernels that walk a grid plane by plane build one resource per plane,
// whose base (the plane's first node) is a scalar, keep each thread's byte
// offsets inside a plane in registers, and give a node outside the grid the
// offset kBufOob: no 64-bit address arithmetic, select or branch per access.
constexpr unsigned kBufOob = 0x80000000u;
constexpr int kBufRsrcFlags = 0x00020000;   // buffer resource word 3 (gfx9)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const double *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(base), (short)0, int(bytes),
                                             kBufRsrcFlags);
}

__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, int(off), 0, 0));
}

__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned off, double v)
{
    using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, int(off), 0, 0);
}

struct Hess {
    double xx, yy, zz, xy, xz, yz;
};

// Discrete Hessian at a node from three pointers at that node's position in
// the planes k-1 (D), k (C) and k+1 (U).  Inside a plane, C[xp] / C[xm] are
// the x+1 / x-1 neighbours and C[sy] / C[-sy] the y+1 / y-1 neighbours
// (xp = 1, xm = -1 for plain x-fastest storage; other values for layouts
// that de-interleave even and odd x).  s = 1/h^2, s4 = 1/(4h^2).  Second
// differences are taken as differences of first differences, exact
// (Sterbenz) when neighbouring values are close, which keeps round-off at
// the scale of the first differences instead of |u|.  Every smoother,
// residual and restriction kernel evaluates the Hessian through this one
// expression tree, so the same neighbour values give bitwise equal results.
template <typename T>
__device__ __forceinline__ Hess hessian3(const T *__restrict__ D, const T *__restrict__ C,
                                        const T *__restrict__ U, long xp, long xm, long sy,
                                        double s, double s4)
{
    const double c = C[0];
    Hess g;
    g.xx = ((double(C[xp]) - c) - (c - double(C[xm]))) * s;
    g.yy = ((double(C[sy]) - c) - (c - double(C[-sy]))) * s;
    g.zz = ((double(U[0]) - c) - (c - double(D[0]))) * s;
    g.xy = ((double(C[xp + sy]) - double(C[xm + sy])) - (double(C[xp - sy]) - double(C[xm - sy])))
           * s4;
    g.xz = ((double(U[xp]) - double(U[xm])) - (double(D[xp]) - double(D[xm]))) * s4;
    g.yz = ((double(U[sy]) - double(U[-sy])) - (double(D[sy]) - double(D[-sy]))) * s4;
    return g;
}

// Hessian at linear index p of an x-fastest array with strides (sx, sy, sz).
template <typename T>
__device__ __forceinline__ Hess hessian_at(const T *__restrict__ u, long p, long sx, long sy,
                                           long sz, double s, double s4)
{
    return hessian3(u + p - sz, u + p, u + p + sz, sx, -sx, sy, s, s4);
}

// 7-point Laplacian from differences of first differences (same pointer
// and offset convention as hessian3).
template <typename T>
__device__ __forceinline__ double laplacian3(const T *__restrict__ D, const T *__restrict__ C,
                                             const T *__restrict__ U, long xp, long xm, long sy,
                                             double s)
{
    const double c = C[0];
    return (((double(C[xp]) - c) - (c - double(C[xm])))
            + ((double(C[sy]) - c) - (c - double(C[-sy])))
            + ((double(U[0]) - c) - (c - double(D[0])))) * s;
}

template <typename T>
__device__ __forceinline__ double laplacian_at(const T *__restrict__ u, long p, long sx, long sy,
                                               long sz, double s)
{
    return laplacian3(u + p - sz, u + p, u + p + sz, sx, -sx, sy, s);
}

__device__ __forceinline__ double det3(const Hess &g)
{
    return g.xx * g.yy * g.zz + 2.0 * g.xy * g.yz * g.xz - g.xx * (g.yz * g.yz)
           - g.yy * (g.xz * g.xz) - g.zz * (g.xy * g.xy);
}

// det(G - sig I) - F and its derivative, from the shifted matrix.
__device__ __forceinline__ void shifted_cubic(const Hess &g, double F, double sig, double &q,
                                              double &dq)
{
    const double a = g.xx - sig, b = g.yy - sig, c = g.zz - sig;
    const double mab = a * b - g.xy * g.xy;
    const double mac = a * c - g.xz * g.xz;
    const double mbc = b * c - g.yz * g.yz;
    q = a * mbc - g.xy * (g.xy * c - g.yz * g.xz) + g.xz * (g.xy * g.yz - b * g.xz) - F;
    dq = -(mab + mac + mbc);
}

// General smallest real root of det(G - sig I) = F, used only off the
// convex branch (F <= 0, a Newton iteration that did not settle, or a
// non-finite result).  With m = tr G / 3 and
// y = sig - m the cubic is y^3 - P y + (F - det(G - m I)) = 0, P = tr(B^2)/2
// for the traceless B = G - m I.  Writing y = 2 t cos(phi), t = sqrt(P/3),
// gives cos(3 phi) = -(F - det B)/(2 t^3); the smallest of the three real
// roots takes phi = (acos(.) + 2 pi)/3.  With a single real root the
// hyperbolic form y = +-2 t cosh(acosh|.|/3) applies.  Two Newton steps on
// the shifted form then polish the result, each kept only if |q| drops.
//
// The closed form and the polishing steps are two out-of-line functions,
// each with few values live: a call counts its callee's registers against
// the calling kernel, and one body holding the Hessian across the
// transcendental functions would take more registers than the colour-sweep
// kernels may hold at eight waves per SIMD.
__device__ __noinline__ double general_start(Hess g, double F)
{
    const double m = (g.xx + g.yy + g.zz) * (1.0 / 3.0);
    const double a = g.xx - m, b = g.yy - m, c = g.zz - m;
    const double P = 0.5 * (a * a + b * b + c * c) + (g.xy * g.xy + g.xz * g.xz + g.yz * g.yz);
    const double D = a * (b * c - g.yz * g.yz) - g.xy * (g.xy * c - g.yz * g.xz)
                     + g.xz * (g.xy * g.yz - b * g.xz);
    const double Q = F - D;
    double y;
    if (P > 0.0) {
        const double t = sqrt(P * (1.0 / 3.0));
        const double arg = -0.5 * Q / (t * t * t);
        // F > 0 with a double smallest eigenvalue puts arg just below 1
        // (three real roots, the lower two close); rounding can push it past
        // 1, where the hyperbolic form would return the largest root, so a
        // rounding-sized excess is read as 1.
        const bool near_double = F > 0.0 && arg > 1.0 && arg <= 1.0 + 1e-10;
        if ((arg >= -1.0 && arg <= 1.0) || near_double) {
            y = 2.0 * t * cos((acos(fmin(arg, 1.0)) + 2.0 * M_PI) * (1.0 / 3.0));
        } else if (arg > 1.0) {
            y = 2.0 * t * cosh(acosh(arg) * (1.0 / 3.0));
        } else {
            y = -2.0 * t * cosh(acosh(-arg) * (1.0 / 3.0));
        }
    } else {
        y = cbrt(-Q);
    }
    return y + m;
}

__device__ __noinline__ double general_polish(Hess g, double F, double sig)
{
    double q, dq;
    shifted_cubic(g, F, sig, q, dq);
    for (int it = 0; it < 2; ++it) {
        if (!(dq != 0.0))
            break;
        const double cand = sig - q / dq;
        double qc, dqc;
        shifted_cubic(g, F, cand, qc, dqc);
        if (!(fabs(qc) < fabs(q)))
            break;
        sig = cand;
        q = qc;
        dq = dqc;
    }
    return sig;
}

__device__ __forceinline__ double smallest_root_general(const Hess &g, double F)
{
    return general_polish(g, F, general_start(g, F));
}

// Newton start for a Hessian that is not SPD: a Gershgorin lower bound of
// lambda_min minus F^{1/3}, where q >= 0.  Kept out of line: the compiler
// would otherwise compute the cube root for every node ahead of the branch,
// while nearly every node takes the SPD start sigma = 0.
__device__ __noinline__ double gershgorin_start(Hess g, double F)
{
    const double lx = g.xx - (fabs(g.xy) + fabs(g.xz));
    const double ly = g.yy - (fabs(g.xy) + fabs(g.yz));
    const double lz = g.zz - (fabs(g.xz) + fabs(g.yz));
    return fmin(lx, fmin(ly, lz)) - cbrt(F);
}

// Smallest real root sigma* of q(sig) = det(G - sig I) - F, which makes
// G - sig* I the Hessian after the centre update u_p += sig* h^2 / 2.
//
// For F > 0 the root is the unique one below lambda_min(G) (Theorem 2.2), and
// on (-inf, lambda_min) q is decreasing and convex, so Newton converges
// monotonically from any start in that interval after at most one step that
// lands on the left of the root.  Start: sig = 0 when G is SPD (Sylvester
// minors), else a Gershgorin lower bound of lambda_min minus F^{1/3}, where
// q >= 0 (the left end of the Theorem 2.2 bracket or further left).
// The Newton quotient uses the hardware reciprocal as it is (relative error
// below 5e-8 on gfx950, measured over 4M random operands): an inexact
// quotient scales a step by 1 + eps, which leaves the iteration's fixed point
// where it is, and at the stop below (a step under 1e-9 of the scale) the
// error it leaves is under eps x 1e-9 of the scale, i.e. round-off.  Stop
// when the step is below 1e-9 of the eigenvalue scale AND below 1e-3 of the
// previous step: in the quadratic phase the error after such a step is
// O(step^2 / scale), i.e. at round-off.
// The test starts after the second step: nearly every node needs two steps
// (one to reach the root, one to show it has), a second step from a root
// moves it by round-off at most, and in a wavefront the two steps then run
// as one branch-free sequence instead of two passes through the loop's
// exit logic.  A node whose first step is already below 1e-9 of the scale
// is settled after the second, as it would have been after the first.
// Near a double smallest eigenvalue with tiny F the iteration converges only
// linearly (steps halve), and a small step says nothing about the remaining
// error; the ratio test keeps it going until the root separates, and a node
// that has not settled after 64 steps is not trusted.
//
// nonconvex is set when F <= 0, when Newton does not settle within 64
// steps, or when the result is not finite; such nodes take the general
// closed form.
__device__ __forceinline__ double smallest_root(const Hess &g, double F, bool &nonconvex)
{
    const double mab = g.xx * g.yy - g.xy * g.xy;
    const double I1 = g.xx + g.yy + g.zz;
    const double I2 = mab + (g.xx * g.zz - g.xz * g.xz) + (g.yy * g.zz - g.yz * g.yz);
    const double I3 = det3(g);
    const double c0 = I3 - F;
    const bool spd = g.xx > 0.0 && mab > 0.0 && I3 > 0.0;
    // one Newton step; returns |step|
    double sig = 0.0;
    auto newton = [&]() {
        const double q = ((I1 - sig) * sig - I2) * sig + c0;
        const double dq = (2.0 * I1 - 3.0 * sig) * sig - I2;
        const double d = q * __builtin_amdgcn_rcp(dq);
        sig -= d;
        return fabs(d);
    };
    // a first step already below the threshold settles the node as it
    // would have alone (the second is then round-off, as large as the first
    // may be, and the ratio test says nothing)
    // (bitwise operators: all three comparisons are cheap, and a
    // short-circuit would cost a divergent branch)
    auto test = [](double ad, double dprev, double thr) {
        return bool(!(ad > thr) & (!(ad > 1e-3 * dprev) | !(dprev > thr)));
    };
    // Every lane takes the two steps from the SPD start sig = 0; one branch
    // then sends the rest (a non-SPD Hessian, no settling yet, a non-finite
    // iterate, F <= 0) down the full rule, which redoes the start where it
    // differs.  A wavefront whose lanes all settle takes no other branch.
    // From sig = 0 the first step's cubic and slope are c0 and -I2 (the
    // general expressions give exactly these for finite invariants; a
    // non-finite one makes the second step non-finite and takes the full
    // rule), and the threshold is 1e-9 |I1|.
    double thr = 1e-9 * fabs(I1);
    double dprev;
    {
        const double d = c0 * __builtin_amdgcn_rcp(-I2);
        sig = -d;
        dprev = fabs(d);
    }
    double ad = newton();
    bool settled = test(ad, dprev, thr);
    if (!((F > 0.0) & spd & settled & bool(isfinite(sig)))) {
        if (F > 0.0) {
            if (!spd) {
                sig = gershgorin_start(g, F);
                thr = 1e-9 * (fabs(I1) + fabs(sig));
                dprev = newton();
                ad = newton();
                settled = test(ad, dprev, thr);
            }
            if (!settled) {
                dprev = ad;
                for (int it = 2; it < 64; ++it) {
                    ad = newton();
                    if (!(ad > thr) && !(ad > 1e-3 * dprev)) {
                        settled = true;
                        break;
                    }
                    dprev = ad;
                }
            }
        }
        if (!(F > 0.0) || !settled || !isfinite(sig)) {
            nonconvex = true;
            sig = smallest_root_general(g, F);
        }
    }
    return sig;
}

// New centre value of one nonlinear Gauss-Seidel update (eq. 2.9 in the
// shifted form): u_p + sigma* h^2 / 2, with half_h2 = 0.5 / s = h^2 / 2
// computed once on the host.
__device__ __forceinline__ double ma_point_update(const Hess &g, double c, double F,
                                                  double half_h2, bool &nonconvex)
{
    const double sig = smallest_root(g, F, nonconvex);
    return c + sig * half_h2;
}

// Blocks are dispatched round-robin over the 8 XCDs of the chip.  Map block
// b of nb to work item tile_of_block(b, nb) so that every XCD gets a
// contiguous range of work items: neighbouring rows / tiles, which read each
// other's data as stencil halos, then share one L2.
__device__ __forceinline__ int tile_of_block(int b, int nb)
{
    const int xcd = b & 7, idx = b >> 3;
    const int q = nb >> 3, rem = nb & 7;
    return xcd * q + min(xcd, rem) + idx;
}

// New centre value of one linear Gauss-Seidel update for Lap_h u = F;
// inv6s = 1 / (6 s) computed once on the host.
__device__ __forceinline__ double lap_point_update(double lap, double c, double F, double inv6s)
{
    return c - (F - lap) * inv6s;
}

} // namespace mafas
