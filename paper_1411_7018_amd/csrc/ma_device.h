// Device-side pointwise pieces of the nonlinear Gauss-Seidel smoother:
// discrete Hessian (eqs. 2.1-2.6), its determinant (the explicit operator of
// Section 1) and the smallest-real-root rule for the local cubic (eqs.
// 2.8-2.9, Theorems 2.1-2.2), in FP64.
#pragma once

#include <hip/hip_runtime.h>

namespace mafas {

struct Hess {
    double xx, yy, zz, xy, xz, yz;
};

// Hessian at linear index p of an x-fastest array with strides (sx, sy, sz);
// s = 1/h^2, s4 = 1/(4h^2) for the grid step h those strides span.  Second differences are taken as
// differences of first differences, which are exact (Sterbenz) when the
// neighbouring values are close; this keeps round-off at the scale of the
// first differences instead of |u|.
template <typename T>
__device__ __forceinline__ Hess hessian_at(const T *__restrict__ u, long p, long sx, long sy,
                                           long sz, double s, double s4)
{
    const double c = u[p];
    Hess g;
    g.xx = ((double(u[p + sx]) - c) - (c - double(u[p - sx]))) * s;
    g.yy = ((double(u[p + sy]) - c) - (c - double(u[p - sy]))) * s;
    g.zz = ((double(u[p + sz]) - c) - (c - double(u[p - sz]))) * s;
    g.xy = ((double(u[p + sx + sy]) - double(u[p - sx + sy]))
            - (double(u[p + sx - sy]) - double(u[p - sx - sy]))) * s4;
    g.xz = ((double(u[p + sx + sz]) - double(u[p - sx + sz]))
            - (double(u[p + sx - sz]) - double(u[p - sx - sz]))) * s4;
    g.yz = ((double(u[p + sy + sz]) - double(u[p - sy + sz]))
            - (double(u[p + sy - sz]) - double(u[p - sy - sz]))) * s4;
    return g;
}

// 7-point Laplacian from differences of first differences.
template <typename T>
__device__ __forceinline__ double laplacian_at(const T *__restrict__ u, long p, long sx, long sy,
                                               long sz, double s)
{
    const double c = u[p];
    return (((double(u[p + sx]) - c) - (c - double(u[p - sx])))
            + ((double(u[p + sy]) - c) - (c - double(u[p - sy])))
            + ((double(u[p + sz]) - c) - (c - double(u[p - sz])))) * s;
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
// convex branch (F <= 0 or a failed Newton bracket).  With m = tr G / 3 and
// y = sig - m the cubic is y^3 - P y + (F - det(G - m I)) = 0, P = tr(B^2)/2
// for the traceless B = G - m I.  Writing y = 2 t cos(phi), t = sqrt(P/3),
// gives cos(3 phi) = -(F - det B)/(2 t^3); the smallest of the three real
// roots takes phi = (acos(.) + 2 pi)/3.  With a single real root the
// hyperbolic form y = +-2 t cosh(acosh|.|/3) applies.  Two Newton steps on
// the shifted form then polish the result, each kept only if |q| drops.
__device__ __noinline__ double smallest_root_general(Hess g, double F)
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
        if (arg >= -1.0 && arg <= 1.0) {
            y = 2.0 * t * cos((acos(arg) + 2.0 * M_PI) * (1.0 / 3.0));
        } else if (arg > 1.0) {
            y = 2.0 * t * cosh(acosh(arg) * (1.0 / 3.0));
        } else {
            y = -2.0 * t * cosh(acosh(-arg) * (1.0 / 3.0));
        }
    } else {
        y = cbrt(-Q);
    }
    double sig = y + m, q, dq;
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

// Smallest real root sigma* of q(sig) = det(G - sig I) - F, which makes
// G - sig* I the Hessian after the centre update u_p += sig* h^2 / 2.
//
// For F > 0 the root is the unique one below lambda_min(G) (Theorem 2.2), and
// on (-inf, lambda_min) q is decreasing and convex, so Newton converges
// monotonically from any start in that interval after at most one step that
// lands on the left of the root.  Start: sig = 0 when G is SPD (Sylvester
// minors), else a Gershgorin lower bound of lambda_min minus F^{1/3}, where
// q >= 0 (the left end of the Theorem 2.2 bracket or further left).
// Stop when the step is below 1e-9 of the eigenvalue scale: the error after
// that step is O(step^2 / scale), i.e. at round-off.
//
// nonconvex is set when F <= 0 or the result is not finite; such nodes take
// the general closed form.
__device__ __forceinline__ double smallest_root(const Hess &g, double F, bool &nonconvex)
{
    const double mab = g.xx * g.yy - g.xy * g.xy;
    const double I1 = g.xx + g.yy + g.zz;
    const double I2 = mab + (g.xx * g.zz - g.xz * g.xz) + (g.yy * g.zz - g.yz * g.yz);
    const double I3 = det3(g);
    if (!(F > 0.0)) {
        nonconvex = true;
        return smallest_root_general(g, F);
    }
    double sig = 0.0;
    if (!(g.xx > 0.0 && mab > 0.0 && I3 > 0.0)) {
        const double lx = g.xx - (fabs(g.xy) + fabs(g.xz));
        const double ly = g.yy - (fabs(g.xy) + fabs(g.yz));
        const double lz = g.zz - (fabs(g.xz) + fabs(g.yz));
        sig = fmin(lx, fmin(ly, lz)) - cbrt(F);
    }
    const double c0 = I3 - F;
    const double scale = fabs(I1) + fabs(sig);
    for (int it = 0; it < 64; ++it) {
        const double q = ((I1 - sig) * sig - I2) * sig + c0;
        const double dq = (2.0 * I1 - 3.0 * sig) * sig - I2;
        const double d = q / dq;
        sig -= d;
        if (!(fabs(d) > 1e-9 * (scale + fabs(sig))))
            break;
    }
    if (!isfinite(sig)) {
        nonconvex = true;
        return smallest_root_general(g, F);
    }
    return sig;
}

} // namespace mafas
