// Device-side pieces of the FP32/FP64 mixed-precision inner problem
// T(delta) = det(H + D^2 delta) - det(H) = r (see ma_mixed.hip).
#pragma once

#include "ma_device.h"

namespace mafas {

struct Sym32 {
    float xx, yy, zz, xy, xz, yz;
};

__device__ __forceinline__ Sym32 to32(const Hess &h)
{
    return Sym32{float(h.xx), float(h.yy), float(h.zz), float(h.xy), float(h.xz), float(h.yz)};
}

// E = D^2 delta at index p (FP32 data, FP32 arithmetic).
__device__ __forceinline__ Sym32 hess32(const float *__restrict__ d, long p, long sx, long sy,
                                        long sz, float s, float s4)
{
    const float c = d[p];
    Sym32 e;
    e.xx = ((d[p + sx] - c) - (c - d[p - sx])) * s;
    e.yy = ((d[p + sy] - c) - (c - d[p - sy])) * s;
    e.zz = ((d[p + sz] - c) - (c - d[p - sz])) * s;
    e.xy = ((d[p + sx + sy] - d[p - sx + sy]) - (d[p + sx - sy] - d[p - sx - sy])) * s4;
    e.xz = ((d[p + sx + sz] - d[p - sx + sz]) - (d[p + sx - sz] - d[p - sx - sz])) * s4;
    e.yz = ((d[p + sy + sz] - d[p - sy + sz]) - (d[p + sy - sz] - d[p - sy - sz])) * s4;
    return e;
}

__device__ __forceinline__ Sym32 adj32(const Sym32 &a)
{
    return Sym32{a.yy * a.zz - a.yz * a.yz, a.xx * a.zz - a.xz * a.xz, a.xx * a.yy - a.xy * a.xy,
                 a.xz * a.yz - a.xy * a.zz, a.xy * a.yz - a.xz * a.yy, a.xy * a.xz - a.xx * a.yz};
}

// tr(A B) for symmetric A, B.
__device__ __forceinline__ float trprod(const Sym32 &a, const Sym32 &b)
{
    return a.xx * b.xx + a.yy * b.yy + a.zz * b.zz
           + 2.0f * (a.xy * b.xy + a.xz * b.xz + a.yz * b.yz);
}

__device__ __forceinline__ float det32(const Sym32 &a, const Sym32 &adja)
{
    return a.xx * adja.xx + a.xy * adja.xy + a.xz * adja.xz;
}

// T(E) = det(H + E) - det(H) through the identity.
__device__ __forceinline__ float t_of(const Sym32 &H, const Sym32 &adjH, const Sym32 &E)
{
    const Sym32 adjE = adj32(E);
    return trprod(adjH, E) + trprod(H, adjE) + det32(E, adjE);
}

// FP64 recomputation of one node: sigma of det(H + E - sigma I) = det(H) + r.
static __device__ __noinline__ double mixed_fp64_root(Hess H, const float *__restrict__ d, long p,
                                               long sy, long sz, double s, double s4, float r,
                                               bool &nonconvex)
{
    const Hess E = hessian_at(d, p, 1, sy, sz, s, s4);
    const double F = det3(H) + double(r);
    Hess G;
    G.xx = H.xx + E.xx;
    G.yy = H.yy + E.yy;
    G.zz = H.zz + E.zz;
    G.xy = H.xy + E.xy;
    G.xz = H.xz + E.xz;
    G.yz = H.yz + E.yz;
    return smallest_root(G, F, nonconvex);
}

// New delta at node p (level grid n): returns the updated value and flags.
__device__ __forceinline__ float mixed_point(const float *__restrict__ d, const double *__restrict__ U,
                                             float b, long p, long sy, long sz, double s, double s4,
                                             float sf, float s4f, float hkf, bool &fallback,
                                             bool &nonconvex)
{
    const Hess H64 = hessian_at(U, p, 1, sy, sz, s, s4);
    const Sym32 H = to32(H64);
    const Sym32 adjH = adj32(H);
    const Sym32 E = hess32(d, p, 1, sy, sz, sf, s4f);
    const float T = t_of(H, adjH, E);
    const float detH = det32(H, adjH);
    const Sym32 G{H.xx + E.xx, H.yy + E.yy, H.zz + E.zz, H.xy + E.xy, H.xz + E.xz, H.yz + E.yz};
    const float I1 = G.xx + G.yy + G.zz;
    const float mab = G.xx * G.yy - G.xy * G.xy;
    const float I2 = mab + (G.xx * G.zz - G.xz * G.xz) + (G.yy * G.zz - G.yz * G.yz);
    const float detG = G.xx * (G.yy * G.zz - G.yz * G.yz) - G.xy * (G.xy * G.zz - G.yz * G.xz)
                       + G.xz * (G.xy * G.yz - G.yy * G.xz);
    const float sc = fabsf(I1) * (1.0f / 3.0f);
    const float m = 1e-3f;
    bool ok = G.xx > m * sc && mab > m * sc * sc && detG > m * sc * sc * sc &&
              detH + b > m * fabsf(detH);
    float sig = 0.0f;
    if (ok) {
        // Stop once the step is below 2e-6 of sigma: the quadratic error
        // left is ~1e-11 of sigma, far below the FP32 noise of q itself,
        // and the outer FP64 residual absorbs what FP32 cannot resolve.
        const float c0 = T - b;
        int it = 0;
        for (; it < 16; ++it) {
            const float q = ((I1 - sig) * sig - I2) * sig + c0;
            const float dq = (2.0f * I1 - 3.0f * sig) * sig - I2;
            const float dd = q / dq;
            sig -= dd;
            if (!(fabsf(dd) > 2e-6f * fabsf(sig)))
                break;
        }
        ok = it < 16 && isfinite(sig);
    }
    if (!ok) {
        fallback = true;
        const double sg = mixed_fp64_root(H64, d, p, sy, sz, s, s4, b, nonconvex);
        return float(double(d[p]) + sg * (0.5 / s));
    }
    return d[p] + sig * hkf;
}

struct LevelConst {
    double s, s4;
    float sf, s4f, hkf;
};

__host__ __device__ inline LevelConst level_const(int n)
{
    LevelConst c;
    c.s = double(n) * double(n);
    c.s4 = 0.25 * c.s;
    c.sf = float(c.s);
    c.s4f = float(c.s4);
    c.hkf = float(0.5 / c.s);
    return c;
}


} // namespace mafas
