// Solver object behind the opaque ma_solver handle of include/ma.h.
#pragma once

#include "ma.h"
#include "ma_internal.h"

#include <string>
#include <vector>

#define MA_TRY(expr)                                                                             \
    do {                                                                                         \
        const ma_status st_ = (expr);                                                            \
        if (st_ != MA_OK)                                                                        \
            return st_;                                                                          \
    } while (0)

#define MA_HIP(obj, expr)                                                                        \
    do {                                                                                         \
        const hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                                    \
            return (obj)->fail(MA_ERR_DEVICE,                                                    \
                               std::string(#expr) + ": " + hipGetErrorString(e_));             \
    } while (0)

namespace mafas {

struct Level {
    int n = 0;
    double *u = nullptr;   // iterate (level 0: the caller's array)
    double *b = nullptr;   // right-hand side (level 0: the caller's f or R)
    double *w = nullptr;   // injected fine approximation (coarse levels)
    double *r = nullptr;   // residual
    double *t = nullptr;   // out-of-place sweep target
};

// FP32 inner hierarchy of the mixed-precision form (one per level).
struct MixedLevel {
    int n = 0;
    float *d = nullptr;    // correction delta
    float *b = nullptr;    // right-hand side of T(delta) = b
    float *w = nullptr;    // injected delta
    float *r = nullptr;    // residual of the inner problem
    float *t = nullptr;    // out-of-place sweep target
    double *U = nullptr;   // injected FP64 approximation (coarse levels)
};

struct Stats {
    double updates = 0.0;  // nonlinear GS point updates
    double bytes = 0.0;    // algorithmic bytes of the kernels launched
    int smooth_launches = 0;       // finest-level smoother launches (profile)
    double smooth_bytes = 0.0;     // their algorithmic bytes
};

size_t hierarchy_bytes(const ma_params *p);
size_t mixed_bytes(const ma_params *p);

hipError_t launch_fill(hipStream_t st, size_t count, double v, double *dst);
hipError_t launch_fill_u64(hipStream_t st, size_t count, unsigned long long v,
                           unsigned long long *dst);

} // namespace mafas

struct ma_solver {
    ma_params p{};
    hipStream_t stream = nullptr;
    std::vector<mafas::Level> lv;
    double *R = nullptr;                  // Poisson right-hand side, finest level
    double *partials = nullptr;
    size_t npartials = 0;
    double *dsum = nullptr;
    unsigned long long *dcount = nullptr; // non-certified update counter
    unsigned long long *dfallback = nullptr;
    double *hpin = nullptr;               // pinned host scalars
    unsigned long long *hpin_u64 = nullptr;
    std::vector<double *> owned;
    std::string err;
    mafas::Stats stats;
    std::vector<hipEvent_t> ev_pool;      // profile: start/stop pairs
    size_t ev_used = 0;

    // mixed precision
    std::vector<mafas::MixedLevel> mx;
    double *r64 = nullptr;                // finest FP64 residual f - S(u)
    std::vector<void *> mixed_owned;

    ~ma_solver();
    ma_status fail(ma_status st, const std::string &msg);
    ma_status alloc(double **q, size_t count);
    ma_status allocate();
    void bind_finest(double *u, const double *f);
    bool use_fused(int l) const;
    int rmode() const;
    ma_status smooth(int l, double *u, const double *F, int count, int op);
    ma_status vcycle(int l, int op);
    ma_status finish_norm(int n, double *l2);
    ma_status norm(int op, const double *u, const double *F, double *l2);
    ma_status poisson_init(double *u, const double *f, int *cycles);
    ma_status read_nonconvex(long long *out);
    ma_status prof_mark(hipEvent_t *ev);
    ma_status prof_collect(double *seconds);
    ma_status solve(double *u, const double *f, double tol, unsigned flags, ma_report *r);
    ma_status solve_fp64(double *u, const double *f, double tol, ma_report *r);

    // mixed precision (ma_mixed.hip)
    ma_status mixed_allocate();
    void mixed_release();
    ma_status solve_mixed(double *u, const double *f, double tol, ma_report *r);
};
