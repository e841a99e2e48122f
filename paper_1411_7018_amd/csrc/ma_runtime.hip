// Host runtime behind the C ABI of include/ma.h: hierarchy allocation, the
// FAS V-cycle driver (Algorithm 1), the stopping rule of Section 4, the
// Poisson initial guess, and the resident batch used for serving.
#include "ma.h"
#include "ma_internal.h"
#include "ma_runtime.h"

#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

using namespace mafas;

namespace {

thread_local std::string g_create_error;

bool valid_params(const ma_params *p, std::string &why)
{
    if (!p) {
        why = "params is NULL";
        return false;
    }
    if (p->n < 2) {
        why = "n must be >= 2";
        return false;
    }
    if (p->n > 2048) {
        why = "n must be <= 2048";
        return false;
    }
    if (p->nu1 < 0 || p->nu2 < 0 || p->nu0 < 1 || p->nu1 > 64 || p->nu2 > 64 || p->nu0 > 64) {
        why = "smoothing counts must satisfy 0 <= nu1, nu2 <= 64 and 1 <= nu0 <= 64";
        return false;
    }
    if (p->order != MA_COLOR4 && p->order != MA_COLOR8) {
        why = "order must be MA_COLOR4 or MA_COLOR8";
        return false;
    }
    if (p->restriction != MA_RESTRICT_FULL && p->restriction != MA_RESTRICT_HALF) {
        why = "restriction must be MA_RESTRICT_FULL or MA_RESTRICT_HALF";
        return false;
    }
    if (p->precision != MA_FP64 && p->precision != MA_MIXED) {
        why = "precision must be MA_FP64 or MA_MIXED";
        return false;
    }
    if (p->smoother < MA_SMOOTHER_AUTO || p->smoother > MA_SMOOTHER_FUSED) {
        why = "unknown smoother";
        return false;
    }
    if (p->tile_config < 0 || p->tile_config > fused_num_configs() || p->zchunk < 0) {
        why = "tile_config must be 0..fused_num_configs() and zchunk >= 0";
        return false;
    }
    if (p->max_cycles < 0 || p->init_max_cycles < 0 || p->inner_cycles < 1) {
        why = "cycle counts must be >= 0 (inner_cycles >= 1)";
        return false;
    }
    if (!std::isfinite(p->tol) || !std::isfinite(p->init_tol)) {
        why = "tolerances must be finite";
        return false;
    }
    return true;
}

} // namespace

// ---------------------------------------------------------------------------
// Hierarchy layout (all FP64, (n_l+1)^3 each):
//   level 0: r (residual), R (Poisson right-hand side), t (sweep target);
//   level l >= 1: u, b (right-hand side), w (injected approximation), r, t.
// Plus the residual partial sums (sized for level 0), one device scalar and
// one device counter.  The MA_MIXED buffers are added by the mixed module.
// ---------------------------------------------------------------------------
size_t mafas::hierarchy_bytes(const ma_params *p)
{
    int ns[32];
    const int L = ma_levels(p->n, ns, 32);
    size_t b = 0;
    for (int l = 0; l < L; ++l) {
        const size_t c = npts(ns[l]) * sizeof(double);
        b += (l == 0) ? 3 * c : 5 * c;
    }
    b += residual_partials(p->n) * sizeof(double) + 256;
    if (p->precision == MA_MIXED)
        b += mixed_bytes(p);
    return b;
}

extern "C" {

void ma_params_default(ma_params *p, int n)
{
    std::memset(p, 0, sizeof(*p));
    p->n = n;
    p->nu1 = 2;
    p->nu2 = 2;
    p->nu0 = 1;
    p->order = MA_COLOR4;
    p->restriction = MA_RESTRICT_FULL;
    p->precision = MA_FP64;
    p->smoother = MA_SMOOTHER_AUTO;
    p->max_cycles = 100;
    p->tol = 1e-8;
    p->init_tol = 1e-6;
    p->init_max_cycles = 30;
    p->inner_cycles = 2;
}

int ma_levels(int n, int *ns, int cap)
{
    int L = 0;
    if (n < 2 || cap < 1 || !ns)
        return 0;
    ns[L++] = n;
    while (n % 2 == 0 && n >= 4 && L < cap) {
        n /= 2;
        ns[L++] = n;
    }
    return L;
}

size_t ma_footprint_bytes(const ma_params *p)
{
    std::string why;
    if (!valid_params(p, why))
        return 0;
    return hierarchy_bytes(p);
}

ma_status ma_create(const ma_params *p, void *hip_stream, ma_solver **out)
{
    std::string why;
    if (!out) {
        g_create_error = "out is NULL";
        return MA_ERR_ARG;
    }
    *out = nullptr;
    if (!valid_params(p, why)) {
        g_create_error = why;
        return MA_ERR_ARG;
    }
    ma_solver *s = new ma_solver();
    s->p = *p;
    s->stream = static_cast<hipStream_t>(hip_stream);
    const ma_status st = s->allocate();
    if (st != MA_OK) {
        g_create_error = s->err;
        delete s;
        return st;
    }
    *out = s;
    return MA_OK;
}

void ma_destroy(ma_solver *s) { delete s; }

const char *ma_last_error(const ma_solver *s)
{
    return s ? s->err.c_str() : g_create_error.c_str();
}

ma_status ma_set_stream(ma_solver *s, void *hip_stream)
{
    if (!s)
        return MA_ERR_ARG;
    s->stream = static_cast<hipStream_t>(hip_stream);
    return MA_OK;
}

ma_status ma_solve(ma_solver *s, double *u, const double *f, double tol, unsigned flags,
                   ma_report *rep)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f)
        return s->fail(MA_ERR_ARG, "u and f must be device pointers");
    ma_report local;
    ma_report *r = rep ? rep : &local;
    return s->solve(u, f, tol > 0.0 ? tol : s->p.tol, flags, r);
}

ma_status ma_vcycle(ma_solver *s, double *u, const double *f)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f)
        return s->fail(MA_ERR_ARG, "u and f must be device pointers");
    if (s->p.precision == MA_MIXED)
        return s->fail(MA_ERR_ARG, "ma_vcycle runs FP64 cycles; MA_MIXED solvers use ma_solve");
    s->bind_finest(u, f);
    return s->vcycle(0, OP_MA);
}

ma_status ma_residual(ma_solver *s, const double *u, const double *f, double *r_or_null,
                      double *l2_host)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f)
        return s->fail(MA_ERR_ARG, "u and f must be device pointers");
    if (r_or_null) {
        MA_HIP(s, launch_fill(s->stream, npts(s->p.n), 0.0, r_or_null));
    }
    MA_HIP(s, launch_residual(s->stream, OP_MA, s->p.n, u, f, r_or_null, s->partials));
    if (l2_host) {
        double l2;
        const ma_status st = s->finish_norm(s->p.n, &l2);
        if (st != MA_OK)
            return st;
        *l2_host = l2;
    }
    return MA_OK;
}

ma_status ma_sweep(ma_solver *s, double *u, const double *f, int count, long long *nonconvex_host)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f || count < 0)
        return s->fail(MA_ERR_ARG, "u, f must be device pointers and count >= 0");
    MA_HIP(s, launch_fill_u64(s->stream, 1, 0ull, s->dcount));
    MA_TRY(s->smooth(0, u, f, count, OP_MA));
    if (nonconvex_host) {
        unsigned long long c = 0;
        MA_HIP(s, hipMemcpyAsync(s->hpin_u64, s->dcount, sizeof(c), hipMemcpyDeviceToHost,
                                 s->stream));
        MA_HIP(s, hipStreamSynchronize(s->stream));
        *nonconvex_host = (long long)s->hpin_u64[0];
    }
    return MA_OK;
}

ma_status ma_restrict(ma_solver *s, const double *u, const double *f, double *w_c, double *b_c)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f || !w_c || !b_c)
        return s->fail(MA_ERR_ARG, "null device pointer");
    if (s->lv.size() < 2)
        return s->fail(MA_ERR_ARG, "n must be even and >= 4 for a coarser level");
    const int n = s->p.n;
    MA_HIP(s, launch_residual(s->stream, OP_MA, n, u, f, s->lv[0].r, s->partials));
    MA_HIP(s, launch_restrict(s->stream, OP_MA, s->rmode(), n, u, s->lv[0].r, w_c,
                              s->lv[1].u, b_c));
    return MA_OK;
}

ma_status ma_prolong_correct(ma_solver *s, double *u, const double *u_c, const double *w_c)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !u_c || !w_c)
        return s->fail(MA_ERR_ARG, "null device pointer");
    if (s->p.n % 2 || s->p.n < 4)
        return s->fail(MA_ERR_ARG, "n must be even and >= 4");
    MA_HIP(s, launch_prolong(s->stream, s->p.n, u, u_c, w_c));
    return MA_OK;
}

ma_status ma_poisson_init(ma_solver *s, double *u, const double *f, int *cycles_host)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f)
        return s->fail(MA_ERR_ARG, "u and f must be device pointers");
    int c = 0;
    MA_TRY(s->poisson_init(u, f, &c));
    if (cycles_host)
        *cycles_host = c;
    return MA_OK;
}

} // extern "C"

// ---------------------------------------------------------------------------
// ma_solver methods
// ---------------------------------------------------------------------------
ma_solver::~ma_solver()
{
    for (hipEvent_t e : ev_pool)
        (void)hipEventDestroy(e);
    for (double *q : owned)
        (void)hipFree(q);
    if (hpin)
        (void)hipHostFree(hpin);
    if (hpin_u64)
        (void)hipHostFree(hpin_u64);
    mixed_release();
}

ma_status ma_solver::fail(ma_status st, const std::string &msg)
{
    err = msg;
    return st;
}

ma_status ma_solver::alloc(double **q, size_t count)
{
    *q = nullptr;
    if (count == 0)
        return MA_OK;
    const hipError_t e = hipMalloc(reinterpret_cast<void **>(q), count * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *q = nullptr;
        return fail(e == hipErrorOutOfMemory ? MA_ERR_OOM : MA_ERR_DEVICE,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    owned.push_back(*q);
    const hipError_t z = launch_fill(stream, count, 0.0, *q);
    if (z != hipSuccess)
        return fail(MA_ERR_DEVICE, std::string("fill: ") + hipGetErrorString(z));
    return MA_OK;
}

ma_status ma_solver::allocate()
{
    int ns[32];
    const int L = ma_levels(p.n, ns, 32);
    lv.resize(L);
    for (int l = 0; l < L; ++l) {
        Level &v = lv[l];
        v.n = ns[l];
        const size_t c = npts(v.n);
        if (l == 0) {
            MA_TRY(alloc(&v.r, c));
            MA_TRY(alloc(&R, c));
            MA_TRY(alloc(&v.t, c));
        } else {
            MA_TRY(alloc(&v.u, c));
            MA_TRY(alloc(&v.b, c));
            MA_TRY(alloc(&v.w, c));
            MA_TRY(alloc(&v.r, c));
            MA_TRY(alloc(&v.t, c));
        }
    }
    npartials = residual_partials(p.n);
    MA_TRY(alloc(&partials, npartials));
    MA_TRY(alloc(&dsum, 4));
    {
        const hipError_t e = hipMalloc(reinterpret_cast<void **>(&dcount), 64);
        if (e != hipSuccess)
            return fail(MA_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
        owned.push_back(reinterpret_cast<double *>(dcount));
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&hpin), 4 * sizeof(double)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&hpin_u64), 4 * sizeof(unsigned long long)) !=
            hipSuccess)
        return fail(MA_ERR_OOM, "hipHostMalloc failed");
    if (p.precision == MA_MIXED)
        MA_TRY(mixed_allocate());
    const hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess)
        return fail(MA_ERR_DEVICE, std::string("allocate: ") + hipGetErrorString(e));
    return MA_OK;
}

void ma_solver::bind_finest(double *u, const double *f)
{
    lv[0].u = u;
    lv[0].b = const_cast<double *>(f);
}

bool ma_solver::use_fused(int l) const
{
    if (p.order != MA_COLOR4 || p.smoother == MA_SMOOTHER_COLOR)
        return false;
    if (p.smoother == MA_SMOOTHER_FUSED)
        return lv[l].n >= 4;
    return fused_supported(lv[l].n);
}

// Profiling: events are recorded in pairs around finest-level smoothing and
// read back (elapsed time summed) when the solve synchronises anyway.
ma_status ma_solver::prof_mark(hipEvent_t *ev)
{
    if (ev_used == ev_pool.size()) {
        hipEvent_t e;
        MA_HIP(this, hipEventCreate(&e));
        ev_pool.push_back(e);
    }
    *ev = ev_pool[ev_used++];
    MA_HIP(this, hipEventRecord(*ev, stream));
    return MA_OK;
}

ma_status ma_solver::prof_collect(double *seconds)
{
    double t = 0.0;
    for (size_t q = 0; q + 1 < ev_used; q += 2) {
        float ms = 0.f;
        MA_HIP(this, hipEventSynchronize(ev_pool[q + 1]));
        MA_HIP(this, hipEventElapsedTime(&ms, ev_pool[q], ev_pool[q + 1]));
        t += 1e-3 * double(ms);
    }
    ev_used = 0;
    *seconds = t;
    return MA_OK;
}

// count sweeps of op on u (level l) with right-hand side F; the result is in u.
ma_status ma_solver::smooth(int l, double *u, const double *F, int count, int op)
{
    const int n = lv[l].n;
    const bool prof = p.profile && l == 0 && op == OP_MA && count > 0;
    hipEvent_t e0, e1;
    if (prof)
        MA_TRY(prof_mark(&e0));
    int done = 0;
    if (use_fused(l) && count >= 2) {
        double *t = lv[l].t;
        MA_HIP(this, launch_copy_boundary(stream, n, u, t));
        for (; done + 2 <= count; done += 2) {
            MA_HIP(this, launch_sweep_fused(stream, op, n, u, t, F, dcount, p.tile_config - 1,
                                            p.zchunk));
            MA_HIP(this, launch_sweep_fused(stream, op, n, t, u, F, dcount, p.tile_config - 1,
                                            p.zchunk));
        }
    }
    const int fused_launches = done;
    for (; done < count; ++done)
        MA_HIP(this, launch_sweep_color(stream, op, p.order, n, u, F, dcount));
    if (op == OP_MA) {
        stats.updates += double(count) * interior(n);
        stats.bytes += double(count) * 24.0 * interior(n);
    }
    if (prof) {
        MA_TRY(prof_mark(&e1));
        stats.smooth_launches += fused_launches + (count - fused_launches) * (p.order == 1 ? 8 : 4);
        stats.smooth_bytes += double(count) * 24.0 * interior(n);
    }
    return MA_OK;
}

int ma_solver::rmode() const { return p.restriction == MA_RESTRICT_HALF ? 1 : 0; }

// Algorithm 1 on level l: u = lv[l].u, right-hand side lv[l].b.
ma_status ma_solver::vcycle(int l, int op)
{
    Level &v = lv[l];
    const int L = int(lv.size());
    if (l == L - 1)
        return smooth(l, v.u, v.b, p.nu0, op);
    MA_TRY(smooth(l, v.u, v.b, p.nu1, op));
    Level &c = lv[l + 1];
    MA_HIP(this, launch_residual(stream, op, v.n, v.u, v.b, v.r, partials));
    MA_HIP(this, launch_restrict(stream, op, rmode(), v.n, v.u, v.r, c.w, c.u, c.b));
    const double fine = interior(v.n), coarse = double(npts(c.n));
    stats.bytes += 24.0 * fine + 8.0 * fine + 8.0 * coarse + 24.0 * coarse;
    MA_TRY(vcycle(l + 1, op));
    MA_HIP(this, launch_prolong(stream, v.n, v.u, c.u, c.w));
    stats.bytes += 16.0 * fine + 16.0 * coarse;
    return smooth(l, v.u, v.b, p.nu2, op);
}

// partials of level n -> host l2 = sqrt(h^3 sum r^2) (synchronises).
ma_status ma_solver::finish_norm(int n, double *l2)
{
    MA_HIP(this, launch_reduce(stream, partials, residual_partials(n), dsum));
    MA_HIP(this, hipMemcpyAsync(hpin, dsum, sizeof(double), hipMemcpyDeviceToHost, stream));
    MA_HIP(this, hipStreamSynchronize(stream));
    const double h = 1.0 / double(n);
    *l2 = std::sqrt(hpin[0] * h * h * h);
    return MA_OK;
}

ma_status ma_solver::norm(int op, const double *u, const double *F, double *l2)
{
    MA_HIP(this, launch_residual(stream, op, p.n, u, F, nullptr, partials));
    stats.bytes += 16.0 * interior(p.n);
    return finish_norm(p.n, l2);
}

ma_status ma_solver::poisson_init(double *u, const double *f, int *cycles)
{
    *cycles = 0;
    MA_HIP(this, launch_poisson_rhs(stream, p.n, f, R));
    bind_finest(u, R);
    double r0, r;
    MA_TRY(norm(OP_LAP, u, R, &r0));
    if (!std::isfinite(r0))
        return fail(MA_ERR_NONFINITE, "Poisson initial residual is not finite");
    if (r0 == 0.0)
        return MA_OK;
    while (*cycles < p.init_max_cycles) {
        MA_TRY(vcycle(0, OP_LAP));
        ++*cycles;
        MA_TRY(norm(OP_LAP, u, R, &r));
        if (!std::isfinite(r))
            return fail(MA_ERR_NONFINITE, "Poisson residual is not finite");
        if (r <= p.init_tol * r0)
            break;
    }
    return MA_OK;
}

ma_status ma_solver::read_nonconvex(long long *out)
{
    MA_HIP(this, hipMemcpyAsync(hpin_u64, dcount, sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, stream));
    MA_HIP(this, hipStreamSynchronize(stream));
    *out = (long long)hpin_u64[0];
    return MA_OK;
}

ma_status ma_solver::solve(double *u, const double *f, double tol, unsigned flags, ma_report *r)
{
    const auto t0 = std::chrono::steady_clock::now();
    std::memset(r, 0, sizeof(*r));
    stats = Stats();
    ev_used = 0;
    MA_HIP(this, launch_fill_u64(stream, 1, 0ull, dcount));
    if (flags & MA_INIT_POISSON)
        MA_TRY(poisson_init(u, f, &r->init_cycles));
    ma_status st;
    if (p.precision == MA_MIXED)
        st = solve_mixed(u, f, tol, r);
    else
        st = solve_fp64(u, f, tol, r);
    long long nc = 0;
    if (read_nonconvex(&nc) == MA_OK)
        r->nonconvex += nc;
    r->point_updates = stats.updates;
    r->alg_bytes = stats.bytes;
    if (p.profile) {
        double t = 0.0;
        if (prof_collect(&t) == MA_OK) {
            r->smooth_seconds = t;
            r->smooth_launches = stats.smooth_launches;
            r->smooth_bytes = stats.smooth_bytes;
        }
    }
    r->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return st;
}

ma_status ma_solver::solve_fp64(double *u, const double *f, double tol, ma_report *r)
{
    bind_finest(u, f);
    MA_TRY(norm(OP_MA, u, f, &r->res0));
    r->res = r->res0;
    if (!std::isfinite(r->res0))
        return fail(MA_ERR_NONFINITE, "initial residual is not finite");
    if (r->res0 == 0.0) {
        r->converged = 1;
        return MA_OK;
    }
    for (int c = 0; c < p.max_cycles; ++c) {
        MA_TRY(vcycle(0, OP_MA));
        r->cycles = c + 1;
        MA_TRY(norm(OP_MA, u, f, &r->res));
        if (c < 64)
            r->history[c] = r->res;
        r->rel_res = r->res / r->res0;
        if (!std::isfinite(r->res))
            return fail(MA_ERR_NONFINITE, "residual is not finite");
        if (r->res <= tol * r->res0) {
            r->converged = 1;
            return MA_OK;
        }
    }
    return fail(MA_ERR_NOT_CONVERGED, "max_cycles reached before the tolerance");
}
