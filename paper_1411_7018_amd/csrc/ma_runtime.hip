// Host runtime behind the C ABI of include/ma.h: parameter checks, hierarchy
// allocation, the component entry points (single-grid kernels) and the
// solve driver.  Full solves run through the batched engine (a single solve
// is a batch of one), following Algorithm 1 repeated under the stopping rule
// of Section 4 after the Poisson initial guess.
#include "ma.h"
#include "ma_engine.h"
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
    if (p->n < 2 || p->n > 2048) {
        why = "n must satisfy 2 <= n <= 2048";
        return false;
    }
    if (p->nu1 < 0 || p->nu2 < 0 || p->nu0 < 1 || p->nu1 > 16 || p->nu2 > 16 || p->nu0 > 16) {
        why = "smoothing counts must satisfy 0 <= nu1, nu2 <= 16 and 1 <= nu0 <= 16";
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
    if (p->tile_config < 0 || p->tile_config > bsweep_num_configs() || p->block_n < -1 ||
        p->block_n > 2048) {
        why = "tile_config must be in 0..12 and block_n in -1..2048";
        return false;
    }
    if (p->max_cycles < 0 || p->init_max_cycles < 0 || p->inner_cycles < 1 ||
        p->inner_cycles > 16) {
        why = "cycle counts must be >= 0 and 1 <= inner_cycles <= 16";
        return false;
    }
    if (p->coarse_n < 0 || p->coarse_n > 32) {
        why = "coarse_n must be in 0..32";
        return false;
    }
    if (p->max_blocks < 0 || p->max_blocks % 8 != 0 || p->max_blocks > (1 << 20)) {
        why = "max_blocks must be 0 or a multiple of 8 up to 2^20";
        return false;
    }
    if (p->strip_rows < 0 || p->strip_rows > 4096) {
        why = "strip_rows must be in 0..4096";
        return false;
    }
    if (p->zsweep_n < -1 || p->zsweep_n > 2048) {
        why = "zsweep_n must be in -1..2048";
        return false;
    }
    if (p->fuse_prolong != 0 && p->fuse_prolong != -1) {
        why = "fuse_prolong must be 0 or -1";
        return false;
    }
    if (p->graphs != 0 && p->graphs != 1) {
        why = "graphs must be 0 or 1";
        return false;
    }
    if (!std::isfinite(p->tol) || !std::isfinite(p->init_tol)) {
        why = "tolerances must be finite";
        return false;
    }
    return true;
}

} // namespace

// the message ma_last_error(NULL) returns, for calls that have no solver
void mafas::set_global_error(const std::string &why) { g_create_error = why; }

double mafas::now_seconds()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// ---------------------------------------------------------------------------
// Hierarchy layout (FP64, (n_l+1)^3 each):
//   level 0: r (residual), R (Poisson right-hand side), t (block-sweep target),
//            fs (colour-ordered right-hand side, FP64 4-colour solvers);
//   level l >= 1: u, b, w, r, t.
// Plus the single-grid norm partials, the batch-of-one engine's partials and
// lists, and the MA_MIXED FP32 hierarchy.
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
    if (p->order == MA_COLOR4 && p->precision == MA_FP64 && p->n >= 2)
        b += size_t(4 * fs_colour_count(p->n)) * sizeof(double);
    b += residual_partials(p->n) * sizeof(double);
    const size_t rows = size_t((p->n - 1 + 63) / 64) * size_t(p->n - 1) * size_t(p->n - 1);
    b += rows * sizeof(double) + (64 << 10) + 4096;
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
    p->graphs = 1;
    p->coarse_n = 16;
    p->max_blocks = 0;
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

ma_status ma_retune(ma_solver *s, int coarse_n, int max_blocks, int strip_rows, int block_n)
{
    if (!s)
        return MA_ERR_ARG;
    ma_params q = s->p;
    q.coarse_n = coarse_n;
    q.max_blocks = max_blocks;
    q.strip_rows = strip_rows;
    q.block_n = block_n;
    std::string why;
    if (!valid_params(&q, why))
        return s->fail(MA_ERR_ARG, why);
    s->p = q;
    return MA_OK;
}

ma_status ma_retune_smoother(ma_solver *s, int block_n, int zsweep_n, int tile_config)
{
    if (!s)
        return MA_ERR_ARG;
    ma_params q = s->p;
    q.block_n = block_n;
    q.zsweep_n = zsweep_n;
    q.tile_config = tile_config;
    std::string why;
    if (!valid_params(&q, why))
        return s->fail(MA_ERR_ARG, why);
    s->p = q;
    return MA_OK;
}

ma_status ma_solve(ma_solver *s, double *u, const double *f, double tol, unsigned flags,
                   ma_report *rep)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f)
        return s->fail(MA_ERR_ARG, "u and f must be device pointers");
    if ((flags & MA_INIT_POISSON) && (flags & MA_INIT_FMG))
        return s->fail(MA_ERR_ARG, "MA_INIT_POISSON and MA_INIT_FMG exclude each other");
    SolveState st;
    st.tol = tol > 0.0 ? tol : s->p.tol;
    st.phase = (flags & MA_INIT_POISSON) ? SolveState::INIT0 : SolveState::MAIN0;
    st.t0 = now_seconds();
    std::memset(&st.rep, 0, sizeof(st.rep));
    if (flags & MA_INIT_FMG)
        MA_TRY(fmg_start(s, u, f, st));
    Engine *E = nullptr;
    MA_TRY(s->own_engine(&E, u, f));
    if (E->reset_counters(0) != MA_OK)
        return s->fail(MA_ERR_DEVICE, E->error());
    std::vector<SolveState *> states{&st};
    while (st.phase != SolveState::DONE) {
        if (drive_step(*E, states, false, true) != MA_OK)
            return s->fail(MA_ERR_DEVICE, E->error());
    }
    std::vector<unsigned long long> nc, fb;
    if (E->read_counters(nc, fb) == MA_OK) {
        st.rep.nonconvex = (long long)nc[0] + st.fmg_nonconvex;
        st.rep.fp64_fallbacks = (long long)fb[0];
    }
    if (s->p.profile) {
        int launches = 0;
        E->take_profile(&st.rep.smooth_seconds, &launches, &st.rep.smooth_bytes);
        st.rep.smooth_launches = launches;
    }
    st.rep.seconds = now_seconds() - st.t0;
    if (rep)
        *rep = st.rep;
    if (st.status != MA_OK)
        return s->fail(st.status, st.err);
    return MA_OK;
}

ma_status ma_vcycle(ma_solver *s, double *u, const double *f)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f)
        return s->fail(MA_ERR_ARG, "u and f must be device pointers");
    if (s->p.precision == MA_MIXED)
        return s->fail(MA_ERR_ARG, "ma_vcycle runs FP64 cycles; MA_MIXED solvers use ma_solve");
    Engine *E = nullptr;
    MA_TRY(s->own_engine(&E, u, f));
    std::vector<double> norms;
    if (E->tick(Engine::MODE_MA, std::vector<char>{1}, norms) != MA_OK)
        return s->fail(MA_ERR_DEVICE, E->error());
    return MA_OK;
}

ma_status ma_residual(ma_solver *s, const double *u, const double *f, double *r_or_null,
                      double *l2_host)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f)
        return s->fail(MA_ERR_ARG, "u and f must be device pointers");
    if (r_or_null)
        MA_HIP(s, launch_fill(s->stream, npts(s->p.n), 0.0, r_or_null));
    MA_HIP(s, launch_residual(s->stream, OP_MA, s->p.n, u, f, r_or_null, s->partials));
    if (l2_host) {
        double l2;
        MA_TRY(s->finish_norm(s->p.n, &l2));
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
        MA_HIP(s, hipMemcpyAsync(s->hpin_u64, s->dcount, sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, s->stream));
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
    MA_HIP(s, launch_restrict(s->stream, OP_MA, s->rmode(), n, u, s->lv[0].r, w_c, s->lv[1].u,
                              b_c));
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

ma_status ma_gs_solve(ma_solver *s, double *u, const double *f, double tol, int max_sweeps,
                      ma_report *rep)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f || max_sweeps < 0)
        return s->fail(MA_ERR_ARG, "u, f must be device pointers and max_sweeps >= 0");
    const double t0 = now_seconds();
    const int n = s->p.n;
    const double target = tol > 0.0 ? tol : s->p.tol;
    ma_report r;
    std::memset(&r, 0, sizeof(r));
    auto norm = [&](double *l2) -> ma_status {
        MA_HIP(s, launch_residual(s->stream, OP_MA, n, u, f, nullptr, s->partials));
        return s->finish_norm(n, l2);
    };
    MA_TRY(norm(&r.res0));
    r.res = r.res0;
    MA_HIP(s, launch_fill_u64(s->stream, 1, 0ull, s->dcount));
    ma_status st = MA_ERR_NOT_CONVERGED;
    if (!std::isfinite(r.res0)) {
        st = MA_ERR_NONFINITE;
    } else if (r.res0 == 0.0) {
        st = MA_OK;
    } else {
        const double in = interior(n);
        while (r.cycles < max_sweeps) {
            MA_TRY(s->smooth(0, u, f, 1, OP_MA));
            r.cycles += 1;
            r.point_updates += in;
            r.alg_bytes += 24.0 * in + 16.0 * in;   // sweep + residual check
            MA_TRY(norm(&r.res));
            if (r.cycles <= 64)
                r.history[r.cycles - 1] = r.res;
            if (!std::isfinite(r.res)) {
                st = MA_ERR_NONFINITE;
                break;
            }
            if (r.res <= target * r.res0) {
                st = MA_OK;
                break;
            }
        }
    }
    r.rel_res = r.res0 > 0.0 ? r.res / r.res0 : 0.0;
    r.converged = st == MA_OK;
    MA_HIP(s, hipMemcpyAsync(s->hpin_u64, s->dcount, sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, s->stream));
    MA_HIP(s, hipStreamSynchronize(s->stream));
    r.nonconvex = (long long)s->hpin_u64[0];
    r.seconds = now_seconds() - t0;
    if (rep)
        *rep = r;
    if (st == MA_ERR_NOT_CONVERGED)
        return s->fail(st, "max_sweeps reached before the tolerance");
    if (st == MA_ERR_NONFINITE)
        return s->fail(st, "residual is not finite");
    return MA_OK;
}

ma_status ma_fmg(ma_solver *s, double *u, const double *f, long long *nonconvex_host)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f)
        return s->fail(MA_ERR_ARG, "u and f must be device pointers");
    long long nc = 0;
    MA_TRY(s->fmg(u, f, &nc, nullptr, nullptr));
    if (nonconvex_host)
        *nonconvex_host = nc;
    return MA_OK;
}

ma_status ma_poisson_init(ma_solver *s, double *u, const double *f, int *cycles_host)
{
    if (!s)
        return MA_ERR_ARG;
    if (!u || !f)
        return s->fail(MA_ERR_ARG, "u and f must be device pointers");
    Engine *E = nullptr;
    MA_TRY(s->own_engine(&E, u, f));
    SolveState st;
    st.phase = SolveState::INIT0;
    std::memset(&st.rep, 0, sizeof(st.rep));
    std::vector<SolveState *> states{&st};
    // drive the Poisson phases only: stop once the solve would start its
    // main phase (the residual of the guess is not needed here)
    while (st.phase == SolveState::INIT0 || st.phase == SolveState::INIT) {
        if (drive_step(*E, states, true) != MA_OK)
            return s->fail(MA_ERR_DEVICE, E->error());
    }
    if (st.status != MA_OK)
        return s->fail(st.status, st.err);
    if (cycles_host)
        *cycles_host = st.rep.init_cycles;
    return MA_OK;
}

} // extern "C"

// ---------------------------------------------------------------------------
// ma_solver methods
// ---------------------------------------------------------------------------
ma_solver::~ma_solver()
{
    for (ma_solver *v : views)
        delete v;
    delete eng;
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
            if (p.order == MA_COLOR4 && p.precision == MA_FP64 && v.n >= 2) {
                fs_cs = fs_colour_count(v.n);
                MA_TRY(alloc(&fs, size_t(4 * fs_cs)));
            }
        } else {
            MA_TRY(alloc(&v.u, c));
            MA_TRY(alloc(&v.b, c));
            MA_TRY(alloc(&v.w, c));
            MA_TRY(alloc(&v.r, c));
            MA_TRY(alloc(&v.t, c));
        }
    }
    MA_TRY(alloc(&partials, residual_partials(p.n)));
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

// Block sweeps (4-colour FP64 sweeps of level l in one launch each): every
// level with MA_SMOOTHER_FUSED, levels with coarse_n < n <= block_n with
// MA_SMOOTHER_AUTO.
bool ma_solver::use_block(int l) const
{
    if (p.order != MA_COLOR4 || p.smoother == MA_SMOOTHER_COLOR)
        return false;
    if (p.smoother == MA_SMOOTHER_FUSED)
        return true;
    const int n = lv[l].n;
    return n <= block_limit(p) && n > p.coarse_n;
}

int ma_solver::rmode() const { return p.restriction == MA_RESTRICT_HALF ? 1 : 0; }

// count single-grid sweeps of op on level l; the result ends in u.
ma_status ma_solver::smooth(int l, double *u, const double *F, int count, int op)
{
    const int n = lv[l].n;
    int done = 0;
    if (use_block(l) && count >= 2) {
        double *t = lv[l].t;
        for (; done + 2 <= count; done += 2) {
            MA_HIP(this, launch_bsweep_one(stream, op, p.tile_config - 1, n, u, t, F, dcount));
            MA_HIP(this, launch_bsweep_one(stream, op, p.tile_config - 1, n, t, u, F, dcount));
        }
    }
    for (; done < count; ++done)
        MA_HIP(this, launch_sweep_color(stream, op, p.order, n, u, F, dcount));
    return MA_OK;
}

// partials of an n grid -> host l2 = sqrt(h^3 sum r^2) (synchronises).
ma_status ma_solver::finish_norm(int n, double *l2)
{
    MA_HIP(this, launch_reduce(stream, partials, residual_partials(n), dsum));
    MA_HIP(this, hipMemcpyAsync(hpin, dsum, sizeof(double), hipMemcpyDeviceToHost, stream));
    MA_HIP(this, hipStreamSynchronize(stream));
    const double h = 1.0 / double(n);
    *l2 = std::sqrt(hpin[0] * h * h * h);
    return MA_OK;
}

ma_status ma_solver::own_engine(Engine **out, double *u, const double *f)
{
    if (!eng)
        eng = new Engine();
    std::vector<SolveRef> refs(1);
    refs[0].s = this;
    refs[0].u = u;
    refs[0].f = f;
    if (eng->set(refs, stream, p.graphs != 0, p.profile != 0) != MA_OK)
        return fail(MA_ERR_DEVICE, eng->error());
    *out = eng;
    return MA_OK;
}

// A solver over levels l..L-1 of this one: it owns nothing (its level
// arrays are this solver's), and its level 0 takes u and F from the caller
// of its engine (here: this solver's level-l u and b).
ma_solver *ma_solver::view(int l)
{
    if (views.size() < lv.size())
        views.resize(lv.size(), nullptr);
    if (!views[l]) {
        ma_solver *v = new ma_solver();
        v->p = p;
        v->p.n = lv[l].n;
        v->p.precision = MA_FP64;
        v->p.profile = 0;
        v->lv.assign(lv.begin() + l, lv.end());
        v->lv[0].u = v->lv[0].b = v->lv[0].w = nullptr;
        views[l] = v;
    }
    views[l]->stream = stream;
    views[l]->p.coarse_n = p.coarse_n;
    views[l]->p.max_blocks = p.max_blocks;
    views[l]->p.strip_rows = p.strip_rows;
    views[l]->p.block_n = p.block_n;
    views[l]->p.zsweep_n = p.zsweep_n;
    views[l]->p.fuse_prolong = p.fuse_prolong;
    views[l]->p.tile_config = p.tile_config;
    return views[l];
}

// Algorithm 2 unrolled: inject f (b_H := injection of b_h) and the
// Dirichlet data of u down the hierarchy; on the coarsest grid start from
// zero and sweep nu0 times; then on the way up interpolate (cubic FMG
// interpolation) and run one FAS V-cycle per level.
ma_status ma_solver::fmg(double *u, const double *f, long long *nonconvex, double *updates,
                         double *bytes)
{
    const int L = int(lv.size());
    auto U = [&](int l) { return l == 0 ? u : lv[l].u; };
    auto B = [&](int l) -> const double * { return l == 0 ? f : lv[l].b; };
    for (int l = 1; l < L; ++l) {
        MA_HIP(this, launch_inject_all(stream, lv[l - 1].n, B(l - 1), lv[l].b));
        MA_HIP(this, launch_inject_all(stream, lv[l - 1].n, U(l - 1), lv[l].u));
    }
    // coarsest grid: zero inside, then an approximate solve -- nu0 sweeps
    // solve a one-unknown grid exactly; a 3-interval grid (8 unknowns)
    // takes 8 sweeps
    const int c = L - 1;
    const int csweeps = (lv[c].n == 3 && p.nu0 < 8) ? 8 : p.nu0;
    MA_HIP(this, launch_zero_interior(stream, lv[c].n, U(c)));
    MA_HIP(this, launch_fill_u64(stream, 1, 0ull, dcount));
    MA_TRY(smooth(c, U(c), B(c), csweeps, OP_MA));
    MA_HIP(this, hipMemcpyAsync(hpin_u64, dcount, sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, stream));
    MA_HIP(this, hipStreamSynchronize(stream));
    long long nc = (long long)hpin_u64[0];
    double up = double(csweeps) * interior(lv[c].n), by = 24.0 * up;
    std::vector<double> nrm;
    std::vector<unsigned long long> cnt, fb;
    for (int l = L - 2; l >= 0; --l) {
        MA_HIP(this, launch_fmg_interp(stream, lv[l + 1].n, U(l + 1), U(l)));
        ma_solver *v = l == 0 ? this : view(l);
        Engine *E = nullptr;
        MA_TRY(v->own_engine(&E, U(l), B(l)));
        if (E->reset_counters(0) != MA_OK || E->tick(Engine::MODE_MA, {1}, nrm) != MA_OK ||
            E->read_counters(cnt, fb) != MA_OK)
            return fail(MA_ERR_DEVICE, E->error());
        nc += (long long)cnt[0];
        double tu, tb;
        E->tick_cost(Engine::MODE_MA, 0, &tu, &tb);
        up += tu;
        by += tb;
    }
    if (nonconvex)
        *nonconvex += nc;
    if (updates)
        *updates += up;
    if (bytes)
        *bytes += by;
    return MA_OK;
}

ma_status mafas::fmg_start(ma_solver *s, double *u, const double *f, SolveState &st)
{
    MA_HIP(s, launch_zero_interior(s->stream, s->p.n, u));
    Engine *E = nullptr;
    MA_TRY(s->own_engine(&E, u, f));
    std::vector<double> nrm;
    if (E->norms_only(Engine::MODE_MA, {1}, nrm) != MA_OK)
        return s->fail(MA_ERR_DEVICE, E->error());
    st.rep.res0 = st.rep.res = nrm[0];
    MA_TRY(s->fmg(u, f, &st.fmg_nonconvex, &st.rep.point_updates, &st.rep.alg_bytes));
    st.fmg = true;
    st.phase = SolveState::MAIN0;
    return MA_OK;
}

// ---------------------------------------------------------------------------
// Per-solve phase machine shared by ma_solve, ma_solve_batch and ma_batch.
// ---------------------------------------------------------------------------
ma_status mafas::drive_step(Engine &eng, std::vector<SolveState *> &states, bool init_only,
                            bool ahead)
{
    const int S = int(states.size());
    std::vector<char> act(S, 0);
    std::vector<double> nrm;
    auto finish = [&](SolveState *st, ma_status s, const char *why) {
        st->status = s;
        if (s != MA_OK)
            st->err = why;
        st->phase = SolveState::DONE;
    };
    auto select = [&](SolveState::Phase ph) {
        bool any = false;
        for (int i = 0; i < S; ++i) {
            act[i] = states[i] && states[i]->phase == ph;
            any |= act[i] != 0;
        }
        return any;
    };
    const Engine::Mode main_mode = eng.mixed() ? Engine::MODE_MIXED : Engine::MODE_MA;

    // 1. Poisson right-hand sides and the linear residuals of the start
    if (select(SolveState::INIT0)) {
        for (int i = 0; i < S; ++i)
            if (act[i]) {
                const SolveRef &r = eng.ref(i);
                if (launch_poisson_rhs(eng.user(), r.s->p.n, r.f, r.s->R) != hipSuccess)
                    return MA_ERR_DEVICE;
                eng.mark_user();
                eng.rhs_changed(i);
            }
        MA_TRY(eng.norms_only(Engine::MODE_LAP, act, nrm));
        for (int i = 0; i < S; ++i)
            if (act[i]) {
                SolveState *st = states[i];
                st->lin0 = st->last = nrm[i];
                st->prev = 0.0;
                if (!std::isfinite(nrm[i]))
                    finish(st, MA_ERR_NONFINITE, "Poisson initial residual is not finite");
                else if (nrm[i] == 0.0 || eng.ref(i).s->p.init_max_cycles == 0)
                    st->phase = SolveState::MAIN0;
                else
                    st->phase = SolveState::INIT;
            }
    }
    // A tick is queued ahead of the host's stopping test only while every
    // live solve is in the phase being ticked and none can reach its cycle
    // limit at the tick being read: every other reason to stop is one the
    // device sees (the tolerance test and a non-finite norm, on the same sum
    // through sum_threshold), so a solve that stops skips the tick queued
    // after it.
    auto only = [&](SolveState::Phase ph) {
        for (int i = 0; i < S; ++i)
            if (states[i] && states[i]->phase != SolveState::DONE && states[i]->phase != ph)
                return false;
        return true;
    };
    // the host's and the device's stopping decisions on the tick just read
    auto agree = [&](int i, bool host_stop) {
        return eng.halted(i) == host_stop;
    };
    // Whether the tick about to be read will leave solve st above its
    // threshold c, guessed from its contraction so far (a factor of 10 per
    // cycle before two norms are known) with a margin of 8: a tick queued
    // ahead of a solve that then stops is skipped on the device but still
    // costs its launches, while one not queued costs only a host round trip.
    auto goes_on = [](const SolveState *st, double c) {
        const double rho = st->prev > 0.0 ? st->last / st->prev : 0.1;
        return st->last * rho > 8.0 * c;
    };
    // The same guess one tick further: what is queued ahead may be two ticks
    // in one graph (one graph boundary fewer) when the solve is guessed to
    // go on after the tick following the one being read as well.
    auto goes_on2 = [](const SolveState *st, double c) {
        const double rho = st->prev > 0.0 ? st->last / st->prev : 0.1;
        return st->last * rho * rho > 8.0 * c;
    };
    // 2. one linear V-cycle of the Poisson guess
    bool init_ahead = false;
    if (select(SolveState::INIT)) {
        std::vector<double> thr(S, -1.0);
        bool spec = ahead && only(SolveState::INIT);
        bool pair = spec;
        for (int i = 0; i < S; ++i)
            if (act[i]) {
                const ma_params &p = eng.ref(i).s->p;
                const double c = p.init_tol * states[i]->lin0;
                thr[i] = sum_threshold(c, p.n);
                spec &= states[i]->rep.init_cycles + 2 <= p.init_max_cycles &&
                        goes_on(states[i], c);
                pair &= states[i]->rep.init_cycles + 3 <= p.init_max_cycles &&
                        goes_on2(states[i], c);
            }
        MA_TRY(eng.tick_ahead(Engine::MODE_LAP, act, thr, spec, nrm, spec && pair));
        init_ahead = eng.pending() > 0;
        for (int i = 0; i < S; ++i)
            if (act[i]) {
                SolveState *st = states[i];
                const ma_params &p = eng.ref(i).s->p;
                if (!agree(i, !std::isfinite(nrm[i]) || nrm[i] <= p.init_tol * st->lin0))
                    return eng.fail(MA_ERR_DEVICE, "internal: device stopping flag disagrees "
                                                   "with the Poisson stopping test");
                double up, by;
                eng.tick_cost(Engine::MODE_LAP, i, &up, &by);
                st->rep.alg_bytes += by;
                st->rep.init_cycles += 1;
                st->prev = st->last;
                st->last = nrm[i];
                if (!std::isfinite(nrm[i]))
                    finish(st, MA_ERR_NONFINITE, "Poisson residual is not finite");
                else if (nrm[i] <= p.init_tol * st->lin0 ||
                         st->rep.init_cycles >= p.init_max_cycles)
                    st->phase = SolveState::MAIN0;
            }
    }
    // When this step's Poisson tick left one queued ahead, the solves that
    // left the phase start the next one in the next step: a launch for them
    // now would queue behind a tick that other solves have yet to read.  (A
    // queued tick that no solve reads any more is one they all skip; the
    // next launch waits for it.)
    if (init_only || init_ahead)
        return MA_OK;
    // 3. residual of the initial guess (res0 of the stopping rule)
    if (select(SolveState::MAIN0)) {
        MA_TRY(eng.norms_only(main_mode, act, nrm));
        for (int i = 0; i < S; ++i)
            if (act[i]) {
                SolveState *st = states[i];
                const int maxc = eng.ref(i).s->p.max_cycles;
                if (st->fmg) {
                    // the FMG-FAS iteration is the first cycle; res0 is the
                    // residual of the zero-interior start
                    ma_report &r = st->rep;
                    r.cycles = 1;
                    r.outer = eng.mixed() ? 1 : 0;
                    r.res = r.history[0] = nrm[i];
                    st->last = nrm[i];
                    st->prev = 0.0;
                    st->best = r.res0;
                    st->stall = 0;
                    r.rel_res = r.res0 > 0.0 ? r.res / r.res0 : 0.0;
                    if (!std::isfinite(nrm[i]))
                        finish(st, MA_ERR_NONFINITE, "residual after FMG is not finite");
                    else if (r.res <= st->tol * r.res0) {
                        r.converged = 1;
                        finish(st, MA_OK, "");
                    } else if (maxc <= 1) {
                        finish(st, MA_ERR_NOT_CONVERGED, "max_cycles reached before the tolerance");
                    } else {
                        st->phase = SolveState::MAIN;
                    }
                    continue;
                }
                st->rep.res0 = st->rep.res = st->last = nrm[i];
                st->prev = 0.0;
                st->best = nrm[i];
                st->stall = 0;
                if (!std::isfinite(nrm[i]))
                    finish(st, MA_ERR_NONFINITE, "initial residual is not finite");
                else if (nrm[i] == 0.0) {
                    st->rep.converged = 1;
                    finish(st, MA_OK, "");
                } else if (maxc == 0) {
                    finish(st, MA_ERR_NOT_CONVERGED, "max_cycles is 0");
                } else {
                    st->phase = SolveState::MAIN;
                }
            }
    }
    // 4. one V-cycle (FP64) or one outer correction (mixed)
    if (select(SolveState::MAIN)) {
        std::vector<double> thr(S, -1.0);
        bool spec = ahead && only(SolveState::MAIN);
        bool pair = spec;
        for (int i = 0; i < S; ++i)
            if (act[i]) {
                const ma_params &p = eng.ref(i).s->p;
                const ma_report &r = states[i]->rep;
                const double c = states[i]->tol * r.res0;
                thr[i] = sum_threshold(c, p.n);
                const int done = main_mode == Engine::MODE_MIXED ? r.outer : r.cycles;
                // a stall stop is the host's own decision too: no tick ahead
                // of one that could make it
                spec &= done + 2 <= p.max_cycles && goes_on(states[i], c) &&
                        states[i]->stall + 1 < 3;
                pair &= done + 3 <= p.max_cycles && goes_on2(states[i], c) &&
                        states[i]->stall + 2 < 3;
            }
        MA_TRY(eng.tick_ahead(main_mode, act, thr, spec, nrm, spec && pair));
        for (int i = 0; i < S; ++i)
            if (act[i]) {
                SolveState *st = states[i];
                const ma_params &p = eng.ref(i).s->p;
                ma_report &r = st->rep;
                if (!agree(i, !std::isfinite(nrm[i]) || nrm[i] <= st->tol * r.res0))
                    return eng.fail(MA_ERR_DEVICE, "internal: device stopping flag disagrees "
                                                   "with the stopping test");
                double up, by;
                eng.tick_cost(main_mode, i, &up, &by);
                r.point_updates += up;
                r.alg_bytes += by;
                int steps;
                if (main_mode == Engine::MODE_MIXED) {
                    r.cycles += p.inner_cycles;
                    r.outer += 1;
                    steps = r.outer;
                } else {
                    r.cycles += 1;
                    steps = r.cycles;
                }
                if (steps - 1 < 64)
                    r.history[steps - 1] = nrm[i];
                r.res = nrm[i];
                st->prev = st->last;
                st->last = nrm[i];
                r.rel_res = r.res / r.res0;
                const int stalled = r.res < 0.9 * st->best ? 0 : st->stall + 1;
                if (stalled == 0)
                    st->best = r.res;
                st->stall = stalled;
                if (!std::isfinite(r.res)) {
                    finish(st, MA_ERR_NONFINITE, "residual is not finite");
                } else if (r.res <= st->tol * r.res0) {
                    r.converged = 1;
                    finish(st, MA_OK, "");
                } else if (st->stall >= 3) {
                    finish(st, MA_ERR_NOT_CONVERGED,
                           "the residual stagnated above the tolerance (round-off floor)");
                } else if (steps >= p.max_cycles) {
                    finish(st, MA_ERR_NOT_CONVERGED, "max_cycles reached before the tolerance");
                }
            }
    }
    return MA_OK;
}
