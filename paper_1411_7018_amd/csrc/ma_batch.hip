// Batched solves and the resident batch used for continuous serving.  Both
// drive many solves through one Engine: every level phase of every tick is
// one launch over all active solves (the engine's device tables), and each
// solve follows the same phase machine as ma_solve, so its arithmetic and
// its stopping decisions do not depend on its co-tenants.
#include "ma_engine.h"
#include "ma_runtime.h"

#include <cstring>
#include <string>
#include <vector>

using namespace mafas;

struct ma_batch {
    hipStream_t stream = nullptr;
    Engine eng;
    std::vector<SolveRef> refs;
    std::vector<SolveState> st;
    std::vector<char> used;
    bool graphs = true;   // tick replay mode, taken from the first solver added
    std::string err;
    ma_status fail(ma_status s, const std::string &m)
    {
        err = m;
        return s;
    }
    bool any() const
    {
        for (char c : used)
            if (c)
                return true;
        return false;
    }
};

namespace {

void start_state(SolveState &st, const ma_solver *s, double tol, unsigned flags)
{
    st = SolveState();
    std::memset(&st.rep, 0, sizeof(st.rep));
    st.tol = tol > 0.0 ? tol : s->p.tol;
    st.phase = (flags & MA_INIT_POISSON) ? SolveState::INIT0 : SolveState::MAIN0;
    st.t0 = now_seconds();
}

} // namespace

extern "C" {

ma_status ma_solve_batch(ma_solver *const *solvers, double *const *u, const double *const *f,
                         int count, double tol, unsigned flags, ma_report *reps)
{
    if (count < 0 || (count > 0 && (!solvers || !u || !f)))
        return MA_ERR_ARG;
    if ((flags & MA_INIT_POISSON) && (flags & MA_INIT_FMG))
        return MA_ERR_ARG;
    for (int i = 0; i < count; ++i)
        if (!solvers[i] || !u[i] || !f[i])
            return MA_ERR_ARG;
    ma_status first = MA_OK;
    for (int base = 0; base < count; base += kMaxGrids) {
        const int m = std::min(kMaxGrids, count - base);
        Engine eng;
        std::vector<SolveRef> refs(m);
        for (int i = 0; i < m; ++i) {
            refs[i].s = solvers[base + i];
            refs[i].u = u[base + i];
            refs[i].f = f[base + i];
        }
        ma_solver *s0 = solvers[base];
        if (eng.set(refs, s0->stream, s0->p.graphs != 0, s0->p.profile != 0) != MA_OK)
            return s0->fail(MA_ERR_ARG, eng.error());
        std::vector<SolveState> st(m);
        std::vector<SolveState *> ptr(m);
        for (int i = 0; i < m; ++i) {
            start_state(st[i], refs[i].s, tol, flags);
            ptr[i] = &st[i];
            if (flags & MA_INIT_FMG) {
                // each solve's FMG-FAS iteration runs on its own before the
                // solves cycle together
                const ma_status fs = fmg_start(refs[i].s, refs[i].u, refs[i].f, st[i]);
                if (fs != MA_OK)
                    return fs;
            }
        }
        if (eng.reset_counters(-1) != MA_OK)
            return s0->fail(MA_ERR_DEVICE, eng.error());
        for (;;) {
            bool live = false;
            for (const SolveState &x : st)
                live |= x.phase != SolveState::DONE;
            if (!live)
                break;
            if (drive_step(eng, ptr, false, true) != MA_OK)
                return s0->fail(MA_ERR_DEVICE, eng.error());
        }
        std::vector<unsigned long long> nc, fb;
        if (eng.read_counters(nc, fb) != MA_OK)
            return s0->fail(MA_ERR_DEVICE, eng.error());
        double psec = 0.0, pbytes = 0.0;
        int plaunch = 0;
        if (s0->p.profile)
            eng.take_profile(&psec, &plaunch, &pbytes);
        const double t1 = now_seconds();
        for (int i = 0; i < m; ++i) {
            SolveState &x = st[i];
            x.rep.smooth_seconds = psec;
            x.rep.smooth_launches = plaunch;
            x.rep.smooth_bytes = pbytes;
            x.rep.nonconvex = (long long)nc[i] + x.fmg_nonconvex;
            x.rep.fp64_fallbacks = (long long)fb[i];
            x.rep.seconds = t1 - x.t0;
            if (reps)
                reps[base + i] = x.rep;
            if (x.status != MA_OK) {
                refs[i].s->err = x.err;
                if (first == MA_OK)
                    first = x.status;
            }
        }
    }
    return first;
}

ma_status ma_batch_create(int max_solves, void *hip_stream, ma_batch **out)
{
    if (!out || max_solves < 1 || max_solves > kMaxGrids)
        return MA_ERR_ARG;
    ma_batch *b = new ma_batch();
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->refs.resize(max_solves);
    b->st.resize(max_solves);
    b->used.assign(max_solves, 0);
    *out = b;
    return MA_OK;
}

void ma_batch_destroy(ma_batch *b) { delete b; }

const char *ma_batch_last_error(const ma_batch *b) { return b ? b->err.c_str() : "null batch"; }

ma_status ma_batch_add(ma_batch *b, ma_solver *s, double *u, const double *f, double tol,
                       unsigned flags, int *slot_out)
{
    if (!b || !s || !u || !f || !slot_out)
        return MA_ERR_ARG;
    if ((flags & MA_INIT_POISSON) && (flags & MA_INIT_FMG))
        return b->fail(MA_ERR_ARG, "MA_INIT_POISSON and MA_INIT_FMG exclude each other");
    int slot = -1;
    for (size_t i = 0; i < b->used.size(); ++i)
        if (!b->used[i]) {
            slot = int(i);
            break;
        }
    if (slot < 0)
        return b->fail(MA_ERR_ARG, "no free slot");
    for (size_t i = 0; i < b->used.size(); ++i)
        if (b->used[i] && b->refs[i].s == s)
            return b->fail(MA_ERR_ARG, "this solver already holds a slot");
    if (!b->any())
        b->graphs = s->p.graphs != 0;
    b->refs[slot].s = s;
    b->refs[slot].u = u;
    b->refs[slot].f = f;
    const ma_status st = b->eng.set(b->refs, b->stream, b->graphs, false);
    if (st != MA_OK) {
        b->refs[slot] = SolveRef();
        if (b->any())
            (void)b->eng.set(b->refs, b->stream, b->graphs, false);
        return b->fail(st, b->eng.error());
    }
    start_state(b->st[slot], s, tol, flags);
    if (flags & MA_INIT_FMG) {
        const ma_status fs = fmg_start(s, u, f, b->st[slot]);
        if (fs != MA_OK) {
            b->refs[slot] = SolveRef();
            if (b->any())
                (void)b->eng.set(b->refs, b->stream, b->graphs, false);
            return b->fail(fs, s->err);
        }
    }
    b->used[slot] = 1;
    if (b->eng.reset_counters(slot) != MA_OK)
        return b->fail(MA_ERR_DEVICE, b->eng.error());
    *slot_out = slot;
    return MA_OK;
}

ma_status ma_batch_tick(ma_batch *b, int *done_out)
{
    if (!b)
        return MA_ERR_ARG;
    const int S = int(b->used.size());
    if (done_out)
        for (int i = 0; i < S; ++i)
            done_out[i] = 0;
    std::vector<SolveState *> ptr(S, nullptr);
    std::vector<char> was_live(S, 0);
    bool live = false;
    for (int i = 0; i < S; ++i)
        if (b->used[i] && b->st[i].phase != SolveState::DONE) {
            ptr[i] = &b->st[i];
            was_live[i] = 1;
            live = true;
        }
    if (!live)
        return MA_OK;
    // the caller may have queued work for its solves since the last tick
    b->eng.mark_user();
    if (drive_step(b->eng, ptr) != MA_OK)
        return b->fail(MA_ERR_DEVICE, b->eng.error());
    bool any_done = false;
    for (int i = 0; i < S; ++i)
        any_done |= was_live[i] && b->st[i].phase == SolveState::DONE;
    if (!any_done)
        return MA_OK;
    std::vector<unsigned long long> nc, fb;
    if (b->eng.read_counters(nc, fb) != MA_OK)
        return b->fail(MA_ERR_DEVICE, b->eng.error());
    const double t1 = now_seconds();
    for (int i = 0; i < S; ++i)
        if (was_live[i] && b->st[i].phase == SolveState::DONE) {
            SolveState &x = b->st[i];
            x.rep.nonconvex = (long long)nc[i];
            x.rep.fp64_fallbacks = (long long)fb[i];
            x.rep.nonconvex += x.fmg_nonconvex;
            x.rep.seconds = t1 - x.t0;
            if (done_out)
                done_out[i] = x.status == MA_OK ? 1 : 2;
        }
    return MA_OK;
}

ma_status ma_batch_report(const ma_batch *b, int slot, ma_report *rep)
{
    if (!b || !rep || slot < 0 || slot >= int(b->used.size()) || !b->used[slot])
        return MA_ERR_ARG;
    *rep = b->st[slot].rep;
    return MA_OK;
}

ma_status ma_batch_remove(ma_batch *b, int slot)
{
    if (!b || slot < 0 || slot >= int(b->used.size()) || !b->used[slot])
        return MA_ERR_ARG;
    b->used[slot] = 0;
    b->refs[slot] = SolveRef();
    b->st[slot] = SolveState();
    if (b->any()) {
        const ma_status st = b->eng.set(b->refs, b->stream, b->graphs, false);
        if (st != MA_OK)
            return b->fail(st, b->eng.error());
    }
    return MA_OK;
}

} // extern "C"
