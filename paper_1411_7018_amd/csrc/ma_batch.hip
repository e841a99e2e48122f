// Batched solves and the resident batch used for continuous serving.
#include "ma_runtime.h"

#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

using namespace mafas;

struct ma_batch {
    struct Slot {
        bool active = false;
        ma_solver *s = nullptr;
        double *u = nullptr;
        const double *f = nullptr;
        double tol = 0.0;
        ma_report rep{};
        std::chrono::steady_clock::time_point t0;
    };
    hipStream_t stream = nullptr;
    std::vector<Slot> slots;
    std::string err;
    ma_status fail(ma_status st, const std::string &m)
    {
        err = m;
        return st;
    }
};

extern "C" {

ma_status ma_solve_batch(ma_solver *const *solvers, double *const *u, const double *const *f,
                         int count, double tol, unsigned flags, ma_report *reps)
{
    if (count < 0 || (count > 0 && (!solvers || !u || !f)))
        return MA_ERR_ARG;
    ma_status first = MA_OK;
    for (int i = 0; i < count; ++i) {
        if (!solvers[i])
            return MA_ERR_ARG;
        ma_report local;
        const ma_status st = ma_solve(solvers[i], u[i], f[i], tol, flags, reps ? &reps[i] : &local);
        if (st != MA_OK && first == MA_OK)
            first = st;
    }
    return first;
}

ma_status ma_batch_create(int max_solves, void *hip_stream, ma_batch **out)
{
    if (!out || max_solves < 1)
        return MA_ERR_ARG;
    ma_batch *b = new ma_batch();
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->slots.resize(max_solves);
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
    int slot = -1;
    for (size_t i = 0; i < b->slots.size(); ++i)
        if (!b->slots[i].active) {
            slot = int(i);
            break;
        }
    if (slot < 0)
        return b->fail(MA_ERR_ARG, "no free slot");
    ma_batch::Slot &sl = b->slots[slot];
    sl = ma_batch::Slot();
    sl.s = s;
    sl.u = u;
    sl.f = f;
    sl.tol = tol > 0.0 ? tol : s->p.tol;
    sl.t0 = std::chrono::steady_clock::now();
    s->stream = b->stream;
    s->stats = Stats();
    ma_report &r = sl.rep;
    std::memset(&r, 0, sizeof(r));
    ma_status st = launch_fill_u64(b->stream, 1, 0ull, s->dcount) == hipSuccess ? MA_OK
                                                                                  : MA_ERR_DEVICE;
    if (st == MA_OK && (flags & MA_INIT_POISSON))
        st = s->poisson_init(u, f, &r.init_cycles);
    if (st == MA_OK) {
        s->bind_finest(u, f);
        st = s->norm(OP_MA, u, f, &r.res0);
    }
    if (st != MA_OK)
        return b->fail(st, s->err);
    r.res = r.res0;
    sl.active = true;
    *slot_out = slot;
    return MA_OK;
}

ma_status ma_batch_tick(ma_batch *b, int *done_out)
{
    if (!b)
        return MA_ERR_ARG;
    ma_status first = MA_OK;
    for (size_t i = 0; i < b->slots.size(); ++i) {
        ma_batch::Slot &sl = b->slots[i];
        if (done_out)
            done_out[i] = 0;
        if (!sl.active || sl.rep.converged)
            continue;
        ma_solver *s = sl.s;
        ma_report &r = sl.rep;
        ma_status st = MA_OK;
        if (r.res0 == 0.0) {
            r.converged = 1;
        } else {
            s->bind_finest(sl.u, sl.f);
            st = s->vcycle(0, OP_MA);
            if (st == MA_OK)
                st = s->norm(OP_MA, sl.u, sl.f, &r.res);
            if (st == MA_OK) {
                if (r.cycles < 64)
                    r.history[r.cycles] = r.res;
                r.cycles += 1;
                r.rel_res = r.res / r.res0;
                if (!std::isfinite(r.res))
                    st = MA_ERR_NONFINITE;
                else if (r.res <= sl.tol * r.res0)
                    r.converged = 1;
                else if (r.cycles >= s->p.max_cycles)
                    st = MA_ERR_NOT_CONVERGED;
            }
        }
        r.point_updates = s->stats.updates;
        r.alg_bytes = s->stats.bytes;
        r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - sl.t0).count();
        if (st != MA_OK && first == MA_OK) {
            first = st;
            b->err = s->err;
        }
        if (done_out && (r.converged || st != MA_OK))
            done_out[i] = st == MA_OK ? 1 : 2;
    }
    return first;
}

ma_status ma_batch_report(const ma_batch *b, int slot, ma_report *rep)
{
    if (!b || !rep || slot < 0 || slot >= int(b->slots.size()) || !b->slots[slot].active)
        return MA_ERR_ARG;
    *rep = b->slots[slot].rep;
    return MA_OK;
}

ma_status ma_batch_remove(ma_batch *b, int slot)
{
    if (!b || slot < 0 || slot >= int(b->slots.size()) || !b->slots[slot].active)
        return MA_ERR_ARG;
    b->slots[slot] = ma_batch::Slot();
    return MA_OK;
}

} // extern "C"
