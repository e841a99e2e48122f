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

class Engine;

struct Level {
    int n = 0;
    double *u = nullptr;   // iterate (coarse levels; level 0 is the caller's array)
    double *b = nullptr;   // right-hand side (coarse levels)
    double *w = nullptr;   // injected fine approximation (coarse levels)
    double *r = nullptr;   // residual
    double *t = nullptr;   // out-of-place target of the block sweep
};

// FP32 inner hierarchy of the mixed-precision form (one per level).
struct MixedLevel {
    int n = 0;
    float *d = nullptr;    // correction delta
    float *b = nullptr;    // right-hand side of T(delta) = b
    float *w = nullptr;    // injected delta
    float *r = nullptr;    // residual of the inner problem
    double *U = nullptr;   // injected FP64 approximation (coarse levels)
};

size_t hierarchy_bytes(const ma_params *p);
// Doubles per colour of the colour-ordered right-hand side of an n grid
// (rows of the 4-colour sweep x 64 lanes).
inline long fs_colour_count(int n)
{
    const long gx = ((n + 1) / 2 + 63) / 64, gy = n - 1, gz = n / 2;
    return gx * gy * gz * 64;
}
// Largest n whose sweeps MA_SMOOTHER_AUTO runs as block sweeps (-1: none).
inline int block_limit(const ma_params &p) { return p.block_n == 0 ? 64 : p.block_n; }
size_t mixed_bytes(const ma_params *p);

hipError_t launch_fill(hipStream_t st, size_t count, double v, double *dst);
hipError_t launch_fill_u64(hipStream_t st, size_t count, unsigned long long v,
                           unsigned long long *dst);

double now_seconds();

// Sets the message ma_last_error(NULL) returns (calls without a solver).
void set_global_error(const std::string &why);

} // namespace mafas

struct ma_solver {
    ma_params p{};
    hipStream_t stream = nullptr;
    std::vector<mafas::Level> lv;
    double *R = nullptr;                  // Poisson right-hand side, finest level
    // The finest right-hand side in the order the 4-colour sweep visits it:
    // colour c, work item (row) q, lane t at fs[c * fs_cs + 64 q + t]
    // (FP64 4-colour solvers; filled by the engine when stale).
    double *fs = nullptr;
    long fs_cs = 0;
    double *partials = nullptr;           // norm partials of the single-grid kernels
    double *dsum = nullptr;
    unsigned long long *dcount = nullptr; // counter of the single-grid kernels
    double *hpin = nullptr;               // pinned host scalars
    unsigned long long *hpin_u64 = nullptr;
    std::vector<double *> owned;
    std::vector<void *> mixed_owned;
    std::vector<mafas::MixedLevel> mx;
    std::string err;
    mafas::Engine *eng = nullptr;         // batch-of-one engine of ma_solve / ma_vcycle
    // FMG: solvers that alias this hierarchy from level l down (no storage
    // of their own), so that a V-cycle rooted at level l runs through the
    // same engine code as the finest one
    std::vector<ma_solver *> views;

    ~ma_solver();
    ma_status fail(ma_status st, const std::string &msg);
    ma_status alloc(double **q, size_t count);
    ma_status allocate();
    bool use_block(int l) const;
    int rmode() const;
    // single-grid kernels behind the component entry points
    ma_status smooth(int l, double *u, const double *F, int count, int op);
    ma_status finish_norm(int n, double *l2);
    ma_status own_engine(mafas::Engine **out, double *u, const double *f);
    ma_solver *view(int l);
    // One FMG-FAS iteration (Algorithm 2) on u, whose interior is not read;
    // adds its non-certified updates, point updates and algorithmic bytes.
    ma_status fmg(double *u, const double *f, long long *nonconvex, double *updates,
                  double *bytes);
    ma_status mixed_allocate();
    void mixed_release();
};

namespace mafas {

// Progress of one solve driven tick by tick inside an Engine.
struct SolveState {
    enum Phase { INIT0, INIT, MAIN0, MAIN, DONE };
    Phase phase = MAIN0;
    double tol = 1e-8;
    double lin0 = 0.0;      // linear residual of the Poisson guess's start
    ma_status status = MA_OK;
    std::string err;
    ma_report rep{};
    double t0 = 0.0;        // start time (seconds)
    bool fmg = false;       // started by one FMG-FAS iteration: res0 is the
                            // residual of the zero-interior start, and the
                            // FMG iteration is the first cycle
    long long fmg_nonconvex = 0;
    // the phase's last two norms read (prev 0: only the phase's start is
    // known), for the guess whether the tick being read will stop the solve
    double last = 0.0, prev = 0.0;
    // the main phase's best residual so far and the cycles since it last
    // dropped below 0.9 x that best (three in a row: stagnation)
    double best = 0.0;
    int stall = 0;
};

// The FMG start of a solve (Section 4 protocol): zero the interior of u, take
// r^0 there, run one FMG-FAS iteration; st then continues at MAIN0.
ma_status fmg_start(ma_solver *s, double *u, const double *f, SolveState &st);

// One scheduling step over the engine's slots: the entry residuals of solves
// starting a phase, then one tick of every solve that is cycling (Poisson
// guess, FAS V-cycle or mixed correction).  states[i] may be null (empty
// slot).  Per-solve outcomes land in the states; the return value reports
// engine failures only.
// init_only: stop after the Poisson phases.
// ahead: let the engine queue a tick ahead of the stopping test (a closed
// set of solves: the caller adds or removes none between steps).
ma_status drive_step(Engine &eng, std::vector<SolveState *> &states, bool init_only = false,
                     bool ahead = false);

} // namespace mafas
