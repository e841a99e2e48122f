// Batched execution engine.  Every level phase of the FAS V-cycle
// (Algorithm 1) -- a colour phase of a sweep, the residual, the FAS
// restriction, the prolongation, the norm -- runs for ALL solves of a batch
// as ONE launch over a device-resident table of grids.  The launches use a
// fixed number of persistent blocks, so one V-cycle (a "tick") has a static
// shape that is captured once into a hipGraph and replayed; a change of the
// batch composition only rewrites the device tables.  A single solve is a
// batch of one.
#pragma once

#include "ma_runtime.h"

#include <vector>

namespace mafas {

constexpr int kMaxGrids = 64;         // grids (solve, level) per batched launch
constexpr int kPersistBlocks = 4096;  // blocks of 64 threads in every batched launch

// One grid of one solve inside a batched launch.  The grid's work items are
// [start, start + gx*gy*gz), item = bx + gx*(by + gy*bz); every item is one
// wavefront handling 64 nodes of one x-row.
struct GridItem {
    int n;         // intervals per side of this grid
    int start;     // first work item
    int gx, gy;    // item decomposition (gz implied by the next start)
    int slot;      // solve index: norm and counter slot
    int pbase;     // first partial-sum slot (norm lists)
    double s;      // 1/h^2 of this grid
    double hk;     // h^2/2 (nonlinear update) or 1/(6s) (linear update)
    void *p[6];    // operands, meaning set by the list kind
};

// Lists live in one device buffer at a fixed stride of list_bytes(slots):
// the header followed by ngrids descriptors (g[] below is only the bound).
struct BatchList {
    int ngrids;
    int total;     // work items over all grids
    int pad[2];
    GridItem g[kMaxGrids];
};
constexpr size_t list_bytes(int ngrids) { return 16 + sizeof(GridItem) * size_t(ngrids); }

enum ListKind {
    LK_SWEEP,      // p: u, F                        items: rows of one colour
    LK_RESIDUAL,   // p: u, F, r                     items: interior rows
    LK_RESTRICT,   // p: uf, rf, wc, uc, bc          items: coarse rows (n = fine n)
    LK_PROLONG,    // p: uf, uc, wc                  items: fine interior rows
    LK_NORM,       // p: u, F, partials              items: interior rows
    LK_MSWEEP,     // p: d, b, U                     items: rows of one colour
    LK_MRESIDUAL,  // p: d, b, U, r                  items: interior rows
    LK_MRESTRICT,  // p: df, rf, Uc, wc, dc, bc      items: coarse rows (n = fine n)
    LK_MPROLONG,   // p: df, dc, wc                  items: fine interior rows
    LK_INJECT,     // p: Uf, Uc                      items: coarse rows (n = fine n)
    LK_ACCUM,      // p: u64, d                      items: interior rows
    LK_ZERO,       // p: d (FP32)                    items: all rows
    LK_RES32,      // p: u64, f, b0, partials        items: interior rows
};

void item_dims(int kind, int order, int n, int *gx, int *gy, int *gz);

hipError_t launch_batched(hipStream_t st, int kind, int op, int order, int color, int rmode,
                          const BatchList *dlist, unsigned long long *ncount,
                          unsigned long long *nfall);
hipError_t launch_batched_reduce(hipStream_t st, const BatchList *dlist, const double *partials,
                                 double *out);

struct SolveRef {
    ma_solver *s = nullptr;
    double *u = nullptr;
    const double *f = nullptr;
};

class Engine {
  public:
    enum Mode { MODE_MA = 0, MODE_LAP = 1, MODE_MIXED = 2 };

    Engine() = default;
    ~Engine();
    Engine(const Engine &) = delete;
    Engine &operator=(const Engine &) = delete;

    // Define the solves (at most kMaxGrids) and the stream the caller orders
    // its work on.  All solvers must share nu1, nu2, nu0, order, restriction
    // and precision.  graphs: replay ticks from captured hipGraphs.
    ma_status set(const std::vector<SolveRef> &solves, hipStream_t user, bool graphs,
                  bool profile);
    // One V-cycle (MA, LAP) or one outer correction (MIXED) of every active
    // solve, then its discrete L2 residual norm into norms[i].
    ma_status tick(Mode mode, const std::vector<char> &active, std::vector<double> &norms);
    // The residual norms alone (MIXED: also stores r64 in FP32 for the next
    // correction).
    ma_status norms_only(Mode mode, const std::vector<char> &active, std::vector<double> &norms);
    ma_status reset_counters(int slot);  // slot < 0: all
    ma_status read_counters(std::vector<unsigned long long> &nonconvex,
                            std::vector<unsigned long long> &fallbacks);
    // Work of one tick of mode for solve i: point updates and algorithmic bytes.
    void tick_cost(Mode mode, int i, double *updates, double *bytes) const;
    // profile: finest-level smoothing time, launches and bytes since the last call
    void take_profile(double *seconds, int *launches, double *bytes);
    const std::string &error() const { return err_; }
    size_t size() const { return solves_.size(); }
    const SolveRef &ref(int i) const { return solves_[i]; }
    hipStream_t user() const { return user_; }
    bool mixed() const { return mixed_; }

  private:
    ma_status fail(ma_status st, const std::string &m)
    {
        err_ = m;
        return st;
    }
    ma_status rebuild(Mode mode, const std::vector<char> &active);
    ma_status enqueue(Mode mode, bool cycle);
    ma_status run(Mode mode, bool cycle, const std::vector<char> &active,
                  std::vector<double> &norms);
    ma_status upload();
    void drop_graphs();
    const double *level_u(int i, int l, Mode mode) const;
    const double *level_F(int i, int l, Mode mode) const;
    GridItem grid(int kind, int i, int l, Mode mode) const;

    std::vector<SolveRef> solves_;
    hipStream_t user_ = nullptr, stream_ = nullptr;
    hipEvent_t ev_in_ = nullptr;
    bool graphs_ = true, profile_ = false, fused_ = false;
    std::string err_;
    int D_ = 0;
    int nu1_ = 2, nu2_ = 2, nu0_ = 1, order_ = 0, rmode_ = 0, inner_ = 2;

    std::vector<char> hbuf_;               // packed host copy of the lists
    std::vector<size_t> loff_;             // byte offset of each list
    std::vector<int> lng_;                 // grids per list
    char *dl_ = nullptr;                   // packed device lists
    size_t dl_cap_ = 0;
    char *hstage_ = nullptr;               // pinned staging for uploads
    size_t hstage_cap_ = 0;
    bool mixed_ = false;

    std::vector<std::vector<int>> swd_, swu_;  // [depth][sweep] list indices
    std::vector<int> res_, rst_, pro_, inj_;
    int norm_ = -1, accum_ = -1, zero_ = -1;

    double *partials_ = nullptr;
    size_t partials_cap_ = 0;
    double *dnorm_ = nullptr, *hnorm_ = nullptr;
    unsigned long long *dcount_ = nullptr, *dfall_ = nullptr, *hcount_ = nullptr;

    Mode built_mode_ = MODE_MA;
    std::vector<char> built_active_;
    bool built_ = false;
    // Captured ticks, one slot per mode; slot mode + 3 is the profiled form:
    // the tick split into segments at the finest-level sweep boundaries, so
    // the timing events are recorded on the stream between segment launches.
    static constexpr int kSlots = 6;
    std::vector<hipGraphExec_t> gseg_[kSlots];
    int graph_D_[kSlots] = {-1, -1, -1, -1, -1, -1};
    const char *graph_dl_[kSlots] = {};
    size_t graph_stride_[kSlots] = {};   // list stride a graph was captured with
    size_t graph_nl_[kSlots] = {};       // list count a graph was captured with
    size_t stride_ = 0;                  // bytes per list: list_bytes(slots)
    bool seg_capture_ = false;           // prof_mark() cuts the capture
    std::vector<hipGraph_t> seg_tmp_;
    ma_status capture(int slot, Mode mode);

    std::vector<hipEvent_t> pev_;          // profile event pairs (finest sweeps)
    size_t pev_used_ = 0;
    double prof_seconds_ = 0.0, prof_bytes_ = 0.0;
    int prof_launches_ = 0;
    double prof_bytes_tick_ = 0.0;
    int prof_launches_tick_ = 0;
    ma_status prof_mark();
};

} // namespace mafas
