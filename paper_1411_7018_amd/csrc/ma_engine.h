// Batched execution engine.  Every level phase of the FAS V-cycle
// (Algorithm 1) -- a colour phase of a sweep, the residual, the FAS
// restriction, the prolongation, the norm -- runs for ALL solves of a batch
// as ONE launch over a device-resident table of grids.  The levels of every
// solve whose size is at most coarse_n (the coarse end of each V-cycle) run
// instead inside ONE kernel with one workgroup per solve, the phases
// separated by workgroup barriers.  One V-cycle (a "tick") therefore has a
// static shape that is captured once into a hipGraph and replayed; a change
// of the batch composition only rewrites the device tables.  A single solve
// is a batch of one.
#pragma once

#include "ma_fsweep.h"
#include "ma_runtime.h"

#include <cstddef>
#include <deque>
#include <vector>

namespace mafas {

constexpr int kMaxGrids = 64;          // grids (solve, level) per batched launch
// Sums of squares per slot held by the pinned norm ring: one per tick in
// flight (at most two queued entries of at most two ticks each).
constexpr int kNormRing = 4;
// z-stream sweeps (ma_zsweep.h): first shape index among the block-sweep
// configurations, and the smallest level that takes them when zsweep_n = 0
constexpr int kZsFirstConfig = 7;
constexpr int kZsweepAuto = 192;      // Monge-Ampere sweeps
constexpr int kZsweepAutoLap = 192;   // linear sweeps of the Poisson guess
constexpr int kDefaultMaxBlocks = 16384;
constexpr int kTailThreads = 512;      // threads of the coarse-level kernel
constexpr int kMaxTail = 6;            // levels per solve inside that kernel
constexpr int kTailLdsThreads = 1024;  // threads of its LDS form
constexpr int kTailLdsDoubles = 18432; // LDS of that form (144 KiB): levels 16, 8, 4, 2

// One grid of one solve inside a batched launch.  Every work item is one
// wavefront handling 64 nodes of one x-row (bx, by, bz) of a gx x gy x gz
// decomposition.  The items of a grid are ordered in y-strips of w rows
// walked along z: item - start = bx + gx*(jj + w*(bz + gz*strip)), by =
// strip*w + jj (items with by >= gy are idle), so the rows a stencil
// reads above, below and on both sides are fetched while they are still
// in the XCD's L2.
struct GridItem {
    int n;         // intervals per side of this grid
    int start;     // first work item
    int gx, gy, gz;
    int w;         // rows per y-strip
    int slot;      // solve index: norm and counter slot
    int pbase;     // first partial-sum slot (norm lists): gx*gy*gz slots
    double s;      // 1/h^2 of this grid
    double hk;     // h^2/2 (nonlinear update) or 1/(6s) (linear update)
    void *p[6];    // operands, meaning set by the list kind
};

// Work items of a grid, idle padding of the last y-strip included.
inline int padded_items(int gx, int gy, int gz, int w)
{
    return gx * ((gy + w - 1) / w) * w * gz;
}

// Lists live in one device buffer at a fixed stride of list_bytes(slots):
// the header followed by ngrids descriptors (g[] below is only the bound).
// stopped (every list header, at byte 8): bit s set when solve s has met its
// stopping test.  Work of such a solve is skipped, so a tick queued before
// the host has read the previous tick's norm does nothing for a solve that
// has stopped.  The mask sits beside ngrids and total, so a kernel reads it
// with the header it loads anyway.
struct BatchList {
    int ngrids;
    int total;     // work items over all grids
    unsigned long long stopped;
    GridItem g[kMaxGrids];
};
constexpr size_t list_bytes(int ngrids) { return 16 + sizeof(GridItem) * size_t(ngrids); }
static_assert(offsetof(BatchList, g) == 16, "list header is 16 bytes");

// The coarse levels of one solve: per level the descriptors of its sweep,
// residual, restriction (to the next level) and prolongation (from it).
struct TailLevel {
    GridItem sw, res, rst, pro;
};
// One grid of a fused residual-restriction launch: fine grid n (u, F) and
// the coarse arrays w, u, b of n/2; tiles of kRrTile^3 coarse nodes.
constexpr int kRrTile = 4;
struct RrGrid {
    const double *uf, *F;
    double *wc, *uc, *bc;
    int n;
    int tiles_x, tiles_y, tiles_z;
    int start;      // first tile of this grid in the launch
    int slot;       // solve index
    double s;       // 1/h^2 of the fine grid
};
struct RrList {
    int ngrids;
    int total;
    unsigned long long stopped;
    RrGrid g[kMaxGrids];
};
constexpr size_t rr_list_bytes(int ngrids) { return 16 + sizeof(RrGrid) * size_t(ngrids); }
static_assert(offsetof(RrList, g) == 16, "list header is 16 bytes");

// LDS form: offsets (in doubles) of each level's u, b, w, r in LDS, -1
// where the level has no such array (w above the first level, r on the
// coarsest).
struct TailLds {
    int u[kMaxTail], b[kMaxTail], w[kMaxTail], r[kMaxTail];
};
struct TailEntry {
    int nlev;
    int lds;        // 1: the levels fit kTailLdsDoubles
    int pad[2];
    TailLds L;
    TailLevel lv[kMaxTail];
};
struct TailList {
    int nsolves;
    int pad;
    unsigned long long stopped;
    TailEntry e[kMaxGrids];
};
constexpr size_t tail_bytes(int nsolves) { return 16 + sizeof(TailEntry) * size_t(nsolves); }
static_assert(offsetof(TailList, e) == 16, "list header is 16 bytes");

enum ListKind {
    LK_SWEEP,      // p: u, F                        items: rows of one colour
    LK_RESIDUAL,   // p: u, F, r                     items: interior rows
    LK_RESTRICT,   // p: uf, rf, wc, uc, bc          items: coarse rows (n = fine n)
    LK_PROLONG,    // p: uf, uc, wc                  items: fine interior rows
    LK_NORM,       // p: u, F, partials              items: interior rows x plane chunks
    LK_MSWEEP,     // p: d, b, U                     items: rows of one colour
    LK_MRESIDUAL,  // p: d, b, U, r                  items: interior rows
    LK_MRESTRICT,  // p: df, rf, Uc, wc, dc, bc      items: coarse rows (n = fine n)
    LK_MPROLONG,   // p: df, dc, wc                  items: fine interior rows
    LK_INJECT,     // p: Uf, Uc                      items: coarse rows (n = fine n)
    LK_ACCUM,      // p: u64, d                      items: interior rows
    LK_ZERO,       // p: d (FP32)                    items: all rows
    LK_RES32,      // p: u64, f, b0, partials        items: interior rows
};

// planes per work item of a norm list (a lane walks them along z)
constexpr int kNormPlanes = 8;
void item_dims(int kind, int order, int n, int *gx, int *gy, int *gz);

// blocks: grid size (a multiple of 8; blocks are split evenly over the XCDs)
hipError_t launch_batched(hipStream_t st, int kind, int op, int order, int color, int rmode,
                          const BatchList *dlist, int blocks, unsigned long long *ncount,
                          unsigned long long *nfall);
// Where the norm reduction puts each solve's sum of squares (see
// k_batched_reduce): sum and stamp are pinned host rings of 2 * kMaxGrids
// entries (device aliases), seq and thr per-slot device arrays.  base is the
// device list table and stop points into it: stop[0] list headers follow,
// as byte offsets from base, whose stopped masks a stopping solve sets.
struct NormRing {
    double *sum;
    unsigned *stamp;
    unsigned *seq;
    const double *thr;
    char *base;
    const unsigned *stop;
};
// Thresholds to arm (k_arm), at most kMaxGrids per launch.
struct ArmSet {
    int count;
    int slot[kMaxGrids];
    double thr[kMaxGrids];
};
// one block per grid of the norm list (grids = its grid count)
hipError_t launch_batched_reduce(hipStream_t st, const BatchList *dlist, int grids,
                                 const double *partials, const NormRing &ring);
// base, stop: the list table and its header offsets as in NormRing, or null
// before any list exists.
hipError_t launch_arm(hipStream_t st, const ArmSet &a, double *thr, char *base,
                      const unsigned *stop);
// Largest sum of squares x >= 0 of an n grid whose norm sqrt(x / n^3), as
// the engine computes it, is at most c (-1 when c is negative or NaN).
double sum_threshold(double c, int n);
// fs = F in the order of the 4-colour sweep rows of an n grid (ma_solver::fs)
hipError_t launch_fsplit(hipStream_t st, int n, const double *F, double *fs, long cs);
// block sweeps of an FsList (ma_fsweep.h): cfg block shape, blocks >= tiles;
// prolong: a z-stream shape whose grids carry the coarse u and w (cu, cw)
// and add the interpolated coarse correction to u_in as they read it
hipError_t launch_bsweep(hipStream_t st, int op, int cfg, const FsList *L, int blocks,
                         unsigned long long *nonconvex, bool prolong = false);
// whether block shape cfg is a z-stream shape
bool bsweep_is_zstream(int cfg);
void bsweep_grid(int cfg, int n, const double *uin, double *uout, const double *F, int op,
                 int slot, FsGrid *G);
// one workgroup per TailList entry (blocks >= entries); mode: Engine::Mode
hipError_t launch_tail(hipStream_t st, int mode, int order, int rmode, const TailList *T,
                       int blocks, int nu1, int nu2, int nu0, unsigned long long *ncount,
                       unsigned long long *nfall);
// fused residual + restriction (op: OP_MA / OP_LAP), one block per tile
hipError_t launch_rrestrict(hipStream_t st, int op, int rmode, const RrList *L, int blocks);
// the LDS form (MODE_MA, MODE_LAP; every entry with lds = 1)
hipError_t launch_tail_lds(hipStream_t st, int mode, int order, int rmode, const TailList *T,
                           int blocks, int nu1, int nu2, int nu0, unsigned long long *ncount);

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
    // its work on.  All solvers must share nu1, nu2, nu0, order, restriction,
    // precision, inner_cycles, coarse_n, max_blocks, strip_rows, smoother,
    // tile_config and block_n.  graphs: replay ticks from captured hipGraphs.
    ma_status set(const std::vector<SolveRef> &solves, hipStream_t user, bool graphs,
                  bool profile);
    // One V-cycle (MA, LAP) or one outer correction (MIXED) of every active
    // solve, then its discrete L2 residual norm into norms[i].  The solves
    // run unconditionally (their stopping thresholds are disarmed).
    ma_status tick(Mode mode, const std::vector<char> &active, std::vector<double> &norms);
    // The residual norms alone (MIXED: also stores r64 in FP32 for the next
    // correction).
    ma_status norms_only(Mode mode, const std::vector<char> &active, std::vector<double> &norms);
    // A tick for the cycle driver.  thr[i] arms solve i's stopping threshold
    // on its sum of squares (sum_threshold; negative: none): the tick that
    // meets it sets the solve's device halt flag.  ahead: queue one more tick
    // of the same solves before waiting for this one, so the GPU does not
    // idle while the host reads the norms; a later tick_ahead call with
    // these solves consumes it, and a solve that stopped skips it on the
    // device.  The caller queues ahead only while no solve can stop for a
    // reason the device does not see (a cycle limit).  pair: what is queued
    // ahead may be two ticks in one graph (one graph boundary instead of
    // two), or one tick behind such a pair while its first tick is read; the
    // caller asks for it only while no solve can stop for such a reason at
    // the tick read now or the next.
    ma_status tick_ahead(Mode mode, const std::vector<char> &active, const std::vector<double> &thr,
                         bool ahead, std::vector<double> &norms, bool pair = false);
    // Wait for ticks still queued ahead (each solve in them must have stopped).
    ma_status settle();
    // Ticks queued and not yet read.
    int pending() const { return int(fifo_.size()); }
    // Drop queued ticks after a failed step and resynchronise the host's
    // view of the stopping state with the device.
    ma_status abandon();
    // Work may have been queued on the caller's stream since the engine's
    // last launch: the next launch orders itself after it.  set() implies
    // this; within one call, launches order after each other on the engine
    // stream and skip the cross-stream wait.
    void mark_user() { user_dirty_ = true; }
    // The device halt flag of solve i as last seen by the host.
    bool halted(int i) const { return halted_[i] != 0; }
    ma_status reset_counters(int slot);  // slot < 0: all
    // The right-hand side behind solve i's finest level changed (its
    // colour-ordered copy is rebuilt before the next tick that reads it).
    void rhs_changed(int i);
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

    ma_status fail(ma_status st, const std::string &m)
    {
        err_ = m;
        return st;
    }

  private:
    ma_status rebuild(Mode mode, const std::vector<char> &active);
    ma_status enqueue(Mode mode, bool cycle);
    ma_status launch(Mode mode, bool cycle, const std::vector<char> &active, int ticks = 1);
    ma_status collect(std::vector<double> &norms);
    ma_status plain(Mode mode, bool cycle, const std::vector<char> &active,
                    std::vector<double> &norms);
    void arm(int slot, double thr);
    ma_status flush_arms();
    ma_status upload();
    ma_status refresh_fs(Mode mode, const std::vector<char> &active);
    void drop_graphs();
    const double *level_u(int i, int l, Mode mode) const;
    const double *level_F(int i, int l, Mode mode) const;
    GridItem grid(int kind, int i, int l, Mode mode) const;
    int levels(int i) const;
    int multiblock_levels(int i) const;  // leading levels with n > coarse_n
    ma_status capture(int slot, Mode mode, int ticks);
    std::vector<int> shape() const;
    ma_status prof_mark();

    std::vector<SolveRef> solves_;
    hipStream_t user_ = nullptr, stream_ = nullptr;
    hipEvent_t ev_in_ = nullptr;
    bool user_dirty_ = true;
    bool graphs_ = true, profile_ = false;
    std::string err_;
    int D_ = 0;      // multi-block depth of the active solves
    int Dall_ = 0;   // full depth of the active solves
    int nu1_ = 2, nu2_ = 2, nu0_ = 1, order_ = 0, rmode_ = 0, inner_ = 2;
    int coarse_n_ = 16, max_blocks_ = kDefaultMaxBlocks, strip_rows_ = 0;
    int smoother_ = MA_SMOOTHER_AUTO, tile_config_ = 0, block_n_ = 0, zsweep_n_ = 0;
    bool fuse_prolong_ = true;
    int strip_width(int gy) const;
    // sweeps of a multi-block n grid as block sweeps, and among them as
    // z-stream sweeps (the mode sets the automatic choice)
    bool block_level(int n, Mode mode) const;
    bool zs_level(int n, Mode mode) const;

    std::vector<char> hbuf_;               // host copy of the lists and the tail table
    std::vector<size_t> loff_;             // byte offset of each list
    std::vector<int> lng_;                 // grids per list
    std::vector<int> lgrid_;               // blocks per list launch (0: never any grid)
    size_t toff_ = 0;                      // byte offset of the tail table
    int tail_blocks_ = 0;                  // blocks of the tail launch (0: no tail)
    bool tail_lds_ = false;                // the tail launch is the LDS form
    char *dl_ = nullptr;                   // device lists
    size_t dl_cap_ = 0;
    char *hstage_ = nullptr;               // pinned staging for uploads
    size_t hstage_cap_ = 0;
    bool mixed_ = false;

    std::vector<std::vector<int>> swd_, swu_;  // [depth][sweep] list indices
    // Block sweeps: [depth][sweep] index of the first of two FsLists (u -> t,
    // t -> u) running sweeps 2q and 2q + 1 together, or -1 (colour phases);
    // entries at odd sweeps are unused.
    std::vector<std::vector<int>> bsd_, bsu_;
    std::vector<size_t> fsoff_;            // byte offset of each FsList
    std::vector<int> fsblocks_;            // blocks per FsList launch (0: no grid)
    std::vector<int> fscfg_;               // block shape per FsList
    std::vector<char> fspro_;              // the FsList's sweep also prolongs
    std::vector<char> pro_fused_;          // [depth] prolongation inside the up-leg's first sweep
    size_t fs_stride_ = 0;
    std::vector<int> res_, rst_, pro_, inj_;
    std::vector<const double *> fs_src_;   // right-hand side held in each solve's fs
    // fused residual-restriction list of each depth (-1: separate launches)
    std::vector<int> rr_;
    std::vector<size_t> rroff_;            // byte offset of each RrList
    std::vector<int> rrblocks_;            // blocks per RrList launch
    size_t rr_stride_ = 0;
    int norm_ = -1, accum_ = -1, zero_ = -1;

    double *partials_ = nullptr;
    size_t partials_cap_ = 0;
    // Norm ring (k_batched_reduce): hnorm_ / hstamp_ pinned coherent host
    // memory, kNormRing * kMaxGrids entries each, dnorm_ / dstamp_ their
    // device aliases; dseq_, dthr_ per-slot device state.
    double *dnorm_ = nullptr, *hnorm_ = nullptr;
    unsigned *dstamp_ = nullptr, *hstamp_ = nullptr, *dseq_ = nullptr;
    double *dthr_ = nullptr;
    size_t stoff_ = 0;   // byte offset of the header-offset table in the lists
    // host view of the device state: sums consumed per slot, armed
    // thresholds and halt flags, and thresholds queued for the next launch
    std::vector<unsigned> seq_ = std::vector<unsigned>(kMaxGrids, 0u);
    std::vector<double> thr_dev_ = std::vector<double>(kMaxGrids, -1.0);
    std::vector<char> halted_ = std::vector<char>(kMaxGrids, 0);
    std::vector<char> armq_ = std::vector<char>(kMaxGrids, 0);
    std::vector<double> armv_ = std::vector<double>(kMaxGrids, -1.0);
    // queued entries (one graph of one or two ticks), oldest first, and
    // spare events.  When an entry's event has completed, the ring entries
    // its ticks may have written are copied out (sum[j * kMaxGrids + i],
    // stamp likewise, for its tick j and slot i): a later entry may reuse
    // them before the host has read the entry's last tick.
    struct Pending {
        Mode mode;
        bool cycle;
        std::vector<char> active;
        hipEvent_t ev;
        size_t nev;     // profile events recorded by the tick
        int ticks = 1;  // ticks in the entry
        int done = 0;   // ticks the host has read
        bool synced = false;
        std::vector<double> sum;
        std::vector<unsigned> stamp;
    };
    std::deque<Pending> fifo_;
    std::vector<hipEvent_t> evpool_;
    hipStream_t side_ = nullptr;  // counter reads while a skipped tick is queued
    unsigned long long *dcount_ = nullptr, *dfall_ = nullptr, *hcount_ = nullptr;

    Mode built_mode_ = MODE_MA;
    std::vector<char> built_active_;
    bool built_ = false;
    // Captured ticks, one slot per mode; slot mode + 3 is the profiled form:
    // the tick split into segments at the finest-level sweep boundaries, so
    // the timing events are recorded on the stream between segment launches;
    // slot mode + 6 is two ticks in one graph.  A graph is replayed only
    // while the launch shapes it was captured with (depths, list table
    // address and stride, blocks per launch) still hold.
    static constexpr int kSlots = 9;
    std::vector<hipGraphExec_t> gseg_[kSlots];
    std::vector<int> graph_shape_[kSlots];
    const char *graph_dl_[kSlots] = {};
    size_t stride_ = 0;                  // bytes per list: list_bytes(slots)
    bool seg_capture_ = false;           // prof_mark() cuts the capture
    std::vector<hipGraph_t> seg_tmp_;

    std::vector<hipEvent_t> pev_;          // profile event pairs (finest sweeps)
    size_t pev_used_ = 0;
    double prof_seconds_ = 0.0, prof_bytes_ = 0.0;
    int prof_launches_ = 0;
    double prof_bytes_tick_ = 0.0;
    int prof_launches_tick_ = 0;
};

} // namespace mafas
