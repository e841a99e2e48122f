/*
 * ma.h -- C ABI of the MI355X FAS multigrid solver for the 3D Monge-Ampere
 * equation  det(D^2 u) = f > 0  in the unit cube,  u = g  on its boundary,
 * u convex  (Liu, Froese, Oberman, Xiao, "A multigrid scheme for 3D
 * Monge-Ampere equations", Section 1, eqs. 1.1-1.2).
 *
 * Grid and layout (Section 2): h = 1/n, nodes x_i = i h, i = 0..n in each
 * direction.  Every grid function is one contiguous array of (n+1)^3 doubles
 * in DEVICE memory, x fastest: index(i,j,k) = i + (n+1)*(j + (n+1)*k).  Nodes
 * with any index in {0, n} are Dirichlet nodes: the solver reads them and
 * never writes them.
 *
 * Ownership: the caller owns u and f (device pointers, e.g. torch tensors);
 * a solver owns every scratch array of its multigrid hierarchy from
 * ma_create to ma_destroy.  All device work is ordered on the HIP stream
 * given to ma_create (or ma_set_stream); functions that return a number to
 * the host (norms, reports) synchronise that stream.
 *
 * Errors: no function throws or aborts.  Each returns an ma_status and keeps
 * a message readable through ma_last_error(solver).  A solver is not
 * thread-safe: use it from one host thread at a time.
 */
#ifndef MA_H
#define MA_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ma_solver ma_solver;
typedef struct ma_batch ma_batch;

typedef enum {
    MA_OK = 0,
    MA_ERR_ARG = 1,            /* invalid argument (sizes, null pointers)      */
    MA_ERR_OOM = 2,            /* device allocation failed                     */
    MA_ERR_DEVICE = 3,         /* a HIP call or kernel launch failed           */
    MA_ERR_NOT_CONVERGED = 4,  /* max_cycles spent, or the residual stagnated
                                  above the tolerance; the report is filled    */
    MA_ERR_NONFINITE = 5       /* a residual norm became NaN or Inf            */
} ma_status;

typedef enum { MA_FP64 = 0, MA_MIXED = 1 } ma_precision;

/* Multicolour orderings of the nonlinear Gauss-Seidel sweep.  The 19-point
 * stencil (Section 2, eqs. 2.1-2.6) needs four or more colours to decouple:
 *   MA_COLOR4: colour = ((i+j) mod 2) + 2 ((i+k) mod 2), phases 0..3;
 *   MA_COLOR8: colour = (i mod 2) + 2 (j mod 2) + 4 (k mod 2), phases 0..7. */
typedef enum { MA_COLOR4 = 0, MA_COLOR8 = 1 } ma_order;

/* Residual restriction I_h^H of Algorithm 1 step 3.  Section 3 gives the
 * 7-point half-weighting and allows other operators; with multicolour
 * Gauss-Seidel the half-weighted V-cycle does not contract, so full
 * weighting (27 points, tensor product of 1/4, 1/2, 1/4) is the default. */
typedef enum { MA_RESTRICT_FULL = 0, MA_RESTRICT_HALF = 1 } ma_restriction;

/* Smoother kernel selection.  Every choice computes bitwise the same sweep
 * (the same pointwise update on the same neighbour values); they differ in
 * data movement.  The block sweep runs the four colour phases of one sweep
 * in one launch: each workgroup updates a block of the grid with a halo in
 * LDS, recomputing the halo's updates, out of place into a second array
 * (pairs of sweeps go u -> t -> u; an odd last sweep runs per colour).  It
 * applies to the 4-colour ordering in MA_FP64 only. */
typedef enum {
    MA_SMOOTHER_AUTO = 0,      /* block sweeps on levels with n <= block_n that
                                  have more than coarse_n intervals, one
                                  launch per colour phase elsewhere           */
    MA_SMOOTHER_COLOR = 1,     /* one in-place launch per colour phase          */
    MA_SMOOTHER_FUSED = 2      /* block sweeps on every level                    */
} ma_smoother;

/* ma_solve flag: replace the interior of u by the initial guess that solves
 * Lap_h u0 = 3 f^{1/3} with the Dirichlet data of u (7-point Laplacian,
 * linear V-cycles with the same ordering and transfers). */
#define MA_INIT_POISSON 1u

/* ma_solve flag: the protocol of Section 4 -- r^0 is the residual of the
 * start that holds the Dirichlet data of u and zero inside, one FMG-FAS
 * iteration (Algorithm 2, see ma_fmg) is the first cycle, FAS V-cycles
 * follow until the tolerance.  Excludes MA_INIT_POISSON. */
#define MA_INIT_FMG 2u

typedef struct {
    int n;                 /* intervals per side, n >= 2; grid (n+1)^3, h = 1/n  */
    int nu1, nu2, nu0;     /* pre-, post-smoothing sweeps, sweeps on the coarsest
                              grid (Algorithm 1; Section 4 uses 2, 2, 1)         */
    int order;             /* ma_order                                           */
    int restriction;       /* ma_restriction                                     */
    int precision;         /* ma_precision                                       */
    int smoother;          /* ma_smoother                                        */
    int max_cycles;        /* V-cycles (MA_FP64) or outer corrections (MA_MIXED) */
    double tol;            /* default relative discrete-L2 residual (Section 4)  */
    double init_tol;       /* relative linear residual for MA_INIT_POISSON       */
    int init_max_cycles;   /* cap on the linear V-cycles of MA_INIT_POISSON      */
    int inner_cycles;      /* MA_MIXED: FP32 V-cycles per outer correction       */
    int profile;           /* 1: time finest-level smoothing with HIP events     */
    int tile_config;       /* block sweep shape: 0 automatic, 1..7 fixed (8^3
                              blocks of 256, 512, 1024 threads; 16x8x4 of 256;
                              16x16x8 of 512; 8x8x4 of 512, 256); 8..12 the
                              z-stream sweep's columns (32x26 of 1024, 512
                              threads, 32x26 with twice the chunks, 40x20,
                              32x24 with one colour per wavefront); on
                              z-stream levels 0 picks 32x26 or 32x24 by a
                              model of the chunks' rounds                     */
    int block_n;           /* MA_SMOOTHER_AUTO: block sweeps on levels with
                              n <= block_n; 0 automatic (64), -1 never          */
    int graphs;            /* 1: replay each cycle from a captured hipGraph      */
    int coarse_n;          /* levels with n <= coarse_n (0..32) run inside one
                              single-workgroup kernel per solve; 0: off         */
    int max_blocks;        /* cap on the blocks of one batched launch (multiple
                              of 8, 0 automatic = 16384)                         */
    int strip_rows;        /* x-rows per y-strip in the work order of a batched
                              launch (strips are walked along z; 0 automatic)    */
    int zsweep_n;          /* MA_SMOOTHER_AUTO, 4-colour FP64: z-stream sweeps
                              (all four colour phases of a sweep in one launch,
                              each workgroup walking a column of the grid plane
                              by plane, out of place) on levels with
                              n >= zsweep_n; 0 automatic, -1 never              */
    int fuse_prolong;      /* FP64 levels with z-stream post-smoothing pairs:
                              0 the first post-smoothing sweep also applies the
                              coarse-grid correction (no separate prolongation
                              pass; bitwise the same result), -1 separate
                              prolongation pass                                */
} ma_params;

typedef struct {
    int cycles;            /* FAS V-cycles run (MA_MIXED: FP32 inner cycles);
                              with MA_INIT_FMG the FMG-FAS iteration counts as
                              the first (Section 4's 'Iter')                    */
    int outer;             /* MA_MIXED outer FP64 corrections, the FMG start
                              included (0 for MA_FP64)                           */
    int init_cycles;       /* linear V-cycles of the Poisson initial guess       */
    int converged;         /* 1 when res <= tol * res0                           */
    double res0;           /* discrete L2 residual sqrt(h^3 sum r^2) of u0       */
    double res;            /* final discrete L2 residual                         */
    double rel_res;        /* res / res0                                         */
    long long nonconvex;   /* point updates with F <= 0 or a non-SPD Hessian     */
    long long fp64_fallbacks; /* MA_MIXED nodes recomputed in FP64               */
    double seconds;        /* wall time of the call                              */
    double point_updates;  /* nonlinear GS point updates performed               */
    double alg_bytes;      /* algorithmic HBM bytes of the kernels launched      */
    double history[64];    /* residual after each cycle (first 64)              */
    /* params.profile = 1 only: finest-level smoother launches, their total
     * device time (HIP events on the solver's stream) and algorithmic bytes
     * (24 B per interior node per FP64 sweep: read u, read f, write u). */
    int smooth_launches;
    double smooth_seconds;
    double smooth_bytes;
} ma_report;

/* Fill p with the defaults for an n-interval grid: V(2,2), one coarsest
 * sweep, 4 colours, full weighting, FP64, auto smoother, 100 cycles,
 * tol 1e-8, Poisson guess to 1e-6 relative in at most 30 cycles, two FP32
 * cycles per mixed correction, hipGraph replay on. */
void ma_params_default(ma_params *p, int n);

/* Device bytes ma_create would allocate for p (0 if p is invalid).  Does not
 * allocate; used for admission against an HBM budget. */
size_t ma_footprint_bytes(const ma_params *p);

/* Number of multigrid levels for n: n_0 = n, n_{l+1} = n_l / 2 while n_l is
 * even and >= 4, so the coarsest grid has n_L = 2 (one unknown, h0 = 1/2 as
 * in Section 4) or an odd n_L >= 3.  Writes up to cap sizes into ns. */
int ma_levels(int n, int *ns, int cap);

/* Create a solver for p on the current HIP device; hip_stream is a
 * hipStream_t (NULL = default stream).  MA_ERR_ARG for invalid p,
 * MA_ERR_OOM when the hierarchy does not fit. */
ma_status ma_create(const ma_params *p, void *hip_stream, ma_solver **out);

/* Release the hierarchy; s may be NULL. */
void ma_destroy(ma_solver *s);

/* Message of the last failed call on s (or of the last failed ma_create when
 * s is NULL).  Valid until the next call on s. */
const char *ma_last_error(const ma_solver *s);

/* Order later work on another hipStream_t. */
ma_status ma_set_stream(ma_solver *s, void *hip_stream);

/* Change the launch shape of later cycles without touching the hierarchy:
 * coarse_n, max_blocks, strip_rows and block_n as in ma_params (the
 * autotuner's knobs).  The arithmetic, and so every result, is the same for
 * every value.  Errors: MA_ERR_ARG for values outside their ranges (nothing
 * changes). */
ma_status ma_retune(ma_solver *s, int coarse_n, int max_blocks, int strip_rows, int block_n);

/* The same for the smoother's shape: block_n, zsweep_n and tile_config as in
 * ma_params.  Results are unchanged by every value. */
ma_status ma_retune_smoother(ma_solver *s, int block_n, int zsweep_n, int tile_config);

/* Solve det(D^2 u) = f (Algorithm 1 repeated under the stopping rule of
 * Section 4): run V(nu1,nu2) cycles until the discrete L2 residual is
 * <= tol * res0 (tol <= 0 selects params.tol), res0 being the residual of
 * the initial guess.  u: device (n+1)^3, Dirichlet layer = g, interior = the
 * initial guess on entry (or replaced when flags has MA_INIT_POISSON) and
 * the solution on exit.  f: device (n+1)^3, interior read.  rep may be NULL.
 * Returns MA_ERR_NOT_CONVERGED when max_cycles run out, or when the residual
 * has failed to drop below 0.9 x its best value for three cycles in a row
 * while above the tolerance (it sits on the round-off floor: a start so
 * close to the solution that tol * res0 lies under the floor); u holds the
 * last iterate.  MA_ERR_NONFINITE when a norm is not finite. */
ma_status ma_solve(ma_solver *s, double *u, const double *f, double tol, unsigned flags,
                   ma_report *rep);

/* One FAS V(nu1,nu2) cycle of Algorithm 1 on u in place (MA_FP64 solvers);
 * returns once the cycle has run. */
ma_status ma_vcycle(ma_solver *s, double *u, const double *f);

/* Residual r = f - det(D^2_h u) at interior nodes (r = 0 on the Dirichlet
 * layer), the discrete Monge-Ampere operator of Section 1 / eq. 2.7.
 * r_or_null: device (n+1)^3 output or NULL.  l2_host (may be NULL): host
 * double receiving sqrt(h^3 sum r^2); synchronises the stream when given. */
ma_status ma_residual(ma_solver *s, const double *u, const double *f, double *r_or_null,
                      double *l2_host);

/* For callers that cannot allocate device memory -- code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the
 * residual and norm of ma_residual with no solver and no allocation.
 * n (2 <= n <= MA_NOALLOC_MAX_N): intervals per side; u, f: device
 * (n+1)^3 FP64, x fastest; r_or_null: device (n+1)^3 or NULL, receives
 * r = f - det(D^2_h u) inside and 0 on the boundary; l2_dev: one device
 * double, receives sqrt(h^3 sum r^2).  Everything is enqueued on hip_stream
 * (NULL: the null stream) and nothing is waited for.  The norm partials live
 * in a fixed device array of 4 MiB that the library holds on every device it
 * runs on until the process ends; all calls on one device share it, so calls
 * that overlap on one device race.  Errors: MA_ERR_ARG for n outside
 * 2..MA_NOALLOC_MAX_N or null u, f, l2_dev (message in ma_last_error(NULL)),
 * MA_ERR_DEVICE when a launch fails. */
#define MA_NOALLOC_MAX_N 512
ma_status ma_residual_noalloc(int n, const double *u, const double *f, double *r_or_null,
                              double *l2_dev, void *hip_stream);

/* count nonlinear Gauss-Seidel sweeps (Section 2, eqs. 2.8-2.9: each point
 * takes the smallest real root of its local cubic) on the finest grid, in
 * the solver's colour ordering.  u in place, f read.  nonconvex_host (may be
 * NULL) receives the number of updates that were not certified convex. */
ma_status ma_sweep(ma_solver *s, double *u, const double *f, int count,
                   long long *nonconvex_host);

/* FAS restriction from the finest grid (n) to the next (n/2), Algorithm 1
 * steps 3-5: w_c = injection of u (all coarse nodes), b_c = S_H(w_c) +
 * I_h^H (f - S_h(u)) at coarse interior nodes, 0 on the coarse boundary.
 * u, f: device (n+1)^3; w_c, b_c: device (n/2+1)^3 outputs.  MA_ERR_ARG if n
 * is odd or n < 4. */
ma_status ma_restrict(ma_solver *s, const double *u, const double *f, double *w_c,
                      double *b_c);

/* Coarse-grid correction, Algorithm 1 steps 7-8: u += I_H^h (u_c - w_c) at
 * fine interior nodes, trilinear interpolation (weights 1, 1/2, 1/4, 1/8).
 * u: device (n+1)^3 in place; u_c, w_c: device (n/2+1)^3. */
ma_status ma_prolong_correct(ma_solver *s, double *u, const double *u_c, const double *w_c);

/* One FMG-FAS iteration (Algorithm 2): f and the Dirichlet layer of u are
 * injected down the hierarchy (b_H := injection of b_h); on the coarsest
 * grid u starts from zero inside and takes nu0 sweeps; on the way up each
 * level's u is the FMG interpolation of the coarser one (tensor product of
 * 4-point cubic Lagrange rules, one-sided next to the boundary, quadratic
 * on a 3-node coarse grid; the paper asks for a cubic interpolation without
 * fixing the stencil) followed by one FAS V-cycle.  The interior of u on
 * entry is not read.  FP64 for both precisions.  nonconvex_host (may be
 * NULL) receives the non-certified updates.  Synchronises the stream. */
ma_status ma_fmg(ma_solver *s, double *u, const double *f, long long *nonconvex_host);

/* The standalone nonlinear Gauss-Seidel solver the paper compares against
 * (Section 4, the Gauss-Seidel halves of Tables 3 and 5-7): sweeps of the
 * smoother on the finest grid alone, u's interior as the start, until the
 * relative discrete L2 residual is <= tol (tol <= 0: the solver's tol) or
 * max_sweeps ran (MA_ERR_NOT_CONVERGED, report still filled).  The residual
 * is checked after every sweep, as in Section 4.  rep (may be NULL):
 * cycles = sweeps, res0, res, rel_res, history of the first 64 sweeps,
 * nonconvex, point_updates, alg_bytes, seconds.  Synchronises the stream. */
ma_status ma_gs_solve(ma_solver *s, double *u, const double *f, double tol, int max_sweeps,
                      ma_report *rep);

/* The MA_INIT_POISSON initial guess alone: linear V-cycles on
 * Lap_h u = 3 f^{1/3} until the relative linear residual is <= init_tol or
 * init_max_cycles ran.  cycles_host (may be NULL) receives the cycle count. */
ma_status ma_poisson_init(ma_solver *s, double *u, const double *f, int *cycles_host);

/* ---------------------------------------------------------------------- */
/* Batched solves: many independent problems of different sizes advance     */
/* together, one launch per level phase for all of them.                    */
/* ---------------------------------------------------------------------- */

/* Solve count independent problems together (up to 64 per engine pass;
 * larger counts run in consecutive groups of 64).  solvers[i] must have
 * been created for the size of u[i], f[i] and all with the same precision,
 * ordering, smoothing counts, inner_cycles, coarse_n and max_blocks
 * (else MA_ERR_ARG).  Each result equals that of ma_solve on the same
 * solver alone.  reps (may be NULL) receives count reports; when the first
 * solver of a group has profile set, the smooth_* fields of every report of
 * that group hold the group's totals (finest-level smoothing of all its
 * solves together).  Returns the first non-OK status over the solves (all
 * solves still complete).  Synchronises the first solver's stream. */
ma_status ma_solve_batch(ma_solver *const *solvers, double *const *u, const double *const *f,
                         int count, double tol, unsigned flags, ma_report *reps);

/* A resident batch for continuous serving: solves join and leave between
 * ticks; one tick runs one V-cycle (MA_MIXED: one outer correction) of every
 * active solve, batched by level.  The batch does not own the solvers. */
ma_status ma_batch_create(int max_solves, void *hip_stream, ma_batch **out);
void ma_batch_destroy(ma_batch *b);
const char *ma_batch_last_error(const ma_batch *b);

/* Join: claims a free slot (*slot_out) and resets its counters; no solver
 * work runs here.  The solve's own phases follow in the next ticks: with
 * MA_INIT_POISSON its Poisson guess (one linear V-cycle per tick), then its
 * entry residual res0, then its V-cycles.  All solvers of a batch share
 * nu1, nu2, nu0, order, restriction, precision and inner_cycles (else
 * MA_ERR_ARG); a solver holds at most one slot.  The tick replay mode
 * (graphs) is that of the first solver added to an empty batch.
 * Errors: MA_ERR_ARG (null argument, no free slot, incompatible solver). */
ma_status ma_batch_add(ma_batch *b, ma_solver *s, double *u, const double *f, double tol,
                       unsigned flags, int *slot_out);

/* One tick over all active slots; done_out[slot] (host, max_solves entries,
 * may be NULL) is set to 1 for slots that converged this tick and to 2 for
 * slots that stopped with an error (its status: ma_batch_report's fields and
 * ma_batch_last_error); 0 otherwise.  Synchronises the batch's stream. */
ma_status ma_batch_tick(ma_batch *b, int *done_out);

/* Report of a slot (valid while it is in the batch). */
ma_status ma_batch_report(const ma_batch *b, int slot, ma_report *rep);

/* Leave: frees the slot for another solve. */
ma_status ma_batch_remove(ma_batch *b, int slot);

#ifdef __cplusplus
}
#endif

#endif /* MA_H */
