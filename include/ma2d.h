/*
 * ma2d.h -- C ABI of the two-dimensional variant of the solver:
 *
 *     u_xx u_yy - u_xy^2 = f   on the unit square,  u = g on the boundary,
 *
 * (the 2D equation of Section 1; the FMG-FAS runs of Section 4, Tables 1-2).
 * The discretisation is the 9-point centred stencil: u_xx and u_yy as
 * second differences, u_xy as the 4-point cross difference / (4 h^2).  The
 * nonlinear Gauss-Seidel update takes the smaller root of the local
 * quadratic (the one that keeps the discrete Hessian positive definite),
 * written in the shifted form det(G - sigma I) = f_p, u_p += sigma h^2 / 2.
 *
 * Layout: h = 1/n, every grid function is one (n+1)^2 FP64 array, x
 * fastest: index = i + (n+1) j.  Ownership, streams and errors follow ma.h:
 * the caller owns u and f (device pointers); the solver owns its hierarchy
 * from ma2d_create to ma2d_destroy; work is ordered on the given stream;
 * functions that return numbers to the host synchronise it; nothing throws.
 */
#ifndef MA2D_H
#define MA2D_H

#include <stddef.h>

#include "ma.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ma2d_solver ma2d_solver;

/* Orderings of the 2D sweep.  MA2D_COLOR4: colour (i mod 2) + 2 (j mod 2),
 * which decouples the 9-point stencil (true Gauss-Seidel).  MA2D_RED_BLACK:
 * the red-black ordering of Section 4, every node of a colour updated at
 * once from the values before that colour's phase (diagonal neighbours share
 * a colour in the 9-point stencil, so each phase is a Jacobi step). */
typedef enum { MA2D_COLOR4 = 0, MA2D_RED_BLACK = 1 } ma2d_order;

typedef struct {
    int n;               /* intervals per side, n >= 2                        */
    int nu1, nu2, nu0;   /* pre-, post-, coarsest sweeps (Section 4: 2, 2, 1)   */
    int order;           /* ma2d_order (default MA2D_RED_BLACK)                 */
    int restriction;     /* MA_RESTRICT_HALF (5-point, default) or
                            MA_RESTRICT_FULL (9-point)                          */
    int max_cycles;      /* V-cycles, the FMG start included                   */
    double tol;          /* default relative discrete L2 residual (1e-6)       */
} ma2d_params;

void ma2d_params_default(ma2d_params *p, int n);

/* Device bytes ma2d_create allocates for p (0 for invalid parameters). */
size_t ma2d_footprint_bytes(const ma2d_params *p);

/* Allocate the hierarchy (coarsen while n is even and >= 4).  Errors:
 * MA_ERR_ARG (invalid parameters, message by ma2d_last_error(NULL)),
 * MA_ERR_OOM, MA_ERR_DEVICE. */
ma_status ma2d_create(const ma2d_params *p, void *hip_stream, ma2d_solver **out);
void ma2d_destroy(ma2d_solver *s);
const char *ma2d_last_error(const ma2d_solver *s);

/* count sweeps of the nonlinear Gauss-Seidel smoother on u in place;
 * nonconvex_host (may be NULL): updates without a convex root. */
ma_status ma2d_sweep(ma2d_solver *s, double *u, const double *f, int count,
                     long long *nonconvex_host);

/* r = f - (u_xx u_yy - u_xy^2) at interior nodes (r_or_null may be NULL;
 * 0 on the boundary) and its discrete L2 norm sqrt(h^2 sum r^2) into
 * *l2_host (may be NULL). */
ma_status ma2d_residual(ma2d_solver *s, const double *u, const double *f, double *r_or_null,
                        double *l2_host);

/* One FAS V(nu1, nu2) cycle (Algorithm 1 in two dimensions): injection of
 * u into w_H = u_H, b_H = S_H(w_H) + I_h^H r, bilinear prolongation of
 * u_H - w_H. */
ma_status ma2d_vcycle(ma2d_solver *s, double *u, const double *f);

/* One FMG-FAS iteration (Algorithm 2 in two dimensions), FMG interpolation
 * as in ma_fmg (tensor product of cubic Lagrange rules); the interior of u
 * is not read.  Synchronises the stream. */
ma_status ma2d_fmg(ma2d_solver *s, double *u, const double *f, long long *nonconvex_host);

/* Solve under the stopping rule of Section 4.  flags: MA_INIT_FMG (the
 * Section 4 protocol: r^0 of the zero-interior start, one FMG-FAS iteration
 * as the first cycle) or 0 (u's interior is the start).  tol <= 0: the
 * solver's tol.  rep (may be NULL): cycles, res0, res, rel_res, converged,
 * history, nonconvex, point_updates, alg_bytes, seconds.  Errors as
 * ma_solve. */
ma_status ma2d_solve(ma2d_solver *s, double *u, const double *f, double tol, unsigned flags,
                     ma_report *rep);

#ifdef __cplusplus
}
#endif

#endif /* MA2D_H */
