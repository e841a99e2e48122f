// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mafas {

enum Op { OP_MA = 0, OP_LAP = 1 };

inline size_t npts(int n) { return size_t(n + 1) * size_t(n + 1) * size_t(n + 1); }
inline double interior(int n) { return double(n - 1) * double(n - 1) * double(n - 1); }

// Number of blocks (and partial sums) the residual-norm kernel produces for
// an n grid; the partial buffer must hold at least this many doubles.
size_t residual_partials(int n);

// --- smoother -------------------------------------------------------------
// One sweep of the operator op (MA: nonlinear GS, LAP: linear 7-point GS) on
// u in place, one launch per colour phase.  order 0: 4 colours, 1: 8 colours.
// nonconvex: device counter (may be null) incremented per non-certified update.
hipError_t launch_sweep_color(hipStream_t st, int op, int order, int n, double *u,
                              const double *F, unsigned long long *nonconvex);

// The block sweep (ma_fsweep.h): one sweep, all four colour phases in a
// single launch reading u_in and writing u_out (4-colour ordering only);
// u_out receives the Dirichlet layer too.  cfg: block shape index (< 0:
// automatic for n).  Bitwise equal to launch_sweep_color.
hipError_t launch_bsweep_one(hipStream_t st, int op, int cfg, int n, const double *u_in,
                             double *u_out, const double *F, unsigned long long *nonconvex);
int bsweep_num_configs();
// Automatic block shape for grids of up to n intervals whose 8^3 tiles number
// tiles8 in all.
int bsweep_pick(int n, long tiles8);
// automatic z-stream shape (config index) of an n grid
int bsweep_zs_pick(int n);

// --- residual and norm ----------------------------------------------------
// r = F - S(u) (interior; 0 on the boundary; r may be null) and per-block sums
// of r^2 into partials[0..residual_partials(n)).
hipError_t launch_residual(hipStream_t st, int op, int n, const double *u, const double *F,
                           double *r, double *partials);
// out[0] = sum of partials[0..count) in a fixed order (one block).
hipError_t launch_reduce(hipStream_t st, const double *partials, size_t count, double *out);

// --- transfers --------------------------------------------------------------
// FAS restriction nf -> nf/2: wc = uc = injection of uf; bc = S_H(wc) + I rf.
// rmode 0: full weighting, 1: half-weighting.
hipError_t launch_restrict(hipStream_t st, int op, int rmode, int nf, const double *uf,
                           const double *rf, double *wc, double *uc, double *bc);
// uf += trilinear(uc - wc) at fine interior nodes.
hipError_t launch_prolong(hipStream_t st, int nf, double *uf, const double *uc,
                          const double *wc);
// R = 3 cbrt(f) at every node.
hipError_t launch_poisson_rhs(hipStream_t st, int n, const double *f, double *R);
// dst = src (count doubles).
hipError_t launch_copy(hipStream_t st, size_t count, const double *src, double *dst);
// Copy the Dirichlet layer of src into dst.
hipError_t launch_copy_boundary(hipStream_t st, int n, const double *src, double *dst);
// vc (nf/2 intervals) = injection of vf at every coarse node.
hipError_t launch_inject_all(hipStream_t st, int nf, const double *vf, double *vc);
// Interior of uf (2 nc intervals) = FMG cubic interpolation of uc.
hipError_t launch_fmg_interp(hipStream_t st, int nc, const double *uc, double *uf);
// Interior of u = 0.
hipError_t launch_zero_interior(hipStream_t st, int n, double *u);

} // namespace mafas
