/*
 * Serial FP64 CPU oracle for the FAS multigrid solver of the 3D Monge-Ampere
 * equation det(D^2 u) = f (Liu, Froese, Oberman, Xiao, "A multigrid scheme
 * for 3D Monge-Ampere equations").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can check the HIP implementation against a
 * plain, slow, obviously correct computation.  It shares no code, header or
 * table with the HIP library.
 *
 * Conventions (Section 2, discretisation): unit cube, h = 1/n, an (n+1)^3
 * array per grid function with x fastest: index = i + (n+1)(j + (n+1)k).
 * Nodes with any index in {0, n} carry Dirichlet data and are never written.
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *   - the local cubic (eq. 2.8) is solved in the shifted form
 *     det(G - sigma I) = F, G = discrete Hessian with the current centre
 *     value; P3(v) = h^6 q(sigma) for v = u_p + sigma h^2/2, an increasing
 *     affine map, so the smallest real root maps to the smallest real root
 *     (eq. 2.9);
 *   - second differences are formed as differences of first differences;
 *   - the ordering is a 4-colour (or 8-colour) decoupling of the 19-point
 *     stencil, colours swept 0..3 (0..7); lexicographic ordering is kept as
 *     the paper's own variant;
 *   - Algorithm 1: u_H and w_H are both the injection of w_h; the residual
 *     is restricted by the 7-point half-weighting of Section 3 or by 27-point
 *     full weighting (Section 3 leaves other transfers open; half-weighting
 *     makes the V-cycle diverge under multicolour orderings, so the colour
 *     orderings are paired with full weighting); the prolongation is trilinear interpolation (weights 1, 1/2, 1/4, 1/8;
 *     the printed 1/64 prefactor is read as 1/8), S_H is the same
 *     discretisation at step H = 2h;
 *   - coarsening continues while n is even and >= 4, so the coarsest grid
 *     has n = 2 (one unknown, the paper's h0 = 1/2) or n = 3;
 *   - the stopping rule is the relative discrete L2 residual of Section 4
 *     with r^0 the residual of the initial guess; a residual that stalls on
 *     the round-off floor above the tolerance (three cycles in a row without
 *     dropping below 0.9 x its best) ends the solve, not converged;
 *   - the local root for F > 0 is the one below lambda_min (Theorem 2.2):
 *     with q < 0 in the depressed cubic the three-root form is used even
 *     when rounding leaves the discriminant at or just above zero (a double
 *     smallest eigenvalue), where Cardano would give the largest root.
 *
 * Every function here is pinned by tests against values the paper prints,
 * closed forms, invariants or brute force.  Not pinned: the per-cycle
 * contraction and cycle counts of the 4-colour V-cycle ("parity unpinned":
 * the paper reports lexicographic counts only).
 *
 * Compile: gcc -O2 -ffp-contract=off -fPIC -shared ma_oracle.c -lm
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define MAO_MAX_LEVELS 32

#define IX(n, i, j, k) \
    ((size_t)(i) + (size_t)((n) + 1) * ((size_t)(j) + (size_t)((n) + 1) * (size_t)(k)))

/* ------------------------------------------------------------------ */
/* Level hierarchy                                                     */
/* ------------------------------------------------------------------ */

/* n_0 = n; n_{l+1} = n_l / 2 while n_l is even and >= 4.  Returns the number
 * of levels and writes them to ns (at most cap entries). */
int mao_levels(int n, int *ns, int cap)
{
    int L = 0;
    if (n < 2 || cap < 1)
        return 0;
    ns[L++] = n;
    while (n % 2 == 0 && n >= 4 && L < cap) {
        n /= 2;
        ns[L++] = n;
    }
    return L;
}

/* ------------------------------------------------------------------ */
/* Discrete Hessian (eqs. 2.1-2.6) and determinant (the explicit form  */
/* of det D^2 u in Section 1)                                          */
/* ------------------------------------------------------------------ */

/* g = {Gxx, Gyy, Gzz, Gxy, Gxz, Gyz} at interior node (i,j,k). */
void mao_hessian(int n, const double *u, int i, int j, int k, double *g)
{
    const double s = (double)n * (double)n;      /* 1/h^2 */
    const double s4 = 0.25 * s;                  /* 1/(4h^2) */
    const size_t sx = 1, sy = (size_t)(n + 1), sz = sy * sy;
    const size_t p = IX(n, i, j, k);
    const double up = u[p];
    double dxx = (u[p + sx] - up) - (up - u[p - sx]);
    double dyy = (u[p + sy] - up) - (up - u[p - sy]);
    double dzz = (u[p + sz] - up) - (up - u[p - sz]);
    double dxy = (u[p + sx + sy] - u[p - sx + sy]) - (u[p + sx - sy] - u[p - sx - sy]);
    double dxz = (u[p + sx + sz] - u[p - sx + sz]) - (u[p + sx - sz] - u[p - sx - sz]);
    double dyz = (u[p + sy + sz] - u[p - sy + sz]) - (u[p + sy - sz] - u[p - sy - sz]);
    g[0] = dxx * s;
    g[1] = dyy * s;
    g[2] = dzz * s;
    g[3] = dxy * s4;
    g[4] = dxz * s4;
    g[5] = dyz * s4;
}

/* det of the symmetric matrix g, in the term order of the explicit
 * operator: xx yy zz + 2 xy yz xz - xx yz^2 - yy xz^2 - zz xy^2. */
double mao_det3(const double *g)
{
    const double xx = g[0], yy = g[1], zz = g[2], xy = g[3], xz = g[4], yz = g[5];
    return xx * yy * zz + 2.0 * xy * yz * xz - xx * (yz * yz) - yy * (xz * xz)
           - zz * (xy * xy);
}

/* 1 if the symmetric matrix g is positive definite (Sylvester minors). */
int mao_is_spd(const double *g)
{
    const double m1 = g[0];
    const double m2 = g[0] * g[1] - g[3] * g[3];
    const double m3 = mao_det3(g);
    return m1 > 0.0 && m2 > 0.0 && m3 > 0.0;
}

/* ------------------------------------------------------------------ */
/* Local equation and root selection (eqs. 2.8-2.9, Theorems 2.1-2.2) */
/* ------------------------------------------------------------------ */

/* q(sigma) = det(G - sigma I) - F evaluated on the shifted matrix, and its
 * derivative q'(sigma) = -(sum of the principal 2x2 minors of G - sigma I). */
static void shifted_q(const double *g, double F, double sig, double *q, double *dq)
{
    double m[6];
    m[0] = g[0] - sig;
    m[1] = g[1] - sig;
    m[2] = g[2] - sig;
    m[3] = g[3];
    m[4] = g[4];
    m[5] = g[5];
    *q = mao_det3(m) - F;
    *dq = -((m[0] * m[1] - m[3] * m[3]) + (m[0] * m[2] - m[4] * m[4])
            + (m[1] * m[2] - m[5] * m[5]));
}

/* Smallest real root sigma of det(G - sigma I) = F.
 *
 * Closed form: with m = tr(G)/3 and B = G - m I (traceless), y = sigma - m
 * solves the depressed cubic y^3 - P y + (F - det B) = 0, P = tr(B^2)/2 >= 0.
 * Three real roots -> trigonometric form, smallest one; otherwise Cardano's
 * real root.  Then up to two Newton steps on the shifted form, each kept only
 * if it reduces |q|.  This is a textbook cubic solve; it does not use the
 * monotone Newton bracket that the GPU smoother uses, so the two serve as
 * cross-checks. */
double mao_local_root(const double *g, double F)
{
    const double xx = g[0], yy = g[1], zz = g[2], xy = g[3], xz = g[4], yz = g[5];
    const double m = (xx + yy + zz) / 3.0;
    const double bx = xx - m, by = yy - m, bz = zz - m;
    const double P = 0.5 * (bx * bx + by * by + bz * bz) + (xy * xy + xz * xz + yz * yz);
    const double detB = bx * (by * bz - yz * yz) - xy * (xy * bz - yz * xz)
                        + xz * (xy * yz - by * xz);
    const double q = F - detB;        /* y^3 + p y + q = 0 with p = -P */
    double y;
    const double D = 0.25 * q * q - P * P * P / 27.0;
    /* F > 0 and q < 0: by Theorem 2.2 a root lies below lambda_min <= m, i.e.
     * y < 0, while Cardano's single real root would be positive, so the
     * cubic has three real roots and D < 0.  With a double smallest
     * eigenvalue D is within rounding of 0 and can come out >= 0, where
     * Cardano would return the largest root: such a D is taken as the
     * three-root case. */
    const int near_double = F > 0.0 && P > 0.0 && q < 0.0 && D >= 0.0
                            && D <= 1e-10 * (P * P * P / 27.0);
    if ((P <= 0.0 || D >= 0.0) && !near_double) {
        /* one real root (or a multiple root): Cardano without cancellation */
        const double sq = sqrt(D > 0.0 ? D : 0.0);
        const double A = -copysign(cbrt(0.5 * fabs(q) + sq), q);
        const double Bc = (A != 0.0) ? P / (3.0 * A) : 0.0;
        y = A + Bc;
    } else {
        /* three real roots: y_k = 2 sqrt(P/3) cos(theta/3 - 2 pi k/3),
         * cos(theta) = -(3 q / (2 P)) sqrt(3/P); smallest is k = 2. */
        const double rr = sqrt(P / 3.0);
        double c = -(1.5 * q / P) * sqrt(3.0 / P);
        if (c > 1.0)
            c = 1.0;
        if (c < -1.0)
            c = -1.0;
        const double th = acos(c);
        y = 2.0 * rr * cos(th / 3.0 + 2.0 * M_PI / 3.0);
    }
    double sig = y + m;
    /* safeguarded Newton polish */
    double qv, dq;
    shifted_q(g, F, sig, &qv, &dq);
    for (int it = 0; it < 2; ++it) {
        if (!(dq != 0.0) || !isfinite(qv))
            break;
        const double cand = sig - qv / dq;
        double qc, dqc;
        shifted_q(g, F, cand, &qc, &dqc);
        if (!(fabs(qc) < fabs(qv)))
            break;
        sig = cand;
        qv = qc;
        dq = dqc;
    }
    return sig;
}

/* One nonlinear GS point update at an interior node; returns 1 when the node
 * is not certified convex (F <= 0 or G - sigma I not positive definite). */
static int ma_update(int n, double *u, const double *F, int i, int j, int k)
{
    double g[6];
    const size_t p = IX(n, i, j, k);
    const double s = (double)n * (double)n;
    const double half_h2 = 0.5 / s;
    mao_hessian(n, u, i, j, k, g);
    const double sig = mao_local_root(g, F[p]);
    u[p] = u[p] + sig * half_h2;
    g[0] -= sig;
    g[1] -= sig;
    g[2] -= sig;
    return (F[p] > 0.0 && mao_is_spd(g)) ? 0 : 1;
}

/* Linear 7-point Gauss-Seidel update for Lap_h u = R:
 * u_p <- u_p - (R - Lap_h u)/(6 s), Lap_h from differences of differences. */
static void lap_update(int n, double *u, const double *R, int i, int j, int k)
{
    const size_t p = IX(n, i, j, k);
    const size_t sy = (size_t)(n + 1), sz = sy * sy;
    const double s = (double)n * (double)n;
    const double up = u[p];
    const double lap = (((u[p + 1] - up) - (up - u[p - 1])) + ((u[p + sy] - up) - (up - u[p - sy]))
                        + ((u[p + sz] - up) - (up - u[p - sz]))) * s;
    u[p] = up - (R[p] - lap) * (1.0 / (6.0 * s));
}

/* Colour of node (i,j,k).  order 0: 4 colours ((i+j) mod 2) + 2((i+k) mod 2);
 * order 1: 8 colours (i mod 2) + 2 (j mod 2) + 4 (k mod 2). */
int mao_color(int order, int i, int j, int k)
{
    if (order == 1)
        return (i & 1) + 2 * (j & 1) + 4 * (k & 1);
    return ((i + j) & 1) + 2 * ((i + k) & 1);
}

int mao_num_colors(int order) { return order == 1 ? 8 : (order == 0 ? 4 : 1); }

/* op 0: Monge-Ampere update, op 1: 7-point Laplacian update. */
static long sweep_color(int n, double *u, const double *F, int order, int c, int op)
{
    long nc = 0;
    for (int k = 1; k < n; ++k)
        for (int j = 1; j < n; ++j)
            for (int i = 1; i < n; ++i) {
                if (mao_color(order, i, j, k) != c)
                    continue;
                if (op == 0)
                    nc += ma_update(n, u, F, i, j, k);
                else
                    lap_update(n, u, F, i, j, k);
            }
    return nc;
}

static long sweep_op(int n, double *u, const double *F, int order, int op)
{
    long nc = 0;
    if (order == 2) {                           /* lexicographic: k, j, i */
        for (int k = 1; k < n; ++k)
            for (int j = 1; j < n; ++j)
                for (int i = 1; i < n; ++i) {
                    if (op == 0)
                        nc += ma_update(n, u, F, i, j, k);
                    else
                        lap_update(n, u, F, i, j, k);
                }
        return nc;
    }
    const int nc_colors = mao_num_colors(order);
    for (int c = 0; c < nc_colors; ++c)
        nc += sweep_color(n, u, F, order, c, op);
    return nc;
}

/* One nonlinear GS sweep (order 0: 4 colours, 1: 8 colours, 2: lexicographic).
 * Returns the number of updates not certified convex. */
long mao_sweep(int n, double *u, const double *F, int order)
{
    return sweep_op(n, u, F, order, 0);
}

/* One colour phase of the nonlinear sweep. */
long mao_sweep_color(int n, double *u, const double *F, int order, int color)
{
    return sweep_color(n, u, F, order, color, 0);
}

void mao_poisson_sweep(int n, double *u, const double *R, int order)
{
    (void)sweep_op(n, u, R, order, 1);
}

/* ------------------------------------------------------------------ */
/* Residuals                                                           */
/* ------------------------------------------------------------------ */

static double residual_op(int n, const double *u, const double *F, double *r, int op)
{
    double acc = 0.0;
    const double s = (double)n * (double)n;
    const size_t sy = (size_t)(n + 1), sz = sy * sy;
    if (r)
        memset(r, 0, sizeof(double) * sz * sy);
    for (int k = 1; k < n; ++k)
        for (int j = 1; j < n; ++j)
            for (int i = 1; i < n; ++i) {
                const size_t p = IX(n, i, j, k);
                double rv;
                if (op == 0) {
                    double g[6];
                    mao_hessian(n, u, i, j, k, g);
                    rv = F[p] - mao_det3(g);
                } else {
                    const double up = u[p];
                    const double lap = (((u[p + 1] - up) - (up - u[p - 1]))
                                        + ((u[p + sy] - up) - (up - u[p - sy]))
                                        + ((u[p + sz] - up) - (up - u[p - sz]))) * s;
                    rv = F[p] - lap;
                }
                if (r)
                    r[p] = rv;
                acc += rv * rv;
            }
    return acc;
}

/* r = F - det(D^2_h u) at interior nodes, 0 on the Dirichlet layer; returns
 * sum of r^2 over interior nodes (r may be NULL). */
double mao_residual(int n, const double *u, const double *F, double *r)
{
    return residual_op(n, u, F, r, 0);
}

double mao_poisson_residual(int n, const double *u, const double *R, double *r)
{
    return residual_op(n, u, R, r, 1);
}

/* Discrete L2 norm sqrt(h^3 sum r^2) from a raw sum of squares. */
static double l2_from_sumsq(int n, double ss)
{
    const double h = 1.0 / (double)n;
    return sqrt(ss * h * h * h);
}

/* ------------------------------------------------------------------ */
/* Transfers (Algorithm 1 steps 3-5 and 7-8, Section 3 stencils)       */
/* ------------------------------------------------------------------ */

/* Restricted residual at coarse interior node (I,J,K).
 * rmode 0: the 7-point half-weighting of Section 3, (6 centre + 6 faces)/12;
 * rmode 1: 27-point full weighting, tensor product of (1/4, 1/2, 1/4),
 *          summed with k, then j, then i ascending. */
static double restrict_point(int nf, const double *rf, int I, int J, int K, int rmode)
{
    const size_t fy = (size_t)(nf + 1), fz = fy * fy;
    const size_t f = IX(nf, 2 * I, 2 * J, 2 * K);
    if (rmode == 0)
        return (6.0 * rf[f] + (rf[f - 1] + rf[f + 1]) + (rf[f - fy] + rf[f + fy])
                + (rf[f - fz] + rf[f + fz])) / 12.0;
    static const double w[3] = {0.25, 0.5, 0.25};
    double acc = 0.0;
    for (int c = -1; c <= 1; ++c)
        for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a)
                acc += (w[c + 1] * w[b + 1] * w[a + 1])
                       * rf[IX(nf, 2 * I + a, 2 * J + b, 2 * K + c)];
    return acc;
}

/* FAS restriction from the fine grid nf to the coarse grid nc = nf/2:
 *   wc = injection of uf at every coarse node (Dirichlet layer included),
 *   bc = S_H(wc) + I_h^H rf at coarse interior nodes, 0 on the boundary,
 * where I_h^H is selected by rmode (see restrict_point) and S_H is the
 * Monge-Ampere operator (op 0) or the 7-point Laplacian (op 1) at step 2h. */
void mao_restrict(int nf, const double *uf, const double *rf, double *wc, double *bc, int op,
                  int rmode)
{
    const int nc = nf / 2;
    for (int K = 0; K <= nc; ++K)
        for (int J = 0; J <= nc; ++J)
            for (int I = 0; I <= nc; ++I)
                wc[IX(nc, I, J, K)] = uf[IX(nf, 2 * I, 2 * J, 2 * K)];
    const double s = (double)nc * (double)nc;
    const size_t cy = (size_t)(nc + 1), cz = cy * cy;
    memset(bc, 0, sizeof(double) * cz * cy);
    for (int K = 1; K < nc; ++K)
        for (int J = 1; J < nc; ++J)
            for (int I = 1; I < nc; ++I) {
                const double rh = restrict_point(nf, rf, I, J, K, rmode);
                double sh;
                if (op == 0) {
                    double g[6];
                    mao_hessian(nc, wc, I, J, K, g);
                    sh = mao_det3(g);
                } else {
                    const size_t c = IX(nc, I, J, K);
                    const double w = wc[c];
                    sh = (((wc[c + 1] - w) - (w - wc[c - 1])) + ((wc[c + cy] - w) - (w - wc[c - cy]))
                          + ((wc[c + cz] - w) - (w - wc[c - cz]))) * s;
                }
                bc[IX(nc, I, J, K)] = sh + rh;
            }
}

/* u_h += I_H^h (u_H - w_H) at fine interior nodes, trilinear interpolation.
 * For each axis an even fine index takes the coincident coarse node with
 * weight 1, an odd one the two neighbours with weight 1/2; corner
 * contributions are summed with k, then j, then i ascending. */
void mao_prolong_correct(int nf, double *uf, const double *uc, const double *wc)
{
    const int nc = nf / 2;
    for (int k = 1; k < nf; ++k)
        for (int j = 1; j < nf; ++j)
            for (int i = 1; i < nf; ++i) {
                int ia[2], ja[2], ka[2];
                double wi[2], wj[2], wk[2];
                int ni, nj, nk;
                if (i % 2 == 0) { ia[0] = i / 2; wi[0] = 1.0; ni = 1; }
                else { ia[0] = i / 2; ia[1] = i / 2 + 1; wi[0] = wi[1] = 0.5; ni = 2; }
                if (j % 2 == 0) { ja[0] = j / 2; wj[0] = 1.0; nj = 1; }
                else { ja[0] = j / 2; ja[1] = j / 2 + 1; wj[0] = wj[1] = 0.5; nj = 2; }
                if (k % 2 == 0) { ka[0] = k / 2; wk[0] = 1.0; nk = 1; }
                else { ka[0] = k / 2; ka[1] = k / 2 + 1; wk[0] = wk[1] = 0.5; nk = 2; }
                double d = 0.0;
                for (int c = 0; c < nk; ++c)
                    for (int b = 0; b < nj; ++b)
                        for (int a = 0; a < ni; ++a) {
                            const size_t q = IX(nc, ia[a], ja[b], ka[c]);
                            d += (wk[c] * wj[b] * wi[a]) * (uc[q] - wc[q]);
                        }
                uf[IX(nf, i, j, k)] += d;
            }
}

/* R = 3 f^{1/3}: the right-hand side of the Poisson problem whose solution
 * is the initial guess (Laplacian = trace = 3 x geometric mean of the
 * Hessian eigenvalues when they are equal). */
void mao_poisson_rhs(int n, const double *f, double *R)
{
    const size_t cnt = (size_t)(n + 1) * (size_t)(n + 1) * (size_t)(n + 1);
    for (size_t p = 0; p < cnt; ++p)
        R[p] = 3.0 * cbrt(f[p]);
}

/* ------------------------------------------------------------------ */
/* V-cycle (Algorithm 1) and solve                                     */
/* ------------------------------------------------------------------ */

typedef struct {
    int nu1, nu2, nu0;       /* pre, post, coarsest sweeps (2, 2, 1) */
    int order;               /* 0: 4 colours, 1: 8 colours, 2: lexicographic */
    int rmode;               /* residual restriction: 0 half-, 1 full weighting */
    int max_cycles;
    double tol;              /* relative L2 residual; < 0 selects limit mode */
    int init;                /* 0: use u as given, 1: Poisson initial guess,
                                2: one FMG-FAS iteration (Algorithm 2) */
    double init_tol;         /* relative linear residual for the Poisson guess */
    int init_max_cycles;
} mao_params;

typedef struct {
    int cycles;
    int init_cycles;
    int converged;
    double res0;             /* discrete L2 residual of the initial guess */
    double res;              /* final discrete L2 residual */
    double seconds;
    long nonconvex;          /* updates not certified convex */
} mao_report;

typedef struct {
    int L;                   /* number of levels */
    int ns[MAO_MAX_LEVELS];
    double *u[MAO_MAX_LEVELS];
    double *b[MAO_MAX_LEVELS];
    double *w[MAO_MAX_LEVELS];
    double *r[MAO_MAX_LEVELS];
} hier;

static size_t npts(int n) { return (size_t)(n + 1) * (size_t)(n + 1) * (size_t)(n + 1); }

static int hier_alloc(hier *H, int n)
{
    memset(H, 0, sizeof(*H));
    H->L = mao_levels(n, H->ns, MAO_MAX_LEVELS);
    for (int l = 0; l < H->L; ++l) {
        const size_t c = npts(H->ns[l]);
        H->r[l] = (double *)calloc(c, sizeof(double));
        if (l > 0) {
            H->u[l] = (double *)calloc(c, sizeof(double));
            H->b[l] = (double *)calloc(c, sizeof(double));
            H->w[l] = (double *)calloc(c, sizeof(double));
        }
        if (!H->r[l] || (l > 0 && (!H->u[l] || !H->b[l] || !H->w[l])))
            return -1;
    }
    return 0;
}

static void hier_free(hier *H)
{
    for (int l = 0; l < H->L; ++l) {
        free(H->u[l]);
        free(H->b[l]);
        free(H->w[l]);
        free(H->r[l]);
    }
}

static long vcycle_rec(hier *H, int l, double *u, const double *b, const mao_params *p, int op)
{
    const int n = H->ns[l];
    long nc = 0;
    if (l == H->L - 1) {
        for (int s = 0; s < p->nu0; ++s)
            nc += sweep_op(n, u, b, p->order, op);
        return nc;
    }
    for (int s = 0; s < p->nu1; ++s)
        nc += sweep_op(n, u, b, p->order, op);
    (void)residual_op(n, u, b, H->r[l], op);
    mao_restrict(n, u, H->r[l], H->w[l + 1], H->b[l + 1], op, p->rmode);
    memcpy(H->u[l + 1], H->w[l + 1], sizeof(double) * npts(H->ns[l + 1]));
    nc += vcycle_rec(H, l + 1, H->u[l + 1], H->b[l + 1], p, op);
    mao_prolong_correct(n, u, H->u[l + 1], H->w[l + 1]);
    for (int s = 0; s < p->nu2; ++s)
        nc += sweep_op(n, u, b, p->order, op);
    return nc;
}

/* One FAS V(nu1, nu2) cycle on det(D^2 u) = f.  Returns -1 on allocation
 * failure, otherwise the number of non-certified updates. */
long mao_vcycle(int n, double *u, const double *f, const mao_params *p)
{
    hier H;
    if (hier_alloc(&H, n)) {
        hier_free(&H);
        return -1;
    }
    const long nc = vcycle_rec(&H, 0, u, f, p, 0);
    hier_free(&H);
    return nc;
}

/* One linear V-cycle on Lap_h u = R (same ordering and transfers). */
int mao_poisson_vcycle(int n, double *u, const double *R, const mao_params *p)
{
    hier H;
    if (hier_alloc(&H, n)) {
        hier_free(&H);
        return -1;
    }
    (void)vcycle_rec(&H, 0, u, R, p, 1);
    hier_free(&H);
    return 0;
}

/* Initial guess: solve Lap_h u = 3 f^{1/3} with the Dirichlet layer of u by
 * linear V-cycles until the relative linear residual is <= init_tol or
 * init_max_cycles are spent.  Returns the number of cycles (or -1). */
int mao_poisson_init(int n, double *u, const double *f, const mao_params *p)
{
    hier H;
    const size_t c = npts(n);
    double *R = (double *)malloc(sizeof(double) * c);
    if (!R || hier_alloc(&H, n)) {
        free(R);
        hier_free(&H);
        return -1;
    }
    mao_poisson_rhs(n, f, R);
    const double r0 = sqrt(residual_op(n, u, R, NULL, 1));
    int cyc = 0;
    if (r0 > 0.0) {
        while (cyc < p->init_max_cycles) {
            (void)vcycle_rec(&H, 0, u, R, p, 1);
            ++cyc;
            const double r = sqrt(residual_op(n, u, R, NULL, 1));
            if (r <= p->init_tol * r0)
                break;
        }
    }
    free(R);
    hier_free(&H);
    return cyc;
}

/* ------------------------------------------------------------------ */
/* Full multigrid (Algorithm 2)                                         */
/* ------------------------------------------------------------------ */

/* Injection (the operator written with a tilde in Section 3): the coarse
 * value at every coarse node, boundary included, is the fine value at the
 * same point. */
void mao_inject(int nf, const double *vf, double *vc)
{
    const int nc = nf / 2;
    for (int K = 0; K <= nc; ++K)
        for (int J = 0; J <= nc; ++J)
            for (int I = 0; I <= nc; ++I)
                vc[IX(nc, I, J, K)] = vf[IX(nf, 2 * I, 2 * J, 2 * K)];
}

/* 1D weights of the FMG interpolation at fine index i of a fine grid with
 * nf = 2 nc intervals: a coarse node copies (weight 1); a midpoint takes the
 * cubic Lagrange value through the four nearest coarse nodes, one-sided
 * next to the boundary, and the quadratic value when the coarse grid has
 * only three nodes.  Writes the first coarse index and up to 4 weights;
 * returns their count. */
static int fmg_weights(int nc, int i, int *first, double *w)
{
    if ((i & 1) == 0) {
        *first = i / 2;
        w[0] = 1.0;
        return 1;
    }
    const int I0 = (i - 1) / 2;          /* midpoint between I0 and I0 + 1 */
    if (nc < 3) {                         /* nodes 0, 1, 2: quadratic */
        *first = 0;
        if (I0 == 0) {
            w[0] = 3.0 / 8.0; w[1] = 6.0 / 8.0; w[2] = -1.0 / 8.0;
        } else {
            w[0] = -1.0 / 8.0; w[1] = 6.0 / 8.0; w[2] = 3.0 / 8.0;
        }
        return 3;
    }
    if (I0 == 0) {                        /* nodes 0..3, point at 0.5 */
        *first = 0;
        w[0] = 5.0 / 16.0; w[1] = 15.0 / 16.0; w[2] = -5.0 / 16.0; w[3] = 1.0 / 16.0;
    } else if (I0 + 1 == nc) {            /* nodes nc-3..nc, point at nc-0.5 */
        *first = nc - 3;
        w[0] = 1.0 / 16.0; w[1] = -5.0 / 16.0; w[2] = 15.0 / 16.0; w[3] = 5.0 / 16.0;
    } else {                              /* nodes I0-1..I0+2 */
        *first = I0 - 1;
        w[0] = -1.0 / 16.0; w[1] = 9.0 / 16.0; w[2] = 9.0 / 16.0; w[3] = -1.0 / 16.0;
    }
    return 4;
}

/* FMG interpolation (Algorithm 2, step 4): the interior of the fine grid
 * from the coarse grid by the tensor product of the 1D rule above; the
 * fine boundary layer is left as it is (Dirichlet data). */
void mao_fmg_interp(int nc, const double *uc, double *uf)
{
    const int nf = 2 * nc;
    for (int k = 1; k < nf; ++k) {
        int fk, ck;
        double wk[4];
        ck = fmg_weights(nc, k, &fk, wk);
        for (int j = 1; j < nf; ++j) {
            int fj, cj;
            double wj[4];
            cj = fmg_weights(nc, j, &fj, wj);
            for (int i = 1; i < nf; ++i) {
                int fi, ci;
                double wi[4];
                ci = fmg_weights(nc, i, &fi, wi);
                double v = 0.0;
                for (int c = 0; c < ck; ++c)
                    for (int b = 0; b < cj; ++b)
                        for (int a = 0; a < ci; ++a)
                            v += wk[c] * wj[b] * wi[a] * uc[IX(nc, fi + a, fj + b, fk + c)];
                uf[IX(nf, i, j, k)] = v;
            }
        }
    }
}

/* Algorithm 2 at level l: w_l := FMG(l, b_l).  u holds the Dirichlet data
 * of level l on its boundary layer on entry. */
static long fmg_rec(hier *H, int l, double *u, const double *b, const mao_params *p)
{
    const int n = H->ns[l];
    long nc = 0;
    if (l == H->L - 1) {
        /* coarsest: initial guess zero inside, then an approximate solve.
         * The paper's coarsest grid (h0 = 1/2) has one unknown, which one
         * sweep solves exactly; a 3-interval coarsest grid has 8 unknowns
         * and takes 8 sweeps here, enough for the same accuracy */
        for (int k = 1; k < n; ++k)
            for (int j = 1; j < n; ++j)
                for (int i = 1; i < n; ++i)
                    u[IX(n, i, j, k)] = 0.0;
        const int sweeps = (n == 3 && p->nu0 < 8) ? 8 : p->nu0;
        for (int s = 0; s < sweeps; ++s)
            nc += sweep_op(n, u, b, p->order, 0);
        return nc;
    }
    mao_inject(n, b, H->b[l + 1]);       /* b_H := injection of b_h */
    mao_inject(n, u, H->u[l + 1]);       /* boundary data of level l + 1 */
    nc += fmg_rec(H, l + 1, H->u[l + 1], H->b[l + 1], p);
    mao_fmg_interp(H->ns[l + 1], H->u[l + 1], u);
    nc += vcycle_rec(H, l, u, b, p, 0);  /* one FAS V-cycle */
    return nc;
}

/* One FMG-FAS iteration (Algorithm 2) on det(D^2 u) = f; u carries the
 * Dirichlet data on its boundary layer, its interior is not read.  Returns
 * -1 on allocation failure, otherwise the number of non-certified updates. */
long mao_fmg(int n, double *u, const double *f, const mao_params *p)
{
    hier H;
    if (hier_alloc(&H, n)) {
        hier_free(&H);
        return -1;
    }
    const long nc = fmg_rec(&H, 0, u, f, p);
    hier_free(&H);
    return nc;
}

/* Full solve (Algorithm 1 repeated under the Section 4 stopping rule).
 * hist (optional, hist_cap entries) receives the discrete L2 residual after
 * each cycle.  The residual stalls when it fails to drop below 0.9 x its
 * best value for three cycles in a row, i.e. it sits on the round-off floor.
 * Limit mode (tol < 0): cycle until it stalls.  With a tolerance: cycle
 * until the relative residual is <= tol, or until it stalls above it (a start
 * so close to the solution that tol x r0 lies under the floor: not
 * converged), or max_cycles.  Returns 0 when converged, 1 when not, -1 on
 * allocation failure. */
int mao_solve(int n, double *u, const double *f, const mao_params *p, mao_report *rep,
              double *hist, int hist_cap)
{
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    memset(rep, 0, sizeof(*rep));
    if (p->init == 1) {
        rep->init_cycles = mao_poisson_init(n, u, f, p);
        if (rep->init_cycles < 0)
            return -1;
    }
    hier H;
    if (hier_alloc(&H, n)) {
        hier_free(&H);
        return -1;
    }
    if (p->init == 2) {
        /* Section 4 protocol: r^0 is the residual of the start that has
         * the Dirichlet data and zero inside; one FMG-FAS iteration
         * (Algorithm 2) counts as the first cycle */
        for (int k = 1; k < n; ++k)
            for (int j = 1; j < n; ++j)
                for (int i = 1; i < n; ++i)
                    u[IX(n, i, j, k)] = 0.0;
    }
    rep->res0 = l2_from_sumsq(n, residual_op(n, u, f, NULL, 0));
    rep->res = rep->res0;
    if (p->init == 2) {
        rep->nonconvex += fmg_rec(&H, 0, u, f, p);
        rep->init_cycles = 1;
        rep->res = l2_from_sumsq(n, residual_op(n, u, f, NULL, 0));
        if (hist && hist_cap > 0)
            hist[0] = rep->res;
    }
    double best = rep->res0;
    int stall = 0;
    int status = 1;
    if (rep->res0 == 0.0 && p->tol >= 0.0) {
        status = 0;
    } else {
        const int c0 = p->init == 2 ? 1 : 0;   /* FMG is cycle 1 */
        rep->cycles = c0;
        if (c0 && p->tol >= 0.0 && rep->res <= p->tol * rep->res0) {
            status = 0;
            rep->cycles = 1;
        }
        for (int c = c0; status != 0 && c < p->max_cycles; ++c) {
            rep->nonconvex += vcycle_rec(&H, 0, u, f, p, 0);
            rep->cycles = c + 1;
            rep->res = l2_from_sumsq(n, residual_op(n, u, f, NULL, 0));
            if (hist && c < hist_cap)
                hist[c] = rep->res;
            /* the residual's best value so far and the cycles since it last
             * dropped below 0.9 x that best */
            const int stalled = rep->res < 0.9 * best ? 0 : stall + 1;
            if (stalled == 0)
                best = rep->res;
            stall = stalled;
            if (p->tol >= 0.0) {
                if (rep->res <= p->tol * rep->res0) {
                    status = 0;
                    break;
                }
                /* stagnation above the tolerance: three cycles in a row on
                 * the round-off floor cannot reach it; not converged */
                if (stall >= 3)
                    break;
            } else if (stall >= 3) {
                status = 0;
                break;
            }
        }
    }
    hier_free(&H);
    rep->converged = (status == 0);
    clock_gettime(CLOCK_MONOTONIC, &t1);
    rep->seconds = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
    return status;
}
