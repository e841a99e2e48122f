/*
 * Serial FP64 CPU oracle for the two-dimensional version of the method
 * (u_xx u_yy - u_xy^2 = f, Section 1; the FMG-FAS runs of Section 4,
 * Tables 1-2).  TEST INFRASTRUCTURE ONLY: nothing in the product path may
 * call, link or load it; it shares no code with the HIP library.
 *
 * Conventions: unit square, h = 1/n, an (n+1)^2 array per grid function
 * with x fastest: index = i + (n+1) j.  Nodes with an index in {0, n} carry
 * Dirichlet data and are never written.
 *
 * Readings (listed in the design notes):
 *   - 9-point stencil: u_xx, u_yy as second differences (differences of
 *     first differences), u_xy as the 4-point cross difference / (4 h^2);
 *   - local update in the shifted form (G - sigma I has determinant F,
 *     u_p += sigma h^2 / 2): the smaller root of
 *     sigma^2 - tr(G) sigma + det(G) - F = 0, evaluated without
 *     cancellation; when F is so negative that no real root exists the
 *     vertex tr(G) / 2 is taken and the node is counted as not convex;
 *   - orderings: 4-colour (i mod 2) + 2 (j mod 2), which decouples the
 *     9-point stencil; red-black with every node of a colour updated at
 *     once from the values before the colour phase (diagonal neighbours
 *     share the colour, so a red-black sweep is a Jacobi step per colour);
 *     lexicographic, j outer, i inner;
 *   - transfers: injection of u into u_H = w_H, the residual restricted by
 *     5-point half-weighting (4 r_c + sum of the 4 edge neighbours) / 8 or
 *     9-point full weighting (tensor product of 1/4, 1/2, 1/4), bilinear
 *     prolongation of the correction; FMG interpolation as in 3D: tensor
 *     product of 4-point cubic Lagrange rules, one-sided at the boundary,
 *     quadratic on a 3-node grid;
 *   - hierarchy: coarsen while n is even and >= 4; FMG's coarsest solve
 *     starts from zero inside and takes nu0 sweeps (8 when the coarsest
 *     grid has 3 intervals).
 *
 * Compile: gcc -O2 -ffp-contract=off -fPIC -shared ma2_oracle.c -lm
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define M2_MAX_LEVELS 32
#define IX2(n, i, j) ((size_t)(i) + (size_t)((n) + 1) * (size_t)(j))

typedef struct {
    int nu1, nu2, nu0;   /* pre, post, coarsest sweeps */
    int order;           /* 0: 4 colours, 1: red-black (simultaneous), 2: lexicographic */
    int rmode;           /* 0: half-weighting, 1: full weighting */
    int max_cycles;
    double tol;          /* relative L2 residual; < 0: limit mode */
    int init;            /* 0: u as given, 2: FMG-FAS start (Section 4 protocol) */
} ma2_params;

typedef struct {
    int cycles;
    int converged;
    double res0, res;
    long nonconvex;
} ma2_report;

int ma2_levels(int n, int *ns, int cap)
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

/* Discrete Hessian (g[0] = xx, g[1] = yy, g[2] = xy) at (i, j). */
void ma2_hessian(int n, const double *u, int i, int j, double *g)
{
    const double s = (double)n * (double)n, s4 = 0.25 * s;
    const double c = u[IX2(n, i, j)];
    g[0] = ((u[IX2(n, i + 1, j)] - c) - (c - u[IX2(n, i - 1, j)])) * s;
    g[1] = ((u[IX2(n, i, j + 1)] - c) - (c - u[IX2(n, i, j - 1)])) * s;
    g[2] = ((u[IX2(n, i + 1, j + 1)] - u[IX2(n, i - 1, j + 1)])
            - (u[IX2(n, i + 1, j - 1)] - u[IX2(n, i - 1, j - 1)])) * s4;
}

/* Smaller root of (g0 - sigma)(g1 - sigma) - g2^2 = F; *nc set when no
 * real root exists (vertex returned) or F <= 0. */
double ma2_local_root(const double *g, double F, int *nc)
{
    const double t = g[0] + g[1];
    const double d = g[0] * g[1] - g[2] * g[2];
    const double a = g[0] - g[1];
    const double disc = a * a + 4.0 * g[2] * g[2] + 4.0 * F;
    if (!(F > 0.0))
        *nc = 1;
    if (disc < 0.0) {
        *nc = 1;
        return 0.5 * t;
    }
    const double r = sqrt(disc);
    if (t > 0.0)
        return 2.0 * (d - F) / (t + r);   /* (t - r) / 2 without cancellation */
    return 0.5 * (t - r);
}

static double det2(const double *g) { return g[0] * g[1] - g[2] * g[2]; }

static int color4(int i, int j) { return (i & 1) + 2 * (j & 1); }

/* op 0: Monge-Ampere update; op 1: Laplacian update for Lap u = F. */
static double update_value(int n, const double *u, const double *F, int i, int j, int op,
                           int *nc)
{
    const size_t p = IX2(n, i, j);
    const double s = (double)n * (double)n;
    if (op == 0) {
        double g[3];
        ma2_hessian(n, u, i, j, g);
        const double sig = ma2_local_root(g, F[p], nc);
        return u[p] + sig * (0.5 / s);
    }
    double g[3];
    ma2_hessian(n, u, i, j, g);
    return u[p] - (F[p] - (g[0] + g[1])) * (1.0 / (4.0 * s));
}

static long sweep_op(int n, double *u, const double *F, int order, int op, double *tmp)
{
    long ncount = 0;
    if (order == 2) {
        for (int j = 1; j < n; ++j)
            for (int i = 1; i < n; ++i) {
                int nc = 0;
                u[IX2(n, i, j)] = update_value(n, u, F, i, j, op, &nc);
                ncount += nc;
            }
    } else if (order == 0) {
        for (int c = 0; c < 4; ++c)
            for (int j = 1; j < n; ++j)
                for (int i = 1; i < n; ++i)
                    if (color4(i, j) == c) {
                        int nc = 0;
                        u[IX2(n, i, j)] = update_value(n, u, F, i, j, op, &nc);
                        ncount += nc;
                    }
    } else {
        /* red-black: every node of a colour from the values before the
         * colour phase */
        for (int c = 0; c < 2; ++c) {
            for (int j = 1; j < n; ++j)
                for (int i = 1; i < n; ++i)
                    if (((i + j) & 1) == c) {
                        int nc = 0;
                        tmp[IX2(n, i, j)] = update_value(n, u, F, i, j, op, &nc);
                        ncount += nc;
                    }
            for (int j = 1; j < n; ++j)
                for (int i = 1; i < n; ++i)
                    if (((i + j) & 1) == c)
                        u[IX2(n, i, j)] = tmp[IX2(n, i, j)];
        }
    }
    return ncount;
}

static double residual_op(int n, const double *u, const double *F, double *r, int op)
{
    double ss = 0.0;
    if (r)
        memset(r, 0, sizeof(double) * (size_t)(n + 1) * (size_t)(n + 1));
    for (int j = 1; j < n; ++j)
        for (int i = 1; i < n; ++i) {
            double g[3];
            ma2_hessian(n, u, i, j, g);
            const double v = F[IX2(n, i, j)] - (op == 0 ? det2(g) : g[0] + g[1]);
            if (r)
                r[IX2(n, i, j)] = v;
            ss += v * v;
        }
    return ss;
}

/* sqrt(h^2 sum r^2), the discrete L2 norm */
static double l2(int n, double ss) { return sqrt(ss / ((double)n * (double)n)); }

long ma2_sweep(int n, double *u, const double *F, int order)
{
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(n + 1) * (size_t)(n + 1));
    if (!tmp)
        return -1;
    const long nc = sweep_op(n, u, F, order, 0, tmp);
    free(tmp);
    return nc;
}

double ma2_residual(int n, const double *u, const double *F, double *r)
{
    return residual_op(n, u, F, r, 0);
}

static double restrict_point(int nf, const double *rf, int I, int J, int rmode)
{
    const int i = 2 * I, j = 2 * J;
    if (rmode == 0)
        return (4.0 * rf[IX2(nf, i, j)] + (rf[IX2(nf, i - 1, j)] + rf[IX2(nf, i + 1, j)])
                + (rf[IX2(nf, i, j - 1)] + rf[IX2(nf, i, j + 1)])) / 8.0;
    const double w[3] = {0.25, 0.5, 0.25};
    double v = 0.0;
    for (int b = -1; b <= 1; ++b)
        for (int a = -1; a <= 1; ++a)
            v += (w[b + 1] * w[a + 1]) * rf[IX2(nf, i + a, j + b)];
    return v;
}

/* FAS restriction: w_H = u_H = injection of u; b_H = S_H(w_H) + I r at
 * coarse interior nodes (0 on the boundary). */
void ma2_restrict(int nf, const double *uf, const double *rf, double *wc, double *bc, int op,
                  int rmode)
{
    const int nc = nf / 2;
    for (int J = 0; J <= nc; ++J)
        for (int I = 0; I <= nc; ++I)
            wc[IX2(nc, I, J)] = uf[IX2(nf, 2 * I, 2 * J)];
    memset(bc, 0, sizeof(double) * (size_t)(nc + 1) * (size_t)(nc + 1));
    for (int J = 1; J < nc; ++J)
        for (int I = 1; I < nc; ++I) {
            double g[3];
            ma2_hessian(nc, wc, I, J, g);
            bc[IX2(nc, I, J)] = (op == 0 ? det2(g) : g[0] + g[1])
                                + restrict_point(nf, rf, I, J, rmode);
        }
}

/* u_f += bilinear interpolation of (u_c - w_c) at fine interior nodes. */
void ma2_prolong_correct(int nf, double *uf, const double *uc, const double *wc)
{
    const int nc = nf / 2;
    for (int j = 1; j < nf; ++j)
        for (int i = 1; i < nf; ++i) {
            const int I0 = i / 2, J0 = j / 2;
            const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1;
            const double wi = (i & 1) ? 0.5 : 1.0, wj = (j & 1) ? 0.5 : 1.0;
            double d = 0.0;
            for (int b = 0; b < nj; ++b)
                for (int a = 0; a < ni; ++a)
                    d += (wj * wi) * (uc[IX2(nc, I0 + a, J0 + b)] - wc[IX2(nc, I0 + a, J0 + b)]);
            uf[IX2(nf, i, j)] += d;
        }
}

void ma2_inject(int nf, const double *vf, double *vc)
{
    const int nc = nf / 2;
    for (int J = 0; J <= nc; ++J)
        for (int I = 0; I <= nc; ++I)
            vc[IX2(nc, I, J)] = vf[IX2(nf, 2 * I, 2 * J)];
}

static int fmg_rule(int nc, int i, int *first, double *w)
{
    if ((i & 1) == 0) {
        *first = i / 2;
        w[0] = 1.0;
        return 1;
    }
    const int m = (i - 1) / 2;
    if (nc < 3) {
        *first = 0;
        w[0] = m == 0 ? 3.0 / 8.0 : -1.0 / 8.0;
        w[1] = 6.0 / 8.0;
        w[2] = m == 0 ? -1.0 / 8.0 : 3.0 / 8.0;
        return 3;
    }
    if (m == 0) {
        *first = 0;
        w[0] = 5.0 / 16.0; w[1] = 15.0 / 16.0; w[2] = -5.0 / 16.0; w[3] = 1.0 / 16.0;
    } else if (m + 1 == nc) {
        *first = nc - 3;
        w[0] = 1.0 / 16.0; w[1] = -5.0 / 16.0; w[2] = 15.0 / 16.0; w[3] = 5.0 / 16.0;
    } else {
        *first = m - 1;
        w[0] = -1.0 / 16.0; w[1] = 9.0 / 16.0; w[2] = 9.0 / 16.0; w[3] = -1.0 / 16.0;
    }
    return 4;
}

void ma2_fmg_interp(int nc, const double *uc, double *uf)
{
    const int nf = 2 * nc;
    for (int j = 1; j < nf; ++j) {
        int fj;
        double wj[4];
        const int cj = fmg_rule(nc, j, &fj, wj);
        for (int i = 1; i < nf; ++i) {
            int fi;
            double wi[4];
            const int ci = fmg_rule(nc, i, &fi, wi);
            double v = 0.0;
            for (int b = 0; b < cj; ++b)
                for (int a = 0; a < ci; ++a)
                    v += wj[b] * wi[a] * uc[IX2(nc, fi + a, fj + b)];
            uf[IX2(nf, i, j)] = v;
        }
    }
}

typedef struct {
    int L;
    int ns[M2_MAX_LEVELS];
    double *u[M2_MAX_LEVELS], *b[M2_MAX_LEVELS], *w[M2_MAX_LEVELS], *r[M2_MAX_LEVELS];
    double *tmp;
} hier2;

static void h2_free(hier2 *H)
{
    for (int l = 0; l < H->L; ++l) {
        free(H->u[l]);
        free(H->b[l]);
        free(H->w[l]);
        free(H->r[l]);
    }
    free(H->tmp);
}

static int h2_alloc(hier2 *H, int n)
{
    memset(H, 0, sizeof(*H));
    H->L = ma2_levels(n, H->ns, M2_MAX_LEVELS);
    for (int l = 0; l < H->L; ++l) {
        const size_t c = (size_t)(H->ns[l] + 1) * (size_t)(H->ns[l] + 1);
        H->u[l] = (double *)calloc(c, sizeof(double));
        H->b[l] = (double *)calloc(c, sizeof(double));
        H->w[l] = (double *)calloc(c, sizeof(double));
        H->r[l] = (double *)calloc(c, sizeof(double));
        if (!H->u[l] || !H->b[l] || !H->w[l] || !H->r[l])
            return -1;
    }
    H->tmp = (double *)calloc((size_t)(n + 1) * (size_t)(n + 1), sizeof(double));
    return H->tmp ? 0 : -1;
}

static long vcycle2(hier2 *H, int l, double *u, const double *b, const ma2_params *p)
{
    const int n = H->ns[l];
    long nc = 0;
    if (l == H->L - 1) {
        for (int s = 0; s < p->nu0; ++s)
            nc += sweep_op(n, u, b, p->order, 0, H->tmp);
        return nc;
    }
    for (int s = 0; s < p->nu1; ++s)
        nc += sweep_op(n, u, b, p->order, 0, H->tmp);
    (void)residual_op(n, u, b, H->r[l], 0);
    ma2_restrict(n, u, H->r[l], H->w[l + 1], H->b[l + 1], 0, p->rmode);
    memcpy(H->u[l + 1], H->w[l + 1],
           sizeof(double) * (size_t)(H->ns[l + 1] + 1) * (size_t)(H->ns[l + 1] + 1));
    nc += vcycle2(H, l + 1, H->u[l + 1], H->b[l + 1], p);
    ma2_prolong_correct(n, u, H->u[l + 1], H->w[l + 1]);
    for (int s = 0; s < p->nu2; ++s)
        nc += sweep_op(n, u, b, p->order, 0, H->tmp);
    return nc;
}

static long fmg2(hier2 *H, int l, double *u, const double *b, const ma2_params *p)
{
    const int n = H->ns[l];
    long nc = 0;
    if (l == H->L - 1) {
        for (int j = 1; j < n; ++j)
            for (int i = 1; i < n; ++i)
                u[IX2(n, i, j)] = 0.0;
        const int sweeps = (n == 3 && p->nu0 < 8) ? 8 : p->nu0;
        for (int s = 0; s < sweeps; ++s)
            nc += sweep_op(n, u, b, p->order, 0, H->tmp);
        return nc;
    }
    ma2_inject(n, b, H->b[l + 1]);
    ma2_inject(n, u, H->u[l + 1]);
    nc += fmg2(H, l + 1, H->u[l + 1], H->b[l + 1], p);
    ma2_fmg_interp(H->ns[l + 1], H->u[l + 1], u);
    nc += vcycle2(H, l, u, b, p);
    return nc;
}

long ma2_vcycle(int n, double *u, const double *f, const ma2_params *p)
{
    hier2 H;
    if (h2_alloc(&H, n)) {
        h2_free(&H);
        return -1;
    }
    const long nc = vcycle2(&H, 0, u, f, p);
    h2_free(&H);
    return nc;
}

long ma2_fmg(int n, double *u, const double *f, const ma2_params *p)
{
    hier2 H;
    if (h2_alloc(&H, n)) {
        h2_free(&H);
        return -1;
    }
    const long nc = fmg2(&H, 0, u, f, p);
    h2_free(&H);
    return nc;
}

/* Solve under the stopping rule of Section 4; with init = 2 the start is
 * zero inside (r^0 taken there) and one FMG-FAS iteration is cycle 1.
 * Limit mode (tol < 0) cycles until the residual stops dropping below 0.9
 * of its best for three cycles.  Returns 0 converged, 1 not, -1 on
 * allocation failure. */
int ma2_solve(int n, double *u, const double *f, const ma2_params *p, ma2_report *rep)
{
    memset(rep, 0, sizeof(*rep));
    hier2 H;
    if (h2_alloc(&H, n)) {
        h2_free(&H);
        return -1;
    }
    if (p->init == 2)
        for (int j = 1; j < n; ++j)
            for (int i = 1; i < n; ++i)
                u[IX2(n, i, j)] = 0.0;
    rep->res0 = l2(n, residual_op(n, u, f, NULL, 0));
    rep->res = rep->res0;
    int c = 0;
    if (p->init == 2) {
        rep->nonconvex += fmg2(&H, 0, u, f, p);
        rep->res = l2(n, residual_op(n, u, f, NULL, 0));
        c = 1;
    }
    rep->cycles = c;
    int status = 1;
    double best = rep->res;
    int stall = 0;
    if (p->tol >= 0.0 && rep->res <= p->tol * rep->res0)
        status = 0;
    for (; status != 0 && c < p->max_cycles; ++c) {
        rep->nonconvex += vcycle2(&H, 0, u, f, p);
        rep->cycles = c + 1;
        rep->res = l2(n, residual_op(n, u, f, NULL, 0));
        if (p->tol >= 0.0) {
            if (rep->res <= p->tol * rep->res0)
                status = 0;
        } else if (rep->res < 0.9 * best) {
            best = rep->res;
            stall = 0;
        } else if (++stall >= 3) {
            status = 0;
        }
    }
    h2_free(&H);
    rep->converged = status == 0;
    return status;
}
