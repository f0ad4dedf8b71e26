/*
 * oracle.c -- plain, slow, obviously-correct CPU reference for the multi-cell
 * stiff chemistry path (rate constants, f(y), J(y), one BDF outer step).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls this code.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source, header or table with the HIP
 * library: it reads the mechanism as plain arrays and computes everything
 * from the definitions, cell by cell, in double precision.
 *
 * What it computes (paper, Section 2 "Background"):
 *   reaction   c_1 y_1 + ... + c_m y_m -> c_{m+1} y_{m+1} + ... + c_n y_n
 *   tendency   (dy_i/dt)_j = -c_i r_j for reactants, +c_i r_j for products
 *   derivative f_i = sum_j (dy_i/dt)_j
 * Multi-cells (Section 3): every cell k has its own y_ik and f_ik and cells do
 * not interact, so the Jacobian is block-diagonal and each cell is solved on
 * its own.
 *
 * Readings where the paper is silent:
 *   - r_j is mass action, r_j = k_j * prod over reactant slots of y_s (a
 *     repeated reactant index is a stoichiometric multiplicity).
 *   - k_j = A_j exp(-theta_j / T) for thermal (Arrhenius, theta = Ea/R in K),
 *     k_j = A_j * s for photolysis (A_j is the J-rate, s a per-cell scale).
 *   - The integrator is a quasi-constant step-size, variable-order (1..5) BDF
 *     in backward-difference form (Shampine & Reichelt 1997, "The MATLAB ODE
 *     Suite", kappa = 0), with a simplified Newton iteration on a freshly
 *     evaluated Jacobian at every step attempt, the Hairer-Norsett-Wanner
 *     starting step size, and exact landing on the end of the outer step.
 *     The constants are inputs (orc_opts).
 *   - Linear systems are solved by dense Gaussian elimination with partial
 *     pivoting (a deliberately different algorithm from a sparse
 *     static-pivot factorisation).
 *
 * Layout of batch arrays: [entity][n_cells], cell index fastest.
 *
 * Parity pins (tests): finite-difference and homogeneity checks of J against
 * f, atom-balance conservation, hand-derived special cases, closed-form
 * solutions of small mechanisms, scipy.linalg.expm for linear mechanisms, an
 * independent implicit Runge-Kutta integrator (scipy Radau) on sampled
 * cells, and hand-worked values of the step-size controller (starting step,
 * rejection factor, order selection) on constructed inputs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t n_species, n_reactions;
    const int32_t *rxn_type;             /* [R] 0 thermal, 1 photolysis */
    const int32_t *reac_ptr, *reac_idx;  /* CSR over reactant slots */
    const int32_t *prod_ptr, *prod_idx;  /* CSR over products */
    const double *prod_yield;            /* [nprod] */
    const double *A, *theta;             /* [R] */
} orc_mech;

typedef struct {
    double rtol, atol;        /* weights w_i = 1 / (rtol |y_i| + atol) */
    double eta_newton;        /* Newton convergence: rho/(1-rho)*|dy| < eta */
    double safety;            /* step-size safety factor */
    double fac_min, fac_max;  /* bounds of the step-size change factor */
    double fac_newton_fail;   /* step-size factor after a Newton failure */
    double h_min_rel;         /* failure once h < h_min_rel * dt or t + h == t */
    int32_t max_order;        /* 1..5 */
    int32_t max_newton;       /* Newton iterations per attempt */
    int32_t max_steps;        /* step attempts per outer step */
    int32_t warm_start;       /* 1: start from the previous step's h_next (stats in/out) */
} orc_opts;

typedef struct {
    int32_t steps, rejects, newton_fails, newton_iters, f_evals, jac_evals, lu_count, order;
    double h_last, y_min;
    double h_next;            /* the step size chosen before the landing cut */
} orc_stats;

enum { ORC_OK = 0, ORC_TOO_MUCH_WORK = 1, ORC_CONV_FAIL = 2, ORC_ERR_FAIL = 3,
       ORC_NONFINITE = 4, ORC_SINGULAR = 5 };

#define ORC_MAXORD 5

/* ------------------------------------------------------------------ rates */

/* Rate constant of reaction j in a cell at temperature T with photolysis scale s. */
static double rate_constant(const orc_mech *m, int j, double T, double s)
{
    if (m->rxn_type[j] == 1)
        return m->A[j] * s;
    return m->A[j] * exp(-m->theta[j] / T);
}

void orc_rate_constants(const orc_mech *m, int64_t n_cells, const double *T,
                        const double *jscale, double *k)
{
    for (int j = 0; j < m->n_reactions; ++j)
        for (int64_t c = 0; c < n_cells; ++c)
            k[(int64_t)j * n_cells + c] = rate_constant(m, j, T[c], jscale[c]);
}

/* ------------------------------------------------------- one cell: f and J */

/* Reaction rate r_j = k_j * prod_{reactant slots} y_s. */
static double reaction_rate(const orc_mech *m, int j, double kj, const double *y)
{
    double r = kj;
    for (int p = m->reac_ptr[j]; p < m->reac_ptr[j + 1]; ++p)
        r *= y[m->reac_idx[p]];
    return r;
}

/* f_i = sum_j nu_ij r_j, with nu_ij = (yield as product) - (count as reactant).
 * fscale_i = sum over the same contributions of their absolute values. */
static void cell_deriv(const orc_mech *m, const double *kc, const double *y,
                       double *f, double *fscale)
{
    const int N = m->n_species;
    for (int i = 0; i < N; ++i) {
        f[i] = 0.0;
        if (fscale) fscale[i] = 0.0;
    }
    for (int j = 0; j < m->n_reactions; ++j) {
        const double r = reaction_rate(m, j, kc[j], y);
        for (int p = m->reac_ptr[j]; p < m->reac_ptr[j + 1]; ++p) {
            f[m->reac_idx[p]] -= r;
            if (fscale) fscale[m->reac_idx[p]] += fabs(r);
        }
        for (int p = m->prod_ptr[j]; p < m->prod_ptr[j + 1]; ++p) {
            f[m->prod_idx[p]] += m->prod_yield[p] * r;
            if (fscale) fscale[m->prod_idx[p]] += fabs(m->prod_yield[p] * r);
        }
    }
}

/* Dense J[i*N + s] = d f_i / d y_s.  For reaction j and reactant slot l
 * (species s = reac[l]) the partial of the rate product with respect to that
 * slot is k_j times the product of the other slots; summing over the slots
 * that hold s gives d r_j / d y_s (so 2A contributes 2 k y_A).
 * Jscale accumulates absolute values of the same contributions. */
static void cell_jac(const orc_mech *m, const double *kc, const double *y,
                     double *J, double *Jscale)
{
    const int N = m->n_species;
    memset(J, 0, sizeof(double) * (size_t)N * N);
    if (Jscale) memset(Jscale, 0, sizeof(double) * (size_t)N * N);
    for (int j = 0; j < m->n_reactions; ++j) {
        const int b = m->reac_ptr[j], e = m->reac_ptr[j + 1];
        for (int l = b; l < e; ++l) {
            double part = kc[j];
            for (int q = b; q < e; ++q)
                if (q != l) part *= y[m->reac_idx[q]];
            const int s = m->reac_idx[l];
            for (int q = b; q < e; ++q) {
                J[(size_t)m->reac_idx[q] * N + s] -= part;
                if (Jscale) Jscale[(size_t)m->reac_idx[q] * N + s] += fabs(part);
            }
            for (int q = m->prod_ptr[j]; q < m->prod_ptr[j + 1]; ++q) {
                J[(size_t)m->prod_idx[q] * N + s] += m->prod_yield[q] * part;
                if (Jscale) Jscale[(size_t)m->prod_idx[q] * N + s] += fabs(m->prod_yield[q] * part);
            }
        }
    }
}

/* ----------------------------------------------------------- batch f and J */

static void gather_cell(const double *src, int n, int64_t n_cells, int64_t c, double *dst)
{
    for (int i = 0; i < n; ++i)
        dst[i] = src[(int64_t)i * n_cells + c];
}

static void scatter_cell(const double *src, int n, int64_t n_cells, int64_t c, double *dst)
{
    for (int i = 0; i < n; ++i)
        dst[(int64_t)i * n_cells + c] = src[i];
}

/* f and its scale for every cell.  k: [R][C], y, f, fscale: [N][C]. */
void orc_deriv(const orc_mech *m, int64_t n_cells, const double *k, const double *y,
               double *f, double *fscale)
{
    const int N = m->n_species, R = m->n_reactions;
    double *kc = malloc(sizeof(double) * R), *yc = malloc(sizeof(double) * N);
    double *fc = malloc(sizeof(double) * N), *sc = malloc(sizeof(double) * N);
    for (int64_t c = 0; c < n_cells; ++c) {
        gather_cell(k, R, n_cells, c, kc);
        gather_cell(y, N, n_cells, c, yc);
        cell_deriv(m, kc, yc, fc, sc);
        scatter_cell(fc, N, n_cells, c, f);
        if (fscale) scatter_cell(sc, N, n_cells, c, fscale);
    }
    free(kc); free(yc); free(fc); free(sc);
}

/* Dense Jacobian of every cell: J, Jscale: [C][N][N] (row i, column s). */
void orc_jac(const orc_mech *m, int64_t n_cells, const double *k, const double *y,
             double *J, double *Jscale)
{
    const int N = m->n_species, R = m->n_reactions;
    double *kc = malloc(sizeof(double) * R), *yc = malloc(sizeof(double) * N);
    for (int64_t c = 0; c < n_cells; ++c) {
        gather_cell(k, R, n_cells, c, kc);
        gather_cell(y, N, n_cells, c, yc);
        cell_jac(m, kc, yc, J + (size_t)c * N * N, Jscale ? Jscale + (size_t)c * N * N : NULL);
    }
    free(kc); free(yc);
}

/* Vector-Jacobian products of f for every cell, from the definitions:
 * gy_s = sum_i v_i J_is (J from cell_jac) and, with respect to the log rate
 * constants, glnk_j = sum_i v_i d f_i / d ln k_j = sum_i v_i nu_ij r_j
 * (f is linear in each k_j, so d f / d ln k_j = nu_j r_j).
 * k: [R][C]; y, v, gy: [N][C]; glnk: [R][C]; gy or glnk may be NULL. */
void orc_vjp(const orc_mech *m, int64_t n_cells, const double *k, const double *y, const double *v,
             double *gy, double *glnk)
{
    const int N = m->n_species, R = m->n_reactions;
    double *kc = malloc(sizeof(double) * R), *yc = malloc(sizeof(double) * N);
    double *vc = malloc(sizeof(double) * N), *g = malloc(sizeof(double) * (N > R ? N : R));
    double *J = malloc(sizeof(double) * (size_t)N * N);
    for (int64_t c = 0; c < n_cells; ++c) {
        gather_cell(k, R, n_cells, c, kc);
        gather_cell(y, N, n_cells, c, yc);
        gather_cell(v, N, n_cells, c, vc);
        if (gy) {
            cell_jac(m, kc, yc, J, NULL);
            for (int s = 0; s < N; ++s) {
                double acc = 0.0;
                for (int i = 0; i < N; ++i) acc += vc[i] * J[(size_t)i * N + s];
                g[s] = acc;
            }
            scatter_cell(g, N, n_cells, c, gy);
        }
        if (glnk) {
            for (int j = 0; j < R; ++j) {
                const double r = reaction_rate(m, j, kc[j], yc);
                double acc = 0.0;
                for (int p = m->reac_ptr[j]; p < m->reac_ptr[j + 1]; ++p) acc -= vc[m->reac_idx[p]] * r;
                for (int p = m->prod_ptr[j]; p < m->prod_ptr[j + 1]; ++p)
                    acc += vc[m->prod_idx[p]] * m->prod_yield[p] * r;
                g[j] = acc;
            }
            scatter_cell(g, R, n_cells, c, glnk);
        }
    }
    free(kc); free(yc); free(vc); free(g); free(J);
}

/* -------------------------------------------- dense LU with partial pivoting */

/* In-place LU of the n x n row-major matrix a, row interchanges in piv.
 * Returns 0 on success, 1 if a pivot is zero or not finite. */
static int lu_factor(int n, double *a, int *piv)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(a[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            const double v = fabs(a[(size_t)i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        piv[k] = p;
        if (!(best > 0.0) || !isfinite(best))
            return 1;
        if (p != k)
            for (int j = 0; j < n; ++j) {
                const double t = a[(size_t)k * n + j];
                a[(size_t)k * n + j] = a[(size_t)p * n + j];
                a[(size_t)p * n + j] = t;
            }
        const double piv_val = a[(size_t)k * n + k];
        for (int i = k + 1; i < n; ++i) {
            const double l = a[(size_t)i * n + k] / piv_val;
            a[(size_t)i * n + k] = l;
            if (l != 0.0)
                for (int j = k + 1; j < n; ++j)
                    a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
        }
    }
    return 0;
}

/* Solve (LU) x = b in place, using the factors and interchanges of lu_factor. */
static void lu_solve(int n, const double *a, const int *piv, double *b)
{
    for (int k = 0; k < n; ++k)
        if (piv[k] != k) {
            const double t = b[k];
            b[k] = b[piv[k]];
            b[piv[k]] = t;
        }
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int j = 0; j < i; ++j)
            s -= a[(size_t)i * n + j] * b[j];
        b[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < n; ++j)
            s -= a[(size_t)i * n + j] * b[j];
        b[i] = s / a[(size_t)i * n + i];
    }
}

/* ------------------------------------------------------------ BDF helpers */

/* Weighted root-mean-square norm sqrt(mean((v_i w_i)^2)). */
static double wrms(int n, const double *v, const double *w)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        const double t = v[i] * w[i];
        s += t * t;
    }
    return sqrt(s / n);
}

/* gamma_j = sum_{i=1..j} 1/i, gamma_0 = 0 (BDF coefficients for kappa = 0). */
static double bdf_gamma(int j)
{
    double g = 0.0;
    for (int i = 1; i <= j; ++i)
        g += 1.0 / i;
    return g;
}

/* Re-sample the backward differences D[0..order] of the interpolating
 * polynomial from spacing h to spacing rho*h.  With
 *   R_ij(rho) = prod_{l=1..i} (l - 1 - rho*j) / l,  i, j = 0..order
 * the values at the new points are R(rho)^T D, the differences of values at
 * unit spacing are obtained with U = R(1) (an involution), so the new
 * differences are (R(rho) U)^T D. */
/* RU[j][i]: D'_i = sum_j RU[j][i] D_j (i, j <= order). */
static void rescale_matrix(int order, double rho, double RU[ORC_MAXORD + 1][ORC_MAXORD + 1])
{
    double R[ORC_MAXORD + 1][ORC_MAXORD + 1], U[ORC_MAXORD + 1][ORC_MAXORD + 1];
    const int n = order + 1;
    for (int j = 0; j < n; ++j) {
        R[0][j] = 1.0;
        U[0][j] = 1.0;
        for (int i = 1; i < n; ++i) {
            R[i][j] = R[i - 1][j] * ((i - 1) - rho * j) / i;
            U[i][j] = U[i - 1][j] * ((double)(i - 1) - (double)j) / i;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int l = 0; l < n; ++l)
                s += R[i][l] * U[l][j];
            RU[i][j] = s;
        }
}

static void rescale_differences(int N, double *D, int order, double rho)
{
    double RU[ORC_MAXORD + 1][ORC_MAXORD + 1];
    double tmp[ORC_MAXORD + 1];
    const int n = order + 1;
    rescale_matrix(order, rho, RU);
    for (int s = 0; s < N; ++s) {
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int j = 0; j < n; ++j)
                acc += RU[j][i] * D[(size_t)j * N + s];
            tmp[i] = acc;
        }
        for (int i = 0; i < n; ++i)
            D[(size_t)i * N + s] = tmp[i];
    }
}

static int all_finite(int n, const double *v)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* ------------------------------------------------- step-size controller */

/* Starting step size, first stage (Hairer, Norsett & Wanner, Vol. I,
 * Sec. II.4, starting step size algorithm, steps (a)-(b)): d0 = |y0|,
 * d1 = |f(y0)| in the weighted norm; h0 = 0.01 d0 / d1, or 1e-6 dt when
 * either is below 1e-5. */
static double start_h0(int n, const double *y0, const double *f0, const double *w, double dt)
{
    const double d0 = wrms(n, y0, w), d1 = wrms(n, f0, w);
    return (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 * dt : 0.01 * d0 / d1;
}

/* Second stage (steps (c)-(f), order p = 1): with f1 = f(y0 + h0 f0),
 * d2 = |f1 - f0| / h0, h1 = (0.01 / max(d1, d2))^(1/(p+1)), or
 * max(1e-6, 1e-3 h0) when max(d1, d2) <= 1e-15; the step is
 * min(100 h0, h1), and never beyond the end of the outer step. */
static double start_h(int n, const double *f0, const double *f1, const double *w, double h0, double dt)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        const double t = (f1[i] - f0[i]) * w[i];
        s += t * t;
    }
    const double d1 = wrms(n, f0, w), d2 = sqrt(s / n) / h0;
    const double dm = d1 > d2 ? d1 : d2;
    const double h1 = dm <= 1e-15 ? fmax(1e-6, 1e-3 * h0) : sqrt(0.01 / dm);
    return fmin(100.0 * h0, fmin(h1, dt));
}

/* Step-size factor after a failed error test of a step of the given order
 * (local error ~ h^(order+1)): safety * err^(-1/(order+1)), at least fac_min.
 * The order is kept. */
static double reject_factor(double err_norm, int order, double safety, double fac_min)
{
    double fac = safety * pow(err_norm, -1.0 / (order + 1));
    return fac < fac_min ? fac_min : fac;
}

/* Order and step-size selection once order+1 steps of equal size have been
 * accepted (Shampine & Reichelt 1997, Sec. 2.3, with kappa = 0).  D holds the
 * updated differences [order+3][n]: the error estimates of orders k-1, k and
 * k+1 are |D_k| / k, err_norm (= |d| / (k+1)) and |D_{k+2}| / (k+2); each
 * allows the factor e^(-1/(order'+1)); the largest wins, ties going to the
 * current order, then the lower one.  Returns safety * best, at most
 * fac_max, and the chosen order in *new_order. */
static double select_order(int n, const double *D, const double *w, int order, int maxord, double err_norm,
                           double safety, double fac_max, int *new_order)
{
    const double e_low = order > 1 ? wrms(n, D + (size_t)order * n, w) / order : INFINITY;
    const double e_high = order < maxord ? wrms(n, D + (size_t)(order + 2) * n, w) / (order + 2) : INFINITY;
    const double r_cur = pow(err_norm, -1.0 / (order + 1));
    const double r_low = order > 1 ? pow(e_low, -1.0 / order) : 0.0;
    const double r_high = order < maxord ? pow(e_high, -1.0 / (order + 2)) : 0.0;
    int k = order;
    double best = r_cur;
    if (r_low > best) { best = r_low; k = order - 1; }
    if (r_high > best) { best = r_high; k = order + 1; }
    *new_order = k;
    const double fac = safety * best;
    return fac > fac_max ? fac_max : fac;
}

/* --------------------------------------------------------- BDF, one cell */

typedef struct {
    double *D, *f, *w, *ypred, *psi, *d, *ycur, *rhs, *J, *tmp;
    int *piv;
} orc_work;

static void work_alloc(orc_work *wk, int N)
{
    wk->D = calloc((size_t)(ORC_MAXORD + 3) * N, sizeof(double));
    wk->f = malloc(sizeof(double) * N);
    wk->w = malloc(sizeof(double) * N);
    wk->ypred = malloc(sizeof(double) * N);
    wk->psi = malloc(sizeof(double) * N);
    wk->d = malloc(sizeof(double) * N);
    wk->ycur = malloc(sizeof(double) * N);
    wk->rhs = malloc(sizeof(double) * N);
    wk->tmp = malloc(sizeof(double) * N);
    wk->J = malloc(sizeof(double) * (size_t)N * N);
    wk->piv = malloc(sizeof(int) * N);
}

static void work_free(orc_work *wk)
{
    free(wk->D); free(wk->f); free(wk->w); free(wk->ypred); free(wk->psi);
    free(wk->d); free(wk->ycur); free(wk->rhs); free(wk->tmp); free(wk->J); free(wk->piv);
}

/* Accepting a step of order k with Newton correction d: the new differences
 * are D_{k+2} = d - D_{k+1}, D_{k+1} = d, then D_j += D_{j+1} for j = k..0. */
static void accept_differences(int N, double *D, const double *d, int order)
{
    for (int i = 0; i < N; ++i) {
        D[(size_t)(order + 2) * N + i] = d[i] - D[(size_t)(order + 1) * N + i];
        D[(size_t)(order + 1) * N + i] = d[i];
    }
    for (int j = order; j >= 0; --j)
        for (int i = 0; i < N; ++i)
            D[(size_t)j * N + i] += D[(size_t)(j + 1) * N + i];
}

/* ------------------------------------------- the step tape (reverse mode) */

/* The sequence of operations one outer step applied to the backward
 * differences, recorded so that the same discrete map can be replayed with
 * other parameters and differentiated in reverse: START (D_0 = y0,
 * D_1 = h f(y0)), RESCALE (D <- re-sampled at spacing rho * h, orders
 * 0..order), STEP (an accepted step of the given order with c = h / gamma_k,
 * followed by N values: the converged state z = the new D_0).  Each entry:
 * type, order, value, then the payload. */
enum { TAPE_START = 0, TAPE_RESCALE = 1, TAPE_STEP = 2 };
typedef struct {
    double *v;
    size_t n, cap;
} orc_tape;

static void tape_push(orc_tape *t, double x)
{
    if (t->n == t->cap) {
        t->cap = t->cap ? 2 * t->cap : 1024;
        t->v = realloc(t->v, sizeof(double) * t->cap);
    }
    t->v[t->n++] = x;
}

static void tape_op(orc_tape *t, int type, int order, double x, const double *payload, int n)
{
    if (!t) return;
    tape_push(t, type);
    tape_push(t, order);
    tape_push(t, x);
    for (int i = 0; i < n; ++i) tape_push(t, payload[i]);
}

static void rescale_differences(int N, double *D, int order, double rho);

static void rescale_rec(int N, double *D, int order, double rho, orc_tape *tape)
{
    rescale_differences(N, D, order, rho);
    tape_op(tape, TAPE_RESCALE, order, rho, NULL, 0);
}

/* Integrate y' = f(y) of one cell from t = 0 to t = dt; y is overwritten
 * with y(dt).  h_warm > 0 (finite): the first step size, taken at order 1
 * instead of the starting-step algorithm (a warm start from the previous
 * outer step's h_next; the paper's per-cell calls re-initialise the solver
 * every time, Section 3).  Returns an ORC_* status. */
static int cell_solve(const orc_mech *m, const double *kc, double *y, double dt,
                      const orc_opts *o, orc_stats *st, orc_work *wk, orc_tape *tape, double h_warm)
{
    const int N = m->n_species;
    const int maxord = o->max_order < 1 ? 1 : (o->max_order > ORC_MAXORD ? ORC_MAXORD : o->max_order);
    double *D = wk->D;
    memset(st, 0, sizeof(*st));
    memset(D, 0, sizeof(double) * (size_t)(ORC_MAXORD + 3) * N);

    /* starting step size (Hairer, Norsett & Wanner, Vol. I, Sec. II.4, p = 1) */
    cell_deriv(m, kc, y, wk->f, NULL);
    st->f_evals++;
    if (!all_finite(N, y) || !all_finite(N, wk->f))
        return ORC_NONFINITE;
    double h;
    if (h_warm > 0.0 && isfinite(h_warm)) {
        h = fmin(h_warm, dt);
    } else {
        for (int i = 0; i < N; ++i)
            wk->w[i] = 1.0 / (o->rtol * fabs(y[i]) + o->atol);
        const double h0 = start_h0(N, y, wk->f, wk->w, dt);
        for (int i = 0; i < N; ++i)
            wk->ycur[i] = y[i] + h0 * wk->f[i];
        cell_deriv(m, kc, wk->ycur, wk->tmp, NULL);
        st->f_evals++;
        h = start_h(N, wk->f, wk->tmp, wk->w, h0, dt);
    }
    if (!(h > 0.0) || !isfinite(h))
        return ORC_NONFINITE;

    for (int i = 0; i < N; ++i) {
        D[i] = y[i];
        D[(size_t)N + i] = h * wk->f[i];
    }
    tape_op(tape, TAPE_START, 0, h, NULL, 0);
    int order = 1, n_equal = 0, attempts = 0;
    double t = 0.0, h_uncut = 0.0, h_next = 0.0;

    while (t < dt) {
        /* one accepted step: attempts until the error test passes */
        int accepted = 0, landing = 0;
        double err_norm = 0.0;
        while (!accepted) {
            if (attempts >= o->max_steps) {
                for (int i = 0; i < N; ++i) y[i] = D[i];
                st->order = order; st->h_last = h; st->h_next = h;
                return ORC_TOO_MUCH_WORK;
            }
            attempts++;
            landing = 0;
            if (h >= dt - t) {
                const double hn = dt - t;
                h_uncut = h;
                rescale_rec(N, D, order, hn / h, tape);
                h = hn;
                n_equal = 0;
                landing = 1;
            }
            const double gk = bdf_gamma(order);
            const double c = h / gk;
            for (int i = 0; i < N; ++i) {
                double yp = 0.0, ps = 0.0;
                for (int j = 0; j <= order; ++j)
                    yp += D[(size_t)j * N + i];
                for (int j = 1; j <= order; ++j)
                    ps += bdf_gamma(j) * D[(size_t)j * N + i];
                wk->ypred[i] = yp;
                wk->psi[i] = ps / gk;
                wk->w[i] = 1.0 / (o->rtol * fabs(D[i]) + o->atol);
                wk->d[i] = 0.0;
            }
            /* Newton matrix M = I - c J(ypred) */
            cell_jac(m, kc, wk->ypred, wk->J, NULL);
            st->jac_evals++;
            for (size_t q = 0; q < (size_t)N * N; ++q)
                wk->J[q] = -c * wk->J[q];
            for (int i = 0; i < N; ++i)
                wk->J[(size_t)i * N + i] += 1.0;
            st->lu_count++;
            int converged = 0, singular = lu_factor(N, wk->J, wk->piv);
            if (!singular) {
                double nrm_old = 0.0;
                for (int it = 0; it < o->max_newton; ++it) {
                    for (int i = 0; i < N; ++i)
                        wk->ycur[i] = wk->ypred[i] + wk->d[i];
                    cell_deriv(m, kc, wk->ycur, wk->f, NULL);
                    st->f_evals++;
                    if (!all_finite(N, wk->f)) break;
                    for (int i = 0; i < N; ++i)
                        wk->rhs[i] = c * wk->f[i] - wk->psi[i] - wk->d[i];
                    lu_solve(N, wk->J, wk->piv, wk->rhs);
                    st->newton_iters++;
                    const double nrm = wrms(N, wk->rhs, wk->w);
                    if (!isfinite(nrm)) break;
                    double rho = 0.0;
                    if (it >= 1) {
                        rho = nrm / nrm_old;
                        if (rho >= 1.0) break;
                    }
                    for (int i = 0; i < N; ++i)
                        wk->d[i] += wk->rhs[i];
                    if (nrm == 0.0 || (it >= 1 && rho / (1.0 - rho) * nrm < o->eta_newton)) {
                        converged = 1;
                        break;
                    }
                    nrm_old = nrm;
                }
            }
            if (!converged) {
                st->newton_fails++;
                rescale_rec(N, D, order, o->fac_newton_fail, tape);
                h *= o->fac_newton_fail;
                n_equal = 0;
                if (h < o->h_min_rel * dt || t + h == t) {
                    for (int i = 0; i < N; ++i) y[i] = D[i];
                    st->order = order; st->h_last = h; st->h_next = h;
                    return singular ? ORC_SINGULAR : ORC_CONV_FAIL;
                }
                continue;
            }
            /* local error estimate: d / (order + 1) */
            err_norm = wrms(N, wk->d, wk->w) / (order + 1);
            if (err_norm > 1.0) {
                st->rejects++;
                const double fac = reject_factor(err_norm, order, o->safety, o->fac_min);
                rescale_rec(N, D, order, fac, tape);
                h *= fac;
                n_equal = 0;
                if (h < o->h_min_rel * dt || t + h == t) {
                    for (int i = 0; i < N; ++i) y[i] = D[i];
                    st->order = order; st->h_last = h; st->h_next = h;
                    return ORC_ERR_FAIL;
                }
                continue;
            }
            accepted = 1;
        }
        /* accept: t advances, differences are updated */
        t = landing ? dt : t + h;
        if (t >= dt) h_next = landing ? h_uncut : h;
        st->steps++;
        accept_differences(N, D, wk->d, order);
        tape_op(tape, TAPE_STEP, order, h / bdf_gamma(order), D, N);  /* z = the new D_0 */
        n_equal++;
        if (t >= dt)
            break;
        if (n_equal < order + 1)
            continue;
        /* order and step-size selection after order+1 steps at constant h */
        int new_order;
        const double fac = select_order(N, D, wk->w, order, maxord, err_norm, o->safety, o->fac_max, &new_order);
        order = new_order;
        rescale_rec(N, D, order, fac, tape);
        h *= fac;
        n_equal = 0;
    }
    double ymin = INFINITY;
    for (int i = 0; i < N; ++i) {
        y[i] = D[i];
        if (D[i] < ymin) ymin = D[i];
    }
    st->order = order;
    st->h_last = h;
    st->y_min = ymin;
    st->h_next = h_next;
    return all_finite(N, y) ? ORC_OK : ORC_NONFINITE;
}

/* One outer step of length dt for every cell.  k: [R][C]; y: [N][C] in/out;
 * status: [C]; stats: [C] (may be NULL; with o->warm_start each record's
 * h_next is read as the cell's first step size, then the record is
 * overwritten).  n_threads <= 0: OpenMP default.
 * Returns the number of cells whose status is not ORC_OK. */
int orc_solve(const orc_mech *m, int64_t n_cells, const double *k, double *y, double dt,
              const orc_opts *o, int32_t *status, orc_stats *stats, int n_threads)
{
    const int N = m->n_species, R = m->n_reactions;
    int failed = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel reduction(+:failed)
    {
        orc_work wk;
        work_alloc(&wk, N);
        double *kc = malloc(sizeof(double) * R), *yc = malloc(sizeof(double) * N);
#pragma omp for schedule(dynamic, 16)
        for (int64_t c = 0; c < n_cells; ++c) {
            orc_stats st;
            gather_cell(k, R, n_cells, c, kc);
            gather_cell(y, N, n_cells, c, yc);
            const double h_warm = o->warm_start && stats ? stats[c].h_next : 0.0;
            const int s = cell_solve(m, kc, yc, dt, o, &st, &wk, NULL, h_warm);
            scatter_cell(yc, N, n_cells, c, y);
            status[c] = s;
            if (stats) stats[c] = st;
            failed += s != ORC_OK;
        }
        free(kc); free(yc);
        work_free(&wk);
    }
    return failed;
}

/* ------------------------------------ replay and adjoint of a taped step */

orc_tape *orc_tape_new(void) { return calloc(1, sizeof(orc_tape)); }
void orc_tape_free(orc_tape *t)
{
    if (t) free(t->v);
    free(t);
}
int64_t orc_tape_size(const orc_tape *t) { return (int64_t)t->n; }
/* The tape's entries: type, order, value, then (a step) the N state values. */
const double *orc_tape_data(const orc_tape *t) { return t->v; }
/* Replace a tape's entries by n given values (a tape recorded elsewhere). */
void orc_tape_assign(orc_tape *t, const double *v, int64_t n)
{
    t->n = 0;
    for (int64_t i = 0; i < n; ++i) tape_push(t, v[i]);
}

/* One outer step of one cell as cell_solve, recording the tape.  kc [R],
 * y [N] in/out; st out (with o->warm_start, st->h_next in). */
int orc_cell_solve_taped(const orc_mech *m, const double *kc, double *y, double dt, const orc_opts *o,
                         orc_stats *st, orc_tape *tape)
{
    orc_work wk;
    work_alloc(&wk, m->n_species);
    tape->n = 0;
    const double h_warm = o->warm_start ? st->h_next : 0.0;
    const int s = cell_solve(m, kc, y, dt, o, st, &wk, tape, h_warm);
    work_free(&wk);
    return s;
}

/* Newton matrix M = I - c J(z), factored. */
static int newton_matrix_at(const orc_mech *m, const double *kc, const double *z, double c, double *J, int *piv)
{
    const int N = m->n_species;
    cell_jac(m, kc, z, J, NULL);
    for (size_t q = 0; q < (size_t)N * N; ++q) J[q] = -c * J[q];
    for (int i = 0; i < N; ++i) J[(size_t)i * N + i] += 1.0;
    return lu_factor(N, J, piv);
}

/* The taped discrete map with the step sequence frozen: the same operations
 * on the differences, every implicit step solved again with these kc and y0
 * by Newton's method with a fresh Jacobian per iteration until the
 * correction stops changing (at most 50 iterations).  Writes y(dt) and a
 * copy of the tape whose STEP payloads are the replay's converged states
 * (the points the adjoint linearises at).  Returns 0, or 1 if a solve fails. */
int orc_cell_replay(const orc_mech *m, const double *kc, const double *y0, const orc_tape *tape, double *y,
                    orc_tape *out)
{
    const int N = m->n_species;
    double *D = calloc((size_t)(ORC_MAXORD + 3) * N, sizeof(double));
    double *ypred = malloc(sizeof(double) * N), *psi = malloc(sizeof(double) * N), *d = malloc(sizeof(double) * N);
    double *z = malloc(sizeof(double) * N), *f = malloc(sizeof(double) * N), *r = malloc(sizeof(double) * N);
    double *J = malloc(sizeof(double) * (size_t)N * N);
    int *piv = malloc(sizeof(int) * N), bad = 0;
    out->n = 0;
    size_t p = 0;
    while (p < tape->n && !bad) {
        const int type = (int)tape->v[p], order = (int)tape->v[p + 1];
        const double x = tape->v[p + 2];
        p += 3;
        if (type == TAPE_START) {
            cell_deriv(m, kc, y0, f, NULL);
            memset(D, 0, sizeof(double) * (size_t)(ORC_MAXORD + 3) * N);
            for (int i = 0; i < N; ++i) {
                D[i] = y0[i];
                D[(size_t)N + i] = x * f[i];
            }
            tape_op(out, TAPE_START, 0, x, NULL, 0);
        } else if (type == TAPE_RESCALE) {
            rescale_rec(N, D, order, x, out);
        } else {
            const int k = order;
            const double c = x, gk = bdf_gamma(k);
            for (int i = 0; i < N; ++i) {
                double yp = 0.0, ps = 0.0;
                for (int j = 0; j <= k; ++j) yp += D[(size_t)j * N + i];
                for (int j = 1; j <= k; ++j) ps += bdf_gamma(j) * D[(size_t)j * N + i];
                ypred[i] = yp;
                psi[i] = ps / gk;
                d[i] = tape->v[p + i] - yp;  /* start from the taped state */
            }
            p += N;
            /* Newton on d - c f(ypred + d) + psi = 0 */
            for (int it = 0; it < 50; ++it) {
                for (int i = 0; i < N; ++i) z[i] = ypred[i] + d[i];
                cell_deriv(m, kc, z, f, NULL);
                for (int i = 0; i < N; ++i) r[i] = c * f[i] - psi[i] - d[i];
                if (newton_matrix_at(m, kc, z, c, J, piv)) { bad = 1; break; }
                lu_solve(N, J, piv, r);
                double nr = 0.0;  /* largest correction relative to its own component */
                for (int i = 0; i < N; ++i) {
                    d[i] += r[i];
                    nr = fmax(nr, fabs(r[i]) / (fabs(ypred[i] + d[i]) + 1e-300));
                }
                if (nr <= 1e-15) break;
            }
            accept_differences(N, D, d, k);
            tape_op(out, TAPE_STEP, k, c, D, N);
        }
    }
    for (int i = 0; i < N; ++i) y[i] = D[i];
    free(D); free(ypred); free(psi); free(d); free(z); free(f); free(r); free(J); free(piv);
    return bad;
}

/* lam += c * (d f / d ln k)^T mu at z: lam_j += c r_j(z) sum_i nu_ij mu_i. */
static void add_lnk_term(const orc_mech *m, const double *kc, const double *z, const double *mu, double c,
                         double *glnk)
{
    for (int j = 0; j < m->n_reactions; ++j) {
        const double r = reaction_rate(m, j, kc[j], z);
        double w = 0.0;
        for (int q = m->reac_ptr[j]; q < m->reac_ptr[j + 1]; ++q) w -= mu[m->reac_idx[q]];
        for (int q = m->prod_ptr[j]; q < m->prod_ptr[j + 1]; ++q) w += m->prod_yield[q] * mu[m->prod_idx[q]];
        glnk[j] += c * r * w;
    }
}

/* Reverse sweep of a replayed tape (the discrete adjoint of the frozen
 * step sequence).  lam [N]: in, dL/dy(dt); out, dL/dy0.  glnk [R]: out,
 * dL/d ln k_j.  Each STEP is linearised at its taped converged state z: the
 * implicit step d - c f(ypred + d) + psi = 0 gives mu = (I - c J(z))^-T lam_d,
 * then lam_ypred = c J(z)^T mu, lam_psi = -mu, glnk += c (df/dlnk)^T mu. */
void orc_cell_adjoint(const orc_mech *m, const double *kc, const double *y0, const orc_tape *tape, double *lam,
                      double *glnk)
{
    const int N = m->n_species, R = m->n_reactions, NW = ORC_MAXORD + 3;
    double *L = calloc((size_t)NW * N, sizeof(double));
    double *mu = malloc(sizeof(double) * N), *g = malloc(sizeof(double) * N);
    double *J = malloc(sizeof(double) * (size_t)N * N), *Jt = malloc(sizeof(double) * (size_t)N * N);
    int *piv = malloc(sizeof(int) * N);
    for (int j = 0; j < R; ++j) glnk[j] = 0.0;
    for (int i = 0; i < N; ++i) L[i] = lam[i];  /* y(dt) = D_0 */
    /* entry offsets, walked backwards */
    size_t cap = 64, ne = 0, p = 0;
    size_t *at = malloc(sizeof(size_t) * cap);
    while (p < tape->n) {
        if (ne == cap) at = realloc(at, sizeof(size_t) * (cap *= 2));
        at[ne++] = p;
        p += 3 + ((int)tape->v[p] == TAPE_STEP ? (size_t)N : 0);
    }
    for (size_t e = ne; e-- > 0;) {
        const size_t q = at[e];
        const int type = (int)tape->v[q], order = (int)tape->v[q + 1];
        const double x = tape->v[q + 2];
        if (type == TAPE_RESCALE) {
            double RU[ORC_MAXORD + 1][ORC_MAXORD + 1], tmp[ORC_MAXORD + 1];
            rescale_matrix(order, x, RU);
            for (int s = 0; s < N; ++s) {
                for (int j = 0; j <= order; ++j) {
                    double acc = 0.0;
                    for (int i = 0; i <= order; ++i) acc += RU[j][i] * L[(size_t)i * N + s];
                    tmp[j] = acc;
                }
                for (int j = 0; j <= order; ++j) L[(size_t)j * N + s] = tmp[j];
            }
        } else if (type == TAPE_START) {
            /* D_0 = y0, D_1 = h f(y0) */
            cell_jac(m, kc, y0, J, NULL);
            for (int s = 0; s < N; ++s) {
                double acc = 0.0;
                for (int i = 0; i < N; ++i) acc += J[(size_t)i * N + s] * L[(size_t)N + i];
                lam[s] = L[s] + x * acc;
            }
            add_lnk_term(m, kc, y0, L + N, x, glnk);
        } else {
            const int k = order;
            const double c = x, gk = bdf_gamma(k);
            const double *z = tape->v + q + 3;
            /* the difference update, reversed */
            for (int j = 0; j <= k; ++j)
                for (int i = 0; i < N; ++i) L[(size_t)(j + 1) * N + i] += L[(size_t)j * N + i];
            for (int i = 0; i < N; ++i) {
                mu[i] = L[(size_t)(k + 1) * N + i] + L[(size_t)(k + 2) * N + i];  /* lam_d */
                L[(size_t)(k + 1) * N + i] = -L[(size_t)(k + 2) * N + i];
                L[(size_t)(k + 2) * N + i] = 0.0;
            }
            /* mu = (I - c J(z))^-T lam_d: solve with the transposed matrix */
            cell_jac(m, kc, z, Jt, NULL);  /* Jt holds J(z) */
            {
                double *Mt = malloc(sizeof(double) * (size_t)N * N);
                for (int i = 0; i < N; ++i)
                    for (int j = 0; j < N; ++j) Mt[(size_t)i * N + j] = (i == j ? 1.0 : 0.0) - c * Jt[(size_t)j * N + i];
                lu_factor(N, Mt, piv);
                lu_solve(N, Mt, piv, mu);
                free(Mt);
            }
            /* lam_ypred = c J^T mu, lam_psi = -mu */
            for (int s = 0; s < N; ++s) {
                double acc = 0.0;
                for (int i = 0; i < N; ++i) acc += Jt[(size_t)i * N + s] * mu[i];
                g[s] = c * acc;
            }
            add_lnk_term(m, kc, z, mu, c, glnk);
            for (int j = 0; j <= k; ++j)
                for (int i = 0; i < N; ++i) L[(size_t)j * N + i] += g[i];
            for (int j = 1; j <= k; ++j)
                for (int i = 0; i < N; ++i) L[(size_t)j * N + i] -= bdf_gamma(j) / gk * mu[i];
        }
    }
    free(at); free(L); free(mu); free(g); free(J); free(Jt); free(piv);
}

/* ----------------------------------------------- Multi-cells (Section 3) */

/* The Multi-cells reading: all C cells form one ODE system of N*C unknowns
 * (cell c's species i at c*N + i), integrated with the same BDF steps as
 * cell_solve but with one shared t, h and order, every WRMS norm taken over
 * all N*C components, and one Newton iteration for the whole system.  Cells
 * do not interact, so the Jacobian is block-diagonal: the Newton matrix is
 * factorised block by block (the same elimination that dense LU with partial
 * pivoting performs on the whole matrix, whose pivot search never leaves a
 * block).  k: [R][C], y: [N][C] in/out; one status and one stats record for
 * the whole system.  Every call starts afresh (o->warm_start is not used). */
int orc_solve_multicell(const orc_mech *m, int64_t n_cells, const double *k, double *y, double dt,
                        const orc_opts *o, orc_stats *st)
{
    const int N = m->n_species, R = m->n_reactions, C = (int)n_cells;
    const int NC = N * C;
    const int maxord = o->max_order < 1 ? 1 : (o->max_order > ORC_MAXORD ? ORC_MAXORD : o->max_order);
    double *kc = malloc(sizeof(double) * (size_t)R * C);   /* cell-major copies */
    double *Y = malloc(sizeof(double) * NC);
    double *D = calloc((size_t)(ORC_MAXORD + 3) * NC, sizeof(double));
    double *f = malloc(sizeof(double) * NC), *w = malloc(sizeof(double) * NC);
    double *ypred = malloc(sizeof(double) * NC), *psi = malloc(sizeof(double) * NC);
    double *d = malloc(sizeof(double) * NC), *ycur = malloc(sizeof(double) * NC);
    double *rhs = malloc(sizeof(double) * NC), *tmp = malloc(sizeof(double) * NC);
    double *J = malloc(sizeof(double) * (size_t)N * N * C);
    int *piv = malloc(sizeof(int) * NC);
    int status = ORC_OK;
    memset(st, 0, sizeof(*st));
    for (int c = 0; c < C; ++c) {
        gather_cell(k, R, n_cells, c, kc + (size_t)c * R);
        gather_cell(y, N, n_cells, c, Y + (size_t)c * N);
    }
#define SYS_DERIV(yin, fout)                                                          \
    for (int c = 0; c < C; ++c)                                                       \
        cell_deriv(m, kc + (size_t)c * R, (yin) + (size_t)c * N, (fout) + (size_t)c * N, NULL);

    SYS_DERIV(Y, f);
    st->f_evals++;
    double h = 0.0;
    int order = 1;
    if (!all_finite(NC, Y) || !all_finite(NC, f)) {
        status = ORC_NONFINITE;
        goto done;
    }
    for (int i = 0; i < NC; ++i) w[i] = 1.0 / (o->rtol * fabs(Y[i]) + o->atol);
    {
        const double h0 = start_h0(NC, Y, f, w, dt);
        for (int i = 0; i < NC; ++i) ycur[i] = Y[i] + h0 * f[i];
        SYS_DERIV(ycur, tmp);
        st->f_evals++;
        h = start_h(NC, f, tmp, w, h0, dt);
    }
    if (!(h > 0.0) || !isfinite(h)) {
        status = ORC_NONFINITE;
        h = 0.0;
        goto done;
    }
    for (int i = 0; i < NC; ++i) {
        D[i] = Y[i];
        D[(size_t)NC + i] = h * f[i];
    }
    {
        int n_equal = 0, attempts = 0;
        double t = 0.0;
        while (t < dt) {
            int accepted = 0, landing = 0;
            double err_norm = 0.0;
            while (!accepted) {
                if (attempts >= o->max_steps) {
                    status = ORC_TOO_MUCH_WORK;
                    goto finish;
                }
                attempts++;
                landing = 0;
                if (h >= dt - t) {
                    const double hn = dt - t;
                    rescale_differences(NC, D, order, hn / h);
                    h = hn;
                    n_equal = 0;
                    landing = 1;
                }
                const double gk = bdf_gamma(order);
                const double cc = h / gk;
                for (int i = 0; i < NC; ++i) {
                    double yp = 0.0, ps = 0.0;
                    for (int j = 0; j <= order; ++j) yp += D[(size_t)j * NC + i];
                    for (int j = 1; j <= order; ++j) ps += bdf_gamma(j) * D[(size_t)j * NC + i];
                    ypred[i] = yp;
                    psi[i] = ps / gk;
                    w[i] = 1.0 / (o->rtol * fabs(D[i]) + o->atol);
                    d[i] = 0.0;
                }
                /* block-diagonal Newton matrix, one N x N block per cell */
                int singular = 0;
                for (int c = 0; c < C; ++c) {
                    double *Jc = J + (size_t)c * N * N;
                    cell_jac(m, kc + (size_t)c * R, ypred + (size_t)c * N, Jc, NULL);
                    for (size_t q = 0; q < (size_t)N * N; ++q) Jc[q] = -cc * Jc[q];
                    for (int i = 0; i < N; ++i) Jc[(size_t)i * N + i] += 1.0;
                    singular |= lu_factor(N, Jc, piv + (size_t)c * N);
                }
                st->jac_evals++;
                st->lu_count++;
                int converged = 0;
                if (!singular) {
                    double nrm_old = 0.0;
                    for (int it = 0; it < o->max_newton; ++it) {
                        for (int i = 0; i < NC; ++i) ycur[i] = ypred[i] + d[i];
                        SYS_DERIV(ycur, f);
                        st->f_evals++;
                        if (!all_finite(NC, f)) break;
                        for (int i = 0; i < NC; ++i) rhs[i] = cc * f[i] - psi[i] - d[i];
                        for (int c = 0; c < C; ++c)
                            lu_solve(N, J + (size_t)c * N * N, piv + (size_t)c * N, rhs + (size_t)c * N);
                        st->newton_iters++;
                        const double nrm = wrms(NC, rhs, w);
                        if (!isfinite(nrm)) break;
                        double rho = 0.0;
                        if (it >= 1) {
                            rho = nrm / nrm_old;
                            if (rho >= 1.0) break;
                        }
                        for (int i = 0; i < NC; ++i) d[i] += rhs[i];
                        if (nrm == 0.0 || (it >= 1 && rho / (1.0 - rho) * nrm < o->eta_newton)) {
                            converged = 1;
                            break;
                        }
                        nrm_old = nrm;
                    }
                }
                if (!converged) {
                    st->newton_fails++;
                    rescale_differences(NC, D, order, o->fac_newton_fail);
                    h *= o->fac_newton_fail;
                    n_equal = 0;
                    if (h < o->h_min_rel * dt || t + h == t) {
                        status = singular ? ORC_SINGULAR : ORC_CONV_FAIL;
                        goto finish;
                    }
                    continue;
                }
                err_norm = wrms(NC, d, w) / (order + 1);
                if (err_norm > 1.0) {
                    st->rejects++;
                    const double fac = reject_factor(err_norm, order, o->safety, o->fac_min);
                    rescale_differences(NC, D, order, fac);
                    h *= fac;
                    n_equal = 0;
                    if (h < o->h_min_rel * dt || t + h == t) {
                        status = ORC_ERR_FAIL;
                        goto finish;
                    }
                    continue;
                }
                accepted = 1;
            }
            t = landing ? dt : t + h;
            st->steps++;
            for (int i = 0; i < NC; ++i) {
                D[(size_t)(order + 2) * NC + i] = d[i] - D[(size_t)(order + 1) * NC + i];
                D[(size_t)(order + 1) * NC + i] = d[i];
            }
            for (int j = order; j >= 0; --j)
                for (int i = 0; i < NC; ++i) D[(size_t)j * NC + i] += D[(size_t)(j + 1) * NC + i];
            n_equal++;
            if (t >= dt) break;
            if (n_equal < order + 1) continue;
            int new_order;
            const double fac = select_order(NC, D, w, order, maxord, err_norm, o->safety, o->fac_max, &new_order);
            order = new_order;
            rescale_differences(NC, D, order, fac);
            h *= fac;
            n_equal = 0;
        }
    }
finish:
    {
        double ymin = INFINITY;
        for (int i = 0; i < NC; ++i) {
            Y[i] = D[i];
            if (D[i] < ymin) ymin = D[i];
        }
        if (status == ORC_OK) st->y_min = ymin;  /* as cell_solve: only after a normal finish */
        if (status == ORC_OK && !all_finite(NC, Y)) status = ORC_NONFINITE;
        for (int c = 0; c < C; ++c) scatter_cell(Y + (size_t)c * N, N, n_cells, c, y);
    }
done:
#undef SYS_DERIV
    st->order = order;
    st->h_last = h;
    free(kc); free(Y); free(D); free(f); free(w); free(ypred); free(psi); free(d); free(ycur);
    free(rhs); free(tmp); free(J); free(piv);
    return status;
}

/* Number of OpenMP threads a parallel region would use. */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------- pieces exported for pinning */

/* Re-sample the backward differences D[(order+1)][N] to spacing rho*h. */
void orc_rescale_differences(int32_t N, double *D, int32_t order, double rho)
{
    rescale_differences(N, D, order, rho);
}

/* Solve the dense n x n row-major system a x = b (a is overwritten by its
 * factors, b by x).  Returns 0, or 1 if a pivot is zero or not finite. */
int orc_dense_solve(int32_t n, double *a, double *b)
{
    int *piv = malloc(sizeof(int) * (size_t)n);
    const int s = lu_factor(n, a, piv);
    if (!s)
        lu_solve(n, a, piv, b);
    free(piv);
    return s;
}

/* The step-size controller's pieces, exported for pinning: the two stages
 * of the starting step (n components, weights w), the factor after a failed
 * error test, and the order and step-size selection on a difference table
 * D [order+3][n].  The per-cell and the Multi-cells solves both call these. */
double orc_start_h0(int32_t n, const double *y0, const double *f0, const double *w, double dt)
{
    return start_h0(n, y0, f0, w, dt);
}

double orc_start_h(int32_t n, const double *f0, const double *f1, const double *w, double h0, double dt)
{
    return start_h(n, f0, f1, w, h0, dt);
}

double orc_reject_factor(double err_norm, int32_t order, double safety, double fac_min)
{
    return reject_factor(err_norm, order, safety, fac_min);
}

double orc_select_order(int32_t n, const double *D, const double *w, int32_t order, int32_t maxord, double err_norm,
                        double safety, double fac_max, int32_t *new_order)
{
    int k;
    const double fac = select_order(n, D, w, order, maxord, err_norm, safety, fac_max, &k);
    *new_order = k;
    return fac;
}
