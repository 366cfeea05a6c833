/*
 * FP64 CPU oracle for the box-constrained Euclidean median solved by
 * EM-ADMM, the IRLS method for its smooth surrogate, and the Non-Local
 * Euclidean Medians (NLEM) denoiser with the Non-Local Means estimate it is
 * compared with and optionally started from.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header or constant with the
 * GPU library.
 *
 * Source: K. N. Chaudhury and K. R. Ramakrishnan, "A new ADMM algorithm for
 * the Euclidean median and its application to robust patch regression"
 * (arXiv:1501.03879).
 *
 * Everything is IEEE binary64 with round-to-nearest, no fast-math, points
 * summed sequentially k = 1..n exactly in the order Algorithm 1 gives.
 * Readings where the paper is silent (stopping rule, tolerance scale, border
 * handling, flags) are stated next to the code that implements them.
 *
 * Parity unpinned: the NLEM output after a finite number of iterations at
 * image scale is checked only through its parts (weights, patches, window,
 * centre pixel, one-step and converged pins); the paper prints no per-pixel
 * values to compare with.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_CONVERGED 1
#define OR_MAXITER 2
#define OR_EMPTY 4
#define OR_BAD_INPUT 8

#define OR_INIT_GIVEN 0
#define OR_INIT_MAXW 1
#define OR_INIT_WMEAN 2

/*
 * Proximal map of f(x) = lambda * ||x - u||_2, equation (closed-form):
 *   Psi_lambda(v, u) = v - min(lambda, ||v - u||) (v - u) / ||v - u||.
 * When ||v - u|| <= lambda the minimum picks ||v - u|| and the result is u
 * exactly; this also covers v = u, where the printed quotient is 0/0.
 */
void oracle_prox(int64_t d, const double *v, const double *u, double lambda, double *out)
{
    double nu2 = 0.0;
    for (int64_t j = 0; j < d; ++j) {
        double t = v[j] - u[j];
        nu2 += t * t;
    }
    double nu = sqrt(nu2);
    if (nu <= lambda) {
        for (int64_t j = 0; j < d; ++j) out[j] = u[j];
    } else {
        for (int64_t j = 0; j < d; ++j) out[j] = v[j] - lambda * (v[j] - u[j]) / nu;
    }
}

/* Coordinate-wise projection onto the box [lo, hi]^d (Section 3). */
static double clamp_box(double x, double lo, double hi)
{
    if (x < lo) return lo;
    if (x > hi) return hi;
    return x;
}

/*
 * The convex set C of (EM).  Section 3 uses a box; the general statement of
 * (EM) allows any closed convex set, and the Euclidean ball
 * {z : ||z - center|| <= radius} is the other set with a closed-form
 * projection supported here: P(z) = center + (z - center) min(1, radius /
 * ||z - center||).  center != NULL selects the ball.
 */
typedef struct {
    const double *lo, *hi;   /* box bounds per coordinate */
    const double *center;    /* ball centre (d values) or NULL */
    double radius;           /* ball radius (>= 0, may be +inf) */
} or_set_t;

static void project_set(const or_set_t *C, int64_t d, const double *m, double *out)
{
    if (C->center) {
        double q = 0.0;
        for (int64_t j = 0; j < d; ++j) {
            double t = m[j] - C->center[j];
            q += t * t;
        }
        double nr = sqrt(q);
        double f = (nr > C->radius) ? C->radius / nr : 1.0;
        for (int64_t j = 0; j < d; ++j) out[j] = C->center[j] + (m[j] - C->center[j]) * f;
    } else {
        for (int64_t j = 0; j < d; ++j) out[j] = clamp_box(m[j], C->lo[j], C->hi[j]);
    }
}

/*
 * Scale D of the relative stopping tolerance: the largest box width
 * max_j (hi_j - lo_j) (hi - lo for a scalar box), or the ball's diameter,
 * when it is finite and positive; otherwise max(1, max_k ||a_k||_inf).
 */
static double tol_scale_set(int64_t n, int64_t d, const double *a, const or_set_t *C)
{
    double wmax = 0.0;
    if (C->center) {
        wmax = 2.0 * C->radius;
    } else {
        for (int64_t j = 0; j < d; ++j) {
            double wj = C->hi[j] - C->lo[j];
            if (!(wj <= wmax)) wmax = wj;   /* also takes inf */
        }
    }
    if (isfinite(wmax) && wmax > 0.0) return wmax;
    double m = 1.0;
    for (int64_t i = 0; i < n * d; ++i) {
        double t = fabs(a[i]);
        if (t > m) m = t;
    }
    return m;
}

/* A box is valid when lo_j <= hi_j (no NaN); a ball when its centre is finite
 * and its radius >= 0 (not NaN). */
static int set_ok(int64_t d, const or_set_t *C)
{
    if (C->center) {
        if (!(C->radius >= 0.0)) return 0;
        for (int64_t j = 0; j < d; ++j)
            if (!isfinite(C->center[j])) return 0;
        return 1;
    }
    for (int64_t j = 0; j < d; ++j)
        if (!(C->lo[j] <= C->hi[j])) return 0;
    return 1;
}

/*
 * EM-ADMM (Section 2, Algorithm 1).
 *
 * The splitting of equation (splitting) gives every term of (EM) its own copy
 * x_k of the variable and ties the copies to one global z in C:
 *
 *     minimise  sum_k w_k ||x_k - a_k||  +  i_C(z)     subject to  x_k = z  (all k),
 *
 * i_C the indicator of C.  With a multiplier y_k and a penalty rho_k for the
 * constraint of point k, the augmented Lagrangian is
 *
 *     L = sum_k [ w_k ||x_k - a_k|| + y_k.(x_k - z) + (rho_k / 2) ||x_k - z||^2 ] + i_C(z).
 *
 * Algorithm 1 takes rho_k = mu for every k.  One ADMM sweep minimises L over
 * the block of local copies (which separates into one small problem per
 * point), then over z, and then moves every multiplier up the gradient of
 * the dual function.  Each of these three steps, and the residuals measured
 * after them, is a function of its own below; the solvers chain them.
 *
 * The multipliers are kept unscaled, as the paper writes them.  Points of a
 * constraint with penalty zero (the weighted variant's points of weight zero)
 * take no part: they have no term in the objective and no constraint.
 */
typedef struct {
    int64_t n, d;
    const double *a;    /* n x d points, point-major */
    const double *w;    /* n weights */
    const double *pen;  /* per-constraint penalties rho_k (n), or NULL for rho_k = mu */
    double mu;
} admm_problem_t;

static double admm_penalty(const admm_problem_t *P, int64_t k)
{
    return P->pen ? P->pen[k] : P->mu;
}

static int admm_active(const admm_problem_t *P, int64_t k)
{
    return P->pen == NULL || P->pen[k] > 0.0;
}

/*
 * Local block, equation (updatex).  For each point, L restricted to x_k is
 *   w_k ||x_k - a_k|| + (rho_k / 2) ||x_k - (z - y_k / rho_k)||^2 + const,
 * so x_k is the prox of (w_k / rho_k) ||. - a_k|| at v_k = z - y_k / rho_k:
 * the block soft-threshold of equation (closed-form), oracle_prox above.
 * z and y are read at their values from the previous sweep (Gauss-Seidel
 * order: x first).
 */
static void admm_local_block(const admm_problem_t *P, const double *z, const double *y, double *x,
                             double *v)
{
    const int64_t d = P->d;
    for (int64_t k = 0; k < P->n; ++k) {
        if (!admm_active(P, k)) continue;
        const double rho = admm_penalty(P, k);
        const double *yk = y + k * d;
        for (int64_t j = 0; j < d; ++j) v[j] = z[j] - yk[j] / rho;
        oracle_prox(d, v, P->a + k * d, P->w[k] / rho, x + k * d);
    }
}

/*
 * Global block, equation (updatez).  L restricted to z is, up to a constant,
 *   sum_k (rho_k / 2) ||z - (x_k + y_k / rho_k)||^2 + i_C(z),
 * an isotropic quadratic, so its minimiser over C is the projection of the
 * rho-weighted mean of x_k + y_k / rho_k.  With rho_k = mu the weights cancel
 * and the mean is over the N = n points present, unweighted.  When every
 * penalty is zero there is nothing to average and z stays where it is (then
 * projected).  `sum` is a d-vector of scratch; points are summed in order
 * k = 1..n.
 */
static void admm_global_block(const admm_problem_t *P, const or_set_t *C, const double *x,
                              const double *y, double *sum, double *z)
{
    const int64_t d = P->d;
    for (int64_t j = 0; j < d; ++j) sum[j] = 0.0;
    double total = 0.0;
    for (int64_t k = 0; k < P->n; ++k) {
        if (!admm_active(P, k)) continue;
        const double rho = admm_penalty(P, k);
        const double *xk = x + k * d, *yk = y + k * d;
        if (P->pen) {
            for (int64_t j = 0; j < d; ++j) sum[j] += rho * (xk[j] + yk[j] / rho);
            total += rho;
        } else {
            for (int64_t j = 0; j < d; ++j) sum[j] += xk[j] + yk[j] / rho;
        }
    }
    if (!P->pen) total = (double)P->n;
    for (int64_t j = 0; j < d; ++j) sum[j] = (total > 0.0) ? sum[j] / total : z[j];
    project_set(C, d, sum, z);
}

/*
 * Multiplier step, equation (updatey): gradient ascent on the dual function
 * with step rho_k, whose gradient in y_k is the constraint violation
 * x_k - z at the new z:  y_to_k = y_from_k + rho_k (x_k - z).
 * y_to may equal y_from.
 */
static void admm_multiplier_step(const admm_problem_t *P, const double *x, const double *z,
                                 const double *y_from, double *y_to)
{
    const int64_t d = P->d;
    for (int64_t k = 0; k < P->n; ++k) {
        if (!admm_active(P, k)) continue;
        const double rho = admm_penalty(P, k);
        for (int64_t j = 0; j < d; ++j)
            y_to[k * d + j] = y_from[k * d + j] + rho * (x[k * d + j] - z[j]);
    }
}

/*
 * Squared residuals after a sweep: primal sum_k ||x_k - z||^2 over the
 * constraints that take part (how far the copies are from agreeing) and dual
 * ||z - z_prev||^2 (how far z moved).  Returns the number of constraints.
 */
static int64_t admm_residuals(const admm_problem_t *P, const double *x, const double *z,
                              const double *z_prev, double *sp, double *sd)
{
    const int64_t d = P->d;
    int64_t m = 0;
    *sp = 0.0;
    *sd = 0.0;
    for (int64_t k = 0; k < P->n; ++k) {
        if (!admm_active(P, k)) continue;
        ++m;
        for (int64_t j = 0; j < d; ++j) {
            double e = x[k * d + j] - z[j];
            *sp += e * e;
        }
    }
    for (int64_t j = 0; j < d; ++j) {
        double e = z[j] - z_prev[j];
        *sd += e * e;
    }
    return m;
}

/*
 * Common checks: n = 0 is EMPTY (z left as given); a negative or non-finite
 * weight, a non-finite point or starting z, or an invalid set is BAD_INPUT
 * (z set to NaN).  Returns 0 when the instance can be solved.
 */
static int admm_screen(int64_t n, int64_t d, const double *a, const double *w, const or_set_t *C,
                       double *z)
{
    if (n == 0) return OR_EMPTY;
    int bad = !set_ok(d, C);
    for (int64_t k = 0; k < n; ++k)
        if (!isfinite(w[k]) || w[k] < 0.0) bad = 1;
    for (int64_t i = 0; i < n * d; ++i)
        if (!isfinite(a[i])) bad = 1;
    for (int64_t j = 0; j < d; ++j)
        if (!isfinite(z[j])) bad = 1;
    if (bad) {
        for (int64_t j = 0; j < d; ++j) z[j] = NAN;
        return OR_BAD_INPUT;
    }
    return 0;
}

/*
 * One instance of Algorithm 1 (penalty mu for every constraint).
 *
 * Stopping (the paper only asks for "convergence"): after each sweep,
 *   r_pri  = sqrt(sum_k ||x_k - z||^2 / (n d)),   r_dual = sqrt(||z - z_prev||^2 / d),
 * and the solve ends when tol > 0 and both are <= tol * D, else after
 * max_iter sweeps.
 *
 * Adaptive penalty (adapt_every > 0; the conclusion names it as future work,
 * the rule is residual balancing, Boyd et al. 2011, Section 3.4.1): after a
 * sweep t that did not stop, with t a multiple of adapt_every, the stacked
 * residual norms ||r|| = (sum_k ||x_k - z||^2)^(1/2) and
 * ||s|| = mu (n ||z - z_prev||^2)^(1/2) are compared; mu is multiplied by
 * adapt_factor when ||r|| > adapt_ratio ||s|| and divided by it when
 * ||s|| > adapt_ratio ||r||.  The unscaled y_k are kept, so nothing else
 * changes.  *mu_out (nullable) receives the final penalty.
 *
 * a: n*d points (point-major), w: n weights, z: d values in/out (the starting
 * z is used unprojected), y: n*d multipliers in/out (NULL: start from zero,
 * discarded), x_out: n*d last local copies (NULL to skip).  Returns the flag
 * word; *iters, *r_pri, *r_dual receive the sweep count and the residuals of
 * the last sweep (0 when none ran).
 */
static int em_solve_set(int64_t n, int64_t d, const double *a, const double *w, double mu,
                        const or_set_t *C, double *z, double *y, double *x_out, int64_t max_iter,
                        double tol, int64_t adapt_every, double adapt_ratio, double adapt_factor,
                        int64_t *iters, double *r_pri, double *r_dual, double *mu_out)
{
    *iters = 0;
    *r_pri = 0.0;
    *r_dual = 0.0;
    if (mu_out) *mu_out = mu;
    int screened = admm_screen(n, d, a, w, C, z);
    if (screened) return screened;
    const double D = tol_scale_set(n, d, a, C);

    admm_problem_t P = {n, d, a, w, NULL, mu};
    double *mult = y ? y : (double *)calloc((size_t)(n * d), sizeof(double));
    double *x = (double *)calloc((size_t)(n * d), sizeof(double));
    double *v = (double *)malloc((size_t)d * sizeof(double));
    double *sum = (double *)malloc((size_t)d * sizeof(double));
    double *z_prev = (double *)malloc((size_t)d * sizeof(double));

    int flags = OR_MAXITER;
    for (int64_t t = 1; t <= max_iter; ++t) {
        memcpy(z_prev, z, (size_t)d * sizeof(double));
        admm_local_block(&P, z, mult, x, v);
        admm_global_block(&P, C, x, mult, sum, z);
        admm_multiplier_step(&P, x, z, mult, mult);
        double sp, sd;
        admm_residuals(&P, x, z, z_prev, &sp, &sd);
        *r_pri = sqrt(sp / (double)(n * d));
        *r_dual = sqrt(sd / (double)d);
        *iters = t;
        if (tol > 0.0 && *r_pri <= tol * D && *r_dual <= tol * D) {
            flags = OR_CONVERGED;
            break;
        }
        if (adapt_every > 0 && t % adapt_every == 0) {
            const double rnorm = sqrt(sp);
            const double snorm = P.mu * sqrt((double)n * sd);
            if (rnorm > adapt_ratio * snorm)
                P.mu *= adapt_factor;
            else if (snorm > adapt_ratio * rnorm)
                P.mu /= adapt_factor;
        }
    }
    if (mu_out) *mu_out = P.mu;
    if (x_out) memcpy(x_out, x, (size_t)(n * d) * sizeof(double));
    if (!y) free(mult);
    free(x);
    free(v);
    free(sum);
    free(z_prev);
    return flags;
}

/* Algorithm 1 over the box prod_j [lo_j, hi_j] (adapt_every > 0: adaptive penalty). */
int oracle_em_solve_ex(int64_t n, int64_t d, const double *a, const double *w,
                       double mu, const double *lo, const double *hi, double *z, double *y,
                       double *x_out, int64_t max_iter, double tol, int64_t adapt_every,
                       double adapt_ratio, double adapt_factor, int64_t *iters, double *r_pri,
                       double *r_dual, double *mu_out)
{
    or_set_t C = {lo, hi, NULL, 0.0};
    return em_solve_set(n, d, a, w, mu, &C, z, y, x_out, max_iter, tol, adapt_every, adapt_ratio,
                        adapt_factor, iters, r_pri, r_dual, mu_out);
}

/* Algorithm 1 over the ball ||z - center|| <= radius (adapt_every > 0: adaptive penalty). */
int oracle_em_solve_ball(int64_t n, int64_t d, const double *a, const double *w, double mu,
                         const double *center, double radius, double *z, double *y,
                         double *x_out, int64_t max_iter, double tol, int64_t adapt_every,
                         double adapt_ratio, double adapt_factor, int64_t *iters, double *r_pri,
                         double *r_dual, double *mu_out)
{
    or_set_t C = {NULL, NULL, center, radius};
    return em_solve_set(n, d, a, w, mu, &C, z, y, x_out, max_iter, tol, adapt_every, adapt_ratio,
                        adapt_factor, iters, r_pri, r_dual, mu_out);
}

/*
 * The weighted-mean variant (a different algorithm from Algorithm 1): the
 * constraint of point k gets the penalty rho_k = mu w_k instead of mu.  The
 * same three blocks then give a prox threshold w_k / rho_k = 1 / mu for every
 * point and a z-update that projects the w-weighted mean of x_k + y_k / rho_k
 * (exact over a box or a ball: the z-subproblem is an isotropic quadratic).
 * A point of weight zero has no term and no constraint and is left out; with
 * every weight zero z = P_C(z).  The primal residual runs over the n' points
 * of positive weight, r_pri = sqrt(sum_k ||x_k - z||^2 / (n' d)) (0 when
 * n' = 0); r_dual, D, stopping and the screening are those of em_solve_set.
 */
static int em_solve_wpen_set(int64_t n, int64_t d, const double *a, const double *w, double mu,
                             const or_set_t *C, double *z, int64_t max_iter, double tol,
                             int64_t *iters, double *r_pri, double *r_dual)
{
    *iters = 0;
    *r_pri = 0.0;
    *r_dual = 0.0;
    int screened = admm_screen(n, d, a, w, C, z);
    if (screened) return screened;
    const double D = tol_scale_set(n, d, a, C);
    double *pen = (double *)malloc((size_t)(n + 1) * sizeof(double));
    for (int64_t k = 0; k < n; ++k) pen[k] = (w[k] > 0.0) ? mu * w[k] : 0.0;
    admm_problem_t P = {n, d, a, w, pen, mu};
    double *y = (double *)calloc((size_t)(n * d + 1), sizeof(double));
    double *x = (double *)calloc((size_t)(n * d + 1), sizeof(double));
    double *v = (double *)malloc((size_t)d * sizeof(double));
    double *sum = (double *)malloc((size_t)d * sizeof(double));
    double *z_prev = (double *)malloc((size_t)d * sizeof(double));

    int flags = OR_MAXITER;
    for (int64_t t = 1; t <= max_iter; ++t) {
        memcpy(z_prev, z, (size_t)d * sizeof(double));
        admm_local_block(&P, z, y, x, v);
        admm_global_block(&P, C, x, y, sum, z);
        admm_multiplier_step(&P, x, z, y, y);
        double sp, sd;
        const int64_t npos = admm_residuals(&P, x, z, z_prev, &sp, &sd);
        *r_pri = (npos > 0) ? sqrt(sp / (double)(npos * d)) : 0.0;
        *r_dual = sqrt(sd / (double)d);
        *iters = t;
        if (tol > 0.0 && *r_pri <= tol * D && *r_dual <= tol * D) {
            flags = OR_CONVERGED;
            break;
        }
    }
    free(pen);
    free(y);
    free(x);
    free(v);
    free(sum);
    free(z_prev);
    return flags;
}

/* The weighted-mean variant over the box prod_j [lo_j, hi_j]. */
int oracle_em_solve_wpen(int64_t n, int64_t d, const double *a, const double *w, double mu,
                         const double *lo, const double *hi, double *z, int64_t max_iter,
                         double tol, int64_t *iters, double *r_pri, double *r_dual)
{
    or_set_t C = {lo, hi, NULL, 0.0};
    return em_solve_wpen_set(n, d, a, w, mu, &C, z, max_iter, tol, iters, r_pri, r_dual);
}

/* The weighted-mean variant over the ball ||z - center|| <= radius. */
int oracle_em_solve_wpen_ball(int64_t n, int64_t d, const double *a, const double *w, double mu,
                              const double *center, double radius, double *z, int64_t max_iter,
                              double tol, int64_t *iters, double *r_pri, double *r_dual)
{
    or_set_t C = {NULL, NULL, center, radius};
    return em_solve_wpen_set(n, d, a, w, mu, &C, z, max_iter, tol, iters, r_pri, r_dual);
}

/* Algorithm 1 with the scalar box [lo, hi]^d and a fixed penalty. */
int oracle_em_solve(int64_t n, int64_t d, const double *a, const double *w,
                    double mu, double lo, double hi, double *z, double *y,
                    double *x_out, int64_t max_iter, double tol,
                    int64_t *iters, double *r_pri, double *r_dual)
{
    double *lv = (double *)malloc((size_t)(d + 1) * sizeof(double));
    double *hv = (double *)malloc((size_t)(d + 1) * sizeof(double));
    for (int64_t j = 0; j < d; ++j) {
        lv[j] = lo;
        hv[j] = hi;
    }
    int f = oracle_em_solve_ex(n, d, a, w, mu, lv, hv, z, y, x_out, max_iter, tol, 0, 10.0, 2.0,
                               iters, r_pri, r_dual, NULL);
    free(lv);
    free(hv);
    return f;
}

/*
 * Accelerated ADMM, the second extension the conclusion names: fast ADMM with
 * restart for weakly convex problems [Goldstein2012], applied to the same
 * splitting (first block the local copies x_k, second block z, constraint
 * x_k - z = 0, penalty mu).
 *
 * The sweeps are those of Algorithm 1 except that the local and global blocks
 * start from predicted values z_hat, y_hat instead of the last z, y:
 *   x     = local block at (z_hat, y_hat),
 *   z     = global block from (x, y_hat),
 *   y     = y_hat + mu (x - z)                       (multiplier step from y_hat).
 * The progress measure of the sweep is
 *   c = mu sum_k ||x_k - z||^2 + mu n ||z - z_hat||^2
 * (the squared multiplier change over mu plus mu times the squared change of
 * B z with B the stacked -I blocks).  When c < eta' c_prev, with eta' = eta
 * (1 - 2^-16), the next
 * predictions extrapolate along the last step with Nesterov's weight: alpha'
 * = (1 + sqrt(1 + 4 alpha^2)) / 2, beta = (alpha - 1) / alpha', z_hat = z +
 * beta (z - z_prev), y_hat = y + beta (y - y_prev), and c_prev = c.  Otherwise
 * the sweep is restarted from the previous iterate: z_hat = z_prev, y_hat =
 * y_prev, alpha' = 1, and c_prev becomes c_prev / eta.  Initially z_hat = z_prev
 * = z0, y_hat = y_prev = 0, alpha = 1 and c_prev = +inf (so the first sweep
 * takes the momentum branch with beta = 0).
 * The guard factor 1 - 2^-16 is this implementation's reading of the test
 * c < eta c_prev of [Goldstein2012]: once the iterate stalls (e.g. z held at
 * a bound of the box with every prox returning its own point) each sweep
 * repeats the same c, and after a restart the test compares c with
 * eta (c_prev / eta) = c, an exact tie that exact arithmetic sends to the
 * restart branch and that rounding sends either way; with the guard the tie
 * is 1.5e-5 c on the restart side, wider than the rounding of an FP32 run.
 * Only decisions with c within that band below eta c_prev change branch.
 * Residuals and stopping as for em_solve_set (r_dual from z - z_prev).
 * *restarts (nullable) receives the number of restarts.  *ties (nullable,
 * batch entry only) counts the decisions with a finite c_prev and
 * |c - eta' c_prev| <= tie_band eta' c_prev: there c and the threshold agree
 * to within the rounding of a lower-precision run of the same sweeps, so
 * either branch is a correct run.  No decision is
 * taken after the last allowed sweep (nothing follows it), so a solve that
 * stops at sweep T, by the tolerance or by max_iter = T, reports the
 * decisions of sweeps 1..T-1.
 */
static int em_solve_fast_set(int64_t n, int64_t d, const double *a, const double *w, double mu,
                             const double *lo, const double *hi, double *z, int64_t max_iter,
                             double tol, double eta, double tie_band, int64_t *iters,
                             double *r_pri, double *r_dual, int64_t *restarts, int64_t *ties)
{
    *iters = 0;
    *r_pri = 0.0;
    *r_dual = 0.0;
    if (restarts) *restarts = 0;
    if (ties) *ties = 0;
    or_set_t C = {lo, hi, NULL, 0.0};
    int screened = admm_screen(n, d, a, w, &C, z);
    if (screened) return screened;
    const double D = tol_scale_set(n, d, a, &C);
    admm_problem_t P = {n, d, a, w, NULL, mu};
    const size_t nd = (size_t)(n * d);
    double *y = (double *)calloc(nd, sizeof(double));
    double *y_prev = (double *)calloc(nd, sizeof(double));
    double *y_hat = (double *)calloc(nd, sizeof(double));
    double *x = (double *)calloc(nd, sizeof(double));
    double *v = (double *)malloc((size_t)d * sizeof(double));
    double *sum = (double *)malloc((size_t)d * sizeof(double));
    double *z_prev = (double *)malloc((size_t)d * sizeof(double));
    double *z_hat = (double *)malloc((size_t)d * sizeof(double));
    memcpy(z_prev, z, (size_t)d * sizeof(double));
    memcpy(z_hat, z, (size_t)d * sizeof(double));
    double alpha = 1.0, c_prev = INFINITY;
    const double eta_g = eta * (1.0 - 0x1p-16);

    int flags = OR_MAXITER;
    for (int64_t t = 1; t <= max_iter; ++t) {
        memcpy(z_prev, z, (size_t)d * sizeof(double));
        memcpy(y_prev, y, nd * sizeof(double));
        admm_local_block(&P, z_hat, y_hat, x, v);
        admm_global_block(&P, &C, x, y_hat, sum, z);
        admm_multiplier_step(&P, x, z, y_hat, y);
        double sp, sd;
        admm_residuals(&P, x, z, z_prev, &sp, &sd);
        double sh = 0.0;
        for (int64_t j = 0; j < d; ++j) {
            double e = z[j] - z_hat[j];
            sh += e * e;
        }
        *r_pri = sqrt(sp / (double)(n * d));
        *r_dual = sqrt(sd / (double)d);
        *iters = t;
        if (tol > 0.0 && *r_pri <= tol * D && *r_dual <= tol * D) {
            flags = OR_CONVERGED;
            break;
        }
        if (t == max_iter) break;   /* the decision would change nothing */
        const double c = mu * (sp + (double)n * sh);
        const double thr = eta_g * c_prev;
        if (ties && isfinite(c_prev) && fabs(c - thr) <= tie_band * thr) ++*ties;
        if (c < thr) {
            const double alpha_next = 0.5 * (1.0 + sqrt(1.0 + 4.0 * alpha * alpha));
            const double beta = (alpha - 1.0) / alpha_next;
            for (int64_t j = 0; j < d; ++j) z_hat[j] = z[j] + beta * (z[j] - z_prev[j]);
            for (size_t i = 0; i < nd; ++i) y_hat[i] = y[i] + beta * (y[i] - y_prev[i]);
            alpha = alpha_next;
            c_prev = c;
        } else {
            memcpy(z_hat, z_prev, (size_t)d * sizeof(double));
            memcpy(y_hat, y_prev, nd * sizeof(double));
            alpha = 1.0;
            c_prev = c_prev / eta;
            if (restarts) ++*restarts;
        }
    }
    free(y);
    free(y_prev);
    free(y_hat);
    free(x);
    free(v);
    free(sum);
    free(z_prev);
    free(z_hat);
    return flags;
}

int oracle_em_solve_fast(int64_t n, int64_t d, const double *a, const double *w, double mu,
                         const double *lo, const double *hi, double *z, int64_t max_iter,
                         double tol, double eta, int64_t *iters, double *r_pri, double *r_dual,
                         int64_t *restarts)
{
    return em_solve_fast_set(n, d, a, w, mu, lo, hi, z, max_iter, tol, eta, 0.0, iters, r_pri,
                             r_dual, restarts, NULL);
}

/*
 * Objective of (EM) at z: sum_k w_k ||z - a_k||_2.
 */
double oracle_em_objective(int64_t n, int64_t d, const double *a, const double *w, const double *z)
{
    double f = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double q = 0.0;
        for (int64_t j = 0; j < d; ++j) {
            double t = z[j] - a[k * d + j];
            q += t * t;
        }
        f += w[k] * sqrt(q);
    }
    return f;
}

/*
 * The smooth surrogate of (EM) that the IRLS method of the paper's reference
 * [Chaudhury2012] minimises, equation (EM_surrogate):
 *   sum_k w_k (||z - a_k||^2 + eps)^(1/2),  eps > 0.
 */
double oracle_surrogate_objective(int64_t n, int64_t d, const double *a, const double *w,
                                  double eps, const double *z)
{
    double f = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double q = 0.0;
        for (int64_t j = 0; j < d; ++j) {
            double t = z[j] - a[k * d + j];
            q += t * t;
        }
        f += w[k] * sqrt(q + eps);
    }
    return f;
}

/*
 * IRLS for the surrogate (EM_surrogate) over the box C = prod_j [lo_j, hi_j].  The
 * paper names the method but does not print its steps; they follow from
 * majorise-minimise: sqrt is concave, so at the current iterate z^t
 *   (q + eps)^(1/2) <= (q_t + eps)^(1/2) + (q - q_t) / (2 (q_t + eps)^(1/2)),
 * q = ||z - a_k||^2, with equality at z = z^t.  The majoriser is, up to a
 * constant, sum_k omega_k ||z - a_k||^2 / 2 with
 *   omega_k = w_k / (||z^t - a_k||^2 + eps)^(1/2),
 * an isotropic quadratic centred at the omega-weighted mean, so its minimiser
 * over the box is that mean projected coordinate-wise onto C:
 *   z^{t+1} = P_C( sum_k omega_k a_k / sum_k omega_k ).
 * Every step therefore decreases the surrogate (unless z^t is its minimiser).
 * Stopping: after iteration t, r_dual = sqrt(||z^{t+1} - z^t||^2 / d) <= tol D
 * with D as for EM-ADMM (there is no primal residual; *r_pri is set to 0).
 * All weights zero: every point of C minimises the surrogate over C; the
 * start projected onto C is returned (as EM-ADMM returns after its first
 * z-update) and the solve reports CONVERGED after one iteration.
 * Flags, init and the n = 0 / bad-input rules are those of oracle_em_solve.
 */
static int irls_solve_set(int64_t n, int64_t d, const double *a, const double *w, double eps,
                          const or_set_t *C, double *z, int64_t max_iter, double tol,
                          int64_t *iters, double *r_pri, double *r_dual)
{
    *iters = 0;
    *r_pri = 0.0;
    *r_dual = 0.0;
    if (n == 0) return OR_EMPTY;
    int bad = !(eps > 0.0) || !set_ok(d, C);
    for (int64_t k = 0; k < n; ++k)
        if (!isfinite(w[k]) || w[k] < 0.0) bad = 1;
    for (int64_t i = 0; i < n * d; ++i)
        if (!isfinite(a[i])) bad = 1;
    for (int64_t j = 0; j < d; ++j)
        if (!isfinite(z[j])) bad = 1;
    if (bad) {
        for (int64_t j = 0; j < d; ++j) z[j] = NAN;
        return OR_BAD_INPUT;
    }
    double D = tol_scale_set(n, d, a, C);
    double *num = (double *)malloc((size_t)d * sizeof(double));
    double *zn = (double *)malloc((size_t)d * sizeof(double));
    int flags = OR_MAXITER;
    for (int64_t t = 1; t <= max_iter; ++t) {
        double den = 0.0;
        for (int64_t j = 0; j < d; ++j) num[j] = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            double q = 0.0;
            for (int64_t j = 0; j < d; ++j) {
                double e = z[j] - a[k * d + j];
                q += e * e;
            }
            double om = w[k] / sqrt(q + eps);
            den += om;
            for (int64_t j = 0; j < d; ++j) num[j] += om * a[k * d + j];
        }
        double sd = 0.0;
        if (den > 0.0) {
            for (int64_t j = 0; j < d; ++j) num[j] = num[j] / den;
            project_set(C, d, num, zn);
        } else {
            project_set(C, d, z, zn);   /* the problem is posed over C */
        }
        for (int64_t j = 0; j < d; ++j) {
            double e = zn[j] - z[j];
            sd += e * e;
            z[j] = zn[j];
        }
        *r_dual = sqrt(sd / (double)d);
        *iters = t;
        if (den == 0.0 || (tol > 0.0 && *r_dual <= tol * D)) {
            flags = OR_CONVERGED;
            break;
        }
    }
    free(num);
    free(zn);
    return flags;
}

/* IRLS over the box prod_j [lo_j, hi_j]. */
int oracle_irls_solve_ex(int64_t n, int64_t d, const double *a, const double *w, double eps,
                         const double *lo, const double *hi, double *z, int64_t max_iter,
                         double tol, int64_t *iters, double *r_pri, double *r_dual)
{
    or_set_t C = {lo, hi, NULL, 0.0};
    return irls_solve_set(n, d, a, w, eps, &C, z, max_iter, tol, iters, r_pri, r_dual);
}

/* IRLS over the ball ||z - center|| <= radius. */
int oracle_irls_solve_ball(int64_t n, int64_t d, const double *a, const double *w, double eps,
                           const double *center, double radius, double *z, int64_t max_iter,
                           double tol, int64_t *iters, double *r_pri, double *r_dual)
{
    or_set_t C = {NULL, NULL, center, radius};
    return irls_solve_set(n, d, a, w, eps, &C, z, max_iter, tol, iters, r_pri, r_dual);
}

/* IRLS over the scalar box [lo, hi]^d. */
int oracle_irls_solve(int64_t n, int64_t d, const double *a, const double *w, double eps,
                      double lo, double hi, double *z, int64_t max_iter, double tol,
                      int64_t *iters, double *r_pri, double *r_dual)
{
    double *lv = (double *)malloc((size_t)(d + 1) * sizeof(double));
    double *hv = (double *)malloc((size_t)(d + 1) * sizeof(double));
    for (int64_t j = 0; j < d; ++j) {
        lv[j] = lo;
        hv[j] = hi;
    }
    int f = oracle_irls_solve_ex(n, d, a, w, eps, lv, hv, z, max_iter, tol, iters, r_pri, r_dual);
    free(lv);
    free(hv);
    return f;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * A batch of independent instances (the points and weights are the float32
 * buffers the GPU reads, widened to binary64 here).  Instance b has n[b]
 * points of dimension d[b] at a + a_off[b], weights at w + w_off[b] and its
 * result at z + z_off[b].  init = GIVEN uses z as the initial value; init =
 * MAXW starts from the point of largest weight (lowest index on ties); init =
 * WMEAN from the weighted mean sum_k w_k a_k / sum_k w_k (the counterpart of
 * the NLM patch that Section 3 starts from), or the plain mean of the points
 * when every weight is zero.
 * max_iter_each (nullable) overrides max_iter per instance.
 * solver: 0 = EM-ADMM (adapt_every > 0 adds the adaptive penalty), 1 = IRLS
 * on the surrogate with eps, 3 = accelerated ADMM with restart parameter eta,
 * 4 = the weighted-mean variant (penalties mu w_k).
 * ball_radius (nullable, one per instance) selects the ball constraint with
 * centres ball_center (nullable = origin, indexed like z; solvers 0, 1 and 4).
 * Otherwise box_lo / box_hi (nullable, float32, indexed like
 * z) give per-coordinate bounds; otherwise [lo, hi] for every coordinate.
 * mu_out (nullable): the final penalty per instance; restarts_out (nullable):
 * the accelerated ADMM's restart count per instance; ties_out (nullable): its
 * count of decisions within tie_band (relative) of the threshold.
 */
int oracle_em_batch_ex(int64_t B, const float *a, const float *w, const int64_t *a_off,
                       const int64_t *w_off, const int64_t *z_off, const int32_t *n_arr,
                       const int32_t *d_arr, int solver, double mu, double eps, double lo, double hi,
                       const float *box_lo, const float *box_hi, const float *ball_center,
                       const float *ball_radius, int64_t max_iter,
                       const int32_t *max_iter_each, double tol, int init, int64_t adapt_every,
                       double adapt_ratio, double adapt_factor, double *z, int32_t *iters,
                       int32_t *flags, double *r_pri, double *r_dual, double *mu_out, double eta,
                       int32_t *restarts_out, int nthreads, double tie_band, int32_t *ties_out)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < B; ++b) {
        int64_t n = n_arr[b], d = d_arr[b];
        double *ab = (double *)malloc((size_t)(n * d + 1) * sizeof(double));
        double *wb = (double *)malloc((size_t)(n + 1) * sizeof(double));
        double *lv = (double *)malloc((size_t)(d + 1) * sizeof(double));
        double *hv = (double *)malloc((size_t)(d + 1) * sizeof(double));
        for (int64_t i = 0; i < n * d; ++i) ab[i] = (double)a[a_off[b] + i];
        for (int64_t k = 0; k < n; ++k) wb[k] = (double)w[w_off[b] + k];
        for (int64_t j = 0; j < d; ++j) {
            lv[j] = box_lo ? (double)box_lo[z_off[b] + j] : lo;
            hv[j] = box_hi ? (double)box_hi[z_off[b] + j] : hi;
            if (ball_radius) lv[j] = ball_center ? (double)ball_center[z_off[b] + j] : 0.0;
        }
        /* ball_radius != NULL selects the ball (centre in lv, origin when no centres) */
        or_set_t C = {lv, hv, ball_radius ? lv : NULL, ball_radius ? (double)ball_radius[b] : 0.0};
        double *zb = z + z_off[b];
        if (init == OR_INIT_MAXW && n > 0) {
            int64_t best = 0;
            for (int64_t k = 1; k < n; ++k)
                if (wb[k] > wb[best]) best = k;
            for (int64_t j = 0; j < d; ++j) zb[j] = ab[best * d + j];
        }
        if (init == OR_INIT_WMEAN && n > 0) {
            double W = 0.0;
            for (int64_t k = 0; k < n; ++k) W += wb[k];
            for (int64_t j = 0; j < d; ++j) {
                double s = 0.0;
                for (int64_t k = 0; k < n; ++k) s += (W > 0.0 ? wb[k] : 1.0) * ab[k * d + j];
                zb[j] = s / (W > 0.0 ? W : (double)n);
            }
        }
        int64_t it = 0, rs = 0, ti = 0;
        double rp = 0.0, rd = 0.0, mf = mu;
        int64_t mi = max_iter_each ? max_iter_each[b] : max_iter;
        int f;
        if (solver == 1)
            f = irls_solve_set(n, d, ab, wb, eps, &C, zb, mi, tol, &it, &rp, &rd);
        else if (solver == 4)
            f = em_solve_wpen_set(n, d, ab, wb, mu, &C, zb, mi, tol, &it, &rp, &rd);
        else if (solver == 3)
            f = em_solve_fast_set(n, d, ab, wb, mu, lv, hv, zb, mi, tol, eta, tie_band, &it, &rp, &rd,
                                  &rs, &ti);
        else
            f = em_solve_set(n, d, ab, wb, mu, &C, zb, NULL, NULL, mi, tol, adapt_every, adapt_ratio,
                             adapt_factor, &it, &rp, &rd, &mf);
        if (iters) iters[b] = (int32_t)it;
        if (flags) flags[b] = f;
        if (r_pri) r_pri[b] = rp;
        if (r_dual) r_dual[b] = rd;
        if (mu_out) mu_out[b] = mf;
        if (restarts_out) restarts_out[b] = (int32_t)rs;
        if (ties_out) ties_out[b] = (int32_t)ti;
        free(ab);
        free(wb);
        free(lv);
        free(hv);
    }
    return 0;
}

/* The batch with EM-ADMM, a fixed penalty and the scalar box. */
int oracle_em_batch(int64_t B, const float *a, const float *w, const int64_t *a_off,
                    const int64_t *w_off, const int64_t *z_off, const int32_t *n_arr,
                    const int32_t *d_arr, double mu, double lo, double hi,
                    int64_t max_iter, const int32_t *max_iter_each, double tol, int init,
                    double *z, int32_t *iters, int32_t *flags, double *r_pri,
                    double *r_dual, int nthreads)
{
    return oracle_em_batch_ex(B, a, w, a_off, w_off, z_off, n_arr, d_arr, 0, mu, 1.0, lo, hi, NULL,
                              NULL, NULL, NULL, max_iter, max_iter_each, tol, init, 0, 10.0, 2.0, z,
                              iters, flags, r_pri, r_dual, NULL, 0.999, NULL, nthreads, 0.0, NULL);
}

/* Symmetric (edge-repeating) reflection of index i into [0, N); needs |overhang| <= N. */
static int64_t reflect(int64_t i, int64_t N)
{
    if (i < 0) return -i - 1;
    if (i >= N) return 2 * N - i - 1;
    return i;
}

/*
 * Patch P_i of Section 3: the (2pr+1) x (2pr+1) square of the noisy image
 * centred at pixel (iy, ix), row-major, pixels outside the image taken by
 * symmetric reflection.
 */
static void extract_patch(const float *img, int64_t H, int64_t W, int64_t pr,
                          int64_t iy, int64_t ix, double *P)
{
    int64_t side = 2 * pr + 1;
    for (int64_t dy = -pr; dy <= pr; ++dy)
        for (int64_t dx = -pr; dx <= pr; ++dx)
            P[(dy + pr) * side + (dx + pr)] =
                (double)img[reflect(iy + dy, H) * W + reflect(ix + dx, W)];
}

/*
 * NLEM (Section 3): for each requested pixel i, the points are the patches
 * P_j of every pixel j of the (2wr+1) x (2wr+1) search window centred at i
 * that lies inside the image (the window is truncated at borders, j = i
 * included, row-major order), the weights are w_ij = exp(-||P_i - P_j||^2 /
 * h^2) (not normalised), the box is [lo, hi]^d and y starts at zero.  The
 * denoised pixel is the centre coordinate of the returned patch, z[(d - 1) / 2].
 *
 * solver: 0 = EM-ADMM (Algorithm 1, penalty mu), 1 = IRLS on the surrogate
 * (EM_surrogate) with parameter eps (oracle_irls_solve).
 * init: 0 = the noisy patch P_i (unprojected), 1 = the NLM patch
 * sum_j w_ij P_j / sum_j w_ij (the two starting points Section 3 compares).
 * With init = 1 and max_iter = 0 the output is the Non-Local Means estimate.
 *
 * pix: npix linear pixel indices (NULL: all H*W pixels in order).
 * max_iter_each (nullable): per requested pixel iteration cap.
 * out: npix denoised values; zfull (nullable): npix*d patches;
 * weights_out (nullable): npix * (2wr+1)^2 weights in window order, slots of
 * points outside the image set to -1.
 */
int oracle_nlem_ex(int64_t H, int64_t W, const float *img, int64_t pr, int64_t wr,
                   double h, double lo, double hi, int solver, int init, double mu,
                   double eps, int64_t max_iter, const int32_t *max_iter_each, double tol,
                   int64_t npix, const int64_t *pix, double *out, double *zfull,
                   double *weights_out, int32_t *iters, int32_t *flags, double *r_pri,
                   double *r_dual, int nthreads)
{
    int64_t side = 2 * pr + 1, d = side * side;
    int64_t wside = 2 * wr + 1, nmax = wside * wside;
    set_threads(nthreads);
    if (!pix) npix = H * W;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < npix; ++q) {
        int64_t i = pix ? pix[q] : q;
        int64_t iy = i / W, ix = i % W;
        double *a = (double *)malloc((size_t)(nmax * d) * sizeof(double));
        double *wk = (double *)malloc((size_t)nmax * sizeof(double));
        double *z = (double *)malloc((size_t)d * sizeof(double));
        double *Pi = (double *)malloc((size_t)d * sizeof(double));
        extract_patch(img, H, W, pr, iy, ix, Pi);
        int64_t n = 0;
        for (int64_t dy = -wr; dy <= wr; ++dy)
            for (int64_t dx = -wr; dx <= wr; ++dx) {
                int64_t jy = iy + dy, jx = ix + dx;
                int64_t slot = (dy + wr) * wside + (dx + wr);
                if (jy < 0 || jy >= H || jx < 0 || jx >= W) {
                    if (weights_out) weights_out[q * nmax + slot] = -1.0;
                    continue;
                }
                double *Pj = a + n * d;
                extract_patch(img, H, W, pr, jy, jx, Pj);
                double dist2 = 0.0;
                for (int64_t c = 0; c < d; ++c) {
                    double t = Pi[c] - Pj[c];
                    dist2 += t * t;
                }
                wk[n] = exp(-dist2 / (h * h));
                if (weights_out) weights_out[q * nmax + slot] = wk[n];
                ++n;
            }
        if (init == 1) {
            /* NLM patch: the weighted mean of the window's patches */
            double ws = 0.0;
            for (int64_t k = 0; k < n; ++k) ws += wk[k];
            for (int64_t c = 0; c < d; ++c) {
                double acc = 0.0;
                for (int64_t k = 0; k < n; ++k) acc += wk[k] * a[k * d + c];
                z[c] = acc / ws;
            }
        } else {
            memcpy(z, Pi, (size_t)d * sizeof(double));
        }
        int64_t it = 0;
        double rp = 0.0, rd = 0.0;
        int64_t mi = max_iter_each ? max_iter_each[q] : max_iter;
        int f = (solver == 1)
                    ? oracle_irls_solve(n, d, a, wk, eps, lo, hi, z, mi, tol, &it, &rp, &rd)
                    : oracle_em_solve(n, d, a, wk, mu, lo, hi, z, NULL, NULL, mi, tol, &it, &rp, &rd);
        out[q] = z[(d - 1) / 2];
        if (zfull) memcpy(zfull + q * d, z, (size_t)d * sizeof(double));
        if (iters) iters[q] = (int32_t)it;
        if (flags) flags[q] = f;
        if (r_pri) r_pri[q] = rp;
        if (r_dual) r_dual[q] = rd;
        free(a);
        free(wk);
        free(z);
        free(Pi);
    }
    return 0;
}

/* NLEM with EM-ADMM started from the noisy patch (oracle_nlem_ex, solver 0, init 0). */
int oracle_nlem(int64_t H, int64_t W, const float *img, int64_t pr, int64_t wr,
                double h, double lo, double hi, double mu, int64_t max_iter,
                const int32_t *max_iter_each, double tol, int64_t npix,
                const int64_t *pix, double *out, double *zfull, double *weights_out,
                int32_t *iters, int32_t *flags, double *r_pri, double *r_dual,
                int nthreads)
{
    return oracle_nlem_ex(H, W, img, pr, wr, h, lo, hi, 0, 0, mu, 1.0, max_iter, max_iter_each,
                          tol, npix, pix, out, zfull, weights_out, iters, flags, r_pri, r_dual,
                          nthreads);
}
