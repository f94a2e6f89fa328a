/*
 * Plain FP64 CPU oracle for the nonlocal obstacle-potential phase-field step
 * (arXiv 2310.10750, Sections 2.1 and 4), case beta2 = 0.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the CPU baseline leg of
 * the benchmark do.  It shares no code, header or table with the HIP path.
 *
 * What it computes, in the paper's terms:
 *   - periodic n x n lattice on the unit square, h = 1/n, nodes (x h, y h);
 *   - the horizon disc: lattice offsets d with |d| h <= delta (closed ball,
 *     kernel support in Sec. 2.1; truncation in eq. kernel_gauss);
 *   - nodal (lumped) quadrature of the convolution:
 *        (gamma * u)_i = sum_{d in D} w_d u_{i+d},   w_d = h^2 gamma(h |d|)
 *     and c_gamma = sum_{d in D} w_d   (eq. nonl_operator, c_gamma = gamma * 1);
 *   - xi = c_gamma - c_F                                    (eq. xi_constant);
 *   - implicit Euler with the convolution taken explicitly (Sec. 4,
 *     discretisation paragraph) for  du/dt + beta1 w = 0,
 *     w = L u + dF_obs(u)  (eq. nonl_CH_nm with beta2 = 0, obstacle potential
 *     eq. potential_obstacle and its subdifferential):
 *        (u^k - u^{k-1})/tau + beta1 (c_gamma u^k - (gamma*u^{k-1})
 *                                     - c_F u^k + mu^k) = 0,
 *        mu^k in the normal cone of [-1,1] at u^k.
 *     For 1 + tau beta1 xi > 0 the unique solution is the projection
 *        u^k = clamp((u^{k-1} + tau beta1 (gamma*u^{k-1})) / (1 + tau beta1 xi),
 *                    -1, 1);
 *   - the output of interest f_1 = (1 + mean(u))/2 at the final step
 *     (eq. ooi, lumped quadrature, |Omega| = 1);
 *   - the discrete nonlocal energy
 *        E_h(u) = h^2 [ 1/4 sum_i sum_{d in D} w_d (u_i - u_{i+d})^2
 *                       + c_F/2 sum_i (1 - u_i^2) ]
 *     (the Ginzburg-Landau energy of Sec. 2 with the nonlocal interaction in
 *     place of the gradient term), used as a diagnostic.
 *
 * Readings of points the paper leaves open (disc inclusion test, self term,
 * discrete c_gamma, periodic torus) are listed in the design notes; every
 * function below states the one it uses.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC nlch_oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_KERNEL_CONSTANT 0
#define ORC_KERNEL_GAUSSIAN 1

/* ---------------------------------------------------------------------
 * Disc geometry (integer work).
 * Offsets d = (dy, dx) belong to the disc iff dy^2 + dx^2 <= R2, with
 * R2 = floor((delta n)^2 + 1e-9): the closed ball |d| h <= delta of
 * Sec. 2.1, with a 1e-9 guard so that delta*n a hair below an integer (from
 * decimal input) does not drop the boundary ring.
 * m = largest integer with m^2 <= R2; halfw[dy + m] = largest dx >= 0 with
 * dy^2 + dx^2 <= R2.  Found by plain scanning (no square roots).
 * Returns 0, or -1 if the arguments are out of range or cap is too small.
 * ------------------------------------------------------------------- */
int orc_disc(int n, double delta, int64_t *R2_out, int *m_out, int64_t *N_out,
             int *halfw, int cap)
{
    if (n <= 0 || !(delta >= 0.0) || !isfinite(delta)) return -1;
    double r = delta * (double)n;
    int64_t R2 = (int64_t)floor(r * r + 1e-9);
    int m = 0;
    while ((int64_t)(m + 1) * (m + 1) <= R2) m++;
    if (halfw && 2 * m + 1 > cap) return -1;
    int64_t N = 0;
    for (int dy = -m; dy <= m; dy++) {
        int w = 0;
        while ((int64_t)dy * dy + (int64_t)(w + 1) * (w + 1) <= R2) w++;
        if (halfw) halfw[dy + m] = w;
        N += 2 * w + 1;
    }
    if (R2_out) *R2_out = R2;
    if (m_out) *m_out = m;
    if (N_out) *N_out = N;
    return 0;
}

/* Kernel gamma(r) for r <= delta (Sec. 4, eq. kernel_gauss; constant kernel
 * on the same disc).  Gaussian: amp * exp(-r^2 / sigma^2). */
double orc_gamma(int kind, double amp, double sigma, double r)
{
    if (kind == ORC_KERNEL_GAUSSIAN) return amp * exp(-(r * r) / (sigma * sigma));
    return amp;
}

/* Disc offsets and weights in canonical order (dy ascending, then dx
 * ascending).  w_d = h^2 gamma(h |d|) (nodal quadrature, self term d = 0
 * included).  c_gamma_h = sum of all w_d in that order.  Returns N, or -1. */
int64_t orc_weights(int n, double delta, int kind, double amp, double sigma,
                    int *ddy, int *ddx, double *wd, int64_t cap,
                    double *c_gamma_h)
{
    int64_t R2, N;
    int m;
    if (orc_disc(n, delta, &R2, &m, &N, NULL, 0) != 0) return -1;
    if (N > cap) return -1;
    double h = 1.0 / (double)n;
    int64_t k = 0;
    double c = 0.0;
    for (int dy = -m; dy <= m; dy++) {
        for (int dx = -m; dx <= m; dx++) {
            if ((int64_t)dy * dy + (int64_t)dx * dx > R2) continue;
            double r = h * sqrt((double)dy * dy + (double)dx * dx);
            double w = h * h * orc_gamma(kind, amp, sigma, r);
            if (ddy) ddy[k] = dy;
            if (ddx) ddx[k] = dx;
            if (wd) wd[k] = w;
            c += w;
            k++;
        }
    }
    if (c_gamma_h) *c_gamma_h = c;
    return k;
}

typedef struct {
    int n, N;
    int *ddy, *ddx;
    double *wd;
    double c_gamma;     /* discrete kernel mass, self term included */
} orc_op;

static int op_init(orc_op *op, int n, double delta, int kind, double amp,
                   double sigma)
{
    int64_t R2, N;
    int m;
    memset(op, 0, sizeof(*op));
    if (orc_disc(n, delta, &R2, &m, &N, NULL, 0) != 0) return -1;
    /* The lattice must be wider than the disc, so that every offset reaches
     * a distinct node of the torus. */
    if (n <= 2 * m) return -1;
    op->n = n;
    op->N = (int)N;
    op->ddy = (int *)malloc(sizeof(int) * N);
    op->ddx = (int *)malloc(sizeof(int) * N);
    op->wd = (double *)malloc(sizeof(double) * N);
    if (!op->ddy || !op->ddx || !op->wd) return -1;
    orc_weights(n, delta, kind, amp, sigma, op->ddy, op->ddx, op->wd, N,
                &op->c_gamma);
    return 0;
}

static void op_free(orc_op *op)
{
    free(op->ddy);
    free(op->ddx);
    free(op->wd);
}

static inline int wrap(int a, int n)
{
    a %= n;
    return a < 0 ? a + n : a;
}

/* (gamma * u)_i at site (y, x): nodal quadrature over the disc, periodic. */
static double conv_at(const orc_op *op, const double *u, int y, int x)
{
    int n = op->n;
    double g = 0.0;
    for (int k = 0; k < op->N; k++) {
        /* |dy|, |dx| < n/2, so one conditional shift wraps onto the torus */
        int yy = y + op->ddy[k];
        int xx = x + op->ddx[k];
        yy += (yy < 0) ? n : ((yy >= n) ? -n : 0);
        xx += (xx < 0) ? n : ((xx >= n) ? -n : 0);
        g += op->wd[k] * u[(int64_t)yy * n + xx];
    }
    return g;
}

static inline double clamp1(double v)
{
    return v < -1.0 ? -1.0 : (v > 1.0 ? 1.0 : v);
}

/* One time step of the scheme above at every site.  denom = 1 + tau beta1 xi. */
static void step_all(const orc_op *op, double tb, double denom, const double *u,
                     double *out, int parallel)
{
    int n = op->n;
    if (parallel) {
#pragma omp parallel for schedule(static)
        for (int y = 0; y < n; y++)
            for (int x = 0; x < n; x++) {
                double g = conv_at(op, u, y, x);
                out[(int64_t)y * n + x] =
                    clamp1((u[(int64_t)y * n + x] + tb * g) / denom);
            }
    } else {
        for (int y = 0; y < n; y++)
            for (int x = 0; x < n; x++) {
                double g = conv_at(op, u, y, x);
                out[(int64_t)y * n + x] =
                    clamp1((u[(int64_t)y * n + x] + tb * g) / denom);
            }
    }
}

/* Kahan-compensated accumulation: the energy sums n^2 N positive terms, and
 * a plain running sum would carry ~sqrt(n^2 N) eps of its own rounding. */
static void kahan_add(double *sum, double *comp, double v)
{
    double y = v - *comp;
    double t = *sum + y;
    *comp = (t - *sum) - y;
    *sum = t;
}

/* Discrete energy E_h(u), definition in the header.  Per site the N
 * interaction terms are summed in canonical order; the per-site sums and the
 * potential terms are accumulated with compensation. */
static double energy(const orc_op *op, double c_F, const double *u)
{
    int n = op->n;
    double h2 = 1.0 / ((double)n * n);
    double inter = 0.0, inter_c = 0.0, pot = 0.0, pot_c = 0.0;
    for (int y = 0; y < n; y++)
        for (int x = 0; x < n; x++) {
            double ui = u[(int64_t)y * n + x];
            double site = 0.0;
            for (int k = 0; k < op->N; k++) {
                int yy = wrap(y + op->ddy[k], n);
                int xx = wrap(x + op->ddx[k], n);
                double d = ui - u[(int64_t)yy * n + xx];
                site += op->wd[k] * d * d;
            }
            kahan_add(&inter, &inter_c, site);
            kahan_add(&pot, &pot_c, 1.0 - ui * ui);
        }
    return h2 * (0.25 * inter + 0.5 * c_F * pot);
}

/* Scheme coefficients; returns -1 unless 1 + tau beta1 xi > 0. */
static int coeffs(const orc_op *op, double c_F, double beta1, double tau,
                  double *tb, double *denom)
{
    double xi = op->c_gamma - c_F;
    *tb = tau * beta1;
    *denom = 1.0 + tau * beta1 * xi;
    return (*denom > 0.0) ? 0 : -1;
}

/* Model-level constants: c_gamma_h, xi_h = c_gamma_h - c_F. */
int orc_constants(int n, double delta, int kind, double amp, double sigma,
                  double c_F, double *c_gamma_h, double *xi_h, int64_t *N)
{
    orc_op op;
    if (op_init(&op, n, delta, kind, amp, sigma) != 0) {
        op_free(&op);
        return -1;
    }
    if (c_gamma_h) *c_gamma_h = op.c_gamma;
    if (xi_h) *xi_h = op.c_gamma - c_F;
    if (N) *N = op.N;
    op_free(&op);
    return 0;
}

/* (gamma * u) at every site (the explicit convolution term). */
int orc_convolve(int n, double delta, int kind, double amp, double sigma,
                 const double *u, double *g)
{
    orc_op op;
    if (op_init(&op, n, delta, kind, amp, sigma) != 0) {
        op_free(&op);
        return -1;
    }
    for (int y = 0; y < n; y++)
        for (int x = 0; x < n; x++) g[(int64_t)y * n + x] = conv_at(&op, u, y, x);
    op_free(&op);
    return 0;
}

/* One step of the scheme from state u (no initial projection). */
int orc_step(int n, double delta, int kind, double amp, double sigma, double c_F,
             double beta1, double tau, const double *u, double *out)
{
    orc_op op;
    double tb, denom;
    if (op_init(&op, n, delta, kind, amp, sigma) != 0 ||
        coeffs(&op, c_F, beta1, tau, &tb, &denom) != 0) {
        op_free(&op);
        return -1;
    }
    step_all(&op, tb, denom, u, out, 1);
    op_free(&op);
    return 0;
}

/* One step evaluated only at the listed sites (flat indices y n + x). */
int orc_step_sites(int n, double delta, int kind, double amp, double sigma,
                   double c_F, double beta1, double tau, const double *u,
                   const int64_t *sites, int64_t nsites, double *out)
{
    orc_op op;
    double tb, denom;
    if (op_init(&op, n, delta, kind, amp, sigma) != 0 ||
        coeffs(&op, c_F, beta1, tau, &tb, &denom) != 0) {
        op_free(&op);
        return -1;
    }
    for (int64_t s = 0; s < nsites; s++) {
        int64_t i = sites[s];
        if (i < 0 || i >= (int64_t)n * n) {
            op_free(&op);
            return -1;
        }
        int y = (int)(i / n), x = (int)(i % n);
        out[s] = clamp1((u[i] + tb * conv_at(&op, u, y, x)) / denom);
    }
    op_free(&op);
    return 0;
}

double orc_energy(int n, double delta, int kind, double amp, double sigma,
                  double c_F, const double *u)
{
    orc_op op;
    if (op_init(&op, n, delta, kind, amp, sigma) != 0) {
        op_free(&op);
        return NAN;
    }
    double e = energy(&op, c_F, u);
    op_free(&op);
    return e;
}

/* Sum of u (left to right) -> mean and f_1 = (1 + mean)/2 (eq. ooi). */
static void ooi(int n, const double *u, double *mean_f1)
{
    double s = 0.0;
    for (int64_t i = 0; i < (int64_t)n * n; i++) s += u[i];
    double mean = s / ((double)n * n);
    mean_f1[0] = mean;
    mean_f1[1] = 0.5 * (1.0 + mean);
}

/* Full solve of one sample: u^0 = clamp(u0) (the initial datum projected
 * onto the admissible set), then nsteps steps, then the output of interest.
 * energy_out (nsteps + 1 values, or NULL) receives E_h(u^k) for k = 0..nsteps.
 * parallel != 0 spreads each step's rows over OpenMP threads. */
static int solve_one(const orc_op *op, double c_F, double beta1, double tau,
                     int nsteps, const double *u0, double *u_out,
                     double *mean_f1, double *energy_out, int parallel)
{
    double tb, denom;
    if (coeffs(op, c_F, beta1, tau, &tb, &denom) != 0 || nsteps < 0) return -1;
    int64_t nn = (int64_t)op->n * op->n;
    double *a = (double *)malloc(sizeof(double) * nn);
    double *b = (double *)malloc(sizeof(double) * nn);
    if (!a || !b) {
        free(a);
        free(b);
        return -1;
    }
    for (int64_t i = 0; i < nn; i++) a[i] = clamp1(u0[i]);
    if (energy_out) energy_out[0] = energy(op, c_F, a);
    for (int k = 1; k <= nsteps; k++) {
        step_all(op, tb, denom, a, b, parallel);
        double *t = a;
        a = b;
        b = t;
        if (energy_out) energy_out[k] = energy(op, c_F, a);
    }
    if (u_out) memcpy(u_out, a, sizeof(double) * nn);
    if (mean_f1) ooi(op->n, a, mean_f1);
    free(a);
    free(b);
    return 0;
}

int orc_solve(int n, double delta, int kind, double amp, double sigma,
              double c_F, double beta1, double tau, int nsteps,
              const double *u0, double *u_out, double *mean_f1,
              double *energy_out)
{
    orc_op op;
    if (op_init(&op, n, delta, kind, amp, sigma) != 0) {
        op_free(&op);
        return -1;
    }
    int rc = solve_one(&op, c_F, beta1, tau, nsteps, u0, u_out, mean_f1,
                       energy_out, 1);
    op_free(&op);
    return rc;
}

/* Many independent samples of one lattice/horizon/kernel shape, each with its
 * own c_F and kernel amplitude (the sampled inputs of Sec. 4).  u0 and u_out
 * hold nsamp consecutive n x n states; mean_f1 holds 2 values per sample.
 * Samples are spread over OpenMP threads; each sample is solved serially. */
int orc_solve_many(int n, double delta, int kind, double sigma, double beta1,
                   double tau, int nsteps, int64_t nsamp, const double *c_F,
                   const double *amp, const double *u0, double *u_out,
                   double *mean_f1)
{
    int64_t nn = (int64_t)n * n;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int64_t s = 0; s < nsamp; s++) {
        orc_op op;
        if (op_init(&op, n, delta, kind, amp[s], sigma) != 0) {
            bad |= 1;
        } else {
            bad |= (solve_one(&op, c_F[s], beta1, tau, nsteps, u0 + s * nn,
                              u_out ? u_out + s * nn : NULL, mean_f1 + 2 * s,
                              NULL, 0) != 0);
        }
        op_free(&op);
    }
    return bad ? -1 : 0;
}

/* Number of OpenMP threads the parallel loops above use. */
int orc_threads(void) { return omp_get_max_threads(); }
