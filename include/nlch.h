/*
 * nlch.h -- C ABI of libnlch.so, the MI355X (gfx950) solver for the nonlocal
 * phase-field model with obstacle potential and its multifidelity Monte Carlo
 * estimator (arXiv 2310.10750).
 *
 * The model (Sec. 2.1, eq. nonl_CH_nm with beta2 = 0, the non-mass-conserving
 * nonlocal Allen-Cahn case the paper names there):
 *     du/dt + beta1 w = 0,   w = L u + dF_obs(u),
 *     L u = c_gamma u - gamma * u                         (eq. nonl_operator)
 *     F_obs(u) = c_F/2 (1 - u^2) + indicator of [-1, 1]   (eq. potential_obstacle)
 * on the periodic unit square, discretised on an n x n lattice (h = 1/n) with
 * nodal (lumped) quadrature of the convolution over the horizon disc
 *     D = { d in Z^2 : |d|^2 <= R2 },  R2 = floor((delta n)^2 + 1e-9),
 *     w_d = h^2 gamma(h |d|),  c_gamma_h = sum_{d in D} w_d (self term included),
 *     xi_h = c_gamma_h - c_F                               (eq. xi_constant)
 * and implicit Euler with the convolution explicit (Sec. 4):
 *     u^k = clamp((u^{k-1} + tau beta1 (gamma*u^{k-1})) / (1 + tau beta1 xi_h), -1, 1),
 * which the library evaluates in the algebraically equal difference form
 *     v = u + c1 (c_F u - sum_{d != 0} w_d (u - u_{+d})),
 *     c1 = tau beta1 / (1 + tau beta1 xi_h),   u' = clamp(v, -1, 1).
 * The output of interest is f_1 = (1 + mean(u^T)) / 2 (eq. ooi).
 *
 * With beta2 > 0 (eq. nonl_CH_nm with both terms, du/dt + A w = 0,
 * A = beta1 I - beta2 Delta; Delta_h the periodic 5-point Laplacian of lumped
 * P1 elements) each step solves the coupled variational inequality
 *     u + tau A (xi_h u + mu) = u^{k-1} + tau A (gamma*u^{k-1}),
 *     mu in the normal cone of [-1, 1]^{n^2} at u,
 * which for xi_h > 0 has a unique solution: with z = xi_h u + mu,
 * u = clamp(z / xi_h) and z is the root of a strictly convex gradient, found
 * by semismooth Newton with Jacobi-preconditioned conjugate-gradient inner
 * solves (one workgroup per sample, n <= 256; the Newton residual and its
 * convergence test are FP64, the on-chip variant for n = 64, 88, 128 keeps
 * the CG direction in FP32 and the CG solution as an FP32 pair).  For
 * xi_h <= 0 the term xi_h u is concave, and the literal step may have
 * several solutions; the library then takes it at the previous step (convex
 * splitting):
 *     u + tau A mu = u^{k-1} + tau A (gamma*u^{k-1} - xi_h u^{k-1}),
 * whose unique solution is found by a primal-dual active-set iteration with
 * conjugate-gradient solves on the active rows of tau A (same layouts and
 * precisions; converged when the active sets repeat and the FP64 residual of
 * the active rows is below 1e-13 max(1, |right-hand side|)).  A batch may mix
 * both signs.  A sample whose Newton (or active-set) iteration does not
 * converge within its iteration cap gets a NaN state and output of interest.
 * Per sample the library keeps 7 n^2 doubles of workspace with the batch;
 * within one nlch_solve_batch call each step starts from the previous step's
 * z (xi_h > 0) or mu (xi_h <= 0) held there (from xi_h u, or from mu = 0, at
 * the call's first step), so a solve split over several calls agrees with one
 * call to the solver tolerance (~1e-13 relative), not bit for bit.
 *
 * Bounded domain (NLCH_BOUNDARY_VOLUME; Sec. 2.1: the operator integrates
 * over Omega = (0,1)^2 together with the interaction region Omega_I of points
 * outside Omega within delta of it).  The paper does not state the values
 * imposed on Omega_I; this library reads them as a volume constraint: u on
 * Omega_I is data that the evolution keeps fixed.  Omega's lattice is n x n
 * (h = 1/n) and is continued by m = floor(sqrt(R2)) nodes on every side,
 * which holds every node of Omega_I a disc centred in Omega reaches.  A
 * sample's state is then the (n + 2m) x (n + 2m) array (row-major, element
 * (y, x) at y*(n + 2m) + x) whose inner n x n block, rows and columns
 * m .. m + n - 1, is Omega and whose ring of width m holds the Omega_I data.
 * Every disc centred in Omega lies in Omega and Omega_I, so c_gamma_h, xi_h
 * and the update are those of the torus; only Omega's nodes are updated, the
 * ring is copied (after the initial projection onto [-1, 1], which covers
 * every node), and the output of interest is the mean over Omega's n^2
 * nodes.  This mode needs beta2 = 0 and runs without the energy trace; every
 * algorithm applies (RESIDENT for n = 64 and 128).
 *
 * Conventions for every entry point:
 *  - Status: 0 on success, else one of the NLCH_E* codes; the message of the
 *    last failure on the calling thread is returned by nlch_last_error().
 *  - All arguments are validated on the host before anything is enqueued, so
 *    a call that fails validation leaves every buffer untouched.  Errors of
 *    enqueued device work (NLCH_EDEVICE) may surface at a later call or when
 *    the caller synchronises the stream.
 *  - Device buffers are owned by the caller and must stay valid until the
 *    enqueued work completes; the library only allocates small internal
 *    tables (geometry, sample descriptors, graph caches) that it reuses.
 *  - Lattice states are row-major, element (y, x) at index y*n + x, with the
 *    element type given by the precision: double (NLCH_F64), float (NLCH_F32)
 *    or IEEE binary16 (NLCH_F16_STORE: state stored in FP16, arithmetic in
 *    FP32, every stored value rounded to nearest-even).
 *  - hip_stream is a hipStream_t (NULL = the null stream).
 *  - Calls that enqueue work on the same device buffers must not overlap.
 *  - Calls with the same signature (models, samples, precision, algorithm
 *    word, and whether it is nlch_step or a batch solve) share small device
 *    scratch the library keeps for that signature (output-of-interest chunk
 *    sums, energy partials, beta2 > 0 workspaces).  The library orders such
 *    calls: a call on another stream than the previous one of its signature
 *    waits for it with an event.  Work enqueued while hip_stream is capturing
 *    a graph is not ordered this way: the caller orders captured calls of
 *    one signature.
 */
#ifndef NLCH_H
#define NLCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define NLCH_OK 0
#define NLCH_EINVAL (-1)       /* invalid argument (nothing enqueued)           */
#define NLCH_EUNSUPPORTED (-2) /* valid model outside what the library supports */
#define NLCH_EDEVICE (-3)      /* HIP runtime error                              */
#define NLCH_ENOMEM (-4)       /* internal table allocation failed               */

/* Kernel gamma on |r| <= delta (Sec. 4, eq. kernel_gauss). */
#define NLCH_KERNEL_CONSTANT 0 /* gamma(r) = amp                                 */
#define NLCH_KERNEL_GAUSSIAN 1 /* gamma(r) = amp * exp(-r^2 / sigma^2)           */

/* State element type / arithmetic. */
#define NLCH_F64 0       /* FP64 storage, FP64 arithmetic                       */
#define NLCH_F32 1       /* FP32 storage, FP32 arithmetic                       */
#define NLCH_F16_STORE 2 /* FP16 storage, FP32 arithmetic                       */

/* Algorithm selection (low byte) and flags. */
#define NLCH_ALGO_AUTO 0     /* RESIDENT where a sample fits in LDS, else ROWRUN
                                where built for the disc, else DIRECT          */
#define NLCH_ALGO_DIRECT 1   /* per-site disc sum, one launch per step         */
#define NLCH_ALGO_ROWRUN 2   /* disc as row runs of window sums, one launch per
                                step (discs with R2 in nlch_rowrun_supported)  */
#define NLCH_ALGO_RESIDENT 3 /* whole sample in LDS for all steps, one launch  */
#define NLCH_ALGO_ACC64 0x100    /* accumulate disc sums in FP64 (F32/F16 only)  */
#define NLCH_ALGO_NOGRAPH 0x200  /* enqueue launches directly, no graph replay   */
#define NLCH_ALGO_CHECK_FINITE 0x400 /* reject non-finite u0 with NLCH_EINVAL;
                                        synchronises hip_stream                 */
#define NLCH_ALGO_AUTOTUNE 0x800 /* on the first call of a batch, time the
                                    streaming kernel's launch shapes (lanes'
                                    columns, band height, waves per band,
                                    row phases per wave) on
                                    the caller's buffers (reads state, writes
                                    scratch), and the resident kernel's
                                    layouts (see nlch_set_resident_shape) on
                                    a copy of the states in a temporary
                                    device buffer (min(nsteps, 10) steps;
                                    the default layout unless another is 3%
                                    faster); keep the fastest (cached per
                                    process);
                                    synchronises hip_stream (the resident
                                    layouts are not tuned while hip_stream is
                                    being captured).  Shapes that split a band
                                    over several waves or two row phases, and
                                    resident layouts
                                    other than the default, sum some outputs
                                    in a different grouping: results can
                                    differ from the default by rounding only.
                                    Without this flag the shape is a fixed
                                    function of the batch, so results repeat
                                    exactly. */

/* Domain of a model. */
#define NLCH_BOUNDARY_PERIODIC 0 /* periodic unit square, state n x n          */
#define NLCH_BOUNDARY_VOLUME 1   /* Omega = (0,1)^2 with fixed values on
                                    Omega_I, state (n + 2m) x (n + 2m)         */

/* One fidelity level ("model"): lattice, horizon, kernel and evolution
 * parameters (Sec. 2.1 and Sec. 4). */
typedef struct nlch_model {
    int32_t n;           /* lattice size n x n on [0,1)^2, h = 1/n; n > 2m     */
    int32_t kernel;      /* NLCH_KERNEL_*                                       */
    double delta;        /* horizon; m = floor(sqrt(R2)) must be <= 48         */
    double kernel_amp;   /* amp > 0                                             */
    double kernel_sigma; /* Gaussian width > 0 (ignored for the constant kernel)*/
    double c_F;          /* obstacle-potential constant > 0                     */
    double beta1;        /* > 0                                                 */
    double beta2;        /* >= 0; > 0 needs n <= 256 (either sign of xi_h)     */
    double tau;          /* time step > 0; with beta2 = 0, 1 + tau beta1 xi_h > 0 */
    int32_t boundary;    /* NLCH_BOUNDARY_*                                     */
    int32_t reserved;    /* must be 0                                           */
} nlch_model;

/* One sampled input of a batch: its model, its own c_F and kernel amplitude
 * (the random parameters of Sec. 4), and the element offset of its state
 * (n x n elements, (n + 2m) x (n + 2m) under NLCH_BOUNDARY_VOLUME) inside the
 * batch buffers. */
typedef struct nlch_sample {
    int32_t model;      /* index into the models array                          */
    int32_t reserved;   /* must be 0                                            */
    double c_F;         /* > 0                                                  */
    double kernel_amp;  /* > 0                                                  */
    int64_t offset;     /* element offset; states must not overlap             */
} nlch_sample;

/* Results of mfmc_estimate (K <= NLCH_MFMC_MAX_K models). */
#define NLCH_MFMC_MAX_K 8
typedef struct mfmc_result {
    double q_mfmc;                     /* eq. MFMC_estimator                     */
    double q_mc;                       /* mean of model 1 over its m_1 samples   */
    double mean_mj[NLCH_MFMC_MAX_K];   /* mean of model j over its first m_j     */
    double mean_mjm1[NLCH_MFMC_MAX_K]; /* over its first m_{j-1} (j >= 2)        */
    double var[NLCH_MFMC_MAX_K];       /* sample variance over the first m_1     */
    double rho[NLCH_MFMC_MAX_K];       /* correlation with model 1, first m_1    */
    double alpha[NLCH_MFMC_MAX_K];     /* coefficients used (alpha[0] = 1)       */
} mfmc_result;

/* Disc geometry (host only, no device needed).  Writes R2, m = floor(sqrt(R2)),
 * N = |D| and, if halfw != NULL, the row half-widths halfw[dy + m] =
 * floor(sqrt(R2 - dy^2)) for dy = -m..m (cap >= 2m+1 entries).
 * NLCH_EINVAL for n <= 0, a negative or non-finite delta, or a short cap. */
int nlch_disc(int32_t n, double delta, int64_t *R2, int32_t *m, int64_t *N,
              int32_t *halfw, int32_t cap);

/* Discrete model constants (host only): c_gamma_h (kernel mass with the self
 * term), xi_h = c_gamma_h - c_F and c1 = tau beta1 / (1 + tau beta1 xi_h), for
 * the model's own c_F and amplitude (c1 = 0 for a beta2 > 0 model with
 * 1 + tau beta1 xi_h <= 0, whose step does not use it).  Any output pointer
 * may be NULL.
 * NLCH_EINVAL if the model is invalid (see nlch_model). */
int nlch_model_constants(const nlch_model *model, double *c_gamma_h,
                         double *xi_h, double *c1);

/* One time step of the scheme for a single n x n state (model's c_F and
 * kernel_amp): u_out = step(u_in).  u_in, u_out: device arrays of n*n
 * elements of the precision's type, distinct and non-overlapping (the stencil
 * reads neighbours).  ooi_out: NULL, or a device array of 2 doubles that
 * receives {mean(u_out), f_1(u_out)} (eq. ooi).  algo: NLCH_ALGO_DIRECT or
 * NLCH_ALGO_ROWRUN (AUTO picks one), optionally | NLCH_ALGO_ACC64.  No initial
 * projection: u_in is used as given.  Exactly one launch of the step kernel
 * (plus one reduction launch if ooi_out != NULL).  NLCH_BOUNDARY_VOLUME:
 * u_in and u_out hold (n + 2m)^2 elements; the ring of u_out receives the
 * ring of u_in projected onto [-1, 1] (one more elementwise launch before the
 * step). */
int nlch_step(const nlch_model *model, int32_t precision, int32_t algo,
              const void *u_in, void *u_out, double *ooi_out, void *hip_stream);

/* nlch_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and results as nlch_step, but the model's device
 * tables and the chunk sums of the output-of-interest reduction live in one
 * static device area of 128 KiB per GPU, written by small kernels whose
 * arguments carry the values: the call allocates no device memory and copies
 * nothing from the host.  Limits: beta2 = 0 only, and the tables plus
 * ceil(n^2 / 16384) doubles of chunk sums (when ooi_out != NULL) must fit
 * the area: n <= 16287 on the row-run kernel, down to n <= 14354 on the
 * direct kernel at the widest horizon (m = 48); larger requests are
 * NLCH_EUNSUPPORTED before any device work.  Every call on a GPU uses that
 * GPU's area and leaves its tables there: calls that overlap on one GPU
 * (other streams, concurrent graph replays) race on it, so the caller must
 * order them. */
int nlch_step_noalloc(const nlch_model *model, int32_t precision, int32_t algo,
                      const void *u_in, void *u_out, double *ooi_out, void *hip_stream);

/* Solve a batch: for every sample s, u^0 = clamp(state_s, -1, 1) (the initial
 * datum projected onto [-1, 1]), nsteps steps of the scheme with the sample's
 * model, c_F and amplitude, then u^nsteps is left in state_s and
 * {mean, f_1} in ooi_out[2s], ooi_out[2s+1] (FP64).
 * models: n_models >= 1 host structs; samples: n_samples >= 1 host structs.
 * state: device buffer holding every sample's state at its offset
 * (in: u0, out: final state).  scratch: device buffer of the same extent,
 * used as the ping-pong partner (may be NULL when every sample runs
 * RESIDENT; under NLCH_BOUNDARY_VOLUME the streaming kernels write the
 * projected ring to both buffers, the resident kernel to state only).
 * ooi_out: device array of 2*n_samples doubles.
 * Samples of different models (uneven n and horizon) may be mixed; the
 * library never reorders outputs.  Without NLCH_ALGO_NOGRAPH the sequence of
 * launches is captured once into a HIP graph per distinct call signature
 * (buffers, batch, nsteps, algo) and replayed on later calls; a batch keeps
 * up to 16 graphs (a 17th signature drops them after synchronising the
 * device).
 * NaN in u0 propagates to the outputs unless NLCH_ALGO_CHECK_FINITE is set. */
int nlch_solve_batch(const nlch_model *models, int32_t n_models,
                     const nlch_sample *samples, int64_t n_samples,
                     int32_t nsteps, int32_t precision, int32_t algo,
                     void *state, void *scratch, double *ooi_out,
                     void *hip_stream);

/* nlch_solve_batch with the discrete energy trace (diagnostic; the energy of
 * Sec. 2 with the nonlocal interaction term and the obstacle potential):
 *   E_h(u) = h^2 [ 1/4 sum_i sum_{d in D} w_d (u_i - u_{i+d})^2
 *                  + c_F/2 sum_i (1 - u_i^2) ],   w_d = h^2 gamma(h|d|),
 * evaluated in FP64 on the stored states as h^2 [ 1/2 sum_i u_i L_i +
 * c_F/2 sum_i (1 - u_i^2) ] with L_i the operator sum of the step (equal on
 * the torus because the disc is symmetric); L_i is accumulated in the
 * arithmetic of the step, the two sums in FP64.
 * energy_out: device array of (nsteps + 1) * n_samples doubles, caller-owned;
 * energy_out[k * n_samples + s] = E_h(u^k) of sample s, k = 0 (projected
 * initial state) .. nsteps, with the sample's own c_F and kernel amplitude.
 * The energy is reduced inside the step kernels; it costs one more operator
 * evaluation per sample for k = nsteps (whose update goes to `scratch`, whose
 * contents are unspecified afterwards) and, for the streaming kernels, one
 * small reduction launch per step.  All other arguments, results and errors
 * are those of nlch_solve_batch; energy_out == NULL is NLCH_EINVAL, and a
 * model with NLCH_BOUNDARY_VOLUME is NLCH_EUNSUPPORTED. */
int nlch_solve_batch_energy(const nlch_model *models, int32_t n_models,
                            const nlch_sample *samples, int64_t n_samples,
                            int32_t nsteps, int32_t precision, int32_t algo,
                            void *state, void *scratch, double *ooi_out,
                            double *energy_out, void *hip_stream);

/* Manual launch shape of the streaming (ROWRUN) kernel for later
 * nlch_solve_batch calls in this process, overriding the default shape and
 * NLCH_ALGO_AUTOTUNE: R columns per lane (1 or 2), W waves per band (1, 2,
 * 4 or 8), each of the first W-1 waves walking `periods` ring periods of
 * 2m+1 rows (W > 1), and band height B (W = 1); 0 keeps the default of a
 * field, and (0, 0, 0, 0) restores the default shape.  W > 1 applies to
 * groups with FP32 arithmetic and m <= 32 (others use W = 1); a group whose
 * partial-sum areas for W waves would not fit in LDS uses fewer waves.
 * Results change with W > 1 by rounding only (see NLCH_ALGO_AUTOTUNE).
 * R = 4 (other fields 0) selects the tiled one-step kernel (32 x 32 output
 * tiles with their halo staged in LDS) for the groups and discs it is built
 * for (FP32 or FP16 arithmetic, m <= 16), with states bit-identical to
 * R = 1, W = 1; it is also the default for one or a few samples of a lattice,
 * where the streaming shape would give fewer than 1024 waves.
 * Host only; returns NLCH_EINVAL for values outside those ranges. */
int nlch_set_stream_shape(int32_t R, int32_t W, int32_t periods, int32_t B);

/* Row phases per wave of the streaming (ROWRUN) kernel for later
 * nlch_solve_batch calls in this process, with the shape of
 * nlch_set_stream_shape and overriding NLCH_ALGO_AUTOTUNE.  phases = 2
 * (groups with FP32 arithmetic and W = 1): the two halves of each wave walk
 * alternate rows of the band (even and odd input rows) over a strip of 32R
 * columns, each forming the window sums of its own rows, and every output
 * adds the partial sums of its two halves (one lane swap).  For a band
 * height this gives twice the waves, so that bands can be twice as tall
 * for the same parallelism and the 2m halo rows of a band (the disc rows
 * above and below it, Sec. 2 eq. nonl_operator) weigh half as much.  Every
 * disc sum is then formed in two parts, so results differ from phases = 1
 * by rounding only.  phases = 1: one phase (one wave or W waves per band;
 * the tiled kernel is then not used); 0: not forced (the default, or the
 * autotuner's choice).  Host only; NLCH_EINVAL outside 0..2. */
int nlch_set_stream_phases(int32_t phases);

/* Layout of the LDS-resident (RESIDENT) kernel for later nlch_solve_batch
 * calls in this process, overriding the default and NLCH_ALGO_AUTOTUNE.
 * 128^2 lattices (FP32 state; periodic, or Omega inside its fixed ring, where
 * (4, 8) and (2, 16) are built and (4, 16) runs as (2, 16)): each lane owns
 * cols_per_lane adjacent columns and walks rows_per_lane rows of a 16-row
 * band.
 *   (2, 16): one band per wave; every resident case.
 *   (4, 16): two bands per wave (one per half-wave), 16-byte LDS window
 *            loads; bit-identical to (2, 16).
 *   (4, 8):  one band per wave, its two half-waves walking 8 rows each and
 *            adding each other's sums with a lane swap; 8 waves per sample,
 *            so that a CU's two resident samples give four waves per SIMD.
 *            Band sums are formed in two parts, so results differ from
 *            (2, 16) by FP32 rounding only.
 * 64^2 lattices (periodic domain): one column per lane, one band of
 * rows_per_lane rows per wave:
 *   (1, 8) (discs with m <= 8; FP32 or FP64 state), (1, 16), (1, 32) (FP32
 *            state): 8, 4 or 2 waves per sample.  The partial sums a band
 *            hands to its neighbours group the disc rows differently, so
 *            results differ from (1, 16) by rounding only.
 * A shape applies to the groups of the lattice it names; other groups, and
 * cases a layout is not built for, keep their default.
 *   (0, 0):  the default: (4, 8) on 128^2 where built, else 16-row bands
 *            ((2, 16) on 128^2, (1, 16) on 64^2); with NLCH_ALGO_AUTOTUNE,
 *            the layout timed fastest for the batch signature.
 * With the energy trace the same layouts run.  Host only; NLCH_EINVAL for
 * other values. */
int nlch_set_resident_shape(int32_t cols_per_lane, int32_t rows_per_lane);

/* Multifidelity Monte Carlo estimate (Sec. 3.2) from K model outputs.
 * y_dev[j]: device pointer to the outputs of model j+1, the output for
 * parameter draw i at y_dev[j][i * y_stride] for i < m[j] (draws shared
 * across models: model j+1 uses draws 0..m[j]-1).  y_stride >= 1; pass 2
 * and &ooi_out[2*s0 + 1] to read the f_1 values of nlch_solve_batch output
 * in place.  m: host array, non-decreasing, m[0] >= 2 (m[0] >= 1 when
 * alpha is given: the below-minimum-budget allocation of Sec. 4 can give
 * m_1 = 1; var and rho are then NaN).
 * alpha: NULL (estimate alpha_j = rho_{1j} sigma_1 / sigma_j, eq. alpha, from
 * the first m[0] shared draws; zero-variance models get alpha = 0) or K-1 host
 * values for models 2..K.  Moments are accumulated in FP64 on the device
 * (two-pass); the call synchronises hip_stream and fills *out on the host.
 * Q_MFMC = mean_1(m_1) + sum_j alpha_j (mean_j(m_j) - mean_j(m_{j-1}))
 * (eq. MFMC_estimator). */
int mfmc_estimate(int32_t K, const int64_t *m, const double *const *y_dev,
                  int64_t y_stride, const double *alpha, mfmc_result *out,
                  void *hip_stream);

/* Model selection (Sec. 3.1): a pool of K models (K <= NLCH_MFMC_MAX_POOL),
 * model 0 the high-fidelity one, with per-sample costs cost[k] > 0 and
 * correlations rho[k] = rho_{1,k} (rho[0] = 1, |rho[k]| <= 1).  Every subset
 * holding model 0 and at least one surrogate (2^(K-1) - 1 candidates) is
 * ordered by decreasing rho^2 and kept if the squared correlations strictly
 * decrease (eq. conditiona) and eq. conditionb holds for j = 2..|S| with
 * rho_{i_{|S|+1}} = 0.  Kept subsets are written to out (up to cap of them),
 * sorted by increasing variance reduction ratio V (eq.
 * variance_reduction_ratio; ties keep candidate order), each with
 * B_min / C_1 = sqrt(V / (1 - rho_{1,i_2}^2)) (eq. bmin).  Returns the number
 * of kept subsets (>= 0) or an NLCH_E* code; *n_candidates (if not NULL)
 * receives 2^(K-1) - 1.  Host only. */
#define NLCH_MFMC_MAX_POOL 16
typedef struct mfmc_subset {
    int32_t size;                        /* |S|                                 */
    int32_t models[NLCH_MFMC_MAX_POOL];  /* pool indices, decreasing rho^2      */
    double V;                            /* variance reduction ratio            */
    double bmin_over_c1;                 /* minimum budget / C_1                */
} mfmc_subset;
int mfmc_select(int32_t K, const double *cost, const double *rho, mfmc_subset *out,
                int32_t cap, int32_t *n_candidates);

/* Sample allocation for budget B (Sec. 3.2): for a subset of S pool indices
 * (model 0 first, decreasing rho^2), oversampling ratios r_j (eq. rk),
 * m_1* = B / sum_j C_{i_j} r_j and m_j = m_1* r_j (eq. samples), written to
 * m_real; m_int gets their floors (the Remark after eq. bmin).  When m_1* < 1
 * (B below B_min) the samples follow the below-minimum-budget rule of Sec. 4:
 * while some model j < S has m_j < j, the smallest such j and the models
 * before it take m_l = l and the remaining budget B - sum_{l<=j} l C_{i_l} is
 * shared by the later models with ratios relative to model j+1; budgets with
 * B < sum_l l C_{i_l} are rejected (NLCH_EINVAL).  *m1_star (if not NULL)
 * receives m_1* of eq. samples.  Host only. */
int mfmc_allocate(int32_t S, const int32_t *subset, const double *cost, const double *rho,
                  double budget, double *m_real, int64_t *m_int, double *m1_star);

/* The disc sizes R2 for which ROWRUN kernels are compiled for a precision
 * (NLCH_F*; RESIDENT uses the subset with m <= 8): writes up to cap values
 * into r2_list and returns the total count, or NLCH_EINVAL.  Host only. */
int nlch_rowrun_supported(int32_t precision, int64_t *r2_list, int32_t cap);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char *nlch_last_error(void);

/* Failure injection, for tests of callers' and the library's error handling
 * (host only): the nth checked HIP runtime call the library makes from now on
 * (nth >= 1; counted over all threads) is not made and reports failure, so
 * the entry point that reaches it returns NLCH_EDEVICE with a message that
 * contains "injected"; nth = 0 disarms.  Nothing is issued to the device in
 * place of the skipped call, and the library stays usable: work enqueued
 * before the failure may have run on the caller's buffers, later calls work
 * as usual.  NLCH_EINVAL for nth < 0. */
int nlch_debug_inject_device_error(int32_t nth);

/* ABI version: 6 (increments on any change to a struct, constant or function
 * signature declared here). */
int nlch_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NLCH_H */
