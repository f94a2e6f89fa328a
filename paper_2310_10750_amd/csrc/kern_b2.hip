// The time step with beta2 > 0: eq. nonl_CH_nm with beta1 > 0 and beta2 > 0
// (the non-mass-conserving model of the paper's experiments), discretised as
// in Sec. 4 -- implicit Euler with the convolution explicit, nodal
// quadrature of the convolution, A = beta1 I - beta2 Delta_h with the
// periodic 5-point Laplacian (lumped P1 elements on the uniform mesh):
//
//     u + tau A (xi u + mu) = r,   r = u_old + tau A g,   g = gamma * u_old,
//     mu in the normal cone of K = [-1, 1]^{n^2} at u.
//
// For xi > 0 write z = xi u + mu: then u = P_K(z / xi), and z is the root of
// F(z) = tau A z + P_K(z / xi) - r, the gradient of the strictly convex
// Phi(z) = tau/2 z'Az + sum_i phi(z_i) - r'z with phi(s) = s^2/(2 xi) for
// |s| <= xi and |s| - xi/2 otherwise, so the step is unique.  Semismooth
// Newton on F: the Jacobian tau A + diag(1/xi where |z| < xi) is symmetric
// positive definite and each system is solved by conjugate gradients with
// the matrix-free 5-point stencil; the step length comes from Armijo
// backtracking on Phi.  The first step of a solve starts Newton from
// z = xi u_old; every later step of the same solve starts from the previous
// step's z, kept in the workspace (warm start), so a solve split over several
// calls agrees with one call to the Newton tolerance, not bit for bit.
//
// For xi <= 0 the term xi u is concave and is taken at the previous step
// (convex splitting; with xi > 0 it stays implicit as above):
//
//     u + tau A mu = r',   r' = u_old + tau A (g - xi u_old),   mu in N_K(u),
//
// a strictly convex problem (u is the projection of r' onto K in the norm of
// (tau A)^{-1}) with a unique solution.  It is solved by the primal-dual
// active-set iteration on the complementarity problem in mu, whose matrix
// tau A is an M-matrix: the active sets A+ = {mu + c (u - 1) > 0} and
// A- = {mu + c (u + 1) < 0} (c = diag(tau A)) fix u = +-1 there and mu = 0
// elsewhere; conjugate
// gradients solve (tau A)_AA mu_A = r'_A - u_A (the rows and columns of the
// inactive sites removed; warm-started from the previous mu), and the
// inactive sites take u_I = r'_I - (tau A mu)_I.  The iteration stops when the
// sets repeat and the residual of the active rows, evaluated afresh in FP64,
// is below 1e-13 max(1, |r'|).  Within a call each step starts from the
// previous step's mu; a call's first step from mu = 0, u = r'.  A batch whose
// samples have both signs of xi launches both kernels; each workgroup of a
// kernel whose sign is not its sample's returns at once.
//
// One workgroup per sample.  k_b2_step keeps every vector in FP64 in a
// per-sample global workspace.  The on-chip variant k_b2_step_lds keeps the
// Newton-level vectors (z, r, F, the Newton direction) and the CG residual in
// FP64, but the CG direction in FP32 and the CG solution as an FP32 pair (high
// part in LDS, low part in registers); the Newton residual test is FP64 in
// both.  Every decision is taken on block-reduced scalars, so control
// flow is uniform across the workgroup; every loop has a fixed cap, and a
// sample whose Newton (or active-set) iteration has not converged at the cap
// gets a NaN state (hence a NaN output of interest).
#include <algorithm>
#include <type_traits>

#include "nlch_device.h"

namespace nlch {

namespace {

constexpr int kB2Threads = 256;
constexpr int kB2Waves = kB2Threads / 64;
constexpr int kMaxNewton = 40;
constexpr int kMaxCg = 4000;
constexpr int kMaxHalvings = 30;
constexpr int kPdasPhase = 20;  // active-set iterations per start (three starts at most)

// Active-set code of a site from (u, mu): +1 (A+: mu + c (u - 1) > 0), -1
// (A-: mu + c (u + 1) < 0), or 0.  Once u = +-1 on the active sites and
// mu = 0 elsewhere, c only decides whether a site may jump from one bound to
// the other in one iteration (|mu| > 2c) rather than pass through the
// inactive set.  On the two-sided constraint the iteration can cycle from
// some starts for any fixed c (the M-matrix convergence result covers
// one-sided obstacles), so a step makes up to three starts of kPdasPhase
// iterations each: from the previous step's mu with c = diag(tau A) (within
// a call), then from mu = 0, u = r' with c = diag(tau A), then from mu = 0,
// u = r' with c = 1.
__device__ __forceinline__ double pdas_code(double u, double mu, double c) {
    return mu + c * (u - 1.0) > 0.0 ? 1.0 : (mu + c * (u + 1.0) < 0.0 ? -1.0 : 0.0);
}

// Stopping level of a split-step CG solve in the norm s.M^-1 s (M^-1 = d_act
// on the active rows): the residual below 1e-14 max(1, |r'|), or, while the
// active sets still change, reduced 10-fold (the sets, not the solve, are
// what those iterations settle; the residual test after the sets repeat
// still asks for the full accuracy).
__device__ __forceinline__ double pdas_cg_stop(double rz0, double d_act, double scale,
                                               bool changed) {
    const double target = d_act * (1e-14 * scale) * (1e-14 * scale);
    return changed ? fmax(1e-2 * rz0, target) : target;
}

__device__ __forceinline__ double clampd(double v) {
    return v < -1.0 ? -1.0 : (v > 1.0 ? 1.0 : v);
}

__device__ __forceinline__ double phi(double s, double xi) {
    const double a = fabs(s);
    return a <= xi ? s * s / (2.0 * xi) : a - 0.5 * xi;
}

// phi(z + d) - phi(z) - d phi'(z), phi'(z) = clamp(z / xi): the part of the
// change of phi beyond its linearisation, exact where z and z + d lie in one
// piece (d^2 / (2 xi) in the quadratic piece, 0 in a linear one), so that the
// line search's decrease test has no cancellation between large terms.
__device__ __forceinline__ double phi_rem(double z, double d, double xi) {
    const double t = z + d;
    const bool qz = fabs(z) <= xi, qt = fabs(t) <= xi;
    if (qz && qt) return d * d / (2.0 * xi);
    if (!qz && !qt && (z > 0.0) == (t > 0.0)) return 0.0;
    return phi(t, xi) - phi(z, xi) - d * clampd(z / xi);
}

// (tau A v)_i = tau beta1 v_i - tau beta2 n^2 (v_E + v_W + v_N + v_S - 4 v_i),
// periodic neighbours of site i = y n + x.
__device__ __forceinline__ double tau_a(const double *v, int i, int y, int x, int n, int nn,
                                        double tb1, double tb2n2) {
    const int ie = x + 1 < n ? i + 1 : i + 1 - n;
    const int iw = x > 0 ? i - 1 : i - 1 + n;
    const int in_ = y + 1 < n ? i + n : i + n - nn;
    const int is = y > 0 ? i - n : i - n + nn;
    const double c = v[i];
    return tb1 * c - tb2n2 * (v[ie] + v[iw] + v[in_] + v[is] - 4.0 * c);
}

// K block-wide FP64 sums in a fixed order (shuffle tree, then the waves in
// order); every thread receives the results.  `red` holds kB2Waves * K.
template <int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double *red) {
#pragma unroll
    for (int k = 0; k < K; ++k)
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();  // the previous use of red is over; this call's stores are done
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) red[w * K + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int i = 0; i < kB2Waves; ++i) s += red[i * K + k];
        v[k] = s;
    }
}

__device__ __forceinline__ double block_sum1(double v, double *red) {
    double a[1] = {v};
    block_sums<1>(a, red);
    return a[0];
}

// SPLIT: the step for xi <= 0 (active-set iteration); else the step for
// xi > 0 (Newton).  Workgroups of the other sign return at once.
template <class TS, bool GAUSS, bool SPLIT>
__global__ __launch_bounds__(kB2Threads) void k_b2_step(
    const SampleDesc *__restrict__ sd, const int32_t *__restrict__ ids,
    const ModelGeo *__restrict__ geo, const double *__restrict__ ewd,
    const TS *__restrict__ in, TS *__restrict__ out, double *__restrict__ ws,
    double *__restrict__ epart, int warm) {
    __shared__ double red[kB2Waves * 4];
    const int j = blockIdx.x;
    const SampleDesc d = sd[ids[j]];
    if ((d.xi > 0.0) == SPLIT) return;
    const int n = geo->n, m = geo->m;
    const int nn = n * n;
    const TS *u = in + d.offset;
    TS *uo = out + d.offset;
    double *R = ws + (int64_t)j * 7 * nn;  // right-hand side r
    double *Z = R + nn;                    // Newton iterate z
    double *F = Z + nn;                    // F(z)
    double *X = F + nn;                    // Newton direction
    double *S = X + nn;                    // CG residual
    double *P = S + nn;                    // CG direction
    double *Q = P + nn;                    // g, then operator products
    const double xi = d.xi;
    const double tb1 = geo->tau_b1, tb2n2 = geo->tau_b2 * (double)nn;
    const double gs = 2.0 * d.e_int * (double)nn;  // h^2 amp
    const double *e = ewd + geo->e_off;
    const int tid = threadIdx.x;

    // g = h^2 amp sum_{d in D} e_d u_{i+d}; energy partials of u_old
    double e_ul = 0.0, e_pot = 0.0;
    for (int i = tid; i < nn; i += kB2Threads) {
        const int y = i / n, x = i - y * n;
        const double ui = (double)u[i];
        double acc = 0.0, lsum = 0.0;
        for (int dy = -m; dy <= m; ++dy) {
            const int ady = dy < 0 ? -dy : dy;
            const int w = geo->halfw[ady];
            const TS *row = u + (int64_t)wrap_once(y + dy, n) * n;
            for (int dx = -w; dx <= w; ++dx) {
                const double v = (double)row[wrap_once(x + dx, n)];
                const double wt = GAUSS ? e[ady * (m + 1) + (dx < 0 ? -dx : dx)] : 1.0;
                acc += wt * v;
                lsum += wt * (ui - v);
            }
        }
        Q[i] = SPLIT ? gs * acc - xi * ui : gs * acc;  // g, or g - xi u_old
        e_ul += ui * lsum;
        e_pot += 1.0 - ui * ui;
    }
    if (epart) {
        double v[2] = {e_ul, e_pot};
        block_sums<2>(v, red);
        if (tid == 0) {
            epart[2 * (int64_t)j] = v[0];
            epart[2 * (int64_t)j + 1] = v[1];
        }
    }
    __syncthreads();
    if constexpr (SPLIT) {
        // r' = u_old + tau A (g - xi u_old); u (U), mu (M, kept between the
        // steps of a call) and the active-set code of the last iteration (C;
        // 2 before the first, so that it counts as a change)
        double *U = Z, *M = F, *C = X;
        double rr = 0.0;
        for (int i = tid; i < nn; i += kB2Threads) {
            const int y = i / n, x = i - y * n;
            const double r = (double)u[i] + tau_a(Q, i, y, x, n, nn, tb1, tb2n2);
            R[i] = r;
            if (!warm) M[i] = 0.0;
            C[i] = 2.0;
            rr += r * r;
        }
        const double scale = fmax(1.0, sqrt(block_sum1(rr, red)));  // (its barrier: R, M done)
        for (int i = tid; i < nn; i += kB2Threads) {
            const int y = i / n, x = i - y * n;
            U[i] = warm ? R[i] - tau_a(M, i, y, x, n, nn, tb1, tb2n2) : R[i];
        }
        __syncthreads();
        const double diag = tb1 + 4.0 * tb2n2;  // diag(tau A)
        const double d_act = 1.0 / diag;         // Jacobi: one value on the active rows
        int start = warm ? 0 : 1, start_it = 0;  // see pdas_code
        double c_pd = diag;
        bool ok = false;
        for (;;) {
            // active sets from (u, mu); u = +-1 on them, mu = 0 off them
            double cs[2] = {0.0, 0.0};  // changed sites, |s|^2
            for (int i = tid; i < nn; i += kB2Threads) {
                const double c = pdas_code(U[i], M[i], c_pd);
                if (c != C[i]) cs[0] += 1.0;
                C[i] = c;
                if (c != 0.0)
                    U[i] = c;
                else
                    M[i] = 0.0;
            }
            __syncthreads();
            // residual of the active rows, s = r'_A - u_A - (tau A mu)_A
            for (int i = tid; i < nn; i += kB2Threads) {
                const int y = i / n, x = i - y * n;
                const double sv =
                    C[i] != 0.0 ? R[i] - U[i] - tau_a(M, i, y, x, n, nn, tb1, tb2n2) : 0.0;
                S[i] = sv;
                P[i] = sv * d_act;
                cs[1] += sv * sv;
            }
            block_sums<2>(cs, red);
            if (cs[0] == 0.0 && sqrt(cs[1]) <= 1e-13 * scale) {
                ok = true;
                break;
            }
            if (++start_it == kPdasPhase) {
                // no settled sets from this start: the next one, from mu = 0
                if (start == 2) break;
                ++start;
                start_it = 0;
                c_pd = start == 2 ? 1.0 : diag;
                for (int i = tid; i < nn; i += kB2Threads) {
                    M[i] = 0.0;
                    U[i] = R[i];
                    C[i] = 2.0;
                }
                __syncthreads();
                continue;
            }
            // CG on (tau A)_AA from the current mu (directions vanish on the
            // inactive sites)
            double rz = cs[1] * d_act;
            const double stop = pdas_cg_stop(rz, d_act, scale, cs[0] != 0.0);
            for (int k = 0; k < kMaxCg && rz > stop; ++k) {
                double pq = 0.0;
                for (int i = tid; i < nn; i += kB2Threads) {
                    const int y = i / n, x = i - y * n;
                    const double q = C[i] != 0.0 ? tau_a(P, i, y, x, n, nn, tb1, tb2n2) : 0.0;
                    Q[i] = q;
                    pq += P[i] * q;
                }
                pq = block_sum1(pq, red);
                if (!(pq > 0.0)) break;
                const double alpha = rz / pq;
                double rn = 0.0;
                for (int i = tid; i < nn; i += kB2Threads) {
                    M[i] += alpha * P[i];
                    const double sv = S[i] - alpha * Q[i];
                    S[i] = sv;
                    rn += sv * (sv * d_act);
                }
                rn = block_sum1(rn, red);
                const double beta = rn / rz;
                rz = rn;
                for (int i = tid; i < nn; i += kB2Threads) P[i] = S[i] * d_act + beta * P[i];
                __syncthreads();
            }
            __syncthreads();
            // u on the inactive sites
            for (int i = tid; i < nn; i += kB2Threads) {
                const int y = i / n, x = i - y * n;
                if (C[i] == 0.0) U[i] = R[i] - tau_a(M, i, y, x, n, nn, tb1, tb2n2);
            }
            __syncthreads();
        }
        const double nan = __builtin_nan("");
        for (int i = tid; i < nn; i += kB2Threads) uo[i] = to_store<TS>(ok ? U[i] : nan);
        return;
    }
    // r = u_old + tau A g; Newton starts from z = xi u_old, or (warm) from
    // the previous step's z, which the workspace still holds
    double rr = 0.0;
    for (int i = tid; i < nn; i += kB2Threads) {
        const int y = i / n, x = i - y * n;
        const double ui = (double)u[i];
        const double r = ui + tau_a(Q, i, y, x, n, nn, tb1, tb2n2);
        R[i] = r;
        if (!warm) Z[i] = xi * ui;  // else z of the previous step, in place
        rr += r * r;
    }
    const double scale = fmax(1.0, sqrt(block_sum1(rr, red)));
    // inverse diagonal of J (Jacobi preconditioner): active and inactive sites
    const double d_act = 1.0 / (tb1 + 4.0 * tb2n2), d_ina = 1.0 / (tb1 + 4.0 * tb2n2 + 1.0 / xi);

    bool ok = false;
    for (int it = 0;; ++it) {
        // F(z); converged when |F| <= 1e-13 max(1, |r|)
        double f2r[2] = {0.0, 0.0};  // |F|^2 and F.M^-1 F
        for (int i = tid; i < nn; i += kB2Threads) {
            const int y = i / n, x = i - y * n;
            const double f = tau_a(Z, i, y, x, n, nn, tb1, tb2n2) + clampd(Z[i] / xi) - R[i];
            const double dv = fabs(Z[i]) < xi ? d_ina : d_act;
            F[i] = f;
            X[i] = 0.0;
            S[i] = -f;
            P[i] = -f * dv;
            f2r[0] += f * f;
            f2r[1] += f * (f * dv);
        }
        block_sums<2>(f2r, red);
        const double f2 = f2r[0];
        if (sqrt(f2) <= 1e-13 * scale) {
            ok = true;
            break;
        }
        if (it == kMaxNewton) break;
        // Jacobi-preconditioned conjugate gradients on J x = -F (x0 = 0),
        // relative tolerance min(0.1, |F| / scale) in the norm s.M^-1 s of
        // the residual (inexact Newton: superlinear near the root)
        const double eta = fmin(0.1, sqrt(f2) / scale);
        const double stop = eta * eta * f2r[1];
        double rz = f2r[1];
        for (int k = 0; k < kMaxCg && rz > stop; ++k) {
            double pq = 0.0;
            for (int i = tid; i < nn; i += kB2Threads) {
                const int y = i / n, x = i - y * n;
                const double q = tau_a(P, i, y, x, n, nn, tb1, tb2n2) +
                                 (fabs(Z[i]) < xi ? P[i] / xi : 0.0);
                Q[i] = q;
                pq += P[i] * q;
            }
            pq = block_sum1(pq, red);
            if (!(pq > 0.0)) break;
            const double alpha = rz / pq;
            double rn = 0.0;  // s.M^-1 s
            for (int i = tid; i < nn; i += kB2Threads) {
                X[i] += alpha * P[i];
                const double sv = S[i] - alpha * Q[i];
                S[i] = sv;
                rn += sv * (sv * (fabs(Z[i]) < xi ? d_ina : d_act));
            }
            rn = block_sum1(rn, red);
            const double beta = rn / rz;
            rz = rn;
            for (int i = tid; i < nn; i += kB2Threads)
                P[i] = S[i] * (fabs(Z[i]) < xi ? d_ina : d_act) + beta * P[i];
            __syncthreads();
        }
        // Armijo backtracking on Phi along x, with the change written as
        // Phi(z + a x) - Phi(z) = a F.x + a^2/2 x.tau A x
        //                         + sum(phi(z + a x) - phi(z) - a x phi'(z))
        // (every term of the size of the decrease, none cancelling)
        double sm[2] = {0.0, 0.0};  // x.tau A x, F.x
        for (int i = tid; i < nn; i += kB2Threads) {
            const int y = i / n, x = i - y * n;
            sm[0] += X[i] * tau_a(X, i, y, x, n, nn, tb1, tb2n2);
            sm[1] += F[i] * X[i];
        }
        block_sums<2>(sm, red);
        double a = 1.0;
        for (int h = 0; h < kMaxHalvings; ++h) {
            double rem = 0.0;
            for (int i = tid; i < nn; i += kB2Threads) rem += phi_rem(Z[i], a * X[i], xi);
            rem = block_sum1(rem, red);
            if (a * sm[1] + 0.5 * a * a * sm[0] + rem <= 1e-4 * a * sm[1]) break;
            a *= 0.5;
        }
        for (int i = tid; i < nn; i += kB2Threads) Z[i] += a * X[i];
        __syncthreads();
    }
    const double nan = __builtin_nan("");
    for (int i = tid; i < nn; i += kB2Threads)
        uo[i] = to_store<TS>(ok ? clampd(Z[i] / xi) : nan);
}

// On-chip variant for n = 64, 88, 128: the same iteration, with the conjugate-
// gradient loop -- all but a few passes of a step -- kept on the compute
// unit.  512 threads (1024 at n = 128) own up to 16 sites each (site
// t + THREADS k); the CG residual (FP64) lives in registers, the CG
// direction (FP32; the only vector read at neighbouring sites) in LDS, the
// CG solution as an FP32 pair (high part in LDS, low part in registers), and
// the inactive-set mask in a register bitmask.  z, r, F and the Newton direction stay in the
// global workspace, touched a few times per Newton step.  The Newton level
// (F, convergence test, line search, z) is the same FP64 arithmetic as in
// k_b2_step; only the inner directions differ by rounding.
// Workgroup size: 1024 threads (16 sites each) from n = 128 on, else 512.
constexpr int b2_lds_threads(int nn) { return nn >= 128 * 128 ? 1024 : 512; }
constexpr size_t kB2LdsLimit = 159 * 1024;

// Whether the g pass's copy of u with a periodic halo of m on every side
// (elements of tu bytes; side n + 2m) fits in LDS with the weight table:
// the kernel and its launch decide alike.
__host__ __device__ constexpr bool b2_padded_fits(int n, int m, int tu) {
    return tu == 4 && (size_t)tu * (n + 2 * m) * (n + 2 * m) +
                              sizeof(double) * (size_t)(m + 1) * (m + 1) <= kB2LdsLimit;
}
constexpr int kB2LdsMaxWaves = 16;
constexpr int kB2Spt = 16;  // sites per thread

// One FP64 value moved between lanes by a DPP pattern (both halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// A value that every lane holds alike, moved to scalar registers (the
// kernel's vector registers are its limit).
__device__ __forceinline__ double uniform_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)b);
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Wave-wide FP64 sum in a fixed order, returned to every lane: pairs, quads,
// half rows and rows of 16 lanes by DPP exchanges (each step adds two
// partial sums that both partners hold, so a row ends with one value in all
// its lanes), then the four rows as (r0 + r1) + (r2 + r3).  No LDS traffic
// and no lane-address registers, unlike a shuffle tree.
__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) +
           (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Workgroup sums with one barrier: successive calls must alternate between
// two `red` areas (a thread writes area A for sum k + 2 only after the
// barrier of sum k + 1, which every thread passes after reading sum k).
template <int K, int WAVES>
__device__ __forceinline__ void block_sums_lds(double (&v)[K], double *red) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum_f64(v[k]);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) red[w * K + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int i = 0; i < WAVES; ++i) s += red[i * K + k];
        v[k] = s;
    }
}

template <int WAVES>
__device__ __forceinline__ double sum1_lds(double v, double *red) {
    double a[1] = {v};
    block_sums_lds<1, WAVES>(a, red);
    return a[0];
}

template <class TS, bool GAUSS, bool SPLIT, int NN, int THREADS = b2_lds_threads(NN * NN)>
__global__ __launch_bounds__(THREADS) void k_b2_step_lds(
    const SampleDesc *__restrict__ sd, const int32_t *__restrict__ ids,
    const ModelGeo *__restrict__ geo, const double *__restrict__ ewd,
    const TS *__restrict__ in, TS *__restrict__ out, double *__restrict__ ws,
    double *__restrict__ epart, int warm) {
    constexpr int kB2LdsThreads = THREADS, kB2LdsWaves = THREADS / 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *Pl = reinterpret_cast<float *>(smem_raw);  // CG direction, (n+2)^2
    float *Xl = Pl + (NN + 2) * (NN + 2);             // CG solution, n^2 (own sites)
    __shared__ double red2[2][kB2LdsMaxWaves * 4];
    int rsel = 0;  // the two areas of the workgroup sums, used in turn
    auto red = [&]() { rsel ^= 1; return red2[rsel]; };
    const int j = blockIdx.x;
    const SampleDesc d = sd[ids[j]];
    if ((d.xi > 0.0) == SPLIT) return;
    // the lattice size is a compile-time constant, so that the stencil's
    // LDS offsets are instruction immediates rather than registers
    constexpr int n = NN;
    constexpr int nn = NN * NN;
    const int m = geo->m;
    const TS *u = in + d.offset;
    TS *uo = out + d.offset;
    double *R = ws + (int64_t)j * 7 * nn;
    double *Z = R + nn;
    double *F = Z + nn;
    double *X = F + nn;  // Newton direction (for the line search)
    double *G = X + nn;  // g
    const double xi = d.xi;
    const double tb1 = geo->tau_b1, tb2n2 = geo->tau_b2 * (double)nn;
    const double gs = 2.0 * d.e_int * (double)nn;
    const double *e = ewd + geo->e_off;
    const int tid = threadIdx.x;

    // g and the energy partials of u_old, from copies of u_old (exact: FP64
    // for FP64 storage, else FP32) and of the weight table in LDS, which the
    // CG direction reuses afterwards.  Where it fits (FP32 copies), the copy
    // carries a periodic halo of m on every side, so that the disc rows are
    // read without wrapping and the two points at -dx and +dx, which share
    // a weight, are added before it multiplies them.
    using TU = typename std::conditional<std::is_same<TS, double>::value, double, float>::type;
    const bool padded = b2_padded_fits(n, m, (int)sizeof(TU));
    const int S = n + 2 * m;  // side of the padded copy
    TU *Ul = reinterpret_cast<TU *>(smem_raw);
    double *El = reinterpret_cast<double *>(
        smem_raw + sizeof(TU) * (padded ? (size_t)S * S : (size_t)nn));
    if (padded) {
        for (int i = tid; i < S * S; i += kB2LdsThreads) {
            const int Y = i / S, X = i - Y * S;
            Ul[i] = (TU)(double)u[wrap_once(Y - m, n) * n + wrap_once(X - m, n)];
        }
    } else {
        for (int i = tid; i < nn; i += kB2LdsThreads) Ul[i] = (TU)(double)u[i];
    }
    if (GAUSS)
        for (int i = tid; i < (m + 1) * (m + 1); i += kB2LdsThreads) El[i] = e[i];
    __syncthreads();
    double e_ul = 0.0, e_pot = 0.0;
    auto gpass = [&](auto EN) {
        constexpr bool EN_ = decltype(EN)::value;  // with the energy partials
        for (int i = tid; i < nn; i += kB2LdsThreads) {
            const int y = i / n, x = i - y * n;
            double acc = 0.0, lsum = 0.0, ui;
            if (padded) {
                const TU *c = Ul + (y + m) * S + (x + m);
                ui = (double)c[0];
                for (int dy = -m; dy <= m; ++dy) {
                    const int ady = dy < 0 ? -dy : dy;
                    const int w = geo->halfw[ady];
                    const TU *row = c + dy * S;
                    const double *er = El + ady * (m + 1);
                    const double v0 = (double)row[0];
                    const double w0 = GAUSS ? er[0] : 1.0;
                    acc += w0 * v0;
                    if (EN_) lsum += w0 * (ui - v0);
                    for (int k = 1; k <= w; ++k) {
                        const double pr = (double)row[-k] + (double)row[k];
                        const double wk = GAUSS ? er[k] : 1.0;
                        acc += wk * pr;
                        if (EN_) lsum += wk * (2.0 * ui - pr);
                    }
                }
            } else {
                ui = (double)Ul[i];
                for (int dy = -m; dy <= m; ++dy) {
                    const int ady = dy < 0 ? -dy : dy;
                    const int w = geo->halfw[ady];
                    const TU *row = Ul + wrap_once(y + dy, n) * n;
                    const double *er = El + ady * (m + 1);
                    for (int dx = -w; dx <= w; ++dx) {
                        const double v = (double)row[wrap_once(x + dx, n)];
                        const double wt = GAUSS ? er[dx < 0 ? -dx : dx] : 1.0;
                        acc += wt * v;
                        if (EN_) lsum += wt * (ui - v);
                    }
                }
            }
            G[i] = SPLIT ? gs * acc - xi * ui : gs * acc;  // g, or g - xi u_old
            if (EN_) {
                e_ul += ui * lsum;
                e_pot += 1.0 - ui * ui;
            }
        }
    };
    if (epart)
        gpass(std::true_type{});
    else
        gpass(std::false_type{});
    if (epart) {
        double v[2] = {e_ul, e_pot};
        block_sums_lds<2, kB2LdsWaves>(v, red());
        if (tid == 0) {
            epart[2 * (int64_t)j] = v[0];
            epart[2 * (int64_t)j + 1] = v[1];
        }
    }
    __syncthreads();
    double rr = 0.0;
    for (int i = tid; i < nn; i += kB2LdsThreads) {
        const int y = i / n, x = i - y * n;
        const double ui = (double)u[i];
        const double r = ui + tau_a(G, i, y, x, n, nn, tb1, tb2n2);
        R[i] = r;
        if constexpr (SPLIT) {
            if (!warm) F[i] = 0.0;  // mu; else the previous step's, in place
            X[i] = 2.0;             // active-set code (2: none yet)
        } else {
            if (!warm) Z[i] = xi * ui;  // else z of the previous step, in place
        }
        rr += r * r;
    }
    const double scale = fmax(1.0, sqrt(sum1_lds<kB2LdsWaves>(rr, red())));

    // Sites of this thread (t + THREADS k, k < SPT) and their places in the
    // LDS copy of the CG direction, which carries a one-cell periodic halo
    // ((n+2)^2, row W): the 5-point stencil then needs no wrap-around, and a
    // boundary site writes its value to the halo cell opposite as well.
    // Where THREADS is a multiple of n and divides n^2 (n = 64, 128), a
    // thread's sites share one column and step THREADS/n rows, so their LDS
    // places are one base plus compile-time offsets (no address registers).
    constexpr int W = n + 2;
    constexpr int SPT = (nn + kB2LdsThreads - 1) / kB2LdsThreads;
    static_assert(SPT <= kB2Spt, "sites per thread");
    constexpr bool EXACT = nn % kB2LdsThreads == 0 && kB2LdsThreads % n == 0;
    constexpr int RSTEP = kB2LdsThreads / n;  // rows between a thread's sites (EXACT)
    auto pad = [](int i) { return i + 2 * (i / n) + n + 3; };  // (y+1) W + x + 1
    const int q0 = pad(tid), y0 = tid / n, x0 = tid - (tid / n) * n;
    auto site = [&](int k) { return tid + kB2LdsThreads * k; };
    auto valid = [&](int k) { return EXACT || site(k) < nn; };
    auto qk = [&](int k) { return EXACT ? q0 + k * RSTEP * W : pad(site(k)); };
    auto put = [&](int k, double vd) {
        const int q = qk(k);
        const int y = EXACT ? y0 + k * RSTEP : site(k) / n;
        const int x = EXACT ? x0 : site(k) - (site(k) / n) * n;
        const float v = (float)vd;
        Pl[q] = v;
        if (x == 0) Pl[q + n] = v;
        if (x == n - 1) Pl[q - n] = v;
        if (y == 0) Pl[q + n * W] = v;
        if (y == n - 1) Pl[q - n * W] = v;
    };

    // inverse diagonal of the CG operator (Jacobi preconditioner): active
    // and inactive sites (the split step's inactive rows are removed)
    const double d_act = uniform_f64(1.0 / (tb1 + 4.0 * tb2n2)),
                 d_ina = SPLIT ? 0.0 : uniform_f64(1.0 / (tb1 + 4.0 * tb2n2 + 1.0 / xi));
    const double inv_xi = SPLIT ? 0.0 : uniform_f64(1.0 / xi);
    // Conjugate gradients from the solution 0 (Xl + Xlo, zeroed by the
    // caller) with residual Sr and first direction M^-1 Sr already in Pl, on
    // tau A + diag(1/xi on the inactive sites) (Newton), or on tau A with the
    // rows and columns of the inactive sites removed (SPLIT: the residual and
    // the direction vanish there and stay zero).
    auto cg = [&](unsigned mask, double(&Sr)[SPT], float(&Xlo)[SPT], double rz, double stop) {
        for (int kk = 0; kk < kMaxCg && rz > stop; ++kk) {
            // the per-site selections of the preconditioner are made in
            // every iteration: an empty asm statement hides the two values
            // from the optimiser, which would otherwise hoist 16 selected
            // FP64 values (32 registers) out of the loop and spill them
            double da = d_act, di = d_ina;
            __asm__ volatile("" : "+v"(da), "+v"(di));
            auto dinv = [&](int k) { return (mask >> k) & 1u ? di : da; };
            // J p at site k from the direction's five LDS values (evaluated
            // twice per iteration, for p.Jp and for the residual update,
            // instead of being kept in registers).  Where the sites sit at
            // fixed offsets (n = 64, 128), each site's values are loaded
            // while the previous site is computed (elsewhere that costs
            // spills); the scheduling barriers keep the sites in that order.
            struct Nb {
                float c, e, w, n, s;
            };
            auto ld = [&](int k) {
                Nb v{0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                if (valid(k)) {
                    const int q = qk(k);
                    v = Nb{Pl[q], Pl[q + 1], Pl[q - 1], Pl[q + W], Pl[q - W]};
                }
                return v;
            };
            auto jp = [&](int k, const Nb &v) {
                const double pi = v.c;
                const double ap = tb1 * pi - tb2n2 * ((double)v.e + (double)v.w + (double)v.n +
                                                      (double)v.s - 4.0 * pi);
                if constexpr (SPLIT) return (mask >> k) & 1u ? 0.0 : ap;
                return ap + ((mask >> k) & 1u ? pi * inv_xi : 0.0);
            };
            double pq = 0.0;
            {
                Nb nxt = EXACT ? ld(0) : Nb{};
#pragma unroll
                for (int k = 0; k < SPT; ++k) {
                    const Nb cur = EXACT ? nxt : ld(k);
                    if (EXACT && k + 1 < SPT) nxt = ld(k + 1);
                    if (valid(k)) pq += (double)cur.c * jp(k, cur);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            pq = sum1_lds<kB2LdsWaves>(pq, red());
            if (!(pq > 0.0)) break;
            const double alpha = uniform_f64(rz / pq);
            double rn = 0.0;  // s.M^-1 s
            {
                Nb nxt = EXACT ? ld(0) : Nb{};
                float xnxt = EXACT ? Xl[site(0)] : 0.0f;
#pragma unroll
                for (int k = 0; k < SPT; ++k) {
                    const Nb cur = EXACT ? nxt : ld(k);
                    const float xc = EXACT ? xnxt : (valid(k) ? Xl[site(k)] : 0.0f);
                    if (EXACT && k + 1 < SPT) {
                        nxt = ld(k + 1);
                        xnxt = Xl[site(k + 1)];
                    }
                    if (valid(k)) {
                        const double t = ((double)xc + (double)Xlo[k]) + alpha * (double)cur.c;
                        const float hi = (float)t;
                        Xl[site(k)] = hi;
                        Xlo[k] = (float)(t - (double)hi);
                        Sr[k] -= alpha * jp(k, cur);
                        rn += Sr[k] * (Sr[k] * dinv(k));
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            rn = sum1_lds<kB2LdsWaves>(rn, red());  // every thread has read Pl before it changes
            const double beta = uniform_f64(rn / rz);
            rz = rn;
#pragma unroll
            for (int k = 0; k < SPT; ++k) {
                if (valid(k)) put(k, Sr[k] * dinv(k) + beta * (double)Pl[qk(k)]);
                __builtin_amdgcn_sched_barrier(0);
            }
            __syncthreads();
        }
    };

    bool ok = false;
    if constexpr (SPLIT) {
        // u (U), mu (M; kept between the steps of a call) and the active-set
        // code of the last iteration (C) in the workspace; each CG solve
        // accumulates the change of mu in Xl + Xlo
        double *U = Z, *M = F, *C = X;
        const double diag = uniform_f64(tb1 + 4.0 * tb2n2);  // diag(tau A)
        int start = warm ? 0 : 1, start_it = 0;  // see pdas_code
        double c_pd = diag;
        for (int i = tid; i < nn; i += kB2LdsThreads) {
            const int y = i / n, x = i - y * n;
            U[i] = warm ? R[i] - tau_a(M, i, y, x, n, nn, tb1, tb2n2) : R[i];
        }
        __syncthreads();
        for (;;) {
            // active sets from (u, mu); u = +-1 on them, mu = 0 off them
            double cs[2] = {0.0, 0.0};  // changed sites, |s|^2
            unsigned mask = 0;          // bit k: site t + THREADS k inactive
#pragma unroll 1
            for (int k = 0; k < SPT; ++k) {
                const int i = site(k);
                if (valid(k)) {
                    const double c = pdas_code(U[i], M[i], c_pd);
                    if (c != C[i]) cs[0] += 1.0;
                    C[i] = c;
                    if (c != 0.0) {
                        U[i] = c;
                    } else {
                        M[i] = 0.0;
                        mask |= 1u << k;
                    }
                }
            }
            __syncthreads();
            // residual of the active rows, s = r'_A - u_A - (tau A mu)_A, in
            // FP64 from mu (to G, whose g is no longer needed); the CG start
#pragma unroll 1
            for (int k = 0; k < SPT; ++k) {
                const int i = site(k);
                if (valid(k)) {
                    const int y = i / n, x = i - y * n;
                    const double sv = (mask >> k) & 1u
                                          ? 0.0
                                          : R[i] - U[i] - tau_a(M, i, y, x, n, nn, tb1, tb2n2);
                    G[i] = sv;
                    put(k, sv * d_act);
                    cs[1] += sv * sv;
                }
            }
            double Sr[SPT];
            float Xlo[SPT];
#pragma unroll
            for (int k = 0; k < SPT; ++k) {
                Sr[k] = valid(k) ? G[site(k)] : 0.0;
                if (valid(k)) Xl[site(k)] = 0.0f;
                Xlo[k] = 0.0f;
            }
            block_sums_lds<2, kB2LdsWaves>(cs, red());  // also makes Pl visible
            if (cs[0] == 0.0 && sqrt(cs[1]) <= 1e-13 * scale) {
                ok = true;
                break;
            }
            if (++start_it == kPdasPhase) {
                // no settled sets from this start: the next one, from mu = 0
                if (start == 2) break;
                ++start;
                start_it = 0;
                c_pd = start == 2 ? 1.0 : diag;
                for (int i = tid; i < nn; i += kB2LdsThreads) {
                    M[i] = 0.0;
                    U[i] = R[i];
                    C[i] = 2.0;
                }
                __syncthreads();
                continue;
            }
            const double rz = cs[1] * d_act;
            cg(mask, Sr, Xlo, rz, pdas_cg_stop(rz, d_act, scale, cs[0] != 0.0));
#pragma unroll
            for (int k = 0; k < SPT; ++k)
                if (valid(k)) M[site(k)] += (double)Xl[site(k)] + (double)Xlo[k];
            __syncthreads();
            // u on the inactive sites
            for (int i = tid; i < nn; i += kB2LdsThreads) {
                const int y = i / n, x = i - y * n;
                if (C[i] == 0.0) U[i] = R[i] - tau_a(M, i, y, x, n, nn, tb1, tb2n2);
            }
            __syncthreads();
        }
        const double nan = __builtin_nan("");
        for (int i = tid; i < nn; i += kB2LdsThreads) uo[i] = to_store<TS>(ok ? U[i] : nan);
        return;
    }
    for (int it = 0;; ++it) {
        // F(z), the CG start (direction -M^-1 F, to LDS) and the inactive-set mask
        double f2r[2] = {0.0, 0.0};  // |F|^2 and F.M^-1 F
        unsigned mask = 0;  // bit k: site t + THREADS k inactive (|z| < xi)
#pragma unroll 1
        for (int k = 0; k < SPT; ++k) {
            const int i = site(k);
            if (valid(k)) {
                const int y = i / n, x = i - y * n;
                const double zi = Z[i];
                const double f = tau_a(Z, i, y, x, n, nn, tb1, tb2n2) + clampd(zi / xi) - R[i];
                const bool ina = fabs(zi) < xi;
                const double dv = ina ? d_ina : d_act;
                F[i] = f;
                put(k, -f * dv);
                if (ina) mask |= 1u << k;
                f2r[0] += f * f;
                f2r[1] += f * (f * dv);
            }
        }
        block_sums_lds<2, kB2LdsWaves>(f2r, red());  // also makes Pl visible
        const double f2 = f2r[0];
        if (sqrt(f2) <= 1e-13 * scale) {
            ok = true;
            break;
        }
        if (it == kMaxNewton) break;
        // The CG residual in FP64 (registers); the solution as an FP32 pair
        // (a plain FP32 solution limits how much each inexact Newton step
        // gains, which costs extra Newton steps).  The CG direction is kept
        // in FP32: the solution and the residual are updated with the same
        // rounded direction and its FP64 operator product, so they stay
        // consistent and the residual reaches FP64 tolerances; the rounding
        // only perturbs the conjugacy of the directions.
        double Sr[SPT];
        float Xlo[SPT];  // the solution is Xl + Xlo (an FP32 pair, ~48 bits)
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            Sr[k] = valid(k) ? -F[site(k)] : 0.0;
            if (valid(k)) Xl[site(k)] = 0.0f;  // a thread's own sites only
            Xlo[k] = 0.0f;
        }
        const double eta = fmin(0.1, sqrt(f2) / scale);
        const double stop = eta * eta * f2r[1];
        double rz = f2r[1];
        cg(mask, Sr, Xlo, rz, stop);
#pragma unroll
        for (int k = 0; k < SPT; ++k)
            if (valid(k)) X[site(k)] = (double)Xl[site(k)] + (double)Xlo[k];
        __syncthreads();
        // Armijo backtracking as in k_b2_step
        double sm[2] = {0.0, 0.0};  // x.tau A x, F.x
        for (int i = tid; i < nn; i += kB2LdsThreads) {
            const int y = i / n, x = i - y * n;
            sm[0] += X[i] * tau_a(X, i, y, x, n, nn, tb1, tb2n2);
            sm[1] += F[i] * X[i];
        }
        block_sums_lds<2, kB2LdsWaves>(sm, red());
        double a = 1.0;
        for (int h = 0; h < kMaxHalvings; ++h) {
            double rem = 0.0;
            for (int i = tid; i < nn; i += kB2LdsThreads) rem += phi_rem(Z[i], a * X[i], xi);
            rem = sum1_lds<kB2LdsWaves>(rem, red());
            if (a * sm[1] + 0.5 * a * a * sm[0] + rem <= 1e-4 * a * sm[1]) break;
            a *= 0.5;
        }
        for (int i = tid; i < nn; i += kB2LdsThreads) Z[i] += a * X[i];
        __syncthreads();
    }
    const double nan = __builtin_nan("");
    for (int i = tid; i < nn; i += kB2LdsThreads)
        uo[i] = to_store<TS>(ok ? clampd(Z[i] / xi) : nan);
}

template <class TS, bool SPLIT>
hipError_t b2_typed(const Group &g, const void *in, void *out, hipStream_t s, double *epart,
                    bool warm) {
    // on-chip variant for the lattices of the multifidelity study
    auto lds_launch = [&](auto f, int n) {
        // the CG direction and solution (FP32), or, before them, u_old (with
        // its halo where that fits) and the weight table
        const int tu = std::is_same<TS, double>::value ? 8 : 4;
        const size_t side = b2_padded_fits(n, g.m, tu) ? (size_t)(n + 2 * g.m) : (size_t)n;
        const size_t lds = std::max(
            sizeof(float) * ((size_t)(n + 2) * (n + 2) + (size_t)n * n),
            tu * side * side + sizeof(double) * (size_t)(g.m + 1) * (g.m + 1));
        if (lds > kB2LdsLimit) return hipErrorInvalidValue;
        if (lds > 64 * 1024 &&
            hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kB2LdsLimit) != hipSuccess)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(f, dim3((unsigned)g.nids), dim3(b2_lds_threads(n * n)), lds, s,
                           g.sd, g.ids, g.geo, g.ewd, (const TS *)in, (TS *)out, g.ws, epart,
                           (int)warm);
        return hipGetLastError();
    };
    const bool gauss = g.kernel == 1;
    switch (g.n) {
        case 64:
            return gauss ? lds_launch(k_b2_step_lds<TS, true, SPLIT, 64>, 64)
                         : lds_launch(k_b2_step_lds<TS, false, SPLIT, 64>, 64);
        case 88:
            return gauss ? lds_launch(k_b2_step_lds<TS, true, SPLIT, 88>, 88)
                         : lds_launch(k_b2_step_lds<TS, false, SPLIT, 88>, 88);
        case 128:
            return gauss ? lds_launch(k_b2_step_lds<TS, true, SPLIT, 128>, 128)
                         : lds_launch(k_b2_step_lds<TS, false, SPLIT, 128>, 128);
        default:
            break;
    }
    dim3 grid((unsigned)g.nids), block(kB2Threads);
    if (g.kernel == 1)
        hipLaunchKernelGGL((k_b2_step<TS, true, SPLIT>), grid, block, 0, s, g.sd, g.ids, g.geo,
                           g.ewd, (const TS *)in, (TS *)out, g.ws, epart, (int)warm);
    else
        hipLaunchKernelGGL((k_b2_step<TS, false, SPLIT>), grid, block, 0, s, g.sd, g.ids, g.geo,
                           g.ewd, (const TS *)in, (TS *)out, g.ws, epart, (int)warm);
    return hipGetLastError();
}

// The Newton kernel for the group's samples with xi > 0, then the split-step
// kernel for those with xi <= 0 (each launched only if it has samples).
template <class TS>
hipError_t b2_both(const Group &g, const void *in, void *out, hipStream_t s, double *epart,
                   bool warm) {
    if (g.b2_newton > 0) {
        const hipError_t e = b2_typed<TS, false>(g, in, out, s, epart, warm);
        if (e != hipSuccess) return e;
    }
    if (g.b2_split > 0) return b2_typed<TS, true>(g, in, out, s, epart, warm);
    return hipSuccess;
}

}  // namespace

hipError_t launch_b2_step(int prec, const Group &g, const void *in, void *out, hipStream_t s,
                          double *epart, bool warm) {
    if (!g.ws || g.n > kB2MaxN || g.lo != 0) return hipErrorInvalidValue;
    switch (prec) {
        case kF64: return b2_both<double>(g, in, out, s, epart, warm);
        case kF32: return b2_both<float>(g, in, out, s, epart, warm);
        default: return b2_both<half_t>(g, in, out, s, epart, warm);
    }
}

}  // namespace nlch
