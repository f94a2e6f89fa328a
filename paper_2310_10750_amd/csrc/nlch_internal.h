// Internal declarations shared by the host runtime (nlch_api.cpp) and the
// kernel translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nlch {

// Largest horizon in lattice units the kernels accept (m = floor(sqrt(R2))).
constexpr int kMaxM = 48;

enum Prec { kF64 = 0, kF32 = 1, kF16 = 2 };

// Per-model geometry and kernel factors, resident in device memory.
//   halfw[|dy|] = floor(sqrt(R2 - dy^2))      (row half-widths of the disc)
//   gf/gd[k]    = exp(-k^2 h^2 / sigma^2)      (Gaussian), 1 (constant kernel)
//   ce          = sum_{d in D} g(|dy|) g(|dx|) (unit-amplitude mass, separable)
// The exact 2-D unit weights e(|dy|,|dx|) = exp(-h^2 |d|^2 / sigma^2) used by
// the direct kernel live in a separate table at offset e_off, row-major
// (m+1) x (m+1).
// n is the side of a sample's stored array.  The kernels update the block of
// rows and columns [lo, n - lo): the whole periodic lattice (lo = 0), or,
// under a volume constraint, the lattice of Omega inside a ring of lo = m
// rows and columns of fixed values on the interaction region.
struct ModelGeo {
    int32_t n, m, R2, N;
    int32_t kernel, lo;
    int64_t e_off;
    double ced;
    double tau_b1, tau_b2;  // tau beta1, tau beta2 (the beta2 > 0 step)
    float cef, pad1;
    float gf[kMaxM + 1];
    double gd[kMaxM + 1];
    int32_t halfw[kMaxM + 1];
};

// Per-sample update coefficients: with Lsum the unit-amplitude operator sum
// sum_{d != 0} e_d (u - u_{+d}),  v = u + (a u - b Lsum),  u' = clamp(v).
//   a = c1 c_F,  b = c1 h^2 amp,  c1 = tau beta1 / (1 + tau beta1 xi_h).
// Energy factors: E_h(u) = e_int sum_i u_i Lsum_i + e_pot sum_i (1 - u_i^2)
//   with e_int = h^4 amp / 2 and e_pot = h^2 c_F / 2.
// xi = xi_h = c_gamma_h - c_F of the sample (used by the beta2 > 0 step).
// ap = a - b ce = c1 (c_F - h^2 amp ce): the update as u + (ap u + b G) from
// the unit-amplitude disc sum G = ce u - Lsum.
struct SampleDesc {
    int64_t offset;   // element offset of the sample's n x n state
    int32_t model;
    int32_t n;
    double a, b;
    float af, bf;
    double e_int, e_pot;
    double xi;
    double ap;
    float apf, pad;
};

// One launch group: samples of one model, processed by one kernel variant.
struct Group {
    const ModelGeo *geo;    // device pointer to this model's geometry
    const float *ewf;       // device pointer to the 2-D unit weight tables
    const double *ewd;      //   (FP32 and FP64 copies, indexed from e_off)
    const SampleDesc *sd;   // device pointer to all sample descriptors
    const int32_t *ids;     // device pointer to this group's sample indices
    double *partial;        // device scratch: ooi_chunks(n) doubles per sample
    double *ws;             // beta2 > 0 groups: b2_ws_doubles(n) doubles per sample
    int32_t nids;
    int32_t n, m, R2;        // n: side of the stored array (as ModelGeo::n)
    int32_t lo, ni;          // updated block [lo, lo + ni)^2, ni = n - 2 lo
    int32_t kernel;
    int32_t model;
    int32_t tune_R, tune_B;  // streaming shape (0 = heuristic): columns per
    int32_t tune_W, tune_L;  //   lane, band rows, waves per band, rows per wave
    int32_t ta_bytes;        // size of the arithmetic type (4 or 8)
    int32_t res_cols;        // resident kernel: columns per lane and rows each
    int32_t res_rows;        //   lane walks (0 = default)
    int32_t tile;            // row-run steps on 32 x 32 output tiles (k_tile)
    int32_t tune_PH;         // 2: rows walked in two interleaved phases (k_phase)
    int32_t b2_newton;       // beta2 > 0 groups: samples with xi_h > 0 (Newton step)
    int32_t b2_split;        //   and with xi_h <= 0 (split step)
};

// Heuristic streaming shape of the row-run kernel: lanes own R columns of a
// 64R-column strip; a wave's band height B trades parallelism (about 12
// waves per CU) against the 2m-row window overhead of each band, and is at
// least max(16, 2m) rows.
inline int stream_band_rows(int n, int M, int TX, int nids) {
    const int strips = (n + TX - 1) / TX;
    const int64_t target_waves = 3072;
    const int64_t have = (int64_t)strips * nids;
    int64_t bands = (target_waves + have - 1) / have;
    if (bands < 1) bands = 1;
    int B = (int)((n + bands - 1) / bands);
    const int bmin = M * 2 > 16 ? M * 2 : 16;
    if (B < bmin) B = bmin;
    if (B > n) B = n;
    return B;
}

inline int stream_lanes_cols(int n, int M, int nids) {
    if (M >= 24) return 1;  // wide discs: keep the register ring small
    // waves available with R = 2 at the minimum band height
    const int bmin = M * 2 > 16 ? M * 2 : 16;
    const int64_t waves2 = (int64_t)((n + 127) / 128) * ((n + bmin - 1) / bmin) * nids;
    return waves2 < 2048 ? 1 : 2;
}

// Launch shape of the streaming kernel: R columns per lane, W waves per
// workgroup, band of B output rows; with W > 1 every wave but the last walks
// L rows (a multiple of the ring period 2m+1) and B = W L - 2m.  PH = 2
// (W = 1, FP32 arithmetic): the two half-waves walk alternate rows of the
// band over a strip of 32R columns (k_phase).
struct StreamShape {
    int R, W, L, B, per_sample, PH;
};

// LDS bytes of the streaming kernel: per wave a two-row staging ring of
// 64 ceil((64R + 2m)/64) elements, and for W > 1 2m x 64R partial sums.
inline size_t stream_lds_bytes(int R, int M, int W, int ta_bytes) {
    const size_t ring = 2 * 64 * (size_t)((64 * R + 2 * M + 63) / 64);
    const size_t head = W > 1 ? (size_t)2 * M * 64 * R : 0;
    return (size_t)W * (ring + head) * ta_bytes;
}

// Shared-band kernels are built for FP32 arithmetic and horizons m <= 32 (the
// 2m rows of partial sums per wave: 4 waves of one column per lane take
// 70 KB of LDS at m = 32).
constexpr bool band_built(int M, int ta_bytes) { return ta_bytes == 4 && M <= 32; }

// Tiled one-step kernel (k_tile, FP32 arithmetic, m <= 16): built for a disc,
// workgroups one sample takes, launch (one step of every sample).
bool tile_supported(int prec, bool acc64, int R2);
int tile_blocks_per_sample(int ni);
hipError_t launch_tile_step(int prec, const Group &g, const void *in, void *out,
                            hipStream_t s);

inline StreamShape stream_shape(const Group &g) {
    StreamShape sh;
    sh.R = (g.tune_R == 1 || g.tune_R == 2) ? g.tune_R : stream_lanes_cols(g.ni, g.m, g.nids);
    sh.W = g.tune_W > 1 && band_built(g.m, g.ta_bytes) ? g.tune_W : 1;
    sh.PH = sh.W == 1 && g.tune_PH == 2 && g.ta_bytes == 4 ? 2 : 1;
    // fewer waves per band where the partial-sum areas would not fit in LDS
    while (sh.W > 1 && stream_lds_bytes(sh.R, g.m, sh.W, g.ta_bytes) > 159 * 1024) sh.W /= 2;
    if (sh.W > 1) {
        sh.L = g.tune_L;
        sh.B = sh.W * sh.L - 2 * g.m;
    } else {
        sh.L = 2 * g.m + 1;
        sh.B = g.tune_B > 0 ? g.tune_B
                            : stream_band_rows(g.ni, g.m, 64 * sh.R / sh.PH, g.nids);
    }
    if (sh.B > g.ni) sh.B = g.ni;
    const int tx = 64 * sh.R / sh.PH;  // strip columns
    sh.per_sample = ((g.ni + tx - 1) / tx) * ((g.ni + sh.B - 1) / sh.B);
    return sh;
}

// Tile of the direct kernel and the workgroups one sample occupies.
constexpr int kDirTX = 64, kDirTY = 16;
inline int direct_tiles(int n) { return ((n + kDirTX - 1) / kDirTX) * ((n + kDirTY - 1) / kDirTY); }

// Kernel variants.
enum Variant { kDirect = 1, kRowrun = 2, kResident = 3, kB2 = 4 };

// The beta2 > 0 step: largest lattice, per-sample FP64 workspace (seven
// n x n vectors: right-hand side, z, F, Newton direction, CG residual, CG
// direction, operator product).
constexpr int kB2MaxN = 256;
inline int64_t b2_ws_doubles(int n) { return 7 * (int64_t)n * n; }

// Launch wrappers (return the launch status).  `acc64` selects FP64
// accumulation for the F32/F16 storage types (always on for F64).
hipError_t launch_project(int prec, const Group &g, const void *src, void *dst,
                          hipStream_t s);
hipError_t launch_count_nonfinite(int prec, const Group &g, const void *src,
                                  unsigned int *counter, hipStream_t s);
int ooi_chunks(int n);
hipError_t launch_ooi(int prec, const Group &g, const void *state, double *ooi,
                      int per_sample_slots, hipStream_t s);
// Step launches take an optional `epart` (two FP64 energy partial sums per
// workgroup, workgroups of one sample consecutive); nullptr skips the energy.
hipError_t launch_direct_step(int prec, bool acc64, const Group &g,
                              const void *in, void *out, hipStream_t s,
                              double *epart = nullptr);
bool rowrun_supported(int prec, bool acc64, int R2, int kernel);
hipError_t launch_rowrun_step(int prec, bool acc64, const Group &g,
                              const void *in, void *out, hipStream_t s,
                              double *epart = nullptr);
bool resident_supported(int prec, bool acc64, int R2, int kernel, int n, bool vol);
// `energy` (nullable): E_h(u^k) of sample s at energy[k * estride + s].
hipError_t launch_resident(int prec, bool acc64, const Group &g, void *state,
                           int nsteps, double *ooi, hipStream_t s,
                           double *energy = nullptr, int64_t estride = 0);
// The resident kernels with four columns per lane (FP32 state, n = 128,
// periodic): built for these discs.  energy (nullable) as in launch_resident.
bool resident4_built(int R2);
hipError_t resident4_launch_f32(const Group &g, void *state, int nsteps, double *ooi,
                                hipStream_t s, double *energy, int64_t estride);
// One beta2 > 0 step of every sample of the group (one workgroup per sample,
// workspace g.ws); epart (nullable) receives one energy partial pair per
// sample.  warm: start Newton from the z the workspace holds (the previous
// step's, within one solve) instead of xi_h u_old.
hipError_t launch_b2_step(int prec, const Group &g, const void *in, void *out, hipStream_t s,
                          double *epart, bool warm = false);
// Per sample of the group, the workgroup partials in order -> energy[ids[j]].
hipError_t launch_energy_final(const Group &g, const double *epart, int per_sample,
                               double *energy, hipStream_t s);
hipError_t launch_moments(int K, const double *const *y, const int64_t *m,
                          int64_t stride, double *out, hipStream_t s);

// Records the calling thread's error message (see nlch_last_error) and
// returns code.
int set_error(int code, const char *msg);

// List of R2 values with compiled row-run kernels for a precision.
int rowrun_r2_list(int prec, int64_t *out, int cap);

}  // namespace nlch
