// Host-side helpers shared by the translation units behind the C ABI:
// argument validation, disc tables, per-sample coefficients, kernel choice
// and the device-table images of a model and a sample.  Not part of the
// public ABI.
#pragma once

#include <stdint.h>

#include <vector>

#include "nlch.h"
#include "nlch_internal.h"

namespace nlch {

// Records the calling thread's error message (see nlch_last_error) and
// returns code.
int fail(int code, const char *fmt, ...);

// Failure injection (nlch_debug_inject_device_error): true for the one
// checked HIP call that is to report failure instead of being made.
bool inject_device_error();

// A checked HIP runtime call: its failure (or an injected one, in which case
// the call is not made) returns NLCH_EDEVICE from the enclosing function.  The
// error is reported through the library's code and message, and cleared from
// HIP's per-thread last error, so that it does not resurface at the caller's
// next, unrelated HIP call.
#define HIP_TRY(expr)                                                             \
    do {                                                                          \
        if (::nlch::inject_device_error())                                        \
            return ::nlch::fail(NLCH_EDEVICE, "%s: injected device error", #expr); \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) {                                                   \
            (void)hipGetLastError();                                              \
            return ::nlch::fail(NLCH_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
        }                                                                         \
    } while (0)

// A validated model's disc and kernel tables.
struct ModelInfo {
    int64_t R2 = 0, N = 0;
    int m = 0;
    int lo = 0;                  // ring width: m under a volume constraint, else 0
    int side = 0;                // side of a stored state, n + 2 lo
    std::vector<int32_t> halfw;  // |dy| = 0..m
    double sum_e = 0.0;          // sum_{d in D} e_d, e_d exact 2-D unit weights
    double ce_sep = 0.0;         // sum_{d in D} g(|dy|) g(|dx|)
    std::vector<double> g;       // g(k), k = 0..m
    std::vector<double> e2;      // e(|dy|, |dx|), (m+1) x (m+1)
};

// Discrete constants of one sample (its own c_F and kernel amplitude).
struct Coef {
    double c_gamma_h, xi_h, c1, a, b;
};

bool finite_pos(double v);

// Validates a model and builds its tables (host only, no device work).
int analyze_model(const nlch_model &md, ModelInfo &mi, const char *what);

// c_gamma_h, xi_h and the update coefficients of a sample; NLCH_EINVAL when
// 1 + tau beta1 xi_h <= 0.
int sample_coef(const nlch_model &md, const ModelInfo &mi, double c_F, double amp, Coef &c,
                const char *what);

// NLCH_EINVAL for unknown flags or algorithm.
int check_algo_flags(int32_t algo);

// Kernel variant of a model under the requested algorithm (batch: a whole
// solve, where the LDS-resident kernel applies).
int choose_variant(int base, int prec, bool acc64, const ModelInfo &mi, const nlch_model &md,
                   bool batch, int *variant);

// Device-table images: the model's geometry (weights of the direct kernel at
// element e_off of the weight tables) and a sample's descriptor.
void fill_model_geo(const nlch_model &md, const ModelInfo &mi, int64_t e_off, ModelGeo &gm);
void fill_sample_desc(const nlch_model &md, const ModelInfo &mi, const nlch_sample &sm,
                      const Coef &c, SampleDesc &d);

// A launch group of n_ids samples of one model (device pointers unset).
Group make_group(const nlch_model &md, const ModelInfo &mi, int model_index, int n_ids, int prec);

size_t prec_size(int prec);

// The default launch shape of a row-run group (the tiled kernel for one or
// a few samples where it is built, else one wave per band).
void set_default_shape(Group &g);

}  // namespace nlch
