// Host runtime behind the C ABI of include/nlch.h: argument validation, disc
// geometry and kernel tables, per-sample coefficients, launch grouping, and
// HIP-graph capture/replay of whole solves.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "nlch.h"
#include "nlch_host.h"
#include "nlch_internal.h"

namespace nlch {
// per-type-pair units (kern_rowrun_*.hip)
#define NLCH_DECL(SUF)                                                                   \
    int rowrun_r2_##SUF(int64_t *out, int cap);                                          \
    bool rowrun_has_##SUF(int R2);                                                       \
    bool resident_has_##SUF(int R2, int n, bool vol);                                    \
    hipError_t rowrun_step_##SUF(const Group &g, const void *in, void *out, hipStream_t s, \
                                 double *epart);                                         \
    hipError_t resident_##SUF(const Group &g, void *state, int nsteps, double *ooi,      \
                              hipStream_t s, double *energy, int64_t estride);
NLCH_DECL(f64)
NLCH_DECL(f32)
NLCH_DECL(f16)
#undef NLCH_DECL

// Row-run and resident kernels exist for FP64 arithmetic on FP64 state and
// FP32 arithmetic on FP32/FP16 state; FP64 accumulation of narrower states
// (NLCH_ALGO_ACC64) runs on the direct kernel.
bool rowrun_supported(int prec, bool acc64, int R2, int) {
    switch (prec) {
        case kF64: return rowrun_has_f64(R2);
        case kF32: return !acc64 && rowrun_has_f32(R2);
        default: return !acc64 && rowrun_has_f16(R2);
    }
}

bool resident_supported(int prec, bool acc64, int R2, int, int n, bool vol) {
    switch (prec) {
        case kF64: return resident_has_f64(R2, n, vol);
        case kF32: return !acc64 && resident_has_f32(R2, n, vol);
        default: return !acc64 && resident_has_f16(R2, n, vol);
    }
}

hipError_t launch_rowrun_step(int prec, bool acc64, const Group &g, const void *in, void *out,
                              hipStream_t s, double *epart) {
    // the tiled kernel has no energy partials: the trace keeps the streaming
    // kernel, whose states are the same bit for bit
    if (g.tile && !epart && tile_supported(prec, acc64, g.R2))
        return launch_tile_step(prec, g, in, out, s);
    switch (prec) {
        case kF64: return rowrun_step_f64(g, in, out, s, epart);
        case kF32: return rowrun_step_f32(g, in, out, s, epart);
        default: return rowrun_step_f16(g, in, out, s, epart);
    }
}

hipError_t launch_resident(int prec, bool, const Group &g, void *state, int nsteps,
                           double *ooi, hipStream_t s, double *energy, int64_t estride) {
    switch (prec) {
        case kF64: return resident_f64(g, state, nsteps, ooi, s, energy, estride);
        case kF32: return resident_f32(g, state, nsteps, ooi, s, energy, estride);
        default: return resident_f16(g, state, nsteps, ooi, s, energy, estride);
    }
}

int rowrun_r2_list(int prec, int64_t *out, int cap) {
    switch (prec) {
        case kF64: return rowrun_r2_f64(out, cap);
        case kF32: return rowrun_r2_f32(out, cap);
        default: return rowrun_r2_f16(out, cap);
    }
}

}  // namespace nlch

using namespace nlch;

// ------------------------------------------------------------------ errors --

static thread_local std::string g_last_error;

int nlch::fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int nlch::set_error(int code, const char *msg) { return fail(code, "%s", msg); }

// Checked HIP calls still to be made before the injected failure (0: none
// armed).  The armed call reports failure without being made, so nothing
// invalid reaches the device.
static std::atomic<int64_t> g_inject{0};

bool nlch::inject_device_error() {
    if (g_inject.load(std::memory_order_relaxed) <= 0) return false;
    return g_inject.fetch_sub(1) == 1;
}

// Scope of a named roctx range (visible to rocprofv3 --marker-trace).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
};

// ---------------------------------------------------------------- geometry --

static int64_t isqrt64(int64_t v) {
    if (v <= 0) return 0;
    int64_t r = (int64_t)std::sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}


bool nlch::finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Validates a model and builds its tables (host only, no device work).
int nlch::analyze_model(const nlch_model &md, ModelInfo &mi, const char *what) {
    if (md.n < 3 || md.n > 32768)
        return fail(NLCH_EINVAL, "%s: n = %d outside [3, 32768]", what, md.n);
    if (md.kernel != NLCH_KERNEL_CONSTANT && md.kernel != NLCH_KERNEL_GAUSSIAN)
        return fail(NLCH_EINVAL, "%s: unknown kernel %d", what, md.kernel);
    if (!std::isfinite(md.delta) || md.delta < 0.0 || md.delta * md.n > 1e6)
        return fail(NLCH_EINVAL, "%s: delta must be finite and >= 0", what);
    if (!finite_pos(md.kernel_amp)) return fail(NLCH_EINVAL, "%s: kernel_amp must be > 0", what);
    if (md.kernel == NLCH_KERNEL_GAUSSIAN && !finite_pos(md.kernel_sigma))
        return fail(NLCH_EINVAL, "%s: kernel_sigma must be > 0", what);
    if (!finite_pos(md.c_F)) return fail(NLCH_EINVAL, "%s: c_F must be > 0", what);
    if (!finite_pos(md.beta1)) return fail(NLCH_EINVAL, "%s: beta1 must be > 0", what);
    if (!std::isfinite(md.beta2) || md.beta2 < 0.0)
        return fail(NLCH_EINVAL, "%s: beta2 must be finite and >= 0", what);
    if (md.beta2 > 0.0 && md.n > kB2MaxN)
        return fail(NLCH_EUNSUPPORTED, "%s: beta2 > 0 is built for n <= %d (one workgroup "
                    "per sample)", what, kB2MaxN);
    if (!finite_pos(md.tau)) return fail(NLCH_EINVAL, "%s: tau must be > 0", what);
    if (md.boundary != NLCH_BOUNDARY_PERIODIC && md.boundary != NLCH_BOUNDARY_VOLUME)
        return fail(NLCH_EINVAL, "%s: unknown boundary %d", what, md.boundary);
    if (md.reserved != 0) return fail(NLCH_EINVAL, "%s: reserved field must be 0", what);
    if (md.boundary == NLCH_BOUNDARY_VOLUME && md.beta2 > 0.0)
        return fail(NLCH_EUNSUPPORTED, "%s: the volume-constrained domain is built for "
                    "beta2 = 0 only", what);

    const double r = md.delta * (double)md.n;
    mi.R2 = (int64_t)std::floor(r * r + 1e-9);
    mi.m = (int)isqrt64(mi.R2);
    if (mi.m > kMaxM)
        return fail(NLCH_EUNSUPPORTED, "%s: horizon of %d lattice units exceeds %d", what, mi.m,
                    kMaxM);
    if (md.n <= 2 * mi.m)
        return fail(NLCH_EINVAL, "%s: lattice n = %d must exceed twice the horizon (%d)", what,
                    md.n, mi.m);
    const int m = mi.m;
    mi.lo = md.boundary == NLCH_BOUNDARY_VOLUME ? m : 0;
    mi.side = md.n + 2 * mi.lo;
    mi.halfw.resize(m + 1);
    mi.N = 0;
    for (int dy = -m; dy <= m; ++dy) {
        const int w = (int)isqrt64(mi.R2 - (int64_t)dy * dy);
        if (dy >= 0) mi.halfw[dy] = w;
        mi.N += 2 * w + 1;
    }
    const double h = 1.0 / md.n;
    mi.g.assign(m + 1, 1.0);
    mi.e2.assign((size_t)(m + 1) * (m + 1), 1.0);
    if (md.kernel == NLCH_KERNEL_GAUSSIAN) {
        const double s2 = md.kernel_sigma * md.kernel_sigma;
        for (int k = 0; k <= m; ++k) mi.g[k] = std::exp(-(double)k * k * h * h / s2);
        for (int i = 0; i <= m; ++i)
            for (int j = 0; j <= m; ++j)
                mi.e2[(size_t)i * (m + 1) + j] = std::exp(-(double)(i * i + j * j) * h * h / s2);
    }
    mi.sum_e = 0.0;
    mi.ce_sep = 0.0;
    for (int dy = -m; dy <= m; ++dy) {
        const int ady = dy < 0 ? -dy : dy;
        const int w = mi.halfw[ady];
        for (int dx = -w; dx <= w; ++dx) {
            const int adx = dx < 0 ? -dx : dx;
            mi.sum_e += mi.e2[(size_t)ady * (m + 1) + adx];
            mi.ce_sep += mi.g[ady] * mi.g[adx];
        }
    }
    return NLCH_OK;
}


int nlch::sample_coef(const nlch_model &md, const ModelInfo &mi, double c_F, double amp,
                      Coef &c, const char *what) {
    const double h2 = 1.0 / ((double)md.n * md.n);
    c.c_gamma_h = h2 * amp * mi.sum_e;
    c.xi_h = c.c_gamma_h - c_F;
    const double tb = md.tau * md.beta1;
    const double den = 1.0 + tb * c.xi_h;
    // beta2 > 0: a strictly convex step for either sign of xi_h (the Newton
    // step for xi_h > 0, the split step for xi_h <= 0), which does not use
    // c1, a and b; they are 0 where 1 + tau beta1 xi_h <= 0
    if (md.beta2 > 0.0 && !(den > 0.0)) {
        if (!std::isfinite(c.xi_h))
            return fail(NLCH_EINVAL, "%s: xi_h = %g is not finite", what, c.xi_h);
        c.c1 = c.a = c.b = 0.0;
        return NLCH_OK;
    }
    if (!(den > 0.0))
        return fail(NLCH_EINVAL, "%s: 1 + tau*beta1*xi_h = %g must be > 0", what, den);
    c.c1 = tb / den;
    c.a = c.c1 * c_F;
    c.b = c.c1 * h2 * amp;
    return NLCH_OK;
}

size_t nlch::prec_size(int prec) { return prec == kF64 ? 8 : (prec == kF32 ? 4 : 2); }

static float rne_f32(double v) { return (float)v; }

// Chooses the kernel variant for a model under the requested algorithm.
int nlch::choose_variant(int base, int prec, bool acc64, const ModelInfo &mi, const nlch_model &md,
                   bool batch, int *variant) {
    if (md.beta2 > 0.0) {
        // the coupled step has one kernel, whatever the algorithm word asks
        if (base == NLCH_ALGO_RESIDENT)
            return fail(NLCH_EUNSUPPORTED, "RESIDENT is built for beta2 = 0 only");
        *variant = kB2;
        return NLCH_OK;
    }
    const bool res = batch && resident_supported(prec, acc64, (int)mi.R2, md.kernel, md.n,
                                                 mi.lo != 0);
    const bool row = rowrun_supported(prec, acc64, (int)mi.R2, md.kernel);
    switch (base) {
        case NLCH_ALGO_AUTO:
            *variant = res ? kResident : (row ? kRowrun : kDirect);
            return NLCH_OK;
        case NLCH_ALGO_DIRECT:
            *variant = kDirect;
            return NLCH_OK;
        case NLCH_ALGO_ROWRUN:
            if (!row)
                return fail(NLCH_EUNSUPPORTED, "ROWRUN is not built for R2 = %lld",
                            (long long)mi.R2);
            *variant = kRowrun;
            return NLCH_OK;
        case NLCH_ALGO_RESIDENT:
            if (!batch) return fail(NLCH_EINVAL, "RESIDENT applies to nlch_solve_batch only");
            if (!res)
                return fail(NLCH_EUNSUPPORTED,
                            "RESIDENT needs n = 64 or 128, a sample that fits in LDS and a "
                            "built R2 (n = %d, R2 = %lld)", md.n, (long long)mi.R2);
            *variant = kResident;
            return NLCH_OK;
        default:
            return fail(NLCH_EINVAL, "unknown algorithm %d", base);
    }
}


void nlch::fill_model_geo(const nlch_model &md, const ModelInfo &mi, int64_t e_off,
                          ModelGeo &gm) {
    std::memset(&gm, 0, sizeof(gm));
    gm.n = mi.side;
    gm.lo = mi.lo;
    gm.m = mi.m;
    gm.R2 = (int32_t)mi.R2;
    gm.N = (int32_t)mi.N;
    gm.kernel = md.kernel;
    gm.e_off = e_off;
    gm.ced = mi.ce_sep;
    gm.cef = rne_f32(mi.ce_sep);
    gm.tau_b1 = md.tau * md.beta1;
    gm.tau_b2 = md.tau * md.beta2;
    for (int k = 0; k <= mi.m; ++k) {
        gm.gd[k] = mi.g[k];
        gm.gf[k] = rne_f32(mi.g[k]);
        gm.halfw[k] = mi.halfw[k];
    }
}

void nlch::fill_sample_desc(const nlch_model &md, const ModelInfo &mi, const nlch_sample &sm,
                            const Coef &c, SampleDesc &d) {
    std::memset(&d, 0, sizeof(d));
    d.offset = sm.offset;
    d.model = sm.model;
    d.n = mi.side;
    d.a = c.a;
    d.b = c.b;
    d.af = rne_f32(c.a);
    d.bf = rne_f32(c.b);
    // a - b ce with the kernels' unit-amplitude mass ce (separable form)
    d.ap = c.c1 * (sm.c_F - sm.kernel_amp * mi.ce_sep / ((double)md.n * md.n));
    d.apf = rne_f32(d.ap);
    const double h2 = 1.0 / ((double)md.n * md.n);
    d.e_int = 0.5 * h2 * h2 * sm.kernel_amp;
    d.e_pot = 0.5 * h2 * sm.c_F;
    d.xi = c.xi_h;
}

Group nlch::make_group(const nlch_model &md, const ModelInfo &mi, int model_index, int n_ids,
                       int prec) {
    Group g;
    std::memset(&g, 0, sizeof(g));
    g.nids = n_ids;
    g.n = mi.side;
    g.lo = mi.lo;
    g.ni = md.n;
    g.m = mi.m;
    g.R2 = (int32_t)mi.R2;
    g.kernel = md.kernel;
    g.model = model_index;
    g.ta_bytes = prec == kF64 ? 8 : 4;
    return g;
}

int nlch::check_algo_flags(int32_t algo) {
    const int32_t known = 0xff | NLCH_ALGO_ACC64 | NLCH_ALGO_NOGRAPH | NLCH_ALGO_CHECK_FINITE |
                          NLCH_ALGO_AUTOTUNE;
    if (algo & ~known) return fail(NLCH_EINVAL, "unknown algorithm flags 0x%x", algo & ~known);
    const int base = algo & 0xff;
    if (base < NLCH_ALGO_AUTO || base > NLCH_ALGO_RESIDENT)
        return fail(NLCH_EINVAL, "unknown algorithm %d", base);
    return NLCH_OK;
}


// ------------------------------------------------------------ device state --

namespace {

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

// Device tables of one batch signature.
struct Batch {
    std::vector<uint8_t> key;
    int device = -1;
    DevBuf geo, ewf, ewd, sd, ids, partial;
    DevBuf epart;                        // energy partial sums (allocated on demand)
    size_t epart_cap = 0;                // doubles in epart
    DevBuf b2ws;                         // beta2 > 0 workspaces (allocated on demand)
    std::vector<Group> groups;           // launch groups
    std::vector<int> variant;            // per group
    bool tuned = false;
    std::map<std::vector<uint8_t>, hipGraphExec_t> graphs;
    // Calls with the same signature share the tables and device scratch
    // above (OoI chunk sums, energy partials, beta2 workspaces): `done` is
    // recorded after each call's work on its stream `last`, and a call on
    // another stream waits for it first.
    hipEvent_t done = nullptr;
    hipStream_t last = nullptr;
    bool used = false;
    ~Batch() {
        for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
        if (done) (void)hipEventDestroy(done);
    }
};

// Streams the launch groups of one solve run on: the caller's stream and
// up to kAuxStreams more (default priority), forked and joined with events.
constexpr int kAuxStreams = 3;

struct DevCtx {
    bool ready = false;  // every resource below created
    hipStream_t capture = nullptr;
    hipStream_t aux[kAuxStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kAuxStreams] = {};
    unsigned int *counter = nullptr;   // non-finite counter (device)
    unsigned int *counter_h = nullptr; // pinned host copy
    double *mom = nullptr;             // moments (device)
    double *mom_h = nullptr;           // pinned host copy
};

std::mutex g_mu;
std::map<int, DevCtx> g_dev;
std::vector<std::unique_ptr<Batch>> g_batches;  // most recent last
constexpr size_t kMaxBatches = 32;
constexpr size_t kMaxGraphsPerBatch = 16;

int dev_ctx(DevCtx **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    DevCtx &c = g_dev[dev];
    if (!c.ready) {
        // each resource once: a failure part-way leaves the rest to the next call
        if (!c.capture) HIP_TRY(hipStreamCreateWithFlags(&c.capture, hipStreamNonBlocking));
        for (int i = 0; i < kAuxStreams; ++i) {
            if (!c.aux[i]) HIP_TRY(hipStreamCreateWithFlags(&c.aux[i], hipStreamNonBlocking));
            if (!c.join[i]) HIP_TRY(hipEventCreateWithFlags(&c.join[i], hipEventDisableTiming));
        }
        if (!c.fork) HIP_TRY(hipEventCreateWithFlags(&c.fork, hipEventDisableTiming));
        if (!c.counter) HIP_TRY(hipMalloc((void **)&c.counter, sizeof(unsigned int)));
        if (!c.counter_h)
            HIP_TRY(hipHostMalloc((void **)&c.counter_h, sizeof(unsigned int),
                                  hipHostMallocDefault));
        if (!c.mom) HIP_TRY(hipMalloc((void **)&c.mom, sizeof(double) * 8 * NLCH_MFMC_MAX_K));
        if (!c.mom_h)
            HIP_TRY(hipHostMalloc((void **)&c.mom_h, sizeof(double) * 8 * NLCH_MFMC_MAX_K,
                                  hipHostMallocDefault));
        c.ready = true;
    }
    *out = &c;
    return NLCH_OK;
}

template <class T>
void append_bytes(std::vector<uint8_t> &k, const T &v) {
    const uint8_t *p = reinterpret_cast<const uint8_t *>(&v);
    k.insert(k.end(), p, p + sizeof(T));
}

// Builds (or finds) the device tables for a batch.
int get_batch(const nlch_model *models, int32_t n_models, const std::vector<ModelInfo> &mi,
              const nlch_sample *samples, int64_t n_samples, int prec, int algo, bool is_batch,
              Batch **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::vector<uint8_t> key;
    append_bytes(key, dev);
    append_bytes(key, prec);
    append_bytes(key, algo & (0xff | NLCH_ALGO_ACC64 | NLCH_ALGO_AUTOTUNE));
    // nlch_step and nlch_solve_batch choose kernels differently (RESIDENT is
    // a whole-solve kernel): the same model and sample must not share a batch
    append_bytes(key, is_batch);
    append_bytes(key, n_models);
    append_bytes(key, n_samples);
    for (int i = 0; i < n_models; ++i) append_bytes(key, models[i]);
    const uint8_t *sp = reinterpret_cast<const uint8_t *>(samples);
    key.insert(key.end(), sp, sp + sizeof(nlch_sample) * (size_t)n_samples);
    for (size_t i = 0; i < g_batches.size(); ++i) {
        if (g_batches[i]->key == key) {
            std::unique_ptr<Batch> b = std::move(g_batches[i]);
            g_batches.erase(g_batches.begin() + i);
            g_batches.push_back(std::move(b));
            *out = g_batches.back().get();
            return NLCH_OK;
        }
    }

    const bool acc64 = (algo & NLCH_ALGO_ACC64) != 0 || prec == kF64;
    std::unique_ptr<Batch> b(new Batch());
    b->key = key;
    b->device = dev;
    HIP_TRY(hipEventCreateWithFlags(&b->done, hipEventDisableTiming));

    // Geometry and weight tables.
    std::vector<ModelGeo> geo(n_models);
    std::vector<float> ewf;
    std::vector<double> ewd;
    for (int i = 0; i < n_models; ++i) {
        fill_model_geo(models[i], mi[i], (int64_t)ewd.size(), geo[i]);
        for (double e : mi[i].e2) {
            ewd.push_back(e);
            ewf.push_back(rne_f32(e));
        }
    }
    // Sample descriptors.
    std::vector<SampleDesc> sd((size_t)n_samples);
    for (int64_t s = 0; s < n_samples; ++s) {
        const nlch_sample &sm = samples[s];
        Coef c;
        char what[64];
        snprintf(what, sizeof(what), "sample %lld", (long long)s);
        int rc = sample_coef(models[sm.model], mi[sm.model], sm.c_F, sm.kernel_amp, c, what);
        if (rc) return rc;
        fill_sample_desc(models[sm.model], mi[sm.model], sm, c, sd[(size_t)s]);
    }
    // Groups: per model, samples in batch order.
    std::vector<std::vector<int32_t>> per_model(n_models);
    for (int64_t s = 0; s < n_samples; ++s) per_model[samples[s].model].push_back((int32_t)s);
    std::vector<int32_t> ids;
    std::vector<size_t> id_off;
    const int base = algo & 0xff;
    for (int i = 0; i < n_models; ++i) {
        if (per_model[i].empty()) continue;
        int variant = 0;
        int rc = choose_variant(base, prec, acc64, mi[i], models[i], is_batch, &variant);
        if (rc) return rc;
        Group g = make_group(models[i], mi[i], i, (int)per_model[i].size(), prec);
        for (int32_t id : per_model[i]) {
            if (sd[(size_t)id].xi > 0.0)
                ++g.b2_newton;
            else
                ++g.b2_split;
        }
        id_off.push_back(ids.size());
        ids.insert(ids.end(), per_model[i].begin(), per_model[i].end());
        b->groups.push_back(g);
        b->variant.push_back(variant);
    }
    // Upload (synchronous; once per signature).
    HIP_TRY(hipMalloc(&b->geo.p, sizeof(ModelGeo) * geo.size()));
    HIP_TRY(hipMemcpy(b->geo.p, geo.data(), sizeof(ModelGeo) * geo.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&b->ewf.p, sizeof(float) * ewf.size()));
    HIP_TRY(hipMemcpy(b->ewf.p, ewf.data(), sizeof(float) * ewf.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&b->ewd.p, sizeof(double) * ewd.size()));
    HIP_TRY(hipMemcpy(b->ewd.p, ewd.data(), sizeof(double) * ewd.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&b->sd.p, sizeof(SampleDesc) * sd.size()));
    HIP_TRY(hipMemcpy(b->sd.p, sd.data(), sizeof(SampleDesc) * sd.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&b->ids.p, sizeof(int32_t) * ids.size()));
    HIP_TRY(hipMemcpy(b->ids.p, ids.data(), sizeof(int32_t) * ids.size(), hipMemcpyHostToDevice));
    // Chunk sums of the output-of-interest reduction (streaming groups).
    std::vector<size_t> part_off(b->groups.size(), 0);
    size_t npart = 1;
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        part_off[gi] = npart;
        if (b->variant[gi] != kResident)
            npart += (size_t)ooi_chunks(b->groups[gi].ni) * b->groups[gi].nids;
    }
    HIP_TRY(hipMalloc(&b->partial.p, sizeof(double) * npart));
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        Group &g = b->groups[gi];
        g.partial = reinterpret_cast<double *>(b->partial.p) + part_off[gi];
        g.geo = reinterpret_cast<const ModelGeo *>(b->geo.p) + g.model;
        g.ewf = reinterpret_cast<const float *>(b->ewf.p);
        g.ewd = reinterpret_cast<const double *>(b->ewd.p);
        g.sd = reinterpret_cast<const SampleDesc *>(b->sd.p);
        g.ids = reinterpret_cast<const int32_t *>(b->ids.p) + id_off[gi];
    }
    if (g_batches.size() >= kMaxBatches) {
        // work enqueued earlier may still read the oldest batch's tables
        HIP_TRY(hipDeviceSynchronize());
        g_batches.erase(g_batches.begin());
    }
    g_batches.push_back(std::move(b));
    *out = g_batches.back().get();
    return NLCH_OK;
}

// True when s is capturing a graph (the caller then orders the captured
// work; events recorded outside the capture cannot be waited on inside it).
int stream_capturing(hipStream_t s, bool *cap) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &st));
    *cap = st != hipStreamCaptureStatusNone;
    return NLCH_OK;
}

// Orders a call's work after the previous call of the same batch when the
// two run on different streams (they share the batch's device scratch).
int batch_begin(Batch &b, hipStream_t s, bool *cap) {
    int rc = stream_capturing(s, cap);
    if (rc) return rc;
    if (!*cap && b.used && b.last != s) HIP_TRY(hipStreamWaitEvent(s, b.done, 0));
    return NLCH_OK;
}

int batch_end(Batch &b, hipStream_t s, bool cap) {
    if (cap) return NLCH_OK;
    HIP_TRY(hipEventRecord(b.done, s));
    b.last = s;
    b.used = true;
    return NLCH_OK;
}

// Autotuner of the streaming launch shape, cached per (device, precision,
// disc, kernel, lattice, group size).  Candidates, for R = 1 and R = 2
// columns per lane: one wave per band with band heights
// max(16, 2m) 2^k, and (shared-band kernels: FP32, m <= 16) W = 2, 4, 8
// waves per band walking L = k (2m+1) rows each (k = 1, 2, 4).  Every
// candidate is timed over three launches after a warm-up.
struct TuneKey {
    int dev, prec, R2, kernel, n, lo, nids;
    bool operator<(const TuneKey &o) const {
        return std::tie(dev, prec, R2, kernel, n, lo, nids) <
               std::tie(o.dev, o.prec, o.R2, o.kernel, o.n, o.lo, o.nids);
    }
};
struct TuneVal {
    int R, B, W, L;
    int PH;  // 2: two interleaved row phases per wave (W = 1)
};
std::map<TuneKey, TuneVal> g_tuned;
TuneVal g_force{0, 0, 0, 0, 0};  // nlch_set_stream_shape (L in ring periods),
                                 // nlch_set_stream_phases
int g_force_res_cols = 0;     // nlch_set_resident_shape
int g_force_res_rows = 0;

// Default for R = 0: the tiled kernel where the default streaming shape
// (one wave per band) would give fewer than 1024 waves in all, i.e. for one
// or a few samples of a lattice; R = 4 asks for it.
void set_shape(Group &g, const TuneVal &v) {
    g.tune_R = v.R == 4 ? 0 : v.R;
    g.tune_B = v.B;
    g.tune_W = v.W;
    g.tune_L = v.L;
    g.tune_PH = v.R == 4 ? 0 : v.PH;
    const bool built = tile_supported(g.ta_bytes == 8 ? kF64 : kF32, g.ta_bytes == 8, g.R2);
    if (v.R == 4) {
        g.tile = built;
    } else if (v.R == 0 && v.W == 0 && v.B == 0 && v.PH == 0) {
        const StreamShape sh = stream_shape(g);
        g.tile = built && (int64_t)sh.per_sample * g.nids < 1024;
    } else {
        g.tile = 0;
    }
}

int autotune_group(Group &g, int dev, int prec, bool acc64, const void *in, void *out,
                   hipStream_t s) {
    const TuneKey key{dev, prec, g.R2, g.kernel, g.n, g.lo, g.nids};
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
        set_shape(g, it->second);
        return NLCH_OK;
    }
    const int P = 2 * g.m + 1;
    const int bmin = g.m * 2 > 16 ? g.m * 2 : 16;
    std::vector<TuneVal> cands;
    for (int R = 1; R <= 2; ++R) {
        const int strips = (g.ni + 64 * R - 1) / (64 * R);
        for (int B = bmin;; B *= 2) {
            const int Bc = B < g.ni ? B : g.ni;
            const int64_t waves = (int64_t)strips * ((g.ni + Bc - 1) / Bc) * g.nids;
            if (waves >= 128 || Bc == bmin || Bc == g.ni) cands.push_back({R, Bc, 1, 0, 0});
            if (Bc >= g.ni) break;
        }
        // two row phases per wave: strips of 32R columns, twice the waves;
        // band heights bmin 2^k and 1.5 bmin 2^k
        for (int B = bmin; g.ta_bytes == 4; B *= 2) {
            for (int Bc : {B < g.ni ? B : g.ni, 3 * B / 2}) {
                if (Bc > g.ni || (Bc != B && Bc == g.ni)) continue;
                const int64_t waves =
                    (int64_t)((g.ni + 32 * R - 1) / (32 * R)) * ((g.ni + Bc - 1) / Bc) * g.nids;
                if (waves >= 128 || Bc == bmin || Bc == g.ni) cands.push_back({R, Bc, 1, 0, 2});
            }
            if (B >= g.ni) break;
        }
        if (R == 1 && tile_supported(prec, acc64, g.R2)) cands.push_back({4, 0, 0, 0});
        for (int W = 2; W <= 8 && band_built(g.m, g.ta_bytes); W *= 2)
            for (int k = 1; k <= 4; k *= 2) {
                const int L = k * P;
                if (W * L - 2 * g.m > 2 * g.ni) continue;  // far more rows than the lattice
                cands.push_back({R, 0, W, L});
            }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = 1e30f;
    TuneVal pick{0, 0, 0, 0, 0};
    for (const TuneVal &c : cands) {
        set_shape(g, c);
        hipError_t e = launch_rowrun_step(prec, acc64, g, in, out, s);  // warm-up
        if (e != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        HIP_TRY(hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r) HIP_TRY(launch_rowrun_step(prec, acc64, g, in, out, s));
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
            best = ms;
            pick = c;
        }
        const char *verbose = std::getenv("NLCH_VERBOSE");
        if (verbose && std::atoi(verbose) >= 2)
            std::fprintf(stderr, "nlch autotune: n=%d R2=%d samples=%d candidate R=%d W=%d L=%d "
                         "B=%d PH=%d: %.4f ms per launch\n", g.n, g.R2, g.nids, c.R, c.W, c.L,
                         stream_shape(g).B, stream_shape(g).PH, ms / 3.0f);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    set_shape(g, pick);
    g_tuned[key] = pick;
    if (std::getenv("NLCH_VERBOSE"))
        std::fprintf(stderr, "nlch autotune: n=%d R2=%d samples=%d -> R=%d W=%d L=%d B=%d "
                     "PH=%d (%.3f ms per launch)\n", g.n, g.R2, g.nids, pick.R, pick.W, pick.L,
                     stream_shape(g).B, stream_shape(g).PH, best / 3.0f);
    return NLCH_OK;
}

// Resident layout of a group from nlch_set_resident_shape: the forced shape
// where it names this group's lattice (cols 2 or 4: 128^2; cols 1: 64^2).
bool forced_resident_shape(const Group &g, int *cols, int *rows) {
    const int c = g_force_res_cols, r = g_force_res_rows;
    if (c == 0) return false;
    const bool fits = (g.ni == 128 && (c == 2 || c == 4)) || (g.ni == 64 && c == 1);
    *cols = fits ? c : 0;
    *rows = fits ? r : 0;
    return true;
}

// Autotuner of the resident layout, cached per (device, precision, disc,
// kernel, lattice, group size): FP32 periodic groups of 128^2 time (2, 16),
// (4, 16) and (4, 8); of 64^2, bands of 8 (m <= 8), 16 and 32 rows.  Each
// candidate runs min(nsteps, 10) steps of the whole group -- once to warm
// up, then twice timed (the faster counts) -- on a copy of the caller's
// states in a buffer of the tuner's own, which it frees afterwards.  The
// default layout ((4, 8) where built, else 16-row bands) is kept unless
// another is at least 3% faster, so that near-equal timings do not switch
// the layout (and the rounding of the results) from run to run.
struct ResTune {
    int cols, rows;
};
std::map<TuneKey, ResTune> g_tuned_res;

int autotune_resident(Group &g, int dev, int prec, bool acc64, const nlch_sample *samples,
                      int64_t n_samples, const void *state, int nsteps, hipStream_t s) {
    g.res_cols = g.res_rows = 0;
    std::vector<ResTune> cands;
    if (prec == kF32 && !acc64 && g.lo == 0) {
        if (g.ni == 128 && resident4_built(g.R2)) cands = {{2, 16}, {4, 16}, {4, 8}};
        if (g.ni == 64) {
            if (g.m <= 8) cands.push_back({1, 8});
            cands.push_back({1, 16});
            cands.push_back({1, 32});
        }
    }
    if (prec == kF64 && g.lo == 0 && g.ni == 64 && g.m <= 8) cands = {{1, 8}, {1, 16}};
    if (cands.empty() || nsteps < 1) return NLCH_OK;
    const TuneKey key{dev, prec, g.R2, g.kernel, g.n, g.lo, g.nids};
    auto it = g_tuned_res.find(key);
    if (it != g_tuned_res.end()) {
        g.res_cols = it->second.cols;
        g.res_rows = it->second.rows;
        return NLCH_OK;
    }
    int64_t end = 0;  // elements of the state buffer the group's samples span
    for (int64_t i = 0; i < n_samples; ++i)
        if (samples[i].model == g.model)
            end = std::max<int64_t>(end, samples[i].offset + (int64_t)g.n * g.n);
    void *tmp = nullptr;
    double *tooi = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (tmp) (void)hipFree(tmp);
        if (tooi) (void)hipFree(tooi);
    };
    int rc = [&]() -> int {
        HIP_TRY(hipMalloc(&tmp, (size_t)end * prec_size(prec)));
        HIP_TRY(hipMalloc((void **)&tooi, sizeof(double) * 2 * (size_t)n_samples));
        HIP_TRY(hipMemcpyAsync(tmp, state, (size_t)end * prec_size(prec),
                               hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        const int nt = nsteps < 10 ? nsteps : 10;
        const ResTune def = g.ni == 128 ? ResTune{4, 8} : ResTune{1, 16};
        float best = 1e30f, def_ms = 1e30f;
        ResTune pick{0, 0};
        for (const ResTune &c : cands) {
            g.res_cols = c.cols;
            g.res_rows = c.rows;
            HIP_TRY(launch_resident(prec, acc64, g, tmp, nt, tooi, s, nullptr, 0));
            for (int r = 0; r < 2; ++r) {
                HIP_TRY(hipEventRecord(e0, s));
                HIP_TRY(launch_resident(prec, acc64, g, tmp, nt, tooi, s, nullptr, 0));
                HIP_TRY(hipEventRecord(e1, s));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    pick = c;
                }
                if (c.cols == def.cols && c.rows == def.rows && ms < def_ms) def_ms = ms;
            }
        }
        if (best > 0.97f * def_ms) {
            pick = def;
            best = def_ms;
        }
        g.res_cols = pick.cols;
        g.res_rows = pick.rows;
        g_tuned_res[key] = pick;
        if (std::getenv("NLCH_VERBOSE"))
            std::fprintf(stderr, "nlch autotune (resident): n=%d R2=%d samples=%d -> "
                         "cols=%d rows=%d (%.3f ms per %d steps)\n", g.n, g.R2, g.nids,
                         pick.cols, pick.rows, best, nt);
        return NLCH_OK;
    }();
    cleanup();
    if (rc) g.res_cols = g.res_rows = 0;
    return rc;
}

hipError_t launch_step(int variant, int prec, bool acc64, const Group &g, const void *in,
                       void *out, hipStream_t s, double *epart = nullptr, bool warm = false) {
    if (variant == kRowrun) return launch_rowrun_step(prec, acc64, g, in, out, s, epart);
    if (variant == kB2) return launch_b2_step(prec, g, in, out, s, epart, warm);
    return launch_direct_step(prec, acc64, g, in, out, s, epart);
}

// Workspaces of the beta2 > 0 groups (b2_ws_doubles(n) per sample), allocated
// on first use and kept with the batch.
int ensure_b2ws(Batch &b) {
    size_t need = 0;
    for (size_t gi = 0; gi < b.groups.size(); ++gi)
        if (b.variant[gi] == kB2)
            need += (size_t)b2_ws_doubles(b.groups[gi].n) * b.groups[gi].nids;
    if (need == 0 || b.b2ws.p) return NLCH_OK;
    HIP_TRY(hipMalloc(&b.b2ws.p, sizeof(double) * need));
    size_t off = 0;
    for (size_t gi = 0; gi < b.groups.size(); ++gi)
        if (b.variant[gi] == kB2) {
            b.groups[gi].ws = reinterpret_cast<double *>(b.b2ws.p) + off;
            off += (size_t)b2_ws_doubles(b.groups[gi].n) * b.groups[gi].nids;
        }
    return NLCH_OK;
}

// Workgroups one sample of a streaming group occupies per step launch.
int step_blocks_per_sample(int variant, const Group &g) {
    if (variant == kRowrun) return stream_shape(g).per_sample;
    if (variant == kB2) return 1;
    return direct_tiles(g.ni);
}

// Energy partial-sum area of streaming group gi (after ensure_epart).
double *group_epart(Batch &b, size_t gi) {
    size_t off = 0;
    for (size_t i = 0; i < gi; ++i)
        if (b.variant[i] != kResident)
            off += 2 * (size_t)step_blocks_per_sample(b.variant[i], b.groups[i]) * b.groups[i].nids;
    return reinterpret_cast<double *>(b.epart.p) + off;
}

int ensure_epart(Batch &b) {
    size_t need = 2;
    for (size_t gi = 0; gi < b.groups.size(); ++gi)
        if (b.variant[gi] != kResident)
            need += 2 * (size_t)step_blocks_per_sample(b.variant[gi], b.groups[gi]) *
                    b.groups[gi].nids;
    if (need <= b.epart_cap) return NLCH_OK;
    if (b.epart.p) {
        HIP_TRY(hipDeviceSynchronize());  // a queued graph may still read the old area
        HIP_TRY(hipFree(b.epart.p));
        b.epart.p = nullptr;
        b.epart_cap = 0;
        for (auto &kv : b.graphs) (void)hipGraphExecDestroy(kv.second);
        b.graphs.clear();
    }
    HIP_TRY(hipMalloc(&b.epart.p, sizeof(double) * need));
    b.epart_cap = need;
    return NLCH_OK;
}

// Enqueues one launch group's whole solve on stream s.  With `energy`
// (n_samples-strided rows k = 0..nsteps), every step launch also reduces E_h
// of its input state, and one more launch evaluates E_h(u^nsteps) (its
// update goes to `scratch` and is dropped).  Streaming groups ping-pong
// between state and scratch, projecting into whichever buffer makes the last
// step land in `state`; every group touches only its own samples' elements.
int enqueue_group(Batch &b, size_t gi, int prec, bool acc64, int nsteps, void *state,
                  void *scratch, double *ooi, double *energy, int64_t estride,
                  hipStream_t s) {
    const Group &g = b.groups[gi];
    const int variant = b.variant[gi];
    if (variant == kResident) {
        HIP_TRY(launch_resident(prec, acc64, g, state, nsteps, ooi, s, energy, estride));
        return NLCH_OK;
    }
    void *buf0 = (nsteps % 2) ? scratch : state;
    void *buf1 = (buf0 == state) ? scratch : state;
    // the steps write the updated block only: under a volume constraint both
    // buffers need the (projected) ring of fixed values
    if (g.lo != 0 && nsteps > 0) HIP_TRY(launch_project(prec, g, state, buf1, s));
    HIP_TRY(launch_project(prec, g, state, buf0, s));
    double *ep = energy ? group_epart(b, gi) : nullptr;
    const int ps = step_blocks_per_sample(variant, g);
    void *cur = buf0, *nxt = buf1;
    for (int k = 0; k <= nsteps; ++k) {
        if (k == nsteps) {
            if (!energy) break;
            cur = state;
            nxt = scratch;
        }
        // (beta2 > 0: every step after a solve's first starts Newton from
        // the previous step's z)
        HIP_TRY(launch_step(variant, prec, acc64, g, cur, nxt, s, ep, k > 0));
        if (energy) HIP_TRY(launch_energy_final(g, ep, ps, energy + (int64_t)k * estride, s));
        std::swap(cur, nxt);
    }
    HIP_TRY(launch_ooi(prec, g, state, ooi, 2, s));
    return NLCH_OK;
}

// Enqueues a whole batch solve on stream s.  The launch groups are
// independent, so with several groups each runs on its own stream (the
// caller's and the context's auxiliary streams, forked from and joined back
// into s with events): a long lattice's step chain overlaps the other
// levels' launches.
int enqueue_solve(Batch &b, DevCtx &ctx, int prec, bool acc64, int nsteps, void *state,
                  void *scratch, double *ooi, double *energy, int64_t estride, hipStream_t s) {
    const size_t G = b.groups.size();
    if (G == 1)
        return enqueue_group(b, 0, prec, acc64, nsteps, state, scratch, ooi, energy, estride, s);
    const int naux = (int)std::min<size_t>(G - 1, (size_t)kAuxStreams);
    HIP_TRY(hipEventRecord(ctx.fork, s));
    int forked = 0, rc = NLCH_OK;
    for (; forked < naux && !rc; ++forked) {
        if (inject_device_error()) {
            rc = fail(NLCH_EDEVICE, "hipStreamWaitEvent(aux): injected device error");
            break;
        }
        const hipError_t e = hipStreamWaitEvent(ctx.aux[forked], ctx.fork, 0);
        if (e != hipSuccess) {
            rc = fail(NLCH_EDEVICE, "hipStreamWaitEvent(aux): %s", hipGetErrorString(e));
            break;
        }
    }
    // group 0 (the first model, the high-fidelity level in an MFMC batch) on
    // the caller's stream, the rest round-robin on the auxiliary streams.
    // The launches are enqueued step-major (step k of every streaming group,
    // then step k + 1), not group by group: the runtime keeps only a few
    // launches in flight ahead of the device, so a group-major order would
    // hold the later groups back until the host had nearly finished enqueuing
    // the first group's chain, and the levels would hardly overlap.
    if (!rc) rc = [&]() -> int {
        struct Run {
            size_t gi;
            hipStream_t s;
            void *cur, *nxt;
            double *ep;
            int ps;
        };
        std::vector<Run> runs;
        for (size_t gi = 0; gi < G; ++gi) {
            hipStream_t sg = gi == 0 ? s : ctx.aux[(gi - 1) % naux];
            const Group &g = b.groups[gi];
            if (b.variant[gi] == kResident) {
                HIP_TRY(launch_resident(prec, acc64, g, state, nsteps, ooi, sg, energy, estride));
                continue;
            }
            // as enqueue_group: the steps ping-pong so that the last lands in
            // state; under a volume constraint both buffers get the ring
            void *buf0 = (nsteps % 2) ? scratch : state;
            void *buf1 = (buf0 == state) ? scratch : state;
            if (g.lo != 0 && nsteps > 0) HIP_TRY(launch_project(prec, g, state, buf1, sg));
            HIP_TRY(launch_project(prec, g, state, buf0, sg));
            runs.push_back({gi, sg, buf0, buf1, energy ? group_epart(b, gi) : nullptr,
                            step_blocks_per_sample(b.variant[gi], g)});
        }
        for (int k = 0; k <= nsteps; ++k) {
            if (k == nsteps && !energy) break;
            for (Run &r : runs) {
                const Group &g = b.groups[r.gi];
                if (k == nsteps) {
                    r.cur = state;
                    r.nxt = scratch;
                }
                HIP_TRY(launch_step(b.variant[r.gi], prec, acc64, g, r.cur, r.nxt, r.s, r.ep,
                                    k > 0));
                if (energy)
                    HIP_TRY(launch_energy_final(g, r.ep, r.ps, energy + (int64_t)k * estride,
                                                r.s));
                std::swap(r.cur, r.nxt);
            }
        }
        for (const Run &r : runs) HIP_TRY(launch_ooi(prec, b.groups[r.gi], state, ooi, 2, r.s));
        return NLCH_OK;
    }();
    // Join every forked stream back into s, after a failure too: a capture
    // must end joined, and later work on s must follow what the auxiliary
    // streams already hold.  (Not subject to failure injection.)
    for (int i = 0; i < forked; ++i) {
        hipError_t e = hipEventRecord(ctx.join[i], ctx.aux[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, ctx.join[i], 0);
        if (e != hipSuccess && !rc)
            rc = fail(NLCH_EDEVICE, "joining the auxiliary streams: %s", hipGetErrorString(e));
    }
    return rc;
}

}  // namespace

void nlch::set_default_shape(Group &g) { set_shape(g, {0, 0, 0, 0}); }

// nlch_solve_batch and nlch_solve_batch_energy (energy_out nullable here).
static int solve_impl(const nlch_model *models, int32_t n_models, const nlch_sample *samples,
                      int64_t n_samples, int32_t nsteps, int32_t precision, int32_t algo,
                      void *state, void *scratch, double *ooi_out, double *energy_out,
                      void *hip_stream) {
    if (!models || n_models < 1) return fail(NLCH_EINVAL, "need at least one model");
    if (!samples || n_samples < 1) return fail(NLCH_EINVAL, "need at least one sample");
    if (n_samples > (int64_t)1 << 30) return fail(NLCH_EINVAL, "too many samples");
    if (nsteps < 0) return fail(NLCH_EINVAL, "nsteps must be >= 0");
    if (precision < NLCH_F64 || precision > NLCH_F16_STORE)
        return fail(NLCH_EINVAL, "unknown precision %d", precision);
    int rc = check_algo_flags(algo);
    if (rc) return rc;
    if (!state || !ooi_out) return fail(NLCH_EINVAL, "state and ooi_out must be non-NULL");
    std::vector<ModelInfo> mi((size_t)n_models);
    for (int i = 0; i < n_models; ++i) {
        char what[48];
        snprintf(what, sizeof(what), "model %d", i);
        rc = analyze_model(models[i], mi[i], what);
        if (rc) return rc;
        if (energy_out && mi[i].lo != 0)
            return fail(NLCH_EUNSUPPORTED, "%s: the energy trace is built for the periodic "
                        "domain only", what);
    }
    // Samples: indices, parameters, non-overlapping states.
    std::vector<std::pair<int64_t, int64_t>> extents((size_t)n_samples);
    for (int64_t s = 0; s < n_samples; ++s) {
        const nlch_sample &sm = samples[s];
        if (sm.model < 0 || sm.model >= n_models)
            return fail(NLCH_EINVAL, "sample %lld: model index %d out of range", (long long)s,
                        sm.model);
        if (sm.reserved != 0)
            return fail(NLCH_EINVAL, "sample %lld: reserved field must be 0", (long long)s);
        if (!finite_pos(sm.c_F) || !finite_pos(sm.kernel_amp))
            return fail(NLCH_EINVAL, "sample %lld: c_F and kernel_amp must be > 0", (long long)s);
        if (sm.offset < 0) return fail(NLCH_EINVAL, "sample %lld: negative offset", (long long)s);
        const int64_t side = mi[sm.model].side;
        extents[(size_t)s] = {sm.offset, sm.offset + side * side};
        Coef c;
        char what[48];
        snprintf(what, sizeof(what), "sample %lld", (long long)s);
        rc = sample_coef(models[sm.model], mi[sm.model], sm.c_F, sm.kernel_amp, c, what);
        if (rc) return rc;
    }
    std::sort(extents.begin(), extents.end());
    for (size_t i = 1; i < extents.size(); ++i)
        if (extents[i].first < extents[i - 1].second)
            return fail(NLCH_EINVAL, "sample states overlap in the state buffer");
    // Kernel variant per model (host decision, before any device work).
    const bool acc64 = (algo & NLCH_ALGO_ACC64) != 0 || precision == kF64;
    std::vector<char> used((size_t)n_models, 0);
    for (int64_t s = 0; s < n_samples; ++s) used[(size_t)samples[s].model] = 1;
    bool need_scratch = false;
    for (int i = 0; i < n_models; ++i) {
        if (!used[(size_t)i]) continue;
        int variant = 0;
        rc = choose_variant(algo & 0xff, precision, acc64, mi[i], models[i], true, &variant);
        if (rc) return rc;
        need_scratch |= (variant != kResident);
    }
    if (need_scratch && !scratch)
        return fail(NLCH_EINVAL, "scratch must be non-NULL unless every sample runs RESIDENT");

    std::lock_guard<std::mutex> lk(g_mu);
    DevCtx *ctx = nullptr;
    rc = dev_ctx(&ctx);
    if (rc) return rc;
    Batch *b = nullptr;
    rc = get_batch(models, n_models, mi, samples, n_samples, precision, algo, true, &b);
    if (rc) return rc;
    // the cached batch's kernels decide whether scratch is read
    for (size_t gi = 0; gi < b->groups.size(); ++gi)
        if (b->variant[gi] != kResident && !scratch)
            return fail(NLCH_EINVAL, "scratch must be non-NULL unless every sample runs RESIDENT");
    hipStream_t s = (hipStream_t)hip_stream;
    bool capturing = false;
    rc = batch_begin(*b, s, &capturing);
    if (rc) return rc;

    if (algo & NLCH_ALGO_CHECK_FINITE) {
        HIP_TRY(hipMemsetAsync(ctx->counter, 0, sizeof(unsigned int), s));
        for (const Group &g : b->groups)
            HIP_TRY(launch_count_nonfinite(precision, g, state, ctx->counter, s));
        HIP_TRY(hipMemcpyAsync(ctx->counter_h, ctx->counter, sizeof(unsigned int),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (*ctx->counter_h)
            return fail(NLCH_EINVAL, "initial state holds %u non-finite values", *ctx->counter_h);
    }

    if (g_force.R || g_force.W || g_force.L || g_force.B || g_force.PH) {
        // shape set by nlch_set_stream_shape (k periods per wave -> rows)
        for (size_t gi = 0; gi < b->groups.size(); ++gi) {
            if (b->variant[gi] != kRowrun) continue;
            Group &g = b->groups[gi];
            const int k = g_force.L > 0 ? g_force.L : 1;
            set_shape(g, {g_force.R, g_force.B, g_force.W, k * (2 * g.m + 1), g_force.PH});
        }
        b->tuned = false;
    } else if ((algo & NLCH_ALGO_AUTOTUNE) && !b->tuned) {
        TraceRange tr("nlch autotune");
        for (size_t gi = 0; gi < b->groups.size(); ++gi) {
            if (b->variant[gi] != kRowrun) continue;
            rc = autotune_group(b->groups[gi], b->device, precision, acc64, state, scratch, s);
            if (rc) return rc;
        }
        b->tuned = true;
    } else if (!(algo & NLCH_ALGO_AUTOTUNE)) {
        for (Group &g : b->groups) set_shape(g, {0, 0, 0, 0});
    }

    // resident layouts: forced (nlch_set_resident_shape), tuned, or default
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        Group &g = b->groups[gi];
        g.res_cols = g.res_rows = 0;
        if (b->variant[gi] != kResident || forced_resident_shape(g, &g.res_cols, &g.res_rows))
            continue;
        if ((algo & NLCH_ALGO_AUTOTUNE) && !capturing) {
            TraceRange tr("nlch autotune (resident)");
            rc = autotune_resident(g, b->device, precision, acc64, samples, n_samples, state,
                                   nsteps, s);
            if (rc) return rc;
        }
    }

    if (energy_out) {
        rc = ensure_epart(*b);
        if (rc) return rc;
    }
    rc = ensure_b2ws(*b);
    if (rc) return rc;

    if (algo & NLCH_ALGO_NOGRAPH) {
        TraceRange tr("nlch enqueue (no graph)");
        rc = enqueue_solve(*b, *ctx, precision, acc64, nsteps, state, scratch, ooi_out,
                           energy_out, n_samples, s);
        if (rc) return rc;
        return batch_end(*b, s, capturing);
    }

    std::vector<uint8_t> gk;
    append_bytes(gk, state);
    append_bytes(gk, scratch);
    append_bytes(gk, ooi_out);
    append_bytes(gk, energy_out);
    append_bytes(gk, nsteps);
    for (const Group &g : b->groups) {
        append_bytes(gk, g.tune_R);
        append_bytes(gk, g.tune_B);
        append_bytes(gk, g.tune_W);
        append_bytes(gk, g.tune_L);
        append_bytes(gk, g.tune_PH);
        append_bytes(gk, g.res_cols);
        append_bytes(gk, g.res_rows);
        append_bytes(gk, g.tile);
    }
    auto it = b->graphs.find(gk);
    if (it == b->graphs.end()) {
        if (b->graphs.size() >= kMaxGraphsPerBatch) {
            // a caller cycling through many buffers or step counts: drop the
            // cached graphs (after the device has finished any of them)
            HIP_TRY(hipDeviceSynchronize());
            for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
            b->graphs.clear();
        }
        TraceRange tr("nlch graph capture");
        HIP_TRY(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeRelaxed));
        rc = enqueue_solve(*b, *ctx, precision, acc64, nsteps, state, scratch, ooi_out,
                           energy_out, n_samples, ctx->capture);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->capture, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();  // the error is reported here, not to the next HIP call
            return rc;
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(NLCH_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(NLCH_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
        }
        it = b->graphs.emplace(gk, exec).first;
    }
    {
        TraceRange tr("nlch graph replay");
        HIP_TRY(hipGraphLaunch(it->second, s));
    }
    return batch_end(*b, s, capturing);
}

// --------------------------------------------------------------------- ABI --

extern "C" {

int nlch_version(void) { return 6; }

const char *nlch_last_error(void) { return g_last_error.c_str(); }

int nlch_debug_inject_device_error(int32_t nth) {
    if (nth < 0) return fail(NLCH_EINVAL, "nth must be >= 0 (0 disarms)");
    g_inject.store(nth);
    return NLCH_OK;
}

int nlch_rowrun_supported(int32_t precision, int64_t *r2_list, int32_t cap) {
    if (precision < NLCH_F64 || precision > NLCH_F16_STORE)
        return fail(NLCH_EINVAL, "unknown precision %d", precision);
    if (cap < 0 || (cap > 0 && !r2_list)) return fail(NLCH_EINVAL, "bad output array");
    return rowrun_r2_list(precision, r2_list, cap);
}

int nlch_disc(int32_t n, double delta, int64_t *R2, int32_t *m, int64_t *N, int32_t *halfw,
              int32_t cap) {
    if (n <= 0) return fail(NLCH_EINVAL, "n must be > 0");
    if (!std::isfinite(delta) || delta < 0.0 || delta * n > 1e6)
        return fail(NLCH_EINVAL, "delta must be finite and >= 0");
    const double r = delta * (double)n;
    const int64_t r2 = (int64_t)std::floor(r * r + 1e-9);
    const int64_t mm = isqrt64(r2);
    if (halfw && cap < 2 * mm + 1) return fail(NLCH_EINVAL, "halfw needs %lld entries",
                                                (long long)(2 * mm + 1));
    int64_t cnt = 0;
    for (int64_t dy = -mm; dy <= mm; ++dy) {
        const int64_t w = isqrt64(r2 - dy * dy);
        if (halfw) halfw[dy + mm] = (int32_t)w;
        cnt += 2 * w + 1;
    }
    if (R2) *R2 = r2;
    if (m) *m = (int32_t)mm;
    if (N) *N = cnt;
    return NLCH_OK;
}

int nlch_model_constants(const nlch_model *model, double *c_gamma_h, double *xi_h, double *c1) {
    if (!model) return fail(NLCH_EINVAL, "model is NULL");
    ModelInfo mi;
    int rc = analyze_model(*model, mi, "model");
    if (rc) return rc;
    Coef c;
    rc = sample_coef(*model, mi, model->c_F, model->kernel_amp, c, "model");
    if (rc) return rc;
    if (c_gamma_h) *c_gamma_h = c.c_gamma_h;
    if (xi_h) *xi_h = c.xi_h;
    if (c1) *c1 = c.c1;
    return NLCH_OK;
}

int nlch_step(const nlch_model *model, int32_t precision, int32_t algo, const void *u_in,
              void *u_out, double *ooi_out, void *hip_stream) {
    if (!model) return fail(NLCH_EINVAL, "model is NULL");
    if (precision < NLCH_F64 || precision > NLCH_F16_STORE)
        return fail(NLCH_EINVAL, "unknown precision %d", precision);
    int rc = check_algo_flags(algo);
    if (rc) return rc;
    if ((algo & 0xff) == NLCH_ALGO_RESIDENT)
        return fail(NLCH_EINVAL, "RESIDENT applies to nlch_solve_batch only");
    if (!u_in || !u_out) return fail(NLCH_EINVAL, "state pointers must be non-NULL");
    ModelInfo mi;
    rc = analyze_model(*model, mi, "model");
    if (rc) return rc;
    const size_t bytes = prec_size(precision) * (size_t)mi.side * mi.side;
    const char *pi = (const char *)u_in, *po = (const char *)u_out;
    if (pi < po + bytes && po < pi + bytes)
        return fail(NLCH_EINVAL, "u_in and u_out overlap (the stencil reads neighbours)");
    nlch_sample smp;
    std::memset(&smp, 0, sizeof(smp));
    smp.model = 0;
    smp.c_F = model->c_F;
    smp.kernel_amp = model->kernel_amp;
    smp.offset = 0;
    Coef c;
    rc = sample_coef(*model, mi, smp.c_F, smp.kernel_amp, c, "model");
    if (rc) return rc;
    {
        int variant = 0;
        rc = choose_variant(algo & 0xff, precision,
                            (algo & NLCH_ALGO_ACC64) != 0 || precision == kF64, mi, *model,
                            false, &variant);
        if (rc) return rc;
    }

    std::lock_guard<std::mutex> lk(g_mu);
    DevCtx *ctx = nullptr;
    rc = dev_ctx(&ctx);
    if (rc) return rc;
    std::vector<ModelInfo> mis{mi};
    Batch *b = nullptr;
    rc = get_batch(model, 1, mis, &smp, 1, precision, algo & ~NLCH_ALGO_CHECK_FINITE, false, &b);
    if (rc) return rc;
    const bool acc64 = (algo & NLCH_ALGO_ACC64) != 0 || precision == kF64;
    hipStream_t s = (hipStream_t)hip_stream;
    rc = ensure_b2ws(*b);
    if (rc) return rc;
    bool capturing = false;
    rc = batch_begin(*b, s, &capturing);
    if (rc) return rc;
    Group &g = b->groups[0];
    set_shape(g, {0, 0, 0, 0});  // the default shape (tiled for one sample where built)
    // the step writes the updated block only; the fixed ring is carried over
    if (g.lo != 0) HIP_TRY(launch_project(precision, g, u_in, u_out, s));
    HIP_TRY(launch_step(b->variant[0], precision, acc64, g, u_in, u_out, s));
    if (ooi_out) HIP_TRY(launch_ooi(precision, g, u_out, ooi_out, 2, s));
    return batch_end(*b, s, capturing);
}

int nlch_set_stream_shape(int32_t R, int32_t W, int32_t periods, int32_t B) {
    if (!(R == 0 || R == 1 || R == 2 || R == 4) || !(W == 0 || W == 1 || W == 2 || W == 4 || W == 8) ||
        periods < 0 || periods > 64 || B < 0 || (R == 4 && (W > 1 || periods || B)))
        return fail(NLCH_EINVAL, "bad streaming shape (R in {0,1,2,4}, W in {0,1,2,4,8}, "
                                 "periods 0..64, B >= 0; R = 4 takes no other field)");
    std::lock_guard<std::mutex> lk(g_mu);
    g_force = {R, B, W, periods, g_force.PH};
    return NLCH_OK;
}

int nlch_set_stream_phases(int32_t phases) {
    if (phases < 0 || phases > 2)
        return fail(NLCH_EINVAL, "row phases per wave must be 0 (default), 1 or 2");
    std::lock_guard<std::mutex> lk(g_mu);
    g_force.PH = phases;
    return NLCH_OK;
}

int nlch_set_resident_shape(int32_t cols_per_lane, int32_t rows_per_lane) {
    const int c = cols_per_lane, r = rows_per_lane;
    if (!((c == 0 && r == 0) || (c == 2 && r == 16) || (c == 4 && (r == 16 || r == 8)) ||
          (c == 1 && (r == 8 || r == 16 || r == 32))))
        return fail(NLCH_EINVAL, "resident shape must be (0, 0) (default), (2, 16), (4, 16) or "
                    "(4, 8) (128^2), or (1, 8), (1, 16) or (1, 32) (64^2) columns and rows "
                    "per lane");
    std::lock_guard<std::mutex> lk(g_mu);
    g_force_res_cols = c;
    g_force_res_rows = r;
    return NLCH_OK;
}

int nlch_solve_batch(const nlch_model *models, int32_t n_models, const nlch_sample *samples,
                     int64_t n_samples, int32_t nsteps, int32_t precision, int32_t algo,
                     void *state, void *scratch, double *ooi_out, void *hip_stream) {
    return solve_impl(models, n_models, samples, n_samples, nsteps, precision, algo, state,
                      scratch, ooi_out, nullptr, hip_stream);
}

int nlch_solve_batch_energy(const nlch_model *models, int32_t n_models,
                            const nlch_sample *samples, int64_t n_samples, int32_t nsteps,
                            int32_t precision, int32_t algo, void *state, void *scratch,
                            double *ooi_out, double *energy_out, void *hip_stream) {
    if (!energy_out) return fail(NLCH_EINVAL, "energy_out must be non-NULL");
    return solve_impl(models, n_models, samples, n_samples, nsteps, precision, algo, state,
                      scratch, ooi_out, energy_out, hip_stream);
}

int mfmc_estimate(int32_t K, const int64_t *m, const double *const *y_dev, int64_t y_stride,
                  const double *alpha, mfmc_result *out, void *hip_stream) {
    if (K < 1 || K > NLCH_MFMC_MAX_K)
        return fail(NLCH_EINVAL, "K must be in [1, %d]", NLCH_MFMC_MAX_K);
    if (!m || !y_dev || !out) return fail(NLCH_EINVAL, "m, y_dev and out must be non-NULL");
    if (m[0] < (alpha ? 1 : 2))
        return fail(NLCH_EINVAL, alpha ? "m[0] must be >= 1" : "m[0] must be >= 2 without alpha");
    if (y_stride < 1) return fail(NLCH_EINVAL, "y_stride must be >= 1");
    for (int j = 1; j < K; ++j)
        if (m[j] < m[j - 1]) return fail(NLCH_EINVAL, "sample counts must be non-decreasing");
    for (int j = 0; j < K; ++j)
        if (!y_dev[j]) return fail(NLCH_EINVAL, "y_dev[%d] is NULL", j);
    if (alpha)
        for (int j = 0; j + 1 < K; ++j)
            if (!std::isfinite(alpha[j])) return fail(NLCH_EINVAL, "alpha[%d] not finite", j);

    std::lock_guard<std::mutex> lk(g_mu);
    DevCtx *ctx = nullptr;
    int rc = dev_ctx(&ctx);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_TRY(launch_moments(K, y_dev, m, y_stride, ctx->mom, s));
    HIP_TRY(hipMemcpyAsync(ctx->mom_h, ctx->mom, sizeof(double) * 8 * K, hipMemcpyDeviceToHost,
                           s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memset(out, 0, sizeof(*out));
    const double *mo = ctx->mom_h;
    const double var1 = mo[2];
    for (int j = 0; j < K; ++j) {
        out->mean_mj[j] = mo[8 * j + 0];
        out->mean_mjm1[j] = j > 0 ? mo[8 * j + 1] : NAN;
        out->var[j] = mo[8 * j + 2];
        const double cov = mo[8 * j + 3];
        out->rho[j] = (var1 == 0.0 || out->var[j] == 0.0)
                          ? 0.0
                          : cov / std::sqrt(var1 * out->var[j]);
    }
    out->alpha[0] = 1.0;
    for (int j = 1; j < K; ++j) {
        if (alpha)
            out->alpha[j] = alpha[j - 1];
        else
            out->alpha[j] = out->var[j] == 0.0
                                ? 0.0
                                : out->rho[j] * std::sqrt(var1) / std::sqrt(out->var[j]);
    }
    double q = out->mean_mj[0];
    for (int j = 1; j < K; ++j) q += out->alpha[j] * (out->mean_mj[j] - out->mean_mjm1[j]);
    out->q_mfmc = q;
    out->q_mc = out->mean_mj[0];
    return NLCH_OK;
}

}  // extern "C"
