// nlch_step_noalloc: nlch_step for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).
//
// nlch_step keeps a model's device tables (geometry, sample descriptor,
// 2-D weights of the direct kernel) and the chunk sums of its FP64
// output-of-interest reduction in memory the library allocates per call
// signature.  This entry point keeps them in one file-scope device array of
// fixed size instead, and writes the tables with small kernels whose
// arguments carry the values (no allocation, no host-to-device copy, nothing
// that a graph capture could not record).  It launches the same step and
// reduction kernels on the same tables, so its results equal nlch_step's.
//
// The array exists once per GPU and every call on that GPU uses it: calls
// that overlap on one GPU (concurrent streams, or graphs replayed
// concurrently) race on it and must be ordered by the caller.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "nlch.h"
#include "nlch_host.h"
#include "nlch_internal.h"

namespace {

using namespace nlch;

// Size of the static device area (per GPU).
constexpr size_t kScratchBytes = 128 * 1024;

// Layout: geometry, sample descriptor, sample index, then (direct kernel)
// the FP64 and FP32 2-D unit weights, then the OoI chunk sums; every part
// starts on a 256-byte boundary.
constexpr size_t kOffGeo = 0;
constexpr size_t kOffDesc = 1024;
constexpr size_t kOffIds = 1280;
constexpr size_t kOffTables = 1536;
static_assert(sizeof(ModelGeo) <= kOffDesc - kOffGeo, "ModelGeo outgrew its slot");
static_assert(sizeof(SampleDesc) <= kOffIds - kOffDesc, "SampleDesc outgrew its slot");

constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Writes nwords 32-bit words carried in the kernel arguments at word offset
// off of dst.
constexpr int kFillWords = 480;
struct FillChunk {
    uint32_t off, nwords;
    uint32_t w[kFillWords];
};

__global__ __launch_bounds__(256) void k_fill_words(uint32_t *__restrict__ dst, FillChunk c) {
    for (uint32_t i = threadIdx.x; i < c.nwords; i += 256) dst[c.off + i] = c.w[i];
}

// Device address of this GPU's array, looked up once per device with that
// device current (the array's name is a host-side stand-in).
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

int scratch_address(void **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(NLCH_EUNSUPPORTED, "device %d beyond the %d this library tracks", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(NLCH_EDEVICE, "hipGetSymbolAddress returned no address");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return NLCH_OK;
}

// Enqueues the word image img (bytes [0, img.size() * 4) of the area) in
// chunks of kFillWords, skipping all-zero chunks past the fixed slots.
int fill_area(void *area, const std::vector<uint32_t> &img, hipStream_t s) {
    FillChunk c;
    for (size_t i = 0; i < img.size(); i += kFillWords) {
        const size_t cnt = img.size() - i < (size_t)kFillWords ? img.size() - i : kFillWords;
        c.off = (uint32_t)i;
        c.nwords = (uint32_t)cnt;
        std::memcpy(c.w, img.data() + i, cnt * 4);
        hipLaunchKernelGGL(k_fill_words, dim3(1), dim3(256), 0, s,
                           reinterpret_cast<uint32_t *>(area), c);
        HIP_TRY(hipGetLastError());
    }
    return NLCH_OK;
}

}  // namespace

extern "C" int nlch_step_noalloc(const nlch_model *model, int32_t precision, int32_t algo,
                                 const void *u_in, void *u_out, double *ooi_out,
                                 void *hip_stream) {
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
    if (model->beta2 > 0.0)
        return fail(NLCH_EUNSUPPORTED, "nlch_step_noalloc is built for beta2 = 0 (the beta2 > 0 "
                    "step needs a workspace of 7 n^2 doubles)");
    nlch_sample smp;
    std::memset(&smp, 0, sizeof(smp));
    smp.c_F = model->c_F;
    smp.kernel_amp = model->kernel_amp;
    Coef c;
    rc = sample_coef(*model, mi, smp.c_F, smp.kernel_amp, c, "model");
    if (rc) return rc;
    const bool acc64 = (algo & NLCH_ALGO_ACC64) != 0 || precision == kF64;
    int variant = 0;
    rc = choose_variant(algo & 0xff, precision, acc64, mi, *model, false, &variant);
    if (rc) return rc;

    // Layout and size check before any device work.
    const size_t ne2 = (size_t)(mi.m + 1) * (mi.m + 1);
    const bool direct = variant == kDirect;
    const size_t off_ewd = kOffTables;
    const size_t off_ewf = align256(off_ewd + (direct ? ne2 * sizeof(double) : 0));
    const size_t off_part = align256(off_ewf + (direct ? ne2 * sizeof(float) : 0));
    const size_t need = off_part + (ooi_out ? (size_t)ooi_chunks(model->n) * sizeof(double) : 0);
    if (need > kScratchBytes)
        return fail(NLCH_EUNSUPPORTED, "nlch_step_noalloc needs %zu bytes of device scratch for "
                    "this lattice and horizon; its static area holds %zu (an %d x %d lattice "
                    "with the output of interest needs %zu bytes of chunk sums)",
                    need, kScratchBytes, model->n, model->n,
                    (size_t)ooi_chunks(model->n) * sizeof(double));
    const size_t bytes = prec_size(precision) * (size_t)mi.side * mi.side;
    const char *pi = (const char *)u_in, *po = (const char *)u_out;
    if (pi < po + bytes && po < pi + bytes)
        return fail(NLCH_EINVAL, "u_in and u_out overlap (the stencil reads neighbours)");

    void *area = nullptr;
    rc = scratch_address(&area);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;

    // Table image: geometry, descriptor, sample index 0, direct weights.
    const size_t img_bytes = direct ? off_ewf + ne2 * sizeof(float) : kOffTables;
    std::vector<uint32_t> img((img_bytes + 3) / 4, 0u);
    unsigned char *ib = reinterpret_cast<unsigned char *>(img.data());
    ModelGeo gm;
    fill_model_geo(*model, mi, 0, gm);
    std::memcpy(ib + kOffGeo, &gm, sizeof(gm));
    SampleDesc d;
    fill_sample_desc(*model, mi, smp, c, d);
    std::memcpy(ib + kOffDesc, &d, sizeof(d));
    const int32_t id0 = 0;
    std::memcpy(ib + kOffIds, &id0, sizeof(id0));
    if (direct) {
        for (size_t k = 0; k < ne2; ++k) {
            const double e = mi.e2[k];
            const float f = (float)e;
            std::memcpy(ib + off_ewd + k * sizeof(double), &e, sizeof(e));
            std::memcpy(ib + off_ewf + k * sizeof(float), &f, sizeof(f));
        }
    }
    rc = fill_area(area, img, s);
    if (rc) return rc;

    unsigned char *ab = reinterpret_cast<unsigned char *>(area);
    Group g = make_group(*model, mi, 0, 1, precision);
    g.geo = reinterpret_cast<const ModelGeo *>(ab + kOffGeo);
    g.sd = reinterpret_cast<const SampleDesc *>(ab + kOffDesc);
    g.ids = reinterpret_cast<const int32_t *>(ab + kOffIds);
    g.ewd = reinterpret_cast<const double *>(ab + off_ewd);
    g.ewf = reinterpret_cast<const float *>(ab + off_ewf);
    g.partial = reinterpret_cast<double *>(ab + off_part);
    g.ws = nullptr;
    set_default_shape(g);  // as nlch_step
    // the step writes the updated block only; the fixed ring is carried over
    if (g.lo != 0) HIP_TRY(launch_project(precision, g, u_in, u_out, s));
    if (direct)
        HIP_TRY(launch_direct_step(precision, acc64, g, u_in, u_out, s));
    else
        HIP_TRY(launch_rowrun_step(precision, acc64, g, u_in, u_out, s));
    if (ooi_out) HIP_TRY(launch_ooi(precision, g, u_out, ooi_out, 2, s));
    return NLCH_OK;
}
