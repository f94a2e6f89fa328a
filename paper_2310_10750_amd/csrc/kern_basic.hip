// Elementwise and reduction kernels, and the per-site ("direct") disc-sum step.
//
//  * k_project: u^0 = clamp(u0, -1, 1), the projection of the initial datum
//    onto the admissible set [-1, 1] (obstacle potential, Sec. 2).
//  * k_count_nonfinite: optional validation of u0.
//  * k_ooi: per-sample FP64 sum -> mean and f_1 = (1 + mean)/2 (eq. ooi).
//  * k_direct: one step, every site summing over the whole horizon disc in
//    difference form  Lsum = sum_{d != 0} e_d (u_i - u_{i+d})  (eq.
//    nonl_operator with nodal quadrature), then the projected update.  Halo
//    tile staged in LDS; any horizon up to kMaxM.
//  * k_energy_final: per sample, the step kernels' workgroup partial sums of
//    sum u Lsum and sum (1 - u^2) in workgroup order -> the discrete energy
//    E_h(u) = h^2 [ 1/2 sum_i u_i L_i + c_F/2 sum_i (1 - u_i^2) ] (the energy of
//    Sec. 2 with the nonlocal interaction; 1/4 sum_i sum_d w_d (u_i - u_{i+d})^2
//    equals 1/2 sum_i u_i L_i on the torus because the disc is symmetric).
#include "nlch_device.h"

namespace nlch {

namespace {

constexpr int kElemThreads = 256;
constexpr int kElemItems = 8;
constexpr int64_t kOoiChunk = 16384;

template <class TS>
__global__ __launch_bounds__(kElemThreads) void k_project(
    const SampleDesc *__restrict__ sd, const int32_t *__restrict__ ids,
    int64_t nn, int chunks, const TS *src, TS *dst) {
    const int b = blockIdx.x;
    const SampleDesc d = sd[ids[b / chunks]];
    const int64_t chunk = (int64_t)kElemThreads * kElemItems;
    const int64_t lo = (int64_t)(b % chunks) * chunk;
    const int64_t hi = lo + chunk < nn ? lo + chunk : nn;
    const TS *s = src + d.offset;
    TS *o = dst + d.offset;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kElemThreads) {
        TS v = s[i];
        o[i] = v < TS(-1) ? TS(-1) : (v > TS(1) ? TS(1) : v);
    }
}

template <class TS>
__global__ __launch_bounds__(kElemThreads) void k_count_nonfinite(
    const SampleDesc *__restrict__ sd, const int32_t *__restrict__ ids,
    int64_t nn, int chunks, const TS *__restrict__ src,
    unsigned int *__restrict__ counter) {
    const int b = blockIdx.x;
    const SampleDesc d = sd[ids[b / chunks]];
    const int64_t chunk = (int64_t)kElemThreads * kElemItems;
    const int64_t lo = (int64_t)(b % chunks) * chunk;
    const int64_t hi = lo + chunk < nn ? lo + chunk : nn;
    const TS *s = src + d.offset;
    unsigned int bad = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kElemThreads) {
        double v = (double)s[i];
        bad += (v - v != 0.0) ? 1u : 0u;  // NaN or +-inf
    }
    if (bad) atomicAdd(counter, bad);
}

// Output of interest, pass 1: FP64 partial sums of fixed chunks of every
// sample's state (one workgroup per chunk).  The sum runs over the ni x ni
// block that starts at row and column `ring` of the side x side array: the
// whole state on the torus (ring = 0, ni = side), the lattice of Omega
// without the fixed ring under a volume constraint.
template <class TS>
__global__ __launch_bounds__(256) void k_ooi_partial(const SampleDesc *__restrict__ sd,
                                                     const int32_t *__restrict__ ids,
                                                     int64_t nn, int chunks, int ni,
                                                     int side, int ring,
                                                     const TS *__restrict__ st,
                                                     double *__restrict__ partial) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    const SampleDesc d = sd[ids[b / chunks]];
    const int64_t lo = (int64_t)(b % chunks) * kOoiChunk;
    const int64_t hi = lo + kOoiChunk < nn ? lo + kOoiChunk : nn;
    const TS *s = st + d.offset;
    double acc = 0.0;
    if (ring == 0) {
        for (int64_t i = lo + threadIdx.x; i < hi; i += 256) acc += (double)s[i];
    } else {
        for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
            const int64_t y = i / ni, x = i - y * ni;
            acc += (double)s[(y + ring) * side + x + ring];
        }
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) partial[b] = tot;
}

// Pass 2: per sample, the chunk sums in chunk order -> mean and
// f_1 = (1 + mean)/2 (eq. ooi).
__global__ __launch_bounds__(64) void k_ooi_final(const int32_t *__restrict__ ids, int64_t nn,
                                                  int chunks,
                                                  const double *__restrict__ partial,
                                                  double *__restrict__ ooi) {
    const int j = blockIdx.x;
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += partial[(int64_t)j * chunks + c];
    const double mean = s / (double)nn;
    const int64_t sidx = ids[j];
    ooi[2 * sidx] = mean;
    ooi[2 * sidx + 1] = 0.5 * (1.0 + mean);
}

constexpr int kDirThreads = 256;

template <class TS, class TA, bool GAUSS>
__global__ __launch_bounds__(kDirThreads) void k_direct(
    const SampleDesc *__restrict__ sd, const int32_t *__restrict__ ids,
    const ModelGeo *__restrict__ geo, const TA *__restrict__ ew,
    const TS *__restrict__ in, TS *__restrict__ out, int tiles_x,
    int tiles_per_sample, int nblocks, double *__restrict__ epart) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[kDirThreads / 64];
    TA *tile = reinterpret_cast<TA *>(smem_raw);
    const int n = geo->n, m = geo->m;
    const int ne = n - geo->lo;  // updated block [lo, ne)^2 (see ModelGeo)
    const int b = xcd_remap(blockIdx.x, nblocks);
    const SampleDesc d = sd[ids[b / tiles_per_sample]];
    const int t = b % tiles_per_sample;
    const int x0 = geo->lo + (t % tiles_x) * kDirTX, y0 = geo->lo + (t / tiles_x) * kDirTY;
    const TS *src = in + d.offset;
    TS *dst = out + d.offset;
    const int W = kDirTX + 2 * m, H = kDirTY + 2 * m;

    for (int i = threadIdx.x; i < W * H; i += kDirThreads) {
        const int r = i / W, c = i - r * W;
        int gy = (y0 - m + r) % n;
        gy += gy < 0 ? n : 0;
        int gx = (x0 - m + c) % n;
        gx += gx < 0 ? n : 0;
        tile[i] = to_acc<TA>(src[(int64_t)gy * n + gx]);
    }
    __syncthreads();

    const TA a = coef_a<TA>(d), bb = coef_b<TA>(d);
    const TA *ewm = ew + geo->e_off;
    const int lx = threadIdx.x & 63;
    double e_ul = 0.0, e_pot = 0.0;
    for (int ly = threadIdx.x >> 6; ly < kDirTY; ly += kDirThreads / 64) {
        const int y = y0 + ly, x = x0 + lx;
        const TA *cen = tile + (ly + m) * W + lx + m;
        const TA uc = *cen;
        TA acc = TA(0);
        for (int dy = -m; dy <= m; ++dy) {
            const int ady = dy < 0 ? -dy : dy;
            const int w = geo->halfw[ady];
            const TA *row = cen + dy * W;
            for (int dx = -w; dx <= w; ++dx) {
                const TA diff = uc - row[dx];
                if (GAUSS) {
                    const int adx = dx < 0 ? -dx : dx;
                    acc = madd(ewm[ady * (m + 1) + adx], diff, acc);
                } else {
                    acc += diff;
                }
            }
        }
        if (y < ne && x < ne) {
            dst[(int64_t)y * n + x] = to_store<TS>(update<TA>(uc, acc, a, bb));
            e_ul += (double)uc * (double)acc;
            e_pot += 1.0 - (double)uc * (double)uc;
        }
    }
    if (epart) {
        e_ul = block_sum(e_ul, red);
        e_pot = block_sum(e_pot, red);
        if (threadIdx.x == 0) {
            epart[2 * (int64_t)b] = e_ul;
            epart[2 * (int64_t)b + 1] = e_pot;
        }
    }
}

// One wave per sample of the group: lane l sums partials l, l + 64, ... in
// order, then a fixed shuffle tree (the result does not depend on timing).
__global__ __launch_bounds__(64) void k_energy_final(const SampleDesc *__restrict__ sd,
                                                     const int32_t *__restrict__ ids,
                                                     int per_sample,
                                                     const double *__restrict__ epart,
                                                     double *__restrict__ energy) {
    const int j = blockIdx.x;
    const double *p = epart + 2 * (int64_t)j * per_sample;
    double s_ul = 0.0, s_pot = 0.0;
    for (int i = threadIdx.x; i < per_sample; i += 64) {
        s_ul += p[2 * i];
        s_pot += p[2 * i + 1];
    }
    for (int o = 32; o > 0; o >>= 1) {
        s_ul += __shfl_xor(s_ul, o, 64);
        s_pot += __shfl_xor(s_pot, o, 64);
    }
    if (threadIdx.x == 0) {
        const int64_t sidx = ids[j];
        const SampleDesc d = sd[sidx];
        energy[sidx] = d.e_int * s_ul + d.e_pot * s_pot;
    }
}

template <class TS>
inline int chunks_for(int64_t nn) {
    const int64_t chunk = (int64_t)kElemThreads * kElemItems;
    return (int)((nn + chunk - 1) / chunk);
}

}  // namespace

hipError_t launch_project(int prec, const Group &g, const void *src, void *dst,
                          hipStream_t s) {
    const int64_t nn = (int64_t)g.n * g.n;
    const int ch = chunks_for<float>(nn);
    dim3 grid((unsigned)(ch * g.nids)), block(kElemThreads);
    switch (prec) {
        case kF64:
            hipLaunchKernelGGL((k_project<double>), grid, block, 0, s, g.sd, g.ids, nn, ch,
                               (const double *)src, (double *)dst);
            break;
        case kF32:
            hipLaunchKernelGGL((k_project<float>), grid, block, 0, s, g.sd, g.ids, nn, ch,
                               (const float *)src, (float *)dst);
            break;
        default:
            hipLaunchKernelGGL((k_project<half_t>), grid, block, 0, s, g.sd, g.ids, nn, ch,
                               (const half_t *)src, (half_t *)dst);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(int prec, const Group &g, const void *src,
                                  unsigned int *counter, hipStream_t s) {
    const int64_t nn = (int64_t)g.n * g.n;
    const int ch = chunks_for<float>(nn);
    dim3 grid((unsigned)(ch * g.nids)), block(kElemThreads);
    switch (prec) {
        case kF64:
            hipLaunchKernelGGL((k_count_nonfinite<double>), grid, block, 0, s, g.sd, g.ids, nn,
                               ch, (const double *)src, counter);
            break;
        case kF32:
            hipLaunchKernelGGL((k_count_nonfinite<float>), grid, block, 0, s, g.sd, g.ids, nn,
                               ch, (const float *)src, counter);
            break;
        default:
            hipLaunchKernelGGL((k_count_nonfinite<half_t>), grid, block, 0, s, g.sd, g.ids, nn,
                               ch, (const half_t *)src, counter);
            break;
    }
    return hipGetLastError();
}

int ooi_chunks(int n) { return (int)(((int64_t)n * n + kOoiChunk - 1) / kOoiChunk); }

hipError_t launch_ooi(int prec, const Group &g, const void *state, double *ooi, int,
                      hipStream_t s) {
    const int64_t nn = (int64_t)g.ni * g.ni;
    const int ch = ooi_chunks(g.ni);
    dim3 grid((unsigned)(ch * g.nids)), block(256);
    switch (prec) {
        case kF64:
            hipLaunchKernelGGL((k_ooi_partial<double>), grid, block, 0, s, g.sd, g.ids, nn, ch,
                               g.ni, g.n, g.lo, (const double *)state, g.partial);
            break;
        case kF32:
            hipLaunchKernelGGL((k_ooi_partial<float>), grid, block, 0, s, g.sd, g.ids, nn, ch,
                               g.ni, g.n, g.lo, (const float *)state, g.partial);
            break;
        default:
            hipLaunchKernelGGL((k_ooi_partial<half_t>), grid, block, 0, s, g.sd, g.ids, nn, ch,
                               g.ni, g.n, g.lo, (const half_t *)state, g.partial);
            break;
    }
    hipLaunchKernelGGL(k_ooi_final, dim3((unsigned)g.nids), dim3(64), 0, s, g.ids, nn, ch,
                       g.partial, ooi);
    return hipGetLastError();
}

template <class TA>
static const TA *ew_for(const Group &g);
template <>
const float *ew_for<float>(const Group &g) { return g.ewf; }
template <>
const double *ew_for<double>(const Group &g) { return g.ewd; }

template <class TS, class TA>
static hipError_t direct_typed(const Group &g, const void *in, void *out, hipStream_t s,
                               double *epart) {
    const int tiles_x = (g.ni + kDirTX - 1) / kDirTX;
    const int tiles_y = (g.ni + kDirTY - 1) / kDirTY;
    const int tps = tiles_x * tiles_y;
    const int64_t nb = (int64_t)tps * g.nids;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    const size_t lds = sizeof(TA) * (size_t)(kDirTX + 2 * g.m) * (kDirTY + 2 * g.m);
    dim3 grid((unsigned)nb), block(kDirThreads);
    if (g.kernel == 1) {
        auto f = k_direct<TS, TA, true>;
        if (lds > 64 * 1024 &&
            hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) != hipSuccess)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(f, grid, block, lds, s, g.sd, g.ids, g.geo, ew_for<TA>(g),
                           (const TS *)in, (TS *)out, tiles_x, tps, (int)nb, epart);
    } else {
        auto f = k_direct<TS, TA, false>;
        if (lds > 64 * 1024 &&
            hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) != hipSuccess)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(f, grid, block, lds, s, g.sd, g.ids, g.geo, ew_for<TA>(g),
                           (const TS *)in, (TS *)out, tiles_x, tps, (int)nb, epart);
    }
    return hipGetLastError();
}

hipError_t launch_direct_step(int prec, bool acc64, const Group &g, const void *in,
                              void *out, hipStream_t s, double *epart) {
    switch (prec) {
        case kF64:
            return direct_typed<double, double>(g, in, out, s, epart);
        case kF32:
            return acc64 ? direct_typed<float, double>(g, in, out, s, epart)
                         : direct_typed<float, float>(g, in, out, s, epart);
        default:
            return acc64 ? direct_typed<half_t, double>(g, in, out, s, epart)
                         : direct_typed<half_t, float>(g, in, out, s, epart);
    }
}

hipError_t launch_energy_final(const Group &g, const double *epart, int per_sample,
                               double *energy, hipStream_t s) {
    if (per_sample < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_energy_final, dim3((unsigned)g.nids), dim3(64), 0, s, g.sd, g.ids,
                       per_sample, epart, energy);
    return hipGetLastError();
}

}  // namespace nlch
