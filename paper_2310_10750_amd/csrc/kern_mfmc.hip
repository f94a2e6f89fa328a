// FP64 moment accumulation for the multifidelity Monte Carlo estimator
// (Sec. 3.2): per model j, the Monte Carlo means over its first m_j and first
// m_{j-1} draws (eq. MFMC_estimator), and, over the first m_1 draws that all
// models share, the sample variance and the covariance with model 1 (the
// statistics of eq. alpha).  Two passes (means, then centred sums), fixed
// reduction order.
#include "nlch_device.h"

namespace nlch {

namespace {

struct MomArgs {
    const double *y[8];
    int64_t m[8];
    int64_t stride;
    int K;
};

__global__ __launch_bounds__(256) void k_moments(MomArgs a, double *__restrict__ out) {
    __shared__ double red[4];
    const int j = blockIdx.x;
    const double *yj = a.y[j];
    const double *y1 = a.y[0];
    const int64_t m0 = a.m[0], mj = a.m[j], mjm1 = j > 0 ? a.m[j - 1] : 0;

    double s_mj = 0.0, s_mjm1 = 0.0, s0j = 0.0, s01 = 0.0;
    const int64_t st = a.stride;
    for (int64_t i = threadIdx.x; i < mj; i += 256) {
        const double v = yj[i * st];
        s_mj += v;
        if (i < mjm1) s_mjm1 += v;
        if (i < m0) s0j += v;
    }
    for (int64_t i = threadIdx.x; i < m0; i += 256) s01 += y1[i * st];
    s_mj = block_sum(s_mj, red);
    s_mjm1 = block_sum(s_mjm1, red);
    s0j = block_sum(s0j, red);
    s01 = block_sum(s01, red);
    const double mean0j = s0j / (double)m0, mean01 = s01 / (double)m0;

    double sv = 0.0, sc = 0.0;
    for (int64_t i = threadIdx.x; i < m0; i += 256) {
        const double dj = yj[i * st] - mean0j, d1 = y1[i * st] - mean01;
        sv += dj * dj;
        sc += d1 * dj;
    }
    sv = block_sum(sv, red);
    sc = block_sum(sc, red);
    if (threadIdx.x == 0) {
        double *o = out + 8 * j;
        o[0] = s_mj / (double)mj;
        o[1] = j > 0 ? s_mjm1 / (double)mjm1 : 0.0;
        // one shared draw (below-minimum-budget allocations): no variance
        o[2] = m0 > 1 ? sv / (double)(m0 - 1) : __builtin_nan("");
        o[3] = m0 > 1 ? sc / (double)(m0 - 1) : __builtin_nan("");
        o[4] = mean0j;
    }
}

}  // namespace

hipError_t launch_moments(int K, const double *const *y, const int64_t *m, int64_t stride,
                          double *out, hipStream_t s) {
    MomArgs a{};
    a.stride = stride;
    for (int j = 0; j < K; ++j) {
        a.y[j] = y[j];
        a.m[j] = m[j];
    }
    a.K = K;
    hipLaunchKernelGGL(k_moments, dim3((unsigned)K), dim3(256), 0, s, a, out);
    return hipGetLastError();
}

}  // namespace nlch
