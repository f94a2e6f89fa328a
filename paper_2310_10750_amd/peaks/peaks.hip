// Measured peaks of one MI355X (gfx950) for the rooflines of the library's
// kernels: HBM copy bandwidth, LDS read bandwidth, and the issue rates of
// FP32 add / FMA and FP64 FMA.  Built with packed-FP32 instructions disabled,
// like the library, so the FP32 rates are those its kernels can reach.
// Prints one line per measurement (best of five launches) and a JSON line.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                               \
    do {                                                                       \
        hipError_t e_ = (x);                                                   \
        if (e_ != hipSuccess) {                                                \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
            exit(1);                                                           \
        }                                                                      \
    } while (0)

namespace {

// HBM: a copy of n4 16-byte elements, one per thread (each read and written
// once; of the copy shapes tried, one element per thread and a grid that
// covers the array was the fastest).
__global__ __launch_bounds__(256) void k_copy(const float4 *__restrict__ src,
                                              float4 *__restrict__ dst, long n4) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) dst[i] = src[i];
}

// LDS: lane-contiguous W-byte reads (W = 8 or 16) of a 64 KB buffer, no bank
// conflicts; the index is masked into the buffer.
template <int W>
__global__ __launch_bounds__(256) void k_lds(float *out, int iters) {
    __shared__ __align__(16) float buf[16384];
    for (int i = threadIdx.x; i < 16384; i += 256) buf[i] = 1e-7f * (float)(i & 31);
    __syncthreads();
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int base = ((it * 8 + r) * 256 * (W / 4) + (int)threadIdx.x * (W / 4)) & (16384 - W / 4);
            if constexpr (W == 8) {
                const float2 v = *reinterpret_cast<const float2 *>(buf + base);
                s0 += v.x;
                s1 += v.y;
            } else {
                const float4 v = *reinterpret_cast<const float4 *>(buf + base);
                s0 += v.x;
                s1 += v.y;
                s2 += v.z;
                s3 += v.w;
            }
        }
    }
    out[blockIdx.x * 256 + threadIdx.x] = s0 + s1 + s2 + s3;
}

// VALU: 8 independent chains per lane of OP (0 = FP32 add, 1 = FP32 FMA,
// 2 = FP64 FMA), 32 operations per chain and iteration, no memory in the loop.
template <int OP, class T>
__global__ __launch_bounds__(256) void k_valu(const T *in, T *out, int iters) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    T a[8], b[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        a[j] = in[(t + j) & 1023];
        b[j] = in[(t * 3 + j) & 1023];
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if constexpr (OP == 0)
                    a[j] = a[j] + b[j];
                else if constexpr (sizeof(T) == 4)
                    a[j] = __builtin_fmaf(a[j], b[(j + 1) & 7], b[j]);
                else
                    a[j] = __builtin_fma(a[j], b[(j + 1) & 7], b[j]);
            }
    }
    T s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += a[j];
    out[t] = s;
}

template <class F>
float best_ms(F launch) {
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    launch();  // warm-up
    CHECK(hipGetLastError());
    float best = 1e30f;
    for (int rep = 0; rep < 5; ++rep) {
        CHECK(hipEventRecord(e0, 0));
        launch();
        CHECK(hipEventRecord(e1, 0));
        CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) best = ms;
    }
    CHECK(hipGetLastError());
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return best;
}

}  // namespace

int main() {
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    printf("device %s, %d CUs\n", prop.gcnArchName, cus);

    // HBM copy: 1 GiB read, 1 GiB written per launch
    const long n4 = (1L << 30) / 16;
    float4 *src = nullptr, *dst = nullptr;
    CHECK(hipMalloc(&src, n4 * 16));
    CHECK(hipMalloc(&dst, n4 * 16));
    CHECK(hipMemset(src, 0, n4 * 16));
    const float ms_copy = best_ms([&] {
        hipLaunchKernelGGL(k_copy, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, 0, src, dst, n4);
    });
    const double hbm = 2.0 * n4 * 16 / (ms_copy * 1e-3) / 1e12;
    printf("hbm copy: %.3f ms, %.2f TB/s (read + write)\n", ms_copy, hbm);
    CHECK(hipFree(src));
    CHECK(hipFree(dst));

    // LDS reads: 8 workgroups of 4 waves per CU
    const int lblocks = cus * 8, liters = 2048;
    float *lout = nullptr;
    CHECK(hipMalloc(&lout, (size_t)lblocks * 256 * sizeof(float)));
    double lds[2];
    for (int w = 0; w < 2; ++w) {
        const float ms = best_ms([&] {
            if (w == 0)
                hipLaunchKernelGGL(k_lds<8>, dim3(lblocks), dim3(256), 0, 0, lout, liters);
            else
                hipLaunchKernelGGL(k_lds<16>, dim3(lblocks), dim3(256), 0, 0, lout, liters);
        });
        const double bytes = (double)lblocks * 256 * liters * 8 * (w ? 16 : 8);
        lds[w] = bytes / (ms * 1e-3) / 1e12;
        printf("lds read %d B/lane: %.3f ms, %.1f TB/s (%.1f B/clock/CU at 2.4 GHz)\n", w ? 16 : 8,
               ms, lds[w], bytes / (ms * 1e-3) / 2.4e9 / cus);
    }
    CHECK(hipFree(lout));

    // VALU issue rates: 32 workgroups of 4 waves per CU
    const int vblocks = cus * 32, viters = 4096, nthr = vblocks * 256;
    float *fin = nullptr, *fout = nullptr;
    double *din = nullptr, *dout = nullptr;
    CHECK(hipMalloc(&fin, 1024 * sizeof(float)));
    CHECK(hipMalloc(&fout, (size_t)nthr * sizeof(float)));
    CHECK(hipMalloc(&din, 1024 * sizeof(double)));
    CHECK(hipMalloc(&dout, (size_t)nthr * sizeof(double)));
    {
        float hf[1024];
        double hd[1024];
        for (int i = 0; i < 1024; ++i) {
            hf[i] = 1e-7f * (float)(i % 17);
            hd[i] = 1e-7 * (double)(i % 17);
        }
        CHECK(hipMemcpy(fin, hf, sizeof(hf), hipMemcpyHostToDevice));
        CHECK(hipMemcpy(din, hd, sizeof(hd), hipMemcpyHostToDevice));
    }
    const double lane_ops = (double)nthr * viters * 32;
    const float ms_add = best_ms([&] {
        hipLaunchKernelGGL((k_valu<0, float>), dim3(vblocks), dim3(256), 0, 0, fin, fout, viters);
    });
    const float ms_fma = best_ms([&] {
        hipLaunchKernelGGL((k_valu<1, float>), dim3(vblocks), dim3(256), 0, 0, fin, fout, viters);
    });
    const float ms_d = best_ms([&] {
        hipLaunchKernelGGL((k_valu<1, double>), dim3(vblocks), dim3(256), 0, 0, din, dout, viters);
    });
    const double add = lane_ops / (ms_add * 1e-3) / 1e12, fma = lane_ops / (ms_fma * 1e-3) / 1e12,
                 dfma = lane_ops / (ms_d * 1e-3) / 1e12;
    printf("fp32 add: %.3f ms, %.2f T lane-ops/s\n", ms_add, add);
    printf("fp32 fma: %.3f ms, %.2f T lane-ops/s (%.1f TFLOP/s)\n", ms_fma, fma, 2 * fma);
    printf("fp64 fma: %.3f ms, %.2f T lane-ops/s (%.1f TFLOP/s)\n", ms_d, dfma, 2 * dfma);
    CHECK(hipFree(fin));
    CHECK(hipFree(fout));
    CHECK(hipFree(din));
    CHECK(hipFree(dout));
    printf("{\"hbm_copy_tbs\": %.3f, \"lds_read_b64_tbs\": %.2f, \"lds_read_b128_tbs\": %.2f, "
           "\"fp32_add_tops\": %.2f, \"fp32_fma_tops\": %.2f, \"fp64_fma_tops\": %.2f, \"cus\": %d}\n",
           hbm, lds[0], lds[1], add, fma, dfma, cus);
    return 0;
}
