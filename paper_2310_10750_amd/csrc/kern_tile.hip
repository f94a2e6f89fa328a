// Tiled one-step kernel for lattices with few samples (a single
// high-fidelity sample of 512^2, say), where the streaming kernels' per-wave
// row walks leave most of the chip idle.
//
// A workgroup owns a TY x TX tile of outputs and stages the tile with its
// m-wide periodic halo, (TY + 2m) x (TX + 2m) values, in LDS.  Pass 1 forms
// the window sums of every staged row for every output column of the tile,
// growing H_k = H_{k-1} + g(k) (u(x-k) + u(x+k)) as row_windows does, and
// keeps H at each half-width that the disc uses (w(dy) for some dy) in an
// LDS plane per half-width.  Pass 2 sums, for each output, g(|dy|) H_{w(dy)}
// of the 2m + 1 rows y + dy in row order, and updates and projects the site.
// The window sums and the order in which each output adds them are those of
// the streaming kernel, so both kernels give bit-identical states.  Every
// output row's work is independent, so a 512^2 lattice gives 256 workgroups
// of 4 waves instead of one row walk per wave.
#include "kern_rowrun_impl.h"

namespace nlch {

namespace {

constexpr int kTileX = 32, kTileY = 32, kTileThreads = 512;

// Half-widths the disc uses, in increasing order, and the plane of each.
template <int R2>
struct TileClasses {
    static constexpr int M = Disc<R2>::M;
    static constexpr bool used(int k) {
        for (int dy = 0; dy <= M; ++dy)
            if (Disc<R2>::w(dy) == k) return true;
        return false;
    }
    static constexpr int count() {
        int c = 0;
        for (int k = 0; k <= M; ++k) c += used(k) ? 1 : 0;
        return c;
    }
    static constexpr CArr<int, M + 1> make_plane() {
        CArr<int, M + 1> a{};
        int c = 0;
        for (int k = 0; k <= M; ++k) a.v[k] = used(k) ? c++ : -1;
        return a;
    }
    static constexpr int NC = count();
    static constexpr CArr<int, M + 1> plane = make_plane();
};

template <int R2>
constexpr size_t tile_lds_bytes() {
    constexpr int M = Disc<R2>::M;
    constexpr int TXH = kTileX + 2 * M, TYH = kTileY + 2 * M;
    constexpr int US = (TXH + 3) & ~3;  // staged row stride (16-byte rows)
    return (size_t)TYH * US * 4 + (size_t)TileClasses<R2>::NC * TYH * kTileX * 4;
}

template <int R2, class TS, bool GAUSS>
__global__ __launch_bounds__(kTileThreads) void k_tile(
    const SampleDesc *__restrict__ sd, const int32_t *__restrict__ ids,
    const ModelGeo *__restrict__ geo, const TS *__restrict__ in, TS *__restrict__ out,
    int tiles_x, int tiles_per_sample, int nblocks) {
    using C = TileClasses<R2>;
    constexpr int M = Disc<R2>::M, NC = C::NC;
    constexpr int TXH = kTileX + 2 * M, TYH = kTileY + 2 * M;
    constexpr int US = (TXH + 3) & ~3;
    constexpr int WIN4 = (2 * M + 4 + 3) / 4;  // 16-byte loads of a 4-column window
    static_assert(US % 4 == 0 && 4 * (kTileX / 4 - 1) + 4 * WIN4 <= US, "windows stay in a row");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *ut = reinterpret_cast<float *>(smem_raw);  // TYH x US staged values
    float *hs = ut + TYH * US;                        // NC planes of TYH x TX sums

    const int n = geo->n;
    const int lo = geo->lo, ne = n - geo->lo;  // updated block [lo, ne)^2
    const int b = xcd_remap(blockIdx.x, nblocks);
    const SampleDesc d = sd[ids[b / tiles_per_sample]];
    const int t = b % tiles_per_sample;
    const int x0 = lo + (t % tiles_x) * kTileX, y0 = lo + (t / tiles_x) * kTileY;
    const TS *src = in + d.offset;
    TS *dst = out + d.offset;

    // Stage the tile and its halo (periodic indices of the stored array;
    // under a volume constraint the halo is the ring, which lies inside it).
    // Where a 4-column chunk never straddles the wrap (the tile's first
    // staged column and n are multiples of 4, as for FP32 lattices of a
    // multiple of 4 with m a multiple of 4, and a 16-byte aligned sample)
    // every thread stages whole chunks with 16-byte loads; otherwise element
    // by element.
    if (sizeof(TS) == 4 && (M % 4) == 0 && (n % 4) == 0 && ((x0 - M) % 4 + 4) % 4 == 0 &&
        n >= TYH && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
        constexpr int CH = TXH / 4;  // chunks per staged row
        for (int i = threadIdx.x; i < TYH * CH; i += kTileThreads) {
            const int r = i / CH, c = i - r * CH;
            int gy = y0 - M + r, gx = x0 - M + 4 * c;
            gy += gy < 0 ? n : 0;
            gy -= gy >= n ? n : 0;
            gx += gx < 0 ? n : 0;
            gx -= gx >= n ? n : 0;
            const float4 v = *reinterpret_cast<const float4 *>(
                reinterpret_cast<const float *>(src) + (int64_t)gy * n + gx);
            *reinterpret_cast<float4 *>(ut + r * US + 4 * c) = v;
        }
    } else {
        for (int i = threadIdx.x; i < TYH * TXH; i += kTileThreads) {
            const int r = i / TXH, c = i - r * TXH;
            // (a lattice smaller than the tile wraps more than once)
            const int gy = ((y0 - M + r) % n + n) % n, gx = ((x0 - M + c) % n + n) % n;
            ut[r * US + c] = to_acc<float>(src[(int64_t)gy * n + gx]);
        }
    }
    float g[M + 1];
#pragma unroll
    for (int k = 0; k <= M; ++k) g[k] = GAUSS ? geo_g<float>(geo, k) : 1.0f;
    __syncthreads();

    // Pass 1: window sums of staged row r for output columns 4 xg .. 4 xg + 3.
    for (int task = threadIdx.x; task < TYH * (kTileX / 4); task += kTileThreads) {
        const int r = task / (kTileX / 4), xg = task - r * (kTileX / 4);
        const float *rp = ut + r * US + 4 * xg;
        float win[4 * WIN4];
#pragma unroll
        for (int j = 0; j < WIN4; ++j) {
            const float4 v = reinterpret_cast<const float4 *>(rp)[j];
            win[4 * j] = v.x;
            win[4 * j + 1] = v.y;
            win[4 * j + 2] = v.z;
            win[4 * j + 3] = v.w;
        }
        float H[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) H[c] = GAUSS ? g[0] * win[c + M] : win[c + M];
        sfor<0, M + 1>([&](auto K) {
            constexpr int k = K;
            if constexpr (k > 0) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float pair = win[c + M - k] + win[c + M + k];
                    H[c] = GAUSS ? madd(g[k], pair, H[c]) : (H[c] + pair);
                }
            }
            if constexpr (C::plane[k] >= 0) {
                *reinterpret_cast<float4 *>(hs + ((size_t)C::plane[k] * TYH + r) * kTileX +
                                            4 * xg) = make_float4(H[0], H[1], H[2], H[3]);
            }
        });
    }
    __syncthreads();

    // Pass 2: output row y (tile-relative), columns 2 xg .. 2 xg + 1: the
    // disc rows in row order, as the streaming kernel adds them.
    const float ap = coef_ap<float>(d), bcoef = coef_b<float>(d);
    for (int task = threadIdx.x; task < kTileY * (kTileX / 2); task += kTileThreads) {
        const int y = task / (kTileX / 2), xg = task - y * (kTileX / 2);
        float acc[2] = {-0.0f, -0.0f};
        sfor<0, 2 * M + 1>([&](auto E) {
            constexpr int dy = (int)E - M;
            constexpr int p = C::plane[Disc<R2>::w(dy < 0 ? -dy : dy)];
            const float2 v = *reinterpret_cast<const float2 *>(
                hs + ((size_t)p * TYH + y + M + dy) * kTileX + 2 * xg);
            const float hv[2] = {v.x, v.y};
#pragma unroll
            for (int c = 0; c < 2; ++c)
                acc[c] = GAUSS ? madd(g[dy < 0 ? -dy : dy], hv[c], acc[c]) : (acc[c] + hv[c]);
        });
        const int gy = y0 + y;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int gx = x0 + 2 * xg + c;
            const float u = ut[(y + M) * US + M + 2 * xg + c];
            if (gy < ne && gx < ne)
                dst[(int64_t)gy * n + gx] = to_store<TS>(update_g<float>(u, acc[c], ap, bcoef));
        }
    }
}

template <int R2, class TS, bool GAUSS>
hipError_t tile_go(const Group &g, const void *in, void *out, hipStream_t s) {
    const int tx = (g.ni + kTileX - 1) / kTileX, ty = (g.ni + kTileY - 1) / kTileY;
    const int64_t nb = (int64_t)tx * ty * g.nids;
    constexpr size_t lds = tile_lds_bytes<R2>();
    if (nb > 0x7fffffff || lds > 159 * 1024) return hipErrorInvalidValue;
    auto f = k_tile<R2, TS, GAUSS>;
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3((unsigned)nb), dim3(kTileThreads), lds, s, g.sd, g.ids, g.geo,
                       (const TS *)in, (TS *)out, tx, tx * ty, (int)nb);
    return hipGetLastError();
}

}  // namespace

// Discs with a tiled kernel (m <= 16: the planes of window sums fit in LDS).
#define NLCH_TILE_R2_LIST(X) \
    X(1) X(4) X(9) X(16) X(25) X(64) X(121) X(144) X(256) X(272)

bool tile_supported(int prec, bool acc64, int R2) {
    if (prec == kF64 || acc64) return false;
#define NLCH_X(v) \
    if (R2 == v) return true;
    NLCH_TILE_R2_LIST(NLCH_X)
#undef NLCH_X
    return false;
}

int tile_blocks_per_sample(int ni) {
    return ((ni + kTileX - 1) / kTileX) * ((ni + kTileY - 1) / kTileY);
}

hipError_t launch_tile_step(int prec, const Group &g, const void *in, void *out,
                            hipStream_t s) {
#define NLCH_X(v)                                                                     \
    if (g.R2 == v) {                                                                  \
        if (prec == kF32)                                                             \
            return g.kernel == 1 ? tile_go<v, float, true>(g, in, out, s)             \
                                 : tile_go<v, float, false>(g, in, out, s);           \
        return g.kernel == 1 ? tile_go<v, half_t, true>(g, in, out, s)                \
                             : tile_go<v, half_t, false>(g, in, out, s);              \
    }
    if (prec != kF64) {
        NLCH_TILE_R2_LIST(NLCH_X)
    }
#undef NLCH_X
    return hipErrorInvalidValue;
}

}  // namespace nlch
