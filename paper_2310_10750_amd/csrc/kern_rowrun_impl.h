// Row-run ("window sum") kernels for the horizon disc, with the disc geometry
// fixed at compile time.
//
// The nodal-quadrature convolution over the disc D (eq. nonl_operator) is
// evaluated per output site (y, x) as a sum over disc rows dy of horizontal
// window sums
//     G(y, x) = sum_{dy=-m}^{m} g(|dy|) H_{w(dy)}(y + dy, x),
//     H_w(r, x) = sum_{|dx| <= w} g(|dx|) u(r, x + dx),   w(dy) = isqrt(R2 - dy^2),
// where g == 1 for the constant kernel and g(k) = exp(-k^2 h^2 / sigma^2) for
// the Gaussian kernel, whose weights factor as g(|dy|) g(|dx|).  The unit
// operator sum of the difference form is then Lsum = ce u - G with
// ce = sum_{d in D} g(|dy|) g(|dx|).  Per site this costs 2m + (2m+1) adds
// (plus m + 2m+1 multiplies for the Gaussian) instead of |D| ~ pi m^2.
//
// A lane owns R adjacent columns and walks down the rows.  Window sums of one
// input row are grown incrementally (H_k = H_{k-1} + g(k) (u(x-k) + u(x+k)))
// and each is added, as soon as it is formed, into every pending output row
// whose disc row has that half-width.  All register indices are compile-time
// constants (template loops), so nothing is demoted to scratch memory.
#pragma once

#include <type_traits>

#include "nlch_device.h"

namespace nlch {

constexpr int cisqrt(int v) {
    int r = 0;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

template <class T, int N>
struct CArr {
    T v[N];
    constexpr T operator[](int i) const { return v[i]; }
};

// Compile-time disc geometry: half-widths, and the disc rows dy grouped by
// half-width (rows whose window sum has width k are dy_by_w[start[k]] ..
// dy_by_w[start[k+1]-1]).
template <int R2>
struct Disc {
    static constexpr int M = cisqrt(R2);
    static constexpr int P = 2 * M + 1;
    static constexpr int w(int ady) { return cisqrt(R2 - ady * ady); }
    static constexpr CArr<int, P> make_dy() {
        CArr<int, P> a{};
        int e = 0;
        for (int k = 0; k <= M; ++k)
            for (int dy = -M; dy <= M; ++dy)
                if (w(dy < 0 ? -dy : dy) == k) a.v[e++] = dy;
        return a;
    }
    static constexpr CArr<int, M + 2> make_start() {
        CArr<int, M + 2> a{};
        int e = 0;
        for (int k = 0; k <= M; ++k) {
            a.v[k] = e;
            for (int dy = -M; dy <= M; ++dy)
                if (w(dy < 0 ? -dy : dy) == k) ++e;
        }
        a.v[M + 1] = e;
        return a;
    }
    static constexpr CArr<int, P> dy_by_w = make_dy();
    static constexpr CArr<int, M + 2> start = make_start();
};

// Loads win[0..WIN) = p[0..WIN) as TA, in pairs when the caller guarantees
// that p is aligned to two elements (halves the LDS instructions and avoids
// the bank conflicts of lane-strided 4-byte reads).
template <int WIN, bool PAIRS, class TS, class TA>
__device__ __forceinline__ void load_window(const TS *p, TA *win) {
    if constexpr (PAIRS && sizeof(TS) >= 4) {
        struct alignas(2 * sizeof(TS)) Pair { TS v[2]; };
        const Pair *pp = reinterpret_cast<const Pair *>(p);
#pragma unroll
        for (int j = 0; j < WIN / 2; ++j) {
            const Pair t = pp[j];
            win[2 * j] = to_acc<TA>(t.v[0]);
            win[2 * j + 1] = to_acc<TA>(t.v[1]);
        }
        if constexpr (WIN % 2) win[WIN - 1] = to_acc<TA>(p[WIN - 1]);
    } else {
#pragma unroll
        for (int j = 0; j < WIN; ++j) win[j] = to_acc<TA>(p[j]);
    }
}

template <int B, int E, class F>
__device__ __forceinline__ void sfor(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

constexpr int cabs(int v) { return v < 0 ? -v : v; }

// Accumulators start at -0.0, the exact identity of IEEE addition (x + -0 is
// x for every x, +0 included), so the first add of each sum folds away.

// Window sums of one input row for column c (window values win[c .. c+2M])
// grown incrementally, each added into the outputs that use its half-width:
// acc(dy) names the accumulator of the output that disc row dy of this input
// row feeds, and receives g(|dy|) * H_{w(dy)} (a fused multiply-add; H for
// the constant kernel).
template <int R2, bool GAUSS, class TA, class Acc>
__device__ __forceinline__ void row_windows(const TA *win, const TA *g, Acc &&acc) {
    using D = Disc<R2>;
    constexpr int M = D::M;
    TA H = GAUSS ? g[0] * win[M] : win[M];
    sfor<0, M + 1>([&](auto K) {
        constexpr int k = K;
        if constexpr (k > 0) {
            const TA pair = win[M - k] + win[M + k];
            H = GAUSS ? madd(g[k], pair, H) : (H + pair);
        }
        sfor<D::start[k], D::start[k + 1]>([&](auto E) {
            constexpr int dy = D::dy_by_w[E];
            TA &r = acc(dy);
            r = GAUSS ? madd(g[cabs(dy)], H, r) : (r + H);
        });
    });
}

// row_windows for C adjacent columns at once (column c's window is
// win[c .. c + 2M]): the columns' window growth and accumulation are
// interleaved, k by k, so that C independent chains are in flight; per column
// the operations and their order are those of row_windows.  acc(dy, c) names
// the accumulator of column c's output fed by disc row dy.
template <int R2, bool GAUSS, int C, class TA, class Acc>
__device__ __forceinline__ void row_windows_cols(const TA *win, const TA *g, Acc &&acc) {
    using D = Disc<R2>;
    constexpr int M = D::M;
    TA H[C];
#pragma unroll
    for (int c = 0; c < C; ++c) H[c] = GAUSS ? g[0] * win[c + M] : win[c + M];
    sfor<0, M + 1>([&](auto K) {
        constexpr int k = K;
        if constexpr (k > 0) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const TA pair = win[c + M - k] + win[c + M + k];
                H[c] = GAUSS ? madd(g[k], pair, H[c]) : (H[c] + pair);
            }
        }
        sfor<D::start[k], D::start[k + 1]>([&](auto E) {
            constexpr int dy = D::dy_by_w[E];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                TA &r = acc(dy, c);
                r = GAUSS ? madd(g[cabs(dy)], H[c], r) : (r + H[c]);
            }
        });
    });
}

// ---------------------------------------------------------------------------
// Streaming step: a workgroup is one wave that owns a strip of 64R columns
// and a band of B output rows of one sample.  It walks the B + 2m input rows
// of its band once: each row segment (its 64R columns plus the m-column
// periodic halo on either side) is fetched with coalesced loads one row
// ahead, staged through a two-row LDS ring private to the wave, turned into
// window sums and added into a register ring of 2m+1 pending output rows.
// A finished row is updated and written straight to the output buffer.
// Occupancy is bounded only by registers, not by shared tiles.
// ---------------------------------------------------------------------------
template <int R2, int R, class TS, class TA, bool GAUSS>
__global__ __launch_bounds__(64) void k_stream(
    const SampleDesc *__restrict__ sd, const int32_t *__restrict__ ids,
    const ModelGeo *__restrict__ geo, const TS *__restrict__ in,
    TS *__restrict__ out, int B, int strips, int bands, int nblocks,
    double *__restrict__ epart) {
    constexpr int M = Disc<R2>::M, P = Disc<R2>::P;
    constexpr int TX = 64 * R;
    constexpr int TW = TX + 2 * M;
    constexpr int WIN = 2 * M + R;
    constexpr int CPL = (TW + 63) / 64;  // row-segment elements per lane
    // the ring holds the arithmetic type: a narrow state is widened once per
    // staged element instead of once per window read; rows are padded to
    // 64 CPL elements so that every lane stores
    __shared__ __align__(16) TA ring[2][64 * CPL];

    const int n = geo->n;
    // updated block: rows and columns [lo, ne) (the whole lattice on the
    // torus; without the ring of fixed values under a volume constraint)
    const int lo = geo->lo, ne = n - geo->lo;
    const int bidx = xcd_remap(blockIdx.x, nblocks);
    const int per_sample = strips * bands;
    const SampleDesc d = sd[ids[bidx / per_sample]];
    const int t = bidx % per_sample;
    const int x0 = lo + (t % strips) * TX;
    const int y0 = lo + (t / strips) * B;
    const TS *src = in + d.offset;
    TS *dst = out + d.offset;
    const int lane = threadIdx.x;
    const int c0 = lane * R;
    const int bq = y0 + B <= ne ? B : ne - y0;  // output rows of this band
    const int rows = bq + 2 * M;

    // wrapped source columns of this lane's staged elements; lanes past the
    // segment end re-read column 0 into the ring's padding
    int gxs[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        int gx = (x0 - M + lane + 64 * k) % n;
        gx += gx < 0 ? n : 0;
        gxs[k] = lane + 64 * k < TW ? gx : 0;
    }
    // rows are fetched two ahead: pre holds the next row to stage, pre2 the
    // one after (gy is pre2's row)
    int gy = (y0 - M) % n;
    gy += gy < 0 ? n : 0;
    TS pre[CPL], pre2[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) pre[k] = src[(int64_t)gy * n + gxs[k]];
    gy = gy + 1 < n ? gy + 1 : 0;
#pragma unroll
    for (int k = 0; k < CPL; ++k) pre2[k] = src[(int64_t)gy * n + gxs[k]];

    const TA ap = coef_ap<TA>(d), bcoef = coef_b<TA>(d), ce = geo_ce<TA>(geo);
    TA g[M + 1];
#pragma unroll
    for (int k = 0; k <= M; ++k) g[k] = GAUSS ? geo_g<TA>(geo, k) : TA(1);

    // Centre values are fetched one row ahead of their use and before that
    // row's prefetch, so that waiting for them never waits for the prefetch.
    int xcl[R];
    TS cnext[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const int x = x0 + c0 + c;
        xcl[c] = x < ne ? x : 0;
        cnext[c] = src[(int64_t)y0 * n + xcl[c]];
    }

    TA acc[P][R];
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
        for (int c = 0; c < R; ++c) acc[i][c] = TA(-0.0);
    // energy partial sums of the input state (only with epart): sum u Lsum
    // and sum (1 - u^2) over this lane's outputs in the arithmetic type, then
    // across the wave in FP64
    TA e_ul = TA(0), e_pot = TA(0);

    for (int pb = 0; pb < rows; pb += P) {
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int p = pb + i;
            if (p < rows) {
                // stage row p, prefetch row p + 1
                TA *slot = ring[i & 1 ? (pb & 1) ^ 1 : (pb & 1)];
                // centre values of the output finishing at this row (fetched
                // at the previous row), then those of the next row's output
                // (row index clamped into the band: always a valid address)
                const int q = p - 2 * M;
                const int y = y0 + q;
                TS cen[R];
#pragma unroll
                for (int c = 0; c < R; ++c) cen[c] = cnext[c];
                {
                    int qn = q + 1;
                    qn = qn < 0 ? 0 : (qn < bq ? qn : bq - 1);
#pragma unroll
                    for (int c = 0; c < R; ++c)
                        cnext[c] = src[(int64_t)(y0 + qn) * n + xcl[c]];
                }
#pragma unroll
                for (int k = 0; k < CPL; ++k)
                    slot[lane + 64 * k] = to_acc<TA>(pre[k]);
                gy = gy + 1 < n ? gy + 1 : 0;
                // unconditional (up to two rows past the band at the end; the
                // row index wraps, so the address stays inside the sample)
#pragma unroll
                for (int k = 0; k < CPL; ++k) {
                    pre[k] = pre2[k];
                    pre2[k] = src[(int64_t)gy * n + gxs[k]];
                }
                __syncthreads();  // one wave: makes the staged row visible
                TA win[WIN];
                load_window<WIN, (R % 2 == 0)>(slot + c0, win);
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    // input row p feeds output q' = p - M - dy, ring slot q' mod P
                    row_windows<R2, GAUSS>(win + c, g, [&](int dy) -> TA & {
                        return acc[((i - M - dy) % P + P) % P][c];
                    });
                }
                const int done = (i + 1) % P;
                if (q >= 0) {
#pragma unroll
                    for (int c = 0; c < R; ++c) {
                        const int x = x0 + c0 + c;
                        const TA u = to_acc<TA>(cen[c]);
                        if (x < ne) {
                            dst[(int64_t)y * n + x] =
                                to_store<TS>(update_g<TA>(u, acc[done][c], ap, bcoef));
                            if (epart) {
                                e_ul += u * lsum_of(ce, u, acc[done][c]);
                                e_pot += TA(1) - u * u;
                            }
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c < R; ++c) acc[done][c] = TA(-0.0);
            }
        }
    }
    if (epart) {
        // fixed shuffle tree: the partials do not depend on timing
        double s_ul = (double)e_ul, s_pot = (double)e_pot;
        for (int o = 32; o > 0; o >>= 1) {
            s_ul += __shfl_xor(s_ul, o, 64);
            s_pot += __shfl_xor(s_pot, o, 64);
        }
        if (lane == 0) {
            epart[2 * (int64_t)bidx] = s_ul;
            epart[2 * (int64_t)bidx + 1] = s_pot;
        }
    }
}

// ---------------------------------------------------------------------------
// Shared-band streaming step (W >= 2 waves per workgroup).  The workgroup
// owns a strip of 64R columns and a band of BW output rows and walks the
// band's BW + 2m input rows once, split into consecutive runs, one per wave;
// each wave walks its run as k_stream does.  The runs meet inside the band:
// the first 2m outputs a wave retires (missing the rows of the wave above)
// go to LDS, and after one barrier the wave above adds them to its last 2m
// pending outputs and finishes those.  Every wave but the last walks exactly
// L rows, a multiple of the ring period, so that its pending outputs sit in
// known registers at the end; the last walks the rest (at least 2m rows).
// Compared with one wave per band, the 2m halo rows are walked once per
// band of W runs instead of once per run.
// ---------------------------------------------------------------------------

// LDS layout of k_band (arithmetic type TA): per wave a two-row staging
// ring and 2m rows of 64R partial sums.
template <int R2, int R, class TA>
struct StreamLds {
    static constexpr int M = Disc<R2>::M;
    static constexpr int TW = 64 * R + 2 * M;
    static constexpr int CPL = (TW + 63) / 64;  // row-segment elements per lane
    static constexpr int RING = 2 * 64 * CPL;   // ring elements per wave
    static constexpr int HEAD = 2 * M * 64 * R;  // partial-sum elements per wave
    static constexpr size_t bytes(int W) { return (size_t)W * (RING + HEAD) * sizeof(TA); }
    static_assert(RING == 2 * 64 * ((64 * R + 2 * M + 63) / 64), "see stream_lds_bytes");
};

template <int R2, int R, class TS, class TA, bool GAUSS>
__global__ __launch_bounds__(512) void k_band(
    const SampleDesc *__restrict__ sd, const int32_t *__restrict__ ids,
    const ModelGeo *__restrict__ geo, const TS *__restrict__ in,
    TS *__restrict__ out, int BW, int L, int strips, int bands, int nblocks,
    double *__restrict__ epart) {
    using LD = StreamLds<R2, R, TA>;
    constexpr int M = Disc<R2>::M, P = Disc<R2>::P;
    constexpr int TX = 64 * R;
    constexpr int TW = LD::TW;
    constexpr int WIN = 2 * M + R;
    constexpr int CPL = LD::CPL;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[16];

    const int W = blockDim.x >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // the ring holds the arithmetic type: a narrow state is widened once per
    // staged element instead of once per window read; rows are padded to
    // 64 CPL elements so that every lane stores
    TA *ring = reinterpret_cast<TA *>(smem_raw) + (size_t)wv * LD::RING;
    TA *heads = reinterpret_cast<TA *>(smem_raw) + (size_t)W * LD::RING;

    const int n = geo->n;
    const int lo = geo->lo, ne = n - geo->lo;  // updated block [lo, ne)^2
    const int bidx = xcd_remap(blockIdx.x, nblocks);
    const int per_sample = strips * bands;
    const SampleDesc d = sd[ids[bidx / per_sample]];
    const int tile = bidx % per_sample;
    const int x0 = lo + (tile % strips) * TX;
    const int y0 = lo + (tile / strips) * BW;
    const TS *src = in + d.offset;
    TS *dst = out + d.offset;
    const int c0 = lane * R;
    const int bq = y0 + BW <= ne ? BW : ne - y0;  // output rows of this band
    const int T = bq + 2 * M;                    // input rows of this band
    // waves with rows to walk; wave wv walks input rows [s, s + Lw) of the
    // band's T rows and retires outputs q = s + t - 2m (q relative to y0)
    const int weff = bq / L + 1 < W ? bq / L + 1 : W;
    const int s = wv * L;
    const int Lw = wv < weff - 1 ? L : T - s;

    const TA ap = coef_ap<TA>(d), bcoef = coef_b<TA>(d), ce = geo_ce<TA>(geo);
    TA g[M + 1];
#pragma unroll
    for (int k = 0; k <= M; ++k) g[k] = GAUSS ? geo_g<TA>(geo, k) : TA(1);

    int xcl[R];  // centre columns (clamped in range for idle lanes)
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const int x = x0 + c0 + c;
        xcl[c] = x < ne ? x : 0;
    }

    TA acc[P][R];
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
        for (int c = 0; c < R; ++c) acc[i][c] = TA(-0.0);
    // energy partial sums of the input state (only with epart): sum u Lsum
    // and sum (1 - u^2) over this lane's outputs in the arithmetic type, then
    // across the workgroup in FP64
    TA e_ul = TA(0), e_pot = TA(0);

    if (wv < weff) {
        // wrapped source columns of this lane's staged elements; lanes past
        // the segment end re-read column 0 into the ring's padding
        int gxs[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            int gx = (x0 - M + lane + 64 * k) % n;
            gx += gx < 0 ? n : 0;
            gxs[k] = lane + 64 * k < TW ? gx : 0;
        }
        // rows are fetched two ahead (as in k_stream)
        int gy = (y0 - M + s) % n;
        gy += gy < 0 ? n : 0;
        TS pre[CPL], pre2[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) pre[k] = src[(int64_t)gy * n + gxs[k]];
        gy = gy + 1 < n ? gy + 1 : 0;
#pragma unroll
        for (int k = 0; k < CPL; ++k) pre2[k] = src[(int64_t)gy * n + gxs[k]];
        // Centre values are fetched one row ahead of their use, so that the
        // wait before staging a row covers exactly the previous row's loads.
        TS cnext[R];
        {
            int q0 = s - 2 * M;
            q0 = q0 < 0 ? 0 : (q0 < bq ? q0 : bq - 1);
#pragma unroll
            for (int c = 0; c < R; ++c) cnext[c] = src[(int64_t)(y0 + q0) * n + xcl[c]];
        }

        for (int pb = 0; pb < Lw; pb += P) {
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const int t = pb + i;
                if (t < Lw) {
                    TA *slot = ring + (i & 1 ? (pb & 1) ^ 1 : (pb & 1)) * (64 * CPL);
                    // centre values of the output retiring at this row, then
                    // those of the next (row clamped into the band)
                    const int q = s + t - 2 * M;
                    TS cen[R];
#pragma unroll
                    for (int c = 0; c < R; ++c) cen[c] = cnext[c];
                    {
                        int qn = q + 1;
                        qn = qn < 0 ? 0 : (qn < bq ? qn : bq - 1);
#pragma unroll
                        for (int c = 0; c < R; ++c)
                            cnext[c] = src[(int64_t)(y0 + qn) * n + xcl[c]];
                    }
#pragma unroll
                    for (int k = 0; k < CPL; ++k) slot[lane + 64 * k] = to_acc<TA>(pre[k]);
                    gy = gy + 1 < n ? gy + 1 : 0;
                    // unconditional (up to two rows past the run at the end;
                    // the row index wraps, so the address stays inside the
                    // sample)
#pragma unroll
                    for (int k = 0; k < CPL; ++k) {
                        pre[k] = pre2[k];
                        pre2[k] = src[(int64_t)gy * n + gxs[k]];
                    }
                    // the ring is private to the wave and LDS operations of
                    // one wave complete in order: only keep the compiler from
                    // reordering the staging stores and the window loads
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    TA win[WIN];
                    load_window<WIN, (R % 2 == 0)>(slot + c0, win);
#pragma unroll
                    for (int c = 0; c < R; ++c) {
                        // input row t feeds output t - m - dy (walk-relative),
                        // ring slot (t - m - dy) mod P
                        row_windows<R2, GAUSS>(win + c, g, [&](int dy) -> TA & {
                            return acc[((i - M - dy) % P + P) % P][c];
                        });
                    }
                    const int done = (i + 1) % P;
                    if (t >= 2 * M) {
                        // complete: every input row of this output is in the run
                        const int y = y0 + q;
#pragma unroll
                        for (int c = 0; c < R; ++c) {
                            const int x = x0 + c0 + c;
                            const TA u = to_acc<TA>(cen[c]);
                            if (x < ne) {
                                dst[(int64_t)y * n + x] =
                                    to_store<TS>(update_g<TA>(u, acc[done][c], ap, bcoef));
                                if (epart) {
                                    e_ul += u * lsum_of(ce, u, acc[done][c]);
                                    e_pot += TA(1) - u * u;
                                }
                            }
                        }
                    } else if (wv > 0) {
                        // partial (rows of the wave above missing): hand over
#pragma unroll
                        for (int c = 0; c < R; ++c)
                            heads[((size_t)wv * 2 * M + t) * TX + c0 + c] = acc[done][c];
                    }
#pragma unroll
                    for (int c = 0; c < R; ++c) acc[done][c] = TA(-0.0);
                }
            }
        }
    }

    {
        __syncthreads();
        if (wv < weff - 1) {
            // Last 2m pending outputs q = s + L - 2m + k: ring slot (k + 1)
            // mod P (L is a multiple of P), plus the next wave's first 2m.
#pragma unroll
            for (int k = 0; k < 2 * M; ++k) {
                const int y = y0 + s + L - 2 * M + k;
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    const int x = x0 + c0 + c;
                    const TA sum = acc[(k + 1) % P][c] +
                                   heads[((size_t)(wv + 1) * 2 * M + k) * TX + c0 + c];
                    const TA u = to_acc<TA>(src[(int64_t)y * n + xcl[c]]);
                    if (x < ne) {
                        dst[(int64_t)y * n + x] = to_store<TS>(update_g<TA>(u, sum, ap, bcoef));
                        if (epart) {
                            e_ul += u * lsum_of(ce, u, sum);
                            e_pot += TA(1) - u * u;
                        }
                    }
                }
            }
        }
    }
    if (epart) {
        // fixed shuffle tree, then the waves in order: the partials do not
        // depend on timing
        double s_ul = (double)e_ul, s_pot = (double)e_pot;
        for (int o = 32; o > 0; o >>= 1) {
            s_ul += __shfl_xor(s_ul, o, 64);
            s_pot += __shfl_xor(s_pot, o, 64);
        }
        __syncthreads();
        if (lane == 0) {
            red[2 * wv] = s_ul;
            red[2 * wv + 1] = s_pot;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a0 = 0.0, a1 = 0.0;
            for (int w = 0; w < W; ++w) {
                a0 += red[2 * w];
                a1 += red[2 * w + 1];
            }
            epart[2 * (int64_t)bidx] = a0;
            epart[2 * (int64_t)bidx + 1] = a1;
        }
    }
}

// ---------------------------------------------------------------------------
// Two-phase streaming step: one wave owns a strip of 32R columns and a band of
// B output rows, and its two half-waves walk the band's input rows in
// alternation (lanes 0-31 rows 0, 2, 4, ... of the B + 2m rows, lanes 32-63
// rows 1, 3, 5, ...), each over the whole strip.  Every input row's window
// sums are formed once, by the half that walks it, and each half keeps the
// partial sums of its own rows for the outputs they feed; an output is the
// sum of its two partial sums, exchanged by one lane swap
// (v_permlane32_swap) when both are complete.  Against one wave per band
// (k_stream) this gives twice the waves for a band height, so bands can be
// twice as tall for the same number of waves and the 2m halo rows cost half
// as much, with no hand-over through LDS.  Each output's disc sum is formed
// in two parts (its even and its odd input rows), so results differ from
// k_stream's by rounding only.
//
// Register ring.  Both halves run the same instructions, so a register names
// a different output in each half: at iteration i half h walks input row
// p = 2i + h and adds the window sum of disc row dy to slot
// (2i - m - dy) mod S, which holds output q = slot + h (q relative to the
// band's first row).  S = 2m + 2 slots hold every output a half can have
// pending.  At iteration i the outputs 2i - 2m (finished by half 0) and
// 2i - 2m + 1 (half 1) are complete: half 0 takes its own slot 2i - 2m and
// half 1's slot 2i - 2m - 1, half 1 its own slot 2i - 2m and half 0's slot
// 2i - 2m + 1; those slots are then cleared in the half that owned them.
// ---------------------------------------------------------------------------
template <int R2, int R, class TS, class TA, bool GAUSS>
__global__ __launch_bounds__(64) void k_phase(
    const SampleDesc *__restrict__ sd, const int32_t *__restrict__ ids,
    const ModelGeo *__restrict__ geo, const TS *__restrict__ in,
    TS *__restrict__ out, int B, int strips, int bands, int nblocks,
    double *__restrict__ epart) {
    constexpr int M = Disc<R2>::M;
    constexpr int TX = 32 * R;            // strip columns
    constexpr int TW = TX + 2 * M;        // staged row segment
    constexpr int WIN = 2 * M + R;
    constexpr int CPL = (TW + 31) / 32;   // staged elements per lane
    // register ring slots (at least 2m + 2) and iterations per ring period;
    // U is even, so that an iteration's parity is static in the unrolled
    // loop and the prefetch buffers alternate without register moves
    constexpr int U = (M + 2) & ~1;
    constexpr int S = 2 * U;
    constexpr int HS = 32 * CPL;          // ring elements per half-wave row
    static_assert(sizeof(TA) == 4, "the lane swap moves 32-bit values");
    // [row parity][half][element]; the ring holds the arithmetic type
    __shared__ __align__(16) TA ring[2][2][HS];

    const int n = geo->n;
    const int lo = geo->lo, ne = n - geo->lo;  // updated block [lo, ne)^2
    const int bidx = xcd_remap(blockIdx.x, nblocks);
    const int per_sample = strips * bands;
    const SampleDesc d = sd[ids[bidx / per_sample]];
    const int t = bidx % per_sample;
    const int x0 = lo + (t % strips) * TX;
    const int y0 = lo + (t / strips) * B;
    const TS *src = in + d.offset;
    TS *dst = out + d.offset;
    const int lane = threadIdx.x;
    const int half = lane >> 5;
    const int hl = lane & 31;
    const int c0 = hl * R;
    const int bq = y0 + B <= ne ? B : ne - y0;  // output rows of this band
    const int iters = (bq + 2 * M + 1) / 2;     // input row pairs

    // wrapped source columns of this lane's staged elements; lanes past the
    // segment end re-read column 0 into the ring's padding
    int gxs[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        int gx = (x0 - M + hl + 32 * k) % n;
        gx += gx < 0 ? n : 0;
        gxs[k] = hl + 32 * k < TW ? gx : 0;
    }
    // rows are fetched two iterations ahead into two buffers: iteration i
    // stages pre[i & 1] and then loads the row of iteration i + 2 into it
    // (gy is the last row fetched); a half's rows advance by two
    int gy = (y0 - M + half) % n;
    gy += gy < 0 ? n : 0;
    TS pre[2][CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) pre[0][k] = src[(int64_t)gy * n + gxs[k]];
    gy += 2;
    gy -= gy >= n ? n : 0;
#pragma unroll
    for (int k = 0; k < CPL; ++k) pre[1][k] = src[(int64_t)gy * n + gxs[k]];

    const TA ap = coef_ap<TA>(d), bcoef = coef_b<TA>(d), ce = geo_ce<TA>(geo);
    TA g[M + 1];
#pragma unroll
    for (int k = 0; k <= M; ++k) g[k] = GAUSS ? geo_g<TA>(geo, k) : TA(1);

    // centre values of the output this half finishes at iteration i, fetched
    // two iterations ahead into cnext[i & 1] (row index clamped into the
    // band: always a valid address)
    int xcl[R];
    TS cnext[2][R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const int x = x0 + c0 + c;
        xcl[c] = x < ne ? x : 0;
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        int q0 = 2 * e + half - 2 * M;
        q0 = q0 < 0 ? 0 : (q0 < bq ? q0 : bq - 1);
#pragma unroll
        for (int c = 0; c < R; ++c) cnext[e][c] = src[(int64_t)(y0 + q0) * n + xcl[c]];
    }

    TA acc[S][R];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
        for (int c = 0; c < R; ++c) acc[i][c] = TA(-0.0);
    TA e_ul = TA(0), e_pot = TA(0);

    for (int ib = 0; ib < iters; ib += U) {
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int i = ib + j;
            if (i < iters) {
                TA *slot = ring[j & 1][half];  // ib is even (U is)
                // this half finishes output q = 2i - 2m + half
                const int q = 2 * i - 2 * M + half;
                const int y = y0 + q;
#pragma unroll
                for (int k = 0; k < CPL; ++k) slot[hl + 32 * k] = to_acc<TA>(pre[j & 1][k]);
                gy += 2;
                gy -= gy >= n ? n : 0;
                // unconditional (up to four rows past the band at the end;
                // the row index wraps, so the address stays in the sample)
#pragma unroll
                for (int k = 0; k < CPL; ++k) pre[j & 1][k] = src[(int64_t)gy * n + gxs[k]];
                __syncthreads();  // one wave: makes the staged rows visible
                TA win[WIN];
                load_window<WIN, (R % 2 == 0)>(slot + c0, win);
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    // a row past the band's last input row (odd row count)
                    // feeds only outputs past the band, which are never
                    // finished
                    row_windows<R2, GAUSS>(win + c, g, [&](int dy) -> TA & {
                        return acc[((2 * j - M - dy) % S + S) % S][c];
                    });
                }
                // (static after unrolling)
                const int own = ((2 * j - 2 * M) % S + S) % S;
                const int sdn = (own + S - 1) % S;  // half 1's part of half 0's output
                const int sup = (own + 1) % S;      // half 0's part of half 1's output
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    const auto sw = __builtin_amdgcn_permlane32_swap(
                        __float_as_uint(acc[sdn][c]), __float_as_uint(acc[sup][c]), false,
                        false);
                    const TA other = __uint_as_float(half ? sw[0] : sw[1]);
                    const TA G = acc[own][c] + other;
                    const int x = x0 + c0 + c;
                    const TA u = to_acc<TA>(cnext[j & 1][c]);
                    if (q >= 0 && q < bq && x < ne) {
                        dst[(int64_t)y * n + x] = to_store<TS>(update_g<TA>(u, G, ap, bcoef));
                        if (epart) {
                            e_ul += u * lsum_of(ce, u, G);
                            e_pot += TA(1) - u * u;
                        }
                    }
                    acc[own][c] = TA(-0.0);
                    acc[sdn][c] = half ? TA(-0.0) : acc[sdn][c];
                    acc[sup][c] = half ? acc[sup][c] : TA(-0.0);
                }
                {
                    // centre values of iteration i + 2
                    int qn = q + 4;
                    qn = qn < 0 ? 0 : (qn < bq ? qn : bq - 1);
#pragma unroll
                    for (int c = 0; c < R; ++c)
                        cnext[j & 1][c] = src[(int64_t)(y0 + qn) * n + xcl[c]];
                }
            }
        }
    }
    if (epart) {
        // fixed shuffle tree: the partials do not depend on timing
        double s_ul = (double)e_ul, s_pot = (double)e_pot;
        for (int o = 32; o > 0; o >>= 1) {
            s_ul += __shfl_xor(s_ul, o, 64);
            s_pot += __shfl_xor(s_pot, o, 64);
        }
        if (lane == 0) {
            epart[2 * (int64_t)bidx] = s_ul;
            epart[2 * (int64_t)bidx + 1] = s_pot;
        }
    }
}

// ---------------------------------------------------------------------------
// LDS-resident multi-step kernel: one workgroup holds one whole n x n sample
// in LDS (rows padded with an m-column periodic halo) and runs every step
// without touching HBM.  Wave b owns the band of B rows starting at b*B
// (n is a multiple of B) and R columns per lane; it keeps its sites in
// registers.  Per step it publishes them to LDS, then walks only its own B
// input rows: window sums of a row feed the 2m+1 output rows around it,
// including the m rows above and below the band, whose partial sums go to
// the neighbouring bands through an LDS exchange area.  After a barrier
// each band adds the partial sums it received and updates its sites.  Every
// input row is read and turned into window sums exactly once per step.
// The initial projection and the final FP64 output-of-interest reduction
// are fused in.
//
// VOL (volume constraint): the stored array is (n + 2m)^2 with the n x n
// lattice of Omega inside a ring of m rows and columns of fixed values.  The
// ring columns of a band's rows sit in the LDS halo for the whole solve, and
// the ring rows above and below Omega, whose contribution to the first and
// last m rows never changes, are turned into window sums once, before the
// first step; bands 0 and n/B - 1 add those instead of a neighbour's sums.
// ---------------------------------------------------------------------------

// LDS row stride of the resident kernel: n plus the 2m halo, rounded up to
// an even count so that paired window loads stay aligned.
__host__ __device__ constexpr int resident_row_stride(int n, int M) {
    return (n + 2 * M + 1) & ~1;
}

// In-place exchange: a band reads only its own rows of the LDS state while
// it walks them, so once its walk is done it can hand its partial sums over
// in those rows (2m x n values in B rows of the state's type) instead of in
// an area of their own.  That halves the LDS of the kernel, so that two
// workgroups share a CU (four waves per SIMD).  Used where the partial sums
// fit and have the state's type, without the energy trace or a volume
// constraint (whose variants keep more values in registers).
__host__ __device__ constexpr bool resident_inplace(int n, int M, int B, size_t ts, size_t ta,
                                                    bool energy, bool vol) {
    return !energy && !vol && ts == ta && 2 * M * n <= B * resident_row_stride(n, M);
}

// LDS bytes of the resident kernel: the state rows, then (unless the
// exchange is in place) for every band an "up" and a "down" exchange block of
// m rows of n partial sums, and with a volume constraint the fixed sums of the
// ring rows above and below.
__host__ __device__ constexpr size_t resident_lds_bytes(int n, int M, int B, size_t ts,
                                                        size_t ta, bool energy = false,
                                                        bool vol = false) {
    return (size_t)n * resident_row_stride(n, M) * ts +
           (resident_inplace(n, M, B, ts, ta, energy, vol)
                ? 0
                : (2 * (size_t)(n / B) + (vol ? 2 : 0)) * M * n * ta);
}

// In-place layouts: FP32 arithmetic keeps to the 128 registers that four
// waves per SIMD allow; FP64, whose values take two registers each, would
// spill there and may use 256 (two waves per SIMD).
template <int R2, int N, int B, class TS, class TA, bool GAUSS, bool ENERGY, bool VOL,
          bool INPLACE = resident_inplace(N, Disc<R2>::M, B, sizeof(TS), sizeof(TA), ENERGY,
                                          VOL)>
__global__ __launch_bounds__(512, INPLACE ? (sizeof(TA) == 8 ? 2 : 4) : 1) void k_resident(
    const SampleDesc *__restrict__ sd, const int32_t *__restrict__ ids,
    const ModelGeo *__restrict__ geo, TS *__restrict__ state, int nsteps,
    double *__restrict__ ooi, double *__restrict__ energy, int64_t estride) {
    // The lattice size is a compile-time constant so that every LDS offset
    // below is an instruction immediate rather than a register.
    constexpr int M = Disc<R2>::M;
    constexpr int R = N <= 64 ? 1 : 2;  // columns per lane, n <= 64 R
    constexpr int WIN = 2 * M + R;
    constexpr int Q = B + 2 * M;  // outputs fed by one band: its rows +- m
    static_assert(M <= B, "partial sums must only reach the adjacent bands");
    static_assert(N % B == 0 && N <= 64 * R, "one wave per band");
    static_assert(!(VOL && ENERGY), "no energy trace under a volume constraint");
    constexpr int S = VOL ? N + 2 * M : N;  // side of the stored array
    constexpr int OFF = VOL ? M : 0;        // its row and column of Omega's (0, 0)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[16];

    constexpr int n = N;
    constexpr int TW = resident_row_stride(N, M);
    constexpr int NB = N / B;
    TS *lds = reinterpret_cast<TS *>(smem_raw);
    TA *xup = reinterpret_cast<TA *>(smem_raw + (size_t)n * TW * sizeof(TS));
    TA *xdn = xup + (size_t)NB * M * n;
    TA *rtop = xdn + (size_t)NB * M * n;  // VOL: ring rows above, outputs 0..m-1
    TA *rbot = rtop + (size_t)M * n;      // VOL: ring rows below, outputs n-m..n-1
    const int sidx = ids[blockIdx.x];
    const SampleDesc d = sd[sidx];
    TS *g_state = state + d.offset;
    // one wave per band (n <= 64 R); band arithmetic stays scalar
    const int band = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xb = (threadIdx.x & 63) * R;
    const int y0 = band * B;
    const int xr = xb + R <= n ? xb : n - R;  // in-row read position for idle lanes
    const int bup = band + 1 < NB ? band + 1 : 0;
    const int bdn = band > 0 ? band - 1 : NB - 1;

    const TA ap = coef_ap<TA>(d), bcoef = coef_b<TA>(d), ce = geo_ce<TA>(geo);
    TA g[M + 1];
#pragma unroll
    for (int k = 0; k <= M; ++k) g[k] = GAUSS ? geo_g<TA>(geo, k) : TA(1);

    // Load and project u0 onto [-1, 1].
    TA st[B][R];
#pragma unroll
    for (int q = 0; q < B; ++q)
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int x = xb + c;
            TA v = TA(0);
            if (x < n) v = to_acc<TA>(g_state[(int64_t)(y0 + q + OFF) * S + x + OFF]);
            st[q][c] = clamp1(v);
        }

    if constexpr (VOL) {
        // The projected ring: columns of this band's rows into the LDS halo
        // (and back to HBM, projected), for the whole solve.
        for (int k = threadIdx.x & 63; k < B * 2 * M; k += 64) {
            const int q = k / (2 * M), j = k - q * 2 * M;
            const int col = j < M ? j : N + j;  // stored column = LDS column
            TS *gp = g_state + (int64_t)(y0 + q + M) * S + col;
            const TS v = to_store<TS>(clamp1(to_acc<TA>(*gp)));
            lds[(y0 + q) * TW + col] = v;
            *gp = v;
        }
        // Window sums of the ring rows above (band 0) and below (last band),
        // accumulated into the outputs of Omega's first and last m rows.
        // r0: Omega row index of the first ring row; qlo: first output row
        // (both compile-time, so that every register index below is static)
        auto ring_rows = [&](auto R0, auto QLO, TA *dst) {
            constexpr int r0 = decltype(R0)::value, qlo = decltype(QLO)::value;
            TA ac[M][R];
#pragma unroll
            for (int q = 0; q < M; ++q)
#pragma unroll
                for (int c = 0; c < R; ++c) ac[q][c] = TA(-0.0);
#pragma unroll
            for (int i = 0; i < M; ++i) {
                // input row r0 + i (Omega row index; stored row r0 + i + m)
                TS *gp = g_state + (int64_t)(r0 + i + M) * S + xr;
                TA win[WIN];
#pragma unroll
                for (int k = 0; k < WIN; ++k) win[k] = clamp1(to_acc<TA>(gp[k]));
                // the projected ring back to HBM (the lanes' windows overlap:
                // lanes storing the same element store the same value)
#pragma unroll
                for (int k = 0; k < WIN; ++k) gp[k] = to_store<TS>(win[k]);
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    TA sink = TA(0);  // outputs outside Omega's first/last m rows
                    row_windows<R2, GAUSS>(win + c, g, [&](int dy) -> TA & {
                        const int q = r0 + i - dy - qlo;
                        return (q >= 0 && q < M) ? ac[q][c] : sink;
                    });
                }
            }
#pragma unroll
            for (int c = 0; c < R; ++c) {
                const int x = xb + c;
                if (x < n) {
#pragma unroll
                    for (int q = 0; q < M; ++q) dst[q * n + x] = ac[q][c];
                }
            }
        };
        if (band == 0)
            ring_rows(std::integral_constant<int, -M>{}, std::integral_constant<int, 0>{}, rtop);
        if (band == NB - 1)
            ring_rows(std::integral_constant<int, N>{}, std::integral_constant<int, N - M>{},
                      rbot);
    }

    // With the energy trace, one more pass evaluates E_h(u^nsteps); its
    // update is discarded and the state is written back from the LDS copy.
    const int passes = nsteps + (ENERGY ? 1 : 0);
    for (int step = 0; step < passes; ++step) {
        // Publish the state to LDS.  The lanes next to the lattice edge then
        // write the periodic column halo in a store of their own (a volume
        // constraint keeps the fixed ring columns there instead): folded into
        // every lane's store, the halo copies hit LDS banks that other lanes
        // of the same store use at other addresses.
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int x = xb + c;
            if (N == 64 * R || x < n) {
#pragma unroll
                for (int q = 0; q < B; ++q)
                    lds[(y0 + q) * TW + M + x] = to_store<TS>(st[q][c]);
            }
        }
        if constexpr (!VOL && M % R == 0 && N == 64 * R) {
            // a lane's R columns are all halo columns or none: one store of
            // R adjacent values per row
            if (xb < M || xb >= n - M) {
                const int xh = xb < M ? xb + n : xb - n;
#pragma unroll
                for (int q = 0; q < B; ++q)
#pragma unroll
                    for (int c = 0; c < R; ++c)
                        lds[(y0 + q) * TW + M + xh + c] = to_store<TS>(st[q][c]);
            }
        } else if constexpr (!VOL) {
#pragma unroll
            for (int c = 0; c < R; ++c) {
                const int x = xb + c;
                if (x < M || (x >= n - M && x < n)) {
                    const int xh = x < M ? x + n : x - n;
#pragma unroll
                    for (int q = 0; q < B; ++q)
                        lds[(y0 + q) * TW + M + xh] = to_store<TS>(st[q][c]);
                }
            }
        }
        __syncthreads();

        // acc[M + q] collects output row y0 + q, q in [-m, B + m).
        TA acc[Q][R];
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int c = 0; c < R; ++c) acc[q][c] = TA(-0.0);
        const TS *rp0 = lds + y0 * TW + xr;
        // The window of row i + 1 is loaded while row i is summed (two
        // window buffers); the empty asm keeps the compiler from hoisting
        // every row's loads, and their registers, to the top of the walk.
        TA win[2][WIN];
        load_window<WIN, (R % 2 == 0)>(rp0, win[0]);
#pragma unroll
        for (int i = 0; i < B; ++i) {
            asm volatile("" ::: "memory");
            if (i + 1 < B) load_window<WIN, (R % 2 == 0)>(rp0 + (i + 1) * TW, win[(i + 1) & 1]);
#pragma unroll
            for (int c = 0; c < R; ++c) {
                // input row i feeds output q = i - dy
                row_windows<R2, GAUSS>(win[i & 1] + c, g, [&](int dy) -> TA & {
                    return acc[M + i - dy][c];
                });
            }
        }
        // Hand the overhanging partial sums to the adjacent bands (in place:
        // in this band's own rows, after taking back its sites' values).
        TA *myup = xup + (size_t)band * M * n, *mydn = xdn + (size_t)band * M * n;
        const TA *above = xdn + (size_t)bdn * M * n;
        const TA *below = xup + (size_t)bup * M * n;
        if constexpr (INPLACE) {
#pragma unroll
            for (int q = 0; q < B; ++q)
#pragma unroll
                for (int c = 0; c < R; ++c) st[q][c] = to_acc<TA>(lds[(y0 + q) * TW + M + xr + c]);
            // the wave's own reads of its rows come before its writes there
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            myup = reinterpret_cast<TA *>(lds + y0 * TW);
            mydn = myup + (size_t)M * n;
            above = reinterpret_cast<const TA *>(lds + bdn * B * TW) + (size_t)M * n;
            below = reinterpret_cast<const TA *>(lds + bup * B * TW);
        }
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int x = xb + c;
            if (x < n) {
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    myup[(size_t)j * n + x] = acc[j][c];
                    mydn[(size_t)j * n + x] = acc[B + M + j][c];
                }
            }
        }
        __syncthreads();
        if constexpr (VOL) {
            if (band == 0) above = rtop;
            if (band == NB - 1) below = rbot;
        }
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int x = xr + c;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                acc[M + j][c] += above[(size_t)j * n + x];
                acc[B + j][c] += below[(size_t)j * n + x];
            }
        }
        // (in place) the neighbours have read this band's rows before it
        // publishes the next state there
        if constexpr (INPLACE) __syncthreads();
        // (energy trace) E_h of the state this pass started from, from the
        // per-site terms u Lsum and 1 - u^2 accumulated in FP64
        double e_ul = 0.0, e_pot = 0.0;
#pragma unroll
        for (int q = 0; q < B; ++q)
#pragma unroll
            for (int c = 0; c < R; ++c) {
                const TA u = st[q][c];
                if constexpr (ENERGY) {
                    if (xb + c < n) {
                        const TA lsum = lsum_of(ce, u, acc[M + q][c]);
                        e_ul += (double)u * (double)lsum;
                        e_pot += 1.0 - (double)u * (double)u;
                    }
                }
                st[q][c] = to_acc<TA>(to_store<TS>(update_g<TA>(u, acc[M + q][c], ap, bcoef)));
            }
        if constexpr (ENERGY) {
            e_ul = block_sum(e_ul, red);
            e_pot = block_sum(e_pot, red);
            if (threadIdx.x == 0)
                energy[(int64_t)step * estride + sidx] = d.e_int * e_ul + d.e_pot * e_pot;
        }
    }

    // Write back and reduce the output of interest in FP64 (with the energy
    // trace the last pass's update is dropped: u^nsteps is the LDS copy).
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < B; ++q)
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int x = xb + c;
            if (x < n) {
                const TA v = ENERGY ? to_acc<TA>(lds[(y0 + q) * TW + M + x]) : st[q][c];
                g_state[(int64_t)(y0 + q + OFF) * S + x + OFF] = to_store<TS>(v);
                part += (double)v;
            }
        }
    const double tot = block_sum(part, red);
    if (threadIdx.x == 0) {
        const double mean = tot / ((double)n * n);
        ooi[2 * (int64_t)sidx] = mean;
        ooi[2 * (int64_t)sidx + 1] = 0.5 * (1.0 + mean);
    }
}


}  // namespace nlch
