// LDS-resident kernel with four columns per lane (FP32, 128^2, periodic) and
// its launcher, in a unit of its own.
#include "kern_rowrun_impl.h"

namespace nlch {

// ---------------------------------------------------------------------------
// LDS-resident kernel with four columns per lane (FP32 state and arithmetic,
// n = 128, periodic).  The layout of k_resident, with two changes that cut
// the LDS traffic of the row walk:
//  * a lane owns 4 adjacent columns, so a row of 128 columns takes 32 lanes
//    and one wave walks two bands (lanes 0-31 band 2w, lanes 32-63 band
//    2w + 1; four waves hold the 8 bands of 16 rows);
//  * the row stride is a multiple of 4 floats, so a lane's window of 2m + 4
//    values, which starts at its first column minus m, is 16-byte aligned
//    and read with 16-byte LDS loads (2m + 4 values for 4 sites instead of
//    2m + 2 for 2).
// Every site sums the same window sums in the same order as k_resident (own
// rows in order, then the band above's partial sums, then the band below's),
// so the two kernels give bit-identical states.  The partial sums are handed
// over in place, in the band's own rows, as in k_resident.
// ---------------------------------------------------------------------------

// Row stride of the four-column layout: n plus the 2m halo, plus two columns
// for odd m (the last lane's rounded-up window read), rounded up to 4 floats.
__host__ __device__ constexpr int resident4_row_stride(int n, int M) {
    return (n + 2 * M + (M % 2 ? 2 : 0) + 3) & ~3;
}

__host__ __device__ constexpr size_t resident4_lds_bytes(int n, int M) {
    return (size_t)n * resident4_row_stride(n, M) * sizeof(float);
}

// Built where the partial sums of a band fit in its own rows.
__host__ __device__ constexpr bool resident4_fits(int n, int M, int B) {
    return n == 128 && M <= B && 2 * M * n <= B * resident4_row_stride(n, M);
}

template <int R2, bool GAUSS, bool ENERGY>
__global__ __launch_bounds__(256, 2) void k_resident4(
    const SampleDesc *__restrict__ sd, const int32_t *__restrict__ ids,
    const ModelGeo *__restrict__ geo, float *__restrict__ state, int nsteps,
    double *__restrict__ ooi, double *__restrict__ energy, int64_t estride) {
    constexpr int N = 128, R = 4, B = 16;
    constexpr int M = Disc<R2>::M;
    constexpr int WIN = 2 * M + R;
    constexpr int WIN4 = (WIN + 3) / 4;  // 16-byte loads per window
    constexpr int Q = B + 2 * M;         // outputs fed by one band: its rows +- m
    constexpr int TW = resident4_row_stride(N, M);
    constexpr int NB = N / B;
    static_assert(resident4_fits(N, M, B), "partial sums must fit in the band's rows");
    static_assert(TW % 4 == 0 && M + 4 * 31 + 4 * WIN4 - M <= TW, "aligned windows");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[4];

    float *lds = reinterpret_cast<float *>(smem_raw);
    const int sidx = ids[blockIdx.x];
    const SampleDesc d = sd[sidx];
    float *g_state = state + d.offset;
    const int lane = threadIdx.x & 63;
    const int band = 2 * (threadIdx.x >> 6) + (lane >> 5);
    const int xb = 4 * (lane & 31);  // this lane's columns xb .. xb + 3
    const int y0 = band * B;
    const int bup = band + 1 < NB ? band + 1 : 0;  // the band below (rows y0 + B ..)
    const int bdn = band > 0 ? band - 1 : NB - 1;  // the band above

    const float ap = coef_ap<float>(d), bcoef = coef_b<float>(d), ce = geo_ce<float>(geo);
    float g[M + 1];
#pragma unroll
    for (int k = 0; k <= M; ++k) g[k] = GAUSS ? geo_g<float>(geo, k) : 1.0f;

    // Stores the 4 values of a lane at LDS element index i (i = row start +
    // m + column): one 16-byte store when m is a multiple of 4, else two
    // 8-byte or four 4-byte stores.
    auto put4 = [&](int i, const float *v) {
        if constexpr (M % 4 == 0) {
            *reinterpret_cast<float4 *>(lds + i) = make_float4(v[0], v[1], v[2], v[3]);
        } else if constexpr (M % 2 == 0) {
            reinterpret_cast<float2 *>(lds + i)[0] = make_float2(v[0], v[1]);
            reinterpret_cast<float2 *>(lds + i)[1] = make_float2(v[2], v[3]);
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) lds[i + c] = v[c];
        }
    };
    auto get4 = [&](int i, float *v) {
        if constexpr (M % 4 == 0) {
            const float4 t = *reinterpret_cast<const float4 *>(lds + i);
            v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
        } else if constexpr (M % 2 == 0) {
            const float2 t0 = reinterpret_cast<const float2 *>(lds + i)[0];
            const float2 t1 = reinterpret_cast<const float2 *>(lds + i)[1];
            v[0] = t0.x; v[1] = t0.y; v[2] = t1.x; v[3] = t1.y;
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] = lds[i + c];
        }
    };

    // Load and project u0 onto [-1, 1] (16-byte global loads, coalesced).
    float st[B][R];
#pragma unroll
    for (int q = 0; q < B; ++q) {
        const float4 t = *reinterpret_cast<const float4 *>(g_state + (int64_t)(y0 + q) * N + xb);
        st[q][0] = clamp1(t.x);
        st[q][1] = clamp1(t.y);
        st[q][2] = clamp1(t.z);
        st[q][3] = clamp1(t.w);
    }

    // With the energy trace one more pass evaluates E_h(u^nsteps) and keeps
    // the state.
    const int passes = nsteps + (ENERGY ? 1 : 0);
    for (int step = 0; step < passes; ++step) {
        // Publish the state; then the lanes at the lattice edge write the
        // periodic column halo in stores of their own.
#pragma unroll
        for (int q = 0; q < B; ++q) put4((y0 + q) * TW + M + xb, st[q]);
        if constexpr (M % 4 == 0) {
            // a lane's 4 columns are all halo columns or none
            if (xb < M || xb >= N - M) {
                const int xh = xb < M ? xb + N : xb - N;
#pragma unroll
                for (int q = 0; q < B; ++q) put4((y0 + q) * TW + M + xh, st[q]);
            }
        } else if (xb < M || xb + 4 > N - M) {
#pragma unroll
            for (int c = 0; c < R; ++c) {
                const int x = xb + c;
                if (x < M || x >= N - M) {
                    const int xh = x < M ? x + N : x - N;
#pragma unroll
                    for (int q = 0; q < B; ++q) lds[(y0 + q) * TW + M + xh] = st[q][c];
                }
            }
        }
        __syncthreads();

        // acc[M + q] collects output row y0 + q, q in [-m, B + m).
        float acc[Q][R];
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int c = 0; c < R; ++c) acc[q][c] = -0.0f;
        const float *rp0 = lds + y0 * TW + xb;
        float win[2][4 * WIN4];
        auto load_win = [&](const float *p, float *w) {
#pragma unroll
            for (int j = 0; j < WIN4; ++j) {
                const float4 t = reinterpret_cast<const float4 *>(p)[j];
                w[4 * j] = t.x;
                w[4 * j + 1] = t.y;
                w[4 * j + 2] = t.z;
                w[4 * j + 3] = t.w;
            }
        };
        load_win(rp0, win[0]);
#pragma unroll
        for (int i = 0; i < B; ++i) {
            asm volatile("" ::: "memory");
            if (i + 1 < B) load_win(rp0 + (i + 1) * TW, win[(i + 1) & 1]);
            // input row i feeds output q = i - dy
            row_windows_cols<R2, GAUSS, R>(win[i & 1], g, [&](int dy, int c) -> float & {
                return acc[M + i - dy][c];
            });
        }
        // Take the band's sites back into registers, then hand the
        // overhanging partial sums over in the band's own rows (each half of
        // a wave touches only its own band's rows, and one wave's LDS
        // operations complete in order).
#pragma unroll
        for (int q = 0; q < B; ++q) get4((y0 + q) * TW + M + xb, st[q]);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float *myup = lds + y0 * TW;
        float *mydn = myup + M * N;
        const float *above = lds + bdn * B * TW + M * N;
        const float *below = lds + bup * B * TW;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            *reinterpret_cast<float4 *>(myup + j * N + xb) =
                make_float4(acc[j][0], acc[j][1], acc[j][2], acc[j][3]);
            *reinterpret_cast<float4 *>(mydn + j * N + xb) =
                make_float4(acc[B + M + j][0], acc[B + M + j][1], acc[B + M + j][2],
                            acc[B + M + j][3]);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const float4 t = *reinterpret_cast<const float4 *>(above + j * N + xb);
            acc[M + j][0] += t.x;
            acc[M + j][1] += t.y;
            acc[M + j][2] += t.z;
            acc[M + j][3] += t.w;
        }
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const float4 t = *reinterpret_cast<const float4 *>(below + j * N + xb);
            acc[B + j][0] += t.x;
            acc[B + j][1] += t.y;
            acc[B + j][2] += t.z;
            acc[B + j][3] += t.w;
        }
        // the neighbours have read this band's rows before it publishes the
        // next state there
        __syncthreads();
        if constexpr (ENERGY) {
            // E_h of the state this pass started from, from the per-site
            // terms u Lsum and 1 - u^2 accumulated in FP64
            double e_ul = 0.0, e_pot = 0.0;
#pragma unroll
            for (int q = 0; q < B; ++q)
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    const float u = st[q][c];
                    e_ul += (double)u * (double)lsum_of(ce, u, acc[M + q][c]);
                    e_pot += 1.0 - (double)u * (double)u;
                }
            e_ul = block_sum(e_ul, red);
            e_pot = block_sum(e_pot, red);
            if (threadIdx.x == 0)
                energy[(int64_t)step * estride + sidx] = d.e_int * e_ul + d.e_pot * e_pot;
            if (step == nsteps) break;
        }
#pragma unroll
        for (int q = 0; q < B; ++q)
#pragma unroll
            for (int c = 0; c < R; ++c) {
                st[q][c] = update_g<float>(st[q][c], acc[M + q][c], ap, bcoef);
            }
    }

    // Write back and reduce the output of interest in FP64.
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < B; ++q) {
        *reinterpret_cast<float4 *>(g_state + (int64_t)(y0 + q) * N + xb) =
            make_float4(st[q][0], st[q][1], st[q][2], st[q][3]);
#pragma unroll
        for (int c = 0; c < R; ++c) part += (double)st[q][c];
    }
    const double tot = block_sum(part, red);
    if (threadIdx.x == 0) {
        const double mean = tot / ((double)N * N);
        ooi[2 * (int64_t)sidx] = mean;
        ooi[2 * (int64_t)sidx + 1] = 0.5 * (1.0 + mean);
    }
}

// Window sums of one input row for the C adjacent columns of a lane at once,
// constant kernel: the lane's window win[0 .. 2m + C) is split at
// s = m + C/2 into running sums leftwards from s - 1 and rightwards from s,
//     LS[j] = win[j] + ... + win[s - 1],   RS[j] = win[s] + ... + win[j],
// so that a column's window of half-width w that straddles the split,
// [m + c - w, m + c + w], sums to LS[m + c - w] + RS[m + c + w]: one addition
// per column and half-width used by the disc, after 2m + C - 2 additions
// shared by the C columns, instead of 2m per column.  Windows on one side of
// the split (w = 0, and w = 1 next to it) are summed directly.  acc(dy, c)
// names the accumulator of column c's output fed by disc row dy; each
// receives the window sum of its row's half-width.  The running sums have at
// most m + C/2 terms, like the window sums grown outwards from each column's
// centre, so the rounding is of the same size; its grouping differs.  (For
// m < 3 the shared sums cost as much as they save: not used there.)
template <int R2, int C, class Acc>
__device__ __forceinline__ void row_windows_split(const float *win, Acc &&acc) {
    using D = Disc<R2>;
    constexpr int M = D::M, S = M + C / 2, WIN = 2 * M + C;
    float LS[S], RS[WIN];  // LS[j] for j < S, RS[j] for j >= S
    LS[S - 1] = win[S - 1];
#pragma unroll
    for (int j = S - 2; j >= 0; --j) LS[j] = LS[j + 1] + win[j];
    RS[S] = win[S];
#pragma unroll
    for (int j = S + 1; j < WIN; ++j) RS[j] = RS[j - 1] + win[j];
    sfor<0, M + 1>([&](auto K) {
        constexpr int w = K;
        if constexpr (D::start[w] < D::start[w + 1]) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int lo = M + c - w, hi = M + c + w;
                float H;
                if (lo <= S - 1 && hi >= S) {
                    H = LS[lo] + RS[hi];
                } else {
                    H = win[lo];
#pragma unroll
                    for (int j = lo + 1; j <= hi; ++j) H += win[j];
                }
                sfor<D::start[w], D::start[w + 1]>([&](auto E) {
                    constexpr int dy = D::dy_by_w[E];
                    float &r = acc(dy, c);
                    r = r + H;
                });
            }
        }
    });
}

// ---------------------------------------------------------------------------
// Split-band variant (k_resident4h): four columns per lane as in
// k_resident4, but one 16-row band per wave whose two half-waves walk 8
// contiguous rows each (lanes 0-31 rows 0-7, lanes 32-63 rows 8-15).  A
// lane then keeps partial sums for 8 + 2m output rows instead of 16 + 2m, so
// the kernel fits 128 registers and a sample takes 8 waves: two samples per
// CU give four waves per SIMD (k_resident4: two), which a SIMD needs to keep
// its VALU issuing while some waves wait on LDS or barriers.
//
// LDS layout.  As in k_resident4 (rows of n values plus the periodic halo,
// 16-byte aligned windows), except that half 1 stores its 8 rows in its
// walk order: LDS row yh + k holds lattice row yh + H - 1 - k.  No other
// half reads a half's state rows, so the order is private, and every LDS
// address in the step loop is a per-lane base plus an immediate offset.
//
// Register naming.  Every lane runs the same instructions, so a register
// index names a different output row in each half: half 0 walks its rows
// downwards and acc[r] holds output row r - m of the half; half 1 walks its
// rows upwards (the disc is symmetric, so input row i + dy feeds output i
// with the weight of |dy| either way) and acc[r] holds output row
// H + m - 1 - r.  Then in both halves acc[0..m) are the sums that go to the
// neighbouring band (above for half 0, below for half 1), acc[m..H+m) the
// half's own rows, and acc[H+m..H+2m) the sums for the other half's rows,
// which arrive by one lane swap (v_permlane32_swap) per value.  The sums for
// the neighbouring bands are handed over in place, in the half's own rows
// (their values are back in registers by then).
// Each band sum is formed in two parts, so states differ from k_resident4's
// by FP32 rounding only.
//
// Volume constraint (VOL): Omega's 128 x 128 lattice inside a ring of m fixed
// rows and columns, stored (128 + 2m)^2.  The ring columns of Omega's rows
// fill the LDS halo once for the whole solve (the halo holds the periodic
// copies otherwise); the window sums of the m ring rows above and below are
// formed once into two blocks after the state rows, which Omega's first and
// last half-bands receive every step in place of a neighbour's hand-over.
// The hand-over then goes into the Omega columns of the half's rows (row
// stride n + 2m), so the ring columns are never overwritten; the periodic
// kernel packs it contiguously (row stride n) over a halo that the next
// publish rewrites anyway.
// ---------------------------------------------------------------------------
// The energy variant's FP64 sums do not fit the 128 registers of four waves
// per SIMD without spilling; it runs at two (one sample per CU).
template <int R2, bool GAUSS, bool ENERGY, bool VOL>
__global__ __launch_bounds__(512, ENERGY ? 2 : 4) void k_resident4h(
    const SampleDesc *__restrict__ sd, const int32_t *__restrict__ ids,
    const ModelGeo *__restrict__ geo, float *__restrict__ state, int nsteps,
    double *__restrict__ ooi, double *__restrict__ energy, int64_t estride) {
    constexpr int N = 128, R = 4, B = 16, H = 8;
    constexpr int M = Disc<R2>::M;
    constexpr int WIN4 = (2 * M + R + 3) / 4;  // 16-byte loads per window
    constexpr int Q = H + 2 * M;              // outputs fed by half a band
    constexpr int TW = resident4_row_stride(N, M);
    constexpr int NB = N / B;
    static_assert(M <= H && M * N <= H * TW, "partial sums must fit in the half-band's rows");
    static_assert(TW % 4 == 0 && 4 * 31 + 4 * WIN4 <= TW, "aligned windows");
    static_assert(!(VOL && ENERGY), "no energy trace under a volume constraint");
    // the stored array: Omega (N x N) inside a ring of m fixed rows and
    // columns under a volume constraint, else the periodic lattice itself
    constexpr int S = VOL ? N + 2 * M : N;
    constexpr int OFF = VOL ? M : 0;
    static_assert(!VOL || S <= TW, "the ring columns sit in the LDS halo");
    extern __shared__ __align__(16) unsigned char smem_raw[];

    float *lds = reinterpret_cast<float *>(smem_raw);
    // Under a volume constraint the LDS holds, after the state rows, the fixed
    // sums of the m ring rows above and below Omega (m rows of N each), and
    // no static area (two samples per CU fill the LDS): the final reduction
    // then uses the start of the state rows, which the solve no longer needs.
    double *red;
    if constexpr (VOL) {
        red = reinterpret_cast<double *>(smem_raw);
    } else {
        __shared__ double red_s[8];
        red = red_s;
    }
    const int sidx = ids[blockIdx.x];
    const SampleDesc d = sd[sidx];
    float *g_state = state + d.offset;
    const int lane = threadIdx.x & 63;
    const int band = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int half = lane >> 5;
    const int xb = 4 * (lane & 31);  // this lane's columns xb .. xb + 3
    const int y0 = band * B;
    // lattice row of this half's k-th site row (= LDS row yh + k): yh + k
    // (half 0) or yh + H - 1 - k (half 1), k = 0 .. H-1
    const int yh = y0 + H * half;
    const int rbase = half ? yh + H - 1 : yh;
    const int rstep = half ? -1 : 1;
    const int bup = band + 1 < NB ? band + 1 : 0;  // the band below
    const int bdn = band > 0 ? band - 1 : NB - 1;  // the band above
    // Sums this half receives: the band above's half 1 (for half 0), the
    // band below's half 0 (for half 1), each handed over in that half's own
    // rows (LDS rows from rrow).  Under a volume constraint the hand-over goes
    // through the Omega columns of those rows (LDS row rrow + j holds slot j;
    // the halo keeps the fixed ring columns), and Omega's first half-band
    // instead receives the fixed sums of the ring rows above it, its last
    // those of the ring rows below (blocks of m rows of N).
    const int rrow = half ? bup * B : bdn * B + H;
    const bool edge = VOL && ((band == 0 && !half) || (band == NB - 1 && half));
    const float *blk = lds + N * TW + (half ? M * N : 0);
    // periodic lattice: the hand-over blocks are m rows of N values from the
    // start of a half's rows (contiguous; the halo is rewritten every step)
    float *mine = lds + yh * TW;
    const float *recv = lds + rrow * TW;

    const float ap = coef_ap<float>(d), bcoef = coef_b<float>(d), ce = geo_ce<float>(geo);
    float g[M + 1];
#pragma unroll
    for (int k = 0; k <= M; ++k) g[k] = GAUSS ? geo_g<float>(geo, k) : 1.0f;

    auto put4 = [&](int i, const float *v) {
        if constexpr (M % 4 == 0) {
            *reinterpret_cast<float4 *>(lds + i) = make_float4(v[0], v[1], v[2], v[3]);
        } else if constexpr (M % 2 == 0) {
            reinterpret_cast<float2 *>(lds + i)[0] = make_float2(v[0], v[1]);
            reinterpret_cast<float2 *>(lds + i)[1] = make_float2(v[2], v[3]);
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) lds[i + c] = v[c];
        }
    };
    auto get4 = [&](int i, float *v) {
        if constexpr (M % 4 == 0) {
            const float4 t = *reinterpret_cast<const float4 *>(lds + i);
            v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
        } else if constexpr (M % 2 == 0) {
            const float2 t0 = reinterpret_cast<const float2 *>(lds + i)[0];
            const float2 t1 = reinterpret_cast<const float2 *>(lds + i)[1];
            v[0] = t0.x; v[1] = t0.y; v[2] = t1.x; v[3] = t1.y;
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] = lds[i + c];
        }
    };

    // Load and project u0 onto [-1, 1]; st[k] is site row rbase + k rstep.
    float st[H][R];
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const float *gp = g_state + (int64_t)(rbase + k * rstep + OFF) * S + xb + OFF;
        if constexpr (OFF % 4 == 0) {
            const float4 t = *reinterpret_cast<const float4 *>(gp);
            st[k][0] = clamp1(t.x);
            st[k][1] = clamp1(t.y);
            st[k][2] = clamp1(t.z);
            st[k][3] = clamp1(t.w);
        } else {
#pragma unroll
            for (int c = 0; c < R; ++c) st[k][c] = clamp1(gp[c]);
        }
    }

    if constexpr (VOL) {
        // The ring columns of this half's rows, projected, into the LDS halo
        // for the whole solve (and back to HBM); LDS column = stored column.
        for (int t = lane & 31; t < H * 2 * M; t += 32) {
            const int k = t / (2 * M), j = t - k * 2 * M;
            const int col = j < M ? j : N + j;
            float *gp = g_state + (int64_t)(rbase + k * rstep + M) * S + col;
            const float v = clamp1(*gp);
            lds[(yh + k) * TW + col] = v;
            *gp = v;
        }
        // The window sums of the ring rows, accumulated into the outputs of
        // Omega's first and last m rows (band 0: half 0 the ring above, half
        // 1 the ring below).  Half 1 walks the ring below from the bottom
        // up, and by the symmetry of the disc (row dy and row -dy have the
        // same half-width and weight) its register at[q] then collects
        // Omega row N - 1 - q, as half 0's collects row q: both halves run
        // the same code.  Stored as the hand-over blocks their receivers
        // read: slot j holds Omega row m - 1 - j (above) or N - m + j (below),
        // both at[m - 1 - j].
        if (band == 0) {
            float at[M][R];
#pragma unroll
            for (int q = 0; q < M; ++q)
#pragma unroll
                for (int c = 0; c < R; ++c) at[q][c] = -0.0f;
            sfor<0, M>([&](auto I) {
                constexpr int i = I;
                // stored row of ring row i: above Omega (Omega row i - m) or
                // below it (Omega row N + m - 1 - i)
                float *gp = g_state + (int64_t)(half ? N + 2 * M - 1 - i : i) * S + xb;
                float win[2 * M + R];
#pragma unroll
                for (int t = 0; t < 2 * M + R; ++t) win[t] = clamp1(gp[t]);
                // the projected ring rows back to HBM (the lanes' windows
                // overlap: lanes storing the same element store the same value)
#pragma unroll
                for (int t = 0; t < 2 * M + R; ++t) gp[t] = win[t];
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    float sink = 0.0f;
                    row_windows<R2, GAUSS>(win + c, g, [&](int dy) -> float & {
                        const int q = i - M - dy;  // output fed by disc row dy
                        return (q >= 0 && q < M) ? at[q][c] : sink;
                    });
                }
            });
            float *blk = lds + N * TW + (half ? M * N : 0);
#pragma unroll
            for (int j = 0; j < M; ++j)
                *reinterpret_cast<float4 *>(blk + j * N + xb) =
                    make_float4(at[M - 1 - j][0], at[M - 1 - j][1], at[M - 1 - j][2],
                                at[M - 1 - j][3]);
        }
    }

    // With the energy trace one more pass evaluates E_h(u^nsteps) and keeps
    // the state.
    const int passes = nsteps + (ENERGY ? 1 : 0);
    for (int step = 0; step < passes; ++step) {
        // Publish this half's rows; then the periodic column halo.  (Under a
        // volume constraint the halo holds the fixed ring columns.)
#pragma unroll
        for (int k = 0; k < H; ++k) put4((yh + k) * TW + M + xb, st[k]);
        if constexpr (!VOL && M % 4 == 0) {
            // The halo of the half's H rows is H * m/2 chunks of 4 values
            // (32 for m = 8): each lane copies at most one chunk from the
            // published row, one read and one write, instead of the edge
            // lanes' H stores that every lane would issue.  Chunk q of row k:
            // q < m/4 the left halo (LDS columns 4q.., copies of Omega columns
            // N - m + 4q..), else the right halo (LDS columns m + N + 4q'..,
            // copies of Omega columns 4q'.., q' = q - m/4).
            constexpr int QC = M / 2;
            static_assert(H * QC <= 32, "one chunk per lane of the half-wave");
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int hl = lane & 31;
            if (hl < H * QC) {
                const int k = hl / QC, q = hl - k * QC;
                const int left = q < QC / 2;
                const int dst = left ? 4 * q : M + N + 4 * (q - QC / 2);
                const int src = left ? N + 4 * q : M + 4 * (q - QC / 2);
                const float4 t = *reinterpret_cast<const float4 *>(lds + (yh + k) * TW + src);
                *reinterpret_cast<float4 *>(lds + (yh + k) * TW + dst) = t;
            }
        } else if (!VOL && (xb < M || xb + 4 > N - M)) {
#pragma unroll
            for (int c = 0; c < R; ++c) {
                const int x = xb + c;
                if (x < M || x >= N - M) {
                    const int xh = x < M ? x + N : x - N;
#pragma unroll
                    for (int k = 0; k < H; ++k) lds[(yh + k) * TW + M + xh] = st[k][c];
                }
            }
        }
        // the walk reads only rows this half-wave wrote
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        float acc[Q][R];
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int c = 0; c < R; ++c) acc[q][c] = -0.0f;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            // each row's window loads stay in its own iteration (registers);
            // arithmetic may still overlap neighbouring rows
            asm volatile("" ::: "memory");
            const float *rp = lds + (yh + i) * TW + xb;
            float win[4 * WIN4];
#pragma unroll
            for (int j = 0; j < WIN4; ++j) {
                const float4 t = reinterpret_cast<const float4 *>(rp)[j];
                win[4 * j] = t.x;
                win[4 * j + 1] = t.y;
                win[4 * j + 2] = t.z;
                win[4 * j + 3] = t.w;
            }
            if constexpr (GAUSS || M < 3) {
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    row_windows<R2, GAUSS>(win + c, g, [&](int dy) -> float & {
                        return acc[M + i - dy][c];
                    });
                }
            } else {
                row_windows_split<R2, R>(win, [&](int dy, int c) -> float & {
                    return acc[M + i - dy][c];
                });
            }
        }
        // The other half's sums for this half's rows: acc[H + m - 1 - k] +=
        // (the other half's acc[H + m + k]).  Swapping a value with itself
        // (v_permlane32_swap: the upper 32 lanes of the first operand trade
        // places with the lower 32 lanes of the second) leaves lanes 32-63's
        // value in lanes 0-31 of the second result and lanes 0-31's value in
        // lanes 32-63 of the first.
#pragma unroll
        for (int k = 0; k < M; ++k)
#pragma unroll
            for (int c = 0; c < R; ++c) {
                const unsigned x = __float_as_uint(acc[H + M + k][c]);
                const auto sw = __builtin_amdgcn_permlane32_swap(x, x, false, false);
                acc[H + M - 1 - k][c] += __uint_as_float(half ? sw[0] : sw[1]);
            }
        // Take this half's sites back (after the swaps have freed the other
        // half's sums: not scheduled earlier), then hand its sums for the
        // neighbouring band over in its own rows: slot j holds acc[j].
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < H; ++k) get4((yh + k) * TW + M + xb, st[k]);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if constexpr (VOL) {
                const float v[4] = {acc[j][0], acc[j][1], acc[j][2], acc[j][3]};
                put4((yh + j) * TW + M + xb, v);
            } else {
                *reinterpret_cast<float4 *>(mine + j * N + xb) =
                    make_float4(acc[j][0], acc[j][1], acc[j][2], acc[j][3]);
            }
        }
        __syncthreads();
        // slot j of the neighbour's half is its acc[j]: output row m - 1 - j
        // of that half's walk direction, this half's acc[2m - 1 - j]
#pragma unroll
        for (int j = 0; j < M; ++j) {
            float v[4];
            if (VOL && !edge) {
                get4((rrow + j) * TW + M + xb, v);
            } else {
                const float4 t =
                    *reinterpret_cast<const float4 *>((VOL ? blk : recv) + j * N + xb);
                v[0] = t.x;
                v[1] = t.y;
                v[2] = t.z;
                v[3] = t.w;
            }
            acc[2 * M - 1 - j][0] += v[0];
            acc[2 * M - 1 - j][1] += v[1];
            acc[2 * M - 1 - j][2] += v[2];
            acc[2 * M - 1 - j][3] += v[3];
        }
        // the neighbours have read this half's rows before it publishes the
        // next state there
        __syncthreads();
        if constexpr (ENERGY) {
            // E_h of the state this pass started from (per-site terms in FP64)
            double e_ul = 0.0, e_pot = 0.0;
#pragma unroll
            for (int k = 0; k < H; ++k)
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    const float u = st[k][c];
                    e_ul += (double)u * (double)lsum_of(ce, u, acc[M + k][c]);
                    e_pot += 1.0 - (double)u * (double)u;
                }
            e_ul = block_sum(e_ul, red);
            e_pot = block_sum(e_pot, red);
            if (threadIdx.x == 0)
                energy[(int64_t)step * estride + sidx] = d.e_int * e_ul + d.e_pot * e_pot;
            if (step == nsteps) break;
        }
#pragma unroll
        for (int k = 0; k < H; ++k)
#pragma unroll
            for (int c = 0; c < R; ++c) {
                st[k][c] = update_g<float>(st[k][c], acc[M + k][c], ap, bcoef);
            }
    }

    // the write-back addresses are formed afresh: the compiler would
    // otherwise keep the initial loads' 64-bit addresses through the whole
    // solve (spilled, at 32 bytes of scratch traffic per lane)
    int rb = rbase, rs = rstep, xw = xb;
    asm volatile("" : "+v"(rb), "+v"(rs), "+v"(xw));
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < H; ++k) {
        float *gp = g_state + (int64_t)(rb + k * rs + OFF) * S + xw + OFF;
        if constexpr (OFF % 4 == 0) {
            *reinterpret_cast<float4 *>(gp) = make_float4(st[k][0], st[k][1], st[k][2], st[k][3]);
        } else {
#pragma unroll
            for (int c = 0; c < R; ++c) gp[c] = st[k][c];
        }
#pragma unroll
        for (int c = 0; c < R; ++c) part += (double)st[k][c];
    }
    const double tot = block_sum(part, red);
    if (threadIdx.x == 0) {
        const double mean = tot / ((double)N * N);
        ooi[2 * (int64_t)sidx] = mean;
        ooi[2 * (int64_t)sidx + 1] = 0.5 * (1.0 + mean);
    }
}

#define NLCH_RESIDENT4_R2_LIST(X) X(1) X(4) X(9) X(16) X(25) X(64)

bool resident4_built(int R2) {
#define NLCH_X(v) \
    if (R2 == v) return resident4_fits(128, Disc<v>::M, 16);
    NLCH_RESIDENT4_R2_LIST(NLCH_X)
#undef NLCH_X
    return false;
}

template <int R2, bool GAUSS>
static hipError_t resident4_go(const Group &g, void *state, int nsteps, double *ooi,
                               hipStream_t s, double *energy, int64_t estride) {
    constexpr int M = Disc<R2>::M;
    if constexpr (resident4_fits(128, M, 16)) {
        constexpr size_t kLds = 160 * 1024;
        // a volume constraint: Omega (128^2) inside a ring of m, split bands,
        // the ring rows' fixed sums after the state rows
        const bool vol = g.lo != 0;
        const size_t lds4 =
            resident4_lds_bytes(128, M) + (vol ? (size_t)2 * M * 128 * sizeof(float) : 0);
        // rows per lane: 8 (split bands, 8 waves) unless 16 are asked for
        const bool split = vol || g.res_rows != 16;
        auto f = vol ? k_resident4h<R2, GAUSS, false, true>
                     : split ? (energy ? k_resident4h<R2, GAUSS, true, false>
                                       : k_resident4h<R2, GAUSS, false, false>)
                             : (energy ? k_resident4<R2, GAUSS, true> : k_resident4<R2, GAUSS, false>);
        if (g.ni != 128 || (vol && (g.lo != M || energy || g.n != 128 + 2 * M)) ||
            lds4 > kLds - 1024 ||
            (lds4 > 64 * 1024 &&
             hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)(kLds - 1024)) != hipSuccess))
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(f, dim3((unsigned)g.nids), dim3(split ? 512 : 256), lds4, s, g.sd,
                           g.ids, g.geo, (float *)state, nsteps, ooi, energy, estride);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

hipError_t resident4_launch_f32(const Group &g, void *state, int nsteps, double *ooi,
                                hipStream_t s, double *energy, int64_t estride) {
#define NLCH_X(v)                                                                         \
    if (g.R2 == v)                                                                        \
        return g.kernel == 1 ? resident4_go<v, true>(g, state, nsteps, ooi, s, energy, estride) \
                             : resident4_go<v, false>(g, state, nsteps, ooi, s, energy, estride);
    NLCH_RESIDENT4_R2_LIST(NLCH_X)
#undef NLCH_X
    return hipErrorInvalidValue;
}

}  // namespace nlch
