// Host-side launch logic of the row-run kernels for one (storage, arithmetic)
// type pair; included once per pair by the kern_rowrun_*.hip units so that the
// instantiations compile in parallel.
#pragma once

#include "kern_rowrun_impl.h"

namespace nlch {

// Horizons (as R2 = floor((delta n)^2)) with compiled row-run kernels: the
// recipes' horizons for every type pair, plus (units that define
// NLCH_ROWRUN_EXTRA_R2 before including this header) the other horizons of
// the nine (h, delta) models of the multifidelity study in Sec. 4
// (delta n = 11, 12, 22, 24).
#ifndef NLCH_ROWRUN_EXTRA_R2
#define NLCH_ROWRUN_EXTRA_R2(X)
#endif
#define NLCH_ROWRUN_R2_LIST(X) \
    X(1) X(4) X(9) X(16) X(25) X(64) X(256) X(272) X(1024) NLCH_ROWRUN_EXTRA_R2(X)
#define NLCH_RESIDENT_R2_LIST(X) X(1) X(4) X(9) X(16) X(25) X(64)

constexpr size_t kLdsBytes = 160 * 1024;

// Streaming shape (see stream_shape): lanes own R columns of a 64R-column
// strip (R = 2 halves the window reads per site, R = 1 halves the register
// ring); a band of B output rows is walked by W waves.  One wave per band
// (k_stream) repeats the 2m halo rows of every band; W > 1 waves (k_band,
// built for FP32 and m <= 32) share a band and hand partial sums over in LDS
// instead; PH = 2 (k_phase, FP32 arithmetic) lets the two halves of one wave
// walk alternate rows of a band over a 32R-column strip.  Shapes with W = 1
// and PH = 1 give bit-identical results for every (R, B): each site sums the
// same window sums in the same row order; with W > 1 the sums of the outputs
// next to a hand-over point, with PH = 2 every sum, are formed in two parts,
// which changes their rounding only.
template <int R2, int R, class TS, class TA, bool GAUSS>
hipError_t stream_launch(const Group &g, const StreamShape &sh, const void *in, void *out,
                         hipStream_t s, double *epart) {
    constexpr int P = Disc<R2>::P;
    const int TX = 64 * R / sh.PH;
    const int strips = (g.ni + TX - 1) / TX;
    const int bands = (g.ni + sh.B - 1) / sh.B;
    const int64_t nb = (int64_t)strips * bands * g.nids;
    if (nb > 0x7fffffff || sh.B < 1 || sh.W < 1 || sh.W > 8 || (sh.PH != 1 && sh.PH != 2))
        return hipErrorInvalidValue;
    if (sh.PH == 2) {
        if constexpr (sizeof(TA) == 4) {
            if (sh.W != 1) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_phase<R2, R, TS, TA, GAUSS>), dim3((unsigned)nb), dim3(64), 0,
                               s, g.sd, g.ids, g.geo, (const TS *)in, (TS *)out, sh.B, strips,
                               bands, (int)nb, epart);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (sh.W == 1) {
        hipLaunchKernelGGL((k_stream<R2, R, TS, TA, GAUSS>), dim3((unsigned)nb), dim3(64), 0, s,
                           g.sd, g.ids, g.geo, (const TS *)in, (TS *)out, sh.B, strips, bands,
                           (int)nb, epart);
        return hipGetLastError();
    }
    if constexpr (band_built(Disc<R2>::M, (int)sizeof(TA))) {
        const size_t lds = StreamLds<R2, R, TA>::bytes(sh.W);
        if (lds > kLdsBytes - 1024 ||
            lds != stream_lds_bytes(R, Disc<R2>::M, sh.W, (int)sizeof(TA)) ||
            sh.L % P != 0 || sh.L < P)
            return hipErrorInvalidValue;
        auto f = k_band<R2, R, TS, TA, GAUSS>;
        if (lds > 64 * 1024 &&
            hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(kLdsBytes - 1024)) != hipSuccess)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(f, dim3((unsigned)nb), dim3(64 * sh.W), lds, s, g.sd, g.ids, g.geo,
                           (const TS *)in, (TS *)out, sh.B, sh.L, strips, bands, (int)nb,
                           epart);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

template <int R2, class TS, class TA, bool GAUSS>
hipError_t rowrun_launch(const Group &g, const void *in, void *out, hipStream_t s,
                         double *epart) {
    const StreamShape sh = stream_shape(g);
    if (sh.R == 1) return stream_launch<R2, 1, TS, TA, GAUSS>(g, sh, in, out, s, epart);
    return stream_launch<R2, 2, TS, TA, GAUSS>(g, sh, in, out, s, epart);
}

// Resident layout: one wave per band of kResB rows, lanes own one (n = 64)
// or two (n = 128) adjacent columns; built for these two lattice sizes.
constexpr int kResB = 16;

// Band height of a resident group: 16 rows, or for FP32 64^2 periodic
// lattices the 8 or 32 rows, for FP64 ones the 8 rows, that
// nlch_set_resident_shape or the autotuner chose (m <= B: partial sums only
// reach the adjacent bands).
template <class TS, class TA>
int resident_band_rows(const Group &g, int M, bool vol) {
    if (g.ni != 64 || vol || M > g.res_rows) return kResB;
    if (std::is_same<TS, float>::value && std::is_same<TA, float>::value &&
        (g.res_rows == 8 || g.res_rows == 32))
        return g.res_rows;
    if (std::is_same<TS, double>::value && std::is_same<TA, double>::value && g.res_rows == 8)
        return 8;
    return kResB;
}

template <int R2, class TS, class TA, bool GAUSS>
hipError_t resident_launch(const Group &g, void *state, int nsteps, double *ooi,
                           hipStream_t s, double *energy, int64_t estride) {
    constexpr int M = Disc<R2>::M;
    const bool vol = g.lo != 0;  // Omega's g.ni x g.ni lattice inside a ring of m
    const int B = resident_band_rows<TS, TA>(g, M, vol);
    const int threads = 64 * (g.ni / B);
    const size_t lds =
        resident_lds_bytes(g.ni, M, B, sizeof(TS), sizeof(TA), energy != nullptr, vol);
    if ((g.ni != 64 && g.ni != 128) || (vol && (g.lo != M || energy)) ||
        lds > kLdsBytes - 1024)
        return hipErrorInvalidValue;
    auto go = [&](auto f) {
        // per kernel (every instantiation has the same pointer type, so no
        // per-type static flag here)
        if (lds > 64 * 1024 &&
            hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(kLdsBytes - 1024)) != hipSuccess)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(f, dim3((unsigned)g.nids), dim3(threads), lds, s, g.sd, g.ids,
                           g.geo, (TS *)state, nsteps, ooi, energy, estride);
        return hipGetLastError();
    };
    if (vol) {
        if constexpr (std::is_same<TS, float>::value && std::is_same<TA, float>::value) {
            // 128^2 Omega: four columns per lane in split bands, unless the
            // two-column layout is asked for
            if (g.ni == 128 && g.res_cols != 2 && g.res_rows != 16 && resident4_built(g.R2))
                return resident4_launch_f32(g, state, nsteps, ooi, s, energy, estride);
        }
        return g.ni == 64 ? go(k_resident<R2, 64, kResB, TS, TA, GAUSS, false, true>)
                          : go(k_resident<R2, 128, kResB, TS, TA, GAUSS, false, true>);
    }
    if constexpr (std::is_same<TS, float>::value && std::is_same<TA, float>::value) {
        // four columns per lane where built, unless two are asked for (with
        // or without the energy trace, so that the trace runs the layout of
        // the plain solve)
        if (g.ni == 128 && g.res_cols != 2 && resident4_built(g.R2))
            return resident4_launch_f32(g, state, nsteps, ooi, s, energy, estride);
        if constexpr (M <= 8) {
            if (g.ni == 64 && B == 8)
                return energy ? go(k_resident<R2, 64, 8, TS, TA, GAUSS, true, false>)
                              : go(k_resident<R2, 64, 8, TS, TA, GAUSS, false, false>);
        }
        if (g.ni == 64 && B == 32)
            return energy ? go(k_resident<R2, 64, 32, TS, TA, GAUSS, true, false>)
                          : go(k_resident<R2, 64, 32, TS, TA, GAUSS, false, false>);
    }
    if constexpr (std::is_same<TS, double>::value && std::is_same<TA, double>::value && M <= 8) {
        // FP64 64^2 in 8-row bands: 8 waves for one sample (latency)
        if (g.ni == 64 && B == 8)
            return energy ? go(k_resident<R2, 64, 8, TS, TA, GAUSS, true, false>)
                          : go(k_resident<R2, 64, 8, TS, TA, GAUSS, false, false>);
    }
    if (energy)
        return g.ni == 64 ? go(k_resident<R2, 64, kResB, TS, TA, GAUSS, true, false>)
                          : go(k_resident<R2, 128, kResB, TS, TA, GAUSS, true, false>);
    return g.ni == 64 ? go(k_resident<R2, 64, kResB, TS, TA, GAUSS, false, false>)
                      : go(k_resident<R2, 128, kResB, TS, TA, GAUSS, false, false>);
}

template <class TS, class TA>
bool rowrun_has_typed(int R2) {
#define NLCH_X(v) \
    if (R2 == v) return true;
    NLCH_ROWRUN_R2_LIST(NLCH_X)
#undef NLCH_X
    return false;
}

template <class TS, class TA>
bool resident_has_typed(int R2, int n, bool vol) {
    bool in_list = false;
#define NLCH_X(v) \
    if (R2 == v) in_list = true;
    NLCH_RESIDENT_R2_LIST(NLCH_X)
#undef NLCH_X
    // built for n = 64 and n = 128 (whole bands, one wave per band)
    if (!in_list || (n != 64 && n != 128)) return false;
    const int M = cisqrt(R2);
    return M <= kResB &&
           // the largest layout of the variants (the energy trace keeps a
           // separate exchange area)
           resident_lds_bytes(n, M, kResB, sizeof(TS), sizeof(TA), !vol, vol) <=
               kLdsBytes - 1024;
}

template <class TS, class TA>
hipError_t rowrun_step_typed(const Group &g, const void *in, void *out, hipStream_t s,
                             double *epart) {
#define NLCH_X(v)                                                              \
    if (g.R2 == v)                                                             \
        return g.kernel == 1 ? rowrun_launch<v, TS, TA, true>(g, in, out, s, epart) \
                             : rowrun_launch<v, TS, TA, false>(g, in, out, s, epart);
    NLCH_ROWRUN_R2_LIST(NLCH_X)
#undef NLCH_X
    return hipErrorInvalidValue;
}

template <class TS, class TA>
hipError_t resident_typed(const Group &g, void *state, int nsteps, double *ooi,
                          hipStream_t s, double *energy, int64_t estride) {
#define NLCH_X(v)                                                                      \
    if (g.R2 == v)                                                                     \
        return g.kernel == 1                                                           \
                   ? resident_launch<v, TS, TA, true>(g, state, nsteps, ooi, s, energy, \
                                                      estride)                         \
                   : resident_launch<v, TS, TA, false>(g, state, nsteps, ooi, s, energy, \
                                                       estride);
    NLCH_RESIDENT_R2_LIST(NLCH_X)
#undef NLCH_X
    return hipErrorInvalidValue;
}

}  // namespace nlch

#define NLCH_R2_ITEM(v) v,
// Defines the entry points of one type pair under the given suffix.
#define NLCH_ROWRUN_UNIT(SUFFIX, TS, TA)                                                    \
    namespace nlch {                                                                        \
    int rowrun_r2_##SUFFIX(int64_t *out, int cap) {                                         \
        const int64_t list[] = {NLCH_ROWRUN_R2_LIST(NLCH_R2_ITEM)};                         \
        const int cnt = (int)(sizeof(list) / sizeof(list[0]));                              \
        for (int i = 0; i < cnt && i < cap; ++i) out[i] = list[i];                          \
        return cnt;                                                                         \
    }                                                                                       \
    bool rowrun_has_##SUFFIX(int R2) { return rowrun_has_typed<TS, TA>(R2); }               \
    bool resident_has_##SUFFIX(int R2, int n, bool vol) {                                   \
        return resident_has_typed<TS, TA>(R2, n, vol);                                      \
    }                                                                                       \
    hipError_t rowrun_step_##SUFFIX(const Group &g, const void *in, void *out,              \
                                    hipStream_t s, double *epart) {                         \
        return rowrun_step_typed<TS, TA>(g, in, out, s, epart);                             \
    }                                                                                       \
    hipError_t resident_##SUFFIX(const Group &g, void *state, int nsteps, double *ooi,      \
                                 hipStream_t s, double *energy, int64_t estride) {          \
        return resident_typed<TS, TA>(g, state, nsteps, ooi, s, energy, estride);           \
    }                                                                                       \
    }
