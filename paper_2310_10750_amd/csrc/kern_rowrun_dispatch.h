// Host-side launch logic of the row-run kernels for one (storage, arithmetic)
// type pair; included once per pair by the kern_rowrun_*.hip units so that the
// instantiations compile in parallel.
#pragma once

#include "kern_rowrun_impl.h"

namespace nlch {

// Horizons (as R2 = floor((delta n)^2)) with compiled row-run kernels.
#define NLCH_ROWRUN_R2_LIST(X) X(1) X(4) X(9) X(16) X(25) X(64) X(256) X(272) X(1024)
#define NLCH_RESIDENT_R2_LIST(X) X(1) X(4) X(9) X(16) X(25) X(64)

constexpr size_t kLdsBytes = 160 * 1024;

template <int R2>
struct RowrunShape {
    static constexpr int M = Disc<R2>::M;
    static constexpr int R = (M >= 24) ? 1 : 2;
    static constexpr int NW = (M >= 24) ? 2 : 4;
    static constexpr int TX = 64 * R;
    static constexpr int TW = TX + 2 * M;
};

template <int R2, class TS, class TA, bool GAUSS>
hipError_t rowrun_launch(const Group &g, const void *in, void *out, hipStream_t s) {
    using S = RowrunShape<R2>;
    constexpr int M = S::M;
    int B = (M >= 24) ? 64 : 32;
    while (B > 8 && (size_t)(S::NW * B + 2 * M) * S::TW * sizeof(TS) > kLdsBytes) B /= 2;
    while (B > 8 && S::NW * (B / 2) >= g.n) B /= 2;  // small lattices: short tiles
    const int TY = S::NW * B;
    const size_t lds = (size_t)(TY + 2 * M) * S::TW * sizeof(TS);
    if (lds > kLdsBytes) return hipErrorInvalidValue;
    const int tiles_x = (g.n + S::TX - 1) / S::TX;
    const int tiles_y = (g.n + TY - 1) / TY;
    const int tps = tiles_x * tiles_y;
    const int64_t nb = (int64_t)tps * g.nids;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    auto f = k_rowrun<R2, S::R, S::NW, TS, TA, GAUSS>;
    static bool attr = false;
    if (!attr) {
        hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kLdsBytes);
        attr = true;
    }
    hipLaunchKernelGGL(f, dim3((unsigned)nb), dim3(S::NW * 64), lds, s, g.sd, g.ids, g.geo,
                       (const TS *)in, (TS *)out, B, tiles_x, tps, (int)nb);
    return hipGetLastError();
}

// Resident layout: lanes own R adjacent columns, waves own bands of B rows.
inline void resident_shape(int n, int *R, int *B) {
    *R = n <= 64 ? 1 : 2;
    *B = 16;
}

template <int R2, class TS, class TA, bool GAUSS>
hipError_t resident_launch(const Group &g, void *state, int nsteps, double *ooi,
                           hipStream_t s) {
    constexpr int M = Disc<R2>::M;
    int R, B;
    resident_shape(g.n, &R, &B);
    const int tpb = ((g.n + R - 1) / R + 63) / 64 * 64;
    const int nbands = (g.n + B - 1) / B;
    const int threads = tpb * nbands;
    const size_t lds = (size_t)g.n * resident_row_stride(g.n, M) * sizeof(TS);
    if (threads > 512 || lds > kLdsBytes - 1024) return hipErrorInvalidValue;
    auto go = [&](auto f) {
        static bool attr = false;
        if (!attr) {
            hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(kLdsBytes - 1024));
            attr = true;
        }
        hipLaunchKernelGGL(f, dim3((unsigned)g.nids), dim3(threads), lds, s, g.sd, g.ids,
                           g.geo, (TS *)state, nsteps, ooi, tpb);
    };
    if (R == 1)
        go(k_resident<R2, 1, 16, TS, TA, GAUSS>);
    else
        go(k_resident<R2, 2, 16, TS, TA, GAUSS>);
    return hipGetLastError();
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
bool resident_has_typed(int R2, int n) {
    bool in_list = false;
#define NLCH_X(v) \
    if (R2 == v) in_list = true;
    NLCH_RESIDENT_R2_LIST(NLCH_X)
#undef NLCH_X
    // 16 <= n keeps the band walk within two periods of the torus
    if (!in_list || n > 128 || n < 16) return false;
    const int M = cisqrt(R2);
    return (size_t)n * resident_row_stride(n, M) * sizeof(TS) <= kLdsBytes - 1024;
}

template <class TS, class TA>
hipError_t rowrun_step_typed(const Group &g, const void *in, void *out, hipStream_t s) {
#define NLCH_X(v)                                                       \
    if (g.R2 == v)                                                      \
        return g.kernel == 1 ? rowrun_launch<v, TS, TA, true>(g, in, out, s) \
                             : rowrun_launch<v, TS, TA, false>(g, in, out, s);
    NLCH_ROWRUN_R2_LIST(NLCH_X)
#undef NLCH_X
    return hipErrorInvalidValue;
}

template <class TS, class TA>
hipError_t resident_typed(const Group &g, void *state, int nsteps, double *ooi,
                          hipStream_t s) {
#define NLCH_X(v)                                                                   \
    if (g.R2 == v)                                                                  \
        return g.kernel == 1 ? resident_launch<v, TS, TA, true>(g, state, nsteps, ooi, s) \
                             : resident_launch<v, TS, TA, false>(g, state, nsteps, ooi, s);
    NLCH_RESIDENT_R2_LIST(NLCH_X)
#undef NLCH_X
    return hipErrorInvalidValue;
}

}  // namespace nlch

// Defines the entry points of one type pair under the given suffix.
#define NLCH_ROWRUN_UNIT(SUFFIX, TS, TA)                                                    \
    namespace nlch {                                                                        \
    bool rowrun_has_##SUFFIX(int R2) { return rowrun_has_typed<TS, TA>(R2); }               \
    bool resident_has_##SUFFIX(int R2, int n) { return resident_has_typed<TS, TA>(R2, n); } \
    hipError_t rowrun_step_##SUFFIX(const Group &g, const void *in, void *out,              \
                                    hipStream_t s) {                                        \
        return rowrun_step_typed<TS, TA>(g, in, out, s);                                    \
    }                                                                                       \
    hipError_t resident_##SUFFIX(const Group &g, void *state, int nsteps, double *ooi,      \
                                 hipStream_t s) {                                           \
        return resident_typed<TS, TA>(g, state, nsteps, ooi, s);                            \
    }                                                                                       \
    }
