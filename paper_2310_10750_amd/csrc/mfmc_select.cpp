// MFMC model selection and sample allocation (Sec. 3.1, 3.2 and the
// below-minimum-budget rule of Sec. 4), host code behind mfmc_select and
// mfmc_allocate in include/nlch.h.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "nlch.h"
#include "nlch_internal.h"

namespace {

int bad(const char *msg) { return nlch::set_error(NLCH_EINVAL, msg); }

// rho^2 of the model after position j of the subset (0 past the end).
double rho2_after(const std::vector<int> &sub, const double *rho, size_t j) {
    return j + 1 < sub.size() ? rho[sub[j + 1]] * rho[sub[j + 1]] : 0.0;
}

bool cond_a(const std::vector<int> &sub, const double *rho) {
    for (size_t j = 0; j + 1 < sub.size(); ++j)
        if (!(rho[sub[j]] * rho[sub[j]] > rho[sub[j + 1]] * rho[sub[j + 1]])) return false;
    return true;
}

bool cond_b(const std::vector<int> &sub, const double *cost, const double *rho) {
    for (size_t j = 1; j < sub.size(); ++j) {
        const double lhs = cost[sub[j - 1]] / cost[sub[j]];
        const double r2p = rho[sub[j - 1]] * rho[sub[j - 1]];
        const double r2c = rho[sub[j]] * rho[sub[j]];
        if (!(lhs > (r2p - r2c) / (r2c - rho2_after(sub, rho, j)))) return false;
    }
    return true;
}

double vratio(const std::vector<int> &sub, const double *cost, const double *rho) {
    double s = 0.0;
    for (size_t j = 0; j < sub.size(); ++j) {
        const double r2 = rho[sub[j]] * rho[sub[j]];
        s += std::sqrt(cost[sub[j]] / cost[0] * (r2 - rho2_after(sub, rho, j)));
    }
    return s * s;
}

}  // namespace

extern "C" int mfmc_select(int32_t K, const double *cost, const double *rho, mfmc_subset *out,
                           int32_t cap, int32_t *n_candidates) {
    if (K < 2 || K > NLCH_MFMC_MAX_POOL) return bad("K must be in [2, NLCH_MFMC_MAX_POOL]");
    if (!cost || !rho || (cap > 0 && !out) || cap < 0) return bad("null or invalid array");
    for (int k = 0; k < K; ++k) {
        if (!(std::isfinite(cost[k]) && cost[k] > 0.0)) return bad("costs must be > 0");
        if (!(std::isfinite(rho[k]) && std::fabs(rho[k]) <= 1.0))
            return bad("correlations must lie in [-1, 1]");
    }
    for (int k = 1; k < K; ++k)
        if (rho[k] * rho[k] > rho[0] * rho[0])
            return bad("model 0 must have the largest squared correlation");
    // decreasing rho^2, ties in pool order
    std::vector<int> order(K);
    for (int k = 0; k < K; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return rho[a] * rho[a] > rho[b] * rho[b]; });
    std::vector<int> pos(K);
    for (int k = 0; k < K; ++k) pos[order[k]] = k;

    struct Kept {
        std::vector<int> sub;
        double V, bmin;
    };
    std::vector<Kept> kept;
    const int ncand = (1 << (K - 1)) - 1;
    for (int mask = 1; mask <= ncand; ++mask) {
        std::vector<int> sub{0};
        for (int k = 0; k < K - 1; ++k)
            if (mask >> k & 1) sub.push_back(k + 1);
        std::sort(sub.begin(), sub.end(), [&](int a, int b) { return pos[a] < pos[b]; });
        if (sub[0] != 0) continue;
        if (!cond_a(sub, rho) || !cond_b(sub, cost, rho)) continue;
        const double V = vratio(sub, cost, rho);
        const double r2 = rho[sub[1]] * rho[sub[1]];
        kept.push_back({sub, V, std::sqrt(V / (1.0 - r2))});
    }
    std::stable_sort(kept.begin(), kept.end(), [](const Kept &a, const Kept &b) { return a.V < b.V; });
    for (int i = 0; i < (int)kept.size() && i < cap; ++i) {
        mfmc_subset &o = out[i];
        o.size = (int32_t)kept[i].sub.size();
        for (int j = 0; j < NLCH_MFMC_MAX_POOL; ++j)
            o.models[j] = j < o.size ? kept[i].sub[j] : -1;
        o.V = kept[i].V;
        o.bmin_over_c1 = kept[i].bmin;
    }
    if (n_candidates) *n_candidates = ncand;
    return (int)kept.size();
}

extern "C" int mfmc_allocate(int32_t S, const int32_t *subset, const double *cost,
                             const double *rho, double budget, double *m_real, int64_t *m_int,
                             double *m1_star) {
    if (S < 2 || S > NLCH_MFMC_MAX_POOL) return bad("S must be in [2, NLCH_MFMC_MAX_POOL]");
    if (!subset || !cost || !rho || !m_real || !m_int) return bad("null array");
    if (!(std::isfinite(budget) && budget > 0.0)) return bad("budget must be > 0");
    if (subset[0] != 0) return bad("the subset must start with model 0");
    std::vector<int> sub(subset, subset + S);
    for (int j = 0; j < S; ++j) {
        if (sub[j] < 0 || sub[j] >= NLCH_MFMC_MAX_POOL) return bad("model index out of range");
        if (!(std::isfinite(cost[sub[j]]) && cost[sub[j]] > 0.0)) return bad("costs must be > 0");
    }
    if (!cond_a(sub, rho)) return bad("squared correlations must strictly decrease");
    const double r22 = rho[sub[1]] * rho[sub[1]];
    std::vector<double> r(S), m(S);
    double denom = 0.0;
    for (int j = 0; j < S; ++j) {
        const double r2 = rho[sub[j]] * rho[sub[j]];
        r[j] = std::sqrt(cost[0] * (r2 - rho2_after(sub, rho, j)) / (cost[sub[j]] * (1.0 - r22)));
        denom += cost[sub[j]] * r[j];
    }
    const double m1 = budget / denom;
    for (int j = 0; j < S; ++j) m[j] = m1 * r[j];
    if (m1 < 1.0) {
        double floor_cost = 0.0;
        for (int l = 0; l < S; ++l) floor_cost += (l + 1) * cost[sub[l]];
        if (budget < floor_cost) return bad("budget below sum_l l C_{i_l}");
        for (;;) {
            int j = -1;
            for (int l = 0; l + 1 < S; ++l)
                if (m[l] < l + 1) {
                    j = l;
                    break;
                }
            if (j < 0) break;
            for (int l = 0; l <= j; ++l) m[l] = l + 1;
            const int head = sub[j + 1];
            const double gap = rho[head] * rho[head] - rho2_after(sub, rho, j + 1);
            double rest = budget, den2 = 0.0;
            for (int l = 0; l <= j; ++l) rest -= (l + 1) * cost[sub[l]];
            std::vector<double> rr(S, 0.0);
            for (int l = j + 1; l < S; ++l) {
                const double r2 = rho[sub[l]] * rho[sub[l]];
                rr[l] = std::sqrt(cost[head] * (r2 - rho2_after(sub, rho, l)) / (cost[sub[l]] * gap));
                den2 += cost[sub[l]] * rr[l];
            }
            const double mh = rest / den2;
            for (int l = j + 1; l < S; ++l) m[l] = mh * rr[l];
        }
    }
    for (int j = 0; j < S; ++j) {
        m_real[j] = m[j];
        m_int[j] = (int64_t)std::floor(m[j]);
    }
    if (m1_star) *m1_star = m1;
    return NLCH_OK;
}
