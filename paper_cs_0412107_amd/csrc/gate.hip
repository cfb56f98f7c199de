// The surrogate's gate: which rows may take the network's prediction of
// c_ii (C^-1)_ii and which go back to the sampler (eq 1/C).
//
// Fit: rows of validation matrices with sampler labels y (and their standard
// errors) are binned on two features, each by its quantile edges (the sorted
// values at floor(k N / bins), k = 1..bins-1; bin = number of edges <= x).  A
// bin's validated relative error is sqrt(max(sum r^2 - sum s^2, 0) / count)
// with r = (pred - y) / y and s = se / y: the observed spread less the part
// the label noise explains.  With ucb_z > 0 the error is replaced by an upper
// confidence bound: the bin's rows give a chi-square with count degrees of
// freedom for (sum of squared errors) / (true mean square), so dividing by
// that distribution's lower quantile (Wilson-Hilferty approximation) bounds
// the true error from above.  A bin needs the sampler when it holds fewer than
// min_rows rows or its error exceeds tol.  The outer bins are open-ended, so
// a row whose binning features lie outside the range the validation rows
// covered has no validated error at all: it goes to the sampler too.  Host
// code, float64, rows summed in order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mcinv.h"
#include "boundary.h"
#include "surrogate_internal.h"

struct mcinv_gate {
    mcinv_gate_config cfg{};
    std::vector<double> ea, eb, err;
    double lo_a = 0.0, hi_a = 0.0, lo_b = 0.0, hi_b = 0.0;   // validated feature ranges
    std::vector<int64_t> count;
    std::vector<uint8_t> fallback;
};

namespace {

void set_err(const std::string& m);

std::vector<double> quantile_edges(const float* X, int64_t N, int32_t f, int32_t bins)
{
    std::vector<double> v(N);
    for (int64_t i = 0; i < N; ++i) v[i] = (double)X[i * MCINV_N_FEATURES + f];
    std::sort(v.begin(), v.end());
    std::vector<double> e(bins - 1);
    for (int32_t k = 1; k < bins; ++k) e[k - 1] = v[(size_t)(((int64_t)k * N) / bins)];
    return e;
}

// Lower quantile of a chi-square with k degrees of freedom at the standard
// normal quantile -z (Wilson and Hilferty, 1931); floored at a small positive
// value for tiny k, where the cube can turn negative.
double chi2_lower(double k, double z)
{
    const double c = 2.0 / (9.0 * k);
    const double t = 1.0 - c - z * std::sqrt(c);
    return std::max(k * t * t * t, 1e-3);
}

int64_t bin_of(const std::vector<double>& edges, double x)
{
    return std::upper_bound(edges.begin(), edges.end(), x) - edges.begin();
}

thread_local std::string g_gerr;
void set_err(const std::string& m) { g_gerr = m; }

}  // namespace

namespace mcinv {

void gate_fallback_rows(const mcinv_gate* g, int64_t N, const float* X, int64_t ld, int32_t ca, int32_t cb,
                        uint8_t* fallback)
{
    const int32_t B = g->cfg.bins;
    for (int64_t i = 0; i < N; ++i) {
        const double xa = X[i * ld + ca];
        const double xb = X[i * ld + cb];
        if (!(xa >= g->lo_a && xa <= g->hi_a && xb >= g->lo_b && xb <= g->hi_b)) {
            fallback[i] = 1;   // NaN, or outside what the validation rows covered
            continue;
        }
        fallback[i] = g->fallback[(size_t)(bin_of(g->ea, xa) * B + bin_of(g->eb, xb))];
    }
}

int32_t gate_feature_a(const mcinv_gate* g) { return g->cfg.feature_a; }
int32_t gate_feature_b(const mcinv_gate* g) { return g->cfg.feature_b; }

}  // namespace mcinv

extern "C" {

mcinv_status mcinv_gate_fit(const mcinv_gate_config* cfg, int64_t N, const float* X, const double* pred,
                            const double* y, const double* y_se, mcinv_gate** out)
try {
    if (!cfg || !X || !pred || !y || !y_se || !out || N < 1) {
        set_err("mcinv_gate_fit: null argument or no rows");
        return MCINV_EINVAL;
    }
    *out = nullptr;
    if (cfg->feature_a < 0 || cfg->feature_a >= MCINV_N_FEATURES || cfg->feature_b < 0 ||
        cfg->feature_b >= MCINV_N_FEATURES || cfg->bins < 1 || cfg->bins > 256 || cfg->min_rows < 0 ||
        !(cfg->tol >= 0.0) || !(cfg->ucb_z >= 0.0) || !(cfg->ucb_z < 10.0)) {
        set_err("mcinv_gate_fit: bad configuration");
        return MCINV_EINVAL;
    }
    for (int64_t i = 0; i < N; ++i)
        if (!std::isfinite(X[i * MCINV_N_FEATURES + cfg->feature_a]) ||
            !std::isfinite(X[i * MCINV_N_FEATURES + cfg->feature_b]) || !(y[i] != 0.0) || !std::isfinite(y[i])) {
            set_err("mcinv_gate_fit: non-finite binning feature or zero / non-finite label at row " +
                    std::to_string(i));
            return MCINV_EINVAL;
        }
    std::unique_ptr<mcinv_gate> owner(new mcinv_gate());
    mcinv_gate* g = owner.get();
    g->cfg = *cfg;
    const int32_t B = cfg->bins;
    g->ea = quantile_edges(X, N, cfg->feature_a, B);
    g->eb = quantile_edges(X, N, cfg->feature_b, B);
    g->lo_a = g->hi_a = X[cfg->feature_a];
    g->lo_b = g->hi_b = X[cfg->feature_b];
    for (int64_t i = 1; i < N; ++i) {
        const double xa = X[i * MCINV_N_FEATURES + cfg->feature_a], xb = X[i * MCINV_N_FEATURES + cfg->feature_b];
        g->lo_a = std::min(g->lo_a, xa);
        g->hi_a = std::max(g->hi_a, xa);
        g->lo_b = std::min(g->lo_b, xb);
        g->hi_b = std::max(g->hi_b, xb);
    }
    std::vector<double> r2((size_t)B * B, 0.0), s2((size_t)B * B, 0.0);
    g->count.assign((size_t)B * B, 0);
    for (int64_t i = 0; i < N; ++i) {
        const int64_t b = bin_of(g->ea, X[i * MCINV_N_FEATURES + cfg->feature_a]) * B +
                          bin_of(g->eb, X[i * MCINV_N_FEATURES + cfg->feature_b]);
        const double r = (pred[i] - y[i]) / y[i], s = y_se[i] / y[i];
        g->count[b] += 1;
        r2[b] += r * r;
        s2[b] += s * s;
    }
    g->err.assign((size_t)B * B, INFINITY);
    g->fallback.assign((size_t)B * B, 1);
    for (size_t b = 0; b < g->err.size(); ++b) {
        if (g->count[b] > 0) {
            const double k = (double)g->count[b];
            const double q = cfg->ucb_z > 0.0 ? chi2_lower(k, cfg->ucb_z) : k;
            g->err[b] = std::sqrt(std::max(r2[b] - s2[b], 0.0) / q);
        }
        g->fallback[b] = (g->count[b] < cfg->min_rows || !(g->err[b] <= cfg->tol)) ? 1 : 0;
    }
    *out = owner.release();
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status, const std::string& m_) { set_err(m_); });
}

mcinv_status mcinv_gate_apply(const mcinv_gate* g, int64_t N, const float* X, uint8_t* fallback)
try {
    if (!g || (N > 0 && (!X || !fallback)) || N < 0) {
        set_err("mcinv_gate_apply: bad arguments");
        return MCINV_EINVAL;
    }
    mcinv::gate_fallback_rows(g, N, X, MCINV_N_FEATURES, g->cfg.feature_a, g->cfg.feature_b, fallback);
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status, const std::string& m_) { set_err(m_); });
}

mcinv_status mcinv_gate_read(const mcinv_gate* g, double* edges_a, double* edges_b, double* bin_err,
                             int64_t* bin_count, uint8_t* bin_fallback, double* range)
try {
    if (!g) {
        set_err("mcinv_gate_read: null gate");
        return MCINV_EINVAL;
    }
    if (edges_a) std::memcpy(edges_a, g->ea.data(), sizeof(double) * g->ea.size());
    if (edges_b) std::memcpy(edges_b, g->eb.data(), sizeof(double) * g->eb.size());
    if (bin_err) std::memcpy(bin_err, g->err.data(), sizeof(double) * g->err.size());
    if (bin_count) std::memcpy(bin_count, g->count.data(), sizeof(int64_t) * g->count.size());
    if (bin_fallback) std::memcpy(bin_fallback, g->fallback.data(), g->fallback.size());
    if (range) {
        range[0] = g->lo_a;
        range[1] = g->hi_a;
        range[2] = g->lo_b;
        range[3] = g->hi_b;
    }
    return MCINV_OK;
} catch (...) {
    return mcinv::exception_status([&](mcinv_status, const std::string& m_) { set_err(m_); });
}

void mcinv_gate_destroy(mcinv_gate* g) { delete g; }

const char* mcinv_gate_last_error(void) { return g_gerr.c_str(); }

}  // extern "C"
