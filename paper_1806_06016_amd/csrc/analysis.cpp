// Population analysis on the host, FP64: errors of population averages under
// the correlations resampling creates, and the multiple-histogram (WHAM)
// refinement of the free energies recorded as sum ln Q.
//
// Paper: Christiansen, Weigel & Janke, arXiv:1806.06016 -- the paragraph on
// correlations after resampling (copies of one configuration are correlated;
// errors by binning over the population) and the paragraph on the recorded
// normalisers (sum ln Q gives ln Z(T_i) - ln Z(T_0) and the starting values of
// the WHAM self-consistency iterations).
//
// Every loop runs in a fixed order (WHAM: fixed chunks of samples, combined in
// chunk order, spread over threads), so results do not depend on the thread
// count.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <thread>
#include <utility>
#include <vector>

#include "pamd.h"

namespace {

constexpr int64_t kChunk = 4096;

// running log-sum-exp: value = m + ln s
struct Lse {
    double m = -std::numeric_limits<double>::infinity();
    double s = 0.0;
    void add(double x)
    {
        if (x <= m) {
            s += std::exp(x - m);
        } else {
            s = s * std::exp(m - x) + 1.0;
            m = x;
        }
    }
    void merge(const Lse& o)
    {
        if (o.s == 0.0)
            return;
        if (o.m <= m) {
            s += o.s * std::exp(o.m - m);
        } else {
            s = s * std::exp(m - o.m) + o.s;
            m = o.m;
        }
    }
    double value() const { return m + std::log(s); }
};

template <typename F>
void parallel_chunks(int64_t n_chunks, F&& f)
{
    unsigned hw = std::thread::hardware_concurrency();
    const int64_t nt = std::max<int64_t>(1, std::min<int64_t>(n_chunks, hw ? std::min(hw, 16u) : 1));
    if (nt == 1) {
        for (int64_t c = 0; c < n_chunks; ++c)
            f(c);
        return;
    }
    std::vector<std::thread> th;
    for (int64_t t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (int64_t c = t; c < n_chunks; c += nt)
                f(c);
        });
    for (auto& x : th)
        x.join();
}

struct WhamData {
    int32_t L;
    const double* beta;
    std::vector<double> lnN;
    std::vector<int64_t> start;   // sample offsets per temperature (size L + 1)
    const double* E;
    int64_t n;
};

bool wham_setup(int32_t n_temps, const double* beta, const int64_t* n_samples, const double* E, WhamData* w)
{
    if (n_temps < 1 || !beta || !n_samples || !E)
        return false;
    w->L = n_temps;
    w->beta = beta;
    w->E = E;
    w->lnN.resize(n_temps);
    w->start.assign(n_temps + 1, 0);
    for (int l = 0; l < n_temps; ++l) {
        if (n_samples[l] < 1 || !std::isfinite(beta[l]))
            return false;
        w->lnN[l] = std::log((double)n_samples[l]);
        w->start[l + 1] = w->start[l] + n_samples[l];
    }
    w->n = w->start[n_temps];
    for (int64_t i = 0; i < w->n; ++i)
        if (!std::isfinite(E[i]))
            return false;
    return true;
}

// ln D(E_i) = logsumexp_l (ln N_l - beta_l E_i - ln Z_l) for every sample
void wham_denominators(const WhamData& w, const double* lnZ, std::vector<double>& lnD)
{
    lnD.resize(w.n);
    const int64_t nc = (w.n + kChunk - 1) / kChunk;
    parallel_chunks(nc, [&](int64_t c) {
        const int64_t i1 = std::min(w.n, (c + 1) * kChunk);
        for (int64_t i = c * kChunk; i < i1; ++i) {
            Lse a;
            for (int l = 0; l < w.L; ++l)
                a.add(w.lnN[l] - w.beta[l] * w.E[i] - lnZ[l]);
            lnD[i] = a.value();
        }
    });
}

// logsumexp_i (-b E_i - ln D_i) over all samples, chunk partials combined in order
double wham_numerator(const WhamData& w, const std::vector<double>& lnD, double b, std::vector<Lse>& part)
{
    const int64_t nc = (w.n + kChunk - 1) / kChunk;
    part.assign(nc, Lse());
    parallel_chunks(nc, [&](int64_t c) {
        const int64_t i1 = std::min(w.n, (c + 1) * kChunk);
        Lse a;
        for (int64_t i = c * kChunk; i < i1; ++i)
            a.add(-b * w.E[i] - lnD[i]);
        part[c] = a;
    });
    Lse t;
    for (const Lse& p : part)
        t.merge(p);
    return t.value();
}

}  // namespace

extern "C" pamd_status pamd_family_error(const double* O, const int32_t* ancestor, int64_t R,
                                         pamd_family_stats* out)
{
    if (!O || !ancestor || R < 1 || !out)
        return PAMD_ERR_ARG;
    double sum = 0.0;
    for (int64_t j = 0; j < R; ++j) {
        if (!std::isfinite(O[j]))
            return PAMD_ERR_NONFINITE;
        sum += O[j];
    }
    const double mean = sum / (double)R;
    // families: slots sorted by ancestor (stable: slot order within a family)
    std::vector<std::pair<int32_t, int64_t>> key(R);
    for (int64_t j = 0; j < R; ++j)
        key[j] = {ancestor[j], j};
    std::stable_sort(key.begin(), key.end(),
                     [](const std::pair<int32_t, int64_t>& a, const std::pair<int32_t, int64_t>& b) {
                         return a.first < b.first;
                     });
    double ss = 0.0, sf = 0.0, sum_nu2 = 0.0, ent = 0.0;
    int64_t families = 0;
    for (int64_t j = 0; j < R; ++j) {
        const double d = O[j] - mean;
        ss += d * d;
    }
    for (int64_t a = 0; a < R;) {
        int64_t b = a;
        double s = 0.0;
        while (b < R && key[b].first == key[a].first) {
            s += O[key[b].second] - mean;
            ++b;
        }
        const double nu = (double)(b - a) / (double)R;
        sf += s * s;
        sum_nu2 += nu * nu;
        ent -= nu * std::log(nu);
        ++families;
        a = b;
    }
    const double denom = R > 1 ? (double)R * (double)(R - 1) : std::numeric_limits<double>::infinity();
    out->mean = mean;
    out->naive_se = std::sqrt(ss / denom);
    out->family_se = std::sqrt(sf / denom);
    out->rho_t = (double)R * sum_nu2;
    out->family_entropy = ent;
    out->families = families;
    return PAMD_OK;
}

extern "C" pamd_status pamd_binning_error(const double* O, int64_t R, int64_t bin, double* se)
{
    if (!O || !se || bin < 1 || R / bin < 2)
        return PAMD_ERR_ARG;
    const int64_t nb = R / bin;
    std::vector<double> m(nb);
    double tot = 0.0;
    for (int64_t k = 0; k < nb; ++k) {
        double s = 0.0;
        for (int64_t j = k * bin; j < (k + 1) * bin; ++j) {
            if (!std::isfinite(O[j]))
                return PAMD_ERR_NONFINITE;
            s += O[j];
        }
        m[k] = s / (double)bin;
        tot += m[k];
    }
    const double mm = tot / (double)nb;
    double v = 0.0;
    for (int64_t k = 0; k < nb; ++k)
        v += (m[k] - mm) * (m[k] - mm);
    *se = std::sqrt(v / (double)(nb - 1) / (double)nb);
    return PAMD_OK;
}

extern "C" pamd_status pamd_wham(int32_t n_temps, const double* beta, const int64_t* n_samples, const double* E,
                                 double* lnZ, int32_t max_iter, double tol, int32_t* iterations)
{
    WhamData w;
    if (!lnZ || max_iter < 1 || !(tol > 0.0) || !wham_setup(n_temps, beta, n_samples, E, &w))
        return PAMD_ERR_ARG;
    for (int l = 0; l < n_temps; ++l)
        if (!std::isfinite(lnZ[l]))
            return PAMD_ERR_ARG;
    std::vector<double> lnD, cur(lnZ, lnZ + n_temps), nxt(n_temps);
    std::vector<Lse> part;
    int32_t it = 0;
    while (it < max_iter) {
        ++it;
        wham_denominators(w, cur.data(), lnD);
        for (int k = 0; k < n_temps; ++k)
            nxt[k] = wham_numerator(w, lnD, beta[k], part);
        const double shift = cur[0] - nxt[0];
        double delta = 0.0;
        for (int k = 0; k < n_temps; ++k) {
            nxt[k] = k == 0 ? cur[0] : nxt[k] + shift;   // the gauge: ln Z_0 exactly as given
            delta = std::max(delta, std::fabs(nxt[k] - cur[k]));
        }
        cur.swap(nxt);
        if (delta < tol)
            break;
    }
    std::copy(cur.begin(), cur.end(), lnZ);
    if (iterations)
        *iterations = it;
    return PAMD_OK;
}

extern "C" pamd_status pamd_wham_average(int32_t n_temps, const double* beta, const int64_t* n_samples,
                                         const double* E, const double* lnZ, double beta_q, double* E_mean,
                                         double* E2_mean)
{
    WhamData w;
    if (!lnZ || !E_mean || !E2_mean || !std::isfinite(beta_q) || !wham_setup(n_temps, beta, n_samples, E, &w))
        return PAMD_ERR_ARG;
    std::vector<double> lnD;
    wham_denominators(w, lnZ, lnD);
    double mx = -std::numeric_limits<double>::infinity();
    for (int64_t i = 0; i < w.n; ++i)
        mx = std::max(mx, -beta_q * E[i] - lnD[i]);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t i = 0; i < w.n; ++i) {
        const double q = std::exp(-beta_q * E[i] - lnD[i] - mx);
        s0 += q;
        s1 += q * E[i];
        s2 += q * E[i] * E[i];
    }
    *E_mean = s1 / s0;
    *E2_mean = s2 / s0;
    return PAMD_OK;
}
