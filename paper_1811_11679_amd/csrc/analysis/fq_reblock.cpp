// On-the-fly blocking analysis of correlated estimator series (Sec. 3.1: the
// reblocking of Flyvbjerg and Petersen, accumulated as the data arrive, which
// lets a run stop once a requested statistical error is reached).
//
// Level 0 holds the raw observations; level k + 1 holds the averages of
// consecutive pairs of level-k values, (a + b) / 2, so a level-k value is the
// mean of a block of 2^k consecutive observations and an incomplete last block
// is left out, exactly as in the post-hoc analysis. Every level keeps the
// running mean and co-moment matrix of its values over all series (Welford's
// update), so its covariance of block means is available at any time in
// O(levels x series^2) memory, independent of the run length.
//
// Host code only: no device call, usable without a GPU.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../../include/fciqmc.h"

struct fq_reblock {
    int S = 0, L = 0;
    std::vector<int64_t> cnt;      // [L] values seen at each level
    std::vector<double> mean;      // [L][S]
    std::vector<double> comom;     // [L][S][S] sum of (x_i - mean_i)(x_j - mean_j)
    std::vector<double> pend;      // [L][S] first value of an incomplete pair
    std::vector<char> has;         // [L]
};

extern "C" {

fq_status fq_reblock_create(fq_reblock **out, int32_t n_series, int32_t n_levels)
{
    if (!out) return FQ_EINVAL;
    *out = nullptr;
    if (n_series < 1 || n_series > 64 || n_levels < 1 || n_levels > 62) return FQ_EINVAL;
    fq_reblock *r = new (std::nothrow) fq_reblock;
    if (!r) return FQ_EINVAL;
    r->S = n_series;
    r->L = n_levels;
    r->cnt.assign(n_levels, 0);
    r->mean.assign((size_t)n_levels * n_series, 0.0);
    r->comom.assign((size_t)n_levels * n_series * n_series, 0.0);
    r->pend.assign((size_t)n_levels * n_series, 0.0);
    r->has.assign(n_levels, 0);
    *out = r;
    return FQ_OK;
}

fq_status fq_reblock_add(fq_reblock *r, const double *x)
{
    if (!r || !x) return FQ_EINVAL;
    const int S = r->S;
    for (int s = 0; s < S; ++s)
        if (!std::isfinite(x[s])) return FQ_EINVAL;
    std::vector<double> v(x, x + S), d(S);
    for (int k = 0; k < r->L; ++k) {
        const int64_t n = ++r->cnt[k];
        double *m = &r->mean[(size_t)k * S];
        double *c = &r->comom[(size_t)k * S * S];
        for (int i = 0; i < S; ++i) {
            d[i] = v[i] - m[i];  // deviation from the old mean
            m[i] += d[i] / (double)n;
        }
        for (int i = 0; i < S; ++i)
            for (int j = 0; j < S; ++j) c[(size_t)i * S + j] += d[i] * (v[j] - m[j]);
        double *p = &r->pend[(size_t)k * S];
        if (!r->has[k]) {
            std::memcpy(p, v.data(), sizeof(double) * S);
            r->has[k] = 1;
            break;
        }
        for (int i = 0; i < S; ++i) v[i] = (p[i] + v[i]) * 0.5;  // the pair's average moves up a level
        r->has[k] = 0;
    }
    return FQ_OK;
}

fq_status fq_reblock_level(const fq_reblock *r, int32_t level, int64_t *n_blocks, double *mean, double *cov)
{
    if (!r || level < 0 || level >= r->L || !n_blocks) return FQ_EINVAL;
    const int S = r->S;
    const int64_t n = r->cnt[level];
    *n_blocks = n;
    if (mean) std::memcpy(mean, &r->mean[(size_t)level * S], sizeof(double) * S);
    if (cov) {
        const double *c = &r->comom[(size_t)level * S * S];
        for (int i = 0; i < S * S; ++i) cov[i] = n > 1 ? c[i] / (double)(n - 1) : NAN;
    }
    return FQ_OK;
}

// Smallest level whose block length B = 2^k satisfies B^3 > 2 n (e_k / e_0)^4,
// with n the number of observations and e_k the standard error of the mean
// estimated from level k (Lee, Needs and Towler, Phys. Rev. E 83, 066706).
fq_status fq_reblock_optimal(const fq_reblock *r, int32_t series, int32_t *level)
{
    if (!r || series < 0 || series >= r->S || !level) return FQ_EINVAL;
    *level = -1;
    const int S = r->S;
    const int64_t n0 = r->cnt[0];
    if (n0 < 2) return FQ_OK;
    auto se2 = [&](int k) { return r->comom[((size_t)k * S + series) * S + series] / (double)(r->cnt[k] - 1) / (double)r->cnt[k]; };
    const double e0 = se2(0);
    if (!(e0 > 0.0)) {
        *level = 0;  // a constant series: every level agrees
        return FQ_OK;
    }
    for (int k = 0; k < r->L && r->cnt[k] >= 2; ++k) {
        const double ratio2 = se2(k) / e0;
        if (std::ldexp(1.0, 3 * k) > 2.0 * (double)n0 * ratio2 * ratio2) {
            *level = k;
            return FQ_OK;
        }
    }
    return FQ_OK;
}

// Ratio of two series' means at one level and its standard error to first
// order (the projected energy: numerator and reference population averaged
// separately, then divided).
fq_status fq_reblock_ratio(const fq_reblock *r, int32_t level, int32_t num, int32_t den, double *ratio, double *err)
{
    if (!r || level < 0 || level >= r->L || num < 0 || num >= r->S || den < 0 || den >= r->S || !ratio || !err)
        return FQ_EINVAL;
    const int S = r->S;
    const int64_t n = r->cnt[level];
    const double *m = &r->mean[(size_t)level * S];
    const double *c = &r->comom[(size_t)level * S * S];
    const double a = m[num], b = m[den];
    *ratio = a / b;
    if (n < 2 || b == 0.0) {
        *err = NAN;
        return FQ_OK;
    }
    const double f = 1.0 / ((double)(n - 1) * (double)n);  // co-moment -> covariance of the means
    const double vaa = c[(size_t)num * S + num] * f, vbb = c[(size_t)den * S + den] * f, vab = c[(size_t)num * S + den] * f;
    const double q = a / b;
    const double v = (vaa - 2.0 * q * vab + q * q * vbb) / (b * b);
    *err = v > 0.0 ? std::sqrt(v) : 0.0;
    return FQ_OK;
}

void fq_reblock_destroy(fq_reblock *r) { delete r; }

}  // extern "C"
