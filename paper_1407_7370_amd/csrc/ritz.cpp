// Host-side tridiagonal eigenproblems of the Lanczos modes: the Ritz values
// and bounds of Sec. 2 eq. error_est.
#include "ritz.h"

#include "dirac_lanczos.h"

#include <algorithm>
#include <atomic>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <thread>

namespace dlh {

void tridiag_full(std::vector<double> d, std::vector<double> e, std::vector<double> &lam,
                  std::vector<double> &v)
{
    const int k = (int)d.size();
    v.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) v[(size_t)i * k + i] = 1.0;
    e.resize(k, 0.0);
    const double eps = 2.220446049250313e-16;
    int h = k - 1, iter = 0;
    while (h > 0) {
        if (std::fabs(e[h - 1]) <= eps * (std::fabs(d[h - 1]) + std::fabs(d[h]))) {
            e[h - 1] = 0.0;
            --h;
            iter = 0;
            continue;
        }
        if (++iter > 200) break;
        int l = h - 1;
        while (l > 0 && std::fabs(e[l - 1]) > eps * (std::fabs(d[l - 1]) + std::fabs(d[l]))) --l;
        const double delta = 0.5 * (d[h - 1] - d[h]);
        const double b2 = e[h - 1] * e[h - 1];
        const double mu = d[h] - b2 / (delta + std::copysign(std::sqrt(delta * delta + b2), delta));
        double x = d[l] - mu, z = e[l];
        for (int q = l; q < h; ++q) {
            const double r = std::hypot(x, z);
            double c = 1.0, s = 0.0;
            if (r != 0.0) {
                c = x / r;
                s = -z / r;
            }
            if (q > l) e[q - 1] = r;
            const double aq = d[q], aq1 = d[q + 1], bq = e[q];
            const double cc = c * c, ss = s * s, cs = c * s;
            d[q] = cc * aq - 2.0 * cs * bq + ss * aq1;
            d[q + 1] = ss * aq + 2.0 * cs * bq + cc * aq1;
            e[q] = cs * (aq - aq1) + (cc - ss) * bq;
            if (q + 1 < h) {
                const double bq1 = e[q + 1];
                x = e[q];
                z = -s * bq1;
                e[q + 1] = c * bq1;
            }
            for (int row = 0; row < k; ++row) {
                double &zq = v[(size_t)row * k + q], &zq1 = v[(size_t)row * k + q + 1];
                const double a0 = zq, a1 = zq1;
                zq = c * a0 - s * a1;
                zq1 = s * a0 + c * a1;
            }
        }
    }
    lam = d;
}

namespace {

constexpr double kEps = 2.220446049250313e-16;
constexpr int kShifts = 8;  // Sturm sequences evaluated side by side

// Number of eigenvalues at or below x[s] for kShifts shifts at once: the signs of
// the pivots of the LDL^T factorisation of T - x (Sturm's theorem); a pivot
// smaller than pivmin in magnitude is taken as -pivmin.  The shifts run
// interleaved so that the divisions of different sequences overlap.
void sturm_counts(const double *d, const double *e2, int k, const double *x, double pivmin, int *cnt)
{
    double q[kShifts];
    int c[kShifts];
    for (int s = 0; s < kShifts; ++s) {
        double t = d[0] - x[s];
        if (std::fabs(t) < pivmin) t = -pivmin;
        q[s] = t;
        c[s] = t < 0.0;
    }
    for (int i = 1; i < k; ++i) {
        const double di = d[i], b2 = e2[i - 1];
        for (int s = 0; s < kShifts; ++s) {
            double t = (di - x[s]) - b2 / q[s];
            if (std::fabs(t) < pivmin) t = -pivmin;
            q[s] = t;
            c[s] += t < 0.0;
        }
    }
    for (int s = 0; s < kShifts; ++s) cnt[s] = c[s];
}

struct Interval {
    double a, b;  // eigenvalues ca .. cb-1 (ascending order) lie in (a, b]
    int ca, cb;
};

// All eigenvalues in (lo, hi] by bisection, shared between eigenvalues until
// their intervals separate; each leaf is narrowed to a few units in the last
// place.  Values are returned ascending with multiplicity.
void bisect_window(const std::vector<double> &d, const std::vector<double> &e2, double lo, double hi, double pivmin,
                   std::vector<double> &lam)
{
    const int k = (int)d.size();
    lam.clear();
    double x[kShifts];
    int c[kShifts];
    // a zero pivot counts as negative, so count(x) is the number of eigenvalues
    // at or below x and the window is (lo, hi]
    for (int s = 0; s < kShifts; ++s) x[s] = s == 0 ? lo : hi;
    sturm_counts(d.data(), e2.data(), k, x, pivmin, c);
    if (c[1] <= c[0]) return;
    std::vector<Interval> work{{lo, hi, c[0], c[1]}}, batch;
    std::vector<std::pair<double, int>> leaves;
    while (!work.empty()) {
        batch.clear();
        while (!work.empty() && (int)batch.size() < kShifts) {
            const Interval iv = work.back();
            work.pop_back();
            const double mid = 0.5 * (iv.a + iv.b);
            const double width = iv.b - iv.a;
            if (width <= 2.0 * kEps * std::max(std::fabs(iv.a), std::fabs(iv.b)) + 2.0 * pivmin || mid <= iv.a ||
                mid >= iv.b)
                leaves.push_back({mid, iv.cb - iv.ca});
            else
                batch.push_back(iv);
        }
        if (batch.empty()) continue;
        // multisection: the kShifts points are shared out over the intervals
        // of the batch (kShifts / batch size interior points each, equally
        // spaced), so that a lone interval gains log2(kShifts + 1) bits a pass
        const int nb = (int)batch.size(), per = kShifts / nb;
        for (int s = 0; s < kShifts; ++s) {
            const int i = std::min(s / per, nb - 1), r = std::min(s - i * per, per - 1);
            const Interval &iv = batch[i];
            const double x_r = iv.a + (iv.b - iv.a) * ((double)(r + 1) / (double)(per + 1));
            x[s] = std::min(std::max(x_r, iv.a), iv.b);
        }
        sturm_counts(d.data(), e2.data(), k, x, pivmin, c);
        for (int i = 0; i < nb; ++i) {
            const Interval &iv = batch[i];
            double a = iv.a;
            int ca = iv.ca;
            for (int r = 0; r <= per; ++r) {
                const double b = r < per ? x[i * per + r] : iv.b;
                const int cb = r < per ? std::min(std::max(c[i * per + r], ca), iv.cb) : iv.cb;
                if (cb > ca && b > a) work.push_back({a, b, ca, cb});
                if (b > a) {
                    a = b;
                    ca = cb;
                }
            }
        }
    }
    std::sort(leaves.begin(), leaves.end());
    for (const auto &l : leaves)
        for (int r = 0; r < l.second; ++r) lam.push_back(l.first);
}

// LU factors with partial (row) pivoting of T - theta I for inverse
// iteration: row i of U holds u0 (column i), u1 (i+1) and u2 (i+2, non-zero
// only after an interchange); mult and swap record the elimination.
struct TriLU {
    std::vector<double> u0, u1, u2, mult;
    std::vector<char> swap;

    void factor(const std::vector<double> &d, const std::vector<double> &e, double theta, double tiny)
    {
        const int k = (int)d.size();
        u0.assign(k, 0.0);
        u1.assign(k, 0.0);
        u2.assign(k, 0.0);
        mult.assign(k, 0.0);
        swap.assign(k, 0);
        // the active row (the part of row i not yet eliminated): columns i, i+1
        double a0 = d[0] - theta, a1 = k > 1 ? e[0] : 0.0;
        for (int i = 0; i + 1 < k; ++i) {
            const double s0 = e[i], s1 = d[i + 1] - theta, s2 = i + 2 < k ? e[i + 1] : 0.0;  // row i+1 of T
            if (std::fabs(s0) > std::fabs(a0)) {
                const double l = a0 / s0;
                u0[i] = s0;
                u1[i] = s1;
                u2[i] = s2;
                mult[i] = l;
                swap[i] = 1;
                a0 = a1 - l * s1;
                a1 = -l * s2;
            } else {
                const double l = a0 != 0.0 ? s0 / a0 : 0.0;
                u0[i] = a0;
                u1[i] = a1;
                mult[i] = l;
                a0 = s1 - l * a1;
                a1 = s2;
            }
        }
        u0[k - 1] = a0;
        // a zero (or negligible) pivot becomes tiny: the solve then returns a
        // large multiple of the eigenvector instead of failing
        for (int i = 0; i < k; ++i)
            if (std::fabs(u0[i]) < tiny) u0[i] = u0[i] < 0.0 ? -tiny : tiny;
    }

    // b <- (T - theta I)^-1 b
    void solve(std::vector<double> &b) const
    {
        const int k = (int)u0.size();
        for (int i = 0; i + 1 < k; ++i) {
            if (swap[i]) {
                const double bi = b[i];
                b[i] = b[i + 1];
                b[i + 1] = bi - mult[i] * b[i + 1];
            } else {
                b[i + 1] -= mult[i] * b[i];
            }
        }
        for (int i = k - 1; i >= 0; --i) {
            double r = b[i];
            if (i + 1 < k) r -= u1[i] * b[i + 1];
            if (i + 2 < k) r -= u2[i] * b[i + 2];
            b[i] = r / u0[i];
        }
    }
};

double norm2(const std::vector<double> &x)
{
    double s = 0.0;
    for (double v : x) s += v * v;
    return std::sqrt(s);
}

}  // namespace

void tridiag_window(const std::vector<double> &d, const std::vector<double> &e, double lo, double hi, double group,
                    std::vector<double> &lam, std::vector<double> &zlast)
{
    const int k = (int)d.size();
    lam.clear();
    zlast.clear();
    if (k == 0 || !(hi >= lo)) return;
    if (k == 1) {
        if (d[0] >= lo && d[0] <= hi) {
            lam.push_back(d[0]);
            zlast.push_back(1.0);
        }
        return;
    }
    std::vector<double> e2(k - 1);
    double tnorm = 0.0, emax2 = 0.0;
    for (int i = 0; i < k; ++i) {
        const double el = i > 0 ? std::fabs(e[i - 1]) : 0.0, er = i + 1 < k ? std::fabs(e[i]) : 0.0;
        tnorm = std::max(tnorm, std::fabs(d[i]) + el + er);
        if (i + 1 < k) {
            e2[i] = e[i] * e[i];
            emax2 = std::max(emax2, e2[i]);
        }
    }
    const double pivmin = DBL_MIN * std::max(1.0, emax2);
    bisect_window(d, e2, lo, hi, pivmin, lam);
    const int nw = (int)lam.size();
    zlast.assign(nw, 0.0);
    if (nw == 0) return;

    const double gap_group = std::max(group, 1e-8 * tnorm);
    const double tiny = kEps * std::max(tnorm, DBL_MIN);
    const double accept = 1e3 * kEps * std::max(tnorm, DBL_MIN);  // residual ||(T - theta) x|| of an accepted x
    std::vector<std::vector<double>> grp;                         // unit vectors of the current group
    std::vector<double> x(k);
    TriLU lu;
    uint64_t seed = 0x9E3779B97F4A7C15ull;
    double prev = 0.0;
    for (int j = 0; j < nw; ++j) {
        double theta = lam[j];
        if (j > 0 && theta - lam[j - 1] > gap_group) grp.clear();
        // equal shifts would give equal vectors: separate them by a few ulps
        if (j > 0 && !grp.empty()) theta = std::max(theta, prev + 10.0 * kEps * std::max(std::fabs(theta), tnorm * 1e-3));
        prev = theta;
        lu.factor(d, e, theta, tiny);
        for (int i = 0; i < k; ++i) {  // a fixed pseudo-random start (xorshift64*)
            seed ^= seed >> 12;
            seed ^= seed << 25;
            seed ^= seed >> 27;
            x[i] = (double)((seed * 0x2545F4914F6CDD1Dull) >> 11) * (2.0 / 9007199254740992.0) - 1.0;
        }
        double nx = norm2(x);
        for (double &v : x) v /= nx;
        int extra = -1;  // iterations still to do after acceptance
        for (int it = 0; it < 8 && extra != 0; ++it) {
            lu.solve(x);
            for (const auto &g : grp) {
                double dot = 0.0;
                for (int i = 0; i < k; ++i) dot += g[i] * x[i];
                for (int i = 0; i < k; ++i) x[i] -= dot * g[i];
            }
            nx = norm2(x);
            if (!(nx > 0.0) || !std::isfinite(nx)) break;
            for (double &v : x) v /= nx;
            if (extra > 0)
                --extra;
            else if (extra < 0 && 1.0 / nx <= accept)
                extra = 1;
        }
        zlast[j] = x[k - 1];
        grp.push_back(x);
    }
}

int ritz_select(const std::vector<double> &lam, const std::vector<double> &zl, double beta_k, double e_lo,
                double e_hi, double tol, int n_wanted, double *evals, double *bounds, std::vector<int> *rep)
{
    // candidates in the window, ascending, with their index into lam
    std::vector<int> cand;
    for (int i = 0; i < (int)lam.size(); ++i)
        if (lam[i] >= e_lo && lam[i] <= e_hi) cand.push_back(i);
    std::sort(cand.begin(), cand.end(), [&](int a, int b) { return lam[a] < lam[b]; });
    int nf = 0;
    for (size_t a = 0; a < cand.size();) {
        size_t b = a + 1;
        while (b < cand.size() && lam[cand[b]] - lam[cand[b - 1]] <= tol) ++b;
        double sum = 0.0, t2s = 0.0;
        int best = cand[a];
        for (size_t c = a; c < b; ++c) {
            sum += lam[cand[c]];
            t2s += zl[cand[c]] * zl[cand[c]];
            if (std::fabs(zl[cand[c]]) < std::fabs(zl[best])) best = cand[c];
        }
        const double bound = std::fabs(beta_k) * std::sqrt(t2s);
        if (bound <= tol && nf < n_wanted) {
            evals[nf] = sum / (double)(b - a);
            bounds[nf] = bound;
            if (rep) rep->push_back(best);
            ++nf;
        }
        a = b;
    }
    return nf;
}

int ritz_chain(const double *alpha1, const double *beta1, int k, double e_lo, double e_hi, double tol, int n_wanted,
               double *evals, double *bounds, std::vector<int> *rep, std::vector<double> *V)
{
    std::vector<double> d(alpha1, alpha1 + k), e(k, 0.0), lam, zl;
    for (int j = 0; j + 1 < k; ++j) e[j] = beta1[j];
    if (V) {
        tridiag_full(d, e, lam, *V);
        zl.assign(V->begin() + (size_t)(k - 1) * k, V->begin() + (size_t)k * k);
    } else {
        tridiag_window(d, e, e_lo, e_hi, tol, lam, zl);
    }
    return ritz_select(lam, zl, beta1[k - 1], e_lo, e_hi, tol, n_wanted, evals, bounds, rep);
}

void merge_converged(std::vector<std::pair<double, double>> &found, const double *ev, const double *bd, int n,
                     double tol)
{
    for (int i = 0; i < n; ++i) {
        bool merged = false;
        for (auto &f : found)
            if (std::fabs(f.first - ev[i]) <= tol) {
                if (bd[i] < f.second) f = {ev[i], bd[i]};
                merged = true;
                break;
            }
        if (!merged) found.push_back({ev[i], bd[i]});
    }
    std::sort(found.begin(), found.end());
}

int host_threads()
{
    const unsigned n = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(n, 16u));
}

void converged_union(const double *alpha1, const double *beta1, int k, double e_lo, double e_hi, double tol,
                     int every, int threads, std::vector<std::pair<double, double>> &found)
{
    std::vector<int> marks;
    for (int j = every; j < k; j += every) marks.push_back(j);
    if (k > 0) marks.push_back(k);
    const int nm = (int)marks.size();
    std::vector<std::vector<double>> ev(nm), bd(nm);
    std::vector<int> nf(nm, 0);
    auto one = [&](int m) {
        const int j = marks[m];
        ev[m].assign(j, 0.0);
        bd[m].assign(j, 0.0);
        nf[m] = ritz_chain(alpha1, beta1, j, e_lo, e_hi, tol, j, ev[m].data(), bd[m].data(), nullptr, nullptr);
    };
    const int nt = std::max(1, std::min(threads, nm));
    if (nt == 1) {
        for (int m = 0; m < nm; ++m) one(m);
    } else {
        // largest blocks first; results merge in checkpoint order below
        std::atomic<int> next{0};
        std::vector<std::thread> pool;
        for (int t = 0; t < nt; ++t)
            pool.emplace_back([&] {
                for (int i; (i = next.fetch_add(1)) < nm;) one(nm - 1 - i);
            });
        for (auto &th : pool) th.join();
    }
    for (int m = 0; m < nm; ++m) merge_converged(found, ev[m].data(), bd[m].data(), nf[m], tol);
}

}  // namespace dlh

extern "C" dl_status dirac_lanczos_ritz(const double *alpha, const double *beta, int32_t k, double e_lo,
                                        double e_hi, double tol, int32_t check_every, int32_t n_wanted,
                                        double *evals, double *bounds, int32_t *n_found)
{
    if (!alpha || !beta || !evals || !bounds || !n_found || k < 1 || check_every < 0 || n_wanted < 1 ||
        !(tol >= 0.0) || !(e_hi >= e_lo))
        return DL_ERR_INVALID;
    std::vector<std::pair<double, double>> found;
    dlh::converged_union(alpha, beta, k, e_lo, e_hi, tol, check_every > 0 ? check_every : k, dlh::host_threads(),
                         found);
    const int nf = std::min((int)found.size(), (int)n_wanted);
    for (int i = 0; i < nf; ++i) {
        evals[i] = found[i].first;
        bounds[i] = found[i].second;
    }
    *n_found = nf;
    return DL_OK;
}
