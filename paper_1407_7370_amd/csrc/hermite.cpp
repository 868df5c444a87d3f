// Host runtime of the Hermite pseudospectral discretisation (Sec. 5): the
// collocation points and weights, the differentiation matrix, the device
// tables of a batch of problems, and the eigenvalue mode (Ritz values of the
// tridiagonal T from the device's Lanczos recurrence, Sec. 2 eq. error_est).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "context.h"

using namespace dlh;

namespace {

thread_local std::string g_herm_error;

dl_status herm_fail(dl_status s, const std::string &msg)
{
    g_herm_error = msg;
    return s;
}

const char *herm_validate(const dl_hermite_params &p)
{
    if (p.n < 16 || p.n > 64 || p.n % 16 != 0) return "n must be 16, 32, 48 or 64";
    if (!(p.scale > 0.0) || !std::isfinite(p.scale)) return "scale must be positive";
    if (!(p.c > 0.0) || !std::isfinite(p.c)) return "c must be positive";
    if (!(p.mass >= 0.0) || !std::isfinite(p.mass)) return "mass must be >= 0";
    if (!std::isfinite(p.charge) || !std::isfinite(p.bz)) return "charge and bz must be finite";
    if (p.chirality < -1 || p.chirality > 1) return "chirality must be -1, 0 or +1";
    if (p.pot_kind < 0 || p.pot_kind > 2) return "unknown pot_kind";
    if (p.pot_kind == 1 && !(p.pot_a != 0.0 && std::isfinite(p.pot_a) && std::isfinite(p.pot_z)))
        return "soft-core potential needs pot_a != 0";
    if (p.pot_kind == 2 && !(p.pot_z != 0.0 && std::isfinite(p.pot_z))) return "paper soft-core potential needs pot_z != 0";
    return nullptr;
}

// Orthonormal Hermite function values h_{n-1}(x), h_n(x) (recurrence).
void hermite_pair(int n, double x, double &hm1, double &hn)
{
    double a = std::pow(3.14159265358979323846, -0.25) * std::exp(-0.5 * x * x), b = 0.0;
    // a = h_k, b = h_{k-1}
    for (int k = 0; k < n; ++k) {
        const double next = std::sqrt(2.0 / (k + 1)) * x * a - std::sqrt((double)k / (k + 1)) * b;
        b = a;
        a = next;
    }
    hm1 = b;
    hn = a;
}

// Roots xi (ascending) of the n-th Hermite polynomial and the weights w_i of
// the collocation variables (Christoffel numbers of the Hermite functions):
// Golub-Welsch (eigenvalues of the Jacobi matrix with off-diagonal sqrt(k/2))
// polished by Newton steps on h_n, and w_i = 1 / (n h_{n-1}(xi_i)^2)
// (Christoffel-Darboux at the zeros of h_n).
void nodes(int n, std::vector<double> &xi, std::vector<double> &w)
{
    std::vector<double> d(n, 0.0), e(n, 0.0), lam, v;
    for (int k = 1; k < n; ++k) e[k - 1] = std::sqrt(0.5 * k);
    tridiag_full(d, e, lam, v);
    xi = lam;
    std::sort(xi.begin(), xi.end());
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double x = xi[i], hm1 = 0.0, hn = 0.0;
        for (int it = 0; it < 8; ++it) {
            hermite_pair(n, x, hm1, hn);
            const double dx = hn / (std::sqrt(2.0 * n) * hm1 - x * hn);  // h_n' = sqrt(2n) h_{n-1} - x h_n
            x -= dx;
            if (std::fabs(dx) <= 1e-16 * (1.0 + std::fabs(x))) break;
        }
        hermite_pair(n, x, hm1, hn);
        xi[i] = x;
        w[i] = 1.0 / (n * hm1 * hm1);
    }
}

// The device image of one problem: D~ / scale with D~_ij = (-1)^(i+j) /
// (xi_i - xi_j) (i != j; the derivative of the interpolant in the span of the
// first n Hermite functions, in the variables sqrt(w) f), and the nodes times
// scale.
// The nodes depend on n only: computed once per n for the process.
const std::vector<double> &cached_nodes(int n)
{
    static std::mutex mu;
    static std::map<int, std::vector<double>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(n);
    if (it == cache.end()) {
        std::vector<double> xi, w;
        nodes(n, xi, w);
        it = cache.emplace(n, std::move(xi)).first;
    }
    return it->second;
}

void tables(const dl_hermite_params &p, double *dm, double *x)
{
    const std::vector<double> xi = cached_nodes(p.n);
    for (int i = 0; i < p.n; ++i)
        for (int j = 0; j < p.n; ++j)
            dm[(size_t)i * p.n + j] = i == j ? 0.0 : (((i + j) & 1) ? -1.0 : 1.0) / ((xi[i] - xi[j]) * p.scale);
    for (int i = 0; i < p.n; ++i) x[i] = xi[i] * p.scale;
}

dl::HermOp make_hop(const dl_hermite_params &p, const double *dmat, const double *x)
{
    dl::HermOp o{};
    o.n = p.n;
    o.c = p.c;
    o.chi = p.chirality < 0 ? -1.0 : 1.0;
    o.mc2 = p.mass * p.c * p.c;
    o.bq = p.c * p.charge * p.bz * 0.5;
    o.pot_kind = p.pot_kind ? 1 : 0;
    if (p.pot_kind == 1) {
        o.vz = p.pot_z;
        o.va2 = p.pot_a * p.pot_a;
    } else if (p.pot_kind == 2) {
        o.vz = 1.5 * p.pot_z;
        o.va2 = 3.0 / (p.pot_z * p.pot_z);
    }
    o.dmat = dmat;
    o.x = x;
    return o;
}

// Workspace: the problem table, the run table, the pointer table and the
// per-problem D and nodes (one block, uploaded in one copy), then the alpha
// and beta arrays of every problem (one block, downloaded in one copy).
struct HermLayout {
    size_t ops = 0, runs = 0, ptrs = 0, tables_end = 0, ab0 = 0, total = 0;
    std::vector<size_t> dmat, x, ab;
};

HermLayout herm_plan(const dl_hermite_params *p, int np, int k_max)
{
    HermLayout L;
    size_t off = 0;
    L.ops = off;
    off = align256(off + sizeof(dl::HermOp) * np);
    L.runs = off;
    off = align256(off + sizeof(dl::HermRun) * np);
    L.ptrs = off;
    off = align256(off + sizeof(void *) * 2 * np);
    for (int i = 0; i < np; ++i) {
        const size_t n2 = (size_t)p[i].n * p[i].n;
        L.dmat.push_back(off);
        off = align256(off + sizeof(double) * n2);
        L.x.push_back(off);
        off = align256(off + sizeof(double) * p[i].n);
    }
    L.tables_end = off;
    L.ab0 = off;
    for (int i = 0; i < np; ++i) {
        L.ab.push_back(off);
        off += sizeof(double) * 2 * (size_t)std::max(k_max, 1);
    }
    L.total = align256(off);
    return L;
}

}  // namespace

extern "C" {

dl_status dirac_lanczos_hermite_nodes(int32_t n, double scale, double *x, double *w)
{
    if (n < 1 || n > 4096 || !(scale > 0.0) || !std::isfinite(scale) || !x || !w)
        return herm_fail(DL_ERR_INVALID, "need 1 <= n <= 4096, scale > 0 and output arrays");
    std::vector<double> xi, wi;
    nodes(n, xi, wi);
    for (int i = 0; i < n; ++i) {
        x[i] = xi[i] * scale;
        w[i] = wi[i] * scale;
    }
    return DL_OK;
}

size_t dirac_lanczos_hermite_workspace_bytes(const dl_hermite_params *params, int32_t n_problems, int32_t k_max)
{
    if (!params || n_problems < 1 || k_max < 1 || k_max > 1000000) return 0;
    for (int i = 0; i < n_problems; ++i)
        if (herm_validate(params[i])) return 0;
    return herm_plan(params, n_problems, k_max).total;
}

dl_status dirac_lanczos_hermite_apply(const dl_hermite_params *params, const void *x, void *y, void *workspace,
                                      size_t ws_bytes, void *hip_stream)
{
    if (!params) return herm_fail(DL_ERR_INVALID, "params is NULL");
    if (const char *m = herm_validate(*params)) return herm_fail(DL_ERR_INVALID, m);
    if (!x || !y || x == y) return herm_fail(DL_ERR_INVALID, "apply needs distinct non-NULL x and y");
    const HermLayout L = herm_plan(params, 1, 1);
    if (!workspace || ((uintptr_t)workspace & 255u) != 0 || ws_bytes < L.total)
        return herm_fail(DL_ERR_WORKSPACE, "workspace must be 256-byte aligned with " + std::to_string(L.total) +
                                               " bytes");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    char *ws = static_cast<char *>(workspace);
    std::vector<char> img(L.tables_end, 0);
    tables(*params, reinterpret_cast<double *>(img.data() + L.dmat[0]), reinterpret_cast<double *>(img.data() + L.x[0]));
    const dl::HermOp op = make_hop(*params, reinterpret_cast<double *>(ws + L.dmat[0]),
                                   reinterpret_cast<double *>(ws + L.x[0]));
    const void *ptrs[2] = {x, y};
    std::memcpy(img.data() + L.ops, &op, sizeof(op));
    std::memcpy(img.data() + L.ptrs, ptrs, sizeof(ptrs));
    if (hipMemcpyAsync(ws, img.data(), img.size(), hipMemcpyHostToDevice, st) != hipSuccess)
        return herm_fail(DL_ERR_DEVICE, "upload of the problem tables failed");
    const void *const *dp = reinterpret_cast<const void *const *>(ws + L.ptrs);
    dl::launch_herm_apply(reinterpret_cast<const dl::HermOp *>(ws + L.ops),
                          reinterpret_cast<const double2 *const *>(dp),
                          reinterpret_cast<double2 *const *>(const_cast<void **>(dp) + 1), 1, st);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        return herm_fail(DL_ERR_DEVICE, "kernel launch failed");
    return DL_OK;
}

dl_status dirac_lanczos_hermite_eigen(const dl_hermite_params *params, int32_t n_problems, const void *const *psi0,
                                      int32_t k_max, const double *e_lo, const double *e_hi, double tol,
                                      int32_t n_wanted, void *workspace, size_t ws_bytes, void *hip_stream,
                                      double *evals, double *bounds, int32_t *n_found)
{
    if (!params || n_problems < 1 || !psi0 || !e_lo || !e_hi || !evals || !bounds || !n_found || n_wanted < 1 ||
        k_max < 1 || k_max > 1000000 || !(tol >= 0.0))
        return herm_fail(DL_ERR_INVALID, "invalid Hermite eigen arguments");
    for (int i = 0; i < n_problems; ++i) {
        if (const char *m = herm_validate(params[i])) return herm_fail(DL_ERR_INVALID, m);
        if (!psi0[i] || !(e_hi[i] >= e_lo[i])) return herm_fail(DL_ERR_INVALID, "invalid start vector or window");
        n_found[i] = 0;
    }
    const HermLayout L = herm_plan(params, n_problems, k_max);
    if (!workspace || ((uintptr_t)workspace & 255u) != 0 || ws_bytes < L.total)
        return herm_fail(DL_ERR_WORKSPACE, "workspace must be 256-byte aligned with " + std::to_string(L.total) +
                                               " bytes");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    char *ws = static_cast<char *>(workspace);
    // host image of the tables block, uploaded in one copy
    std::vector<char> img(L.tables_end, 0);
    dl::HermOp *ops = reinterpret_cast<dl::HermOp *>(img.data() + L.ops);
    dl::HermRun *runs0 = reinterpret_cast<dl::HermRun *>(img.data() + L.runs);
    for (int i = 0; i < n_problems; ++i) {
        tables(params[i], reinterpret_cast<double *>(img.data() + L.dmat[i]),
               reinterpret_cast<double *>(img.data() + L.x[i]));
        ops[i] = make_hop(params[i], reinterpret_cast<double *>(ws + L.dmat[i]), reinterpret_cast<double *>(ws + L.x[i]));
        dl::HermRun r{};
        r.b = static_cast<const double2 *>(psi0[i]);
        r.alpha = reinterpret_cast<double *>(ws + L.ab[i]);
        r.beta = r.alpha + k_max;
        runs0[i] = r;
    }
    if (hipMemcpyAsync(ws, img.data(), img.size(), hipMemcpyHostToDevice, st) != hipSuccess)
        return herm_fail(DL_ERR_DEVICE, "upload of the problem tables failed");
    dl::launch_herm_lanczos(reinterpret_cast<const dl::HermOp *>(ws + L.ops), reinterpret_cast<dl::HermRun *>(ws + L.runs),
                            n_problems, k_max, st);
    if (hipGetLastError() != hipSuccess) return herm_fail(DL_ERR_DEVICE, "kernel launch failed");
    std::vector<double> ab((size_t)2 * k_max * n_problems);
    std::vector<dl::HermRun> runs(n_problems);
    if (hipMemcpyAsync(ab.data(), ws + L.ab0, sizeof(double) * ab.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(runs.data(), ws + L.runs, sizeof(dl::HermRun) * n_problems, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return herm_fail(DL_ERR_DEVICE, "synchronisation failed");
    bool nonfinite = false;
    for (int i = 0; i < n_problems; ++i) {
        if (runs[i].keff < 0) nonfinite = true;
        n_found[i] = 0;
    }
    // converged clusters accumulated over the leading blocks k = 64, 128, ...
    // and k; problems are independent and spread over host threads
    std::atomic<int> next{0};
    const int nt = std::max(1, std::min<int>(n_problems, host_threads()));
    const int per_problem = std::max(1, host_threads() / nt);  // a few problems: checkpoints in parallel too
    auto worker = [&] {
        for (int i; (i = next.fetch_add(1)) < n_problems;) {
            const int k = runs[i].keff;
            if (k <= 0) continue;
            const double *al = ab.data() + (size_t)2 * k_max * i, *be = al + k_max;
            std::vector<std::pair<double, double>> found;
            converged_union(al, be, k, e_lo[i], e_hi[i], tol, kEigenCheckEvery, per_problem, found);
            const int nf = std::min((int)found.size(), n_wanted);
            for (int r = 0; r < nf; ++r) {
                evals[(size_t)i * n_wanted + r] = found[r].first;
                bounds[(size_t)i * n_wanted + r] = found[r].second;
            }
            n_found[i] = nf;
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
    worker();
    for (auto &th : pool) th.join();
    if (nonfinite) return herm_fail(DL_ERR_NONFINITE, "non-finite Lanczos reduction in a Hermite problem");
    return DL_OK;
}

const char *dirac_lanczos_hermite_last_error(void) { return g_herm_error.c_str(); }

}  // extern "C"
