// Batched propagation of independent packets (C ABI dirac_lanczos_batch_*):
// every packet has its own grid, fields, Krylov basis and scalars; all share
// the Krylov dimension, the precision and the boundary kind in y.  One step of
// the whole batch is m + 2 launches (iteration 1, iterations 2..m, the small
// exponentials, the recombination) whatever the number of packets.
//
// Launch shape.  The sweeps of all packets use one common number R of rows per
// chunk: the smallest power of two (>= 16) for which the batch has at most
// eight block entries per resident workgroup, or one chunk per strip when
// even that is more.  A packet's tasks (strip, chunk) are padded to a
// multiple of four so that a block entry's waves belong to one packet; the
// entries of a packet form a contiguous segment (partials slots).  The
// recombination gives every packet a number of workgroups proportional to its
// tiles (DL_BATCH_COMB_WGS_PER_CU workgroups per compute unit in total).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "context.h"

// Workgroups per compute unit of the batched recombination, shared among the
// packets in proportion to their tiles.
#ifndef DL_BATCH_COMB_WGS_PER_CU
#define DL_BATCH_COMB_WGS_PER_CU 4
#endif

// Fixed cost of one block entry of the resident sweeps, in rows of its march
// (the march starts a FIFO depth plus four rows early; the entry's table
// loads and its segment reduction), for balancing the entries.
#ifndef DL_BATCH_ENTRY_ROWS
#define DL_BATCH_ENTRY_ROWS 16
#endif

using namespace dlh;

struct dl_batch {
    int n = 0, m = 0;
    bool mixed = false, py = false;
    int terms = 0;  // site-dependent terms present in any packet (dl::kTermPot | dl::kTermB)
    std::vector<dl_params> p;
    std::vector<std::vector<double>> coef;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int cus = 256;
    // device tables (in the workspace)
    dl::BatchPacket *d_pk = nullptr;
    dl::BatchBlock *d_blk[dl::kGridKinds] = {nullptr, nullptr, nullptr};
    dl::BatchTask *d_task[2] = {nullptr, nullptr};
    int *d_wgf[2] = {nullptr, nullptr};  // per resident workgroup: first entry (and the end)
    int nwg[2] = {0, 0};                 // resident workgroups of the sweeps and of iteration 1
    double *partials = nullptr;
    double *fields = nullptr;     // n x 2 x kChunk
    dl::StepStat *stats = nullptr; // n x kChunk
    char *scalars = nullptr;       // n x scalar stride
    size_t sc_stride = 0;
    int nblk[dl::kGridKinds] = {0, 0, 0};
    size_t max_blocks[dl::kGridKinds] = {0, 0, 0};
    int rows = 0;  // rows per chunk of the sweeps
    std::vector<dl::BatchPacket> h_pk;
    std::vector<double> h_fields;
    std::vector<dl::StepStat> h_stats;
    std::vector<char> h_scalars;
    std::string err;

    dl_status fail(dl_status s, const std::string &msg)
    {
        err = msg;
        return s;
    }
    dl_status hip_fail(hipError_t e, const char *what)
    {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return DL_ERR_DEVICE;
    }
};

namespace {

thread_local std::string g_batch_init_error;

struct BatchPlan {
    // layout
    size_t pk = 0, blk[dl::kGridKinds] = {0, 0, 0}, task[2] = {0, 0}, wgf[2] = {0, 0}, partials = 0, fields = 0,
           stats = 0,
           scalars = 0, alpha = 0, gamma = 0, vecs = 0, total = 0;
    size_t sc_stride = 0, ab_stride = 0;
    std::vector<size_t> vec_off;  // per packet: state vector, then the basis
    size_t max_blocks[dl::kGridKinds] = {0, 0, 0};
};

// The potential or a potential table make the diagonal vary over the grid, a
// magnetic field the coupling.
int site_terms(const dl_params &p)
{
    return ((p.pot_kind != 0 || p.v_table != nullptr) ? dl::kTermPot : 0) | (p.bz != 0.0 ? dl::kTermB : 0);
}

int strips(int nx, int halo) { return (nx + (64 - 2 * halo) - 1) / (64 - 2 * halo); }

size_t ceil_div(size_t a, size_t b) { return (a + b - 1) / b; }

// Upper bounds of the tables (rows per chunk >= 4) and the workspace layout.
BatchPlan batch_plan(const dl_params *params, int n)
{
    BatchPlan B;
    const int m = params[0].krylov_dim;
    const bool mixed = params[0].precision == DL_PREC_MIXED;
    size_t off = 0;
    B.pk = off;
    off = align256(off + sizeof(dl::BatchPacket) * n);
    size_t tasks[2] = {0, 0}, cblk = 0;
    for (int i = 0; i < n; ++i) {
        const size_t rows4 = ceil_div((size_t)params[i].ny, 4);
        for (int k = 0; k < 2; ++k) {
            const size_t t = (size_t)strips(params[i].nx, k == 0 ? 2 : 1) * rows4;
            tasks[k] += ceil_div(t, dl::kWaves) * dl::kWaves;
        }
        const size_t sites = (size_t)params[i].nx * params[i].ny;
        cblk += ceil_div(sites, (size_t)dl::combine_tile_sites(mixed));
    }
    B.max_blocks[dl::kGridSweep] = tasks[0] / dl::kWaves;
    B.max_blocks[dl::kGridFirst] = tasks[1] / dl::kWaves;
    B.max_blocks[dl::kGridCombine] = cblk;
    for (int k = 0; k < dl::kGridKinds; ++k) {
        B.blk[k] = off;
        off = align256(off + sizeof(dl::BatchBlock) * B.max_blocks[k]);
    }
    for (int k = 0; k < 2; ++k) {
        B.task[k] = off;
        off = align256(off + sizeof(dl::BatchTask) * tasks[k]);
        B.wgf[k] = off;
        off = align256(off + sizeof(int) * (tasks[k] / dl::kWaves + 1));
    }
    const size_t maxb = std::max({B.max_blocks[0], B.max_blocks[1], B.max_blocks[2]});
    B.partials = off;
    off = align256(off + sizeof(double) * dl::kPartialStride * maxb);
    B.fields = off;
    off = align256(off + sizeof(double) * 2 * dl::kChunk * n);
    B.stats = off;
    off = align256(off + sizeof(dl::StepStat) * dl::kChunk * n);
    B.sc_stride = align256(sizeof(dl::Scalars));
    B.scalars = off;
    off += B.sc_stride * n;
    B.ab_stride = align256(sizeof(double) * (m + 3));
    B.alpha = off;
    off += B.ab_stride * n;
    B.gamma = off;
    off += B.ab_stride * n;
    B.vecs = off;
    const size_t belem = mixed ? 8 : 16;
    for (int i = 0; i < n; ++i) {
        const size_t ne = vec_elems(params[i]);
        B.vec_off.push_back(off);
        off += align256(ne * 16) + (size_t)(m - 1) * vec_stride(ne, belem);
    }
    B.total = off;
    return B;
}

const char *batch_validate(const dl_params *params, int n)
{
    if (!params) return "params is NULL";
    if (n < 1 || n > 65536) return "n_packets must be in 1..65536";
    for (int i = 0; i < n; ++i) {
        if (const char *msg = validate(&params[i])) return msg;
        if (params[i].krylov_dim != params[0].krylov_dim) return "all packets must share krylov_dim";
        if (params[i].precision != params[0].precision) return "all packets must share the precision";
    }
    return nullptr;
}

// Task and workgroup tables for rows_per_chunk R (0: the default choice):
// the smallest power of two >= 16 with at most eight block entries per
// resident workgroup, or one chunk per strip when even that is more (256
// packets of 128^2..512^2, 2 resident workgroups per CU, ms per step:
// R = 32 5.54, 64 5.58, 128 5.75).
dl_status build_tables(dl_batch *b, int rows_per_chunk)
{
    const int n = b->n;
    const std::vector<dl_params> &params = b->p;
    int R = rows_per_chunk;
    if (R <= 0) {
        const size_t target = (size_t)8 * dl::kBatchWgsPerCu * b->cus;
        int max_ny = 0;
        for (int i = 0; i < n; ++i) max_ny = std::max(max_ny, params[i].ny);
        R = 16;
        for (;;) {
            size_t e = 0;
            for (int i = 0; i < n; ++i)
                e += ceil_div((size_t)strips(params[i].nx, 2) * ceil_div(params[i].ny, R), dl::kWaves);
            if (e <= target || R >= max_ny) break;
            R *= 2;
        }
    }
    if (R < 4) return b->fail(DL_ERR_INVALID, "rows per chunk must be >= 4");
    b->rows = R;
    std::vector<dl::BatchBlock> blk[dl::kGridKinds];
    std::vector<dl::BatchTask> task[2];
    for (int k = 0; k < 2; ++k) {
        const int halo = k == 0 ? 2 : 1;
        const int kind = k == 0 ? dl::kGridSweep : dl::kGridFirst;
        for (int i = 0; i < n; ++i) {
            const int ns = strips(params[i].nx, halo), nch = (int)ceil_div(params[i].ny, R);
            const size_t first_task = task[k].size();
            for (int c = 0; c < nch; ++c)
                for (int s = 0; s < ns; ++s)
                    task[k].push_back(dl::BatchTask{s, c * R, std::min((c + 1) * R, params[i].ny), 0});
            while ((task[k].size() - first_task) % dl::kWaves) task[k].push_back(dl::BatchTask{0, 0, 0, 0});
            const int nb = (int)((task[k].size() - first_task) / dl::kWaves);
            const int first = (int)blk[kind].size();
            for (int l = 0; l < nb; ++l) blk[kind].push_back(dl::BatchBlock{i, l, nb, first});
            dl::Tiles &t = b->h_pk[i].tiles[k];
            t.halo = halo;
            t.own = 64 - 2 * halo;
            t.nstrips = ns;
            t.rows = R;
            t.nchunks = nch;
        }
    }
    {
        const int tile = dl::combine_tile_sites(b->mixed);
        size_t total_tiles = 0;
        std::vector<size_t> tiles(n);
        for (int i = 0; i < n; ++i) {
            tiles[i] = ceil_div((size_t)params[i].nx * params[i].ny, tile);
            total_tiles += tiles[i];
        }
        const double per = (double)(DL_BATCH_COMB_WGS_PER_CU * b->cus) / (double)total_tiles;  // workgroups per tile
        for (int i = 0; i < n; ++i) {
            int nb = (int)std::ceil(per * (double)tiles[i]);
            nb = std::max(1, std::min(nb, (int)tiles[i]));
            const int first = (int)blk[dl::kGridCombine].size();
            for (int l = 0; l < nb; ++l) blk[dl::kGridCombine].push_back(dl::BatchBlock{i, l, nb, first});
        }
    }
    // The entries of the resident sweeps are spread over the G resident
    // workgroups by longest-processing-time-first: in order of decreasing cost
    // (rows of the longest march plus a fixed cost per entry), each to the
    // workgroup with the least total so far.  A workgroup runs its entries as
    // one contiguous range of the list.  An entry keeps its packet segment and
    // index (partials slot and fold order), so the assignment changes no
    // result.
    const int pwg = dl::kBatchWgsPerCu * b->cus;
    std::vector<int> wgf[2];
    for (int k = 0; k < 2; ++k) {
        const int kind = k == 0 ? dl::kGridSweep : dl::kGridFirst;
        const size_t ne = blk[kind].size();
        std::vector<long> cost(ne, 0);
        std::vector<int> order(ne);
        for (size_t e = 0; e < ne; ++e) {
            order[e] = (int)e;
            int rows = 0;
            for (int w = 0; w < dl::kWaves; ++w) {
                const dl::BatchTask &t = task[k][e * dl::kWaves + w];
                rows = std::max(rows, t.y1 - t.y0);
            }
            cost[e] = rows + DL_BATCH_ENTRY_ROWS;
        }
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
        const int G = (int)std::min<size_t>(ne, (size_t)pwg);
        std::vector<long> load(G, 0);
        std::vector<std::vector<int>> own(G);
        // least-loaded workgroup, ties to the lowest index: a heap of (load, index)
        std::vector<std::pair<long, int>> heap;
        for (int g = 0; g < G; ++g) heap.push_back({0L, g});
        auto later = [](const std::pair<long, int> &x, const std::pair<long, int> &y) { return x > y; };
        std::make_heap(heap.begin(), heap.end(), later);
        for (size_t i = 0; i < ne; ++i) {
            std::pop_heap(heap.begin(), heap.end(), later);
            auto &h = heap.back();
            own[h.second].push_back(order[i]);
            h.first += cost[order[i]];
            std::push_heap(heap.begin(), heap.end(), later);
        }
        std::vector<dl::BatchBlock> nb;
        std::vector<dl::BatchTask> nt;
        nb.reserve(ne);
        nt.reserve(task[k].size());
        wgf[k].assign(1, 0);
        for (int g = 0; g < G; ++g) {
            for (int e : own[g]) {
                nb.push_back(blk[kind][e]);
                for (int w = 0; w < dl::kWaves; ++w) nt.push_back(task[k][(size_t)e * dl::kWaves + w]);
            }
            wgf[k].push_back((int)nb.size());
        }
        blk[kind].swap(nb);
        task[k].swap(nt);
        b->nwg[k] = G;
    }
    for (int k = 0; k < dl::kGridKinds; ++k) {
        if (blk[k].size() > b->max_blocks[k]) return b->fail(DL_ERR_WORKSPACE, "batch tables exceed the workspace");
        b->nblk[k] = (int)blk[k].size();
        DL_HIP(b, hipMemcpyAsync(b->d_blk[k], blk[k].data(), sizeof(dl::BatchBlock) * blk[k].size(),
                                 hipMemcpyHostToDevice, b->stream));
    }
    for (int k = 0; k < 2; ++k) {
        DL_HIP(b, hipMemcpyAsync(b->d_task[k], task[k].data(), sizeof(dl::BatchTask) * task[k].size(),
                                 hipMemcpyHostToDevice, b->stream));
        DL_HIP(b, hipMemcpyAsync(b->d_wgf[k], wgf[k].data(), sizeof(int) * wgf[k].size(), hipMemcpyHostToDevice,
                                 b->stream));
    }
    DL_HIP(b, hipStreamSynchronize(b->stream));
    return DL_OK;
}

}  // namespace

extern "C" {

size_t dirac_lanczos_batch_workspace_bytes(const dl_params *params, int32_t n_packets)
{
    if (batch_validate(params, n_packets)) return 0;
    return batch_plan(params, n_packets).total;
}

dl_status dirac_lanczos_batch_init(const dl_params *params, int32_t n_packets, void *workspace, size_t ws_bytes,
                                   void *hip_stream, dl_batch **out)
{
    if (!out) {
        g_batch_init_error = "out is NULL";
        return DL_ERR_INVALID;
    }
    *out = nullptr;
    if (const char *msg = batch_validate(params, n_packets)) {
        g_batch_init_error = msg;
        return DL_ERR_INVALID;
    }
    for (int i = 1; i < n_packets; ++i)
        if (params[i].bc_y != params[0].bc_y) {
            g_batch_init_error = "all packets of a batch must share bc_y";
            return DL_ERR_UNSUPPORTED;
        }
    const BatchPlan B = batch_plan(params, n_packets);
    if (!workspace || ((uintptr_t)workspace & 255u) != 0) {
        g_batch_init_error = "workspace must be a non-NULL, 256-byte aligned device pointer";
        return DL_ERR_WORKSPACE;
    }
    if (ws_bytes < B.total) {
        g_batch_init_error = "workspace too small: need " + std::to_string(B.total) + " bytes";
        return DL_ERR_WORKSPACE;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        g_batch_init_error = "no HIP device";
        return DL_ERR_DEVICE;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_batch_init_error = std::string("built for gfx950 only, device is ") + prop.gcnArchName;
        return DL_ERR_DEVICE;
    }
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, workspace) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        g_batch_init_error = "workspace is not device memory";
        return DL_ERR_WORKSPACE;
    }
    const int n = n_packets;
    dl_batch *b = new dl_batch();
    b->n = n;
    b->m = params[0].krylov_dim;
    b->mixed = params[0].precision == DL_PREC_MIXED;
    b->py = params[0].bc_y != 0;
    b->p.assign(params, params + n);
    b->coef.resize(n);
    for (int i = 0; i < n; ++i) {
        if (params[i].pulse_kind == DL_PULSE_FOURIER_SIN2)
            b->coef[i].assign(params[i].coef, params[i].coef + params[i].n_coef);
        b->p[i].coef = nullptr;
        b->terms |= site_terms(b->p[i]);
    }
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->ws = static_cast<char *>(workspace);
    b->ws_bytes = ws_bytes;
    b->cus = prop.multiProcessorCount;
    b->sc_stride = B.sc_stride;

    // packet table (the operator is filled per call, it depends on dt)
    b->h_pk.resize(n);
    const size_t belem = b->mixed ? 8 : 16;
    for (int i = 0; i < n; ++i) {
        dl::BatchPacket &pk = b->h_pk[i];
        std::memset(&pk, 0, sizeof(pk));
        const dl_params &pi = b->p[i];
        const size_t ne = vec_elems(pi);
        pk.psi = nullptr;
        pk.state = reinterpret_cast<double2 *>(b->ws + B.vec_off[i]);
        pk.basis = b->ws + B.vec_off[i] + align256(ne * 16);
        pk.vstride = vec_stride(ne, belem);
        pk.sites = ne / 2;
        pk.alpha = reinterpret_cast<double *>(b->ws + B.alpha + B.ab_stride * i);
        pk.gamma = reinterpret_cast<double *>(b->ws + B.gamma + B.ab_stride * i);
        pk.sc = reinterpret_cast<dl::Scalars *>(b->ws + B.scalars + B.sc_stride * i);
        pk.stats = reinterpret_cast<dl::StepStat *>(b->ws + B.stats) + (size_t)dl::kChunk * i;
        pk.fields = reinterpret_cast<double *>(b->ws + B.fields) + (size_t)2 * dl::kChunk * i;
        store_rounding(pi, pk.reps, pk.rabs);
    }
    b->d_pk = reinterpret_cast<dl::BatchPacket *>(b->ws + B.pk);
    for (int k = 0; k < dl::kGridKinds; ++k) {
        b->d_blk[k] = reinterpret_cast<dl::BatchBlock *>(b->ws + B.blk[k]);
        b->max_blocks[k] = B.max_blocks[k];
    }
    for (int k = 0; k < 2; ++k) {
        b->d_task[k] = reinterpret_cast<dl::BatchTask *>(b->ws + B.task[k]);
        b->d_wgf[k] = reinterpret_cast<int *>(b->ws + B.wgf[k]);
    }
    b->partials = reinterpret_cast<double *>(b->ws + B.partials);
    b->fields = reinterpret_cast<double *>(b->ws + B.fields);
    b->stats = reinterpret_cast<dl::StepStat *>(b->ws + B.stats);
    b->scalars = b->ws + B.scalars;
    const dl_status sb = build_tables(b, 0);
    if (sb != DL_OK) {
        g_batch_init_error = b->err;
        delete b;
        return sb;
    }
    *out = b;
    return DL_OK;
}

dl_status dirac_lanczos_batch_step(dl_batch *b, void *const *psi, double t0, double dt, int32_t n_steps,
                                   dl_step_stat *stats)
{
    if (!b) return DL_ERR_INVALID;
    if (!psi) return b->fail(DL_ERR_INVALID, "psi is NULL");
    for (int i = 0; i < b->n; ++i)
        if (!psi[i]) return b->fail(DL_ERR_INVALID, "psi[" + std::to_string(i) + "] is NULL");
    if (n_steps < 0) return b->fail(DL_ERR_INVALID, "n_steps must be >= 0");
    if (!(dt != 0.0) || !std::isfinite(dt) || !std::isfinite(t0))
        return b->fail(DL_ERR_INVALID, "dt must be finite and non-zero, t0 finite");
    if (n_steps == 0) return DL_OK;
    const int n = b->n, m = b->m;
    hipStream_t st = b->stream;
    for (int i = 0; i < n; ++i) {
        b->h_pk[i].op = make_op(b->p[i], dt);
        b->h_pk[i].psi = static_cast<double2 *>(psi[i]);
    }
    DL_HIP(b, hipMemcpyAsync(b->d_pk, b->h_pk.data(), sizeof(dl::BatchPacket) * n, hipMemcpyHostToDevice, st));
    dl::launch_reset_batch(b->d_pk, n, st);
    DL_HIP(b, hipGetLastError());
    b->h_fields.resize((size_t)2 * dl::kChunk * n);
    b->h_stats.resize((size_t)dl::kChunk * n);
    b->h_scalars.resize(b->sc_stride * n);
    std::vector<int> completed(n, 0);
    std::vector<double> cum(n, 0.0);
    bool any_abort = false;
    dl::BatchArgs a{};
    a.pk = b->d_pk;
    a.partials = b->partials;
    a.m = m;
    for (int s0 = 0; s0 < n_steps; s0 += dl::kChunk) {
        const int nc = std::min(dl::kChunk, n_steps - s0);
        for (int i = 0; i < n; ++i) {
            const double kf = -dt * b->p[i].c * b->p[i].charge;
            for (int j = 0; j < nc; ++j) {
                double av[2];
                pulse_average(b->p[i], b->coef[i], t0 + (double)(s0 + j) * dt, dt, av);
                b->h_fields[(size_t)2 * dl::kChunk * i + 2 * j] = kf * av[0];
                b->h_fields[(size_t)2 * dl::kChunk * i + 2 * j + 1] = kf * chir(b->p[i]) * av[1];
            }
        }
        DL_HIP(b, hipMemcpy2DAsync(b->fields, sizeof(double) * 2 * dl::kChunk, b->h_fields.data(),
                                   sizeof(double) * 2 * dl::kChunk, sizeof(double) * 2 * nc, n, hipMemcpyHostToDevice,
                                   st));
        for (int j = 0; j < nc; ++j) {
            a.step = j;
            a.parity = (s0 + j) & 1;
            a.pass = 1;
            a.blocks = b->d_blk[dl::kGridFirst];
            a.tasks = b->d_task[1];
            a.wg_first = b->d_wgf[1];
            a.ntasks = b->nblk[dl::kGridFirst];
            dl::launch_first_batch(a, b->nwg[1], b->py, b->terms, st);
            a.blocks = b->d_blk[dl::kGridSweep];
            a.tasks = b->d_task[0];
            a.wg_first = b->d_wgf[0];
            a.ntasks = b->nblk[dl::kGridSweep];
            for (int p = 2; p <= m; ++p) {
                a.pass = p;
                dl::launch_recur_batch(a, b->nwg[0], b->mixed, b->py, b->terms, st);
            }
            dl::launch_tridiag_batch(a, n, st);
            a.blocks = b->d_blk[dl::kGridCombine];
            a.tasks = nullptr;
            a.wg_first = nullptr;
            dl::launch_combine_batch(a, b->nblk[dl::kGridCombine], b->mixed, st);
        }
        DL_HIP(b, hipGetLastError());
        DL_HIP(b, hipMemcpy2DAsync(b->h_stats.data(), sizeof(dl::StepStat) * dl::kChunk, b->stats,
                                   sizeof(dl::StepStat) * dl::kChunk, sizeof(dl::StepStat) * nc, n,
                                   hipMemcpyDeviceToHost, st));
        DL_HIP(b, hipMemcpyAsync(b->h_scalars.data(), b->scalars, b->sc_stride * n, hipMemcpyDeviceToHost, st));
        DL_HIP(b, hipStreamSynchronize(st));
        for (int i = 0; i < n; ++i) {
            const dl::Scalars &hs = *reinterpret_cast<const dl::Scalars *>(b->h_scalars.data() + b->sc_stride * i);
            const int done_here = hs.steps_done - completed[i];
            for (int j = 0; j < nc && stats; ++j) {
                dl_step_stat &o = stats[(size_t)i * n_steps + s0 + j];
                const dl::StepStat &h = b->h_stats[(size_t)dl::kChunk * i + j];
                if (j < done_here) {
                    cum[i] += h.err_est;
                    o.k_eff = h.keff;
                    o.err_est = h.err_est;
                    o.cum_bound = cum[i];
                    o.norm2 = h.norm2;
                    o.round_bound = h.round_bound;
                } else {
                    o.k_eff = -1;
                    o.err_est = o.cum_bound = o.norm2 = o.round_bound = 0.0;
                }
            }
            completed[i] = hs.steps_done;
            if (hs.status != 0) any_abort = true;
        }
    }
    // the state of a packet after an odd number of completed steps is in the workspace
    for (int i = 0; i < n; ++i)
        if (completed[i] % 2 == 1)
            DL_HIP(b, hipMemcpyAsync(psi[i], b->h_pk[i].state, vec_elems(b->p[i]) * 16, hipMemcpyDeviceToDevice, st));
    DL_HIP(b, hipStreamSynchronize(st));
    if (any_abort) {
        std::string who;
        for (int i = 0; i < n; ++i)
            if (completed[i] < n_steps) who += (who.empty() ? "" : ", ") + std::to_string(i);
        return b->fail(DL_ERR_NONFINITE, "non-finite Lanczos reduction in packet(s) " + who);
    }
    return DL_OK;
}

dl_status dirac_lanczos_batch_set_launch(dl_batch *b, int32_t rows_per_chunk, int32_t *rows_out)
{
    if (!b) return DL_ERR_INVALID;
    const dl_status s = build_tables(b, rows_per_chunk);
    if (s == DL_OK && rows_out) *rows_out = b->rows;
    return s;
}

dl_status dirac_lanczos_batch_destroy(dl_batch *b)
{
    delete b;
    return DL_OK;
}

const char *dirac_lanczos_batch_last_error(const dl_batch *b)
{
    if (!b) return g_batch_init_error.c_str();
    return b->err.c_str();
}

}  // extern "C"
