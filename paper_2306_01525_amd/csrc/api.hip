// Host side of the MLBM C-ABI: argument checks, buffer layout, build
// orchestration, stepping, graphs and errors. Every entry point returns an
// mlbm_status; no exception leaves this file.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <utility>
#include <vector>

#include "common.h"

namespace mlbm {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string &msg) { g_error = msg; }

mlbm_status fail(mlbm_status st, const std::string &msg) {
    g_error = msg;
    return st;
}

mlbm_status hip_fail(hipError_t e, const char *what) {
    g_error = std::string(what) + ": " + hipGetErrorString(e);
    return MLBM_EHIP;
}

namespace {

// Power of two nearest to v (at least 1).
int pow2_near(double v) {
    if (v <= 1.0) return 1;
    int e = (int)std::lround(std::log2(v));
    return 1 << std::max(0, std::min(e, 15));
}

// Uniform search grid with about two nodes per cell.
void choose_grid(int n, double Lx, double Ly, int &gx, int &gy, int &hb) {
    double aspect = (Lx > 0 && Ly > 0) ? Lx / Ly : 1.0;
    double cells = std::max(1.0, n / 2.0);
    gx = pow2_near(std::sqrt(cells * aspect));
    gy = pow2_near(std::sqrt(cells / aspect));
    hb = 0;
    while ((1 << hb) < std::max(gx, gy)) ++hb;
}

mlbm_status check_params(const mlbm_cloud &c, const mlbm_params &p, bool device_cloud) {
    if (c.n <= 0) return fail(MLBM_EINVAL, "cloud has no nodes");
    // the departure points (8 per node) are listed per owner with 32-bit offsets
    if ((int64_t)8 * c.n > (int64_t)INT32_MAX)
        return fail(MLBM_EUNSUPPORTED, "clouds above 268,435,455 nodes are not supported");
    if (device_cloud && (!c.x || !c.y)) return fail(MLBM_EINVAL, "cloud coordinates are null");
    if (p.degree < 2 || p.degree > 4)
        return fail(MLBM_EINVAL, "polynomial degree must be 2, 3 or 4");
    const int M = poly_count(p.degree);
    if (p.K < 6 || p.K > kMaxK) return fail(MLBM_EINVAL, "stencil size K must be in [6, 48]");
    if (p.K < M) return fail(MLBM_EINVAL, "stencil size K is smaller than the polynomial count");
    if (p.K + M > 64) return fail(MLBM_EUNSUPPORTED, "K + M > 64 is not supported");
    if (c.n < p.K) return fail(MLBM_EINVAL, "cloud has fewer nodes than the stencil size");
    if (!(p.tau > 0.5)) return fail(MLBM_EINVAL, "tau must exceed 0.5");
    if (!(p.dx > 0.0)) return fail(MLBM_EINVAL, "dx must be positive");
    if ((c.period_x > 0 && !(p.dx < 0.5 * c.period_x)) ||
        (c.period_y > 0 && !(p.dx < 0.5 * c.period_y)))
        return fail(MLBM_EINVAL, "dx must be below half the period");
    if (c.period_x < 0 || c.period_y < 0) return fail(MLBM_EINVAL, "negative period");
    if (p.precision != MLBM_FP32_DEV && p.precision != MLBM_FP64)
        return fail(MLBM_EINVAL, "unknown precision");
    if (p.stencil_mode != MLBM_STENCIL_PAPER && p.stencil_mode != MLBM_STENCIL_OWN)
        return fail(MLBM_EINVAL, "unknown stencil mode");
    if (p.force_kind != 0 && p.force_kind != 1) return fail(MLBM_EINVAL, "unknown force kind");
    if (p.wall_kind < 0 || p.wall_kind > 2) return fail(MLBM_EINVAL, "unknown wall kind");
    if (p.wall_kind == 2 && (!c.node_type || !c.normal_x || !c.normal_y))
        return fail(MLBM_EINVAL, "bounce-back walls need node types and wall normals");
    if (!(p.rho0 > 0.0)) return fail(MLBM_EINVAL, "rho0 must be positive");
    if (p.wall_kind == 1 && !(p.rho_wall > 0.0)) return fail(MLBM_EINVAL, "rho_wall must be positive");
    if (p.with_adjoint && (p.force_kind != 0 || p.wall_kind != 0))
        return fail(MLBM_EUNSUPPORTED, "the adjoint supports periodic clouds without walls or force");
    // the transposed operator's rows are indexed with 32-bit offsets
    if (p.with_adjoint && (int64_t)8 * p.K * c.n > (int64_t)INT32_MAX)
        return fail(MLBM_EUNSUPPORTED, "the adjoint tables of this cloud exceed 2^31 entries");
    if (p.fp32_weights_only != 0 && p.fp32_weights_only != 1)
        return fail(MLBM_EINVAL, "fp32_weights_only must be 0 or 1");
    if (p.fp32_weights_only && p.precision != MLBM_FP32_DEV)
        return fail(MLBM_EINVAL, "fp32_weights_only needs the FP32 state");
    return MLBM_OK;
}

struct BuildWs {
    uint32_t *keys = nullptr, *skeys = nullptr;
    int32_t *vals = nullptr;
    int32_t *cstart = nullptr, *cend = nullptr;
    void *sort_tmp = nullptr;
    size_t sort_bytes = 0;
    void *tr_tmp = nullptr;
    size_t tr_bytes = 0;
    void *rbf_tmp = nullptr;
    size_t rbf_bytes = 0;
    int gx = 1, gy = 1, hb = 0;
};

// Plan layout of one cloud. With null bases only the sizes are computed.
void layout_cloud(const mlbm_cloud &c, const mlbm_params &p, int precision, Carve &pl,
                  Carve *ws, CloudPlan &cp, BuildWs *bw) {
    const int n = c.n, K = p.K;
    cp.n = n;
    cp.prm = p;
    cp.K = K;
    cp.m = p.degree;
    cp.M = poly_count(p.degree);
    cp.Lx = c.period_x;
    cp.Ly = c.period_y;
    cp.has_walls = p.wall_kind == 1;
    cp.geo = pl.take<Geo>(1);
    cp.xs = pl.take<double>(n);
    cp.ys = pl.take<double>(n);
    cp.perm = pl.take<int32_t>(n);
    cp.iperm = pl.take<int32_t>(n);
    cp.ntype = pl.take<uint8_t>(n);
    cp.links = p.wall_kind == 2 ? pl.take<uint8_t>(n) : nullptr;
    cp.nbr = pl.take<int32_t>((size_t)K * n);
    cp.owner = p.stencil_mode == MLBM_STENCIL_PAPER ? pl.take<int32_t>((size_t)8 * n) : nullptr;
    // FP64 shape vectors: in the plan, or with fp32_weights_only in the
    // workspace, where only the build uses them (solve, then FP32 packing)
    cp.W32 = precision == MLBM_FP32_DEV ? pl.take<float>((size_t)8 * K * n) : nullptr;
    if (p.fp32_weights_only && precision == MLBM_FP32_DEV)
        cp.W64 = ws ? ws->take<double>((size_t)8 * K * n) : nullptr;
    else
        cp.W64 = pl.take<double>((size_t)8 * K * n);
    if (p.force_kind) {
        cp.force64 = pl.take<double>((size_t)2 * n);
        cp.force32 = precision == MLBM_FP32_DEV ? pl.take<float>((size_t)2 * n) : nullptr;
    }
    {   // gather tables of the LDS-staged steps (both precisions)
        const int ntiles = (n + kTile - 1) / kTile;
        cp.hcap = kHaloCap;
        cp.ocap = std::min(512, (65536 - 8 * cp.hcap * 4) / (4 * ((K + 2) / 3)));
        cp.tdesc = pl.take<int32_t>((size_t)2 * ntiles);
        if (p.stencil_mode == MLBM_STENCIL_PAPER) cp.ownerL = pl.take<uint16_t>((size_t)8 * n);
        cp.nbrL = pl.take<uint32_t>((size_t)ntiles * cp.ocap * ((K + 2) / 3));
        cp.hlist = pl.take<int32_t>((size_t)ntiles * cp.hcap);
    }
    if (p.with_adjoint) {
        cp.tr_ptr = pl.take<int32_t>((size_t)8 * n + 1);
        cp.tr_col = pl.take<int32_t>((size_t)8 * K * n);
        cp.tr_val = precision == MLBM_FP64 ? (void *)pl.take<double>((size_t)8 * K * n)
                                           : (void *)pl.take<float>((size_t)8 * K * n);
        cp.tr_lw = K + 4;
        const size_t hn = (size_t)head_nodes(n);
        cp.ell_col = pl.take<int32_t>((size_t)8 * cp.tr_lw * hn);
        cp.ell_val = precision == MLBM_FP64
                         ? (void *)pl.take<double>((size_t)8 * cp.tr_lw * hn)
                         : (void *)pl.take<float>((size_t)8 * cp.tr_lw * hn);
        const int ntiles = (n + kTile - 1) / kTile;
        cp.tdescT = pl.take<int32_t>((size_t)ntiles);
        cp.ilist = pl.take<int32_t>((size_t)ntiles * cp.hcap);
        cp.elocal = pl.take<uint32_t>((size_t)8 * ((cp.tr_lw + 2) / 3) * hn);
        // 8 values of lam per inverse-halo node (64 KiB in FP64 at the cap)
        cp.adj_cap = cp.hcap;
    }
    if (ws && bw) {
        choose_grid(n, c.period_x, c.period_y, bw->gx, bw->gy, bw->hb);
        const size_t ncells = (size_t)bw->gx * bw->gy;
        bw->keys = ws->take<uint32_t>(n);
        bw->skeys = ws->take<uint32_t>(n);
        bw->vals = ws->take<int32_t>(n);
        bw->cstart = ws->take<int32_t>(ncells);
        bw->cend = ws->take<int32_t>(ncells);
        bw->sort_bytes = sort_pairs_temp_bytes(n);
        bw->sort_tmp = ws->take<char>(bw->sort_bytes);
        bw->rbf_bytes = rbf_temp_bytes(n);
        bw->rbf_tmp = ws->take<char>(bw->rbf_bytes);
        if (p.with_adjoint) {
            bw->tr_bytes = transpose_temp_bytes(n, K);
            bw->tr_tmp = ws->take<char>(bw->tr_bytes);
        }
    }
}

void layout_common(Carve &pl, mlbm_plan &plan, int64_t n_total, int n_clouds = 1) {
    plan.dev_err = pl.take<int32_t>(64);
    plan.stats = pl.take<int32_t>((size_t)kStats * n_clouds);
    plan.scratch64 =
        pl.take<double>(16 + 4 * (size_t)n_clouds + (size_t)blocks_for(n_total, 256) * 4);
}

// Error words to "none": no singular node, no flags, no reported node.
hipError_t reset_errors(mlbm_plan *plan, hipStream_t s) {
    hipError_t e = launch_fill_i32(plan->dev_err, INT_MAX, 3, s);
    if (e == hipSuccess) e = launch_fill_i32(plan->dev_err + kErrFlags, 0, 1, s);
    return e;
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

mlbm_status check_singular(mlbm_plan *plan, hipStream_t s) {
    if (capturing(s)) return MLBM_OK;
    MLBM_HIP(hipStreamSynchronize(s));
    int32_t v = 0;
    MLBM_HIP(hipMemcpy(&v, plan->dev_err, sizeof(v), hipMemcpyDeviceToHost));
    if (v != INT_MAX)
        return fail(MLBM_ESINGULAR, "local RBF system is numerically singular at node " +
                                        std::to_string(v - 1) + " (user index)");
    return MLBM_OK;
}

// Gather tables of the LDS-staged step and of the adjoint. Their kernels
// record per cloud (stats + kStats * cloud): [0] the largest LDS need of a
// step tile, [1] step tiles without tables, [2] the largest inverse halo,
// [3] adjoint tiles without one. The tables are enqueued for every cloud
// first; finish_tables then reads all the records at once (one
// synchronisation), or, while the stream is being captured, takes the
// capacity bounds instead.
mlbm_status enqueue_tables(CloudPlan &cp, int32_t *stats, hipStream_t s) {
    if (cp.tdescT) MLBM_HIP(launch_adj_tiles(cp, stats + 2, s));
    if (cp.tdesc) MLBM_HIP(launch_tiles(cp, stats, s));
    return MLBM_OK;
}

mlbm_status finish_tables(mlbm_plan *plan, hipStream_t s) {
    const size_t nc = plan->c.size();
    if (capturing(s)) {
        for (CloudPlan &cp : plan->c) {
            if (cp.tdesc) {
                // the capacity bound; the FP32 step checks every tile against
                // its launch's LDS and sends a larger one to the global-gather
                // path, so up to K = 30 it takes 40 KiB (four workgroups per
                // CU; the tables measured up to 38 KiB) instead of 53 KiB
                const unsigned cap =
                    (unsigned)(8 * cp.hcap * 4 + cp.ocap * ((cp.K + 2) / 3) * 4);
                cp.lds_bytes = cp.prm.precision != MLBM_FP64 && cp.K <= 30
                                   ? std::min(cap, kCaptureLds) : cap;
                cp.fallback_tiles = -1;
            }
            if (cp.tdescT) cp.adj_ni = cp.adj_cap;
        }
        return MLBM_OK;
    }
    std::vector<int32_t> h(kStats * nc);
    MLBM_HIP(hipStreamSynchronize(s));
    MLBM_HIP(hipMemcpy(h.data(), plan->stats, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost));
    for (size_t c = 0; c < nc; ++c) {
        CloudPlan &cp = plan->c[c];
        if (cp.tdesc) {
            cp.lds_bytes = (unsigned)h[kStats * c];
            cp.fallback_tiles = h[kStats * c + 1];
        }
        if (cp.tdescT) cp.adj_ni = h[kStats * c + 2];
    }
    return MLBM_OK;
}

void drop_graph(mlbm_plan *plan) {
    if (plan->graph_exec) {
        (void)hipGraphExecDestroy(plan->graph_exec);
        plan->graph_exec = nullptr;
    }
    if (plan->graph) {
        (void)hipGraphDestroy(plan->graph);
        plan->graph = nullptr;
    }
}

const CloudPlan *single(const mlbm_plan *plan) {
    if (!plan || plan->c.empty()) {
        set_error("null plan");
        return nullptr;
    }
    return &plan->c[0];
}

}  // namespace
}  // namespace mlbm

using namespace mlbm;

// Workspace of mlbm_build_weights_static: a fixed array in device memory, one
// per GPU the library runs on, held until the process ends. In host code the
// array's name only stands in for it; kernels get its device address, which
// hipGetSymbolAddress gives once per device (each GPU holds its own copy at
// its own address). Every call on one GPU shares it; the build clears what it
// needs (cell ranges, counters) with its own fill kernels before use.
namespace {
constexpr size_t kStaticWorkspaceBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

mlbm_status static_workspace(void **out) {
    static std::mutex mu;
    static std::map<int, void *> addr;
    int dev = 0;
    MLBM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void *p = nullptr;
        MLBM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(MLBM_EHIP, "hipGetSymbolAddress returned a null workspace");
        it = addr.emplace(dev, p).first;
    }
    *out = it->second;
    return MLBM_OK;
}
}  // namespace

namespace {
// Order in which the batched step lays out the clouds' tiles: by stencil
// size, then as given. The states keep the caller's order; only the launch's
// sequence of tiles changes. Clouds of one K next to each other measured 1.6 %
// faster than a random mix on a 64-cloud workload of K 20, 25 and 30 (0.710
// against 0.722 ms per step, with the split below in both).
std::vector<int> tile_order(const mlbm_plan &plan) {
    std::vector<int> o(plan.c.size());
    std::iota(o.begin(), o.end(), 0);
    std::stable_sort(o.begin(), o.end(),
                     [&](int a, int b) { return plan.c[a].prm.K < plan.c[b].prm.K; });
    return o;
}
}  // namespace

extern "C" {

const char *mlbm_last_error(void) { return g_error.c_str(); }

namespace {

// Layout of a whole plan (clouds back to back, then the batch tables and the
// shared words). With null bases only the sizes are computed.
struct PlanLayout {
    std::vector<CloudPlan> cps;
    std::vector<BuildWs> bws;
    size_t plan_used = 0, ws_max = 0;   // ws_max: the whole workspace (all lanes)
    int lanes = 1;                      // clouds built concurrently (c on lane c % lanes)
};

mlbm_status check_batch(const mlbm_cloud *clouds, const mlbm_params *params, int32_t n_clouds,
                        bool device_cloud) {
    if (!clouds || !params || n_clouds < 1) return fail(MLBM_EINVAL, "null argument or n_clouds < 1");
    int64_t total = 0;
    for (int c = 0; c < n_clouds; ++c) {
        mlbm_status st = check_params(clouds[c], params[c], device_cloud);
        if (st != MLBM_OK) return fail(st, "cloud " + std::to_string(c) + ": " + g_error);
        if (params[c].precision != params[0].precision)
            return fail(MLBM_EINVAL, "all clouds of a plan need the same precision");
        if (n_clouds > 1 && params[c].with_adjoint)
            return fail(MLBM_EUNSUPPORTED, "the adjoint needs a single-cloud plan");
        if (clouds[c].period_x > 0 != clouds[c].period_y > 0)
            return fail(MLBM_EUNSUPPORTED, "clouds periodic along one axis only");
        total += clouds[c].n;
    }
    if (total > INT32_MAX / 2) return fail(MLBM_EUNSUPPORTED, "too many nodes in one plan");
    return MLBM_OK;
}

bool batchable(const mlbm_params *params, int32_t n_clouds) {
    if (n_clouds < 2 || params[0].precision != MLBM_FP32_DEV) return false;
    for (int c = 0; c < n_clouds; ++c)
        if (params[c].stencil_mode != params[0].stencil_mode || params[c].force_kind ||
            params[c].wall_kind)
            return false;
    return true;
}

void layout_plan(const mlbm_cloud *clouds, const mlbm_params *params, int32_t n_clouds,
                 void *plan_buf, void *workspace, PlanLayout &L, mlbm_plan &plan,
                 int max_lanes = kBuildLanes) {
    Carve pl(plan_buf);
    L.cps.assign(n_clouds, CloudPlan());
    L.bws.assign(n_clouds, BuildWs());
    // Clouds are built on up to kBuildLanes streams at once; each lane has a
    // workspace region of the largest cloud's need, reused cloud after cloud.
    size_t stride = 0;
    for (int c = 0; c < n_clouds; ++c) {
        Carve p0(nullptr), w0(nullptr);
        CloudPlan cp0;
        BuildWs bw0;
        layout_cloud(clouds[c], params[c], params[0].precision, p0, &w0, cp0, &bw0);
        stride = std::max(stride, (w0.used + 255) & ~size_t(255));
    }
    L.lanes = std::max(1, std::min(n_clouds, max_lanes));
    int64_t off = 0, tiles = 0;
    for (int c = 0; c < n_clouds; ++c) {
        Carve ws(workspace ? (char *)workspace + (size_t)(c % L.lanes) * stride : nullptr);
        layout_cloud(clouds[c], params[c], params[0].precision, pl, &ws, L.cps[c], &L.bws[c]);
        L.cps[c].off = off;
        off += clouds[c].n;
        tiles += (clouds[c].n + kTile - 1) / kTile;
    }
    L.ws_max = stride * L.lanes;
    plan.n_total = off;
    plan.total_tiles = tiles;
    plan.batched = batchable(params, n_clouds);
    plan.batch_mode = params[0].stencil_mode;
    if (plan.batched) {
        plan.descs = pl.take<Step32Args>(n_clouds);
        plan.tile2cloud = pl.take<int32_t>(tiles);
    }
    layout_common(pl, plan, off, n_clouds);
    L.plan_used = pl.used;
}

// Enqueue the build of one cloud (steps 1-4 of mlbm_build_weights).
mlbm_status build_cloud(mlbm_plan *plan, CloudPlan &cp, const mlbm_cloud &c,
                        const mlbm_params &p, BuildWs &bw, int32_t *stats, hipStream_t s) {
    const int n = c.n;
    if (c.period_x > 0 && c.period_y > 0)
        MLBM_HIP(launch_geo_periodic(cp.geo, c.period_x, c.period_y, bw.gx, bw.gy, bw.hb, s));
    else
        MLBM_HIP(launch_geo_bbox(cp.geo, c.x, c.y, n, bw.gx, bw.gy, bw.hb, s));
    MLBM_HIP(launch_keys(cp.geo, c.x, c.y, n, bw.keys, bw.vals, s));
    MLBM_HIP(sort_pairs(bw.sort_tmp, bw.sort_bytes, bw.keys, bw.skeys, bw.vals, cp.perm, n,
                        std::max(1, 2 * bw.hb), s));
    MLBM_HIP(launch_scatter_sorted(cp.geo, c.x, c.y, c.node_type, cp.perm, bw.skeys, n, cp.xs,
                                   cp.ys, cp.ntype, cp.iperm, bw.cstart, bw.cend, bw.gx * bw.gy, s));
    MLBM_HIP(launch_knn(cp.geo, cp.xs, cp.ys, cp.perm, cp.iperm, bw.cstart, bw.cend, n, p.K,
                        cp.nbr, s));
    if (p.stencil_mode == MLBM_STENCIL_PAPER)
        MLBM_HIP(launch_owner(cp.geo, cp.xs, cp.ys, cp.perm, cp.iperm, bw.cstart, bw.cend, n,
                              p.dx, cp.owner, s));
    MLBM_HIP(launch_rbf(cp.geo, cp.xs, cp.ys, cp.perm, cp.nbr, cp.owner, n, p.K, p.degree, p.dx,
                        p.stencil_mode, bw.rbf_tmp, bw.rbf_bytes, cp.W64, plan->dev_err, s));
    if (cp.W32) MLBM_HIP(launch_pack_w32(cp.W64, n, p.K, cp.W32, s));
    // with fp32_weights_only the FP64 shape vectors were workspace, used up here
    if (p.fp32_weights_only) cp.W64 = nullptr;
    // equilibrium wall nodes receive no force; with bounce-back every node does
    MLBM_HIP(launch_force(cp.xs, cp.ys, p.wall_kind == 1 ? cp.ntype : nullptr, n, p.force_kind,
                          p.force_mag, cp.force32, cp.force64, s));
    if (cp.links)
        MLBM_HIP(launch_links(cp.ntype, cp.perm, c.normal_x, c.normal_y, n, cp.links, s));
    if (p.with_adjoint) MLBM_HIP(launch_transpose(cp, p.precision, bw.tr_tmp, bw.tr_bytes, s));
    return enqueue_tables(cp, stats, s);
}

// Descriptor table and tile map of the batched step.
// Streams and events that let the clouds of one plan build concurrently: per
// device, created once (outside any graph capture) and kept for the process.
struct LanePool {
    hipStream_t st[kBuildLanes - 1] = {};
    hipEvent_t ev[kBuildLanes] = {};
    std::mutex mu;
};

LanePool *lane_pool() {
    static std::mutex m;
    static std::map<int, std::unique_ptr<LanePool>> pools;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lock(m);
    std::unique_ptr<LanePool> &p = pools[dev];
    if (!p) {
        auto q = std::make_unique<LanePool>();
        for (int i = 0; i < kBuildLanes - 1; ++i)
            if (hipStreamCreateWithFlags(&q->st[i], hipStreamNonBlocking) != hipSuccess)
                return nullptr;
        for (int i = 0; i < kBuildLanes; ++i)
            if (hipEventCreateWithFlags(&q->ev[i], hipEventDisableTiming) != hipSuccess)
                return nullptr;
        p = std::move(q);
    }
    return p.get();
}

// Enqueue the builds of all clouds: cloud c on lane c % lanes, lane 0 being
// the caller's stream and the others forked from it and joined back to it (in
// a captured stream the lanes become parallel branches of the graph).
mlbm_status build_clouds(mlbm_plan *plan, const mlbm_cloud *clouds, const mlbm_params *params,
                         PlanLayout &L, hipStream_t s) {
    const int nc = (int)plan->c.size();
    LanePool *pool = L.lanes > 1 ? lane_pool() : nullptr;
    if (!pool) {
        if (L.lanes > 1) return fail(MLBM_EHIP, "could not create the build streams");
        for (int c = 0; c < nc; ++c) {
            mlbm_status st = build_cloud(plan, plan->c[c], clouds[c], params[c], L.bws[c],
                                         plan->stats + kStats * c, s);
            if (st != MLBM_OK) return st;
        }
        return MLBM_OK;
    }
    std::lock_guard<std::mutex> lock(pool->mu);
    MLBM_HIP(hipEventRecord(pool->ev[0], s));
    for (int l = 1; l < L.lanes; ++l) MLBM_HIP(hipStreamWaitEvent(pool->st[l - 1], pool->ev[0], 0));
    mlbm_status st = MLBM_OK;
    for (int c = 0; c < nc && st == MLBM_OK; ++c) {
        const int l = c % L.lanes;
        st = build_cloud(plan, plan->c[c], clouds[c], params[c], L.bws[c],
                         plan->stats + kStats * c, l ? pool->st[l - 1] : s);
    }
    // join every lane, also after an error, so no capture is left forked
    for (int l = 1; l < L.lanes; ++l) {
        hipError_t e = hipEventRecord(pool->ev[l], pool->st[l - 1]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, pool->ev[l], 0);
        if (e != hipSuccess && st == MLBM_OK) st = hip_fail(e, "joining the build streams");
    }
    return st;
}

// The batched step's descriptor of a cloud whose tiles start at tile_begin.
Step32Args batch_desc(const CloudPlan &cp, int64_t tile_begin) {
    Step32Args a = step32_args(cp, nullptr);
    a.soff = (int64_t)kQ * cp.off;
    a.tile_begin = tile_begin;
    return a;
}

// Splits the batch's tiles into eight contiguous ranges of about equal cost,
// one per XCD. A node-update costs its algorithmic bytes, 4 (9K + 18) + 32
// with the paper's stencils, plus about 170 bytes' worth of work that does not
// grow with K (staging, collision, stores): a linear fit to the batched step's
// time per node over clouds of K = 20, 25 and 30. The tile that crosses a
// boundary goes to the earlier XCD.
void split_xcds(mlbm_plan &plan, const std::vector<int> &order) {
    auto node_cost = [&](const CloudPlan &cp) {
        return 4.0 * (9 * cp.prm.K + 18) + (plan.batch_mode == MLBM_STENCIL_PAPER ? 32 : 0) +
               170.0;
    };
    double total = 0.0;
    for (const CloudPlan &cp : plan.c) total += node_cost(cp) * cp.n;
    XcdSplit &r = plan.xcd;
    r.begin[0] = 0;
    int x = 1;
    int64_t t = 0;
    double acc = 0.0;
    for (int c : order) {
        const CloudPlan &cp = plan.c[c];
        const double w = node_cost(cp);
        for (int64_t p = 0; p < cp.n; p += kTile, ++t) {
            acc += w * (double)std::min<int64_t>(kTile, cp.n - p);
            while (x < 8 && acc >= total * x / 8.0) r.begin[x++] = t + 1;
        }
    }
    while (x < 9) r.begin[x++] = plan.total_tiles;
    plan.xcd_longest = 0;
    for (int i = 0; i < 8; ++i)
        plan.xcd_longest = std::max(plan.xcd_longest, r.begin[i + 1] - r.begin[i]);
}

mlbm_status build_batch(mlbm_plan *plan, hipStream_t s) {
    if (!plan->batched) return MLBM_OK;
    const std::vector<int> order = tile_order(*plan);
    int64_t tb = 0;
    unsigned lds = 0;
    for (int c : order) {
        const CloudPlan &cp = plan->c[c];
        const int64_t nt = (cp.n + kTile - 1) / kTile;
        MLBM_HIP(launch_set_desc(plan->descs + c, batch_desc(cp, tb), s));
        MLBM_HIP(launch_fill_i32(plan->tile2cloud + tb, (int32_t)c, nt, s));
        tb += nt;
        lds = std::max(lds, cp.lds_bytes);
    }
    plan->batch_lds = lds;
    split_xcds(*plan, order);
    return MLBM_OK;
}

}  // namespace

namespace {

// Plan and workspace sizes with at most max_lanes clouds built at once.
mlbm_status query_lanes(const mlbm_cloud *clouds, const mlbm_params *params, int32_t n_clouds,
                        int max_lanes, size_t *plan_bytes, size_t *workspace_bytes) {
    if (!plan_bytes || !workspace_bytes) return fail(MLBM_EINVAL, "null output pointer");
    mlbm_status st = check_batch(clouds, params, n_clouds, false);
    if (st != MLBM_OK) return st;
    PlanLayout L;
    mlbm_plan tmp;
    layout_plan(clouds, params, n_clouds, nullptr, nullptr, L, tmp, max_lanes);
    *plan_bytes = L.plan_used + 256;
    *workspace_bytes = L.ws_max + 256;
    return MLBM_OK;
}

mlbm_status build_weights_lanes(const mlbm_cloud *clouds, const mlbm_params *params,
                                int32_t n_clouds, void *plan_buf, size_t plan_bytes,
                                void *workspace, size_t workspace_bytes, int max_lanes,
                                mlbm_plan **out, hipStream_t s) {
    if (!out) return fail(MLBM_EINVAL, "null output pointer");
    *out = nullptr;
    size_t need_p = 0, need_w = 0;
    mlbm_status st = query_lanes(clouds, params, n_clouds, max_lanes, &need_p, &need_w);
    if (st != MLBM_OK) return st;
    st = check_batch(clouds, params, n_clouds, true);
    if (st != MLBM_OK) return st;
    if (!plan_buf || !workspace) return fail(MLBM_EINVAL, "null plan buffer or workspace");
    if (plan_bytes < need_p || workspace_bytes < need_w)
        return fail(MLBM_ESMALLBUF, "plan or workspace buffer smaller than queried");
    mlbm_plan *plan = new (std::nothrow) mlbm_plan();
    if (!plan) return fail(MLBM_EINVAL, "out of host memory");
    plan->precision = params[0].precision;
    PlanLayout L;
    layout_plan(clouds, params, n_clouds, plan_buf, workspace, L, *plan, max_lanes);
    plan->c = L.cps;
    for (CloudPlan &cp : plan->c) cp.err = plan->dev_err;
    auto cleanup = [&](mlbm_status r) {
        delete plan;
        return r;
    };
    hipError_t e = reset_errors(plan, s);
    if (e == hipSuccess) e = launch_fill_i32(plan->stats, 0, (int64_t)kStats * n_clouds, s);
    if (e != hipSuccess) return cleanup(hip_fail(e, "launch_fill_i32"));
    st = build_clouds(plan, clouds, params, L, s);
    if (st != MLBM_OK) return cleanup(st);
    st = finish_tables(plan, s);
    if (st != MLBM_OK) return cleanup(st);
    st = build_batch(plan, s);
    if (st != MLBM_OK) return cleanup(st);
    st = check_singular(plan, s);
    if (st != MLBM_OK) return cleanup(st);
    *out = plan;
    return MLBM_OK;
}

}  // namespace

mlbm_status mlbm_weights_query(const mlbm_cloud *clouds, const mlbm_params *params,
                               int32_t n_clouds, size_t *plan_bytes, size_t *workspace_bytes) {
    return query_lanes(clouds, params, n_clouds, kBuildLanes, plan_bytes, workspace_bytes);
}

mlbm_status mlbm_build_weights(const mlbm_cloud *clouds, const mlbm_params *params,
                               int32_t n_clouds, void *plan_buf, size_t plan_bytes,
                               void *workspace, size_t workspace_bytes, mlbm_plan **out,
                               hipStream_t s) {
    return build_weights_lanes(clouds, params, n_clouds, plan_buf, plan_bytes, workspace,
                               workspace_bytes, kBuildLanes, out, s);
}

mlbm_status mlbm_build_weights_static(const mlbm_cloud *clouds, const mlbm_params *params,
                                      int32_t n_clouds, void *plan_buf, size_t plan_bytes,
                                      mlbm_plan **out, hipStream_t s) {
    if (!out) return fail(MLBM_EINVAL, "null output pointer");
    *out = nullptr;
    size_t need_p = 0, need_w = 0;
    mlbm_status st = query_lanes(clouds, params, n_clouds, 1, &need_p, &need_w);
    if (st != MLBM_OK) return st;
    if (need_w > kStaticWorkspaceBytes)
        return fail(MLBM_EUNSUPPORTED,
                    "the build needs a workspace of " + std::to_string(need_w) +
                        " bytes, more than the library's static workspace of " +
                        std::to_string(kStaticWorkspaceBytes) +
                        " bytes: use mlbm_build_weights with a caller workspace");
    void *ws = nullptr;
    st = static_workspace(&ws);
    if (st != MLBM_OK) return st;
    return build_weights_lanes(clouds, params, n_clouds, plan_buf, plan_bytes, ws,
                               kStaticWorkspaceBytes, 1, out, s);
}

mlbm_status mlbm_import_query(int32_t n, const mlbm_params *params, size_t *plan_bytes) {
    if (!params || !plan_bytes) return fail(MLBM_EINVAL, "null argument");
    mlbm_cloud c{};
    c.n = n;
    mlbm_status st = check_params(c, *params, false);
    if (st != MLBM_OK) return st;
    if (params->fp32_weights_only)
        return fail(MLBM_EUNSUPPORTED, "imported plans keep their FP64 shape vectors");
    Carve pl(nullptr);
    CloudPlan cp;
    mlbm_plan tmp;
    mlbm_params p = *params;
    layout_cloud(c, p, p.precision, pl, nullptr, cp, nullptr);
    layout_common(pl, tmp, n);
    *plan_bytes = pl.used + 256;
    return MLBM_OK;
}

mlbm_status mlbm_import_weights(int32_t n, const double *x, const double *y,
                                const uint8_t *node_type, const int32_t *nbr,
                                const int32_t *owner, const double *W,
                                const mlbm_params *params, void *plan_buf, size_t plan_bytes,
                                mlbm_plan **out, hipStream_t s) {
    if (!out) return fail(MLBM_EINVAL, "null output pointer");
    *out = nullptr;
    size_t need = 0;
    mlbm_status st = mlbm_import_query(n, params, &need);
    if (st != MLBM_OK) return st;
    if (!x || !y || !nbr || !owner || !W || !plan_buf)
        return fail(MLBM_EINVAL, "null input array");
    if (plan_bytes < need) return fail(MLBM_ESMALLBUF, "plan buffer smaller than queried");
    const mlbm_params &p = *params;
    const int K = p.K;
    for (int64_t i = 0; i < (int64_t)n * K; ++i)
        if (nbr[i] < 0 || nbr[i] >= n) return fail(MLBM_EINVAL, "stencil index out of range");
    for (int64_t i = 0; i < (int64_t)n * 9; ++i)
        if (owner[i] < 0 || owner[i] >= n) return fail(MLBM_EINVAL, "owner index out of range");
    mlbm_plan *plan = new (std::nothrow) mlbm_plan();
    if (!plan) return fail(MLBM_EINVAL, "out of host memory");
    plan->precision = p.precision;
    plan->n_total = n;
    mlbm_cloud c{};
    c.n = n;
    Carve pl(plan_buf);
    CloudPlan cp;
    layout_cloud(c, p, p.precision, pl, nullptr, cp, nullptr);
    layout_common(pl, *plan, n);
    cp.imported = true;
    std::vector<int32_t> ident(n), hn((size_t)K * n), ho;
    std::vector<uint8_t> nt(n, 0);
    std::vector<double> hw((size_t)8 * K * n);
    for (int i = 0; i < n; ++i) ident[i] = i;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < K; ++j) hn[(size_t)j * n + i] = nbr[(size_t)i * K + j];
    if (cp.owner) {
        ho.resize((size_t)8 * n);
        for (int i = 0; i < n; ++i)
            for (int k = 1; k < 9; ++k) ho[(size_t)(k - 1) * n + i] = owner[(size_t)i * 9 + k];
    }
    for (int i = 0; i < n; ++i)
        for (int k = 1; k < 9; ++k)
            for (int j = 0; j < K; ++j)
                hw[w64_at(k, j, n, i)] = W[((size_t)i * 9 + k) * K + j];
    if (node_type)
        for (int i = 0; i < n; ++i) nt[i] = node_type[i];
    cp.has_walls = p.wall_kind == 1;
    auto cleanup = [&](mlbm_status r) {
        delete plan;
        return r;
    };
#define STEP(call)                                                      \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) return cleanup(hip_fail(e_, #call));      \
    } while (0)
    STEP(hipMemcpyAsync(cp.xs, x, sizeof(double) * n, hipMemcpyHostToDevice, s));
    STEP(hipMemcpyAsync(cp.ys, y, sizeof(double) * n, hipMemcpyHostToDevice, s));
    STEP(hipMemcpyAsync(cp.perm, ident.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    STEP(hipMemcpyAsync(cp.iperm, ident.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    STEP(hipMemcpyAsync(cp.ntype, nt.data(), n, hipMemcpyHostToDevice, s));
    STEP(hipMemcpyAsync(cp.nbr, hn.data(), sizeof(int32_t) * hn.size(), hipMemcpyHostToDevice, s));
    if (cp.owner)
        STEP(hipMemcpyAsync(cp.owner, ho.data(), sizeof(int32_t) * ho.size(),
                            hipMemcpyHostToDevice, s));
    STEP(hipMemcpyAsync(cp.W64, hw.data(), sizeof(double) * hw.size(), hipMemcpyHostToDevice, s));
    if (cp.W32) STEP(launch_pack_w32(cp.W64, n, K, cp.W32, s));
    STEP(launch_force(cp.xs, cp.ys, cp.ntype, n, p.force_kind, p.force_mag, cp.force32,
                      cp.force64, s));
    cp.err = plan->dev_err;
    STEP(reset_errors(plan, s));
    if (p.with_adjoint) {
        // This path has no workspace argument, so the transposed operator is
        // assembled on the host (rows filled in ascending arriving node, which
        // is the order the GPU build sorts to) and copied in.
        std::vector<int32_t> cnt((size_t)8 * n, 0), ptr((size_t)8 * n + 1, 0), col;
        std::vector<double> v64;
        std::vector<float> v32;
        const size_t nnz = (size_t)8 * K * n;
        col.resize(nnz);
        if (p.precision == MLBM_FP64) v64.resize(nnz);
        else v32.resize(nnz);
        std::vector<float> w32;
        if (p.precision != MLBM_FP64) {
            w32.resize((size_t)8 * K * n);
            STEP(hipMemcpyAsync(w32.data(), cp.W32, sizeof(float) * w32.size(),
                                hipMemcpyDeviceToHost, s));
            STEP(hipStreamSynchronize(s));
        }
        auto src = [&](int i, int k, int j) {
            int sidx = p.stencil_mode == MLBM_STENCIL_OWN ? i : owner[(size_t)i * 9 + k];
            return nbr[(size_t)sidx * K + j];
        };
        for (int i = 0; i < n; ++i)
            for (int k = 1; k < 9; ++k)
                for (int j = 0; j < K; ++j) cnt[(size_t)(k - 1) * n + src(i, k, j)]++;
        for (size_t r = 0; r < (size_t)8 * n; ++r) ptr[r + 1] = ptr[r] + cnt[r];
        std::vector<int32_t> cur(ptr.begin(), ptr.end() - 1);
        for (int i = 0; i < n; ++i)   // ascending i: rows come out sorted by arriving node
            for (int k = 1; k < 9; ++k)
                for (int j = 0; j < K; ++j) {
                    size_t r = (size_t)(k - 1) * n + src(i, k, j);
                    int pos = cur[r]++;
                    col[pos] = i;
                    if (p.precision == MLBM_FP64)
                        v64[pos] = hw[w64_at(k, j, n, i)];
                    else
                        v32[pos] = w32[(((size_t)j * 2 + ((k - 1) >> 2)) * n + i) * 4 + ((k - 1) & 3)];
                }
        STEP(hipMemcpyAsync(cp.tr_ptr, ptr.data(), sizeof(int32_t) * ptr.size(),
                            hipMemcpyHostToDevice, s));
        STEP(hipMemcpyAsync(cp.tr_col, col.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s));
        if (p.precision == MLBM_FP64)
            STEP(hipMemcpyAsync(cp.tr_val, v64.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, s));
        else
            STEP(hipMemcpyAsync(cp.tr_val, v32.data(), sizeof(float) * nnz, hipMemcpyHostToDevice, s));
        STEP(launch_ell_fill(cp, p.precision, s));
    }
    STEP(launch_fill_i32(plan->stats, 0, kStats, s));
#undef STEP
    st = enqueue_tables(cp, plan->stats, s);
    if (st != MLBM_OK) return cleanup(st);
    plan->c.push_back(cp);
    st = finish_tables(plan, s);
    if (st != MLBM_OK) return cleanup(st);
    *out = plan;
    return MLBM_OK;
}

mlbm_status mlbm_plan_get_info(const mlbm_plan *plan, mlbm_plan_info *info) {
    const CloudPlan *cp = single(plan);
    if (!cp || !info) return fail(MLBM_EINVAL, "null argument");
    info->n_clouds = (int32_t)plan->c.size();
    info->n_total = plan->n_total;
    info->K = cp->K;
    info->degree = cp->m;
    info->stencil_mode = cp->prm.stencil_mode;
    info->precision = plan->precision;
    info->state_bytes = (size_t)9 * plan->n_total * state_elem_bytes(plan->precision);
    info->tile_nodes = kTile;
    info->step_lds_bytes = (int32_t)cp->lds_bytes;
    info->fallback_tiles = cp->fallback_tiles;
    info->variant = cp->variant;
    return MLBM_OK;
}

mlbm_status mlbm_plan_export(const mlbm_plan *plan, int32_t cloud, int32_t what, void *dst,
                             size_t dst_bytes) {
    if (!plan || cloud < 0 || cloud >= (int32_t)plan->c.size() || !dst)
        return fail(MLBM_EINVAL, "bad plan, cloud or destination");
    const CloudPlan &cp = plan->c[cloud];
    const int n = cp.n, K = cp.K;
    const size_t ntiles = (size_t)(n + kTile - 1) / kTile;
    size_t need = what == 0 ? sizeof(int32_t) * n
                : what == 1 ? sizeof(int32_t) * (size_t)n * K
                : what == 2 ? sizeof(int32_t) * (size_t)n * 9
                : what == 3 ? sizeof(double) * (size_t)n * 9 * K
                : what == 4 ? sizeof(int32_t) * 2 * ntiles
                : what == 5 ? sizeof(int32_t) * ntiles * cp.hcap
                : what == 6 ? sizeof(uint32_t) * ntiles * cp.ocap * ((K + 2) / 3)
                : what == 7 ? sizeof(uint16_t) * 8 * (size_t)n
                : what == 8 ? sizeof(int32_t) * 2
                : what == 9 ? sizeof(int32_t) * ntiles
                : what == 10 ? sizeof(int32_t) * ntiles * cp.hcap
                : what == 11 ? sizeof(uint32_t) * 8 * (size_t)((cp.tr_lw + 2) / 3) * head_nodes(n)
                : what == 12 ? sizeof(int32_t) * ((size_t)8 * n + 1)
                : what == 13 ? sizeof(int32_t) * 8 * (size_t)cp.tr_lw * head_nodes(n) : 0;
    if (need == 0) return fail(MLBM_EINVAL, "unknown export item");
    if (what >= 9 && !cp.tdescT) return fail(MLBM_EINVAL, "plan was built without with_adjoint");
    if (what >= 4 && what <= 6 && !cp.tdesc) return fail(MLBM_EINVAL, "plan has no tile tables");
    if (what == 7 && !cp.ownerL) return fail(MLBM_EINVAL, "plan has no local owners");
    if (what == 3 && !cp.W64)
        return fail(MLBM_EUNSUPPORTED, "plan was built with fp32_weights_only: no FP64 shape vectors");
    if (dst_bytes != need) return fail(MLBM_ESMALLBUF, "export size mismatch");
    MLBM_HIP(hipDeviceSynchronize());
    if (what == 8) {
        int32_t caps[2] = {cp.ocap, cp.hcap};
        std::memcpy(dst, caps, sizeof(caps));
        return MLBM_OK;
    }
    if (what >= 9) {
        const void *src = what == 9 ? (const void *)cp.tdescT
                        : what == 10 ? (const void *)cp.ilist
                        : what == 11 ? (const void *)cp.elocal
                        : what == 12 ? (const void *)cp.tr_ptr : (const void *)cp.ell_col;
        MLBM_HIP(hipMemcpy(dst, src, need, hipMemcpyDeviceToHost));
        return MLBM_OK;
    }
    if (what >= 4) {
        const void *src = what == 4 ? (const void *)cp.tdesc
                        : what == 5 ? (const void *)cp.hlist
                        : what == 6 ? (const void *)cp.nbrL : (const void *)cp.ownerL;
        MLBM_HIP(hipMemcpy(dst, src, need, hipMemcpyDeviceToHost));
        return MLBM_OK;
    }
    std::vector<int32_t> perm(n), iperm(n);
    MLBM_HIP(hipMemcpy(perm.data(), cp.perm, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    for (int p = 0; p < n; ++p) iperm[perm[p]] = p;
    if (what == 0) {
        std::memcpy(dst, perm.data(), need);
        return MLBM_OK;
    }
    if (what == 1) {
        std::vector<int32_t> nb((size_t)K * n);
        MLBM_HIP(hipMemcpy(nb.data(), cp.nbr, sizeof(int32_t) * nb.size(), hipMemcpyDeviceToHost));
        int32_t *o = (int32_t *)dst;
        for (int u = 0; u < n; ++u)
            for (int j = 0; j < K; ++j) o[(size_t)u * K + j] = perm[nb[(size_t)j * n + iperm[u]]];
        return MLBM_OK;
    }
    if (what == 2) {
        std::vector<int32_t> ow;
        if (cp.owner) {
            ow.resize((size_t)8 * n);
            MLBM_HIP(hipMemcpy(ow.data(), cp.owner, sizeof(int32_t) * ow.size(), hipMemcpyDeviceToHost));
        }
        int32_t *o = (int32_t *)dst;
        for (int u = 0; u < n; ++u) {
            o[(size_t)u * 9] = u;
            for (int k = 1; k < 9; ++k)
                o[(size_t)u * 9 + k] = cp.owner ? perm[ow[(size_t)(k - 1) * n + iperm[u]]] : u;
        }
        return MLBM_OK;
    }
    std::vector<double> w((size_t)8 * K * n);
    MLBM_HIP(hipMemcpy(w.data(), cp.W64, sizeof(double) * w.size(), hipMemcpyDeviceToHost));
    double *o = (double *)dst;
    for (int u = 0; u < n; ++u) {
        const int p = iperm[u];
        for (int j = 0; j < K; ++j) o[((size_t)u * 9) * K + j] = j == 0 ? 1.0 : 0.0;
        for (int k = 1; k < 9; ++k)
            for (int j = 0; j < K; ++j)
                o[((size_t)u * 9 + k) * K + j] = w[w64_at(k, j, n, p)];
    }
    return MLBM_OK;
}

mlbm_status mlbm_plan_destroy(mlbm_plan *plan) {
    if (!plan) return MLBM_OK;
    if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
    return MLBM_OK;
}

mlbm_status mlbm_plan_set_tau(mlbm_plan *plan, double tau) {
    if (!plan || plan->c.empty()) return fail(MLBM_EINVAL, "null plan");
    if (!(tau > 0.5)) return fail(MLBM_EINVAL, "tau must exceed 0.5");
    for (auto &cp : plan->c) cp.prm.tau = tau;
    drop_graph(plan);
    if (plan->batched) {
        // the batched step reads each cloud's relaxation rate from the device
        // descriptor table: rewrite the table (synchronous copies)
        MLBM_HIP(hipDeviceSynchronize());
        int64_t tb = 0;
        for (int c : tile_order(*plan)) {
            const CloudPlan &cp = plan->c[c];
            const Step32Args a = batch_desc(cp, tb);
            tb += (cp.n + kTile - 1) / kTile;
            MLBM_HIP(hipMemcpy(plan->descs + c, &a, sizeof(a), hipMemcpyHostToDevice));
        }
    }
    return MLBM_OK;
}

namespace {
mlbm_status read_errors(const mlbm_plan *plan, int32_t (&w)[3]) {
    MLBM_HIP(hipDeviceSynchronize());
    MLBM_HIP(hipMemcpy(w, plan->dev_err, sizeof(w), hipMemcpyDeviceToHost));
    return MLBM_OK;
}
}  // namespace

int32_t mlbm_device_error(const mlbm_plan *plan) {
    if (!plan || !plan->dev_err) return 0;
    int32_t w[3];
    if (read_errors(plan, w) != MLBM_OK) return -1;
    return (w[kErrSingular] != INT_MAX ? MLBM_DEVERR_SINGULAR : 0) | w[kErrFlags];
}

mlbm_status mlbm_device_error_nodes(const mlbm_plan *plan, int32_t *singular_node,
                                    int32_t *diverged_node) {
    if (!plan || !plan->dev_err) return fail(MLBM_EINVAL, "null plan");
    int32_t w[3];
    mlbm_status st = read_errors(plan, w);
    if (st != MLBM_OK) return st;
    if (singular_node) *singular_node = w[kErrSingular] == INT_MAX ? -1 : w[kErrSingular] - 1;
    if (diverged_node) *diverged_node = w[kErrNode] == INT_MAX ? -1 : w[kErrNode];
    return MLBM_OK;
}

mlbm_status mlbm_device_error_clear(mlbm_plan *plan, hipStream_t s) {
    if (!plan || !plan->dev_err) return fail(MLBM_EINVAL, "null plan");
    MLBM_HIP(reset_errors(plan, s));
    return MLBM_OK;
}

namespace {

// Sub-array of cloud c inside a state-shaped array (cloud blocks of [9][n_c]).
inline void *state_at(const mlbm_plan *plan, const void *base, const CloudPlan &cp) {
    return (char *)base + (size_t)kQ * cp.off * state_elem_bytes(plan->precision);
}
inline const double *node_at(const double *base, const CloudPlan &cp) {
    return base ? base + cp.off : nullptr;
}
inline double *out_at(double *base, const CloudPlan &cp) { return base ? base + cp.off : nullptr; }

// One timestep of every cloud: the batched kernel when the plan allows it,
// else one launch per cloud.
hipError_t step_once(const mlbm_plan *plan, const void *gin, void *gout, void *frec,
                     hipStream_t s) {
    if (plan->batched && !frec) return launch_step_batch(*plan, gin, gout, s);
    for (const CloudPlan &cp : plan->c) {
        hipError_t e = launch_step(cp, plan->precision, state_at(plan, gin, cp),
                                   state_at(plan, gout, cp),
                                   frec ? state_at(plan, frec, cp) : nullptr, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

mlbm_status mlbm_init(const mlbm_plan *plan, const double *rho, const double *ux,
                      const double *uy, void *g, hipStream_t s) {
    if (!single(plan) || !g) return fail(MLBM_EINVAL, "null plan or state");
    for (const CloudPlan &cp : plan->c)
        MLBM_HIP(launch_init(cp, plan->precision, node_at(rho, cp), node_at(ux, cp),
                             node_at(uy, cp), state_at(plan, g, cp), true, s));
    return MLBM_OK;
}

mlbm_status mlbm_init_f(const mlbm_plan *plan, const double *rho, const double *ux,
                        const double *uy, void *f, hipStream_t s) {
    if (!single(plan) || !f) return fail(MLBM_EINVAL, "null plan or state");
    for (const CloudPlan &cp : plan->c)
        MLBM_HIP(launch_init(cp, plan->precision, node_at(rho, cp), node_at(ux, cp),
                             node_at(uy, cp), state_at(plan, f, cp), false, s));
    return MLBM_OK;
}

mlbm_status mlbm_collide(const mlbm_plan *plan, const void *f, void *g, hipStream_t s) {
    if (!single(plan) || !f || !g) return fail(MLBM_EINVAL, "null plan or state");
    if (f == g) return fail(MLBM_EINVAL, "collide needs distinct input and output");
    for (const CloudPlan &cp : plan->c)
        MLBM_HIP(launch_collide(cp, plan->precision, state_at(plan, f, cp), state_at(plan, g, cp), s));
    return MLBM_OK;
}

mlbm_status mlbm_step(const mlbm_plan *plan, void *g_a, void *g_b, int32_t n_steps,
                      int32_t *result_in_b, hipStream_t s) {
    if (!single(plan) || !g_a || !g_b || n_steps < 0) return fail(MLBM_EINVAL, "bad step arguments");
    if (g_a == g_b) return fail(MLBM_EINVAL, "ping-pong buffers must differ");
    void *cur = g_a, *nxt = g_b;
    for (int t = 0; t < n_steps; ++t) {
        MLBM_HIP(step_once(plan, cur, nxt, nullptr, s));
        std::swap(cur, nxt);
    }
    if (result_in_b) *result_in_b = (n_steps & 1) ? 1 : 0;
    return MLBM_OK;
}

mlbm_status mlbm_step_record(const mlbm_plan *plan, void *g_a, void *g_b, int32_t n_steps,
                             void *f_rec, int32_t *result_in_b, hipStream_t s) {
    if (!single(plan) || !g_a || !g_b || !f_rec || n_steps < 0)
        return fail(MLBM_EINVAL, "bad step arguments");
    if (g_a == g_b) return fail(MLBM_EINVAL, "ping-pong buffers must differ");
    const size_t sb = (size_t)9 * plan->n_total * state_elem_bytes(plan->precision);
    void *cur = g_a, *nxt = g_b;
    for (int t = 0; t < n_steps; ++t) {
        MLBM_HIP(step_once(plan, cur, nxt, (char *)f_rec + sb * t, s));
        std::swap(cur, nxt);
    }
    if (result_in_b) *result_in_b = (n_steps & 1) ? 1 : 0;
    return MLBM_OK;
}

mlbm_status mlbm_moments(const mlbm_plan *plan, const void *g, double *rho, double *ux,
                         double *uy, hipStream_t s) {
    if (!single(plan) || !g) return fail(MLBM_EINVAL, "null plan or state");
    for (const CloudPlan &cp : plan->c)
        MLBM_HIP(launch_moments(cp, plan->precision, state_at(plan, g, cp), out_at(rho, cp),
                                out_at(ux, cp), out_at(uy, cp), true, s));
    return MLBM_OK;
}

mlbm_status mlbm_interpolate(const mlbm_plan *plan, const double *field, double *out,
                             hipStream_t s) {
    if (!single(plan) || !field || !out) return fail(MLBM_EINVAL, "null argument");
    for (const CloudPlan &cp : plan->c)
        if (!cp.W64)
            return fail(MLBM_EUNSUPPORTED, "plan was built with fp32_weights_only: no FP64 shape vectors");
    for (const CloudPlan &cp : plan->c)
        MLBM_HIP(launch_interpolate(cp, node_at(field, cp), plan->n_total, out_at(out, cp), s));
    return MLBM_OK;
}

mlbm_status mlbm_l2_sums(const mlbm_plan *plan, const void *g, const double *ux_t,
                         const double *uy_t, double *out, hipStream_t s) {
    if (!single(plan) || !g || !ux_t || !uy_t || !out) return fail(MLBM_EINVAL, "null argument");
    if (plan->c.size() == 1) {
        MLBM_HIP(launch_l2(plan->c[0], plan->precision, g, ux_t, uy_t, out, plan->scratch64, s));
        return MLBM_OK;
    }
    // per-cloud sums into the scratch head, then one fixed-order sum of those
    double *sums = plan->scratch64;
    double *part = plan->scratch64 + 4 * plan->c.size();
    for (size_t c = 0; c < plan->c.size(); ++c) {
        const CloudPlan &cp = plan->c[c];
        MLBM_HIP(launch_l2(cp, plan->precision, state_at(plan, g, cp), node_at(ux_t, cp),
                           node_at(uy_t, cp), sums + 4 * c, part, s));
    }
    MLBM_HIP(launch_l2_final(sums, (int64_t)plan->c.size(), out, s));
    return MLBM_OK;
}

mlbm_status mlbm_residual(const mlbm_plan *plan, const void *g, double *speed, double *out,
                          hipStream_t s) {
    if (!single(plan) || !g || !speed || !out) return fail(MLBM_EINVAL, "null argument");
    if (plan->c.size() == 1) {
        MLBM_HIP(launch_residual(plan->c[0], plan->precision, g, speed, out, plan->scratch64, s));
        return MLBM_OK;
    }
    double *sums = plan->scratch64;
    double *part = plan->scratch64 + 4 * plan->c.size();
    for (size_t c = 0; c < plan->c.size(); ++c) {
        const CloudPlan &cp = plan->c[c];
        MLBM_HIP(launch_residual(cp, plan->precision, state_at(plan, g, cp),
                                 speed + cp.off, sums + 4 * c, part, s));
    }
    MLBM_HIP(launch_l2_final(sums, (int64_t)plan->c.size(), out, s));
    return MLBM_OK;
}

namespace {
mlbm_status check_lattice(int32_t nx, int32_t ny, int32_t precision) {
    if (nx < 1 || ny < 1 || (int64_t)nx * ny > INT32_MAX / kQ)
        return fail(MLBM_EINVAL, "lattice size out of range");
    if (precision != MLBM_FP32_DEV && precision != MLBM_FP64)
        return fail(MLBM_EINVAL, "unknown precision");
    return MLBM_OK;
}
}  // namespace

mlbm_status mlbm_lbm_init(int32_t nx, int32_t ny, int32_t precision, double rho0,
                          const double *rho, const double *ux, const double *uy, void *g,
                          hipStream_t s) {
    mlbm_status st = check_lattice(nx, ny, precision);
    if (st != MLBM_OK) return st;
    if (!g) return fail(MLBM_EINVAL, "null state");
    MLBM_HIP(launch_lbm_init(nx * ny, precision, rho0, rho, ux, uy, g, s));
    return MLBM_OK;
}

mlbm_status mlbm_lbm_step(int32_t nx, int32_t ny, int32_t precision, double tau, double rho0,
                          void *g_a, void *g_b, int32_t n_steps, int32_t *result_in_b,
                          hipStream_t s) {
    mlbm_status st = check_lattice(nx, ny, precision);
    if (st != MLBM_OK) return st;
    if (!g_a || !g_b || g_a == g_b) return fail(MLBM_EINVAL, "two distinct state buffers needed");
    if (!(tau > 0.5)) return fail(MLBM_EINVAL, "tau must exceed 1/2");
    if (n_steps < 0) return fail(MLBM_EINVAL, "negative step count");
    void *a = g_a, *b = g_b;
    for (int32_t t = 0; t < n_steps; ++t) {
        MLBM_HIP(launch_lbm_step(nx, ny, precision, tau, rho0, a, b, s));
        std::swap(a, b);
    }
    if (result_in_b) *result_in_b = (n_steps & 1) ? 1 : 0;
    return MLBM_OK;
}

mlbm_status mlbm_lbm_moments(int32_t nx, int32_t ny, int32_t precision, double rho0,
                             const void *g, double *rho, double *ux, double *uy, hipStream_t s) {
    mlbm_status st = check_lattice(nx, ny, precision);
    if (st != MLBM_OK) return st;
    if (!g) return fail(MLBM_EINVAL, "null state");
    MLBM_HIP(launch_lbm_moments(nx * ny, precision, rho0, g, rho, ux, uy, s));
    return MLBM_OK;
}

mlbm_status mlbm_loss_seed(const mlbm_plan *plan, const void *f_T, const double *ux_t,
                           const double *uy_t, void *lamf_T, double *J, hipStream_t s) {
    const CloudPlan *cp = single(plan);
    if (cp && plan->c.size() != 1) return fail(MLBM_EUNSUPPORTED, "the adjoint needs a single-cloud plan");
    if (!cp || !f_T || !ux_t || !uy_t || !lamf_T || !J) return fail(MLBM_EINVAL, "null argument");
    if (cp->prm.force_kind || cp->has_walls)
        return fail(MLBM_EUNSUPPORTED, "adjoint without walls or force only");
    MLBM_HIP(launch_loss_seed(*cp, plan->precision, f_T, ux_t, uy_t, lamf_T, J,
                              plan->scratch64, s));
    return MLBM_OK;
}

mlbm_status mlbm_step_adjoint(const mlbm_plan *plan, const void *f_n, const void *lamf_next,
                              void *lamf_n, double *dJ_dtau, hipStream_t s) {
    const CloudPlan *cp = single(plan);
    if (cp && plan->c.size() != 1) return fail(MLBM_EUNSUPPORTED, "the adjoint needs a single-cloud plan");
    if (!cp || !f_n || !lamf_next || !lamf_n || !dJ_dtau) return fail(MLBM_EINVAL, "null argument");
    if (!cp->tr_ptr) return fail(MLBM_EINVAL, "plan was built without with_adjoint");
    if (lamf_next == lamf_n) return fail(MLBM_EINVAL, "adjoint buffers must differ");
    MLBM_HIP(launch_step_adjoint(*cp, plan->precision, f_n, lamf_next, lamf_n, dJ_dtau,
                                 plan->scratch64, s));
    return MLBM_OK;
}

mlbm_status mlbm_init_adjoint(const mlbm_plan *plan, const double *u0x, const double *u0y,
                              const void *lamf_0, double *dJ_du0x, double *dJ_du0y,
                              hipStream_t s) {
    const CloudPlan *cp = single(plan);
    if (cp && plan->c.size() != 1) return fail(MLBM_EUNSUPPORTED, "the adjoint needs a single-cloud plan");
    if (!cp || !lamf_0 || !dJ_du0x || !dJ_du0y) return fail(MLBM_EINVAL, "null argument");
    MLBM_HIP(launch_init_adjoint(*cp, plan->precision, u0x, u0y, lamf_0, dJ_du0x, dJ_du0y, s));
    return MLBM_OK;
}

mlbm_status mlbm_plan_set_variant(mlbm_plan *plan, int32_t variant) {
    if (!plan || plan->c.empty()) return fail(MLBM_EINVAL, "null plan");
    if (variant < 0 || variant >= kStepVariants) return fail(MLBM_EINVAL, "unknown variant");
    for (auto &cp : plan->c) cp.variant = variant;
    drop_graph(plan);
    return MLBM_OK;
}

mlbm_status mlbm_autotune(mlbm_plan *plan, void *g_a, void *g_b, int32_t n_steps,
                          float *ms_out, int32_t *n_variants, hipStream_t s) {
    if (!plan || plan->c.empty() || !g_a || !g_b || n_steps < 1)
        return fail(MLBM_EINVAL, "bad autotune arguments");
    if (g_a == g_b) return fail(MLBM_EINVAL, "ping-pong buffers must differ");
    const int nv = plan->precision == MLBM_FP64 ? 1 : kStepVariants;
    if (n_variants) *n_variants = nv;
    if (nv == 1) {
        if (ms_out) ms_out[0] = 0.0f;
        return MLBM_OK;
    }
    hipEvent_t e0, e1;
    MLBM_HIP(hipEventCreate(&e0));
    hipError_t err = hipEventCreate(&e1);
    if (err != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(err, "hipEventCreate");
    }
    int best = 0;
    float best_ms = 0.0f;
    mlbm_status st = MLBM_OK;
    for (int v = 0; v < nv && st == MLBM_OK; ++v) {
        for (auto &cp : plan->c) cp.variant = v;
        int32_t rb = 0;
        st = mlbm_step(plan, g_a, g_b, 1, &rb, s);               // warm-up
        if (st != MLBM_OK) break;
        void *a = rb ? g_b : g_a, *b = rb ? g_a : g_b;
        if ((err = hipEventRecord(e0, s)) != hipSuccess) { st = hip_fail(err, "hipEventRecord"); break; }
        st = mlbm_step(plan, a, b, n_steps, &rb, s);
        if (st != MLBM_OK) break;
        if ((err = hipEventRecord(e1, s)) != hipSuccess) { st = hip_fail(err, "hipEventRecord"); break; }
        if ((err = hipEventSynchronize(e1)) != hipSuccess) { st = hip_fail(err, "hipEventSynchronize"); break; }
        float ms = 0.0f;
        if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { st = hip_fail(err, "hipEventElapsedTime"); break; }
        ms /= (float)n_steps;
        if (ms_out) ms_out[v] = ms;
        if (v == 0 || ms < best_ms) {
            best_ms = ms;
            best = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (auto &cp : plan->c) cp.variant = best;
    drop_graph(plan);
    return st;
}

mlbm_status mlbm_graph_create(mlbm_plan *plan, void *g_a, void *g_b, int32_t n_steps,
                              hipStream_t s) {
    if (!single(plan) || !g_a || !g_b || n_steps < 1) return fail(MLBM_EINVAL, "bad graph arguments");
    if (!s) return fail(MLBM_EINVAL, "graph capture needs a non-default stream");
    if (g_a == g_b) return fail(MLBM_EINVAL, "ping-pong buffers must differ");
    drop_graph(plan);
    MLBM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    void *cur = g_a, *nxt = g_b;
    hipError_t err = hipSuccess;
    for (int t = 0; t < n_steps && err == hipSuccess; ++t) {
        err = step_once(plan, cur, nxt, nullptr, s);
        std::swap(cur, nxt);
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (err != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(err, "step launch under capture");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    plan->graph = graph;
    MLBM_HIP(hipGraphInstantiate(&plan->graph_exec, graph, nullptr, nullptr, 0));
    return MLBM_OK;
}

mlbm_status mlbm_build_graph(const mlbm_cloud *clouds, const mlbm_params *params,
                             int32_t n_clouds, void *plan_buf, size_t plan_bytes,
                             void *workspace, size_t workspace_bytes, const double *rho,
                             const double *ux, const double *uy, void *g_a, void *g_b,
                             int32_t n_steps, int32_t variant, mlbm_plan **out, hipStream_t s) {
    if (!out) return fail(MLBM_EINVAL, "null output pointer");
    *out = nullptr;
    if (!s) return fail(MLBM_EINVAL, "graph capture needs a non-default stream");
    if (!g_a || !g_b || g_a == g_b || n_steps < 0) return fail(MLBM_EINVAL, "bad state buffers");
    if (variant < 0 || variant >= kStepVariants) return fail(MLBM_EINVAL, "unknown variant");
    if (n_clouds > 1 && !lane_pool()) return fail(MLBM_EHIP, "could not create the build streams");
    MLBM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    mlbm_plan *plan = nullptr;
    mlbm_status st = mlbm_build_weights(clouds, params, n_clouds, plan_buf, plan_bytes, workspace,
                                        workspace_bytes, &plan, s);
    if (st == MLBM_OK) {
        for (auto &cp : plan->c) cp.variant = variant;
        st = mlbm_init(plan, rho, ux, uy, g_a, s);
    }
    if (st == MLBM_OK) st = mlbm_step(plan, g_a, g_b, n_steps, nullptr, s);
    const std::string msg = g_error;
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (st != MLBM_OK || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (plan) mlbm_plan_destroy(plan);
        return st != MLBM_OK ? fail(st, msg) : hip_fail(e2, "hipStreamEndCapture");
    }
    plan->graph = graph;
    hipError_t e3 = hipGraphInstantiate(&plan->graph_exec, graph, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
        mlbm_plan_destroy(plan);
        return hip_fail(e3, "hipGraphInstantiate");
    }
    *out = plan;
    return MLBM_OK;
}

mlbm_status mlbm_graph_launch(mlbm_plan *plan, hipStream_t s) {
    if (!plan || !plan->graph_exec) return fail(MLBM_EINVAL, "no graph on this plan");
    MLBM_HIP(hipGraphLaunch(plan->graph_exec, s));
    return MLBM_OK;
}

}  // extern "C"
