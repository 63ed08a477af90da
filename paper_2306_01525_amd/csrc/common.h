// Internal declarations of the MLBM HIP library (gfx950). Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mlbm.h"

namespace mlbm {

// ---------------------------------------------------------------------------
// D2Q9 lattice (Sec. 2.1): directions k = 0..8 in the paper's order
// (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1); weights 4/9,
// 1/9 (axes), 1/36 (diagonals); c_s^2 = 1/3.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int lat_ex(int k) {
    return (k == 1 || k == 5 || k == 8) ? 1 : (k == 3 || k == 6 || k == 7) ? -1 : 0;
}
__host__ __device__ constexpr int lat_ey(int k) {
    return (k == 2 || k == 5 || k == 6) ? 1 : (k == 4 || k == 7 || k == 8) ? -1 : 0;
}
__host__ __device__ constexpr double lat_w(int k) {
    return k == 0 ? 4.0 / 9.0 : (k <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
}
// opposite direction: 1<->3, 2<->4, 5<->7, 6<->8
__host__ __device__ constexpr int lat_opp(int k) {
    return k == 0 ? 0 : (k <= 4 ? ((k + 1) & 3) + 1 : ((k - 3) & 3) + 5);
}
static_assert(lat_opp(1) == 3 && lat_opp(2) == 4 && lat_opp(3) == 1 && lat_opp(4) == 2 &&
              lat_opp(5) == 7 && lat_opp(6) == 8 && lat_opp(7) == 5 && lat_opp(8) == 6,
              "opposite directions");

constexpr int kQ = 9;

// w_k x for a lattice weight w_k. 4/9, 1/9 and 1/36 are not binary fractions,
// and their FP32 roundings are all high by the same relative 7.5e-9: an FP32
// equilibrium built on them carries that much excess mass and momentum, which
// every collision feeds back (a gain of 7.5e-9/tau per step that accumulates
// linearly in time). In FP32 the weight is therefore applied as two FP32 parts
// whose sum is w_k to 48 bits, so the product is rounded once from a nearly
// exact value.
template <class T>
__device__ __forceinline__ T lat_wmul(int k, T x) {
    return (T)lat_w(k) * x;
}
template <>
__device__ __forceinline__ float lat_wmul<float>(int k, float x) {
    const float hi = (float)lat_w(k);
    const float lo = (float)(lat_w(k) - (double)hi);
    return __builtin_fmaf(hi, x, lo * x);
}

// FP64 shape vectors, layout [K][4][n][2]: slot j of directions (1,2), (3,4),
// (5,6), (7,8) of node p form one 16-byte pair, so a lane reads two directions
// per load and a wavefront reads 1 KiB of consecutive memory.
__host__ __device__ inline int64_t w64_at(int k, int j, int64_t n, int64_t p) {
    return (((int64_t)j * 4 + ((k - 1) >> 1)) * n + p) * 2 + ((k - 1) & 1);
}
constexpr int kMaxK = 48;       // largest stencil supported
constexpr unsigned kCaptureLds = 40 * 1024;   // FP32 step LDS of a plan built under capture
// Nodes rounded up to whole wavefronts: the row heads of the transposed
// operator are compacted per group of 64 nodes, and each slot of a group has
// room for all 64.
inline int64_t head_nodes(int n) { return ((int64_t)n + 63) / 64 * 64; }
constexpr int kTile = 256;      // nodes per workgroup in the step kernels
constexpr int kHaloCap = 1024;  // largest halo a tile stages (10-bit positions)
constexpr int kStepVariants = MLBM_STEP_VARIANTS; // FP32 step tuning variants
constexpr int kBuildLanes = 4;   // clouds of one plan built concurrently
constexpr int kStats = 4;        // build records per cloud (tile tables)

inline int poly_count(int m) { return (m + 1) * (m + 2) / 2; }

// Geometry of the uniform search grid of one cloud (device resident).
struct Geo {
    double x0, y0;      // grid origin
    double cw, ch;      // cell width and height
    double Lx, Ly;      // periods (0 = open)
    int gx, gy;         // cells per axis (powers of two)
    int hb;             // Hilbert order: grid side 2^hb >= max(gx, gy)
    int pad;
};

// One cloud inside a plan. Pointers are device addresses inside the caller's
// plan buffer; arrays are in internal (Hilbert) node order unless stated.
struct CloudPlan {
    int64_t off = 0;          // offset of this cloud's nodes in state arrays
    int32_t n = 0;
    mlbm_params prm{};
    int K = 0, m = 0, M = 0;
    double Lx = 0, Ly = 0;
    bool has_walls = false;      // equilibrium wall nodes (wall_kind 1)
    uint8_t *links = nullptr;    // [n] bounce-back link masks (wall_kind 2)
    bool imported = false;
    Geo *geo = nullptr;       // device
    double *xs = nullptr, *ys = nullptr;     // [n]
    int32_t *perm = nullptr;  // [n] internal -> user index
    int32_t *iperm = nullptr; // [n] user -> internal
    uint8_t *ntype = nullptr; // [n]
    int32_t *nbr = nullptr;   // [K][n], internal indices, centre first
    int32_t *owner = nullptr; // [8][n] for k = 1..8 (paper mode only)
    double *W64 = nullptr;    // [K][4][n][2] FP64 shape vectors, k = 1..8 (w64_at)
    float *W32 = nullptr;     // [K][2][n][4] FP32 shape vectors, k = 1..8
    float *force32 = nullptr; // [2][n] body force (lattice units), FP32 state
    double *force64 = nullptr;// [2][n] body force, FP64 state
    // tile-local gather tables of the LDS-staged FP32 step (tiles.hip)
    int ocap = 0, hcap = 0;       // capacities per tile: owners, halo nodes
    int32_t *tdesc = nullptr;     // [ntiles][2]: |O_t|, |H_t| (0: global path)
    uint16_t *ownerL = nullptr;   // [8][n] position of owner_k(p) in O_t
    uint32_t *nbrL = nullptr;     // [ntiles][ocap][ceil(K/3)] positions in H_t, 3 x 10 bit
    int32_t *hlist = nullptr;     // [ntiles][hcap] global index of H_t entries
    unsigned lds_bytes = 0;       // dynamic LDS of the step launch (0: no tables)
    int fallback_tiles = -1;      // tiles stepped with global gathers (-1: unknown)
    int variant = 0;              // FP32 step tuning variant (mlbm_autotune)
    // transposed streaming (adjoint): per direction k = 1..8, CSR over the
    // source node m of (arriving node i, weight)
    int32_t *tr_ptr = nullptr;  // [8n+1] row offsets, row (k-1)*n + m
    int32_t *tr_col = nullptr;  // [8Kn] arriving node, ascending within a row
    void *tr_val = nullptr;     // [8Kn] float (FP32 plans) or double (FP64)
    // the first tr_lw = K + 4 entries of every row again (the row heads),
    // compacted per group of 64 nodes: node m's head length hd(m) is the
    // longest of its eight rows (at most tr_lw); group g starts at unit
    // 64 g tr_lw, and its slot e holds one unit (eight directions) for each node
    // of the group with hd > e, in node order, stored as the block's first
    // halves (directions 1-4) and then its second halves (adjoint.hip,
    // unit_entry)
    int tr_lw = 0;
    int32_t *ell_col = nullptr;   // [tr_lw * n64][8], n64 = n rounded up to 64
    void *ell_val = nullptr;      // same layout, float or double
    // inverse halos of source tiles for the LDS-staged adjoint gather
    int32_t *tdescT = nullptr;    // [ntiles] |I_t| (0: global gathers)
    int32_t *ilist = nullptr;     // [ntiles][hcap] arriving nodes, sorted
    uint32_t *elocal = nullptr;   // the row heads' columns as three 10-bit positions
                                  // in I_t per word, compacted like ell_col over
                                  // triples of slots: [ceil(tr_lw/3) * n64][8]
    int adj_cap = 0;              // largest |I_t| kept (10-bit positions: at most 1024)
    int adj_ni = 0;               // largest |I_t| (LDS of the adjoint launch: 8 |I_t| values)
    int32_t *err = nullptr;       // the plan's device error words (kErrWords)
};

// Device error words of a plan (int32, sticky until cleared):
//   [kErrSingular] 1 + user index of the first node with a singular local
//                  system, INT_MAX when none (build);
//   [kErrFlags]    MLBM_DEVERR_* bits found by the steps and the diagnostics;
//   [kErrNode]     user index of the first node found non-finite or too fast,
//                  INT_MAX when none or not known.
constexpr int kErrSingular = 0, kErrFlags = 1, kErrNode = 2, kErrWords = 64;
// Largest speed (lattice units) before a node is reported as diverging: BGK
// with the second-order equilibrium is only consistent well below c_s = 0.577.
constexpr float kMaxSpeed2 = 0.09f;

// Check of one node's squared speed uu: a NaN fails every comparison, so a
// node whose moments are not finite or whose speed exceeds the limit is
// reported (code MLBM_DEVERR_NONFINITE or MLBM_DEVERR_SPEED, and the lowest
// such user index). The branch is taken only by a diverging run.
// A diverging run fails at most of its nodes every step, so the words are
// read first and written only when that adds a bit or lowers the node: the
// atomics stay rare instead of serialising every lane on one address.
template <class T>
__device__ __forceinline__ void check_speed(int32_t *err, T uu, const int32_t *perm, int p,
                                            int uoff) {
    if (uu <= (T)kMaxSpeed2 || !err) return;
    const bool finite = (uu - uu) == (T)0;   // false for NaN and Inf
    const int code = finite ? MLBM_DEVERR_SPEED : MLBM_DEVERR_NONFINITE;
    const int user = uoff + (perm ? perm[p] : p);
    if ((__atomic_load_n(err + kErrFlags, __ATOMIC_RELAXED) & code) != code)
        atomicOr(err + kErrFlags, code);
    if (user < __atomic_load_n(err + kErrNode, __ATOMIC_RELAXED)) atomicMin(err + kErrNode, user);
}
__device__ __forceinline__ void report_index(int32_t *err) {
    if (err && !(__atomic_load_n(err + kErrFlags, __ATOMIC_RELAXED) & MLBM_DEVERR_INDEX))
        atomicOr(err + kErrFlags, MLBM_DEVERR_INDEX);
}

// Arguments of the FP32 step for one cloud; also the per-cloud descriptor
// of the batched step (soff: element offset of the cloud's state, tile_begin:
// its first tile in the batch).
struct Step32Args {
    int n, K, ocap, hcap;
    const float4 *W;
    const int32_t *nbr, *owner;
    const float *force;
    const uint8_t *ntype;
    float rtau, rho0, rho_w;
    float *frec;
    const int32_t *tdesc;
    const uint16_t *ownerL;
    const uint32_t *nbrL;
    const int32_t *hlist;
    int64_t soff, tile_begin;
    int32_t *err;            // device error words (may be null)
    const int32_t *perm;     // internal -> user index of this cloud
    int uoff;                // offset of this cloud's nodes in the plan's user order
    int lcap;                // LDS bytes of the launch: a tile whose tables need more
                             // gathers from global memory instead
};

// Tile ranges of the eight XCDs in a launch over several clouds: XCD x takes
// tiles [begin[x], begin[x + 1]). The ranges are contiguous and carry about
// equal work rather than equal tile counts, tiles of clouds with larger
// stencils costing more; the grid is 8 * the longest range.
struct XcdSplit {
    int64_t begin[9];
};

// Bump allocator over a caller buffer (a null base computes sizes only).
struct Carve {
    char *base;
    size_t used = 0;
    explicit Carve(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        used = (used + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += count * sizeof(T);
        return p;
    }
};

}  // namespace mlbm

struct mlbm_plan {
    std::vector<mlbm::CloudPlan> c;
    int64_t n_total = 0;
    // batched FP32 step over several clouds (one launch per step)
    bool batched = false;           // every cloud can use the batched kernel
    int batch_mode = 0;             // common stencil mode of the batch
    int64_t total_tiles = 0;
    mlbm::Step32Args *descs = nullptr;   // device [n_clouds]
    int32_t *tile2cloud = nullptr;       // device [total_tiles]
    unsigned batch_lds = 0;
    mlbm::XcdSplit xcd{};                // tile ranges of the XCDs
    int64_t xcd_longest = 0;             // longest of those ranges
    int precision = MLBM_FP32_DEV;
    int32_t *dev_err = nullptr;     // device error words (kErrWords int32)
    int32_t *stats = nullptr;       // device [n_clouds][kStats]: tile-table records
    double *scratch64 = nullptr;    // device, small reductions
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
};

namespace mlbm {

// Thread-local error message.
void set_error(const std::string &msg);
mlbm_status fail(mlbm_status st, const std::string &msg);
mlbm_status hip_fail(hipError_t e, const char *what);

#define MLBM_HIP(call)                                      \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return ::mlbm::hip_fail(e_, #call); \
    } while (0)

inline size_t state_elem_bytes(int precision) {
    return precision == MLBM_FP64 ? sizeof(double) : sizeof(float);
}

// Grid sizes for launches.
inline unsigned blocks_for(int64_t n, int threads) {
    return static_cast<unsigned>((n + threads - 1) / threads);
}

// Workgroup -> tile map that gives each XCD a contiguous range of tiles (the
// hardware deals workgroups round-robin over the 8 XCDs, each with its own
// L2), so neighbouring tiles, which share stencil members, share an L2. The
// grid is xcd_grid(nblocks); workgroups mapped past the last tile do nothing.
__device__ __forceinline__ int64_t xcd_tile(int64_t nblocks) {
    const int64_t b = blockIdx.x;
    const int64_t per = (nblocks + 7) / 8;
    return (b & 7) * per + (b >> 3);
}

inline unsigned xcd_grid(int64_t nblocks) { return (unsigned)(((nblocks + 7) / 8) * 8); }


// This workgroup's tile under an XcdSplit, or -1 past the end of its XCD's range.
__device__ __forceinline__ int64_t xcd_split_tile(const XcdSplit &r) {
    const int x = blockIdx.x & 7;
    int64_t b = r.begin[0], e = r.begin[1];
#pragma unroll
    for (int i = 1; i < 8; ++i)
        if (x == i) {
            b = r.begin[i];
            e = r.begin[i + 1];
        }
    const int64_t t = b + (blockIdx.x >> 3);
    return t < e ? t : -1;
}

// ---- build stages (build.hip) ----
hipError_t launch_geo_periodic(Geo *geo, double Lx, double Ly, int gx, int gy, int hb,
                               hipStream_t s);
hipError_t launch_geo_bbox(Geo *geo, const double *x, const double *y, int n, int gx,
                           int gy, int hb, hipStream_t s);
hipError_t launch_keys(const Geo *geo, const double *x, const double *y, int n,
                       uint32_t *keys, int32_t *vals, hipStream_t s);
hipError_t launch_scatter_sorted(const Geo *geo, const double *x, const double *y,
                                 const uint8_t *nt, const int32_t *perm,
                                 const uint32_t *skeys, int n, double *xs, double *ys,
                                 uint8_t *ntype, int32_t *iperm, int32_t *cstart,
                                 int32_t *cend, int ncells, hipStream_t s);
hipError_t launch_knn(const Geo *geo, const double *xs, const double *ys,
                      const int32_t *perm, const int32_t *iperm, const int32_t *cstart,
                      const int32_t *cend, int n, int K, int32_t *nbr, hipStream_t s);
hipError_t launch_owner(const Geo *geo, const double *xs, const double *ys,
                        const int32_t *perm, const int32_t *iperm, const int32_t *cstart,
                        const int32_t *cend, int n, double dx, int32_t *owner,
                        hipStream_t s);
// workspace of the paper-mode owner lists: counts [n], offsets [n+1],
// points [8n], scan temp
size_t rbf_temp_bytes(int n);
hipError_t launch_rbf(const Geo *geo, const double *xs, const double *ys,
                      const int32_t *perm, const int32_t *nbr, const int32_t *owner,
                      int n, int K, int m, double dx, int mode, void *tmp, size_t tmp_bytes,
                      double *W64, int32_t *dev_err, hipStream_t s);
hipError_t launch_pack_w32(const double *W64, int n, int K, float *W32, hipStream_t s);
hipError_t launch_force(const double *xs, const double *ys, const uint8_t *ntype, int n,
                        int kind, double mag, float *f32, double *f64, hipStream_t s);
// bounce-back links of wall nodes: links[p] bit k-1 set where ntype[p] and
// e_k . n(user(p)) < 0
hipError_t launch_links(const uint8_t *ntype, const int32_t *perm, const double *nx,
                        const double *ny, int n, uint8_t *links, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);

// ---- tile tables (tiles.hip) ----
// stats[0] <- max LDS bytes over tiles, stats[1] <- number of fallback tiles
hipError_t launch_tiles(const CloudPlan &cp, int32_t *stats, hipStream_t s);

// ---- sort / scan (sort.hip) ----
size_t sort_pairs_temp_bytes(int n);
hipError_t sort_pairs(void *tmp, size_t tmp_bytes, const uint32_t *kin, uint32_t *kout,
                      const int32_t *vin, int32_t *vout, int n, int end_bit, hipStream_t s);
size_t scan_temp_bytes(int n);
hipError_t exclusive_scan(void *tmp, size_t tmp_bytes, const int32_t *in, int32_t *out,
                          int n, hipStream_t s);

// ---- stepping (step.hip) ----
hipError_t launch_init(const CloudPlan &cp, int precision, const double *rho,
                       const double *ux, const double *uy, void *g, bool collide,
                       hipStream_t s);
hipError_t launch_step(const CloudPlan &cp, int precision, const void *gin, void *gout,
                       void *frec, hipStream_t s);
Step32Args step32_args(const CloudPlan &cp, void *frec);
hipError_t launch_step_batch(const mlbm_plan &plan, const void *gin, void *gout,
                             hipStream_t s);
hipError_t launch_set_desc(Step32Args *dst, const Step32Args &v, hipStream_t s);
hipError_t launch_moments(const CloudPlan &cp, int precision, const void *g, double *rho,
                          double *ux, double *uy, bool post_collision, hipStream_t s);
hipError_t launch_l2(const CloudPlan &cp, int precision, const void *g, const double *uxt,
                     const double *uyt, double *out, double *part, hipStream_t s);
// speed: device FP64 [n] user order, in/out; out[0..3] as launch_l2
hipError_t launch_residual(const CloudPlan &cp, int precision, const void *g, double *speed,
                           double *out, double *part, hipStream_t s);
// field: device FP64 [n] of this cloud (user order); out[k-1][u] at out + (k-1)*out_stride
hipError_t launch_interpolate(const CloudPlan &cp, const double *field, int64_t out_stride,
                              double *out, hipStream_t s);
// standard lattice Boltzmann on a periodic nx x ny lattice, state [9][ny][nx]
hipError_t launch_lbm_step(int nx, int ny, int precision, double tau, double rho0,
                           const void *g, void *go, hipStream_t s);
hipError_t launch_lbm_init(int n, int precision, double rho0, const double *rho, const double *ux,
                           const double *uy, void *g, hipStream_t s);
hipError_t launch_lbm_moments(int n, int precision, double rho0, const void *g, double *rho,
                              double *ux, double *uy, hipStream_t s);
hipError_t launch_collide(const CloudPlan &cp, int precision, const void *f, void *g,
                          hipStream_t s);
hipError_t launch_l2_final(const double *part, int64_t nparts, double *out, hipStream_t s);

// ---- adjoint (adjoint.hip) ----
// workspace of the transpose build: counts/cursors [8n] + scan temp
size_t transpose_temp_bytes(int n, int K);
hipError_t launch_transpose(const CloudPlan &cp, int precision, void *tmp, size_t tmp_bytes,
                            hipStream_t s);
hipError_t launch_ell_fill(const CloudPlan &cp, int precision, hipStream_t s);
// stats[0] <- largest inverse halo, stats[1] <- tiles without one
hipError_t launch_adj_tiles(const CloudPlan &cp, int32_t *stats, hipStream_t s);
hipError_t launch_loss_seed(const CloudPlan &cp, int precision, const void *fT,
                            const double *uxt, const double *uyt, void *lam, double *J,
                            double *part, hipStream_t s);
hipError_t launch_step_adjoint(const CloudPlan &cp, int precision, const void *fn,
                               const void *lam_next, void *lam_n, double *dtau, double *part,
                               hipStream_t s);
hipError_t launch_init_adjoint(const CloudPlan &cp, int precision, const double *u0x,
                               const double *u0y, const void *lam0, double *gx, double *gy,
                               hipStream_t s);

}  // namespace mlbm
