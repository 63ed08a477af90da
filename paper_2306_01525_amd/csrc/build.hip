// Weight build of the MLBM on gfx950: space-filling-curve ordering, stencil
// and owner searches on a uniform cell grid, and the FP64 local RBF solves.
//
// This translation unit is compiled with -ffp-contract=off: squared distances
// are rounded exactly as written, so stencil ties are decided on bitwise equal
// distances and then by user index, as in the definition of the stencil.
#include <cfloat>
#include <climits>

#include "common.h"

namespace mlbm {
namespace {

__device__ __forceinline__ double min_image(double d, double L) {
    if (L > 0.0) {
        if (d > 0.5 * L) d -= L;
        else if (d < -0.5 * L) d += L;
    }
    return d;
}

__device__ __forceinline__ double dist2(double ax, double ay, double bx, double by,
                                        double Lx, double Ly) {
    double dx = min_image(bx - ax, Lx);
    double dy = min_image(by - ay, Ly);
    return dx * dx + dy * dy;
}

// Index of cell (x, y) along the Hilbert curve of a 2^order x 2^order grid
// (the classic quadrant-rotation construction).
__device__ uint32_t hilbert_index(uint32_t x, uint32_t y, int order) {
    uint32_t d = 0;
    const uint32_t side = 1u << order;
    for (uint32_t s = side >> 1; s > 0; s >>= 1) {
        uint32_t rx = (x & s) ? 1u : 0u;
        uint32_t ry = (y & s) ? 1u : 0u;
        d += s * s * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = side - 1 - x;
                y = side - 1 - y;
            }
            uint32_t t = x;
            x = y;
            y = t;
        }
    }
    return d;
}

__device__ __forceinline__ void cell_of(const Geo &g, double x, double y, int &cx, int &cy) {
    double fx = floor((x - g.x0) / g.cw);
    double fy = floor((y - g.y0) / g.ch);
    cx = fx < 0 ? 0 : (fx >= g.gx ? g.gx - 1 : (int)fx);
    cy = fy < 0 ? 0 : (fy >= g.gy ? g.gy - 1 : (int)fy);
}

__global__ void k_geo_periodic(Geo *geo, double Lx, double Ly, int gx, int gy, int hb) {
    Geo g;
    g.x0 = 0.0;
    g.y0 = 0.0;
    g.cw = Lx / gx;
    g.ch = Ly / gy;
    g.Lx = Lx;
    g.Ly = Ly;
    g.gx = gx;
    g.gy = gy;
    g.hb = hb;
    g.pad = 0;
    *geo = g;
}

// Bounding box of an open cloud (one workgroup).
__global__ __launch_bounds__(1024) void k_geo_bbox(Geo *geo, const double *x, const double *y,
                                                   int n, int gx, int gy, int hb) {
    __shared__ double s[4][1024];
    double mnx = DBL_MAX, mny = DBL_MAX, mxx = -DBL_MAX, mxy = -DBL_MAX;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        mnx = fmin(mnx, x[i]);
        mxx = fmax(mxx, x[i]);
        mny = fmin(mny, y[i]);
        mxy = fmax(mxy, y[i]);
    }
    s[0][threadIdx.x] = mnx;
    s[1][threadIdx.x] = mxx;
    s[2][threadIdx.x] = mny;
    s[3][threadIdx.x] = mxy;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + w]);
            s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][threadIdx.x + w]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double ex = s[1][0] - s[0][0], ey = s[3][0] - s[2][0];
        double e = fmax(fmax(ex, ey), 1e-300);
        Geo g;
        g.x0 = s[0][0] - 1e-9 * e;
        g.y0 = s[2][0] - 1e-9 * e;
        g.cw = (ex + 2e-9 * e) / gx;
        g.ch = (ey + 2e-9 * e) / gy;
        if (!(g.cw > 0)) g.cw = 1.0;
        if (!(g.ch > 0)) g.ch = 1.0;
        g.Lx = 0.0;
        g.Ly = 0.0;
        g.gx = gx;
        g.gy = gy;
        g.hb = hb;
        g.pad = 0;
        *geo = g;
    }
}

__global__ void k_keys(const Geo *__restrict__ geo, const double *__restrict__ x,
                       const double *__restrict__ y, int n, uint32_t *keys, int32_t *vals) {
    int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    Geo g = *geo;
    int cx, cy;
    cell_of(g, x[u], y[u], cx, cy);
    keys[u] = hilbert_index((uint32_t)cx, (uint32_t)cy, g.hb);
    vals[u] = u;
}

__global__ void k_scatter_sorted(const Geo *__restrict__ geo, const double *__restrict__ x,
                                 const double *__restrict__ y, const uint8_t *__restrict__ nt,
                                 const int32_t *__restrict__ perm,
                                 const uint32_t *__restrict__ skeys, int n, double *xs,
                                 double *ys, uint8_t *ntype, int32_t *iperm, int32_t *cstart,
                                 int32_t *cend) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    Geo g = *geo;
    int u = perm[p];
    double px = x[u], py = y[u];
    xs[p] = px;
    ys[p] = py;
    ntype[p] = nt ? nt[u] : (uint8_t)0;
    iperm[u] = p;
    int cx, cy;
    cell_of(g, px, py, cx, cy);
    int c = cy * g.gx + cx;
    uint32_t k = skeys[p];
    if (p == 0 || skeys[p - 1] != k) cstart[c] = p;
    if (p == n - 1 || skeys[p + 1] != k) cend[c] = p + 1;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Ordered insertion of (d, u) into the ascending list held in registers. The
// live entries occupy the tail of the array; the head holds sentinels with
// distance -1 that nothing displaces, so the worst live entry is always the
// last element. Branch-free: entry q of the new list is the old entry q-1
// when the new pair sorts before it, else the new pair when it sorts before
// the old entry q, else the old entry q (the comparisons are independent, so
// the list stays in registers).
template <int KMAX>
__device__ __forceinline__ void topk_insert(double (&bd)[KMAX], int (&bu)[KMAX], double d,
                                            int u) {
    if (!(d < bd[KMAX - 1] || (d == bd[KMAX - 1] && u < bu[KMAX - 1]))) return;
    bool lt[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) lt[q] = d < bd[q] || (d == bd[q] && u < bu[q]);
#pragma unroll
    for (int q = KMAX - 1; q > 0; --q) {
        const double dq = lt[q - 1] ? bd[q - 1] : (lt[q] ? d : bd[q]);
        const int uq = lt[q - 1] ? bu[q - 1] : (lt[q] ? u : bu[q]);
        bd[q] = dq;
        bu[q] = uq;
    }
    if (lt[0]) {
        bd[0] = d;
        bu[0] = u;
    }
}

// Cell of Chebyshev ring r around (cx, cy) number t (0 <= t < 8r, or t = 0 for
// r = 0): its index, or -1 where an open axis has no such cell. Periodic axes
// wrap.
__device__ __forceinline__ int ring_cell(const Geo &g, int cx, int cy, int r, int t) {
    const int span = 2 * r + 1;
    int dx, dy;
    if (r == 0) {
        dx = 0;
        dy = 0;
    } else if (t < span) {        // bottom row
        dx = t - r;
        dy = -r;
    } else if (t < 2 * span) {    // top row
        dx = t - span - r;
        dy = r;
    } else {                      // left and right columns without corners
        const int v = t - 2 * span;
        dx = (v & 1) ? r : -r;
        dy = (v >> 1) - r + 1;
    }
    int ix = cx + dx, iy = cy + dy;
    if (g.Lx > 0.0) ix = (ix % g.gx + g.gx) % g.gx;
    else if (ix < 0 || ix >= g.gx) return -1;
    if (g.Ly > 0.0) iy = (iy % g.gy + g.gy) % g.gy;
    else if (iy < 0 || iy >= g.gy) return -1;
    return iy * g.gx + ix;
}

// Scan the cells of Chebyshev ring r around (cx, cy); `body(q)` runs for every
// node q in those cells.
template <class F>
__device__ __forceinline__ void for_ring(const Geo &g, const int32_t *__restrict__ cstart,
                                         const int32_t *__restrict__ cend, int cx, int cy,
                                         int r, F &&body) {
    const int count = r == 0 ? 1 : 8 * r;
    for (int t = 0; t < count; ++t) {
        const int c = ring_cell(g, cx, cy, r, t);
        if (c < 0) continue;
        const int e = cend[c];
        for (int q = cstart[c]; q < e; ++q) body(q);
    }
}

// Stencil of node p: p itself, then the K-1 closest other nodes by
// (squared distance, user index). Rings of cells are scanned outwards until
// every unscanned node is provably farther than the current (K-1)-th.
template <int KMAX>
__global__ __launch_bounds__(256) void k_knn(const Geo *__restrict__ geo,
                                             const double *__restrict__ xs,
                                             const double *__restrict__ ys,
                                             const int32_t *__restrict__ perm,
                                             const int32_t *__restrict__ iperm,
                                             const int32_t *__restrict__ cstart,
                                             const int32_t *__restrict__ cend, int n, int K,
                                             int32_t *__restrict__ nbr) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const Geo g = *geo;
    const int live = K - 1, first = KMAX - live;
    double bd[KMAX];
    int bu[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
        bd[q] = q < first ? -1.0 : DBL_MAX;
        bu[q] = q < first ? -1 : INT_MAX;
    }
    const double px = xs[p], py = ys[p];
    int cx, cy;
    cell_of(g, px, py, cx, cy);
    const double cmin = fmin(g.cw, g.ch);
    for (int r = 0;; ++r) {
        bool wraps = (g.Lx > 0.0 && 2 * r + 1 > g.gx) || (g.Ly > 0.0 && 2 * r + 1 > g.gy);
        if (wraps) {  // tiny periodic grid: rings would revisit cells, scan all nodes
#pragma unroll
            for (int q = 0; q < KMAX; ++q) {   // static indices keep the list in registers
                bd[q] = q < first ? bd[q] : DBL_MAX;
                bu[q] = q < first ? bu[q] : INT_MAX;
            }
            for (int q = 0; q < n; ++q)
                if (q != p) topk_insert<KMAX>(bd, bu, dist2(px, py, xs[q], ys[q], g.Lx, g.Ly), perm[q]);
            break;
        }
        // (the ring is walked here rather than through for_ring, whose
        // closure would take the list's address)
        const int count = r == 0 ? 1 : 8 * r;
        for (int t = 0; t < count; ++t) {
            const int c = ring_cell(g, cx, cy, r, t);
            if (c < 0) continue;
            const int e = cend[c];
            for (int q = cstart[c]; q < e; ++q)
                if (q != p) topk_insert<KMAX>(bd, bu, dist2(px, py, xs[q], ys[q], g.Lx, g.Ly), perm[q]);
        }
        double reach = r * cmin;
        if (bd[KMAX - 1] < reach * reach) break;
        if (r > g.gx && r > g.gy) break;
    }
    nbr[p] = p;
#pragma unroll
    for (int q = 0; q < KMAX; ++q)
        if (q >= first) nbr[(int64_t)(q - first + 1) * n + p] = iperm[bu[q]];
}

// Owner of each departure point x_p - e_k dx (k = 1..8): the closest node,
// ties to the lower user index.
__global__ __launch_bounds__(256) void k_owner(const Geo *__restrict__ geo,
                                               const double *__restrict__ xs,
                                               const double *__restrict__ ys,
                                               const int32_t *__restrict__ perm,
                                               const int32_t *__restrict__ iperm,
                                               const int32_t *__restrict__ cstart,
                                               const int32_t *__restrict__ cend, int n,
                                               double dx, int32_t *__restrict__ owner) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const Geo g = *geo;
    const double cmin = fmin(g.cw, g.ch);
    for (int k = 1; k < kQ; ++k) {
        double qx = xs[p] - lat_ex(k) * dx;
        double qy = ys[p] - lat_ey(k) * dx;
        // cell of the departure point (wrapped into the periodic box)
        double wx = qx, wy = qy;
        if (g.Lx > 0.0) wx = wx - g.Lx * floor(wx / g.Lx);
        if (g.Ly > 0.0) wy = wy - g.Ly * floor(wy / g.Ly);
        int cx, cy;
        cell_of(g, wx, wy, cx, cy);
        double bd = DBL_MAX;
        int bu = INT_MAX;
        auto take = [&](int q) {
            double d = dist2(qx, qy, xs[q], ys[q], g.Lx, g.Ly);
            int u = perm[q];
            if (d < bd || (d == bd && u < bu)) {
                bd = d;
                bu = u;
            }
        };
        for (int r = 0;; ++r) {
            bool wraps = (g.Lx > 0.0 && 2 * r + 1 > g.gx) || (g.Ly > 0.0 && 2 * r + 1 > g.gy);
            if (wraps) {
                bd = DBL_MAX;
                bu = INT_MAX;
                for (int q = 0; q < n; ++q) take(q);
                break;
            }
            for_ring(g, cstart, cend, cx, cy, r, take);
            double reach = r * cmin;
            if (bd < reach * reach) break;
            if (r > g.gx && r > g.gy) break;
        }
        owner[(int64_t)(k - 1) * n + p] = iperm[bu];
    }
}

// x^e for 0 <= e <= 4, without branches on e, so that a lane-dependent
// exponent costs no divergent code.
__device__ __forceinline__ double pow_upto4(double x, int e) {
    double p = 1.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) p = t < e ? p * x : p;
    return p;
}

__device__ __forceinline__ double cube_dist(double ax, double ay, double bx, double by) {
    double dx = ax - bx, dy = ay - by;
    double r = sqrt(dx * dx + dy * dy);
    return r * r * r;
}

// Departure point t of the right-hand-side list of owner s: node p and
// direction k. Own-node stencils: the eight departure points of s itself.
// Paper stencils: the points whose closest node is s (CSR list pts).
struct RhsList {
    const int32_t *ptr, *pts;   // null for own-node stencils
};

__device__ __forceinline__ void rhs_point(const RhsList &L, int s, int t, int &p, int &k) {
    if (!L.ptr) {
        p = s;
        k = t + 1;
    } else {
        const int e = L.pts[L.ptr[s] + t];
        p = e >> 3;
        k = (e & 7) + 1;
    }
}

// Largest 32-bit key over each group of 64/SYS lanes of a wavefront (all
// lanes active; SYS = 1 or 2), the same in every lane of the group: DPP
// exchanges inside each row of 16 lanes (swap neighbours, swap pairs, mirror
// the half-rows, mirror the row) leave the row's largest key in all its lanes;
// the rows of a group are then combined from scalar reads.
template <int SYS>
__device__ __forceinline__ uint32_t group_max_u32(uint32_t v, int half) {
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
    const uint32_t r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const uint32_t r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    if constexpr (SYS == 1)
        return max(max(r0, r1), max(r2, r3));
    else
        return half ? max(r2, r3) : max(r0, r1);
}

// Row stride (doubles) of the pivot-row buffers: NB + R + 1 values, padded
// so that the two buffers of a paired wavefront start at least four LDS
// banks apart and their same-index reads do not collide.
constexpr int row_stride(int NB, int R, int SYS) {
    int rs = NB + R + 1;
    if (SYS == 2)
        while ((2 * rs) % 64 < 8 || (2 * rs) % 64 > 56) ++rs;
    return rs;
}

// The double in lane l of a wavefront (l uniform), in scalar registers.
__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// 1/x to within about an ulp: the hardware estimate (about 2^-23 relative
// error for the magnitudes met here) refined by two Newton steps r += r(1 - xr),
// each of which squares the relative error. Zero gives NaN, which the
// singularity test catches where it matters (a zero pivot).
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return r;
}

// Orders the LDS accesses of one wavefront: LDS operations of a wavefront
// complete in issue order, so only the compiler has to be kept from moving
// accesses across this point.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wavefront solves the local systems of SYS owner nodes (SYS = 2 when a
// system has at most 32 unknowns: lanes 0-31 and 32-63 then hold one system
// each), Phi w = phi(p) (eqs. rbf_interp_set_augmented and shape_vector) of
// owner s for every departure point that uses the stencil of s, by
// Gauss-Jordan elimination with partial pivoting. Lane r of a system's group
// holds row r of the system (K RBF rows, M polynomial rows, then identity
// rows that pad the system to NB unknowns) in registers. Rows are never
// moved: the pivot of column k is a not-yet-used lane with the largest |a_k|,
// compared on the upper 32 bits of its binary64 encoding (exponent and 20
// mantissa bits, so within a factor 1 + 2^-20 of the largest, which keeps the
// growth bound of partial pivoting; ties: lowest lane). It copies its row and
// its reciprocal 1/a_k to its group's LDS buffer, and every other lane of the
// group, pivot rows of earlier steps included, subtracts its multiple of that
// row and keeps the multiplier in a_k. At the end the pivot row of step j
// holds a_j x_j = b, so unknown j (the weight of stencil member j, j < K) is
// one product with the kept reciprocal away, with no back substitution. The
// right-hand sides (departure points) are taken R at a time: the first group
// is eliminated along with the matrix, later groups by replaying the stored
// multipliers.
template <int NB, int R, int SYS, bool REPLAY>
__device__ __forceinline__ void rbf_solve(const Geo *__restrict__ geo,
                                          const double *__restrict__ xs,
                                          const double *__restrict__ ys,
                                          const int32_t *__restrict__ perm,
                                          const int32_t *__restrict__ nbr, RhsList L, int n,
                                          int K, int m, double dx, double *__restrict__ W64,
                                          int32_t *__restrict__ dev_err) {
    static_assert(SYS == 1 || (SYS == 2 && NB <= 32), "two systems need 32 lanes each");
    constexpr int LW = 64 / SYS;                   // lanes per system
    constexpr int KT = SYS == 2 ? 32 : kMaxK;      // table rows per system
    constexpr int MP = 15;   // monomials of degree <= 4 (table row stride, odd)
    constexpr int RS = row_stride(NB, R, SYS);
    __shared__ double s_row[4][SYS * RS];
    __shared__ double2 s_c[4][64];
    __shared__ double s_P[4][SYS * KT * MP];
    __shared__ double2 s_q[4][SYS * R];
    __shared__ int2 s_pk[4][SYS * R];
    const int lane = threadIdx.x & 63;
    const int half = SYS == 2 ? lane >> 5 : 0;     // this lane's system
    const int ll = lane & (LW - 1);                // row within it
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // each XCD takes a contiguous range of owners: the shape vectors they
    // store land at neighbouring nodes, so the L2 of one XCD collects whole
    // lines of them (grid xcd_grid of the workgroup count)
    const int64_t blk = xcd_tile(((int64_t)n + 4 * SYS - 1) / (4 * SYS));
    const int64_t s0 = (blk * 4 + wv) * SYS;
    if (s0 >= n) return;   // uniform across the wavefront
    // a group past the last node solves its neighbour's system again and
    // stores nothing
    const bool live = s0 + half < n;
    const int s = (int)(live ? s0 + half : s0);
    // (without REPLAY every owner has at most R departure points)
    const int count = live ? (L.ptr ? L.ptr[s + 1] - L.ptr[s] : 8) : 0;
    int cmax = __builtin_amdgcn_readlane(count, 0);
    if constexpr (SYS == 2) cmax = max(cmax, __builtin_amdgcn_readlane(count, 32));
    if (cmax == 0) return;
    const Geo g = *geo;
    const int M = (m + 1) * (m + 2) / 2;
    const int nn = K + M;
    double *row = s_row[wv] + half * RS;
    double *P = s_P[wv] + half * KT * MP;
    const double2 *cw = s_c[wv] + half * LW;
    double2 *qw = s_q[wv] + half * R;
    int2 *pkw = s_pk[wv] + half * R;

    // stencil member coordinates relative to the centre s, scaled by the
    // stencil radius (the interpolant is invariant to this; it helps the
    // conditioning)
    double rx = 0.0, ry = 0.0;
    if (ll < K) {
        int q = nbr[(int64_t)ll * n + s];
        rx = min_image(xs[q] - xs[s], g.Lx);
        ry = min_image(ys[q] - ys[s], g.Ly);
    }
    double rad = sqrt(rx * rx + ry * ry);
#pragma unroll
    for (int off = LW / 2; off > 0; off >>= 1) rad = fmax(rad, __shfl_xor(rad, off));
    if (!(rad > 0.0)) rad = 1.0;
    const double sx = rx / rad, sy = ry / rad;
    s_c[wv][lane] = make_double2(sx, sy);
    // monomials of each member (eq. poly_sets, graded order 1, x, y, x^2, xy,
    // y^2, x^3, ..., y^4: monomial q of degree d at offset j is x^(d-j) y^j),
    // row `ll` of the table
    if (ll < K) {
        double xp[5], yp[5];
        xp[0] = yp[0] = 1.0;
#pragma unroll
        for (int e = 1; e < 5; ++e) {
            xp[e] = xp[e - 1] * sx;
            yp[e] = yp[e - 1] * sy;
        }
        int q = 0;
#pragma unroll
        for (int d = 0; d <= 4; ++d)
#pragma unroll
            for (int j = 0; j <= d; ++j) P[ll * MP + q++] = xp[d - j] * yp[j];
    }
    wave_lds_sync();
    const bool rbf_row = ll < K;
    const bool poly_row = ll >= K && ll < nn;
    const int qrow = ll - K;
    // table entries this lane reads: polynomial q of every member (polynomial
    // rows), every polynomial of its own member (RBF rows)
    const int pcol = poly_row ? qrow : 0;
    const int prow = (rbf_row ? ll : 0) * MP - K;

    // row `ll` of the padded system; the branches on the column are uniform
    double a[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        if (c < K) {
            const double2 cc = cw[c];
            const double r3 = cube_dist(sx, sy, cc.x, cc.y);
            const double pc = P[c * MP + pcol];
            a[c] = rbf_row ? r3 : (poly_row ? pc : 0.0);
        } else if (c < nn) {
            const double pr = P[prow + c];
            a[c] = rbf_row ? pr : 0.0;
        } else {
            a[c] = c == ll ? 1.0 : 0.0;
        }
    }
    // infinity norm for the singularity threshold
    double rs = 0.0;
#pragma unroll
    for (int c = 0; c < NB; ++c) rs += fabs(a[c]);
    if (ll >= NB) rs = 0.0;
#pragma unroll
    for (int off = LW / 2; off > 0; off >>= 1) rs = fmax(rs, __shfl_xor(rs, off));
    const double tiny = 1e3 * DBL_EPSILON * rs;
    bool singular = false;
    // elimination step at which this lane was the pivot (-1: padding lane)
    // and the reciprocal of its pivot value
    int pstep = ll < NB ? NB : -1;
    double pinv = 1.0;

    // right-hand sides c0 .. c0+R-1 (row `ll` of each). Lane t < R of each
    // group first locates departure point c0 + t (node p, direction k) and its
    // position x_p - e_k dx relative to s, scaled, for the whole group.
    const double irad = 1.0 / rad;
    // exponents of monomial qrow (degree qd, offset qey within it)
    const int qd = (qrow >= 1) + (qrow >= 3) + (qrow >= 6) + (qrow >= 10);
    const int qey = poly_row ? qrow - qd * (qd + 1) / 2 : 0;
    const int qex = poly_row ? qd - qey : 0;
    auto load_rhs = [&](int c0, double(&b)[R]) {
        if (ll < R) {
            double qx = 0.0, qy = 0.0;
            int p = 0, k = 1;
            if (c0 + ll < count) {
                rhs_point(L, s, c0 + ll, p, k);
                qx = (L.ptr ? min_image(xs[p] - lat_ex(k) * dx - xs[s], g.Lx)
                            : -lat_ex(k) * dx) * irad;
                qy = (L.ptr ? min_image(ys[p] - lat_ey(k) * dx - ys[s], g.Ly)
                            : -lat_ey(k) * dx) * irad;
            }
            qw[ll] = make_double2(qx, qy);
            pkw[ll] = make_int2(p, k);
        }
        wave_lds_sync();
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const double2 q = qw[t];
            const double r3 = cube_dist(sx, sy, q.x, q.y);
            const double pq = pow_upto4(q.x, qex) * pow_upto4(q.y, qey);
            b[t] = c0 + t < count ? (rbf_row ? r3 : (poly_row ? pq : 0.0)) : 0.0;
        }
    };
    // the pivot row of step j < K holds a_j x_j = b: x_j is the weight of
    // stencil member j for each departure point
    auto store = [&](int c0, const double(&b)[R]) {
        if (pstep >= 0 && pstep < K) {
#pragma unroll
            for (int t = 0; t < R; ++t) {
                if (c0 + t < count) {
                    const int2 pk = pkw[t];
                    W64[w64_at(pk.y, pstep, n, pk.x)] = b[t] * pinv;
                }
            }
        }
    };

    double b[R];
    load_rhs(0, b);
    if constexpr (SYS == 1) {
        // One system per wavefront: the pivot row is broadcast through scalar
        // registers (two lane reads per value, used directly as the scalar
        // operand of the updates) instead of LDS, which the four SIMDs of a
        // compute unit share and which every lane would otherwise read the
        // whole row from. Lane k keeps the pivot lane of step k for the
        // replay of further groups.
        // Steps from nn on pivot on the identity rows that pad the system
        // and change nothing, and columns from nn on stay zero in every row
        // that holds a pivot before (a zero pivot there only happens in a
        // singular system, which is reported): both are skipped with uniform
        // branches.
        int plog = 0;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            if (k >= nn) continue;
            const uint32_t key =
                pstep > k ? ((uint32_t)(__double_as_longlong(a[k]) >> 32) & 0x7FFFFFFFu) | 1u : 0u;
            const double rk = recip(a[k]);
            const uint32_t km = group_max_u32<1>(key, 0);
            const int pl = __builtin_amdgcn_readfirstlane(__builtin_ctzll(__ballot(key == km)));
            const double pv = readlane_d(a[k], pl), pi = readlane_d(rk, pl);
            if (!(fabs(pv) > tiny)) singular = true;
            if (lane == pl) {
                pstep = k;
                pinv = pi;
            }
            if (lane == k) plog = pl;
            const double l = lane != pl ? a[k] * pi : 0.0;
            // (four lane reads ahead of their updates, so that the scalar
            // results are not waited for one by one)
#pragma unroll
            for (int c = k + 1; c < NB; c += 4) {
                if (c >= nn) continue;
                const double r0 = readlane_d(a[c], pl);
                const double r1 = c + 1 < NB ? readlane_d(a[c + 1], pl) : 0.0;
                const double r2 = c + 2 < NB ? readlane_d(a[c + 2], pl) : 0.0;
                const double r3 = c + 3 < NB ? readlane_d(a[c + 3], pl) : 0.0;
                a[c] = __builtin_fma(-l, r0, a[c]);
                if (c + 1 < NB) a[c + 1] = __builtin_fma(-l, r1, a[c + 1]);
                if (c + 2 < NB) a[c + 2] = __builtin_fma(-l, r2, a[c + 2]);
                if (c + 3 < NB) a[c + 3] = __builtin_fma(-l, r3, a[c + 3]);
            }
#pragma unroll
            for (int t = 0; t < R; t += 2) {
                const double r0 = readlane_d(b[t], pl), r1 = readlane_d(b[t + 1], pl);
                b[t] = __builtin_fma(-l, r0, b[t]);
                b[t + 1] = __builtin_fma(-l, r1, b[t + 1]);
            }
            if (lane != pl) a[k] = l;
        }
        store(0, b);
        for (int c0 = R; REPLAY && c0 < cmax; c0 += R) {
            load_rhs(c0, b);
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if (k >= nn) continue;
                const int pk = __builtin_amdgcn_readlane(plog, k);
                const double l = lane != pk ? a[k] : 0.0;
#pragma unroll
                for (int t = 0; t < R; ++t) b[t] = __builtin_fma(-l, readlane_d(b[t], pk), b[t]);
            }
            store(c0, b);
        }
        if (singular && count > 0 && ll == 0) atomicMin(dev_err, perm[s] + 1);
        return;
    }
    // elimination, carrying the first group of right-hand sides (padding
    // steps and columns skipped as above)
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        if (k >= nn) continue;
        const uint32_t key =
            pstep > k ? ((uint32_t)(__double_as_longlong(a[k]) >> 32) & 0x7FFFFFFFu) | 1u : 0u;
        const double rk = recip(a[k]);
        const uint32_t km = group_max_u32<SYS>(key, half);
        // every group has an open lane (NB - k of them), so its mask is not empty
        const uint64_t hit = __ballot(key == km);
        int pl;
        if constexpr (SYS == 1) {
            pl = __builtin_amdgcn_readfirstlane(__builtin_ctzll(hit));
        } else {
            const int pa = __builtin_amdgcn_readfirstlane(__builtin_ctz((uint32_t)hit));
            const int pb = __builtin_amdgcn_readfirstlane(32 + __builtin_ctz((uint32_t)(hit >> 32)));
            pl = half ? pb : pa;
        }
        if (lane == pl) {
#pragma unroll
            for (int c = k; c < NB; ++c) row[c] = a[c];
#pragma unroll
            for (int t = 0; t < R; ++t) row[NB + t] = b[t];
            row[NB + R] = rk;
            pstep = k;
            pinv = rk;
        }
        wave_lds_sync();
        if (!(fabs(row[k]) > tiny)) singular = true;
        const double l = lane != pl ? a[k] * row[NB + R] : 0.0;
        // (the LDS reads are issued 16 at a time, which bounds the registers
        // they hold; the updates are explicit fused multiply-adds, since only
        // the distances that decide stencil ties must round like the oracle)
#pragma unroll
        for (int c0 = k + 1; c0 < NB; c0 += 4) {
            if (c0 >= nn) continue;
#pragma unroll
            for (int c = c0; c < c0 + 4 && c < NB; ++c) a[c] = __builtin_fma(-l, row[c], a[c]);
            if ((c0 - k + 3) % 16 == 0) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int t = 0; t < R; ++t) b[t] = __builtin_fma(-l, row[NB + t], b[t]);
        if (lane != pl) a[k] = l;
        wave_lds_sync();
    }
    store(0, b);
    // further groups: replay the stored multipliers
    for (int c0 = R; REPLAY && c0 < cmax; c0 += R) {
        load_rhs(c0, b);
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            if (k >= nn) continue;
            if (pstep == k) {
#pragma unroll
                for (int t = 0; t < R; ++t) row[NB + t] = b[t];
            }
            wave_lds_sync();
            if (pstep != k) {
#pragma unroll
                for (int t = 0; t < R; ++t) b[t] = __builtin_fma(-a[k], row[NB + t], b[t]);
            }
            wave_lds_sync();
        }
        store(c0, b);
    }
    // a system whose weights no departure point uses (count 0, or a group
    // past the last node) reports nothing, as if it had not been solved
    if (singular && count > 0 && ll == 0) atomicMin(dev_err, perm[s] + 1);
}

// Occupancy against registers: 24 and 32 unknowns fit four wavefronts per
// SIMD, 48 three, 64 two (with the replay, nothing spills except at 48
// without it; a small spill costs less than the latency fewer wavefronts leave
// exposed). Up to 32 unknowns a wavefront holds two systems.
template <int NB, int R, int WPE, int SYS, bool REPLAY>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_rbf(
    const Geo *__restrict__ geo, const double *__restrict__ xs, const double *__restrict__ ys,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ nbr, RhsList L, int n, int K,
    int m, double dx, double *__restrict__ W64, int32_t *__restrict__ dev_err) {
    rbf_solve<NB, R, SYS, REPLAY>(geo, xs, ys, perm, nbr, L, n, K, m, dx, W64, dev_err);
}

// ---- the same solve with the FP64 matrix cores ------------------------------
// The systems and the elimination of rbf_solve (Gauss-Jordan, partial
// pivoting on the upper 32 bits of |a_k|, ties to the lowest row, rows never
// moved, pivot rows left unscaled), taken four pivot columns at a time so that
// the bulk of the arithmetic runs on v_mfma_f64_16x16x4:
//  - the augmented matrix [Phi | b_0 .. b_15] (NB = 16 RT unknowns, up to 16
//    departure points) lives in the registers of one wavefront as RT x (RT+1)
//    tiles of 16 x 16 in the result layout of that instruction (register i of
//    lane l holds row l / 16 + 4 i, column l % 16 of its tile);
//  - a panel of four columns is copied to LDS and eliminated with one row per
//    lane, pivot search and row reads as in rbf_solve but on four columns. Its
//    four steps E_j = I - l_j e_{p_j}^T (l_j the multipliers, zero at the pivot
//    row p_j) multiply to I - Lt S^T, S^T selecting the pivot rows; the new
//    column of Lt is the step's multipliers and the earlier ones are reduced
//    by the step like matrix columns;
//  - every column right of the panel, right-hand sides included, then takes
//    the rank-4 product -Lt U, U the four pivot rows as they stood before the
//    panel: RT x (tiles right of the panel) matrix-core products, with Lt in
//    the A layout (lane 16 k + r holds row r, column k) and U in the B layout
//    (lane 16 k + c holds row k, column c).
// The pivot row of step j ends as d_j e_j on the matrix part, so unknown j is
// its right-hand-side entry times 1/d_j. Owners with more than 16 departure
// points solve again for each further group of 16. Each lane assembles its own
// tile entries (monomials from a per-member table in LDS).
// The FP64 matrix-core rate of gfx950 equals its FP64 vector rate: what the
// products save is issue slots (108 products a system at 48 unknowns against
// about 2,700 vector FMAs). The pivot steps (reduction, lane reads) stay
// serial and dominate what remains.
typedef double dbl4 __attribute__((ext_vector_type(4)));

// v from the lane CTRL names (a DPP row pattern), both halves of a double
template <int CTRL> __device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Three wavefronts per SIMD at 48 unknowns (167 VGPRs, a 20-byte spill);
// without the hint the compiler keeps the tiles in 460 registers and runs one.
template <int RT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(RT == 3 ? 3 : 2))) void k_rbf_mfma(
    const Geo *__restrict__ geo, const double *__restrict__ xs, const double *__restrict__ ys,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ nbr, RhsList L, int n, int K,
    int m, double dx, double *__restrict__ W64, int32_t *__restrict__ dev_err) {
    constexpr int NB = 16 * RT, CT = RT + 1, NC = 16 * CT;
    __shared__ double2 s_c[64];          // scaled stencil members
    __shared__ double2 s_q[16];          // scaled departure points of the group
    __shared__ int2 s_pk[16];            // their (node, direction)
    __shared__ double s_pan[4][NB + 4];  // panel columns (rows padded: see below)
    __shared__ double s_L[4][NB];        // Lt, column-major
    // the row groups that hold the pivot rows; element e of column c sits at
    // e ^ ((c >> 2) & 3), so that the sixteen lanes of a row group, which
    // read one element of sixteen consecutive columns, hit distinct banks
    // (unswizzled they read 32 bytes apart, four to a bank); the panel rows
    // are padded for the same reason. Both measured 4.7 % off the solve.
    __shared__ double s_U[4][NC][4];
    __shared__ int s_step[NB];
    __shared__ double s_pinv[NB];
    constexpr int PQ = NB * 15;          // the departure points' monomials follow the members'
    static_assert(PQ + 16 * 15 <= 4 * NC * 4, "the monomial tables fit in s_U");
    const int lane = threadIdx.x;
    // owners in XCD-contiguous ranges, as in k_rbf (grid xcd_grid(n))
    const int64_t so = xcd_tile(n);
    if (so >= n) return;
    const int s = (int)so;
    const int count = L.ptr ? L.ptr[s + 1] - L.ptr[s] : 8;
    if (count == 0) return;
    const Geo g = *geo;
    const int M = (m + 1) * (m + 2) / 2;
    const int nn = K + M;

    double rx = 0.0, ry = 0.0;
    if (lane < K) {
        const int q = nbr[(int64_t)lane * n + s];
        rx = min_image(xs[q] - xs[s], g.Lx);
        ry = min_image(ys[q] - ys[s], g.Ly);
    }
    double rad = sqrt(rx * rx + ry * ry);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) rad = fmax(rad, __shfl_xor(rad, off));
    if (!(rad > 0.0)) rad = 1.0;
    const double sx = rx / rad, sy = ry / rad, irad = 1.0 / rad;
    s_c[lane] = make_double2(sx, sy);
    bool singular = false;

    for (int c0 = 0; c0 < count; c0 += 16) {
        const int cnt = min(16, count - c0);
        if (lane < 16) {
            double qx = 0.0, qy = 0.0;
            int p = 0, k = 1;
            if (lane < cnt) {
                rhs_point(L, s, c0 + lane, p, k);
                qx = (L.ptr ? min_image(xs[p] - lat_ex(k) * dx - xs[s], g.Lx) : -lat_ex(k) * dx) *
                     irad;
                qy = (L.ptr ? min_image(ys[p] - lat_ey(k) * dx - ys[s], g.Ly) : -lat_ey(k) * dx) *
                     irad;
            }
            s_q[lane] = make_double2(qx, qy);
            s_pk[lane] = make_int2(p, k);
        }
        wave_lds_sync();

        // monomials of the stencil members (lanes below K) and of the group's
        // departure points (lanes 48 + t), row stride 15, in the space that
        // the elimination uses for U; powers first, then each product
        double *tab = &s_U[0][0][0];
        // the lane index again, opaque to the compiler: what depends on it is
        // recomputed for each group rather than kept live from the first
        int lid = lane;
        __asm__ volatile("" : "+v"(lid));
        const int g4 = lid >> 4, cl = lid & 15;
        {
            const int t = lid - 48;
            const bool mem = lid < K, dep = t >= 0 && t < cnt;
            double px = sx, py = sy;
            if (dep) {
                const double2 q = s_q[t];
                px = q.x;
                py = q.y;
            }
            double xp[5], yp[5];
            xp[0] = yp[0] = 1.0;
#pragma unroll
            for (int e = 1; e < 5; ++e) {
                xp[e] = xp[e - 1] * px;
                yp[e] = yp[e - 1] * py;
            }
            double *row = tab + (mem ? lid * 15 : PQ + (dep ? t : 0) * 15);
            if (mem || dep) {
#pragma unroll
                for (int d = 0, q = 0; d <= 4; ++d)
#pragma unroll
                    for (int ey = 0; ey <= d; ++ey, ++q)
                        if (q < M) row[q] = xp[d - ey] * yp[ey];
            }
        }
        wave_lds_sync();

        // assembly: every lane computes its own entries of the tiles; the
        // branches on a tile's place against K are uniform
        dbl4 T[RT][CT];
        double rsum[RT][4];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * rt + g4 + 4 * i;
                const double2 xr = s_c[r];
                const bool rr = r < K, pr = r >= K && r < nn;
                double acc = 0.0;
#pragma unroll
                for (int ct = 0; ct < RT; ++ct) {
                    const int c = 16 * ct + cl;
                    const bool rc = c < K, pc = c >= K && c < nn;
                    double r3 = 0.0;
                    if (16 * rt < K && 16 * ct < K) {
                        const double2 xc = s_c[c];
                        r3 = cube_dist(xr.x, xr.y, xc.x, xc.y);
                    }
                    const int ti = rr && pc ? r * 15 + (c - K) : pr && rc ? c * 15 + (r - K) : 0;
                    const double tv = tab[ti];
                    const double a = rr ? (rc ? r3 : (pc ? tv : 0.0))
                                        : pr ? (rc ? tv : 0.0) : (r == c ? 1.0 : 0.0);
                    T[rt][ct][i] = a;
                    acc += fabs(a);
                }
                rsum[rt][i] = acc;
                {
                    const int t = cl;
                    double r3 = 0.0;
                    if (16 * rt < K) {
                        const double2 q = s_q[t];
                        r3 = cube_dist(xr.x, xr.y, q.x, q.y);
                    }
                    const double tv = tab[pr ? PQ + t * 15 + (r - K) : 0];
                    T[rt][RT][i] = t < cnt ? (rr ? r3 : (pr ? tv : 0.0)) : 0.0;
                }
                // one row at a time: keeps the compiler from hoisting every
                // row's table reads (and their registers) to the start
                __asm__ volatile("" ::: "memory");
            }
        // infinity norm of the matrix: row sums over the sixteen lanes that
        // share a row group, then the largest row
        double rs = 0.0;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                double v = rsum[rt][i];
                v += dpp_d<0x128>(v);
                v += dpp_d<0x124>(v);
                v += dpp_d<0x122>(v);
                v += dpp_d<0x121>(v);
                rs = fmax(rs, v);
            }
        rs = fmax(fmax(readlane_d(rs, 0), readlane_d(rs, 16)),
                  fmax(readlane_d(rs, 32), readlane_d(rs, 48)));
        const double tiny = 1e3 * DBL_EPSILON * rs;
        wave_lds_sync();   // the table's space is U's from here on

        int pstep = lane < NB ? NB : -1;
        double pinv = 1.0;
        // panels: the column tile of the panel is unrolled (register tiles
        // take compile-time indices), the four panels inside it are not; the
        // products cover the panel's own tile too (for its last panel only
        // finished columns change there)
#pragma unroll
        for (int ctp = 0; ctp < RT; ++ctp) {
#pragma unroll 1
            for (int cp0 = 0; cp0 < 16; cp0 += 4) {
                const int k0 = 16 * ctp + cp0;
                if (k0 >= nn) break;                  // uniform
                if (cl >= cp0 && cl < cp0 + 4) {
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            s_pan[cl - cp0][16 * rt + g4 + 4 * i] = T[rt][ctp][i];
                }
                wave_lds_sync();
                double pv[4] = {0.0, 0.0, 0.0, 0.0}, Lt[4] = {0.0, 0.0, 0.0, 0.0};
                if (lane < NB) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) pv[j] = s_pan[j][lane];
                }
                int plist[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = k0 + j;
                    plist[j] = -1;
                    if (k >= nn) continue;            // uniform
                    const uint32_t key =
                        pstep > k
                            ? ((uint32_t)(__double_as_longlong(pv[j]) >> 32) & 0x7FFFFFFFu) | 1u
                            : 0u;
                    const double rk = recip(pv[j]);
                    const uint32_t km = group_max_u32<1>(key, 0);
                    const int pl =
                        __builtin_amdgcn_readfirstlane(__builtin_ctzll(__ballot(key == km)));
                    const double pvv = readlane_d(pv[j], pl), pi = readlane_d(rk, pl);
                    if (!(fabs(pvv) > tiny)) singular = true;
                    if (lane == pl) {
                        pstep = k;
                        pinv = pi;
                    }
                    const double l = lane != pl ? pv[j] * pi : 0.0;
#pragma unroll
                    for (int jj = j + 1; jj < 4; ++jj)
                        pv[jj] = __builtin_fma(-l, readlane_d(pv[jj], pl), pv[jj]);
#pragma unroll
                    for (int jj = 0; jj < j; ++jj)
                        Lt[jj] = __builtin_fma(-l, readlane_d(Lt[jj], pl), Lt[jj]);
                    Lt[j] = l;
                    plist[j] = pl;
                }
                if (lane < NB) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) s_L[j][lane] = Lt[j];
                }
                // U: the row group of each pivot row writes its four rows of
                // every tile from the panel's on; a step past nn gives a zero row
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int p = plist[j];
                    if (p < 0) {
                        if (g4 == 0) {
#pragma unroll
                            for (int ct = ctp; ct < CT; ++ct)
                                *reinterpret_cast<dbl4 *>(&s_U[j][16 * ct + cl][0]) =
                                    dbl4{0.0, 0.0, 0.0, 0.0};
                        }
                        continue;
                    }
                    const int rtp = p >> 4, gp = p & 3;
                    // one branch per row tile (uniform); the empty asm keeps
                    // the compiler from merging the stores into one store of
                    // a value selected across every tile
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt) {
                        if (rt == rtp) {
                            __asm__ volatile("" ::: "memory");
                            if (g4 == gp) {
#pragma unroll
                                for (int ct = ctp; ct < CT; ++ct)
#pragma unroll
                                    for (int e = 0; e < 4; ++e)
                                        s_U[j][16 * ct + cl][e ^ ((cl >> 2) & 3)] = T[rt][ct][e];
                            }
                        }
                    }
                }
                wave_lds_sync();
                const int pk =
                    g4 == 0 ? plist[0] : g4 == 1 ? plist[1] : g4 == 2 ? plist[2] : plist[3];
                const int ik = pk < 0 ? 0 : ((pk & 15) >> 2);
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    const double a = -s_L[g4][16 * rt + cl];
#pragma unroll
                    for (int ct = ctp; ct < CT; ++ct) {
                        const double b = s_U[g4][16 * ct + cl][ik ^ ((cl >> 2) & 3)];
                        T[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, T[rt][ct], 0, 0, 0);
                    }
                }
                wave_lds_sync();
            }
        }
        if (lane < NB) {
            s_step[lane] = pstep;
            s_pinv[lane] = pinv;
        }
        wave_lds_sync();
        if (cl < cnt) {
            const int2 pk = s_pk[cl];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 16 * rt + g4 + 4 * i;
                    const int j = s_step[r];
                    if (j < K) W64[w64_at(pk.y, j, n, pk.x)] = T[rt][RT][i] * s_pinv[r];
                }
        }
        wave_lds_sync();
    }
    if (singular && lane == 0) atomicMin(dev_err, perm[s] + 1);
}

// Owner -> departure-point lists of the paper's stencil rule (CSR): count,
// then fill (the order inside a list does not affect the solved weights).
__global__ void k_owned_count(int n, const int32_t *__restrict__ owner, int32_t *__restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)8 * n) return;
    atomicAdd(&cnt[owner[i]], 1);
}

__global__ void k_owned_fill(int n, const int32_t *__restrict__ owner,
                             const int32_t *__restrict__ ptr, int32_t *__restrict__ cur,
                             int32_t *__restrict__ pts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)8 * n) return;
    const int k0 = (int)(i / n), p = (int)(i - (int64_t)k0 * n);   // owner is [8][n]
    const int s = owner[i];
    pts[ptr[s] + atomicAdd(&cur[s], 1)] = p * 8 + k0;
}

__global__ void k_set_last(int32_t *ptr, int n, int32_t v) { ptr[n] = v; }

// FP32 copy of the shape vectors in the streaming layout [K][2][n][4]
// (directions 1..4 and 5..8 as float4). After rounding, the weights of each
// (node, direction) no longer sum to one; the defect 1 - sum (evaluated in
// FP64) is added to one weight, the smallest in magnitude among those at least
// 64 times larger than the defect, so the rounded weights keep the partition
// of unity that the deviation-stored populations rely on. One thread per
// (node, direction), numbered like the FP32 layout: four consecutive lanes
// fill one node's float4, so a wavefront stores whole lines of each member
// plane (numbered like the FP64 layout instead, two far-apart workgroups each
// wrote half of every float4, and the partly written lines doubled the
// writes). Its loads are two 256-byte runs per wavefront and member, one in
// each direction pair's plane of the FP64 layout. The weights stay in
// registers between the three passes.
template <int KB>
__global__ __launch_bounds__(256) void k_pack_w32(const double *__restrict__ W64, int n, int K,
                                                  float *__restrict__ W32) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)8 * n) return;
    const int64_t plane = (int64_t)8 * n;   // distance between members j and j+1
    const int c = (int)(t & 3);              // direction within the half
    const int64_t hp = t >> 2;
    const int hh = (int)(hp / n);            // half: directions 1-4 or 5-8
    const int p = (int)(hp - (int64_t)hh * n);
    const int k = 4 * hh + c + 1;
    const int64_t src = w64_at(k, 0, n, p);
    double w[KB];
    double sum = 0.0;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        w[j] = j < K ? W64[j * plane + src] : 0.0;
        sum += (double)(float)w[j];
    }
    const double defect = 1.0 - sum;
    int jstar = -1;
    double best = DBL_MAX;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        const double a = fabs(w[j]);
        if (j < K && a >= 64.0 * fabs(defect) && a < best) {
            best = a;
            jstar = j;
        }
    }
    float *out = W32 + ((int64_t)hh * n + p) * 4 + c;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        if (j < K) {
            float f = (float)w[j];
            if (j == jstar) f = (float)((double)f + defect);
            out[(int64_t)j * 8 * n] = f;
        }
    }
}

// Constant azimuthal acceleration about the origin (Sec. 3): a = g (-y, x)/r at
// fluid nodes, zero at wall nodes.
__global__ void k_force(const double *__restrict__ xs, const double *__restrict__ ys,
                        const uint8_t *__restrict__ nt, int n, double mag, float *f32,
                        double *f64) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double x = xs[p], y = ys[p];
    double r = sqrt(x * x + y * y);
    double ax = 0.0, ay = 0.0;
    if (!(nt && nt[p]) && r > 0.0) {
        ax = -mag * y / r;
        ay = mag * x / r;
    }
    if (f32) {
        f32[p] = (float)ax;
        f32[n + p] = (float)ay;
    }
    if (f64) {
        f64[p] = ax;
        f64[n + p] = ay;
    }
}

// Bounce-back link masks (Sec. 3): at wall node p (internal order), bit k-1
// is set when e_k . n < 0 for the outward normal n of the fluid domain, i.e.
// population k enters the fluid from outside the wall.
__global__ void k_links(const uint8_t *__restrict__ ntype, const int32_t *__restrict__ perm,
                        const double *__restrict__ nx, const double *__restrict__ ny, int n,
                        uint8_t *__restrict__ links) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    unsigned m = 0;
    if (ntype[p]) {
        const int u = perm[p];
        const double a = nx[u], b = ny[u];
        for (int k = 1; k < kQ; ++k)
            if (lat_ex(k) * a + lat_ey(k) * b < 0.0) m |= 1u << (k - 1);
    }
    links[p] = (uint8_t)m;
}

}  // namespace

hipError_t launch_links(const uint8_t *ntype, const int32_t *perm, const double *nx,
                        const double *ny, int n, uint8_t *links, hipStream_t s) {
    hipLaunchKernelGGL(k_links, dim3(blocks_for(n, 256)), dim3(256), 0, s, ntype, perm, nx, ny,
                       n, links);
    return hipGetLastError();
}

hipError_t launch_geo_periodic(Geo *geo, double Lx, double Ly, int gx, int gy, int hb,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_geo_periodic, dim3(1), dim3(1), 0, s, geo, Lx, Ly, gx, gy, hb);
    return hipGetLastError();
}

hipError_t launch_geo_bbox(Geo *geo, const double *x, const double *y, int n, int gx, int gy,
                           int hb, hipStream_t s) {
    hipLaunchKernelGGL(k_geo_bbox, dim3(1), dim3(1024), 0, s, geo, x, y, n, gx, gy, hb);
    return hipGetLastError();
}

hipError_t launch_keys(const Geo *geo, const double *x, const double *y, int n,
                       uint32_t *keys, int32_t *vals, hipStream_t s) {
    hipLaunchKernelGGL(k_keys, dim3(blocks_for(n, 256)), dim3(256), 0, s, geo, x, y, n, keys,
                       vals);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_scatter_sorted(const Geo *geo, const double *x, const double *y,
                                 const uint8_t *nt, const int32_t *perm,
                                 const uint32_t *skeys, int n, double *xs, double *ys,
                                 uint8_t *ntype, int32_t *iperm, int32_t *cstart,
                                 int32_t *cend, int ncells, hipStream_t s) {
    hipError_t e = launch_fill_i32(cstart, 0, ncells, s);
    if (e != hipSuccess) return e;
    e = launch_fill_i32(cend, 0, ncells, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter_sorted, dim3(blocks_for(n, 256)), dim3(256), 0, s, geo, x, y,
                       nt, perm, skeys, n, xs, ys, ntype, iperm, cstart, cend);
    return hipGetLastError();
}

hipError_t launch_knn(const Geo *geo, const double *xs, const double *ys,
                      const int32_t *perm, const int32_t *iperm, const int32_t *cstart,
                      const int32_t *cend, int n, int K, int32_t *nbr, hipStream_t s) {
    dim3 grid(blocks_for(n, 256)), block(256);
    if (K - 1 <= 16)
        hipLaunchKernelGGL(k_knn<16>, grid, block, 0, s, geo, xs, ys, perm, iperm, cstart, cend, n, K, nbr);
    else if (K - 1 <= 24)   // (the list's cost per candidate grows with its length)
        hipLaunchKernelGGL(k_knn<24>, grid, block, 0, s, geo, xs, ys, perm, iperm, cstart, cend, n, K, nbr);
    else if (K - 1 <= 32)
        hipLaunchKernelGGL(k_knn<32>, grid, block, 0, s, geo, xs, ys, perm, iperm, cstart, cend, n, K, nbr);
    else
        hipLaunchKernelGGL(k_knn<48>, grid, block, 0, s, geo, xs, ys, perm, iperm, cstart, cend, n, K, nbr);
    return hipGetLastError();
}

hipError_t launch_owner(const Geo *geo, const double *xs, const double *ys,
                        const int32_t *perm, const int32_t *iperm, const int32_t *cstart,
                        const int32_t *cend, int n, double dx, int32_t *owner,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_owner, dim3(blocks_for(n, 256)), dim3(256), 0, s, geo, xs, ys, perm,
                       iperm, cstart, cend, n, dx, owner);
    return hipGetLastError();
}

template <int NB>
static hipError_t launch_rbf_nb(const Geo *geo, const double *xs, const double *ys,
                                const int32_t *perm, const int32_t *nbr, RhsList L, int n, int K,
                                int m, double dx, double *W64, int32_t *dev_err, hipStream_t s) {
    // 48 unknowns: the matrix-core solver (measured 10 % faster on the
    // 262,144-node lattice, K 30, degree 4); at 64 unknowns the register
    // tiles leave two wavefronts per SIMD and the row-per-lane solver is faster
    if constexpr (NB == 48) {
        hipLaunchKernelGGL((k_rbf_mfma<NB / 16>), dim3(xcd_grid(n)), dim3(64), 0, s, geo, xs, ys,
                           perm, nbr, L, n, K, m, dx, W64, dev_err);
        return hipGetLastError();
    }
    constexpr int wpe = NB <= 32 ? 4 : NB == 64 ? 2 : 3;
    constexpr int sys = NB <= 32 ? 2 : 1;   // systems per wavefront
    dim3 grid(xcd_grid(blocks_for(n, 4 * sys))), block(256);
    // own-node stencils (exactly 8 departure points per owner) take the
    // kernel without the replay, which need not keep the multipliers (the
    // register allocator would park them in scratch memory). Splitting the
    // paper rule's owners the same way (at most 8 departure points, then the
    // rest) measured slower: the second launch runs a sparse tail.
    if (L.ptr)
        hipLaunchKernelGGL((k_rbf<NB, 8, wpe, sys, true>), grid, block, 0, s, geo, xs, ys, perm,
                           nbr, L, n, K, m, dx, W64, dev_err);
    else   // fewer registers live: one more wavefront per SIMD at 64 unknowns (at 24
           // and 32 four is the most the registers allow either way)
        hipLaunchKernelGGL((k_rbf<NB, 8, NB <= 32 ? 4 : wpe + 1, sys, false>), grid, block, 0, s,
                           geo, xs, ys, perm, nbr, L, n, K, m, dx, W64, dev_err);
    return hipGetLastError();
}

size_t rbf_temp_bytes(int n) {
    const size_t a = ((size_t)n * 4 + 255) & ~size_t(255);
    const size_t b = (((size_t)n + 1) * 4 + 255) & ~size_t(255);
    const size_t c = ((size_t)8 * n * 4 + 255) & ~size_t(255);
    return a + b + c + scan_temp_bytes(n) + 256;
}

hipError_t launch_rbf(const Geo *geo, const double *xs, const double *ys,
                      const int32_t *perm, const int32_t *nbr, const int32_t *owner,
                      int n, int K, int m, double dx, int mode, void *tmp, size_t tmp_bytes,
                      double *W64, int32_t *dev_err, hipStream_t s) {
    RhsList L{nullptr, nullptr};
    hipError_t e;
    if (mode == MLBM_STENCIL_PAPER) {
        char *b = (char *)tmp;
        int32_t *cnt = (int32_t *)b;
        b += ((size_t)n * 4 + 255) & ~size_t(255);
        int32_t *ptr = (int32_t *)b;
        b += (((size_t)n + 1) * 4 + 255) & ~size_t(255);
        int32_t *pts = (int32_t *)b;
        b += ((size_t)8 * n * 4 + 255) & ~size_t(255);
        const size_t scan_bytes = tmp_bytes - (size_t)(b - (char *)tmp);
        if ((e = launch_fill_i32(cnt, 0, n, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_owned_count, dim3(blocks_for((int64_t)8 * n, 256)), dim3(256), 0, s, n,
                           owner, cnt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = exclusive_scan(b, scan_bytes, cnt, ptr, n, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_set_last, dim3(1), dim3(1), 0, s, ptr, n, 8 * n);
        if ((e = launch_fill_i32(cnt, 0, n, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_owned_fill, dim3(blocks_for((int64_t)8 * n, 256)), dim3(256), 0, s, n,
                           owner, ptr, cnt, pts);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        L.ptr = ptr;
        L.pts = pts;
    }
    const int nn = K + poly_count(m);
    if (nn <= 24) return launch_rbf_nb<24>(geo, xs, ys, perm, nbr, L, n, K, m, dx, W64, dev_err, s);
    if (nn <= 32) return launch_rbf_nb<32>(geo, xs, ys, perm, nbr, L, n, K, m, dx, W64, dev_err, s);
    if (nn <= 48) return launch_rbf_nb<48>(geo, xs, ys, perm, nbr, L, n, K, m, dx, W64, dev_err, s);
    return launch_rbf_nb<64>(geo, xs, ys, perm, nbr, L, n, K, m, dx, W64, dev_err, s);
}

hipError_t launch_pack_w32(const double *W64, int n, int K, float *W32, hipStream_t s) {
    const dim3 grid(blocks_for((int64_t)8 * n, 256)), block(256);
    if (K <= 16)
        hipLaunchKernelGGL(k_pack_w32<16>, grid, block, 0, s, W64, n, K, W32);
    else if (K <= 32)
        hipLaunchKernelGGL(k_pack_w32<32>, grid, block, 0, s, W64, n, K, W32);
    else
        hipLaunchKernelGGL(k_pack_w32<kMaxK>, grid, block, 0, s, W64, n, K, W32);
    return hipGetLastError();
}

hipError_t launch_force(const double *xs, const double *ys, const uint8_t *ntype, int n,
                        int kind, double mag, float *f32, double *f64, hipStream_t s) {
    if (kind == 0) return hipSuccess;
    hipLaunchKernelGGL(k_force, dim3(blocks_for(n, 256)), dim3(256), 0, s, xs, ys, ntype, n,
                       mag, f32, f64);
    return hipGetLastError();
}

}  // namespace mlbm
