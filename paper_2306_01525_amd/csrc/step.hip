// Time stepping of the MLBM on gfx950: initial equilibrium, the fused
// stream + collide step, moments and error reductions.
//
// One lane owns one node. Per step and node the kernel
//   1. interpolates every moving population k = 1..8 at its departure point:
//      f_k(i) = sum_j W[k][j][i] * g_k(nbr[j][s]), s the stencil owner
//      (Sec. 2.3; Appendix A, STREAM); k = 0 departs from the node itself;
//   2. imposes the wall rule at wall nodes;
//   3. takes the moments (eq. macro_var) and applies BGK collision with the
//      optional body force (eqs. LBM_collision, feq; Sec. 3);
//   4. writes the post-collision populations g for the next step.
// The state g is kept post-collision, so one kernel per step reads each
// population once and writes it once; this is the paper's COLLIDE-STREAM order
// shifted by half a step.
//
// The FP32 form stores every population as its deviation from w_k rho0 (the
// populations are O(1) while the flow lives in O(u) corrections); the weights
// reproduce constants, so the streamed deviation is the interpolated
// deviation. The FP64 form stores plain populations.
//
// Memory: the stencil weights dominate the traffic (8K per node per step); they
// are read once, unit-stride across the lanes of a wavefront. The populations
// gathered through nbr are re-used by neighbouring nodes and are served from
// L2; nodes are in Hilbert order so the gathers of a workgroup stay local.
#include "common.h"

namespace mlbm {
namespace {

// ------------------------------------------------------------------------
// FP32, deviation-stored populations
// ------------------------------------------------------------------------

// Bounce-back wall rule (Sec. 3): each population flagged in the node's link
// mask (bit k-1: it enters the fluid from outside the wall) takes the
// streamed value of the opposite direction. Flagged directions point into the
// fluid, so their opposites are never flagged.
template <class T>
__device__ __forceinline__ void bounce_back(unsigned links, T (&f)[kQ]) {
    if (!links) return;
    T g[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) g[k] = f[k];
#pragma unroll
    for (int k = 1; k < kQ; ++k)
        if ((links >> (k - 1)) & 1u) f[k] = g[lat_opp(k)];
}

// Moments, wall rule, BGK collision with force, and the stores of one node.
// WALL: 0 none; 1 equilibrium wall nodes (ntype = node types); 2 bounce-back
// (ntype = the nodes' link masks).
// Directions k0 <= k < k1 are stored (all of them by default; the two lanes
// of a node in the split step store one part each).
template <bool FORCE, int WALL, bool REC>
__device__ __forceinline__ void collide_store32(int n, int p, float (&f)[kQ],
                                                float *__restrict__ go,
                                                const float *__restrict__ force,
                                                const uint8_t *__restrict__ ntype, float rtau,
                                                float rho0, float rho_w,
                                                float *__restrict__ frec, int32_t *err,
                                                const int32_t *perm, int uoff, int k0 = 0,
                                                int k1 = kQ) {
    if (WALL == 1 && ntype[p]) {
#pragma unroll
        for (int k = 0; k < kQ; ++k) {
            if (k < k0 || k >= k1) continue;
            const float v = lat_wmul(k, rho_w - rho0);
            go[(int64_t)k * n + p] = v;
            if (REC) frec[(int64_t)k * n + p] = v;
        }
        return;
    }
    if (WALL == 2) bounce_back(ntype[p], f);
    float drho = 0.0f, jx = 0.0f, jy = 0.0f;
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        drho += f[k];
        jx += f[k] * (float)lat_ex(k);
        jy += f[k] * (float)lat_ey(k);
    }
    const float rho = rho0 + drho;
    const float ux = jx / rho, uy = jy / rho;
    const float uu = ux * ux + uy * uy;
    if (k0 == 0) check_speed(err, uu, perm, p, uoff);
    float ax = 0.0f, ay = 0.0f;
    if (FORCE) {
        ax = force[p];
        ay = force[n + p];
    }
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        if (k < k0 || k >= k1) continue;
        const float eu = (float)lat_ex(k) * ux + (float)lat_ey(k) * uy;
        const float feq = lat_wmul(k, drho + rho * (3.0f * eu + 4.5f * eu * eu - 1.5f * uu));
        float v = f[k] - (f[k] - feq) * rtau;
        if (FORCE) v += lat_wmul(k, 3.0f * ((float)lat_ex(k) * ax + (float)lat_ey(k) * ay));
        go[(int64_t)k * n + p] = v;
        if (REC) frec[(int64_t)k * n + p] = f[k];
    }
}

// One workgroup per tile of kTile nodes. Tiles with gather tables (tdesc
// |H_t| > 0) stage the 8 moving populations of the tile's halo H_t and the
// tile-local stencils of its owners in LDS, then every interpolation reads LDS
// only; HBM sees the weights, the tile tables and the halo rows, all
// contiguous. Tiles without tables gather through global memory.
typedef float f32x4 __attribute__((ext_vector_type(4)));

// One row of four FP32 weights; non-temporal loads do not keep the line in
// the caches.
__device__ __forceinline__ float4 load_w(const float4 *p, bool nt) {
    const f32x4 *q = reinterpret_cast<const f32x4 *>(p);
    const f32x4 v = nt ? __builtin_nontemporal_load(q) : *q;
    return make_float4(v.x, v.y, v.z, v.w);
}

// One pair of FP64 weights, non-temporal.
__device__ __forceinline__ double2 load_w2(const double2 *p) {
    typedef double f64x2 __attribute__((ext_vector_type(2)));
    const f64x2 v = __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(p));
    return make_double2(v.x, v.y);
}

// Staging of a tile (before its barrier), NTH threads. Every load of a lane
// is issued before the first LDS store, so the L2 round trips overlap
// instead of following one another: the halo populations (a halo holds at
// most kHaloCap nodes, so at most kHaloCap / NTH per lane) and the index
// words (in batches of four per lane).
template <int NTH>
__device__ __forceinline__ void stage_halo32(const float *__restrict__ g, int n,
                                             const int32_t *__restrict__ hl, int nh,
                                             float *__restrict__ gl, int32_t *err, int tid) {
    constexpr int U = (kHaloCap + NTH - 1) / NTH;
    int q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int h = tid + u * NTH;
        int v = h < nh ? hl[h] : 0;
        if ((unsigned)v >= (unsigned)n) {   // a bad table must not fault
            v = 0;
            report_index(err);
        }
        q[u] = v;
    }
    float v[U][8];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int d = 0; d < 8; ++d)
            v[u][d] = tid + u * NTH < nh ? g[(int64_t)(d + 1) * n + q[u]] : 0.0f;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int h = tid + u * NTH;
        if (h < nh) {
#pragma unroll
            for (int d = 0; d < 8; ++d) gl[d * nh + h] = v[u][d];
        }
    }
}

template <int NTH>
__device__ __forceinline__ void stage_words(uint32_t *__restrict__ dst,
                                            const uint32_t *__restrict__ src, int count,
                                            int tid) {
    for (int b = 0; b < count; b += 4 * NTH) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int w = b + tid + u * NTH;
            v[u] = w < count ? src[w] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int w = b + tid + u * NTH;
            if (w < count) dst[w] = v[u];
        }
    }
}

// Halo size of a tile that stages its tables, 0 for one that gathers from
// global memory: no tables, or tables larger than the launch's LDS (a plan
// built inside a graph capture sizes its LDS before the tables exist).
__device__ __forceinline__ int tile_halo(const Step32Args &a, int64_t tile) {
    if (!a.tdesc) return 0;
    const int nh = a.tdesc[2 * tile + 1];
    const int no = a.tdesc[2 * tile];
    return nh > 0 && 32 * nh + 4 * no * ((a.K + 2) / 3) <= a.lcap ? nh : 0;
}

template <int MODE, bool FORCE, int WALL, bool REC, int UNROLL, bool NT>
__device__ __forceinline__ void step32_tile(const Step32Args &a, const float *__restrict__ g,
                                            float *__restrict__ go, int64_t tile,
                                            unsigned char *smem) {
    const int n = a.n, K = a.K;
    const int base = (int)(tile * kTile);
    const int cnt = min(kTile, n - base);
    const int tid = threadIdx.x;
    const int nh = tile_halo(a, tile);
    const float4 *__restrict__ W = a.W;

    float acc[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) acc[d] = 0.0f;

    if (nh > 0) {
        const int no = a.tdesc[2 * tile];
        const int Kw = (K + 2) / 3;                                  // index words per owner
        float *gl = reinterpret_cast<float *>(smem);                 // [8][nh]
        uint32_t *nl = reinterpret_cast<uint32_t *>(gl + 8 * nh);    // [no][Kw]
        const int32_t *hl = a.hlist + tile * (int64_t)a.hcap;
        stage_halo32<kTile>(g, n, hl, nh, gl, a.err, tid);
        stage_words<kTile>(nl, a.nbrL + tile * (int64_t)a.ocap * Kw, no * Kw, tid);
        __syncthreads();
        if (tid >= cnt) return;
        const int p = base + tid;
        int ol[8];
#pragma unroll
        for (int d = 0; d < 8; ++d)
            ol[d] = (MODE == MLBM_STENCIL_OWN ? tid : (int)a.ownerL[(int64_t)d * n + p]) * Kw;
        // stencil slots j = 3w, 3w+1, 3w+2 share index word w (10 bits each)
#pragma unroll UNROLL
        for (int w = 0; w < Kw; ++w) {
            uint32_t word[8];
#pragma unroll
            for (int d = 0; d < 8; ++d)
                word[d] = (MODE == MLBM_STENCIL_OWN && d > 0) ? word[0] : nl[ol[d] + w];
#pragma unroll
            for (int sft = 0; sft < 3; ++sft) {
                const int jj = 3 * w + sft;
                if (jj < K) {
                    const float4 wa = load_w(W + ((int64_t)jj * 2) * n + p, NT);
                    const float4 wb = load_w(W + ((int64_t)jj * 2 + 1) * n + p, NT);
                    const float wv[8] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
#pragma unroll
                    for (int d = 0; d < 8; ++d)
                        acc[d] = __builtin_fmaf(
                            wv[d], gl[d * nh + (int)((word[d] >> (10 * sft)) & 1023u)], acc[d]);
                }
            }
        }
        float f[kQ];
        f[0] = g[p];
#pragma unroll
        for (int d = 0; d < 8; ++d) f[d + 1] = acc[d];
        collide_store32<FORCE, WALL, REC>(n, p, f, go, a.force, a.ntype, a.rtau, a.rho0,
                                          a.rho_w, a.frec, a.err, a.perm, a.uoff);
        return;
    }

    if (tid >= cnt) return;
    const int p = base + tid;
    constexpr int UJ = 3 * UNROLL;
    int s[8];
#pragma unroll
    for (int d = 0; d < 8; ++d)
        s[d] = MODE == MLBM_STENCIL_OWN ? p : a.owner[(int64_t)d * n + p];
#pragma unroll UJ
    for (int j = 0; j < K; ++j) {
        const float4 wa = load_w(W + ((int64_t)j * 2) * n + p, NT);
        const float4 wb = load_w(W + ((int64_t)j * 2 + 1) * n + p, NT);
        const float w[8] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
        if (MODE == MLBM_STENCIL_OWN) {
            const int q = a.nbr[(int64_t)j * n + p];
#pragma unroll
            for (int d = 0; d < 8; ++d)
                acc[d] = __builtin_fmaf(w[d], g[(int64_t)(d + 1) * n + q], acc[d]);
        } else {
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const int q = a.nbr[(int64_t)j * n + s[d]];
                acc[d] = __builtin_fmaf(w[d], g[(int64_t)(d + 1) * n + q], acc[d]);
            }
        }
    }
    float f[kQ];
    f[0] = g[p];
#pragma unroll
    for (int d = 0; d < 8; ++d) f[d + 1] = acc[d];
    collide_store32<FORCE, WALL, REC>(n, p, f, go, a.force, a.ntype, a.rtau, a.rho0, a.rho_w,
                                      a.frec, a.err, a.perm, a.uoff);
}

// The same tile with two lanes per node (adjacent lanes; 2 kTile threads):
// lane h of node l interpolates directions 4h+1 .. 4h+4, the pair swaps its
// four sums with a DPP exchange, and both lanes finish the node identically
// (same values, same order), lane 0 storing directions 0..4 and lane 1 5..8.
// The tile's LDS is unchanged, so a compute unit holds twice the wavefronts
// for the same tiles. Per direction the sums run in the same order as in
// step32_tile, so the results are bitwise the same.
__device__ __forceinline__ float swap_pair(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF,
                                                      false));   // quad_perm [1,0,3,2]
}

template <int MODE, bool FORCE, int WALL, bool REC, bool NT, int UNROLL>
__device__ __forceinline__ void step32_tile_split(const Step32Args &a,
                                                  const float *__restrict__ g,
                                                  float *__restrict__ go, int64_t tile,
                                                  unsigned char *smem) {
    const int n = a.n, K = a.K;
    const int base = (int)(tile * kTile);
    const int cnt = min(kTile, n - base);
    const int tid = threadIdx.x, l = tid >> 1, h = tid & 1;
    const int nh = tile_halo(a, tile);
    const float4 *__restrict__ W = a.W;
    float acc[4];
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) acc[dd] = 0.0f;

    if (nh > 0) {
        const int no = a.tdesc[2 * tile];
        const int Kw = (K + 2) / 3;
        float *gl = reinterpret_cast<float *>(smem);                 // [8][nh]
        uint32_t *nl = reinterpret_cast<uint32_t *>(gl + 8 * nh);    // [no][Kw]
        const int32_t *hl = a.hlist + tile * (int64_t)a.hcap;
        stage_halo32<2 * kTile>(g, n, hl, nh, gl, a.err, tid);
        stage_words<2 * kTile>(nl, a.nbrL + tile * (int64_t)a.ocap * Kw, no * Kw, tid);
        __syncthreads();
        if (l >= cnt) return;   // both lanes of a node leave together
        const int p = base + l;
        int ol[4];
#pragma unroll
        for (int dd = 0; dd < 4; ++dd)
            ol[dd] = (MODE == MLBM_STENCIL_OWN ? l
                                               : (int)a.ownerL[(int64_t)(4 * h + dd) * n + p]) * Kw;
        const float *glh = gl + 4 * h * nh;
#pragma unroll UNROLL
        for (int w = 0; w < Kw; ++w) {
            uint32_t word[4];
#pragma unroll
            for (int dd = 0; dd < 4; ++dd)
                word[dd] = (MODE == MLBM_STENCIL_OWN && dd > 0) ? word[0] : nl[ol[dd] + w];
#pragma unroll
            for (int sft = 0; sft < 3; ++sft) {
                const int jj = 3 * w + sft;
                if (jj < K) {
                    const float4 wv = load_w(W + ((int64_t)jj * 2 + h) * n + p, NT);
                    const float wt[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
                    for (int dd = 0; dd < 4; ++dd)
                        acc[dd] = __builtin_fmaf(
                            wt[dd], glh[dd * nh + (int)((word[dd] >> (10 * sft)) & 1023u)], acc[dd]);
                }
            }
        }
    } else {
        if (l >= cnt) return;
        const int p = base + l;
        int s[4];
#pragma unroll
        for (int dd = 0; dd < 4; ++dd)
            s[dd] = MODE == MLBM_STENCIL_OWN ? p : a.owner[(int64_t)(4 * h + dd) * n + p];
        for (int j = 0; j < K; ++j) {
            const float4 wv = load_w(W + ((int64_t)j * 2 + h) * n + p, NT);
            const float wt[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
            for (int dd = 0; dd < 4; ++dd) {
                const int q = a.nbr[(int64_t)j * n + s[dd]];
                acc[dd] = __builtin_fmaf(wt[dd], g[(int64_t)(4 * h + dd + 1) * n + q], acc[dd]);
            }
        }
    }
    const int p = base + l;
    float oth[4];
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) oth[dd] = swap_pair(acc[dd]);
    float f[kQ];
    f[0] = g[p];
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) {
        f[1 + dd] = h ? oth[dd] : acc[dd];
        f[5 + dd] = h ? acc[dd] : oth[dd];
    }
    collide_store32<FORCE, WALL, REC>(n, p, f, go, a.force, a.ntype, a.rtau, a.rho0, a.rho_w,
                                      a.frec, a.err, a.perm, a.uoff, h ? 5 : 0, h ? kQ : 5);
}

template <int MODE, bool FORCE, int WALL, bool REC, bool NT, int UNROLL>
__global__ __launch_bounds__(2 * kTile) void k_step32s(Step32Args a, const float *__restrict__ g,
                                                       float *__restrict__ go, int64_t nblocks) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t tile = xcd_tile(nblocks);
    if (tile >= nblocks) return;
    step32_tile_split<MODE, FORCE, WALL, REC, NT, UNROLL>(a, g, go, tile, smem);
}

template <int MODE, bool FORCE, int WALL, bool REC, int UNROLL, bool NT>
__global__ __launch_bounds__(kTile) void k_step32(Step32Args a, const float *__restrict__ g,
                                                  float *__restrict__ go, int64_t nblocks) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t tile = xcd_tile(nblocks);
    if (tile >= nblocks) return;
    step32_tile<MODE, FORCE, WALL, REC, UNROLL, NT>(a, g, go, tile, smem);
}

// All tiles of all clouds of a batched plan in one launch: the tile's cloud
// comes from tile2cloud, its arrays and parameters from the descriptor table;
// the state of cloud c starts soff elements into g and go.
template <int MODE, int UNROLL, bool NT>
__global__ __launch_bounds__(kTile) void k_step32_batch(const Step32Args *__restrict__ descs,
                                                        const int32_t *__restrict__ tile2cloud,
                                                        const float *__restrict__ g,
                                                        float *__restrict__ go,
                                                        XcdSplit xs) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t t = xcd_split_tile(xs);
    if (t < 0) return;
    const Step32Args a = descs[tile2cloud[t]];
    step32_tile<MODE, false, false, false, UNROLL, NT>(a, g + a.soff, go + a.soff,
                                                        t - a.tile_begin, smem);
}

template <int MODE, bool NT, int UNROLL>
__global__ __launch_bounds__(2 * kTile) void k_step32s_batch(const Step32Args *__restrict__ descs,
                                                             const int32_t *__restrict__ tile2cloud,
                                                             const float *__restrict__ g,
                                                             float *__restrict__ go,
                                                             XcdSplit xs) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t t = xcd_split_tile(xs);
    if (t < 0) return;
    const Step32Args a = descs[tile2cloud[t]];
    step32_tile_split<MODE, false, false, false, NT, UNROLL>(a, g + a.soff, go + a.soff,
                                                             t - a.tile_begin, smem);
}

// Writes one batch descriptor (a kernel, so that graph capture records it).
__global__ void k_set_desc(Step32Args *dst, Step32Args v) { *dst = v; }

// ------------------------------------------------------------------------
// FP64, plain populations
// ------------------------------------------------------------------------
template <bool FORCE, int WALL, bool REC>
__device__ __forceinline__ void collide_store64(int n, int p, double (&f)[kQ],
                                                double *__restrict__ go,
                                                const double *__restrict__ force,
                                                const uint8_t *__restrict__ ntype, double rtau,
                                                double rho_w, double *__restrict__ frec,
                                                int32_t *err, const int32_t *perm, int uoff) {
    if (WALL == 1 && ntype[p]) {
#pragma unroll
        for (int k = 0; k < kQ; ++k) {
            const double v = lat_w(k) * rho_w;
            go[(int64_t)k * n + p] = v;
            if (REC) frec[(int64_t)k * n + p] = v;
        }
        return;
    }
    if (WALL == 2) bounce_back(ntype[p], f);
    double rho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        rho += f[k];
        jx += f[k] * lat_ex(k);
        jy += f[k] * lat_ey(k);
    }
    const double ux = jx / rho, uy = jy / rho;
    const double uu = ux * ux + uy * uy;
    check_speed(err, uu, perm, p, uoff);
    double ax = 0.0, ay = 0.0;
    if (FORCE) {
        ax = force[p];
        ay = force[n + p];
    }
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        const double eu = lat_ex(k) * ux + lat_ey(k) * uy;
        const double feq = lat_w(k) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        double v = f[k] - (f[k] - feq) * rtau;
        if (FORCE) v += 3.0 * lat_w(k) * (lat_ex(k) * ax + lat_ey(k) * ay);
        go[(int64_t)k * n + p] = v;
        if (REC) frec[(int64_t)k * n + p] = f[k];
    }
}

// Same structure as the FP32 step, with the same tile tables: a tile stages
// its halo four directions at a time (4 x |H_t| doubles take the LDS that 8 x
// |H_t| floats take), so the directions are interpolated in two passes. (One
// pass over 8 x |H_t| doubles fits the LDS too, but the larger footprint
// lowers the workgroups per CU and measured slower.)
template <int MODE, bool FORCE, int WALL, bool REC>
__global__ __launch_bounds__(kTile) void k_step64(
    int n, int K, int64_t nblocks, const double *__restrict__ g, double *__restrict__ go,
    const double *__restrict__ W, const int32_t *__restrict__ nbr,
    const int32_t *__restrict__ owner, const double *__restrict__ force,
    const uint8_t *__restrict__ ntype, double rtau, double rho_w, double *__restrict__ frec,
    const int32_t *__restrict__ tdesc, const uint16_t *__restrict__ ownerL,
    const uint32_t *__restrict__ nbrL, const int32_t *__restrict__ hlist, int ocap, int hcap,
    int32_t *err, const int32_t *__restrict__ perm, int uoff) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t tile = xcd_tile(nblocks);
    if (tile >= nblocks) return;
    const int base = (int)(tile * kTile);
    const int cnt = min(kTile, n - base);
    const int tid = threadIdx.x;
    const int p = base + tid;
    const int nh = tdesc ? tdesc[2 * tile + 1] : 0;

    double acc[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) acc[d] = 0.0;
    const double2 *W2 = reinterpret_cast<const double2 *>(W);   // [K][4][n] pairs

    if (nh > 0) {
        const int no = tdesc[2 * tile];
        const int Kw = (K + 2) / 3;
        double *gl = reinterpret_cast<double *>(smem);               // [4][nh]
        uint32_t *nl = reinterpret_cast<uint32_t *>(gl + 4 * nh);    // [no][Kw]
        const int32_t *hl = hlist + tile * (int64_t)hcap;
        const uint32_t *src = nbrL + tile * (int64_t)ocap * Kw;
        for (int w = tid; w < no * Kw; w += kTile) nl[w] = src[w];
        int ol[8];
#pragma unroll
        for (int d = 0; d < 8; ++d)
            ol[d] = tid < cnt ? (MODE == MLBM_STENCIL_OWN ? tid : (int)ownerL[(int64_t)d * n + p]) * Kw
                              : 0;
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            if (pass) __syncthreads();   // the first half is read by everyone
            for (int h = tid; h < nh; h += kTile) {
                int q = hl[h];
                if ((unsigned)q >= (unsigned)n) {   // a bad table must not fault
                    q = 0;
                    report_index(err);
                }
#pragma unroll
                for (int dd = 0; dd < 4; ++dd)
                    gl[dd * nh + h] = g[(int64_t)(4 * pass + dd + 1) * n + q];
            }
            __syncthreads();
            if (tid < cnt) {
#pragma unroll 2
                for (int w = 0; w < Kw; ++w) {
                    uint32_t word[4];
#pragma unroll
                    for (int dd = 0; dd < 4; ++dd)
                        word[dd] = nl[ol[MODE == MLBM_STENCIL_OWN ? 0 : 4 * pass + dd] + w];
#pragma unroll
                    for (int sft = 0; sft < 3; ++sft) {
                        const int jj = 3 * w + sft;
                        if (jj < K) {
                            // directions 4 pass + 1 .. 4 pass + 4 as two pairs
                            // streamed once per step: non-temporal
                            const double2 wa = load_w2(W2 + ((int64_t)jj * 4 + 2 * pass) * n + p);
                            const double2 wb =
                                load_w2(W2 + ((int64_t)jj * 4 + 2 * pass + 1) * n + p);
                            const double wt[4] = {wa.x, wa.y, wb.x, wb.y};
#pragma unroll
                            for (int dd = 0; dd < 4; ++dd)
                                acc[4 * pass + dd] = __builtin_fma(
                                    wt[dd], gl[dd * nh + (int)((word[dd] >> (10 * sft)) & 1023u)],
                                    acc[4 * pass + dd]);
                        }
                    }
                }
            }
        }
        if (tid >= cnt) return;
    } else {
        if (tid >= cnt) return;
        int s[8];
#pragma unroll
        for (int d = 0; d < 8; ++d) s[d] = MODE == MLBM_STENCIL_OWN ? p : owner[(int64_t)d * n + p];
        for (int j = 0; j < K; ++j) {
            int qo = 0;
            if (MODE == MLBM_STENCIL_OWN) qo = nbr[(int64_t)j * n + p];
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const double w = W[w64_at(d + 1, j, n, p)];
                const int q = MODE == MLBM_STENCIL_OWN ? qo : nbr[(int64_t)j * n + s[d]];
                acc[d] = __builtin_fma(w, g[(int64_t)(d + 1) * n + q], acc[d]);
            }
        }
    }
    double f[kQ];
    f[0] = g[p];
#pragma unroll
    for (int d = 0; d < 8; ++d) f[d + 1] = acc[d];
    collide_store64<FORCE, WALL, REC>(n, p, f, go, force, ntype, rtau, rho_w, frec, err, perm,
                                      uoff);
}

// ------------------------------------------------------------------------
// Initial state, moments, L2 sums
// ------------------------------------------------------------------------
template <class T>
__global__ void k_init(int n, const int32_t *__restrict__ perm, const double *__restrict__ rho,
                       const double *__restrict__ ux, const double *__restrict__ uy,
                       const uint8_t *__restrict__ ntype, const double *__restrict__ force,
                       double rho0, double rho_w, int wall, int dev, int collide,
                       T *__restrict__ g) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int u = perm ? perm[p] : p;
    double r = rho ? rho[u] : rho0;
    double vx = ux ? ux[u] : 0.0, vy = uy ? uy[u] : 0.0;
    const bool is_wall = wall && ntype && ntype[p];
    if (is_wall) {
        r = rho_w;
        vx = vy = 0.0;
    }
    const double uu = vx * vx + vy * vy;
    for (int k = 0; k < kQ; ++k) {
        const double eu = lat_ex(k) * vx + lat_ey(k) * vy;
        // feq - w rho0 = w [(rho - rho0) + rho (3 eu + 4.5 eu^2 - 1.5 u^2)]
        double v = dev ? lat_w(k) * ((r - rho0) + r * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu))
                       : lat_w(k) * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        if (collide && force && !is_wall)
            v += 3.0 * lat_w(k) * (lat_ex(k) * force[p] + lat_ey(k) * force[n + p]);
        g[(int64_t)k * n + p] = (T)v;
    }
}

template <class T>
__global__ void k_moments(int n, const int32_t *__restrict__ perm, const T *__restrict__ g,
                          const float *__restrict__ f32, const double *__restrict__ f64,
                          const uint8_t *__restrict__ ntype, double rho0, int dev,
                          double *__restrict__ rho, double *__restrict__ ux,
                          double *__restrict__ uy, int32_t *err, int uoff) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double r = 0.0, jx = 0.0, jy = 0.0;
    for (int k = 0; k < kQ; ++k) {
        const double v = (double)g[(int64_t)k * n + p];
        r += v;
        jx += v * lat_ex(k);
        jy += v * lat_ey(k);
    }
    if (dev) r += rho0;
    if (!(ntype && ntype[p])) {   // the force term added momentum a at fluid nodes
        if (f32) {
            jx -= (double)f32[p];
            jy -= (double)f32[n + p];
        } else if (f64) {
            jx -= f64[p];
            jy -= f64[n + p];
        }
    }
    const int u = perm ? perm[p] : p;
    const double vx = jx / r, vy = jy / r;
    check_speed(err, vx * vx + vy * vy, perm, p, uoff);
    if (rho) rho[u] = r;
    if (ux) ux[u] = vx;
    if (uy) uy[u] = vy;
}

// Per-block partial sums, then a single workgroup adds the partials in a fixed
// order (deterministic, no floating-point atomics).
template <class T>
__global__ __launch_bounds__(256) void k_l2_partial(
    int n, const int32_t *__restrict__ perm, const T *__restrict__ g,
    const float *__restrict__ f32, const double *__restrict__ f64,
    const uint8_t *__restrict__ ntype, double rho0, int dev, const double *__restrict__ uxt,
    const double *__restrict__ uyt, double *__restrict__ part, int32_t *err, int uoff) {
    __shared__ double sh[4][256];
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    if (p < n) {
        double r = 0.0, jx = 0.0, jy = 0.0;
        for (int k = 0; k < kQ; ++k) {
            const double v = (double)g[(int64_t)k * n + p];
            r += v;
            jx += v * lat_ex(k);
            jy += v * lat_ey(k);
        }
        if (dev) r += rho0;
        if (!(ntype && ntype[p])) {
            if (f32) {
                jx -= (double)f32[p];
                jy -= (double)f32[n + p];
            } else if (f64) {
                jx -= f64[p];
                jy -= f64[n + p];
            }
        }
        const int u = perm[p];
        const double vx = jx / r, vy = jy / r;
        check_speed(err, vx * vx + vy * vy, perm, p, uoff);
        const double ex = vx - uxt[u], ey = vy - uyt[u];
        a0 = ex * ex + ey * ey;
        a1 = uxt[u] * uxt[u] + uyt[u] * uyt[u];
        a2 = ex * ex;
        a3 = uxt[u] * uxt[u];
    }
    sh[0][threadIdx.x] = a0;
    sh[1][threadIdx.x] = a1;
    sh[2][threadIdx.x] = a2;
    sh[3][threadIdx.x] = a3;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[(int64_t)blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

// Speed |u| of every node against the speed of an earlier check (user order,
// overwritten with the current speed): part[block] = (sum (|u| - |u_prev|)^2,
// sum |u|^2, 0, 0). The relative residual of the steady-state runs is
// sqrt(out[0] / out[1]).
template <class T>
__global__ __launch_bounds__(256) void k_residual_partial(
    int n, const int32_t *__restrict__ perm, const T *__restrict__ g,
    const float *__restrict__ f32, const double *__restrict__ f64,
    const uint8_t *__restrict__ ntype, double rho0, int dev, double *__restrict__ speed,
    double *__restrict__ part, int32_t *err, int uoff) {
    __shared__ double sh[2][256];
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    double a0 = 0, a1 = 0;
    if (p < n) {
        double r = 0.0, jx = 0.0, jy = 0.0;
        for (int k = 0; k < kQ; ++k) {
            const double v = (double)g[(int64_t)k * n + p];
            r += v;
            jx += v * lat_ex(k);
            jy += v * lat_ey(k);
        }
        if (dev) r += rho0;
        if (!(ntype && ntype[p])) {
            if (f32) {
                jx -= (double)f32[p];
                jy -= (double)f32[n + p];
            } else if (f64) {
                jx -= f64[p];
                jy -= f64[n + p];
            }
        }
        const int u = perm[p];
        const double U = sqrt(jx * jx + jy * jy) / r;
        check_speed(err, U * U, perm, p, uoff);
        const double d = U - speed[u];
        a0 = d * d;
        a1 = U * U;
        speed[u] = U;
    }
    sh[0][threadIdx.x] = a0;
    sh[1][threadIdx.x] = a1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x * 4 + 0] = sh[0][0];
        part[blockIdx.x * 4 + 1] = sh[1][0];
        part[blockIdx.x * 4 + 2] = 0.0;
        part[blockIdx.x * 4 + 3] = 0.0;
    }
}

__global__ __launch_bounds__(256) void k_l2_final(int64_t nparts, const double *__restrict__ part,
                                                  double *__restrict__ out) {
    __shared__ double sh[4][256];
    double a[4] = {0, 0, 0, 0};
    for (int64_t b = threadIdx.x; b < nparts; b += 256)
        for (int c = 0; c < 4; ++c) a[c] += part[b * 4 + c];
    for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = a[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) out[threadIdx.x] = sh[threadIdx.x][0];
}

// Collision only (g = C(f)), same arithmetic as the fused step after its
// streaming part.
template <class T>
__global__ void k_collide(int n, const T *__restrict__ f, T *__restrict__ g,
                          const double *__restrict__ force, const uint8_t *__restrict__ ntype,
                          int wall, double rtau, double rho0, double rho_w, int dev) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    if (wall && ntype && ntype[p]) {
        for (int k = 0; k < kQ; ++k)
            g[(int64_t)k * n + p] = (T)(dev ? lat_w(k) * (rho_w - rho0) : lat_w(k) * rho_w);
        return;
    }
    T fk[kQ];
    T drho = 0, jx = 0, jy = 0;
    for (int k = 0; k < kQ; ++k) {
        fk[k] = f[(int64_t)k * n + p];
        drho += fk[k];
        jx += fk[k] * (T)lat_ex(k);
        jy += fk[k] * (T)lat_ey(k);
    }
    const T rho = dev ? (T)rho0 + drho : drho;
    const T ux = jx / rho, uy = jy / rho, uu = ux * ux + uy * uy;
    for (int k = 0; k < kQ; ++k) {
        const T eu = (T)lat_ex(k) * ux + (T)lat_ey(k) * uy;
        const T poly = (T)3 * eu + (T)4.5 * eu * eu - (T)1.5 * uu;
        const T feq = dev ? lat_wmul(k, drho + rho * poly) : lat_wmul(k, rho * ((T)1 + poly));
        T v = fk[k] - (fk[k] - feq) * (T)rtau;
        if (force)
            v += (T)(3.0 * lat_w(k) * (lat_ex(k) * force[p] + lat_ey(k) * force[n + p]));
        g[(int64_t)k * n + p] = v;
    }
}

// Tuning variants of the FP32 step: unroll depth of the stencil loop over
// index words (1, 2 or 3 words = 3, 6 or 9 weight rows a lane has in flight)
// and non-temporal weight loads (the weights are streamed once per step and
// need not displace the halo rows in L2). Variant v < 6: one lane per node,
// unroll {1, 2, 3}[v / 2], non-temporal v % 2. Tiles without tables unroll
// their row loop 3x that. Variants 6-9: two lanes per node (directions split
// in halves), non-temporal v % 2, the index-word loop unrolled 2x from 8 on.
template <int MODE, bool FORCE, int WALL, bool REC, int UNROLL, bool NT>
void launch32(const CloudPlan &cp, const void *gin, void *gout, void *frec, int64_t nblocks,
              hipStream_t s) {
    const Step32Args a = step32_args(cp, frec);
    hipLaunchKernelGGL((k_step32<MODE, FORCE, WALL, REC, UNROLL, NT>), dim3(xcd_grid(nblocks)),
                       dim3(kTile), cp.lds_bytes, s, a, (const float *)gin, (float *)gout,
                       nblocks);
}

template <int MODE, bool FORCE, int WALL, bool REC, bool NT, int UNROLL = 1>
void launch32s(const CloudPlan &cp, const void *gin, void *gout, void *frec, int64_t nblocks,
               hipStream_t s) {
    const Step32Args a = step32_args(cp, frec);
    hipLaunchKernelGGL((k_step32s<MODE, FORCE, WALL, REC, NT, UNROLL>), dim3(xcd_grid(nblocks)),
                       dim3(2 * kTile), cp.lds_bytes, s, a, (const float *)gin, (float *)gout,
                       nblocks);
}

template <int MODE, bool NT, int UNROLL = 1>
void launch32s_batch(const mlbm_plan &plan, const void *gin, void *gout, hipStream_t s) {
    hipLaunchKernelGGL((k_step32s_batch<MODE, NT, UNROLL>), dim3(8 * plan.xcd_longest),
                       dim3(2 * kTile), plan.batch_lds, s, plan.descs, plan.tile2cloud,
                       (const float *)gin, (float *)gout, plan.xcd);
}

template <int MODE, int UNROLL, bool NT>
void launch32_batch(const mlbm_plan &plan, const void *gin, void *gout, hipStream_t s) {
    hipLaunchKernelGGL((k_step32_batch<MODE, UNROLL, NT>), dim3(8 * plan.xcd_longest),
                       dim3(kTile), plan.batch_lds, s, plan.descs, plan.tile2cloud,
                       (const float *)gin, (float *)gout, plan.xcd);
}

template <int MODE>
void launch32_batch_v(const mlbm_plan &plan, const void *gin, void *gout, hipStream_t s) {
    switch (plan.c[0].variant) {
        case 1: launch32_batch<MODE, 1, true>(plan, gin, gout, s); break;
        case 2: launch32_batch<MODE, 2, false>(plan, gin, gout, s); break;
        case 3: launch32_batch<MODE, 2, true>(plan, gin, gout, s); break;
        case 4: launch32_batch<MODE, 3, false>(plan, gin, gout, s); break;
        case 5: launch32_batch<MODE, 3, true>(plan, gin, gout, s); break;
        case 6: launch32s_batch<MODE, false>(plan, gin, gout, s); break;
        case 7: launch32s_batch<MODE, true>(plan, gin, gout, s); break;
        case 8: launch32s_batch<MODE, false, 2>(plan, gin, gout, s); break;
        case 9: launch32s_batch<MODE, true, 2>(plan, gin, gout, s); break;
        default: launch32_batch<MODE, 1, false>(plan, gin, gout, s); break;
    }
}

template <int MODE, bool FORCE, int WALL, bool REC>
void launch32_tuned(const CloudPlan &cp, const void *gin, void *gout, void *frec,
                    int64_t nblocks, hipStream_t s) {
    if (WALL == 2 || FORCE != (WALL == 1)) {   // other wall/force mixes: default variant
        launch32<MODE, FORCE, WALL, REC, 1, false>(cp, gin, gout, frec, nblocks, s);
        return;
    }
    switch (cp.variant) {
        case 1: launch32<MODE, FORCE, WALL, REC, 1, true>(cp, gin, gout, frec, nblocks, s); break;
        case 2: launch32<MODE, FORCE, WALL, REC, 2, false>(cp, gin, gout, frec, nblocks, s); break;
        case 3: launch32<MODE, FORCE, WALL, REC, 2, true>(cp, gin, gout, frec, nblocks, s); break;
        case 4: launch32<MODE, FORCE, WALL, REC, 3, false>(cp, gin, gout, frec, nblocks, s); break;
        case 5: launch32<MODE, FORCE, WALL, REC, 3, true>(cp, gin, gout, frec, nblocks, s); break;
        case 6: launch32s<MODE, FORCE, WALL, REC, false>(cp, gin, gout, frec, nblocks, s); break;
        case 7: launch32s<MODE, FORCE, WALL, REC, true>(cp, gin, gout, frec, nblocks, s); break;
        case 8: launch32s<MODE, FORCE, WALL, REC, false, 2>(cp, gin, gout, frec, nblocks, s); break;
        case 9: launch32s<MODE, FORCE, WALL, REC, true, 2>(cp, gin, gout, frec, nblocks, s); break;
        default: launch32<MODE, FORCE, WALL, REC, 1, false>(cp, gin, gout, frec, nblocks, s); break;
    }
}

template <int MODE, bool FORCE, int WALL, bool REC>
hipError_t step_variant(const CloudPlan &cp, int precision, const void *gin, void *gout,
                        void *frec, hipStream_t s) {
    const int n = cp.n;
    const int64_t nblocks = (n + kTile - 1) / kTile;
    if (precision == MLBM_FP64) {
        hipLaunchKernelGGL((k_step64<MODE, FORCE, WALL, REC>), dim3(xcd_grid(nblocks)),
                           dim3(kTile), cp.lds_bytes, s, n, cp.K, nblocks, (const double *)gin,
                           (double *)gout, cp.W64, cp.nbr, cp.owner, cp.force64,
                           cp.prm.wall_kind == 2 ? cp.links : cp.ntype,
                           1.0 / cp.prm.tau, cp.prm.rho_wall, (double *)frec,
                           cp.lds_bytes ? cp.tdesc : nullptr, cp.ownerL, cp.nbrL, cp.hlist,
                           cp.ocap, cp.hcap, cp.err, cp.perm, (int)cp.off);
    } else {
        launch32_tuned<MODE, FORCE, WALL, REC>(cp, gin, gout, frec, nblocks, s);
    }
    return hipGetLastError();
}

template <int MODE, bool FORCE, int WALL>
hipError_t step_rec(const CloudPlan &cp, int precision, const void *gin, void *gout,
                    void *frec, hipStream_t s) {
    return frec ? step_variant<MODE, FORCE, WALL, true>(cp, precision, gin, gout, frec, s)
                : step_variant<MODE, FORCE, WALL, false>(cp, precision, gin, gout, frec, s);
}

template <int MODE, bool FORCE>
hipError_t step_wall(const CloudPlan &cp, int precision, const void *gin, void *gout,
                     void *frec, hipStream_t s) {
    switch (cp.prm.wall_kind) {
        case 1: return step_rec<MODE, FORCE, 1>(cp, precision, gin, gout, frec, s);
        case 2: return step_rec<MODE, FORCE, 2>(cp, precision, gin, gout, frec, s);
        default: return step_rec<MODE, FORCE, 0>(cp, precision, gin, gout, frec, s);
    }
}

template <int MODE>
hipError_t step_force(const CloudPlan &cp, int precision, const void *gin, void *gout,
                      void *frec, hipStream_t s) {
    return cp.prm.force_kind ? step_wall<MODE, true>(cp, precision, gin, gout, frec, s)
                             : step_wall<MODE, false>(cp, precision, gin, gout, frec, s);
}

// ------------------------------------------------------------------------
// Standard lattice Boltzmann (eq. LBM_streaming): the reference method of the
// paper on a periodic nx x ny lattice, state [9][ny][nx] with x fastest.
// Streaming is a pull by the index shift x - e_k (wrapped), followed by the
// same moments and BGK collision as the fused MLBM step. Workgroups cover 256
// consecutive nodes of a row; the XCD map keeps neighbouring rows, which read
// each other's populations, in one L2.
// ------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_lbm_step(int nx, int ny, int64_t nblocks,
                                                  const T *__restrict__ g, T *__restrict__ go,
                                                  double rtau, double rho0) {
    const int64_t b = xcd_tile(nblocks);
    if (b >= nblocks) return;
    const int bx = (nx + 255) / 256;
    const int y = (int)(b / bx);
    const int x = (int)(b - (int64_t)y * bx) * 256 + threadIdx.x;
    if (x >= nx) return;
    const int64_t n = (int64_t)nx * ny;
    const int p = y * nx + x;
    T f[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        int sx = x - (int)lat_ex(k), sy = y - (int)lat_ey(k);
        sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
        sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
        f[k] = g[(int64_t)k * n + (int64_t)sy * nx + sx];
    }
    if constexpr (sizeof(T) == 4)
        collide_store32<false, false, false>((int)n, p, f, go, nullptr, nullptr, (float)rtau,
                                             (float)rho0, 0.0f, nullptr, nullptr, nullptr, 0);
    else
        collide_store64<false, false, false>((int)n, p, f, go, nullptr, nullptr, rtau, 0.0,
                                             nullptr, nullptr, nullptr, 0);
}

// Interpolation alone (Sec. 4, Fig. interp_test): the streaming operator of
// the plan applied to a scalar field, in FP64 with the FP64 shape vectors.
// out[k-1][u] = sum_j W_k[j](p) field[user(nbr[j][owner_k(p)])], u = user(p).
__global__ __launch_bounds__(256) void k_interpolate(int n, int K, int mode,
                                                     const double *__restrict__ W64,
                                                     const int32_t *__restrict__ nbr,
                                                     const int32_t *__restrict__ owner,
                                                     const int32_t *__restrict__ perm,
                                                     const double *__restrict__ field,
                                                     int64_t out_stride, double *__restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int u = perm[p];
    for (int k = 1; k < kQ; ++k) {
        const int s = mode == MLBM_STENCIL_OWN ? p : owner[(int64_t)(k - 1) * n + p];
        double acc = 0.0;
        for (int j = 0; j < K; ++j)
            acc = __builtin_fma(W64[w64_at(k, j, n, p)], field[perm[nbr[(int64_t)j * n + s]]], acc);
        out[(int64_t)(k - 1) * out_stride + u] = acc;
    }
}

}  // namespace

hipError_t launch_interpolate(const CloudPlan &cp, const double *field, int64_t out_stride,
                              double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_interpolate, dim3(blocks_for(cp.n, 256)), dim3(256), 0, s, cp.n, cp.K,
                       cp.prm.stencil_mode, cp.W64, cp.nbr, cp.owner, cp.perm, field, out_stride,
                       out);
    return hipGetLastError();
}

// Nodes whose populations carry no body force (so the moments need no
// correction there): the equilibrium wall nodes; with bounce-back, none.
inline const uint8_t *fmask(const CloudPlan &cp) { return cp.has_walls ? cp.ntype : nullptr; }

Step32Args step32_args(const CloudPlan &cp, void *frec) {
    Step32Args a{};
    a.n = cp.n;
    a.K = cp.K;
    a.ocap = cp.ocap;
    a.hcap = cp.hcap;
    a.W = reinterpret_cast<const float4 *>(cp.W32);
    a.nbr = cp.nbr;
    a.owner = cp.owner;
    a.force = cp.force32;
    a.ntype = cp.prm.wall_kind == 2 ? cp.links : cp.ntype;   // link masks for bounce-back
    a.rtau = (float)(1.0 / cp.prm.tau);
    a.rho0 = (float)cp.prm.rho0;
    a.rho_w = (float)cp.prm.rho_wall;
    a.frec = (float *)frec;
    a.tdesc = cp.lds_bytes ? cp.tdesc : nullptr;
    a.lcap = (int)cp.lds_bytes;
    a.ownerL = cp.ownerL;
    a.nbrL = cp.nbrL;
    a.hlist = cp.hlist;
    a.soff = 0;
    a.tile_begin = 0;
    a.err = cp.err;
    a.perm = cp.perm;
    a.uoff = (int)cp.off;
    return a;
}

hipError_t launch_step_batch(const mlbm_plan &plan, const void *gin, void *gout,
                             hipStream_t s) {
    if (plan.batch_mode == MLBM_STENCIL_OWN)
        launch32_batch_v<MLBM_STENCIL_OWN>(plan, gin, gout, s);
    else
        launch32_batch_v<MLBM_STENCIL_PAPER>(plan, gin, gout, s);
    return hipGetLastError();
}

hipError_t launch_set_desc(Step32Args *dst, const Step32Args &v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(1), 0, s, dst, v);
    return hipGetLastError();
}

hipError_t launch_step(const CloudPlan &cp, int precision, const void *gin, void *gout,
                       void *frec, hipStream_t s) {
    return cp.prm.stencil_mode == MLBM_STENCIL_OWN
               ? step_force<MLBM_STENCIL_OWN>(cp, precision, gin, gout, frec, s)
               : step_force<MLBM_STENCIL_PAPER>(cp, precision, gin, gout, frec, s);
}

hipError_t launch_init(const CloudPlan &cp, int precision, const double *rho,
                       const double *ux, const double *uy, void *g, bool collide,
                       hipStream_t s) {
    const int n = cp.n;
    const int wall = cp.has_walls ? 1 : 0;
    if (precision == MLBM_FP64)
        hipLaunchKernelGGL(k_init<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n,
                           cp.perm, rho, ux, uy, cp.ntype, cp.force64, cp.prm.rho0,
                           cp.prm.rho_wall, wall, 0, collide ? 1 : 0, (double *)g);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n,
                           cp.perm, rho, ux, uy, cp.ntype, cp.force64, cp.prm.rho0,
                           cp.prm.rho_wall, wall, 1, collide ? 1 : 0, (float *)g);
    return hipGetLastError();
}

hipError_t launch_moments(const CloudPlan &cp, int precision, const void *g, double *rho,
                          double *ux, double *uy, bool post_collision, hipStream_t s) {
    const int n = cp.n;
    const float *f32 = post_collision && precision != MLBM_FP64 ? cp.force32 : nullptr;
    const double *f64 = post_collision && precision == MLBM_FP64 ? cp.force64 : nullptr;
    if (precision == MLBM_FP64)
        hipLaunchKernelGGL(k_moments<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n,
                           cp.perm, (const double *)g, f32, f64, fmask(cp), cp.prm.rho0, 0, rho,
                           ux, uy, cp.err, (int)cp.off);
    else
        hipLaunchKernelGGL(k_moments<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n,
                           cp.perm, (const float *)g, f32, f64, fmask(cp), cp.prm.rho0, 1, rho,
                           ux, uy, cp.err, (int)cp.off);
    return hipGetLastError();
}

hipError_t launch_l2(const CloudPlan &cp, int precision, const void *g, const double *uxt,
                     const double *uyt, double *out, double *part, hipStream_t s) {
    const int n = cp.n;
    const int64_t nb = blocks_for(n, 256);
    const float *f32 = precision != MLBM_FP64 ? cp.force32 : nullptr;
    const double *f64 = precision == MLBM_FP64 ? cp.force64 : nullptr;
    if (precision == MLBM_FP64)
        hipLaunchKernelGGL(k_l2_partial<double>, dim3(nb), dim3(256), 0, s, n, cp.perm,
                           (const double *)g, f32, f64, fmask(cp), cp.prm.rho0, 0, uxt, uyt, part,
                           cp.err, (int)cp.off);
    else
        hipLaunchKernelGGL(k_l2_partial<float>, dim3(nb), dim3(256), 0, s, n, cp.perm,
                           (const float *)g, f32, f64, fmask(cp), cp.prm.rho0, 1, uxt, uyt, part,
                           cp.err, (int)cp.off);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_l2_final, dim3(1), dim3(256), 0, s, nb, (const double *)part, out);
    return hipGetLastError();
}

hipError_t launch_residual(const CloudPlan &cp, int precision, const void *g, double *speed,
                           double *out, double *part, hipStream_t s) {
    const int n = cp.n;
    const int64_t nb = blocks_for(n, 256);
    const float *f32 = precision != MLBM_FP64 ? cp.force32 : nullptr;
    const double *f64 = precision == MLBM_FP64 ? cp.force64 : nullptr;
    if (precision == MLBM_FP64)
        hipLaunchKernelGGL(k_residual_partial<double>, dim3(nb), dim3(256), 0, s, n, cp.perm,
                           (const double *)g, f32, f64, fmask(cp), cp.prm.rho0, 0, speed, part,
                           cp.err, (int)cp.off);
    else
        hipLaunchKernelGGL(k_residual_partial<float>, dim3(nb), dim3(256), 0, s, n, cp.perm,
                           (const float *)g, f32, f64, fmask(cp), cp.prm.rho0, 1, speed, part,
                           cp.err, (int)cp.off);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_l2_final, dim3(1), dim3(256), 0, s, nb, (const double *)part, out);
    return hipGetLastError();
}

hipError_t launch_collide(const CloudPlan &cp, int precision, const void *f, void *g,
                          hipStream_t s) {
    const int n = cp.n;
    const int wall = cp.has_walls ? 1 : 0;
    const double *force = cp.prm.force_kind ? cp.force64 : nullptr;
    if (precision == MLBM_FP64)
        hipLaunchKernelGGL(k_collide<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n,
                           (const double *)f, (double *)g, force, cp.ntype, wall,
                           1.0 / cp.prm.tau, cp.prm.rho0, cp.prm.rho_wall, 0);
    else
        hipLaunchKernelGGL(k_collide<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n,
                           (const float *)f, (float *)g, force, cp.ntype, wall,
                           1.0 / cp.prm.tau, cp.prm.rho0, cp.prm.rho_wall, 1);
    return hipGetLastError();
}

hipError_t launch_l2_final(const double *part, int64_t nparts, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_l2_final, dim3(1), dim3(256), 0, s, nparts, part, out);
    return hipGetLastError();
}

hipError_t launch_lbm_step(int nx, int ny, int precision, double tau, double rho0,
                           const void *g, void *go, hipStream_t s) {
    const int64_t nblocks = (int64_t)ny * ((nx + 255) / 256);
    if (precision == MLBM_FP64)
        hipLaunchKernelGGL(k_lbm_step<double>, dim3(xcd_grid(nblocks)), dim3(256), 0, s, nx, ny,
                           nblocks, (const double *)g, (double *)go, 1.0 / tau, rho0);
    else
        hipLaunchKernelGGL(k_lbm_step<float>, dim3(xcd_grid(nblocks)), dim3(256), 0, s, nx, ny,
                           nblocks, (const float *)g, (float *)go, 1.0 / tau, rho0);
    return hipGetLastError();
}

hipError_t launch_lbm_init(int n, int precision, double rho0, const double *rho, const double *ux,
                           const double *uy, void *g, hipStream_t s) {
    if (precision == MLBM_FP64)
        hipLaunchKernelGGL(k_init<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n,
                           (const int32_t *)nullptr, rho, ux, uy, (const uint8_t *)nullptr,
                           (const double *)nullptr, rho0, rho0, 0, 0, 0, (double *)g);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n,
                           (const int32_t *)nullptr, rho, ux, uy, (const uint8_t *)nullptr,
                           (const double *)nullptr, rho0, rho0, 0, 1, 0, (float *)g);
    return hipGetLastError();
}

hipError_t launch_lbm_moments(int n, int precision, double rho0, const void *g, double *rho,
                              double *ux, double *uy, hipStream_t s) {
    if (precision == MLBM_FP64)
        hipLaunchKernelGGL(k_moments<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n,
                           (const int32_t *)nullptr, (const double *)g, (const float *)nullptr,
                           (const double *)nullptr, (const uint8_t *)nullptr, rho0, 0, rho, ux,
                           uy, (int32_t *)nullptr, 0);
    else
        hipLaunchKernelGGL(k_moments<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n,
                           (const int32_t *)nullptr, (const float *)g, (const float *)nullptr,
                           (const double *)nullptr, (const uint8_t *)nullptr, rho0, 1, rho, ux,
                           uy, (int32_t *)nullptr, 0);
    return hipGetLastError();
}

}  // namespace mlbm
