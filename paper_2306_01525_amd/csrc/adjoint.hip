// Discrete adjoint of the MLBM time loop on gfx950 (periodic, no walls, no
// force). The forward step is f^{n+1} = S(C(f^n)): C the BGK collision
// (eqs. LBM_collision, feq), S the semi-Lagrangian streaming through the
// shape vectors (Sec. 2.3). Its adjoint is lam^n = C'(f^n)^T S^T lam^{n+1}.
//
// S^T is applied as a gather, not a scatter: for every direction k and source
// node m, the list of (arriving node i, weight) pairs whose stencil reads m is
// stored as a CSR row sorted by i. Each lane owns one source node and sums its
// row in that fixed order, so the adjoint needs no atomics and is
// deterministic. The weights are the ones the forward step uses (FP32 after
// the partition-of-unity correction, or FP64).
#include <climits>

#include "common.h"

namespace mlbm {
namespace {

__device__ __forceinline__ int stencil_owner(const int32_t *owner, int mode, int k, int n,
                                             int i) {
    return mode == MLBM_STENCIL_OWN ? i : owner[(int64_t)(k - 1) * n + i];
}

// Row lengths and fill of the transposed operator. Entries (arriving node i,
// direction k, stencil slot j) are gathered by row (k, source node m) in an
// LDS hash table per tile of arriving nodes, so that a tile adds to a row, or
// claims a run of it, with a single atomic. Keys that find no slot within
// kTrProbe probes (an unusually wide tile) fall back to one atomic per entry;
// k_tr_sort orders every row afterwards.
constexpr int kTrHash = 4096;    // counts: keys of four directions
constexpr int kTrHashF = 1024;   // fill: keys of one direction
constexpr int kTrProbe = 32;
constexpr uint32_t kTrEmpty = 0xFFFFFFFFu;

template <int HS = kTrHash>
__device__ __forceinline__ int tr_slot(uint32_t *hkey, uint32_t key, bool insert) {
    static_assert((HS & (HS - 1)) == 0, "power of two");
    const uint32_t h = (key * 2654435761u) >> (32 - __builtin_ctz(HS));
    for (int p = 0; p < kTrProbe; ++p) {
        const int sl = (int)((h + p) & (HS - 1));
        const uint32_t cur = hkey[sl];
        if (cur == key) return sl;
        if (cur == kTrEmpty) {
            if (!insert) return -1;
            const uint32_t prev = atomicCAS(&hkey[sl], kTrEmpty, key);
            if (prev == kTrEmpty || prev == key) return sl;
        }
    }
    return -1;
}

// Source node m of entry (i, direction 4 h + kk + 1, slot j).
__device__ __forceinline__ int tr_source(const int32_t *nbr, const int32_t *owner, int mode,
                                         int n, int h, int kk, int j, int i) {
    const int s = stencil_owner(owner, mode, 4 * h + kk + 1, n, i);
    return nbr[(int64_t)j * n + s];
}

// Pass over the workgroup's entries: per-key counts in hcnt; entries without
// a slot add to cnt_direct[row] directly (when it is given).
__device__ __forceinline__ void tr_count_tile(int n, int K, int mode, int h, int i,
                                              const int32_t *nbr, const int32_t *owner,
                                              uint32_t *hkey, int32_t *hcnt,
                                              int32_t *cnt_direct) {
    if (i >= n) return;
    for (int j = 0; j < K; ++j) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int m = tr_source(nbr, owner, mode, n, h, kk, j, i);
            const int sl = tr_slot(hkey, (uint32_t)(kk * n + m), true);
            if (sl >= 0)
                atomicAdd(&hcnt[sl], 1);
            else if (cnt_direct)
                atomicAdd(&cnt_direct[(int64_t)(4 * h + kk) * n + m], 1);
        }
    }
}

__device__ __forceinline__ void tr_hash_clear(uint32_t *hkey, int32_t *hcnt) {
    for (int t = threadIdx.x; t < kTrHash; t += blockDim.x) {
        hkey[t] = kTrEmpty;
        hcnt[t] = 0;
    }
}

__device__ __forceinline__ int64_t tr_key_row(uint32_t key, int n, int h) {
    const int kk = (int)(key / (uint32_t)n), m = (int)(key - (uint32_t)kk * n);
    return (int64_t)(4 * h + kk) * n + m;
}

// Counts: a workgroup per tile of 256 arriving nodes and half of the
// directions (1-4 or 5-8), keys (k - 1 - 4 h) n + m.
__global__ __launch_bounds__(256) void k_tr_count(int n, int K, int mode,
                                                  const int32_t *__restrict__ nbr,
                                                  const int32_t *__restrict__ owner,
                                                  int32_t *__restrict__ cnt) {
    __shared__ uint32_t hkey[kTrHash];
    __shared__ int32_t hcnt[kTrHash];
    const int64_t nt = ((int64_t)n + 255) / 256, t = xcd_tile(nt);
    if (t >= nt) return;   // uniform
    const int h = blockIdx.y, i = (int)(t * 256) + (int)threadIdx.x;
    tr_hash_clear(hkey, hcnt);
    __syncthreads();
    tr_count_tile(n, K, mode, h, i, nbr, owner, hkey, hcnt, cnt);
    __syncthreads();
    for (int t = threadIdx.x; t < kTrHash; t += blockDim.x)
        if (hkey[t] != kTrEmpty) atomicAdd(&cnt[tr_key_row(hkey[t], n, h)], hcnt[t]);
}

// Fill: a workgroup of kTrJs TT threads takes a tile of TT arriving nodes
// (kTrJs threads a node, each on every kTrJs-th stencil slot: the LDS the
// tile needs leaves room for few workgroups, so each brings many wavefronts)
// and a half of the directions, one direction after another. For each it counts the
// tile's entries per row, claims one run of each row, gathers the entries in
// LDS run by run with their places, and then writes the runs out with
// consecutive lanes on consecutive places. The LDS holds TT K entries (the
// host picks TT so that they fit).
constexpr int kTrJs = 4;
template <class T, int TT>
__global__ __launch_bounds__(kTrJs * TT) void k_tr_fill(int n, int K, int mode,
                                                const int32_t *__restrict__ nbr,
                                                const int32_t *__restrict__ owner,
                                                const float *__restrict__ W32,
                                                const double *__restrict__ W64,
                                                const int32_t *__restrict__ ptr,
                                                int32_t *__restrict__ cur,
                                                int32_t *__restrict__ col, T *__restrict__ val) {
    extern __shared__ __align__(16) unsigned char s_stage[];
    __shared__ uint32_t hkey[kTrHashF];
    __shared__ int32_t hcnt[kTrHashF];
    __shared__ int32_t hbase[kTrHashF];
    __shared__ int32_t hloc[kTrHashF];
    constexpr int NT = kTrJs * TT;
    __shared__ int32_t s_part[NT];
    constexpr int SPT = kTrHashF / NT;   // hash slots per thread in the scan
    static_assert(kTrHashF % NT == 0, "whole slots per thread");
    const int64_t nt = ((int64_t)n + TT - 1) / TT, t = xcd_tile(nt);
    if (t >= nt) return;   // uniform
    const int h = blockIdx.y, tid = threadIdx.x;
    const int i = (int)(t * TT) + tid % TT, j0 = tid / TT;
    const size_t words = ((size_t)TT * K * sizeof(int32_t) + 15) & ~size_t(15);
    int32_t *scol = reinterpret_cast<int32_t *>(s_stage);
    int32_t *spos = reinterpret_cast<int32_t *>(s_stage + words);
    T *sval = reinterpret_cast<T *>(s_stage + 2 * words);
    for (int kk = 0; kk < 4; ++kk) {
        const int k = 4 * h + kk + 1;
        for (int q = tid; q < kTrHashF; q += NT) {
            hkey[q] = kTrEmpty;
            hcnt[q] = 0;
        }
        __syncthreads();
        const int s = i < n ? stencil_owner(owner, mode, k, n, i) : 0;
        if (i < n) {
            for (int j = j0; j < K; j += kTrJs) {
                const int sl = tr_slot<kTrHashF>(hkey, (uint32_t)nbr[(int64_t)j * n + s], true);
                if (sl >= 0) atomicAdd(&hcnt[sl], 1);
            }
        }
        __syncthreads();
        // local run starts in slot order (exclusive scan), the rows' runs
        int mine = 0;
#pragma unroll
        for (int q = 0; q < SPT; ++q) mine += hcnt[tid * SPT + q];
        s_part[tid] = mine;
        __syncthreads();
        for (int w = 1; w < NT; w <<= 1) {
            const int add = tid >= w ? s_part[tid - w] : 0;
            __syncthreads();
            s_part[tid] += add;
            __syncthreads();
        }
        int run = s_part[tid] - mine;
        const int total = s_part[NT - 1];
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int sl = tid * SPT + q;
            const int c = hcnt[sl];
            hloc[sl] = run;
            run += c;
            if (c > 0) {
                const int64_t row = (int64_t)(k - 1) * n + hkey[sl];
                hbase[sl] = ptr[row] + atomicAdd(&cur[row], c);
            }
            hcnt[sl] = 0;
        }
        __syncthreads();
        if (i < n) {
            for (int j = j0; j < K; j += kTrJs) {
                const int m = nbr[(int64_t)j * n + s];
                const int sl = tr_slot<kTrHashF>(hkey, (uint32_t)m, false);
                const T w = W64 ? (T)W64[w64_at(k, j, n, i)]
                                : (T)W32[(((int64_t)j * 2 + ((k - 1) >> 2)) * n + i) * 4 +
                                         ((k - 1) & 3)];
                if (sl >= 0) {
                    const int r = atomicAdd(&hcnt[sl], 1), q = hloc[sl] + r;
                    scol[q] = i;
                    spos[q] = hbase[sl] + r;
                    sval[q] = w;
                } else {   // no slot: a place of its own
                    const int64_t row = (int64_t)(k - 1) * n + m;
                    const int pos = ptr[row] + atomicAdd(&cur[row], 1);
                    col[pos] = i;
                    val[pos] = w;
                }
            }
        }
        __syncthreads();
        for (int q = tid; q < total; q += NT) {
            const int pos = spos[q];
            col[pos] = scol[q];
            val[pos] = sval[q];
        }
        __syncthreads();
    }
}

// Sort each CSR row by arriving node. An arriving node appears at most once
// in a row, so the rank of an entry (how many entries of the row have a
// smaller column) is its sorted position. A wavefront takes two rows: when
// both have at most 32 entries, each half of the wavefront ranks one;
// otherwise the whole wavefront ranks one row after the other, and a row
// longer than a wavefront (not met with K <= 48 on clouds of even spacing)
// takes an insertion sort by one lane.
template <class T>
__device__ __forceinline__ void tr_sort_row_wave(int lane, int b, int len, int32_t *col, T *val) {
    if (len <= 64) {
        int c = INT_MAX;
        T v = 0;
        if (lane < len) {
            c = col[b + lane];
            v = val[b + lane];
        }
        int rank = 0;
        for (int j = 0; j < len; ++j) rank += __shfl(c, j, 64) < c;   // len: uniform
        if (lane < len) {
            col[b + rank] = c;
            val[b + rank] = v;
        }
        return;
    }
    if (lane != 0) return;
    for (int a = b + 1; a < b + len; ++a) {
        const int c = col[a];
        const T v = val[a];
        int q = a - 1;
        while (q >= b && col[q] > c) {
            col[q + 1] = col[q];
            val[q + 1] = val[q];
            --q;
        }
        col[q + 1] = c;
        val[q + 1] = v;
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_tr_sort(int64_t rows, const int32_t *__restrict__ ptr,
                                                 int32_t *__restrict__ col, T *__restrict__ val) {
    const int lane = threadIdx.x & 63;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 2;
    if (r0 >= rows) return;   // uniform across the wavefront
    const int half = lane >> 5, hl = lane & 31;
    const int64_t r = r0 + half;
    const int b = r < rows ? ptr[r] : 0;
    const int len = r < rows ? ptr[r + 1] - b : 0;
    const int len0 = __builtin_amdgcn_readlane(len, 0), len1 = __builtin_amdgcn_readlane(len, 32);
    const int lmax = max(len0, len1);
    if (lmax <= 32) {
        int c = INT_MAX;
        T v = 0;
        if (hl < len) {
            c = col[b + hl];
            v = val[b + hl];
        }
        int rank = 0;
        for (int j = 0; j < lmax; ++j) rank += __shfl(c, j, 32) < c;   // pads hold INT_MAX
        if (hl < len) {
            col[b + rank] = c;
            val[b + rank] = v;
        }
        return;
    }
    tr_sort_row_wave(lane, __builtin_amdgcn_readlane(b, 0), len0, col, val);
    if (r0 + 1 < rows) tr_sort_row_wave(lane, __builtin_amdgcn_readlane(b, 32), len1, col, val);
}

__global__ void k_set_i32(int32_t *p, int32_t v) { *p = v; }

// Row heads of the transposed operator, compacted per group of 64 nodes (one
// wavefront, consecutive internal indices). Node m's head length is
//   hd(m) = max over its eight rows of min(row length, lw),
// and slot e of a group holds, in node order, one unit for each node of the
// group with hd > e: the eight rows' entry e (directions 1-4 and 5-8 as two
// 16-byte FP32 vectors, as the forward weights; zero weight and column m past
// a row's end). The group's slots follow one another from unit g * 64 * lw.
// A wavefront walking slots in order finds its units with a ballot: the
// active lanes of slot e are consecutive units, so every load is coalesced,
// and the lines fetched hold only nodes that use them. The 10-bit local
// columns of the inverse halo are compacted the same way over triples of
// slots (a node takes part in triple w when 3w < hd), from unit g * 64 * lw3.
// Number of lanes below this one whose bit is set in the wavefront mask.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Entry k (0..7) of unit r of a block of c units whose first unit is u0. A
// block is stored as two halves, entries 0-3 of its c units and then entries
// 4-7, so that a wavefront reads each half as one contiguous run.
__device__ __forceinline__ int64_t unit_entry(int64_t u0, int c, int r, int k) {
    return u0 * 8 + (int64_t)((k >> 2) * c + r) * 4 + (k & 3);
}

// Compacted copy of the first lw entries of every sorted CSR row, one
// wavefront per group of 64 nodes (lanes past the last node take part in the
// ballots with hd = 0). Slot by slot, each lane of a node with hd > e builds
// its unit: the eight rows' entry e, padded with (m, 0) past a row's end, and
// stores it as two 16-byte column vectors and two weight vectors. Consecutive
// active lanes hold consecutive units, so the stores are coalesced. A lane
// reads kEllChunk consecutive entries of a row back to back, so that the
// lines they share are used while they are still in the cache (one slot at a
// time, with every wavefront of a CU walking its own rows, they were not).
constexpr int kEllMaxLw = kMaxK + 4;
constexpr int kEllChunk = 8;
template <class T> struct Vec4;
template <> struct Vec4<float> { typedef float4 type; };
template <> struct Vec4<double> { typedef double __attribute__((ext_vector_type(4))) type; };

template <class T>
__global__ __launch_bounds__(256) void k_ell_fill(int n, int lw, const int32_t *__restrict__ ptr,
                                                  const int32_t *__restrict__ col,
                                                  const T *__restrict__ val,
                                                  int32_t *__restrict__ ecol, T *__restrict__ eval) {
    typedef typename Vec4<T>::type V4;
    const int lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t m0 = g * 64;
    if (m0 >= n) return;   // uniform across the wavefront
    const int m = (int)(m0 + lane);
    int b[8], len[8], hd = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        b[k] = len[k] = 0;
        if (m < n) {
            const int64_t row = (int64_t)k * n + m;
            b[k] = ptr[row];
            len[k] = ptr[row + 1] - b[k];
            hd = max(hd, min(len[k], lw));
        }
    }
    const int64_t g0 = g * 64 * lw;
    int64_t off = 0;
    for (int e0 = 0; e0 < lw; e0 += kEllChunk) {
        if (__ballot(e0 < hd) == 0) break;   // hd is fixed: no later slot has a unit
        int rk[kEllChunk], ck[kEllChunk];
#pragma unroll
        for (int t = 0; t < kEllChunk; ++t) {
            const uint64_t mask = __ballot(e0 + t < hd);
            rk[t] = lanes_below(mask);
            ck[t] = __popcll(mask);
        }
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            // the chunk's entries of the half's four rows, read row by row
            int cv[4][kEllChunk];
            T wv[4][kEllChunk];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 4 * hh + kk;
#pragma unroll
                for (int t = 0; t < kEllChunk; ++t) {
                    cv[kk][t] = m;
                    wv[kk][t] = (T)0;
                    if (e0 + t < len[k]) {
                        cv[kk][t] = col[b[k] + e0 + t];
                        wv[kk][t] = val[b[k] + e0 + t];
                    }
                }
            }
            int64_t u = off;
#pragma unroll
            for (int t = 0; t < kEllChunk; ++t) {
                if (e0 + t < hd) {
                    const int64_t at = unit_entry(g0 + u, ck[t], rk[t], 4 * hh);
                    *reinterpret_cast<int4 *>(ecol + at) =
                        make_int4(cv[0][t], cv[1][t], cv[2][t], cv[3][t]);
                    V4 vv;
                    vv[0] = wv[0][t];
                    vv[1] = wv[1][t];
                    vv[2] = wv[2][t];
                    vv[3] = wv[3][t];
                    *reinterpret_cast<V4 *>(eval + at) = vv;
                }
                u += ck[t];
            }
        }
#pragma unroll
        for (int t = 0; t < kEllChunk; ++t) off += ck[t];
    }
}

// Workgroup sum of one double per lane (NT lanes) into part[at].
template <int NT = 256>
__device__ __forceinline__ void block_sum_to(double v, double *part, int64_t at) {
    __shared__ double sh[NT];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[at] = sh[0];
}

__global__ __launch_bounds__(256) void k_sum_final(int64_t nparts, const double *__restrict__ part,
                                                   double *__restrict__ out, int accumulate) {
    __shared__ double sh[256];
    double a = 0.0;
    for (int64_t b = threadIdx.x; b < nparts; b += 256) a += part[b];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = accumulate ? *out + sh[0] : sh[0];
}

template <class T>
__device__ __forceinline__ void moments_of(const T *f, int n, int p, int dev, double rho0,
                                           T (&fk)[kQ], T &rho, T &ux, T &uy, T &drho) {
    T r = 0, jx = 0, jy = 0;
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        fk[k] = f[(int64_t)k * n + p];
        r += fk[k];
        jx += fk[k] * (T)lat_ex(k);
        jy += fk[k] * (T)lat_ey(k);
    }
    rho = dev ? (T)rho0 + r : r;
    drho = dev ? r : r - (T)rho0;
    ux = jx / rho;
    uy = jy / rho;
}

// Inverse halo of a tile of source nodes: every arriving node that the head
// (first lw entries) of the transposed rows of the tile's nodes reads, sorted
// (LDS hash set, then a bitonic network), capped at cap. The slot-major
// columns of those rows are rewritten as positions in that set, three 10-bit
// fields per word: word w of row k of node m (compacted like the heads, over
// triples of slots) holds slots 3w, 3w+1, 3w+2; fields past the end of the
// row are 0.
constexpr int kAHash = 4096;

__device__ void bitonic_sort_a(int *a, int npow2) {
    for (int k = 2; k <= npow2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < npow2; i += blockDim.x) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const bool up = (i & k) == 0;
                    const int ai = a[i], aj = a[ixj];
                    if ((ai > aj) == up) {
                        a[i] = aj;
                        a[ixj] = ai;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ int lower_bound_a(const int *a, int len, int v) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(1024) void k_adj_tiles(int n, int lw, int hcap, int cap,
                                                    const int32_t *__restrict__ ptr,
                                                    const int32_t *__restrict__ col,
                                                    const int32_t *__restrict__ ecol,
                                                    int32_t *__restrict__ tdescT,
                                                    int32_t *__restrict__ ilist,
                                                    uint32_t *__restrict__ elocal,
                                                    int32_t *__restrict__ stats) {
    __shared__ int hset[kAHash];
    __shared__ int hsorted[kAHash];
    __shared__ int s_n, s_over, s_fill;
    const int t = blockIdx.x, tid = threadIdx.x;
    const int base = t * kTile, cnt = min(kTile, n - base);
    const int lw3 = (lw + 2) / 3;
    for (int i = tid; i < kAHash; i += blockDim.x) hset[i] = -1;
    if (tid == 0) {
        s_n = 0;
        s_over = 0;
        s_fill = 0;
    }
    __syncthreads();
    for (int e = tid; e < 8 * cnt * lw; e += blockDim.x) {
        const int k0 = e / (cnt * lw), r = e - k0 * cnt * lw;
        const int l = r / lw, sl = r - l * lw;
        const int m = base + l;
        const int64_t row = (int64_t)k0 * n + m;
        if (sl >= ptr[row + 1] - ptr[row]) continue;
        const int q = col[ptr[row] + sl];
        uint32_t h = ((uint32_t)q * 2654435761u) >> 20;
        for (int probe = 0; probe < kAHash; ++probe) {
            const int old = atomicCAS(&hset[h], -1, q);
            if (old == -1) {
                atomicAdd(&s_n, 1);
                break;
            }
            if (old == q) break;
            h = (h + 1) & (kAHash - 1);
            if (probe == kAHash - 1) atomicOr(&s_over, 1);
        }
    }
    __syncthreads();
    const int ni = s_n;
    const bool fits = !s_over && ni <= cap && cap <= hcap && cap <= 1024;
    if (fits) {
        for (int i = tid; i < kAHash; i += blockDim.x) hsorted[i] = INT_MAX;
        __syncthreads();
        for (int i = tid; i < kAHash; i += blockDim.x) {
            const int v = hset[i];
            if (v != -1) hsorted[atomicAdd(&s_fill, 1)] = v;
        }
        __syncthreads();
        int np2 = 1;
        while (np2 < ni) np2 <<= 1;
        bitonic_sort_a(hsorted, np2);
        for (int h = tid; h < ni; h += blockDim.x) ilist[(int64_t)t * hcap + h] = hsorted[h];
        // local columns, one lane per node of the tile (the first four
        // wavefronts, one per group of 64 nodes): the columns come from the
        // compacted heads, slot by slot (contiguous over the lanes; the rows
        // themselves would be read with a stride across the lanes, triple
        // after triple), and each lane stores its unit's two halves
        if (tid < kTile) {
            typedef int32_t I4 __attribute__((ext_vector_type(4)));
            typedef uint32_t U4 __attribute__((ext_vector_type(4)));
            const int m = base + tid;
            int len[8], hd = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                len[k] = 0;
                if (m < n) {
                    const int64_t row = (int64_t)k * n + m;
                    len[k] = ptr[row + 1] - ptr[row];
                    hd = max(hd, min(len[k], lw));
                }
            }
            const int64_t g0 = (int64_t)(m >> 6) * 64 * lw3;   // words of the group
            const int64_t gv = (int64_t)(m >> 6) * 64 * lw;    // heads of the group
            int64_t off = 0, voff = 0;
            for (int w = 0; w < lw3; ++w) {
                const bool on = 3 * w < hd;
                const uint64_t mask = __ballot(on);
                if (mask == 0) break;
                U4 wa = (U4)0, wb = (U4)0;
#pragma unroll
                for (int sft = 0; sft < 3; ++sft) {
                    const int sl = 3 * w + sft;
                    const bool ons = sl < hd;
                    const uint64_t ms = __ballot(ons);
                    const int cs = __popcll(ms);
                    if (ons) {
                        const int rs = lanes_below(ms);
                        const int32_t *u = ecol + unit_entry(gv + voff, cs, rs, 0);
                        const I4 ca = *reinterpret_cast<const I4 *>(u);
                        const I4 cb = *reinterpret_cast<const I4 *>(u + 4 * cs);
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            if (sl < len[k])
                                wa[k] |= (uint32_t)lower_bound_a(hsorted, ni, ca[k]) << (10 * sft);
                            if (sl < len[k + 4])
                                wb[k] |= (uint32_t)lower_bound_a(hsorted, ni, cb[k]) << (10 * sft);
                        }
                    }
                    voff += cs;
                }
                if (on) {
                    const int r = lanes_below(mask), c = __popcll(mask);
                    *reinterpret_cast<U4 *>(elocal + unit_entry(g0 + off, c, r, 0)) = wa;
                    *reinterpret_cast<U4 *>(elocal + unit_entry(g0 + off, c, r, 4)) = wb;
                }
                off += __popcll(mask);
            }
        }
    }
    if (tid == 0) {
        tdescT[t] = fits ? ni : 0;
        if (fits) atomicMax(&stats[0], ni);
        else atomicAdd(&stats[1], 1);
    }
}

// lam_n = C'(f^n)^T (S^T lam_next); part[block] = sum of (S^T lam).(dC/dtau).
//   d feq_a / d rho = w_a [1 - 4.5 (e_a.u)^2 + 1.5 u^2]
//   d feq_a / d j   = w_a [3 e_a + 9 (e_a.u) e_a - 3 u]
//   C_a = f_a - (f_a - feq_a)/tau, so
//   lam_b = (1 - 1/tau) lg_b + (1/tau) (A + B . e_b),
//   A = sum_a lg_a d feq_a / d rho, B = sum_a lg_a d feq_a / d j,
//   d C_a / d tau = (f_a - feq_a) / tau^2.
// One workgroup per tile of source nodes. Tiles with an inverse halo stage
// lam_next of that halo in LDS and read the row heads through local indices;
// other tiles (and the rare row tails beyond lw entries) read global memory.
// Every row is summed in its sorted order, so both paths give identical sums.
// Two wavefronts per group of 64 source nodes (512 threads per tile):
// wavefront 2g + h walks group g's units for directions 1-4 (h = 0) or 5-8
// (h = 1) and loads only its half of each unit (each half is one contiguous
// run per slot block), which doubles the wavefronts that keep loads in flight.
// Both take the same ballots (over the longest of the node's eight rows),
// exchange their four row sums through LDS and finish the node together:
// h = 0 reads f^n, passes its moments over and stores lambda_0..4 and the
// tau partial, h = 1 stores lambda_5..8.
template <class T>
__global__ __launch_bounds__(2 * kTile) void k_adj_step(
    int n, const T *__restrict__ fn, const T *__restrict__ lam_next, T *__restrict__ lam_n,
    const int32_t *__restrict__ ptr, const int32_t *__restrict__ col, const T *__restrict__ val,
    int lw, const int32_t *__restrict__ ecol, const T *__restrict__ eval,
    const int32_t *__restrict__ tdescT, const int32_t *__restrict__ ilist,
    const uint32_t *__restrict__ elocal, int hcap, double rtau, double rho0, int dev,
    double *__restrict__ part, int32_t *err) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ T s_x[kTile / 64][2][4][64];   // row sums exchanged between the halves
    __shared__ T s_m[kTile / 64][4][64];      // moments of f^n, from half 0 to half 1
    __shared__ int s_hd[kTile / 64][2][64];   // head length over each half's rows
    typedef T T4 __attribute__((ext_vector_type(4)));
    typedef uint32_t U4 __attribute__((ext_vector_type(4)));
    typedef int32_t I4 __attribute__((ext_vector_type(4)));
    const int64_t ntiles = ((int64_t)n + kTile - 1) / kTile;
    const int64_t tt = xcd_tile(ntiles);
    if (tt >= ntiles) return;
    const int t = (int)tt, tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63;
    const int hv = wv & 1, gq = wv >> 1;    // direction half, group within the tile
    const int m = t * kTile + gq * 64 + lane;
    const int ni = tdescT ? tdescT[t] : 0;
    T *L = reinterpret_cast<T *>(smem);   // [8][ni]

    T acc[4] = {0, 0, 0, 0};   // rows 4 hv + i
    // each half reads its own four row lengths; the head length over all
    // eight is exchanged across the staging barrier
    int hmax = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (m < n) {
            const int64_t row = (int64_t)(4 * hv + i) * n + m;
            hmax = max(hmax, min(ptr[row + 1] - ptr[row], lw));
        }
    }
    s_hd[gq][hv][lane] = hmax;
    // The heads are compacted per group of 64 nodes: slot e holds one unit
    // for each node with hmax > e (ballot and masked bit count give a lane's
    // unit), slots past a row's end hold weight 0, and a triple of slots is
    // loaded together, non-temporal (the heads are streamed once per step and
    // need not displace the lambda rows from L2); fetching one triple ahead
    // measured slower. A lane past its head (or past the last node) reads its
    // group's first unit (a line the group fetches anyway; one shared address
    // for all such lanes would be a hot spot) and adds nothing: its weights
    // are zeroed and its local columns point at position 0.
    const T4 *ev = reinterpret_cast<const T4 *>(eval);
    const U4 *elw = reinterpret_cast<const U4 *>(elocal);
    const int lw3 = (lw + 2) / 3;
    const int64_t grp = min(m, n - 1) >> 6;   // lanes past the last node: its group
    const int64_t gv = grp * 64 * lw, gw = grp * 64 * lw3;
    int64_t voff = 0, woff = 0;
    if (ni > 0) {
        const int32_t *il = ilist + (int64_t)t * hcap;
        for (int h = tid; h < ni; h += 2 * kTile) {
            int q = il[h];
            if ((unsigned)q >= (unsigned)n) {   // a bad table must not fault
                q = 0;
                report_index(err);
            }
#pragma unroll
            for (int k = 1; k < kQ; ++k) L[(k - 1) * ni + h] = lam_next[(int64_t)k * n + q];
        }
    }
    __syncthreads();
    hmax = max(hmax, s_hd[gq][1 - hv][lane]);
    int wmax = hmax;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) wmax = max(wmax, __shfl_xor(wmax, off));
    const int ntrip = (wmax + 2) / 3;
    if (ni > 0) {
        const T *Lh = L + 4 * hv * ni;
        for (int w = 0; w < ntrip; ++w) {
            const bool onw = 3 * w < hmax;
            const uint64_t mw = __ballot(onw);
            const int cw = __popcll(mw);
            const int64_t aw = onw ? 2 * (gw + woff) + lanes_below(mw) + hv * cw : 2 * gw;
            U4 wd = __builtin_nontemporal_load(elw + aw);
            wd = onw ? wd : (U4)0;
            woff += cw;
            T4 v[3];
#pragma unroll
            for (int sft = 0; sft < 3; ++sft) {
                const bool on = 3 * w + sft < hmax;
                const uint64_t me = __ballot(on);
                const int ce = __popcll(me);
                const int64_t a = on ? 2 * (gv + voff) + lanes_below(me) + hv * ce : 2 * gv;
                const T4 va = __builtin_nontemporal_load(ev + a);
                v[sft] = on ? va : (T4)0;
                voff += ce;
            }
#pragma unroll
            for (int sft = 0; sft < 3; ++sft) {
                const int sh = 10 * sft;
                acc[0] += v[sft].x * Lh[0 * ni + ((wd.x >> sh) & 1023u)];
                acc[1] += v[sft].y * Lh[1 * ni + ((wd.y >> sh) & 1023u)];
                acc[2] += v[sft].z * Lh[2 * ni + ((wd.z >> sh) & 1023u)];
                acc[3] += v[sft].w * Lh[3 * ni + ((wd.w >> sh) & 1023u)];
            }
        }
    }
    if (m < n) {
        if (ni == 0) {
            const I4 *ec = reinterpret_cast<const I4 *>(ecol);
            const T *lk = lam_next + (int64_t)(1 + 4 * hv) * n;
            for (int e = 0; e < lw; ++e) {
                const bool on = e < hmax;
                const uint64_t me = __ballot(on);
                if (me == 0) break;
                const int ce = __popcll(me);
                const int64_t a = on ? 2 * (gv + voff) + lanes_below(me) + hv * ce : 2 * gv;
                const T4 va = on ? ev[a] : (T4)0;
                const I4 ca = ec[a];
                acc[0] += va.x * lk[0 * (int64_t)n + ca.x];
                acc[1] += va.y * lk[1 * (int64_t)n + ca.y];
                acc[2] += va.z * lk[2 * (int64_t)n + ca.z];
                acc[3] += va.w * lk[3 * (int64_t)n + ca.w];
                voff += ce;
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * hv + i;
            const T *lk = lam_next + (int64_t)(k + 1) * n;
            const int64_t row = (int64_t)k * n + m;
            const int b0 = ptr[row], b1 = ptr[row + 1];
            for (int e = b0 + lw; e < b1; ++e) acc[i] += val[e] * lk[col[e]];
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) s_x[gq][hv][i][lane] = acc[i];
    T fk[kQ], rho = 0, ux = 0, uy = 0, drho = 0;
    if (hv == 0 && m < n) {
        moments_of<T>(fn, n, m, dev, rho0, fk, rho, ux, uy, drho);
        s_m[gq][0][lane] = rho;
        s_m[gq][1][lane] = ux;
        s_m[gq][2][lane] = uy;
        s_m[gq][3][lane] = drho;
    }
    __syncthreads();
    double dt = 0.0;
    if (m < n) {
        T lg[kQ];
        lg[0] = lam_next[m];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            lg[1 + i] = hv ? s_x[gq][0][i][lane] : acc[i];
            lg[5 + i] = hv ? acc[i] : s_x[gq][1][i][lane];
        }
        if (hv) {
            rho = s_m[gq][0][lane];
            ux = s_m[gq][1][lane];
            uy = s_m[gq][2][lane];
            drho = s_m[gq][3][lane];
        }
        const T uu = ux * ux + uy * uy;
        T A = 0, Bx = 0, By = 0;
        double dtl = 0.0;
#pragma unroll
        for (int a = 0; a < kQ; ++a) {
            const T ex = (T)lat_ex(a), ey = (T)lat_ey(a);
            const T eu = ex * ux + ey * uy;
            const T wl = lat_wmul(a, lg[a]);
            A += wl * ((T)1 - (T)4.5 * eu * eu + (T)1.5 * uu);
            Bx += wl * ((T)3 * ex + (T)9 * eu * ex - (T)3 * ux);
            By += wl * ((T)3 * ey + (T)9 * eu * ey - (T)3 * uy);
            if (hv == 0) {   // the tau partial, from the half that holds f^n
                const T poly = (T)3 * eu + (T)4.5 * eu * eu - (T)1.5 * uu;
                const T fneq = dev ? fk[a] - lat_wmul(a, drho + rho * poly)
                                   : fk[a] - lat_wmul(a, rho * ((T)1 + poly));
                dtl += (double)lg[a] * (double)fneq;
            }
        }
        dt = hv ? 0.0 : dtl * rtau * rtau;
        const T rt = (T)rtau;
        const int b0 = hv ? 5 : 0, b1 = hv ? kQ : 5;
#pragma unroll
        for (int b = 0; b < kQ; ++b)
            if (b >= b0 && b < b1)
                lam_n[(int64_t)b * n + m] =
                    ((T)1 - rt) * lg[b] + rt * (A + Bx * (T)lat_ex(b) + By * (T)lat_ey(b));
    }
    block_sum_to<2 * kTile>(dt, part, t);
}

// dJ/df_b for J = 1/2 sum |u - u*|^2: (r . (e_b - u)) / rho, r = u - u*.
template <class T>
__global__ __launch_bounds__(256) void k_loss_seed(int n, const int32_t *__restrict__ perm,
                                                   const T *__restrict__ fT,
                                                   const double *__restrict__ uxt,
                                                   const double *__restrict__ uyt,
                                                   T *__restrict__ lam, double rho0, int dev,
                                                   double *__restrict__ part) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    double jl = 0.0;
    if (p < n) {
        T fk[kQ], rho, ux, uy, drho;
        moments_of<T>(fT, n, p, dev, rho0, fk, rho, ux, uy, drho);
        const int u = perm[p];
        const double rx = (double)ux - uxt[u], ry = (double)uy - uyt[u];
        jl = 0.5 * (rx * rx + ry * ry);
#pragma unroll
        for (int b = 0; b < kQ; ++b)
            lam[(int64_t)b * n + p] =
                (T)((rx * ((double)lat_ex(b) - (double)ux) + ry * ((double)lat_ey(b) - (double)uy)) /
                    (double)rho);
    }
    block_sum_to(jl, part, blockIdx.x);
}

// dJ/du0 = sum_k lam_k d feq_k(rho0, u0) / d u0.
template <class T>
__global__ void k_init_adjoint(int n, const int32_t *__restrict__ perm,
                               const double *__restrict__ u0x, const double *__restrict__ u0y,
                               const T *__restrict__ lam, double rho0, double *__restrict__ gx,
                               double *__restrict__ gy) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int u = perm[p];
    const double ux = u0x ? u0x[u] : 0.0, uy = u0y ? u0y[u] : 0.0;
    double sx = 0.0, sy = 0.0;
    for (int k = 0; k < kQ; ++k) {
        const double l = (double)lam[(int64_t)k * n + p];
        const double eu = lat_ex(k) * ux + lat_ey(k) * uy;
        sx += l * lat_w(k) * rho0 * (3.0 * lat_ex(k) + 9.0 * eu * lat_ex(k) - 3.0 * ux);
        sy += l * lat_w(k) * rho0 * (3.0 * lat_ey(k) + 9.0 * eu * lat_ey(k) - 3.0 * uy);
    }
    gx[u] = sx;
    gy[u] = sy;
}

}  // namespace

size_t transpose_temp_bytes(int n, int K) {
    (void)K;
    const size_t rows = (size_t)8 * n;
    return ((rows * sizeof(int32_t) + 255) & ~size_t(255)) + scan_temp_bytes((int)rows) + 256;
}

hipError_t launch_transpose(const CloudPlan &cp, int precision, void *tmp, size_t tmp_bytes,
                            hipStream_t s) {
    const int n = cp.n, K = cp.K, mode = cp.prm.stencil_mode;
    const int64_t rows = (int64_t)8 * n;
    int32_t *cnt = (int32_t *)tmp;
    const size_t cnt_bytes = ((size_t)rows * sizeof(int32_t) + 255) & ~size_t(255);
    void *scan_tmp = (char *)tmp + cnt_bytes;
    const size_t scan_bytes = tmp_bytes - cnt_bytes;
    hipError_t e = launch_fill_i32(cnt, 0, rows, s);
    if (e != hipSuccess) return e;
    if (n >= (1 << 29)) return hipErrorInvalidValue;   // hash keys 4 n + m in 32 bits
    // tiles of 256 arriving nodes (neighbouring tiles on one XCD, whose L2
    // then merges the runs they write into shared rows) x half of the directions
    const dim3 egrid(xcd_grid(blocks_for(n, 256)), 2);
    hipLaunchKernelGGL(k_tr_count, egrid, dim3(256), 0, s, n, K, mode, cp.nbr, cp.owner, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = exclusive_scan(scan_tmp, scan_bytes, cnt, cp.tr_ptr, (int)rows, s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, cp.tr_ptr + rows,
                       (int32_t)(rows * K));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_fill_i32(cnt, 0, rows, s)) != hipSuccess) return e;
    // staging of the fill: TT K entries of a tile (column, place, weight),
    // 128 nodes a tile while they take at most 46 KiB (with the hash table,
    // under 64 KiB), else 64
    const size_t esz = precision == MLBM_FP64 ? sizeof(double) : sizeof(float);
    auto stage_bytes = [&](int tt) {
        return 2 * (((size_t)tt * K * 4 + 15) & ~size_t(15)) + (size_t)tt * K * esz;
    };
    const bool wide = stage_bytes(128) <= 46 * 1024;
    const unsigned lds = (unsigned)stage_bytes(wide ? 128 : 64);
    const dim3 fgrid(xcd_grid(blocks_for(n, wide ? 128 : 64)), 2);
    if (precision == MLBM_FP64) {
        if (wide)
            hipLaunchKernelGGL((k_tr_fill<double, 128>), fgrid, dim3(kTrJs * 128), lds, s, n, K, mode,
                               cp.nbr, cp.owner, (const float *)nullptr, cp.W64, cp.tr_ptr, cnt,
                               cp.tr_col, (double *)cp.tr_val);
        else
            hipLaunchKernelGGL((k_tr_fill<double, 64>), fgrid, dim3(kTrJs * 64), lds, s, n, K, mode,
                               cp.nbr, cp.owner, (const float *)nullptr, cp.W64, cp.tr_ptr, cnt,
                               cp.tr_col, (double *)cp.tr_val);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_tr_sort<double>, dim3(blocks_for(rows, 8)), dim3(256), 0, s, rows,
                           cp.tr_ptr, cp.tr_col, (double *)cp.tr_val);
    } else {
        if (wide)
            hipLaunchKernelGGL((k_tr_fill<float, 128>), fgrid, dim3(kTrJs * 128), lds, s, n, K, mode,
                               cp.nbr, cp.owner, cp.W32, (const double *)nullptr, cp.tr_ptr, cnt,
                               cp.tr_col, (float *)cp.tr_val);
        else
            hipLaunchKernelGGL((k_tr_fill<float, 64>), fgrid, dim3(kTrJs * 64), lds, s, n, K, mode,
                               cp.nbr, cp.owner, cp.W32, (const double *)nullptr, cp.tr_ptr, cnt,
                               cp.tr_col, (float *)cp.tr_val);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_tr_sort<float>, dim3(blocks_for(rows, 8)), dim3(256), 0, s, rows,
                           cp.tr_ptr, cp.tr_col, (float *)cp.tr_val);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_ell_fill(cp, precision, s);
}

hipError_t launch_ell_fill(const CloudPlan &cp, int precision, hipStream_t s) {
    if (cp.tr_lw > kEllMaxLw) return hipErrorInvalidValue;
    const dim3 grid(blocks_for(cp.n, 256)), block(256);
    if (precision == MLBM_FP64)
        hipLaunchKernelGGL(k_ell_fill<double>, grid, block, 0, s, cp.n,
                           cp.tr_lw, cp.tr_ptr, cp.tr_col, (const double *)cp.tr_val, cp.ell_col,
                           (double *)cp.ell_val);
    else
        hipLaunchKernelGGL(k_ell_fill<float>, grid, block, 0, s, cp.n,
                           cp.tr_lw, cp.tr_ptr, cp.tr_col, (const float *)cp.tr_val, cp.ell_col,
                           (float *)cp.ell_val);
    return hipGetLastError();
}

hipError_t launch_loss_seed(const CloudPlan &cp, int precision, const void *fT,
                            const double *uxt, const double *uyt, void *lam, double *J,
                            double *part, hipStream_t s) {
    const int n = cp.n;
    const int64_t nb = blocks_for(n, 256);
    if (precision == MLBM_FP64)
        hipLaunchKernelGGL(k_loss_seed<double>, dim3(nb), dim3(256), 0, s, n, cp.perm,
                           (const double *)fT, uxt, uyt, (double *)lam, cp.prm.rho0, 0, part);
    else
        hipLaunchKernelGGL(k_loss_seed<float>, dim3(nb), dim3(256), 0, s, n, cp.perm,
                           (const float *)fT, uxt, uyt, (float *)lam, cp.prm.rho0, 1, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, nb, (const double *)part, J, 0);
    return hipGetLastError();
}

hipError_t launch_step_adjoint(const CloudPlan &cp, int precision, const void *fn,
                               const void *lam_next, void *lam_n, double *dtau, double *part,
                               hipStream_t s) {
    const int n = cp.n;
    const int64_t nb = blocks_for(n, 256);
    const double rtau = 1.0 / cp.prm.tau;
    const size_t esz = precision == MLBM_FP64 ? sizeof(double) : sizeof(float);
    const unsigned lds = cp.adj_ni ? (unsigned)(8 * cp.adj_ni * esz) : 0;
    const int32_t *td = cp.adj_ni ? cp.tdescT : nullptr;
    if (precision == MLBM_FP64)
        hipLaunchKernelGGL(k_adj_step<double>, dim3(xcd_grid(nb)), dim3(2 * kTile), lds, s, n,
                           (const double *)fn, (const double *)lam_next, (double *)lam_n,
                           cp.tr_ptr, cp.tr_col, (const double *)cp.tr_val, cp.tr_lw,
                           cp.ell_col, (const double *)cp.ell_val, td, cp.ilist, cp.elocal,
                           cp.hcap, rtau, cp.prm.rho0, 0, part, cp.err);
    else
        hipLaunchKernelGGL(k_adj_step<float>, dim3(xcd_grid(nb)), dim3(2 * kTile), lds, s, n,
                           (const float *)fn, (const float *)lam_next, (float *)lam_n,
                           cp.tr_ptr, cp.tr_col, (const float *)cp.tr_val, cp.tr_lw,
                           cp.ell_col, (const float *)cp.ell_val, td, cp.ilist, cp.elocal,
                           cp.hcap, rtau, cp.prm.rho0, 1, part, cp.err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, nb, (const double *)part, dtau, 1);
    return hipGetLastError();
}

hipError_t launch_init_adjoint(const CloudPlan &cp, int precision, const double *u0x,
                               const double *u0y, const void *lam0, double *gx, double *gy,
                               hipStream_t s) {
    const int n = cp.n;
    if (precision == MLBM_FP64)
        hipLaunchKernelGGL(k_init_adjoint<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n,
                           cp.perm, u0x, u0y, (const double *)lam0, cp.prm.rho0, gx, gy);
    else
        hipLaunchKernelGGL(k_init_adjoint<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n,
                           cp.perm, u0x, u0y, (const float *)lam0, cp.prm.rho0, gx, gy);
    return hipGetLastError();
}

hipError_t launch_adj_tiles(const CloudPlan &cp, int32_t *stats, hipStream_t s) {
    const int ntiles = (cp.n + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_adj_tiles, dim3(ntiles), dim3(1024), 0, s, cp.n, cp.tr_lw, cp.hcap,
                       cp.adj_cap, cp.tr_ptr, cp.tr_col, cp.ell_col, cp.tdescT, cp.ilist,
                       cp.elocal, stats);
    return hipGetLastError();
}

}  // namespace mlbm
