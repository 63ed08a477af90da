// Tile-local gather tables for the LDS-staged step kernel.
//
// The step kernel processes tiles of kTile consecutive nodes (Hilbert order,
// so a tile is a compact patch). For tile t it needs the post-collision
// populations of every stencil member of every owner used by the tile's
// departure points. This kernel (one workgroup per tile) computes
//   O_t: the sorted set of owners {owner_k(p) : p in tile, k = 1..8}
//        (the tile's own nodes in own-stencil mode),
//   H_t: the sorted set of stencil members {nbr[j][o] : o in O_t, j < K},
// and stores, with indices local to the tile,
//   ownerL[k][p]   = position of owner_k(p) in O_t (16 bit, paper mode),
//   nbrL[t][o][w]  = positions of nbr[j][O_t[o]] in H_t for j = 3w, 3w+1, 3w+2,
//                    packed as three 10-bit fields of one word (|H_t| <= 1024),
//   hlist[t][h]    = global index of H_t[h],
//   tdesc[t]       = (|O_t|, |H_t|), |H_t| = 0 marks a tile that does not fit
//                    the caps and is stepped with global gathers instead.
// H_t is collected in an LDS hash set (bounded linear probing), compacted and
// sorted by a bitonic network.
#include <climits>

#include "common.h"

namespace mlbm {
namespace {

constexpr int kOCand = 8 * kTile;   // owner candidates per tile
constexpr int kHashSize = 4096;     // LDS hash set for H_t (power of two)
constexpr int kEmpty = -1;

__device__ void bitonic_sort(int *a, int npow2) {
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

// Exclusive prefix sum of v over the workgroup (at most 16 wavefronts), and
// the sum of all v in `total`. Every thread of the workgroup must call it.
__device__ int block_scan_excl(int v, int *s_wsum, int &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_wsum[w] = x;
    __syncthreads();
    int before = 0, all = 0;
    for (int i = 0; i < nw; ++i) {
        const int c = s_wsum[i];
        before += i < w ? c : 0;
        all += c;
    }
    __syncthreads();
    total = all;
    return before + x - v;
}

// Position of v in the sorted array a[0..len) (v is present).
__device__ __forceinline__ int lower_bound(const int *a, int len, int v) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(1024) void k_tiles(int n, int K, int mode,
                                                const int32_t *__restrict__ nbr,
                                                const int32_t *__restrict__ owner, int ocap,
                                                int hcap, int32_t *__restrict__ tdesc,
                                                uint16_t *__restrict__ ownerL,
                                                uint32_t *__restrict__ nbrL,
                                                int32_t *__restrict__ hlist,
                                                int32_t *__restrict__ stats) {
    __shared__ int ocand[kOCand];
    __shared__ int hset[kHashSize];
    __shared__ int hsorted[kHashSize];
    __shared__ int s_no, s_nh, s_over, s_fill;
    __shared__ int s_wsum[16];
    static_assert(2 * 1024 == kOCand, "two owner candidates per thread");
    const int t = blockIdx.x;
    const int base = t * kTile;
    const int cnt = min(kTile, n - base);
    const int tid = threadIdx.x;

    // ---- O_t --------------------------------------------------------------
    if (mode == MLBM_STENCIL_OWN) {
        for (int i = tid; i < kOCand; i += blockDim.x) ocand[i] = i < cnt ? base + i : INT_MAX;
    } else {
        for (int i = tid; i < kOCand; i += blockDim.x) {
            const int k = i / kTile, l = i - k * kTile;
            ocand[i] = l < cnt ? owner[(int64_t)k * n + base + l] : INT_MAX;
        }
    }
    for (int i = tid; i < kHashSize; i += blockDim.x) hset[i] = kEmpty;
    if (tid == 0) {
        s_no = 0;
        s_nh = 0;
        s_over = 0;
        s_fill = 0;
    }
    __syncthreads();
    if (mode != MLBM_STENCIL_OWN) bitonic_sort(ocand, kOCand);
    // unique: thread tid keeps entries 2 tid and 2 tid + 1 where they differ
    // from their predecessor, and a block scan of the kept counts gives their
    // positions (compacted through hsorted, unused until H_t is sorted)
    {
        const int e0 = 2 * tid, v0 = ocand[e0], v1 = ocand[e0 + 1];
        const int k0 = v0 != INT_MAX && (e0 == 0 || ocand[e0 - 1] != v0);
        const int k1 = v1 != INT_MAX && v1 != v0;
        int total;
        const int pos = block_scan_excl(k0 + k1, s_wsum, total);
        if (k0) hsorted[pos] = v0;
        if (k1) hsorted[pos + k0] = v1;
        __syncthreads();
        for (int i = tid; i < total; i += blockDim.x) ocand[i] = hsorted[i];
        if (tid == 0) s_no = total;
        __syncthreads();
    }
    const int no = s_no;
    bool fits = no <= ocap;

    // ---- H_t through an LDS hash set ----------------------------------------
    if (fits) {
        for (int e = tid; e < no * K; e += blockDim.x) {
            const int o = e / K, j = e - o * K;
            const int q = nbr[(int64_t)j * n + ocand[o]];
            uint32_t h = ((uint32_t)q * 2654435761u) >> 20;   // 12-bit slot
            for (int probe = 0; probe < kHashSize; ++probe) {
                const int old = atomicCAS(&hset[h], kEmpty, q);
                if (old == kEmpty) {
                    atomicAdd(&s_nh, 1);
                    break;
                }
                if (old == q) break;
                h = (h + 1) & (kHashSize - 1);
                if (probe == kHashSize - 1) atomicOr(&s_over, 1);
            }
        }
    }
    __syncthreads();
    const int nh = s_nh;
    fits = fits && !s_over && nh <= hcap;
    if (fits) {
        // s_nh is read by every thread above; the compaction counts with its
        // own counter so that no shared value changes after it was read
        for (int i = tid; i < kHashSize; i += blockDim.x) hsorted[i] = INT_MAX;
        __syncthreads();
        for (int i = tid; i < kHashSize; i += blockDim.x) {
            const int v = hset[i];
            if (v != kEmpty) hsorted[atomicAdd(&s_fill, 1)] = v;
        }
        __syncthreads();
        int np2 = 1;
        while (np2 < nh) np2 <<= 1;
        bitonic_sort(hsorted, np2);
        // tables
        int32_t *hl = hlist + (int64_t)t * hcap;
        for (int h = tid; h < nh; h += blockDim.x) hl[h] = hsorted[h];
        const int Kw = (K + 2) / 3;
        uint32_t *nl = nbrL + (int64_t)t * ocap * Kw;
        for (int e = tid; e < no * Kw; e += blockDim.x) {
            const int o = e / Kw, w = e - o * Kw;
            uint32_t word = 0;
            for (int sft = 0; sft < 3; ++sft) {
                const int j = 3 * w + sft;
                if (j < K) {
                    const int q = nbr[(int64_t)j * n + ocand[o]];
                    word |= (uint32_t)lower_bound(hsorted, nh, q) << (10 * sft);
                }
            }
            nl[e] = word;
        }
        if (mode != MLBM_STENCIL_OWN) {
            for (int i = tid; i < 8 * cnt; i += blockDim.x) {
                const int k = i / cnt, l = i - k * cnt;
                const int q = owner[(int64_t)k * n + base + l];
                ownerL[(int64_t)k * n + base + l] = (uint16_t)lower_bound(ocand, no, q);
            }
        }
    }
    if (tid == 0) {
        tdesc[2 * t] = no;
        tdesc[2 * t + 1] = fits ? nh : 0;
        if (fits) {
            // LDS bytes of this tile in the step kernel: 8 directions x nh
            // populations (float) + no x ceil(K/3) index words
            atomicMax(&stats[0], 8 * nh * 4 + no * ((K + 2) / 3) * 4);
        } else {
            atomicAdd(&stats[1], 1);
        }
    }
}

}  // namespace

hipError_t launch_tiles(const CloudPlan &cp, int32_t *stats, hipStream_t s) {
    const int ntiles = (cp.n + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_tiles, dim3(ntiles), dim3(1024), 0, s, cp.n, cp.K, cp.prm.stencil_mode,
                       cp.nbr, cp.owner, cp.ocap, cp.hcap, cp.tdesc, cp.ownerL, cp.nbrL,
                       cp.hlist, stats);
    return hipGetLastError();
}

}  // namespace mlbm
