// Device kernels of the row-wise Gustavson SpGEMM C = A * B for gfx950.
//
// Method: FSpGEMM Sec. II-B (row-wise Gustavson, Fig. 1): row i of C is the
// merge of the scaled rows A(i,k) * B(k,:), equal column indices added, no
// zero test (Algorithm 1 adds on equal indices and emits every element).
//
// The FPGA design streams B rows to processing elements that sort-and-merge
// (Sec. IV-B3).  On CDNA4 the same sums are formed with per-row accumulators
// sized by a bound on the row's output:
//   * a symbolic pass counts row_nnz_i = |union of the column sets| with an
//     LDS hash of keys (sub-wave lane groups or whole workgroups per row) or
//     an n-bit bitmap for the largest rows;
//   * a numeric pass adds a_ik * b_kj into an LDS hash of (key, FP64 value)
//     sized by the exact row_nnz_i, then writes the row in column order (a
//     rank count for short rows, an LDS bitonic sort for long rows); rows
//     too large for LDS use a global dense FP64 accumulator whose bitmap is
//     scanned in column order, so they need no sort.
// Products of a row are enumerated "flattened": a lane group loads a chunk
// of A's row, prefix-sums the B-row lengths, and every lane takes the next
// product index and finds its A entry by binary search, so that the lanes
// stay busy whatever the B-row lengths are.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "types.hpp"

namespace msp {

// Multiplicative (Fibonacci) hashing: top log2(T) bits of key * 2^32/phi.
template <int T>
__device__ __forceinline__ uint32_t hash_slot(int32_t key) {
    constexpr int LOGT = __builtin_ctz(T);
    return (uint32_t)((uint32_t)key * 2654435761u) >> (32 - LOGT);
}

template <typename VT>
__device__ __forceinline__ double to_f64(VT v) { return (double)v; }

// Loads that must observe device-scope atomics performed by other lanes of
// the same workgroup (global dense accumulator): bypass the non-coherent L1.
__device__ __forceinline__ double load_coherent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_coherent(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Lane-group primitives (G lanes of one wave, G a power of two <= 64)
// ---------------------------------------------------------------------------

template <int G>
__device__ __forceinline__ long long group_incl_scan(long long x, int gl) {
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        long long y = __shfl_up(x, d, G);
        if (gl >= d) x += y;
    }
    return x;
}

template <int G>
__device__ __forceinline__ int group_sum(int x) {
#pragma unroll
    for (int d = G / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, G);
    return x;
}

template <int G>
__device__ __forceinline__ uint64_t group_ballot(bool p, int lane) {
    uint64_t b = __ballot(p);
    if constexpr (G == 64) return b;
    else return (b >> (lane & ~(G - 1))) & ((1ull << G) - 1);
}

// ---------------------------------------------------------------------------
// Workgroup primitives (BS threads)
// ---------------------------------------------------------------------------

template <int BS>
struct BlockScanSmem {
    long long wave_tot[BS / kWave];
};

// Inclusive scan over the workgroup; returns the inclusive value and sets
// *total.  Contains two __syncthreads.
template <int BS>
__device__ __forceinline__ long long block_incl_scan(long long x, BlockScanSmem<BS>& sm,
                                                     long long* total) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    long long v = group_incl_scan<kWave>(x, lane);
    if (lane == kWave - 1) sm.wave_tot[w] = v;
    __syncthreads();
    long long pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < BS / kWave; ++i) {
        long long t = sm.wave_tot[i];
        if (i < w) pre += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return v + pre;
}

template <int BS>
__device__ __forceinline__ long long block_sum(long long x, BlockScanSmem<BS>& sm) {
    long long t;
    block_incl_scan<BS>(x, sm, &t);
    return t;
}

// smallest t in [0, n) with off[t] > q (off inclusive, non-decreasing, off[n-1] > q)
template <typename OffT>
__device__ __forceinline__ int owner_search(const OffT* off, int n, long long q) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((long long)off[mid] > q) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// XCD-aware block order: blocks are dealt round-robin to the 8 XCDs, so
// block b runs on XCD b % 8.  Give XCD x the x-th contiguous eighth of the
// logical blocks so that neighbouring rows (which share B rows) meet in the
// same L2.  Requires gridDim.x % 8 == 0 (the host pads the grid).
__device__ __forceinline__ unsigned xcd_block() {
    const unsigned g = gridDim.x, b = blockIdx.x;
    if (g & 7u) return b;
    return (b & 7u) * (g >> 3) + (b >> 3);
}

// ===========================================================================
// Fill a small int buffer (graph-safe replacement for memset)
// ===========================================================================
static __global__ void k_zero_words(int* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// ===========================================================================
// Per-row statistics and symbolic binning
// ===========================================================================
//
// One wave per 64 consecutive rows.  Rows with at most kShortRow entries are
// summed by their own lane; longer rows are summed by the whole wave, one
// after another, so hub rows of power-law matrices do not serialise a lane.
// Outputs: u_i = min(prod_i, ncols(B)) (int32), optional int64 prod_i,
// optional min/max B-row length and column span, the per-bin histogram of
// u_i, the total product count, and row_nnz_i = 0 for rows with u_i = 0.

constexpr int kShortRow = 32;

template <bool FEAT>
__global__ void __launch_bounds__(256)
k_row_stats(int m, long long ncols, const int64_t* __restrict__ arp, const int32_t* __restrict__ acol,
            const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol,
            int32_t* __restrict__ u_out, int64_t* __restrict__ prod_out,
            int32_t* __restrict__ row_nnz, BinTable bins, DevInfo* info,
            float* __restrict__ feat) {
    __shared__ int hist[kMaxBins + 1];
    __shared__ long long prod_acc;
    if (threadIdx.x <= kMaxBins) hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) prod_acc = 0;
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const long long row = (long long)blockIdx.x * 256 + threadIdx.x;
    const bool valid = row < m;
    long long a0 = 0, a1 = 0;
    if (valid) { a0 = arp[row]; a1 = arp[row + 1]; }
    const long long len = a1 - a0;

    long long s = 0, mn = -1, mx = 0, lo = -1, hi = -1;
    if (valid && len <= kShortRow) {
        for (long long p = a0; p < a1; ++p) {
            const int32_t k = acol[p];
            const long long b0 = brp[k], b1 = brp[k + 1];
            const long long l = b1 - b0;
            s += l;
            if (FEAT) {
                mn = (mn < 0 || l < mn) ? l : mn;
                mx = l > mx ? l : mx;
                if (l > 0) {
                    const long long f = bcol[b0], e = bcol[b1 - 1];
                    lo = (lo < 0 || f < lo) ? f : lo;
                    hi = (hi < 0 || e > hi) ? e : hi;
                }
            }
        }
    }
    uint64_t longmask = __ballot(valid && len > kShortRow);
    while (longmask) {
        const int r = __builtin_ctzll(longmask);
        longmask &= longmask - 1;
        const long long ra0 = __shfl(a0, r), ra1 = __shfl(a1, r);
        long long ls = 0, lmn = -1, lmx = 0, llo = -1, lhi = -1;
        for (long long p = ra0 + lane; p < ra1; p += 64) {
            const int32_t k = acol[p];
            const long long b0 = brp[k], b1 = brp[k + 1];
            const long long l = b1 - b0;
            ls += l;
            if (FEAT) {
                lmn = (lmn < 0 || l < lmn) ? l : lmn;
                lmx = l > lmx ? l : lmx;
                if (l > 0) {
                    const long long f = bcol[b0], e = bcol[b1 - 1];
                    llo = (llo < 0 || f < llo) ? f : llo;
                    lhi = (lhi < 0 || e > lhi) ? e : lhi;
                }
            }
        }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) {
            ls += __shfl_xor(ls, d);
            if (FEAT) {
                long long o;
                o = __shfl_xor(lmn, d); lmn = (lmn < 0) ? o : ((o < 0) ? lmn : (o < lmn ? o : lmn));
                o = __shfl_xor(lmx, d); lmx = o > lmx ? o : lmx;
                o = __shfl_xor(llo, d); llo = (llo < 0) ? o : ((o < 0) ? llo : (o < llo ? o : llo));
                o = __shfl_xor(lhi, d); lhi = o > lhi ? o : lhi;
            }
        }
        if (lane == r) { s = ls; mn = lmn; mx = lmx; lo = llo; hi = lhi; }
    }

    if (valid) {
        const long long u = s < ncols ? s : ncols;
        u_out[row] = (int32_t)u;
        if (prod_out) prod_out[row] = s;
        if (u == 0 && row_nnz) row_nnz[row] = 0;
        atomicAdd(&hist[bin_of(bins, u)], 1);
        if (FEAT && feat) {
            const float n = (float)(ncols > 0 ? ncols : 1);
            const float fl = (float)len, fs = (float)s;
            const float mean = len > 0 ? (float)((double)s / (double)len) : 0.f;
            float* f = feat + row * 8;
            f[0] = log2f(1.f + fl);
            f[1] = log2f(1.f + fs);
            f[2] = log2f(1.f + (float)(mn < 0 ? 0 : mn));
            f[3] = log2f(1.f + mean);
            f[4] = log2f(1.f + (float)mx);
            f[5] = log2f(1.f + (float)ncols);
            f[6] = fminf(1.f, (float)((double)s / (double)n));
            f[7] = (float)((double)(lo < 0 ? 0 : hi - lo) / (double)n);
        }
    }
    // block total of products
    long long ws = s;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) ws += __shfl_xor(ws, d);
    if (lane == 0) atomicAdd((unsigned long long*)&prod_acc, (unsigned long long)ws);
    __syncthreads();
    if (threadIdx.x <= kMaxBins && hist[threadIdx.x]) {
        if (bins.nb > 0) atomicAdd(&info->sym_count[threadIdx.x], hist[threadIdx.x]);
    }
    if (threadIdx.x == 0 && prod_acc) atomicAdd((unsigned long long*)&info->total_prod, (unsigned long long)prod_acc);
}

// ===========================================================================
// Scatter row ids into per-bin lists
// ===========================================================================
// Bin b's rows go to perm[start_b ...], start_b = sum of the counts of the
// bins before it.  Rows of one workgroup reserve one range per bin with a
// single global atomic.
static __global__ void __launch_bounds__(256)
k_scatter(int m, const int32_t* __restrict__ key, BinTable bins, const int* __restrict__ counts,
          int* cursor, int32_t* __restrict__ perm) {
    __shared__ int cnt[kMaxBins + 1];
    __shared__ int base[kMaxBins + 1];
    if (threadIdx.x <= kMaxBins) cnt[threadIdx.x] = 0;
    __syncthreads();
    const long long row = (long long)blockIdx.x * 256 + threadIdx.x;
    int b = -1, r = 0;
    if (row < m) {
        b = bin_of(bins, key[row]);
        r = atomicAdd(&cnt[b], 1);
    }
    __syncthreads();
    if (threadIdx.x <= bins.nb && cnt[threadIdx.x]) {
        int start = 0;
        for (int i = 0; i < (int)threadIdx.x; ++i) start += counts[i];
        base[threadIdx.x] = start + atomicAdd(&cursor[threadIdx.x], cnt[threadIdx.x]);
    }
    __syncthreads();
    if (b >= 0) perm[base[b] + r] = (int32_t)row;
}

// ===========================================================================
// Symbolic pass
// ===========================================================================

// Insert key j into an LDS key table of T slots; returns 1 if it was new.
// Linear probing; the table holds at most T/2 keys by construction, the
// probe bound is a guard that reports instead of spinning.
template <int T>
__device__ __forceinline__ int hash_insert_key(int32_t* keys, int32_t j, int* err) {
    uint32_t h = hash_slot<T>(j);
    for (int probe = 0; probe < T; ++probe) {
        int32_t k = keys[h];
        if (k == j) return 0;
        if (k == kEmpty) {
            int32_t old = atomicCAS(&keys[h], kEmpty, j);
            if (old == kEmpty) return 1;
            if (old == j) return 0;
        }
        h = (h + 1) & (T - 1);
    }
    *err = 1;
    return 0;
}

// Slot of key j in an LDS (key, value) table, inserting it if absent.
template <int T>
__device__ __forceinline__ int hash_slot_of(int32_t* keys, int32_t j, int* err) {
    uint32_t h = hash_slot<T>(j);
    for (int probe = 0; probe < T; ++probe) {
        int32_t k = keys[h];
        if (k == j) return (int)h;
        if (k == kEmpty) {
            int32_t old = atomicCAS(&keys[h], kEmpty, j);
            if (old == kEmpty || old == j) return (int)h;
        }
        h = (h + 1) & (T - 1);
    }
    *err = 1;
    return -1;
}

// Rows per workgroup for a lane-group kernel of G lanes.
template <int G>
struct GroupCfg {
    static constexpr int BS = 256;
    static constexpr int NG = BS / G;
};

// Symbolic, sub-wave lane groups: G lanes per row, T key slots per row.
// rows = perm (bin list) or identity when perm == nullptr.
template <int G, int T>
__global__ void __launch_bounds__(256)
k_sym_group(int nrows_bin, const int32_t* __restrict__ perm, int m,
            const int64_t* __restrict__ arp, const int32_t* __restrict__ acol,
            const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol,
            int32_t* __restrict__ row_nnz, DevInfo* info) {
    constexpr int NG = GroupCfg<G>::NG;
    __shared__ int32_t keys[NG][T];
    __shared__ long long s_off[NG][G];
    __shared__ long long s_bst[NG][G];
    const int lane = threadIdx.x & 63;
    const int gl = threadIdx.x & (G - 1);
    const int g = threadIdx.x / G;
    const long long slot = (long long)xcd_block() * NG + g;
    if (slot >= nrows_bin) return;               // group-uniform
    const int row = perm ? perm[slot] : (int)slot;
    (void)lane;
    int err = 0;
    int32_t* kt = keys[g];
#pragma unroll
    for (int s = gl; s < T; s += G) kt[s] = kEmpty;
    lds_fence();
    const long long a0 = arp[row], a1 = arp[row + 1];
    int cnt = 0;
    for (long long c0 = a0; c0 < a1; c0 += G) {
        const long long p = c0 + gl;
        long long len = 0, bst = 0;
        if (p < a1) {
            const int32_t k = acol[p];
            bst = brp[k];
            len = brp[k + 1] - bst;
        }
        const long long incl = group_incl_scan<G>(len, gl);
        const long long total = __shfl(incl, G - 1, G);
        s_off[g][gl] = incl;
        s_bst[g][gl] = bst - (incl - len);
        lds_fence();
        const int nact = (int)((a1 - c0) < G ? (a1 - c0) : G);
        for (long long q = gl; q < total; q += G) {
            const int t = owner_search(s_off[g], nact, q);
            const int32_t j = bcol[s_bst[g][t] + q];
            cnt += hash_insert_key<T>(kt, j, &err);
        }
        lds_fence();
    }
    cnt = group_sum<G>(cnt);
    if (gl == 0) row_nnz[row] = cnt;
    if (err) atomicOr(&info->err, kErrProbe);
}

// Symbolic, one workgroup of BS threads per row, T key slots (LDS).
template <int BS, int T>
__global__ void __launch_bounds__(BS)
k_sym_block(int nrows_bin, const int32_t* __restrict__ perm,
            const int64_t* __restrict__ arp, const int32_t* __restrict__ acol,
            const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol,
            int32_t* __restrict__ row_nnz, DevInfo* info) {
    __shared__ int32_t keys[T];
    __shared__ long long s_off[BS];
    __shared__ long long s_bst[BS];
    __shared__ BlockScanSmem<BS> sm;
    const int tid = threadIdx.x;
    int err = 0;
    for (long long slot = blockIdx.x; slot < nrows_bin; slot += gridDim.x) {
        const int row = perm ? perm[slot] : (int)slot;
        for (int s = tid; s < T; s += BS) keys[s] = kEmpty;
        __syncthreads();
        const long long a0 = arp[row], a1 = arp[row + 1];
        long long cnt = 0;
        for (long long c0 = a0; c0 < a1; c0 += BS) {
            const long long p = c0 + tid;
            long long len = 0, bst = 0;
            if (p < a1) {
                const int32_t k = acol[p];
                bst = brp[k];
                len = brp[k + 1] - bst;
            }
            long long total;
            const long long incl = block_incl_scan<BS>(len, sm, &total);
            s_off[tid] = incl;
            s_bst[tid] = bst - (incl - len);
            __syncthreads();
            const int nact = (int)((a1 - c0) < BS ? (a1 - c0) : BS);
            for (long long q = tid; q < total; q += BS) {
                const int t = owner_search(s_off, nact, q);
                const int32_t j = bcol[s_bst[t] + q];
                cnt += hash_insert_key<T>(keys, j, &err);
            }
            __syncthreads();
        }
        const long long tot = block_sum<BS>(cnt, sm);
        if (tid == 0) row_nnz[row] = (int32_t)tot;
        __syncthreads();
    }
    if (err) atomicOr(&info->err, kErrProbe);
}

// Symbolic for the largest rows: an n-bit bitmap (LDS when it fits, else a
// per-workgroup global slab), counting bits that an atomic OR newly sets.
template <int BS, bool LDSBM>
__global__ void __launch_bounds__(BS)
k_sym_bitmap(int nrows_bin, const int32_t* __restrict__ perm, long long ncols,
             const int64_t* __restrict__ arp, const int32_t* __restrict__ acol,
             const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol,
             int32_t* __restrict__ row_nnz, uint32_t* gslab, DevInfo* info) {
    extern __shared__ uint32_t dyn_smem[];
    __shared__ long long s_off[BS];
    __shared__ long long s_bst[BS];
    __shared__ BlockScanSmem<BS> sm;
    const int tid = threadIdx.x;
    const long long words = (ncols + 31) >> 5;
    uint32_t* bm = LDSBM ? dyn_smem : gslab + (long long)blockIdx.x * words;
    for (long long slot = blockIdx.x; slot < nrows_bin; slot += gridDim.x) {
        const int row = perm ? perm[slot] : (int)slot;
        for (long long w = tid; w < words; w += BS) bm[w] = 0u;
        if (!LDSBM) __threadfence();
        __syncthreads();
        const long long a0 = arp[row], a1 = arp[row + 1];
        long long cnt = 0;
        for (long long c0 = a0; c0 < a1; c0 += BS) {
            const long long p = c0 + tid;
            long long len = 0, bst = 0;
            if (p < a1) {
                const int32_t k = acol[p];
                bst = brp[k];
                len = brp[k + 1] - bst;
            }
            long long total;
            const long long incl = block_incl_scan<BS>(len, sm, &total);
            s_off[tid] = incl;
            s_bst[tid] = bst - (incl - len);
            __syncthreads();
            const int nact = (int)((a1 - c0) < BS ? (a1 - c0) : BS);
            for (long long q = tid; q < total; q += BS) {
                const int t = owner_search(s_off, nact, q);
                const int32_t j = bcol[s_bst[t] + q];
                const uint32_t bit = 1u << (j & 31);
                const uint32_t old = atomicOr(&bm[j >> 5], bit);
                cnt += (old & bit) ? 0 : 1;
            }
            __syncthreads();
        }
        const long long tot = block_sum<BS>(cnt, sm);
        if (tid == 0) row_nnz[row] = (int32_t)tot;
        __syncthreads();
    }
    (void)info;
}

// ===========================================================================
// Exclusive prefix sum of row_nnz -> row_ptr (int64), fused with the
// numeric binning histogram.  Three kernels: tile sums, a scan of the tile
// sums in one workgroup, and the tile scans with their offsets.
// ===========================================================================
constexpr int kScanBS = 1024;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanBS * kScanPer;

static __global__ void __launch_bounds__(kScanBS)
k_scan_tiles(int m, const int32_t* __restrict__ cnt, long long* __restrict__ tile_sum) {
    __shared__ BlockScanSmem<kScanBS> sm;
    const long long base = (long long)blockIdx.x * kScanTile;
    long long s = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        const long long r = base + (long long)i * kScanBS + threadIdx.x;
        if (r < m) s += cnt[r];
    }
    const long long t = block_sum<kScanBS>(s, sm);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = t;
}

static __global__ void __launch_bounds__(kScanBS)
k_scan_tile_sums(int ntiles, long long* __restrict__ tile_sum, DevInfo* info) {
    __shared__ BlockScanSmem<kScanBS> sm;
    long long carry = 0;
    for (int c0 = 0; c0 < ntiles; c0 += kScanBS) {
        const int i = c0 + threadIdx.x;
        const long long v = i < ntiles ? tile_sum[i] : 0;
        long long tot;
        const long long incl = block_incl_scan<kScanBS>(v, sm, &tot);
        if (i < ntiles) tile_sum[i] = carry + incl - v;   // exclusive
        carry += tot;
    }
    if (threadIdx.x == 0) info->nnz = carry;
}

static __global__ void __launch_bounds__(kScanBS)
k_scan_apply(int m, const int32_t* __restrict__ cnt, const long long* __restrict__ tile_off,
             int64_t* __restrict__ row_ptr, BinTable bins, DevInfo* info) {
    __shared__ BlockScanSmem<kScanBS> sm;
    __shared__ int hist[kMaxBins + 1];
    if (threadIdx.x <= kMaxBins) hist[threadIdx.x] = 0;
    const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanPer;
    int v[kScanPer];
    long long s = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        const long long r = base + i;
        v[i] = r < m ? cnt[r] : 0;
        s += v[i];
    }
    long long tot;
    const long long incl = block_incl_scan<kScanBS>(s, sm, &tot);   // has __syncthreads
    long long run = tile_off[blockIdx.x] + incl - s;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        const long long r = base + i;
        if (r < m) {
            row_ptr[r] = run;
            if (bins.nb > 0) atomicAdd(&hist[bin_of(bins, v[i])], 1);
        }
        run += v[i];
    }
    if (m == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) row_ptr[0] = 0;
    } else if (base <= m - 1 && m - 1 < base + kScanPer) {
        row_ptr[m] = run;      // the thread holding row m-1 closes row_ptr
    }
    __syncthreads();
    if (bins.nb > 0 && threadIdx.x <= kMaxBins && hist[threadIdx.x])
        atomicAdd(&info->num_count[threadIdx.x], hist[threadIdx.x]);
}

// ===========================================================================
// Numeric pass with in-row column sort
// ===========================================================================

// Numeric, sub-wave lane groups.  T slots of (int32 key, FP64 value); a row
// with r = row_nnz_i <= T/2 entries.  After accumulation the occupied slots
// are compacted (group ballot) and each entry's output position is its
// rank among the row's keys (keys are distinct).
template <int G, int T, typename VT>
__global__ void __launch_bounds__(256)
k_num_group(int nrows_bin, const int32_t* __restrict__ perm,
            const int64_t* __restrict__ arp, const int32_t* __restrict__ acol, const VT* __restrict__ aval,
            const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol, const VT* __restrict__ bval,
            const int64_t* __restrict__ crp, int32_t* __restrict__ ccol, VT* __restrict__ cval,
            DevInfo* info) {
    constexpr int NG = GroupCfg<G>::NG;
    __shared__ int32_t keys[NG][T];
    __shared__ double vals[NG][T];
    __shared__ int32_t ck[NG][T / 2];
    __shared__ double cv[NG][T / 2];
    __shared__ long long s_off[NG][G];
    __shared__ long long s_bst[NG][G];
    __shared__ double s_a[NG][G];
    const int lane = threadIdx.x & 63;
    const int gl = threadIdx.x & (G - 1);
    const int g = threadIdx.x / G;
    const long long slot = (long long)xcd_block() * NG + g;
    if (slot >= nrows_bin) return;
    const int row = perm ? perm[slot] : (int)slot;
    int err = 0;
    int32_t* kt = keys[g];
    double* vt = vals[g];
#pragma unroll
    for (int s = gl; s < T; s += G) { kt[s] = kEmpty; vt[s] = 0.0; }
    lds_fence();
    const long long a0 = arp[row], a1 = arp[row + 1];
    for (long long c0 = a0; c0 < a1; c0 += G) {
        const long long p = c0 + gl;
        long long len = 0, bst = 0;
        double a = 0.0;
        if (p < a1) {
            const int32_t k = acol[p];
            a = to_f64(aval[p]);
            bst = brp[k];
            len = brp[k + 1] - bst;
        }
        const long long incl = group_incl_scan<G>(len, gl);
        const long long total = __shfl(incl, G - 1, G);
        s_off[g][gl] = incl;
        s_bst[g][gl] = bst - (incl - len);
        s_a[g][gl] = a;
        lds_fence();
        const int nact = (int)((a1 - c0) < G ? (a1 - c0) : G);
        for (long long q = gl; q < total; q += G) {
            const int t = owner_search(s_off[g], nact, q);
            const long long bi = s_bst[g][t] + q;
            const int32_t j = bcol[bi];
            const double prod = s_a[g][t] * to_f64(bval[bi]);
            const int h = hash_slot_of<T>(kt, j, &err);
            if (h >= 0) atomicAdd(&vt[h], prod);
        }
        lds_fence();
    }
    // compact the occupied slots
    int n = 0;
    for (int s0 = 0; s0 < T; s0 += G) {
        const int s = s0 + gl;
        const int32_t k = kt[s];
        const bool occ = k != kEmpty;
        const uint64_t mask = group_ballot<G>(occ, lane);
        if (occ) {
            const int pos = n + __builtin_popcountll(mask & ((1ull << gl) - 1));
            if (pos < T / 2) { ck[g][pos] = k; cv[g][pos] = vt[s]; }
        }
        n += __builtin_popcountll(mask);
    }
    lds_fence();
    const long long rp = crp[row];
    const int expect = (int)(crp[row + 1] - rp);
    if (n != expect || n > T / 2) {
        if (gl == 0) atomicOr(&info->err, kErrCount);
        return;
    }
    for (int e = gl; e < n; e += G) {
        const int32_t k = ck[g][e];
        int rank = 0;
        for (int f = 0; f < n; ++f) rank += (ck[g][f] < k) ? 1 : 0;
        ccol[rp + rank] = k;
        cval[rp + rank] = (VT)cv[g][e];
    }
    if (err) atomicOr(&info->err, kErrProbe);
}

// Numeric, one workgroup per row: LDS hash of T (key, FP64) slots, then the
// occupied slots are compacted to the front and bitonic-sorted by key in
// LDS, and the row is written with coalesced stores.
template <int BS, int T, typename VT>
__global__ void __launch_bounds__(BS)
k_num_block(int nrows_bin, const int32_t* __restrict__ perm,
            const int64_t* __restrict__ arp, const int32_t* __restrict__ acol, const VT* __restrict__ aval,
            const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol, const VT* __restrict__ bval,
            const int64_t* __restrict__ crp, int32_t* __restrict__ ccol, VT* __restrict__ cval,
            DevInfo* info) {
    constexpr int PER = T / BS;    // slots per thread in the compaction
    static_assert(PER >= 1, "T must be >= BS");
    __shared__ int32_t keys[T];
    __shared__ double vals[T];
    __shared__ long long s_off[BS];
    __shared__ long long s_bst[BS];
    __shared__ double s_a[BS];
    __shared__ BlockScanSmem<BS> sm;
    const int tid = threadIdx.x;
    int err = 0;
    for (long long slot = blockIdx.x; slot < nrows_bin; slot += gridDim.x) {
        const int row = perm ? perm[slot] : (int)slot;
        for (int s = tid; s < T; s += BS) { keys[s] = kEmpty; vals[s] = 0.0; }
        __syncthreads();
        const long long a0 = arp[row], a1 = arp[row + 1];
        for (long long c0 = a0; c0 < a1; c0 += BS) {
            const long long p = c0 + tid;
            long long len = 0, bst = 0;
            double a = 0.0;
            if (p < a1) {
                const int32_t k = acol[p];
                a = to_f64(aval[p]);
                bst = brp[k];
                len = brp[k + 1] - bst;
            }
            long long total;
            const long long incl = block_incl_scan<BS>(len, sm, &total);
            s_off[tid] = incl;
            s_bst[tid] = bst - (incl - len);
            s_a[tid] = a;
            __syncthreads();
            const int nact = (int)((a1 - c0) < BS ? (a1 - c0) : BS);
            for (long long q = tid; q < total; q += BS) {
                const int t = owner_search(s_off, nact, q);
                const long long bi = s_bst[t] + q;
                const int32_t j = bcol[bi];
                const double prod = s_a[t] * to_f64(bval[bi]);
                const int h = hash_slot_of<T>(keys, j, &err);
                if (h >= 0) atomicAdd(&vals[h], prod);
            }
            __syncthreads();
        }
        // compaction: thread tid owns slots [tid*PER, tid*PER + PER)
        int32_t rk[PER];
        double rv[PER];
        int c = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            rk[i] = keys[tid * PER + i];
            rv[i] = vals[tid * PER + i];
            c += rk[i] != kEmpty;
        }
        long long n;
        const long long incl = block_incl_scan<BS>(c, sm, &n);   // syncs: all reads done
        int pos = (int)(incl - c);
        const long long rp = crp[row];
        const int expect = (int)(crp[row + 1] - rp);
        const bool bad = (n != expect) || (n > T / 2);
        if (!bad) {
#pragma unroll
            for (int i = 0; i < PER; ++i)
                if (rk[i] != kEmpty) { keys[pos] = rk[i]; vals[pos] = rv[i]; ++pos; }
        }
        int P = 1;
        while (P < n) P <<= 1;
        if (!bad)
            for (int s = (int)n + tid; s < P; s += BS) keys[s] = 0x7fffffff;   // pad: sorts last
        __syncthreads();
        if (bad) {
            if (tid == 0) atomicOr(&info->err, kErrCount);
            continue;
        }
        // bitonic sort of keys[0..P) ascending, values follow
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int t = tid; t < P / 2; t += BS) {
                    const int i = 2 * j * (t / j) + (t % j);
                    const int l = i + j;
                    const bool up = (i & k) == 0;
                    const int32_t ki = keys[i], kl = keys[l];
                    if ((ki > kl) == up) {
                        keys[i] = kl; keys[l] = ki;
                        const double vi = vals[i];
                        vals[i] = vals[l]; vals[l] = vi;
                    }
                }
                __syncthreads();
            }
        }
        for (int e = tid; e < n; e += BS) {
            ccol[rp + e] = keys[e];
            cval[rp + e] = (VT)vals[e];
        }
        __syncthreads();
    }
    if (err) atomicOr(&info->err, kErrProbe);
}

// ===========================================================================
// Global spill for rows too large for LDS
// ===========================================================================
// Each workgroup owns a dense FP64 slab of ncols values (all zero between
// rows) and an ncols-bit bitmap (LDS when it fits, else a global slab).
// Products are added with device-scope FP64 atomics; the bitmap is then
// scanned in column order, which writes the row already sorted and returns
// the touched slab entries to zero.
template <int BS, bool LDSBM, typename VT>
__global__ void __launch_bounds__(BS)
k_num_dense(int nrows_bin, const int32_t* __restrict__ perm, long long ncols,
            const int64_t* __restrict__ arp, const int32_t* __restrict__ acol, const VT* __restrict__ aval,
            const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol, const VT* __restrict__ bval,
            const int64_t* __restrict__ crp, int32_t* __restrict__ ccol, VT* __restrict__ cval,
            double* dslab, uint32_t* gbm, DevInfo* info) {
    extern __shared__ uint32_t dyn_smem[];
    __shared__ long long s_off[BS];
    __shared__ long long s_bst[BS];
    __shared__ double s_a[BS];
    __shared__ BlockScanSmem<BS> sm;
    const int tid = threadIdx.x;
    const long long words = (ncols + 31) >> 5;
    double* dense = dslab + (long long)blockIdx.x * ncols;
    uint32_t* bm = LDSBM ? dyn_smem : gbm + (long long)blockIdx.x * words;
    for (long long slot = blockIdx.x; slot < nrows_bin; slot += gridDim.x) {
        const int row = perm ? perm[slot] : (int)slot;
        if (LDSBM) {
            for (long long w = tid; w < words; w += BS) bm[w] = 0u;
        }
        __syncthreads();
        const long long a0 = arp[row], a1 = arp[row + 1];
        for (long long c0 = a0; c0 < a1; c0 += BS) {
            const long long p = c0 + tid;
            long long len = 0, bst = 0;
            double a = 0.0;
            if (p < a1) {
                const int32_t k = acol[p];
                a = to_f64(aval[p]);
                bst = brp[k];
                len = brp[k + 1] - bst;
            }
            long long total;
            const long long incl = block_incl_scan<BS>(len, sm, &total);
            s_off[tid] = incl;
            s_bst[tid] = bst - (incl - len);
            s_a[tid] = a;
            __syncthreads();
            const int nact = (int)((a1 - c0) < BS ? (a1 - c0) : BS);
            for (long long q = tid; q < total; q += BS) {
                const int t = owner_search(s_off, nact, q);
                const long long bi = s_bst[t] + q;
                const int32_t j = bcol[bi];
                const double prod = s_a[t] * to_f64(bval[bi]);
                unsafeAtomicAdd(&dense[j], prod);
                atomicOr(&bm[j >> 5], 1u << (j & 31));
            }
            __syncthreads();
        }
        __threadfence();
        __syncthreads();
        // ordered extraction
        const long long rp = crp[row];
        long long run = 0;
        for (long long w0 = 0; w0 < words; w0 += BS) {
            const long long w = w0 + tid;
            uint32_t bits = 0;
            if (w < words) bits = LDSBM ? bm[w] : load_coherent(&bm[w]);
            const int c = __builtin_popcount(bits);
            long long tot;
            const long long incl = block_incl_scan<BS>(c, sm, &tot);
            long long pos = rp + run + incl - c;
            while (bits) {
                const int b = __builtin_ctz(bits);
                bits &= bits - 1;
                const long long col = w * 32 + b;
                const double v = load_coherent(&dense[col]);
                ccol[pos] = (int32_t)col;
                cval[pos] = (VT)v;
                dense[col] = 0.0;
                ++pos;
            }
            if (w < words && !LDSBM) gbm[(long long)blockIdx.x * words + w] = 0u;
            run += tot;
        }
        if (tid == 0 && run != crp[row + 1] - rp) atomicOr(&info->err, kErrCount);
        __threadfence();
        __syncthreads();
    }
}

// ===========================================================================
// Input validation (canonical CSR)
// ===========================================================================
static __global__ void __launch_bounds__(256)
k_validate(long long nrows, long long ncols, long long nnz, const int64_t* __restrict__ rp,
           const int32_t* __restrict__ col, DevInfo* info) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const long long a = rp[r], b = rp[r + 1];
    if (r == 0 && a != 0) { atomicOr(&info->err, kErrRange); return; }
    if (b < a || b > nnz) { atomicOr(&info->err, kErrRange); return; }
    if (r == nrows - 1 && b != nnz) { atomicOr(&info->err, kErrRange); return; }
    int prev = -1;
    for (long long p = a; p < b; ++p) {
        const int c = col[p];
        if (c < 0 || c >= ncols) { atomicOr(&info->err, kErrRange); return; }
        if (c <= prev) { atomicOr(&info->err, kErrUnsorted); return; }
        prev = c;
    }
}

}  // namespace msp
