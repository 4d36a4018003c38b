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
//     too large for LDS are cut into column slices whose bitmap, word ranks
//     and FP64 accumulator (indexed by the column's rank) fit the LDS, and
//     each slice goes out in column order from its bitmap, with no sort.
// Products of a row are enumerated "flattened": a lane group loads a chunk
// of A's row, prefix-sums the B-row lengths, and every lane takes the next
// product index and finds its A entry by binary search, so that the lanes
// stay busy whatever the B-row lengths are.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <climits>
#include <type_traits>

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

// Gather p[i].  With a 32-bit index type the caller guarantees that every
// byte offset i * sizeof(T) fits in 32 bits: the load then takes the array
// base from scalar registers and a 32-bit offset per lane, which also
// spares the registers of a 64-bit address per lane.
template <typename IT, typename T>
__device__ __forceinline__ T gat(const T* __restrict__ p, IT i) {
    if constexpr (sizeof(IT) == 4) {
        const uint32_t off = (uint32_t)i * (uint32_t)sizeof(T);
        return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + (uint64_t)off);
    } else {
        return p[i];
    }
}

// Loads that must observe atomics other lanes of the workgroup performed on
// global memory (the symbolic bitmap's global slab): bypass the
// non-coherent L1.
__device__ __forceinline__ double load_coherent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_coherent(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int load_coherent(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ long long load_coherent(const long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// After a pass (kernel boundary: its counters are complete), sum the
// partitioned bin counters and write the host summary, seq last.
// One workgroup of 64 threads.
static __global__ void __launch_bounds__(64)
k_publish(const DevInfo* info, int numeric, int nb, HostSummary* hs, int seq) {
    const int t = threadIdx.x;
    const int* part = numeric ? &info->num_part[0][0] : &info->sym_part[0][0];
    if (t < kNB) {
        int c = 0;
        if (t <= nb)
            for (int p = 0; p < kParts; ++p) c += part[p * kPartStride + t];
        hs->counts[t] = c;
    }
    __syncthreads();
    if (t == 0) {
        hs->nnz = numeric ? info->nnz : 0;
        hs->err = info->err;
        hs->neg_count = info->neg_count;
        __threadfence_system();
        __hip_atomic_store(&hs->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
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

// Length of the run of set bits at the bottom of a lane mask: 64 when every
// bit is set (count-trailing-zeros of 0 is undefined, so it is not used
// for that case).
__device__ __forceinline__ int leading_run(uint64_t m) {
    const uint64_t z = ~m;
    return z ? __builtin_ctzll(z) : 64;
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

// Row slots of a persistent workgroup kernel.  With a queue q (two counters
// in the device info block: slots handed out, workgroups done), a workgroup
// takes the next free slot each time it finishes a row, so that rows of very
// different cost (a skewed matrix's hub rows) spread over the compute units;
// without one (q null) workgroup b takes slots b, b + grid, ...  Every
// thread calls these (they synchronize the workgroup), and block_slots_done
// follows the loop.
__device__ __forceinline__ long long block_first(unsigned* q, long long* s_slot) {
    if (!q) return blockIdx.x;
    if (threadIdx.x == 0) *s_slot = atomicAdd(q, 1u);
    __syncthreads();
    return *s_slot;
}

__device__ __forceinline__ long long block_next(unsigned* q, long long slot, long long* s_slot) {
    if (!q) return slot + gridDim.x;
    __syncthreads();                            // every thread has read the previous slot
    if (threadIdx.x == 0) *s_slot = atomicAdd(q, 1u);
    __syncthreads();
    return *s_slot;
}

// The last workgroup out resets the queue: every other workgroup has taken
// its last slot by then, and the next launch on the stream finds zeros.
__device__ __forceinline__ void block_slots_done(unsigned* q) {
    if (!q || threadIdx.x != 0) return;
    __threadfence();
    if (atomicAdd(q + 1, 1u) == gridDim.x - 1) {
        atomicExch(q, 0u);
        atomicExch(q + 1, 0u);
    }
}

// ===========================================================================
// Fill a small int buffer (graph-safe replacement for memset)
// ===========================================================================
static __global__ void k_zero_words(int* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// Clear the device info block of a new call; the error bits the previous
// call's numeric kernels left there go to the host's pending word first
// (pending may be null).  One workgroup.
static __global__ void __launch_bounds__(256) k_zero_info(int* p, int n, int* pending) {
    if (threadIdx.x == 0 && pending) {
        // only the numeric kernels' bits: input-check bits were reported by
        // the call that set them
        const int e = p[offsetof(DevInfo, err) / 4] & (kErrProbe | kErrCount);
        if (e) __hip_atomic_store(pending, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 256) p[i] = 0;
}

// ===========================================================================
// Per-row statistics and symbolic binning
// ===========================================================================
//
// Add the wave's rows to an LDS histogram with one atomic per distinct bin
// present in the wave; returns the lane's rank among the workgroup's rows of
// its bin (b < 0: no row).  Wave-uniform control flow required.
__device__ __forceinline__ int wave_hist_add(int* hist, int b) {
    const int lane = threadIdx.x & 63;
    uint64_t todo = __ballot(b >= 0);
    int rank = 0;
    while (todo) {
        const int leader = __builtin_ctzll(todo);
        const int bl = __shfl(b, leader);
        const uint64_t same = __ballot(b == bl);
        int base = 0;
        if (lane == leader) base = atomicAdd(&hist[bl], __builtin_popcountll(same));
        base = __shfl(base, leader);
        if (b == bl) rank = base + __builtin_popcountll(same & ((1ull << lane) - 1));
        todo &= ~same;
    }
    return rank;
}

// As wave_hist_add with a weight per lane (lanes with b < 0 add nothing).
// Wave-uniform control flow required.
__device__ __forceinline__ void wave_hist_add_w(int* hist, int b, int w) {
    const int lane = threadIdx.x & 63;
    uint64_t todo = __ballot(b >= 0);
    while (todo) {
        const int leader = __builtin_ctzll(todo);
        const int bl = __shfl(b, leader);
        const uint64_t same = __ballot(b == bl);
        int x = b == bl ? w : 0;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d);
        if (lane == leader) atomicAdd(&hist[bl], x);
        todo &= ~same;
    }
}

// One wave per 64 consecutive rows.  The wave walks the A entries of its
// rows flattened (lane = entry), so a row's B-row lengths are gathered in
// parallel; each entry finds its row by binary search in the 65 row
// pointers held in LDS and adds into the row's LDS accumulator (after a
// reduction across the wave when the step's entries are all of one row).
// Outputs: u_i = min(prod_i, ncols(B)) (int32), optional int64 prod_i and
// FP32 features, row_nnz_i = 0 for rows with u_i = 0, and the bin
// histogram of u_i (partitioned global counters).
// The eight predictor inputs of a row from its statistics: A entries len,
// products s, shortest / longest B row mn / mx, and the column span hi - lo
// (hi < 0: no nonempty B row).
__device__ __forceinline__ void write_features(float* __restrict__ f, long long len, long long s, int mn, int mx,
                                               int lo, int hi, long long ncols) {
    const double n = (double)(ncols > 0 ? ncols : 1);
    const float mean = len > 0 ? (float)((double)s / (double)len) : 0.f;
    f[0] = log2f(1.f + (float)len) * kFeatLogScale;
    f[1] = log2f(1.f + (float)s) * kFeatLogScale;
    f[2] = log2f(1.f + (float)(len > 0 ? mn : 0)) * kFeatLogScale;
    f[3] = log2f(1.f + mean) * kFeatLogScale;
    f[4] = log2f(1.f + (float)mx) * kFeatLogScale;
    f[5] = log2f(1.f + (float)ncols) * kFeatLogScale;
    f[6] = fminf(1.f, (float)((double)s / n));
    f[7] = (float)((double)(hi < 0 ? 0 : hi - lo) / n);
}

// Rows with more than kLongRow A entries (single products, when lr.list is
// set) are left out of the wave's walk: each is listed with a contiguous
// range of kLongChunk-entry chunks for k_row_stats_long, and
// k_row_stats_long_fin writes its outputs.
template <bool FEAT, bool BATCH = false>
__global__ void __launch_bounds__(256)
k_row_stats(int m, long long ncols, const int64_t* __restrict__ arp, const int32_t* __restrict__ acol,
            const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol,
            int32_t* __restrict__ u_out, int64_t* __restrict__ prod_out,
            int32_t* __restrict__ row_nnz, BinTable bins, DevInfo* info,
            float* __restrict__ feat, int32_t* __restrict__ lo_out, RowMap mp, LongRows lr = LongRows{}) {
    static_assert(!(FEAT && BATCH), "features are computed for single products");
    __shared__ int hist[kNB];
    __shared__ long long s_bo[BATCH ? 4 : 1][64];   // batched: B-row offset and width of each row
    __shared__ long long s_nc[BATCH ? 4 : 1][64];
    __shared__ long long s_rp[4][65];
    __shared__ long long s_cp[4][65];               // prefix of the walked entries (long rows count 0)
    __shared__ unsigned long long s_prod[4][64];
    __shared__ int s_mn[FEAT ? 4 : 1][64], s_mx[FEAT ? 4 : 1][64];
    __shared__ int s_lo[FEAT ? 4 : 1][64], s_hi[FEAT ? 4 : 1][64];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    if (threadIdx.x < kNB) hist[threadIdx.x] = 0;
    const long long r0 = ((long long)blockIdx.x * 4 + w) * 64;
    const int nr = r0 < m ? (int)(m - r0 < 64 ? m - r0 : 64) : 0;
    // row pointers of the wave's rows: entries 0..nr (nr + 1 <= 65 values)
    if (lane < nr) s_rp[w][lane] = arp[r0 + lane];
    if (lane == 0 && nr > 0) s_rp[w][nr] = arp[r0 + nr];
    if constexpr (BATCH) {
        if (lane < nr) {
            const int pb = map_prob(mp, r0 + lane);
            s_bo[w][lane] = mp.boff[pb];
            s_nc[w][lane] = mp.ncols[pb];
        }
    }
    s_prod[w][lane] = 0;
    if constexpr (FEAT) {
        s_mn[w][lane] = 0x7fffffff; s_mx[w][lane] = 0; s_lo[w][lane] = 0x7fffffff; s_hi[w][lane] = -1;
    }
    __syncthreads();
    bool longr = false;
    if (nr > 0) {
        // the walked entries: every row's, except the long rows when they are
        // taken apart
        const long long len = lane < nr ? s_rp[w][lane + 1] - s_rp[w][lane] : 0;
        longr = !BATCH && lr.list && len > kLongRow;
        const long long cinc = group_incl_scan<64>(longr ? 0 : len, lane);
        s_cp[w][lane + 1] = cinc;
        if (lane == 0) s_cp[w][0] = 0;
        if (longr) {
            const int idx = atomicAdd(&info->long_n, 1);
            if (idx < lr.list_cap) {               // (the host sizes the lists for every long row)
                const int nch = (int)((len + kLongChunk - 1) / kLongChunk);
                const int b = atomicAdd(&info->long_chunks, nch);
                lr.list[idx] = (int)(r0 + lane);
                lr.base[idx] = b;
                lr.acc[idx] = LongAcc{0ull, 0x7fffffff, 0, 0x7fffffff, -1};
                for (int c = 0; c < nch; ++c)
                    if (b + c < lr.chunk_cap) lr.chunk_row[b + c] = idx;
            }
        }
        lds_fence();
        // RU entries per lane have their loads in flight together; a step
        // whose active lanes all belong to one row is reduced across the wave
        // first, so its accumulators take one atomic each instead of 64 on
        // one address
        constexpr int RU = 4;
        const long long ew = s_cp[w][nr];
        for (long long pb = 0; pb < ew; pb += 64 * RU) {       // wave-uniform
            int rw[RU];
            long long b0[RU], b1[RU];
            int c0[RU], c1[RU];
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const long long pc = pb + u * 64 + lane;
                rw[u] = -1;
                b0[u] = b1[u] = 0;
                if (pc < ew) {
                    // last row r with s_cp[r] <= pc (skips empty and long rows)
                    int lo = 0, hi = nr;       // s_cp[lo] <= pc < s_cp[hi]
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (s_cp[w][mid] <= pc) lo = mid; else hi = mid;
                    }
                    rw[u] = lo;
                    const long long p = s_rp[w][lo] + (pc - s_cp[w][lo]);
                    b0[u] = (long long)acol[p] + (BATCH ? s_bo[w][lo] : 0);   // the B row, for now
                }
            }
#pragma unroll
            for (int u = 0; u < RU; ++u)
                if (rw[u] >= 0) {
                    const long long k = b0[u];
                    b0[u] = brp[k];
                    b1[u] = brp[k + 1];
                }
            if constexpr (FEAT) {
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    c0[u] = 0x7fffffff;
                    c1[u] = -1;
                    if (rw[u] >= 0 && b1[u] > b0[u]) {
                        c0[u] = bcol[b0[u]];
                        c1[u] = bcol[b1[u] - 1];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const bool ok = rw[u] >= 0;
                const long long l = b1[u] - b0[u];
                const int r0l = __shfl(rw[u], 0);
                const uint64_t act = __ballot(ok);
                if (act && __ballot(ok && rw[u] == r0l) == act) {       // one row: reduce first
                    unsigned long long sl = ok ? (unsigned long long)l : 0ull;
                    int mn = ok ? (int)l : 0x7fffffff, mx = ok ? (int)l : 0;
                    int lo = FEAT ? c0[u] : 0, hi = FEAT ? c1[u] : 0;
#pragma unroll
                    for (int d = 32; d > 0; d >>= 1) {
                        sl += __shfl_xor(sl, d);
                        if constexpr (FEAT) {
                            mn = min(mn, __shfl_xor(mn, d));
                            mx = max(mx, __shfl_xor(mx, d));
                            lo = min(lo, __shfl_xor(lo, d));
                            hi = max(hi, __shfl_xor(hi, d));
                        }
                    }
                    if (lane == 0) {
                        atomicAdd(&s_prod[w][r0l], sl);
                        if constexpr (FEAT) {
                            atomicMin(&s_mn[w][r0l], mn);
                            atomicMax(&s_mx[w][r0l], mx);
                            if (hi >= 0) {
                                atomicMin(&s_lo[w][r0l], lo);
                                atomicMax(&s_hi[w][r0l], hi);
                            }
                        }
                    }
                } else if (ok) {
                    const int lo = rw[u];
                    atomicAdd(&s_prod[w][lo], (unsigned long long)l);
                    if constexpr (FEAT) {
                        atomicMin(&s_mn[w][lo], (int)l);
                        atomicMax(&s_mx[w][lo], (int)l);
                        if (l > 0) {
                            atomicMin(&s_lo[w][lo], c0[u]);
                            atomicMax(&s_hi[w][lo], c1[u]);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    const long long row = r0 + lane;
    const bool valid = lane < nr && !longr;        // (a long row's outputs come later)
    int bin = -1;
    if (valid) {
        const long long s = (long long)s_prod[w][lane];
        const long long nc = BATCH ? s_nc[w][lane] : ncols;
        const long long u = s < nc ? s : nc;
        u_out[row] = (int32_t)u;
        if (prod_out) prod_out[row] = s;
        if (u == 0 && row_nnz) row_nnz[row] = 0;
        bin = bin_of(bins, u);
        if constexpr (FEAT) {
            const long long len = s_rp[w][lane + 1] - s_rp[w][lane];
            const int mx = s_mx[w][lane];
            write_features(feat + row * 8, len, s, s_mn[w][lane], mx, s_lo[w][lane], s_hi[w][lane], ncols);
            if (lo_out) lo_out[row] = mx;
        }
    }
    if (bins.nb > 0) wave_hist_add(hist, bin);
    __syncthreads();
    if (bins.nb > 0 && threadIdx.x < kNB && hist[threadIdx.x])
        atomicAdd(&info->sym_part[blockIdx.x % kParts][threadIdx.x], hist[threadIdx.x]);
}

// Chunks of the long rows: one workgroup per chunk of kLongChunk entries
// (eight per thread, their loads in flight together), reduced in the
// workgroup, then one global atomic per statistic into the row's LongAcc.
template <bool FEAT>
__global__ void __launch_bounds__(256)
k_row_stats_long(const DevInfo* __restrict__ info, const int64_t* __restrict__ arp,
                 const int32_t* __restrict__ acol, const int64_t* __restrict__ brp,
                 const int32_t* __restrict__ bcol, LongRows lr) {
    __shared__ unsigned long long r_s[4];
    __shared__ int r_mn[4], r_mx[4], r_lo[4], r_hi[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nch = min(__hip_atomic_load(&info->long_chunks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                        lr.chunk_cap);
    constexpr int PT = kLongChunk / 256;
    for (int c = blockIdx.x; c < nch; c += gridDim.x) {
        const int idx = lr.chunk_row[c];
        const int row = lr.list[idx];
        const long long a0 = arp[row] + (long long)(c - lr.base[idx]) * kLongChunk;
        const long long a1 = min(arp[row + 1], a0 + kLongChunk);
        long long k[PT], b0[PT], b1[PT];
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const long long p = a0 + j * 256 + threadIdx.x;
            k[j] = p < a1 ? (long long)acol[p] : -1;
        }
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            b0[j] = b1[j] = 0;
            if (k[j] >= 0) {
                b0[j] = brp[k[j]];
                b1[j] = brp[k[j] + 1];
            }
        }
        unsigned long long sl = 0;
        int mn = 0x7fffffff, mx = 0, lo = 0x7fffffff, hi = -1;
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            if (k[j] < 0) continue;
            const long long l = b1[j] - b0[j];
            sl += (unsigned long long)l;
            if constexpr (FEAT) {
                mn = min(mn, (int)l);
                mx = max(mx, (int)l);
                if (l > 0) {
                    lo = min(lo, bcol[b0[j]]);
                    hi = max(hi, bcol[b1[j] - 1]);
                }
            }
        }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) {
            sl += __shfl_xor(sl, d);
            if constexpr (FEAT) {
                mn = min(mn, __shfl_xor(mn, d));
                mx = max(mx, __shfl_xor(mx, d));
                lo = min(lo, __shfl_xor(lo, d));
                hi = max(hi, __shfl_xor(hi, d));
            }
        }
        if (lane == 0) { r_s[w] = sl; r_mn[w] = mn; r_mx[w] = mx; r_lo[w] = lo; r_hi[w] = hi; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int v = 1; v < 4; ++v) {
                sl += r_s[v];
                mn = min(mn, r_mn[v]); mx = max(mx, r_mx[v]);
                lo = min(lo, r_lo[v]); hi = max(hi, r_hi[v]);
            }
            LongAcc* a = &lr.acc[idx];
            atomicAdd(&a->prod, sl);
            if constexpr (FEAT) {
                atomicMin(&a->mn, mn);
                atomicMax(&a->mx, mx);
                if (hi >= 0) {
                    atomicMin(&a->lo, lo);
                    atomicMax(&a->hi, hi);
                }
            }
        }
        __syncthreads();                          // r_* are reused by the next chunk
    }
}

// Outputs of the long rows (as k_row_stats writes them for the others); the
// bin counts go to the partition of the row's 256-row block, as the scatter
// expects.
template <bool FEAT>
__global__ void __launch_bounds__(256)
k_row_stats_long_fin(DevInfo* info, long long ncols, const int64_t* __restrict__ arp, LongRows lr,
                     int32_t* __restrict__ u_out, int64_t* __restrict__ prod_out, int32_t* __restrict__ row_nnz,
                     BinTable bins, float* __restrict__ feat, int32_t* __restrict__ lo_out) {
    const int nl = min(__hip_atomic_load(&info->long_n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), lr.list_cap);
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nl; idx += gridDim.x * blockDim.x) {
        const int row = lr.list[idx];
        const LongAcc a = lr.acc[idx];
        const long long s = (long long)a.prod;
        const long long u = s < ncols ? s : ncols;
        u_out[row] = (int32_t)u;
        if (prod_out) prod_out[row] = s;
        if (u == 0 && row_nnz) row_nnz[row] = 0;          // every B row it selects is empty
        if (bins.nb > 0) atomicAdd(&info->sym_part[(row / 256) % kParts][bin_of(bins, u)], 1);
        if constexpr (FEAT) {
            write_features(feat + (long long)row * 8, arp[row + 1] - arp[row], s, a.mn, a.mx, a.lo, a.hi, ncols);
            if (lo_out) lo_out[row] = a.mx;
        }
    }
}

// ===========================================================================
// Scatter row ids into per-bin lists
// ===========================================================================
// Bin b's rows occupy perm[start_b ...) with start_b the total of the bins
// before it; inside a bin, partition p's rows follow those of partitions
// < p, and each workgroup reserves its range from partition p's cursor.
// part_counts are the per-partition counts of the pass that binned the
// rows, which counted rows in workgroups of count_rows rows.  The whole
// counter table (kParts x kPartStride) is read once per workgroup, with
// coalesced loads, into LDS, where the bins' totals and this partition's
// prefix are summed.
static __global__ void __launch_bounds__(256)
k_scatter(int m, const int32_t* __restrict__ key, BinTable bins, const int* __restrict__ part_counts,
          int count_rows, int* cursor, int32_t* __restrict__ perm) {
    static_assert(kNB <= kPartStride && kPartStride <= 256, "a thread per bin");
    __shared__ int tab[kParts * kPartStride];
    __shared__ int tot[kPartStride];
    __shared__ int pre[kPartStride];
    __shared__ int cnt[kNB];
    __shared__ int base[kNB];
    if (threadIdx.x < kNB) cnt[threadIdx.x] = 0;
    for (int i = threadIdx.x; i < kParts * kPartStride; i += 256) tab[i] = part_counts[i];
    __syncthreads();
    const long long row = (long long)blockIdx.x * 256 + threadIdx.x;
    const int b = row < m ? bin_of(bins, key[row]) : -1;
    const int r = wave_hist_add(cnt, b);
    const int part = (int)(((long long)blockIdx.x * 256 / count_rows) % kParts);
    if (threadIdx.x <= bins.nb) {
        // bin t: its rows in every partition, and in the partitions before this one
        const int t = threadIdx.x;
        int all = 0, before = 0;
        for (int p = 0; p < kParts; ++p) {
            const int c = tab[p * kPartStride + t];
            all += c;
            before += p < part ? c : 0;
        }
        tot[t] = all;
        pre[t] = before;
    }
    __syncthreads();
    if (threadIdx.x <= bins.nb && cnt[threadIdx.x]) {
        const int me = threadIdx.x;
        int start = pre[me];
        for (int i = 0; i < me; ++i) start += tot[i];
        base[me] = start + atomicAdd(&cursor[part * kPartStride + me], cnt[me]);
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
    *err |= 1;
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
    *err |= 1;
    return -1;
}

// Window record of a symbolic row with `tot` outputs, for the numeric
// global bin (see WinRec), in two steps around the kernel's own count of the
// row's outputs per window: win_record_open clears the counts in s_wc and
// takes a record slot (false: no record for this row); the kernel adds into
// s_wc with LDS atomics; win_record_close writes the counts out.  Called by
// the whole workgroup with a uniform tot; both end with a barrier.
__device__ __forceinline__ bool win_record_open(int* cnt_ptr_nonnull, int nw, int thresh, int* nrec, long long tot,
                                                int* s_wc, int* s_slot) {
    if (!cnt_ptr_nonnull || tot <= thresh) return false;
    for (int w = threadIdx.x; w < nw; w += blockDim.x) s_wc[w] = 0;
    if (threadIdx.x == 0) *s_slot = atomicAdd(nrec, 1);
    __syncthreads();
    return true;
}

__device__ __forceinline__ void win_record_close(const WinRec& rec, int row, const int* s_wc, const int* s_slot,
                                                 int bm_slot = -1) {
    __syncthreads();
    const int slot = *s_slot;
    if (slot < rec.cap) {
        uint16_t* out = rec.cnt + (long long)slot * rec.nw;
        for (int w = threadIdx.x; w < rec.nw; w += blockDim.x) out[w] = (uint16_t)s_wc[w];
        if (threadIdx.x == 0) {
            rec.islot[row] = slot;
            rec.row[slot] = row;
            rec.rec_bm[slot] = bm_slot;
        }
    }
    __syncthreads();
}

// Rows per workgroup for a lane-group kernel of G lanes.
template <int G>
struct GroupCfg {
    static constexpr int BS = 256;
    static constexpr int NG = BS / G;
};

// Symbolic, sub-wave lane groups: G lanes per row, T key slots per row.
// rows = perm (bin list) or identity when perm == nullptr.  Every per-group
// LDS row is padded by one word so that the groups of a wave start on
// different banks.
template <int G, int T, bool BATCH = false>
__global__ void __launch_bounds__(256)
k_sym_group(Work wk, int m,
            const int64_t* __restrict__ arp, const int32_t* __restrict__ acol,
            const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol,
            int32_t* __restrict__ row_nnz, DevInfo* info, RowMap mp) {
    constexpr int NG = GroupCfg<G>::NG;
    static_assert(T % G == 0, "the table clears in T / G whole steps of the group");
    int nrows_bin;
    const int32_t* perm;
    work_rows(wk, &nrows_bin, &perm);
    __shared__ int32_t keys[NG][T + 1];
    __shared__ long long s_off[NG][G + 1];
    __shared__ long long s_bst[NG][G + 1];
    const int gl = threadIdx.x & (G - 1);
    const int g = threadIdx.x / G;
    (void)m;
    int err = 0;
    int32_t* kt = keys[g];
    // persistent: workgroup lb owns the contiguous slot range [lo, hi)
    const long long per = (nrows_bin + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)xcd_block() * per;
    const long long hi = lo + per < nrows_bin ? lo + per : nrows_bin;
    for (long long slot = lo + g; slot < hi; slot += NG) {      // group-uniform
    const int row = perm ? perm[slot] : (int)slot;
    const long long bo = row_boff<BATCH>(mp, row);
    const long long a0 = arp[row], a1 = arp[row + 1];
    // a one-chunk row's B-row position and length, loaded once for both paths
    bool pre = false;
    long long pre_len = 0, pre_bst = 0;
    if constexpr (G == 64) {
        // a whole-wave row of at most 64 A entries whose products' columns
        // (bounded by the first and last column of each B row) span less
        // than 32 T: its distinct columns are the bits set in a bitmap of
        // the span, the key table's T words, with one OR per product
        if (a1 - a0 <= 64) {                                      // wave-uniform
            const long long p = a0 + gl;
            long long len = 0, bst = 0;
            int fmn = 0x7fffffff, fmx = -1;
            if (p < a1) {
                const long long k = acol[p] + bo;
                bst = brp[k];
                len = brp[k + 1] - bst;
                if (len > 0) {
                    fmn = bcol[bst];
                    fmx = bcol[bst + len - 1];
                }
            }
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) {
                fmn = min(fmn, __shfl_xor(fmn, d));
                fmx = max(fmx, __shfl_xor(fmx, d));
            }
            if (fmx >= 0 && (long long)fmx - fmn < 32LL * T) {    // wave-uniform
                uint32_t* bm = reinterpret_cast<uint32_t*>(kt);
                const int nwd = ((fmx - fmn) >> 5) + 1;           // <= T
                for (int i = gl; i < nwd; i += 64) bm[i] = 0u;
                const long long incl = group_incl_scan<64>(len, gl);
                const long long total = __shfl(incl, 63);
                s_off[g][gl] = incl;
                s_bst[g][gl] = bst - (incl - len);
                lds_fence();
                const int nact = (int)(a1 - a0);
                int t = -1;
                for (long long q = gl; q < total; q += 64) {
                    if (t < 0) t = owner_search(s_off[g], nact, q);
                    else while (s_off[g][t] <= q) ++t;
                    const int d = bcol[s_bst[g][t] + q] - fmn;
                    // (in the span for canonical B; unsorted rows, which
                    // the input contract excludes, stay in bounds)
                    if ((unsigned)d < (unsigned)(nwd << 5)) atomicOr(&bm[d >> 5], 1u << (d & 31));
                }
                lds_fence();
                int c = 0;
                for (int i = gl; i < nwd; i += 64) c += __builtin_popcount(bm[i]);
                c = group_sum<64>(c);
                if (gl == 0) row_nnz[row] = c;
                lds_fence();
                continue;
            }
            pre = true;
            pre_len = len;
            pre_bst = bst;
        }
    }
#pragma unroll
    for (int i = 0; i < T / G; ++i) kt[gl + i * G] = kEmpty;
    lds_fence();
    int cnt = 0;
    for (long long c0 = a0; c0 < a1; c0 += G) {
        const long long p = c0 + gl;
        long long len = pre_len, bst = pre_bst;
        if (!pre && p < a1) {
            const long long k = acol[p] + bo;
            bst = brp[k];
            len = brp[k + 1] - bst;
        }
        const long long incl = group_incl_scan<G>(len, gl);
        const long long total = __shfl(incl, G - 1, G);
        s_off[g][gl] = incl;
        s_bst[g][gl] = bst - (incl - len);
        lds_fence();
        const int nact = (int)((a1 - c0) < G ? (a1 - c0) : G);
        int t = -1;                                  // owner of q: one search, then it only moves forward
        for (long long q = gl; q < total; q += G) {
            if (t < 0) t = owner_search(s_off[g], nact, q);
            else while (s_off[g][t] <= q) ++t;
            const int32_t j = bcol[s_bst[g][t] + q];
            cnt += hash_insert_key<T>(kt, j, &err);
        }
        lds_fence();
    }
    cnt = group_sum<G>(cnt);
    if (gl == 0) row_nnz[row] = cnt;
    lds_fence();
    }
    if (err) atomicOr(&info->err, kErrProbe);
}

// Symbolic, one workgroup of BS threads per row, T key slots (LDS).
template <int BS, int T, bool BATCH = false>
__global__ void __launch_bounds__(BS)
k_sym_block(Work wk,
            const int64_t* __restrict__ arp, const int32_t* __restrict__ acol,
            const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol,
            int32_t* __restrict__ row_nnz, DevInfo* info, RowMap mp, WinRec rec,
            unsigned* q) {
    int nrows_bin;
    const int32_t* perm;
    work_rows(wk, &nrows_bin, &perm);
    __shared__ long long s_slot;
    __shared__ int32_t keys[T];
    __shared__ int s_wc[BATCH ? 1 : kWinMaxNw];
    __shared__ int s_rslot;
    __shared__ long long s_off[BS];
    __shared__ long long s_bst[BS];
    __shared__ BlockScanSmem<BS> sm;
    const int tid = threadIdx.x;
    int err = 0;
    for (long long slot = block_first(q, &s_slot); slot < nrows_bin; slot = block_next(q, slot, &s_slot)) {
        const int row = perm ? perm[slot] : (int)slot;
        const long long bo = row_boff<BATCH>(mp, row);
        for (int s = tid; s < T; s += BS) keys[s] = kEmpty;
        __syncthreads();
        const long long a0 = arp[row], a1 = arp[row + 1];
        long long cnt = 0;
        for (long long c0 = a0; c0 < a1; c0 += BS) {
            const long long p = c0 + tid;
            long long len = 0, bst = 0;
            if (p < a1) {
                const long long k = acol[p] + bo;
                bst = brp[k];
                len = brp[k + 1] - bst;
            }
            long long total;
            const long long incl = block_incl_scan<BS>(len, sm, &total);
            s_off[tid] = incl;
            s_bst[tid] = bst - (incl - len);
            __syncthreads();
            const int nact = (int)((a1 - c0) < BS ? (a1 - c0) : BS);
            int t = -1;                     // owner of q: one search, then it only moves forward
            for (long long q = tid; q < total; q += BS) {
                if (t < 0) t = owner_search(s_off, nact, q);
                else while ((long long)s_off[t] <= q) ++t;
                const int32_t j = bcol[s_bst[t] + q];
                cnt += hash_insert_key<T>(keys, j, &err);
            }
            __syncthreads();
        }
        const long long tot = block_sum<BS>(cnt, sm);
        if (tid == 0) row_nnz[row] = (int32_t)tot;
        if constexpr (!BATCH) {
            if (win_record_open((int*)rec.cnt, rec.nw, rec.thresh, rec.nrec, tot, s_wc, &s_rslot)) {
                for (int i = tid; i < T; i += BS) {
                    const int32_t k = keys[i];
                    if (k != kEmpty) atomicAdd(&s_wc[k >> kWinLog], 1);
                }
                win_record_close(rec, row, s_wc, &s_rslot);
            }
        }
        __syncthreads();
    }
    block_slots_done(q);
    if (err) atomicOr(&info->err, kErrProbe);
}

// Symbolic for the largest rows: an n-bit bitmap (LDS when it fits, else a
// per-workgroup global slab), counting bits that an atomic OR newly sets.
template <int BS, bool LDSBM, bool BATCH = false>
__global__ void __launch_bounds__(BS)
k_sym_bitmap(Work wk, long long ncols,
             const int64_t* __restrict__ arp, const int32_t* __restrict__ acol,
             const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol,
             int32_t* __restrict__ row_nnz, uint32_t* gslab, DevInfo* info, RowMap mp, WinRec rec,
             unsigned* q) {
    int nrows_bin;
    const int32_t* perm;
    work_rows(wk, &nrows_bin, &perm);
    __shared__ long long s_slot;
    extern __shared__ uint32_t dyn_smem[];
    __shared__ int s_wc[BATCH ? 1 : kWinMaxNw];
    __shared__ int s_rslot, s_bmslot;
    __shared__ long long s_off[BS];
    __shared__ long long s_bst[BS];
    __shared__ BlockScanSmem<BS> sm;
    const int tid = threadIdx.x;
    const long long words = (ncols + 31) >> 5;
    uint32_t* bm = LDSBM ? dyn_smem : gslab + (long long)blockIdx.x * words;
    for (long long slot = block_first(q, &s_slot); slot < nrows_bin; slot = block_next(q, slot, &s_slot)) {
        const int row = perm ? perm[slot] : (int)slot;
        const long long bo = row_boff<BATCH>(mp, row);
        for (long long w = tid; w < words; w += BS) bm[w] = 0u;
        __syncthreads();
        const long long a0 = arp[row], a1 = arp[row + 1];
        long long cnt = 0, prod_row = 0;
        for (long long c0 = a0; c0 < a1; c0 += BS) {
            const long long p = c0 + tid;
            long long len = 0, bst = 0;
            if (p < a1) {
                const long long k = acol[p] + bo;
                bst = brp[k];
                len = brp[k + 1] - bst;
            }
            long long total;
            const long long incl = block_incl_scan<BS>(len, sm, &total);
            prod_row += total;
            s_off[tid] = incl;
            s_bst[tid] = bst - (incl - len);
            __syncthreads();
            const int nact = (int)((a1 - c0) < BS ? (a1 - c0) : BS);
            int t = -1;                     // owner of q: one search, then it only moves forward
            // SU products per thread and round, their loads issued before any
            // is used: one workgroup per compute unit leaves few waves to hide
            // the gathers
            constexpr int SU = 4;
            for (long long q0 = tid; q0 < total; q0 += SU * BS) {
                int32_t j[SU];
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const long long q = q0 + (long long)u * BS;
                    j[u] = -1;
                    if (q < total) {
                        if (t < 0) t = owner_search(s_off, nact, q);
                else while ((long long)s_off[t] <= q) ++t;
                        j[u] = bcol[s_bst[t] + q];
                    }
                }
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    if (j[u] < 0) continue;
                    const uint32_t bit = 1u << (j[u] & 31);
                    // the slab is this workgroup's own: workgroup scope suffices
                    const uint32_t old = LDSBM ? atomicOr(&bm[j[u] >> 5], bit)
                                               : __hip_atomic_fetch_or(&bm[j[u] >> 5], bit, __ATOMIC_RELAXED,
                                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                    cnt += (old & bit) ? 0 : 1;
                }
            }
            __syncthreads();
        }
        const long long tot = block_sum<BS>(cnt, sm);
        if (tid == 0) row_nnz[row] = (int32_t)tot;
        if constexpr (!BATCH) {
            if (win_record_open((int*)rec.cnt, rec.nw, rec.thresh, rec.nrec, tot, s_wc, &s_rslot)) {
                // a wave sums 64 consecutive words (half a window) with one atomic
                const int lane = tid & 63;
                for (long long w0 = (long long)(tid >> 6) * 64; w0 < words; w0 += BS) {
                    const long long w = w0 + lane;
                    int c = 0;
                    if (w < words) c = __builtin_popcount(LDSBM ? bm[w] : load_coherent(bm + w));
#pragma unroll
                    for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d);
                    if (lane == 0 && c) atomicAdd(&s_wc[(int)(w0 >> (kWinLog - 5))], c);
                }
                // the bitmap itself for a row with many products per column
                int bm_slot = -1;
                if (rec.bms && prod_row >= rec.bms_min_prod) {
                    if (tid == 0) s_bmslot = atomicAdd(rec.nbms, 1);
                    __syncthreads();
                    bm_slot = s_bmslot < rec.bms_cap ? s_bmslot : -1;
                    if (bm_slot >= 0) {
                        const long long sw = (long long)rec.nw * (kWin / 32);   // words of whole windows
                        uint32_t* dst = rec.bms + (long long)bm_slot * sw;
                        for (long long w = tid; w < sw; w += BS)
                            dst[w] = w < words ? (LDSBM ? bm[w] : load_coherent(bm + w)) : 0u;
                    }
                }
                win_record_close(rec, row, s_wc, &s_rslot, bm_slot);
            }
        }
        __syncthreads();
    }
    block_slots_done(q);
    (void)info;
}

// ===========================================================================
// Small-row kernels: wave-local row batches, one A entry per lane
// ===========================================================================
// Each wave owns a contiguous range of slots of the bin list and walks it in
// batches: it takes the longest run of consecutive rows (at most RM) whose
// A entries fit in the 64 lanes (always at least one row), so every lane
// holds one A entry and streams that entry's B row, four independent loads
// at a time, into its row's LDS hash table.  Waves never wait for each
// other (no workgroup barriers).  In the bins these kernels serve every B
// row has at most umax <= T/2 entries, so the per-lane loop is short.

template <int RM>
struct WaveRows {
    long long off[RM + 1];    // exclusive prefix of the rows' A-entry counts
    long long a0[RM];         // first A entry of each row
    long long c0[RM];         // C row start (numeric)
    long long c1[RM];         // C row end (numeric)
    long long bo[RM];         // batched: offset of the row's B rows
    int row[RM];
    int cnt[RM];
    int ovf[RM];              // capacity mode: the row's table overflowed
};

// Take the next batch starting at slot pos (< hi); returns the number of
// rows nb >= 1 and leaves E = wr.off[nb].  Whole wave.
template <int RM, bool NUMERIC, bool BATCH>
__device__ __forceinline__ int wave_rows_take(WaveRows<RM>& wr, long long pos, long long hi,
                                              const int32_t* __restrict__ perm,
                                              const int64_t* __restrict__ arp,
                                              const int64_t* __restrict__ crp, const RowMap& mp) {
    const int lane = threadIdx.x & 63;
    const int ncand = (int)(hi - pos < RM ? hi - pos : RM);
    long long a0 = 0, len = 0;
    int r = -1;
    if (lane < ncand) {
        r = perm ? perm[pos + lane] : (int)(pos + lane);
        a0 = arp[r];
        len = arp[r + 1] - a0;
    }
    const long long incl = group_incl_scan<64>(len, lane);
    const uint64_t fits = __ballot(lane < ncand && incl <= 64);
    int nb = leading_run(fits);               // leading run of rows that fit
    if (nb == 0) nb = 1;
    if (lane < nb) {
        wr.off[lane] = incl - len;
        wr.a0[lane] = a0;
        wr.row[lane] = r;
        wr.cnt[lane] = 0;
        wr.ovf[lane] = 0;
        wr.bo[lane] = row_boff<BATCH>(mp, r);
        if (NUMERIC) { wr.c0[lane] = crp[r]; wr.c1[lane] = crp[r + 1]; }
    }
    if (lane == nb - 1) wr.off[nb] = incl;
    return nb;
}

template <int RM>
__device__ __forceinline__ int wave_row_of(const WaveRows<RM>& wr, int nb, long long e) {
    int lo = 0, hi = nb;                    // wr.off[lo] <= e < wr.off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (wr.off[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// contiguous slot range of this wave (4 waves per workgroup)
__device__ __forceinline__ void wave_range(long long n, long long* lo, long long* hi);

// The rows [lo, hi) of the launch's n that a wave takes next.  Without a
// ticket counter: one contiguous range per wave (wave_range), once.  With
// one: blocks of wk.tk consecutive rows, drawn in turn from the counter that
// every wave of the launch shares (a work queue: a wave that finishes early
// takes more blocks); false once the rows run out.
__device__ __forceinline__ bool wave_block(const Work& wk, long long n, bool first, long long* lo, long long* hi) {
    if (!wk.ticket) {
        if (!first) return false;
        wave_range(n, lo, hi);
        return true;
    }
    int t = 0;
    if ((threadIdx.x & 63) == 0) t = atomicAdd(wk.ticket, 1);
    t = __shfl(t, 0);
    *lo = (long long)t * wk.tk;
    if (*lo >= n) return false;
    *hi = *lo + wk.tk < n ? *lo + wk.tk : n;
    return true;
}

__device__ __forceinline__ void wave_range(long long n, long long* lo, long long* hi) {
    const long long nw = (long long)gridDim.x * 4;
    const long long wid = (long long)xcd_block() * 4 + (threadIdx.x >> 6);
    const long long per = (n + nw - 1) / nw;
    *lo = wid * per;
    *hi = *lo + per < n ? *lo + per : n;
}

template <int T, int RM, bool BATCH = false>
__global__ void __launch_bounds__(256)
k_sym_wave(Work wk,
           const int64_t* __restrict__ arp, const int32_t* __restrict__ acol,
           const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol,
           int32_t* __restrict__ row_nnz, DevInfo* info, RowMap mp) {
    int nrows_bin;
    const int32_t* perm;
    work_rows(wk, &nrows_bin, &perm);
    __shared__ int32_t keys_all[4][RM][T + 1];
    __shared__ WaveRows<RM> wr_all[4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    auto& keys = keys_all[w];
    WaveRows<RM>& wr = wr_all[w];
    int err = 0;
    long long lo, hi;
    wave_range(nrows_bin, &lo, &hi);
    for (long long pos = lo; pos < hi;) {
        const int nb = wave_rows_take<RM, false, BATCH>(wr, pos, hi, perm, arp, nullptr, mp);
        for (int i = lane; i < nb * T; i += 64) keys[i / T][i % T] = kEmpty;
        lds_fence();
        const long long E = wr.off[nb];
        for (long long e = lane; e < E; e += 64) {
            const int r = wave_row_of<RM>(wr, nb, e);
            const long long p = wr.a0[r] + (e - wr.off[r]);
            const long long k = acol[p] + (BATCH ? wr.bo[r] : 0);
            const long long q0 = brp[k], q1 = brp[k + 1];
            int added = 0;
            for (long long q = q0; q < q1; q += 4) {
                int32_t j[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) j[u] = q + u < q1 ? bcol[q + u] : kEmpty;
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (j[u] != kEmpty) added += hash_insert_key<T>(keys[r], j[u], &err);
            }
            if (added) atomicAdd(&wr.cnt[r], added);
        }
        lds_fence();
        if (lane < nb) row_nnz[wr.row[lane]] = wr.cnt[lane];
        lds_fence();
        pos += nb;
    }
    if (err) atomicOr(&info->err, kErrProbe);
}

// Numeric counterpart: (key, FP64 value) tables.  Extraction: L = min(T, 64)
// lanes per row; each occupied slot's output position is the number of
// smaller keys in its row's table (unsigned compare, so empty slots count
// as larger than every key), read 16 bytes at a time and broadcast to the
// row's lanes.  Writes are guarded by the row's symbolic size.
template <int T, int RM, typename VT, bool BATCH = false>
__global__ void __launch_bounds__(256)
k_num_wave(Work wk,
           const int64_t* __restrict__ arp, const int32_t* __restrict__ acol, const VT* __restrict__ aval,
           const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol, const VT* __restrict__ bval,
           const int64_t* __restrict__ crp, int32_t* __restrict__ ccol, VT* __restrict__ cval,
           int32_t* __restrict__ cnt_out, DevInfo* info, RowMap mp) {
    int nrows_bin;
    const int32_t* perm;
    work_rows(wk, &nrows_bin, &perm);
    constexpr int KS = T + 4;                 // 16-byte aligned key rows, shifted banks
    constexpr int L = T < 64 ? T : 64;        // extraction lanes per row
    __shared__ __align__(16) int32_t keys_all[4][RM][KS];
    __shared__ double vals_all[4][RM][T + 1];
    __shared__ WaveRows<RM> wr_all[4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    auto& keys = keys_all[w];
    auto& vals = vals_all[w];
    WaveRows<RM>& wr = wr_all[w];
    int err = 0;
    long long lo, hi;
    wave_range(nrows_bin, &lo, &hi);
    for (long long pos = lo; pos < hi;) {
        const int nb = wave_rows_take<RM, true, BATCH>(wr, pos, hi, perm, arp, crp, mp);
        for (int i = lane; i < nb * T; i += 64) { keys[i / T][i % T] = kEmpty; vals[i / T][i % T] = 0.0; }
        lds_fence();
        const long long E = wr.off[nb];
        for (long long e = lane; e < E; e += 64) {
            const int r = wave_row_of<RM>(wr, nb, e);
            const long long p = wr.a0[r] + (e - wr.off[r]);
            const long long k = acol[p] + (BATCH ? wr.bo[r] : 0);
            const double a = to_f64(aval[p]);
            const long long q0 = brp[k], q1 = brp[k + 1];
            for (long long q = q0; q < q1; q += 4) {
                int32_t j[4];
                double v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool in = q + u < q1;
                    j[u] = in ? bcol[q + u] : kEmpty;
                    v[u] = in ? to_f64(bval[q + u]) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (j[u] != kEmpty) {
                        int e2 = 0;
                        const int h = hash_slot_of<T>(keys[r], j[u], &e2);
                        if (h >= 0) atomicAdd(&vals[r][h], a * v[u]);
                        else if (cnt_out) wr.ovf[r] = 1;
                        else err |= e2;
                    }
            }
        }
        lds_fence();
        for (int rr = lane / L; rr < nb; rr += 64 / L) {
            for (int sl = lane % L; sl < T; sl += L) {
                const uint32_t key = (uint32_t)keys[rr][sl];
                if (key == (uint32_t)kEmpty) continue;
                int rank = 0;
#pragma unroll 4
                for (int f = 0; f < T; f += 4) {
                    const int4 q = *reinterpret_cast<const int4*>(&keys[rr][f]);
                    rank += ((uint32_t)q.x < key) + ((uint32_t)q.y < key) + ((uint32_t)q.z < key) +
                            ((uint32_t)q.w < key);
                }
                const long long c0 = wr.c0[rr];
                if (rank < wr.c1[rr] - c0) {
                    ccol[c0 + rank] = (int32_t)key;
                    cval[c0 + rank] = (VT)vals[rr][sl];
                }
                atomicAdd(&wr.cnt[rr], 1);
            }
        }
        lds_fence();
        if (lane < nb) {
            const int cap = (int)(wr.c1[lane] - wr.c0[lane]);
            if (cnt_out) cnt_out[wr.row[lane]] = (wr.ovf[lane] || wr.cnt[lane] > cap) ? -1 : wr.cnt[lane];
            else if (wr.cnt[lane] != cap) err |= 2;
        }
        lds_fence();
        pos += nb;
    }
    if (err & 1) atomicOr(&info->err, kErrProbe);
    if (err & 2) atomicOr(&info->err, kErrCount);
}

// ===========================================================================
// Merge accumulator for short rows (FSpGEMM Alg. 1, one row per lane)
// ===========================================================================
// The paper's sort-and-merge unit adds sparse partial rows by merging them
// in column order.  Here one lane owns one output row and merges the (at
// most K) sorted B rows its A entries select: every step takes the smallest
// head column, adds a_ik * b_kj over the heads equal to it, and advances
// those heads.  The row comes out in column order (no hash table, no sort)
// in exactly row_nnz steps.  Rows with more than K A entries are taken by
// the whole wave afterwards, one at a time, with an LDS hash of FT slots
// (the bins served here bound the row's distinct columns by FT/2).

constexpr int kMergeFT = 64;     // fallback table: the merge bins bound rows by 32

template <int K, bool BATCH = false>
__global__ void __launch_bounds__(256)
k_sym_merge(Work wk,
            const int64_t* __restrict__ arp, const int32_t* __restrict__ acol,
            const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol,
            const int32_t* __restrict__ ufilter, int umax,
            int32_t* __restrict__ row_nnz, DevInfo* info, RowMap mp) {
    int nrows_bin;
    const int32_t* perm;
    work_rows(wk, &nrows_bin, &perm);
    __shared__ int32_t fb_keys[4][kMergeFT + 1];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int err = 0;
    long long lo, hi;
    wave_range(nrows_bin, &lo, &hi);
    for (long long base = lo; base < hi; base += 64) {
        const long long slot = base + lane;
        const bool valid = slot < hi;
        int row = -1;
        long long a0 = 0, a1 = 0, bo = 0;
        bool take = valid;
        if (valid) {
            row = perm ? perm[slot] : (int)slot;
            // with a filter, only rows whose bound is in (0, umax] are taken
            if (ufilter) { const int u = ufilter[row]; take = u > 0 && u <= umax; }
            if (take) {
                a0 = arp[row];
                a1 = arp[row + 1];
                bo = row_boff<BATCH>(mp, row);
            }
        }
        const bool mine = take && a1 - a0 <= K;
        if (mine) {
            const int len = (int)(a1 - a0);
            int hk[K];
            long long hp[K], he[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                hk[k] = 0x7fffffff;
                hp[k] = 0;
                he[k] = 0;
                if (k < len) {
                    const long long kk = acol[a0 + k] + bo;
                    hp[k] = brp[kk];
                    he[k] = brp[kk + 1];
                    if (hp[k] < he[k]) hk[k] = bcol[hp[k]];
                }
            }
            int cnt = 0;
            while (true) {
                int m = hk[0];
#pragma unroll
                for (int k = 1; k < K; ++k) m = hk[k] < m ? hk[k] : m;
                if (m == 0x7fffffff) break;
                ++cnt;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (hk[k] == m) {
                        ++hp[k];
                        hk[k] = hp[k] < he[k] ? bcol[hp[k]] : 0x7fffffff;
                    }
            }
            row_nnz[row] = cnt;
        }
        uint64_t fb = __ballot(take && !mine);
        while (fb) {                                   // wave-uniform
            const int r = __builtin_ctzll(fb);
            fb &= fb - 1;
            const int frow = __shfl(row, r);
            const long long fa0 = __shfl(a0, r), fa1 = __shfl(a1, r), fbo = __shfl(bo, r);
            for (int i = lane; i < kMergeFT; i += 64) fb_keys[w][i] = kEmpty;
            lds_fence();
            int c = 0;
            for (long long p = fa0; p < fa1; ++p) {
                const long long kk = acol[p] + fbo;
                const long long q1 = brp[kk + 1];
                for (long long q = brp[kk] + lane; q < q1; q += 64)
                    c += hash_insert_key<kMergeFT>(fb_keys[w], bcol[q], &err);
            }
            c = group_sum<64>(c);
            if (lane == 0) row_nnz[frow] = c;
            lds_fence();
        }
    }
    if (err) atomicOr(&info->err, kErrProbe);
}

// Tiles of the single-pass scan: numeric bin counts are kept per
// partition (tile mod kParts) of kScanTile rows, where the bin scatter
// looks for them.
constexpr int kScanBS = 1024;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanBS * kScanPer;

// Row statistics fused with the symbolic merge bin, for products whose bin
// plan starts with a merge bin.  One wave takes 64 consecutive rows.  A row
// with at most K A entries loads its B-row bounds once: they give its
// product count, and when the bound u = min(products, ncols) falls in the
// merge bin (0 < u <= umax) they are the merge's heads, so the row's
// distinct columns are counted right away.  Rows with more A entries sum
// their B-row lengths with the whole wave and, in the merge bin, take the
// hash fallback.  Every row's bound and bin count are recorded as the
// statistics pass records them; rows of the other bins are left for their
// own kernels.
template <int K, typename IT, bool BATCH = false>
__global__ void __launch_bounds__(256)
k_sym_fused(int m, long long ncols, const int64_t* __restrict__ arp, const int32_t* __restrict__ acol,
            const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol, int32_t* __restrict__ u_out,
            int32_t* __restrict__ row_nnz, BinTable bins, int umax, DevInfo* info, BinTable nbins,
            long long* __restrict__ bsum, long long super_rows, RowMap mp = RowMap{}) {
    __shared__ int hist[kNB];
    __shared__ int nhist[kNB];
    __shared__ long long s_sum[4];
    __shared__ int s_unknown;
    __shared__ int s_na;
    __shared__ int32_t fb_keys[4][kMergeFT + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x < kNB) { hist[threadIdx.x] = 0; nhist[threadIdx.x] = 0; }
    if (threadIdx.x == 0) { s_unknown = 0; s_na = 0; }
    __syncthreads();
    const long long r0 = ((long long)blockIdx.x * 4 + w) * 64;
    const long long row = r0 + lane;
    const bool valid = row < m;
    long long a0 = 0, a1 = 0, bo = 0, nc = ncols;
    if (valid) {
        a0 = arp[row];
        a1 = arp[row + 1];
        if constexpr (BATCH) {                         // the row's problem: B-row offset and width
            const int pb = map_prob(mp, row);
            bo = mp.boff[pb];
            nc = mp.ncols[pb];
        }
    }
    const bool shortrow = valid && a1 - a0 <= K;
    long long prod = 0;
    // rows with more than K A entries: the wave sums their B-row lengths
    uint64_t lr = __ballot(valid && !shortrow);
    while (lr) {                                       // wave-uniform
        const int r = __builtin_ctzll(lr);
        lr &= lr - 1;
        const long long la0 = __shfl(a0, r), la1 = __shfl(a1, r), lbo = __shfl(bo, r);
        long long s = 0;
        for (long long p = la0 + lane; p < la1; p += 64) {
            const long long kk = acol[p] + lbo;
            s += brp[kk + 1] - brp[kk];
        }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d);
        if (lane == r) prod = s;
    }
    // short rows: B-row bounds, which are also the merge's heads; IT is
    // 32-bit when the byte offsets into acol, brp and bcol fit 32 bits
    IT hp[K], he[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        hp[k] = 0;
        he[k] = 0;
        if (shortrow && k < (int)(a1 - a0)) {
            const IT kk = (IT)(gat(acol, (IT)(a0 + k)) + bo);
            hp[k] = (IT)gat(brp, kk);
            he[k] = (IT)gat(brp, (IT)(kk + 1));
            prod += (long long)(he[k] - hp[k]);
        }
    }
    int bin = -1;
    bool take = false;
    long long u = 0;
    if (valid) {
        u = prod < nc ? prod : nc;
        u_out[row] = (int32_t)u;
        if (u == 0) row_nnz[row] = 0;
        bin = bin_of(bins, u);
        take = u > 0 && u <= umax;
    }
    if (bins.nb > 0) wave_hist_add(hist, bin);
    int err = 0;
    int cnt = 0;                                       // the row's count, when counted here
    if (take && shortrow) {
        const int len = (int)(a1 - a0);
        int hk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) hk[k] = k < len && hp[k] < he[k] ? gat(bcol, hp[k]) : 0x7fffffff;
        while (true) {
            int mn = hk[0];
#pragma unroll
            for (int k = 1; k < K; ++k) mn = hk[k] < mn ? hk[k] : mn;
            if (mn == 0x7fffffff) break;
            ++cnt;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (hk[k] == mn) {
                    ++hp[k];
                    hk[k] = hp[k] < he[k] ? gat(bcol, hp[k]) : 0x7fffffff;
                }
        }
        row_nnz[row] = cnt;
    }
    uint64_t fb = __ballot(take && !shortrow);
    while (fb) {                                       // wave-uniform
        const int r = __builtin_ctzll(fb);
        fb &= fb - 1;
        const long long fa0 = __shfl(a0, r), fa1 = __shfl(a1, r), fbo = __shfl(bo, r);
        for (int i = lane; i < kMergeFT; i += 64) fb_keys[w][i] = kEmpty;
        lds_fence();
        int c = 0;
        for (long long p = fa0; p < fa1; ++p) {
            const long long kk = acol[p] + fbo;
            const long long q1 = brp[kk + 1];
            for (long long q = brp[kk] + lane; q < q1; q += 64)
                c += hash_insert_key<kMergeFT>(fb_keys[w], bcol[q], &err);
        }
        c = group_sum<64>(c);
        if (lane == r) { row_nnz[row] = c; cnt = c; }
        lds_fence();
    }
    if (err) atomicOr(&info->err, kErrProbe);
    // Rows of this pass have their final counts: their numeric bins and the
    // workgroup's total serve the speculative scan (valid when no row of the
    // whole product was left for another bin).
    const bool known = !valid || u == 0 || take;
    if (__ballot(!known) && lane == 0) s_unknown = 1;
    int na_max = take && shortrow ? (int)(a1 - a0) : 0;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) na_max = max(na_max, __shfl_xor(na_max, d));
    if (lane == 0 && na_max > 0) atomicMax(&s_na, na_max);
    if (nbins.nb > 0) wave_hist_add(nhist, valid && known ? bin_of(nbins, cnt) : -1);
    long long ws = known ? cnt : 0;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) ws += __shfl_xor(ws, d);
    if (lane == 0) s_sum[w] = ws;
    __syncthreads();
    if (bins.nb > 0 && threadIdx.x < kNB && hist[threadIdx.x])
        atomicAdd(&info->sym_part[blockIdx.x % kParts][threadIdx.x], hist[threadIdx.x]);
    if (threadIdx.x == 64 && s_na > 0) atomicMax(&info->sym_part[blockIdx.x % kParts][kPartMergeNA], s_na);
    if (threadIdx.x == 128 && s_unknown) atomicOr(&info->fused_other, 1);
    if (!s_unknown && nbins.nb > 0 && threadIdx.x < kNB && nhist[threadIdx.x])
        atomicAdd(&info->num_part[(blockIdx.x / (kScanTile / 256)) % kParts][threadIdx.x], nhist[threadIdx.x]);
    if (threadIdx.x == 0) {
        const long long tot = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
        bsum[blockIdx.x] = tot;
        if (tot && super_rows)
            atomicAdd(reinterpret_cast<unsigned long long*>(&info->ssum[(long long)blockIdx.x * 256 / super_rows]),
                      (unsigned long long)tot);
    }
}

// The speculative scan behind k_sym_fused.  When no row was left for a
// symbolic bin other than the empty and merge bins, every row count is
// final and the fused pass has stored each 256-row workgroup's total and
// the numeric bin sizes: a workgroup here adds the totals before its tile
// and scans its own rows, with no wait on any other workgroup, and the
// workgroup of the last rows publishes the host summary by itself.
// Otherwise every workgroup leaves and workgroup 0 publishes the symbolic
// bin sizes with nnz = -1, so that the host runs the other bins and a full
// scan.
constexpr int kWsBS = 512;
constexpr int kWsPer = 8;
constexpr int kWsTile = kWsBS * kWsPer;                // rows per workgroup: 16 fused workgroups
constexpr int kWsWaves = kWsBS / kWave;

// Rows per super-tile for a scan of `tiles` tiles: the fewest whole tiles
// that keep the number of super-tiles within kSupers, or 0 (no super-tiles:
// each tile sums the block totals before it) up to kDirectTiles tiles,
// where those reads cost less than the fused pass's device-scope atomics.
constexpr int kDirectTiles = 512;
inline long long super_tile_rows(int tiles) {
    if (tiles <= kDirectTiles) return 0;
    return ((long long)tiles + kSupers - 1) / kSupers * kWsTile;
}
static_assert(kParts * kPartStride == 2 * kWsBS, "the last tile loads the partition counters two per thread");
static_assert(kPartStride == 32 && kWave == 64, "a wave holds four partition rows");

static __global__ void __launch_bounds__(kWsBS)
k_scan_fused(int m, const int32_t* __restrict__ cnt, const long long* __restrict__ bsum, long long super_rows,
             int64_t* __restrict__ row_ptr, int spec_nb, DevInfo* info, HostSummary* hs, int seq) {
    __shared__ long long s_pre[kWsWaves], s_own[kWsWaves];
    __shared__ int s_cnt[kWsWaves][kPartStride];
    __shared__ int s_na;
    const int tile = blockIdx.x;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const bool last = tile == (int)gridDim.x - 1;
    // Every load is issued before the first wait: the flag, the totals
    // before this tile (the sums of the super-tiles before its own, if there
    // are super-tiles, then the fused workgroups' totals from the start of
    // its super-tile, in pairs: both bounds are multiples of 16
    // workgroups), this tile's row counts and, in the last tile, the
    // partitioned numeric bin counters.
    const bool other = load_coherent(&info->fused_other) != 0;
    const long long sup = super_rows ? (long long)tile * kWsTile / super_rows : 0;
    const long long b0 = sup * (super_rows / 256);
    const long long npair = ((long long)tile * (kWsTile / 256) - b0) / 2;
    const longlong2* bs2 = reinterpret_cast<const longlong2*>(bsum + b0);
    long long acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
    for (long long j = threadIdx.x; j < sup; j += kWsBS) acc1 += info->ssum[j];
    long long i = threadIdx.x;
    for (; i + 3 * kWsBS < npair; i += 4 * kWsBS) {
        const longlong2 q0 = bs2[i], q1 = bs2[i + kWsBS], q2 = bs2[i + 2 * kWsBS], q3 = bs2[i + 3 * kWsBS];
        acc0 += q0.x + q0.y;
        acc1 += q1.x + q1.y;
        acc2 += q2.x + q2.y;
        acc3 += q3.x + q3.y;
    }
    for (; i < npair; i += kWsBS) {
        const longlong2 q = bs2[i];
        acc0 += q.x + q.y;
    }
    const long long base = (long long)tile * kWsTile + (long long)threadIdx.x * kWsPer;
    static_assert(kWsPer == 8, "the vector path loads two int4");
    int v[kWsPer];
    const bool full = base + kWsPer <= m;
    if (full && ((uintptr_t)cnt & 15) == 0) {
        const int4 q0 = *reinterpret_cast<const int4*>(cnt + base);
        const int4 q1 = *reinterpret_cast<const int4*>(cnt + base + 4);
        v[0] = q0.x; v[1] = q0.y; v[2] = q0.z; v[3] = q0.w;
        v[4] = q1.x; v[5] = q1.y; v[6] = q1.z; v[7] = q1.w;
    } else {
#pragma unroll
        for (int j = 0; j < kWsPer; ++j) v[j] = base + j < m ? cnt[base + j] : 0;
    }
    int2 np2 = make_int2(0, 0);
    int na = 0;
    if (last) {
        np2 = reinterpret_cast<const int2*>(&info->num_part[0][0])[threadIdx.x];
        if (threadIdx.x < kParts) na = info->sym_part[threadIdx.x][kPartMergeNA];
    }
    if (other) {
        // one flag raised by the fused pass's workgroups that left rows for
        // other bins; workgroup 0 sums the symbolic bin sizes for the host
        if (hs && tile == 0 && threadIdx.x < 64) {
            const int t = threadIdx.x;
            int c = 0;
            if (t < kNB && t <= spec_nb)
                for (int p = 0; p < kParts; ++p) c += load_coherent(&info->sym_part[p][t]);
            if (t < kNB) hs->counts[t] = c;
            if (t == 0) {
                hs->nnz = -1;
                hs->err = load_coherent(&info->err);
                hs->neg_count = 0;
            }
            __threadfence_system();
            if (t == 0) __hip_atomic_store(&hs->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        return;                                         // uniform: the flag is fixed during this kernel
    }
    // one workgroup pass: the sum of the totals before the tile and the
    // exclusive scan of the tile's rows
    long long pre = (acc0 + acc1) + (acc2 + acc3);
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) pre += __shfl_xor(pre, d);
    long long s = 0;
#pragma unroll
    for (int j = 0; j < kWsPer; ++j) s += v[j];
    const long long incl = group_incl_scan<kWave>(s, lane);
    if (lane == kWave - 1) { s_pre[w] = pre; s_own[w] = incl; }
    if (last) {
        // lanes 16q..16q+15 of a wave hold partition 4w+q, two bins a lane
        int c0 = np2.x, c1 = np2.y;
        c0 += __shfl_xor(c0, 16); c1 += __shfl_xor(c1, 16);
        c0 += __shfl_xor(c0, 32); c1 += __shfl_xor(c1, 32);
        if (lane < 16) { s_cnt[w][2 * lane] = c0; s_cnt[w][2 * lane + 1] = c1; }
        if (w == 0) {
#pragma unroll
            for (int d = 16; d > 0; d >>= 1) na = max(na, __shfl_xor(na, d));
            if (lane == 0) s_na = na;
        }
    }
    __syncthreads();
    long long prefix = 0, before = 0, tot = 0;
#pragma unroll
    for (int j = 0; j < kWsWaves; ++j) {
        prefix += s_pre[j];
        const long long t = s_own[j];
        if (j < w) before += t;
        tot += t;
    }
    long long run = prefix + before + incl - s;
    long long rp[kWsPer];
#pragma unroll
    for (int j = 0; j < kWsPer; ++j) {
        rp[j] = run;
        run += v[j];
    }
    if (row_ptr) {
        if (full && ((uintptr_t)row_ptr & 15) == 0) {
#pragma unroll
            for (int j = 0; j < kWsPer; j += 2)
                *reinterpret_cast<longlong2*>(row_ptr + base + j) = make_longlong2(rp[j], rp[j + 1]);
        } else {
#pragma unroll
            for (int j = 0; j < kWsPer; ++j)
                if (base + j < m) row_ptr[base + j] = rp[j];
        }
        if (base <= m - 1 && m - 1 < base + kWsPer) row_ptr[m] = run;
    }
    if (last && threadIdx.x < 64) {
        // the last tile: nnz(C) is its prefix plus its total; the numeric
        // bin sizes were counted by the fused pass
        const long long nnz = prefix + tot;
        int c = 0;
        if (threadIdx.x < kNB)
#pragma unroll
            for (int j = 0; j < kWsWaves; ++j) c += s_cnt[j][threadIdx.x];
        if (threadIdx.x == 0) info->nnz = nnz;
        if (hs) {
            if (threadIdx.x < kNB) hs->counts[threadIdx.x] = c;
            if (threadIdx.x == 0) {
                hs->merge_na = s_na;
                hs->nnz = nnz;
                hs->err = load_coherent(&info->err);
                hs->neg_count = 0;
            }
            __threadfence_system();
            if (threadIdx.x == 0) __hip_atomic_store(&hs->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// Numeric merge.  A wave takes the longest run of its rows (at most 64)
// whose outputs fit an LDS staging area of kMergeStage entries; every row's
// output is merged into its own staging segment (its size is known from the
// symbolic pass) and the whole batch is then copied to C with coalesced
// stores, so each cache line of C is written once and completely.
// 704 outputs (12 B each) per wave: with the fallback tables a workgroup
// holds about 40 KB of LDS, four per compute unit, and a wave takes about 54
// rows of 13 outputs at once.  Measured on the 2D Laplacian product, the
// numeric pass takes 97-99 us at 704, 108 us at 512 (five workgroups per
// compute unit, 39 rows a wave), 116 us at 440 and 149 us at 1000 (two
// workgroups per compute unit).
constexpr int kMergeStage = 704;

// Numeric rows of a merge batch that the per-lane merge does not take
// (more A entries than heads), taken in groups: consecutive such rows (lane
// order) whose A entries fit the 64 lanes, then of those the leading rows
// whose products fit them too.  One lane per A entry finds its B row; one
// lane per product loads (column, a * b) with the key (row lane, column);
// the wave sorts the keys (bitonic network over lane shuffles), sums equal
// keys with a segmented scan, and the last lane of each run writes the sum
// at the column's rank in its row's staging area.  The rank of a run is the
// number of runs before it in its row, so the row comes out in column order.
// Every lane takes part (the lookups are shuffles); a row with more than
// 64 A entries or products is returned in the result mask for the LDS-hash
// path.  Per-lane inputs describe the lane's row of the batch.
template <typename VT>
__device__ __forceinline__ uint64_t merge_fallback_sorted(
    uint64_t todo, long long a0, long long a1, long long bo, long long nn, int row, const int* st_off,
    int32_t* st_k, double* st_v, const int32_t* __restrict__ acol, const VT* __restrict__ aval,
    const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol, const VT* __restrict__ bval,
    int32_t* __restrict__ cnt_out, int* err) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t left = 0;                                     // rows for the LDS-hash path
    while (todo) {                                         // wave-uniform
        const bool cand = (todo >> lane) & 1ull;
        const long long na = cand ? (a1 - a0 < 65 ? a1 - a0 : 65) : 0;
        const long long ia = group_incl_scan<64>(na, lane);          // A slots of the candidates before
        const uint64_t take = __ballot(cand && ia <= 64);
        if (!take) {                                       // the first candidate alone has > 64 A entries
            const uint64_t first = todo & (~todo + 1ull);
            left |= first;
            todo &= ~first;
            continue;
        }
        const long long total_a = __shfl(ia, 63 - __builtin_clzll(take));
        // A slot `lane`: its row r (the first lane whose prefix passes it),
        // its entry, and that entry's B row
        int r = 0;
        {
            int lo = 0, hi = 63;
#pragma unroll
            for (int st = 0; st < 6; ++st) {
                const int mid = (lo + hi) >> 1;
                const long long v = __shfl(ia, mid);
                if (v > lane) hi = mid; else lo = mid + 1;
            }
            r = lo;
        }
        const long long r_start = __shfl(ia - na, r), r_a0 = __shfl(a0, r), r_bo = __shfl(bo, r);
        long long bst = 0, blen = 0;
        double av = 0.0;
        if (lane < total_a) {
            const long long p = r_a0 + (lane - r_start);
            const long long k = acol[p] + r_bo;
            av = to_f64(aval[p]);
            bst = brp[k];
            blen = brp[k + 1] - bst;
        }
        const long long ip = group_incl_scan<64>(blen, lane);        // products of the slots up to this one
        // products of the rows up to each taken row: the prefix at its last slot
        const long long last_slot = ia - 1 < 63 ? (ia - 1 > 0 ? ia - 1 : 0) : 63;
        const long long upto = __shfl(ip, (int)last_slot);
        const uint64_t fin = __ballot(((take >> lane) & 1ull) && upto <= 64);
        if (!fin) {                                        // the first row alone has > 64 products
            const uint64_t first = take & (~take + 1ull);
            left |= first;
            todo &= ~first;
            continue;
        }
        const long long P = __shfl(upto, 63 - __builtin_clzll(fin));
        // product `lane`: its slot s (the first slot whose prefix passes it)
        int sl = 0;
        {
            int lo = 0, hi = 63;
#pragma unroll
            for (int st = 0; st < 6; ++st) {
                const int mid = (lo + hi) >> 1;
                const long long v = __shfl(ip, mid);
                if (v > lane) hi = mid; else lo = mid + 1;
            }
            sl = lo;
        }
        const long long s_bst = __shfl(bst - (ip - blen), sl);
        const double s_av = __shfl(av, sl);
        const int s_row = __shfl(r, sl);
        unsigned long long key = ~0ull;
        double v = 0.0;
        if (lane < P) {
            const long long bi = s_bst + lane;
            key = ((unsigned long long)(unsigned)s_row << 32) | (unsigned)bcol[bi];
            v = s_av * to_f64(bval[bi]);
        }
        // ascending bitonic sort of (key, v) across the wave
#pragma unroll
        for (int kk = 2; kk <= 64; kk <<= 1) {
#pragma unroll
            for (int j = kk >> 1; j > 0; j >>= 1) {
                const unsigned long long ok = __shfl_xor(key, j);
                const double ov = __shfl_xor(v, j);
                const bool up = (lane & kk) == 0, low = (lane & j) == 0;
                if (low == up ? ok < key : ok > key) {
                    key = ok;
                    v = ov;
                }
            }
        }
        // segmented inclusive sums of equal keys; a run's last lane holds its sum
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const unsigned long long ok = __shfl_up(key, d);
            const double ov = __shfl_up(v, d);
            if (lane >= d && ok == key) v += ov;
        }
        // (every lane takes part in each shuffle: none sits under a condition)
        const unsigned long long knext = __shfl_down(key, 1), kprev = __shfl_up(key, 1);
        const bool valid = key != ~0ull;
        const bool tail = valid && (lane == 63 || knext != key);
        const uint64_t tails = __ballot(tail);
        const int rl = (int)(key >> 32);
        const bool row_head = lane == 0 || (int)(kprev >> 32) != rl;
        int hd = row_head ? lane : 0;                      // first lane of this lane's row
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int o = __shfl_up(hd, d);
            if (lane >= d && o > hd) hd = o;
        }
        const int rank = __builtin_popcountll(tails & below) - __builtin_popcountll(tails & ((1ull << hd) - 1ull));
        const int so = st_off[valid ? rl : 0];
        const long long rnn = __shfl(nn, valid ? rl : 0);
        const int rrow = __shfl(row, valid ? rl : 0);
        if (tail && rank < rnn) {
            st_k[so + rank] = (int32_t)(key & 0xffffffffu);
            st_v[so + rank] = v;
        }
        // the row's last run gives its count
        const bool row_end = tail && (lane == 63 || (int)(knext >> 32) != rl);
        if (row_end) {
            const int c = rank + 1;
            if (cnt_out) cnt_out[rrow] = c <= rnn ? c : -1;
            else if (c != rnn) *err |= 2;
        }
        todo &= ~fin;
    }
    return left;
}

// B-row sharing across the rows of a merge batch (Sec. IV-A, Fig. 3).  The
// paper's processing elements each take one row of A, and a row of B that
// they all need is read from off-chip memory once and buffered for all of
// them.  Here the lanes of a wave take one row each: the wave stages every
// distinct B row that its merge rows reference once in LDS (in ascending B
// row order, one lane copying each row), and the lanes' merges read B from
// LDS.  A batch is staged when its B rows span at most 64 kShareSpanWords
// rows, number at most kShareRows and hold at most share_entries<VT>()
// entries; otherwise it reads B from global memory as without sharing.
constexpr int kShareSpanWords = 64;               // span bitmap: 64-bit words per wave
constexpr int kShareRows = 256;                   // distinct B rows per staged batch
template <typename VT>
constexpr int share_entries() { return sizeof(VT) == 8 ? 512 : 768; }

template <typename T>
__device__ __forceinline__ T wave_min(T x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        const T y = __shfl_xor(x, d);
        x = y < x ? y : x;
    }
    return x;
}
template <typename T>
__device__ __forceinline__ T wave_max(T x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        const T y = __shfl_xor(x, d);
        x = y > x ? y : x;
    }
    return x;
}

// With SHARE, a batch takes at most share_g rows (the group of rows that
// share the staged B rows).
template <int K, typename VT, typename IT, bool BATCH = false, bool SHARE = false>
__global__ void __launch_bounds__(256)
k_num_merge(Work wk,
            const int64_t* __restrict__ arp, const int32_t* __restrict__ acol, const VT* __restrict__ aval,
            const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol, const VT* __restrict__ bval,
            const int64_t* __restrict__ crp, int32_t* __restrict__ ccol, VT* __restrict__ cval,
            int32_t* __restrict__ cnt_out, DevInfo* info, RowMap mp, int share_g) {
    int nrows_bin;
    const int32_t* perm;
    work_rows(wk, &nrows_bin, &perm);
    constexpr int FT = kMergeFT;
    constexpr int SN = kMergeStage;
    static_assert(SN >= FT / 2, "a fallback row must fit the staging area");
    __shared__ int32_t st_k[4][SN];             // staged output columns
    __shared__ double st_v[4][SN];              // staged output values
    __shared__ __align__(16) int32_t fb_keys[4][FT + 4];
    __shared__ double fb_vals[4][FT + 1];
    __shared__ int st_off[4][65];               // staging offset of each row of the batch
    __shared__ long long st_c0[4][64];          // C row start of each row of the batch
    // shared B rows (SHARE only): bit d of the span bitmap is B row kmin + d;
    // sh_wr holds the rank of each bitmap word's first row, sh_row the
    // distinct rows in order (as d, then as their start in B), sh_off their
    // offsets in the stage
    constexpr int SE = SHARE ? share_entries<VT>() : 1;
    __shared__ unsigned long long sh_bm[4][SHARE ? kShareSpanWords : 1];
    __shared__ int sh_wr[4][SHARE ? kShareSpanWords : 1];
    __shared__ int sh_row[4][SHARE ? kShareRows : 1];
    __shared__ int sh_off[4][SHARE ? kShareRows + 1 : 1];
    __shared__ int32_t sh_col[4][SE];
    __shared__ VT sh_val[4][SE];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int err = 0;
    // sharing figures of the wave's batches, added to the totals once at the end
    unsigned long long sh_batches = 0, sh_nnz = 0, sh_rows = 0;
    long long lo, hi;
    for (bool first = true; wave_block(wk, nrows_bin, first, &lo, &hi); first = false)
    for (long long pos = lo; pos < hi;) {
        const int ncand = (int)(hi - pos < 64 ? hi - pos : 64);
        int row = -1;
        long long a0 = 0, a1 = 0, c0 = 0, c1 = 0, bo = 0;
        if (lane < ncand) {
            row = perm ? perm[pos + lane] : (int)(pos + lane);
            a0 = arp[row];
            a1 = arp[row + 1];
            c0 = crp[row];
            c1 = crp[row + 1];
            bo = row_boff<BATCH>(mp, row);
        }
        const long long nn = c1 - c0;           // row's output size (symbolic)
        const long long incl = group_incl_scan<64>(nn, lane);
        const uint64_t fits = __ballot(lane < ncand && incl <= SN);
        int nb = leading_run(fits);             // all 64 rows may fit
        if (nb == 0) nb = 1;                    // never happens in bins with nnz <= SN
        if (SHARE && nb > share_g) nb = share_g;
        const bool in = lane < nb;
        if (in) { st_off[w][lane] = (int)(incl - nn); st_c0[w][lane] = c0; }
        if (lane == nb - 1) st_off[w][nb] = (int)incl;
        lds_fence();
        const bool mine = in && a1 - a0 <= K && nn <= SN;
        bool shared = false;                    // wave-uniform
        long long kmin = 0;
        if constexpr (SHARE) {
            // the span of the B rows the merge rows reference (A rows are sorted)
            long long k_lo = LLONG_MAX, k_hi = -1;
            if (mine && a1 > a0) {
                k_lo = acol[a0] + bo;
                k_hi = acol[a1 - 1] + bo;
            }
            kmin = wave_min(k_lo);
            k_hi = wave_max(k_hi);
            if (k_hi >= 0 && k_hi - kmin < 64LL * kShareSpanWords) {
                sh_bm[w][lane] = 0ull;
                lds_fence();
                if (mine)
                    for (long long p = a0; p < a1; ++p) {
                        const int d = (int)(acol[p] + bo - kmin);
                        atomicOr(&sh_bm[w][d >> 6], 1ull << (d & 63));
                    }
                lds_fence();
                unsigned long long bits = sh_bm[w][lane];
                const int c = __builtin_popcountll(bits);
                const int wincl = (int)group_incl_scan<64>(c, lane);
                const int nd = __shfl(wincl, 63);
                if (nd <= kShareRows) {
                    sh_wr[w][lane] = wincl - c;
                    int r = wincl - c;
                    while (bits) {
                        const int t = __builtin_ctzll(bits);
                        bits &= bits - 1ull;
                        sh_row[w][r++] = lane * 64 + t;
                    }
                    lds_fence();
                    // stage offsets: the prefix of the distinct rows' lengths;
                    // sh_row[d] then holds row d's start in B (positions are
                    // 32-bit where sharing runs)
                    int tot = 0;
                    for (int d0 = 0; d0 < nd; d0 += 64) {
                        const int d = d0 + lane;
                        long long len = 0, src = 0;
                        if (d < nd) {
                            const long long k = kmin + sh_row[w][d];
                            src = brp[k];
                            len = brp[k + 1] - src;
                        }
                        const long long li = group_incl_scan<64>(len, lane);
                        if (d < nd) {
                            sh_off[w][d] = (int)(tot + li - len);
                            sh_row[w][d] = (int)src;
                        }
                        tot += (int)__shfl(li, 63);
                        if (tot > SE) break;                // uniform
                    }
                    if (tot <= SE) {
                        if (lane == 0) sh_off[w][nd] = tot;
                        lds_fence();
                        // the stage entry by entry: consecutive lanes take
                        // consecutive entries (coalesced within a B row), and
                        // CU rounds of loads are in flight before any store;
                        // entry e is in the last row d with sh_off[d] <= e
                        constexpr int CU = 4;
                        for (int e0 = 0; e0 < tot; e0 += 64 * CU) {
                            int32_t cc[CU];
                            VT vv[CU];
#pragma unroll
                            for (int u = 0; u < CU; ++u) {
                                const int e = e0 + u * 64 + lane;
                                if (e < tot) {
                                    int dlo = 0, dhi = nd;      // sh_off[dlo] <= e < sh_off[dhi]
                                    while (dhi - dlo > 1) {
                                        const int mid = (dlo + dhi) >> 1;
                                        if (sh_off[w][mid] <= e) dlo = mid; else dhi = mid;
                                    }
                                    const long long q = (long long)sh_row[w][dlo] + (e - sh_off[w][dlo]);
                                    cc[u] = bcol[q];
                                    vv[u] = bval[q];
                                }
                            }
#pragma unroll
                            for (int u = 0; u < CU; ++u) {
                                const int e = e0 + u * 64 + lane;
                                if (e < tot) {
                                    sh_col[w][e] = cc[u];
                                    sh_val[w][e] = vv[u];
                                }
                            }
                        }
                        lds_fence();
                        shared = true;
                        sh_batches += 1;
                        sh_nnz += group_sum<64>(mine ? (int)(a1 - a0) : 0);
                        sh_rows += nd;
                    }
                }
            }
        }
        // the merge of one lane's row over B's columns cs and values vs;
        // range(k, &p, &e) gives head k's entries [p, e) there
        auto merge_row = [&](const int32_t* __restrict__ cs, const VT* __restrict__ vs, auto&& range) {
            // heads: column hk at position hp (end he) in B, scale ha; the
            // head's value is loaded when it is consumed.  IT is int32 when
            // nnz(B) fits.
            // With PRE (K = 8, where the registers are there) a head's value
            // is loaded with its column, so a step waits on no value load;
            // otherwise it is loaded when the head is consumed.
            constexpr bool PRE = K >= 8;
            int hk[K];
            double ha[K];
            double hv[PRE ? K : 1];
            IT hp[K], he[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                hk[k] = 0x7fffffff;
                ha[k] = 0.0;
                if constexpr (PRE) hv[k] = 0.0;
                hp[k] = 0;
                he[k] = 0;
                if (k < (int)(a1 - a0)) {
                    ha[k] = to_f64(aval[a0 + k]);
                    range(k, &hp[k], &he[k]);
                    if (hp[k] < he[k]) {
                        hk[k] = cs[hp[k]];
                        if constexpr (PRE) hv[k] = to_f64(vs[hp[k]]);
                    }
                }
            }
            const int so = (int)(incl - nn);
            int t = 0;
            while (true) {
                int m = hk[0];
#pragma unroll
                for (int k = 1; k < K; ++k) m = hk[k] < m ? hk[k] : m;
                if (m == 0x7fffffff) break;
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (hk[k] == m) {
                        if constexpr (PRE) {
                            acc += ha[k] * hv[k];
                            ++hp[k];
                            if (hp[k] < he[k]) {
                                hk[k] = cs[hp[k]];
                                hv[k] = to_f64(vs[hp[k]]);
                            } else {
                                hk[k] = 0x7fffffff;
                            }
                        } else {
                            acc += ha[k] * to_f64(vs[hp[k]]);
                            ++hp[k];
                            hk[k] = hp[k] < he[k] ? cs[hp[k]] : 0x7fffffff;
                        }
                    }
                if (t < nn) { st_k[w][so + t] = m; st_v[w][so + t] = acc; }
                ++t;
            }
            if (cnt_out) cnt_out[row] = t <= nn ? t : -1;
            else if (t != nn) err |= 2;
        };
        if (mine) {
            if (SHARE && shared) {
                // head k's B row is distinct row number rank(d) of the stage
                merge_row(sh_col[w], sh_val[w], [&](int k, IT* p, IT* e) {
                    const int d = (int)(acol[a0 + k] + bo - kmin);
                    const int wd = d >> 6;
                    const int rk = sh_wr[w][wd] + __builtin_popcountll(sh_bm[w][wd] & ((1ull << (d & 63)) - 1ull));
                    *p = (IT)sh_off[w][rk];
                    *e = (IT)sh_off[w][rk + 1];
                });
            } else {
                merge_row(bcol, bval, [&](int k, IT* p, IT* e) {
                    const long long kk = acol[a0 + k] + bo;
                    *p = (IT)brp[kk];
                    *e = (IT)brp[kk + 1];
                });
            }
        }
        // rows with more than K A entries: groups of them whose A entries
        // and products each fit the 64 lanes go through a register sort;
        // the rest, the whole wave with an LDS hash, one row at a time
        uint64_t fb = merge_fallback_sorted<VT>(__ballot(in && !mine), a0, a1, bo, nn, row, st_off[w], st_k[w],
                                                st_v[w], acol, aval, brp, bcol, bval, cnt_out, &err);
        while (fb) {                                   // wave-uniform
            const int r = __builtin_ctzll(fb);
            fb &= fb - 1;
            const long long fa0 = __shfl(a0, r), fa1 = __shfl(a1, r), fbo = __shfl(bo, r);
            const long long fnn = __shfl(nn, r);
            const int frow = __shfl(row, r);
            const int fso = st_off[w][r];
            int fe = 0;
            for (int i = lane; i < FT; i += 64) { fb_keys[w][i] = kEmpty; fb_vals[w][i] = 0.0; }
            lds_fence();
            for (long long p = fa0; p < fa1; ++p) {
                const long long kk = acol[p] + fbo;
                const double a = to_f64(aval[p]);
                const long long q1 = brp[kk + 1];
                for (long long q = brp[kk] + lane; q < q1; q += 64) {
                    const int h = hash_slot_of<FT>(fb_keys[w], bcol[q], &fe);
                    if (h >= 0) atomicAdd(&fb_vals[w][h], a * to_f64(bval[q]));
                }
            }
            const bool failed = __ballot(fe != 0) != 0;
            lds_fence();
            int c = 0;
            for (int sl = lane; sl < FT; sl += 64) {
                const uint32_t key = (uint32_t)fb_keys[w][sl];
                if (key == (uint32_t)kEmpty) continue;
                int rank = 0;
                for (int f = 0; f < FT; f += 4) {
                    const int4 q = *reinterpret_cast<const int4*>(&fb_keys[w][f]);
                    rank += ((uint32_t)q.x < key) + ((uint32_t)q.y < key) + ((uint32_t)q.z < key) +
                            ((uint32_t)q.w < key);
                }
                if (rank < fnn) { st_k[w][fso + rank] = (int32_t)key; st_v[w][fso + rank] = fb_vals[w][sl]; }
                ++c;
            }
            c = group_sum<64>(c);
            if (cnt_out) {
                if (lane == 0) cnt_out[frow] = (failed || c > fnn) ? -1 : c;
            } else {
                if (failed) err |= 1;
                if (c != fnn) err |= 2;
            }
            lds_fence();
        }
        lds_fence();
        // copy the batch's staged rows to C
        const int total = st_off[w][nb];
        if (!perm) {
            const long long cb = st_c0[w][0];       // consecutive rows: one contiguous range
            for (int i = lane; i < total; i += 64) {
                ccol[cb + i] = st_k[w][i];
                cval[cb + i] = (VT)st_v[w][i];
            }
        } else {
            for (int i = lane; i < total; i += 64) {
                int lo2 = 0, hi2 = nb;                  // row r with st_off[r] <= i < st_off[r+1]
                while (hi2 - lo2 > 1) {
                    const int mid = (lo2 + hi2) >> 1;
                    if (st_off[w][mid] <= i) lo2 = mid; else hi2 = mid;
                }
                const long long dst = st_c0[w][lo2] + (i - st_off[w][lo2]);
                ccol[dst] = st_k[w][i];
                cval[dst] = (VT)st_v[w][i];
            }
        }
        lds_fence();
        pos += nb;
    }
    if (SHARE && lane == 0 && sh_batches) {
        atomicAdd(reinterpret_cast<unsigned long long*>(&info->share_batches), sh_batches);
        atomicAdd(reinterpret_cast<unsigned long long*>(&info->share_nnz), sh_nnz);
        atomicAdd(reinterpret_cast<unsigned long long*>(&info->share_rows), sh_rows);
    }
    if (err & 1) atomicOr(&info->err, kErrProbe);
    if (err & 2) atomicOr(&info->err, kErrCount);
}

// ===========================================================================
// Exclusive prefix sum of row_nnz -> row_ptr (int64), fused with the
// numeric binning histogram
// ===========================================================================

// Single-pass prefix sum with decoupled look-back (Merrill and Garland,
// 2016).  Workgroups take tiles in ticket order; each publishes its tile
// total, then walks back over its predecessors' published totals until it
// meets an inclusive prefix.  A state word packs a 2-bit flag, a 16-bit
// epoch (the call's number, so that no clearing pass is needed between
// calls) and a 46-bit value.  The wait is bounded and reports instead of
// spinning forever.
constexpr int kFlagAgg = 1, kFlagIncl = 2;
constexpr unsigned long long kValMask = (1ull << 46) - 1;

__device__ __forceinline__ unsigned long long scan_word(int flag, int epoch, long long v) {
    return ((unsigned long long)flag << 62) | ((unsigned long long)(epoch & 0xffff) << 46) |
           ((unsigned long long)v & kValMask);
}

static __global__ void __launch_bounds__(kScanBS)
k_scan_lookback(int m, const int32_t* __restrict__ cnt, unsigned long long* tile_state, int epoch,
                int64_t* __restrict__ row_ptr, BinTable bins, DevInfo* info, HostSummary* hs, int seq) {
    __shared__ BlockScanSmem<kScanBS> sm;
    __shared__ int hist[kNB];
    __shared__ int s_tile;
    __shared__ int s_neg;
    __shared__ long long s_prefix;
    if (threadIdx.x < kNB) hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_neg = 0;
    if (threadIdx.x == 0) s_tile = atomicAdd(&info->scan_ticket, 1);
    __syncthreads();
    const int tile = s_tile;
    if (tile >= (int)gridDim.x) {            // tickets not reset: report, touch nothing
        if (threadIdx.x == 0) atomicOr(&info->err, kErrScan);
        return;
    }
    const long long base = (long long)tile * kScanTile + (long long)threadIdx.x * kScanPer;
    static_assert(kScanPer == 8, "the vector path loads two int4");
    int v[kScanPer];
    long long s = 0;
    int neg = 0;
    const bool full = base + kScanPer <= m;
    if (full && ((uintptr_t)cnt & 15) == 0) {
        const int4 q0 = *reinterpret_cast<const int4*>(cnt + base);
        const int4 q1 = *reinterpret_cast<const int4*>(cnt + base + 4);
        v[0] = q0.x; v[1] = q0.y; v[2] = q0.z; v[3] = q0.w;
        v[4] = q1.x; v[5] = q1.y; v[6] = q1.z; v[7] = q1.w;
    } else {
#pragma unroll
        for (int i = 0; i < kScanPer; ++i) v[i] = base + i < m ? cnt[base + i] : 0;
    }
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        if (v[i] < 0) { ++neg; v[i] = 0; }   // an overflowed row: counted, sums as 0
        s += v[i];
    }
    if (__ballot(neg != 0)) {
        int wn = neg;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) wn += __shfl_xor(wn, d);
        if ((threadIdx.x & 63) == 0 && wn) atomicAdd(&s_neg, wn);
    }
    // the tile's numeric bin histogram (before the tile publishes its state)
    if (bins.nb > 0) {
        // a thread's rows usually share one bin: one weighted add then
        const int b0 = base < m ? bin_of(bins, v[0]) : -1;
        int nv = 0;
        bool same = true;
#pragma unroll
        for (int i = 0; i < kScanPer; ++i)
            if (base + i < m) {
                ++nv;
                same = same && bin_of(bins, v[i]) == b0;
            }
        if (__ballot(!same) == 0) {
            wave_hist_add_w(hist, b0, nv);
        } else {
#pragma unroll
            for (int i = 0; i < kScanPer; ++i)
                wave_hist_add(hist, base + i < m ? bin_of(bins, v[i]) : -1);
        }
    }
    long long tot;
    const long long incl = block_incl_scan<kScanBS>(s, sm, &tot);   // (its barriers complete hist, s_neg)
    if (threadIdx.x < 64) {
        // wave 0: add the tile's bins and overflow count to the global
        // counters, publish the tile total (the release orders those adds
        // before it), then look back over 64 predecessor states per round
        // trip until an inclusive prefix is found
        const int lane = threadIdx.x;
        if (bins.nb > 0 && lane < kNB && hist[lane]) atomicAdd(&info->num_part[tile % kParts][lane], hist[lane]);
        if (lane == 0 && s_neg) atomicAdd(&info->neg_count, s_neg);
        if (lane == 0)
            __hip_atomic_store(&tile_state[tile], scan_word(tile == 0 ? kFlagIncl : kFlagAgg, epoch, tot),
                               __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        long long prefix = 0;
        int p = tile - 1;                       // nearest predecessor not yet added
        long long spins = 0;
        while (p >= 0) {
            const int idx = p - lane;           // lane 0 reads the nearest one
            int flag = kFlagIncl, ep = epoch & 0xffff;
            long long val = 0;                  // before tile 0: an empty inclusive prefix
            if (idx >= 0) {
                const unsigned long long wd =
                    __hip_atomic_load(&tile_state[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                flag = (int)(wd >> 62);
                ep = (int)((wd >> 46) & 0xffff);
                val = (long long)(wd & kValMask);
            }
            const bool ready = flag != 0 && ep == (epoch & 0xffff);
            const uint64_t incl_mask = __ballot(ready && flag == kFlagIncl);
            const uint64_t wait_mask = __ballot(!ready);
            const int first = incl_mask ? __builtin_ctzll(incl_mask) : 64;
            const uint64_t need = first >= 63 ? ~0ull : ((2ull << first) - 1);
            if (wait_mask & need) {             // a state we need is not published yet
                // (the row pointers are then wrong: the call reports the error)
                if (++spins > (1LL << 26)) { if (lane == 0) atomicOr(&info->err, kErrScan); break; }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            long long part = lane <= first ? val : 0;
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) part += __shfl_xor(part, d);
            prefix += part;
            if (first < 64) break;
            p -= 64;
        }
        // the states read above were published with release stores: this
        // fence makes the counters added before them visible from here on
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (lane == 0) {
            if (tile > 0)
                __hip_atomic_store(&tile_state[tile], scan_word(kFlagIncl, epoch, prefix + tot), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            s_prefix = prefix;
        }
    }
    __syncthreads();
    long long run = s_prefix + incl - s;
    long long rp[kScanPer];
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        rp[i] = run;
        run += v[i];
    }
    if (row_ptr) {
        if (full && ((uintptr_t)row_ptr & 15) == 0) {
#pragma unroll
            for (int i = 0; i < kScanPer; i += 2)
                *reinterpret_cast<longlong2*>(row_ptr + base + i) = make_longlong2(rp[i], rp[i + 1]);
        } else {
#pragma unroll
            for (int i = 0; i < kScanPer; ++i)
                if (base + i < m) row_ptr[base + i] = rp[i];
        }
    }
    if (m > 0 && base <= m - 1 && m - 1 < base + kScanPer) {
        if (row_ptr) row_ptr[m] = run;     // the thread holding row m-1 closes row_ptr
        info->nnz = run;
    }
    if (m == 0 && tile == 0 && threadIdx.x == 0) {
        if (row_ptr) row_ptr[0] = 0;
        info->nnz = 0;
    }
    // The tile of the last rows has seen every other tile's state (directly
    // or through an inclusive prefix), so every tile's counters are in: it
    // publishes the host summary.
    if (hs && tile == (int)gridDim.x - 1) {
        if (threadIdx.x < kNB) {
            int c = 0;
            if ((int)threadIdx.x <= bins.nb)
                for (int p = 0; p < kParts; ++p) c += load_coherent(&info->num_part[p][threadIdx.x]);
            hs->counts[threadIdx.x] = c;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            hs->nnz = s_prefix + tot;
            hs->err = load_coherent(&info->err);
            hs->neg_count = load_coherent(&info->neg_count);
            __threadfence_system();
            __hip_atomic_store(&hs->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// ===========================================================================
// Numeric pass with in-row column sort
// ===========================================================================

// Column order of a row's n (<= 64 R) distinct outputs held by one wave:
// the (column, slot) pairs kt[0..n) are sorted ascending by a bitonic
// network over 64 R elements (element e = r 64 + lane, pads last), lane
// shuffles for partners in other lanes and register swaps for partners in
// the lane's other registers; element e then goes to position e of the row
// with its slot's value (coalesced stores).
template <int R, typename VT>
__device__ __forceinline__ void wave_sort_out(const int32_t* kt, const double* vt, int n, int32_t* oc, VT* ov,
                                              int lane) {
    constexpr int N = 64 * R;
    unsigned long long x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = r * 64 + lane;
        x[r] = e < n ? ((unsigned long long)(unsigned)kt[e] << 32) | (unsigned)e : ~0ull;
    }
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int rr = r ^ (j >> 6);
                    if (rr > r) {
                        const bool up = ((r * 64 + lane) & k) == 0;
                        const unsigned long long a = x[r], b = x[rr];
                        if (up ? a > b : a < b) {
                            x[r] = b;
                            x[rr] = a;
                        }
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const unsigned long long o = __shfl_xor(x[r], j);
                    const bool up = ((r * 64 + lane) & k) == 0, low = (lane & j) == 0;
                    x[r] = (low == up) ? (o < x[r] ? o : x[r]) : (o > x[r] ? o : x[r]);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = r * 64 + lane;
        if (e < n) {
            oc[e] = (int32_t)(x[r] >> 32);
            ov[e] = (VT)vt[(unsigned)x[r]];
        }
    }
}

// Numeric, sub-wave lane groups.  T slots of (int32 key, FP64 value); a row
// with r = row_nnz_i <= T/2 entries.  After accumulation the occupied slots
// are compacted (group ballot) and each entry's output position is its
// rank among the row's keys (keys are distinct): for a whole-wave row whose
// columns span less than 32 T, from a bitmap of the span, else counted with
// 16-byte LDS reads (or, past 160 entries, by a sort across the wave).
// Other whole-wave rows of at least 64 entries are ordered through 64
// buckets of equal column width when no bucket holds more than kBucketMax
// keys.  Per-group LDS rows are padded so groups start on different banks.
constexpr int kBucketMax = 24;
template <int G, int T, typename VT, bool BATCH = false>
__global__ void __launch_bounds__(256)
k_num_group(Work wk,
            const int64_t* __restrict__ arp, const int32_t* __restrict__ acol, const VT* __restrict__ aval,
            const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol, const VT* __restrict__ bval,
            const int64_t* __restrict__ crp, int32_t* __restrict__ ccol, VT* __restrict__ cval,
            int32_t* __restrict__ cnt_out, DevInfo* info, RowMap mp) {
    int nrows_bin;
    const int32_t* perm;
    work_rows(wk, &nrows_bin, &perm);
    constexpr int NG = GroupCfg<G>::NG;
    static_assert(T % G == 0, "the table clears in T / G whole steps of the group");
    // (rows of 16-byte multiples: the rank count reads four keys at a time;
    // the occupied slots are compacted to the front of the table in place)
    __shared__ __align__(16) int32_t keys[NG][T + 4];
    __shared__ double vals[NG][T + 1];
    __shared__ long long s_off[NG][G + 1];
    __shared__ long long s_bst[NG][G + 1];
    __shared__ double s_a[NG][G + 1];
    const int lane = threadIdx.x & 63;
    const int gl = threadIdx.x & (G - 1);
    const int g = threadIdx.x / G;
    int err = 0;
    int32_t* kt = keys[g];
    double* vt = vals[g];
    // persistent: workgroup lb owns the contiguous slot range [lo, hi)
    const long long per = (nrows_bin + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)xcd_block() * per;
    const long long hi = lo + per < nrows_bin ? lo + per : nrows_bin;
    for (long long slot = lo + g; slot < hi; slot += NG) {      // group-uniform
    const int row = perm ? perm[slot] : (int)slot;
    const long long bo = row_boff<BATCH>(mp, row);
    int re = 0;                                  // this row's table overflowed
    const long long a0 = arp[row], a1 = arp[row + 1];
    const long long rp = crp[row];
    const int expect = (int)(crp[row + 1] - rp);
    // a whole-wave row of one chunk with as many products as outputs has no
    // two products in one column: they go straight to the table's first
    // slots, without the hash and the compaction
    bool direct = false;
    if (a1 <= a0) {
#pragma unroll
        for (int i = 0; i < T / G; ++i) { kt[gl + i * G] = kEmpty; vt[gl + i * G] = 0.0; }
        lds_fence();
    }
    for (long long c0 = a0; c0 < a1; c0 += G) {
        const long long p = c0 + gl;
        long long len = 0, bst = 0;
        double a = 0.0;
        if (p < a1) {
            const long long k = acol[p] + bo;
            a = to_f64(aval[p]);
            bst = brp[k];
            len = brp[k + 1] - bst;
        }
        const long long incl = group_incl_scan<G>(len, gl);
        const long long total = __shfl(incl, G - 1, G);
        s_off[g][gl] = incl;
        s_bst[g][gl] = bst - (incl - len);
        s_a[g][gl] = a;
        if (c0 == a0) {                              // group-uniform
            direct = G == 64 && !cnt_out && a1 - a0 <= G && total == expect && total <= T / 2;
            if (!direct) {
#pragma unroll
                for (int i = 0; i < T / G; ++i) { kt[gl + i * G] = kEmpty; vt[gl + i * G] = 0.0; }
            }
        }
        lds_fence();
        const int nact = (int)((a1 - c0) < G ? (a1 - c0) : G);
        int t = -1;                                  // owner of q: one search, then it only moves forward
        if (direct) {
            for (long long q = gl; q < total; q += G) {
                if (t < 0) t = owner_search(s_off[g], nact, q);
                else while (s_off[g][t] <= q) ++t;
                const long long bi = s_bst[g][t] + q;
                kt[q] = bcol[bi];
                vt[q] = 0.0 + s_a[g][t] * to_f64(bval[bi]);      // (a sum from zero, as in the table: -0 becomes +0)
            }
        } else {
            for (long long q = gl; q < total; q += G) {
                if (t < 0) t = owner_search(s_off[g], nact, q);
                else while (s_off[g][t] <= q) ++t;
                const long long bi = s_bst[g][t] + q;
                const int32_t j = bcol[bi];
                const double prod = s_a[g][t] * to_f64(bval[bi]);
                const int h = hash_slot_of<T>(kt, j, &re);
                if (h >= 0) atomicAdd(&vt[h], prod);
            }
        }
        lds_fence();
    }
    // compact the occupied slots to the front, in place: a slot moves to a
    // position no later than its own, and the group reads its G slots before
    // any of them is written
    int n = direct ? expect : 0;
    if (!direct) {
#pragma unroll
        for (int s0 = 0; s0 < T; s0 += G) {
            const int s = s0 + gl;
            const int32_t k = kt[s];
            const double v = vt[s];
            const bool occ = k != kEmpty;
            const uint64_t mask = group_ballot<G>(occ, lane);
            if (occ) {
                const int pos = n + __builtin_popcountll(mask & ((1ull << gl) - 1));
                kt[pos] = k;
                vt[pos] = v;
            }
            n += __builtin_popcountll(mask);
        }
    }
    const bool failed = group_ballot<G>(re != 0, lane) != 0;
    if (cnt_out) {                               // capacity mode
        const bool fits = !failed && n <= expect && n <= T / 2;
        if (gl == 0) cnt_out[row] = fits ? n : -1;
        if (!fits) { lds_fence(); continue; }
    } else if (failed || n != expect || n > T / 2) {
        if (gl == 0) atomicOr(&info->err, failed ? kErrProbe : kErrCount);
        lds_fence();
        continue;
    }
    if constexpr (G == 64) {
        // rows whose columns span less than 32 T: column order from a
        // bitmap of the span (the free upper half of the value table, T / 2
        // words) and a rank per word (the free upper half of the key
        // table), O(n / 64 + T / 128) steps a lane instead of a sort
        int kmn = 0x7fffffff, kmx = -1;
        for (int e = lane; e < n; e += 64) {
            kmn = min(kmn, kt[e]);
            kmx = max(kmx, kt[e]);
        }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) {
            kmn = min(kmn, __shfl_xor(kmn, d));
            kmx = max(kmx, __shfl_xor(kmx, d));
        }
        if (n > 0 && (long long)kmx - kmn < 32LL * T) {       // wave-uniform
            unsigned long long* bm = reinterpret_cast<unsigned long long*>(vt + T / 2);
            int* wr = kt + T / 2;
            const int nwd = ((kmx - kmn) >> 6) + 1;            // <= T / 2
            for (int i = lane; i < nwd; i += 64) bm[i] = 0ull;
            lds_fence();
            for (int e = lane; e < n; e += 64) {
                const int d = kt[e] - kmn;
                atomicOr(&bm[d >> 6], 1ull << (d & 63));
            }
            lds_fence();
            // lane l ranks the E consecutive words from l E
            const int E = (nwd + 63) >> 6;
            const int i0 = lane * E, i1 = min(i0 + E, nwd);
            int loc = 0;
            for (int i = i0; i < i1; ++i) loc += __builtin_popcountll(bm[i]);
            int run = (int)group_incl_scan<64>(loc, lane) - loc;
            for (int i = i0; i < i1; ++i) {
                wr[i] = run;
                run += __builtin_popcountll(bm[i]);
            }
            lds_fence();
            for (int e = lane; e < n; e += 64) {
                const int32_t k = kt[e];
                const int d = k - kmn;
                const int rank = wr[d >> 6] + __builtin_popcountll(bm[d >> 6] & ((1ull << (d & 63)) - 1ull));
                ccol[rp + rank] = k;
                cval[rp + rank] = (VT)vt[e];
            }
            lds_fence();
            continue;
        }
        // (the counters and slots below need T >= 256)
        if (T >= 256 && n >= 64) {                            // wave-uniform
            // wider rows: the keys counted into 64 buckets of equal column
            // width, placed bucket by bucket, and each ranked by comparison
            // within its bucket; taken while no bucket holds more than
            // kBucketMax keys (else the sort or the rank count below)
            int* cnt = reinterpret_cast<int*>(vt + T / 2);    // the free upper half
            int* cur = cnt + 64;
            int* sidx = cur + 64;                             // n <= T / 2 entries
            int32_t* skey = kt + T / 2;                       // n <= T / 2 entries
            const float scale = 64.0f / (float)((long long)kmx - kmn + 1);
            auto bucket = [&](int32_t k) { return min(63, (int)((float)(k - kmn) * scale)); };
            cnt[lane] = 0;
            lds_fence();
            for (int e = lane; e < n; e += 64) atomicAdd(&cnt[bucket(kt[e])], 1);
            lds_fence();
            const int c = cnt[lane];
            int cmax = c;
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) cmax = max(cmax, __shfl_xor(cmax, d));
            if (cmax <= kBucketMax) {                         // wave-uniform
                cur[lane] = (int)group_incl_scan<64>(c, lane) - c;
                lds_fence();
                for (int e = lane; e < n; e += 64) {
                    const int32_t k = kt[e];
                    const int slot = atomicAdd(&cur[bucket(k)], 1);
                    skey[slot] = k;
                    sidx[slot] = e;
                }
                lds_fence();
                // cur[b] is now the end of bucket b
                for (int sl = lane; sl < n; sl += 64) {
                    const int32_t k = skey[sl];
                    const int b = bucket(k);
                    const int b1 = cur[b], b0 = b1 - cnt[b];
                    int rank = b0;
                    for (int j = b0; j < b1; ++j) rank += skey[j] < k;
                    ccol[rp + rank] = k;
                    cval[rp + rank] = (VT)vt[sidx[sl]];
                }
                lds_fence();
                continue;
            }
        }
    }
    if constexpr (G == 64 && T / 2 > 128) {
        // long rows: a bitonic sort across the wave (the rank count below
        // costs n / 4 LDS reads and n compares per output, n / 64 outputs a
        // lane; the sort of T / 2 elements costs less from about 160 on)
        if (n > 160) {                                  // wave-uniform (a row per wave)
            lds_fence();
            wave_sort_out<T / 128>(kt, vt, n, ccol + rp, cval + rp, lane);
            lds_fence();
            continue;
        }
    }
    const int n4 = (n + 3) & ~3;
    if (gl < n4 - n) kt[n + gl] = 0x7fffffff;         // pads sort after every key
    lds_fence();
    for (int e = gl; e < n; e += G) {
        const int32_t k = kt[e];
        int rank = 0;
        for (int f = 0; f < n4; f += 4) {
            const int4 q = *reinterpret_cast<const int4*>(&kt[f]);
            rank += (q.x < k) + (q.y < k) + (q.z < k) + (q.w < k);
        }
        ccol[rp + rank] = k;
        cval[rp + rank] = (VT)vt[e];
    }
    lds_fence();
    }
    if (err) atomicOr(&info->err, kErrProbe);
}

// Numeric, one workgroup per row: LDS hash of T (key, FP64) slots, then the
// occupied slots are compacted to the front and put in column order: rows of
// at most kBlockRankMax outputs by counting each key's smaller keys, longer
// rows by a radix sort of (column, slot) pairs when their columns span less
// than 2^20, else by a bitonic sort with its short-range stages in the
// waves' registers; then coalesced stores.
constexpr int kBlockRankMax = 512;
template <int BS, int T, typename VT, bool BATCH = false>
__global__ void __launch_bounds__(BS)
k_num_block(Work wk,
            const int64_t* __restrict__ arp, const int32_t* __restrict__ acol, const VT* __restrict__ aval,
            const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol, const VT* __restrict__ bval,
            const int64_t* __restrict__ crp, int32_t* __restrict__ ccol, VT* __restrict__ cval,
            int32_t* __restrict__ cnt_out, DevInfo* info, RowMap mp,
            unsigned* q) {
    int nrows_bin;
    const int32_t* perm;
    work_rows(wk, &nrows_bin, &perm);
    __shared__ long long s_slot;
    constexpr int PER = T / BS;    // slots per thread in the compaction
    static_assert(PER >= 1, "T must be >= BS");
    __shared__ __align__(16) int32_t keys[T];
    __shared__ double vals[T];
    // the A entries' product offsets and B positions; the sort's digit
    // counters take their place afterwards
    __shared__ __align__(16) long long s_ob[2 * BS];
    long long* const s_off = s_ob;
    long long* const s_bst = s_ob + BS;
    __shared__ double s_a[BS];
    __shared__ BlockScanSmem<BS> sm;
    __shared__ int s_fail;
    __shared__ int s_mm[2][BS / 64];
    const int tid = threadIdx.x;
    int err = 0;
    for (long long slot = block_first(q, &s_slot); slot < nrows_bin; slot = block_next(q, slot, &s_slot)) {
        const int row = perm ? perm[slot] : (int)slot;
        const long long bo = row_boff<BATCH>(mp, row);
        for (int s = tid; s < T; s += BS) { keys[s] = kEmpty; vals[s] = 0.0; }
        if (tid == 0) s_fail = 0;
        __syncthreads();
        const long long a0 = arp[row], a1 = arp[row + 1];
        for (long long c0 = a0; c0 < a1; c0 += BS) {
            const long long p = c0 + tid;
            long long len = 0, bst = 0;
            double a = 0.0;
            if (p < a1) {
                const long long k = acol[p] + bo;
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
            int t = -1;                     // owner of q: one search, then it only moves forward
            for (long long q = tid; q < total; q += BS) {
                if (t < 0) t = owner_search(s_off, nact, q);
                else while ((long long)s_off[t] <= q) ++t;
                const long long bi = s_bst[t] + q;
                const int32_t j = bcol[bi];
                const double prod = s_a[t] * to_f64(bval[bi]);
                int e2 = 0;
                const int h = hash_slot_of<T>(keys, j, &e2);
                if (h >= 0) atomicAdd(&vals[h], prod);
                else s_fail = 1;
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
        const bool failed = s_fail != 0;         // read after the scan's barriers
        const bool bad = cnt_out ? (failed || n > expect || n > T / 2) : (failed || n != expect || n > T / 2);
        if (cnt_out && tid == 0) cnt_out[row] = bad ? -1 : (int)n;
        if (!bad) {
#pragma unroll
            for (int i = 0; i < PER; ++i)
                if (rk[i] != kEmpty) { keys[pos] = rk[i]; vals[pos] = rv[i]; ++pos; }
        }
        int P = 1;
        while (P < n) P <<= 1;
        // pad to the sort's power of two, and to the rank count's four
        // (both within T: n <= T / 2)
        if (!bad)
            for (int s = (int)n + tid; s < (P < 4 ? 4 : P); s += BS) keys[s] = 0x7fffffff;   // sorts last
        __syncthreads();
        if (bad) {
            if (tid == 0 && !cnt_out) atomicOr(&info->err, failed ? kErrProbe : kErrCount);
            continue;
        }
        if (n <= kBlockRankMax) {
            // a short row: each key's rank is the number of smaller keys
            // (one pass over the padded keys, no barrier between stages)
            const int n4 = ((int)n + 3) & ~3;
            for (int e = tid; e < n; e += BS) {
                const int32_t k = keys[e];
                int rank = 0;
                for (int f = 0; f < n4; f += 4) {
                    const int4 q = *reinterpret_cast<const int4*>(&keys[f]);
                    rank += (q.x < k) + (q.y < k) + (q.z < k) + (q.w < k);
                }
                ccol[rp + rank] = k;
                cval[rp + rank] = (VT)vals[e];
            }
            __syncthreads();
            continue;
        }
        // a long row whose columns span less than 2^20: stable LSD radix sort
        // of (column - smallest column, slot) packed in 32 bits (slots take the
        // low 12 bits), 8 bits a pass.  Each wave ranks its chunk of elements
        // (lane order within 64-element steps, steps in order) against its own
        // digit counters, from the lanes that share its digit (8 ballots); an
        // exclusive scan of the counters in (digit, wave) order gives every
        // element its place in the other half of the key area.
        {
            constexpr int NW = BS / 64;
            const int lane = tid & 63, wv = tid >> 6;
            int mn = 0x7fffffff, mx = -1;
            for (int e = tid; e < n; e += BS) {
                const int k = keys[e];
                mn = k < mn ? k : mn;
                mx = k > mx ? k : mx;
            }
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) {
                mn = min(mn, __shfl_xor(mn, d));
                mx = max(mx, __shfl_xor(mx, d));
            }
            if (lane == 0) {
                s_mm[0][wv] = mn;
                s_mm[1][wv] = mx;
            }
            __syncthreads();
            mn = s_mm[0][0];
            mx = s_mm[1][0];
#pragma unroll
            for (int w = 1; w < NW; ++w) {
                mn = min(mn, s_mm[0][w]);
                mx = max(mx, s_mm[1][w]);
            }
            if (mx - mn < (1 << 20)) {                      // uniform
                constexpr int MAXI = (T / 2 + BS - 1) / BS;  // elements a lane
                constexpr int CH = MAXI * 64;                // elements a wave
                static_assert(T / 2 <= 4096, "slots take 12 bits");
                static_assert(NW * 256 == 4 * BS, "each thread scans four digit counters");
                unsigned* const buf = reinterpret_cast<unsigned*>(keys);     // two halves of T / 2 words
                int* const hist = reinterpret_cast<int*>(s_ob);              // [NW][256]
                unsigned x[MAXI];
#pragma unroll
                for (int i = 0; i < MAXI; ++i) {
                    const int e = wv * CH + i * 64 + lane;
                    x[i] = e < n ? ((unsigned)(keys[e] - mn) << 12) | (unsigned)e : 0u;
                }
                const int bits = 32 - __builtin_clz((unsigned)(mx - mn) | 1u);
                int half = 1;                                // half of the key area written next
                for (int sh = 12; sh < 12 + bits; sh += 8) {
                    __syncthreads();                         // the last pass's reads are done
                    for (int i = tid; i < NW * 256; i += BS) hist[i] = 0;
                    __syncthreads();
                    int pos[MAXI];
#pragma unroll
                    for (int i = 0; i < MAXI; ++i) {
                        const int e = wv * CH + i * 64 + lane;
                        const bool ok = e < n;
                        const int d = (int)((x[i] >> sh) & 255u);
                        uint64_t peers = __ballot(ok);
#pragma unroll
                        for (int b = 0; b < 8; ++b) {
                            const bool bit = (d >> b) & 1;
                            const uint64_t m = __ballot(bit);
                            peers &= bit ? m : ~m;
                        }
                        const int below = __builtin_popcountll(peers & ((1ull << lane) - 1ull));
                        int base = 0;
                        if (ok) base = hist[wv * 256 + d];
                        if (ok && below == 0) hist[wv * 256 + d] = base + __builtin_popcountll(peers);
                        pos[i] = base + below;
                    }
                    __syncthreads();
                    {
                        int v[4], sum = 0;
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const int f = tid * 4 + k;
                            v[k] = hist[(f % NW) * 256 + f / NW];
                            sum += v[k];
                        }
                        long long tot;
                        int run = (int)(block_incl_scan<BS>(sum, sm, &tot) - sum);
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const int f = tid * 4 + k;
                            hist[(f % NW) * 256 + f / NW] = run;
                            run += v[k];
                        }
                    }
                    __syncthreads();
                    unsigned* const dst = buf + half * (T / 2);
#pragma unroll
                    for (int i = 0; i < MAXI; ++i) {
                        const int e = wv * CH + i * 64 + lane;
                        if (e < n) dst[hist[wv * 256 + (int)((x[i] >> sh) & 255u)] + pos[i]] = x[i];
                    }
                    __syncthreads();
#pragma unroll
                    for (int i = 0; i < MAXI; ++i) {
                        const int e = wv * CH + i * 64 + lane;
                        x[i] = e < n ? dst[e] : 0u;
                    }
                    half ^= 1;
                }
#pragma unroll
                for (int i = 0; i < MAXI; ++i) {
                    const int e = wv * CH + i * 64 + lane;
                    if (e < n) {
                        ccol[rp + e] = (int32_t)((x[i] >> 12) + (unsigned)mn);
                        cval[rp + e] = (VT)vals[x[i] & 4095u];
                    }
                }
                __syncthreads();
                continue;
            }
        }
        // a long row: bitonic sort of P (column, slot) pairs (pads last).  The
        // pairs take the place of the keys (P <= T / 2 pairs of 8 bytes); the
        // values stay where they are and are read by slot at the end.  Stages
        // whose partners lie within one 128-element block run in a wave's
        // registers (lane shuffles; lane l holds elements 128 b + l and
        // 128 b + 64 + l), the others in LDS with a barrier each.
        {
            constexpr int MAXI = (T / 2 + BS - 1) / BS;
            int32_t kr[MAXI];
#pragma unroll
            for (int i = 0; i < MAXI; ++i) {
                const int e = tid + i * BS;
                kr[i] = e < n ? keys[e] : 0;
            }
            __syncthreads();
            unsigned long long* pk = reinterpret_cast<unsigned long long*>(keys);
#pragma unroll
            for (int i = 0; i < MAXI; ++i) {
                const int e = tid + i * BS;
                if (e < P) pk[e] = e < n ? ((unsigned long long)(unsigned)kr[i] << 32) | (unsigned)e : ~0ull;
            }
            __syncthreads();
            constexpr int NW = BS / 64;
            const int lane = tid & 63, wv = tid >> 6;
            // the stages j <= 64 of phases k0 .. k1, in registers
            auto wave_stages = [&](int k0, int k1) {
                for (int b = wv; b < P / 128; b += NW) {                // wave-uniform
                    const int e0 = 128 * b + lane, e1 = e0 + 64;
                    unsigned long long x0 = pk[e0], x1 = pk[e1];
                    for (int k = k0; k <= k1; k <<= 1) {
                        const bool up0 = (e0 & k) == 0, up1 = (e1 & k) == 0;
                        for (int jj = (k >> 1) < 64 ? (k >> 1) : 64; jj >= 1; jj >>= 1) {
                            if (jj == 64) {
                                if ((x0 > x1) == up0) {
                                    const unsigned long long t = x0;
                                    x0 = x1;
                                    x1 = t;
                                }
                            } else {
                                const unsigned long long o0 = __shfl_xor(x0, jj), o1 = __shfl_xor(x1, jj);
                                const bool low = (lane & jj) == 0;
                                x0 = (low == up0) ? (o0 < x0 ? o0 : x0) : (o0 > x0 ? o0 : x0);
                                x1 = (low == up1) ? (o1 < x1 ? o1 : x1) : (o1 > x1 ? o1 : x1);
                            }
                        }
                    }
                    pk[e0] = x0;
                    pk[e1] = x1;
                }
                __syncthreads();
            };
            wave_stages(2, 128);
            for (int k = 256; k <= P; k <<= 1) {
                for (int j = k >> 1; j >= 128; j >>= 1) {
                    for (int t = tid; t < P / 2; t += BS) {
                        const int i = 2 * j * (t / j) + (t % j);
                        const int l = i + j;
                        const bool up = (i & k) == 0;
                        const unsigned long long a = pk[i], c = pk[l];
                        if ((a > c) == up) {
                            pk[i] = c;
                            pk[l] = a;
                        }
                    }
                    __syncthreads();
                }
                wave_stages(k, k);
            }
            for (int e = tid; e < n; e += BS) {
                const unsigned long long x = pk[e];
                ccol[rp + e] = (int32_t)(x >> 32);
                cval[rp + e] = (VT)vals[(unsigned)x];
            }
        }
        __syncthreads();
    }
    block_slots_done(q);
    if (err) atomicOr(&info->err, kErrProbe);
}

// ===========================================================================
// Global bin: rows too large for the LDS hash bins
// ===========================================================================

// Products each thread of the slice kernel loads before using any: one
// workgroup per compute unit leaves few waves to hide the gathers.
constexpr int kProductUnroll = 4;

// Rows of the global bin (too large for the LDS hash bins), accumulated in
// LDS one column slice at a time.  The columns are taken in super-ranges
// whose bitmap fits the LDS (all of them at once when they fit).  For each
// super-range, the bitmap pass sets the row's column bitmap in LDS and
// keeps a copy of it in the workgroup's global scratch.  The super-range is
// then cut at 256-column block boundaries into slices whose bitmap segment,
// count of outputs before every segment word and FP64 accumulator (one
// entry per output of the slice) fit the same LDS together: a block costs
// 64 bytes plus 8 per output, and a slice takes the blocks whose running
// cost falls in one budget-sized interval.  For each slice, every A entry's
// B row is searched for the slice's column range, the products in it add
// into the accumulator with LDS atomics, and the segment goes out in column
// order from the slice's first output's position in C.  No accumulator
// atomic leaves LDS.
constexpr int kSliceBS = 1024;               // threads of the slice kernel
constexpr int kSliceMax = 256;               // slices per row
constexpr int kSliceBlockFixed = 8 * 4 + 8 * 4;          // a 256-column block's bitmap words and word ranks
constexpr int kSliceBlockCost = kSliceBlockFixed + 8 * 256;   // most bytes one block can need

__device__ __forceinline__ long long lower_bound_col(const int32_t* __restrict__ col, long long lo, long long hi,
                                                     long long c) {
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if ((long long)col[mid] < c) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <int BS, typename VT, bool BATCH = false, bool MULTI = false>
__global__ void __launch_bounds__(BS)
k_num_slice(Work wk, long long ncols, long long span,
            const int64_t* __restrict__ arp, const int32_t* __restrict__ acol, const VT* __restrict__ aval,
            const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol, const VT* __restrict__ bval,
            const int64_t* __restrict__ crp, int32_t* __restrict__ ccol, VT* __restrict__ cval,
            uint32_t* __restrict__ gbm, long long lds_bytes, int32_t* __restrict__ cnt_out, DevInfo* info,
            RowMap mp,
            unsigned* q) {
    int nrows_bin;
    const int32_t* perm;
    work_rows(wk, &nrows_bin, &perm);
    __shared__ long long s_slot;
    constexpr int RU = kProductUnroll;
    extern __shared__ __align__(16) uint32_t dyn_slice[];   // bitmap; then a slice's segment and accumulator
    uint32_t* const dyn_smem = dyn_slice;
    __shared__ long long s_off[BS];
    __shared__ long long s_bst[BS];
    __shared__ double s_a[BS];
    __shared__ BlockScanSmem<BS> sm;
    __shared__ int s_sb[kSliceMax + 1];         // first 256-column block of each slice
    __shared__ int s_sr[kSliceMax];             // rank of each slice's first output
    __shared__ int s_ns;
    const int tid = threadIdx.x;
    const long long budget = lds_bytes - kSliceBlockCost - 16;   // > kSliceBlockCost (host); 16: alignment pad
    const long long span_words = (span + 31) >> 5;
    uint32_t* gb = gbm + (long long)blockIdx.x * span_words;
    for (long long slot = block_first(q, &s_slot); slot < nrows_bin; slot = block_next(q, slot, &s_slot)) {
        const int row = perm ? perm[slot] : (int)slot;
        const long long bo = row_boff<BATCH>(mp, row);
        const long long a0 = arp[row], a1 = arp[row + 1];
        const long long rp = crp[row];
        const long long rend = crp[row + 1];
        // a row whose A entries fit one chunk keeps, per thread, its entry's
        // B-row range in the current super-range and the position where the
        // previous slice ended: one search per slice and super-range
        const bool one_chunk = a1 - a0 <= BS;
        long long sr_lo = -1, sr_hi = -1, cur = -1;
        long long done = 0;                            // outputs of the super-ranges before
        bool bad = false;
        // Column super-ranges [C0, C1) whose bitmap fits the LDS; the
        // instance for ncols <= span (MULTI false) takes all columns at once
        for (long long C0 = 0; C0 < ncols && !bad; C0 += span) {
            const long long C1 = MULTI && C0 + span < ncols ? C0 + span : ncols;
            const bool whole = !MULTI || (C0 == 0 && C1 == ncols);
            const long long words = (C1 - C0 + 31) >> 5;
            const long long nr8 = (words + 7) >> 3;    // 256-column blocks
            uint32_t* bm = dyn_smem;
            __syncthreads();                           // the previous super-range is done with LDS
            for (long long w = tid; w < words; w += BS) bm[w] = 0u;
            __syncthreads();
            // bitmap pass: the row's columns in [C0, C1)
            for (long long c0 = a0; c0 < a1; c0 += BS) {
                const long long p = c0 + tid;
                long long len = 0, bst = 0;
                if (p < a1) {
                    const long long k = acol[p] + bo;
                    long long lo = brp[k], hi = brp[k + 1];
                    if (!whole) {
                        lo = one_chunk && sr_hi >= 0 ? sr_hi : lower_bound_col(bcol, lo, hi, C0);
                        if (C1 < ncols) hi = lower_bound_col(bcol, lo, hi, C1);
                    }
                    if (one_chunk) { sr_lo = lo; sr_hi = hi; }
                    bst = lo;
                    len = hi - lo;
                }
                long long total;
                const long long incl = block_incl_scan<BS>(len, sm, &total);
                s_off[tid] = incl;
                s_bst[tid] = bst - (incl - len);
                __syncthreads();
                const int nact = (int)((a1 - c0) < BS ? (a1 - c0) : BS);
                int t = -1;
                for (long long q0 = tid; q0 < total; q0 += RU * BS) {
                    int32_t j[RU];
#pragma unroll
                    for (int u = 0; u < RU; ++u) {
                        const long long q = q0 + (long long)u * BS;
                        j[u] = -1;
                        if (q < total) {
                            if (t < 0) t = owner_search(s_off, nact, q);
                else while ((long long)s_off[t] <= q) ++t;
                            j[u] = (int32_t)(bcol[s_bst[t] + q] - C0);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < RU; ++u)
                        if (j[u] >= 0) atomicOr(&bm[j[u] >> 5], 1u << (j[u] & 31));
                }
                __syncthreads();
            }
            // the bitmap's copy and the slices; a block costs F + 8 c bytes (c
            // its outputs), so the outputs before block i are (cost before i -
            // F i) / 8
            long long nsr;                             // outputs of this super-range
            {
                const long long E = (nr8 + BS - 1) / BS;
                const long long i0 = (long long)tid * E, i1 = i0 + E < nr8 ? i0 + E : nr8;
                long long loc = 0;
                for (long long w = 8 * i0; w < 8 * i1 && w < words; ++w) loc += __builtin_popcount(bm[w]);
                const long long cost = kSliceBlockFixed * (i1 > i0 ? i1 - i0 : 0) + 8 * loc;
                long long ctot;
                long long pc = block_incl_scan<BS>(cost, sm, &ctot) - cost;   // running cost before block i0
                nsr = (ctot - kSliceBlockFixed * nr8) / 8;
                for (long long i = i0; i < i1; ++i) {
                    const long long prev = pc;
                    long long c = 0;
                    for (long long w = 8 * i; w < 8 * i + 8 && w < words; ++w) c += __builtin_popcount(bm[w]);
                    pc += kSliceBlockFixed + 8 * c;
                    const long long sid = (pc - 1) / budget;
                    if ((i == 0 || sid != (prev - 1) / budget) && sid < kSliceMax) {
                        s_sb[sid] = (int)i;
                        s_sr[sid] = (int)((prev - kSliceBlockFixed * i) / 8);
                    }
                }
                if (tid == 0) {
                    const long long n = nr8 > 0 ? (ctot - 1) / budget + 1 : 0;
                    s_ns = n <= kSliceMax ? (int)n : -1;
                    if (n <= kSliceMax) s_sb[n] = (int)nr8;
                }
                for (long long w = tid; w < words; w += BS) gb[w] = bm[w];
            }
            __syncthreads();
            const int ns = s_ns;
            if (ns < 0) {                              // uniform; the host bounds the slice count
                bad = true;
                break;
            }
            cur = sr_lo;
            for (int sl = 0; sl < ns; ++sl) {
                const long long b0 = s_sb[sl], b1 = s_sb[sl + 1];
                const long long w0 = 8 * b0, w1 = 8 * b1 < words ? 8 * b1 : words;
                const long long nw = w1 - w0;
                const long long c_lo = C0 + w0 * 32, c_hi = C0 + w1 * 32 < C1 ? C0 + w1 * 32 : C1;
                uint32_t* sbm = dyn_smem;
                int* swr = reinterpret_cast<int*>(dyn_smem + nw);          // outputs before each segment word
                double* acc = reinterpret_cast<double*>(dyn_smem + 2 * nw);
                __syncthreads();                       // the previous slice (or the bitmap) is done with LDS
                for (long long w = tid; w < nw; w += BS) sbm[w] = gb[w0 + w];
                __syncthreads();
                long long nout;                        // outputs of the slice
                {
                    const long long E = (nw + BS - 1) / BS;
                    const long long i0 = (long long)tid * E, i1 = i0 + E < nw ? i0 + E : nw;
                    long long loc = 0;
                    for (long long w = i0; w < i1; ++w) loc += __builtin_popcount(sbm[w]);
                    long long tot;
                    long long run = block_incl_scan<BS>(loc, sm, &tot) - loc;
                    nout = tot;
                    for (long long w = i0; w < i1; ++w) {
                        swr[w] = (int)run;
                        run += __builtin_popcount(sbm[w]);
                    }
                }
                for (long long r = tid; r < nout; r += BS) acc[r] = 0.0;
                __syncthreads();
                // the products whose columns fall in [c_lo, c_hi)
                for (long long c0 = a0; c0 < a1; c0 += BS) {
                    const long long p = c0 + tid;
                    long long len = 0, bst = 0;
                    double a = 0.0;
                    if (p < a1) {
                        const long long k = acol[p] + bo;
                        a = to_f64(aval[p]);
                        long long lo = brp[k], hi = brp[k + 1];
                        if (ns > 1 || !whole) {
                            lo = one_chunk ? cur : lower_bound_col(bcol, lo, hi, c_lo);
                            if (sl + 1 < ns) hi = lower_bound_col(bcol, lo, hi, c_hi);
                            else if (one_chunk) hi = sr_hi;
                            else if (C1 < ncols) hi = lower_bound_col(bcol, lo, hi, C1);
                            if (one_chunk) cur = hi;
                        }
                        bst = lo;
                        len = hi - lo;
                    }
                    long long total;
                    const long long incl = block_incl_scan<BS>(len, sm, &total);
                    s_off[tid] = incl;
                    s_bst[tid] = bst - (incl - len);
                    s_a[tid] = a;
                    __syncthreads();
                    const int nact = (int)((a1 - c0) < BS ? (a1 - c0) : BS);
                    int t = -1;
                    for (long long q0 = tid; q0 < total; q0 += RU * BS) {
                        int32_t j[RU];
                        double pv[RU];
#pragma unroll
                        for (int u = 0; u < RU; ++u) {
                            const long long q = q0 + (long long)u * BS;
                            j[u] = -1;
                            pv[u] = 0.0;
                            if (q < total) {
                                if (t < 0) t = owner_search(s_off, nact, q);
                else while ((long long)s_off[t] <= q) ++t;
                                const long long bi = s_bst[t] + q;
                                j[u] = (int32_t)(bcol[bi] - c_lo);
                                pv[u] = s_a[t] * to_f64(bval[bi]);
                            }
                        }
#pragma unroll
                        for (int u = 0; u < RU; ++u) {
                            if (j[u] < 0) continue;
                            const int w = j[u] >> 5;
                            const int r = swr[w] + __builtin_popcount(sbm[w] & ((1u << (j[u] & 31)) - 1u));
                            atomicAdd(&acc[r], pv[u]);
                        }
                    }
                    __syncthreads();
                }
                // the slice in column order: wave wv walks the segment words [wv WS, wv WS + WS)
                const long long base = rp + done + s_sr[sl];
                constexpr int NW = BS / 64;
                const int wv = tid >> 6, ln = tid & 63;
                const long long WS = (nw + NW - 1) / NW;
                const long long wb = (long long)wv * WS, we = wb + WS < nw ? wb + WS : nw;
                long long wc = 0;
                for (long long w = wb + ln; w < we; w += 64) wc += __builtin_popcount(sbm[w]);
#pragma unroll
                for (int d = 32; d > 0; d >>= 1) wc += __shfl_xor(wc, d);
                long long run;
                const long long wincl = block_incl_scan<BS>(ln == 0 ? wc : 0, sm, &run);
                long long r0 = __shfl(wincl, 0) - wc;  // rank in the slice of the wave's first column
                for (long long x0 = wb; x0 < we; x0 += 64) {
                    const long long w = x0 + ln;
                    uint32_t bits = w < we ? sbm[w] : 0u;
                    const long long c = __builtin_popcount(bits);
                    const long long incl = group_incl_scan<64>(c, ln);
                    long long r = r0 + incl - c;
                    r0 += __shfl(incl, 63);
                    while (bits) {
                        const int bt = __builtin_ctz(bits);
                        bits &= bits - 1;
                        if (base + r < rend) {
                            ccol[base + r] = (int32_t)(c_lo + w * 32 + bt);
                            cval[base + r] = (VT)acc[r];
                        }
                        ++r;
                    }
                }
            }
            done += nsr;
            if (!MULTI) break;
        }
        if (tid == 0) {
            const long long cap = rend - rp;
            if (cnt_out) cnt_out[row] = !bad && done <= cap ? (int)done : -1;
            else if (bad || done != cap) atomicOr(&info->err, kErrCount);
        }
        __syncthreads();
    }
    block_slots_done(q);
}

// ===========================================================================
// Global bin in column windows (rows the symbolic pass recorded)
// ===========================================================================

// Window index of B: a wave per 64 consecutive B rows.  A row with at least
// min_len entries takes a slot (while slots last) and stores, for every
// boundary w = 0..nw, the position (from the row's start) of its first entry
// with column >= w kWin; rows without a slot get bslot = -1.  An entry with
// column j whose predecessor has column j' is the first at or past the
// boundaries w with j' < w kWin <= j; the boundaries past the last entry get
// the length.
static __global__ void __launch_bounds__(256)
k_bwin_index(long long brows, const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol, int nw,
             int min_len, long long max_slots, int32_t* __restrict__ bslot, int32_t* __restrict__ wpos,
             DevInfo* info) {
    const int lane = threadIdx.x & 63;
    const long long nwave = (long long)gridDim.x * (blockDim.x >> 6);
    // a wave takes 64 consecutive B rows: one atomic gives slots to all of
    // its long enough rows, then the wave fills each one's positions
    for (long long k0 = ((long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64; k0 < brows;
         k0 += nwave * 64) {
        const long long k = k0 + lane;
        const bool take = k < brows && brp[k + 1] - brp[k] >= min_len;
        const uint64_t tk = __ballot(take);
        int base = 0;
        if (lane == 0 && tk) base = atomicAdd(&info->win_nbs, __builtin_popcountll(tk));
        base = __shfl(base, 0);
        int slot = take ? base + __builtin_popcountll(tk & ((1ull << lane) - 1ull)) : -1;
        if (slot >= max_slots) slot = -1;               // rows past the slots keep their binary searches
        if (k < brows) bslot[k] = slot;
        uint64_t todo = __ballot(slot >= 0);
        while (todo) {                                  // wave-uniform
            const int r = __builtin_ctzll(todo);
            todo &= todo - 1;
            const long long kr = k0 + r;
            const long long s = brp[kr], e = brp[kr + 1];
            int32_t* wp = wpos + (long long)__shfl(slot, r) * (nw + 1);
            for (long long p = s + lane; p < e; p += 64) {
                const int j = bcol[p];
                const int w_lo = p > s ? (bcol[p - 1] >> kWinLog) + 1 : 0;
                for (int w = w_lo; w <= (j >> kWinLog); ++w) wp[w] = (int32_t)(p - s);
                if (p == e - 1)
                    for (int w = (j >> kWinLog) + 1; w <= nw; ++w) wp[w] = (int32_t)(e - s);
            }
        }
    }
}

// Numeric pass of a global-bin row with a window record.  The row's windows
// are grouped into slices whose LDS cost (kWinFixed per window, kWinOut per
// output, known exactly from the record) fits the budget; the greedy
// grouping takes the longest run of windows from the current one that fits,
// and any single window fits by construction.  For each slice:
//   1. every A entry's part of its B row in the slice's columns (two loads
//      from the window index, or a search in a short B row);
//   2. bitmap pass: the products' columns set bits in an LDS bitmap of the
//      slice's columns;
//   3. each 64-bit word's rank (outputs before it) by a workgroup scan; the
//      total must equal the record's count;
//   4. accumulation pass: each product adds into the FP64 accumulator at its
//      column's rank (LDS atomics);
//   5. the slice's columns are listed in rank order from the bitmap, and the
//      slice goes out with coalesced stores at its first output's place in C.
// The products are dealt to the waves in contiguous runs, so the lanes of a
// wave gather neighbouring entries of one B row.  Rows without a valid
// record are appended to fb_list (their count in info->win_fb[0]) for the
// self-counting global-bin kernel.
constexpr int kWinBS = 1024;                   // threads of the windowed kernel (one workgroup per CU)
constexpr int kWinRU = 4;                      // products per lane and pipeline stage
constexpr bool kWinPipe = false;               // gathers of the next stage issued before the current LDS work
constexpr bool kWinOr32 = true;                // bitmap pass: 32-bit atomic ORs instead of 64-bit
constexpr bool kWinSwizzle = true;             // accumulator index swizzled within 32-entry groups

// Accumulator slots of a slice of n outputs, and the slot of rank r: with
// the swizzle, ranks are permuted within groups of 32 (the group padded to
// full size), so that lanes adding at ranks a fixed stride apart spread
// over more LDS banks.
constexpr int kWinSlack = kWinSwizzle ? 31 * 8 : 0;    // LDS bytes of the last group's padding
__device__ __forceinline__ int win_acc_len(int n) { return kWinSwizzle ? (n + 31) & ~31 : n; }
__device__ __forceinline__ int win_swz(int r) { return kWinSwizzle ? r ^ ((r >> 5) & 31) : r; }

template <int BS, typename VT>
__global__ void __launch_bounds__(BS)
k_num_win(Work wk, int nw, const int64_t* __restrict__ arp, const int32_t* __restrict__ acol,
          const VT* __restrict__ aval, const int64_t* __restrict__ brp, const int32_t* __restrict__ bcol,
          const VT* __restrict__ bval, const int32_t* __restrict__ bslot, const int32_t* __restrict__ wpos,
          WinRec rec, const int64_t* __restrict__ crp, int32_t* __restrict__ ccol, VT* __restrict__ cval,
          long long budget, int32_t* __restrict__ fb_list, DevInfo* info,
          unsigned* q) {
    static_assert(BS >= kWinMaxNw, "one window count per thread");
    int nrows_bin;
    const int32_t* perm;
    work_rows(wk, &nrows_bin, &perm);
    __shared__ long long s_slot;
    constexpr int RU = kWinRU;
    // FP64 values double the pipeline's registers: the second stage is kept for FP32 only
    constexpr bool PIPE = kWinPipe && sizeof(VT) == 4;
    constexpr int NWV = BS / 64;
    extern __shared__ __align__(16) unsigned long long dyn_win[];
    __shared__ long long s_off[BS];
    __shared__ long long s_bst[BS];
    __shared__ double s_a[BS];
    __shared__ BlockScanSmem<BS> sm;
    __shared__ int s_rk[kWinMaxNw + 1];         // outputs of the row before window w
    __shared__ int s_sb[kWinMaxNw + 1];         // first window of each slice
    __shared__ int s_ns, s_rec;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nrec = min(__hip_atomic_load(rec.nrec, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), rec.cap);
    bool bad = false;
    for (long long slot = block_first(q, &s_slot); slot < nrows_bin; slot = block_next(q, slot, &s_slot)) {
        const int row = perm ? perm[slot] : (int)slot;
        const long long rp = crp[row], rlen = crp[row + 1] - rp;
        if (tid == 0) {
            int r = -1;
            if (rlen > 0) {                             // (an empty row has nothing to write)
                r = rec.islot[row];
                if (r < 0 || r >= nrec || rec.row[r] != row) {
                    r = -1;
                    fb_list[atomicAdd(&info->win_fb[0], 1)] = row;
                }
            }
            s_rec = r;
        }
        __syncthreads();
        const int r = s_rec;
        if (r >= 0) {
            const int rbm = rec.bms ? rec.rec_bm[r] : -1;     // the row's stored bitmap, if any
            const unsigned long long* sbm =
                rbm >= 0 ? reinterpret_cast<const unsigned long long*>(rec.bms) + (long long)rbm * nw * kWinWords
                         : nullptr;
            // exclusive prefix of the window counts
            const int c = tid < nw ? (int)rec.cnt[(long long)r * nw + tid] : 0;
            long long tot;
            const long long incl = block_incl_scan<BS>(c, sm, &tot);
            if (tid < nw) s_rk[tid] = (int)(incl - c);
            if (tid == 0) s_rk[nw] = (int)tot;
            if (tot != rlen) bad = true;               // uniform
            __syncthreads();
            // slices: wave 0 takes, from each start, the longest run of windows that fits
            if (wv == 0) {
                int start = 0, ns = 0;
                while (start < nw) {
                    int e = start + 1;
                    for (int b0 = start + 1; b0 <= nw; b0 += 64) {
                        const int cand = b0 + lane;
                        const bool fit = cand <= nw && (long long)kWinFixed * (cand - start) +
                                                               (long long)kWinOut * (s_rk[cand] - s_rk[start]) +
                                                               kWinSlack <= budget;
                        const int run = leading_run(__ballot(fit));
                        if (run > 0) e = b0 + run - 1;
                        if (run < 64) break;
                    }
                    if (lane == 0) s_sb[ns] = start;
                    ++ns;
                    start = e;
                }
                if (lane == 0) {
                    s_sb[ns] = nw;
                    s_ns = ns;
                }
            }
            __syncthreads();
            const int ns = s_ns;
            const long long a0 = arp[row], a1 = arp[row + 1];
            const bool one_chunk = a1 - a0 <= BS;
            // a one-chunk row keeps its thread's A entry across the slices
            int my_bsl = -1;
            long long my_s = 0, my_e = 0, my_cur = 0;
            VT my_a = 0;
            if (one_chunk && a0 + tid < a1) {
                const long long p = a0 + tid;
                const int k = acol[p];
                my_a = aval[p];
                my_s = brp[k];
                my_e = brp[k + 1];
                my_bsl = bslot[k];
                my_cur = my_s;
            }
            for (int sl = 0; sl < ns && !bad; ++sl) {
                const int w0 = s_sb[sl], w1 = s_sb[sl + 1];
                const int nout = s_rk[w1] - s_rk[w0];
                if (nout == 0) continue;                // uniform
                const long long c_lo = (long long)w0 << kWinLog, c_hi = (long long)w1 << kWinLog;
                const int nwd = (w1 - w0) * kWinWords;
                unsigned long long* bm = dyn_win;
                // word ranks within the slice (below 2^16: a slice holds at most budget / kWinOut outputs)
                uint16_t* wr = reinterpret_cast<uint16_t*>(bm + nwd);
                double* acc = reinterpret_cast<double*>(wr + nwd);            // nwd is a multiple of 64: 8-byte aligned
                int32_t* colbuf = reinterpret_cast<int32_t*>(acc + win_acc_len(nout));
                __syncthreads();                        // the previous slice is done with LDS
                if (sbm) {
                    for (int i = tid; i < nwd; i += BS) bm[i] = sbm[(long long)w0 * kWinWords + i];
                } else {
                    for (int i = tid; i < nwd; i += BS) bm[i] = 0ull;
                }
                __syncthreads();
                // the part [lo, hi) of A entry p's B row in [c_lo, c_hi)
                auto range = [&](long long s0, long long e0, int bsl, long long from, long long* lo, long long* hi) {
                    if (bsl >= 0) {
                        const int32_t* wp = wpos + (long long)bsl * (nw + 1);
                        *lo = s0 + wp[w0];
                        *hi = s0 + wp[w1];
                    } else {
                        *lo = lower_bound_col(bcol, from, e0, c_lo);
                        *hi = lower_bound_col(bcol, *lo, e0, c_hi);
                    }
                };
                // both passes walk the same products: PASS 0 sets bitmap bits,
                // PASS 1 adds a * b at the column's rank
                auto products = [&](auto pass_tag) {
                    constexpr int PASS = decltype(pass_tag)::value;
                    for (long long c0 = a0; c0 < a1; c0 += BS) {
                        if (!(one_chunk && PASS == 1)) {     // a one-chunk row's ranges stay in LDS
                            long long len = 0, bst = 0;
                            double a = 0.0;
                            const long long p = c0 + tid;
                            if (p < a1) {
                                long long lo, hi;
                                if (one_chunk) {
                                    range(my_s, my_e, my_bsl, my_cur, &lo, &hi);
                                    my_cur = hi;
                                    a = to_f64(my_a);
                                } else {
                                    const int k = acol[p];
                                    a = to_f64(aval[p]);
                                    const long long s0 = brp[k];
                                    range(s0, brp[k + 1], bslot[k], s0, &lo, &hi);
                                }
                                bst = lo;
                                len = hi - lo;
                            }
                            long long total;
                            const long long incl = block_incl_scan<BS>(len, sm, &total);
                            s_off[tid] = incl;
                            s_bst[tid] = bst - (incl - len);
                            s_a[tid] = a;
                            __syncthreads();
                        }
                        const long long total = s_off[BS - 1] > 0 ? s_off[BS - 1] : 0;
                        const int nact = (int)((a1 - c0) < BS ? (a1 - c0) : BS);
                        // contiguous runs of products per wave, whole 64-lane steps
                        const long long per = ((total + NWV - 1) / NWV + 63) & ~63LL;
                        const long long qb = (long long)wv * per;
                        const long long qe = qb + per < total ? qb + per : total;
                        // owner t of the lane's current product, with its end offset,
                        // B base and value kept in registers (LDS reads only when t moves)
                        int t = -1;
                        long long t_end = 0, t_base = 0;
                        VT t_a = 0;
                        // two-stage pipeline: the gathers of the next RU products are
                        // in flight while the current ones go into LDS
                        int32_t jc[RU], jn[RU];
                        VT vc[RU], vn[RU], ac[RU], an[RU];
                        auto gather = [&](long long q0, int32_t* jj, VT* vv, VT* aa) {
#pragma unroll
                            for (int u = 0; u < RU; ++u) {
                                const long long q = q0 + u * 64 + lane;
                                jj[u] = -1;
                                if (q < qe) {
                                    if (t < 0 || t_end <= q) {
                                        if (t < 0) t = owner_search(s_off, nact, q);
                                        else do ++t; while (s_off[t] <= q);
                                        t_end = s_off[t];
                                        t_base = s_bst[t];
                                        if constexpr (PASS == 1) t_a = (VT)s_a[t];
                                    }
                                    const long long bi = t_base + q;
                                    jj[u] = bcol[bi];
                                    if constexpr (PASS == 1) {
                                        vv[u] = bval[bi];
                                        aa[u] = t_a;
                                    }
                                }
                            }
                        };
                        auto consume = [&](const int32_t* jj, const VT* vv, const VT* aa) {
#pragma unroll
                            for (int u = 0; u < RU; ++u) {
                                if (jj[u] < 0) continue;
                                const int jl = (int)(jj[u] - c_lo);
                                const int w = jl >> 6;
                                const unsigned long long bit = 1ull << (jl & 63);
                                if constexpr (PASS == 0) {
                                    if constexpr (kWinOr32)
                                        atomicOr(reinterpret_cast<uint32_t*>(bm) + (jl >> 5), 1u << (jl & 31));
                                    else
                                        atomicOr(&bm[w], bit);
                                } else {
                                    const int rk = (int)wr[w] + __builtin_popcountll(bm[w] & (bit - 1ull));
                                    atomicAdd(&acc[win_swz(rk)], to_f64(aa[u]) * to_f64(vv[u]));
                                }
                            }
                        };
                        if constexpr (PIPE) {
                            if (qb < qe) gather(qb, jc, vc, ac);
                            for (long long q0 = qb; q0 < qe; q0 += 64 * RU) {
                                const bool more = q0 + 64 * RU < qe;      // wave-uniform
                                if (more) gather(q0 + 64 * RU, jn, vn, an);
                                consume(jc, vc, ac);
#pragma unroll
                                for (int u = 0; u < RU; ++u) {
                                    jc[u] = jn[u];
                                    vc[u] = vn[u];
                                    ac[u] = an[u];
                                }
                            }
                        } else {
                            for (long long q0 = qb; q0 < qe; q0 += 64 * RU) {
                                gather(q0, jc, vc, ac);
                                consume(jc, vc, ac);
                            }
                        }
                        __syncthreads();
                    }
                };
                if (sbm && one_chunk) {
                    // the bitmap came from the symbolic pass: the ranges the
                    // accumulation pass reuses are all that is needed
                    long long len = 0, bst = 0;
                    double a = 0.0;
                    if (a0 + tid < a1) {
                        long long lo, hi;
                        range(my_s, my_e, my_bsl, my_cur, &lo, &hi);
                        my_cur = hi;
                        a = to_f64(my_a);
                        bst = lo;
                        len = hi - lo;
                    }
                    long long total;
                    const long long incl = block_incl_scan<BS>(len, sm, &total);
                    s_off[tid] = incl;
                    s_bst[tid] = bst - (incl - len);
                    s_a[tid] = a;
                    __syncthreads();
                } else if (!sbm) {
                    products(std::integral_constant<int, 0>{});
                }
                // word ranks: thread tid takes E consecutive words
                {
                    const int E = (nwd + BS - 1) / BS;
                    const int i0 = tid * E, i1 = min(i0 + E, nwd);
                    int loc = 0;
                    for (int i = i0; i < i1; ++i) loc += __builtin_popcountll(bm[i]);
                    long long tw;
                    long long run = block_incl_scan<BS>(loc, sm, &tw) - loc;
                    for (int i = i0; i < i1; ++i) {
                        wr[i] = (uint16_t)run;
                        run += __builtin_popcountll(bm[i]);
                    }
                    if (tw != nout) bad = true;         // uniform
                }
                for (int i = tid; i < win_acc_len(nout); i += BS) acc[i] = 0.0;
                __syncthreads();
                if (bad) break;
                products(std::integral_constant<int, 1>{});
                // columns in rank order (a thread per 32-bit half of a bitmap
                // word: a dense word's bits take two lanes), then the slice out
                // with coalesced stores
                for (int i = tid; i < 2 * nwd; i += BS) {
                    const unsigned long long word = bm[i >> 1];
                    const int o = (i & 1) * 32;
                    unsigned bits = (unsigned)(word >> o);
                    int rk = (int)wr[i >> 1] + (o ? __builtin_popcount((unsigned)word) : 0);
                    while (bits) {
                        const int b = __builtin_ctz(bits);
                        bits &= bits - 1u;
                        colbuf[rk++] = (int32_t)(c_lo + (long long)i * 32 + b);
                    }
                }
                __syncthreads();
                const long long base = rp + s_rk[w0];
                for (int i = tid; i < nout; i += BS) {
                    ccol[base + i] = colbuf[i];
                    cval[base + i] = (VT)acc[win_swz(i)];
                }
            }
        }
        __syncthreads();                                // s_rec, s_rk and the LDS are reused by the next row
    }
    block_slots_done(q);
    if (bad && tid == 0) atomicOr(&info->err, kErrCount);
}

// ===========================================================================
// Off-chip access reduction of B-row sharing (Eq. 1)
// ===========================================================================

// Taking A's rows in groups of `group` consecutive rows (the last group may
// be shorter), a row of B is read once per distinct (group, column) pair
// instead of once per entry of A.  Counts those pairs: an entry is the first
// of its pair when no earlier row of its group holds its column (a binary
// search in each of them).  One thread per entry, one atomic per wave.
static __global__ void __launch_bounds__(256)
k_omar(long long nrows, long long nnz, const int64_t* __restrict__ arp, const int32_t* __restrict__ acol,
       long long group, unsigned long long* __restrict__ distinct) {
    unsigned long long firsts = 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += stride) {
        long long lo = 0, hi = nrows;               // arp[lo] <= p < arp[hi]
        while (hi - lo > 1) {
            const long long mid = (lo + hi) >> 1;
            if (arp[mid] <= p) lo = mid; else hi = mid;
        }
        const int c = acol[p];
        bool first = true;
        for (long long q = lo - lo % group; q < lo && first; ++q) {
            long long s = arp[q], e = arp[q + 1];
            const long long end = e;
            while (s < e) {
                const long long mid = (s + e) >> 1;
                if (acol[mid] < c) s = mid + 1; else e = mid;
            }
            if (s < end && acol[s] == c) first = false;
        }
        firsts += first ? 1ull : 0ull;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) firsts += __shfl_xor(firsts, d);
    if ((threadIdx.x & 63) == 0 && firsts) atomicAdd(distinct, firsts);
}

// ===========================================================================
// Input validation (canonical CSR)
// ===========================================================================
static __global__ void __launch_bounds__(256)
k_validate(long long nrows, long long ncols, long long nnz, const int64_t* __restrict__ rp,
           const int32_t* __restrict__ col, DevInfo* info) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    // row_ptr values index col directly: a view of rows inside a larger
    // array starts above 0 and may end below nnz
    const long long a = rp[r], b = rp[r + 1];
    if (a < 0 || b < a || b > nnz) { atomicOr(&info->err, kErrRange); return; }
    int prev = -1;
    for (long long p = a; p < b; ++p) {
        const int c = col[p];
        if (c < 0 || c >= ncols) { atomicOr(&info->err, kErrRange); return; }
        if (c <= prev) { atomicOr(&info->err, kErrUnsorted); return; }
        prev = c;
    }
}

}  // namespace msp
