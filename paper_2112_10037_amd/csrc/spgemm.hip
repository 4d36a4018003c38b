// The plain two-phase product: bin plans, per-bin kernel dispatch and the
// msp_spgemm / msp_spgemm_symbolic / msp_row_features entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "msp.h"

using namespace msp;

namespace msp {

static int next_pow2(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// ---------------------------------------------------------------------------
// bin plans
// ---------------------------------------------------------------------------
// Bounds up to block_rows go to the merge kernel (<= 32), wave-local row
// batches and lane groups (16, 32, 64, 128 with 8, 16, 32, 64 lanes, scaled
// by group_scale), and whole waves per row with LDS tables of up to 2048
// keys (symbolic) or 512 (key, value) slots (numeric); workgroup kernels
// cover the middle; the last bin is the global path.  Hash tables get
// nextpow2(bound) << hash_scale slots, so they are at most half full.

static void add_bin(BinPlan& p, int umax, BinSpec s) {
    const int b = p.table.nb;          // bins are appended after bin 0
    p.table.umax[b] = umax;
    p.spec[b] = s;
    p.table.nb = b + 1;
}

// Small bins (bound <= 128).  Symbolic: wave-local row batches (k_sym_wave) of
// at most R rows with T key slots.  Numeric: wave batches while T <= 64, lane groups of
// G lanes per row (k_num_group) for larger tables.
static int sym_batch_rows(int T) { return T <= 64 ? 16 : 1024 / T; }

static void add_small_bins(BinPlan& p, const msp_tuning& t, int limit, bool numeric) {
    static const int umax[7] = {16, 32, 64, 128, 256, 512, 1024};
    static const int g0[7] = {8, 16, 32, 64, 64, 64, 64};
    int covered = 0;
    // the merge takes row_nnz steps of K comparisons each: worth it for the
    // shortest rows only
    if (t.merge_k > 0 && limit >= 32) {
        add_bin(p, 32, BinSpec{Kind::Merge, t.merge_k, kMergeFT, numeric && t.share_g > 0 ? t.share_g : 0});
        covered = 32;
    }
    for (int i = 0; i < 7; ++i) {
        if (umax[i] > limit) break;
        if (umax[i] <= covered) continue;
        const int T = next_pow2(umax[i]) << t.hash_scale;
        if (!numeric) {
            if (T <= 256) add_bin(p, umax[i], BinSpec{Kind::Batch, sym_batch_rows(T), T});
            else if (T <= 2048) add_bin(p, umax[i], BinSpec{Kind::Group, 64, T});
            else break;
        } else if (T <= 64) {
            const int R = (T == 32 ? (t.group_scale == 0 ? 12 : 8 >> (t.group_scale - 1)) : 8 >> t.group_scale);
            add_bin(p, umax[i], BinSpec{Kind::Batch, R, T});
        } else if (T <= 512) {
            int G = std::min(64, g0[i] << t.group_scale);
            G = std::min(G, T / 2);
            add_bin(p, umax[i], BinSpec{Kind::Group, G, T});
        } else {
            break;
        }
    }
}

BinPlan symbolic_plan(const msp_tuning& t, bool force_spill) {
    BinPlan p;
    memset(&p.table, 0, sizeof(p.table));
    p.table.nb = 1;                    // bin 0: u == 0
    if (!force_spill) {
        add_small_bins(p, t, t.block_rows, false);
        static const int umax[4] = {512, 2048, 8192, 16384};
        static const int bs[4] = {256, 512, 1024, 1024};
        int last = p.table.umax[p.table.nb - 1];
        for (int i = 0; i < 4; ++i) {
            int T = std::min(32768, next_pow2(umax[i]) << t.hash_scale);
            int u = std::min(umax[i], T / 2);
            if (u <= last) continue;
            add_bin(p, u, BinSpec{Kind::Block, bs[i], T});
            last = u;
        }
    }
    p.spec[p.table.nb] = BinSpec{Kind::Bitmap, 1024, 0};
    return p;
}

BinPlan numeric_plan(const msp_tuning& t, bool force_spill) {
    BinPlan p;
    memset(&p.table, 0, sizeof(p.table));
    p.table.nb = 1;
    if (!force_spill) {
        add_small_bins(p, t, std::min(t.block_rows, t.spill_nnz), true);
        int last = p.table.umax[p.table.nb - 1];
        int list[4] = {512, 2048, 4096, t.spill_nnz};
        std::sort(list, list + 4);
        for (int i = 0; i < 4; ++i) {
            const int u0 = list[i];
            if (u0 > t.spill_nnz || u0 <= last) continue;
            const int bs = u0 <= 512 ? 256 : (u0 <= 2048 ? 512 : 1024);
            const int T = std::min(8192, next_pow2(u0) << t.hash_scale);
            const int u = std::min(u0, T / 2);
            if (u <= last) continue;
            add_bin(p, u, BinSpec{Kind::Block, bs, T});
            last = u;
        }
    }
    p.spec[p.table.nb] = BinSpec{Kind::Dense, 1024, 0};
    return p;
}

// ---------------------------------------------------------------------------
// kernel tables
// ---------------------------------------------------------------------------
constexpr int kLdsReserve = 26 * 1024;     // static LDS of the symbolic bitmap kernel
constexpr int kSliceReserve = 27 * 1024;   // static LDS of k_num_slice<kSliceBS>
constexpr int kWinReserve = 30 * 1024;     // static LDS of k_num_win<kWinBS>
constexpr int kWinPerCU = 1;               // workgroups of k_num_win per compute unit

// Dynamic LDS of the windowed global-bin kernel (a share of the compute
// unit's LDS for each of its workgroups), or 0 when a window of full
// density would not fit.
static int win_lds(const msp_handle* h) {
    // (a slice then holds fewer than 2^16 outputs: its word ranks are 16-bit)
    const int dyn = std::min(h->lds_per_block / kWinPerCU - kWinReserve, 65535 * kWinOut);
    return dyn >= kWinFixed + kWinOut * kWin + kWinSlack ? dyn : 0;
}

#define MSP_GROUP_SHAPES(X) \
    X(8, 32) X(16, 32) X(8, 64) X(16, 64) X(32, 64) X(16, 128) X(32, 128) X(64, 128) \
    X(32, 256) X(64, 256) X(64, 512)
#define MSP_SYM_GROUP_SHAPES(X) MSP_GROUP_SHAPES(X) X(64, 1024) X(64, 2048)
#define MSP_SYM_BATCH_SHAPES(X) X(32, 16) X(64, 16) X(128, 8) X(256, 4) X(512, 2)
#define MSP_NUM_BATCH_SHAPES(X) X(32, 12) X(32, 8) X(32, 4) X(64, 8) X(64, 4) X(64, 2)
#define MSP_SYM_BLOCK_SHAPES(X) \
    X(256, 1024) X(256, 2048) X(512, 4096) X(512, 8192) X(1024, 16384) X(1024, 32768)
#define MSP_NUM_BLOCK_SHAPES(X) \
    X(256, 512) X(256, 1024) X(256, 2048) X(512, 2048) X(512, 4096) X(512, 8192) X(1024, 8192)

static bool spec_supported(const BinSpec& sp, bool numeric) {
    switch (sp.kind) {
        case Kind::Merge: return sp.lanes == 4 || sp.lanes == 8;
        case Kind::Batch:
#define X(T, R) if (sp.slots == T && sp.lanes == R) return true;
            if (numeric) { MSP_NUM_BATCH_SHAPES(X) } else { MSP_SYM_BATCH_SHAPES(X) }
#undef X
            return false;
        case Kind::Group:
#define X(G, T) if (sp.lanes == G && sp.slots == T) return true;
            if (numeric) { MSP_GROUP_SHAPES(X) } else { MSP_SYM_GROUP_SHAPES(X) }
#undef X
            return false;
        case Kind::Block:
#define X(BS, T) if (sp.lanes == BS && sp.slots == T) return true;
            if (numeric) { MSP_NUM_BLOCK_SHAPES(X) } else { MSP_SYM_BLOCK_SHAPES(X) }
#undef X
            return false;
        case Kind::Bitmap: return !numeric;
        case Kind::Dense: return numeric;
        default: return false;
    }
}

// Number of (tuning, bin) pairs whose plan names a kernel shape that is not
// instantiated; 0 means every accepted tuning can run.  Host-only check.
int count_unsupported_plans(int verbose) {
    int bad = 0;
    for (int hs = 1; hs <= 2; ++hs)
        for (int gs = 0; gs <= 2; ++gs)
            for (int sp : {64, 128, 256, 512, 1024, 2048, 4096})
                for (int br : {32, 64, 128, 256, 512, 1024})
                    for (int fs = 0; fs <= 1; ++fs) {
                      for (int mk : {4, 8, -1}) {
                        msp_tuning t{hs, gs, sp, br, mk};
                        if (check_tuning(&t) != MSP_OK) continue;
                        const BinPlan a = symbolic_plan(t, fs), b = numeric_plan(t, fs);
                        for (int i = 1; i <= a.table.nb; ++i)
                            if (!spec_supported(a.spec[i], false)) {
                                ++bad;
                                if (verbose) fprintf(stderr, "symbolic t=(%d,%d,%d,%d) bin %d kind %d shape (%d,%d)\n", hs, gs, sp, br, i, (int)a.spec[i].kind, a.spec[i].lanes, a.spec[i].slots);
                            }
                        for (int i = 1; i <= b.table.nb; ++i)
                            if (!spec_supported(b.spec[i], true)) {
                                ++bad;
                                if (verbose) fprintf(stderr, "numeric t=(%d,%d,%d,%d) bin %d kind %d shape (%d,%d)\n", hs, gs, sp, br, i, (int)b.spec[i].kind, b.spec[i].lanes, b.spec[i].slots);
                            }
                        for (int i = 2; i < a.table.nb; ++i) bad += a.table.umax[i] <= a.table.umax[i - 1];
                        for (int i = 2; i < b.table.nb; ++i) bad += b.table.umax[i] <= b.table.umax[i - 1];
                      }
                    }
    return bad;
}

msp_status configure_kernels(msp_handle* h) {
    // allow the bitmap kernels the device's full LDS for their dynamic part
    const int dyn = std::max(0, h->lds_per_block - kLdsReserve);
    void* fns[] = {(void*)k_sym_bitmap<1024, true, false>, (void*)k_sym_bitmap<1024, true, true>};
    for (void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return hip_fail(e, "hipFuncSetAttribute(MaxDynamicSharedMemorySize)");
        }
    }
    const int dyn_slice = std::max(0, h->lds_per_block - kSliceReserve);
    void* slice_fns[] = {(void*)k_num_slice<kSliceBS, float, false, false>,
                         (void*)k_num_slice<kSliceBS, double, false, false>,
                         (void*)k_num_slice<kSliceBS, float, true, false>,
                         (void*)k_num_slice<kSliceBS, double, true, false>,
                         (void*)k_num_slice<kSliceBS, float, false, true>,
                         (void*)k_num_slice<kSliceBS, double, false, true>,
                         (void*)k_num_slice<kSliceBS, float, true, true>,
                         (void*)k_num_slice<kSliceBS, double, true, true>};
    for (void* f : slice_fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_slice);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return hip_fail(e, "hipFuncSetAttribute(MaxDynamicSharedMemorySize)");
        }
    }
    const int dyn_win = win_lds(h);
    if (dyn_win > 0) {
        void* win_fns[] = {(void*)k_num_win<kWinBS, float>, (void*)k_num_win<kWinBS, double>};
        for (void* f : win_fns) {
            hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_win);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return hip_fail(e, "hipFuncSetAttribute(MaxDynamicSharedMemorySize)");
            }
        }
    }
    return MSP_OK;
}

// Grid of a persistent lane-group kernel: as many workgroups as can be
// resident (occupancy from the kernel's registers and LDS), a multiple of 8
// for the XCD-aware order, and no more than the rows need.
static int group_grid(msp_handle* h, const void* fn, int rows, int rows_per_block) {
    // shared by every handle, and handles may be used from several threads
    static std::mutex occ_mutex;
    static std::unordered_map<const void*, int> occ_cache;
    int occ = 0;
    {
        std::lock_guard<std::mutex> lock(occ_mutex);
        auto it = occ_cache.find(fn);
        if (it != occ_cache.end()) occ = it->second;
    }
    if (occ == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, 256, 0) != hipSuccess || occ < 1) {
            (void)hipGetLastError();
            occ = 1;
        }
        std::lock_guard<std::mutex> lock(occ_mutex);
        occ_cache[fn] = occ;
    }
    const int need = (rows + rows_per_block - 1) / rows_per_block;
    const int full = occ * h->num_cu;
    const int blocks = std::max(1, std::min(need, full));
    return (blocks + 7) & ~7;
}

static msp_status launch_check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return MSP_OK;
}

// symbolic kernel of one bin over the rows of `wk`; `rows` (the row count,
// or an estimate when wk reads it from the device) sizes persistent grids
template <bool BATCH>
static msp_status launch_symbolic_t(msp_handle* h, const BinSpec& s, Work wk, int rows, const Operands& op,
                                    int32_t* rnnz, const RowMap& mp, const int32_t* ufilter = nullptr,
                                    int umax = 0) {
    if (rows <= 0) return MSP_OK;
    DevInfo* info = h->info.as<DevInfo>();
    hipStream_t st = h->stream;
    unsigned* const rq = BATCH ? nullptr : wk.rowq;   // (the batched graph's kernels keep static slots)
    // window records for the numeric global bin (plain products only)
    const WinRec rec = BATCH ? WinRec{} : h->cur_rec;
    if (s.kind == Kind::Merge) {
        const void* fn = s.lanes == 4 ? (const void*)k_sym_merge<4, BATCH> : (const void*)k_sym_merge<8, BATCH>;
        const int grid = group_grid(h, fn, rows, 256);
        if (s.lanes == 4)
            k_sym_merge<4, BATCH><<<grid, 256, 0, st>>>(wk, op.arp, op.acol, op.brp, op.bcol, ufilter, umax, rnnz,
                                                        info, mp);
        else
            k_sym_merge<8, BATCH><<<grid, 256, 0, st>>>(wk, op.arp, op.acol, op.brp, op.bcol, ufilter, umax, rnnz,
                                                        info, mp);
        return launch_check("k_sym_merge");
    } else if (s.kind == Kind::Batch) {
#define X(T, R)                                                                                        \
    if (s.slots == T && s.lanes == R) {                                                                \
        const int grid = group_grid(h, (const void*)k_sym_wave<T, R, BATCH>, rows, 4 * R);            \
        k_sym_wave<T, R, BATCH><<<grid, 256, 0, st>>>(wk, op.arp, op.acol, op.brp, op.bcol, rnnz, info, mp); \
        return launch_check("k_sym_wave");                                                            \
    }
        MSP_SYM_BATCH_SHAPES(X)
#undef X
    } else if (s.kind == Kind::Group) {
#define X(G, T)                                                                                       \
    if (s.lanes == G && s.slots == T) {                                                               \
        const int grid = group_grid(h, (const void*)k_sym_group<G, T, BATCH>, rows, 256 / G);        \
        k_sym_group<G, T, BATCH><<<grid, 256, 0, st>>>(wk, (int)op.m, op.arp, op.acol, op.brp, op.bcol, rnnz, \
                                                       info, mp);                                     \
        return launch_check("k_sym_group");                                                           \
    }
        MSP_SYM_GROUP_SHAPES(X)
#undef X
    } else if (s.kind == Kind::Block) {
        const int grid = std::min(rows, 4 * h->num_cu);
#define X(BS, T)                                                                                       \
    if (s.lanes == BS && s.slots == T) {                                                               \
        k_sym_block<BS, T, BATCH><<<grid, BS, 0, st>>>(wk, op.arp, op.acol, op.brp, op.bcol, rnnz, info, mp, rec, \
                                                       rq);                                              \
        return launch_check("k_sym_block");                                                            \
    }
        MSP_SYM_BLOCK_SHAPES(X)
#undef X
    } else if (s.kind == Kind::Bitmap) {
        const long long n = op.ncols;
        const long long words = (n + 31) / 32;
        const bool lds = words * 4 <= h->lds_per_block - kLdsReserve;
        const int grid = std::min(rows, (lds ? 1 : 2) * h->num_cu);
        uint32_t* slab = nullptr;
        if (!lds) {
            msp_status r = h->sbm.ensure((size_t)grid * words * 4);
            if (r != MSP_OK) return r;
            slab = h->sbm.as<uint32_t>();
        }
        if (lds)
            k_sym_bitmap<1024, true, BATCH><<<grid, 1024, words * 4, st>>>(wk, n, op.arp, op.acol, op.brp, op.bcol,
                                                                           rnnz, slab, info, mp, rec,
                                                                           rq);
        else
            k_sym_bitmap<1024, false, BATCH><<<grid, 1024, 0, st>>>(wk, n, op.arp, op.acol, op.brp, op.bcol, rnnz,
                                                                    slab, info, mp, rec, rq);
        return launch_check("k_sym_bitmap");
    }
    return fail(MSP_ERR_UNSUPPORTED, "no symbolic kernel for bin shape (%d, %d)", s.lanes, s.slots);
}

// The windowed global-bin kernel over the rows of wk, after B's window
// index; rows without a record are left in h->win_fb for the self-counting
// kernel (their count in the device info block).
template <typename VT>
static msp_status launch_window_bin(msp_handle* h, Work wk, int rows, const Operands& op, const int64_t* crp,
                                    int32_t* ccol, VT* cval) {
    DevInfo* info = h->info.as<DevInfo>();
    hipStream_t st = h->stream;
    const WinRec& rec = h->cur_rec;
    const int nw = rec.nw;
    // B rows of at least min_len entries get a slot, up to 1/64 of the
    // device's memory (the allocation-free product, whose scratch is small,
    // indexes only rows of 64 entries or more); rows without one find their
    // windows by binary search
    const int min_len = h->win_wpos.arena ? 64 : kWinMinLen;
    const long long cap = std::max(1LL, (long long)(h->total_mem / 64) / ((long long)(nw + 1) * 4));
    const long long max_slots = std::max(1LL, std::min({op.brows, op.bnnz / min_len, cap}));
    msp_status r;
    if ((r = h->win_bslot.ensure((size_t)std::max(op.brows, 1LL) * 4)) != MSP_OK) return r;
    if ((r = h->win_wpos.ensure((size_t)max_slots * (size_t)(nw + 1) * 4)) != MSP_OK) return r;
    if ((r = h->win_fb.ensure((size_t)std::max(rows, 1) * 4)) != MSP_OK) return r;
    if (op.brows > 0) {
        const long long blocks = std::min<long long>((op.brows + 255) / 256, 16LL * h->num_cu);
        k_bwin_index<<<(int)blocks, 256, 0, st>>>(op.brows, op.brp, op.bcol, nw, min_len, max_slots,
                                                  h->win_bslot.as<int32_t>(), h->win_wpos.as<int32_t>(), info);
        if ((r = launch_check("k_bwin_index")) != MSP_OK) return r;
    }
    const int lds = win_lds(h);
    const int grid = std::max(1, std::min(rows, kWinPerCU * h->num_cu));
    hipEvent_t ev = h->prof.sub_begin(MSP_PHASE_GLOBAL_BIN, st);
    k_num_win<kWinBS, VT><<<grid, kWinBS, (size_t)lds, st>>>(
        wk, nw, op.arp, op.acol, (const VT*)op.aval, op.brp, op.bcol, (const VT*)op.bval,
        h->win_bslot.as<int32_t>(), h->win_wpos.as<int32_t>(), rec, crp, ccol, cval, (long long)lds,
        h->win_fb.as<int32_t>(), info, wk.rowq);
    r = launch_check("k_num_win");
    h->prof.sub_end(MSP_PHASE_GLOBAL_BIN, ev, st);
    return r;
}

template <typename VT, bool BATCH>
static msp_status launch_numeric_t(msp_handle* h, const BinSpec& s, Work wk, int rows, const Operands& op,
                                   const int64_t* crp, int32_t* ccol, VT* cval, int32_t* cnt_out,
                                   const RowMap& mp) {
    DevInfo* info = h->info.as<DevInfo>();
    hipStream_t st = h->stream;
    const VT* av = (const VT*)op.aval;
    const VT* bv = (const VT*)op.bval;
    unsigned* rq = BATCH ? nullptr : wk.rowq;         // (the batched graph's kernels keep static slots)
    if (s.kind == Kind::Merge) {
        const bool small = op.bnnz < INT32_MAX;     // 32-bit positions into B
#define MSP_MERGE(KK, IT, SH)                                                                            \
    {                                                                                                    \
        const int grid = group_grid(h, (const void*)k_num_merge<KK, VT, IT, BATCH, SH>, rows, 256);     \
        k_num_merge<KK, VT, IT, BATCH, SH><<<grid, 256, 0, st>>>(wk, op.arp, op.acol, av, op.brp, op.bcol, bv, \
                                                                 crp, ccol, cval, cnt_out, info, mp,    \
                                                                 s.share);                              \
        return launch_check("k_num_merge");                                                              \
    }
        // B-row sharing stages rows of B with 32-bit positions only
        if (s.share > 0 && small) {
            if (s.lanes == 4) MSP_MERGE(4, int, true)
            else if (s.lanes == 6) MSP_MERGE(6, int, true)
            else MSP_MERGE(8, int, true)
        }
        if (s.lanes == 4) { if (small) MSP_MERGE(4, int, false) else MSP_MERGE(4, long long, false) }
        else if (s.lanes == 6) { if (small) MSP_MERGE(6, int, false) else MSP_MERGE(6, long long, false) }
        else { if (small) MSP_MERGE(8, int, false) else MSP_MERGE(8, long long, false) }
#undef MSP_MERGE
    } else if (s.kind == Kind::Batch) {
#define X(T, R)                                                                                          \
    if (s.slots == T && s.lanes == R) {                                                                  \
        const int grid = group_grid(h, (const void*)k_num_wave<T, R, VT, BATCH>, rows, 4 * R);          \
        k_num_wave<T, R, VT, BATCH><<<grid, 256, 0, st>>>(wk, op.arp, op.acol, av, op.brp, op.bcol, bv, crp, ccol, \
                                                          cval, cnt_out, info, mp);                      \
        return launch_check("k_num_wave");                                                              \
    }
        MSP_NUM_BATCH_SHAPES(X)
#undef X
    } else if (s.kind == Kind::Group) {
#define X(G, T)                                                                                            \
    if (s.lanes == G && s.slots == T) {                                                                    \
        const int grid = group_grid(h, (const void*)k_num_group<G, T, VT, BATCH>, rows, 256 / G);         \
        k_num_group<G, T, VT, BATCH><<<grid, 256, 0, st>>>(wk, op.arp, op.acol, av, op.brp, op.bcol, bv, crp, \
                                                           ccol, cval, cnt_out, info, mp);                \
        return launch_check("k_num_group");                                                                \
    }
        MSP_GROUP_SHAPES(X)
#undef X
    } else if (s.kind == Kind::Block) {
        const int grid = std::min(rows, 4 * h->num_cu);
#define X(BS, T)                                                                                             \
    if (s.lanes == BS && s.slots == T) {                                                                     \
        k_num_block<BS, T, VT, BATCH><<<grid, BS, 0, st>>>(wk, op.arp, op.acol, av, op.brp, op.bcol, bv, crp,   \
                                                           ccol, cval, cnt_out, info, mp, rq);              \
        return launch_check("k_num_block");                                                                  \
    }
        MSP_NUM_BLOCK_SHAPES(X)
#undef X
    } else if (s.kind == Kind::Dense) {
        const long long n = op.ncols;
        if constexpr (!BATCH) {
            if (!cnt_out && h->cur_rec.cnt) {
                msp_status r = launch_window_bin<VT>(h, wk, rows, op, crp, ccol, cval);
                if (r != MSP_OK) return r;
                // the rows without a record: their list and count are in device memory
                wk = Work{h->win_fb.as<int32_t>(), 0, &info->win_fb[0]};
                wk.rowq = &info->queue[1][kNB][0];
                rows = h->num_cu;
                rq = wk.rowq;
            }
        }
        {
            // accumulate in LDS slice by slice, over column super-ranges whose
            // bitmap fits the LDS (one when all columns fit)
            const long long avail = h->lds_per_block - kSliceReserve;
            const long long span_max = avail / 32 * 256;              // whole 256-column blocks
            const long long span = n <= span_max ? std::max(n, 1LL) : span_max;
            const long long sw = (span + 31) / 32;
            const long long nr8 = (sw + 7) / 8;
            const long long lds = std::min(avail, sw * 4 + 65536);
            const long long budget = lds - kSliceBlockCost - 16;
            if (span_max > 0 && budget > kSliceBlockCost &&
                (kSliceBlockFixed * nr8 + 8 * span) / budget + 1 <= kSliceMax) {
                const int grid = std::max(1, std::min(rows, h->num_cu));
                msp_status r = h->gsl.ensure((size_t)grid * (size_t)sw * 4);
                if (r != MSP_OK) return r;
                if (n <= span_max)
                    k_num_slice<kSliceBS, VT, BATCH, false><<<grid, kSliceBS, (size_t)lds, st>>>(
                        wk, n, span, op.arp, op.acol, av, op.brp, op.bcol, bv, crp, ccol, cval,
                        h->gsl.as<uint32_t>(), lds, cnt_out, info, mp, rq);
                else
                    k_num_slice<kSliceBS, VT, BATCH, true><<<grid, kSliceBS, (size_t)lds, st>>>(
                        wk, n, span, op.arp, op.acol, av, op.brp, op.bcol, bv, crp, ccol, cval,
                        h->gsl.as<uint32_t>(), lds, cnt_out, info, mp, rq);
                return launch_check("k_num_slice");
            }
        }
        return fail(MSP_ERR_UNSUPPORTED, "internal: the global bin's slices do not fit the LDS");
    }
    return fail(MSP_ERR_UNSUPPORTED, "no numeric kernel for bin shape (%d, %d)", s.lanes, s.slots);
}

template <bool BATCH>
msp_status launch_symbolic_bin(msp_handle* h, const BinSpec& s, Work wk, int rows, const Operands& op,
                               int32_t* rnnz, const RowMap& mp, const int32_t* ufilter, int umax) {
    return launch_symbolic_t<BATCH>(h, s, wk, rows, op, rnnz, mp, ufilter, umax);
}

template <bool BATCH>
msp_status launch_numeric_bin(msp_handle* h, const BinSpec& s, Work wk, int rows, const Operands& op,
                              const int64_t* crp, int32_t* ccol, void* cval, int32_t* cnt_out, const RowMap& mp) {
    if (rows <= 0) return MSP_OK;
    if (op.dtype == MSP_F64)
        return launch_numeric_t<double, BATCH>(h, s, wk, rows, op, crp, ccol, (double*)cval, cnt_out, mp);
    return launch_numeric_t<float, BATCH>(h, s, wk, rows, op, crp, ccol, (float*)cval, cnt_out, mp);
}

template msp_status launch_symbolic_bin<true>(msp_handle*, const BinSpec&, Work, int, const Operands&, int32_t*,
                                              const RowMap&, const int32_t*, int);
template msp_status launch_numeric_bin<true>(msp_handle*, const BinSpec&, Work, int, const Operands&,
                                             const int64_t*, int32_t*, void*, int32_t*, const RowMap&);

Operands operands_of(const msp_csr* A, const msp_csr* B) {
    Operands op;
    op.arp = A->row_ptr;
    op.acol = A->col;
    op.aval = A->val;
    op.brp = B->row_ptr;
    op.bcol = B->col;
    op.bval = B->val;
    op.ncols = B->ncols;
    op.bnnz = B->nnz;
    op.m = A->nrows;
    op.dtype = A->dtype;
    op.annz = A->nnz;
    op.brows = B->nrows;
    return op;
}

// plain product: rows listed in perm (or all rows)
static msp_status launch_symbolic(msp_handle* h, const BinSpec& s, int rows, const int32_t* perm,
                                  const msp_csr* A, const msp_csr* B, int32_t* rnnz, unsigned* rowq) {
    Work wk{perm, rows, nullptr};
    wk.rowq = rowq;
    return launch_symbolic_t<false>(h, s, wk, rows, operands_of(A, B), rnnz, RowMap{});
}

static msp_status launch_numeric(msp_handle* h, const BinSpec& s, int rows, const int32_t* perm,
                                 const msp_csr* A, const msp_csr* B, const int64_t* crp,
                                 int32_t* ccol, void* cval, int32_t* cnt_out, unsigned* rowq) {
    Work wk{perm, rows, nullptr};
    wk.rowq = rowq;
    return launch_numeric_bin<false>(h, s, wk, rows, operands_of(A, B), crp, ccol, cval, cnt_out, RowMap{});
}

// ---------------------------------------------------------------------------
// pipeline pieces
// ---------------------------------------------------------------------------
msp_status zero_info(msp_handle* h) {
    const int words = (int)(sizeof(DevInfo) / 4);
    k_zero_info<<<1, 256, 0, h->stream>>>((int*)h->info.ptr, words, h->dpending);
    return launch_check("k_zero_info");
}

// The summary is a posted write to host memory: the stream can report its
// work complete a little before that write is visible.  After completion
// the wait keeps polling for a while, then takes the same figures from a
// copy of the device info block.
msp_status wait_summary(msp_handle* h, int seq, bool with_nnz, const int (*part)[kPartStride], int spec_nb) {
    auto seen = [&] { return __atomic_load_n(&h->hsum->seq, __ATOMIC_ACQUIRE) == seq; };
    bool ok = false;
    for (unsigned long long it = 1; !ok; ++it) {
        if (seen()) { ok = true; break; }
        if ((it & 1023) == 0) {
            const hipError_t q = hipStreamQuery(h->stream);
            if (q == hipSuccess) {
                for (int k = 0; k < 200000 && !ok; ++k) {
                    ok = seen();
                    __builtin_ia32_pause();
                }
                break;
            }
            if (q != hipErrorNotReady) return hip_fail(q, "hipStreamQuery");
        }
        __builtin_ia32_pause();
    }
    if (!ok) {
        ++h->summary_fallbacks;
        msp_status s = read_info(h);
        if (s != MSP_OK) return s;
        const DevInfo* d = h->hinfo;
        const int(*pp)[kPartStride] = (const int(*)[kPartStride])((const char*)d + ((const char*)part - (const char*)h->info.ptr));
        h->hsum->nnz = with_nnz ? d->nnz : 0;
        h->hsum->err = d->err;
        h->hsum->neg_count = d->neg_count;
        sum_parts(pp, h->hsum->counts);
        h->hsum->merge_na = 0;
        for (int p = 0; p < kParts; ++p) h->hsum->merge_na = std::max(h->hsum->merge_na, d->sym_part[p][kPartMergeNA]);
        if (spec_nb > 0) {
            // the speculative scan left when the fused pass left rows for a
            // symbolic bin other than the empty and merge bins
            int sym[kNB];
            sum_parts(d->sym_part, sym);
            const bool other = d->fused_other != 0;
            if (other) {
                h->hsum->nnz = -1;
                for (int b = 0; b < kNB; ++b) h->hsum->counts[b] = b <= spec_nb ? sym[b] : 0;
            }
        }
    }
    if (h->prof.on) h->prof.collect();
    return take_pending_error(h);
}

msp_status take_pending_error(msp_handle* h) {
    const int pend = *h->hpending;
    if (!pend) return MSP_OK;
    *h->hpending = 0;
    if (pend & kErrProbe) return fail(MSP_ERR_HIP, "internal: hash probe bound exceeded (earlier call)");
    return fail(MSP_ERR_HIP, "internal: numeric row count differs from symbolic count (earlier call)");
}

msp_status read_info(msp_handle* h) {
    hipError_t e = hipMemcpyAsync(h->hinfo, h->info.ptr, sizeof(DevInfo), hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(info)");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (h->prof.on) h->prof.collect();
    return take_pending_error(h);
}

msp_status run_row_stats(msp_handle* h, const msp_csr* A, const msp_csr* B, const BinPlan& plan,
                         int64_t* prod_out, float* feat, int32_t* lo_out, int publish_seq) {

    const int m = (int)A->nrows;
    msp_status s = h->u.ensure((size_t)std::max(m, 1) * 4);
    if (s != MSP_OK) return s;
    if (m == 0) return MSP_OK;
    const int grid = (m + 255) / 256;
    // lists of the rows with more than kLongRow A entries (every such row
    // fits: at most nnz / (kLongRow + 1) rows, nnz / kLongChunk + rows chunks)
    LongRows lr;
    if (A->nnz > kLongRow) {
        const long long nl = A->nnz / (kLongRow + 1) + 1;
        const long long nc = A->nnz / kLongChunk + nl + 1;
        if (nl > INT32_MAX || nc > INT32_MAX) return fail(MSP_ERR_INDEX_OVERFLOW, "too many long rows");
        if ((s = h->lr_list.ensure((size_t)nl * 4)) != MSP_OK || (s = h->lr_base.ensure((size_t)nl * 4)) != MSP_OK ||
            (s = h->lr_chunk.ensure((size_t)nc * 4)) != MSP_OK ||
            (s = h->lr_acc.ensure((size_t)nl * sizeof(LongAcc))) != MSP_OK)
            return s;
        lr = LongRows{h->lr_list.as<int>(), h->lr_base.as<int>(), h->lr_chunk.as<int>(), h->lr_acc.as<LongAcc>(),
                      (int)nl, (int)nc};
    }
    DevInfo* info = h->info.as<DevInfo>();
    if (feat)
        k_row_stats<true><<<grid, 256, 0, h->stream>>>(m, B->ncols, A->row_ptr, A->col, B->row_ptr, B->col,
                                                      h->u.as<int32_t>(), prod_out, h->rnnz.as<int32_t>(),
                                                      plan.table, info, feat, lo_out, RowMap{}, lr);
    else
        k_row_stats<false><<<grid, 256, 0, h->stream>>>(m, B->ncols, A->row_ptr, A->col, B->row_ptr, B->col,
                                                       h->u.as<int32_t>(), prod_out, h->rnnz.as<int32_t>(),
                                                       plan.table, info, nullptr, nullptr, RowMap{}, lr);
    msp_status s2 = launch_check("k_row_stats");
    if (s2 == MSP_OK && lr.list) {
        // (both kernels read their counts on the device; with no long row they end at once)
        const int gl = 4 * h->num_cu;
        if (feat) {
            k_row_stats_long<true><<<gl, 256, 0, h->stream>>>(info, A->row_ptr, A->col, B->row_ptr, B->col, lr);
            k_row_stats_long_fin<true><<<4, 256, 0, h->stream>>>(info, B->ncols, A->row_ptr, lr, h->u.as<int32_t>(),
                                                                 prod_out, h->rnnz.as<int32_t>(), plan.table, feat,
                                                                 lo_out);
        } else {
            k_row_stats_long<false><<<gl, 256, 0, h->stream>>>(info, A->row_ptr, A->col, B->row_ptr, B->col, lr);
            k_row_stats_long_fin<false><<<4, 256, 0, h->stream>>>(info, B->ncols, A->row_ptr, lr, h->u.as<int32_t>(),
                                                                  prod_out, h->rnnz.as<int32_t>(), plan.table, nullptr,
                                                                  nullptr);
        }
        s2 = launch_check("k_row_stats_long");
    }
    if (s2 != MSP_OK || !publish_seq) return s2;
    k_publish<<<1, 64, 0, h->stream>>>(h->info.as<DevInfo>(), 0, plan.table.nb, h->dsum, publish_seq);
    return launch_check("k_publish");
}

void sum_parts(const int (*part)[kPartStride], int out[kNB]) {
    for (int b = 0; b < kNB; ++b) {
        int t = 0;
        for (int p = 0; p < kParts; ++p) t += part[p][b];
        out[b] = t;
    }
}

// Launch the kernels of every nonempty bin.  With one nonempty bin, or when
// every nonempty bin is a hash bin of the small kernels (whose larger tables
// subsume the smaller ones), one kernel takes all rows in their natural
// order (no scatter; these kernels handle smaller and empty rows too).
// Otherwise row ids are scattered into per-bin lists first.
static msp_status run_bins(msp_handle* h, const msp_csr* A, const msp_csr* B, const BinPlan& plan,
                           const int* counts, const int32_t* key, bool numeric,
                           const int64_t* crp, int32_t* ccol, void* cval, int32_t* rnnz, int done_bin,
                           int32_t* cnt_out = nullptr) {
    const int m = (int)A->nrows;
    const int nb = plan.table.nb;
    int nonempty = 0, last = -1;
    bool all_group = true;
    for (int b = 1; b <= nb; ++b)
        if (counts[b] > 0 && b != done_bin) {
            ++nonempty;
            last = b;
            all_group = all_group && (plan.spec[b].kind == Kind::Group || plan.spec[b].kind == Kind::Batch);
        }
    if (nonempty == 0) return MSP_OK;
    DevInfo* info = h->info.as<DevInfo>();
    auto rowq = [&](int b) { return &info->queue[numeric ? 1 : 0][b][0]; };
    // bin done_bin was already processed: its rows must not be taken again
    const bool done_rows = done_bin > 0 && counts[done_bin] > 0;
    if (!done_rows && (nonempty == 1 || all_group)) {
        return numeric ? launch_numeric(h, plan.spec[last], m, nullptr, A, B, crp, ccol, cval, cnt_out, rowq(last))
                       : launch_symbolic(h, plan.spec[last], m, nullptr, A, B, rnnz, rowq(last));
    }
    msp_status s = h->perm.ensure((size_t)m * 4);
    if (s != MSP_OK) return s;
    int32_t* perm = h->perm.as<int32_t>();
    int* cursor = &info->cursor[0][0];
    k_zero_words<<<1, 256, 0, h->stream>>>(cursor, kParts * kPartStride);
    if ((s = launch_check("k_zero_words")) != MSP_OK) return s;
    k_scatter<<<(m + 255) / 256, 256, 0, h->stream>>>(
        m, key, plan.table, numeric ? &info->num_part[0][0] : &info->sym_part[0][0],
        numeric ? kScanTile : 256, cursor, perm);
    if ((s = launch_check("k_scatter")) != MSP_OK) return s;
    // The bins are independent.  A bin with fewer rows than it takes to fill
    // the GPU ("narrow": under 8 a compute unit) runs on a side stream, forked
    // after the scatter and joined before the stream goes on, so that its
    // few long-latency rows overlap the other bins' work; wide bins stay on
    // the handle's stream (with no wide bin, it takes narrow ones too).  A
    // global bin with a row for every compute unit fills the GPU with its
    // persistent kernel by itself: it runs alone first.  Largest rows first.
    int first[kNB];
    int start = counts[0];
    for (int b = 1; b <= nb; ++b) {
        first[b] = start;
        start += counts[b];
    }
    auto launch = [&](int b, unsigned* q) {
        return numeric ? launch_numeric(h, plan.spec[b], counts[b], perm + first[b], A, B, crp, ccol, cval, cnt_out, q)
                       : launch_symbolic(h, plan.spec[b], counts[b], perm + first[b], A, B, rnnz, q);
    };
    const Kind gk = plan.spec[nb].kind;
    int alone = -1;
    if ((gk == Kind::Dense || gk == Kind::Bitmap) && nb != done_bin && counts[nb] >= h->num_cu) {
        if ((s = launch(nb, rowq(nb))) != MSP_OK) return s;
        alone = nb;
    }
    auto todo = [&](int b) { return counts[b] > 0 && b != done_bin && b != alone; };
    auto narrow = [&](int b) { return counts[b] < 8 * h->num_cu; };
    int nnarrow = 0, nwide = 0;
    for (int b = 1; b <= nb; ++b)
        if (todo(b)) ++(narrow(b) ? nnarrow : nwide);
    // workers for the narrow bins: the side streams, and the handle's stream
    // when no wide bin needs it
    const int nside = h->fork_ev && nnarrow > 0 && nnarrow + nwide >= 2
                          ? std::min(kSideStreams, nwide > 0 ? nnarrow : nnarrow - 1) : 0;
    const hipStream_t main_st = h->stream;
    hipError_t e = hipSuccess;
    if (nside > 0) {
        if ((e = hipEventRecord(h->fork_ev, main_st)) != hipSuccess) return hip_fail(e, "hipEventRecord(fork)");
        for (int i = 0; i < nside; ++i)
            if ((e = hipStreamWaitEvent(h->side[i], h->fork_ev, 0)) != hipSuccess)
                return hip_fail(e, "hipStreamWaitEvent(fork)");
    }
    const int nworkers = nside + (nwide > 0 ? 0 : 1);
    int k = 0;
    for (int b = nb; b >= 1 && s == MSP_OK; --b) {
        if (!todo(b)) continue;
        int w = -1;                                  // -1: the handle's stream
        if (nside > 0 && narrow(b)) {
            w = k++ % nworkers;
            if (nwide == 0) --w;                     // worker 0 is the handle's stream
        }
        h->stream = w < 0 ? main_st : h->side[w];
        s = launch(b, rowq(b));
    }
    h->stream = main_st;
    // join whatever was forked, also after a failed launch
    for (int i = 0; i < nside && e == hipSuccess; ++i)
        if ((e = hipEventRecord(h->join_ev[i], h->side[i])) == hipSuccess)
            e = hipStreamWaitEvent(main_st, h->join_ev[i], 0);
    if (s != MSP_OK) return s;
    return e == hipSuccess ? MSP_OK : hip_fail(e, "joining the side streams");
}

msp_status run_symbolic_bins(msp_handle* h, const msp_csr* A, const msp_csr* B, const BinPlan& plan,
                             const int* counts_host, int32_t* row_nnz, int done_bin) {
    return run_bins(h, A, B, plan, counts_host, h->u.as<int32_t>(), false, nullptr, nullptr, nullptr, row_nnz,
                    done_bin);
}

msp_status run_scan(msp_handle* h, int m, const int32_t* row_nnz, int64_t* row_ptr, const BinPlan* plan,
                    int publish_seq) {
    const int tiles = std::max(1, (m + kScanTile - 1) / kScanTile);
    const size_t need = (size_t)tiles * 8;
    if (need > h->tiles.bytes || h->scan_epoch == 0 || h->scan_epoch >= 0xffff || h->tiles.arena) {
        // fresh tile states (or tiles in a scratch whose contents are
        // unknown): zero them with a fill kernel and restart the epochs
        msp_status s = h->tiles.ensure(need);
        if (s != MSP_OK) return s;
        const int words = (int)(h->tiles.bytes / 4);
        k_zero_words<<<std::min(1024, (words + 255) / 256), 256, 0, h->stream>>>((int*)h->tiles.ptr, words);
        if ((s = launch_check("k_zero_words(scan state)")) != MSP_OK) return s;
        h->scan_epoch = 0;
    }
    ++h->scan_epoch;
    BinTable bt;
    memset(&bt, 0, sizeof(bt));
    if (plan) bt = plan->table;
    k_scan_lookback<<<tiles, kScanBS, 0, h->stream>>>(m, row_nnz, h->tiles.as<unsigned long long>(),
                                                     h->scan_epoch, row_ptr, bt, h->info.as<DevInfo>(),
                                                     publish_seq ? h->dsum : nullptr, publish_seq);
    return launch_check("k_scan_lookback");
}

msp_status run_numeric_bins(msp_handle* h, const msp_csr* A, const msp_csr* B, const BinPlan& plan,
                            const int* counts_host, const int32_t* key, const int64_t* crp,
                            int32_t* ccol, void* cval, int32_t* cnt_out) {
    return run_bins(h, A, B, plan, counts_host, key, true, crp, ccol, cval, nullptr, 0, cnt_out);
}

msp_status check_pair(const msp_csr* A, const msp_csr* B) {
    msp_status s;
    if ((s = check_csr(A, "A")) != MSP_OK) return s;
    if ((s = check_csr(B, "B")) != MSP_OK) return s;
    if (A->ncols != B->nrows)
        return fail(MSP_ERR_SHAPE, "A is %lld x %lld but B is %lld x %lld", (long long)A->nrows,
                    (long long)A->ncols, (long long)B->nrows, (long long)B->ncols);
    if (A->dtype != B->dtype) return fail(MSP_ERR_DTYPE, "A and B value types differ");
    return MSP_OK;
}

msp_status validate_inputs(msp_handle* h, const msp_csr* A, const msp_csr* B) {
    msp_status s;
    if ((s = zero_info(h)) != MSP_OK) return s;
    for (const msp_csr* M : {A, B}) {
        if (M->nrows == 0) continue;
        k_validate<<<(int)((M->nrows + 255) / 256), 256, 0, h->stream>>>(M->nrows, M->ncols, M->nnz, M->row_ptr,
                                                                         M->col, h->info.as<DevInfo>());
        if ((s = launch_check("k_validate")) != MSP_OK) return s;
    }
    if ((s = read_info(h)) != MSP_OK) return s;
    const int err = h->hinfo->err;
    if (err & kErrRange) return fail(MSP_ERR_INVALID_ARG, "input CSR has an index out of range or a non-monotone row_ptr");
    if (err & kErrUnsorted) return fail(MSP_ERR_UNSORTED_OR_DUP, "input CSR has unsorted or duplicate columns");
    return MSP_OK;
}

msp_status device_error(int err) {
    if (err & kErrScan) return fail(MSP_ERR_HIP, "internal: prefix-sum look-back wait exceeded its bound");
    if (err & kErrProbe) return fail(MSP_ERR_HIP, "internal: hash probe bound exceeded");
    if (err & kErrCount) return fail(MSP_ERR_HIP, "internal: numeric row count differs from symbolic count");
    return MSP_OK;
}

// Window records for the numeric global bin of this product, sized from the
// symbolic bin sizes (the rows of the workgroup-hash bins whose bound exceeds
// the numeric threshold, and of the bitmap bin); none (cur_rec.cnt null)
// without a numeric plan, when the windowed kernel does not fit the LDS,
// for more than kWinMaxNw windows, or above 4 GiB of records.
static msp_status setup_records(msp_handle* h, const msp_csr* A, const msp_csr* B, const BinPlan& sp,
                                const int* counts, const BinPlan* np) {
    h->cur_rec = WinRec{};
    if (!np || win_lds(h) == 0) return MSP_OK;
    const long long nw = (B->ncols + kWin - 1) / kWin;
    if (nw <= 0 || nw > kWinMaxNw) return MSP_OK;
    const int thresh = np->table.nb > 1 ? np->table.umax[np->table.nb - 1] : 0;
    long long cap = counts[sp.table.nb];
    for (int b = 1; b < sp.table.nb; ++b)
        if (sp.spec[b].kind == Kind::Block && sp.table.umax[b] > thresh) cap += counts[b];
    if (cap <= 0 || cap * nw * 2 > (4LL << 30)) return MSP_OK;
    // without room for the records the global bin counts its rows itself
    msp_status r;
    if ((r = h->win_islot.ensure((size_t)std::max<long long>(A->nrows, 1) * 4)) != MSP_OK ||
        (r = h->win_row.ensure((size_t)cap * 4)) != MSP_OK ||
        (r = h->win_cnt.ensure((size_t)cap * (size_t)nw * 2)) != MSP_OK ||
        (r = h->win_rbm.ensure((size_t)cap * 4)) != MSP_OK)
        return r == MSP_ERR_OOM ? MSP_OK : r;
    WinRec rec;
    rec.islot = h->win_islot.as<int32_t>();
    rec.row = h->win_row.as<int32_t>();
    rec.cnt = h->win_cnt.as<uint16_t>();
    rec.nrec = &h->info.as<DevInfo>()->win_nrec;
    rec.cap = (int)cap;
    rec.nw = (int)nw;
    rec.thresh = thresh;
    rec.rec_bm = h->win_rbm.as<int32_t>();
    // bitmap store for the bitmap bin's rows with at least one product per
    // 16 columns (a bitmap pass over their products would move at least
    // twice the bitmap's bytes); at most min(16 GiB, 1/16 of the device)
    rec.bms = nullptr;
    rec.nbms = &h->info.as<DevInfo>()->win_nbms;
    rec.bms_cap = 0;
    rec.bms_min_prod = nw * (long long)kWin / 16;
    const long long row_bytes = nw * (long long)kWin / 8;
    const long long budget = std::min<long long>(16LL << 30, (long long)(h->total_mem / 16));
    const long long bcap = std::min<long long>(counts[sp.table.nb], budget / row_bytes);
    if (bcap > 0 && (r = h->win_bms.ensure((size_t)(bcap * row_bytes))) == MSP_OK) {
        rec.bms = h->win_bms.as<uint32_t>();
        rec.bms_cap = (int)bcap;
    } else if (r != MSP_OK && r != MSP_ERR_OOM) {
        return r;
    }
    h->cur_rec = rec;
    return MSP_OK;
}

// symbolic phase up to row_nnz (shared by msp_spgemm and msp_spgemm_symbolic).
// When the plan starts with a merge bin, the statistics pass and that bin
// run as one kernel with a speculative scan queued behind it (into
// `row_ptr`, with the numeric histogram of `np`); if every row was counted
// there, the scan's summary (nnz and numeric bin sizes) is in h->hsum and
// *scanned is set.
static msp_status symbolic_phase(msp_handle* h, const msp_csr* A, const msp_csr* B, const msp_opts* opts,
                                 const msp_tuning& t, int64_t* row_ptr, const BinPlan* np, bool* scanned) {
    const int m = (int)A->nrows;
    msp_status s;
    *scanned = false;
    h->cur_rec = WinRec{};
    if ((s = h->rnnz.ensure((size_t)std::max(m, 1) * 4)) != MSP_OK) return s;
    const BinPlan sp = symbolic_plan(t, opts && opts->force_spill);
    if ((s = zero_info(h)) != MSP_OK) return s;
    const bool merge_first = m > 0 && sp.table.nb > 1 && sp.spec[1].kind == Kind::Merge;
    if (merge_first) {
        const int grid = (m + 255) / 256;
        if ((s = h->u.ensure((size_t)m * 4)) != MSP_OK) return s;
        if ((s = h->bsum.ensure((size_t)grid * 8)) != MSP_OK) return s;
        DevInfo* info = h->info.as<DevInfo>();
        BinTable nt;
        memset(&nt, 0, sizeof(nt));
        if (np) nt = np->table;
        h->prof.begin(MSP_PHASE_SYMBOLIC, h->stream);
        const bool small = narrow_symbolic(operands_of(A, B));   // 32-bit positions and offsets
        const int tiles = (m + kWsTile - 1) / kWsTile;
        const long long super_rows = super_tile_rows(tiles);
#define MSP_FUSED(KK, IT)                                                                                 \
    k_sym_fused<KK, IT><<<grid, 256, 0, h->stream>>>(m, B->ncols, A->row_ptr, A->col, B->row_ptr, B->col,   \
                                                     h->u.as<int32_t>(), h->rnnz.as<int32_t>(), sp.table,  \
                                                     sp.table.umax[1], info, nt, h->bsum.as<long long>(),  \
                                                     super_rows)
        if (sp.spec[1].lanes == 4) { if (small) MSP_FUSED(4, int); else MSP_FUSED(4, long long); }
        else { if (small) MSP_FUSED(8, int); else MSP_FUSED(8, long long); }
#undef MSP_FUSED
        if ((s = launch_check("k_sym_fused")) != MSP_OK) return s;
        h->prof.end(h->stream);
        h->prof.begin(MSP_PHASE_SCAN, h->stream);
        const int seq = ++h->sum_seq;
        k_scan_fused<<<tiles, kWsBS, 0, h->stream>>>(m, h->rnnz.as<int32_t>(), h->bsum.as<long long>(), super_rows,
                                                     row_ptr,
                                                     sp.table.nb, info, h->dsum, seq);
        if ((s = launch_check("k_scan_fused")) != MSP_OK) return s;
        h->prof.end(h->stream);
        if ((s = wait_summary(h, seq, true, h->info.as<DevInfo>()->num_part, sp.table.nb)) != MSP_OK) return s;
        if ((s = device_error(h->hsum->err)) != MSP_OK) return s;
        if (h->hsum->nnz >= 0) {
            *scanned = true;
            return MSP_OK;
        }
        // other symbolic bins have rows: run them (the merge bin is done);
        // the full scan counts the numeric bins afresh
        int counts[kNB];
        for (int b = 0; b < kNB; ++b) counts[b] = h->hsum->counts[b];
        k_zero_words<<<1, 256, 0, h->stream>>>(&info->num_part[0][0], kParts * kPartStride);
        if ((s = launch_check("k_zero_words")) != MSP_OK) return s;
        if ((s = setup_records(h, A, B, sp, counts, np)) != MSP_OK) return s;
        h->prof.begin(MSP_PHASE_SYMBOLIC, h->stream);
        s = run_symbolic_bins(h, A, B, sp, counts, h->rnnz.as<int32_t>(), 1);
        h->prof.end(h->stream);
        return s;
    }
    // no merge bin (or no rows): the statistics pass, its bin sizes
    // (published to the host by a one-workgroup kernel), then the bins
    h->prof.begin(MSP_PHASE_ROW_STATS, h->stream);
    const int seq = m > 0 ? ++h->sum_seq : 0;
    if ((s = run_row_stats(h, A, B, sp, nullptr, nullptr, nullptr, seq)) != MSP_OK) return s;
    h->prof.end(h->stream);
    h->prof.begin(MSP_PHASE_SYMBOLIC, h->stream);
    int counts[kNB] = {};
    if (m > 0) {
        if ((s = wait_summary(h, seq, false, h->info.as<DevInfo>()->sym_part)) != MSP_OK) return s;
        if ((s = device_error(h->hsum->err)) != MSP_OK) return s;
        for (int b = 0; b < kNB; ++b) counts[b] = h->hsum->counts[b];
    } else if ((s = take_pending_error(h)) != MSP_OK) {
        return s;
    }
    if ((s = setup_records(h, A, B, sp, counts, np)) != MSP_OK) return s;
    s = run_symbolic_bins(h, A, B, sp, counts, h->rnnz.as<int32_t>(), 0);
    h->prof.end(h->stream);
    return s;
}

}  // namespace msp

namespace msp {

// The plain two-phase product; `alloc_cv` provides the single allocation of
// C's columns and values once nnz(C) is known (the caller's allocator, or a
// workspace for internal sub-products).
msp_status spgemm_core(msp_handle* h, const msp_csr* A, const msp_csr* B, msp_csr_out* C, const msp_opts* opts,
                       const std::function<void*(size_t)>& alloc_cv, const std::function<void(void*)>& free_cv,
                       const CPlace* place) {
    if (!h) return fail(MSP_ERR_INVALID_ARG, "null handle");
    if (!C) return fail(MSP_ERR_INVALID_ARG, "C is NULL");
    if (place && (!C->row_ptr || (place->cap > 0 && (!place->col || !place->val)) || place->cap < 0))
        return fail(MSP_ERR_INVALID_ARG, "C's row_ptr, col and val buffers are required (capacity %lld)",
                    (long long)place->cap);
    msp_status s = check_pair(A, B);
    if (s != MSP_OK) return s;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const msp_tuning t = effective_tuning(h, opts);
    const int m = (int)A->nrows;
    if (opts && opts->validate && (s = validate_inputs(h, A, B)) != MSP_OK) return s;
    // the window records belong to this product only
    struct RecScope {
        msp_handle* h;
        ~RecScope() { h->cur_rec = WinRec{}; }
    } rec_scope{h};

    bool own_rp = false;
    if (!C->row_ptr) {
        C->row_ptr = (int64_t*)h->alloc(h->alloc_ctx, (size_t)(m + 1) * 8, h->stream);
        if (!C->row_ptr) return fail(MSP_ERR_OOM, "allocation of C.row_ptr failed");
        own_rp = true;
    }
    C->col = nullptr;
    C->val = nullptr;
    auto cleanup = [&](msp_status st) {
        if (C->col && !place) free_cv(C->col);   // col and val share it
        C->col = nullptr;
        C->val = nullptr;
        if (own_rp) { h->free_fn(h->alloc_ctx, C->row_ptr, h->stream); C->row_ptr = nullptr; }
        return st;
    };

    BinPlan np = numeric_plan(t, opts && opts->force_spill);
    bool scanned = false;
    if ((s = symbolic_phase(h, A, B, opts, t, C->row_ptr, &np, &scanned)) != MSP_OK) return cleanup(s);
    if (scanned && np.table.nb > 1 && np.spec[1].kind == Kind::Merge && np.spec[1].lanes == 8) {
        // every merge row of this product was seen by the fused pass: the
        // numeric merge needs no more heads than its longest A row (fewer
        // heads, fewer registers, more waves in flight)
        const int na = h->hsum->merge_na;
        if (na <= 4) np.spec[1].lanes = 4;
        else if (na <= 6) np.spec[1].lanes = 6;
    }
    if (!scanned) {
        h->prof.begin(MSP_PHASE_SCAN, h->stream);
        const int seq = ++h->sum_seq;         // the scan publishes nnz(C) and the numeric bin sizes
        if ((s = run_scan(h, m, h->rnnz.as<int32_t>(), C->row_ptr, &np, seq)) != MSP_OK) return cleanup(s);
        h->prof.end(h->stream);
        if ((s = wait_summary(h, seq, true, h->info.as<DevInfo>()->num_part)) != MSP_OK) return cleanup(s);
        if ((s = device_error(h->hsum->err)) != MSP_OK) return cleanup(s);
    }
    const long long nnz = h->hsum->nnz;
    int counts[kNB];
    for (int b = 0; b < kNB; ++b) counts[b] = h->hsum->counts[b];
    const size_t vsz = A->dtype == MSP_F64 ? 8 : 4;
    C->nrows = m;
    C->ncols = B->ncols;
    C->nnz = nnz;
    C->dtype = A->dtype;
    if (place && nnz > place->cap) {
        C->col = nullptr;
        return fail(MSP_ERR_INVALID_ARG, "C has %lld nonzeros, more than the capacity %lld given", nnz,
                    (long long)place->cap);
    }
    if (nnz > 0) {
        // one allocation: columns, then values at the next 256-byte boundary
        const size_t voff = ((size_t)nnz * 4 + 255) & ~(size_t)255;
        void* vals;
        if (place) {
            C->col = place->col;
            vals = place->val;
        } else {
            void* base = alloc_cv(voff + (size_t)nnz * vsz);
            if (!base) return cleanup(fail(MSP_ERR_OOM, "allocation of C (%lld nonzeros) failed", nnz));
            C->col = (int32_t*)base;
            vals = (char*)base + voff;
        }
        h->prof.begin(MSP_PHASE_NUMERIC, h->stream);
        if ((s = run_numeric_bins(h, A, B, np, counts, h->rnnz.as<int32_t>(), C->row_ptr, C->col, vals,
                                  nullptr)) != MSP_OK)
            return cleanup(s);
        h->prof.end(h->stream);
        C->val = vals;
        // the numeric kernels' consistency flags reach the host through the
        // next call's first kernel, or through msp_sync
    }
    return MSP_OK;
}

}  // namespace msp

extern "C" msp_status msp_spgemm(msp_handle* h, const msp_csr* A, const msp_csr* B, msp_csr_out* C,
                                 const msp_opts* opts) {
    if (!h) return fail(MSP_ERR_INVALID_ARG, "null handle");
    return spgemm_core(
        h, A, B, C, opts, [h](size_t bytes) -> void* { return h->alloc(h->alloc_ctx, bytes, h->stream); },
        [h](void* ptr) { h->free_fn(h->alloc_ctx, ptr, h->stream); });
}

extern "C" msp_status msp_spgemm_symbolic(msp_handle* h, const msp_csr* A, const msp_csr* B, int32_t* row_nnz,
                                          int64_t* nnz_total, const msp_opts* opts) {
    if (!h) return fail(MSP_ERR_INVALID_ARG, "null handle");
    msp_status s = check_pair(A, B);
    if (s != MSP_OK) return s;
    if (!row_nnz && A->nrows > 0) return fail(MSP_ERR_INVALID_ARG, "row_nnz is NULL");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const msp_tuning t = effective_tuning(h, opts);
    if (opts && opts->validate && (s = validate_inputs(h, A, B)) != MSP_OK) return s;
    bool scanned = false;     // total through the scan (no row_ptr output)
    if ((s = symbolic_phase(h, A, B, opts, t, nullptr, nullptr, &scanned)) != MSP_OK) return s;
    const int m = (int)A->nrows;
    if (m > 0) {
        e = hipMemcpyAsync(row_nnz, h->rnnz.ptr, (size_t)m * 4, hipMemcpyDeviceToDevice, h->stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(row_nnz)");
    }
    if (!scanned) {
        const int seq = ++h->sum_seq;
        if ((s = run_scan(h, m, h->rnnz.as<int32_t>(), nullptr, nullptr, seq)) != MSP_OK) return s;
        if ((s = wait_summary(h, seq, true, h->info.as<DevInfo>()->num_part)) != MSP_OK) return s;
        if ((s = device_error(h->hsum->err)) != MSP_OK) return s;
    }
    if (nnz_total) *nnz_total = h->hsum->nnz;
    return MSP_OK;
}

extern "C" msp_status msp_row_features(msp_handle* h, const msp_csr* A, const msp_csr* B, int64_t* prod,
                                       float* features) {
    if (!h) return fail(MSP_ERR_INVALID_ARG, "null handle");
    msp_status s = check_pair(A, B);
    if (s != MSP_OK) return s;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const int m = (int)A->nrows;
    if ((s = h->rnnz.ensure((size_t)std::max(m, 1) * 4)) != MSP_OK) return s;
    BinPlan none;
    memset(&none, 0, sizeof(none));
    if ((s = zero_info(h)) != MSP_OK) return s;
    return run_row_stats(h, A, B, none, prod, features ? features : nullptr, nullptr);
}

extern "C" msp_status msp_omar(msp_handle* h, const msp_csr* A, int64_t group, int64_t* distinct) {
    if (!h) return fail(MSP_ERR_INVALID_ARG, "null handle");
    if (!distinct) return fail(MSP_ERR_INVALID_ARG, "distinct is NULL");
    msp_status s = check_csr(A, "A");
    if (s != MSP_OK) return s;
    if (group < 1 || group > kOmarMaxGroup) return fail(MSP_ERR_INVALID_ARG, "group must be in 1..4096");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if ((s = zero_info(h)) != MSP_OK) return s;
    if (A->nnz > 0) {
        const long long blocks = std::min<long long>((A->nnz + 255) / 256, 64LL * h->num_cu);
        DevInfo* info = h->info.as<DevInfo>();
        k_omar<<<(int)blocks, 256, 0, h->stream>>>(A->nrows, A->nnz, A->row_ptr, A->col, group,
                                                    &info->omar_distinct);
        if ((s = launch_check("k_omar")) != MSP_OK) return s;
    }
    if ((s = read_info(h)) != MSP_OK) return s;
    *distinct = (int64_t)h->hinfo->omar_distinct;
    return MSP_OK;
}

extern "C" msp_status msp_share_stats_get(msp_handle* h, msp_share_stats* out) {
    if (!h || !out) return fail(MSP_ERR_INVALID_ARG, "null argument");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    msp_status s = read_info(h);
    if (s != MSP_OK) return s;
    out->batches = h->hinfo->share_batches;
    out->a_entries = h->hinfo->share_nnz;
    out->b_rows = h->hinfo->share_rows;
    return MSP_OK;
}

extern "C" long long msp_internal_summary_fallbacks(const msp_handle* h) { return h ? h->summary_fallbacks : -1; }

extern "C" int msp_internal_unsupported_plans(int verbose) { return msp::count_unsupported_plans(verbose); }

extern "C" msp_status msp_autotune(msp_handle* h, const msp_csr* A, const msp_csr* B, const msp_tuning* cand,
                                   int ncand, int reps, msp_tuning* best, double* times_ms) {
    if (!h || !cand || ncand <= 0 || reps <= 0 || !best) return fail(MSP_ERR_INVALID_ARG, "bad argument");
    msp_status s = check_pair(A, B);
    if (s != MSP_OK) return s;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return hip_fail(e, "hipEventCreate"); }
    // one product: C's row pointers from the allocator, its columns and
    // values released through it once the call has completed
    auto run = [&](const msp_opts* o, bool timed, float* ms) -> msp_status {
        msp_csr_out C;
        memset(&C, 0, sizeof(C));
        hipError_t er;
        if (timed && (er = hipEventRecord(e0, h->stream)) != hipSuccess) return hip_fail(er, "hipEventRecord");
        msp_status st = msp_spgemm(h, A, B, &C, o);
        if (st == MSP_OK && timed && (er = hipEventRecord(e1, h->stream)) != hipSuccess)
            st = hip_fail(er, "hipEventRecord");
        const msp_status sy = msp_sync(h);
        if (st == MSP_OK) st = sy;
        if (st == MSP_OK && timed && (er = hipEventElapsedTime(ms, e0, e1)) != hipSuccess)
            st = hip_fail(er, "hipEventElapsedTime");
        if (C.col) h->free_fn(h->alloc_ctx, C.col, h->stream);
        if (C.row_ptr) h->free_fn(h->alloc_ctx, C.row_ptr, h->stream);
        return st;
    };
    double best_ms = INFINITY;
    int best_i = -1;
    msp_status last_err = MSP_OK;
    for (int c = 0; c < ncand; ++c) {
        double med = INFINITY;
        msp_opts o;
        memset(&o, 0, sizeof(o));
        o.tuning = cand[c];
        s = check_tuning(&o.tuning);
        if (s == MSP_OK) s = run(&o, false, nullptr);          // warm
        std::vector<double> ts;
        for (int r = 0; r < reps && s == MSP_OK; ++r) {
            float ms = 0.f;
            if ((s = run(&o, true, &ms)) == MSP_OK) ts.push_back(ms);
        }
        if (s == MSP_OK && !ts.empty()) {
            std::sort(ts.begin(), ts.end());
            med = ts[ts.size() / 2];
        } else {
            last_err = s;
        }
        if (s == MSP_ERR_HIP) {        // the device reported an error: try nothing more on it
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return s;
        }
        if (times_ms) times_ms[c] = med;
        if (med < best_ms) {
            best_ms = med;
            best_i = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best_i < 0) return last_err != MSP_OK ? last_err : fail(MSP_ERR_INVALID_ARG, "no candidate ran");
    *best = cand[best_i];
    return check_tuning(best);
}

// Every per-call workspace of the plain product in the device's fixed
// scratch array (the handle's own workspaces are set aside meanwhile), C
// in the caller's buffers, no profiling events: nothing is allocated.
extern "C" msp_status msp_spgemm_noalloc(msp_handle* h, const msp_csr* A, const msp_csr* B, msp_csr_out* C,
                                         int64_t capacity, const msp_opts* opts) {
    if (!h) return fail(MSP_ERR_INVALID_ARG, "null handle");
    if (!C) return fail(MSP_ERR_INVALID_ARG, "C is NULL");
    msp_status s = check_pair(A, B);
    if (s != MSP_OK) return s;
    if (!h->scratch) return fail(MSP_ERR_UNSUPPORTED, "no scratch on this device");
    // the per-row workspaces alone must fit: refused before anything runs
    const long long m = A->nrows;
    if (m * 24 + (1 << 20) > (long long)MSP_NOALLOC_SCRATCH_BYTES)
        return fail(MSP_ERR_INVALID_ARG, "%lld rows exceed the no-allocation scratch (%lld bytes, about %lld rows)",
                    m, (long long)MSP_NOALLOC_SCRATCH_BYTES, ((long long)MSP_NOALLOC_SCRATCH_BYTES - (1 << 20)) / 24);
    Arena ar;
    ar.base = (char*)h->scratch;
    ar.size = MSP_NOALLOC_SCRATCH_BYTES;
    DevBuf* bufs[] = {&h->u, &h->rnnz, &h->perm, &h->tiles, &h->sbm, &h->prod, &h->bsum, &h->gsl,
                      &h->win_islot, &h->win_row, &h->win_cnt, &h->win_bslot, &h->win_wpos, &h->win_fb,
                      &h->win_rbm, &h->win_bms, &h->lr_list, &h->lr_base, &h->lr_chunk, &h->lr_acc};
    constexpr int nb = sizeof(bufs) / sizeof(bufs[0]);
    DevBuf saved[nb];
    for (int i = 0; i < nb; ++i) {
        saved[i] = *bufs[i];
        *bufs[i] = DevBuf{};
        bufs[i]->arena = &ar;
    }
    const bool prof_on = h->prof.on;
    h->prof.on = false;
    g_noalloc = true;
    CPlace place{C->col, C->val, capacity};
    s = spgemm_core(
        h, A, B, C, opts, [](size_t) -> void* { return nullptr; }, [](void*) {}, &place);
    g_noalloc = false;
    h->prof.on = prof_on;
    for (int i = 0; i < nb; ++i) *bufs[i] = saved[i];
    C->col = place.col;                 // the caller's buffers, whatever happened
    C->val = place.val;
    return s;
}
