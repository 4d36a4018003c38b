// Batched products in one graph launch.
//
// A batch of independent products (or of Galerkin triple products
// R_p (A_p P_p)) is stored packed: one row_ptr array with global offsets, one
// col/val array, columns local to each problem.  Every pass of the plain
// pipeline (row statistics, binning, symbolic counts, prefix sum, numeric
// accumulation) then runs once over the rows of all problems together: the
// kernels map a row to its problem only to find that problem's B rows.
//
// A plan is made once per batch shape.  Its first, eager run reads the bin
// sizes and nnz(C) on the host, sizes the plan's own workspace and output
// arenas, and records which bins need kernels; the same launch sequence is
// then captured into a hipGraph.  In the graph every bin kernel reads its
// row count from device memory (written by a small kernel from the bin
// counters), so a replay never waits for the host.  A replay whose rows
// would need a kernel that the plan lacks, or whose output outgrows the
// arena, sets an error flag and skips the remaining work; the flag is
// reported when the caller collects the results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "msp.h"

using namespace msp;

namespace msp {

// ---------------------------------------------------------------------------
// device helpers of the batched pipeline
// ---------------------------------------------------------------------------
// Per-bin work items {count, start} of one pass from the partitioned bin
// counters, plus an "all rows" item at index kNB.  Bins without a kernel in
// the plan must be empty, and nnz (when given) must fit the arena; otherwise
// the flag is set and every count becomes 0, so the rest of the replay is a
// sequence of empty kernels.
static __global__ void __launch_bounds__(64)
k_bin_work(const int* __restrict__ part, int nb, unsigned planned, long long rows, const long long* nnz,
           long long cap, int* __restrict__ work, int* flag) {
    __shared__ int cnt[kNB];
    const int t = threadIdx.x;
    if (t < kNB) {
        int c = 0;
        if (t <= nb)
            for (int p = 0; p < kParts; ++p) c += part[p * kPartStride + t];
        cnt[t] = c;
    }
    __syncthreads();
    if (t == 0) {
        int f = *flag;
        for (int b = 1; b <= nb; ++b)
            if (cnt[b] > 0 && !((planned >> b) & 1u)) f |= kErrPlan;
        if (nnz && *nnz > cap) f |= kErrCapacity;
        *flag = f;
        int start = 0;
        for (int b = 0; b < kNB; ++b) {
            work[2 * b] = f ? 0 : cnt[b];
            work[2 * b + 1] = start;
            start += cnt[b];
        }
        work[2 * kNB] = f ? 0 : (int)rows;
        work[2 * kNB + 1] = 0;
    }
}

// fold a pass's internal error bits into the plan's flag
static __global__ void k_fold_err(const DevInfo* info, int* flag) {
    if (threadIdx.x == 0 && info->err) *flag |= info->err;
}

// Canonical per-problem row pointers of the final product: problem p's
// array starts at rp_local + row_start[p] + p; bases[p] = first entry of
// problem p in the arena (bases[nprob] = nnz).
static __global__ void __launch_bounds__(256)
k_batch_finalize(long long M, int nprob, const int64_t* __restrict__ crp, RowMap mp, int64_t* __restrict__ rp_local,
                 int64_t* __restrict__ bases, const int* flag) {
    if (*flag) return;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < M) {
        const int p = map_prob(mp, i);
        rp_local[i + p] = crp[i] - crp[mp.row_start[p]];
    }
    if (i <= nprob) {
        const long long b0 = crp[mp.row_start[i]];
        bases[i] = b0;
        if (i < nprob) rp_local[mp.row_start[i + 1] + i] = crp[mp.row_start[i + 1]] - b0;
    }
}

// ---------------------------------------------------------------------------
// plan state
// ---------------------------------------------------------------------------
struct BatchStage {
    Operands op{};
    long long M = 0;
    DevBuf tile_prob, row_start, boff, ncols;    // the RowMap arrays
    RowMap mp{};
    BinPlan sp{}, np{};
    unsigned sym_planned = 0, num_planned = 0;  // bins with kernels
    int sym_rows[kNB] = {}, num_rows[kNB] = {}; // plan-time bin sizes (grid sizes)
    bool sym_merge_all = false;                 // merge bin runs over all rows, filtering by bound
    bool sym_scatter = false;                   // other symbolic bins need the row lists
    bool sym_fused = false;                     // replays: statistics and merge bin in one kernel
    int num_single = -1;                        // numeric bin that takes all rows in order
    DevBuf crp, cv, wsym, wnum;                 // row pointers, col+val arena, work items
    DevBuf tick;                                // work-queue counter of each numeric bin
    long long nnz = 0, cap = 0;
    size_t voff = 0;                            // values start at cv + voff
};

}  // namespace msp

struct msp_batch {
    int device = 0;
    msp_handle inner;               // private workspace and capture stream
    int nstage = 0;
    msp::BatchStage st[2];
    int nprob = 0;
    std::vector<int64_t> row_start;  // rows of each output problem (host)
    std::vector<int64_t> ncols;      // columns of each output problem (host)
    msp::DevBuf rp_local, bases, flag;
    int queue_rows = 0;              // rows per ticket of the numeric merge's queue (0: static ranges)
    int64_t* hbases = nullptr;       // pinned
    int* hflag = nullptr;            // pinned
    bool pending = false;            // a replay whose flag has not been read
    bool have_result = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    msp_dtype dtype = MSP_F64;
};

namespace msp {

static msp_status launch_ok(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return MSP_OK;
}

static msp_status check_batch_csr(const msp_batch_csr* M, const char* name) {
    if (!M) return fail(MSP_ERR_INVALID_ARG, "%s is NULL", name);
    if (M->nprob <= 0) return fail(MSP_ERR_INVALID_ARG, "%s: a batch needs at least one problem", name);
    if (!M->row_start || !M->ncols) return fail(MSP_ERR_INVALID_ARG, "%s: row_start/ncols are NULL", name);
    if (M->row_start[0] != 0) return fail(MSP_ERR_INVALID_ARG, "%s: row_start[0] must be 0", name);
    for (int p = 0; p < M->nprob; ++p) {
        if (M->row_start[p + 1] < M->row_start[p]) return fail(MSP_ERR_INVALID_ARG, "%s: row_start decreases", name);
        if (M->ncols[p] < 0 || M->ncols[p] > INT32_MAX)
            return fail(MSP_ERR_INVALID_ARG, "%s: problem %d has %lld columns", name, p, (long long)M->ncols[p]);
    }
    if (M->row_start[M->nprob] > kMaxRows)
        return fail(MSP_ERR_INDEX_OVERFLOW, "%s: a batch holds at most %lld rows", name, kMaxRows);
    if (M->dtype != MSP_F32 && M->dtype != MSP_F64) return fail(MSP_ERR_DTYPE, "%s: dtype must be F32 or F64", name);
    if (!M->row_ptr) return fail(MSP_ERR_INVALID_ARG, "%s.row_ptr is NULL", name);
    if (M->nnz < 0 || (M->nnz > 0 && (!M->col || !M->val))) return fail(MSP_ERR_INVALID_ARG, "%s: bad nnz/col/val", name);
    return MSP_OK;
}

// X_p * Y_p for every p: X_p's columns are Y_p's rows
static msp_status check_batch_pair(const msp_batch_csr* X, const msp_batch_csr* Y, const char* xn, const char* yn) {
    if (X->nprob != Y->nprob) return fail(MSP_ERR_SHAPE, "%s and %s hold different numbers of problems", xn, yn);
    if (X->dtype != Y->dtype) return fail(MSP_ERR_DTYPE, "%s and %s value types differ", xn, yn);
    for (int p = 0; p < X->nprob; ++p) {
        const long long yr = Y->row_start[p + 1] - Y->row_start[p];
        if (X->ncols[p] != yr)
            return fail(MSP_ERR_SHAPE, "problem %d: %s has %lld columns but %s has %lld rows", p, xn,
                        (long long)X->ncols[p], yn, yr);
    }
    return MSP_OK;
}

static msp_status upload(DevBuf& b, const void* src, size_t bytes, hipStream_t s) {
    msp_status r = b.ensure(std::max(bytes, (size_t)8));
    if (r != MSP_OK) return r;
    hipError_t e = hipMemcpyAsync(b.ptr, src, bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? MSP_OK : hip_fail(e, "hipMemcpyAsync(batch map)");
}

// RowMap of a stage: rows of X (row_start), B-row offsets into the packed Y
// (y_row_start) and the output widths
static msp_status build_map(BatchStage& S, int nprob, const int64_t* x_row_start, const int64_t* y_row_start,
                            const int64_t* out_ncols, hipStream_t s) {
    const long long M = x_row_start[nprob];
    const long long tiles = std::max(1LL, (M + 63) / 64);
    std::vector<int32_t> tp((size_t)tiles);
    int p = 0;
    for (long long t = 0; t < tiles; ++t) {
        const long long g = t * 64;
        while (p + 1 < nprob && x_row_start[p + 1] <= g) ++p;   // last p with row_start[p] <= g
        tp[(size_t)t] = p;
    }
    msp_status r;
    if ((r = upload(S.tile_prob, tp.data(), tp.size() * 4, s)) != MSP_OK) return r;
    if ((r = upload(S.row_start, x_row_start, (size_t)(nprob + 1) * 8, s)) != MSP_OK) return r;
    if ((r = upload(S.boff, y_row_start, (size_t)nprob * 8, s)) != MSP_OK) return r;
    if ((r = upload(S.ncols, out_ncols, (size_t)nprob * 8, s)) != MSP_OK) return r;
    S.mp = RowMap{S.tile_prob.as<int32_t>(), S.row_start.as<int64_t>(), S.boff.as<int64_t>(), S.ncols.as<int64_t>()};
    S.M = M;
    return MSP_OK;
}

// One stage: eager (sizes on the host, allocations) or queued for capture.
static msp_status run_stage(msp_batch* b, int si, bool eager) {
    msp_handle* h = &b->inner;
    BatchStage& S = b->st[si];
    hipStream_t st = h->stream;
    const int M = (int)S.M;
    DevInfo* info = h->info.as<DevInfo>();
    int* flag = b->flag.as<int>();
    msp_status s;
    if (eager) {
        if ((s = h->u.ensure((size_t)std::max(M, 1) * 4)) != MSP_OK) return s;
        if ((s = h->rnnz.ensure((size_t)std::max(M, 1) * 4)) != MSP_OK) return s;
        if ((s = h->perm.ensure((size_t)std::max(M, 1) * 4)) != MSP_OK) return s;
        if ((s = S.crp.ensure((size_t)(M + 1) * 8)) != MSP_OK) return s;
        if ((s = S.wsym.ensure((kNB + 1) * 2 * 4)) != MSP_OK) return s;
        if ((s = S.wnum.ensure((kNB + 1) * 2 * 4)) != MSP_OK) return s;
        if ((s = S.tick.ensure((kNB + 1) * 4)) != MSP_OK) return s;
        const int tiles = std::max(1, (M + kScanTile - 1) / kScanTile);
        if ((s = h->tiles.ensure((size_t)tiles * 8)) != MSP_OK) return s;
        if ((s = h->bsum.ensure((size_t)std::max((M + 255) / 256, 1) * 8)) != MSP_OK) return s;
    }
    if ((s = zero_info(h)) != MSP_OK) return s;
    // Replays of a stage whose rows all fell in the merge bin at plan time
    // run the statistics and that bin as one kernel, with the scan that
    // needs no look-back behind it; a replay with rows in another bin is
    // caught by k_bin_work like any other change of structure.
    const bool fused = !eager && S.sym_fused && M > 0;
    if (fused) {
        const bool small = narrow_symbolic(S.op);
        const int grid = (M + 255) / 256;
        const long long super_rows = super_tile_rows((M + kWsTile - 1) / kWsTile);
#define MSP_FUSED(KK, IT)                                                                                  \
    k_sym_fused<KK, IT, true><<<grid, 256, 0, st>>>(M, S.op.ncols, S.op.arp, S.op.acol, S.op.brp, S.op.bcol, \
                                                    h->u.as<int32_t>(), h->rnnz.as<int32_t>(), S.sp.table,   \
                                                    S.sp.table.umax[1], info, S.np.table,                    \
                                                    h->bsum.as<long long>(), super_rows, S.mp)
        if (S.sp.spec[1].lanes == 4) { if (small) MSP_FUSED(4, int); else MSP_FUSED(4, long long); }
        else { if (small) MSP_FUSED(8, int); else MSP_FUSED(8, long long); }
#undef MSP_FUSED
        if ((s = launch_ok("k_sym_fused")) != MSP_OK) return s;
    }
    // 1. row statistics and the symbolic bin histogram
    if (M > 0 && !fused) {
        k_row_stats<false, true><<<(M + 255) / 256, 256, 0, st>>>(M, S.op.ncols, S.op.arp, S.op.acol, S.op.brp,
                                                                  S.op.bcol, h->u.as<int32_t>(), nullptr,
                                                                  h->rnnz.as<int32_t>(), S.sp.table, info, nullptr,
                                                                  nullptr, S.mp);
        if ((s = launch_ok("k_row_stats")) != MSP_OK) return s;
    }
    if (eager) {
        if ((s = read_info(h)) != MSP_OK) return s;
        sum_parts(h->hinfo->sym_part, S.sym_rows);
        S.sym_planned = 0;
        S.sym_merge_all = false;
        S.sym_scatter = false;
        for (int bn = 1; bn <= S.sp.table.nb; ++bn) {
            if (S.sym_rows[bn] == 0) continue;
            S.sym_planned |= 1u << bn;
            if (bn == 1 && S.sp.spec[1].kind == Kind::Merge) S.sym_merge_all = true;
            else S.sym_scatter = true;
        }
        S.sym_fused = S.sym_merge_all && !S.sym_scatter &&
                      (S.sp.spec[1].lanes == 4 || S.sp.spec[1].lanes == 8);
    }
    k_bin_work<<<1, 64, 0, st>>>(&info->sym_part[0][0], S.sp.table.nb, S.sym_planned, S.M, nullptr, 0,
                                 S.wsym.as<int>(), flag);
    if ((s = launch_ok("k_bin_work")) != MSP_OK) return s;
    // 2. symbolic pass
    const int* wsym = S.wsym.as<int>();
    if (S.sym_merge_all && !fused)
        if ((s = launch_symbolic_bin<true>(h, S.sp.spec[1], Work{nullptr, M, wsym + 2 * kNB}, M, S.op,
                                           h->rnnz.as<int32_t>(), S.mp, h->u.as<int32_t>(), S.sp.table.umax[1])) !=
            MSP_OK)
            return s;
    if (S.sym_scatter) {
        k_zero_words<<<1, 256, 0, st>>>(&info->cursor[0][0], kParts * kPartStride);
        k_scatter<<<(M + 255) / 256, 256, 0, st>>>(M, h->u.as<int32_t>(), S.sp.table, &info->sym_part[0][0], 256,
                                                   &info->cursor[0][0], h->perm.as<int32_t>());
        if ((s = launch_ok("k_scatter")) != MSP_OK) return s;
        for (int bn = 1; bn <= S.sp.table.nb; ++bn) {
            if (!((S.sym_planned >> bn) & 1u) || (bn == 1 && S.sym_merge_all)) continue;
            if ((s = launch_symbolic_bin<true>(h, S.sp.spec[bn], Work{h->perm.as<int32_t>(), 0, wsym + 2 * bn},
                                               S.sym_rows[bn], S.op, h->rnnz.as<int32_t>(), S.mp, nullptr, 0)) !=
                MSP_OK)
                return s;
        }
    }
    // 3. prefix sum (fresh tile states every replay) with the numeric histogram
    if (fused) {
        k_scan_fused<<<(M + kWsTile - 1) / kWsTile, kWsBS, 0, st>>>(M, h->rnnz.as<int32_t>(),
                                                                   h->bsum.as<long long>(),
                                                                   super_tile_rows((M + kWsTile - 1) / kWsTile),
                                                                   S.crp.as<int64_t>(),
                                                                   S.sp.table.nb, info, nullptr, 0);
        if ((s = launch_ok("k_scan_fused")) != MSP_OK) return s;
    } else {
        const int tiles = std::max(1, (M + kScanTile - 1) / kScanTile);
        k_zero_words<<<(2 * tiles + 255) / 256, 256, 0, st>>>((int*)h->tiles.ptr, 2 * tiles);
        k_scan_lookback<<<tiles, kScanBS, 0, st>>>(M, h->rnnz.as<int32_t>(), h->tiles.as<unsigned long long>(), 1,
                                                   S.crp.as<int64_t>(), S.np.table, info, nullptr, 0);
        if ((s = launch_ok("k_scan_lookback")) != MSP_OK) return s;
    }
    if (eager) {
        if ((s = read_info(h)) != MSP_OK) return s;
        if ((s = device_error(h->hinfo->err)) != MSP_OK) return s;
        S.nnz = h->hinfo->nnz;
        S.cap = S.nnz;
        const size_t vsz = S.op.dtype == MSP_F64 ? 8 : 4;
        S.voff = ((size_t)std::max(S.cap, 1LL) * 4 + 255) & ~(size_t)255;
        if ((s = S.cv.ensure(S.voff + (size_t)std::max(S.cap, 1LL) * vsz)) != MSP_OK) return s;
        sum_parts(h->hinfo->num_part, S.num_rows);
        S.num_planned = 0;
        int nonempty = 0, last = -1;
        for (int bn = 1; bn <= S.np.table.nb; ++bn)
            if (S.num_rows[bn] > 0) {
                S.num_planned |= 1u << bn;
                ++nonempty;
                last = bn;
            }
        // one bin of the kernels that also handle smaller and empty rows:
        // all rows in natural order, no row lists
        S.num_single = -1;
        if (nonempty == 1) {
            const Kind k = S.np.spec[last].kind;
            if (k == Kind::Merge || k == Kind::Batch || k == Kind::Group) S.num_single = last;
        }
    }
    k_bin_work<<<1, 64, 0, st>>>(&info->num_part[0][0], S.np.table.nb, S.num_planned, S.M, &info->nnz, S.cap,
                                 S.wnum.as<int>(), flag);
    if ((s = launch_ok("k_bin_work")) != MSP_OK) return s;
    // 4. numeric pass into the arena; the merge bins' waves draw their rows
    // from a shared work queue (one counter per bin, zeroed by a kernel)
    const int* wnum = S.wnum.as<int>();
    int32_t* ccol = S.cv.as<int32_t>();
    void* cval = (char*)S.cv.ptr + S.voff;
    int* tick = b->queue_rows > 0 ? S.tick.as<int>() : nullptr;
    if (tick) {
        k_zero_words<<<1, 64, 0, st>>>(tick, kNB + 1);
        if ((s = launch_ok("k_zero_words")) != MSP_OK) return s;
    }
    auto queue = [&](int bn) { return tick ? tick + bn : nullptr; };
    if (S.num_single >= 0) {
        if ((s = launch_numeric_bin<true>(h, S.np.spec[S.num_single],
                                          Work{nullptr, M, wnum + 2 * kNB, queue(S.num_single), b->queue_rows}, M,
                                          S.op, S.crp.as<int64_t>(), ccol, cval, nullptr, S.mp)) != MSP_OK)
            return s;
    } else if (S.num_planned) {
        k_zero_words<<<1, 256, 0, st>>>(&info->cursor[0][0], kParts * kPartStride);
        k_scatter<<<(M + 255) / 256, 256, 0, st>>>(M, h->rnnz.as<int32_t>(), S.np.table, &info->num_part[0][0],
                                                   kScanTile, &info->cursor[0][0], h->perm.as<int32_t>());
        if ((s = launch_ok("k_scatter")) != MSP_OK) return s;
        for (int bn = 1; bn <= S.np.table.nb; ++bn) {
            if (!((S.num_planned >> bn) & 1u)) continue;
            if ((s = launch_numeric_bin<true>(h, S.np.spec[bn],
                                              Work{h->perm.as<int32_t>(), 0, wnum + 2 * bn, queue(bn), b->queue_rows},
                                              S.num_rows[bn], S.op, S.crp.as<int64_t>(), ccol, cval, nullptr,
                                              S.mp)) != MSP_OK)
                return s;
        }
    }
    k_fold_err<<<1, 64, 0, st>>>(info, flag);
    return launch_ok("k_fold_err");
}

// the whole replay: both stages and the output row pointers
static msp_status run_all(msp_batch* b, bool eager) {
    msp_handle* h = &b->inner;
    k_zero_words<<<1, 64, 0, h->stream>>>(b->flag.as<int>(), 1);
    msp_status s = launch_ok("k_zero_words");
    for (int i = 0; i < b->nstage && s == MSP_OK; ++i) s = run_stage(b, i, eager);
    if (s != MSP_OK) return s;
    const BatchStage& L = b->st[b->nstage - 1];
    const long long n = std::max(L.M, (long long)b->nprob + 1);
    k_batch_finalize<<<(int)((n + 255) / 256), 256, 0, h->stream>>>(L.M, b->nprob, L.crp.as<int64_t>(), L.mp,
                                                                     b->rp_local.as<int64_t>(), b->bases.as<int64_t>(),
                                                                     b->flag.as<int>());
    return launch_ok("k_batch_finalize");
}

static void release_batch(msp_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (BatchStage& S : b->st)
        for (DevBuf* d : {&S.tile_prob, &S.row_start, &S.boff, &S.ncols, &S.crp, &S.cv, &S.wsym, &S.wnum, &S.tick})
            d->release();
    for (DevBuf* d : {&b->rp_local, &b->bases, &b->flag}) d->release();
    msp_handle* h = &b->inner;
    for (DevBuf* d : {&h->info, &h->u, &h->rnnz, &h->perm, &h->tiles, &h->sbm, &h->prod,
                      &h->bsum, &h->gsl})
        d->release();
    if (h->hinfo) (void)hipHostFree(h->hinfo);
    if (h->hpending) (void)hipHostFree(h->hpending);
    if (b->hbases) (void)hipHostFree(b->hbases);
    if (b->hflag) (void)hipHostFree(b->hflag);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    delete b;
}

static msp_status flag_status(int f) {
    if (!f) return MSP_OK;
    if (f & kErrPlan)
        return fail(MSP_ERR_INVALID_ARG, "batch replay: the inputs' structure changed (a row needs a bin kernel the "
                                         "plan lacks); make a new plan");
    if (f & kErrCapacity)
        return fail(MSP_ERR_INVALID_ARG, "batch replay: the inputs' structure changed (the output outgrew the plan's "
                                         "arena); make a new plan");
    return device_error(f);
}

}  // namespace msp

extern "C" msp_status msp_batch_create(msp_handle* h, const msp_batch_csr* R, const msp_batch_csr* A,
                                       const msp_batch_csr* P, const msp_opts* opts, msp_batch** out) {
    if (!h || !out) return fail(MSP_ERR_INVALID_ARG, "null handle or output");
    *out = nullptr;
    msp_status s;
    if ((s = check_batch_csr(A, "A")) != MSP_OK || (s = check_batch_csr(P, "P")) != MSP_OK) return s;
    if ((s = check_batch_pair(A, P, "A", "P")) != MSP_OK) return s;
    if (R) {
        if ((s = check_batch_csr(R, "R")) != MSP_OK) return s;
        // R_p's columns are the rows of A_p P_p, i.e. A_p's rows
        if ((s = check_batch_pair(R, A, "R", "A")) != MSP_OK) return s;
    }
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (opts && opts->validate) return fail(MSP_ERR_INVALID_ARG, "validate is not supported for batches");
    if (opts && opts->force_spill) return fail(MSP_ERR_INVALID_ARG, "force_spill is not supported for batches");
    const int qr = opts ? opts->queue_rows : 0;
    if (qr != 0 && qr != -1 && (qr < 64 || qr > 65536 || qr % 64 != 0))
        return fail(MSP_ERR_INVALID_ARG, "queue_rows must be 0, -1 or a multiple of 64 in 64..65536");
    msp_batch* b = new (std::nothrow) msp_batch();
    if (!b) return fail(MSP_ERR_OOM, "host allocation failed");
    b->device = h->device;
    b->dtype = A->dtype;
    b->nprob = A->nprob;
    b->nstage = R ? 2 : 1;
    b->queue_rows = qr == 0 ? 1024 : (qr < 0 ? 0 : qr);
    msp_handle* in = &b->inner;
    in->device = h->device;
    in->alloc = h->alloc;
    in->free_fn = h->free_fn;
    in->alloc_ctx = h->alloc_ctx;
    in->num_cu = h->num_cu;
    in->lds_per_block = h->lds_per_block;
    in->tuning = effective_tuning(h, opts);
    auto bail = [&](msp_status r) { release_batch(b); return r; };
    // private stream (default priority): the eager run and the capture
    if ((e = hipStreamCreateWithFlags(&in->stream, hipStreamNonBlocking)) != hipSuccess)
        return bail(hip_fail(e, "hipStreamCreate"));
    if ((e = hipHostMalloc((void**)&in->hinfo, sizeof(DevInfo), hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&in->hpending, sizeof(int), hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&b->hflag, sizeof(int), hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&b->hbases, (size_t)(b->nprob + 1) * 8, hipHostMallocDefault)) != hipSuccess)
        return bail(hip_fail(e, "hipHostMalloc"));
    *in->hpending = 0;
    *b->hflag = 0;
    if ((s = in->info.ensure(sizeof(DevInfo))) != MSP_OK || (s = b->flag.ensure(sizeof(int))) != MSP_OK) return bail(s);
    // inputs must be ready before the private stream reads them
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return bail(hip_fail(e, "hipStreamSynchronize"));
    const msp_tuning t = in->tuning;
    const size_t vsz = A->dtype == MSP_F64 ? 8 : 4;
    (void)vsz;
    long long maxc = 0;
    for (int p = 0; p < b->nprob; ++p) maxc = std::max<long long>(maxc, P->ncols[p]);
    // stage 0: A_p P_p
    BatchStage& S0 = b->st[0];
    S0.op = Operands{A->row_ptr, A->col, A->val, P->row_ptr, P->col, P->val, maxc, P->nnz, A->row_start[A->nprob],
                     A->dtype, A->nnz, P->row_start[P->nprob]};
    if ((s = build_map(S0, b->nprob, A->row_start, P->row_start, P->ncols, in->stream)) != MSP_OK) return bail(s);
    S0.sp = symbolic_plan(t, false);
    S0.np = numeric_plan(t, false);
    const int64_t* out_rows = A->row_start;
    if (R) {
        BatchStage& S1 = b->st[1];
        S1.sp = symbolic_plan(t, false);
        S1.np = numeric_plan(t, false);
        if ((s = build_map(S1, b->nprob, R->row_start, A->row_start, P->ncols, in->stream)) != MSP_OK) return bail(s);
        out_rows = R->row_start;
    }
    b->row_start.assign(out_rows, out_rows + b->nprob + 1);
    b->ncols.assign(P->ncols, P->ncols + b->nprob);
    const long long Mout = out_rows[b->nprob];
    if ((s = b->rp_local.ensure((size_t)(Mout + b->nprob) * 8)) != MSP_OK ||
        (s = b->bases.ensure((size_t)(b->nprob + 1) * 8)) != MSP_OK)
        return bail(s);
    // eager run: sizes and bins (the second stage's operands point into the
    // first stage's arena, known once the first stage has been sized)
    if ((e = hipMemsetAsync(b->flag.ptr, 0, sizeof(int), in->stream)) != hipSuccess)
        return bail(hip_fail(e, "hipMemsetAsync"));
    if ((s = run_stage(b, 0, true)) != MSP_OK) return bail(s);
    if (R) {
        BatchStage& S1 = b->st[1];
        S1.op = Operands{R->row_ptr, R->col, R->val, S0.crp.as<int64_t>(), S0.cv.as<int32_t>(),
                         (char*)S0.cv.ptr + S0.voff, maxc, S0.cap, R->row_start[R->nprob], A->dtype, R->nnz,
                         A->row_start[A->nprob]};
        if ((s = run_stage(b, 1, true)) != MSP_OK) return bail(s);
    }
    if ((e = hipStreamSynchronize(in->stream)) != hipSuccess) return bail(hip_fail(e, "hipStreamSynchronize"));
    // capture the whole replay
    if ((e = hipStreamBeginCapture(in->stream, hipStreamCaptureModeRelaxed)) != hipSuccess)
        return bail(hip_fail(e, "hipStreamBeginCapture"));
    g_capturing = true;
    s = run_all(b, false);
    g_capturing = false;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(in->stream, &g);
    b->graph = g;
    if (s != MSP_OK) return bail(s);
    if (e != hipSuccess) return bail(hip_fail(e, "hipStreamEndCapture"));
    if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess)
        return bail(hip_fail(e, "hipGraphInstantiate"));
    *out = b;
    return MSP_OK;
}

extern "C" msp_status msp_batch_destroy(msp_batch* b) {
    release_batch(b);
    return MSP_OK;
}

extern "C" msp_status msp_batch_execute(msp_handle* h, msp_batch* b) {
    if (!h || !b) return fail(MSP_ERR_INVALID_ARG, "null handle or plan");
    if (h->device != b->device) return fail(MSP_ERR_INVALID_ARG, "the plan belongs to another device");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (b->pending) {     // collect the previous replay's flag first
        msp_status s = msp_batch_sync(h, b);
        if (s != MSP_OK) return s;
    }
    if ((e = hipGraphLaunch(b->exec, h->stream)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    if ((e = hipMemcpyAsync(b->hflag, b->flag.ptr, sizeof(int), hipMemcpyDeviceToHost, h->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(b->hbases, b->bases.ptr, (size_t)(b->nprob + 1) * 8, hipMemcpyDeviceToHost, h->stream)) !=
            hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(batch results)");
    b->pending = true;
    b->have_result = false;
    return MSP_OK;
}

extern "C" msp_status msp_batch_sync(msp_handle* h, msp_batch* b) {
    if (!h || !b) return fail(MSP_ERR_INVALID_ARG, "null handle or plan");
    if (!b->pending) return MSP_OK;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    b->pending = false;
    const int f = *b->hflag;
    b->have_result = f == 0;
    return flag_status(f);
}

extern "C" msp_status msp_batch_result(msp_handle* h, msp_batch* b, int p, msp_csr* C) {
    if (!h || !b || !C) return fail(MSP_ERR_INVALID_ARG, "null argument");
    if (p < 0 || p >= b->nprob) return fail(MSP_ERR_INVALID_ARG, "problem %d outside [0, %d)", p, b->nprob);
    msp_status s = msp_batch_sync(h, b);
    if (s != MSP_OK) return s;
    if (!b->have_result) return fail(MSP_ERR_INVALID_ARG, "the plan has no completed replay");
    const BatchStage& L = b->st[b->nstage - 1];
    C->nrows = b->row_start[p + 1] - b->row_start[p];
    C->ncols = b->ncols[p];
    C->nnz = b->hbases[p + 1] - b->hbases[p];
    C->row_ptr = b->rp_local.as<int64_t>() + b->row_start[p] + p;
    C->col = L.cv.as<int32_t>() + b->hbases[p];
    C->val = (const char*)L.cv.ptr + L.voff + (size_t)b->hbases[p] * (b->dtype == MSP_F64 ? 8 : 4);
    C->dtype = b->dtype;
    return MSP_OK;
}

extern "C" msp_status msp_batch_copy_result(msp_handle* h, msp_batch* b, int p, msp_csr_out* C) {
    if (!C) return fail(MSP_ERR_INVALID_ARG, "C is NULL");
    msp_csr v;
    msp_status s = msp_batch_result(h, b, p, &v);
    if (s != MSP_OK) return s;
    bool own_rp = false;
    if (!C->row_ptr) {
        C->row_ptr = (int64_t*)h->alloc(h->alloc_ctx, (size_t)(v.nrows + 1) * 8, h->stream);
        if (!C->row_ptr) return fail(MSP_ERR_OOM, "allocation of C.row_ptr failed");
        own_rp = true;
    }
    C->nrows = v.nrows;
    C->ncols = v.ncols;
    C->nnz = v.nnz;
    C->dtype = v.dtype;
    C->col = nullptr;
    C->val = nullptr;
    const size_t vsz = v.dtype == MSP_F64 ? 8 : 4;
    hipError_t e = hipMemcpyAsync(C->row_ptr, v.row_ptr, (size_t)(v.nrows + 1) * 8, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess && v.nnz > 0) {
        const size_t voff = ((size_t)v.nnz * 4 + 255) & ~(size_t)255;
        void* base = h->alloc(h->alloc_ctx, voff + (size_t)v.nnz * vsz, h->stream);
        if (!base) {
            if (own_rp) { h->free_fn(h->alloc_ctx, C->row_ptr, h->stream); C->row_ptr = nullptr; }
            return fail(MSP_ERR_OOM, "allocation of C (%lld nonzeros) failed", (long long)v.nnz);
        }
        C->col = (int32_t*)base;
        C->val = (char*)base + voff;
        e = hipMemcpyAsync(C->col, v.col, (size_t)v.nnz * 4, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(C->val, v.val, (size_t)v.nnz * vsz, hipMemcpyDeviceToDevice, h->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(batch result)");
    return MSP_OK;
}

extern "C" msp_status msp_batch_info(const msp_batch* b, msp_batch_stats* st) {
    if (!b || !st) return fail(MSP_ERR_INVALID_ARG, "null argument");
    memset(st, 0, sizeof(*st));
    st->nstage = b->nstage;
    for (int i = 0; i < b->nstage; ++i) {
        const BatchStage& S = b->st[i];
        st->rows[i] = S.M;
        st->nnz[i] = S.nnz;
        for (int bn = 1; bn <= S.sp.table.nb; ++bn) st->sym_bins[i] += (S.sym_planned >> bn) & 1u;
        for (int bn = 1; bn <= S.np.table.nb; ++bn) st->num_bins[i] += (S.num_planned >> bn) & 1u;
    }
    return MSP_OK;
}

// ---------------------------------------------------------------------------
// autotuner: median replay time of each candidate tuning
// ---------------------------------------------------------------------------
extern "C" msp_status msp_batch_autotune(msp_handle* h, const msp_batch_csr* R, const msp_batch_csr* A,
                                         const msp_batch_csr* P, const msp_tuning* cand, int ncand, int reps,
                                         msp_tuning* best, double* times_ms) {
    if (!h || !cand || ncand <= 0 || reps <= 0 || !best) return fail(MSP_ERR_INVALID_ARG, "bad argument");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return hip_fail(e, "hipEventCreate"); }
    double best_ms = INFINITY;
    int best_i = -1;
    msp_status last_err = MSP_OK;
    for (int c = 0; c < ncand; ++c) {
        double med = INFINITY;
        msp_tuning t = cand[c];
        msp_opts o;
        memset(&o, 0, sizeof(o));
        o.tuning = t;
        msp_batch* b = nullptr;
        msp_status s = check_tuning(&o.tuning);
        if (s == MSP_OK) s = msp_batch_create(h, R, A, P, &o, &b);
        if (s == MSP_OK) s = msp_batch_execute(h, b);
        if (s == MSP_OK) s = msp_batch_sync(h, b);          // warm
        std::vector<double> ts;
        for (int r = 0; r < reps && s == MSP_OK; ++r) {
            if ((e = hipEventRecord(e0, h->stream)) != hipSuccess) { s = hip_fail(e, "hipEventRecord"); break; }
            if ((s = msp_batch_execute(h, b)) != MSP_OK) break;
            if ((e = hipEventRecord(e1, h->stream)) != hipSuccess) { s = hip_fail(e, "hipEventRecord"); break; }
            if ((s = msp_batch_sync(h, b)) != MSP_OK) break;
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { s = hip_fail(e, "hipEventElapsedTime"); break; }
            ts.push_back(ms);
        }
        if (s == MSP_OK && !ts.empty()) {
            std::sort(ts.begin(), ts.end());
            med = ts[ts.size() / 2];
        } else {
            last_err = s;
        }
        if (b) msp_batch_destroy(b);
        if (s == MSP_ERR_HIP) {       // the device reported an error: try nothing more on it
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
    msp_status s = check_tuning(best);
    return s;
}

// ---------------------------------------------------------------------------
// tuning <-> JSON (a flat object of the integer fields; share_g may be
// absent, meaning the default)
// ---------------------------------------------------------------------------
extern "C" int msp_tuning_to_json(const msp_tuning* t, char* buf, size_t n) {
    if (!t) return -1;
    return snprintf(buf, buf ? n : 0,
                    "{\"hash_scale\": %d, \"group_scale\": %d, \"spill_nnz\": %d, \"block_rows\": %d, \"merge_k\": %d, "
                    "\"share_g\": %d}",
                    t->hash_scale, t->group_scale, t->spill_nnz, t->block_rows, t->merge_k, t->share_g);
}

static bool json_int(const char* js, const char* key, int* out) {
    const std::string k = std::string("\"") + key + "\"";
    const char* p = strstr(js, k.c_str());
    if (!p) return false;
    p += k.size();
    while (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r') ++p;
    if (*p != ':') return false;
    ++p;
    char* end = nullptr;
    const long v = strtol(p, &end, 10);
    if (end == p || v < INT32_MIN || v > INT32_MAX) return false;
    *out = (int)v;
    return true;
}

extern "C" msp_status msp_tuning_from_json(const char* js, msp_tuning* t) {
    if (!js || !t) return fail(MSP_ERR_INVALID_ARG, "null argument");
    msp_tuning x;
    if (!json_int(js, "hash_scale", &x.hash_scale) || !json_int(js, "group_scale", &x.group_scale) ||
        !json_int(js, "spill_nnz", &x.spill_nnz) || !json_int(js, "block_rows", &x.block_rows) ||
        !json_int(js, "merge_k", &x.merge_k))
        return fail(MSP_ERR_INVALID_ARG, "tuning JSON lacks one of its five integer fields");
    if (!json_int(js, "share_g", &x.share_g)) x.share_g = 0;
    msp_status s = check_tuning(&x);
    if (s != MSP_OK) return s;
    *t = x;
    return MSP_OK;
}
