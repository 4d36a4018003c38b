// Internal host-side declarations shared by the translation units of the
// library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <vector>

#include "msp.h"
#include "types.hpp"

namespace msp {

// A fixed block of device memory that workspaces are carved from in order
// (the allocation-free entry point's scratch); nothing is returned to it
// before the call ends.
struct Arena {
    char* base = nullptr;
    size_t size = 0, used = 0;
};

struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    Arena* arena = nullptr;         // set: ensure() takes memory from the arena, release() frees nothing
    msp_status ensure(size_t need);
    void release();
    template <typename T> T* as() const { return (T*)ptr; }
};

// One accumulator class of a bin: the kernel family and its shape.
enum class Kind { None, Merge, Batch, Group, Block, Bitmap, Dense };

struct BinSpec {
    Kind kind = Kind::None;
    int lanes = 0;      // K lists for Merge, rows per batch R for Batch, G for Group,
                        // BS for Block/Bitmap/Dense
    int slots = 0;      // T (hash slots) for Group/Block
    int share = 0;      // Merge, numeric: rows per batch that share staged B rows (0: off)
};

struct BinPlan {
    BinTable table;                 // thresholds, consumed by the kernels
    BinSpec spec[kMaxBins + 1];     // spec[b] for b in 1..nb (nb = the global path)
};

// Operand pointers of one product, or of a packed batch of products (then
// ncols is the widest problem's and the RowMap of the launch gives each
// row's problem).
struct Operands {
    const int64_t* arp;
    const int32_t* acol;
    const void* aval;
    const int64_t* brp;
    const int32_t* bcol;
    const void* bval;
    long long ncols;       // columns of B
    long long bnnz;        // entries of B (length of its col and val arrays)
    long long m;           // rows of A
    msp_dtype dtype;
    long long annz;        // entries of A (length of its col and val arrays)
    long long brows;       // rows of B
};

// The fused symbolic kernel may gather with 32-bit byte offsets when they
// fit: 4-byte columns of A and B under 2^30 entries, 8-byte row pointers of
// B under 2^29.
inline bool narrow_symbolic(const Operands& op) {
    return op.annz < (1LL << 30) && op.bnnz < (1LL << 30) && op.brows + 1 < (1LL << 29);
}

struct ExtraState;                  // learned / batched state (other units)

// Per-phase event timing: intervals are recorded on the handle's stream and
// folded into the accumulators once they have completed.
struct Profiler {
    bool on = false;
    unsigned mask = ~0u;     // phases timed (bit p: phase p)
    double ms[MSP_NUM_PHASES] = {};
    int64_t count[MSP_NUM_PHASES] = {};
    struct Pending { int phase; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    int open_phase = -1;
    hipEvent_t open_ev = nullptr;
    hipEvent_t get();
    void begin(int phase, hipStream_t s);
    void end(hipStream_t s);
    // an interval inside the open phase (one kernel), timed the same way
    hipEvent_t sub_begin(int phase, hipStream_t s);
    void sub_end(int phase, hipEvent_t a, hipStream_t s);
    void collect();          // fold completed intervals (after a sync)
    void reset();
    void release();
};

}  // namespace msp

struct msp_handle {
    int device = 0;
    hipStream_t stream = nullptr;
    // side streams for the bins of a phase (default priority), and the
    // events that fork them from `stream` and join them back
    hipStream_t side[msp::kSideStreams] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[msp::kSideStreams] = {};
    msp_alloc_fn alloc = nullptr;
    msp_free_fn free_fn = nullptr;
    void* alloc_ctx = nullptr;
    int num_cu = 256;
    int lds_per_block = 65536;
    msp_tuning tuning{};
    msp::DevBuf info, u, rnnz, perm, tiles, sbm, prod;
    msp::DevBuf bsum;               // 256-row workgroup totals of the fused symbolic pass
    msp::DevBuf gsl;                // per-workgroup bitmap copies of the sliced global-bin kernel
    // column windows of the global bin (plain product): the symbolic pass's
    // per-window row counts, B's window index, and the rows left to the
    // self-counting kernel
    msp::DevBuf win_islot, win_row, win_cnt, win_bslot, win_wpos, win_fb, win_rbm, win_bms;
    // row statistics: the rows with more than kLongRow A entries and their chunks
    msp::DevBuf lr_list, lr_base, lr_chunk, lr_acc;
    size_t total_mem = 0;           // device memory (bounds the bitmap store)
    void* scratch = nullptr;        // device address of this device's no-allocation scratch
    msp::WinRec cur_rec{};          // records of the product in progress (cnt null: none)
    msp::DevInfo* hinfo = nullptr;  // pinned mirror of info
    int* hpending = nullptr;        // pinned: error bits of the last call's numeric
                                    // kernels, forwarded by the next call's first kernel
    int* dpending = nullptr;        // device address of hpending (null: not forwarded)
    msp::HostSummary* hsum = nullptr;   // pinned, coherent: summaries the kernels publish
    msp::HostSummary* dsum = nullptr;   // its device address
    int sum_seq = 0;                // sequence number of the last summary requested
    long long summary_fallbacks = 0;    // summaries taken from a device copy instead
    int scan_epoch = 0;             // epoch of the single-pass scan's tile states
    msp::ExtraState* extra = nullptr;
    msp::Profiler prof;
};

namespace msp {

// Set while a batch plan's launches are being captured into a graph: any
// workspace growth or memset then is an internal error instead of a
// silently recorded graph node.
extern thread_local bool g_capturing;
// Set during the allocation-free product: a workspace that was not moved
// into the scratch array and would grow is then an internal error instead
// of a hidden hipMalloc.
extern thread_local bool g_noalloc;

msp_status fail(msp_status s, const char* fmt, ...);
msp_status hip_fail(hipError_t e, const char* what);
msp_status check_csr(const msp_csr* M, const char* name);
msp_tuning default_tuning();
msp_status check_tuning(msp_tuning* t);
msp_tuning effective_tuning(const msp_handle* h, const msp_opts* o);
msp_status configure_kernels(msp_handle* h);
void release_extra(msp_handle* h);

int count_unsupported_plans(int verbose);
void sum_parts(const int (*part)[kPartStride], int out[kNB]);
BinPlan symbolic_plan(const msp_tuning& t, bool force_spill);
BinPlan numeric_plan(const msp_tuning& t, bool force_spill);

// The plain pipeline pieces, reused by the learned and batched forms.
msp_status read_info(msp_handle* h);
msp_status zero_info(msp_handle* h);
// Wait until the kernel given sequence number `seq` has published its host
// summary (spinning on pinned memory, checking the stream for errors).
// With spec_nb > 0 the summary is a speculative scan's: when it was skipped
// (nnz = -1) its counts are the symbolic bin sizes.
msp_status wait_summary(msp_handle* h, int seq, bool with_nnz, const int (*part)[kPartStride], int spec_nb = 0);
msp_status run_row_stats(msp_handle* h, const msp_csr* A, const msp_csr* B, const BinPlan& plan,
                         int64_t* prod_out, float* feat, int32_t* lo_out, int publish_seq = 0);
msp_status run_symbolic_bins(msp_handle* h, const msp_csr* A, const msp_csr* B, const BinPlan& plan,
                             const int* counts_host, int32_t* row_nnz, int done_bin);
msp_status run_scan(msp_handle* h, int m, const int32_t* row_nnz, int64_t* row_ptr, const BinPlan* plan,
                    int publish_seq = 0);
msp_status take_pending_error(msp_handle* h);
msp_status check_pair(const msp_csr* A, const msp_csr* B);
msp_status validate_inputs(msp_handle* h, const msp_csr* A, const msp_csr* B);
msp_status device_error(int err);
// Caller-provided C buffers (col and val of `cap` entries each).
struct CPlace {
    int32_t* col;
    void* val;
    long long cap;
};
msp_status spgemm_core(msp_handle* h, const msp_csr* A, const msp_csr* B, msp_csr_out* C, const msp_opts* opts,
                       const std::function<void*(size_t)>& alloc_cv, const std::function<void(void*)>& free_cv,
                       const CPlace* place = nullptr);
msp_status run_numeric_bins(msp_handle* h, const msp_csr* A, const msp_csr* B, const BinPlan& plan,
                            const int* counts_host, const int32_t* key, const int64_t* crp,
                            int32_t* ccol, void* cval, int32_t* cnt_out);

// One bin's kernel over the rows of wk (BATCH: packed operands, rows mapped
// to problems by mp); `rows` sizes the persistent grid.
Operands operands_of(const msp_csr* A, const msp_csr* B);
template <bool BATCH>
msp_status launch_symbolic_bin(msp_handle* h, const BinSpec& s, Work wk, int rows, const Operands& op,
                               int32_t* rnnz, const RowMap& mp, const int32_t* ufilter, int umax);
template <bool BATCH>
msp_status launch_numeric_bin(msp_handle* h, const BinSpec& s, Work wk, int rows, const Operands& op,
                              const int64_t* crp, int32_t* ccol, void* cval, int32_t* cnt_out, const RowMap& mp);

}  // namespace msp
