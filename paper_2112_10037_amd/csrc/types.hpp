// Types and constants shared by the device kernels and the host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msp {

constexpr int kWave = 64;
// Most rows of one matrix (or of a whole batch): grid sizes are rounded up
// from the row count in int arithmetic, with at most 8192 added.
constexpr long long kMaxRows = 2147483647LL - 8192;
constexpr int kMaxBins = 16;
constexpr int32_t kEmpty = -1;

// error bits reported in DevInfo::err
constexpr int kErrProbe = 1;      // a hash probe sequence exceeded the table (bug guard)
constexpr int kErrUnsorted = 2;   // input columns not strictly increasing
constexpr int kErrRange = 4;      // input index out of range / row_ptr not monotone
constexpr int kErrCount = 8;      // numeric count disagrees with the symbolic count
constexpr int kErrPlan = 16;      // batch replay: a row fell in a bin the plan has no kernel for
constexpr int kErrCapacity = 32;  // batch replay: the output outgrew the plan's arena
constexpr int kErrScan = 64;      // prefix sum: a look-back wait passed its bound, or tile tickets were stale

// Predictor features 0..5 are log2(1 + x) scaled by this factor so that
// every network input is of order one.
constexpr float kFeatLogScale = 1.0f / 16.0f;

// Global bin counters are split over kParts partitions (workgroup w counts
// into partition w % kParts), each padded to its own 128-byte line, so that
// thousands of workgroups do not serialise on one address.
constexpr int kParts = 32;
constexpr int kNB = kMaxBins + 1;
constexpr int kSideStreams = 3;    // streams beside the handle's that run a phase's bins concurrently
constexpr int kPartStride = 32;    // ints per partition row (128 bytes)
// On long inputs the fused symbolic pass also adds each workgroup's
// row-count total into one of at most kSupers super-tile sums, so that a
// scan tile finds the total before it in a bounded number of reads.
constexpr int kSupers = 1024;

constexpr long long kOmarMaxGroup = 4096;   // largest row group of the sharing count

// Row statistics of rows with more than kLongRow A entries are taken apart:
// chunks of kLongChunk entries go to whole workgroups, which add into the
// row's LongAcc with global atomics.  A wave walks 64 consecutive rows, and
// a skewed matrix's longest rows sit together (R-MAT's at the lowest
// indices): with long rows up to 4096 entries left in the walk, one wave of
// a 2^18-row R-MAT had 62 times the mean walk and set the kernel's time.
constexpr int kLongRow = 256;
constexpr int kLongChunk = 2048;
struct LongAcc {
    unsigned long long prod;              // sum of the B-row lengths
    int mn, mx;                           // shortest and longest B row
    int lo, hi;                           // smallest first and largest last column
};
struct LongRows {                         // work lists of the long rows (list == nullptr: not taken apart)
    int* list = nullptr;                  // row of each long row
    int* base = nullptr;                  // its first chunk
    int* chunk_row = nullptr;             // long row (index into list) of each chunk
    LongAcc* acc = nullptr;               // statistics of each long row
    int list_cap = 0, chunk_cap = 0;
};

struct DevInfo {
    long long nnz;                        // nnz(C) after the scan
    int err;                              // error bits of the current call
    int scan_ticket;                      // tile tickets of the single-pass scan
    int neg_count;                        // scan inputs < 0 (rows that overflowed)
    int fused_other;                      // the fused symbolic pass left rows for other bins
    int win_nrec;                         // window records the symbolic pass made
    int win_fb[2];                        // global-bin rows without a record: {count, 0}
    int win_nbs;                          // B rows given a window index
    int win_nbms;                         // rows whose bitmap the symbolic pass stored
    int learned_big;                      // learned product: rows sent to the exact path by capacity
    long long share_batches;              // merge batches that read B from a shared LDS stage
    long long share_nnz;                  // A entries of those batches' merge rows
    long long share_rows;                 // distinct B rows those batches staged
    unsigned long long omar_distinct;     // distinct (row group, column) pairs of A (Eq. 1)
    unsigned long long learned_big_hi;    // learned product: upper bounds of the rows sent to the exact path
    int long_n;                           // row statistics: rows taken apart as long rows
    int long_chunks;                      // and their chunks
    // row queues of the persistent one-row-per-workgroup kernels, per phase
    // (symbolic, numeric) and bin, plus [1][kNB] for the global bin's rows
    // without a window record: {slots handed out, workgroups done}, zero
    // between launches
    unsigned queue[2][kNB + 1][2];
    int sym_part[kParts][kPartStride];    // rows per symbolic bin, per partition
    int num_part[kParts][kPartStride];    // rows per numeric bin, per partition
    int cursor[kParts][kPartStride];      // scatter cursors
    long long ssum[kSupers];              // rows' counts per super-tile of the fused symbolic pass
};

// What the host needs between passes, written by a one-workgroup kernel
// straight into pinned host memory (no copy, no stream wait); seq is
// written last and tells the host that the rest is complete.
struct HostSummary {
    long long nnz;
    int err;
    int neg_count;
    int counts[kNB];                      // rows per bin, summed over partitions
    int merge_na;                         // most A entries of a row the fused pass merged
    int seq;
};

// Spare slot of each symbolic partition row: the largest A-row length among
// the rows the fused statistics and merge pass counted with the merge.
constexpr int kPartMergeNA = kPartStride - 1;
static_assert(kNB < kPartMergeNA, "partition rows hold the bins and one spare slot");

// Column windows of the global bin.  The symbolic pass records, for every
// row with more outputs than the numeric threshold, how many of its outputs
// fall in each window of kWin columns; B rows with at least kWinMinLen
// entries get the position of their first entry at or past every window
// boundary.  The numeric pass then cuts such rows into slices of whole
// windows sized from the exact counts, and finds each slice's part of a B
// row with two loads instead of a search.
constexpr int kWinLog = 12;
constexpr int kWin = 1 << kWinLog;               // columns per window
constexpr int kWinWords = kWin / 64;             // 64-bit bitmap words per window
constexpr int kWinFixed = kWinWords * (8 + 2);   // LDS bytes per window: bitmap and 16-bit word ranks
constexpr int kWinOut = 8 + 4;                   // LDS bytes per output: FP64 sum and column
constexpr int kWinMaxNw = 512;                   // most windows per row (ncols <= 2^21)
constexpr int kWinMinLen = 16;                   // shortest B row given a window index

struct WinRec {
    int32_t* islot;      // per row of A: index of its record (stale values are caught by `row`)
    int32_t* row;        // per record: its row of A
    uint16_t* cnt;       // per record: outputs in each of the nw windows
    int* nrec;           // records made so far (counter in the device info block)
    int cap;             // records that fit
    int nw;              // windows per row; cnt == nullptr: no records are made
    int thresh;          // rows with more outputs than this get a record
    // bitmap store: a recorded row of the bitmap kernel with at least
    // bms_min_prod products also leaves its column bitmap (nw * kWin bits),
    // so that the numeric pass need not rebuild it
    int32_t* rec_bm;     // per record: its bitmap slot, or -1
    uint32_t* bms;       // bitmap slots (nullptr: no store)
    int* nbms;           // slots taken (counter in the device info block)
    int bms_cap;         // slots that fit
    long long bms_min_prod;
};

// Bin b (1 <= b < nb) holds rows with umax[b-1] < u <= umax[b]; bin 0 holds
// u == 0; bin nb holds everything above umax[nb-1] (the global path).
struct BinTable {
    int nb;
    int umax[kMaxBins];
};

// The rows one bin kernel processes: perm[0..n) (perm null: rows 0..n-1).
// Kernels queued before the bin sizes reach the host (captured batch graphs)
// read n and perm's offset from device memory instead: dev[0], dev[1].
struct Work {
    const int32_t* perm;
    int n;
    const int* dev;
    int* ticket;        // shared work queue of the launch (zero at launch), or null
    int tk;             // rows per ticket
    unsigned* rowq = nullptr;   // row queue of a one-row-per-workgroup kernel (see block_first)
};

__device__ __forceinline__ void work_rows(const Work& w, int* n, const int32_t** perm) {
    if (w.dev) {
        *n = w.dev[0];
        *perm = w.perm ? w.perm + w.dev[1] : nullptr;
    } else {
        *n = w.n;
        *perm = w.perm;
    }
}

// Batched inputs in packed form.  Problem p owns the global rows
// [row_start[p], row_start[p+1]) of the packed A (one row_ptr array with
// global offsets into one col/val array).  Its column indices are local:
// column k of problem p is row boff[p] + k of the packed B, and its output
// columns are B's local columns (< ncols[p]).  tile_prob[t] is the problem
// of global row 64 t.
struct RowMap {
    const int32_t* tile_prob;
    const int64_t* row_start;
    const int64_t* boff;
    const int64_t* ncols;
};

__device__ __forceinline__ int map_prob(const RowMap& mp, long long g) {
    int p = mp.tile_prob[g >> 6];
    while (g >= mp.row_start[p + 1]) ++p;      // skip problems that end inside the tile
    return p;
}

// offset of the B rows of global row g's problem (0 when not batched)
template <bool BATCH>
__device__ __forceinline__ long long row_boff(const RowMap& mp, long long g) {
    if constexpr (BATCH) return mp.boff[map_prob(mp, g)];
    else return 0;
}

__device__ __forceinline__ int bin_of(const BinTable& t, long long u) {
    if (u <= 0) return 0;
    for (int b = 1; b < t.nb; ++b)
        if (u <= t.umax[b]) return b;
    return t.nb;
}

}  // namespace msp
