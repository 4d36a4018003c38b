// Host side of the C ABI declared in include/msp.h: handle, workspace,
// bin tables and the dispatch of the per-bin kernels of kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "msp.h"
#include "internal.hpp"

using namespace msp;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
namespace msp {
thread_local char g_last_error[512] = "";

msp_status fail(msp_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return s;
}

msp_status hip_fail(hipError_t e, const char* what) {
    return fail(MSP_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}
}  // namespace msp

extern "C" const char* msp_last_error(void) { return g_last_error; }

extern "C" const char* msp_status_string(msp_status s) {
    switch (s) {
        case MSP_OK: return "ok";
        case MSP_ERR_INVALID_ARG: return "invalid argument";
        case MSP_ERR_SHAPE: return "shape mismatch";
        case MSP_ERR_DTYPE: return "value type mismatch";
        case MSP_ERR_UNSORTED_OR_DUP: return "input columns not strictly increasing";
        case MSP_ERR_OOM: return "out of memory";
        case MSP_ERR_HIP: return "HIP runtime error";
        case MSP_ERR_INDEX_OVERFLOW: return "size exceeds index types";
        case MSP_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

extern "C" int msp_version(void) { return 1; }

// ---------------------------------------------------------------------------
// handle and workspace
// ---------------------------------------------------------------------------
namespace msp {

thread_local bool g_capturing = false;
thread_local bool g_noalloc = false;

msp_status DevBuf::ensure(size_t need) {
    if (need <= bytes) return MSP_OK;
    if (arena) {
        const size_t at = (arena->used + 255) & ~(size_t)255;
        const size_t want = std::max(need, (size_t)256);
        if (at > arena->size || arena->size - at < want)
            return fail(MSP_ERR_OOM,
                        "the no-allocation scratch (%zu bytes) cannot hold this product's workspace "
                        "(%zu bytes in use, %zu more needed)", arena->size, at, want);
        ptr = arena->base + at;
        bytes = want;
        arena->used = at + want;
        return MSP_OK;
    }
    if (g_capturing) return fail(MSP_ERR_HIP, "internal: workspace growth during graph capture");
    if (g_noalloc) return fail(MSP_ERR_HIP, "internal: workspace growth in the allocation-free product");
    if (ptr) {
        hipError_t e = hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
        if (e != hipSuccess) return hip_fail(e, "hipFree(workspace)");
    }
    size_t want = std::max(need, (size_t)256);
    hipError_t e = hipMalloc(&ptr, want);
    if (e != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        return fail(MSP_ERR_OOM, "workspace allocation of %zu bytes failed", want);
    }
    bytes = want;
    return MSP_OK;
}

void DevBuf::release() {
    if (ptr && !arena) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

}  // namespace msp

// The allocation-free entry point's workspace: one fixed array per device,
// held until the process ends and shared by every handle on that device.
// Host code uses only the device address hipGetSymbolAddress gives for it
// (the array's name is a host-side stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[MSP_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mutex;
static void* g_scratch_addr[256] = {};

// Device address of `scratch` on the current device `device` (looked up once).
static msp_status scratch_address(int device, void** out) {
    if (device < 0 || device >= 256) return fail(MSP_ERR_UNSUPPORTED, "device index %d", device);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        }
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return MSP_OK;
}

static void* default_alloc(void*, size_t bytes, void*) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}
static void default_free(void*, void* p, void*) {
    if (p) (void)hipFree(p);
}

// Side streams and fork/join events of a handle (null members are skipped).
static void release_streams(msp_handle* h) {
    for (int i = 0; i < kSideStreams; ++i) {
        if (h->side[i]) (void)hipStreamDestroy(h->side[i]);
        if (h->join_ev[i]) (void)hipEventDestroy(h->join_ev[i]);
        h->side[i] = nullptr;
        h->join_ev[i] = nullptr;
    }
    if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
    h->fork_ev = nullptr;
}

static hipError_t create_streams(msp_handle* h) {
    hipError_t e = hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming);
    for (int i = 0; i < kSideStreams && e == hipSuccess; ++i) {
        if ((e = hipStreamCreateWithFlags(&h->side[i], hipStreamNonBlocking)) == hipSuccess)
            e = hipEventCreateWithFlags(&h->join_ev[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) release_streams(h);
    return e;
}

extern "C" msp_status msp_create(msp_handle** out, int device, void* stream) {
    if (!out) return fail(MSP_ERR_INVALID_ARG, "msp_create: null handle pointer");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(MSP_ERR_INVALID_ARG, "device %d out of range (%d devices)", device, ndev);
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(MSP_ERR_UNSUPPORTED, "device %d is %s; this library is built for gfx950 only", device, prop.gcnArchName);
    void* scr = nullptr;
    msp_status ss = scratch_address(device, &scr);
    if (ss != MSP_OK) return ss;
    msp_handle* h = new (std::nothrow) msp_handle();
    if (!h) return fail(MSP_ERR_OOM, "msp_create: host allocation failed");
    h->scratch = scr;
    h->device = device;
    h->stream = (hipStream_t)stream;
    h->alloc = default_alloc;
    h->free_fn = default_free;
    h->alloc_ctx = nullptr;
    h->num_cu = prop.multiProcessorCount;
    h->lds_per_block = (int)prop.sharedMemPerBlock;
    h->total_mem = prop.totalGlobalMem;
    h->tuning = default_tuning();
    msp_status s = h->info.ensure(sizeof(DevInfo));
    if (s != MSP_OK) { delete h; return s; }
    // the first call forwards the error bits it finds here: start from zero,
    // not from whatever the reused allocation held
    if ((e = hipMemset(h->info.ptr, 0, sizeof(DevInfo))) != hipSuccess) {
        h->info.release();
        delete h;
        return hip_fail(e, "hipMemset(info)");
    }
    if ((e = hipHostMalloc((void**)&h->hinfo, sizeof(DevInfo), hipHostMallocDefault)) != hipSuccess) {
        h->info.release();
        delete h;
        return hip_fail(e, "hipHostMalloc");
    }
    // pending error word and host summaries: coherent, written by kernels
    if ((e = hipHostMalloc((void**)&h->hpending, sizeof(int), hipHostMallocCoherent)) != hipSuccess ||
        (e = hipHostMalloc((void**)&h->hsum, sizeof(HostSummary), hipHostMallocCoherent)) != hipSuccess ||
        (e = hipHostGetDevicePointer((void**)&h->dpending, h->hpending, 0)) != hipSuccess ||
        (e = hipHostGetDevicePointer((void**)&h->dsum, h->hsum, 0)) != hipSuccess) {
        if (h->hsum) (void)hipHostFree(h->hsum);
        if (h->hpending) (void)hipHostFree(h->hpending);
        (void)hipHostFree(h->hinfo);
        h->info.release();
        delete h;
        return hip_fail(e, "pinned host memory");
    }
    *h->hpending = 0;
    memset(h->hsum, 0, sizeof(HostSummary));
    if ((s = configure_kernels(h)) != MSP_OK || (e = create_streams(h)) != hipSuccess) {
        if (s == MSP_OK) s = hip_fail(e, "side streams");
        (void)hipHostFree(h->hsum);
        (void)hipHostFree(h->hpending);
        (void)hipHostFree(h->hinfo);
        h->info.release();
        delete h;
        return s;
    }
    *out = h;
    return MSP_OK;
}

extern "C" msp_status msp_destroy(msp_handle* h) {
    if (!h) return MSP_OK;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream); else (void)hipDeviceSynchronize();
    for (DevBuf* b : {&h->info, &h->u, &h->rnnz, &h->perm, &h->tiles, &h->sbm, &h->prod,
                      &h->bsum, &h->gsl, &h->win_islot, &h->win_row, &h->win_cnt, &h->win_bslot,
                      &h->win_wpos, &h->win_fb, &h->win_rbm, &h->win_bms,
                      &h->lr_list, &h->lr_base, &h->lr_chunk, &h->lr_acc})
        b->release();
    release_extra(h);
    h->prof.release();
    release_streams(h);
    if (h->hinfo) (void)hipHostFree(h->hinfo);
    if (h->hpending) (void)hipHostFree(h->hpending);
    if (h->hsum) (void)hipHostFree(h->hsum);
    delete h;
    return MSP_OK;
}

extern "C" msp_status msp_set_stream(msp_handle* h, void* stream) {
    if (!h) return fail(MSP_ERR_INVALID_ARG, "null handle");
    const hipStream_t ns = (hipStream_t)stream;
    if (ns == h->stream) return MSP_OK;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    // Calls share the handle's workspaces: work queued later on the new
    // stream waits for everything already queued on the old one.
    hipEvent_t ev = nullptr;
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "hipEventCreateWithFlags");
    e = hipEventRecord(ev, h->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(ns, ev, 0);
    (void)hipEventDestroy(ev);                  // the queued wait keeps what it needs
    if (e != hipSuccess) return hip_fail(e, "ordering the new stream after the old one");
    h->stream = ns;
    return MSP_OK;
}

extern "C" msp_status msp_set_allocator(msp_handle* h, msp_alloc_fn a, msp_free_fn f, void* ctx) {
    if (!h) return fail(MSP_ERR_INVALID_ARG, "null handle");
    if ((a == nullptr) != (f == nullptr)) return fail(MSP_ERR_INVALID_ARG, "alloc and free must both be set or both be NULL");
    h->alloc = a ? a : default_alloc;
    h->free_fn = f ? f : default_free;
    h->alloc_ctx = a ? ctx : nullptr;
    return MSP_OK;
}

extern "C" msp_status msp_set_tuning(msp_handle* h, const msp_tuning* t) {
    if (!h || !t) return fail(MSP_ERR_INVALID_ARG, "null argument");
    msp_tuning c = *t;
    msp_status s = check_tuning(&c);
    if (s != MSP_OK) return s;
    h->tuning = c;
    return MSP_OK;
}

extern "C" msp_status msp_get_tuning(const msp_handle* h, msp_tuning* t) {
    if (!h || !t) return fail(MSP_ERR_INVALID_ARG, "null argument");
    *t = h->tuning;
    return MSP_OK;
}

// ---------------------------------------------------------------------------
// argument checks
// ---------------------------------------------------------------------------
namespace msp {

msp_status check_csr(const msp_csr* M, const char* name) {
    if (!M) return fail(MSP_ERR_INVALID_ARG, "%s is NULL", name);
    if (M->nrows < 0 || M->ncols < 0 || M->nnz < 0) return fail(MSP_ERR_INVALID_ARG, "%s has a negative size", name);
    if (M->nrows > kMaxRows || M->ncols > INT32_MAX)
        return fail(MSP_ERR_INDEX_OVERFLOW, "%s: at most %lld rows and 2^31 - 1 columns (%lld x %lld)", name,
                    kMaxRows, (long long)M->nrows, (long long)M->ncols);
    if (M->dtype != MSP_F32 && M->dtype != MSP_F64) return fail(MSP_ERR_DTYPE, "%s: dtype must be MSP_F32 or MSP_F64", name);
    if (!M->row_ptr) return fail(MSP_ERR_INVALID_ARG, "%s.row_ptr is NULL", name);
    if (M->nnz > 0 && (!M->col || !M->val)) return fail(MSP_ERR_INVALID_ARG, "%s.col/val is NULL with nnz > 0", name);
    return MSP_OK;
}

msp_tuning default_tuning() {
    msp_tuning t;
    t.hash_scale = 1;
    t.group_scale = 0;
    t.spill_nnz = 4096;
    t.block_rows = 1024;
    t.merge_k = 8;
    t.share_g = -1;
    return t;
}

msp_status check_tuning(msp_tuning* t) {
    const msp_tuning d = default_tuning();
    if (t->hash_scale == 0) t->hash_scale = d.hash_scale;
    if (t->spill_nnz == 0) t->spill_nnz = d.spill_nnz;
    if (t->block_rows == 0) t->block_rows = d.block_rows;
    if (t->merge_k == 0) t->merge_k = d.merge_k;
    if (t->merge_k != 4 && t->merge_k != 8 && t->merge_k != -1)
        return fail(MSP_ERR_INVALID_ARG, "tuning.merge_k must be 4, 8 or -1");
    if (t->share_g == 0) t->share_g = d.share_g;
    if (t->share_g != -1 && (t->share_g < 8 || t->share_g > 64))
        return fail(MSP_ERR_INVALID_ARG, "tuning.share_g must be -1 or in 8..64");
    if (t->hash_scale < 1 || t->hash_scale > 2) return fail(MSP_ERR_INVALID_ARG, "tuning.hash_scale must be 1 or 2");
    if (t->group_scale < 0 || t->group_scale > 2) return fail(MSP_ERR_INVALID_ARG, "tuning.group_scale must be 0..2");
    if (t->spill_nnz < 256 || t->spill_nnz > 4096 || (t->spill_nnz & (t->spill_nnz - 1)))
        return fail(MSP_ERR_INVALID_ARG, "tuning.spill_nnz must be a power of two in 256..4096");
    if (t->block_rows < 32 || t->block_rows > 1024 || (t->block_rows & (t->block_rows - 1)))
        return fail(MSP_ERR_INVALID_ARG, "tuning.block_rows must be a power of two in 32..1024");
    return MSP_OK;
}

msp_tuning effective_tuning(const msp_handle* h, const msp_opts* o) {
    if (!o) return h->tuning;
    const msp_tuning& t = o->tuning;
    if (t.hash_scale == 0 && t.group_scale == 0 && t.spill_nnz == 0 && t.block_rows == 0 && t.merge_k == 0 &&
        t.share_g == 0)
        return h->tuning;
    msp_tuning c = t;
    if (check_tuning(&c) != MSP_OK) return h->tuning;
    return c;
}

}  // namespace msp

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------
namespace msp {

hipEvent_t Profiler::get() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

void Profiler::begin(int phase, hipStream_t s) {
    if (!on) return;
    if (open_phase >= 0) end(s);
    if (!((mask >> phase) & 1u)) return;
    open_ev = get();
    if (!open_ev) return;
    open_phase = phase;
    (void)hipEventRecord(open_ev, s);
}

void Profiler::end(hipStream_t s) {
    if (!on || open_phase < 0) return;
    hipEvent_t b = get();
    if (b) {
        (void)hipEventRecord(b, s);
        pending.push_back({open_phase, open_ev, b});
    } else {
        pool.push_back(open_ev);
    }
    open_phase = -1;
    open_ev = nullptr;
}

hipEvent_t Profiler::sub_begin(int phase, hipStream_t s) {
    if (!on || !((mask >> phase) & 1u)) return nullptr;
    hipEvent_t a = get();
    if (a) (void)hipEventRecord(a, s);
    return a;
}

void Profiler::sub_end(int phase, hipEvent_t a, hipStream_t s) {
    if (!a) return;
    hipEvent_t b = get();
    if (!b) {
        pool.push_back(a);
        return;
    }
    (void)hipEventRecord(b, s);
    pending.push_back({phase, a, b});
}

void Profiler::collect() {
    std::vector<Pending> keep;
    for (const Pending& p : pending) {
        if (hipEventQuery(p.b) != hipSuccess) {
            (void)hipGetLastError();
            keep.push_back(p);
            continue;
        }
        float t = 0.f;
        if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
            ms[p.phase] += t;
            count[p.phase] += 1;
        } else {
            (void)hipGetLastError();
        }
        pool.push_back(p.a);
        pool.push_back(p.b);
    }
    pending.swap(keep);
}

void Profiler::reset() {
    for (int i = 0; i < MSP_NUM_PHASES; ++i) { ms[i] = 0; count[i] = 0; }
}

void Profiler::release() {
    for (const Pending& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    if (open_ev) (void)hipEventDestroy(open_ev);
    pending.clear();
    pool.clear();
    open_ev = nullptr;
    open_phase = -1;
}

}  // namespace msp

extern "C" msp_status msp_profile_enable(msp_handle* h, int phase_mask) {
    if (!h) return fail(MSP_ERR_INVALID_ARG, "null handle");
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream); else (void)hipDeviceSynchronize();
    h->prof.collect();
    h->prof.reset();
    h->prof.on = phase_mask != 0;
    h->prof.mask = (unsigned)phase_mask;
    return MSP_OK;
}

extern "C" msp_status msp_profile_get(msp_handle* h, msp_profile* out) {
    if (!h || !out) return fail(MSP_ERR_INVALID_ARG, "null argument");
    h->prof.collect();
    for (int i = 0; i < MSP_NUM_PHASES; ++i) { out->ms[i] = h->prof.ms[i]; out->count[i] = h->prof.count[i]; }
    return MSP_OK;
}

extern "C" msp_status msp_sync(msp_handle* h) {
    if (!h) return fail(MSP_ERR_INVALID_ARG, "null handle");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (h->prof.on) h->prof.collect();
    // error bits of the last call's numeric kernels (taken here, so that
    // the next call does not report them again)
    int err = 0;
    DevInfo* info = h->info.as<DevInfo>();
    e = hipMemcpy(&err, &info->err, sizeof(int), hipMemcpyDeviceToHost);
    if (e == hipSuccess && err) e = hipMemset(&info->err, 0, sizeof(int));
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(error flags)");
    if (err & (kErrProbe | kErrCount)) __atomic_fetch_or(h->hpending, err, __ATOMIC_RELAXED);
    return take_pending_error(h);
}
