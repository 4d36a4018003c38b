// Learned output-size predictor and the one-pass product it enables.
//
// The network is a fully connected 8-64-64-1 ReLU MLP in FP32.  Its inputs
// are the per-row features of the row-statistics kernel; its output
// estimates log2(1 + row_nnz) / 16.  The capacity of row i is
//     cap_i = clamp(ceil(2^(16 y_i + delta)), lo_i, hi_i)
// with the exact bounds lo_i = max_k nnz(B(k,:)) (the union is at least its
// largest set) and hi_i = min(prod_i, ncols(B)); delta is a calibrated
// quantile of the training residuals.  Rows whose bounds are small take
// cap_i = hi_i without running the network.
//
// The one-pass product bins rows by capacity, runs the numeric kernels in
// capacity mode into a padded C (each row's true count, or -1 when it did
// not fit), recomputes the overflowed rows exactly with the plain two-phase
// path on the sub-matrix of those rows, and compacts everything into a
// tight CSR.  The structure is exact whatever the network predicts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "msp.h"

using namespace msp;

namespace msp {

constexpr int kNF = 8, kH1 = 64, kH2 = 64;
constexpr int kOffW1 = 0, kOffB1 = 512, kOffW2 = 576, kOffB2 = 4672, kOffW3 = 4736, kOffB3 = 4800;
constexpr int kNParam = 4801;
constexpr int kSmallCap = 32;      // rows with hi <= this skip the network

// ---------------------------------------------------------------------------
// network evaluation (weights in LDS, one row per thread)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float mlp_eval(const float* __restrict__ w, const float* __restrict__ xin) {
    float x[kNF];
#pragma unroll
    for (int f = 0; f < kNF; ++f) x[f] = xin[f];
    float h1[kH1];
#pragma unroll
    for (int i = 0; i < kH1; ++i) {
        float z = w[kOffB1 + i];
#pragma unroll
        for (int f = 0; f < kNF; ++f) z += w[kOffW1 + i * kNF + f] * x[f];
        h1[i] = z > 0.f ? z : 0.f;
    }
    float y = w[kOffB3];
#pragma unroll 1
    for (int j = 0; j < kH2; ++j) {
        const float4* row = reinterpret_cast<const float4*>(w + kOffW2 + j * kH1);
        float z = w[kOffB2 + j];
#pragma unroll
        for (int i4 = 0; i4 < kH1 / 4; ++i4) {
            const float4 q = row[i4];
            z += q.x * h1[4 * i4] + q.y * h1[4 * i4 + 1] + q.z * h1[4 * i4 + 2] + q.w * h1[4 * i4 + 3];
        }
        y += w[kOffW3 + j] * (z > 0.f ? z : 0.f);
    }
    return y;
}

// (at least 4 waves per SIMD: the weight loads are not hoisted into registers)
__global__ void __launch_bounds__(256, 4)
k_mlp_predict(long long n, const float* __restrict__ feats, const float* __restrict__ params, float* __restrict__ y) {
    __shared__ __align__(16) float w[kNParam + 3];
    for (int i = threadIdx.x; i < kNParam; i += 256) w[i] = params[i];
    __syncthreads();
    // one row per thread (a row loop would let the compiler hoist every
    // weight load out of it into registers)
    const long long r = (long long)blockIdx.x * 256 + threadIdx.x;
    if (r < n) y[r] = mlp_eval(w, feats + r * kNF);
}

// capacity rule; rows with small bounds skip the network.  Rows without
// products (cap 0) are in no numeric bin: their count is set to 0 here.
__global__ void __launch_bounds__(256, 4)
k_capacity(int m, const float* __restrict__ feats, const int32_t* __restrict__ hi, const int32_t* __restrict__ lo,
           const float* __restrict__ params, float delta, int32_t* __restrict__ cap, int32_t* __restrict__ cnt,
           BinTable nt, int big, int* __restrict__ nbig, unsigned long long* __restrict__ big_hi) {
    __shared__ __align__(16) float w[kNParam + 3];
    for (int i = threadIdx.x; i < kNParam; i += 256) w[i] = params[i];
    __syncthreads();
    const long long r = (long long)blockIdx.x * 256 + threadIdx.x;
    bool to_exact = false;
    unsigned long long exact_hi = 0;
    if (r < m) {
        const int h = hi[r];
        const int l = lo[r] < h ? lo[r] : h;
        int c = h;
        if (h > kSmallCap && l < h) {
            const float y = mlp_eval(w, feats + r * kNF);
            const double est = exp2((double)(16.f * y + delta));
            c = est < (double)h ? (int)ceil(est) : h;    // NaN or overflow: the upper bound
            c = c < l ? l : c;
            if (nt.nb > 0) {
                // the margin alone lifts the row past the bound of its point
                // prediction's bin: keep it in that bin, at the bin's bound
                const double pt = exp2((double)(16.f * y));
                if (pt < (double)h) {
                    int cp = (int)ceil(pt);
                    cp = cp < l ? l : cp;
                    const int bp = bin_of(nt, cp);
                    if (bp < nt.nb && bin_of(nt, c) > bp) c = nt.umax[bp];
                }
            }
            // the exact bound costs nothing more when it keeps the row in
            // the same numeric bin (same kernel, same accumulator): only
            // unused padding, which the compaction never reads; and it
            // costs at most twice the predicted room when it is within a
            // factor 2, where a row just above the prediction would
            // otherwise overflow into the exact recomputation
            if ((long long)h <= 2LL * c || (nt.nb > 0 && bin_of(nt, c) == bin_of(nt, h))) c = h;
        }
        // a capacity in the global bin: the row goes to the exact two-phase
        // path (its per-window counts come from the symbolic pass there),
        // with no padded room here
        to_exact = big >= 0 && c > big;
        if (to_exact) {
            c = 0;
            exact_hi = (unsigned long long)h;
        }
        cap[r] = c;
        if (c == 0) cnt[r] = to_exact ? -2 : 0;
    }
    const uint64_t bm = __ballot(to_exact);
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) exact_hi += __shfl_xor(exact_hi, d);
    if (bm && (threadIdx.x & 63) == __builtin_ctzll(bm)) {
        atomicAdd(nbig, __builtin_popcountll(bm));
        atomicAdd(big_hi, exact_hi);
    }
}

// ---------------------------------------------------------------------------
// training: forward + per-sample backward, gradient reduction, Adam
// ---------------------------------------------------------------------------
// Per sample s of the batch: activations and the backward deltas of the
// mean-squared error, stored for the reduction kernel.
__global__ void __launch_bounds__(256)
k_mlp_fwd_bwd(int batch, long long n, const int32_t* __restrict__ idx, const float* __restrict__ feats,
              const float* __restrict__ targets, const float* __restrict__ params,
              float* __restrict__ X, float* __restrict__ H1, float* __restrict__ H2,
              float* __restrict__ DZ1, float* __restrict__ DZ2, float* __restrict__ D, int* __restrict__ bad) {
    __shared__ __align__(16) float w[kNParam + 3];
    for (int i = threadIdx.x; i < kNParam; i += 256) w[i] = params[i];
    __syncthreads();
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= batch) return;
    long long r = idx[s];
    if (r < 0 || r >= n) {          // flagged; the sample reads row 0 instead
        atomicOr(bad, 1);
        r = 0;
    }
    float x[kNF];
#pragma unroll
    for (int f = 0; f < kNF; ++f) { x[f] = feats[r * kNF + f]; X[(long long)s * kNF + f] = x[f]; }
    // forward; activity masks of both hidden layers
    uint64_t act1 = 0, act2 = 0;
    float y = w[kOffB3];
    {
        float h1[kH1];
#pragma unroll
        for (int i = 0; i < kH1; ++i) {
            float z = w[kOffB1 + i];
#pragma unroll
            for (int f = 0; f < kNF; ++f) z += w[kOffW1 + i * kNF + f] * x[f];
            h1[i] = z > 0.f ? z : 0.f;
            act1 |= (uint64_t)(z > 0.f) << i;
            H1[(long long)s * kH1 + i] = h1[i];
        }
#pragma unroll 1
        for (int j = 0; j < kH2; ++j) {
            const float4* row = reinterpret_cast<const float4*>(w + kOffW2 + j * kH1);
            float z = w[kOffB2 + j];
#pragma unroll
            for (int i4 = 0; i4 < kH1 / 4; ++i4) {
                const float4 q = row[i4];
                z += q.x * h1[4 * i4] + q.y * h1[4 * i4 + 1] + q.z * h1[4 * i4 + 2] + q.w * h1[4 * i4 + 3];
            }
            const float h2 = z > 0.f ? z : 0.f;
            act2 |= (uint64_t)(z > 0.f) << j;
            H2[(long long)s * kH2 + j] = h2;
            y += w[kOffW3 + j] * h2;
        }
    }
    const float d = y - targets[r];
    D[s] = d;
    const float dy = 2.f * d / (float)batch;
    // backward: dz2_j = dy W3_j [z2_j > 0]; dz1_i = [z1_i > 0] sum_j W2[j][i] dz2_j
    float dz1[kH1];
#pragma unroll
    for (int i = 0; i < kH1; ++i) dz1[i] = 0.f;
#pragma unroll 1
    for (int j = 0; j < kH2; ++j) {
        const float dz2 = (act2 >> j) & 1 ? dy * w[kOffW3 + j] : 0.f;
        DZ2[(long long)s * kH2 + j] = dz2;
        const float4* row = reinterpret_cast<const float4*>(w + kOffW2 + j * kH1);
#pragma unroll
        for (int i4 = 0; i4 < kH1 / 4; ++i4) {
            const float4 q = row[i4];
            dz1[4 * i4] += q.x * dz2;
            dz1[4 * i4 + 1] += q.y * dz2;
            dz1[4 * i4 + 2] += q.z * dz2;
            dz1[4 * i4 + 3] += q.w * dz2;
        }
    }
#pragma unroll
    for (int i = 0; i < kH1; ++i) DZ1[(long long)s * kH1 + i] = (act1 >> i) & 1 ? dz1[i] : 0.f;
}

// Gradient, first level: workgroup t sums the batch tile [t TS, t TS + TS)
// for every parameter, in FP64, in sample order, into partial[t][p]; the
// tile's activations and deltas are staged in LDS first.  (The tiles
// replace one long serial loop per parameter; the sums stay in a fixed
// order, so the gradient is deterministic.)
constexpr int kGradTS = 32;                    // samples per tile
__global__ void __launch_bounds__(256)
k_mlp_grad_tile(int batch, const float* __restrict__ X, const float* __restrict__ H1, const float* __restrict__ H2,
                const float* __restrict__ DZ1, const float* __restrict__ DZ2, const float* __restrict__ D,
                double* __restrict__ partial, double* __restrict__ partial_loss) {
    __shared__ float sx[kGradTS][kNF], sh1[kGradTS][kH1], sh2[kGradTS][kH2], sd1[kGradTS][kH1 + 1],
        sd2[kGradTS][kH2 + 1], sd[kGradTS];
    const int t = blockIdx.x, tid = threadIdx.x;
    const int s0 = t * kGradTS;
    const int ns = batch - s0 < kGradTS ? batch - s0 : kGradTS;
    for (int e = tid; e < kGradTS * kH1; e += 256) {
        const int a = e / kH1, b = e % kH1;
        const bool in = a < ns;
        const long long g = (long long)(s0 + a);
        sh1[a][b] = in ? H1[g * kH1 + b] : 0.f;
        sh2[a][b] = in ? H2[g * kH2 + b] : 0.f;
        sd1[a][b] = in ? DZ1[g * kH1 + b] : 0.f;
        sd2[a][b] = in ? DZ2[g * kH2 + b] : 0.f;
        if (b < kNF) sx[a][b] = in ? X[g * kNF + b] : 0.f;
        if (b == 0) sd[a] = in ? D[g] : 0.f;
    }
    __syncthreads();
    const double scale = 2.0 / (double)batch;
    for (int p = tid; p < kNParam; p += 256) {
        double acc = 0.0;
        if (p < kOffB1) {
            const int i = p / kNF, f = p % kNF;
            for (int a = 0; a < ns; ++a) acc += (double)sd1[a][i] * sx[a][f];
        } else if (p < kOffW2) {
            const int i = p - kOffB1;
            for (int a = 0; a < ns; ++a) acc += sd1[a][i];
        } else if (p < kOffB2) {
            const int q = p - kOffW2, j = q / kH1, i = q % kH1;
            for (int a = 0; a < ns; ++a) acc += (double)sd2[a][j] * sh1[a][i];
        } else if (p < kOffW3) {
            const int j = p - kOffB2;
            for (int a = 0; a < ns; ++a) acc += sd2[a][j];
        } else if (p < kOffB3) {
            const int j = p - kOffW3;
            for (int a = 0; a < ns; ++a) acc += scale * sd[a] * sh2[a][j];
        } else {
            double l = 0.0;
            for (int a = 0; a < ns; ++a) {
                acc += scale * sd[a];
                l += (double)sd[a] * sd[a];
            }
            partial_loss[t] = l;
        }
        partial[(long long)t * kNParam + p] = acc;
    }
}

// Gradient, second level: the tiles' partial sums in tile order.
__global__ void __launch_bounds__(256)
k_mlp_grad_sum(int tiles, int batch, const double* __restrict__ partial, const double* __restrict__ partial_loss,
               float* __restrict__ grad, float* __restrict__ loss) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < kNParam) {
        double acc = 0.0;
        for (int t = 0; t < tiles; ++t) acc += partial[(long long)t * kNParam + p];
        grad[p] = (float)acc;
    }
    if (p == 0 && loss) {
        double l = 0.0;
        for (int t = 0; t < tiles; ++t) l += partial_loss[t];
        *loss = (float)(l / batch);
    }
}

// Adam (Kingma and Ba, 2015) with bias-corrected moments; step is 1-based.
__global__ void __launch_bounds__(256)
k_adam(float* __restrict__ params, const float* __restrict__ grad, float* __restrict__ m, float* __restrict__ v,
       int step, float lr, float beta1, float beta2, float eps) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kNParam) return;
    const float g = grad[p];
    const float mm = beta1 * m[p] + (1.f - beta1) * g;
    const float vv = beta2 * v[p] + (1.f - beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mhat = mm / (1.f - powf(beta1, (float)step));
    const float vhat = vv / (1.f - powf(beta2, (float)step));
    params[p] -= lr * mhat / (sqrtf(vhat) + eps);
}

// training target of a row: log2(1 + row_nnz) / 16
__global__ void __launch_bounds__(256)
k_targets(int m, const int32_t* __restrict__ row_nnz, float* __restrict__ t) {
    const long long r = (long long)blockIdx.x * 256 + threadIdx.x;
    if (r < m) t[r] = log2f(1.f + (float)row_nnz[r]) * kFeatLogScale;
}

// ---------------------------------------------------------------------------
// one-pass product helpers
// ---------------------------------------------------------------------------
// Overflowed rows (cnt < 0): list them in row order per wave, with their A
// lengths, and count them.
__global__ void __launch_bounds__(256)
k_collect_overflow(int m, const int32_t* __restrict__ cnt, const int64_t* __restrict__ arp,
                   int32_t* __restrict__ list, int* __restrict__ count, unsigned long long* __restrict__ sum_len) {
    const long long r = (long long)blockIdx.x * 256 + threadIdx.x;
    const bool o = r < m && cnt[r] < 0;
    const int lane = threadIdx.x & 63;
    const uint64_t mask = __ballot(o);
    if (!mask) return;
    int base = 0;
    const int leader = __builtin_ctzll(mask);
    if (lane == leader) base = atomicAdd(count, __builtin_popcountll(mask));
    base = __shfl(base, leader);
    if (o) {
        list[base + __builtin_popcountll(mask & ((1ull << lane) - 1))] = (int32_t)r;
        atomicAdd(sum_len, (unsigned long long)(arp[r + 1] - arp[r]));
    }
}

// Row pointers of the gathered sub-matrix (rows of A listed in `list`),
// computed serially per block chunk: lens then a single-block scan.
__global__ void __launch_bounds__(1024)
k_sub_rowptr(int ns, const int32_t* __restrict__ list, const int64_t* __restrict__ arp, int64_t* __restrict__ srp) {
    __shared__ BlockScanSmem<1024> sm;
    long long carry = 0;
    for (int c0 = 0; c0 < ns; c0 += 1024) {
        const int j = c0 + threadIdx.x;
        const long long len = j < ns ? arp[list[j] + 1] - arp[list[j]] : 0;
        long long tot;
        const long long incl = block_incl_scan<1024>(len, sm, &tot);
        if (j < ns) srp[j] = carry + incl - len;
        carry += tot;
    }
    if (threadIdx.x == 0) srp[ns] = carry;
}

template <typename VT>
__global__ void __launch_bounds__(256)
k_sub_gather(int ns, const int32_t* __restrict__ list, const int64_t* __restrict__ arp,
             const int32_t* __restrict__ acol, const VT* __restrict__ aval, const int64_t* __restrict__ srp,
             int32_t* __restrict__ scol, VT* __restrict__ sval) {
    // one wave per listed row
    const long long wid = ((long long)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wid >= ns) return;
    const long long a0 = arp[list[wid]], a1 = arp[list[wid] + 1], d0 = srp[wid];
    for (long long p = a0 + lane; p < a1; p += 64) {
        scol[d0 + p - a0] = acol[p];
        sval[d0 + p - a0] = aval[p];
    }
}

// Overflowed rows take their counts and sources from the sub-product.
__global__ void __launch_bounds__(256)
k_patch_overflow(int ns, const int32_t* __restrict__ list, const int64_t* __restrict__ crp_sub,
                 int32_t* __restrict__ cnt, int64_t* __restrict__ src_off) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= ns) return;
    const int r = list[j];
    cnt[r] = (int32_t)(crp_sub[j + 1] - crp_sub[j]);
    src_off[r] = -(crp_sub[j] + 1);              // negative: from the sub-product
}

// Compaction into the tight CSR, balanced by output entries: workgroup b
// writes destination entries [b CH, (b+1) CH) whatever the row lengths, so
// a hub row is spread over many workgroups.  chunk_row[b] is the row that
// holds entry b CH.  A row's source is the padded product at rp_pad[row],
// or the sub-product at -src_off[row]-1 when src_off[row] < 0.
constexpr int kCompactChunk = 4096;
constexpr int kCompactRows = 1024;      // rows staged in LDS per chunk

static __global__ void __launch_bounds__(256)
k_chunk_rows(int m, const int64_t* __restrict__ rp, int32_t* __restrict__ chunk_row) {
    const long long r = (long long)blockIdx.x * 256 + threadIdx.x;
    if (r >= m) return;
    const long long d0 = rp[r], d1 = rp[r + 1];
    for (long long c = (d0 + kCompactChunk - 1) / kCompactChunk; c * kCompactChunk < d1; ++c)
        chunk_row[c] = (int32_t)r;
}

template <typename VT>
__global__ void __launch_bounds__(256)
k_compact(int m, long long nnz, const int32_t* __restrict__ chunk_row, const int64_t* __restrict__ rp,
          const int64_t* __restrict__ rp_pad, const int64_t* __restrict__ src_off, const int32_t* __restrict__ pcol,
          const VT* __restrict__ pval, const int32_t* __restrict__ scol, const VT* __restrict__ sval,
          int32_t* __restrict__ ccol, VT* __restrict__ cval) {
    __shared__ long long s_rp[kCompactRows + 1];
    __shared__ long long s_src[kCompactRows];
    const long long nch = (nnz + kCompactChunk - 1) / kCompactChunk;
    const long long b = blockIdx.x;
    const long long d0 = b * kCompactChunk;
    const long long d1 = d0 + kCompactChunk < nnz ? d0 + kCompactChunk : nnz;
    const int r0 = chunk_row[b];
    const int r1 = b + 1 < nch ? chunk_row[b + 1] : m - 1;   // rows r0..r1 cover [d0, d1)
    const int nr = r1 - r0 + 1;
    // a row's source position of its first entry (negative: from the sub-product)
    auto src_of = [&](int r) -> long long {
        const long long so = src_off ? src_off[r] : 0;
        return so < 0 ? so : rp_pad[r];
    };
    if (nr <= kCompactRows) {
        for (int j = threadIdx.x; j <= nr; j += 256) {
            s_rp[j] = rp[r0 + j];
            if (j < nr) s_src[j] = src_of(r0 + j);
        }
        __syncthreads();
        for (long long d = d0 + threadIdx.x; d < d1; d += 256) {
            int lo = 0, hi = nr;                       // s_rp[lo] <= d < s_rp[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_rp[mid] <= d) lo = mid; else hi = mid;
            }
            const long long so = s_src[lo];
            const long long k = d - s_rp[lo];
            if (so < 0) { ccol[d] = scol[-so - 1 + k]; cval[d] = sval[-so - 1 + k]; }
            else { ccol[d] = pcol[so + k]; cval[d] = pval[so + k]; }
        }
    } else {
        // many short rows: one thread per row, clipped to the chunk
        for (int j = threadIdx.x; j < nr; j += 256) {
            const int r = r0 + j;
            const long long e0 = rp[r], e1 = rp[r + 1];
            const long long a = e0 > d0 ? e0 : d0, z = e1 < d1 ? e1 : d1;
            if (a >= z) continue;
            const long long so = src_of(r);
            for (long long d = a; d < z; ++d) {
                const long long k = d - e0;
                if (so < 0) { ccol[d] = scol[-so - 1 + k]; cval[d] = sval[-so - 1 + k]; }
                else { ccol[d] = pcol[so + k]; cval[d] = pval[so + k]; }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// predictor object
// ---------------------------------------------------------------------------
struct ExtraState {
    DevBuf feat, lo, cap, rp_pad, cnt, src_off, pad, list, sub_rp, sub_a, sub_c, sub_crp, chunk;
};

static ExtraState* extra(msp_handle* h) {
    if (!h->extra) h->extra = new (std::nothrow) ExtraState();
    return h->extra;
}

void release_extra(msp_handle* h) {
    if (!h->extra) return;
    ExtraState* x = h->extra;
    for (DevBuf* b : {&x->feat, &x->lo, &x->cap, &x->rp_pad, &x->cnt, &x->src_off, &x->pad, &x->list, &x->sub_rp,
                      &x->sub_a, &x->sub_c, &x->sub_crp, &x->chunk})
        b->release();
    delete x;
    h->extra = nullptr;
}

static msp_status launch_check2(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return MSP_OK;
}

}  // namespace msp

struct msp_predictor {
    int device = 0;
    msp::DevBuf params, m, v, grad, loss, bad, X, H1, H2, DZ1, DZ2, D, part, part_loss;
    int batch_cap = 0;
    float delta = 0.f;
    long long step = 0;
};

extern "C" msp_status msp_predictor_create(msp_handle* h, const float* init_params, msp_predictor** out) {
    if (!h || !init_params || !out) return fail(MSP_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    msp_predictor* p = new (std::nothrow) msp_predictor();
    if (!p) return fail(MSP_ERR_OOM, "host allocation failed");
    p->device = h->device;
    msp_status s;
    for (DevBuf* b : {&p->params, &p->m, &p->v, &p->grad, &p->bad}) {
        if ((s = b->ensure(kNParam * sizeof(float))) != MSP_OK) { msp_predictor_destroy(p); return s; }
        if ((e = hipMemsetAsync(b->ptr, 0, kNParam * sizeof(float), h->stream)) != hipSuccess) {
            msp_predictor_destroy(p);
            return hip_fail(e, "hipMemsetAsync");
        }
    }
    if ((e = hipMemcpyAsync(p->params.ptr, init_params, kNParam * sizeof(float), hipMemcpyHostToDevice, h->stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(h->stream)) != hipSuccess) {
        msp_predictor_destroy(p);
        return hip_fail(e, "hipMemcpyAsync(params)");
    }
    *out = p;
    return MSP_OK;
}

extern "C" msp_status msp_predictor_destroy(msp_predictor* p) {
    if (!p) return MSP_OK;
    (void)hipSetDevice(p->device);
    for (DevBuf* b :
         {&p->params, &p->m, &p->v, &p->grad, &p->loss, &p->bad, &p->X, &p->H1, &p->H2, &p->DZ1, &p->DZ2, &p->D,
          &p->part, &p->part_loss})
        b->release();
    delete p;
    return MSP_OK;
}

extern "C" msp_status msp_predictor_get(msp_handle* h, const msp_predictor* p, float* params, float* delta) {
    if (!h || !p) return fail(MSP_ERR_INVALID_ARG, "null argument");
    if (params) {
        hipError_t e = hipMemcpyAsync(params, p->params.ptr, kNParam * sizeof(float), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(params)");
    }
    if (delta) *delta = p->delta;
    return MSP_OK;
}

extern "C" msp_status msp_predictor_set(msp_handle* h, msp_predictor* p, const float* params, float delta) {
    if (!h || !p) return fail(MSP_ERR_INVALID_ARG, "null argument");
    if (params) {
        hipError_t e = hipMemcpyAsync(p->params.ptr, params, kNParam * sizeof(float), hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(params)");
    }
    p->delta = delta;
    return MSP_OK;
}

// ---------------------------------------------------------------------------
// serialized form (little-endian): magic "MSPP", u32 version, u32 parameter
// count, f32 delta, i64 Adam step count, then the parameters and Adam's two
// moment arrays (f32 each), then a u64 FNV-1a hash of every byte before it
// ---------------------------------------------------------------------------
namespace {
constexpr uint32_t kBlobVersion = 1;
constexpr size_t kBlobHeader = 24;
constexpr size_t kBlobBytes = kBlobHeader + 3 * (size_t)kNParam * 4 + 8;
static_assert(kBlobBytes == MSP_PREDICTOR_BLOB_BYTES, "blob layout and its declared size agree");

uint64_t fnv1a64(const unsigned char* p, size_t n) {
    uint64_t x = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; ++i) {
        x ^= p[i];
        x *= 0x100000001b3ull;
    }
    return x;
}
}  // namespace

extern "C" msp_status msp_predictor_blob_pack(const float* params, const float* adam_m, const float* adam_v,
                                              float delta, int64_t step, void* blob, size_t cap, size_t* size) {
    if (size) *size = kBlobBytes;
    if (!blob) return size ? MSP_OK : fail(MSP_ERR_INVALID_ARG, "blob and size are both NULL");
    if (!params) return fail(MSP_ERR_INVALID_ARG, "params is NULL");
    if (cap < kBlobBytes) return fail(MSP_ERR_INVALID_ARG, "blob buffer of %zu bytes, %zu needed", cap, kBlobBytes);
    unsigned char* b = (unsigned char*)blob;
    const uint32_t np = kNParam;
    memcpy(b, "MSPP", 4);
    memcpy(b + 4, &kBlobVersion, 4);
    memcpy(b + 8, &np, 4);
    memcpy(b + 12, &delta, 4);
    memcpy(b + 16, &step, 8);
    unsigned char* q = b + kBlobHeader;
    for (const float* a : {params, adam_m, adam_v}) {
        if (a) memcpy(q, a, (size_t)kNParam * 4);
        else memset(q, 0, (size_t)kNParam * 4);
        q += (size_t)kNParam * 4;
    }
    const uint64_t hsh = fnv1a64(b, kBlobBytes - 8);
    memcpy(q, &hsh, 8);
    return MSP_OK;
}

extern "C" msp_status msp_predictor_blob_unpack(const void* blob, size_t size, float* params, float* adam_m,
                                                float* adam_v, float* delta, int64_t* step) {
    if (!blob) return fail(MSP_ERR_INVALID_ARG, "blob is NULL");
    const unsigned char* b = (const unsigned char*)blob;
    if (size < kBlobHeader || memcmp(b, "MSPP", 4) != 0)
        return fail(MSP_ERR_INVALID_ARG, "not a predictor blob (magic)");
    uint32_t ver = 0, np = 0;
    memcpy(&ver, b + 4, 4);
    memcpy(&np, b + 8, 4);
    if (ver != kBlobVersion)
        return fail(MSP_ERR_UNSUPPORTED, "predictor blob version %u; this library reads version %u", ver, kBlobVersion);
    if (np != (uint32_t)kNParam) return fail(MSP_ERR_INVALID_ARG, "predictor blob holds %u parameters, not %d", np, kNParam);
    if (size != kBlobBytes) return fail(MSP_ERR_INVALID_ARG, "predictor blob of %zu bytes, %zu expected", size, kBlobBytes);
    uint64_t hsh = 0;
    memcpy(&hsh, b + kBlobBytes - 8, 8);
    if (hsh != fnv1a64(b, kBlobBytes - 8)) return fail(MSP_ERR_INVALID_ARG, "predictor blob checksum mismatch");
    if (delta) memcpy(delta, b + 12, 4);
    if (step) memcpy(step, b + 16, 8);
    const unsigned char* q = b + kBlobHeader;
    for (float* a : {params, adam_m, adam_v}) {
        if (a) memcpy(a, q, (size_t)kNParam * 4);
        q += (size_t)kNParam * 4;
    }
    return MSP_OK;
}

extern "C" msp_status msp_predictor_save(msp_handle* h, const msp_predictor* p, void* blob, size_t cap, size_t* size) {
    if (!h || !p) return fail(MSP_ERR_INVALID_ARG, "null argument");
    if (size) *size = kBlobBytes;
    if (!blob) return size ? MSP_OK : fail(MSP_ERR_INVALID_ARG, "blob and size are both NULL");
    if (cap < kBlobBytes) return fail(MSP_ERR_INVALID_ARG, "blob buffer of %zu bytes, %zu needed", cap, kBlobBytes);
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    std::vector<float> host(3 * (size_t)kNParam);
    const DevBuf* src[3] = {&p->params, &p->m, &p->v};
    for (int i = 0; i < 3 && e == hipSuccess; ++i)
        e = hipMemcpyAsync(host.data() + (size_t)i * kNParam, src[i]->ptr, (size_t)kNParam * 4, hipMemcpyDeviceToHost,
                           h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(predictor state)");
    return msp_predictor_blob_pack(host.data(), host.data() + kNParam, host.data() + 2 * kNParam, p->delta, p->step,
                                   blob, cap, nullptr);
}

extern "C" msp_status msp_predictor_load(msp_handle* h, msp_predictor* p, const void* blob, size_t size) {
    if (!h || !p) return fail(MSP_ERR_INVALID_ARG, "null argument");
    std::vector<float> host(3 * (size_t)kNParam);
    float delta = 0.f;
    int64_t step = 0;
    msp_status s = msp_predictor_blob_unpack(blob, size, host.data(), host.data() + kNParam,
                                             host.data() + 2 * kNParam, &delta, &step);
    if (s != MSP_OK) return s;
    if (step < 0) return fail(MSP_ERR_INVALID_ARG, "predictor blob has a negative step count");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    DevBuf* dst[3] = {&p->params, &p->m, &p->v};
    for (int i = 0; i < 3 && e == hipSuccess; ++i)
        e = hipMemcpyAsync(dst[i]->ptr, host.data() + (size_t)i * kNParam, (size_t)kNParam * 4, hipMemcpyHostToDevice,
                           h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(predictor state)");
    p->delta = delta;
    p->step = step;
    return MSP_OK;
}

static msp_status ensure_batch(msp_predictor* p, int batch) {
    if (batch <= p->batch_cap) return MSP_OK;
    msp_status s;
    const size_t b = (size_t)batch;
    if ((s = p->X.ensure(b * kNF * 4)) != MSP_OK || (s = p->H1.ensure(b * kH1 * 4)) != MSP_OK ||
        (s = p->H2.ensure(b * kH2 * 4)) != MSP_OK || (s = p->DZ1.ensure(b * kH1 * 4)) != MSP_OK ||
        (s = p->DZ2.ensure(b * kH2 * 4)) != MSP_OK || (s = p->D.ensure(b * 4)) != MSP_OK)
        return s;
    const size_t tiles = (b + kGradTS - 1) / kGradTS;
    if ((s = p->part.ensure(tiles * kNParam * 8)) != MSP_OK || (s = p->part_loss.ensure(tiles * 8)) != MSP_OK)
        return s;
    p->batch_cap = batch;
    return MSP_OK;
}

// one forward/backward + gradient reduction on batch rows idx[0..batch)
static msp_status grad_step(msp_handle* h, msp_predictor* p, const float* feats, const float* targets, int64_t n,
                            const int32_t* idx, int batch, float* loss_dev) {
    msp_status s = ensure_batch(p, batch);
    if (s != MSP_OK) return s;
    k_mlp_fwd_bwd<<<(batch + 255) / 256, 256, 0, h->stream>>>(
        batch, n, idx, feats, targets, p->params.as<float>(), p->X.as<float>(), p->H1.as<float>(), p->H2.as<float>(),
        p->DZ1.as<float>(), p->DZ2.as<float>(), p->D.as<float>(), p->bad.as<int>());
    if ((s = launch_check2("k_mlp_fwd_bwd")) != MSP_OK) return s;
    const int tiles = (batch + kGradTS - 1) / kGradTS;
    k_mlp_grad_tile<<<tiles, 256, 0, h->stream>>>(batch, p->X.as<float>(), p->H1.as<float>(), p->H2.as<float>(),
                                                  p->DZ1.as<float>(), p->DZ2.as<float>(), p->D.as<float>(),
                                                  p->part.as<double>(), p->part_loss.as<double>());
    if ((s = launch_check2("k_mlp_grad_tile")) != MSP_OK) return s;
    k_mlp_grad_sum<<<(kNParam + 255) / 256, 256, 0, h->stream>>>(tiles, batch, p->part.as<double>(),
                                                                  p->part_loss.as<double>(), p->grad.as<float>(),
                                                                  loss_dev);
    return launch_check2("k_mlp_grad_sum");
}

// Sample indices outside [0, n) were flagged by the forward/backward kernel:
// report them (and clear the flag) once the stream has drained.
static msp_status take_bad_index(msp_handle* h, msp_predictor* p) {
    int bad = 0;
    hipError_t e = hipMemcpyAsync(&bad, p->bad.ptr, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(index flag)");
    if (!bad) return MSP_OK;
    if ((e = hipMemsetAsync(p->bad.ptr, 0, sizeof(int), h->stream)) != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    return fail(MSP_ERR_INVALID_ARG, "a batch index is outside [0, n)");
}

extern "C" msp_status msp_predictor_grad(msp_handle* h, msp_predictor* p, const float* feats, const float* targets,
                                         int64_t n, const int32_t* idx, int batch, float* grad_host,
                                         float* loss_host) {
    if (!h || !p || !feats || !targets || !idx || batch <= 0 || n <= 0) return fail(MSP_ERR_INVALID_ARG, "bad argument");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    msp_status s = p->loss.ensure(sizeof(float));
    if (s != MSP_OK) return s;
    if ((s = grad_step(h, p, feats, targets, n, idx, batch, p->loss.as<float>())) != MSP_OK) return s;
    if (grad_host &&
        (e = hipMemcpyAsync(grad_host, p->grad.ptr, kNParam * 4, hipMemcpyDeviceToHost, h->stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(grad)");
    if (loss_host && (e = hipMemcpyAsync(loss_host, p->loss.ptr, 4, hipMemcpyDeviceToHost, h->stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(loss)");
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return take_bad_index(h, p);
}

extern "C" msp_status msp_predictor_train(msp_handle* h, msp_predictor* p, const float* feats, const float* targets,
                                          int64_t n, const int32_t* batch_idx, int steps, int batch,
                                          const msp_train_opts* o, float* losses_host) {
    if (!h || !p || !feats || !targets || !batch_idx || n <= 0 || steps < 0 || batch <= 0)
        return fail(MSP_ERR_INVALID_ARG, "bad argument");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const float lr = o && o->lr > 0 ? o->lr : 1e-3f;
    const float b1 = o && o->beta1 > 0 ? o->beta1 : 0.9f;
    const float b2 = o && o->beta2 > 0 ? o->beta2 : 0.999f;
    const float eps = o && o->eps > 0 ? o->eps : 1e-8f;
    msp_status s = p->loss.ensure((size_t)std::max(steps, 1) * sizeof(float));
    if (s != MSP_OK) return s;
    for (int t = 0; t < steps; ++t) {
        if ((s = grad_step(h, p, feats, targets, n, batch_idx + (size_t)t * batch, batch, p->loss.as<float>() + t)) !=
            MSP_OK)
            return s;
        ++p->step;
        k_adam<<<(kNParam + 255) / 256, 256, 0, h->stream>>>(p->params.as<float>(), p->grad.as<float>(),
                                                             p->m.as<float>(), p->v.as<float>(), (int)p->step, lr, b1,
                                                             b2, eps);
        if ((s = launch_check2("k_adam")) != MSP_OK) return s;
    }
    if (losses_host && steps > 0 &&
        (e = hipMemcpyAsync(losses_host, p->loss.ptr, (size_t)steps * 4, hipMemcpyDeviceToHost, h->stream)) !=
            hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(losses)");
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return take_bad_index(h, p);
}

extern "C" msp_status msp_predictor_infer(msp_handle* h, const msp_predictor* p, const float* feats, int64_t n,
                                          float* y) {
    if (!h || !p || (n > 0 && (!feats || !y)) || n < 0) return fail(MSP_ERR_INVALID_ARG, "bad argument");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (n == 0) return MSP_OK;
    const long long blocks = (n + 255) / 256;
    if (blocks > INT32_MAX) return fail(MSP_ERR_INDEX_OVERFLOW, "too many rows");
    k_mlp_predict<<<(int)blocks, 256, 0, h->stream>>>(n, feats, p->params.as<float>(), y);
    return launch_check2("k_mlp_predict");
}

// delta = the q-quantile of 16 (t - y) over the rows given (log2 units).
extern "C" msp_status msp_predictor_calibrate(msp_handle* h, msp_predictor* p, const float* feats,
                                              const float* targets, int64_t n, double q) {
    if (!h || !p || !feats || !targets || n <= 0 || !(q > 0 && q < 1)) return fail(MSP_ERR_INVALID_ARG, "bad argument");
    DevBuf y;
    msp_status s = y.ensure((size_t)n * 4);
    if (s != MSP_OK) return s;
    if ((s = msp_predictor_infer(h, p, feats, n, y.as<float>())) != MSP_OK) { y.release(); return s; }
    std::vector<float> yh((size_t)n), th((size_t)n);
    hipError_t e = hipMemcpyAsync(yh.data(), y.ptr, (size_t)n * 4, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(th.data(), targets, (size_t)n * 4, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    y.release();
    if (e != hipSuccess) return hip_fail(e, "calibration copy");
    std::vector<float> res((size_t)n);
    for (size_t i = 0; i < (size_t)n; ++i) res[i] = 16.f * (th[i] - yh[i]);
    const size_t k = std::min((size_t)n - 1, (size_t)std::ceil(q * (double)n) - 1);
    std::nth_element(res.begin(), res.begin() + k, res.end());
    p->delta = res[k];
    return MSP_OK;
}

// ---------------------------------------------------------------------------
// the one-pass product
// ---------------------------------------------------------------------------
extern "C" msp_status msp_spgemm_learned(msp_handle* h, const msp_predictor* p, const msp_csr* A, const msp_csr* B,
                                         msp_csr_out* C, const msp_opts* opts, msp_learned_stats* st) {
    if (!h || !p) return fail(MSP_ERR_INVALID_ARG, "null handle or predictor");
    if (!C) return fail(MSP_ERR_INVALID_ARG, "C is NULL");
    msp_status s = check_pair(A, B);
    if (s != MSP_OK) return s;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    ExtraState* x = extra(h);
    if (!x) return fail(MSP_ERR_OOM, "host allocation failed");
    const msp_tuning t = effective_tuning(h, opts);
    const int m = (int)A->nrows;
    const size_t vsz = A->dtype == MSP_F64 ? 8 : 4;
    if (opts && opts->validate && (s = validate_inputs(h, A, B)) != MSP_OK) return s;
    msp_learned_stats stats;
    memset(&stats, 0, sizeof(stats));

    const size_t mm = (size_t)std::max(m, 1);
    if ((s = h->rnnz.ensure(mm * 4)) != MSP_OK || (s = x->feat.ensure(mm * kNF * 4)) != MSP_OK ||
        (s = x->lo.ensure(mm * 4)) != MSP_OK || (s = x->cap.ensure(mm * 4)) != MSP_OK ||
        (s = x->rp_pad.ensure((mm + 1) * 8)) != MSP_OK || (s = x->cnt.ensure(mm * 4)) != MSP_OK)
        return s;

    bool own_rp = false;
    if (!C->row_ptr) {
        C->row_ptr = (int64_t*)h->alloc(h->alloc_ctx, (size_t)(m + 1) * 8, h->stream);
        if (!C->row_ptr) return fail(MSP_ERR_OOM, "allocation of C.row_ptr failed");
        own_rp = true;
    }
    C->col = nullptr;
    C->val = nullptr;
    auto cleanup = [&](msp_status r) {
        if (C->col) h->free_fn(h->alloc_ctx, C->col, h->stream);
        C->col = nullptr;
        C->val = nullptr;
        if (own_rp) { h->free_fn(h->alloc_ctx, C->row_ptr, h->stream); C->row_ptr = nullptr; }
        return r;
    };

    // 1. features and bounds, 2. capacities
    BinPlan none;
    memset(&none, 0, sizeof(none));
    if ((s = zero_info(h)) != MSP_OK) return cleanup(s);
    h->prof.begin(MSP_PHASE_ROW_STATS, h->stream);
    if ((s = run_row_stats(h, A, B, none, nullptr, x->feat.as<float>(), x->lo.as<int32_t>())) != MSP_OK)
        return cleanup(s);
    h->prof.end(h->stream);
    const BinPlan np = numeric_plan(t, opts && opts->force_spill);
    h->prof.begin(MSP_PHASE_PREDICT, h->stream);
    if (m > 0) {
        const int blocks = (m + 255) / 256;
        // rows whose capacity falls in the global bin take the exact path
        const int big = (opts && opts->force_spill) || np.table.nb <= 1 ? -1 : np.table.umax[np.table.nb - 1];
        k_capacity<<<blocks, 256, 0, h->stream>>>(m, x->feat.as<float>(), h->u.as<int32_t>(), x->lo.as<int32_t>(),
                                                  p->params.as<float>(), p->delta, x->cap.as<int32_t>(),
                                                  x->cnt.as<int32_t>(), np.table, big,
                                                  &h->info.as<DevInfo>()->learned_big,
                                                  &h->info.as<DevInfo>()->learned_big_hi);
        if ((s = launch_check2("k_capacity")) != MSP_OK) return cleanup(s);
    }
    h->prof.end(h->stream);
    // 3. padded row pointers and bins by capacity
    h->prof.begin(MSP_PHASE_SCAN, h->stream);
    if ((s = run_scan(h, m, x->cap.as<int32_t>(), x->rp_pad.as<int64_t>(), &np)) != MSP_OK) return cleanup(s);
    h->prof.end(h->stream);
    if ((s = read_info(h)) != MSP_OK) return cleanup(s);
    if ((s = device_error(h->hinfo->err)) != MSP_OK) return cleanup(s);
    const long long sum_cap = h->hinfo->nnz;
    stats.sum_cap = sum_cap;
    stats.exact_rows = h->hinfo->learned_big;
    if (stats.exact_rows > 0 && (long long)h->hinfo->learned_big_hi > sum_cap) {
        // more of the bounded work is in rows that take the exact path anyway
        // than in the predicted rows: the two-phase product of the whole
        // matrix does less than the two paths together
        msp_opts so;
        memset(&so, 0, sizeof(so));
        so.tuning = t;
        s = spgemm_core(
            h, A, B, C, &so, [h](size_t bytes) -> void* { return h->alloc(h->alloc_ctx, bytes, h->stream); },
            [h](void* ptr) { h->free_fn(h->alloc_ctx, ptr, h->stream); });
        if (s != MSP_OK) return cleanup(s);
        stats.exact_rows = m;
        stats.sum_cap = 0;
        stats.overflow_rows = 0;
        stats.nnz = C->nnz;
        if (st) *st = stats;
        return MSP_OK;
    }
    int counts[kNB];
    sum_parts(h->hinfo->num_part, counts);
    // 4. numeric pass in capacity mode into the padded area
    if ((s = x->pad.ensure((size_t)std::max(sum_cap, 1LL) * (4 + vsz) + 256)) != MSP_OK) return cleanup(s);
    int32_t* pcol = x->pad.as<int32_t>();
    char* pval = (char*)x->pad.ptr + (((size_t)std::max(sum_cap, 1LL) * 4 + 255) & ~(size_t)255);
    // (the device info is not cleared here: the scatter of rows into bins
    // reads the per-partition bin counts that the scan just wrote)
    h->prof.begin(MSP_PHASE_NUMERIC, h->stream);
    if ((s = run_numeric_bins(h, A, B, np, counts, x->cap.as<int32_t>(), x->rp_pad.as<int64_t>(), pcol, pval,
                              x->cnt.as<int32_t>())) != MSP_OK)
        return cleanup(s);
    h->prof.end(h->stream);
    // 5. final row pointers (overflowed rows count 0 for now) and overflow count
    h->prof.begin(MSP_PHASE_COMPACT, h->stream);
    if ((s = zero_info(h)) != MSP_OK) return cleanup(s);
    if ((s = run_scan(h, m, x->cnt.as<int32_t>(), C->row_ptr, nullptr)) != MSP_OK) return cleanup(s);
    h->prof.end(h->stream);
    if ((s = read_info(h)) != MSP_OK) return cleanup(s);
    if ((s = device_error(h->hinfo->err)) != MSP_OK) return cleanup(s);
    const int novf = h->hinfo->neg_count;
    stats.overflow_rows = novf - stats.exact_rows;
    int64_t* src_off = nullptr;
    int32_t* scol = nullptr;
    char* sval = nullptr;
    if (novf > 0) {
        // 6. exact recomputation of the overflowed rows on their sub-matrix
        h->prof.begin(MSP_PHASE_FALLBACK, h->stream);
        if ((s = x->list.ensure((size_t)novf * 4)) != MSP_OK || (s = x->src_off.ensure(mm * 8)) != MSP_OK ||
            (s = x->sub_rp.ensure(((size_t)novf + 1) * 8)) != MSP_OK)
            return cleanup(s);
        if ((e = hipMemsetAsync(x->src_off.ptr, 0, mm * 8, h->stream)) != hipSuccess)
            return cleanup(hip_fail(e, "hipMemsetAsync"));
        if ((s = zero_info(h)) != MSP_OK) return cleanup(s);
        DevInfo* info = h->info.as<DevInfo>();
        k_collect_overflow<<<(m + 255) / 256, 256, 0, h->stream>>>(m, x->cnt.as<int32_t>(), A->row_ptr,
                                                                   x->list.as<int32_t>(), &info->neg_count,
                                                                   (unsigned long long*)&info->nnz);
        if ((s = launch_check2("k_collect_overflow")) != MSP_OK) return cleanup(s);
        if ((s = read_info(h)) != MSP_OK) return cleanup(s);
        const long long sub_nnz = h->hinfo->nnz;
        if (h->hinfo->neg_count != novf) return cleanup(fail(MSP_ERR_HIP, "internal: overflow list size"));
        if ((s = x->sub_a.ensure((size_t)std::max(sub_nnz, 1LL) * (4 + vsz) + 256)) != MSP_OK) return cleanup(s);
        int32_t* sacol = x->sub_a.as<int32_t>();
        char* saval = (char*)x->sub_a.ptr + (((size_t)std::max(sub_nnz, 1LL) * 4 + 255) & ~(size_t)255);
        k_sub_rowptr<<<1, 1024, 0, h->stream>>>(novf, x->list.as<int32_t>(), A->row_ptr, x->sub_rp.as<int64_t>());
        if ((s = launch_check2("k_sub_rowptr")) != MSP_OK) return cleanup(s);
        const int gb = (int)(((long long)novf * 64 + 255) / 256);
        if (A->dtype == MSP_F64)
            k_sub_gather<double><<<gb, 256, 0, h->stream>>>(novf, x->list.as<int32_t>(), A->row_ptr, A->col,
                                                            (const double*)A->val, x->sub_rp.as<int64_t>(), sacol,
                                                            (double*)saval);
        else
            k_sub_gather<float><<<gb, 256, 0, h->stream>>>(novf, x->list.as<int32_t>(), A->row_ptr, A->col,
                                                           (const float*)A->val, x->sub_rp.as<int64_t>(), sacol,
                                                           (float*)saval);
        if ((s = launch_check2("k_sub_gather")) != MSP_OK) return cleanup(s);
        msp_csr Asub{novf, A->ncols, sub_nnz, x->sub_rp.as<int64_t>(), sacol, saval, A->dtype};
        if ((s = x->sub_crp.ensure(((size_t)novf + 1) * 8)) != MSP_OK) return cleanup(s);
        msp_csr_out Csub;
        memset(&Csub, 0, sizeof(Csub));
        Csub.row_ptr = x->sub_crp.as<int64_t>();
        DevBuf* subc = &x->sub_c;
        auto ws_alloc = [subc](size_t bytes) -> void* {
            if (subc->ensure(std::max(bytes, (size_t)256)) != MSP_OK) return nullptr;
            return subc->ptr;
        };
        msp_opts so;
        memset(&so, 0, sizeof(so));
        so.tuning = t;
        if ((s = spgemm_core(h, &Asub, B, &Csub, &so, ws_alloc, [](void*) {})) != MSP_OK) return cleanup(s);
        scol = Csub.col;
        sval = (char*)Csub.val;
        k_patch_overflow<<<(novf + 255) / 256, 256, 0, h->stream>>>(novf, x->list.as<int32_t>(), Csub.row_ptr,
                                                                    x->cnt.as<int32_t>(), x->src_off.as<int64_t>());
        if ((s = launch_check2("k_patch_overflow")) != MSP_OK) return cleanup(s);
        if ((s = zero_info(h)) != MSP_OK) return cleanup(s);
        if ((s = run_scan(h, m, x->cnt.as<int32_t>(), C->row_ptr, nullptr)) != MSP_OK) return cleanup(s);
        if ((s = read_info(h)) != MSP_OK) return cleanup(s);
        if ((s = device_error(h->hinfo->err)) != MSP_OK) return cleanup(s);
        if (h->hinfo->neg_count != 0) return cleanup(fail(MSP_ERR_HIP, "internal: rows left after the fallback"));
        src_off = x->src_off.as<int64_t>();
        h->prof.end(h->stream);
    }
    // 7. tight output
    const long long nnz = h->hinfo->nnz;
    stats.nnz = nnz;
    C->nrows = m;
    C->ncols = B->ncols;
    C->nnz = nnz;
    C->dtype = A->dtype;
    if (nnz > 0) {
        const size_t voff = ((size_t)nnz * 4 + 255) & ~(size_t)255;
        void* base = h->alloc(h->alloc_ctx, voff + (size_t)nnz * vsz, h->stream);
        if (!base) return cleanup(fail(MSP_ERR_OOM, "allocation of C (%lld nonzeros) failed", nnz));
        C->col = (int32_t*)base;
        C->val = (char*)base + voff;
        const long long nch = (nnz + kCompactChunk - 1) / kCompactChunk;
        if (nch > INT32_MAX) return cleanup(fail(MSP_ERR_INDEX_OVERFLOW, "too many output entries"));
        if ((s = x->chunk.ensure((size_t)nch * 4)) != MSP_OK) return cleanup(s);
        h->prof.begin(MSP_PHASE_COMPACT, h->stream);
        k_chunk_rows<<<(m + 255) / 256, 256, 0, h->stream>>>(m, C->row_ptr, x->chunk.as<int32_t>());
        if ((s = launch_check2("k_chunk_rows")) != MSP_OK) return cleanup(s);
        if (A->dtype == MSP_F64)
            k_compact<double><<<(int)nch, 256, 0, h->stream>>>(m, nnz, x->chunk.as<int32_t>(), C->row_ptr,
                                                              x->rp_pad.as<int64_t>(), src_off, pcol,
                                                              (const double*)pval, scol, (const double*)sval, C->col,
                                                              (double*)C->val);
        else
            k_compact<float><<<(int)nch, 256, 0, h->stream>>>(m, nnz, x->chunk.as<int32_t>(), C->row_ptr,
                                                             x->rp_pad.as<int64_t>(), src_off, pcol,
                                                             (const float*)pval, scol, (const float*)sval, C->col,
                                                             (float*)C->val);
        if ((s = launch_check2("k_compact")) != MSP_OK) return cleanup(s);
        h->prof.end(h->stream);
        hipError_t e2 = hipMemcpyAsync(h->hpending, &h->info.as<DevInfo>()->err, sizeof(int), hipMemcpyDeviceToHost,
                                       h->stream);
        if (e2 != hipSuccess) return cleanup(hip_fail(e2, "hipMemcpyAsync(error flags)"));
    }
    if (st) *st = stats;
    return MSP_OK;
}

extern "C" msp_status msp_training_rows(msp_handle* h, const msp_csr* A, const msp_csr* B, float* features,
                                        float* targets) {
    if (!h) return fail(MSP_ERR_INVALID_ARG, "null handle");
    msp_status s = check_pair(A, B);
    if (s != MSP_OK) return s;
    const int m = (int)A->nrows;
    if (m > 0 && (!features || !targets)) return fail(MSP_ERR_INVALID_ARG, "null output");
    if ((s = msp_row_features(h, A, B, nullptr, features)) != MSP_OK) return s;
    int64_t tot = 0;
    DevBuf rn;
    if ((s = rn.ensure((size_t)std::max(m, 1) * 4)) != MSP_OK) return s;
    if ((s = msp_spgemm_symbolic(h, A, B, rn.as<int32_t>(), &tot, nullptr)) != MSP_OK) { rn.release(); return s; }
    if (m > 0) k_targets<<<(m + 255) / 256, 256, 0, h->stream>>>(m, rn.as<int32_t>(), targets);
    s = launch_check2("k_targets");
    hipError_t e = hipStreamSynchronize(h->stream);
    rn.release();
    if (s == MSP_OK && e != hipSuccess) s = hip_fail(e, "hipStreamSynchronize");
    return s;
}
