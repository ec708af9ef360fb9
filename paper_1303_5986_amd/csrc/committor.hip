// committor.hip -- a learned progress coordinate for binning (gfx950).
//
// The paper bins on hand-chosen coordinates and names optimal, automatic
// binning an open problem (Sec. IV.B).  This module learns a committor
// q(x) ~ P(reach B before A | x) from the WE trajectories themselves and bins
// on it; WE stays unbiased for any binning (Sec. II.B), so a poor model only
// costs efficiency.
//
//  1. records: after every iteration the resampled ensemble (states, parent
//     slots, and whether the parent reached B in that interval) is copied to
//     a record buffer in HBM;
//  2. labels (reverse pass over the records, one launch per iteration):
//     every walker adds to its parent the first outcome of each child --
//     B if the child's parent was recycled in that interval, A if the child
//     sits in the A region, otherwise the child's own counts.  Integer
//     atomics, so the counts are exact and order-free.  Label
//     y = n_B / (n_A + n_B) for walkers with a resolved descendant;
//  3. dataset: resolved walkers compacted in record order (block counts,
//     one scan, in-block ballot ranks);
//  4. features: phi_s = (log1p(x_s) - mean_s) / std_s, statistics reduced in
//     a fixed order per species;
//  5. model: n_in -> 64 -> 64 -> 1, tanh, tanh, sigmoid, FP32; loss: binary
//     cross-entropy with the soft label; Adam (beta 0.9/0.999, eps 1e-8).
//     Forward/backward is one wave per sample; each parameter's gradient is
//     summed over the minibatch by one wave in a fixed order (lane-strided
//     partial sums, then a butterfly), so a training run is reproducible;
//  6. bins: n_bins equal-count quantile edges over the dataset, taken on
//     the logit z = log(q/(1-q)) (quantiles do not change under a monotone
//     map, and the logit resolves the q ~ 1e-10 values near A that FP32 q
//     cannot); a 65536-cell integer histogram over z in [-40, 40]; with the
//     committor active every walker's bin is bin_index(edges, z(x)) after
//     recycling.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "we_internal.h"

#define CM_H 64
#define Q_HIST 65536

// ------------------------------------------------------------------ layout
__host__ __device__ inline int32_t cm_n_params(int32_t n_in) {
    return CM_H * n_in + CM_H + CM_H * CM_H + CM_H + CM_H + 1;
}
struct ParamView {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
};
__host__ __device__ inline ParamView cm_view(const float *p, int32_t n_in) {
    ParamView v;
    v.W1 = p;
    v.b1 = v.W1 + CM_H * n_in;
    v.W2 = v.b1 + CM_H;
    v.b2 = v.W2 + CM_H * CM_H;
    v.W3 = v.b2 + CM_H;
    v.b3 = v.W3 + CM_H;
    return v;
}

__device__ __forceinline__ float feature(int32_t x, const float *feat, int32_t k, int32_t n_in) {
    return (log1pf((float)x) - feat[k]) * feat[n_in + k];
}

// logit z(x) of the committor, q = 1 / (1 + e^-z); phi recomputed on the fly.
__device__ float mlp_z(const ParamView &P, const float *feat, const int32_t *xr, int32_t n_in) {
    float h1[CM_H];
#pragma unroll
    for (int j = 0; j < CM_H; ++j) h1[j] = P.b1[j];
    for (int k = 0; k < n_in; ++k) {
        const float f = feature(xr[k], feat, k, n_in);
#pragma unroll
        for (int j = 0; j < CM_H; ++j) h1[j] = fmaf(P.W1[j * n_in + k], f, h1[j]);
    }
#pragma unroll
    for (int j = 0; j < CM_H; ++j) h1[j] = tanhf(h1[j]);
    float z3 = P.b3[0];
    for (int i = 0; i < CM_H; ++i) {
        float z = P.b2[i];
#pragma unroll
        for (int j = 0; j < CM_H; ++j) z = fmaf(P.W2[i * CM_H + j], h1[j], z);
        z3 = fmaf(P.W3[i], tanhf(z), z3);
    }
    return z3;
}

// Orders the LDS accesses of the lanes of one wave.
__device__ __forceinline__ void cm_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Quantile histogram cell of a logit: 65536 cells over [-Z_SPAN, Z_SPAN].
#define Z_SPAN 40.0f
__device__ __forceinline__ int32_t z_cell(float z) {
    int32_t c = (int32_t)((z + Z_SPAN) * ((float)Q_HIST / (2.0f * Z_SPAN)));
    return c < 0 ? 0 : (c >= Q_HIST ? Q_HIST - 1 : c);
}

// ------------------------------------------------------------------ records
__global__ __launch_bounds__(256) void cm_record_kernel(SimArgs a, const int32_t *__restrict__ x_nxt,
                                                        int32_t *__restrict__ rx, int32_t *__restrict__ rorig,
                                                        uint8_t *__restrict__ rrec, int32_t *__restrict__ rn) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t run = (int32_t)(gid / a.cap);
    const int32_t k = (int32_t)(gid - (int64_t)run * a.cap);
    if (run >= a.n_runs) return;
    const int32_t n = a.n_walk[run];
    if (k == 0) rn[run] = n;
    if (k >= n) return;
    const size_t idx = (size_t)run * a.cap + k;
    const int32_t o = a.origin[idx];
    rorig[idx] = o;
    rrec[idx] = (uint8_t)(a.s_rec[(size_t)run * a.cap + o] != 0);
    for (int32_t s = 0; s < a.S; ++s) rx[idx * a.S + s] = x_nxt[idx * a.S + s];
}

hipError_t committor_record(we_sim *s, hipStream_t st) {
    Records &R = s->rec;
    if (R.cap_iters <= 0 || R.n_iters >= R.cap_iters) return hipSuccess;
    const size_t W = (size_t)s->n_runs * s->cap;
    const int32_t i = R.n_iters;
    const int64_t total = (int64_t)W;
    hipLaunchKernelGGL(cm_record_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       s->args, s->x[s->cur], R.d_x + i * W * s->S, R.d_origin + i * W, R.d_rec + i * W,
                       R.d_n + (size_t)i * s->n_runs);
    R.n_iters += 1;
    return hipGetLastError();
}

// ------------------------------------------------------------------ labels
__global__ __launch_bounds__(256) void cm_label_kernel(int32_t n_runs, int32_t cap, int32_t S,
                                                       const int32_t *__restrict__ x_child,
                                                       const int32_t *__restrict__ orig_child,
                                                       const uint8_t *__restrict__ rec_child,
                                                       const int32_t *__restrict__ n_child,
                                                       const uint32_t *__restrict__ cnt_child,
                                                       uint32_t *__restrict__ cnt_parent,
                                                       const double *__restrict__ a_coef, double a_thr) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t run = (int32_t)(gid / cap);
    const int32_t k = (int32_t)(gid - (int64_t)run * cap);
    if (run >= n_runs) return;
    if (k >= n_child[run]) return;
    const size_t idx = (size_t)run * cap + k;
    uint32_t nA, nB;
    if (rec_child[idx]) {
        nA = 0; nB = 1;
    } else {
        double q = 0.0;
        for (int32_t s = 0; s < S; ++s) q = q + a_coef[s] * (double)x_child[idx * S + s];
        if (q <= a_thr) { nA = 1; nB = 0; }
        else { nA = cnt_child[2 * idx]; nB = cnt_child[2 * idx + 1]; }
    }
    const int32_t p = orig_child[idx];
    if (p < 0 || p >= cap) return;
    const size_t pidx = (size_t)run * cap + p;
    if (nA) atomicAdd(&cnt_parent[2 * pidx], nA);
    if (nB) atomicAdd(&cnt_parent[2 * pidx + 1], nB);
}

// ------------------------------------------------------------------ dataset
__global__ __launch_bounds__(256) void cm_count_kernel(int64_t n_items, int32_t n_runs, int32_t cap,
                                                       const int32_t *__restrict__ rn,
                                                       const uint32_t *__restrict__ cnt,
                                                       int32_t *__restrict__ blk) {
    __shared__ int32_t part[256];
    const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int32_t v = 0;
    if (f < n_items) {
        const int64_t W = (int64_t)n_runs * cap;
        const int64_t i = f / W;
        const int32_t run = (int32_t)((f - i * W) / cap);
        const int32_t k = (int32_t)(f - i * W - (int64_t)run * cap);
        v = (k < rn[i * n_runs + run]) && (cnt[2 * f] + cnt[2 * f + 1] > 0);
    }
    part[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t c = 0;
        for (int t = 0; t < 256; ++t) c += part[t];
        blk[blockIdx.x] = c;
    }
}

__global__ void cm_scan_kernel(int32_t n_blk, int32_t *__restrict__ blk, int32_t *__restrict__ total) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int32_t acc = 0;
    for (int32_t b = 0; b < n_blk; ++b) {
        const int32_t c = blk[b];
        blk[b] = acc;
        acc += c;
    }
    *total = acc;
}

__global__ __launch_bounds__(256) void cm_compact_kernel(int64_t n_items, int32_t n_runs, int32_t cap,
                                                         const int32_t *__restrict__ rn,
                                                         const uint32_t *__restrict__ cnt,
                                                         const int32_t *__restrict__ blk,
                                                         int64_t *__restrict__ ds_idx,
                                                         float *__restrict__ ds_y, int32_t ds_cap) {
    __shared__ int32_t part[256];
    const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int32_t v = 0;
    if (f < n_items) {
        const int64_t W = (int64_t)n_runs * cap;
        const int64_t i = f / W;
        const int32_t run = (int32_t)((f - i * W) / cap);
        const int32_t k = (int32_t)(f - i * W - (int64_t)run * cap);
        v = (k < rn[i * n_runs + run]) && (cnt[2 * f] + cnt[2 * f + 1] > 0);
    }
    part[threadIdx.x] = v;
    __syncthreads();
    if (!v) return;
    int32_t rank = 0;
    for (int t = 0; t < (int)threadIdx.x; ++t) rank += part[t];
    const int32_t pos = blk[blockIdx.x] + rank;
    if (pos >= ds_cap) return;
    ds_idx[pos] = f;
    const float nA = (float)cnt[2 * f], nB = (float)cnt[2 * f + 1];
    ds_y[pos] = nB / (nA + nB);
}

// per-species mean and 1/std of log1p(x) over the dataset (FP64, fixed order)
__global__ __launch_bounds__(256) void cm_feat_kernel(int32_t n, int32_t S, const int64_t *__restrict__ ds_idx,
                                                      const int32_t *__restrict__ rx, float *__restrict__ feat) {
    __shared__ double s1[256], s2[256];
    const int32_t sp = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int32_t i = threadIdx.x; i < n; i += 256) {
        const double v = log1p((double)rx[ds_idx[i] * S + sp]);
        a += v;
        b += v * v;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            s1[threadIdx.x] += s1[threadIdx.x + off];
            s2[threadIdx.x] += s2[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mean = n > 0 ? s1[0] / n : 0.0;
        const double var = n > 0 ? s2[0] / n - mean * mean : 0.0;
        const double sd = var > 1e-12 ? sqrt(var) : 1.0;
        feat[sp] = (float)mean;
        feat[S + sp] = (float)(1.0 / sd);
    }
}

// ------------------------------------------------------------------ training
// Glorot-uniform weights from Philox (counter (index, 0, 0, 2)), zero biases.
__global__ void cm_init_kernel(float *__restrict__ p, int32_t n_in, uint32_t k0, uint32_t k1) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t np = cm_n_params(n_in);
    if (i >= np) return;
    const int32_t nW1 = CM_H * n_in, nW2 = CM_H * CM_H;
    const int32_t b1 = nW1, w2 = b1 + CM_H, b2 = w2 + nW2, w3 = b2 + CM_H, b3 = w3 + CM_H;
    float limit = 0.0f;
    if (i < b1) limit = sqrtf(6.0f / (float)(n_in + CM_H));
    else if (i >= w2 && i < b2) limit = sqrtf(6.0f / (float)(CM_H + CM_H));
    else if (i >= w3 && i < b3) limit = sqrtf(6.0f / (float)(CM_H + 1));
    const U4 r = philox4x32_10((uint32_t)i, 0u, 0u, 2u, k0, k1);
    const float u = (float)uniform53(r.x, r.y);
    p[i] = limit * (2.0f * u - 1.0f);
}

struct Scratch {
    float *phi, *h1, *h2, *g1, *g2, *g3, *loss;   // [feature][B] layout
};

// Forward and backward of one sample per wave, one hidden unit per lane;
// the sample is either drawn from the dataset with Philox (counter
// (b, step, 1, 2)) or given directly.  Every dot product runs over its inputs
// in ascending order, on the lane that owns the output.
inline size_t cm_fwd_bwd_lds(int32_t n_in) { return 4 * sizeof(float) * ((size_t)n_in + 3 * CM_H); }

__global__ __launch_bounds__(256) void cm_fwd_bwd_kernel(const float *__restrict__ params, const float *__restrict__ feat,
                                                         int32_t n_in, int32_t B, int32_t step,
                                                         uint32_t k0, uint32_t k1, int32_t n_ds,
                                                         const int64_t *__restrict__ ds_idx,
                                                         const float *__restrict__ ds_y,
                                                         const int32_t *__restrict__ rx,
                                                         const int32_t *__restrict__ direct_x,
                                                         const float *__restrict__ direct_y, Scratch sc) {
    extern __shared__ float cm_lds[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int32_t b = (int32_t)blockIdx.x * 4 + wv;
    if (b >= B) return;   // uniform over the wave
    float *lphi = cm_lds + (size_t)wv * (n_in + 3 * CM_H);
    float *lh1 = lphi + n_in, *lh2 = lh1 + CM_H, *lg2 = lh2 + CM_H;
    const ParamView P = cm_view(params, n_in);
    const int32_t *xr;
    float y;
    if (direct_x) {
        xr = direct_x + (size_t)b * n_in;
        y = direct_y[b];
    } else {
        const U4 r = philox4x32_10((uint32_t)b, (uint32_t)step, 1u, 2u, k0, k1);
        int32_t pick = (int32_t)(uniform53(r.x, r.y) * (double)n_ds);
        if (pick >= n_ds) pick = n_ds - 1;
        xr = rx + ds_idx[pick] * n_in;
        y = ds_y[pick];
    }
    for (int32_t k = lane; k < n_in; k += 64) {
        const float f = feature(xr[k], feat, k, n_in);
        lphi[k] = f;
        sc.phi[(size_t)k * B + b] = f;
    }
    cm_wave_sync();
    const int j = lane;   // this lane's hidden unit in both layers
    float z1 = P.b1[j];
    for (int32_t k = 0; k < n_in; ++k) z1 = fmaf(P.W1[j * n_in + k], lphi[k], z1);
    const float h1 = tanhf(z1);
    lh1[j] = h1;
    sc.h1[(size_t)j * B + b] = h1;
    cm_wave_sync();
    float z2 = P.b2[j];
    for (int i = 0; i < CM_H; ++i) z2 = fmaf(P.W2[j * CM_H + i], lh1[i], z2);
    const float h2 = tanhf(z2);
    lh2[j] = h2;
    sc.h2[(size_t)j * B + b] = h2;
    cm_wave_sync();
    float z3 = P.b3[0];
    for (int i = 0; i < CM_H; ++i) z3 = fmaf(P.W3[i], lh2[i], z3);
    const float q = 1.0f / (1.0f + expf(-z3));
    const float g3 = (q - y) / (float)B;
    if (lane == 0) {
        // binary cross-entropy with a soft label, in the stable form
        sc.loss[b] = fmaxf(z3, 0.0f) - z3 * y + log1pf(expf(-fabsf(z3)));
        sc.g3[b] = g3;
    }
    const float g2 = g3 * P.W3[j] * (1.0f - h2 * h2);
    lg2[j] = g2;
    sc.g2[(size_t)j * B + b] = g2;
    cm_wave_sync();
    float acc = 0.0f;
    for (int i = 0; i < CM_H; ++i) acc = fmaf(P.W2[i * CM_H + j], lg2[i], acc);
    sc.g1[(size_t)j * B + b] = acc * (1.0f - h1 * h1);
}

// One wave per parameter (and one for the mean loss): lane l sums samples
// l, l+64, l+128, ... in that order, then a fixed butterfly adds the 64 lane
// sums -- coalesced loads, and the same order on every run.
__global__ __launch_bounds__(256) void cm_grad_kernel(int32_t n_in, int32_t B, Scratch sc, float *__restrict__ grad,
                                                      float *__restrict__ loss_out) {
    const int32_t i = (int32_t)blockIdx.x * 4 + (int32_t)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int32_t np = cm_n_params(n_in);
    if (i > np || (i == np && !loss_out)) return;   // uniform over the wave
    const int32_t nW1 = CM_H * n_in, nW2 = CM_H * CM_H;
    const int32_t b1 = nW1, w2 = b1 + CM_H, b2 = w2 + nW2, w3 = b2 + CM_H, b3 = w3 + CM_H;
    const float *u, *v = nullptr;
    if (i == np) { u = sc.loss; }
    else if (i < b1) { u = sc.g1 + (size_t)(i / n_in) * B; v = sc.phi + (size_t)(i % n_in) * B; }
    else if (i < w2) { u = sc.g1 + (size_t)(i - b1) * B; }
    else if (i < b2) { const int32_t r = i - w2; u = sc.g2 + (size_t)(r / CM_H) * B; v = sc.h1 + (size_t)(r % CM_H) * B; }
    else if (i < w3) { u = sc.g2 + (size_t)(i - b2) * B; }
    else if (i < b3) { u = sc.g3; v = sc.h2 + (size_t)(i - w3) * B; }
    else { u = sc.g3; }
    float acc = 0.0f;
    if (v) for (int32_t b = lane; b < B; b += 64) acc = fmaf(u[b], v[b], acc);
    else for (int32_t b = lane; b < B; b += 64) acc += u[b];
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if (lane == 0) {
        if (i == np) *loss_out = acc / (float)B;
        else grad[i] = acc;
    }
}

__global__ void cm_adam_kernel(int32_t np, float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                               const float *__restrict__ g, float lr, int32_t t) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - powf(b1, (float)t));
    const float vh = vi / (1.0f - powf(b2, (float)t));
    p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// ------------------------------------------------------------------ inference
__global__ __launch_bounds__(256) void cm_eval_kernel(const float *__restrict__ params, const float *__restrict__ feat,
                                                      int32_t n_in, int32_t n, const int64_t *__restrict__ ds_idx,
                                                      const int32_t *__restrict__ rx, float *__restrict__ q_out,
                                                      uint32_t *__restrict__ qhist) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const ParamView P = cm_view(params, n_in);
    const int32_t *xr = ds_idx ? rx + ds_idx[i] * n_in : rx + (size_t)i * n_in;
    const float z = mlp_z(P, feat, xr, n_in);
    if (q_out) q_out[i] = 1.0f / (1.0f + expf(-z));
    if (qhist) atomicAdd(&qhist[z_cell(z)], 1u);
}

// Equal-count edges in logit space: edge b is the upper end of the cell where
// the cumulative count first reaches b*n/nb; edges stay strictly increasing.
// One block of 1024 threads: thread t owns cells [64t, 64t+64); a block scan
// of the threads' totals gives each its starting count, each thread marks
// the edges (or quantile cells) its cells reach first, and thread 0 writes
// the edges in order (the nudges of edges sharing a cell are sequential).
#define CM_EDGE_THREADS 1024
#define CM_EDGE_MAX_BINS 8192
__global__ __launch_bounds__(CM_EDGE_THREADS) void cm_edges_kernel(const uint32_t *__restrict__ qhist, int32_t n,
                                                                  int32_t nb, double *__restrict__ edges,
                                                                  int32_t mode) {
    constexpr int32_t PER = Q_HIST / CM_EDGE_THREADS;
    __shared__ int64_t part[CM_EDGE_THREADS];
    __shared__ int32_t cellof[CM_EDGE_MAX_BINS];
    __shared__ int32_t q_lo, q_hi;
    const int32_t t = threadIdx.x;
    int64_t own = 0;
    for (int32_t i = 0; i < PER; ++i) own += qhist[t * PER + i];
    part[t] = own;
    if (t == 0) {
        q_lo = -1;
        q_hi = -1;
    }
    for (int32_t b = t; b < CM_EDGE_MAX_BINS; b += CM_EDGE_THREADS) cellof[b] = -1;   // not reached
    __syncthreads();
    for (int32_t d = 1; d < CM_EDGE_THREADS; d <<= 1) {     // inclusive scan of the totals
        const int64_t v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t cum = part[t] - own;
    const int64_t N = n > 0 ? (int64_t)n : 1;
    for (int32_t i = 0; i < PER; ++i) {
        const int32_t c = t * PER + i;
        const int64_t prev = cum;
        cum += qhist[c];
        if (cum == prev) continue;
        if (mode == 1) {
            if (prev * 200 < N && cum * 200 >= N) q_lo = c;
            if (prev * 200 < N * 199 && cum * 200 >= N * 199) q_hi = c;
        } else {
            // edges b with prev*nb < b*n <= cum*nb start in this cell
            const int64_t b_from = prev * nb / N + 1, b_to = cum * nb / N;
            for (int64_t b = b_from < 1 ? 1 : b_from; b <= b_to && b < nb; ++b) cellof[b] = c;
        }
    }
    __syncthreads();
    if (t != 0) return;
    const double cell = 2.0 * (double)Z_SPAN / (double)Q_HIST;
    const double nudge = cell / 64.0;
    edges[0] = -(double)Z_SPAN;
    if (mode == 1) {
        // uniform in the logit between the 0.5% and 99.5% quantiles of the data
        const double zlo = q_lo >= 0 ? -(double)Z_SPAN + q_lo * cell : -(double)Z_SPAN;
        double zhi = q_hi >= 0 ? -(double)Z_SPAN + (q_hi + 1) * cell : (double)Z_SPAN;
        if (!(zhi > zlo)) zhi = zlo + cell;
        for (int32_t b = 1; b < nb; ++b) edges[b] = zlo + (zhi - zlo) * (double)b / (double)nb;
        edges[nb] = edges[nb - 1] + (double)Z_SPAN;
        return;
    }
    for (int32_t b = 1; b < nb; ++b) {
        double e = cellof[b] >= 0 ? -(double)Z_SPAN + (double)(cellof[b] + 1) * cell : edges[b - 1];
        if (e <= edges[b - 1]) e = edges[b - 1] + nudge;
        edges[b] = e;
    }
    edges[nb] = edges[nb - 1] + (double)Z_SPAN;
}

// W1 and W2 transposed, so the lanes of a wave (one hidden unit each) read
// consecutive words: wt[k*64 + j] = W1[j][k], wt[64*n_in + i*64 + j] = W2[j][i].
__global__ void cm_transpose_kernel(const float *__restrict__ params, int32_t n_in, float *__restrict__ wt) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t n1 = CM_H * n_in;
    const ParamView P = cm_view(params, n_in);
    if (t < n1) {
        const int32_t k = t / CM_H, j = t % CM_H;
        wt[t] = P.W1[j * n_in + k];
    } else if (t < n1 + CM_H * CM_H) {
        const int32_t u = t - n1, i = u / CM_H, j = u % CM_H;
        wt[t] = P.W2[j * CM_H + i];
    }
}

// The same z as mlp_z (every dot product over the same terms in the same
// order, on the lane that owns its output), one walker per wave, one hidden
// unit per lane; wt is cm_transpose_kernel's output; lphi/lh1/lh2 are the
// wave's LDS slices (n_in, 64, 64 floats).
__device__ float mlp_z_wave(const ParamView &P, const float *__restrict__ wt, const float *feat, const int32_t *xr,
                            int32_t n_in, float *lphi, float *lh1, float *lh2) {
    const int lane = threadIdx.x & 63;
    const float *W1t = wt, *W2t = wt + CM_H * n_in;
    for (int32_t k = lane; k < n_in; k += 64) lphi[k] = feature(xr[k], feat, k, n_in);
    cm_wave_sync();
    float z1 = P.b1[lane];
    for (int32_t k = 0; k < n_in; ++k) z1 = fmaf(W1t[k * CM_H + lane], lphi[k], z1);
    lh1[lane] = tanhf(z1);
    cm_wave_sync();
    float z2 = P.b2[lane];
    for (int j = 0; j < CM_H; ++j) z2 = fmaf(W2t[j * CM_H + lane], lh1[j], z2);
    lh2[lane] = tanhf(z2);
    cm_wave_sync();
    float z3 = P.b3[0];
    for (int i = 0; i < CM_H; ++i) z3 = fmaf(P.W3[i], lh2[i], z3);
    cm_wave_sync();
    return z3;
}

// Learned bins after recycling: one wave per walker slot.
__global__ __launch_bounds__(256) void cm_bin_kernel(SimArgs a, const int32_t *__restrict__ x_cur,
                                                     const float *__restrict__ params, const float *__restrict__ wt,
                                                     const float *__restrict__ feat,
                                                     const double *__restrict__ qedges) {
    extern __shared__ float cm_lds[];
    const int wv = threadIdx.x >> 6;
    const int64_t gid = (int64_t)blockIdx.x * 4 + wv;
    const int32_t run = (int32_t)(gid / a.cap);
    const int32_t k = (int32_t)(gid - (int64_t)run * a.cap);
    if (run >= a.n_runs) return;          // uniform over the wave
    if (k >= a.n_walk[run]) return;
    const size_t idx = (size_t)run * a.cap + k;
    float *lphi = cm_lds + (size_t)wv * (a.S + 2 * CM_H);
    const ParamView P = cm_view(params, a.S);
    const float z = mlp_z_wave(P, wt, feat, x_cur + idx * a.S, a.S, lphi, lphi + a.S, lphi + a.S + CM_H);
    if ((threadIdx.x & 63) == 0) a.s_bin[idx] = bin_index(qedges, a.n_bins, (double)z);
}

hipError_t committor_bin(we_sim *s, int32_t *x_cur, hipStream_t st) {
    const int64_t total = (int64_t)s->n_runs * s->cap;
    const size_t lds = 4 * sizeof(float) * ((size_t)s->S + 2 * CM_H);
    hipLaunchKernelGGL(cm_bin_kernel, dim3((unsigned)((total + 3) / 4)), dim3(256), lds, st, s->args, x_cur,
                       s->cm.d_params, s->cm.d_wt, s->cm.d_feat, s->cm.d_qedges);
    return hipGetLastError();
}

// Learned bins of every batch member whose committor is active, after the
// batched recycle/bin: grid (CM_BATCH_BLOCKS, members), one wave per walker
// slot as in cm_bin_kernel, each wave striding over its member's slots (a
// grid sized for the largest member would spend most of its workgroups on
// members with no slots left for them); members without a model (params
// NULL) return at once.
#define CM_BATCH_BLOCKS 256
__global__ __launch_bounds__(256) void cm_batch_bin_kernel(const SimArgs *__restrict__ args,
                                                           int32_t *const *__restrict__ x_cur,
                                                           const CmBatchModel *__restrict__ models,
                                                           int32_t s_lds) {
    extern __shared__ float cm_lds[];
    const int32_t i = blockIdx.y;
    const CmBatchModel m = models[i];
    if (!m.params) return;
    const SimArgs &a = args[i];
    const int wv = threadIdx.x >> 6;
    float *lphi = cm_lds + (size_t)wv * (s_lds + 2 * CM_H);
    const ParamView P = cm_view(m.params, a.S);
    const int64_t slots = (int64_t)a.n_runs * a.cap;
    for (int64_t gid = (int64_t)blockIdx.x * 4 + wv; gid < slots; gid += (int64_t)gridDim.x * 4) {
        const int32_t run = (int32_t)(gid / a.cap);   // uniform over the wave
        const int32_t k = (int32_t)(gid - (int64_t)run * a.cap);
        if (k >= a.n_walk[run]) continue;
        const size_t idx = (size_t)run * a.cap + k;
        const float z =
            mlp_z_wave(P, m.wt, m.feat, x_cur[i] + idx * a.S, a.S, lphi, lphi + s_lds, lphi + s_lds + CM_H);
        if ((threadIdx.x & 63) == 0) a.s_bin[idx] = bin_index(m.qedges, a.n_bins, (double)z);
    }
}

CmBatchModel committor_batch_model(const we_sim *s) {
    CmBatchModel m{};
    if (s->cm.active) {
        m.params = s->cm.d_params;
        m.wt = s->cm.d_wt;
        m.feat = s->cm.d_feat;
        m.qedges = s->cm.d_qedges;
    }
    return m;
}

hipError_t committor_bin_batch(const SimArgs *d_args, int32_t *const *d_x, const CmBatchModel *d_models,
                               int32_t n_sims, int64_t max_slots, int32_t s_max, hipStream_t st) {
    const size_t lds = 4 * sizeof(float) * ((size_t)s_max + 2 * CM_H);
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((max_slots + 3) / 4, CM_BATCH_BLOCKS));
    hipLaunchKernelGGL(cm_batch_bin_kernel, dim3(gx, (unsigned)n_sims), dim3(256), lds, st, d_args, d_x, d_models,
                       s_max);
    return hipGetLastError();
}

void committor_free(we_sim *s) {
    Committor &c = s->cm;
    (void)hipFree(c.d_params);
    (void)hipFree(c.d_adam_m);
    (void)hipFree(c.d_adam_v);
    (void)hipFree(c.d_grad);
    (void)hipFree(c.d_feat);
    (void)hipFree(c.d_qedges);
    (void)hipFree(c.d_wt);
    c = Committor();
}

// The trained model as host arrays, and back (checkpoints).
we_status committor_export(we_sim *s, CommittorHost &h) {
    const Committor &C = s->cm;
    h = CommittorHost();
    h.trained = C.trained;
    h.active = C.active;
    if (!C.trained) return WE_OK;
    h.n_in = C.n_in;
    h.n_qbins = C.n_qbins;
    const size_t np = (size_t)C.n_params, nwt = (size_t)CM_H * C.n_in + (size_t)CM_H * CM_H;
    h.params.resize(np);
    h.adam_m.resize(np);
    h.adam_v.resize(np);
    h.feat.resize(2 * (size_t)C.n_in);
    h.qedges.resize((size_t)C.n_qbins + 1);
    h.wt.resize(nwt);
    HIP_TRY(hipMemcpyAsync(h.params.data(), C.d_params, 4 * np, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(h.adam_m.data(), C.d_adam_m, 4 * np, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(h.adam_v.data(), C.d_adam_v, 4 * np, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(h.feat.data(), C.d_feat, 8 * (size_t)C.n_in, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(h.qedges.data(), C.d_qedges, 8 * h.qedges.size(), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(h.wt.data(), C.d_wt, 4 * nwt, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return WE_OK;
}

we_status committor_import(we_sim *s, const CommittorHost &h) {
    committor_free(s);
    if (!h.trained) return WE_OK;
    if (h.n_in != s->S || h.n_qbins != s->NB) return we_fail(WE_EINVAL, "checkpoint committor does not fit the sim");
    Committor &C = s->cm;
    C.n_in = h.n_in;
    C.n_params = cm_n_params(h.n_in);
    C.n_qbins = h.n_qbins;
    const size_t np = (size_t)C.n_params, nwt = (size_t)CM_H * C.n_in + (size_t)CM_H * CM_H;
    if (h.params.size() != np || h.adam_m.size() != np || h.adam_v.size() != np ||
        h.feat.size() != 2 * (size_t)C.n_in || h.qedges.size() != (size_t)C.n_qbins + 1 || h.wt.size() != nwt)
        return we_fail(WE_EINVAL, "checkpoint committor arrays have the wrong sizes");
    HIP_TRY(hipMalloc(&C.d_params, 4 * np));
    HIP_TRY(hipMalloc(&C.d_adam_m, 4 * np));
    HIP_TRY(hipMalloc(&C.d_adam_v, 4 * np));
    HIP_TRY(hipMalloc(&C.d_grad, 4 * np));
    HIP_TRY(hipMalloc(&C.d_feat, 8 * (size_t)C.n_in));
    HIP_TRY(hipMalloc(&C.d_qedges, 8 * h.qedges.size()));
    HIP_TRY(hipMalloc(&C.d_wt, 4 * nwt));
    HIP_TRY(hipMemcpyAsync(C.d_params, h.params.data(), 4 * np, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(C.d_adam_m, h.adam_m.data(), 4 * np, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(C.d_adam_v, h.adam_v.data(), 4 * np, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemsetAsync(C.d_grad, 0, 4 * np, s->stream));
    HIP_TRY(hipMemcpyAsync(C.d_feat, h.feat.data(), 8 * (size_t)C.n_in, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(C.d_qedges, h.qedges.data(), 8 * h.qedges.size(), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(C.d_wt, h.wt.data(), 4 * nwt, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    C.trained = true;
    C.active = h.active;
    return WE_OK;
}

// ------------------------------------------------------------------ C ABI
namespace {

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    hipError_t alloc(size_t bytes) { return hipMalloc(&p, std::max<size_t>(bytes, 16)); }
    template <class T> T *as() { return static_cast<T *>(p); }
};

struct ScratchBufs {
    DevBuf phi, h1, h2, g1, g2, g3, loss;
    hipError_t alloc(int32_t n_in, int32_t B) {
        hipError_t e;
        if ((e = phi.alloc(4ull * n_in * B)) != hipSuccess) return e;
        if ((e = h1.alloc(4ull * CM_H * B)) != hipSuccess) return e;
        if ((e = h2.alloc(4ull * CM_H * B)) != hipSuccess) return e;
        if ((e = g1.alloc(4ull * CM_H * B)) != hipSuccess) return e;
        if ((e = g2.alloc(4ull * CM_H * B)) != hipSuccess) return e;
        if ((e = g3.alloc(4ull * B)) != hipSuccess) return e;
        return loss.alloc(4ull * B);
    }
    Scratch view() {
        return Scratch{phi.as<float>(), h1.as<float>(), h2.as<float>(), g1.as<float>(), g2.as<float>(),
                       g3.as<float>(), loss.as<float>()};
    }
};

// record-buffer counts of outcomes, [n_iters][n_runs*cap][2]
we_status run_labels(we_sim *s, const double *a_coef_h, double a_thr, DevBuf &cnt) {
    Records &R = s->rec;
    const size_t W = (size_t)s->n_runs * s->cap;
    HIP_TRY(cnt.alloc(8 * W * std::max(R.n_iters, 1)));
    HIP_TRY(hipMemsetAsync(cnt.p, 0, 8 * W * std::max(R.n_iters, 1), s->stream));
    DevBuf coef;
    HIP_TRY(coef.alloc(8 * (size_t)s->S));
    HIP_TRY(hipMemcpyAsync(coef.p, a_coef_h, 8 * (size_t)s->S, hipMemcpyHostToDevice, s->stream));
    uint32_t *c = cnt.as<uint32_t>();
    for (int32_t i = R.n_iters - 1; i >= 1; --i) {
        hipLaunchKernelGGL(cm_label_kernel, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, s->stream, s->n_runs,
                           s->cap, s->S, R.d_x + i * W * s->S, R.d_origin + i * W, R.d_rec + i * W,
                           R.d_n + (size_t)i * s->n_runs, c + 2 * i * W, c + 2 * (i - 1) * W, coef.as<double>(),
                           a_thr);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    return WE_OK;
}

}  // namespace

extern "C" we_status we_record_labels(we_sim *s, const double *a_coef, double a_thr, uint32_t *counts,
                                      int32_t *n_iters) {
    if (!s || !a_coef) return we_fail(WE_EINVAL, "NULL argument");
    if (s->rec.cap_iters <= 0) return we_fail(WE_ESTATE, "no records were requested at init");
    DevBuf cnt;
    we_status st = run_labels(s, a_coef, a_thr, cnt);
    if (st != WE_OK) return st;
    const size_t W = (size_t)s->n_runs * s->cap;
    if (counts) HIP_TRY(hipMemcpy(counts, cnt.p, 8 * W * s->rec.n_iters, hipMemcpyDeviceToHost));
    if (n_iters) *n_iters = s->rec.n_iters;
    return WE_OK;
}

extern "C" we_status we_get_record(we_sim *s, int32_t i, int32_t *n, int32_t *x, int32_t *origin,
                                   uint8_t *recycled) {
    if (!s) return we_fail(WE_EINVAL, "NULL sim");
    if (i < 0 || i >= s->rec.n_iters) return we_fail(WE_EINVAL, "record index out of range");
    HIP_TRY(hipStreamSynchronize(s->stream));
    const size_t W = (size_t)s->n_runs * s->cap;
    if (n) HIP_TRY(hipMemcpy(n, s->rec.d_n + (size_t)i * s->n_runs, 4 * (size_t)s->n_runs, hipMemcpyDeviceToHost));
    if (x) HIP_TRY(hipMemcpy(x, s->rec.d_x + i * W * s->S, 4 * W * s->S, hipMemcpyDeviceToHost));
    if (origin) HIP_TRY(hipMemcpy(origin, s->rec.d_origin + i * W, 4 * W, hipMemcpyDeviceToHost));
    if (recycled) HIP_TRY(hipMemcpy(recycled, s->rec.d_rec + i * W, W, hipMemcpyDeviceToHost));
    return WE_OK;
}

extern "C" we_status we_train_committor(we_sim *s, const we_train_params *tp, float *loss_out,
                                        int32_t *n_samples) {
    if (!s || !tp || !tp->a_coef) return we_fail(WE_EINVAL, "NULL argument");
    if (s->rec.cap_iters <= 0 || s->rec.n_iters < 2) return we_fail(WE_ESTATE, "need at least two recorded iterations");
    if (tp->steps < 0 || tp->batch <= 0 || tp->batch % 256 || !(tp->lr > 0.0f))
        return we_fail(WE_EINVAL, "steps >= 0, batch a positive multiple of 256, lr > 0");
    if (tp->edge_mode < 0 || tp->edge_mode > 1) return we_fail(WE_EINVAL, "edge_mode must be 0 or 1");
    const int32_t n_in = s->S;
    if (n_in > 1024) return we_fail(WE_EINVAL, "committor supports up to 1024 species");
    Records &R = s->rec;
    const size_t W = (size_t)s->n_runs * s->cap;
    DevBuf cnt;
    we_status st = run_labels(s, tp->a_coef, tp->a_thr, cnt);
    if (st != WE_OK) return st;

    // dataset: resolved walkers, in record order
    const int64_t n_items = (int64_t)R.n_iters * (int64_t)W;
    const int32_t n_blk = (int32_t)((n_items + 255) / 256);
    DevBuf blk, total, ds_idx, ds_y;
    HIP_TRY(blk.alloc(4ull * n_blk));
    HIP_TRY(total.alloc(4));
    hipLaunchKernelGGL(cm_count_kernel, dim3(n_blk), dim3(256), 0, s->stream, n_items, s->n_runs, s->cap, R.d_n,
                       cnt.as<uint32_t>(), blk.as<int32_t>());
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(cm_scan_kernel, dim3(1), dim3(64), 0, s->stream, n_blk, blk.as<int32_t>(), total.as<int32_t>());
    HIP_TRY(hipGetLastError());
    int32_t n_ds = 0;
    HIP_TRY(hipMemcpyAsync(&n_ds, total.p, 4, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (n_ds < 1) return we_fail(WE_ESTATE, "no recorded walker has a resolved outcome yet");
    HIP_TRY(ds_idx.alloc(8ull * n_ds));
    HIP_TRY(ds_y.alloc(4ull * n_ds));
    hipLaunchKernelGGL(cm_compact_kernel, dim3(n_blk), dim3(256), 0, s->stream, n_items, s->n_runs, s->cap, R.d_n,
                       cnt.as<uint32_t>(), blk.as<int32_t>(), ds_idx.as<int64_t>(), ds_y.as<float>(), n_ds);
    HIP_TRY(hipGetLastError());

    // model buffers
    Committor &C = s->cm;
    committor_free(s);
    C.n_in = n_in;
    C.n_params = cm_n_params(n_in);
    C.n_qbins = s->NB;
    const size_t pb = 4ull * C.n_params;
    HIP_TRY(hipMalloc(&C.d_params, pb));
    HIP_TRY(hipMalloc(&C.d_adam_m, pb));
    HIP_TRY(hipMalloc(&C.d_adam_v, pb));
    HIP_TRY(hipMalloc(&C.d_grad, pb));
    HIP_TRY(hipMalloc(&C.d_feat, 8ull * n_in));
    HIP_TRY(hipMalloc(&C.d_qedges, 8ull * (C.n_qbins + 1)));
    HIP_TRY(hipMalloc(&C.d_wt, 4ull * (CM_H * n_in + CM_H * CM_H)));
    HIP_TRY(hipMemsetAsync(C.d_adam_m, 0, pb, s->stream));
    HIP_TRY(hipMemsetAsync(C.d_adam_v, 0, pb, s->stream));
    const uint32_t k0 = (uint32_t)tp->seed, k1 = (uint32_t)(tp->seed >> 32);
    hipLaunchKernelGGL(cm_init_kernel, dim3((C.n_params + 255) / 256), dim3(256), 0, s->stream, C.d_params, n_in, k0, k1);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(cm_feat_kernel, dim3(n_in), dim3(256), 0, s->stream, n_ds, n_in, ds_idx.as<int64_t>(), R.d_x,
                       C.d_feat);
    HIP_TRY(hipGetLastError());

    // Adam steps
    const int32_t B = tp->batch;
    ScratchBufs sb;
    HIP_TRY(sb.alloc(n_in, B));
    DevBuf dloss;
    HIP_TRY(dloss.alloc(4ull * std::max(tp->steps, 1)));
    for (int32_t step = 0; step < tp->steps; ++step) {
        hipLaunchKernelGGL(cm_fwd_bwd_kernel, dim3((B + 3) / 4), dim3(256), cm_fwd_bwd_lds(n_in), s->stream,
                           C.d_params, C.d_feat, n_in, B,
                           step, k0, k1, n_ds, ds_idx.as<int64_t>(), ds_y.as<float>(), R.d_x,
                           (const int32_t *)nullptr, (const float *)nullptr, sb.view());
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(cm_grad_kernel, dim3((C.n_params + 1 + 3) / 4), dim3(256), 0, s->stream, n_in, B,
                           sb.view(), C.d_grad, dloss.as<float>() + step);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(cm_adam_kernel, dim3((C.n_params + 255) / 256), dim3(256), 0, s->stream, C.n_params,
                           C.d_params, C.d_adam_m, C.d_adam_v, C.d_grad, tp->lr, step + 1);
        HIP_TRY(hipGetLastError());
    }

    const int32_t nt = CM_H * n_in + CM_H * CM_H;
    hipLaunchKernelGGL(cm_transpose_kernel, dim3((nt + 255) / 256), dim3(256), 0, s->stream, C.d_params, n_in, C.d_wt);
    HIP_TRY(hipGetLastError());

    // equal-count quantile edges of q over the dataset
    DevBuf qhist;
    HIP_TRY(qhist.alloc(4ull * Q_HIST));
    HIP_TRY(hipMemsetAsync(qhist.p, 0, 4ull * Q_HIST, s->stream));
    hipLaunchKernelGGL(cm_eval_kernel, dim3((n_ds + 255) / 256), dim3(256), 0, s->stream, C.d_params, C.d_feat, n_in,
                       n_ds, ds_idx.as<int64_t>(), R.d_x, (float *)nullptr, qhist.as<uint32_t>());
    HIP_TRY(hipGetLastError());
    if (C.n_qbins > CM_EDGE_MAX_BINS) return we_fail(WE_EINVAL, "at most 8192 learned bins");
    hipLaunchKernelGGL(cm_edges_kernel, dim3(1), dim3(CM_EDGE_THREADS), 0, s->stream, qhist.as<uint32_t>(), n_ds,
                       C.n_qbins, C.d_qedges, tp->edge_mode);
    HIP_TRY(hipGetLastError());
    if (loss_out && tp->steps > 0)
        HIP_TRY(hipMemcpyAsync(loss_out, dloss.p, 4ull * tp->steps, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    C.trained = true;
    if (n_samples) *n_samples = n_ds;
    return WE_OK;
}

extern "C" we_status we_use_committor_bins(we_sim *s, int32_t enable) {
    if (!s) return we_fail(WE_EINVAL, "NULL sim");
    if (enable && !s->cm.trained) return we_fail(WE_ESTATE, "no trained committor");
    if (enable && s->args.rw_period > 0)
        return we_fail(WE_EINVAL, "reweighting needs fixed grid bins, not learned ones");
    if (s->graph_exec) return we_fail(WE_ESTATE, "recapture the graph after switching bins");
    s->cm.active = enable != 0;
    return WE_OK;
}

// Caller-given logit edges for the learned bins (we_set_bins).
we_status committor_set_edges(we_sim *s, const double *edges) {
    if (!s->cm.trained) return we_fail(WE_ESTATE, "no trained committor");
    const int32_t nb = s->cm.n_qbins;
    for (int32_t b = 1; b + 1 < nb; ++b)
        if (!(edges[b] < edges[b + 1])) return we_fail(WE_EINVAL, "inner logit edges must increase strictly");
    for (int32_t b = 0; b <= nb; ++b)
        if (!std::isfinite(edges[b])) return we_fail(WE_EINVAL, "logit edges must be finite");
    HIP_TRY(hipMemcpyAsync(s->cm.d_qedges, edges, 8ull * (nb + 1), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return WE_OK;
}

extern "C" we_status we_committor_eval(we_sim *s, int32_t n, const int32_t *x, float *q) {
    if (!s || (n > 0 && (!x || !q))) return we_fail(WE_EINVAL, "NULL argument");
    if (!s->cm.trained) return we_fail(WE_ESTATE, "no trained committor");
    DevBuf dx, dq;
    HIP_TRY(dx.alloc(4ull * n * s->S));
    HIP_TRY(dq.alloc(4ull * n));
    HIP_TRY(hipMemcpyAsync(dx.p, x, 4ull * n * s->S, hipMemcpyHostToDevice, s->stream));
    hipLaunchKernelGGL(cm_eval_kernel, dim3((n + 255) / 256), dim3(256), 0, s->stream, s->cm.d_params, s->cm.d_feat,
                       s->S, n, (const int64_t *)nullptr, dx.as<int32_t>(), dq.as<float>(), (uint32_t *)nullptr);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(q, dq.p, 4ull * n, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return WE_OK;
}

extern "C" we_status we_committor_state(we_sim *s, float *params, float *feat, double *qedges, int32_t *n_params) {
    if (!s) return we_fail(WE_EINVAL, "NULL sim");
    if (!s->cm.trained) return we_fail(WE_ESTATE, "no trained committor");
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (n_params) *n_params = s->cm.n_params;
    if (params) HIP_TRY(hipMemcpy(params, s->cm.d_params, 4ull * s->cm.n_params, hipMemcpyDeviceToHost));
    if (feat) HIP_TRY(hipMemcpy(feat, s->cm.d_feat, 8ull * s->cm.n_in, hipMemcpyDeviceToHost));
    if (qedges) HIP_TRY(hipMemcpy(qedges, s->cm.d_qedges, 8ull * (s->cm.n_qbins + 1), hipMemcpyDeviceToHost));
    return WE_OK;
}

extern "C" we_status we_mlp_loss_grad(int32_t n_in, const float *params, const float *feat, int32_t batch,
                                      const int32_t *x, const float *y, float *loss, float *grad) {
    if (n_in < 1 || n_in > 1024 || batch < 1 || !params || !feat || !x || !y)
        return we_fail(WE_EINVAL, "bad arguments");
    const int32_t np = cm_n_params(n_in);
    DevBuf dp, df, dx, dy, dg, dl;
    HIP_TRY(dp.alloc(4ull * np));
    HIP_TRY(df.alloc(8ull * n_in));
    HIP_TRY(dx.alloc(4ull * batch * n_in));
    HIP_TRY(dy.alloc(4ull * batch));
    HIP_TRY(dg.alloc(4ull * np));
    HIP_TRY(dl.alloc(4));
    HIP_TRY(hipMemcpy(dp.p, params, 4ull * np, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(df.p, feat, 8ull * n_in, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dx.p, x, 4ull * batch * n_in, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dy.p, y, 4ull * batch, hipMemcpyHostToDevice));
    ScratchBufs sb;
    HIP_TRY(sb.alloc(n_in, batch));
    hipLaunchKernelGGL(cm_fwd_bwd_kernel, dim3((batch + 3) / 4), dim3(256), cm_fwd_bwd_lds(n_in), nullptr, dp.as<float>(),
                       df.as<float>(), n_in, batch, 0, 0u, 0u, 0, (const int64_t *)nullptr, (const float *)nullptr,
                       (const int32_t *)nullptr, dx.as<int32_t>(), dy.as<float>(), sb.view());
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(cm_grad_kernel, dim3((np + 1 + 3) / 4), dim3(256), 0, nullptr, n_in, batch, sb.view(),
                       dg.as<float>(), dl.as<float>());
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipDeviceSynchronize());
    if (grad) HIP_TRY(hipMemcpy(grad, dg.p, 4ull * np, hipMemcpyDeviceToHost));
    if (loss) HIP_TRY(hipMemcpy(loss, dl.p, 4, hipMemcpyDeviceToHost));
    return WE_OK;
}

// ------------------------------------------------- allocation-free loss/gradient
// Fixed device scratch of we_mlp_loss_grad_noalloc: the per-sample features,
// activations and deltas ([feature][batch] layout) of one minibatch.  Each
// GPU holds its own copy for the life of the process.  Host code must never
// pass `scratch` itself to a kernel (in host code the name is a host-side
// stand-in, not a device address): it uses the per-device address looked up
// once with hipGetSymbolAddress.
static __device__ __align__(256) float scratch[WE_MLP_NOALLOC_FLOATS];

namespace {
std::mutex g_scratch_mu;
float *g_scratch_dev[WE_MAX_DEVICES] = {};

// The current device's address of `scratch`, looked up on the first call
// made with that device current.
we_status scratch_address(float **out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= WE_MAX_DEVICES) return we_fail(WE_EDEVICE, "device index beyond WE_MAX_DEVICES");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return we_fail(WE_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_dev[dev] = static_cast<float *>(p);
    }
    *out = g_scratch_dev[dev];
    return WE_OK;
}
}  // namespace

extern "C" we_status we_mlp_loss_grad_noalloc(int32_t n_in, const float *params, const float *feat, int32_t batch,
                                              const int32_t *x, const float *y, float *loss, float *grad,
                                              void *hip_stream) {
    if (n_in < 1 || n_in > 1024 || batch < 1 || !params || !feat || !x || !y || !loss || !grad)
        return we_fail(WE_EINVAL, "bad arguments");
    const size_t need = (size_t)batch * ((size_t)n_in + 4 * CM_H + 2);
    if (need > (size_t)WE_MLP_NOALLOC_FLOATS)
        return we_fail(WE_ECAPACITY, "batch * (n_in + 258) exceeds the fixed scratch of WE_MLP_NOALLOC_FLOATS floats");
    float *base = nullptr;
    we_status st = scratch_address(&base);
    if (st != WE_OK) return st;
    const size_t B = (size_t)batch;
    Scratch sc;
    sc.phi = base;
    sc.h1 = sc.phi + (size_t)n_in * B;
    sc.h2 = sc.h1 + CM_H * B;
    sc.g1 = sc.h2 + CM_H * B;
    sc.g2 = sc.g1 + CM_H * B;
    sc.g3 = sc.g2 + CM_H * B;
    sc.loss = sc.g3 + B;
    hipStream_t st_h = static_cast<hipStream_t>(hip_stream);
    const int32_t np = cm_n_params(n_in);
    hipLaunchKernelGGL(cm_fwd_bwd_kernel, dim3((batch + 3) / 4), dim3(256), cm_fwd_bwd_lds(n_in), st_h, params, feat,
                       n_in, batch, 0, 0u, 0u, 0, (const int64_t *)nullptr, (const float *)nullptr,
                       (const int32_t *)nullptr, x, y, sc);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(cm_grad_kernel, dim3((np + 1 + 3) / 4), dim3(256), 0, st_h, n_in, batch, sc, grad, loss);
    HIP_TRY(hipGetLastError());
    return WE_OK;
}

extern "C" we_status we_adam_step(int32_t n, float *params, float *m, float *v, const float *grad, float lr,
                                  int32_t t) {
    if (n < 1 || !params || !m || !v || !grad || t < 1) return we_fail(WE_EINVAL, "bad arguments");
    DevBuf dp, dm, dv, dg;
    HIP_TRY(dp.alloc(4ull * n));
    HIP_TRY(dm.alloc(4ull * n));
    HIP_TRY(dv.alloc(4ull * n));
    HIP_TRY(dg.alloc(4ull * n));
    HIP_TRY(hipMemcpy(dp.p, params, 4ull * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dm.p, m, 4ull * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dv.p, v, 4ull * n, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dg.p, grad, 4ull * n, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(cm_adam_kernel, dim3((n + 255) / 256), dim3(256), 0, nullptr, n, dp.as<float>(), dm.as<float>(),
                       dv.as<float>(), dg.as<float>(), lr, t);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(params, dp.p, 4ull * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(m, dm.p, 4ull * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(v, dv.p, 4ull * n, hipMemcpyDeviceToHost));
    return WE_OK;
}
