// Learned scheduling: features of K-block work units, a 4 -> 64 -> 64 -> 1
// FP32 MLP (forward, backward, Adam) and the binned launch order.
//
// The model only orders work: which units of a class launch are dispatched
// first (heaviest predicted first, a longest-processing-time list schedule).
// It never decides culling -- the Eq. (8) bound test in the class kernels
// does -- and K is bitwise independent of the order, because every K block
// is reduced in a fixed order inside its unit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fx_costmodel.h"
#include "fx_internal.h"

// ---------------------------------------------------------------------------
// features of (unit, class): f0 class cost log2(flops of one quartet), f1
// log2(nprim_a * nprim_d), f2 log10 of the unit's Schwarz row bound
// (max_b Qn_ab * max_c Qn_cd), f3 log2(1 + candidate entries of the unit)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void fx_k_unit_features(const int* __restrict__ units, const long* __restrict__ ulh,
                                                          const long* __restrict__ bc_off,
                                                          const long* __restrict__ cls_off, int seg,
                                                          const int* __restrict__ nprim,
                                                          const double* __restrict__ qrow, float class_cost,
                                                          float4* __restrict__ feat, const long* __restrict__ feat_off) {
    const long lo = ulh[0], n = ulh[1] - lo;
    float4* out = feat + (feat_off ? *feat_off : 0);
    for (long u = (long)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (long)gridDim.x * blockDim.x) {
        const int item = units[3 * (lo + u)], a = units[3 * (lo + u) + 1], d = units[3 * (lo + u) + 2];
        const long ne = cls_off ? (cls_off[(long)item * 10 + seg + 1] - cls_off[(long)item * 10 + seg])
                                : (bc_off[item + 1] - bc_off[item]);
        const double qb = qrow[a] * qrow[d];
        float4 f;
        f.x = class_cost;
        f.y = log2f((float)(nprim[a] * nprim[d]));
        f.z = (float)log10(qb > 1e-300 ? qb : 1e-300);
        f.w = log2f(1.0f + (float)ne);
        out[u] = f;
    }
}

static long fx_cm_grid(long n, int block) {
    long g = (n + block - 1) / block;
    if (g > 8192) g = 8192;
    return g < 1 ? 1 : g;
}

void fx_launch_unit_features(const int* units, const long* ulh, long n_max, const long* bc_off, const long* cls_off,
                             int seg, const int* nprim, const double* qrow, float class_cost, float4* feat,
                             const long* feat_off, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_unit_features, dim3(fx_cm_grid(n_max, 256)), dim3(256), 0, st, units, ulh, bc_off, cls_off,
                       seg, nprim, qrow, class_cost, feat, feat_off);
}

// bound-only estimate: log2(class flops) + log2(nprim_a nprim_d) + log2(1 + entries)
__global__ __launch_bounds__(256) void fx_k_bound_cost(const float4* __restrict__ feat, const long* __restrict__ ulh,
                                                       float* __restrict__ out) {
    const long n = ulh[1] - ulh[0];
    for (long u = (long)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (long)gridDim.x * blockDim.x) {
        const float4 f = feat[u];
        out[u] = f.x + f.y + f.w;
    }
}

void fx_launch_bound_cost(const float4* feat, const long* ulh, long n_max, float* out, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_bound_cost, dim3(fx_cm_grid(n_max, 256)), dim3(256), 0, st, feat, ulh, out);
}

// max_b Qn[s][b] for every shell s
__global__ void fx_k_qrow(const double* __restrict__ Qn, int S, double* __restrict__ qrow) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    double m = 0.0;
    for (int b = 0; b < S; ++b) m = fmax(m, Qn[(long)s * S + b]);
    qrow[s] = m;
}

void fx_launch_qrow(const double* Qn, int S, double* qrow, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_qrow, dim3((S + 255) / 256), dim3(256), 0, st, Qn, S, qrow);
}

// ---------------------------------------------------------------------------
// MLP: z1 = W1 x + b1, h1 = relu(z1); z2 = W2 h1 + b2, h2 = relu(z2);
// y = w3 . h2 + b3, on standardised inputs (x - mean) / std.
// Parameters packed in one FP32 vector (see fx_costmodel.h offsets).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void fx_mlp_forward(const float* __restrict__ W, const float* __restrict__ norm, float4 f,
                                               float* h1, float* h2, float& y) {
    const float x[4] = {(f.x - norm[0]) / norm[4], (f.y - norm[1]) / norm[5], (f.z - norm[2]) / norm[6],
                        (f.w - norm[3]) / norm[7]};
    for (int i = 0; i < FX_MLP_H; ++i) {
        float z = W[FX_MLP_B1 + i];
        for (int k = 0; k < FX_MLP_IN; ++k) z += W[FX_MLP_W1 + i * FX_MLP_IN + k] * x[k];
        h1[i] = z > 0.f ? z : 0.f;
    }
    for (int i = 0; i < FX_MLP_H; ++i) {
        float z = W[FX_MLP_B2 + i];
        for (int k = 0; k < FX_MLP_H; ++k) z += W[FX_MLP_W2 + i * FX_MLP_H + k] * h1[k];
        h2[i] = z > 0.f ? z : 0.f;
    }
    float o = W[FX_MLP_B3];
    for (int k = 0; k < FX_MLP_H; ++k) o += W[FX_MLP_W3 + k] * h2[k];
    y = o;
}

// prediction in target units: y * ystd + ymean; n = ulh[1] - ulh[0] when
// ulh is given, else n_host
__global__ __launch_bounds__(128) void fx_k_mlp_predict(const float* __restrict__ W, const float* __restrict__ norm,
                                                        const float4* __restrict__ feat, const long* __restrict__ ulh,
                                                        long n_host, float* __restrict__ out) {
    const long n = ulh ? ulh[1] - ulh[0] : n_host;
    for (long s = (long)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (long)gridDim.x * blockDim.x) {
        float h1[FX_MLP_H], h2[FX_MLP_H], y;
        fx_mlp_forward(W, norm, feat[s], h1, h2, y);
        out[s] = y * norm[9] + norm[8];
    }
}

void fx_launch_mlp_predict(const float* W, const float* norm, const float4* feat, const long* ulh, long n_max,
                           float* out, hipStream_t st) {
    if (n_max > 0)
        hipLaunchKernelGGL(fx_k_mlp_predict, dim3(fx_cm_grid(n_max, 128)), dim3(128), 0, st, W, norm, feat, ulh,
                           n_max, out);
}

// Per-sample forward and backward of the squared error on standardised
// targets: stores h1, h2 (64 each), dz2 (64), dz1 (64), dy, and the loss term.
__global__ void fx_k_mlp_backprop(const float* __restrict__ W, const float* __restrict__ norm,
                                  const float4* __restrict__ feat, const float* __restrict__ target,
                                  const int* __restrict__ idx, long n, float* __restrict__ act,
                                  float* __restrict__ loss) {
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const long j = idx ? idx[s] : s;
    float h1[FX_MLP_H], h2[FX_MLP_H], y;
    const float4 f = feat[j];
    fx_mlp_forward(W, norm, f, h1, h2, y);
    const float t = (target[j] - norm[8]) / norm[9];
    const float dy = 2.f * (y - t) / (float)n;   // d/dy of mean (y - t)^2
    float* a = act + s * FX_MLP_ACT;
    float dz2[FX_MLP_H];
    for (int i = 0; i < FX_MLP_H; ++i) {
        a[i] = h1[i];
        a[FX_MLP_H + i] = h2[i];
        dz2[i] = h2[i] > 0.f ? dy * W[FX_MLP_W3 + i] : 0.f;
        a[2 * FX_MLP_H + i] = dz2[i];
    }
    for (int k = 0; k < FX_MLP_H; ++k) {
        float g = 0.f;
        for (int i = 0; i < FX_MLP_H; ++i) g += W[FX_MLP_W2 + i * FX_MLP_H + k] * dz2[i];
        a[3 * FX_MLP_H + k] = h1[k] > 0.f ? g : 0.f;
    }
    a[4 * FX_MLP_H] = dy;
    const float x[4] = {(f.x - norm[0]) / norm[4], (f.y - norm[1]) / norm[5], (f.z - norm[2]) / norm[6],
                        (f.w - norm[3]) / norm[7]};
    for (int k = 0; k < 4; ++k) a[4 * FX_MLP_H + 1 + k] = x[k];
    loss[s] = (y - t) * (y - t) / (float)n;
}

// Gradient of every parameter: one thread per parameter, summing over the
// samples in index order (deterministic).
__global__ void fx_k_mlp_grad(const float* __restrict__ act, long n, float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= FX_MLP_NPARAM) return;
    float g = 0.f;
    if (p < FX_MLP_B1) {   // W1[i][k] : dz1_i * x_k
        const int i = p / FX_MLP_IN, k = p % FX_MLP_IN;
        for (long s = 0; s < n; ++s) g += act[s * FX_MLP_ACT + 3 * FX_MLP_H + i] * act[s * FX_MLP_ACT + 4 * FX_MLP_H + 1 + k];
    } else if (p < FX_MLP_W2) {   // b1
        const int i = p - FX_MLP_B1;
        for (long s = 0; s < n; ++s) g += act[s * FX_MLP_ACT + 3 * FX_MLP_H + i];
    } else if (p < FX_MLP_B2) {   // W2[i][k] : dz2_i * h1_k
        const int q = p - FX_MLP_W2, i = q / FX_MLP_H, k = q % FX_MLP_H;
        for (long s = 0; s < n; ++s) g += act[s * FX_MLP_ACT + 2 * FX_MLP_H + i] * act[s * FX_MLP_ACT + k];
    } else if (p < FX_MLP_W3) {   // b2
        const int i = p - FX_MLP_B2;
        for (long s = 0; s < n; ++s) g += act[s * FX_MLP_ACT + 2 * FX_MLP_H + i];
    } else if (p < FX_MLP_B3) {   // w3[k] : dy * h2_k
        const int k = p - FX_MLP_W3;
        for (long s = 0; s < n; ++s) g += act[s * FX_MLP_ACT + 4 * FX_MLP_H] * act[s * FX_MLP_ACT + FX_MLP_H + k];
    } else {   // b3
        for (long s = 0; s < n; ++s) g += act[s * FX_MLP_ACT + 4 * FX_MLP_H];
    }
    grad[p] = g;
}

__global__ void fx_k_sum_f32(const float* __restrict__ x, long n, float* __restrict__ out) {
    // single block, fixed order: thread t sums t, t+256, ...; then a fixed tree
    __shared__ float part[256];
    float s = 0.f;
    for (long i = threadIdx.x; i < n; i += 256) s += x[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0];
}

// Adam step t (1-based) on every parameter.
__global__ void fx_k_adam(float* __restrict__ W, const float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v, float lr, float b1, float b2, float eps, int t) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= FX_MLP_NPARAM) return;
    const float mi = b1 * m[p] + (1.f - b1) * g[p];
    const float vi = b2 * v[p] + (1.f - b2) * g[p] * g[p];
    m[p] = mi;
    v[p] = vi;
    const float mh = mi / (1.f - powf(b1, (float)t));
    const float vh = vi / (1.f - powf(b2, (float)t));
    W[p] -= lr * mh / (sqrtf(vh) + eps);
}

void fx_mlp_backprop_grad(const float* W, const float* norm, const float4* feat, const float* target, const int* idx,
                          long n, float* act, float* loss_terms, float* grad, float* loss, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_mlp_backprop, dim3((n + 127) / 128), dim3(128), 0, st, W, norm, feat, target, idx, n, act,
                       loss_terms);
    hipLaunchKernelGGL(fx_k_mlp_grad, dim3((FX_MLP_NPARAM + 63) / 64), dim3(64), 0, st, act, n, grad);
    hipLaunchKernelGGL(fx_k_sum_f32, dim3(1), dim3(256), 0, st, loss_terms, n, loss);
}

void fx_mlp_adam(float* W, const float* g, float* m, float* v, float lr, int t, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_adam, dim3((FX_MLP_NPARAM + 255) / 256), dim3(256), 0, st, W, g, m, v, lr, 0.9f, 0.999f,
                       1e-8f, t);
}

// ---------------------------------------------------------------------------
// Binned launch order: key = bin of the predicted log-cost (heaviest first),
// a stable counting sort.  bin_count: per block of 256 units the count of
// each bin (laid out bin-major, [bin][block]); one exclusive scan of the
// counts; bin_scatter: position = scanned count of (bin, block) + rank of
// the unit among the block's units of its bin (wave ballots).  Units keep
// their list order inside a bin.  The unit count is read on the device.
// ---------------------------------------------------------------------------
#define FX_BIN_BLOCK 256

__device__ __forceinline__ int fx_bin_of(float c, float top, float width, int nbins) {
    const float b = (top - c) / width;
    int k = b < 0.f ? 0 : (b >= (float)(nbins - 1) ? nbins - 1 : (int)b);
    if (!(c == c)) k = nbins - 1;   // NaN last
    return k;
}

__global__ __launch_bounds__(FX_BIN_BLOCK) void fx_k_bin_count(const float* __restrict__ cost,
                                                               const long* __restrict__ ulh, float top, float width,
                                                               int nbins, long nblk, uint8_t* __restrict__ key,
                                                               int* __restrict__ bcount) {
    __shared__ int h[64];
    const long n = ulh[1] - ulh[0];
    for (long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        if (threadIdx.x < 64) h[threadIdx.x] = 0;
        __syncthreads();
        const long u = blk * FX_BIN_BLOCK + threadIdx.x;
        if (u < n) {
            const int k = fx_bin_of(cost[u], top, width, nbins);
            key[u] = (uint8_t)k;
            atomicAdd(&h[k], 1);   // an integer count: independent of the order of the additions
        }
        __syncthreads();
        if ((int)threadIdx.x < nbins) bcount[(long)threadIdx.x * nblk + blk] = h[threadIdx.x];
        __syncthreads();
    }
}

__global__ __launch_bounds__(FX_BIN_BLOCK) void fx_k_bin_scatter(const uint8_t* __restrict__ key,
                                                                 const long* __restrict__ ulh, int nbins, long nblk,
                                                                 const long* __restrict__ bpos,
                                                                 int* __restrict__ order) {
    __shared__ int wc[FX_BIN_BLOCK / 64][64];
    const long n = ulh[1] - ulh[0];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long u = blk * FX_BIN_BLOCK + threadIdx.x;
        const int k = u < n ? (int)key[u] : -1;
        int rank = 0;
        for (int q = 0; q < nbins; ++q) {
            const uint64_t m = __ballot(k == q);
            if (k == q) rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if (lane == 0) wc[w][q] = __popcll(m);
        }
        __syncthreads();
        if (k >= 0) {
            long p = bpos[(long)k * nblk + blk] + rank;
            for (int v = 0; v < w; ++v) p += wc[v][k];
            order[p] = (int)u;
        }
        __syncthreads();
    }
}

long fx_bin_blocks(long n_max) { return (n_max + FX_BIN_BLOCK - 1) / FX_BIN_BLOCK; }

void fx_launch_bin_order(const float* cost, const long* ulh, long n_max, float top, float width, int nbins,
                         uint8_t* key, int* bcount, long* bpos, long* partial, long* total, int* order, hipStream_t st,
                         void (*scan)(const int*, long, long*, long*, long*, hipStream_t)) {
    const long nblk = fx_bin_blocks(n_max);
    if (nblk <= 0) return;
    const long g = nblk < 8192 ? nblk : 8192;
    hipLaunchKernelGGL(fx_k_bin_count, dim3(g), dim3(FX_BIN_BLOCK), 0, st, cost, ulh, top, width, nbins, nblk, key,
                       bcount);
    scan(bcount, (long)nbins * nblk, bpos, partial, total, st);
    hipLaunchKernelGGL(fx_k_bin_scatter, dim3(g), dim3(FX_BIN_BLOCK), 0, st, key, ulh, nbins, nblk, bpos, order);
}
