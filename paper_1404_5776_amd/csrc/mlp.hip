// Learned starting guess for the truncated Hotelling inverse: a two-layer
// perceptron (tanh hidden layer of width H) maps the descriptor of an
// atom-pair block,
//     d = [ (r_i - r_j)/R, |r_i - r_j|/R, S_ij (b*b entries) ],
// to a correction of the first-order start 2 delta_ij I - S_ij of that block.
// Weights are used in FP16 with FP32 accumulation; training keeps FP32 master
// weights and updates them with Adam.  All reductions over samples are
// deterministic (fixed partition, fixed order).
#include <hip/hip_fp16.h>

#include <cmath>

#include "internal.h"

namespace rtdm {

constexpr int kMlpT = 128;   // threads per workgroup (= hidden width)

// ---------------------------------------------------------------- descriptors

// One thread per (sample, feature).  blk[s] is the position of the sample's
// block (i, j) in S's pattern.
__global__ void k_mlp_desc(int64_t n, int b, const int32_t *__restrict__ blk,
                           const int32_t *__restrict__ rowof, const int32_t *__restrict__ col,
                           const double *__restrict__ xyz, const double *__restrict__ sv, double inv_r,
                           float *__restrict__ desc)
{
    const int in = 4 + b * b;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * in) return;
    const int64_t s = e / in;
    const int f = (int)(e - s * in);
    const int p = blk[s];
    const int i = rowof[p], j = col[p];
    float v;
    if (f < 3) {
        v = (float)((xyz[3 * i + f] - xyz[3 * j + f]) * inv_r);
    } else if (f == 3) {
        const double dx = xyz[3 * i] - xyz[3 * j], dy = xyz[3 * i + 1] - xyz[3 * j + 1],
                     dz = xyz[3 * i + 2] - xyz[3 * j + 2];
        v = (float)(sqrt(dx * dx + dy * dy + dz * dz) * inv_r);
    } else {
        v = (float)sv[(int64_t)p * b * b + (f - 4)];
    }
    desc[e] = v;
}

void launch_mlp_desc(hipStream_t s, int64_t n, int b, const int32_t *blk, const int32_t *rowof,
                     const int32_t *col, const double *xyz, const double *sv, double inv_r, float *desc)
{
    const int64_t tot = n * (4 + b * b);
    if (tot == 0) return;
    hipLaunchKernelGGL(k_mlp_desc, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, b, blk, rowof,
                       col, xyz, sv, inv_r, desc);
    RT_HIP(hipGetLastError());
}

// Target correction: X_ij - (2 delta_ij I - S_ij) for sample block p of S's
// pattern; x_of[s] is the position of the same pair in X's pattern.
__global__ void k_mlp_target(int64_t n, int b, const int32_t *__restrict__ blk,
                             const int32_t *__restrict__ x_of, const int32_t *__restrict__ rowof,
                             const int32_t *__restrict__ col, const double *__restrict__ sv,
                             const double *__restrict__ xv, float *__restrict__ tgt)
{
    const int bb = b * b;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * bb) return;
    const int64_t s = e / bb;
    const int w = (int)(e - s * bb);
    const int p = blk[s];
    const double diag = (rowof[p] == col[p] && w % (b + 1) == 0) ? 2.0 : 0.0;
    const double start = diag - sv[(int64_t)p * bb + w];
    tgt[e] = (float)(xv[(int64_t)x_of[s] * bb + w] - start);
}

void launch_mlp_target(hipStream_t s, int64_t n, int b, const int32_t *blk, const int32_t *x_of,
                       const int32_t *rowof, const int32_t *col, const double *sv, const double *xv,
                       float *tgt)
{
    const int64_t tot = n * b * b;
    if (tot == 0) return;
    hipLaunchKernelGGL(k_mlp_target, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, b, blk, x_of,
                       rowof, col, sv, xv, tgt);
    RT_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- forward

// One workgroup of H = 128 threads per sample: thread h forms hidden unit h,
// then threads o < out form the outputs.  hid (pre-activation tanh output) is
// kept for the backward pass when non-null.
__global__ __launch_bounds__(kMlpT) void k_mlp_forward(int64_t n, int in, int out,
                                                       const int32_t *__restrict__ idx,
                                                       const float *__restrict__ x,
                                                       const __half *__restrict__ w1,
                                                       const float *__restrict__ b1,
                                                       const __half *__restrict__ w2,
                                                       const float *__restrict__ b2,
                                                       float *__restrict__ hid, float *__restrict__ y)
{
    __shared__ float xs[512];
    __shared__ float hs[kMlpT];
    const int64_t s = blockIdx.x;
    if (s >= n) return;
    const int64_t src = idx ? idx[s] : s;
    const int t = threadIdx.x;
    for (int f = t; f < in; f += kMlpT) xs[f] = x[src * in + f];
    __syncthreads();
    float a = b1[t];
    for (int f = 0; f < in; ++f) a += __half2float(w1[(int64_t)t * in + f]) * xs[f];
    const float h = tanhf(a);
    hs[t] = h;
    if (hid) hid[s * kMlpT + t] = h;
    __syncthreads();
    for (int o = t; o < out; o += kMlpT) {
        float v = b2[o];
        for (int k = 0; k < kMlpT; ++k) v += __half2float(w2[(int64_t)o * kMlpT + k]) * hs[k];
        y[s * out + o] = v;
    }
}

void launch_mlp_forward(hipStream_t s, int64_t n, int in, int out, const int32_t *idx, const float *x,
                        const __half *w1, const float *b1, const __half *w2, const float *b2, float *hid,
                        float *y)
{
    RT_CHECK(in <= 512, RTDM_E_UNSUPPORTED, "descriptor longer than 512");
    if (n == 0) return;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)n), dim3(kMlpT), 0, s, n, in, out, idx, x, w1, b1, w2,
                       b2, hid, y);
    RT_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- backward

// Per sample: dy = 2 (y - t) / (n * out) (gradient of the mean squared error),
// dh = (W2^T dy) * (1 - h^2).  Also the per-sample squared error sum.
__global__ __launch_bounds__(kMlpT) void k_mlp_delta(int64_t n, int out, const int32_t *__restrict__ idx,
                                                     const float *__restrict__ tgt,
                                                     const float *__restrict__ y,
                                                     const float *__restrict__ hid,
                                                     const __half *__restrict__ w2,
                                                     float *__restrict__ dy, float *__restrict__ dh,
                                                     float *__restrict__ sqerr)
{
    __shared__ float ds[512];
    __shared__ float red[kMlpT];
    const int64_t s = blockIdx.x;
    if (s >= n) return;
    const int64_t src = idx ? idx[s] : s;
    const int t = threadIdx.x;
    const float scale = 2.0f / ((float)n * (float)out);
    float e2 = 0.0f;
    for (int o = t; o < out; o += kMlpT) {
        const float d = y[s * out + o] - tgt[src * out + o];
        e2 += d * d;
        ds[o] = scale * d;
        dy[s * out + o] = scale * d;
    }
    red[t] = e2;
    __syncthreads();
    for (int w = kMlpT / 2; w >= 1; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) sqerr[s] = red[0];
    float g = 0.0f;
    for (int o = 0; o < out; ++o) g += __half2float(w2[(int64_t)o * kMlpT + t]) * ds[o];
    const float h = hid[s * kMlpT + t];
    dh[s * kMlpT + t] = g * (1.0f - h * h);
}

void launch_mlp_delta(hipStream_t s, int64_t n, int out, const int32_t *idx, const float *tgt, const float *y,
                      const float *hid, const __half *w2, float *dy, float *dh, float *sqerr)
{
    RT_CHECK(out <= 512, RTDM_E_UNSUPPORTED, "output longer than 512");
    if (n == 0) return;
    hipLaunchKernelGGL(k_mlp_delta, dim3((unsigned)n), dim3(kMlpT), 0, s, n, out, idx, tgt, y, hid, w2, dy, dh,
                       sqerr);
    RT_HIP(hipGetLastError());
}

// Parameter gradients as sums over samples, in a fixed order:
//   dW1[h][f] = sum_s dh[s][h] x[s][f],  db1[h] = sum_s dh[s][h],
//   dW2[o][h] = sum_s dy[s][o] hid[s][h], db2[o] = sum_s dy[s][o].
// Parameters are laid out W1 (H x in), b1 (H), W2 (out x H), b2 (out).  One
// thread per parameter loops over every sample (n is a mini-batch).
__global__ void k_mlp_grad(int64_t n, int in, int out, const int32_t *__restrict__ idx,
                           const float *__restrict__ x, const float *__restrict__ hid,
                           const float *__restrict__ dy, const float *__restrict__ dh,
                           float *__restrict__ grad)
{
    const int64_t np = (int64_t)kMlpT * in + kMlpT + (int64_t)out * kMlpT + out;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    float acc = 0.0f;
    if (p < (int64_t)kMlpT * in) {
        const int h = (int)(p / in), f = (int)(p % in);
        for (int64_t s = 0; s < n; ++s) {
            const int64_t src = idx ? idx[s] : s;
            acc += dh[s * kMlpT + h] * x[src * in + f];
        }
    } else if (p < (int64_t)kMlpT * in + kMlpT) {
        const int h = (int)(p - (int64_t)kMlpT * in);
        for (int64_t s = 0; s < n; ++s) acc += dh[s * kMlpT + h];
    } else if (p < (int64_t)kMlpT * in + kMlpT + (int64_t)out * kMlpT) {
        const int64_t q = p - ((int64_t)kMlpT * in + kMlpT);
        const int o = (int)(q / kMlpT), h = (int)(q % kMlpT);
        for (int64_t s = 0; s < n; ++s) acc += dy[s * out + o] * hid[s * kMlpT + h];
    } else {
        const int o = (int)(p - ((int64_t)kMlpT * in + kMlpT + (int64_t)out * kMlpT));
        for (int64_t s = 0; s < n; ++s) acc += dy[s * out + o];
    }
    grad[p] = acc;
}

void launch_mlp_grad(hipStream_t s, int64_t n, int in, int out, const int32_t *idx, const float *x,
                     const float *hid, const float *dy, const float *dh, float *grad)
{
    const int64_t np = (int64_t)kMlpT * in + kMlpT + (int64_t)out * kMlpT + out;
    hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, n, in, out, idx, x, hid,
                       dy, dh, grad);
    RT_HIP(hipGetLastError());
}

// Adam (Kingma & Ba 2015) on the FP32 master weights, then the FP16 copies
// used by the forward pass.  t is the 1-based step count.
// omb1 = 1 - beta1, omb2 = 1 - beta2, c1 = 1 - beta1^t, c2 = 1 - beta2^t are
// formed in double on the host and rounded once (1 - 0.999f^t in single
// precision would lose three digits to cancellation).
__global__ void k_adam(int64_t np, int64_t nw1, int64_t nb1, int64_t nw2, const float *__restrict__ grad,
                       float *__restrict__ w, float *__restrict__ m, float *__restrict__ v, float lr,
                       float beta1, float beta2, float omb1, float omb2, float eps, float c1, float c2,
                       __half *__restrict__ w1h, __half *__restrict__ w2h)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const float g = grad[p];
    const float mi = beta1 * m[p] + omb1 * g;
    const float vi = beta2 * v[p] + omb2 * g * g;
    m[p] = mi;
    v[p] = vi;
    const float wi = w[p] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[p] = wi;
    if (p < nw1) w1h[p] = __float2half(wi);
    else if (p >= nw1 + nb1 && p < nw1 + nb1 + nw2) w2h[p - nw1 - nb1] = __float2half(wi);
}

void launch_adam(hipStream_t s, int64_t np, int64_t nw1, int64_t nb1, int64_t nw2, const float *grad, float *w,
                 float *m, float *v, float lr, double beta1, double beta2, float eps, int step, __half *w1h,
                 __half *w2h)
{
    const double b1 = beta1, b2 = beta2;
    const float c1 = (float)(1.0 - std::pow(b1, step)), c2 = (float)(1.0 - std::pow(b2, step));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, np, nw1, nb1, nw2, grad, w,
                       m, v, lr, (float)beta1, (float)beta2, (float)(1.0 - b1), (float)(1.0 - b2), eps, c1, c2, w1h, w2h);
    RT_HIP(hipGetLastError());
}

__global__ void k_to_half(int64_t n, const float *__restrict__ x, __half *__restrict__ y)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) y[e] = __float2half(x[e]);
}

void launch_to_half(hipStream_t s, int64_t n, const float *x, __half *y)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_to_half, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, x, y);
    RT_HIP(hipGetLastError());
}

// X0 block p of X's pattern = (2 delta I - S_ij) + y[s] for the predicted
// blocks (x_of[s] = p), written into a zeroed X.
__global__ void k_mlp_apply(int64_t n, int b, const int32_t *__restrict__ blk, const int32_t *__restrict__ x_of,
                            const int32_t *__restrict__ rowof, const int32_t *__restrict__ col,
                            const double *__restrict__ sv, const float *__restrict__ y,
                            double *__restrict__ xv)
{
    const int bb = b * b;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * bb) return;
    const int64_t s = e / bb;
    const int w = (int)(e - s * bb);
    const int p = blk[s];
    const double diag = (rowof[p] == col[p] && w % (b + 1) == 0) ? 2.0 : 0.0;
    xv[(int64_t)x_of[s] * bb + w] = diag - sv[(int64_t)p * bb + w] + (double)y[e];
}

void launch_mlp_apply(hipStream_t s, int64_t n, int b, const int32_t *blk, const int32_t *x_of,
                      const int32_t *rowof, const int32_t *col, const double *sv, const float *y, double *xv)
{
    const int64_t tot = n * b * b;
    if (tot == 0) return;
    hipLaunchKernelGGL(k_mlp_apply, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, b, blk, x_of, rowof,
                       col, sv, y, xv);
    RT_HIP(hipGetLastError());
}

// Deterministic sum of n floats (fixed tree in one workgroup).
__global__ __launch_bounds__(256) void k_sum_f32(int64_t n, const float *__restrict__ x, double *__restrict__ out)
{
    __shared__ double sh[256];
    double a = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += 256) a += (double)x[e];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

void launch_sum_f32(hipStream_t s, int64_t n, const float *x, double *out)
{
    hipLaunchKernelGGL(k_sum_f32, dim3(1), dim3(256), 0, s, n, x, out);
    RT_HIP(hipGetLastError());
}

}  // namespace rtdm
