// Training kernels of the learned search range: a 2-layer perceptron
// F -> H (ReLU) -> T trained with a weighted mean squared error and Adam,
// all in f32.  Gradient sums over the batch use a fixed reduction order, so
// results are deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "pred_inputs.h"
#include "onng_internal.h"

namespace onng {

namespace {

// one thread per sample: hidden activations, outputs and, when target is
// given, dL/dy and dL/dh (the per-sample pieces of the gradient)
__global__ void mlp_sample_kernel(const float *X, int batch, int F, const float *W1,
                                  const float *b1, int H, const float *W2, const float *b2, int T,
                                  const float *target, const float *w, float *hid, float *Y,
                                  float *dy, float *dh, float *lossp) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= batch) return;
    const float *x = X + (int64_t)n * F;
    float h[64], a[64];
    for (int j = 0; j < H; j++) {
        float s = b1[j];
        for (int i = 0; i < F; i++) s = fmaf(W1[j * F + i], x[i], s);
        a[j] = s;
        h[j] = fmaxf(s, 0.0f);
        if (hid) hid[(int64_t)n * H + j] = h[j];
    }
    float g[16];
    float l = 0.0f;
    const float scale = 1.0f / ((float)batch * (float)T);
    for (int t = 0; t < T; t++) {
        float y = b2[t];
        for (int j = 0; j < H; j++) y = fmaf(W2[t * H + j], h[j], y);
        if (Y) Y[(int64_t)n * T + t] = y;
        if (target) {
            float wt = w ? w[(int64_t)n * T + t] : 1.0f;
            float e = y - target[(int64_t)n * T + t];
            l += wt * e * e;
            g[t] = 2.0f * wt * e * scale;
            dy[(int64_t)n * T + t] = g[t];
        }
    }
    if (!target) return;
    lossp[n] = l * scale;
    for (int j = 0; j < H; j++) {
        float s = 0.0f;
        for (int t = 0; t < T; t++) s = fmaf(W2[t * H + j], g[t], s);
        dh[(int64_t)n * H + j] = a[j] > 0.0f ? s : 0.0f;
    }
}

// one block per parameter: sum over the batch of the per-sample product
//   kind 0: gW1[j][i] = sum_n dh[n][j] x[n][i]      (p = j*F + i)
//   kind 1: gb1[j]    = sum_n dh[n][j]
//   kind 2: gW2[t][j] = sum_n dy[n][t] h[n][j]      (p = t*H + j)
//   kind 3: gb2[t]    = sum_n dy[n][t]
//   kind 4: loss      = sum_n lossp[n]
__global__ void __launch_bounds__(256) mlp_reduce_kernel(const float *X, int batch, int F, int H,
                                                         int T, const float *hid, const float *dy,
                                                         const float *dh, const float *lossp,
                                                         float *gW1, float *gb1, float *gW2,
                                                         float *gb2, float *loss) {
    __shared__ float red[256];
    int p = blockIdx.x;
    int kind, i0 = 0, i1 = 0;
    int nW1 = H * F, nW2 = T * H;
    if (p < nW1) { kind = 0; i0 = p / F; i1 = p % F; }
    else if ((p -= nW1) < H) { kind = 1; i0 = p; }
    else if ((p -= H) < nW2) { kind = 2; i0 = p / H; i1 = p % H; }
    else if ((p -= nW2) < T) { kind = 3; i0 = p; }
    else kind = 4;
    float s = 0.0f;
    for (int n = threadIdx.x; n < batch; n += 256) {
        switch (kind) {
        case 0: s = fmaf(dh[(int64_t)n * H + i0], X[(int64_t)n * F + i1], s); break;
        case 1: s += dh[(int64_t)n * H + i0]; break;
        case 2: s = fmaf(dy[(int64_t)n * T + i0], hid[(int64_t)n * H + i1], s); break;
        case 3: s += dy[(int64_t)n * T + i0]; break;
        default: s += lossp[n]; break;
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int m = 128; m >= 1; m >>= 1) {
        if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float v = red[0];
        switch (kind) {
        case 0: gW1[i0 * F + i1] = v; break;
        case 1: gb1[i0] = v; break;
        case 2: gW2[i0 * H + i1] = v; break;
        case 3: gb2[i0] = v; break;
        default: *loss = v; break;
        }
    }
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float mi = b1 * m[i] + (1.0f - b1) * g[i];
    float vi = b2 * v[i] + (1.0f - b2) * g[i] * g[i];
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// the transform the fused predictor of the search applies before z-scoring
__global__ void feature_transform_kernel(const float *raw, int64_t n, int metric, float *out) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const float *f = raw + r * ONNG_NFEAT;
    float *x = out + r * ONNG_NFEAT;
    for (int t = 0; t < ONNG_NFEAT; t++) x[t] = feature_input(t, f[t], f[0], metric);
}

// Per-column mean and standard deviation of x [n][cols] (weights w [n][cols]
// or all ones): one block per column, sums in double, the deviations in a
// second pass over the column.  A standard deviation below 1e-6 becomes 1.
__global__ void column_stats_kernel(const float *x, const float *w, int64_t n, int cols,
                                    float *mean, float *stdv) {
    __shared__ double red[2][256];
    const int c = blockIdx.x;
    double sw = 0.0, sx = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
        const double wi = w ? (double)w[r * cols + c] : 1.0;
        sw += wi;
        sx += wi * (double)x[r * cols + c];
    }
    red[0][threadIdx.x] = sw;
    red[1][threadIdx.x] = sx;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    const double tot = red[0][0] > 1e-12 ? red[0][0] : 1e-12;
    const double mu = red[1][0] / tot;
    __syncthreads();
    double sv = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
        const double wi = w ? (double)w[r * cols + c] : 1.0;
        const double d = (double)x[r * cols + c] - mu;
        sv += wi * d * d;
    }
    red[0][threadIdx.x] = sv;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) red[0][threadIdx.x] += red[0][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double sd = sqrt(red[0][0] / tot);
        mean[c] = (float)mu;
        stdv[c] = sd < 1e-6 ? 1.0f : (float)sd;
    }
}

__global__ void standardize_kernel(const float *x, int64_t n, int cols, const float *mean,
                                   const float *stdv, float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * cols) return;
    const int c = (int)(i % cols);
    out[i] = (x[i] - mean[c]) / stdv[c];
}

// W2 [T][H] and b2 [T] of a network trained on targets (y - shift) / scale:
// the same network on the targets themselves.
__global__ void fold_output_kernel(float *w2, float *b2, int T, int H, const float *scale,
                                   const float *shift) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < T * H) w2[i] *= scale[i / H];
    if (i < T) b2[i] = b2[i] * scale[i] + shift[i];
}

}  // namespace

onng_status column_stats_launch(const float *x, const float *w, int64_t n, int32_t cols,
                                float *mean, float *stdv, hipStream_t st) {
    if (cols == 0) return ONNG_OK;
    hipLaunchKernelGGL(column_stats_kernel, dim3((unsigned)cols), dim3(256), 0, st, x, w, n, cols,
                       mean, stdv);
    ONNG_HIP(hipGetLastError());
    return ONNG_OK;
}

onng_status standardize_launch(const float *x, int64_t n, int32_t cols, const float *mean,
                               const float *stdv, float *out, hipStream_t st) {
    if (n == 0 || cols == 0) return ONNG_OK;
    hipLaunchKernelGGL(standardize_kernel, dim3((unsigned)((n * cols + 255) / 256)), dim3(256), 0,
                       st, x, n, cols, mean, stdv, out);
    ONNG_HIP(hipGetLastError());
    return ONNG_OK;
}

onng_status fold_output_launch(float *w2, float *b2, int32_t T, int32_t H, const float *scale,
                               const float *shift, hipStream_t st) {
    if (T == 0) return ONNG_OK;
    const int m = T * H > T ? T * H : T;
    hipLaunchKernelGGL(fold_output_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, w2,
                       b2, T, H, scale, shift);
    ONNG_HIP(hipGetLastError());
    return ONNG_OK;
}

size_t mlp_backward_ws(int32_t batch, int32_t H, int32_t T) {
    Carver c(nullptr);
    c.take<float>((size_t)batch * H);   // hidden
    c.take<float>((size_t)batch * T);   // dy
    c.take<float>((size_t)batch * H);   // dh
    c.take<float>((size_t)batch);       // per-sample loss
    return c.size() + 256;
}

onng_status mlp_forward_launch(const float *X, int32_t batch, int32_t F, const float *W1,
                               const float *b1, int32_t H, const float *W2, const float *b2,
                               int32_t T, float *hidden, float *Y, hipStream_t st) {
    if (batch == 0) return ONNG_OK;
    hipLaunchKernelGGL(mlp_sample_kernel, dim3((batch + 127) / 128), dim3(128), 0, st, X, batch,
                       F, W1, b1, H, W2, b2, T, nullptr, nullptr, hidden, Y, nullptr, nullptr,
                       nullptr);
    ONNG_HIP(hipGetLastError());
    return ONNG_OK;
}

onng_status mlp_backward_launch(const float *X, const float *target, const float *w,
                                int32_t batch, int32_t F, const float *W1, const float *b1,
                                int32_t H, const float *W2, const float *b2, int32_t T,
                                float *gW1, float *gb1, float *gW2, float *gb2, float *loss,
                                void *ws, hipStream_t st) {
    Carver c(ws);
    float *hid = c.take<float>((size_t)batch * H);
    float *dy = c.take<float>((size_t)batch * T);
    float *dh = c.take<float>((size_t)batch * H);
    float *lp = c.take<float>((size_t)batch);
    hipLaunchKernelGGL(mlp_sample_kernel, dim3((batch + 127) / 128), dim3(128), 0, st, X, batch,
                       F, W1, b1, H, W2, b2, T, target, w, hid, nullptr, dy, dh, lp);
    int nparam = H * F + H + T * H + T + 1;
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3(nparam), dim3(256), 0, st, X, batch, F, H, T, hid,
                       dy, dh, lp, gW1, gb1, gW2, gb2, loss);
    ONNG_HIP(hipGetLastError());
    return ONNG_OK;
}

onng_status adam_launch(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                        float b1, float b2, float eps, int32_t t, hipStream_t st) {
    if (n == 0) return ONNG_OK;
    float c1 = (float)(1.0 - std::pow((double)b1, (double)t));
    float c2 = (float)(1.0 - std::pow((double)b2, (double)t));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, g, m,
                       v, n, lr, b1, b2, eps, c1, c2);
    ONNG_HIP(hipGetLastError());
    return ONNG_OK;
}

onng_status feature_transform_launch(const float *raw, int64_t n, int32_t metric, float *out,
                                     hipStream_t st) {
    if (n == 0) return ONNG_OK;
    hipLaunchKernelGGL(feature_transform_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       st, raw, n, metric, out);
    ONNG_HIP(hipGetLastError());
    return ONNG_OK;
}

}  // namespace onng
