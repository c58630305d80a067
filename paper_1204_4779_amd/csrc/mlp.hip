// MLP cost model of the kernel tuner: in -> H -> H -> 1, ReLU hidden layers,
// mean-squared-error loss, Adam.  Predicting a variant's score before
// benchmarking it is the machine-learning extension the paper names as
// future work for its tuner (section "Conclusion and Discussion").
//
// Parameters are one packed FP32 array:
//   W1[in][H], b1[H], W2[H][H], b2[H], w3[H], b3
// (row-major, input index first).  Every reduction runs in a fixed order
// (one thread per output, a serial loop over the reduced index), so results
// are bitwise reproducible.  The layers are a few thousand multiply-adds per
// sample; they stay on plain FP32 FMA rather than matrix cores.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "paraiso.h"

// the library's per-thread error message (runtime.hip)
void paraiso_set_error(const std::string& msg);

namespace {

struct ErrSink {
  ErrSink& operator=(const std::string& m) {
    paraiso_set_error(m);
    return *this;
  }
  ErrSink& operator=(const char* m) { return *this = std::string(m); }
};
ErrSink g_mlp_err;

struct Offsets {
  int64_t w1, b1, w2, b2, w3, b3, total;
};

Offsets offsets(int in, int H) {
  Offsets o;
  o.w1 = 0;
  o.b1 = o.w1 + (int64_t)in * H;
  o.w2 = o.b1 + H;
  o.b2 = o.w2 + (int64_t)H * H;
  o.w3 = o.b2 + H;
  o.b3 = o.w3 + H;
  o.total = o.b3 + 1;
  return o;
}

// workspace: H1[B][H], H2[B][H], Y[B], dY[B], dH2[B][H], dH1[B][H]
struct Work {
  float *h1, *h2, *y, *dy, *dh2, *dh1;
};

size_t work_bytes(int B, int H) { return sizeof(float) * ((size_t)B * H * 4 + (size_t)B * 2) + 256; }

Work carve(void* ws, int B, int H) {
  float* p = reinterpret_cast<float*>(ws);
  Work w;
  w.h1 = p;
  p += (size_t)B * H;
  w.h2 = p;
  p += (size_t)B * H;
  w.dh2 = p;
  p += (size_t)B * H;
  w.dh1 = p;
  p += (size_t)B * H;
  w.y = p;
  p += B;
  w.dy = p;
  return w;
}

// out[b][j] = act(bias[j] + sum_k A[b][k] W[k][j])
__global__ void k_dense(const float* A, int B, int K, const float* W, const float* bias, int N, float* out,
                        int relu) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * N) return;
  const int b = idx / N, j = idx % N;
  float s = bias[j];
  for (int k = 0; k < K; ++k) s = fmaf(A[(size_t)b * K + k], W[(size_t)k * N + j], s);
  out[idx] = relu ? fmaxf(s, 0.0f) : s;
}

// dY = 2 (Y - T) / B ; loss = mean (Y - T)^2 (single block, fixed order)
__global__ void k_loss(const float* y, const float* t, int B, float* dy, float* loss) {
  __shared__ float s[256];
  float acc = 0.0f;
  for (int b = threadIdx.x; b < B; b += 256) {
    const float e = y[b] - t[b];
    dy[b] = 2.0f * e / (float)B;
    acc = fmaf(e, e, acc);
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = s[0] / (float)B;
}

// dH2[b][j] = dY[b] w3[j] [H2 > 0]
__global__ void k_back_out(const float* dy, const float* w3, const float* h2, int B, int H, float* dh2) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * H) return;
  const int b = idx / H, j = idx % H;
  dh2[idx] = h2[idx] > 0.0f ? dy[b] * w3[j] : 0.0f;
}

// dH1[b][i] = sum_j dH2[b][j] W2[i][j]  [H1 > 0]
__global__ void k_back_hidden(const float* dh2, const float* w2, const float* h1, int B, int H, float* dh1) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * H) return;
  const int b = idx / H, i = idx % H;
  float s = 0.0f;
  for (int j = 0; j < H; ++j) s = fmaf(dh2[(size_t)b * H + j], w2[(size_t)i * H + j], s);
  dh1[idx] = h1[idx] > 0.0f ? s : 0.0f;
}

// One thread per parameter: gradient as a fixed-order sum over the batch.
__global__ void k_param_grads(const float* X, int B, int in, int H, const float* h1, const float* h2,
                              const float* dh1, const float* dh2, const float* dy, float* g) {
  const Offsets o = {0, (int64_t)in * H, (int64_t)in * H + H, (int64_t)in * H + H + (int64_t)H * H,
                     (int64_t)in * H + 2 * H + (int64_t)H * H, (int64_t)in * H + 3 * H + (int64_t)H * H,
                     (int64_t)in * H + 3 * H + (int64_t)H * H + 1};
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= o.total) return;
  float s = 0.0f;
  if (p < o.b1) {  // W1[k][i]
    const int k = (int)(p / H), i = (int)(p % H);
    for (int b = 0; b < B; ++b) s = fmaf(X[(size_t)b * in + k], dh1[(size_t)b * H + i], s);
  } else if (p < o.w2) {  // b1[i]
    const int i = (int)(p - o.b1);
    for (int b = 0; b < B; ++b) s += dh1[(size_t)b * H + i];
  } else if (p < o.b2) {  // W2[i][j]
    const int64_t q = p - o.w2;
    const int i = (int)(q / H), j = (int)(q % H);
    for (int b = 0; b < B; ++b) s = fmaf(h1[(size_t)b * H + i], dh2[(size_t)b * H + j], s);
  } else if (p < o.w3) {  // b2[j]
    const int j = (int)(p - o.b2);
    for (int b = 0; b < B; ++b) s += dh2[(size_t)b * H + j];
  } else if (p < o.b3) {  // w3[j]
    const int j = (int)(p - o.w3);
    for (int b = 0; b < B; ++b) s = fmaf(h2[(size_t)b * H + j], dy[b], s);
  } else {  // b3
    for (int b = 0; b < B; ++b) s += dy[b];
  }
  g[p] = s;
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  p[i] -= lr * mh / (sqrtf(vh) + eps);
}

int check_dims(int B, int in, int H) {
  if (B < 1 || in < 1 || H < 1 || in > 4096 || H > 1024 || (int64_t)B * H > (int64_t(1) << 30)) {
    g_mlp_err = "mlp: batch, in_dim and hidden must be >= 1 (in_dim <= 4096, hidden <= 1024)";
    return PARAISO_ERR_INVALID_ARG;
  }
  return PARAISO_OK;
}

int forward(const float* X, int B, int in, int H, const float* P, Work w, hipStream_t s) {
  const Offsets o = offsets(in, H);
  const int t = 256;
  hipLaunchKernelGGL(k_dense, dim3((B * H + t - 1) / t), dim3(t), 0, s, X, B, in, P + o.w1, P + o.b1, H, w.h1, 1);
  hipLaunchKernelGGL(k_dense, dim3((B * H + t - 1) / t), dim3(t), 0, s, w.h1, B, H, P + o.w2, P + o.b2, H, w.h2,
                     1);
  hipLaunchKernelGGL(k_dense, dim3((B + t - 1) / t), dim3(t), 0, s, w.h2, B, H, P + o.w3, P + o.b3, 1, w.y, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_mlp_err = std::string("mlp launch: ") + hipGetErrorString(e);
    return PARAISO_ERR_HIP;
  }
  return PARAISO_OK;
}

}  // namespace

extern "C" {

int32_t paraiso_mlp_sizes(int32_t in_dim, int32_t hidden, int32_t batch, int64_t* n_params,
                          size_t* workspace_bytes) {
  int rc = check_dims(batch, in_dim, hidden);
  if (rc) return rc;
  if (n_params) *n_params = offsets(in_dim, hidden).total;
  if (workspace_bytes) *workspace_bytes = work_bytes(batch, hidden);
  return PARAISO_OK;
}

int32_t paraiso_mlp_forward(const float* X, int32_t batch, int32_t in_dim, int32_t hidden, const float* params,
                            float* y, void* workspace, size_t workspace_bytes, void* stream) {
  int rc = check_dims(batch, in_dim, hidden);
  if (rc) return rc;
  if (!X || !params || !y || !workspace) {
    g_mlp_err = "mlp_forward: null pointer";
    return PARAISO_ERR_INVALID_ARG;
  }
  if (workspace_bytes < work_bytes(batch, hidden)) {
    g_mlp_err = "mlp_forward: workspace too small";
    return PARAISO_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  Work w = carve(workspace, batch, hidden);
  rc = forward(X, batch, in_dim, hidden, params, w, s);
  if (rc) return rc;
  if (hipMemcpyAsync(y, w.y, sizeof(float) * batch, hipMemcpyDeviceToDevice, s) != hipSuccess) {
    g_mlp_err = "mlp_forward: copy of the outputs failed";
    return PARAISO_ERR_HIP;
  }
  return PARAISO_OK;
}

int32_t paraiso_mlp_loss_grad(const float* X, const float* target, int32_t batch, int32_t in_dim, int32_t hidden,
                              const float* params, float* grad, float* loss, void* workspace,
                              size_t workspace_bytes, void* stream) {
  int rc = check_dims(batch, in_dim, hidden);
  if (rc) return rc;
  if (!X || !target || !params || !grad || !workspace) {
    g_mlp_err = "mlp_loss_grad: null pointer";
    return PARAISO_ERR_INVALID_ARG;
  }
  if (workspace_bytes < work_bytes(batch, hidden)) {
    g_mlp_err = "mlp_loss_grad: workspace too small";
    return PARAISO_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  Work w = carve(workspace, batch, hidden);
  rc = forward(X, batch, in_dim, hidden, params, w, s);
  if (rc) return rc;
  const Offsets o = offsets(in_dim, hidden);
  const int t = 256;
  const int BH = batch * hidden;
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, s, w.y, target, batch, w.dy, loss);
  hipLaunchKernelGGL(k_back_out, dim3((BH + t - 1) / t), dim3(t), 0, s, w.dy, params + o.w3, w.h2, batch, hidden,
                     w.dh2);
  hipLaunchKernelGGL(k_back_hidden, dim3((BH + t - 1) / t), dim3(t), 0, s, w.dh2, params + o.w2, w.h1, batch,
                     hidden, w.dh1);
  hipLaunchKernelGGL(k_param_grads, dim3((unsigned)((o.total + t - 1) / t)), dim3(t), 0, s, X, batch, in_dim,
                     hidden, w.h1, w.h2, w.dh1, w.dh2, w.dy, grad);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_mlp_err = std::string("mlp_loss_grad launch: ") + hipGetErrorString(e);
    return PARAISO_ERR_HIP;
  }
  return PARAISO_OK;
}

int32_t paraiso_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t n, float lr, float beta1,
                         float beta2, float eps, int32_t step, void* stream) {
  if (!params || !grad || !m || !v || n < 1 || step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
      !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f)) {
    g_mlp_err = "mlp_adam: invalid argument";
    return PARAISO_ERR_INVALID_ARG;
  }
  const float c1 = 1.0f - powf(beta1, (float)step);
  const float c2 = 1.0f - powf(beta2, (float)step);
  const int t = 256;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + t - 1) / t)), dim3(t), 0, (hipStream_t)stream, params, grad, m,
                     v, n, lr, beta1, beta2, eps, c1, c2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_mlp_err = std::string("mlp_adam launch: ") + hipGetErrorString(e);
    return PARAISO_ERR_HIP;
  }
  return PARAISO_OK;
}

}  // extern "C"
