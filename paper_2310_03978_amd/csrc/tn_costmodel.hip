// Learned step-time cost model: a 2 x 64 ReLU MLP trained and evaluated with
// the library's own HIP kernels (forward, backward, deterministic gradient
// reduction, Adam).  It predicts log(microseconds) of one launch of a step
// from the step's shape, layout and kernel features (tn_plan_step_features),
// and steers the choice of tile shapes (tn_plan_tune_with_model).  The paper
// ranks contractions by measured time (Sec. 4.1) and scores contraction trees
// with a hardware-weighted cost (Sec. 3.2); here that cost is learned from
// per-launch timings of the library's own kernels, taken with HIP events on the
// plan's stream (a rocprofv3 kernel trace of the same launches agrees with them).
//
// Parameters (FP32, one flat array): W1 [H x F], b1 [H], W2 [H x H], b2 [H],
// w3 [H], b3 [1].  Inputs are standardised with a per-feature mean and std.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tn.h"
#include "tn_internal.h"

namespace {

constexpr int H = 64;          // hidden width
constexpr int MAXF = 32;       // largest feature count

tn_status cm_fail(tn_status s, const std::string& m) {
  tn_set_error_detail(m.c_str());
  return s;
}

tn_status cm_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return cm_fail(TN_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return TN_OK;
}

struct Offsets {
  int64_t w1, b1, w2, b2, w3, b3, total;
  __host__ __device__ explicit Offsets(int F) {
    w1 = 0;
    b1 = w1 + (int64_t)H * F;
    w2 = b1 + H;
    b2 = w2 + (int64_t)H * H;
    w3 = b2 + H;
    b3 = w3 + H;
    total = b3 + 1;
  }
};

// One thread per sample: standardise, forward through both layers; optionally
// keep the standardised input and pre-activations for the backward pass.
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ X, const int32_t* __restrict__ idx,
                                                     int64_t n, int F, const float* __restrict__ mean,
                                                     const float* __restrict__ stdv, const float* __restrict__ p,
                                                     float* __restrict__ Xs, float* __restrict__ Z1,
                                                     float* __restrict__ Z2, float* __restrict__ Y) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const Offsets o(F);
  const int64_t row = idx ? idx[s] : s;
  float x[MAXF];
  for (int f = 0; f < F; ++f) {
    x[f] = (X[row * F + f] - mean[f]) / stdv[f];
    if (Xs) Xs[s * F + f] = x[f];
  }
  float h1[H];
  for (int j = 0; j < H; ++j) {
    float z = p[o.b1 + j];
    for (int f = 0; f < F; ++f) z = fmaf(p[o.w1 + (int64_t)j * F + f], x[f], z);
    if (Z1) Z1[s * H + j] = z;
    h1[j] = z > 0.f ? z : 0.f;
  }
  float y = p[o.b3];
  for (int j = 0; j < H; ++j) {
    float z = p[o.b2 + j];
    for (int i = 0; i < H; ++i) z = fmaf(p[o.w2 + (int64_t)j * H + i], h1[i], z);
    if (Z2) Z2[s * H + j] = z;
    y = fmaf(p[o.w3 + j], z > 0.f ? z : 0.f, y);
  }
  Y[s] = y;
}

// Per-sample deltas: dy = 2 (y - t) / n, dz2 = dy w3 relu'(z2), dz1 = (dz2 W2) relu'(z1).
__global__ __launch_bounds__(256) void k_mlp_deltas(const float* __restrict__ T, const int32_t* __restrict__ idx,
                                                    int64_t n, int F, const float* __restrict__ p,
                                                    const float* __restrict__ Y, const float* __restrict__ Z1,
                                                    const float* __restrict__ Z2, float* __restrict__ DY,
                                                    float* __restrict__ D1, float* __restrict__ D2) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const Offsets o(F);
  const int64_t row = idx ? idx[s] : s;
  const float dy = 2.f * (Y[s] - T[row]) / (float)n;
  DY[s] = dy;
  float d2[H];
  for (int j = 0; j < H; ++j) {
    d2[j] = Z2[s * H + j] > 0.f ? dy * p[o.w3 + j] : 0.f;
    D2[s * H + j] = d2[j];
  }
  for (int i = 0; i < H; ++i) {
    float acc = 0.f;
    for (int j = 0; j < H; ++j) acc = fmaf(d2[j], p[o.w2 + (int64_t)j * H + i], acc);
    D1[s * H + i] = Z1[s * H + i] > 0.f ? acc : 0.f;
  }
}

// One thread per parameter: sum its gradient over the batch in sample order
// (deterministic; no atomics).
__global__ __launch_bounds__(256) void k_mlp_grad(int64_t n, int F, const float* __restrict__ Xs,
                                                  const float* __restrict__ Z1, const float* __restrict__ Z2,
                                                  const float* __restrict__ DY, const float* __restrict__ D1,
                                                  const float* __restrict__ D2, float* __restrict__ G) {
  const Offsets o(F);
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= o.total) return;
  float acc = 0.f;
  if (q < o.b1) {
    const int j = (int)(q / F), f = (int)(q % F);
    for (int64_t s = 0; s < n; ++s) acc = fmaf(D1[s * H + j], Xs[s * F + f], acc);
  } else if (q < o.w2) {
    const int j = (int)(q - o.b1);
    for (int64_t s = 0; s < n; ++s) acc += D1[s * H + j];
  } else if (q < o.b2) {
    const int j = (int)((q - o.w2) / H), i = (int)((q - o.w2) % H);
    for (int64_t s = 0; s < n; ++s) {
      const float h = Z1[s * H + i];
      acc = fmaf(D2[s * H + j], h > 0.f ? h : 0.f, acc);
    }
  } else if (q < o.w3) {
    const int j = (int)(q - o.b2);
    for (int64_t s = 0; s < n; ++s) acc += D2[s * H + j];
  } else if (q < o.b3) {
    const int j = (int)(q - o.w3);
    for (int64_t s = 0; s < n; ++s) {
      const float h = Z2[s * H + j];
      acc = fmaf(DY[s], h > 0.f ? h : 0.f, acc);
    }
  } else {
    for (int64_t s = 0; s < n; ++s) acc += DY[s];
  }
  G[q] = acc;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int64_t n, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.f - b1) * gq;
  const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// Mean squared error of Y against T[idx] with one block, in sample order per thread.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                             const int32_t* __restrict__ idx, int64_t n, float* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t s = threadIdx.x; s < n; s += blockDim.x) {
    const double d = (double)Y[s] - (double)T[idx ? idx[s] : s];
    acc += d * d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(red[0] / (double)(n > 0 ? n : 1));
}

// splitmix64 (Steele, Lea, Flood 2014): counter-based, for the weight initialisation
uint64_t splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

float uniform(uint64_t seed, uint64_t i) { return (float)((splitmix64(seed ^ splitmix64(i)) >> 11) * 0x1.0p-53); }

}  // namespace

struct tn_costmodel_s {
  int F = 0;
  int64_t P = 0;
  float* d_p = nullptr;
  float* d_m = nullptr;
  float* d_v = nullptr;
  float* d_g = nullptr;
  float* d_mean = nullptr;
  float* d_std = nullptr;
  int64_t step = 0;
  // workspace for a batch
  int64_t cap = 0;
  float *d_x = nullptr, *d_t = nullptr, *d_xs = nullptr, *d_z1 = nullptr, *d_z2 = nullptr, *d_y = nullptr,
        *d_dy = nullptr, *d_d1 = nullptr, *d_d2 = nullptr, *d_loss = nullptr;
  int32_t* d_idx = nullptr;
  int64_t xcap = 0;
  ~tn_costmodel_s() {
    hipDeviceSynchronize();
    float* ps[] = {d_p, d_m, d_v, d_g, d_mean, d_std, d_x, d_t, d_xs, d_z1, d_z2, d_y, d_dy, d_d1, d_d2, d_loss};
    for (float* q : ps)
      if (q) hipFree(q);
    if (d_idx) hipFree(d_idx);
  }
};

namespace {

tn_status cm_alloc(void** p, size_t bytes) {
  if (hipMalloc(p, bytes < 64 ? 64 : bytes) != hipSuccess) {
    hipGetLastError();
    return cm_fail(TN_E_NOMEM, "cost model allocation failed");
  }
  return TN_OK;
}

// Batch workspace for up to `b` samples and `nx` resident input rows.
tn_status cm_reserve(tn_costmodel_s* m, int64_t b, int64_t nx) {
  tn_status st = TN_OK;
  if (b > m->cap) {
    float** ws[] = {&m->d_xs, &m->d_z1, &m->d_z2, &m->d_y, &m->d_dy, &m->d_d1, &m->d_d2};
    for (float** q : ws)
      if (*q) {
        hipFree(*q);
        *q = nullptr;
      }
    if (m->d_idx) hipFree(m->d_idx);
    m->d_idx = nullptr;
    m->cap = 0;
    if ((st = cm_alloc((void**)&m->d_xs, b * m->F * 4))) return st;
    if ((st = cm_alloc((void**)&m->d_z1, b * H * 4))) return st;
    if ((st = cm_alloc((void**)&m->d_z2, b * H * 4))) return st;
    if ((st = cm_alloc((void**)&m->d_y, b * 4))) return st;
    if ((st = cm_alloc((void**)&m->d_dy, b * 4))) return st;
    if ((st = cm_alloc((void**)&m->d_d1, b * H * 4))) return st;
    if ((st = cm_alloc((void**)&m->d_d2, b * H * 4))) return st;
    if ((st = cm_alloc((void**)&m->d_idx, b * 4))) return st;
    m->cap = b;
  }
  if (nx > m->xcap) {
    if (m->d_x) hipFree(m->d_x);
    if (m->d_t) hipFree(m->d_t);
    m->d_x = m->d_t = nullptr;
    m->xcap = 0;
    if ((st = cm_alloc((void**)&m->d_x, nx * m->F * 4))) return st;
    if ((st = cm_alloc((void**)&m->d_t, nx * 4))) return st;
    m->xcap = nx;
  }
  return st;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// forward + deltas + gradient over rows idx[0..n) of the resident inputs
tn_status cm_gradient(tn_costmodel_s* m, const int32_t* d_idx, int64_t n) {
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks_for(n)), dim3(256), 0, nullptr, m->d_x, d_idx, n, m->F, m->d_mean,
                     m->d_std, m->d_p, m->d_xs, m->d_z1, m->d_z2, m->d_y);
  hipLaunchKernelGGL(k_mlp_deltas, dim3(blocks_for(n)), dim3(256), 0, nullptr, m->d_t, d_idx, n, m->F, m->d_p, m->d_y,
                     m->d_z1, m->d_z2, m->d_dy, m->d_d1, m->d_d2);
  hipLaunchKernelGGL(k_mlp_grad, dim3(blocks_for(m->P)), dim3(256), 0, nullptr, n, m->F, m->d_xs, m->d_z1, m->d_z2,
                     m->d_dy, m->d_d1, m->d_d2, m->d_g);
  return cm_check(hipGetLastError(), "mlp gradient");
}

tn_status cm_adam(tn_costmodel_s* m, float lr) {
  m->step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(m->P)), dim3(256), 0, nullptr, m->d_p, m->d_g, m->d_m, m->d_v, m->P, lr,
                     b1, b2, eps, c1, c2);
  return cm_check(hipGetLastError(), "adam");
}

tn_status cm_upload(tn_costmodel_s* m, const float* X, const float* T, int64_t n) {
  tn_status st = cm_reserve(m, 1, n);
  if (st) return st;
  if ((st = cm_check(hipMemcpy(m->d_x, X, n * m->F * 4, hipMemcpyHostToDevice), "upload X"))) return st;
  if (T) st = cm_check(hipMemcpy(m->d_t, T, n * 4, hipMemcpyHostToDevice), "upload t");
  return st;
}

}  // namespace

extern "C" {

tn_status tn_costmodel_create(tn_costmodel* out, int32_t n_features, uint64_t seed) {
  TN_TRY
  if (!out || n_features < 1 || n_features > MAXF) return cm_fail(TN_E_ARG, "n_features must be in [1, 32]");
  *out = nullptr;
  tn_costmodel_s* m = new (std::nothrow) tn_costmodel_s();
  if (!m) return cm_fail(TN_E_NOMEM, "host allocation failed");
  m->F = n_features;
  m->P = Offsets(n_features).total;
  tn_status st = TN_OK;
  float** bufs[] = {&m->d_p, &m->d_m, &m->d_v, &m->d_g};
  for (float** b : bufs)
    if (!st) st = cm_alloc((void**)b, m->P * 4);
  if (!st) st = cm_alloc((void**)&m->d_mean, MAXF * 4);
  if (!st) st = cm_alloc((void**)&m->d_std, MAXF * 4);
  // He-uniform weights, zero biases; identity standardisation
  std::vector<float> p(m->P, 0.f);
  const Offsets o(n_features);
  const float a1 = std::sqrt(6.f / n_features), a2 = std::sqrt(6.f / H);
  for (int64_t i = 0; i < (int64_t)H * n_features; ++i) p[o.w1 + i] = a1 * (2.f * uniform(seed, o.w1 + i) - 1.f);
  for (int64_t i = 0; i < (int64_t)H * H; ++i) p[o.w2 + i] = a2 * (2.f * uniform(seed, o.w2 + i) - 1.f);
  for (int64_t i = 0; i < H; ++i) p[o.w3 + i] = a2 * (2.f * uniform(seed, o.w3 + i) - 1.f);
  std::vector<float> zeros(m->P, 0.f), mean(MAXF, 0.f), one(MAXF, 1.f);
  if (!st) st = cm_check(hipMemcpy(m->d_p, p.data(), m->P * 4, hipMemcpyHostToDevice), "init");
  if (!st) st = cm_check(hipMemcpy(m->d_m, zeros.data(), m->P * 4, hipMemcpyHostToDevice), "init");
  if (!st) st = cm_check(hipMemcpy(m->d_v, zeros.data(), m->P * 4, hipMemcpyHostToDevice), "init");
  if (!st) st = cm_check(hipMemcpy(m->d_mean, mean.data(), MAXF * 4, hipMemcpyHostToDevice), "init");
  if (!st) st = cm_check(hipMemcpy(m->d_std, one.data(), MAXF * 4, hipMemcpyHostToDevice), "init");
  if (st) {
    delete m;
    return st;
  }
  *out = m;
  return TN_OK;
  TN_CATCH
}

void tn_costmodel_destroy(tn_costmodel m) {
  TN_TRY_VOID
  delete m;
  TN_CATCH_VOID
}

tn_status tn_costmodel_describe(tn_costmodel m, int32_t* n_features, int32_t* hidden, int64_t* n_params) {
  TN_TRY
  if (!m) return cm_fail(TN_E_ARG, "null model");
  if (n_features) *n_features = m->F;
  if (hidden) *hidden = H;
  if (n_params) *n_params = m->P;
  return TN_OK;
  TN_CATCH
}

tn_status tn_costmodel_set_normalization(tn_costmodel m, const float* mean, const float* stdv) {
  TN_TRY
  if (!m || !mean || !stdv) return cm_fail(TN_E_ARG, "null argument");
  for (int f = 0; f < m->F; ++f)
    if (!(stdv[f] > 0.f)) return cm_fail(TN_E_ARG, "std must be positive");
  tn_status st = cm_check(hipMemcpy(m->d_mean, mean, m->F * 4, hipMemcpyHostToDevice), "mean");
  if (!st) st = cm_check(hipMemcpy(m->d_std, stdv, m->F * 4, hipMemcpyHostToDevice), "std");
  return st;
  TN_CATCH
}

tn_status tn_costmodel_get_params(tn_costmodel m, float* out, int64_t n) {
  TN_TRY
  if (!m || !out || n != m->P) return cm_fail(TN_E_ARG, "n must equal the parameter count");
  return cm_check(hipMemcpy(out, m->d_p, n * 4, hipMemcpyDeviceToHost), "params");
  TN_CATCH
}

tn_status tn_costmodel_set_params(tn_costmodel m, const float* in, int64_t n) {
  TN_TRY
  if (!m || !in || n != m->P) return cm_fail(TN_E_ARG, "n must equal the parameter count");
  m->step = 0;
  std::vector<float> zeros(m->P, 0.f);
  tn_status st = cm_check(hipMemcpy(m->d_p, in, n * 4, hipMemcpyHostToDevice), "params");
  if (!st) st = cm_check(hipMemcpy(m->d_m, zeros.data(), n * 4, hipMemcpyHostToDevice), "moments");
  if (!st) st = cm_check(hipMemcpy(m->d_v, zeros.data(), n * 4, hipMemcpyHostToDevice), "moments");
  return st;
  TN_CATCH
}

tn_status tn_costmodel_predict(tn_costmodel m, const float* X, int64_t n, float* y) {
  TN_TRY
  if (!m || (n > 0 && (!X || !y)) || n < 0) return cm_fail(TN_E_ARG, "bad arguments");
  if (n == 0) return TN_OK;
  tn_status st = cm_upload(m, X, nullptr, n);
  if (!st) st = cm_reserve(m, n, n);
  if (st) return st;
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks_for(n)), dim3(256), 0, nullptr, m->d_x, nullptr, n, m->F, m->d_mean,
                     m->d_std, m->d_p, nullptr, nullptr, nullptr, m->d_y);
  if ((st = cm_check(hipGetLastError(), "predict"))) return st;
  return cm_check(hipMemcpy(y, m->d_y, n * 4, hipMemcpyDeviceToHost), "predict copy");
  TN_CATCH
}

tn_status tn_costmodel_gradient(tn_costmodel m, const float* X, const float* t, int64_t n, float* grad,
                                float* loss) {
  TN_TRY
  if (!m || !X || !t || n < 1) return cm_fail(TN_E_ARG, "bad arguments");
  tn_status st = cm_upload(m, X, t, n);
  if (!st) st = cm_reserve(m, n, n);
  if (!st) st = cm_gradient(m, nullptr, n);
  if (!st && loss) {
    if (!m->d_loss && (st = cm_alloc((void**)&m->d_loss, 64))) return st;
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, nullptr, m->d_y, m->d_t, nullptr, n, m->d_loss);
    st = cm_check(hipMemcpy(loss, m->d_loss, 4, hipMemcpyDeviceToHost), "loss");
  }
  if (!st && grad) st = cm_check(hipMemcpy(grad, m->d_g, m->P * 4, hipMemcpyDeviceToHost), "grad");
  return st;
  TN_CATCH
}

tn_status tn_costmodel_adam_step(tn_costmodel m, const float* grad, int64_t n, float lr) {
  TN_TRY
  if (!m || !grad || n != m->P) return cm_fail(TN_E_ARG, "bad arguments");
  tn_status st = cm_check(hipMemcpy(m->d_g, grad, n * 4, hipMemcpyHostToDevice), "grad");
  if (!st) st = cm_adam(m, lr);
  if (!st) st = cm_check(hipDeviceSynchronize(), "adam sync");
  return st;
  TN_CATCH
}

tn_status tn_costmodel_train(tn_costmodel m, const float* X, const float* t, int64_t n, int32_t epochs,
                             int32_t batch, float lr, uint64_t seed, float* final_loss) {
  TN_TRY
  if (!m || !X || !t || n < 1 || epochs < 0 || batch < 1) return cm_fail(TN_E_ARG, "bad arguments");
  tn_status st = cm_upload(m, X, t, n);
  if (!st) st = cm_reserve(m, std::max<int64_t>(batch, n), n);
  if (st) return st;
  std::vector<int32_t> perm(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int e = 0; e < epochs && !st; ++e) {
    // Fisher-Yates with the counter-based generator
    for (int64_t i = n - 1; i > 0; --i) {
      const int64_t j = (int64_t)(splitmix64(seed ^ splitmix64((uint64_t)e * 0x100000000ull + (uint64_t)i)) %
                                  (uint64_t)(i + 1));
      std::swap(perm[i], perm[j]);
    }
    st = cm_check(hipMemcpy(m->d_idx, perm.data(), n * 4, hipMemcpyHostToDevice), "perm");
    for (int64_t off = 0; off < n && !st; off += batch) {
      const int64_t b = std::min<int64_t>(batch, n - off);
      st = cm_gradient(m, m->d_idx + off, b);
      if (!st) st = cm_adam(m, lr);
    }
  }
  if (!st && final_loss) {
    // full-data loss
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks_for(n)), dim3(256), 0, nullptr, m->d_x, nullptr, n, m->F,
                       m->d_mean, m->d_std, m->d_p, nullptr, nullptr, nullptr, m->d_y);
    if (!m->d_loss) st = cm_alloc((void**)&m->d_loss, 64);
    if (!st) hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, nullptr, m->d_y, m->d_t, nullptr, n, m->d_loss);
    if (!st) st = cm_check(hipMemcpy(final_loss, m->d_loss, 4, hipMemcpyDeviceToHost), "loss");
  }
  if (!st) st = cm_check(hipDeviceSynchronize(), "train sync");
  return st;
  TN_CATCH
}

}  // extern "C"
