// Size predictor behind the kc_pred_* entry points of include/kc.h: a
// two-layer fp32 perceptron y = w2 . relu(W1 x + b1) + b2 that maps features
// of a counting job to an estimate (the log of its number of distinct keys).
// It only informs memory reservations of the request server; it never touches
// a count. Training (forward, backward, Adam) runs in the kernels below.
//
// Parameters, one fp32 array: W1 [H][F] row-major, b1 [H], w2 [H], b2 [1].
// Loss: mean over the batch of (y - t)^2 / 2.
// Gradients are reduced per parameter over the samples in a fixed order, so
// they are deterministic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/kc.h"
#include "kc_host.h"

namespace {

constexpr int kMaxF = 32, kMaxH = 128;

__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ prm, int F, int H,
                                                     const float* __restrict__ x, uint64_t B,
                                                     float* __restrict__ y) {
  extern __shared__ float sp[];
  const int np = H * F + 2 * H + 1;
  for (int i = threadIdx.x; i < np; i += blockDim.x) sp[i] = prm[i];
  __syncthreads();
  const float* W1 = sp;
  const float* b1 = sp + H * F;
  const float* w2 = b1 + H;
  const float b2 = w2[H];
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  float xi[kMaxF];
  for (int f = 0; f < F; ++f) xi[f] = x[i * F + f];
  float acc = b2;
  for (int j = 0; j < H; ++j) {
    float z = b1[j];
    for (int f = 0; f < F; ++f) z = fmaf(W1[j * F + f], xi[f], z);
    acc = fmaf(w2[j], fmaxf(z, 0.0f), acc);
  }
  y[i] = acc;
}

// Per sample: dy = (y - t) / B, the hidden activations h, and
// dh_j = dy * w2_j * [z_j > 0]; also the sample's loss term.
__global__ void __launch_bounds__(256) k_mlp_backprop(const float* __restrict__ prm, int F, int H,
                                                      const float* __restrict__ x,
                                                      const float* __restrict__ t, uint64_t B,
                                                      float* __restrict__ dy,
                                                      float* __restrict__ hbuf,
                                                      float* __restrict__ dh,
                                                      float* __restrict__ lossv) {
  extern __shared__ float sp[];
  const int np = H * F + 2 * H + 1;
  for (int i = threadIdx.x; i < np; i += blockDim.x) sp[i] = prm[i];
  __syncthreads();
  const float* W1 = sp;
  const float* b1 = sp + H * F;
  const float* w2 = b1 + H;
  const float b2 = w2[H];
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  float xi[kMaxF];
  for (int f = 0; f < F; ++f) xi[f] = x[i * F + f];
  float acc = b2;
  for (int j = 0; j < H; ++j) {
    float z = b1[j];
    for (int f = 0; f < F; ++f) z = fmaf(W1[j * F + f], xi[f], z);
    const float h = fmaxf(z, 0.0f);
    hbuf[i * H + j] = h;
    acc = fmaf(w2[j], h, acc);
  }
  const float e = acc - t[i];
  const float g = e / (float)B;
  dy[i] = g;
  lossv[i] = 0.5f * e * e / (float)B;
  for (int j = 0; j < H; ++j) dh[i * H + j] = hbuf[i * H + j] > 0.0f ? g * w2[j] : 0.0f;
}

// One thread per parameter (plus one for the loss): sums over the samples in
// index order.
__global__ void __launch_bounds__(256) k_mlp_reduce(int F, int H, const float* __restrict__ x,
                                                    uint64_t B, const float* __restrict__ dy,
                                                    const float* __restrict__ hbuf,
                                                    const float* __restrict__ dh,
                                                    const float* __restrict__ lossv,
                                                    float* __restrict__ grad,
                                                    float* __restrict__ loss) {
  const int np = H * F + 2 * H + 1;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > np) return;
  float s = 0.0f;
  if (p < H * F) {
    const int j = p / F, f = p % F;
    for (uint64_t i = 0; i < B; ++i) s = fmaf(dh[i * H + j], x[i * F + f], s);
  } else if (p < H * F + H) {
    const int j = p - H * F;
    for (uint64_t i = 0; i < B; ++i) s += dh[i * H + j];
  } else if (p < H * F + 2 * H) {
    const int j = p - H * F - H;
    for (uint64_t i = 0; i < B; ++i) s = fmaf(dy[i], hbuf[i * H + j], s);
  } else if (p == np - 1) {
    for (uint64_t i = 0; i < B; ++i) s += dy[i];
  } else {  // p == np: the loss
    for (uint64_t i = 0; i < B; ++i) s += lossv[i];
    *loss = s;
    return;
  }
  grad[p] = s;
}

// Adam (Kingma & Ba, 2015) with bias correction.
__global__ void k_adam(float* __restrict__ prm, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float gi = g[p];
  const float mi = b1 * m[p] + (1.0f - b1) * gi;
  const float vi = b2 * v[p] + (1.0f - b2) * gi * gi;
  m[p] = mi;
  v[p] = vi;
  prm[p] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

struct Fail {
  int code;
};

[[noreturn]] void fail(int code, const std::string& msg) {
  kc::set_last_error(msg);
  throw Fail{code};
}

void hipchk(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? KC_E_NOMEM : KC_E_DEVICE,
         std::string(what) + ": " + hipGetErrorString(e));
  }
}

template <class F>
int guarded(F f) {
  kc::set_last_error("");
  try {
    return f();
  } catch (const Fail& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    kc::set_last_error("host allocation failed");
    return KC_E_NOMEM;
  } catch (...) {
    kc::set_last_error("unexpected C++ exception");
    return KC_E_INTERNAL;
  }
}

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

struct kc_predictor {
  int device = 0;
  int F = 0, H = 0, np = 0;
  int step = 0;
  float* prm = nullptr;   // device: parameters, then gradients, m, v, loss
  float* grad = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* loss = nullptr;
  float* scratch = nullptr;  // dy, h, dh, loss terms of the last batch
  uint64_t scratch_b = 0;
  float* host = nullptr;     // pinned staging

  ~kc_predictor() {
    int prev = -1;
    if (hipGetDevice(&prev) == hipSuccess) (void)hipSetDevice(device);
    if (prm) (void)hipFree(prm);
    if (scratch) (void)hipFree(scratch);
    if (host) (void)hipHostFree(host);
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

namespace {

void check_batch(kc_predictor* p, const void* x, uint64_t B) {
  if (!p) fail(KC_E_INVAL, "predictor is NULL");
  if (B && !x) fail(KC_E_INVAL, "feature array is NULL");
  if (B > (1ull << 24)) fail(KC_E_INVAL, "batch larger than 2^24");
}

unsigned blocks(uint64_t n, unsigned tb) { return (unsigned)((n + tb - 1) / tb); }

}  // namespace

extern "C" {

int kc_pred_create(int n_features, int hidden, uint64_t seed, kc_predictor** out) {
  return guarded([&]() -> int {
    if (!out) fail(KC_E_INVAL, "predictor pointer is NULL");
    *out = nullptr;
    if (n_features < 1 || n_features > kMaxF) fail(KC_E_INVAL, "features must be in [1, 32]");
    if (hidden < 1 || hidden > kMaxH) fail(KC_E_INVAL, "hidden units must be in [1, 128]");
    std::unique_ptr<kc_predictor> p(new kc_predictor());
    hipchk(hipGetDevice(&p->device), "hipGetDevice");
    p->F = n_features;
    p->H = hidden;
    p->np = hidden * n_features + 2 * hidden + 1;
    const size_t n = (size_t)p->np;
    hipchk(hipMalloc(&p->prm, (4 * n + 1) * sizeof(float)), "hipMalloc");
    p->grad = p->prm + n;
    p->m = p->grad + n;
    p->v = p->m + n;
    p->loss = p->v + n;
    hipchk(hipHostMalloc((void**)&p->host, (4 * n + 1) * sizeof(float), hipHostMallocDefault),
           "hipHostMalloc");
    // He-uniform first layer, Glorot-uniform second layer, zero biases
    uint64_t s = seed;
    std::vector<float> h(4 * n + 1, 0.0f);
    const double a1 = std::sqrt(6.0 / n_features), a2 = std::sqrt(6.0 / (hidden + 1));
    for (int i = 0; i < hidden * n_features; ++i)
      h[i] = (float)(a1 * (2.0 * (double)(splitmix(s) >> 11) / 9007199254740992.0 - 1.0));
    for (int j = 0; j < hidden; ++j)
      h[hidden * n_features + hidden + j] =
          (float)(a2 * (2.0 * (double)(splitmix(s) >> 11) / 9007199254740992.0 - 1.0));
    hipchk(hipMemcpy(p->prm, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice),
           "hipMemcpy");
    *out = p.release();
    return KC_OK;
  });
}

uint64_t kc_pred_num_params(const kc_predictor* p) { return p ? (uint64_t)p->np : 0; }

int kc_pred_get_params(const kc_predictor* p, float* host, uint64_t n) {
  return guarded([&]() -> int {
    if (!p || !host || n != (uint64_t)p->np) fail(KC_E_INVAL, "bad arguments");
    hipchk(hipMemcpy(host, p->prm, n * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
    return KC_OK;
  });
}

int kc_pred_set_params(kc_predictor* p, const float* host, uint64_t n) {
  return guarded([&]() -> int {
    if (!p || !host || n != (uint64_t)p->np) fail(KC_E_INVAL, "bad arguments");
    hipchk(hipMemcpy(p->prm, host, n * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
    // a new starting point: restart the optimiser's moments
    hipchk(hipMemset(p->m, 0, 2 * n * sizeof(float)), "hipMemset");
    p->step = 0;
    return KC_OK;
  });
}

int kc_pred_get_grads(const kc_predictor* p, float* host, uint64_t n) {
  return guarded([&]() -> int {
    if (!p || !host || n != (uint64_t)p->np) fail(KC_E_INVAL, "bad arguments");
    hipchk(hipMemcpy(host, p->grad, n * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
    return KC_OK;
  });
}

int kc_pred_forward(kc_predictor* p, const float* x, uint64_t batch, float* y, void* stream) {
  return guarded([&]() -> int {
    check_batch(p, x, batch);
    if (batch && !y) fail(KC_E_INVAL, "output array is NULL");
    if (!batch) return KC_OK;
    const hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks(batch, 256)), dim3(256),
                       p->np * sizeof(float), st, p->prm, p->F, p->H, x, batch, y);
    hipchk(hipGetLastError(), "forward launch");
    hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
    return KC_OK;
  });
}

int kc_pred_gradient(kc_predictor* p, const float* x, const float* target, uint64_t batch,
                     float* host_loss, void* stream) {
  return guarded([&]() -> int {
    check_batch(p, x, batch);
    if (!batch || !target) fail(KC_E_INVAL, "empty batch or NULL targets");
    const hipStream_t st = (hipStream_t)stream;
    if (p->scratch_b < batch) {
      if (p->scratch) hipchk(hipFree(p->scratch), "hipFree");
      p->scratch = nullptr;
      p->scratch_b = 0;
      hipchk(hipMalloc(&p->scratch, batch * (2 * (size_t)p->H + 2) * sizeof(float)), "hipMalloc");
      p->scratch_b = batch;
    }
    float* dy = p->scratch;
    float* lossv = dy + batch;
    float* hbuf = lossv + batch;
    float* dh = hbuf + batch * p->H;
    hipLaunchKernelGGL(k_mlp_backprop, dim3(blocks(batch, 256)), dim3(256),
                       p->np * sizeof(float), st, p->prm, p->F, p->H, x, target, batch, dy, hbuf,
                       dh, lossv);
    hipchk(hipGetLastError(), "backprop launch");
    hipLaunchKernelGGL(k_mlp_reduce, dim3(blocks((uint64_t)p->np + 1, 256)), dim3(256), 0, st,
                       p->F, p->H, x, batch, dy, hbuf, dh, lossv, p->grad, p->loss);
    hipchk(hipGetLastError(), "gradient reduce launch");
    if (host_loss) {
      hipchk(hipMemcpyAsync(p->host, p->loss, sizeof(float), hipMemcpyDeviceToHost, st),
             "hipMemcpyAsync");
      hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
      *host_loss = p->host[0];
    }
    return KC_OK;
  });
}

int kc_pred_adam_step(kc_predictor* p, float lr, void* stream) {
  return guarded([&]() -> int {
    if (!p) fail(KC_E_INVAL, "predictor is NULL");
    if (!(lr > 0.0f)) fail(KC_E_INVAL, "learning rate must be > 0");
    const float b1 = 0.9f, b2 = 0.999f;
    ++p->step;
    const float c1 = 1.0f - std::pow(b1, (float)p->step);
    const float c2 = 1.0f - std::pow(b2, (float)p->step);
    hipLaunchKernelGGL(k_adam, dim3(blocks(p->np, 256)), dim3(256), 0, (hipStream_t)stream,
                       p->prm, p->grad, p->m, p->v, p->np, lr, b1, b2, 1e-8f, c1, c2);
    hipchk(hipGetLastError(), "adam launch");
    return KC_OK;
  });
}

void kc_pred_free(kc_predictor* p) {
  try {
    delete p;
  } catch (...) {
  }
}

}  // extern "C"
