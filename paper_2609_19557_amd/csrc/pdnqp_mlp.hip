// The learned outer-step controller's network on gfx950: a fully connected
// 16 -> 64 -> 64 -> 3 network with ReLU after the hidden layers, in FP32.
// Forward pass, gradient of the mean squared error over a batch of samples,
// and Adam updates, plus the host training loop over minibatches.
//
// Parameters are one flat FP32 vector: W1 (16x64, input index major), b1,
// W2 (64x64), b2, W3 (64x3), b3 -- 5443 values.  The contractions are tiny
// (at most 64x64 per sample), so they are plain FMA loops: one thread per
// hidden unit, the sample's activations in LDS; matrix cores would idle.
//
// Gradients are deterministic: each workgroup sums its samples' parameter
// gradients in a fixed order into its own partial vector, and a second
// kernel adds the partials in workgroup order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "../../include/pdnqp.h"

namespace pdnqp {

namespace {

constexpr int kIn = 16, kH = 64, kOut = 3;
constexpr int oW1 = 0, ob1 = oW1 + kIn * kH, oW2 = ob1 + kH, ob2 = oW2 + kH * kH,
              oW3 = ob2 + kH, ob3 = oW3 + kH * kOut, kParams = ob3 + kOut;  // 5443
constexpr int kSamplesPerBlock = 64;

// One workgroup of 64 threads per group of samples; thread j owns hidden
// unit j.  Forward only.
__global__ __launch_bounds__(kH) void k_mlp_forward(const float *__restrict__ th,
                                                    const float *__restrict__ X, int count,
                                                    float *__restrict__ Y) {
  __shared__ float x[kIn], h1[kH], h2[kH];
  const int j = threadIdx.x;
  for (int b = blockIdx.x; b < count; b += gridDim.x) {
    if (j < kIn) x[j] = X[(size_t)b * kIn + j];
    __syncthreads();
    float z = th[ob1 + j];
    for (int i = 0; i < kIn; ++i) z += x[i] * th[oW1 + i * kH + j];
    h1[j] = z > 0.f ? z : 0.f;
    __syncthreads();
    z = th[ob2 + j];
    for (int i = 0; i < kH; ++i) z += h1[i] * th[oW2 + i * kH + j];
    h2[j] = z > 0.f ? z : 0.f;
    __syncthreads();
    if (j < kOut) {
      float o = th[ob3 + j];
      for (int i = 0; i < kH; ++i) o += h2[i] * th[oW3 + i * kOut + j];
      Y[(size_t)b * kOut + j] = o;
    }
    __syncthreads();
  }
}

// Gradient of L = (1 / (count * 3)) sum (out - y)^2 for the samples of this
// workgroup, summed in sample order into partial[blockIdx.x][:], and the
// workgroup's part of the loss into lossp[blockIdx.x].
__global__ __launch_bounds__(kH) void k_mlp_grad(const float *__restrict__ th,
                                                 const float *__restrict__ X,
                                                 const float *__restrict__ Yt, int count,
                                                 float *__restrict__ partial,
                                                 float *__restrict__ lossp) {
  __shared__ float x[kIn], z1[kH], h1[kH], z2[kH], h2[kH], g2[kH], g1[kH], go[kOut];
  __shared__ float acc[kParams];
  __shared__ float lsum;
  const int j = threadIdx.x;
  for (int p = j; p < kParams; p += kH) acc[p] = 0.f;
  if (j == 0) lsum = 0.f;
  const float scale = 2.f / ((float)count * kOut);
  const int b0 = blockIdx.x * kSamplesPerBlock;
  const int b1 = std::min(count, b0 + kSamplesPerBlock);
  __syncthreads();
  for (int b = b0; b < b1; ++b) {
    if (j < kIn) x[j] = X[(size_t)b * kIn + j];
    __syncthreads();
    float z = th[ob1 + j];
    for (int i = 0; i < kIn; ++i) z += x[i] * th[oW1 + i * kH + j];
    z1[j] = z;
    h1[j] = z > 0.f ? z : 0.f;
    __syncthreads();
    z = th[ob2 + j];
    for (int i = 0; i < kH; ++i) z += h1[i] * th[oW2 + i * kH + j];
    z2[j] = z;
    h2[j] = z > 0.f ? z : 0.f;
    __syncthreads();
    if (j < kOut) {
      float o = th[ob3 + j];
      for (int i = 0; i < kH; ++i) o += h2[i] * th[oW3 + i * kOut + j];
      const float d = o - Yt[(size_t)b * kOut + j];
      go[j] = scale * d;
    }
    __syncthreads();
    if (j == 0) lsum += (go[0] * go[0] + go[1] * go[1] + go[2] * go[2]) / (scale * scale);
    // output layer
    for (int k = 0; k < kOut; ++k) acc[oW3 + j * kOut + k] += h2[j] * go[k];
    if (j < kOut) acc[ob3 + j] += go[j];
    // second hidden layer
    float gh = 0.f;
    for (int k = 0; k < kOut; ++k) gh += go[k] * th[oW3 + j * kOut + k];
    g2[j] = z2[j] > 0.f ? gh : 0.f;
    __syncthreads();
    for (int i = 0; i < kH; ++i) acc[oW2 + i * kH + j] += h1[i] * g2[j];
    acc[ob2 + j] += g2[j];
    gh = 0.f;
    for (int k = 0; k < kH; ++k) gh += g2[k] * th[oW2 + j * kH + k];
    g1[j] = z1[j] > 0.f ? gh : 0.f;
    __syncthreads();
    for (int i = 0; i < kIn; ++i) acc[oW1 + i * kH + j] += x[i] * g1[j];
    acc[ob1 + j] += g1[j];
    __syncthreads();
  }
  for (int p = j; p < kParams; p += kH) partial[(size_t)blockIdx.x * kParams + p] = acc[p];
  if (j == 0) lossp[blockIdx.x] = lsum;
}

// Loss of the batch from the workgroups' parts, added in workgroup order in
// FP64 (one thread: the same order and arithmetic as the host sum).
__global__ void k_mlp_loss(const float *__restrict__ lossp, int nblk, int count,
                           double *__restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += (double)lossp[b];
  *loss = s / ((double)count * kOut);
}

// Adds the workgroups' partial gradients in workgroup order.
__global__ __launch_bounds__(256) void k_mlp_reduce(const float *__restrict__ partial, int nblk,
                                                    float *__restrict__ grad) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= kParams) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += partial[(size_t)b * kParams + p];
  grad[p] = s;
}

__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ th,
                                                  const float *__restrict__ g,
                                                  float *__restrict__ m, float *__restrict__ v,
                                                  float lr, float c1, float c2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= kParams) return;
  const float gp = g[p];
  const float mn = 0.9f * m[p] + 0.1f * gp;
  const float vn = 0.999f * v[p] + 0.001f * gp * gp;
  m[p] = mn;
  v[p] = vn;
  th[p] -= lr * (mn / c1) / (sqrtf(vn / c2) + 1e-8f);
}

struct Dev {
  void *p = nullptr;
  ~Dev() {
    if (p) hipFree(p);
  }
  template <typename T>
  T *as() const {
    return (T *)p;
  }
};

int dev_alloc(Dev &d, size_t bytes, std::string &err) {
  if (hipMalloc(&d.p, bytes ? bytes : 16) != hipSuccess) {
    err = "device allocation failed";
    return PDNQP_E_NOMEM;
  }
  return PDNQP_OK;
}

int hipc(hipError_t e, const char *what, std::string &err) {
  if (e == hipSuccess) return PDNQP_OK;
  err = std::string(what) + ": " + hipGetErrorString(e);
  return PDNQP_E_DEVICE;
}

int nblocks(int count) { return (count + kSamplesPerBlock - 1) / kSamplesPerBlock; }

// gradient and loss of a device batch into device grad / host loss
int grad_on_device(const float *th, const float *X, const float *Y, int count, float *partial,
                   float *lossp, float *grad, double *loss, std::string &err) {
  const int nb = nblocks(count);
  hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(kH), 0, 0, th, X, Y, count, partial, lossp);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kParams + 255) / 256), dim3(256), 0, 0, partial, nb,
                     grad);
  if (loss) {
    std::vector<float> lp(nb);
    int r = hipc(hipMemcpy(lp.data(), lossp, nb * sizeof(float), hipMemcpyDeviceToHost),
                 "loss copy", err);
    if (r) return r;
    double s = 0.0;
    for (float x : lp) s += x;
    *loss = s / ((double)count * kOut);
  }
  return hipc(hipGetLastError(), "mlp kernels", err);
}

// Scratch of the allocation-free gradient: the per-workgroup partial
// gradients (kParams floats each) and loss parts of at most
// kNoAllocMaxBlocks workgroups, i.e. kNoAllocMaxSamples samples (5.6 MB).
// Each GPU the library runs on holds its own copy until the process ends.
constexpr int kNoAllocMaxSamples = PDNQP_MLP_NOALLOC_MAX;
constexpr int kNoAllocMaxBlocks = kNoAllocMaxSamples / kSamplesPerBlock;
static_assert(kNoAllocMaxSamples % kSamplesPerBlock == 0, "whole workgroups");
constexpr size_t kScratchFloats = (size_t)kNoAllocMaxBlocks * kParams + kNoAllocMaxBlocks;

}  // namespace

static __device__ __align__(256) float scratch[kScratchFloats];

namespace {

// Device address of `scratch` per device, looked up once per device with the
// device current (in host code the array's name is only a stand-in).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};

int scratch_on_current_device(float **out, std::string &err) {
  int dev = 0;
  int r = hipc(hipGetDevice(&dev), "hipGetDevice", err);
  if (r) return r;
  if (dev < 0 || dev >= kMaxDevices) {
    err = "device index out of range";
    return PDNQP_E_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if ((r = hipc(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress", err)))
      return r;
    if (!p) {
      err = "hipGetSymbolAddress returned no address";
      return PDNQP_E_DEVICE;
    }
    g_scratch_ptr[dev] = (float *)p;
  }
  *out = g_scratch_ptr[dev];
  return PDNQP_OK;
}

}  // namespace

int mlp_param_count() { return kParams; }

// The gradient of mlp_gradient on caller-owned device buffers, with the
// per-workgroup partials in the static scratch array: no device allocation,
// no synchronisation (the work is enqueued on `st`).
int mlp_gradient_noalloc(const float *theta, const float *X, const float *Y, int count,
                         float *grad, double *loss, hipStream_t st, std::string &err) {
  if (count < 1 || count > kNoAllocMaxSamples) {
    err = "count must be in [1, " + std::to_string(kNoAllocMaxSamples) + "]";
    return PDNQP_E_INVALID;
  }
  float *sp = nullptr;
  int r = scratch_on_current_device(&sp, err);
  if (r) return r;
  const int nb = nblocks(count);
  float *partial = sp;
  float *lossp = sp + (size_t)kNoAllocMaxBlocks * kParams;
  hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(kH), 0, st, theta, X, Y, count, partial, lossp);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kParams + 255) / 256), dim3(256), 0, st, partial, nb,
                     grad);
  if (loss) hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(64), 0, st, lossp, nb, count, loss);
  return hipc(hipGetLastError(), "mlp kernels", err);
}

// Device-side forward of one feature vector with parameters already on the
// device (the solver's controller).
void mlp_forward_device(hipStream_t st, const float *th, const float *x, float *y) {
  hipLaunchKernelGGL(k_mlp_forward, dim3(1), dim3(kH), 0, st, th, x, 1, y);
}

int mlp_forward(const float *theta, const float *X, int count, float *Y, std::string &err) {
  Dev t, x, y;
  int r;
  if ((r = dev_alloc(t, kParams * 4, err)) || (r = dev_alloc(x, (size_t)count * kIn * 4, err)) ||
      (r = dev_alloc(y, (size_t)count * kOut * 4, err)))
    return r;
  if ((r = hipc(hipMemcpy(t.p, theta, kParams * 4, hipMemcpyHostToDevice), "copy", err)) ||
      (r = hipc(hipMemcpy(x.p, X, (size_t)count * kIn * 4, hipMemcpyHostToDevice), "copy", err)))
    return r;
  const int grid = std::max(1, std::min(count, 4096));
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(kH), 0, 0, t.as<float>(), x.as<float>(),
                     count, y.as<float>());
  if ((r = hipc(hipGetLastError(), "mlp forward", err))) return r;
  return hipc(hipMemcpy(Y, y.p, (size_t)count * kOut * 4, hipMemcpyDeviceToHost), "copy", err);
}

int mlp_gradient(const float *theta, const float *X, const float *Y, int count, float *grad,
                 double *loss, std::string &err) {
  Dev t, x, y, part, lp, g;
  const int nb = nblocks(count);
  int r;
  if ((r = dev_alloc(t, kParams * 4, err)) || (r = dev_alloc(x, (size_t)count * kIn * 4, err)) ||
      (r = dev_alloc(y, (size_t)count * kOut * 4, err)) ||
      (r = dev_alloc(part, (size_t)nb * kParams * 4, err)) || (r = dev_alloc(lp, nb * 4, err)) ||
      (r = dev_alloc(g, kParams * 4, err)))
    return r;
  if ((r = hipc(hipMemcpy(t.p, theta, kParams * 4, hipMemcpyHostToDevice), "copy", err)) ||
      (r = hipc(hipMemcpy(x.p, X, (size_t)count * kIn * 4, hipMemcpyHostToDevice), "copy", err)) ||
      (r = hipc(hipMemcpy(y.p, Y, (size_t)count * kOut * 4, hipMemcpyHostToDevice), "copy", err)))
    return r;
  if ((r = grad_on_device(t.as<float>(), x.as<float>(), y.as<float>(), count, part.as<float>(),
                          lp.as<float>(), g.as<float>(), loss, err)))
    return r;
  return hipc(hipMemcpy(grad, g.p, kParams * 4, hipMemcpyDeviceToHost), "copy", err);
}

// Adam over shuffled minibatches (seeded); loss_curve[e] = training loss
// after epoch e.
int mlp_train(float *theta, const float *X, const float *Y, int count, int epochs, int batch,
              float lr, uint64_t seed, float *loss_curve, std::string &err) {
  Dev t, x, y, xb, yb, part, lp, g, m, v;
  const int nb = nblocks(batch);
  int r;
  if ((r = dev_alloc(t, kParams * 4, err)) || (r = dev_alloc(x, (size_t)count * kIn * 4, err)) ||
      (r = dev_alloc(y, (size_t)count * kOut * 4, err)) ||
      (r = dev_alloc(xb, (size_t)batch * kIn * 4, err)) ||
      (r = dev_alloc(yb, (size_t)batch * kOut * 4, err)) ||
      (r = dev_alloc(part, (size_t)std::max(nb, nblocks(count)) * kParams * 4, err)) ||
      (r = dev_alloc(lp, (size_t)std::max(nb, nblocks(count)) * 4, err)) ||
      (r = dev_alloc(g, kParams * 4, err)) || (r = dev_alloc(m, kParams * 4, err)) ||
      (r = dev_alloc(v, kParams * 4, err)))
    return r;
  if ((r = hipc(hipMemcpy(t.p, theta, kParams * 4, hipMemcpyHostToDevice), "copy", err)) ||
      (r = hipc(hipMemcpy(x.p, X, (size_t)count * kIn * 4, hipMemcpyHostToDevice), "copy", err)) ||
      (r = hipc(hipMemcpy(y.p, Y, (size_t)count * kOut * 4, hipMemcpyHostToDevice), "copy", err)) ||
      (r = hipc(hipMemset(m.p, 0, kParams * 4), "memset", err)) ||
      (r = hipc(hipMemset(v.p, 0, kParams * 4), "memset", err)))
    return r;
  std::mt19937_64 rng(seed);
  std::vector<int> idx(count);
  std::vector<float> hx((size_t)batch * kIn), hy((size_t)batch * kOut);
  int64_t step = 0;
  for (int e = 0; e < epochs; ++e) {
    for (int i = 0; i < count; ++i) idx[i] = i;
    std::shuffle(idx.begin(), idx.end(), rng);
    for (int s0 = 0; s0 + batch <= count || (s0 < count && s0 == 0); s0 += batch) {
      const int bs = std::min(batch, count - s0);
      for (int k = 0; k < bs; ++k) {
        std::memcpy(&hx[(size_t)k * kIn], &X[(size_t)idx[s0 + k] * kIn], kIn * 4);
        std::memcpy(&hy[(size_t)k * kOut], &Y[(size_t)idx[s0 + k] * kOut], kOut * 4);
      }
      if ((r = hipc(hipMemcpy(xb.p, hx.data(), (size_t)bs * kIn * 4, hipMemcpyHostToDevice),
                    "copy", err)) ||
          (r = hipc(hipMemcpy(yb.p, hy.data(), (size_t)bs * kOut * 4, hipMemcpyHostToDevice),
                    "copy", err)))
        return r;
      if ((r = grad_on_device(t.as<float>(), xb.as<float>(), yb.as<float>(), bs, part.as<float>(),
                              lp.as<float>(), g.as<float>(), nullptr, err)))
        return r;
      ++step;
      const float c1 = 1.f - std::pow(0.9f, (float)step);
      const float c2 = 1.f - std::pow(0.999f, (float)step);
      hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + 255) / 256), dim3(256), 0, 0, t.as<float>(),
                         g.as<float>(), m.as<float>(), v.as<float>(), lr, c1, c2);
    }
    if (loss_curve) {
      double l = 0.0;
      if ((r = grad_on_device(t.as<float>(), x.as<float>(), y.as<float>(), count,
                              part.as<float>(), lp.as<float>(), g.as<float>(), &l, err)))
        return r;
      loss_curve[e] = (float)l;
    }
  }
  if ((r = hipc(hipGetLastError(), "mlp training", err))) return r;
  return hipc(hipMemcpy(theta, t.p, kParams * 4, hipMemcpyDeviceToHost), "copy", err);
}

}  // namespace pdnqp
