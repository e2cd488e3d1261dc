// Random-gather rate probe: the bound of the sparse products.
//
// The products with Q, A and A' read every nonzero's column value x[col]
// from a vector that is gathered at random positions (the instance family
// draws its columns uniformly).  Their speed is set by how many such
// gathers the memory system serves per second, which depends on the
// gathered vector's size against the caches, not by the matrix stream's
// bytes.  This probe measures that rate with the access pattern of the
// CSR-stream kernels: each thread loads kStreamE indices with unit stride
// (non-temporal, like the matrix stream), then issues its kStreamE
// gathers at once and adds them; one sum per workgroup is written.
//
// With P > 1 column panels, the positions of tile b are drawn from panel
// b mod P only (the vector's P equal slices), and workgroup i processes the
// tiles b = i (mod grid) with grid a multiple of 8: since workgroups are
// dispatched round-robin over the 8 XCDs, the workgroups of one XCD then
// read one slice only, which is what a column-panel split of a sparse
// product would give.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <random>
#include <string>
#include <vector>

#include "../../include/pdnqp.h"
#include "pdnqp_kernels.hpp"

namespace pdnqp {

namespace {

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather_probe(const T *__restrict__ x,
                                                         const int32_t *__restrict__ idx,
                                                         int64_t count, double *__restrict__ out) {
  __shared__ double red[kBlock / 64];
  double s = 0.0;
  const int64_t per_block = (int64_t)kTile;
  for (int64_t base = (int64_t)blockIdx.x * per_block; base < count;
       base += (int64_t)gridDim.x * per_block) {
    int col[kStreamE];
#pragma unroll
    for (int e = 0; e < kStreamE; ++e) {
      const int64_t k = base + e * kBlock + threadIdx.x;
      col[e] = k < count ? __builtin_nontemporal_load(&idx[k]) : -1;
    }
#pragma unroll
    for (int e = 0; e < kStreamE; ++e)
      if (col[e] >= 0) s += (double)x[col[e]];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += red[w];
    out[blockIdx.x] = t;
  }
}

struct Buf {
  void *p = nullptr;
  ~Buf() {
    if (p) hipFree(p);
  }
};

int hipc(hipError_t e, const char *what, std::string &err) {
  if (e == hipSuccess) return PDNQP_OK;
  err = std::string(what) + ": " + hipGetErrorString(e);
  return PDNQP_E_DEVICE;
}

}  // namespace

int probe_gather(int32_t vec_len, int32_t elem_bytes, int64_t gathers, int32_t panels,
                 int32_t reps, uint64_t seed, double *rate, double *launch_us, std::string &err) {
  if (vec_len < 1 || (elem_bytes != 4 && elem_bytes != 8) || gathers < 1 || reps < 1 ||
      panels < 1 || panels > 8 || (8 % panels) != 0 || panels > vec_len) {
    err = "invalid probe arguments";
    return PDNQP_E_INVALID;
  }
  std::vector<int32_t> hidx((size_t)gathers);
  std::mt19937_64 rng(seed);
  const int32_t width = vec_len / panels;  // the last panel also takes the remainder
  for (int64_t k = 0; k < gathers; ++k) {
    const int p = (int)((k / kTile) % panels);
    const int32_t lo = p * width, hi = (p == panels - 1) ? vec_len - 1 : lo + width - 1;
    hidx[(size_t)k] = std::uniform_int_distribution<int32_t>(lo, hi)(rng);
  }
  int64_t tiles = (gathers + kTile - 1) / kTile;
  const int grid = (int)std::min<int64_t>((tiles + 7) / 8 * 8, 65536);
  Buf x, idx, out;
  int r;
  if ((r = hipc(hipMalloc(&x.p, (size_t)vec_len * elem_bytes), "hipMalloc", err)) ||
      (r = hipc(hipMalloc(&idx.p, (size_t)gathers * 4), "hipMalloc", err)) ||
      (r = hipc(hipMalloc(&out.p, (size_t)grid * 8), "hipMalloc", err)))
    return r;
  if ((r = hipc(hipMemset(x.p, 0, (size_t)vec_len * elem_bytes), "hipMemset", err)) ||
      (r = hipc(hipMemcpy(idx.p, hidx.data(), (size_t)gathers * 4, hipMemcpyHostToDevice),
                "index upload", err)))
    return r;
  auto launch = [&]() {
    if (elem_bytes == 8)
      hipLaunchKernelGGL(k_gather_probe<double>, dim3(grid), dim3(kBlock), 0, 0,
                         (const double *)x.p, (const int32_t *)idx.p, gathers, (double *)out.p);
    else
      hipLaunchKernelGGL(k_gather_probe<float>, dim3(grid), dim3(kBlock), 0, 0,
                         (const float *)x.p, (const int32_t *)idx.p, gathers, (double *)out.p);
  };
  launch();  // warm-up: brings the vector into the caches it fits
  if ((r = hipc(hipDeviceSynchronize(), "probe warm-up", err))) return r;
  hipEvent_t e0, e1;
  if ((r = hipc(hipEventCreate(&e0), "event", err))) return r;
  if ((r = hipc(hipEventCreate(&e1), "event", err))) {
    hipEventDestroy(e0);
    return r;
  }
  hipEventRecord(e0, 0);
  for (int k = 0; k < reps; ++k) launch();
  hipEventRecord(e1, 0);
  r = hipc(hipEventSynchronize(e1), "probe", err);
  float ms = 0.f;
  if (!r) r = hipc(hipEventElapsedTime(&ms, e0, e1), "probe timing", err);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (r) return r;
  if ((r = hipc(hipGetLastError(), "probe kernel", err))) return r;
  const double us = 1000.0 * ms / reps;
  if (launch_us) *launch_us = us;
  if (rate) *rate = (double)gathers / (us * 1e-6);
  return PDNQP_OK;
}

}  // namespace pdnqp
