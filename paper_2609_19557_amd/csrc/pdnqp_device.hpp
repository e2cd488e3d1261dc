// Device helpers shared by the kernel files: sparse row products (row-group
// and CSR-stream forms), deterministic block reductions, row/element loops.
//
// Reductions are deterministic: each workgroup writes its partial in a fixed
// slot and a later one-workgroup kernel (or the last workgroup of a cold
// kernel) combines the partials in a fixed order.  There are no
// floating-point atomics.
#pragma once

#include "pdnqp_kernels.hpp"

namespace pdnqp {
namespace dev {

constexpr int kWaves = kBlock / 64;
constexpr int kDecideThreads = 1024;
// slots of the reduction buffer used by the per-trial kernels
constexpr int PS_X = 0;    // x trial: sum dx^2 / taub_x
constexpr int PS_ROW = 1;  // rows (4 slots)
constexpr int PS_AT = 5;   // A' kernel (2 slots)

template <typename T>
__device__ __forceinline__ T clampv(T v, T lo, T hi) {
  // NaN propagates (comparisons with NaN are false), like numpy.clip.
  return v < lo ? lo : (v > hi ? hi : v);
}

template <typename T>
__device__ __forceinline__ T maxv(T v, T lo) {
  return v < lo ? lo : v;
}

// Row-group product: G consecutive lanes share a row, read its entries with
// unit stride and combine with in-group shuffles.  All lanes of the group
// receive the sum.
template <int G, typename T>
__device__ __forceinline__ T row_dot(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                     const T *__restrict__ val, const T *__restrict__ x, int row,
                                     int lane) {
  const int beg = rp[row];
  const int end = rp[row + 1];
  T acc = T(0);
  for (int k = beg + lane; k < end; k += G) {
    acc += __builtin_nontemporal_load(&val[k]) * x[__builtin_nontemporal_load(&ci[k])];
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
  return acc;
}

// Block-level reduction of K values (bit k of maxmask: max instead of sum);
// thread 0 writes out[k * kMaxParts + slot].
template <int K>
__device__ __forceinline__ void block_reduce(double (&v)[K], uint32_t maxmask, double *out,
                                             int slot) {
  __shared__ double sh[kWaves][K];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = v[k];
    const bool mx = (maxmask >> k) & 1u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_down(x, off, 64);
      x = mx ? fmax(x, o) : x + o;
    }
    if (lane == 0) sh[wid][k] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool mx = (maxmask >> k) & 1u;
      double acc = sh[0][k];
      for (int w = 1; w < kWaves; ++w) acc = mx ? fmax(acc, sh[w][k]) : acc + sh[w][k];
      out[k * kMaxParts + slot] = acc;
    }
  }
}

// Called by every thread after block_reduce in kernels that run a few times
// per outer step.  Returns true in the last workgroup of the grid to arrive;
// its threads then see every partial.  (The device-scope fence writes back
// the XCD's L2, so per-trial kernels use a separate reduction kernel.)
__device__ __forceinline__ bool last_block(uint32_t *ticket, uint32_t nblocks) {
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t t = atomicAdd(ticket, 1u);
    s_last = (t == nblocks - 1u);
  }
  __syncthreads();
  if (s_last) __threadfence();
  return s_last != 0;
}

// Fixed-order combination of nparts partials of K values (all threads of the
// block take part); thread 0 receives the results.
template <int K>
__device__ __forceinline__ void final_reduce(const double *part, int nparts, uint32_t maxmask,
                                             double (&res)[K]) {
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double x = __builtin_nontemporal_load(&part[k * kMaxParts + i]);
      v[k] = ((maxmask >> k) & 1u) ? fmax(v[k], x) : v[k] + x;
    }
  }
  __shared__ double sh[kWaves][K];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = v[k];
    const bool mx = (maxmask >> k) & 1u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_down(x, off, 64);
      x = mx ? fmax(x, o) : x + o;
    }
    if (lane == 0) sh[wid][k] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool mx = (maxmask >> k) & 1u;
      double acc = sh[0][k];
      for (int w = 1; w < kWaves; ++w) acc = mx ? fmax(acc, sh[w][k]) : acc + sh[w][k];
      res[k] = acc;
    }
  }
}

// Iterates the rows of one part: calls f(row, lane) for every row handled by
// this workgroup (`b` = block index within the part, `nb` = blocks of the part).
template <int G, typename F>
__device__ __forceinline__ void for_rows(int rows, int b, int nb, F &&f) {
  constexpr int RPB = kBlock / G;
  const int lane = threadIdx.x % G;
  const int rl = threadIdx.x / G;
  for (int r0 = b * RPB; r0 < rows; r0 += nb * RPB) {
    const int row = r0 + rl;
    if (row < rows) f(row, lane);
  }
}

template <typename F>
__device__ __forceinline__ void for_elems(int n, int b, int nb, F &&f) {
  for (int i = b * kBlock + threadIdx.x; i < n; i += nb * kBlock) f(i);
}

// One row block of a CSR-stream product as a pipeline stage: the matrix it
// belongs to (tag tells the caller which), its rows [r0, r1), its nonzeros
// [base, base + cnt) and, once loaded, this thread's E of them.
template <typename T, int E>
struct StreamTile {
  const int32_t *p;
  const int32_t *ci;
  const T *cv;
  int tag, r0, r1, base, cnt;
  int col[E];
  T val[E];
};

// Fills the bounds of row block b of M: the row range from M.rb[0..nrb] and
// the nonzero range from the offsets stored after it, M.rb[nrb + 1 + b].
template <typename T, int E>
__device__ __forceinline__ void tile_bounds(const CsrT<T> &M, int b, int tag,
                                            StreamTile<T, E> &t) {
  t.p = M.p;
  t.ci = M.i;
  t.cv = M.v;
  t.tag = tag;
  t.r0 = M.rb[b];
  t.r1 = M.rb[b + 1];
  const int32_t *nz = M.rb + M.nrb + 1;
  t.base = nz[b];
  t.cnt = nz[b + 1] - t.base;
}

// Loads this thread's nonzeros of a tile with unit stride (nothing for a
// block holding a single row longer than a tile).
template <typename T, int E>
__device__ __forceinline__ void tile_load(StreamTile<T, E> &t) {
  const bool fits = t.cnt <= E * kBlock;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = e * kBlock + threadIdx.x;
    t.col[e] = 0;
    t.val[e] = T(0);
    if (fits && k < t.cnt) {
      t.col[e] = __builtin_nontemporal_load(&t.ci[t.base + k]);
      t.val[e] = __builtin_nontemporal_load(&t.cv[t.base + k]);
    }
  }
}

// Software-pipelined CSR-stream products over the row blocks it0, it0 +
// step, ... (< items) of one workgroup, for row blocks of at most E * kBlock
// nonzeros (a longer block holds a single row).  sel(it, tile) fills a
// tile's bounds.  While the gathers of block it are in flight the nonzeros
// of the next block are loaded, and the bounds of the one after are read at
// the end of each step, so a workgroup keeps the matrix stream and the
// gathers of x busy at the same time instead of in turn.  Products are
// staged in LDS (sprod: E * kBlock entries) and one thread per row adds its
// products in order, so each row's sum does not depend on the grid;
// emit(tag, row, sum) runs on that thread.  A block holding a single row
// longer than a tile sums it with a block reduction instead and calls emit
// on thread 0.
template <typename T, int E, typename Sel, typename Emit>
__device__ __forceinline__ void stream_pipelined(int it0, int items, int step,
                                                 const T *__restrict__ x, T *__restrict__ sprod,
                                                 Sel &&sel, Emit &&emit) {
  if (it0 >= items) return;
  StreamTile<T, E> cur, nxt;
  sel(it0, cur);
  tile_load(cur);
  int nit = it0 + step;
  if (nit < items) sel(nit, nxt);
  for (;;) {
    const bool more = nit < items;
    if (cur.cnt <= E * kBlock) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int k = e * kBlock + threadIdx.x;
        if (k < cur.cnt) cur.val[e] = cur.val[e] * x[cur.col[e]];
      }
      if (more) tile_load(nxt);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int k = e * kBlock + threadIdx.x;
        if (k < cur.cnt) sprod[k] = cur.val[e];
      }
      __syncthreads();
      for (int row = cur.r0 + (int)threadIdx.x; row < cur.r1; row += kBlock) {
        const int a = cur.p[row] - cur.base;
        const int b = cur.p[row + 1] - cur.base;
        T s = T(0);
        for (int k = a; k < b; ++k) s += sprod[k];
        emit(cur.tag, row, s);
      }
      __syncthreads();
    } else {
      if (more) tile_load(nxt);
      __shared__ T red[kWaves];
      T s = T(0);
      for (int k = threadIdx.x; k < cur.cnt; k += kBlock)
        s += cur.cv[cur.base + k] * x[cur.ci[cur.base + k]];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
      __syncthreads();
      if (threadIdx.x == 0) {
        T t = red[0];
        for (int w = 1; w < kWaves; ++w) t += red[w];
        emit(cur.tag, cur.r0, t);
      }
      __syncthreads();
    }
    if (!more) break;
    cur = nxt;
    nit += step;
    if (nit < items) sel(nit, nxt);
  }
}

}  // namespace dev
}  // namespace pdnqp

// Dispatch on the lanes-per-row template parameter.
#define PDNQP_DISPATCH_G(G, ...)                            \
  switch (G) {                                              \
    case 2: { constexpr int GV = 2; __VA_ARGS__; break; }   \
    case 4: { constexpr int GV = 4; __VA_ARGS__; break; }   \
    case 8: { constexpr int GV = 8; __VA_ARGS__; break; }   \
    case 16: { constexpr int GV = 16; __VA_ARGS__; break; } \
    default: { constexpr int GV = 32; __VA_ARGS__; break; } \
  }
