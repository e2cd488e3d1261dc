// gfx950 kernels of the PDNQP hot path.
//
// Sparse products use CSR with G consecutive lanes per row (G a power of
// two chosen from the mean row length): the lanes of a group read the row's
// values and column indices with unit stride, so a wave64 covers 64/G
// consecutive rows in one contiguous stretch of the value/index arrays; the
// gathered vector entries are the only irregular accesses.  Row sums are
// combined with in-group shuffles.  Nothing here is a dense contraction, so
// no matrix-core instructions are used: every kernel is bound by HBM (or
// cache) bandwidth.
//
// Reductions are deterministic: each workgroup writes its partial in a fixed
// slot, and the last workgroup to finish (integer ticket) combines the
// partials in a fixed order.  There are no floating-point atomics.
#include "pdnqp_kernels.hpp"

#include <cmath>

namespace pdnqp {

namespace {

constexpr int kWaves = kBlock / 64;
constexpr int kDecideThreads = 1024;
// slots of the reduction buffer used by the per-trial kernels
constexpr int PS_X = 0;    // x trial: sum dx^2 / taub_x
constexpr int PS_ROW = 1;  // rows (4 slots)
constexpr int PS_AT = 5;   // A' kernel (2 slots)

__device__ __forceinline__ double clampd(double v, double lo, double hi) {
  // NaN propagates (comparisons with NaN are false), like numpy.clip.
  return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ double maxd(double v, double lo) { return v < lo ? lo : v; }

template <int G>
__device__ __forceinline__ double row_dot(const int32_t *__restrict__ rp,
                                          const int32_t *__restrict__ ci,
                                          const double *__restrict__ val,
                                          const double *__restrict__ x, int row, int lane) {
  const int beg = rp[row];
  const int end = rp[row + 1];
  double acc = 0.0;
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

// Called by every thread after block_reduce.  Returns true in the last
// workgroup of the grid to arrive; its threads then see every partial.
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
// last block take part); thread 0 receives the results.
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

// CSR-stream row sums of rows [r0, r1) of M x.  The workgroup loads the
// block's nonzeros with unit stride (kStreamE per thread, all independent),
// gathers x for all of them at once, stages the products in LDS and lets
// one thread per row add its products in order; f(row, sum) runs on that
// thread.  A block holding a single row longer than a tile sums it with a
// block reduction instead and calls f on thread 0.
template <typename F>
__device__ __forceinline__ void stream_rows(const Csr &M, const double *__restrict__ x, int r0,
                                            int r1, double *__restrict__ sprod, F &&f) {
  const int base = M.p[r0];
  const int cnt = M.p[r1] - base;
  if (cnt <= kTile) {
    int col[kStreamE];
    double val[kStreamE];
#pragma unroll
    for (int e = 0; e < kStreamE; ++e) {
      const int k = e * kBlock + threadIdx.x;
      col[e] = 0;
      val[e] = 0.0;
      if (k < cnt) {
        col[e] = __builtin_nontemporal_load(&M.i[base + k]);
        val[e] = __builtin_nontemporal_load(&M.v[base + k]);
      }
    }
#pragma unroll
    for (int e = 0; e < kStreamE; ++e) {
      const int k = e * kBlock + threadIdx.x;
      if (k < cnt) sprod[k] = val[e] * x[col[e]];
    }
    __syncthreads();
    for (int row = r0 + (int)threadIdx.x; row < r1; row += kBlock) {
      const int a = M.p[row] - base;
      const int b = M.p[row + 1] - base;
      double s = 0.0;
      for (int k = a; k < b; ++k) s += sprod[k];
      f(row, s);
    }
    __syncthreads();
  } else {
    __shared__ double red[kWaves];
    double s = 0.0;
    for (int k = threadIdx.x; k < cnt; k += kBlock) s += M.v[base + k] * x[M.i[base + k]];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = red[0];
      for (int w = 1; w < kWaves; ++w) t += red[w];
      f(r0, t);
    }
    __syncthreads();
  }
}

// Dispatch on the lanes-per-row template parameter.
#define PDNQP_DISPATCH_G(G, ...)                        \
  switch (G) {                                          \
    case 2: { constexpr int GV = 2; __VA_ARGS__; break; }   \
    case 4: { constexpr int GV = 4; __VA_ARGS__; break; }   \
    case 8: { constexpr int GV = 8; __VA_ARGS__; break; }   \
    case 16: { constexpr int GV = 16; __VA_ARGS__; break; } \
    default: { constexpr int GV = 32; __VA_ARGS__; break; } \
  }

// ===========================================================================
// Trial step, x block (eq. (pdqp-trial), primal line, x components):
//   x_tr = clip(x - tau (q_x + (1-a) H xbar + a H x - A'y), xl, xu),
// H x = Q x + x / gamma.  Also applies the previous accept's averaging
// (xbar <- (1-a') xbar + a' x, Q xbar likewise) and accumulates
// sum dx^2 / taub_x for the acceptance test.
// ===========================================================================
__global__ __launch_bounds__(kBlock) void k_xtrial(Ctrl *__restrict__ c, InnerParams p, Vecs v,
                                                   Part px) {
  if (c->state != ST_RUNNING) return;
  const int cur = c->cur;
  const int pend = c->pending;
  const double ap = c->alpha_pend;
  const double Nd = (double)c->N;
  const double alpha = 2.0 / (Nd + 2.0);
  const double sct = c->step_scale / c->omega;
  const double gi = p.gamma_inv;
  const double *__restrict__ x = v.X[cur];
  const double *__restrict__ qx = v.QX[cur];
  const double *__restrict__ aty = v.ATY[cur];
  const double *__restrict__ ql = v.qx;
  const double *__restrict__ tbx = v.taub_x;
  const double *__restrict__ lo = v.lo;
  const double *__restrict__ hi = v.hi;
  double *__restrict__ xt = v.X[cur ^ 1];
  double *__restrict__ xbar = v.xbar;
  double *__restrict__ qxbar = v.qxbar;
  constexpr int U = 4;
  const int stride = gridDim.x * kBlock;
  double acc = 0.0;
  for (int i0 = blockIdx.x * kBlock + threadIdx.x; i0 < p.n; i0 += U * stride) {
    double xi[U], qxi[U], xb[U], qb[U], ay[U], qv[U], tb[U], l[U], h[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * stride;
      if (i < p.n) {
        xi[u] = x[i]; qxi[u] = qx[i]; xb[u] = xbar[i]; qb[u] = qxbar[i]; ay[u] = aty[i];
        qv[u] = ql[i]; tb[u] = tbx[i]; l[u] = lo[i]; h[u] = hi[i];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * stride;
      if (i < p.n) {
        double xbu = xb[u], qbu = qb[u];
        if (pend) {
          xbu = (1.0 - ap) * xbu + ap * xi[u];
          qbu = (1.0 - ap) * qbu + ap * qxi[u];
          xbar[i] = xbu;
          qxbar[i] = qbu;
        }
        const double hx = qxi[u] + gi * xi[u];
        const double hb = qbu + gi * xbu;
        const double g = qv[u] + (1.0 - alpha) * hb + alpha * hx - ay[u];
        const double xn = clampd(xi[u] - (sct * tb[u]) * g, l[u], h[u]);
        xt[i] = xn;
        const double d = xn - xi[u];
        acc += d * d / tb[u];
      }
    }
  }
  double vals[1] = {acc};
  block_reduce<1>(vals, 0u, v.partial + PS_X * kMaxParts, blockIdx.x);
}

// ===========================================================================
// Trial step, sparse part 1, CSR-stream form (one launch, two partitions):
// row blocks of Q (Q x_tr) and of A (A x_tr with the row-local s/r/y trial,
// the previous accept's averaging of ybar, rbar, sbar and the row-block
// acceptance sums).  Same arithmetic as the row-group form below.
// ===========================================================================
__global__ __launch_bounds__(kBlock) void k_qa_stream(Ctrl *__restrict__ c, InnerParams p,
                                                      Vecs v, Csr Q, Csr A, int gq, int ga) {
  if (c->state != ST_RUNNING) return;
  __shared__ double sprod[kTile];
  const int cur = c->cur;
  const int nxt = cur ^ 1;
  const double *__restrict__ xt = v.X[nxt];
  if ((int)blockIdx.x < gq) {
    double *__restrict__ qxt = v.QX[nxt];
    const double *__restrict__ qd = v.qdiag;
    for (int rb = blockIdx.x; rb < Q.nrb; rb += gq)
      stream_rows(Q, xt, Q.rb[rb], Q.rb[rb + 1], sprod,
                  [&](int row, double s) { qxt[row] = s + qd[row] * xt[row]; });
  } else {
    const int b = blockIdx.x - gq;
    const int pend = c->pending;
    const double ap = c->alpha_pend;
    const double Nd = (double)c->N;
    const double alpha = 2.0 / (Nd + 2.0);
    const double beta = Nd / (Nd + 1.0);
    const double sct = c->step_scale / c->omega;
    const double scy = c->step_scale * c->omega;
    const int me = p.me;
    double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
    for (int rb = b; rb < A.nrb; rb += ga) {
      stream_rows(A, xt, A.rb[rb], A.rb[rb + 1], sprod, [&](int j, double ax) {
        const double y = v.Y[cur][j];
        const double bw = v.BW[cur][j];
        const double r = v.R[cur][j];
        const double sg = v.sigma[j];
        const double lm = v.lam[j];
        const double bj = v.b[j];
        double rb_ = v.rbar[j];
        if (pend) {
          v.ybar[j] = (1.0 - ap) * v.ybar[j] + ap * y;
          rb_ = (1.0 - ap) * rb_ + ap * r;
          v.rbar[j] = rb_;
        }
        const double gr = (1.0 - alpha) * (sg * rb_) + alpha * (sg * r) + lm + y;
        const double tbr = v.taub_r[j];
        const double rt = r - (sct * tbr) * gr;
        double bwt, hj, ds = 0.0, ds2t = 0.0;
        if (j < me) {
          bwt = ax - rt;
          hj = bj;
        } else {
          const int k = j - me;
          const double sv = v.S[cur][k];
          if (pend) v.sbar[k] = (1.0 - ap) * v.sbar[k] + ap * sv;
          const double tbs = v.taub_s[k];
          const double st = maxd(sv - (sct * tbs) * y, bj);
          v.S[nxt][k] = st;
          bwt = ax - st - rt;
          hj = 0.0;
          ds = st - sv;
          ds2t = ds * ds / tbs;
        }
        const double eb = v.etab[j];
        const double yt = y + (scy * eb) * (hj - bwt - beta * (bwt - bw));
        v.R[nxt][j] = rt;
        v.BW[nxt][j] = bwt;
        v.Y[nxt][j] = yt;
        const double dr = rt - r;
        const double dy = yt - y;
        s1 += dr * dr / tbr + ds2t;
        s2 += dy * dy / eb;
        s3 += fabs(dr * (sg * dr));
        s4 += fabs(dr * dy) + fabs(ds * dy);
      });
    }
    double vals[4] = {s1, s2, s3, s4};
    block_reduce<4>(vals, 0u, v.partial + PS_ROW * kMaxParts, b);
  }
}

// Decision of the acceptance test (adaptive-condition) from the three
// kernels' sums; run by one thread.  All control-block fields are loaded
// first (one batch of independent loads) and written back at the end.
__device__ void accept_decision(Ctrl *__restrict__ c, const InnerParams &p, const Vecs &v,
                                double sx, const double (&sr)[4], double sum_hdx,
                                double sum_bdy) {
  const int cur = c->cur;
  const int N = c->N, t = c->t, t_call = c->t_call, rejects = c->rejects;
  const int ntr = c->trace_trials_n;
  const double sc = c->step_scale;
  const double om = c->omega;
  const int64_t trials = c->trials, accepted = c->accepted, rejected = c->rejected;
  const double L = 0.5 * ((om / sc) * (sx + sr[0]) + sr[1] / (sc * om));
  const double R = 0.5 * (sum_hdx + sr[2]) + (sum_bdy + sr[3]);
  c->sum_x = sx;
  for (int k = 0; k < 4; ++k) c->sum_row[k] = sr[k];
  c->L = L;
  c->R = R;
  c->trials = trials + 1;
  const bool finite = isfinite(L) && isfinite(R);
  const bool acc = finite && (L >= R);
  if (ntr < p.trace_trials_cap) {
    v.trace_tr[3 * ntr + 0] = L;
    v.trace_tr[3 * ntr + 1] = R;
    v.trace_tr[3 * ntr + 2] = acc ? 1.0 : 0.0;
    c->trace_trials_n = ntr + 1;
  }
  c->last_acc = acc ? 1 : 0;
  if (!finite) {
    c->state = ST_NUMERR;
    c->pending = 0;
  } else if (acc) {
    c->alpha_pend = 2.0 / ((double)N + 2.0);
    c->pending = 1;
    c->cur = cur ^ 1;
    c->N = N + 1;
    c->t = t + 1;
    c->t_call = t_call + 1;
    c->rejects = 0;
    c->accepted = accepted + 1;
    if (((t + 1) % p.check_every) == 0 || t_call + 1 >= p.max_inner) c->state = ST_CHECK_DUE;
  } else {
    double kappa = p.shrink_safety * L / R;
    kappa = kappa < p.shrink_min ? p.shrink_min : (kappa > p.shrink_max ? p.shrink_max : kappa);
    c->step_scale = kappa * sc;
    c->pending = 0;
    c->rejects = rejects + 1;
    c->rejected = rejected + 1;
    if (rejects + 1 >= p.max_rejects) c->state = ST_NUMERR;
  }
}

// Trial step, sparse part 2, CSR-stream form: row blocks of A' (A' y_tr),
// the x-block acceptance sums, and the decision in the last workgroup.
__global__ __launch_bounds__(kBlock) void k_at_stream(Ctrl *__restrict__ c, InnerParams p,
                                                      Vecs v, Csr AT) {
  if (c->state != ST_RUNNING) return;
  __shared__ double sprod[kTile];
  const int cur = c->cur;
  const int nxt = cur ^ 1;
  const double gi = p.gamma_inv;
  const double *__restrict__ yt = v.Y[nxt];
  double s5 = 0.0, s6 = 0.0;
  for (int rb = blockIdx.x; rb < AT.nrb; rb += gridDim.x) {
    stream_rows(AT, yt, AT.rb[rb], AT.rb[rb + 1], sprod, [&](int i, double a) {
      v.ATY[nxt][i] = a;
      const double dx = v.X[nxt][i] - v.X[cur][i];
      const double hdx = (v.QX[nxt][i] - v.QX[cur][i]) + gi * dx;
      const double ady = a - v.ATY[cur][i];
      s5 += fabs(dx * hdx);
      s6 += fabs(dx * ady);
    });
  }
  double vals[2] = {s5, s6};
  block_reduce<2>(vals, 0u, v.partial + PS_AT * kMaxParts, blockIdx.x);
}

// Acceptance test of the trial: one workgroup adds the partials of the three
// trial kernels in a fixed order (the kernel boundaries order their writes;
// no fences are needed) and takes the decision.
__global__ __launch_bounds__(kDecideThreads) void k_decide(Ctrl *__restrict__ c, InnerParams p,
                                                           Vecs v, int gx, int ga, int gt) {
  const int state = c->state;
  const double *part = v.partial;
  double a[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) a[k] = 0.0;
  // all loads of this thread are independent (one batch of up to 28)
  constexpr int PER = kMaxParts / kDecideThreads;
  double lx[PER], lr[PER][4], lt[PER][2];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int i = threadIdx.x + j * kDecideThreads;
    lx[j] = i < gx ? part[PS_X * kMaxParts + i] : 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) lr[j][k] = i < ga ? part[(PS_ROW + k) * kMaxParts + i] : 0.0;
    lt[j][0] = i < gt ? part[PS_AT * kMaxParts + i] : 0.0;
    lt[j][1] = i < gt ? part[(PS_AT + 1) * kMaxParts + i] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    a[0] += lx[j];
#pragma unroll
    for (int k = 0; k < 4; ++k) a[1 + k] += lr[j][k];
    a[5] += lt[j][0];
    a[6] += lt[j][1];
  }
  if (state != ST_RUNNING) return;
  __shared__ double sh[kDecideThreads / 64][7];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    double x = a[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) sh[wid][k] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[7];
    for (int k = 0; k < 7; ++k) {
      double acc = sh[0][k];
      for (int w = 1; w < kDecideThreads / 64; ++w) acc += sh[w][k];
      r[k] = acc;
    }
    const double sr[4] = {r[1], r[2], r[3], r[4]};
    accept_decision(c, p, v, r[0], sr, r[5], r[6]);
  }
}

// Copies the accepted iterate (x, s, r, y) into the trace buffers.
__global__ __launch_bounds__(kBlock) void k_trace(Ctrl *__restrict__ c, InnerParams p, Vecs v) {
  if (!c->last_acc || c->trace_iters_n >= p.trace_iters_cap) return;
  const int k = c->trace_iters_n;
  const int cur = c->cur;
  const int n = p.n, mi = p.mi, m = p.m, dw = p.dw;
  double *tw = v.trace_w + (size_t)k * dw;
  double *ty = v.trace_y + (size_t)k * m;
  for_elems(dw + m, blockIdx.x, gridDim.x, [&](int i) {
    if (i < n) tw[i] = v.X[cur][i];
    else if (i < n + mi) tw[i] = v.S[cur][i - n];
    else if (i < dw) tw[i] = v.R[cur][i - n - mi];
    else ty[i - dw] = v.Y[cur][i - dw];
  });
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    s_last = (atomicAdd(&c->ticket[TK_TRACE], 1u) == gridDim.x - 1u);
  }
  __syncthreads();
  if (s_last && threadIdx.x == 0) {
    c->trace_iters_n = k + 1;
    c->last_acc = 0;
    c->ticket[TK_TRACE] = 0;
  }
}

// ===========================================================================
// Periodic check (stopping test of (inner-residuals)/(inner-scales)/
// (inner-termination) on the current and the averaged candidate, then the
// restart rule and primal-weight update (primal-weight-update)).
// ===========================================================================

// Brings the averages up to date (the averaging of the last accept is
// otherwise folded into the next trial).
__global__ __launch_bounds__(kBlock) void k_flush(Ctrl *__restrict__ c, InnerParams p, Vecs v,
                                                  Part px, Part pr) {
  if (c->state != ST_CHECK_DUE || !c->pending) return;
  const int cur = c->cur;
  const double ap = c->alpha_pend;
  if ((int)blockIdx.x < px.blocks) {
    for_elems(p.n, blockIdx.x, px.blocks, [&](int i) {
      v.xbar[i] = (1.0 - ap) * v.xbar[i] + ap * v.X[cur][i];
      v.qxbar[i] = (1.0 - ap) * v.qxbar[i] + ap * v.QX[cur][i];
    });
  } else {
    const int b = blockIdx.x - px.blocks;
    for_elems(p.m, b, pr.blocks, [&](int j) {
      v.ybar[j] = (1.0 - ap) * v.ybar[j] + ap * v.Y[cur][j];
      v.rbar[j] = (1.0 - ap) * v.rbar[j] + ap * v.R[cur][j];
      if (j >= p.me) {
        const int k = j - p.me;
        v.sbar[k] = (1.0 - ap) * v.sbar[k] + ap * v.S[cur][k];
      }
    });
  }
}

// A xbar and A' ybar for the averaged candidate.
template <int GA, int GT>
__global__ __launch_bounds__(kBlock) void k_check_spmv(Ctrl *__restrict__ c, Vecs v, Csr A,
                                                       Csr AT, Part pa, Part pt) {
  if (c->state != ST_CHECK_DUE) return;
  if ((int)blockIdx.x < pa.blocks) {
    for_rows<GA>(A.rows, blockIdx.x, pa.blocks, [&](int j, int lane) {
      const double s = row_dot<GA>(A.p, A.i, A.v, v.xbar, j, lane);
      if (lane == 0) v.axbar[j] = s;
    });
  } else {
    for_rows<GT>(AT.rows, blockIdx.x - pa.blocks, pt.blocks, [&](int i, int lane) {
      const double s = row_dot<GT>(AT.p, AT.i, AT.v, v.ybar, i, lane);
      if (lane == 0) v.atybar[i] = s;
    });
  }
}

// Reduction slots of k_check (per candidate cd = 0 current, 1 average).
enum ChkSlot : int {
  CK_RP = 0,   // max |B w - h|                     (2 slots)
  CK_BW = 2,   // max |B w|
  CK_RD = 4,   // max |w - P(w - g)|
  CK_HW = 6,   // max |H w|
  CK_BTY = 8,  // max |B' y|
  CK_Q = 10,   // max |q|                            (1 slot)
  CK_P = 11,   // sum Ey^2 (h - B w)^2               (2 slots, sums from here on)
  CK_D = 13,   // sum (w - P(w - Sw^2 g))^2 / Sw^2
  CK_DW = 15,  // sum (w - w_anchor)^2 / Sw^2
  CK_DY = 17,  // sum (y - y_anchor)^2 / Ey^2
  CK_N = 19
};
constexpr uint32_t kChkMaxMask = (1u << CK_P) - 1u;

// Residual quantities of both candidates over the x, s and row blocks, then
// (last workgroup) the stopping test, candidate choice and restart rule.
// Gradient g = H w + q - B'y of (inner-qp):
//   x: Q x + x/gamma + (c - z/gamma) - A'y;  s: y_I;  r: sigma r + lambda + y.
__global__ __launch_bounds__(kBlock) void k_check(Ctrl *__restrict__ c, InnerParams p, Vecs v,
                                                  Part px, Part ps, Part pr) {
  if (c->state != ST_CHECK_DUE) return;
  const int cur = c->cur;
  const double gi = p.gamma_inv;
  double a[CK_N];
#pragma unroll
  for (int k = 0; k < CK_N; ++k) a[k] = 0.0;
  const int ncand = p.mode_init ? 1 : 2;
  if ((int)blockIdx.x < px.blocks) {
    for_elems(p.n, blockIdx.x, px.blocks, [&](int i) {
      const double q = v.qx[i];
      a[CK_Q] = fmax(a[CK_Q], fabs(q));
      const double s2 = v.S2x[i];
      const double lo = v.lo[i], hi = v.hi[i];
      for (int cd = 0; cd < ncand; ++cd) {
        const double xv = cd ? v.xbar[i] : v.X[cur][i];
        const double qxv = cd ? v.qxbar[i] : v.QX[cur][i];
        const double atyv = cd ? v.atybar[i] : v.ATY[cur][i];
        const double hx = qxv + gi * xv;
        const double g = hx + q - atyv;
        a[CK_RD + cd] = fmax(a[CK_RD + cd], fabs(xv - clampd(xv - g, lo, hi)));
        a[CK_HW + cd] = fmax(a[CK_HW + cd], fabs(hx));
        a[CK_BTY + cd] = fmax(a[CK_BTY + cd], fabs(atyv));
        const double dh = xv - clampd(xv - s2 * g, lo, hi);
        a[CK_D + cd] += dh * dh / s2;
        const double dwv = xv - v.xa[i];
        a[CK_DW + cd] += dwv * dwv / s2;
      }
    });
  } else if ((int)blockIdx.x < px.blocks + ps.blocks) {
    const int b = blockIdx.x - px.blocks;
    for_elems(p.mi, b, ps.blocks, [&](int k) {
      const int j = p.me + k;
      const double s2 = v.S2s[k];
      const double bj = v.b[j];
      for (int cd = 0; cd < ncand; ++cd) {
        const double sv = cd ? v.sbar[k] : v.S[cur][k];
        const double yv = cd ? v.ybar[j] : v.Y[cur][j];
        a[CK_RD + cd] = fmax(a[CK_RD + cd], fabs(sv - maxd(sv - yv, bj)));
        a[CK_BTY + cd] = fmax(a[CK_BTY + cd], fabs(yv));
        const double dh = sv - maxd(sv - s2 * yv, bj);
        a[CK_D + cd] += dh * dh / s2;
        const double dwv = sv - v.sa[k];
        a[CK_DW + cd] += dwv * dwv / s2;
      }
    });
  } else {
    const int b = blockIdx.x - px.blocks - ps.blocks;
    for_elems(p.m, b, pr.blocks, [&](int j) {
      const double sg = v.sigma[j];
      const double lm = v.lam[j];
      a[CK_Q] = fmax(a[CK_Q], fabs(lm));
      const double s2 = v.S2r[j];
      const double e2 = v.E2[j];
      const double hj = (j < p.me) ? v.b[j] : 0.0;
      for (int cd = 0; cd < ncand; ++cd) {
        const double rv = cd ? v.rbar[j] : v.R[cur][j];
        const double yv = cd ? v.ybar[j] : v.Y[cur][j];
        double bwv;
        if (cd) {
          bwv = v.axbar[j] - rv;
          if (j >= p.me) bwv = v.axbar[j] - v.sbar[j - p.me] - rv;
        } else {
          bwv = v.BW[cur][j];
        }
        const double hr = sg * rv;
        const double g = hr + lm + yv;
        a[CK_RD + cd] = fmax(a[CK_RD + cd], fabs(g));
        a[CK_HW + cd] = fmax(a[CK_HW + cd], fabs(hr));
        a[CK_BTY + cd] = fmax(a[CK_BTY + cd], fabs(yv));
        a[CK_D + cd] += s2 * g * g;
        const double dwv = rv - v.ra[j];
        a[CK_DW + cd] += dwv * dwv / s2;
        const double pres = hj - bwv;
        a[CK_RP + cd] = fmax(a[CK_RP + cd], fabs(pres));
        a[CK_BW + cd] = fmax(a[CK_BW + cd], fabs(bwv));
        a[CK_P + cd] += e2 * pres * pres;
        const double dyv = yv - v.ya[j];
        a[CK_DY + cd] += dyv * dyv / e2;
      }
    });
  }
  block_reduce<CK_N>(a, kChkMaxMask, v.partial, blockIdx.x);
}

// Decision of a check: one workgroup combines k_check's partials in a fixed
// order, then (thread 0) the stopping test, candidate choice, restart rule
// and primal-weight update.
__global__ __launch_bounds__(kDecideThreads) void k_check_decide(Ctrl *__restrict__ c,
                                                                 InnerParams p, Vecs v,
                                                                 int nparts) {
  if (c->state != ST_CHECK_DUE) return;
  double a[CK_N];
#pragma unroll
  for (int k = 0; k < CK_N; ++k) a[k] = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kDecideThreads) {
#pragma unroll
    for (int k = 0; k < CK_N; ++k) {
      const double x = v.partial[k * kMaxParts + i];
      a[k] = ((kChkMaxMask >> k) & 1u) ? fmax(a[k], x) : a[k] + x;
    }
  }
  __shared__ double sh[kDecideThreads / 64][CK_N];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < CK_N; ++k) {
    double x = a[k];
    const bool mx = (kChkMaxMask >> k) & 1u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_down(x, off, 64);
      x = mx ? fmax(x, o) : x + o;
    }
    if (lane == 0) sh[wid][k] = x;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double r[CK_N];
  for (int k = 0; k < CK_N; ++k) {
    const bool mx = (kChkMaxMask >> k) & 1u;
    double acc = sh[0][k];
    for (int w = 1; w < kDecideThreads / 64; ++w) acc = mx ? fmax(acc, sh[w][k]) : acc + sh[w][k];
    r[k] = acc;
  }
  c->pending = 0;  // the averages were brought up to date by k_flush
  for (int k = 0; k < CK_N; ++k) c->chk[k] = r[k];
  const double om = c->omega;
  const double k0 = sqrt(om * om * r[CK_P] + r[CK_D] / (om * om));
  if (p.mode_init) {
    c->kkt_anchor = k0;
    c->kkt_prev = INFINITY;
    c->state = ST_RUNNING;
    return;
  }
  c->checks += 1;
  const double da = p.delta_a, dr = p.delta_r;
  bool pass[2];
  for (int cd = 0; cd < 2; ++cd) {
    const double spv = fmax(1.0, fmax(r[CK_BW + cd], p.h_norm));
    const double sdv = fmax(fmax(1.0, r[CK_HW + cd]), fmax(r[CK_Q], r[CK_BTY + cd]));
    pass[cd] = (r[CK_RP + cd] <= da + dr * spv) && (r[CK_RD + cd] <= da + dr * sdv);
  }
  int kind, which = 0;
  c->restart_flag = 0;
  c->copy_avg = 0;
  if (pass[0] || pass[1]) {
    which = pass[0] ? 0 : 1;
    kind = 2;
    c->copy_avg = which;
    c->state = ST_CONVERGED;
  } else {
    const double k1 = sqrt(om * om * r[CK_P + 1] + r[CK_D + 1] / (om * om));
    const int use_avg = (k1 < k0) ? 1 : 0;
    const double kc = use_avg ? k1 : k0;
    const bool restart = (kc <= p.restart_suff * c->kkt_anchor) ||
                         (kc <= p.restart_nec * c->kkt_anchor && kc > c->kkt_prev) ||
                         ((double)c->N >= p.restart_art * (double)c->t);
    which = use_avg;
    if (restart) {
      kind = 1;
      const double dW = sqrt(r[CK_DW + use_avg]);
      const double dY = sqrt(r[CK_DY + use_avg]);
      double omn = om;
      if (dW > 0.0 && dY > 0.0) omn = exp(0.25 * log(dY / dW) + 0.75 * log(om));
      c->omega = omn;
      c->step_scale = 1.0;
      c->N = 0;
      c->kkt_anchor = sqrt(omn * omn * r[CK_P + use_avg] + r[CK_D + use_avg] / (omn * omn));
      c->kkt_prev = INFINITY;
      c->restarts += 1;
      c->restart_flag = 1;
      c->copy_avg = use_avg;
    } else {
      kind = 0;
      c->kkt_prev = kc;
    }
    c->state = (c->t_call >= p.max_inner) ? ST_ITER_LIMIT : ST_RUNNING;
  }
  c->check_kind = kind;
  c->check_which = which;
  if (c->trace_checks_n < p.trace_trials_cap) {
    const int k = c->trace_checks_n;
    v.trace_ck[4 * k + 0] = kind;
    v.trace_ck[4 * k + 1] = c->t;
    v.trace_ck[4 * k + 2] = which;
    v.trace_ck[4 * k + 3] = (int32_t)c->trials;
    c->trace_checks_n = k + 1;
  }
}

// Applies a check's outcome to the vectors: the average becomes the
// current iterate (with its products), and/or a restart resets the
// averages and anchors to the current iterate.
__global__ __launch_bounds__(kBlock) void k_apply(Ctrl *__restrict__ c, InnerParams p, Vecs v,
                                                  Part px, Part pr) {
  const int copy_avg = c->copy_avg;
  const int restart = c->restart_flag;
  if (!copy_avg && !restart) return;
  const int cur = c->cur;
  if ((int)blockIdx.x < px.blocks) {
    for_elems(p.n, blockIdx.x, px.blocks, [&](int i) {
      double xv = v.X[cur][i], qv = v.QX[cur][i];
      if (copy_avg) {
        xv = v.xbar[i];
        qv = v.qxbar[i];
        v.X[cur][i] = xv;
        v.QX[cur][i] = qv;
        v.ATY[cur][i] = v.atybar[i];
      }
      if (restart) {
        v.xbar[i] = xv;
        v.qxbar[i] = qv;
        v.xa[i] = xv;
      }
    });
  } else {
    const int b = blockIdx.x - px.blocks;
    for_elems(p.m, b, pr.blocks, [&](int j) {
      double rv = v.R[cur][j], yv = v.Y[cur][j];
      const bool ineq = j >= p.me;
      const int k = j - p.me;
      double sv = ineq ? v.S[cur][k] : 0.0;
      if (copy_avg) {
        rv = v.rbar[j];
        yv = v.ybar[j];
        v.R[cur][j] = rv;
        v.Y[cur][j] = yv;
        if (ineq) {
          sv = v.sbar[k];
          v.S[cur][k] = sv;
          v.BW[cur][j] = v.axbar[j] - sv - rv;
        } else {
          v.BW[cur][j] = v.axbar[j] - rv;
        }
      }
      if (restart) {
        v.rbar[j] = rv;
        v.ybar[j] = yv;
        v.ra[j] = rv;
        v.ya[j] = yv;
        if (ineq) {
          v.sbar[k] = sv;
          v.sa[k] = sv;
        }
      }
    });
  }
}

// Clears the flags k_apply acted on (one thread, after k_apply).
__global__ void k_apply_done(Ctrl *__restrict__ c) {
  c->copy_avg = 0;
  c->restart_flag = 0;
}

// ===========================================================================
// Inner QP formation.
// ===========================================================================

// Products of the starting point (Q x, A'y) and averages/anchors set to it;
// resets the epoch counters.  Row part: copies only.
template <int GQ, int GT>
__global__ __launch_bounds__(kBlock) void k_inner_init(Ctrl *__restrict__ c, InnerParams p,
                                                       Vecs v, Csr Q, Csr AT, Part pq, Part pr) {
  const int cur = c->cur;
  if ((int)blockIdx.x < pq.blocks) {
    for_rows<GQ>(Q.rows, blockIdx.x, pq.blocks, [&](int i, int lane) {
      const double qx = row_dot<GQ>(Q.p, Q.i, Q.v, v.X[cur], i, lane);
      const double aty = row_dot<GT>(AT.p, AT.i, AT.v, v.Y[cur], i, lane);
      if (lane == 0) {
        const double xv = v.X[cur][i];
        v.QX[cur][i] = qx;
        v.ATY[cur][i] = aty;
        v.xbar[i] = xv;
        v.qxbar[i] = qx;
        v.xa[i] = xv;
      }
    });
  } else {
    for_elems(p.m, blockIdx.x - pq.blocks, pr.blocks, [&](int j) {
      const double rv = v.R[cur][j], yv = v.Y[cur][j];
      v.rbar[j] = rv;
      v.ra[j] = rv;
      v.ybar[j] = yv;
      v.ya[j] = yv;
      if (j >= p.me) {
        const int k = j - p.me;
        const double sv = v.S[cur][k];
        v.sbar[k] = sv;
        v.sa[k] = sv;
      }
    });
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c->state = ST_CHECK_DUE;  // the init-mode check computes the anchor metric
    c->N = 0;
    c->t = 0;
    c->t_call = 0;
    c->rejects = 0;
    c->pending = 0;
    c->step_scale = 1.0;
    c->restart_flag = 0;
    c->copy_avg = 0;
    c->last_acc = 0;
  }
}

// One sweep of inner Ruiz on B diag(Pw), Pw = (1, 1, 1/sqrt(sigma)):
// rows j: E_j * max(max_k |A_jk| Fx_k, [I] Fs, Fr_j / sqrt(sigma_j));
// x columns via A' rows; s and r columns are row-local.
template <int GA, int GT>
__global__ __launch_bounds__(kBlock) void k_inner_ruiz(InnerParams p, Vecs v, Csr A, Csr AT,
                                                       Part pa, Part pt, double *Fx_new,
                                                       double *Fs_new, double *Fr_new,
                                                       double *E_new) {
  if ((int)blockIdx.x < pa.blocks) {
    for_rows<GA>(A.rows, blockIdx.x, pa.blocks, [&](int j, int lane) {
      const double e = v.tmp_m[j];  // current E
      double mx = 0.0;
      for (int k = A.p[j] + lane; k < A.p[j + 1]; k += GA)
        mx = fmax(mx, (e * fabs(A.v[k])) * v.Fx[A.i[k]]);
#pragma unroll
      for (int off = GA / 2; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, GA));
      if (lane == 0) {
        const double pr = 1.0 / sqrt(v.sigma[j]);
        const double er = (e * pr) * v.Fr[j];
        mx = fmax(mx, er);
        if (j >= p.me) {
          const int k = j - p.me;
          const double es = e * v.Fs[k];
          mx = fmax(mx, es);
          Fs_new[k] = v.Fs[k] / sqrt(es > 0.0 ? es : 1.0);
        }
        Fr_new[j] = v.Fr[j] / sqrt(er > 0.0 ? er : 1.0);
        E_new[j] = e / sqrt(mx > 0.0 ? mx : 1.0);
      }
    });
  } else {
    for_rows<GT>(AT.rows, blockIdx.x - pa.blocks, pt.blocks, [&](int i, int lane) {
      double mx = 0.0;
      const double f = v.Fx[i];
      for (int k = AT.p[i] + lane; k < AT.p[i + 1]; k += GT)
        mx = fmax(mx, (v.tmp_m[AT.i[k]] * fabs(AT.v[k])) * f);
#pragma unroll
      for (int off = GT / 2; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, GT));
      if (lane == 0) Fx_new[i] = f / sqrt(mx > 0.0 ? mx : 1.0);
    });
  }
}

// Diagonal scales and steps (eq. (diagonal-scales), (diagonal-steps)) of the
// scaled inner QP, expressed for the unscaled iteration:
//   taub = boost * 0.99 * Sw^2 / m_w,   etab = boost * 0.99 * Ey^2 / m_y
// (the primal weight and the rejection shrink factor are applied as scalars).
// Pass 1 (x columns, rows of Q and of A'): m_w,x and u = Sx^2 / m_w,x.
template <int G>
__global__ __launch_bounds__(kBlock) void k_steps_x(InnerParams p, Vecs v, Csr Q, Csr AT, Part pq,
                                                    double gamma_inv, double boost) {
  for_rows<G>(Q.rows, blockIdx.x, pq.blocks, [&](int i, int lane) {
    const double si = v.Fx[i];  // Sw on x = Fx
    double off = 0.0, dg = 0.0;
    for (int k = Q.p[i] + lane; k < Q.p[i + 1]; k += G) {
      const int col = Q.i[k];
      if (col == i) dg += Q.v[k];
      else off += fabs(Q.v[k]) * v.Fx[col];
    }
    double b1 = 0.0, b2 = 0.0;
    for (int k = AT.p[i] + lane; k < AT.p[i + 1]; k += G) {
      const int j = AT.i[k];
      const double eb = v.tmp_m[j] * fabs(AT.v[k]);  // Ey_j |A_ji|
      b1 += eb;
      b2 += v.sigma[j] * (eb * eb);
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
      off += __shfl_xor(off, o, G);
      dg += __shfl_xor(dg, o, G);
      b1 += __shfl_xor(b1, o, G);
      b2 += __shfl_xor(b2, o, G);
    }
    if (lane == 0) {
      const double h1 = (off + fabs(dg + gamma_inv) * si) * si;
      const double bn1 = b1 * si;
      const double bn2 = sqrt(b2) * si;
      const double mw = h1 + (bn1 > bn2 ? bn1 : bn2);
      const double s2 = si * si;
      v.S2x[i] = s2;
      v.taub_x[i] = boost * 0.99 * s2 / mw;
      v.tmp_n[i] = s2 / mw;
    }
  });
}

// Pass 2 (rows of A): s and r columns (row-local), m_y and the dual steps.
template <int GA>
__global__ __launch_bounds__(kBlock) void k_steps_rows(InnerParams p, Vecs v, Csr A, Part pa,
                                                       double boost) {
  for_rows<GA>(A.rows, blockIdx.x, pa.blocks, [&](int j, int lane) {
    double acc = 0.0;
    for (int k = A.p[j] + lane; k < A.p[j + 1]; k += GA) {
      const double a = A.v[k];
      acc += (a * a) * v.tmp_n[A.i[k]];
    }
#pragma unroll
    for (int off = GA / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, GA);
    if (lane == 0) {
      const double e = v.tmp_m[j];
      const double sg = v.sigma[j];
      const double e2 = e * e;
      // r column: H_hat = Sr^2 sigma, B_hat = -e * Sr
      const double sr = (1.0 / sqrt(sg)) * v.Fr[j];
      const double mwr = (sr * sg) * sr + e * sr;
      double my = e2 * acc + (e * sr) * (e * sr) / mwr;
      v.S2r[j] = sr * sr;
      v.taub_r[j] = boost * 0.99 * (sr * sr) / mwr;
      if (j >= p.me) {
        const int k = j - p.me;
        const double ss = v.Fs[k];
        const double b1 = e * ss;
        const double b2 = sqrt(sg * (b1 * b1));
        const double mws = b1 > b2 ? b1 : b2;
        my += b1 * b1 / mws;
        v.S2s[k] = ss * ss;
        v.taub_s[k] = boost * 0.99 * (ss * ss) / mws;
      }
      v.E2[j] = e2;
      v.etab[j] = boost * 0.99 * e2 / my;
    }
  });
}

// Warm start of the inner variables (eq. (inner-warm-start)) from A x:
// s = max(b_I, A_I x + lambda_I / sigma_I), r_E = A_E x - b_E, r_I = A_I x - s,
// and B w = A x - [s] - r; also q_x = c - z / gamma.
__global__ __launch_bounds__(kBlock) void k_warm(InnerParams p, Vecs v, int cur, double gamma) {
  const int m = p.m, n = p.n;
  for_elems(m + n, blockIdx.x, gridDim.x, [&](int idx) {
    if (idx < m) {
      const int j = idx;
      const double ax = v.ax[j];
      if (j < p.me) {
        const double r = ax - v.b[j];
        v.R[cur][j] = r;
        v.BW[cur][j] = ax - r;
      } else {
        const int k = j - p.me;
        const double s = maxd(ax + v.lam[j] / v.sigma[j], v.b[j]);
        const double r = ax - s;
        v.S[cur][k] = s;
        v.R[cur][j] = r;
        v.BW[cur][j] = ax - s - r;
      }
    } else {
      const int i = idx - m;
      v.qx[i] = v.c[i] - v.z[i] / gamma;
    }
  });
}

// ===========================================================================
// Outer step (eq. (practical-multiplier-update), (outer-residuals),
// (outer-scales)).
// ===========================================================================
template <int GA>
__global__ __launch_bounds__(kBlock) void k_outer_rows(Ctrl *__restrict__ c, InnerParams p,
                                                       Vecs v, Csr A, Part pa) {
  const int cur = c->cur;
  double a[4] = {0.0, 0.0, 0.0, 0.0};  // r_p part, |A_E x|, |A_I x|, |r_row|
  for_rows<GA>(A.rows, blockIdx.x, gridDim.x, [&](int j, int lane) {
    const double ax = row_dot<GA>(A.p, A.i, A.v, v.X[cur], j, lane);
    if (lane == 0) {
      v.ax[j] = ax;
      const double bj = v.b[j];
      const double sg = v.sigma[j];
      const double lm = v.lam[j];
      double rr;
      if (j < p.me) {
        const double res = ax - bj;
        v.lam[j] = lm + sg * res;
        rr = res;
        a[0] = fmax(a[0], fabs(res));
        a[1] = fmax(a[1], fabs(ax));
      } else {
        const double s = maxd(ax + lm / sg, bj);
        const double ln = lm + sg * (ax - bj);
        v.lam[j] = ln < 0.0 ? ln : 0.0;
        rr = ax - s;
        a[0] = fmax(a[0], maxd(bj - ax, 0.0));
        a[2] = fmax(a[2], fabs(ax));
      }
      v.rrow[j] = rr;
      a[3] = fmax(a[3], fabs(rr));
    }
  });
  block_reduce<4>(a, 0xFu, v.partial, blockIdx.x);
  if (last_block(&c->ticket[TK_OUTER_ROWS], gridDim.x)) {
    double r[4];
    final_reduce<4>(v.partial, gridDim.x, 0xFu, r);
    if (threadIdx.x == 0) {
      for (int k = 0; k < 4; ++k) c->outv[k] = r[k];
      c->ticket[TK_OUTER_ROWS] = 0;
    }
  }
}

template <int GQ, int GT>
__global__ __launch_bounds__(kBlock) void k_outer_cols(Ctrl *__restrict__ c, InnerParams p,
                                                       Vecs v, Csr Q, Csr AT, Part pq) {
  const int cur = c->cur;
  double a[4] = {0.0, 0.0, 0.0, 0.0};  // r_d, |Q x|, |A' lambda|, |x - z|
  for_rows<GQ>(Q.rows, blockIdx.x, gridDim.x, [&](int i, int lane) {
    const double qx = row_dot<GQ>(Q.p, Q.i, Q.v, v.X[cur], i, lane);
    const double atl = row_dot<GT>(AT.p, AT.i, AT.v, v.lam, i, lane);
    if (lane == 0) {
      const double x = v.X[cur][i];
      const double pr = clampd(x - qx - v.c[i] - atl, v.lo[i], v.hi[i]);
      a[0] = fmax(a[0], fabs(x - pr));
      a[1] = fmax(a[1], fabs(qx));
      a[2] = fmax(a[2], fabs(atl));
      a[3] = fmax(a[3], fabs(x - v.z[i]));
      v.qxo[i] = qx;
      v.atl[i] = atl;
    }
  });
  block_reduce<4>(a, 0xFu, v.partial, blockIdx.x);
  if (last_block(&c->ticket[TK_OUTER_COLS], gridDim.x)) {
    double r[4];
    final_reduce<4>(v.partial, gridDim.x, 0xFu, r);
    if (threadIdx.x == 0) {
      for (int k = 0; k < 4; ++k) c->outv[4 + k] = r[k];
      c->ticket[TK_OUTER_COLS] = 0;
    }
  }
}

// Row-wise penalty update (eq. (penalty-trigger-eq)): a row is raised when
// its residual did not fall below theta times the previous one (equality
// rows, and inequality rows with lambda < 0), by the factor
// max(1, growth |r_i| / ||r||_inf), capped.
__global__ __launch_bounds__(kBlock) void k_penalty(InnerParams p, Vecs v, int have_prev,
                                                    double rnorm, double theta, double growth,
                                                    double sig_max, int gate, double gate_tol) {
  for_elems(p.m, blockIdx.x, gridDim.x, [&](int j) {
    const double r = v.rrow[j];
    if (have_prev && rnorm > 0.0) {
      const bool active = (j < p.me) || (v.lam[j] < 0.0);
      bool trig = fabs(r) > theta * fabs(v.rprev[j]) && active;
      if (gate) trig = trig && (fabs(r) > gate_tol);
      if (trig) {
        const double fac = fmax(1.0, growth * fabs(r) / rnorm);
        const double sn = v.sigma[j] * fac;
        v.sigma[j] = sn < sig_max ? sn : sig_max;
      }
    }
    v.rprev[j] = r;
  });
}

__global__ __launch_bounds__(kBlock) void k_copy(double *dst, const double *src, int32_t n) {
  for_elems(n, blockIdx.x, gridDim.x, [&](int i) { dst[i] = src[i]; });
}

__global__ __launch_bounds__(kBlock) void k_fill(double *dst, double val, int32_t n) {
  for_elems(n, blockIdx.x, gridDim.x, [&](int i) { dst[i] = val; });
}

// ===========================================================================
// Set-up helpers.
// ===========================================================================
template <int G>
__global__ __launch_bounds__(kBlock) void k_row_absmax(Csr M, const double *wrow,
                                                       const double *wcol, double *out) {
  for_rows<G>(M.rows, blockIdx.x, gridDim.x, [&](int r, int lane) {
    const double wr = wrow[r];
    double mx = 0.0;
    for (int k = M.p[r] + lane; k < M.p[r + 1]; k += G)
      mx = fmax(mx, (wr * fabs(M.v[k])) * wcol[M.i[k]]);
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, G));
    if (lane == 0) out[r] = mx;
  });
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_spmv(Csr M, const double *x, double *y, double alpha) {
  for_rows<G>(M.rows, blockIdx.x, gridDim.x, [&](int r, int lane) {
    const double s = row_dot<G>(M.p, M.i, M.v, x, r, lane);
    if (lane == 0) y[r] = alpha * s;
  });
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_scale_csr(const int32_t *rp, const int32_t *ci,
                                                      double *val, int32_t rows,
                                                      const double *wrow, const double *wcol,
                                                      double s) {
  for_rows<G>(rows, blockIdx.x, gridDim.x, [&](int r, int lane) {
    const double wr = wrow[r];
    for (int k = rp[r] + lane; k < rp[r + 1]; k += G) val[k] = s * ((wr * val[k]) * wcol[ci[k]]);
  });
}

__global__ __launch_bounds__(kBlock) void k_dot(Ctrl *c, const double *a, const double *b,
                                                int32_t n, int slot, double *partial) {
  double acc = 0.0;
  for_elems(n, blockIdx.x, gridDim.x, [&](int i) { acc += a[i] * b[i]; });
  double vals[1] = {acc};
  block_reduce<1>(vals, 0u, partial, blockIdx.x);
  if (last_block(&c->ticket[TK_GEN], gridDim.x)) {
    double r[1];
    final_reduce<1>(partial, gridDim.x, 0u, r);
    if (threadIdx.x == 0) {
      c->gen[slot] = r[0];
      c->ticket[TK_GEN] = 0;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_absmax(Ctrl *c, const double *a, int32_t n, int slot,
                                                   double *partial) {
  double acc = 0.0;
  for_elems(n, blockIdx.x, gridDim.x, [&](int i) { acc = fmax(acc, fabs(a[i])); });
  double vals[1] = {acc};
  block_reduce<1>(vals, 1u, partial, blockIdx.x);
  if (last_block(&c->ticket[TK_GEN], gridDim.x)) {
    double r[1];
    final_reduce<1>(partial, gridDim.x, 1u, r);
    if (threadIdx.x == 0) {
      c->gen[slot] = r[0];
      c->ticket[TK_GEN] = 0;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_lanczos_update(Ctrl *c, double *w, const double *v,
                                                           const double *vprev, double beta_prev,
                                                           int32_t n, double *partial) {
  const double alpha = c->gen[0];
  double acc = 0.0;
  for_elems(n, blockIdx.x, gridDim.x, [&](int i) {
    const double wn = (w[i] - alpha * v[i]) - beta_prev * vprev[i];
    w[i] = wn;
    acc += wn * wn;
  });
  double vals[1] = {acc};
  block_reduce<1>(vals, 0u, partial, blockIdx.x);
  if (last_block(&c->ticket[TK_GEN], gridDim.x)) {
    double r[1];
    final_reduce<1>(partial, gridDim.x, 0u, r);
    if (threadIdx.x == 0) {
      c->gen[1] = r[0];
      c->ticket[TK_GEN] = 0;
    }
  }
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_row_abssum(Csr M, double *out) {
  for_rows<G>(M.rows, blockIdx.x, gridDim.x, [&](int r, int lane) {
    double acc = 0.0;
    for (int k = M.p[r] + lane; k < M.p[r + 1]; k += G) acc += fabs(M.v[k]);
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
    if (lane == 0) out[r] = acc;
  });
}

// Ruiz update: D /= sqrt(norm) (norm 0 keeps the scale); cnq optional.
__global__ __launch_bounds__(kBlock) void k_ruiz_update(double *Dc, const double *rn, int32_t m,
                                                        double *Dx, const double *cn,
                                                        const double *cnq, int32_t n) {
  for_elems(m + n, blockIdx.x, gridDim.x, [&](int idx) {
    if (idx < m) {
      const double r = rn[idx];
      Dc[idx] = Dc[idx] / sqrt(r > 0.0 ? r : 1.0);
    } else {
      const int i = idx - m;
      double cv = cn[i];
      if (cnq) cv = fmax(cv, cnq[i]);
      Dx[i] = Dx[i] / sqrt(cv > 0.0 ? cv : 1.0);
    }
  });
}

__global__ __launch_bounds__(kBlock) void k_gather(double *dst, const double *src,
                                                   const int32_t *perm, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    dst[i] = src[perm[i]];
}

// Small elementwise operations of the set-up (ElemOp).

__global__ __launch_bounds__(kBlock) void k_elem(int op, double *a, const double *b,
                                                 const double *c, double s, int32_t n) {
  for_elems(n, blockIdx.x, gridDim.x, [&](int i) {
    switch (op) {
      case EL_GRAD: a[i] = b[i] * (a[i] + c[i]); break;
      case EL_MULS: a[i] = (s * b[i]) * c[i]; break;
      case EL_DIV: a[i] = b[i] / c[i]; break;
      case EL_MUL: a[i] = b[i] * c[i]; break;
      case EL_SCALE_DIV: a[i] = s * b[i] / c[i]; break;
      case EL_NEG: a[i] = -b[i]; break;
      case EL_AXPBY: a[i] = b[i] / s; break;
      case EL_DIAG: a[i] = s * ((b[i] * c[i]) * b[i]); break;
      default: a[i] = a[i] / b[i]; break;
    }
  });
}

// Violation of A x0 against its projection onto the feasible row values:
// equality rows A x - b, inequality rows A x - max(b, A x).
__global__ __launch_bounds__(kBlock) void k_viol(InnerParams p, Vecs v, double *out) {
  for_elems(p.m, blockIdx.x, gridDim.x, [&](int j) {
    const double ax = v.ax[j];
    out[j] = (j < p.me) ? ax - v.b[j] : ax - maxd(ax, v.b[j]);
  });
}


}  // namespace

// ===========================================================================
// Launch wrappers.
// ===========================================================================
Part make_part(int32_t rows, int32_t G, int32_t max_blocks) {
  Part pt;
  pt.rows = rows;
  pt.G = G;
  const int64_t rpb = kBlock / G;
  int64_t nb = (rows + rpb - 1) / rpb;
  if (nb > max_blocks) nb = max_blocks;
  pt.blocks = (int32_t)nb;
  return pt;
}

static inline int nz(int b) { return b > 0 ? b : 1; }

static inline int xtrial_blocks(int n) {
  return nz((int)std::min<int64_t>(((int64_t)n + 4 * kBlock - 1) / (4 * kBlock), kMaxParts));
}

void launch_xtrial(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v, const Part &px) {
  hipLaunchKernelGGL(k_xtrial, dim3(xtrial_blocks(p.n)), dim3(kBlock), 0, st, c, p, v, px);
}

void stream_row_blocks(const int32_t *rp, int32_t rows, int32_t max_rows, int32_t *out_nrb,
                       int32_t *rb) {
  int32_t nb = 0;
  rb[0] = 0;
  int32_t r = 0;
  while (r < rows) {
    const int32_t start = r;
    const int32_t base = rp[r];
    ++r;
    while (r < rows && rp[r + 1] - base <= kTile && r - start < max_rows) ++r;
    rb[++nb] = r;
  }
  *out_nrb = nb;
}

void launch_qa(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v, const Csr &Q,
               const Csr &A, const Part &pq, const Part &pa) {
  (void)pq;
  (void)pa;
  const int gq = std::min(Q.nrb, kMaxParts);
  const int ga = std::min(A.nrb, kMaxParts);
  hipLaunchKernelGGL(k_qa_stream, dim3(nz(gq + ga)), dim3(kBlock), 0, st, c, p, v, Q, A, gq, ga);
}

void launch_at(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v, const Csr &AT,
               const Part &pt) {
  (void)pt;
  const int g = std::min(AT.nrb, kMaxParts);
  hipLaunchKernelGGL(k_at_stream, dim3(nz(g)), dim3(kBlock), 0, st, c, p, v, AT);
}

void launch_decide(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v, const Csr &A,
                   const Csr &AT) {
  const int gx = xtrial_blocks(p.n);
  const int ga = std::min(A.nrb, kMaxParts);
  const int gt = nz(std::min(AT.nrb, kMaxParts));
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(kDecideThreads), 0, st, c, p, v, gx, ga, gt);
}

void launch_trace(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v, const Part &px,
                  const Part &pr) {
  (void)pr;
  const int blocks = (int)std::min<int64_t>(((int64_t)p.dw + p.m + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_trace, dim3(nz(blocks)), dim3(kBlock), 0, st, c, p, v);
  (void)px;
}

void launch_flush(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v, const Part &px,
                  const Part &pr) {
  hipLaunchKernelGGL(k_flush, dim3(nz(px.blocks + pr.blocks)), dim3(kBlock), 0, st, c, p, v, px,
                     pr);
}

void launch_check_spmv(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v,
                       const Csr &A, const Csr &AT, const Part &pa, const Part &pt) {
  (void)p;
  PDNQP_DISPATCH_G(A.G, {
    constexpr int GA_ = GV;
    PDNQP_DISPATCH_G(AT.G, {
      hipLaunchKernelGGL((k_check_spmv<GA_, GV>), dim3(nz(pa.blocks + pt.blocks)), dim3(kBlock),
                         0, st, c, v, A, AT, pa, pt);
    });
  });
}

void launch_check(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v, const Part &px,
                  const Part &ps, const Part &pr) {
  const int g = nz(px.blocks + ps.blocks + pr.blocks);
  hipLaunchKernelGGL(k_check, dim3(g), dim3(kBlock), 0, st, c, p, v, px, ps, pr);
  hipLaunchKernelGGL(k_check_decide, dim3(1), dim3(kDecideThreads), 0, st, c, p, v, g);
}

void launch_apply(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v, const Part &px,
                  const Part &pr) {
  hipLaunchKernelGGL(k_apply, dim3(nz(px.blocks + pr.blocks)), dim3(kBlock), 0, st, c, p, v, px,
                     pr);
  hipLaunchKernelGGL(k_apply_done, dim3(1), dim3(1), 0, st, c);
}

void launch_inner_init(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v,
                       const Csr &Q, const Csr &AT, const Part &pq, const Part &pr,
                       double gamma) {
  (void)gamma;
  // one G for both matrices in this (cold) kernel: the larger of the two
  const int G = Q.G > AT.G ? Q.G : AT.G;
  Part pqq = make_part(Q.rows, G, pq.blocks > 0 ? 1024 : 1);
  PDNQP_DISPATCH_G(G, {
    hipLaunchKernelGGL((k_inner_init<GV, GV>), dim3(pqq.blocks + pr.blocks), dim3(kBlock), 0, st,
                       c, p, v, Q, AT, pqq, pr);
  });
}

void launch_inner_ruiz_sweep(hipStream_t st, const InnerParams &p, const Vecs &v, const Csr &A,
                             const Csr &AT, const Part &pa, const Part &pt, double *Fx_new,
                             double *Fs_new, double *Fr_new, double *E_new) {
  PDNQP_DISPATCH_G(A.G, {
    constexpr int GA_ = GV;
    PDNQP_DISPATCH_G(AT.G, {
      hipLaunchKernelGGL((k_inner_ruiz<GA_, GV>), dim3(nz(pa.blocks + pt.blocks)), dim3(kBlock), 0,
                         st, p, v, A, AT, pa, pt, Fx_new, Fs_new, Fr_new, E_new);
    });
  });
}

void launch_steps(hipStream_t st, const InnerParams &p, const Vecs &v, const Csr &Q,
                  const Csr &A, const Csr &AT, double gamma_inv, double boost) {
  const int G = Q.G > AT.G ? Q.G : AT.G;
  Part pq = make_part(Q.rows, G, 1024);
  PDNQP_DISPATCH_G(G, {
    hipLaunchKernelGGL((k_steps_x<GV>), dim3(nz(pq.blocks)), dim3(kBlock), 0, st, p, v, Q, AT, pq,
                       gamma_inv, boost);
  });
  if (A.rows == 0) return;
  Part pa = make_part(A.rows, A.G, 1024);
  PDNQP_DISPATCH_G(A.G, {
    hipLaunchKernelGGL((k_steps_rows<GV>), dim3(nz(pa.blocks)), dim3(kBlock), 0, st, p, v, A, pa,
                       boost);
  });
}

void launch_warm(hipStream_t st, const InnerParams &p, const Vecs &v, int cur, double gamma) {
  const int blocks = (int)std::min<int64_t>(((int64_t)p.m + p.n + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_warm, dim3(nz(blocks)), dim3(kBlock), 0, st, p, v, cur, gamma);
}

void launch_row_abssum(hipStream_t st, const Csr &M, double *out, const Part &pm) {
  if (M.rows == 0) return;
  PDNQP_DISPATCH_G(M.G, {
    hipLaunchKernelGGL((k_row_abssum<GV>), dim3(nz(pm.blocks)), dim3(kBlock), 0, st, M, out);
  });
}

void launch_ruiz_update(hipStream_t st, double *Dc, const double *rn, int32_t m, double *Dx,
                        const double *cn, const double *cnq, int32_t n) {
  const int blocks = (int)std::min<int64_t>(((int64_t)m + n + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_ruiz_update, dim3(nz(blocks)), dim3(kBlock), 0, st, Dc, rn, m, Dx, cn, cnq,
                     n);
}

void launch_elem(hipStream_t st, int op, double *a, const double *b, const double *c, double s,
                 int32_t n) {
  if (n <= 0) return;
  const int blocks = (int)std::min<int64_t>(((int64_t)n + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_elem, dim3(blocks), dim3(kBlock), 0, st, op, a, b, c, s, n);
}

void launch_gather(hipStream_t st, double *dst, const double *src, const int32_t *perm,
                   int64_t n) {
  if (n <= 0) return;
  const int blocks = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 2048);
  hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(kBlock), 0, st, dst, src, perm, n);
}

void launch_viol(hipStream_t st, const InnerParams &p, const Vecs &v, double *out) {
  if (p.m == 0) return;
  const int blocks = (int)std::min<int64_t>(((int64_t)p.m + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_viol, dim3(blocks), dim3(kBlock), 0, st, p, v, out);
}

void launch_outer_rows(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v,
                       const Csr &A, const Part &pa) {
  PDNQP_DISPATCH_G(A.G, {
    hipLaunchKernelGGL((k_outer_rows<GV>), dim3(nz(pa.blocks)), dim3(kBlock), 0, st, c, p, v, A,
                       pa);
  });
}

void launch_outer_cols(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v,
                       const Csr &Q, const Csr &AT, const Part &pq) {
  const int G = Q.G > AT.G ? Q.G : AT.G;
  Part pqq = make_part(Q.rows, G, 1024);
  PDNQP_DISPATCH_G(G, {
    hipLaunchKernelGGL((k_outer_cols<GV, GV>), dim3(nz(pqq.blocks)), dim3(kBlock), 0, st, c, p, v,
                       Q, AT, pqq);
  });
  (void)pq;
}

void launch_penalty(hipStream_t st, const InnerParams &p, const Vecs &v, const Part &pr,
                    int have_prev, double rnorm, double theta, double growth, double sig_max,
                    int gate, double gate_tol) {
  if (p.m == 0) return;
  hipLaunchKernelGGL(k_penalty, dim3(nz(pr.blocks)), dim3(kBlock), 0, st, p, v, have_prev, rnorm,
                     theta, growth, sig_max, gate, gate_tol);
}

void launch_copy(hipStream_t st, double *dst, const double *src, int32_t n) {
  if (n <= 0) return;
  const int blocks = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(kBlock), 0, st, dst, src, n);
}

void launch_fill(hipStream_t st, double *dst, double val, int32_t n) {
  if (n <= 0) return;
  const int blocks = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(kBlock), 0, st, dst, val, n);
}

void launch_row_absmax(hipStream_t st, const Csr &M, const double *wrow, const double *wcol,
                       double *out, const Part &pm) {
  if (M.rows == 0) return;
  PDNQP_DISPATCH_G(M.G, {
    hipLaunchKernelGGL((k_row_absmax<GV>), dim3(nz(pm.blocks)), dim3(kBlock), 0, st, M, wrow, wcol,
                       out);
  });
}

void launch_spmv(hipStream_t st, const Csr &M, const double *x, double *y, double alpha,
                 const Part &pm) {
  if (M.rows == 0) return;
  PDNQP_DISPATCH_G(M.G, {
    hipLaunchKernelGGL((k_spmv<GV>), dim3(nz(pm.blocks)), dim3(kBlock), 0, st, M, x, y, alpha);
  });
}

void launch_scale_csr(hipStream_t st, const int32_t *p, const int32_t *i, double *v, int32_t rows,
                      const double *wrow, const double *wcol, double s, const Part &pm) {
  if (rows == 0) return;
  PDNQP_DISPATCH_G(pm.G, {
    hipLaunchKernelGGL((k_scale_csr<GV>), dim3(nz(pm.blocks)), dim3(kBlock), 0, st, p, i, v, rows,
                       wrow, wcol, s);
  });
}

void launch_dot(hipStream_t st, Ctrl *c, const double *a, const double *b, int32_t n, int slot,
                double *partial) {
  const int blocks = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_dot, dim3(nz(blocks)), dim3(kBlock), 0, st, c, a, b, n, slot, partial);
}

void launch_absmax(hipStream_t st, Ctrl *c, const double *a, int32_t n, int slot,
                   double *partial) {
  const int blocks = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_absmax, dim3(nz(blocks)), dim3(kBlock), 0, st, c, a, n, slot, partial);
}

void launch_lanczos_update(hipStream_t st, Ctrl *c, double *w, const double *v,
                           const double *vprev, double beta_prev, int32_t n, double *partial) {
  const int blocks = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_lanczos_update, dim3(nz(blocks)), dim3(kBlock), 0, st, c, w, v, vprev,
                     beta_prev, n, partial);
}

}  // namespace pdnqp
