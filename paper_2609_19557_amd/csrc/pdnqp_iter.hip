// gfx950 kernels of the inner PDHG iteration (Algorithm "practical diagonal
// PDHG"), templated on the storage/arithmetic type T of the bulk work:
// double for the FP64 path, float for the FP32-bulk path.  Every reduction
// (acceptance sums, KKT and restart norms) accumulates in FP64 whatever T is.
//
// Per trial: k_xtrial -> k_qa_stream (or, with two column panels,
// k_qa_panels -> k_qa_rows) -> k_at_stream -> k_decide.  Per check:
// k_flush -> k_check_spmv -> k_check -> k_check_decide -> k_apply ->
// k_apply_done.  Every kernel reads the device control block and does
// nothing when its phase is not due, so the host can enqueue fixed chunks.
#include "pdnqp_device.hpp"

#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>

namespace pdnqp {

using namespace dev;

namespace {

// ===========================================================================
// Trial step, x block (eq. (pdqp-trial), primal line, x components):
//   x_tr = clip(x - tau (q_x + (1-a) H xbar + a H x - A'y), xl, xu),
// H x = Q x + x / gamma.  Also applies the previous accept's averaging
// (xbar <- (1-a') xbar + a' x, Q xbar likewise) and accumulates
// sum dx^2 / taub_x for the acceptance test.  Four elements per thread are
// loaded before any is used.
// ===========================================================================
template <typename T>
__global__ __launch_bounds__(kBlock) void k_xtrial(Ctrl *__restrict__ c, InnerParams p,
                                                   IterVecs<T> v) {
  if (c->state != ST_RUNNING) return;
  const int cur = c->cur;
  const int pend = c->pending;
  const T ap = (T)c->alpha_pend;
  const double Nd = (double)c->N;
  const T alpha = (T)(2.0 / (Nd + 2.0));
  const T sct = (T)(c->step_scale / c->omega);
  const T gi = (T)p.gamma_inv;
  const T *__restrict__ x = v.X[cur];
  const T *__restrict__ qx = v.QX[cur];
  const T *__restrict__ aty = v.ATY[cur];
  const T *__restrict__ ql = v.qx;
  const T *__restrict__ tbx = v.taub_x;
  const T *__restrict__ lo = v.lo;
  const T *__restrict__ hi = v.hi;
  T *__restrict__ xt = v.X[cur ^ 1];
  T *__restrict__ xbar = v.xbar;
  T *__restrict__ qxbar = v.qxbar;
  constexpr int U = 4;
  const int stride = gridDim.x * kBlock;
  double acc = 0.0;
  for (int i0 = blockIdx.x * kBlock + threadIdx.x; i0 < p.n; i0 += U * stride) {
    T xi[U], qxi[U], xb[U], qb[U], ay[U], qv[U], tb[U], l[U], h[U];
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
        T xbu = xb[u], qbu = qb[u];
        if (pend) {
          xbu = (T(1) - ap) * xbu + ap * xi[u];
          qbu = (T(1) - ap) * qbu + ap * qxi[u];
          xbar[i] = xbu;
          qxbar[i] = qbu;
        }
        const T hx = qxi[u] + gi * xi[u];
        const T hb = qbu + gi * xbu;
        const T g = qv[u] + (T(1) - alpha) * hb + alpha * hx - ay[u];
        const T xn = clampv<T>(xi[u] - (sct * tb[u]) * g, l[u], h[u]);
        xt[i] = xn;
        const double d = (double)xn - (double)xi[u];
        acc += d * d / (double)tb[u];
      }
    }
  }
  double vals[1] = {acc};
  block_reduce<1>(vals, 0u, v.partial + PS_X * kMaxParts, blockIdx.x);
}

// ===========================================================================
// Trial step, sparse part 1, CSR-stream form (one launch, two partitions):
//  * row blocks of Q without its diagonal: Q x_tr = Q_off x_tr + diag(Q) x_tr
//  * row blocks of A: A x_tr, then row-locally (eq. (pdqp-trial)):
//      s_tr = max(b_I, s - tau_s y_I)                  (s block: gradient y_I)
//      r_tr = r - tau_r ((1-a) sigma rbar + a sigma r + lambda + y)
//      (B w_tr)_j = (A x_tr)_j - [s_tr] - r_tr
//      y_tr = y + eta (h - B w_tr - beta (B w_tr - B w))
//    plus the previous accept's averaging of ybar, rbar, sbar and the
//    row-block parts of the acceptance sums (FP64).
// ===========================================================================
// Row-local part of the trial for constraint row j, given (A x_tr)_j: the
// s and r trials, (B w_tr)_j, the dual extrapolation, the previous accept's
// averaging of ybar, rbar, sbar, and the row parts of the acceptance sums.
template <typename T>
struct RowTrial {
  int cur, nxt, pend, me;
  T ap, alpha, beta, sct, scy;
  double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;

  __device__ __forceinline__ RowTrial(const Ctrl *__restrict__ c, const InnerParams &p) {
    cur = c->cur;
    nxt = cur ^ 1;
    pend = c->pending;
    me = p.me;
    ap = (T)c->alpha_pend;
    const double Nd = (double)c->N;
    alpha = (T)(2.0 / (Nd + 2.0));
    beta = (T)(Nd / (Nd + 1.0));
    sct = (T)(c->step_scale / c->omega);
    scy = (T)(c->step_scale * c->omega);
  }

  __device__ __forceinline__ void operator()(const IterVecs<T> &v, int j, T ax) {
    const T y = v.Y[cur][j];
    const T bw = v.BW[cur][j];
    const T r = v.R[cur][j];
    const T sg = v.sigma[j];
    const T lm = v.lam[j];
    const T bj = v.b[j];
    T rb_ = v.rbar[j];
    if (pend) {
      v.ybar[j] = (T(1) - ap) * v.ybar[j] + ap * y;
      rb_ = (T(1) - ap) * rb_ + ap * r;
      v.rbar[j] = rb_;
    }
    const T gr = (T(1) - alpha) * (sg * rb_) + alpha * (sg * r) + lm + y;
    const T tbr = v.taub_r[j];
    const T rt = r - (sct * tbr) * gr;
    T bwt, hj;
    double ds = 0.0, ds2t = 0.0;
    if (j < me) {
      bwt = ax - rt;
      hj = bj;
    } else {
      const int k = j - me;
      const T sv = v.S[cur][k];
      if (pend) v.sbar[k] = (T(1) - ap) * v.sbar[k] + ap * sv;
      const T tbs = v.taub_s[k];
      const T st = maxv<T>(sv - (sct * tbs) * y, bj);
      v.S[nxt][k] = st;
      bwt = ax - st - rt;
      hj = T(0);
      ds = (double)st - (double)sv;
      ds2t = ds * ds / (double)tbs;
    }
    const T eb = v.etab[j];
    const T yt = y + (scy * eb) * (hj - bwt - beta * (bwt - bw));
    v.R[nxt][j] = rt;
    v.BW[nxt][j] = bwt;
    v.Y[nxt][j] = yt;
    const double dr = (double)rt - (double)r;
    const double dy = (double)yt - (double)y;
    s1 += dr * dr / (double)tbr + ds2t;
    s2 += dy * dy / (double)eb;
    s3 += fabs(dr * ((double)sg * dr));
    s4 += fabs(dr * dy) + fabs(ds * dy);
  }

  __device__ __forceinline__ void reduce(const IterVecs<T> &v, int slot) {
    double vals[4] = {s1, s2, s3, s4};
    block_reduce<4>(vals, 0u, v.partial + PS_ROW * kMaxParts, slot);
  }
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_qa_stream(Ctrl *__restrict__ c, InnerParams p,
                                                      IterVecs<T> v, CsrT<T> Q, CsrT<T> A, int gq,
                                                      int ga) {
  if (c->state != ST_RUNNING) return;
  __shared__ T sprod[kPipeTile];
  const int cur = c->cur;
  const int nxt = cur ^ 1;
  const T *__restrict__ xt = v.X[nxt];
  if ((int)blockIdx.x < gq) {
    T *__restrict__ qxt = v.QX[nxt];
    const T *__restrict__ qd = v.qdiag;
    stream_pipelined<T, kPipeE>(
        (int)blockIdx.x, Q.nrb, gq, xt, sprod,
        [&](int b, StreamTile<T, kPipeE> &t) { tile_bounds(Q, b, 0, t); },
        [&](int, int row, T s) { qxt[row] = s + qd[row] * xt[row]; });
  } else {
    const int b = blockIdx.x - gq;
    RowTrial<T> rt(c, p);
    stream_pipelined<T, kPipeE>(
        b, A.nrb, ga, xt, sprod,
        [&](int rb, StreamTile<T, kPipeE> &t) { tile_bounds(A, rb, 0, t); },
        [&](int, int j, T ax) { rt(v, j, ax); });
    rt.reduce(v, b);
  }
}

// ===========================================================================
// Column-panel form of the same trial part (two launches).  The columns of
// Q_off and A are split at n/2 into two panels; each panel is a CSR of its
// own over all rows, with its own stream row blocks.  k_qa_panels: workgroup
// i works on panel i & 1 only -- workgroups are dispatched round-robin over
// the 8 XCDs, so the workgroups of an XCD gather from one half of x_tr,
// which stays in that XCD's L2 -- and writes each row's partial sum of its
// panel.  k_qa_rows then adds the two partials of every row in panel order
// and runs the same row epilogues as k_qa_stream.
// ===========================================================================
template <typename T>
struct QAPanels {
  CsrT<T> q0, q1, a0, a1;   // Q_off and A restricted to the two column panels
  T *pq0, *pq1, *pa0, *pa1; // per-row partial sums of each panel
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_qa_panels(Ctrl *__restrict__ c, IterVecs<T> v,
                                                      QAPanels<T> P) {
  if (c->state != ST_RUNNING) return;
  __shared__ T sprod[kPipeTile];
  const T *__restrict__ xt = v.X[c->cur ^ 1];
  const bool h = (blockIdx.x & 1) != 0;
  const CsrT<T> Q = h ? P.q1 : P.q0;
  const CsrT<T> A = h ? P.a1 : P.a0;
  T *__restrict__ pq = h ? P.pq1 : P.pq0;
  T *__restrict__ pa = h ? P.pa1 : P.pa0;
  const int items = Q.nrb + A.nrb;
  const int step = (int)(gridDim.x >> 1);
  stream_pipelined<T, kPipeE>(
      (int)(blockIdx.x >> 1), items, step, xt, sprod,
      [&](int it, StreamTile<T, kPipeE> &t) {
        if (it < Q.nrb)
          tile_bounds(Q, it, 0, t);
        else
          tile_bounds(A, it - Q.nrb, 1, t);
      },
      [&](int tag, int row, T s) { (tag ? pa : pq)[row] = s; });
}

// The constraint rows of the two-panel form: panel sums of A x_tr (panel 0
// first) and the row-local trial; one acceptance partial per workgroup.
// (The Q rows' panel sums are formed where they are first needed, in the
// epilogue of the A' product.)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_qa_rows(Ctrl *__restrict__ c, InnerParams p,
                                                    IterVecs<T> v, QAPanels<T> P, int ga) {
  if (c->state != ST_RUNNING) return;
  const int b = (int)blockIdx.x;
  if (b >= ga) return;  // no constraint rows: one idle workgroup
  RowTrial<T> rt(c, p);
  for_elems(p.m, b, ga, [&](int j) { rt(v, j, P.pa0[j] + P.pa1[j]); });
  rt.reduce(v, b);
}

// Trial step, sparse part 2, CSR-stream form: row blocks of A' (A' y_tr)
// and the x-block acceptance sums |dx (H dx)|, |dx (A' dy)| (FP64).  With
// the two-panel form (pq0, pq1 non-null) the epilogue also forms Q x_tr of
// its x element from the two panels' partial sums (panel 0 first) and the
// diagonal, the Q-row part of the first product that k_qa_rows leaves out.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_at_stream(Ctrl *__restrict__ c, InnerParams p,
                                                      IterVecs<T> v, CsrT<T> AT,
                                                      const T *__restrict__ pq0,
                                                      const T *__restrict__ pq1) {
  if (c->state != ST_RUNNING) return;
  __shared__ T sprod[kPipeTile];
  const int cur = c->cur;
  const int nxt = cur ^ 1;
  const double gi = p.gamma_inv;
  const T *__restrict__ yt = v.Y[nxt];
  const bool form_qx = pq0 != nullptr;
  double s5 = 0.0, s6 = 0.0;
  stream_pipelined<T, kPipeE>(
      (int)blockIdx.x, AT.nrb, (int)gridDim.x, yt, sprod,
      [&](int b, StreamTile<T, kPipeE> &t) { tile_bounds(AT, b, 0, t); },
      [&](int, int i, T a) {
        v.ATY[nxt][i] = a;
        const T xn = v.X[nxt][i];
        T qn;
        if (form_qx) {
          qn = (pq0[i] + pq1[i]) + v.qdiag[i] * xn;
          v.QX[nxt][i] = qn;
        } else {
          qn = v.QX[nxt][i];
        }
        const double dx = (double)xn - (double)v.X[cur][i];
        const double hdx = ((double)qn - (double)v.QX[cur][i]) + gi * dx;
        const double ady = (double)a - (double)v.ATY[cur][i];
        s5 += fabs(dx * hdx);
        s6 += fabs(dx * ady);
      });
  double vals[2] = {s5, s6};
  block_reduce<2>(vals, 0u, v.partial + PS_AT * kMaxParts, blockIdx.x);
}

// Control-block fields the acceptance decision reads, loaded at the start of
// the decision kernel so that their latency overlaps the partial loads.
struct DecideIn {
  int cur, N, t, t_call, rejects, ntr;
  double sc, om;
  int64_t trials, accepted, rejected;
};

__device__ __forceinline__ DecideIn load_decide_in(const Ctrl *__restrict__ c) {
  DecideIn d;
  d.cur = c->cur;
  d.N = c->N;
  d.t = c->t;
  d.t_call = c->t_call;
  d.rejects = c->rejects;
  d.ntr = c->trace_trials_n;
  d.sc = c->step_scale;
  d.om = c->omega;
  d.trials = c->trials;
  d.accepted = c->accepted;
  d.rejected = c->rejected;
  return d;
}

// Decision of the acceptance test (adaptive-condition) from the three
// kernels' sums; run by one thread.
__device__ void accept_decision(Ctrl *__restrict__ c, const DecideIn &d, const InnerParams &p,
                                double *trace_tr, double sx, const double (&sr)[4],
                                double sum_hdx, double sum_bdy) {
  const double sc = d.sc;
  const double om = d.om;
  const double L = 0.5 * ((om / sc) * (sx + sr[0]) + sr[1] / (sc * om));
  const double R = 0.5 * (sum_hdx + sr[2]) + (sum_bdy + sr[3]);
  c->sum_x = sx;
  for (int k = 0; k < 4; ++k) c->sum_row[k] = sr[k];
  c->L = L;
  c->R = R;
  c->trials = d.trials + 1;
  const bool finite = isfinite(L) && isfinite(R);
  const bool acc = finite && (L >= R);
  if (d.ntr < p.trace_trials_cap) {
    trace_tr[3 * d.ntr + 0] = L;
    trace_tr[3 * d.ntr + 1] = R;
    trace_tr[3 * d.ntr + 2] = acc ? 1.0 : 0.0;
    c->trace_trials_n = d.ntr + 1;
  }
  c->last_acc = acc ? 1 : 0;
  if (!finite) {
    c->state = ST_NUMERR;
    c->pending = 0;
  } else if (acc) {
    c->alpha_pend = 2.0 / ((double)d.N + 2.0);
    c->pending = 1;
    c->cur = d.cur ^ 1;
    c->N = d.N + 1;
    c->t = d.t + 1;
    c->t_call = d.t_call + 1;
    c->rejects = 0;
    c->accepted = d.accepted + 1;
    if (((d.t + 1) % p.check_every) == 0 || d.t_call + 1 >= p.max_inner) c->state = ST_CHECK_DUE;
  } else {
    double kappa = p.shrink_safety * L / R;
    kappa = kappa < p.shrink_min ? p.shrink_min : (kappa > p.shrink_max ? p.shrink_max : kappa);
    c->step_scale = kappa * sc;
    c->pending = 0;
    c->rejects = d.rejects + 1;
    c->rejected = d.rejected + 1;
    if (d.rejects + 1 >= p.max_rejects) c->state = ST_NUMERR;
  }
}

// Acceptance test of the trial: one workgroup adds the partials of the three
// trial kernels in a fixed order (the kernel boundaries order their writes;
// no fences are needed) and takes the decision.
__global__ __launch_bounds__(kDecideThreads) void k_decide(Ctrl *__restrict__ c, InnerParams p,
                                                           const double *__restrict__ part,
                                                           double *trace_tr, int gx, int ga,
                                                           int gt) {
  const int state = c->state;
  const DecideIn din = load_decide_in(c);
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
    accept_decision(c, din, p, trace_tr, r[0], sr, r[5], r[6]);
  }
}

// Copies the accepted iterate (x, s, r, y) into the FP64 trace buffers.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_trace(Ctrl *__restrict__ c, InnerParams p,
                                                  IterVecs<T> v) {
  if (!c->last_acc || c->trace_iters_n >= p.trace_iters_cap) return;
  const int k = c->trace_iters_n;
  const int cur = c->cur;
  const int n = p.n, mi = p.mi, m = p.m, dw = p.dw;
  double *tw = v.trace_w + (size_t)k * dw;
  double *ty = v.trace_y + (size_t)k * m;
  for_elems(dw + m, blockIdx.x, gridDim.x, [&](int i) {
    if (i < n) tw[i] = (double)v.X[cur][i];
    else if (i < n + mi) tw[i] = (double)v.S[cur][i - n];
    else if (i < dw) tw[i] = (double)v.R[cur][i - n - mi];
    else ty[i - dw] = (double)v.Y[cur][i - dw];
  });
}

// Advances the trace counter (one thread, after k_trace).
__global__ void k_trace_done(Ctrl *__restrict__ c, InnerParams p) {
  if (!c->last_acc || c->trace_iters_n >= p.trace_iters_cap) return;
  c->trace_iters_n += 1;
  c->last_acc = 0;
}

// ===========================================================================
// Periodic check (stopping test of (inner-residuals)/(inner-scales)/
// (inner-termination) on the current and the averaged candidate, then the
// restart rule and primal-weight update (primal-weight-update)).
// ===========================================================================

// Brings the averages up to date (the averaging of the last accept is
// otherwise folded into the next trial).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_flush(Ctrl *__restrict__ c, InnerParams p,
                                                  IterVecs<T> v, Part px, Part pr) {
  if (c->state != ST_CHECK_DUE || !c->pending) return;
  const int cur = c->cur;
  const T ap = (T)c->alpha_pend;
  if ((int)blockIdx.x < px.blocks) {
    for_elems(p.n, blockIdx.x, px.blocks, [&](int i) {
      v.xbar[i] = (T(1) - ap) * v.xbar[i] + ap * v.X[cur][i];
      v.qxbar[i] = (T(1) - ap) * v.qxbar[i] + ap * v.QX[cur][i];
    });
  } else {
    const int b = blockIdx.x - px.blocks;
    for_elems(p.m, b, pr.blocks, [&](int j) {
      v.ybar[j] = (T(1) - ap) * v.ybar[j] + ap * v.Y[cur][j];
      v.rbar[j] = (T(1) - ap) * v.rbar[j] + ap * v.R[cur][j];
      if (j >= p.me) {
        const int k = j - p.me;
        v.sbar[k] = (T(1) - ap) * v.sbar[k] + ap * v.S[cur][k];
      }
    });
  }
}

// A xbar and A' ybar for the averaged candidate.
template <int GA, int GT, typename T>
__global__ __launch_bounds__(kBlock) void k_check_spmv(Ctrl *__restrict__ c, IterVecs<T> v,
                                                       CsrT<T> A, CsrT<T> AT, Part pa, Part pt) {
  if (c->state != ST_CHECK_DUE) return;
  if ((int)blockIdx.x < pa.blocks) {
    for_rows<GA>(A.rows, blockIdx.x, pa.blocks, [&](int j, int lane) {
      const T s = row_dot<GA, T>(A.p, A.i, A.v, v.xbar, j, lane);
      if (lane == 0) v.axbar[j] = s;
    });
  } else {
    for_rows<GT>(AT.rows, blockIdx.x - pa.blocks, pt.blocks, [&](int i, int lane) {
      const T s = row_dot<GT, T>(AT.p, AT.i, AT.v, v.ybar, i, lane);
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

// Residual quantities of both candidates over the x, s and row blocks, in
// FP64 from the stored values.  Gradient g = H w + q - B'y of (inner-qp):
//   x: Q x + x/gamma + (c - z/gamma) - A'y;  s: y_I;  r: sigma r + lambda + y.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_check(Ctrl *__restrict__ c, InnerParams p,
                                                  IterVecs<T> v, Part px, Part ps, Part pr) {
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
        a[CK_RD + cd] = fmax(a[CK_RD + cd], fabs(xv - clampv<double>(xv - g, lo, hi)));
        a[CK_HW + cd] = fmax(a[CK_HW + cd], fabs(hx));
        a[CK_BTY + cd] = fmax(a[CK_BTY + cd], fabs(atyv));
        const double dh = xv - clampv<double>(xv - s2 * g, lo, hi);
        a[CK_D + cd] += dh * dh / s2;
        const double dwv = xv - (double)v.xa[i];
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
        a[CK_RD + cd] = fmax(a[CK_RD + cd], fabs(sv - maxv<double>(sv - yv, bj)));
        a[CK_BTY + cd] = fmax(a[CK_BTY + cd], fabs(yv));
        const double dh = sv - maxv<double>(sv - s2 * yv, bj);
        a[CK_D + cd] += dh * dh / s2;
        const double dwv = sv - (double)v.sa[k];
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
      const double hj = (j < p.me) ? (double)v.b[j] : 0.0;
      for (int cd = 0; cd < ncand; ++cd) {
        const double rv = cd ? v.rbar[j] : v.R[cur][j];
        const double yv = cd ? v.ybar[j] : v.Y[cur][j];
        double bwv;
        if (cd) {
          bwv = (double)v.axbar[j] - rv;
          if (j >= p.me) bwv = (double)v.axbar[j] - (double)v.sbar[j - p.me] - rv;
        } else {
          bwv = v.BW[cur][j];
        }
        const double hr = sg * rv;
        const double g = hr + lm + yv;
        a[CK_RD + cd] = fmax(a[CK_RD + cd], fabs(g));
        a[CK_HW + cd] = fmax(a[CK_HW + cd], fabs(hr));
        a[CK_BTY + cd] = fmax(a[CK_BTY + cd], fabs(yv));
        a[CK_D + cd] += s2 * g * g;
        const double dwv = rv - (double)v.ra[j];
        a[CK_DW + cd] += dwv * dwv / s2;
        const double pres = hj - bwv;
        a[CK_RP + cd] = fmax(a[CK_RP + cd], fabs(pres));
        a[CK_BW + cd] = fmax(a[CK_BW + cd], fabs(bwv));
        a[CK_P + cd] += e2 * pres * pres;
        const double dyv = yv - (double)v.ya[j];
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
                                                                 InnerParams p,
                                                                 const double *__restrict__ part,
                                                                 int32_t *trace_ck, int nparts) {
  if (c->state != ST_CHECK_DUE) return;
  double a[CK_N];
#pragma unroll
  for (int k = 0; k < CK_N; ++k) a[k] = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kDecideThreads) {
#pragma unroll
    for (int k = 0; k < CK_N; ++k) {
      const double x = part[k * kMaxParts + i];
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
    c->state = ((double)c->trials >= p.pass_limit)
                   ? ST_PASS_LIMIT
                   : ((c->t_call >= p.max_inner) ? ST_ITER_LIMIT : ST_RUNNING);
  }
  c->check_kind = kind;
  c->check_which = which;
  if (c->trace_checks_n < p.trace_trials_cap) {
    const int k = c->trace_checks_n;
    trace_ck[4 * k + 0] = kind;
    trace_ck[4 * k + 1] = c->t;
    trace_ck[4 * k + 2] = which;
    trace_ck[4 * k + 3] = (int32_t)c->trials;
    c->trace_checks_n = k + 1;
  }
}

// Applies a check's outcome to the vectors: the average becomes the
// current iterate (with its products), and/or a restart resets the
// averages and anchors to the current iterate.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_apply(Ctrl *__restrict__ c, InnerParams p,
                                                  IterVecs<T> v, Part px, Part pr) {
  const int copy_avg = c->copy_avg;
  const int restart = c->restart_flag;
  if (!copy_avg && !restart) return;
  const int cur = c->cur;
  if ((int)blockIdx.x < px.blocks) {
    for_elems(p.n, blockIdx.x, px.blocks, [&](int i) {
      T xv = v.X[cur][i], qv = v.QX[cur][i];
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
      T rv = v.R[cur][j], yv = v.Y[cur][j];
      const bool ineq = j >= p.me;
      const int k = j - p.me;
      T sv = ineq ? v.S[cur][k] : T(0);
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

// Products of the starting point (Q x = Q_off x + diag(Q) x, A'y) and
// averages/anchors set to it; resets the epoch counters.  Row part: copies.
template <int G, typename T>
__global__ __launch_bounds__(kBlock) void k_inner_init(Ctrl *__restrict__ c, InnerParams p,
                                                       IterVecs<T> v, CsrT<T> Q, CsrT<T> AT,
                                                       Part pq, Part pr) {
  const int cur = c->cur;
  if ((int)blockIdx.x < pq.blocks) {
    for_rows<G>(Q.rows, blockIdx.x, pq.blocks, [&](int i, int lane) {
      const T xv = v.X[cur][i];
      const T qx = row_dot<G, T>(Q.p, Q.i, Q.v, v.X[cur], i, lane) + v.qdiag[i] * xv;
      const T aty = row_dot<G, T>(AT.p, AT.i, AT.v, v.Y[cur], i, lane);
      if (lane == 0) {
        v.QX[cur][i] = qx;
        v.ATY[cur][i] = aty;
        v.xbar[i] = xv;
        v.qxbar[i] = qx;
        v.xa[i] = xv;
      }
    });
  } else {
    for_elems(p.m, blockIdx.x - pq.blocks, pr.blocks, [&](int j) {
      const T rv = v.R[cur][j], yv = v.Y[cur][j];
      v.rbar[j] = rv;
      v.ra[j] = rv;
      v.ybar[j] = yv;
      v.ya[j] = yv;
      if (j >= p.me) {
        const int k = j - p.me;
        const T sv = v.S[cur][k];
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

template <typename D, typename S>
__global__ __launch_bounds__(kBlock) void k_cast(D *__restrict__ dst, const S *__restrict__ src,
                                                 int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    dst[i] = (D)src[i];
}

inline int nz(int b) { return b > 0 ? b : 1; }

// Workgroups of the single-launch first product: the pipelined grid
// (kPipeGrid or the caller's stream_grid) split between the row blocks of
// Q_off (gq) and of A (ga, one acceptance partial each) in proportion to
// their counts; no A workgroups without constraint rows.
void qa_split(int qnrb, int anrb, int stream_grid, int &gq, int &ga) {
  const int G = stream_grid > 0 ? stream_grid : kPipeGrid;
  if (anrb <= 0) {
    gq = nz(std::min(qnrb, G));
    ga = 0;
    return;
  }
  const int64_t tot = (int64_t)qnrb + anrb;
  int q = (int)(((int64_t)G * qnrb + tot / 2) / tot);
  q = std::max(1, std::min(q, G - 1));
  gq = nz(std::min(qnrb, q));
  ga = nz(std::min(anrb, G - q));
}

}  // namespace

// Workgroups of the x step (one acceptance partial each): four elements per
// thread and pass, at most 512 workgroups (larger x takes several passes; the
// acceptance kernel then has fewer partials to add: measured 0.4 us faster
// per trial at n = 1M than one pass with 977 workgroups).
int xtrial_blocks(int n) {
  return nz((int)std::min<int64_t>(((int64_t)n + 4 * kBlock - 1) / (4 * kBlock), 512));
}

// ===========================================================================
// Launch wrappers.
// ===========================================================================
// Plain launch, or a launch whose dispatch records `ev` when timing is asked for.
template <typename... KArgs, typename... Args>
void launch_ev(void (*k)(KArgs...), dim3 grid, dim3 block, hipStream_t st, LaunchEvents ev,
               Args... args) {
  if (ev.start) {
    hipExtLaunchKernelGGL(k, grid, block, 0, st, ev.start, ev.stop, 0, static_cast<KArgs>(args)...);
  } else {
    hipLaunchKernelGGL(k, grid, block, 0, st, static_cast<KArgs>(args)...);
  }
}

template <typename T>
void launch_xtrial(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
                   LaunchEvents ev) {
  launch_ev(k_xtrial<T>, dim3(xtrial_blocks(p.n)), dim3(kBlock), st, ev, c, p, v);
}

template <typename T>
void launch_qa(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
               const CsrT<T> &Q, const CsrT<T> &A, LaunchEvents ev) {
  int gq, ga;
  qa_split(Q.nrb, A.nrb, p.stream_grid, gq, ga);
  launch_ev(k_qa_stream<T>, dim3(gq + ga), dim3(kBlock), st, ev, c, p, v, Q, A, gq, ga);
}

// Grid of the two-panel launch: both panels' items, interleaved (even
// workgroups panel 0, odd panel 1), at most kPipeGrid workgroups or the
// caller's stream_grid.
static int qa_panels_grid(int items0, int items1, int stream_grid) {
  const int cap = std::max((stream_grid > 0 ? stream_grid : kPipeGrid) / 2, 1);
  const int half = std::min(std::max(items0, items1), cap);
  return 2 * nz(half);
}

// Grid of the A' launch (one acceptance partial per workgroup).
static int at_grid(int nrb, int stream_grid) {
  return nz(std::min(nrb, stream_grid > 0 ? stream_grid : kPipeGrid));
}

// Workgroups of the constraint-row launch of the two-panel form, one
// acceptance partial each (four partial slots): at most 512 (measured at
// n = 1M: 512 instead of 1024 leaves the row kernel's time unchanged and
// takes 1.3 us off the acceptance kernel; 256 slows the row kernel).
static int qa_rows_blocks(int rows) {
  return nz((int)std::min<int64_t>(((int64_t)rows + kBlock - 1) / kBlock, 512));
}

template <typename T>
void launch_qa_panels(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
                      const QAPanelSet<T> &P, LaunchEvents ev) {
  QAPanels<T> k{P.q[0], P.q[1], P.a[0], P.a[1], P.pq[0], P.pq[1], P.pa[0], P.pa[1]};
  const int grid =
      qa_panels_grid(P.q[0].nrb + P.a[0].nrb, P.q[1].nrb + P.a[1].nrb, p.stream_grid);
  launch_ev(k_qa_panels<T>, dim3(grid), dim3(kBlock), st, ev, c, v, k);
}

template <typename T>
void launch_qa_rows(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
                    const QAPanelSet<T> &P, LaunchEvents ev) {
  QAPanels<T> k{P.q[0], P.q[1], P.a[0], P.a[1], P.pq[0], P.pq[1], P.pa[0], P.pa[1]};
  const int ga = p.m ? qa_rows_blocks(p.m) : 0;
  launch_ev(k_qa_rows<T>, dim3(nz(ga)), dim3(kBlock), st, ev, c, p, v, k, ga);
}

template <typename T>
void launch_at(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
               const CsrT<T> &AT, LaunchEvents ev, const T *pq0, const T *pq1) {
  launch_ev(k_at_stream<T>, dim3(at_grid(AT.nrb, p.stream_grid)), dim3(kBlock), st, ev, c, p, v,
            AT, pq0, pq1);
}

void launch_decide(hipStream_t st, Ctrl *c, const InnerParams &p, const double *partial,
                   double *trace_tr, int q_nrb, int a_nrb, int at_nrb, LaunchEvents ev,
                   bool panels) {
  const int gx = xtrial_blocks(p.n);
  int gq_unused = 0, ga = 0;
  if (panels)
    ga = p.m ? qa_rows_blocks(p.m) : 0;
  else
    qa_split(q_nrb, a_nrb, p.stream_grid, gq_unused, ga);
  const int gt = at_grid(at_nrb, p.stream_grid);
  launch_ev(k_decide, dim3(1), dim3(kDecideThreads), st, ev, c, p, partial, trace_tr, gx, ga, gt);
}

template <typename T>
void launch_trace(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v) {
  const int blocks = (int)std::min<int64_t>(((int64_t)p.dw + p.m + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_trace<T>, dim3(nz(blocks)), dim3(kBlock), 0, st, c, p, v);
  hipLaunchKernelGGL(k_trace_done, dim3(1), dim3(1), 0, st, c, p);
}

template <typename T>
void launch_flush(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
                  const Part &px, const Part &pr) {
  hipLaunchKernelGGL(k_flush<T>, dim3(nz(px.blocks + pr.blocks)), dim3(kBlock), 0, st, c, p, v,
                     px, pr);
}

template <typename T>
void launch_check_spmv(hipStream_t st, Ctrl *c, const IterVecs<T> &v, const CsrT<T> &A,
                       const CsrT<T> &AT, const Part &pa, const Part &pt) {
  PDNQP_DISPATCH_G(A.G, {
    constexpr int GA_ = GV;
    PDNQP_DISPATCH_G(AT.G, {
      hipLaunchKernelGGL((k_check_spmv<GA_, GV, T>), dim3(nz(pa.blocks + pt.blocks)),
                         dim3(kBlock), 0, st, c, v, A, AT, pa, pt);
    });
  });
}

template <typename T>
void launch_check(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
                  const Part &px, const Part &ps, const Part &pr) {
  const int g = nz(px.blocks + ps.blocks + pr.blocks);
  hipLaunchKernelGGL(k_check<T>, dim3(g), dim3(kBlock), 0, st, c, p, v, px, ps, pr);
  hipLaunchKernelGGL(k_check_decide, dim3(1), dim3(kDecideThreads), 0, st, c, p, v.partial,
                     v.trace_ck, g);
}

template <typename T>
void launch_apply(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
                  const Part &px, const Part &pr) {
  hipLaunchKernelGGL(k_apply<T>, dim3(nz(px.blocks + pr.blocks)), dim3(kBlock), 0, st, c, p, v,
                     px, pr);
  hipLaunchKernelGGL(k_apply_done, dim3(1), dim3(1), 0, st, c);
}

template <typename T>
void launch_inner_init(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
                       const CsrT<T> &Qoff, const CsrT<T> &AT, const Part &pr) {
  // one G for both matrices in this (cold) kernel: the larger of the two
  const int G = Qoff.G > AT.G ? Qoff.G : AT.G;
  Part pq = make_part(Qoff.rows, G, 1024);
  PDNQP_DISPATCH_G(G, {
    hipLaunchKernelGGL((k_inner_init<GV, T>), dim3(pq.blocks + pr.blocks), dim3(kBlock), 0, st, c,
                       p, v, Qoff, AT, pq, pr);
  });
}

template <typename D, typename S>
void launch_cast(hipStream_t st, D *dst, const S *src, int64_t n) {
  if (n <= 0) return;
  const int blocks = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 2048);
  hipLaunchKernelGGL((k_cast<D, S>), dim3(blocks), dim3(kBlock), 0, st, dst, src, n);
}

#define PDNQP_INSTANTIATE(T)                                                                      \
  template void launch_xtrial<T>(hipStream_t, Ctrl *, const InnerParams &, const IterVecs<T> &,  \
                                 LaunchEvents);                                                  \
  template void launch_qa<T>(hipStream_t, Ctrl *, const InnerParams &, const IterVecs<T> &,      \
                             const CsrT<T> &, const CsrT<T> &, LaunchEvents);                    \
  template void launch_at<T>(hipStream_t, Ctrl *, const InnerParams &, const IterVecs<T> &,      \
                             const CsrT<T> &, LaunchEvents, const T *, const T *);               \
  template void launch_qa_panels<T>(hipStream_t, Ctrl *, const InnerParams &,                    \
                                    const IterVecs<T> &, const QAPanelSet<T> &, LaunchEvents);   \
  template void launch_qa_rows<T>(hipStream_t, Ctrl *, const InnerParams &, const IterVecs<T> &, \
                                  const QAPanelSet<T> &, LaunchEvents);                          \
  template void launch_trace<T>(hipStream_t, Ctrl *, const InnerParams &, const IterVecs<T> &);  \
  template void launch_flush<T>(hipStream_t, Ctrl *, const InnerParams &, const IterVecs<T> &,   \
                                const Part &, const Part &);                                     \
  template void launch_check_spmv<T>(hipStream_t, Ctrl *, const IterVecs<T> &, const CsrT<T> &,  \
                                     const CsrT<T> &, const Part &, const Part &);               \
  template void launch_check<T>(hipStream_t, Ctrl *, const InnerParams &, const IterVecs<T> &,   \
                                const Part &, const Part &, const Part &);                       \
  template void launch_apply<T>(hipStream_t, Ctrl *, const InnerParams &, const IterVecs<T> &,   \
                                const Part &, const Part &);                                     \
  template void launch_inner_init<T>(hipStream_t, Ctrl *, const InnerParams &,                   \
                                     const IterVecs<T> &, const CsrT<T> &, const CsrT<T> &,      \
                                     const Part &);

PDNQP_INSTANTIATE(double)
PDNQP_INSTANTIATE(float)
template void launch_cast<float, double>(hipStream_t, float *, const double *, int64_t);
template void launch_cast<double, float>(hipStream_t, double *, const float *, int64_t);

}  // namespace pdnqp
