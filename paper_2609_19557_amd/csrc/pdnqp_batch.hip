// Persistent batched PDNQP kernel for gfx950: one workgroup solves one
// instance at a time, from the outer scaling to the unscaled result, then
// takes the next instance from a device queue.
//
// The steps and their arithmetic are those of the multi-kernel path (set-up
// of Section 3.1 with the Lanczos choice of the proximal step, the inner-QP
// formation of (inner-qp)/(inner-warm-start)/(diagonal-steps), the trial
// step (pdqp-trial) with the acceptance test (adaptive-condition), the
// periodic check with restarts (inner-termination), (primal-weight-update),
// and the outer update (practical-multiplier-update)/(penalty-trigger-eq)/
// (inner-tolerance-factor)/(center-update)), with three differences of
// form, not of result:
//  * control state lives in registers, identical in every thread: each
//    decision is taken by all threads from the same block-reduced values;
//    the clock and the queue are read by thread 0 and broadcast;
//  * sparse products walk the instance's stream row blocks one tile at a
//    time (unit-stride loads of a tile's nonzeros, products staged in LDS,
//    one thread per row adds its products in order);
//  * when they fit, the trial iterate x_tr and y_tr (and at checks the
//    averages) are staged in LDS, so the products' gathers read LDS.
// Reductions are deterministic (fixed shuffle tree, then waves in order).
#include "pdnqp_batch.hpp"
#include "pdnqp_device.hpp"

#include <cmath>
#include <cstdint>
#include <type_traits>

namespace pdnqp {

namespace {

using dev::clampv;
using dev::maxv;

constexpr int kRed = 20;  // values per block reduction (the check uses 19)

struct BShared {
  double red[16][kRed];
  double res[kRed];
  double bc[4];
  double aam[kAAMem][kAAMem + 1];  // Anderson Gram system (thread 0)
  uint64_t clock;
  int32_t inst;
  int32_t aawin[kAAMem + 1];       // Anderson window: history slots, oldest first
};

// Check reduction slots (per candidate cd = 0 current, 1 average).
enum : int {
  BK_RP = 0, BK_BW = 2, BK_RD = 4, BK_HW = 6, BK_BTY = 8, BK_Q = 10,
  BK_P = 11, BK_D = 13, BK_DW = 15, BK_DY = 17, BK_N = 19
};
constexpr uint32_t kBkMaxMask = (1u << BK_P) - 1u;

template <typename T>
__device__ __forceinline__ T vmax(T a, T b) {
  return fmax(a, b);
}

// Values every lane holds identically (read back from LDS broadcasts) are
// moved to scalar registers.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ double uni(double x) {
  const uint64_t b = __double_as_longlong(x);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ uint64_t uni(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Smallest eigenvalue of the symmetric tridiagonal (a, b) by bisection on
// Sturm counts from the Gershgorin interval (one thread).
__device__ double tridiag_min_eig_dev(const double *a, const double *b, int k) {
  double lo = INFINITY, hi = -INFINITY, bmax2 = 0.0;
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i < k - 1 ? fabs(b[i]) : 0.0);
    lo = fmin(lo, a[i] - r);
    hi = fmax(hi, a[i] + r);
    if (i < k - 1) bmax2 = fmax(bmax2, b[i] * b[i]);
  }
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, bmax2);
  const double eps = 2.220446049250313e-16;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin) break;
    if (mid <= lo || mid >= hi) break;
    int cnt = 0;
    double d = a[0] - mid;
    if (fabs(d) < pivmin) d = -pivmin;
    if (d < 0) ++cnt;
    for (int i = 1; i < k; ++i) {
      d = a[i] - mid - b[i - 1] * b[i - 1] / d;
      if (fabs(d) < pivmin) d = -pivmin;
      if (d < 0) ++cnt;
    }
    if (cnt >= 1) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// Control state of the inner iteration (uniform across the workgroup).
struct CtrlR {
  int state, cur, N, t, t_call, rejects, pending, last_acc;
  int restart_flag, copy_avg;
  int trace_iters_n, trace_trials_n, trace_checks_n;
  double alpha_pend, step_scale, omega, kkt_anchor, kkt_prev;
  int64_t trials, accepted, rejected, restarts, checks;
};

// Pointers in the global address space, held in scalar registers.  Each
// phase loads the few it needs from the instance descriptor at its start,
// so that no more than those stay live.
template <typename T>
using gp = __attribute__((address_space(1))) T *;
template <typename T>
using lp = __attribute__((address_space(3))) T *;

template <typename T>
__device__ __forceinline__ gp<T> G(T *p) {
  const uint64_t b = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return (gp<T>)(((uint64_t)hi << 32) | lo);
}

template <typename T, int BT, bool STAGE>
struct BSolver {
  static constexpr int W = BT / 64;
  static constexpr int TILE = (BT * 8 < 4096) ? BT * 8 : 4096;
  static constexpr int E = TILE / BT;
  static constexpr bool F32 = std::is_same<T, float>::value;

  const BatchInst &I;
  BShared &sh;
  lp<double> prod64;  // LDS, TILE doubles
  lp<T> prodT;        // same memory as prod64
  lp<T> lx, ly;       // LDS staging of gathered vectors (STAGE)
  int n, m, me, mi;
  CtrlR c;
  double gamma_inv, delta_a, delta_r, h_norm;
  int mode_init;
  int rpar;  // which of the two buffers of the inner Ruiz scalings is current

  __device__ BSolver(const BatchInst &inst, BShared &s, lp<double> lds)
      : I(inst), sh(s), prod64(lds), prodT((lp<T>)lds) {
    n = uni(I.n);
    m = uni(I.m);
    me = uni(I.me);
    mi = uni(I.mi);
    lp<char> base = (lp<char>)lds + (size_t)TILE * 8;
    lx = (lp<T>)base;
    ly = (lp<T>)(base + ((size_t)n * sizeof(T) + 15) / 16 * 16);
    rpar = 0;
  }

  __device__ __forceinline__ const IterVecs<T> &iv() const {
    if constexpr (F32) return I.w32;
    else return I.w64;
  }
  __device__ __forceinline__ const T *qo_vals() const {
    if constexpr (F32) return I.Qo32;
    else return I.Qov;
  }
  __device__ __forceinline__ const T *a_vals() const {
    if constexpr (F32) return I.A32;
    else return I.Av;
  }
  __device__ __forceinline__ const T *at_vals() const {
    if constexpr (F32) return I.AT32;
    else return I.ATv;
  }
  // inner Ruiz scalings: current (alt = false) or the other buffer
  __device__ __forceinline__ gp<double> fx(bool alt) const { return G((rpar ^ (int)alt) ? I.Fx2 : I.v.Fx); }
  __device__ __forceinline__ gp<double> fs(bool alt) const { return G((rpar ^ (int)alt) ? I.Fs2 : I.v.Fs); }
  __device__ __forceinline__ gp<double> fr(bool alt) const { return G((rpar ^ (int)alt) ? I.Fr2 : I.v.Fr); }
  __device__ __forceinline__ gp<double> ee(bool alt) const { return G((rpar ^ (int)alt) ? I.E2buf : I.v.tmp_m); }

  // ---- block primitives ---------------------------------------------------
  template <int K>
  __device__ __forceinline__ void allreduce(double (&v)[K], uint32_t maxmask) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double x = v[k];
      const bool mx = (maxmask >> k) & 1u;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_down(x, off, 64);
        x = mx ? fmax(x, o) : x + o;
      }
      if (lane == 0) sh.red[wid][k] = x;
    }
    __syncthreads();
    if ((int)threadIdx.x < K) {
      const int k = threadIdx.x;
      const bool mx = (maxmask >> k) & 1u;
      double acc = sh.red[0][k];
      for (int w = 1; w < W; ++w) acc = mx ? fmax(acc, sh.red[w][k]) : acc + sh.red[w][k];
      sh.res[k] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = uni(sh.res[k]);
  }

  __device__ __forceinline__ double bcast0(double x) {
    if (threadIdx.x == 0) sh.bc[0] = x;
    __syncthreads();
    const double r = uni(sh.bc[0]);
    __syncthreads();
    return r;
  }

  __device__ __forceinline__ uint64_t clock_now() {
    if (threadIdx.x == 0) sh.clock = wall_clock64();
    __syncthreads();
    const uint64_t r = uni(sh.clock);
    __syncthreads();
    return r;
  }

  template <typename F>
  __device__ __forceinline__ void elems(int count, F &&f) {
    for (int i = threadIdx.x; i < count; i += BT) f(i);
  }

  // Row-wise combination over a CSR matrix: for every row, the in-order sum
  // (or max when MAX) of entry(col, val) over the row's entries, passed to
  // fin(row, acc) on one thread.  S is the staging type.  Ends with a
  // barrier, so fin's writes are visible to the whole workgroup afterwards.
  //
  // Row block b holds rows [rb[b], rb[b+1]) (at most 2 BT of them) and
  // nonzeros [tb[b], tb[b+1]).  While block b is staged and summed, the
  // indices, values and row bounds of block b+1 and the extent of block b+2
  // are in flight: no load that a block's own sums depend on is issued in
  // that block's iteration.
  template <typename S, bool MAX, typename V, typename P, typename Fn>
  __device__ __forceinline__ void rows(const BCsr &M, const V *val_, lp<S> stage, P &&entry,
                                       Fn &&fin) {
    const gp<const int32_t> rp = G(M.p);
    const gp<const int32_t> ci = G(M.i);
    const gp<const int32_t> rb = G(M.rb);
    const gp<const int32_t> tb = G(M.tb);
    const gp<const V> val = G(val_);
    const int nrb = uni(M.nrb);
    if (nrb <= 0) return;
    int col[E], ncol[E];
    V vv[E], nvv[E];
    // row bounds of this thread's rows t and t + BT of a block: p[row], p[row + 1]
    int bnd[4], nbnd[4];
    auto load_block = [&](int r0_, int r1_, int bs, int cn, int (&cc)[E], V (&vl)[E],
                          int (&bd)[4]) {
      if (cn <= TILE) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int k = e * BT + threadIdx.x;
          cc[e] = 0;
          vl[e] = V(0);
          if (k < cn) {
            cc[e] = __builtin_nontemporal_load(&ci[bs + k]);
            vl[e] = __builtin_nontemporal_load(&val[bs + k]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int row = r0_ + j * BT + (int)threadIdx.x;
        bd[2 * j] = 0;
        bd[2 * j + 1] = 0;
        if (row < r1_) {
          bd[2 * j] = rp[row];
          bd[2 * j + 1] = rp[row + 1];
        }
      }
    };
    int r0 = uni(rb[0]), r1 = uni(rb[1]);
    int base = uni(tb[0]), end = uni(tb[1]);
    int r2 = 0, end2 = 0;  // end of the block after this one
    if (nrb > 1) {
      r2 = uni(rb[2]);
      end2 = uni(tb[2]);
    }
    load_block(r0, r1, base, end - base, col, vv, bnd);
    for (int bk = 0; bk < nrb; ++bk) {
      const int cnt = end - base;
      const int nr0 = r1, nr1 = r2, nbase = end, nend = end2;
      if (bk + 1 < nrb) {
        load_block(nr0, nr1, nbase, nend - nbase, ncol, nvv, nbnd);
        if (bk + 2 < nrb) {
          r2 = uni(rb[bk + 3]);
          end2 = uni(tb[bk + 3]);
        }
      }
      if (cnt <= TILE) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int k = e * BT + threadIdx.x;
          if (k < cnt) stage[k] = entry(col[e], vv[e]);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int row = r0 + j * BT + (int)threadIdx.x;
          if (row < r1) {
            const int a = bnd[2 * j] - base;
            const int b = bnd[2 * j + 1] - base;
            S acc = S(0);
#pragma unroll 4
            for (int k = a; k < b; ++k) acc = MAX ? vmax<S>(acc, stage[k]) : acc + stage[k];
            fin(row, acc);
          }
        }
        __syncthreads();
      } else {
        // a single row longer than a tile: block reduction in FP64
        double acc = 0.0;
        for (int k = threadIdx.x; k < cnt; k += BT) {
          const double x = (double)entry(ci[base + k], val[base + k]);
          acc = MAX ? fmax(acc, x) : acc + x;
        }
        double vals[1] = {acc};
        allreduce<1>(vals, MAX ? 1u : 0u);
        if (threadIdx.x == 0) fin(r0, (S)vals[0]);
        __syncthreads();
      }
      r0 = nr0;
      r1 = nr1;
      base = nbase;
      end = nend;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        col[e] = ncol[e];
        vv[e] = nvv[e];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) bnd[j] = nbnd[j];
    }
  }

  // FP64 product M x: g(row, sum)
  template <typename Gf>
  __device__ __forceinline__ void spmv64(const BCsr &M, const double *val, gp<const double> x, Gf &&g) {
    rows<double, false>(M, val, prod64, [&](int col, double a) { return a * x[col]; }, g);
  }

  __device__ __forceinline__ double absmax64(gp<const double> a, int count) {
    double acc = 0.0;
    elems(count, [&](int i) { acc = fmax(acc, fabs(a[i])); });
    double vals[1] = {acc};
    allreduce<1>(vals, 1u);
    return vals[0];
  }

  // ---- set-up (Section 3.1) ------------------------------------------------
  __device__ __forceinline__ void outer_ruiz() {
    const gp<double> Dc = G(I.v.Dc), Dx = G(I.v.Dx);
    elems(m, [&](int j) { Dc[j] = 1.0; });
    elems(n, [&](int i) { Dx[i] = 1.0; });
    __syncthreads();
    if (I.st.outer_scaling == PDNQP_SCALE_NONE) return;
    const bool withq = I.st.outer_scaling == PDNQP_SCALE_RUIZ_QA;
    const gp<double> tm = G(I.v.tmp_m), tn = G(I.v.tmp_n), tq = G(I.v.qxo);
    const int sweeps = uni(I.st.ruiz_sweeps);
    for (int sw = 0; sw < sweeps; ++sw) {
      // row norms of Dc A Dx, column norms (rows of A'), optionally of Dx Q Dx
      rows<double, true>(I.A, I.Araw, prod64, [&](int col, double a) { return fabs(a) * Dx[col]; },
                         [&](int r, double mx) { tm[r] = Dc[r] * mx; });
      rows<double, true>(I.AT, I.ATraw, prod64, [&](int col, double a) { return fabs(a) * Dc[col]; },
                         [&](int r, double mx) { tn[r] = Dx[r] * mx; });
      if (withq)
        rows<double, true>(I.Q, I.Qraw, prod64, [&](int col, double a) { return fabs(a) * Dx[col]; },
                           [&](int r, double mx) { tq[r] = Dx[r] * mx; });
      elems(m, [&](int j) {
        const double r = tm[j];
        Dc[j] = Dc[j] / sqrt(r > 0.0 ? r : 1.0);
      });
      elems(n, [&](int i) {
        double cv = tn[i];
        if (withq) cv = fmax(cv, tq[i]);
        Dx[i] = Dx[i] / sqrt(cv > 0.0 ? cv : 1.0);
      });
      __syncthreads();
    }
  }

  __device__ __forceinline__ double scale_data() {
    const gp<const double> Dc = G(I.v.Dc), Dx = G(I.v.Dx);
    const gp<double> X0 = G(I.v.X[0]);
    const gp<double> tn = G(I.v.tmp_n);
    const gp<const double> craw = G(I.craw);
    // c_obj = 1 / max(1, ||Dx (Q x0 + c)||_inf)
    spmv64(I.Q, I.Qraw, X0, [&](int r, double s) { tn[r] = Dx[r] * (s + craw[r]); });
    const double co = 1.0 / fmax(1.0, absmax64(tn, n));
    // scaled values: Q <- c_obj Dx Q Dx, A <- Dc A Dx, A' gathered from A
    auto scale_rows = [&](const BCsr &M, const double *raw_, double *out_, gp<const double> wr,
                          gp<const double> wc, double s) {
      const gp<const int32_t> rp = G(M.p), ci = G(M.i);
      const gp<const double> raw = G(raw_);
      const gp<double> out = G(out_);
      elems(uni(M.rows), [&](int r) {
        const double w = wr[r];
        for (int k = rp[r]; k < rp[r + 1]; ++k) out[k] = s * ((w * raw[k]) * wc[ci[k]]);
      });
    };
    scale_rows(I.Q, I.Qraw, I.Qv, Dx, Dx, co);
    scale_rows(I.Qo, I.Qoraw, I.Qov, Dx, Dx, co);
    scale_rows(I.A, I.Araw, I.Av, Dc, Dx, 1.0);
    {
      const gp<double> qd = G(I.qdiag), c = G(I.c), lo = G(I.lo), hi = G(I.hi);
      const gp<const double> qdr = G(I.qdiag_raw), xl = G(I.xlraw), xu = G(I.xuraw);
      elems(n, [&](int i) {
        const double d = Dx[i];
        qd[i] = co * ((d * qdr[i]) * d);
        c[i] = (co * d) * craw[i];
        lo[i] = xl[i] / d;
        hi[i] = xu[i] / d;
        X0[i] = X0[i] / d;
      });
    }
    {
      const gp<double> b = G(I.b), lam = G(I.v.lam);
      const gp<const double> braw = G(I.braw);
      elems(m, [&](int j) {
        b[j] = Dc[j] * braw[j];
        lam[j] = co * lam[j] / Dc[j];
      });
    }
    __syncthreads();
    if (m > 0) {
      const gp<double> atv = G(I.ATv);
      const gp<const double> av = G(I.Av);
      const gp<const int32_t> perm = G(I.atperm);
      const int nnz = uni(G(I.A.p)[m]);
      elems(nnz, [&](int k) { atv[k] = av[perm[k]]; });
    }
    __syncthreads();
    return co;
  }

  // initial penalty and norms of the scaled data; returns sigma0
  __device__ __forceinline__ double penalty0(double &bE, double &bI, double &cn) {
    const gp<const double> X0 = G(I.v.X[0]);
    const gp<double> tn = G(I.v.tmp_n), ax = G(I.v.ax);
    spmv64(I.Q, I.Qv, X0, [&](int r, double s) { tn[r] = s; });
    spmv64(I.A, I.Av, X0, [&](int r, double s) { ax[r] = s; });
    const gp<const double> c = G(I.c), b = G(I.b);
    double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // x'Qx, c'x, |viol|^2, |b_E|, |b_I|, |c|
    elems(n, [&](int i) {
      a[0] += X0[i] * tn[i];
      a[1] += c[i] * X0[i];
      a[5] = fmax(a[5], fabs(c[i]));
    });
    elems(m, [&](int j) {
      const double axj = ax[j];
      const double bj = b[j];
      const double vj = (j < me) ? axj - bj : axj - maxv<double>(axj, bj);
      a[2] += vj * vj;
      if (j < me) a[3] = fmax(a[3], fabs(bj));
      else a[4] = fmax(a[4], fabs(bj));
    });
    allreduce<6>(a, 0x38u);
    const double f = 0.5 * a[0] + a[1];
    const double vv = m ? a[2] : 0.0;
    bE = (m && me) ? a[3] : 0.0;
    bI = (m && m > me) ? a[4] : 0.0;
    cn = a[5];
    double s0 = I.st.sigma_init * fmax(1.0, fabs(f)) / fmax(1.0, 0.5 * vv);
    return fmin(fmax(s0, I.st.sigma0_min), I.st.sigma0_max);
  }

  __device__ __forceinline__ void setup(double &c_obj, double &gamma, double &lam_hat, double &bE, double &bI,
                        double &cn) {
    outer_ruiz();
    c_obj = scale_data();
    // proximal step (R-choice)
    if (I.st.gamma_override > 0) {
      gamma = I.st.gamma_override;
      lam_hat = NAN;
    } else {
      const gp<double> tn = G(I.v.tmp_n);
      rows<double, false>(I.Q, I.Qv, prod64, [&](int, double a) { return fabs(a); },
                          [&](int r, double s) { tn[r] = s; });
      const double qn = absmax64(tn, n);
      lam_hat = lanczos(fmax(1.0, qn));
      gamma = 1.0 / (fmax(0.0, -lam_hat) + I.st.delta_gamma * fmax(1.0, qn));
    }
    const double s0 = penalty0(bE, bI, cn);
    {
      const gp<double> sig = G(I.v.sigma), y0 = G(I.v.Y[0]), z = G(I.v.z);
      const gp<const double> lam = G(I.v.lam), X0 = G(I.v.X[0]);
      elems(m, [&](int j) {
        sig[j] = s0;
        y0[j] = -lam[j];
      });
      elems(n, [&](int i) { z[i] = X0[i]; });
    }
    if constexpr (F32) {
      const IterVecs<float> &w = I.w32;
      {
        const gp<float> d = G(I.Qo32);
        const gp<const double> s = G(I.Qov);
        elems(uni(G(I.Qo.p)[n]), [&](int k) { d[k] = (float)s[k]; });
      }
      if (m > 0) {
        const gp<float> a32 = G(I.A32), at32 = G(I.AT32);
        const gp<const double> av = G(I.Av), atv = G(I.ATv);
        elems(uni(G(I.A.p)[m]), [&](int k) {
          a32[k] = (float)av[k];
          at32[k] = (float)atv[k];
        });
      }
      {
        const gp<float> qd = G(const_cast<float *>(w.qdiag)), lo = G(const_cast<float *>(w.lo)),
                        hi = G(const_cast<float *>(w.hi)), b = G(const_cast<float *>(w.b));
        const gp<const double> qd64 = G(I.qdiag), lo64 = G(I.lo), hi64 = G(I.hi), b64 = G(I.b);
        elems(n, [&](int i) {
          qd[i] = (float)qd64[i];
          lo[i] = (float)lo64[i];
          hi[i] = (float)hi64[i];
        });
        elems(m, [&](int j) { b[j] = (float)b64[j]; });
      }
    }
    __syncthreads();
  }

  // Plain Lanczos on the scaled Q from the normalised all-ones vector.
  __device__ __forceinline__ double lanczos(double qnorm) {
    const int k = uni(I.st.lanczos_iters) < n ? uni(I.st.lanczos_iters) : n;
    const gp<double> vv = G(I.v.qxo), vp = G(I.v.atl), w = G(I.v.tmp_n), lz = G(I.lz);
    const double v0 = 1.0 / sqrt((double)n);
    elems(n, [&](int i) {
      vv[i] = v0;
      vp[i] = 0.0;
    });
    __syncthreads();
    double beta_prev = 0.0;
    int cnt = 0;
    for (int j = 0; j < k; ++j) {
      spmv64(I.Q, I.Qv, vv, [&](int r, double s) { w[r] = s; });
      double a1[1] = {0.0};
      elems(n, [&](int i) { a1[0] += vv[i] * w[i]; });
      allreduce<1>(a1, 0u);
      const double alpha = a1[0];
      double a2[1] = {0.0};
      elems(n, [&](int i) {
        const double wn = (w[i] - alpha * vv[i]) - beta_prev * vp[i];
        w[i] = wn;
        a2[0] += wn * wn;
      });
      allreduce<1>(a2, 0u);
      const double beta = sqrt(a2[0]);
      if (threadIdx.x == 0) lz[j] = alpha;
      cnt = j + 1;
      if (j == k - 1 || beta <= 1e-14 * qnorm) break;
      if (threadIdx.x == 0) lz[k + j] = beta;
      elems(n, [&](int i) {
        vp[i] = vv[i];
        vv[i] = w[i] / beta;
      });
      __syncthreads();
      beta_prev = beta;
    }
    double lam = 0.0;
    if (threadIdx.x == 0) {
      const double *l = (const double *)I.lz;
      lam = cnt == 1 ? l[0] : tridiag_min_eig_dev(l, l + k, cnt);
    }
    return bcast0(lam);
  }

  // ---- inner-QP formation ---------------------------------------------------
  __device__ __forceinline__ void warm(double gamma) {
    const int cur = c.cur;
    const gp<double> ax = G(I.v.ax);
    spmv64(I.A, I.Av, G(I.v.X[cur]), [&](int r, double s) { ax[r] = s; });
    {
      const gp<double> R = G(I.v.R[cur]), BW = G(I.v.BW[cur]), S = G(I.v.S[cur]);
      const gp<const double> b = G(I.b), lam = G(I.v.lam), sig = G(I.v.sigma);
      elems(m, [&](int j) {
        const double axj = ax[j];
        if (j < me) {
          const double r = axj - b[j];
          R[j] = r;
          BW[j] = axj - r;
        } else {
          const int k = j - me;
          const double s = maxv<double>(axj + lam[j] / sig[j], b[j]);
          const double r = axj - s;
          S[k] = s;
          R[j] = r;
          BW[j] = axj - s - r;
        }
      });
    }
    {
      const gp<double> qx = G(I.v.qx);
      const gp<const double> cc = G(I.c), z = G(I.v.z);
      elems(n, [&](int i) { qx[i] = cc[i] - z[i] / gamma; });
    }
    {
      const gp<double> E = ee(false), Fr = fr(false), Fx = fx(false), Fs = fs(false);
      elems(m, [&](int j) {
        E[j] = 1.0;
        Fr[j] = 1.0;
      });
      elems(n, [&](int i) { Fx[i] = 1.0; });
      elems(mi, [&](int k) { Fs[k] = 1.0; });
    }
    __syncthreads();
  }

  __device__ __forceinline__ void form_inner(double gamma) {
    warm(gamma);
    if (m > 0) {
      const int sweeps = uni(I.st.ruiz_sweeps);
      for (int sw = 0; sw < sweeps; ++sw) {
        inner_ruiz_sweep();
        rpar ^= 1;
      }
    }
    steps(1.0 / gamma, I.st.step_boost);
    if constexpr (F32) cast_inner_to32();
    inner_init();
    mode_init = 1;
    check();
    mode_init = 0;
  }

  __device__ __forceinline__ void cast_inner_to32() {
    const IterVecs<float> &w = I.w32;
    const int cur = c.cur;
    {
      const gp<float> sg = G(w.sigma), lm = G(w.lam), tr = G(w.taub_r), eb = G(w.etab),
                      s2 = G(w.S2r), e2 = G(w.E2), R = G(w.R[cur]), Y = G(w.Y[cur]),
                      BW = G(w.BW[cur]);
      const gp<const double> sg6 = G(I.v.sigma), lm6 = G(I.v.lam), tr6 = G(I.v.taub_r),
                             eb6 = G(I.v.etab), s26 = G(I.v.S2r), e26 = G(I.v.E2),
                             R6 = G(I.v.R[cur]), Y6 = G(I.v.Y[cur]), BW6 = G(I.v.BW[cur]);
      elems(m, [&](int j) {
        sg[j] = (float)sg6[j];
        lm[j] = (float)lm6[j];
        tr[j] = (float)tr6[j];
        eb[j] = (float)eb6[j];
        s2[j] = (float)s26[j];
        e2[j] = (float)e26[j];
        R[j] = (float)R6[j];
        Y[j] = (float)Y6[j];
        BW[j] = (float)BW6[j];
      });
    }
    {
      const gp<float> qx = G(w.qx), tx = G(w.taub_x), s2 = G(w.S2x), X = G(w.X[cur]);
      const gp<const double> qx6 = G(I.v.qx), tx6 = G(I.v.taub_x), s26 = G(I.v.S2x),
                             X6 = G(I.v.X[cur]);
      elems(n, [&](int i) {
        qx[i] = (float)qx6[i];
        tx[i] = (float)tx6[i];
        s2[i] = (float)s26[i];
        X[i] = (float)X6[i];
      });
    }
    {
      const gp<float> ts = G(w.taub_s), s2 = G(w.S2s), S = G(w.S[cur]);
      const gp<const double> ts6 = G(I.v.taub_s), s26 = G(I.v.S2s), S6 = G(I.v.S[cur]);
      elems(mi, [&](int k) {
        ts[k] = (float)ts6[k];
        s2[k] = (float)s26[k];
        S[k] = (float)S6[k];
      });
    }
    __syncthreads();
  }

  // One inner Ruiz sweep on B diag(1, 1, 1/sqrt(sigma)).
  __device__ __forceinline__ void inner_ruiz_sweep() {
    const gp<const double> Fxo = fx(false), Fso = fs(false), Fro = fr(false), Eo = ee(false);
    const gp<double> Fxn = fx(true), Fsn = fs(true), Frn = fr(true), En = ee(true);
    const gp<const double> sig = G(I.v.sigma);
    rows<double, true>(I.A, I.Av, prod64, [&](int col, double a) { return fabs(a) * Fxo[col]; },
                       [&](int j, double mxa) {
                         const double e = Eo[j];
                         double mx = e * mxa;
                         const double pr = 1.0 / sqrt(sig[j]);
                         const double er = (e * pr) * Fro[j];
                         mx = fmax(mx, er);
                         if (j >= me) {
                           const int k = j - me;
                           const double es = e * Fso[k];
                           mx = fmax(mx, es);
                           Fsn[k] = Fso[k] / sqrt(es > 0.0 ? es : 1.0);
                         }
                         Frn[j] = Fro[j] / sqrt(er > 0.0 ? er : 1.0);
                         En[j] = e / sqrt(mx > 0.0 ? mx : 1.0);
                       });
    rows<double, true>(I.AT, I.ATv, prod64, [&](int col, double a) { return Eo[col] * fabs(a); },
                       [&](int i, double mxa) {
                         const double f = Fxo[i];
                         const double mx = mxa * f;
                         Fxn[i] = f / sqrt(mx > 0.0 ? mx : 1.0);
                       });
  }

  // Diagonal scales and steps (diagonal-scales), (diagonal-steps).
  __device__ __forceinline__ void steps(double gi, double boost) {
    const gp<const double> Fx = fx(false), Ec = ee(false), sig = G(I.v.sigma);
    const gp<double> offq = G(I.v.atl), b1v = G(I.v.qxo), tn = G(I.v.tmp_n);
    rows<double, false>(I.Qo, I.Qov, prod64, [&](int col, double a) { return fabs(a) * Fx[col]; },
                        [&](int i, double s) { offq[i] = s; });
    rows<double, false>(I.AT, I.ATv, prod64, [&](int col, double a) { return Ec[col] * fabs(a); },
                        [&](int i, double s) { b1v[i] = s; });
    {
      const gp<const double> qd = G(I.qdiag);
      const gp<double> S2x = G(I.v.S2x), tbx = G(I.v.taub_x);
      rows<double, false>(I.AT, I.ATv, prod64,
                          [&](int col, double a) {
                            const double eb = Ec[col] * fabs(a);
                            return sig[col] * (eb * eb);
                          },
                          [&](int i, double b2) {
                            const double si = Fx[i];
                            const double h1 = (offq[i] + fabs(qd[i] + gi) * si) * si;
                            const double bn1 = b1v[i] * si;
                            const double bn2 = sqrt(b2) * si;
                            const double mw = h1 + (bn1 > bn2 ? bn1 : bn2);
                            const double s2 = si * si;
                            S2x[i] = s2;
                            tbx[i] = boost * 0.99 * s2 / mw;
                            tn[i] = s2 / mw;
                          });
    }
    if (m == 0) return;
    const gp<const double> Fr = fr(false), Fs = fs(false);
    const gp<double> S2r = G(I.v.S2r), tbr = G(I.v.taub_r), S2s = G(I.v.S2s),
                     tbs = G(I.v.taub_s), E2 = G(I.v.E2), etab = G(I.v.etab);
    rows<double, false>(I.A, I.Av, prod64, [&](int col, double a) { return (a * a) * tn[col]; },
                        [&](int j, double acc) {
                          const double e = Ec[j];
                          const double sg = sig[j];
                          const double e2 = e * e;
                          const double sr = (1.0 / sqrt(sg)) * Fr[j];
                          const double mwr = (sr * sg) * sr + e * sr;
                          double my = e2 * acc + (e * sr) * (e * sr) / mwr;
                          S2r[j] = sr * sr;
                          tbr[j] = boost * 0.99 * (sr * sr) / mwr;
                          if (j >= me) {
                            const int k = j - me;
                            const double ss = Fs[k];
                            const double b1 = e * ss;
                            const double b2 = sqrt(sg * (b1 * b1));
                            const double mws = b1 > b2 ? b1 : b2;
                            my += b1 * b1 / mws;
                            S2s[k] = ss * ss;
                            tbs[k] = boost * 0.99 * (ss * ss) / mws;
                          }
                          E2[j] = e2;
                          etab[j] = boost * 0.99 * e2 / my;
                        });
  }

  // Products of the starting point, averages and anchors set to it.
  __device__ __forceinline__ void inner_init() {
    const IterVecs<T> &w = iv();
    const int cur = c.cur;
    {
      const gp<const T> x = G(w.X[cur]), qd = G(w.qdiag);
      const gp<T> QX = G(w.QX[cur]);
      rows<T, false>(I.Qo, qo_vals(), prodT, [&](int col, T a) { return a * x[col]; },
                     [&](int i, T s) { QX[i] = s + qd[i] * x[i]; });
    }
    {
      const gp<const T> y = G(w.Y[cur]);
      const gp<T> ATY = G(w.ATY[cur]);
      rows<T, false>(I.AT, at_vals(), prodT, [&](int col, T a) { return a * y[col]; },
                     [&](int i, T s) { ATY[i] = s; });
    }
    {
      const gp<const T> x = G(w.X[cur]), QX = G(w.QX[cur]);
      const gp<T> xbar = G(w.xbar), qxbar = G(w.qxbar), xa = G(w.xa);
      elems(n, [&](int i) {
        const T xv = x[i];
        xbar[i] = xv;
        qxbar[i] = QX[i];
        xa[i] = xv;
      });
    }
    {
      const gp<const T> R = G(w.R[cur]), Y = G(w.Y[cur]), S = G(w.S[cur]);
      const gp<T> rbar = G(w.rbar), ra = G(w.ra), ybar = G(w.ybar), ya = G(w.ya),
                  sbar = G(w.sbar), sa = G(w.sa);
      elems(m, [&](int j) {
        const T rv = R[j], yv = Y[j];
        rbar[j] = rv;
        ra[j] = rv;
        ybar[j] = yv;
        ya[j] = yv;
        if (j >= me) {
          const int k = j - me;
          const T sv = S[k];
          sbar[k] = sv;
          sa[k] = sv;
        }
      });
    }
    __syncthreads();
    c.state = ST_CHECK_DUE;
    c.N = 0;
    c.t = 0;
    c.t_call = 0;
    c.rejects = 0;
    c.pending = 0;
    c.step_scale = 1.0;
    c.restart_flag = 0;
    c.copy_avg = 0;
    c.last_acc = 0;
  }

  // ---- one trial step (pdqp-trial) and its acceptance test -------------------
  // Elementwise passes load U consecutive-stride elements per thread before
  // using any, so each pass pays a few memory round trips, not one per element.
  static constexpr int U = F32 ? 4 : 2;

  __device__ __forceinline__ void trial() {
    const IterVecs<T> &w = iv();
    const int cur = c.cur, nxt = cur ^ 1;
    const int pend = c.pending;
    const T ap = (T)c.alpha_pend;
    const double Nd = (double)c.N;
    const T alpha = (T)(2.0 / (Nd + 2.0));
    const T beta = (T)(Nd / (Nd + 1.0));
    const T sct = (T)(c.step_scale / c.omega);
    const T scy = (T)(c.step_scale * c.omega);
    const T gi = (T)gamma_inv;
    double sums[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // x block
    {
      const gp<const T> x = G(w.X[cur]), qx = G(w.QX[cur]), aty = G(w.ATY[cur]), ql = G(w.qx),
                        tbx = G(w.taub_x), lo = G(w.lo), hi = G(w.hi);
      const gp<T> xt = G(w.X[nxt]), xbar = G(w.xbar), qxbar = G(w.qxbar);
      const lp<T> sx = lx;
      for (int i0 = threadIdx.x; i0 < n; i0 += U * BT) {
        T xi[U], qxi[U], xb[U], qb[U], ay[U], qv[U], tb[U], l[U], h[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * BT;
          if (i < n) {
            xi[u] = x[i]; qxi[u] = qx[i]; xb[u] = xbar[i]; qb[u] = qxbar[i]; ay[u] = aty[i];
            qv[u] = ql[i]; tb[u] = tbx[i]; l[u] = lo[i]; h[u] = hi[i];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * BT;
          if (i < n) {
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
            if constexpr (STAGE) sx[i] = xn;
            const double d = (double)xn - (double)xi[u];
            sums[0] += d * d / (double)tb[u];
          }
        }
      }
    }
    __syncthreads();
    // Q_off x_tr; the diagonal term is added in the x-block pass below (its
    // first reader), where its loads are batched
    {
      const gp<const T> xtg = G(w.X[nxt]);
      const gp<T> QXn = G(w.QX[nxt]);
      const lp<T> sx = lx;
      auto xat = [&](int col) -> T {
        if constexpr (STAGE) return sx[col];
        else return xtg[col];
      };
      rows<T, false>(I.Qo, qo_vals(), prodT, [&](int col, T a) { return a * xat(col); },
                     [&](int i, T s) { QXn[i] = s; });
    }
    // A x_tr, parked (in LDS when staged, else in the check buffer A x_bar,
    // which is free between checks); then the row-local part of the trial
    {
      const gp<const T> xtg = G(w.X[nxt]);
      const lp<T> sx = lx;
      const lp<T> sy = ly;
      const gp<T> axp = G(w.axbar);
      auto xat = [&](int col) -> T {
        if constexpr (STAGE) return sx[col];
        else return xtg[col];
      };
      rows<T, false>(I.A, a_vals(), prodT, [&](int col, T a) { return a * xat(col); },
                     [&](int j, T ax) {
                       if constexpr (STAGE) sy[j] = ax;
                       else axp[j] = ax;
                     });
      const gp<const T> Yc = G(w.Y[cur]), BWc = G(w.BW[cur]), Rc = G(w.R[cur]), sig = G(w.sigma),
                        lam = G(w.lam), b = G(w.b), tbr_ = G(w.taub_r), Sc = G(w.S[cur]),
                        tbs_ = G(w.taub_s), etab = G(w.etab);
      const gp<T> ybar = G(w.ybar), rbar = G(w.rbar), sbar = G(w.sbar), Sn = G(w.S[nxt]),
                  Rn = G(w.R[nxt]), BWn = G(w.BW[nxt]), Yn = G(w.Y[nxt]);
      for (int j0 = threadIdx.x; j0 < m; j0 += U * BT) {
        T axv[U], y[U], bw[U], r[U], sg[U], lm[U], bj[U], rbv[U], tbr[U], eb[U], yb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int j = j0 + u * BT;
          if (j < m) {
            if constexpr (STAGE) axv[u] = sy[j];
            else axv[u] = axp[j];
            y[u] = Yc[j]; bw[u] = BWc[j]; r[u] = Rc[j]; sg[u] = sig[j]; lm[u] = lam[j];
            bj[u] = b[j]; rbv[u] = rbar[j]; tbr[u] = tbr_[j]; eb[u] = etab[j];
            yb[u] = pend ? ybar[j] : T(0);
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int j = j0 + u * BT;
          if (j < m) {
            T rb_ = rbv[u];
            if (pend) {
              ybar[j] = (T(1) - ap) * yb[u] + ap * y[u];
              rb_ = (T(1) - ap) * rb_ + ap * r[u];
              rbar[j] = rb_;
            }
            const T gr = (T(1) - alpha) * (sg[u] * rb_) + alpha * (sg[u] * r[u]) + lm[u] + y[u];
            const T rt = r[u] - (sct * tbr[u]) * gr;
            T bwt, hj;
            double ds = 0.0, ds2t = 0.0;
            if (j < me) {
              bwt = axv[u] - rt;
              hj = bj[u];
            } else {
              const int k = j - me;
              const T sv = Sc[k];
              if (pend) sbar[k] = (T(1) - ap) * sbar[k] + ap * sv;
              const T tbs = tbs_[k];
              const T st = maxv<T>(sv - (sct * tbs) * y[u], bj[u]);
              Sn[k] = st;
              bwt = axv[u] - st - rt;
              hj = T(0);
              ds = (double)st - (double)sv;
              ds2t = ds * ds / (double)tbs;
            }
            const T yt = y[u] + (scy * eb[u]) * (hj - bwt - beta * (bwt - bw[u]));
            Rn[j] = rt;
            BWn[j] = bwt;
            Yn[j] = yt;
            if constexpr (STAGE) sy[j] = yt;
            const double dr = (double)rt - (double)r[u];
            const double dy = (double)yt - (double)y[u];
            sums[1] += dr * dr / (double)tbr[u] + ds2t;
            sums[2] += dy * dy / (double)eb[u];
            sums[3] += fabs(dr * ((double)sg[u] * dr));
            sums[4] += fabs(dr * dy) + fabs(ds * dy);
          }
        }
      }
    }
    __syncthreads();
    // A' y_tr, then Q x_tr = Q_off x_tr + diag(Q) x_tr and the x-block
    // acceptance sums
    {
      const gp<const T> ytg = G(w.Y[nxt]);
      const lp<T> sy = ly;
      auto yat = [&](int col) -> T {
        if constexpr (STAGE) return sy[col];
        else return ytg[col];
      };
      const gp<T> ATYn = G(w.ATY[nxt]);
      rows<T, false>(I.AT, at_vals(), prodT, [&](int col, T a) { return a * yat(col); },
                     [&](int i, T a) { ATYn[i] = a; });
      const gp<const T> Xn = G(w.X[nxt]), Xc = G(w.X[cur]), QXc = G(w.QX[cur]),
                        ATYc = G(w.ATY[cur]), ATYr = G(w.ATY[nxt]), qd = G(w.qdiag);
      const gp<T> QXn = G(w.QX[nxt]);
      const double gid = gamma_inv;
      for (int i0 = threadIdx.x; i0 < n; i0 += U * BT) {
        T xn[U], xc[U], qn[U], qc[U], an[U], ac[U], dg[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * BT;
          if (i < n) {
            xn[u] = Xn[i]; xc[u] = Xc[i]; qn[u] = QXn[i]; qc[u] = QXc[i]; an[u] = ATYr[i];
            ac[u] = ATYc[i]; dg[u] = qd[i];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * BT;
          if (i < n) {
            qn[u] = qn[u] + dg[u] * xn[u];
            QXn[i] = qn[u];
            const double dx = (double)xn[u] - (double)xc[u];
            const double hdx = ((double)qn[u] - (double)qc[u]) + gid * dx;
            const double ady = (double)an[u] - (double)ac[u];
            sums[5] += fabs(dx * hdx);
            sums[6] += fabs(dx * ady);
          }
        }
      }
    }
    allreduce<7>(sums, 0u);
    decide(sums);
  }

  __device__ __forceinline__ void decide(const double (&r)[7]) {
    const double sc = c.step_scale;
    const double om = c.omega;
    const double L = 0.5 * ((om / sc) * (r[0] + r[1]) + r[2] / (sc * om));
    const double R = 0.5 * (r[5] + r[3]) + (r[6] + r[4]);
    c.trials += 1;
    const bool finite = isfinite(L) && isfinite(R);
    const bool acc = finite && (L >= R);
    if (c.trace_trials_n < uni(I.st.trace_trials)) {
      if (threadIdx.x == 0) {
        const gp<double> tr = G(I.v.trace_tr);
        tr[3 * c.trace_trials_n + 0] = L;
        tr[3 * c.trace_trials_n + 1] = R;
        tr[3 * c.trace_trials_n + 2] = acc ? 1.0 : 0.0;
      }
      c.trace_trials_n += 1;
    }
    c.last_acc = acc ? 1 : 0;
    if (!finite) {
      c.state = ST_NUMERR;
      c.pending = 0;
    } else if (acc) {
      c.alpha_pend = 2.0 / ((double)c.N + 2.0);
      c.pending = 1;
      c.cur ^= 1;
      c.N += 1;
      c.t += 1;
      c.t_call += 1;
      c.rejects = 0;
      c.accepted += 1;
      if ((c.t % uni(I.st.check_every)) == 0 || c.t_call >= uni(I.st.max_inner))
        c.state = ST_CHECK_DUE;
    } else {
      const double smin = I.st.shrink_min, smax = I.st.shrink_max;
      double kappa = I.st.shrink_safety * L / R;
      kappa = kappa < smin ? smin : (kappa > smax ? smax : kappa);
      c.step_scale = kappa * sc;
      c.pending = 0;
      c.rejects += 1;
      c.rejected += 1;
      if (c.rejects >= uni(I.st.max_rejects)) c.state = ST_NUMERR;
    }
  }

  __device__ __forceinline__ void trace_iterate() {
    const IterVecs<T> &w = iv();
    const int k = c.trace_iters_n;
    const int cur = c.cur;
    const int dw = n + mi + m;
    const gp<double> tw = G(I.v.trace_w + (size_t)k * dw);
    const gp<double> ty = G(I.v.trace_y + (size_t)k * m);
    const gp<const T> X = G(w.X[cur]), S = G(w.S[cur]), R = G(w.R[cur]), Y = G(w.Y[cur]);
    elems(dw + m, [&](int i) {
      if (i < n) tw[i] = (double)X[i];
      else if (i < n + mi) tw[i] = (double)S[i - n];
      else if (i < dw) tw[i] = (double)R[i - n - mi];
      else ty[i - dw] = (double)Y[i - dw];
    });
    c.trace_iters_n += 1;
  }

  // ---- periodic check (inner-termination), restart, primal weight ----------
  __device__ __forceinline__ void check_products() {
    const IterVecs<T> &w = iv();
    const int cur = c.cur;
    const lp<T> sx = lx, sy = ly;
    {
      const gp<T> xbar = G(w.xbar), qxbar = G(w.qxbar);
      const gp<const T> X = G(w.X[cur]), QX = G(w.QX[cur]);
      const int pend = c.pending;
      const T ap = (T)c.alpha_pend;
      elems(n, [&](int i) {
        T xb = xbar[i];
        if (pend) {
          xb = (T(1) - ap) * xb + ap * X[i];
          xbar[i] = xb;
          qxbar[i] = (T(1) - ap) * qxbar[i] + ap * QX[i];
        }
        if constexpr (STAGE) sx[i] = xb;
      });
    }
    {
      const gp<T> ybar = G(w.ybar), rbar = G(w.rbar), sbar = G(w.sbar);
      const gp<const T> Y = G(w.Y[cur]), R = G(w.R[cur]), S = G(w.S[cur]);
      const int pend = c.pending;
      const T ap = (T)c.alpha_pend;
      elems(m, [&](int j) {
        T yb = ybar[j];
        if (pend) {
          yb = (T(1) - ap) * yb + ap * Y[j];
          ybar[j] = yb;
          rbar[j] = (T(1) - ap) * rbar[j] + ap * R[j];
          if (j >= me) {
            const int k = j - me;
            sbar[k] = (T(1) - ap) * sbar[k] + ap * S[k];
          }
        }
        if constexpr (STAGE) sy[j] = yb;
      });
    }
    __syncthreads();
    {
      const gp<const T> xg = G(w.xbar);
      auto xat = [&](int col) -> T {
        if constexpr (STAGE) return sx[col];
        else return xg[col];
      };
      const gp<T> axbar = G(w.axbar);
      rows<T, false>(I.A, a_vals(), prodT, [&](int col, T a) { return a * xat(col); },
                     [&](int j, T s) { axbar[j] = s; });
    }
    {
      const gp<const T> yg = G(w.ybar);
      auto yat = [&](int col) -> T {
        if constexpr (STAGE) return sy[col];
        else return yg[col];
      };
      const gp<T> atybar = G(w.atybar);
      rows<T, false>(I.AT, at_vals(), prodT, [&](int col, T a) { return a * yat(col); },
                     [&](int i, T s) { atybar[i] = s; });
    }
  }

  __device__ __forceinline__ void check() {
    const IterVecs<T> &w = iv();
    const int cur = c.cur;
    const int ncand = mode_init ? 1 : 2;
    if (!mode_init) check_products();
    const double gi = gamma_inv;
    double a[BK_N];
#pragma unroll
    for (int k = 0; k < BK_N; ++k) a[k] = 0.0;
    {
      const gp<const T> qxv_ = G(w.qx), S2x = G(w.S2x), lo_ = G(w.lo), hi_ = G(w.hi),
                        X = G(w.X[cur]), xbar = G(w.xbar), QX = G(w.QX[cur]),
                        qxbar = G(w.qxbar), ATY = G(w.ATY[cur]), atybar = G(w.atybar),
                        xa = G(w.xa);
      elems(n, [&](int i) {
        const double q = qxv_[i];
        a[BK_Q] = fmax(a[BK_Q], fabs(q));
        const double s2 = S2x[i];
        const double lo = lo_[i], hi = hi_[i];
        for (int cd = 0; cd < ncand; ++cd) {
          const double xv = cd ? xbar[i] : X[i];
          const double qxv = cd ? qxbar[i] : QX[i];
          const double atyv = cd ? atybar[i] : ATY[i];
          const double hx = qxv + gi * xv;
          const double g = hx + q - atyv;
          a[BK_RD + cd] = fmax(a[BK_RD + cd], fabs(xv - clampv<double>(xv - g, lo, hi)));
          a[BK_HW + cd] = fmax(a[BK_HW + cd], fabs(hx));
          a[BK_BTY + cd] = fmax(a[BK_BTY + cd], fabs(atyv));
          const double dh = xv - clampv<double>(xv - s2 * g, lo, hi);
          a[BK_D + cd] += dh * dh / s2;
          const double dwv = xv - (double)xa[i];
          a[BK_DW + cd] += dwv * dwv / s2;
        }
      });
    }
    {
      const gp<const T> S2s = G(w.S2s), b = G(w.b), S = G(w.S[cur]), sbar = G(w.sbar),
                        Y = G(w.Y[cur]), ybar = G(w.ybar), sa = G(w.sa);
      elems(mi, [&](int k) {
        const int j = me + k;
        const double s2 = S2s[k];
        const double bj = b[j];
        for (int cd = 0; cd < ncand; ++cd) {
          const double sv = cd ? sbar[k] : S[k];
          const double yv = cd ? ybar[j] : Y[j];
          a[BK_RD + cd] = fmax(a[BK_RD + cd], fabs(sv - maxv<double>(sv - yv, bj)));
          a[BK_BTY + cd] = fmax(a[BK_BTY + cd], fabs(yv));
          const double dh = sv - maxv<double>(sv - s2 * yv, bj);
          a[BK_D + cd] += dh * dh / s2;
          const double dwv = sv - (double)sa[k];
          a[BK_DW + cd] += dwv * dwv / s2;
        }
      });
    }
    {
      const gp<const T> sig = G(w.sigma), lam = G(w.lam), S2r = G(w.S2r), E2 = G(w.E2),
                        b = G(w.b), R = G(w.R[cur]), rbar = G(w.rbar), Y = G(w.Y[cur]),
                        ybar = G(w.ybar), axbar = G(w.axbar), sbar = G(w.sbar),
                        BW = G(w.BW[cur]), ra = G(w.ra), ya = G(w.ya);
      elems(m, [&](int j) {
        const double sg = sig[j];
        const double lm = lam[j];
        a[BK_Q] = fmax(a[BK_Q], fabs(lm));
        const double s2 = S2r[j];
        const double e2 = E2[j];
        const double hj = (j < me) ? (double)b[j] : 0.0;
        for (int cd = 0; cd < ncand; ++cd) {
          const double rv = cd ? rbar[j] : R[j];
          const double yv = cd ? ybar[j] : Y[j];
          double bwv;
          if (cd) {
            bwv = (double)axbar[j] - rv;
            if (j >= me) bwv = (double)axbar[j] - (double)sbar[j - me] - rv;
          } else {
            bwv = BW[j];
          }
          const double hr = sg * rv;
          const double g = hr + lm + yv;
          a[BK_RD + cd] = fmax(a[BK_RD + cd], fabs(g));
          a[BK_HW + cd] = fmax(a[BK_HW + cd], fabs(hr));
          a[BK_BTY + cd] = fmax(a[BK_BTY + cd], fabs(yv));
          a[BK_D + cd] += s2 * g * g;
          const double dwv = rv - (double)ra[j];
          a[BK_DW + cd] += dwv * dwv / s2;
          const double pres = hj - bwv;
          a[BK_RP + cd] = fmax(a[BK_RP + cd], fabs(pres));
          a[BK_BW + cd] = fmax(a[BK_BW + cd], fabs(bwv));
          a[BK_P + cd] += e2 * pres * pres;
          const double dyv = yv - (double)ya[j];
          a[BK_DY + cd] += dyv * dyv / e2;
        }
      });
    }
    allreduce<BK_N>(a, kBkMaxMask);
    check_decide(a);
    if (c.copy_avg || c.restart_flag) apply();
    c.copy_avg = 0;
    c.restart_flag = 0;
  }

  __device__ __forceinline__ void check_decide(const double (&r)[BK_N]) {
    c.pending = 0;
    const double om = c.omega;
    const double k0 = sqrt(om * om * r[BK_P] + r[BK_D] / (om * om));
    if (mode_init) {
      c.kkt_anchor = k0;
      c.kkt_prev = INFINITY;
      c.state = ST_RUNNING;
      return;
    }
    c.checks += 1;
    bool pass[2];
    for (int cd = 0; cd < 2; ++cd) {
      const double spv = fmax(1.0, fmax(r[BK_BW + cd], h_norm));
      const double sdv = fmax(fmax(1.0, r[BK_HW + cd]), fmax(r[BK_Q], r[BK_BTY + cd]));
      pass[cd] = (r[BK_RP + cd] <= delta_a + delta_r * spv) &&
                 (r[BK_RD + cd] <= delta_a + delta_r * sdv);
    }
    int kind, which = 0;
    c.restart_flag = 0;
    c.copy_avg = 0;
    if (pass[0] || pass[1]) {
      which = pass[0] ? 0 : 1;
      kind = 2;
      c.copy_avg = which;
      c.state = ST_CONVERGED;
    } else {
      const double k1 = sqrt(om * om * r[BK_P + 1] + r[BK_D + 1] / (om * om));
      const int use_avg = (k1 < k0) ? 1 : 0;
      const double kc = use_avg ? k1 : k0;
      const bool restart = (kc <= I.st.restart_suff * c.kkt_anchor) ||
                           (kc <= I.st.restart_nec * c.kkt_anchor && kc > c.kkt_prev) ||
                           ((double)c.N >= I.st.restart_art * (double)c.t);
      which = use_avg;
      if (restart) {
        kind = 1;
        const double dW = sqrt(r[BK_DW + use_avg]);
        const double dY = sqrt(r[BK_DY + use_avg]);
        double omn = om;
        if (dW > 0.0 && dY > 0.0) omn = exp(0.25 * log(dY / dW) + 0.75 * log(om));
        c.omega = omn;
        c.step_scale = 1.0;
        c.N = 0;
        c.kkt_anchor = sqrt(omn * omn * r[BK_P + use_avg] + r[BK_D + use_avg] / (omn * omn));
        c.kkt_prev = INFINITY;
        c.restarts += 1;
        c.restart_flag = 1;
        c.copy_avg = use_avg;
      } else {
        kind = 0;
        c.kkt_prev = kc;
      }
      c.state = ((double)c.trials >= I.st.kkt_pass_limit)
                    ? ST_PASS_LIMIT
                    : ((c.t_call >= uni(I.st.max_inner)) ? ST_ITER_LIMIT : ST_RUNNING);
    }
    if (c.trace_checks_n < uni(I.st.trace_trials)) {
      if (threadIdx.x == 0) {
        const gp<int32_t> ck = G(I.v.trace_ck);
        ck[4 * c.trace_checks_n + 0] = kind;
        ck[4 * c.trace_checks_n + 1] = c.t;
        ck[4 * c.trace_checks_n + 2] = which;
        ck[4 * c.trace_checks_n + 3] = (int32_t)c.trials;
      }
      c.trace_checks_n += 1;
    }
  }

  __device__ __forceinline__ void apply() {
    const IterVecs<T> &w = iv();
    const int cur = c.cur;
    const int copy_avg = c.copy_avg, restart = c.restart_flag;
    {
      const gp<T> X = G(w.X[cur]), QX = G(w.QX[cur]), ATY = G(w.ATY[cur]), xbar = G(w.xbar),
                  qxbar = G(w.qxbar), xa = G(w.xa);
      const gp<const T> atybar = G(w.atybar);
      elems(n, [&](int i) {
        T xv = X[i], qv = QX[i];
        if (copy_avg) {
          xv = xbar[i];
          qv = qxbar[i];
          X[i] = xv;
          QX[i] = qv;
          ATY[i] = atybar[i];
        }
        if (restart) {
          xbar[i] = xv;
          qxbar[i] = qv;
          xa[i] = xv;
        }
      });
    }
    {
      const gp<T> R = G(w.R[cur]), Y = G(w.Y[cur]), S = G(w.S[cur]), BW = G(w.BW[cur]),
                  rbar = G(w.rbar), ybar = G(w.ybar), sbar = G(w.sbar), ra = G(w.ra),
                  ya = G(w.ya), sa = G(w.sa);
      const gp<const T> axbar = G(w.axbar);
      elems(m, [&](int j) {
        T rv = R[j], yv = Y[j];
        const bool ineq = j >= me;
        const int k = j - me;
        T sv = ineq ? S[k] : T(0);
        if (copy_avg) {
          rv = rbar[j];
          yv = ybar[j];
          R[j] = rv;
          Y[j] = yv;
          if (ineq) {
            sv = sbar[k];
            S[k] = sv;
            BW[j] = axbar[j] - sv - rv;
          } else {
            BW[j] = axbar[j] - rv;
          }
        }
        if (restart) {
          rbar[j] = rv;
          ybar[j] = yv;
          ra[j] = rv;
          ya[j] = yv;
          if (ineq) {
            sbar[k] = sv;
            sa[k] = sv;
          }
        }
      });
    }
    __syncthreads();
  }

  // Inner solve until convergence, the iteration limit, a numerical error
  // or the deadline (returns ST_RUNNING then).
  __device__ __forceinline__ int run_inner(uint64_t deadline) {
    int since_clock = 0;
    const int trace_cap = uni(I.st.trace_iters);
    const int check_every = uni(I.st.check_every);
    for (;;) {
      trial();
      if (c.last_acc && c.trace_iters_n < trace_cap) trace_iterate();
      c.last_acc = 0;
      if (c.state == ST_NUMERR) return ST_NUMERR;
      if (c.state == ST_CHECK_DUE) {
        check();
        if (c.state != ST_RUNNING) return c.state;
      }
      if (++since_clock >= 64 || c.t % check_every == 0) {
        since_clock = 0;
        if (clock_now() > deadline) return ST_RUNNING;
      }
    }
  }

  // multiplier update and outer residuals (o: twelve maxima).  o[0..7] on
  // the scaled data: r_p part, |A_E x|, |A_I x|, |r_row|, r_d, |Q x|,
  // |A' lambda|, |x - z|.  o[8..11] on the caller's data for the external
  // test of the experimental protocol: r_p part, max(|A x|, |b|), r_d,
  // max(|Q x|, |c|, |A' lambda|), with (A x)_j = (bar A bar x)_j / D_c,j,
  // x = D_x bar x clipped into the caller's box, Q x and A' lambda divided by
  // c_obj D_x.
  __device__ __forceinline__ void outer_update(double (&o)[12], double c_obj) {
    const int cur = c.cur;
    const gp<const double> x = G(I.v.X[cur]);
    for (int k = 0; k < 12; ++k) o[k] = 0.0;
    if (m) {
      const gp<double> ax = G(I.v.ax), lam = G(I.v.lam), rrow = G(I.v.rrow);
      const gp<const double> b = G(I.b), sig = G(I.v.sigma), Dc = G(I.v.Dc), br = G(I.braw);
      spmv64(I.A, I.Av, x, [&](int j, double axj) {
        ax[j] = axj;
        const double bj = b[j];
        const double sg = sig[j];
        const double lm = lam[j];
        const double axr = axj / Dc[j];
        const double brj = br[j];
        double rr;
        if (j < me) {
          const double res = axj - bj;
          lam[j] = lm + sg * res;
          rr = res;
          o[0] = fmax(o[0], fabs(res));
          o[1] = fmax(o[1], fabs(axj));
          o[8] = fmax(o[8], fabs(axr - brj));
        } else {
          const double s = maxv<double>(axj + lm / sg, bj);
          const double ln = lm + sg * (axj - bj);
          lam[j] = ln < 0.0 ? ln : 0.0;
          rr = axj - s;
          o[0] = fmax(o[0], maxv<double>(bj - axj, 0.0));
          o[2] = fmax(o[2], fabs(axj));
          o[8] = fmax(o[8], maxv<double>(brj - axr, 0.0));
        }
        rrow[j] = rr;
        o[3] = fmax(o[3], fabs(rr));
        o[9] = fmax(o[9], fmax(fabs(axr), fabs(brj)));
      });
    }
    const gp<double> qxo = G(I.v.qxo), atl = G(I.v.atl);
    spmv64(I.Q, I.Qv, x, [&](int i, double s) { qxo[i] = s; });
    spmv64(I.AT, I.ATv, G(I.v.lam), [&](int i, double s) { atl[i] = s; });
    const gp<const double> cc = G(I.c), lo = G(I.lo), hi = G(I.hi), z = G(I.v.z);
    const gp<const double> Dx = G(I.v.Dx), cr = G(I.craw), xlr = G(I.xlraw), xur = G(I.xuraw);
    elems(n, [&](int i) {
      const double xv = x[i];
      const double qx = qxo[i], al = atl[i];
      const double pr = clampv<double>(xv - qx - cc[i] - al, lo[i], hi[i]);
      o[4] = fmax(o[4], fabs(xv - pr));
      o[5] = fmax(o[5], fabs(qx));
      o[6] = fmax(o[6], fabs(al));
      o[7] = fmax(o[7], fabs(xv - z[i]));
      const double dx = Dx[i];
      const double sc = 1.0 / (c_obj * dx);
      const double xl = xlr[i], xu = xur[i];
      const double xr = clampv<double>(dx * xv, xl, xu);
      const double qr = qx * sc, ar = al * sc, ci = cr[i];
      const double prr = clampv<double>(xr - qr - ci - ar, xl, xu);
      o[10] = fmax(o[10], fabs(xr - prr));
      o[11] = fmax(o[11], fmax(fmax(fabs(qr), fabs(ci)), fabs(ar)));
    });
    allreduce<12>(o, 0xFFFu);
  }

  // row penalties (penalty-trigger-eq); returns whether a penalty changed
  __device__ __forceinline__ bool penalties(bool have_prev, double rn, double gate_tol) {
    const double theta = I.st.theta_sigma, growth = I.st.sigma_growth;
    const double sig_max = I.st.sigma_max;
    const int gate = uni(I.st.penalty_gate);
    const gp<double> sig = G(I.v.sigma), rprev = G(I.v.rprev);
    const gp<const double> rrow = G(I.v.rrow), lam = G(I.v.lam);
    double moved[1] = {0.0};
    elems(m, [&](int j) {
      const double r = rrow[j];
      if (have_prev && rn > 0.0) {
        const bool active = (j < me) || (lam[j] < 0.0);
        bool trig = fabs(r) > theta * fabs(rprev[j]) && active;
        if (gate) trig = trig && (fabs(r) > gate_tol);
        if (trig) {
          const double fac = fmax(1.0, growth * fabs(r) / rn);
          const double so = sig[j];
          const double sn = so * fac;
          const double s2 = sn < sig_max ? sn : sig_max;
          sig[j] = s2;
          if (s2 != so) moved[0] = 1.0;
        }
      }
      rprev[j] = r;
    });
    allreduce<1>(moved, 1u);
    return moved[0] != 0.0;
  }

  // ---- Anderson acceleration of (lambda_E, lambda_I, z) (Section 3.2) ------
  // Same readings as the oracle: active when r_p meets the tolerance, no
  // penalty changed and r_d decreased; history cleared when the residuals
  // grew after an extrapolation; lambda_I <= 0 and z in the box after it;
  // the inner dual warm start follows (y = -lambda).
  struct AAState {
    int count;  // entries of the window sh.aawin
    int form_slot;
    bool last_valid;
    double last_rp, last_rd;
    int steps;
  };

  __device__ __forceinline__ int aa_win(int j) { return uni((int)sh.aawin[j]); }

  __device__ __forceinline__ void aa_pack(double *dst_) {
    const gp<double> dst = G(dst_);
    const gp<const double> lam = G(I.v.lam), z = G(I.v.z);
    elems(m + n, [&](int i) { dst[i] = i < m ? lam[i] : z[i - m]; });
    __syncthreads();
  }

  __device__ __forceinline__ void aa_form(AAState &a) {
    const int cap = uni(I.st.anderson_mem) + 2;
    int slot = 0;
    for (; slot < cap; ++slot) {
      bool used = false;
      for (int j = 0; j < a.count; ++j) used = used || (aa_win(j) == slot);
      if (!used) break;
    }
    a.form_slot = slot;
    aa_pack(I.AU + (size_t)slot * (n + m));
  }

  __device__ __forceinline__ void aa_step(AAState &a, double rp, double rd, double tol_p,
                                          double rd_prev, bool moved) {
    const int mem = uni(I.st.anderson_mem);
    const size_t len = (size_t)n + m;
    if (a.last_valid && (rp > a.last_rp || rd > a.last_rd)) a.count = 0;
    a.last_valid = false;
    const bool contracting = rd < rd_prev;
    if (!(rp <= tol_p) || moved || !contracting) {
      a.count = 0;
      return;
    }
    aa_pack(I.AG + (size_t)a.form_slot * len);
    // append the slot, dropping the oldest beyond mem + 1 entries
    if (threadIdx.x == 0) {
      int cnt = a.count;
      sh.aawin[cnt++] = a.form_slot;
      while (cnt > mem + 1) {
        for (int j = 0; j + 1 < cnt; ++j) sh.aawin[j] = sh.aawin[j + 1];
        cnt -= 1;
      }
    }
    __syncthreads();
    a.count = a.count + 1 > mem + 1 ? mem + 1 : a.count + 1;
    if (a.count < 2) return;
    const int p = a.count - 1;
    const gp<const double> U = G((const double *)I.AU), Gh = G((const double *)I.AG);
    const size_t op = (size_t)aa_win(p) * len;
    // Gram of dF_j = f_{j+1} - f_j (f = G - U) and dF'f_p, one row per pass
    for (int i = 0; i < p; ++i) {
      double v[kAAMem + 1];
#pragma unroll
      for (int k = 0; k <= kAAMem; ++k) v[k] = 0.0;
      const size_t oi0 = (size_t)aa_win(i) * len, oi1 = (size_t)aa_win(i + 1) * len;
      size_t oj0[kAAMem], oj1[kAAMem];
#pragma unroll
      for (int j = 0; j < kAAMem; ++j) {
        oj0[j] = j < p ? (size_t)aa_win(j) * len : 0;
        oj1[j] = j < p ? (size_t)aa_win(j + 1) * len : 0;
      }
      elems((int)len, [&](int e) {
        const double di = (Gh[oi1 + e] - U[oi1 + e]) - (Gh[oi0 + e] - U[oi0 + e]);
#pragma unroll
        for (int j = 0; j < kAAMem; ++j) {
          if (j >= i && j < p) {
            const double dj = (Gh[oj1[j] + e] - U[oj1[j] + e]) - (Gh[oj0[j] + e] - U[oj0[j] + e]);
            v[j] += di * dj;
          }
        }
        v[kAAMem] += di * (Gh[op + e] - U[op + e]);
      });
      allreduce<kAAMem + 1>(v, 0u);
      if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < kAAMem; ++j)
          if (j >= i && j < p) sh.aam[i][j] = sh.aam[j][i] = v[j];
        sh.aam[i][kAAMem] = v[kAAMem];
      }
    }
    __syncthreads();
    // thread 0 solves (partial pivoting; gamma = 0 if singular) and broadcasts
    if (threadIdx.x == 0) {
      double(*M)[kAAMem + 1] = sh.aam;
      double tr = 0.0;
      for (int i = 0; i < p; ++i) tr += M[i][i];
      const double tik = I.st.anderson_reg * tr / p;
      for (int i = 0; i < p; ++i) M[i][i] += tik;
      bool singular = false;
      for (int cc = 0; cc < p && !singular; ++cc) {
        int piv = cc;
        for (int i = cc + 1; i < p; ++i)
          if (fabs(M[i][cc]) > fabs(M[piv][cc])) piv = i;
        if (M[piv][cc] == 0.0) {
          singular = true;
          break;
        }
        if (piv != cc) {
          for (int j = 0; j < p; ++j) {
            const double t = M[cc][j];
            M[cc][j] = M[piv][j];
            M[piv][j] = t;
          }
          const double t = M[cc][kAAMem];
          M[cc][kAAMem] = M[piv][kAAMem];
          M[piv][kAAMem] = t;
        }
        for (int i = cc + 1; i < p; ++i) {
          const double f = M[i][cc] / M[cc][cc];
          for (int j = cc; j < p; ++j) M[i][j] -= f * M[cc][j];
          M[i][kAAMem] -= f * M[cc][kAAMem];
        }
      }
      for (int i = 0; i < kAAMem; ++i) sh.res[i] = 0.0;
      if (!singular) {
        for (int i = p - 1; i >= 0; --i) {
          double acc = M[i][kAAMem];
          for (int j = i + 1; j < p; ++j) acc -= M[i][j] * sh.res[j];
          sh.res[i] = acc / M[i][i];
        }
      }
    }
    __syncthreads();
    double gam[kAAMem];
    size_t og[kAAMem + 1];
#pragma unroll
    for (int i = 0; i < kAAMem; ++i) gam[i] = uni(sh.res[i]);
#pragma unroll
    for (int j = 0; j <= kAAMem; ++j) og[j] = j <= p ? (size_t)aa_win(j) * len : 0;
    __syncthreads();
    // combination and projections; inner dual start y = -lambda
    {
      const gp<double> lam = G(I.v.lam), z = G(I.v.z), Y = G(I.v.Y[c.cur]);
      const gp<const double> lo = G(I.lo), hi = G(I.hi);
      elems((int)len, [&](int e) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < kAAMem; ++j)
          if (j < p) acc += gam[j] * (Gh[og[j + 1] + e] - Gh[og[j] + e]);
        const double v = Gh[og[p] + e] - acc;
        if (e < m) {
          const double l = (e >= me && v > 0.0) ? 0.0 : v;
          lam[e] = l;
          Y[e] = -l;
        } else {
          z[e - m] = clampv<double>(v, lo[e - m], hi[e - m]);
        }
      });
    }
    __syncthreads();
    a.last_valid = true;
    a.last_rp = rp;
    a.last_rd = rd;
    a.steps += 1;
  }

  // ---- the whole method ------------------------------------------------------
  __device__ __forceinline__ void solve(uint64_t t_begin) {
    const uint64_t limit = uni((uint64_t)I.limit_ticks);
    const uint64_t deadline = limit > ~0ull - t_begin ? ~0ull : t_begin + limit;
    c = CtrlR{};
    c.state = ST_RUNNING;
    c.omega = I.st.omega0;
    c.step_scale = 1.0;
    c.kkt_prev = INFINITY;
    mode_init = 0;
    double c_obj = 1.0, gamma = 0.0, lam_hat = 0.0, bE = 0.0, bI = 0.0, cn = 0.0;
    setup(c_obj, gamma, lam_hat, bE, bI, cn);
    const uint64_t t_setup = clock_now();
    gamma_inv = 1.0 / gamma;
    h_norm = bE;
    const double eps_abs = I.eps_abs, eps_rel = I.eps_rel;
    // internal tolerances, halved by the calibration of the external test
    double ea = eps_abs, er = eps_rel;
    int32_t halvings = 0;
    const int32_t max_halvings = uni(I.st.external_halvings);
    double eps_ak = 1.0, eps_rk = 1.0;
    delta_a = I.st.delta0;
    delta_r = I.st.delta0;
    bool have_prev = false, need_form = true;
    int status = PDNQP_MAX_ITER;
    int64_t k = 0;
    const int64_t max_outer = I.st.max_outer;
    double rp = NAN, rd = NAN, sp = NAN, sd = NAN;
    const bool aa_on = uni(I.st.anderson_mem) > 0;
    AAState aa;
    aa.count = 0;
    aa.form_slot = 0;
    aa.last_valid = false;
    aa.last_rp = aa.last_rd = 0.0;
    aa.steps = 0;
    double rd_prev = NAN;
    while (k < max_outer) {
      if (need_form) {
        if (aa_on) aa_form(aa);
        form_inner(gamma);
      }
      const int ist = run_inner(deadline);
      if constexpr (F32) {
        const int cur = c.cur;
        const gp<double> X = G(I.v.X[cur]), Y = G(I.v.Y[cur]);
        const gp<const float> X32 = G(I.w32.X[cur]), Y32 = G(I.w32.Y[cur]);
        elems(n, [&](int i) { X[i] = (double)X32[i]; });
        elems(m, [&](int j) { Y[j] = (double)Y32[j]; });
        __syncthreads();
      }
      k += 1;
      if (ist == ST_NUMERR) {
        status = PDNQP_NUMERICAL_ERROR;
        break;
      }
      if (ist == ST_RUNNING) {
        status = PDNQP_TIME_LIMIT;
        break;
      }
      if (ist == ST_PASS_LIMIT) {
        status = PDNQP_MAX_ITER;
        break;
      }
      if (ist == ST_ITER_LIMIT) {
        need_form = false;
        c.state = ST_RUNNING;
        c.t_call = 0;
        if (clock_now() > deadline) {
          status = PDNQP_TIME_LIMIT;
          break;
        }
        continue;
      }
      double o[12];
      outer_update(o, c_obj);
      rp = m ? o[0] : 0.0;
      sp = fmax(fmax(fmax(1.0, m ? o[1] : 0.0), fmax(bE, m ? o[2] : 0.0)), bI);
      rd = o[4];
      sd = fmax(fmax(1.0, o[5]), fmax(cn, o[6]));
      const double dxz = o[7];
      const double rn = m ? o[3] : 0.0;
      if (rp <= ea + er * sp && rd <= ea + er * sd) {
        // external test on the caller's data; on failure the internal
        // tolerances are halved and the iteration continues
        const double rpu = m ? o[8] : 0.0, spu = fmax(1.0, m ? o[9] : 0.0);
        const double rdu = o[10], sdu = fmax(1.0, o[11]);
        if (max_halvings == 0 ||
            (rpu <= eps_abs + eps_rel * spu && rdu <= eps_abs + eps_rel * sdu)) {
          status = PDNQP_SOLVED;
          break;
        }
        if (halvings >= max_halvings) {
          status = PDNQP_INACCURATE;
          break;
        }
        halvings += 1;
        ea *= 0.5;
        er *= 0.5;
      }
      const bool moved = penalties(have_prev, rn, ea + er * sp);
      have_prev = true;
      // inner tolerances (inner-tolerance-factor)
      const double ratio = (rd == 0.0) ? 1.0 : fmin(1.0, dxz / gamma / rd);
      const double rho = I.st.rho_in_max - (I.st.rho_in_max - I.st.rho_in_min) * ratio;
      delta_a = fmax(I.st.delta_floor * ea, rho * delta_a);
      delta_r = fmax(I.st.delta_floor * er, rho * delta_r);
      // proximal centre (center-update)
      if (rp <= eps_ak + eps_rk * sp) {
        const gp<double> z = G(I.v.z);
        const gp<const double> x = G(I.v.X[c.cur]);
        elems(n, [&](int i) { z[i] = x[i]; });
        eps_ak *= I.st.rho_z;
        eps_rk *= I.st.rho_z;
        if (I.st.center_floor) {
          eps_ak = fmax(eps_ak, ea);
          eps_rk = fmax(eps_rk, er);
        }
      }
      __syncthreads();
      if (aa_on) aa_step(aa, rp, rd, ea + er * sp, rd_prev, moved);
      rd_prev = rd;
      need_form = true;
      if (clock_now() > deadline) {
        status = PDNQP_TIME_LIMIT;
        break;
      }
    }
    // unscale: x = Dx x_bar, lambda = Dc lambda_bar (divided by c_obj on the host)
    const int cur = c.cur;
    {
      const gp<double> tn = G(I.v.tmp_n), tm = G(I.v.tmp_m);
      const gp<const double> Dx = G(I.v.Dx), Dc = G(I.v.Dc), X = G(I.v.X[cur]),
                             lam = G(I.v.lam);
      elems(n, [&](int i) { tn[i] = Dx[i] * X[i]; });
      elems(m, [&](int j) { tm[j] = Dc[j] * lam[j]; });
    }
    __syncthreads();
    const uint64_t t_end = clock_now();
    if (threadIdx.x == 0) {
      BatchOut *op = I.out;
      gp<BatchOut> o = G(op);
      o->status = status;
      o->cur = cur;
      o->trace_iters_n = c.trace_iters_n;
      o->trace_trials_n = c.trace_trials_n;
      o->trace_checks_n = c.trace_checks_n;
      o->staged = STAGE ? 1 : 0;
      o->anderson_steps = aa_on ? aa.steps : 0;
      o->outer_iters = k;
      o->halvings = halvings;
      o->trials = c.trials;
      o->accepted = c.accepted;
      o->rejected = c.rejected;
      o->restarts = c.restarts;
      o->checks = c.checks;
      o->rp = rp;
      o->rd = rd;
      o->sp = sp;
      o->sd = sd;
      o->gamma = gamma;
      o->lam_hat = lam_hat;
      o->omega = c.omega;
      o->c_obj = c_obj;
      o->t_begin = t_begin;
      o->t_setup = t_setup;
      o->t_end = t_end;
    }
    __syncthreads();
  }
};

template <typename T, int BT, int WAVES>
__global__ __launch_bounds__(BT, WAVES) void k_batch(const BatchInst *__restrict__ insts,
                                              const int32_t *__restrict__ order, int count,
                                              uint32_t *__restrict__ queue, int lds_bytes) {
  extern __shared__ double bsmem[];
  __shared__ BShared sh;
  for (;;) {
    if (threadIdx.x == 0) {
      sh.inst = (int32_t)atomicAdd(queue, 1u);
      sh.clock = wall_clock64();
    }
    __syncthreads();
    const int idx = uni((int)sh.inst);
    const uint64_t t0 = uni(sh.clock);
    __syncthreads();
    if (idx >= count) return;
    const BatchInst &inst = *(const BatchInst *)(G(insts) + uni(G(order)[idx]));
    const size_t need = batch_lds_bytes(BT, inst.n, inst.m, std::is_same<T, float>::value
                                                                ? PDNQP_FP32
                                                                : PDNQP_FP64);
    if (need <= (size_t)lds_bytes) {
      BSolver<T, BT, true> s(inst, sh, (lp<double>)bsmem);
      s.solve(t0);
    } else {
      BSolver<T, BT, false> s(inst, sh, (lp<double>)bsmem);
      s.solve(t0);
    }
  }
}

}  // namespace

// Configurations: workgroup size, and the minimum waves per SIMD the
// compiler must allow (1: its own register budget; 4: at most 128 VGPRs).
#define PDNQP_BATCH_CONFIGS(X, TT) \
  X(TT, 256, 1, 0)                 \
  X(TT, 512, 1, 1)                 \
  X(TT, 1024, 1, 2)                \
  X(TT, 256, 4, 3)                 \
  X(TT, 512, 4, 4)

int batch_launch(hipStream_t st, int precision, int config, int grid, size_t lds_bytes,
                 const BatchInst *insts, const int32_t *order, int count, uint32_t *queue) {
  if (grid < 1 || count < 1) return PDNQP_OK;
  const int lb = (int)lds_bytes;
  bool found = false;
#define PDNQP_BATCH_CASE(TT, BB, WW, ID)                                                       \
  if (config == ID) {                                                                          \
    hipLaunchKernelGGL((k_batch<TT, BB, WW>), dim3(grid), dim3(BB), lds_bytes, st, insts, order, \
                       count, queue, lb);                                                      \
    found = true;                                                                              \
  }
  if (precision == PDNQP_FP32) {
    PDNQP_BATCH_CONFIGS(PDNQP_BATCH_CASE, float)
  } else {
    PDNQP_BATCH_CONFIGS(PDNQP_BATCH_CASE, double)
  }
#undef PDNQP_BATCH_CASE
  if (!found) return PDNQP_E_INVALID;
  return hipGetLastError() == hipSuccess ? PDNQP_OK : PDNQP_E_DEVICE;
}

int batch_occupancy(int precision, int config, size_t lds_bytes) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define PDNQP_BATCH_OCC(TT, BB, WW, ID) \
  if (config == ID) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<TT, BB, WW>, BB, lds_bytes);
  if (precision == PDNQP_FP32) {
    PDNQP_BATCH_CONFIGS(PDNQP_BATCH_OCC, float)
  } else {
    PDNQP_BATCH_CONFIGS(PDNQP_BATCH_OCC, double)
  }
#undef PDNQP_BATCH_OCC
  return e == hipSuccess ? nb : 0;
}

}  // namespace pdnqp
