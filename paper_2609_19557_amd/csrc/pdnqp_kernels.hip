// gfx950 FP64 kernels of the PDNQP set-up, inner-QP formation and outer
// update (the inner iteration itself is in pdnqp_iter.hip).
//
// These run once per solve or once per outer step.  Sparse products use the
// row-group form: G consecutive lanes per row (G a power of two chosen from
// the mean row length) read the row's values and column indices with unit
// stride and combine with in-group shuffles.  Nothing here is a dense
// contraction, so no matrix-core instructions are used.
#include "pdnqp_device.hpp"

#include <algorithm>
#include <cmath>

namespace pdnqp {

using namespace dev;

namespace {

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
        const double s = maxv<double>(ax + v.lam[j] / v.sigma[j], v.b[j]);
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
// Multiplier update (practical-multiplier-update) and the row part of the
// outer residuals (outer-residuals)/(outer-scales), on the scaled data and,
// for the external test of the experimental protocol, on the caller's data:
// row j of the unscaled problem reads (A x)_j = (bar A bar x)_j / D_c,j
// against the raw right-hand side.  outv[0..3]: scaled r_p part, |A_E x|,
// |A_I x|, |r_row|; outv[8]: unscaled r_p part; outv[9]: max of |A x| and
// |b| unscaled.
template <int GA>
__global__ __launch_bounds__(kBlock) void k_outer_rows(Ctrl *__restrict__ c, InnerParams p,
                                                       Vecs v, Csr A, Part pa, RawData raw) {
  const int cur = c->cur;
  double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for_rows<GA>(A.rows, blockIdx.x, gridDim.x, [&](int j, int lane) {
    const double ax = row_dot<GA, double>(A.p, A.i, A.v, v.X[cur], j, lane);
    if (lane == 0) {
      v.ax[j] = ax;
      const double bj = v.b[j];
      const double sg = v.sigma[j];
      const double lm = v.lam[j];
      const double axr = ax / v.Dc[j];
      const double br = raw.b[j];
      double rr;
      if (j < p.me) {
        const double res = ax - bj;
        v.lam[j] = lm + sg * res;
        rr = res;
        a[0] = fmax(a[0], fabs(res));
        a[1] = fmax(a[1], fabs(ax));
        a[4] = fmax(a[4], fabs(axr - br));
      } else {
        const double s = maxv<double>(ax + lm / sg, bj);
        const double ln = lm + sg * (ax - bj);
        v.lam[j] = ln < 0.0 ? ln : 0.0;
        rr = ax - s;
        a[0] = fmax(a[0], maxv<double>(bj - ax, 0.0));
        a[2] = fmax(a[2], fabs(ax));
        a[4] = fmax(a[4], maxv<double>(br - axr, 0.0));
      }
      v.rrow[j] = rr;
      a[3] = fmax(a[3], fabs(rr));
      a[5] = fmax(a[5], fmax(fabs(axr), fabs(br)));
    }
  });
  block_reduce<6>(a, 0x3Fu, v.partial, blockIdx.x);
  if (last_block(&c->ticket[TK_OUTER_ROWS], gridDim.x)) {
    double r[6];
    final_reduce<6>(v.partial, gridDim.x, 0x3Fu, r);
    if (threadIdx.x == 0) {
      for (int k = 0; k < 4; ++k) c->outv[k] = r[k];
      c->outv[8] = r[4];
      c->outv[9] = r[5];
      c->ticket[TK_OUTER_ROWS] = 0;
    }
  }
}

// Column part of the outer residuals: projected stationarity and its scale
// on the scaled data (outv[4..7]: r_d, |Q x|, |A' lambda|, |x - z|) and on
// the caller's data (outv[10]: unscaled r_d; outv[11]: max of |Q x|, |c|,
// |A' lambda| unscaled), with x = D_x bar x clipped into the caller's box,
// Q x = (bar Q bar x) / (c_obj D_x), A' lambda = (bar A' bar lambda) /
// (c_obj D_x).
template <int GQ, int GT>
__global__ __launch_bounds__(kBlock) void k_outer_cols(Ctrl *__restrict__ c, InnerParams p,
                                                       Vecs v, Csr Q, Csr AT, Part pq,
                                                       RawData raw) {
  const int cur = c->cur;
  double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for_rows<GQ>(Q.rows, blockIdx.x, gridDim.x, [&](int i, int lane) {
    const double qx = row_dot<GQ, double>(Q.p, Q.i, Q.v, v.X[cur], i, lane);
    const double atl = row_dot<GT, double>(AT.p, AT.i, AT.v, v.lam, i, lane);
    if (lane == 0) {
      const double x = v.X[cur][i];
      const double pr = clampv<double>(x - qx - v.c[i] - atl, v.lo[i], v.hi[i]);
      a[0] = fmax(a[0], fabs(x - pr));
      a[1] = fmax(a[1], fabs(qx));
      a[2] = fmax(a[2], fabs(atl));
      a[3] = fmax(a[3], fabs(x - v.z[i]));
      v.qxo[i] = qx;
      v.atl[i] = atl;
      const double dx = v.Dx[i];
      const double sc = 1.0 / (raw.c_obj * dx);
      const double xl = raw.xl[i], xu = raw.xu[i];
      const double xr = clampv<double>(dx * x, xl, xu);
      const double qr = qx * sc, ar = atl * sc, cr = raw.c[i];
      const double prr = clampv<double>(xr - qr - cr - ar, xl, xu);
      a[4] = fmax(a[4], fabs(xr - prr));
      a[5] = fmax(a[5], fmax(fmax(fabs(qr), fabs(cr)), fabs(ar)));
    }
  });
  block_reduce<6>(a, 0x3Fu, v.partial, blockIdx.x);
  if (last_block(&c->ticket[TK_OUTER_COLS], gridDim.x)) {
    double r[6];
    final_reduce<6>(v.partial, gridDim.x, 0x3Fu, r);
    if (threadIdx.x == 0) {
      for (int k = 0; k < 4; ++k) c->outv[4 + k] = r[k];
      c->outv[10] = r[4];
      c->outv[11] = r[5];
      c->ticket[TK_OUTER_COLS] = 0;
    }
  }
}

// Row-wise penalty update (eq. (penalty-trigger-eq)): a row is raised when
// its residual did not fall below theta times the previous one (equality
// rows, and inequality rows with lambda < 0), by the factor
// max(1, growth |r_i| / ||r||_inf), capped.
__global__ __launch_bounds__(kBlock) void k_penalty(Ctrl *__restrict__ c, InnerParams p, Vecs v,
                                                    int have_prev, double rnorm, double theta,
                                                    double growth, double sig_max, int gate,
                                                    double gate_tol) {
  int moved = 0;
  for_elems(p.m, blockIdx.x, gridDim.x, [&](int j) {
    const double r = v.rrow[j];
    if (have_prev && rnorm > 0.0) {
      const bool active = (j < p.me) || (v.lam[j] < 0.0);
      bool trig = fabs(r) > theta * fabs(v.rprev[j]) && active;
      if (gate) trig = trig && (fabs(r) > gate_tol);
      if (trig) {
        const double fac = fmax(1.0, growth * fabs(r) / rnorm);
        const double so = v.sigma[j];
        const double sn = so * fac;
        const double s2 = sn < sig_max ? sn : sig_max;
        v.sigma[j] = s2;
        moved |= (s2 != so);
      }
    }
    v.rprev[j] = r;
  });
  if (moved) atomicOr(&c->pen_moved, 1);
}

// min (as 1 / max 1/sigma), sum and max of the row penalties into gen[5],
// gen[6], gen[7]
__global__ __launch_bounds__(kBlock) void k_sigma_stats(Ctrl *c, const double *sig, int32_t m,
                                                        double *partial) {
  double a[3] = {0.0, 0.0, 0.0};  // max(1 / sigma), sum, max(sigma); sigma > 0
  for_elems(m, blockIdx.x, gridDim.x, [&](int j) {
    const double s = sig[j];
    a[0] = fmax(a[0], 1.0 / s);
    a[1] += s;
    a[2] = fmax(a[2], s);
  });
  block_reduce<3>(a, 0x5u, partial, blockIdx.x);
  if (last_block(&c->ticket[TK_GEN], gridDim.x)) {
    double r[3];
    final_reduce<3>(partial, gridDim.x, 0x5u, r);
    if (threadIdx.x == 0) {
      c->gen[5] = 1.0 / r[0];
      c->gen[6] = r[1];
      c->gen[7] = r[2];
      c->ticket[TK_GEN] = 0;
    }
  }
}

// ===========================================================================
// Anderson acceleration of the outer duals and the centre (Section 3.2,
// "Anderson acceleration"): Type-II mixing over the stored points.
// ===========================================================================
__global__ __launch_bounds__(kBlock) void k_aa_pack(double *dst, const double *lam,
                                                    const double *z, int32_t m, int32_t n) {
  for_elems(m + n, blockIdx.x, gridDim.x, [&](int i) { dst[i] = i < m ? lam[i] : z[i - m]; });
}

// Gram matrix dF'dF (upper triangle, row by row) and dF'f_p of the residual
// differences dF_j = f_{j+1} - f_j, f_j = G_j - U_j, over the points
// slot[0..p]; per-block partials, fixed-order combination by the last block.
__global__ __launch_bounds__(kBlock) void k_aa_gram(Ctrl *__restrict__ c, const double *U,
                                                    const double *G, int64_t len, AASlots sl,
                                                    int p, double *partial) {
  double a[kAASums];
#pragma unroll
  for (int k = 0; k < kAASums; ++k) a[k] = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * kBlock) {
    double f[kAAMem + 1];
#pragma unroll
    for (int j = 0; j <= kAAMem; ++j) {
      f[j] = 0.0;
      if (j <= p) {
        const int64_t off = (int64_t)sl.s[j] * len + e;
        f[j] = G[off] - U[off];
      }
    }
    double d[kAAMem];
#pragma unroll
    for (int j = 0; j < kAAMem; ++j) d[j] = (j < p) ? f[j + 1] - f[j] : 0.0;
    int k = 0;
#pragma unroll
    for (int i = 0; i < kAAMem; ++i) {
#pragma unroll
      for (int j = i; j < kAAMem; ++j) a[k++] += d[i] * d[j];
    }
    double fp = 0.0;
#pragma unroll
    for (int j = 0; j <= kAAMem; ++j)
      if (j == p) fp = f[j];
#pragma unroll
    for (int i = 0; i < kAAMem; ++i) a[k++] += d[i] * fp;
  }
  block_reduce<kAASums>(a, 0u, partial, blockIdx.x);
  if (last_block(&c->ticket[TK_AA], gridDim.x)) {
    double r[kAASums];
    final_reduce<kAASums>(partial, gridDim.x, 0u, r);
    if (threadIdx.x == 0) {
      for (int k = 0; k < kAASums; ++k) c->aa[k] = r[k];
      c->ticket[TK_AA] = 0;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_aa_combine(const double *G, int64_t len, AASlots sl,
                                                       int p, double *lam, double *z,
                                                       const double *lo, const double *hi,
                                                       int32_t me, int32_t m, int32_t n) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * kBlock) {
    double acc = 0.0;
    for (int j = 0; j < p; ++j)
      acc += sl.gamma[j] * (G[(int64_t)sl.s[j + 1] * len + e] - G[(int64_t)sl.s[j] * len + e]);
    const double v = G[(int64_t)sl.s[p] * len + e] - acc;
    if (e < m) {
      lam[e] = (e >= me && v > 0.0) ? 0.0 : v;
    } else {
      const int i = (int)(e - m);
      z[i] = clampv<double>(v, lo[i], hi[i]);
    }
  }
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
    const double s = row_dot<G, double>(M.p, M.i, M.v, x, r, lane);
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
    out[j] = (j < p.me) ? ax - v.b[j] : ax - maxv<double>(ax, v.b[j]);
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

void stream_row_blocks(const int32_t *rp, int32_t rows, int32_t max_rows, int32_t *out_nrb,
                       int32_t *rb, int32_t tile) {
  int32_t nb = 0;
  rb[0] = 0;
  int32_t r = 0;
  while (r < rows) {
    const int32_t start = r;
    const int32_t base = rp[r];
    ++r;
    while (r < rows && rp[r + 1] - base <= tile && r - start < max_rows) ++r;
    rb[++nb] = r;
  }
  *out_nrb = nb;
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
                       const Csr &A, const Part &pa, const RawData &raw) {
  PDNQP_DISPATCH_G(A.G, {
    hipLaunchKernelGGL((k_outer_rows<GV>), dim3(nz(pa.blocks)), dim3(kBlock), 0, st, c, p, v, A,
                       pa, raw);
  });
}

void launch_outer_cols(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v,
                       const Csr &Q, const Csr &AT, const Part &pq, const RawData &raw) {
  const int G = Q.G > AT.G ? Q.G : AT.G;
  Part pqq = make_part(Q.rows, G, 1024);
  PDNQP_DISPATCH_G(G, {
    hipLaunchKernelGGL((k_outer_cols<GV, GV>), dim3(nz(pqq.blocks)), dim3(kBlock), 0, st, c, p, v,
                       Q, AT, pqq, raw);
  });
  (void)pq;
}

void launch_penalty(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v,
                    const Part &pr, int have_prev, double rnorm, double theta, double growth,
                    double sig_max, int gate, double gate_tol) {
  if (p.m == 0) return;
  hipLaunchKernelGGL(k_penalty, dim3(nz(pr.blocks)), dim3(kBlock), 0, st, c, p, v, have_prev,
                     rnorm, theta, growth, sig_max, gate, gate_tol);
}

void launch_sigma_stats(hipStream_t st, Ctrl *c, const double *sig, int32_t m, double *partial) {
  const int blocks = (int)std::min<int64_t>(((int64_t)m + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_sigma_stats, dim3(nz(blocks)), dim3(kBlock), 0, st, c, sig, m, partial);
}

void launch_aa_pack(hipStream_t st, double *dst, const double *lam, const double *z, int32_t m,
                    int32_t n) {
  const int blocks = (int)std::min<int64_t>(((int64_t)m + n + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_aa_pack, dim3(nz(blocks)), dim3(kBlock), 0, st, dst, lam, z, m, n);
}

void launch_aa_gram(hipStream_t st, Ctrl *c, const double *U, const double *G, int64_t len,
                    const AASlots &sl, int p, double *partial) {
  const int blocks = (int)std::min<int64_t>((len + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_aa_gram, dim3(nz(blocks)), dim3(kBlock), 0, st, c, U, G, len, sl, p,
                     partial);
}

void launch_aa_combine(hipStream_t st, const double *G, int64_t len, const AASlots &sl, int p,
                       double *lam, double *z, const double *lo, const double *hi, int32_t me,
                       int32_t m, int32_t n) {
  const int blocks = (int)std::min<int64_t>((len + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_aa_combine, dim3(nz(blocks)), dim3(kBlock), 0, st, G, len, sl, p, lam, z,
                     lo, hi, me, m, n);
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
