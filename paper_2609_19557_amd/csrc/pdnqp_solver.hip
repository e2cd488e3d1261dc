// Host driver of the gfx950 PDNQP solver (see pdnqp_solver.hpp).
//
// Per outer step (Algorithm "practical outer iteration"): form the inner QP
// on the device (warm start, penalty + inner Ruiz scaling folded into the
// step vectors, diagonal steps), run the inner PDHG in chunks of trial
// slots whose accept/reject/restart decisions are taken on the device, read
// back the control block once per chunk, then update multipliers, residuals,
// penalties, tolerances and the proximal centre.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <limits>

#include "pdnqp_solver.hpp"

namespace pdnqp {

namespace {

double now_s() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

int pick_G(int64_t nnz, int32_t rows) {
  const double avg = rows > 0 ? (double)nnz / rows : 1.0;
  int G = 2;
  while (G < avg && G < 32) G *= 2;
  return G;
}

// Smallest eigenvalue of the symmetric tridiagonal matrix (a, b) by
// bisection on Sturm-sequence counts (Gershgorin starting interval).
double tridiag_min_eig(const std::vector<double> &a, const std::vector<double> &b) {
  const int k = (int)a.size();
  double lo = std::numeric_limits<double>::infinity(), hi = -lo, bmax2 = 0.0;
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < k - 1 ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
    if (i < k - 1) bmax2 = std::max(bmax2, b[i] * b[i]);
  }
  const double pivmin = std::numeric_limits<double>::min() * std::max(1.0, bmax2);
  auto count_below = [&](double x) {
    int cnt = 0;
    double d = a[0] - x;
    if (std::fabs(d) < pivmin) d = -pivmin;
    if (d < 0) ++cnt;
    for (int i = 1; i < k; ++i) {
      d = a[i] - x - b[i - 1] * b[i - 1] / d;
      if (std::fabs(d) < pivmin) d = -pivmin;
      if (d < 0) ++cnt;
    }
    return cnt;
  };
  const double eps = std::numeric_limits<double>::epsilon();
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (hi - lo <= 2.0 * eps * std::max(std::fabs(lo), std::fabs(hi)) + pivmin) break;
    if (mid <= lo || mid >= hi) break;
    if (count_below(mid) >= 1) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

double ninf(const std::vector<double> &v) {
  double m = 0.0;
  for (double x : v) m = std::max(m, std::fabs(x));
  return m;
}

enum TimerId { TM_XTRIAL = 0, TM_QA = 1, TM_AT = 2, TM_DECIDE = 3, TM_QA_ROWS = 4, TM_COUNT = 5 };

// The columns of a CSR split at `mid` into two CSRs over all rows: panel 0
// holds the entries with column < mid, panel 1 the others, each in the
// original order within a row; perm[h][k] is the original position of entry
// k of panel h.
struct ColumnSplit {
  std::vector<int32_t> p[2], i[2], perm[2];
};

ColumnSplit split_columns(const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                          int32_t rows, int32_t mid) {
  ColumnSplit s;
  for (int h = 0; h < 2; ++h) s.p[h].assign((size_t)rows + 1, 0);
  for (int32_t r = 0; r < rows; ++r) {
    for (int32_t k = rp[r]; k < rp[r + 1]; ++k) {
      const int h = ci[k] < mid ? 0 : 1;
      s.i[h].push_back(ci[k]);
      s.perm[h].push_back(k);
    }
    for (int h = 0; h < 2; ++h) s.p[h][(size_t)r + 1] = (int32_t)s.i[h].size();
  }
  return s;
}

}  // namespace

Solver::~Solver() {
  if (stream_) hipStreamSynchronize(stream_);
  if (gexec_) hipGraphExecDestroy(gexec_);
  if (cap_stream_) hipStreamDestroy(cap_stream_);
  for (auto &t : timers_)
    for (auto e : t.ev) hipEventDestroy(e);
  for (void *p : allocs_) dfree(p);
  if (hctrl_) hipHostFree(hctrl_);
  if (own_stream_ && stream_) hipStreamDestroy(stream_);
}

void *Solver::dalloc(size_t bytes) {
  if (bytes == 0) bytes = 8;
  bytes = (bytes + 255) & ~size_t(255);
  void *p = nullptr;
  if (st_.dev_alloc) {
    p = st_.dev_alloc(bytes, st_.alloc_user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) allocs_.push_back(p);
  return p;
}

void Solver::dfree(void *p) {
  if (!p) return;
  if (st_.dev_free) st_.dev_free(p, st_.alloc_user);
  else hipFree(p);
}

int Solver::check(hipError_t e, const char *what, std::string &err) {
  if (e == hipSuccess) return PDNQP_OK;
  err = std::string(what) + ": " + hipGetErrorString(e);
  return PDNQP_E_DEVICE;
}

int Solver::init(HostQP &&qp, const pdnqp_settings &st, std::string &err) {
  qp_ = std::move(qp);
  st_ = st;
  hipGetDevice(&device_);
  const int32_t n = qp_.n, m = qp_.m, mi = qp_.mi;
  const int64_t nzq = qp_.Qi.size(), nza = qp_.Ai.size();
  if (st_.hip_stream) {
    stream_ = (hipStream_t)st_.hip_stream;
  } else {
    int r = check(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking), "hipStreamCreate", err);
    if (r) return r;
    own_stream_ = true;
  }
  int r = check(hipHostMalloc((void **)&hctrl_, sizeof(Ctrl), hipHostMallocDefault),
                "hipHostMalloc", err);
  if (r) return r;
  std::memset(hctrl_, 0, sizeof(Ctrl));

  bool ok = true;
  auto D = [&](size_t count) -> double * {
    double *p = (double *)dalloc(count * sizeof(double));
    ok = ok && p;
    return p;
  };
  auto I = [&](size_t count) -> int32_t * {
    int32_t *p = (int32_t *)dalloc(count * sizeof(int32_t));
    ok = ok && p;
    return p;
  };
  ctrl_ = (Ctrl *)dalloc(sizeof(Ctrl));
  ok = ok && ctrl_;
  Qp_ = I(n + 1); Qi_ = I(nzq); Qraw_ = D(nzq); Qv_ = D(nzq);
  Ap_ = I(m + 1); Ai_ = I(nza); Araw_ = D(nza); Av_ = D(nza);
  ATp_ = I(n + 1); ATi_ = I(nza); ATraw_ = D(nza); ATv_ = D(nza);
  atperm_ = I(nza);
  // off-diagonal part of Q for the hot product, diagonal kept as a vector
  {
    qp_.Qop.assign(n + 1, 0);
    qp_.Qdiag.assign(n, 0.0);
    for (int32_t i = 0; i < n; ++i) {
      for (int32_t k = qp_.Qp[i]; k < qp_.Qp[i + 1]; ++k) {
        if (qp_.Qi[k] == i) {
          qp_.Qdiag[i] = qp_.Qx[k];
        } else {
          qp_.Qoi.push_back(qp_.Qi[k]);
          qp_.Qox.push_back(qp_.Qx[k]);
        }
      }
      qp_.Qop[i + 1] = (int32_t)qp_.Qoi.size();
    }
  }
  const int64_t nzo = qp_.Qoi.size();
  Qop_ = I(n + 1); Qoi_ = I(nzo); Qoraw_ = D(nzo); Qov_ = D(nzo);
  qdiag_raw_ = D(n); qdiag_ = D(n);
  craw_ = D(n); xlraw_ = D(n); xuraw_ = D(n); braw_ = D(m);
  c_ = D(n); lo_ = D(n); hi_ = D(n); b_ = D(m);
  v_.c = c_; v_.lo = lo_; v_.hi = hi_; v_.b = b_;
  v_.sigma = D(m); v_.lam = D(m); v_.z = D(n); v_.qx = D(n);
  v_.taub_x = D(n); v_.taub_s = D(mi); v_.taub_r = D(m); v_.etab = D(m);
  v_.S2x = D(n); v_.S2s = D(mi); v_.S2r = D(m); v_.E2 = D(m);
  for (int k = 0; k < 2; ++k) {
    v_.X[k] = D(n); v_.QX[k] = D(n); v_.ATY[k] = D(n);
    v_.S[k] = D(mi); v_.R[k] = D(m); v_.Y[k] = D(m); v_.BW[k] = D(m);
  }
  v_.xbar = D(n); v_.qxbar = D(n); v_.sbar = D(mi); v_.rbar = D(m); v_.ybar = D(m);
  v_.xa = D(n); v_.sa = D(mi); v_.ra = D(m); v_.ya = D(m);
  v_.axbar = D(m); v_.atybar = D(n);
  v_.ax = D(m); v_.rrow = D(m); v_.rprev = D(m); v_.atl = D(n); v_.qxo = D(n);
  v_.Dx = D(n); v_.Dc = D(m); v_.Ex = nullptr;
  v_.Fx = D(n); v_.Fs = D(mi); v_.Fr = D(m); v_.tmp_n = D(n); v_.tmp_m = D(m);
  Fx2_ = D(n); Fs2_ = D(mi); Fr2_ = D(m); E2buf_ = D(m);
  v_.partial = D((size_t)kMaxParts * 48);
  if (st_.anderson_mem > 0) {
    const size_t len = (size_t)n + m;
    AU_ = D((size_t)(st_.anderson_mem + 2) * len);
    AG_ = D((size_t)(st_.anderson_mem + 2) * len);
  }
  fp32_ = st_.precision == PDNQP_FP32;
  if (fp32_) {
    auto F = [&](size_t count) -> float * {
      float *p = (float *)dalloc(count * sizeof(float));
      ok = ok && p;
      return p;
    };
    IterVecs<float> &w = iv32_;
    float *lo = F(n), *hi = F(n), *b = F(m), *qd = F(n);
    w.lo = lo; w.hi = hi; w.b = b; w.qdiag = qd;
    w.sigma = F(m); w.lam = F(m); w.qx = F(n);
    w.taub_x = F(n); w.taub_s = F(mi); w.taub_r = F(m); w.etab = F(m);
    w.S2x = F(n); w.S2s = F(mi); w.S2r = F(m); w.E2 = F(m);
    for (int k = 0; k < 2; ++k) {
      w.X[k] = F(n); w.QX[k] = F(n); w.ATY[k] = F(n);
      w.S[k] = F(mi); w.R[k] = F(m); w.Y[k] = F(m); w.BW[k] = F(m);
    }
    w.xbar = F(n); w.qxbar = F(n); w.sbar = F(mi); w.rbar = F(m); w.ybar = F(m);
    w.xa = F(n); w.sa = F(mi); w.ra = F(m); w.ya = F(m);
    w.axbar = F(m); w.atybar = F(n);
    Qo32v_ = F(nzo); A32v_ = F(nza); AT32v_ = F(nza);
    w.partial = v_.partial;
  }
  if (!ok) {
    err = "device allocation failed";
    return PDNQP_E_NOMEM;
  }
  auto H2D = [&](void *dst, const void *src, size_t bytes) {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream_);
  };
  hipError_t e = hipSuccess;
  auto chain = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  chain(H2D(Qp_, qp_.Qp.data(), (n + 1) * 4));
  chain(H2D(Qi_, qp_.Qi.data(), nzq * 4));
  chain(H2D(Qraw_, qp_.Qx.data(), nzq * 8));
  chain(H2D(Ap_, qp_.Ap.data(), (m + 1) * 4));
  chain(H2D(Ai_, qp_.Ai.data(), nza * 4));
  chain(H2D(Araw_, qp_.Ax.data(), nza * 8));
  chain(H2D(ATp_, qp_.ATp.data(), (n + 1) * 4));
  chain(H2D(ATi_, qp_.ATi.data(), nza * 4));
  chain(H2D(ATraw_, qp_.ATx.data(), nza * 8));
  chain(H2D(atperm_, qp_.ATperm.data(), nza * 4));
  chain(H2D(Qop_, qp_.Qop.data(), (n + 1) * 4));
  chain(H2D(Qoi_, qp_.Qoi.data(), nzo * 4));
  chain(H2D(Qoraw_, qp_.Qox.data(), nzo * 8));
  chain(H2D(qdiag_raw_, qp_.Qdiag.data(), n * 8));
  chain(H2D(craw_, qp_.c.data(), n * 8));
  chain(H2D(xlraw_, qp_.xl.data(), n * 8));
  chain(H2D(xuraw_, qp_.xu.data(), n * 8));
  chain(H2D(braw_, qp_.b.data(), m * 8));
  chain(hipStreamSynchronize(stream_));
  if ((r = check(e, "upload", err))) return r;

  const int GQ = pick_G(nzq, n), GA = pick_G(nza, m), GT = pick_G(nza, n);
  // CSR-stream row blocks of the three matrices
  // (tile: nonzeros per block; kPipeTile for the matrices the pipelined
  // trial products stream: Q_off, A, A' and the column panels)
  auto blocks_of = [&](const std::vector<int32_t> &rp, int32_t rows, int32_t *&dev,
                       int32_t &nrb, int32_t tile) -> bool {
    // row boundaries of the nrb blocks, then the nonzero offset of each
    std::vector<int32_t> rb(2 * (size_t)rows + 4);
    stream_row_blocks(rp.data(), rows, 4 * kBlock, &nrb, rb.data(), tile);
    for (int32_t b = 0; b <= nrb; ++b) rb[nrb + 1 + b] = rp[rb[b]];
    dev = (int32_t *)dalloc((size_t)(nrb + 1) * 8);
    if (!dev) return false;
    return hipMemcpyAsync(dev, rb.data(), (size_t)(nrb + 1) * 8, hipMemcpyHostToDevice,
                          stream_) == hipSuccess;
  };
  int32_t *qrb = nullptr, *arb = nullptr, *atrb = nullptr, *qorb = nullptr;
  int32_t nq = 0, na = 0, nt = 0, nqo = 0;
  if (!blocks_of(qp_.Qp, n, qrb, nq, kTile) || !blocks_of(qp_.Ap, m, arb, na, kPipeTile) ||
      !blocks_of(qp_.ATp, n, atrb, nt, kPipeTile) ||
      !blocks_of(qp_.Qop, n, qorb, nqo, kPipeTile)) {
    err = "row-block upload failed";
    return PDNQP_E_DEVICE;
  }
  if ((r = check(hipStreamSynchronize(stream_), "row-block upload", err))) return r;
  Q_ = Csr{Qp_, Qi_, Qv_, n, GQ, qrb, nq, 0};
  Qo_ = Csr{Qop_, Qoi_, Qov_, n, pick_G(nzo, n), qorb, nqo, 0};
  Qo32_ = CsrT<float>{Qop_, Qoi_, Qo32v_, n, Qo_.G, qorb, nqo, 0};
  A32_ = CsrT<float>{Ap_, Ai_, A32v_, m, GA, arb, na, 0};
  AT32_ = CsrT<float>{ATp_, ATi_, AT32v_, n, GT, atrb, nt, 0};
  v_.qdiag = qdiag_;
  A_ = Csr{Ap_, Ai_, Av_, m, GA, arb, na, 0};
  AT_ = Csr{ATp_, ATi_, ATv_, n, GT, atrb, nt, 0};
  Qr_ = Csr{Qp_, Qi_, Qraw_, n, GQ, qrb, nq, 0};
  Ar_ = Csr{Ap_, Ai_, Araw_, m, GA, arb, na, 0};
  ATr_ = Csr{ATp_, ATi_, ATraw_, n, GT, atrb, nt, 0};
  // two column panels for the first trial product when the gathered vector
  // x_tr is larger than one XCD's L2 (4 MiB): FP64 from n > 512Ki, FP32 from
  // n > 1Mi (settings.col_panels: 0 that rule, 1 never, 2 always)
  constexpr double kL2Bytes = 4.0 * 1024 * 1024;
  panels64_ = st_.col_panels == 2 || (st_.col_panels == 0 && 8.0 * n > kL2Bytes);
  panels32_ = fp32_ && (st_.col_panels == 2 || (st_.col_panels == 0 && 4.0 * n > kL2Bytes));
  if (panels64_ || panels32_) {
    const int32_t mid = n / 2;
    const ColumnSplit sq = split_columns(qp_.Qop, qp_.Qoi, n, mid);
    const ColumnSplit sa = split_columns(qp_.Ap, qp_.Ai, m, mid);
    for (int h = 0; h < 2; ++h) {
      pnnz_q_[h] = (int64_t)sq.i[h].size();
      pnnz_a_[h] = (int64_t)sa.i[h].size();
      const size_t nq1 = (size_t)std::max<int64_t>(pnnz_q_[h], 1);
      const size_t na1 = (size_t)std::max<int64_t>(pnnz_a_[h], 1);
      int32_t *qp = I(n + 1), *qi = I(nq1), *ap = I(m + 1), *ai = I(na1);
      pperm_q_[h] = I(nq1);
      pperm_a_[h] = I(na1);
      double *qv = D(nq1), *av = D(na1);
      qap64_.pq[h] = D(n);
      qap64_.pa[h] = D(std::max(m, 1));
      if (!ok) {
        err = "device allocation failed";
        return PDNQP_E_NOMEM;
      }
      chain(H2D(qp, sq.p[h].data(), (size_t)(n + 1) * 4));
      chain(H2D(qi, sq.i[h].data(), (size_t)pnnz_q_[h] * 4));
      chain(H2D(pperm_q_[h], sq.perm[h].data(), (size_t)pnnz_q_[h] * 4));
      chain(H2D(ap, sa.p[h].data(), (size_t)(m + 1) * 4));
      chain(H2D(ai, sa.i[h].data(), (size_t)pnnz_a_[h] * 4));
      chain(H2D(pperm_a_[h], sa.perm[h].data(), (size_t)pnnz_a_[h] * 4));
      int32_t *qrbh = nullptr, *arbh = nullptr, nqh = 0, nah = 0;
      if (!blocks_of(sq.p[h], n, qrbh, nqh, kPipeTile) ||
          !blocks_of(sa.p[h], m, arbh, nah, kPipeTile)) {
        err = "row-block upload failed";
        return PDNQP_E_DEVICE;
      }
      qap64_.q[h] = Csr{qp, qi, qv, n, 1, qrbh, nqh, 0};
      qap64_.a[h] = Csr{ap, ai, av, m, 1, arbh, nah, 0};
      if (panels32_) {
        float *qv32 = (float *)dalloc((size_t)std::max<int64_t>(pnnz_q_[h], 1) * 4);
        float *av32 = (float *)dalloc((size_t)std::max<int64_t>(pnnz_a_[h], 1) * 4);
        float *pq32 = (float *)dalloc((size_t)n * 4);
        float *pa32 = (float *)dalloc((size_t)std::max(m, 1) * 4);
        if (!qv32 || !av32 || !pq32 || !pa32) {
          err = "device allocation failed";
          return PDNQP_E_NOMEM;
        }
        qap32_.q[h] = CsrT<float>{qp, qi, qv32, n, 1, qrbh, nqh, 0};
        qap32_.a[h] = CsrT<float>{ap, ai, av32, m, 1, arbh, nah, 0};
        qap32_.pq[h] = pq32;
        qap32_.pa[h] = pa32;
      }
    }
    chain(hipStreamSynchronize(stream_));
    if ((r = check(e, "panel upload", err))) return r;
  }
  px_ = make_part(n, 1, 512);
  ps_ = make_part(mi, 1, 256);
  pr_ = make_part(m, 1, 256);
  pq_ = make_part(n, GQ, 1024);
  pa_ = make_part(m, GA, 1024);
  pt_ = make_part(n, GT, 1024);
  ip_ = InnerParams{};
  ip_.n = n; ip_.m = m; ip_.me = qp_.me; ip_.mi = mi; ip_.dw = n + mi + m;
  ip_.stream_grid = st_.stream_grid;
  ip_.pass_limit = st_.kkt_pass_limit;
  timers_.resize(TM_COUNT);
  timers_[TM_XTRIAL].name = "xtrial";
  timers_[TM_QA].name = "qa_spmv";
  timers_[TM_AT].name = "at_spmv";
  timers_[TM_DECIDE].name = "decide";
  timers_[TM_QA_ROWS].name = "qa_rows";
  const double me = qp_.me;
  const double vb = fp32_ ? 4.0 : 8.0;  // bytes per value of the bulk type
  timers_[TM_XTRIAL].bytes = 12.0 * vb * n;
  // Q part: off-diagonal values+indices, row pointers, x_tr once, diagonal, Q x_tr written;
  // A part: values+indices, row pointers, x_tr once, row-local vectors
  timers_[TM_QA].bytes = (4.0 + vb) * nzo + 4.0 * (n + 1) + 3.0 * vb * n + (4.0 + vb) * nza +
                         4.0 * (m + 1) + vb * n + 15.0 * vb * me + 20.0 * vb * mi;
  timers_[TM_AT].bytes = (4.0 + vb) * nza + 4.0 * (n + 1) + vb * m + vb * n + 5.0 * vb * n;
  timers_[TM_DECIDE].bytes = 0.0;
  timers_[TM_QA_ROWS].bytes = 0.0;
  if (fp32_ ? panels32_ : panels64_) {
    // the two-panel form: values and indices once, both panels' row
    // pointers, x_tr once, one partial per row and panel written; then the
    // A partials read back with the A row epilogue of the one-launch form;
    // the Q partials and the diagonal are read, and Q x_tr written, by the
    // A' launch instead of reading Q x_tr
    timers_[TM_QA].name = "qa_panels";
    timers_[TM_QA].bytes = (4.0 + vb) * (nzo + nza) + 8.0 * (n + 1) + 8.0 * (m + 1) + vb * n +
                           2.0 * vb * (n + m);
    timers_[TM_QA_ROWS].bytes = 2.0 * vb * m + 15.0 * vb * me + 20.0 * vb * mi;
    timers_[TM_AT].bytes += 3.0 * vb * n;
  }
  return PDNQP_OK;
}

void Solver::timed_launch(int which, const std::function<void(LaunchEvents)> &f) {
  if (!sample_now_) {
    f(LaunchEvents{});
    return;
  }
  KernelTimer &t = timers_[which];
  if ((int)t.ev.size() < 2 * (t.used + 1)) {
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    t.ev.push_back(a);
    t.ev.push_back(b);
  }
  f(LaunchEvents{t.ev[2 * t.used], t.ev[2 * t.used + 1]});
  t.used += 1;
}

void Solver::harvest_timers() {
  if (!st_.profile) return;
  for (auto &t : timers_) {
    for (int k = 0; k < t.used; ++k) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, t.ev[2 * k], t.ev[2 * k + 1]) == hipSuccess) {
        t.total_ms += ms;
        t.launches += 1;
      }
    }
    t.used = 0;
  }
}

int Solver::read_ctrl(std::string &err) {
  int r = check(hipMemcpyAsync(hctrl_, ctrl_, sizeof(Ctrl), hipMemcpyDeviceToHost, stream_),
                "ctrl readback", err);
  if (r) return r;
  r = check(hipStreamSynchronize(stream_), "hipStreamSynchronize", err);
  if (r) return r;
  harvest_timers();
  return PDNQP_OK;
}

// Smallest eigenvalue estimate of the scaled Q by plain Lanczos (three-term
// recurrence from the normalised all-ones vector, no reorthogonalisation).
double Solver::lanczos(std::string &err, bool &ok) {
  const int32_t n = qp_.n;
  const int k = std::min<int>(st_.lanczos_iters, n);
  // ||Q||_inf for the breakdown threshold
  launch_row_abssum(stream_, Q_, v_.tmp_n, pq_);
  launch_absmax(stream_, ctrl_, v_.tmp_n, n, 3, v_.partial);
  ok = read_ctrl(err) == PDNQP_OK;
  if (!ok) return 0.0;
  const double qnorm = std::max(1.0, hctrl_->gen[3]);
  double *vv = v_.qxo, *vp = v_.atl, *w = v_.tmp_n;
  launch_fill(stream_, vv, 1.0 / std::sqrt((double)n), n);
  launch_fill(stream_, vp, 0.0, n);
  std::vector<double> al, be;
  double beta_prev = 0.0;
  for (int j = 0; j < k; ++j) {
    launch_spmv(stream_, Q_, vv, w, 1.0, pq_);
    launch_dot(stream_, ctrl_, vv, w, n, 0, v_.partial);
    launch_lanczos_update(stream_, ctrl_, w, vv, vp, beta_prev, n, v_.partial);
    ok = read_ctrl(err) == PDNQP_OK;
    if (!ok) return 0.0;
    const double alpha = hctrl_->gen[0];
    const double beta = std::sqrt(hctrl_->gen[1]);
    al.push_back(alpha);
    if (j == k - 1 || beta <= 1e-14 * qnorm) break;
    be.push_back(beta);
    launch_copy(stream_, vp, vv, n);
    launch_elem(stream_, EL_AXPBY, vv, w, nullptr, beta, n);
    beta_prev = beta;
  }
  if (al.size() == 1) return al[0];
  return tridiag_min_eig(al, be);
}

// Outer scaling (Section 3.1), objective scalar, scaled data.
int Solver::setup(const double *x0c, const double *lam0_int, double &c_obj, double &gamma,
                  double &lam_hat, std::string &err) {
  const int32_t n = qp_.n, m = qp_.m, me = qp_.me;
  hipError_t e = hipMemcpyAsync(v_.X[0], x0c, n * 8, hipMemcpyHostToDevice, stream_);
  if (m) {
    hipError_t e2 = hipMemcpyAsync(v_.lam, lam0_int, m * 8, hipMemcpyHostToDevice, stream_);
    if (e == hipSuccess) e = e2;
  }
  int r = check(e, "upload x0/lambda0", err);
  if (r) return r;
  launch_fill(stream_, v_.Dc, 1.0, m);
  launch_fill(stream_, v_.Dx, 1.0, n);
  if (st_.outer_scaling != PDNQP_SCALE_NONE) {
    const bool withq = st_.outer_scaling == PDNQP_SCALE_RUIZ_QA;
    for (int sw = 0; sw < st_.ruiz_sweeps; ++sw) {
      launch_row_absmax(stream_, Ar_, v_.Dc, v_.Dx, v_.tmp_m, pa_);
      launch_fill(stream_, v_.tmp_n, 0.0, n);
      launch_row_absmax(stream_, ATr_, v_.Dx, v_.Dc, v_.tmp_n, pt_);
      if (withq) launch_row_absmax(stream_, Qr_, v_.Dx, v_.Dx, v_.qxo, pq_);
      launch_ruiz_update(stream_, v_.Dc, v_.tmp_m, m, v_.Dx, v_.tmp_n, withq ? v_.qxo : nullptr,
                         n);
    }
  }
  // c_obj = 1 / max(1, ||Dx (Q x0 + c)||_inf)
  launch_spmv(stream_, Qr_, v_.X[0], v_.tmp_n, 1.0, pq_);
  launch_elem(stream_, EL_GRAD, v_.tmp_n, v_.Dx, craw_, 0.0, n);
  launch_absmax(stream_, ctrl_, v_.tmp_n, n, 0, v_.partial);
  if ((r = read_ctrl(err))) return r;
  c_obj = 1.0 / std::max(1.0, hctrl_->gen[0]);
  // scaled values: Q <- c_obj Dx Q Dx, A <- Dc A Dx, A' gathered from A
  hipMemcpyAsync(Qv_, Qraw_, Q_.rows ? qp_.Qi.size() * 8 : 0, hipMemcpyDeviceToDevice, stream_);
  hipMemcpyAsync(Av_, Araw_, qp_.Ai.size() * 8, hipMemcpyDeviceToDevice, stream_);
  launch_scale_csr(stream_, Qp_, Qi_, Qv_, n, v_.Dx, v_.Dx, c_obj, pq_);
  if (!qp_.Qoi.empty())
    hipMemcpyAsync(Qov_, Qoraw_, qp_.Qoi.size() * 8, hipMemcpyDeviceToDevice, stream_);
  launch_scale_csr(stream_, Qop_, Qoi_, Qov_, n, v_.Dx, v_.Dx, c_obj, make_part(n, Qo_.G, 1024));
  launch_elem(stream_, EL_DIAG, qdiag_, v_.Dx, qdiag_raw_, c_obj, n);
  launch_scale_csr(stream_, Ap_, Ai_, Av_, m, v_.Dc, v_.Dx, 1.0, pa_);
  launch_gather(stream_, ATv_, Av_, atperm_, (int64_t)qp_.Ai.size());
  if (panels64_ || panels32_) {
    for (int h = 0; h < 2; ++h) {
      launch_gather(stream_, const_cast<double *>(qap64_.q[h].v), Qov_, pperm_q_[h], pnnz_q_[h]);
      launch_gather(stream_, const_cast<double *>(qap64_.a[h].v), Av_, pperm_a_[h], pnnz_a_[h]);
    }
  }
  launch_elem(stream_, EL_MULS, c_, v_.Dx, craw_, c_obj, n);
  launch_elem(stream_, EL_MUL, b_, v_.Dc, braw_, 0.0, m);
  launch_elem(stream_, EL_DIV, lo_, xlraw_, v_.Dx, 0.0, n);
  launch_elem(stream_, EL_DIV, hi_, xuraw_, v_.Dx, 0.0, n);
  launch_elem(stream_, EL_DIVINTO, v_.X[0], v_.Dx, nullptr, 0.0, n);
  launch_elem(stream_, EL_SCALE_DIV, v_.lam, v_.lam, v_.Dc, c_obj, m);
  // proximal step (R-choice)
  if (st_.gamma_override > 0) {
    gamma = st_.gamma_override;
    lam_hat = std::numeric_limits<double>::quiet_NaN();
  } else {
    bool ok = true;
    lam_hat = lanczos(err, ok);
    if (!ok) return PDNQP_E_DEVICE;
    launch_row_abssum(stream_, Q_, v_.tmp_n, pq_);
    launch_absmax(stream_, ctrl_, v_.tmp_n, n, 3, v_.partial);
    if ((r = read_ctrl(err))) return r;
    const double qn = hctrl_->gen[3];
    gamma = 1.0 / (std::max(0.0, -lam_hat) + st_.delta_gamma * std::max(1.0, qn));
  }
  // initial penalty (QPALM-style) and norms of the scaled data
  launch_spmv(stream_, Q_, v_.X[0], v_.tmp_n, 1.0, pq_);
  launch_dot(stream_, ctrl_, v_.X[0], v_.tmp_n, n, 0, v_.partial);
  launch_dot(stream_, ctrl_, c_, v_.X[0], n, 1, v_.partial);
  if (m) {
    launch_spmv(stream_, A_, v_.X[0], v_.ax, 1.0, pa_);
    launch_viol(stream_, ip_, v_, v_.tmp_m);
    launch_dot(stream_, ctrl_, v_.tmp_m, v_.tmp_m, m, 2, v_.partial);
    launch_absmax(stream_, ctrl_, b_, me, 4, v_.partial);
    launch_absmax(stream_, ctrl_, b_ + me, m - me, 5, v_.partial);
  }
  launch_absmax(stream_, ctrl_, c_, n, 6, v_.partial);
  if ((r = read_ctrl(err))) return r;
  const double f = 0.5 * hctrl_->gen[0] + hctrl_->gen[1];
  const double vv = m ? hctrl_->gen[2] : 0.0;
  bE_norm_ = (m && me) ? hctrl_->gen[4] : 0.0;
  bI_norm_ = (m && m > me) ? hctrl_->gen[5] : 0.0;
  c_norm_ = hctrl_->gen[6];
  double s0 = st_.sigma_init * std::max(1.0, std::fabs(f)) / std::max(1.0, 0.5 * vv);
  s0 = std::min(std::max(s0, st_.sigma0_min), st_.sigma0_max);
  launch_fill(stream_, v_.sigma, s0, m);
  launch_copy(stream_, v_.z, v_.X[0], n);
  launch_elem(stream_, EL_NEG, v_.Y[0], v_.lam, nullptr, 0.0, m);
  if (fp32_) {
    launch_cast<float, double>(stream_, Qo32v_, Qov_, (int64_t)qp_.Qoi.size());
    launch_cast<float, double>(stream_, A32v_, Av_, (int64_t)qp_.Ai.size());
    launch_cast<float, double>(stream_, AT32v_, ATv_, (int64_t)qp_.Ai.size());
    if (panels32_) {
      for (int h = 0; h < 2; ++h) {
        launch_cast<float, double>(stream_, const_cast<float *>(qap32_.q[h].v), qap64_.q[h].v,
                                   pnnz_q_[h]);
        launch_cast<float, double>(stream_, const_cast<float *>(qap32_.a[h].v), qap64_.a[h].v,
                                   pnnz_a_[h]);
      }
    }
    launch_cast<float, double>(stream_, const_cast<float *>(iv32_.qdiag), qdiag_, n);
    launch_cast<float, double>(stream_, const_cast<float *>(iv32_.lo), lo_, n);
    launch_cast<float, double>(stream_, const_cast<float *>(iv32_.hi), hi_, n);
    launch_cast<float, double>(stream_, const_cast<float *>(iv32_.b), b_, m);
  }
  return check(hipGetLastError(), "setup kernels", err);
}

// Warm start, inner scaling and steps, starting products and anchor metric.
void Solver::form_inner(double gamma) {
  const int cur = hctrl_->cur;
  launch_spmv(stream_, A_, v_.X[cur], v_.ax, 1.0, pa_);
  launch_warm(stream_, ip_, v_, cur, gamma);
  launch_fill(stream_, v_.tmp_m, 1.0, qp_.m);
  launch_fill(stream_, v_.Fx, 1.0, qp_.n);
  launch_fill(stream_, v_.Fs, 1.0, qp_.mi);
  launch_fill(stream_, v_.Fr, 1.0, qp_.m);
  if (qp_.m > 0) {
    for (int sw = 0; sw < st_.ruiz_sweeps; ++sw) {
      launch_inner_ruiz_sweep(stream_, ip_, v_, A_, AT_, pa_, pt_, Fx2_, Fs2_, Fr2_, E2buf_);
      std::swap(v_.Fx, Fx2_);
      std::swap(v_.Fs, Fs2_);
      std::swap(v_.Fr, Fr2_);
      std::swap(v_.tmp_m, E2buf_);
    }
  }
  launch_steps(stream_, ip_, v_, Q_, A_, AT_, 1.0 / gamma, st_.step_boost);
  InnerParams pi = ip_;
  pi.mode_init = 1;
  if (bulk32_) {
    // per-outer-step data and the warm-started state into the FP32 bulk buffers
    const int32_t n = qp_.n, m = qp_.m, mi = qp_.mi;
    launch_cast<float, double>(stream_, iv32_.sigma, v_.sigma, m);
    launch_cast<float, double>(stream_, iv32_.lam, v_.lam, m);
    launch_cast<float, double>(stream_, iv32_.qx, v_.qx, n);
    launch_cast<float, double>(stream_, iv32_.taub_x, v_.taub_x, n);
    launch_cast<float, double>(stream_, iv32_.taub_s, v_.taub_s, mi);
    launch_cast<float, double>(stream_, iv32_.taub_r, v_.taub_r, m);
    launch_cast<float, double>(stream_, iv32_.etab, v_.etab, m);
    launch_cast<float, double>(stream_, iv32_.S2x, v_.S2x, n);
    launch_cast<float, double>(stream_, iv32_.S2s, v_.S2s, mi);
    launch_cast<float, double>(stream_, iv32_.S2r, v_.S2r, m);
    launch_cast<float, double>(stream_, iv32_.E2, v_.E2, m);
    cast_state_to32(cur);
    launch_inner_init<float>(stream_, ctrl_, ip_, iv32_, Qo32_, AT32_, pr_);
    launch_check<float>(stream_, ctrl_, pi, iv32_, px_, ps_, pr_);
  } else {
    const IterVecs<double> iv = iv64();
    launch_inner_init<double>(stream_, ctrl_, ip_, iv, Qo_, AT_, pr_);
    launch_check<double>(stream_, ctrl_, pi, iv, px_, ps_, pr_);
  }
}

// The FP64 iteration vectors alias the solver's FP64 buffers.
IterVecs<double> Solver::iv64() const {
  IterVecs<double> iv{};
  iv.lo = v_.lo; iv.hi = v_.hi; iv.b = v_.b; iv.qdiag = v_.qdiag;
  iv.sigma = v_.sigma; iv.lam = v_.lam; iv.qx = v_.qx;
  iv.taub_x = v_.taub_x; iv.taub_s = v_.taub_s; iv.taub_r = v_.taub_r; iv.etab = v_.etab;
  iv.S2x = v_.S2x; iv.S2s = v_.S2s; iv.S2r = v_.S2r; iv.E2 = v_.E2;
  for (int k = 0; k < 2; ++k) {
    iv.X[k] = v_.X[k]; iv.QX[k] = v_.QX[k]; iv.ATY[k] = v_.ATY[k]; iv.S[k] = v_.S[k];
    iv.R[k] = v_.R[k]; iv.Y[k] = v_.Y[k]; iv.BW[k] = v_.BW[k];
  }
  iv.xbar = v_.xbar; iv.qxbar = v_.qxbar; iv.sbar = v_.sbar; iv.rbar = v_.rbar; iv.ybar = v_.ybar;
  iv.xa = v_.xa; iv.sa = v_.sa; iv.ra = v_.ra; iv.ya = v_.ya;
  iv.axbar = v_.axbar; iv.atybar = v_.atybar;
  iv.partial = v_.partial;
  iv.trace_w = v_.trace_w; iv.trace_y = v_.trace_y; iv.trace_tr = v_.trace_tr;
  iv.trace_ck = v_.trace_ck;
  return iv;
}

void Solver::cast_state_to32(int cur) {
  launch_cast<float, double>(stream_, iv32_.X[cur], v_.X[cur], qp_.n);
  launch_cast<float, double>(stream_, iv32_.S[cur], v_.S[cur], qp_.mi);
  launch_cast<float, double>(stream_, iv32_.R[cur], v_.R[cur], qp_.m);
  launch_cast<float, double>(stream_, iv32_.Y[cur], v_.Y[cur], qp_.m);
  launch_cast<float, double>(stream_, iv32_.BW[cur], v_.BW[cur], qp_.m);
}

// The outer update works on FP64 copies of the inner iterate.
void Solver::cast_state_to64(int cur) {
  launch_cast<double, float>(stream_, v_.X[cur], iv32_.X[cur], qp_.n);
  launch_cast<double, float>(stream_, v_.Y[cur], iv32_.Y[cur], qp_.m);
}

template <>
bool Solver::use_panels<double>() const {
  return panels64_;
}
template <>
bool Solver::use_panels<float>() const {
  return panels32_;
}
template <>
const QAPanelSet<double> &Solver::panel_set<double>() const {
  return qap64_;
}
template <>
const QAPanelSet<float> &Solver::panel_set<float>() const {
  return qap32_;
}

// One chunk of trial slots followed by the check kernels.  Slots after a
// due check (or after the inner limit) find the state not running and exit
// at once, so the full chunk can always be enqueued.
template <typename T>
void Solver::enqueue_chunk(int slots, bool sampled, const IterVecs<T> &iv, const CsrT<T> &Qo,
                           const CsrT<T> &A, const CsrT<T> &AT) {
  const bool panels = use_panels<T>();
  for (int s = 0; s < slots; ++s) {
    sample_now_ = sampled && st_.profile > 0 && (slot_count_++ % st_.profile) == 0;
    timed_launch(TM_XTRIAL, [&](LaunchEvents e) { launch_xtrial<T>(stream_, ctrl_, ip_, iv, e); });
    if (panels) {
      const QAPanelSet<T> &ps = panel_set<T>();
      timed_launch(TM_QA, [&](LaunchEvents e) { launch_qa_panels<T>(stream_, ctrl_, ip_, iv, ps, e); });
      timed_launch(TM_QA_ROWS,
                   [&](LaunchEvents e) { launch_qa_rows<T>(stream_, ctrl_, ip_, iv, ps, e); });
    } else {
      timed_launch(TM_QA, [&](LaunchEvents e) { launch_qa<T>(stream_, ctrl_, ip_, iv, Qo, A, e); });
    }
    timed_launch(TM_AT, [&](LaunchEvents e) {
      if (panels) {
        const QAPanelSet<T> &ps = panel_set<T>();
        launch_at<T>(stream_, ctrl_, ip_, iv, AT, e, ps.pq[0], ps.pq[1]);
      } else {
        launch_at<T>(stream_, ctrl_, ip_, iv, AT, e);
      }
    });
    timed_launch(TM_DECIDE, [&](LaunchEvents e) {
      launch_decide(stream_, ctrl_, ip_, iv.partial, iv.trace_tr, Qo.nrb, A.nrb, AT.nrb, e,
                    panels);
    });
    if (trace_iters_cap_ > 0) launch_trace<T>(stream_, ctrl_, ip_, iv);
  }
  sample_now_ = false;
  launch_flush<T>(stream_, ctrl_, ip_, iv, px_, pr_);
  launch_check_spmv<T>(stream_, ctrl_, iv, A, AT, pa_, pt_);
  launch_check<T>(stream_, ctrl_, ip_, iv, px_, ps_, pr_);
  launch_apply<T>(stream_, ctrl_, ip_, iv, px_, pr_);
}

// Captures a full chunk (check_every slots and the check) with the current
// inner parameters.
template <typename T>
int Solver::capture_chunk(std::string &err, const IterVecs<T> &iv, const CsrT<T> &Qo,
                          const CsrT<T> &A, const CsrT<T> &AT) {
  // captured on a private stream (the solver's stream may be the legacy
  // default stream, which cannot be captured) and replayed on the solver's
  if (!cap_stream_) {
    const int rc = check(hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking),
                         "hipStreamCreate", err);
    if (rc) return rc;
  }
  hipGraph_t g = nullptr;
  hipStream_t launch_stream = stream_;
  int r = check(hipStreamBeginCapture(cap_stream_, hipStreamCaptureModeThreadLocal),
                "graph capture", err);
  if (r) return r;
  stream_ = cap_stream_;
  enqueue_chunk<T>(st_.check_every, false, iv, Qo, A, AT);
  stream_ = launch_stream;
  r = check(hipStreamEndCapture(cap_stream_, &g), "graph capture", err);
  if (r) return r;
  if (gexec_) {
    hipGraphExecDestroy(gexec_);
    gexec_ = nullptr;
  }
  r = check(hipGraphInstantiate(&gexec_, g, nullptr, nullptr, 0), "graph instantiate", err);
  hipGraphDestroy(g);
  if (r) return r;
  graph_valid_ = true;
  return PDNQP_OK;
}

template <typename T>
int Solver::run_inner(double deadline, std::string &err, const IterVecs<T> &iv, const CsrT<T> &Qo,
                      const CsrT<T> &A, const CsrT<T> &AT) {
  for (;;) {
    const int t = hctrl_->t, tc = hctrl_->t_call;
    int slots = st_.check_every - (t % st_.check_every);
    slots = std::min(slots, ip_.max_inner - tc);
    slots = std::max(slots, 1);
    // with profiling on, one chunk in `profile` is launched directly so that
    // its slots can be sampled
    const bool sampled = st_.profile > 0 && (!st_.graph || (chunk_count_ % st_.profile) == 0);
    ++chunk_count_;
    if (st_.graph && !sampled) {
      if (!graph_valid_) {
        const int rc = capture_chunk<T>(err, iv, Qo, A, AT);
        if (rc) return -1000 + rc;
      }
      const int rc = check(hipGraphLaunch(gexec_, stream_), "graph launch", err);
      if (rc) return -1000 + rc;
    } else {
      enqueue_chunk<T>(slots, sampled, iv, Qo, A, AT);
    }
    int r = check(hipGetLastError(), "inner launches", err);
    if (r) return -1000 + r;
    if ((r = read_ctrl(err))) return -1000 + r;
    const int state = hctrl_->state;
    if (state == ST_RUNNING) {
      if (now_s() > deadline) return ST_RUNNING;
      continue;
    }
    return state;
  }
}

// Start shared by both paths: trace buffers, x0 clipped into the box,
// lambda0 mapped to the internal rows (inequality rows kept <= 0).
int Solver::begin(const double *x0, const double *lam0, std::vector<double> &x0c,
                  std::vector<double> &lam0i, std::string &err) {
  const int32_t n = qp_.n, m = qp_.m, me = qp_.me;
  const int dw = n + qp_.mi + m;
  // trace buffers
  traced_ = false;
  trace_iters_cap_ = std::max(0, st_.trace_iters);
  trace_trials_cap_ = std::max(0, st_.trace_trials);
  if (trace_iters_cap_ > 0 && !tw_) {
    tw_ = (double *)dalloc((size_t)trace_iters_cap_ * dw * 8);
    ty_ = (double *)dalloc((size_t)trace_iters_cap_ * std::max(m, 1) * 8);
    if (!tw_ || !ty_) {
      err = "trace allocation failed";
      return PDNQP_E_NOMEM;
    }
  }
  if (trace_trials_cap_ > 0 && !ttr_) {
    ttr_ = (double *)dalloc((size_t)trace_trials_cap_ * 3 * 8);
    tck_ = (int32_t *)dalloc((size_t)trace_trials_cap_ * 4 * 4);
    if (!ttr_ || !tck_) {
      err = "trace allocation failed";
      return PDNQP_E_NOMEM;
    }
  }
  v_.trace_w = tw_;
  v_.trace_y = ty_;
  v_.trace_tr = ttr_;
  v_.trace_ck = tck_;
  // the FP32 iteration vectors share the reduction and trace buffers; they
  // must be set before the first inner-QP formation launches a check
  iv32_.partial = v_.partial;
  iv32_.trace_w = tw_;
  iv32_.trace_y = ty_;
  iv32_.trace_tr = ttr_;
  iv32_.trace_ck = tck_;
  ip_.trace_iters_cap = trace_iters_cap_;
  ip_.trace_trials_cap = trace_trials_cap_;
  for (auto &t : timers_) {
    t.launches = 0;
    t.total_ms = 0.0;
    t.used = 0;
  }
  x0c.assign(n, 0.0);
  lam0i.assign(m, 0.0);
  for (int i = 0; i < n; ++i) {
    double x = x0 ? x0[i] : 0.0;
    x0c[i] = x < qp_.xl[i] ? qp_.xl[i] : (x > qp_.xu[i] ? qp_.xu[i] : x);
  }
  if (lam0) {
    for (int j = 0; j < m; ++j) {
      double l = qp_.sign_of[j] * lam0[qp_.row_of[j]];
      if (j >= me) l = std::min(l, 0.0);
      lam0i[j] = l;
    }
  }
  return PDNQP_OK;
}

int Solver::solve(double eps_abs, double eps_rel, const double *x0, const double *lam0,
                  double *x_out, double *lam_out, pdnqp_info *info, std::string &err) {
  const double t_start = now_s();
  const double deadline =
      std::isfinite(st_.time_limit_s) ? t_start + st_.time_limit_s : std::numeric_limits<double>::infinity();
  const int32_t n = qp_.n, m = qp_.m, me = qp_.me, mi = qp_.mi;
  const int dw = n + mi + m;
  int r;
  std::vector<double> x0c, lam0i;
  if ((r = begin(x0, lam0, x0c, lam0i, err))) return r;
  aa_win_.clear();
  aa_last_valid_ = false;
  aa_steps_ = 0;
  // control block
  Ctrl hc;
  std::memset(&hc, 0, sizeof(hc));
  hc.state = ST_RUNNING;
  hc.cur = 0;
  hc.omega = st_.omega0;
  hc.step_scale = 1.0;
  hc.kkt_prev = std::numeric_limits<double>::infinity();
  *hctrl_ = hc;
  if ((r = check(hipMemcpyAsync(ctrl_, hctrl_, sizeof(Ctrl), hipMemcpyHostToDevice, stream_),
                 "ctrl upload", err)))
    return r;
  double c_obj = 1.0, gamma = 0.0, lam_hat = 0.0;
  if ((r = setup(x0c.data(), lam0i.data(), c_obj, gamma, lam_hat, err))) return r;
  if ((r = read_ctrl(err))) return r;
  const double t_setup = now_s() - t_start;
  gamma_ = gamma;
  ip_.gamma_inv = 1.0 / gamma;
  ip_.h_norm = bE_norm_;
  ip_.check_every = st_.check_every;
  ip_.max_inner = st_.max_inner;
  ip_.max_rejects = st_.max_rejects;
  ip_.shrink_safety = st_.shrink_safety;
  ip_.shrink_min = st_.shrink_min;
  ip_.shrink_max = st_.shrink_max;
  ip_.restart_suff = st_.restart_suff;
  ip_.restart_nec = st_.restart_nec;
  ip_.restart_art = st_.restart_art;
  ip_.mode_init = 0;

  double delta_a = st_.delta0, delta_r = st_.delta0, eps_ak = 1.0, eps_rk = 1.0;
  // internal tolerances: the requested ones, halved by the calibration of
  // the external test (reading of the experimental protocol)
  double ea = eps_abs, er = eps_rel;
  int32_t halvings = 0;
  const RawData raw{braw_, xlraw_, xuraw_, craw_, c_obj};
  double rd_prev = NAN;  // r_d of the previous outer step (none yet: not contracting)
  bool have_prev = false, need_form = true;
  int status = PDNQP_MAX_ITER;
  int64_t k = 0;
  double rp = NAN, rd = NAN, sp = NAN, sd = NAN;
  // learned controller state
  const bool ctl_on = st_.controller == 1 && ctl_loaded_;
  bool ctl_fallback = false;
  int ctl_stall = 0;
  double ctl_best = std::numeric_limits<double>::infinity();
  double rp_prev = NAN;
  log_n_ = 0;
  log_feat_.assign((size_t)std::max(0, st_.outer_log) * PDNQP_FEATURES, 0.0);
  log_rec_.assign((size_t)std::max(0, st_.outer_log) * PDNQP_OUTER_RECORD, 0.0);
  ip_.max_inner = st_.max_inner;
  bulk32_ = fp32_;
  int32_t promoted_outer = 0;
  double p32_best = std::numeric_limits<double>::infinity();
  int p32_stall = 0;
  while (k < st_.max_outer) {
    // FP32 storage bounds the inner residual the FP32 iteration can reach:
    // at or below the promotion level the inner iteration continues in FP64 (the
    // FP64 copy of the iterate is current after every FP32 inner call)
    if (bulk32_ && std::max(delta_a, delta_r) <= st_.fp32_promote) {
      bulk32_ = false;
      promoted_outer = (int32_t)(k + 1);
      need_form = true;
    }
    ip_.delta_a = delta_a;
    ip_.delta_r = delta_r;
    const double delta_used = delta_a;
    const int64_t acc_before = hctrl_->accepted, rst_before = hctrl_->restarts;
    if (need_form) {
      if (st_.anderson_mem > 0) anderson_form();
      form_inner(gamma);
      graph_valid_ = false;  // the inner parameters of the chunk changed
      if ((r = read_ctrl(err))) return r;
    }
    int ist;
    if (bulk32_) {
      ist = run_inner<float>(deadline, err, iv32_, Qo32_, A32_, AT32_);
      if (ist > -1000) cast_state_to64(hctrl_->cur);
    } else {
      ist = run_inner<double>(deadline, err, iv64(), Qo_, A_, AT_);
    }
    if (ist <= -1000) return ist + 1000;
    k += 1;
    if (ist == ST_NUMERR) {
      status = PDNQP_NUMERICAL_ERROR;
      break;
    }
    if (ist == ST_RUNNING) {  // deadline inside the inner solve
      status = PDNQP_TIME_LIMIT;
      break;
    }
    if (ist == ST_PASS_LIMIT) {
      status = PDNQP_MAX_ITER;
      break;
    }
    // with the learned controller, the inner iteration budget ends the inner
    // solve like its stopping test
    if (ist == ST_ITER_LIMIT && !(ctl_on && !ctl_fallback)) {
      // keep the outer variables and continue the inner solve
      if (st_.verbose >= 2) {
        std::fprintf(stderr,
                     "[pdnqp] inner call %lld hit the iteration limit: inner %lld  restarts %lld  "
                     "omega %.3g  %.2fs\n",
                     (long long)k, (long long)hctrl_->accepted, (long long)hctrl_->restarts,
                     hctrl_->omega, now_s() - t_start);
        std::fflush(stderr);
      }
      need_form = false;
      hctrl_->state = ST_RUNNING;
      hctrl_->t_call = 0;
      if ((r = check(hipMemcpyAsync(ctrl_, hctrl_, offsetof(Ctrl, alpha_pend),
                                    hipMemcpyHostToDevice, stream_),
                     "ctrl update", err)))
        return r;
      if (now_s() > deadline) {
        status = PDNQP_TIME_LIMIT;
        break;
      }
      continue;
    }
    // multiplier update and outer residuals
    if (m) launch_outer_rows(stream_, ctrl_, ip_, v_, A_, pa_, raw);
    launch_outer_cols(stream_, ctrl_, ip_, v_, Q_, AT_, pq_, raw);
    if ((r = read_ctrl(err))) return r;
    const double *ov = hctrl_->outv;
    rp = m ? ov[0] : 0.0;
    sp = std::max({1.0, m ? ov[1] : 0.0, bE_norm_, m ? ov[2] : 0.0, bI_norm_});
    rd = ov[4];
    sd = std::max({1.0, ov[5], c_norm_, ov[6]});
    const double dxz = ov[7];
    const double rn = m ? ov[3] : 0.0;
    // controller features of this outer step (and the outer log)
    float feat[PDNQP_FEATURES];
    if (ctl_on || log_n_ < st_.outer_log) {
      double smin = 1.0, smean = 1.0, smax = 1.0;
      if (m) {
        launch_sigma_stats(stream_, ctrl_, v_.sigma, m, v_.partial);
        if ((r = read_ctrl(err))) return r;
        smin = hctrl_->gen[5];
        smean = hctrl_->gen[6] / m;
        smax = hctrl_->gen[7];
      }
      auto lg = [](double v) { return std::log10(std::max(v, 1e-30)); };
      const double inner_step = (double)(hctrl_->accepted - acc_before);
      const double rst_step = (double)(hctrl_->restarts - rst_before);
      double f[PDNQP_FEATURES] = {
          lg(rp), lg(rd), lg(sp), lg(sd), lg(dxz / gamma), lg(delta_used), lg(eps_ak),
          lg(hctrl_->omega), lg(smin), lg(smean), lg(smax),
          std::isfinite(rp_prev) ? lg(rp) - lg(rp_prev) : 0.0,
          std::isfinite(rd_prev) ? lg(rd) - lg(rd_prev) : 0.0,
          std::log10(1.0 + inner_step), std::log10(1.0 + rst_step), std::log10(1.0 + (double)k)};
      for (int i = 0; i < PDNQP_FEATURES; ++i) feat[i] = (float)f[i];
      if (log_n_ < st_.outer_log) {
        std::memcpy(&log_feat_[(size_t)log_n_ * PDNQP_FEATURES], f, sizeof(f));
        const double rec[PDNQP_OUTER_RECORD] = {rp, rd, sp, sd, hctrl_->omega, inner_step,
                                                rst_step, delta_used};
        std::memcpy(&log_rec_[(size_t)log_n_ * PDNQP_OUTER_RECORD], rec, sizeof(rec));
        log_n_ += 1;
      }
    }
    if (st_.verbose) {
      std::fprintf(stderr,
                   "[pdnqp] outer %lld  r_p %.3e (tol %.3e)  r_d %.3e (tol %.3e)  inner %lld  "
                   "restarts %lld  omega %.3g  delta %.2e  %.2fs\n",
                   (long long)k, rp, eps_abs + eps_rel * sp, rd, eps_abs + eps_rel * sd,
                   (long long)hctrl_->accepted, (long long)hctrl_->restarts, hctrl_->omega,
                   delta_a, now_s() - t_start);
      std::fflush(stderr);
    }
    if (rp <= ea + er * sp && rd <= ea + er * sd) {
      // the external test on the caller's data (experimental protocol):
      // accepted when it passes too; otherwise every internal use of the
      // tolerances is halved and the iteration continues, at most
      // external_halvings times
      const double rpu = m ? ov[8] : 0.0, spu = std::max(1.0, m ? ov[9] : 0.0);
      const double rdu = ov[10], sdu = std::max(1.0, ov[11]);
      if (st_.external_halvings == 0 ||
          (rpu <= eps_abs + eps_rel * spu && rdu <= eps_abs + eps_rel * sdu)) {
        status = PDNQP_SOLVED;
        break;
      }
      if (halvings >= st_.external_halvings) {
        status = PDNQP_INACCURATE;
        break;
      }
      halvings += 1;
      ea *= 0.5;
      er *= 0.5;
      if (st_.verbose)
        std::fprintf(stderr, "[pdnqp] outer %lld  external test failed (r_p %.3e, r_d %.3e): "
                     "internal tolerances halved to %.3e, %.3e\n",
                     (long long)k, rpu, rdu, ea, er);
    }
    // FP32 bulk that no longer improves the outer KKT measure hands the rest
    // of the solve to the FP64 inner iteration (from the next formation)
    if (bulk32_ && st_.fp32_stall > 0) {
      const double kkt = std::max(rp / (eps_abs + eps_rel * sp), rd / (eps_abs + eps_rel * sd));
      if (kkt < 0.9 * p32_best) {
        p32_best = kkt;
        p32_stall = 0;
      } else if (++p32_stall >= st_.fp32_stall) {
        bulk32_ = false;
        promoted_outer = (int32_t)(k + 1);
      }
    }
    // row penalties (penalty-trigger-eq)
    if (st_.anderson_mem > 0) {
      hctrl_->pen_moved = 0;
      hipMemcpyAsync(&ctrl_->pen_moved, &hctrl_->pen_moved, sizeof(int32_t),
                     hipMemcpyHostToDevice, stream_);
    }
    launch_penalty(stream_, ctrl_, ip_, v_, pr_, have_prev ? 1 : 0, rn, st_.theta_sigma,
                   st_.sigma_growth, st_.sigma_max, st_.penalty_gate, ea + er * sp);
    have_prev = true;
    // inner tolerances (inner-tolerance-factor)
    const double ratio = (rd == 0.0) ? 1.0 : std::min(1.0, dxz / gamma / rd);
    const double rho = st_.rho_in_max - (st_.rho_in_max - st_.rho_in_min) * ratio;
    delta_a = std::max(st_.delta_floor * ea, rho * delta_a);
    delta_r = std::max(st_.delta_floor * er, rho * delta_r);
    // proximal centre (center-update)
    if (rp <= eps_ak + eps_rk * sp) {
      launch_copy(stream_, v_.z, v_.X[hctrl_->cur], n);
      eps_ak *= st_.rho_z;
      eps_rk *= st_.rho_z;
      if (st_.center_floor) {
        eps_ak = std::max(eps_ak, ea);
        eps_rk = std::max(eps_rk, er);
      }
    }
    // Anderson step on (lambda_E, lambda_I, z), Section 3.2
    if (st_.anderson_mem > 0 &&
        (r = anderson(rp, rd, sp, ea, er, rd_prev, err)))
      return r;
    // learned controller: next inner tolerance, iteration budget and primal
    // weight; after 3 outer steps without progress of the outer KKT measure
    // the adaptive rule takes over for the rest of the solve
    if (ctl_on && !ctl_fallback) {
      const double kkt = std::max(rp / (eps_abs + eps_rel * sp), rd / (eps_abs + eps_rel * sd));
      if (kkt < ctl_best) {
        ctl_best = kkt;
        ctl_stall = 0;
      } else if (++ctl_stall >= 3) {
        ctl_fallback = true;
        ip_.max_inner = st_.max_inner;
      }
    }
    if (ctl_on && !ctl_fallback) {
      float y[3];
      hipMemcpyAsync(ctl_x_, feat, sizeof(feat), hipMemcpyHostToDevice, stream_);
      mlp_forward_device(stream_, ctl_theta_, ctl_x_, ctl_y_);
      hipMemcpyAsync(y, ctl_y_, sizeof(y), hipMemcpyDeviceToHost, stream_);
      if ((r = check(hipStreamSynchronize(stream_), "controller", err))) return r;
      auto clampd = [](double v, double lo, double hi) {
        return std::isfinite(v) ? std::min(std::max(v, lo), hi) : hi;
      };
      const double dl = std::exp(clampd((double)y[0], -60.0, 0.0));
      delta_a = std::max(st_.delta_floor * ea, dl);
      delta_r = std::max(st_.delta_floor * er, dl);
      ip_.max_inner = (int32_t)clampd(std::exp(clampd((double)y[1], 0.0, 30.0)),
                                      (double)st_.check_every, (double)st_.max_inner);
      hctrl_->omega = std::exp(clampd((double)y[2], -9.2, 9.2));
      hipMemcpyAsync(&ctrl_->omega, &hctrl_->omega, sizeof(double), hipMemcpyHostToDevice,
                     stream_);
    }
    rp_prev = rp;
    rd_prev = rd;
    need_form = true;
    if (now_s() > deadline) {
      status = PDNQP_TIME_LIMIT;
      break;
    }
  }
  // unscale: x = Dx x_bar, lambda = Dc lambda_bar (divided by c_obj in finish)
  const int cur = hctrl_->cur;
  launch_elem(stream_, EL_MUL, v_.tmp_n, v_.Dx, v_.X[cur], 0.0, n);
  launch_elem(stream_, EL_MUL, v_.tmp_m, v_.Dc, v_.lam, 0.0, m);
  Outcome oc;
  oc.status = status;
  oc.outer_iters = k;
  oc.trials = hctrl_->trials;
  oc.accepted = hctrl_->accepted;
  oc.rejected = hctrl_->rejected;
  oc.restarts = hctrl_->restarts;
  oc.checks = hctrl_->checks;
  oc.rp = rp;
  oc.rd = rd;
  oc.sp = sp;
  oc.sd = sd;
  oc.gamma = gamma;
  oc.lam_hat = lam_hat;
  oc.omega = hctrl_->omega;
  oc.c_obj = c_obj;
  oc.setup_s = t_setup;
  oc.trace_iters = hctrl_->trace_iters_n;
  oc.trace_trials = hctrl_->trace_trials_n;
  oc.trace_checks = hctrl_->trace_checks_n;
  oc.anderson_steps = aa_steps_;
  oc.controller_fallback = ctl_fallback ? 1 : 0;
  oc.promoted_outer = promoted_outer;
  oc.halvings = halvings;
  if ((r = finish(oc, x_out, lam_out, info, err))) return r;
  if (info) info->solve_s = now_s() - t_start;
  return PDNQP_OK;
}

// Copies the unscaled result (x in tmp_n, Dc lambda in tmp_m) and the trace
// back, maps lambda to the caller's rows and fills the info record.
int Solver::finish(const Outcome &oc, double *x_out, double *lam_out, pdnqp_info *info,
                   std::string &err) {
  const int32_t n = qp_.n, m = qp_.m;
  const int dw = n + qp_.mi + m;
  int r;
  std::vector<double> xs(n), ls(m);
  hipMemcpyAsync(xs.data(), v_.tmp_n, n * 8, hipMemcpyDeviceToHost, stream_);
  if (m) hipMemcpyAsync(ls.data(), v_.tmp_m, m * 8, hipMemcpyDeviceToHost, stream_);
  if (trace_iters_cap_ > 0 || trace_trials_cap_ > 0) {
    got_iters_ = oc.trace_iters;
    got_trials_ = oc.trace_trials;
    got_checks_ = oc.trace_checks;
    h_tw_.assign((size_t)got_iters_ * dw, 0.0);
    h_ty_.assign((size_t)got_iters_ * m, 0.0);
    h_ttr_.assign((size_t)got_trials_ * 3, 0.0);
    h_tck_.assign((size_t)got_checks_ * 4, 0);
    if (got_iters_) {
      hipMemcpyAsync(h_tw_.data(), tw_, h_tw_.size() * 8, hipMemcpyDeviceToHost, stream_);
      if (m) hipMemcpyAsync(h_ty_.data(), ty_, h_ty_.size() * 8, hipMemcpyDeviceToHost, stream_);
    }
    if (got_trials_)
      hipMemcpyAsync(h_ttr_.data(), ttr_, h_ttr_.size() * 8, hipMemcpyDeviceToHost, stream_);
    if (got_checks_)
      hipMemcpyAsync(h_tck_.data(), tck_, h_tck_.size() * 4, hipMemcpyDeviceToHost, stream_);
    traced_ = true;
  }
  if ((r = check(hipStreamSynchronize(stream_), "final copy", err))) return r;
  if ((r = check(hipGetLastError(), "final kernels", err))) return r;
  for (int j = 0; j < m; ++j) ls[j] = ls[j] / oc.c_obj;
  // the iterate lies in the scaled box; unscaling (and FP32 storage of the
  // scaled bounds) can leave it an ulp-level step outside the caller's box
  for (int i = 0; i < n; ++i) xs[i] = std::min(std::max(xs[i], qp_.xl[i]), qp_.xu[i]);
  std::vector<double> lam_orig(qp_.m_orig, 0.0);
  for (int j = 0; j < m; ++j) lam_orig[qp_.row_of[j]] += qp_.sign_of[j] * ls[j];
  if (x_out) std::memcpy(x_out, xs.data(), n * 8);
  if (lam_out && qp_.m_orig) std::memcpy(lam_out, lam_orig.data(), qp_.m_orig * 8);
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = oc.status;
    info->outer_iters = oc.outer_iters;
    info->inner_trials = oc.trials;
    info->inner_accepted = oc.accepted;
    info->inner_rejected = oc.rejected;
    info->restarts = oc.restarts;
    info->checks = oc.checks;
    info->r_p_scaled = oc.rp;
    info->r_d_scaled = oc.rd;
    info->s_p_scaled = oc.sp;
    info->s_d_scaled = oc.sd;
    info->gamma = oc.gamma;
    info->lambda_hat = oc.lam_hat;
    info->omega = oc.omega;
    info->setup_s = oc.setup_s;
    info->anderson_steps = oc.anderson_steps;
    info->controller_fallback = oc.controller_fallback;
    info->outer_logged = log_n_;
    info->promoted_outer = oc.promoted_outer;
    info->halvings = oc.halvings;
    external_check(xs, lam_orig, info);
  }
  return PDNQP_OK;
}

// KKT test on the caller's (unscaled) problem: primal residual with bound
// violation, projected stationarity, scales as in (outer-scales).
void Solver::external_check(const std::vector<double> &x, const std::vector<double> &lam,
                            pdnqp_info *info) const {
  const int32_t n = qp_.n, mo = qp_.m_orig;
  std::vector<double> ax(mo, 0.0), qx(n, 0.0), atl(n, 0.0);
  for (int j = 0; j < mo; ++j) {
    double s = 0.0;
    for (int k = qp_.oAp[j]; k < qp_.oAp[j + 1]; ++k) s += qp_.oAx[k] * x[qp_.oAi[k]];
    ax[j] = s;
    for (int k = qp_.oAp[j]; k < qp_.oAp[j + 1]; ++k) atl[qp_.oAi[k]] += qp_.oAx[k] * lam[j];
  }
  double obj = 0.0;
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int k = qp_.Qp[i]; k < qp_.Qp[i + 1]; ++k) s += qp_.Qx[k] * x[qp_.Qi[k]];
    qx[i] = s;
    obj += 0.5 * x[i] * s + qp_.c[i] * x[i];
  }
  double rp = 0.0, rd = 0.0, sp = 1.0, sd = 1.0;
  for (int j = 0; j < mo; ++j) {
    const double v = std::max({qp_.orl[j] - ax[j], ax[j] - qp_.oru[j], 0.0});
    rp = std::max(rp, v);
    sp = std::max(sp, std::fabs(ax[j]));
    if (std::isfinite(qp_.orl[j])) sp = std::max(sp, std::fabs(qp_.orl[j]));
    if (std::isfinite(qp_.oru[j])) sp = std::max(sp, std::fabs(qp_.oru[j]));
  }
  for (int i = 0; i < n; ++i) {
    rp = std::max({rp, qp_.xl[i] - x[i], x[i] - qp_.xu[i]});
    double t = x[i] - qx[i] - qp_.c[i] - atl[i];
    t = t < qp_.xl[i] ? qp_.xl[i] : (t > qp_.xu[i] ? qp_.xu[i] : t);
    rd = std::max(rd, std::fabs(x[i] - t));
    sd = std::max({sd, std::fabs(qx[i]), std::fabs(qp_.c[i]), std::fabs(atl[i])});
  }
  info->r_p = rp;
  info->r_d = rd;
  info->s_p = sp;
  info->s_d = sd;
  info->objective = obj;
}

int Solver::trace(int32_t *iters, double *w, double *y, int32_t *trials, double *tr,
                  int32_t *checks, int32_t *ck) const {
  if (!traced_) return PDNQP_E_STATE;
  if (iters) *iters = got_iters_;
  if (trials) *trials = got_trials_;
  if (checks) *checks = got_checks_;
  if (w && !h_tw_.empty()) std::memcpy(w, h_tw_.data(), h_tw_.size() * 8);
  if (y && !h_ty_.empty()) std::memcpy(y, h_ty_.data(), h_ty_.size() * 8);
  if (tr && !h_ttr_.empty()) std::memcpy(tr, h_ttr_.data(), h_ttr_.size() * 8);
  if (ck && !h_tck_.empty()) std::memcpy(ck, h_tck_.data(), h_tck_.size() * 4);
  return PDNQP_OK;
}

int Solver::kernel_stats(pdnqp_kernel_stat *out, int32_t cap, int32_t *count) const {
  const int nt = (int)timers_.size();
  if (count) *count = nt;
  for (int k = 0; k < nt && k < cap && out; ++k) {
    std::memset(&out[k], 0, sizeof(out[k]));
    std::strncpy(out[k].name, timers_[k].name.c_str(), sizeof(out[k].name) - 1);
    out[k].launches = timers_[k].launches;
    out[k].total_ms = timers_[k].total_ms;
    out[k].avg_us = timers_[k].launches ? 1000.0 * timers_[k].total_ms / timers_[k].launches : 0.0;
    out[k].bytes_per_launch = timers_[k].bytes;
  }
  return PDNQP_OK;
}

// ===========================================================================
// Batched path (pdnqp_batch.hip runs the method; these prepare and collect).
// ===========================================================================
int Solver::batch_prepare(double eps_abs, double eps_rel, const double *x0, const double *lam0,
                          int block, double ticks_per_s, BatchOut *dev_out, BatchInst &bi,
                          std::string &err) {
  const int32_t n = qp_.n, m = qp_.m;
  std::vector<double> x0c, lam0i;
  int r = begin(x0, lam0, x0c, lam0i, err);
  if (r) return r;
  hipError_t e = hipMemcpyAsync(v_.X[0], x0c.data(), n * 8, hipMemcpyHostToDevice, stream_);
  if (m && e == hipSuccess)
    e = hipMemcpyAsync(v_.lam, lam0i.data(), m * 8, hipMemcpyHostToDevice, stream_);
  if ((r = check(e, "upload x0/lambda0", err))) return r;
  // row blocks of the launch's tile (at most two rows per thread), each
  // followed by the blocks' first nonzeros
  const int tile = batch_tile(block);
  BatchBlocks *bb = nullptr;
  for (auto &x : bblocks_)
    if (x.block == block) bb = &x;
  if (!bb) {
    BatchBlocks nb;
    nb.block = block;
    auto build = [&](const std::vector<int32_t> &rp, int32_t rows, int32_t *&dev,
                     int32_t &nrb) -> bool {
      std::vector<int32_t> rb(2 * (size_t)rows + 4);
      stream_row_blocks(rp.data(), rows, 2 * block, &nrb, rb.data(), tile);
      for (int32_t b = 0; b <= nrb; ++b) rb[nrb + 1 + b] = rp[rb[b]];
      dev = (int32_t *)dalloc((size_t)(nrb + 1) * 8);
      if (!dev) return false;
      return hipMemcpyAsync(dev, rb.data(), (size_t)(nrb + 1) * 8, hipMemcpyHostToDevice,
                            stream_) == hipSuccess;
    };
    if (!build(qp_.Qp, n, nb.q, nb.nq) || !build(qp_.Qop, n, nb.qo, nb.nqo) ||
        !build(qp_.Ap, m, nb.a, nb.na) || !build(qp_.ATp, n, nb.at, nb.nat)) {
      err = "batch row-block upload failed";
      return PDNQP_E_DEVICE;
    }
    bblocks_.push_back(nb);
    bb = &bblocks_.back();
  }
  if (!lz_) {
    lz_ = (double *)dalloc((size_t)2 * std::max(1, st_.lanczos_iters) * 8);
    if (!lz_) {
      err = "device allocation failed";
      return PDNQP_E_NOMEM;
    }
  }
  std::memset(&bi, 0, sizeof(bi));
  bi.n = n;
  bi.m = m;
  bi.me = qp_.me;
  bi.mi = qp_.mi;
  bi.st = st_;
  bi.eps_abs = eps_abs;
  bi.eps_rel = eps_rel;
  // an infinite limit becomes 3600 s: every workgroup of the launch ends
  const double lim = std::isfinite(st_.time_limit_s) ? std::min(st_.time_limit_s, 1e9) : 3600.0;
  bi.limit_ticks = (uint64_t)(lim * ticks_per_s);
  bi.Q = BCsr{Qp_, Qi_, bb->q, bb->q + bb->nq + 1, n, bb->nq};
  bi.Qo = BCsr{Qop_, Qoi_, bb->qo, bb->qo + bb->nqo + 1, n, bb->nqo};
  bi.A = BCsr{Ap_, Ai_, bb->a, bb->a + bb->na + 1, m, bb->na};
  bi.AT = BCsr{ATp_, ATi_, bb->at, bb->at + bb->nat + 1, n, bb->nat};
  bi.atperm = atperm_;
  bi.Qraw = Qraw_;
  bi.Qoraw = Qoraw_;
  bi.qdiag_raw = qdiag_raw_;
  bi.Araw = Araw_;
  bi.ATraw = ATraw_;
  bi.craw = craw_;
  bi.xlraw = xlraw_;
  bi.xuraw = xuraw_;
  bi.braw = braw_;
  bi.Qv = Qv_;
  bi.Qov = Qov_;
  bi.qdiag = qdiag_;
  bi.Av = Av_;
  bi.ATv = ATv_;
  bi.c = c_;
  bi.lo = lo_;
  bi.hi = hi_;
  bi.b = b_;
  bi.Qo32 = Qo32v_;
  bi.A32 = A32v_;
  bi.AT32 = AT32v_;
  bi.v = v_;
  bi.Fx2 = Fx2_;
  bi.Fs2 = Fs2_;
  bi.Fr2 = Fr2_;
  bi.E2buf = E2buf_;
  bi.lz = lz_;
  bi.AU = AU_;
  bi.AG = AG_;
  bi.w64 = iv64();
  bi.w32 = iv32_;
  bi.out = dev_out;
  return check(hipStreamSynchronize(stream_), "batch prepare", err);
}

int Solver::batch_finish(const BatchOut &o, double ticks_per_s, double *x_out, double *lam_out,
                         pdnqp_info *info, std::string &err) {
  Outcome oc;
  oc.status = o.status;
  oc.outer_iters = o.outer_iters;
  oc.trials = o.trials;
  oc.accepted = o.accepted;
  oc.rejected = o.rejected;
  oc.restarts = o.restarts;
  oc.checks = o.checks;
  oc.rp = o.rp;
  oc.rd = o.rd;
  oc.sp = o.sp;
  oc.sd = o.sd;
  oc.gamma = o.gamma;
  oc.lam_hat = o.lam_hat;
  oc.omega = o.omega;
  oc.c_obj = o.c_obj;
  oc.setup_s = (double)(o.t_setup - o.t_begin) / ticks_per_s;
  oc.trace_iters = o.trace_iters_n;
  oc.trace_trials = o.trace_trials_n;
  oc.trace_checks = o.trace_checks_n;
  oc.anderson_steps = o.anderson_steps;
  oc.halvings = o.halvings;
  gamma_ = o.gamma;
  const int r = finish(oc, x_out, lam_out, info, err);
  if (r) return r;
  if (info) info->solve_s = (double)(o.t_end - o.t_begin) / ticks_per_s;
  return PDNQP_OK;
}

// ===========================================================================
// Anderson acceleration of (lambda_E, lambda_I, z) (Section 3.2).  The
// readings (activation, safeguard, projections, Tikhonov weight) are those
// of the oracle; the Gram system is formed on the device and solved here.
// ===========================================================================
void Solver::anderson_form() {
  const int cap = st_.anderson_mem + 2;
  int slot = 0;
  for (; slot < cap; ++slot)
    if (std::find(aa_win_.begin(), aa_win_.end(), slot) == aa_win_.end()) break;
  aa_form_slot_ = slot;
  const int64_t len = (int64_t)qp_.n + qp_.m;
  launch_aa_pack(stream_, AU_ + slot * len, v_.lam, v_.z, qp_.m, qp_.n);
}

int Solver::anderson(double rp, double rd, double sp, double eps_abs, double eps_rel,
                     double rd_prev, std::string &err) {
  const int32_t n = qp_.n, m = qp_.m;
  const int64_t len = (int64_t)n + m;
  int r = read_ctrl(err);  // penalty flag
  if (r) return r;
  const bool moved = hctrl_->pen_moved != 0;
  if (aa_last_valid_ && (rp > aa_rp_ || rd > aa_rd_)) aa_win_.clear();
  aa_last_valid_ = false;
  // active: primal feasible, penalties unchanged, the plain map contracting
  const bool contracting = rd < rd_prev;
  if (!(rp <= eps_abs + eps_rel * sp) || moved || !contracting) {
    aa_win_.clear();
    return PDNQP_OK;
  }
  launch_aa_pack(stream_, AG_ + aa_form_slot_ * len, v_.lam, v_.z, m, n);
  aa_win_.push_back(aa_form_slot_);
  while ((int)aa_win_.size() > st_.anderson_mem + 1) aa_win_.erase(aa_win_.begin());
  if (aa_win_.size() < 2) return PDNQP_OK;
  const int p = (int)aa_win_.size() - 1;
  AASlots sl{};
  for (int j = 0; j <= p; ++j) sl.s[j] = aa_win_[j];
  launch_aa_gram(stream_, ctrl_, AU_, AG_, len, sl, p, v_.partial);
  if ((r = read_ctrl(err))) return r;
  // unpack the upper triangle (kernel order) and the right-hand side
  double M[kAAMem][kAAMem], rhs[kAAMem];
  int k = 0;
  for (int i = 0; i < kAAMem; ++i)
    for (int j = i; j < kAAMem; ++j) {
      M[i][j] = M[j][i] = hctrl_->aa[k];
      ++k;
    }
  for (int i = 0; i < kAAMem; ++i) rhs[i] = hctrl_->aa[k++];
  double tr = 0.0;
  for (int i = 0; i < p; ++i) tr += M[i][i];
  const double tik = st_.anderson_reg * tr / p;
  for (int i = 0; i < p; ++i) M[i][i] += tik;
  // Gaussian elimination with partial pivoting; an exactly singular system
  // (all differences zero) gives gamma = 0, the plain point
  double g[kAAMem] = {0.0};
  bool singular = false;
  for (int c = 0; c < p && !singular; ++c) {
    int piv = c;
    for (int i = c + 1; i < p; ++i)
      if (std::fabs(M[i][c]) > std::fabs(M[piv][c])) piv = i;
    if (M[piv][c] == 0.0) {
      singular = true;
      break;
    }
    if (piv != c) {
      for (int j = 0; j < p; ++j) std::swap(M[c][j], M[piv][j]);
      std::swap(rhs[c], rhs[piv]);
    }
    for (int i = c + 1; i < p; ++i) {
      const double f = M[i][c] / M[c][c];
      for (int j = c; j < p; ++j) M[i][j] -= f * M[c][j];
      rhs[i] -= f * rhs[c];
    }
  }
  if (!singular) {
    for (int i = p - 1; i >= 0; --i) {
      double acc = rhs[i];
      for (int j = i + 1; j < p; ++j) acc -= M[i][j] * g[j];
      g[i] = acc / M[i][i];
    }
  }
  for (int j = 0; j < p; ++j) sl.gamma[j] = g[j];
  launch_aa_combine(stream_, AG_, len, sl, p, v_.lam, v_.z, lo_, hi_, qp_.me, m, n);
  // the inner dual warm start follows the extrapolated multipliers (y = -lambda)
  launch_elem(stream_, EL_NEG, v_.Y[hctrl_->cur], v_.lam, nullptr, 0.0, m);
  aa_last_valid_ = true;
  aa_rp_ = rp;
  aa_rd_ = rd;
  aa_steps_ += 1;
  return check(hipGetLastError(), "anderson kernels", err);
}

// ===========================================================================
// Learned controller parameters and the outer-step log.
// ===========================================================================
int Solver::set_controller(const float *theta, std::string &err) {
  if (!ctl_theta_) {
    ctl_theta_ = (float *)dalloc((size_t)PDNQP_MLP_PARAMS * 4);
    ctl_x_ = (float *)dalloc(PDNQP_FEATURES * 4);
    ctl_y_ = (float *)dalloc(16);
    if (!ctl_theta_ || !ctl_x_ || !ctl_y_) {
      err = "device allocation failed";
      return PDNQP_E_NOMEM;
    }
  }
  int r = check(hipMemcpyAsync(ctl_theta_, theta, (size_t)PDNQP_MLP_PARAMS * 4,
                               hipMemcpyHostToDevice, stream_),
                "controller upload", err);
  if (r) return r;
  r = check(hipStreamSynchronize(stream_), "controller upload", err);
  if (r) return r;
  ctl_loaded_ = true;
  return PDNQP_OK;
}

int Solver::outer_log(int32_t *steps, double *feat, double *rec) const {
  if (steps) *steps = log_n_;
  if (feat && log_n_)
    std::memcpy(feat, log_feat_.data(), (size_t)log_n_ * PDNQP_FEATURES * sizeof(double));
  if (rec && log_n_)
    std::memcpy(rec, log_rec_.data(), (size_t)log_n_ * PDNQP_OUTER_RECORD * sizeof(double));
  return PDNQP_OK;
}

}  // namespace pdnqp
