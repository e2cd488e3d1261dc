// C ABI of the PDNQP library: argument validation, row normalisation into
// the paper's form (A_E x = b_E, A_I x >= b_I; Section 2, problem (qp)),
// and forwarding to the device solver.
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "../../include/pdnqp.h"
#include "pdnqp_solver.hpp"

struct pdnqp_solver {
  pdnqp::Solver s;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

bool check_csr(int32_t rows, int32_t cols, const int32_t *p, const int32_t *idx, const double *val,
               const char *name, std::string &err) {
  if (!p) {
    err = std::string(name) + ": row pointer array is NULL";
    return false;
  }
  if (p[0] != 0) {
    err = std::string(name) + ": row pointers must start at 0";
    return false;
  }
  for (int32_t r = 0; r < rows; ++r) {
    if (p[r + 1] < p[r]) {
      err = std::string(name) + ": row pointers decrease at row " + std::to_string(r);
      return false;
    }
  }
  const int32_t nnz = p[rows];
  if (nnz > 0 && (!idx || !val)) {
    err = std::string(name) + ": index or value array is NULL";
    return false;
  }
  for (int32_t r = 0; r < rows; ++r) {
    for (int32_t k = p[r]; k < p[r + 1]; ++k) {
      const int32_t c = idx[k];
      if (c < 0 || c >= cols) {
        err = std::string(name) + ": column index out of range in row " + std::to_string(r);
        return false;
      }
      if (k > p[r] && c <= idx[k - 1]) {
        err = std::string(name) + ": column indices not strictly increasing in row " +
              std::to_string(r);
        return false;
      }
      if (!std::isfinite(val[k])) {
        err = std::string(name) + ": non-finite value in row " + std::to_string(r);
        return false;
      }
    }
  }
  return true;
}

// CSR transpose by counting; perm[k] is the position in the input of the
// k-th entry of the output.
void transpose(int32_t rows, int32_t cols, const int32_t *p, const int32_t *idx, const double *val,
               std::vector<int32_t> &tp, std::vector<int32_t> &ti, std::vector<double> &tv,
               std::vector<int32_t> &perm) {
  const int32_t nnz = p[rows];
  tp.assign(cols + 1, 0);
  ti.resize(nnz);
  tv.resize(nnz);
  perm.resize(nnz);
  for (int32_t k = 0; k < nnz; ++k) tp[idx[k] + 1] += 1;
  for (int32_t c = 0; c < cols; ++c) tp[c + 1] += tp[c];
  std::vector<int32_t> next(tp.begin(), tp.end() - 1);
  for (int32_t r = 0; r < rows; ++r) {
    for (int32_t k = p[r]; k < p[r + 1]; ++k) {
      const int32_t dst = next[idx[k]]++;
      ti[dst] = r;
      tv[dst] = val[k];
      perm[dst] = k;
    }
  }
}

}  // namespace

extern "C" {

void pdnqp_default_settings(pdnqp_settings *s) {
  if (!s) return;
  std::memset(s, 0, sizeof(*s));
  s->max_outer = 2147483647LL;
  s->max_inner = 40000;
  s->ruiz_sweeps = 8;
  s->time_limit_s = std::numeric_limits<double>::infinity();
  s->sigma_init = 20.0;
  s->theta_sigma = 0.25;
  s->delta_gamma = 1e-2;
  s->rho_in_min = 0.3;
  s->rho_in_max = 0.95;
  s->rho_z = 0.95;
  s->check_every = 64;
  s->max_rejects = 50;
  s->restart_suff = 0.2;
  s->restart_nec = 0.8;
  s->restart_art = 0.36;
  s->shrink_safety = 0.95;
  s->shrink_min = 0.1;
  s->shrink_max = 0.9;
  s->omega0 = 1.0;
  s->sigma_growth = 10.0;
  s->sigma_max = 1e4;
  s->sigma0_min = 1e-4;
  s->sigma0_max = 1e4;
  s->penalty_gate = 1;
  s->center_floor = 1;
  s->lanczos_iters = 100;
  s->gamma_override = 0.0;
  s->step_boost = 1.0;
  s->outer_scaling = PDNQP_SCALE_RUIZ_A;
  s->anderson_mem = 0;
  s->anderson_reg = 1e-10;
  s->fp32_promote = 1e-5;
  s->delta_floor = 1.0;
  s->fp32_stall = 50;
  s->external_halvings = 7;
  s->delta0 = 1.0;
  s->kkt_pass_limit = std::numeric_limits<double>::infinity();
}

size_t pdnqp_settings_size(void) { return sizeof(pdnqp_settings); }
size_t pdnqp_info_size(void) { return sizeof(pdnqp_info); }

int pdnqp_create(pdnqp_solver **out, int32_t n, int32_t m, const int32_t *Qp, const int32_t *Qi,
                 const double *Qx, const int32_t *Ap, const int32_t *Ai, const double *Ax,
                 const double *c, const double *xl, const double *xu, const double *rl,
                 const double *ru, const pdnqp_settings *settings) {
  g_err.clear();
  if (!out) return fail(PDNQP_E_INVALID, "out is NULL");
  *out = nullptr;
  try {
    if (n < 1) return fail(PDNQP_E_INVALID, "n must be >= 1");
    if (m < 0) return fail(PDNQP_E_INVALID, "m must be >= 0");
    if (!c || !xl || !xu) return fail(PDNQP_E_INVALID, "c, xl, xu must not be NULL");
    if (m > 0 && (!rl || !ru)) return fail(PDNQP_E_INVALID, "rl, ru must not be NULL when m > 0");
    pdnqp_settings st;
    if (settings) st = *settings;
    else pdnqp_default_settings(&st);
    if (st.ruiz_sweeps < 0 || st.check_every < 1 || st.max_inner < 1 || st.max_rejects < 1 ||
        st.max_outer < 0 || st.lanczos_iters < 1 || !(st.omega0 > 0) || !(st.sigma_init > 0) ||
        !(st.delta_gamma > 0) || !(st.step_boost > 0) || st.outer_scaling < 0 ||
        st.outer_scaling > 2 || st.trace_iters < 0 || st.trace_trials < 0 ||
        (st.precision != PDNQP_FP64 && st.precision != PDNQP_FP32) ||
        (st.graph != 0 && st.graph != 1) || st.anderson_mem < 0 ||
        st.anderson_mem > PDNQP_ANDERSON_MAX || !(st.anderson_reg >= 0) ||
        (st.controller != 0 && st.controller != 1) || st.outer_log < 0 ||
        !(st.fp32_promote >= 0) || !(st.delta_floor >= 0) || !std::isfinite(st.delta_floor) ||
        st.fp32_stall < 0 || st.external_halvings < 0 || st.external_halvings > 30 ||
        !(st.delta0 > 0) || !std::isfinite(st.delta0) || st.col_panels < 0 || st.col_panels > 2 ||
        st.stream_grid < 0 || st.stream_grid == 1 || st.stream_grid > 4096 ||
        !(st.kkt_pass_limit >= 1.0))
      return fail(PDNQP_E_INVALID, "invalid settings value");
    std::string err;
    if (!check_csr(n, n, Qp, Qi, Qx, "Q", err)) return fail(PDNQP_E_INVALID, err);
    if (!check_csr(m, n, Ap, Ai, Ax, "A", err)) return fail(PDNQP_E_INVALID, err);
    // Q must be symmetric (both triangles stored, equal values)
    {
      std::vector<int32_t> tp, ti, perm;
      std::vector<double> tv;
      transpose(n, n, Qp, Qi, Qx, tp, ti, tv, perm);
      for (int32_t k = 0; k < Qp[n]; ++k) {
        if (ti[k] != Qi[k] || tv[k] != Qx[k]) return fail(PDNQP_E_INVALID, "Q is not symmetric");
      }
      for (int32_t r = 0; r <= n; ++r)
        if (tp[r] != Qp[r]) return fail(PDNQP_E_INVALID, "Q is not symmetric");
    }
    for (int32_t i = 0; i < n; ++i) {
      if (!std::isfinite(c[i])) return fail(PDNQP_E_INVALID, "c has a non-finite entry");
      if (std::isnan(xl[i]) || std::isnan(xu[i]) || xl[i] > xu[i] || xl[i] == INFINITY ||
          xu[i] == -INFINITY)
        return fail(PDNQP_E_INVALID, "invalid variable bounds at index " + std::to_string(i));
    }
    pdnqp::HostQP qp;
    qp.n = n;
    qp.m_orig = m;
    std::vector<int32_t> erows, irows;
    std::vector<double> isign, ib;
    for (int32_t j = 0; j < m; ++j) {
      const double lo = rl[j], hi = ru[j];
      if (std::isnan(lo) || std::isnan(hi) || lo > hi || lo == INFINITY || hi == -INFINITY)
        return fail(PDNQP_E_INVALID, "invalid row bounds at row " + std::to_string(j));
      if (lo == hi) {
        erows.push_back(j);
        continue;
      }
      if (std::isfinite(lo)) {
        irows.push_back(j);
        isign.push_back(1.0);
        ib.push_back(lo);
      }
      if (std::isfinite(hi)) {
        irows.push_back(j);
        isign.push_back(-1.0);
        ib.push_back(-hi);
      }
    }
    qp.me = (int32_t)erows.size();
    qp.mi = (int32_t)irows.size();
    qp.m = qp.me + qp.mi;
    qp.Ap.assign(1, 0);
    auto add_row = [&](int32_t j, double sg) {
      for (int32_t k = Ap[j]; k < Ap[j + 1]; ++k) {
        qp.Ai.push_back(Ai[k]);
        qp.Ax.push_back(sg * Ax[k]);
      }
      qp.Ap.push_back((int32_t)qp.Ai.size());
    };
    for (int32_t j : erows) {
      add_row(j, 1.0);
      qp.row_of.push_back(j);
      qp.sign_of.push_back(1.0);
      qp.b.push_back(rl[j]);
    }
    for (size_t t = 0; t < irows.size(); ++t) {
      add_row(irows[t], isign[t]);
      qp.row_of.push_back(irows[t]);
      qp.sign_of.push_back(isign[t]);
      qp.b.push_back(ib[t]);
    }
    if ((int64_t)qp.Ai.size() > 2147483647LL)
      return fail(PDNQP_E_INVALID, "too many nonzeros after row splitting");
    transpose(qp.m, n, qp.Ap.data(), qp.Ai.data(), qp.Ax.data(), qp.ATp, qp.ATi, qp.ATx,
              qp.ATperm);
    qp.Qp.assign(Qp, Qp + n + 1);
    qp.Qi.assign(Qi, Qi + Qp[n]);
    qp.Qx.assign(Qx, Qx + Qp[n]);
    qp.c.assign(c, c + n);
    qp.xl.assign(xl, xl + n);
    qp.xu.assign(xu, xu + n);
    qp.oAp.assign(Ap, Ap + m + 1);
    qp.oAi.assign(Ai, Ai + Ap[m]);
    qp.oAx.assign(Ax, Ax + Ap[m]);
    if (m) {
      qp.orl.assign(rl, rl + m);
      qp.oru.assign(ru, ru + m);
    }
    pdnqp_solver *h = new pdnqp_solver();
    const int r = h->s.init(std::move(qp), st, err);
    if (r != PDNQP_OK) {
      delete h;
      return fail(r, err);
    }
    *out = h;
    return PDNQP_OK;
  } catch (const std::bad_alloc &) {
    return fail(PDNQP_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(PDNQP_E_DEVICE, "unexpected exception");
  }
}

int pdnqp_solve(pdnqp_solver *s, double eps_abs, double eps_rel, const double *x0,
                const double *lambda0, double *x_out, double *lambda_out, pdnqp_info *info) {
  g_err.clear();
  if (!s) return fail(PDNQP_E_INVALID, "solver is NULL");
  if (!(eps_abs >= 0) || !(eps_rel >= 0) || !std::isfinite(eps_abs) || !std::isfinite(eps_rel))
    return fail(PDNQP_E_INVALID, "tolerances must be finite and >= 0");
  if (!x_out) return fail(PDNQP_E_INVALID, "x_out is NULL");
  if (s->s.qp().m_orig > 0 && !lambda_out) return fail(PDNQP_E_INVALID, "lambda_out is NULL");
  if (x0)
    for (int32_t i = 0; i < s->s.qp().n; ++i)
      if (!std::isfinite(x0[i])) return fail(PDNQP_E_INVALID, "x0 has a non-finite entry");
  if (lambda0)
    for (int32_t j = 0; j < s->s.qp().m_orig; ++j)
      if (!std::isfinite(lambda0[j])) return fail(PDNQP_E_INVALID, "lambda0 has a non-finite entry");
  try {
    std::string err;
    const int r = s->s.solve(eps_abs, eps_rel, x0, lambda0, x_out, lambda_out, info, err);
    if (r != PDNQP_OK) return fail(r, err);
    return PDNQP_OK;
  } catch (const std::bad_alloc &) {
    return fail(PDNQP_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(PDNQP_E_DEVICE, "unexpected exception");
  }
}

namespace {
thread_local pdnqp_batch_report g_batch_report{};
thread_local std::vector<double> g_batch_done;

int batch_request(int32_t count, pdnqp_solver *const *solvers, pdnqp::BatchRequest &req) {
  if (count < 0) return fail(PDNQP_E_INVALID, "count must be >= 0");
  if (count > 0 && !solvers) return fail(PDNQP_E_INVALID, "NULL array argument");
  req.solvers.resize(count);
  for (int32_t k = 0; k < count; ++k) {
    if (!solvers[k]) return fail(PDNQP_E_INVALID, "solver " + std::to_string(k) + " is NULL");
    for (int32_t j = 0; j < k; ++j)
      if (solvers[j] == solvers[k])
        return fail(PDNQP_E_INVALID, "the same handle appears twice in the batch");
    req.solvers[k] = &solvers[k]->s;
  }
  return PDNQP_OK;
}
}  // namespace

int pdnqp_solve_batch(int32_t count, pdnqp_solver *const *solvers, double eps_abs, double eps_rel,
                      double *const *x_out, double *const *lambda_out, pdnqp_info *infos) {
  g_err.clear();
  if (!(eps_abs >= 0) || !(eps_rel >= 0) || eps_abs + eps_rel <= 0)
    return fail(PDNQP_E_INVALID, "tolerances must be >= 0 and not both 0");
  if (count > 0 && (!x_out || !lambda_out)) return fail(PDNQP_E_INVALID, "NULL array argument");
  pdnqp::BatchRequest req;
  int r = batch_request(count, solvers, req);
  if (r) return r;
  for (int32_t k = 0; k < count; ++k)
    if (!x_out[k] || (!lambda_out[k] && solvers[k]->s.qp().m_orig > 0))
      return fail(PDNQP_E_INVALID, "NULL output buffer for instance " + std::to_string(k));
  req.eps_abs = eps_abs;
  req.eps_rel = eps_rel;
  req.x_out = x_out;
  req.lam_out = lambda_out;
  req.infos = infos;
  std::string err;
  r = pdnqp::run_batch(req, &g_batch_report, &g_batch_done, err);
  if (r) return fail(r, err);
  return PDNQP_OK;
}

int pdnqp_batch_last_report(pdnqp_batch_report *rep, double *done_ms, int32_t cap) {
  if (rep) *rep = g_batch_report;
  if (done_ms)
    for (int32_t i = 0; i < cap && i < (int32_t)g_batch_done.size(); ++i) done_ms[i] = g_batch_done[i];
  return PDNQP_OK;
}

int pdnqp_batch_set_config(int32_t block, int32_t waves) {
  g_err.clear();
  if (pdnqp::set_batch_config(block, waves) != PDNQP_OK)
    return fail(PDNQP_E_INVALID,
                "configuration must be (256,1), (512,1), (1024,1), (256,4), (512,4) or block 0");
  return PDNQP_OK;
}

int pdnqp_batch_autotune(int32_t count, pdnqp_solver *const *solvers, int32_t probe_inner,
                         int32_t *block_out, int32_t *waves_out, double *ms_out) {
  g_err.clear();
  if (count < 1) return fail(PDNQP_E_INVALID, "count must be >= 1");
  if (probe_inner < 1) return fail(PDNQP_E_INVALID, "probe_inner must be >= 1");
  pdnqp::BatchRequest req;
  int r = batch_request(count, solvers, req);
  if (r) return r;
  req.probe_inner = probe_inner;
  std::string err;
  r = pdnqp::autotune_batch(req, block_out, waves_out, ms_out, err);
  if (r) return fail(r, err);
  return PDNQP_OK;
}

int pdnqp_mlp_forward(const float *theta, const float *x, int32_t count, float *y) {
  g_err.clear();
  if (count < 1 || !theta || !x || !y) return fail(PDNQP_E_INVALID, "invalid network arguments");
  std::string err;
  const int r = pdnqp::mlp_forward(theta, x, count, y, err);
  return r ? fail(r, err) : PDNQP_OK;
}

int pdnqp_mlp_gradient(const float *theta, const float *x, const float *y, int32_t count,
                       float *grad, double *loss) {
  g_err.clear();
  if (count < 1 || !theta || !x || !y || !grad)
    return fail(PDNQP_E_INVALID, "invalid network arguments");
  std::string err;
  const int r = pdnqp::mlp_gradient(theta, x, y, count, grad, loss, err);
  return r ? fail(r, err) : PDNQP_OK;
}

int pdnqp_mlp_gradient_noalloc(const float *theta, const float *x, const float *y, int32_t count,
                               float *grad, double *loss, void *hip_stream) {
  g_err.clear();
  if (!theta || !x || !y || !grad) return fail(PDNQP_E_INVALID, "invalid network arguments");
  std::string err;
  const int r = pdnqp::mlp_gradient_noalloc(theta, x, y, count, grad, loss,
                                            (hipStream_t)hip_stream, err);
  return r ? fail(r, err) : PDNQP_OK;
}

int pdnqp_probe_gather(int32_t vec_len, int32_t elem_bytes, int64_t gathers, int32_t panels,
                       int32_t reps, uint64_t seed, double *gathers_per_s, double *launch_us) {
  g_err.clear();
  std::string err;
  const int r = pdnqp::probe_gather(vec_len, elem_bytes, gathers, panels, reps, seed,
                                    gathers_per_s, launch_us, err);
  return r ? fail(r, err) : PDNQP_OK;
}

int pdnqp_mlp_train(float *theta, const float *x, const float *y, int32_t count, int32_t epochs,
                    int32_t batch, float lr, uint64_t seed, float *loss_curve) {
  g_err.clear();
  if (count < 1 || epochs < 0 || batch < 1 || !(lr > 0) || !theta || !x || !y)
    return fail(PDNQP_E_INVALID, "invalid training arguments");
  std::string err;
  const int r = pdnqp::mlp_train(theta, x, y, count, epochs, batch, lr, seed, loss_curve, err);
  return r ? fail(r, err) : PDNQP_OK;
}

int pdnqp_set_controller(pdnqp_solver *s, const float *theta) {
  g_err.clear();
  if (!s || !theta) return fail(PDNQP_E_INVALID, "solver or parameters NULL");
  std::string err;
  const int r = s->s.set_controller(theta, err);
  return r ? fail(r, err) : PDNQP_OK;
}

int pdnqp_get_outer_log(const pdnqp_solver *s, int32_t *steps, double *features, double *record) {
  g_err.clear();
  if (!s) return fail(PDNQP_E_INVALID, "solver is NULL");
  return s->s.outer_log(steps, features, record);
}

void pdnqp_destroy(pdnqp_solver *s) { delete s; }

const char *pdnqp_last_error(void) { return g_err.c_str(); }

int pdnqp_dims(const pdnqp_solver *s, int32_t *m_e, int32_t *m_i, int32_t *d_w) {
  if (!s) return fail(PDNQP_E_INVALID, "solver is NULL");
  if (m_e) *m_e = s->s.qp().me;
  if (m_i) *m_i = s->s.qp().mi;
  if (d_w) *d_w = s->s.dw();
  return PDNQP_OK;
}

int pdnqp_get_trace(const pdnqp_solver *s, int32_t *iters, double *w, double *y, int32_t *trials,
                    double *tr, int32_t *checks, int32_t *ck) {
  if (!s) return fail(PDNQP_E_INVALID, "solver is NULL");
  const int r = s->s.trace(iters, w, y, trials, tr, checks, ck);
  if (r != PDNQP_OK) return fail(r, "no trace recorded (set trace_iters / trace_trials)");
  return PDNQP_OK;
}

int pdnqp_kernel_stats(const pdnqp_solver *s, pdnqp_kernel_stat *out, int32_t cap,
                       int32_t *count) {
  if (!s) return fail(PDNQP_E_INVALID, "solver is NULL");
  return s->s.kernel_stats(out, cap, count);
}

}  // extern "C"
