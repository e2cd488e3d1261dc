// Host driver of the gfx950 PDNQP solver: owns the device buffers of one QP
// and runs the practical outer iteration (paper, Section 3.2) around the
// device-resident inner PDHG (Section 3.3).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/pdnqp.h"
#include "pdnqp_kernels.hpp"

namespace pdnqp {

// Problem after row normalisation (host copy; int32 CSR, FP64 values).
struct HostQP {
  int32_t n = 0, m = 0, me = 0, mi = 0, m_orig = 0;
  std::vector<int32_t> Qp, Qi, Ap, Ai, ATp, ATi;
  std::vector<int32_t> ATperm;   // ATx[k] == Ax[ATperm[k]]
  std::vector<int32_t> Qop, Qoi;  // Q without its diagonal
  std::vector<double> Qox, Qdiag;
  std::vector<double> Qx, Ax, ATx;
  std::vector<double> c, xl, xu, b;
  std::vector<int32_t> row_of;   // original row of each internal row
  std::vector<double> sign_of;   // +1, or -1 for a negated upper-bound row
  // original data for the external check
  std::vector<int32_t> oAp, oAi;
  std::vector<double> oAx, orl, oru;
};

struct KernelTimer {
  std::string name;
  std::vector<hipEvent_t> ev;  // pairs
  int used = 0;
  int64_t launches = 0;
  double total_ms = 0.0;
  double bytes = 0.0;
};

class Solver {
 public:
  Solver() = default;
  ~Solver();
  // Returns PDNQP_OK or an error code (message in err).
  int init(HostQP &&qp, const pdnqp_settings &st, std::string &err);
  int solve(double eps_abs, double eps_rel, const double *x0, const double *lam0, double *x_out,
            double *lam_out, pdnqp_info *info, std::string &err);
  int trace(int32_t *iters, double *w, double *y, int32_t *trials, double *tr, int32_t *checks,
            int32_t *ck) const;
  int kernel_stats(pdnqp_kernel_stat *out, int32_t cap, int32_t *count) const;
  const HostQP &qp() const { return qp_; }
  int dw() const { return qp_.n + qp_.mi + qp_.m; }

 private:
  void *dalloc(size_t bytes);
  void dfree(void *p);
  int check(hipError_t e, const char *what, std::string &err);
  int setup(const double *x0c, const double *lam0_int, double &c_obj, double &gamma,
            double &lam_hat, std::string &err);
  template <typename T>
  int run_inner(double deadline, std::string &err, const IterVecs<T> &iv, const CsrT<T> &Qo,
                const CsrT<T> &A, const CsrT<T> &AT);
  IterVecs<double> iv64() const;
  void cast_state_to32(int cur);
  void cast_state_to64(int cur);
  int read_ctrl(std::string &err);
  void form_inner(double gamma);
  void ruiz_outer();
  double lanczos(std::string &err, bool &ok);
  void timed_launch(int which, const std::function<void()> &f);
  void harvest_timers();
  void external_check(const std::vector<double> &x, const std::vector<double> &lam,
                      pdnqp_info *info) const;

  HostQP qp_;
  pdnqp_settings st_{};
  hipStream_t stream_ = nullptr;
  bool own_stream_ = false;
  // device memory
  std::vector<void *> allocs_;
  Ctrl *ctrl_ = nullptr;
  Ctrl *hctrl_ = nullptr;  // pinned host mirror
  Vecs v_{};
  // raw and scaled matrices
  int32_t *Qp_ = nullptr, *Qi_ = nullptr, *Ap_ = nullptr, *Ai_ = nullptr, *ATp_ = nullptr,
          *ATi_ = nullptr;
  double *Qraw_ = nullptr, *Araw_ = nullptr, *ATraw_ = nullptr;
  double *Qv_ = nullptr, *Av_ = nullptr, *ATv_ = nullptr;
  int32_t *atperm_ = nullptr;
  int32_t *Qop_ = nullptr, *Qoi_ = nullptr;
  double *Qoraw_ = nullptr, *Qov_ = nullptr, *qdiag_raw_ = nullptr, *qdiag_ = nullptr;
  bool sample_now_ = false;
  int64_t slot_count_ = 0;
  double bE_norm_ = 0.0, bI_norm_ = 0.0, c_norm_ = 0.0;
  double *craw_ = nullptr, *xlraw_ = nullptr, *xuraw_ = nullptr, *braw_ = nullptr;
  double *c_ = nullptr, *lo_ = nullptr, *hi_ = nullptr, *b_ = nullptr;
  double *Fx2_ = nullptr, *Fs2_ = nullptr, *Fr2_ = nullptr, *E2buf_ = nullptr;
  Csr Q_{}, A_{}, AT_{}, Qr_{}, Ar_{}, ATr_{}, Qo_{};
  // FP32 bulk path
  bool fp32_ = false;
  IterVecs<float> iv32_{};
  CsrT<float> Qo32_{}, A32_{}, AT32_{};
  float *Qo32v_ = nullptr, *A32v_ = nullptr, *AT32v_ = nullptr;
  Part px_{}, ps_{}, pr_{}, pq_{}, pa_{}, pt_{};
  InnerParams ip_{};
  double gamma_ = 0.0;
  // trace buffers
  int32_t trace_iters_cap_ = 0, trace_trials_cap_ = 0;
  double *tw_ = nullptr, *ty_ = nullptr, *ttr_ = nullptr;
  int32_t *tck_ = nullptr;
  std::vector<double> h_tw_, h_ty_, h_ttr_;
  std::vector<int32_t> h_tck_;
  int32_t got_iters_ = 0, got_trials_ = 0, got_checks_ = 0;
  bool traced_ = false;
  // profiling
  std::vector<KernelTimer> timers_;
};

}  // namespace pdnqp
