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
#include "pdnqp_batch.hpp"
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

// What a solve reports besides the vectors (filled by either path).
struct Outcome {
  int status = PDNQP_MAX_ITER;
  int64_t outer_iters = 0, trials = 0, accepted = 0, rejected = 0, restarts = 0, checks = 0;
  double rp = 0, rd = 0, sp = 0, sd = 0, gamma = 0, lam_hat = 0, omega = 0, c_obj = 1;
  double setup_s = 0;
  int32_t trace_iters = 0, trace_trials = 0, trace_checks = 0;
  int32_t anderson_steps = 0;
  int32_t controller_fallback = 0;
  int32_t promoted_outer = 0;
  int32_t halvings = 0;
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
  int precision() const { return st_.precision; }
  int device() const { return device_; }
  hipStream_t stream() const { return stream_; }
  // Batched path: fills the instance descriptor (uploads the start point,
  // builds the row blocks of the launch's tile) and, after the kernel,
  // copies the result back like solve does.
  int batch_prepare(double eps_abs, double eps_rel, const double *x0, const double *lam0,
                    int block, double ticks_per_s, BatchOut *dev_out, BatchInst &bi,
                    std::string &err);
  int batch_finish(const BatchOut &o, double ticks_per_s, double *x_out, double *lam_out,
                   pdnqp_info *info, std::string &err);

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
  void timed_launch(int which, const std::function<void(LaunchEvents)> &f);
  void harvest_timers();
  void external_check(const std::vector<double> &x, const std::vector<double> &lam,
                      pdnqp_info *info) const;
  int begin(const double *x0, const double *lam0, std::vector<double> &x0c,
            std::vector<double> &lam0i, std::string &err);
  int finish(const Outcome &oc, double *x_out, double *lam_out, pdnqp_info *info,
             std::string &err);

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
  bool bulk32_ = false;  // this outer step's inner iteration runs in FP32 (fp32_ until promoted)
  IterVecs<float> iv32_{};
  CsrT<float> Qo32_{}, A32_{}, AT32_{};
  float *Qo32v_ = nullptr, *A32v_ = nullptr, *AT32v_ = nullptr;
  // two-column-panel form of the first trial product (settings.col_panels):
  // per precision whether it is used, the panels (values gathered from the
  // scaled Q_off and A through the permutations) and the partial sums
  bool panels64_ = false, panels32_ = false;
  QAPanelSet<double> qap64_{};
  QAPanelSet<float> qap32_{};
  int32_t *pperm_q_[2] = {nullptr, nullptr}, *pperm_a_[2] = {nullptr, nullptr};
  int64_t pnnz_q_[2] = {0, 0}, pnnz_a_[2] = {0, 0};
  template <typename T>
  bool use_panels() const;
  template <typename T>
  const QAPanelSet<T> &panel_set() const;
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
  int64_t chunk_count_ = 0;
  // captured chunk of the current outer step (settings.graph)
  hipGraphExec_t gexec_ = nullptr;
  hipStream_t cap_stream_ = nullptr;
  bool graph_valid_ = false;
  template <typename T>
  void enqueue_chunk(int slots, bool sampled, const IterVecs<T> &iv, const CsrT<T> &Qo,
                     const CsrT<T> &A, const CsrT<T> &AT);
  template <typename T>
  int capture_chunk(std::string &err, const IterVecs<T> &iv, const CsrT<T> &Qo, const CsrT<T> &A,
                    const CsrT<T> &AT);
  // batched path: row blocks per tile size (Q, Q_off, A, A'), Lanczos coefficients
  struct BatchBlocks {
    int block = 0;
    int32_t *q = nullptr, *qo = nullptr, *a = nullptr, *at = nullptr;
    int32_t nq = 0, nqo = 0, na = 0, nat = 0;
  };
  std::vector<BatchBlocks> bblocks_;
  double *lz_ = nullptr;
  int device_ = 0;
  // Anderson acceleration: histories of points and images, (anderson_mem + 2)
  // slots of (lambda, z) each; the window lists the slots in use, oldest first
  double *AU_ = nullptr, *AG_ = nullptr;
  std::vector<int> aa_win_;
  int aa_form_slot_ = 0;
  bool aa_last_valid_ = false;
  double aa_rp_ = 0.0, aa_rd_ = 0.0;
  int aa_steps_ = 0;
  void anderson_form();
  // learned controller (settings.controller) and the outer-step log
  float *ctl_theta_ = nullptr, *ctl_x_ = nullptr, *ctl_y_ = nullptr;
  bool ctl_loaded_ = false;
  std::vector<double> log_feat_, log_rec_;
  int32_t log_n_ = 0;

 public:
  int set_controller(const float *theta, std::string &err);
  int outer_log(int32_t *steps, double *feat, double *rec) const;

 private:
  int anderson(double rp, double rd, double sp, double eps_abs, double eps_rel, double rd_prev,
               std::string &err);
};

// The controller network (pdnqp_mlp.hip).
void mlp_forward_device(hipStream_t st, const float *theta, const float *x, float *y);
int mlp_forward(const float *theta, const float *X, int count, float *Y, std::string &err);
int mlp_gradient(const float *theta, const float *X, const float *Y, int count, float *grad,
                 double *loss, std::string &err);
int mlp_gradient_noalloc(const float *theta, const float *X, const float *Y, int count,
                         float *grad, double *loss, hipStream_t st, std::string &err);
int probe_gather(int32_t vec_len, int32_t elem_bytes, int64_t gathers, int32_t panels,
                 int32_t reps, uint64_t seed, double *rate, double *launch_us, std::string &err);
int mlp_train(float *theta, const float *X, const float *Y, int count, int epochs, int batch,
              float lr, uint64_t seed, float *loss_curve, std::string &err);

// Batched persistent solve over several handles (pdnqp_batch_host.cpp).
struct BatchRequest {
  std::vector<Solver *> solvers;
  double eps_abs = 1e-4, eps_rel = 1e-4;
  double *const *x_out = nullptr;
  double *const *lam_out = nullptr;
  pdnqp_info *infos = nullptr;
  int config = -1;      // launch configuration index; -1: tuned or default
  int probe_inner = 0;  // > 0: tuning probe (one outer step, this many inner iterations)
};
int run_batch(const BatchRequest &req, pdnqp_batch_report *rep, std::vector<double> *done_ms,
              std::string &err);
int autotune_batch(const BatchRequest &req, int32_t *block_out, int32_t *waves_out,
                   double *ms_out, std::string &err);
int set_batch_config(int block, int waves);

}  // namespace pdnqp
