// Device data structures and launch wrappers of the gfx950 PDNQP kernels.
//
// The inner QP (paper, eq. (inner-qp)) is iterated in its own coordinates
// w = (x, s_I, r_E, r_I), y = (y_E, y_I) -- outer-scaled, but neither
// penalty-scaled (eq. (inner-penalty-scaling)) nor inner-Ruiz-scaled.  Both
// of those scalings are diagonal changes of variables w = Sw * w_hat,
// y = Ey * y_hat; the PDHG trial step (pdqp-trial) taken in the scaled
// coordinates with steps tau_hat, eta_hat is exactly the step taken here
// with tau = Sw^2 tau_hat and eta = Ey^2 eta_hat, and the acceptance sums
// (adaptive-condition) are invariant under the change.  So the fixed CSR
// values of Q, A and A' are never rescaled per outer step; only the step
// vectors and the weights of the restart metric carry the scaling.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace pdnqp {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64s)
constexpr int kMaxParts = 4096;    // upper bound of reduction partials per launch
constexpr int kStreamE = 8;        // CSR-stream: nonzeros per thread per row block
constexpr int kTile = kStreamE * kBlock;  // CSR-stream: nonzeros per row block (2048)
// software-pipelined CSR-stream kernels (two row blocks in flight per
// workgroup): nonzeros per thread and per row block, and the default grid
// (measured at n = 1M: 4 nonzeros per thread is no faster; grids of 1024
// to 4096 tie in FP64, 1024 is fastest in FP32 and leaves the fewest
// partials to add; 512 is slower)
constexpr int kPipeE = 8;
constexpr int kPipeTile = kPipeE * kBlock;
constexpr int kPipeGrid = 1024;

enum State : int32_t {
  ST_RUNNING = 0,
  ST_CHECK_DUE = 1,
  ST_CONVERGED = 2,
  ST_NUMERR = 3,
  ST_ITER_LIMIT = 4,
  ST_PASS_LIMIT = 5,  // the KKT pass limit was reached at a check
};

// Ticket counters of the "last workgroup finishes the reduction" pattern.
enum Ticket : int {
  TK_XTRIAL = 0,
  TK_QA = 1,
  TK_AT = 2,
  TK_FLUSH = 3,
  TK_CHECK = 4,
  TK_TRACE = 5,
  TK_OUTER_ROWS = 6,
  TK_OUTER_COLS = 7,
  TK_GEN = 8,
  TK_APPLY = 9,
  TK_AA = 10,
  TK_COUNT = 16
};

// Device-resident control block: the state of the inner iteration that the
// kernels update without the host (accept/reject, counters, restart).
struct Ctrl {
  int32_t state;
  int32_t cur;         // index of the current buffer of each double-buffered vector
  int32_t N;           // accepted trials in this restart epoch
  int32_t t;           // accepted trials since the inner QP was formed
  int32_t t_call;      // accepted trials in this inner call
  int32_t rejects;     // consecutive rejected trials
  int32_t pending;     // averages owe the update with weight alpha_pend
  int32_t last_acc;    // last trial accepted
  int32_t restart_flag;
  int32_t copy_avg;    // the average candidate becomes the current iterate
  int32_t check_kind;  // 0 continue, 1 restart, 2 converged
  int32_t check_which; // 0 current, 1 average
  int32_t trace_iters_n;
  int32_t trace_trials_n;
  int32_t trace_checks_n;
  int32_t pad0;
  double alpha_pend;
  double step_scale;   // product of shrink factors since the last step rebuild
  double omega;        // primal weight
  double kkt_anchor;
  double kkt_prev;
  double L, R;         // last trial's acceptance sums
  double sum_x;        // x-block: sum dx^2 / taub_x
  double sum_row[4];   // row blocks: sum dw^2/taub, sum dy^2/etab, sum |dr sigma dr|, sum |dw (B'dy)|
  double chk[32];      // check reductions
  double outv[16];     // outer reductions
  double gen[8];       // general-purpose reductions (set-up)
  int64_t trials, accepted, rejected, restarts, checks;
  uint32_t ticket[TK_COUNT];
  int32_t pen_moved;   // set by the penalty update when a row penalty changed
  int32_t pad1;
  double aa[48];       // Anderson Gram matrix (upper triangle) and right-hand side
};

// Anderson acceleration (outer duals and centre): at most kAAMem + 1 stored
// points; the Gram system has at most kAAMem unknowns.
constexpr int kAAMem = 8;
constexpr int kAASums = kAAMem * (kAAMem + 1) / 2 + kAAMem;  // 44

// Read-only parameters of one inner QP, passed by value.
struct InnerParams {
  int32_t n, m, me, mi;
  int32_t check_every, max_inner, max_rejects, mode_init;
  int32_t trace_iters_cap, trace_trials_cap, dw;
  int32_t stream_grid;  // workgroups of the CSR-stream product launches (0: automatic)
  double gamma_inv;
  double delta_a, delta_r;
  double h_norm;       // ||h||_inf = ||b_E||_inf
  double shrink_safety, shrink_min, shrink_max;
  double restart_suff, restart_nec, restart_art;
  double pass_limit;   // KKT pass limit (cumulative trials of the solve)
};

template <typename T>
struct CsrT {
  const int32_t *p;
  const int32_t *i;
  const T *v;
  int32_t rows;
  int32_t G;           // lanes per row (power of two, 2..32) of the row-group kernels
  const int32_t *rb;   // CSR-stream row blocks: block b owns rows [rb[b], rb[b+1]) and
                       // nonzeros [rb[nrb+1+b], rb[nrb+2+b])
  int32_t nrb;         // number of row blocks
  int32_t pad;
};
using Csr = CsrT<double>;

// The vectors of the inner iteration, in the bulk type T (double for the
// FP64 path, float for the FP32-bulk path; the FP64 path aliases Vecs).
// Reductions and traces stay FP64.
template <typename T>
struct IterVecs {
  const T *lo, *hi, *b, *qdiag;
  T *sigma, *lam, *qx;
  T *taub_x, *taub_s, *taub_r, *etab;
  T *S2x, *S2s, *S2r, *E2;
  T *X[2], *QX[2], *ATY[2], *S[2], *R[2], *Y[2], *BW[2];
  T *xbar, *qxbar, *sbar, *rbar, *ybar;
  T *xa, *sa, *ra, *ya;
  T *axbar, *atybar;
  double *partial;
  double *trace_w, *trace_y, *trace_tr;
  int32_t *trace_ck;
};

// Row blocks for the CSR-stream kernels: consecutive rows whose nonzeros fit
// in one tile of kTile entries (a longer row gets a block of its own), at
// most max_rows rows per block.
void stream_row_blocks(const int32_t *rp, int32_t rows, int32_t max_rows, int32_t *out_nrb,
                       int32_t *rb /* capacity rows + 1 */, int32_t tile = kTile);

// Every device vector the kernels touch, passed by value.
struct Vecs {
  // outer-scaled problem data
  const double *c, *lo, *hi, *b;   // b: b_E on equality rows, b_I on inequality rows
  const double *qdiag;             // diagonal of the scaled Q (the hot Q product uses Q without it)
  // inner QP of the current outer step
  double *sigma, *lam, *z, *qx;    // qx = c - z / gamma
  double *taub_x, *taub_s, *taub_r, *etab;  // steps without omega and shrink factor
  double *S2x, *S2s, *S2r, *E2;    // squared scalings (restart metric weights)
  // iterate (double buffered: [cur] current, [1-cur] trial)
  double *X[2], *QX[2], *ATY[2], *S[2], *R[2], *Y[2], *BW[2];
  double *xbar, *qxbar, *sbar, *rbar, *ybar;
  double *xa, *sa, *ra, *ya;       // restart anchors
  double *axbar, *atybar;          // A xbar, A' ybar at checks
  // outer step
  double *ax, *rrow, *rprev, *atl, *qxo;
  // set-up
  double *Dx, *Dc, *Ex, *Fx, *Fs, *Fr, *tmp_n, *tmp_m;
  // reductions
  double *partial;                 // kMaxParts * 48 doubles
  // trace
  double *trace_w, *trace_y, *trace_tr;
  int32_t *trace_ck;
};

// Grid geometry of one row-partitioned part of a launch.
struct Part {
  int32_t rows;
  int32_t G;
  int32_t blocks;
};

Part make_part(int32_t rows, int32_t G, int32_t max_blocks);

// ---- inner iteration (templated on the bulk type; pdnqp_iter.hip) ----------
// Optional timing events of one launch: when set, the dispatch itself stamps
// its start and end into them (the same interval a kernel tracer reports).
struct LaunchEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
int xtrial_blocks(int n);
template <typename T>
void launch_xtrial(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
                   LaunchEvents ev = {});
// Qoff: Q without its diagonal (the diagonal is v.qdiag)
template <typename T>
void launch_qa(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
               const CsrT<T> &Qoff, const CsrT<T> &A, LaunchEvents ev = {});
// A' product and x-block sums; pq0/pq1 (the two-panel form's Q partial
// sums, or null) make its epilogue form Q x_tr as well
template <typename T>
void launch_at(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
               const CsrT<T> &AT, LaunchEvents ev = {}, const T *pq0 = nullptr,
               const T *pq1 = nullptr);
// Two-panel form of launch_qa: Q_off and A split by columns at n/2, each
// half a CSR over all rows with its own stream row blocks, and the per-row
// partial sums of each half (device buffers of n and m values).
template <typename T>
struct QAPanelSet {
  CsrT<T> q[2], a[2];
  T *pq[2], *pa[2];
};
template <typename T>
void launch_qa_panels(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
                      const QAPanelSet<T> &P, LaunchEvents ev = {});
template <typename T>
void launch_qa_rows(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
                    const QAPanelSet<T> &P, LaunchEvents ev = {});
// acceptance test of the trial (one workgroup), after launch_at; the row
// block counts of Q_off, A and A' give the partial counts of the launches
// before it; `panels`: the row part of the sums came from launch_qa_rows
void launch_decide(hipStream_t st, Ctrl *c, const InnerParams &p, const double *partial,
                   double *trace_tr, int q_nrb, int a_nrb, int at_nrb, LaunchEvents ev = {},
                   bool panels = false);
template <typename T>
void launch_trace(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v);
template <typename T>
void launch_flush(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
                  const Part &px, const Part &pr);
template <typename T>
void launch_check_spmv(hipStream_t st, Ctrl *c, const IterVecs<T> &v, const CsrT<T> &A,
                       const CsrT<T> &AT, const Part &pa, const Part &pt);
template <typename T>
void launch_check(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
                  const Part &px, const Part &ps, const Part &pr);
template <typename T>
void launch_apply(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
                  const Part &px, const Part &pr);
template <typename T>
void launch_inner_init(hipStream_t st, Ctrl *c, const InnerParams &p, const IterVecs<T> &v,
                       const CsrT<T> &Qoff, const CsrT<T> &AT, const Part &pr);
template <typename D, typename S>
void launch_cast(hipStream_t st, D *dst, const S *src, int64_t n);

// ---- inner QP formation (FP64) ---------------------------------------------
void launch_inner_ruiz_sweep(hipStream_t st, const InnerParams &p, const Vecs &v, const Csr &A,
                             const Csr &AT, const Part &pa, const Part &pt, double *Fx_new,
                             double *Fs_new, double *Fr_new, double *E_new);
void launch_steps(hipStream_t st, const InnerParams &p, const Vecs &v, const Csr &Q,
                  const Csr &A, const Csr &AT, double gamma_inv, double boost);
void launch_warm(hipStream_t st, const InnerParams &p, const Vecs &v, int cur, double gamma);

// ---- outer step --------------------------------------------------------------
// The caller's (unscaled) data in internal row order, for the external KKT
// test inside the outer loop: right-hand sides b, variable bounds, linear
// term, and the objective scalar of the outer scaling.
struct RawData {
  const double *b, *xl, *xu, *c;
  double c_obj;
};
void launch_outer_rows(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v,
                       const Csr &A, const Part &pa, const RawData &raw);
void launch_outer_cols(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v,
                       const Csr &Q, const Csr &AT, const Part &pq, const RawData &raw);
void launch_penalty(hipStream_t st, Ctrl *c, const InnerParams &p, const Vecs &v,
                    const Part &pr, int have_prev, double rnorm, double theta, double growth,
                    double sig_max, int gate, double gate_tol);
void launch_copy(hipStream_t st, double *dst, const double *src, int32_t n);
// min, sum and max of sigma (m > 0) into c->gen[5..7]
void launch_sigma_stats(hipStream_t st, Ctrl *c, const double *sig, int32_t m, double *partial);
// Anderson: dst = (lam, z); Gram of the residual differences of the points
// slot[0..p] (oldest first) of the histories U, G (row stride len);
// combination G_p - sum gamma_j (G_{j+1} - G_j) into (lam, z) with
// lam_I <= 0 and z in [lo, hi].
void launch_aa_pack(hipStream_t st, double *dst, const double *lam, const double *z, int32_t m,
                    int32_t n);
struct AASlots {
  int32_t s[kAAMem + 1];
  double gamma[kAAMem];
};
void launch_aa_gram(hipStream_t st, Ctrl *c, const double *U, const double *G, int64_t len,
                    const AASlots &sl, int p, double *partial);
void launch_aa_combine(hipStream_t st, const double *G, int64_t len, const AASlots &sl, int p,
                       double *lam, double *z, const double *lo, const double *hi, int32_t me,
                       int32_t m, int32_t n);
void launch_fill(hipStream_t st, double *dst, double val, int32_t n);

// ---- set-up ----------------------------------------------------------------
// out[r] = max_k |M_rk| * wcol[k] * wrow[r]   (row infinity norms of a scaled matrix)
void launch_row_absmax(hipStream_t st, const Csr &M, const double *wrow, const double *wcol,
                       double *out, const Part &pm);
// out[r] = sum_k |M_rk|
void launch_row_abssum(hipStream_t st, const Csr &M, double *out, const Part &pm);
// Dc /= sqrt(rn), Dx /= sqrt(max(cn, cnq)) (zero norms keep the scale; cnq may be NULL)
void launch_ruiz_update(hipStream_t st, double *Dc, const double *rn, int32_t m, double *Dx,
                        const double *cn, const double *cnq, int32_t n);
enum ElemOp : int { EL_GRAD = 0, EL_MULS = 1, EL_DIV = 2, EL_MUL = 3, EL_SCALE_DIV = 4,
                    EL_NEG = 5, EL_AXPBY = 6, EL_DIVINTO = 7, EL_DIAG = 8 };
void launch_elem(hipStream_t st, int op, double *a, const double *b, const double *c, double s,
                 int32_t n);
// out[j] = A x0 - P_C(A x0) from v.ax
void launch_viol(hipStream_t st, const InnerParams &p, const Vecs &v, double *out);
// dst[k] = src[perm[k]]
void launch_gather(hipStream_t st, double *dst, const double *src, const int32_t *perm, int64_t n);
// y = alpha * M x (plain SpMV)
void launch_spmv(hipStream_t st, const Csr &M, const double *x, double *y, double alpha,
                 const Part &pm);
// scale CSR values in place: v_rk = s * wrow[r] * v_rk * wcol[k]
void launch_scale_csr(hipStream_t st, const int32_t *p, const int32_t *i, double *v, int32_t rows,
                      const double *wrow, const double *wcol, double s, const Part &pm);
// deterministic reductions into ctrl->gen[slot]: sum a.b, sum a^2, max |a|
void launch_dot(hipStream_t st, Ctrl *c, const double *a, const double *b, int32_t n, int slot,
                double *partial);
void launch_absmax(hipStream_t st, Ctrl *c, const double *a, int32_t n, int slot,
                   double *partial);
// Lanczos three-term update: w <- w - alpha v - beta_prev v_prev (alpha from ctrl->gen[0]),
// then ctrl->gen[1] = ||w||^2
void launch_lanczos_update(hipStream_t st, Ctrl *c, double *w, const double *v,
                           const double *vprev, double beta_prev, int32_t n, double *partial);

}  // namespace pdnqp
