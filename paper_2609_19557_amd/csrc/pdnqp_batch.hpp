// Batched persistent solve of many independent PDNQP instances.
//
// One workgroup runs the whole method for one instance at a time (outer
// scaling, Lanczos proximal step, initial penalties, then the outer loop of
// Algorithm "practical outer iteration" with its inner rAPDHG solves) and
// takes the next instance from a device queue when it finishes.  The
// instances' data are the buffers their solver handles already hold; a
// BatchInst descriptor lists them.
#pragma once

#include "../../include/pdnqp.h"
#include "pdnqp_kernels.hpp"

namespace pdnqp {

// CSR structure with its stream row blocks for the tile size of the launch.
struct BCsr {
  const int32_t *p;
  const int32_t *i;
  const int32_t *rb;  // block b owns rows [rb[b], rb[b+1]) (at most 2 rows per thread)
  const int32_t *tb;  // and nonzeros [tb[b], tb[b+1]): tb[b] = p[rb[b]]
  int32_t rows;
  int32_t nrb;
};

// Per-instance results written by the kernel.
struct BatchOut {
  int32_t status;
  int32_t cur;
  int32_t trace_iters_n, trace_trials_n, trace_checks_n;
  int32_t staged;     // 1 when the gathered vectors were staged in LDS
  int32_t anderson_steps;
  int32_t halvings;   // internal tolerance halvings of the external-test calibration
  int64_t outer_iters, trials, accepted, rejected, restarts, checks;
  double rp, rd, sp, sd;  // scaled outer residuals and scales at exit
  double gamma, lam_hat, omega, c_obj;
  uint64_t t_begin, t_setup, t_end;  // device wall-clock ticks
};

// Everything the kernel needs for one instance (device pointers).
struct BatchInst {
  int32_t n, m, me, mi;
  pdnqp_settings st;
  double eps_abs, eps_rel;
  uint64_t limit_ticks;  // time limit in wall-clock ticks from the instance's start
  BCsr Q, Qo, A, AT;     // full Q, Q without its diagonal, A, A'
  const int32_t *atperm; // A' values gathered from A's
  // unscaled data (internal rows)
  const double *Qraw, *Qoraw, *qdiag_raw, *Araw, *ATraw, *craw, *xlraw, *xuraw, *braw;
  // scaled data, written by the set-up
  double *Qv, *Qov, *qdiag, *Av, *ATv, *c, *lo, *hi, *b;
  float *Qo32, *A32, *AT32;  // FP32 copies (FP32 bulk)
  Vecs v;
  double *Fx2, *Fs2, *Fr2, *E2buf;
  double *lz;  // Lanczos coefficients: alpha [0, k), beta [k, 2k)
  double *AU, *AG;  // Anderson histories: (anderson_mem + 2) slots of (lambda, z)
  IterVecs<double> w64;
  IterVecs<float> w32;
  BatchOut *out;
};

// Nonzeros per stream tile for a workgroup size.
__host__ __device__ inline int batch_tile(int block) { return block * 8 < 4096 ? block * 8 : 4096; }

// Dynamic LDS bytes a launch needs to stage the gathered vectors of an
// instance with n columns and m rows (0: products only).
__host__ __device__ inline size_t batch_lds_bytes(int block, int n, int m, int precision) {
  const size_t vb = precision == PDNQP_FP32 ? 4 : 8;
  size_t bytes = (size_t)batch_tile(block) * 8;
  if (n + m > 0) bytes += ((size_t)n * vb + 15) / 16 * 16 + (size_t)m * vb;
  return bytes;
}

// Launch configurations of the persistent kernel: workgroup size and the
// minimum waves per SIMD given to the compiler (1: its own register budget,
// 4: at most 128 VGPRs, more workgroups per CU, some spills).
struct BatchConfig {
  int block;
  int waves;
};
constexpr BatchConfig kBatchConfigs[] = {{256, 1}, {512, 1}, {1024, 1}, {256, 4}, {512, 4}};
constexpr int kBatchNumConfigs = 5;

// Launches the persistent kernel (configuration index `config`) over
// `count` instances taken in the order `order` (device array); `queue` is
// a zeroed device counter.
int batch_launch(hipStream_t st, int precision, int config, int grid, size_t lds_bytes,
                 const BatchInst *insts, const int32_t *order, int count, uint32_t *queue);

// Resident workgroups per CU for a configuration (0 if it cannot launch).
int batch_occupancy(int precision, int config, size_t lds_bytes);

}  // namespace pdnqp
