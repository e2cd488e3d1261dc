// Host driver of the batched persistent solve: checks the handles, prepares
// their instance descriptors, picks the launch configuration (workgroup
// size from the autotuner's cache, LDS for staging the gathered vectors,
// one resident wave of workgroups), launches the persistent kernel once and
// collects the results.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <thread>
#include <tuple>

#include "pdnqp_solver.hpp"

namespace pdnqp {

namespace {

double now_s() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

std::mutex g_mu;
std::map<std::tuple<int, int, int>, int> g_tuned;  // batch class -> configuration index
int g_forced_config = -1;

int config_index(int block, int waves) {
  for (int i = 0; i < kBatchNumConfigs; ++i)
    if (kBatchConfigs[i].block == block && kBatchConfigs[i].waves == waves) return i;
  return -1;
}

int ilog2(double x) {
  int k = 0;
  while (x >= 2.0 && k < 62) {
    x *= 0.5;
    ++k;
  }
  return k;
}

double instance_cost(const Solver &s) {
  const HostQP &q = s.qp();
  return (double)q.Qi.size() + 2.0 * (double)q.Ai.size() + q.n + q.m;
}

std::tuple<int, int, int> batch_class(const std::vector<Solver *> &S) {
  double nz = 0.0;
  for (const Solver *s : S) nz += instance_cost(*s);
  const int count = (int)S.size();
  return std::make_tuple(S[0]->precision(), ilog2(count), ilog2(nz / std::max(1, count)));
}

struct DevMem {
  void *p = nullptr;
  ~DevMem() {
    if (p) hipFree(p);
  }
};

int hip_check(hipError_t e, const char *what, std::string &err) {
  if (e == hipSuccess) return PDNQP_OK;
  err = std::string(what) + ": " + hipGetErrorString(e);
  return PDNQP_E_DEVICE;
}

}  // namespace

int set_batch_config(int block, int waves) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (block == 0) {
    g_forced_config = -1;
    return PDNQP_OK;
  }
  const int c = config_index(block, waves);
  if (c < 0) return PDNQP_E_INVALID;
  g_forced_config = c;
  return PDNQP_OK;
}

int run_batch(const BatchRequest &req, pdnqp_batch_report *rep, std::vector<double> *done_ms,
              std::string &err) {
  const double t0 = now_s();
  const std::vector<Solver *> &S = req.solvers;
  const int count = (int)S.size();
  pdnqp_batch_report R;
  std::memset(&R, 0, sizeof(R));
  R.count = count;
  if (count == 0) {
    if (rep) *rep = R;
    return PDNQP_OK;
  }
  const int prec = S[0]->precision();
  const int dev = S[0]->device();
  for (const Solver *s : S) {
    if (s->precision() != prec || s->device() != dev) {
      err = "batched solve: all handles must share one device and one precision";
      return PDNQP_E_INVALID;
    }
  }
  int r;
  if ((r = hip_check(hipSetDevice(dev), "hipSetDevice", err))) return r;
  // launch configuration
  int config = req.config;
  bool tuned = false;
  if (config < 0) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_forced_config >= 0) {
      config = g_forced_config;
    } else {
      auto it = g_tuned.find(batch_class(S));
      if (it != g_tuned.end()) {
        config = it->second;
        tuned = true;
      } else {
        config = 0;
      }
    }
  }
  if (config < 0 || config >= kBatchNumConfigs) {
    err = "batched solve: unknown launch configuration";
    return PDNQP_E_INVALID;
  }
  const int block = kBatchConfigs[config].block;
  hipDeviceProp_t prop;
  if ((r = hip_check(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties", err))) return r;
  int rate_khz = 0;
  if ((r = hip_check(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev),
                     "wall clock rate", err)))
    return r;
  if (rate_khz <= 0) {
    err = "batched solve: device reports no wall-clock rate";
    return PDNQP_E_DEVICE;
  }
  const double tps = 1000.0 * rate_khz;
  // dynamic LDS: the products' tile, plus staging for the largest instance
  // that fits in this configuration's share of the CU's LDS (the register
  // budget fixes how many workgroups share a CU)
  size_t lds = (size_t)batch_tile(block) * 8;
  const int per_cu_regs = batch_occupancy(prec, config, lds);
  if (per_cu_regs < 1) {
    err = "batched solve: the kernel cannot be resident with this configuration";
    return PDNQP_E_DEVICE;
  }
  const size_t cu_lds = prop.maxSharedMemoryPerMultiProcessor > 0
                            ? (size_t)prop.maxSharedMemoryPerMultiProcessor
                            : (size_t)prop.sharedMemPerBlock;
  size_t lds_cap = cu_lds / per_cu_regs;
  lds_cap = std::min(lds_cap, (size_t)prop.sharedMemPerBlock);
  lds_cap = lds_cap > 8192 ? lds_cap - 8192 : 0;
  for (const Solver *s : S) {
    const size_t need = batch_lds_bytes(block, s->qp().n, s->qp().m, prec);
    if (need <= lds_cap) lds = std::max(lds, need);
  }
  const int per_cu = batch_occupancy(prec, config, lds);
  if (per_cu < 1) {
    err = "batched solve: the kernel cannot be resident with this configuration";
    return PDNQP_E_DEVICE;
  }
  const int grid = std::min(count, per_cu * prop.multiProcessorCount);
  // device arrays of the launch
  DevMem d_insts, d_outs, d_order, d_queue;
  if ((r = hip_check(hipMalloc(&d_insts.p, sizeof(BatchInst) * count), "hipMalloc", err)) ||
      (r = hip_check(hipMalloc(&d_outs.p, sizeof(BatchOut) * count), "hipMalloc", err)) ||
      (r = hip_check(hipMalloc(&d_order.p, sizeof(int32_t) * count), "hipMalloc", err)) ||
      (r = hip_check(hipMalloc(&d_queue.p, 256), "hipMalloc", err)))
    return r;
  BatchOut *outs = (BatchOut *)d_outs.p;
  std::vector<BatchInst> hb(count);
  for (int i = 0; i < count; ++i) {
    if ((r = S[i]->batch_prepare(req.eps_abs, req.eps_rel, nullptr, nullptr, block, tps,
                                 outs + i, hb[i], err)))
      return r;
    if (req.probe_inner > 0) {
      hb[i].st.max_outer = 1;
      hb[i].st.max_inner = req.probe_inner;
      hb[i].st.trace_iters = 0;
      hb[i].st.trace_trials = 0;
    }
  }
  // largest first
  std::vector<int32_t> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::vector<double> cost(count);
  for (int i = 0; i < count; ++i) cost[i] = instance_cost(*S[i]);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
  hipStream_t st = S[0]->stream();
  hipError_t e = hipMemcpyAsync(d_insts.p, hb.data(), sizeof(BatchInst) * count,
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_order.p, order.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice,
                       st);
  if (e == hipSuccess) e = hipMemsetAsync(d_queue.p, 0, 256, st);
  if (e == hipSuccess) e = hipMemsetAsync(d_outs.p, 0, sizeof(BatchOut) * count, st);
  if ((r = hip_check(e, "batch upload", err))) return r;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEventCreate(&ev0);
  hipEventCreate(&ev1);
  const double t_prep = now_s();
  hipEventRecord(ev0, st);
  r = batch_launch(st, prec, config, grid, lds, (const BatchInst *)d_insts.p,
                   (const int32_t *)d_order.p, count, (uint32_t *)d_queue.p);
  hipEventRecord(ev1, st);
  hipError_t es = hipStreamSynchronize(st);
  float kms = 0.f;
  hipEventElapsedTime(&kms, ev0, ev1);
  hipEventDestroy(ev0);
  hipEventDestroy(ev1);
  if (r) {
    err = "batched solve: kernel launch failed";
    return r;
  }
  if ((r = hip_check(es, "batched kernel", err))) return r;
  std::vector<BatchOut> ho(count);
  if ((r = hip_check(hipMemcpy(ho.data(), d_outs.p, sizeof(BatchOut) * count,
                               hipMemcpyDeviceToHost),
                     "batch results", err)))
    return r;
  const double t_kernel = now_s();
  // results: copies back, unscaling and external checks, in parallel
  if (req.probe_inner <= 0) {
    const int nt = std::max(1, std::min(count, 16));
    std::vector<std::string> errs(nt);
    std::vector<int> rcs(nt, PDNQP_OK);
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) {
      th.emplace_back([&, t] {
        for (int i = t; i < count && rcs[t] == PDNQP_OK; i += nt) {
          rcs[t] = S[i]->batch_finish(ho[i], tps, req.x_out ? req.x_out[i] : nullptr,
                                      req.lam_out ? req.lam_out[i] : nullptr,
                                      req.infos ? &req.infos[i] : nullptr, errs[t]);
        }
      });
    }
    for (auto &x : th) x.join();
    for (int t = 0; t < nt; ++t) {
      if (rcs[t] != PDNQP_OK) {
        err = errs[t];
        return rcs[t];
      }
    }
  }
  uint64_t first = ~0ull;
  for (const BatchOut &o : ho) first = std::min(first, o.t_begin);
  if (done_ms) {
    done_ms->resize(count);
    for (int i = 0; i < count; ++i) (*done_ms)[i] = 1e3 * (double)(ho[i].t_end - first) / tps;
  }
  R.block = block;
  R.waves = kBatchConfigs[config].waves;
  R.grid = grid;
  R.lds_bytes = (int32_t)lds;
  for (const BatchOut &o : ho) R.staged += o.staged;
  R.tuned = tuned ? 1 : 0;
  R.kernel_ms = kms;
  R.prepare_s = t_prep - t0;
  R.finish_s = now_s() - t_kernel;
  R.wall_s = now_s() - t0;
  if (rep) *rep = R;
  return PDNQP_OK;
}

int autotune_batch(const BatchRequest &req, int32_t *block_out, int32_t *waves_out,
                   double *ms_out, std::string &err) {
  if (req.solvers.empty()) {
    err = "autotune: empty batch";
    return PDNQP_E_INVALID;
  }
  int best = -1;
  double best_ms = 0.0;
  for (int c = 0; c < kBatchNumConfigs; ++c) {
    BatchRequest q = req;
    q.config = c;
    q.probe_inner = req.probe_inner > 0 ? req.probe_inner : 64;
    pdnqp_batch_report rep;
    const int r = run_batch(q, &rep, nullptr, err);
    if (r) return r;
    if (ms_out) ms_out[c] = rep.kernel_ms;
    if (best < 0 || rep.kernel_ms < best_ms) {
      best = c;
      best_ms = rep.kernel_ms;
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuned[batch_class(req.solvers)] = best;
  }
  if (block_out) *block_out = kBatchConfigs[best].block;
  if (waves_out) *waves_out = kBatchConfigs[best].waves;
  return PDNQP_OK;
}

}  // namespace pdnqp
