"""Python binding of ``libpdnqp.so`` (the gfx950 PDNQP library).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  The library must have been built (``build.py``); loading fails
loudly otherwise.  PyTorch, when asked for (``use_torch=True``), provides the
HIP stream and the device memory (its caching allocator) -- nothing else.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdnqp.so")

OK = 0
E_INVALID, E_NOMEM, E_DEVICE, E_STATE = -1, -2, -3, -4
SOLVED, MAX_ITER, TIME_LIMIT, NUMERICAL_ERROR, INACCURATE = 1, 2, 3, 4, 7
STATUS_NAMES = {SOLVED: "solved", MAX_ITER: "max_iter", TIME_LIMIT: "time_limit",
                NUMERICAL_ERROR: "numerical_error", INACCURATE: "inaccurate"}
SCALE_RUIZ_A, SCALE_NONE, SCALE_RUIZ_QA = 0, 1, 2
FP64, FP32 = 0, 1

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Settings(ctypes.Structure):
    _fields_ = [
        ("max_outer", ctypes.c_int64),
        ("max_inner", ctypes.c_int32),
        ("ruiz_sweeps", ctypes.c_int32),
        ("time_limit_s", ctypes.c_double),
        ("sigma_init", ctypes.c_double),
        ("theta_sigma", ctypes.c_double),
        ("delta_gamma", ctypes.c_double),
        ("rho_in_min", ctypes.c_double),
        ("rho_in_max", ctypes.c_double),
        ("rho_z", ctypes.c_double),
        ("check_every", ctypes.c_int32),
        ("max_rejects", ctypes.c_int32),
        ("restart_suff", ctypes.c_double),
        ("restart_nec", ctypes.c_double),
        ("restart_art", ctypes.c_double),
        ("shrink_safety", ctypes.c_double),
        ("shrink_min", ctypes.c_double),
        ("shrink_max", ctypes.c_double),
        ("omega0", ctypes.c_double),
        ("sigma_growth", ctypes.c_double),
        ("sigma_max", ctypes.c_double),
        ("sigma0_min", ctypes.c_double),
        ("sigma0_max", ctypes.c_double),
        ("penalty_gate", ctypes.c_int32),
        ("lanczos_iters", ctypes.c_int32),
        ("gamma_override", ctypes.c_double),
        ("step_boost", ctypes.c_double),
        ("outer_scaling", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("trace_iters", ctypes.c_int32),
        ("trace_trials", ctypes.c_int32),
        ("verbose", ctypes.c_int32),
        ("center_floor", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("anderson_mem", ctypes.c_int32),
        ("anderson_reg", ctypes.c_double),
        ("controller", ctypes.c_int32),
        ("outer_log", ctypes.c_int32),
        ("fp32_promote", ctypes.c_double),
        ("delta_floor", ctypes.c_double),
        ("fp32_stall", ctypes.c_int32),
        ("external_halvings", ctypes.c_int32),
        ("hip_stream", ctypes.c_void_p),
        ("dev_alloc", _ALLOC_FN),
        ("dev_free", _FREE_FN),
        ("alloc_user", ctypes.c_void_p),
        ("delta0", ctypes.c_double),
        ("col_panels", ctypes.c_int32),
        ("stream_grid", ctypes.c_int32),
        ("kkt_pass_limit", ctypes.c_double),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("anderson_steps", ctypes.c_int32),
        ("outer_iters", ctypes.c_int64),
        ("inner_trials", ctypes.c_int64),
        ("inner_accepted", ctypes.c_int64),
        ("inner_rejected", ctypes.c_int64),
        ("restarts", ctypes.c_int64),
        ("checks", ctypes.c_int64),
        ("r_p", ctypes.c_double),
        ("r_d", ctypes.c_double),
        ("s_p", ctypes.c_double),
        ("s_d", ctypes.c_double),
        ("r_p_scaled", ctypes.c_double),
        ("r_d_scaled", ctypes.c_double),
        ("s_p_scaled", ctypes.c_double),
        ("s_d_scaled", ctypes.c_double),
        ("objective", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("lambda_hat", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("setup_s", ctypes.c_double),
        ("solve_s", ctypes.c_double),
        ("controller_fallback", ctypes.c_int32),
        ("outer_logged", ctypes.c_int32),
        ("promoted_outer", ctypes.c_int32),
        ("halvings", ctypes.c_int32),
    ]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["status_name"] = STATUS_NAMES.get(self.status, str(self.status))
        return d


class KernelStat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 32),
        ("launches", ctypes.c_int64),
        ("total_ms", ctypes.c_double),
        ("avg_us", ctypes.c_double),
        ("bytes_per_launch", ctypes.c_double),
    ]


class BatchReport(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("grid", ctypes.c_int32),
        ("lds_bytes", ctypes.c_int32),
        ("staged", ctypes.c_int32),
        ("tuned", ctypes.c_int32),
        ("waves", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("kernel_ms", ctypes.c_double),
        ("prepare_s", ctypes.c_double),
        ("finish_s", ctypes.c_double),
        ("wall_s", ctypes.c_double),
    ]


EXPORTED = ["pdnqp_default_settings", "pdnqp_settings_size", "pdnqp_info_size", "pdnqp_create",
            "pdnqp_solve", "pdnqp_solve_batch", "pdnqp_destroy", "pdnqp_last_error",
            "pdnqp_dims", "pdnqp_get_trace", "pdnqp_kernel_stats", "pdnqp_batch_last_report",
            "pdnqp_batch_set_config", "pdnqp_batch_autotune", "pdnqp_mlp_forward",
            "pdnqp_mlp_gradient", "pdnqp_mlp_gradient_noalloc", "pdnqp_mlp_train",
            "pdnqp_set_controller",
            "pdnqp_get_outer_log", "pdnqp_probe_gather"]

MLP_PARAMS, N_FEATURES, OUTER_RECORD = 5443, 16, 8

_lib = None


class PdnqpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pdnqp error {code}: {msg}")
        self.code = code


def _one_hip_runtime():
    """Makes PyTorch's HIP runtime the process's only one, before the
    library is loaded.  PyTorch's ROCm build ships its own runtime and asks
    for it under the unversioned name ``libamdhip64.so``; the library asks
    for ``libamdhip64.so.7``.  Loaded first, the library would map the
    system runtime and a later ``import torch`` a second one, and device
    pointers and streams would then cross runtimes.  With torch imported
    first, the library's request is met by the runtime already mapped (same
    soname).  Without PyTorch the library uses the system runtime."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def load(path=None):
    """Loads the library (once).  Raises if it is missing or mismatched."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} not found: build it first (python -m paper_2609_19557_amd.build)")
    _one_hip_runtime()
    lib = ctypes.CDLL(p)
    i32, i64, dbl, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    P = ctypes.POINTER
    lib.pdnqp_default_settings.argtypes = [P(Settings)]
    lib.pdnqp_default_settings.restype = None
    lib.pdnqp_settings_size.restype = ctypes.c_size_t
    lib.pdnqp_info_size.restype = ctypes.c_size_t
    lib.pdnqp_create.argtypes = [P(vp), i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                 P(Settings)]
    lib.pdnqp_create.restype = ctypes.c_int
    lib.pdnqp_solve.argtypes = [vp, dbl, dbl, vp, vp, vp, vp, P(Info)]
    lib.pdnqp_solve.restype = ctypes.c_int
    lib.pdnqp_solve_batch.argtypes = [i32, P(vp), dbl, dbl, P(vp), P(vp), P(Info)]
    lib.pdnqp_solve_batch.restype = ctypes.c_int
    lib.pdnqp_destroy.argtypes = [vp]
    lib.pdnqp_destroy.restype = None
    lib.pdnqp_last_error.restype = ctypes.c_char_p
    lib.pdnqp_dims.argtypes = [vp, P(i32), P(i32), P(i32)]
    lib.pdnqp_dims.restype = ctypes.c_int
    lib.pdnqp_get_trace.argtypes = [vp, P(i32), vp, vp, P(i32), vp, P(i32), vp]
    lib.pdnqp_get_trace.restype = ctypes.c_int
    lib.pdnqp_kernel_stats.argtypes = [vp, P(KernelStat), i32, P(i32)]
    lib.pdnqp_kernel_stats.restype = ctypes.c_int
    lib.pdnqp_batch_last_report.argtypes = [P(BatchReport), vp, i32]
    lib.pdnqp_batch_last_report.restype = ctypes.c_int
    lib.pdnqp_batch_set_config.argtypes = [i32, i32]
    lib.pdnqp_batch_set_config.restype = ctypes.c_int
    lib.pdnqp_batch_autotune.argtypes = [i32, P(vp), i32, P(i32), P(i32), vp]
    lib.pdnqp_batch_autotune.restype = ctypes.c_int
    lib.pdnqp_mlp_forward.argtypes = [vp, vp, i32, vp]
    lib.pdnqp_mlp_forward.restype = ctypes.c_int
    lib.pdnqp_mlp_gradient.argtypes = [vp, vp, vp, i32, vp, P(dbl)]
    lib.pdnqp_mlp_gradient.restype = ctypes.c_int
    lib.pdnqp_probe_gather.argtypes = [i32, i32, ctypes.c_int64, i32, i32, ctypes.c_uint64,
                                       P(dbl), P(dbl)]
    lib.pdnqp_probe_gather.restype = ctypes.c_int
    lib.pdnqp_mlp_gradient_noalloc.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    lib.pdnqp_mlp_gradient_noalloc.restype = ctypes.c_int
    lib.pdnqp_mlp_train.argtypes = [vp, vp, vp, i32, i32, i32, ctypes.c_float, ctypes.c_uint64, vp]
    lib.pdnqp_mlp_train.restype = ctypes.c_int
    lib.pdnqp_set_controller.argtypes = [vp, vp]
    lib.pdnqp_set_controller.restype = ctypes.c_int
    lib.pdnqp_get_outer_log.argtypes = [vp, P(i32), vp, vp]
    lib.pdnqp_get_outer_log.restype = ctypes.c_int
    if lib.pdnqp_settings_size() != ctypes.sizeof(Settings):
        raise ImportError("pdnqp_settings layout mismatch between library and binding")
    if lib.pdnqp_info_size() != ctypes.sizeof(Info):
        raise ImportError("pdnqp_info layout mismatch between library and binding")
    if path is None:
        _lib = lib
    return lib


def _err(lib, code):
    return PdnqpError(code, lib.pdnqp_last_error().decode())


def default_settings(**overrides):
    lib = load()
    s = Settings()
    lib.pdnqp_default_settings(ctypes.byref(s))
    for k, v in overrides.items():
        if not hasattr(s, k):
            raise KeyError(k)
        setattr(s, k, v)
    return s


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


def _csr_parts(M, rows, cols):
    import scipy.sparse as sp
    M = sp.csr_matrix(M)
    if M.shape != (rows, cols):
        raise ValueError(f"matrix shape {M.shape} != {(rows, cols)}")
    M.sort_indices()
    return (np.ascontiguousarray(M.indptr, dtype=np.int32),
            np.ascontiguousarray(M.indices, dtype=np.int32),
            np.ascontiguousarray(M.data, dtype=np.float64))


class _TorchPlumbing:
    """Stream and caching-allocator callbacks from PyTorch."""

    def __init__(self):
        import torch
        self.torch = torch
        self.stream = torch.cuda.current_stream()
        dev = torch.cuda.current_device()

        def alloc(nbytes, user):
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, self.stream)

        def free(ptr, user):
            torch.cuda.caching_allocator_delete(int(ptr))

        self.alloc_cb = _ALLOC_FN(alloc)
        self.free_cb = _FREE_FN(free)


class Solver:
    """One QP on the GPU: ``min 1/2 x'Qx + c'x, rl <= Ax <= ru, xl <= x <= xu``."""

    def __init__(self, Q, A, c, xl, xu, rl, ru, settings=None, use_torch=False, **overrides):
        self.lib = load()
        n = int(np.asarray(c).shape[0])
        m = int(A.shape[0])
        self.n, self.m = n, m
        st = settings if settings is not None else default_settings()
        for k, v in overrides.items():
            setattr(st, k, v)
        self._torch = None
        if use_torch:
            self._torch = _TorchPlumbing()
            st.hip_stream = ctypes.c_void_p(self._torch.stream.cuda_stream)
            st.dev_alloc = self._torch.alloc_cb
            st.dev_free = self._torch.free_cb
        self.settings = st
        Qp, Qi, Qx = _csr_parts(Q, n, n)
        Ap, Ai, Ax = _csr_parts(A, m, n)
        self._keep = [np.ascontiguousarray(v, dtype=np.float64) for v in (c, xl, xu, rl, ru)]
        c_, xl_, xu_, rl_, ru_ = self._keep
        h = ctypes.c_void_p()
        code = self.lib.pdnqp_create(ctypes.byref(h), n, m, _ptr(Qp), _ptr(Qi), _ptr(Qx),
                                     Ap.ctypes.data_as(ctypes.c_void_p), _ptr(Ai), _ptr(Ax),
                                     _ptr(c_), _ptr(xl_), _ptr(xu_), _ptr(rl_), _ptr(ru_),
                                     ctypes.byref(st))
        if code != OK:
            raise _err(self.lib, code)
        self.h = h

    @classmethod
    def from_problem(cls, prob, **kw):
        return cls(prob["Q"], prob["A"], prob["c"], prob["xl"], prob["xu"], prob["rl"],
                   prob["ru"], **kw)

    def solve(self, eps_abs=1e-4, eps_rel=1e-4, x0=None, lam0=None):
        x = np.zeros(self.n)
        lam = np.zeros(max(self.m, 1))
        info = Info()
        x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        l0a = None if lam0 is None else np.ascontiguousarray(lam0, dtype=np.float64)
        code = self.lib.pdnqp_solve(self.h, eps_abs, eps_rel, _ptr(x0a), _ptr(l0a),
                                    x.ctypes.data_as(ctypes.c_void_p),
                                    lam.ctypes.data_as(ctypes.c_void_p), ctypes.byref(info))
        if code != OK:
            raise _err(self.lib, code)
        return x, lam[:self.m], info.as_dict()

    def dims(self):
        me, mi, dw = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        code = self.lib.pdnqp_dims(self.h, ctypes.byref(me), ctypes.byref(mi), ctypes.byref(dw))
        if code != OK:
            raise _err(self.lib, code)
        return me.value, mi.value, dw.value

    def trace(self):
        it, ntr, nck = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        code = self.lib.pdnqp_get_trace(self.h, ctypes.byref(it), None, None, ctypes.byref(ntr),
                                        None, ctypes.byref(nck), None)
        if code != OK:
            raise _err(self.lib, code)
        me, mi, dw = self.dims()
        mint = me + mi
        w = np.zeros((it.value, dw))
        y = np.zeros((it.value, max(mint, 1)))
        tr = np.zeros((ntr.value, 3))
        ck = np.zeros((nck.value, 4), dtype=np.int32)
        code = self.lib.pdnqp_get_trace(self.h, ctypes.byref(it), _ptr(w), _ptr(y),
                                        ctypes.byref(ntr), _ptr(tr), ctypes.byref(nck), _ptr(ck))
        if code != OK:
            raise _err(self.lib, code)
        return dict(w=w, y=y[:, :mint], trials=tr, checks=ck)

    def set_controller(self, theta):
        """Loads the controller network's parameters (MLP_PARAMS floats)."""
        th = np.ascontiguousarray(theta, dtype=np.float32)
        if th.size != MLP_PARAMS:
            raise ValueError(f"expected {MLP_PARAMS} parameters")
        code = self.lib.pdnqp_set_controller(self.h, _ptr(th))
        if code != OK:
            raise _err(self.lib, code)

    def outer_log(self):
        """Features (steps x 16) and raw records (steps x 8) of the outer
        steps recorded by the last solve (settings.outer_log)."""
        n = ctypes.c_int32()
        code = self.lib.pdnqp_get_outer_log(self.h, ctypes.byref(n), None, None)
        if code != OK:
            raise _err(self.lib, code)
        f = np.zeros((max(n.value, 1), N_FEATURES))
        r = np.zeros((max(n.value, 1), OUTER_RECORD))
        self.lib.pdnqp_get_outer_log(self.h, ctypes.byref(n), _ptr(f), _ptr(r))
        return f[:n.value], r[:n.value]

    def kernel_stats(self):
        cnt = ctypes.c_int32()
        self.lib.pdnqp_kernel_stats(self.h, None, 0, ctypes.byref(cnt))
        arr = (KernelStat * max(cnt.value, 1))()
        self.lib.pdnqp_kernel_stats(self.h, arr, cnt.value, ctypes.byref(cnt))
        return [dict(name=a.name.decode(), launches=a.launches, total_ms=a.total_ms,
                     avg_us=a.avg_us, bytes_per_launch=a.bytes_per_launch)
                for a in arr[:cnt.value]]

    def close(self):
        if getattr(self, "h", None):
            self.lib.pdnqp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(solvers, eps_abs=1e-4, eps_rel=1e-4):
    """``pdnqp_solve_batch`` over a list of ``Solver``s (one persistent
    kernel launch; see ``batch_report`` for its configuration and timing)."""
    lib = load()
    k = len(solvers)
    xs = [np.zeros(s.n) for s in solvers]
    ls = [np.zeros(max(s.m, 1)) for s in solvers]
    hs = (ctypes.c_void_p * k)(*[s.h.value for s in solvers])
    xp = (ctypes.c_void_p * k)(*[x.ctypes.data for x in xs])
    lp = (ctypes.c_void_p * k)(*[l.ctypes.data for l in ls])
    infos = (Info * k)()
    code = lib.pdnqp_solve_batch(k, hs, eps_abs, eps_rel, xp, lp, infos)
    if code != OK:
        raise _err(lib, code)
    return [(xs[i], ls[i][:solvers[i].m], infos[i].as_dict()) for i in range(k)]


def batch_report(count=None):
    """Report of the last ``solve_batch`` on this thread: launch configuration,
    kernel and host times, and each instance's finish time (ms after the
    first instance started)."""
    lib = load()
    rep = BatchReport()
    cap = count if count is not None else 0
    done = np.zeros(max(cap, 1))
    code = lib.pdnqp_batch_last_report(ctypes.byref(rep), _ptr(done) if cap else None, cap)
    if code != OK:
        raise _err(lib, code)
    d = {name: getattr(rep, name) for name, _ in rep._fields_}
    if cap:
        d["done_ms"] = done[:min(cap, rep.count)].copy()
    return d


BATCH_CONFIGS = [(256, 1), (512, 1), (1024, 1), (256, 4), (512, 4)]


def batch_set_config(block, waves=1):
    """Launch configuration of later batched solves (see BATCH_CONFIGS);
    block 0 returns to the autotuned choice."""
    lib = load()
    code = lib.pdnqp_batch_set_config(int(block), int(waves))
    if code != OK:
        raise _err(lib, code)


def batch_autotune(solvers, probe_inner=64):
    """Times each launch configuration on the batch (short probe) and caches
    the fastest for the batch's class; returns ((block, waves), [ms per
    configuration in BATCH_CONFIGS order])."""
    lib = load()
    k = len(solvers)
    hs = (ctypes.c_void_p * k)(*[s.h.value for s in solvers])
    blk, wv = ctypes.c_int32(), ctypes.c_int32()
    ms = np.zeros(len(BATCH_CONFIGS))
    code = lib.pdnqp_batch_autotune(k, hs, int(probe_inner), ctypes.byref(blk), ctypes.byref(wv),
                                    _ptr(ms))
    if code != OK:
        raise _err(lib, code)
    return (blk.value, wv.value), ms.tolist()


def mlp_forward(theta, X):
    """Controller network on the GPU: (count x 16) -> (count x 3)."""
    lib = load()
    th = np.ascontiguousarray(theta, dtype=np.float32)
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.zeros((X.shape[0], 3), dtype=np.float32)
    code = lib.pdnqp_mlp_forward(_ptr(th), _ptr(X), X.shape[0], _ptr(Y))
    if code != OK:
        raise _err(lib, code)
    return Y


def mlp_gradient(theta, X, Y):
    """Gradient and value of the mean squared error, on the GPU."""
    lib = load()
    th = np.ascontiguousarray(theta, dtype=np.float32)
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    g = np.zeros(MLP_PARAMS, dtype=np.float32)
    loss = ctypes.c_double()
    code = lib.pdnqp_mlp_gradient(_ptr(th), _ptr(X), _ptr(Y), X.shape[0], _ptr(g),
                                  ctypes.byref(loss))
    if code != OK:
        raise _err(lib, code)
    return g, loss.value


def probe_gather(vec_len, elem_bytes=8, gathers=8_000_000, reps=20, seed=1, panels=1):
    """Random-gather rate of the current device (pdnqp_probe_gather):
    returns (gathers per second, average launch microseconds)."""
    lib = load()
    rate, us = ctypes.c_double(), ctypes.c_double()
    code = lib.pdnqp_probe_gather(int(vec_len), int(elem_bytes), int(gathers), int(panels),
                                  int(reps), int(seed), ctypes.byref(rate), ctypes.byref(us))
    if code != OK:
        raise _err(lib, code)
    return rate.value, us.value


def mlp_gradient_noalloc(theta, x, y, count, grad, loss=None, stream=None):
    """The allocation-free gradient entry point: every argument is a device
    address (int) of a caller-owned buffer -- theta, x (count x 16), y
    (count x 3), grad (written) and loss (one double, written; None to skip)
    -- and ``stream`` a hipStream_t address (None: the default stream).  The
    work is enqueued, not synchronised."""
    lib = load()
    code = lib.pdnqp_mlp_gradient_noalloc(theta, x, y, int(count), grad, loss, stream)
    if code != OK:
        raise _err(lib, code)


def mlp_train(theta, X, Y, epochs=200, batch=256, lr=1e-3, seed=0):
    """Adam training on the GPU; returns (theta, loss per epoch)."""
    lib = load()
    th = np.array(theta, dtype=np.float32, copy=True)
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    curve = np.zeros(max(epochs, 1), dtype=np.float32)
    code = lib.pdnqp_mlp_train(_ptr(th), _ptr(X), _ptr(Y), X.shape[0], int(epochs), int(batch),
                               float(lr), int(seed), _ptr(curve))
    if code != OK:
        raise _err(lib, code)
    return th, curve[:epochs]
