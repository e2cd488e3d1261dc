"""C ABI checks that need no GPU: the library loads, exports every function
the public header declares, its struct layouts match the binding, the
defaults are the paper's, and malformed input is rejected before any device
call (PDNQP_E_INVALID with a message)."""

import ctypes
import math
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import qpgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdnqp.h")


@pytest.fixture(scope="module")
def P():
    import paper_2609_19557_amd as P
    try:
        P.load()
    except ImportError as e:
        pytest.fail(f"library not built: {e}")
    return P


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(pdnqp_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_functions_are_exported(P):
    lib = P.load()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), f"{name} declared in pdnqp.h but not exported"
    assert set(names) == set(P.pdnqp.EXPORTED)


def test_struct_layouts_and_defaults(P):
    lib = P.load()
    assert lib.pdnqp_settings_size() == ctypes.sizeof(P.pdnqp.Settings)
    assert lib.pdnqp_info_size() == ctypes.sizeof(P.pdnqp.Info)
    s = P.default_settings()
    # the paper's default parameter table
    assert s.max_outer == 2**31 - 1
    assert s.max_inner == 40000
    assert math.isinf(s.time_limit_s)
    assert s.sigma_init == 20.0
    assert s.theta_sigma == 0.25
    assert s.delta_gamma == 1e-2
    assert (s.rho_in_min, s.rho_in_max, s.rho_z) == (0.3, 0.95, 0.95)
    assert s.ruiz_sweeps == 8
    assert s.outer_scaling == P.SCALE_RUIZ_A


def _args(p):
    return (p["Q"], p["A"], p["c"], p["xl"], p["xu"], p["rl"], p["ru"])


def _expect_invalid(P, *args, match=None, **kw):
    with pytest.raises(P.PdnqpError) as ei:
        P.Solver(*args, **kw)
    assert ei.value.code == -1
    if match:
        assert match in str(ei.value)


def test_rejects_asymmetric_q(P):
    p = qpgen.workload("small", 1)
    Q = p["Q"].tolil()
    Q[0, 1] = Q[0, 1] + 1.0
    _expect_invalid(P, sp.csr_matrix(Q), *_args(p)[1:], match="symmetric")


def test_rejects_nonfinite_and_bad_bounds(P):
    p = qpgen.workload("small", 2)
    c = p["c"].copy()
    c[3] = np.nan
    _expect_invalid(P, p["Q"], p["A"], c, p["xl"], p["xu"], p["rl"], p["ru"], match="c has")
    xl = p["xl"].copy()
    xl[0] = 2.0
    _expect_invalid(P, p["Q"], p["A"], p["c"], xl, p["xu"], p["rl"], p["ru"], match="bounds")
    rl = p["rl"].copy()
    rl[p["m"] - 1] = np.inf
    _expect_invalid(P, p["Q"], p["A"], p["c"], p["xl"], p["xu"], rl, p["ru"], match="row bounds")
    A = p["A"].copy()
    A.data[0] = np.inf
    _expect_invalid(P, p["Q"], A, p["c"], p["xl"], p["xu"], p["rl"], p["ru"], match="non-finite")


def test_rejects_bad_csr_structure(P):
    lib = P.load()
    n, m = 3, 1
    Qp = np.array([0, 1, 2, 3], dtype=np.int32)
    Qi = np.array([0, 1, 2], dtype=np.int32)
    Qx = np.ones(3)
    c = np.zeros(3)
    xl = np.zeros(3)
    xu = np.ones(3)
    rl = np.zeros(1)
    ru = np.ones(1)
    vp = ctypes.c_void_p
    h = vp()

    def create(Ap, Ai, Ax):
        return lib.pdnqp_create(ctypes.byref(h), n, m, Qp.ctypes.data, Qi.ctypes.data,
                                Qx.ctypes.data, Ap.ctypes.data, Ai.ctypes.data, Ax.ctypes.data,
                                c.ctypes.data, xl.ctypes.data, xu.ctypes.data, rl.ctypes.data,
                                ru.ctypes.data, None)
    # unsorted column indices
    assert create(np.array([0, 2], np.int32), np.array([2, 1], np.int32), np.ones(2)) == -1
    assert b"increasing" in lib.pdnqp_last_error()
    # out-of-range column
    assert create(np.array([0, 1], np.int32), np.array([3], np.int32), np.ones(1)) == -1
    assert b"range" in lib.pdnqp_last_error()
    # row pointers not starting at zero
    assert create(np.array([1, 2], np.int32), np.array([0, 1], np.int32), np.ones(2)) == -1
    assert h.value is None
    # NULL output handle
    assert lib.pdnqp_create(None, n, m, None, None, None, None, None, None, None, None, None,
                            None, None, None) == -1
    # bad settings value
    s = P.default_settings(check_every=0)
    assert lib.pdnqp_create(ctypes.byref(h), n, m, Qp.ctypes.data, Qi.ctypes.data,
                            Qx.ctypes.data, np.array([0, 1], np.int32).ctypes.data,
                            np.array([0], np.int32).ctypes.data, np.ones(1).ctypes.data,
                            c.ctypes.data, xl.ctypes.data, xu.ctypes.data, rl.ctypes.data,
                            ru.ctypes.data, ctypes.byref(s)) == -1
    assert b"settings" in lib.pdnqp_last_error()


def test_null_handle_calls_are_errors(P):
    lib = P.load()
    i = ctypes.c_int32()
    assert lib.pdnqp_dims(None, ctypes.byref(i), None, None) == -1
    assert lib.pdnqp_solve(None, 1e-4, 1e-4, None, None, None, None, None) == -1
    assert lib.pdnqp_get_trace(None, None, None, None, None, None, None, None) == -1
    lib.pdnqp_destroy(None)


@pytest.mark.parametrize("field,value", [("graph", 2), ("anderson_mem", 9), ("anderson_mem", -1),
                                         ("anderson_reg", -1.0), ("controller", 2),
                                         ("outer_log", -1), ("precision", 3),
                                         ("fp32_promote", -1e-5),
                                         ("fp32_promote", float("nan")),
                                         ("delta_floor", -0.5), ("delta_floor", float("inf")),
                                         ("fp32_stall", -1), ("external_halvings", -1),
                                         ("external_halvings", 31), ("delta0", 0.0),
                                         ("delta0", float("nan")), ("col_panels", 3),
                                         ("stream_grid", -1), ("stream_grid", 1),
                                         ("stream_grid", 4097), ("kkt_pass_limit", 0.5),
                                         ("kkt_pass_limit", float("nan"))])
def test_rejects_bad_extension_settings(P, field, value):
    p = qpgen.workload("small", 3)
    _expect_invalid(P, *_args(p), match="settings", **{field: value})


def test_extension_defaults(P):
    s = P.default_settings()
    assert (s.graph, s.anderson_mem, s.controller, s.outer_log, s.precision) == (0, 0, 0, 0, 0)
    assert s.anderson_reg == 1e-10
    assert s.fp32_promote == 1e-5
    assert s.delta_floor == 1.0
    assert s.fp32_stall == 50
    assert s.external_halvings == 7
    assert s.delta0 == 1.0
    assert (s.col_panels, s.stream_grid) == (0, 0)
    assert s.kkt_pass_limit == float("inf")  # the paper's table


def test_batch_and_network_argument_errors(P):
    """Argument checks of the batched, tuning and network entry points that
    fail before any device call."""
    lib = P.load()
    assert lib.pdnqp_batch_set_config(300, 1) == -1
    assert lib.pdnqp_batch_set_config(512, 2) == -1
    assert lib.pdnqp_batch_set_config(0, 0) == 0
    assert lib.pdnqp_solve_batch(-1, None, 1e-4, 1e-4, None, None, None) == -1
    assert lib.pdnqp_solve_batch(0, None, 1e-4, 1e-4, None, None, None) == 0
    assert lib.pdnqp_solve_batch(0, None, 0.0, 0.0, None, None, None) == -1
    assert lib.pdnqp_batch_autotune(0, None, 64, None, None, None) == -1
    rep = P.pdnqp.BatchReport()
    assert lib.pdnqp_batch_last_report(ctypes.byref(rep), None, 0) == 0
    assert lib.pdnqp_mlp_forward(None, None, 1, None) == -1
    th = np.zeros(P.MLP_PARAMS, dtype=np.float32)
    x = np.zeros(16, dtype=np.float32)
    y = np.zeros(3, dtype=np.float32)
    assert lib.pdnqp_mlp_forward(th.ctypes.data, x.ctypes.data, 0, y.ctypes.data) == -1
    assert lib.pdnqp_mlp_gradient(th.ctypes.data, x.ctypes.data, None, 1, None, None) == -1
    assert lib.pdnqp_mlp_train(th.ctypes.data, x.ctypes.data, y.ctypes.data, 1, 1, 0,
                               ctypes.c_float(1e-3), 0, None) == -1
    assert lib.pdnqp_set_controller(None, th.ctypes.data) == -1
    assert lib.pdnqp_get_outer_log(None, None, None, None) == -1


def test_one_hip_runtime_with_torch():
    """Loading the library and then importing PyTorch maps one HIP runtime
    (a second one would split device pointers and streams between
    runtimes).  Runs in a fresh interpreter: the load order is what is
    tested."""
    import subprocess
    import sys
    code = ("import paper_2609_19557_amd as P; P.load(); import torch, re; "
            "maps = open('/proc/self/maps').read(); "
            "libs = sorted({m for m in re.findall(r'/\\S*libamdhip64\\S*', maps)}); "
            "print(len(libs), libs)")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.startswith("1 "), out.stdout
