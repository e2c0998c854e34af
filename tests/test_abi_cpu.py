"""CPU-side checks of the C-ABI library: it loads and exports every entry
point include/hipcone.h declares (no compute calls: there is no GPU here)."""
import os
import re

import pytest

from paper_2412_19027_amd import hipcone

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hipcone.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int32_t|void|const char\*)\s+(hc_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_binding_exports():
    assert set(declared_functions()) == set(hipcone.EXPORTS)


@pytest.mark.skipif(not os.path.exists(hipcone.LIB_PATH), reason="libhipcone.so not built")
def test_library_exports_every_declared_symbol():
    L = hipcone.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


@pytest.mark.skipif(not os.path.exists(hipcone.LIB_PATH), reason="libhipcone.so not built")
def test_settings_defaults_and_status_strings():
    st = hipcone.default_settings()
    assert st.eps_feas == 1e-8 and st.max_iter == 200 and st.ir_max == 10 and st.backtrack == 0.8
    assert hipcone.lib().hc_status_str(1) == b"solved"


@pytest.mark.skipif(not os.path.exists(hipcone.LIB_PATH), reason="libhipcone.so not built")
def test_setup_validation_errors_on_host():
    """hc_setup validates on the host without touching a device."""
    import ctypes as C
    import numpy as np
    L = hipcone.lib()
    rp = np.array([0, 1, 2], dtype=np.int64)
    ci = np.array([0, 0], dtype=np.int32)
    v = np.array([1.0, np.nan])
    q = np.zeros(1)
    b = np.zeros(2)
    cones = (hipcone.hc_cone * 1)(hipcone.hc_cone(1, 2, 0.0))
    pr = hipcone.hc_problem(1, 2, None, None, None, q.ctypes.data_as(C.POINTER(C.c_double)),
                            rp.ctypes.data_as(C.POINTER(C.c_int64)), ci.ctypes.data_as(C.POINTER(C.c_int32)),
                            v.ctypes.data_as(C.POINTER(C.c_double)), b.ctypes.data_as(C.POINTER(C.c_double)), cones, 1)
    h = C.c_void_p()
    assert L.hc_setup(C.byref(h), C.byref(pr), None) == -5          # HC_ERR_NONFINITE
    v[1] = 2.0
    cones[0] = hipcone.hc_cone(1, 3, 0.0)
    assert L.hc_setup(C.byref(h), C.byref(pr), None) == -2          # rows do not add up
    cones[0] = hipcone.hc_cone(2, 2, 0.0)
    assert L.hc_setup(C.byref(h), C.byref(pr), None) == 0
    L.hc_destroy(h)


def test_two_level_split_on_host():
    """The host analysis splits the logistic-regression Schur complement into
    one leaf per sample and per |theta_j| <= r_j pair, with theta as the dense
    tail; dense-coupled problems stay one dense block."""
    from paper_2412_19027_amd import workloads as W
    N, F = 400, 30
    p = W.logreg_exp(0, samples=N, features=F)
    a = hipcone.analyze(p)
    assert a["n_ordered"] == F                     # theta
    assert a["n_leaves"] == N + F                  # (t, w1, w2) per sample, r_j per feature
    assert a["leaf_columns"] == p.n - F
    off = hipcone.analyze(p, leaf_blocks=0)
    assert off["n_ordered"] == p.n and off["n_leaves"] == 0
    assert off["factor_flops"] > 100 * a["factor_flops"]
    socp = W.sparse_socp(0, nx=600, rank=5, n_zero=150, n_nonneg=400, n_soc=500)
    s = hipcone.analyze(socp)                      # the dense factor rows touch every column
    assert s["n_ordered"] == socp.n and s["n_leaves"] == 0


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors have the sizes the C compiler gives the header's structs."""
    import ctypes as C
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include "hipcone.h"\nint main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n",'
                   'sizeof(hc_settings), sizeof(hc_info), sizeof(hc_problem), sizeof(hc_device),'
                   'sizeof(hc_server_config), sizeof(hc_result), sizeof(hc_server_report));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    want = [C.sizeof(t) for t in (hipcone.hc_settings, hipcone.hc_info, hipcone.hc_problem, hipcone.hc_device,
                                  hipcone.hc_server_config, hipcone.hc_result, hipcone.hc_server_report)]
    assert got == want


def test_update_data_on_host():
    """hc_update_data recomputes the scaled data on the host (no device
    bound): new values of the same structure are accepted, non-finite values
    are rejected with HC_ERR_NONFINITE, and an unchanged update leaves the
    analysis the same."""
    import ctypes as C
    import numpy as np
    from paper_2412_19027_amd import workloads as W
    L = hipcone.lib()
    a, b = W.mpc_socp(0, 0, T=12, nx=5, nu=3), W.mpc_socp(1, 0, T=12, nx=5, nu=3)
    h, keep = hipcone._setup(a, hipcone.default_settings())
    try:
        before = hipcone.hc_info()
        assert L.hc_get_info(h, C.byref(before)) == 0
        Pb, Ab = b.P.tocsr(), b.A.tocsr()
        Pv = np.ascontiguousarray(Pb.data, dtype=np.float64)
        Av = np.ascontiguousarray(Ab.data, dtype=np.float64)
        q = np.ascontiguousarray(b.q, dtype=np.float64)
        bb = np.ascontiguousarray(b.b, dtype=np.float64)
        assert L.hc_update_data(h, Pv.ctypes.data, q.ctypes.data, Av.ctypes.data, bb.ctypes.data) == 0
        bad = bb.copy()
        bad[3] = np.inf
        assert L.hc_update_data(h, None, None, None, bad.ctypes.data) == -5   # HC_ERR_NONFINITE
        assert L.hc_update_data(h, None, None, None, None) == 0
        after = hipcone.hc_info()
        assert L.hc_get_info(h, C.byref(after)) == 0
        assert (after.n_ordered, after.n_leaves) == (before.n_ordered, before.n_leaves)
    finally:
        L.hc_destroy(h)


def test_large_soc_setup_on_host():
    """Second-order cones above 16 rows: the host analysis accepts them, keeps
    every column they touch in the dense tail (their rank-2 rows are dense
    there) and leaves the z variables of the multistage problem as leaves."""
    import ctypes as C
    from paper_2412_19027_amd import workloads as W
    L = hipcone.lib()
    n, k, T = 40, 4, 3
    prob = W.multistage_portfolio(0, n=n, k=k, T=T)
    h, keep = hipcone._setup(prob, hipcone.default_settings())
    try:
        inf = hipcone.hc_info()
        assert L.hc_get_info(h, C.byref(inf)) == 0
        assert inf.n_ordered == T * (n + k + 1) and inf.n_leaves == T * n
        nb = C.c_size_t()
        assert L.hc_workspace_bytes(h, C.byref(nb)) == 0 and nb.value > 0
    finally:
        L.hc_destroy(h)


def test_cone_size_limits_on_host():
    """PSD sides 1..32 are accepted (33 is HC_ERR_CONE, as in the paper's
    limit); second-order cones of any dimension up to 2^24 are accepted."""
    import scipy.sparse as sp
    from paper_2412_19027_amd.workloads import PSD, SOC, Problem
    from tests import problems_small as PS
    for k in (12, 13, 32):
        prob, _ = PS.trace_min(0, k=k)
        info = hipcone.analyze(prob)
        assert info["n_ordered"] == k * (k + 1) // 2
    k = 33
    sd = k * (k + 1) // 2
    bad = Problem(sd, sd, sp.csr_matrix((sd, sd)), [0.0] * sd, -sp.identity(sd, format="csr"), [0.0] * sd,
                  [(PSD, k, 0.0)], "psd33")
    with pytest.raises(hipcone.HipconeError) as e:
        hipcone.analyze(bad)
    assert e.value.code == -4   # HC_ERR_CONE
    prob, _ = PS.soc_ball(0, n=5000)
    assert hipcone.analyze(prob)["n_ordered"] == 5000
