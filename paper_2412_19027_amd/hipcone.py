"""Python binding of the hipcone C-ABI (include/hipcone.h): argument marshalling only.

Every step of the interior-point method runs in libhipcone.so's HIP kernels;
PyTorch supplies the device arena and the stream.  The library must be built
in-tree first (`python -m paper_2412_19027_amd.build`); importing the binding
without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhipcone.so")

ZERO, NONNEG, SOC, EXP, POW, PSD = 0, 1, 2, 3, 4, 5
PRECISION_FP64, PRECISION_MIXED = 0, 1
STATUS = {0: "unsolved", 1: "solved", 2: "primal_infeasible", 3: "dual_infeasible", 4: "max_iter",
          5: "insufficient_progress", 6: "numerical_error", 7: "cancelled"}

EXPORTS = ["hc_settings_default", "hc_setup", "hc_workspace_bytes", "hc_bind", "hc_solve", "hc_get_info",
           "hc_get_solution", "hc_solve_noalloc", "hc_host_stage_bytes", "hc_batch_check", "hc_solve_batch", "hc_get_iterate", "hc_set_iterate", "hc_update_data", "hc_test_kkt_solve", "hc_test_kkt_ops",
           "hc_test_schur", "hc_destroy", "hc_last_error", "hc_status_str",
           "hc_test_cone_scale", "hc_test_cone_ds", "hc_test_cone_step", "hc_test_cone_step_min", "hc_test_dense_chol_solve",
           "hc_test_dense_chol_solve_env",
           "hc_test_copy", "hc_test_symbolic", "hc_test_ordered_sums", "hc_test_cone_mblock", "hc_server_config_default", "hc_server_create", "hc_server_submit", "hc_server_poll",
           "hc_server_wait", "hc_server_stats", "hc_server_destroy"]


class hc_cone(C.Structure):
    _fields_ = [("type", C.c_int32), ("dim", C.c_int32), ("alpha", C.c_double)]


class hc_problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64),
                ("P_rowptr", C.POINTER(C.c_int64)), ("P_col", C.POINTER(C.c_int32)), ("P_val", C.POINTER(C.c_double)),
                ("q", C.POINTER(C.c_double)),
                ("A_rowptr", C.POINTER(C.c_int64)), ("A_col", C.POINTER(C.c_int32)), ("A_val", C.POINTER(C.c_double)),
                ("b", C.POINTER(C.c_double)),
                ("cones", C.POINTER(hc_cone)), ("ncones", C.c_int32)]


class hc_settings(C.Structure):
    _fields_ = [("eps_feas", C.c_double), ("eps_inf", C.c_double), ("max_iter", C.c_int32),
                ("precision", C.c_int32), ("static_reg", C.c_double), ("dyn_reg", C.c_double),
                ("ir_abstol", C.c_double), ("ir_reltol", C.c_double), ("ir_max", C.c_int32),
                ("beta", C.c_double), ("backtrack", C.c_double), ("step_fraction", C.c_double),
                ("equilibrate", C.c_int32), ("equil_iters", C.c_int32), ("force_dual_scaling", C.c_int32),
                ("verbose", C.c_int32), ("profile", C.c_int32), ("leaf_blocks", C.c_int32),
                ("warm_start", C.c_int32), ("warm_blend", C.c_double), ("ir_mu_frac", C.c_double)]


class hc_device(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("stream", C.c_void_p),
                ("device", C.c_int32), ("host_stage", C.c_void_p), ("host_stage_bytes", C.c_size_t)]


class hc_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("obj_primal", C.c_double),
                ("obj_dual", C.c_double), ("res_primal", C.c_double), ("res_dual", C.c_double),
                ("gap", C.c_double), ("mu", C.c_double), ("setup_ms", C.c_double), ("solve_ms", C.c_double),
                ("factor_ms", C.c_double), ("solve_kkt_ms", C.c_double), ("cone_ms", C.c_double),
                ("ir_solves", C.c_int64), ("pivot_guard_hits", C.c_int64), ("dual_switches", C.c_int64),
                ("n_ordered", C.c_int64), ("factor_flops", C.c_double), ("factorizations", C.c_int64),
                ("gemm_ms", C.c_double), ("gemm_flops", C.c_double), ("gemm_launches", C.c_int64),
                ("fp64_fallbacks", C.c_int64), ("n_leaves", C.c_int64), ("leaf_columns", C.c_int64),
                ("psd_gathered_rows", C.c_int64), ("cone_kernel_ms", C.c_double), ("cone_bytes", C.c_double),
                ("cone_launches", C.c_int64), ("sym_split_columns", C.c_int64), ("sym_supernodes", C.c_int64),
                ("sym_levels", C.c_int64), ("sym_nnz_l", C.c_int64)]


class hc_server_config(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_int32), ("workers", C.c_int32),
                ("settings", hc_settings), ("device", C.c_int32), ("batched", C.c_int32),
                ("batch_slots", C.c_int32), ("pool", C.c_void_p)]


class hc_result(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("status", C.c_int32), ("error", C.c_int32), ("iterations", C.c_int32),
                ("obj_primal", C.c_double), ("obj_dual", C.c_double), ("res_primal", C.c_double),
                ("res_dual", C.c_double), ("queue_ms", C.c_double), ("solve_ms", C.c_double),
                ("latency_ms", C.c_double), ("n", C.c_int64), ("m", C.c_int64),
                ("x", C.POINTER(C.c_double)), ("s", C.POINTER(C.c_double)), ("z", C.POINTER(C.c_double))]


class hc_server_report(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("cancelled", C.c_int64), ("active", C.c_int64), ("pending", C.c_int64), ("iterations", C.c_int64),
                ("p50_latency_ms", C.c_double), ("p99_latency_ms", C.c_double), ("mean_latency_ms", C.c_double),
                ("solves_per_s", C.c_double), ("busy_ms", C.c_double), ("hbm_in_use", C.c_size_t),
                ("hbm_peak", C.c_size_t)]


HC_PENDING = 1
ERR_UNSUPPORTED = -9
ERR_TOO_LARGE = -10
NOALLOC_BYTES = 64 << 20     # the static device workspace of hc_solve_noalloc (HC_NOALLOC_BYTES)

_lib = None


def lib():
    """Load libhipcone.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2412_19027_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.hc_settings_default.argtypes = [C.POINTER(hc_settings)]
        L.hc_setup.argtypes = [C.POINTER(vp), C.POINTER(hc_problem), C.POINTER(hc_settings)]
        L.hc_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.hc_bind.argtypes = [vp, C.POINTER(hc_device)]
        L.hc_solve.argtypes = [vp]
        L.hc_get_info.argtypes = [vp, C.POINTER(hc_info)]
        L.hc_get_solution.argtypes = [vp, vp, vp, vp, i32]
        L.hc_solve_noalloc.argtypes = [vp, vp, i32, vp, vp, vp, C.POINTER(hc_info)]
        L.hc_test_symbolic.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(i32), C.POINTER(i32)]
        L.hc_test_ordered_sums.argtypes = [vp, C.POINTER(i32), vp]
        L.hc_host_stage_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.hc_batch_check.argtypes = [vp, C.POINTER(i32)]
        L.hc_solve_batch.argtypes = [vp, i32, vp, i32, vp]
        L.hc_get_iterate.argtypes = [vp, vp, vp, vp, C.POINTER(dbl), C.POINTER(dbl), vp]
        L.hc_set_iterate.argtypes = [vp, vp, vp, vp, dbl, dbl]
        L.hc_update_data.argtypes = [vp, vp, vp, vp, vp]
        L.hc_test_kkt_solve.argtypes = [vp, dbl, C.c_int32, vp, vp, vp, vp, vp]
        L.hc_test_schur.argtypes = [vp, dbl, C.c_int32, vp, vp, vp]
        L.hc_test_kkt_ops.argtypes = [vp, dbl, C.c_int32, vp, vp, vp, vp, vp, vp]
        L.hc_destroy.argtypes = [vp]
        L.hc_destroy.restype = None
        L.hc_last_error.argtypes = [vp]
        L.hc_last_error.restype = C.c_char_p
        L.hc_status_str.argtypes = [i32]
        L.hc_status_str.restype = C.c_char_p
        L.hc_test_cone_scale.argtypes = [i32, i64, i32, vp, vp, vp, dbl, i32, vp, vp, vp, vp]
        L.hc_test_cone_ds.argtypes = [i32, i64, i32, vp, vp, vp, vp, vp, dbl, i32, dbl, vp, vp]
        L.hc_test_cone_step.argtypes = [i32, i64, i32, vp, vp, vp, vp, vp, dbl, vp, vp]
        L.hc_test_cone_step_min.argtypes = [i32, i64, i32, vp, vp, vp, vp, vp, C.POINTER(dbl), vp]
        L.hc_test_dense_chol_solve.argtypes = [i32, i64, i64, vp, i32, vp, C.POINTER(i64), vp]
        L.hc_test_dense_chol_solve_env.argtypes = [i32, i64, i64, vp, vp, i32, vp, C.POINTER(i64), vp]
        L.hc_test_copy.argtypes = [vp, vp, i64, vp]
        L.hc_test_cone_mblock.argtypes = [i32, i64, i32, vp, vp, vp, C.c_double, i32, C.c_double, vp, vp]
        L.hc_server_config_default.argtypes = [C.POINTER(hc_server_config)]
        L.hc_server_create.argtypes = [C.POINTER(vp), C.POINTER(hc_server_config)]
        L.hc_server_submit.argtypes = [vp, C.POINTER(hc_problem), C.c_uint64, C.POINTER(C.c_uint64)]
        L.hc_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(hc_result)]
        L.hc_server_wait.argtypes = [vp, C.c_uint64, C.POINTER(hc_result)]
        L.hc_server_stats.argtypes = [vp, C.POINTER(hc_server_report)]
        L.hc_server_destroy.argtypes = [vp]
        L.hc_server_destroy.restype = None
        for name in EXPORTS:
            getattr(L, name)
        _lib = L
    return _lib


class HipconeError(RuntimeError):
    pass


def _check(rc, handle=None):
    if rc != 0:
        msg = lib().hc_last_error(handle).decode(errors="replace")
        err = HipconeError(f"hipcone error {rc}: {msg}")
        err.code = rc
        raise err


def default_settings(**overrides) -> hc_settings:
    st = hc_settings()
    _check(lib().hc_settings_default(C.byref(st)))
    for k, v in overrides.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISION_MIXED if v == "mixed" else PRECISION_FP64
        setattr(st, k, v)
    return st


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _problem(prob):
    """hc_problem view of a workloads.Problem: (struct, buffers kept alive for it)."""
    P = prob.P.tocsr()
    A = prob.A.tocsr()
    keep = dict(
        Prp=np.ascontiguousarray(P.indptr, dtype=np.int64), Pci=np.ascontiguousarray(P.indices, dtype=np.int32),
        Pv=np.ascontiguousarray(P.data, dtype=np.float64), q=np.ascontiguousarray(prob.q, dtype=np.float64),
        Arp=np.ascontiguousarray(A.indptr, dtype=np.int64), Aci=np.ascontiguousarray(A.indices, dtype=np.int32),
        Av=np.ascontiguousarray(A.data, dtype=np.float64), b=np.ascontiguousarray(prob.b, dtype=np.float64))
    cones = (hc_cone * len(prob.cones))(*[hc_cone(int(k), int(d), float(a)) for k, d, a in prob.cones])
    keep["cones"] = cones
    k = keep
    pr = hc_problem(prob.n, prob.m, _ptr(k["Prp"], C.c_int64), _ptr(k["Pci"], C.c_int32), _ptr(k["Pv"], C.c_double),
                    _ptr(k["q"], C.c_double), _ptr(k["Arp"], C.c_int64), _ptr(k["Aci"], C.c_int32),
                    _ptr(k["Av"], C.c_double), _ptr(k["b"], C.c_double), cones, len(prob.cones))
    return pr, keep


def _setup(prob, settings):
    """hc_setup on the host: returns (handle, buffers kept alive for it)."""
    pr, keep = _problem(prob)
    h = C.c_void_p()
    _check(lib().hc_setup(C.byref(h), C.byref(pr), C.byref(settings)))
    return h, keep


def analyze(prob, **settings) -> dict:
    """Host-only setup (no device): the hc_info fields known after the
    analysis (n_ordered, n_leaves, leaf_columns, factor_flops) and the device
    workspace in bytes."""
    L = lib()
    h, _ = _setup(prob, default_settings(**settings))
    try:
        nbytes = C.c_size_t()
        _check(L.hc_workspace_bytes(h, C.byref(nbytes)), h)
        inf = hc_info()
        _check(L.hc_get_info(h, C.byref(inf)), h)
        out = {f: getattr(inf, f) for f, _ in hc_info._fields_}
        out["workspace_bytes"] = int(nbytes.value)
        return out
    finally:
        L.hc_destroy(h)


def solve_noalloc(prob, device=0, stream=None, **settings):
    """hc_solve_noalloc: set-up on the host, then the solve in the library's
    static device workspace (no device or pinned allocation); returns (info,
    x, s, z) with the solution in host arrays.  stream: a torch stream of the
    device (default: its current stream)."""
    import torch
    L = lib()
    h, keep = _setup(prob, default_settings(**settings))
    try:
        st = stream if stream is not None else torch.cuda.current_stream(device)
        x, s, z = np.zeros(prob.n), np.zeros(prob.m), np.zeros(prob.m)
        inf = hc_info()
        _check(L.hc_solve_noalloc(h, st.cuda_stream, int(device), x.ctypes.data, s.ctypes.data, z.ctypes.data,
                                  C.byref(inf)), h)
        out = {f: getattr(inf, f) for f, _ in hc_info._fields_}
        out["status_name"] = STATUS.get(inf.status, "unknown")
        return out, x, s, z
    finally:
        L.hc_destroy(h)


def ordered_sums_check(prob, **settings) -> dict:
    """hc_test_ordered_sums on a set-up handle (host only): the ordered Schur
    sums against every product added where it lands."""
    h, _ = _setup(prob, default_settings(**settings))
    try:
        flag = C.c_int32()
        out = np.zeros(3)
        _check(lib().hc_test_ordered_sums(h, C.byref(flag), out.ctypes.data), h)
        return {"ordered": bool(flag.value), "rel_diff": float(out[0]), "bad_slots": int(out[1]),
                "destinations": int(out[2])}
    finally:
        lib().hc_destroy(h)


def symbolic(n, ptr, adj):
    """The setup's symbolic analysis of a symmetric graph (host only):
    dict with order, parent, count (numpy arrays), supernodes (first, parent,
    level) and nlevels."""
    ptr = np.ascontiguousarray(ptr, dtype=np.int64)
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    order = np.zeros(n, np.int32)
    parent = np.zeros(n, np.int32)
    count = np.zeros(n, np.int64)
    first = np.zeros(n + 1, np.int32)
    sp = np.zeros(max(n, 1), np.int32)
    sl = np.zeros(max(n, 1), np.int32)
    ns, nl = C.c_int32(), C.c_int32()
    _check(lib().hc_test_symbolic(int(n), ptr.ctypes.data, adj.ctypes.data, order.ctypes.data, parent.ctypes.data,
                                  count.ctypes.data, first.ctypes.data, sp.ctypes.data, sl.ctypes.data,
                                  C.byref(ns), C.byref(nl)))
    k = ns.value
    return dict(order=order, parent=parent, count=count, sn_first=first[:k + 1], sn_parent=sp[:k],
                sn_level=sl[:k], nlevels=nl.value)


def batch_band(prob, **settings):
    """Band half-width of the problem's Schur complement under the batched
    engine's ordering, or None when the engine does not take it."""
    L = lib()
    h, keep = _setup(prob, default_settings(**settings))
    try:
        w = C.c_int32(0)
        rc = L.hc_batch_check(h, C.byref(w))
        return int(w.value) if rc == 0 else None
    finally:
        L.hc_destroy(h)


def solve_batch(probs, device=0, stream=None, **settings):
    """Solves a list of problems together on the batched engine (one
    wavefront per problem).  Returns a list of result dicts with x, s, z."""
    import torch
    L = lib()
    handles, keeps = [], []
    try:
        for p in probs:
            h, k = _setup(p, default_settings(**settings))
            handles.append(h)
            keeps.append(k)
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        res = (hc_result * len(probs))()
        outs = []
        for i, p in enumerate(probs):
            x, s, z = np.zeros(p.n), np.zeros(p.m), np.zeros(p.m)
            outs.append((x, s, z))
            res[i].x = _ptr(x, C.c_double)
            res[i].s = _ptr(s, C.c_double)
            res[i].z = _ptr(z, C.c_double)
        arr = (C.c_void_p * len(handles))(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
        _check(L.hc_solve_batch(arr, len(handles), st.cuda_stream, dev.index or 0, res))
        out = []
        for i in range(len(probs)):
            r = {f: getattr(res[i], f) for f, _ in hc_result._fields_ if f not in ("x", "s", "z")}
            r["status_name"] = STATUS.get(r["status"], "unknown")
            r["x"], r["s"], r["z"] = outs[i]
            out.append(r)
        return out
    finally:
        for h in handles:
            L.hc_destroy(h)


class Solver:
    """One problem on one GPU.  `prob` is a workloads.Problem (or any object
    with n, m, P (upper CSR), q, A (CSR), b, cones)."""

    def __init__(self, prob, device=0, stream=None, pinned_stage=False, **settings):
        """With pinned_stage the read-back staging is a pinned host buffer of
        hc_host_stage_bytes owned by this object (as the served form's workers
        pass theirs) instead of one the library allocates."""
        import torch
        self._torch = torch
        L = lib()
        self.settings = default_settings(**settings)
        self.n, self.m = prob.n, prob.m
        h, self._keep = _setup(prob, self.settings)
        self._h = h
        self._nnzP, self._nnzA = len(self._keep["Pv"]), len(self._keep["Av"])
        nbytes = C.c_size_t()
        _check(L.hc_workspace_bytes(h, C.byref(nbytes)), h)
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.arena = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        stage, stage_bytes = None, 0
        if pinned_stage:
            sb = C.c_size_t()
            _check(L.hc_host_stage_bytes(h, C.byref(sb)), h)
            self.stage = torch.empty(int(sb.value), dtype=torch.uint8, pin_memory=True)
            stage, stage_bytes = self.stage.data_ptr(), int(sb.value)
        dev = hc_device(self.arena.data_ptr(), int(nbytes.value), self.stream.cuda_stream, self.device.index or 0,
                        stage, stage_bytes)
        _check(L.hc_bind(h, C.byref(dev)), h)

    def solve(self):
        _check(lib().hc_solve(self._h), self._h)
        return self.info()

    def info(self) -> dict:
        inf = hc_info()
        _check(lib().hc_get_info(self._h, C.byref(inf)), self._h)
        out = {f: getattr(inf, f) for f, _ in hc_info._fields_}
        out["status_name"] = STATUS.get(inf.status, "unknown")
        return out

    def solution(self, on_device=False):
        """x, s, z in the user's coordinates (divided by tau; the certificate
        for an infeasible status): numpy arrays, or torch cuda tensors written
        on the device when on_device."""
        if on_device:
            torch = self._torch
            x = torch.empty(self.n, dtype=torch.float64, device=self.device)
            s = torch.empty(self.m, dtype=torch.float64, device=self.device)
            z = torch.empty(self.m, dtype=torch.float64, device=self.device)
            _check(lib().hc_get_solution(self._h, x.data_ptr(), s.data_ptr(), z.data_ptr(), 1), self._h)
            return x, s, z
        x = np.zeros(self.n)
        s = np.zeros(self.m)
        z = np.zeros(self.m)
        _check(lib().hc_get_solution(self._h, x.ctypes.data, s.ctypes.data, z.ctypes.data, 0), self._h)
        return x, s, z

    def iterate(self):
        x = np.zeros(self.n)
        s = np.zeros(self.m)
        z = np.zeros(self.m)
        perm = np.zeros(self.m, dtype=np.int64)
        tau, kappa = C.c_double(), C.c_double()
        _check(lib().hc_get_iterate(self._h, x.ctypes.data, s.ctypes.data, z.ctypes.data, C.byref(tau),
                                    C.byref(kappa), perm.ctypes.data), self._h)
        return x, s, z, tau.value, kappa.value, perm

    def update_data(self, P_val=None, q=None, A_val=None, b=None):
        """New values for a problem of the same structure (hc_update_data); None keeps an array."""
        keep = []

        def ptr(v, size):
            if v is None:
                return None
            a = np.ascontiguousarray(v, dtype=np.float64)
            assert a.shape == (size,), (a.shape, size)
            keep.append(a)
            return a.ctypes.data
        _check(lib().hc_update_data(self._h, ptr(P_val, self._nnzP), ptr(q, self.n), ptr(A_val, self._nnzA),
                                    ptr(b, self.m)), self._h)

    def set_iterate(self, x, s, z, tau, kappa):
        """Replace the internal iterate (internal order and scaling, as `iterate()` returns it)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        s = np.ascontiguousarray(s, dtype=np.float64)
        z = np.ascontiguousarray(z, dtype=np.float64)
        assert x.shape == (self.n,) and s.shape == (self.m,) and z.shape == (self.m,)
        _check(lib().hc_set_iterate(self._h, x.ctypes.data, s.ctypes.data, z.ctypes.data, float(tau), float(kappa)),
               self._h)

    def test_kkt_solve(self, mu, r1, r2, force_dual=False):
        """One KKT solve at the current iterate (hc_test_kkt_solve); returns x, z, stats dict."""
        r1 = np.ascontiguousarray(r1, dtype=np.float64)
        r2 = np.ascontiguousarray(r2, dtype=np.float64)
        assert r1.shape == (self.n,) and r2.shape == (self.m,)
        x = np.zeros(self.n)
        z = np.zeros(self.m)
        st = np.zeros(4)
        _check(lib().hc_test_kkt_solve(self._h, float(mu), int(bool(force_dual)), r1.ctypes.data, r2.ctypes.data,
                                       x.ctypes.data, z.ctypes.data, st.ctypes.data), self._h)
        return x, z, {"solves": int(st[0]), "delta": st[1], "pd_scaled": int(st[2]), "fp64_refactor": int(st[3])}

    def test_kkt_ops(self, mu, r1, r2, force_dual=False):
        """One regularised solve and the unregularised product K [xr; zr] (hc_test_kkt_ops)."""
        r1 = np.ascontiguousarray(r1, dtype=np.float64)
        r2 = np.ascontiguousarray(r2, dtype=np.float64)
        assert r1.shape == (self.n,) and r2.shape == (self.m,)
        xr, kx = np.zeros(self.n), np.zeros(self.n)
        zr, kz = np.zeros(self.m), np.zeros(self.m)
        _check(lib().hc_test_kkt_ops(self._h, float(mu), int(bool(force_dual)), r1.ctypes.data, r2.ctypes.data,
                                     xr.ctypes.data, zr.ctypes.data, kx.ctypes.data, kz.ctypes.data), self._h)
        return xr, zr, kx, kz

    def test_schur(self, mu, force_dual=False, factor=True):
        """Schur complement at the current iterate and its Cholesky factor
        (hc_test_schur; lower triangles, requires leaf_blocks=0)."""
        S = np.zeros((self.n, self.n), order="F")
        L = np.zeros((self.n, self.n), order="F") if factor else None
        st = np.zeros(3)
        _check(lib().hc_test_schur(self._h, float(mu), int(bool(force_dual)), S.ctypes.data,
                                   L.ctypes.data if factor else None, st.ctypes.data), self._h)
        S = np.tril(S)
        S = S + np.tril(S, -1).T
        return S, (np.tril(L) if factor else None), {"delta": st[0], "pd_scaled": int(st[1]), "bits": int(st[2])}

    def close(self):
        if getattr(self, "_h", None):
            lib().hc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# kernel test entry points (device tensors)
# --------------------------------------------------------------------------
def _dptr(t):
    return None if t is None else t.data_ptr()


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def test_cone_scale(kind, dim, s, z, mu, alpha=None, force_dual=False):
    """Scaling of `count` cones given cone by cone (torch cuda float64, shape (count, rows))."""
    import torch
    count, rows = s.shape
    H = torch.zeros((count, rows, rows), dtype=torch.float64, device=s.device)
    lam = torch.zeros((count, rows), dtype=torch.float64, device=s.device)
    br = torch.zeros(count, dtype=torch.int32, device=s.device)
    _check(lib().hc_test_cone_scale(kind, count, dim, _dptr(alpha), _dptr(s.contiguous()), _dptr(z.contiguous()),
                                    float(mu), int(bool(force_dual)), _dptr(H), _dptr(lam), _dptr(br), _stream()))
    torch.cuda.synchronize()
    return H, lam, br


def test_cone_mblock(kind, dim, s, z, mu, delta, alpha=None, force_dual=False):
    """Explicit M = (H + delta I)^-1 blocks used in the Schur assembly, (count, rows, rows)."""
    import torch
    count, rows = s.shape
    M = torch.zeros((count, rows, rows), dtype=torch.float64, device=s.device)
    _check(lib().hc_test_cone_mblock(kind, count, dim, _dptr(alpha), _dptr(s.contiguous()), _dptr(z.contiguous()),
                                     float(mu), int(bool(force_dual)), float(delta), _dptr(M), _stream()))
    torch.cuda.synchronize()
    return M


def test_cone_ds(kind, dim, s, z, dsa, dza, mu, sm, alpha=None, force_dual=False):
    import torch
    out = torch.zeros_like(s)
    _check(lib().hc_test_cone_ds(kind, s.shape[0], dim, _dptr(alpha), _dptr(s.contiguous()), _dptr(z.contiguous()),
                                 _dptr(dsa.contiguous()), _dptr(dza.contiguous()), float(mu), int(bool(force_dual)),
                                 float(sm), _dptr(out),
                                 _stream()))
    torch.cuda.synchronize()
    return out


def test_cone_step(kind, dim, s, z, ds, dz, amax, alpha=None):
    import torch
    out = torch.zeros(s.shape[0], dtype=torch.float64, device=s.device)
    _check(lib().hc_test_cone_step(kind, s.shape[0], dim, _dptr(alpha), _dptr(s.contiguous()), _dptr(z.contiguous()),
                                   _dptr(ds.contiguous()), _dptr(dz.contiguous()), float(amax), _dptr(out), _stream()))
    torch.cuda.synchronize()
    return out


def test_cone_step_min(kind, dim, s, z, ds, dz, alpha=None):
    """Minimum over all cones of the exact boundary step, by the solver's own
    step-length launch (nonneg, SOC, PSD)."""
    import torch
    out = C.c_double(0.0)
    _check(lib().hc_test_cone_step_min(kind, s.shape[0], dim, _dptr(alpha), _dptr(s.contiguous()),
                                       _dptr(z.contiguous()), _dptr(ds.contiguous()), _dptr(dz.contiguous()),
                                       C.byref(out), _stream()))
    torch.cuda.synchronize()
    return out.value


def test_dense_chol_solve(A, B, precision=PRECISION_FP64, ld=None, last=None):
    """A: (n, n) SPD (torch cuda float64); B: (n, nrhs).  A is stored
    column-major with leading dimension ld (default n) as the library keeps
    its Schur complement.  `last` (int sequence, optional): the envelope of A
    (hc_test_dense_chol_solve_env).  Returns (X, L, pivot-guard hits)."""
    import numpy as np
    import torch
    n = A.shape[0]
    ld = n if ld is None else int(ld)
    At = torch.zeros((n, ld), dtype=A.dtype, device=A.device)   # row j = column j of the matrix
    At[:, :n] = A.t()
    Bt = B.t().contiguous()          # column-major (n x nrhs)
    hits = C.c_int64()
    if last is None:
        _check(lib().hc_test_dense_chol_solve(precision, n, ld, _dptr(At), Bt.shape[0], _dptr(Bt), C.byref(hits),
                                              _stream()))
    else:
        env = np.ascontiguousarray(last, dtype=np.int64)
        _check(lib().hc_test_dense_chol_solve_env(precision, n, ld, _dptr(At), env.ctypes.data, Bt.shape[0],
                                                  _dptr(Bt), C.byref(hits), _stream()))
    torch.cuda.synchronize()
    return Bt.t().contiguous(), At[:, :n].t().contiguous(), hits.value


def test_copy(src, dst):
    """Reference copy kernel: dst[:] = src[:] (torch cuda tensors of equal byte size)."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    _check(lib().hc_test_copy(_dptr(src), _dptr(dst), nbytes, _stream()))


class Server:
    """Continuous-batching server (hc_server_*): many problems in flight on one
    GPU, admitted by device-memory footprint."""

    def __init__(self, hbm_budget_bytes=64 << 30, max_slots=64, workers=4, device=0, batched=True,
                 batch_slots=1024, pool=None, **settings):
        """pool: a caller-owned device buffer (e.g. a torch uint8 tensor) of at
        least hbm_budget_bytes to carve the workspaces from; it must outlive
        close()."""
        L = lib()
        cfg = hc_server_config()
        _check(L.hc_server_config_default(C.byref(cfg)))
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.max_slots = int(max_slots)
        cfg.workers = int(workers)
        cfg.device = int(device)
        cfg.batched = 1 if batched else 0
        cfg.batch_slots = int(batch_slots)
        cfg.settings = default_settings(**settings)
        if pool is not None:
            if pool.numel() * pool.element_size() < cfg.hbm_budget_bytes:
                raise ValueError("pool smaller than hbm_budget_bytes")
            cfg.pool = pool.data_ptr()
            self._pool = pool
        self._h = C.c_void_p()
        _check(L.hc_server_create(C.byref(self._h), C.byref(cfg)))
        self._shapes = {}

    def submit(self, prob, tag=0):
        """Queues `prob` (copied); returns its ticket."""
        pr, _keep = _problem(prob)
        t = C.c_uint64()
        _check(lib().hc_server_submit(self._h, C.byref(pr), int(tag), C.byref(t)))
        self._shapes[t.value] = (prob.n, prob.m)
        return t.value

    def _result(self, fn, ticket, solution):
        n, m = self._shapes[ticket]
        r = hc_result()
        bufs = None
        if solution:
            bufs = (np.zeros(n), np.zeros(m), np.zeros(m))
            r.x, r.s, r.z = (_ptr(b, C.c_double) for b in bufs)
        rc = fn(self._h, C.c_uint64(ticket), C.byref(r))
        if rc == HC_PENDING:
            return None
        _check(rc)
        del self._shapes[ticket]
        out = {f: getattr(r, f) for f, _ in hc_result._fields_ if f not in ("x", "s", "z")}
        out["status_name"] = STATUS.get(r.status, "unknown")
        if solution:
            out["x"], out["s"], out["z"] = bufs
        return out

    def poll(self, ticket, solution=False):
        """Result dict once finished (the ticket is then retired), else None."""
        return self._result(lib().hc_server_poll, ticket, solution)

    def wait(self, ticket, solution=False):
        return self._result(lib().hc_server_wait, ticket, solution)

    def stats(self) -> dict:
        r = hc_server_report()
        _check(lib().hc_server_stats(self._h, C.byref(r)))
        return {f: getattr(r, f) for f, _ in hc_server_report._fields_}

    def close(self):
        if self._h:
            lib().hc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
