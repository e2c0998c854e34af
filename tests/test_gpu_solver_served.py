"""Served form (hc_server_*) through the C-ABI: every request of a stream of
uneven MPC and LP problems is solved as by a direct hc_solve, memory stays
within the HBM budget, oversize requests are rejected, and closing a server
with work in flight cancels it."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2412_19027_amd import hipcone as HC  # noqa: E402
from paper_2412_19027_amd import workloads as W  # noqa: E402
from tests.test_gpu_solver import MPC_STREAM, certify, gpu_solve, mpc_reference  # noqa: E402


@pytest.mark.parametrize("batched", [True, False], ids=["batched", "per_slot"])
def test_server_matches_direct_solves(batched):
    """Every request as by a direct solve, on the batched engine or on the
    per-slot workers (which bind each problem into the pool with a pinned
    read-back block of their own)."""
    probs = [W.mpc_socp(0, i) for i in range(10)] + [W.tiny_lp(s) for s in range(4)]
    budget = 2 << 30
    srv = HC.Server(hbm_budget_bytes=budget, max_slots=6, workers=3, batched=batched)
    tickets = [srv.submit(p, tag=100 + i) for i, p in enumerate(probs)]
    res = [srv.wait(t, solution=True) for t in tickets]
    st = srv.stats()
    srv.close()
    print({k: st[k] for k in ("completed", "p50_latency_ms", "p99_latency_ms", "solves_per_s", "hbm_peak")})
    assert st["completed"] == len(probs) and st["active"] == 0 and st["pending"] == 0
    assert st["p50_latency_ms"] <= st["p99_latency_ms"] and 0 < st["hbm_peak"] <= budget
    for i, (p, r) in enumerate(zip(probs, res)):
        assert r["tag"] == 100 + i and r["status_name"] == "solved", r
        info, x, _, _ = gpu_solve(p)
        assert abs(r["obj_primal"] - info["obj_primal"]) <= 1e-9 * max(1.0, abs(info["obj_primal"]))
        if not batched:   # the same kernels in the same order: bitwise, alone or in the mix
            assert r["iterations"] == info["iterations"] and np.array_equal(r["x"], x)
        certify(p, r["x"], r["s"], r["z"])
        assert r["latency_ms"] >= r["solve_ms"] >= 0


@pytest.mark.parametrize("batched", [True, False], ids=["batched", "per_slot"])
def test_server_in_caller_pool(batched):
    """hc_server_config.pool: the workspaces are carved from the caller's
    device buffer (no pool allocation by the server); results as by direct
    solves, the buffer untouched past the budget."""
    probs = [W.mpc_socp(2, i) for i in range(6)] + [W.tiny_lp(s) for s in range(2)]
    budget = 512 << 20
    pool = torch.empty(budget + 4096, dtype=torch.uint8, device="cuda")
    pool[budget:].fill_(0x5A)
    torch.cuda.synchronize()
    srv = HC.Server(hbm_budget_bytes=budget, max_slots=4, workers=2, batched=batched, pool=pool)
    res = [srv.wait(t, solution=True) for t in [srv.submit(p) for p in probs]]
    st = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    assert st["completed"] == len(probs) and 0 < st["hbm_peak"] <= budget
    assert bool((pool[budget:] == 0x5A).all())
    for p, r in zip(probs, res):
        info, x, _, _ = gpu_solve(p)
        assert r["status_name"] == "solved", r
        assert abs(r["obj_primal"] - info["obj_primal"]) <= 1e-9 * max(1.0, abs(info["obj_primal"]))


def test_server_budget_bounds_memory():
    probs = [W.mpc_socp(1, i) for i in range(6)]
    need = max(HC.analyze(p)["workspace_bytes"] for p in probs)
    budget = (need + 255) // 256 * 256 + 256
    srv = HC.Server(hbm_budget_bytes=budget, max_slots=4, workers=2)
    tickets = [srv.submit(p) for p in probs]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert all(r["status_name"] == "solved" for r in res)
    assert st["hbm_peak"] <= budget and st["completed"] == len(probs)


def test_server_rejects_oversize_request():
    p = W.tiny_lp(0)
    need = HC.analyze(p)["workspace_bytes"]
    srv = HC.Server(hbm_budget_bytes=max(4096, need // 2), max_slots=2, workers=1)
    with pytest.raises(HC.HipconeError) as e:
        srv.submit(p)
    assert e.value.code == HC.ERR_TOO_LARGE
    assert srv.stats()["rejected"] == 1
    srv.close()


def test_server_close_with_work_in_flight():
    srv = HC.Server(hbm_budget_bytes=1 << 30, max_slots=1, workers=1)
    for i in range(8):
        srv.submit(W.mpc_socp(2, i))
    srv.close()   # queued and active problems end as cancelled; must return promptly


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_server_mpc_stream_against_oracle(precision):
    """The served form on 24 MPC requests of uneven size in flight together:
    every result against the oracle's objective and the optimality
    inequalities on the user's data."""
    refs = [mpc_reference(seed, i) for seed, i in MPC_STREAM]
    srv = HC.Server(hbm_budget_bytes=4 << 30, max_slots=8, workers=2,
                    precision=HC.PRECISION_FP64 if precision == "fp64" else HC.PRECISION_MIXED)
    tickets = [srv.submit(p, tag=i) for i, (p, _) in enumerate(refs)]
    res = [srv.wait(t, solution=True) for t in tickets]
    srv.close()
    for (p, fo), r in zip(refs, res):
        assert r["status_name"] == "solved", (p.name, r)
        gp = certify(p, r["x"], r["s"], r["z"])
        assert abs(gp - fo) <= 1e-7 * max(1.0, abs(fo)), (p.name, gp, fo)
