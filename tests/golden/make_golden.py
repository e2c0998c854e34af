"""Write oracle reference values for full-size parity tests.

Calls only the CPU oracle (oracle/) on the seeded generators; run from the
repository root:  python tests/golden/make_golden.py [names...]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ipm  # noqa: E402
from paper_2412_19027_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_objectives.json")

CASES = {
    "tiny_lp_s0": lambda: W.tiny_lp(0),
    "tiny_lp_s1": lambda: W.tiny_lp(1),
    "tiny_lp_s2": lambda: W.tiny_lp(2),
    "tiny_lp_s3": lambda: W.tiny_lp(3),
    "tiny_lp_s4": lambda: W.tiny_lp(4),
    "sparse_socp_full_s0": lambda: W.sparse_socp(0),
    "psd_pow_full_s0": lambda: W.psd_pow(0),
    "logreg_exp_2k_s0": lambda: W.logreg_exp(0, samples=2000, features=50),
    "logreg_exp_20k_s0": lambda: W.logreg_exp(0, samples=20000, features=100),
    "logreg_exp_full_s0": lambda: W.logreg_exp(0),
}
for _s in (1, 2, 3, 4):
    CASES[f"sparse_socp_full_s{_s}"] = (lambda s: lambda: W.sparse_socp(s))(_s)
    CASES[f"psd_pow_full_s{_s}"] = (lambda s: lambda: W.psd_pow(s))(_s)
    CASES[f"logreg_exp_full_s{_s}"] = (lambda s: lambda: W.logreg_exp(s))(_s)


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names or CASES:
        t = time.time()
        prob = CASES[name]()
        s = ipm.solve(prob)
        data[name] = {"problem": prob.name, "status": ipm.STATUS_NAMES[s.status], "objective": s.objective,
                      "iterations": s.iterations, "res_primal": s.result["nrp"], "res_dual": s.result["nrd"],
                      "oracle_seconds": time.time() - t}
        print(name, data[name], flush=True)
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
