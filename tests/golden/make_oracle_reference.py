"""Write tests/golden/oracle_workloads.json: the FP64 oracle's own solve of the
benchmark workloads (iteration count and final true relative residual).

Calls only the oracle and the seeded input generators.  The benchmark's CPU
baseline uses the iteration count to scale its bounded oracle sample to whole
solves.  Run:  python tests/golden/make_oracle_reference.py [--sizes 32 128]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import nps_inputs as gi  # noqa: E402
from oracle import npsdo  # noqa: E402


def workload(n):
    spec = gi.scene_c1() if n == 32 else gi.scene_serving(n)
    lab = gi.gen_labels(spec, seed=1)
    b = gi.gen_rhs(lab, seed=2)
    return lab, b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="+", default=[32, 128])
    args = ap.parse_args()
    path = os.path.join(HERE, "oracle_workloads.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    for n in args.sizes:
        lab, b = workload(n)
        t0 = time.time()
        res = npsdo.solve_with_network(lab, b, gi.multilevel_params(6), 6, tol=1e-6, max_iter=2000)
        out[f"{n}^3"] = {
            "scene": "scene_c1() seed 1" if n == 32 else f"scene_serving({n}) seed 1",
            "rhs": "gen_rhs seed 2", "weights": "multilevel_params(6)", "tol": 1e-6, "n_ortho": 2,
            "iterations": res.iterations, "status": res.status, "rel_residual": res.rel_residual,
            "n_fluid": int((lab == gi.FLUID).sum()),
        }
        print(n, out[f"{n}^3"], f"{time.time() - t0:.1f}s", flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
