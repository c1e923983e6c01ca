"""Write the oracle's expected values for the full-size workloads (calls only oracle/).

  python tests/golden/make_golden.py c1      -> tests/golden/c1_oracle.json
  python tests/golden/make_golden.py c2      -> tests/golden/c2_oracle.json

c1: 64x64 Q1 channels, 2 levels (full oracle run, solution stored in full).
c2: 512x512 Q1 inclusions, 3 levels (full oracle run; the solution is stored as
    norms and values at fixed sampled dofs).
The oracle is the plain CPU FP64 implementation in oracle/; these files are
regenerated only by this script.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from msdd_inputs import problems as P  # noqa: E402
from oracle.msdd_oracle import Oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def run(name):
    prob = {"c1": P.config1, "c2": P.config2}[name]()
    t0 = time.time()
    o = Oracle(prob, verbose=True)
    t1 = time.time()
    res = o.solve(rtol=1e-8, maxit=2000, record=False)
    t2 = time.time()
    L = prob.n_levels - 1
    out = {
        "workload": prob.name, "n": prob.n, "n_levels": prob.n_levels, "eta": prob.eta,
        "level_sizes": [int(v) for v in o.level_sizes()],
        "levels": {},
        "pcg": {"iters": res.iters, "converged": res.converged,
                "resnorms": [float(v) for v in res.resnorms],
                "kappa": res.kappa(),
                "x_norm": float(np.linalg.norm(res.x)),
                "true_relres": float(np.linalg.norm(prob.b - prob.A @ res.x) / np.linalg.norm(prob.b))},
        "oracle_seconds": {"setup": t1 - t0, "solve": t2 - t1},
    }
    rng = np.random.Generator(np.random.PCG64(12345))
    idx = np.sort(rng.choice(prob.n, size=min(prob.n, 256), replace=False))
    out["pcg"]["x_sample_idx"] = [int(v) for v in idx]
    out["pcg"]["x_sample"] = [float(v) for v in res.x[idx]]
    if name == "c1":
        out["pcg"]["x"] = [float(v) for v in res.x]
    for l in range(L, 0, -1):
        lev = o.levels[l]
        out["levels"][str(l)] = {
            "m": [int(v) for v in lev.m],
            "lam": [[float(v) for v in lev.lam[i][: int(lev.m[i]) + 4]] for i in range(lev.n_sub)],
        }
    with open(os.path.join(HERE, f"{name}_oracle.json"), "w") as f:
        json.dump(out, f)
    print(name, "done", t1 - t0, t2 - t1, res.iters, flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:]:
        run(nm)
