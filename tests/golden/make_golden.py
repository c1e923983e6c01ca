"""Write the oracle's expected values for the full-size workloads (calls only oracle/).

  python tests/golden/make_golden.py c1    -> tests/golden/c1_oracle.json (+ .npz)
  python tests/golden/make_golden.py c2    -> tests/golden/c2_oracle.json (+ .npz)
  python tests/golden/make_golden.py c4s   -> tests/golden/c4s_oracle.json (+ .npz)

c1:  64x64 Q1 channels, 2 levels.
c2:  512x512 Q1 inclusions, 3 levels.
c4s: the three smallest problems of the 32-problem log-normal batch (each on its own;
     the batch shares nothing between problems), 3 levels.

For every workload: a full oracle run (setup and PCG), and for every finest-level
subdomain the eigenvalues of the m selected pairs and the next ones refined in
binary128 from the oracle's own eigenvectors (oracle.refine_pairs), each with its
residual bound and its FP64 uncertainty u * cond (the change that entrywise relative
perturbations of the FP64 element data at unit roundoff cause, to first order).  The
.npz holds the full PCG solution, the iterates at a few fixed iteration counts and the
finest-level coarse basis blocks of sampled subdomains (plus every coarse level's
blocks).  The oracle is the plain CPU FP64 implementation in oracle/; these files are
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
from oracle.msdd_oracle import Oracle, refine_pairs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
EXTRA_VEC = 8        # start vectors beyond m for the refinement
REFINE_ITERS = 8
N_EXTRA = 2          # eigenvalues stored beyond the m selected ones (the first certifies m)
ITERATES = (5, 20, 60)


def oracle_run(prob, workers, sample_subs=16, iterates=ITERATES):
    t0 = time.time()
    o = Oracle(prob, verbose=True, fine_vectors=EXTRA_VEC, workers=workers)
    t1 = time.time()
    res = o.solve(rtol=1e-8, maxit=2000, record=True)
    t2 = time.time()
    L = prob.n_levels - 1
    fine = o.levels[L]
    ref = {"lam": [], "lam_lo": [], "bound": [], "unc": []}
    for i in range(prob.n_sub):
        k = int(fine.m[i]) + N_EXTRA
        r = refine_pairs(prob.elem_dofs, prob.elem_mat, prob.sub_elems(i), prob.sub_dofs(i),
                         prob.sub_weights(i), o.fine_vecs[i], iters=REFINE_ITERS)
        ref["lam"].append([float(v) for v in r.lam[:k]])
        ref["lam_lo"].append([float(v) for v in r.lam_lo[:k]])
        ref["bound"].append([float(v) for v in r.bound[:k]])
        ref["unc"].append([float(v) for v in r.fp64_uncertainty[:k]])
        if i % 32 == 0:
            print(f"  refined sub {i}", flush=True)
    t3 = time.time()
    out = {
        "workload": prob.name, "n": prob.n, "n_levels": prob.n_levels, "eta": prob.eta,
        "level_sizes": [int(v) for v in o.level_sizes()],
        "levels": {},
        "pcg": {"iters": res.iters, "converged": res.converged,
                "resnorms": [float(v) for v in res.resnorms],
                "kappa": res.kappa(),
                "x_norm": float(np.linalg.norm(res.x)),
                "true_relres": float(np.linalg.norm(prob.b - prob.A @ res.x) / np.linalg.norm(prob.b))},
        "oracle_seconds": {"setup": t1 - t0, "solve": t2 - t1, "refine": t3 - t2,
                           "workers": workers, "host_cpus": os.cpu_count()},
    }
    rng = np.random.Generator(np.random.PCG64(12345))
    idx = np.sort(rng.choice(prob.n, size=min(prob.n, 256), replace=False))
    out["pcg"]["x_sample_idx"] = [int(v) for v in idx]
    out["pcg"]["x_sample"] = [float(v) for v in res.x[idx]]
    for l in range(L, 0, -1):
        lev = o.levels[l]
        out["levels"][str(l)] = {
            "m": [int(v) for v in lev.m],
            "lam": [[float(v) for v in lev.lam[i][: int(lev.m[i]) + 4]] for i in range(lev.n_sub)],
        }
    out["levels"][str(L)]["lam_ref"] = ref
    subs = np.sort(np.random.Generator(np.random.PCG64(777)).choice(
        prob.n_sub, size=min(prob.n_sub, sample_subs), replace=False))
    out["basis_subdomains"] = [int(v) for v in subs]
    arrays = {"x": res.x}
    for k in iterates:
        if k < len(res.iterates):
            arrays[f"x_it{k}"] = res.iterates[k]
    for i in subs:
        arrays[f"basis_{L}_{int(i)}"] = fine.basis[int(i)]
    for l in range(L - 1, 0, -1):
        lev = o.levels[l]
        for i in range(lev.n_sub):
            arrays[f"basis_{l}_{i}"] = lev.basis[i]
    out["iterates"] = [k for k in iterates if k < len(res.iterates)]
    print(prob.name, "setup", t1 - t0, "solve", t2 - t1, "refine", t3 - t2, "iters", res.iters,
          flush=True)
    return out, arrays


def c4_smallest(count=3):
    """Positions (in the batch order) and parameters of the smallest batch problems."""
    members = P.config4_members()
    order = sorted(range(len(members)), key=lambda t: members[t][0])[:count]
    return [(t, members[t]) for t in sorted(order)]


def run(name, workers):
    if name in ("c1", "c2"):
        prob = {"c1": P.config1, "c2": P.config2}[name]()
        out, arrays = oracle_run(prob, workers)
        with open(os.path.join(HERE, f"{name}_oracle.json"), "w") as f:
            json.dump(out, f)
        np.savez_compressed(os.path.join(HERE, f"{name}_oracle.npz"), **arrays)
    elif name == "c4s":
        outs, arrays = [], {}
        for t, mem in c4_smallest():
            prob = P.config4_problem(*mem)
            o, a = oracle_run(prob, workers, sample_subs=4, iterates=(5, 20))
            o["batch_position"] = t
            o["member"] = list(mem)
            outs.append(o)
            for k, v in a.items():
                arrays[f"m{t}_{k}"] = v
        with open(os.path.join(HERE, "c4s_oracle.json"), "w") as f:
            json.dump({"members": outs}, f)
        np.savez_compressed(os.path.join(HERE, "c4s_oracle.npz"), **arrays)
    else:
        raise SystemExit(f"unknown workload {name}")


if __name__ == "__main__":
    workers = int(os.environ.get("GOLDEN_WORKERS", "1"))
    for nm in sys.argv[1:]:
        run(nm, workers)
