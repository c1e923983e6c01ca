"""Benchmark: setup + solve of the multilevel spectral domain decomposition on one MI355X.

One step = msdd_setup (local matrices, batched local GEVPs, coarse levels) +
msdd_solve (PCG to relative residual 1e-8) on the 2D Q1 512x512 inclusions
workload (3 levels, 256 -> 16 -> 1 subdomains, FP64), inputs resident in HBM.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "setup+solve sec to rel-res 1e-8 (plain FP64 vs mixed/learned); local GEVPs/s"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VALU_PEAK_TFS = 78.6      # MI355X FP64 vector (256 CUs, 2.4 GHz)

# Kernel classes bound by arithmetic rather than HBM traffic (the rest are priced
# against HBM with their algorithmic bytes).
ALU_CLASSES = {"coarse_gevp"}

WORKLOADS = {
    "c2": ("2D scalar diffusion, Q1 512x512, seeded binary inclusions (10%, squares 2-8, k=1e6), "
           "16x16 subdomains overlap 2, 3 levels (256->16->1), eta=0.1, FP64, PCG to 1e-8"),
    "c1": ("2D scalar diffusion, Q1 64x64, 4 channels k=1e6, 4x4 subdomains overlap 2, 2 levels, "
           "eta=0.1, FP64, PCG to 1e-8"),
    "c3": ("3D linear elasticity, trilinear Q1 48^3 (3 dofs/node), 16 plies 3 elements thick "
           "(fibre E=1e3 0/90 deg, resin E=1, nu=0.3), clamped x=0, body force -z, 6x6x6 "
           "subdomains overlap 1, 3 levels (216->27->1), eta=0.1, PCG to 1e-8"),
    "c5": ("3D scalar diffusion, Q1 96^3, seeded bars (k=1e6) over a log-normal field "
           "(sigma^2=4), 8x8x8 subdomains overlap 1, 3 levels (512->64->1), eta=0.1, PCG to 1e-8"),
}


C4_DESC = ("batch of 32 independent 2D log-normal diffusion problems (Gaussian field, exponential "
           "covariance, correlation length 0.05, sigma^2=4), Q1 N x N with N uniform in 128..1024 "
           "(seed 4), P_side = clamp(round(N/32), 4, 32) subdomains per side, overlap 2, 3 levels, "
           "eta=0.1; one setup for all problems, one PCG per problem to 1e-8; FP32 preconditioner "
           "(scaled FP32 Dirichlet factors), FP64 PCG")


def _c4_member(args):
    from msdd_inputs import problems as P
    return P.config4_problem(*args)


def bench_batch(args):
    """The batched workload: all 32 problems in one msdd_setup_batch, one CG per problem."""
    import multiprocessing as mp
    import torch
    from msdd_inputs import problems as P
    from paper_2106_06404_amd import binding as B
    members = P.config4_members()
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        probs = pool.map(_c4_member, members)
    arrs = B.batch_arrays(probs, device="cuda:0")
    b = torch.from_numpy(np.concatenate([p.b for p in probs])).cuda()
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    ctx = B.Msdd(verbose=1 if args.verbose else 0, precision=B.MSDD_MIXED)

    def step():
        ctx.setup_batch(**arrs)
        x.zero_()
        return ctx.solve_batch(b, x, 1e-8, 5000)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    setup_ms, solve_ms = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        its, rels, _ = step()
        st = ctx.stats()
        setup_ms.append(st["t_setup_ms"])
        solve_ms.append(st["t_solve_ms"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # one profiled step (outside the timed region) for the kernel classes
    ctx.profile(True)
    step()
    ctx.profile(False)
    prof = ctx.profile_query()
    ctx.close()
    rl_all = {k: roofline_entry(k, v, counters=False) for k, v in prof.items() if v[1] > 0}
    dom = max(rl_all, key=lambda k: prof[k][0])
    xh = x.cpu().numpy()
    true_rel, base = [], 0
    for p in probs:
        xi = xh[base:base + p.n]
        true_rel.append(float(np.linalg.norm(p.b - p.A @ xi) / np.linalg.norm(p.b)))
        base += p.n
    ms = (t1 - t0) * 1e3 / args.steps
    out = {
        "metric": METRIC, "value": ms * 1e-3, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32/f64", "data": "synthetic",
        "config": {"workload": C4_DESC, "problems": len(probs), "n_total": int(arrs["n"]),
                   "subdomains": st["n_sub"], "levels": 3, "precision": "mixed"},
        "setup_s": float(np.median(setup_ms)) * 1e-3, "solve_s": float(np.median(solve_ms)) * 1e-3,
        "pcg_iters_min_max": [int(its.min()), int(its.max())],
        "true_relres_max": max(true_rel),
        "local_gevps_per_s": sum(st["n_sub"][1:]) / ((st["t_gevp_ms"] + st["t_coarse_ms"]) * 1e-3),
        "roofline": dict(rl_all[dom], kernel=dom),
        "roofline_by_kernel": {k: {"ms_per_step": prof[k][0], "launches_per_step": prof[k][1],
                                   "bound": r["bound"], "achieved": r["achieved"],
                                   "unit": r["unit"], "frac": r["frac"]}
                               for k, r in sorted(rl_all.items(), key=lambda kv: -prof[kv[0]][0])},
    }
    print(json.dumps(out))


LEARN_SEEDS = tuple(range(100, 108))  # training problems (the benched problem uses seed 2)
LEARN_EPOCHS = 40


def _learn_member(seed):
    from msdd_inputs import problems as P
    p = P.config2(seed=seed)
    f, sp, n_pos = P.warm_frame(p, 2)
    return p, f, sp, n_pos


def learn_inputs():
    """Seeded training problems (host only; generated before the GPU is touched)."""
    import multiprocessing as mp
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        members = pool.map(_learn_member, LEARN_SEEDS)
    return members, time.perf_counter() - t0


def train_warm_start(members, t_gen, verbose=False):
    """The learned warm start for the 512x512 inclusions workload: the network is trained
    on the converged local eigenvectors of 8 further seeded problems of the same family
    (2048 subdomain GEVP solves, collected by the library's own setups) with the
    library's FP32 training kernels.  Returns the network and a summary (offline cost,
    not part of a timed step)."""
    import torch
    from paper_2106_06404_amd import binding as B, warm as W
    t0 = time.perf_counter()
    parts = [W.collect_targets(p, f, sp, n_pos, m_cap=16)[:4] for p, f, sp, n_pos in members]
    feat, tgt, mask, cnt = (torch.cat([q[k] for q in parts]) for k in range(4))
    torch.cuda.synchronize()
    t_collect = time.perf_counter() - t0
    n_pos = members[0][3]
    net = B.MsddNet(feat.shape[1], 256, 16, n_pos, seed=7)
    t0 = time.perf_counter()
    losses = W.train(net, feat, tgt, mask, cnt, epochs=LEARN_EPOCHS, batch=64, lr=1e-3,
                     lr_final=1e-4, seed=3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    info = {"problems": len(LEARN_SEEDS), "samples": int(feat.shape[0]), "epochs": LEARN_EPOCHS,
            "batch": 64, "hidden": 256, "n_vec": 16, "n_in": int(feat.shape[1]), "n_pos": n_pos,
            "params": net.n_params, "loss_epoch1": losses[0], "loss_final": losses[-1],
            "inputs_s": t_gen, "collect_s": t_collect, "train_s": t_train}
    if verbose:
        print(f"warm start: {info}", file=sys.stderr)
    return net, info


# Table 3 of the paper (Q1, overlap 3h, eta = 0.3, CG): coarsest-space size n_0 and CG
# iterations per subdomain count and level count, quoted beside the measured ones.
TABLE3 = {64: {"dofs": 410881, 2: (306, 25)},
          256: {"dofs": 1640961, 2: (1348, 26), 3: (130, 32)},
          1024: {"dofs": 6558721, 2: (5523, 27), 3: (431, 31), 4: (207, 40)}}


def bench_islands(args):
    """Weak scaling on the islands shape of Table 3: P x P subdomains of 80 x 80 Q1 elements,
    overlap 3, eta 0.3, Dirichlet on x = 0 and x = 1; one setup + PCG (to 1e-8) per case, and
    GMRES with the hybrid form on the same setup.  Cases 'P:L[:factor]' (coarse levels group
    factor x factor subdomains)."""
    import torch
    from msdd_inputs import problems as P
    from paper_2106_06404_amd import binding as B
    cases = [tuple(int(v) for v in c.split(":")) for c in args.islands.split(",")]
    u = 2.0 ** -53
    rows = []
    for cs in cases:
        Ps, L = cs[0], cs[1]
        fac = cs[2] if len(cs) > 2 else 4
        prob = P.table3_islands(Ps, L, factor=fac)
        print(f"islands P={Ps}x{Ps} L={L} factor={fac}: n={prob.n}", file=sys.stderr, flush=True)
        arrs = B.problem_arrays(prob, device="cuda:0")
        b = torch.from_numpy(prob.b).cuda()
        torch.cuda.synchronize()
        m = B.Msdd(verbose=1 if args.verbose else 0)
        rec = {}
        for rep in range(max(1, args.steps)):
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m.setup(**arrs)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            it, rel, _ = m.solve(b, x, 1e-8, 2000)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            rec.setdefault("setup", []).append(t1 - t0)
            rec.setdefault("solve", []).append(t2 - t1)
        st = m.stats()
        xg = torch.zeros_like(b)
        t3 = time.perf_counter()
        itg, relg, _ = m.solve_gmres(b, xg, 1e-8, 300, 600, allow_noconv=True)
        torch.cuda.synchronize()
        tg = time.perf_counter() - t3
        xc = x.cpu().numpy()
        bn = float(np.linalg.norm(prob.b))
        paper = TABLE3.get(Ps * Ps, {})
        rows.append({
            "subdomains": Ps * Ps, "levels": L, "group_factor": fac, "dofs": prob.n,
            "setup_s": float(np.median(rec["setup"])), "solve_s": float(np.median(rec["solve"])),
            "cg_iters": it, "n0": st["n"][0], "level_sizes": st["n"],
            "cg_true_relres": float(np.linalg.norm(prob.b - prob.A @ xc) / bn),
            "fp64_residual_floor": float(u * np.linalg.norm(abs(prob.A) @ np.abs(xc)
                                                             + np.abs(prob.b)) / bn),
            "hybrid_gmres_iters": itg, "hybrid_gmres_s": tg,
            "eig_iters_max": st["eig_iters_max"], "t_gevp_ms": st["t_gevp_ms"],
            "t_coarse_ms": st["t_coarse_ms"], "t_local_ms": st["t_local_ms"],
            "t_plan_ms": st["t_plan_ms"],
            "paper": ({"dofs": paper["dofs"], "n0": paper[L][0], "cg_iters": paper[L][1]}
                      if L in paper else None)})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        m.close()
        del arrs, b, x, xg
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "islands weak scaling (Table 3 shape)", "steps": args.steps,
                      "data": "synthetic (seeded inclusion field standing in for the paper's "
                              "island field)", "cases": rows}))


# Table 1 of the paper (Laplace, Q1, 16 subdomains, eta = 0.15, CG): #IT and n_0 per mesh
# size for overlap ~ h and overlap ~ H
TABLE1 = {320: {"h": (30, 56), "H": (30, 56)}, 640: {"h": (29, 114), "H": (32, 50)},
          1280: {"h": (27, 236), "H": (25, 54)}, 2560: {"h": (26, 488), "H": (26, 54)}}


def bench_table1(args):
    """The Laplace column of Table 1: cases 'N:delta:kind' (kind h = overlap of a fixed number
    of element layers, H = overlap a fixed fraction of the subdomain); one setup + CG each."""
    import torch
    from msdd_inputs import problems as P
    from paper_2106_06404_amd import binding as B
    rows = []
    for c in args.table1.split(","):
        N, delta, kind = c.split(":")
        N, delta = int(N), int(delta)
        prob = P.table1_laplace(N, delta)
        print(f"table1 N={N} delta={delta} ({kind}): n={prob.n}", file=sys.stderr, flush=True)
        arrs = B.problem_arrays(prob, device="cuda:0")
        b = torch.from_numpy(prob.b).cuda()
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        m = B.Msdd()
        t0 = time.perf_counter()
        m.setup(**arrs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        it, rel, _ = m.solve(b, x, 1e-8, 2000)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        st = m.stats()
        ref = TABLE1.get(N, {}).get(kind)
        rows.append({"h_inv": N, "delta": delta, "overlap": kind, "dofs": prob.n,
                     "cg_iters": it, "n0": st["n"][0], "setup_s": t1 - t0, "solve_s": t2 - t1,
                     "eig_iters_max": st["eig_iters_max"], "max_band": st["max_band"],
                     "paper": {"cg_iters": ref[0], "n0": ref[1]} if ref else None})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        m.close()
        del arrs, b, x
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "Laplace two-level (Table 1 shape)", "data": "synthetic",
                      "cases": rows}))


def bench_skeleton(args):
    """Conforming Q1 (CG), cell-centred finite volumes (FV) and WSIP-DG-Q1 (DG) on one
    log-normal field at about 1M dofs each (the discretisation comparison of the paper's
    SPE10 runs, with a synthetic field): 16 x 16 subdomains, overlap 2, eta = 0.3, 2 or 3
    levels (256 -> 16 -> 1); setup + CG, and GMRES with the hybrid form on the same setup.
    Cases 'kind:levels', comma separated."""
    import torch
    from msdd_inputs import problems as P
    from paper_2106_06404_amd import binding as B
    N = 1024
    field = np.exp(P.gaussian_field(2, N, 11, sigma2=args.skeleton_sigma2))
    coarse = np.exp(np.log(field).reshape(N // 2, 2, N // 2, 2).mean(axis=(1, 3))).reshape(-1)
    rows = []
    for c in args.skeleton.split(","):
        kind, L = c.split(":")
        L = int(L)
        groups = (4,) if L == 3 else ()
        t0 = time.perf_counter()
        if kind == "cg":
            prob = P.build_problem("cg", 2, N, field, P=16, delta=2, n_levels=L, eta=0.3,
                                   groups=groups)
        elif kind == "fv":
            prob = P.fv_problem(N, field, 16, 2, n_levels=L, groups=groups, eta=0.3)
        else:
            prob = P.dg_problem(N // 2, coarse, 16, 2, n_levels=L, groups=groups, eta=0.3)
        tgen = time.perf_counter() - t0
        print(f"skeleton {kind} L={L}: n={prob.n} (generated in {tgen:.0f} s)", file=sys.stderr,
              flush=True)
        opts = {"dirichlet_rule": 1} if prob.dirichlet_rule == "all" else {}
        arrs = B.problem_arrays(prob, device="cuda:0")
        b = torch.from_numpy(prob.b).cuda()
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        m = B.Msdd(**opts)
        t0 = time.perf_counter()
        m.setup(**arrs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        it, rel, _ = m.solve(b, x, 1e-8, 2000)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        xg = torch.zeros_like(b)
        itg, relg, _ = m.solve_gmres(b, xg, 1e-8, 300, 600, allow_noconv=True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        st = m.stats()
        rows.append({"discretisation": kind, "levels": L, "dofs": prob.n, "n0": st["n"][0],
                     "level_sizes": st["n"], "cg_iters": it, "hybrid_gmres_iters": itg,
                     "setup_s": t1 - t0, "cg_solve_s": t2 - t1, "gmres_solve_s": t3 - t2,
                     "max_band": st["max_band"], "eig_iters_max": st["eig_iters_max"]})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        m.close()
        del arrs, b, x, xg
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "CG / FV / DG on one log-normal field (SPE10-style comparison)",
                      "data": "synthetic", "sigma2": args.skeleton_sigma2, "cases": rows}))


def make_problem(name):
    from msdd_inputs import problems as P
    return {"c1": P.config1, "c2": P.config2, "c3": P.config3, "c5": P.config5}[name]()


def host_cores():
    """(cores the oracle may use, logical CPUs the process may run on, CPUs the host has).
    A one-GPU share of the GPU hosts is 16 cores, whatever the machine has in all."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return min(16, avail), avail, os.cpu_count() or 1


def full_oracle_run(name):
    """The full oracle run (setup and PCG) of the workload as measured when its stored
    expected values were written (tests/golden/<name>_oracle.json), or None."""
    path = os.path.join(ROOT, "tests", "golden", f"{name}_oracle.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    t = g.get("oracle_seconds")
    if not t:
        return None
    return {"setup_s": t["setup"], "solve_s": t["solve"], "total_s": t["setup"] + t["solve"],
            "pcg_iters": g["pcg"]["iters"], "workers": t.get("workers"),
            "host_cpus": t.get("host_cpus"),
            "where": "the build host (8 CPUs), not the GPU host: measured once, when the "
                     "stored expected values were written"}


def cpu_baseline(prob, name, budget_s=20.0):
    """The oracle (plain CPU FP64) on a bounded sample of the same workload: the finest-level
    per-subdomain work (Neumann matrix, GEVP, Dirichlet Cholesky) for interior subdomains,
    until the time budget is spent; extrapolated linearly to all subdomains.  The full
    oracle run of the workload, where one was recorded, is attached beside it."""
    cores, avail, ncpu = host_cores()
    os.environ["ORACLE_THREADS"] = str(cores)
    from oracle import msdd_oracle as O
    P = prob.n_sub
    side = int(round(P ** 0.5))
    order = [side * (side // 2) + side // 2, side * (side // 2 - 1) + side // 2 - 1, 0, P - 1]
    t0 = time.time()
    done = 0
    for i in order:
        dofs = prob.sub_dofs(i)
        d = prob.sub_weights(i)
        el = prob.sub_elems(i)
        dm = O.dirichlet_mask(prob.elem_dofs, el, dofs)
        Ab = O.neumann_matrix(prob.elem_dofs, prob.elem_mat, el, dofs)
        O.gevp_definite(Ab, d[:, None] * Ab * d[None, :], prob.eta)
        O.cholesky(prob.A[dofs[dm]][:, dofs[dm]].toarray())
        done += 1
        if time.time() - t0 > budget_s:
            break
    dt = time.time() - t0
    per = dt / done
    return {"value": per * P, "unit": "s", "cores": cores, "kind": "oracle",
            "sample": (f"{done} of {P} finest-level subdomains (Neumann matrix + GEVP by Cholesky "
                       f"and Jacobi + Dirichlet Cholesky), {per:.2f} s each, extrapolated x{P}; "
                       f"coarse levels and PCG not timed"),
            "local_gevps_per_s": 1.0 / per, "cpus_available": avail, "cpus_host": ncpu,
            "full_oracle_run": full_oracle_run(name)}


def roofline_entry(name, rec, counters=True):
    """Achieved = algorithmic work per launch / average launch duration (HIP events on
    the launching stream), against the MI355X peak of the resource that bounds it.
    counters: attach the rocprofv3 traffic per launch, which was measured on the 512x512
    inclusions workload only (False for any other workload)."""
    tot_ms, launches, byts, flops = rec
    avg_ms = tot_ms / launches
    if name in ALU_CLASSES:
        ach = (flops / launches) / (avg_ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": ach, "peak": FP64_VALU_PEAK_TFS, "unit": "TFLOP/s",
                "frac": ach / FP64_VALU_PEAK_TFS,
                "traffic": traffic_for(name) if counters else None,
                "alg_flops_per_launch": flops / launches, "avg_launch_ms": avg_ms,
                "launches": launches}
    ach = (byts / launches) / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic_for(name) if counters else None,
            "alg_bytes_per_launch": byts / launches, "avg_launch_ms": avg_ms, "launches": launches}


def traffic_for(name):
    """HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE + WRITE_SIZE,
    scaled by the copy-kernel calibration), from profiles/traffic.md; None when no
    measurement exists or the kernel's source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.md")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 4 and cells[0] == name:
                h = hashlib.sha256()
                for fn in cells[2].split("+"):
                    src = os.path.join(ROOT, "paper_2106_06404_amd", "csrc", fn.strip())
                    if not os.path.exists(src):
                        return None
                    with open(src, "rb") as g:
                        h.update(g.read())
                if h.hexdigest()[:16] != cells[3]:
                    return None
                return float(cells[1])
    return None


def copy_calibration(nbytes=1 << 30):
    """A plain device copy of known size: run under rocprofv3 --pmc FETCH_SIZE (then
    WRITE_SIZE) to calibrate the counters (it reads and writes nbytes once)."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2",
                    choices=sorted(WORKLOADS) + ["c4", "islands", "table1", "skeleton"])
    ap.add_argument("--skeleton", default="cg:2,fv:2,dg:2,cg:3,fv:3,dg:3",
                    help="discretisation:levels cases (--workload skeleton)")
    ap.add_argument("--skeleton-sigma2", type=float, default=4.0)
    ap.add_argument("--table1", default="320:2:h,640:2:h,320:5:H,640:10:H",
                    help="Table 1 cases N:delta:kind (kind h or H), comma separated")
    ap.add_argument("--islands", default="8:2,16:2,16:3,32:3,32:4:2",
                    help="islands cases P:L[:factor], comma separated (--workload islands)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the launch shapes chosen by problem shape (no msdd_autotune)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned warm-start leg (training + warm-started steps)")
    ap.add_argument("--no-eig32", action="store_true",
                    help="skip the setups with the FP32-factor eigensolver (c2)")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the sharding of the "
              f"subdomains over several GPUs is not built.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c4":
        bench_batch(args)
        return
    if args.workload == "islands":
        bench_islands(args)
        return
    if args.workload == "table1":
        bench_table1(args)
        return
    if args.workload == "skeleton":
        bench_skeleton(args)
        return
    import torch
    from paper_2106_06404_amd import binding as B

    prob = make_problem(args.workload)
    learned = args.workload == "c2" and not args.no_learned
    members = learn_inputs() if learned else None
    dev = "cuda:0"
    arrs = B.problem_arrays(prob, device=dev)
    b = torch.from_numpy(prob.b).to(dev)
    torch.cuda.synchronize()

    def measure(precision, warm=None):
        """warm-up steps, then exactly args.steps timed steps (setup + solve), inputs
        resident in HBM; synchronised on both sides of the timed region.  warm: (network,
        features, frame positions, n_pos) attached to every setup (network inference is
        part of the timed setup)."""
        x = torch.zeros_like(b)
        ctx = B.Msdd(verbose=1 if args.verbose else 0, precision=precision)
        if warm is not None:
            net, feat_t, sub_pos, n_pos = warm
            ctx.warm_start(net, prob.n_sub, sub_pos, n_pos, feat=feat_t)

        def step(profile_solve):
            # kernel-class counters run during the setup; the solve runs with them paused
            # (its iterations are then replayed as HIP graphs) unless profile_solve
            ctx.profile(True, reset=False)
            ctx.setup(**arrs)
            if not profile_solve:
                ctx.profile(False)
            x.zero_()
            it, rel, _ = ctx.solve(b, x, 1e-8, 5000)
            ctx.profile(False)
            return it, rel

        for _ in range(args.warmup):
            step(False)
        tuning = None
        if not args.no_autotune:
            # launch shapes timed on this context's data (one-off, outside the timed steps),
            # then one more untimed step so that the timed ones run the tuned shapes
            if args.warmup == 0:
                step(False)  # the tuner works on a completed setup
            tuning = ctx.autotune(reps=5)
            step(False)
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile(False)
        setup_ms, solve_ms, iters = [], [], []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            it, rel = step(False)
            st = ctx.stats()
            setup_ms.append(st["t_setup_ms"])
            solve_ms.append(st["t_solve_ms"])
            iters.append(it)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof_setup = ctx.profile_query()
        # one more step, solve phase profiled kernel by kernel (outside the timed region)
        ctx.profile(True)
        ctx.profile(False)
        x.zero_()
        ctx.profile(True, reset=False)
        ctx.solve(b, x, 1e-8, 5000)
        ctx.profile(False)
        prof_solve = ctx.profile_query()
        # per step: setup classes averaged over the timed steps, solve classes from one solve
        prof = {}
        for k in prof_setup:
            a, bq = prof_setup[k], prof_solve[k]
            prof[k] = tuple(v / args.steps for v in a) if a[1] else tuple(bq)
        st = ctx.stats()
        ctx.close()
        # true residual of the last solution (host check, outside the timed region)
        xh = x.cpu().numpy()
        true_rel = float(np.linalg.norm(prob.b - prob.A @ xh) / np.linalg.norm(prob.b))
        return dict(ms_per_step=(t1 - t0) * 1e3 / args.steps, prof=prof, st=st, iters=iters,
                    setup_ms=setup_ms, solve_ms=solve_ms, true_rel=true_rel, tuning=tuning)

    r64 = measure(B.MSDD_FP64)
    r32 = measure(B.MSDD_MIXED)
    prof, st, iters = r64["prof"], r64["st"], r64["iters"]
    setup_ms, solve_ms, true_rel = r64["setup_ms"], r64["solve_ms"], r64["true_rel"]
    ms_per_step = r64["ms_per_step"]
    n_gevp = sum(st["n_sub"][1:])
    gevp_s = (st["t_gevp_ms"] + st["t_coarse_ms"]) * 1e-3
    # roofline of every kernel class, and of the dominant one (largest time per step)
    rl_all = {k: roofline_entry(k, v, counters=args.workload == "c2")
              for k, v in prof.items() if v[1] > 0}
    dom = max(rl_all, key=lambda k: prof[k][0])
    out = {
        "metric": METRIC,
        "value": ms_per_step * 1e-3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "n": prob.n, "subdomains": st["n_sub"],
                   "levels": prob.n_levels, "precision": "fp64"},
        "setup_s": float(np.median(setup_ms)) * 1e-3,
        "solve_s": float(np.median(solve_ms)) * 1e-3,
        "pcg_iters": iters[-1],
        "true_relres": true_rel,
        "local_gevps_per_s": n_gevp / gevp_s,
        "coarse_sizes": st["n"],
        "roofline": dict(rl_all[dom], kernel=dom),
        "tuning": r64["tuning"],
        "roofline_by_kernel": {k: {"ms_per_step": prof[k][0],
                                   "launches_per_step": prof[k][1],
                                   "bound": r["bound"], "achieved": r["achieved"],
                                   "unit": r["unit"], "frac": r["frac"]}
                               for k, r in sorted(rl_all.items(), key=lambda kv: -prof[kv[0]][0])},
    }
    p32 = r32["prof"]
    out["mixed"] = {
        "what": ("finest-level Dirichlet factorisations and the fine-level solves of the "
                 "preconditioner apply in FP32 (diagonally scaled); eigensolves, coarse levels "
                 "and PCG in FP64; same stopping rule"),
        "s_per_step": r32["ms_per_step"] * 1e-3,
        "setup_s": float(np.median(r32["setup_ms"])) * 1e-3,
        "solve_s": float(np.median(r32["solve_ms"])) * 1e-3,
        "pcg_iters": r32["iters"][-1],
        "true_relres": r32["true_rel"],
        "speedup_vs_fp64": ms_per_step / r32["ms_per_step"],
        "solve_speedup_vs_fp64": (float(np.median(solve_ms)) / float(np.median(r32["solve_ms"]))),
        "apply_fine_solve": (dict(roofline_entry("apply_fine_solve", p32["apply_fine_solve"]),
                                  traffic=None)
                             if p32.get("apply_fine_solve", (0, 0))[1] else None),
    }
    if args.workload == "c2" and not args.no_eig32:
        # finest-level eigensolver with the single-precision factor of the shifted pencil
        # (opt-in eig_fp32) against the FP64 factor: setups only, same launch shapes (no
        # tuning on either side), one untimed setup then three timed
        def setups(**opts):
            ctx = B.Msdd(**opts)
            ctx.setup(**arrs)
            ts, gv = [], []
            for _ in range(3):
                ctx.setup(**arrs)
                s_ = ctx.stats()
                ts.append(s_["t_setup_ms"])
                gv.append(s_["t_gevp_ms"])
            ctx.close()
            return float(np.median(ts)), float(np.median(gv)), s_
        t64, g64, _ = setups()
        te, ge, se = setups(eig_fp32=1)
        out["eig_fp32"] = {
            "what": ("finest-level eigensolver preconditioned by the FP32 factor of the scaled "
                     "shifted pencil, FP64 residuals and Rayleigh-Ritz (same pairs and counts); "
                     "subdomains not certified within 64 iterations re-solved with the FP64 "
                     "factor; setup only, untuned launch shapes on both sides"),
            "setup_s": te * 1e-3, "gevp_ms": ge,
            "fp64_setup_s": t64 * 1e-3, "fp64_gevp_ms": g64,
            "setup_speedup_vs_fp64": t64 / te,
            "eig_iters_sum": se["eig_iters_sum"], "fp64_fallbacks": se["eig_fp64_fallbacks"],
        }
    if learned:
        from msdd_inputs import problems as P
        net, info = train_warm_start(*members, verbose=args.verbose)
        f, sp, n_pos = P.warm_frame(prob, 2)
        warm = (net, torch.from_numpy(f).to(dev), sp, n_pos)
        # loss of the trained network on this (unseen) problem's own eigenvectors
        from paper_2106_06404_amd import warm as W
        ft, tg, mk, ct, _ = W.collect_targets(prob, f, sp, n_pos, m_cap=16)
        info["loss_benched_problem"] = W.mean_loss(net, ft, tg, mk, ct)
        rw64 = measure(B.MSDD_FP64, warm)
        rw32 = measure(B.MSDD_MIXED, warm)

        def leg(r):
            return {"s_per_step": r["ms_per_step"] * 1e-3,
                    "setup_s": float(np.median(r["setup_ms"])) * 1e-3,
                    "solve_s": float(np.median(r["solve_ms"])) * 1e-3,
                    "pcg_iters": r["iters"][-1], "true_relres": r["true_rel"],
                    "eig_iters_sum": r["st"]["eig_iters_sum"],
                    "eig_iters_max": r["st"]["eig_iters_max"],
                    "warm_fallbacks": r["st"]["warm_fallbacks"],
                    "t_gevp_ms": r["st"]["t_gevp_ms"],
                    "warm_infer_ms": r["prof"].get("warm_infer", (0.0,))[0],
                    "speedup_vs_fp64": ms_per_step / r["ms_per_step"]}
        out["learned"] = {
            "what": ("finest-level eigensolver started from the trained network's block (BF16 "
                     "inference on the matrix cores, inside the timed setup); eigen-residual "
                     "test unchanged, cold restart for non-converged subdomains"),
            "training": info,
            "plain_eig_iters_sum": st["eig_iters_sum"],
            "plain_eig_iters_max": st["eig_iters_max"],
            "plain_t_gevp_ms": st["t_gevp_ms"],
            "fp64": leg(rw64),
            "mixed": leg(rw32),
        }
        net.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.workload)
    if args.verbose:
        for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0]):
            if v[1]:
                gbs = v[2] / (v[0] * 1e-3) / 1e9 if v[0] > 0 else 0
                print(f"  {k:20s} {v[0]:9.3f} ms/step  {v[1]:7.0f} launches"
                      f"  {gbs:8.1f} GB/s alg", file=sys.stderr)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
