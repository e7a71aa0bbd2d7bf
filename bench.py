"""Benchmark: IPM iterations per second of the sketch-preconditioned IPM on one MI355X.

One step = one IPM iteration (Algorithm 3): residual pass, sketch, Gram, Cholesky and
inverse, preconditioned CG to tol 1e-10, direction pass, perturbation v, step lengths and
update. Inputs are resident in HBM before timing starts. The timed window starts at iteration 0
of a fresh solve (x = s = 1, y = 0); when a solve reaches the stop test (relative gap and
residuals <= 1e-8) the state is reset to the start and timing goes on, so exactly --steps
iterations are timed. Beside that window the line carries the whole-solve rate (iterations to
the stop test over the wall time of complete solves).

The default workload is the largest one-GPU dense LP, 2000 x 2*10^6 with A i.i.d. N(0, 1)
stored in BF16 (8 GB) and an FP64 copy of the same values (32 GB): `value` is the plain FP64
form's rate, and the same line compares it with the mixed-precision form (BF16 storage) with and
without the learned warm start on the same LP, each form's result certified on the host in FP64.

Prints one JSON line with the throughput, the roofline record of the CG matvec pass (its average
duration measured with HIP events on the library's stream during the timed region) and the
oracle's CPU baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix

WORKLOADS = {
    "dense_2000x2000000": dict(m=2000, n=2_000_000, w=16000, s=2, seed=64, device=True, storage="bf16",
              desc="dense 2000x2000000 LP, A iid N(0,1) stored in BF16 (8 GB) with an FP64 copy of the same "
                   "values (32 GB) for the plain form, feasible/bounded generator (matrix seed 0, (b, c) seed 64), "
                   "sparse embedding w=16000 s=2, PCG tol 1e-10, to gap 1e-8"),
    "dense_500x100000": dict(m=500, n=100_000, w=2000, s=2, seed=0,
              desc="dense 500x100000 FP64 LP (A iid N(0,1), feasible/bounded generator), "
                   "sparse embedding w=2000 s=2, PCG tol 1e-10, to gap 1e-8"),
    "dense_50x2000": dict(m=50, n=2000, w=200, s=1, seed=0,
              desc="dense 50x2000 FP64 LP, CountSketch w=200 s=1, PCG tol 1e-10, to gap 1e-8"),
}


# HIP events are recorded on every TIMING_PERIOD-th launch of each measured kernel inside the
# timed region (recording them on every launch costs about 7 % of the IPM rate at 500 x 100000)
TIMING_PERIOD = 8


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


MATVEC_SOURCES = ("strip.hip", "strip_ops.hpp", "common.hpp")


def kernel_source_hash() -> str:
    """SHA-256 over the sources that define the CG matvec kernel."""
    h = hashlib.sha256()
    for name in MATVEC_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2209_08722_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def traffic_record(workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when the
    kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "matvec_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        if rec.get("source_sha256") != kernel_source_hash():
            return None
        return rec.get("per_launch_bytes", {}).get(workload)
    except Exception:
        return None


def host_info() -> dict:
    """CPU model, logical CPUs, RAM and the BLAS library NumPy calls (with its thread count)."""
    info = {"cpu_model": None, "logical_cpus": os.cpu_count(), "ram_gb": None, "blas": None, "blas_threads": None}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                info["ram_gb"] = round(int(line.split()[1]) / 2**20, 1)
                break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if blas:
            info["blas"] = f"{blas[0].get('internal_api')} {blas[0].get('version')}"
            info["blas_threads"] = int(blas[0].get("num_threads", 1))
    except Exception:
        pass
    return info


def _baseline_record(it, el, hi, sample):
    cores = hi.get("blas_threads") or hi.get("logical_cpus") or 1
    return {"value": it / el, "unit": "IPM iter/s", "cores": int(cores), "kind": "oracle",
            "sample": sample, "seconds": el, "iterations": it, "cpu_model": hi.get("cpu_model"),
            "blas": hi.get("blas"), "ram_gb": hi.get("ram_gb"), "logical_cpus": hi.get("logical_cpus")}


def cpu_baseline(lp, budget_s: float):
    """The oracle (direct-solver FP64 IPM) on the host cores for about budget_s seconds."""
    from oracle import ipm as oipm
    hi = host_info()
    st = oipm.initial_state(lp.A, lp.b, lp.c)
    prm = oipm.Params()
    it = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        new, info = oipm.step(lp.A, lp.b, lp.c, st, prm, "exact")
        if info.status == oipm.CONVERGED:
            st = oipm.initial_state(lp.A, lp.b, lp.c)
            continue
        st = new
        it += 1
    el = time.perf_counter() - t0
    return _baseline_record(it, el, hi, f"first {it} iterations of the same LP with the oracle's direct-solver "
                                        f"(dense Cholesky of A D^2 A^T) FP64 IPM, {el:.1f} s wall")


def cpu_baseline_device_lp(lp, budget_s: float):
    """The oracle's direct-solver FP64 IPM on the host for a device-resident LP: A copied to the
    host in FP64 (the stored values widened; the copy is not timed), then the oracle's iterations
    from its start point until budget_s has passed (at least one)."""
    import torch
    from oracle import ipm as oipm
    hi = host_info()
    A = lp.A64[:, :lp.n].cpu().numpy() if lp.A64 is not None else lp.A[:, :lp.n].to(torch.float64).cpu().numpy()
    b, c = lp.b.cpu().numpy(), lp.c.cpu().numpy()
    st = oipm.initial_state(A, b, c)
    prm = oipm.Params()
    it = 0
    t0 = time.perf_counter()
    while it == 0 or time.perf_counter() - t0 < budget_s:
        new, info = oipm.step(A, b, c, st, prm, "exact")
        if info.status != oipm.OK:
            break
        st = new
        it += 1
        log(f"  oracle iteration {it}: {time.perf_counter() - t0:.1f} s")
    el = time.perf_counter() - t0
    del A
    return _baseline_record(it, el, hi, f"first {it} iteration(s) of the same {lp.m}x{lp.n} LP with the oracle's "
                                        f"direct-solver (dense Cholesky of A D^2 A^T, 8e12 flop per iteration) FP64 "
                                        f"IPM, A widened to FP64 on the host, {el:.1f} s wall")


def host_certificate(lp, state, block: int = 1 << 17) -> dict:
    """The stop test of a device LP's final point recomputed on the host in FP64 from the stored
    A (streamed in column blocks): relative gap and residuals. With x > 0, s > 0 and residuals at
    rounding level, the objective c^T x is an upper bound of the optimum within the gap."""
    import torch
    x, y, s = (t.cpu().numpy() for t in (state.x, state.y, state.s))
    b, c = lp.b.cpu().numpy(), lp.c.cpu().numpy()
    Ax = np.zeros(lp.m)
    rd2 = 0.0
    for j0 in range(0, lp.n, block):
        j1 = min(lp.n, j0 + block)
        Ab = lp.A[:, j0:j1].to(torch.float64).cpu().numpy()
        Ax += Ab @ x[j0:j1]
        r = Ab.T @ y + s[j0:j1] - c[j0:j1]
        rd2 += float(r @ r)
    obj, dual = float(c @ x), float(b @ y)
    return {"objective": obj, "relgap": abs(obj - dual) / (1 + abs(obj)),
            "rp_rel": float(np.linalg.norm(Ax - b) / (1 + np.linalg.norm(b))),
            "rd_rel": float(np.sqrt(rd2) / (1 + np.linalg.norm(c))),
            "positive": bool(np.all(x > 0) and np.all(s > 0))}


def timed_solve(P, ctx, prob, prm, net=None, timing=False, start=None):
    """One full solve from x = s = 1, y = 0 (or from ``start()``, a fresh State), wall-clocked
    between device synchronizations; with ``timing`` the measured kernels carry HIP events on
    every TIMING_PERIOD-th launch. The result object is under "_res" (dropped before output)."""
    import torch
    st = start() if start is not None else None
    torch.cuda.synchronize()
    if timing:
        ctx.set_timing(TIMING_PERIOD)
    t0 = time.perf_counter()
    res = P.solve(ctx, prob, prm, net=net, st=st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = {}
    if timing:
        for name, kid in (("matvec64", P.native.IPM_KERNEL_MATVEC), ("matvec32", P.native.IPM_KERNEL_MATVEC32),
                          ("resid64", P.native.IPM_KERNEL_RESID64), ("sketch", P.native.IPM_KERNEL_SKETCH),
                          ("gram", P.native.IPM_KERNEL_GRAM), ("warm", P.native.IPM_KERNEL_WARM)):
            kt[name] = ctx.kernel_time(kid)
        ctx.set_timing(False)
    last = res.infos[-1]
    steps = [i for i in res.infos if i["rc"] != P.IPM_CONVERGED]
    return {"_res": res,
        "converged": bool(res.converged), "iterations": res.iterations, "seconds": el,
        "iter_per_s": res.iterations / el if el > 0 else None,
        "cg_iterations": int(sum(i["pcg_iters"] for i in steps)),
        "max_cg_iterations": int(max([i["pcg_iters"] for i in steps] or [0])),
        "refine_rounds": int(sum(i["refine_rounds"] for i in steps)),
        "warm_kept": int(sum(i["warm_used"] for i in steps)),
        "final_relgap": last["relgap"], "final_rp_rel": last["rp_rel"], "final_rd_rel": last["rd_rel"],
        "objective": last["obj"], "kernels": kt,
    }


def algorithm2_comparison(P, ctx, lp, prob, w, s):
    """The feasible IPM (Algorithm 2) from the generator's strictly feasible pair against the
    infeasible IPM (Algorithm 3) from x = s = 1, y = 0 on the same LP: one warm-up solve each,
    then one timed solve each."""
    import torch
    from dataclasses import replace
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    n = lp.A.shape[1]

    def witness():
        return P.State(dev(lp.x0), dev(lp.y0), dev(lp.s0), 0, float(lp.x0 @ lp.s0) / n, 0.0)

    base = P.Params(w=w, s=s, seed=0)
    out = {}
    for name, prm, start in (("algorithm3_infeasible", base, None),
                             ("algorithm2_feasible", replace(base, feasible=1), witness)):
        timed_solve(P, ctx, prob, prm, start=start)
        out[name] = timed_solve(P, ctx, prob, prm, start=start)
        out[name].pop("kernels", None)
        out[name].pop("_res", None)
        log(f"  {name}: {out[name]['iterations']} iterations, {out[name]['iter_per_s']:.1f} it/s")
    return out


def vcorr_ablation(P, ctx):
    """The paper's no-correction comparison (Section 7): the IPM with and without the
    perturbation v on l1-SVM LPs of the experiments' four shapes and sketch widths (Table 1),
    synthetic data; outer iterations, largest and total inner (CG) iterations, time."""
    import lpgen
    out = {}
    for name, sh in lpgen.SVM_SHAPES.items():
        lp = lpgen.svm_lp(sh["m"], sh["N"], seed=0)
        prob = P.Problem.from_lp(lp)
        rec = {"lp_shape": list(lp.A.shape), "w": sh["w"]}
        for tag, v in (("with_v", 1), ("without_v", 0)):
            prm = P.Params(w=sh["w"], s=2, seed=0, vcorr=v)
            timed_solve(P, ctx, prob, prm)
            r = timed_solve(P, ctx, prob, prm)
            rec[tag] = {k: r[k] for k in ("converged", "iterations", "max_cg_iterations", "cg_iterations",
                                          "seconds", "objective", "final_relgap")}
        log(f"  {name} {lp.A.shape}: outer {rec['with_v']['iterations']} / {rec['without_v']['iterations']}, "
            f"inner sum {rec['with_v']['cg_iterations']} / {rec['without_v']['cg_iterations']} (with / without v)")
        out[name] = rec
    return out


def sketch_comparison(P, ctx, prob, m, n, w, s):
    """The sparse embedding (Section 2) against the Gaussian sketch (the experiments' choice,
    Section 7) on the same LP: whole solves, and the Gaussian sketch's MFMA rate (2 m n w flop)."""
    out = {}
    for name, kind in (("sparse_embedding", 0), ("gaussian", 1)):
        prm = P.Params(w=w, s=s, seed=0, sketch=kind)
        timed_solve(P, ctx, prob, prm)
        r = timed_solve(P, ctx, prob, prm, timing=True)
        sk_ms, sk_n = r["kernels"]["sketch"]
        r.pop("kernels")
        r["sketch_ms"] = sk_ms / max(sk_n, 1)
        if kind == 1:
            r["sketch_tflops"] = 2.0 * m * n * w / (r["sketch_ms"] * 1e-3) / 1e12
        out[name] = {k: r[k] for k in ("iterations", "iter_per_s", "cg_iterations", "seconds", "objective",
                                       "sketch_ms") + (("sketch_tflops",) if kind == 1 else ())}
        log(f"  {name}: {r['iterations']} IPM / {r['cg_iterations']} CG iterations, {r['iter_per_s']:.1f} it/s, "
            f"sketch {r['sketch_ms']:.3f} ms")
    return out


def solver_comparison(P, ctx, prob, w, s):
    """CG against the Chebyshev iteration (Section 3.2; eigenvalue interval from a 10-step CG
    probe) as the inner solver on the same LP: whole solves, inner iterations and the time per
    inner iteration (solve time over inner iterations, an upper bound that includes the sketch,
    factorization and step work)."""
    out = {}
    for name, kind in (("cg", 0), ("chebyshev", 1)):
        prm = P.Params(w=w, s=s, seed=0, solver=kind)
        timed_solve(P, ctx, prob, prm)
        r = timed_solve(P, ctx, prob, prm)
        r["us_per_inner_iteration"] = 1e6 * r["seconds"] / max(r["cg_iterations"], 1)
        out[name] = {k: r[k] for k in ("converged", "iterations", "iter_per_s", "cg_iterations",
                                       "max_cg_iterations", "us_per_inner_iteration", "seconds", "objective")}
        log(f"  {name}: {r['iterations']} IPM / {r['cg_iterations']} inner iterations, {r['iter_per_s']:.1f} it/s, "
            f"{r['us_per_inner_iteration']:.1f} us per inner iteration")
    return out


FORM_KEYS = ("converged", "iterations", "seconds", "iter_per_s", "cg_iterations", "max_cg_iterations",
             "refine_rounds", "warm_kept", "final_relgap", "final_rp_rel", "final_rd_rel", "objective")


def family_setup(family: str, test_lp=None):
    """(m, n, w, s, storage, make(seed) -> device LP, description) of a warm-start family: LPs that
    share one A and differ in (b, c)."""
    from lpgen import device as gdev
    if family == "illcond_2000x200000":
        m, n, w, s, storage = 2000, 200_000, 8000, 2, "f32"
        make = lambda sd: gdev.illcond_lp(m, n, seed=sd, storage=storage)  # noqa: E731
        desc = ("ill-conditioned A = U diag(sigma) V^T, 2000x200000, sigma log-spaced 1..1e4, FP32 storage "
                "(FP64 copy for the plain form), w=8000 s=2")
    else:
        m, n, w, s, storage = 2000, 2_000_000, 16000, 2, "bf16"
        base = test_lp if test_lp is not None else gdev.dense_lp(m, n, seed=64, storage=storage, matrix_seed=0)
        make = lambda sd: gdev.with_seed(base, sd)  # noqa: E731
        desc = ("dense 2000x2000000 A iid N(0,1) (one A, (b, c) per seed), BF16 storage (FP64 copy for the "
                "plain form), w=16000 s=2")
    return m, n, w, s, storage, make, desc


def train_warm_start(P, ctx, make, seeds, prm_plain, m: int, epochs: int, tag: str):
    """Plain-form trajectories of the family's LPs ``seeds``, then the network trained on them (Adam,
    batch 64, lr 1e-4, width 256): returns (net, training record)."""
    import torch
    from paper_2209_08722_amd import learned as L
    t0 = time.perf_counter()
    feats, targs, its, cgs = [], [], 0, 0
    for sd in seeds:
        lp = make(sd)
        wide = P.Problem(P.Matrix(lp.A64, lp.n), lp.b, lp.c)
        tr = L.collect(ctx, [wide], prm_plain)
        feats.append(tr.X)
        targs.append(tr.T)
        its += tr.iterations
        cgs += tr.cg_iterations
        log(f"{tag}: training seed {sd}: {tr.iterations} IPM iterations, {tr.cg_iterations} CG iterations")
        del lp, wide
    X, T = torch.cat(feats), torch.cat(targs)
    t_collect = time.perf_counter() - t0
    net = L.Mlp(m + L.N_EXTRA, 256, m, __import__("lpgen").mlp_init(m + L.N_EXTRA, 256, m, 0, out_scale=1.0))
    l0 = L.evaluate(ctx, net, X, T)
    hist = L.train(ctx, net, X, T, epochs=epochs, batch=64, lr=1e-4, seed=0)
    t_train = time.perf_counter() - t0 - t_collect
    log(f"{tag}: {X.shape[0]} samples, loss {l0:.3f} -> {hist[-1]:.3f} ({t_collect:.1f} s collecting, "
        f"{t_train:.1f} s training)")
    rec = {"seeds": [int(seeds[0]), int(seeds[-1])] if len(seeds) else [], "n_seeds": len(seeds),
           "samples": int(X.shape[0]), "ipm_iterations": its, "cg_iterations": cgs, "epochs": epochs,
           "loss_first": l0, "loss_last": hist[-1], "seconds_collect": t_collect, "seconds_train": t_train}
    del X, T
    return net, rec


def learned_protocol(P, ctx, family: str, n_train: int, n_test: int, epochs: int) -> dict:
    """The learned warm start's train / held-out protocol: the network is trained on plain-form
    trajectories of seeds 0..n_train-1 of a family, then every held-out seed n_train..n_train+
    n_test-1 is solved to the stop test in the plain FP64 and the mixed form from the zero, the
    previous-dy and the learned start (one whole solve each, same stop test). Reports per seed and
    in total: IPM and CG iterations, wall time and IPM it/s, and the objective spread."""
    import torch
    m, n, w, s, storage, make, desc = family_setup(family)
    prm = {"plain": P.Params(w=w, s=s, seed=0), "mixed": P.Params(w=w, s=s, seed=0, precision=P.IPM_MIXED)}
    net, rec = train_warm_start(P, ctx, make, list(range(n_train)), prm["plain"], m, epochs, "protocol")
    out = {"family": family, "workload": desc, "m": m, "n": n, "w": w, "s": s, "training": rec,
           "held_out": [n_train, n_train + n_test - 1], "per_seed": []}
    starts = ("zero", "prev", "learned")
    tot = {(f, st): {"ipm": 0, "cg": 0, "seconds": 0.0, "warm_kept": 0, "converged": 0,
                     "warm_ms": 0.0, "warm_launches": 0, "matvec_ms": 0.0, "matvec_launches": 0}
           for f in prm for st in starts}
    warmed = False
    for sd in range(n_train, n_train + n_test):
        lp = make(sd)
        probs = {"plain": P.Problem(P.Matrix(lp.A64, n), lp.b, lp.c), "mixed": P.Problem(P.Matrix(lp.A, n), lp.b, lp.c)}
        if not warmed:
            for f in prm:   # a few untimed steps per form first (workspaces, code paths)
                st0 = P.State.initial(m, n)
                for _ in range(3):
                    P.ipm_step(ctx, probs[f], st0, prm[f])
            warmed = True
        row = {"seed": sd}
        objs = []
        for f in prm:
            for stt in starts:
                pr = prm[f]
                if stt == "prev":
                    from dataclasses import replace
                    pr = replace(pr, warm_start=P.IPM_WARM_PREV)
                r = timed_solve(P, ctx, probs[f], pr, net=net if stt == "learned" else None, timing=True)
                r.pop("_res")
                t = tot[(f, stt)]
                for key, kname in (("warm", "warm"), ("matvec", "matvec64")):
                    ms_, cnt_ = r["kernels"].get(kname, (0.0, 0))
                    t[f"{key}_ms"] += ms_
                    t[f"{key}_launches"] += cnt_
                t["ipm"] += r["iterations"]
                t["cg"] += r["cg_iterations"]
                t["seconds"] += r["seconds"]
                t["warm_kept"] += r["warm_kept"]
                t["converged"] += int(r["converged"])
                objs.append(r["objective"])
                row[f"{f}_{stt}"] = {"ipm": r["iterations"], "cg": r["cg_iterations"], "seconds": r["seconds"],
                                     "iter_per_s": r["iter_per_s"], "objective": r["objective"],
                                     "converged": r["converged"], "warm_kept": r["warm_kept"]}
        row["objective_spread"] = (max(objs) - min(objs)) / (1 + abs(objs[0]))
        out["per_seed"].append(row)
        log(f"protocol seed {sd}: " + ", ".join(f"{f}/{stt} CG {row[f'{f}_{stt}']['cg']} "
                                                 f"({row[f'{f}_{stt}']['iter_per_s']:.2f} it/s)"
                                                 for f in prm for stt in starts))
        del lp, probs
    totals = {}
    for (f, stt), t in tot.items():
        totals[f"{f}_{stt}"] = {**t, "iter_per_s": t["ipm"] / t["seconds"] if t["seconds"] > 0 else None,
                                "cg_per_ipm": t["cg"] / t["ipm"] if t["ipm"] else None,
                                "warm_ms_per_launch": t["warm_ms"] / t["warm_launches"] if t["warm_launches"] else None,
                                "matvec_ms_per_launch": (t["matvec_ms"] / t["matvec_launches"]
                                                         if t["matvec_launches"] else None)}
    out["totals"] = totals
    for f in prm:
        z, pv, ln = (totals[f"{f}_{k}"] for k in starts)
        out[f"{f}_learned_vs_prev"] = {"cg_saving": 1.0 - ln["cg"] / pv["cg"] if pv["cg"] else None,
                                       "rate_ratio": ln["iter_per_s"] / pv["iter_per_s"] if pv["iter_per_s"] else None}
        out[f"{f}_learned_vs_zero"] = {"cg_saving": 1.0 - ln["cg"] / z["cg"] if z["cg"] else None,
                                       "rate_ratio": ln["iter_per_s"] / z["iter_per_s"] if z["iter_per_s"] else None}
    out["max_objective_spread"] = max(r["objective_spread"] for r in out["per_seed"]) if out["per_seed"] else None
    torch.cuda.empty_cache()
    return out


def forms_comparison(P, ctx, family: str, train_seeds: int, epochs: int, test_lp=None, plain=None):
    """The plain FP64 form against the mixed-precision forms (low-precision storage of the same
    values) with zero, previous-dy and learned warm starts on one held-out LP of a family, every
    form solved to the same stop test, one whole solve each (HIP events on every TIMING_PERIOD-th
    launch of the measured kernels). The network is trained first (untimed) on plain-form
    trajectories of the family's training seeds. Every form's final point is certified on the
    host in FP64 (host_certificate). ``test_lp`` / ``plain``: the held-out LP and its plain-form
    record when the caller already has them."""
    import torch
    m, n, w, s, storage, make, desc = family_setup(family, test_lp)
    test_seed = 64
    prm_plain = P.Params(w=w, s=s, seed=0)
    prm_mixed = P.Params(w=w, s=s, seed=0, precision=P.IPM_MIXED)

    def problems(lp):
        return P.Problem(P.Matrix(lp.A, lp.n), lp.b, lp.c), P.Problem(P.Matrix(lp.A64, lp.n), lp.b, lp.c)

    log(f"forms: training the warm-start network on {train_seeds} plain-form solves ({desc})")
    net, rec = train_warm_start(P, ctx, make, list(range(train_seeds)), prm_plain, m, epochs, "forms")

    lp = test_lp if test_lp is not None else make(test_seed)
    low, wide = problems(lp)
    out = {"workload": desc, "m": m, "n": n, "w": w, "s": s, "test_seed": test_seed, "training": rec}
    runs = [("plain_fp64", wide, prm_plain, None), ("mixed", low, prm_mixed, None),
            ("mixed_prev", low, P.Params(w=w, s=s, seed=0, precision=P.IPM_MIXED, warm_start=P.IPM_WARM_PREV), None),
            ("mixed_learned", low, prm_mixed, net),
            ("mixed_f32acc", low, P.Params(w=w, s=s, seed=0, precision=P.IPM_MIXED_F32ACC), None)]
    warmed = {P.IPM_PLAIN} if train_seeds > 0 else set()
    for name, prob, prm, nt in runs:
        if name == "plain_fp64" and plain is not None:
            out[name] = plain
            continue
        if prm.precision not in warmed:
            # a few untimed steps per precision first (workspaces, code paths)
            st = P.State.initial(m, n)
            for _ in range(3):
                P.ipm_step(ctx, prob, st, prm)
            warmed.add(prm.precision)
        r = timed_solve(P, ctx, prob, prm, net=nt, timing=True)
        r["host_certificate"] = host_certificate(lp, r.pop("_res").state)
        log(f"forms: {name}: {r['iterations']} iterations in {r['seconds']:.3f} s "
            f"({r['iter_per_s']:.2f} it/s), CG {r['cg_iterations']}, obj {r['objective']:.12e}, "
            f"host relgap {r['host_certificate']['relgap']:.2e}")
        out[name] = r
    ref = out["plain_fp64"]["objective"]
    for name, *_ in runs:
        out[name]["objective_rel_diff_vs_plain"] = abs(out[name]["objective"] - ref) / (1 + abs(ref))
    out["speedup_mixed_learned_vs_plain"] = out["mixed_learned"]["iter_per_s"] / out["plain_fp64"]["iter_per_s"]
    out["time_to_gap_ratio"] = out["plain_fp64"]["seconds"] / out["mixed_learned"]["seconds"]
    esz = 4 if storage == "f32" else 2
    ms, cnt = out["mixed_learned"]["kernels"].get("matvec64", (0.0, 0))
    if cnt:
        out["matvec_lowprec_storage_hbm_gbps"] = (m * n * esz + n * 8) / (ms / cnt * 1e-3) / 1e9
    ms, cnt = out["plain_fp64"]["kernels"].get("matvec64", (0.0, 0))
    if cnt:
        out["matvec_fp64_hbm_gbps"] = (m * n * 8 + n * 8) / (ms / cnt * 1e-3) / 1e9
    del low, wide
    if test_lp is None:
        del lp
    torch.cuda.empty_cache()
    return out


def stream_probe(P, ctx, nbytes: int, reps: int = 20) -> dict:
    """Attainable HBM bandwidth on this GPU for the streaming passes' access pattern: the read
    pass of ipm_stream_read and the copy pass of ipm_stream_copy over nbytes (HIP events at each
    pass's own start and end, every launch; the first launch of each is a warm-up)."""
    import torch
    count = nbytes // 8
    x = torch.full((count,), 0.5, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    out = {"bytes": count * 8}
    for name, kid, call, moved in (
            ("read", P.native.IPM_KERNEL_STREAM_READ, lambda: P.ipm_stream_read(ctx, x), count * 8),
            ("copy", P.native.IPM_KERNEL_STREAM_COPY, lambda: P.ipm_stream_copy(ctx, x, y), 2 * count * 8)):
        call()
        torch.cuda.synchronize()
        ctx.set_timing(1)
        for _ in range(reps):
            call()
        ms, cnt = ctx.kernel_time(kid)
        ctx.set_timing(False)
        out[f"{name}_gbps"] = moved / (ms / cnt * 1e-3) / 1e9
        out[f"{name}_us"] = ms / cnt * 1e3
    del x, y
    return out


def random_rows(torch, g, m: int, n: int, tdt):
    """An m x n N(0,1) matrix in the storage type, rows padded to 128 bytes, drawn 256 rows at a
    time in FP32 (bounded temporary memory)."""
    esz = torch.empty((), dtype=tdt).element_size()
    ld = (n + 128 // esz - 1) // (128 // esz) * (128 // esz)
    A = torch.empty((m, ld), dtype=tdt, device="cuda:0")
    for r0 in range(0, m, 256):
        r1 = min(m, r0 + 256)
        A[r0:r1] = torch.randn((r1 - r0, ld), dtype=torch.float32, device="cuda:0", generator=g).to(tdt)
    return A


def kernel_only(args) -> int:
    """One kernel family on a seeded random input, for rocprofv3 runs: the factorization of a
    random FP64 sketch B (m x w), the Gaussian sketch of a random FP64 A, the sparse-embedding
    sketch (s = 2), the matvec over a random A (m x n, N(0,1) in the storage type) or the
    bandwidth probes. Prints the time per call and the rate against the algorithmic work."""
    import torch
    import paper_2209_08722_amd as P
    ctx = P.Context(0)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(0)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if args.gram:
        m, w = (int(t) for t in args.gram.lower().split("x"))
        B = torch.randn((m, w), dtype=torch.float64, device="cuda:0", generator=g) / math.sqrt(w)
        for rep in range(3):
            ev0.record()
            P.ipm_precond_factor(ctx, B, want_L=False)
            ev1.record()
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1)
            log(f"factor {m} x {w}: {ms:.3f} ms (Gram {m * m * w / 1e12:.3f} TFLOP SYRK count, "
                f"{m * m * w / (ms * 1e-3) / 1e12:.1f} TFLOP/s over the whole factorization)")
    elif args.gauss:
        shape, ws = args.gauss.lower().split(":")
        m, n = (int(t) for t in shape.split("x"))
        w = int(ws)
        A = torch.randn((m, n), dtype=torch.float64, device="cuda:0", generator=g)
        mat = P.Matrix(A, n) if n % 16 == 0 else P.Matrix.from_numpy(A.cpu().numpy())
        d = torch.exp(torch.empty(n, dtype=torch.float64, device="cuda:0").uniform_(-3, 3, generator=g))
        for rep in range(3):
            ev0.record()
            P.ipm_sketch_gaussian(ctx, mat, d, 5, rep, w)
            ev1.record()
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1)
            log(f"gaussian sketch {m} x {n}, w = {w}: {ms:.3f} ms ({2.0 * m * n * w / (ms * 1e-3) / 1e12:.1f} "
                f"TFLOP/s on 2 m n w)")
    elif args.stream:
        r = stream_probe(P, ctx, args.stream)
        log(f"stream probe {r['bytes'] / 1e9:.3f} GB: read {r['read_us']:.1f} us = {r['read_gbps']:.0f} GB/s; "
            f"copy {r['copy_us']:.1f} us = {r['copy_gbps']:.0f} GB/s (read + written bytes)")
    elif args.sketch:
        shape, ws, dt = args.sketch.lower().split(":")
        m, n = (int(t) for t in shape.split("x"))
        w = int(ws)
        tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dt]
        esz = torch.empty((), dtype=tdt).element_size()
        mat = P.Matrix(random_rows(torch, g, m, n, tdt), n)
        d = torch.exp(torch.empty(n, dtype=torch.float64, device="cuda:0").uniform_(-3, 3, generator=g))
        nbytes = m * n * esz + 8 * n + m * w * 8
        for rep in range(5):
            ev0.record()
            P.ipm_sketch(ctx, mat, d, 5, rep, w, 2)
            ev1.record()
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1)
            log(f"sparse sketch {m} x {n} {dt}, w = {w}, s = 2: {ms:.3f} ms ({nbytes / (ms * 1e-3) / 1e9:.0f} "
                f"GB/s of {nbytes / 1e9:.3f} GB algorithmic bytes: A, d and B once)")
    else:
        shape, dt = args.matvec.lower().split(":")
        m, n = (int(t) for t in shape.split("x"))
        tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dt]
        esz = torch.empty((), dtype=tdt).element_size()
        mat = P.Matrix(random_rows(torch, g, m, n, tdt), n)
        d2 = torch.exp(torch.empty(n, dtype=torch.float64, device="cuda:0").uniform_(-3, 3, generator=g))
        v = torch.randn(m, dtype=torch.float64, device="cuda:0", generator=g)
        nbytes = m * n * esz + 8 * n
        for rep in range(5):
            ev0.record()
            P.ipm_normal_matvec(ctx, mat, d2, v)
            ev1.record()
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1)
            log(f"matvec {m} x {n} {dt}: {ms:.3f} ms ({nbytes / (ms * 1e-3) / 1e9:.0f} GB/s of "
                f"{nbytes / 1e9:.2f} GB algorithmic bytes)")
    ctx.close()
    return 0


def timed_window(P, ctx, prob, prm, m, n, steps: int, warmup: int):
    """`warmup` untimed steps from a fresh start, then `steps` steps timed from iteration 0 of a
    fresh solve (the state is reset to the start after each converged solve), bracketed by
    device synchronizations; HIP events on every TIMING_PERIOD-th launch of the measured kernels."""
    import torch
    st = P.State.initial(m, n)
    conv = []

    def one_step(st):
        while True:
            info = P.ipm_step(ctx, prob, st, prm)
            if info["rc"] == P.IPM_CONVERGED:
                conv.append((st.k, info))
                st = P.State.initial(m, n)
                continue
            return st, info

    log(f"warmup {warmup} steps")
    for _ in range(warmup):
        st, _ = one_step(st)
    st = P.State.initial(m, n)
    torch.cuda.synchronize()
    ctx.set_timing(TIMING_PERIOD)
    pcg = []
    log(f"timing {steps} steps from iteration 0 of a fresh solve")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        st, info = one_step(st)
        pcg.append(info["pcg_iters"])
        if (i + 1) % 10 == 0:
            log(f"  step {i + 1}/{steps}")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = {name: ctx.kernel_time(kid) for name, kid in (("matvec", P.native.IPM_KERNEL_MATVEC),
                                                     ("sketch", P.native.IPM_KERNEL_SKETCH),
                                                     ("gram", P.native.IPM_KERNEL_GRAM))}
    ctx.set_timing(False)
    return {"seconds": el, "pcg_iters": pcg, "kernels": kt, "last_k": st.k}


def roofline_record(kernel_ms, launches, nbytes, probe_gbps, traffic, kernel, probe_desc):
    avg = kernel_ms / max(launches, 1) * 1e-3
    gbs = nbytes / avg / 1e9 if launches else None
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (gbs / HBM_PEAK_GBS) if gbs else None, "traffic": traffic, "kernel": kernel,
            "algorithmic_bytes_per_launch": nbytes, "avg_launch_us": avg * 1e6, "timed_launches": launches,
            "timing_period": TIMING_PERIOD, "measured_peak": probe_gbps,
            "frac_measured": (gbs / probe_gbps) if (gbs and probe_gbps) else None,
            "measured_peak_kernel": probe_desc}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="dense_2000x2000000", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", action="store_true",
                    help="also run the Algorithm 2 comparison, the v-correction ablation, the sketch and inner-solver "
                         "comparisons (on the workload's LP; host workloads only)")
    ap.add_argument("--forms", default="auto", choices=["auto", "illcond_2000x200000", "dense_2000x2000000", "none"],
                    help="family of the plain vs mixed+learned comparison (auto: the 2000x2000000 workload itself "
                         "when it is the benchmark's, else none)")
    ap.add_argument("--train-seeds", type=int, default=2)
    ap.add_argument("--solves", type=int, default=3,
                    help="whole plain solves timed after the window; their median rate is reported")
    ap.add_argument("--learned-protocol", default="", choices=["", "illcond_2000x200000", "dense_2000x2000000"],
                    help="only run the learned warm start's train / held-out protocol on this family "
                         "(--protocol-train seeds for training, the next --protocol-test held out)")
    ap.add_argument("--ipm-steps", default="", metavar="WORKLOAD:FORM:K",
                    help="only run K IPM steps of a named seeded workload (lpgen.WORKLOADS, built on the host; "
                         "FORM plain, mixed or f32acc), for kernel profiling of the sparse passes")
    ap.add_argument("--protocol-train", type=int, default=64)
    ap.add_argument("--protocol-test", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (HBM counter calibration)")
    ap.add_argument("--gram", default="", metavar="MxW",
                    help="only run the preconditioner factorization (Gram B B^T, Cholesky, L^-1) of a "
                         "random FP64 m x w sketch, three times (kernel profiling)")
    ap.add_argument("--gauss", default="", metavar="MxN:W",
                    help="only run the Gaussian sketch B = A D W of a random FP64 m x n matrix with w "
                         "columns of W, three times (kernel profiling)")
    ap.add_argument("--stream", type=int, default=0, metavar="BYTES",
                    help="only run the bandwidth probes (ipm_stream_read, ipm_stream_copy) over BYTES "
                         "bytes, 21 times each (kernel profiling)")
    ap.add_argument("--sketch", default="", metavar="MxN:W:DTYPE",
                    help="only run the sparse-embedding sketch (s = 2) of a random m x n matrix stored "
                         "as f64, f32 or bf16 with w buckets, five times (kernel profiling)")
    ap.add_argument("--matvec", default="", metavar="MxN:DTYPE",
                    help="only run the normal-equations matvec A D^2 A^T v on a random m x n matrix "
                         "stored as f64, f32 or bf16, five times (kernel profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding is a design note, not built", file=sys.stderr)
        return 2

    import torch
    if args.calibrate_copy:
        nel = args.calibrate_copy // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {nel * 8} bytes")
        return 0
    if args.gram or args.matvec or args.gauss or args.sketch or args.stream:
        return kernel_only(args)
    import lpgen
    import paper_2209_08722_amd as P
    if args.ipm_steps:
        name, form, ks = args.ipm_steps.split(":")
        lp = lpgen.workload(name)
        tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[lp.storage]
        prob = P.Problem.from_lp(lp, dtype=tdt)
        prec = {"plain": P.IPM_PLAIN, "mixed": P.IPM_MIXED, "f32acc": P.IPM_MIXED_F32ACC}[form]
        ctx = P.Context(0)
        prm = P.Params(w=lp.meta["w"], s=lp.meta["s"], seed=0, precision=prec)
        st = P.State.initial(lp.m, lp.n)
        for k in range(int(ks)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = P.ipm_step(ctx, prob, st, prm)
            torch.cuda.synchronize()
            log(f"{name} {form} step {k}: {1e3 * (time.perf_counter() - t0):.2f} ms, CG {info['pcg_iters']}, "
                f"relgap {info['relgap']:.2e}")
        ctx.close()
        return 0
    if args.learned_protocol:
        ctx = P.Context(0)
        res = learned_protocol(P, ctx, args.learned_protocol, args.protocol_train, args.protocol_test, args.epochs)
        print(json.dumps(res))
        return 0

    wl = WORKLOADS[args.workload]
    m, n, w, s = wl["m"], wl["n"], wl["w"], wl["s"]
    on_device = wl.get("device", False)
    log(f"generating workload {args.workload}: {wl['desc']}")
    if on_device:
        from lpgen import device as gdev
        lp = gdev.dense_lp(m, n, seed=wl["seed"], storage=wl["storage"], matrix_seed=0)
        prob = P.Problem(P.Matrix(lp.A64, n), lp.b, lp.c)
        esz = 8
    else:
        lp = lpgen.workload(args.workload, seed=wl["seed"])
        prob = P.Problem.from_lp(lp)
        esz = 8
    ctx = P.Context(0)
    prm = P.Params(w=w, s=s, seed=0 if on_device else wl["seed"])
    torch.cuda.synchronize()

    win = timed_window(P, ctx, prob, prm, m, n, args.steps, args.warmup)
    el = win["seconds"]
    mv_ms, mv_n = win["kernels"]["matvec"]
    sk_ms, sk_n = win["kernels"]["sketch"]
    gr_ms, gr_n = win["kernels"]["gram"]

    # whole solves from the start: the rate over complete solves (iterations to the stop test over
    # wall time), which the window above only samples; the median of --solves solves is quoted
    runs = []
    for i in range(max(1, args.solves)):
        log(f"whole solve {i + 1} of {max(1, args.solves)} (plain FP64)")
        r = timed_solve(P, ctx, prob, prm, timing=(i == 0))
        if i > 0:
            r.pop("_res")
        runs.append(r)
        log(f"  {r['iterations']} iterations in {r['seconds']:.2f} s = {r['iter_per_s']:.2f} it/s")
    whole = runs[0]
    rates = sorted(r["iter_per_s"] for r in runs)
    whole["iter_per_s_solves"] = [r["iter_per_s"] for r in runs]
    whole["iter_per_s_median"] = rates[len(rates) // 2]
    res = whole.pop("_res")
    if on_device:
        whole["host_certificate"] = host_certificate(lp, res.state)
    else:
        x, y, s_ = (t.cpu().numpy() for t in (res.state.x, res.state.y, res.state.s))
        obj = float(lp.c @ x)
        whole["host_certificate"] = {
            "objective": obj, "relgap": abs(obj - float(lp.b @ y)) / (1 + abs(obj)),
            "rp_rel": float(np.linalg.norm(lp.A @ x - lp.b) / (1 + np.linalg.norm(lp.b))),
            "rd_rel": float(np.linalg.norm(lp.A.T @ y + s_ - lp.c) / (1 + np.linalg.norm(lp.c))),
            "positive": bool(np.all(x > 0) and np.all(s_ > 0))}
    del res
    log(f"  {whole['iterations']} iterations in {whole['seconds']:.2f} s = {whole['iter_per_s']:.2f} it/s, "
        f"CG {whole['cg_iterations']}, host relgap {whole['host_certificate']['relgap']:.2e}")

    a_bytes = m * n * esz
    mv_bytes = a_bytes + n * 8                     # A once + d^2 (algorithmic, per launch)
    probe_bytes = min(mv_bytes, 8 * 10**9)
    log(f"stream probe over {probe_bytes / 1e9:.2f} GB")
    probe = stream_probe(P, ctx, probe_bytes)
    sk_bytes = a_bytes + n * 8 + m * w * 8         # A once + d + B written
    gram_flops = float(m) * m * w                  # SYRK count m^2 w
    sk_gbs = sk_bytes / (sk_ms / max(sk_n, 1) * 1e-3) / 1e9 if sk_n else None
    gr_tf = gram_flops / (gr_ms / max(gr_n, 1) * 1e-3) / 1e12 if gr_n else None
    probe_desc = (f"ipm_stream_read: read-only pass over {probe_bytes / 1e9:.2f} GB, the same access pattern "
                  f"(k_stream_read)")
    roof = roofline_record(mv_ms, mv_n, mv_bytes, probe["read_gbps"], traffic_record(args.workload),
                           "CG matvec pass q = A D^2 A^T v, FP64 storage (k_strip OpMatvec)", probe_desc)

    out = {
        "metric": "IPM iter/s + matvec HBM GB/s, FP64 plain vs mixed+learned at gap 1e-8",
        "value": args.steps / el,
        "unit": "IPM iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": wl["desc"], "m": m, "n": n, "w": w, "s": s,
                   "form": "plain FP64", "window": f"IPM iterations 0-{args.steps - 1} of a fresh solve",
                   "mean_pcg_iters_window": float(np.mean(win["pcg_iters"])), "parallelism": "1 GPU"},
        "whole_solve": {**whole, "note": "complete solves from the start (iter_per_s: the first, with kernel "
                                         "timing on every 8th launch; iter_per_s_median over all): the rate to "
                                         "quote"},
        "roofline": roof,
        "stream_probe": probe,
        "matvec_hbm_gbps": roof["achieved"],
        "sketch_hbm_gbps": sk_gbs,
        "gram_tflops": gr_tf,
        "gram_mfma_frac": (gr_tf / FP64_MFMA_PEAK_TFLOPS) if gr_tf else None,
    }
    if args.extras and not on_device:
        log("feasible (Algorithm 2) vs infeasible (Algorithm 3) IPM")
        out["algorithms"] = algorithm2_comparison(P, ctx, lp, prob, w, s)
        log("v-correction ablation on l1-SVM LPs")
        out["v_correction_ablation"] = vcorr_ablation(P, ctx)
        log("sparse embedding vs Gaussian sketch")
        out["sketches"] = sketch_comparison(P, ctx, prob, m, n, w, s)
        log("CG vs Chebyshev inner solver")
        out["inner_solvers"] = solver_comparison(P, ctx, prob, w, s)
    forms = args.forms
    if forms == "auto":
        forms = "dense_2000x2000000" if args.workload == "dense_2000x2000000" else "none"
    if forms != "none":
        same = forms == args.workload
        out["forms"] = forms_comparison(P, ctx, forms, args.train_seeds, args.epochs,
                                        test_lp=lp if same else None,
                                        plain={k: v for k, v in whole.items()} if same else None)
        f = out["forms"]
        ms, cnt = f["mixed_learned"]["kernels"].get("matvec64", (0.0, 0))
        esz_low = 2 if forms == "dense_2000x2000000" else 4
        if cnt:
            out["roofline_mixed_matvec"] = roofline_record(
                ms, cnt, f["m"] * f["n"] * esz_low + f["n"] * 8, probe["read_gbps"],
                traffic_record(f"{forms}_bf16") if esz_low == 2 else None,
                f"CG matvec pass of the mixed form, {'BF16' if esz_low == 2 else 'FP32'} storage, FP64 "
                f"accumulation (k_strip OpMatvec)", probe_desc)
        out["headline_comparison"] = {
            "plain_fp64_iter_per_s": f["plain_fp64"]["iter_per_s"],
            "mixed_learned_iter_per_s": f["mixed_learned"]["iter_per_s"],
            "ratio": f["speedup_mixed_learned_vs_plain"],
            "objective_rel_diff": f["mixed_learned"]["objective_rel_diff_vs_plain"],
            "host_relgap_plain": f["plain_fp64"]["host_certificate"]["relgap"],
            "host_relgap_mixed_learned": f["mixed_learned"]["host_certificate"]["relgap"],
            "note": "whole solves of the same LP; each objective is an upper bound of the optimum within its "
                    "host-recomputed FP64 relative gap (x, s > 0, residuals at rounding level)"}
    if not args.no_cpu_baseline:
        log(f"cpu baseline (oracle) for ~{args.cpu_budget:.0f} s")
        out["cpu_baseline"] = cpu_baseline_device_lp(lp, args.cpu_budget) if on_device \
            else cpu_baseline(lp, args.cpu_budget)
    ctx.close()
    print(json.dumps(out, default=float), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
