#!/usr/bin/env python3
"""IMEX-TR benchmark on the 128^3 BCC Landau-Brazovskii workload, one GPU.

A step is one pass of the whole hot path on the workload: a full IMEX-TR
solve (energy and gradient, Algorithm 3's FFT-based subproblem iteration with
its Newton multiplier update and stop test, the ratio test and CONTRACT of
Algorithms 1-2) from the BCC trial state to ||grad E|| < 1e-8, followed by a
60-step preconditioned Lanczos estimate of the smallest Hessian eigenvalue (second-order
check). The input field is resident on the GPU before timing starts; each step
starts from a device copy of it.

Printed: one JSON line with solves/s (FP64), Hessian-vector products/s at
128^3 in FP64 and FP32, the FP32-inner solve rate, the roofline of the
dominant kernel (timed live with HIP events on the plan's stream during the
timed steps) and the CPU oracle's rate on a bounded sample.
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

METRIC = "Hessian-vector products/s + IMEX-TR solves/s at 128³ (FP64 vs FP32+FP64, batched)"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
TOL = 1e-8
LANCZOS_STEPS = 60
# Relative stop floor of FP32 inner loops (||r|| < 1e-5 ||g||): the absolute
# 1e-13 of Section 4 lies below FP32 rounding, and the residual computed through
# FP32 transforms carries a relative error of about eps_32 log2(N) (1.3e-6 at
# 128^3), so a floor of 1e-6 sits on that noise and subproblems end only when
# it happens to dip below; 1e-5 stays clear of it.
FP32_SUB_REL = 1e-5
# kernels of one inner IMEX iteration (Algorithm 3): the unit whose method
# bytes (32 N: read the iterate's spectrum, g and psi-dependent Gamma', write
# b) the roofline figure is quoted on; cubic grids take the plane pass, the
# others the axis-1 and row passes
INNER_KERNELS = ("col0_inv_scale_d", "plane_inner", "col1_inv", "rows_inner", "col1_fwd", "col0_fwd_update", "newton")
TIMING_EVERY = 8  # time one launch in 8 of each inner-iteration kernel during the timed steps
# the default run also times the phase sweep and the 256^3 solve unless the
# run has already taken this long (the whole bench must stay within minutes)
EXTRA_CONFIG_BUDGET_S = 330.0


def kernel_bytes(name: str, prec: str, n) -> float | None:
    """Compulsory bytes one launch of a hot-path kernel must move (each array it
    reads or writes, once), for one instance. c = complex size, r = real."""
    c = 16 if prec == "fp64" else 8
    r = 8 if prec == "fp64" else 4
    N = math.prod(n)
    nh = N // n[-1] * (n[-1] // 2 + 1)
    table = {
        # read T d, b_prev, g; write b_next (the moment partials are a few KB)
        "col0_fwd_update": nh * 4 * c,
        "col0_inv_scale_d": nh * 2 * c,  # read b_prev, write the partial transform
        # read/write the partial transform, read Gamma' (one plane per workgroup)
        "plane_inner": nh * 2 * c + N * r,
        "rows_inner": nh * 2 * c + N * r,
        "col1_inv": nh * 2 * c,
        "col1_fwd": nh * 2 * c,
        "col0_inv": nh * 2 * c,
        "col0_fwd": nh * 2 * c,
        # the three passes of one Hessian-vector product (24 N bytes at the
        # method level: read psi and v, write the product)
        "plane_fwd_phys": 2 * N * r + nh * c,  # read v and psi (mean partial), write the half spectrum
        "col0_fwd_mul_inv": nh * 2 * c,
        "plane_inv_phys": nh * c + 3 * N * r,  # read the spectrum, psi and v, write the product
    }
    return table.get(name)


# the files that define the profiled kernels and their launch shapes (the
# host logic in lb_lib.hip chooses among them; the variant is checked apart)
KERNEL_SOURCES = ("fft.hpp", "kernels.hpp", "launch.hpp")


def source_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2603_03933_amd", "csrc")
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def _pmc():
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    return d if d.get("source_hash") == source_hash() else None


def traffic_from_profiles(kernel: str, section: str = "kernels", variant=None):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources and (for the inner iteration) in the
    variant the benchmark ran (else None)."""
    d = _pmc()
    if d is None:
        return None
    if variant is not None and section == "kernels":
        want = d.get("variant")
        if want is None or any(variant.get(k) != v for k, v in want.items()):
            return None
    k = d.get(section, {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _one_thread():
    """Limit BLAS/OpenMP pools to one thread (numpy's FFT is single-threaded already)."""
    try:
        from threadpoolctl import threadpool_limits

        return threadpool_limits(1)
    except Exception:  # pragma: no cover - threadpoolctl missing
        import contextlib

        return contextlib.nullcontext()


def oracle_endpoint(inst, psi_np, lanczos_steps: int = 12):
    """The oracle's check of a GPU solve's endpoint: its gradient norm and energy
    at the returned field and a preconditioned Lanczos estimate of sigma_1 (an
    upper bound on it)."""
    from oracle import lb_oracle as O
    from paper_2603_03933_amd import inputs as I

    with _one_thread():
        m = O.Model(O.Grid(inst.grid.n, inst.grid.box), inst.params.tau, inst.params.gamma)
        g = O.gradient(m, psi_np)
        ritz, res = O.lanczos_min(m, psi_np, O.fwd(I.hessvec_direction(inst.grid.n, 9)), lanczos_steps, precond_shift=1.0)
        return {"gnorm": O.norm(g), "energy": O.energy(m, psi_np), f"lanczos{lanczos_steps}_precond_ritz": ritz,
                "ritz_residual": res}


def cpu_baseline(inst, inner_total: int, outer_total: int, cg_total: int, budget_s: float):
    """Time the CPU oracle on a bounded sample of the same workload and scale to solves/s."""
    with _one_thread():
        return _cpu_baseline(inst, inner_total, outer_total, cg_total, budget_s)


def _cpu_baseline(inst, inner_total: int, outer_total: int, cg_total: int, budget_s: float):
    import numpy as np

    from oracle import lb_oracle as O

    m = O.Model(O.Grid(inst.grid.n, inst.grid.box), inst.params.tau, inst.params.gamma)
    psi = inst.psi0
    t0 = time.perf_counter()
    g = O.gradient(m, psi)
    E = O.energy(m, psi)
    t_eg = time.perf_counter() - t0
    gmax = float(np.max(np.abs(O.Gamma_p(psi, m.tau, m.gamma))))
    eta = min(0.1, 0.9 / gmax)
    # one inner iteration at a time until the budget is spent
    k = 0
    t1 = time.perf_counter()
    while True:
        O.imex_subproblem(m, psi, g, 1.0, O.SubOpts(eta=eta, max_inner=1))
        k += 1
        if time.perf_counter() - t1 > budget_s or k >= 64:
            break
    t_in = (time.perf_counter() - t1) / k
    # an outer iteration evaluates energy and gradient about twice; a CG step costs one Hv (~ one inner step)
    t_solve = t_in * (inner_total + cg_total) + 2.0 * t_eg * outer_total
    return {
        "value": 1.0 / t_solve,
        "unit": "solves/s",
        "cores": 1,
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
        "kind": "oracle",
        "sample": (
            f"oracle (NumPy FP64, pocketfft, BLAS limited to 1 thread) on the 128^3 BCC input: {k} inner IMEX iterations "
            f"({t_in:.3f} s each) and one energy+gradient ({t_eg:.3f} s); scaled by the GPU solve's counts "
            f"({inner_total} inner, {cg_total} CG, {outer_total} outer)"
        ),
    }


SWEEP_CAPS = {"max_outer": 100, "max_inner": 2000, "eps_sub_rel": {"fp32": FP32_SUB_REL, "fp64": 1e-6}}


def phase_sweep(torch, I, lb, dev, prec="fp32", workers=8, progress=True, batch=8):
    """64 independent 2D solves (n in {64..512}^2, (tau, gamma) on an 8 x 8 grid)
    through lb_imex_tr_solve_many: instances of one grid size are grouped into
    batched plans of up to `batch` instances (one launch per pass for the
    group), and the groups run concurrently on `workers` streams. Capped (the
    tau = 0 row has a degenerate quartic minimum and converges sublinearly):
    the rate counts converged solves only, and the capped ones are listed."""
    insts = I.phase_sweep(64)
    opts = lb.tr_opts(grad_norm_inf=0, eps=TOL, max_outer=SWEEP_CAPS["max_outer"],
                      sub={"max_inner": SWEEP_CAPS["max_inner"], "poll_every": 64, "eps_sub_rel": SWEEP_CAPS["eps_sub_rel"][prec]})
    by_n = {}
    for k, inst in enumerate(insts):
        by_n.setdefault(inst.grid.n[0], []).append(k)
    groups = []  # (plan, instance ids, field)
    for n in sorted(by_n, reverse=True):
        ids = by_n[n]
        for c0 in range(0, len(ids), batch):
            g = ids[c0:c0 + batch]
            plan = lb.Plan(insts[g[0]].grid.n, insts[g[0]].grid.box, batch=len(g), precision=prec)
            psi = torch.from_numpy(np.stack([insts[k].psi0 for k in g])).to(dev)
            groups.append((plan, g, psi))
    res = [None] * len(insts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    half = (len(groups) + 1) // 2
    for part in (groups[:half], groups[half:]):  # progress after each half
        if not part:
            continue
        out = lb.lb_imex_tr_solve_many([g[0] for g in part], [lb.Params(insts[k].params.tau, insts[k].params.gamma)
                                                              for g in part for k in g[1]], [g[2] for g in part], opts,
                                       workers=workers)
        for k, r in zip([k for g in part for k in g[1]], out):
            res[k] = r
        if progress:
            print(f"phase sweep: {sum(r is not None for r in res)}/{len(insts)} solves, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    conv = [k for k in range(len(insts)) if res[k][1] == 0]
    return {
        "metric": "converged IMEX-TR solves/s, 64-instance 2D phase sweep (batched plans, concurrent groups)",
        "value": len(conv) / dt, "unit": "solves/s", "dtype": "f32" if prec == "fp32" else "f64",
        "config": {"workload": "phase_sweep 64 x 2D, n in {64,96,128,256,512}, box 8 pi n/64, tau x gamma 8 x 8",
                   "caps": SWEEP_CAPS, "tol": TOL, "workers": workers, "batch": batch, "groups": len(groups)},
        "seconds": dt, "converged": len(conv), "all_instances_per_s": len(insts) / dt,
        "capped": [{"i": k, "n": insts[k].grid.n[0], "tau": insts[k].params.tau, "gamma": insts[k].params.gamma,
                    "outer": res[k][0].outer, "gnorm": res[k][0].gnorm} for k in range(len(insts)) if res[k][1] != 0],
        "outer": sum(i.outer for i, _ in res), "inner": sum(i.inner_total for i, _ in res),
        "sub_capped": sum(i.sub_capped for i, _ in res),
    }


LARGE_CAPS = {"max_outer": 400, "max_inner": 2000, "eps_sub_rel": FP32_SUB_REL}  # relative floor: FP32 only
LARGE_TOL = 1e-7


def large_solve(torch, I, lb, dev, prec="fp32", verbose=1):
    """The 256^3 mixed-precision workload (tau=-0.25, gamma=0.4, N(0, 0.05^2)
    start): one IMEX-TR solve to ||g||_2 < 1e-7 (FP32 FFT and pointwise
    stages, FP64 reductions and ratio; or FP64 throughout), then 30 steps of
    preconditioned Lanczos from three random starts on the FP64 Hessian product
    (the smallest Ritz value is an upper bound on lambda_min). Progress: one
    line per outer iteration on stderr."""
    inst = I.large_3d(256)
    plan = lb.Plan(inst.grid.n, inst.grid.box, precision=prec)
    prm = lb.Params(inst.params.tau, inst.params.gamma)
    psi = torch.from_numpy(inst.psi0).to(dev)
    # the inner iteration's order for this grid, as at 128^3 (inside the timed region)
    opts = lb.tr_opts(grad_norm_inf=0, eps=LARGE_TOL, max_outer=LARGE_CAPS["max_outer"], verbose=verbose,
                      sub={"max_inner": LARGE_CAPS["max_inner"], "poll_every": 64,
                           "eps_sub_rel": LARGE_CAPS["eps_sub_rel"] if prec == "fp32" else 0.0})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.lb_plan_autotune(prm, psi, reps=10)
    variant = plan.lb_plan_get_variant()
    info, rc = plan.lb_imex_tr_solve(prm, psi, opts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del plan
    p64 = lb.Plan(inst.grid.n, inst.grid.box, precision="fp64")
    ritz = []
    for k in range(3):
        v0 = torch.from_numpy(I.hessvec_direction(inst.grid.n, 100 + k)).to(dev)
        ritz.append(p64.lb_lanczos_min(prm, psi, v0, 30, precond_shift=1.0))
    return {
        "metric": "IMEX-TR solves/s, 256^3 single solve", "value": 1.0 / dt, "unit": "solves/s",
        "dtype": "f32" if prec == "fp32" else "f64",
        "config": {"workload": "large_3d 256^3, box 16 pi, tau -0.25, gamma 0.4, psi0 N(0, 0.05^2) seed 0",
                   "caps": LARGE_CAPS, "tol": LARGE_TOL},
        "seconds": dt, "status": "converged" if rc == 0 else "not_converged", "energy": info.energy,
        "gnorm": info.gnorm, "outer": info.outer, "inner": info.inner_total, "cg": info.cg_total,
        "sub_capped": info.sub_capped,
        "autotune": {"split": variant[0], "plane_pass_threads": variant[1], "column_plan": variant[2]},
        "lanczos30": [{"ritz": r, "residual": e} for r, e in ritz],
        "lambda_min_upper_bound": min(r for r, _ in ritz),
        "sp2_check_passed": min(r for r, _ in ritz) >= -1e-7,
    }


def fp32_floor_scan(torch, I, lb, dev, n=128):
    """The residual floor of FP32 inner iterations: Algorithm 3 at the 128^3 BCC
    input (r = 1) in FP32 and FP64 with stop floors eps_rel ||g|| from 1e-5 down
    to 1e-8, capped at 4000 iterations; a floor below the FP32 transforms'
    noise is never met (the cap is reached)."""
    inst = I.bcc_3d(n)
    prm = lb.Params(inst.params.tau, inst.params.gamma)
    psi = torch.from_numpy(inst.psi0).to(dev)
    out = {}
    for prec in ("fp32", "fp64"):
        plan = lb.Plan(inst.grid.n, inst.grid.box, precision=prec)
        E, g = plan.lb_energy_grad(prm, psi)
        rows = []
        for rel in (1e-5, 3e-6, 1e-6, 3e-7, 1e-7, 3e-8, 1e-8):
            d, info, rc = plan.lb_tr_subproblem(prm, psi, g, 1.0, lb.sub_opts(eta=0.0132, eps_sub=0.0, eps_sub_rel=rel, max_inner=4000, poll_every=64))
            rows.append({"eps_rel": rel, "iters": info.iters, "reached": rc == 0, "resid_rel": info.resid / info.gnorm})
            print(f"floor scan {prec} {rel:g}: {info.iters} iterations, resid/|g| {info.resid / info.gnorm:.2e}", file=sys.stderr, flush=True)
        out[prec] = rows
    return {"fp32_floor_scan": {"workload": f"bcc_3d {n}^3, Algorithm 3 at psi0, r = 1, eta 0.0132, cap 4000", "rows": out}}


def main():
    t_start = time.perf_counter()
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-extra-configs", action="store_true", help="skip the phase sweep and the 256^3 solve")
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--kernel-sample", type=int, default=0, metavar="K",
                    help="only run K iterations of Algorithm 3 on the workload (for counter collection) and exit")
    ap.add_argument("--sample-precision", choices=["fp64", "fp32"], default="fp64",
                    help="precision of the plan that --kernel-sample runs")
    ap.add_argument("--hv-sample", type=int, default=0, metavar="K",
                    help="only run K FP64 Hessian-vector products on the workload (for counter collection) and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (scales HBM counters) and exit")
    ap.add_argument("--large-solve", action="store_true",
                    help="only run the 256^3 single solve (+ 30-step Lanczos, three starts) and exit")
    ap.add_argument("--large-precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--phase-sweep", action="store_true",
                    help="only run the 64-instance 2D phase sweep (concurrent solves) and exit")
    ap.add_argument("--sweep-precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--sweep-workers", type=int, default=8)
    ap.add_argument("--sweep-batch", type=int, default=8, help="instances per batched plan in the phase sweep (1: no batching)")
    ap.add_argument("--plane-split", choices=["auto", "0", "1"], default="auto",
                    help="inner-iteration order of the 128^3 plans: autotuned (default), one workgroup per plane (0), "
                         "or pair-split with the half-plane pass (1)")
    ap.add_argument("--fp32-floor-scan", action="store_true",
                    help="only run the FP32/FP64 subproblem stop-floor scan at 128^3 and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2603_03933_amd import inputs as I
    from paper_2603_03933_amd import lb

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"kernel": "torch.neg float64", "read_bytes": 8 << 27, "write_bytes": 8 << 27, "launches": 5}}))
        return
    if args.phase_sweep:
        r = phase_sweep(torch, I, lb, dev, args.sweep_precision, args.sweep_workers, batch=args.sweep_batch)
        r.update({"n_gpus": 1, "higher_is_better": True, "data": "synthetic"})
        print(json.dumps(r), flush=True)
        return
    if args.large_solve:
        r = large_solve(torch, I, lb, dev, args.large_precision)
        r.update({"n_gpus": 1, "higher_is_better": True, "data": "synthetic"})
        print(json.dumps(r), flush=True)
        return
    if args.fp32_floor_scan:
        print(json.dumps(fp32_floor_scan(torch, I, lb, dev, args.size)), flush=True)
        return
    inst = I.bcc_3d(args.size)
    n, box = inst.grid.n, inst.grid.box
    N = inst.grid.N
    prm = lb.Params(inst.params.tau, inst.params.gamma)
    psi0 = torch.from_numpy(inst.psi0).to(dev)
    v0 = torch.from_numpy(I.hessvec_direction(n, 2)).to(dev)
    psi = torch.empty_like(psi0)
    plan = lb.Plan(n, box, precision="fp64")
    opts = lb.tr_opts(grad_norm_inf=0, eps=TOL, max_outer=500, sub={"max_inner": 10000, "poll_every": 64})

    def step(p, o, out=psi):
        out.copy_(psi0)
        info, rc = p.lb_imex_tr_solve(prm, out, o)
        ritz, res = p.lb_lanczos_min(prm, out, v0, LANCZOS_STEPS, precond_shift=1.0)
        return info, rc, ritz, res

    def choose_variant(p):
        """The inner iteration's plane stage: autotuned, or pinned by --plane-split."""
        if args.plane_split == "auto":
            p.lb_plan_autotune(prm, psi0, reps=50)
        else:
            p.lb_plan_set_plane_split(int(args.plane_split), 0)
        split, threads, cplan = p.lb_plan_get_variant()
        return {"pair_split": split, "plane_pass_threads": threads, "column_plan": cplan,
                "chosen_by": "autotuner" if args.plane_split == "auto" else "pinned"}

    if args.kernel_sample:
        sp = plan if args.sample_precision == "fp64" else lb.Plan(n, box, precision="fp32")
        choose_variant(sp)
        E, g = sp.lb_energy_grad(prm, psi0)
        d, sinfo, src = sp.lb_tr_subproblem(prm, psi0, g, 1.0, lb.sub_opts(eta=0.0132, max_inner=args.kernel_sample))
        torch.cuda.synchronize()
        print(json.dumps({"kernel_sample": {"iterations": sinfo.iters, "workload": f"bcc_3d {n[0]}^3 {args.sample_precision.upper()}, Algorithm 3 at psi0, r = 1"}}))
        return
    if args.hv_sample:
        hv = torch.empty_like(psi0)
        for _ in range(args.hv_sample):
            plan.lb_hessvec(prm, psi0, v0, out=hv)
        torch.cuda.synchronize()
        print(json.dumps({"hv_sample": {"products": args.hv_sample, "workload": f"bcc_3d {n[0]}^3 FP64, H(psi0) v"}}))
        return

    # choose the plane-pass variant for this grid (autotuner), then warm up
    # with every kernel timed (the kernel shares)
    tuned = choose_variant(plan)
    plan.lb_plan_set_timing(True, "")
    for _ in range(max(1, args.warmup)):
        info, rc, ritz, res = step(plan, opts)
    warm = plan.timings()
    total_ms = sum(v[1] for v in warm.values())

    # timed steps: one launch in TIMING_EVERY of each inner-iteration kernel
    # carries start/stop events (on the plan's stream)
    plan.lb_plan_set_timing(True, ",".join(INNER_KERNELS), every=TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        infos.append(step(plan, opts))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = plan.timings()
    plan.lb_plan_set_timing(False, "")
    elapsed = t1 - t0
    info, rc, ritz, res = infos[-1]
    psi_fp64_end = psi.detach().cpu().numpy()

    # roofline of the benchmarked unit, one inner IMEX iteration: its method
    # bytes (32 N, FP64) over the summed average durations of its kernels
    # (the kernels launched once per inner iteration; a pass of the same name
    # outside the inner loop, e.g. an axis-1 pass of a gradient, is excluded)
    most = max((tm[k][0] for k in INNER_KERNELS if k in tm), default=0)
    per_kernel = {k: {"avg_us": tm[k][1] / tm[k][0] * 1e3, "launches_timed": tm[k][0]}
                  for k in INNER_KERNELS if k in tm and tm[k][0] >= 0.5 * most}
    unit_s = sum(v["avg_us"] for v in per_kernel.values()) * 1e-6
    unit_bytes = 32.0 * N
    achieved = unit_bytes / unit_s / 1e9 if unit_s > 0 else None
    counter = [traffic_from_profiles(k, variant=tuned) for k in per_kernel if k != "newton"]
    traffic = sum(counter) if counter and all(c is not None for c in counter) else None
    dominant = max(per_kernel, key=lambda k: per_kernel[k]["avg_us"])
    dom_alg = kernel_bytes(dominant, "fp64", n)
    dom_s = per_kernel[dominant]["avg_us"] * 1e-6
    roofline = {
        "kernel": "inner IMEX iteration (" + " + ".join(per_kernel) + ")",
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS if achieved else None,
        "traffic": traffic,
        "traffic_over_alg": traffic / unit_bytes if traffic else None,
        "alg_bytes_per_unit": unit_bytes,
        "avg_unit_us": unit_s * 1e6,
        "kernels": per_kernel,
        "timing_sample_every": TIMING_EVERY,
        "dominant_kernel_pass_bytes": {
            "kernel": dominant, "alg_bytes_per_launch": dom_alg, "avg_launch_us": dom_s * 1e6,
            "achieved": dom_alg / dom_s / 1e9, "frac": dom_alg / dom_s / 1e9 / HBM_PEAK_GBS,
            "traffic": traffic_from_profiles(dominant, variant=tuned)},
        "wall_iteration_us": elapsed / max(1, sum(i[0].inner_total for i in infos)) * 1e6,
    }

    # Hessian-vector products/s (lb_hessvec, projected) in FP64 and FP32, one
    # field per call and a batch of 8 fields per call (aggregate products/s)
    v_dev = v0.contiguous()

    def hv_rate(precision, batch=1):
        p = plan if (precision == "fp64" and batch == 1) else lb.Plan(n, box, batch=batch, precision=precision)
        ps = psi0 if batch == 1 else psi0.expand(batch, *psi0.shape).contiguous()
        vv = v_dev if batch == 1 else v_dev.expand(batch, *v_dev.shape).contiguous()
        out = torch.empty_like(vv)
        for _ in range(5):
            p.lb_hessvec(prm, ps, vv, out=out)
        torch.cuda.synchronize()
        reps = 200 if batch == 1 else 40
        s = time.perf_counter()
        for _ in range(reps):
            p.lb_hessvec(prm, ps, vv, out=out)
        torch.cuda.synchronize()
        return batch * reps / (time.perf_counter() - s)

    hv = {"fp64": hv_rate("fp64"), "fp64_batch8": hv_rate("fp64", 8)}
    fp32 = fp64_floor = tuned32 = None
    psi_fp32_end = None
    if not args.no_fp32:
        hv["fp32"] = hv_rate("fp32")
        hv["fp32_batch8"] = hv_rate("fp32", 8)

        def timed_solve(p, o):
            out = torch.empty_like(psi0)
            torch.cuda.synchronize()
            s = time.perf_counter()
            i_, rc_, ritz_, _ = step(p, o, out)
            torch.cuda.synchronize()
            d = time.perf_counter() - s
            return out, {
                "solves_per_s": 1.0 / d, "status": "converged" if rc_ == 0 else "not_converged", "energy": i_.energy,
                "gnorm": i_.gnorm, "outer": i_.outer, "inner": i_.inner_total, "cg": i_.cg_total,
                "sub_capped": i_.sub_capped, "lambda_min_ritz": ritz_,
                "inner_iteration_us": d / max(1, i_.inner_total) * 1e6,
                "subproblem_stop": f"||r|| < max(1e-13, {FP32_SUB_REL:g} ||g||)",
            }

        p32 = lb.Plan(n, box, precision="fp32")
        tuned32 = choose_variant(p32)
        sub_rel = {"max_inner": 10000, "poll_every": 64, "eps_sub_rel": FP32_SUB_REL}
        o_rel = lb.tr_opts(grad_norm_inf=0, eps=TOL, max_outer=500, sub=sub_rel)
        out32, fp32 = timed_solve(p32, o_rel)
        psi_fp32_end = out32.cpu().numpy()
        # the same stop rule in FP64 throughout: the precisions compared like for like
        _, fp64_floor = timed_solve(plan, o_rel)
        del p32
    # lb_hessvec reads psi and v and writes hv as FP64 arrays in either precision: 24 N bytes
    for k in list(hv):
        hv[k + "_alg_hbm_frac"] = 24.0 * N * hv[k] / (HBM_PEAK_GBS * 1e9)

    # the other single-GPU configurations: the 64^2 2D solve, Hv at 256^3,
    # and (time permitting) the 64-instance phase sweep and the 256^3 solve
    extra = {}
    if not args.no_fp32:
        c1 = I.single_2d(64)
        p1 = lb.Plan(c1.grid.n, c1.grid.box)
        prm1 = lb.Params(c1.params.tau, c1.params.gamma)
        o1 = lb.tr_opts(grad_norm_inf=0, eps=TOL, sub={"max_inner": 10000})
        psi1 = torch.from_numpy(c1.psi0).to(dev)
        p1.lb_imex_tr_solve(prm1, psi1.clone(), o1)  # warm
        torch.cuda.synchronize()
        s = time.perf_counter()
        i1, rc1 = p1.lb_imex_tr_solve(prm1, psi1, o1)
        torch.cuda.synchronize()
        d1 = time.perf_counter() - s
        v1 = torch.from_numpy(I.hessvec_direction(c1.grid.n, 3)).to(dev)
        r1, _ = p1.lb_lanczos_min(prm1, psi1, v1, 60, precond_shift=1.0)
        extra["solve_64x64_fp64"] = {"solves_per_s": 1.0 / d1, "status": "converged" if rc1 == 0 else "not_converged",
                                     "energy": i1.energy, "gnorm": i1.gnorm, "outer": i1.outer, "inner": i1.inner_total,
                                     "lambda_min_ritz": r1}
        big = I.large_3d(256)
        vb = torch.from_numpy(I.hessvec_direction(big.grid.n, 1)).to(dev)
        pb = torch.from_numpy(big.psi0).to(dev)
        prmb = lb.Params(big.params.tau, big.params.gamma)
        hv256 = {}
        for precision in ("fp64", "fp32"):
            plb = lb.Plan(big.grid.n, big.grid.box, precision=precision)
            ob = torch.empty_like(vb)
            for _ in range(3):
                plb.lb_hessvec(prmb, pb, vb, out=ob)
            torch.cuda.synchronize()
            s = time.perf_counter()
            for _ in range(30):
                plb.lb_hessvec(prmb, pb, vb, out=ob)
            torch.cuda.synchronize()
            hv256[precision] = 30 / (time.perf_counter() - s)
            hv256[precision + "_alg_hbm_frac"] = 24.0 * big.grid.N * hv256[precision] / (HBM_PEAK_GBS * 1e9)
            del plb, ob
        extra["hessvec_256cubed_per_s"] = hv256
        del vb, pb
        if not args.no_extra_configs:
            for name, fn in (("phase_sweep_64x2d_fp32", lambda: phase_sweep(torch, I, lb, dev, "fp32", args.sweep_workers, progress=True, batch=args.sweep_batch)),
                             ("solve_256cubed_fp32_inner", lambda: large_solve(torch, I, lb, dev, "fp32", verbose=0))):
                if time.perf_counter() - t_start > EXTRA_CONFIG_BUDGET_S:
                    extra[name] = {"skipped": f"the run had taken more than {EXTRA_CONFIG_BUDGET_S:g} s"}
                    continue
                print(f"bench: {name}", file=sys.stderr, flush=True)
                extra[name] = fn()

    cpu = None
    endpoint = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(inst, info.inner_total, info.outer, info.cg_total, args.cpu_budget)
        endpoint = {"fp64": oracle_endpoint(inst, psi_fp64_end)}
        if psi_fp32_end is not None:
            endpoint["fp32_inner"] = oracle_endpoint(inst, psi_fp32_end)

    inner_per_s = sum(i[0].inner_total for i in infos) / elapsed
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"bcc_3d {n[0]}^3 FP64 IMEX-TR solve to ||g||<{TOL:g} + 60-step preconditioned Lanczos",
            "grid": list(n),
            "box": box[0],
            "tau": inst.params.tau,
            "gamma": inst.params.gamma,
            "psi0": "BCC {110} unit amplitude + N(0,0.01^2), seed 0",
        },
        "solve": {
            "status": "converged" if rc == 0 else "not_converged",
            "energy": info.energy,
            "gnorm": info.gnorm,
            "outer": info.outer,
            "inner": info.inner_total,
            "cg": info.cg_total,
            "sub_capped": info.sub_capped,
            "newton_steps": info.newton_total,
            "newton_direct_evals": info.newton_direct,
            "accepted": info.accepted,
            "contracted": info.contracted,
            "lambda_min_ritz": ritz,
            "ritz_residual": res,
            "inner_iterations_per_s": inner_per_s,
        },
        "hessvec_per_s": hv,
        "solve_fp32_inner": fp32,
        "solve_fp64_same_floor": fp64_floor,
        "autotune": {"fp64": tuned, "fp32": tuned32},
        "other_configs": extra,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "oracle_endpoint_check": endpoint,
        "kernel_share_warmup": {k: round(v[1] / total_ms, 4) for k, v in sorted(warm.items(), key=lambda kv: -kv[1][1])[:8]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
