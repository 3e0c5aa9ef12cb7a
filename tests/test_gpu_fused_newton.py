"""The multiplier step of Algorithm 3 (Newton on the secular equation of
Section 3.2, eq. lambda_update_rule, and the stop test) taken at the start of
the next iteration's axis-0 inverse pass (lb_sub_opts.fused_newton: by default
where it pays, forced here with 2) against the separate one-workgroup Newton
launch (fused_newton = 0): the same bits (iterate, multiplier, residual,
iteration and Newton counts) on grids with one and with several hundred update
workgroups, in the split orders, in FP32, at an iteration cap, on a subproblem
whose first steps need sums over the spectrum (the fused pass pauses there and
the Newton kernel takes the step), and in batched solves whose instances pause
and stop at different steps. Parity of both forms with the oracle is in
test_gpu_newton_workgroups and the other subproblem tests, which run the
default."""
import math

import numpy as np
import pytest
import torch

from oracle import lb_oracle as O
from paper_2603_03933_amd import inputs as I
from paper_2603_03933_amd import lb

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


INFO_FIELDS = ("lambda_", "resid", "dnorm", "iters", "newton_iters", "newton_direct", "status")

# name: grid, box, radius (None: half the norm of the unconstrained step, so
# that the constraint is active), noise seed, precision, plane split (None:
# built in)
CASES = {
    # 32^3: 9 update workgroups of 64 columns, the last one half full
    "3d_32": ((32, 32, 32), (8 * math.pi,) * 3, 0.29, 33, "fp64", None),
    "3d_32_fp32": ((32, 32, 32), (8 * math.pi,) * 3, 0.29, 33, "fp32", None),
    # non-square 2D (multi-kernel path)
    "2d_48x96": ((48, 96), (12 * math.pi, 24 * math.pi), 0.28, 34, "fp64", None),
    # lambda ~ 37: the first steps need sums over the spectrum, so the fused
    # pass pauses and the Newton kernel takes those steps
    "2d_48x96_far": ((48, 96), (12 * math.pi, 24 * math.pi), 0.2, 34, "fp64", None),
    # split orders with two parts (lanes 16 apart) and four (16 columns per
    # workgroup, groups within rows of 16 lanes)
    "3d_64_split2": ((64, 64, 64), (16 * math.pi,) * 3, None, 35, "fp64", 1),
    "3d_128x64x64_split4": ((128, 64, 64), (32 * math.pi, 16 * math.pi, 16 * math.pi), None, 36, "fp64", 2),
    # axis-0 passes in radix plan 2 (16 first): 96 threads per workgroup, one
    # whole wave and a half-full one
    "3d_96_split2_plan16": ((96, 96, 96), (24 * math.pi,) * 3, None, 37, "fp64", 1, 2),
}


def active_radius(plan, prm, psi, g, max_inner=3000):
    """Half the norm of the (nearly) unconstrained step from a run with a
    radius no step reaches."""
    so = lb.sub_opts(eta=0.1, eps_sub=1e-10, max_inner=max_inner)
    _, info, rc = plan.lb_tr_subproblem(prm, psi, g, 1e6, so)
    assert rc >= 0 and info.dnorm > 0
    return 0.5 * info.dnorm


def _run(plan, prm, psi, g, r, **kw):
    so = lb.sub_opts(eta=0.1, eps_sub=1e-10, max_inner=3000, poll_every=16, **kw)
    d, info, rc = plan.lb_tr_subproblem(prm, psi, g, r, so)
    torch.cuda.synchronize()
    return d.cpu().numpy(), {f: getattr(info, f) for f in INFO_FIELDS}, rc


@pytest.mark.parametrize("name", sorted(CASES))
def test_fused_multiplier_step_equals_separate_launch(name):
    shape, box, r, seed, prec, split, *cplan = CASES[name]
    print(f"fused Newton {name}", flush=True)
    m = O.Model(O.Grid(shape, box), 0.05, 0.25)
    psi = I.zero_mean_noise(shape, 0.3, seed)
    g = O.inv(O.gradient(m, psi))
    plan = lb.Plan(shape, box, precision=prec)
    if cplan:
        plan.lb_plan_set_column_plan(cplan[0])
    if split is not None:
        plan.lb_plan_set_plane_split(split, 0)
        assert plan.lb_plan_get_variant()[0] == split
    prm = lb.Params(m.tau, m.gamma)
    if r is None:
        r = active_radius(plan, prm, dev(psi), dev(g))
    extra = {"eps_sub_rel": 1e-6} if prec == "fp32" else {}
    d1, i1, rc1 = _run(plan, prm, dev(psi), dev(g), r, fused_newton=2, **extra)
    d0, i0, rc0 = _run(plan, prm, dev(psi), dev(g), r, fused_newton=0, **extra)
    print(f"  iters {i1['iters']} newton {i1['newton_iters']} direct {i1['newton_direct']} lambda {i1['lambda_']:.6g}")
    assert rc1 == rc0 == lb.LB_OK
    assert i1 == i0
    assert np.array_equal(d1, d0)
    assert i1["newton_iters"] > 0  # the constraint is active
    if name.endswith("_far"):
        assert i1["newton_direct"] >= 1  # the pause path ran


def test_fused_multiplier_step_at_the_iteration_cap():
    shape, box, r, seed, prec, _ = CASES["3d_32"][:6]
    m = O.Model(O.Grid(shape, box), 0.05, 0.25)
    psi = I.zero_mean_noise(shape, 0.3, seed)
    g = O.inv(O.gradient(m, psi))
    plan = lb.Plan(shape, box)
    prm = lb.Params(m.tau, m.gamma)
    for cap in (1, 7, 40):
        so1 = lb.sub_opts(eta=0.1, eps_sub=1e-10, max_inner=cap, poll_every=16, fused_newton=2)
        so0 = lb.sub_opts(eta=0.1, eps_sub=1e-10, max_inner=cap, poll_every=16, fused_newton=0)
        d1, i1, rc1 = plan.lb_tr_subproblem(prm, dev(psi), dev(g), r, so1)
        d0, i0, rc0 = plan.lb_tr_subproblem(prm, dev(psi), dev(g), r, so0)
        assert rc1 == rc0 == lb.LB_NOT_CONVERGED
        assert i1.iters == i0.iters == cap
        assert (i1.lambda_, i1.resid, i1.newton_iters) == (i0.lambda_, i0.resid, i0.newton_iters)
        assert torch.equal(d1, d0)


def test_fused_multiplier_step_on_the_128_cubed_benchmark_kernels():
    """300 iterations on the 128^3 BCC benchmark grid (520 update workgroups,
    the built-in split order): the same bits either way."""
    print("fused Newton 128^3", flush=True)
    inst = I.bcc_3d(128)
    plan = lb.Plan(inst.grid.n, inst.grid.box)
    prm = lb.Params(inst.params.tau, inst.params.gamma)
    psi = dev(inst.psi0)
    _, g = plan.lb_energy_grad(prm, psi)
    r = active_radius(plan, prm, psi, g, max_inner=300)
    outs = []
    for fused in (2, 0):
        so = lb.sub_opts(eta=0.1, eps_sub=1e-13, max_inner=300, fused_newton=fused)
        d, info, rc = plan.lb_tr_subproblem(prm, psi, g, r, so)
        outs.append((d.cpu().numpy(), {f: getattr(info, f) for f in INFO_FIELDS}, rc))
    (d1, i1, rc1), (d0, i0, rc0) = outs
    print(f"  iters {i1['iters']} newton {i1['newton_iters']} lambda {i1['lambda_']:.6g}")
    assert rc1 == rc0
    assert i1 == i0
    assert i1["newton_iters"] > 0
    assert np.array_equal(d1, d0)


def test_fused_batched_solves_with_paused_instances():
    """Batched solves of three 48 x 96 instances whose first subproblems start
    far from their multiplier (sums over the spectrum in the first steps, so
    instances pause, at different steps, and resume): the same bits with the
    fused and the separate multiplier step, and as single solves."""
    print("fused Newton batched 48x96", flush=True)
    shape, box = (48, 96), (12 * math.pi, 24 * math.pi)
    B = 3
    prms = [lb.Params(0.05 - 0.02 * k, 0.25 + 0.03 * k) for k in range(B)]
    psi0 = np.stack([I.zero_mean_noise(shape, 0.3, 40 + k) for k in range(B)])
    res = {}
    for fused in (1, 0):
        opts = lb.tr_opts(grad_norm_inf=0, eps=1e-8, max_outer=80, r0=0.2,
                          sub={"max_inner": 3000, "poll_every": 16, "fused_newton": 2 * fused})
        pb = lb.Plan(shape, box, batch=B)
        psi = dev(psi0)
        out = pb.lb_imex_tr_solve_batch(prms, psi, opts)
        res[fused] = (out, psi.cpu().numpy())
        if fused:
            single = []
            p1 = lb.Plan(shape, box)
            for k in range(B):
                x = dev(psi0[k])
                info, rc = p1.lb_imex_tr_solve(prms[k], x, opts)
                single.append((info, rc, x.cpu().numpy()))
    keys = ("energy", "gnorm", "outer", "inner_total", "cg_total", "accepted", "contracted", "newton_total",
            "newton_direct", "sub_capped")
    (o1, x1), (o0, x0) = res[1], res[0]
    direct = []
    for k in range(B):
        a = {f: getattr(o1[k][0], f) for f in keys}
        b = {f: getattr(o0[k][0], f) for f in keys}
        s = {f: getattr(single[k][0], f) for f in keys}
        assert o1[k][1] == o0[k][1] == single[k][1], k
        assert a == b == s, k
        assert np.array_equal(x1[k], x0[k]) and np.array_equal(x1[k], single[k][2]), k
        direct.append(a["newton_direct"])
    print(f"  newton_direct per instance {direct}, outer {[o1[k][0].outer for k in range(B)]}")
    assert max(direct) >= 1  # some instance paused


def test_default_fuses_the_step_only_where_it_pays():
    """fused_newton = 1 (the default) takes the step in the inverse pass while
    the redundant partial reads stay small (32^3: 9 update workgroups) and
    keeps the separate launch at 128^3 (520 workgroups: 48 MB of such reads
    per pass), with the same results as either forced form."""
    for n, expect_fused in ((32, True), (128, False)):
        inst = I.bcc_3d(n)
        plan = lb.Plan(inst.grid.n, inst.grid.box)
        prm = lb.Params(inst.params.tau, inst.params.gamma)
        psi = dev(inst.psi0)
        _, g = plan.lb_energy_grad(prm, psi)
        r = active_radius(plan, prm, psi, g, max_inner=100)
        outs = {}
        for mode in (1, 0, 2):
            so = lb.sub_opts(eta=0.1, eps_sub=1e-300, max_inner=40, fused_newton=mode)
            plan.lb_plan_set_timing(mode == 1, "")
            d, info, rc = plan.lb_tr_subproblem(prm, psi, g, r, so)
            torch.cuda.synchronize()
            if mode == 1:
                tm = plan.timings()
                plan.lb_plan_set_timing(False, "")
            outs[mode] = (d.cpu().numpy(), info.lambda_, info.iters, rc)
            if mode == 1:
                direct = info.newton_direct
        launched = tm.get("newton", (0, 0.0))[0]
        print(f"  {n}^3: separate Newton launches {launched} (steps needing full sums {direct})")
        if expect_fused:  # only steps whose series needs full sums go to the separate kernel
            assert launched <= direct < 41
        else:
            assert launched == 41  # steps 0 .. 40, one launch each
        for mode in (0, 2):
            assert np.array_equal(outs[1][0], outs[mode][0]) and outs[1][1:] == outs[mode][1:]
