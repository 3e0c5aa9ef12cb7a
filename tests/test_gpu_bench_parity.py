"""GPU parity at the benchmarked 128^3 BCC workload (the kernels and launch
shapes the benchmark times: the 1024-thread plane pass, 520 column workgroups
per axis-0 pass, the Newton kernel with its series and full-sum forms), the
endpoint of the 128^3 solves checked by the oracle, and the endpoint of a
solve whose inner iterations run in FP32 (with the relative stop floor)
against the oracle's FP64 solve with the same floor."""
import functools
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import lb_oracle as O
from paper_2603_03933_amd import inputs as I
from paper_2603_03933_amd import lb

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def rms(a):
    return math.sqrt(float(np.mean(a * a)))


@functools.lru_cache(maxsize=1)
def _bcc128():
    inst = I.bcc_3d(128)
    m = O.Model(O.Grid(inst.grid.n, inst.grid.box), inst.params.tau, inst.params.gamma)
    g_hat = O.gradient(m, inst.psi0)
    # the step size rule of the benchmark's first outer iteration: min(0.1, 0.9 / max |Gamma'|)
    eta = min(0.1, 0.9 / float(np.max(np.abs(O.Gamma_p(inst.psi0, m.tau, m.gamma)))))
    return inst, m, g_hat, eta


@functools.lru_cache(maxsize=4)
def _oracle_iterations(r, k):
    inst, m, g_hat, eta = _bcc128()
    return O.imex_subproblem(m, inst.psi0, g_hat, r, O.SubOpts(eta=eta, eps_sub=0.0, max_inner=k))


@pytest.mark.parametrize("r,direct", [(0.1, 0), (0.1, 1), (1.0, 0)])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("split", [0, 1])
def test_bcc128_subproblem_iterations_match_oracle(r, direct, precision, tol, split):
    """Five iterations of Algorithm 3 at the 128^3 BCC input through the
    benchmark's kernels, element by element against the oracle's five. With
    r = 0.1 the constraint is active (lambda > 0): the Newton kernel's series
    form (direct = 0, the benchmark's) and its full spectral sums (direct = 1)
    are both checked; with r = 1 the iterates stay interior (lambda = 0).
    Both orders of the inner iteration the benchmark's autotuner chooses from:
    one 1024-thread workgroup per plane, and the pair-split order with its
    half-plane pass (built-in thread count)."""
    inst, m, g_hat, eta = _bcc128()
    print(f"bcc 128^3 subproblem r={r} direct={direct} {precision} split={split}", flush=True)
    ref = _oracle_iterations(r, 5)
    plan = lb.Plan(inst.grid.n, inst.grid.box, precision=precision)
    if split:
        plan.lb_plan_set_plane_split(1, 0)
    else:
        plan.lb_plan_set_plane_threads(1024)
    d, info, rc = plan.lb_tr_subproblem(lb.Params(m.tau, m.gamma), dev(inst.psi0), dev(O.inv(g_hat)), r,
                                        lb.sub_opts(eta=eta, eps_sub=0.0, max_inner=5, newton_direct=direct))
    d = host(d)
    d_or = O.inv(ref.d)
    print(f"  lambda {info.lambda_:.15e} (oracle {ref.lam:.15e}), newton {info.newton_iters}, "
          f"full sums {info.newton_direct}, iterate error {rms(d - d_or) / rms(d_or):.2e}")
    assert info.iters == ref.iters == 5 and rc == lb.LB_NOT_CONVERGED
    assert abs(info.lambda_ - ref.lam) <= tol * max(1.0, ref.lam)
    assert rms(d - d_or) <= tol * rms(d_or)
    if r == 0.1:
        assert ref.lam > 0 and info.newton_iters > 0
        if direct:
            assert info.newton_direct >= info.newton_iters  # every evaluation summed over the spectrum
        assert abs(info.dnorm - r) <= 1e-12 * r
    else:
        assert ref.lam == 0.0 and info.lambda_ == 0.0 and info.dnorm < r


@functools.lru_cache(maxsize=1)
def _solve128(precision):
    inst = I.bcc_3d(128)
    plan = lb.Plan(inst.grid.n, inst.grid.box, precision=precision)
    prm = lb.Params(inst.params.tau, inst.params.gamma)
    psi = dev(inst.psi0)
    sub = {"max_inner": 10000, "poll_every": 64}
    if precision == "fp32":
        sub["eps_sub_rel"] = 1e-5
    info, rc = plan.lb_imex_tr_solve(prm, psi, lb.tr_opts(grad_norm_inf=0, eps=1e-8, max_outer=500, sub=sub))
    return inst, info, rc, host(psi)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bcc128_solve_endpoint_checked_by_the_oracle(precision):
    """The benchmark's 128^3 solve (FP64, and FP32 inner iterations with the
    1e-5 relative floor): at the returned field the oracle's gradient norm is
    below the 1e-8 target, the oracle's energy equals the reported one, and
    the oracle's preconditioned Lanczos estimate of sigma_1 is >= -1e-8."""
    print(f"bcc 128^3 solve, inner iterations in {precision}", flush=True)
    inst, info, rc, psi = _solve128(precision)
    m = O.Model(O.Grid(inst.grid.n, inst.grid.box), inst.params.tau, inst.params.gamma)
    print(f"  outer {info.outer}, inner {info.inner_total}, subproblems stopped at the cap {info.sub_capped}")
    assert rc == lb.LB_OK and 0 <= info.sub_capped <= info.outer
    g = O.gradient(m, psi)
    gn = O.norm(g)
    E = O.energy(m, psi)
    print(f"  E {info.energy:.15e} (oracle {E:.15e}), |g| {info.gnorm:.3e} (oracle {gn:.3e})")
    assert gn < 1e-8 and abs(gn - info.gnorm) <= 1e-12 * (O.norm(m.Lam * O.fwd(psi)) + rms(O.dF_bulk(psi, m.tau, m.gamma)))
    assert abs(E - info.energy) <= 1e-12 * abs(E)
    ritz, res = O.lanczos_min(m, psi, O.fwd(I.hessvec_direction(inst.grid.n, 9)), 12, precond_shift=1.0)
    print(f"  oracle preconditioned Lanczos (12 steps): {ritz:.3e} (residual {res:.2e})")
    assert ritz >= -1e-8


def test_bcc128_fp32_and_fp64_solves_reach_the_same_state():
    _, i64, rc64, p64 = _solve128("fp64")
    _, i32, rc32, p32 = _solve128("fp32")
    assert rc64 == rc32 == lb.LB_OK
    assert abs(i32.energy - i64.energy) <= 1e-10 * abs(i64.energy)
    pw = lambda p: np.sort(np.abs(np.fft.rfftn(p) / p.size).ravel() ** 2)[-64:]
    assert np.max(np.abs(pw(p32) - pw(p64))) <= 1e-7 * np.max(pw(p64))


def test_fp32_inner_solve_endpoint_matches_the_oracle():
    """The FP32-inner solve (FP32 transforms and pointwise stages, FP64
    reductions, multiplier and ratio; stop floor 1e-5 ||g||) on the 32^3 BCC
    workload, a cubic grid that takes the plane pass, against the oracle's FP64
    solve with the same stop rule (tests/golden/bcc_32_relfloor_oracle.json,
    written by make_bcc_32_relfloor.py from the oracle alone): the oracle's
    gradient norm at the returned field is below 1e-8, the energy matches the
    oracle's endpoint, the power spectrum too (the state is the same up to a
    translation), and the oracle's preconditioned Lanczos estimate is >= -1e-8."""
    gold = json.load(open(os.path.join(GOLDEN, "bcc_32_relfloor_oracle.json")))
    inst = I.bcc_3d(32)
    m = O.Model(O.Grid(inst.grid.n, inst.grid.box), inst.params.tau, inst.params.gamma)
    plan = lb.Plan(inst.grid.n, inst.grid.box, precision="fp32")
    psi = dev(inst.psi0)
    info, rc = plan.lb_imex_tr_solve(lb.Params(m.tau, m.gamma), psi, lb.tr_opts(
        grad_norm_inf=0, eps=1e-8, sub={"max_inner": 10000, "eps_sub_rel": 1e-5}))
    out = host(psi)
    print(f"32^3 FP32-inner: E {info.energy:.15e} (oracle {gold['energy']:.15e}), outer {info.outer} "
          f"(oracle {gold['outer']}), inner {info.inner_total} (oracle {gold['inner_total']})")
    print(f"  subproblems stopped at the cap: {info.sub_capped} (oracle {gold['sub_capped']})")
    assert rc == lb.LB_OK and 0 <= info.sub_capped <= info.outer
    assert O.norm(O.gradient(m, out)) < 1e-8
    assert abs(info.energy - gold["energy"]) <= 1e-10 * abs(gold["energy"])
    assert abs(O.energy(m, out) - gold["energy"]) <= 1e-10 * abs(gold["energy"])
    power = np.abs(np.fft.fftn(out) / out.size) ** 2
    for i, pw in gold["top_power"]:
        assert abs(power.ravel()[i] - pw) <= 1e-6 * gold["top_power"][0][1], i
    ritz, _ = O.lanczos_min(m, out, O.fwd(I.hessvec_direction(inst.grid.n, 5)), 60, precond_shift=1.0)
    assert ritz >= -1e-8 and gold["lanczos60_precond_ritz"] >= -1e-8
