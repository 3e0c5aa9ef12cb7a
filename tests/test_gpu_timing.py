"""Kernel timing (lb_plan_set_timing / lb_plan_timing_entry), which bench.py's
roofline figure rests on: every launch of a timed kernel is counted once,
whether its events are read during the subproblem loop or afterwards, and
timing does not change results."""
import math

import numpy as np
import pytest
import torch

from paper_2603_03933_amd import inputs as I
from paper_2603_03933_amd import lb

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

SHAPE, BOX = (32, 32, 32), (4 * math.sqrt(2) * math.pi,) * 3


def _subproblem(plan, psi, g, max_inner, poll_every, fused=0):
    # eps_sub far below rounding: the subproblem runs to max_inner, launching
    # steps 0 .. max_inner (one per plane pass) with the separate Newton
    # kernel; with the multiplier step in the inverse pass, steps 0 ..
    # max_inner + 1 (the last one's inverse pass takes the step that stops)
    so = lb.sub_opts(eta=0.1, eps_sub=1e-300, max_inner=max_inner, poll_every=poll_every, fused_newton=fused)
    d, info, rc = plan.lb_tr_subproblem(lb.Params(-0.2, 0.3), psi, g, 0.5, so)
    torch.cuda.synchronize()
    return d.detach().cpu().numpy(), info, rc


@pytest.mark.parametrize("fused", [0, 2])
@pytest.mark.parametrize("poll_every", [1, 7, 32, 200])
def test_every_timed_launch_is_counted_once(poll_every, fused):
    plan = lb.Plan(SHAPE, BOX)
    psi = torch.from_numpy(I.zero_mean_noise(SHAPE, 0.3, 3)).to(DEV)
    _, g = plan.lb_energy_grad(lb.Params(-0.2, 0.3), psi)
    max_inner = 100
    d_off, info_off, rc_off = _subproblem(plan, psi, g, max_inner, poll_every, fused)
    assert rc_off == lb.LB_NOT_CONVERGED and info_off.iters == max_inner

    plan.lb_plan_set_timing(True, "")  # every kernel
    d_all, info_all, _ = _subproblem(plan, psi, g, max_inner, poll_every, fused)
    tm = plan.timings()
    plan.lb_plan_set_timing(True, "plane_inner")  # only the dominant pass, as bench.py's timed steps
    d_one, info_one, _ = _subproblem(plan, psi, g, max_inner, poll_every, fused)
    tm_one = plan.timings()
    plan.lb_plan_set_timing(False, "")

    steps = max_inner + (2 if fused else 1)
    # fused: the separate kernel runs only for a step whose series needs full
    # sums (none in this case), which would also re-launch the steps after it
    assert not fused or ("newton" not in tm and info_all.newton_direct == 0)
    for k in ("col0_inv_scale_d", "plane_inner", "col0_fwd_update") + (() if fused else ("newton",)):
        count, ms = tm[k]
        assert count == steps and ms > 0.0, (k, count, ms)
    assert set(tm_one) == {"plane_inner"}
    count, ms = tm_one["plane_inner"]
    assert count == steps and 0.0 < ms < 1e3
    # timing changes nothing the kernels compute
    assert np.array_equal(d_all, d_off) and np.array_equal(d_one, d_off)
    assert info_all.lambda_ == info_off.lambda_ == info_one.lambda_
