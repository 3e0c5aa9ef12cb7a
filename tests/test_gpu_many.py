"""GPU: concurrent independent solves (lb_imex_tr_solve_many) give the same
results, bit for bit, as the same solves run one at a time, and the oracle's
endpoint; misuse is rejected."""
import math

import numpy as np
import pytest
import torch

from oracle import lb_oracle as O
from paper_2603_03933_amd import inputs as I
from paper_2603_03933_amd import lb

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def _jobs():
    spec = [(16, -0.15, 0.25, 1), (24, -0.2, 0.3, 2), (32, -0.1, 0.2, 3), (16, -0.25, 0.35, 4), (48, -0.15, 0.25, 5), (24, -0.3, 0.1, 6)]
    out = []
    for n, tau, gam, seed in spec:
        box = (2 * math.pi * n / 16, 2 * math.pi * n / 16)
        out.append(((n, n), box, lb.Params(tau, gam), I.zero_mean_noise((n, n), 0.2, seed)))
    return out


def test_solve_many_matches_sequential_and_oracle():
    jobs = _jobs()
    opts = lb.tr_opts(grad_norm_inf=0, eps=1e-9, max_outer=200, sub={"max_inner": 5000})
    seq = []
    for shape, box, prm, psi0 in jobs:
        plan = lb.Plan(shape, box)
        psi = torch.from_numpy(psi0).to(DEV)
        info, rc = plan.lb_imex_tr_solve(prm, psi, opts)
        seq.append((info, rc, psi.cpu().numpy()))
    plans = [lb.Plan(s, b) for s, b, _, _ in jobs]
    psis = [torch.from_numpy(p0).to(DEV) for _, _, _, p0 in jobs]
    res = lb.lb_imex_tr_solve_many(plans, [p for _, _, p, _ in jobs], psis, opts, workers=3)
    for (info, rc), (sinfo, src, spsi), psi in zip(res, seq, psis):
        assert rc == src
        assert (info.outer, info.inner_total, info.cg_total, info.accepted) == (sinfo.outer, sinfo.inner_total, sinfo.cg_total, sinfo.accepted)
        assert info.energy == sinfo.energy
        assert np.array_equal(psi.cpu().numpy(), spsi)  # same kernels, same order: identical bits
    # one endpoint against the oracle
    shape, box, prm, psi0 = jobs[0]
    m = O.Model(O.Grid(shape, box), prm.tau, prm.gamma)
    ref = O.imex_tr_solve(m, psi0, O.TROpts(grad_norm="l2", eps=1e-9, max_outer=200, max_inner=5000))
    assert res[0][1] == lb.LB_OK and ref.converged
    assert abs(res[0][0].energy - ref.energy) < 1e-10 * max(1.0, abs(ref.energy))


def test_solve_many_rejects_shared_plan_and_batched_plans():
    shape, box, prm, psi0 = _jobs()[0]
    plan = lb.Plan(shape, box)
    psis = [torch.from_numpy(psi0).to(DEV) for _ in range(2)]
    with pytest.raises(lb.LBError):
        lb.lb_imex_tr_solve_many([plan, plan], [prm, prm], psis)
    bplan = lb.Plan(shape, box, batch=2)
    with pytest.raises(lb.LBError):
        lb.lb_imex_tr_solve_many([bplan], [prm], [torch.zeros(psi0.size, dtype=torch.float64, device=DEV)])
