"""GPU: the random feasible initial point (Philox4x64-10 + Box-Muller, uniform
in the zero-mean ball), the Lanczos Ritz vector, and the hard-case strategy of
the outer loop on the paper's Section 4.3 experiment, against the oracle."""
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


@pytest.mark.parametrize("shape", [(8, 8, 8), (16, 24), (32, 32, 32)])
@pytest.mark.parametrize("seed,draw", [(0, 0), (1, 5), (2**40 + 3, 2**33 + 1)])
def test_random_ball_matches_oracle(shape, seed, draw):
    plan = lb.Plan(shape, tuple(float(n) for n in shape))
    r = 0.37
    d = host(plan.lb_random_ball(r, seed, draw))
    ref = O.ball_point(shape, r, seed, draw)
    # normals pass through log and cos: a few ulps apart between the two math libraries
    assert np.max(np.abs(d - ref)) < 1e-13 * np.max(np.abs(ref))
    assert abs(d.mean()) < 1e-15 and math.sqrt(np.mean(d * d)) <= r * (1 + 1e-14)


@pytest.mark.parametrize("precond", [0.0, 1.0])
def test_lanczos_ritz_vector_matches_oracle(precond):
    shape, box = (16, 16), (2 * math.pi, 2 * math.pi)
    m = O.Model(O.Grid(shape, box), -0.15, 0.25)
    psi = I.zero_mean_noise(shape, 0.3, 61)
    v0 = O.ball_point(shape, 1.0, 3, 1)
    plan = lb.Plan(shape, box)
    evec = torch.empty(shape, dtype=torch.float64, device=DEV)
    rho, res = plan.lb_lanczos_min(lb.Params(m.tau, m.gamma), dev(psi), dev(v0), 40, precond_shift=precond, evec=evec)
    rho_or, res_or, xi = O.lanczos_min(m, psi, O.fwd(v0), 40, precond, want_vector=True)
    x = host(evec)
    assert abs(rho - rho_or) < 1e-10 * max(1.0, abs(rho_or))
    assert abs(math.sqrt(np.mean(x * x)) - 1.0) < 1e-12 and abs(x.mean()) < 1e-14
    assert abs(abs(np.mean(x * O.inv(xi))) - 1.0) < 1e-8  # same unit vector up to sign


def _lam_start(M):
    L = 2 * math.sqrt(2) * math.pi
    x = np.arange(M) * L / M
    return (L, L, L), 0.6 * np.cos(x[:, None, None] / math.sqrt(2)) + np.zeros((M, M, M))


def test_hard_case_strategy_section_4_3():
    """Section 4.3 on the GPU: deterministic start -> negative curvature left;
    random feasible start in the nearly hard subproblems -> HEX at the printed
    energy, nonnegative Hessian spectrum (dense, on the oracle, at the GPU's
    final state); the first hard-case decisions agree with the oracle's."""
    gold = json.load(open(os.path.join(GOLDEN, "paper_energies.json")))["hard_case_experiment"]
    M = 8
    box, psi0 = _lam_start(M)
    m = O.Model(O.Grid((M, M, M), box), gold["tau"], gold["gamma"])
    plan = lb.Plan((M, M, M), box)
    prm = lb.Params(gold["tau"], gold["gamma"])
    base = dict(eps=1e-10, max_outer=400, sub={"max_inner": 20000})
    psi = dev(psi0 - psi0.mean())
    info, rc = plan.lb_imex_tr_solve(prm, psi, lb.tr_opts(**base))
    assert rc == lb.LB_OK and info.hard_cases == 0
    assert O.hessian_eigs(m, host(psi))[0] < -1e-3
    psi = dev(psi0 - psi0.mean())
    info, rc = plan.lb_imex_tr_solve(prm, psi, lb.tr_opts(hard_case=1, seed=1, hard_tol=gold["hard_tol"], **base))
    assert rc == lb.LB_OK and info.hard_cases >= 1
    assert abs(info.energy - gold["randomized_energy"]) <= 0.5e-4
    assert O.hessian_eigs(m, host(psi))[0] >= -1e-8
    # the oracle with the same rule flags the same first subproblems
    log = []
    prov = O.hard_case_d0_provider(m, seed=1, tol=gold["hard_tol"], log=log)
    O.imex_tr_solve(m, psi0, O.TROpts(eps=1e-10, max_outer=3, max_inner=20000), d0_provider=prov)
    assert [e["hard"] for e in log] == [True, True, True][: len(log)]
