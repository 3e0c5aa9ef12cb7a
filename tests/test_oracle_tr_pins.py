"""Pins of the oracle's outer loop (Algorithm 1) and of CONTRACT (Algorithm 2).

The scalar bookkeeping of Algorithm 1 (radius r, bound nu, multiplier bound
mu) is driven with scripted subproblem results and ratios; the expected
values are worked out by hand from the algorithm's lines and written here as
numbers, chosen so that a plausible misreading (min and max exchanged, the
accept test without its nu alternative, mu updated in the wrong branch) gives
a different number. CONTRACT is checked on a small dense problem against
shifted systems solved with numpy.linalg.solve, with the cases chosen so that
lambda_hat without its square root, gamma_C applied to the old step, or the
wrong branch would each fail.
"""
import math

import numpy as np
import pytest

from oracle import lb_oracle as O
from paper_2603_03933_amd import inputs as I


# ---------------------------------------------------------------------------
# Algorithm 1: branch and radius updates on scripted values
# ---------------------------------------------------------------------------

OPTS = O.TROpts()  # theta 1e-4, gamma_E 2, gamma_C 0.5, gamma_lambda 1.5, mu_lo 1, mu_hi 1e5


def _no_contract():
    raise AssertionError("CONTRACT must not be called in this branch")


@pytest.mark.parametrize(
    "rho,lam,sn,r,nu,mu,expect",
    [
        # accept on the boundary: nu = max(5, 2) = 5, r = min(5, max(1, 2)) = 2, mu = max(1, 0.3) = 1
        (0.5, 0.3, 1.0, 1.0, 5.0, 1.0, ("accept", 2.0, 5.0, 1.0)),
        # accept, step larger than nu/2: nu = max(5, 6) = 6, r = min(6, max(3, 6)) = 6
        (0.5, 0.3, 3.0, 3.0, 5.0, 1.0, ("accept", 6.0, 6.0, 1.0)),
        # accept, r kept: gamma_E s = 3 < r = 4 -> r = min(5, max(4, 3)) = 4 (exchanging min
        # and max gives max(5, min(4, 3)) = 5)
        (0.5, 0.3, 1.5, 4.0, 5.0, 1.0, ("accept", 4.0, 5.0, 1.0)),
        # accept raises mu: lambda / ||s|| = 2.5 / 0.5 = 5 <= mu = 6 -> mu = max(6, 5) = 6
        (0.2, 2.5, 0.5, 0.5, 5.0, 6.0, ("accept", 1.0, 5.0, 6.0)),
        # accept with lambda / ||s|| = 8 > mu = 2 but ||s|| = nu = 5: accepted through the nu
        # alternative; nu = max(5, 10) = 10, r = min(10, max(5, 10)) = 10, mu = max(2, 8) = 8
        (0.01, 40.0, 5.0, 5.0, 5.0, 2.0, ("accept", 10.0, 10.0, 8.0)),
        # the ratio is exactly theta: accepted (rho >= theta)
        (1e-4, 0.0, 0.25, 0.25, 5.0, 1.0, ("accept", 0.5, 5.0, 1.0)),
        # expand: rho >= theta, lambda / ||s|| = 4 > mu = 1, ||s|| < nu -> r = min(5, 2 / 1) = 2
        (0.3, 2.0, 0.5, 0.5, 5.0, 1.0, ("expand", 2.0, 5.0, 1.0)),
        # expand capped by nu: r = min(5, 30 / 2) = 5, mu unchanged
        (0.3, 30.0, 1.0, 1.0, 5.0, 2.0, ("expand", 5.0, 5.0, 2.0)),
    ],
)
def test_outer_branch_scripted(rho, lam, sn, r, nu, mu, expect):
    got = O.outer_branch(OPTS, rho, lam, sn, r, nu, mu, _no_contract)
    assert got[0] == expect[0]
    assert got[1:] == pytest.approx(expect[1:], rel=0, abs=1e-15)


def test_outer_branch_contract_keeps_nu_and_mu():
    calls = []

    def contract():
        calls.append(1)
        return 0.125

    # rho < theta: CONTRACT decides the radius, nu and mu are carried over
    assert O.outer_branch(OPTS, -0.7, 0.4, 1.0, 1.0, 5.0, 3.0, contract) == ("contract", 0.125, 5.0, 3.0)
    assert O.outer_branch(OPTS, 0.99e-4, 0.0, 1.0, 1.0, 5.0, 3.0, contract) == ("contract", 0.125, 5.0, 3.0)
    assert len(calls) == 2


@pytest.mark.parametrize(
    "j,rho_prev,mu,lam,sn,expect",
    [
        (0, None, 1.0, 6.0, 2.0, 1.0),  # first iteration: no update
        (3, 0.5, 1.0, 6.0, 2.0, 1.0),  # previous step accepted with rho >= theta: no update
        (3, 1e-5, 1.0, 6.0, 2.0, 3.0),  # after a rejection: max(1, 6 / 2) = 3
        (3, -2.0, 4.0, 6.0, 2.0, 4.0),  # ... but never below mu_{j-1}: max(4, 3) = 4
    ],
)
def test_mu_update_after_a_rejected_step(j, rho_prev, mu, lam, sn, expect):
    assert O.mu_before_ratio(OPTS, j, rho_prev, mu, lam, sn) == expect


def test_imex_tr_solve_follows_the_scripted_branches(monkeypatch):
    """The oracle's outer loop driven with scripted subproblem results
    (lambda_j, ||s_j||) and ratios rho_j, CONTRACT returning scripted radii:
    the radius, nu and mu sequence and the accepted iterates are those worked
    out by hand from Algorithm 1."""
    n, box = (4, 4), (2 * math.pi, 2 * math.pi)
    m = O.Model(O.Grid(n, box), -0.2, 0.3)
    psi0 = I.zero_mean_noise(n, 0.2, 3)
    direction = O.project(O.fwd(I.zero_mean_noise(n, 1.0, 4)))
    direction = direction / O.norm(direction)
    # j: (lambda_j, ||s_j||, rho_j); radius returned by CONTRACT where it is called
    script = [
        (0.2, 1.0, 0.5),  # accept: nu 5, r min(5, max(1, 2)) = 2, mu max(1, 0.2) = 1
        (0.0, 2.0, 1e-6),  # contract -> 0.7 (mu: j > 0 but rho_0 >= theta, stays 1)
        (1.4, 0.7, 0.3),  # mu = max(1, 1.4 / 0.7) = 2 (rho_1 < theta); 1.4 / 0.7 = 2 <= 2: accept,
        #                  nu max(5, 1.4) = 5, r min(5, max(0.7, 1.4)) = 1.4, mu max(2, 2) = 2
        (6.0, 1.4, 0.3),  # 6 / 1.4 > mu = 2, ||s|| != nu: expand, r = min(5, 6 / 2) = 3
        (9.0, 3.0, -1.0),  # contract -> 0.9
        (1.0, 0.9, 0.4),  # mu = max(2, 1 / 0.9) = 2; accept: nu 5, r = min(5, max(0.9, 1.8)) = 1.8
    ]
    expect_after = [
        ("accept", 2.0, 5.0, 1.0),
        ("contract", 0.7, 5.0, 1.0),
        ("accept", 1.4, 5.0, 2.0),
        ("expand", 3.0, 5.0, 2.0),
        ("contract", 0.9, 5.0, 2.0),
        ("accept", 1.8, 5.0, 2.0),
    ]
    contract_radii = iter([0.7, 0.9])
    contract_args = []
    state = {"j": 0}

    def fake_sub(m_, psi, g_hat, r, opts, d0=None, record=False):
        lam, sn, _ = script[state["j"]]
        return O.SubResult(direction * sn, lam, 1, 0, 0.0, True)

    def fake_delta(m_, psi, g_hat, s_hat):
        _, sn, rho = script[state["j"]]
        state["j"] += 1
        return rho * sn**3

    def fake_contract(m_, psi, g_hat, r, mu, s_hat, lam, o):
        contract_args.append((r, mu, O.norm(s_hat), lam))
        return next(contract_radii), {}

    monkeypatch.setattr(O, "imex_subproblem", fake_sub)
    monkeypatch.setattr(O, "delta_energy_taylor", fake_delta)
    monkeypatch.setattr(O, "contract", fake_contract)
    res = O.imex_tr_solve(m, psi0, O.TROpts(grad_norm="l2", eps=1e-30, max_outer=len(script)))
    hist = res.history
    assert [h["branch"] for h in hist] == [e[0] for e in expect_after]
    # the radius used at iteration j + 1 is r_{j+1}
    for j in range(len(script) - 1):
        assert hist[j + 1]["r"] == pytest.approx(expect_after[j][1], abs=1e-14), j
        assert hist[j + 1]["nu"] == pytest.approx(expect_after[j][2], abs=1e-14), j
    # mu as used in the ratio test of iteration j (after the update that follows a rejection)
    assert [h["mu"] for h in hist] == pytest.approx([1.0, 1.0, 2.0, 2.0, 2.0, 2.0], abs=1e-14)
    # CONTRACT receives r_j, mu_j, s_j and lambda_j of its iteration
    assert contract_args == [pytest.approx((2.0, 1.0, 2.0, 0.0)), pytest.approx((3.0, 2.0, 3.0, 9.0))]
    # three accepted steps along `direction` of lengths 1, 0.7 and 0.9
    moved = O.inv(direction) * (1.0 + 0.7 + 0.9)
    assert np.max(np.abs(res.psi - (psi0 - psi0.mean()) - moved)) < 1e-13


# ---------------------------------------------------------------------------
# Algorithm 2 (CONTRACT) against dense shifted solves
# ---------------------------------------------------------------------------


def _dense_problem(tau=0.15, seed=7):
    n, box = (4, 4), (2 * math.pi, 2 * math.pi)
    m = O.Model(O.Grid(n, box), tau, 0.3)
    psi = I.zero_mean_noise(n, 0.4, seed)
    g_hat = O.gradient(m, psi)
    Hs, Q = O.dense_hessian(m, psi)
    gs = Q.T @ O.inv(g_hat).reshape(-1) / math.sqrt(m.grid.N)
    return m, psi, g_hat, Hs, gs


def _snorm(Hs, gs, lam):
    """||s|| for (H + lam I) s = -g, dense (the RMS norm is the 2-norm in this basis)."""
    return float(np.linalg.norm(np.linalg.solve(Hs + lam * np.eye(len(gs)), -gs)))


def _step(m, sn):
    # a step of norm sn (its direction is not used by CONTRACT, only its length)
    s = np.zeros(m.grid.n, dtype=complex)
    s[1, 0] = s[-1, 0] = sn / math.sqrt(2)
    return s


def test_contract_lambda_hat_branch():
    """lambda_j < mu_lo ||s_j||: lambda_hat = lambda_j + (mu_lo ||g_j||)^(1/2) and, when
    lambda_hat / ||s(lambda_hat)|| <= mu_hi, r_{j+1} = ||s(lambda_hat)||."""
    m, psi, g_hat, Hs, gs = _dense_problem()
    assert np.linalg.eigvalsh(Hs)[0] > 0
    gn = O.norm(g_hat)
    assert abs(gn - np.linalg.norm(gs)) < 1e-12 * gn
    lam, sn, mu_lo = 0.05, 1.0, 2.0
    o = O.TROpts(mu_lo=mu_lo, mu0=mu_lo)
    expect = _snorm(Hs, gs, lam + math.sqrt(mu_lo * gn))
    r, info = O.contract(m, psi, g_hat, 1.0, mu_lo, _step(m, sn), lam, o)
    assert info["contract_branch"] == "hat"
    assert abs(r - expect) < 1e-10 * expect
    # the pin tells the printed square root from its plausible misreadings
    for wrong in (lam + mu_lo * gn, lam + math.sqrt(gn), math.sqrt(mu_lo * gn)):
        assert abs(_snorm(Hs, gs, wrong) - expect) > 1e-3 * expect


def test_contract_bisection_branch():
    """lambda_hat / ||s(lambda_hat)|| > mu_hi: the returned radius is ||s(lambda~)|| for
    some lambda~ in (lambda_j, lambda_hat) with mu_lo <= lambda~ / ||s(lambda~)|| <= mu_hi."""
    m, psi, g_hat, Hs, gs = _dense_problem()
    gn = O.norm(g_hat)
    lam, sn = 0.02, 1.0
    lam_hat = lam + math.sqrt(gn)
    ratio_hat = lam_hat / _snorm(Hs, gs, lam_hat)
    o = O.TROpts(mu_lo=1.0, mu_hi=0.5 * ratio_hat)
    assert ratio_hat > o.mu_hi and lam / _snorm(Hs, gs, lam) < o.mu_lo  # the search interval brackets [mu_lo, mu_hi]
    r, info = O.contract(m, psi, g_hat, 1.0, 1.0, _step(m, sn), lam, o)
    assert info["contract_branch"] == "bisect"
    lt = info["lam_tilde"]
    assert lam < lt < lam_hat
    rd = _snorm(Hs, gs, lt)
    assert abs(r - rd) < 1e-10 * rd
    assert o.mu_lo <= lt / rd <= o.mu_hi


@pytest.mark.parametrize("else_old_step", [False, True])
def test_contract_gamma_lambda_branch(else_old_step):
    """lambda_j >= mu_lo ||s_j||: lambda~ = gamma_lambda lambda_j; r = ||s|| when
    ||s|| >= gamma_C ||s_j||, else gamma_C ||s|| (the new s, as printed; the
    option reads it as gamma_C ||s_j||)."""
    m, psi, g_hat, Hs, gs = _dense_problem()
    o = O.TROpts(contract_else_old_step=else_old_step)
    # if-branch: a small old step, ||s(1.5 lambda)|| >= 0.5 ||s_j||
    lam, sn = 0.3, 0.3
    s_new = _snorm(Hs, gs, 1.5 * lam)
    assert s_new >= 0.5 * sn and lam >= sn
    r, info = O.contract(m, psi, g_hat, 1.0, 1.0, _step(m, sn), lam, o)
    assert info["contract_branch"] == "gamma_lambda"
    assert abs(r - s_new) < 1e-10 * s_new
    # else-branch: a long old step, ||s(1.5 lambda)|| < 0.5 ||s_j||
    lam, sn = 3.0, 2.5
    s_new = _snorm(Hs, gs, 1.5 * lam)
    assert s_new < 0.5 * sn and lam >= sn
    r, _ = O.contract(m, psi, g_hat, 1.0, 1.0, _step(m, sn), lam, o)
    expect = 0.5 * sn if else_old_step else 0.5 * s_new
    assert abs(r - expect) < 1e-10 * expect
    # the pin tells gamma_lambda from gamma_E (2) and the two else-branch readings apart
    assert abs(_snorm(Hs, gs, 2.0 * lam) - s_new) > 1e-3 * s_new
    assert abs(0.5 * sn - 0.5 * s_new) > 1e-3 * s_new
