"""GPU: the raw-coordinate derivatives of the library against the oracle, and
the torch.autograd wrapper against finite differences (gradcheck, gradgradcheck,
and exact central differences of the quartic energy on the 8-instance
differentiation batch)."""
import math

import numpy as np
import pytest
import torch

from oracle import lb_oracle as O
from paper_2603_03933_amd import autograd as A
from paper_2603_03933_amd import inputs as I
from paper_2603_03933_amd import lb

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize(
    "shape,box",
    [((16, 24), (2 * math.pi, 3 * math.pi)), ((32, 32, 32), (4 * math.sqrt(2) * math.pi,) * 3), ((8, 12, 16), (2.0, 3.0, 4.0))],
)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_raw_gradient_hessvec_moments_match_oracle(shape, box, precision, tol):
    m = O.Model(O.Grid(shape, box), -0.2, 0.3, 1.1, 0.9)
    psi = I.zero_mean_noise(shape, 0.3, 41) + 0.25  # nonzero mean: the k = 0 terms count
    v = I.zero_mean_noise(shape, 1.0, 42) - 0.5
    plan = lb.Plan(shape, box, precision=precision)
    prm = lb.Params(m.tau, m.gamma, m.xi, m.q)
    E, g = plan.lb_energy_grad_raw(prm, dev(psi))
    hv = plan.lb_hessvec_raw(prm, dev(psi), dev(v))
    mom = plan.lb_field_moments(dev(psi), dev(v))
    torch.cuda.synchronize()
    N = psi.size
    assert abs(host(E)[0] - O.energy(m, psi)) < 1e-12 * max(1.0, abs(O.energy(m, psi)))
    g_or = O.gradient_raw(m, psi)
    assert np.max(np.abs(host(g) - g_or)) < 1e-12 * np.max(np.abs(g_or))  # the gradient is always FP64
    h_or = O.hessvec_raw(m, psi, v)
    scale = (np.max(np.abs(O.inv(m.Lam * O.fwd(v)))) + np.max(np.abs(O.Gamma_p(psi, m.tau, m.gamma) * v))) / N
    assert np.max(np.abs(host(hv) - h_or)) < tol * scale
    assert np.allclose(host(mom), O.field_moments(psi, v), rtol=1e-13, atol=1e-15)
    pg = plan.lb_param_grad(dev(psi), dev(v))
    assert np.allclose(host(pg), O.param_grad(psi, v), rtol=1e-13, atol=1e-15)
    ct = dev(np.array([0.7, -1.9]))
    vjp = plan.lb_param_grad_vjp(dev(psi), ct)
    ref = O.param_grad_vjp(psi, 0.7, -1.9)
    assert np.max(np.abs(host(vjp) - ref)) < 1e-15 * np.max(np.abs(ref)) * 4


def test_autograd_gradcheck_and_gradgradcheck():
    shape, box = (8, 8), (2 * math.pi, 2 * math.pi)
    plan = lb.Plan(shape, box, batch=2)
    psi = dev(np.stack([I.zero_mean_noise(shape, 0.4, 43) + 0.1, I.zero_mean_noise(shape, 0.4, 44)])).requires_grad_(True)
    tau = torch.tensor([-0.2, -0.1], dtype=torch.float64, requires_grad=True)
    gam = torch.tensor([0.3, 0.25], dtype=torch.float64, requires_grad=True)

    def f(p, t, g):
        return A.energy(plan, p, t, g)

    assert torch.autograd.gradcheck(f, (psi, tau, gam), eps=1e-6, atol=1e-8, rtol=1e-6)
    assert torch.autograd.gradgradcheck(f, (psi, tau, gam), eps=1e-6, atol=1e-8, rtol=1e-6)


@pytest.mark.parametrize("n,eps,tol", [(24, 1e-3, 1e-9), (96, 1e-6, 1e-7)])
def test_autograd_exact_central_differences_on_the_differentiation_batch(n, eps, tol):
    """8 instances of n^3 ((tau, gamma) per instance; 96^3 is the full
    differentiation workload): the central difference of the quartic E along a
    direction e equals <dE/dpsi, e> + eps^2/6 sum (psi - gamma) e^3 / N, and the
    same for the gradient with the Hessian; tau and gamma enter affinely. At
    eps = 1e-6 rounding (~ u |E| / eps) sets the tolerance, not the identity."""
    print(f"differentiation batch 8 x {n}^3, eps {eps}", flush=True)
    insts = I.diff_3d(n)
    shape, box = insts[0].grid.n, insts[0].grid.box
    B = len(insts)
    plan = lb.Plan(shape, box, batch=B)
    psi = dev(np.stack([i.psi0 for i in insts])).requires_grad_(True)
    tau = torch.tensor([i.params.tau for i in insts], dtype=torch.float64, requires_grad=True)
    gam = torch.tensor([i.params.gamma for i in insts], dtype=torch.float64, requires_grad=True)
    e = dev(np.stack([I.hessvec_direction(shape, 50 + k) for k in range(B)]))
    E = A.energy(plan, psi, tau, gam)
    (gpsi,) = torch.autograd.grad(E.sum(), psi, create_graph=True)
    hv = torch.autograd.grad((gpsi * e).sum(), psi)[0]
    gt, gg = torch.autograd.grad(A.energy(plan, psi, tau, gam).sum(), (tau, gam))
    N = math.prod(shape)
    with torch.no_grad():
        Ep = A.energy(plan, psi + eps * e, tau, gam)
        Em = A.energy(plan, psi - eps * e, tau, gam)
        fd = host((Ep - Em) / (2 * eps))
        cub = host(((psi - gam.to(DEV).reshape(B, 1, 1, 1)) * e**3).sum(dim=(1, 2, 3))) / N
        lin = host((gpsi * e).sum(dim=(1, 2, 3)))
        assert np.max(np.abs(fd - (lin + eps**2 / 6 * cub))) < tol * np.max(np.abs(lin))
        gp = host(torch.autograd.functional.vjp(lambda p: A.energy(plan, p, tau, gam), psi + eps * e, torch.ones(B, dtype=torch.float64, device=DEV))[1])
        gm = host(torch.autograd.functional.vjp(lambda p: A.energy(plan, p, tau, gam), psi - eps * e, torch.ones(B, dtype=torch.float64, device=DEV))[1])
        hfd = (gp - gm) / (2 * eps) - eps**2 / 6 * host(e) ** 3 / N
        assert np.max(np.abs(hfd - host(hv))) < tol * np.max(np.abs(host(hv)))
        p_np = host(psi)
        assert np.allclose(host(gt), (p_np**2).mean(axis=(1, 2, 3)) / 2, rtol=1e-12)
        assert np.allclose(host(gg), -(p_np**3).mean(axis=(1, 2, 3)) / 6, rtol=1e-12)
        h = 0.3
        dtau_fd = host(A.energy(plan, psi, tau + h, gam) - A.energy(plan, psi, tau - h, gam)) / (2 * h)
        assert np.allclose(dtau_fd, host(gt), rtol=1e-10, atol=1e-14)
