"""GPU: the inner iteration in the split order (lb_plan_set_plane_split: the
axis-1 transform split by x1 mod K, K = 2 or 4, its first inverse and last
forward K-point steps done across column groups in the axis-0 passes, a
split-plane pass with K workgroups per plane) against the oracle's Algorithm 3
(Section 3.2), on orthorhombic boxes and a general lattice, in FP64 and FP32,
for each thread count of the split-plane pass; the Hessian product in the
same orders; batched instances equal single ones bit for bit; the variant
API and the autotuner."""
import functools
import math

import numpy as np
import pytest
import torch

from oracle import lb_oracle as O
from paper_2603_03933_amd import inputs as I
from paper_2603_03933_amd import lb

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")

TRICLINIC = np.array([[4.0, 1.1, 0.6], [0.3, 3.8, 0.9], [-0.4, 0.2, 4.3]])


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def rms(a):
    return math.sqrt(float(np.mean(a * a)))


# grids with a pair-split order: square planes (n1 = n2) of 32, 64, 96 and 128
# points; the axis-0 column workgroups are 32, 64, 16 and 16 columns wide, so
# the pair lanes are 16 (lane permute), 32 (lane permute) and 8 (DPP rotate
# within rows of 16 lanes) apart
GRIDS = [
    ((64, 32, 32), (8 * math.sqrt(2) * math.pi, 4 * math.sqrt(2) * math.pi, 4 * math.sqrt(2) * math.pi)),
    ((24, 64, 64), (3 * math.pi, 8 * math.pi, 8 * math.pi)),
    ((96, 96, 96), (12 * math.pi,) * 3),
    ((128, 128, 128), (8 * math.sqrt(2) * math.pi,) * 3),
]


def _subproblem(plan, m, psi, g_hat, r, k, eta=0.1):
    return plan.lb_tr_subproblem(lb.Params(m.tau, m.gamma, m.xi, m.q), dev(psi), dev(O.inv(g_hat)), r,
                                 lb.sub_opts(eta=eta, eps_sub=0.0, max_inner=k))


@pytest.mark.parametrize("n,box", GRIDS)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_split_subproblem_matches_oracle(n, box, precision, tol):
    """Iterations of Algorithm 3 with the constraint active, pair-split order
    with each built thread count of the half-plane pass, element by element
    against the oracle; the plane order gives the same iterates to rounding."""
    print(f"pair-split subproblem {n} {precision}", flush=True)
    m = O.Model(O.Grid(n, box), -0.15, 0.25, 1.05, 0.95)
    psi = I.zero_mean_noise(n, 0.2, 91)
    g_hat = O.gradient(m, psi)
    k, r = 6, 0.05
    ref = O.imex_subproblem(m, psi, g_hat, r, O.SubOpts(eta=0.1, eps_sub=0.0, max_inner=k))
    d_or = O.inv(ref.d)
    plan = lb.Plan(n, box, precision=precision)
    d_plane, info_p, _ = _subproblem(plan, m, psi, g_hat, r, k)
    assert plan.lb_plan_get_variant()[0] == 0
    for threads in (256, 512, 1024):
        plan.lb_plan_set_plane_split(1, threads)
        assert plan.lb_plan_get_variant() == (1, threads, 0)
        d, info, rc = _subproblem(plan, m, psi, g_hat, r, k)
        d = host(d)
        err = rms(d - d_or) / rms(d_or)
        print(f"  threads {threads}: lambda {info.lambda_:.15e} (oracle {ref.lam:.15e}), iterate error {err:.2e}")
        assert info.iters == ref.iters == k and rc == lb.LB_NOT_CONVERGED
        assert ref.lam > 0 and abs(info.lambda_ - ref.lam) <= tol * max(1.0, ref.lam)
        assert err <= tol
        assert rms(d - host(d_plane)) <= tol * rms(d_or)
    plan.lb_plan_set_plane_split(0, 0)
    assert plan.lb_plan_get_variant()[0] == 0


# grids with a four-part order (axis-0 workgroups of 16 columns): 128^3 and a
# 128 x 64 x 64 grid (parts of 32 and 16 rows)
GRIDS4 = [
    ((128, 128, 128), (8 * math.sqrt(2) * math.pi,) * 3),
    ((128, 64, 64), (8 * math.sqrt(2) * math.pi, 4 * math.sqrt(2) * math.pi, 4 * math.sqrt(2) * math.pi)),
]


@pytest.mark.parametrize("n,box", GRIDS4)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_four_part_subproblem_and_hessvec_match_oracle(n, box, precision, tol):
    """Four parts (DPP rotates by 4, 8 and 12 within rows of 16 lanes): the
    subproblem iterations and the Hessian product against the oracle."""
    print(f"four-part split {n} {precision}", flush=True)
    m = O.Model(O.Grid(n, box), -0.15, 0.25, 1.05, 0.95)
    psi = I.zero_mean_noise(n, 0.2, 91)
    g_hat = O.gradient(m, psi)
    k, r = 6, 0.05
    ref = O.imex_subproblem(m, psi, g_hat, r, O.SubOpts(eta=0.1, eps_sub=0.0, max_inner=k))
    d_or = O.inv(ref.d)
    plan = lb.Plan(n, box, precision=precision)
    for threads in (256, 512, 1024):
        plan.lb_plan_set_plane_split(2, threads)
        assert plan.lb_plan_get_variant() == (2, threads, 0)
        d, info, rc = _subproblem(plan, m, psi, g_hat, r, k)
        err = rms(host(d) - d_or) / rms(d_or)
        print(f"  threads {threads}: lambda {info.lambda_:.15e} (oracle {ref.lam:.15e}), iterate error {err:.2e}")
        assert info.iters == ref.iters == k and ref.lam > 0
        assert abs(info.lambda_ - ref.lam) <= tol * max(1.0, ref.lam) and err <= tol
    v = I.hessvec_direction(n, 96)
    prm = lb.Params(m.tau, m.gamma, m.xi, m.q)
    plan.lb_plan_set_hessvec_split(2)
    hv = host(plan.lb_hessvec(prm, dev(psi), dev(v)))
    raw = host(plan.lb_hessvec_raw(prm, dev(psi), dev(v)))
    scale = rms(O.inv(m.Lam * O.fwd(v))) + rms(O.Gamma_p(psi, m.tau, m.gamma) * v)
    err = rms(hv - O.hessvec_phys(m, psi, v)) / scale
    print(f"  Hv: error {err:.2e} of the term scale")
    assert err <= tol and rms(raw - O.hessvec_raw(m, psi, v)) <= tol * scale / psi.size


@functools.lru_cache(maxsize=4)
def _oracle_case(i):
    n, box = GRIDS[i]
    m = O.Model(O.Grid(n, box), -0.15, 0.25, 1.05, 0.95)
    psi = I.zero_mean_noise(n, 0.2, 91)
    g_hat = O.gradient(m, psi)
    ref = O.imex_subproblem(m, psi, g_hat, 0.05, O.SubOpts(eta=0.1, eps_sub=0.0, max_inner=6))
    return m, psi, g_hat, ref


@pytest.mark.parametrize("i", [0, 2, 3])  # axis-0 lengths 64, 96, 128
@pytest.mark.parametrize("column_plan", [1, 2, 3])
@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_column_plans_match_oracle(i, column_plan, split, precision, tol):
    """The axis-0 passes in radix plans 1 (4 first) and 2 (16 first) and in
    plan 3 (twice the columns per workgroup), in both orders of the inner
    iteration, against the oracle's iterations. Plan 3 with two parts needs
    each part's columns to fill its workgroups (not at 64 x 32 x 32, which
    then runs plan 0)."""
    n, box = GRIDS[i]
    print(f"column plan {column_plan}, split {split}, {n} {precision}", flush=True)
    m, psi, g_hat, ref = _oracle_case(i)
    plan = lb.Plan(n, box, precision=precision)
    plan.lb_plan_set_column_plan(column_plan)
    if split:
        plan.lb_plan_set_plane_split(1, 0)
    run_plan = 0 if (column_plan == 3 and split and n[1] == 32) else column_plan
    assert plan.lb_plan_get_variant()[0::2] == (split, run_plan)
    d, info, rc = _subproblem(plan, m, psi, g_hat, 0.05, 6)
    d_or = O.inv(ref.d)
    err = rms(host(d) - d_or) / rms(d_or)
    print(f"  lambda {info.lambda_:.15e} (oracle {ref.lam:.15e}), iterate error {err:.2e}")
    assert info.iters == ref.iters == 6
    assert abs(info.lambda_ - ref.lam) <= tol * max(1.0, ref.lam) and err <= tol


@pytest.mark.parametrize("n,box", GRIDS)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_split_hessvec_matches_oracle(n, box, precision, tol):
    """lb_hessvec (projected) and lb_hessvec_raw in the pair-split order
    against the oracle's products (Section 2: Lambda in reciprocal space,
    Gamma'(psi) pointwise), and against the plane order to rounding; a batch
    of two fields."""
    print(f"pair-split Hv {n} {precision}", flush=True)
    m = O.Model(O.Grid(n, box), -0.2, 0.3, 1.1, 0.9)
    psi = I.zero_mean_noise(n, 0.4, 95)
    v = I.hessvec_direction(n, 96)
    prm = lb.Params(m.tau, m.gamma, m.xi, m.q)
    plan = lb.Plan(n, box, precision=precision)
    plan.lb_plan_set_hessvec_split(0)
    hv_plane = host(plan.lb_hessvec(prm, dev(psi), dev(v)))
    plan.lb_plan_set_hessvec_split(1)
    hv = host(plan.lb_hessvec(prm, dev(psi), dev(v)))
    raw = host(plan.lb_hessvec_raw(prm, dev(psi), dev(v)))
    h_or = O.hessvec_phys(m, psi, v)
    scale = rms(O.inv(m.Lam * O.fwd(v))) + rms(O.Gamma_p(psi, m.tau, m.gamma) * v)
    err = rms(hv - h_or) / scale
    print(f"  projected: error {err:.2e} of the term scale, vs plane order {rms(hv - hv_plane) / scale:.2e}")
    assert err <= tol and rms(hv - hv_plane) <= tol * scale
    r_or = O.hessvec_raw(m, psi, v)
    assert rms(raw - r_or) <= tol * scale / psi.size
    # a batch of two fields: instance 1 with other parameters
    prm2 = [prm, lb.Params(-0.1, 0.2, 1.1, 0.9)]
    psi2 = np.stack([psi, I.zero_mean_noise(n, 0.3, 97)])
    v2 = np.stack([v, I.hessvec_direction(n, 98)])
    pb = lb.Plan(n, box, batch=2, precision=precision)
    pb.lb_plan_set_hessvec_split(1)
    hb = host(pb.lb_hessvec(prm2, dev(psi2), dev(v2)))
    assert np.array_equal(hb[0], hv)  # same kernels, same order: identical bits
    m2 = O.Model(O.Grid(n, box), -0.1, 0.2, 1.1, 0.9)
    scale2 = rms(O.inv(m2.Lam * O.fwd(v2[1]))) + rms(O.Gamma_p(psi2[1], m2.tau, m2.gamma) * v2[1])
    assert rms(hb[1] - O.hessvec_phys(m2, psi2[1], v2[1])) <= tol * scale2


def test_split_general_lattice_matches_oracle():
    """A triclinic cell (cross terms in |Bk|^2, the general-lattice kernels):
    pair-split subproblem iterations against the oracle."""
    n, A = (64, 32, 32), 5.0 * TRICLINIC @ np.diag([2.0, 1.0, 1.0])
    m = O.Model(O.Grid(n, lattice=A), -0.15, 0.25)
    psi = I.zero_mean_noise(n, 0.2, 92)
    g_hat = O.gradient(m, psi)
    ref = O.imex_subproblem(m, psi, g_hat, 0.05, O.SubOpts(eta=0.1, eps_sub=0.0, max_inner=50))
    plan = lb.Plan(n, [1.0] * 3)
    plan.lb_plan_set_lattice(A)
    plan.lb_plan_set_plane_split(1, 0)
    d, info, rc = _subproblem(plan, m, psi, g_hat, 0.05, 50)
    d = host(d)
    print(f"triclinic pair-split: lambda {info.lambda_:.15e} (oracle {ref.lam:.15e})")
    assert info.iters == ref.iters == 50
    assert ref.lam > 0 and abs(info.lambda_ - ref.lam) <= 1e-10 * max(1.0, ref.lam)
    assert rms(d - O.inv(ref.d)) <= 1e-10 * rms(O.inv(ref.d))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_split_batched_solve_equals_single_solves(precision):
    """Three 64 x 32 x 32 instances in one batch, pair-split order, against the
    same instances solved one at a time in that order: identical bits; the
    oracle's gradient norm and energy at the returned fields."""
    n, box = (64, 32, 32), (8 * math.sqrt(2) * math.pi, 4 * math.sqrt(2) * math.pi, 4 * math.sqrt(2) * math.pi)
    print(f"pair-split batched solve {n} {precision}", flush=True)
    B = 3
    prms = [lb.Params(-0.15 - 0.03 * k, 0.2 + 0.05 * k) for k in range(B)]
    psi0 = np.stack([I.zero_mean_noise(n, 0.1, 93 + k) for k in range(B)])
    sub = {"max_inner": 3000, "poll_every": 16}
    if precision == "fp32":
        sub["eps_sub_rel"] = 1e-5
    opts = lb.tr_opts(grad_norm_inf=0, eps=1e-8, max_outer=60, sub=sub)
    p1 = lb.Plan(n, box, precision=precision)
    p1.lb_plan_set_plane_split(1, 0)
    single = []
    for k in range(B):
        x = dev(psi0[k])
        info, rc = p1.lb_imex_tr_solve(prms[k], x, opts)
        single.append((info, rc, host(x)))
    pb = lb.Plan(n, box, batch=B, precision=precision)
    pb.lb_plan_set_plane_split(1, 0)
    x = dev(psi0)
    res = pb.lb_imex_tr_solve_batch(prms, x, opts)
    out = host(x)
    for k, ((info, rc), (sinfo, src, sx)) in enumerate(zip(res, single)):
        assert rc == src and info.outer == sinfo.outer and info.inner_total == sinfo.inner_total, k
        assert info.energy == sinfo.energy and np.array_equal(out[k], sx), k
    # the oracle at the returned fields: a stationary point (FP64) and the reported energy
    for k in range(B):
        if res[k][1] != lb.LB_OK:
            continue
        m = O.Model(O.Grid(n, box), prms[k].tau, prms[k].gamma)
        gn = O.norm(O.gradient(m, out[k]))
        E = O.energy(m, out[k])
        print(f"  instance {k}: outer {res[k][0].outer}, oracle |g| {gn:.2e}, E {E:.12e} (GPU {res[k][0].energy:.12e})")
        assert abs(res[k][0].energy - E) <= 1e-12 * max(1.0, abs(E))
        if precision == "fp64":
            assert gn < 1e-8


def test_split_api_and_autotune():
    # a grid without a plane pass, and grids whose column pairs do not fill
    # whole workgroups ((n1/2)(n2/2 + 1) = 600 and 272 columns against 16 and
    # 32 per workgroup half)
    with pytest.raises(lb.LBError):
        lb.Plan((32, 32), (4 * math.pi,) * 2).lb_plan_set_plane_split(1, 0)
    with pytest.raises(lb.LBError):
        lb.Plan((48, 48, 48), (6 * math.pi,) * 3).lb_plan_set_plane_split(1, 0)
    with pytest.raises(lb.LBError):
        lb.Plan((32, 32, 32), (4 * math.pi,) * 3).lb_plan_set_plane_split(1, 0)
    plan = lb.Plan((64, 64, 64), (8 * math.pi,) * 3)
    with pytest.raises(lb.LBError):
        plan.lb_plan_set_plane_split(3, 0)
    with pytest.raises(lb.LBError):
        plan.lb_plan_set_plane_split(1, 384)
    prm = lb.Params(-0.15, 0.25)
    psi = dev(I.zero_mean_noise((64, 64, 64), 0.2, 94))
    threads = plan.lb_plan_autotune(prm, psi, reps=5)
    split, t2, cp = plan.lb_plan_get_variant()
    print(f"autotune 64^3: split {split}, threads {threads}, column plan {cp}")
    assert threads in (256, 512, 1024) and t2 == threads and split in (0, 1) and cp in (0, 1, 2, 3)
    with pytest.raises(lb.LBError):
        plan.lb_plan_set_column_plan(4)
    with pytest.raises(lb.LBError):
        plan.lb_plan_set_hessvec_split(3)
    with pytest.raises(lb.LBError):
        lb.Plan((32, 32, 32), (4 * math.pi,) * 3).lb_plan_set_hessvec_split(1)
    with pytest.raises(lb.LBError):  # four parts need 16 columns per axis-0 workgroup (64^3 has 32)
        plan.lb_plan_set_plane_split(2, 0)
    big = lb.Plan((256, 256, 256), (16 * math.pi,) * 3, precision="fp32")
    assert big.lb_plan_get_variant()[:2] == (0, 0)  # built in: the five passes where the plane does not fit
    big.lb_plan_set_plane_split(2, 0)
    assert big.lb_plan_get_variant() == (2, 512, 0)  # four parts, the built-in 512 threads
    big.lb_plan_set_plane_split(0, 0)
    assert big.lb_plan_get_variant()[:2] == (0, 0)
    with pytest.raises(lb.LBError):  # only the built-in thread count at 256
        big.lb_plan_set_plane_split(2, 1024)
    with pytest.raises(lb.LBError):  # axis-0 length 32: only the built-in plan
        lb.Plan((32, 32, 32), (4 * math.pi,) * 3).lb_plan_set_column_plan(1)
