"""GPU: the allocation-free Hessian-vector product (lb_hessvec_noalloc, the
library's fixed workspace) against lb_hessvec through a plan, on two calls in
a row, the second on a smaller grid; and its size limit."""
import math

import numpy as np
import pytest
import torch

from paper_2603_03933_amd import inputs as I
from paper_2603_03933_amd import lb

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def rms(a):
    return math.sqrt(float(torch.mean(a * a)))


CASES = [((64, 64, 64), (8 * math.sqrt(2) * math.pi,) * 3, True), ((24, 16, 48), (3 * math.pi, 2 * math.pi, 6 * math.pi), False),
         ((48, 96), (6 * math.pi, 12 * math.pi), True)]


def test_noalloc_hessvec_equals_plan_hessvec_on_consecutive_calls():
    prm = lb.Params(-0.2, 0.3, 1.1, 0.9)
    for k, (n, box, project) in enumerate(CASES):  # large grid first, then smaller ones
        print(f"noalloc case {k}: grid {n} project {project}", flush=True)
        psi = dev(I.zero_mean_noise(n, 0.4, 60 + k))
        v = dev(I.hessvec_direction(n, 70 + k))
        ref = lb.Plan(n, box).lb_hessvec(prm, psi, v, project=project)
        out = torch.full_like(v, float("nan"))
        lb.lb_hessvec_noalloc(n, box, prm, psi, v, out=out, project=project)
        torch.cuda.synchronize()
        assert torch.isfinite(out).all()
        assert rms(out - ref) <= 1e-12 * rms(ref), (n, rms(out - ref) / rms(ref))
        out2 = lb.lb_hessvec_noalloc(n, box, prm, psi, v, project=project)  # repeat: same workspace, same bits
        torch.cuda.synchronize()
        assert torch.equal(out2, out)


def test_noalloc_hessvec_rejects_grids_beyond_its_workspace():
    n, box = (128, 128, 128), (8 * math.sqrt(2) * math.pi,) * 3
    psi = torch.zeros(n, dtype=torch.float64, device=DEV)
    with pytest.raises(lb.LBError):
        lb.lb_hessvec_noalloc(n, box, lb.Params(-0.2, 0.3), psi, psi.clone())
    with pytest.raises(lb.LBError):
        lb.lb_hessvec_noalloc((10, 16), (1.0, 1.0), lb.Params(-0.2, 0.3), psi[0, :10, :16].contiguous(), psi[0, :10, :16].contiguous())
