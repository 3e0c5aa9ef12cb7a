"""Writes single_2d_64_oracle.json: the oracle's IMEX-TR solve of the 2D 64 x 64
single-instance workload (box 8 pi, xi = q = 1, tau = -0.15, gamma = 0.25,
zero-mean N(0, 0.1^2) start, seed 0), run to ||grad E||_2 < 1e-8 with the
Section 4 parameters. Calls only the oracle and the seeded input generator
(about a minute on one core).

    python3 tests/golden/make_single_2d_64.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lb_oracle as O  # noqa: E402
from paper_2603_03933_amd import inputs as I  # noqa: E402


def main():
    inst = I.single_2d(64)
    m = O.Model(O.Grid(inst.grid.n, inst.grid.box), inst.params.tau, inst.params.gamma)
    ref = O.imex_tr_solve(m, inst.psi0, O.TROpts(grad_norm="l2", eps=1e-8, max_inner=10000))
    assert ref.converged
    psi = ref.psi
    power = np.abs(np.fft.fft2(psi) / psi.size) ** 2
    top = np.argsort(power.ravel())[::-1][:8]
    out = {
        "workload": "single_2d 64x64, box 8 pi, xi = q = 1, tau = -0.15, gamma = 0.25, N(0, 0.1^2) zero-mean, seed 0",
        "solver": "oracle imex_tr_solve, ||g||_2 < 1e-8, max_inner 10000, Section 4 parameters",
        "energy": ref.energy,
        "gnorm": ref.gnorm,
        "outer": ref.outer,
        "inner_total": ref.inner_total,
        "psi_min": float(psi.min()),
        "psi_max": float(psi.max()),
        "psi_rms": float(np.sqrt(np.mean(psi ** 2))),
        "dense_lambda_min": float(O.hessian_eigs(m, psi)[0]) if psi.size <= 4096 else None,
        "top_power": [[int(i // psi.shape[1]), int(i % psi.shape[1]), float(power.ravel()[i])] for i in top],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "single_2d_64_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["energy"], out["outer"], out["inner_total"])


if __name__ == "__main__":
    main()
