"""Seeded synthetic inputs for the Landau-Brazovskii (LB) workloads.

This module only draws random numbers and builds initial order-parameter
fields; it holds none of the energy, gradient, Hessian or trust-region
arithmetic. Both the CPU oracle tests and the GPU path consume the arrays it
returns, so the two sides always start from identical host data.

Every field is a real array in C order (last axis fastest) on the periodic
grid x_i = i * L / n of a box [0, L_0) x ... x [0, L_{d-1}) (Section 2, grid
set T_M^d with an orthorhombic lattice).

Workloads (the paper's experiments are synthetic too, Section 4, Tables 1-2):
  * ``single_2d``   64x64, box 8*pi, tau=-0.15, gamma=0.25, noise N(0, 0.1^2)
  * ``bcc_3d``      128^3, box 8*sqrt(2)*pi, tau=-0.2, gamma=0.3, BCC trial
                    function (unit amplitude on the 12 {110} modes at integer
                    index (+-4, +-4, 0) and permutations, |Bk|^2 = 1) plus
                    N(0, 0.01^2) noise
  * ``phase_sweep`` 64 2D instances, n drawn from {64,96,128,256,512},
                    box 8*pi*n/64, (tau, gamma) on an 8x8 grid
  * ``diff_3d``     96^3, box 6*sqrt(2)*pi, batch 8, (tau, gamma) in
                    {-0.1,-0.2} x {0.2,0.3,0.4,0.5}
  * ``large_3d``    256^3, box 16*pi, tau=-0.25, gamma=0.4, N(0, 0.05^2)
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np


@dataclass(frozen=True)
class GridSpec:
    """A periodic orthorhombic grid: ``n`` points per axis on a box of sides ``box``."""

    n: Tuple[int, ...]
    box: Tuple[float, ...]

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))


@dataclass(frozen=True)
class LBParams:
    """Model coefficients: interaction xi^2 (Delta + q^2)^2, bulk tau/2 psi^2 - gamma/6 psi^3 + psi^4/24."""

    tau: float
    gamma: float
    xi: float = 1.0
    q: float = 1.0


def zero_mean_noise(shape: Sequence[int], sigma: float, seed: int) -> np.ndarray:
    """N(0, sigma^2) samples from ``numpy.random.default_rng(seed)``, mean removed (zero mass)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(tuple(shape)) * sigma
    return x - x.mean()


def cosine_modes(n: Sequence[int], modes: Sequence[Sequence[int]], amplitude: float) -> np.ndarray:
    """Real field sum_{k in S} a * exp(i 2 pi k.j/n) for a set S closed under k -> -k.

    ``modes`` lists integer reciprocal indices; S must contain -k with every k,
    so the sum is the real field sum_k a*cos(2 pi k.j/n).
    """
    S = [tuple(int(c) for c in k) for k in modes]
    Sset = set(S)
    for k in S:
        if tuple(-c for c in k) not in Sset:
            raise ValueError("mode set must be closed under negation")
    axes = [np.arange(m) for m in n]
    mesh = np.meshgrid(*axes, indexing="ij")
    out = np.zeros(tuple(n))
    for k in S:
        phase = sum(2.0 * math.pi * k[a] * mesh[a] / n[a] for a in range(len(n)))
        out += amplitude * np.cos(phase)
    return out


def bcc_110_modes(m: int) -> List[Tuple[int, int, int]]:
    """The 12 {110} reciprocal indices scaled by m: all permutations of (+-m, +-m, 0)."""
    out = set()
    for s1, s2 in itertools.product((1, -1), repeat=2):
        for perm in set(itertools.permutations((s1 * m, s2 * m, 0))):
            out.add(perm)
    return sorted(out)


def hex_2d_modes(m: int) -> List[Tuple[int, int]]:
    """Six 2D hexagonal-lattice indices for a box of sides (2*m*2pi, 2*m*2pi/sqrt(3)).

    With box (4*pi*m, 4*pi*m/sqrt(3)) the indices (+-2m, 0) and (+-m, +-m)
    all have |Bk| = 1, and they form the two triangles of the hexagonal phase.
    """
    return [(2 * m, 0), (-2 * m, 0), (m, m), (-m, -m), (m, -m), (-m, m)]


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------


@dataclass
class Instance:
    grid: GridSpec
    params: LBParams
    psi0: np.ndarray
    label: str = ""


def single_2d(n: int = 64, seed: int = 0) -> Instance:
    """64x64 on [0, 8 pi)^2 (critical shell |k| = 4), tau=-0.15, gamma=0.25, psi0 ~ N(0, 0.1^2) zero-mean."""
    L = 8.0 * math.pi * n / 64.0
    g = GridSpec((n, n), (L, L))
    return Instance(g, LBParams(-0.15, 0.25), zero_mean_noise(g.n, 0.1, seed), f"single_2d_{n}")


def bcc_3d(n: int = 128, seed: int = 0, amplitude: float = 1.0, noise: float = 0.01) -> Instance:
    """128^3 on [0, 8 sqrt(2) pi)^3 (shell |k|^2 = 32), tau=-0.2, gamma=0.3; BCC {110} trial + noise.

    The {110} index is scaled so that |Bk|^2 = 1 for every grid size: with the
    box side 8*sqrt(2)*pi * n/128 the index is (+-4n/128, +-4n/128, 0).
    """
    if n % 32:
        raise ValueError("bcc_3d needs n divisible by 32 so the {110} modes sit on the shell")
    m = 4 * n // 128
    L = 8.0 * math.sqrt(2.0) * math.pi * n / 128.0
    g = GridSpec((n, n, n), (L, L, L))
    psi = cosine_modes(g.n, bcc_110_modes(m), amplitude)
    psi = psi + zero_mean_noise(g.n, noise, seed)
    psi = psi - psi.mean()
    return Instance(g, LBParams(-0.2, 0.3), psi, f"bcc_3d_{n}")


def hessvec_direction(n: Sequence[int], seed: int = 1) -> np.ndarray:
    """Direction v ~ N(0, 1) zero-mean used for timing and checking Hessian-vector products."""
    return zero_mean_noise(n, 1.0, seed)


PHASE_SWEEP_SIZES = (64, 96, 128, 256, 512)


def phase_sweep(count: int = 64, sizes: Sequence[int] = PHASE_SWEEP_SIZES, draw_seed: int = 2603) -> List[Instance]:
    """Batched 2D phase sweep: n_i drawn uniformly from ``sizes`` (seeded), box 8 pi n_i/64.

    (tau, gamma) lie on linspace(-0.3, 0, 8) x linspace(0, 0.5, 8); instance
    i = 8a + b takes tau_a, gamma_b and psi0 ~ N(0, 0.1^2) zero-mean from seed i.
    """
    rng = np.random.default_rng(draw_seed)
    ns = rng.choice(np.array(sizes), size=count)
    taus = np.linspace(-0.3, 0.0, 8)
    gammas = np.linspace(0.0, 0.5, 8)
    out = []
    for i in range(count):
        n = int(ns[i])
        a, b = divmod(i % 64, 8)
        L = 8.0 * math.pi * n / 64.0
        g = GridSpec((n, n), (L, L))
        out.append(Instance(g, LBParams(float(taus[a]), float(gammas[b])), zero_mean_noise(g.n, 0.1, i), f"sweep_{i}_{n}"))
    return out


def diff_3d(n: int = 96) -> List[Instance]:
    """96^3 on [0, 6 sqrt(2) pi)^3 (3 BCC cells), batch 8 = {-0.1,-0.2} x {0.2,0.3,0.4,0.5}, N(0,0.1^2)."""
    L = 6.0 * math.sqrt(2.0) * math.pi * n / 96.0
    g = GridSpec((n, n, n), (L, L, L))
    out = []
    i = 0
    for tau in (-0.1, -0.2):
        for gamma in (0.2, 0.3, 0.4, 0.5):
            out.append(Instance(g, LBParams(tau, gamma), zero_mean_noise(g.n, 0.1, i), f"diff_{i}"))
            i += 1
    return out


def large_3d(n: int = 256, seed: int = 0) -> Instance:
    """256^3 on [0, 16 pi)^3 (shell |k| = 8), tau=-0.25, gamma=0.4, psi0 ~ N(0, 0.05^2) zero-mean."""
    L = 16.0 * math.pi * n / 256.0
    g = GridSpec((n, n, n), (L, L, L))
    return Instance(g, LBParams(-0.25, 0.4), zero_mean_noise(g.n, 0.05, seed), f"large_3d_{n}")
