"""Plain FP64 CPU oracle for the IMEX trust-region (IMEX-TR) method on the
Landau-Brazovskii (LB) energy (Bao, Deng, Jiang, Zhang, arXiv 2603.03933).

THIS IS TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it. The GPU library never
calls it and shares no code with it.

Conventions (Section 2; readings listed in the project design notes):
  * grid T_M^d: x_j = j * L / n per axis, N = prod(n) points, orthorhombic
    lattice A = diag(L), reciprocal B = diag(2 pi / L) so A B^T = 2 pi I;
  * reciprocal indices K_M^d: signed k in [-n/2, n/2) per axis;
  * normalised DFT: psi_hat(k) = (1/N) sum_x psi(x) exp(-i (Bk).x);
  * every vector of the optimisation lives in Psi_hat coordinates (Section 3):
    <a, b> = Re sum_k a_k conj(b_k) = (1/N) sum_x a(x) b(x) (Parseval), and
    ||a|| = sqrt(<a, a>); the k = 0 entry is removed by P (mass constraint);
  * Lambda_k = xi^2 (q^2 - |Bk|^2)^2 (the paper has xi = q = 1), bulk
    F(psi) = tau/2 psi^2 - gamma/6 psi^3 + psi^4/24, with
    Gamma psi = F'(psi) and Gamma' = F''(psi) = tau - gamma psi + psi^2/2.

Spectral arrays are full complex arrays of the grid's shape (Hermitian because
the fields are real). Nothing here is blocked, fused or reordered beyond what
the paper's definitions and algorithms state.

Pins (tests/test_oracle_*.py): trial-function closed forms, exact finite
differences of a quartic, the exact Taylor expansion, the psi = 0 spectrum,
symmetry / mass / translation invariants, naive DFT, dense global minimiser of
the trust-region subproblem (Conn-Gould-Toint Cor. 7.2.2), the Carmon-Duchi
sign condition, and dense Hessian eigenvalues at the end of a full solve.
The outer iteration path beyond its first few iterations is compared only
through its endpoint (rounding can flip accept/reject decisions).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# Grid and reciprocal space (Section 2: T_M^d, K_M^d, normalised DFT)
# ---------------------------------------------------------------------------


class Grid:
    """Periodic grid T_M^d (Section 2) with n[a] points per axis.

    Either an orthorhombic box (``box``: sides L_a, lattice A = diag(L)) or a
    general Bravais lattice (``lattice``: the d x d matrix A whose column a is
    the cell vector along grid axis a; grid points x_j = A (j / n)). The
    reciprocal matrix is B = 2 pi A^{-T} (A B^T = 2 pi I), so the Fourier mode
    of index k is exp(i (Bk).x) with Bk = sum_a k_a B[:, a], and
    |Bk|^2 = k^T B^T B k.
    """

    def __init__(self, n: Sequence[int], box: Optional[Sequence[float]] = None, lattice=None):
        self.n = tuple(int(m) for m in n)
        self.dim = len(self.n)
        if self.dim not in (1, 2, 3):
            raise ValueError("dimension must be 1, 2 or 3")
        if lattice is None:
            if box is None or len(box) != self.dim:
                raise ValueError("dimension mismatch")
            self.box = tuple(float(L) for L in box)
            self.A = np.diag(self.box)
        else:
            self.A = np.array(lattice, dtype=float).reshape(self.dim, self.dim)
            self.box = None
        self.B = 2.0 * math.pi * np.linalg.inv(self.A).T
        self.N = int(np.prod(self.n))
        # signed reciprocal index per axis, K_M: -n/2 <= k < n/2
        self.kidx = [signed_index(m) for m in self.n]
        mesh = np.meshgrid(*self.kidx, indexing="ij")
        if lattice is None:
            # |Bk|^2 with B = diag(2 pi / L)
            self.kk = sum((2.0 * math.pi * mesh[a] / self.box[a]) ** 2 for a in range(self.dim))
        else:
            self.kk = kk_general(self.B, self.n, mesh)
        self.zero = (0,) * self.dim


def kk_general(B: np.ndarray, n: Sequence[int], mesh) -> np.ndarray:
    """|Bk|^2 = sum_ab G_ab k_a k_b, G = B^T B, over the signed index set K_M.

    An index k_a = -n_a/2 (Nyquist) stands for the same DFT entry as +n_a/2,
    so the conjugate partner of entry k, which a real field fixes to the
    complex conjugate, is k with every Nyquist coordinate negated. With
    off-diagonal G the two carry different |Bk|^2; both take their mean, so
    that the multiplier maps real fields to real fields: the cross term
    k_a k_b is kept when axes a and b are both at Nyquist or both not, and
    dropped when exactly one is (the mean of the two signs).
    """
    G = B.T @ B
    d = len(n)
    nyq = [mesh[a] == -(n[a] // 2) if n[a] % 2 == 0 else np.zeros_like(mesh[a], dtype=bool) for a in range(d)]
    out = np.zeros(mesh[0].shape)
    for a in range(d):
        out = out + G[a, a] * mesh[a].astype(float) ** 2
    for a in range(d):
        for b in range(a + 1, d):
            keep = nyq[a] == nyq[b]
            out = out + np.where(keep, 2.0 * G[a, b] * mesh[a].astype(float) * mesh[b].astype(float), 0.0)
    return out


def signed_index(n: int) -> np.ndarray:
    """Integer reciprocal indices in DFT storage order, mapped to [-n/2, n/2)."""
    j = np.arange(n)
    return np.where(j < (n + 1) // 2, j, j - n) if n % 2 else np.where(j < n // 2, j, j - n)


def Lambda(grid: Grid, xi: float = 1.0, q: float = 1.0) -> np.ndarray:
    """Interaction multiplier Lambda_k = xi^2 (q^2 - |Bk|^2)^2 (Section 2, gradient of G)."""
    return xi * xi * (q * q - grid.kk) ** 2


def fwd(psi: np.ndarray) -> np.ndarray:
    """psi_hat = F_N psi with the 1/N normalisation of Section 2."""
    return np.fft.fftn(psi) / psi.size


def inv(psi_hat: np.ndarray) -> np.ndarray:
    """Inverse of ``fwd``; the input is Hermitian so the result is real."""
    x = np.fft.ifftn(psi_hat) * psi_hat.size
    return x.real


def dft_naive(psi: np.ndarray) -> np.ndarray:
    """O(N^2) direct normalised DFT (1/N) sum_x psi(x) exp(-2 pi i sum_a k_a j_a / n_a).

    Used only on tiny grids to pin the FFT-based path (Section 2 definition).
    """
    n = psi.shape
    N = psi.size
    xs = np.stack(np.meshgrid(*[np.arange(m) for m in n], indexing="ij"), -1).reshape(N, len(n))
    ks = xs.copy()  # storage order indices 0..n-1; exp is periodic so signs do not matter
    phase = np.zeros((N, N))
    for a in range(len(n)):
        phase += np.outer(ks[:, a], xs[:, a]) / n[a]
    W = np.exp(-2j * math.pi * phase)
    return (W @ psi.reshape(N)).reshape(n) / N


def project(a_hat: np.ndarray) -> np.ndarray:
    """P^T P: remove the k = 0 entry (discrete mass constraint e_1^T Psi_hat = 0, Section 3)."""
    out = a_hat.copy()
    out[(0,) * a_hat.ndim] = 0.0
    return out


def dot(a_hat: np.ndarray, b_hat: np.ndarray) -> float:
    """Real inner product Re sum_k a_k conj(b_k) of the Psi_hat coordinates."""
    return float(np.real(np.vdot(b_hat, a_hat)))


def norm(a_hat: np.ndarray) -> float:
    return math.sqrt(max(dot(a_hat, a_hat), 0.0))


def norm_inf(a_hat: np.ndarray) -> float:
    return float(np.max(np.abs(a_hat)))


# ---------------------------------------------------------------------------
# Bulk polynomial and its derivatives (equation lb_energy)
# ---------------------------------------------------------------------------


def F_bulk(psi, tau, gamma):
    return tau / 2.0 * psi**2 - gamma / 6.0 * psi**3 + psi**4 / 24.0


def dF_bulk(psi, tau, gamma):
    """F'(psi) = Gamma psi with Gamma = tau - gamma psi / 2 + psi^2 / 6."""
    return tau * psi - gamma / 2.0 * psi**2 + psi**3 / 6.0


def Gamma_p(psi, tau, gamma):
    """Gamma' = F''(psi) = tau - gamma psi + psi^2 / 2 (diagonal of grad^2 F in physical space)."""
    return tau - gamma * psi + psi**2 / 2.0


# ---------------------------------------------------------------------------
# Energy, gradient, Hessian-vector product (Section 2, eq. interaction_bulk_energy)
# ---------------------------------------------------------------------------


@dataclass
class Model:
    grid: Grid
    tau: float
    gamma: float
    xi: float = 1.0
    q: float = 1.0

    def __post_init__(self):
        self.Lam = Lambda(self.grid, self.xi, self.q)


def energy_parts(m: Model, psi: np.ndarray) -> Tuple[float, float]:
    """(G, F): G = 1/2 sum_k Lambda_k |psi_hat_k|^2, F = (1/N) sum_x F(psi(x)).

    The cubic and quartic sums of eq. interaction_bulk_energy are evaluated in
    physical space, pseudospectrally and without dealiasing.
    """
    ph = fwd(psi)
    G = 0.5 * float(np.sum(m.Lam * np.abs(ph) ** 2))
    F = float(np.mean(F_bulk(psi, m.tau, m.gamma)))
    return G, F


def energy(m: Model, psi: np.ndarray) -> float:
    G, F = energy_parts(m, psi)
    return G + F


def energy_spectral_sums(m: Model, psi_hat: np.ndarray) -> float:
    """E evaluated directly from the convolution sums of eq. interaction_bulk_energy.

    sum_{k1+k2=0}, sum_{k1+k2+k3=0}, sum_{k1+..+k4=0} over K_M^d with index
    arithmetic modulo n (the discrete orthogonality relation of Section 2).
    O(N^3) work: tiny grids only.
    """
    n = psi_hat.shape
    idx = list(np.ndindex(*n))
    val = {k: psi_hat[k] for k in idx}

    def neg(k):
        return tuple((-k[a]) % n[a] for a in range(len(n)))

    def add(k, h):
        return tuple((k[a] + h[a]) % n[a] for a in range(len(n)))

    G = 0.0
    S2 = 0.0
    for k in idx:
        G += m.Lam[k] * val[k] * val[neg(k)]
        S2 += val[k] * val[neg(k)]
    S3 = 0.0
    S4 = 0.0
    for k1 in idx:
        for k2 in idx:
            k12 = add(k1, k2)
            S3 += val[k1] * val[k2] * val[neg(k12)]
            for k3 in idx:
                S4 += val[k1] * val[k2] * val[k3] * val[neg(add(k12, k3))]
    E = 0.5 * G + m.tau / 2.0 * S2 - m.gamma / 6.0 * S3 + S4 / 24.0
    return float(np.real(E))


def gradient(m: Model, psi: np.ndarray) -> np.ndarray:
    """Projected gradient in Psi_hat coordinates: g = P(Lambda psi_hat + F_N F'(psi)).

    grad G = Lambda Psi_hat and grad F = F_N Gamma F_N^{-1} Psi_hat (Section 2);
    P removes the k = 0 entry (Section 3, E_bar(v) = E(P^T v)).
    """
    ph = fwd(psi)
    return project(m.Lam * ph + fwd(dF_bulk(psi, m.tau, m.gamma)))


def hessvec(m: Model, psi: np.ndarray, v_hat: np.ndarray) -> np.ndarray:
    """H v = P(Lambda v + F_N Gamma'(psi) F_N^{-1} v) for v in Psi_hat coordinates.

    grad^2 G = Lambda (diagonal in reciprocal space), grad^2 F = F_N Gamma' F_N^{-1}
    (diagonal in physical space); H = D + T with D = P Lambda P^T and
    T = P grad^2 F P^T (Section 3.2).
    """
    return project(m.Lam * v_hat) + T_apply(m, psi, v_hat)


def T_apply(m: Model, psi: np.ndarray, v_hat: np.ndarray) -> np.ndarray:
    """T v = P F_N (Gamma'(psi) * F_N^{-1} v): pointwise product in physical space + FFT (Remark, Section 3.2)."""
    return project(fwd(Gamma_p(psi, m.tau, m.gamma) * inv(v_hat)))


# physical-space helpers --------------------------------------------------


def gradient_phys(m: Model, psi: np.ndarray) -> np.ndarray:
    return inv(gradient(m, psi))


def gradient_raw(m: Model, psi: np.ndarray) -> np.ndarray:
    """dE/dpsi_x for E of eq. lb_energy as a function of all N grid values (sum
    over every k, no mass constraint): (F_N^{-1}(Lambda psi_hat) + F'(psi)) / N."""
    return (inv(m.Lam * fwd(psi)) + dF_bulk(psi, m.tau, m.gamma)) / psi.size


def hessvec_raw(m: Model, psi: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Hessian of the same function times v: (F_N^{-1} Lambda F_N v + Gamma'(psi) v) / N."""
    return (inv(m.Lam * fwd(v)) + Gamma_p(psi, m.tau, m.gamma) * v) / psi.size


def field_moments(psi: np.ndarray, w: Optional[np.ndarray] = None) -> np.ndarray:
    """[mean(psi^2), mean(psi^3), mean(w psi), mean(w psi^2)]: dE/dtau = first / 2,
    dE/dgamma = -second / 6 (eq. lb_energy); the last two are the tau and gamma
    derivatives (times 1 and -1/2) of <w, grad_raw E>."""
    z = np.zeros_like(psi) if w is None else w
    return np.array([np.mean(psi**2), np.mean(psi**3), np.mean(z * psi), np.mean(z * psi**2)])


def param_grad(psi: np.ndarray, w: Optional[np.ndarray] = None) -> np.ndarray:
    """[dE/dtau, dE/dgamma, d<w, grad_raw E>/dtau, d<w, grad_raw E>/dgamma] for E of
    eq. lb_energy (tau/2 psi^2 and -gamma/6 psi^3 are the only terms in tau and
    gamma; grad_raw E has tau psi / N and -gamma psi^2 / (2 N)); <w, .> sums over
    the grid points."""
    z = np.zeros_like(psi) if w is None else w
    return np.array([np.mean(psi**2) / 2.0, -np.mean(psi**3) / 6.0, np.mean(z * psi), -np.mean(z * psi**2) / 2.0])


def param_grad_vjp(psi: np.ndarray, a: float, b: float) -> np.ndarray:
    """Gradient with respect to the grid values of a dE/dtau + b dE/dgamma."""
    return (a * psi - b * psi**2 / 2.0) / psi.size


def hessvec_phys(m: Model, psi: np.ndarray, v: np.ndarray) -> np.ndarray:
    return inv(hessvec(m, psi, project(fwd(v))))


# ---------------------------------------------------------------------------
# Dense operators on tiny grids
# ---------------------------------------------------------------------------


def dense_L(grid: Grid, xi: float = 1.0, q: float = 1.0) -> np.ndarray:
    """Matrix of v -> F_N^{-1} Lambda F_N v built from the explicit DFT matrix (no FFT)."""
    N = grid.N
    xs = np.stack(np.meshgrid(*[np.arange(m) for m in grid.n], indexing="ij"), -1).reshape(N, grid.dim)
    phase = np.zeros((N, N))
    for a in range(grid.dim):
        phase += np.outer(xs[:, a], xs[:, a]) / grid.n[a]
    W = np.exp(-2j * math.pi * phase)  # W[k, x]
    lam = Lambda(grid, xi, q).reshape(N)
    L = (W.conj().T * lam) @ W / N
    return L.real


def zero_mean_basis(N: int) -> np.ndarray:
    """Orthonormal basis Q (N x (N-1)) of the zero-mean subspace 1^perp (Householder reflection)."""
    e = np.ones(N) / math.sqrt(N)
    u = e.copy()
    u[0] += 1.0
    u /= np.linalg.norm(u)
    Hh = np.eye(N) - 2.0 * np.outer(u, u)  # maps e1 -> -e
    return Hh[:, 1:]


def dense_hessian(m: Model, psi: np.ndarray, L: Optional[np.ndarray] = None) -> Tuple[np.ndarray, np.ndarray]:
    """(H_sub, Q): Hessian restricted to 1^perp in an orthonormal basis Q of it.

    With e_x = sqrt(N) delta_x (orthonormal for <.,.>_N) the matrix of the
    operator L + diag(Gamma') in that basis is its plain standard-basis matrix.
    The constant mode is excluded by Q (it would add a spurious zero eigenvalue).
    """
    if L is None:
        L = dense_L(m.grid, m.xi, m.q)
    Hfull = L + np.diag(Gamma_p(psi, m.tau, m.gamma).reshape(-1))
    Q = zero_mean_basis(m.grid.N)
    return Q.T @ Hfull @ Q, Q


def hessian_fft_columns(m: Model, psi: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Same as dense_hessian but the operator columns come from ``hessvec_phys`` (larger grids)."""
    N = m.grid.N
    Q = zero_mean_basis(N)
    cols = np.empty((N, N - 1))
    for j in range(N - 1):
        cols[:, j] = hessvec_phys(m, psi, Q[:, j].reshape(m.grid.n)).reshape(N)
    Hs = Q.T @ cols
    return 0.5 * (Hs + Hs.T), Q


def hessian_eigs(m: Model, psi: np.ndarray, dense: bool = True) -> np.ndarray:
    """Ascending eigenvalues sigma_1 <= ... <= sigma_{N-1} of H on 1^perp."""
    Hs, _ = dense_hessian(m, psi) if dense else hessian_fft_columns(m, psi)
    return np.linalg.eigvalsh(Hs)


# ---------------------------------------------------------------------------
# Trust-region subproblem: global minimiser by eigendecomposition
# (Section 3.1, optimality conditions tr_subproblem_optimal_condition)
# ---------------------------------------------------------------------------


@dataclass
class DenseTRS:
    d: np.ndarray
    lam: float
    hard_case: bool
    sigma1: float


def trs_global_dense(Hs: np.ndarray, gs: np.ndarray, r: float) -> DenseTRS:
    """Global minimiser of g^T d + d^T H d / 2 on ||d|| <= r (Conn-Gould-Toint Cor. 7.2.2).

    H = V diag(sigma) V^T. If H is positive definite and ||H^{-1} g|| <= r the
    interior Newton point is optimal with lambda = 0. Otherwise lambda >
    max(0, -sigma_1) solves ||(H + lambda I)^{-1} g|| = r, found by bisection
    on this strictly decreasing function; if no such lambda exists (g has no
    component on the sigma_1 eigenspace and the shifted solution is short),
    this is the hard case: lambda = -sigma_1 and an eigenvector of sigma_1 is
    added to reach the boundary.
    """
    sig, V = np.linalg.eigh(Hs)
    gt = V.T @ gs
    s1 = float(sig[0])

    def dnorm(lam):
        return float(np.linalg.norm(gt / (sig + lam)))

    if s1 > 0:
        d0 = -gt / sig
        if np.linalg.norm(d0) <= r:
            return DenseTRS(V @ d0, 0.0, False, s1)
    lo = max(0.0, -s1)
    # hard case test: components on the bottom eigenspace
    tol_deg = 1e-12 * max(1.0, abs(s1))
    bottom = np.abs(sig - s1) <= tol_deg
    gb = float(np.linalg.norm(gt[bottom]))
    if gb <= 1e-14 * max(1.0, np.linalg.norm(gt)) and lo > 0:
        rest = ~bottom
        dr = np.zeros_like(gt)
        dr[rest] = -gt[rest] / (sig[rest] - s1)
        nr = float(np.linalg.norm(dr))
        if nr <= r:
            dr[np.argmax(bottom)] = math.sqrt(max(r * r - nr * nr, 0.0))
            return DenseTRS(V @ dr, lo, True, s1)
    hi = lo + 1.0
    while dnorm(hi) > r:
        hi = lo + 2.0 * (hi - lo)
    for _ in range(300):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if dnorm(mid) > r:
            lo = mid
        else:
            hi = mid
    lam = 0.5 * (lo + hi)
    return DenseTRS(V @ (-gt / (sig + lam)), lam, False, s1)


# ---------------------------------------------------------------------------
# Algorithm 3: adaptive implicit-explicit iteration for the subproblem
# ---------------------------------------------------------------------------


@dataclass
class SubOpts:
    eta: float = 0.1  # step size (Section 4 value)
    eps_sub: float = 1e-13  # stop when ||g + (H + lambda I) d|| < eps_sub
    # ... or < eps_sub_rel * ||g||: a relative floor for iterations whose
    # transforms run in single precision, where an absolute 1e-13 lies below
    # rounding (0 disables it; the paper's test is the absolute one)
    eps_sub_rel: float = 0.0
    max_inner: int = 10000
    max_newton: int = 100
    newton_rtol: float = 1e-14  # stop Newton when phi - r^2 <= newton_rtol * r^2
    newton_steptol: float = 1e-15  # or |delta lambda| <= newton_steptol * max(1, lambda)


@dataclass
class SubResult:
    d: np.ndarray
    lam: float
    iters: int
    newton_iters: int
    resid: float
    converged: bool
    history: List[dict] = field(default_factory=list)


def newton_lambda(bsq: np.ndarray, D: np.ndarray, eta: float, r: float, opts: SubOpts) -> Tuple[float, int]:
    """lambda_{k+1} by the rule lambda_update_rule (Section 3.2).

    phi(lambda) = sum_i [b]_i^2 / (1 + eta (D_ii + lambda))^2 is decreasing; if
    phi(0) <= r^2 then lambda = 0, else Newton's method from lambda_0 = 0 on
    phi(lambda) = r^2. Newton from below on this convex decreasing function
    increases monotonically and never reaches phi <= r^2 exactly, so it stops
    when phi - r^2 <= newton_rtol r^2 or the step is below newton_steptol.
    ``bsq`` holds |b_i|^2 over the modes i != 0, ``D`` the matching D_ii.
    """
    r2 = r * r

    def phi_and_dphi(lam):
        den = 1.0 + eta * (D + lam)
        phi = float(np.sum(bsq / den**2))
        dphi = float(np.sum(-2.0 * eta * bsq / den**3))
        return phi, dphi

    phi0, dphi = phi_and_dphi(0.0)
    if phi0 <= r2:
        return 0.0, 0
    lam = 0.0
    phi = phi0
    it = 0
    while it < opts.max_newton:
        if phi - r2 <= opts.newton_rtol * r2:
            break
        step = (phi - r2) / dphi
        new = lam - step
        it += 1
        if abs(new - lam) <= opts.newton_steptol * max(1.0, abs(lam)):
            lam = new
            break
        lam = new
        phi, dphi = phi_and_dphi(lam)
    return lam, it


def imex_subproblem(
    m: Model,
    psi: np.ndarray,
    g_hat: np.ndarray,
    r: float,
    opts: SubOpts = SubOpts(),
    d0: Optional[np.ndarray] = None,
    record: bool = False,
) -> SubResult:
    """Algorithm 3 (adaptive implicit-explicit iteration) in Psi_hat coordinates.

    Input: step size eta, radius r, gradient g, H = D + T, initial value
    d_0 = -r g / ||g|| (or a caller-supplied feasible d_0 for the hard case,
    Remark hard_case_strategy), tolerance eps_sub. Each iteration:
      b_k = d_k - eta (g + T d_k)                       (eq. imex-scheme)
      lambda_{k+1} from phi_k (eq. lambda_update_rule, Newton from 0)
      d_{k+1} = b_k / (1 + eta (D + lambda_{k+1}))     (diagonal solve)
      return d_{k+1} when ||g + (H + lambda_{k+1} I) d_{k+1}|| < eps_sub.
    """
    D = project(m.Lam)  # D = P grad^2 G P^T; the k = 0 entry is not a variable
    mask = np.ones(m.grid.n, dtype=bool)
    mask[m.grid.zero] = False
    if d0 is None:
        gn = norm(g_hat)
        d = -r * g_hat / gn
    else:
        d = project(d0.copy())
    hist = []
    newton_total = 0
    lam = 0.0
    resid = float("inf")
    k = 0
    converged = False
    tol = max(opts.eps_sub, opts.eps_sub_rel * norm(g_hat))
    while k < opts.max_inner:
        Td = T_apply(m, psi, d)
        b = d - opts.eta * (g_hat + Td)
        b = project(b)
        lam, nit = newton_lambda(np.abs(b[mask]) ** 2, D[mask], opts.eta, r, opts)
        newton_total += nit
        d_new = b / (1.0 + opts.eta * (D + lam))
        d_new = project(d_new)
        res_vec = g_hat + hessvec(m, psi, d_new) + lam * d_new
        resid = norm(res_vec)
        k += 1
        if record:
            hist.append(dict(k=k, lam=lam, dnorm=norm(d_new), resid=resid, f=model_value(m, psi, g_hat, d_new), step=norm(d_new - d)))
        d = d_new
        if resid < tol:
            converged = True
            break
    return SubResult(d, lam, k, newton_total, resid, converged, hist)


def model_value(m: Model, psi: np.ndarray, g_hat: np.ndarray, d_hat: np.ndarray) -> float:
    """f(d) = g^T d + d^T H d / 2 (eq. tr_subproblem)."""
    return dot(g_hat, d_hat) + 0.5 * dot(d_hat, hessvec(m, psi, d_hat))


# ---------------------------------------------------------------------------
# Algorithms 1 and 2: IMEX-TR outer loop (TRACE framework) with CONTRACT
# ---------------------------------------------------------------------------


@dataclass
class TROpts:
    # Section 4 parameter values
    theta: float = 1e-4
    gamma_c: float = 0.5
    gamma_e: float = 2.0
    gamma_lambda: float = 1.5
    mu_lo: float = 1.0
    mu_hi: float = 1e5
    mu0: float = 1.0
    r0: float = 1.0
    nu0: float = 5.0
    eps: float = 1e-10
    eta: float = 0.1
    eps_sub: float = 1e-13
    eps_sub_rel: float = 0.0  # relative floor of the subproblem stop test (SubOpts.eps_sub_rel)
    # readings where the paper leaves a choice open
    grad_norm: str = "inf"  # "inf" (Algorithm 1) or "l2"
    eta_rule: str = "safe"  # "safe": min(eta, 0.9 / max|Gamma'|) per outer iteration; "fixed": eta
    rho_numerator: str = "taylor"  # "taylor" (exact quartic expansion) or "direct" (E(v) - E(v+s))
    contract_else_old_step: bool = False  # False: r = gamma_C ||s|| with the new s, as printed
    max_outer: int = 500
    max_inner: int = 10000
    max_newton: int = 100
    cg_rtol: float = 1e-12
    cg_maxiter: int = 1000
    cg_precond_shift: float = 1.0  # CONTRACT's CG preconditioned by (Lambda + lam~ + c)^-1; 0: plain CG
    nu_tol: float = 1e-12  # ||s_j|| = nu_j tested as | ||s_j|| - nu_j | <= nu_tol nu_j


@dataclass
class TRResult:
    psi: np.ndarray
    energy: float
    gnorm: float
    gnorm_inf: float
    outer: int
    inner_total: int
    converged: bool
    history: List[dict] = field(default_factory=list)
    sub_capped: int = 0  # subproblems that stopped at max_inner before their stop test held


def delta_energy_taylor(m: Model, psi: np.ndarray, g_hat: np.ndarray, s_hat: np.ndarray) -> float:
    """E(psi) - E(psi + s) by the exact expansion of the quartic energy.

    E(psi + s) - E(psi) = <g, s> + 1/2 sum_k Lambda_k |s_k|^2
        + (1/N) sum_x [Gamma'(psi) s^2 / 2 + (psi - gamma) s^3 / 6 + s^4 / 24]
    (F''' = psi - gamma, F'''' = 1; s has zero mean so the projected gradient
    gives the same first-order term). Identical to the direct difference in
    exact arithmetic, without its cancellation for small steps.
    """
    s = inv(s_hat)
    quad = 0.5 * float(np.sum(m.Lam * np.abs(s_hat) ** 2))
    pw = float(np.mean(Gamma_p(psi, m.tau, m.gamma) * s**2 / 2.0 + (psi - m.gamma) * s**3 / 6.0 + s**4 / 24.0))
    return -(dot(g_hat, s_hat) + quad + pw)


def cg_shifted(m: Model, psi: np.ndarray, g_hat: np.ndarray, lam: float, rtol: float, maxiter: int,
               precond_shift: float = 0.0) -> Tuple[np.ndarray, int]:
    """Conjugate gradients for (H + lam I) s = -g (H + lam I positive definite),
    stopped when ||r|| <= rtol ||g|| or after maxiter steps.

    With precond_shift c > 0 the textbook preconditioned form, with the
    diagonal M = (Lambda + lam + c)^(-1): the interaction part of H + lam I,
    which spans the stiff range of its spectrum (the bulk part is bounded by
    max |Gamma'|). The system solved is the same; c = 0 is plain CG.
    """
    b = -g_hat
    x = np.zeros_like(g_hat)
    res = b.copy()
    Minv = project(1.0 / (m.Lam + lam + precond_shift)) if precond_shift > 0 else None
    z = Minv * res if Minv is not None else res
    p = z.copy()
    rz = dot(res, z)
    rr = dot(res, res)
    bn = math.sqrt(rr)
    it = 0
    while it < maxiter and math.sqrt(rr) > rtol * bn:
        Ap = hessvec(m, psi, p) + lam * p
        alpha = rz / dot(p, Ap)
        x = x + alpha * p
        res = res - alpha * Ap
        rr = dot(res, res)
        z = Minv * res if Minv is not None else res
        rz_new = dot(res, z) if Minv is not None else rr
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return project(x), it


def contract(m: Model, psi: np.ndarray, g_hat: np.ndarray, r: float, mu: float, s_hat: np.ndarray, lam: float, o: TROpts) -> Tuple[float, dict]:
    """Algorithm 2 (CONTRACT): the new radius from a shifted Newton system (H + lam~ I) s = -g."""
    sn = norm(s_hat)
    info = {}
    if lam < o.mu_lo * sn:
        lam_hat = lam + math.sqrt(o.mu_lo * norm(g_hat))
        s_new, it = cg_shifted(m, psi, g_hat, lam_hat, o.cg_rtol, o.cg_maxiter, o.cg_precond_shift)
        info.update(contract_branch="hat", cg=it)
        if lam_hat / norm(s_new) <= o.mu_hi:
            return norm(s_new), info
        # find lam~ in (lam, lam_hat) with mu_lo <= lam~ / ||s(lam~)|| <= mu_hi;
        # lam~ / ||s(lam~)|| increases with lam~, so bisect
        lo, hi = lam, lam_hat
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            s_mid, it = cg_shifted(m, psi, g_hat, mid, o.cg_rtol, o.cg_maxiter, o.cg_precond_shift)
            ratio = mid / norm(s_mid)
            if ratio < o.mu_lo:
                lo = mid
            elif ratio > o.mu_hi:
                hi = mid
            else:
                info.update(contract_branch="bisect", lam_tilde=mid)
                return norm(s_mid), info
        return norm(s_mid), info
    lam_t = o.gamma_lambda * lam
    s_new, it = cg_shifted(m, psi, g_hat, lam_t, o.cg_rtol, o.cg_maxiter, o.cg_precond_shift)
    info.update(contract_branch="gamma_lambda", cg=it)
    if norm(s_new) >= o.gamma_c * sn:
        return norm(s_new), info
    return (o.gamma_c * sn if o.contract_else_old_step else o.gamma_c * norm(s_new)), info


def safe_eta(m: Model, psi: np.ndarray, o: TROpts) -> float:
    if o.eta_rule == "fixed":
        return o.eta
    gmax = float(np.max(np.abs(Gamma_p(psi, m.tau, m.gamma))))
    return min(o.eta, 0.9 / gmax) if gmax > 0 else o.eta


def mu_before_ratio(o: TROpts, j: int, rho_prev: Optional[float], mu: float, lam: float, sn: float) -> float:
    """Algorithm 1, after the subproblem: if j > 0 and rho_{j-1} < theta then
    mu_j = max(mu_{j-1}, lambda_j / ||s_j||), else mu_j = mu_{j-1}."""
    if j > 0 and rho_prev is not None and rho_prev < o.theta:
        return max(mu, lam / sn)
    return mu


def outer_branch(o: TROpts, rho: float, lam: float, sn: float, r: float, nu: float, mu: float,
                 contract_radius: Callable[[], float]) -> Tuple[str, float, float, float]:
    """Algorithm 1 from the ratio rho_j on: returns (branch, r_{j+1}, nu_{j+1}, mu_{j+1}).

    accept   if rho_j >= theta and (lambda_j <= mu_j ||s_j|| or ||s_j|| = nu_j):
             nu_{j+1} = max(nu_j, gamma_E ||s_j||), r_{j+1} = min(nu_{j+1}, max(r_j, gamma_E ||s_j||)),
             mu_{j+1} = max(mu_j, lambda_j / ||s_j||);
    contract if rho_j < theta: r_{j+1} = CONTRACT(...) (Algorithm 2), nu and mu carried over;
    expand   otherwise: r_{j+1} = min(nu_{j+1}, lambda_j / mu_j), nu and mu carried over.
    The caller moves v to v + s_j on "accept". lambda_j <= mu_j ||s_j|| is tested
    as lambda_j / ||s_j|| <= mu_j: right after a contraction mu_j was raised to
    exactly lambda_j / ||s_j||, and the two sides must then compare equal, not
    by the rounding of (lambda_j / ||s_j||) ||s_j||.
    """
    on_nu = abs(sn - nu) <= o.nu_tol * nu
    if rho >= o.theta and (lam / sn <= mu or on_nu):
        nu_new = max(nu, o.gamma_e * sn)
        return "accept", min(nu_new, max(r, o.gamma_e * sn)), nu_new, max(mu, lam / sn)
    if rho < o.theta:
        return "contract", contract_radius(), nu, mu
    return "expand", min(nu, lam / mu), nu, mu


def imex_tr_solve(
    m: Model,
    psi0: np.ndarray,
    o: TROpts = TROpts(),
    record: bool = True,
    d0_provider: Optional[Callable[[int, float, np.ndarray, np.ndarray], Optional[np.ndarray]]] = None,
) -> TRResult:
    """Algorithm 1 (IMEX-TR): TRACE outer loop with Algorithm 3 as subproblem solver.

    The iterate is psi = P^T v (zero mean). Per iteration j:
      g_j = grad E_bar(v_j); return if ||g_j|| < eps;
      (s_j, lambda_j) from Algorithm 3 with radius r_j;
      mu_j from ``mu_before_ratio``;
      rho_j = (E_bar(v_j) - E_bar(v_j + s_j)) / ||s_j||^3;
      the branch and r_{j+1}, nu_{j+1}, mu_{j+1} from ``outer_branch``.
    """
    psi = psi0 - psi0.mean()
    r, nu, mu = o.r0, o.nu0, o.mu0
    rho_prev = None
    hist = []
    inner_total = 0
    sub_capped = 0
    E = energy(m, psi)
    g = gradient(m, psi)
    for j in range(o.max_outer):
        gn2, gninf = norm(g), norm_inf(g)
        gtest = gninf if o.grad_norm == "inf" else gn2
        if gtest < o.eps:
            return TRResult(psi, E, gn2, gninf, j, inner_total, True, hist, sub_capped)
        eta = safe_eta(m, psi, o)
        sub_opts = SubOpts(eta=eta, eps_sub=o.eps_sub, eps_sub_rel=o.eps_sub_rel, max_inner=o.max_inner,
                           max_newton=o.max_newton)
        d0 = d0_provider(j, r, g, psi) if d0_provider else None
        sub = imex_subproblem(m, psi, g, r, sub_opts, d0=d0)
        inner_total += sub.iters
        sub_capped += 0 if sub.converged else 1
        s_hat, lam = sub.d, sub.lam
        sn = norm(s_hat)
        mu = mu_before_ratio(o, j, rho_prev, mu, lam, sn)
        if o.rho_numerator == "taylor":
            dE = delta_energy_taylor(m, psi, g, s_hat)
        else:
            dE = E - energy(m, psi + inv(s_hat))
        rho = dE / sn**3
        rec = dict(j=j, E=E, gnorm=gn2, gnorm_inf=gninf, r=r, nu=nu, mu=mu, lam=lam, snorm=sn, rho=rho, eta=eta, inner=sub.iters, sub_resid=sub.resid)
        cinfo = {}

        def contract_radius():
            r_new, info = contract(m, psi, g, r, mu, s_hat, lam, o)
            cinfo.update(info)
            return r_new

        branch, r, nu, mu = outer_branch(o, rho, lam, sn, r, nu, mu, contract_radius)
        rec["branch"] = branch
        rec.update(cinfo)
        if branch == "accept":
            psi = psi + inv(s_hat)
            E = energy(m, psi)
            g = gradient(m, psi)
        rho_prev = rho
        if record:
            hist.append(rec)
    return TRResult(psi, E, norm(g), norm_inf(g), o.max_outer, inner_total, False, hist, sub_capped)


# ---------------------------------------------------------------------------
# Lanczos estimate of the smallest Hessian eigenvalue (second-order check)
# ---------------------------------------------------------------------------


def lanczos_min(
    m: Model, psi: np.ndarray, v0_hat: np.ndarray, steps: int, precond_shift: float = 0.0, want_vector: bool = False
):
    """Smallest Ritz value of H after ``steps`` Lanczos steps with full reorthogonalisation.

    Returns (value, residual_norm). Without preconditioning (precond_shift <= 0)
    value is the smallest Ritz value of H and the residual the usual Ritz
    residual |beta_m y_m|. With precond_shift = c > 0 the iteration runs on
    K = S H S, S = diag((Lambda_k + c)^(-1/2)) in Fourier space; K is congruent
    to H (Sylvester: same inertia) and its spectrum is clustered, so the lowest
    Ritz vector y of K converges quickly; the result is the Rayleigh quotient
    rho = <x, Hx>/<x, x> of H at x = S y and ||Hx - rho x|| / ||x||. Either
    value bounds sigma_1 from above; it is an estimate, not a certificate.
    With want_vector the unit Ritz vector (x / ||x||, Psi_hat coordinates) is
    returned as a third value.
    """
    if precond_shift > 0:
        Sd = np.where(np.arange(m.Lam.size).reshape(m.Lam.shape) == 0, 0.0, 1.0 / np.sqrt(m.Lam + precond_shift))

        def op(v):
            return Sd * hessvec(m, psi, Sd * v)

    else:
        Sd = None

        def op(v):
            return hessvec(m, psi, v)

    q = project(v0_hat)
    q = q / norm(q)
    Qs = [q]
    alpha, beta = [], []
    b = 0.0
    q_prev = np.zeros_like(q)
    for i in range(steps):
        w = op(q) - b * q_prev
        a = dot(w, q)
        w = w - a * q
        for qq in Qs:  # full reorthogonalisation
            w = w - dot(w, qq) * qq
        alpha.append(a)
        b = norm(w)
        beta.append(b)
        if i == steps - 1 or b < 1e-300:
            break
        q_prev = q
        q = w / b
        Qs.append(q)
    k = len(alpha)
    Tm = np.diag(alpha) + np.diag(beta[: k - 1], 1) + np.diag(beta[: k - 1], -1)
    ev, evec = np.linalg.eigh(Tm)
    y = sum(evec[i, 0] * Qs[i] for i in range(k))
    if Sd is None:
        out = (float(ev[0]), float(abs(beta[k - 1] * evec[k - 1, 0])))
        return out + (y / norm(y),) if want_vector else out
    x = Sd * y
    Hx = hessvec(m, psi, x)
    rho = dot(x, Hx) / dot(x, x)
    out = (float(rho), float(norm(Hx - rho * x) / norm(x)))
    return out + (x / norm(x),) if want_vector else out


# ---------------------------------------------------------------------------
# Random initial point for nearly hard subproblems (Remark on the hard case,
# Section 3.2; Section 4.3)
# ---------------------------------------------------------------------------
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_M32 = np.uint64(0xFFFFFFFF)


def _mulhilo64(a: np.ndarray, b: int) -> Tuple[np.ndarray, np.ndarray]:
    """High and low 64-bit words of a * b (a: uint64 array, b: constant), from 32-bit halves."""
    s32 = np.uint64(32)
    a_lo, a_hi = a & _M32, a >> s32
    b_lo, b_hi = np.uint64(b & 0xFFFFFFFF), np.uint64(b >> 32)
    ll, hl, lh, hh = a_lo * b_lo, a_hi * b_lo, a_lo * b_hi, a_hi * b_hi
    cross = (ll >> s32) + (hl & _M32) + (lh & _M32)
    lo = (ll & _M32) | ((cross & _M32) << s32)
    hi = hh + (hl >> s32) + (lh >> s32) + (cross >> s32)
    return hi, lo


def philox4x64(counter: Sequence[np.ndarray], key: Tuple[int, int], rounds: int = 10) -> List[np.ndarray]:
    """Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC'11): a counter-based
    generator; each round multiplies words 0 and 2 by fixed constants, mixes the
    high/low halves with words 1, 3 and the key, and bumps the key by Weyl
    constants."""
    c = [np.asarray(x, dtype=np.uint64) for x in counter]
    n = max(x.size for x in c)
    c = [np.broadcast_to(x, (n,)).copy() for x in c]
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    with np.errstate(over="ignore"):
        for _ in range(rounds):
            hi0, lo0 = _mulhilo64(c[0], 0xD2E7470EE14C6C93)
            hi1, lo1 = _mulhilo64(c[2], 0xCA5A826395121157)
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
            k0 = k0 + np.uint64(0x9E3779B97F4A7C15)
            k1 = k1 + np.uint64(0xBB67AE8584CAA73B)
    return c


def unit_open(w: np.ndarray) -> np.ndarray:
    """Uniform in (0, 1) from the top 53 bits of a 64-bit word."""
    return ((w >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0**-53


def ball_point(shape: Tuple[int, ...], r: float, seed: int, draw: int) -> np.ndarray:
    """A zero-mean field uniformly distributed in the ball ||d|| <= r of the
    (N-1)-dimensional zero-mean subspace (||.|| = RMS): z_x standard normal
    (Box-Muller from Philox4x64-10 at counter (x, 0, 0, 0), key (seed, draw)),
    projected to zero mean and scaled to radius r u^(1/(N-1)), u uniform from
    counter (0, 1, 0, 0)."""
    N = int(np.prod(shape))
    idx = np.arange(N, dtype=np.uint64)
    w = philox4x64([idx, 0, 0, 0], (seed, draw))
    z = np.sqrt(-2.0 * np.log(unit_open(w[0]))) * np.cos(2.0 * math.pi * unit_open(w[1]))
    z = z - z.mean()
    u = float(unit_open(philox4x64([0, 1, 0, 0], (seed, draw))[0])[0])
    return (r * u ** (1.0 / (N - 1)) / math.sqrt(np.mean(z * z)) * z).reshape(shape)


def hard_case_d0_provider(m: Model, seed: int = 0, tol: float = 1e-12, lanczos_steps: int = 30,
                          precond_shift: float = 1.0, log: Optional[list] = None):
    """d0 rule for Algorithm 3 inside Algorithm 1: when the subproblem is
    nearly hard, i.e. H has a negative eigenvalue sigma_1 and its unit
    eigenvector xi has |g^(1)| = |<xi, g>| <= tol, start from ball_point(r)
    (draw 2j at outer iteration j) instead of -r g/||g||. sigma_1 and xi are
    Lanczos estimates from the start vector ball_point(1) of draw 2j + 1."""

    def provider(j: int, r: float, g_hat: np.ndarray, psi: np.ndarray) -> Optional[np.ndarray]:
        v0 = fwd(ball_point(m.grid.n, 1.0, seed, 2 * j + 1))
        sig, _, xi = lanczos_min(m, psi, v0, lanczos_steps, precond_shift, want_vector=True)
        g1 = dot(g_hat, xi)
        hard = sig < 0 and abs(g1) <= tol
        if log is not None:
            log.append(dict(j=j, sigma1=sig, g1=g1, hard=hard))
        return fwd(ball_point(m.grid.n, r, seed, 2 * j)) if hard else None

    return provider
