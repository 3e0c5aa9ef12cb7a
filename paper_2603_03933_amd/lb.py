"""ctypes binding of the C ABI in include/lb.h (argument marshalling only).

Every computation runs in liblbtr.so on the GPU. Arrays are torch tensors on a
ROCm device, float64, contiguous; their data pointers and torch's current HIP
stream are passed straight through. There is no CPU fallback: a missing
library or a CPU tensor raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch  # imported first: its HIP runtime is the one the library binds to

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbtr.so")

LB_OK = 0
LB_NOT_CONVERGED = 1
LB_FP64 = 0
LB_FP32 = 1


class LbGrid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("box", C.c_double * 3)]


class LbParams(C.Structure):
    _fields_ = [("tau", C.c_double), ("gamma", C.c_double), ("xi", C.c_double), ("q", C.c_double)]


class LbSubOpts(C.Structure):
    _fields_ = [
        ("eta", C.c_double),
        ("eps_sub", C.c_double),
        ("eps_sub_rel", C.c_double),
        ("max_inner", C.c_int),
        ("max_newton", C.c_int),
        ("newton_rtol", C.c_double),
        ("newton_steptol", C.c_double),
        ("poll_every", C.c_int),
        ("newton_phi", C.c_int),
        ("newton_direct", C.c_int),
        ("single_workgroup", C.c_int),
        ("graph", C.c_int),
        ("fused_newton", C.c_int),
    ]


class LbSubInfo(C.Structure):
    _fields_ = [
        ("lambda_", C.c_double),
        ("resid", C.c_double),
        ("dnorm", C.c_double),
        ("gnorm", C.c_double),
        ("iters", C.c_int),
        ("newton_iters", C.c_int),
        ("newton_direct", C.c_int),
        ("status", C.c_int),
    ]


class LbTrOpts(C.Structure):
    _fields_ = [
        ("theta", C.c_double),
        ("gamma_c", C.c_double),
        ("gamma_e", C.c_double),
        ("gamma_lambda", C.c_double),
        ("mu_lo", C.c_double),
        ("mu_hi", C.c_double),
        ("mu0", C.c_double),
        ("r0", C.c_double),
        ("nu0", C.c_double),
        ("eps", C.c_double),
        ("grad_norm_inf", C.c_int),
        ("eta", C.c_double),
        ("eta_safe", C.c_int),
        ("rho_taylor", C.c_int),
        ("contract_else_old_step", C.c_int),
        ("nu_tol", C.c_double),
        ("max_outer", C.c_int),
        ("sub", LbSubOpts),
        ("cg_rtol", C.c_double),
        ("cg_maxiter", C.c_int),
        ("verbose", C.c_int),
        ("hard_case", C.c_int),
        ("hard_tol", C.c_double),
        ("hard_lanczos_steps", C.c_int),
        ("hard_precond_shift", C.c_double),
        ("seed", C.c_ulonglong),
        ("cg_precond_shift", C.c_double),
        ("capped_reject", C.c_int),
    ]


class LbTrInfo(C.Structure):
    _fields_ = [
        ("energy", C.c_double),
        ("gnorm", C.c_double),
        ("gnorm_inf", C.c_double),
        ("outer", C.c_int),
        ("inner_total", C.c_int),
        ("cg_total", C.c_int),
        ("accepted", C.c_int),
        ("contracted", C.c_int),
        ("expanded", C.c_int),
        ("status", C.c_int),
        ("hard_cases", C.c_int),
        ("newton_total", C.c_int),
        ("newton_direct", C.c_int),
        ("sub_capped", C.c_int),
    ]


class LBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"liblbtr error {code}: {msg}")
        self.code = code


_lib = None

_P = C.c_void_p
_D = C.c_double
_I = C.c_int
_SIGS = {
    "lb_version": (_I, []),
    "lb_last_error": (C.c_char_p, []),
    "lb_sub_opts_default": (None, [C.POINTER(LbSubOpts)]),
    "lb_tr_opts_default": (None, [C.POINTER(LbTrOpts)]),
    "lb_plan_create": (_I, [C.POINTER(_P), C.POINTER(LbGrid), _I, _I, _P]),
    "lb_plan_destroy": (_I, [_P]),
    "lb_plan_set_stream": (_I, [_P, _P]),
    "lb_plan_set_lattice": (_I, [_P, C.POINTER(_D)]),
    "lb_plan_workspace_bytes": (C.c_size_t, [_P]),
    "lb_plan_set_timing": (_I, [_P, _I, C.c_char_p]),
    "lb_plan_set_timing_sampled": (_I, [_P, _I, C.c_char_p, _I]),
    "lb_plan_timing_entry": (_I, [_P, _I, C.c_char_p, _I, C.POINTER(C.c_long), C.POINTER(_D)]),
    "lb_energy_grad": (_I, [_P, C.POINTER(LbParams), _P, _P, _P]),
    "lb_hessvec": (_I, [_P, C.POINTER(LbParams), _P, _P, _P, _I]),
    "lb_energy_grad_raw": (_I, [_P, C.POINTER(LbParams), _P, _P, _P]),
    "lb_hessvec_raw": (_I, [_P, C.POINTER(LbParams), _P, _P, _P]),
    "lb_field_moments": (_I, [_P, _P, _P, _P]),
    "lb_param_grad": (_I, [_P, _P, _P, _P]),
    "lb_hessvec_noalloc": (_I, [C.POINTER(LbGrid), C.POINTER(LbParams), _P, _P, _P, _I, _P]),
    "lb_param_grad_vjp": (_I, [_P, _P, _P, _P]),
    "lb_tr_subproblem": (_I, [_P, C.POINTER(LbParams), _P, _P, _D, C.POINTER(LbSubOpts), _P, _P, C.POINTER(LbSubInfo)]),
    "lb_imex_tr_solve": (_I, [_P, C.POINTER(LbParams), _P, C.POINTER(LbTrOpts), C.POINTER(LbTrInfo)]),
    "lb_shifted_solve": (_I, [_P, C.POINTER(LbParams), _P, _P, _D, _D, _I, _D, _P, C.POINTER(_I)]),
    "lb_lanczos_min": (_I, [_P, C.POINTER(LbParams), _P, _P, _I, _D, C.POINTER(_D), C.POINTER(_D), _P]),
    "lb_random_ball": (_I, [_P, _D, C.c_ulonglong, C.c_ulonglong, _P]),
    "lb_imex_tr_solve_many": (_I, [C.POINTER(_P), C.POINTER(LbParams), C.POINTER(_P), _I, C.POINTER(LbTrOpts), _I, C.POINTER(LbTrInfo), C.POINTER(_I)]),
    "lb_imex_tr_solve_batch": (_I, [_P, C.POINTER(LbParams), _P, C.POINTER(LbTrOpts), C.POINTER(LbTrInfo), C.POINTER(_I)]),
    "lb_plan_autotune": (_I, [_P, C.POINTER(LbParams), _P, _I, C.POINTER(_I)]),
    "lb_plan_set_plane_threads": (_I, [_P, _I]),
    "lb_plan_set_plane_split": (_I, [_P, _I, _I]),
    "lb_plan_set_column_plan": (_I, [_P, _I]),
    "lb_plan_set_hessvec_split": (_I, [_P, _I]),
    "lb_plan_get_variant": (_I, [_P, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I)]),
}


def lib():
    """Load liblbtr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_03933_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise LBError(rc, lib().lb_last_error().decode())
    return rc


def _ptr(t: Optional[torch.Tensor], numel: Optional[int] = None, name: str = "array"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a torch tensor on a ROCm GPU")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class Params:
    tau: float
    gamma: float
    xi: float = 1.0
    q: float = 1.0


def _params_array(params, batch: int):
    if isinstance(params, (Params,)) or hasattr(params, "tau"):
        params = [params] * batch
    params = list(params)
    if len(params) != batch:
        raise ValueError(f"need {batch} parameter sets")
    arr = (LbParams * batch)()
    for i, p in enumerate(params):
        arr[i] = LbParams(float(p.tau), float(p.gamma), float(getattr(p, "xi", 1.0)), float(getattr(p, "q", 1.0)))
    return arr


def sub_opts(**kw) -> LbSubOpts:
    o = LbSubOpts()
    lib().lb_sub_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def tr_opts(**kw) -> LbTrOpts:
    o = LbTrOpts()
    lib().lb_tr_opts_default(C.byref(o))
    sub = kw.pop("sub", None)
    for k, v in kw.items():
        setattr(o, k, v)
    if sub:
        for k, v in sub.items():
            setattr(o.sub, k, v)
    return o


class Plan:
    """A plan for `batch` instances of an n[0] x ... grid on a box (lb_plan_create)."""

    def __init__(self, n: Sequence[int], box: Sequence[float], batch: int = 1, precision: str = "fp64"):
        self.n = tuple(int(x) for x in n)
        self.box = tuple(float(x) for x in box)
        self.dim = len(self.n)
        self.batch = int(batch)
        self.N = math.prod(self.n)
        self.precision = precision
        g = LbGrid()
        g.dim = self.dim
        for a in range(self.dim):
            g.n[a] = self.n[a]
            g.box[a] = self.box[a]
        h = C.c_void_p()
        prec = {"fp64": LB_FP64, "fp32": LB_FP32}[precision]
        _check(lib().lb_plan_create(C.byref(h), C.byref(g), self.batch, prec, _stream()))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().lb_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        _check(lib().lb_plan_set_stream(self._h, _stream()))

    def lb_plan_set_lattice(self, A=None):
        """General Bravais lattice: A (dim x dim, column a = cell vector along grid axis a); None: the box."""
        if A is None:
            _check(lib().lb_plan_set_lattice(self._h, None))
            return
        rows = [[float(x) for x in r] for r in A]
        if len(rows) != self.dim or any(len(r) != self.dim for r in rows):
            raise ValueError(f"lattice matrix must be {self.dim} x {self.dim}")
        arr = (_D * (self.dim * self.dim))(*[x for r in rows for x in r])
        _check(lib().lb_plan_set_lattice(self._h, arr))

    @property
    def workspace_bytes(self) -> int:
        return int(lib().lb_plan_workspace_bytes(self._h))

    def lb_plan_set_timing(self, enable: bool, filter: str = "", every: int = 1):
        """Time the kernels named in `filter` (comma-separated; all when empty), one launch in `every`."""
        self._sync_stream()
        _check(lib().lb_plan_set_timing_sampled(self._h, 1 if enable else 0, filter.encode(), int(every)))

    def timings(self):
        """{kernel name: (launches, total ms)} accumulated since timing was set."""
        out = {}
        buf = C.create_string_buffer(128)
        cnt = C.c_long()
        ms = C.c_double()
        i = 0
        while lib().lb_plan_timing_entry(self._h, i, buf, 128, C.byref(cnt), C.byref(ms)) == 0:
            out[buf.value.decode()] = (cnt.value, ms.value)
            i += 1
        return out

    def lb_plan_autotune(self, params, psi, reps=20):
        """Time the inner iteration's plane-stage variants (both orders, each thread count) and keep the
        fastest; returns its thread count (0: nothing to tune)."""
        self._sync_stream()
        nt = C.c_int()
        _check(lib().lb_plan_autotune(self._h, _params_array(params, self.batch), _ptr(psi, self.N * self.batch, "psi"), int(reps), C.byref(nt)))
        return nt.value

    def lb_plan_set_plane_threads(self, threads):
        """Pin the plane-pass variant (256, 512 or 1024 threads; 0: the built-in choice)."""
        _check(lib().lb_plan_set_plane_threads(self._h, int(threads)))

    def lb_plan_set_plane_split(self, split, threads=0):
        """Inner iteration in the split order with two (1) or four (2) split-plane workgroups per plane, or one
        workgroup per plane (0); threads 0: the built-in thread count."""
        _check(lib().lb_plan_set_plane_split(self._h, int(split), int(threads)))

    def lb_plan_set_hessvec_split(self, split):
        """lb_hessvec in pair-split order (1), one workgroup per plane (0) or the built-in choice (-1)."""
        _check(lib().lb_plan_set_hessvec_split(self._h, int(split)))

    def lb_plan_set_column_plan(self, column_plan):
        """Plan of the inner iteration's axis-0 passes (0: radix 8 first, 1: 4 first, 2: 16 first, 3: 8 first with
        twice the columns per workgroup, one or two parts only)."""
        _check(lib().lb_plan_set_column_plan(self._h, int(column_plan)))

    def lb_plan_get_variant(self):
        """(split, threads, column_plan) of the inner iteration in use."""
        sp, nt, cp = C.c_int(), C.c_int(), C.c_int()
        _check(lib().lb_plan_get_variant(self._h, C.byref(sp), C.byref(nt), C.byref(cp)))
        return sp.value, nt.value, cp.value

    def lb_energy_grad(self, params, psi, energy=None, grad=None, want_grad=True):
        self._sync_stream()
        n = self.N * self.batch
        if energy is None:
            energy = torch.empty(self.batch, dtype=torch.float64, device=psi.device)
        if grad is None and want_grad:
            grad = torch.empty_like(psi)
        _check(lib().lb_energy_grad(self._h, _params_array(params, self.batch), _ptr(psi, n, "psi"), _ptr(energy, self.batch, "energy"), _ptr(grad, n, "grad")))
        return energy, grad

    def lb_hessvec(self, params, psi, v, out=None, project=True):
        self._sync_stream()
        n = self.N * self.batch
        if out is None:
            out = torch.empty_like(v)
        _check(lib().lb_hessvec(self._h, _params_array(params, self.batch), _ptr(psi, n, "psi"), _ptr(v, n, "v"), _ptr(out, n, "hv"), 1 if project else 0))
        return out

    def lb_energy_grad_raw(self, params, psi, energy=None, grad=None):
        self._sync_stream()
        n = self.N * self.batch
        if energy is None:
            energy = torch.empty(self.batch, dtype=torch.float64, device=psi.device)
        if grad is None:
            grad = torch.empty_like(psi)
        _check(lib().lb_energy_grad_raw(self._h, _params_array(params, self.batch), _ptr(psi, n, "psi"), _ptr(energy, self.batch, "energy"), _ptr(grad, n, "grad")))
        return energy, grad

    def lb_hessvec_raw(self, params, psi, v, out=None):
        self._sync_stream()
        n = self.N * self.batch
        if out is None:
            out = torch.empty_like(v)
        _check(lib().lb_hessvec_raw(self._h, _params_array(params, self.batch), _ptr(psi, n, "psi"), _ptr(v, n, "v"), _ptr(out, n, "hv")))
        return out

    def lb_field_moments(self, psi, w=None, out=None):
        self._sync_stream()
        n = self.N * self.batch
        if out is None:
            out = torch.empty(4 * self.batch, dtype=torch.float64, device=psi.device)
        _check(lib().lb_field_moments(self._h, _ptr(psi, n, "psi"), _ptr(w, n, "w"), _ptr(out, 4 * self.batch, "out")))
        return out

    def lb_param_grad(self, psi, w=None, out=None):
        """[dE/dtau, dE/dgamma, d<w, grad_raw E>/dtau, d<w, grad_raw E>/dgamma] per instance (4 * batch)."""
        self._sync_stream()
        n = self.N * self.batch
        if out is None:
            out = torch.empty(4 * self.batch, dtype=torch.float64, device=psi.device)
        _check(lib().lb_param_grad(self._h, _ptr(psi, n, "psi"), _ptr(w, n, "w"), _ptr(out, 4 * self.batch, "out")))
        return out

    def lb_param_grad_vjp(self, psi, ct, out=None):
        """Gradient in psi of ct[2b] dE/dtau + ct[2b+1] dE/dgamma (ct: 2 * batch doubles on the device)."""
        self._sync_stream()
        n = self.N * self.batch
        if out is None:
            out = torch.empty_like(psi)
        _check(lib().lb_param_grad_vjp(self._h, _ptr(psi, n, "psi"), _ptr(ct, 2 * self.batch, "ct"), _ptr(out, n, "out")))
        return out

    def lb_tr_subproblem(self, params, psi, grad, radius, opts: Optional[LbSubOpts] = None, d0=None, out=None):
        self._sync_stream()
        if out is None:
            out = torch.empty_like(psi)
        info = LbSubInfo()
        rc = _check(
            lib().lb_tr_subproblem(
                self._h, _params_array(params, 1), _ptr(psi, self.N, "psi"), _ptr(grad, self.N, "grad"), float(radius),
                C.byref(opts) if opts is not None else None, _ptr(d0, self.N, "d0"), _ptr(out, self.N, "d_out"), C.byref(info),
            )
        )
        return out, info, rc

    def lb_imex_tr_solve(self, params, psi, opts: Optional[LbTrOpts] = None):
        self._sync_stream()
        info = LbTrInfo()
        rc = _check(lib().lb_imex_tr_solve(self._h, _params_array(params, 1), _ptr(psi, self.N, "psi"), C.byref(opts) if opts is not None else None, C.byref(info)))
        return info, rc

    def lb_imex_tr_solve_batch(self, params, psi, opts: Optional[LbTrOpts] = None):
        """Solves of the plan's batch instances together; psi [batch, *grid] updated; returns [(info, status)]."""
        self._sync_stream()
        B = self.batch
        infos = (LbTrInfo * B)()
        st = (_I * B)()
        lib().lb_imex_tr_solve_batch(self._h, _params_array(params, B), _ptr(psi, self.N * B, "psi"),
                                     C.byref(opts) if opts is not None else None, infos, st)
        for k in range(B):
            if st[k] < 0:
                raise LBError(st[k], lib().lb_last_error().decode())
        return [(infos[k], st[k]) for k in range(B)]

    def lb_shifted_solve(self, params, psi, grad, shift, rtol=1e-12, maxiter=1000, out=None, precond_shift=0.0):
        self._sync_stream()
        if out is None:
            out = torch.empty_like(psi)
        it = C.c_int()
        _check(lib().lb_shifted_solve(self._h, _params_array(params, 1), _ptr(psi, self.N, "psi"), _ptr(grad, self.N, "grad"), float(shift), float(rtol), int(maxiter), float(precond_shift), _ptr(out, self.N, "s_out"), C.byref(it)))
        return out, it.value

    def lb_lanczos_min(self, params, psi, v0, steps, precond_shift=0.0, evec=None):
        """(ritz, residual); with evec (a device tensor) also the unit Ritz vector in it."""
        self._sync_stream()
        ritz = C.c_double()
        res = C.c_double()
        _check(lib().lb_lanczos_min(self._h, _params_array(params, 1), _ptr(psi, self.N, "psi"), _ptr(v0, self.N, "v0"), int(steps), float(precond_shift), C.byref(ritz), C.byref(res), _ptr(evec, self.N, "evec")))
        return ritz.value, res.value

    def lb_random_ball(self, radius, seed, draw, out=None, device=None):
        self._sync_stream()
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device=device or torch.device("cuda"))
        _check(lib().lb_random_ball(self._h, float(radius), int(seed), int(draw), _ptr(out, self.N, "d_out")))
        return out


def lb_imex_tr_solve_many(plans, params, psis, opts: Optional[LbTrOpts] = None, workers: int = 4):
    """Concurrent independent jobs (one per plan, each solving its plan's batch);
    params: one entry per instance, job after job; returns [(info, rc)] per instance."""
    n = len(plans)
    if len(psis) != n:
        raise ValueError("plans and psis must have the same length")
    total = sum(pl.batch for pl in plans)
    if len(params) != total:
        raise ValueError(f"need {total} parameter sets (one per instance)")
    for pl in plans:
        pl._sync_stream()
    hp = (_P * n)(*[pl._h for pl in plans])
    pa = (LbParams * total)()
    for i, p in enumerate(params):
        pa[i] = LbParams(float(p.tau), float(p.gamma), float(getattr(p, "xi", 1.0)), float(getattr(p, "q", 1.0)))
    ps = (_P * n)(*[_ptr(x, pl.N * pl.batch, "psi") for x, pl in zip(psis, plans)])
    infos = (LbTrInfo * total)()
    st = (_I * total)()
    _check(lib().lb_imex_tr_solve_many(hp, pa, ps, n, C.byref(opts) if opts is not None else None, int(workers), infos, st))
    return [(infos[i], st[i]) for i in range(total)]


def lb_hessvec_noalloc(n: Sequence[int], box: Sequence[float], params, psi, v, out=None, project=True):
    """Hessian-vector product of one FP64 instance with the library's fixed
    workspace: no plan and no device allocation by the library (out is
    allocated here by torch when not given)."""
    g = LbGrid()
    g.dim = len(n)
    for a in range(g.dim):
        g.n[a] = int(n[a])
        g.box[a] = float(box[a])
    N = math.prod(int(x) for x in n)
    if out is None:
        out = torch.empty_like(v)
    _check(lib().lb_hessvec_noalloc(C.byref(g), _params_array(params, 1), _ptr(psi, N, "psi"), _ptr(v, N, "v"),
                                    _ptr(out, N, "hv"), 1 if project else 0, _stream()))
    return out


def exported_symbols():
    """Names of the C entry points this binding knows about."""
    return sorted(_SIGS)
