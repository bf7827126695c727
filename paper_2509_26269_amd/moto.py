"""Python binding of libmoto.so (argument marshalling only).

Each function has the name of the C entry point it calls and takes torch
tensors that already live on the GPU; every step of the computation runs in
the HIP kernels of the library.  There is no CPU fallback: a missing library
raises at import of the first call.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmoto.so")

MOTO_F32, MOTO_F64 = 0, 1
MOTO_AMBIENT, MOTO_FRAME = 0, 1
MAX_SHELLS = 36

MOTO_ASYNC = 1  # option flag: no host synchronisation, outcome in device memory
SADDLE = CONVERGED = 0
NOT_CONVERGED, DEGENERATE, HIGHER_INDEX, NAN, BREAKDOWN = 1, 2, 3, 4, 5
STATUS_NAMES = {0: "SADDLE/CONVERGED", 1: "NOT_CONVERGED", 2: "DEGENERATE", 3: "HIGHER_INDEX", 4: "NAN",
                5: "BREAKDOWN"}


class MotoError(RuntimeError):
    pass


class _Ham(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32), ("n_shells", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("J", ctypes.c_double * MAX_SHELLS),
                ("D", ctypes.c_double * MAX_SHELLS), ("K", ctypes.c_double), ("B", ctypes.c_double * 3)]


class EigOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("guard", ctypes.c_int32),
                ("warm", ctypes.c_int32), ("check_every", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("use_graph", ctypes.c_int32), ("flags", ctypes.c_int32)]


class LanczosOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("m_max", ctypes.c_int32), ("keep", ctypes.c_int32),
                ("max_restarts", ctypes.c_int32), ("warm", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("use_graph", ctypes.c_int32), ("block", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("n_hvp", ctypes.c_int64)]


class StepOpts(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("mem", ctypes.c_int32), ("theta_max", ctypes.c_double),
                ("alpha0", ctypes.c_double), ("sy_min", ctypes.c_double), ("tau_F", ctypes.c_double)]


class DescendOpts(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("tau_F", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("step", StepOpts), ("eig", EigOpts),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class DescendResult(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int32), ("iters", ctypes.c_int32), ("E", ctypes.c_double),
                ("Q", ctypes.c_double), ("fnorm", ctypes.c_double), ("lambda1", ctypes.c_double)]


class SearchOpts(ctypes.Structure):
    _fields_ = [("tau_F", ctypes.c_double), ("tau_lam", ctypes.c_double), ("k", ctypes.c_int32),
                ("k_cert", ctypes.c_int32), ("k_reflect", ctypes.c_int32), ("max_outer", ctypes.c_int32),
                ("step", StepOpts), ("eig", EigOpts)]


class SearchResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("n_hvp", ctypes.c_int64),
                ("E", ctypes.c_double), ("fnorm", ctypes.c_double), ("lambda1", ctypes.c_double),
                ("lambda2", ctypes.c_double)]


class ExplorerOpts(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("reserved", ctypes.c_int32), ("Q_target", ctypes.c_double),
                ("eig", EigOpts)]


class ExplorerResult(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("lambda1", ctypes.c_double), ("lambda2", ctypes.c_double),
                ("gap", ctypes.c_double), ("Q", ctypes.c_double), ("violation", ctypes.c_double),
                ("l1_sum", ctypes.c_double), ("l1_min", ctypes.c_double), ("status", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("n_hvp", ctypes.c_int64)]


_lib = None
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_i32 = ctypes.c_int32


def lib():
    """Load libmoto.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MotoError(f"{LIB_PATH} not found: build it with `python -m paper_2509_26269_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "moto_plan_create": (_i32, [ctypes.POINTER(_Ham), ctypes.POINTER(_vp)]),
        "moto_plan_destroy": (_i32, [_vp]),
        "moto_status_string": (ctypes.c_char_p, [_i32]),
        "moto_hessian_norm_bound": (ctypes.c_double, [_vp]),
        "moto_plan_graph_replays": (ctypes.c_int64, [_vp]),
        "moto_n_params": (_i32, [_vp]),
        "moto_energy_grad_workspace": (_sz, [_vp, _i32]),
        "moto_energy_grad": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
        "moto_energy_grad_noalloc": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
        "moto_tangent_hvp": (_i32, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp]),
        "moto_hessian_apply": (_i32, [_vp, _i32, _i32, _i32, _vp, _vp, _vp]),
        "moto_tangent_hvp_variants": (_i32, []),
        "moto_plan_set_hvp_variant": (_i32, [_vp, _i32, _i32, _i32, _i32]),
        "moto_tangent_hvp_variant_name": (ctypes.c_char_p, [_i32]),
        "moto_tangent_hvp_autotune": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _i32,
                                             ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_float), _vp]),
        "moto_param_mixed": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
        "moto_param_grad_apply": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _vp]),
        "moto_min_modes_workspace": (_sz, [_vp, _i32, _i32, _i32]),
        "moto_min_modes": (_i32, [_vp, _i32, _vp, _vp, _i32, ctypes.POINTER(EigOpts), _vp, _vp, _vp,
                                  _vp, _vp, _sz, _vp]),
        "moto_default_lanczos_opts": (None, [_i32, ctypes.POINTER(LanczosOpts)]),
        "moto_min_modes_lanczos_workspace": (_sz, [_vp, _i32, _i32]),
        "moto_min_modes_lanczos": (_i32, [_vp, _i32, _vp, _vp, _i32, ctypes.POINTER(LanczosOpts), _vp, _vp, _vp,
                                          ctypes.POINTER(Info), _vp, _sz, _vp]),
        "moto_min_modes_population_workspace": (_sz, [_vp, _i32, _i32, _i32, _i32]),
        "moto_min_modes_population": (_i32, [_vp, _i32, _i32, _vp, _vp, _i32, ctypes.POINTER(EigOpts), _vp, _vp,
                                             _vp, _vp, _vp, _sz, _vp]),
        "moto_step_state_bytes": (_sz, [_vp, _i32]),
        "moto_reflected_step": (_i32, [_vp, _vp, _vp, _vp, _i32, ctypes.POINTER(StepOpts), _vp, _vp, _vp]),
        "moto_descend_workspace": (_sz, [_vp, _i32, ctypes.POINTER(DescendOpts)]),
        "moto_descend": (_i32, [_vp, _i32, _vp, _vp, _i32, ctypes.POINTER(DescendOpts),
                                _vp, _vp, _sz, _vp]),
        "moto_saddle_search_workspace": (_sz, [_vp, _i32, ctypes.POINTER(SearchOpts)]),
        "moto_saddle_search": (_i32, [_vp, _i32, _vp, _vp, ctypes.POINTER(SearchOpts), ctypes.POINTER(SearchResult),
                                      _vp, _vp, _vp, _sz, _vp]),
        "moto_default_eig_opts": (None, [_i32, ctypes.POINTER(EigOpts)]),
        "moto_default_step_opts": (None, [ctypes.POINTER(StepOpts)]),
        "moto_default_descend_opts": (None, [_i32, ctypes.POINTER(DescendOpts)]),
        "moto_default_search_opts": (None, [_i32, ctypes.POINTER(SearchOpts)]),
        "moto_topological_charge": (_i32, [_vp, _i32, _vp, _vp, _vp, _sz, _vp]),
    }
    sig.update({
        "moto_saddle_search_population_workspace": (_sz, [_vp, _i32, _i32, ctypes.POINTER(SearchOpts)]),
        "moto_saddle_search_population": (_i32, [_vp, _i32, _i32, _vp, _vp, ctypes.POINTER(SearchOpts), _vp, _vp,
                                                 _vp, _vp, _sz, _vp]),
        "moto_default_explorer_opts": (None, [_i32, ctypes.POINTER(ExplorerOpts)]),
        "moto_explorer_workspace": (_sz, [_vp, _i32, _i32, _i32, ctypes.POINTER(ExplorerOpts)]),
        "moto_explorer_objectives": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _i32, _vp,
                                            ctypes.POINTER(ExplorerOpts), _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    })
    sig.update({
        "moto_saddle_search_batched_workspace": (_sz, [_i32, ctypes.POINTER(ctypes.c_int32),
                                                       ctypes.POINTER(SearchOpts)]),
        "moto_saddle_search_batched_autotune_workspace": (_sz, [_i32, ctypes.POINTER(ctypes.c_int32),
                                                                 ctypes.POINTER(SearchOpts)]),
        "moto_saddle_search_batched_autotune": (_i32, [ctypes.POINTER(_Ham), _i32, ctypes.POINTER(ctypes.c_int32), _vp,
                                                       _vp, ctypes.POINTER(SearchOpts),
                                                       ctypes.POINTER(ctypes.c_int32), _vp, _sz, _vp]),
        "moto_saddle_search_batched": (_i32, [ctypes.POINTER(_Ham), _i32, ctypes.POINTER(ctypes.c_int32), _vp, _vp,
                                              ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(SearchOpts), _vp, _vp, _sz, _vp]),
    })
    optional = {}
    for name, (res, args) in list(sig.items()) + list(optional.items()):
        if not hasattr(L, name):
            if name in sig:
                raise MotoError(f"libmoto.so lacks {name}")
            continue
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != 0:
        raise MotoError(f"{what}: {lib().moto_status_string(rc).decode()} ({rc})")


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise MotoError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise MotoError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dt(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return MOTO_F64
    if t.dtype == torch.float32:
        return MOTO_F32
    raise MotoError(f"unsupported dtype {t.dtype}")


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class Plan:
    """moto_plan: a validated Hamiltonian on an Lx x Ly lattice."""

    def __init__(self, Lx: int, Ly: int, J: Sequence[float], D: Sequence[float] = (), K: float = 0.0,
                 B: Sequence[float] = (0.0, 0.0, 0.0)):
        h = _Ham()
        h.Lx, h.Ly = int(Lx), int(Ly)
        h.n_shells = max(len(J), len(D), 1)
        h.reserved = 0
        for s in range(MAX_SHELLS):
            h.J[s] = float(J[s]) if s < len(J) else 0.0
            h.D[s] = float(D[s]) if s < len(D) else 0.0
        h.K = float(K)
        for a in range(3):
            h.B[a] = float(B[a])
        self._h = h
        self.Lx, self.Ly, self.N = h.Lx, h.Ly, h.Lx * h.Ly
        self.n_shells = h.n_shells
        p = ctypes.c_void_p()
        _check(lib().moto_plan_create(ctypes.byref(h), ctypes.byref(p)), "moto_plan_create")
        self._p = p

    @classmethod
    def from_params(cls, p) -> "Plan":
        return cls(p.Lx, p.Ly, list(p.J), list(p.D), p.K, tuple(p.B))

    @property
    def handle(self):
        return self._p

    def hessian_norm_bound(self) -> float:
        return float(lib().moto_hessian_norm_bound(self._p))

    def n_params(self) -> int:
        return int(lib().moto_n_params(self._p))

    def close(self):
        if getattr(self, "_p", None) is not None and self._p.value:
            lib().moto_plan_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
def graph_replays(plan: Plan) -> int:
    """Replays of the eigen-solvers' own iteration graphs made with this plan."""
    return int(lib().moto_plan_graph_replays(plan.handle))


def moto_energy_grad(plan: Plan, m: torch.Tensor, mask: Optional[torch.Tensor] = None, want_grad: bool = True,
                     want_c: bool = True, want_F: bool = True, want_dtheta: bool = False, stream=None):
    """E [batch] (FP64), grad, c, F (dtype of m), dE/dtheta [batch][n_params] (FP64)."""
    batch = m.numel() // (3 * plan.N)
    dev = m.device
    E = torch.empty(batch, dtype=torch.float64, device=dev)
    g = torch.empty_like(m) if want_grad else None
    c = torch.empty(m.shape[:-2] + (plan.N,), dtype=m.dtype, device=dev) if want_c else None
    F = torch.empty_like(m) if want_F else None
    dth = torch.empty(batch, plan.n_params(), dtype=torch.float64, device=dev) if want_dtheta else None
    nb = lib().moto_energy_grad_workspace(plan.handle, batch)
    ws = _ws(nb, dev)
    _check(lib().moto_energy_grad(plan.handle, _dt(m), batch, _ptr(m), _ptr(mask), _ptr(E), _ptr(g), _ptr(c),
                                  _ptr(F), _ptr(dth), _ptr(ws), nb, _stream(stream)), "moto_energy_grad")
    return E, g, c, F, dth


def moto_energy_grad_noalloc(plan: Plan, m: torch.Tensor, mask: Optional[torch.Tensor] = None,
                             want_grad: bool = True, want_c: bool = True, want_F: bool = True,
                             want_dtheta: bool = False, out=None, stream=None):
    """moto_energy_grad without a workspace (the library's static per-GPU
    scratch).  `out` = (E, grad, c, F, dE/dtheta) preallocated by the caller
    (entries may be None), so that the call itself allocates nothing."""
    batch = m.numel() // (3 * plan.N)
    if out is None:
        dev = m.device
        out = (torch.empty(batch, dtype=torch.float64, device=dev),
               torch.empty_like(m) if want_grad else None,
               torch.empty(m.shape[:-2] + (plan.N,), dtype=m.dtype, device=dev) if want_c else None,
               torch.empty_like(m) if want_F else None,
               torch.empty(batch, plan.n_params(), dtype=torch.float64, device=dev) if want_dtheta else None)
    E, g, c, F, dth = out
    _check(lib().moto_energy_grad_noalloc(plan.handle, _dt(m), batch, _ptr(m), _ptr(mask), _ptr(E), _ptr(g),
                                          _ptr(c), _ptr(F), _ptr(dth), _stream(stream)), "moto_energy_grad_noalloc")
    return E, g, c, F, dth


NOALLOC_SCRATCH_BYTES = 8 << 20


def moto_tangent_hvp(plan: Plan, m: torch.Tensor, c: torch.Tensor, V: torch.Tensor, layout: int = MOTO_FRAME,
                     mask: Optional[torch.Tensor] = None, W: Optional[torch.Tensor] = None, batch: int = 1,
                     stream=None) -> torch.Tensor:
    """W = M H(m) M V; V is [batch][n_vec][2|3][N]."""
    dv = 2 if layout == MOTO_FRAME else 3
    n_vec = V.numel() // (batch * dv * plan.N)
    if W is None:
        W = torch.empty_like(V)
    _check(lib().moto_tangent_hvp(plan.handle, _dt(m), layout, batch, _ptr(m), _ptr(c), _ptr(mask), n_vec,
                                  _ptr(V), _ptr(W), _stream(stream)), "moto_tangent_hvp")
    return W


def moto_plan_set_hvp_variant(plan: Plan, dtype: int, batch: int, n_vec: int, variant: int):
    _check(lib().moto_plan_set_hvp_variant(plan.handle, dtype, batch, n_vec, variant), "moto_plan_set_hvp_variant")


def moto_tangent_hvp_autotune(plan: Plan, m: torch.Tensor, c: torch.Tensor, V: torch.Tensor, W: torch.Tensor,
                              batch: int = 1, mask: Optional[torch.Tensor] = None, reps: int = 3, stream=None):
    """Time every frame-layout HVP variant on these buffers; the plan keeps
    the fastest for (dtype, batch, n_vec).  Returns (chosen, {name: ms})."""
    n_vec = V.numel() // (batch * 2 * plan.N)
    nv = int(lib().moto_tangent_hvp_variants())
    times = (ctypes.c_float * nv)()
    chosen = _i32()
    _check(lib().moto_tangent_hvp_autotune(plan.handle, _dt(m), batch, _ptr(m), _ptr(c), _ptr(mask), n_vec, _ptr(V),
                                           _ptr(W), reps, ctypes.byref(chosen), times, _stream(stream)),
           "moto_tangent_hvp_autotune")
    names = [lib().moto_tangent_hvp_variant_name(i).decode() for i in range(nv)]
    return chosen.value, {names[i]: float(times[i]) for i in range(nv) if times[i] >= 0}


def moto_hessian_apply(plan: Plan, V: torch.Tensor, batch: int = 1, W: Optional[torch.Tensor] = None,
                       stream=None) -> torch.Tensor:
    n_vec = V.numel() // (batch * 3 * plan.N)
    if W is None:
        W = torch.empty_like(V)
    _check(lib().moto_hessian_apply(plan.handle, _dt(V), batch, n_vec, _ptr(V), _ptr(W), _stream(stream)),
           "moto_hessian_apply")
    return W


def moto_param_mixed(plan: Plan, m: torch.Tensor, U: torch.Tensor, batch: int = 1, stream=None) -> torch.Tensor:
    out = torch.empty(batch, plan.n_params(), dtype=torch.float64, device=m.device)
    nb = lib().moto_energy_grad_workspace(plan.handle, batch)
    ws = _ws(nb, m.device)
    _check(lib().moto_param_mixed(plan.handle, _dt(m), batch, _ptr(m), _ptr(U), _ptr(out), _ptr(ws), nb,
                                  _stream(stream)), "moto_param_mixed")
    return out


def moto_topological_charge(plan: Plan, m: torch.Tensor, batch: int = 1, stream=None) -> torch.Tensor:
    Q = torch.empty(batch, dtype=torch.float64, device=m.device)
    nb = lib().moto_energy_grad_workspace(plan.handle, batch)
    ws = _ws(nb, m.device)
    _check(lib().moto_topological_charge(plan.handle, batch, _ptr(m), _ptr(Q), _ptr(ws), nb, _stream(stream)),
           "moto_topological_charge")
    return Q


def eig_opts(dtype: int = MOTO_F64, **kw) -> EigOpts:
    o = EigOpts()
    lib().moto_default_eig_opts(dtype, ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


RULE_LBFGS, RULE_FIXED, RULE_CG = 0, 1, 2


def step_opts(**kw) -> StepOpts:
    o = StepOpts()
    lib().moto_default_step_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def descend_opts(dtype: int = MOTO_F64, step: Optional[dict] = None, eig: Optional[dict] = None,
                 **kw) -> DescendOpts:
    o = DescendOpts()
    lib().moto_default_descend_opts(dtype, ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    for k, v in (step or {}).items():
        setattr(o.step, k, v)
    for k, v in (eig or {}).items():
        setattr(o.eig, k, v)
    return o


def search_opts(dtype: int = MOTO_F64, step: Optional[dict] = None, eig: Optional[dict] = None,
                **kw) -> SearchOpts:
    o = SearchOpts()
    lib().moto_default_search_opts(dtype, ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    for k, v in (step or {}).items():
        setattr(o.step, k, v)
    for k, v in (eig or {}).items():
        setattr(o.eig, k, v)
    return o


@dataclass
class MinModes:
    evals: torch.Tensor
    V: torch.Tensor
    resid: torch.Tensor
    status: int
    iters: int
    n_hvp: int


def lanczos_opts(dtype: int = MOTO_F64, **kw) -> LanczosOpts:
    o = LanczosOpts()
    lib().moto_default_lanczos_opts(dtype, ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class LanczosWorkspace:
    """Reusable workspace of the Lanczos solver (Krylov basis of m_max + 1 vectors)."""

    def __init__(self, plan: Plan, hvp: int, m_max: int = 32, device="cuda"):
        self.nbytes = int(lib().moto_min_modes_lanczos_workspace(plan.handle, hvp, m_max))
        if self.nbytes == 0:
            raise MotoError("moto_min_modes_lanczos_workspace: invalid arguments")
        self.buf = _ws(self.nbytes, device)


def moto_min_modes_lanczos(plan: Plan, m: torch.Tensor, k: int, hvp: int = MOTO_F64,
                           mask: Optional[torch.Tensor] = None, opts: Optional[LanczosOpts] = None,
                           V0: Optional[torch.Tensor] = None, ws: Optional[LanczosWorkspace] = None,
                           stream=None) -> "MinModes":
    o = opts if opts is not None else lanczos_opts(hvp)
    dev = m.device
    V = torch.zeros(k, 3, plan.N, dtype=torch.float64, device=dev) if V0 is None else V0.clone().contiguous()
    if V0 is not None and o.warm == 0:
        o.warm = 1
    evals = torch.empty(k, dtype=torch.float64, device=dev)
    resid = torch.empty(k, dtype=torch.float64, device=dev)
    if ws is None:
        ws = LanczosWorkspace(plan, hvp, o.m_max, dev)
    info = Info()
    _check(lib().moto_min_modes_lanczos(plan.handle, hvp, _ptr(m), _ptr(mask), k, ctypes.byref(o), _ptr(evals),
                                        _ptr(V), _ptr(resid), ctypes.byref(info), _ptr(ws.buf), ws.nbytes,
                                        _stream(stream)),
           "moto_min_modes_lanczos")
    return MinModes(evals, V, resid, info.status, info.iters, info.n_hvp)


class EigWorkspace:
    """Reusable eigen-solve workspace (keeps the block for warm == 2)."""

    def __init__(self, plan: Plan, hvp: int, k: int, guard: int = -1, device="cuda"):
        self.nbytes = int(lib().moto_min_modes_workspace(plan.handle, hvp, k, guard))
        self.buf = _ws(self.nbytes, device)


def moto_min_modes(plan: Plan, m: torch.Tensor, k: int, hvp: int = MOTO_F64, mask: Optional[torch.Tensor] = None,
                   opts: Optional[EigOpts] = None, V0: Optional[torch.Tensor] = None,
                   ws: Optional[EigWorkspace] = None, info_dev: Optional[torch.Tensor] = None,
                   stream=None) -> MinModes:
    """With opts.flags = MOTO_ASYNC the call does not synchronise: the outcome
    (moto_info: status, iterations, HVP columns) goes to the 16-byte device
    tensor info_dev (or nowhere), and status/iters/n_hvp of the result are None."""
    o = opts if opts is not None else eig_opts(hvp)
    dev = m.device
    V = torch.zeros(k, 3, plan.N, dtype=torch.float64, device=dev) if V0 is None else V0.clone().contiguous()
    if V0 is not None and o.warm == 0:
        o.warm = 1
    evals = torch.empty(k, dtype=torch.float64, device=dev)
    resid = torch.empty(k, dtype=torch.float64, device=dev)
    if ws is None:
        ws = EigWorkspace(plan, hvp, k, o.guard, dev)
    if o.flags & MOTO_ASYNC:
        if info_dev is not None and info_dev.numel() * info_dev.element_size() < ctypes.sizeof(Info):
            raise MotoError("info_dev must hold one moto_info (16 bytes)")
        _check(lib().moto_min_modes(plan.handle, hvp, _ptr(m), _ptr(mask), k, ctypes.byref(o), _ptr(evals), _ptr(V),
                                    _ptr(resid), _ptr(info_dev), _ptr(ws.buf), ws.nbytes, _stream(stream)),
               "moto_min_modes")
        return MinModes(evals, V, resid, None, None, None)
    info = Info()
    _check(lib().moto_min_modes(plan.handle, hvp, _ptr(m), _ptr(mask), k, ctypes.byref(o), _ptr(evals), _ptr(V),
                                _ptr(resid), ctypes.addressof(info), _ptr(ws.buf), ws.nbytes, _stream(stream)),
           "moto_min_modes")
    return MinModes(evals, V, resid, info.status, info.iters, info.n_hvp)


MAX_POPULATION = 256


@dataclass
class PopulationModes:
    evals: torch.Tensor  # [P, k]
    V: torch.Tensor      # [P, k, 3, N]
    resid: torch.Tensor  # [P, k]
    status: list
    iters: list
    n_hvp: list


class PopulationWorkspace:
    def __init__(self, plan: Plan, hvp: int, P: int, k: int, guard: int = -1, device="cuda"):
        self.nbytes = int(lib().moto_min_modes_population_workspace(plan.handle, hvp, P, k, guard))
        if self.nbytes == 0:
            raise MotoError("population size or k out of range")
        self.buf = _ws(self.nbytes, device)


def moto_min_modes_population(plan: Plan, m: torch.Tensor, k: int, hvp: int = MOTO_F64,
                              mask: Optional[torch.Tensor] = None, opts: Optional[EigOpts] = None,
                              V0: Optional[torch.Tensor] = None, ws: Optional[PopulationWorkspace] = None,
                              stream=None) -> PopulationModes:
    """k lowest modes of each of the P states m [P, 3, N] (mask [P, N] or None)."""
    if m.dim() != 3 or m.shape[1] != 3 or m.shape[2] != plan.N:
        raise MotoError("m must be [P, 3, N]")
    P = int(m.shape[0])
    if mask is not None and (mask.dtype != torch.uint8 or mask.numel() != P * plan.N):
        raise MotoError("mask must be uint8 [P, N]")
    if V0 is not None and V0.numel() != P * k * 3 * plan.N:
        raise MotoError("V0 must be [P, k, 3, N]")
    o = opts if opts is not None else eig_opts(hvp)
    if o.flags & MOTO_ASYNC:
        raise MotoError("moto_min_modes_population: this binding reads the outcome on the host (no MOTO_ASYNC)")
    dev = m.device
    V = torch.zeros(P, k, 3, plan.N, dtype=torch.float64, device=dev) if V0 is None else V0.clone().contiguous()
    if V0 is not None and o.warm == 0:
        o.warm = 1
    evals = torch.empty(P, k, dtype=torch.float64, device=dev)
    resid = torch.empty(P, k, dtype=torch.float64, device=dev)
    if ws is None:
        ws = PopulationWorkspace(plan, hvp, P, k, o.guard, dev)
    info = (Info * P)()
    _check(lib().moto_min_modes_population(plan.handle, hvp, P, _ptr(m), _ptr(mask), k, ctypes.byref(o),
                                           _ptr(evals), _ptr(V), _ptr(resid), info, _ptr(ws.buf), ws.nbytes,
                                           _stream(stream)),
           "moto_min_modes_population")
    return PopulationModes(evals, V, resid, [i.status for i in info], [i.iters for i in info],
                           [i.n_hvp for i in info])


class StepState:
    def __init__(self, plan: Plan, mem: int = 8, device="cuda"):
        self.nbytes = int(lib().moto_step_state_bytes(plan.handle, mem))
        self.buf = torch.zeros(self.nbytes, dtype=torch.uint8, device=device)
        self.out = torch.zeros(2, dtype=torch.float64, device=device)

    def reset(self):
        self.buf.zero_()
        self.out.zero_()


def moto_reflected_step(plan: Plan, m: torch.Tensor, F: torch.Tensor, V: Optional[torch.Tensor], k_reflect: int,
                        state: StepState, opts: Optional[StepOpts] = None, stream=None) -> torch.Tensor:
    o = opts if opts is not None else step_opts()
    _check(lib().moto_reflected_step(plan.handle, _ptr(m), _ptr(F), _ptr(V), k_reflect, ctypes.byref(o),
                                     _ptr(state.buf), _ptr(state.out), _stream(stream)), "moto_reflected_step")
    return state.out


def moto_descend(plan: Plan, m: torch.Tensor, v1: torch.Tensor, sign: int, hvp: int = MOTO_F64,
                 opts: Optional[DescendOpts] = None, res_dev: Optional[torch.Tensor] = None,
                 stream=None) -> Optional[DescendResult]:
    """With opts.flags = MOTO_ASYNC the result struct goes to the device
    tensor res_dev (sizeof(DescendResult) bytes) and None is returned."""
    o = opts if opts is not None else descend_opts(hvp)
    nb = int(lib().moto_descend_workspace(plan.handle, hvp, ctypes.byref(o)))
    ws = _ws(nb, m.device)
    if o.flags & MOTO_ASYNC:
        if res_dev is None or res_dev.numel() * res_dev.element_size() < ctypes.sizeof(DescendResult):
            raise MotoError("res_dev must hold one moto_descend_result")
        _check(lib().moto_descend(plan.handle, hvp, _ptr(m), _ptr(v1), int(sign), ctypes.byref(o), _ptr(res_dev),
                                  _ptr(ws), nb, _stream(stream)), "moto_descend")
        return None
    res = DescendResult()
    _check(lib().moto_descend(plan.handle, hvp, _ptr(m), _ptr(v1), int(sign), ctypes.byref(o),
                              ctypes.addressof(res), _ptr(ws), nb, _stream(stream)), "moto_descend")
    return res


def moto_saddle_search_population(plan: Plan, m: torch.Tensor, hvp: int = MOTO_F64,
                                  mask: Optional[torch.Tensor] = None, opts: Optional[SearchOpts] = None,
                                  stream=None):
    """P searches in lock step on m [P, 3, N] (updated in place).  Returns
    (list of SearchResult, evals [P, k_cert], V [P, k_cert, 3, N])."""
    if m.dim() != 3 or m.shape[1] != 3 or m.shape[2] != plan.N:
        raise MotoError("m must be [P, 3, N]")
    P = int(m.shape[0])
    if mask is not None and (mask.dtype != torch.uint8 or mask.numel() != P * plan.N):
        raise MotoError("mask must be uint8 [P, N]")
    o = opts if opts is not None else search_opts(hvp)
    kc = max(o.k_cert, 2)
    nb = int(lib().moto_saddle_search_population_workspace(plan.handle, hvp, P, ctypes.byref(o)))
    if nb == 0:
        raise MotoError("population size or options out of range")
    ws = _ws(nb, m.device)
    ev = torch.empty(P, kc, dtype=torch.float64, device=m.device)
    V = torch.empty(P, kc, 3, plan.N, dtype=torch.float64, device=m.device)
    res = (SearchResult * P)()
    _check(lib().moto_saddle_search_population(plan.handle, hvp, P, _ptr(m), _ptr(mask), ctypes.byref(o), res,
                                               _ptr(ev), _ptr(V), _ptr(ws), nb, _stream(stream)),
           "moto_saddle_search_population")
    return list(res), ev, V


def moto_saddle_search(plan: Plan, m: torch.Tensor, hvp: int = MOTO_F64, mask: Optional[torch.Tensor] = None,
                       opts: Optional[SearchOpts] = None, stream=None):
    """Returns (SearchResult, evals [k_cert], V [k_cert][3][N]); m is updated in place."""
    o = opts if opts is not None else search_opts(hvp)
    kc = max(o.k_cert, 2)
    nb = int(lib().moto_saddle_search_workspace(plan.handle, hvp, ctypes.byref(o)))
    ws = _ws(nb, m.device)
    ev = torch.empty(kc, dtype=torch.float64, device=m.device)
    V = torch.empty(kc, 3, plan.N, dtype=torch.float64, device=m.device)
    res = SearchResult()
    _check(lib().moto_saddle_search(plan.handle, hvp, _ptr(m), _ptr(mask), ctypes.byref(o), ctypes.byref(res),
                                    _ptr(ev), _ptr(V), _ptr(ws), nb, _stream(stream)), "moto_saddle_search")
    return res, ev, V


TILE_32x8, TILE_16x16, TILE_64x4 = 0, 1, 2


def _batch_ham(params) -> "_Ham":
    h = _Ham()
    h.Lx, h.Ly = 1, 1
    h.n_shells = max(len(params.J), len(params.D), 1)
    h.reserved = 0
    for s in range(MAX_SHELLS):
        h.J[s] = float(params.J[s]) if s < len(params.J) else 0.0
        h.D[s] = float(params.D[s]) if s < len(params.D) else 0.0
    h.K = float(params.K)
    for a in range(3):
        h.B[a] = float(params.B[a])
    return h


def moto_saddle_search_batched_autotune(params, Ls: Sequence[int], m_all: torch.Tensor,
                                        opts: Optional[SearchOpts] = None, mask_all: Optional[torch.Tensor] = None,
                                        stream=None):
    """Tile shape per lattice (MOTO_TILE_*) chosen by timing short batched runs
    per lattice-size bucket; m_all and mask_all are left unchanged."""
    o = opts if opts is not None else search_opts(MOTO_F32)
    n = len(Ls)
    Larr = (ctypes.c_int32 * n)(*[int(v) for v in Ls])
    nb = int(lib().moto_saddle_search_batched_autotune_workspace(n, Larr, ctypes.byref(o)))
    if nb == 0:
        raise MotoError("moto_saddle_search_batched_autotune_workspace: invalid sizes or options")
    ws = _ws(nb, m_all.device)
    tiles = (ctypes.c_int32 * n)()
    h = _batch_ham(params)
    _check(lib().moto_saddle_search_batched_autotune(ctypes.byref(h), n, Larr, _ptr(m_all), _ptr(mask_all),
                                                     ctypes.byref(o), tiles, _ptr(ws), nb, _stream(stream)),
           "moto_saddle_search_batched_autotune")
    return list(tiles)


def moto_saddle_search_batched(params, Ls: Sequence[int], m_all: torch.Tensor, opts: Optional[SearchOpts] = None,
                               mask_all: Optional[torch.Tensor] = None, tiles: Optional[Sequence[int]] = None,
                               stream=None):
    """Saddle searches on square lattices of sides Ls in one persistent launch
    (FP32 HVP, FP64 state).  m_all holds the starts back to back
    ([3][L_b^2] each, FP64) and is updated in place; tiles: tile shape per
    lattice (None: 32 x 8).  Returns a list of SearchResult (one per lattice,
    input order)."""
    o = opts if opts is not None else search_opts(MOTO_F32)
    n = len(Ls)
    Larr = (ctypes.c_int32 * n)(*[int(v) for v in Ls])
    tarr = None if tiles is None else (ctypes.c_int32 * n)(*[int(v) for v in tiles])
    nb = int(lib().moto_saddle_search_batched_workspace(n, Larr, ctypes.byref(o)))
    if nb == 0:
        raise MotoError("moto_saddle_search_batched_workspace: invalid sizes or options")
    ws = _ws(nb, m_all.device)
    res = torch.empty(n * ctypes.sizeof(SearchResult), dtype=torch.uint8, device=m_all.device)
    h = _batch_ham(params)
    if mask_all is not None and (mask_all.dtype != torch.uint8 or mask_all.numel() != sum(int(v) ** 2 for v in Ls)):
        raise MotoError("mask_all must be uint8 with one entry per site of every lattice")
    _check(lib().moto_saddle_search_batched(ctypes.byref(h), n, Larr, _ptr(m_all), _ptr(mask_all), tarr,
                                            ctypes.byref(o), _ptr(res),
                                            _ptr(ws), nb, _stream(stream)), "moto_saddle_search_batched")
    raw = bytes(res.cpu().numpy())
    sz = ctypes.sizeof(SearchResult)
    return [SearchResult.from_buffer_copy(raw[i * sz:(i + 1) * sz]) for i in range(n)]


# ---------------------------------------------------------------------------
# Explorer objectives
# ---------------------------------------------------------------------------
def explorer_opts(dtype: int = MOTO_F32, eig: Optional[dict] = None, **kw) -> ExplorerOpts:
    o = ExplorerOpts()
    lib().moto_default_explorer_opts(dtype, ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    for k, v in (eig or {}).items():
        setattr(o.eig, k, v)
    return o


@dataclass
class Explorer:
    X: torch.Tensor          # [P, 3, N] candidates
    res: dict                # per-candidate arrays: E, lambda1, lambda2, gap, Q, violation, l1_sum, l1_min,
                             # status, iters, n_hvp
    evals: torch.Tensor      # [P, k]
    V: Optional[torch.Tensor]
    D: torch.Tensor          # [P, P + A]


def moto_explorer_objectives(plan: Plan, x0: torch.Tensor, delta: torch.Tensor, hvp: int = MOTO_F32,
                             mask: Optional[torch.Tensor] = None, archive: Optional[torch.Tensor] = None,
                             opts: Optional[ExplorerOpts] = None, want_V: bool = False, stream=None) -> Explorer:
    """Objectives of the P candidates x0 + P_Omega delta (delta [P, 3, N])."""
    N = plan.N
    if x0.numel() != 3 * N or delta.dim() != 3 or delta.shape[1] != 3 or delta.shape[2] != N:
        raise MotoError("x0 must be [3, N] and delta [P, 3, N]")
    if mask is not None and (mask.dtype != torch.uint8 or mask.numel() != N):
        raise MotoError("mask must be uint8 [N]")
    P = int(delta.shape[0])
    A = 0 if archive is None else int(archive.shape[0])
    if archive is not None and archive.numel() != A * 3 * N:
        raise MotoError("archive must be [A, 3, N]")
    o = opts if opts is not None else explorer_opts(hvp)
    nb = int(lib().moto_explorer_workspace(plan.handle, hvp, P, A, ctypes.byref(o)))
    if nb == 0:
        raise MotoError("explorer arguments out of range")
    dev = delta.device
    ws = _ws(nb, dev)
    X = torch.empty(P, 3, N, dtype=torch.float64, device=dev)
    res = torch.empty(P * ctypes.sizeof(ExplorerResult), dtype=torch.uint8, device=dev)
    evals = torch.empty(P, o.k, dtype=torch.float64, device=dev)
    V = torch.empty(P, o.k, 3, N, dtype=torch.float64, device=dev) if want_V else None
    D = torch.empty(P, P + A, dtype=torch.float64, device=dev)
    _check(lib().moto_explorer_objectives(plan.handle, hvp, P, _ptr(x0), _ptr(mask), _ptr(delta), A, _ptr(archive),
                                          ctypes.byref(o), _ptr(X), _ptr(res), _ptr(evals), _ptr(V), _ptr(D),
                                          _ptr(ws), nb, _stream(stream)),
           "moto_explorer_objectives")
    raw = (ExplorerResult * P).from_buffer_copy(bytes(res.cpu().numpy()))
    out = {f: np.array([getattr(r, f) for r in raw]) for f, _ in ExplorerResult._fields_}
    return Explorer(X, out, evals, V, D)
