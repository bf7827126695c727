"""Plain FP64 CPU oracle for the bilayer minimum-mode kernel (arXiv 2509.26269).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library in ``paper_2509_26269_amd`` and never imports it.

The stencil arithmetic (energy, gradient, Hessian) lives in ``moto_oracle.c``
as single-threaded loops over ordered site pairs; the iterations (eigen-solve,
climb, descent) are written here in numpy, in the order the paper gives them.

Parity status of each function is stated in its docstring.  Every function
listed here is pinned by at least one CPU test in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmoto_oracle.so")
MAX_SHELLS = 36


def _load():
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # noqa: WPS433 (oracle-local build helper)

        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    hp = ctypes.POINTER(_CHam)
    lib.orc_shells.argtypes = [ctypes.c_int, ip, ip, ip, ctypes.c_int]
    lib.orc_shells.restype = ctypes.c_int
    lib.orc_energy.argtypes = [hp, dp, dp, dp]
    lib.orc_gradient.argtypes = [hp, dp, dp]
    lib.orc_apply_A.argtypes = [hp, dp, dp]
    lib.orc_force.argtypes = [ctypes.c_int, dp, dp, dp, dp]
    lib.orc_tangent_hvp.argtypes = [hp, dp, dp, ctypes.c_void_p, dp, dp]
    lib.orc_dense_hessian_fd.argtypes = [hp, dp, ctypes.c_double, dp]
    lib.orc_jacobi_eig.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_double, ctypes.c_int]
    lib.orc_jacobi_eig.restype = ctypes.c_int
    lib.orc_topological_charge.argtypes = [ctypes.c_int, ctypes.c_int, dp]
    lib.orc_topological_charge.restype = ctypes.c_double
    return lib


class _CHam(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_int32),
        ("Ly", ctypes.c_int32),
        ("n_shells", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("J", ctypes.c_double * MAX_SHELLS),
        ("D", ctypes.c_double * MAX_SHELLS),
        ("K", ctypes.c_double),
        ("B", ctypes.c_double * 3),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _load()
    return _lib


@dataclass
class Ham:
    """Spin Hamiltonian of the Methods section (Eq. param-hamiltonian) on a
    periodic rhombic Lx x Ly triangular lattice.  J[s], D[s] per shell s
    (D_delta = D[s] * (z x dhat)), uniaxial K along e_z, Zeeman field B
    (mu_i = 1)."""

    Lx: int
    Ly: int
    J: Sequence[float]
    D: Sequence[float] = ()
    K: float = 0.0
    B: Sequence[float] = (0.0, 0.0, 0.0)

    @property
    def N(self) -> int:
        return self.Lx * self.Ly

    @property
    def n_shells(self) -> int:
        return max(len(self.J), len(self.D))

    def c(self) -> _CHam:
        h = _CHam()
        h.Lx, h.Ly, h.n_shells = self.Lx, self.Ly, self.n_shells
        for s in range(MAX_SHELLS):
            h.J[s] = float(self.J[s]) if s < len(self.J) else 0.0
            h.D[s] = float(self.D[s]) if s < len(self.D) else 0.0
        h.K = float(self.K)
        for a in range(3):
            h.B[a] = float(self.B[a])
        return h

    def theta(self) -> np.ndarray:
        """Parameter vector (J_0..J_{ns-1}, D_0..D_{ns-1}, K, Bx, By, Bz)."""
        ns = self.n_shells
        J = [float(self.J[s]) if s < len(self.J) else 0.0 for s in range(ns)]
        D = [float(self.D[s]) if s < len(self.D) else 0.0 for s in range(ns)]
        return np.array(J + D + [self.K] + list(self.B), dtype=np.float64)

    def h_est(self) -> float:
        """Rigorous bound on the tangent-Hessian norm:
        4 sum_delta(|J_delta| + |D_delta|) + 4|K| + |B| (6 offsets per shell
        for the first three shells; counted from the shell generator)."""
        cnt = shell_counts(self.n_shells)
        sJ = sum(cnt[s] * abs(self.J[s]) for s in range(len(self.J)))
        sD = sum(cnt[s] * abs(self.D[s]) for s in range(len(self.D)))
        return 4.0 * (sJ + sD) + 4.0 * abs(self.K) + float(np.linalg.norm(self.B))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# Lattice
# ---------------------------------------------------------------------------
def shells(n_shells: int):
    """Offsets (dx, dy, shell) of the first n_shells shells of the triangular
    lattice, sorted by |dx a1 + dy a2|."""
    cap = 1024
    dx = (ctypes.c_int * cap)()
    dy = (ctypes.c_int * cap)()
    sh = (ctypes.c_int * cap)()
    n = lib().orc_shells(n_shells, dx, dy, sh, cap)
    if n < 0:
        raise ValueError("bad shell count")
    return [(dx[i], dy[i], sh[i]) for i in range(n)]


def shell_counts(n_shells: int):
    c = [0] * n_shells
    for _, _, s in shells(n_shells):
        c[s] += 1
    return c


# ---------------------------------------------------------------------------
# Energy, gradient, Hessian (exact quantities; pinned by closed forms, FD,
# identities -- see tests/test_oracle_energy.py)
# ---------------------------------------------------------------------------
def energy_terms(ham: Ham, m) -> np.ndarray:
    """(E_exchange, E_dmi, E_zeeman, E_anisotropy, E_total) of Eq.
    param-hamiltonian, sums over ordered pairs."""
    m = _f64(m).reshape(3, ham.N)
    out = np.zeros(5)
    lib().orc_energy(ctypes.byref(ham.c()), _dp(m), _dp(out), None)
    return out


def energy(ham: Ham, m) -> float:
    return float(energy_terms(ham, m)[4])


def param_grad(ham: Ham, m) -> np.ndarray:
    """dE/dtheta for theta = (J_0.., D_0.., K, Bx, By, Bz); E is linear in theta."""
    m = _f64(m).reshape(3, ham.N)
    out = np.zeros(5)
    dth = np.zeros(2 * ham.n_shells + 4)
    lib().orc_energy(ctypes.byref(ham.c()), _dp(m), _dp(out), _dp(dth))
    return dth


def gradient(ham: Ham, m) -> np.ndarray:
    """Euclidean gradient dE/dm, shape (3, N)."""
    m = _f64(m).reshape(3, ham.N)
    g = np.zeros((3, ham.N))
    lib().orc_gradient(ctypes.byref(ham.c()), _dp(m), _dp(g))
    return g


def apply_A(ham: Ham, v) -> np.ndarray:
    """Euclidean Hessian (constant) applied to v, shape (3, N)."""
    v = _f64(v).reshape(3, ham.N)
    out = np.zeros((3, ham.N))
    lib().orc_apply_A(ctypes.byref(ham.c()), _dp(v), _dp(out))
    return out


def force(m, g):
    """c_i = m_i.g_i and F_i = -(I - m_i m_i^T) g_i."""
    m = _f64(m)
    g = _f64(g)
    N = m.shape[-1]
    c = np.zeros(N)
    F = np.zeros((3, N))
    lib().orc_force(N, _dp(m), _dp(g), _dp(c), _dp(F))
    return c, F


def energy_grad(ham: Ham, m):
    """(E, g, c, F) at m."""
    g = gradient(ham, m)
    c, F = force(_f64(m).reshape(3, ham.N), g)
    return energy(ham, m), g, c, F


def tangent_hvp(ham: Ham, m, c, v, mask=None) -> np.ndarray:
    """Riemannian Hessian-vector product (H v)_i = P_i (A v)_i - c_i v_i,
    masked as M H (M v).  v may be (3, N) or (n, 3, N)."""
    m = _f64(m).reshape(3, ham.N)
    c = _f64(c).reshape(ham.N)
    v = _f64(v)
    single = v.ndim == 2
    vv = v.reshape(-1, 3, ham.N)
    out = np.zeros_like(vv)
    mk = None
    if mask is not None:
        mk_arr = np.ascontiguousarray(mask, dtype=np.uint8)
        mk = mk_arr.ctypes.data_as(ctypes.c_void_p)
    for q in range(vv.shape[0]):
        vq = np.ascontiguousarray(vv[q])
        oq = np.zeros((3, ham.N))
        lib().orc_tangent_hvp(ctypes.byref(ham.c()), _dp(m), _dp(c), mk, _dp(vq), _dp(oq))
        out[q] = oq
    return out[0] if single else out


def dense_hessian_fd(ham: Ham, m, h_fd: float = 1.0) -> np.ndarray:
    """Euclidean Hessian from the energy alone (exact 4-point differences)."""
    m = _f64(m).reshape(3, ham.N)
    n = 3 * ham.N
    H = np.zeros((n, n))
    lib().orc_dense_hessian_fd(ctypes.byref(ham.c()), _dp(m), h_fd, _dp(H))
    return H


def dense_A(ham: Ham) -> np.ndarray:
    """Euclidean Hessian as a dense (3N, 3N) matrix, column by column."""
    n = 3 * ham.N
    A = np.zeros((n, n))
    e = np.zeros(n)
    for a in range(n):
        e[:] = 0.0
        e[a] = 1.0
        A[:, a] = apply_A(ham, e.reshape(3, ham.N)).reshape(n)
    return A


def topological_charge(ham_or_L, m, Ly: Optional[int] = None) -> float:
    if isinstance(ham_or_L, Ham):
        Lx, Ly = ham_or_L.Lx, ham_or_L.Ly
    else:
        Lx = int(ham_or_L)
    m = _f64(m).reshape(3, Lx * Ly)
    return float(lib().orc_topological_charge(Lx, Ly, _dp(m)))


# ---------------------------------------------------------------------------
# Tangent frames (the frame coordinate convention of the library boundary):
# branchless orthonormal basis of Duff et al., "Building an Orthonormal
# Basis, Revisited", JCGT 6(1), 2017, for a unit vector n:
#   s = copysign(1, n_z); a = -1/(s + n_z); b = n_x n_y a;
#   e1 = (1 + s n_x^2 a, s b, -s n_x);   e2 = (b, s + n_y^2 a, -n_y).
# ---------------------------------------------------------------------------
def frame(m):
    m = _f64(m)
    nx, ny, nz = m[0], m[1], m[2]
    s = np.copysign(1.0, nz)
    a = -1.0 / (s + nz)
    b = nx * ny * a
    e1 = np.stack([1.0 + s * nx * nx * a, s * b, -s * nx])
    e2 = np.stack([b, s + ny * ny * a, -ny])
    return e1, e2


def to_frame(m, v) -> np.ndarray:
    """Ambient tangent vectors (..., 3, N) -> frame coordinates (..., 2, N)."""
    e1, e2 = frame(m)
    v = _f64(v)
    return np.stack([(v * e1).sum(-2), (v * e2).sum(-2)], axis=-2)


def from_frame(m, a) -> np.ndarray:
    """Frame coordinates (..., 2, N) -> ambient tangent vectors (..., 3, N)."""
    e1, e2 = frame(m)
    a = _f64(a)
    return a[..., 0:1, :] * e1 + a[..., 1:2, :] * e2


def project(m, v) -> np.ndarray:
    """P_i v_i = v_i - (m_i . v_i) m_i."""
    m = _f64(m)
    v = _f64(v)
    return v - (v * m).sum(-2, keepdims=True) * m


# ---------------------------------------------------------------------------
# Dense tangent Hessian and full eigensolve (the explicit-Hessian reference of
# the Methods section, in the 2N tangent coordinates).
# ---------------------------------------------------------------------------
def dense_tangent_hessian(ham: Ham, m, c=None, mask=None) -> np.ndarray:
    """H_T = U^T (A - diag(c) (x) I3) U with U the block-diagonal frame basis,
    restricted to the active sites if a mask is given.  Coordinates are
    ordered (frame index, site) = (0, s) ... (1, s) over active sites."""
    m = _f64(m).reshape(3, ham.N)
    if c is None:
        c, _ = force(m, gradient(ham, m))
    A = dense_A(ham)
    e1, e2 = frame(m)
    N = ham.N
    act = np.arange(N) if mask is None else np.nonzero(np.asarray(mask))[0]
    na = len(act)
    U = np.zeros((3 * N, 2 * na))
    for col, i in enumerate(act):
        for comp in range(3):
            U[comp * N + i, col] = e1[comp, i]
            U[comp * N + i, na + col] = e2[comp, i]
    HT = U.T @ A @ U
    cc = np.concatenate([c[act], c[act]])
    HT -= np.diag(cc)
    return 0.5 * (HT + HT.T)


def jacobi_eigh(A, tol: float = 1e-15, max_sweeps: int = 60):
    """Cyclic Jacobi (Golub & Van Loan).  Returns ascending (w, V)."""
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    n = A.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n))
    sweeps = lib().orc_jacobi_eig(n, _dp(A), _dp(w), _dp(V), tol, max_sweeps)
    if sweeps < 0:
        raise RuntimeError("Jacobi did not converge")
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order]


def sign_fix(v) -> np.ndarray:
    """Sign rule of the boundary: the component of largest |value| (first in
    [3][N] order on ties) is made positive."""
    v = np.array(v, dtype=np.float64, copy=True)
    flat = v.reshape(-1)
    i = int(np.argmax(np.abs(flat)))
    if flat[i] < 0:
        v = -v
    return v


def min_modes_dense(ham: Ham, m, k: int, mask=None):
    """k smallest eigenpairs of the tangent Hessian by dense Jacobi.
    Returns (evals[k], V[k,3,N] ambient unit vectors, sign-fixed)."""
    m = _f64(m).reshape(3, ham.N)
    HT = dense_tangent_hessian(ham, m, mask=mask)
    w, Z = jacobi_eigh(HT)
    N = ham.N
    act = np.arange(N) if mask is None else np.nonzero(np.asarray(mask))[0]
    na = len(act)
    e1, e2 = frame(m)
    V = np.zeros((k, 3, N))
    for j in range(k):
        a = np.zeros((2, N))
        a[0, act] = Z[:na, j]
        a[1, act] = Z[na:, j]
        V[j] = sign_fix(a[0] * e1 + a[1] * e2)
    return w[:k], V


# ---------------------------------------------------------------------------
# Inner layer: block LOBPCG (Knyazev 2001) on the tangent Hessian, FP64, no
# preconditioner, Rayleigh-Ritz on span[X, W, P] with an SVQB-orthonormalised
# basis (Stathopoulos & Wu 2002).  Parity: pinned against Jacobi and the
# closed-form ferromagnet spectra.
# ---------------------------------------------------------------------------
def _svqb(S, drop: float = 1e-12):
    G = S.T @ S
    G = 0.5 * (G + G.T)
    d = np.sqrt(np.maximum(np.diag(G), 1e-300))
    Gs = G / np.outer(d, d)
    th, Z = np.linalg.eigh(Gs)
    keep = th > drop * th.max()
    return (Z[:, keep] / np.sqrt(th[keep])) / d[:, None]


@dataclass
class EigResult:
    evals: np.ndarray
    V: np.ndarray          # (k, 3, N) ambient, sign-fixed
    resid: np.ndarray      # ||H v - lambda v||_2 per returned pair
    iters: int
    n_hvp: int
    converged: bool
    X_block: np.ndarray = field(repr=False, default=None)  # full block, frame coords (2N', m)


def lobpcg(op, X0, k: int, tol_abs: float, max_iter: int = 200):
    """Block LOBPCG minimising the trace of the Rayleigh quotient.
    op(Y) applies the operator to the columns of Y.  Returns
    (lam[:block], X[:, :block], rnorm[:block], iters, n_hvp_columns, converged)."""
    X = X0 @ _svqb(X0)
    X = X @ _svqb(X)
    X = X[:, : X0.shape[1]]
    mb = X.shape[1]
    HX = op(X)
    n_hvp = mb
    lam, C = np.linalg.eigh(0.5 * (X.T @ HX + HX.T @ X))
    X, HX = X @ C, HX @ C
    P = HP = None
    it = 0
    conv = False
    while True:
        R = HX - X * lam
        rn = np.linalg.norm(R, axis=0)
        if np.all(rn[:k] <= tol_abs):
            conv = True
            break
        if it >= max_iter:
            break
        it += 1
        W = R - X @ (X.T @ R)
        HW = op(W)
        n_hvp += W.shape[1]
        if P is None:
            S, HS = np.hstack([X, W]), np.hstack([HX, HW])
        else:
            S, HS = np.hstack([X, W, P]), np.hstack([HX, HW, HP])
        T = _svqb(S)
        T = T @ _svqb(S @ T)
        Q, HQ = S @ T, HS @ T
        Am = Q.T @ HQ
        theta, Y = np.linalg.eigh(0.5 * (Am + Am.T))
        Cf = T @ Y[:, :mb]
        lam = theta[:mb]
        Xn, HXn = S @ Cf, HS @ Cf
        Cwp = Cf.copy()
        Cwp[:mb] = 0.0
        P, HP = S @ Cwp, HS @ Cwp
        X, HX = Xn, HXn
    return lam, X, rn, it, n_hvp, conv


def min_modes(ham: Ham, m, k: int, tol: float = 1e-10, max_iter: int = 200,
              guard: Optional[int] = None, mask=None, X0=None, seed: int = 0,
              c=None) -> EigResult:
    """k smallest eigenpairs of the (masked) tangent Hessian by FP64 LOBPCG in
    frame coordinates.  Stopping rule: ||H v_j - lambda_j v_j||_2 <= tol *
    h_est for j < k.  Vectors returned ambient and sign-fixed."""
    m = _f64(m).reshape(3, ham.N)
    N = ham.N
    if c is None:
        c, _ = force(m, gradient(ham, m))
    act = np.ones(N, dtype=bool) if mask is None else np.asarray(mask).astype(bool)
    if guard is None:
        guard = max(2, (k + 1) // 2)
    mb = k + guard
    e1, e2 = frame(m)

    def to_amb(Y):  # (2N, b) frame -> (b, 3, N) ambient
        a = Y.T.reshape(-1, 2, N)
        return a[:, 0:1, :] * e1 + a[:, 1:2, :] * e2

    def op(Y):
        Y = Y.copy()
        Y[:N][~act] = 0.0
        Y[N:][~act] = 0.0
        V = to_amb(Y)
        HV = tangent_hvp(ham, m, c, V, mask=None if mask is None else act.astype(np.uint8))
        out = np.concatenate([(HV * e1).sum(1), (HV * e2).sum(1)], axis=1).T
        out[:N][~act] = 0.0
        out[N:][~act] = 0.0
        return out

    rng = np.random.default_rng(seed)
    X = rng.standard_normal((2 * N, mb))
    if X0 is not None:
        X0 = np.asarray(X0, dtype=np.float64)
        ncol = min(X0.shape[1], mb)
        X[:, :ncol] = X0[:, :ncol]
    X[:N][~act] = 0.0
    X[N:][~act] = 0.0
    lam, Xb, rn, it, n_hvp, conv = lobpcg(op, X, k, tol * ham.h_est(), max_iter)
    V = np.stack([sign_fix(v) for v in to_amb(Xb[:, :k])])
    nrm = np.linalg.norm(V.reshape(k, -1), axis=1)
    V = V / nrm[:, None, None]
    return EigResult(lam[:k].copy(), V, rn[:k].copy(), it, n_hvp, conv, Xb)


# ---------------------------------------------------------------------------
# Inner layer, second solver: thick-restart band Lanczos with full
# reorthogonalisation (the paper's HVP-Lanczos operator mode; the Krylov depth
# and the reorthogonalisation are its named hyperparameters).  A start block of
# b orthonormal vectors; step j applies the operator to basis vector j and
# orthogonalises the image against every vector so far (the band Lanczos of
# Ruhe 1979), so the Krylov space grows from b directions at once and a split
# pair of eigenvalues enters it as fast as a single one (a single start vector
# can leave the second member of a close pair out of the space long after the
# first has converged).  The projected matrix is accumulated column by column
# from the reorthogonalisation coefficients, so after a restart it holds the
# kept Ritz values and their couplings to the residual block (Wu & Simon
# 2000).  Parity: pinned against Jacobi, the ferromagnet closed form and the
# LOBPCG oracle.
# ---------------------------------------------------------------------------
def lanczos(op, V0, k: int, tol_abs: float, m_max: int = 32, keep: Optional[int] = None,
            max_restarts: int = 100, fresh=None):
    """k smallest eigenpairs of the symmetric operator op (applied to one
    vector), from the start block V0 (n, b) (a single vector (n,) is a block
    of one).  fresh() returns a new random vector for a direction the Krylov
    space can no longer supply.  Returns (theta[:keep], Ritz vectors
    X[:, :keep], residual norms, restarts, n_hvp, converged)."""
    V0 = np.asarray(V0, dtype=np.float64)
    if V0.ndim == 1:
        V0 = V0[:, None]
    n, b = V0.shape
    if keep is None:
        keep = max(k + 2, m_max // 2)
    assert k <= keep and keep + b <= m_max
    if fresh is None:
        rng = np.random.default_rng(12345)
        fresh = lambda: rng.standard_normal(n)  # noqa: E731
    Q = np.zeros((n, m_max + b))
    T = np.zeros((m_max + b, m_max + b))

    def put(c, v):
        """Column c <- v orthogonalised twice against columns 0..c-1 and
        normalised; a dependent v is replaced by fresh random directions."""
        for _ in range(8):
            for _ in range(2):
                v = v - Q[:, :c] @ (Q[:, :c].T @ v)
            nv = float(np.linalg.norm(v))
            if nv > 1e-8:
                Q[:, c] = v / nv
                return
            v = fresh()
        raise RuntimeError("no independent direction left")

    for l in range(b):
        put(l, V0[:, l] / max(np.linalg.norm(V0[:, l]), 1e-300))
    j0 = 0
    n_hvp = 0
    restarts = 0
    while True:
        m = m_max
        for j in range(j0, m_max):
            c = j + b
            w = op(Q[:, j])
            n_hvp += 1
            h = Q[:, :c].T @ w              # classical Gram-Schmidt, twice
            w = w - Q[:, :c] @ h
            h2 = Q[:, :c].T @ w
            w = w - Q[:, :c] @ h2
            h = h + h2
            T[:c, j] = h                    # column j of Q^T H Q
            T[j, :c] = h
            beta = float(np.linalg.norm(w))
            T[c, j] = T[j, c] = beta
            if beta <= 1e-14 * max(1.0, abs(h[j])):   # the block Krylov space is invariant
                m = j + 1
                break
            Q[:, c] = w / beta
        theta, Y = np.linalg.eigh(T[:m, :m])
        # H Q_m Y - Q_m Y diag(theta) = Q[:, m:m+b] T[m:m+b, :m] Y
        rn = np.linalg.norm(T[m:m + b, :m] @ Y, axis=0)
        conv = m >= k and bool(np.all(rn[:k] <= tol_abs))
        kk = min(keep, m)
        if conv or restarts >= max_restarts:
            X = Q[:, :m] @ Y[:, :kk]
            return theta[:kk], X, rn[:kk], restarts, n_hvp, conv
        # thick restart: the kk lowest Ritz vectors and the residual block
        # (re-orthonormalised; after a breakdown its dependent last column is
        # a fresh direction)
        restarts += 1
        Xk = Q[:, :m] @ Y[:, :kk]
        Rb = Q[:, m:m + b].copy()
        if m < m_max:
            Rb[:, b - 1] = fresh()
        Q[:] = 0.0
        Q[:, :kk] = Xk
        for l in range(b):
            put(kk + l, Rb[:, l])
        T[:] = 0.0
        T[np.arange(kk), np.arange(kk)] = theta[:kk]
        j0 = kk


def min_modes_lanczos(ham: Ham, m, k: int, tol: float = 1e-10, m_max: int = 32, keep: Optional[int] = None,
                      max_restarts: int = 100, mask=None, seed: int = 0, c=None, block: int = 2) -> EigResult:
    """k smallest eigenpairs of the (masked) tangent Hessian by FP64
    thick-restart band Lanczos (start block of `block` random vectors) in
    frame coordinates; same stopping rule and output conventions as
    min_modes."""
    m = _f64(m).reshape(3, ham.N)
    N = ham.N
    if c is None:
        c, _ = force(m, gradient(ham, m))
    act = np.ones(N, dtype=bool) if mask is None else np.asarray(mask).astype(bool)
    e1, e2 = frame(m)

    def op(y):
        y = y.copy()
        y[:N][~act] = 0.0
        y[N:][~act] = 0.0
        v = y[:N] * e1 + y[N:] * e2
        hv = tangent_hvp(ham, m, c, v[None], mask=None if mask is None else act.astype(np.uint8))[0]
        out = np.concatenate([(hv * e1).sum(0), (hv * e2).sum(0)])
        out[:N][~act] = 0.0
        out[N:][~act] = 0.0
        return out

    rng = np.random.default_rng(seed)

    def fresh():
        v = rng.standard_normal(2 * N)
        v[:N][~act] = 0.0
        v[N:][~act] = 0.0
        return v

    V0 = np.stack([fresh() for _ in range(block)], axis=1)
    lam, X, rn, it, n_hvp, conv = lanczos(op, V0, k, tol * ham.h_est(), m_max, keep, max_restarts, fresh)
    a = X[:, :k].T.reshape(k, 2, N)
    V = np.stack([sign_fix(a[j, 0] * e1 + a[j, 1] * e2) for j in range(k)])
    V = V / np.linalg.norm(V.reshape(k, -1), axis=1)[:, None, None]
    return EigResult(lam[:k].copy(), V, rn[:k].copy(), it, n_hvp, conv, X)


# ---------------------------------------------------------------------------
# Outer layer: reflected force, step rule, rotation retraction.
# ---------------------------------------------------------------------------
def reflected_force(F, V, k_reflect: int = 1) -> np.ndarray:
    """F_mmf = F - 2 sum_{r < k_reflect} (F . v_r) v_r (Results, Bilayer MMF
    equation; the subspace variant when k_reflect > 1)."""
    F = _f64(F)
    out = F.copy()
    for r in range(k_reflect):
        v = V[r]
        out -= 2.0 * float((F * v).sum()) * v
    return out


def rotate(m, d) -> np.ndarray:
    """Exponential-map retraction: m_i <- cos|d_i| m_i + sin|d_i| d_i/|d_i|,
    then renormalised."""
    m = _f64(m)
    d = _f64(d)
    th = np.sqrt((d * d).sum(0))
    safe = np.where(th > 0, th, 1.0)
    out = np.cos(th) * m + np.sin(th) * d / safe
    out = np.where(th > 0, out, m)
    return out / np.sqrt((out * out).sum(0))


CG_RESTART = 50   # conjugate-gradient restart period (steps)


@dataclass
class StepRule:
    """Outer optimiser (shared rule for climb and descent): L-BFGS two-loop on
    G (memory `mem`, projection transport of the stored pairs, pairs with
    s.y <= sy_min skipped, gamma = s.y / y.y of the newest valid pair,
    gamma0 = alpha0 when none; reset when the direction does not point along
    -G), or a fixed step alpha0 * (-G), or nonlinear conjugate gradients
    ("cg", the paper's second outer optimiser): p = -G + beta p_prev on the
    transported previous direction with the Fletcher-Reeves beta = |G|^2 /
    |P G_prev|^2, restarted (beta = 0) every CG_RESTART steps and whenever p
    is not a descent direction, step alpha0 p; then the per-spin rotation cap
    theta_max; no line search."""

    kind: str = "lbfgs"           # "lbfgs" | "fixed" | "cg"
    mem: int = 8
    theta_max: float = 0.1
    alpha0: Optional[float] = None  # default 1 / h_est
    sy_min: float = 1e-12


class LBFGS:
    def __init__(self, rule: StepRule, alpha0: float):
        self.rule = rule
        self.alpha0 = alpha0
        self.S: list = []
        self.Y: list = []
        self.d_prev = None
        self.G_prev = None
        self.c_prev = 1.0
        self.n_dir = 0   # directions computed so far

    def reset(self):
        self.S, self.Y = [], []

    def direction(self, m, G) -> np.ndarray:
        r = self.rule
        alpha_cg = None
        if r.kind == "fixed":
            d = -self.alpha0 * G
        elif r.kind == "cg":
            alpha_cg = self.alpha0
            p = -G
            if self.d_prev is not None and self.n_dir % CG_RESTART != 0:
                s = project(m, self.d_prev)          # = c_prev * (transported p_prev)
                gp = project(m, self.G_prev)
                gpgp = float((gp * gp).sum())
                beta = float((G * G).sum()) / gpgp if gpgp > 0.0 else 0.0
                p = -G + (beta / self.c_prev) * s
                if float((p * G).sum()) >= 0.0:
                    p = -G
            d = alpha_cg * p
        else:
            if self.d_prev is not None:
                self.S = [project(m, s) for s in self.S]
                self.Y = [project(m, y) for y in self.Y]
                s = project(m, self.d_prev)
                y = G - project(m, self.G_prev)
                self.S.append(s)
                self.Y.append(y)
                if len(self.S) > r.mem:
                    self.S.pop(0)
                    self.Y.pop(0)
            valid = [j for j in range(len(self.S))
                     if float((self.S[j] * self.Y[j]).sum()) > r.sy_min]
            q = G.copy()
            alph = {}
            for j in reversed(valid):
                rho = 1.0 / float((self.S[j] * self.Y[j]).sum())
                alph[j] = rho * float((self.S[j] * q).sum())
                q = q - alph[j] * self.Y[j]
            if valid:
                jn = valid[-1]
                gamma = float((self.S[jn] * self.Y[jn]).sum()) / float((self.Y[jn] * self.Y[jn]).sum())
            else:
                gamma = self.alpha0
            z = gamma * q
            for j in valid:
                rho = 1.0 / float((self.S[j] * self.Y[j]).sum())
                beta = rho * float((self.Y[j] * z).sum())
                z = z + (alph[j] - beta) * self.S[j]
            d = -z
            if float((d * G).sum()) >= 0.0:
                self.reset()
                d = -self.alpha0 * G
        d = project(m, d)
        th = np.sqrt((d * d).sum(0))
        tmax = float(th.max()) if th.size else 0.0
        cap = r.theta_max / tmax if tmax > r.theta_max else 1.0
        d = d * cap
        if alpha_cg is not None:
            self.c_prev = alpha_cg * cap   # the step taken is c_prev times the direction
        self.n_dir += 1
        self.d_prev = d
        self.G_prev = G.copy()
        return d


# Status codes (mirrors the values documented at the library boundary).
SADDLE, NOT_CONVERGED, DEGENERATE, HIGHER_INDEX, NAN_STATUS = 0, 1, 2, 3, 4


@dataclass
class SearchResult:
    status: int
    m: np.ndarray
    E: float
    fnorm: float
    iters: int
    n_hvp: int
    evals: np.ndarray
    V: np.ndarray
    trace: list


def certify(evals, tau_lam: float, converged: bool = True, n_negative: Optional[int] = None) -> int:
    """Index-1 signature lambda_1 < 0 < lambda_2 with tolerance tau_lam
    (Supplementary Note 1, item ii).  The two eigenvalues must come from a
    converged solve: an unconverged Ritz value only bounds its eigenvalue
    from above, so lambda_2 > tau_lam would not exclude a second negative
    mode -- such a point is NOT_CONVERGED.  n_negative, when given, is the
    exact count of tangent eigenvalues below -tau_lam (dense inertia); more
    than one makes the point HIGHER_INDEX whatever the two Ritz values say."""
    l1, l2 = float(evals[0]), float(evals[1])
    if not (np.isfinite(l1) and np.isfinite(l2)):
        return NAN_STATUS
    if not converged:
        return NOT_CONVERGED
    if n_negative is not None and n_negative >= 2:
        return HIGHER_INDEX
    if l1 < -tau_lam and l2 > tau_lam:
        return SADDLE if n_negative is None or n_negative == 1 else DEGENERATE
    if l2 < -tau_lam:
        return HIGHER_INDEX
    return DEGENERATE


DENSE_INERTIA_MAX_DOF = 2048   # tangent DOF up to which certification also counts negatives exactly


def negative_count(ham: Ham, m, tau_lam: float, mask=None) -> int:
    """Number of eigenvalues of the dense (masked) tangent Hessian below
    -tau_lam: the exact inertia the certification criterion asks for."""
    w = np.linalg.eigvalsh(dense_tangent_hessian(ham, m, mask=mask))
    return int((w < -tau_lam).sum())


def saddle_search(ham: Ham, m0, tau_F: float = 1e-6, k: int = 1, k_cert: int = 2,
                  eig_tol: float = 1e-10, eig_max_iter: int = 200, tau_lam: Optional[float] = None,
                  max_outer: int = 5000, rule: Optional[StepRule] = None, mask=None,
                  k_reflect: int = 1, seed: int = 0, trace: bool = False,
                  cert_max_iter: Optional[int] = None) -> SearchResult:
    """Bilayer MMF climb (Supplementary Note 1, Algorithm 1, bilayer-kernel
    loop): min mode -> force -> reflected force -> rotation step, until
    ||F_mmf||_2 <= tau_F; then a k_cert >= 2 solve certifies
    lambda_1 < 0 < lambda_2."""
    rule = rule or StepRule()
    hest = ham.h_est()
    alpha0 = rule.alpha0 if rule.alpha0 is not None else 1.0 / hest
    tau_lam = 1e-6 * hest if tau_lam is None else tau_lam
    opt = LBFGS(rule, alpha0)
    m = _f64(m0).reshape(3, ham.N).copy()
    m = m / np.sqrt((m * m).sum(0))
    act = None if mask is None else np.asarray(mask).astype(np.uint8)
    Xw = None
    n_hvp = 0
    tr = []
    status = NOT_CONVERGED
    fnorm = np.inf
    it = 0
    for it in range(max_outer + 1):
        E, g, c, F = energy_grad(ham, m)
        if act is not None:
            F = F * act
        er = min_modes(ham, m, k, tol=eig_tol, max_iter=eig_max_iter, mask=act, X0=Xw, seed=seed, c=c)
        Xw = er.X_block
        n_hvp += er.n_hvp
        Fm = reflected_force(F, er.V, k_reflect)
        fnorm = float(np.linalg.norm(Fm))
        if trace:
            tr.append((it, E, fnorm, float(er.evals[0])))
        if not np.isfinite(fnorm):
            status = NAN_STATUS
            break
        if fnorm <= tau_F:
            status = NOT_CONVERGED
            break
        if it == max_outer:
            break
        d = opt.direction(m, -Fm)
        if act is not None:
            d = d * act
        m = rotate(m, d)
    E, g, c, F = energy_grad(ham, m)
    kc = max(k_cert, 2)
    ec = min_modes(ham, m, kc, tol=eig_tol, max_iter=eig_max_iter if cert_max_iter is None else cert_max_iter,
                   mask=act, seed=seed + 1, c=c)
    n_hvp += ec.n_hvp
    if fnorm <= tau_F:
        n_act = ham.N if act is None else int(np.count_nonzero(act))
        n_neg = negative_count(ham, m, tau_lam, mask=act) if 2 * n_act <= DENSE_INERTIA_MAX_DOF else None
        status = certify(ec.evals, tau_lam, converged=ec.converged, n_negative=n_neg)
    return SearchResult(status, m, E, fnorm, it, n_hvp, ec.evals, ec.V, tr)


@dataclass
class DescentResult:
    m: np.ndarray
    E: float
    Q: float
    fnorm: float
    iters: int
    lam1: float
    converged: bool


def descend(ham: Ham, m_saddle, v1, sign: int, eta: float = 0.1, tau_F: float = 1e-6,
            max_outer: int = 5000, rule: Optional[StepRule] = None, eig_tol: float = 1e-10,
            mask=None, seed: int = 0) -> DescentResult:
    """Two-sided minimum-mode descent (Supplementary Note 1, item iii):
    displace the saddle along sign*v1, scaled so that the largest per-spin
    rotation is eta, then relax downhill with the same step rule on F
    (no reflection) until ||F||_2 <= tau_F."""
    rule = rule or StepRule()
    hest = ham.h_est()
    alpha0 = rule.alpha0 if rule.alpha0 is not None else 1.0 / hest
    opt = LBFGS(rule, alpha0)
    m = _f64(m_saddle).reshape(3, ham.N)
    v1 = _f64(v1).reshape(3, ham.N)
    vmax = float(np.sqrt((v1 * v1).sum(0)).max())
    m = rotate(m, (sign * eta / vmax) * v1)
    act = None if mask is None else np.asarray(mask).astype(np.uint8)
    fnorm = np.inf
    it = 0
    for it in range(max_outer + 1):
        E, g, c, F = energy_grad(ham, m)
        if act is not None:
            F = F * act
        fnorm = float(np.linalg.norm(F))
        if fnorm <= tau_F or it == max_outer or not np.isfinite(fnorm):
            break
        d = opt.direction(m, -F)
        if act is not None:
            d = d * act
        m = rotate(m, d)
    E, g, c, F = energy_grad(ham, m)
    er = min_modes(ham, m, 1, tol=eig_tol, mask=act, seed=seed, c=c)
    return DescentResult(m, E, topological_charge(ham, m), fnorm, it, float(er.evals[0]),
                         fnorm <= tau_F)


def max_site_angle(m1, m2) -> float:
    """Largest per-site angle between two spin configurations (dedupe metric)."""
    m1 = _f64(m1)
    m2 = _f64(m2)
    cr = np.cross(m1.T, m2.T)
    dt = (m1 * m2).sum(0)
    return float(np.arctan2(np.sqrt((cr * cr).sum(1)), dt).max())


# ---------------------------------------------------------------------------
# Explorer objectives (Methods, "Multi-objective initial-configuration
# explorer"; Supplementary Note 1, Algorithm 1 population loop; Results,
# "Multi-objective explorer over generations").  NSGA-II itself is not here:
# these are the per-candidate quantities it ranks.
# ---------------------------------------------------------------------------
def explorer_candidates(x0, deltas, mask=None) -> np.ndarray:
    """Candidates x = x0 + P_Omega delta followed by the projection onto the
    spin manifold (the Methods' candidate equation): on an active site the
    spin is (x0_i + delta_i) / |x0_i + delta_i|; an inactive site keeps x0_i,
    and so does an active site whose sum vanishes (no nearest unit vector).
    deltas: (P, 3, N) ambient perturbations.  Returns (P, 3, N)."""
    x0 = _f64(x0)
    N = x0.shape[1]
    D = _f64(deltas).reshape(-1, 3, N)
    act = np.ones(N, bool) if mask is None else np.asarray(mask).astype(bool)
    out = np.empty_like(D)
    for p in range(D.shape[0]):
        x = x0.copy()
        for i in range(N):
            if not act[i]:
                continue
            v = x0[:, i] + D[p][:, i]
            n = np.sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2])
            if n > 0.0:
                x[:, i] = v / n
        out[p] = x
    return out


def l1_distance_matrix(X, Y) -> np.ndarray:
    """D[p, q] = sum over sites and components |X_p - Y_q| (the l1 distance
    of the Results' diversity measures), one pair at a time."""
    X = _f64(X)
    Y = _f64(Y)
    X = X.reshape(X.shape[0], -1)
    Y = Y.reshape(Y.shape[0], X.shape[1])
    D = np.zeros((X.shape[0], Y.shape[0]))
    for p in range(X.shape[0]):
        for q in range(Y.shape[0]):
            D[p, q] = np.abs(X[p] - Y[q]).sum()
    return D


@dataclass
class ExplorerResult:
    X: np.ndarray          # (P, 3, N) candidates
    E: np.ndarray          # energies
    evals: np.ndarray      # (P, k) lowest eigenvalues of the (masked) tangent Hessian
    gap: np.ndarray        # lambda_2 - lambda_1
    Q: np.ndarray          # topological charges
    violation: np.ndarray  # |Q - Q_target|
    l1_sum: np.ndarray     # sum of l1 distances to the other candidates
    l1_min: np.ndarray     # smallest l1 distance to another candidate or an archive member
    D: np.ndarray          # (P, P + A) l1 distances to the candidates, then the archive
    converged: np.ndarray


def explorer_objectives(ham: Ham, x0, deltas, mask=None, archive=None, Q_target: Optional[float] = None,
                        k: int = 2, tol: float = 1e-10, max_iter: int = 200) -> ExplorerResult:
    """The three objectives of every candidate of a population (Methods,
    objectives (i)-(iii); Algorithm 1 evaluates them against S u A):
      (i)   diversity: l1 distances to the other candidates and to the
            archive A; per candidate their sum over the population and their
            minimum over S u A (the Results plot the total pairwise l1
            distance and the maximin distance);
      (ii)  feasibility: the topological-charge violation |Q(x) - Q_target|
            (Q_target = Q(x0) when not given);
      (iii) separability: the gap lambda_2 - lambda_1 of the two lowest
            eigenvalues of the tangent Hessian, restricted to the masked
            subspace when a mask is given (the subspace the climb then moves
            in), from the LOBPCG oracle."""
    x0 = _f64(x0).reshape(3, ham.N)
    X = explorer_candidates(x0, deltas, mask)
    P = X.shape[0]
    A = np.zeros((0, 3, ham.N)) if archive is None else _f64(archive).reshape(-1, 3, ham.N)
    qt = topological_charge(ham, x0) if Q_target is None else float(Q_target)
    E = np.array([energy(ham, X[p]) for p in range(P)])
    ev = np.zeros((P, k))
    conv = np.zeros(P, bool)
    for p in range(P):
        r = min_modes(ham, X[p], k, tol=tol, max_iter=max_iter, mask=mask)
        ev[p] = r.evals[:k]
        conv[p] = r.converged
    Q = np.array([topological_charge(ham, X[p]) for p in range(P)])
    D = np.concatenate([l1_distance_matrix(X, X), l1_distance_matrix(X, A)], axis=1)
    l1_sum = np.array([sum(D[p, q] for q in range(P) if q != p) for p in range(P)])
    l1_min = np.array([min([D[p, q] for q in range(P + A.shape[0]) if q != p], default=np.inf)
                       for p in range(P)])
    return ExplorerResult(X, E, ev, ev[:, 1] - ev[:, 0], Q, np.abs(Q - qt), l1_sum, l1_min, D, conv)
