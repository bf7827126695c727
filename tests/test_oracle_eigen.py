"""Pins of the oracle's inner layer (dense Jacobi, LOBPCG) against a library
eigensolver, the closed-form ferromagnet spectra and residual bounds.  CPU."""
import numpy as np
import pytest

import oracle as O
from paper_2509_26269_amd import synth as S
from tests import closed_forms as CF


def _ham(p):
    return O.Ham(**p.asdict())


def test_jacobi_matches_library_eigh():
    rng = np.random.default_rng(0)
    for n in (1, 2, 7, 40):
        X = rng.standard_normal((n, n))
        A = X + X.T
        w, V = O.jacobi_eigh(A)
        assert np.allclose(w, np.linalg.eigvalsh(A), atol=1e-12 * max(1, np.abs(w).max()))
        assert np.allclose(V.T @ V, np.eye(n), atol=1e-12)
        assert np.allclose(A @ V, V * w, atol=1e-11)
    # exactly degenerate spectrum
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    d = np.array([1.0] * 4 + [2.0] * 6 + [-3.0] * 2)
    w, V = O.jacobi_eigh(Q @ np.diag(d) @ Q.T)
    assert np.allclose(w, np.sort(d), atol=1e-13)


@pytest.mark.parametrize("L", [6, 8])
def test_fm_z_full_spectrum_closed_form(L):
    p = S.ham_3shell(L)
    h = _ham(p)
    HT = O.dense_tangent_hessian(h, S.uniform(h.N))
    w = np.linalg.eigvalsh(HT) if L > 6 else O.jacobi_eigh(HT)[0]
    ref = CF.fm_z_spectrum(L, L, p.J, p.K, p.B[2])
    assert np.abs(w - ref).max() < 1e-12 * h.h_est()


@pytest.mark.parametrize("D1", [0.0, 0.3])
def test_fm_x_full_spectrum_closed_form_pins_dmi(D1):
    L = 8
    p = S.HamParams(L, L, [1.0], [D1], 0.05, (0.7, 0.0, 0.0))
    h = _ham(p)
    HT = O.dense_tangent_hessian(h, S.uniform(h.N, (1, 0, 0)))
    w = np.linalg.eigvalsh(HT)
    ref = CF.fm_x_spectrum(L, L, p.J, D1, p.K, p.B[0])
    assert np.abs(w - ref).max() < 1e-12 * h.h_est()


def test_tangent_spectrum_independent_of_frame():
    p = S.ham_3shell(6)
    h = _ham(p)
    rng = np.random.default_rng(9)
    m = S.random_texture(h.N, rng)
    HT = O.dense_tangent_hessian(h, m)
    # a second orthonormal tangent basis: rotate each frame by a random angle
    e1, e2 = O.frame(m)
    ang = rng.uniform(0, 2 * np.pi, h.N)
    f1 = np.cos(ang) * e1 + np.sin(ang) * e2
    f2 = -np.sin(ang) * e1 + np.cos(ang) * e2
    A = O.dense_A(h)
    _, _, c, _ = O.energy_grad(h, m)
    N = h.N
    U = np.zeros((3 * N, 2 * N))
    for i in range(N):
        for comp in range(3):
            U[comp * N + i, i] = f1[comp, i]
            U[comp * N + i, N + i] = f2[comp, i]
    H2 = U.T @ A @ U - np.diag(np.concatenate([c, c]))
    assert np.allclose(np.linalg.eigvalsh(HT), np.linalg.eigvalsh(0.5 * (H2 + H2.T)), atol=1e-12)


def test_lobpcg_matches_jacobi_random_texture():
    p = S.ham_3shell(8)
    h = _ham(p)
    m = S.random_texture(h.N, np.random.default_rng(11))
    wd, Vd = O.min_modes_dense(h, m, 4)
    r = O.min_modes(h, m, 4, tol=1e-11)
    assert r.converged
    assert np.abs(r.evals - wd).max() < 1e-9 * h.h_est()
    for j in range(4):
        assert abs(float((r.V[j] * Vd[j]).sum())) > 1 - 1e-8
        assert r.resid[j] <= 1e-11 * h.h_est()


def test_lobpcg_skyrmion_matches_library_eigh_and_residual_bound():
    p = S.ham_nn(16)
    h = _ham(p)
    m = S.nn_start(0)
    HT = O.dense_tangent_hessian(h, m)
    w = np.linalg.eigvalsh(HT)
    r = O.min_modes(h, m, 2, tol=1e-10)
    assert r.converged
    # an eigenvalue lies within ||r|| of every Ritz value of a symmetric matrix
    for j in range(2):
        assert np.min(np.abs(w - r.evals[j])) <= r.resid[j] + 1e-12
    assert np.allclose(r.evals, w[:2], atol=1e-9)


def test_lobpcg_masked_matches_dense_masked():
    L = 12
    p = S.ham_nn(L)
    h = _ham(p)
    m = S.nn_start(3, L=L)
    mask = S.random_mask_disc(L, L, 3.5)
    wd, Vd = O.min_modes_dense(h, m, 2, mask=mask)
    r = O.min_modes(h, m, 2, tol=1e-11, mask=mask)
    assert r.converged
    assert np.allclose(r.evals, wd, atol=1e-9)
    assert np.all(r.V[:, :, mask == 0] == 0)
    assert abs(float((r.V[0] * Vd[0]).sum())) > 1 - 1e-8


def test_lobpcg_fm_closed_form_large_lattice():
    """48x48, three shells: the k = 4 lowest eigenvalues equal the closed form.
    The 4th eigenvalue sits inside a 12-fold cluster, so the block carries
    guard vectors past the whole cluster."""
    L = 48
    p = S.ham_3shell(L)
    h = _ham(p)
    ref = CF.fm_z_spectrum(L, L, p.J, p.K, p.B[2])[:4]
    r = O.min_modes(h, S.uniform(h.N), 4, tol=1e-9, max_iter=400, guard=12)
    assert r.converged
    assert np.abs(r.evals - ref).max() < 1e-8 * h.h_est()


def test_sign_rule():
    v = np.zeros((3, 4))
    v[1, 2] = -0.8
    v[2, 3] = 0.8
    v[0, 0] = 0.1
    out = O.sign_fix(v)
    assert out[1, 2] == 0.8  # first of the tied largest components made positive


# --- thick-restart Lanczos (second inner solver) ---------------------------
def test_lanczos_matches_jacobi_random_texture_with_restarts():
    """A small Krylov depth forces several thick restarts."""
    p = S.ham_3shell(8)
    h = _ham(p)
    m = S.random_texture(h.N, np.random.default_rng(11))
    wd, Vd = O.min_modes_dense(h, m, 4)
    r = O.min_modes_lanczos(h, m, 4, tol=1e-11, m_max=12, keep=6)
    assert r.converged and r.iters >= 2
    assert np.abs(r.evals - wd).max() < 1e-9 * h.h_est()
    for j in range(4):
        assert abs(float((r.V[j] * Vd[j]).sum())) > 1 - 1e-8


def test_lanczos_residual_estimate_is_the_true_residual():
    p = S.ham_nn(16)
    h = _ham(p)
    m = S.nn_start(0)
    r = O.min_modes_lanczos(h, m, 2, tol=1e-9, m_max=20)
    assert r.converged
    _, _, c, _ = O.energy_grad(h, m)
    HV = O.tangent_hvp(h, m, c, r.V)
    for j in range(2):
        true = np.linalg.norm(HV[j] - r.evals[j] * r.V[j])
        assert abs(true - r.resid[j]) <= 1e-9 * h.h_est() + 1e-3 * true


def test_lanczos_masked_matches_dense_masked():
    L = 12
    p = S.ham_nn(L)
    h = _ham(p)
    m = S.nn_start(3, L=L)
    mask = S.random_mask_disc(L, L, 3.5)
    wd, Vd = O.min_modes_dense(h, m, 2, mask=mask)
    r = O.min_modes_lanczos(h, m, 2, tol=1e-11, mask=mask, m_max=16)
    assert r.converged
    assert np.allclose(r.evals, wd, atol=1e-9)
    assert np.all(r.V[:, :, mask == 0] == 0)
    assert abs(float((r.V[0] * Vd[0]).sum())) > 1 - 1e-8


def test_lanczos_fm_closed_form_and_lobpcg_agree():
    """24x24 three-shell ferromagnet: the 4 lowest eigenvalues (2-fold pairs)
    equal the closed form, and the two independent solvers agree."""
    L = 24
    p = S.ham_3shell(L)
    h = _ham(p)
    ref = CF.fm_z_spectrum(L, L, p.J, p.K, p.B[2])[:4]
    r = O.min_modes_lanczos(h, S.uniform(h.N), 4, tol=1e-9, m_max=40, keep=16, max_restarts=200)
    assert r.converged
    assert np.abs(r.evals - ref).max() < 1e-8 * h.h_est()
    m = S.three_shell_start(L, seed=5)
    a = O.min_modes_lanczos(h, m, 2, tol=1e-9, m_max=32)
    b = O.min_modes(h, m, 2, tol=1e-9, max_iter=400)
    assert a.converged and b.converged
    assert np.abs(a.evals - b.evals).max() < 1e-8 * h.h_est()
