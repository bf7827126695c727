"""Pins of the explorer-objective oracle (candidates x = x0 + P_Omega delta
projected onto the spin manifold; l1 diversity; topological-charge
feasibility; spectral gap lambda_2 - lambda_1) against closed forms, a
library routine and hand-computed values -- never against the oracle's own
formulas retyped."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle as O
from paper_2509_26269_amd import synth as S
from tests import closed_forms as CF


def test_candidates_closed_forms():
    N = 16
    z = S.uniform(N)
    t = 0.7
    d = np.zeros((4, 3, N))
    d[1] = 0.5 * z                       # radial: projects back onto x0
    d[2] = -z                            # vanishing sum: x0 kept
    d[3, 0] = t                          # tangent push along x
    X = O.explorer_candidates(z, d)
    assert np.array_equal(X[0], z) and np.allclose(X[1], z, atol=1e-15) and np.array_equal(X[2], z)
    ref = np.array([t, 0.0, 1.0]) / np.sqrt(1 + t * t)
    assert np.allclose(X[3], ref[:, None], atol=1e-15)
    # a mask freezes the inactive sites whatever delta holds there
    rng = np.random.default_rng(1)
    dr = rng.standard_normal((2, 3, N))
    mask = (np.arange(N) % 3 == 0).astype(np.uint8)
    Xm = O.explorer_candidates(z, dr, mask)
    assert np.array_equal(Xm[:, :, mask == 0], np.broadcast_to(z[:, mask == 0], Xm[:, :, mask == 0].shape))
    assert np.allclose((Xm * Xm).sum(1), 1.0, atol=1e-15)
    # the projection is the nearest unit vector: angle to x0 + delta is zero
    v = z[:, mask == 1] + dr[0][:, mask == 1]
    cosang = (Xm[0][:, mask == 1] * v).sum(0) / np.linalg.norm(v, axis=0)
    assert np.allclose(cosang, 1.0, atol=1e-14)


def test_l1_hand_computed_population_and_archive():
    """+z, -z and (x + z)/sqrt2 from x0 = +z, archive {+z}: per-site l1
    distances 2, 1 and 1 + sqrt2 (by hand)."""
    N = 12
    z = S.uniform(N)
    tgt = [S.uniform(N, (0, 0, -1)), S.uniform(N, (1 / np.sqrt(2), 0, 1 / np.sqrt(2)))]
    d = np.stack([np.zeros((3, N))] + [t - z for t in tgt])
    p = S.ham_nn(4, 3)
    h = O.Ham(**p.asdict())
    r = O.explorer_objectives(h, z, d, archive=z[None], k=2)
    r2 = np.sqrt(2.0)
    assert np.allclose(r.l1_sum, [3 * N, (3 + r2) * N, (2 + r2) * N], rtol=1e-14)
    assert np.allclose(r.l1_min, [0.0, 2 * N, N], atol=1e-12)
    assert np.allclose(r.D[:, 3], [0.0, 2 * N, N], atol=1e-12)


def test_l1_matrix_against_library_and_metric_axioms():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((5, 3, 20))
    Y = rng.standard_normal((3, 3, 20))
    D = O.l1_distance_matrix(X, Y)
    assert np.allclose(D, cdist(X.reshape(5, -1), Y.reshape(3, -1), metric="cityblock"), rtol=1e-13)
    DX = O.l1_distance_matrix(X, X)
    assert np.all(np.diag(DX) == 0) and np.allclose(DX, DX.T)
    for a in range(5):
        for b in range(5):
            for c in range(5):
                assert DX[a, c] <= DX[a, b] + DX[b, c] + 1e-12


def test_gap_closed_forms_stoner_wohlfarth():
    """Coherent-rotation model: at the saddle (uniform +x) the two lowest
    eigenvalues are b - 2K and b (gap 2K); at a minimum (h, 0, s), h = b/2K,
    they are 2K s^2 and 2K (gap b^2 / 2K)."""
    p = S.ham_sw(8)
    h = O.Ham(**p.asdict())
    b, K = p.B[0], p.K
    z = S.uniform(h.N)
    mp, _ = CF.sw_minima(b, K)
    d = np.stack([S.uniform(h.N, (1, 0, 0)) - z, S.uniform(h.N, tuple(mp)) - z])
    r = O.explorer_objectives(h, z, d, k=2, tol=1e-12)
    assert r.converged.all()
    s2 = 1 - (b / (2 * K)) ** 2
    assert np.allclose(r.evals[0], [b - 2 * K, b], atol=1e-10)
    assert np.allclose(r.evals[1], [2 * K * s2, 2 * K], atol=1e-10)
    assert np.allclose(r.gap, [2 * K, b * b / (2 * K)], atol=1e-10)


def test_gap_masked_matches_dense_spectrum():
    p = S.ham_nn(6)
    h = O.Ham(**p.asdict())
    x0 = S.nn_start(1, L=6, R=1.5)
    rng = np.random.default_rng(3)
    mask = S.random_mask_disc(6, 6, 2.0)
    d = 0.2 * rng.standard_normal((2, 3, h.N))
    r = O.explorer_objectives(h, x0, d, mask=mask, k=2, tol=1e-12)
    for q in range(2):
        w, _ = O.min_modes_dense(h, r.X[q], 2, mask=mask)
        assert np.allclose(r.evals[q], w, atol=1e-9)


def test_feasibility_topological_charge():
    """A skyrmion start (Q = +1) keeps Q under a zero perturbation and loses
    it when every spin is pushed to the uniform state."""
    L = 16
    p = S.ham_nn(L)
    h = O.Ham(**p.asdict())
    x0 = S.skyrmion(L, L, 3.0)
    assert abs(O.topological_charge(h, x0) - 1.0) < 1e-9
    d = np.stack([np.zeros_like(x0), S.uniform(h.N) - x0])
    r = O.explorer_objectives(h, x0, d, k=2)
    assert np.allclose(r.Q, [1.0, 0.0], atol=1e-9)
    assert np.allclose(r.violation, [0.0, 1.0], atol=1e-9)
    r = O.explorer_objectives(h, x0, d, Q_target=0.0, k=2)
    assert np.allclose(r.violation, [1.0, 0.0], atol=1e-9)
