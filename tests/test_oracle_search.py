"""Pins of the oracle's outer layer: reflected-force algebra, the rotation
retraction, the climb to an index-1 saddle (closed-form Stoner-Wohlfarth
saddle, exact inertia count) and the two-sided descent.  CPU."""
import numpy as np
import pytest

import oracle as O
from paper_2509_26269_amd import synth as S
from tests import closed_forms as CF


def _ham(p):
    return O.Ham(**p.asdict())


def test_reflected_force_is_a_reflection():
    rng = np.random.default_rng(0)
    m = S.random_texture(64, rng)
    F, v = S.random_tangent(m, 2, rng)
    v = v / np.linalg.norm(v)
    Fm = O.reflected_force(F, v[None])
    assert np.linalg.norm(Fm) == pytest.approx(np.linalg.norm(F), rel=1e-14)
    assert float((Fm * v).sum()) == pytest.approx(-float((F * v).sum()), rel=1e-13)
    assert np.allclose(O.reflected_force(F, -v[None]), Fm, atol=1e-15)
    # component orthogonal to v unchanged
    perp = F - float((F * v).sum()) * v
    assert np.allclose(Fm - float((Fm * v).sum()) * v, perp, atol=1e-14)


def test_rotation_retraction():
    rng = np.random.default_rng(1)
    m = S.random_texture(128, rng)
    d = S.random_tangent(m, 1, rng)[0] * 0.3
    r = O.rotate(m, d)
    assert np.abs(np.linalg.norm(r, axis=0) - 1).max() < 1e-15
    # exact angle: the rotation by d_i turns m_i by |d_i|
    ang = np.arccos(np.clip((r * m).sum(0), -1, 1))
    assert np.allclose(ang, np.linalg.norm(d, axis=0), atol=1e-7)
    # first order: R(h d) = m + h d + O(h^2)
    h = 1e-6
    assert np.abs((O.rotate(m, h * d) - m) / h - d).max() < 1e-5


def test_step_cap_and_fixed_step():
    rng = np.random.default_rng(2)
    m = S.random_texture(32, rng)
    G = S.random_tangent(m, 1, rng)[0]
    opt = O.LBFGS(O.StepRule(kind="fixed", theta_max=0.05), alpha0=10.0)
    d = opt.direction(m, G)
    assert np.linalg.norm(d, axis=0).max() == pytest.approx(0.05, rel=1e-12)
    assert float((d * G).sum()) < 0


def test_stoner_wohlfarth_saddle_and_minima_closed_form():
    """Uniform m = x with B = b x, easy axis z, D = 0, 0 < b < 2K: the
    coherent-rotation saddle (lambda_1 = b - 2K, lambda_2 = b) and minima
    (h, 0, +-sqrt(1 - h^2)), h = b / 2K, barrier N K (1 - h)^2."""
    p = S.ham_sw(8)
    h = _ham(p)
    b, K = p.B[0], p.K
    m0 = S.add_tilt_noise(S.uniform(h.N, (1, 0, 0)), 0.02, np.random.default_rng(0))
    r = O.saddle_search(h, m0, tau_F=1e-8)
    assert r.status == O.SADDLE
    assert np.abs(r.m - S.uniform(h.N, (1, 0, 0))).max() < 1e-6
    assert r.evals[0] == pytest.approx(b - 2 * K, abs=1e-8)
    assert r.evals[1] == pytest.approx(b, abs=1e-8)
    mp, mm = CF.sw_minima(b, K)
    seen = []
    for sgn in (+1, -1):
        d = O.descend(h, r.m, r.V[0], sgn, tau_F=1e-8)
        assert d.converged and d.lam1 > 0
        assert r.E - d.E == pytest.approx(CF.sw_barrier(h.N, b, K), rel=1e-9)
        dev = min(np.abs(d.m - mp[:, None]).max(), np.abs(d.m - mm[:, None]).max())
        assert dev < 1e-6
        seen.append(np.sign(d.m[2, 0]))
    assert sorted(seen) == [-1, 1]  # the two sides reach the two distinct minima


@pytest.mark.parametrize("seed", [0])
def test_collapse_saddle_is_index_one_by_exact_inertia(seed):
    """NN model 16x16, radius-1 start: the climb reaches a saddle whose dense
    tangent Hessian has exactly one negative eigenvalue; both descents go
    downhill, one of them to the skyrmion (Q = 1)."""
    p = S.ham_nn(16)
    h = _ham(p)
    m0 = S.add_tilt_noise(S.skyrmion(16, 16, 1.0), 0.05, np.random.default_rng(seed))
    r = O.saddle_search(h, m0, tau_F=1e-6)
    assert r.status == O.SADDLE
    w = np.linalg.eigvalsh(O.dense_tangent_hessian(h, r.m))
    tau = 1e-6 * h.h_est()
    assert int((w < -tau).sum()) == 1
    assert np.allclose(r.evals, w[:2], atol=1e-8)
    Es = []
    Qs = []
    for sgn in (+1, -1):
        d = O.descend(h, r.m, r.V[0], sgn, tau_F=1e-6)
        assert d.converged
        assert d.lam1 >= -tau
        Es.append(d.E)
        Qs.append(round(d.Q))
    assert r.E > max(Es)
    assert 1 in Qs


def test_literal_start_is_degenerate_goldstone_point():
    """NN model 16x16, radius-3 start: the climb stalls at the translated
    relaxed skyrmion, a point with two near-zero (Goldstone) modes."""
    p = S.ham_nn(16)
    h = _ham(p)
    r = O.saddle_search(h, S.nn_start(0), tau_F=1e-6)
    assert r.status == O.DEGENERATE
    assert np.all(np.abs(r.evals) < 1e-6 * h.h_est())
    assert abs(O.topological_charge(h, r.m) - 1) < 1e-6


def test_dedupe_metric():
    rng = np.random.default_rng(3)
    m = S.random_texture(50, rng)
    assert O.max_site_angle(m, m) < 1e-7
    d = S.random_tangent(m, 1, rng)[0]
    d = 0.01 * d / np.linalg.norm(d, axis=0).max()
    assert O.max_site_angle(m, O.rotate(m, d)) == pytest.approx(0.01, rel=1e-6)


# --- the second outer optimiser: nonlinear conjugate gradients ------------
def test_cg_rule_stoner_wohlfarth_closed_form():
    """The CG rule climbs to the coherent-rotation saddle and both descents
    reach the closed-form minima with the closed-form barrier."""
    p = S.ham_sw(8)
    h = _ham(p)
    b, K = p.B[0], p.K
    cg = O.StepRule(kind="cg")
    m0 = S.add_tilt_noise(S.uniform(h.N, (1, 0, 0)), 0.02, np.random.default_rng(0))
    r = O.saddle_search(h, m0, tau_F=1e-8, rule=cg)
    assert r.status == O.SADDLE
    assert r.evals[0] == pytest.approx(b - 2 * K, abs=1e-8)
    assert r.evals[1] == pytest.approx(b, abs=1e-8)
    mp, mm = CF.sw_minima(b, K)
    for sgn in (+1, -1):
        d = O.descend(h, r.m, r.V[0], sgn, tau_F=1e-8, rule=cg)
        assert d.converged and d.lam1 > 0
        assert r.E - d.E == pytest.approx(CF.sw_barrier(h.N, b, K), rel=1e-9)
        assert min(np.abs(d.m - mp[:, None]).max(), np.abs(d.m - mm[:, None]).max()) < 1e-6


def test_cg_rule_first_step_is_steepest_and_beta_is_fletcher_reeves():
    """First step: alpha0 (-G).  Second step written out by hand from the
    transported quantities: beta = |G|^2 / |P G_prev|^2, p = -G + beta
    P p_prev, step alpha0 p; the restart period resets to steepest."""
    p = S.ham_nn(8)
    h = _ham(p)
    m = S.nn_start(4, L=8)
    rule = O.StepRule(kind="cg", theta_max=10.0)
    a0 = 1.0 / h.h_est()
    opt = O.LBFGS(rule, a0)
    G1 = -O.energy_grad(h, m)[3]
    d1 = opt.direction(m, G1)
    assert np.allclose(d1, O.project(m, -a0 * G1), atol=1e-15)
    m2 = O.rotate(m, d1)
    G2 = -O.energy_grad(h, m2)[3]
    d2 = opt.direction(m2, G2)
    gp = O.project(m2, G1)
    beta = float((G2 * G2).sum()) / float((gp * gp).sum())
    p_prev = O.project(m2, -G1)                 # the first direction, transported
    pdir = -G2 + beta * p_prev
    if float((pdir * G2).sum()) >= 0:
        pdir = -G2
    assert np.allclose(d2, O.project(m2, a0 * pdir), rtol=1e-10, atol=1e-14)
    # at the restart period the direction is steepest again
    opt.n_dir = O.CG_RESTART
    m3 = O.rotate(m2, d2)
    G3 = -O.energy_grad(h, m3)[3]
    assert np.allclose(opt.direction(m3, G3), O.project(m3, -a0 * G3), atol=1e-15)


def test_cg_rule_reaches_an_index_one_saddle_by_exact_inertia():
    p = S.ham_nn(16)
    h = _ham(p)
    m0 = S.add_tilt_noise(S.skyrmion(16, 16, 1.0), 0.05, np.random.default_rng(0))
    r = O.saddle_search(h, m0, tau_F=1e-6, rule=O.StepRule(kind="cg"))
    assert r.status == O.SADDLE
    w = np.linalg.eigvalsh(O.dense_tangent_hessian(h, r.m))
    assert int((w < -1e-6 * h.h_est()).sum()) == 1


# --- the L-BFGS two-loop rule (Methods, outer ascent optimisers) -----------
def _tangent_pairs(m, n, rng, scale=1.0):
    """n random tangent pairs (s, y) at m with s.y > 0: y = B s + small noise
    for a random symmetric positive definite B acting per site."""
    N = m.shape[1]
    pairs = []
    for _ in range(n):
        s = O.project(m, rng.standard_normal((3, N))) * scale
        y = O.project(m, 2.0 * s + 0.3 * O.project(m, rng.standard_normal((3, N))) * scale)
        assert float((s * y).sum()) > 0
        pairs.append((s, y))
    return pairs


def _preloaded(m, pairs, alpha0=0.05):
    """An optimiser whose history holds `pairs` at m and no pending step (so
    a call of direction() runs the two-loop on exactly these pairs)."""
    opt = O.LBFGS(O.StepRule(kind="lbfgs", mem=8, theta_max=1e9), alpha0)
    opt.S = [s.copy() for s, _ in pairs]
    opt.Y = [y.copy() for _, y in pairs]
    return opt


def _dense_lbfgs(pairs, gamma):
    """The L-BFGS inverse-Hessian approximation as a dense matrix, built by
    applying the BFGS update H <- V^T H V + rho s s^T, V = I - rho y s^T, for
    every pair from the oldest to the newest, starting from gamma I
    (Nocedal & Wright, Numerical Optimization, Eq. 7.19 expanded)."""
    n = pairs[0][0].size
    H = gamma * np.eye(n)
    for s, y in pairs:
        s, y = s.reshape(-1), y.reshape(-1)
        rho = 1.0 / float(s @ y)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


def test_lbfgs_secant_condition_on_the_newest_pair():
    """The two-loop matrix H maps the newest y onto the newest s, whatever the
    older pairs and the initial scaling: d(G = y_new) = -s_new."""
    rng = np.random.default_rng(10)
    m = S.random_texture(16, rng)
    for n in (1, 2, 3, 5):
        pairs = _tangent_pairs(m, n, rng)
        opt = _preloaded(m, pairs)
        d = opt.direction(m, pairs[-1][1].copy())
        assert np.allclose(d, -pairs[-1][0], rtol=1e-11, atol=1e-13), n


def test_lbfgs_two_pair_step_written_out_densely():
    """Two stored pairs: the direction equals -H G with H the dense BFGS
    recursion from gamma I, gamma = s.y / y.y of the NEWEST pair; a wrong
    gamma (the oldest pair's) or a reversed pair order gives another step."""
    rng = np.random.default_rng(11)
    m = S.random_texture(12, rng)
    pairs = _tangent_pairs(m, 2, rng)
    G = O.project(m, rng.standard_normal(m.shape))
    s1, y1 = pairs[-1]
    gamma = float((s1 * y1).sum()) / float((y1 * y1).sum())
    want = -(_dense_lbfgs(pairs, gamma) @ G.reshape(-1)).reshape(G.shape)
    d = _preloaded(m, pairs).direction(m, G.copy())
    assert np.allclose(d, want, rtol=1e-10, atol=1e-13)
    s0, y0 = pairs[0]
    wrong_gamma = float((s0 * y0).sum()) / float((y0 * y0).sum())
    alt1 = -(_dense_lbfgs(pairs, wrong_gamma) @ G.reshape(-1)).reshape(G.shape)
    alt2 = -(_dense_lbfgs(pairs[::-1], gamma) @ G.reshape(-1)).reshape(G.shape)
    assert np.abs(alt1 - want).max() > 1e-3 * np.abs(want).max()
    assert np.abs(alt2 - want).max() > 1e-3 * np.abs(want).max()


def test_lbfgs_first_step_and_curvature_skip():
    """No pairs: d = -alpha0 G.  A pair with s.y <= sy_min is left out of the
    recursion: the direction equals the one computed without it."""
    rng = np.random.default_rng(12)
    m = S.random_texture(10, rng)
    G = O.project(m, rng.standard_normal(m.shape))
    opt = O.LBFGS(O.StepRule(kind="lbfgs", theta_max=1e9), 0.05)
    assert np.allclose(opt.direction(m, G.copy()), -0.05 * G, atol=1e-15)
    good = _tangent_pairs(m, 2, rng)
    s_bad = O.project(m, rng.standard_normal(m.shape))
    y_bad = -s_bad  # s.y < 0
    mixed = [good[0], (s_bad, y_bad), good[1]]
    d_mixed = _preloaded(m, mixed).direction(m, G.copy())
    d_good = _preloaded(m, good).direction(m, G.copy())
    assert np.allclose(d_mixed, d_good, rtol=1e-12, atol=1e-15)


def test_lbfgs_direction_is_descent_and_reset_clears_history():
    """With curvature-valid pairs the two-loop matrix is positive definite,
    so d.G < 0 for every nonzero G and the reset branch is not taken; when G
    vanishes d.G = 0 triggers the reset: history cleared, d = -alpha0 G = 0."""
    rng = np.random.default_rng(13)
    m = S.random_texture(10, rng)
    for trial in range(5):
        pairs = _tangent_pairs(m, 4, rng)
        G = O.project(m, rng.standard_normal(m.shape))
        opt = _preloaded(m, pairs)
        d = opt.direction(m, G.copy())
        assert float((d * G).sum()) < 0
        assert len(opt.S) == 4
        assert np.all(np.linalg.eigvalsh(_dense_lbfgs(pairs, 0.7)) > 0)
    opt = _preloaded(m, _tangent_pairs(m, 3, rng))
    d = opt.direction(m, np.zeros_like(m))
    assert np.all(d == 0.0) and opt.S == [] and opt.Y == []


def test_lbfgs_projection_transport_and_memory():
    """After a rotation the stored pairs are projected onto the new tangent
    spaces, the new pair is (P d_prev, G - P G_prev), and the ring keeps the
    `mem` newest pairs."""
    p = S.ham_nn(8)
    h = _ham(p)
    m = S.nn_start(2, L=8)
    rule = O.StepRule(kind="lbfgs", mem=2, theta_max=0.05)
    opt = O.LBFGS(rule, 1.0 / h.h_est())
    hist_s, hist_y = [], []
    prev = None
    for step in range(4):
        G = -O.energy_grad(h, m)[3]
        if prev is not None:
            d_prev, G_prev = prev
            hist_s = [O.project(m, s) for s in hist_s] + [O.project(m, d_prev)]
            hist_y = [O.project(m, y) for y in hist_y] + [G - O.project(m, G_prev)]
            hist_s, hist_y = hist_s[-2:], hist_y[-2:]
        d = opt.direction(m, G.copy())
        assert len(opt.S) == len(hist_s) <= 2
        for a, b in zip(opt.S + opt.Y, hist_s + hist_y):
            assert np.allclose(a, b, rtol=1e-13, atol=1e-15)
            assert np.abs((a * m).sum(0)).max() < 1e-13   # tangent at the current m
        prev = (d.copy(), G.copy())
        m = O.rotate(m, d)


# --- certification needs a converged solve (Supplementary Note 1, item ii) --
def test_certify_rejects_unconverged_and_counts_inertia():
    tau = 1e-3
    assert O.certify([-1.0, 0.5], tau) == O.SADDLE
    # an unconverged solve only bounds the eigenvalues from above
    assert O.certify([-1.0, 0.5], tau, converged=False) == O.NOT_CONVERGED
    # the exact inertia overrides the two Ritz values
    assert O.certify([-1.0, 0.5], tau, n_negative=2) == O.HIGHER_INDEX
    assert O.certify([-1.0, 0.5], tau, n_negative=1) == O.SADDLE
    assert O.certify([-1.0, -0.5], tau) == O.HIGHER_INDEX
    assert O.certify([-1e-4, 0.5], tau) == O.DEGENERATE
    assert O.certify([np.nan, 0.5], tau) == O.NAN_STATUS


def test_search_with_capped_certifying_solve_is_not_a_saddle():
    """Stoner-Wohlfarth climb to the coherent-rotation saddle whose final
    k = 2 solve is capped at one iteration: from a random block it cannot
    converge, so the point is not certified, although it is index 1 (the
    uncapped search certifies it)."""
    p = S.ham_sw(8)
    h = _ham(p)
    m0 = S.add_tilt_noise(S.uniform(h.N, (1, 0, 0)), 0.02, np.random.default_rng(0))
    r = O.saddle_search(h, m0, tau_F=1e-8, cert_max_iter=1)
    assert r.fnorm <= 1e-8
    assert r.status == O.NOT_CONVERGED
    assert O.negative_count(h, r.m, 1e-6 * h.h_est()) == 1
    assert O.saddle_search(h, m0, tau_F=1e-8).status == O.SADDLE
