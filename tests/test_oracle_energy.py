"""Pins of the oracle's exact quantities (energy, gradient, Hessian, charge,
shells) against closed forms, finite differences, identities and the paper's
Table S1.  CPU only."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2509_26269_amd import synth as S
from tests import closed_forms as CF

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _ham(p):
    return O.Ham(**p.asdict())


# --- lattice shells: Table S1 of Supplementary Note 4 -----------------------
def test_shells_match_table_s1():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table_s1_shells.txt")) if not l.startswith("#")]
    r_paper = np.array([float(r[0]) for r in rows])
    mult = [int(r[1]) for r in rows]
    offs = O.shells(len(rows))
    got_mult = [0] * len(rows)
    d = {}
    for dx, dy, s in offs:
        got_mult[s] += 1
        d[s] = np.sqrt(dx * dx + dx * dy + dy * dy)
    assert got_mult == mult
    assert sum(mult) == 360
    # printed distances are in units of a with NN distance a/sqrt(2)
    r_ours = np.array([d[s] for s in range(len(rows))]) / np.sqrt(2.0)
    assert np.allclose(r_ours, r_paper, atol=1e-6)


def test_first_three_shells_explicit():
    offs = O.shells(3)
    for s in range(3):
        got = sorted((dx, dy) for dx, dy, ss in offs if ss == s)
        assert got == sorted(CF.SHELL_OFFSETS[s])


# --- energy --------------------------------------------------------------------
@pytest.mark.parametrize("L", [6, 16])
def test_fm_energy_closed_form(L):
    p = S.ham_3shell(L)
    h = _ham(p)
    m = S.uniform(h.N)
    E = O.energy(h, m)
    assert E == pytest.approx(CF.fm_z_energy(h.N, p.J, p.K, p.B[2]), rel=1e-13)


@pytest.mark.parametrize("n1,n2", [(1, 0), (0, 1), (2, 1), (3, 0)])
def test_cycloid_energy_closed_form_fixes_dmi_sign(n1, n2):
    L = 12
    p = S.ham_3shell(L)
    h = _ham(p)
    m, q, _ = CF.cycloid_state(L, L, n1, n2)
    E = O.energy(h, m)
    Ecf = CF.cycloid_energy(L, L, n1, n2, p.J, p.D[0], p.K, p.B[2])
    assert E == pytest.approx(Ecf, rel=1e-12, abs=1e-10)
    # a Bloch helix (rotation plane perpendicular to q) has zero DMI energy
    qh = q / np.linalg.norm(q)
    perp = np.array([-qh[1], qh[0]])
    mb = np.stack([m[0] * 0 + (m[0] * qh[0] + m[1] * qh[1]) * perp[0],
                   (m[0] * qh[0] + m[1] * qh[1]) * perp[1], m[2]])
    assert abs(O.energy_terms(h, mb)[1]) < 1e-10
    # with D > 0 the Neel cycloid of the sense written above lowers the energy
    assert O.energy_terms(h, m)[1] < 0


def test_energy_identity_half_c_sum():
    """E is quadratic plus linear in m: E = 1/2 sum_i c_i - 1/2 B . sum_i m_i."""
    p = S.ham_3shell(10)
    h = _ham(p)
    m = S.random_texture(h.N, np.random.default_rng(3))
    E, g, c, F = O.energy_grad(h, m)
    rhs = 0.5 * c.sum() - 0.5 * np.dot(p.B, m.sum(1))
    assert E == pytest.approx(rhs, rel=1e-12)


def test_energy_linear_in_parameters():
    p = S.ham_3shell(9)
    p.D = [0.25, 0.07, -0.03]
    p.B = (0.01, -0.02, 0.03)
    h = _ham(p)
    m = S.random_texture(h.N, np.random.default_rng(4))
    dth = O.param_grad(h, m)
    th = h.theta()
    assert O.energy(h, m) == pytest.approx(float(th @ dth), rel=1e-12)
    # central differences in each parameter (exact: E is linear in theta)
    for i in range(len(th)):
        for step in (1e-3,):
            tp = th.copy()
            tm = th.copy()
            tp[i] += step
            tm[i] -= step
            ns = h.n_shells

            def mk(t):
                return O.Ham(h.Lx, h.Ly, list(t[:ns]), list(t[ns:2 * ns]), t[2 * ns], tuple(t[2 * ns + 1:]))

            fd = (O.energy(mk(tp), m) - O.energy(mk(tm), m)) / (2 * step)
            assert fd == pytest.approx(dth[i], rel=1e-9, abs=1e-8)


# --- gradient and Hessian -------------------------------------------------------
@pytest.mark.parametrize("L,shells", [(5, 1), (7, 3), (11, 3)])
def test_gradient_matches_energy_fd(L, shells):
    p = S.ham_3shell(L) if shells == 3 else S.ham_nn(L)
    p.B = (0.013, -0.021, 0.03)
    h = _ham(p)
    rng = np.random.default_rng(L)
    m = S.random_texture(h.N, rng)
    g = O.gradient(h, m)
    for _ in range(4):
        u = rng.standard_normal(m.shape)
        step = 1e-3
        fd = (O.energy(h, m + step * u) - O.energy(h, m - step * u)) / (2 * step)
        assert fd == pytest.approx(float((g * u).sum()), rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("L,shells", [(3, 1), (4, 3), (5, 3)])
def test_hessian_from_energy_matches_stencil(L, shells):
    """The Euclidean Hessian assembled from energies alone equals the scatter
    Hessian used by every HVP; small L exercises wrapped offsets."""
    p = S.ham_3shell(L) if shells == 3 else S.ham_nn(L)
    p.D = [0.3, 0.0, 0.0]
    h = _ham(p)
    m = S.random_texture(h.N, np.random.default_rng(1))
    H_fd = O.dense_hessian_fd(h, m, 1.0)
    A = O.dense_A(h)
    assert np.allclose(H_fd, A, atol=1e-10)
    assert np.allclose(A, A.T, atol=1e-14)


def test_force_tangent_and_critical_uniform_states():
    p = S.ham_3shell(8)
    h = _ham(p)
    m = S.random_texture(h.N, np.random.default_rng(2))
    _, g, c, F = O.energy_grad(h, m)
    assert np.abs((F * m).sum(0)).max() < 1e-13
    assert np.allclose(c, (m * g).sum(0))
    # uniform +z with B || z: critical point (sum of DMI vectors is zero)
    _, _, _, F0 = O.energy_grad(h, S.uniform(h.N))
    assert np.abs(F0).max() < 1e-13


def test_riemannian_hvp_matches_fd_of_riemannian_gradient():
    """Hess E[v] = P D(P g)[v] along the exponential retraction curve."""
    p = S.ham_3shell(9)
    h = _ham(p)
    rng = np.random.default_rng(5)
    m = S.random_texture(h.N, rng)
    _, g, c, _ = O.energy_grad(h, m)
    v = S.random_tangent(m, 1, rng)[0]
    Hv = O.tangent_hvp(h, m, c, v)
    step = 1e-4

    def rgrad(mm):
        gg = O.gradient(h, mm)
        return O.project(mm, gg)

    fd = O.project(m, (rgrad(O.rotate(m, step * v)) - rgrad(O.rotate(m, -step * v))) / (2 * step))
    rel = np.linalg.norm(fd - Hv) / np.linalg.norm(Hv)
    assert rel < 1e-7


def test_tangent_hvp_symmetric_and_masked():
    p = S.ham_3shell(8)
    h = _ham(p)
    rng = np.random.default_rng(6)
    m = S.random_texture(h.N, rng)
    _, _, c, _ = O.energy_grad(h, m)
    u, v = S.random_tangent(m, 2, rng)
    Hu = O.tangent_hvp(h, m, c, u)
    Hv = O.tangent_hvp(h, m, c, v)
    assert float((u * Hv).sum()) == pytest.approx(float((Hu * v).sum()), rel=1e-12)
    assert np.abs((Hv * m).sum(0)).max() < 1e-12
    mask = S.random_mask_disc(8, 8, 2.5)
    Hm = O.tangent_hvp(h, m, c, v, mask=mask)
    assert np.all(Hm[:, mask == 0] == 0)
    HT = O.dense_tangent_hessian(h, m, mask=mask)
    # principal-submatrix reading: apply to the frame basis of the active set
    act = np.nonzero(mask)[0]
    e1, e2 = O.frame(m)
    a = rng.standard_normal(2 * len(act))
    amb = np.zeros((3, h.N))
    amb[:, act] = a[: len(act)] * e1[:, act] + a[len(act):] * e2[:, act]
    w = O.tangent_hvp(h, m, c, amb, mask=mask)
    wa = np.concatenate([(w * e1).sum(0)[act], (w * e2).sum(0)[act]])
    assert np.allclose(wa, HT @ a, atol=1e-12)


def test_frame_orthonormal_everywhere():
    rng = np.random.default_rng(7)
    m = S.random_texture(4096, rng)
    m[:, :4] = np.array([[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, 1e-300, -1]]).T
    m = m / np.linalg.norm(m, axis=0)
    e1, e2 = O.frame(m)
    for a, b, val in [(e1, e1, 1), (e2, e2, 1), (e1, e2, 0), (e1, m, 0), (e2, m, 0)]:
        assert np.abs((a * b).sum(0) - val).max() < 1e-14
    v = S.random_tangent(m, 3, rng)
    assert np.allclose(O.from_frame(m, O.to_frame(m, v)), v, atol=1e-14)


# --- topological charge ----------------------------------------------------------
@pytest.mark.parametrize("kind,Q", [("skyrmion", 1), ("antiskyrmion", -1), ("biskyrmion", 2)])
def test_topological_charge_of_seeded_textures(kind, Q):
    L = 32
    m = S.three_shell_start(L, seed=0, kind=kind, R=3.0, sigma=0.0)
    assert O.topological_charge(L, m, L) == pytest.approx(Q, abs=1e-9)
    mn = S.three_shell_start(L, seed=1, kind=kind, R=3.0, sigma=0.05)
    assert O.topological_charge(L, mn, L) == pytest.approx(Q, abs=1e-6)


def test_topological_charge_uniform_zero():
    assert abs(O.topological_charge(8, S.uniform(64), 8)) < 1e-14
