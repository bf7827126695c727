"""Pins of the oracle in the many-shell regime (the Pd/Fe/Ir(111) exchange of
Table S1: 35 shells, 360 bonds), against closed forms whose offsets are
enumerated from the distances and bond counts printed in Table S1."""
import numpy as np
import pytest

import oracle as O
from paper_2509_26269_amd import synth as S
from tests import closed_forms as CF


def _ham(p):
    return O.Ham(**p.asdict())


def test_generator_matches_table_offsets():
    offs = O.shells(35)
    for s in range(35):
        got = sorted((dx, dy) for dx, dy, ss in offs if ss == s)
        assert got == sorted(CF.SHELL_OFFSETS_35[s])


@pytest.mark.parametrize("L", [24, 30])
def test_fm_energy_closed_form_35_shells(L):
    p = S.ham_pdfeir(L)
    h = _ham(p)
    E = O.energy(h, S.uniform(h.N))
    # the oracle sums 360 bonds per site one by one (3e5 terms at L = 30):
    # sequential FP64 rounding reaches ~1e-12 relative
    assert E == pytest.approx(CF.fm_z_energy(h.N, p.J, p.K, p.B[2]), rel=1e-11)


@pytest.mark.parametrize("n1,n2", [(1, 0), (2, 1), (0, 3)])
def test_cycloid_energy_closed_form_35_shells(n1, n2):
    L = 24
    p = S.ham_pdfeir(L)
    h = _ham(p)
    m, _, _ = CF.cycloid_state(L, L, n1, n2)
    E = O.energy(h, m)
    Ecf = CF.cycloid_energy(L, L, n1, n2, p.J, p.D[0], p.K, p.B[2])
    assert E == pytest.approx(Ecf, rel=1e-12, abs=1e-10)


def test_gradient_fd_35_shells():
    p = S.ham_pdfeir(24)
    p.B = (0.013, -0.021, 0.03)
    h = _ham(p)
    rng = np.random.default_rng(35)
    m = S.random_texture(h.N, rng)
    g = O.gradient(h, m)
    for _ in range(3):
        u = rng.standard_normal(m.shape)
        step = 1e-3
        fd = (O.energy(h, m + step * u) - O.energy(h, m - step * u)) / (2 * step)
        assert fd == pytest.approx(float((g * u).sum()), rel=1e-9, abs=1e-9)


def test_fm_spectrum_closed_form_35_shells():
    """Dense tangent Hessian at m = +z on 24 x 24: every eigenvalue is
    2 sum_s J_s S_s(k) + bz + 2K over the 35 Table S1 shells."""
    L = 24
    p = S.ham_pdfeir(L)
    h = _ham(p)
    H = O.dense_tangent_hessian(h, S.uniform(h.N))
    w = np.linalg.eigvalsh(H)
    ref = CF.fm_z_spectrum(L, L, p.J, p.K, p.B[2])
    assert np.abs(w - ref).max() <= 1e-12 * h.h_est()


def test_tangent_hvp_matches_dense_35_shells():
    p = S.ham_pdfeir(24)
    h = _ham(p)
    rng = np.random.default_rng(7)
    m = S.add_tilt_noise(S.uniform(h.N), 0.3, rng)
    _, _, c, _ = O.energy_grad(h, m)
    H = O.dense_tangent_hessian(h, m, c=c)
    v = O.project(m, rng.standard_normal(m.shape))
    hv_amb = O.tangent_hvp(h, m, c, v)
    hv_fr = O.to_frame(m, hv_amb)
    assert np.allclose(H @ O.to_frame(m, v).reshape(-1), hv_fr.reshape(-1), atol=1e-12 * h.h_est())
