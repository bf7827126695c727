"""GPU parity of the inner layer (moto_min_modes: block LOBPCG with device
Rayleigh-Ritz) against the FP64 oracle and the closed-form ferromagnet
spectrum.

Eigenvalues: |d lambda| <= 1e-5 max(|lambda|, h_est) (and 1e-5 |lambda| for
|lambda| >= 1e-3 h_est) in FP64; vectors 1 - |cos| <= 1e-8 (FP64) or
sin(angle) <= 1e-3 (FP32) where the gap is >= 1e-3 h_est."""
import numpy as np
import pytest

import oracle as O
from paper_2509_26269_amd import synth as S
from tests import closed_forms as CF
from tests import parity as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _M():
    from paper_2509_26269_amd import moto as M

    return M


def _dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _np(t):
    return t.detach().double().cpu().numpy()


def _check_pairs(ev, V, ref_ev, ref_V, hest, fp32, gap_ok):
    for j in range(len(ref_ev)):
        assert abs(ev[j] - ref_ev[j]) <= P.eig_bar(ref_ev[j], hest, not fp32), (j, ev[j], ref_ev[j])
        if gap_ok[j]:
            cos = abs(float((V[j] * ref_V[j]).sum()))
            if fp32:
                assert np.sqrt(max(0.0, 1 - cos * cos)) <= 1e-3
            else:
                assert 1 - cos <= 1e-8


@pytest.mark.parametrize("k", [1, 2, 4])
def test_min_modes_fp64_matches_oracle_nn16(k):
    M = _M()
    p = S.ham_nn(16)
    h = O.Ham(**p.asdict())
    plan = M.Plan.from_params(p)
    m = S.nn_start(0)
    r = M.moto_min_modes(plan, _dev(m), k, M.MOTO_F64, opts=M.eig_opts(M.MOTO_F64, tol=1e-10))
    assert r.status == M.CONVERGED
    ro = O.min_modes(h, m, k + 2, tol=1e-11)
    w = ro.evals
    gaps = [min(abs(w[j] - w[i]) for i in range(len(w)) if i != j) >= 1e-3 * h.h_est() for j in range(k)]
    _check_pairs(_np(r.evals), _np(r.V), w[:k], ro.V[:k], h.h_est(), False, gaps)
    assert np.all(_np(r.resid) <= 1e-10 * h.h_est())
    V = _np(r.V)
    assert np.allclose(np.linalg.norm(V.reshape(k, -1), axis=1), 1.0, atol=1e-12)
    assert np.abs((V * m[None]).sum(1)).max() < 1e-12  # tangent


@pytest.mark.parametrize("hvp", ["f64", "f32"])
def test_min_modes_three_shell_64_random_texture(hvp):
    M = _M()
    L = 64
    p = S.ham_3shell(L)
    h = O.Ham(**p.asdict())
    plan = M.Plan.from_params(p)
    m = S.three_shell_start(L, seed=1, kind="antiskyrmion")
    dt = M.MOTO_F64 if hvp == "f64" else M.MOTO_F32
    tol = 1e-10 if hvp == "f64" else 1e-5
    r = M.moto_min_modes(plan, _dev(m), 4, dt, opts=M.eig_opts(dt, tol=tol, max_iter=400))
    assert r.status == M.CONVERGED, (r.status, r.iters, _np(r.resid))
    ro = O.min_modes(h, m, 6, tol=1e-11, max_iter=600)
    w = ro.evals
    gaps = [min(abs(w[j] - w[i]) for i in range(len(w)) if i != j) >= 1e-3 * h.h_est() for j in range(4)]
    _check_pairs(_np(r.evals), _np(r.V), w[:4], ro.V[:4], h.h_est(), hvp == "f32", gaps)


@pytest.fixture(scope="module")
def three_shell_16_reference():
    p = S.ham_3shell(16)
    h = O.Ham(**p.asdict())
    m = S.three_shell_start(16, seed=3, kind="skyrmion")
    return p, h, m, O.min_modes(h, m, 6, tol=1e-11, max_iter=600)


@pytest.mark.parametrize("hvp", ["f64", "f32"])
@pytest.mark.parametrize("guard", [2, 4, 6, 8, 12])
def test_min_modes_every_basis_size_matches_oracle(three_shell_16_reference, hvp, guard):
    """k = 4 with guards 2 .. 12: Rayleigh-Ritz bases of 18, 24, 30, 36 and 48
    columns, so the lowest-eigenpair solver runs in each of its register
    buckets (24, 32, 40, 48 rows), its multisection with 8 .. 16 wanted pairs
    on four waves, and the matrix-core products on square tile grids of side
    2 and 3 and column grids of 2 and 3 tiles; block widths 6 .. 16 (the FP32
    row kernels on the matrix cores from width 5)."""
    M = _M()
    p, h, m, ro = three_shell_16_reference
    plan = M.Plan.from_params(p)
    dt = M.MOTO_F64 if hvp == "f64" else M.MOTO_F32
    tol = 1e-10 if hvp == "f64" else 1e-5
    r = M.moto_min_modes(plan, _dev(m), 4, dt, opts=M.eig_opts(dt, tol=tol, max_iter=400, guard=guard))
    assert r.status == M.CONVERGED, (r.status, r.iters, _np(r.resid))
    w = ro.evals
    gaps = [min(abs(w[j] - w[i]) for i in range(len(w)) if i != j) >= 1e-3 * h.h_est() for j in range(4)]
    _check_pairs(_np(r.evals), _np(r.V), w[:4], ro.V[:4], h.h_est(), hvp == "f32", gaps)
    assert np.all(_np(r.resid) <= tol * h.h_est())


@pytest.mark.parametrize("hvp", ["f64", "f32"])
def test_min_modes_fm_closed_form_128(hvp):
    """Full-size 128x128 three-shell lattice, uniform state: the k = 4 lowest
    eigenvalues equal the closed-form spin-wave spectrum."""
    M = _M()
    L = 128
    p = S.ham_3shell(L)
    plan = M.Plan.from_params(p)
    dt = M.MOTO_F64 if hvp == "f64" else M.MOTO_F32
    tol = 1e-9 if hvp == "f64" else 1e-5
    r = M.moto_min_modes(plan, _dev(S.uniform(L * L)), 4, dt,
                         opts=M.eig_opts(dt, tol=tol, max_iter=400, guard=12))
    assert r.status == M.CONVERGED, (r.status, r.iters)
    ref = CF.fm_z_spectrum(L, L, p.J, p.K, p.B[2])[:4]
    hest = plan.hessian_norm_bound()
    assert np.abs(_np(r.evals) - ref).max() <= (1e-8 if hvp == "f64" else 1e-5) * hest


def test_min_modes_full_size_residual_property_128_skyrmion():
    """128x128 skyrmion start, FP32 HVP, k = 4: every returned pair is an
    eigenpair of the oracle operator within the stopping tolerance."""
    M = _M()
    L = 128
    p = S.ham_3shell(L)
    h = O.Ham(**p.asdict())
    plan = M.Plan.from_params(p)
    m = S.three_shell_start(L, seed=0, kind="skyrmion")
    r = M.moto_min_modes(plan, _dev(m), 4, M.MOTO_F32, opts=M.eig_opts(M.MOTO_F32, tol=1e-5, max_iter=400))
    assert r.status == M.CONVERGED
    _, _, c, _ = O.energy_grad(h, m)
    V = _np(r.V)
    for j in range(4):
        Hv = O.tangent_hvp(h, m, c, V[j])
        res = np.linalg.norm(Hv - _np(r.evals)[j] * V[j])
        assert res <= 2e-5 * h.h_est()


def test_min_modes_masked_matches_oracle():
    M = _M()
    L = 12
    p = S.ham_nn(L)
    h = O.Ham(**p.asdict())
    plan = M.Plan.from_params(p)
    m = S.nn_start(3, L=L)
    mask = S.random_mask_disc(L, L, 3.5)
    r = M.moto_min_modes(plan, _dev(m), 2, M.MOTO_F64, mask=_dev(mask, torch.uint8),
                         opts=M.eig_opts(M.MOTO_F64, tol=1e-11))
    assert r.status == M.CONVERGED
    ro = O.min_modes(h, m, 2, tol=1e-11, mask=mask)
    assert np.allclose(_np(r.evals), ro.evals, atol=1e-9)
    V = _np(r.V)
    assert np.all(V[:, :, mask == 0] == 0)
    assert abs(float((V[0] * ro.V[0]).sum())) > 1 - 1e-8


def test_min_modes_warm_start_and_iteration_cap():
    M = _M()
    p = S.ham_nn(16)
    plan = M.Plan.from_params(p)
    m = _dev(S.nn_start(1))
    r1 = M.moto_min_modes(plan, m, 2, M.MOTO_F64)
    r2 = M.moto_min_modes(plan, m, 2, M.MOTO_F64, V0=r1.V)
    assert r2.status == M.CONVERGED and r2.iters <= 2
    assert np.allclose(_np(r2.evals), _np(r1.evals), atol=1e-9)
    r3 = M.moto_min_modes(plan, m, 2, M.MOTO_F64, opts=M.eig_opts(M.MOTO_F64, max_iter=1))
    assert r3.status == M.NOT_CONVERGED and r3.iters == 1


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_min_modes_fp32_random_start_at_index1_saddle(seed):
    """FP32 blocks from a random start at a point with a negative eigenvalue
    (the 16x16 collapse saddle of the oracle): the basis stays orthonormal
    and the pair (lambda_1 < 0 < lambda_2) is recovered."""
    M = _M()
    p = S.ham_nn(16)
    h = O.Ham(**p.asdict())
    plan = M.Plan.from_params(p)
    m0 = S.add_tilt_noise(S.skyrmion(16, 16, 1.0), 0.05, np.random.default_rng(0))
    ro = O.saddle_search(h, m0, tau_F=1e-6)
    r = M.moto_min_modes(plan, _dev(ro.m), 2, M.MOTO_F32, opts=M.eig_opts(M.MOTO_F32, tol=1e-6, seed=seed))
    assert r.status == M.CONVERGED, (r.status, r.iters, _np(r.evals))
    assert np.allclose(_np(r.evals), ro.evals, atol=1e-5 * h.h_est())


def test_graph_replays_match_eager_bitwise():
    """The captured iteration chunk, replayed across calls with eager work
    and synchronisation in between, gives bit-identical results to eager
    launches (all reductions are fixed-order)."""
    M = _M()
    L = 32
    p = S.ham_3shell(L)
    plan = M.Plan.from_params(p)
    m = _dev(S.three_shell_start(L, seed=4, kind="skyrmion"))
    ws = M.EigWorkspace(plan, M.MOTO_F32, 2)
    ref = M.moto_min_modes(plan, m, 2, M.MOTO_F32, opts=M.eig_opts(M.MOTO_F32, use_graph=0, check_every=4), ws=ws)
    for rep in range(3):
        _ = M.moto_energy_grad(plan, m)  # eager work between replays
        torch.cuda.synchronize()
        r = M.moto_min_modes(plan, m, 2, M.MOTO_F32, opts=M.eig_opts(M.MOTO_F32, use_graph=1, check_every=4),
                             ws=ws)
        assert r.iters == ref.iters and r.status == ref.status
        assert torch.equal(r.evals, ref.evals) and torch.equal(r.V, ref.V)


@pytest.mark.parametrize("solver", ["lobpcg", "lanczos"])
@pytest.mark.parametrize("hvp", ["f64", "f32"])
def test_captured_chunk_follows_the_callers_state(solver, hvp):
    """One workspace, three different states passed in turn with graph
    replay on: every result equals the plain-launch solve of its own state
    (a captured chunk must not keep reading the first caller's spins)."""
    M = _M()
    p = S.ham_3shell(32)
    plan = M.Plan.from_params(p)
    dt = M.MOTO_F64 if hvp == "f64" else M.MOTO_F32
    tol = 1e-10 if hvp == "f64" else 1e-5
    states = [_dev(S.three_shell_start(32, seed=20 + y)) for y in range(3)]
    if solver == "lobpcg":
        ws = M.EigWorkspace(plan, dt, 2)
        run = lambda m, g, w: M.moto_min_modes(plan, m, 2, dt, opts=M.eig_opts(dt, tol=tol, use_graph=g), ws=w)
        fresh = lambda: M.EigWorkspace(plan, dt, 2)
    else:
        ws = M.LanczosWorkspace(plan, dt, 32)
        run = lambda m, g, w: M.moto_min_modes_lanczos(plan, m, 2, dt, opts=M.lanczos_opts(dt, tol=tol, use_graph=g),
                                                       ws=w)
        fresh = lambda: M.LanczosWorkspace(plan, dt, 32)
    for m in states:
        rg = run(m, 1, ws)
        re = run(m, 0, fresh())
        assert rg.status == re.status == M.CONVERGED and rg.iters == re.iters
        assert torch.equal(rg.evals, re.evals) and torch.equal(rg.V, re.V)


def test_min_modes_512_two_skyrmions_residual_property():
    """512x512 with two skyrmions (Q = 2), FP32 HVP: the start has the seeded
    charge and every returned pair is an eigenpair of the oracle's operator
    within the tolerance, in ascending order.  k = 4: the skyrmions' internal
    modes (0.005 .. 0.03); the next levels are the bottom of the magnon band,
    spaced ~1e-4 apart on a lattice this large, which a 12-column block
    resolves only slowly."""
    M = _M()
    L = 512
    p = S.ham_3shell(L)
    h = O.Ham(**p.asdict())
    plan = M.Plan.from_params(p)
    m = S.two_skyrmions(L)
    assert abs(O.topological_charge(h, m) - 2.0) < 1e-6
    r = M.moto_min_modes(plan, _dev(m), 4, M.MOTO_F32, opts=M.eig_opts(M.MOTO_F32, tol=1e-5, max_iter=400))
    assert r.status == M.CONVERGED, (r.status, r.iters)
    ev, V = _np(r.evals), _np(r.V)
    assert np.all(np.diff(ev) >= -1e-6 * h.h_est())
    _, _, c, _ = O.energy_grad(h, m)
    for j in range(4):
        Hv = O.tangent_hvp(h, m, c, V[j])
        assert np.linalg.norm(Hv - ev[j] * V[j]) <= 2e-5 * h.h_est(), j
