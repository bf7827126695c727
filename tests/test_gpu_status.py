"""Status paths of the drivers, forced from the host with numerical inputs
(no GPU fault is involved: every kernel runs to its normal end):

* non-finite spins -> MOTO_NAN from both eigen-solvers, the population
  solve (that member only) and the saddle search;
* a rank-deficient start block (duplicated warm-start columns with no guard
  vectors) -> MOTO_BREAKDOWN; with the default guard the same start converges
  to the cold solve's eigenvalues;
* a Krylov space exhausted by a mask with one active site -> MOTO_BREAKDOWN
  from the Lanczos solver (k larger than the two active directions);
* the isotropic exchange-only model, whose spectrum has exact zero modes
  (global rotations): the climb ends DEGENERATE, as the oracle's does;
* a cap of one iteration on every iterative entry point -> NOT_CONVERGED,
  and a certifying solve capped at one iteration never certifies a saddle
  (an unconverged Ritz value only bounds its eigenvalue from above)."""
import numpy as np
import pytest

import oracle as O
from paper_2509_26269_amd import synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _M():
    from paper_2509_26269_amd import moto as M

    return M


def _dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _np(t):
    return t.detach().double().cpu().numpy()


def _nan_state(L, seed, site):
    m = S.three_shell_start(L, seed=seed, kind="skyrmion").copy()
    m[1, site] = np.nan
    return m


@pytest.mark.parametrize("hvp", ["f64", "f32"])
def test_nan_spins_end_both_eigen_solvers_with_nan_status(hvp):
    M = _M()
    L = 24
    plan = M.Plan.from_params(S.ham_3shell(L))
    dt = M.MOTO_F64 if hvp == "f64" else M.MOTO_F32
    md = _dev(_nan_state(L, 3, 5 * L + 7))
    r = M.moto_min_modes(plan, md, 2, dt)
    assert r.status == M.NAN and r.iters == 0, (r.status, r.iters)
    assert not torch.isfinite(r.evals).any()
    r = M.moto_min_modes_lanczos(plan, md, 2, dt)
    assert r.status == M.NAN, r.status
    assert not torch.isfinite(r.evals).any()


def test_nan_member_of_a_population_alone_reports_nan():
    M = _M()
    L = 24
    plan = M.Plan.from_params(S.ham_3shell(L))
    ms = np.stack([S.three_shell_start(L, seed=10 + y, kind="skyrmion") for y in range(4)])
    ms[2] = _nan_state(L, 12, 3)
    r = M.moto_min_modes_population(plan, _dev(ms), 2, M.MOTO_F32, opts=M.eig_opts(M.MOTO_F32, max_iter=400))
    assert r.status[2] == M.NAN, r.status
    assert all(r.status[y] == M.CONVERGED for y in (0, 1, 3)), r.status
    ev = _np(r.evals)
    assert np.all(np.isfinite(ev[[0, 1, 3]])) and not np.isfinite(ev[2]).any()


def test_nan_spins_end_the_saddle_search_with_nan_status():
    M = _M()
    L = 16
    plan = M.Plan.from_params(S.ham_nn(L))
    m = S.nn_start(0).copy()
    m[2, 17] = np.nan
    res, _, _ = M.moto_saddle_search(plan, _dev(m), M.MOTO_F64, opts=M.search_opts(M.MOTO_F64, max_outer=50))
    assert res.status == M.NAN, res.status


def test_duplicated_warm_start_columns():
    """Two equal warm-start vectors: with no guard vectors the block has rank
    k - 1 < k (MOTO_BREAKDOWN); with the default guard the dependent column is
    dropped and refilled, and the solve converges to the cold eigenvalues."""
    M = _M()
    L = 16
    p = S.ham_nn(L)
    plan = M.Plan.from_params(p)
    md = _dev(S.nn_start(2))
    cold = M.moto_min_modes(plan, md, 2, M.MOTO_F64)
    assert cold.status == M.CONVERGED
    V0 = cold.V.clone()
    V0[1] = V0[0]
    r = M.moto_min_modes(plan, md, 2, M.MOTO_F64, V0=V0, opts=M.eig_opts(M.MOTO_F64, guard=0))
    assert r.status == M.BREAKDOWN, r.status
    r = M.moto_min_modes(plan, md, 2, M.MOTO_F64, V0=V0, opts=M.eig_opts(M.MOTO_F64))
    assert r.status == M.CONVERGED, r.status
    hest = plan.hessian_norm_bound()
    assert np.abs(_np(r.evals) - _np(cold.evals)).max() <= 1e-9 * hest


def test_lanczos_exhausted_krylov_space_is_a_breakdown():
    """Mask with a single active site: the masked tangent space has two
    directions, so three eigenpairs cannot exist (MOTO_BREAKDOWN), not a
    CONVERGED result with fewer pairs than asked for."""
    M = _M()
    L = 4
    plan = M.Plan.from_params(S.ham_nn(L))
    m = S.random_texture(L * L, np.random.default_rng(4))
    mask = np.zeros(L * L, dtype=np.uint8)
    mask[5] = 1
    r = M.moto_min_modes_lanczos(plan, _dev(m), 3, M.MOTO_F64, mask=_dev(mask, torch.uint8),
                                 opts=M.lanczos_opts(M.MOTO_F64, m_max=8, max_restarts=20))
    assert r.status == M.BREAKDOWN, (r.status, r.iters)


def test_isotropic_exchange_climb_is_degenerate_like_the_oracle():
    """J-only model (no DMI, anisotropy or field): every state has exact
    zero modes.  From a tilted ferromagnet with noise both sides relax to a
    uniform state whose two lowest tangent eigenvalues vanish: DEGENERATE,
    same energy."""
    M = _M()
    L = 8
    p = S.HamParams(L, L, [1.0], [0.0], 0.0, (0.0, 0.0, 0.0))
    h = O.Ham(**p.asdict())
    plan = M.Plan.from_params(p)
    m0 = S.add_tilt_noise(S.uniform(L * L, (0.3, 0.2, 1.0)), 0.05, np.random.default_rng(7))
    ro = O.saddle_search(h, m0, tau_F=1e-6)
    assert ro.status == O.DEGENERATE
    md = _dev(m0)
    res, ev, _ = M.moto_saddle_search(plan, md, M.MOTO_F64, opts=M.search_opts(M.MOTO_F64, tau_F=1e-6))
    assert res.status == M.DEGENERATE, (res.status, res.lambda1, res.lambda2)
    tau = 1e-6 * plan.hessian_norm_bound()
    assert abs(res.lambda1) <= tau and abs(res.lambda2) <= tau
    assert abs(res.E - ro.E) <= 1e-10 * abs(ro.E)


def test_one_iteration_cap_on_every_iterative_entry_point():
    M = _M()
    L = 16
    p = S.ham_nn(L)
    plan = M.Plan.from_params(p)
    md = _dev(S.nn_start(1))
    r = M.moto_min_modes(plan, md, 2, M.MOTO_F64, opts=M.eig_opts(M.MOTO_F64, max_iter=1))
    assert r.status == M.NOT_CONVERGED and r.iters == 1
    r = M.moto_min_modes_lanczos(plan, md, 2, M.MOTO_F64, opts=M.lanczos_opts(M.MOTO_F64, max_restarts=0, m_max=8))
    assert r.status == M.NOT_CONVERGED and r.iters == 0
    ms = _dev(np.stack([S.nn_start(s) for s in range(3)]))
    r = M.moto_min_modes_population(plan, ms, 2, M.MOTO_F64, opts=M.eig_opts(M.MOTO_F64, max_iter=1))
    assert r.status == [M.NOT_CONVERGED] * 3 and r.iters == [1, 1, 1]
    res, _, _ = M.moto_saddle_search(plan, md.clone(), M.MOTO_F64, opts=M.search_opts(M.MOTO_F64, max_outer=1))
    assert res.status == M.NOT_CONVERGED
    res_p, _, _ = M.moto_saddle_search_population(plan, ms.clone(), M.MOTO_F64,
                                                  opts=M.search_opts(M.MOTO_F64, max_outer=1))
    assert [x.status for x in res_p] == [M.NOT_CONVERGED] * 3
    v1 = M.moto_min_modes(plan, md, 1, M.MOTO_F64).V[0].contiguous()
    d = M.moto_descend(plan, md.clone(), v1, +1, M.MOTO_F64, opts=M.descend_opts(M.MOTO_F64, max_iter=1))
    assert d.converged == 0
    Ls = [32, 40]
    starts = np.concatenate([S.three_shell_start(Lb, seed=b, kind="skyrmion").ravel() for b, Lb in enumerate(Ls)])
    out = M.moto_saddle_search_batched(S.ham_3shell(32), Ls, _dev(starts),
                                       opts=M.search_opts(M.MOTO_F32, tau_F=1e-5, k=2, max_outer=1))
    assert [x.status for x in out] == [M.NOT_CONVERGED] * 2


def test_certifying_solve_capped_at_one_iteration_never_certifies():
    """At the 16x16 collapse saddle of the oracle (a certified index-1 point)
    the climb stops at once; with the certifying eigen-solve capped at one
    iteration the verdict is NOT_CONVERGED, not SADDLE."""
    M = _M()
    L = 16
    p = S.ham_nn(L)
    h = O.Ham(**p.asdict())
    plan = M.Plan.from_params(p)
    m0 = S.add_tilt_noise(S.skyrmion(L, L, 1.0), 0.05, np.random.default_rng(0))
    ro = O.saddle_search(h, m0, tau_F=1e-6)
    assert ro.status == O.SADDLE
    res, _, _ = M.moto_saddle_search(plan, _dev(ro.m), M.MOTO_F64,
                                     opts=M.search_opts(M.MOTO_F64, tau_F=1e-6, eig={"max_iter": 1}))
    assert res.status == M.NOT_CONVERGED, res.status
    res, _, _ = M.moto_saddle_search(plan, _dev(ro.m), M.MOTO_F64, opts=M.search_opts(M.MOTO_F64, tau_F=1e-6))
    assert res.status == M.SADDLE, res.status
