"""GPU parity of the inner layer over a population (moto_min_modes_population:
P block-LOBPCG solves in lock step) against the FP64 oracle, member by
member.  Same bars as the single-solve tests: eigenvalues
|d lambda| <= 1e-5 max(|lambda|, h_est) (and 1e-5 |lambda| for |lambda| >=
1e-3 h_est in FP64); vectors
1 - |cos| <= 1e-8 (FP64) or sin(angle) <= 1e-3 (FP32) where the gap is
>= 1e-3 h_est."""
import numpy as np
import pytest

import oracle as O
from paper_2509_26269_amd import synth as S
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


def _check_member(ev, V, ro, k, hest, fp32):
    w = ro.evals
    for j in range(k):
        assert abs(ev[j] - w[j]) <= P.eig_bar(w[j], hest, not fp32), (j, ev[j], w[j])
        gap = min(abs(w[j] - w[i]) for i in range(len(w)) if i != j)
        if gap >= 1e-3 * hest:
            cos = abs(float((V[j] * ro.V[j]).sum()))
            if fp32:
                assert np.sqrt(max(0.0, 1 - cos * cos)) <= 1e-3
            else:
                assert 1 - cos <= 1e-8


def test_population_fp64_matches_oracle_member_by_member():
    """Five different states (one the exactly degenerate uniform state, which
    converges at once, beside perturbed skyrmions that take longer)."""
    M = _M()
    p = S.ham_nn(16)
    h = O.Ham(**p.asdict())
    plan = M.Plan.from_params(p)
    ms = [S.nn_start(s) for s in range(4)] + [S.uniform(h.N)]
    k = 2
    r = M.moto_min_modes_population(plan, _dev(np.stack(ms)), k, M.MOTO_F64,
                                    opts=M.eig_opts(M.MOTO_F64, tol=1e-10))
    assert all(st == M.CONVERGED for st in r.status), r.status
    ev, V = _np(r.evals), _np(r.V)
    for y, m in enumerate(ms):
        ro = O.min_modes(h, m, k + 2, tol=1e-11)
        _check_member(ev[y], V[y], ro, k, h.h_est(), False)
        assert np.abs((V[y] * m[None]).sum(1)).max() < 1e-12  # tangent
    # members finish independently: the uniform state needs fewer iterations
    assert r.iters[4] < max(r.iters[:4])


def test_population_fp32_masked_per_member_matches_oracle():
    M = _M()
    L = 48
    p = S.ham_3shell(L)
    h = O.Ham(**p.asdict())
    plan = M.Plan.from_params(p)
    ms, masks = [], []
    for y in range(4):
        ms.append(S.three_shell_start(L, seed=10 + y))
        masks.append(S.random_mask_disc(L, L, 10.0 + 2 * y) if y % 2 else np.ones(L * L, np.uint8))
    k = 2
    r = M.moto_min_modes_population(plan, _dev(np.stack(ms)), k, M.MOTO_F32,
                                    mask=_dev(np.stack(masks), torch.uint8),
                                    opts=M.eig_opts(M.MOTO_F32, tol=1e-5, max_iter=400))
    assert all(st == M.CONVERGED for st in r.status), (r.status, r.iters)
    ev, V = _np(r.evals), _np(r.V)
    for y in range(4):
        ro = O.min_modes(h, ms[y], k + 2, tol=1e-11, max_iter=600, mask=masks[y])
        _check_member(ev[y], V[y], ro, k, h.h_est(), True)
        assert np.all(V[y][:, :, masks[y] == 0] == 0)


def test_population_agrees_with_single_solves_and_graph_replay():
    """Each member equals the single-state solve of the same state to the
    solver tolerance; replays of the captured chunk equal plain launches
    bit for bit."""
    M = _M()
    p = S.ham_3shell(32)
    plan = M.Plan.from_params(p)
    ms = np.stack([S.three_shell_start(32, seed=20 + y) for y in range(3)])
    md = _dev(ms)
    outs = []
    for g in (0, 1, 1):
        o = M.eig_opts(M.MOTO_F64, tol=1e-10, use_graph=g)
        outs.append(M.moto_min_modes_population(plan, md, 2, M.MOTO_F64, opts=o))
    for r in outs[1:]:
        assert r.status == outs[0].status and r.iters == outs[0].iters
        assert torch.equal(r.evals, outs[0].evals) and torch.equal(r.V, outs[0].V)
    hest = plan.hessian_norm_bound()
    for y in range(3):
        rs = M.moto_min_modes(plan, md[y].contiguous(), 2, M.MOTO_F64, opts=M.eig_opts(M.MOTO_F64, tol=1e-10))
        assert np.abs(_np(rs.evals) - _np(outs[0].evals[y])).max() <= 1e-9 * hest


def test_population_full_size_eigenpair_property():
    """24 perturbed 128x128 states (the explorer's population size), FP32 HVP,
    k = 2: every returned pair is an eigenpair of the oracle operator within
    the tolerance, and the ordering holds."""
    M = _M()
    L = 128
    p = S.ham_3shell(L)
    h = O.Ham(**p.asdict())
    plan = M.Plan.from_params(p)
    spec = S.fixed_size_spec(24, L, seed=128)
    ms = np.stack([S.batch_member(spec, y) for y in range(24)])
    r = M.moto_min_modes_population(plan, _dev(ms), 2, M.MOTO_F32,
                                    opts=M.eig_opts(M.MOTO_F32, tol=1e-5, max_iter=400))
    ev, V = _np(r.evals), _np(r.V)
    conv = [y for y in range(24) if r.status[y] == M.CONVERGED]
    assert len(conv) >= 20, (r.status, r.iters)
    for y in conv[::4]:
        _, _, c, _ = O.energy_grad(h, ms[y])
        assert ev[y][0] <= ev[y][1] + 1e-6 * h.h_est()
        for j in range(2):
            Hv = O.tangent_hvp(h, ms[y], c, V[y][j])
            assert np.linalg.norm(Hv - ev[y][j] * V[y][j]) <= 2e-5 * h.h_est(), (y, j)


def test_population_bad_arguments_rejected():
    M = _M()
    plan = M.Plan.from_params(S.ham_nn(8))
    assert M.lib().moto_min_modes_population_workspace(plan.handle, M.MOTO_F64, 0, 2, -1) == 0
    assert M.lib().moto_min_modes_population_workspace(plan.handle, M.MOTO_F64, M.MAX_POPULATION + 1, 2, -1) == 0
    with pytest.raises(M.MotoError):
        M.moto_min_modes_population(plan, _dev(S.uniform(64))[None].expand(2, 3, 64).contiguous(), 17, M.MOTO_F64)


# --- searches in lock step ----------------------------------------------------
def test_population_search_matches_one_at_a_time_searches():
    """Three collapse-type starts on the 16x16 NN model (FP64 HVP) and a
    masked member: every member ends where the one-at-a-time search from the
    same start ends (status, iterations, energy, spins)."""
    M = _M()
    p = S.ham_nn(16)
    h = O.Ham(**p.asdict())
    plan = M.Plan.from_params(p)
    starts = [S.add_tilt_noise(S.skyrmion(16, 16, 1.0), 0.05, np.random.default_rng(s)) for s in range(3)]
    mask = np.ones((3, h.N), np.uint8)
    mask[2] = S.random_mask_disc(16, 16, 5.0)
    so = M.search_opts(M.MOTO_F64, tau_F=1e-6)
    mp = _dev(np.stack(starts))
    res, ev, V = M.moto_saddle_search_population(plan, mp, M.MOTO_F64, mask=_dev(mask, torch.uint8), opts=so)
    for y in range(3):
        md = _dev(starts[y])
        r1, ev1, _ = M.moto_saddle_search(plan, md, M.MOTO_F64, mask=_dev(mask[y], torch.uint8) if y == 2 else None,
                                          opts=so)
        assert res[y].status == r1.status, (y, res[y].status, r1.status)
        assert res[y].iters == r1.iters
        assert abs(res[y].E - r1.E) <= 1e-10 * abs(r1.E)
        assert O.max_site_angle(_np(mp[y]), _np(md)) <= 1e-8
        assert np.abs(_np(ev[y]) - _np(ev1)).max() <= 1e-9 * h.h_est()
    assert res[0].status == M.SADDLE


def test_population_search_stoner_wohlfarth_closed_form():
    M = _M()
    p = S.ham_sw(8)
    h = O.Ham(**p.asdict())
    plan = M.Plan.from_params(p)
    b, K = p.B[0], p.K
    starts = np.stack([S.add_tilt_noise(S.uniform(h.N, (1, 0, 0)), 0.02, np.random.default_rng(s))
                       for s in range(4)])
    res, ev, _ = M.moto_saddle_search_population(plan, _dev(starts), M.MOTO_F64,
                                                 opts=M.search_opts(M.MOTO_F64, tau_F=1e-8))
    for r in res:
        assert r.status == M.SADDLE
        assert abs(r.lambda1 - (b - 2 * K)) < 1e-8 and abs(r.lambda2 - b) < 1e-8


def test_population_search_bad_arguments():
    M = _M()
    plan = M.Plan.from_params(S.ham_nn(8))
    with pytest.raises(M.MotoError):
        M.moto_saddle_search_population(plan, _dev(S.uniform(64))[None].contiguous(), M.MOTO_F64,
                                        opts=M.search_opts(M.MOTO_F64, k=20))


def test_population_search_full_size_masked_128():
    """The benchmark's masked lock-step workload at full size: 64 seeded
    perturbed skyrmion / antiskyrmion / biskyrmion starts on 128x128, climb
    confined to a disc of radius 8 around the core, k = 2, FP32 HVP, at most
    300 outer steps.  Every member: finite unit spins, spins outside the
    disc untouched, iterations within the cap.  Sampled members (the first
    certified saddle and the first other member): the reported energy is
    the oracle energy of the returned state and lambda_1 the oracle's lowest
    masked tangent eigenvalue; at the saddle the oracle's masked force is
    below tau_F and its tangent spectrum has exactly one negative
    eigenvalue."""
    M = _M()
    L, P, cap, tau_F = 128, 64, 300, 1e-5
    p = S.ham_3shell(L)
    h = O.Ham(**p.asdict())
    plan = M.Plan.from_params(p)
    spec = S.fixed_size_spec(P, L, seed=128)
    starts = np.stack([S.batch_member(spec, i) for i in range(P)])
    disc = S.random_mask_disc(L, L, 8.0)
    mp = _dev(starts)
    so = M.search_opts(M.MOTO_F32, tau_F=tau_F, k=2, k_cert=2, max_outer=cap, eig={"tol": 1e-5, "max_iter": 200})
    res, ev, _ = M.moto_saddle_search_population(plan, mp, M.MOTO_F32, mask=_dev(np.stack([disc] * P), torch.uint8),
                                                 opts=so)
    fin = _np(mp)
    off = disc == 0
    for y in range(P):
        assert np.all(np.isfinite(fin[y])), y
        assert np.allclose(np.linalg.norm(fin[y], axis=0), 1.0, atol=1e-12), y
        assert np.array_equal(fin[y][:, off], starts[y][:, off]), y
        assert 0 < res[y].iters <= cap, (y, res[y].iters)
    sad = [y for y in range(P) if res[y].status == M.SADDLE]
    assert sad, "no certified saddle among the masked searches"
    other = next(y for y in range(P) if res[y].status != M.SADDLE)
    for y in (sad[0], other):
        Eo, _, _, F = O.energy_grad(h, fin[y])
        assert abs(res[y].E - Eo) <= 1e-9 * abs(Eo), (y, res[y].E, Eo)
        ro = O.min_modes(h, fin[y], 2, tol=1e-10, max_iter=2000, mask=disc)
        assert ro.converged
        assert abs(res[y].lambda1 - ro.evals[0]) <= 1e-4 * h.h_est(), (y, res[y].lambda1, ro.evals[0])
        if y == sad[0]:
            fo = np.linalg.norm(F[:, disc != 0])
            assert fo <= tau_F and abs(fo - res[y].fnorm) <= 1e-6 * tau_F, (fo, res[y].fnorm)
            assert ro.evals[0] < -1e-3 < 1e-3 < ro.evals[1], ro.evals
