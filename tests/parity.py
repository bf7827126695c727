"""Parity bars shared by the GPU tests (the contract's tolerances made well
defined; the oracle is the reference side of every comparison)."""
import numpy as np


def eig_bar(ref: float, hest: float, fp64: bool) -> float:
    """Largest |lambda - lambda_ref| accepted: 1e-5 max(|lambda_ref|, h_est)
    (the spectral-scale form: an FP32 operator error of ~u32 ||H|| dominates
    near lambda = 0), and in FP64 also 1e-5 |lambda_ref| whenever
    |lambda_ref| >= 1e-3 h_est (relative accuracy away from zero)."""
    bar = 1e-5 * max(abs(ref), hest)
    if fp64 and abs(ref) >= 1e-3 * hest:
        bar = min(bar, 1e-5 * abs(ref))
    return bar


def check_eigs(ev, ref, hest: float, fp64: bool, what: str = ""):
    ev = np.asarray(ev, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    for j in range(len(ref)):
        assert abs(ev[j] - ref[j]) <= eig_bar(ref[j], hest, fp64), (what, j, ev[j], ref[j])


def check_vectors(V, ref_V, ref_ev, k: int, hest: float, fp64: bool):
    """Unit vectors whose eigenvalue is separated from the rest of ref_ev by
    at least 1e-3 h_est: 1 - |cos| <= 1e-8 (FP64) or sin <= 1e-3 (FP32)."""
    w = np.asarray(ref_ev, dtype=np.float64)
    for j in range(k):
        gap = min(abs(w[j] - w[i]) for i in range(len(w)) if i != j)
        if gap < 1e-3 * hest:
            continue
        cos = abs(float((V[j] * ref_V[j]).sum()))
        if fp64:
            assert 1 - cos <= 1e-8, (j, cos)
        else:
            assert np.sqrt(max(0.0, 1 - cos * cos)) <= 1e-3, (j, cos)
