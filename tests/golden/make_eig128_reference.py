"""Write eig128_reference.txt: the six lowest tangent-Hessian eigenvalues of
two 128x128 three-shell states, computed by the FP64 oracle alone (band
Lanczos and LOBPCG, which must agree), for the full-size eigen-solver parity
tests.  States (from the seeded input generators):
  bench_seed2025: skyrmion start, seed 2025, rounded to FP32 and renormalised
                  (the state the eigen-solve benchmark hands to the solvers);
  seed0:          skyrmion start, seed 0 (FP64).
Run: python tests/golden/make_eig128_reference.py   (about ten minutes)."""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2509_26269_amd import synth as S  # noqa: E402

OUT = os.path.join(HERE, "eig128_reference.txt")
K = 6


def states():
    m = S.three_shell_start(128, seed=2025, kind="skyrmion").astype(np.float32).astype(np.float64)
    yield "bench_seed2025", m / np.linalg.norm(m, axis=0)
    yield "seed0", S.three_shell_start(128, seed=0, kind="skyrmion")


def main():
    h = O.Ham(**S.ham_3shell(128).asdict())
    hest = h.h_est()
    lines = [f"# six lowest eigenvalues of the 128x128 three-shell tangent Hessian, FP64 oracle; h_est = {hest!r}",
             "# name lambda_1 .. lambda_6 (band Lanczos, residual <= 1e-10 h_est; LOBPCG agrees to 1e-8 h_est)"]
    for name, m in states():
        t = time.time()
        lz = O.min_modes_lanczos(h, m, K, tol=1e-10, m_max=64, keep=32, max_restarts=2000, block=2)
        assert lz.converged, name
        lo = O.min_modes(h, m, K, tol=1e-8, max_iter=20000, guard=6)
        assert lo.converged, name
        assert np.abs(lz.evals - lo.evals).max() <= 1e-8 * hest, (lz.evals, lo.evals)
        lines.append(name + " " + " ".join(repr(float(x)) for x in lz.evals))
        print(name, lz.evals, f"{time.time() - t:.0f} s", flush=True)
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
