"""Write eig512_reference.txt: the ten lowest eigenvalues of the 512x512
three-shell tangent Hessian at the two-skyrmion state (Q = 2) of the seeded
input generators, computed by the FP64 oracle alone (thick-restart band
Lanczos to 1e-9 h_est), for the full-size k = 8 eigen-solver parity test.
The eight lowest are the four internal modes of the two skyrmions and the
bottom of the magnon band, whose levels lie about 1e-4 apart.
Run: python tests/golden/make_eig512_reference.py   (tens of minutes)."""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2509_26269_amd import synth as S  # noqa: E402

OUT = os.path.join(HERE, "eig512_reference.txt")
K = 10


def main():
    h = O.Ham(**S.ham_3shell(512).asdict())
    m = S.two_skyrmions(512)
    t = time.time()
    r = O.min_modes_lanczos(h, m, K, tol=1e-9, m_max=64, keep=32, max_restarts=4000, block=2)
    assert r.converged
    with open(OUT, "w") as f:
        f.write(f"# ten lowest eigenvalues of the 512x512 three-shell tangent Hessian at the two-skyrmion state, "
                f"FP64 oracle band Lanczos (residual <= 1e-9 h_est); h_est = {h.h_est()!r}\n")
        f.write("two_skyrmions " + " ".join(repr(float(x)) for x in r.evals) + "\n")
    print(r.evals, r.iters, r.n_hvp, f"{time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    main()
