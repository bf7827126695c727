"""Write ragged_search_reference.txt: climbs of the FP64 oracle from four
three-shell starts on small uneven lattices (16x16 and 20x20), the reference
of the batching-form parity test.  Start rule of the seeded input generators
(three_shell_start: Neel texture of radius R plus tilt noise 0.05, seeded);
climb: L-BFGS step rule, k = 2 modes, one reflected, tau_F = 1e-5, eigen
tolerance 1e-8 h_est.  Two skyrmion starts on 20x20 end at different saddles
(distinct energies), the antiskyrmion start at a degenerate point (a soft
translation mode).
Each member: one header line
  L kind R seed status iters E lambda_1 lambda_2
then 3 N final spins ([3][N] order, %.10e).
Run: python tests/golden/make_ragged_search_reference.py   (about a minute)."""
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2509_26269_amd import synth as S  # noqa: E402

OUT = os.path.join(HERE, "ragged_search_reference.txt")
MEMBERS = [(16, "skyrmion", 1.0, 0), (20, "skyrmion", 1.0, 0), (20, "skyrmion", 1.2, 0),
           (16, "antiskyrmion", 1.0, 0)]


def climb(member):
    L, kind, R, seed = member
    h = O.Ham(**S.ham_3shell(L).asdict())
    m0 = S.three_shell_start(L, seed=seed, kind=kind, R=R)
    r = O.saddle_search(h, m0, tau_F=1e-5, k=2, eig_tol=1e-8, max_outer=1500)
    return member, r


def main():
    with Pool(len(MEMBERS)) as pool:
        results = pool.map(climb, MEMBERS)
    lines = ["# oracle climbs on small three-shell lattices: header line, then the final spins"]
    for (L, kind, R, seed), r in results:
        lines.append(f"{L} {kind} {R!r} {seed} {r.status} {r.iters} {float(r.E)!r} {float(r.evals[0])!r} {float(r.evals[1])!r}")
        lines.append(" ".join(f"{x:.10e}" for x in r.m.reshape(-1)))
        print(L, kind, R, seed, r.status, r.iters, r.E, flush=True)
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
