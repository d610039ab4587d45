"""Write tests/golden/kappa_low_modes.txt: the leftmost eigenvalues (smallest real part) of the
oracle's Dirac operator D on the synthetic ensemble of the benchmark (links exp(0.3 i H), seed
2021, c_SW 1.7, periodic space, antiperiodic time) at kappa 0.133 and 0.1365 on 6^4 and 8^4.

D's spectrum moves towards Re lambda = 0 as the volume grows; once an eigenvalue crosses it the
operator is past the critical point and Krylov solvers stall.  The table is the CPU-side evidence
for solving the 64^3 x 128 benchmark at kappa 0.133 rather than 0.1365.  Calls only the oracle
(D by orc_dirac_D) and ARPACK (scipy.sparse.linalg.eigs, which='SR').  Run from the repository
root: python tests/golden/make_kappa_low_modes.py  (about ten minutes on 8 cores)."""
import os
import sys
import time

import numpy as np
import scipy.sparse.linalg as sla

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "kappa_low_modes.txt")


def leftmost(L, kappa, k=6):
    dims = (L, L, L, L)
    U = synth.su3_links(dims, 0.3, 2021).numpy()
    p = O.Params(dims=dims, kappa=kappa, csw=1.7, block=(2, 2, 2, 2))
    C = O.clover_field(p, U)
    shp = p.shape + (3, 4)
    n = int(np.prod(shp))
    op = sla.LinearOperator((n, n), matvec=lambda v: O.dirac_D(p, U, C, v.reshape(shp)).ravel(),
                            dtype=np.complex128)
    w = sla.eigs(op, k=k, which="SR", tol=1e-8, maxiter=50000, return_eigenvectors=False)
    return sorted(w, key=lambda z: z.real)


def main():
    lines = ["# leftmost eigenvalues of D (oracle), links exp(0.3 i H) seed 2021, c_SW 1.7, phases (1,1,1,-1)",
             "# L kappa  Re(lambda_1)  Im(lambda_1)  Re(lambda_3)"]
    for L in (6, 8):
        for kappa in (0.133, 0.1365):
            t0 = time.time()
            w = leftmost(L, kappa)
            lines.append(f"{L} {kappa} {w[0].real:.6e} {w[0].imag:.6e} {w[2].real:.6e}")
            print(lines[-1], f"({time.time() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
