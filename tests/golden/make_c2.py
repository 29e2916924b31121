"""Write the stored oracle results of the FP64 parity cases at N = 16384,
n_b = 256 (tests/test_gpu_c2.py).

Runs only the FP64 CPU oracle (oracle/) on the seeded inputs of
paper_1401_5522_amd/inputs.py, for three of the matrix types of the paper's
random-matrix experiments and of its growth example (Sec. 5.2, Sec. 3.1):
the decision sequence, s_k, m_k, the margins, the solution of one seeded
right-hand side, its backward error, and a 1-norm condition estimate of A
(LAPACK dgecon through scipy).  The SHA-256 of A's column-major bytes is
stored with them so a test can tell that it regenerated the same matrix.

    python tests/golden/make_c2.py            # all cases (~15 min on 8 cores)
    python tests/golden/make_c2.py gaussian   # the cases of one matrix type
"""
import hashlib
import os
import sys
import time

import numpy as np
import scipy.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1401_5522_amd import inputs  # noqa: E402

N, NB = 16384, 256
# (matrix type, criterion, alpha)
CASES = [("gaussian", "max", 1.0), ("diag_dominant", "sum", 0.5), ("growth_prone", "max", 4.0)]


def case_name(kind, crit, alpha):
    return f"c2_{kind}_{crit}_{alpha:g}"


def matrix(kind):
    return inputs.matrix(kind, N, seed=(160,))


def rhs():
    return inputs.rhs(N, seed=(161,))


def sha256(A):
    return hashlib.sha256(memoryview(np.ascontiguousarray(A.T))).hexdigest()


def main(kinds):
    for kind, crit, alpha in CASES:
        if kinds and kind not in kinds:
            continue
        A = matrix(kind)
        b = rhs()
        t0 = time.perf_counter()
        f = O.factor(A, NB, crit, alpha)
        x = f.solve(b)
        t = time.perf_counter() - t0
        dec, s, m, margin, diag = f.dec, f.s, f.m, f.margin, f.diag
        del f
        lu, piv = sla.lu_factor(A)
        anorm = np.abs(A).sum(axis=0).max()
        rcond, info = sla.lapack.dgecon(lu, anorm, norm="1")
        del lu
        out = dict(sha256=sha256(A), dec=dec, s=s, m=m, margin=margin, x=x,
                   eta=O.backward_error(A, x, b), cond1_est=1.0 / rcond, growth_tile=diag[O.DG_GROWTH_TILE],
                   nonfinite=diag[O.DG_NONFINITE], seconds=t, threads=O.num_threads())
        path = os.path.join(HERE, case_name(kind, crit, alpha) + ".npz")
        np.savez_compressed(path, **out)
        print(f"{path}: {''.join('L' if d else 'Q' for d in dec)} eta={out['eta']:.2e} "
              f"cond1~{out['cond1_est']:.2e} {t:.0f} s on {out['threads']} threads", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
