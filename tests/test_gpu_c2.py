"""FP64 parity with the oracle at full size: N = 16384, n_b = 256 (64 x 64
tiles), for three matrix types of the paper's experiments (iid N(0,1) with
Max, N(0,1) + N I with Sum, and the perturbed growth example of Sec. 3.1
with Max).

The oracle takes minutes at this size, so its results were written once by
tests/golden/make_c2.py (which calls only oracle/) and are read here: the
decision sequence, s_k, m_k, the margins, the solution of the seeded
right-hand side, its backward error and a 1-norm condition estimate.  The
test regenerates A from the same seed and checks its SHA-256 against the
stored one before comparing.

Bar (FP64 path): decisions equal on every step up to the first whose oracle
margin is within 1e-6; s_k and m_k to 1e-9 relative (1e-5 for the
growth-prone tiles, whose kappa(A_kk) is ~1e9); the GPU backward error at
most 10 N u; and ||x - x_or|| / ||x_or|| <= 1e-10, or, where the conditioning
does not allow that, within 4 cond_1 (eta_gpu + eta_oracle).
"""
import importlib.util
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
spec = importlib.util.spec_from_file_location("make_c2", os.path.join(HERE, "golden", "make_c2.py"))
C2 = importlib.util.module_from_spec(spec)
spec.loader.exec_module(C2)


@pytest.mark.parametrize("kind,crit,alpha", C2.CASES)
def test_c2_fp64_parity(kind, crit, alpha):
    import torch
    from paper_1401_5522_amd import solver
    path = os.path.join(HERE, "golden", C2.case_name(kind, crit, alpha) + ".npz")
    ref = np.load(path)
    A = C2.matrix(kind)
    assert C2.sha256(A) == str(ref["sha256"]), "regenerated matrix differs from the stored one"
    b = C2.rhs()
    N = C2.N
    Ad = torch.from_numpy(A).cuda()
    del A
    f = solver.factor(Ad, C2.NB, criterion=crit, alpha=alpha, precision="fp64")
    x = f.solve(torch.from_numpy(b).cuda())
    dec, s, m, mg = f.decisions()
    st = f.status()
    assert st.watchdog == 0
    upto = len(dec)
    for k in range(len(dec)):
        if abs(ref["margin"][k]) <= 1e-6:
            upto = k
            break
        assert dec[k] == ref["dec"][k], (k, dec, ref["dec"], ref["margin"][k])
    srt = 1e-5 if kind == "growth_prone" else 1e-9
    assert (np.abs(s[:upto] - ref["s"][:upto]) <= srt * np.abs(ref["s"][:upto])).all()
    assert (np.abs(m[:upto] - ref["m"][:upto]) <= 1e-9 * np.maximum(np.abs(ref["m"][:upto]), 1e-300)).all()
    r = torch.from_numpy(b).cuda() - Ad @ x
    eta = float(r.abs().max() / (Ad.abs().sum(dim=1).max() * x.abs().max()))
    assert eta <= 10 * N * 2.0 ** -53, eta
    if upto == len(dec):
        x = x.cpu().numpy()
        xo = ref["x"]
        rel = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        bound = max(1e-10, 4 * float(ref["cond1_est"]) * (eta + float(ref["eta"])))
        assert rel <= bound, (rel, bound)
