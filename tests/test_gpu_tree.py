"""QR elimination trees (opts.qr_tree = S, Sec. 2.2, Alg. 3/4) on the GPU
against the oracle's trees: TS within groups of S panel tiles, a binary TT
tree over the groups' heads.  FP64: decisions outside the 1e-6 band, s_k to
1e-9, the factored matrix (heads holding GEQRT and TT reflectors) to 1e-10 of
its largest entry, the solution to 1e-10; every forced sequence; with
variant A2; FP32 with refinement; lookahead bit-identical."""
import itertools

import numpy as np
import pytest

from paper_1401_5522_amd import inputs

pytestmark = pytest.mark.gpu

BAND = 1e-6


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available()
    from paper_1401_5522_amd import solver
    return solver


def dev(A):
    import torch
    return torch.from_numpy(np.asfortranarray(A)).cuda()


def compare(O, gpu, A, b, nb, crit, alpha, tree, forced=None, variant=1, tol=1e-10):
    kw = dict(criterion=crit, alpha=alpha, tree=tree, variant=variant)
    if forced is not None:
        kw["forced"] = forced
    f = gpu.factor(dev(A), nb, **kw)
    dec, s, m, mg = f.decisions()
    o = O.factor(A, nb, crit, alpha, forced=forced, tree=tree, variant=variant)
    upto = len(o.dec)
    for k in range(len(o.dec)):
        if crit != "forced" and abs(o.margin[k]) <= BAND:
            upto = k
            break
        assert dec[k] == o.dec[k], (k, dec, o.dec, o.margin[k])
    if crit in ("max", "sum"):
        ok = o.s[:upto] > 0
        assert (np.abs(s[:upto] - o.s[:upto]) <= 1e-9 * np.abs(o.s[:upto]))[ok].all()
    assert f.status().watchdog == 0
    if upto == len(o.dec):
        F = f.export()[0].cpu().numpy()
        err = np.abs(F - o.F).max() / max(np.abs(o.F).max(), 1.0)
        assert err <= tol, err
        x = f.solve(dev(b)).cpu().numpy()
        xo = o.solve(b)
        assert np.linalg.norm(x - xo) <= tol * np.linalg.norm(xo)
    return f, o


CASES = [
    # (kind, N, nb, criterion, alpha, tree)
    ("gaussian", 320, 64, "max", 1.0, 1),        # binary TT tree (five tiles: heads 0..3, tile 4 joins 3)
    ("gaussian", 320, 64, "max", 1.0, 2),
    ("gaussian", 300, 32, "sum", 30.0, 3),       # ragged last tile, hybrid
    ("gaussian", 256, 32, "max", 60.0, 2),       # hybrid
    ("gaussian", 1024, 128, "max", 0.0, 2),      # all QR, eight tiles: three TT levels
    ("gaussian", 1024, 128, "max", 300.0, 3),
    ("gaussian", 2048, 256, "max", 0.0, 1),
    ("gaussian", 2048, 256, "max", 30000.0, 4),
]


@pytest.mark.parametrize("kind,N,nb,crit,alpha,tree", CASES)
def test_tree_parity(O, gpu, kind, N, nb, crit, alpha, tree):
    A = inputs.matrix(kind, N, seed=(820, N))
    b = inputs.rhs(N, seed=(821, N))
    compare(O, gpu, A, b, nb, crit, alpha, tree)


@pytest.mark.parametrize("tree", [1, 2])
def test_tree_every_forced_sequence(O, gpu, tree):
    N, nb = 152, 32  # five tiles, the last one ragged
    A = inputs.gaussian(N, seed=(822,))
    b = inputs.rhs(N, seed=(823,))
    for seq in itertools.product([0, 1], repeat=5):
        compare(O, gpu, A, b, nb, "forced", 1.0, tree, forced=np.array(seq, np.int8))


def test_tree_with_variant_a2(O, gpu):
    A = inputs.gaussian(512, seed=(824,))
    b = inputs.rhs(512, seed=(825,))
    compare(O, gpu, A, b, 64, "max", 60.0, 2, variant=2)


@pytest.mark.parametrize("precision,N,nb,tree", [("fp32", 4096, 256, 4), ("fp32", 2000, 128, 1), ("bf16", 1024, 64, 3)])
def test_tree_mixed_precision_refined(gpu, precision, N, nb, tree):
    A = inputs.usv(N, 1e2, seed=(826, N))
    b = inputs.rhs(N, seed=(827, N))
    f = gpu.factor(dev(A), nb, criterion="max", alpha=50.0, precision=precision, tree=tree)
    x = f.solve_refined(dev(A), dev(b), max_iter=30).cpu().numpy()
    st = f.status()
    assert st.watchdog == 0
    assert st.ir_converged == 1, (st.ir_iters, st.ir_eta)
    eta = np.linalg.norm(A @ x - b, np.inf) / (np.abs(A).sum(1).max() * np.abs(x).max() + np.abs(b).max())
    assert eta <= N * 1e-16, eta


def test_tree_lookahead_bit_identical(gpu):
    N, nb = 1024, 128
    A = inputs.gaussian(N, seed=(828,))
    b = inputs.rhs(N, seed=(829,))
    fa = gpu.factor(dev(A), nb, criterion="max", alpha=300.0, tree=2, lookahead=True)
    fb = gpu.factor(dev(A), nb, criterion="max", alpha=300.0, tree=2, lookahead=False)
    assert np.array_equal(fa.decisions()[0], fb.decisions()[0])
    assert np.array_equal(fa.export()[0].cpu().numpy(), fb.export()[0].cpu().numpy())
    assert np.array_equal(fa.solve(dev(b)).cpu().numpy(), fb.solve(dev(b)).cpu().numpy())


def test_tree_with_domain_and_estimate(O, gpu):
    """The tree changes only the QR steps, the domain and the estimate only the
    LU attempt and the criterion: the combinations against the oracle's."""
    A = inputs.gaussian(384, seed=(830,))
    b = inputs.rhs(384, seed=(831,))
    for kw in (dict(domain=2), dict(estimate=True)):
        f = gpu.factor(dev(A), 64, criterion="max", alpha=60.0, tree=2, **kw)
        o = O.factor(A, 64, "max", 60.0, tree=2, **kw)
        dec = f.decisions()[0]
        for k in range(len(o.dec)):
            if abs(o.margin[k]) <= BAND:
                break
            assert dec[k] == o.dec[k], (kw, k)
        else:
            x = f.solve(dev(b)).cpu().numpy()
            xo = o.solve(b)
            assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo), kw
        assert f.status().watchdog == 0


@pytest.mark.parametrize("precision,tree,variant", [("fp32", 2, 1), ("bf16", 1, 1), ("bf16", 0, 2), ("fp32", 2, 2)])
def test_nb512_tree_and_a2_refined(gpu, precision, tree, variant):
    """n_b = 512 (one QR-step workgroup per compute unit) with trees and with
    variant A2 in FP32/BF16 storage, refined to the FP64 target."""
    N = 3072
    A = inputs.usv(N, 1e1, seed=(832, tree, variant))
    b = inputs.rhs(N, seed=(833,))
    f = gpu.factor(dev(A), 512, criterion="max", alpha=1.0, precision=precision, tree=tree, variant=variant)
    x = f.solve_refined(dev(A), dev(b), max_iter=30).cpu().numpy()
    st = f.status()
    assert st.watchdog == 0
    assert st.ir_converged == 1, (st.ir_iters, st.ir_eta)
    eta = np.linalg.norm(A @ x - b, np.inf) / (np.abs(A).sum(1).max() * np.abs(x).max() + np.abs(b).max())
    assert eta <= N * 1e-16, eta
