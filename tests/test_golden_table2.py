"""The paper's printed Table 2 (Sec. 5.2), as a fixture: it fixes the flop
conventions the benchmark and the oracle use.  A QR step costs exactly twice
an LU step (Tab. 1), so the "true" rate is the "fake" (2/3 N^3) rate times
(2 - f_LU); the oracle's Tab. 1 count reaches the endpoints of that formula."""
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
N_PAPER, PEAK = 20000, 1091.0


def rows():
    out = []
    for line in open(os.path.join(HERE, "golden", "table2_dancer.txt")):
        if line.startswith("#") or not line.strip():
            continue
        a, t, pct, fake, true, fpk, tpk = line.split()
        out.append((math.inf if a == "inf" else float(a), float(t), float(pct) / 100, float(fake), float(true),
                    float(fpk), float(tpk)))
    return out


def test_true_rate_is_fake_rate_times_two_minus_lu_fraction():
    for alpha, t, f, fake, true, _, _ in rows():
        assert abs(fake * (2.0 - f) - true) <= 0.6, (alpha, fake * (2.0 - f), true)


def test_fake_rate_is_two_thirds_n_cubed_over_time():
    for alpha, t, f, fake, true, _, _ in rows():
        flops = 2.0 / 3.0 * N_PAPER ** 3 / 1e9
        assert abs(fake * t - flops) <= 0.005 * flops, (alpha, fake * t, flops)


def test_peak_fractions():
    for alpha, t, f, fake, true, fpk, tpk in rows():
        # percentages printed to 0.1 (0.05), rates printed to 0.1 (0.05 / 10.91), and the
        # peak printed as an integer (+-0.5 of 1091, up to 0.04 on these fractions)
        tol = 0.05 + 0.005 + 0.04
        assert abs(100.0 * fake / PEAK - fpk) <= tol, alpha
        assert abs(100.0 * true / PEAK - tpk) <= tol, alpha


def test_more_qr_steps_never_faster_in_the_table():
    r = sorted(rows(), key=lambda x: -x[2])  # by decreasing LU fraction
    times = [x[1] for x in r]
    assert times == sorted(times)


def test_oracle_flop_count_meets_the_formula_endpoints(O):
    N, nb = 1024, 128
    n = N // nb
    lu = O.true_flops(N, nb, np.ones(n, np.int8))
    qr = O.true_flops(N, nb, np.zeros(n, np.int8))
    assert math.isclose(lu, 2.0 / 3.0 * N ** 3, rel_tol=1e-13) and math.isclose(qr, 4.0 / 3.0 * N ** 3, rel_tol=1e-13)
    # each step switched from LU to QR adds exactly that step's LU cost (QR = 2 x LU, Tab. 1)
    for k in range(n):
        d = np.ones(n, np.int8)
        d[k] = 0
        r = n - 1 - k
        assert math.isclose(O.true_flops(N, nb, d) - lu, (2.0 / 3.0 + 2.0 * r + 2.0 * r * r) * nb ** 3, rel_tol=1e-9)
