"""The low-mode table behind the choice of kappa for the 64^3 x 128 solve
(tests/golden/kappa_low_modes.txt, written by tests/golden/make_kappa_low_modes.py from the
oracle's D and ARPACK).  Re-derives the 6^4 rows (about half a minute) and checks that the
table shows the trend the choice rests on: at fixed volume the leftmost eigenvalue of D lies
closer to the imaginary axis at kappa 0.1365 than at 0.133, and at fixed kappa it moves
towards the axis as the volume grows."""
import importlib.util
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SCRIPT = os.path.join(HERE, "golden", "make_kappa_low_modes.py")
TABLE = os.path.join(HERE, "golden", "kappa_low_modes.txt")


def table():
    rows = {}
    for line in open(TABLE):
        if line.startswith("#") or not line.strip():
            continue
        L, kappa, re1, im1, re3 = line.split()
        rows[(int(L), float(kappa))] = (float(re1), float(im1), float(re3))
    return rows


def test_table_covers_both_kappas_and_volumes():
    rows = table()
    assert set(rows) == {(6, 0.133), (6, 0.1365), (8, 0.133), (8, 0.1365)}
    for L in (6, 8):
        assert rows[(L, 0.1365)][0] < rows[(L, 0.133)][0]  # larger kappa: closer to the axis
    for kappa in (0.133, 0.1365):
        assert rows[(8, kappa)][0] < rows[(6, kappa)][0]  # larger volume: closer to the axis
    for r in rows.values():
        assert r[0] <= r[2]  # sorted by real part


@pytest.mark.parametrize("kappa", [0.133, 0.1365])
def test_6x6x6x6_rows_rederived_from_the_oracle(kappa):
    spec = importlib.util.spec_from_file_location("make_kappa_low_modes", SCRIPT)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    w = mod.leftmost(6, kappa)
    re1, im1, re3 = table()[(6, kappa)]
    assert w[0].real == pytest.approx(re1, rel=1e-5, abs=1e-8)
    assert abs(w[0].imag) == pytest.approx(abs(im1), rel=1e-4, abs=1e-8)
    assert w[2].real == pytest.approx(re3, rel=1e-5, abs=1e-8)
