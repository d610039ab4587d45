"""The flop accounting used for GFLOP/s figures reproduces the theoretical FLOP
columns of the paper's Tables 2 and 3 exactly (Sec. 5)."""
import numpy as np

from paper_2109_10687_amd import flops


def _rows(path):
    rows = []
    with open(path) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = line.split()
                rows.append((tuple(int(a) for a in v[:4]), float(v[4]), float(v[5]), int(v[7])))
    return rows


def test_full_apply_flops():
    assert flops.FULL_HOP_FLOPS == 1320
    assert flops.DIRAC_FLOPS_PER_SITE == 1920
    assert flops.dirac_bytes_per_site(8) == 1536
    assert flops.dirac_bytes_per_site(4) == 768
    assert flops.dirac_bytes_per_site(4, link_reals=12) == 672


def test_table3_flop_column(golden_dir):
    for dims, secs, tflops, flop in _rows(f"{golden_dir}/paper_table3.txt"):
        assert round(flops.table3_flop(dims)) == flop
        # TFLOPS column is per node: four ranks (CMGs) of the given size
        assert abs(4 * flop / secs / 1e12 - tflops) < 6e-5


def test_table2_flop_column(golden_dir):
    for dims, secs, tflops, flop in _rows(f"{golden_dir}/paper_table2.txt"):
        assert round(flops.table2_flop(dims)) == flop
        assert abs(4 * flop / secs / 1e12 - tflops) < 6e-5


def test_headline_rate_is_per_iteration():
    """102 PFLOPS on 192^4 at 0.8 ms per iteration (Sec. 5) with the Table 2 count per site."""
    per_site = (flops.table2_flop((32, 6, 4, 3), iters=1) - flops.TABLE2_SCALAR_FLOPS) / (32 * 6 * 4 * 3)
    rate = per_site * 192 ** 4 / 0.8e-3
    assert abs(rate / 1e15 - 102.1) < 0.1
    assert np.isclose(flops.surface_fraction((16, 6, 4, 3)), 1040 / 1152)
