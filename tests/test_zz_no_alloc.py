"""The allocation-free fermion force, dd_force_noalloc, against dd_force through
the C ABI: the same kernels with the work field in the library's fixed device
array instead of a field the first call allocates, so the results must agree bit
for bit.  Two calls in a row, the second on a smaller lattice (the array keeps
the first call's contents, which the second must not depend on), then a lattice
too large for the array, which is refused before any device work.
"""
import ctypes

import pytest
import torch

import paper_2109_10687_amd as dd
import synth

pytestmark = pytest.mark.gpu

# 64 MiB of work space at 864 bytes per site
MAX_SITES = (64 << 20) // 864


def make(dims, seed):
    gp = dd.Params(dims=dims, kappa=0.125, csw=1.7, block=(4, 4, 4, 4), phases=(1, 1, 1, -1))
    s = dd.Solver(gp, synth.su3_links(dims, 0.3, seed, device="cuda"))
    psi = synth.gaussian_spinor(dims, seed + 1, device="cuda")
    chi = synth.gaussian_spinor(dims, seed + 2, device="cuda")
    return s, psi, chi


def test_noalloc_force_matches_dd_force_on_two_calls():
    cases = [((16, 16, 16, 16), 301, False), ((8, 8, 8, 8), 311, True)]
    assert 16 ** 4 <= MAX_SITES
    runs = []
    for dims, seed, su3 in cases:
        s, psi, chi = make(dims, seed)
        ref, dref = s.force(psi, chi, su3=su3)
        runs.append((s, psi, chi, su3, ref, dref))
    torch.cuda.synchronize()
    outs = []
    for s, psi, chi, su3, ref, dref in runs:  # the two allocation-free calls back to back
        out = torch.full_like(ref, float("nan"))
        d = dd.binding.dd_force_noalloc(s.ctx, out, psi, chi, int(su3), s.shape)
        outs.append((out, d))
    torch.cuda.synchronize()
    for (s, psi, chi, su3, ref, dref), (out, d) in zip(runs, outs):
        assert torch.equal(out, ref), float((out - ref).abs().max())
        assert d == dref
        s.close()


def test_noalloc_force_refuses_a_lattice_beyond_its_array():
    dims = (16, 16, 16, 32)  # 131072 sites
    assert 16 ** 3 * 32 > MAX_SITES
    s, psi, chi = make(dims, 321)
    out = torch.zeros((4,) + s.shape + (3, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(dd.DDError) as e:
        dd.binding.dd_force_noalloc(s.ctx, out, psi, chi, 0, s.shape)
    assert e.value.status == -1 and "too large" in str(e.value) and str(MAX_SITES) in str(e.value)
    assert torch.count_nonzero(out).item() == 0
    L = dd.lib()
    null = ctypes.c_void_p(0)
    assert L.dd_force_noalloc(null, null, None, null, null, 0) == -1
    s.close()
