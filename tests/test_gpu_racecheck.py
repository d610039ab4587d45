"""LDS race check.  libddsolve_racecheck.so is the library with its kernels built under
DD_RACE_CHECK=1: in every kernel whose wavefronts share LDS (the t-streamed and
multi-lattice Dirac applies, both SAP half-sweeps, the reductions) wavefront w of W
waits (W-1-w) sleep periods at entry and after every workgroup barrier, so the
wavefronts of a workgroup run each phase in the reverse of their usual order.  A
missing barrier would then change what some wavefront reads from LDS.  Every result
must equal the product library's bit for bit: the operators, the SAP at every
precision (single, batched and several lattices per launch), A M_SAP with the fused
tail, norms, and whole solves (whose reductions are order-fixed).

Lattices: 8^4 with 4^4 blocks (one block per workgroup everywhere) and 32^4 (4096
blocks: the FP64 / FP32 / FP16-input applies walk four blocks per workgroup and hand
the t-face over in LDS).
"""
import contextlib
import os

import pytest
import torch

import paper_2109_10687_amd as dd
import synth

pytestmark = pytest.mark.gpu

RACE = dd.binding.LIB_RACE_PATH


def outputs(dims, race):
    U = synth.su3_links(dims, 0.3, 61, device="cuda")
    x = synth.gaussian_spinor(dims, 62, device="cuda")
    out, out_ms = {}, [0.0]
    with dd.binding.use_library(RACE) if race else contextlib.nullcontext():
        for arith in (1, 0):
            s = dd.Solver(dd.Params(dims=dims, kappa=0.13, csw=1.7, sap_fp16_arith=arith), U)
            out[f"sap16 arith{arith}"] = s.precondition(x, prec=dd.DD_F16)
            if arith == 0:
                s.close()
                continue
            out["D64"] = s.apply(x, op=dd.DD_OP_D, prec=dd.DD_F64)
            out["Ddag64"] = s.apply(x, op=dd.DD_OP_DDAG, prec=dd.DD_F64)
            out["A32"] = s.apply(x, op=dd.DD_OP_A, prec=dd.DD_F32)
            out["A16"] = s.apply(x, op=dd.DD_OP_A, prec=dd.DD_F16)
            f16 = s.pack(x, dd.DD_F16)
            f32 = s.field(dd.DD_F32)
            s.apply_packed_f16in(f32, f16)
            out["A16in"] = s.unpack(f32, dd.DD_F32)
            out["sap32"] = s.precondition(x, prec=dd.DD_F32)
            out["amsap32"] = s.amsap(x, prec=dd.DD_F32)
            bs = torch.stack([x, 2 * x.flip(0), x.roll(1, 1)])
            out["sap16 batch"] = s.precondition_batch(bs)
            out["norm2"] = torch.tensor([dd.dd_spinor_norm2(s.ctx, x, s.shape)])
            # the SAP half-sweeps' kernel time, to see that the build's waits are in place
            s.timing(True)
            for _ in range(3):
                s.precondition(x, prec=dd.DD_F16)
            out_ms[0] = s.timing_report()["sap"]["ms"]
            s.timing(False)
            for mode in (dd.DD_SOLVE_MIXED, dd.DD_SOLVE_FGMRES):
                xs, info = s.solve(x, tol=1e-10, maxiter=20, mode=mode)
                assert info["status"] == "DD_OK", info
                out[f"solve mode {mode}"] = xs
            s.close()
        if dims == (8, 8, 8, 8):
            ps = [dd.Params(dims=d, kappa=0.13, csw=1.7) for d in ((8, 8, 8, 8), (8, 8, 8, 16))]
            m = dd.Multi(ps)
            xs = []
            for k, p in enumerate(ps):
                m.load_gauge(k, synth.su3_links(p.dims, 0.3, 70 + k, device="cuda"))
                xs.append(synth.gaussian_spinor(p.dims, 80 + k, device="cuda"))
            for k, y in enumerate(m.apply(xs)):
                out[f"multi A {k}"] = y
            sol, infos = m.solve(xs, tol=1e-10)
            assert all(i["status"] == "DD_OK" for i in infos), infos
            for k, y in enumerate(sol):
                out[f"multi solve {k}"] = y
            m.close()
    torch.cuda.synchronize()
    return out, out_ms[0]


@pytest.mark.skipif(not os.path.exists(RACE), reason="race-check library not built")
@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (32, 32, 32, 32)])
def test_reversed_wavefront_order_is_bitwise_identical(dims):
    ref, ms_ref = outputs(dims, race=False)
    got, ms_race = outputs(dims, race=True)
    print(f"SAP kernel time, 3 applications: {ms_ref:.3f} ms product build, {ms_race:.3f} ms race-check build")
    assert ms_race > 1.5 * ms_ref  # the reversed-order waits ran
    assert ref.keys() == got.keys()
    bad = [k for k in ref if not torch.equal(ref[k], got[k])]
    assert not bad, f"results differ under reversed wavefront order: {bad}"
