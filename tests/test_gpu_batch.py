"""Parity of the batched right-hand-side path with the FP64 CPU oracle.

* dirac_apply_batch (FP32 A on the matrix cores) for every kernel variant and
  for the autotuner's choice, full tiles of 12, a partial tile, and 13 right-hand
  sides (two tiles), against the oracle's A applied to each right-hand side:
  the FP32 bar of a single Dirac apply (1e-6, relative L2) per right-hand side;
* the FP64 batched D against the single-field FP64 D, bit for bit;
* bicgstab_solve_batch on the 12 spin-colour point sources at the origin, with
  and without the SAP preconditioner, against 12 independent oracle solves.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2109_10687_amd as dd
import synth

pytestmark = pytest.mark.gpu

CASES = {
    # name: dims, block, kappa, csw, eps, phases
    "4^4": ((4, 4, 4, 4), (2, 2, 2, 2), 0.12, 1.0, 0.5, (1, 1, 1, -1)),
    "aniso": ((8, 4, 16, 8), (4, 2, 4, 2), 0.13, 1.3, 0.4, (1, np.exp(0.3j), 1, np.exp(-0.7j))),
    "8^4": ((8, 8, 8, 8), (4, 4, 4, 4), 0.1365, 1.7, 0.3, (1, 1, 1, -1)),
}

_cache = {}


def setup(name):
    if name not in _cache:
        dims, block, kappa, csw, eps, phases = CASES[name]
        op = O.Params(dims=dims, kappa=kappa, csw=csw, block=block, phases=phases)
        gp = dd.Params(dims=dims, kappa=kappa, csw=csw, block=block, phases=phases)
        U = synth.su3_links(dims, eps, 301)
        _cache[name] = (op, gp, U, O.Oracle(op, U.numpy()), dd.Solver(gp, U.cuda()))
    return _cache[name]


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("variant", [-1] + list(range(13)))
def test_apply_batch_fp32_matches_oracle(name, variant):
    op, gp, U, orc, s = setup(name)
    s.batch_variant(variant)
    try:
        for nrhs in (12, 5, 13):
            xs = synth.gaussian_spinor(op.dims, 311 + nrhs, batch=nrhs)
            out = s.apply_batch(xs.cuda(), op=dd.DD_OP_A, prec=dd.DD_F32).cpu().numpy()
            errs = [rel_l2(out[r], orc.A(xs[r].numpy())) for r in range(nrhs)]
            assert max(errs) < 1e-6, (nrhs, errs)
            # the single right-hand-side FP32 apply agrees to rounding
            one = s.apply(xs[nrhs - 1].cuda(), op=dd.DD_OP_A, prec=dd.DD_F32).cpu().numpy()
            assert rel_l2(out[nrhs - 1], one) < 1e-6
    finally:
        s.batch_variant(-1)
    if variant == -1:
        t = s.batch_tuning(12)
        assert t["variant"] >= 0 and t["timed"] == 13
        assert t["ms"][t["name"]] == min(t["ms"].values())
        print(f"{name}: autotuner picked '{t['name']}' from {t['ms']}")


def test_apply_batch_fp64_D_is_the_single_apply():
    op, gp, U, orc, s = setup("aniso")
    xs = synth.gaussian_spinor(op.dims, 321, batch=3).cuda()
    out = s.apply_batch(xs, op=dd.DD_OP_D, prec=dd.DD_F64)
    for r in range(3):
        assert torch.equal(out[r], s.apply(xs[r], op=dd.DD_OP_D, prec=dd.DD_F64))


@pytest.mark.parametrize("inner", [dd.DD_BATCH_INNER_SAP, dd.DD_BATCH_INNER_PLAIN])
def test_solve_batch_point_sources_match_oracle(inner):
    name = "8^4"
    op, gp, U, orc, s = setup(name)
    # keep this solve well away from criticality: the oracle's plain BiCGStab is the reference
    op2 = O.Params(dims=op.dims, kappa=0.128, csw=op.csw, block=op.block, phases=op.phases)
    gp2 = dd.Params(dims=gp.dims, kappa=0.128, csw=gp.csw, block=gp.block, phases=gp.phases, n_sap=4)
    s2 = dd.Solver(gp2, U.cuda())
    orc2 = O.Oracle(op2, U.numpy())
    bs = torch.stack([synth.point_source(op.dims, c, sp) for c in range(3) for sp in range(4)])
    x, infos = s2.solve_batch(bs.cuda(), tol=1e-10, inner=inner)
    xn = x.cpu().numpy()
    for r in range(12):
        assert infos[r]["status"] == "DD_OK", (r, infos[r])
        assert infos[r]["relres_true"] < 1e-10
        ref = orc2.solve(bs[r].numpy(), tol=1e-12)
        assert ref.status == 0
        assert rel_l2(xn[r], ref.x) < 1e-8, r
        # the oracle's own residual of the GPU solution
        res = np.linalg.norm(orc2.D(xn[r]) - bs[r].numpy()) / np.linalg.norm(bs[r].numpy())
        assert res < 1e-10
    print(f"batched solve ({'SAP' if inner == 0 else 'no preconditioner'}): outer "
          f"{[i['iters_outer'] for i in infos]}, inner {[i['iters_inner_total'] for i in infos]}, "
          f"{infos[0]['seconds']:.2f} s")
    s2.close()


# ---------------------------------------------------------------- several lattices in one launch

# the uneven set of eight lattices (two each of 8^4, 12^4, 16^4, 16^3 x 32), each with its own
# links, kappa and boundary phases; 12^4 takes 2^4 blocks (12 / 4 blocks per direction is odd)
MULTI = [((8, 8, 8, 8), (4, 4, 4, 4), 0.125, 1.7, (1, 1, 1, -1)),
         ((8, 8, 8, 8), (4, 4, 4, 4), 0.12, 1.5, (1, np.exp(0.4j), 1, -1)),
         ((12, 12, 12, 12), (2, 2, 2, 2), 0.125, 1.7, (1, 1, 1, -1)),
         ((12, 12, 12, 12), (2, 2, 2, 2), 0.122, 1.0, (-1, 1, 1, np.exp(0.2j))),
         ((16, 16, 16, 16), (4, 4, 4, 4), 0.125, 1.7, (1, 1, 1, -1)),
         ((16, 16, 16, 16), (4, 4, 4, 4), 0.12, 1.7, (1, 1, np.exp(-0.3j), -1)),
         ((16, 16, 16, 32), (4, 4, 4, 4), 0.125, 1.7, (1, 1, 1, -1)),
         ((16, 16, 16, 32), (4, 4, 4, 4), 0.124, 1.3, (1, 1, 1, -1))]


def multi_setup():
    if "multi" not in _cache:
        ops, gps, Us = [], [], []
        for k, (dims, block, kappa, csw, phases) in enumerate(MULTI):
            ops.append(O.Params(dims=dims, kappa=kappa, csw=csw, block=block, phases=phases))
            gps.append(dd.Params(dims=dims, kappa=kappa, csw=csw, block=block, phases=phases))
            Us.append(synth.su3_links(dims, 0.3, 400 + k))
        m = dd.Multi(gps)
        for k, U in enumerate(Us):
            m.load_gauge(k, U.cuda())
        _cache["multi"] = (ops, gps, Us, m)
    return _cache["multi"]


def test_apply_multi_matches_oracle():
    ops, gps, Us, m = multi_setup()
    xs = [synth.gaussian_spinor(p.dims, 410 + k) for k, p in enumerate(ops)]
    outs = m.apply([x.cuda() for x in xs])
    for k, (p, U, x, o) in enumerate(zip(ops, Us, xs, outs)):
        want = O.dirac_A(p, U.numpy(), O.clover_inverse(p, O.clover_field(p, U.numpy())), x.numpy())
        assert rel_l2(o.cpu().numpy(), want) < 1e-6, k
    # the one-launch result equals the lattice's own FP32 apply to rounding
    s = dd.Solver(gps[2], Us[2].cuda())
    one = s.apply(xs[2].cuda(), op=dd.DD_OP_A, prec=dd.DD_F32)
    assert rel_l2(outs[2].cpu().numpy(), one.cpu().numpy()) < 1e-6
    s.close()


def test_solve_multi_matches_oracle():
    ops, gps, Us, m = multi_setup()
    bs = [synth.gaussian_spinor(p.dims, 420 + k) for k, p in enumerate(ops)]
    xs, infos = m.solve([b.cuda() for b in bs], tol=1e-10)
    for k, (p, U, b, x, inf) in enumerate(zip(ops, Us, bs, xs, infos)):
        assert inf["status"] == "DD_OK" and inf["relres_true"] < 1e-10, (k, inf)
        orc = O.Oracle(p, U.numpy())
        xn = x.cpu().numpy()
        # the oracle's residual of the GPU solution on every lattice
        res = np.linalg.norm(orc.D(xn) - b.numpy()) / np.linalg.norm(b.numpy())
        assert res < 1e-10, (k, res)
        if p.volume <= 12 ** 4:  # the oracle's own solve where it takes seconds
            ref = orc.solve(b.numpy(), tol=1e-12)
            assert ref.status == 0
            assert rel_l2(xn, ref.x) < 1e-8, k
    print("multi-lattice solve: outer", [i["iters_outer"] for i in infos], "inner",
          [i["iters_inner_total"] for i in infos], f"{infos[0]['seconds']:.2f} s")


@pytest.mark.parametrize("fp16_arith", [1, 0])
@pytest.mark.parametrize("name", ["aniso", "8^4", "8^4-twist"])
def test_sap_batch_matches_single_and_oracle(name, fp16_arith):
    """sap_precondition_batch on 5 right-hand sides: with packed FP16 arithmetic every half-sweep is
    one launch for all five (links and C_inv staged once per block), with FP32 arithmetic one SAP
    per right-hand side.  Each result equals sap_precondition on that right-hand side alone, bit
    for bit (the same arithmetic in the same order), and is within the FP16-storage SAP bar of the
    oracle's Alg. 1 (3e-3 packed FP16, 1.2e-3 FP32, relative L2)."""
    cases = dict(CASES)
    cases["8^4-twist"] = ((8, 8, 8, 8), (4, 4, 4, 4), 0.125, 1.5, 0.3,
                          (np.exp(0.3j), np.exp(-0.5j), np.exp(1.1j), -np.exp(0.2j)))
    dims, block, kappa, csw, eps, phases = cases[name]
    op = O.Params(dims=dims, kappa=kappa, csw=csw, block=block, phases=phases, n_sap=2, n_jac=4)
    gp = dd.Params(dims=dims, kappa=kappa, csw=csw, block=block, phases=phases, n_sap=2, n_jac=4,
                   sap_fp16_arith=fp16_arith)
    U = synth.su3_links(dims, eps, 331)
    orc = O.Oracle(op, U.numpy())
    s = dd.Solver(gp, U.cuda())
    bs = synth.gaussian_spinor(dims, 332, batch=5).cuda()
    xb = s.precondition_batch(bs).cpu().numpy()
    for r in range(5):
        one = s.precondition(bs[r], prec=dd.DD_F16).cpu().numpy()
        assert np.array_equal(xb[r], one), r
        err = rel_l2(xb[r], orc.sap(bs[r].cpu().numpy()))
        assert err < (3e-3 if fp16_arith else 1.2e-3), (r, err)
    s.close()


def test_solve_multi_more_lattices_than_one_table_holds():
    """Twenty lattices in one lockstep solve: more than one table launch of the vector kernels
    (16 lattices each) and of the shared half-sweep (12 each).  Every lattice must reach the
    requested true residual, recomputed by the oracle."""
    specs = [((8, 8, 8, 8), (4, 4, 4, 4), 0.12 + 0.0005 * k, 1.0 + 0.05 * k) for k in range(18)]
    specs += [((4, 4, 4, 4), (2, 2, 2, 2), 0.12, 1.0), ((4, 4, 4, 4), (2, 2, 2, 2), 0.118, 1.2)]
    ops, gps, Us = [], [], []
    for k, (dims, block, kappa, csw) in enumerate(specs):
        ops.append(O.Params(dims=dims, kappa=kappa, csw=csw, block=block))
        gps.append(dd.Params(dims=dims, kappa=kappa, csw=csw, block=block))
        Us.append(synth.su3_links(dims, 0.3, 500 + k))
    m = dd.Multi(gps)
    for k, U in enumerate(Us):
        m.load_gauge(k, U.cuda())
    bs = [synth.gaussian_spinor(p.dims, 530 + k) for k, p in enumerate(ops)]
    xs, infos = m.solve([b.cuda() for b in bs], tol=1e-10)
    for k, (p, U, b, x, inf) in enumerate(zip(ops, Us, bs, xs, infos)):
        assert inf["status"] == "DD_OK" and inf["relres_true"] < 1e-10, (k, inf)
        orc = O.Oracle(p, U.numpy())
        res = np.linalg.norm(orc.D(x.cpu().numpy()) - b.numpy()) / np.linalg.norm(b.numpy())
        assert res < 1e-10, (k, res)
    m.close()
