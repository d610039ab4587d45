"""L = |D^{-1} phi|^2 as a differentiable function of the gauge links, the
source and c_SW, behind torch.autograd.Function.

Forward: psi = D^{-1} phi (bicgstab_solve), L = |psi|^2 (dd_spinor_norm2).
Backward: chi = D^{-dagger} psi (bicgstab_solve_dagger, D^dagger = gamma_5 D
gamma_5), then dd_force gives the per-link gradient and dL/dc_SW; the source
gradient is 2 chi (L = phi^dagger D^{-dagger} D^{-1} phi).  All three are in
PyTorch's convention for a real function of complex inputs:
dL/dRe z + i dL/dIm z.  Every step runs in the HIP library; this module only
sequences the calls.
"""
import torch

from . import binding as dd


class QuarkLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, phi, csw, solver, tol, mode):
        c = float(csw)
        if c != solver.params.csw:
            solver.set_csw(c)
        solver.load_gauge(U.detach().contiguous())
        psi, info = solver.solve(phi.detach().contiguous(), tol=tol, mode=mode)
        if info["status"] != "DD_OK":
            raise RuntimeError(f"forward solve: {info}")
        ctx.solver, ctx.tol, ctx.mode, ctx.csw = solver, tol, mode, c
        ctx.gauge_version = solver.gauge_version
        ctx.save_for_backward(U, psi)
        ctx.csw_device = csw.device if isinstance(csw, torch.Tensor) else torch.device("cpu")
        return torch.tensor(solver.norm2(psi), dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, gL):
        U, psi = ctx.saved_tensors
        solver = ctx.solver
        if solver.gauge_version != ctx.gauge_version or solver.params.csw != ctx.csw:
            # the context was used for another field in between: restore this one
            if solver.params.csw != ctx.csw:
                solver.set_csw(ctx.csw)
            solver.load_gauge(U.detach().contiguous())
        chi, info = solver.solve_dagger(psi, tol=ctx.tol, mode=ctx.mode)
        if info["status"] != "DD_OK":
            raise RuntimeError(f"adjoint solve: {info}")
        need_U, need_phi, need_csw = ctx.needs_input_grad[:3]
        gU = gphi = gcsw = None
        if need_U or need_csw:
            G, dcsw = solver.force(psi, chi, su3=False, want_dcsw=need_csw)
            if need_U:
                gU = G.mul_(gL)
            if need_csw:
                gcsw = (gL.to(ctx.csw_device) * dcsw).to(torch.float64)
        if need_phi:
            gphi = chi.mul_(2.0 * gL)
        return gU, gphi, gcsw, None, None, None


def quark_loss(U, phi, csw, solver, tol=1e-10, mode=dd.DD_SOLVE_MIXED):
    """L = |D[U, c_SW]^{-1} phi|^2 on `solver`'s lattice; U, phi complex128 canonical
    tensors on the GPU, csw a float64 scalar tensor (any of them may require grad)."""
    if not isinstance(csw, torch.Tensor):
        csw = torch.tensor(float(csw), dtype=torch.float64)
    return QuarkLoss.apply(U, phi, csw, solver, tol, mode)
