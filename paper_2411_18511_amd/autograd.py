"""torch.autograd.Function wrappers over the HIP library.

The fermion force is the derivative that the HMC (the paper's Sec. 2.1
setting for the even/odd operator) needs; here it is exposed to autograd:

* ``DiracApply``: y = D[U] psi on the full lattice.  Backward:
  grad_psi = D^+ g and grad_U = d/dU Re<g, D[U] psi> (library force kernel).
* ``FermionAction``: S = Re<phi, (D^+ D^)^{-1} phi> on even sites as a
  function of the fundamental SU(2) links; for the adjoint representation the
  links are represented on the GPU and the chain rule back to the
  fundamental links also runs in the library.  Backward:
  grad_U = grad_S * (2/m) G[X, Y] (library action-force kernel), and
  grad_phi = 2 grad_S (D^+ D^)^{-1} phi.

Gradients follow PyTorch's convention for complex tensors,
dL/dRe z + i dL/dIm z; for real (adjoint) links it is the real derivative.
Natural layouts: gauge [4, V, N, N], spinor [V, 4, N], V = T L1 L2 L3.
"""
import torch

from . import hrd


class DiracApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U_nat, psi_nat, dims, rep, m0):
        rep = hrd._REPS[rep]
        U = hrd.pack_gauge(U_nat.contiguous(), dims, rep, "f64")
        psi = hrd.pack_spinor(psi_nat.contiguous(), dims, rep, "f64", "all")
        out = hrd.dirac_apply(U, psi, m0, rep, "full", dims)
        ctx.dims, ctx.rep, ctx.m0 = tuple(dims), rep, float(m0)
        ctx.U, ctx.psi = U, psi
        return hrd.unpack_spinor(out, dims, rep, "f64", "all")

    @staticmethod
    def backward(ctx, g):
        dims, rep = ctx.dims, ctx.rep
        gp = hrd.pack_spinor(g.contiguous(), dims, rep, "f64", "all")
        grad_psi = grad_U = None
        if ctx.needs_input_grad[1]:
            grad_psi = hrd.unpack_spinor(hrd.dirac_apply(ctx.U, gp, ctx.m0, rep, "full", dims, dagger=True), dims,
                                         rep, "f64", "all")
        if ctx.needs_input_grad[0]:
            F = hrd.dirac_force(ctx.U, gp, ctx.psi, dims, rep)
            grad_U = hrd.unpack_gauge(F, dims, rep, "f64")
        return grad_U, grad_psi, None, None, None


class FermionAction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U_fund_nat, phi_nat, dims, rep, m0, tol=1e-10, mode="f64"):
        rep = hrd._REPS[rep]
        Uf64 = hrd.pack_gauge(U_fund_nat.contiguous(), dims, hrd.FUND, "f64")
        U64 = Uf64 if rep == hrd.FUND else hrd.represent(Uf64, dims, "f64")
        U32 = hrd.convert_gauge(U64, dims, rep) if hrd._MODES[mode] == hrd.CG_MIXED else None
        phi = hrd.pack_spinor(phi_nat.contiguous(), dims, rep, "f64", "even")
        xi, info = hrd.cg_solve(U64, phi, m0, tol, dims, rep, mode=mode, U32=U32)
        S = hrd.blas_dot(phi, xi, dims, rep, "f64", 1).real
        ctx.dims, ctx.rep, ctx.m0 = tuple(dims), rep, float(m0)
        ctx.Uf64, ctx.U64, ctx.xi = Uf64, U64, xi
        ctx.info = info
        return torch.tensor(S, dtype=torch.float64, device=phi_nat.device)

    @staticmethod
    def backward(ctx, gS):
        dims, rep = ctx.dims, ctx.rep
        scale = float(gS)
        grad_U = grad_phi = None
        if ctx.needs_input_grad[0]:
            F = hrd.action_force(ctx.U64, ctx.xi, ctx.m0, dims, rep, scale=scale)
            if rep == hrd.ADJ:
                F = hrd.represent_backward(ctx.Uf64, F, dims)
            grad_U = hrd.unpack_gauge(F, dims, hrd.FUND, "f64")
        if ctx.needs_input_grad[1]:
            two_xi = torch.zeros_like(ctx.xi)
            hrd.blas_axpy(2.0 * scale, ctx.xi, two_xi, dims, rep, "f64", 1)
            grad_phi = hrd.unpack_spinor(two_xi, dims, rep, "f64", "even")
        return grad_U, grad_phi, None, None, None, None, None


def dirac_apply(U_nat, psi_nat, dims, rep, m0):
    return DiracApply.apply(U_nat, psi_nat, dims, rep, m0)


def fermion_action(U_fund_nat, phi_nat, dims, rep, m0, tol=1e-10, mode="f64"):
    return FermionAction.apply(U_fund_nat, phi_nat, dims, rep, m0, tol, mode)
