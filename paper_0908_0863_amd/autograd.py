"""torch.autograd wrapper of the absorption cross section and its adjoint
gradient with respect to the per-dipole permittivity.

Forward: set eps on the target, solve A P = E_inc on the GPU, return C_abs per
right-hand side.  Backward: one adjoint solve A mu = W conj(P) (A is complex
symmetric, so the same matrix-vector product serves) and the per-dipole
gradient kernel, both inside libdda (``dda_grad_cabs_eps``).

Convention: for a real loss L of the complex permittivity, the gradient handed
back is dL/dRe eps + i dL/dIm eps, the convention torch uses for complex
leaves (so ``torch.autograd.gradcheck`` applies directly).
"""
from __future__ import annotations

import torch

from . import dda


class CAbs(torch.autograd.Function):
    """C_abs(eps) for every right-hand side of a plane-wave solve.

    ``CAbs.apply(eps, target, khat, ehat, prescription, solve_kw)``
      eps          complex128 tensor [N_d] (any device; moved to the host to set
                   the polarisabilities)
      target       dda.Target with occupancy set and spectrum built
      khat, ehat   [nrhs, 3] propagation directions and polarisations
      prescription "cm" | "rr" | "ldr"
      solve_kw     dict of dda.Target.make_opts keywords for both solves
    returns float64 tensor [nrhs] on the target's device."""

    @staticmethod
    def forward(ctx, eps, target, khat, ehat, prescription="ldr", solve_kw=None):
        kw = dict(solver="qmr_sym", precision="fp64", tol=1e-10)
        kw.update(solve_kw or {})
        e = eps.detach().to("cpu", torch.complex128).numpy()
        target.set_permittivity(e, prescription)
        E = target.incident_field(khat, ehat)
        # the library derives the LDR orientation factors from khat/ehat and
        # reports the ones it used, so the backward pass can hand them back
        P, _ = target.solve(khat=khat, ehat=ehat, **kw)
        S = target.orientation_factors(P.shape[0])
        _, cabs, _ = target.cross_sections(E, P, S=S)
        ctx.target, ctx.prescription, ctx.kw, ctx.S = target, prescription, kw, S
        ctx.eps_host = e
        ctx.eps_device = eps.device
        ctx.save_for_backward(P)
        return torch.as_tensor(cabs, dtype=torch.float64, device=target.dev)

    @staticmethod
    def backward(ctx, grad_out):
        (P,) = ctx.saved_tensors
        t = ctx.target
        # the target may have been given other permittivities since forward
        t.set_permittivity(ctx.eps_host, ctx.prescription)
        g = t.grad_cabs_eps(P, S=ctx.S, **ctx.kw)          # [nrhs, N_d]
        grad = torch.sum(grad_out.to(g.device, torch.float64)[:, None] * g, dim=0)
        return grad.to(ctx.eps_device), None, None, None, None, None


def cabs(eps, target, khat, ehat, prescription="ldr", **solve_kw):
    """Differentiable C_abs [nrhs] (see CAbs)."""
    return CAbs.apply(eps, target, khat, ehat, prescription, solve_kw)
