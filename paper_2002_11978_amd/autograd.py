"""u^M of the fast implicit difference scheme as a differentiable torch op.

`solve(params, kappa, f, phi)` runs the forward levels on the GPU and returns
u^M ([n]); its backward runs the library's discrete adjoint (transposed
solves and the reversed SOE history recurrence) and returns dJ/dkappa,
dJ/df and dJ/dphi.  Unless the parameters already keep every state
(store_states) or checkpoint, the forward snapshots its state every
`checkpoint_every` levels (default 32) and the backward recomputes each
segment from its snapshot.
"""
from __future__ import annotations

import ctypes

import torch

from . import fids


def _adjoint_params(params: fids.Params, checkpoint_every: int) -> fids.Params:
    p = fids.Params()
    ctypes.pointer(p)[0] = params
    if not p.store_states and p.checkpoint_every <= 0:
        p.checkpoint_every = checkpoint_every
    return p


class FidsSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa, f, phi, params, checkpoint_every):
        prm = _adjoint_params(params, checkpoint_every)
        # the handle borrows its inputs: keep contiguous copies alive with it
        k, ff, ph = (t.detach().contiguous() for t in (kappa, f, phi))
        prob = fids.Problem(prm, k, ff, ph)
        uT, _, _ = prob.solve_all()
        ctx.prob = prob
        ctx.reports = prob.last_reports
        return uT

    @staticmethod
    def backward(ctx, grad_uT):
        prob = ctx.prob
        need_k, need_f, need_phi = ctx.needs_input_grad[:3]
        gk, gf, gphi = prob.adjoint(grad_uT.detach().contiguous().to(torch.float64),
                                    allocate=False,
                                    g_kappa=torch.empty_like(prob.kappa) if need_k else None,
                                    g_f=torch.empty_like(prob.f) if need_f else None,
                                    g_phi=torch.empty_like(prob.phi) if need_phi else None)
        prob.close()
        ctx.prob = None
        return gk, gf, gphi, None, None


def solve(params: fids.Params, kappa, f, phi, checkpoint_every: int = 32):
    """u^M for float64 device tensors kappa ([M][n] or [n]), f ([M][n]), phi ([n])."""
    return FidsSolve.apply(kappa, f, phi, params, checkpoint_every)
