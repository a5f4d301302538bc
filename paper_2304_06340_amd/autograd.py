"""torch.autograd bridge: d^2 as a differentiable function of vertex positions.

Forward runs hsd_distance (or hsd_distance_grad when a gradient is needed,
which returns d^2 and d(d^2)/dv from one forward pass plus the adjoint
kernel); backward scales the stored gradient by the incoming grad_output.
"""
from __future__ import annotations

import torch

from .api import Context, Mesh, Params, Rule, distance, distance_grad


class HsdDistance(torch.autograd.Function):
    @staticmethod
    def forward(fctx, verts: torch.Tensor, tris: torch.Tensor, hctx: Context, rule: Rule,
                params: Params, nu: Mesh | None):
        mesh = Mesh(hctx, verts.detach(), tris)
        try:
            if verts.requires_grad:
                grad = torch.empty(verts.shape, dtype=torch.float64, device=verts.device)
                res, _ = distance_grad(hctx, mesh, nu, rule, params, out=grad)
                fctx.save_for_backward(grad)
            else:
                res = distance(hctx, mesh, nu, rule, params)
        finally:
            mesh.close()
        return torch.tensor(res.d2, dtype=torch.float64, device=verts.device)

    @staticmethod
    def backward(fctx, g):
        (grad,) = fctx.saved_tensors
        return (g * grad).to(grad.dtype), None, None, None, None, None


def hsd_distance(verts: torch.Tensor, tris: torch.Tensor, hctx: Context, rule: Rule,
                 params: Params | None = None, nu: Mesh | None = None) -> torch.Tensor:
    """Squared H^-s distance of the mesh (verts, tris) to nu (None: S^2)."""
    return HsdDistance.apply(verts, tris, hctx, rule, params or Params(), nu)
