"""torch.autograd wrapper of the hand-written adjoint, and coefficient refinement.

TriggerPower(strain, C) -> p_i = |rho_{j_i}[n_i]|^2 for a frozen trigger set S,
with rho = C beta (Eq. Beta_eqn) computed by the library (rb_rho_at) and
gradients with respect to the strain and the coefficient matrix C from the
adjoint kernels (rb_backward, seeded with the incoming gradient).

refine_coefficients(): marshals rb_refine, the library's projected gradient
ascent of |rho|^2 over unit-norm coefficient vectors in the span of a trigger
template's coefficients and those of its nearest bank neighbours (largest
|<c_j, c_l>|): the search for a better template "between bank points" that
the basis representation makes cheap.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np
import torch

from . import rbmf


class TriggerPower(torch.autograd.Function):
    @staticmethod
    def forward(fctx, strain: torch.Tensor, C: torch.Tensor, lib_ctx, basis, S) -> torch.Tensor:
        strain = strain.detach().contiguous()
        Cc = C.detach().contiguous()
        n = S.shape[0]
        rho = torch.empty(n, dtype=torch.complex64, device=strain.device)
        rbmf.rho_at(lib_ctx, basis, strain, S, coeffs=Cc, out=rho)
        fctx.save_for_backward(strain, Cc)
        fctx.lib = (lib_ctx, basis, S)
        return rho.real * rho.real + rho.imag * rho.imag

    @staticmethod
    def backward(fctx, grad_p: torch.Tensor):
        strain, Cc = fctx.saved_tensors
        lib_ctx, basis, S = fctx.lib
        want_s, want_C = fctx.needs_input_grad[0], fctx.needs_input_grad[1]
        gC = torch.zeros_like(Cc) if want_C else None
        gs = torch.zeros_like(strain) if want_s else None
        seed = grad_p.detach().to(torch.float32).contiguous()
        rbmf.rb_backward(lib_ctx, basis, strain, S, seed=seed, coeffs=Cc, want_C=want_C,
                         want_strain=want_s, grad_C=gC, grad_strain=gs)
        return gs, gC, None, None, None


def trigger_power(strain, C, lib_ctx, basis, S):
    return TriggerPower.apply(strain, C, lib_ctx, basis, S)


def refine_coefficients(lib_ctx, basis, strain, trig: np.ndarray, neighbours: int = 8, iters: int = 40
                        ) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """Refinement of every trigger in `trig` (rb_refine: neighbour search,
    span basis and projected gradient ascent all run in the library).

    Returns (refined coefficient rows (n x K complex64), neighbours used
    (n x neighbours global template indices), initial |rho|^2, final |rho|^2)."""
    S = np.ascontiguousarray(trig, dtype=rbmf.TRIGGER_NP)
    c, nbr, p = rbmf.refine(lib_ctx, basis, strain, S, neighbours=neighbours, iters=iters)
    return c, nbr, p[:, 0].copy(), p[:, 1].copy()
