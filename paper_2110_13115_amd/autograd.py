"""torch.autograd wrapper of the hand-written adjoint, and coefficient refinement.

TriggerPower(strain, C) -> p_i = |rho_{j_i}[n_i]|^2 for a frozen trigger set S,
with rho = C beta (Eq. Beta_eqn) computed by the library (rb_rho_at) and
gradients with respect to the strain and the coefficient matrix C from the
adjoint kernels (rb_backward, seeded with the incoming gradient).

refine_coefficients(): projected gradient ascent of |rho|^2 over unit-norm
coefficient vectors in the span of a trigger template's coefficients and those
of its nearest bank neighbours (largest |<c_j, c_l>|): the search for a better
template "between bank points" that the basis representation makes cheap.
"""
from __future__ import annotations

from typing import List, Optional, Tuple

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


def nearest_neighbours(c: np.ndarray, j: int, m: int) -> np.ndarray:
    """Indices of the m templates with the largest |<c_j, c_l>| (l != j)."""
    ov = np.abs(c @ np.conj(c[j]))
    ov[j] = -1.0
    return np.argsort(-ov, kind="stable")[:m]


def refine_coefficients(lib_ctx, basis, strain: torch.Tensor, trig: np.ndarray, neighbours: int = 8,
                        iters: int = 40, step: Optional[float] = None
                        ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """One trigger per template (the first occurrence in `trig` is used).

    Returns (C_refined rows for those templates (n x K complex64), initial
    |rho|^2, final |rho|^2)."""
    V, c, lam = basis.export()
    T, K = c.shape
    _, first = np.unique(trig["tmpl"], return_index=True)
    S = np.ascontiguousarray(trig[np.sort(first)])
    n = S.shape[0]
    dev = strain.device
    # orthonormal span (in C = conj(c) space) per trigger
    Q = np.zeros((n, K, neighbours + 1), dtype=np.complex128)
    C0 = np.conj(c).astype(np.complex64)
    for i, j in enumerate(S["tmpl"]):
        idx = np.concatenate([[j], nearest_neighbours(c, int(j), neighbours)])
        q, _ = np.linalg.qr(np.conj(c[idx]).T)
        Q[i] = q
    Qt = torch.from_numpy(Q.astype(np.complex64)).to(dev)
    C = torch.from_numpy(C0).to(dev)
    rows = torch.from_numpy(S["tmpl"].astype(np.int64)).to(dev)
    # S rows point at their own template rows of C
    hist = []
    for it in range(iters + 1):
        Cv = C.clone().requires_grad_(True)
        p = trigger_power(strain, Cv, lib_ctx, basis, S)
        hist.append(p.detach().cpu().numpy())
        if it == iters:
            break
        p.sum().backward()
        g = Cv.grad[rows]                                   # n x K
        cur = C[rows]
        if step is None:
            # step 1/(2 |rho|^2 / |C|^2)-like scale: |rho|^2 <= |Z|^2 for unit C
            lr = 0.5 / torch.clamp(p.detach(), min=1e-12)
        else:
            lr = torch.full_like(p.detach(), step)
        new = cur + lr[:, None] * g
        # project onto the span and renormalise
        coef = torch.einsum("nkr,nk->nr", Qt.conj(), new)
        new = torch.einsum("nkr,nr->nk", Qt, coef)
        new = new / torch.linalg.vector_norm(new, dim=1, keepdim=True)
        C = C.clone()
        C[rows] = new
    return C[rows].cpu().numpy(), hist[0], hist[-1]
