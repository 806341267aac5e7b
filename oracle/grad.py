"""Loss over a frozen trigger set and its gradients (test infrastructure only;
see package docstring).

The loss is L = sum_i g_i |rho_RB_{j_i}[n_i]|^2 with
rho_RB_j[n] = sum_k C_{jk} beta_k[n] (Eq. Beta_eqn, C = conj(c)) and
beta_k[n] = sum_{f in band} d[f] conj(v_k[f]) e^{+2 pi i f n / N},
d[f] = w[f] dt rfft(s)[f], w = sqrt(4 df / Sn).

The forward here evaluates beta only at the trigger samples by direct sums
(an explicit phase matrix), not by inverse FFTs, and torch CPU float64
autograd differentiates it.  Gradients follow torch's convention for complex
leaves (for real L, grad = dL/dRe + i dL/dIm).
"""
from __future__ import annotations

from typing import Tuple

import numpy as np
import torch


def _beta_at(s: torch.Tensor, V: torch.Tensor, w: torch.Tensor, k_lo: int, fs: float,
             samp: torch.Tensor) -> torch.Tensor:
    """beta_k[n_i] (K x m) by direct sums over the band."""
    N = s.shape[0]
    nb = V.shape[1]
    d = torch.fft.rfft(s)[k_lo:k_lo + nb] * w / fs                    # whitened data on the band
    f = torch.arange(k_lo, k_lo + nb, dtype=torch.float64)
    ph = torch.exp(2j * np.pi * torch.outer(f, samp.to(torch.float64)) / N)  # nb x m
    return (d[None, :] * torch.conj(V)) @ ph


def _loss_from_beta(C: torch.Tensor, beta: torch.Tensor, tmpl: torch.Tensor, g: torch.Tensor) -> torch.Tensor:
    """sum_i g_i |sum_k C[j_i, k] beta[k, i]|^2."""
    rho = torch.sum(C[tmpl, :] * beta.T, dim=1)                         # m
    return torch.sum(g * (rho.real ** 2 + rho.imag ** 2))


def _forward(s: torch.Tensor, C: torch.Tensor, V: torch.Tensor, w: torch.Tensor, k_lo: int,
             fs: float, tmpl: torch.Tensor, samp: torch.Tensor, g: torch.Tensor) -> torch.Tensor:
    return _loss_from_beta(C, _beta_at(s, V, w, k_lo, fs, samp), tmpl, g)


def beta_at(s: np.ndarray, V: np.ndarray, w: np.ndarray, k_lo: int, fs: float, samp: np.ndarray) -> np.ndarray:
    """The basis outputs beta_k (Eq. Beta_eqn) at the samples `samp` only,
    K x m complex128.  beta is linear in s, so beta(s + e v) = beta(s) +
    e beta(v): one evaluation per strain direction serves a central
    difference."""
    with torch.no_grad():
        return _beta_at(torch.as_tensor(np.asarray(s, np.float64)), torch.as_tensor(np.asarray(V, np.complex128)),
                        torch.as_tensor(np.asarray(w, np.float64)), k_lo, fs,
                        torch.as_tensor(np.asarray(samp, np.int64))).numpy()


def loss_from_beta(C: np.ndarray, beta: np.ndarray, tmpl: np.ndarray, g: np.ndarray) -> float:
    """The loss given the basis outputs at the trigger samples (column i of
    beta at sample n_i)."""
    with torch.no_grad():
        return float(_loss_from_beta(torch.as_tensor(np.asarray(C, np.complex128)),
                                     torch.as_tensor(np.asarray(beta, np.complex128)),
                                     torch.as_tensor(np.asarray(tmpl, np.int64)),
                                     torch.as_tensor(np.asarray(g, np.float64))))


def loss(s: np.ndarray, C: np.ndarray, V: np.ndarray, w: np.ndarray, k_lo: int, fs: float,
         tmpl: np.ndarray, samp: np.ndarray, g: np.ndarray) -> float:
    with torch.no_grad():
        return float(_forward(torch.as_tensor(np.asarray(s, np.float64)),
                              torch.as_tensor(np.asarray(C, np.complex128)),
                              torch.as_tensor(np.asarray(V, np.complex128)),
                              torch.as_tensor(np.asarray(w, np.float64)), k_lo, fs,
                              torch.as_tensor(np.asarray(tmpl, np.int64)),
                              torch.as_tensor(np.asarray(samp, np.int64)),
                              torch.as_tensor(np.asarray(g, np.float64))))


def loss_and_grads(s: np.ndarray, C: np.ndarray, V: np.ndarray, w: np.ndarray, k_lo: int,
                   fs: float, tmpl: np.ndarray, samp: np.ndarray,
                   g: np.ndarray) -> Tuple[float, np.ndarray, np.ndarray]:
    """(L, dL/dC (T x K complex, torch convention), dL/ds (N real))."""
    st = torch.tensor(np.asarray(s, np.float64), requires_grad=True)
    Ct = torch.tensor(np.asarray(C, np.complex128), requires_grad=True)
    L = _forward(st, Ct, torch.as_tensor(np.asarray(V, np.complex128)),
                 torch.as_tensor(np.asarray(w, np.float64)), k_lo, fs,
                 torch.as_tensor(np.asarray(tmpl, np.int64)),
                 torch.as_tensor(np.asarray(samp, np.int64)),
                 torch.as_tensor(np.asarray(g, np.float64)))
    L.backward()
    return float(L.detach()), Ct.grad.numpy().copy(), st.grad.numpy().copy()


def refine_optimum(Zn: np.ndarray, span: np.ndarray) -> Tuple[np.ndarray, float]:
    """Maximiser of |sum_k conj(c_k) Z_k|^2 over unit-norm c in the span of the
    rows of `span` (each a coefficient vector).  By Cauchy-Schwarz the optimum
    is the normalised orthogonal projection of Z onto that span and its value
    is the squared norm of that projection."""
    Q, _ = np.linalg.qr(np.asarray(span, np.complex128).T)     # K x r orthonormal columns
    p = Q @ (Q.conj().T @ Zn)
    nrm = float(np.linalg.norm(p))
    return p / nrm, nrm ** 2


def nearest_neighbours(c: np.ndarray, j: int) -> np.ndarray:
    """Templates l != j ordered by decreasing |<c_j, c_l>| (ties to the lower
    index), and those overlaps: the neighbour order of the refinement."""
    ov = np.abs(np.asarray(c, np.complex128) @ np.conj(np.asarray(c[j], np.complex128)))
    idx = np.array([l for l in np.lexsort((np.arange(len(ov)), -ov)) if l != j])
    return idx, ov
