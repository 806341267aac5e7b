"""FP64 reduced basis and reduced-basis SNR (test infrastructure only; see
package docstring).

Readings:

* The basis is built from the whitened, unit-norm templates (Sec. III.B: the
  templates are whitened with the PSD and normalised to unity), stored row-wise
  as the T x nb matrix W over the band, with no mean subtraction (Sec. III.B
  skips it).
* Eq. Eq-SVD: W = U S V^H; the basis vectors are the rows v_k of V^H, ranked
  by singular value; the covariance eigenvalues are L = S^2 (Sec. II.A).
* Coefficients (Sec. II.A, III.B): c_{jk} = <w_j, v_k> = sum_f w_j[f]
  conj(v_k[f]), so that w_j ~ sum_k c_{jk} v_k.
* Rank rule (Eq. SNR_loss with the eigenvalues already equal to S^2): the
  smallest K with sum_{k<K} S_k^2 / sum_k S_k^2 >= 1 - tol.
* Reduced-basis SNR (Eqs. basis_SNR, Beta_eqn):
      beta_k[n] = sum_{f in band} d[f] conj(v_k[f]) e^{+2 pi i f n / N},
      rho_RB_j[n] = sum_k conj(c_{jk}) beta_k[n],
  with the whitened data d[f] = s~[f] sqrt(4 df / Sn[f]); no renormalisation
  of the truncated coefficients.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

from . import mf


def whiten_weights(psd: np.ndarray, N: int, fs: float, f_low: float) -> np.ndarray:
    """sqrt(4 df / Sn[k]) on the band, 0 elsewhere (length N/2+1)."""
    df = fs / N
    m = mf.band_mask(N, fs, f_low)
    w = np.zeros(N // 2 + 1)
    w[m] = np.sqrt(4.0 * df / psd[m])
    return w


def whitened_unit_templates(H: np.ndarray, psd: np.ndarray, N: int, fs: float,
                            f_low: float) -> Tuple[np.ndarray, np.ndarray]:
    """(W, sigma): W[j] = h_j w / sigma_j on the band bins k_lo..N/2-1."""
    k_lo, k_hi = mf.band_limits(N, fs, f_low)
    w = whiten_weights(psd, N, fs, f_low)[k_lo:k_hi + 1]
    Hw = H[:, k_lo:k_hi + 1] * w[None, :]
    sig = np.sqrt(np.sum(np.abs(Hw) ** 2, axis=1))
    return Hw / sig[:, None], sig


def svd_basis(W: np.ndarray, rank: int = 0, tol: float = 1e-3):
    """Returns (V, c, s, K, energy): V (K x nb) orthonormal rows, c (T x K)
    coefficients, s all singular values, K the rank, energy the retained
    fraction sum_{k<K} s_k^2 / sum s_k^2."""
    U, s, Vh = np.linalg.svd(W, full_matrices=False)
    e = s ** 2
    cum = np.cumsum(e) / np.sum(e)
    if rank > 0:
        K = min(rank, s.shape[0])
    else:
        K = int(np.searchsorted(cum, 1.0 - tol - 1e-15) + 1)
        K = min(K, s.shape[0])
    V = Vh[:K]
    c = W @ V.conj().T
    return V, c, s, K, float(cum[K - 1])


def whitened_data(s: np.ndarray, psd: np.ndarray, fs: float, f_low: float) -> np.ndarray:
    """d[f] = s~[f] sqrt(4 df / Sn[f]) on the band bins k_lo..N/2-1."""
    N = s.shape[0]
    k_lo, k_hi = mf.band_limits(N, fs, f_low)
    return mf.strain_tilde(s, fs)[k_lo:k_hi + 1] * whiten_weights(psd, N, fs, f_low)[k_lo:k_hi + 1]


def basis_outputs(d: np.ndarray, V: np.ndarray, N: int, k_lo: int) -> np.ndarray:
    """beta_k[n] = sum_f d[f] conj(v_k[f]) e^{+2 pi i f n/N}: K x N complex."""
    K, nb = V.shape
    X = np.zeros((K, N), dtype=np.complex128)
    X[:, k_lo:k_lo + nb] = d[None, :] * np.conj(V)
    return N * np.fft.ifft(X, axis=1)


def rb_snr(beta: np.ndarray, c: np.ndarray) -> np.ndarray:
    """rho_RB = conj(c) @ beta: T x N (Eq. Beta_eqn)."""
    return np.conj(c) @ beta


def mf_whitened(d: np.ndarray, W: np.ndarray, N: int, k_lo: int) -> np.ndarray:
    """rho_j[n] = sum_f d[f] conj(w_j[f]) e^{+2 pi i f n/N} for whitened unit
    templates (the template method in whitened form)."""
    return basis_outputs(d, W, N, k_lo)
