"""FP64 PCA of a bank sampled at non-uniform frequencies, and the linear
interpolation of its basis back onto the uniform rfft grid (Sec. III.A, "PCA
using Non-uniform Sampling"; the interpolation step of Sec. III.C).  Test
infrastructure only (see package docstring).

Readings:

* Frequency set (Sec. III.A): the zero crossings of the real part of one
  reference template (the one with the longest duration) are the edges of
  non-overlapping bins over [f_lo, f_hi]; each bin [e_b, e_{b+1}) is sampled
  at `per_bin` (five in the paper) uniformly spaced frequencies
  e_b + m (e_{b+1} - e_b) / per_bin, m = 0 .. per_bin-1.  The spacing never
  drops below df_min (1/128 Hz in the paper, the grid spacing of its 128 s
  segments): a bin whose per-bin spacing would be finer takes instead the
  multiples of df_min that fall inside it, i.e. the uniform grid itself when
  df_min is the segment's frequency step.  f_hi closes the set.  A crossing
  is a sign change of the real part between consecutive samples of the
  reference, located by linear interpolation, or a sample that is exactly
  zero.
* Extra nodes: the paper's waveforms taper smoothly, TaylorF2 stops
  abruptly at f_ISCO.  Linear interpolation across a wide cell that holds
  such a cut smears it over the cell (a mismatch of order 1e-2 instead of
  1e-5), so the caller may add nodes, merged into the set: for a bank cut at
  f_ISCO, the two uniform frequencies on either side of each template's
  cut.
* Inner product on the set: the cell (midpoint) rule, node i weighing the
  width of the cell between the midpoints to its neighbours, the two end
  cells mirrored (so a set equal to the uniform grid weighs every node by
  the grid step, and the inner product is the uniform one).
* Templates are whitened and normalised to unity in that inner product
  (Sec. III.B), stored row-wise as V (T x N_t) with
  V[j, i] = h_j(f_i) sqrt(4 omega_i / Sn(f_i)) / sigma_j; no mean
  subtraction (Sec. III.B).  The covariance is the N_t x N_t matrix V^H V,
  whose leading eigenvectors (Sec. III.A: EVD ranked by eigenvalue) are the
  basis on the set; the rank rule is that of the uniform basis (smallest K
  whose eigenvalues keep a fraction 1 - tol of the trace), or a fixed rank.
* Interpolation (Sec. III.C): a basis vector divided by sqrt(omega_i) is a
  whitened spectral density; it is interpolated linearly (real and
  imaginary parts) to the uniform frequencies k df of the band and times
  sqrt(df) becomes a vector of the uniform grid's inner product.
* The interpolated vectors are no longer exactly orthonormal on the uniform
  grid; they are orthonormalised there (QR) and the coefficients are the
  projections of the uniform whitened templates onto them, so that the
  reduced-basis SNR keeps its uniform-grid definition.  (The paper projects
  on the non-uniform set instead; this reading trades one uniform T x nb x K
  product for exact least-squares coefficients.)
"""
from __future__ import annotations

from typing import Callable, Tuple

import numpy as np


def zero_crossings(f: np.ndarray, h_re: np.ndarray) -> np.ndarray:
    """Frequencies where the sampled real part changes sign (linear root
    between the two samples) or is exactly zero at an interior sample."""
    f = np.asarray(f, dtype=np.float64)
    y = np.asarray(h_re, dtype=np.float64)
    out = []
    for i in range(f.shape[0] - 1):
        if y[i] == 0.0 and i > 0:
            out.append(f[i])
        elif y[i] * y[i + 1] < 0.0:
            out.append(f[i] + (f[i + 1] - f[i]) * (y[i] / (y[i] - y[i + 1])))
    return np.asarray(out, dtype=np.float64)


def frequency_set(f: np.ndarray, h_re: np.ndarray, per_bin: int = 5, df_min: float = 1.0 / 128,
                  extra=None) -> np.ndarray:
    """Non-uniform frequencies over [f[0], f[-1]] from the reference
    template's samples (f strictly increasing), merged with the `extra`
    frequencies that fall strictly inside (f[0], f[-1])."""
    f = np.asarray(f, dtype=np.float64)
    lo, hi = float(f[0]), float(f[-1])
    edges = [lo] + [e for e in zero_crossings(f, h_re) if lo < e < hi] + [hi]
    nodes = []
    for a, b in zip(edges[:-1], edges[1:]):
        step = (b - a) / per_bin
        if step >= df_min:
            nodes.extend(a + m * step for m in range(per_bin))
        else:
            k = int(np.ceil(a / df_min))
            while k * df_min < a:
                k += 1
            while k > 0 and (k - 1) * df_min >= a:
                k -= 1
            while k * df_min < b:
                nodes.append(k * df_min)
                k += 1
    nodes.append(hi)
    nodes = np.asarray(nodes, dtype=np.float64)
    if extra is not None:
        ex = np.asarray(extra, dtype=np.float64)
        nodes = np.union1d(nodes, ex[(ex > lo) & (ex < hi)])
    return nodes


def cell_weights(nodes: np.ndarray) -> np.ndarray:
    """omega_i: width of node i's cell between the midpoints to its
    neighbours; the end cells are mirrored (width = the spacing to the one
    neighbour)."""
    x = np.asarray(nodes, dtype=np.float64)
    n = x.shape[0]
    if n == 1:
        return np.ones(1)
    w = np.empty(n)
    w[0] = x[1] - x[0]
    w[-1] = x[-1] - x[-2]
    for i in range(1, n - 1):
        w[i] = 0.5 * (x[i + 1] - x[i - 1])
    return w


def whitened_set_templates(H: np.ndarray, psd_nodes: np.ndarray, nodes: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """(V, sigma): V[j, i] = h_j(f_i) sqrt(4 omega_i / Sn(f_i)) / sigma_j."""
    om = cell_weights(nodes)
    g = np.sqrt(4.0 * om / np.asarray(psd_nodes, dtype=np.float64))
    Hw = np.asarray(H, dtype=np.complex128) * g[None, :]
    sig = np.sqrt(np.sum(np.abs(Hw) ** 2, axis=1))
    return Hw / sig[:, None], sig


def covariance_basis(V: np.ndarray, rank: int = 0, tol: float = 1e-3):
    """Leading eigenvectors of the covariance V^H V (N_t x N_t).  Returns
    (U rows = basis on the set (K x N_t), eigenvalues in descending order, K)."""
    Cov = V.conj().T @ V
    lam, E = np.linalg.eigh(Cov)
    order = np.argsort(lam)[::-1]
    lam, E = lam[order], E[:, order]
    lam = np.clip(lam, 0.0, None)
    if rank > 0:
        K = min(rank, V.shape[0], V.shape[1])
    else:
        cum = np.cumsum(lam) / np.sum(lam)
        K = min(int(np.searchsorted(cum, 1.0 - tol - 1e-15) + 1), V.shape[0])
    # the basis vector v_k with w_j ~ sum_k c_jk v_k: the conjugated eigenvector
    # (V^H V e = lam e  <=>  rows of V have coefficients along conj(e))
    return E[:, :K].T.conj(), lam, K


def interpolate_to_grid(U: np.ndarray, nodes: np.ndarray, f_uniform: np.ndarray, df: float) -> np.ndarray:
    """sqrt(df) * linear interpolation of U_k / sqrt(omega) at f_uniform
    (inside [nodes[0], nodes[-1]])."""
    om = cell_weights(nodes)
    dens = U / np.sqrt(om)[None, :]
    out = np.empty((U.shape[0], f_uniform.shape[0]), dtype=np.complex128)
    for k in range(U.shape[0]):
        out[k] = np.interp(f_uniform, nodes, dens[k].real) + 1j * np.interp(f_uniform, nodes, dens[k].imag)
    return np.sqrt(df) * out


def nonuniform_basis(W: np.ndarray, H_nodes: np.ndarray, psd_nodes: np.ndarray, nodes: np.ndarray,
                     f_uniform: np.ndarray, df: float, rank: int = 0, tol: float = 1e-3):
    """The whole preparation: (Vb (K x nb) orthonormal rows on the uniform
    band, c = W Vb^H (T x K), eigenvalues on the set, K, energy kept on the
    uniform grid sum |c|^2 / sum |W|^2).  W is the uniform whitened unit bank
    (T x nb) the coefficients are taken against."""
    Vs, _ = whitened_set_templates(H_nodes, psd_nodes, nodes)
    U, lam, K = covariance_basis(Vs, rank, tol)
    P = interpolate_to_grid(U, nodes, f_uniform, df)
    Q, _ = np.linalg.qr(P.T)          # columns orthonormal, same span
    Vb = Q.T
    c = W @ Vb.conj().T
    energy = float(np.sum(np.abs(c) ** 2) / np.sum(np.abs(W) ** 2))
    return Vb, c, lam, K, energy


def reference_samples(h_of_f: Callable[[np.ndarray], np.ndarray], f_lo: float, f_hi: float,
                      step: float) -> Tuple[np.ndarray, np.ndarray]:
    """The reference template's real part on [f_lo, f_hi] at spacing `step`
    (the last sample at f_hi exactly)."""
    n = int(np.floor((f_hi - f_lo) / step))
    f = f_lo + step * np.arange(n + 1, dtype=np.float64)
    if f[-1] < f_hi:
        f = np.append(f, f_hi)
    return f, np.real(h_of_f(f))
