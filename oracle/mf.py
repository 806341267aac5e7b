"""FP64 template-method matched filter (test infrastructure only; see package
docstring).

Conventions (readings of the paper where it is silent or garbled):

* Forward transform: s~[k] = dt * sum_n s[n] e^{-2 pi i k n / N} (numpy rfft
  times dt), k = 0..N/2.
* Band: k_lo = ceil(f_low / df) .. N/2 - 1 inclusive; DC and Nyquist are
  excluded.  A template is zero outside its own support (f_ISCO cut).
* Complex filter output (Eq. IFFT, discretised):
      z_j[n] = 4 df sum_{k in band} s~[k] conj(h_j[k]) / Sn[k] e^{+2 pi i k n / N}
  for n = 0..N-1 (the one-sided integrand, negative frequencies zero).
* Normalisation (Eq. SNR_def, with the phase maximised by the modulus as
  Sec. II states): sigma_j^2 = 4 df sum_{k in band} |h_j[k]|^2 / Sn[k],
  rho_j[n] = z_j[n] / sigma_j, SNR = |rho_j[n]|.
* Trigger (Sec. II): a sample with |rho| >= threshold (inclusive).
"""
from __future__ import annotations

import math
import os
from typing import Iterator, Tuple

import numpy as np
import scipy.fft as sfft

# threads of the batched inverse transforms (a host CPU share, not the machine's core count)
WORKERS = max(1, min(16, int(os.environ.get("ORACLE_WORKERS", "0")) or (os.cpu_count() or 1)))


def band_limits(N: int, fs: float, f_low: float) -> Tuple[int, int]:
    """(k_lo, k_hi) inclusive."""
    df = fs / N
    k_lo = int(math.ceil(f_low / df - 1e-9))
    return k_lo, N // 2 - 1


def strain_tilde(s: np.ndarray, fs: float) -> np.ndarray:
    """s~ = dt * rfft(s), complex128 of length N/2+1."""
    return np.fft.rfft(np.asarray(s, dtype=np.float64)) / fs


def band_mask(N: int, fs: float, f_low: float) -> np.ndarray:
    k_lo, k_hi = band_limits(N, fs, f_low)
    m = np.zeros(N // 2 + 1, dtype=bool)
    m[k_lo:k_hi + 1] = True
    return m


def sigma(h: np.ndarray, psd: np.ndarray, N: int, fs: float, f_low: float) -> float:
    """sigma = <h|h>^{1/2} with the noise-weighted inner product (Eq. MF_def)."""
    df = fs / N
    m = band_mask(N, fs, f_low)
    return float(np.sqrt(4.0 * df * np.sum(np.abs(h[m]) ** 2 / psd[m])))


def complex_filter(s_t: np.ndarray, h: np.ndarray, psd: np.ndarray, N: int, fs: float,
                   f_low: float) -> np.ndarray:
    """z[n] = 4 df sum_{band} s~ conj(h)/Sn e^{+2 pi i k n/N}, n = 0..N-1 (Eq. IFFT)."""
    df = fs / N
    m = band_mask(N, fs, f_low)
    X = np.zeros(N, dtype=np.complex128)
    X[: N // 2 + 1][m] = s_t[m] * np.conj(h[m]) / psd[m]
    # numpy's ifft carries 1/N; the sum in Eq. IFFT has none.
    return 4.0 * df * N * np.fft.ifft(X)


def snr_rows(s_t: np.ndarray, H: np.ndarray, psd: np.ndarray, N: int, fs: float, f_low: float,
             workers: int = 0) -> np.ndarray:
    """rho_j[n] = z_j[n] / sigma_j for every row of H (templates on all N/2+1
    bins): the same sums as complex_filter and sigma, one inverse transform
    per row, `workers` threads (0: WORKERS)."""
    df = fs / N
    m = band_mask(N, fs, f_low)
    H = np.asarray(H, dtype=np.complex128)
    X = np.zeros((H.shape[0], N), dtype=np.complex128)
    X[:, : N // 2 + 1][:, m] = s_t[m][None, :] * np.conj(H[:, m]) / psd[m][None, :]
    z = (4.0 * df * N) * sfft.ifft(X, axis=1, workers=workers or WORKERS)
    sig = np.sqrt(4.0 * df * np.sum(np.abs(H[:, m]) ** 2 / psd[m][None, :], axis=1))
    return z / sig[:, None]


def snr_series(s: np.ndarray, h: np.ndarray, psd: np.ndarray, fs: float, f_low: float) -> np.ndarray:
    """Complex SNR time series rho[n] = z[n]/sigma for one template."""
    N = s.shape[0]
    z = complex_filter(strain_tilde(s, fs), h, psd, N, fs, f_low)
    return z / sigma(h, psd, N, fs, f_low)


def snr_bank(s: np.ndarray, bank_fill, T: int, psd: np.ndarray, fs: float, f_low: float,
             chunk: int = 16) -> Iterator[Tuple[int, np.ndarray]]:
    """Yields (j, rho_j) for every template; bank_fill(t0, t1) gives the
    complex128 templates [t0, t1) on all N/2+1 bins."""
    N = s.shape[0]
    s_t = strain_tilde(s, fs)
    for t0 in range(0, T, chunk):
        t1 = min(T, t0 + chunk)
        H = bank_fill(t0, t1)
        for i in range(t1 - t0):
            h = H[i]
            yield t0 + i, complex_filter(s_t, h, psd, N, fs, f_low) / sigma(h, psd, N, fs, f_low)


TRIGGER_DTYPE = np.dtype([("tmpl", np.int32), ("sample", np.int32), ("snr", np.float64),
                          ("phase", np.float64)])


def triggers_of(j: int, rho: np.ndarray, thr: float) -> np.ndarray:
    """All samples of template j with |rho| >= thr, sorted by sample."""
    a = np.abs(rho)
    idx = np.nonzero(a >= thr)[0]
    out = np.empty(idx.shape[0], dtype=TRIGGER_DTYPE)
    out["tmpl"] = j
    out["sample"] = idx
    out["snr"] = a[idx]
    out["phase"] = np.angle(rho[idx])
    return out


def triggers(rho_rows, thr: float) -> np.ndarray:
    """Trigger set over (j, rho_j) pairs, sorted by (tmpl, sample)."""
    parts = [triggers_of(j, r, thr) for j, r in rho_rows]
    if not parts:
        return np.empty(0, dtype=TRIGGER_DTYPE)
    out = np.concatenate(parts)
    return out[np.lexsort((out["sample"], out["tmpl"]))]


def peak(rho: np.ndarray) -> Tuple[float, int]:
    """max_n |rho[n]| and its argmax (ties to the lowest n)."""
    a = np.abs(rho)
    n = int(np.argmax(a))      # numpy returns the first maximum
    return float(a[n]), n


def cluster_peaks(trig: np.ndarray, W: int, N: int) -> np.ndarray:
    """Boolean mask over a (tmpl, sample)-sorted trigger list: a trigger is a
    peak when no trigger of the same template within +-W samples (circular)
    has a larger SNR, or an equal SNR at a lower sample."""
    keep = np.zeros(trig.shape[0], dtype=bool)
    for j in np.unique(trig["tmpl"]):
        sel = np.nonzero(trig["tmpl"] == j)[0]
        n = trig["sample"][sel].astype(np.int64)
        v = trig["snr"][sel]
        for a, i in enumerate(sel):
            d = np.abs(n - n[a])
            d = np.minimum(d, N - d)
            near = d <= W
            better = (v > v[a]) | ((v == v[a]) & (n < n[a]))
            keep[i] = not np.any(near & better)
    return keep
