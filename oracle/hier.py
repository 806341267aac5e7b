"""FP64 binned (hierarchical) first stage, fine reconstruction and second
stage (test infrastructure only; see package docstring).

Readings:

* Bins (Sec. III.C, the equation defining beta^avg): fixed, non-overlapping
  bins of w consecutive samples; bin i holds samples i*w .. i*w + w - 1 for
  i = 0 .. N/w - 1 (w divides N).  The averaged basis output is the plain
  mean of the complex beta_k over the bin.
* The averaged SNR series of a template is the same linear combination of
  the averaged outputs as Eq. Beta_eqn, rho_avg_j[i] = sum_k conj(c_jk)
  beta_avg_k[i]; a bin triggers when |rho_avg_j[i]| >= rho_I (inclusive).
* Fine reconstruction (Sec. III.C): every sample of every triggering bin is
  reconstructed with Eq. Beta_eqn.  The samples whose |rho_RB| reaches the
  candidate threshold thr1 are passed on; with w = 1 every sample is its own
  bin and the candidates are the plain first-stage crossings.
* Second stage, three variants (the paper's own is "recon"):
    recon   final triggers are the candidates with |rho_RB| >= thr2, with the
            reconstructed SNR;
    sparse  the exact (template-method) SNR at every candidate sample, final
            where it reaches thr2;
    full    the exact SNR at every sample of every template with a candidate,
            final where it reaches thr2.
* Equivalence with the template method (Sec. III.D, Eqs. avg_fft1,
  double-sum, avg_fft2): the bin mean of a template's complex filter output
  equals an N/w-point inverse transform of the folded spectrum
      Omega(f') = (1/w) sum_{l<w} X[l N/w + f'] G[l N/w + f'],
      G[f] = sum_{r<w} e^{+2 pi i f r / N}   (closed form: a geometric sum),
  where X is the one-sided integrand on all N bins, in the normalisation of
  basis.basis_outputs (no 1/N).  The paper's prefactor 4 w df / N times its
  1/w^2 is the same 1/w once its 4 df / N is folded into X.
* Target SNR (Eq. target_snr_criteria): the smallest rho_II on a grid at
  which the hierarchical search keeps at least a fraction `ratio` of the
  flat search's triggers above rho_II.
"""
from __future__ import annotations

import numpy as np

from . import mf

BIN_DTYPE = np.dtype([("tmpl", np.int32), ("bin", np.int32), ("snr", np.float64)])


def bin_means(x: np.ndarray, w: int) -> np.ndarray:
    """Mean of the last axis over bins of w consecutive samples."""
    N = x.shape[-1]
    if w < 1 or N % w:
        raise ValueError("w must divide N")
    out = np.zeros(x.shape[:-1] + (N // w,), dtype=np.result_type(x, np.complex128))
    for r in range(w):
        out += x[..., r::w]
    return out / w


def averaged_snr(beta: np.ndarray, c: np.ndarray, w: int) -> np.ndarray:
    """rho_avg = conj(c) @ beta_avg: T x N/w."""
    return np.conj(c) @ bin_means(beta, w)


def triggering_bins(rho_avg: np.ndarray, thr_bin: float, t0: int = 0) -> np.ndarray:
    """(tmpl, bin, |rho_avg|) of every bin with |rho_avg| >= thr_bin, sorted."""
    a = np.abs(rho_avg)
    j, i = np.nonzero(a >= thr_bin)
    out = np.empty(j.shape[0], dtype=BIN_DTYPE)
    out["tmpl"] = j + t0
    out["bin"] = i
    out["snr"] = a[j, i]
    return out[np.lexsort((out["bin"], out["tmpl"]))]


def fine_candidates(beta: np.ndarray, c: np.ndarray, bins: np.ndarray, w: int, thr1: float,
                    t0: int = 0) -> np.ndarray:
    """Every sample of every triggering bin, reconstructed with Eq. Beta_eqn
    (one template row at a time), kept when |rho_RB| >= thr1.  Sorted by
    (tmpl, sample); snr and phase are those of rho_RB."""
    parts = []
    for b in bins:
        j = int(b["tmpl"]) - t0
        n = np.arange(int(b["bin"]) * w, int(b["bin"]) * w + w)
        rho = np.conj(c[j]) @ beta[:, n]
        a = np.abs(rho)
        keep = a >= thr1
        t = np.empty(int(keep.sum()), dtype=mf.TRIGGER_DTYPE)
        t["tmpl"] = j + t0
        t["sample"] = n[keep]
        t["snr"] = a[keep]
        t["phase"] = np.angle(rho[keep])
        parts.append(t)
    if not parts:
        return np.empty(0, dtype=mf.TRIGGER_DTYPE)
    out = np.concatenate(parts)
    return out[np.lexsort((out["sample"], out["tmpl"]))]


def second_stage(cand: np.ndarray, thr2: float, mode: str, rho_exact=None) -> np.ndarray:
    """Final triggers from the candidates.  rho_exact(j) -> the template
    method's complex SNR series of template j (needed by "sparse" and
    "full")."""
    if mode == "recon":
        return cand[cand["snr"] >= thr2]
    parts = []
    for j in np.unique(cand["tmpl"]):
        rho = rho_exact(int(j))
        if mode == "full":
            parts.append(mf.triggers_of(int(j), rho, thr2))
        elif mode == "sparse":
            n = cand["sample"][cand["tmpl"] == j]
            a = np.abs(rho[n])
            keep = a >= thr2
            t = np.empty(int(keep.sum()), dtype=mf.TRIGGER_DTYPE)
            t["tmpl"] = j
            t["sample"] = n[keep]
            t["snr"] = a[keep]
            t["phase"] = np.angle(rho[n[keep]])
            parts.append(t)
        else:
            raise ValueError(mode)
    if not parts:
        return np.empty(0, dtype=mf.TRIGGER_DTYPE)
    out = np.concatenate(parts)
    return out[np.lexsort((out["sample"], out["tmpl"]))]


def hierarchical_search(beta: np.ndarray, c: np.ndarray, w: int, thr_bin: float, thr1: float,
                        thr2: float, mode: str = "recon", rho_exact=None, t0: int = 0):
    """The binned first stage, the fine reconstruction and a second stage:
    returns (bins, candidates, final)."""
    bins = triggering_bins(averaged_snr(beta, c, w), thr_bin, t0)
    cand = fine_candidates(beta, c, bins, w, thr1, t0)
    return bins, cand, second_stage(cand, thr2, mode, rho_exact)


def geometric_kernel(N: int, w: int) -> np.ndarray:
    """G[f] = sum_{r<w} e^{+2 pi i f r/N} for f = 0..N-1, in closed form
    (1 - z^w)/(1 - z) with z = e^{2 pi i f/N}, and w where z = 1."""
    f = np.arange(N)
    z = np.exp(2j * np.pi * f / N)
    G = np.empty(N, dtype=np.complex128)
    one = f == 0
    G[one] = w
    G[~one] = (1.0 - z[~one] ** w) / (1.0 - z[~one])
    return G


def folded_average(X: np.ndarray, w: int) -> np.ndarray:
    """The bin means of sum_f X[f] e^{+2 pi i f n/N} through the fold of
    Eq. avg_fft2: Omega on N/w bins, then an N/w-point inverse transform."""
    N = X.shape[-1]
    M = N // w
    G = geometric_kernel(N, w)
    Om = np.zeros(X.shape[:-1] + (M,), dtype=np.complex128)
    for l in range(w):
        Om += X[..., l * M:(l + 1) * M] * G[l * M:(l + 1) * M]
    Om /= w
    return M * np.fft.ifft(Om, axis=-1)


def target_snr(final_snr: np.ndarray, flat_snr: np.ndarray, grid: np.ndarray, ratio: float = 0.99) -> float:
    """Eq. target_snr_criteria: min rho_II on `grid` with
    n_final(rho_II) >= ratio * n_flat(rho_II); inf if none qualifies."""
    for r in np.sort(grid):
        if np.count_nonzero(final_snr >= r) >= ratio * np.count_nonzero(flat_snr >= r):
            return float(r)
    return float("inf")
