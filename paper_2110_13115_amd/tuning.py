"""Choice of the binned first stage's threshold rho_I (Sec. IV.B).

For a bin width w, the hierarchical search keeps fewer of the flat
(template-method) search's triggers as rho_I rises.  The paper's target SNR
(Eq. target_snr_criteria) is the smallest final threshold rho_II at which the
hierarchical search still keeps a fraction `ratio` (0.99) of the flat
search's triggers above rho_II; a choice of (w, rho_I) serves a search at
rho_II when its target SNR is at most rho_II.  The cheapest such rho_I is the
largest one.

Everything here is host-side counting around library calls (mf_full and
rb_filter); it is meant to run on a noise segment other than the one searched.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import rbmf


def target_snr(final_snr, flat_snr, grid: Sequence[float], ratio: float = 0.99) -> float:
    """Smallest rho_II of `grid` with n_final(rho_II) >= ratio * n_flat(rho_II),
    where n(r) counts SNRs >= r; inf when no grid value qualifies."""
    fin = np.sort(np.asarray(final_snr, dtype=np.float64))
    flat = np.sort(np.asarray(flat_snr, dtype=np.float64))
    for r in np.sort(np.asarray(grid, dtype=np.float64)):
        n_fin = fin.shape[0] - np.searchsorted(fin, r, side="left")
        n_flat = flat.shape[0] - np.searchsorted(flat, r, side="left")
        if n_fin >= ratio * n_flat:
            return float(r)
    return float("inf")


def tune_bin_threshold(ctx, bases, bank, strain, w: int, thr1: float, thr2: float,
                       candidates: Sequence[float], ratio: float = 0.99,
                       stage2: int = rbmf.RB_STAGE2_RECON, cap: int = 1 << 22) -> Tuple[float, List[Dict]]:
    """Target SNR of every candidate rho_I on one segment.

    The flat search is mf_full at thr1; the hierarchical one is rb_filter with
    bin width w, threshold rho_I on the averaged series and candidates (and
    final triggers) at thr1, so that both trigger lists reach down to thr1.
    The target SNR is taken on the grid thr1, thr1 + 0.05, ..., thr2 + 1.
    Returns (the largest rho_I whose target SNR is <= thr2, or the smallest
    candidate when none is; one row per candidate)."""
    flat, _, _ = rbmf.mf_full(ctx, bank, strain, thr1, cap=cap)
    flat_hi = {(int(a), int(b)) for a, b, s in zip(flat["tmpl"], flat["sample"], flat["snr"]) if s >= thr2}
    grid = np.arange(thr1, thr2 + 1.0 + 1e-9, 0.05)
    rows = []
    for tb in sorted(candidates):
        fin, _, st = rbmf.rb_filter(ctx, bases, bank, strain, thr1, thr1, stage2=stage2, bin_w=w, thr_bin=tb,
                                    cap=cap)
        kept = sum(1 for a, b in zip(fin["tmpl"], fin["sample"]) if (int(a), int(b)) in flat_hi)
        rows.append({"thr_bin": float(tb), "target_snr": target_snr(fin["snr"], flat["snr"], grid, ratio),
                     "bins": int(st.n_bins), "candidates": int(st.n_stage1),
                     "kept_at_thr2": kept / max(1, len(flat_hi))})
    ok = [r["thr_bin"] for r in rows if r["target_snr"] <= thr2]
    return (max(ok) if ok else float(min(candidates))), rows
