"""Shared helpers for the GPU parity tests: small seeded workloads, oracle
trigger sets and the comparison rule.

Comparison rule (a reading of the +-1e-3 band): trigger sets must agree
exactly except for samples whose oracle |rho| lies within a relative 1e-3 of
the threshold; matched triggers must agree in |rho| to 1e-4 relative (FP32
kernels vs the FP64 oracle)."""
from __future__ import annotations

import numpy as np

from oracle import basis as ob
from oracle import mf as om
from paper_2110_13115_amd import inputs as gi

BAND = 1e-3
SNR_RTOL = 1e-4


class Case:
    """A seeded workload small enough for the oracle to hold all of rho."""

    def __init__(self, N=32768, fs=2048.0, f_low=30.0, T=64, mrange=(5.0, 20.0), order=0, cfg=1,
                 inj=((0, 10.0),), noise=True, seed_shift=0):
        self.N, self.fs, self.f_low, self.T = N, fs, f_low, T
        self.wl = gi.Workload("case", cfg, N, fs, f_low, T, mrange[0], mrange[1], order)
        self.bank = self.wl.bank()
        self.psd = gi.psd_on_grid(N, fs)
        self.H = self.bank.full()
        sig = lambda h: om.sigma(h, self.psd, N, fs, f_low)
        rng = np.random.default_rng([13115, cfg, gi.PURPOSE_INJ, seed_shift])
        injs = [gi.Injection(int(j) % T, float(snr), int(rng.integers(0, N)),
                             float(rng.uniform(0, 2 * np.pi))) for j, snr in inj]
        if noise:
            self.wl.cfg = cfg + 1000 * seed_shift
        self.strain, self.injections = gi.make_strain(self.wl, self.bank, sig, injs, noise=noise,
                                                      dtype=np.float32)
        self.s64 = self.strain.astype(np.float64)
        self._rho = None

    def fill(self, t0, t1, k0, k1):
        return self.H[t0:t1, k0:k1]

    @property
    def rho(self) -> np.ndarray:
        """Oracle complex SNR series (T x N), FP64, of the float32 strain."""
        if self._rho is None:
            st = om.strain_tilde(self.s64, self.fs)
            self._rho = np.stack([om.complex_filter(st, self.H[j], self.psd, self.N, self.fs, self.f_low)
                                  / om.sigma(self.H[j], self.psd, self.N, self.fs, self.f_low)
                                  for j in range(self.T)])
        return self._rho

    def whitened(self):
        W, sig = ob.whitened_unit_templates(self.H, self.psd, self.N, self.fs, self.f_low)
        return W, sig


def compare_triggers(got: np.ndarray, rho: np.ndarray, thr: float, templates=None):
    """Asserts the comparison rule; returns (n_oracle, n_got, n_band_excluded)."""
    a = np.abs(rho)
    if templates is not None:
        mask = np.zeros(a.shape[0], dtype=bool)
        mask[list(templates)] = True
        a = np.where(mask[:, None], a, 0.0)
    ora = a >= thr
    band = (a >= thr * (1 - BAND)) & (a <= thr * (1 + BAND))
    G = np.zeros_like(ora)
    G[got["tmpl"], got["sample"]] = True
    assert len(got) == int(G.sum()), "duplicate GPU triggers"
    miss = ora & ~band & ~G
    extra = G & ~band & ~ora
    assert not miss.any(), f"{int(miss.sum())} oracle triggers missing, e.g. {np.argwhere(miss)[:5]}"
    assert not extra.any(), f"{int(extra.sum())} extra GPU triggers, e.g. {np.argwhere(extra)[:5]}"
    ref = a[got["tmpl"], got["sample"]]
    rel = np.abs(got["snr"].astype(np.float64) - ref) / ref
    assert rel.max(initial=0) <= SNR_RTOL, f"max rel |rho| error {rel.max():.3e}"
    ph = np.angle(rho[got["tmpl"], got["sample"]])
    dph = np.angle(np.exp(1j * (got["phase"].astype(np.float64) - ph)))
    assert np.abs(dph).max(initial=0) <= 1e-3
    order = np.lexsort((got["sample"], got["tmpl"]))
    assert np.all(order == np.arange(len(got))), "triggers not sorted by (tmpl, sample)"
    return int(ora.sum()), len(got), int((band & (ora | G)).sum())


def quant(x, dtype):
    """Round-to-nearest-even of float32 values to bf16 / f16 (numpy emulation), as float64."""
    x = np.asarray(x, np.float32)
    if dtype == "f16":
        return x.astype(np.float16).astype(np.float64)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def quantised_coefficients(c, dtype):
    """C = conj(c) as the 16-bit reconstruction stores it (complex128 values):
    complex64, then (FP16) each row scaled by the power of two that puts its
    largest component in [0.5, 1), rounded to the storage type, scale removed."""
    Cc = np.conj(c).astype(np.complex64)
    if dtype == "f16":
        mx = np.maximum(np.abs(Cc.real), np.abs(Cc.imag)).max(axis=1)
        a = 2.0 ** (-np.frexp(mx)[1])
    else:
        a = np.ones(Cc.shape[0])
    Cs = Cc * a[:, None].astype(np.float32)
    return (quant(Cs.real, dtype) + 1j * quant(Cs.imag, dtype)) / a[:, None]
