"""Seeded synthetic workloads: PSD, template banks, coloured noise, injections.

This module generates *inputs* only.  It holds none of the search's
arithmetic (no whitening, no template normalisation, no matched filter, no
basis): both the HIP library and the FP64 oracle consume what it produces,
and neither is imported here.

Stand-ins for what the paper used but which is not available here:

* PSD: the analytic Advanced-LIGO design fit
  S_h(f) = S0 [x^-4.14 - 5 x^-2 + 111 (1 - x^2 + x^4/2) / (1 + x^2/2)],
  x = f / 215 Hz, S0 = 1e-49 / Hz (Ajith 2011, PRD 84, 084037), standing in
  for the "aLIGO PSD" of Sec. III.B and IV.B.
* Templates: restricted-amplitude, non-spinning TaylorF2 (stationary phase
  approximation) h(f) = f^(-7/6) exp(-i Psi(f)) cut at f_ISCO, with the
  phase coefficients of Buonanno, Iyer, Ochsner, Pan & Sathyaprakash 2009
  (PRD 80, 084043) up to 3.5PN.  Truncated at 0PN it is exactly
  f^(-7/6) exp(-i[2 pi f tc - pi/4 + 3/128 (pi Mc f)^(-5/3)]).  These stand
  in for the O2 bank and IMRPhenomPv2 waveforms of Sec. III.B.
* Noise: stationary coloured Gaussian noise synthesised on the rfft grid
  (Re and Im independent N(0, Sn/(4 df)), DC and Nyquist zero), standing in
  for the PyCBC-simulated noise of Sec. IV.
* Injections: a bank template added in the frequency domain with amplitude A,
  phase phi0 and integer arrival sample n0 (circular), the extrinsic model of
  Eq. (hf_eqn).  The caller chooses A (e.g. target SNR / sigma).

Seeds: ``numpy.random.default_rng([13115, cfg, purpose])`` with purpose
0 = bank, 1 = noise, 2 = injections, 3 = finite-difference directions,
4 = segment lengths.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

MSUN_S = 4.925490947e-6          # G Msun / c^3 in seconds
EULER_GAMMA = 0.5772156649015329

PURPOSE_BANK, PURPOSE_NOISE, PURPOSE_INJ, PURPOSE_FD, PURPOSE_LEN = 0, 1, 2, 3, 4


def rng_for(cfg: int, purpose: int, realisation: int = 0) -> np.random.Generator:
    key = [13115, int(cfg), int(purpose)] + ([int(realisation)] if realisation else [])
    return np.random.default_rng(key)


# --------------------------------------------------------------------------
# PSD
# --------------------------------------------------------------------------
def aligo_psd(f: np.ndarray) -> np.ndarray:
    """Analytic Advanced-LIGO design PSD fit (one-sided, 1/Hz).  f > 0."""
    f = np.asarray(f, dtype=np.float64)
    x = f / 215.0
    with np.errstate(divide="ignore", invalid="ignore"):
        s = 1e-49 * (x ** -4.14 - 5.0 * x ** -2
                     + 111.0 * (1.0 - x ** 2 + 0.5 * x ** 4) / (1.0 + 0.5 * x ** 2))
    return s


def psd_on_grid(N: int, fs: float) -> np.ndarray:
    """PSD at the N/2+1 rfft bin centres.  Bin 0 (DC) gets +inf."""
    f = np.arange(N // 2 + 1, dtype=np.float64) * (fs / N)
    s = np.empty_like(f)
    s[0] = np.inf
    s[1:] = aligo_psd(f[1:])
    return s


# --------------------------------------------------------------------------
# TaylorF2
# --------------------------------------------------------------------------
def f_isco(m1: float, m2: float) -> float:
    M = (m1 + m2) * MSUN_S
    return 1.0 / (6.0 ** 1.5 * np.pi * M)


def tau0(m1: float, m2: float, f0: float) -> float:
    """Leading-order chirp time (s) from frequency f0."""
    M = (m1 + m2) * MSUN_S
    eta = m1 * m2 / (m1 + m2) ** 2
    return 5.0 / (256.0 * np.pi * f0 * eta) * (np.pi * M * f0) ** (-5.0 / 3.0)


def tau0_array(m1: np.ndarray, m2: np.ndarray, f0: float) -> np.ndarray:
    """tau0 of many mass pairs (vectorised form of tau0)."""
    M = (m1 + m2) * MSUN_S
    eta = m1 * m2 / (m1 + m2) ** 2
    return 5.0 / (256.0 * np.pi * f0 * eta) * (np.pi * M * f0) ** (-5.0 / 3.0)


def _pn_phase_series(v: np.ndarray, eta: float, order: int) -> np.ndarray:
    """sum_k phi_k v^k of the TaylorF2 phase, up to PN order `order` (0..7
    in units of half-PN, i.e. order=7 is 3.5PN)."""
    pi = np.pi
    out = np.ones_like(v)
    if order >= 2:
        out += 20.0 / 9.0 * (743.0 / 336.0 + 11.0 / 4.0 * eta) * v ** 2
    if order >= 3:
        out += -16.0 * pi * v ** 3
    if order >= 4:
        out += 10.0 * (3058673.0 / 1016064.0 + 5429.0 / 1008.0 * eta
                       + 617.0 / 144.0 * eta ** 2) * v ** 4
    if order >= 5:
        vlso = 1.0 / np.sqrt(6.0)
        out += pi * (38645.0 / 756.0 - 65.0 / 9.0 * eta) * (1.0 + 3.0 * np.log(v / vlso)) * v ** 5
    if order >= 6:
        c6 = (11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * pi ** 2 - 6848.0 / 21.0 * EULER_GAMMA
              + eta * (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * pi ** 2)
              + 76055.0 / 1728.0 * eta ** 2 - 127825.0 / 1296.0 * eta ** 3)
        out += (c6 - 6848.0 / 21.0 * np.log(4.0 * v)) * v ** 6
    if order >= 7:
        out += pi * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta
                     - 74045.0 / 756.0 * eta ** 2) * v ** 7
    return out


def taylorf2(f: np.ndarray, m1: float, m2: float, order: int = 7,
             f_low: float = 0.0, tc: float = 0.0) -> np.ndarray:
    """Complex128 TaylorF2 h(f) = f^(-7/6) exp(-i Psi(f)), zero outside
    [f_low, f_ISCO].  Masses in solar masses."""
    f = np.asarray(f, dtype=np.float64)
    out = np.zeros(f.shape, dtype=np.complex128)
    fi = f_isco(m1, m2)
    sel = (f > 0) & (f >= f_low) & (f <= fi)
    if not np.any(sel):
        return out
    fv = f[sel]
    M = (m1 + m2) * MSUN_S
    eta = m1 * m2 / (m1 + m2) ** 2
    v = (np.pi * M * fv) ** (1.0 / 3.0)
    psi = 2.0 * np.pi * fv * tc - np.pi / 4.0 + 3.0 / (128.0 * eta * v ** 5) * _pn_phase_series(v, eta, order)
    out[sel] = fv ** (-7.0 / 6.0) * np.exp(-1j * psi)
    return out


class _FreqPowers:
    """Frequency-only factors of the TaylorF2 expression, shared by a chunk."""

    def __init__(self, f: np.ndarray):
        self.f = f
        pos = f > 0
        self.pos = pos
        self.amp = np.zeros_like(f)
        self.amp[pos] = f[pos] ** (-7.0 / 6.0)
        self.f13 = np.zeros_like(f)
        self.f13[pos] = np.cbrt(f[pos])
        self.logf = np.zeros_like(f)
        self.logf[pos] = np.log(f[pos])


def _taylorf2_pre(pre: _FreqPowers, m1: float, m2: float, order: int, f_low: float,
                  out: Optional[np.ndarray] = None) -> np.ndarray:
    """taylorf2() on a precomputed grid (same expression, shared powers of f);
    only the support is written when `out` (zeros) is given."""
    f = pre.f
    if out is None:
        out = np.zeros(f.shape, dtype=np.complex128)
    lo = np.searchsorted(f, max(f_low, 0.0), side="left")
    hi = np.searchsorted(f, f_isco(m1, m2), side="right")
    lo = max(lo, int(np.argmax(pre.pos)) if pre.pos.any() else f.shape[0])
    if hi <= lo:
        return out
    sl = slice(lo, hi)
    M = (m1 + m2) * MSUN_S
    eta = m1 * m2 / (m1 + m2) ** 2
    cM = np.cbrt(np.pi * M)
    v = cM * pre.f13[sl]
    series = _pn_phase_series_pre(v, np.log(cM) + pre.logf[sl] / 3.0, eta, order)
    v2 = v * v
    v5 = v2 * v2 * v
    psi = -np.pi / 4.0 + 3.0 / (128.0 * eta) * series / v5
    out[sl] = pre.amp[sl] * (np.cos(psi) - 1j * np.sin(psi))
    return out


def _pn_phase_series_pre(v: np.ndarray, logv: np.ndarray, eta: float, order: int) -> np.ndarray:
    pi = np.pi
    out = np.ones_like(v)
    if order < 2:
        return out
    v2 = v * v
    out += 20.0 / 9.0 * (743.0 / 336.0 + 11.0 / 4.0 * eta) * v2
    if order >= 3:
        out += -16.0 * pi * v2 * v
    if order >= 4:
        out += 10.0 * (3058673.0 / 1016064.0 + 5429.0 / 1008.0 * eta + 617.0 / 144.0 * eta ** 2) * v2 * v2
    if order >= 5:
        lvlso = np.log(1.0 / np.sqrt(6.0))
        out += pi * (38645.0 / 756.0 - 65.0 / 9.0 * eta) * (1.0 + 3.0 * (logv - lvlso)) * v2 * v2 * v
    if order >= 6:
        c6 = (11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * pi ** 2 - 6848.0 / 21.0 * EULER_GAMMA
              + eta * (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * pi ** 2)
              + 76055.0 / 1728.0 * eta ** 2 - 127825.0 / 1296.0 * eta ** 3)
        out += (c6 - 6848.0 / 21.0 * (np.log(4.0) + logv)) * v2 * v2 * v2
    if order >= 7:
        out += pi * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta
                     - 74045.0 / 756.0 * eta ** 2) * v2 * v2 * v2 * v
    return out


def taylorf2_0pn_closed_form(f: np.ndarray, m1: float, m2: float, f_low: float = 0.0,
                             tc: float = 0.0) -> np.ndarray:
    """The 0PN SPA template written with the chirp mass, as a check of the
    PN truncation: f^-7/6 exp(-i[2 pi f tc - pi/4 + 3/128 (pi Mc f)^(-5/3)])."""
    f = np.asarray(f, dtype=np.float64)
    out = np.zeros(f.shape, dtype=np.complex128)
    sel = (f > 0) & (f >= f_low) & (f <= f_isco(m1, m2))
    mc = (m1 * m2) ** 0.6 / (m1 + m2) ** 0.2 * MSUN_S
    fv = f[sel]
    out[sel] = fv ** (-7.0 / 6.0) * np.exp(
        -1j * (2 * np.pi * fv * tc - np.pi / 4 + 3.0 / 128.0 * (np.pi * mc * fv) ** (-5.0 / 3.0)))
    return out


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
@dataclass
class Bank:
    """A bank of TaylorF2 templates on the rfft grid of (N, fs)."""
    N: int
    fs: float
    f_low: float
    m1: np.ndarray
    m2: np.ndarray
    order: int = 7

    @property
    def T(self) -> int:
        return int(self.m1.shape[0])

    @property
    def df(self) -> float:
        return self.fs / self.N

    def fill(self, t0: int, t1: int, k0: int, k1: int, out: Optional[np.ndarray] = None) -> np.ndarray:
        """Templates [t0, t1) on bins [k0, k1): complex128 (t1-t0, k1-k0),
        written into `out` (zeroed first) when it is given."""
        if out is None:
            out = np.zeros((t1 - t0, k1 - k0), dtype=np.complex128)
        else:
            out[...] = 0
        key = (k0, k1)
        pre = self._pre.get(key) if hasattr(self, "_pre") else None
        if pre is None:     # the frequency powers of the last bin range are kept for the next chunk
            pre = _FreqPowers(np.arange(k0, k1, dtype=np.float64) * self.df)
            self._pre = {key: pre}

        def one(i):
            t = t0 + i
            _taylorf2_pre(pre, float(self.m1[t]), float(self.m2[t]), self.order, self.f_low, out[i])

        n = t1 - t0
        if n >= 8:
            with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
                list(ex.map(one, range(n)))
        else:
            for i in range(n):
                one(i)
        return out

    def fill_at(self, t0: int, t1: int, f: np.ndarray) -> np.ndarray:
        """Templates [t0, t1) at arbitrary frequencies f: complex128 (t1-t0, len(f))."""
        f = np.asarray(f, dtype=np.float64)
        out = np.zeros((t1 - t0, f.shape[0]), dtype=np.complex128)
        pre = _FreqPowers(f)
        for i in range(t1 - t0):
            out[i] = _taylorf2_pre(pre, float(self.m1[t0 + i]), float(self.m2[t0 + i]), self.order, self.f_low)
        return out

    def longest(self) -> int:
        """Index of the template with the largest tau0 at f_low."""
        return int(np.argmax(tau0_array(self.m1, self.m2, self.f_low)))

    def support_ends(self) -> np.ndarray:
        """The grid frequencies on either side of every template's f_ISCO cut."""
        kc = np.floor(np.array([f_isco(a, b) for a, b in zip(self.m1, self.m2)]) / self.df)
        return np.unique(np.concatenate([kc, kc + 1])) * self.df

    def full(self) -> np.ndarray:
        """All templates on all N/2+1 bins (small banks only)."""
        return self.fill(0, self.T, 0, self.N // 2 + 1)

    def subset(self, idx: Sequence[int]) -> "Bank":
        idx = np.asarray(idx)
        return Bank(self.N, self.fs, self.f_low, self.m1[idx], self.m2[idx], self.order)


def random_bank(cfg: int, T: int, N: int, fs: float, f_low: float, mmin: float, mmax: float,
                order: int, sort_tau0: bool = False, parent: int = 0) -> Bank:
    """m1, m2 i.i.d. uniform in [mmin, mmax] (seed purpose 0); optionally
    ordered by tau0 at f_low so that sub-banks are contiguous tau0 slices (the
    split of Sec. III.B).  With parent > T the masses of a `parent`-template
    bank are drawn, ordered by tau0, and the T central ones kept: one tau0
    sub-bank of a dense bank."""
    rng = rng_for(cfg, PURPOSE_BANK)
    if parent > T:
        m = rng.uniform(mmin, mmax, size=(parent, 2))
        t0 = tau0_array(m[:, 0], m[:, 1], f_low)
        m = m[np.argsort(t0, kind="stable")]
        lo = (parent - T) // 2
        m = m[lo:lo + T]
        sort_tau0 = False
    else:
        m = rng.uniform(mmin, mmax, size=(T, 2))
    if sort_tau0:
        t0 = np.array([tau0(a, b, f_low) for a, b in m])
        m = m[np.argsort(t0, kind="stable")]
    return Bank(N, fs, f_low, m[:, 0].copy(), m[:, 1].copy(), order)


def coloured_noise_tilde(psd: np.ndarray, N: int, fs: float, rng: np.random.Generator) -> np.ndarray:
    """Frequency-domain noise on the rfft grid, convention s~ = dt * rfft(s):
    Re, Im ~ N(0, Sn / (4 df)) independently; DC and Nyquist zero."""
    df = fs / N
    nb = N // 2 + 1
    sd = np.zeros(nb)
    sd[1:nb - 1] = np.sqrt(psd[1:nb - 1] / (4.0 * df))
    st = (rng.standard_normal(nb) + 1j * rng.standard_normal(nb)) * sd
    st[0] = 0.0
    st[-1] = 0.0
    return st


def add_injection(s_tilde: np.ndarray, h: np.ndarray, amplitude: float, n0: int, phi0: float,
                  N: int) -> np.ndarray:
    """s~ += A e^{-i phi0} h(f) e^{-2 pi i k n0 / N} (circular arrival at n0)."""
    k = np.arange(s_tilde.shape[0], dtype=np.float64)
    return s_tilde + amplitude * np.exp(-1j * phi0) * h * np.exp(-2j * np.pi * k * (n0 % N) / N)


def strain_from_tilde(s_tilde: np.ndarray, N: int, fs: float) -> np.ndarray:
    """Time series whose dt * rfft equals s_tilde (float64)."""
    return np.fft.irfft(s_tilde * fs, n=N)


@dataclass
class Injection:
    template: int          # index into the bank (or -1 for an off-bank waveform)
    snr: float             # requested optimal SNR
    n0: int
    phi0: float
    m1: float = 0.0
    m2: float = 0.0


def draw_injections(cfg: int, count: int, snrs: Sequence[float], T: int, N: int,
                    on_bank: bool = True, mrange: Tuple[float, float] = (1.0, 3.0),
                    realisation: int = 0) -> List[Injection]:
    rng = rng_for(cfg, PURPOSE_INJ, realisation)
    out = []
    for i in range(count):
        tmpl = int(rng.integers(0, T)) if on_bank else -1
        n0 = int(rng.integers(0, N))
        phi0 = float(rng.uniform(0, 2 * np.pi))
        m1, m2 = (0.0, 0.0) if on_bank else tuple(rng.uniform(*mrange, size=2))
        out.append(Injection(tmpl, float(snrs[i % len(snrs)]), n0, phi0, float(m1), float(m2)))
    return out


# --------------------------------------------------------------------------
# The five workloads (sizes, mass ranges, orders, thresholds)
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    cfg: int
    N: int
    fs: float
    f_low: float
    T: int
    mmin: float
    mmax: float
    order: int
    rank: int = 0              # 0 = by energy tolerance
    tol: float = 1e-3
    thr1: float = 5.0
    thr2: float = 6.0
    inj_snrs: Tuple[float, ...] = ()
    on_bank: bool = True
    subbanks: int = 1              # tau0-ordered sub-banks of about T / subbanks templates, one basis each
    sub_align: int = 1             # inner sub-bank boundaries rounded to multiples of this
    ranks: Tuple[int, ...] = ()    # fixed rank per sub-bank (empty: by energy / `rank`)
    parent: int = 0                # > T: the bank is the central tau0 slice of a parent bank
    bin_w: int = 4                 # binned first stage: samples per bin
    thr_bin_grid: Tuple[float, ...] = (3.0, 3.25, 3.5, 3.75, 4.0)   # rho_I values tried

    @property
    def seconds(self) -> float:
        return self.N / self.fs

    def bank(self) -> Bank:
        return random_bank(self.cfg, self.T, self.N, self.fs, self.f_low, self.mmin, self.mmax,
                           self.order, sort_tau0=self.subbanks > 1, parent=self.parent)

    def bounds(self) -> List[int]:
        """Sub-bank template boundaries [0, ..., T]: the equal split, inner
        boundaries rounded to the nearest multiple of sub_align (ties to the
        even multiple), so that every sub-bank but the last fills whole
        reconstruction tiles when sub_align is the tile height."""
        a = self.sub_align
        b = [a * int(round(i * self.T / self.subbanks / a)) for i in range(self.subbanks)] + [self.T]
        assert all(x < y for x, y in zip(b, b[1:])), b
        return b

    def sub_ranks(self) -> List[int]:
        return list(self.ranks) if self.ranks else [self.rank] * self.subbanks


WORKLOADS = {
    # 64 templates, 0PN, 16 s at 2048 Hz, f_low 30 Hz, one on-bank injection at SNR 10
    "full_mf_16s_64t": Workload("full_mf_16s_64t", 1, 32768, 2048.0, 30.0, 64, 5.0, 20.0, 0,
                                thr1=5.0, thr2=6.0, inj_snrs=(10.0,)),
    # 2000 templates, 3.5PN, 256 s, f_low 20 Hz, 8 off-bank injections; split along tau0
    # into 10 sub-banks of 192 to 224 templates (boundaries on multiples of the 32-template
    # reconstruction tile), each basis keeping >= 0.999 of its energy
    "rb_256s_2000t": Workload("rb_256s_2000t", 2, 524288, 2048.0, 20.0, 2000, 1.0, 3.0, 7,
                              tol=1e-3, thr1=5.0, thr2=6.0,
                              inj_snrs=(5.0, 6.0, 7.0, 8.0, 9.0, 10.0, 11.0, 12.0), on_bank=False,
                              subbanks=10, sub_align=32),
    # 10000 templates, 0PN, 16 s, f_low 30 Hz, m in [1, 20]
    "rb_16s_10000t": Workload("rb_16s_10000t", 3, 32768, 2048.0, 30.0, 10000, 1.0, 20.0, 0,
                              tol=1e-3, thr1=5.0, thr2=6.0, inj_snrs=(10.0,)),
    # one tau0 sub-bank of a dense bank (the regime of the paper's 6250-template sub-bank):
    # the central 6250 of 200000 tau0-ordered templates with m in [1, 3], 128 s, 3.5PN
    "rb_128s_6250t_dense": Workload("rb_128s_6250t_dense", 6, 262144, 2048.0, 20.0, 6250, 1.0, 3.0, 7,
                                    tol=1e-3, thr1=5.0, thr2=6.0, inj_snrs=(8.0, 10.0, 12.0),
                                    parent=200000),
    # 20000 templates, rank 256, 512 s, m in [1, 50]
    "rb_512s_20000t": Workload("rb_512s_20000t", 5, 1048576, 2048.0, 20.0, 20000, 1.0, 50.0, 7,
                               rank=256, thr1=5.0, thr2=6.0,
                               inj_snrs=(8.0, 9.0, 10.0, 11.0, 12.0, 8.5, 9.5, 10.5),
                               on_bank=False),
}


@dataclass
class BatchWorkload:
    """Segments of uneven length, each searched with every sub-bank of a bank
    built on that segment's grid."""
    name: str
    cfg: int
    nseg: int
    durations: Tuple[int, ...]     # seconds, drawn i.i.d. per segment (seed purpose 4)
    fs: float
    f_low: float
    T: int
    mmin: float
    mmax: float
    order: int
    subbanks: int
    ranks: Tuple[int, ...]
    thr1: float = 5.0
    thr2: float = 6.0
    inj_snr: Tuple[float, float] = (6.0, 12.0)
    bin_w: int = 4                 # binned first stage: samples per bin
    thr_bin_grid: Tuple[float, ...] = (3.0, 3.25, 3.5, 3.75, 4.0)   # rho_I values tried

    def segment_lengths(self) -> List[int]:
        rng = rng_for(self.cfg, PURPOSE_LEN)
        return [int(d * self.fs) for d in rng.choice(self.durations, size=self.nseg)]

    def grids(self) -> List[int]:
        return sorted(set(self.segment_lengths()))

    def bank_for(self, N: int) -> Bank:
        """The same (tau0-ordered) masses on the grid of N samples."""
        return random_bank(self.cfg, self.T, N, self.fs, self.f_low, self.mmin, self.mmax, self.order,
                           sort_tau0=True)

    def bounds(self) -> List[int]:
        return [int(round(i * self.T / self.subbanks)) for i in range(self.subbanks + 1)]

    def strain(self, i: int, N: int, bank: Bank, sigma_of) -> np.ndarray:
        rng = np.random.default_rng([13115, self.cfg, PURPOSE_INJ, i])
        inj = [Injection(int(rng.integers(0, bank.T)), float(rng.uniform(*self.inj_snr)), int(rng.integers(0, N)),
                         float(rng.uniform(0, 2 * np.pi)))]
        w = Workload(self.name, self.cfg * 1000 + i, N, self.fs, self.f_low, bank.T, self.mmin, self.mmax,
                     self.order)
        s, _ = make_strain(w, bank, sigma_of, inj, dtype=np.float32)
        return s


BATCH_WORKLOADS = {
    # 64 segments with durations uniform in {64, 128, 256, 512} s, 10000 3.5PN templates with
    # m1, m2 in [1, 50], split along tau0 into 4 sub-banks of 2500 with ranks 64/96/128/192
    "batch_64seg": BatchWorkload("batch_64seg", 4, 64, (64, 128, 256, 512), 2048.0, 20.0, 10000,
                                 1.0, 50.0, 7, 4, (64, 96, 128, 192)),
}


def make_strain(wl: Workload, bank: Bank, sigma_of, injections: Optional[List[Injection]] = None,
                noise: bool = True, dtype=np.float32, realisation: int = 0) -> Tuple[np.ndarray, List[Injection]]:
    """Coloured noise plus injections for workload `wl`.

    `sigma_of(h)` must return the optimal-SNR normalisation of a waveform h on
    the full rfft grid; the caller supplies it (the oracle in tests, the
    library's own FP64 sigma in the benchmark), so that this module stays free
    of the search's arithmetic.  realisation > 0 draws an independent noise
    segment and injection set for the same bank (seeds [13115, cfg,
    purpose, realisation])."""
    N, fs = wl.N, wl.fs
    psd = psd_on_grid(N, fs)
    st = coloured_noise_tilde(psd, N, fs, rng_for(wl.cfg, PURPOSE_NOISE, realisation)) if noise else \
        np.zeros(N // 2 + 1, dtype=np.complex128)
    if injections is None:
        injections = draw_injections(wl.cfg, len(wl.inj_snrs), wl.inj_snrs, bank.T, N, wl.on_bank,
                                     (bank.m1.min(), bank.m1.max()) if bank.T else (1.0, 3.0), realisation)
    f = np.arange(N // 2 + 1, dtype=np.float64) * (fs / N)
    for inj in injections:
        if inj.template >= 0:
            h = bank.fill(inj.template, inj.template + 1, 0, N // 2 + 1)[0]
        else:
            h = taylorf2(f, inj.m1, inj.m2, bank.order, bank.f_low)
        amp = inj.snr / sigma_of(h)
        st = add_injection(st, h, amp, inj.n0, inj.phi0, N)
    return strain_from_tilde(st, N, fs).astype(dtype), injections
