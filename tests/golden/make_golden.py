"""Writes the stored expected values of tests/golden/ from the FP64 oracle
(oracle/) and the seeded input generators only.

    python tests/golden/make_golden.py

mf_16s_64t_thr6.txt: the template-method trigger set (Sec. II: the complex
matched-filter output of Eq. IFFT normalised by the template's sigma, every
sample with |rho| >= 6) of the 16 s / 64-template 0PN workload (seeded bank,
coloured noise, one on-bank injection at SNR 10), computed in FP64 from the
float32 strain that the GPU tests also use."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

from oracle import mf as om                         # noqa: E402
from paper_2110_13115_amd import inputs as gi       # noqa: E402

THR = 6.0
FILE = os.path.join(HERE, "mf_16s_64t_thr6.txt")


def golden_case():
    """Bank, PSD and float32 strain of the 16 s / 64-template workload."""
    wl = gi.WORKLOADS["full_mf_16s_64t"]
    bank = wl.bank()
    psd = gi.psd_on_grid(wl.N, wl.fs)
    sig = lambda h: om.sigma(h, psd, wl.N, wl.fs, wl.f_low)
    strain, inj = gi.make_strain(wl, bank, sig, dtype=np.float32)
    return wl, bank, psd, strain, inj


def oracle_triggers(wl, bank, psd, strain):
    H = bank.full()
    st = om.strain_tilde(strain.astype(np.float64), wl.fs)
    rows = ((j, om.complex_filter(st, H[j], psd, wl.N, wl.fs, wl.f_low) / om.sigma(H[j], psd, wl.N, wl.fs, wl.f_low))
            for j in range(wl.T))
    return om.triggers(rows, THR)


def read_golden(path=FILE):
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    out = np.empty(len(rows), dtype=om.TRIGGER_DTYPE)
    for i, (t, n, s, p) in enumerate(rows):
        out[i] = (int(t), int(n), float(s), float(p))
    return out


def main():
    wl, bank, psd, strain, inj = golden_case()
    trig = oracle_triggers(wl, bank, psd, strain)
    with open(FILE, "w") as f:
        f.write("# template-method triggers |rho| >= 6 (Sec. II, Eq. IFFT), FP64 oracle\n")
        f.write(f"# workload full_mf_16s_64t: N={wl.N} fs={wl.fs} f_low={wl.f_low} T={wl.T} 0PN TaylorF2, "
                f"injection {inj[0].template} at SNR {inj[0].snr} sample {inj[0].n0}\n")
        f.write("# written by tests/golden/make_golden.py\n# tmpl sample snr phase\n")
        for r in trig:
            f.write(f"{r['tmpl']} {r['sample']} {r['snr']:.12g} {r['phase']:.12g}\n")
    print(f"{len(trig)} triggers -> {FILE}")


if __name__ == "__main__":
    main()
