"""Writes whole-bank oracle trigger lists of the large workloads to
tests/golden/, from the FP64 oracle (oracle/) and the seeded input
generators only.

    python tests/golden/make_oracle_sweeps.py [workload ...]

For each workload the strain is the float32 segment that the GPU tests build
(coloured noise plus the workload's injections, injection amplitudes from the
oracle's sigma); the oracle's complex SNR series of every template (Sec. II,
Eq. IFFT normalised by sigma) is computed chunk by chunk and every sample with
|rho| >= LOW[workload] is kept.  The file's header carries the SHA-1 of the
strain bytes so that a test can check that it regenerated the same input.

  oracle_rb_256s_2000t.txt   256 s, 2000 3.5PN templates: |rho| >= 5.99
                             (the final threshold 6 less its +-1e-3 band)
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

from oracle import mf as om                         # noqa: E402
from paper_2110_13115_amd import inputs as gi       # noqa: E402

LOW = {"rb_256s_2000t": 5.99}
CHUNK = {"rb_256s_2000t": 16}


def path_of(name):
    return os.path.join(HERE, f"oracle_{name}.txt")


def case(name):
    """Workload, bank, PSD, float32 strain and injections as the GPU tests build them."""
    wl = gi.WORKLOADS[name]
    bank = wl.bank()
    psd = gi.psd_on_grid(wl.N, wl.fs)
    sig = lambda h: om.sigma(h, psd, wl.N, wl.fs, wl.f_low)
    strain, inj = gi.make_strain(wl, bank, sig, dtype=np.float32)
    return wl, bank, psd, strain, inj


def strain_sha1(strain):
    return hashlib.sha1(np.ascontiguousarray(strain, dtype=np.float32).tobytes()).hexdigest()


def sweep(wl, bank, psd, strain, low, chunk):
    st = om.strain_tilde(strain.astype(np.float64), wl.fs)
    parts = []
    for t0 in range(0, wl.T, chunk):
        t1 = min(wl.T, t0 + chunk)
        rho = om.snr_rows(st, bank.fill(t0, t1, 0, wl.N // 2 + 1), psd, wl.N, wl.fs, wl.f_low)
        parts.extend(om.triggers_of(t0 + i, rho[i], low) for i in range(t1 - t0))
    out = np.concatenate(parts)
    return out[np.lexsort((out["sample"], out["tmpl"]))]


def read(name):
    """(strain sha1, trigger array) of a stored sweep."""
    sha, rows = None, []
    for ln in open(path_of(name)):
        if ln.startswith("# strain_sha1 "):
            sha = ln.split()[2]
        elif ln.strip() and not ln.startswith("#"):
            rows.append(ln.split())
    out = np.empty(len(rows), dtype=om.TRIGGER_DTYPE)
    for i, (t, n, s, p) in enumerate(rows):
        out[i] = (int(t), int(n), float(s), float(p))
    return sha, out


def main(names):
    for name in names:
        t = time.time()
        wl, bank, psd, strain, inj = case(name)
        trig = sweep(wl, bank, psd, strain, LOW[name], CHUNK[name])
        with open(path_of(name), "w") as f:
            f.write(f"# FP64 oracle (template method, Sec. II Eq. IFFT / sigma) over every template of "
                    f"workload {name}: N={wl.N} fs={wl.fs} f_low={wl.f_low} T={wl.T}\n")
            f.write(f"# every sample with |rho| >= {LOW[name]}; injections "
                    + "; ".join(f"SNR {i.snr} at {i.n0}" for i in inj) + "\n")
            f.write(f"# strain_sha1 {strain_sha1(strain)}\n")
            f.write("# written by tests/golden/make_oracle_sweeps.py\n# tmpl sample snr phase\n")
            for r in trig:
                f.write(f"{r['tmpl']} {r['sample']} {r['snr']:.12g} {r['phase']:.12g}\n")
        print(f"{name}: {len(trig)} triggers -> {path_of(name)} ({time.time() - t:.0f} s)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(LOW))
