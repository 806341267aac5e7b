"""GPU parity of the overlap-save search of a long strain (rb_filter_stream)
against the oracle's segmentation (oracle/stream.py) with the FP64 template
method on every segment, through the C ABI."""
import sys

import numpy as np
import pytest

from oracle import mf as om
from oracle import stream as osm
from paper_2110_13115_amd import inputs as gi
from paper_2110_13115_amd import rbmf
from tests.helpers import BAND, SNR_RTOL

pytestmark = pytest.mark.gpu

N, FS, FLOW, T = 16384, 2048.0, 30.0, 40


def log(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def stream_case():
    n = 2 * N + N // 2 + 1000                      # five segments, the last one moved back
    wl_long = gi.Workload("stream", 31, n, FS, FLOW, T, 8.0, 20.0, 7, thr1=5.0, thr2=6.0)
    bank_long = wl_long.bank()
    psd_long = gi.psd_on_grid(n, FS)
    # A stream is high-passed before it is cut into segments (cutting raw noise
    # would leak its seismic-wall power into the band at every segment edge):
    # the noise is synthesised with no power below 20 Hz.
    f = np.arange(n // 2 + 1) * (FS / n)
    psd_hp = np.where(f >= 20.0, psd_long, 0.0)
    psd_hp[0] = 0.0
    st = gi.coloured_noise_tilde(psd_hp, n, FS, gi.rng_for(31, gi.PURPOSE_NOISE))
    for j, snr, n0, phi in ((3, 12.0, 4500, 0.4), (17, 9.0, N - 100, 2.0), (25, 10.0, 2 * N + 900, -1.0),
                            (39, 8.0, n - 300, 0.0)):
        h = bank_long.fill(j, j + 1, 0, n // 2 + 1)[0]
        st = gi.add_injection(st, h, snr / om.sigma(h, psd_long, n, FS, FLOW), n0, phi, n)
    strain = gi.strain_from_tilde(st, n, FS).astype(np.float32)
    wl_seg = gi.Workload("stream_seg", 31, N, FS, FLOW, T, 8.0, 20.0, 7)
    bank_seg = wl_seg.bank()                        # the same masses on the segment grid
    psd = gi.psd_on_grid(N, FS)
    H = bank_seg.full()
    sigs = [om.sigma(h, psd, N, FS, FLOW) for h in H]

    def search(seg):
        st = om.strain_tilde(seg.astype(np.float64), FS)
        rows = [(j, om.complex_filter(st, H[j], psd, N, FS, FLOW) / sigs[j]) for j in range(T)]
        return om.triggers(rows, 6.0 * (1 - BAND))
    ref = osm.stream_triggers(strain.astype(np.float64), N, search)
    return n, strain, psd, bank_seg, ref


def test_stream_matches_oracle_segmentation(stream_case):
    n, strain, psd, bank_seg, ref = stream_case
    ctx = rbmf.Context(0)
    bank = rbmf.Bank(ctx, N, FS, FLOW, psd, T, bank_seg.fill)
    basis = rbmf.Basis(ctx, bank, rank=0, tol=1e-3, dtype="f32")
    got, st = rbmf.rb_filter_stream(ctx, basis, bank, strain, 5.0, 6.0, stage2=rbmf.RB_STAGE2_SPARSE)
    definite = ref[ref["snr"] >= 6.0 * (1 + BAND)]
    amb = {(int(a), int(b)) for a, b, s in zip(ref["tmpl"], ref["sample"], ref["snr"]) if s < 6.0 * (1 + BAND)}
    G = {(int(a), int(b)): float(s) for a, b, s in zip(got["tmpl"], got["sample"], got["snr"])}
    log("stream: gpu", len(got), "oracle", len(definite), "ambiguous", len(amb), "segments stats", st.n_refiltered)
    assert len(definite) > 20
    assert len(G) == len(got), "duplicate triggers"
    for a, b, s in zip(definite["tmpl"], definite["sample"], definite["snr"]):
        assert (int(a), int(b)) in G, (a, b)
        assert abs(G[(int(a), int(b))] - s) <= SNR_RTOL * s
    refset = {(int(a), int(b)) for a, b in zip(ref["tmpl"], ref["sample"])}
    assert all(k in refset or k in amb for k in G)
    # the same order as the oracle's: by segment, then (tmpl, sample) inside one
    assert np.all((got["sample"] >= 0) & (got["sample"] < n))
    dset = {(int(a), int(b)) for a, b in zip(definite["tmpl"], definite["sample"])}
    gk = [(int(a), int(b)) for a, b in zip(got["tmpl"], got["sample"]) if (int(a), int(b)) in dset]
    assert gk == [(int(a), int(b)) for a, b in zip(definite["tmpl"], definite["sample"])]
    # the injections are found at their own template and stream sample
    for j, n0 in ((3, 4500), (17, N - 100), (25, 2 * N + 900), (39, n - 300)):
        assert (j, n0) in G, (j, n0)
    # a device strain gives the same list; a strain shorter than N is an error
    import torch
    got_d, _ = rbmf.rb_filter_stream(ctx, basis, bank, torch.from_numpy(strain).cuda(), 5.0, 6.0,
                                     stage2=rbmf.RB_STAGE2_SPARSE)
    assert got_d.tobytes() == got.tobytes()
    with pytest.raises(rbmf.RbError) as ei:
        rbmf.rb_filter_stream(ctx, basis, bank, strain[:N - 1], 5.0, 6.0)
    assert ei.value.status == rbmf.RB_ERR_ARG
    with pytest.raises(rbmf.RbError) as ei:
        rbmf.rb_filter_stream(ctx, basis, bank, strain, 5.0, 6.0, cap=3)
    assert ei.value.status == rbmf.RB_ERR_CAPACITY
    basis.close()
    bank.close()
