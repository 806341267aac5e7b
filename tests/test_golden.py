"""Stored expected values (tests/golden/, written by make_golden.py from the
FP64 oracle only): the oracle must keep reproducing them (CPU), and the GPU
template method and reduced-basis search must match them (GPU)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_golden as mg  # noqa: E402

BAND = 1e-3


@pytest.fixture(scope="module")
def golden():
    return mg.read_golden()


def test_oracle_reproduces_golden(golden):
    wl, bank, psd, strain, inj = mg.golden_case()
    trig = mg.oracle_triggers(wl, bank, psd, strain)
    assert np.array_equal(trig[["tmpl", "sample"]], golden[["tmpl", "sample"]])
    np.testing.assert_allclose(trig["snr"], golden["snr"], rtol=1e-10)
    # the loudest trigger is the injected template at its arrival sample, SNR near the injected 10
    k = int(np.argmax(golden["snr"]))
    assert golden["tmpl"][k] == inj[0].template and abs(int(golden["sample"][k]) - inj[0].n0) <= 1
    assert 8.0 < golden["snr"][k] < 12.0


def _match(gpu, golden, thr):
    """Same set outside the +-BAND relative band around thr; SNR to 1e-4."""
    key = lambda a: {(int(t), int(n)): float(s) for t, n, s in zip(a["tmpl"], a["sample"], a["snr"])}
    g, o = key(gpu), key(golden)
    for k, s in o.items():
        if s >= thr * (1 + BAND):
            assert k in g, k
            assert abs(g[k] - s) <= 1e-4 * s, (k, g[k], s)
    for k, s in g.items():
        if s >= thr * (1 + BAND):
            assert k in o, k


@pytest.mark.gpu
def test_gpu_matches_golden(golden):
    from paper_2110_13115_amd import rbmf
    wl, bank_def, psd, strain, inj = mg.golden_case()
    ctx = rbmf.Context(0)
    bank = rbmf.Bank(ctx, wl.N, wl.fs, wl.f_low, psd, wl.T, bank_def.fill)
    trig, _, _ = rbmf.mf_full(ctx, bank, strain, mg.THR)
    _match(trig, golden, mg.THR)
    basis = rbmf.Basis(ctx, bank, rank=0, tol=1e-3, dtype="f32")
    for mode in (rbmf.RB_STAGE2_FULL, rbmf.RB_STAGE2_SPARSE, rbmf.RB_STAGE2_AUTO):
        rt, _, _ = rbmf.rb_filter(ctx, basis, bank, strain, 5.0, mg.THR, stage2=mode)
        _match(rt, golden, mg.THR)
    basis.close()
    bank.close()
