"""CPU checks of rb_nonuniform_freqs (host only, through the C ABI) against
the oracle's frequency set, and its argument handling."""
import ctypes as C

import numpy as np
import pytest

from oracle import nonuniform as onu
from paper_2110_13115_amd import inputs as gi
from paper_2110_13115_amd import rbmf


def both(f, h, per_bin, df_min, extra=None):
    return rbmf.nonuniform_freqs(f, h, per_bin, df_min, extra), onu.frequency_set(f, h, per_bin, df_min, extra)


@pytest.mark.parametrize("per_bin,df_min", [(5, 1.0 / 16), (3, 0.01), (1, 0.5), (8, 1e-4)])
def test_chirp_set_equals_oracle(per_bin, df_min):
    f = np.linspace(20.0, 200.0, 400001)
    got, ref = both(f, np.cos(2 * np.pi * 300.0 / f), per_bin, df_min)
    assert got.tolist() == ref.tolist()


def test_tone_and_exact_zeros():
    f = np.arange(0, 101, dtype=np.float64) * 0.5
    h = np.cos(np.pi * f)       # exact zeros only where the cosine rounds to 0
    h[[10, 11, 40]] = 0.0
    got, ref = both(f, h, 5, 0.01)
    assert got.tolist() == ref.tolist()


def test_taylorf2_reference_with_support_ends():
    wl = gi.Workload("nu_host", 77, 1 << 16, 2048.0, 20.0, 40, 1.0, 3.0, 7)
    bank = wl.bank()
    k_lo, k_hi = int(np.ceil(wl.f_low / bank.df - 1e-9)), wl.N // 2 - 1
    j = bank.longest()
    fr, yr = onu.reference_samples(lambda x: bank.fill_at(j, j + 1, x)[0], k_lo * bank.df, k_hi * bank.df,
                                   bank.df / 8)
    for df_min in (bank.df, 1.0 / 128):
        got, ref = both(fr, yr, 5, df_min, bank.support_ends())
        assert got.tolist() == ref.tolist()
        assert np.all(np.diff(got) > 0) and got[0] == fr[0] and got[-1] == fr[-1]
    # the dense part with df_min = df is the grid itself: every node below the
    # first sparse bin is a multiple of df
    got = rbmf.nonuniform_freqs(fr, yr, 5, bank.df)
    k = got / bank.df
    assert np.all(k[:50] == np.round(k[:50]))


def test_capacity_and_errors():
    f = np.linspace(30.0, 40.0, 1001)
    h = np.cos(2 * np.pi * f)
    L = rbmf.lib()
    n = C.c_int64()
    fp, hp = f.ctypes.data, h.ctypes.data
    assert L.rb_nonuniform_freqs(fp, hp, f.shape[0], 5, 0.01, None, 0, None, 0, C.byref(n)) == rbmf.RB_ERR_CAPACITY
    ref = onu.frequency_set(f, h, 5, 0.01)
    assert n.value == ref.shape[0]
    out = np.zeros(n.value - 1)
    assert L.rb_nonuniform_freqs(fp, hp, f.shape[0], 5, 0.01, None, 0, out.ctypes.data, out.shape[0],
                                 C.byref(n)) == rbmf.RB_ERR_CAPACITY
    out = np.zeros(n.value)
    assert L.rb_nonuniform_freqs(fp, hp, f.shape[0], 5, 0.01, None, 0, out.ctypes.data, out.shape[0],
                                 C.byref(n)) == rbmf.RB_OK
    assert out.tolist() == ref.tolist()
    bad = [
        (fp, hp, 1, 5, 0.01),                 # one sample
        (fp, hp, f.shape[0], 0, 0.01),        # per_bin
        (fp, hp, f.shape[0], 2000, 0.01),
        (fp, hp, f.shape[0], 5, 0.0),         # df_min
        (fp, hp, f.shape[0], 5, float("nan")),
    ]
    for a in bad:
        assert L.rb_nonuniform_freqs(*a, None, 0, None, 0, C.byref(n)) == rbmf.RB_ERR_ARG
    fd = f.copy()
    fd[5] = fd[4]
    assert L.rb_nonuniform_freqs(fd.ctypes.data, hp, f.shape[0], 5, 0.01, None, 0, None, 0,
                                 C.byref(n)) == rbmf.RB_ERR_ARG
    hn = h.copy()
    hn[3] = np.inf
    assert L.rb_nonuniform_freqs(fp, hn.ctypes.data, f.shape[0], 5, 0.01, None, 0, None, 0,
                                 C.byref(n)) == rbmf.RB_ERR_ARG
    assert L.rb_nonuniform_freqs(fp, hp, f.shape[0], 5, 0.01, None, 3, None, 0, C.byref(n)) == rbmf.RB_ERR_ARG
    assert L.rb_nonuniform_freqs(fp, hp, f.shape[0], 5, 0.01, None, 0, None, 0, None) == rbmf.RB_ERR_ARG
    with pytest.raises(rbmf.RbError):
        rbmf.nonuniform_freqs(f[::-1].copy(), h, 5, 0.01)
