"""mf_full_noalloc (the template method on the library's fixed device
scratch, for callers that cannot allocate) through the C ABI, against
mf_full's output: two calls in a row, the second on a smaller input (fewer
samples and templates, so it runs over what the first call left in the
scratch), each equal to mf_full's sorted triggers; and its limits, all forced
from the host (device pointers only, a prepared FFT plan, crossings beyond the
scratch's records, a capacity below the count)."""
import ctypes as C

import numpy as np
import pytest

from paper_2110_13115_amd import rbmf
from tests.helpers import Case, compare_triggers

pytestmark = pytest.mark.gpu


def _status(ctx, bank, strain_ptr, thr, out_ptr, cap):
    n = C.c_int64(-1)
    st = rbmf.lib().mf_full_noalloc(ctx.h, bank.h, strain_ptr, float(thr), out_ptr, cap, C.byref(n))
    return st, n.value


def test_noalloc_matches_mf_full_twice_then_smaller():
    import torch
    ctx = rbmf.Context(0)
    cases = [Case(N=32768, T=96, f_low=30.0, mrange=(5.0, 12.0), order=0, cfg=1, inj=((3, 11.0),)),
             Case(N=8192, T=40, f_low=25.0, mrange=(6.0, 14.0), order=0, cfg=1, inj=((7, 9.0),), seed_shift=3)]
    banks, strains, refs = [], [], []
    for cs in cases:     # mf_full first: the reference output, and it prepares each grid's FFT plan
        bank = rbmf.Bank(ctx, cs.N, cs.fs, cs.f_low, cs.psd, cs.T, cs.fill)
        sd = torch.from_numpy(cs.strain).cuda()
        ref, _, _ = rbmf.mf_full(ctx, bank, sd, 4.0)
        assert len(ref) > 0
        banks.append(bank)
        strains.append(sd)
        refs.append(ref)
    for rep in range(2):
        for cs, bank, sd, ref in zip(cases, banks, strains, refs):
            out = torch.full((1 << 16, 4), -1, dtype=torch.int32, device="cuda")
            n = rbmf.mf_full_noalloc(ctx, bank, sd, 4.0, out)
            got = out[:n].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1)
            assert n == len(ref), (rep, cs.N, n, len(ref))
            assert got.tobytes() == ref.tobytes(), (rep, cs.N)
            assert (out[n:].cpu() == -1).all(), "wrote beyond the trigger count"
            compare_triggers(got, cs.rho, 4.0)
    for b in banks:
        b.close()
    ctx.close()


def test_noalloc_limits():
    import torch
    cs = Case(N=32768, T=96, f_low=30.0, mrange=(5.0, 12.0), order=0, cfg=1, inj=((3, 11.0),))
    ctx = rbmf.Context(0)
    bank = rbmf.Bank(ctx, cs.N, cs.fs, cs.f_low, cs.psd, cs.T, cs.fill)
    sd = torch.from_numpy(cs.strain).cuda()
    out = torch.empty((1 << 12, 4), dtype=torch.int32, device="cuda")
    # no FFT plan for this grid in the context yet
    st, _ = _status(ctx, bank, sd.data_ptr(), 5.0, out.data_ptr(), out.shape[0])
    assert st == rbmf.RB_ERR_ARG and b"FFT plan" in rbmf.lib().rb_last_error()
    ref, _, _ = rbmf.mf_full(ctx, bank, sd, 5.0)
    # host pointers are refused
    st, _ = _status(ctx, bank, cs.strain.ctypes.data, 5.0, out.data_ptr(), out.shape[0])
    assert st == rbmf.RB_ERR_ARG
    host_out = np.empty(16, dtype=rbmf.TRIGGER_NP)
    st, _ = _status(ctx, bank, sd.data_ptr(), 5.0, host_out.ctypes.data, 16)
    assert st == rbmf.RB_ERR_ARG
    # capacity below the count: the count is reported
    st, n = _status(ctx, bank, sd.data_ptr(), 5.0, out.data_ptr(), 1)
    assert st == rbmf.RB_ERR_CAPACITY and n == len(ref)
    # more crossings than the scratch holds (|rho| >= 0.5 on most samples)
    st, n = _status(ctx, bank, sd.data_ptr(), 0.5, out.data_ptr(), out.shape[0])
    assert st == rbmf.RB_ERR_UNSUPPORTED and n > 1_000_000, (st, n)
    assert b"fixed scratch" in rbmf.lib().rb_last_error()
    # and the next call is exact again
    n = rbmf.mf_full_noalloc(ctx, bank, sd, 5.0, out)
    got = out[:n].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1)
    assert got.tobytes() == ref.tobytes()
    bank.close()
    ctx.close()
