"""Edge cases of the HIP path against the FP64 oracle: the smallest and the
largest supported grids, a one-template bank, a full-rank basis (where the
reduced-basis reconstruction is the template method itself), duplicated
templates (a rank-deficient bank), one-template sub-banks, thresholds that no
sample reaches, and an all-zero segment."""
import sys

import numpy as np
import pytest

from oracle import mf as om
from paper_2110_13115_amd import rbmf
from tests.helpers import Case, compare_triggers

pytestmark = pytest.mark.gpu


def log(*a):
    print("[gpu-edge]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    yield rbmf.Context(0)


def bank_of(ctx, case, fill=None, T=None):
    return rbmf.Bank(ctx, case.N, case.fs, case.f_low, case.psd, T or case.T, fill or case.fill)


@pytest.mark.parametrize("N,T,mr", [(4096, 5, (4.0, 12.0)), (1 << 21, 3, (2.0, 4.0))])
def test_grid_limits(ctx, N, T, mr):
    """2^12 and 2^21 samples: template method and a full-rank basis vs the oracle."""
    log("grid", N, T)
    case = Case(N=N, T=T, f_low=25.0 if N == 4096 else 20.0, mrange=mr, order=7, cfg=21, inj=((0, 11.0),))
    bank = bank_of(ctx, case)
    trig, _, _ = rbmf.mf_full(ctx, bank, case.strain, 5.0)
    compare_triggers(trig, case.rho, 5.0)
    basis = rbmf.Basis(ctx, bank, rank=T, dtype="f32")          # K = T: exact reconstruction
    assert basis.K == T
    for mode in (rbmf.RB_STAGE2_FULL, rbmf.RB_STAGE2_SPARSE):
        rt, _, st = rbmf.rb_filter(ctx, basis, bank, case.strain, 5.0, 5.0, stage2=mode)
        compare_triggers(rt, case.rho, 5.0)
    log("  triggers", len(trig), "stage1", st.n_stage1)
    basis.close()
    bank.close()


def test_single_template_and_full_rank(ctx):
    """T = 1 (K = 1) and a 9-template bank at K = T: the first-stage SNR equals the
    template method's to FP32 rounding at every sample."""
    case = Case(N=16384, T=9, f_low=25.0, mrange=(3.0, 10.0), order=7, cfg=22, inj=((2, 9.0),))
    one = bank_of(ctx, case, fill=lambda t0, t1, k0, k1: case.H[2:3, k0:k1], T=1)
    b1 = rbmf.Basis(ctx, one, rank=0, tol=1e-3, dtype="f32")
    assert b1.K == 1
    r1 = rbmf.debug_rho(ctx, one, case.strain, b1)
    np.testing.assert_allclose(np.abs(r1[0]), np.abs(case.rho[2]), rtol=0, atol=2e-5 * np.abs(case.rho[2]).max())
    b1.close()
    one.close()
    bank = bank_of(ctx, case)
    full = rbmf.Basis(ctx, bank, rank=case.T, dtype="f32")
    rho = rbmf.debug_rho(ctx, bank, case.strain, full)
    err = np.abs(rho - case.rho) / np.maximum(np.abs(case.rho), 1.0)
    log("  full-rank reconstruction err", err.max())
    assert err.max() <= 1e-4
    full.close()
    bank.close()


def test_duplicate_templates_rank_deficient(ctx):
    """Each template stored twice: the basis keeps the rank of the distinct
    set, and both copies of every template report the same triggers."""
    case = Case(N=8192, T=12, f_low=25.0, mrange=(3.0, 10.0), order=7, cfg=23, inj=((4, 10.0),))
    H2 = np.repeat(case.H, 2, axis=0)
    bank = bank_of(ctx, case, fill=lambda t0, t1, k0, k1: H2[t0:t1, k0:k1], T=2 * case.T)
    basis = rbmf.Basis(ctx, bank, rank=0, tol=1e-6, dtype="f32")
    bank1 = bank_of(ctx, case)
    distinct = rbmf.Basis(ctx, bank1, rank=0, tol=1e-6, dtype="f32")
    log("  K duplicated", basis.K, "K distinct", distinct.K)
    assert abs(basis.K - distinct.K) <= 1 and basis.K <= case.T   # same energy fractions (up to rounding)
    trig, _, _ = rbmf.rb_filter(ctx, basis, bank, case.strain, 5.0, 6.0, stage2=rbmf.RB_STAGE2_SPARSE)
    rho2 = np.repeat(case.rho, 2, axis=0)
    compare_triggers(trig, rho2, 6.0)
    ev, od = trig[trig["tmpl"] % 2 == 0], trig[trig["tmpl"] % 2 == 1]
    assert np.array_equal(ev["tmpl"] // 2, od["tmpl"] // 2) and np.array_equal(ev["sample"], od["sample"])
    basis.close()
    distinct.close()
    bank1.close()
    bank.close()


def test_one_template_subbanks_and_empty_results(ctx):
    """A partition whose last sub-bank holds one template; thresholds no sample
    reaches (no triggers, peaks still reported); an all-zero segment."""
    case = Case(N=8192, T=10, f_low=25.0, mrange=(3.0, 10.0), order=7, cfg=24, inj=((9, 10.0),))
    bank = bank_of(ctx, case)
    bases = rbmf.subbank_bases(ctx, bank, [0, 6, 9, 10], rank=[0, 0, 0], tol=1e-3, dtype="f32")
    assert bases[2].K == 1
    trig, _, _ = rbmf.rb_filter(ctx, bases, bank, case.strain, 5.0, 6.0)
    compare_triggers(trig, case.rho, 6.0)
    for mode in (rbmf.RB_STAGE2_FULL, rbmf.RB_STAGE2_SPARSE, rbmf.RB_STAGE2_AUTO):
        t, pk, st = rbmf.rb_filter(ctx, bases, bank, case.strain, 500.0, 600.0, stage2=mode, peaks=True)
        assert len(t) == 0 and st.n_stage1 == 0 and st.n_refiltered == 0
    t, pk, _ = rbmf.mf_full(ctx, bank, case.strain, 600.0, peaks=True)
    assert len(t) == 0
    ref = np.abs(case.rho).max(axis=1)
    np.testing.assert_allclose(pk["snr"], ref, rtol=1e-4)
    zero = np.zeros(case.N, dtype=np.float32)
    t, pk, _ = rbmf.mf_full(ctx, bank, zero, 1e-3, peaks=True)
    assert len(t) == 0 and np.all(pk["snr"] == 0.0)
    t, _, st = rbmf.rb_filter(ctx, bases, bank, zero, 1e-3, 1e-3)
    assert len(t) == 0 and st.n_stage1 == 0
    for b in bases:
        b.close()
    bank.close()
