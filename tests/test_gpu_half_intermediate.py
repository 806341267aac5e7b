"""The FFT intermediate of 16-bit bases: FP32 by default, FP16 pairs scaled
by the largest power of two that keeps every pass-1 output of a unit-norm
basis vector below 2^15 (chosen from max |d| of each segment) with
RB_OPT_FP16_INTERMEDIATE.  Against the FP64 oracle: final triggers on an
ordinary segment with either intermediate; a very loud signal, where the
option's scale shrinks by several powers of two: the default's first-stage
error on the scale of 16-bit rounding, sum_k |c_jk| |beta_k(n)| (next to a
loud chirp |beta_k| is large over a wide window while rho_j cancels, so the
error is not small relative to |rho| there), and the final triggers of the
full second stage with either intermediate; an all-zero strain (scale 1)."""
import sys

import numpy as np
import pytest

from oracle import basis as ob
from oracle import mf as om
from paper_2110_13115_amd import rbmf
from tests.helpers import Case, compare_triggers

pytestmark = pytest.mark.gpu

# the rounding of one product term is at most about 2 u |c| |beta| (u = 2^-9 BF16, 2^-11
# FP16: C and Z each rounded once), so the sum's error stays inside 2 u of its scale
SCALE_TOL = {"bf16": 2 * 2.0 ** -9, "f16": 2 * 2.0 ** -11}
H16 = rbmf.RB_OPT_FP16_INTERMEDIATE


def log(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = rbmf.Context(0)
    yield c
    c.close()


def oracle_rb(case, basis):
    """(rho_RB, sum_k |c_jk| |beta_k(n)|) of the exported basis, FP64."""
    V, c, _ = basis.export()
    k_lo, _ = om.band_limits(case.N, case.fs, case.f_low)
    d = ob.whitened_data(case.s64, case.psd, case.fs, case.f_low)
    beta = ob.basis_outputs(d, V, case.N, k_lo)
    return ob.rb_snr(beta, c), np.abs(c) @ np.abs(beta)


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_ordinary_segment(ctx, dtype):
    case = Case(N=32768, T=120, f_low=30.0, mrange=(5.0, 9.0), order=7, cfg=33,
                inj=((7, 12.0), (64, 8.0), (119, 6.5)))
    bank = rbmf.Bank(ctx, case.N, case.fs, case.f_low, case.psd, case.T, case.fill)
    basis = rbmf.Basis(ctx, bank, rank=0, tol=1e-3, dtype=dtype)
    try:
        for stage2 in (rbmf.RB_STAGE2_SPARSE, rbmf.RB_STAGE2_FULL):
            trig, _, st = rbmf.rb_filter(ctx, basis, bank, case.strain, 5.0, 6.0, stage2=stage2)
            compare_triggers(trig, case.rho, 6.0)
            trig16, _, st16 = rbmf.rb_filter(ctx, basis, bank, case.strain, 5.0, 6.0, stage2=stage2, flags=H16)
            compare_triggers(trig16, case.rho, 6.0)
            log(f"{dtype} stage2={stage2}: {len(trig)} final, stage-1 {st.n_stage1} (FP16 intermediate {st16.n_stage1})")
            assert abs(st.n_stage1 - st16.n_stage1) <= max(3, st.n_stage1 // 50)
        with pytest.raises(rbmf.RbError):
            rbmf.rb_filter(ctx, basis, bank, case.strain, 5.0, 6.0, flags=2)   # unknown flag
    finally:
        basis.close()
        bank.close()


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_loud_signal(ctx, dtype):
    # an injection at SNR 4000 beside one at 9: |d| peaks far above the noise
    case = Case(N=16384, T=96, f_low=30.0, mrange=(5.0, 9.0), order=7, cfg=31, inj=((11, 4000.0), (60, 9.0)))
    bank = rbmf.Bank(ctx, case.N, case.fs, case.f_low, case.psd, case.T, case.fill)
    basis = rbmf.Basis(ctx, bank, rank=0, tol=1e-3, dtype=dtype)
    try:
        rho = rbmf.debug_rho(ctx, bank, case.strain, basis)   # the default (FP32) intermediate
        ref, scale = oracle_rb(case, basis)
        assert np.isfinite(rho).all() and np.abs(ref).max() > 1000.0
        e = np.abs(rho - ref) / np.maximum(scale, 1.0)
        log(f"{dtype} loud: max |rho| {np.abs(ref).max():.0f}, max |err| {np.abs(rho - ref).max():.2f}, "
            f"err / sum|c||beta| max {e.max():.2e} (bound {SCALE_TOL[dtype]:.2e})")
        assert e.max() <= SCALE_TOL[dtype]
        # final triggers with either intermediate.  Next to a signal this loud the basis's own
        # truncation error (about sqrt(1 - 0.999) of the loud SNR) is far above any margin
        # between the stages, so the sparse second stage would not be exact here; the full one
        # refilters every template that crosses anywhere and finds every oracle trigger
        for flags in (0, H16):
            trig, _, st = rbmf.rb_filter(ctx, basis, bank, case.strain, 5.0, 6.0, stage2=rbmf.RB_STAGE2_FULL,
                                         flags=flags)
            compare_triggers(trig, case.rho, 6.0)
            log(f"{dtype} loud, flags {flags}: {len(trig)} final triggers = oracle's, stage-1 {st.n_stage1}")
    finally:
        basis.close()
        bank.close()


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_zero_strain(ctx, dtype):
    case = Case(N=16384, T=64, f_low=30.0, mrange=(5.0, 9.0), order=7, cfg=32, inj=((5, 10.0),))
    bank = rbmf.Bank(ctx, case.N, case.fs, case.f_low, case.psd, case.T, case.fill)
    basis = rbmf.Basis(ctx, bank, rank=0, tol=1e-3, dtype=dtype)
    try:
        zero = np.zeros(case.N, np.float32)
        trig, _, st = rbmf.rb_filter(ctx, basis, bank, zero, 5.0, 6.0, flags=H16)
        assert len(trig) == 0 and st.n_stage1 == 0
        # the next segment gets its own scale
        trig, _, _ = rbmf.rb_filter(ctx, basis, bank, case.strain, 5.0, 6.0, flags=H16)
        compare_triggers(trig, case.rho, 6.0)
    finally:
        basis.close()
        bank.close()
