"""Every reconstruction-GEMM variant the autotuner may pick (forced with
RBMF_GEMM_VARIANT, read when a basis first runs), on sub-banks whose template
counts exercise whole 64-template tiles, a remainder, and a sub-bank smaller
than one tile: the FP32 variants against the oracle's reduced-basis SNR, the
BF16 / FP16 ones against the FP64 product of the quantised operands the
kernels read (stored 16-bit Z, RNE-rounded C), the split-BF16 ones against
the FP64 split product, every variant against the first, and the threshold
epilogues through the reconstruction second stage."""
import sys

import numpy as np
import pytest

from oracle import basis as ob
from oracle import mf as om
from paper_2110_13115_amd import rbmf
from tests.helpers import Case, quant, quantised_coefficients

pytestmark = pytest.mark.gpu

BOUNDS = [0, 64, 104, 300]        # 64 (one whole tile), 40 (remainder only), 196 (three tiles + 4)
# 16-bit: 0 / 2 realified coefficients on 64 / 128-sample Z tiles, 1 direct
# fragment loads, 3 / 4 compact coefficients (Im-output operand formed in
# registers) on 64 / 128-sample tiles
VARIANTS = {"f32": 7, "bf16": 5, "f16": 5, "bf16x3": 5}


def log(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def vcase():
    case = Case(N=32768, T=300, f_low=30.0, mrange=(5.0, 9.0), order=7, cfg=21,
                inj=((7, 12.0), (150, 8.0), (299, 6.5)))
    ctx = rbmf.Context(0)
    bank = rbmf.Bank(ctx, case.N, case.fs, case.f_low, case.psd, case.T, case.fill)
    yield case, ctx, bank
    bank.close()


def bases_for(ctx, bank, dtype, variant, monkeypatch):
    monkeypatch.setenv("RBMF_GEMM_VARIANT", str(variant))
    monkeypatch.delenv("RBMF_TUNE_FILE", raising=False)
    return [rbmf.Basis(ctx, bank, rank=r, dtype=dtype, t0=a, t1=b)
            for a, b, r in zip(BOUNDS[:-1], BOUNDS[1:], (21, 7, 37))]   # rank 7: a k-loop too short to pipeline


def issued_flop(dtype, variant, T, K, N):
    up = lambda x, m: -(-x // m) * m
    if dtype == "f32" and variant == 6:        # three real products per k-pair, 32-template tiles
        return 6 * up(T, 32) * up(K, 2) * N
    if dtype == "f32":                         # realified, 16-template blocks
        return 8 * up(T, 16) * K * N
    return 8 * up(T, 32) * up(K, 8) * N * (3 if dtype == "bf16x3" else 1)   # 32-template waves, 8-k steps


def keyset(tr, lo):
    return {(int(a), int(b)) for a, b, s in zip(tr["tmpl"], tr["sample"], tr["snr"]) if s >= lo}


@pytest.mark.parametrize("dtype", list(VARIANTS))
def test_every_variant(vcase, dtype, monkeypatch):
    case, ctx, bank = vcase
    k_lo, _ = om.band_limits(case.N, case.fs, case.f_low)
    d = ob.whitened_data(case.s64, case.psd, case.fs, case.f_low)
    ref_rho, ref_trig = None, None
    for v in range(VARIANTS[dtype]):
        bs = bases_for(ctx, bank, dtype, v, monkeypatch)
        rho = np.concatenate([rbmf.debug_rho(ctx, bank, case.strain, b) for b in bs])
        trig, _, st = rbmf.rb_filter(ctx, bs, bank, case.strain, 5.0, 6.0, stage2=rbmf.RB_STAGE2_RECON)
        # the matrix-core work the call reports: every sub-bank's GEMM at this
        # variant's tiling (padding rows and reduction steps included)
        assert st.gemm_mfma_flop == sum(issued_flop(dtype, v, b.T, b.K, case.N) for b in bs), v
        if dtype == "f32":
            # against the oracle's reduced-basis SNR with the exported bases
            ref = []
            for b in bs:
                V, c, _ = b.export()
                ref.append(ob.rb_snr(ob.basis_outputs(d, V, case.N, k_lo), c))
            ref = np.concatenate(ref)
            err = (np.abs(rho - ref) / np.maximum(np.abs(ref), 1.0)).max()
            log(dtype, "variant", v, "rho err vs oracle", err)
            assert err <= 1e-4, (v, err)
        if dtype in ("bf16", "f16"):
            ref = []
            for b in bs:
                V, c, _ = b.export()
                Z = rbmf.debug_basis_outputs(ctx, b, case.strain).astype(np.complex128)   # stored values
                ref.append(quantised_coefficients(c, dtype) @ Z)
            ref = np.concatenate(ref)
            err = (np.abs(rho - ref) / np.maximum(np.abs(ref), 1.0)).max()
            log(dtype, "variant", v, "rho err vs FP64 product of the quantised operands", err)
            assert err <= 1e-5, (v, err)
        if dtype == "bf16x3":
            ref = []
            for b in bs:
                V, c, _ = b.export()
                Zh, Zl = rbmf.debug_basis_outputs(ctx, b, case.strain).astype(np.complex128)
                Cc = np.conj(c).astype(np.complex64)
                hr, hi_ = quant(Cc.real, "bf16"), quant(Cc.imag, "bf16")
                lr = quant(np.asarray(Cc.real, np.float64) - hr, "bf16")
                li = quant(np.asarray(Cc.imag, np.float64) - hi_, "bf16")
                Ch, Cl = hr + 1j * hi_, lr + 1j * li
                ref.append(Ch @ Zh + Ch @ Zl + Cl @ Zh)
            ref = np.concatenate(ref)
            err = (np.abs(rho - ref) / np.maximum(np.abs(ref), 1.0)).max()
            log(dtype, "variant", v, "rho err vs FP64 split product", err)
            assert err <= 1e-5, (v, err)
        if ref_rho is None:
            ref_rho, ref_trig = rho, trig
        else:
            err = (np.abs(rho - ref_rho) / np.maximum(np.abs(ref_rho), 1.0)).max()
            log(dtype, "variant", v, "rho diff vs variant 0", err)
            assert err <= 2e-5, (v, err)
            # the epilogue's appends: the same crossings away from the threshold
            a, b = keyset(trig, 6.0 * (1 + 1e-4)), keyset(ref_trig, 6.0 * (1 + 1e-4))
            assert a <= keyset(ref_trig, 6.0 * (1 - 1e-4)) and b <= keyset(trig, 6.0 * (1 - 1e-4))
        assert len(trig) > 0
        for b in bs:
            b.close()
