"""GPU parity of the binned first stage (rb_filter with bin_w >= 2) and of the
reconstruction second stage (RB_STAGE2_RECON) against the FP64 oracle
(oracle/hier.py), through the C ABI.

Comparison rule: a (template, sample) decision is ambiguous when an oracle
quantity it depends on lies within a relative 1e-3 of its threshold (the
bin's |rho_avg| against thr_bin, |rho_RB| against thr1, the final SNR
against thr2).  The GPU set must hold every unambiguous oracle trigger and
nothing outside the possible ones; matched SNRs agree to 1e-4 relative."""
import sys

import numpy as np
import pytest

from oracle import basis as ob
from oracle import hier as oh
from oracle import mf as om
from paper_2110_13115_amd import rbmf
from tests.helpers import BAND, SNR_RTOL, Case

pytestmark = pytest.mark.gpu


def log(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    return rbmf.Context(0)


@pytest.fixture(scope="module")
def bcase(ctx):
    case = Case(N=32768, T=300, f_low=30.0, mrange=(5.0, 9.0), order=7, cfg=21,
                inj=((7, 12.0), (150, 8.0), (299, 6.5)))
    bank = rbmf.Bank(ctx, case.N, case.fs, case.f_low, case.psd, case.T, case.fill)
    basis = rbmf.Basis(ctx, bank, rank=0, tol=1e-3, dtype="f32")
    V, c, _ = basis.export()
    k_lo, _ = om.band_limits(case.N, case.fs, case.f_low)
    d = ob.whitened_data(case.s64, case.psd, case.fs, case.f_low)
    beta = ob.basis_outputs(d, V, case.N, k_lo)
    yield case, bank, basis, beta, c
    basis.close()
    bank.close()


def _band(x, t):
    return (x >= t * (1 - BAND)) & (x <= t * (1 + BAND))


def candidates_ref(beta, c, w, thr_bin, thr1):
    """(sure, maybe, |rho_RB|): T x N masks of the oracle's candidates whose
    decision is unambiguous / ambiguous, and the FP64 reconstruction."""
    a_avg = np.abs(oh.averaged_snr(beta, c, w))
    a_rb = np.abs(ob.rb_snr(beta, c))
    on = np.repeat(a_avg >= thr_bin, w, axis=1)
    amb = np.repeat(_band(a_avg, thr_bin), w, axis=1)
    sure = on & ~amb & (a_rb >= thr1) & ~_band(a_rb, thr1)
    maybe = (on | amb) & (a_rb >= thr1 * (1 - BAND)) & ~sure
    return sure, maybe, a_rb, a_avg


def check_sets(got, definite, possible, ref_abs):
    G = np.zeros_like(definite)
    G[got["tmpl"], got["sample"]] = True
    assert len(got) == int(G.sum()), "duplicate GPU triggers"
    miss = definite & ~G
    extra = G & ~possible
    assert not miss.any(), f"{int(miss.sum())} oracle triggers missing, e.g. {np.argwhere(miss)[:5]}"
    assert not extra.any(), f"{int(extra.sum())} extra GPU triggers, e.g. {np.argwhere(extra)[:5]}"
    ref = ref_abs[got["tmpl"], got["sample"]]
    rel = np.abs(got["snr"].astype(np.float64) - ref) / ref
    assert rel.max(initial=0) <= SNR_RTOL, f"max rel |rho| error {rel.max():.3e}"
    order = np.lexsort((got["sample"], got["tmpl"]))
    assert np.all(order == np.arange(len(got))), "triggers not sorted by (tmpl, sample)"


@pytest.mark.parametrize("split", [None, 6, 8])
def test_binned_series_matches_oracle(bcase, split, monkeypatch):
    """rho_avg = C beta_avg elementwise, for bins larger and smaller than the
    rows of one pass-2 workgroup (FFT split forced: N1 = 512, 256, 128)."""
    case, bank, basis, beta, c = bcase
    if split is not None:
        monkeypatch.setenv("RBMF_FFT_SPLIT", str(split))
    cx = rbmf.Context(0)          # a fresh context re-reads the split
    bk = rbmf.Bank(cx, case.N, case.fs, case.f_low, case.psd, case.T, case.fill)
    bs = rbmf.Basis(cx, bk, rank=0, tol=1e-3, dtype="f32")
    assert bs.K == basis.K
    V, cc, _ = bs.export()
    k_lo, _ = om.band_limits(case.N, case.fs, case.f_low)
    d = ob.whitened_data(case.s64, case.psd, case.fs, case.f_low)
    bt = ob.basis_outputs(d, V, case.N, k_lo)
    for w in (2, 8, 16, 64):
        log("rho_avg split", split, "w", w)
        got = rbmf.debug_rho_binned(cx, bs, case.strain, w)
        ref = oh.averaged_snr(bt, cc, w)
        err = (np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)).max()
        log("  max err", err)
        assert err <= 2e-5
    bs.close()
    bk.close()


@pytest.mark.parametrize("w,thr_bin", [(2, 3.5), (8, 3.0), (16, 2.0)])
def test_binned_recon_matches_oracle(ctx, bcase, w, thr_bin):
    case, bank, basis, beta, c = bcase
    thr1, thr2 = 4.5, 5.5
    log("recon w", w, "thr_bin", thr_bin)
    got, pk, st = rbmf.rb_filter(ctx, basis, bank, case.strain, thr1, thr2, stage2=rbmf.RB_STAGE2_RECON,
                                 peaks=True, bin_w=w, thr_bin=thr_bin)
    sure, maybe, a_rb, a_avg = candidates_ref(beta, c, w, thr_bin, thr1)
    definite = sure & (a_rb >= thr2) & ~_band(a_rb, thr2)
    possible = (sure | maybe) & (a_rb >= thr2 * (1 - BAND))
    log("  final", len(got), "oracle", int(definite.sum()), "bins", st.n_bins, "cand", st.n_stage1)
    assert definite.sum() > 10
    check_sets(got, definite, possible, a_rb)
    lo, hi = (a_avg >= thr_bin * (1 + BAND)).sum(), (a_avg >= thr_bin * (1 - BAND)).sum()
    assert lo <= st.n_bins <= hi
    assert sure.sum() <= st.n_stage1 <= (sure | maybe).sum()
    # peaks: the maximum reconstructed SNR over each template's candidates
    ev = pk["snr"] >= 0
    cand_t = (sure | maybe).any(axis=1)
    assert np.all(ev <= cand_t) and np.all(sure.any(axis=1) <= ev)
    mx = np.where(sure | maybe, a_rb, 0).max(axis=1)
    np.testing.assert_allclose(pk["snr"][ev & ~maybe.any(axis=1)], mx[ev & ~maybe.any(axis=1)], rtol=1e-4)
    # the injections at SNR 12 and 8 are recovered at their own template
    for inj in case.injections[:2]:
        assert definite[inj.template, inj.n0], inj
    again, _, _ = rbmf.rb_filter(ctx, basis, bank, case.strain, thr1, thr2, stage2=rbmf.RB_STAGE2_RECON,
                                 bin_w=w, thr_bin=thr_bin)
    assert again.tobytes() == got.tobytes()


@pytest.mark.parametrize("mode", ["sparse", "full"])
def test_binned_exact_second_stage(ctx, bcase, mode):
    """Binned first stage, exact second stage: SPARSE evaluates the template
    method at the candidates, FULL filters every candidate template."""
    case, bank, basis, beta, c = bcase
    w, thr_bin, thr1, thr2 = 8, 3.0, 4.5, 5.5
    sure, maybe, a_rb, _ = candidates_ref(beta, c, w, thr_bin, thr1)
    ex = np.abs(case.rho)
    if mode == "sparse":
        st2 = rbmf.RB_STAGE2_SPARSE
        definite = sure & (ex >= thr2) & ~_band(ex, thr2)
        possible = (sure | maybe) & (ex >= thr2 * (1 - BAND))
    else:
        st2 = rbmf.RB_STAGE2_FULL
        ts, tm = sure.any(axis=1), (sure | maybe).any(axis=1)
        definite = ts[:, None] & (ex >= thr2) & ~_band(ex, thr2)
        possible = tm[:, None] & (ex >= thr2 * (1 - BAND))
    got, _, st = rbmf.rb_filter(ctx, basis, bank, case.strain, thr1, thr2, stage2=st2, bin_w=w,
                                thr_bin=thr_bin)
    log(mode, "final", len(got), "oracle", int(definite.sum()), "refiltered", st.n_refiltered)
    assert definite.sum() > 10
    check_sets(got, definite, possible, ex)


def test_recon_without_bins(ctx, bcase):
    """RECON with bin_w = 0: the final triggers are the first-stage samples
    whose |rho_RB| reaches thr2 (FP32 against the oracle; BF16 against the
    library's own BF16 reconstruction, which checks the storage scales)."""
    case, bank, basis, beta, c = bcase
    got, _, st = rbmf.rb_filter(ctx, basis, bank, case.strain, 4.5, 5.5, stage2=rbmf.RB_STAGE2_RECON)
    a_rb = np.abs(ob.rb_snr(beta, c))
    definite = (a_rb >= 5.5) & ~_band(a_rb, 5.5)
    check_sets(got, definite, a_rb >= 5.5 * (1 - BAND), a_rb)
    assert st.n_bins == 0
    b16 = rbmf.Basis(ctx, bank, rank=0, tol=1e-3, dtype="bf16")
    rho16 = np.abs(rbmf.debug_rho(ctx, bank, case.strain, b16).astype(np.complex128))
    g16, _, _ = rbmf.rb_filter(ctx, b16, bank, case.strain, 4.5, 5.5, stage2=rbmf.RB_STAGE2_RECON)
    d16 = (rho16 >= 5.5) & ~(np.abs(rho16 / 5.5 - 1) <= 1e-5)
    check_sets(g16, d16, rho16 >= 5.5 * (1 - 1e-5), rho16)
    b16.close()


def test_binned_argument_errors(ctx, bcase):
    case, bank, basis, beta, c = bcase
    for w, tb in [(3, 2.0), (128, 2.0), (-1, 2.0), (8, 0.0), (8, float("nan"))]:
        with pytest.raises(rbmf.RbError) as ei:
            rbmf.rb_filter(ctx, basis, bank, case.strain, 4.5, 5.5, bin_w=w, thr_bin=tb)
        assert ei.value.status == rbmf.RB_ERR_ARG, (w, tb)
    with pytest.raises(rbmf.RbError) as ei:
        rbmf.debug_rho_binned(ctx, basis, case.strain, 256)     # N / w < 256
    assert ei.value.status == rbmf.RB_ERR_ARG
    with pytest.raises(rbmf.RbError) as ei:
        rbmf.rb_filter(ctx, basis, bank, case.strain, 4.5, 5.5, stage2=7)
    assert ei.value.status == rbmf.RB_ERR_ARG
    # nothing triggers: empty result, every peak unevaluated
    got, pk, st = rbmf.rb_filter(ctx, basis, bank, case.strain, 4.5, 5.5, stage2=rbmf.RB_STAGE2_RECON,
                                 peaks=True, bin_w=64, thr_bin=50.0)
    assert len(got) == 0 and st.n_bins == 0 and st.n_stage1 == 0 and np.all(pk["snr"] == -1)


def test_binned_subbanks_partition(ctx, bcase):
    """Sub-bank bases: the binned search over a partition equals the union of
    the oracle's per-sub-bank searches."""
    case, bank, basis, beta, c = bcase
    bounds = [0, 90, 201, 300]
    subs = [rbmf.Basis(ctx, bank, rank=0, tol=1e-3, dtype="f32", t0=a, t1=b) for a, b in zip(bounds, bounds[1:])]
    w, thr_bin, thr1, thr2 = 8, 3.0, 4.5, 5.5
    got, _, st = rbmf.rb_filter(ctx, subs, bank, case.strain, thr1, thr2, stage2=rbmf.RB_STAGE2_RECON,
                                bin_w=w, thr_bin=thr_bin)
    k_lo, _ = om.band_limits(case.N, case.fs, case.f_low)
    d = ob.whitened_data(case.s64, case.psd, case.fs, case.f_low)
    S, M, A = [], [], []
    for b in subs:
        V, cs, _ = b.export()
        sure, maybe, a_rb, _ = candidates_ref(ob.basis_outputs(d, V, case.N, k_lo), cs, w, thr_bin, thr1)
        S.append(sure)
        M.append(maybe)
        A.append(a_rb)
    sure, maybe, a_rb = np.vstack(S), np.vstack(M), np.vstack(A)
    definite = sure & (a_rb >= thr2) & ~_band(a_rb, thr2)
    possible = (sure | maybe) & (a_rb >= thr2 * (1 - BAND))
    log("subbanks final", len(got), "oracle", int(definite.sum()))
    check_sets(got, definite, possible, a_rb)
    for b in subs:
        b.close()


@pytest.mark.parametrize("dtype", ["bf16", "f16", "bf16x3"])
def test_binned_16bit_storage(ctx, bcase, dtype):
    """Binned first stage on 16-bit storage: the averaged series within the
    rounding of its operands, and the RECON finals (fine reconstruction from
    Z in the basis's storage precision, FP32 accumulation) against the FP64
    reconstruction with a band and tolerance of that precision."""
    case, bank, basis, beta, c = bcase
    tol = {"bf16": 3e-2, "f16": 4e-3, "bf16x3": 1e-4}[dtype]
    b16 = rbmf.Basis(ctx, bank, rank=0, tol=1e-3, dtype=dtype)
    assert b16.K == basis.K
    w, thr_bin, thr1, thr2 = 8, 3.0, 4.5, 5.5
    got_avg = rbmf.debug_rho_binned(ctx, b16, case.strain, w)
    ref_avg = oh.averaged_snr(beta, c, w)
    err = (np.abs(got_avg - ref_avg) / np.maximum(np.abs(ref_avg), 1.0)).max()
    log(dtype, "rho_avg max err", err)
    assert err <= tol
    a_avg = np.abs(ref_avg)
    a_rb = np.abs(ob.rb_snr(beta, c))
    band = lambda x, t: np.abs(x / t - 1) <= tol
    on = np.repeat(a_avg >= thr_bin, w, axis=1)
    amb = np.repeat(band(a_avg, thr_bin), w, axis=1)
    sure = on & ~amb & (a_rb >= thr1) & ~band(a_rb, thr1)
    maybe = (on | amb) & (a_rb >= thr1 * (1 - tol)) & ~sure
    definite = sure & (a_rb >= thr2) & ~band(a_rb, thr2)
    possible = (sure | maybe) & (a_rb >= thr2 * (1 - tol))
    assert definite.sum() > 10
    # BF16 / FP16 also with the FP16 FFT intermediate option (fine Z and bin means from it)
    for flags in ((0,) if dtype == "bf16x3" else (0, rbmf.RB_OPT_FP16_INTERMEDIATE)):
        got, _, st = rbmf.rb_filter(ctx, b16, bank, case.strain, thr1, thr2, stage2=rbmf.RB_STAGE2_RECON,
                                    bin_w=w, thr_bin=thr_bin, flags=flags)
        G = np.zeros_like(definite)
        G[got["tmpl"], got["sample"]] = True
        log(dtype, "flags", flags, "final", len(got), "oracle", int(definite.sum()))
        assert not (definite & ~G).any() and not (G & ~possible).any()
        rel = np.abs(got["snr"] - a_rb[got["tmpl"], got["sample"]]) / a_rb[got["tmpl"], got["sample"]]
        assert rel.max() <= tol
    b16.close()


@pytest.mark.parametrize("mode", ["recon", "sparse"])
def test_template_fold_first_stage(ctx, bcase, mode):
    """bin_source 1: the averaged series from the templates (Sec. III.D, the
    fold of Eq. avg_fft2, exact bin means of the template method), the fine
    stage from the basis.  Bins against the oracle's bin means of the FP64
    template-method series; candidates and finals as in the basis case."""
    case, bank, basis, beta, c = bcase
    w, thr_bin, thr1, thr2 = 8, 3.0, 4.5, 5.5
    st2 = rbmf.RB_STAGE2_RECON if mode == "recon" else rbmf.RB_STAGE2_SPARSE
    got, _, st = rbmf.rb_filter(ctx, basis, bank, case.strain, thr1, thr2, stage2=st2, bin_w=w,
                                thr_bin=thr_bin, bin_source=1)
    a_avg = np.abs(oh.bin_means(case.rho, w))
    a_rb = np.abs(ob.rb_snr(beta, c))
    on = np.repeat(a_avg >= thr_bin, w, axis=1)
    amb = np.repeat(_band(a_avg, thr_bin), w, axis=1)
    sure = on & ~amb & (a_rb >= thr1) & ~_band(a_rb, thr1)
    maybe = (on | amb) & (a_rb >= thr1 * (1 - BAND)) & ~sure
    lo, hi = (a_avg >= thr_bin * (1 + BAND)).sum(), (a_avg >= thr_bin * (1 - BAND)).sum()
    log("fold", mode, "bins", st.n_bins, "oracle", lo, hi, "final", len(got))
    assert lo <= st.n_bins <= hi and lo > 50
    assert sure.sum() <= st.n_stage1 <= (sure | maybe).sum()
    ref = a_rb if mode == "recon" else np.abs(case.rho)
    definite = sure & (ref >= thr2) & ~_band(ref, thr2)
    possible = (sure | maybe) & (ref >= thr2 * (1 - BAND))
    assert definite.sum() > 10
    check_sets(got, definite, possible, ref)


def test_template_fold_arguments(ctx, bcase):
    case, bank, basis, beta, c = bcase
    for kw in ({"bin_w": 16, "thr_bin": 2.0, "bin_source": 1},     # N / w = 2048 < 4096
               {"bin_w": 0, "thr_bin": 2.0, "bin_source": 1},      # needs bins
               {"bin_w": 8, "thr_bin": 2.0, "bin_source": 2}):
        with pytest.raises(rbmf.RbError) as ei:
            rbmf.rb_filter(ctx, basis, bank, case.strain, 4.5, 5.5, **kw)
        assert ei.value.status == rbmf.RB_ERR_ARG, kw
    got, _, st = rbmf.rb_filter(ctx, basis, bank, case.strain, 4.5, 5.5, stage2=rbmf.RB_STAGE2_RECON,
                                bin_w=8, thr_bin=40.0, bin_source=1)
    assert len(got) == 0 and st.n_bins == 0 and st.n_stage1 == 0
