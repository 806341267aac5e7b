"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Sizes are small enough for the oracle to hold every rho series, but span
several FFT tiles, GEMM tiles and ragged tails (T not a multiple of the
128-template tile, K not a multiple of 8, several N)."""
import sys

import numpy as np
import pytest

from oracle import basis as ob
from oracle import mf as om
from paper_2110_13115_amd import rbmf
from tests.helpers import Case, compare_triggers

pytestmark = pytest.mark.gpu


def log(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = rbmf.Context(0)
    yield c


def make_bank(ctx, case):
    return rbmf.Bank(ctx, case.N, case.fs, case.f_low, case.psd, case.T, case.fill)


# ------------------------------------------------------------------ template method
@pytest.mark.parametrize("N,T,f_low,mr,order", [(4096, 37, 25.0, (3.0, 9.0), 7),
                                                 (32768, 64, 30.0, (5.0, 20.0), 0),
                                                 (131072, 19, 20.0, (2.0, 6.0), 7)])
def test_mf_rho_series(ctx, N, T, f_low, mr, order):
    log("mf_rho", N, T)
    case = Case(N=N, T=T, f_low=f_low, mrange=mr, order=order, cfg=11, inj=((1, 12.0),))
    bank = make_bank(ctx, case)
    rho = rbmf.debug_rho(ctx, bank, case.strain)
    ref = case.rho
    err = np.abs(rho - ref) / np.maximum(np.abs(ref), 1.0)
    log("  max err", err.max())
    assert err.max() <= 1e-4
    _, klo, khi, sig = bank.info()
    assert (klo, khi) == om.band_limits(N, case.fs, f_low)
    np.testing.assert_allclose(sig, [om.sigma(h, case.psd, N, case.fs, f_low) for h in case.H], rtol=1e-12)
    bank.close()


@pytest.mark.parametrize("thr", [4.0, 5.0, 6.0])
def test_mf_full_triggers_config1_shape(ctx, thr):
    log("mf_full", thr)
    case = Case(N=32768, T=64, f_low=30.0, mrange=(5.0, 20.0), order=0, cfg=1, inj=((5, 10.0),))
    bank = make_bank(ctx, case)
    trig, peaks, st = rbmf.mf_full(ctx, bank, case.strain, thr, peaks=True)
    n_o, n_g, n_b = compare_triggers(trig, case.rho, thr)
    log("  oracle", n_o, "gpu", n_g, "band", n_b)
    a = np.abs(case.rho)
    np.testing.assert_allclose(peaks["snr"], a.max(axis=1), rtol=1e-4)
    srt = np.sort(a, axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 1e-3 * srt[:, -1]      # argmax unambiguous in FP32
    assert np.all(peaks["sample"][clear] == np.argmax(a, axis=1)[clear])
    inj = case.injections[0]
    hit = trig[(trig["tmpl"] == inj.template) & (trig["sample"] == inj.n0)]
    assert len(hit) == 1
    bank.close()


def test_mf_full_deterministic_and_capacity(ctx):
    case = Case(N=8192, T=40, f_low=25.0, mrange=(3.0, 9.0), order=7, cfg=12, inj=((3, 9.0),))
    bank = make_bank(ctx, case)
    t1, _, _ = rbmf.mf_full(ctx, bank, case.strain, 3.5)
    t2, _, _ = rbmf.mf_full(ctx, bank, case.strain, 3.5)
    assert t1.tobytes() == t2.tobytes()
    assert len(t1) > 10
    with pytest.raises(rbmf.RbError) as ei:
        rbmf.mf_full(ctx, bank, case.strain, 3.5, cap=3)
    assert ei.value.status == rbmf.RB_ERR_CAPACITY
    bad = case.strain.copy()
    bad[100] = np.nan
    with pytest.raises(rbmf.RbError) as ei:
        rbmf.mf_full(ctx, bank, bad, 5.0)
    assert ei.value.status == rbmf.RB_ERR_NUMERIC
    with pytest.raises(rbmf.RbError) as ei:
        rbmf.mf_full(ctx, bank, case.strain, -1.0)
    assert ei.value.status == rbmf.RB_ERR_ARG
    bank.close()


def test_cluster_peaks_match_oracle(ctx):
    case = Case(N=8192, T=24, f_low=25.0, mrange=(3.0, 9.0), order=7, cfg=13, inj=((2, 15.0), (9, 8.0)))
    bank = make_bank(ctx, case)
    trig, _, _ = rbmf.mf_full(ctx, bank, case.strain, 3.0)
    for W in (0, 16, 256, 4096):
        got = rbmf.cluster_peaks(ctx, trig, W, case.N)
        t64 = np.zeros(len(trig), dtype=om.TRIGGER_DTYPE)
        for f in ("tmpl", "sample", "snr", "phase"):
            t64[f] = trig[f]
        ref = om.cluster_peaks(t64, W, case.N)
        assert np.array_equal(got, ref), W
    bank.close()


def test_bank_errors(ctx):
    case = Case(N=4096, T=4, f_low=25.0, mrange=(3.0, 9.0), order=7, cfg=14, inj=())
    psd = case.psd.copy()
    psd[300] = 0.0
    with pytest.raises(rbmf.RbError) as ei:
        rbmf.Bank(ctx, case.N, case.fs, case.f_low, psd, case.T, case.fill)
    assert ei.value.status == rbmf.RB_ERR_ARG

    def boom(*a):
        raise ValueError("boom")
    with pytest.raises(ValueError):
        rbmf.Bank(ctx, case.N, case.fs, case.f_low, case.psd, case.T, boom)
    with pytest.raises(rbmf.RbError) as ei:
        rbmf.Bank(ctx, 5000, case.fs, case.f_low, case.psd, case.T, case.fill)
    assert ei.value.status == rbmf.RB_ERR_ARG


# ------------------------------------------------------------------ reduced basis
@pytest.fixture(scope="module")
def rb_case(ctx):
    case = Case(N=32768, T=300, f_low=30.0, mrange=(5.0, 9.0), order=7, cfg=21,
                inj=((7, 12.0), (150, 8.0), (299, 6.5)))
    bank = make_bank(ctx, case)
    yield case, bank
    bank.close()


def test_basis_properties(ctx, rb_case):
    case, bank = rb_case
    log("basis build")
    basis = rbmf.Basis(ctx, bank, rank=0, tol=1e-3, dtype="f32")
    V, c, lam = basis.export()
    K = basis.K
    log("  K", K, "energy", basis.energy)
    assert basis.energy >= 1 - 1e-3
    assert np.all(np.diff(lam) <= 1e-12 * lam[0])
    G = V @ V.conj().T
    assert np.abs(G - np.eye(K)).max() <= 1e-5        # stored complex64
    W, _ = case.whitened()
    _, so, Vo_h = np.linalg.svd(W, full_matrices=False)
    np.testing.assert_allclose(lam, so[:K] ** 2, rtol=1e-5, atol=1e-9 * so[0] ** 2)
    cum = np.cumsum(so ** 2) / np.sum(so ** 2)
    assert K == int(np.searchsorted(cum, 1 - 1e-3 - 1e-15) + 1)    # same rank as the oracle's rule
    # coefficients are the projections <w_j, v_k>
    np.testing.assert_allclose(c, W @ V.conj().T, atol=2e-6)
    # leading subspace agrees with the oracle SVD (well-separated leading part)
    k0 = min(10, K)
    sv = np.linalg.svd(V[:k0] @ Vo_h[:k0].conj().T, compute_uv=False)
    assert sv.min() >= 1 - 1e-6
    basis.close()


@pytest.mark.parametrize("rank", [8, 37])
def test_basis_outputs_and_rb_rho(ctx, rb_case, rank):
    case, bank = rb_case
    basis = rbmf.Basis(ctx, bank, rank=rank, dtype="f32")
    assert basis.K == rank
    V, c, lam = basis.export()
    k_lo, _ = om.band_limits(case.N, case.fs, case.f_low)
    d = ob.whitened_data(case.s64, case.psd, case.fs, case.f_low)
    beta_ref = ob.basis_outputs(d, V, case.N, k_lo)
    beta = rbmf.debug_basis_outputs(ctx, basis, case.strain)
    e1 = np.abs(beta - beta_ref).max() / np.abs(beta_ref).max()
    log("  beta err", rank, e1)
    assert e1 <= 2e-6 * np.sqrt(case.N / 4096) + 1e-6
    rho = rbmf.debug_rho(ctx, bank, case.strain, basis)
    rho_ref = ob.rb_snr(beta_ref, c)
    e2 = (np.abs(rho - rho_ref) / np.maximum(np.abs(rho_ref), 1.0)).max()
    log("  rho_rb err", rank, e2)
    assert e2 <= 1e-4
    basis.close()


def test_rb_filter_final_triggers(ctx, rb_case):
    case, bank = rb_case
    basis = rbmf.Basis(ctx, bank, rank=0, tol=1e-3, dtype="f32")
    trig, peaks, st = rbmf.rb_filter(ctx, basis, bank, case.strain, 5.0, 6.0, peaks=True)
    n_o, n_g, n_b = compare_triggers(trig, case.rho, 6.0)
    a = np.abs(case.rho)
    need = set(np.nonzero(a.max(axis=1) >= 6.0 * (1 + 1e-3))[0])
    log("  final", n_g, "oracle", n_o, "stage1", st.n_stage1, "refiltered", st.n_refiltered, "need", len(need))
    assert st.n_refiltered >= len(need)
    # peaks of refiltered templates are exact
    ev = peaks["snr"] >= 0
    assert ev.sum() == st.n_refiltered
    np.testing.assert_allclose(peaks["snr"][ev], a.max(axis=1)[ev], rtol=1e-4)
    assert np.all(peaks["snr"][~ev] == -1)
    t2, _, _ = rbmf.rb_filter(ctx, basis, bank, case.strain, 5.0, 6.0)
    assert t2.tobytes() == trig.tobytes()
    # sparse exact second stage: same final set, SNRs to 1e-4, peaks over evaluated samples
    ts, pks, sts = rbmf.rb_filter(ctx, basis, bank, case.strain, 5.0, 6.0, stage2=rbmf.RB_STAGE2_SPARSE,
                                  peaks=True)
    compare_triggers(ts, case.rho, 6.0)
    assert np.array_equal(ts[["tmpl", "sample"]], trig[["tmpl", "sample"]])
    assert sts.n_refiltered == st.n_refiltered
    ev = pks["snr"] >= 0
    assert ev.sum() == st.n_refiltered
    with pytest.raises(rbmf.RbError) as ei:
        rbmf.rb_filter(ctx, basis, bank, case.strain, 6.0, 5.0)
    assert ei.value.status == rbmf.RB_ERR_ARG
    basis.close()


def test_rb_filter_stage2_auto(ctx, rb_case, monkeypatch):
    """AUTO second stage: templates with many first-stage crossings take the
    full matched filter, the rest the direct sums; with the split forced low
    (2 crossings) both paths run, and the final triggers still equal the
    oracle's and the full second stage's."""
    case, bank = rb_case
    basis = rbmf.Basis(ctx, bank, rank=0, tol=1e-3, dtype="f32")
    full, _, st_f = rbmf.rb_filter(ctx, basis, bank, case.strain, 5.0, 6.0, stage2=rbmf.RB_STAGE2_FULL)
    for split in ("2", "1000000"):
        monkeypatch.setenv("RBMF_STAGE2_SPLIT", split)
        auto, _, st_a = rbmf.rb_filter(ctx, basis, bank, case.strain, 5.0, 6.0, stage2=rbmf.RB_STAGE2_AUTO)
        compare_triggers(auto, case.rho, 6.0)
        assert st_a.n_refiltered == st_f.n_refiltered
        log(f"  auto split {split}: {len(auto)} final (full {len(full)})")
    basis.close()


def _quant(x, dtype):
    """Round-to-nearest-even to bf16 / f16 (numpy emulation)."""
    x = np.asarray(x, np.float32)
    if dtype == "f16":
        return x.astype(np.float16).astype(np.float64)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_rb_16bit_matches_quantised_product(ctx, rb_case, dtype):
    case, bank = rb_case
    basis = rbmf.Basis(ctx, bank, rank=0, tol=1e-3, dtype=dtype)
    V, c, lam = basis.export()
    Z = rbmf.debug_basis_outputs(ctx, basis, case.strain).astype(np.complex128)   # stored 16-bit values
    Cc = np.conj(c).astype(np.complex64)
    if dtype == "f16":
        mx = np.maximum(np.abs(Cc.real), np.abs(Cc.imag)).max(axis=1)
        a = 2.0 ** (-np.frexp(mx)[1])
    else:
        a = np.ones(Cc.shape[0])
    Cs = (Cc * a[:, None].astype(np.float32))
    Cq = (_quant(Cs.real, dtype) + 1j * _quant(Cs.imag, dtype)) / a[:, None]
    ref = Cq @ Z
    rho = rbmf.debug_rho(ctx, bank, case.strain, basis)
    e_kernel = (np.abs(rho - ref) / np.maximum(np.abs(ref), 1.0)).max()
    k_lo, _ = om.band_limits(case.N, case.fs, case.f_low)
    d = ob.whitened_data(case.s64, case.psd, case.fs, case.f_low)
    exact = ob.rb_snr(ob.basis_outputs(d, V, case.N, k_lo), c)
    e_quant = (np.abs(rho - exact) / np.maximum(np.abs(exact), 1.0))
    log(f"  {dtype} kernel err {e_kernel:.2e}  vs FP64 max {e_quant.max():.2e} rms {np.sqrt(np.mean(e_quant**2)):.2e}")
    assert e_kernel <= 1e-5
    assert e_quant.max() <= (3e-2 if dtype == "bf16" else 4e-3)
    trig, _, st = rbmf.rb_filter(ctx, basis, bank, case.strain, 5.0, 6.0)
    compare_triggers(trig, case.rho, 6.0)
    basis.close()


def test_rb_bf16x3_fp32_accuracy(ctx, rb_case):
    """Split-BF16 reconstruction (hi + lo of C and Z, three MFMA products):
    equals the emulated split product to FP32 rounding and stays within the
    FP32 path's 1e-4 of the FP64 reduced-basis SNR."""
    case, bank = rb_case
    basis = rbmf.Basis(ctx, bank, rank=0, tol=1e-3, dtype="bf16x3")
    V, c, lam = basis.export()
    Zh, Zl = rbmf.debug_basis_outputs(ctx, basis, case.strain).astype(np.complex128)   # stored planes
    # each plane holds BF16 values, and the low parts are below half an ULP of the high parts
    assert np.array_equal(_quant(Zh.real, "bf16"), Zh.real) and np.array_equal(_quant(Zl.imag, "bf16"), Zl.imag)
    assert (np.abs(Zl.real) <= np.abs(Zh.real) * 2.0 ** -8 + 1e-38).all()
    Cc = np.conj(c).astype(np.complex64)

    def split(x):
        h = _quant(x, "bf16")
        return h, _quant(np.asarray(x, np.float64) - h, "bf16")
    hr, lr = split(Cc.real)
    hi_, li = split(Cc.imag)
    Ch, Cl = hr + 1j * hi_, lr + 1j * li
    ref = Ch @ Zh + Ch @ Zl + Cl @ Zh
    rho = rbmf.debug_rho(ctx, bank, case.strain, basis)
    e_kernel = (np.abs(rho - ref) / np.maximum(np.abs(ref), 1.0)).max()
    k_lo, _ = om.band_limits(case.N, case.fs, case.f_low)
    d = ob.whitened_data(case.s64, case.psd, case.fs, case.f_low)
    exact = ob.rb_snr(ob.basis_outputs(d, V, case.N, k_lo), c)
    e64 = (np.abs(rho - exact) / np.maximum(np.abs(exact), 1.0))
    log(f"  bf16x3 kernel err {e_kernel:.2e}  vs FP64 max {e64.max():.2e} rms {np.sqrt(np.mean(e64**2)):.2e}")
    assert e_kernel <= 1e-5
    assert e64.max() <= 1e-4
    trig, _, st = rbmf.rb_filter(ctx, basis, bank, case.strain, 5.0, 6.0, stage2=rbmf.RB_STAGE2_SPARSE)
    compare_triggers(trig, case.rho, 6.0)
    basis.close()


def test_tune_cache_file(ctx, rb_case, tmp_path, monkeypatch):
    """Tuned choices are written to RBMF_TUNE_FILE as a flat JSON object."""
    import json
    case, bank = rb_case
    path = tmp_path / "tune.json"
    monkeypatch.setenv("RBMF_TUNE_FILE", str(path))
    basis = rbmf.Basis(ctx, bank, rank=7, dtype="f32")          # a (K, T) pair not tuned before
    rbmf.rb_filter(ctx, basis, bank, case.strain, 5.0, 6.0)
    basis.close()
    table = json.loads(path.read_text())
    key = f"/gemm3/dt=0/K=7/T={case.T}/N={case.N}"
    hits = [k for k in table if k.endswith(key)]
    assert len(hits) == 1 and 0 <= table[hits[0]] < 7     # one of the seven FP32 variants
    assert all(isinstance(v, int) for v in table.values())
    log("  tune cache", len(table), "entries")


def test_subbank_bases_partition(ctx, rb_case):
    """Bases of three template ranges (sub-banks, Sec. III.B): the final
    triggers equal the oracle's; per-range reconstruction matches the oracle's
    with each range's own basis; bad partitions are rejected."""
    case, bank = rb_case
    bounds = [0, 97, 211, case.T]
    bases = rbmf.subbank_bases(ctx, bank, bounds, rank=[10, 0, 23], tol=1e-3, dtype="f32")
    assert [b.K for b in bases][0] == 10 and bases[2].K == 23
    trig, _, st = rbmf.rb_filter(ctx, bases, bank, case.strain, 5.0, 6.0)
    compare_triggers(trig, case.rho, 6.0)
    k_lo, _ = om.band_limits(case.N, case.fs, case.f_low)
    d = ob.whitened_data(case.s64, case.psd, case.fs, case.f_low)
    b = bases[1]
    V, c, _ = b.export()
    assert c.shape == (bounds[2] - bounds[1], b.K)
    rho = rbmf.debug_rho(ctx, bank, case.strain, b)
    ref = ob.rb_snr(ob.basis_outputs(d, V, case.N, k_lo), c)
    assert (np.abs(rho - ref) / np.maximum(np.abs(ref), 1.0)).max() <= 1e-4
    S = np.zeros(3, dtype=rbmf.TRIGGER_NP)
    S["tmpl"] = [bounds[1], bounds[1] + 5, bounds[2] - 1]
    S["sample"] = [0, 100, case.N - 1]
    r = rbmf.rho_at(ctx, b, case.strain, S)
    np.testing.assert_allclose(r, rho[S["tmpl"] - bounds[1], S["sample"]], rtol=1e-5, atol=1e-5)
    bad = S.copy()
    bad["tmpl"][0] = 0          # outside the basis's range
    with pytest.raises(rbmf.RbError):
        rbmf.rho_at(ctx, b, case.strain, bad)
    with pytest.raises(rbmf.RbError):          # gap in the partition
        rbmf.rb_filter(ctx, [bases[0], bases[2]], bank, case.strain, 5.0, 6.0)
    for x in bases:
        x.close()
