"""Pins of the FP64 binned first stage (oracle/hier.py) against brute-force
sums, closed forms, the template-method fold of Eq. avg_fft2 and special
cases that reduce to the unbinned search.  CPU only."""
import numpy as np
import pytest

from oracle import basis as ob
from oracle import hier as oh
from oracle import mf as om
from paper_2110_13115_amd import inputs as gi


def test_bin_means_brute_force_and_closed_forms():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 16)) + 1j * rng.standard_normal((3, 16))
    w = 4
    ref = np.zeros((3, 4), dtype=complex)
    for a in range(3):
        for i in range(4):
            s = 0
            for r in range(w):
                s += x[a, i * w + r]
            ref[a, i] = s / w
    np.testing.assert_allclose(oh.bin_means(x, w), ref, rtol=0, atol=1e-15)
    n = np.arange(64.0)
    # a ramp: the mean of bin i is i w + (w - 1)/2
    for w in (1, 2, 8, 64):
        np.testing.assert_allclose(oh.bin_means(n, w).real, np.arange(64 // w) * w + (w - 1) / 2, atol=1e-12)
    # a tone of period w (or w/2) averages to zero over every bin; a constant is kept
    for m in (1, 2):
        tone = np.exp(2j * np.pi * m * n / 8)
        assert np.abs(oh.bin_means(tone, 8)).max() <= 1e-14
    np.testing.assert_allclose(oh.bin_means(np.full(64, 2.5 - 1j), 16), 2.5 - 1j, atol=1e-15)
    with pytest.raises(ValueError):
        oh.bin_means(x, 3)


def test_geometric_kernel_is_the_sum_it_closes():
    for N, w in [(16, 4), (64, 1), (64, 8), (256, 64)]:
        f = np.arange(N)
        direct = sum(np.exp(2j * np.pi * f * r / N) for r in range(w))
        np.testing.assert_allclose(oh.geometric_kernel(N, w), direct, rtol=0, atol=1e-12 * w)


@pytest.fixture(scope="module")
def case():
    N, fs, f_low = 4096, 1024.0, 20.0
    bank = gi.random_bank(905, 24, N, fs, f_low, 3.0, 6.0, 7)
    psd = gi.psd_on_grid(N, fs)
    H = bank.full()
    W, sig = ob.whitened_unit_templates(H, psd, N, fs, f_low)
    rng = np.random.default_rng([13115, 905, 1])
    st = gi.coloured_noise_tilde(psd, N, fs, rng)
    # one template injected at SNR 9 so that the high end is populated
    n0 = 1234
    st = gi.add_injection(st, H[5], 9.0 / om.sigma(H[5], psd, N, fs, f_low), n0, 0.7, N)
    s = gi.strain_from_tilde(st, N, fs)
    k_lo, _ = om.band_limits(N, fs, f_low)
    d = ob.whitened_data(s, psd, fs, f_low)
    return dict(N=N, fs=fs, f_low=f_low, H=H, W=W, psd=psd, s=s, d=d, k_lo=k_lo, n0=n0)


def _integrand(c, j):
    """One-sided X[f] = d[f] conj(w_j[f]) on all N bins."""
    X = np.zeros(c["N"], dtype=complex)
    X[c["k_lo"]:c["k_lo"] + c["W"].shape[1]] = c["d"] * np.conj(c["W"][j])
    return X


@pytest.mark.parametrize("w", [1, 2, 8, 16, 64])
def test_fold_equals_bin_average(case, w):
    """Eq. avg_fft2: the bin mean of the template method's series equals the
    N/w-point inverse transform of the folded integrand Omega."""
    for j in (0, 5, 23):
        rho = ob.mf_whitened(case["d"], case["W"][j:j + 1], case["N"], case["k_lo"])[0]
        a = oh.bin_means(rho, w)
        b = oh.folded_average(_integrand(case, j), w)
        assert np.abs(a - b).max() <= 1e-11 * np.abs(rho).max()
        # the series is the unnormalised inverse transform, as in Eq. IFFT
        np.testing.assert_allclose(rho, om.snr_series(case["s"], case["H"][j], case["psd"], case["fs"],
                                                      case["f_low"]), atol=1e-10 * np.abs(rho).max())


def test_full_rank_binned_stage_equals_template_method(case):
    """With the complete basis, the averaged SNR of Eq. Beta_eqn is the fold of
    the template method, the candidates are the template method's samples
    in the triggering bins, and each variant of the second stage follows."""
    N, W, d, k_lo = case["N"], case["W"], case["d"], case["k_lo"]
    V, cf, *_ = ob.svd_basis(W, rank=W.shape[0])
    beta = ob.basis_outputs(d, V, N, k_lo)
    rho = ob.mf_whitened(d, W, N, k_lo)
    w, thr_bin, thr1, thr2 = 8, 1.2, 2.5, 4.0
    avg = oh.averaged_snr(beta, cf, w)
    fold = np.stack([oh.folded_average(_integrand(case, j), w) for j in range(W.shape[0])])
    assert np.abs(avg - fold).max() <= 1e-10 * np.abs(fold).max()
    bins, cand, fin = oh.hierarchical_search(beta, cf, w, thr_bin, thr1, thr2, "recon")
    assert len(bins) > 10 and len(cand) > 10
    # candidates by brute force from the template method's series
    exp = []
    for j in range(W.shape[0]):
        for i in np.nonzero(np.abs(fold[j]) >= thr_bin)[0]:
            for n in range(i * w, i * w + w):
                if abs(rho[j, n]) >= thr1:
                    exp.append((j, n))
    assert [(int(a), int(b)) for a, b in zip(cand["tmpl"], cand["sample"])] == sorted(exp)
    np.testing.assert_allclose(cand["snr"], np.abs(rho[cand["tmpl"], cand["sample"]]), rtol=1e-10)
    # at full rank the three second stages agree where they overlap
    ex = lambda j: rho[j]
    sp = oh.second_stage(cand, thr2, "sparse", ex)
    assert np.array_equal(fin[["tmpl", "sample"]], sp[["tmpl", "sample"]])
    full = oh.second_stage(cand, thr2, "full", ex)
    ref = om.triggers([(j, rho[j]) for j in np.unique(cand["tmpl"])], thr2)
    assert np.array_equal(full[["tmpl", "sample"]], ref[["tmpl", "sample"]])
    # the injection is found at its sample with its SNR
    hit = fin[(fin["tmpl"] == 5) & (fin["sample"] == case["n0"])]
    assert len(hit) == 1 and hit["snr"][0] > 8.0


def test_every_triggering_bin_holds_a_crossing(case):
    """|mean| <= max |.| over a bin: every bin whose average reaches rho_I has
    at least one sample of the full-rate series that reaches it too."""
    N, W, d, k_lo = case["N"], case["W"], case["d"], case["k_lo"]
    V, cf, *_ = ob.svd_basis(W, tol=1e-3)
    beta = ob.basis_outputs(d, V, N, k_lo)
    for w in (2, 16):
        bins = oh.triggering_bins(oh.averaged_snr(beta, cf, w), 2.0)
        cand = oh.fine_candidates(beta, cf, bins, w, 2.0)
        got = set(zip(cand["tmpl"].tolist(), (cand["sample"] // w).tolist()))
        assert got == set(zip(bins["tmpl"].tolist(), bins["bin"].tolist()))


def test_w1_reduces_to_the_unbinned_search(case):
    N, W, d, k_lo = case["N"], case["W"], case["d"], case["k_lo"]
    V, cf, *_ = ob.svd_basis(W, rank=9)
    beta = ob.basis_outputs(d, V, N, k_lo)
    rb = ob.rb_snr(beta, cf)
    bins, cand, fin = oh.hierarchical_search(beta, cf, 1, 3.0, 3.0, 4.0, "recon", t0=100)
    ref = om.triggers([(j + 100, rb[j]) for j in range(W.shape[0])], 3.0)
    assert np.array_equal(cand[["tmpl", "sample"]], ref[["tmpl", "sample"]])
    np.testing.assert_allclose(cand["snr"], ref["snr"], rtol=1e-12)
    assert np.array_equal(fin, cand[cand["snr"] >= 4.0])
    assert np.array_equal(bins["bin"], cand["sample"])


def test_averaging_lowers_noise_snr(case):
    """Sec. III.C: the bin average of a chirp's complex output rotates through
    its phase, so averaging lowers |rho| and fewer bins reach a fixed rho_I as
    w grows (the reason the first-stage threshold is lowered)."""
    N, W, d, k_lo = case["N"], case["W"], case["d"], case["k_lo"]
    V, cf, *_ = ob.svd_basis(W, tol=1e-3)
    beta = ob.basis_outputs(d, V, N, k_lo)
    frac = []
    for w in (1, 2, 4, 8, 16):
        a = np.abs(oh.averaged_snr(beta, cf, w))
        frac.append(np.mean(a >= 2.0))
    assert all(x > y for x, y in zip(frac, frac[1:]))


def test_target_snr_definition():
    flat = np.array([5.0, 5.2, 6.0, 7.0, 8.0])
    fin = np.array([5.2, 6.0, 7.0, 8.0])          # the 5.0 trigger is lost
    grid = np.array([4.5, 5.0, 5.1, 6.0])
    # 4.5 and 5.0: 4 < 0.99 * 5; 5.1: 4 >= 0.99 * 4
    assert oh.target_snr(fin, flat, grid) == 5.1
    assert oh.target_snr(fin, flat, grid, ratio=0.8) == 4.5
    assert oh.target_snr(np.array([]), flat, np.array([4.0])) == float("inf")


# ----------------------------------------------------------------- overlap-save segments
from oracle import stream as osm   # noqa: E402


@pytest.mark.parametrize("n,N", [(64, 64), (96, 64), (128, 64), (100, 64), (1000, 64), (65, 64)])
def test_segment_windows_partition_the_stream(n, N):
    seg = osm.segments(n, N)
    cover = np.zeros(n, dtype=int)
    for i, (s, lo, hi) in enumerate(seg):
        assert 0 <= s <= n - N and lo < hi
        assert s <= lo and hi <= s + N                       # a window lies inside its segment
        if 0 < i < len(seg) - 2:
            assert (lo, hi) == (s + N // 4, s + 3 * N // 4)  # the central half
        elif 0 < i == len(seg) - 2:                          # may end where the last (moved back) starts its half
            assert lo == s + N // 4 and hi <= s + 3 * N // 4
        cover[lo:hi] += 1
    assert np.all(cover == 1)
    assert [s for s, _, _ in seg[:-1]] == [i * N // 2 for i in range(len(seg) - 1)]
    assert seg[-1][0] == n - N


def test_stream_triggers_report_every_sample_once():
    n, N = 1000, 64
    strain = np.arange(n, dtype=np.float64)

    def everything(x):
        t = np.zeros(x.shape[0], dtype=om.TRIGGER_DTYPE)
        t["sample"] = np.arange(x.shape[0])
        t["snr"] = x                                        # the stream sample itself
        return t
    t = osm.stream_triggers(strain, N, everything)
    assert np.array_equal(t["sample"], np.arange(n))
    assert np.array_equal(t["snr"], strain)                 # shifted to the right sample
    with pytest.raises(ValueError):
        osm.segments(10, 64)


def test_thresholds_are_inclusive():
    """A bin whose |rho_avg| equals rho_I triggers, and a candidate whose
    reconstructed SNR equals thr2 is a final trigger of the reconstruction
    second stage (values chosen exact in binary)."""
    rho_avg = np.array([[0.0, 4.0, 3.5, 4.0 + 2 ** -40, -4.0]], dtype=complex)
    bins = oh.triggering_bins(rho_avg, 4.0)
    assert list(bins["bin"]) == [1, 3, 4]
    assert list(oh.triggering_bins(rho_avg, 4.0 + 2 ** -40)["bin"]) == [3]
    cand = np.zeros(3, dtype=om.TRIGGER_DTYPE)
    cand["tmpl"] = [0, 0, 1]
    cand["sample"] = [3, 9, 4]
    cand["snr"] = [6.0, 6.0 - 2 ** -40, 6.5]
    fin = oh.second_stage(cand, 6.0, "recon")
    assert list(zip(fin["tmpl"], fin["sample"])) == [(0, 3), (1, 4)]
    # the exact second stages on series with |rho| = thr2 exactly at some samples
    series = {0: np.array([0, 0, 0, 6.0j, 0, 0, 0, 0, 0, 6.0 - 2 ** -40, 0]),
              1: np.array([0, 0, 0, 0, -6.0, 0, 0, 0, 0, 0, 0])}
    rho_exact = lambda j: series[j].astype(complex)
    fin = oh.second_stage(cand, 6.0, "sparse", rho_exact)
    assert list(zip(fin["tmpl"], fin["sample"])) == [(0, 3), (1, 4)]
    fin = oh.second_stage(cand, 6.0, "full", rho_exact)
    assert list(zip(fin["tmpl"], fin["sample"])) == [(0, 3), (1, 4)]

