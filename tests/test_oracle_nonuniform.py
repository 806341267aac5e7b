"""Pins of the oracle's non-uniform-frequency PCA (oracle/nonuniform.py)
against closed forms, a different library route and invariants."""
import numpy as np
import pytest

from oracle import basis as ob
from oracle import mf as om
from oracle import nonuniform as onu
from paper_2110_13115_amd import inputs as gi


def test_zero_crossings_of_a_tone():
    # cos(2 pi f t0 + phi) vanishes at f_m = ((m + 1/2) pi - phi) / (2 pi t0)
    t0, phi = 3.7, 0.3
    f = np.linspace(10.0, 20.0, 200001)
    z = onu.zero_crossings(f, np.cos(2 * np.pi * f * t0 + phi))
    m = np.arange(0, 200)
    ref = ((m + 0.5) * np.pi - phi) / (2 * np.pi * t0)
    ref = ref[(ref > 10.0) & (ref < 20.0)]
    assert z.shape == ref.shape
    np.testing.assert_allclose(z, ref, rtol=0, atol=1e-9)


def test_zero_crossings_exact_zero_and_touch():
    f = np.array([0.0, 1.0, 2.0, 3.0, 4.0])
    assert onu.zero_crossings(f, np.array([1.0, 0.0, -1.0, -2.0, 3.0])).tolist() == [1.0, 3.0 + 2.0 / 5.0]
    # a zero first sample is the band edge, not a crossing
    assert onu.zero_crossings(f[:2], np.array([0.0, 1.0])).tolist() == []


def test_frequency_set_sparse_bins():
    # crossings every 1/(2 t0); per-bin spacing 1/(10 t0) above df_min
    t0 = 0.5
    f = np.linspace(30.0, 40.0, 100001)
    nodes = onu.frequency_set(f, np.cos(2 * np.pi * f * t0), per_bin=5, df_min=0.01)
    edges = [30.0] + list(onu.zero_crossings(f, np.cos(2 * np.pi * f * t0))) + [40.0]
    assert nodes.shape[0] == 5 * (len(edges) - 1) + 1
    assert nodes[0] == 30.0 and nodes[-1] == 40.0
    assert np.all(np.diff(nodes) > 0)
    for b, (a, e) in enumerate(zip(edges[:-1], edges[1:])):
        np.testing.assert_allclose(nodes[5 * b:5 * b + 5], a + np.arange(5) * (e - a) / 5, rtol=0, atol=1e-12)


def test_frequency_set_dense_is_the_uniform_grid():
    # crossings far denser than df_min: the set is the multiples of df_min
    df = 2048.0 / 8192
    f = 30.0 + np.arange(int(10 / 0.001) + 1) * 0.001
    nodes = onu.frequency_set(f, np.cos(2 * np.pi * f * 40.0), per_bin=5, df_min=df)
    k = np.arange(int(round(30.0 / df)), int(round(40.0 / df)) + 1)
    assert nodes.tolist() == (k * df).tolist()


def test_frequency_set_spacing_floor_mixed():
    # a chirp: dense crossings at low f, sparse at high f
    f = np.linspace(20.0, 200.0, 400001)
    h = np.cos(2 * np.pi * 300.0 / f)            # phase derivative falls as 1/f^2
    df_min = 1.0 / 16
    nodes = onu.frequency_set(f, h, per_bin=5, df_min=df_min)
    assert np.all(np.diff(nodes) > 0)
    edges = np.concatenate([[20.0], onu.zero_crossings(f, h), [200.0]])
    for a, b in zip(edges[:-1], edges[1:]):
        inside = nodes[(nodes >= a) & (nodes < b)]
        if (b - a) / 5 >= df_min:
            assert inside.shape[0] == 5
        else:
            assert np.all(np.abs(inside / df_min - np.round(inside / df_min)) < 1e-9)
        if inside.shape[0] > 1:
            assert np.min(np.diff(inside)) >= df_min * (1 - 1e-12)


def test_cell_weights_closed_forms():
    x = np.array([1.0, 1.5, 3.0, 3.25, 7.0])
    w = onu.cell_weights(x)
    np.testing.assert_allclose(w, [0.5, 1.0, 0.875, 2.0, 3.75])
    assert np.isclose(w.sum(), (x[-1] - x[0]) + (x[1] - x[0]) / 2 + (x[-1] - x[-2]) / 2)
    u = 0.25 * np.arange(40, 100)
    assert np.all(onu.cell_weights(u) == 0.25)


def _small_bank(T=24, N=8192, fs=2048.0, f_low=30.0):
    wl = gi.Workload("nu_pin", 77, N, fs, f_low, T, 5.0, 20.0, 7)
    return wl.bank(), gi.psd_on_grid(N, fs)


def test_uniform_set_reduces_to_the_uniform_basis():
    bank, psd = _small_bank()
    N, fs, fl = bank.N, bank.fs, bank.f_low
    H = bank.full()
    W, sig = ob.whitened_unit_templates(H, psd, N, fs, fl)
    k_lo, k_hi = om.band_limits(N, fs, fl)
    kk = np.arange(k_lo, k_hi + 1)
    nodes = kk * bank.df
    Vs, sig_s = onu.whitened_set_templates(H[:, k_lo:k_hi + 1], psd[k_lo:k_hi + 1], nodes)
    np.testing.assert_allclose(Vs, W, rtol=0, atol=1e-13)
    np.testing.assert_allclose(sig_s, sig, rtol=1e-13)
    # the covariance route (eigh of V^H V) against the SVD of V: eigenvalues
    # s^2 and the same rank-K projector
    Vu, _, s, K, e_u = ob.svd_basis(W, rank=10)
    U, lam, K2 = onu.covariance_basis(Vs, rank=10)
    assert K2 == K
    np.testing.assert_allclose(lam[:len(s)], s ** 2, rtol=0, atol=1e-10)
    np.testing.assert_allclose(U.conj().T @ U, Vu.conj().T @ Vu, rtol=0, atol=1e-9)
    # the whole preparation: identity interpolation, same coefficients' energy
    Vb, c, _, K3, e = onu.nonuniform_basis(W, H[:, k_lo:k_hi + 1], psd[k_lo:k_hi + 1], nodes, nodes, bank.df,
                                           rank=10)
    np.testing.assert_allclose(Vb.conj().T @ Vb, Vu.conj().T @ Vu, rtol=0, atol=1e-9)
    assert abs(e - e_u) < 1e-12
    np.testing.assert_allclose(np.sum(np.abs(c) ** 2, axis=1),
                               np.sum(np.abs(W @ Vu.conj().T) ** 2, axis=1), rtol=0, atol=1e-10)


def test_interpolation_is_exact_for_linear_densities_and_at_nodes():
    nodes = np.array([30.0, 30.7, 31.0, 33.2, 34.0, 36.5])
    om_ = onu.cell_weights(nodes)
    a, b = 1.5 - 0.5j, 0.25 + 2.0j
    U = ((a + b * nodes) * np.sqrt(om_))[None, :]
    fu = 30.0 + 0.125 * np.arange(0, 49)
    P = onu.interpolate_to_grid(U, nodes, fu, 0.125)
    np.testing.assert_allclose(P[0], np.sqrt(0.125) * (a + b * fu), rtol=1e-13)
    # at the nodes themselves the interpolant returns the node values
    Pn = onu.interpolate_to_grid(U, nodes, nodes, 0.125)
    np.testing.assert_allclose(Pn[0], np.sqrt(0.125) * (a + b * nodes), rtol=1e-13)


def test_set_norm_approximates_the_uniform_norm():
    # the cell rule on the non-uniform set estimates the same integral as the
    # uniform sum: sigma agrees to the quadrature error (a few per cent here,
    # mostly from the cut at f_ISCO falling inside a wide high-frequency
    # cell); a dropped cell weight would change it by orders of magnitude
    bank, psd = _small_bank()
    N, fs, fl = bank.N, bank.fs, bank.f_low
    k_lo, k_hi = om.band_limits(N, fs, fl)
    H = bank.full()
    _, sig = ob.whitened_unit_templates(H, psd, N, fs, fl)
    f_lo, f_hi = k_lo * bank.df, k_hi * bank.df
    j_ref = int(np.argmax(gi.tau0_array(bank.m1, bank.m2, fl)))
    href = lambda f: gi.taylorf2(f, bank.m1[j_ref], bank.m2[j_ref], 7, fl)
    fr, yr = onu.reference_samples(href, f_lo, f_hi, bank.df / 16)
    nodes = onu.frequency_set(fr, yr, 5, bank.df)
    assert nodes.shape[0] < (k_hi - k_lo + 1)
    Hn = np.stack([gi.taylorf2(nodes, bank.m1[j], bank.m2[j], 7, fl) for j in range(bank.T)])
    _, sig_n = onu.whitened_set_templates(Hn, gi.aligo_psd(nodes), nodes)
    np.testing.assert_allclose(sig_n, sig, rtol=5e-2)


def support_ends(bank, f_lo, f_hi):
    """The uniform frequencies on either side of every template's f_ISCO cut."""
    kc = np.array([np.floor(gi.f_isco(a, b) / bank.df) for a, b in zip(bank.m1, bank.m2)])
    return np.unique(np.concatenate([kc, kc + 1])) * bank.df


def test_frequency_set_merges_extra_nodes():
    f = np.linspace(30.0, 40.0, 100001)
    h = np.cos(2 * np.pi * f * 0.5)
    base = onu.frequency_set(f, h, 5, 0.01)
    got = onu.frequency_set(f, h, 5, 0.01, extra=[29.0, 30.0, 31.2345, base[3], 40.0, 41.0])
    assert got.tolist() == sorted(set(base.tolist()) | {31.2345})


def test_nonuniform_basis_energy_is_bounded_by_the_svd():
    # Ky Fan: no rank-K orthonormal basis keeps more energy than the SVD's;
    # the non-uniform one stays close (its loss is the interpolation error,
    # small once the f_ISCO cuts are nodes)
    bank, psd = _small_bank()
    N, fs, fl = bank.N, bank.fs, bank.f_low
    k_lo, k_hi = om.band_limits(N, fs, fl)
    H = bank.full()
    W, _ = ob.whitened_unit_templates(H, psd, N, fs, fl)
    f_lo, f_hi = k_lo * bank.df, k_hi * bank.df
    j_ref = int(np.argmax(gi.tau0_array(bank.m1, bank.m2, fl)))
    fr, yr = onu.reference_samples(lambda f: gi.taylorf2(f, bank.m1[j_ref], bank.m2[j_ref], 7, fl),
                                   f_lo, f_hi, bank.df / 16)
    nodes = onu.frequency_set(fr, yr, 5, bank.df, extra=support_ends(bank, f_lo, f_hi))
    Hn = np.stack([gi.taylorf2(nodes, bank.m1[j], bank.m2[j], 7, fl) for j in range(bank.T)])
    fu = np.arange(k_lo, k_hi + 1) * bank.df
    # the interpolated templates themselves: mismatch of the order the paper
    # quotes for its sampling (below 1e-4 typically, a few 1e-4 at worst here)
    Vs, _ = onu.whitened_set_templates(Hn, gi.aligo_psd(nodes), nodes)
    P = onu.interpolate_to_grid(Vs, nodes, fu, bank.df)
    mm = 1 - np.abs(np.sum(P * W.conj(), axis=1)) / np.linalg.norm(P, axis=1)
    assert np.median(mm) < 1e-4 and mm.max() < 1e-3
    for K in (4, 8, 12):
        _, _, s, _, e_u = ob.svd_basis(W, rank=K)
        Vb, c, lam, K2, e = onu.nonuniform_basis(W, Hn, gi.aligo_psd(nodes), nodes, fu, bank.df, rank=K)
        assert K2 == K
        np.testing.assert_allclose(Vb @ Vb.conj().T, np.eye(K), atol=1e-12)
        assert e <= e_u + 1e-12
        assert e > e_u - 5e-4, (K, e, e_u)
