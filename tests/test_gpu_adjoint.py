"""GPU adjoint (correlation + reconstruction) against the FP64 oracle gradient
and central differences, the torch.autograd wrapper, and coefficient
refinement against its closed-form optimum."""
import sys

import numpy as np
import pytest

from oracle import basis as ob
from oracle import grad as og
from oracle import mf as om
from paper_2110_13115_amd import rbmf
from tests.helpers import Case

pytestmark = pytest.mark.gpu


def log(*a):
    print("[gpu-adj]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def adj():
    case = Case(N=8192, T=160, f_low=25.0, mrange=(3.0, 6.0), order=7, cfg=51, inj=((10, 14.0), (90, 9.0)))
    ctx = rbmf.Context(0)
    bank = rbmf.Bank(ctx, case.N, case.fs, case.f_low, case.psd, case.T, case.fill)
    basis = rbmf.Basis(ctx, bank, rank=24, dtype="f32")
    V, c, lam = basis.export()
    trig, _, _ = rbmf.rb_filter(ctx, basis, bank, case.strain, 4.0, 4.0)
    log("triggers", len(trig))
    yield case, ctx, bank, basis, V, c, trig
    basis.close()
    bank.close()


def oracle_inputs(case, V):
    k_lo, _ = om.band_limits(case.N, case.fs, case.f_low)
    w = ob.whiten_weights(case.psd, case.N, case.fs, case.f_low)[k_lo:k_lo + V.shape[1]]
    return k_lo, w


def test_rho_at_matches_reconstruction(adj):
    case, ctx, bank, basis, V, c, trig = adj
    rho = rbmf.rho_at(ctx, basis, case.strain, trig)
    k_lo, _ = oracle_inputs(case, V)
    d = ob.whitened_data(case.s64, case.psd, case.fs, case.f_low)
    beta = ob.basis_outputs(d, V, case.N, k_lo)
    ref = np.sum(np.conj(c[trig["tmpl"]]) * beta[:, trig["sample"]].T, axis=1)
    err = np.abs(rho - ref) / np.maximum(np.abs(ref), 1.0)
    log("rho_at err", err.max())
    assert err.max() <= 1e-4


def test_backward_matches_oracle_gradient_and_fd(adj):
    case, ctx, bank, basis, V, c, trig = adj
    rng = np.random.default_rng(3)
    sel = np.sort(rng.choice(len(trig), size=min(40, len(trig)), replace=False))
    S = np.ascontiguousarray(trig[sel])
    g = rng.uniform(0.5, 2.0, size=len(S)).astype(np.float32)
    loss, gC, gs = rbmf.rb_backward(ctx, basis, case.strain, S, seed=g)
    C = np.conj(c)
    k_lo, w = oracle_inputs(case, V)
    args = (C, V, w, k_lo, case.fs, S["tmpl"], S["sample"], g.astype(np.float64))
    L, gC_ref, gs_ref = og.loss_and_grads(case.s64, *args)
    log("loss", loss, L)
    assert abs(loss - L) <= 1e-4 * L
    eC = np.abs(gC - gC_ref).max() / np.abs(gC_ref).max()
    es = np.abs(gs - gs_ref).max() / np.abs(gs_ref).max()
    log("grad C err", eC, "grad s err", es)
    assert eC <= 1e-4 and es <= 1e-4
    rows = np.setdiff1d(np.arange(case.T), S["tmpl"])
    assert np.all(gC[rows] == 0)
    # central differences of the FP64 oracle loss (exact for a quadratic) on a few entries
    eps = 1e-3
    for (j, k) in [(int(S["tmpl"][0]), 0), (int(S["tmpl"][-1]), 5)]:
        Cp, Cm = C.copy(), C.copy()
        Cp[j, k] += eps
        Cm[j, k] -= eps
        fd = (og.loss(case.s64, Cp, *args[1:]) - og.loss(case.s64, Cm, *args[1:])) / (2 * eps)
        assert abs(fd - gC[j, k].real) <= 1e-4 * np.abs(gC_ref).max()
    v = np.random.default_rng([13115, 5, 3]).standard_normal(case.N)
    e = 1e-3 * np.sqrt(np.mean(case.s64 ** 2))
    fd = (og.loss(case.s64 + e * v, *args) - og.loss(case.s64 - e * v, *args)) / (2 * e)
    assert abs(fd - float(gs.astype(np.float64) @ v)) <= 1e-4 * abs(fd) + 1e-6 * np.abs(gs_ref).sum()
    # bitwise reproducible
    loss2, gC2, gs2 = rbmf.rb_backward(ctx, basis, case.strain, S, seed=g)
    assert gC2.tobytes() == gC.tobytes() and gs2.tobytes() == gs.tobytes()


def test_autograd_function_and_refinement(adj):
    import torch
    from paper_2110_13115_amd import autograd as ag
    case, ctx, bank, basis, V, c, trig = adj
    dev = torch.device("cuda")
    s = torch.from_numpy(case.strain).to(dev).requires_grad_(True)
    C = torch.from_numpy(np.conj(c).astype(np.complex64)).to(dev).requires_grad_(True)
    S = np.ascontiguousarray(trig[:25])
    p = ag.trigger_power(s, C, ctx, basis, S)
    p.sum().backward()
    loss, gC, gs = rbmf.rb_backward(ctx, basis, case.strain, S)
    assert abs(p.sum().item() - loss) <= 1e-5 * loss
    np.testing.assert_allclose(C.grad.cpu().numpy(), gC, rtol=0, atol=1e-6 * np.abs(gC).max())
    np.testing.assert_allclose(s.grad.cpu().numpy(), gs, rtol=0, atol=1e-6 * np.abs(gs).max())
    log("autograd ok")


def check_refinement(case_s64, psd, fs, f_low, N, basis, V, c, trig, ctx, strain, neighbours=8, tol=2e-4):
    """rb_refine against the oracle: the neighbours are a valid top set of
    |<c_j, c_l>| (FP64, ties within rounding may order either way), the
    refined |rho|^2 reaches the closed-form optimum of that span and never
    falls below the trigger's own."""
    from paper_2110_13115_amd import autograd as ag
    Cr, nbr, p0, p1 = ag.refine_coefficients(ctx, basis, strain, trig, neighbours=neighbours, iters=40)
    k_lo, _ = om.band_limits(N, fs, f_low)
    d = ob.whitened_data(case_s64, psd, fs, f_low)
    samples = np.unique(trig["sample"])
    f = np.arange(k_lo, k_lo + V.shape[1])
    # beta_k[n] by direct sums (Eq. basis_SNR) at the trigger samples: K x samples
    B = (d[None, :] * np.conj(V)) @ np.exp(2j * np.pi * np.outer(f, samples) / N)
    beta = {int(n): B[:, i] for i, n in enumerate(samples)}
    for i, (jg, n) in enumerate(zip(trig["tmpl"], trig["sample"])):
        j = int(jg) - basis.t0
        order, ov = og.nearest_neighbours(c, j)
        loc = nbr[i] - basis.t0
        kth = ov[order[neighbours - 1]]
        assert np.all(ov[loc] >= kth * (1 - 1e-6)), (i, ov[loc], kth)
        assert len(set(loc.tolist())) == neighbours and j not in loc
        idx = np.concatenate([[j], loc])
        copt, best = og.refine_optimum(beta[int(n)], c[idx])
        own = abs(np.sum(np.conj(c[j]) * beta[int(n)])) ** 2
        assert abs(p0[i] - own) <= 1e-4 * own
        assert p1[i] >= p0[i] * (1 - 1e-5)
        assert abs(p1[i] - best) <= tol * best, (i, p0[i], p1[i], best)
        got = abs(np.sum(Cr[i].astype(np.complex128) * beta[int(n)])) ** 2
        assert abs(got - best) <= tol * best
        assert abs(np.linalg.norm(Cr[i]) - 1.0) <= 1e-5
    return p0, p1


def test_refinement_whole_bank(adj):
    import torch
    case, ctx, bank, basis, V, c, trig = adj
    sd = torch.from_numpy(case.strain).cuda()
    top = trig[np.argsort(-trig["snr"], kind="stable")][:40]
    p0, p1 = check_refinement(case.s64, case.psd, case.fs, case.f_low, case.N, basis, V, c, top, ctx, sd)
    log("refined", len(top), "mean gain", float(np.mean(p1 / p0)))


def test_refinement_sub_bank(adj):
    """A basis of the second sub-bank (t0 > 0): trigger rows, neighbours and
    outputs are indexed in the basis's own range."""
    import torch
    case, ctx, bank, basis, V, c, trig = adj
    t0, t1 = 60, 160
    sub = rbmf.Basis(ctx, bank, rank=20, dtype="bf16", t0=t0, t1=t1)
    Vs, cs, _ = sub.export()
    sd = torch.from_numpy(case.strain).cuda()
    first = rbmf.Basis(ctx, bank, rank=20, dtype="f32", t0=0, t1=t0)
    tr, _, _ = rbmf.rb_filter(ctx, [first, sub], bank, case.strain, 4.0, 4.0)
    first.close()
    mine = tr[(tr["tmpl"] >= t0) & (tr["tmpl"] < t1)]
    assert len(mine) > 0
    top = mine[np.argsort(-mine["snr"], kind="stable")][:24]
    check_refinement(case.s64, case.psd, case.fs, case.f_low, case.N, sub, Vs, cs, top, ctx, sd, neighbours=5)
    outside = np.zeros(1, dtype=rbmf.TRIGGER_NP)
    outside["tmpl"] = t0 - 1
    with pytest.raises(rbmf.RbError) as ei:
        rbmf.refine(ctx, sub, sd, outside)
    assert ei.value.status == rbmf.RB_ERR_ARG
    loss, gC, gs = rbmf.rb_backward(ctx, sub, case.strain, top[:5])
    assert gC.shape == (t1 - t0, sub.K)
    sub.close()
