"""The adjoint at the differentiation workload's size: 512 s at 2048 Hz
(N = 2^20), 3.5PN templates with m1, m2 uniform in [1, 50], one basis of rank
256 in FP32, the trigger set S = the first-stage crossings |rho_RB| >= 5 of
the segment.

On a seeded subset of 32 templates that have crossings (S restricted to
them, seeds g uniform in [0.5, 2]), split over four tests that share the
module's fixtures (so that no single test runs for minutes):
  * rb_backward's loss, d|rho|^2/dC and d|rho|^2/d(strain) against the FP64
    oracle gradient (torch CPU autograd through direct sums at the trigger
    samples), 1e-4 relative to the largest entry;
  * FP64 central differences along 8 seeded directions in C (all entries of
    the 32 rows, step 1e-3) and 8 in the strain (step 1e-3 rms(s)) against
    both gradients; the loss is quadratic, so the differences are exact up to
    rounding, and beta is linear in the strain, so each strain direction
    needs one more evaluation of beta at the trigger samples."""
import sys
import time

import numpy as np
import pytest

from oracle import basis as ob
from oracle import grad as og
from oracle import mf as om
from paper_2110_13115_amd import inputs as gi
from paper_2110_13115_amd import rbmf

pytestmark = pytest.mark.gpu
NAME = "rb_512s_20000t"
T_BANK = 20000


def log(*a):
    print("[gpu-cfg5]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def cfg5():
    import torch
    wl = gi.WORKLOADS[NAME]
    t = time.time()
    bank_def = wl.bank()
    if T_BANK < wl.T:
        bank_def = bank_def.subset(np.sort(np.random.default_rng([13115, 5, 7]).choice(wl.T, T_BANK, replace=False)))
    psd = gi.psd_on_grid(wl.N, wl.fs)
    sig = lambda h: om.sigma(h, psd, wl.N, wl.fs, wl.f_low)
    strain, inj = gi.make_strain(wl, bank_def, sig, dtype=np.float32)
    ctx = rbmf.Context(0)
    bank = rbmf.Bank(ctx, wl.N, wl.fs, wl.f_low, psd, bank_def.T, bank_def.fill)
    log(f"bank of {bank_def.T} templates on N = {wl.N} in {time.time() - t:.1f} s")
    t = time.time()
    basis = rbmf.Basis(ctx, bank, rank=wl.rank, dtype="f32")
    log(f"basis K = {basis.K}, energy {basis.energy:.6f}, in {time.time() - t:.1f} s")
    sd = torch.from_numpy(strain).cuda()
    out = torch.empty((1 << 22, 4), dtype=torch.int32, device="cuda")
    n, _, st = rbmf.rb_filter(ctx, basis, bank, sd, wl.thr1, wl.thr1, stage2=rbmf.RB_STAGE2_RECON, out=out)
    S_all = out[:n].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1).copy()
    log(f"first-stage crossings at {wl.thr1}: {n}")
    yield wl, psd, strain, ctx, bank, basis, sd, S_all
    basis.close()
    bank.close()


@pytest.fixture(scope="module")
def at_size(cfg5):
    """The trigger set S on a seeded 32-template subset, rb_backward on it, and
    the FP64 oracle's loss and gradients."""
    wl, psd, strain, ctx, bank, basis, sd, S_all = cfg5
    rng = gi.rng_for(wl.cfg, gi.PURPOSE_FD)
    have = np.unique(S_all["tmpl"])
    assert len(have) >= 32
    sub = np.sort(rng.choice(have, size=32, replace=False))
    S = np.ascontiguousarray(S_all[np.isin(S_all["tmpl"], sub)])
    g = rng.uniform(0.5, 2.0, size=len(S)).astype(np.float32)
    t = time.time()
    loss, gC, gs = rbmf.rb_backward(ctx, basis, sd, S, seed=g)
    log(f"|S| = {len(S)} on 32 templates; rb_backward {1e3 * (time.time() - t):.1f} ms (host copies included)")
    V, c, _ = basis.export()
    C = np.conj(c)
    k_lo, _ = om.band_limits(wl.N, wl.fs, wl.f_low)
    w = ob.whiten_weights(psd, wl.N, wl.fs, wl.f_low)[k_lo:k_lo + V.shape[1]]
    s64 = strain.astype(np.float64)
    tmpl, samp, g64 = S["tmpl"], S["sample"], g.astype(np.float64)
    t = time.time()
    L, gC_ref, gs_ref = og.loss_and_grads(s64, C, V, w, k_lo, wl.fs, tmpl, samp, g64)
    log(f"oracle gradient in {time.time() - t:.1f} s; loss GPU {loss:.8g} oracle {L:.8g}")
    # beta at the distinct trigger samples only (beta is a function of the sample)
    uniq, inv = np.unique(samp, return_inverse=True)
    beta_of = lambda v: og.beta_at(v, V, w, k_lo, wl.fs, uniq)[:, inv]
    return dict(sub=sub, S=S, loss=loss, gC=gC, gs=gs, C=C, L=L, gC_ref=gC_ref, gs_ref=gs_ref, s64=s64,
                tmpl=tmpl, g64=g64, beta_of=beta_of, T=basis.T, N=wl.N)


def test_backward_at_size_matches_oracle(at_size):
    r = at_size
    assert abs(r["loss"] - r["L"]) <= 1e-4 * r["L"]
    eC = np.abs(r["gC"] - r["gC_ref"]).max() / np.abs(r["gC_ref"]).max()
    es = np.abs(r["gs"] - r["gs_ref"]).max() / np.abs(r["gs_ref"]).max()
    log(f"max |grad C - oracle| / max {eC:.2e}; max |grad s - oracle| / max {es:.2e}")
    assert eC <= 1e-4 and es <= 1e-4
    assert np.all(r["gC"][np.setdiff1d(np.arange(r["T"]), r["sub"])] == 0)


@pytest.fixture(scope="module")
def beta_s(at_size):
    r = at_size
    t = time.time()
    beta = r["beta_of"](r["s64"])
    log(f"beta at {beta.shape[1]} trigger samples in {time.time() - t:.1f} s")
    assert og.loss_from_beta(r["C"], beta, r["tmpl"], r["g64"]) == pytest.approx(r["L"], rel=1e-10)
    return beta


def test_fd_coefficient_directions(at_size, beta_s):
    """FP64 central differences along 8 seeded directions in C (all entries of
    the 32 rows, step 1e-3) against both gradients."""
    r = at_size
    C, tmpl, g64, gC_ref, gC = r["C"], r["tmpl"], r["g64"], r["gC_ref"], r["gC"]
    rng = np.random.default_rng([13115, 5, 71])
    eps = 1e-3
    for i in range(8):
        D = np.zeros_like(C)
        D[r["sub"]] = rng.standard_normal((32, C.shape[1])) + 1j * rng.standard_normal((32, C.shape[1]))
        fd = (og.loss_from_beta(C + eps * D, beta_s, tmpl, g64) - og.loss_from_beta(C - eps * D, beta_s, tmpl, g64)) / (2 * eps)
        an_ref = float(np.sum(gC_ref.real * D.real + gC_ref.imag * D.imag))
        an = float(np.sum(gC.real.astype(np.float64) * D.real + gC.imag.astype(np.float64) * D.imag))
        scale = float(np.sum(np.abs(gC_ref) * np.abs(D)))
        log(f"C direction {i}: fd {fd:.8g} oracle {an_ref:.8g} GPU {an:.8g}")
        assert abs(fd - an_ref) <= 1e-9 * scale
        assert abs(fd - an) <= 1e-4 * scale


@pytest.mark.parametrize("half", [0, 1])
def test_fd_strain_directions(at_size, beta_s, half):
    """FP64 central differences along 8 seeded strain directions (step
    1e-3 rms(s)), four per test: beta is linear in the strain, so each
    direction needs one more evaluation of beta at the trigger samples."""
    r = at_size
    C, tmpl, g64, gs_ref, gs = r["C"], r["tmpl"], r["g64"], r["gs_ref"], r["gs"]
    rng = np.random.default_rng([13115, 5, 72, half])
    rms = np.sqrt(np.mean(r["s64"] ** 2))
    for i in range(4):
        v = rms * rng.standard_normal(r["N"])
        bv = r["beta_of"](v)
        e = 1e-3
        fd = (og.loss_from_beta(C, beta_s + e * bv, tmpl, g64) - og.loss_from_beta(C, beta_s - e * bv, tmpl, g64)) / (2 * e)
        an_ref, an = float(gs_ref @ v), float(gs.astype(np.float64) @ v)
        scale = float(np.abs(gs_ref) @ np.abs(v))
        log(f"strain direction {4 * half + i}: fd {fd:.8g} oracle {an_ref:.8g} GPU {an:.8g}")
        assert abs(fd - an_ref) <= 1e-9 * scale
        assert abs(fd - an) <= 1e-4 * scale
