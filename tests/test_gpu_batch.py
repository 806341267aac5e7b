"""Batched search (segments of uneven length x sub-banks) against per-item
rb_filter and the FP64 oracle; hipGraph replays with refilled strain buffers
must reproduce eager results exactly on every replay."""
import sys

import numpy as np
import pytest

from oracle import basis as ob
from oracle import mf as om
from paper_2110_13115_amd import inputs as gi
from paper_2110_13115_amd import rbmf
from tests.helpers import compare_triggers

pytestmark = pytest.mark.gpu


def log(*a):
    print("[gpu-batch]", *a, file=sys.stderr, flush=True)


def strain_for(wl, bank_def, psd, seed):
    rng = np.random.default_rng([13115, 4, seed])
    T = bank_def.T
    inj = [gi.Injection(int(rng.integers(0, T)), float(rng.uniform(8, 12)), int(rng.integers(0, wl.N)),
                        float(rng.uniform(0, 2 * np.pi)))]
    w = gi.Workload(wl.name, 4000 + seed, wl.N, wl.fs, wl.f_low, T, wl.mmin, wl.mmax, wl.order)
    sig = lambda h: om.sigma(h, psd, wl.N, wl.fs, wl.f_low)
    s, _ = gi.make_strain(w, bank_def, sig, inj, dtype=np.float32)
    return s


@pytest.fixture(scope="module")
def batch():
    import torch
    ctx = rbmf.Context(0)
    setups = []
    for N in (8192, 16384, 32768):
        wl = gi.Workload(f"b{N}", 40, N, 2048.0, 25.0, 180, 2.0, 12.0, 7, subbanks=3)
        bank_def = wl.bank()
        psd = gi.psd_on_grid(N, wl.fs)
        bank = rbmf.Bank(ctx, N, wl.fs, wl.f_low, psd, wl.T, bank_def.fill)
        bases = rbmf.subbank_bases(ctx, bank, wl.bounds(), rank=[12, 20, 28], dtype="bf16")
        setups.append((wl, bank_def, psd, bank, bases))
    # 7 segments of uneven length: each item = (segment, bank of its length)
    order = [0, 2, 1, 2, 0, 1, 2]
    items, strains = [], []
    for i, si in enumerate(order):
        wl, bank_def, psd, bank, bases = setups[si]
        s = strain_for(wl, bank_def, psd, i)
        sd = torch.from_numpy(s).cuda()
        strains.append((s, sd, si))
        items.append((sd, bank, bases))
    yield ctx, setups, items, strains


def test_batch_matches_per_item_and_oracle(batch):
    ctx, setups, items, strains = batch
    eager, _ = rbmf.rb_filter_batch(ctx, items, 5.0, 6.0, use_graph=False)
    graph, st = rbmf.rb_filter_batch(ctx, items, 5.0, 6.0, use_graph=True)
    for i, (sd, bank, bases) in enumerate(items):
        one, _, _ = rbmf.rb_filter(ctx, bases, bank, sd, 5.0, 6.0)
        assert one.tobytes() == eager[i].tobytes(), i
        assert one.tobytes() == graph[i].tobytes(), i
    log("items", len(items), "final", [len(x) for x in graph], "stage1", st.n_stage1, "ms", st.ms[6])
    # oracle on two items
    for i in (0, 2):
        s, _, si = strains[i]
        wl, bank_def, psd, bank, bases = setups[si]
        H = bank_def.full()
        st_ = om.strain_tilde(s.astype(np.float64), wl.fs)
        rho = np.stack([om.complex_filter(st_, h, psd, wl.N, wl.fs, wl.f_low) / om.sigma(h, psd, wl.N, wl.fs, wl.f_low)
                        for h in H])
        compare_triggers(graph[i], rho, 6.0)


def test_graph_replays_with_new_data(batch):
    ctx, setups, items, strains = batch
    rbmf.rb_filter_batch(ctx, items, 5.0, 6.0, use_graph=True)     # (re)capture
    for rep in range(3):
        for i, (s, sd, si) in enumerate(strains):
            wl, bank_def, psd, bank, bases = setups[si]
            sd.copy_(__import__("torch").from_numpy(strain_for(wl, bank_def, psd, 100 * rep + i)).cuda())
        g, _ = rbmf.rb_filter_batch(ctx, items, 5.0, 6.0, use_graph=True)
        e, _ = rbmf.rb_filter_batch(ctx, items, 5.0, 6.0, use_graph=False)
        for i in range(len(items)):
            assert g[i].tobytes() == e[i].tobytes(), (rep, i)
        log("replay", rep, "ok", [len(x) for x in g])


def test_batch_sparse_stage2(batch):
    """Sparse exact second stage inside the batch (eager and graph) equals the
    per-item sparse rb_filter; its triggers are the full second stage's at the
    first-stage crossings (the low fixed ranks here leave reconstruction errors
    above thr2 - thr1, so the full stage may find more), with the same SNRs."""
    ctx, setups, items, strains = batch
    sp = rbmf.RB_STAGE2_SPARSE
    full, _ = rbmf.rb_filter_batch(ctx, items, 5.0, 6.0, use_graph=False)
    eager, _ = rbmf.rb_filter_batch(ctx, items, 5.0, 6.0, use_graph=False, stage2=sp)
    for rep in range(2):
        graph, _ = rbmf.rb_filter_batch(ctx, items, 5.0, 6.0, use_graph=True, stage2=sp)
        for i, (sd, bank, bases) in enumerate(items):
            assert graph[i].tobytes() == eager[i].tobytes(), (rep, i)
    missed = []
    for i, (sd, bank, bases) in enumerate(items):
        one, _, _ = rbmf.rb_filter(ctx, bases, bank, sd, 5.0, 6.0, stage2=sp)
        assert one.tobytes() == eager[i].tobytes(), i
        key_f = {(int(t), int(n)): k for k, (t, n) in enumerate(zip(full[i]["tmpl"], full[i]["sample"]))}
        idx = np.array([key_f.get((int(t), int(n)), -1) for t, n in zip(eager[i]["tmpl"], eager[i]["sample"])],
                       dtype=np.int64)
        # sparse triggers are full triggers, except within 1e-4 of the threshold (FFT vs direct sums)
        assert (eager[i]["snr"][idx < 0] < 6.0 * (1 + 1e-4)).all(), i
        np.testing.assert_allclose(eager[i]["snr"][idx >= 0], full[i]["snr"][idx[idx >= 0]], rtol=1e-4)
        missed.append(len(full[i]) - len(eager[i]))
    log("sparse batch ok", [len(x) for x in eager], "full-stage extras", missed)


def test_batch_sparse_against_oracle(batch):
    """The sparse second stage evaluates the exact SNR only at first-stage
    crossings, so its result is defined by the oracle and the first stage:
    the final triggers are the oracle's (|rho| >= thr2) at the samples where
    the first-stage series reaches thr1.  These bases store C and Z in BF16,
    so that decision is taken on the kernel's own BF16 reconstruction (read
    back with rb_debug_rho), which is checked against the FP64 reduced-basis
    SNR of the same bases to the BF16 bound of the precision test (3e-2 of
    max(|rho|, 1)).  Checked on every item (graph replay) outside the +-1e-3
    band of thr2 and a 1e-5 band of thr1 (the epilogue compares squares);
    the stage-1 recall (oracle final triggers kept) is reported, and it is
    below 1 here: the low fixed ranks leave reconstruction errors above
    thr2 - thr1."""
    ctx, setups, items, strains = batch
    thr1, thr2, band = 5.0, 6.0, 1e-3
    got, _ = rbmf.rb_filter_batch(ctx, items, thr1, thr2, use_graph=True, stage2=rbmf.RB_STAGE2_SPARSE)
    kept = total = 0
    for i, (_, sd, si) in enumerate(strains):
        wl, bank_def, psd, bank, bases = setups[si]
        s = sd.cpu().numpy()        # (an earlier test of the module refills the device strains)
        H = bank_def.full()
        st_ = om.strain_tilde(s.astype(np.float64), wl.fs)
        rho = np.abs(om.snr_rows(st_, H, psd, wl.N, wl.fs, wl.f_low))
        k_lo, _ = om.band_limits(wl.N, wl.fs, wl.f_low)
        d = ob.whitened_data(s.astype(np.float64), psd, wl.fs, wl.f_low)
        rb64 = np.zeros_like(rho)
        rbg = np.zeros_like(rho)
        for b in bases:
            V, c, _ = b.export()
            rb64[b.t0:b.t0 + b.T] = np.abs(ob.rb_snr(ob.basis_outputs(d, V, wl.N, k_lo), c))
            rbg[b.t0:b.t0 + b.T] = np.abs(rbmf.debug_rho(ctx, bank, sd, b))
        e = np.abs(rbg - rb64) / np.maximum(rb64, 1.0)
        assert e.max() <= 3e-2, f"item {i}: BF16 first stage {e.max():.3e} from the FP64 reduced basis"
        final = rho >= thr2
        in_band2 = np.abs(rho - thr2) <= band * thr2
        in_band1 = np.abs(rbg - thr1) <= 1e-5 * thr1
        want = final & (rbg >= thr1)
        G = np.zeros_like(final)
        G[got[i]["tmpl"], got[i]["sample"]] = True
        assert len(got[i]) == int(G.sum())
        sure = ~in_band1 & ~in_band2
        miss = want & ~G & sure
        extra = G & ~want & sure
        assert not miss.any(), (f"item {i}: {int(miss.sum())} oracle triggers at first-stage crossings missing, e.g. "
                                f"{[(int(j), int(n), rho[j, n], rbg[j, n], rb64[j, n]) for j, n in np.argwhere(miss)[:4]]}")
        assert not extra.any(), (f"item {i}: {int(extra.sum())} triggers the oracle does not define, e.g. "
                                 f"{[(int(j), int(n), rho[j, n], rbg[j, n]) for j, n in np.argwhere(extra)[:4]]}")
        ref = rho[got[i]["tmpl"], got[i]["sample"]]
        assert np.abs(got[i]["snr"] - ref).max(initial=0) <= 1e-4 * ref.max(initial=1)
        kept += int((G & final).sum())
        total += int(final.sum())
    log(f"sparse batch vs oracle: stage-1 recall {kept}/{total} of the oracle's final triggers")
    assert total > 0


@pytest.mark.parametrize("stage2", ["recon", "sparse"])
def test_batch_binned(batch, stage2):
    """The binned first stage in the batch (eager and graph replays) gives
    each item exactly the triggers of its own binned rb_filter call, at
    several bin widths (the items' grids need different FFT splits)."""
    ctx, setups, items, strains = batch
    mode = rbmf.RB_STAGE2_RECON if stage2 == "recon" else rbmf.RB_STAGE2_SPARSE
    for w, tb in ((4, 3.5), (8, 3.0)):
        eager, _ = rbmf.rb_filter_batch(ctx, items, 5.0, 6.0, use_graph=False, stage2=mode, bin_w=w, thr_bin=tb)
        graph, st = rbmf.rb_filter_batch(ctx, items, 5.0, 6.0, use_graph=True, stage2=mode, bin_w=w, thr_bin=tb)
        again, _ = rbmf.rb_filter_batch(ctx, items, 5.0, 6.0, use_graph=True, stage2=mode, bin_w=w, thr_bin=tb)
        for i, (sd, bank, bases) in enumerate(items):
            one, _, s1 = rbmf.rb_filter(ctx, bases, bank, sd, 5.0, 6.0, stage2=mode, bin_w=w, thr_bin=tb)
            assert one.tobytes() == eager[i].tobytes(), (w, i)
            assert one.tobytes() == graph[i].tobytes(), (w, i)
            assert one.tobytes() == again[i].tobytes(), (w, i)
        log("binned batch", stage2, w, [len(x) for x in graph], "bins", st.n_bins)
        assert sum(len(x) for x in graph) > 0


def test_batch_rejects_auto_stage2(batch):
    ctx, setups, items, strains = batch
    with pytest.raises(rbmf.RbError) as ei:
        rbmf.rb_filter_batch(ctx, items, 5.0, 6.0, use_graph=False, stage2=rbmf.RB_STAGE2_AUTO)
    assert ei.value.status == rbmf.RB_ERR_UNSUPPORTED


def test_batch_capacity(batch):
    ctx, setups, items, strains = batch
    with pytest.raises(rbmf.RbError) as ei:
        rbmf.rb_filter_batch(ctx, items, 3.0, 3.5, use_graph=True, cap_item=2)
    assert ei.value.status == rbmf.RB_ERR_CAPACITY


def test_batch_small_initial_buffers():
    """Trigger buffers that start at a few records (RBMF_TRIG_RECORDS) must
    grow through every cascading overflow (bins -> stage-1 records -> stage-2
    records) and give the same triggers as buffers that fit at once."""
    import os

    import torch
    wl = gi.Workload("b_small", 41, 8192, 2048.0, 25.0, 120, 2.0, 12.0, 7, subbanks=2)
    bank_def = wl.bank()
    psd = gi.psd_on_grid(wl.N, wl.fs)
    strains = [torch.from_numpy(strain_for(wl, bank_def, psd, 300 + i)).cuda() for i in range(3)]

    def run():
        ctx = rbmf.Context(0)
        bank = rbmf.Bank(ctx, wl.N, wl.fs, wl.f_low, psd, wl.T, bank_def.fill)
        bases = rbmf.subbank_bases(ctx, bank, wl.bounds(), rank=[16, 24], dtype="bf16")
        items = [(s, bank, bases) for s in strains]
        out = []
        for mode, w, tb in ((rbmf.RB_STAGE2_SPARSE, 4, 3.0), (rbmf.RB_STAGE2_RECON, 4, 3.0),
                            (rbmf.RB_STAGE2_FULL, 0, 0.0)):
            for graph in (False, True):
                r, st = rbmf.rb_filter_batch(ctx, items, 4.5, 5.0, use_graph=graph, stage2=mode, bin_w=w, thr_bin=tb)
                out.append(([x.tobytes() for x in r], int(st.n_stage1), int(st.n_bins)))
        for b in bases:
            b.close()
        bank.close()
        ctx.close()
        return out

    ref = run()
    old = os.environ.get("RBMF_TRIG_RECORDS")
    os.environ["RBMF_TRIG_RECORDS"] = "3"
    try:
        small = run()
    finally:
        if old is None:
            del os.environ["RBMF_TRIG_RECORDS"]
        else:
            os.environ["RBMF_TRIG_RECORDS"] = old
    assert all(n1 > 3 for _, n1, _ in ref), "the case must overflow the small buffers"
    for a, b in zip(ref, small):
        assert a == b
    log("small initial buffers ok", [(n1, nb) for _, n1, nb in ref])
