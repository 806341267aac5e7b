"""Benchmark: hierarchical reduced-basis search of one 256 s segment on one GPU.

Workload (synthetic, seeded): 2000-template 3.5PN TaylorF2 bank with m1, m2
uniform in [1, 3] Msun, f_low = 20 Hz, fs = 2048 Hz, N = 2^19 (256 s), in
coloured Gaussian noise from the analytic Advanced-LIGO fit with 8 off-bank
injections at SNR 5..12; the bank is split along tau0 into 10 sub-banks of
200 templates with one FP64 basis per sub-bank keeping >= 0.999 of its energy;
first stage threshold 5.0, final threshold 6.0.

A step is one rb_filter call (strain FFT, correlation + basis IFFTs, MFMA
reconstruction with the fused first-stage threshold, exact second stage of
the selected templates at their first-stage crossings, sort and output).  The
full per-template matched filter (mf_full) of the same segment is timed beside
it as the comparator, with the full second stage and the 16-bit / split-BF16
reconstructions as further variants.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f32": 157.3, "bf16": 2500.0, "f16": 2500.0}      # dense MFMA TFLOP/s, MI355X
# split-BF16 (hi + lo) products issue three BF16 MFMAs per FP32-equivalent product
PEAK["bf16x3"] = PEAK["bf16"] / 3
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_inputs(wl, rbmf, ctx, with_sigma=False):
    from paper_2110_13115_amd import inputs as gi
    t0 = time.time()
    bank_def = wl.bank()
    N, fs = wl.N, wl.fs
    psd = gi.psd_on_grid(N, fs)
    bank = rbmf.Bank(ctx, N, fs, wl.f_low, psd, wl.T, bank_def.fill)
    log(f"bank {wl.T} x {N // 2} bins uploaded in {time.time() - t0:.1f} s")

    def sigma_of(h):   # the library's own FP64 sigma of a one-template bank
        b = rbmf.Bank(ctx, N, fs, wl.f_low, psd, 1, lambda t0, t1, k0, k1: h[None, k0:k1])
        s = b.info()[3][0]
        b.close()
        return s

    strain, inj = gi.make_strain(wl, bank_def, sigma_of, dtype=np.float32)
    if with_sigma:
        return bank_def, bank, psd, strain, inj, sigma_of
    return bank_def, bank, psd, strain, inj


def gemm_traffic():
    """HBM bytes per launch of the FP32 reconstruction GEMM, as measured with
    rocprofv3 FETCH_SIZE / WRITE_SIZE (copy-calibrated) and recorded in
    profiles/; None when the kernel source has changed since."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    prof = os.path.join(here, "profiles", "recon_gemm_f32_traffic_rb_256s_2000t.md")
    src = os.path.join(here, "paper_2110_13115_amd", "csrc", "gemm.hip")
    try:
        text = open(prof).read()
        sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch=([0-9.e+]+) launches=\d+ gemm_hip_sha1=([0-9a-f]+)", text)
    if not m or m.group(2) != sha:
        return None
    return float(m.group(1))


def time_calls(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def cpu_baseline(wl, bank_def, psd, strain, budget_s=15.0):
    """The FP64 oracle (single-threaded numpy FFTs) on a bounded template sample."""
    from oracle import mf as om
    s64 = strain.astype(np.float64)
    st = om.strain_tilde(s64, wl.fs)
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s and n < wl.T:
        H = bank_def.fill(n, min(wl.T, n + 8), 0, wl.N // 2 + 1)
        for h in H:
            z = om.complex_filter(st, h, psd, wl.N, wl.fs, wl.f_low) / om.sigma(h, psd, wl.N, wl.fs, wl.f_low)
            om.triggers_of(0, z, wl.thr2)
        n += H.shape[0]
    dt = time.perf_counter() - t0
    return {"value": n * wl.seconds / dt, "unit": "template-s/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} of {wl.T} templates of the same segment, full SNR series + threshold, "
                      f"{dt:.1f} s, numpy pocketfft (1 thread)"}


def binned_runs(ctx, wl, bank_def, bank, bases_by_dt, sd, out, mf_trig, t_mf, sigma_of, args, torch):
    """The binned first stage (Sec. III.C) at bin width wl.bin_w: rho_I chosen
    by the target-SNR rule (Eq. target_snr_criteria, ratio 0.99, final
    threshold thr2) on an independent noise segment of the same bank, then the
    RECON and SPARSE second stages timed on the benchmark segment, with the
    share of the template method's final triggers they keep."""
    from paper_2110_13115_amd import inputs as gi
    from paper_2110_13115_amd import rbmf, tuning
    seg = wl.T * wl.seconds
    strain_t, _ = gi.make_strain(wl, bank_def, sigma_of, dtype=np.float32, realisation=1)
    st_dev = torch.from_numpy(strain_t).cuda()
    thr_bin, table = tuning.tune_bin_threshold(ctx, bases_by_dt["f32"], bank, st_dev, wl.bin_w, wl.thr1, wl.thr2,
                                               wl.thr_bin_grid)
    log(f"binned w={wl.bin_w}: rho_I = {thr_bin} from the tuning segment "
        f"{[(r['thr_bin'], r['target_snr']) for r in table]}")
    mf_pairs = set(zip(mf_trig["tmpl"].tolist(), mf_trig["sample"].tolist()))
    res = {"w": wl.bin_w, "thr_bin": thr_bin, "tuning_segment": table}
    fold_ok = wl.N // wl.bin_w >= 4096
    for dt, bs in bases_by_dt.items():
        runs = [(rbmf.RB_STAGE2_RECON, "recon", 0), (rbmf.RB_STAGE2_SPARSE, "sparse", 0)]
        if fold_ok:   # the averaged series from the templates (Sec. III.D), the basis for the fine stage
            runs.append((rbmf.RB_STAGE2_RECON, "fold_recon", 1))
        for mode, name, src in runs:
            def call():
                n, _, st = rbmf.rb_filter(ctx, bs, bank, sd, wl.thr1, wl.thr2, stage2=mode, bin_w=wl.bin_w,
                                          thr_bin=thr_bin, bin_source=src, out=out)
                return n, st
            t, (n, st) = time_calls(call, args.steps, args.warmup, torch)
            tr = out[:n].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1)
            kept = sum(1 for a, b in zip(tr["tmpl"].tolist(), tr["sample"].tolist()) if (a, b) in mf_pairs)
            res[f"{dt}_{name}"] = {"value": seg / t, "ms_per_step": t * 1e3, "rb_over_mf": t_mf / t,
                                   "kept_of_mf": kept / max(1, len(mf_pairs)), "final": int(n),
                                   "bins": int(st.n_bins), "candidates": int(st.n_stage1),
                                   "stage_ms": [round(x, 4) for x in st.ms]}
            log(f"binned {dt} {name}: {t * 1e3:.2f} ms/step (mf {t_mf * 1e3:.2f}), kept {kept}/{len(mf_pairs)} "
                f"of the template method's triggers, bins {st.n_bins}, stage ms {[round(x, 3) for x in st.ms]}")
    return res


def nonuniform_runs(ctx, wl, bank_def, bank, sd, out, mf_trig, s1_uniform, prep_uniform_s, args, torch):
    """Sub-bank bases by PCA on the non-uniform frequency set (zero crossings
    of the longest template, five frequencies per bin, spacing floor = the
    grid step, f_ISCO cuts as extra nodes), interpolated onto the grid: set
    size, build time beside the uniform bases', kept energy, and the search
    with them (FP32, sparse exact second stage)."""
    from paper_2110_13115_amd import inputs as gi
    from paper_2110_13115_amd import rbmf
    df = bank_def.df
    k_lo, k_hi = int(np.ceil(wl.f_low / df - 1e-9)), wl.N // 2 - 1
    j = bank_def.longest()
    f = k_lo * df + (df / 8) * np.arange(8 * (k_hi - k_lo) + 1, dtype=np.float64)
    t0 = time.time()
    nodes = rbmf.nonuniform_freqs(f, bank_def.fill_at(j, j + 1, f)[0].real, 5, df, bank_def.support_ends())
    t_set = time.time() - t0
    psd_n = gi.aligo_psd(nodes)
    b = wl.bounds()
    fill_s = [0.0]

    def fill_at(t0, t1, fr):        # the host template generator, timed apart from the build
        t = time.time()
        h = bank_def.fill_at(t0, t1, fr)
        fill_s[0] += time.time() - t
        return h
    t0 = time.time()
    nu = [rbmf.Basis.nonuniform(ctx, bank, nodes, psd_n, fill_at, rank=r, tol=wl.tol, dtype="f32",
                                t0=b[i], t1=b[i + 1]) for i, r in enumerate(wl.sub_ranks())]
    t_nu = time.time() - t0
    log(f"non-uniform set: {len(nodes)} of {k_hi - k_lo + 1} band bins ({t_set:.2f} s); bases K={[x.K for x in nu]} "
        f"in {t_nu:.2f} s, of which {fill_s[0]:.2f} s host template generation (uniform {prep_uniform_s:.2f} s)")

    def call():
        n, _, st = rbmf.rb_filter(ctx, nu, bank, sd, wl.thr1, wl.thr2, stage2=rbmf.RB_STAGE2_SPARSE, out=out)
        return n, st
    t, (n, st) = time_calls(call, args.steps, args.warmup, torch)
    tr = out[:n].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1)
    same = n == len(mf_trig) and np.array_equal(tr[["tmpl", "sample"]], mf_trig[["tmpl", "sample"]])
    res = {"nodes": int(len(nodes)), "band_bins": int(k_hi - k_lo + 1), "set_s": t_set, "build_s": t_nu,
           "host_template_s": fill_s[0],
           "uniform_build_s": prep_uniform_s, "ranks": [x.K for x in nu],
           "min_energy": min(x.energy for x in nu), "ms_per_step": t * 1e3,
           "value": wl.T * wl.seconds / t, "final_triggers_equal_mf": bool(same),
           "stage1_crossings": int(st.n_stage1), "stage1_crossings_uniform_basis": int(s1_uniform)}
    log(f"rb_filter with non-uniform bases: {t * 1e3:.2f} ms/step, final == mf: {same}")
    for x in nu:
        x.close()
    return res


def paper_regime(args, torch):
    """The paper's regime: one dense tau0 sub-bank (6250 templates of a
    200 000-template bank, K ~ 40 at 0.999 energy), 128 s: the template method,
    the unbinned search and the binned search on the same GPU."""
    from paper_2110_13115_amd import inputs as gi
    from paper_2110_13115_amd import rbmf
    wl = gi.WORKLOADS["rb_128s_6250t_dense"]
    ctx = rbmf.Context(0)
    bank_def, bank, psd, strain, inj, sigma_of = make_inputs(wl, rbmf, ctx, with_sigma=True)
    seg = wl.T * wl.seconds
    bases = {dt: rbmf.subbank_bases(ctx, bank, wl.bounds(), rank=wl.sub_ranks(), tol=wl.tol, dtype=dt)
             for dt in ("f32", "bf16")}
    sd = torch.from_numpy(strain).cuda()
    out = torch.empty((1 << 21, 4), dtype=torch.int32, device="cuda")
    t_mf, (n_mf, _, _) = time_calls(lambda: rbmf.mf_full(ctx, bank, sd, wl.thr2, out=out), args.steps,
                                    args.warmup, torch)
    mf_trig = out[:n_mf].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1).copy()
    log(f"dense sub-bank: mf_full {t_mf * 1e3:.2f} ms/step, {n_mf} triggers, K = {[b.K for b in bases['f32']]}")
    t_rb, (n_rb, _, st_rb) = time_calls(
        lambda: rbmf.rb_filter(ctx, bases["f32"], bank, sd, wl.thr1, wl.thr2, stage2=rbmf.RB_STAGE2_SPARSE,
                               out=out), args.steps, args.warmup, torch)
    tr = out[:n_rb].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1)
    same = n_rb == n_mf and np.array_equal(tr[["tmpl", "sample"]], mf_trig[["tmpl", "sample"]])
    res = {"workload": wl.name, "N": wl.N, "templates": wl.T, "ranks": [b.K for b in bases["f32"]],
           "mf_full": {"value": seg / t_mf, "ms_per_step": t_mf * 1e3, "triggers": int(n_mf)},
           "rb_f32_sparse_unbinned": {"value": seg / t_rb, "ms_per_step": t_rb * 1e3,
                                      "final_triggers_equal_mf": bool(same),
                                      "stage_ms": [round(x, 4) for x in st_rb.ms[:7]]}}
    log(f"dense sub-bank: rb_filter f32 unbinned {t_rb * 1e3:.2f} ms/step")
    res["binned"] = binned_runs(ctx, wl, bank_def, bank, bases, sd, out, mf_trig, t_mf, sigma_of, args, torch)
    for bs in bases.values():
        for b in bs:
            b.close()
    bank.close()
    ctx.close()
    return res


def run_batch(args, wname):
    """Batched search: segments of uneven length x tau0 sub-banks, one hipGraph
    replay per step."""
    import torch
    from paper_2110_13115_amd import inputs as gi
    from paper_2110_13115_amd import rbmf
    bw = gi.BATCH_WORKLOADS[wname]
    torch.cuda.init()
    ctx = rbmf.Context(0)
    lens = bw.segment_lengths()
    per_n = {}
    t0 = time.time()
    for N in bw.grids():
        bd = bw.bank_for(N)
        psd = gi.psd_on_grid(N, bw.fs)
        bank = rbmf.Bank(ctx, N, bw.fs, bw.f_low, psd, bw.T, bd.fill)
        bases = rbmf.subbank_bases(ctx, bank, bw.bounds(), rank=list(bw.ranks), dtype="bf16")
        per_n[N] = (bd, psd, bank, bases)
        log(f"grid N={N}: bank + {len(bases)} bases ready ({time.time() - t0:.1f} s)")
    items = []
    for i, N in enumerate(lens):
        bd, psd, bank, bases = per_n[N]

        def sigma_of(h, N=N, psd=psd):
            b = rbmf.Bank(ctx, N, bw.fs, bw.f_low, psd, 1, lambda t0, t1, k0, k1: h[None, k0:k1])
            s = b.info()[3][0]
            b.close()
            return s
        s = bw.strain(i, N, bd, sigma_of)
        items.append((torch.from_numpy(s).cuda(), bank, bases))
    prep_s = time.time() - t0
    cap_item = 1 << 20
    sp = rbmf.RB_STAGE2_SPARSE

    def replay():
        return rbmf.rb_filter_batch(ctx, items, bw.thr1, bw.thr2, use_graph=True, cap_item=cap_item, stage2=sp)

    def eager_run():
        return rbmf.rb_filter_batch(ctx, items, bw.thr1, bw.thr2, use_graph=False, cap_item=cap_item, stage2=sp)
    eager, _ = eager_run()
    graph, _ = replay()
    same = all(a.tobytes() == b.tobytes() for a, b in zip(eager, graph))
    log(f"batch prepared in {prep_s:.1f} s; graph == eager: {same}")
    t_g, (res, st) = time_calls(replay, args.steps, args.warmup, torch)
    t_e, _ = time_calls(eager_run, max(1, args.steps // 2), 0, torch)
    tsec = sum(bw.T * n / bw.fs for n in lens)
    # the binned first stage with the paper's own second stage, rho_I by the target-SNR
    # rule on an independent segment of the most frequent length
    from paper_2110_13115_amd import tuning
    Nt = max(set(lens), key=lens.count)
    bd, psd, bank_t, bases_t = per_n[Nt]

    def sigma_t(h):
        b = rbmf.Bank(ctx, Nt, bw.fs, bw.f_low, psd, 1, lambda t0, t1, k0, k1: h[None, k0:k1])
        s = b.info()[3][0]
        b.close()
        return s
    st_t = torch.from_numpy(bw.strain(bw.nseg, Nt, bd, sigma_t)).cuda()
    thr_bin, table = tuning.tune_bin_threshold(ctx, bases_t, bank_t, st_t, bw.bin_w, bw.thr1, bw.thr2,
                                               bw.thr_bin_grid)
    log(f"binned w={bw.bin_w}: rho_I = {thr_bin} from the tuning segment "
        f"{[(r['thr_bin'], r['target_snr']) for r in table]}")

    def replay_binned():
        return rbmf.rb_filter_batch(ctx, items, bw.thr1, bw.thr2, use_graph=True, cap_item=cap_item,
                                    stage2=rbmf.RB_STAGE2_RECON, bin_w=bw.bin_w, thr_bin=thr_bin)
    t_b, (res_b, st_b) = time_calls(replay_binned, args.steps, args.warmup, torch)
    exact = sum(len(x) for x in res)
    kept = sum(len(set(zip(a["tmpl"].tolist(), a["sample"].tolist())) & set(zip(b["tmpl"].tolist(),
                                                                              b["sample"].tolist())))
               for a, b in zip(res, res_b))
    binned = {"value": tsec / t_b, "ms_per_step": t_b * 1e3, "w": bw.bin_w, "thr_bin": thr_bin,
              "stage2": "recon", "kept_of_exact": kept / max(1, exact), "bins": int(st_b.n_bins),
              "final_triggers": int(sum(len(x) for x in res_b)), "tuning_segment": table}
    log(f"binned batch: {t_b * 1e3:.1f} ms/step (exact {t_g * 1e3:.1f}), kept {kept}/{exact}")
    line = {
        "metric": "template-seconds filtered/s: batched RB search (hipGraph), 1 MI355X",
        "value": tsec / t_g, "unit": "template-s/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_g * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": bw.name, "segments": bw.nseg, "durations_s": list(bw.durations),
                   "segment_samples": lens, "templates": bw.T, "subbanks": bw.subbanks, "ranks": list(bw.ranks),
                   "thr1": bw.thr1, "thr2": bw.thr2, "stage2": "sparse exact"},
        "eager_ms_per_step": t_e * 1e3, "graph_equals_eager": bool(same),
        "final_triggers": int(sum(len(x) for x in res)), "stage1_crossings": int(st.n_stage1),
        "refiltered": int(st.n_refiltered), "prep_s": prep_s, "binned_recon": binned,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rb_256s_2000t")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-16bit", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the headline rb_filter call (for profiler runs)")
    ap.add_argument("--mf-only", action="store_true",
                    help="time only the mf_full comparator (for profiler runs)")
    ap.add_argument("--no-binned", action="store_true", help="skip the binned first stage runs")
    ap.add_argument("--binned-only", action="store_true",
                    help="time only the binned search (RECON, FP32 and BF16) at --thr-bin (for profiler runs)")
    ap.add_argument("--thr-bin", type=float, default=4.0, help="rho_I of --binned-only")
    ap.add_argument("--dtypes", default="f32,bf16", help="storage types of --binned-only")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense sub-bank (paper regime) runs")
    ap.add_argument("--no-nonuniform", action="store_true", help="skip the non-uniform-frequency basis runs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run one plain device-to-device copy of MIB MiB and exit (scales HBM byte "
                         "counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 18            # float32 elements in MIB MiB
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": n * 4}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (--gpus {args.gpus} requested); the path "
              "shards by segment / sub-bank / template with no exchange on the forward path, but no "
              "multi-GPU run is made here.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2110_13115_amd import inputs as gi
    from paper_2110_13115_amd import rbmf

    if args.workload in gi.BATCH_WORKLOADS:
        run_batch(args, args.workload)
        return
    wl = gi.WORKLOADS[args.workload]
    torch.cuda.init()
    ctx = rbmf.Context(0)
    bank_def, bank, psd, strain, inj, sigma_of = make_inputs(wl, rbmf, ctx, with_sigma=True)
    t0 = time.time()
    bases = rbmf.subbank_bases(ctx, bank, wl.bounds(), rank=wl.sub_ranks(), tol=wl.tol, dtype="f32")
    prep_basis_s = time.time() - t0
    ranks = [b.K for b in bases]
    log(f"bases K={ranks} min energy={min(b.energy for b in bases):.6f} built in {prep_basis_s:.1f} s")
    sd = torch.from_numpy(strain).cuda()
    cap = 1 << 20
    out = torch.empty((cap, 4), dtype=torch.int32, device="cuda")
    seg = wl.T * wl.seconds

    res = {}

    def mf_step():
        return rbmf.mf_full(ctx, bank, sd, wl.thr2, out=out)

    if args.binned_only:
        res = {}
        for dt in args.dtypes.split(","):
            bs = bases if dt == "f32" else rbmf.subbank_bases(ctx, bank, wl.bounds(), rank=wl.sub_ranks(),
                                                              tol=wl.tol, dtype=dt)
            def call():
                n, _, st = rbmf.rb_filter(ctx, bs, bank, sd, wl.thr1, wl.thr2, stage2=rbmf.RB_STAGE2_RECON,
                                          bin_w=wl.bin_w, thr_bin=args.thr_bin, out=out)
                return n, st
            t, (n, st) = time_calls(call, args.steps, args.warmup, torch)
            res[dt] = {"ms_per_step": t * 1e3, "final": int(n), "bins": int(st.n_bins),
                       "stage_ms": [round(x, 4) for x in st.ms]}
        print(json.dumps({"workload": wl.name, "w": wl.bin_w, "thr_bin": args.thr_bin, **res}), flush=True)
        return

    if args.mf_only:
        t_mf, (n_mf, _, st_mf) = time_calls(mf_step, args.steps, args.warmup, torch)
        print(json.dumps({"mf_full_ms_per_step": t_mf * 1e3, "triggers": int(n_mf),
                          "stage_ms": [round(x, 4) for x in st_mf.ms[:7]]}), flush=True)
        return

    # --- headline: rb_filter, FP32 (the workload's precision), exact second stage evaluated at the
    # first-stage crossings
    gemm_ms, s1, nref = [], [], []

    def rb_timed():
        n, _, st = rbmf.rb_filter(ctx, bases, bank, sd, wl.thr1, wl.thr2, stage2=rbmf.RB_STAGE2_SPARSE, out=out)
        gemm_ms.append(st.ms[2])
        s1.append(st.n_stage1)
        nref.append(st.n_refiltered)
        return n, st

    t_rb, (n_rb, st_rb) = time_calls(rb_timed, args.steps, args.warmup, torch)
    gemm_ms = gemm_ms[args.warmup:]
    rb_trig = out[:n_rb].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1).copy()
    log(f"rb_filter f32 (sparse stage 2): {t_rb * 1e3:.2f} ms/step, final {n_rb}, stage-1 {s1[-1]}, refiltered "
        f"{nref[-1]}, stage ms {[round(x, 3) for x in st_rb.ms[:7]]}")

    if args.headline_only:
        print(json.dumps({"rb_filter_ms_per_step": t_rb * 1e3, "gemm_ms": float(np.mean(gemm_ms)),
                          "stage_ms": [round(x, 4) for x in st_rb.ms[:7]], "ranks": ranks}), flush=True)
        return
    # --- comparator: full matched filter on the same GPU
    t_mf, (n_mf, _, st_mf) = time_calls(mf_step, args.steps, args.warmup, torch)
    mf_trig = out[:n_mf].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1).copy()
    log(f"mf_full: {t_mf * 1e3:.2f} ms/step, {n_mf} triggers")
    same = (n_rb == n_mf and np.array_equal(rb_trig[["tmpl", "sample"]], mf_trig[["tmpl", "sample"]]))
    max_rel = float(np.max(np.abs(rb_trig["snr"] - mf_trig["snr"]) / mf_trig["snr"])) if same and n_rb else None

    extra = {}
    # the second stage as a full matched filter of every crossing template (same final triggers)
    def rb_full2():
        n, _, st = rbmf.rb_filter(ctx, bases, bank, sd, wl.thr1, wl.thr2, stage2=rbmf.RB_STAGE2_FULL, out=out)
        return n, st
    t_f2, (n_f2, st_f2) = time_calls(rb_full2, args.steps, args.warmup, torch)
    tr_f2 = out[:n_f2].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1)
    ok_f2 = n_f2 == n_mf and np.array_equal(tr_f2[["tmpl", "sample"]], mf_trig[["tmpl", "sample"]])
    extra["rb_f32_full_stage2"] = {"value": seg / t_f2, "ms_per_step": t_f2 * 1e3,
                                   "final_triggers_equal_mf": bool(ok_f2),
                                   "stage_ms": [round(x, 4) for x in st_f2.ms[:7]]}
    log(f"rb_filter f32 full stage 2: {t_f2 * 1e3:.2f} ms/step")

    # per-template choice: full matched filter for templates with many crossings, direct sums otherwise
    def rb_auto():
        n, _, st = rbmf.rb_filter(ctx, bases, bank, sd, wl.thr1, wl.thr2, stage2=rbmf.RB_STAGE2_AUTO, out=out)
        return n, st
    t_au, (n_au, st_au) = time_calls(rb_auto, args.steps, args.warmup, torch)
    tr_au = out[:n_au].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1)
    ok_au = n_au == n_mf and np.array_equal(tr_au[["tmpl", "sample"]], mf_trig[["tmpl", "sample"]])
    extra["rb_f32_auto_stage2"] = {"value": seg / t_au, "ms_per_step": t_au * 1e3,
                                   "final_triggers_equal_mf": bool(ok_au),
                                   "stage_ms": [round(x, 4) for x in st_au.ms[:7]]}
    log(f"rb_filter f32 auto stage 2: {t_au * 1e3:.2f} ms/step")
    if not args.skip_16bit:
        for dt in ("bf16x3", "bf16", "f16"):
            b16 = rbmf.subbank_bases(ctx, bank, wl.bounds(), rank=wl.sub_ranks(), tol=wl.tol, dtype=dt)
            g16 = []

            def f16():
                n, _, st = rbmf.rb_filter(ctx, b16, bank, sd, wl.thr1, wl.thr2, stage2=rbmf.RB_STAGE2_SPARSE,
                                          out=out)
                g16.append(st.ms[2])
                return n, st
            t16, (n16, st16) = time_calls(f16, args.steps, args.warmup, torch)
            tr16 = out[:n16].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1)
            ok16 = n16 == n_mf and np.array_equal(tr16[["tmpl", "sample"]], mf_trig[["tmpl", "sample"]])
            gm = float(np.mean(g16[args.warmup:]))
            fl16 = sum(8.0 * b.K * b.T * wl.N for b in b16)
            extra[f"rb_{dt}_sparse_stage2"] = {"value": seg / t16, "ms_per_step": t16 * 1e3, "final_triggers_equal_mf": bool(ok16),
                                 "gemm_ms": gm, "gemm_tflops": fl16 / (gm * 1e-3) / 1e12,
                                 "gemm_frac": fl16 / (gm * 1e-3) / 1e12 / PEAK[dt],
                                 "stage_ms": [round(x, 4) for x in st16.ms[:7]]}
            log(f"rb_filter {dt}: {t16 * 1e3:.2f} ms/step, gemm {gm:.3f} ms")
            for b in b16:
                b.close()

    if not args.no_binned:
        b16 = rbmf.subbank_bases(ctx, bank, wl.bounds(), rank=wl.sub_ranks(), tol=wl.tol, dtype="bf16")
        extra["binned"] = binned_runs(ctx, wl, bank_def, bank, {"f32": bases, "bf16": b16}, sd, out, mf_trig,
                                      t_mf, sigma_of, args, torch)
        for b in b16:
            b.close()
    if not args.no_nonuniform:
        extra["nonuniform_basis"] = nonuniform_runs(ctx, wl, bank_def, bank, sd, out, mf_trig, s1[-1],
                                                    prep_basis_s, args, torch)
    if not args.no_dense:
        extra["paper_regime"] = paper_regime(args, torch)

    gm = float(np.mean(gemm_ms))
    flops = sum(8.0 * b.K * b.T * wl.N for b in bases)
    achieved = flops / (gm * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK["f32"], "unit": "TFLOP/s",
            "frac": achieved / PEAK["f32"], "traffic": gemm_traffic(),
            "kernel": "k_recon_f32_3m / k_recon_f32 / k_recon_f32_w64 (rho = C Z complex GEMM on FP32 MFMA "
                      "32x32x2, variant autotuned per sub-bank)",
            "flop_convention": "8*K*T*N per sub-bank (a complex multiply-add = 8 real flop); the three-product "
                               "(Gauss) kernel issues 6*K*T*N of it on the MFMA units, the realified ones 8*K*T*N",
            "per_step": f"sum over sub-banks of 8*K_m*T_m*N = {flops:.4g} flop", "avg_ms_per_step": gm,
            "traffic_unit": "HBM bytes per sub-bank GEMM launch (its one or two dispatches; mean of the "
                            "ten; profiles/recon_gemm_f32_traffic_rb_256s_2000t.md)"}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, bank_def, psd, strain)
        log(f"cpu baseline {cpu['value']:.4g} template-s/s")
    line = {
        "metric": "template-seconds filtered/s: RB vs full MF, 1 MI355X, <=1e-3 rel SNR err",
        "value": seg / t_rb,
        "unit": "template-s/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_rb * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "N": wl.N, "fs": wl.fs, "f_low": wl.f_low, "templates": wl.T,
                   "seconds": wl.seconds, "subbanks": wl.subbanks, "ranks": ranks,
                   "min_energy": min(b.energy for b in bases), "thr1": wl.thr1,
                   "thr2": wl.thr2, "injections": len(inj), "stage2": "sparse exact"},
        "mf_full": {"value": seg / t_mf, "ms_per_step": t_mf * 1e3, "triggers": int(n_mf)},
        "rb_over_mf": t_mf / t_rb,
        "final_triggers_equal_mf": bool(same),
        "max_rel_snr_diff_vs_mf": max_rel,
        "stage1_crossings": int(s1[-1]),
        "refiltered_fraction": nref[-1] / wl.T,
        "stage_ms": [round(x, 4) for x in st_rb.ms[:7]],
        "prep_basis_s": prep_basis_s,
        "roofline": roof,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(line), flush=True)
    for b in bases:
        b.close()
    bank.close()
    ctx.close()


if __name__ == "__main__":
    main()
