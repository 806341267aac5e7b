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
import math
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


def injection_sigma(psd, N, fs, f_low):
    """sigma(h) = (4 df sum_band |h|^2 / Sn)^(1/2): the optimal SNR of a
    unit-amplitude injection, which sets the injection amplitudes.  Evaluated
    with the same numpy operations as the tests' input recipe, so that the
    benchmark's segment is bit-identical to theirs and to the stored oracle
    sweep's."""
    df = fs / N
    k_lo = int(math.ceil(f_low / df - 1e-9))
    m = np.zeros(N // 2 + 1, dtype=bool)
    m[k_lo:N // 2] = True
    return lambda h: float(np.sqrt(4.0 * df * np.sum(np.abs(h[m]) ** 2 / psd[m])))


def make_inputs(wl, rbmf, ctx, with_sigma=False):
    from paper_2110_13115_amd import inputs as gi
    t0 = time.time()
    bank_def = wl.bank()
    N, fs = wl.N, wl.fs
    psd = gi.psd_on_grid(N, fs)
    bank = rbmf.Bank(ctx, N, fs, wl.f_low, psd, wl.T, bank_def.fill)
    log(f"bank {wl.T} x {N // 2} bins uploaded in {time.time() - t0:.1f} s")

    sigma_of = injection_sigma(psd, N, fs, wl.f_low)
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


def zstage_traffic(vectors):
    """HBM bytes per headline step moved by the Z stage's two FFT passes, as
    measured with rocprofv3 FETCH_SIZE / WRITE_SIZE (copy-calibrated) and
    recorded in profiles/; None when fft.hip has changed since or the bases
    hold another number of vectors."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    prof = os.path.join(here, "profiles", "z_stage_traffic_rb_256s_2000t.md")
    src = os.path.join(here, "paper_2110_13115_amd", "csrc", "fft.hip")
    try:
        text = open(prof).read()
        sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"zstage_bytes_per_step=([0-9.e+]+) vectors=(\d+) fft_hip_sha1=([0-9a-f]+)", text)
    if not m or m.group(3) != sha or int(m.group(2)) != vectors:
        return None
    return float(m.group(1))


def stored_oracle(name, strain):
    """The FP64 oracle's whole-bank list of samples with |rho| >= 5.99 for this
    workload (tests/golden/oracle_<name>.txt, written from oracle/ only), when
    it was computed on exactly these strain bytes; else None."""
    import hashlib
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{name}.txt")
    if not os.path.exists(path):
        return None
    sha, rows = None, []
    for ln in open(path):
        if ln.startswith("# strain_sha1 "):
            sha = ln.split()[2]
        elif ln.strip() and not ln.startswith("#"):
            t, n, snr, _ = ln.split()
            rows.append((int(t), int(n), float(snr)))
    if sha != hashlib.sha1(np.ascontiguousarray(strain, dtype=np.float32).tobytes()).hexdigest():
        return None
    return np.array(rows, dtype=[("tmpl", np.int64), ("sample", np.int64), ("snr", np.float64)])


def oracle_agreement(trig, ora, thr, N, band=1e-3):
    """Final triggers against the oracle's at thr, outside the +-band (relative)
    around thr: the share of the oracle's triggers found (the stage-1 recall
    for the second stages that evaluate the exact SNR only at first-stage
    crossings), triggers the oracle does not have, and the largest relative
    |rho| difference of the common ones."""
    if ora is None:
        return None
    a = ora["snr"]
    key_o = ora["tmpl"] * N + ora["sample"]
    key_g = trig["tmpl"].astype(np.int64) * N + trig["sample"]
    in_band = (a >= thr * (1 - band)) & (a <= thr * (1 + band))
    must = key_o[(a >= thr) & ~in_band]
    found = np.isin(must, key_g)
    pos = np.searchsorted(key_o, key_g)
    hit = (pos < len(key_o)) & (key_o[np.minimum(pos, len(key_o) - 1)] == key_g)
    ok = hit.copy()
    ok[hit] = (a[pos[hit]] >= thr) | in_band[pos[hit]]
    rel = np.abs(trig["snr"][hit] - a[pos[hit]]) / a[pos[hit]]
    return {"oracle_triggers": int(len(must)), "found": int(found.sum()),
            "recall": float(found.mean()) if len(must) else 1.0,
            "extra": int((~ok).sum()), "max_rel_snr_err": float(rel.max()) if len(rel) else None}


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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, bank_def, psd, strain, budget_s=15.0):
    """The FP64 oracle on a bounded template sample: batches of 16 templates,
    one threaded inverse transform per row (scipy.fft, the oracle's worker
    count), thresholded at the final threshold."""
    from oracle import mf as om
    s64 = strain.astype(np.float64)
    st = om.strain_tilde(s64, wl.fs)
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s and n < wl.T:
        t1 = min(wl.T, n + 16)
        rho = om.snr_rows(st, bank_def.fill(n, t1, 0, wl.N // 2 + 1), psd, wl.N, wl.fs, wl.f_low)
        for i in range(t1 - n):
            om.triggers_of(n + i, rho[i], wl.thr2)
        n = t1
    dt = time.perf_counter() - t0
    return {"value": n * wl.seconds / dt, "unit": "template-s/s", "cores": om.WORKERS, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{n} of {wl.T} templates of the same segment (template generation included), full SNR "
                      f"series + threshold, {dt:.1f} s, scipy.fft with {om.WORKERS} workers, batches of 16"}


def binned_runs(ctx, wl, bank_def, bank, bases_by_dt, sd, out, mf_trig, t_mf, sigma_of, args, torch, ora=None):
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
    # the tuning quantities of Sec. IV.B over bin widths on the same tuning segment: the share f of
    # (template, bin) pairs whose averaged SNR reaches rho_I, the target SNR and the share of the
    # template method's triggers at thr2 that the binned search recovers
    sweep = {}
    for w in (2, 4, 8, 16):
        if wl.N // w < 256:
            continue
        _, rows = tuning.tune_bin_threshold(ctx, bases_by_dt["f32"], bank, st_dev, w, wl.thr1, wl.thr2,
                                            (2.0, 2.5, 3.0, 3.5, 4.0, 4.5))
        for r in rows:
            r["f"] = r["bins"] / (wl.T * (wl.N // w))
        sweep[str(w)] = rows
        log(f"tuning sweep w={w}: " + ", ".join(f"rho_I {r['thr_bin']}: f {r['f']:.2e} target {r['target_snr']:.2f} "
                                                f"recovered {r['kept_at_thr2']:.3f}" for r in rows))
    res["sweep_w"] = sweep
    fold_ok = wl.N // wl.bin_w >= 4096
    for dt, bs in bases_by_dt.items():
        runs = [(rbmf.RB_STAGE2_RECON, "recon", 0, 0), (rbmf.RB_STAGE2_SPARSE, "sparse", 0, 0)]
        if fold_ok:   # the averaged series from the templates (Sec. III.D), the basis for the fine stage
            runs.append((rbmf.RB_STAGE2_RECON, "fold_recon", 1, 0))
        if dt in ("bf16", "f16"):   # with the FP16 FFT intermediate option (rb_filter_opts.flags)
            runs.append((rbmf.RB_STAGE2_RECON, "recon_fp16_intermediate", 0, rbmf.RB_OPT_FP16_INTERMEDIATE))
        for mode, name, src, flags in runs:
            def call():
                n, _, st = rbmf.rb_filter(ctx, bs, bank, sd, wl.thr1, wl.thr2, stage2=mode, bin_w=wl.bin_w,
                                          thr_bin=thr_bin, bin_source=src, out=out, flags=flags)
                return n, st
            t, (n, st) = time_calls(call, args.steps, args.warmup, torch)
            tr = out[:n].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1)
            kept = sum(1 for a, b in zip(tr["tmpl"].tolist(), tr["sample"].tolist()) if (a, b) in mf_pairs)
            res[f"{dt}_{name}"] = {"value": seg / t, "ms_per_step": t * 1e3, "rb_over_mf": t_mf / t,
                                   "kept_of_mf": kept / max(1, len(mf_pairs)), "final": int(n),
                                   "vs_oracle": oracle_agreement(tr, ora, wl.thr2, wl.N),
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


def stream_runs(ctx, wl, bank, bases, args, torch, nseg_unique=4):
    """Overlap-save search (Sec. III.E: segments of N overlapping by N/2, each
    reporting its central half) of a stream of nseg_unique * N samples with
    the headline bank and bases: the strain is high-passed noise with four
    injections (on templates of the same masses on the stream's grid), in HBM
    before the timed calls.  Throughput counts unique stream seconds."""
    from paper_2110_13115_amd import inputs as gi
    from paper_2110_13115_amd import rbmf
    n = nseg_unique * wl.N
    t0 = time.time()
    psd_n = gi.psd_on_grid(n, wl.fs)
    f = np.arange(n // 2 + 1) * (wl.fs / n)
    psd_hp = np.where(f >= wl.f_low, psd_n, 0.0)   # (cutting raw noise would leak its low-frequency power)
    psd_hp[0] = 0.0
    st = gi.coloured_noise_tilde(psd_hp, n, wl.fs, gi.rng_for(wl.cfg, gi.PURPOSE_NOISE, 7))
    bank_n = gi.random_bank(wl.cfg, wl.T, n, wl.fs, wl.f_low, wl.mmin, wl.mmax, wl.order,
                            sort_tau0=wl.subbanks > 1, parent=wl.parent)
    sig_n = injection_sigma(psd_n, n, wl.fs, wl.f_low)
    rng = np.random.default_rng([13115, wl.cfg, 77])
    inj = []
    for k in range(4):
        j = int(rng.integers(0, wl.T))
        n0 = int(rng.integers(wl.N // 4, n - wl.N // 4))
        h = bank_n.fill(j, j + 1, 0, n // 2 + 1)[0]
        snr = float(rng.uniform(8.0, 12.0))
        st = gi.add_injection(st, h, snr / sig_n(h), n0, float(rng.uniform(0, 2 * np.pi)), n)
        inj.append((j, n0, snr))
    strain = gi.strain_from_tilde(st, n, wl.fs).astype(np.float32)
    sd = torch.from_numpy(strain).cuda()
    prep = time.time() - t0
    res = {}

    def call():
        tr, stt = rbmf.rb_filter_stream(ctx, bases, bank, sd, wl.thr1, wl.thr2, stage2=rbmf.RB_STAGE2_SPARSE)
        return tr, stt
    t, (tr, stt) = time_calls(call, args.steps, args.warmup, torch)
    hop = wl.N // 2
    nseg = -(-(n - wl.N) // hop) + 1
    found = sum(1 for j, n0, _ in inj if np.any((tr["tmpl"] == j) & (np.abs(tr["sample"] - n0) <= 2)))
    res = {"stream_samples": n, "stream_seconds": n / wl.fs, "segments": int(nseg), "N": wl.N,
           "ms_per_stream": t * 1e3, "value": wl.T * (n / wl.fs) / t, "unit": "template-s/s",
           "ms_per_segment": t * 1e3 / nseg, "final_triggers": int(len(tr)),
           "injections_found": f"{found}/{len(inj)}", "stage2": "sparse (exact SNR at the first-stage crossings)",
           "prep_s": prep, "note": "each stream sample is searched twice (N/2 overlap), so the rate is about "
                                   "(stream / N) / segments of the single-segment rate; the call returns its "
                                   "triggers in host memory"}
    log(f"stream of {n / wl.fs:.0f} s ({nseg} segments): {t * 1e3:.2f} ms, {res['value']:.3g} template-s/s, "
        f"{len(tr)} triggers, injections found {found}/{len(inj)}")
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


def precision_runs(args, torch):
    """The 10 000-template, 16 s workload (0PN, m1, m2 uniform in [1, 20],
    one basis keeping >= 0.999 of the energy): the first-stage series with C
    and Z stored in BF16 and FP16 (per-row power-of-two scales, FP32
    accumulation) against the same basis in FP32 on a seeded subset of 256
    templates, crossing agreement with FP32 over the whole bank at 5 and 6,
    and the search (thresholds 5 / 6, exact second stage at the first-stage
    crossings) per storage type against the template method.  The FP32 path
    itself is within 1.5e-5 of the FP64 oracle on this workload
    (tests/test_gpu_precision.py, which also checks the 16-bit paths against
    FP64 and against the FP64 product of the quantised operands)."""
    from paper_2110_13115_amd import inputs as gi
    from paper_2110_13115_amd import rbmf
    wl = gi.WORKLOADS["rb_16s_10000t"]
    ctx = rbmf.Context(0)
    bank_def, bank, psd, strain, inj = make_inputs(wl, rbmf, ctx)
    sd = torch.from_numpy(strain).cuda()
    out = torch.empty((1 << 22, 4), dtype=torch.int32, device="cuda")
    sub = torch.from_numpy(np.sort(np.random.default_rng([13115, 3, 9]).choice(wl.T, size=256, replace=False))).cuda()
    full = torch.empty((wl.T, wl.N), dtype=torch.complex64, device="cuda")
    t_mf, (n_mf, _, _) = time_calls(lambda: rbmf.mf_full(ctx, bank, sd, wl.thr2, out=out), args.steps, args.warmup,
                                    torch)
    mf_keys = out[:n_mf, :2].cpu().numpy().astype(np.int64)
    mf_keys = mf_keys[:, 0] * wl.N + mf_keys[:, 1]
    res = {"workload": wl.name, "N": wl.N, "templates": wl.T, "mf_full_ms_per_step": t_mf * 1e3}
    ref, ref_mask = None, {}
    for dt in ("f32", "bf16", "f16"):
        basis = rbmf.Basis(ctx, bank, rank=0, tol=wl.tol, dtype=dt)
        rbmf.debug_rho(ctx, bank, sd, basis, out=full)
        a = full.abs()
        r = {"K": basis.K, "energy": basis.energy}
        if dt == "f32":
            ref = full[sub].clone()
            for thr in (5.0, 6.0):
                ref_mask[thr] = a >= thr
        else:
            e = ((full[sub] - ref).abs() / torch.clamp(ref.abs(), min=1.0)).double()
            r["max_err_vs_f32"] = float(e.max())
            r["rms_err_vs_f32"] = float(torch.sqrt(torch.mean(e * e)))
            for thr in (5.0, 6.0):
                m = a >= thr
                r[f"crossings_{thr:g}"] = int(m.sum())
                r[f"crossings_{thr:g}_differ_from_f32"] = int((m ^ ref_mask[thr]).sum())
        if dt == "f32":
            for thr in (5.0, 6.0):
                r[f"crossings_{thr:g}"] = int(ref_mask[thr].sum())
        del a
        t, (n, _, st) = time_calls(lambda: rbmf.rb_filter(ctx, basis, bank, sd, wl.thr1, wl.thr2,
                                                          stage2=rbmf.RB_STAGE2_SPARSE, out=out),
                                   args.steps, args.warmup, torch)
        k = out[:n, :2].cpu().numpy().astype(np.int64)
        k = k[:, 0] * wl.N + k[:, 1]
        r.update({"ms_per_step": t * 1e3, "value": wl.T * wl.seconds / t, "final": int(n),
                  "final_triggers_equal_mf": bool(n == n_mf and np.array_equal(k, mf_keys)),
                  "recall_vs_mf": float(np.isin(mf_keys, k).mean()) if n_mf else 1.0,
                  "stage_ms": [round(x, 4) for x in st.ms[:7]]})
        res[dt] = r
        log(f"precision {dt}: K={basis.K} {r}")
        basis.close()
    del full
    bank.close()
    ctx.close()
    return res


def adjoint_runs(args, torch):
    """The differentiation workload: 20 000 3.5PN templates with m1, m2
    uniform in [1, 50], 512 s (N = 2^20), one FP32 basis of rank 256.  Basis
    build by subspace iteration and by block Lanczos; the search (5 / 6,
    exact second stage at the first-stage crossings); rb_backward of
    sum |rho|^2 over every first-stage crossing at 5 (d/dC and d/d(strain),
    device outputs)."""
    from paper_2110_13115_amd import inputs as gi
    from paper_2110_13115_amd import rbmf
    wl = gi.WORKLOADS["rb_512s_20000t"]
    ctx = rbmf.Context(0)
    t = time.time()
    bank_def, bank, psd, strain, inj = make_inputs(wl, rbmf, ctx)
    t_bank = time.time() - t
    sd = torch.from_numpy(strain).cuda()
    res = {"workload": wl.name, "N": wl.N, "templates": wl.T, "rank": wl.rank, "prep_bank_s": t_bank}
    bases = {}
    for solver in ("subspace", "lanczos"):
        torch.cuda.synchronize()
        t = time.time()
        bases[solver] = rbmf.Basis(ctx, bank, rank=wl.rank, dtype="f32", solver=solver)
        torch.cuda.synchronize()
        res[f"basis_{solver}_s"] = time.time() - t
        res[f"basis_{solver}_energy"] = bases[solver].energy
        log(f"config-5 basis ({solver}): K={bases[solver].K} energy {bases[solver].energy:.6f} in "
            f"{res[f'basis_{solver}_s']:.1f} s")
    bases["lanczos"].close()
    basis = bases["subspace"]
    out = torch.empty((1 << 22, 4), dtype=torch.int32, device="cuda")
    t, (n, _, st) = time_calls(lambda: rbmf.rb_filter(ctx, basis, bank, sd, wl.thr1, wl.thr2,
                                                      stage2=rbmf.RB_STAGE2_SPARSE, out=out),
                               args.steps, args.warmup, torch)
    res["rb_filter"] = {"ms_per_step": t * 1e3, "value": wl.T * wl.seconds / t, "final": int(n),
                        "stage_ms": [round(x, 4) for x in st.ms[:7]]}
    n, _, st1 = rbmf.rb_filter(ctx, basis, bank, sd, wl.thr1, wl.thr1, stage2=rbmf.RB_STAGE2_RECON, out=out)
    S = out[:n].clone()
    res["stage1_at_thr1"] = {"crossings": int(n), "stage_ms": [round(x, 4) for x in st1.ms[:7]]}
    log(f"config-5 first-stage crossings at {wl.thr1}: {n}, stage ms {[round(x, 3) for x in st1.ms[:7]]}")
    gC = torch.zeros((basis.T, basis.K), dtype=torch.complex64, device="cuda")
    gs = torch.zeros(wl.N, dtype=torch.float32, device="cuda")
    loss = [0.0]

    def back():
        loss[0] = rbmf.rb_backward(ctx, basis, sd, S, grad_C=gC, grad_strain=gs)[0]
    t, _ = time_calls(back, args.steps, args.warmup, torch)
    res["backward"] = {"triggers": int(n), "ms_per_call": t * 1e3, "loss": loss[0],
                       "outputs": "d|rho|^2/dC (20000 x 256 complex64) and d|rho|^2/d(strain) (2^20 floats)"}
    log(f"config-5 rb_backward over {n} first-stage crossings: {t * 1e3:.2f} ms")
    # coefficient refinement (Sec. II.A) of the 4096 loudest final triggers: 8 nearest
    # neighbours in coefficient space, 40 projected-ascent steps, device outputs
    nf, _, _ = rbmf.rb_filter(ctx, basis, bank, sd, wl.thr1, wl.thr2, stage2=rbmf.RB_STAGE2_SPARSE, out=out)
    fin = out[:nf].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1)
    sel = np.ascontiguousarray(fin[np.argsort(-fin["snr"], kind="stable")[:4096]])
    S_ref = torch.from_numpy(sel.view(np.int32).reshape(-1, 4).copy()).cuda()
    c_ref = torch.empty((len(sel), basis.K), dtype=torch.complex64, device="cuda")
    p_ref = torch.empty((len(sel), 2), dtype=torch.float32, device="cuda")
    nb_ref = torch.empty((len(sel), 8), dtype=torch.int32, device="cuda")
    t, _ = time_calls(lambda: rbmf.refine(ctx, basis, sd, S_ref, neighbours=8, iters=40, c_out=c_ref,
                                          nbr_out=nb_ref, p_out=p_ref), args.steps, args.warmup, torch)
    p = p_ref.cpu().numpy().astype(np.float64)
    gain = p[:, 1] / np.maximum(p[:, 0], 1e-30)
    res["refine"] = {"triggers": int(len(sel)), "neighbours": 8, "iters": 40, "ms_per_call": t * 1e3,
                     "snr2_gain_median": float(np.median(gain)), "snr2_gain_max": float(gain.max()),
                     "snr2_gain_min": float(gain.min())}
    log(f"config-5 rb_refine of the {len(sel)} loudest final triggers: {t * 1e3:.2f} ms, |rho|^2 gain median "
        f"{np.median(gain):.4f}, max {gain.max():.4f}")
    basis.close()
    bank.close()
    ctx.close()
    return res


def batch_runs(args, wname):
    """Batched search: segments of uneven length x tau0 sub-banks, one hipGraph
    replay per step (sparse exact second stage), beside the binned first stage
    with the paper's own second stage; recall of both against an exact search
    of every segment (the template method, mf_full, on the same GPU)."""
    import torch
    from paper_2110_13115_amd import inputs as gi
    from paper_2110_13115_amd import rbmf
    from paper_2110_13115_amd import tuning
    bw = gi.BATCH_WORKLOADS[wname]
    torch.cuda.init()
    ctx = rbmf.Context(0)
    lens = bw.segment_lengths()
    per_n = {}
    t0 = time.time()
    t_bank = t_basis = 0.0
    for N in bw.grids():
        bd = bw.bank_for(N)
        psd = gi.psd_on_grid(N, bw.fs)
        t = time.time()
        bank = rbmf.Bank(ctx, N, bw.fs, bw.f_low, psd, bw.T, bd.fill)
        t_bank += time.time() - t
        t = time.time()
        bases = rbmf.subbank_bases(ctx, bank, bw.bounds(), rank=list(bw.ranks), dtype="bf16")
        t_basis += time.time() - t
        per_n[N] = (bd, psd, bank, bases)
        log(f"batch grid N={N}: bank + {len(bases)} bases ready ({time.time() - t0:.1f} s)")
    items = []
    for i, N in enumerate(lens):
        bd, psd, bank, bases = per_n[N]
        s = bw.strain(i, N, bd, injection_sigma(psd, N, bw.fs, bw.f_low))
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
    # the exact search of every segment: the template method on the same GPU
    out = torch.empty((1 << 23, 4), dtype=torch.int32, device="cuda")
    exact = []
    t = time.time()

    def keys(tr):      # (template, sample) as one int64, samples < 2^21
        return np.asarray(tr["tmpl"], np.int64) * (1 << 21) + np.asarray(tr["sample"], np.int64)
    for sd, bank, _ in items:
        n, _, _ = rbmf.mf_full(ctx, bank, sd, bw.thr2, out=out)
        exact.append(keys(out[:n].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1)))
    t_mf = time.time() - t
    n_exact = sum(len(x) for x in exact)

    def kept_of(results):
        return int(sum(np.isin(e, keys(r)).sum() for r, e in zip(results, exact)))

    def extra_of(results):
        return int(sum((~np.isin(keys(r), e)).sum() for r, e in zip(results, exact)))
    # the binned first stage with the paper's own second stage, rho_I by the target-SNR
    # rule on an independent segment of the most frequent length
    Nt = max(set(lens), key=lens.count)
    bd, psd, bank_t, bases_t = per_n[Nt]
    st_t = torch.from_numpy(bw.strain(bw.nseg, Nt, bd, injection_sigma(psd, Nt, bw.fs, bw.f_low))).cuda()
    thr_bin, table = tuning.tune_bin_threshold(ctx, bases_t, bank_t, st_t, bw.bin_w, bw.thr1, bw.thr2,
                                               bw.thr_bin_grid)
    log(f"binned w={bw.bin_w}: rho_I = {thr_bin} from the tuning segment "
        f"{[(r['thr_bin'], r['target_snr']) for r in table]}")

    def replay_binned():
        return rbmf.rb_filter_batch(ctx, items, bw.thr1, bw.thr2, use_graph=True, cap_item=cap_item,
                                    stage2=rbmf.RB_STAGE2_RECON, bin_w=bw.bin_w, thr_bin=thr_bin)
    t_b, (res_b, st_b) = time_calls(replay_binned, args.steps, args.warmup, torch)
    binned = {"value": tsec / t_b, "ms_per_step": t_b * 1e3, "w": bw.bin_w, "thr_bin": thr_bin,
              "stage2": "recon", "recall_vs_exact": kept_of(res_b) / max(1, n_exact),
              "not_in_exact": extra_of(res_b), "bins": int(st_b.n_bins),
              "final_triggers": int(sum(len(x) for x in res_b)), "tuning_segment": table}
    log(f"binned batch: {t_b * 1e3:.1f} ms/step (sparse {t_g * 1e3:.1f}), kept {kept_of(res_b)}/{n_exact}")
    out_obj = {
        "workload": bw.name, "value": tsec / t_g, "unit": "template-s/s", "ms_per_step": t_g * 1e3,
        "steps": args.steps, "warmup": args.warmup, "dtype": "bf16",
        "segments": bw.nseg, "durations_s": list(bw.durations), "segment_samples": lens, "templates": bw.T,
        "subbanks": bw.subbanks, "ranks": list(bw.ranks), "thr1": bw.thr1, "thr2": bw.thr2,
        "stage2": "sparse (exact SNR at the first-stage crossings)", "graph_equals_eager": bool(same),
        "eager_ms_per_step": t_e * 1e3, "final_triggers": int(sum(len(x) for x in res)),
        "exact_triggers": n_exact, "recall_vs_exact": kept_of(res) / max(1, n_exact),
        "not_in_exact": extra_of(res), "exact_search_s": t_mf,
        "stage1_crossings": int(st.n_stage1), "refiltered": int(st.n_refiltered),
        "prep_s": prep_s, "prep_bank_s": t_bank, "prep_basis_s": t_basis, "binned_recon": binned,
    }
    log(f"batch: {t_g * 1e3:.1f} ms/step, recall vs the exact search {out_obj['recall_vs_exact']:.4f}")
    for _, _, bank, bases in per_n.values():
        for b in bases:
            b.close()
        bank.close()
    ctx.close()
    return out_obj


def run_batch(args, wname):
    o = batch_runs(args, wname)
    line = {"metric": "template-seconds filtered/s: batched RB search (hipGraph), 1 MI355X", "value": o["value"],
            "unit": "template-s/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": o["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16", "data": "synthetic", "config": {"workload": o["workload"]}, **o}
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
    ap.add_argument("--fp16-intermediate", action="store_true",
                    help="--headline-only: 16-bit bases with the FP16 FFT intermediate (RB_OPT_FP16_INTERMEDIATE)")
    ap.add_argument("--headline-dtype", default="f32", choices=["f32", "bf16", "f16", "bf16x3"],
                    help="storage type of the bases of --headline-only (for profiler runs)")
    ap.add_argument("--mf-only", action="store_true",
                    help="time only the mf_full comparator (for profiler runs)")
    ap.add_argument("--no-binned", action="store_true", help="skip the binned first stage runs")
    ap.add_argument("--no-stream", action="store_true", help="skip the overlap-save stream leg")
    ap.add_argument("--binned-only", action="store_true",
                    help="time only the binned search (RECON, FP32 and BF16) at --thr-bin (for profiler runs)")
    ap.add_argument("--thr-bin", type=float, default=4.0, help="rho_I of --binned-only")
    ap.add_argument("--dtypes", default="f32,bf16", help="storage types of --binned-only")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense sub-bank (paper regime) runs")
    ap.add_argument("--no-nonuniform", action="store_true", help="skip the non-uniform-frequency basis runs")
    ap.add_argument("--no-precision", action="store_true", help="skip the 10 000-template 16-bit precision runs")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the 20 000-template, rank-256 basis builds and rb_backward timing")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-segment batch (uneven lengths x four sub-banks, graph replay)")
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
    head_dt = args.headline_dtype if args.headline_only else "f32"
    bases = rbmf.subbank_bases(ctx, bank, wl.bounds(), rank=wl.sub_ranks(), tol=wl.tol, dtype=head_dt)
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

    ora = stored_oracle(wl.name, strain)
    log("stored oracle sweep: " + ("matches this segment" if ora is not None else "not available for this segment"))

    if args.mf_only:
        t_mf, (n_mf, _, st_mf) = time_calls(mf_step, args.steps, args.warmup, torch)
        print(json.dumps({"mf_full_ms_per_step": t_mf * 1e3, "triggers": int(n_mf),
                          "stage_ms": [round(x, 4) for x in st_mf.ms[:7]]}), flush=True)
        return

    # --- headline: rb_filter, FP32 (the workload's precision), exact second stage evaluated at the
    # first-stage crossings
    gemm_ms, z_ms, s1, nref, issued, s2_ms = [], [], [], [], [], []

    def rb_timed():
        n, _, st = rbmf.rb_filter(ctx, bases, bank, sd, wl.thr1, wl.thr2, stage2=rbmf.RB_STAGE2_SPARSE, out=out,
                                  flags=rbmf.RB_OPT_FP16_INTERMEDIATE if args.fp16_intermediate else 0)
        gemm_ms.append(st.ms[2])
        issued.append(st.gemm_mfma_flop)
        z_ms.append(st.ms[1])
        s1.append(st.n_stage1)
        nref.append(st.n_refiltered)
        s2_ms.append(st.ms[4])
        return n, st

    t_rb, (n_rb, st_rb) = time_calls(rb_timed, args.steps, args.warmup, torch)
    gemm_ms = gemm_ms[args.warmup:]
    z_ms = z_ms[args.warmup:]
    rb_trig = out[:n_rb].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1).copy()
    log(f"rb_filter {head_dt} (sparse stage 2): {t_rb * 1e3:.2f} ms/step, final {n_rb}, stage-1 {s1[-1]}, refiltered "
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
                                   "vs_oracle": oracle_agreement(tr_f2, ora, wl.thr2, wl.N),
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
                                   "vs_oracle": oracle_agreement(tr_au, ora, wl.thr2, wl.N),
                                   "stage_ms": [round(x, 4) for x in st_au.ms[:7]]}
    log(f"rb_filter f32 auto stage 2: {t_au * 1e3:.2f} ms/step")
    if not args.skip_16bit:
        for dt in ("bf16x3", "bf16", "f16"):
            b16 = rbmf.subbank_bases(ctx, bank, wl.bounds(), rank=wl.sub_ranks(), tol=wl.tol, dtype=dt)
            g16, i16 = [], []

            def f16():
                n, _, st = rbmf.rb_filter(ctx, b16, bank, sd, wl.thr1, wl.thr2, stage2=rbmf.RB_STAGE2_SPARSE,
                                          out=out)
                g16.append(st.ms[2])
                i16.append(st.gemm_mfma_flop)
                return n, st
            t16, (n16, st16) = time_calls(f16, args.steps, args.warmup, torch)
            tr16 = out[:n16].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1)
            ok16 = n16 == n_mf and np.array_equal(tr16[["tmpl", "sample"]], mf_trig[["tmpl", "sample"]])
            gm = float(np.mean(g16[args.warmup:]))
            fl16 = sum(8.0 * b.K * b.T * wl.N for b in b16)
            extra[f"rb_{dt}_sparse_stage2"] = {"value": seg / t16, "ms_per_step": t16 * 1e3,
                                 "rb_over_mf": t_mf / t16, "final_triggers_equal_mf": bool(ok16),
                                 "vs_oracle": oracle_agreement(tr16, ora, wl.thr2, wl.N),
                                 "gemm_ms": gm, "gemm_tflops": fl16 / (gm * 1e-3) / 1e12,
                                 "gemm_frac": fl16 / (gm * 1e-3) / 1e12 / PEAK[dt],
                                 # what the matrix cores ran (padding included, three BF16
                                 # products per split-BF16 one) against the 16-bit peak
                                 "gemm_mfma_issued_frac": float(np.mean(i16)) / (gm * 1e-3) / 1e12 / PEAK["bf16"],
                                 "stage_ms": [round(x, 4) for x in st16.ms[:7]]}
            log(f"rb_filter {dt}: {t16 * 1e3:.2f} ms/step, gemm {gm:.3f} ms")
            if dt in ("bf16", "f16"):
                # the FP16 FFT intermediate option (rb_filter_opts.flags): half the Z stage's
                # round-trip traffic, for an error floor that scales with the loudest signal
                def f16h():
                    n, _, st = rbmf.rb_filter(ctx, b16, bank, sd, wl.thr1, wl.thr2, stage2=rbmf.RB_STAGE2_SPARSE,
                                              out=out, flags=rbmf.RB_OPT_FP16_INTERMEDIATE)
                    return n, st
                th, (nh, sth) = time_calls(f16h, args.steps, args.warmup, torch)
                trh = out[:nh].cpu().numpy().view(rbmf.TRIGGER_NP).reshape(-1)
                okh = nh == n_mf and np.array_equal(trh[["tmpl", "sample"]], mf_trig[["tmpl", "sample"]])
                extra[f"rb_{dt}_sparse_stage2_fp16_intermediate"] = {
                    "value": seg / th, "ms_per_step": th * 1e3, "rb_over_mf": t_mf / th,
                    "final_triggers_equal_mf": bool(okh), "vs_oracle": oracle_agreement(trh, ora, wl.thr2, wl.N),
                    "stage_ms": [round(x, 4) for x in sth.ms[:7]]}
                log(f"rb_filter {dt} with the FP16 intermediate: {th * 1e3:.2f} ms/step")
            for b in b16:
                b.close()

    if not args.no_binned:
        b16 = rbmf.subbank_bases(ctx, bank, wl.bounds(), rank=wl.sub_ranks(), tol=wl.tol, dtype="bf16")
        extra["binned"] = binned_runs(ctx, wl, bank_def, bank, {"f32": bases, "bf16": b16}, sd, out, mf_trig,
                                      t_mf, sigma_of, args, torch, ora)
        for b in b16:
            b.close()
    if not args.no_nonuniform:
        extra["nonuniform_basis"] = nonuniform_runs(ctx, wl, bank_def, bank, sd, out, mf_trig, s1[-1],
                                                    prep_basis_s, args, torch)
    if not args.no_stream:
        extra["stream"] = stream_runs(ctx, wl, bank, bases, args, torch)
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
            # the three-product kernel needs 3/4 of the 8KTN count on the MFMA units, so the
            # algorithmic rate can pass the peak; this is the rate of what the units ran
            # (padding rows included) against the same peak
            "mfma_issued": {"flop_per_step": float(np.mean(issued)),
                            "achieved": float(np.mean(issued)) / (gm * 1e-3) / 1e12,
                            "frac": float(np.mean(issued)) / (gm * 1e-3) / 1e12 / PEAK["f32"]},
            "traffic_unit": "HBM bytes per sub-bank GEMM launch (its one or two dispatches; mean of the "
                            "ten; profiles/recon_gemm_f32_traffic_rb_256s_2000t.md)"}
    # the HBM-bound stages: correlation + inverse FFTs writing Z (every basis vector), and the
    # template method's passes (every template), in algorithmic bytes
    df = wl.fs / wl.N
    k_lo = int(math.ceil(wl.f_low / df - 1e-9))
    nb = wl.N // 2 - k_lo
    zm = float(np.mean(z_ms))
    zbytes = sum(b.K for b in bases) * (8.0 * nb + 8.0 * wl.N)
    ztraffic = zstage_traffic(sum(b.K for b in bases)) if wl.name == "rb_256s_2000t" else None
    roof_z = {"bound": "hbm", "achieved": zbytes / (zm * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": zbytes / (zm * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": ztraffic,
              # measured bytes (algorithmic + the intermediate) over the same time: how close the
              # passes run to the HBM peak in what they actually move
              "traffic_frac": (ztraffic / (zm * 1e-3) / 1e9 / HBM_PEAK_GBS) if ztraffic else None,
              "traffic_unit": "HBM bytes per step, both passes (profiles/z_stage_traffic_rb_256s_2000t.md)",
              "kernel": "k_pass1 (correlation prologue, column FFTs) + k_pass2 (row FFTs, planar FP32 Z)",
              "per_step": f"sum over the {sum(b.K for b in bases)} basis vectors of 8*nb (basis row read, nb = "
                          f"{nb}) + 8*N (FP32 Z row written) = {zbytes:.4g} B; the four-step intermediate "
                          f"between the passes adds 16*N B per vector that is not counted",
              "avg_ms_per_step": zm}
    kh = np.minimum(np.floor(np.array([gi.f_isco(a, b) for a, b in zip(bank_def.m1, bank_def.m2)]) / df),
                    wl.N // 2 - 1)
    mfbytes = float(np.sum(8.0 * (kh - k_lo + 1)))
    mf_pass_ms = float(st_mf.ms[4])
    roof_mf = {"bound": "hbm", "achieved": mfbytes / (mf_pass_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": mfbytes / (mf_pass_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "kernel": "mf_full: k_pass1 (correlation prologue on each template's support) + k_pass2 "
                         "(threshold epilogue)",
               "per_step": f"sum over templates of 8 * support bins = {mfbytes:.4g} B (nothing written but "
                           f"triggers); the four-step intermediate adds 16*N B per template that is not counted",
               "avg_ms_per_step": mf_pass_ms}
    # the sparse exact second stage reads each refiltered template's support once per group
    # of at most 8 of its crossings (algorithmic: once per template)
    s2m = float(np.mean(s2_ms[args.warmup:]))
    sup = (kh - k_lo + 1).astype(np.float64)
    s2bytes = float(np.mean(nref[args.warmup:])) * 8.0 * float(np.mean(sup))
    roof_s2 = {"bound": "hbm", "achieved": s2bytes / (s2m * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": s2bytes / (s2m * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "kernel": "k_sparse_exact (direct frequency sums at the first-stage crossings)",
               "per_step": f"refiltered templates x 8 * mean support bins = {s2bytes:.4g} B (every template of this "
                           f"bank spans {int(sup.min())}-{int(sup.max())} bins); the data spectrum, read by every "
                           f"workgroup from L2, is not counted",
               "avg_ms_per_step": s2m}
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
        "mf_full": {"value": seg / t_mf, "ms_per_step": t_mf * 1e3, "triggers": int(n_mf),
                    "vs_oracle": oracle_agreement(mf_trig, ora, wl.thr2, wl.N)},
        "final_triggers_vs_oracle": oracle_agreement(rb_trig, ora, wl.thr2, wl.N),
        "rb_over_mf": t_mf / t_rb,
        "final_triggers_equal_mf": bool(same),
        "max_rel_snr_diff_vs_mf": max_rel,
        "stage1_crossings": int(s1[-1]),
        "refiltered_fraction": nref[-1] / wl.T,
        "stage_ms": [round(x, 4) for x in st_rb.ms[:7]],
        "prep_basis_s": prep_basis_s,
        "roofline": roof,
        "roofline_z_stage": roof_z,
        "roofline_mf_full": roof_mf,
        "roofline_sparse_stage2": roof_s2,
        "cpu_baseline": cpu,
        **extra,
    }
    for b in bases:
        b.close()
    bank.close()
    ctx.close()
    if not args.no_precision:
        line["precision"] = precision_runs(args, torch)
    if not args.no_adjoint:
        line["adjoint"] = adjoint_runs(args, torch)
    if not args.no_batch:
        line["batch_64seg"] = batch_runs(args, "batch_64seg")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
