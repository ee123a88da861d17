"""Benchmark of the correlation hot path on one MI355X.

Workload (the focus-view refinement configuration): an 80x32x20 ensemble with
M = 100 members (FP32, seeded smoothed-Gaussian field with 3 planted
correlated blobs), regions A = x in [0,32) and B = x in [48,80) of 32x32x20 =
20,480 points each. One step is one pass of the focus view:

  * Pearson: every one of the 4.19e8 (pA, pB) pairs, standardised and
    contracted on MFMA (FP16 operands, FP32 accumulation) with the region
    maximum fused into the epilogue (corr_region_max, exhaustive);
  * KSG mutual information (k = 10) on a uniform 1e6-pair sample of A x B,
    with its region maximum fused (corr_region_max over the sample list).

value = (Pearson pairs + KSG pairs) per second of step time, inputs resident
in HBM: the throughput of one whole step. The JSON line also carries a
roofline entry for the step's dominant kernel (KSG; timed live with HIP
events on the stream it runs on), the CPU oracle's rate on a bounded sample
of the same workload, and `per_measure`: point pairs/s of each measure at
M = 100 (this field) and M = 1000 (the 128x128x32 FP16 large-ensemble field:
4e6 random pairs for Pearson and KSG on fields prepared once, and the
exhaustive contraction of two 16^3 regions), each leg with its own roofline
(MFMA for the contractions, HBM for the pair-list gather, VALU for KSG),
oracle baseline and error against the FP64 oracle, and the context view
(batched BOS over the 3828 region pairs of the 352x256x20 field) with its
error against the exhaustive maxima and the oracle BOS on 30 pairs.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_PEARSON = 20480 * 20480
N_KSG = 1_000_000
M = 100
# published FP32 vector rate (157.3 TFLOP/s) in FMA lane-ops/s: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz
VALU_LANE_OPS_PER_S = 256 * 4 * 32 * 2.4e9
MFMA_F16_PEAK = 2.5e15
LDS_BYTES_PER_S = 256 * 128 * 2.4e9  # CUs x LDS bytes per clock x clock
HBM_PEAK = 8.0e12


KSG_SOURCE = os.path.join(ROOT, "paper_2309_03308_amd", "csrc", "ksg.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ksg_focus_1e6_pmc.txt")
AGG_SOURCE = os.path.join(ROOT, "paper_2309_03308_amd", "csrc", "aggregate.hip")
PAIRS_SOURCE = os.path.join(ROOT, "paper_2309_03308_amd", "csrc", "pairs.hip")
PAIRS_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pearson_pairs_gather_m1000_pmc.txt")
KSG1000_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ksg_m1000_4e6_pmc.txt")
AGG_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "block_means_f2_180x640x704x64_pmc.txt")


def source_hash(path):
    import hashlib
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_value(name, summary=TRAFFIC_FILE, source=KSG_SOURCE, key="ksg_source_sha256"):
    """A figure of a committed counter summary, or None when missing or stale."""
    try:
        vals = {}
        for line in open(summary):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
        if vals.get(key) != source_hash(source):
            return None
        return float(vals[name])
    except (OSError, KeyError, ValueError):
        return None


def measured_traffic(summary=TRAFFIC_FILE, source=KSG_SOURCE, key="ksg_source_sha256"):
    """HBM bytes per launch of a kernel from a committed counter summary, or None.

    The summary records FETCH_SIZE and WRITE_SIZE per dispatch of the kernel,
    the factor that scales them to bytes (from a plain copy of known size in
    the same runs) and the hash of the kernel source they were taken with; a
    changed source makes the figures stale and gives None.
    """
    try:
        vals = {}
        for line in open(summary):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
        if vals.get(key) != source_hash(source):
            return None
        return float(vals["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(e, pairs_np, ctx_results, f, ctx, torch, pc):
    """The oracle as it stands, timed on host cores over a bounded sample."""
    import oracle
    rng = np.random.default_rng(77)
    ia = e.regions[0].global_indices(e.nx, e.ny)
    ib = e.regions[1].global_indices(e.nx, e.ny)
    n_p = 40_000_000  # with the KSG sample about 10 s of oracle work on 16 cores
    ps = np.stack([rng.choice(ia, n_p), rng.choice(ib, n_p)], 1).astype(np.int32)
    t0 = time.perf_counter()
    r_ref = oracle.pearson_pairs(e.data, ps)
    t_p = (time.perf_counter() - t0) / n_p
    n_k = 400_000
    ks = pairs_np[rng.choice(pairs_np.shape[0], n_k, replace=False)]
    t0 = time.perf_counter()
    mi_ref, cnt_ref = oracle.ksg_pairs(e.data, ks, 10)
    t_k = (time.perf_counter() - t0) / n_k
    t_step = N_PEARSON * t_p + N_KSG * t_k
    # the same oracle on one core (smaller sample of each kind)
    cores = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.pearson_pairs(e.data, ps[:1_000_000])
        t_p1 = (time.perf_counter() - t0) / 1_000_000
        t0 = time.perf_counter()
        oracle.ksg_pairs(e.data, ks[:10_000], 10, want_counts=False)
        t_k1 = (time.perf_counter() - t0) / 10_000
    finally:
        oracle.set_num_threads(cores)
    t_step1 = N_PEARSON * t_p1 + N_KSG * t_k1
    # errors of the GPU path on the same sample
    r_gpu = ctx.corr_pearson_pairs(f, torch.from_numpy(ps).cuda(), "f16").cpu().numpy()
    mi_gpu, cnt_gpu = ctx.corr_ksg_mi_pairs(f, torch.from_numpy(ks).cuda(), k=10, counts=True)
    ref_max = oracle.pearson_region_max_matmul(e.data, ia, ib, block=2048)
    err = {
        "_ref_max": float(ref_max["value"]),
        "pearson_f16_pairs_max_abs": float(np.max(np.abs(r_gpu - r_ref))),
        "pearson_region_max_abs": float(abs(ctx_results["pearson"]["value"] - ref_max["value"])),
        "ksg_mi_max_abs": float(np.max(np.abs(mi_gpu.cpu().numpy() - mi_ref))),
        "ksg_count_mismatches": int((cnt_gpu.cpu().numpy() != cnt_ref).sum()),
    }
    return {
        "value": (N_PEARSON + N_KSG) / t_step,
        "unit": "point pairs/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"FP64 Pearson on {n_p} uniform A x B pairs ({t_p * 1e9:.1f} ns/pair) and brute-force KSG on "
                   f"{n_k} of the 1e6 sampled pairs ({t_k * 1e6:.1f} us/pair), extrapolated to one step "
                   f"(4.19e8 Pearson + 1e6 KSG pairs)"),
        "cpu_model": cpu_model(),
        "pearson_value": 1.0 / t_p,
        "ksg_value": 1.0 / t_k,
        "single_core_value": (N_PEARSON + N_KSG) / t_step1,
        "single_core_sample": f"1e6 Pearson pairs ({t_p1 * 1e9:.1f} ns/pair), 1e4 KSG pairs ({t_k1 * 1e6:.1f} us/pair)",
    }, err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="f16", choices=["f32", "f16", "bf16", "f16x3", "bf16x3"])
    ap.add_argument("--workload", default="focus", choices=["focus", "context", "large", "onetoall", "meantree", "meantree-dev", "samplers",
                             "proposal", "peaks"],
                    help="focus: the headline focus-view step (default); context: batched BOS over the 3828 "
                         "region pairs of a 352x256x20 field; large: M=1000 FP16 ensemble rates; onetoall: one "
                         "reference point against every point of a 250x352x20 field (M=100) and of the "
                         "128x128x32 field (M=1000); meantree: mean-tree levels f=2,4 of a 180-member "
                         "640x704x64 field; meantree-dev: deviation of brick maxima on those levels over the 3828 "
                         "brick pairs of the 352x256x20 field; samplers: convergence of uniform / Halton / plastic "
                         "sampled maxima over those pairs and on 6-D Gaussian test objectives; proposal: the "
                         "learned BOS proposal trained on ten 88-region context fields and judged on five unseen "
                         "ones against plain BOS and exhaustive maxima; peaks: the device's measured peaks")
    ap.add_argument("--measure", default="pearson", choices=["pearson", "ksg"], help="BOS objective (context)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="focus: leave out the M=1000 legs (large-ensemble field) of the per-measure breakdown")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (scale reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the hot path has no multi-GPU mode "
              "(region pairs would shard across GPUs, one process per GPU).", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import __graft_entry__ as g
    g._ensure_built()
    import paper_2309_03308_amd as pc

    if args.workload == "context":
        return run_context(args, torch, synth, pc)
    if args.workload == "large":
        return run_large(args, torch, synth, pc)
    if args.workload == "onetoall":
        return run_onetoall(args, torch, synth, pc)
    if args.workload == "meantree":
        return run_meantree(args, torch, synth, pc)
    if args.workload == "meantree-dev":
        return run_meantree_dev(args, torch, synth, pc)
    if args.workload == "samplers":
        return run_samplers(args, torch, synth, pc)
    if args.workload == "proposal":
        return run_proposal(args, torch, synth, pc)
    if args.workload == "peaks":
        return run_peaks(args, torch, synth, pc)
    return run_focus(args, torch, synth, pc)


def _line(args, value, ms, config, **extra):
    line = {
        "metric": "point pairs/s for Pearson & KSG-MI at M=100/1000; max-err vs FP64 oracle",
        "value": value, "unit": "point pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic", "config": config,
    }
    line.update(extra)
    return line


FP64_VALU_PEAK = 78.6e12  # MI355X FP64 vector, flop/s


def measure_peaks(torch, pc, reps=3):
    """On-device peaks from the library's probes (include/corr_peaks.h): LDS read
    bandwidth, dense FP16 MFMA, FP32 / FP64 vector FMA and HBM read bandwidth.
    Each figure is the best of `reps` launches timed with HIP events on the
    stream they run on (one untimed launch first); work / time."""
    s = torch.cuda.current_stream()
    nb = 2048                       # 8 workgroups of 256 threads per CU
    o32 = torch.empty(nb * 256, dtype=torch.float32, device="cuda")
    o64 = torch.empty(nb * 256, dtype=torch.float64, device="cuda")
    oi = torch.empty(nb * 256, dtype=torch.int32, device="cuda")
    hbm = torch.empty(4 << 30, dtype=torch.uint8, device="cuda")

    def best_s(fn):
        fn()
        t = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            fn()
            e1.record(s)
            e1.synchronize()
            t.append(e0.elapsed_time(e1) / 1e3)
        return min(t)

    it_lds, it_mfma, it_f32, it_f64 = 3000, 10000, 20000, 40000
    lds = nb * 256 * it_lds * 128 / best_s(lambda: pc.corr_peak_lds(nb, it_lds, oi))
    mfma = nb * 4 * it_mfma * 4 * 32768 / best_s(lambda: pc.corr_peak_mfma_f16(nb, it_mfma, o32, random_operands=True))
    mfma_c = nb * 4 * it_mfma * 4 * 32768 / best_s(lambda: pc.corr_peak_mfma_f16(nb, it_mfma, o32, random_operands=False))
    f32 = nb * 256 * it_f32 * 16 * 2 / best_s(lambda: pc.corr_peak_valu_f32(nb, it_f32, o32))
    med3 = nb * 256 * it_f32 * 16 / best_s(lambda: pc.corr_peak_valu_med3(nb, it_f32, o32))
    f64 = nb * 256 * it_f64 * 8 * 2 / best_s(lambda: pc.corr_peak_valu_f64(nb, it_f64, o64))
    hb = hbm.numel() / best_s(lambda: pc.corr_peak_hbm_read(hbm, nb, oi))
    del hbm
    return {"lds_read_TBps": lds / 1e12, "mfma_f16_TFLOPs": mfma / 1e12,
            "mfma_f16_TFLOPs_repeated_operands": mfma_c / 1e12, "valu_f32_fma_TFLOPs": f32 / 1e12,
            "valu_lane_ops_Tops": f32 / 2 / 1e12, "valu_med3_lane_ops_Tops": med3 / 1e12,
            "valu_f64_fma_TFLOPs": f64 / 1e12, "hbm_read_GBps": hb / 1e9,
            "vendor": {"lds_read_TBps": 78.6, "mfma_f16_TFLOPs": 2500.0, "valu_lane_ops_Tops": 78.6432,
                       "valu_f64_fma_TFLOPs": 78.6, "hbm_read_GBps": 8000.0},
            "method": "corr_peak_* probes, 2048 workgroups of 256 threads, best of 3 launches (HIP events); "
                      "MFMA on random full-mantissa operands (the power-limited rate that applies to "
                      "standardised data; small repeated operands beside); VALU without packed FP32 "
                      "(lane-ops = FMA flops / 2)"}


def with_measured_peak(roof, peaks):
    """Add the measured peak of the roofline's bound (and the fraction of it) beside the vendor one."""
    if not roof or not peaks:
        return roof
    key = {("mfma", "TFLOP/s"): "mfma_f16_TFLOPs", ("alu", "Tops/s"): "valu_lane_ops_Tops",
           ("alu", "TFLOP/s"): "valu_f64_fma_TFLOPs"}.get((roof.get("bound"), roof.get("unit")))
    pm = peaks["hbm_read_GBps"] if roof.get("bound") == "hbm" else (peaks[key] if key else None)
    if pm and roof.get("achieved") is not None:
        roof["peak_measured"] = pm
        roof["frac_of_measured"] = roof["achieved"] / pm
    return roof


def bos_flops(schedule, n_init, C):
    """FP64 flops of one BOS view, counted from the algorithm at each pair's slot count.

    Per pair and batch (n observations, b picks, C candidates): the Matern
    covariance (25 flops per entry of the lower triangle), the Cholesky factor
    (n^3 / 3), the two solves for alpha (2 n^2), per candidate its covariance
    row, mean and solve vector (25 n + n^2 + 2 n), and per believer pick a
    covariance, an O(rows) update and a variance per candidate (25 + 2 rows + 4).
    n is the slot count (an upper bound: repeated cells are not evaluated
    twice). Returns (total, per-iteration list).
    """
    per_iter = {}
    for sched in schedule:
        n = n_init
        for t, b in enumerate(sched):
            f = 25.0 * n * (n + 1) / 2 + n ** 3 / 3.0 + 2.0 * n * n + C * (25.0 * n + n * n + 2.0 * n)
            f += sum(C * (29.0 + 2.0 * (n + m)) for m in range(b))
            per_iter[t] = per_iter.get(t, 0.0) + f
            n += b
    its = [per_iter[t] for t in sorted(per_iter)]
    return sum(its), its


def context_cpu_baseline(e, pairs, measure, gpu_res, truth, n_sub, cfg_gpu):
    """The oracle BOS (FP64 NumPy GP, C objective) on a seeded subset of the region pairs."""
    import oracle
    from oracle import bos_ref as B
    cfg = B.BosConfig(n_init=cfg_gpu.n_init, n_total=cfg_gpu.n_total, n_uniform=cfg_gpu.n_uniform,
                      n_local=cfg_gpu.n_local, kappa=cfg_gpu.kappa, lengthscale=cfg_gpu.lengthscale,
                      local_sd=cfg_gpu.local_sd, jitter=cfg_gpu.jitter, seed=cfg_gpu.seed)
    sub = np.random.default_rng(31).choice(len(pairs), n_sub, replace=False)
    vals, n_eval = [], 0
    t0 = time.perf_counter()
    for p in sub:
        ia, ib = pairs[p]
        ra, rb = e.regions[ia], e.regions[ib]
        dims = (ra.dx, ra.dy, ra.dz, rb.dx, rb.dy, rb.dz)

        def obj(c, ra=ra, rb=rb):
            pa, pb = B.cells_to_points(c, ra, rb, e.nx, e.ny)
            pp = np.stack([pa, pb], 1).astype(np.int32)
            if measure == "pearson":
                return np.abs(oracle.pearson_pairs(e.data, pp))
            return oracle.ksg_pairs(e.data, pp, 10, want_counts=False)[0]
        r = B.run_pair(cfg, int(p), dims, obj)
        vals.append(r["value"])
        n_eval += r["n_evaluated"]
    dt = time.perf_counter() - t0
    vals = np.array(vals)
    gpu = np.array([gpu_res[p]["value"] for p in sub])
    out = {"value": n_eval / dt, "unit": "evaluations/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"oracle BOS (FP64 NumPy GP and acquisition, C objective) on {n_sub} seeded region pairs "
                     f"of the 3828, {n_eval} evaluations in {dt:.1f} s; a whole view extrapolates to "
                     f"{dt * len(pairs) / n_sub:.0f} s",
           "cpu_model": cpu_model(),
           "gpu_vs_oracle_bos_max_abs": float(np.max(np.abs(gpu - vals))),
           "gpu_vs_oracle_bos_equal_within_1e-5": float(np.mean(np.abs(gpu - vals) <= 1e-5))}
    if truth is not None:
        out["oracle_bos_mean_abs_err_vs_exhaustive"] = float(np.mean(np.abs(truth[sub] - vals)))
        out["gpu_bos_mean_abs_err_vs_exhaustive_same_pairs"] = float(np.mean(np.abs(truth[sub] - gpu)))
    return out


def context_view(torch, synth, pc, measure, steps, warmup, cpu_pairs):
    """Batched BOS (20 + 80 samples per pair, uneven batches) over all 3828 region pairs of the
    352x256x20 context field: whole-view time, per-phase HIP-event times, the error against the
    exhaustive FP16x3 maxima per class (Pearson), a bos_kernel roofline and, when cpu_pairs > 0,
    the oracle BOS on that many pairs. Returns (result dict, mean view ms, evaluations)."""
    print("context: generating the 352x256x20 ensemble", file=sys.stderr, flush=True)
    e = synth.make_cfg3()
    ctx = pc.Context(0)
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    regions = [pc.region(*r.as_tuple()) for r in e.regions]
    pairs = synth.region_pair_list(len(e.regions))
    cfg = pc.bos_defaults(measure=measure, k=10, seed=1)

    def view():
        bos = pc.Bos(ctx, f, regions, pairs, cfg)
        n_it = 0
        while bos.bos_sample_step() > 0:
            n_it += 1
        res = bos.bos_results()
        bos.close()
        return res, n_it

    for _ in range(warmup):
        view()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res, _ = view()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    n_eval = sum(r["n_evaluated"] for r in res)
    print(f"context: {ms:.1f} ms per view", file=sys.stderr, flush=True)

    # phases of one more view, each timed with HIP events on the stream the work runs on
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    bos = pc.Bos(ctx, f, regions, pairs, cfg)
    ev[1].record(stream)
    torch.cuda.synchronize()
    create_ms = ev[0].elapsed_time(ev[1])
    it_ms = []
    while True:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        active = bos.bos_sample_step()
        b.record(stream)
        torch.cuda.synchronize()
        it_ms.append(a.elapsed_time(b))
        if active == 0:
            break
    schedule = bos.bos_schedule()
    bos.close()
    flops, _ = bos_flops(schedule, cfg.n_init, cfg.n_uniform + cfg.n_local)
    kern_ms = sum(it_ms)
    out = {"value": n_eval / (ms / 1e3), "unit": "evaluated point pairs/s", "view_ms": ms, "measure": measure,
           "bos_iterations": len(it_ms), "evaluations": n_eval, "region_pairs": len(pairs), "create_ms": create_ms,
           "iteration_ms": it_ms, "bos_kernels_ms": kern_ms, "bos_fp64_gflop_per_view": flops / 1e9}
    truth = None
    if measure == "pearson":
        truth = np.array([ctx.corr_region_max(f, regions[i], regions[j], "pearson", "f16x3")["value"]
                          for i, j in pairs])
        err = truth - np.array([r["value"] for r in res])
        planted = np.zeros(len(pairs), bool)
        for gr in e.groups:
            rs = set(gr["regions"])
            planted |= np.array([(i in rs and j in rs) for i, j in pairs])
        noise = ~planted
        out["bos_error_vs_exhaustive_f16x3"] = {
            "mean_abs": float(np.abs(err).mean()), "max_abs": float(np.abs(err).max()),
            "frac_within_0.01": float(np.mean(np.abs(err) <= 0.01)),
            "planted_pairs": int(planted.sum()),
            "planted_mean_abs": float(np.abs(err[planted]).mean()) if planted.any() else None,
            "planted_frac_within_0.01": float(np.mean(np.abs(err[planted]) <= 0.01)) if planted.any() else None,
            "noise_pairs": int(noise.sum()),
            "noise_mean_abs": float(np.abs(err[noise]).mean()),
            "noise_frac_within_0.01": float(np.mean(np.abs(err[noise]) <= 0.01)),
            "normalized_mean": float((err / truth).mean()),
            "never_above_exhaustive": bool(np.all(err >= -2e-5))}
    out["roofline"] = {"bound": "alu", "achieved": flops / (kern_ms / 1e3) / 1e12, "peak": FP64_VALU_PEAK / 1e12,
                       "unit": "TFLOP/s", "frac": flops / (kern_ms / 1e3) / FP64_VALU_PEAK, "traffic": None,
                       "kernel": "bos_kernel (all iterations of one view)",
                       "work": "FP64 flops of the GP factorisation, posterior over 512 candidates and "
                               "Kriging-believer updates per pair and batch, counted at the slot count; "
                               "iterations timed with HIP events on the stream they run on"}
    if cpu_pairs:
        print(f"context: oracle BOS on {cpu_pairs} region pairs", file=sys.stderr, flush=True)
        out["cpu_baseline"] = context_cpu_baseline(e, pairs, measure, res, truth, cpu_pairs, cfg)
    ctx.close()
    del f
    torch.cuda.empty_cache()
    return out, ms, n_eval


def run_context(args, torch, synth, pc):
    """Context view: batched BOS over all 3828 region pairs; one step is one whole view (bos_create,
    every iteration replayed from a captured HIP graph, the read-back of the 3828 maxima)."""
    out, ms, n_eval = context_view(torch, synth, pc, args.measure, args.steps, args.warmup,
                                   0 if args.no_cpu_baseline else 100)
    extra = {"breakdown": {k: v for k, v in out.items() if k not in ("roofline", "cpu_baseline", "value", "unit")},
             "roofline": out["roofline"]}
    if "cpu_baseline" in out:
        extra["cpu_baseline"] = out["cpu_baseline"]
    line = _line(args, n_eval / (ms / 1e3), ms,
                 {"workload": f"context view: 352x256x20 ensemble, M=100 FP32, 88 regions of 32x32x20, 3828 "
                              f"region pairs, batched BOS ({args.measure}, 20 + 80 samples per pair)",
                  "members": 100, "region_pairs": 3828, "measure": args.measure}, **extra)
    line["unit"] = "evaluated point pairs/s"
    line["dtype"] = "f64 GP, f32 objective"
    print(json.dumps(line), flush=True)


def run_large(args, torch, synth, pc):
    """M=1000 FP16 ensemble: 4e6 random pairs (Pearson, KSG) and the focus contraction."""
    e = synth.make_cfg4()
    P = e.nx * e.ny * e.nz
    ctx = pc.Context(0)
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    pairs = torch.from_numpy(synth.random_pairs(104, 4_000_000, P)).cuda()
    ra, rb = [pc.region(*r.as_tuple()) for r in e.regions]
    out = torch.empty(pairs.shape[0], device="cuda")

    def timed(fn, reps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_p = timed(lambda: ctx.corr_pearson_pairs(f, pairs, "f32", out=out), args.steps)
    t_k = timed(lambda: ctx.corr_ksg_mi_pairs(f, pairs, k=10, out=out), max(1, args.steps // 10))
    t_g = timed(lambda: ctx.corr_region_max(f, ra, rb, "pearson", args.prec), args.steps)
    n_focus = 4096 * 4096
    # two 32x32x20 regions (4.19e8 pairs): many 256x256 tiles per CU, so the
    # contraction's per-tile start-up and epilogue are amortised; kernel time
    # from HIP events on the call's stream
    ctx.set_timing(True)
    wa, wb = pc.region(0, 0, 0, 32, 32, 20), pc.region(64, 64, 0, 32, 32, 20)
    n_wide = (32 * 32 * 20) ** 2
    wide = {}
    for wp in ("f16", "bf16"):
        _, w_ms = _timed(torch, lambda: ctx.corr_region_max(f, wa, wb, "pearson", wp), max(3, args.steps // 2),
                         args.warmup, ctx, "gemm")
        wide[wp] = {"kernel_ms": w_ms, "pairs_per_s": n_wide / (w_ms / 1e3),
                    "tflops_algorithmic": 2.0 * 1000 * n_wide / (w_ms / 1e3) / 1e12}
    ctx.set_timing(False)
    ms = (t_p + t_k + t_g) * 1e3
    value = (2 * pairs.shape[0] + n_focus) / (ms / 1e3)
    line = _line(args, value, ms,
                 {"workload": "large ensemble: 128x128x32, M=1000 FP16 storage, 4e6 random pairs "
                              "(Pearson FP32 and KSG k=10) + focus contraction of two 16^3 regions",
                  "members": 1000, "random_pairs": int(pairs.shape[0]), "focus_pairs": n_focus,
                  "focus_precision": args.prec},
                 breakdown={"pearson_pairs_per_s": pairs.shape[0] / t_p, "ksg_pairs_per_s": pairs.shape[0] / t_k,
                            "focus_pairs_per_s": n_focus / t_g,
                            "focus_tflops_algorithmic": 2.0 * 1000 * n_focus / t_g / 1e12,
                            # FP32 operand rows as gathered (1008 padded members, 4 B each, two rows
                            # per pair); the time also holds standardising the whole field
                            "pearson_gather_gbps_fp32_rows": pairs.shape[0] * 2 * 1008 * 4 / t_p / 1e9,
                            "contraction_32x32x20_regions": wide})
    print(json.dumps(line), flush=True)
    ctx.close()


def run_onetoall(args, torch, synth, pc):
    """One reference point against every grid point (the shape of the paper's performance table)."""
    out = {}
    for label, make, M in (("M100", lambda: synth.make_field("onetoall-250x352x20-M100", 5, 100, 250, 352, 20, [], []),
                            100),
                           ("M1000", synth.make_cfg4, 1000)):
        e = make()
        P = e.nx * e.ny * e.nz
        f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
        ctx = pc.Context(0)
        ref = (e.nx // 2) + e.nx * ((e.ny // 2) + e.ny * (e.nz // 2))
        pairs = torch.stack([torch.full((P,), ref, dtype=torch.int32), torch.arange(P, dtype=torch.int32)], 1).cuda()
        res = torch.empty(P, device="cuda")

        def timed(fn, reps):
            for _ in range(max(1, args.warmup)):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps

        tp = timed(lambda: ctx.corr_pearson_pairs(f, pairs, "f32", out=res), args.steps)
        tk = timed(lambda: ctx.corr_ksg_mi_pairs(f, pairs, k=10, out=res), max(1, args.steps // 5))
        out[label] = {"points": P, "pearson_s": tp, "ksg_s": tk, "pearson_pairs_per_s": P / tp,
                      "ksg_pairs_per_s": P / tk}
        ctx.close()
        del f, pairs, res
        torch.cuda.empty_cache()
    ms = (out["M100"]["pearson_s"] + out["M100"]["ksg_s"]) * 1e3
    line = _line(args, 2 * out["M100"]["points"] / (ms / 1e3), ms,
                 {"workload": "one-to-all: one reference point against all 1.76e6 points of a 250x352x20 ensemble "
                              "(M=100, FP32), Pearson and KSG k=10; also the 524288-point M=1000 FP16 field",
                  "members": 100, "points": out["M100"]["points"]},
                 breakdown=out)
    print(json.dumps(line), flush=True)


def run_meantree(args, torch, synth, pc):
    """Mean-tree levels f = 2 and 4 of a 180-member 640x704x64 field (HBM-bound)."""
    M, nx, ny, nz = 180, 640, 704, 64
    print(f"meantree: generating {M} x {nx}x{ny}x{nz} on the device", file=sys.stderr, flush=True)
    X = synth.smooth_field_torch(M, nx, ny, nz, seed=11)
    A = pc.Field(X, nx, ny, nz)
    ctx = pc.Context(0)
    P = nx * ny * nz
    outs, nbytes = {}, {}
    for fct in (2, 4):
        NX, NY, NZ = pc.level_dims(nx, ny, nz, fct)
        outs[fct] = torch.empty((M, NX * NY * NZ), device="cuda")
        nbytes[fct] = 4.0 * M * (P + NX * NY * NZ)  # read every value once, write every mean once

    def step():
        for fct in (2, 4):
            ctx.corr_block_means(A, fct, "f32", out=outs[fct])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    ctx.set_timing(True)
    kern = {}
    for fct in (2, 4):
        t = []
        for _ in range(args.steps):
            ctx.corr_block_means(A, fct, "f32", out=outs[fct])
            t.append(ctx.kernel_time_ms("block_means"))
        kern[fct] = float(np.mean(t))
    ctx.set_timing(False)
    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
    ctx.close()

    tot_bytes = nbytes[2] + nbytes[4]
    achieved = nbytes[2] / (kern[2] / 1e3) / 1e9
    line = {
        "metric": "HBM bytes/s building mean-tree levels f=2,4 (read the field, write the block means)",
        "value": tot_bytes / (ms / 1e3), "unit": "B/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (device-generated smoothed Gaussian noise)",
        "config": {"workload": "mean-tree levels f=2 and f=4 of a 180-member 640x704x64 FP32 ensemble "
                               "(20.8 GB, each level from the initial data)",
                   "members": M, "points": P},
        "breakdown": {"kernel_ms": {f"f{k}": v for k, v in kern.items()},
                      "kernel_GBps": {f"f{k}": nbytes[k] / (kern[k] / 1e3) / 1e9 for k in kern}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
                     "traffic": measured_traffic(AGG_TRAFFIC_FILE, AGG_SOURCE, "aggregate_source_sha256"),
                     "kernel": "block_means_vec_kernel<float, float, 2>",
                     "work": "4 B read per input value + 4 B written per block mean, 180 x 28.8e6 values per launch"},
    }
    print(json.dumps(line), flush=True)


def run_meantree_dev(args, torch, synth, pc):
    """Brick maxima at f = 1, 2, 4 over every pair of the 88 bricks (32x32x20) of
    the 352x256x20 M=100 field: exhaustive Pearson (the quantity BOS estimates)
    and batched BOS on each level (mean of ten runs of 100 samples per pair),
    with the deviation of the level maxima from those on the initial data."""
    ctx = pc.Context(0)
    e = synth.make_cfg3()
    F1 = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    regs = [pc.region(*r.as_tuple()) for r in e.regions]
    pairs = synth.region_pair_list(len(regs))
    maxima, tmax = {}, {}
    for fct in (1, 2, 4):
        Fl = F1 if fct == 1 else ctx.corr_block_means(F1, fct, "f32")
        lr = [pc.region_at_level(r, fct) for r in regs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        maxima[fct] = np.array([ctx.corr_region_max(Fl, lr[a], lr[b], "pearson", "f16x3")["value"] for a, b in pairs])
        tmax[fct] = time.perf_counter() - t0
        print(f"meantree-dev: f={fct} {len(pairs)} maxima in {tmax[fct]:.2f} s", file=sys.stderr, flush=True)
    # pairs whose bricks hold blobs of one planted group carry a genuine maximum;
    # the others' maxima are the extreme of ~4e8 noise correlations
    planted = np.zeros(len(pairs), bool)
    for gr in e.groups:
        rs = set(gr["regions"])
        planted |= np.array([(int(a) in rs and int(b) in rs) for a, b in pairs])
    # batched BOS on each level (Sec. 3.3: BOS runs on the aggregated data);
    # the paper's comparison averages ten BOS runs of 100 samples per pair
    bos_mean, bos_s = {}, {}
    for fct in (1, 2, 4):
        Fl = F1 if fct == 1 else ctx.corr_block_means(F1, fct, "f32")
        lr = [pc.region_at_level(r, fct) for r in regs]
        runs, t_runs = [], 0.0
        for seed in range(10):
            b = pc.Bos(ctx, Fl, lr, pairs, pc.bos_defaults(seed=seed))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.bos_run()
            torch.cuda.synchronize()
            t_runs += time.perf_counter() - t0
            runs.append(np.array([r["value"] for r in b.bos_results()]))
            b.close()
        bos_mean[fct], bos_s[fct] = np.mean(runs, axis=0), t_runs / 10
        err = maxima[fct] - bos_mean[fct]
        print(f"meantree-dev: f={fct} BOS (10 runs x 100 samples) {bos_s[fct] * 1e3:.1f} ms per view, "
              f"mean |exhaustive - BOS| {np.mean(np.abs(err)):.4f}", file=sys.stderr, flush=True)
    dev = {}
    for fct in (2, 4):
        db = bos_mean[fct] - bos_mean[1]
        relb = np.abs(db) / bos_mean[1]
        dev[f"bos_f{fct}"] = {"mean_rel_dev": float(np.mean(relb)), "mean_signed_dev": float(np.mean(db)),
                              "mean_rel_dev_planted": float(np.mean(relb[planted])) if planted.any() else None}
    for fct in (2, 4):
        d = maxima[fct] - maxima[1]
        rel = np.abs(d) / maxima[1]
        dev[f"f{fct}"] = {"mean_rel_dev": float(np.mean(rel)), "mean_abs_dev": float(np.mean(np.abs(d))),
                          "mean_signed_dev": float(np.mean(d)), "s_all_pairs": tmax[fct],
                          "planted_pairs": int(planted.sum()),
                          "mean_rel_dev_planted": float(np.mean(rel[planted])) if planted.any() else None,
                          "mean_signed_dev_planted": float(np.mean(d[planted])) if planted.any() else None}
    ctx.close()
    ms = tmax[1] * 1e3
    line = _line(args, len(pairs) * (20480.0 ** 2) / tmax[1], ms,
                 {"workload": "brick maxima (exhaustive Pearson, FP16x3) for the 3828 pairs of 32x32x20 bricks of "
                              "the 352x256x20 M=100 field on the initial data and on mean-tree levels f=2, 4, "
                              "with batched BOS (10 runs x 100 samples) on each level",
                  "members": 100, "brick_pairs": int(len(pairs))},
                 breakdown={"deviation_of_maxima": dev, "mean_max_f1": float(np.mean(maxima[1])),
                            "bos_ms_per_view": {f"f{k}": v * 1e3 for k, v in bos_s.items()},
                            "bos_mean_abs_err_vs_exhaustive": {f"f{k}": float(np.mean(np.abs(maxima[k] - bos_mean[k])))
                                                               for k in bos_mean},
                            "mean_max_f1_planted": float(np.mean(maxima[1][planted])) if planted.any() else None,
                            "s_all_pairs": {f"f{k}": v for k, v in tmax.items()}})
    line["steps"], line["warmup"] = 1, 0
    print(json.dumps(line), flush=True)


def _gauss6(rng, dims):
    """A 6-D Gaussian test objective over a brick pair's cell box (a random
    mean in the box, a random rotation, standard deviations of 4 to 8 cells):
    the objective value at cells, its exact maximum over the integer cells (within
    3 cells of the mean per axis, which a condition number of 4 guarantees) and its
    minimum (a corner of the box)."""
    d = np.asarray(dims, np.float64)
    mu = rng.uniform(0, 1, 6) * (d - 1)
    q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    prec = q @ np.diag(1.0 / rng.uniform(4.0, 8.0, 6) ** 2) @ q.T

    def f(c):
        x = np.asarray(c, np.float64) - mu
        return np.exp(-0.5 * np.einsum("ni,ij,nj->n", x, prec, x))

    base = np.round(mu).astype(np.int64)
    g = np.stack(np.meshgrid(*[np.arange(-3, 4)] * 6, indexing="ij"), -1).reshape(-1, 6) + base
    g = g[np.all((g >= 0) & (g < np.asarray(dims)), axis=1)]
    corners = np.array([[(dims[j] - 1) * ((m >> j) & 1) for j in range(6)] for m in range(64)])
    return f, float(f(g).max()), float(f(corners).min())


def run_samplers(args, torch, synth, pc):
    """Uniform / Halton / plastic sampling (Sec. 3.1): maxima against exhaustive truth."""
    ctx = pc.Context(0)
    e = synth.make_cfg3()
    F = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    regs = [r.as_tuple() for r in e.regions]
    rp = synth.region_pair_list(len(regs))
    t0 = time.perf_counter()
    truth = np.array([ctx.corr_region_max(F, pc.region(*regs[a]), pc.region(*regs[b]), "pearson", "f16x3")["value"]
                      for a, b in rp])
    t_ex = time.perf_counter() - t0
    ns = (25, 50, 100, 200, 400, 800, 1600)
    seeds = (0, 1, 2)
    curves, times = {}, {}
    for smp in ("uniform", "halton", "plastic"):
        curves[smp], times[smp] = {}, {}
        for n in ns:
            errs, tt = [], []
            for sd in seeds:
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                res = ctx.corr_sampled_max(F, regs, rp, "pearson", "f32", 10, smp, n, sd)
                tt.append(time.perf_counter() - t1)
                v = np.array([r["value"] for r in res])
                errs.append(float(np.mean((truth - v) / truth)))
            curves[smp][n] = float(np.mean(errs))
            times[smp][n] = float(np.median(tt))
        print(f"samplers: pearson {smp} done", file=sys.stderr, flush=True)
    # KSG: mean sampled maximum (exhaustive KSG truth is out of reach: 4.2e8 pairs per brick pair)
    ksg = {}
    for smp in ("uniform", "halton", "plastic"):
        ksg[smp] = {n: float(np.mean([r["value"] for r in ctx.corr_sampled_max(F, regs, rp, "ksg", "f32", 10, smp, n, 0)]))
                    for n in (25, 100, 400)}
    tk = []
    for sd in seeds:  # the whole KSG context view by random sampling: 3828 pairs x 100 samples
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.corr_sampled_max(F, regs, rp, "ksg", "f32", 10, "uniform", 100, sd)
        tk.append(time.perf_counter() - t1)
    # Gaussian test objectives on 1000 brick pairs of 32^3 cells (the samples come from the library)
    G = pc.Field(torch.zeros((2, 32 * 32 * 32), device="cuda"), 32, 32, 32)
    rng = np.random.default_rng(2309)
    objs = [_gauss6(rng, (32,) * 6) for _ in range(1000)]
    gauss = {}
    for smp in ("uniform", "halton", "plastic"):
        gauss[smp] = {}
        for n in (25, 50, 100, 200, 400, 800):
            cells = ctx.corr_sample_pairs(G, [(0, 0, 0, 32, 32, 32)], np.zeros((1000, 2), np.int32), smp, n, 5)
            c = cells.cpu().numpy().astype(np.int64)
            err = []
            for p, (f, mx, mn) in enumerate(objs):
                pa, pb = c[p, :, 0], c[p, :, 1]
                cc = np.stack([pa % 32, (pa // 32) % 32, pa // 1024, pb % 32, (pb // 32) % 32, pb // 1024], 1)
                err.append((mx - f(cc).max()) / (mx - mn))
            gauss[smp][n] = float(np.mean(err))
    ctx.close()
    n_ref = 100
    line = _line(args, len(rp) * n_ref / times["uniform"][n_ref], times["uniform"][n_ref] * 1e3,
                 {"workload": "sampled Pearson maxima (FP32) of the 3828 pairs of 32x32x20 bricks of the 352x256x20 "
                              "M=100 field, 100 uniform samples per pair (batched); convergence of the three "
                              "samplers against exhaustive FP16x3 maxima", "members": 100, "brick_pairs": int(len(rp))},
                 breakdown={"exhaustive_truth_s": t_ex,
                            "mean_rel_error_pearson": curves, "call_s": times,
                            "mean_sampled_max_ksg": ksg, "ksg_call_s_100_samples": float(np.median(tk)),
                            "gauss6_mean_normalized_error": gauss})
    line["steps"], line["warmup"] = len(seeds), 0
    print(json.dumps(line), flush=True)


def _timed(torch, fn, reps, warmup, ctx=None, cls=None):
    """Mean wall time per call (s) and, with a timing class, mean kernel time (ms) from HIP events."""
    for _ in range(max(1, warmup)):
        fn()
    torch.cuda.synchronize()
    ks = []
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
        if cls:
            ks.append(ctx.kernel_time_ms(cls))
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, (float(np.mean(ks)) if ks else None)


def large_legs(args, torch, synth, pc):
    """The M = 1000 half of the metric on the 128x128x32 large-ensemble field (FP16 storage).

    Pearson and KSG on 4e6 random point pairs (fields prepared once: the
    statistics, rows and sorted rows are computed outside the timed calls and
    their time is reported beside), and the exhaustive contraction of two
    16^3 regions. Each leg carries its own roofline and oracle baseline.
    """
    import oracle
    print("bench: generating the 128x128x32 M=1000 ensemble", file=sys.stderr, flush=True)
    e = synth.make_cfg4()
    P, Mb = e.nx * e.ny * e.nz, e.data.shape[0]
    ctx = pc.Context(0)
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    n = 4_000_000
    pairs_np = synth.random_pairs(104, n, P)
    pairs = torch.from_numpy(pairs_np).cuda()
    out = torch.empty(n, device="cuda")
    ra, rb = [pc.region(*r.as_tuple()) for r in e.regions]
    ctx.set_timing(True)
    legs = {}
    reps = max(3, args.steps // 2)

    # Pearson pair list, FP16 rows (provably within 9.8e-4 of the FP64 value)
    t0 = time.perf_counter()
    pp = ctx.corr_prepare(f, "pearson", "f16")
    torch.cuda.synchronize()
    prep_p = (time.perf_counter() - t0) * 1e3
    t_call, k_ms = _timed(torch, lambda: ctx.corr_pearson_pairs_prepared(pp, pairs, out=out), reps, args.warmup,
                          ctx, "pairs")
    t_unprep, _ = _timed(torch, lambda: ctx.corr_pearson_pairs(f, pairs, "f16", out=out), 3, 1)
    r_gpu = ctx.corr_pearson_pairs_prepared(pp, pairs, out=out).cpu().numpy()
    pp.close()
    byt = n * 2.0 * Mb * 2.0  # two FP16 member rows per pair
    legs["pearson_pairs_m1000"] = {
        "value": n / (k_ms / 1e3), "unit": "point pairs/s", "kernel_ms": k_ms, "call_ms": t_call * 1e3,
        "prepare_ms": prep_p, "per_call_standardising_pairs_per_s": n / t_unprep, "precision": "f16",
        "pairs": n, "roofline": {"bound": "hbm", "achieved": byt / (k_ms / 1e3) / 1e9, "peak": HBM_PEAK / 1e9,
                                 "unit": "GB/s", "frac": byt / (k_ms / 1e3) / HBM_PEAK,
                                 "traffic": measured_traffic(PAIRS_TRAFFIC_FILE, PAIRS_SOURCE, "pairs_source_sha256"),
                                 "kernel": "pearson pair-list gather (FP16 rows)",
                                 "work": "2 x 1000 x 2 B of member values per pair"}}

    # KSG pair list, k = 10
    t0 = time.perf_counter()
    pk = ctx.corr_prepare(f, "ksg")
    torch.cuda.synchronize()
    prep_k = (time.perf_counter() - t0) * 1e3
    t_call, k_ms = _timed(torch, lambda: ctx.corr_ksg_mi_pairs_prepared(pk, pairs, k=10, out=out), 2, 1, ctx, "ksg")
    mi_gpu = ctx.corr_ksg_mi_pairs_prepared(pk, pairs, k=10, out=out).cpu().numpy()
    ops = n * Mb * (Mb - 1) * 3.0
    legs["ksg_m1000"] = {
        "value": n / (k_ms / 1e3), "unit": "point pairs/s", "kernel_ms": k_ms, "call_ms": t_call * 1e3,
        "prepare_ms": prep_k, "k": 10, "pairs": n,
        "roofline": {"bound": "alu", "achieved": ops / (k_ms / 1e3) / 1e12, "peak": VALU_LANE_OPS_PER_S / 1e12,
                     "unit": "Tops/s", "frac": ops / (k_ms / 1e3) / VALU_LANE_OPS_PER_S,
                     "traffic": measured_traffic(KSG1000_TRAFFIC_FILE), "kernel": "ksg_kernel<10, 0, true>",
                     "work": "3 VALU lane-ops per Chebyshev distance, M(M-1) distances per pair"}}

    # exhaustive contraction of the two 16^3 focus regions
    nf = 4096 * 4096
    _, g_ms = _timed(torch, lambda: ctx.corr_region_max(f, ra, rb, "pearson", "f16"), reps, args.warmup, ctx, "gemm")
    g_call, _ = _timed(torch, lambda: ctx.corr_region_max(f, ra, rb, "pearson", "f16"), reps, 1)
    focus = ctx.corr_region_max(f, ra, rb, "pearson", "f16")
    fl = 2.0 * Mb * nf
    legs["pearson_allpairs_m1000"] = {
        "value": nf / (g_ms / 1e3), "unit": "point pairs/s", "kernel_ms": g_ms, "call_ms": g_call * 1e3,
        "precision": "f16", "pairs": nf,
        "roofline": {"bound": "mfma", "achieved": fl / (g_ms / 1e3) / 1e12, "peak": MFMA_F16_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": fl / (g_ms / 1e3) / MFMA_F16_PEAK, "traffic": None,
                     "kernel": "gemm_max_wide_kernel (256 x 256 tiles, K = 1024)", "work": "2 M flops per point pair"}}

    if not args.no_cpu_baseline:
        print("bench: oracle at M = 1000", file=sys.stderr, flush=True)
        rng = np.random.default_rng(78)
        sp = rng.choice(n, 200_000, replace=False)
        t0 = time.perf_counter()
        r_ref = oracle.pearson_pairs(e.data, pairs_np[sp])
        tp = (time.perf_counter() - t0) / sp.size
        sk = sp[:4000]
        t0 = time.perf_counter()
        mi_ref, cnt_ref = oracle.ksg_pairs(e.data, pairs_np[sk], 10)
        tk = (time.perf_counter() - t0) / sk.size
        _, cnt_gpu = ctx.corr_ksg_mi_pairs(f, torch.from_numpy(np.ascontiguousarray(pairs_np[sk[:200]])).cuda(),
                                           k=10, counts=True)
        ia = e.regions[0].global_indices(e.nx, e.ny)
        ib = e.regions[1].global_indices(e.nx, e.ny)
        t0 = time.perf_counter()
        fref = oracle.pearson_region_max_matmul(e.data, ia, ib, block=2048)
        tf = time.perf_counter() - t0
        cores = oracle.num_threads()
        legs["pearson_pairs_m1000"]["max_err_vs_fp64_oracle"] = float(np.max(np.abs(r_gpu[sp] - r_ref)))
        legs["pearson_pairs_m1000"]["cpu_baseline"] = {
            "value": 1.0 / tp, "unit": "point pairs/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 two-pass Pearson on 200000 of the 4e6 pairs ({tp * 1e9:.0f} ns/pair)"}
        legs["ksg_m1000"]["max_err_vs_fp64_oracle"] = float(np.max(np.abs(mi_gpu[sk] - mi_ref)))
        legs["ksg_m1000"]["count_mismatches_200_pairs"] = int((cnt_gpu.cpu().numpy() != cnt_ref[:200]).sum())
        legs["ksg_m1000"]["cpu_baseline"] = {
            "value": 1.0 / tk, "unit": "point pairs/s", "cores": cores, "kind": "oracle",
            "sample": f"brute-force KSG on 4000 of the 4e6 pairs ({tk * 1e3:.2f} ms/pair)"}
        legs["pearson_allpairs_m1000"]["max_err_vs_fp64_oracle"] = float(abs(focus["value"] - fref["value"]))
        legs["pearson_allpairs_m1000"]["cpu_baseline"] = {
            "value": nf / tf, "unit": "point pairs/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 row-block matmul over all 4096 x 4096 focus pairs ({tf:.2f} s)"}
    ctx.close()
    del f, pairs, out
    torch.cuda.empty_cache()
    return legs


def run_proposal(args, torch, synth, pc):
    """Learned BOS proposal at scale: records from ten context fields of the
    352x256x20 generator (seeds 1000-1009, 88 regions, 3828 pairs each) and
    the 4096 sub-brick pairs of a focus field (seed 1010, bricks split
    4 x 4 x 4), the 58 -> 256 -> 256 -> 18 network trained on the GPU, then on
    five unseen fields (seeds 9000-9004) plain GPU BOS at 100 samples per pair against
    GPU BOS seeded with the network's best candidate at 36 and 100 samples,
    each judged by the exhaustive FP16x3 maxima, planted and noise pairs apart.
    One step is one learned-proposal view at 36 samples per pair: inputs,
    inference, prior cells and the batched BOS."""
    from paper_2309_03308_amd import proposal as PR
    ctx = pc.Context(0)
    Xs, Ys = [], []
    t0 = time.perf_counter()
    for s in range(1000, 1010):
        e = synth.make_cfg3(seed=s)
        f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
        regs = [pc.region(*r.as_tuple()) for r in e.regions]
        x, y, _ = PR.make_records(ctx, f, regs, synth.region_pair_list(len(e.regions)))
        Xs.append(x)
        Ys.append(y)
        print(f"proposal: records of field {s}: {x.shape[0]}", file=sys.stderr, flush=True)
        del f
    # sub-brick pairs of a focus field (seed 1010): each brick split 4 x 4 x 4
    e = synth.make_cfg2(seed=1010)
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    subs = []
    for r in e.regions:
        for z in range(4):
            for y in range(4):
                for x in range(4):
                    subs.append(pc.region(r.x0 + x * (r.dx // 4), r.y0 + y * (r.dy // 4), r.z0 + z * (r.dz // 4),
                                          r.dx // 4, r.dy // 4, r.dz // 4))
    sub_pairs = np.array([(a, 64 + b) for a in range(64) for b in range(64)], np.int32)
    x, y, _ = PR.make_records(ctx, f, subs, sub_pairs)
    Xs.append(x)
    Ys.append(y)
    print(f"proposal: records of the focus field's sub-brick pairs: {x.shape[0]}", file=sys.stderr, flush=True)
    del f
    t_rec = time.perf_counter() - t0
    X, Y = torch.cat(Xs), torch.cat(Ys)
    net = pc.PropMlp(ctx, X.shape[1], 256, PR.n_out(), seed=1)
    t0 = time.perf_counter()
    epochs = 50
    hist = PR.train(net, X, Y, epochs=epochs, batch=256, lr=1e-3, wd=1e-4, loss_w=PR.loss_weights())
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    print(f"proposal: trained on {X.shape[0]} records in {t_train:.1f} s", file=sys.stderr, flush=True)
    evals = {}
    view_ms = []
    eval_seeds = (9000, 9001, 9002, 9003, 9004)
    for s in eval_seeds:
        e = synth.make_cfg3(seed=s)
        f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
        regs = [pc.region(*r.as_tuple()) for r in e.regions]
        pairs = synth.region_pair_list(len(e.regions))
        truth = np.array([ctx.corr_region_max(f, regs[a], regs[b], "pearson", "f16x3")["value"] for a, b in pairs])
        planted = np.zeros(len(pairs), bool)
        for gr in e.groups:
            rs = set(gr["regions"])
            planted |= np.array([(a in rs and b in rs) for a, b in pairs])
        for name, nt, learned in (("plain100", 100, False), ("learned36", 36, True), ("learned100", 100, True),
                                  ("plain36", 36, False)):
            PR.run_bos(ctx, f, regs, pairs, n_total=nt, seed=7)  # warm-up (kernels, graph capture)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            prior = None
            if learned:
                x, hot = PR.inputs(ctx, f, regs, pairs)
                _, prior = PR.prior_cells(net, x, hot, regs, pairs, e.nx, e.ny)
            vals, nev = PR.run_bos(ctx, f, regs, pairs, prior=prior, n_total=nt, seed=7)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if name == "learned36":
                view_ms.append(dt * 1e3)
            err = np.abs(truth - vals)
            r = evals.setdefault(name, {"mean_abs_err": [], "planted_mean_abs_err": [], "noise_mean_abs_err": [],
                                        "planted_frac_within_0.01": [], "evaluations": [], "view_ms": []})
            r["mean_abs_err"].append(float(err.mean()))
            r["planted_mean_abs_err"].append(float(err[planted].mean()))
            r["noise_mean_abs_err"].append(float(err[~planted].mean()))
            r["planted_frac_within_0.01"].append(float(np.mean(err[planted] <= 0.01)))
            r["evaluations"].append(int(nev.sum()))
            r["view_ms"].append(dt * 1e3)
        print(f"proposal: evaluated field {s} ({int(planted.sum())} planted pairs)", file=sys.stderr, flush=True)
        del f
    summary = {k: {m: float(np.mean(v)) for m, v in r.items()} for k, r in evals.items()}
    ms = float(np.mean(view_ms))
    n36 = summary["learned36"]["evaluations"]
    extra = {"breakdown": {"training_records": int(X.shape[0]), "record_generation_s": t_rec,
                           "training_s": t_train, "epochs": epochs, "loss_first_last": [hist[0], hist[-1]],
                           "unseen_fields": len(eval_seeds), "per_config": summary, "per_field": evals}}
    if not args.no_cpu_baseline:
        from oracle import mlp_ref
        n_in, H, n_o = X.shape[1], 256, PR.n_out()
        params = net.get_params().astype(np.float64)
        xb = X[:64].cpu().numpy().astype(np.float64)
        yb = Y[:64].cpu().numpy().astype(np.float64)
        w = np.array(PR.loss_weights(), np.float64)
        reps = 20
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):  # one core: the BLAS calls of the oracle run single-threaded
            t0 = time.perf_counter()
            for _ in range(reps):
                mlp_ref.loss_and_grad(params, xb, yb, w, n_in, H, n_o)
            t_cpu = (time.perf_counter() - t0) / reps
        extra["cpu_baseline"] = {"value": 64 / t_cpu, "unit": "training samples/s (forward + backward)",
                                 "cores": 1, "kind": "oracle",
                                 "sample": f"FP64 NumPy MLP forward and backward on a 64-record batch, {reps} reps "
                                           f"({t_cpu * 1e3:.2f} ms each)"}
        extra["gpu_training_samples_per_s"] = X.shape[0] * epochs / t_train
    line = _line(args, n36 / (ms / 1e3), ms,
                 {"workload": "learned BOS proposal: trained on 10 context fields (352x256x20, 88 regions, M=100, "
                              "seeds 1000-1009) and the sub-brick pairs of a focus field (seed 1010), judged on 5 "
                              "unseen fields (seeds 9000-9004); step = one learned-proposal view at 36 samples per "
                              "pair", "members": 100,
                  "region_pairs": 3828, "network": "58-256-256-18 SiLU, BF16-rounded weights, FP32"}, **extra)
    line["unit"] = "evaluated point pairs/s"
    line["steps"], line["warmup"] = 2, 1
    print(json.dumps(line), flush=True)
    net.close()
    ctx.close()


def run_focus(args, torch, synth, pc):
    e = synth.make_cfg2()
    pairs_np = synth.region_pairs_uniform(102, N_KSG, e.regions[0], e.regions[1], e.nx, e.ny)
    ctx = pc.Context(0)
    f = pc.Field(torch.from_numpy(e.data).cuda(), e.nx, e.ny, e.nz)
    pairs = torch.from_numpy(pairs_np).cuda()
    ra, rb = [pc.region(*r.as_tuple()) for r in e.regions]
    # tile shapes from the autotuner (untimed set-up)
    tuned_cfg, tuned_ms = ctx.corr_autotune(f, ra, rb, args.prec, reps=5)
    tuned_pw, tuned_ksg_ms = ctx.corr_ksg_autotune(f, pairs[:200_000], k=10, reps=3)
    ctx.set_timing(True)
    res = {}

    def step():
        res["pearson"] = ctx.corr_region_max(f, ra, rb, "pearson", args.prec)
        res["ksg"] = ctx.corr_region_max(f, ra, rb, "ksg", k=10, samples=pairs)

    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    k_gemm, k_ksg = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        k_gemm.append(ctx.kernel_time_ms("gemm"))
        k_ksg.append(ctx.kernel_time_ms("ksg"))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    value = (N_PEARSON + N_KSG) / (ms / 1e3)
    gemm_ms = float(np.mean(k_gemm))
    ksg_ms = float(np.mean(k_ksg))

    # roofline of the dominant kernel (KSG): algorithmic work = M(M-1) Chebyshev
    # distance evaluations per pair, 3 VALU lane-ops each (2 sub + max|.|)
    ksg_ops = N_KSG * M * (M - 1) * 3.0
    achieved = ksg_ops / (ksg_ms / 1e3) / 1e12
    peak = VALU_LANE_OPS_PER_S / 1e12
    line = {
        "metric": "point pairs/s for Pearson & KSG-MI at M=100/1000; max-err vs FP64 oracle",
        "value": value,
        "unit": "point pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "focus-view refinement: 80x32x20 ensemble, M=100 FP32, regions 32x32x20 x 2, "
                               "Pearson all 4.19e8 pairs (fused region max) + KSG k=10 on 1e6 sampled pairs",
                   "members": M, "pearson_pairs": N_PEARSON, "ksg_pairs": N_KSG, "k": 10,
                   "pearson_precision": args.prec},
        "breakdown": {
            "pearson_region_max_kernel_ms": gemm_ms,
            "pearson_pairs_per_s_kernel": N_PEARSON / (gemm_ms / 1e3),
            "pearson_mfma_tflops_algorithmic": 2.0 * M * N_PEARSON / (gemm_ms / 1e3) / 1e12,
            "pearson_mfma_frac_of_f16_peak": 2.0 * M * N_PEARSON / (gemm_ms / 1e3) / MFMA_F16_PEAK,
            "ksg_kernel_ms": ksg_ms,
            "ksg_pairs_per_s_kernel": N_KSG / (ksg_ms / 1e3),
            "pearson_max": res["pearson"]["value"],
            "ksg_max": res["ksg"]["value"],
            "autotuned": {"contraction_cfg": tuned_cfg, "contraction_ms": tuned_ms, "ksg_workgroups_per_cu": tuned_pw},
            # what binds KSG: the issue of its VALU instructions (counters: wave
            # instructions per SIMD cycle; the insertion network's v_med3_f32 issue
            # once per 4 cycles, add/sub/max/FMA about every 2.5) versus the LDS
            # stream of neighbour samples (8 B per distance) against 256 CU x 128 B/clk x 2.4 GHz
            "ksg_valu_instructions_per_simd_cycle": measured_value("valu_insts_per_simd_cycle"),
            "ksg_lds_frac": N_KSG * M * (M - 1) * 8.0 / (ksg_ms / 1e3) / LDS_BYTES_PER_S,
        },
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tops/s", "frac": achieved / peak,
                     "traffic": measured_traffic(), "kernel": "ksg_kernel<10, 128, false>",
                     "work": "3 VALU lane-ops per Chebyshev distance, M(M-1) distances per pair, 1e6 pairs per launch",
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"},
    }
    # the metric per measure and ensemble size; each leg with its own roofline
    fl = 2.0 * M * N_PEARSON
    per = {"pearson_allpairs_m100": {
        "value": N_PEARSON / (gemm_ms / 1e3), "unit": "point pairs/s", "kernel_ms": gemm_ms, "precision": args.prec,
        "pairs": N_PEARSON,
        "roofline": {"bound": "mfma", "achieved": fl / (gemm_ms / 1e3) / 1e12, "peak": MFMA_F16_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": fl / (gemm_ms / 1e3) / MFMA_F16_PEAK, "traffic": None,
                     "kernel": "gemm_smallk_kernel (K = 112)", "work": "2 M flops per point pair"}}}
    _, g3_ms = _timed(torch, lambda: ctx.corr_region_max(f, ra, rb, "pearson", "f16x3"), 10, 2, ctx, "gemm")
    res3 = ctx.corr_region_max(f, ra, rb, "pearson", "f16x3")
    per["pearson_allpairs_m100_f16x3"] = {
        "value": N_PEARSON / (g3_ms / 1e3), "unit": "point pairs/s", "kernel_ms": g3_ms, "precision": "f16x3",
        "pairs": N_PEARSON, "note": "three FP16 MFMA passes (hi.hi, hi.lo, lo.hi): the FP32-accuracy form",
        "roofline": {"bound": "mfma", "achieved": 3 * fl / (g3_ms / 1e3) / 1e12, "peak": MFMA_F16_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": 3 * fl / (g3_ms / 1e3) / MFMA_F16_PEAK, "traffic": None,
                     "kernel": "gemm_smallk_kernel, split mode", "work": "3 x 2 M flops per point pair"}}
    per["ksg_m100"] = {"value": N_KSG / (ksg_ms / 1e3), "unit": "point pairs/s", "kernel_ms": ksg_ms, "k": 10,
                       "pairs": N_KSG, "roofline": line["roofline"]}
    if not args.no_cpu_baseline:
        cb, err = cpu_baseline(e, pairs_np, res, f, ctx, torch, pc)
        line["cpu_baseline"] = cb
        err["pearson_f16x3_region_max_abs"] = float(abs(res3["value"] - err.pop("_ref_max")))
        line["max_err_vs_fp64_oracle"] = err
        base = {"cores": cb["cores"], "kind": "oracle", "unit": "point pairs/s"}
        per["pearson_allpairs_m100"]["cpu_baseline"] = dict(base, value=cb["pearson_value"],
                                                            sample="FP64 Pearson on 4e7 uniform A x B pairs")
        per["pearson_allpairs_m100"]["max_err_vs_fp64_oracle"] = err["pearson_region_max_abs"]
        per["pearson_allpairs_m100_f16x3"]["max_err_vs_fp64_oracle"] = err["pearson_f16x3_region_max_abs"]
        per["ksg_m100"]["cpu_baseline"] = dict(base, value=cb["ksg_value"],
                                               sample="brute-force KSG on 4e5 of the 1e6 sampled pairs")
        per["ksg_m100"]["max_err_vs_fp64_oracle"] = err["ksg_mi_max_abs"]
        per["ksg_m100"]["count_mismatches"] = err["ksg_count_mismatches"]
    ctx.close()
    if not args.no_large:
        per.update(large_legs(args, torch, synth, pc))
        # the context view: batched BOS over the 3828 region pairs of the 352x256x20 field
        per["bos_context_view_pearson"], _, _ = context_view(torch, synth, pc, "pearson", 3, 1,
                                                              0 if args.no_cpu_baseline else 30)
    line["per_measure"] = per
    # the rooflines against the device's measured peaks, beside the vendor ones (untimed)
    peaks = measure_peaks(torch, pc)
    line["measured_peaks"] = peaks
    with_measured_peak(line["roofline"], peaks)
    for v in per.values():
        if isinstance(v.get("roofline"), dict) and v["roofline"] is not line["roofline"]:
            with_measured_peak(v["roofline"], peaks)
    print(json.dumps(line), flush=True)


def run_peaks(args, torch, synth, pc):
    """The device's measured peaks alone (the default line carries them too)."""
    peaks = measure_peaks(torch, pc)
    line = _line(args, peaks["mfma_f16_TFLOPs"], 0.0, {"workload": "peak probes (LDS, FP16 MFMA, FP32/FP64 VALU, "
                                                                   "HBM read) on the device"}, measured_peaks=peaks)
    line["metric"], line["unit"], line["steps"], line["warmup"] = "measured dense FP16 MFMA peak", "TFLOP/s", 1, 0
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
