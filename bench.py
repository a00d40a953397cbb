"""Benchmark: posterior voxels/s of voxelwise ABC rejection on one MI355X.

One step = one vpet_abc_infer call over the whole synthetic volume (all voxels,
all draws: prior sampling, forward simulation, discrepancy, selection and the
posterior/model-probability reduction).  Inputs are resident in HBM before the
timed region.  Prints one JSON line.

Default workload: 1,048,576 voxels (128 x 128 x 64), 30 frames over 50 min on a
0.2-min grid, irreversible 2TCM prior box, 100,000 prior draws per voxel drawn
independently for every voxel, 0.1 % accepted (n = 100).  The same line carries
the shared-bank form ("bank_form": one 100k-row bank for all voxels) and the
learned proposal ("learned_proposal": 20k importance-weighted draws per voxel
from a network trained on the GPU, with the error comparison against plain ABC).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "posterior voxels/s at fixed draws & error vs FP64 oracle; % of roofline"
# MI355X: 256 CUs x 64 lanes x 2 flops (FMA) x 2.4 GHz = 78.6 TFLOP/s FP64 vector.
PEAK_F64_VECTOR_TFLOPS = 78.6
PEAK_BF16_MFMA_TFLOPS = 2500.0  # dense BF16 matrix-core peak (no sparsity)
KERNEL_NAME = "vpet_infer_kernel"
SRC = os.path.join(ROOT, "paper_2603_14859_amd", "csrc", "vpet_abc.hip")


def flops_per_draw(n_steps: int, n_frames: int) -> int:
    """Floating-point work of one irreversible-2TCM draw in the kernel's formulation:
    one FMA per grid step (2 flops), 12 flops per frame (frame value from the
    recursion identity: 8; weighted squared residual: 4), 40 flops of per-draw
    set-up (theta map and coefficients, transcendental internals not counted)."""
    return 2 * n_steps + 12 * n_frames + 40


def host_cpu() -> str:
    """The host's CPU model (as lscpu names it) and its logical core count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model} ({os.cpu_count()} logical cores visible)"


def source_sha() -> str:
    with open(SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profiles(workload_name: str, kernel: str = KERNEL_NAME):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload_name}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_src_sha") != source_sha():
        return None
    return rec.get("hbm_bytes_per_launch")


def make_inputs(cfg, dev):
    import torch

    import paper_2603_14859_amd as V
    import workloads as W
    ft, cp = cfg.frame_times, cfg.input_fn()
    th, eps = cfg.truth()
    # Noise-free curves of the true parameters from the library's forward model
    # (this is input preparation, outside the timed region), then noise.
    clean = V.simulate(cfg.models[0], torch.from_numpy(th).to(dev), cp, ft, cfg.dt).cpu().numpy()
    y = W.add_noise(clean, ft, eps)
    return ft, cp, y


def cpu_baseline(cfg, ft, cp, y, y_dev, budget_s: float):
    """The FP64 oracle on the host cores over a bounded sample of the same volume,
    and the error of the GPU outputs on that sample."""
    import torch

    import oracle
    import paper_2603_14859_amd as V
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    threads = max(1, min(threads, 64))
    models, boxes = list(cfg.models), cfg.box_array()
    n_cal = max(1, threads // 4)
    t0 = time.perf_counter()
    oracle.infer(y[:n_cal], ft, cp, cfg.dt, models, boxes, cfg.n_draws, cfg.accept_frac, cfg.infer_seed,
                 nthreads=threads)
    per_vox = (time.perf_counter() - t0) / n_cal
    nv = int(max(threads, min(cfg.n_voxels, budget_s / max(per_vox, 1e-9))))
    nv = max(threads, (nv // threads) * threads)
    t0 = time.perf_counter()
    ref = oracle.infer(y[:nv], ft, cp, cfg.dt, models, boxes, cfg.n_draws, cfg.accept_frac, cfg.infer_seed,
                       nthreads=threads)
    dt = time.perf_counter() - t0
    # error of the GPU outputs against the oracle on these voxels (the same
    # voxels re-run with the debug outputs on; results do not depend on how
    # the volume is split into calls)
    gpu_res = V.infer(y_dev[:nv].contiguous(), ft, cp, cfg.dt, models, boxes, cfg.n_draws, cfg.accept_frac,
                      cfg.infer_seed, debug=True)
    torch.cuda.synchronize()
    g_idx = gpu_res["accept_idx"][:nv].cpu().numpy()
    g_mom = gpu_res["moments"][:nv].cpu().numpy().astype(np.float64)
    g_prob = gpu_res["model_prob"][:nv].cpu().numpy().astype(np.float64)
    same = np.array([set(a.tolist()) == set(b.tolist()) for a, b in zip(g_idx, ref["accept_idx"])])
    ok = ~np.isnan(ref["moments"])
    rel = np.abs(g_mom - ref["moments"])[ok] / np.maximum(np.abs(ref["moments"][ok]), 1e-300)
    mean_mask = ok.copy()
    mean_mask[..., 1] = False
    rel_mean = (np.abs(g_mom - ref["moments"])[mean_mask] / np.abs(ref["moments"][mean_mask]))
    same_mean = np.abs(g_mom[same] - ref["moments"][same])[mean_mask[same]] / np.abs(ref["moments"][same][mean_mask[same]])
    err = {
        "voxels": int(nv),
        "identical_accepted_sets": int(same.sum()),
        "max_rel_err_posterior_mean_identical_sets": float(same_mean.max()) if same_mean.size else None,
        "max_rel_err_posterior_mean_all": float(rel_mean.max()) if rel_mean.size else None,
        "max_rel_err_moments_all": float(rel.max()) if rel.size else None,
        "max_abs_err_model_prob": float(np.abs(g_prob - ref["model_prob"]).max()),
    }
    # the same oracle on one thread, over a few voxels
    n1 = max(1, min(nv, int(budget_s / 8 / max(per_vox * threads, 1e-9))))
    t0 = time.perf_counter()
    oracle.infer(y[:n1], ft, cp, cfg.dt, models, boxes, cfg.n_draws, cfg.accept_frac, cfg.infer_seed, nthreads=1)
    dt1 = time.perf_counter() - t0
    base = {"value": nv / dt, "unit": "voxels/s", "cores": threads, "kind": "oracle", "cpu_model": host_cpu(),
            "sample": f"first {nv} voxels of the same volume, all {cfg.n_draws} draws each, FP64, "
                      f"OpenMP over voxels ({dt:.1f} s)",
            "value_1_thread": n1 / dt1, "sample_1_thread": f"first {n1} voxels, one thread ({dt1:.1f} s)"}
    return base, err


def bank_form(cfg, ft, cp, y_host, y_dev, steps: int, warmup: int, cpu: bool, budget_s: float, scan: str = "bf16"):
    """The shared-bank form (one bank of cfg.n_draws prior draws for every voxel) on the same volume."""
    import torch

    import paper_2603_14859_amd as V
    import workloads as W
    models, boxes = list(cfg.models), cfg.box_array()
    F = ft.size - 1
    n_nodes = cp.size
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    thb, xb = V.bank_build(models, boxes, cfg.n_draws, cfg.infer_seed, cp, ft, cfg.dt)
    e1.record()
    torch.cuda.synchronize()
    build_ms = e0.elapsed_time(e1)
    M = len(models)
    res = {"moments": torch.empty((cfg.n_voxels, M, 8, 2), dtype=torch.float32, device=y_dev.device),
           "model_prob": torch.empty((cfg.n_voxels, M), dtype=torch.float32, device=y_dev.device)}

    scan_ms = []

    def step(timed):
        r = V.infer_bank(y_dev, ft, cfg.dt, n_nodes, models, cfg.n_draws, cfg.accept_frac, thb, xb, out=res,
                         bank_scan=scan, time_scan=timed, decay_lambda=cfg.decay_lambda)
        if timed:
            scan_ms.append(r["scan_ms"])

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        step(True)  # the scan kernel is bracketed by HIP events inside the call
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    call_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    kern_ms = float(np.mean(scan_ms))
    ki_rmse = None
    if models == [W.M_2TCM_IRR]:  # the posterior mean of Ki against the truth
        th, _ = cfg.truth()
        ki = th[:, 0].astype(np.float64) * th[:, 2] / (th[:, 1] + th[:, 2])
        m = res["moments"][:, 0, 5, 0].cpu().numpy().astype(np.float64)
        ki_rmse = float(np.sqrt(np.nanmean((m - ki) ** 2)))
    n = V.accept_count(M * cfg.n_draws, cfg.accept_frac)
    n_tot = M * cfg.n_draws
    pairs = cfg.n_voxels * n_tot
    if scan == "bf16":
        # the contraction d - a = sum_k A_vk B_gk over K = 2F real terms: one
        # multiply-add per term and pair (the hi/lo split, the error-bound
        # product and the padding of F to a multiple of 8 are not counted)
        fpp = 2 * 2 * F
        ld = int(V.lib.vpet_abc_bank_ld(F))
        peak, bound = PEAK_BF16_MFMA_TFLOPS, "mfma"
        kname = f"vpet_bank_mfma{'' if ld <= 32 else '_wide'}_kernel<{2 * ld}, false> (BF16 contraction scan)"
        pilot = min(n_tot, -(-11 * n_tot // (2 * n)))
    else:
        fpp = 4 * F  # per frame: subtract, weight, fused multiply-add
        ld = int(V.lib.vpet_abc_bank_ld(F))
        peak, bound, kname = PEAK_F64_VECTOR_TFLOPS, "alu", f"vpet_bank_scan_kernel<{ld}, false, false> (FP64 scan)"
        pilot = min(n_tot, -(-4 * n_tot // n))
    achieved = pairs * fpp / (kern_ms * 1e-3) / 1e12
    out = {"value": cfg.n_voxels / (ms * 1e-3), "unit": "voxels/s", "ms_per_step": round(ms, 3),
           "call_ms_hip_events": round(call_ms, 3), "bank_build_ms": round(build_ms, 3), "ki_rmse": ki_rmse,
           "dtype": "bf16x3 contraction + f64 re-rank" if scan == "bf16" else "f64",
           "config": {"bank_draws": n_tot, "draws": "one Philox4x32-10 bank (stream 1) for all voxels",
                      "n_accept": n, "pilot_rows": pilot, "scan": scan},
           "roofline": {"bound": bound, "achieved": round(achieved, 3), "peak": peak,
                        "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                        "traffic": traffic_from_profiles(cfg.name, "vpet_bank_mfma_kernel") if scan == "bf16" else None,
                        "kernel": kname, "kernel_ms": round(kern_ms, 3), "flops_per_pair": fpp}}
    if cpu:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
        threads = max(1, min(threads, 64))
        t0 = time.perf_counter()
        oracle.bank(models, boxes, cfg.n_draws, cfg.infer_seed, cp, cfg.dt, ft)
        bank_s = time.perf_counter() - t0
        nv = threads
        t0 = time.perf_counter()
        oracle.infer_bank(y_host[:nv], ft, cp, cfg.dt, models, boxes, cfg.n_draws, cfg.accept_frac, cfg.infer_seed,
                          nthreads=threads, lam=cfg.decay_lambda)
        per_vox = max(time.perf_counter() - t0 - bank_s, 1e-6) / nv
        nv = int(min(cfg.n_voxels, max(threads, min(4096, budget_s / per_vox))))
        t0 = time.perf_counter()
        ref = oracle.infer_bank(y_host[:nv], ft, cp, cfg.dt, models, boxes, cfg.n_draws, cfg.accept_frac,
                                cfg.infer_seed, nthreads=threads, lam=cfg.decay_lambda)
        dt = time.perf_counter() - t0
        g = V.infer_bank(y_dev[:nv].contiguous(), ft, cfg.dt, n_nodes, models, cfg.n_draws, cfg.accept_frac, thb, xb,
                         debug=True, decay_lambda=cfg.decay_lambda)
        torch.cuda.synchronize()
        idx = g["accept_idx"].cpu().numpy()
        mom = g["moments"].cpu().numpy().astype(np.float64)
        same = np.array([set(a.tolist()) == set(b.tolist()) for a, b in zip(idx, ref["accept_idx"])])
        ok = ~np.isnan(ref["moments"])
        ok[..., 1] = False
        rel = np.abs(mom[same] - ref["moments"][same])[ok[same]] / np.abs(ref["moments"][same][ok[same]])
        out["cpu_baseline"] = {"value": nv / (dt - bank_s) if dt > bank_s else None, "unit": "voxels/s",
                               "cores": threads, "kind": "oracle", "cpu_model": host_cpu(),
                               "sample": f"first {nv} voxels against the same {M * cfg.n_draws}-row bank, FP64 "
                                         f"({dt:.1f} s incl. a {bank_s:.1f} s bank build, excluded)"}
        out["error_vs_oracle"] = {"voxels": int(nv), "identical_accepted_sets": int(same.sum()),
                                  "max_rel_err_posterior_mean_identical_sets":
                                      float(rel.max()) if rel.size else None}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["large", "small", "lpnt", "tbpet", "learned"], default="large",
                    help="large: 1M voxels x 100k draws (default); small: 1024 voxels x 2000 draws; lpnt: MRTM vs "
                         "lp-ntPET model selection, 1.56M voxels against a 400k-row shared bank (bank form only); "
                         "tbpet: a 10.9M-voxel volume streamed from a file against a 1M-row bank; learned: the large "
                         "volume with 20k draws per voxel from a trained proposal network (importance-weighted), "
                         "compared with plain ABC at 100k and 1M prior draws")
    ap.add_argument("--scratch-dir", default="/tmp", help="tbpet: where the volume file and outputs are written")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bank", action="store_true", help="skip the shared-bank form")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal form")
    ap.add_argument("--bank-scan", choices=["bf16", "f64"], default="bf16",
                    help="pair screening of the shared-bank form: BF16 matrix cores or FP64 vector ALUs")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (HBM counter calibration)")
    ap.add_argument("--no-extra", action="store_true",
                    help="large: skip the MRTM/lp-ntPET and total-body sub-objects")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); voxels are independent, so "
              "a multi-GPU run is one process per GPU on disjoint voxel ranges with no exchange.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2603_14859_amd as V
    import workloads as W
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.workload == "lpnt":
        main_reference(args, dev)
        return
    if args.workload == "tbpet":
        main_tbpet(args, dev)
        return
    if args.workload == "learned":
        main_learned(args, dev)
        return
    cfg = W.CFG_LARGE if args.workload == "large" else W.CFG_SMALL
    ft, cp, y_host = make_inputs(cfg, dev)
    y = torch.from_numpy(y_host).to(dev)
    models, boxes = list(cfg.models), cfg.box_array()
    n_steps = int(round(float(ft[-1] - ft[0]) / np.float32(cfg.dt)))
    F = ft.size - 1

    def step(out):
        return V.infer(y, ft, cp, cfg.dt, models, boxes, cfg.n_draws, cfg.accept_frac, cfg.infer_seed,
                       out=out)

    M = len(models)
    res = {"moments": torch.empty((cfg.n_voxels, M, 8, 2), dtype=torch.float32, device=dev),
           "model_prob": torch.empty((cfg.n_voxels, M), dtype=torch.float32, device=dev)}
    for _ in range(args.warmup):
        step(res)
    torch.cuda.synchronize()
    if args.copy_calibration:
        # a plain copy of 1 GiB whose source was evicted from the 256 MB
        # last-level cache by 1 GiB of other writes (reads 1 GiB, writes 1 GiB)
        a = torch.empty(256 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        flush = torch.empty_like(a).fill_(2.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b, flush

    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ev[s][0].record(stream)
        step(res)
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = wall * 1e3 / args.steps
    kernel_ms = float(np.mean(launch_ms))

    # once more end to end: the TACs from pinned host memory to the device, the
    # call, the outputs back to pinned host memory (not the line's value)
    y_pin = torch.from_numpy(y_host).pin_memory()
    outs = {k: v for k, v in res.items() if torch.is_tensor(v)}
    out_pin = {k: torch.empty(v.shape, dtype=v.dtype).pin_memory() for k, v in outs.items()}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y_e2e = y_pin.to(dev, non_blocking=True)
    V.infer(y_e2e, ft, cp, cfg.dt, models, boxes, cfg.n_draws, cfg.accept_frac, cfg.infer_seed, out=res)
    for k, v in outs.items():
        out_pin[k].copy_(v, non_blocking=True)
    torch.cuda.synchronize()
    e2e_s = time.perf_counter() - t0
    del y_e2e, y_pin, out_pin

    fl = flops_per_draw(n_steps, F) * cfg.n_voxels * cfg.n_draws * len(models)
    achieved = fl / (kernel_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_F64_VECTOR_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_F64_VECTOR_TFLOPS, 4),
                "traffic": traffic_from_profiles(cfg.name),
                "kernel": KERNEL_NAME, "kernel_ms": round(kernel_ms, 3),
                "flops_per_draw": flops_per_draw(n_steps, F)}

    out = {"metric": METRIC, "value": cfg.n_voxels / (ms_per_step * 1e-3), "unit": "voxels/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded Feng input, uniform prior truths, Gaussian frame noise)",
           "config": {"workload": cfg.name, "voxels": cfg.n_voxels, "frames": F, "minutes": float(ft[-1]),
                      "grid_dt_min": cfg.dt, "draws_per_voxel": cfg.n_draws, "accept_frac": cfg.accept_frac,
                      "n_accept": V.accept_count(M * cfg.n_draws, cfg.accept_frac), "models": ["2TCM-irreversible"], "draws": "per-voxel Philox4x32-10",
                      "parallelism": "single GPU"},
           "roofline": roofline,
           "end_to_end_voxels_per_s": cfg.n_voxels / e2e_s,
           "end_to_end_note": "TACs host->device, the call, outputs device->host (pinned host memory), one run"}
    if not args.no_cpu_baseline:
        base, err = cpu_baseline(cfg, ft, cp, y_host, y, args.cpu_budget)
        out["cpu_baseline"] = base
        out["error_vs_oracle"] = err
    if not args.no_bank and F <= V.BANK_MAX_FRAMES:
        out["bank_form"] = bank_form(cfg, ft, cp, y_host, y, args.steps, args.warmup, not args.no_cpu_baseline,
                                     args.cpu_budget / 3, args.bank_scan)
    if not args.no_learned and cfg.name == W.CFG_LARGE.name:
        m_plain = res["moments"][:, 0, 5].cpu().numpy().astype(np.float64)
        del res
        lf = learned_form(cfg, ft, cp, y_host, y, args.steps, args.warmup, not args.no_cpu_baseline,
                          args.cpu_budget / 3, m_plain=m_plain)
        lf["comparison"]["plain_100k_voxels_per_s"] = out["value"]
        ctx = lf.pop("_ctx")
        out["learned_proposal"] = lf
        if not args.no_bank:
            ctx["plain"] = {"per_voxel_100k": {"voxels_per_s": out["value"], "ki_rmse": lf["comparison"]["ki_rmse_plain_100k"]},
                            "bank_100k": {"voxels_per_s": out["bank_form"]["value"],
                                          "ki_rmse": out["bank_form"]["ki_rmse"]}}
            out["learned_bank"] = learned_bank_form(cfg, ft, cp, y_host, y, args.steps, args.warmup, ctx,
                                                    not args.no_cpu_baseline, args.cpu_budget / 3)
        del ctx
    if cfg.name == W.CFG_LARGE.name and not args.no_extra:
        import torch
        torch.cuda.empty_cache()
        sub = max(1, min(args.steps, 3))
        out["lpnt"] = reference_form(args, dev, sub, 1)
        torch.cuda.empty_cache()
        out["tbpet"] = tbpet_form(args, dev)
    print(json.dumps(out), flush=True)


def learned_form(cfg, ft, cp, y_host, y, steps: int, warmup: int, cpu: bool, budget_s: float, m_plain=None):
    """Importance-weighted ABC with a learned proposal on the same volume: the
    network is trained once on 10.24M noisy simulations (5000 Adam steps of
    2048 rows of a 1M-draw bank, fresh noise per pass; outside the timed
    region), then one step = network forward pass + 20k proposal draws per
    voxel (defensive prior share 0.1, sd x 1.5), n = 100 accepted.  Plain ABC
    at 100k prior draws (the whole volume; m_plain if the caller has it) and at
    1M prior draws (a 64k-voxel subset) gives the error / throughput
    comparison.  Returns a dict for the JSON line."""
    import math

    import torch

    import paper_2603_14859_amd as V
    import workloads as W
    IRR = W.M_2TCM_IRR
    dev = y.device
    th, _ = cfg.truth()
    ki = th[:, 0].astype(np.float64) * th[:, 2] / (th[:, 1] + th[:, 2])
    box = cfg.box_array()
    F = ft.size - 1
    n_steps = int(round(float(ft[-1] - ft[0]) / np.float32(cfg.dt)))
    n_is, n_acc, share, scale = 20_000, 100, 0.1, 1.5
    train = {"bank_draws": 1_000_000, "steps": 5000, "batch": 2048, "lr": 5e-4, "noise_level": 0.05}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    thb, xb = V.bank_build([IRR], box, train["bank_draws"], 17, cp, ft, cfg.dt)
    params = V.proposal_init(2)
    losses = V.proposal_train(params, thb, xb, ft, steps=train["steps"], batch=train["batch"], lr=train["lr"],
                              noise_level=train["noise_level"], decay_lambda=W.LAMBDA_F18, seed=9)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del thb, xb
    nv = cfg.n_voxels
    prop_out = torch.empty((nv, V.PROPOSAL_NOUT), dtype=torch.float32, device=dev)
    res = {"moments": torch.empty((nv, 1, 8, 2), dtype=torch.float32, device=dev),
           "model_prob": torch.empty((nv, 1), dtype=torch.float32, device=dev),
           "ess": torch.empty((nv,), dtype=torch.float32, device=dev)}
    stream = torch.cuda.current_stream()

    def step(ev=None):
        V.proposal_forward(params, y, out=prop_out)
        if ev is not None:
            ev[0].record(stream)
        V.infer(y, ft, cp, cfg.dt, [IRR], box, n_is, n_acc / n_is, cfg.infer_seed, proposal=prop_out,
                prior_share=share, sd_scale=scale, out=res)
        if ev is not None:
            ev[1].record(stream)

    for _ in range(warmup):
        step()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        step(ev[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ms_per_step = wall * 1e3 / steps
    m_is = res["moments"][:, 0, 5].cpu().numpy().astype(np.float64)
    ess = res["ess"].cpu().numpy().astype(np.float64)
    del res, prop_out

    # plain ABC: 100k prior draws over the whole volume, 1M on a subset
    if m_plain is None:
        r100 = V.infer(y, ft, cp, cfg.dt, [IRR], box, 100_000, n_acc / 100_000, cfg.infer_seed)
        m_plain = r100["moments"][:, 0, 5].cpu().numpy().astype(np.float64)
        del r100
    sub = 65536
    y_sub = y[:sub].contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r1m = V.infer(y_sub, ft, cp, cfg.dt, [IRR], box, 1_000_000, n_acc / 1_000_000, cfg.infer_seed, debug=True)
    torch.cuda.synchronize()
    t1m = time.perf_counter() - t0
    m1m = r1m["moments"][:, 0, 5].cpu().numpy().astype(np.float64)
    h1m = r1m["threshold"]
    del r1m

    # the judge: importance-weighted ABC restricted to plain-1M's own per-voxel
    # thresholds (the same ABC target, the prior on {d <= h_v}): 20k proposal
    # draws, the 3900 closest kept, those at or below h_v weighted
    n_keep = 3900
    rj = V.infer(y_sub, ft, cp, cfg.dt, [IRR], box, n_is, n_keep / n_is, cfg.infer_seed, debug=True,
                 proposal=V.proposal_forward(params, y_sub), prior_share=share, sd_scale=scale, accept_below=h1m)
    mj = rj["moments"][:, 0, 5].cpu().numpy().astype(np.float64)
    ess_j = rj["ess"].cpu().numpy().astype(np.float64)
    covered = (rj["threshold"] > h1m).cpu().numpy()
    del rj
    within_j = np.abs(mj[:, 0] - m1m[:, 0]) <= 3.0 * np.sqrt(mj[:, 1] / ess_j + m1m[:, 1] / n_acc)
    judge = {"voxels": sub, "plain_prior_draws": 1_000_000, "plain_accepted": n_acc, "learned_draws": n_is,
             "learned_kept": n_keep, "frac_covered": float(covered.mean()),
             "median_ess_at_common_threshold": float(np.nanmedian(ess_j[covered])),
             "frac_ki_within_3_mc_se": float(np.mean(within_j[covered])),
             "note": "h_v = plain ABC's 100th distance of 1M prior draws; covered = the learned run kept every "
                     "proposal draw at or below h_v (its 3900th distance exceeds h_v); SE = sqrt(var_IS / ESS + "
                     "var_plain / 100)"}

    # equal-error sweep on the subset: plain ABC at 100k and 1M prior draws
    # against the learned proposal at a range of draw counts (network forward
    # pass included), n = 100 accepted throughout
    def timed(n_draws, proposal):
        torch.cuda.synchronize()
        t = time.perf_counter()
        kw = {}
        if proposal:
            kw = dict(proposal=V.proposal_forward(params, y_sub), prior_share=share, sd_scale=scale)
        r = V.infer(y_sub, ft, cp, cfg.dt, [IRR], box, n_draws, n_acc / n_draws, cfg.infer_seed, **kw)
        torch.cuda.synchronize()
        dt_ = time.perf_counter() - t
        m = r["moments"][:, 0, 5, 0].cpu().numpy().astype(np.float64)
        return {"draws": n_draws, "ki_rmse": float(math.sqrt(np.nanmean((m - ki[:sub]) ** 2))),
                "voxels_per_s": sub / dt_}
    timed(2500, True)  # warm-up of the subset shapes
    plain_pts = [timed(100_000, False), {"draws": 1_000_000, "ki_rmse": None, "voxels_per_s": sub / t1m}]
    plain_pts[1]["ki_rmse"] = float(math.sqrt(np.nanmean((m1m[:, 0] - ki[:sub]) ** 2)))
    learned_pts = [timed(nd, True) for nd in (2500, 5000, 10_000, 20_000)]
    equal_error = {"subset_voxels": sub, "plain": plain_pts, "learned": learned_pts}
    for pp in plain_pts:  # the fewest learned draws at or below this plain error, and the throughput ratio
        ok = [q for q in learned_pts if q["ki_rmse"] <= pp["ki_rmse"]]
        key = f"speedup_at_plain_{pp['draws'] // 1000}k_error"
        equal_error[key] = (round(ok[0]["voxels_per_s"] / pp["voxels_per_s"], 2) if ok else None)

    def rmse(m, n=nv):
        return float(math.sqrt(np.nanmean((m[:n, 0] - ki[:n]) ** 2)))

    fl = flops_per_draw(n_steps, F) * nv * n_is
    achieved = fl / (kernel_ms * 1e-3) / 1e12
    out = {"value": nv / (ms_per_step * 1e-3), "unit": "voxels/s", "ms_per_step": round(ms_per_step, 3),
           "dtype": "f64 simulation, bf16x3 network (fp32 accumulation)",
           "config": {"voxels": nv, "proposal_draws_per_voxel": n_is, "n_accept": n_acc, "prior_share": share,
                      "sd_scale": scale, "models": ["2TCM-irreversible"]},
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_F64_VECTOR_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / PEAK_F64_VECTOR_TFLOPS, 4),
                        "traffic": traffic_from_profiles(cfg.name.replace("100kdraws", "learned20k"),
                                                         "vpet_infer_is_kernel"),
                        "kernel": "vpet_infer_is_kernel", "kernel_ms": round(kernel_ms, 3),
                        "flops_per_draw": flops_per_draw(n_steps, F)},
           "training": {**train, "samples": train["steps"] * train["batch"], "seconds": round(train_s, 2),
                        "loss_first_100": float(losses[:100].mean()), "loss_last_100": float(losses[-100:].mean())},
           "comparison": {
               "ki_rmse_learned_20k": rmse(m_is), "ki_rmse_plain_100k": rmse(m_plain),
               "subset_voxels": sub, "ki_rmse_learned_20k_subset": rmse(m_is, sub),
               "ki_rmse_plain_1M_subset": rmse(m1m, sub), "plain_1M_voxels_per_s": sub / t1m,
               "median_ess": float(np.nanmedian(ess))},
           "judge_common_threshold": judge,
           "equal_error": equal_error,
           "_ctx": {"params": params, "h1m": h1m, "m1m": m1m, "sub": sub, "t1m": t1m, "ki": ki, "share": share,
                    "scale": scale}}
    if cpu:
        import oracle.proposal as prop
        rng = np.random.default_rng(0)
        t0 = time.perf_counter()
        done = 0
        while time.perf_counter() - t0 < budget_s or done == 0:
            # a mixture centred near the voxel's truth (the oracle's cost does
            # not depend on the mixture: every draw is simulated)
            o = np.zeros(V.PROPOSAL_NOUT)
            o[8:40] = np.tile(np.log(np.maximum(th[done, [0, 1, 2, 4]], 1e-3)), 8) + 0.2 * rng.standard_normal(32)
            o[40:72] = 0.4
            prop.infer_is(y_host[done], ft, cp, cfg.dt, box[0], o, n_is, n_acc / n_is, cfg.infer_seed, done,
                          prior_share=share, sd_scale=scale)
            done += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done / dt, "unit": "voxels/s", "cores": 1, "kind": "oracle",
                               "cpu_model": host_cpu(),
                               "sample": f"first {done} voxels, {n_is} proposal draws each, FP64 numpy + C "
                                         f"(single thread, {dt:.1f} s)"}
    return out


def main_learned(args, dev):
    """The learned-proposal form as the line's value (see learned_form); plain
    ABC at 100k draws is timed once for the comparison."""
    import torch

    import paper_2603_14859_amd as V
    import workloads as W
    cfg = W.CFG_LARGE
    ft, cp, y_host = make_inputs(cfg, dev)
    y = torch.from_numpy(y_host).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r100 = V.infer(y, ft, cp, cfg.dt, [W.M_2TCM_IRR], cfg.box_array(), 100_000, 0.001, cfg.infer_seed)
    torch.cuda.synchronize()
    t100 = time.perf_counter() - t0
    m100 = r100["moments"][:, 0, 5].cpu().numpy().astype(np.float64)
    del r100
    lf = learned_form(cfg, ft, cp, y_host, y, args.steps, args.warmup, not args.no_cpu_baseline, args.cpu_budget,
                      m_plain=m100)
    lf.pop("_ctx")
    lf["comparison"]["plain_100k_voxels_per_s"] = cfg.n_voxels / t100
    out = {"metric": METRIC, "value": lf["value"], "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": lf["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": lf["dtype"],
           "data": "synthetic (seeded Feng input, uniform prior truths, Gaussian frame noise); network trained on "
                   "simulations of the same forward model",
           "config": {"workload": cfg.name + "-learned-proposal", "frames": ft.size - 1, "minutes": float(ft[-1]),
                      "grid_dt_min": cfg.dt, **lf["config"], "parallelism": "single GPU"},
           "roofline": lf["roofline"], "training": lf["training"], "comparison": lf["comparison"],
           "judge_common_threshold": lf["judge_common_threshold"],
           "equal_error": lf["equal_error"]}
    if "cpu_baseline" in lf:
        out["cpu_baseline"] = lf["cpu_baseline"]
    print(json.dumps(out), flush=True)


LB_SETTINGS = {"dims": 4, "bins": 8, "group_voxels": 1024, "prior_share": 0.1, "sd_scale": 1.0}


def learned_bank_form(cfg, ft, cp, y_host, y, steps: int, warmup: int, ctx, cpu: bool, budget_s: float):
    """The shared bank drawn from the learned proposal on the same volume: the
    network of the learned-proposal form groups the voxels (cells of its
    posterior means, groups of 1024 voxels) and each group gets a bank of
    n_bank rows from its Gaussian mixed with the prior (share 0.1); rows carry
    prior / proposal weights; n = 100 accepted.  One step = network forward
    pass + vpet_abc_infer_bank_learned.  A sweep over n_bank gives the Ki
    error against the truth; the line's value is the 10k-row setting; plain
    ABC (per voxel and shared bank, 100k prior draws; 1M prior draws on a
    64k-voxel subset) is the comparison, and the judge compares Ki means with
    plain ABC at 1M prior draws at plain ABC's own thresholds."""
    import math

    import torch

    import paper_2603_14859_amd as V
    import workloads as W
    IRR = W.M_2TCM_IRR
    box = cfg.box_array()
    params, ki, n_acc = ctx["params"], ctx["ki"], 100
    nv = cfg.n_voxels
    F = ft.size - 1
    stream = torch.cuda.current_stream()
    res = {"moments": torch.empty((nv, 1, 8, 2), dtype=torch.float32, device=y.device),
           "model_prob": torch.empty((nv, 1), dtype=torch.float32, device=y.device),
           "ess": torch.empty((nv,), dtype=torch.float32, device=y.device)}
    prop_out = torch.empty((nv, V.PROPOSAL_NOUT), dtype=torch.float32, device=y.device)

    def run(n_bank, ys=y, out=res, po=prop_out, timed=False, **kw):
        V.proposal_forward(params, ys, out=po)
        return V.infer_bank_learned(ys, ft, cp, cfg.dt, [IRR], box, po, n_bank, n_acc / n_bank, cfg.infer_seed,
                                    out=out, time_scan=timed, **LB_SETTINGS, **kw)

    def rmse(m):
        return float(math.sqrt(np.nanmean((m - ki) ** 2)))

    sweep = []
    for nb in (2500, 5000, 10_000, 20_000):
        run(nb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(nb)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        m = res["moments"][:, 0, 5, 0].cpu().numpy().astype(np.float64)
        sweep.append({"bank_rows_per_group": nb, "voxels_per_s": nv / dt, "ki_rmse": rmse(m),
                      "median_ess": float(np.nanmedian(res["ess"].cpu().numpy()))})
    n_bank = 10_000
    for _ in range(warmup):
        run(n_bank)
    torch.cuda.synchronize()
    scan_ms = []
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        r = run(n_bank, timed=True)
        scan_ms.append(r["scan_ms"])
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    call_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    kern_ms = float(np.mean(scan_ms))
    groups = -(-nv // LB_SETTINGS["group_voxels"])
    fpp = 2 * 2 * F
    achieved = nv * n_bank * fpp / (kern_ms * 1e-3) / 1e12
    m_lb = res["moments"][:, 0, 5, 0].cpu().numpy().astype(np.float64)
    # equal error: the fewest bank rows whose Ki error is at or below each plain point's
    plain = dict(ctx["plain"])
    plain["per_voxel_1M_subset"] = {"voxels_per_s": ctx["sub"] / ctx["t1m"],
                                    "ki_rmse_subset": float(math.sqrt(np.nanmean((ctx["m1m"][:, 0] - ki[:ctx["sub"]]) ** 2)))}
    equal = {}
    for key in ("per_voxel_100k", "bank_100k"):
        ok = [q for q in sweep if q["ki_rmse"] <= plain[key]["ki_rmse"]]
        equal[f"speedup_vs_plain_{key}_at_its_error"] = (round(ok[0]["voxels_per_s"] / plain[key]["voxels_per_s"], 2)
                                                          if ok else None)
        equal[f"bank_rows_at_plain_{key}_error"] = ok[0]["bank_rows_per_group"] if ok else None
    # the judge: at plain-1M's own per-voxel thresholds on the subset (500 kept)
    sub = ctx["sub"]
    ys = y[:sub].contiguous()
    po = torch.empty((sub, V.PROPOSAL_NOUT), dtype=torch.float32, device=y.device)
    V.proposal_forward(params, ys, out=po)
    keep, nb_j = 500, 100_000
    rj = V.infer_bank_learned(ys, ft, cp, cfg.dt, [IRR], box, po, nb_j, keep / nb_j, cfg.infer_seed, debug=True,
                              accept_below=ctx["h1m"], **LB_SETTINGS)
    mj = rj["moments"][:, 0, 5].cpu().numpy().astype(np.float64)
    ess_j = rj["ess"].cpu().numpy().astype(np.float64)
    covered = (rj["threshold"] > ctx["h1m"]).cpu().numpy()
    del rj, po, ys
    m1m = ctx["m1m"]
    within = np.abs(mj[:, 0] - m1m[:, 0]) <= 3.0 * np.sqrt(mj[:, 1] / ess_j + m1m[:, 1] / n_acc)
    judge = {"voxels": sub, "plain_prior_draws": 1_000_000, "plain_accepted": n_acc, "bank_rows_per_group": nb_j,
             "kept": keep, "frac_covered": float(covered.mean()),
             "median_ess_at_common_threshold": float(np.nanmedian(ess_j[covered])),
             "frac_ki_within_3_mc_se": float(np.mean(within[covered])),
             "note": "grouping made within the subset; h_v = plain ABC's 100th distance of 1M prior draws"}
    out = {"value": nv / (ms * 1e-3), "unit": "voxels/s", "ms_per_step": round(ms, 3),
           "call_ms_hip_events": round(call_ms, 3), "ki_rmse": rmse(m_lb),
           "dtype": "bf16x3 contraction + f64 re-rank, f64 simulation, bf16x3 network",
           "config": {"voxels": nv, "bank_rows_per_group": n_bank, "groups": groups, "n_accept": n_acc,
                      **LB_SETTINGS, "models": ["2TCM-irreversible"],
                      "step": "network forward pass + grouping + group banks (draw, simulate) + BF16 scan + "
                              "select + weighted reduction"},
           "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_BF16_MFMA_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / PEAK_BF16_MFMA_TFLOPS, 4),
                        "traffic": traffic_from_profiles(cfg.name.replace("100kdraws", "learnedbank10k"),
                                                         "vpet_bank_mfma_kernel"),
                        "kernel": f"vpet_bank_mfma_kernel<{2 * int(V.lib.vpet_abc_bank_ld(F))}, false> (BF16 scan)",
                        "kernel_ms": round(kern_ms, 3), "flops_per_pair": fpp},
           "sweep": sweep, "plain": plain, "equal_error": equal, "judge_common_threshold": judge}
    if cpu:
        # the oracle of the learned bank on one group (the network outputs it
        # groups are synthetic mixtures near the truths: its cost does not
        # depend on them)
        import oracle.learned_bank as olb
        from oracle.proposal import C as NC
        th, _ = cfg.truth(1024)
        rng = np.random.default_rng(0)
        o = np.zeros((1024, 96))
        o[:, NC:NC + 32] = (np.tile(np.log(np.maximum(th[:, [0, 1, 2, 4]], 1e-3)), 8)
                            + 0.2 * rng.standard_normal((1024, 32)))
        o[:, NC + 32:NC + 64] = -1.0
        t0 = time.perf_counter()
        olb.infer_bank_learned(y_host[:1024], ft, cp, cfg.dt, [IRR], box, o, n_bank, n_acc / n_bank, cfg.infer_seed,
                               **LB_SETTINGS)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1024 / dt, "unit": "voxels/s", "cores": 1, "kind": "oracle",
                               "cpu_model": host_cpu(),
                               "sample": f"one 1024-voxel group against its {n_bank}-row bank (built and counted), "
                                         f"FP64 numpy + C (single thread, {dt:.1f} s)"}
    return out


def tbpet_form(args, dev):
    """Total-body scale: a 150 x 150 x 486 volume (irreversible / reversible
    2TCM mixture) written to a file, then streamed in 1M-voxel chunks (file ->
    GPU -> file, resumable): (a) against one shared prior bank of 1M draws
    (500k per model), (b) with the learned proposal: a network with a
    five-parameter head trained on reversible-2TCM simulations groups each
    chunk's voxels, and every group gets a bank of 10k draws per model from its
    proposal (weights prior / proposal).  Model selection and the Ki of the
    preferred model are compared with the truth for both."""
    import torch

    import paper_2603_14859_amd as V
    import workloads as W
    cfg = W.CFG_TBPET
    ft, cp = cfg.frame_times, cfg.input_fn()
    F, M = ft.size - 1, len(cfg.models)
    models, boxes = list(cfg.models), cfg.box_array()
    th, rev, eps = cfg.truth_mixture()
    path = os.path.join(args.scratch_dir, f"vpet_{cfg.name}.f32")
    prefix = os.path.join(args.scratch_dir, f"vpet_{cfg.name}_out")
    t0 = time.perf_counter()
    chunk = 1 << 20
    with open(path, "wb") as fh:  # input preparation: noise-free curves on the GPU, noise on the host
        for v0 in range(0, cfg.n_voxels, chunk):
            sl = slice(v0, min(cfg.n_voxels, v0 + chunk))
            t = torch.from_numpy(th[sl]).to(dev)
            r = torch.from_numpy(rev[sl]).to(dev)
            clean = torch.where(r[:, None], V.simulate(W.M_2TCM_REV, t, cp, ft, cfg.dt),
                                V.simulate(W.M_2TCM_IRR, t, cp, ft, cfg.dt))
            W.add_noise(clean.cpu().numpy(), ft, eps[sl]).tofile(fh)
    prep_s = time.perf_counter() - t0
    del eps
    ki_true = (th[:, 0].astype(np.float64) * th[:, 2] / (th[:, 1] + th[:, 2]))

    def summary(wall):
        mom, prob = V.load_stream_outputs(prefix, cfg.n_voxels, M)
        p_rev = np.asarray(prob[:, 1])
        ok = ~np.isnan(p_rev)
        ki_post = np.where(p_rev > 0.5, mom[:, 1, 5, 0], mom[:, 0, 5, 0]).astype(np.float64)  # preferred model's Ki
        rel = np.abs(ki_post - ki_true) / ki_true
        return {"voxels_per_s": cfg.n_voxels / wall, "seconds": round(wall, 2),
                "model_selection": {"mean_p_rev_reversible": float(p_rev[ok & rev].mean()),
                                    "mean_p_rev_irreversible": float(p_rev[ok & ~rev].mean()),
                                    "accuracy_p_rev_gt_half": float(np.mean((p_rev[ok] > 0.5) == rev[ok]))},
                "ki_preferred_model": {"median_rel_err": float(np.nanmedian(rel)),
                                       "rmse": float(np.sqrt(np.nanmean((ki_post - ki_true) ** 2)))}}

    # (a) the prior bank
    thb, xb = V.bank_build(models, boxes, cfg.n_draws, cfg.infer_seed, cp, ft, cfg.dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = V.stream_bank(path, cfg.n_voxels, ft, cfg.dt, cp.size, models, cfg.n_draws, cfg.accept_frac, thb, xb,
                         prefix, chunk_voxels=chunk, resume=False)
    plain = summary(time.perf_counter() - t0)
    del thb, xb
    torch.cuda.empty_cache()
    # (b) the learned proposal
    t0 = time.perf_counter()
    thr, xr = V.bank_build([W.M_2TCM_REV], boxes[1:], 1_000_000, 17, cp, ft, cfg.dt)
    params = V.proposal_init(2)
    losses = V.proposal_train(params, thr, xr, ft, steps=5000, batch=2048, lr=5e-4, noise_level=0.05,
                              decay_lambda=W.LAMBDA_F18, seed=9, dims=5)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del thr, xr
    torch.cuda.empty_cache()
    n_acc = 100
    lbk = {"dims": 5, "bins": 4, "prior_share": 0.1, "sd_scale": 1.0}
    sweep = []
    for gv, n_lb in ((1024, 10_000), (1024, 30_000), (1024, 50_000), (1024, 100_000), (4096, 50_000),
                     (4096, 75_000)):
        t0 = time.perf_counter()
        done_l = V.stream_bank_learned(path, cfg.n_voxels, ft, cp, cfg.dt, models, boxes, params, n_lb,
                                       n_acc / (M * n_lb), cfg.infer_seed, prefix, chunk_voxels=chunk, resume=False,
                                       group_voxels=gv, **lbk)
        sweep.append({"group_voxels": gv, "bank_rows_per_model_per_group": n_lb,
                      **summary(time.perf_counter() - t0)})
    # the line's value: the fastest setting whose model-selection accuracy and Ki error of the preferred model are
    # at least as good as the prior bank's (else the most accurate one)
    def as_good(q):
        return (q["model_selection"]["accuracy_p_rev_gt_half"] >= plain["model_selection"]["accuracy_p_rev_gt_half"]
                and q["ki_preferred_model"]["median_rel_err"] <= plain["ki_preferred_model"]["median_rel_err"])
    eq = sorted([q for q in sweep if as_good(q)], key=lambda q: -q["voxels_per_s"])
    learned = eq[0] if eq else min(sweep, key=lambda q: q["ki_preferred_model"]["median_rel_err"])
    for f in (path, prefix + ".moments", prefix + ".prob", prefix + ".progress"):
        if os.path.exists(f):
            os.remove(f)
    n = V.accept_count(M * cfg.n_draws, cfg.accept_frac)
    return {"value": learned["voxels_per_s"], "unit": "voxels/s", "ms_per_step": round(learned["seconds"] * 1e3, 1),
            "dtype": "bf16x3 contraction + f64 re-rank",
            "data": "synthetic (seeded Feng input, uniform prior truths, half reversible, Gaussian frame noise); "
                    "every rate includes reading the volume from a file and writing the outputs (disk -> GPU -> disk)",
            "config": {"workload": cfg.name, "voxels": cfg.n_voxels, "frames": F, "minutes": float(ft[-1]),
                       "models": ["2TCM-irreversible", "2TCM-reversible"], "chunk_voxels": chunk,
                       "chunks": [done, done_l], "input_file_gb": round(cfg.n_voxels * F * 4 / 1e9, 3),
                       "input_prep_s": round(prep_s, 1), "n_accept": n_acc,
                       "value_is": "the learned-proposal stream"},
            "prior_bank": {"bank_draws_per_model": cfg.n_draws, "accept_frac": cfg.accept_frac, "n_accept": n, **plain},
            "learned_bank": {**lbk, "training_s": round(train_s, 2),
                             "training_loss_last_100": float(losses[-100:].mean()), **learned, "sweep": sweep,
                             "at_prior_bank_error": bool(eq)},
            "speedup_learned_vs_prior_bank": round(learned["voxels_per_s"] / plain["voxels_per_s"], 2),
            "speedup_note": "the learned stream's fastest setting (group size, rows per model per group) at which both "
                            "the model-selection accuracy and the median Ki error of the preferred model are at least "
                            "as good as the prior bank's (at_prior_bank_error false: none of the sweep is; the most "
                            "accurate setting is shown)"}


def main_tbpet(args, dev):
    """The total-body workload as the line (see tbpet_form)."""
    tb = tbpet_form(args, dev)
    out = {"metric": METRIC, "value": tb["value"], "unit": "voxels/s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": tb["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           **{k: v for k, v in tb.items() if k not in ("value", "unit", "ms_per_step")}}
    out["config"]["parallelism"] = "single GPU"
    print(json.dumps(out), flush=True)


def reference_form(args, dev, steps, warmup):
    """MRTM vs lp-ntPET model selection on a reference-region input (the
    shared-bank form; the per-voxel path does not run these models)."""
    import torch

    import paper_2603_14859_amd as V
    import workloads as W
    cfg = W.CFG_LPNT
    ft, cr = cfg.frame_times, cfg.input_fn()
    th, active, eps = cfg.truth_reference()
    F = ft.size - 1
    clean = np.empty((cfg.n_voxels, F), dtype=np.float32)
    a, z = np.nonzero(active)[0], np.nonzero(~active)[0]
    clean[a] = V.simulate(W.M_LPNTPET, torch.from_numpy(th[a]).to(dev), cr, ft, cfg.dt).cpu().numpy()
    clean[z] = V.simulate(W.M_MRTM, torch.from_numpy(th[z]).to(dev), cr, ft, cfg.dt).cpu().numpy()
    y_host = W.add_noise(clean, ft, eps, lam=cfg.decay_lambda)
    del clean
    y = torch.from_numpy(y_host).to(dev)
    bank = bank_form(cfg, ft, cr, y_host, y, steps, warmup, not args.no_cpu_baseline, args.cpu_budget,
                     args.bank_scan)
    models = list(cfg.models)
    thb, xb = V.bank_build(models, cfg.box_array(), cfg.n_draws, cfg.infer_seed, cr, ft, cfg.dt)
    r = V.infer_bank(y, ft, cfg.dt, cr.size, models, cfg.n_draws, cfg.accept_frac, thb, xb,
                     decay_lambda=cfg.decay_lambda, bank_scan=args.bank_scan)
    p = r["model_prob"][:, 1].cpu().numpy()
    del r, thb, xb, y
    out = {"value": bank["value"], "unit": "voxels/s", "ms_per_step": bank["ms_per_step"], "dtype": bank["dtype"],
           "data": "synthetic (one-tissue reference TAC of the seeded Feng input, half the voxels activated, "
                   "Gaussian frame noise, 11C decay)",
           "config": {"workload": cfg.name, "voxels": cfg.n_voxels, "frames": F, "minutes": float(ft[-1]),
                      "grid_dt_min": cfg.dt, "models": ["MRTM", "lp-ntPET"], "bank_draws_per_model": cfg.n_draws,
                      "accept_frac": cfg.accept_frac, "n_accept": bank["config"]["n_accept"],
                      "pilot_rows": bank["config"]["pilot_rows"], "scan": args.bank_scan, "steps": steps},
           "roofline": bank["roofline"],
           "model_selection": {"activated_voxels": int(active.sum()),
                               "mean_p_lpntpet_activated": float(p[active].mean()),
                               "mean_p_lpntpet_null": float(p[~active].mean()),
                               "sensitivity_p_gt_half": float(np.mean(p[active] > 0.5)),
                               "specificity_p_le_half": float(np.mean(p[~active] <= 0.5))}}
    for k in ("cpu_baseline", "error_vs_oracle"):
        if k in bank:
            out[k] = bank[k]
    return out


def main_reference(args, dev):
    """The MRTM / lp-ntPET workload as the line (see reference_form)."""
    rf = reference_form(args, dev, args.steps, args.warmup)
    out = {"metric": METRIC, "value": rf["value"], "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": rf["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, **{k: v for k, v in rf.items() if k not in ("value", "unit", "ms_per_step")}}
    out["config"]["parallelism"] = "single GPU"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
