#!/usr/bin/env python3
"""Throughput of the RFI-mitigation hot path on one MI355X.

One step = one rfim_pipeline_run over the whole 40-beam batch (1536 channels x
12500 samples uint8 per beam): TD 4.0, 3.5, 3.25 then FD 3.0, 2.75 with
32-channel bins, mean replacement, out-of-place, inputs resident in HBM.
Prints one JSON line: GB/s mitigated (input bytes / time), the roofline of the
dominant kernel (algorithmic bytes / its HIP-event duration) and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--replace", choices=["mean", "median"], default="mean")
    ap.add_argument("--beams", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of the batch size (for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); beams are independent, "
              "so N GPUs would each run this workload on their own share.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2001_03389_amd as rf
    import synth

    assert torch.cuda.is_available(), "bench needs a GPU"
    rf.lib()
    dev = torch.device("cuda:0")
    specs = synth.arts40_specs(args.beams)
    steps = synth.STEPS_ARTS40_MEAN if args.replace == "mean" else synth.STEPS_ARTS40_MEDIAN
    log(f"generating {len(specs)} beams ...")
    t = time.time()
    host = [synth.make_beam(s) for s in specs]
    log(f"  {time.time() - t:.1f} s; uploading")
    ins = [torch.from_numpy(h).to(dev) for h in host]
    outs = [torch.empty_like(x) for x in ins]
    torch.cuda.synchronize()
    in_bytes = sum(x.numel() * x.element_size() for x in ins)

    plan = rf.Plan(ins, steps, outputs=outs)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        rf.rfim_pipeline_run(ins, steps, outputs=outs, plan=plan, stream=stream)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup}); timing {args.steps} steps")

    # whole-job throughput
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        rf.rfim_pipeline_run(ins, steps, outputs=outs, plan=plan, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    gbs = in_bytes / (ms_step * 1e-3) / 1e9
    log(f"  {ms_step:.3f} ms/step, {gbs:.1f} GB/s mitigated")

    # per-kernel durations (HIP events around each launch on the launch stream)
    plan.set_timing(True)
    for _ in range(args.steps):
        rf.rfim_pipeline_run(ins, steps, outputs=outs, plan=plan, stream=stream)
    torch.cuda.synchronize()
    kernels = {}
    nelem = sum(x.numel() for x in ins)
    algo_bytes = {rf.RFIM_KERNEL_TD_ROWS_U8: nelem * 1,        # reads every sample once
                  rf.RFIM_KERNEL_FUSED_U8: nelem * 2}          # reads and writes every sample
    for kind, name in rf.KERNEL_NAMES.items():
        n, ms = plan.kernel_times(kind)
        if n:
            avg = ms / n
            kernels[name] = {"launches": n, "avg_ms": avg, "algo_bytes": algo_bytes[kind],
                             "gbs": algo_bytes[kind] / (avg * 1e-3) / 1e9}
    plan.set_timing(False)
    dom = max(kernels.items(), key=lambda kv: kv[1]["avg_ms"] * kv[1]["launches"])
    log("  kernels: " + json.dumps(kernels))
    roof = {"bound": "hbm", "kernel": dom[0], "achieved": round(dom[1]["gbs"], 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom[1]["gbs"] / HBM_PEAK_GBS, 4),
            "traffic": None}

    if args.copy_calibration:
        a = torch.empty(in_bytes, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: {in_bytes} bytes copied")

    counts = plan.flag_counts()
    plan.close()

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        sample = host[0]
        t = time.time()
        oracle.pipeline(sample, steps)
        dt = time.time() - t
        cpu = {"value": round(sample.nbytes / dt / 1e9, 6), "unit": "GB/s", "cores": 1,
               "kind": "oracle", "seconds": round(dt, 2),
               "sample": f"1 of {len(specs)} beams (1536x12500 uint8, 19.2 MB), all {len(steps)} steps, "
                         "single thread"}
        log(f"cpu oracle: {dt:.1f} s for one beam")

    rec = {
        "metric": "GB/s mitigated (% of HBM peak)",
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"{len(specs)} beams x 1536 ch x 12500 samples uint8, "
                               f"TD 4.0/3.5/3.25 + FD 3.0/2.75 (32-ch bins), {args.replace} replacement",
                   "beams": len(specs), "nchan": 1536, "nsamp": 12500,
                   "steps": [[s.domain, s.k, s.replace, s.bin_size] for s in steps],
                   "out_of_place": True},
        "hbm_frac_whole_step": round(2 * in_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "kernels": kernels,
        "flags_per_step_beam0": counts[0],
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
