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
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    """Hash of the HIP sources: a traffic measurement is valid only for the
    kernels it was taken on."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2001_03389_amd", "csrc", "*")))
    files.append(os.path.join(ROOT, "include", "rfim.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, workload: str):
    """Measured HBM bytes per launch from profiles/traffic_<kernel>_<workload>.txt
    (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by a plain copy of known size),
    or None when missing or taken on other kernel sources."""
    path = os.path.join(PROFILES, f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            a, b = line.split("=", 1)
            kv[a.strip()] = b.strip()
    if kv.get("src_hash") != source_hash():
        return None
    return int(float(kv["traffic_bytes_per_launch"]))


def summarize(stats_csv, fetch_csv, write_csv, command, workload):
    """Writes profiles/ summaries from rocprofv3 CSV output (kernel stats, and
    FETCH_SIZE / WRITE_SIZE counter runs that include one plain device copy of
    the batch size as calibration)."""
    import csv
    os.makedirs(PROFILES, exist_ok=True)
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# rocprofv3 kernel statistics, workload {workload}", "",
             f"command: {command}", f"kernel sources: {source_hash()}", "",
             "| kernel | calls | average ms | min ms | max ms | share % |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {r['Name'].split('(')[0]} | {r['Calls']} | {float(r['AverageNs'])/1e6:.4f} | "
                     f"{float(r['MinNs'])/1e6:.4f} | {float(r['MaxNs'])/1e6:.4f} | {float(r['Percentage']):.2f} |")
    with open(os.path.join(PROFILES, f"kernel_stats_{workload}.md"), "w") as f:
        f.write("\n".join(lines) + "\n")

    def per_kernel(path, counter):
        out = {}
        copy = None
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").split("<")[0]
            v = float(r["Counter_Value"])
            if "copyBuffer" in name:
                if copy is None or v > copy:
                    copy = v   # the calibration copy is the largest
                continue
            out.setdefault(name, []).append(v)
        return {k: sum(v) / len(v) for k, v in out.items()}, copy

    fetch, fcopy = per_kernel(fetch_csv, "FETCH_SIZE")
    write, wcopy = per_kernel(write_csv, "WRITE_SIZE")
    copy_bytes = int(os.environ.get("RFIM_COPY_BYTES", 768000000))
    ff = copy_bytes / (fcopy * 1024.0)
    wf = copy_bytes / (wcopy * 1024.0)
    for k in sorted(set(fetch) & set(write)):
        kern = k.split("::")[-1]
        if kern.startswith("k_zero"):
            continue
        rb, wb = fetch[k] * 1024 * ff, write[k] * 1024 * wf
        with open(os.path.join(PROFILES, f"traffic_{kern}_{workload}.txt"), "w") as f:
            f.write(f"# HBM traffic of {kern} per launch, workload {workload}\n")
            f.write(f"# commands: {command} with --pmc FETCH_SIZE, then with --pmc WRITE_SIZE\n")
            f.write(f"# calibration: plain copy of {copy_bytes} bytes read {fcopy:.1f} KiB (FETCH_SIZE) "
                    f"and wrote {wcopy:.1f} KiB (WRITE_SIZE): scale factors {ff:.4f} and {wf:.4f}\n")
            f.write(f"kernel = {kern}\nsrc_hash = {source_hash()}\n")
            f.write(f"fetch_kib_per_launch = {fetch[k]:.1f}\nwrite_kib_per_launch = {write[k]:.1f}\n")
            f.write(f"read_bytes_per_launch = {rb:.0f}\nwrite_bytes_per_launch = {wb:.0f}\n")
            f.write(f"traffic_bytes_per_launch = {rb + wb:.0f}\n")
    print("profiles written", flush=True)


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
    ap.add_argument("--summarize", nargs=3, metavar=("STATS_CSV", "FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/ summaries from rocprofv3 CSV output and exit")
    ap.add_argument("--profile-command", default="")
    args = ap.parse_args()
    if args.summarize:
        summarize(*args.summarize, args.profile_command, f"arts40_{args.replace}")
        return
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
    traffic = read_traffic(dom[0], f"arts40_{args.replace}")
    roof = {"bound": "hbm", "kernel": dom[0], "achieved": round(dom[1]["gbs"], 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom[1]["gbs"] / HBM_PEAK_GBS, 4),
            "traffic": traffic, "algo_bytes": dom[1]["algo_bytes"]}

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
