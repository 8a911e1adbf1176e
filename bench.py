"""Benchmark of the forward semi-Lagrangian step on one MI355X.

Headline workload: the 3-D deformational flow (period T = 3, max speed 2) on a
512^3 periodic grid carrying one slotted sphere, plain FP64 (values, weights,
sums, positions), Z2 with the jump limiter on, dt = 3h/2 (CFL 3), 60 steps
from t = 0 (the run of the configuration; --steps K times K of them).  A step
is one pass of the whole hot path: the lattice trajectories, the limiter's
order words and the reconstruction of the field, run by sl_advance (each
reconstruction launch also integrates the next step's trajectories).  Inputs
are resident in HBM before timing starts.

Prints one JSON line (metric, value, ms_per_step, roofline, cpu_baseline, ...).
With the defaults it also reports the FP32-value form of the same workload,
the split and plain forms at equal L1 error over whole periods, the other
single-GPU configurations (the 1024^2 three-field swirl with its own roofline,
4096^2, the 3-D Fourier flow, solid-body rotation, Burgers, gridded velocity,
the Kelvin wave) and the serving mix.  --workload swirl / fourier3d / kelvin
make another flow the measured workload (used for kernel profiles).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "node-updates/s at fixed L1 error vs FP64 oracle; serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
# The measured workloads whose reconstruction kernel has an HBM traffic record
# (rocprofv3 FETCH_SIZE / WRITE_SIZE): (workload, n, prec) -> (kernel, file).
TRAFFIC = {
    ("deform3d", 512, "f64"): ("recon3d_kernel<double, 1, 3>", "recon3d_deform512_f64_traffic.json"),
    ("swirl", 1024, "f32"): ("recon2d_tiled_kernel<float, 3, 2>", "recon2d_swirl1024_traffic.json"),
}
HEADLINE = ("deform3d", 512, "f64")


_T0 = time.perf_counter()


def note(msg):
    """Progress of a long run, on stderr (the JSON line stays alone on stdout)."""
    print("[bench %7.1f s] %s" % (time.perf_counter() - _T0, msg), file=sys.stderr, flush=True)


def source_hash() -> str:
    """Hash of every HIP source and the C header, to tell whether recorded
    counters still apply to the kernels as built."""
    return all_sources_hash()


def _pmc_mean(csv_path: str, kernel_sub: str, counter: str):
    import csv
    vals = []
    with open(csv_path) as fh:
        for row in csv.DictReader(fh):
            if kernel_sub in row["Kernel_Name"] and row["Counter_Name"] == counter:
                vals.append(float(row["Counter_Value"]))
    return sum(vals) / len(vals) if vals else None


def record_traffic(key, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, command):
    """Turn four rocprofv3 --pmc runs (FETCH_SIZE / WRITE_SIZE of the measured
    workload `key` and of the plain 256 MiB copy) into the traffic record
    bench.py reports for that workload's reconstruction kernel."""
    kernel, fname = TRAFFIC[key]
    f = _pmc_mean(os.path.join(fetch_dir, "run_counter_collection.csv"), kernel, "FETCH_SIZE")
    w = _pmc_mean(os.path.join(write_dir, "run_counter_collection.csv"), kernel, "WRITE_SIZE")
    cf = _pmc_mean(os.path.join(copy_fetch_dir, "run_counter_collection.csv"), "copyBuffer", "FETCH_SIZE")
    cw = _pmc_mean(os.path.join(copy_write_dir, "run_counter_collection.csv"), "copyBuffer", "WRITE_SIZE")
    copy_kib = 64 * 1024 * 1024 * 4 / 1024.0
    ff, fw = copy_kib / cf, copy_kib / cw
    rec = {"kernel": kernel, "workload": "%s_%d_%s" % key,
           "fetch_kib_per_dispatch": f, "write_kib_per_dispatch": w,
           "copy_fetch_kib": cf, "copy_write_kib": cw, "copy_kib": copy_kib,
           "fetch_factor": ff, "write_factor": fw,
           "traffic_bytes_per_launch": (f * ff + w * fw) * 1024.0,
           "source_hash": source_hash(), "command": command}
    os.makedirs(PROFILES, exist_ok=True)
    with open(os.path.join(PROFILES, fname), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


# VALU issue: a wave64 VALU instruction holds one of the 1024 SIMDs (256 CUs x
# 4) for 4 cycles (16 lanes), at 2.4 GHz.  With packed FP32 disabled this is
# the roof of every kernel here (FP64 and FP32 issue at the same rate).
VALU_SIMDS, VALU_CYCLES_PER_INST, CLOCK_HZ = 1024, 4, 2.4e9
VALU_JSON = os.path.join(PROFILES, "valu_counters.json")
# Workload of each counter directory -> the kernels whose counts are kept.
VALU_KERNELS = {"swirl_f32": ["recon2d_tiled_kernel<float, 3, 2>"],
                "swirl4096_f32": ["recon2d_tiled_kernel<float, 3, 2>"],
                "fourier3d_f32": ["recon3d_kernel<float, 3, 4>"],
                "deform3d_f64": ["recon3d_kernel<double, 1, 3>"],
                "deform3d_f32": ["recon3d_kernel<float, 1, 3>"],
                "kelvin_f64": ["recon2d_tiled_kernel<double, 3, 6>", "sw_stage_kernel<double, 2>"]}


def _code_only(text: str) -> str:
    """C/C++ source without its comments and trailing blanks: a record taken
    for the kernels stays valid when only their comments change."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def all_sources_hash() -> str:
    """Hash of the code (comments left out) of every HIP source and the C
    header."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1410_2817_amd", "csrc")
    names = sorted(n for n in os.listdir(csrc) if n.endswith((".h", ".hip")))
    for rel in ["include/sl.h"] + ["paper_1410_2817_amd/csrc/" + n for n in names]:
        h.update(rel.encode())
        with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def record_valu(dirs, command):
    """Instruction counts per wave (SQ_INSTS_VALU / SQ_WAVES and the SALU, LDS
    and memory counts) of the kernels in VALU_KERNELS, from rocprofv3 --pmc
    directories named sqc_<workload>_<prec>."""
    import csv
    import collections
    rec = {"kernels": {}, "source_hash": all_sources_hash(), "command": command}
    for d in dirs:
        key = os.path.basename(os.path.normpath(d))[len("sqc_"):]
        agg = collections.defaultdict(lambda: collections.defaultdict(list))
        with open(os.path.join(d, "run_counter_collection.csv")) as fh:
            for row in csv.DictReader(fh):
                agg[row["Kernel_Name"]][row["Counter_Name"]].append(float(row["Counter_Value"]))
        for want in VALU_KERNELS.get(key, []):
            for name, c in agg.items():
                if want in name:
                    m = {n: sum(v) / len(v) for n, v in c.items()}
                    waves = m["SQ_WAVES"]
                    rec["kernels"]["%s/%s" % (key, want)] = {
                        "waves_per_dispatch": waves,
                        "valu_per_wave": m["SQ_INSTS_VALU"] / waves,
                        "salu_per_wave": m["SQ_INSTS_SALU"] / waves,
                        "lds_per_wave": m["SQ_INSTS_LDS"] / waves,
                        "vmem_rd_per_wave": m["SQ_INSTS_VMEM_RD"] / waves,
                        "vmem_wr_per_wave": m["SQ_INSTS_VMEM_WR"] / waves,
                        "dispatches": len(c["SQ_WAVES"])}
    os.makedirs(PROFILES, exist_ok=True)
    with open(VALU_JSON, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def valu_roof(key, avg_ms):
    """VALU issue roof of a kernel from its recorded instruction count and its
    live average duration: the fraction of the SIMDs' issue cycles its VALU
    instructions fill.  None when the record is missing or stale."""
    try:
        with open(VALU_JSON) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(key)
    if k is None or rec.get("source_hash") != all_sources_hash() or not avg_ms:
        return None
    inst = k["valu_per_wave"] * k["waves_per_dispatch"]
    achieved = inst / (avg_ms * 1e-3)  # wave-instructions per second
    peak = VALU_SIMDS * CLOCK_HZ / VALU_CYCLES_PER_INST
    return {"bound": "alu", "unit": "wave64 VALU instructions/s", "achieved": achieved,
            "peak": peak, "frac": achieved / peak, "valu_per_wave": k["valu_per_wave"],
            "waves": k["waves_per_dispatch"]}


def recorded_traffic(key):
    """Traffic bytes per reconstruction launch of workload `key` from the
    committed counter record, or None when there is none or the kernel sources
    changed since it was taken."""
    if key not in TRAFFIC:
        return None
    try:
        with open(os.path.join(PROFILES, TRAFFIC[key][1])) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != source_hash():
        return None
    return rec.get("traffic_bytes_per_launch")


def recon_bytes_per_node(dim: int, nfields: int, value_bytes: int) -> int:
    """Algorithmic HBM bytes of one mesh-node reconstruction: the lattice
    displacement (FP64 per axis) plus every field value read once and written
    once."""
    return 8 * dim + 2 * value_bytes * nfields


def traj_bytes_per_node(dim: int) -> int:
    """Algorithmic bytes of one lattice-node trajectory: the FP64 displacement
    written once (a fresh lattice reads nothing)."""
    return 8 * dim


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="deform3d",
                    choices=["deform3d", "swirl", "fourier3d", "kelvin"],
                    help="deform3d: the 3-D deformational flow (default, the headline); swirl: "
                         "the 2-D reversing swirl; fourier3d: the 3-D Fourier-mode flow; kelvin: "
                         "the shallow-water Kelvin wave with source terms (profiling runs)")
    ap.add_argument("--n", type=int, default=None,
                    help="grid side (default 512 deform3d, 1024 swirl and kelvin, 256 fourier3d)")
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 60 deform3d, 1280 swirl = one period, "
                         "50 fourier3d, one unit of time kelvin)")
    ap.add_argument("--prec", default=None, choices=["f32", "f64"],
                    help="value precision (default f64 deform3d and kelvin, f32 swirl and "
                         "fourier3d)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving (continuous batching) measurement")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--serving-budget-gib", type=float, default=8.0)
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the precision forms and the other configurations")
    ap.add_argument("--no-events", action="store_true",
                    help="time without kernel events")
    ap.add_argument("--event-period", type=int, default=8,
                    help="attach timing events to every N-th launch of each kernel kind")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="wall-clock budget of the oracle sample")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (for PMC scaling)")
    ap.add_argument("--record-traffic", nargs=4, metavar="DIR",
                    help="write the traffic record of the measured workload (--workload, --n, "
                         "--prec) from rocprofv3 --pmc output directories: FETCH, WRITE, copy "
                         "FETCH, copy WRITE")
    ap.add_argument("--record-command", default="", help="command line stored in the record")
    ap.add_argument("--record-valu", nargs="+", metavar="DIR",
                    help="write the VALU instruction record from rocprofv3 --pmc SQ counter "
                         "directories named sqc_<workload>_<prec>")
    args = ap.parse_args()
    defaults = {"deform3d": (512, 60, "f64"), "swirl": (1024, 1280, "f32"),
                "fourier3d": (256, 50, "f32"), "kelvin": (1024, None, "f64")}
    n, steps, prec = defaults[args.workload]
    args.n = args.n or n
    args.prec = args.prec or prec
    args.steps = args.steps or steps
    return args


def calibrate_copy():
    import torch
    n = 64 * 1024 * 1024  # 256 MiB of FP32
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                      "dispatches": 5}), flush=True)


def make_workload(W, workload, n, prec):
    if workload == "swirl":
        return W.swirl_three_fields(n, value_prec=prec)
    if workload == "kelvin":
        return W.kelvin(n, amp=1e-4, t_end=1.0, value_prec=prec)
    if workload == "fourier3d":
        return W.fourier3d_three_fields(n, value_prec=prec)
    return W.deform3d_slotted_sphere(n, value_prec=prec)


VALU_KEYS = {("swirl", 1024, "f32"): "swirl_f32/recon2d_tiled_kernel<float, 3, 2>",
             ("swirl", 4096, "f32"): "swirl4096_f32/recon2d_tiled_kernel<float, 3, 2>",
             ("fourier3d", 256, "f32"): "fourier3d_f32/recon3d_kernel<float, 3, 4>",
             ("deform3d", 512, "f64"): "deform3d_f64/recon3d_kernel<double, 1, 3>",
             ("deform3d", 512, "f32"): "deform3d_f32/recon3d_kernel<float, 1, 3>",
             ("kelvin", 1024, "f64"): "kelvin_f64/recon2d_tiled_kernel<double, 3, 6>"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU runs are not "
              "supported (use --gpus 1)", file=sys.stderr, flush=True)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    key = (args.workload, args.n, args.prec)
    if args.record_traffic:
        record_traffic(key, *args.record_traffic, command=args.record_command)
        return
    if args.record_valu:
        record_valu(args.record_valu, command=args.record_command)
        return
    import torch

    from paper_1410_2817_amd import binding as B
    from paper_1410_2817_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    wl = make_workload(W, args.workload, args.n, args.prec)
    if args.workload == "kelvin" and args.steps is None:
        args.steps = wl.nsteps
    dim = wl.dim
    headline = key == HEADLINE
    grid = B.Grid.from_workload(wl, device=dev)
    stored = [np.asarray(f, np.float32 if args.prec == "f32" else np.float64) for f in wl.fields]
    f0 = grid.new_fields(stored)
    bufs = [grid.new_fields(stored), grid.new_fields()]
    stream = torch.cuda.current_stream()
    nodes = grid.nodes

    # Warm-up from the initial state (not timed).
    if args.warmup:
        grid.advance(bufs[0], 0.0, wl.dt, args.warmup, out=bufs[1], stream=stream)
    torch.cuda.synchronize()
    rc, _ = grid.sync(stream)
    if rc != 0:
        raise B.SlError(rc, "warm-up")

    # Timed region: K full steps from t = 0, one sl_advance call; every
    # event_period-th launch of each kernel kind carries HIP timing events in
    # its dispatch packet (on the stream the kernels run on).
    for a_, b_ in zip(bufs[0], f0):
        a_.copy_(b_)
    grid.profile(0 if args.no_events else args.event_period)
    grid.profile_read()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    final = grid.advance(bufs[0], 0.0, wl.dt, args.steps, out=bufs[1], stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = grid.profile_read()
    grid.profile(False)
    rc, stats = grid.sync(stream)
    if rc != 0:
        raise B.SlError(rc, "timed run")
    recon_ms = prof["recon_ms"] / max(prof["recon_launches"], 1)
    traj_ms = prof["traj_ms"] / max(prof["traj_launches"], 1)
    orders_ms = prof["orders_ms"] / max(prof["orders_launches"], 1)
    source_ms = prof["source_ms"] / max(prof["source_launches"], 1)
    sourced = bool(getattr(wl, "source", 0))

    value = nodes * args.steps / elapsed
    vb = 4 if args.prec == "f32" else 8
    # Each reconstruction launch of sl_advance also integrates the next step's
    # trajectories (all launches but the last), so it writes their
    # displacements too.
    per_node = recon_bytes_per_node(dim, wl.nfields, vb) + traj_bytes_per_node(dim)
    if sourced:
        # The source path's reconstructions integrate no trajectories.
        per_node = recon_bytes_per_node(dim, wl.nfields, vb)
    achieved = per_node * nodes / (recon_ms * 1e-3) / 1e9 if recon_ms > 0 else None

    acc = {"order_hist": stats["order_hist"], "search_fail": stats["search_fail"],
           "newton_fail": stats["newton_fail"]}
    if headline:
        acc["vs_oracle_10_steps"] = vs_stored_oracle_run(wl, "deform3d512_10")

    kname = "recon2d_tiled_kernel" if dim == 2 else "recon3d_kernel"
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.prec == "f32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "%s_%dx%d%s_%dfield%s_%s" % (
                wl.name.split("_")[0], args.n, args.n, "x%d" % args.n if dim == 3 else "",
                wl.nfields, "s" if wl.nfields > 1 else "", args.prec),
            "nodes": nodes, "nfields": wl.nfields, "values": args.prec, "positions": "f64",
            "dt": wl.dt, "t_end": args.steps * wl.dt, "limiter": bool(wl.limiter),
            "order": "Z%d" % wl.order_max,
        },
        "roofline": roofline_entry(key, "%s (%s)" % (
            "reconstruction" if sourced else "reconstruction + next step's trajectories", kname),
            achieved, per_node, recon_ms, prof["recon_launches"]),
        "field_node_updates_per_s": value * wl.nfields,
        "kernels": {"trajectories_avg_ms": traj_ms, "reconstruction_avg_ms": recon_ms,
                    "order_words_avg_ms": orders_ms, "source_kernels_avg_ms": source_ms,
                    "event_period": args.event_period},
        "accuracy": acc,
    }
    note("headline: %d steps, %.4g node-updates/s" % (args.steps, value))
    if not args.no_configs and headline:
        out["precision_forms"] = precision_forms()
        out["configs"] = other_configs()
    if not args.no_serving and headline:
        out["serving"] = run_serving(args.serving_requests, args.serving_budget_gib)
    if not args.no_cpu_baseline:
        note("CPU baseline (the oracle on the host)")
        if dim == 3:
            cpu, vs = sampled_cpu_baseline(wl, stored, args.cpu_seconds)
            out["cpu_baseline"] = cpu
            out["accuracy"]["vs_oracle_first_step_sampled"] = vs
        else:
            cpu, ofields = run_cpu_baseline(wl, stored, args.cpu_seconds)
            out["cpu_baseline"] = cpu
            out["accuracy"]["vs_oracle"] = gpu_vs_oracle(wl, stored, cpu["steps"], ofields)
    print(json.dumps(out), flush=True)


def roofline_entry(key, kernel, achieved, per_node, avg_ms, launches):
    """The HBM roofline of the measured reconstruction kernel (algorithmic
    bytes per launch over its live average duration, against 8 TB/s), the
    recorded counter traffic per launch, and the same kernel's VALU issue
    fraction (its binding roof) beside it."""
    valu = valu_roof(VALU_KEYS.get(key, ""), avg_ms)
    return {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": recorded_traffic(key), "bytes_per_node": per_node, "avg_ms": avg_ms,
            "launches": launches,
            "valu": None if valu is None else {k: valu[k] for k in (
                "achieved", "peak", "unit", "frac", "valu_per_wave", "waves")}}


def vs_stored_oracle_run(wl, case):
    """The GPU's run of `wl` over the stored oracle run's steps against it, at
    the stored sample of nodes (tests/golden/oracle_<case>.npz, written from
    the oracle alone)."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_%s.npz" % case)
    if not os.path.exists(path):
        return None
    ref = np.load(path, allow_pickle=False)
    steps = int(ref["steps"])
    out, _, _, _ = run_gpu(wl, steps, t0=float(ref["t0"]), profile=0, warmup=0)
    nodes, want = ref["nodes"], ref["values"]
    num = den = 0.0
    for f, fld in enumerate(out):
        got = fld.double().cpu().numpy().ravel()[nodes]
        num += float(np.abs(got - want[:, f]).sum())
        den += float(np.abs(want[:, f]).sum())
    return {"steps": steps, "sampled_nodes": int(nodes.size), "l1_rel": num / max(den, 1e-300)}


def run_gpu(wl, nsteps, prec=None, t0=0.0, profile=4, warmup=2):
    """nsteps GPU steps of workload wl from its stored initial values (after
    `warmup` untimed steps); returns (fields, seconds, profile, stats)."""
    import torch
    from paper_1410_2817_amd import binding as B
    prec = prec or wl.value_prec
    dt_np = np.float32 if prec == "f32" else np.float64
    g = B.Grid.from_workload(wl, value_prec=prec)
    init = [np.asarray(f, dt_np) for f in wl.fields]
    if warmup:
        g.advance(g.new_fields(init), t0, wl.dt, warmup)
        torch.cuda.synchronize()
    x = g.new_fields(init)
    g.profile(profile)
    g.profile_read()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out = g.advance(x, t0, wl.dt, nsteps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    prof = g.profile_read()
    g.profile(0)
    rc, st = g.sync()
    if rc != 0:
        raise B.SlError(rc, wl.name)
    return out, el, prof, st


def _l1(a, b):
    return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))


def _timed_forms(wl, nsteps):
    """Both precision forms of `wl` over nsteps steps from t = 0: throughput
    and the final fields (FP64 numpy)."""
    res = {}
    for prec in ("f32", "f64"):
        out, el, prof, _ = run_gpu(wl, nsteps, prec=prec)
        res[prec] = ([f.double().cpu().numpy() for f in out], wl.nodes * nsteps / el,
                     prof["recon_ms"] / max(prof["recon_launches"], 1))
        del out
    return res


def precision_forms():
    """The FP32-value / FP64-position split form next to plain FP64, compared
    at their L1 error against the exact solution: over one whole period of
    the reversing swirl (1024^2, 1280 steps) and of the 3-D deformational flow
    (128^3, 256 steps), after which the exact solution is the initial state.
    Each form starts from its own stored initial values and is measured
    against them.  Both forms run their whole period here whatever --steps
    is."""
    from paper_1410_2817_amd import workloads as W
    res = {}
    for name, wl in (("swirl2d_1024x1024_3fields", W.swirl_three_fields(1024)),
                     ("deform3d_128x128x128_1field", W.deform3d_slotted_sphere(128))):
        period = wl.velocity.params[0]
        nsteps = int(round(period / wl.dt))
        assert abs(nsteps * wl.dt - period) < 1e-9
        forms = _timed_forms(wl, nsteps)
        entry = {"workload": "%s, one period (%d steps)" % (name, nsteps)}
        for prec, label in (("f32", "f32_split"), ("f64", "f64_plain")):
            got, rate, rms = forms[prec]
            init = [np.asarray(f, np.float32 if prec == "f32" else np.float64).astype(np.float64)
                    for f in wl.fields]
            entry[label] = {"node_updates_per_s": rate, "reconstruction_avg_ms": rms,
                            "l1_rel_vs_exact": [_l1(g, e) for g, e in zip(got, init)]}
        entry["split_over_plain"] = entry["f32_split"]["node_updates_per_s"] / \
            entry["f64_plain"]["node_updates_per_s"]
        entry["split_vs_plain_l1_rel"] = [_l1(a, b) for a, b in zip(forms["f32"][0],
                                                                      forms["f64"][0])]
        res[name] = entry
        note("precision forms: %s" % name)
    return res


def other_configs():
    """The remaining single-GPU configurations: the 1024^2 three-field swirl
    (FP32 values, its own HBM roofline and traffic record), the same at
    4096^2 (working set beyond the 256 MB last-level cache), SBR 64^2 FP64
    (one revolution, L1 against the exact solution and the oracle), the 3-D
    Fourier flow at 256^3 (FP32 split, 50 steps), the 3-D deformational flow
    at 512^3 in the FP32-value form (60 steps, against the plain FP64 run),
    one GPU's share of it, Burgers' equation, a gridded velocity and the
    Kelvin wave."""
    import oracle
    from paper_1410_2817_amd import workloads as W
    res = {}

    # Swirl 1024^2, FP32 values (one period).
    wl = W.swirl_three_fields(1024, value_prec="f32")
    out, el, prof, st = run_gpu(wl, wl.nsteps, warmup=20)
    rms = prof["recon_ms"] / max(prof["recon_launches"], 1)
    per_node = recon_bytes_per_node(2, wl.nfields, 4) + traj_bytes_per_node(2)
    ach = per_node * wl.nodes / (rms * 1e-3) / 1e9
    note("config swirl1024_f32")
    res["swirl1024_f32"] = {
        "node_updates_per_s": wl.nodes * wl.nsteps / el, "ms_per_step": el * 1e3 / wl.nsteps,
        "steps": wl.nsteps,
        "trajectories_avg_ms": prof["traj_ms"] / max(prof["traj_launches"], 1),
        "roofline": roofline_entry(("swirl", 1024, "f32"),
                                   "reconstruction + next step's trajectories "
                                   "(recon2d_tiled_kernel)", ach, per_node, rms,
                                   prof["recon_launches"]),
        "order_hist": st["order_hist"]}
    del out

    # SBR 64^2: one revolution (100 steps).
    wl = W.solid_body_gaussian(64, 100)
    out, el, prof, st = run_gpu(wl, 100)
    got = out[0].double().cpu().numpy()
    exact = np.asarray(wl.fields[0], np.float64)
    prob = _oracle_problem(oracle, wl)
    rc, ofs, _ = oracle.run(prob, 0.0, wl.dt, 100, [exact])
    note("config sbr64_f64")
    res["sbr64_f64"] = {"node_updates_per_s": wl.nodes * 100 / el, "ms_per_step": el * 1e3 / 100,
                        "l1_rel_vs_exact": _l1(got, exact), "l1_rel_vs_oracle": _l1(got, ofs[0]),
                        "linf_vs_oracle": float(np.abs(got - ofs[0]).max())}

    # Swirl 4096^2: reconstruction at the size whose working set exceeds the
    # 256 MB last-level cache.
    wl = W.swirl_three_fields(4096, value_prec="f32")
    n4 = 40
    out, el, prof, st = run_gpu(wl, n4)
    rms = prof["recon_ms"] / max(prof["recon_launches"], 1)
    per_node = recon_bytes_per_node(2, wl.nfields, 4) + traj_bytes_per_node(2)
    ach = per_node * wl.nodes / (rms * 1e-3) / 1e9
    note("config swirl4096_f32")
    res["swirl4096_f32"] = {"node_updates_per_s": wl.nodes * n4 / el, "ms_per_step": el * 1e3 / n4,
                            "steps": n4, "reconstruction_avg_ms": rms,
                            "trajectories_avg_ms": prof["traj_ms"] / max(prof["traj_launches"], 1),
                            "order_words_avg_ms": prof["orders_ms"] / max(prof["orders_launches"], 1),
                            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                         "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                                         "bytes_per_node": per_node},
                            "valu_roof": valu_roof(VALU_KEYS[("swirl", 4096, "f32")], rms)}
    del out

    # 3-D configurations.
    cases = [("fourier3d_256_f32", W.fourier3d_three_fields(256, value_prec="f32"), 50, "f32"),
             ("deform3d_512_f32", W.deform3d_slotted_sphere(512), 60, "f32"),
             ("deform3d_512_f64", W.deform3d_slotted_sphere(512), 60, "f64")]
    keep = {}
    for name, wl, nsteps, prec in cases:
        out, el, prof, st = run_gpu(wl, nsteps, prec=prec)
        note("config %s" % name)
        rms = prof["recon_ms"] / max(prof["recon_launches"], 1)
        vb = 4 if prec == "f32" else 8
        per_node = recon_bytes_per_node(3, wl.nfields, vb) + traj_bytes_per_node(3)
        ach = per_node * wl.nodes / (rms * 1e-3) / 1e9
        if name.startswith("deform3d"):
            keep[prec] = out[0].double().cpu().numpy()
        del out
        if name == "deform3d_512_f64":
            continue  # the headline; run here for the split form's comparison only
        res[name] = {"node_updates_per_s": wl.nodes * nsteps / el, "ms_per_step": el * 1e3 / nsteps,
                     "steps": nsteps, "reconstruction_avg_ms": rms,
                     "trajectories_avg_ms": prof["traj_ms"] / max(prof["traj_launches"], 1),
                     "order_words_avg_ms": prof["orders_ms"] / max(prof["orders_launches"], 1),
                     "hbm_achieved_gbs": ach, "hbm_frac": ach / HBM_PEAK_GBS,
                     "valu_roof": valu_roof({"fourier3d_256_f32": "fourier3d_f32/recon3d_kernel<float, 3, 4>",
                                             "deform3d_512_f32": "deform3d_f32/recon3d_kernel<float, 1, 3>"}
                                            .get(name, ""), rms),
                     "order_hist": st["order_hist"], "walked": st["walked"]}
    # Split form against plain FP64 after the same 60 steps.
    res["deform3d_512_f32"]["l1_rel_vs_f64_plain"] = _l1(keep["f32"], keep["f64"])
    del keep
    res["deform3d_512_f64_shard"] = shard_config(W.deform3d_slotted_sphere(512), 60)
    note("config deform3d_512_f64_shard")

    # Burgers' equation (velocity carried by the fields), the paper's radial
    # shock test at 512^2 up to t = 0.3, plus its first 20 steps against the
    # oracle.
    wl = W.burgers(512)
    out, el, prof, st = run_gpu(wl, wl.nsteps)
    brms = prof["recon_ms"] / max(prof["recon_launches"], 1)
    # Each launch reconstructs 2 FP64 fields and writes the next displacement.
    bgbs = (recon_bytes_per_node(2, 2, 8) + traj_bytes_per_node(2)) * wl.nodes / (brms * 1e-3) / 1e9
    note("config burgers2d_512_f64")
    res["burgers2d_512_f64"] = {"node_updates_per_s": wl.nodes * wl.nsteps / el,
                                "ms_per_step": el * 1e3 / wl.nsteps, "steps": wl.nsteps,
                                "reconstruction_avg_ms": brms,
                                "reconstruction_hbm_gbs": bgbs, "hbm_frac": bgbs / HBM_PEAK_GBS,
                                "t_end": wl.nsteps * wl.dt, "search_fail": st["search_fail"],
                                "order_hist": st["order_hist"],
                                "max_speed": float(max(np.abs(f.double().cpu().numpy()).max()
                                                       for f in out))}
    out20, _, _, _ = run_gpu(wl, 20, profile=0, warmup=0)
    rc, ofs, _ = oracle.run(_oracle_problem(oracle, wl), 0.0, wl.dt, 20,
                            [np.asarray(f, np.float64) for f in wl.fields])
    res["burgers2d_512_f64"]["l1_rel_vs_oracle_20_steps"] = [
        _l1(g.double().cpu().numpy(), o) for g, o in zip(out20, ofs)]
    # Gridded velocity: the swirl's velocity sampled on the mesh (at t = 1.25,
    # held fixed) and interpolated with the Z2 spline at the trajectory
    # points; 160 steps timed (unfused step: trajectories, then the
    # reconstruction), and 3 steps against the oracle.
    wl = W.gridded(W.swirl_three_fields(1024, value_prec="f32"), 2, t=1.25)
    out, el, prof, st = run_gpu(wl, 160)
    grms = prof["recon_ms"] / max(prof["recon_launches"], 1)
    gtms = prof["traj_ms"] / max(prof["traj_launches"], 1)
    # Unfused step: the reconstruction reads the displacement and the values and
    # writes the values; the trajectories read the two velocity samples of
    # their node's window once (the rest comes from LDS) and write the
    # displacement.
    g_rec = recon_bytes_per_node(2, 3, 4) * wl.nodes / (grms * 1e-3) / 1e9
    g_trj = (16 + traj_bytes_per_node(2)) * wl.nodes / (gtms * 1e-3) / 1e9
    note("config gridded_swirl1024_f32")
    res["gridded_swirl1024_f32"] = {
        "node_updates_per_s": wl.nodes * 160 / el, "ms_per_step": el * 1e3 / 160, "steps": 160,
        "trajectories_avg_ms": gtms, "reconstruction_avg_ms": grms,
        "reconstruction_hbm_gbs": g_rec, "trajectories_hbm_gbs": g_trj,
        "search_fail": st["search_fail"]}
    del out
    out3, _, _, _ = run_gpu(wl, 3, profile=0, warmup=0)
    stored3 = [np.asarray(f, np.float32).astype(np.float64) for f in wl.fields]
    rc, ofs, _ = oracle.run(_oracle_problem(oracle, wl), 0.0, wl.dt, 3, stored3)
    got = [g.double().cpu().numpy() for g in out3]
    res["gridded_swirl1024_f32"]["l1_rel_vs_oracle_3_steps"] = (
        sum(float(np.abs(g - o).sum()) for g, o in zip(got, ofs)) /
        sum(float(np.abs(o).sum()) for o in ofs))
    res.update(kelvin_configs())
    note("config kelvin")
    return res


def shard_config(wl, nsteps, parts=8, halo=8):
    """One GPU's share of `wl` split into `parts` slabs along the slowest axis:
    the owned planes plus `halo` planes on each side, as a grid whose node 0 sits
    at the slab's place in the whole lattice (offset).  Timing only: with one
    GPU no halo exchange runs, so after the first step the halo holds stale
    values (and its outermost nodes, which search across the shard's own
    periodic seam, may report failed searches: `status`); node-updates/s
    counts the owned nodes."""
    import torch
    from paper_1410_2817_amd import binding as B
    own = wl.shape[0] // parts
    lo = (parts // 2) * own
    shape = list(wl.shape)
    shape[0] = own + 2 * halo
    length = list(wl.length)
    length[0] = wl.length[0] * shape[0] / wl.shape[0]
    off = [lo - halo] + [0] * (wl.dim - 1)
    g = B.Grid(shape, wl.nfields, length=length, value_prec=wl.value_prec,
               order_max=wl.order_max, limiter=wl.limiter, theta=wl.theta,
               integrator=wl.integrator, vel_kind=wl.velocity.kind,
               vel_params=wl.velocity.padded_params(), modes=wl.velocity.modes, offset=off)
    init = [np.ascontiguousarray(f[lo - halo:lo + own + halo]) for f in wl.fields]
    g.advance(g.new_fields(init), 0.0, wl.dt, 2)
    torch.cuda.synchronize()
    x = g.new_fields(init)
    g.profile(4)
    g.profile_read()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.advance(x, 0.0, wl.dt, nsteps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    prof = g.profile_read()
    g.profile(0)
    rc, st = g.sync()
    owned = own * int(np.prod(wl.shape[1:]))
    return {"share": "%d of %d slabs: %s owned + %d halo planes per side" % (
                1, parts, "x".join(str(v) for v in [own] + list(wl.shape[1:])), halo),
            "owned_node_updates_per_s": owned * nsteps / el, "ms_per_step": el * 1e3 / nsteps,
            "steps": nsteps, "reconstruction_avg_ms": prof["recon_ms"] / max(prof["recon_launches"], 1),
            "halo_overhead": shape[0] / own, "status": rc}


def kelvin_configs():
    """Shallow-water source terms (Sec. 3): the equatorial Kelvin wave to t = 1,
    relative L2 error of h against the exact wave and the observed order at
    the paper's amplitude 1e-4 on 32^2 .. 256^2, and the 1024^2 run timed."""
    import oracle
    from paper_1410_2817_amd import workloads as W
    res = {}

    def ladder(amp, sizes):
        rows = []
        for n in sizes:
            wl = W.kelvin(n, amp=amp, t_end=1.0)
            out, el, prof, st = run_gpu(wl, wl.nsteps, warmup=0 if n < 1024 else 2)
            ex = W.kelvin_fields(wl.shape, 1.0, amp, 250.0)
            h = out[2].double().cpu().numpy()
            err = float(np.sqrt(((h - ex[2]) ** 2).sum() / (ex[2] ** 2).sum()))
            rows.append({"n": n, "steps": wl.nsteps, "l2_rel_vs_exact": err})
            if n == 1024 and amp == 1e-4:
                rl, sl = max(prof["recon_launches"], 1), max(prof["source_launches"], 1)
                krms, ksms = prof["recon_ms"] / rl, prof["source_ms"] / sl
                # Reconstruction: 3 FP64 fields, no trajectories (64 B/node).
                # Stage kernel, averaged over its three stages: 104 B (stage
                # 0), 184 B (stage 1), 144 B (stage 2, no registers written).
                k_rec = recon_bytes_per_node(2, 3, 8) * wl.nodes / (krms * 1e-3) / 1e9
                k_stg = (104 + 184 + 144) / 3.0 * wl.nodes / (ksms * 1e-3) / 1e9
                res["kelvin_1024_f64"] = {
                    "node_updates_per_s": wl.nodes * wl.nsteps / el,
                    "ms_per_step": el * 1e3 / wl.nsteps, "steps": wl.nsteps,
                    "reconstruction_avg_ms": krms,
                    "source_kernel_avg_ms": ksms,
                    "reconstruction_hbm_gbs": k_rec, "stage_hbm_gbs": k_stg,
                    "valu_roof_reconstruction": valu_roof(
                        "kelvin_f64/recon2d_tiled_kernel<double, 3, 6>", krms),
                    "valu_roof_stage": valu_roof("kelvin_f64/sw_stage_kernel<double, 2>", ksms),
                    "reconstructions_per_step": 3, "source_launches_per_step": 6,
                    "search_fail": st["search_fail"], "l2_rel_vs_exact_t1": err}
            del out
        for a, b in zip(rows, rows[1:]):
            b["order"] = float(np.log2(a["l2_rel_vs_exact"] / b["l2_rel_vs_exact"]))
        return rows

    res["kelvin_convergence_amp1e-4_f64"] = ladder(1e-4, (32, 64, 128, 256))
    ladder(1e-4, (1024,))
    return res


def _oracle_problem(oracle, wl):
    return oracle.Problem(wl.shape, wl.nfields, wl.length, order_max=wl.order_max,
                          limiter=wl.limiter, theta=wl.theta, integrator=wl.integrator,
                          vel_kind=wl.velocity.kind, vp=wl.velocity.padded_params(),
                          modes=wl.velocity.modes, src_kind=getattr(wl, "source", 0),
                          sp=list(getattr(wl, "sp", (0.0,) * 4)),
                          ugrid=getattr(wl, "ugrid", None))


def gpu_vs_oracle(wl, stored, steps, ofields):
    """GPU result after the oracle sample's steps against the oracle's."""
    out, _, _, _ = run_gpu(wl, steps, profile=0, warmup=0)
    got = [f.double().cpu().numpy() for f in out]
    num = sum(float(np.abs(g - o).sum()) for g, o in zip(got, ofields))
    den = sum(float(np.abs(o).sum()) for o in ofields)
    return {"steps": steps, "l1_rel_all_fields": num / max(den, 1e-300),
            "l1_rel": [_l1(g, o) for g, o in zip(got, ofields)],
            "linf": [float(np.abs(g - o).max()) for g, o in zip(got, ofields)]}


SERVING_MODES = (("batched", 1), ("queued", 1), ("queued", 4))


def run_serving(count: int, budget_gib: float):
    """Serving mix: `count` seeded requests (2-D periodic grids with sides in
    {128, ..., 2048}, 1-4 fields, 10-50 steps of a 16-mode Fourier flow, FP32
    values / FP64 positions) through the continuous-batching server with an
    HBM budget of `budget_gib`.  First all requests arrive at once (capacity),
    then with Poisson arrivals at 0.7 x that capacity (latency).  Each launch
    mode of the server is measured (SERVING_MODES: one batched launch per
    tick, and queued launches of 1 and 4 steps from device-side tile queues);
    the first is reported at the top level, all under "modes"."""
    res = None
    modes = {}
    for mode, window in SERVING_MODES:
        r = _serving_mode(count, budget_gib, mode, window)
        note("serving %s window %d" % (mode, window))
        modes["%s_w%d" % (mode, window)] = r
        if res is None:
            res = dict(r)
    res["modes"] = modes
    return res


def _serving_mode(count, budget_gib, mode, window):
    from paper_1410_2817_amd import serving as S
    from paper_1410_2817_amd import workloads as W
    budget = int(budget_gib * (1 << 30))
    burst = W.serving_stream(seed=0, count=count, rate=1e9)
    for r in burst:
        r.arrival = 0.0
    cap = S.run_stream(burst, budget, max_requests=256, mode=mode, window=window)
    rate = 0.7 * count / cap["makespan_s"]
    rep = S.run_stream(W.serving_stream(seed=0, count=count, rate=rate), budget,
                       max_requests=256, mode=mode, window=window)
    keep = ("latency_p50_ms", "latency_p99_ms", "latency_mean_ms", "queue_wait_p50_ms",
            "queue_wait_p99_ms", "node_updates_per_s", "makespan_s", "ticks", "status")
    # Whole-job effective HBM rate of the capacity run: the algorithmic bytes of
    # every step of every request (FP32 values; each reconstruction also writes
    # the next step's displacement) over the makespan, all launches and gaps
    # included.
    alg = sum(r.nodes * r.nsteps * (recon_bytes_per_node(2, r.nfields, 4) + traj_bytes_per_node(2))
              for r in burst)
    eff = alg / cap["makespan_s"] / 1e9
    return {"mode": mode, "window": window, "requests": count, "budget_gib": budget_gib,
            "capacity_node_updates_per_s": cap["node_updates_per_s"],
            "capacity_requests_per_s": count / cap["makespan_s"],
            "capacity_effective_hbm_gbs": eff, "capacity_effective_hbm_frac": eff / HBM_PEAK_GBS,
            "poisson_rate_per_s": rate, **{k: rep[k] for k in keep}}


def sampled_cpu_baseline(wl, stored, seconds):
    """Time the FP64 oracle (unchanged) on the host over a bounded sample of
    the same workload: its sampled step (one step from t = 0 at random mesh
    nodes, every trajectory the element search touches integrated on demand)
    on as many nodes as fill about `seconds`.  The GPU's first step is
    compared with the oracle at those nodes."""
    import oracle
    prob = _oracle_problem(oracle, wl)
    fields = [np.asarray(s, np.float64) for s in stored]
    g = np.random.Generator(np.random.PCG64(2024))
    probe = np.unique(g.integers(0, wl.nodes, 2000)).astype(np.int64)
    t0 = time.perf_counter()
    rc, _, _ = oracle.step_sampled(prob, 0.0, wl.dt, fields, probe)
    per_node = (time.perf_counter() - t0) / probe.size
    count = int(min(max(seconds / max(per_node, 1e-9), 2000), 32_000_000))
    nodes = np.unique(g.integers(0, wl.nodes, count)).astype(np.int64)
    t0 = time.perf_counter()
    rc, vals, _ = oracle.step_sampled(prob, 0.0, wl.dt, fields, nodes)
    spent = time.perf_counter() - t0
    out, _, _, _ = run_gpu(wl, 1, profile=0, warmup=0)
    num = den = 0.0
    linf = 0.0
    for f, fld in enumerate(out):
        got = fld.double().cpu().numpy().ravel()[nodes]
        d = np.abs(got - vals[:, f])
        num += float(d.sum())
        den += float(np.abs(vals[:, f]).sum())
        linf = max(linf, float(d.max()))
    del out
    cpu = {"value": nodes.size / spent, "unit": "node-updates/s", "cores": oracle.threads(),
           "kind": "oracle", "status": rc,
           "sample": "one step from t = 0 of the same %s workload at %d random mesh nodes "
                     "(the oracle's sampled step: each node integrates the trajectories of "
                     "the cells its search touches, which a whole-grid step shares between "
                     "neighbours), %.1f s wall" % ("x".join(str(v) for v in wl.shape[::-1]),
                                                   nodes.size, spent)}
    return cpu, {"steps": 1, "sampled_nodes": int(nodes.size),
                 "l1_rel": num / max(den, 1e-300), "linf": linf}


def run_cpu_baseline(wl, stored, seconds):
    """Time the FP64 oracle (unchanged) on the host over the first steps of the
    same workload; stop once `seconds` of wall time are spent."""
    import oracle
    prob = _oracle_problem(oracle, wl)
    fields = [np.asarray(s, np.float64) for s in stored]
    steps, spent = 0, 0.0
    while spent < seconds:
        t0 = time.perf_counter()
        if getattr(wl, "source", 0):
            rc, fields, _ = oracle.run_source(prob, steps * wl.dt, wl.dt, 1, fields)
        else:
            rc, fields, _ = oracle.run(prob, steps * wl.dt, wl.dt, 1, fields)
        spent += time.perf_counter() - t0
        steps += 1
        if rc != 0:
            break
    return {"value": wl.nodes * steps / spent, "unit": "node-updates/s",
            "cores": oracle.threads(), "kind": "oracle", "steps": steps,
            "sample": "first %d step(s) of the same %dx%d workload, %.1f s wall" % (
                steps, wl.shape[1], wl.shape[0], spent)}, fields


if __name__ == "__main__":
    main()
