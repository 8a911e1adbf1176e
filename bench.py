"""Benchmark of the forward semi-Lagrangian step on one MI355X.

Workload: the 2-D reversing swirl (period T = 5, max speed 1) on a 1024 x 1024
periodic grid carrying three fields (slotted disc, cosine bell, Gaussian), FP32
values with FP64 positions, Z2 with the jump limiter on, dt = 4h (CFL 4), so a
full period is 1280 steps.  A step is one pass of the whole hot path: the
lattice trajectories and the reconstruction of all three fields, run by
sl_advance (in 2-D each reconstruction launch also integrates the next step's
trajectories).  Inputs are resident in HBM before timing starts.

Prints one JSON line (metric, value, ms_per_step, roofline, cpu_baseline, ...);
with the defaults it also reports the plain-FP64 form, the other single-GPU
configurations and the serving mix.  --workload fourier3d / deform3d make a
3-D flow the measured workload instead (used for the 3-D kernel profiles).
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
TRAFFIC_JSON = os.path.join(PROFILES, "recon2d_swirl1024_traffic.json")
RECON_KERNEL = "recon2d_tiled_kernel<float, 3>"


# The sources recon2d_tiled_kernel is compiled from (the kernel the traffic
# record is taken on): its own header and everything it includes.
HEADLINE_KERNEL_SOURCES = ("include/sl.h", "paper_1410_2817_amd/csrc/sl_device.h",
                           "paper_1410_2817_amd/csrc/sl_traj.h",
                           "paper_1410_2817_amd/csrc/sl_recon2d.h")


def source_hash() -> str:
    """Hash of the headline kernel's sources, to tell whether recorded counters
    still apply."""
    import hashlib
    h = hashlib.sha256()
    for rel in HEADLINE_KERNEL_SOURCES:
        h.update(rel.encode())
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _pmc_mean(csv_path: str, kernel_sub: str, counter: str):
    import csv
    vals = []
    with open(csv_path) as fh:
        for row in csv.DictReader(fh):
            if kernel_sub in row["Kernel_Name"] and row["Counter_Name"] == counter:
                vals.append(float(row["Counter_Value"]))
    return sum(vals) / len(vals) if vals else None


def record_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, command):
    """Turn four rocprofv3 --pmc runs (FETCH_SIZE / WRITE_SIZE of the benchmark
    and of the plain 256 MiB copy) into the traffic record bench.py reports."""
    f = _pmc_mean(os.path.join(fetch_dir, "run_counter_collection.csv"), RECON_KERNEL, "FETCH_SIZE")
    w = _pmc_mean(os.path.join(write_dir, "run_counter_collection.csv"), RECON_KERNEL, "WRITE_SIZE")
    cf = _pmc_mean(os.path.join(copy_fetch_dir, "run_counter_collection.csv"), "copyBuffer", "FETCH_SIZE")
    cw = _pmc_mean(os.path.join(copy_write_dir, "run_counter_collection.csv"), "copyBuffer", "WRITE_SIZE")
    copy_kib = 64 * 1024 * 1024 * 4 / 1024.0
    ff, fw = copy_kib / cf, copy_kib / cw
    rec = {"kernel": RECON_KERNEL, "workload": "swirl2d_1024x1024_3fields_f32",
           "fetch_kib_per_dispatch": f, "write_kib_per_dispatch": w,
           "copy_fetch_kib": cf, "copy_write_kib": cw, "copy_kib": copy_kib,
           "fetch_factor": ff, "write_factor": fw,
           "traffic_bytes_per_launch": (f * ff + w * fw) * 1024.0,
           "source_hash": source_hash(), "command": command}
    os.makedirs(PROFILES, exist_ok=True)
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


# VALU issue: a wave64 VALU instruction holds one of the 1024 SIMDs (256 CUs x
# 4) for 4 cycles (16 lanes), at 2.4 GHz.  With packed FP32 disabled this is
# the roof of every kernel here (FP64 and FP32 issue at the same rate).
VALU_SIMDS, VALU_CYCLES_PER_INST, CLOCK_HZ = 1024, 4, 2.4e9
VALU_JSON = os.path.join(PROFILES, "valu_counters.json")
# Workload of each counter directory -> the kernels whose counts are kept.
VALU_KERNELS = {"swirl_f32": ["recon2d_tiled_kernel<float, 3>"],
                "fourier3d_f32": ["recon3d_kernel<float, 3>"],
                "deform3d_f64": ["recon3d_kernel<double, 1>"],
                "deform3d_f32": ["recon3d_kernel<float, 1>"],
                "kelvin_f64": ["recon2d_tiled_kernel<double, 3>", "sw_stage_kernel<double, 2>"]}


def all_sources_hash() -> str:
    """Hash of every HIP source and the C header."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1410_2817_amd", "csrc")
    names = sorted(n for n in os.listdir(csrc) if n.endswith((".h", ".hip")))
    for rel in ["include/sl.h"] + ["paper_1410_2817_amd/csrc/" + n for n in names]:
        h.update(rel.encode())
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
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


def recorded_traffic():
    """Traffic bytes per reconstruction launch from the committed counter
    record, or None when the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_JSON) as fh:
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
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="swirl",
                    choices=["swirl", "fourier3d", "deform3d", "kelvin"],
                    help="swirl: the 2-D reversing swirl (default); fourier3d / deform3d: the "
                         "3-D Fourier-mode and deformational flows; kelvin: the shallow-water "
                         "Kelvin wave with source terms (for profiling runs)")
    ap.add_argument("--n", type=int, default=None,
                    help="grid side (default 1024 swirl and kelvin, 256 fourier3d, 512 deform3d)")
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 1280 swirl = one period, 50 fourier3d, 60 deform3d)")
    ap.add_argument("--prec", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving (continuous batching) measurement")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--serving-budget-gib", type=float, default=8.0)
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other configurations (SBR 64^2, swirl 4096^2, 3-D)")
    ap.add_argument("--no-events", action="store_true",
                    help="time without kernel events")
    ap.add_argument("--event-period", type=int, default=8,
                    help="attach timing events to every N-th launch of each kernel kind")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall-clock budget of the oracle sample")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (for PMC scaling)")
    ap.add_argument("--record-traffic", nargs=4, metavar="DIR",
                    help="write the traffic record from rocprofv3 --pmc output directories: "
                         "FETCH, WRITE, copy FETCH, copy WRITE")
    ap.add_argument("--record-command", default="", help="command line stored in the record")
    ap.add_argument("--record-valu", nargs="+", metavar="DIR",
                    help="write the VALU instruction record from rocprofv3 --pmc SQ counter "
                         "directories named sqc_<workload>_<prec>")
    return ap.parse_args()


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


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU runs are not "
              "supported (use --gpus 1)", file=sys.stderr, flush=True)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.record_traffic:
        record_traffic(*args.record_traffic, command=args.record_command)
        return
    if args.record_valu:
        record_valu(args.record_valu, command=args.record_command)
        return
    import torch

    from paper_1410_2817_amd import binding as B
    from paper_1410_2817_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    dim = 2 if args.workload in ("swirl", "kelvin") else 3
    if args.workload == "swirl":
        args.n = args.n or 1024
        wl = W.swirl_three_fields(args.n, value_prec=args.prec)
        args.steps = args.steps or 1280
    elif args.workload == "kelvin":
        args.n = args.n or 1024
        wl = W.kelvin(args.n, amp=1e-4, t_end=1.0, value_prec=args.prec)
        args.steps = args.steps or wl.nsteps
    elif args.workload == "fourier3d":
        args.n = args.n or 256
        wl = W.fourier3d_three_fields(args.n, value_prec=args.prec)
        args.steps = args.steps or 50
    else:
        args.n = args.n or 512
        wl = W.deform3d_slotted_sphere(args.n, value_prec=args.prec)
        args.steps = args.steps or 60
    headline = args.workload == "swirl" and args.n == 1024 and args.prec == "f32"
    grid = B.Grid.from_workload(wl, device=dev)
    stored = [np.asarray(f, np.float32 if args.prec == "f32" else np.float64) for f in wl.fields]
    f0 = grid.new_fields(stored)
    bufs = [grid.new_fields(stored), grid.new_fields()]
    stream = torch.cuda.current_stream()
    nodes = grid.nodes

    # Warm-up from the initial state (not timed).
    grid.advance(bufs[0], 0.0, wl.dt, args.warmup, out=bufs[1], stream=stream)
    torch.cuda.synchronize()
    rc, _ = grid.sync(stream)
    if rc != 0:
        raise B.SlError(rc, "warm-up")

    # Timed region: K full steps from t = 0, one sl_advance call; every kernel
    # launch carries HIP timing events in its dispatch packet.
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

    # Accuracy: after a whole period the exact solution is the initial state.
    acc = {}
    if args.workload == "swirl" and args.steps * wl.dt >= wl.velocity.params[0] - 1e-9 and \
            abs(args.steps * wl.dt - round(args.steps * wl.dt / wl.velocity.params[0]) * wl.velocity.params[0]) < 1e-9:
        got = [f.double().cpu().numpy() for f in final]
        acc["l1_rel_vs_exact_after_period"] = [
            float(np.abs(g - np.asarray(s, np.float64)).sum() / np.abs(np.asarray(s, np.float64)).sum())
            for g, s in zip(got, stored)]
    acc["order_hist"] = stats["order_hist"]
    acc["search_fail"] = stats["search_fail"]

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
            "workload": wl.name if not headline else
                        "swirl2d_%dx%d_3fields_%s_cfl4_limiter_z2" % (args.n, args.n, args.prec),
            "nodes": nodes, "nfields": wl.nfields, "values": args.prec, "positions": "f64",
            "dt": wl.dt, "t_end": args.steps * wl.dt,
        },
        "roofline": {
            "kernel": ("reconstruction (%s)" if sourced else
                       "reconstruction + next step's trajectories (%s)") % (
                "recon2d_tiled_kernel" if dim == 2 else "recon3d_kernel"),
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": recorded_traffic() if headline else None,
            "bytes_per_node": per_node, "avg_ms": recon_ms,
            "launches": prof["recon_launches"],
        },
        "valu_roof": valu_roof({("swirl", 1024, "f32"): "swirl_f32/recon2d_tiled_kernel<float, 3>",
                                ("fourier3d", 256, "f32"): "fourier3d_f32/recon3d_kernel<float, 3>",
                                ("deform3d", 512, "f64"): "deform3d_f64/recon3d_kernel<double, 1>",
                                ("deform3d", 512, "f32"): "deform3d_f32/recon3d_kernel<float, 1>",
                                ("kelvin", 1024, "f64"): "kelvin_f64/recon2d_tiled_kernel<double, 3>"}
                               .get((args.workload, args.n, args.prec), ""), recon_ms),
        "field_node_updates_per_s": value * wl.nfields,
        "kernels": {"trajectories_avg_ms": traj_ms, "reconstruction_avg_ms": recon_ms,
                    "order_words_avg_ms": orders_ms, "source_kernels_avg_ms": source_ms,
                    "event_period": args.event_period},
        "accuracy": acc,
    }
    if not args.no_configs and headline:
        out["precision_forms"] = precision_forms(wl, stored, value, final)
        out["configs"] = other_configs()
    if not args.no_serving and headline:
        out["serving"] = run_serving(args.serving_requests, args.serving_budget_gib)
    if not args.no_cpu_baseline:
        cpu, ofields = run_cpu_baseline(wl, stored, args.cpu_seconds)
        out["cpu_baseline"] = cpu
        out["accuracy"]["vs_oracle"] = gpu_vs_oracle(wl, stored, cpu["steps"], ofields)
    print(json.dumps(out), flush=True)


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


def precision_forms(wl, stored, value_f32, final_f32):
    """The same swirl workload in plain FP64 next to the FP32-value split form:
    throughput and L1 error against the exact solution (the initial state,
    after a whole period), so the two are compared at their L1 error."""
    out64, el, prof, _ = run_gpu(wl, int(round(wl.velocity.params[0] / wl.dt)), prec="f64")
    # Each form's exact solution is its own initial state.
    l1_64 = [_l1(f.double().cpu().numpy(), np.asarray(e, np.float64))
             for f, e in zip(out64, wl.fields)]
    l1_32 = [_l1(f.double().cpu().numpy(), np.asarray(e, np.float64))
             for f, e in zip(final_f32, stored)]
    nsteps = int(round(wl.velocity.params[0] / wl.dt))
    return {"workload": "swirl2d_1024x1024_3fields, one period (%d steps)" % nsteps,
            "f32_split": {"node_updates_per_s": value_f32, "l1_rel_vs_exact": l1_32},
            "f64_plain": {"node_updates_per_s": wl.nodes * nsteps / el,
                          "reconstruction_avg_ms": prof["recon_ms"] / max(prof["recon_launches"], 1),
                          "l1_rel_vs_exact": l1_64},
            "split_over_plain": value_f32 / (wl.nodes * nsteps / el)}


def other_configs():
    """The remaining single-GPU configurations: SBR 64^2 FP64 (one revolution,
    L1 against the exact solution and the oracle), the swirl at 4096^2 (the
    HBM-roofline size), the 3-D Fourier flow at 256^3 (FP32 split, 50 steps)
    and the 3-D deformation at 512^3 (plain FP64 and FP32 split, 60 steps)."""
    import oracle
    from paper_1410_2817_amd import workloads as W
    res = {}

    # SBR 64^2: one revolution (100 steps).
    wl = W.solid_body_gaussian(64, 100)
    out, el, prof, st = run_gpu(wl, 100)
    got = out[0].double().cpu().numpy()
    exact = np.asarray(wl.fields[0], np.float64)
    prob = _oracle_problem(oracle, wl)
    rc, ofs, _ = oracle.run(prob, 0.0, wl.dt, 100, [exact])
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
    res["swirl4096_f32"] = {"node_updates_per_s": wl.nodes * n4 / el, "ms_per_step": el * 1e3 / n4,
                            "steps": n4, "reconstruction_avg_ms": rms,
                            "trajectories_avg_ms": prof["traj_ms"] / max(prof["traj_launches"], 1),
                            "order_words_avg_ms": prof["orders_ms"] / max(prof["orders_launches"], 1),
                            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                         "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                                         "bytes_per_node": per_node}}
    del out

    # 3-D configurations.
    cases = [("fourier3d_256_f32", W.fourier3d_three_fields(256, value_prec="f32"), 50, "f32"),
             ("deform3d_512_f64", W.deform3d_slotted_sphere(512), 60, "f64"),
             ("deform3d_512_f32", W.deform3d_slotted_sphere(512), 60, "f32")]
    keep = {}
    for name, wl, nsteps, prec in cases:
        out, el, prof, st = run_gpu(wl, nsteps, prec=prec)
        rms = prof["recon_ms"] / max(prof["recon_launches"], 1)
        vb = 4 if prec == "f32" else 8
        per_node = recon_bytes_per_node(3, wl.nfields, vb) + traj_bytes_per_node(3)
        ach = per_node * wl.nodes / (rms * 1e-3) / 1e9
        res[name] = {"node_updates_per_s": wl.nodes * nsteps / el, "ms_per_step": el * 1e3 / nsteps,
                     "steps": nsteps, "reconstruction_avg_ms": rms,
                     "trajectories_avg_ms": prof["traj_ms"] / max(prof["traj_launches"], 1),
                     "order_words_avg_ms": prof["orders_ms"] / max(prof["orders_launches"], 1),
                     "hbm_achieved_gbs": ach, "hbm_frac": ach / HBM_PEAK_GBS,
                     "valu_roof": valu_roof({"fourier3d_256_f32": "fourier3d_f32/recon3d_kernel<float, 3>",
                                             "deform3d_512_f64": "deform3d_f64/recon3d_kernel<double, 1>",
                                             "deform3d_512_f32": "deform3d_f32/recon3d_kernel<float, 1>"}
                                            .get(name, ""), rms),
                     "order_hist": st["order_hist"], "walked": st["walked"]}
        if name.startswith("deform3d"):
            keep[prec] = out[0].double().cpu().numpy()
        del out
    # Split form against plain FP64 after the same 60 steps.
    res["deform3d_512_f32"]["l1_rel_vs_f64_plain"] = _l1(keep["f32"], keep["f64"])
    res["deform3d_512_f64_shard"] = shard_config(W.deform3d_slotted_sphere(512), 60)

    # Burgers' equation (velocity carried by the fields), the paper's radial
    # shock test at 512^2 up to t = 0.3, plus its first 20 steps against the
    # oracle.
    wl = W.burgers(512)
    out, el, prof, st = run_gpu(wl, wl.nsteps)
    brms = prof["recon_ms"] / max(prof["recon_launches"], 1)
    # Each launch reconstructs 2 FP64 fields and writes the next displacement.
    bgbs = (recon_bytes_per_node(2, 2, 8) + traj_bytes_per_node(2)) * wl.nodes / (brms * 1e-3) / 1e9
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
    # Self-convergence at t = 0.3 (the shock has formed): 256^2, 512^2, 1024^2
    # compared at the shared nodes (coarse node i is fine node 2i).
    us = {}
    for n in (256, 512, 1024):
        wln = W.burgers(n)
        o, _, _, _ = run_gpu(wln, wln.nsteps, profile=0, warmup=0)
        us[n] = [f.double().cpu().numpy() for f in o]
        del o
    def _d(a, b):
        return (sum(float(np.abs(x[::2, ::2] - y).sum()) for x, y in zip(us[a], us[b])) /
                sum(float(np.abs(y).sum()) for y in us[b]))
    d1, d2 = _d(512, 256), _d(1024, 512)
    res["burgers2d_512_f64"]["self_convergence_t03"] = {
        "l1_rel_512_vs_256": d1, "l1_rel_1024_vs_512": d2, "order": float(np.log2(d1 / d2))}
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
    relative L2 error of h against the exact wave and the observed order, at
    the paper's amplitude 1e-4 on coarse grids and at 1e-7 (the linear limit,
    where the exact wave is exact for the equations) up to 1024^2; the 1024^2
    run timed; the non-linear viscous run at 1024^2; and 8 non-linear steps at
    256^2 against the oracle."""
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
                        "kelvin_f64/recon2d_tiled_kernel<double, 3>", krms),
                    "valu_roof_stage": valu_roof("kelvin_f64/sw_stage_kernel<double, 2>", ksms),
                    "reconstructions_per_step": 3, "source_launches_per_step": 6,
                    "search_fail": st["search_fail"], "l2_rel_vs_exact_t1": err}
            del out
        for a, b in zip(rows, rows[1:]):
            b["order"] = float(np.log2(a["l2_rel_vs_exact"] / b["l2_rel_vs_exact"]))
        return rows

    res["kelvin_convergence_amp1e-4_f64"] = ladder(1e-4, (32, 64, 128, 256))
    res["kelvin_convergence_amp1e-7_f64"] = ladder(1e-7, (64, 128, 256, 512, 1024))
    ladder(1e-4, (1024,))
    # Non-linear viscous run (Sec. 3, the Kelvin-Poincare dispersion of the
    # paper's figure): timed at 1024^2, and its self-convergence at t = 1 from
    # 256^2, 512^2 and 1024^2 (coarse node i is fine node 2i).
    hs = {}
    for n in (256, 512, 1024):
        wl = W.kelvin(n, amp=0.5, nu=5e-4, t_end=1.0)
        out, el, prof, st = run_gpu(wl, wl.nsteps, warmup=0 if n < 1024 else 2)
        hs[n] = out[2].double().cpu().numpy()
        if n == 1024:
            res["kelvin_nonlinear_1024_f64"] = {
                "node_updates_per_s": wl.nodes * wl.nsteps / el,
                "ms_per_step": el * 1e3 / wl.nsteps, "steps": wl.nsteps,
                "search_fail": st["search_fail"], "walked": st["walked"],
                "max_h": float(out[2].double().abs().max().item())}
        del out
    d1 = float(np.abs(hs[512][::2, ::2] - hs[256]).sum() / np.abs(hs[256]).sum())
    d2 = float(np.abs(hs[1024][::2, ::2] - hs[512]).sum() / np.abs(hs[512]).sum())
    res["kelvin_nonlinear_1024_f64"]["self_convergence_t1"] = {
        "l1_rel_512_vs_256": d1, "l1_rel_1024_vs_512": d2, "order": float(np.log2(d1 / d2))}
    wl = W.kelvin(256, amp=0.5, nu=5e-4, t_end=1.0)
    out, _, _, _ = run_gpu(wl, 8, profile=0, warmup=0)
    rc, ofs, _ = oracle.run_source(_oracle_problem(oracle, wl), 0.0, wl.dt, 8,
                                   [np.asarray(f, np.float64) for f in wl.fields])
    res["kelvin_nonlinear_256_f64"] = {"l1_rel_vs_oracle_8_steps": [
        _l1(g.double().cpu().numpy(), o) for g, o in zip(out, ofs)]}
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


def run_serving(count: int, budget_gib: float):
    """Serving mix: `count` seeded requests (2-D periodic grids with sides in
    {128, ..., 2048}, 1-4 fields, 10-50 steps of a 16-mode Fourier flow, FP32
    values / FP64 positions) through the continuous-batching server with an
    HBM budget of `budget_gib`.  First all requests arrive at once (capacity),
    then with Poisson arrivals at 0.7 x that capacity (latency)."""
    from paper_1410_2817_amd import serving as S
    from paper_1410_2817_amd import workloads as W
    budget = int(budget_gib * (1 << 30))
    burst = W.serving_stream(seed=0, count=count, rate=1e9)
    for r in burst:
        r.arrival = 0.0
    cap = S.run_stream(burst, budget, max_requests=256)
    rate = 0.7 * count / cap["makespan_s"]
    rep = S.run_stream(W.serving_stream(seed=0, count=count, rate=rate), budget,
                       max_requests=256)
    keep = ("latency_p50_ms", "latency_p99_ms", "latency_mean_ms", "queue_wait_p50_ms",
            "queue_wait_p99_ms", "node_updates_per_s", "makespan_s", "ticks", "status")
    # Whole-job effective HBM rate of the capacity run: the algorithmic bytes of
    # every step of every request (FP32 values; each reconstruction also writes
    # the next step's displacement) over the makespan, all launches and gaps
    # included.
    alg = sum(r.nodes * r.nsteps * (recon_bytes_per_node(2, r.nfields, 4) + traj_bytes_per_node(2))
              for r in burst)
    eff = alg / cap["makespan_s"] / 1e9
    return {"requests": count, "budget_gib": budget_gib,
            "capacity_node_updates_per_s": cap["node_updates_per_s"],
            "capacity_requests_per_s": count / cap["makespan_s"],
            "capacity_effective_hbm_gbs": eff, "capacity_effective_hbm_frac": eff / HBM_PEAK_GBS,
            "poisson_rate_per_s": rate, **{k: rep[k] for k in keep}}


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
