#!/usr/bin/env python3
"""Benchmark of the coupled viscoelastic IB-LB step on one MI355X.

One "step" is one full coupled update of every lattice site (fused field kernel + body update).
Prints ONE JSON line with MLUPS (whole job), the roofline of the dominant kernel (the fused field
kernel, HBM-bound, algorithmic bytes / launch duration measured with HIP events on the library's
stream) and the FP64 CPU oracle timed on a bounded sample of the same workload.

After the field-kernel roofline, the surrogate leg trains the network ensemble on 4096 LB runs of
128 x 128 and reports its held-out error and its speedup over the batched LB at a 2% error bound
(the "surrogate" object of the JSON line).

Default workload: the HBM-bound precision form, 2048 x 2048 periodic with 8 bodies (radius 12-24)
and FP16 population offsets (FP32 arithmetic).  --workload c2 runs the 512 x 512 single FP32
simulation (cache-resident), c4 the 256-simulation ensemble.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS and % HBM roofline per coupled step; surrogate-vs-LB speedup at 2% error"
HBM_PEAK_GBS = 8000.0
# MI355X vector peaks from its unit counts: 256 compute units x 4 SIMDs at 2.4 GHz; one wave64 VALU
# instruction per SIMD every 4 cycles (614.4 G wave instructions/s); FP32 157.3 TFLOP/s with
# packed FP32 instructions, half that without (this build forbids them)
VALU_ISSUE_PEAK_G = 1024 * 2.4e9 / 4 / 1e9
FP32_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_per_site(precision: int) -> int:
    """Algorithmic HBM bytes per site update: the state {h, sigma, P} read once and written once,
    populations 9 x (4 B FP32 | 2 B FP16), stress 3 x 4 B and polarization 2 x 4 B: 112 B in the
    FP32 form, 76 B with FP16 populations.  The library's own storage may hold more (its
    state_bytes()); the difference is reported beside the roofline, never counted in it."""
    pop = 9 * (2 if precision == 1 else 4)
    return 2 * (pop + 3 * 4 + 2 * 4)


def workload(name: str, steps: int):
    from paper_2209_14889_amd import workload as wl
    if name == "c2":
        w = wl.c2(steps=steps)
        desc = "D2Q9 512x512 periodic, 1 body R=16 N=100, pull 5e-5, directors 30deg+N(0,0.1), relax 200, D=0.02"
        return w, desc, 0
    if name == "c3":
        w = wl.c3(steps=steps)
        desc = "D2Q9 2048x2048 periodic, 8 bodies R 12-24, FP16 population offsets (x2^10), FP32 math"
        return w, desc, 1
    if name == "c3fp32":
        w = wl.c3(steps=steps)
        desc = "D2Q9 2048x2048 periodic, 8 bodies R 12-24, FP32 populations"
        return w, desc, 0
    if name == "c1":
        w = wl.c1(steps=steps)
        return w, "D2Q9 64x64 periodic, 1 body R=6 N=40, random directors", 0
    if name == "c4":
        w = wl.c4(steps=steps)
        return w, "256-simulation ensemble, sizes {64..512}^2, one body each", 0
    if name == "paper":
        w = wl.paper_case()
        return w, ("the paper's experiment (Tables I-IV): 250x250 closed box, tau 1.25, 157-node droplet dragged 100 "
                   "sites over 25000 steps by the trap, 187500 steps"), 0
    if name == "paper_scalar":
        w = wl.paper_case(scalar=True)
        return w, ("the paper's experiment with the scalar model (Sec. II B, C = 0.01 Pa): 250x250 closed box, "
                   "157-node droplet dragged 100 sites over 25000 steps by the trap, 187500 steps"), 0
    raise SystemExit(f"unknown workload {name}")


KERNEL_SOURCES = ["paper_2209_14889_amd/csrc/lb_kernels.hip", "paper_2209_14889_amd/csrc/lb_device.h",
                  "paper_2209_14889_amd/csrc/lb_common.h"]


def kernel_code_digest() -> str:
    """sha256 of the fused kernel's sources with comments and white space removed, and of the flags
    they are compiled with: only a change of the code or of its compilation makes committed
    counters stale."""
    import hashlib
    import re
    from paper_2209_14889_amd import build as _build
    h = hashlib.sha256()
    h.update(" ".join(_build.flags_for("lb_kernels.hip")).encode())
    for p in KERNEL_SOURCES:
        t = open(os.path.join(ROOT, p)).read()
        t = re.sub(r"/\*.*?\*/", " ", t, flags=re.S)
        t = re.sub(r"//[^\n]*", " ", t)
        h.update(" ".join(t.split()).encode())
    return h.hexdigest()


def counted_traffic(workload_name: str, shape: dict):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary (copy-kernel calibrated), or None when that summary is for another workload or launch
    shape, or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles",
                        f"k_fused_{workload_name}_t{shape['threads']}_s{shape['seg_rows']}_hbm_counters.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("code_sha256") != kernel_code_digest() or d.get("workload") != workload_name:
        return None
    if d["launch"]["threads"] != shape["threads"] or d["launch"]["seg_rows"] != shape["seg_rows"]:
        return None
    return round(d["traffic_bytes"] / 1e9, 4)


def counted_alu(workload_name: str, shape: dict, launch_us: float):
    """The ALU side of the roofline from the committed SQ counters of the fused kernel (VALU
    instructions per launch and their FP32/FP64 add, mul and fma mix), or None when they are for
    another workload or launch shape, or the kernel sources changed since they were taken."""
    path = os.path.join(ROOT, "profiles",
                        f"k_fused_{workload_name}_t{shape['threads']}_s{shape['seg_rows']}_sq_counters.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("code_sha256") != kernel_code_digest() or d.get("workload") != workload_name:
        return None
    if d["launch"]["threads"] != shape["threads"] or d["launch"]["seg_rows"] != shape["seg_rows"]:
        return None
    c = d["counters"]
    sec = launch_us * 1e-6
    f32 = 64 * (c["SQ_INSTS_VALU_ADD_F32"] + c["SQ_INSTS_VALU_MUL_F32"] + 2 * c["SQ_INSTS_VALU_FMA_F32"])
    f64 = 64 * (c["SQ_INSTS_VALU_ADD_F64"] + c["SQ_INSTS_VALU_MUL_F64"] + 2 * c["SQ_INSTS_VALU_FMA_F64"])
    issue = c["SQ_INSTS_VALU"] / sec / 1e9
    return {"bound": "alu", "unit": "TFLOP/s", "achieved": round(f32 / sec / 1e12, 2), "peak": FP32_PEAK_TFLOPS,
            "frac": round(f32 / sec / 1e12 / FP32_PEAK_TFLOPS, 4),
            "frac_of_nonpacked": round(f32 / sec / 1e12 / (FP32_PEAK_TFLOPS / 2), 4),
            "fp32_flops_per_launch": f32, "fp64_flops_per_launch": f64,
            "valu_issue": {"achieved": round(issue, 1), "peak": VALU_ISSUE_PEAK_G, "unit": "G wave instructions/s",
                           "frac": round(issue / VALU_ISSUE_PEAK_G, 4)},
            "source": os.path.relpath(path, ROOT)}


def _db(path: str) -> str:
    import glob
    if path.endswith(".db"):
        return path
    found = sorted(glob.glob(os.path.join(path, "**", "*_results.db"), recursive=True))
    if not found:
        raise SystemExit(f"no rocprofv3 results database under {path}")
    return found[0]


def _counter_kib(db: str, kernel_prefix: str):
    """Mean counter value (KiB) per dispatch of the kernels whose name starts with kernel_prefix."""
    import sqlite3
    con = sqlite3.connect(_db(db))
    rows = con.execute("select kernel_name, counter_name, value from counters_collection").fetchall()
    vals = [v for k, c, v in rows if k.startswith(kernel_prefix)]
    if not vals:
        raise SystemExit(f"no dispatch of {kernel_prefix} in {db}")
    return sum(vals) / len(vals), len(vals), rows[0][1]


def counters_summary(outdir: str, workload_name: str, threads: int, seg_rows: int, command: str):
    """Turn four rocprofv3 --pmc runs (copy FETCH_SIZE, copy WRITE_SIZE, fused FETCH_SIZE, fused
    WRITE_SIZE, in <outdir>/pmc_copy_f, pmc_copy_w, pmc_<workload>_f, pmc_<workload>_w) into the
    calibrated HBM traffic of one fused launch of the given shape:
    profiles/k_fused_<workload>_t<threads>_s<seg_rows>_hbm_counters.{json,md}."""
    copy_bytes = 64 * 1024 * 1024 * 4
    cf, _, _ = _counter_kib(os.path.join(outdir, "pmc_copy_f"), "lbk::k_stream_copy")
    cw, _, _ = _counter_kib(os.path.join(outdir, "pmc_copy_w"), "lbk::k_stream_copy")
    tag = f"{workload_name}_t{threads}_s{seg_rows}"
    kf, nf, _ = _counter_kib(os.path.join(outdir, f"pmc_{tag}_f"), "void lbk::k_fused")
    kw, nw, _ = _counter_kib(os.path.join(outdir, f"pmc_{tag}_w"), "void lbk::k_fused")
    # the copy reads and writes copy_bytes once: the factors that turn each counter into bytes
    fetch_scale = copy_bytes / (cf * 1024.0)
    write_scale = copy_bytes / (cw * 1024.0)
    w, _, precision = workload(workload_name, 1)
    alg = bytes_per_site(precision) * w.sites
    d = {
        "kernel": "k_fused", "workload": workload_name, "launch": {"threads": threads, "seg_rows": seg_rows},
        "copy_bytes": copy_bytes, "fetch_scale": fetch_scale, "write_scale": write_scale,
        "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw, "dispatches": [nf, nw],
        "fetch_bytes": kf * 1024.0 * fetch_scale, "write_bytes": kw * 1024.0 * write_scale,
        "algorithmic_bytes": alg, "sources": KERNEL_SOURCES, "code_sha256": kernel_code_digest(),
    }
    d["traffic_bytes"] = d["fetch_bytes"] + d["write_bytes"]
    base = os.path.join(ROOT, "profiles", f"k_fused_{workload_name}_t{threads}_s{seg_rows}_hbm_counters")
    with open(base + ".json", "w") as f:
        json.dump(d, f, indent=1)
    half = alg / 2
    with open(base + ".md", "w") as f:
        f.write(f"# HBM byte counters: k_fused, workload {workload_name} (threads {threads}, {seg_rows} rows per item)\n\n")
        f.write("Commands (one counter per run, each run alone), then the summary:\n\n```\n" + command.strip() + "\n```\n\n")
        f.write(f"Calibration: a {copy_bytes >> 20} MiB device copy reads FETCH_SIZE = {cf:.1f} KiB and writes "
                f"WRITE_SIZE = {cw:.1f} KiB per dispatch: scale factors {fetch_scale:.4f} (fetch) and "
                f"{write_scale:.4f} (write).\n\n")
        f.write(f"k_fused per dispatch (mean of {nf} and {nw} dispatches): FETCH_SIZE = {kf:.1f} KiB -> "
                f"{d['fetch_bytes'] / 1e6:.1f} MB; WRITE_SIZE = {kw:.1f} KiB -> {d['write_bytes'] / 1e6:.1f} MB.\n\n")
        f.write(f"Algorithmic bytes: {bytes_per_site(precision)} B/site x {w.sites} sites = {alg / 1e6:.1f} MB per launch "
                f"({half / 1e6:.1f} MB each way).\n\n")
        f.write(f"Measured / algorithmic: reads {d['fetch_bytes'] / half:.3f}, writes {d['write_bytes'] / half:.3f}.\n")
    log(f"bench: wrote {base}.json/.md")


def trace_summary(db: str, title: str, command: str, out: str, top: int = 8):
    """Markdown table of the rocprofv3 --kernel-trace --stats top kernels (name, calls, mean us, %)."""
    import sqlite3
    con = sqlite3.connect(_db(db))
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    with open(os.path.join(ROOT, "profiles", out), "w") as f:
        f.write(f"# {title}\n\nCommand:\n\n```\n{command.strip()}\n```\n\n")
        f.write("| kernel | calls | total us | mean us | % |\n|---|---|---|---|---|\n")
        for name, calls, tot, avg, pct in rows[:top]:
            f.write(f"| `{name}` | {calls} | {tot:.1f} | {avg:.2f} | {pct:.1f} |\n")
    log(f"bench: wrote profiles/{out}")


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """GB/s (bytes read + bytes written) of the library's streaming copy kernel (lb_stream_copy)
    over nbytes, best of reps, timed with HIP events on the stream it runs on."""
    import torch
    from paper_2209_14889_amd import lb
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    st = torch.cuda.current_stream()
    lb.stream_copy(a, b, st)
    torch.cuda.synchronize()
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        lb.stream_copy(a, b, st)
        e1.record(st)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    assert bool(torch.equal(a[:4096], b[:4096])) and bool(torch.equal(a[-4096:], b[-4096:]))
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / best / 1e9


def host_cpus() -> dict:
    """The host the oracle runs on: logical CPUs, the CPUs this process may run on, the model."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable": usable, "model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(w, name: str, budget_s: float = 15.0):
    """FP64 oracle on the host: the full coupled step on the workload's first simulation for as
    many steps as fit in about budget_s seconds (at least 2), on every CPU this process may use
    (on a GPU machine that is its share of the host, which OMP_NUM_THREADS also states), then on one
    thread for a third of the budget."""
    import oracle
    cpus = host_cpus()
    oracle.set_threads(cpus["usable"])
    s = w.sims[0]
    p = s.params
    bodies = [oracle.Body(R=b.R.copy(), k_spring=b.k_spring, eps_angle=b.eps_angle, l_eq=b.l_eq, pull=b.pull,
                          t_on=b.t_on, t_off=b.t_off, width=b.width, trap=b.trap) for b in s.bodies]
    sim = oracle.Sim(dict(nx=s.nx, ny=s.ny, tau=p["tau"], Kx=p["Kx"], eta_p=p["eta_p"], D_p=p["D_p"], xi=p["xi"],
                          alpha=p["alpha"], beta=p["beta"], kappa=p["kappa"], Gamma=p["Gamma"],
                          P_clamp=p["P_clamp"], ericksen=p["ericksen"]), bodies=bodies, P=s.P0.copy())
    t0 = time.perf_counter()
    sim.run(1)
    dt1 = time.perf_counter() - t0
    n = max(2, min(200, int(budget_s / max(dt1, 1e-6))))
    t0 = time.perf_counter()
    sim.run(n)
    dt = time.perf_counter() - t0
    sites = s.nx * s.ny
    cores = int(oracle.get_threads())
    # the same oracle on one thread, for a third of the budget
    oracle.set_threads(1)
    t0 = time.perf_counter()
    sim.run(1)
    dt1 = time.perf_counter() - t0
    n1 = max(1, min(200, int(budget_s / 3 / max(dt1, 1e-6))))
    t0 = time.perf_counter()
    sim.run(n1)
    dt_1 = time.perf_counter() - t0
    oracle.set_threads(cores)
    return {"value": round(sites * n / dt / 1e6, 4), "unit": "MLUPS", "cores": cores,
            "kind": "oracle", "sample": (f"{name}: first simulation {s.nx}x{s.ny}, {n} coupled steps after 1 warm-up "
                                         f"step, OpenMP on all {cores} CPUs this process may use"),
            "host": cpus,
            "single_thread": {"value": round(sites * n1 / dt_1 / 1e6, 4), "unit": "MLUPS",
                              "sample": f"{n1} more steps on one thread after 1 warm-up step"}}


def field_kernel_timing(w, precision: int, shape: dict, kernel: int, steps: int):
    """Average duration of the fused field kernel: HIP events recorded on the library's stream
    around each of `steps` plain launches (same kernel and launch shape as the timed run), and the
    body update's the same way."""
    from paper_2209_14889_amd import lb
    topt = lb.make_options(precision=precision, kernel=kernel, timing=1, seg_rows=shape["seg_rows"],
                           fused_threads=shape["threads"],
                           grid=shape["grid"] if shape["grid"] < shape["n_items"] else 0)
    tsim = lb.Sim(w, topt)
    tsim.step(20)
    tsim.timing(reset=True)
    tsim.step(steps)
    tm = tsim.timing()
    stored = tsim.state_bytes()
    tsim.close()
    avg_ms = tm["field_ms"] / max(1, tm["field_launches"])
    ib_ms = tm["ib_ms"] / max(1, tm["ib_launches"]) if tm["ib_launches"] else 0.0
    return avg_ms, ib_ms, stored


def roofline(precision: int, sites: int, avg_ms: float, stored: float, copy_gbps: float | None) -> dict:
    bps = bytes_per_site(precision)
    achieved = bps * sites / (avg_ms * 1e-3) / 1e9
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": "k_fused", "bytes_per_site": bps,
         "algorithmic_gb_per_launch": round(bps * sites / 1e9, 4), "launch_us": round(avg_ms * 1e3, 3),
         "stored_bytes_per_site": stored, "storage_surplus_bytes_per_site": stored - bps,
         "stored_gbps": round(stored * sites / (avg_ms * 1e-3) / 1e9, 1)}
    if copy_gbps:
        r["copy_gbps"] = round(copy_gbps, 1)
        r["frac_of_copy"] = round(achieved / copy_gbps, 4)
    return r


def c4_leg(args) -> dict:
    """The 256-simulation ensemble (the other HBM-bound workload): one handle, one fused launch per
    step over all 14.7 M sites, timed over a graph-replayed run, and its field-kernel roofline."""
    import torch
    from paper_2209_14889_amd import lb
    w, desc, precision = workload("c4", args.c4_steps)
    opt = lb.make_options(precision=precision, graph_chunk=args.graph_chunk, autotune=1)
    sim = lb.Sim(w, opt)
    shape = sim.launch_shape()
    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.c4_steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sim.close()
    avg_ms, ib_ms, stored = field_kernel_timing(w, precision, shape, 0, min(args.timing_steps, 100))
    out = {"workload": f"c4: {desc}", "sites": w.sites, "steps": args.c4_steps,
           "value": round(w.sites * args.c4_steps / dt / 1e6, 2), "unit": "MLUPS",
           "ms_per_step": round(dt / args.c4_steps * 1e3, 5), "threads": shape["threads"],
           "seg_rows": shape["seg_rows"], "work_items": shape["n_items"],
           "roofline": roofline(precision, w.sites, avg_ms, stored, None), "body_update_us": round(ib_ms * 1e3, 3)}
    out["roofline"]["traffic"] = counted_traffic("c4", shape)
    out["roofline"]["traffic_unit"] = "GB per launch"
    out["roofline"]["alu"] = counted_alu("c4", shape, avg_ms * 1e3)
    log(f"bench: c4 ensemble {out['value']} MLUPS, field kernel {avg_ms * 1e3:.1f} us, "
        f"frac {out['roofline']['frac']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--kernel", type=int, default=0, help="0 fused, 1 multi-pass")
    ap.add_argument("--graph-chunk", type=int, default=100)
    ap.add_argument("--seg-rows", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--timing-steps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c4", action="store_true", help="skip the 256-simulation ensemble leg")
    ap.add_argument("--c4-steps", type=int, default=200, help="timed steps of the ensemble leg")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate leg (4096 + 512 LB runs of 128^2, network training, fallback)")
    ap.add_argument("--counters-summary", default="",
                    help="directory holding rocprofv3 --pmc outputs pmc_copy_f/w and "
                         "pmc_<workload>_t<threads>_s<seg_rows>_f/w: "
                         "write the calibrated HBM traffic summary under profiles/ (no GPU use)")
    ap.add_argument("--trace-summary", default="", help="rocprofv3 --kernel-trace --stats output: write a "
                    "markdown table of its top kernels to profiles/<--summary-name> (no GPU use)")
    ap.add_argument("--summary-name", default="")
    ap.add_argument("--summary-title", default="")
    ap.add_argument("--summary-command", default="", help="the command that produced the profiler output")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 256 MiB device buffer 5 times with the library's copy kernel (reference for the "
                         "HBM byte counters)")
    args = ap.parse_args()
    if args.counters_summary:
        counters_summary(args.counters_summary, args.workload, args.threads, args.seg_rows, args.summary_command)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary, args.summary_title or args.summary_name, args.summary_command,
                      args.summary_name)
        return
    if args.copy_calibration:
        import torch
        from paper_2209_14889_amd import lb
        n = 64 * 1024 * 1024
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            lb.stream_copy(src, dst)
        torch.cuda.synchronize()
        log(f"bench: copied {n * 4} bytes 5 times with the library's streaming copy kernel")
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): liblb has no multi-GPU "
              "path; independent simulations shard across GPUs with no exchange and one large lattice would "
              "use slab halos, neither of which is built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2209_14889_amd import lb
    from paper_2209_14889_amd import workload as wl_mod

    w, desc, precision = workload(args.workload, args.steps)
    sites = w.sites
    log(f"bench: workload {args.workload} ({desc}), {sites} sites, warmup {args.warmup}, steps {args.steps}")

    opt = lb.make_options(precision=precision, kernel=args.kernel, graph_chunk=args.graph_chunk,
                          seg_rows=args.seg_rows, fused_threads=args.threads,
                          autotune=0 if (args.no_autotune or args.seg_rows) else 1)
    sim = lb.Sim(w, opt)
    shape = sim.launch_shape()
    log(f"bench: fused launch shape {shape}")
    paper = args.workload.startswith("paper")
    failure = None
    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if paper:
        # the whole protocol in chunks, so a watchdog stop is reported with the step it came at
        done = 0
        while done < args.steps and failure is None:
            n = min(12500, args.steps - done)
            try:
                sim.step(n)
                sim.sync()
            except lb.LBError as e:
                failure = f"stopped at step {sim.t}: {e}"
                break
            done += n
            log(f"bench: {args.warmup + done} steps")
    else:
        sim.step(args.steps)
        sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mlups = sites * args.steps / dt / 1e6
    log(f"bench: {args.steps} steps in {dt:.4f} s -> {mlups:.1f} MLUPS")
    experiment = None
    if paper:
        # the droplet's Return (Sec. III) once the whole protocol has run
        b0 = w.sims[0].bodies[0]
        total = args.warmup + args.steps
        if failure is None:
            com = sim.body_forces()[0, 4:6]
            from paper_2209_14889_amd.experiment import return_value
            ret = (return_value((b0.trap["x0"], b0.trap["y0"]), com, b0.trap["dx"])
                   if total >= wl_mod.PAPER_STEPS else None)
            experiment = {"steps": total, "timed_s": round(dt, 3), "return": None if ret is None else round(ret, 4),
                          "final_com": [round(float(c), 4) for c in com]}
        else:
            experiment = {"steps": total, "timed_s": round(dt, 3), "return": None, "failure": failure}
        experiment["paper_cpu_wall"] = ("about 4 h for 187500 steps of the scalar model on one CPU (App. C)"
                                        if args.workload == "paper_scalar" else
                                        "about 20 h for 187500 steps on one CPU (App. C)")
        log(f"bench: paper experiment {experiment}")
        if failure is not None:
            mlups = sites * done / dt / 1e6
    pcie = None
    if not paper:
        # context, not `value`: the same run with its host traffic, i.e. a handle created from the
        # host arrays (upload, initial spreading) and every field of every simulation read back
        t_r = time.perf_counter()
        for i in range(len(w.sims)):
            sim.fields(i)
        t_read = time.perf_counter() - t_r
        torch.cuda.synchronize()
        t_c = time.perf_counter()
        up = lb.Sim(w, lb.make_options(precision=precision, kernel=args.kernel, graph_chunk=args.graph_chunk,
                                       seg_rows=shape["seg_rows"], fused_threads=shape["threads"]))
        up.sync()
        t_up = time.perf_counter() - t_c
        up.close()
        pcie = {"value": round(sites * args.steps / (dt + t_up + t_read) / 1e6, 2), "unit": "MLUPS",
                "upload_s": round(t_up, 4), "readback_s": round(t_read, 4)}
        log(f"bench: with the host traffic (create from host arrays {t_up:.3f} s, read back every field "
            f"{t_read:.3f} s): {pcie['value']} MLUPS")
    sim.close()

    # roofline of the dominant kernel: HIP events around every field-kernel launch on the
    # library's stream (plain launches, same kernel and launch configuration)
    avg_ms, ib_ms, stored = field_kernel_timing(w, precision, shape, args.kernel, args.timing_steps)
    # the achievable streaming bandwidth on this device: the library's own copy kernel over 1 GiB
    copy_gbps = copy_bandwidth()
    log(f"bench: streaming copy kernel {copy_gbps:.0f} GB/s (read + write)")
    roof = roofline(precision, sites, avg_ms, stored, copy_gbps)
    roof["traffic"] = counted_traffic(args.workload, shape)
    roof["traffic_unit"] = "GB per launch"
    roof["alu"] = counted_alu(args.workload, shape, avg_ms * 1e3)
    log(f"bench: field kernel {avg_ms * 1e3:.2f} us/launch, body kernel {ib_ms * 1e3:.2f} us/launch, "
        f"{roof['achieved']:.0f} GB/s algorithmic ({roof['bytes_per_site']} B/site), frac {roof['frac']}")
    c4 = None
    if args.workload == "c3" and not args.no_c4:
        c4 = c4_leg(args)

    sur = None
    if not args.no_surrogate:
        from paper_2209_14889_amd import surrogate
        log("bench: surrogate study (LB data, ensemble training, held-out error and speedup)")
        sur = surrogate.study(log=log)
        log(f"bench: surrogate speedup {sur['speedup']}x, held-out error with fallback "
            f"max {sur['err_with_fallback']['max']:.4f}")

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on the host")
        cpu = cpu_baseline(w, args.workload)
        log(f"bench: oracle {cpu['value']} MLUPS on {cpu['cores']} threads")

    line = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16-storage/f32" if precision == 1 else "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "sites": sites,
                   "kernel": "fused" if args.kernel == 0 else "multipass", "graph_chunk": args.graph_chunk,
                   "threads": shape["threads"], "seg_rows": shape["seg_rows"], "work_items": shape["n_items"],
                   "grid": shape["grid"]},
        "roofline": roof,
        "body_update_us": round(ib_ms * 1e3, 3),
        "cpu_baseline": cpu,
        "surrogate": sur,
    }
    if c4 is not None:
        line["c4"] = c4
    if pcie is not None:
        line["pcie_inclusive"] = pcie
    if experiment is not None:
        line["experiment"] = experiment
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
