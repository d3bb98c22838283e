#!/usr/bin/env python3
"""Throughput of the fused RR-MHD step on one MI355X.

Workload: decaying 2D MHD turbulence on an 8192^2 periodic grid (random-phase
stream and flux functions, E(k) ~ k^4 exp(-2 (k/4)^2), rms u = b = 0.04),
tau_f = tau_m = 0.52 (the largest relaxation time of the stated range
0.5005-0.52; at 0.51 and below the FP32 run turns non-finite within 2000
steps, while at 0.52 it stays finite over 10,000), FP32 arithmetic, populations stored as FP32 offsets
f - w (``--storage f16`` for the FP16-offset codec).  A step is one fused
stream-and-collide launch over all 67,108,864 nodes; inputs are resident in
HBM before timing starts.  By default 10,000 steps (the configuration's
horizon) are timed after 100 warm-up steps.

Prints one JSON line.  MLUPS = nodes x steps / seconds / 1e6.  The roofline
object prices the step kernel's algorithmic traffic (19 reads + 19 writes
per node: 152 B in FP32 storage, 76 B in FP16) per launch against 8 TB/s.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_NODE = {"f32": 152, "f16": 76, "f16sr": 76}
def kernel_hash():
    from paper_2602_14667_amd import kernel_hash as kh
    return kh()


def measured_traffic(storage, n, dims=2):
    """HBM bytes per launch from committed rocprofv3 counter summaries, or
    None when absent or taken on another kernel source."""
    from paper_2602_14667_amd import kernel3d_hash
    tag = "step" if dims == 2 else "step3d"
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}_{storage}_{n}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_hash") != (kernel_hash() if dims == 2 else kernel3d_hash()):
        return None
    return t.get("bytes_per_launch")


def batch_traffic():
    """HBM bytes per ensemble launch (default launch shape) from the committed
    counter summary, or None when absent or taken on other kernel sources."""
    from paper_2602_14667_amd import batch_hash
    path = os.path.join(ROOT, "profiles", "traffic_batch_f32_256.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    return t.get("bytes_per_launch") if t.get("kernel_hash") == batch_hash() else None


def environment(torch):
    """Where the numbers were taken: GPU, HIP runtime and torch versions, host
    CPU model and thread count."""
    cpu = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    prop = torch.cuda.get_device_properties(0)
    return {"gpu": torch.cuda.get_device_name(0), "arch": getattr(prop, "gcnArchName", None),
            "device_memory_GiB": round(prop.total_memory / 2 ** 30, 1),
            "compute_units": prop.multi_processor_count, "hip": torch.version.hip,
            "torch": torch.__version__, "cpu_model": cpu, "host_threads": os.cpu_count()}


def cpu_baseline(n_sample=2048, steps=60):
    """The FP64 oracle on a bounded sample of the same workload: all host
    threads on 2048^2 x 60 steps, and one thread on 512^2 x 20 steps."""
    import oracle
    from paper_2602_14667_amd import inputs
    u, b = inputs.turbulence(n_sample, 0.04)
    o = oracle.Oracle(n_sample, n_sample, 0.52, 0.52)
    o.init(u, b)
    o.step(1)  # warm-up
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    cores = oracle.threads()
    o.close()
    # one thread, smaller sample of the same field
    n1, s1 = 512, 20
    u1, b1 = inputs.turbulence(n1, 0.04)
    oracle.set_threads(1)
    o1 = oracle.Oracle(n1, n1, 0.52, 0.52)
    o1.init(u1, b1)
    o1.step(1)
    t1 = time.perf_counter()
    o1.step(s1)
    dt1 = time.perf_counter() - t1
    o1.close()
    oracle.set_threads(cores)
    return {"value": n_sample * n_sample * steps / dt / 1e6, "unit": "MLUPS",
            "cores": cores, "kind": "oracle",
            "sample": f"{n_sample}^2 of the same turbulence field, {steps} "
                      f"steps after 1 warm-up step, FP64, OpenMP rows",
            "seconds": dt,
            "single_thread": {"value": n1 * n1 * s1 / dt1 / 1e6, "unit": "MLUPS",
                              "sample": f"{n1}^2, {s1} steps", "seconds": dt1}}


def cpu_baseline_c1():
    """The FP64 oracle on the whole Orszag-Tang 64^2 case (1000 steps), with
    all host threads and with one."""
    import oracle
    from paper_2602_14667_amd import inputs
    u, b = inputs.orszag_tang(64, 0.05, 0.05, perturb=1e-4, seed=0)
    cores = oracle.threads()
    out = {}
    for label, th in (("all_threads", cores), ("single_thread", 1)):
        oracle.set_threads(th)
        o = oracle.Oracle(64, 64, 0.56, 0.56)
        o.init(u, b)
        t0 = time.perf_counter()
        o.step(1000)
        dt = time.perf_counter() - t0
        o.close()
        out[label] = {"seconds": round(dt, 3), "MLUPS": round(64 * 64 * 1000 / dt / 1e6, 3),
                      "threads": th}
    oracle.set_threads(cores)
    out["kind"] = "oracle"
    return out


def cpu_baseline_c2(steps=40_000, to_steady=490_000):
    """The FP64 oracle on the Hartmann channel's x-invariant section (a
    1 x 256 column, the same profile in y) from rest, timed on a bounded
    sample of steps with all host threads and with one; the projected time
    to the step count at which the GPU run meets the 1e-3 criterion."""
    import numpy as np
    import oracle
    from paper_2602_14667_amd import inputs
    h = inputs.hartmann_c2()
    u = np.zeros((2, h.ny, 1))
    b = np.zeros((2, h.ny, 1))
    b[1] = h.B0
    cores = oracle.threads()
    out = {}
    for label, th in (("all_threads", cores), ("single_thread", 1)):
        oracle.set_threads(th)
        o = oracle.Oracle(1, h.ny, h.tau_f, h.tau_m, walls=True, force=(h.G, 0.0),
                          b_wall=(0.0, h.B0))
        o.init(u, b)
        t0 = time.perf_counter()
        o.step(steps)
        dt = time.perf_counter() - t0
        o.close()
        out[label] = {"seconds": round(dt, 3), "MLUPS": round(h.ny * steps / dt / 1e6, 3),
                      "threads": th,
                      "projected_s_to_steady": round(dt * to_steady / steps, 1)}
    oracle.set_threads(cores)
    out["kind"] = "oracle"
    out["sample"] = f"1x{h.ny} column from rest, {steps} steps, FP64"
    out["steady_steps"] = to_steady
    return out


def copy_reference(torch, rrmhd, args):
    """Plain streaming copy of a known byte count (bandwidth reference and
    calibration of memory-traffic counters)."""
    nb = args.copy_bytes
    a = torch.zeros(nb // 4, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    for _ in range(max(args.warmup, 1)):
        rrmhd.bandwidth_probe(c, a)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.steps):
        rrmhd.bandwidth_probe(c, a)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    print(json.dumps({"mode": "copy", "bytes_read": nb, "bytes_written": nb,
                      "ms_per_copy": ms, "GBs": 2 * nb / ms / 1e6}), flush=True)


def launch_sweep(torch, rrmhd, inputs, args):
    """One JSON line per (plane gap, launch shape, XCD order) of the step
    kernel on the benchmark workload (both storages)."""
    import itertools
    n = args.n
    u, b = inputs.turbulence(n, 0.04)
    ud, bd = torch.from_numpy(u).cuda(), torch.from_numpy(b).cuda()
    del u, b
    st = torch.cuda.current_stream()
    shapes = [(256, 1), (128, 2), (64, 4), (128, 1), (64, 1)]
    if args.inplace:
        shapes += [(32, 8), (256, 1), (32, 4), (16, 16)]
        shapes = list(dict.fromkeys(shapes))
    # single-buffer steps alternate two kernels: time an even number
    steps = args.steps + (args.steps % 2 if args.inplace else 0)
    for storage in ("f32", "f16"):
        for gap in ((256,) if args.inplace else (0, 256, 4352, 65792)):
            os.environ["RRMHD_PLANE_PAD_BYTES"] = str(gap)
            s = rrmhd.Solver(n, n, args.tau, args.tau, storage=storage, inplace=args.inplace)
            s.init(ud, bd)
            s.step(4)
            for (bx, by), xcd, nt in itertools.product(shapes, (0, 1, 2),
                                                       (0, 1)):
                s.set_launch(bx, by, 1, xcd, nt)
                s.step(2)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(st)
                s.step(steps)
                e1.record(st)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / steps
                print(json.dumps({"storage": storage, "inplace": args.inplace,
                                  "plane_gap_bytes": gap,
                                  "bx": bx, "by": by, "xcd": xcd, "nt": nt,
                                  "ms": round(ms, 4),
                                  "GBs": round(BYTES_PER_NODE[storage] * n * n
                                               / ms / 1e6, 1)}), flush=True)
            s.close()
            torch.cuda.empty_cache()
    os.environ.pop("RRMHD_PLANE_PAD_BYTES", None)


def time_batch_leg(torch, rrmhd, inputs, steps, autotune, sequential):
    """The 256-domain ensemble (sides 64..1024, tau uniform in [0.501, 0.6]),
    FP32, graph-captured persistent launches: ms per step over `steps` steps
    (whole graph chunks of 100), with the library's default launch or
    autotuned tiles; optionally the same domains stepped one after another
    as standalone grids, for comparison."""
    doms = inputs.batch_domains(256, seed=0)
    shapes = [(d["side"], d["side"]) for d in doms]
    b = rrmhd.Batch(shapes, [d["tau_f"] for d in doms], [d["tau_m"] for d in doms])
    for k, d in enumerate(doms):
        u, bf = inputs.batch_fields(d)
        b.init(k, torch.from_numpy(u).cuda(), torch.from_numpy(bf).cuda())
    t0 = time.perf_counter()
    if autotune:
        b.autotune(None, trials=10)
    tune_s = time.perf_counter() - t0
    chunk = 100
    b.set_graph_chunk(chunk)
    b.step(chunk)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    steps = max(chunk, (steps // chunk) * chunk)
    e0.record(st)
    b.step(steps)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    info = b.info()
    nodes = info["nodes"]
    seq_ms = None
    if sequential:
        seq_ms = 0.0
        for k, d in enumerate(doms):
            s = rrmhd.Solver(d["side"], d["side"], d["tau_f"], d["tau_m"])
            u, bf = inputs.batch_fields(d)
            s.init(torch.from_numpy(u).cuda(), torch.from_numpy(bf).cuda())
            s.step(2)
            f0 = torch.cuda.Event(enable_timing=True)
            f1 = torch.cuda.Event(enable_timing=True)
            f0.record(st)
            s.step(20)
            f1.record(st)
            torch.cuda.synchronize()
            seq_ms += f0.elapsed_time(f1) / 20
            s.close()
    b.close()
    gbs = 152 * nodes / ms / 1e6
    return {
        "value": round(nodes / ms / 1e3, 1), "unit": "MLUPS", "steps": steps,
        "warmup": chunk, "ms_per_step": round(ms, 4),
        "config": {"workload": "256 periodic domains, sides 64..1024, "
                               "OT or turbulence, tau in [0.501, 0.6]",
                   "nodes": nodes, "tiles": info["tiles"],
                   "workgroups_per_launch": info["grid"],
                   "graph_chunk": chunk, "autotuned": autotune,
                   "autotune_s": round(tune_s, 2)},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(gbs / PEAK_HBM_GBS, 4),
                     "traffic": None if autotune else batch_traffic()},
        "sequential_standalone_ms_per_step": None if seq_ms is None else round(seq_ms, 4),
        "speedup_vs_sequential": None if seq_ms is None else round(seq_ms / ms, 3)}


def batch_bench(torch, rrmhd, inputs, args):
    """The ensemble on its own line, autotuned unless --no-autotune, with the
    sequential standalone comparison."""
    leg = time_batch_leg(torch, rrmhd, inputs, args.steps, not args.no_autotune, True)
    out = {"metric": "MLUPS & % HBM roofline (batched ensemble step)",
           "value": leg["value"], "unit": "MLUPS", "n_gpus": 1, "steps": leg["steps"],
           "warmup": leg["warmup"], "ms_per_step": leg["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic"}
    out.update({k: leg[k] for k in ("config", "roofline", "sequential_standalone_ms_per_step",
                                    "speedup_vs_sequential")})
    print(json.dumps(out), flush=True)


def hartmann_bench(torch, rrmhd, inputs, args):
    """Hartmann channel 512 x 256 (walls, body force G = 1e-6, Ha = 10,
    tau_f 0.6, tau_m 0.55) from rest, FP32 and FP16 storage: steps and GPU
    time until the u_x and b_x profiles are within rel L2 1e-3 of the
    analytic steady state (checked every 10^4 steps, at most 1.2e7 steps),
    or until the stored state stops changing (a rounding fixed point).
    Stochastically rounded FP16 never stops changing: it runs a fixed 10^6
    steps and reports the error band of the x-averaged profile over the
    second half, on an 8-wide channel: its noise breaks the x-invariance
    that the deterministic storages keep exactly, and the 512-wide channel
    has a long-wavelength mode in x that grows from any such perturbation
    (FP32 storage included), while every mode of the narrow one decays."""
    import numpy as np
    h = inputs.hartmann_c2()
    u, b = h.initial_fields()
    ud, bd = torch.from_numpy(u).cuda(), torch.from_numpy(b).cuda()
    ue, be = h.profile(np.arange(h.ny))
    st = torch.cuda.current_stream()
    out = {}
    for storage in ("f32", "f16", "f16sr"):
        nx = 8 if storage == "f16sr" else h.nx
        s = rrmhd.Solver(nx, h.ny, h.tau_f, h.tau_m, storage=storage, walls=True,
                         force=(h.G, 0.0), b_wall=(0.0, h.B0))
        s.init(ud[:, :, :nx].contiguous(), bd[:, :, :nx].contiguous())
        prev = None
        gpu_ms = 0.0
        status = "cap"
        cap = 1_000_000 if storage == "f16sr" else 12_000_000
        hist = []
        while s.step_count < cap:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            s.step(10_000)
            e1.record(st)
            _, uu, bb = s.moments()
            torch.cuda.synchronize()
            gpu_ms += e0.elapsed_time(e1)
            gu, gb = uu[0].mean(1).cpu().numpy(), bb[0].mean(1).cpu().numpy()
            eu = np.linalg.norm(gu - ue) / np.linalg.norm(ue)
            eb = np.linalg.norm(gb - be) / np.linalg.norm(be)
            hist.append((s.step_count, float(eu), float(eb)))
            if storage == "f16sr":
                continue
            if eu <= 1e-3 and eb <= 1e-3:
                status = "converged"
                break
            if prev is not None and np.array_equal(gu, prev):
                status = "frozen"
                break
            prev = gu
            if s.step_count % 1_000_000 == 0:
                print(f"hartmann {storage}: {s.step_count} steps, err {eu:.2e}",
                      file=sys.stderr, flush=True)
        out[storage] = {"status": status, "steps": s.step_count,
                        "gpu_s": round(gpu_ms / 1e3, 2),
                        "us_per_step": round(1e3 * gpu_ms / s.step_count, 3),
                        "rel_l2_u": float(eu), "rel_l2_bx": float(eb)}
        if storage == "f16sr":
            late = [r for r in hist if r[0] > cap // 2]
            out[storage]["status"] = "fixed step budget"
            out[storage]["grid"] = f"{nx}x{h.ny}"
            out[storage]["second_half_rel_l2_u"] = [min(r[1] for r in late),
                                                    max(r[1] for r in late)]
            out[storage]["second_half_rel_l2_bx"] = [min(r[2] for r in late),
                                                     max(r[2] for r in late)]
            out[storage]["first_step_u_below_1e-2"] = next(
                (r[0] for r in hist if r[1] < 1e-2), None)
        s.close()
    print(json.dumps({
        "metric": "GPU time to steady state (Hartmann channel)",
        "value": out["f32"]["gpu_s"], "unit": "s", "n_gpus": 1,
        "higher_is_better": False, "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Hartmann channel 512x256, walls in y, G=1e-6, Ha=10, "
                               "tau_f=0.6, tau_m=0.55, from rest",
                   "criterion": "rel L2 of the x-averaged u_x and b_x vs the analytic profile <= 1e-3"},
        "storage": out,
        **({} if args.no_cpu_baseline else
           {"cpu_baseline_c2": cpu_baseline_c2(to_steady=out["f32"]["steps"])})}),
        flush=True)


def ot64_bench(torch, rrmhd, inputs, args):
    """Orszag-Tang on 64^2 (tau 0.56, 1000 steps): a launch-bound case
    (4,096 nodes sit in cache), reported as time per step."""
    u, b = inputs.orszag_tang(64, 0.05, 0.05)
    st = torch.cuda.current_stream()
    out, graphed = {}, {}
    for storage in ("f32", "f16"):
        for chunk, dst in ((0, out), (100, graphed)):
            s = rrmhd.Solver(64, 64, 0.56, 0.56, storage=storage)
            s.set_graph_chunk(chunk)
            s.init(torch.from_numpy(u).cuda(), torch.from_numpy(b).cuda())
            s.step(200)  # includes the graph capture
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            s.step(1000)
            e1.record(st)
            torch.cuda.synchronize()
            dst[storage] = round(e0.elapsed_time(e1), 3)
            s.close()
    print(json.dumps({
        "metric": "time per step (Orszag-Tang 64^2, launch-bound)",
        "value": out["f32"], "unit": "us/step", "n_gpus": 1, "steps": 1000,
        "higher_is_better": False, "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": {"workload": "Orszag-Tang 64x64, tau 0.56"},
        "us_per_step": out, "us_per_step_graph_chunk_100": graphed,
        **({} if args.no_cpu_baseline else {"cpu_baseline_c1_1000_steps": cpu_baseline_c1()})}),
        flush=True)


def turbulence3d_bench(torch, rrmhd, inputs, args):
    """The three-dimensional extension (D3Q27 fluid, D3Q7 magnetic lattice)
    on a periodic n^3 box of random-phase MHD turbulence (rms u = b = 0.04),
    tau 0.52, both storages; roofline against the algorithmic bytes, 48
    planes read and written per node."""
    n = args.n3d
    if args.ic3d == "abc":
        # analytic Arnold-Beltrami-Childress fields built on the device (for
        # boxes whose host-side FFT synthesis would take minutes): u with one
        # wavelength per side, b with two, each scaled to vector rms 0.04
        x = torch.arange(n, dtype=torch.float64, device="cuda") * (2 * math.pi / n)

        def abc(m):
            s1, c1 = torch.sin(m * x), torch.cos(m * x)
            f = torch.empty((3, n, n, n), dtype=torch.float64, device="cuda")
            f[0] = s1[:, None, None] + c1[None, :, None]   # sin z + cos y
            f[1] = s1[None, None, :] + c1[:, None, None]   # sin x + cos z
            f[2] = s1[None, :, None] + c1[None, None, :]   # sin y + cos x
            return f * (0.04 / math.sqrt(3.0))

        ud, bd = abc(1), abc(2)
        workload = f"ABC flow and field on a {n}^3 periodic box, rms 0.04"
    else:
        u, b = inputs.turbulence3d(n, 0.04)
        ud, bd = torch.from_numpy(u).cuda(), torch.from_numpy(b).cuda()
        del u, b
        workload = (f"decaying 3D MHD turbulence {n}^3 periodic, random-phase "
                    "solenoidal u and b, rms 0.04")
    st = torch.cuda.current_stream()
    nodes = n ** 3
    res = {}
    for storage in ("f32", "f16"):
        s = rrmhd.Solver3D(n, n, n, args.tau, args.tau, storage=storage, inplace=args.inplace)
        s.init(ud, bd)
        s.step(args.warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        s.step(args.steps)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        diag = s.diagnostics(allow_nonfinite=True)
        s.close()
        bpn = 2 * 48 * (4 if storage == "f32" else 2)
        gbs = bpn * nodes / ms / 1e6
        res[storage] = dict(mlups=round(nodes / ms / 1e3, 1), ms_per_step=round(ms, 4),
                            bytes_per_node=bpn, achieved_GBs=round(gbs, 1),
                            frac=round(gbs / PEAK_HBM_GBS, 4),
                            traffic=None if args.inplace else measured_traffic(storage, n, dims=3),
                            diagnostics_after=[v if math.isfinite(v) else None for v in diag])
    r = res["f32"]
    print(json.dumps({
        "metric": "MLUPS & % HBM roofline (fused 3D RR-MHD step, D3Q27 + D3Q7)",
        "value": r["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload, "nodes": nodes, "tau_f": args.tau, "tau_m": args.tau,
                   "population_buffers": 1 if args.inplace else 2,
                   "state_GB": round(nodes * 48 * 4 * (1 if args.inplace else 2) / 1e9, 1),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": r["achieved_GBs"], "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": r["frac"],
                     "traffic": None if args.inplace else measured_traffic("f32", n, dims=3)},
        "storages": res}), flush=True)


def closure_step_bench(torch, rrmhd, inputs, args):
    """The fused step with the closure network (BF16 MFMA inside the
    collision) against the plain step on the same grid, FP32 storage, a
    random network with a nonzero output layer."""
    import numpy as np
    n = args.n
    u, b = inputs.turbulence(n, 0.04)
    ud, bd = torch.from_numpy(u).cuda(), torch.from_numpy(b).cuda()
    del u, b
    g = np.random.default_rng(0)
    p = np.zeros(4931, dtype=np.float32)
    p[0:512] = g.standard_normal(512) / np.sqrt(8)
    p[576:4672] = g.standard_normal(4096) / np.sqrt(64)
    p[4736:4928] = g.standard_normal(192) / np.sqrt(64)
    norm = np.concatenate([[1.0, 0, 0, 0, 0, 0, 0, 0], [0.01, 0.04, 0.04, 0.04, 0.04,
                                                        1e-3, 1e-3, 1e-3], [1e-5] * 3])
    pd = torch.from_numpy(p).cuda()
    nd = torch.from_numpy(norm.astype(np.float32)).cuda()
    st = torch.cuda.current_stream()
    res = {}
    for mode in ("plain", "closure"):
        s = rrmhd.Solver(n, n, args.tau, args.tau)
        s.init(ud, bd)
        if mode == "closure":
            s.closure_set(pd, nd)
            s.closure_enable(True)
        s.step(args.warmup)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        s.step(args.steps)
        e1.record(st)
        torch.cuda.synchronize()
        res[mode] = e0.elapsed_time(e1) / args.steps
        s.close()
    ms = res["closure"]
    nodes = n * n
    gbs = 152 * nodes / ms / 1e6
    # the network's algorithmic work: 2 (8 x 64 + 64 x 64 + 64 x 3) FLOP per node
    mfma_tf = 9600 * nodes / ms / 1e9
    print(json.dumps({
        "metric": "MLUPS (fused RR-MHD step with the closure network)",
        "value": round(nodes / ms / 1e3, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+bf16", "data": "synthetic",
        "config": {"workload": f"decaying 2D MHD turbulence {n}x{n} periodic, "
                               "random closure network (8-64-64-3 GELU)",
                   "nodes": nodes, "tau": args.tau},
        "plain_ms_per_step": round(res["plain"], 4),
        "closure_over_plain": round(ms / res["plain"], 3),
        "hbm_GBs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4),
        "mfma_bf16_TFLOPs": round(mfma_tf, 2),
        "mfma_frac": round(mfma_tf / 2500.0, 5)}), flush=True)


def closure_bench(args):
    """Learned-closure protocol: coarse 512^2 (plain and with the trained
    network) against the 4x4-filtered 2048^2 run."""
    from paper_2602_14667_amd import closure_pipeline as cp
    if args.closure_scale == "full":
        kw = dict(n_f=2048, factor=4, tau_f=0.56, fine_steps=64000, snaps=8,
                  train_seeds=range(16), val_seeds=range(16, 20),
                  test_seeds=range(20, 24), train_steps=3000, onestep_steps=2000,
                  batch=65536)
    else:
        kw = dict(n_f=1024, factor=4, tau_f=0.56, fine_steps=16000, snaps=4,
                  train_seeds=range(4), val_seeds=[5], test_seeds=[20],
                  train_steps=1000, onestep_steps=600, batch=65536)
    res = cp.pipeline(log=lambda m: print(m, file=sys.stderr, flush=True), **kw)
    tests = res["tests"]
    worst = {side: max(t[side]["eps_spec"] for t in tests) for side in ("plain", "closure")}
    e_err = {side: max(max(t[side]["ekin_err"], t[side]["emag_err"]) for t in tests)
             for side in ("plain", "closure")}
    ms = {k: sum(t[k] for t in tests) / len(tests)
          for k in ("fine_gpu_ms", "plain_gpu_ms", "closure_gpu_ms")}

    def within_until(rows):
        # last coarse step up to which every comparison time meets the bar
        last = 0
        for r in rows:
            if r["eps_spec"] <= 0.05 and abs(r["ekin_err"]) <= 0.05 and abs(r["emag_err"]) <= 0.05:
                last = r["step"]
            else:
                break
        return last

    horizon = {side: {str(t["seed"]): within_until(t[side + "_rows"]) for t in tests}
               for side in ("plain", "closure")}
    eps_t = {side: {str(t["seed"]): [round(r["eps_spec"], 4) for r in t[side + "_rows"]]
                    for t in tests} for side in ("plain", "closure")}
    # the best velocity a fluid-only closure could give the coarse run: the
    # filtered fine velocity imposed after every coarse step
    n_c = kw["n_f"] // kw["factor"]
    cks = [r["step"] for r in tests[0]["plain_rows"]]
    bound = {}
    for t in tests:
        run, ref, parts = cp.velocity_bound_run(kw["n_f"], kw["tau_f"], kw["factor"], t["seed"],
                                                cks)
        rows, w = cp.judge(run, ref, n_c // 4)
        bound[str(t["seed"])] = {"eps_spec": [round(r["eps_spec"], 4) for r in rows],
                                 "magnetic": [round(parts[c]["magnetic"], 4) for c in cks],
                                 "kinetic_max": max(parts[c]["kinetic"] for c in cks),
                                 "worst": round(w["eps_spec"], 4)}
    print(json.dumps({
        "metric": "closure-vs-fine wall time at 5% spectral error",
        "value": round(ms["closure_gpu_ms"] / 1e3, 3), "unit": "s (GPU, coarse+closure run)",
        "higher_is_better": False, "n_gpus": 1, "vs_baseline": None,
        "dtype": "f32+bf16", "data": "synthetic",
        "config": {"workload": "decaying 2D MHD turbulence, coarse "
                               f"{kw['n_f'] // kw['factor']}^2 vs fine {kw['n_f']}^2",
                   **{k: (list(v) if isinstance(v, range) else v) for k, v in kw.items()}},
        "eps_spec_worst": worst, "energy_err_worst": e_err,
        "within_5pct": {side: all(t[side]["within_5pct"] for t in tests)
                        for side in ("plain", "closure")},
        "gpu_s": {k: round(v / 1e3, 3) for k, v in ms.items()},
        "fine_over_coarse_gpu_time": {"plain": round(ms["fine_gpu_ms"] / ms["plain_gpu_ms"], 1),
                                      "closure": round(ms["fine_gpu_ms"] / ms["closure_gpu_ms"], 1)},
        "within_5pct_until_coarse_step": horizon,
        "comparison_steps": [r["step"] for r in tests[0]["plain_rows"]],
        "eps_spec_per_time": eps_t,
        "train_s": round(res["train_s"], 2), "data_s": round(res["data_s"], 2),
        "train_loss_first_last": [res["train_loss"][0], res["train_loss"][-1]],
        "onestep_objective": {"train": res["onestep_objective"],
                              "validation": res["onestep_objective_val"]},
        "alpha": res["alpha"], "calibration": res["calibration"],
        "fallbacks": [t["fallback_at"] for t in tests],
        "best_velocity_bound": bound}), flush=True)


def time_turbulence_leg(torch, rrmhd, args, fields, storage):
    """Warm-up, then args.steps fused steps of the turbulence workload timed with
    HIP events on the handle's stream, then diagnostics (timed separately)."""
    n = args.n
    ud, bd = fields
    s = rrmhd.Solver(n, n, args.tau, args.tau, storage=storage,
                     equilibrium=args.equilibrium, inplace=args.inplace)
    launch = ("library default (row-interleaved planes, eight neighbouring tiles per "
              "XCD, NT stores; f32: 128x2 threads, two nodes per thread in 64-bit words; "
              "f16: 128x1 threads, four nodes per thread in 64-bit words)")
    if storage == "f16sr":
        launch = ("library default (row-interleaved planes, eight neighbouring tiles per XCD, "
                  "NT stores, 128x1 threads, one node per thread)")
    if args.equilibrium != "algorithm":
        launch = "library default block shape, one node per thread, NT stores"
    if args.inplace and storage == "f16sr":
        launch = ("library default for one buffer (row-interleaved planes, XCD-local order, "
                  "NT stores, 128x1 threads, one node per thread); steps alternate pull+push "
                  "and own-slot forms")
    elif args.inplace:
        launch = ("library default for one buffer (row-interleaved planes, XCD-local order, "
                  "NT stores; f32: 128x1 threads, one node per thread; f16: 64x2 threads, two "
                  "nodes per thread in 32-bit words); steps alternate pull+push and own-slot "
                  "forms")
    s.init(ud, bd)
    s.step(args.warmup)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    s.step(args.steps)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_launches = e0.elapsed_time(e1)
    ek, em, dv = s.diagnostics(allow_nonfinite=True)
    # diagnostics (every K steps in a run, not per step): timed separately
    d0 = torch.cuda.Event(enable_timing=True)
    d1 = torch.cuda.Event(enable_timing=True)
    d0.record(st)
    for _ in range(5):
        s.diagnostics(allow_nonfinite=True)
    d1.record(st)
    torch.cuda.synchronize()
    diag_ms = d0.elapsed_time(d1) / 5
    s.close()
    nodes = n * n
    sec = ms_launches / 1e3
    per_launch = sec / args.steps
    achieved = BYTES_PER_NODE[storage] * nodes / per_launch / 1e9
    # the stored counter readings belong to the method's own step kernel
    traffic = (measured_traffic(storage, n)
               if args.equilibrium == "algorithm" and not args.inplace else None)
    return {"value": round(nodes * args.steps / sec / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(1e3 * per_launch, 4), "launch": launch,
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                         "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic},
            "wall_s_timed": round(wall, 4),
            "diagnostics_after": {k: (v if math.isfinite(v) else None) for k, v in
                                  (("E_kin", ek), ("E_mag", em), ("max_div_b", dv))},
            "diagnostics_ms_per_call": round(diag_ms, 4)}


def load_config(name):
    """A configuration file: `name` as a path, else
    paper_2602_14667_amd/configs/<name>.json."""
    path = name if os.path.exists(name) else os.path.join(
        ROOT, "paper_2602_14667_amd", "configs", f"{name}.json")
    with open(path) as fh:
        return json.load(fh)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 10000 for the turbulence workload, as "
                         "the 8192^2 configuration specifies; 2000 for the ensemble; "
                         "20 for --mode copy/sweep; 200 for closure-step)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps before timing (default 100; 5 for copy/sweep)")
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--n3d", type=int, default=256, help="box side of --workload turbulence3d")
    ap.add_argument("--ic3d", choices=["turbulence", "abc"], default="turbulence",
                    help="initial field of --workload turbulence3d")
    ap.add_argument("--tau", type=float, default=0.52)
    ap.add_argument("--storage", choices=["f32", "f16", "f16sr"], default="f32",
                    help="f16sr: FP16 with stochastically rounded step stores (variant)")
    ap.add_argument("--inplace", action="store_true",
                    help="single-buffer streaming (one population buffer)")
    ap.add_argument("--equilibrium", choices=["algorithm", "full_maxwell"],
                    default="algorithm",
                    help="fluid equilibrium of the turbulence step: the method's "
                         "(default) or the ablation with the u.M cross terms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f16-leg", action="store_true",
                    help="turbulence workload with f32 storage: skip the FP16-storage "
                         "leg timed after it")
    ap.add_argument("--no-ensemble-leg", action="store_true",
                    help="turbulence workload: skip the 256-domain ensemble leg "
                         "(default launch, 1000 steps) timed after it")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batch workload: keep the library's default launch "
                         "(one workgroup per 32x8 tile) instead of autotuning")
    ap.add_argument("--mode", choices=["step", "copy", "sweep"], default="step",
                    help="copy: time the plain device-copy reference; sweep: "
                         "time launch shapes, XCD block orders and plane gaps")
    ap.add_argument("--copy-bytes", type=int, default=4 << 30)
    ap.add_argument("--workload", choices=["turbulence", "batch", "closure",
                                           "closure-step", "hartmann", "ot64",
                                           "turbulence3d"],
                    default="turbulence",
                    help="batch: the 256-domain ensemble; closure: the "
                         "learned-closure protocol (coarse vs fine spectra); "
                         "closure-step: the fused step with the closure "
                         "network against the plain step (--n grid); hartmann: "
                         "time to steady state of the wall-bounded channel; "
                         "ot64: time per step of the 64^2 Orszag-Tang case")
    ap.add_argument("--closure-scale", choices=["full", "reduced"], default="full")
    ap.add_argument("--config", default=None,
                    help="c1..c5 or a path: a JSON file whose 'bench' block sets "
                         "defaults for these flags (flags given here still win) and "
                         "whose 'env' block sets RRMHD_* variables not already set")
    pre, _ = ap.parse_known_args()
    if pre.config:
        cfg = load_config(pre.config)
        unknown = set(cfg.get("bench", {})) - {a.dest for a in ap._actions}
        if unknown:
            ap.error(f"config {pre.config}: unknown keys {sorted(unknown)}")
        ap.set_defaults(**cfg.get("bench", {}))
        for k, v in cfg.get("env", {}).items():
            os.environ.setdefault(k, str(v))
    args = ap.parse_args()
    if args.steps is None:
        args.steps = (20 if args.mode != "step" else
                      {"batch": 2000, "closure-step": 200,
                       "turbulence3d": 1000}.get(args.workload, 10000))
    if args.warmup is None:
        args.warmup = 5 if args.mode != "step" else 100
    if args.gpus != 1:
        print(f"bench.py: this implementation runs on one GPU only (asked for "
              f"--gpus {args.gpus}); the domain-decomposed multi-GPU path is "
              "a design, not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2602_14667_amd import inputs, rrmhd

    torch.cuda.set_device(0)
    if args.mode == "copy":
        copy_reference(torch, rrmhd, args)
        return
    if args.mode == "sweep":
        launch_sweep(torch, rrmhd, inputs, args)
        return
    if args.workload == "batch":
        batch_bench(torch, rrmhd, inputs, args)
        return
    if args.workload == "closure":
        closure_bench(args)
        return
    if args.workload == "closure-step":
        closure_step_bench(torch, rrmhd, inputs, args)
        return
    if args.workload == "hartmann":
        hartmann_bench(torch, rrmhd, inputs, args)
        return
    if args.workload == "ot64":
        ot64_bench(torch, rrmhd, inputs, args)
        return
    if args.workload == "turbulence3d":
        turbulence3d_bench(torch, rrmhd, inputs, args)
        return
    n = args.n
    u, b = inputs.turbulence(n, 0.04)
    fields = (torch.from_numpy(u).cuda(), torch.from_numpy(b).cuda())
    del u, b
    leg = time_turbulence_leg(torch, rrmhd, args, fields, args.storage)
    out = {
        "metric": "MLUPS & % HBM roofline (fused RR-MHD step)",
        "value": leg["value"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"decaying 2D MHD turbulence {n}x{n} periodic, "
                               "random-phase psi/A, rms u=b=0.04",
                   "nodes": n * n, "tau_f": args.tau, "tau_m": args.tau,
                   "storage": f"{args.storage}-shifted (f - w)",
                   "equilibrium": args.equilibrium,
                   "population_buffers": 1 if args.inplace else 2,
                   "launch": leg["launch"],
                   "parallelism": "single GPU"},
        "roofline": leg["roofline"],
        "wall_s_timed": leg["wall_s_timed"],
        "diagnostics_after": leg["diagnostics_after"],
        "diagnostics_ms_per_call": leg["diagnostics_ms_per_call"],
        "kernel_hash": kernel_hash(),
        "env": environment(torch),
    }
    # the FP16-offset storage of the same workload, timed the same way in the
    # same run (the precision form the configuration compares against FP32)
    if args.storage == "f32" and not args.no_f16_leg:
        f16 = time_turbulence_leg(torch, rrmhd, args, fields, "f16")
        out["storage_f16"] = {k: f16[k] for k in ("value", "unit", "ms_per_step", "roofline",
                                                   "launch", "diagnostics_after")}
    del fields
    # the 256-domain ensemble with the library's default launch, timed in the
    # same run (its own configuration, reported beside the headline step)
    if not args.no_ensemble_leg:
        ens = time_batch_leg(torch, rrmhd, inputs, 1000, False, False)
        out["ensemble"] = {k: ens[k] for k in ("value", "unit", "steps", "ms_per_step",
                                               "roofline", "config")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
