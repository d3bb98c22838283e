"""Summarise rocprofv3 CSV output of the step kernel into profiles/.

Usage: python -m paper_2602_14667_amd.profsum PROF_DIR OUT_DIR N

PROF_DIR holds the rocprofv3 output directories written by
  rocprofv3 --kernel-trace --stats --output-format csv -d PROF_DIR/stats_{f32,f16,copy} -o run -- python3 bench.py ...
  rocprofv3 --pmc {FETCH_SIZE,WRITE_SIZE} --output-format csv -d PROF_DIR/pmc_<ctr>_{f32,f16,copy} -o run -- python3 bench.py ...
Counter values (KiB per dispatch) are calibrated against the plain copy
kernel of known size: factor = true bytes / counted bytes for that kernel.

Single-buffer (in-place) steps, per phase, from the same copy calibration:
  rocprofv3 --kernel-trace --stats ... -d PROF_DIR/ip_stats_{f32,f16} ... bench.py --inplace ...
  rocprofv3 --pmc <ctr> ... -d PROF_DIR/ip_pmc_<ctr>_{f32,f16} ... bench.py --inplace ...
  python -m paper_2602_14667_amd.profsum inplace PROF_DIR OUT_DIR N

Three-dimensional step (both storages in one bench run), same calibration:
  rocprofv3 --kernel-trace --stats ... -d PROF_DIR/s3_stats ... bench.py --workload turbulence3d ...
  rocprofv3 --pmc <ctr> ... -d PROF_DIR/s3_pmc_<ctr> ... bench.py --workload turbulence3d ...
  python -m paper_2602_14667_amd.profsum step3d PROF_DIR OUT_DIR N

Batched ensemble step (256 domains), same calibration:
  rocprofv3 --kernel-trace --stats ... -d PROF_DIR/batch_stats ... bench.py --workload batch --no-autotune ...
  rocprofv3 --pmc <ctr> ... -d PROF_DIR/batch_pmc_<ctr> ... bench.py --workload batch --no-autotune ...
  python -m paper_2602_14667_amd.profsum batch PROF_DIR OUT_DIR

Second form, kernel-trace statistics of any workload:
  python -m paper_2602_14667_amd.profsum stats STATS_DIR OUT.md KERNEL BYTES TITLE COMMAND [LAST]
writes the per-kernel table and, for the kernel whose name contains KERNEL,
the average launch time and its algorithmic rate (BYTES per launch); with
LAST, also the average over its last LAST dispatches (the timed region of a
bench run, after any autotuning launches).
"""
import csv
import json
import os
import re
import sys

from . import kernel3d_hash, kernel_hash

COPY_BYTES = 4 << 30  # bench.py --mode copy default


def _rows(path):
    with open(path) as fh:
        return list(csv.DictReader(fh))


def kernel_stats(d):
    out = {}
    for r in _rows(os.path.join(d, "run_kernel_stats.csv")):
        out[r["Name"]] = dict(calls=int(r["Calls"]), avg_ns=float(r["AverageNs"]),
                              min_ns=float(r["MinNs"]), max_ns=float(r["MaxNs"]))
    return out


def counter_mean(d, match):
    vals = [float(r["Counter_Value"]) for r in _rows(os.path.join(d, "run_counter_collection.csv"))
            if match in r["Kernel_Name"]]
    return sum(vals) / len(vals) if vals else None


def main(prof, out, n):
    n = int(n)
    nodes = n * n
    fac = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        kib = counter_mean(os.path.join(prof, f"pmc_{ctr}_copy"), "k_copy16")
        fac[ctr] = COPY_BYTES / (kib * 1024.0)
    copy = kernel_stats(os.path.join(prof, "stats_copy"))
    copy_ns = [v for k, v in copy.items() if "k_copy16" in k][0]["avg_ns"]
    for st, bpn in (("f32", 152), ("f16", 76)):
        stats = kernel_stats(os.path.join(prof, f"stats_{st}"))
        name = [k for k in stats if "k_step" in k][0]
        avg = stats[name]["avg_ns"]
        rd = counter_mean(os.path.join(prof, f"pmc_FETCH_SIZE_{st}"), "k_step") * 1024 * fac["FETCH_SIZE"]
        wr = counter_mean(os.path.join(prof, f"pmc_WRITE_SIZE_{st}"), "k_step") * 1024 * fac["WRITE_SIZE"]
        alg = bpn * nodes
        traffic = {"kernel": name, "kernel_hash": kernel_hash(), "n": n, "storage": st,
                   "bytes_per_launch": rd + wr, "read_bytes": rd, "write_bytes": wr,
                   "algorithmic_bytes": alg, "fetch_factor": fac["FETCH_SIZE"],
                   "write_factor": fac["WRITE_SIZE"]}
        with open(os.path.join(out, f"traffic_step_{st}_{n}.json"), "w") as fh:
            json.dump(traffic, fh, indent=1)
        lines = [
            f"# step kernel, {st.upper()} storage, turbulence {n}x{n}",
            "",
            f"Kernel: `{name}`  (source hash {kernel_hash()})",
            "",
            "Commands (from the repository root, on the MI355X host):",
            "```",
            f"rocprofv3 --kernel-trace --stats --output-format csv -d {prof}/stats_{st} -o run -- python3 bench.py --storage {st} --steps 50 --warmup 5 --no-cpu-baseline --no-f16-leg --no-ensemble-leg",
            f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {prof}/pmc_FETCH_SIZE_{st} -o run -- python3 bench.py --storage {st} --steps 5 --warmup 1 --no-cpu-baseline --no-f16-leg --no-ensemble-leg",
            f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {prof}/pmc_WRITE_SIZE_{st} -o run -- python3 bench.py --storage {st} --steps 5 --warmup 1 --no-cpu-baseline --no-f16-leg --no-ensemble-leg",
            f"rocprofv3 --kernel-trace --stats --output-format csv -d {prof}/stats_copy -o run -- python3 bench.py --mode copy --steps 20",
            f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {prof}/pmc_FETCH_SIZE_copy -o run -- python3 bench.py --mode copy --steps 5 --warmup 1",
            f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {prof}/pmc_WRITE_SIZE_copy -o run -- python3 bench.py --mode copy --steps 5 --warmup 1",
            f"python -m paper_2602_14667_amd.profsum {prof} profiles {n}",
            "```",
            "",
            "| kernel | calls | avg ns | min ns | max ns |",
            "|---|---|---|---|---|",
        ]
        for k, v in sorted(stats.items(), key=lambda kv: -kv[1]["avg_ns"] * kv[1]["calls"]):
            lines.append(f"| `{k[:90]}` | {v['calls']} | {v['avg_ns']:.0f} | {v['min_ns']:.0f} | {v['max_ns']:.0f} |")
        lines += [
            "",
            f"* nodes per launch: {nodes}; algorithmic bytes per launch: {alg / 1e9:.3f} GB ({bpn} B/node)",
            f"* average launch: {avg / 1e3:.1f} us -> {nodes / avg * 1e3:.0f} MLUPS, "
            f"{alg / avg:.1f} GB/s algorithmic = {alg / avg / 8000 * 100:.1f} % of 8 TB/s",
            f"* HBM traffic per launch (PMC, calibrated): read {rd / 1e9:.3f} GB "
            f"({rd / (alg / 2):.3f}x algorithmic), write {wr / 1e9:.3f} GB ({wr / (alg / 2):.3f}x); "
            f"{(rd + wr) / avg:.1f} GB/s actual",
            f"* calibration: plain copy of {COPY_BYTES} B reads as FETCH_SIZE x {fac['FETCH_SIZE']:.4f}, "
            f"WRITE_SIZE x {fac['WRITE_SIZE']:.4f}; copy kernel {2 * COPY_BYTES / copy_ns:.1f} GB/s",
        ]
        # the diagnostics pass (energies, max |div b|) of the same runs: it
        # reads the state once, half the step's bytes per node
        diag = [k for k in stats if "k_diag_tile" in k]
        if diag:
            davg = stats[diag[0]]["avg_ns"]
            dalg = alg / 2
            drd = counter_mean(os.path.join(prof, f"pmc_FETCH_SIZE_{st}"), "k_diag_tile")
            line = (f"* diagnostics pass (`k_diag_tile`, every K steps; reads the state once, "
                    f"{bpn // 2} B/node): average {davg / 1e3:.1f} us -> {dalg / davg:.1f} GB/s "
                    f"algorithmic = {dalg / davg / 8000 * 100:.1f} % of 8 TB/s")
            if drd is not None:
                drd *= 1024 * fac["FETCH_SIZE"]
                line += (f"; HBM reads (PMC, calibrated) {drd / 1e9:.3f} GB "
                         f"({drd / dalg:.3f}x algorithmic, the tile rings included)")
            lines.append(line)
        with open(os.path.join(out, f"step_{st}_{n}.md"), "w") as fh:
            fh.write("\n".join(lines) + "\n")
    print("ok")


def _calibration(prof):
    fac = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        kib = counter_mean(os.path.join(prof, f"pmc_{ctr}_copy"), "k_copy16")
        fac[ctr] = COPY_BYTES / (kib * 1024.0)
    return fac


def inplace_summary(prof, out, n):
    """Per-phase time and calibrated HBM traffic of the single-buffer step."""
    n = int(n)
    nodes = n * n
    fac = _calibration(prof)
    for st, bpn in (("f32", 152), ("f16", 76)):
        stats = kernel_stats(os.path.join(prof, f"ip_stats_{st}"))
        alg = bpn * nodes
        lines = [
            f"# single-buffer (in-place) step kernels, {st.upper()} storage, turbulence {n}x{n}",
            "",
            f"Source hash {kernel_hash()}. The two phases alternate; one step of either moves "
            f"{alg / 1e9:.3f} GB algorithmically ({bpn} B/node).",
            "",
            "Commands (from the repository root, on the MI355X host; calibration runs as for the "
            "two-buffer step summaries):",
            "```",
            f"rocprofv3 --kernel-trace --stats --output-format csv -d {prof}/ip_stats_{st} -o run -- python3 bench.py --storage {st} --inplace --steps 50 --warmup 6 --no-cpu-baseline --no-f16-leg --no-ensemble-leg",
            f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {prof}/ip_pmc_FETCH_SIZE_{st} -o run -- python3 bench.py --storage {st} --inplace --steps 6 --warmup 2 --no-cpu-baseline --no-f16-leg --no-ensemble-leg",
            f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {prof}/ip_pmc_WRITE_SIZE_{st} -o run -- python3 bench.py --storage {st} --inplace --steps 6 --warmup 2 --no-cpu-baseline --no-f16-leg --no-ensemble-leg",
            f"python -m paper_2602_14667_amd.profsum inplace {prof} profiles {n}",
            "```",
            "",
            "| kernel | calls | avg ns | min ns | max ns |",
            "|---|---|---|---|---|",
        ]
        for k, v in sorted(stats.items(), key=lambda kv: -kv[1]["avg_ns"] * kv[1]["calls"]):
            lines.append(f"| `{k[:100]}` | {v['calls']} | {v['avg_ns']:.0f} | {v['min_ns']:.0f} "
                         f"| {v['max_ns']:.0f} |")
        lines.append("")
        tot = 0.0
        for ph in (0, 1):
            # k_step_inplace<codec, walls, forced, phase, nt, row mode> or
            # k_step_inplace_multi<codec, nodes per thread, forced, phase, row mode>
            pat = re.compile(r"k_step_inplace<[^,<>]+, \w+, \w+, %d,|"
                             r"k_step_inplace_multi<[^,<>]+, \d+, \w+, %d," % (ph, ph))
            name = [k for k in stats if pat.search(k)][0]
            avg = stats[name]["avg_ns"]
            tot += avg
            rd = counter_mean(os.path.join(prof, f"ip_pmc_FETCH_SIZE_{st}"), name) * 1024 * fac["FETCH_SIZE"]
            wr = counter_mean(os.path.join(prof, f"ip_pmc_WRITE_SIZE_{st}"), name) * 1024 * fac["WRITE_SIZE"]
            lines.append(f"* phase {ph}: average launch {avg / 1e3:.1f} us -> {alg / avg:.1f} GB/s "
                         f"algorithmic = {alg / avg / 8000 * 100:.1f} % of 8 TB/s; HBM traffic (PMC, "
                         f"calibrated) read {rd / 1e9:.3f} GB ({rd / (alg / 2):.3f}x), write "
                         f"{wr / 1e9:.3f} GB ({wr / (alg / 2):.3f}x)")
        avg2 = tot / 2
        lines.append(f"* both phases: {avg2 / 1e3:.1f} us per step -> {nodes / avg2 * 1e3:.0f} MLUPS, "
                     f"{alg / avg2 / 8000 * 100:.1f} % of 8 TB/s")
        with open(os.path.join(out, f"step_inplace_{st}_{n}.md"), "w") as fh:
            fh.write("\n".join(lines) + "\n")
    print("ok")


def step3d_summary(prof, out, n):
    """Time and calibrated HBM traffic of the 3D step kernel, per storage."""
    n = int(n)
    nodes = n ** 3
    fac = _calibration(prof)
    stats = kernel_stats(os.path.join(prof, "s3_stats"))
    cmd = f"python3 bench.py --workload turbulence3d --n3d {n}"
    for st, codec, bpn in (("f32", "CodecF32>", 384), ("f16", "CodecF16U>", 192)):
        name = [k for k in stats if "k_step3<" in k and codec in k][0]
        avg = stats[name]["avg_ns"]
        rd = counter_mean(os.path.join(prof, "s3_pmc_FETCH_SIZE"), name) * 1024 * fac["FETCH_SIZE"]
        wr = counter_mean(os.path.join(prof, "s3_pmc_WRITE_SIZE"), name) * 1024 * fac["WRITE_SIZE"]
        alg = bpn * nodes
        traffic = {"kernel": name, "kernel_hash": kernel3d_hash(), "n": n, "storage": st,
                   "bytes_per_launch": rd + wr, "read_bytes": rd, "write_bytes": wr,
                   "algorithmic_bytes": alg, "fetch_factor": fac["FETCH_SIZE"],
                   "write_factor": fac["WRITE_SIZE"]}
        with open(os.path.join(out, f"traffic_step3d_{st}_{n}.json"), "w") as fh:
            json.dump(traffic, fh, indent=1)
        lines = [
            f"# 3D step kernel (D3Q27 + D3Q7), {st.upper()} storage, turbulence {n}^3",
            "",
            f"Kernel: `{name}`  (source hash {kernel3d_hash()}); both storages come from the same runs.",
            "",
            "Commands (from the repository root, on the MI355X host; the copy calibration runs as "
            "for the two-dimensional step summaries):",
            "```",
            f"rocprofv3 --kernel-trace --stats --output-format csv -d {prof}/s3_stats -o run -- {cmd} --steps 50 --warmup 5",
            f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {prof}/s3_pmc_FETCH_SIZE -o run -- {cmd} --steps 5 --warmup 1",
            f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {prof}/s3_pmc_WRITE_SIZE -o run -- {cmd} --steps 5 --warmup 1",
            f"python -m paper_2602_14667_amd.profsum step3d {prof} profiles {n}",
            "```",
            "",
            "| kernel | calls | avg ns | min ns | max ns |",
            "|---|---|---|---|---|",
        ]
        for k, v in sorted(stats.items(), key=lambda kv: -kv[1]["avg_ns"] * kv[1]["calls"]):
            lines.append(f"| `{k[:90]}` | {v['calls']} | {v['avg_ns']:.0f} | {v['min_ns']:.0f} "
                         f"| {v['max_ns']:.0f} |")
        lines += [
            "",
            f"* nodes per launch: {nodes}; algorithmic bytes per launch: {alg / 1e9:.3f} GB ({bpn} B/node)",
            f"* average launch: {avg / 1e3:.1f} us -> {nodes / avg * 1e3:.0f} MLUPS, "
            f"{alg / avg:.1f} GB/s algorithmic = {alg / avg / 8000 * 100:.1f} % of 8 TB/s",
            f"* HBM traffic per launch (PMC, calibrated): read {rd / 1e9:.3f} GB "
            f"({rd / (alg / 2):.3f}x algorithmic), write {wr / 1e9:.3f} GB ({wr / (alg / 2):.3f}x); "
            f"{(rd + wr) / avg:.1f} GB/s actual",
            f"* calibration: FETCH_SIZE x {fac['FETCH_SIZE']:.4f}, WRITE_SIZE x {fac['WRITE_SIZE']:.4f} "
            f"(plain copy of {COPY_BYTES} B)",
        ]
        with open(os.path.join(out, f"step3d_{st}_{n}.md"), "w") as fh:
            fh.write("\n".join(lines) + "\n")
    print("ok")


def counter_mean_named(d, match, counter):
    """Mean over dispatches of one named counter for kernels matching `match`:
    per dispatch, the sum over the counter's dimensions (the maximum for the
    GPU-wide busy counter GRBM_GUI_ACTIVE, as rocprof's derived metrics take
    it)."""
    per = {}
    use_max = counter.startswith("GRBM_")
    for r in _rows(os.path.join(d, "run_counter_collection.csv")):
        if match in r["Kernel_Name"] and r["Counter_Name"] == counter:
            key = r.get("Dispatch_Id") or r.get("Correlation_Id") or len(per)
            v = float(r["Counter_Value"])
            per[key] = max(per.get(key, 0.0), v) if use_max else per.get(key, 0.0) + v
    return sum(per.values()) / len(per) if per else None


def closure_summary(prof, out, n):
    """The fused closure step against the plain step at n^2: launch times,
    calibrated HBM traffic and the shader counters that locate its bound."""
    n = int(n)
    nodes = n * n
    fac = _calibration(prof)
    stats = kernel_stats(os.path.join(prof, "cl_stats"))
    cl = [k for k in stats if "k_step_closure" in k][0]
    # the plain step: one node per thread or the multi-node form
    pl = [k for k in stats if "k_step<" in k or "k_step_multi<" in k][0]
    m_pl = "k_step_multi<" if "k_step_multi<" in pl else "k_step<"
    t_cl, t_pl = stats[cl]["avg_ns"], stats[pl]["avg_ns"]
    rd = counter_mean(os.path.join(prof, "cl_pmc_FETCH_SIZE"), "k_step_closure") * 1024 * fac["FETCH_SIZE"]
    wr = counter_mean(os.path.join(prof, "cl_pmc_WRITE_SIZE"), "k_step_closure") * 1024 * fac["WRITE_SIZE"]
    sq = os.path.join(prof, "cl_pmc_sq")
    ctr = {}
    for kern, tag in ((cl, "closure"), (pl, "plain")):
        m = "k_step_closure" if tag == "closure" else m_pl
        ctr[tag] = {c: counter_mean_named(sq, m, c) for c in (
            "SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_MFMA", "SQ_INSTS_LDS", "SQ_ACTIVE_INST_VALU",
            "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_LDS_IDX_ACTIVE", "SQ_LDS_BANK_CONFLICT",
            "GRBM_GUI_ACTIVE")}
    cus, simds = 256, 1024
    alg = 152 * nodes
    cmd = f"python3 bench.py --workload closure-step --n {n}"
    lines = [
        f"# fused step with the closure network vs the plain step, FP32 storage, turbulence {n}x{n}",
        "",
        f"Kernels: `{cl[:100]}` and `{pl[:100]}`",
        "",
        "Commands (from the repository root, on the MI355X host; the copy calibration runs as "
        "for the two-dimensional step summaries):",
        "```",
        f"rocprofv3 --kernel-trace --stats --output-format csv -d {prof}/cl_stats -o run -- {cmd} --steps 50 --warmup 5",
        f"rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_MFMA SQ_INSTS_LDS SQ_ACTIVE_INST_VALU "
        f"SQ_VALU_MFMA_BUSY_CYCLES SQ_LDS_IDX_ACTIVE SQ_LDS_BANK_CONFLICT GRBM_GUI_ACTIVE "
        f"--output-format csv -d {prof}/cl_pmc_sq -o run -- {cmd} --steps 3 --warmup 1",
        f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {prof}/cl_pmc_FETCH_SIZE -o run -- {cmd} --steps 3 --warmup 1",
        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {prof}/cl_pmc_WRITE_SIZE -o run -- {cmd} --steps 3 --warmup 1",
        f"python -m paper_2602_14667_amd.profsum closure {prof} profiles {n}",
        "```",
        "",
        "| kernel | calls | avg ns | min ns | max ns |",
        "|---|---|---|---|---|",
    ]
    for k, v in sorted(stats.items(), key=lambda kv: -kv[1]["avg_ns"] * kv[1]["calls"]):
        lines.append(f"| `{k[:90]}` | {v['calls']} | {v['avg_ns']:.0f} | {v['min_ns']:.0f} "
                     f"| {v['max_ns']:.0f} |")
    lines += [
        "",
        f"* closure step: average launch {t_cl / 1e3:.1f} us = {t_cl / t_pl:.2f}x the plain step "
        f"({t_pl / 1e3:.1f} us); {nodes / t_cl * 1e3:.0f} MLUPS; {alg / t_cl:.1f} GB/s algorithmic "
        f"= {alg / t_cl / 8000 * 100:.1f} % of 8 TB/s; network work 9600 FLOP/node -> "
        f"{9600 * nodes / t_cl / 1e3:.1f} TFLOP/s = {9600 * nodes / t_cl / 1e3 / 2500 * 100:.1f} % of "
        "the 2.5 PFLOP/s BF16 peak",
        f"* HBM traffic per closure launch (PMC, calibrated): read {rd / 1e9:.3f} GB "
        f"({rd / (alg / 2):.3f}x algorithmic), write {wr / 1e9:.3f} GB ({wr / (alg / 2):.3f}x)",
        "",
        "| counter (per launch) | closure step | plain step |",
        "|---|---|---|",
    ]
    for c in ctr["closure"]:
        a, b = ctr["closure"][c], ctr["plain"][c]
        lines.append(f"| {c} | {a:.4g} | {b:.4g} |" if a is not None and b is not None
                     else f"| {c} | {a} | {b} |")
    lines.append("")
    # busy fractions against the kernel's own duration at the 2.4 GHz peak
    # clock: VALU quad-cycles x 4 and MFMA busy cycles over 1024 SIMDs, LDS
    # active cycles over 256 CUs
    clk = 2.4e9
    for tag, t in (("closure", t_cl), ("plain", t_pl)):
        c = ctr[tag]
        if None in c.values():
            continue
        per = 64 / nodes  # wave instructions -> lane instructions per node
        simd_cyc = simds * t * 1e-9 * clk
        cu_cyc = cus * t * 1e-9 * clk
        lines.append(
            f"* {tag}: per node {c['SQ_INSTS_VALU'] * per:.0f} VALU, "
            f"{c['SQ_INSTS_MFMA'] * per:.1f} MFMA and {c['SQ_INSTS_LDS'] * per:.0f} LDS instructions "
            f"({c['SQ_WAVES']:.0f} waves); VALU busy {100 * 4 * c['SQ_ACTIVE_INST_VALU'] / simd_cyc:.0f} %, "
            f"MFMA busy {100 * c['SQ_VALU_MFMA_BUSY_CYCLES'] / simd_cyc:.0f} %, LDS active "
            f"{100 * c['SQ_LDS_IDX_ACTIVE'] / cu_cyc:.0f} % of the launch's cycles; LDS bank conflicts "
            f"{100 * c['SQ_LDS_BANK_CONFLICT'] / max(c['SQ_LDS_IDX_ACTIVE'], 1):.0f} % of LDS-active cycles")
    with open(os.path.join(out, f"closure_step_{n}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("ok")


def batch_summary(prof, out):
    """Time and calibrated HBM traffic of the batched ensemble step (256
    domains, default launch), with the copy calibration of the step
    summaries."""
    from . import batch_hash
    fac = _calibration(prof)
    stats = kernel_stats(os.path.join(prof, "batch_stats"))
    name = [k for k in stats if "k_batch_step" in k][0]
    avg, cnt, _ = last_dispatches(os.path.join(prof, "batch_stats"), "k_batch_step", 100)
    rd = counter_mean(os.path.join(prof, "batch_pmc_FETCH_SIZE"), "k_batch_step") * 1024 * fac["FETCH_SIZE"]
    wr = counter_mean(os.path.join(prof, "batch_pmc_WRITE_SIZE"), "k_batch_step") * 1024 * fac["WRITE_SIZE"]
    from .inputs import batch_domains
    nodes = sum(d["side"] ** 2 for d in batch_domains(256, seed=0))
    alg = 152 * nodes
    traffic = {"kernel": name, "kernel_hash": batch_hash(), "nodes": nodes, "storage": "f32",
               "bytes_per_launch": rd + wr, "read_bytes": rd, "write_bytes": wr,
               "algorithmic_bytes": alg, "fetch_factor": fac["FETCH_SIZE"],
               "write_factor": fac["WRITE_SIZE"]}
    with open(os.path.join(out, "traffic_batch_f32_256.json"), "w") as fh:
        json.dump(traffic, fh, indent=1)
    cmd = "python3 bench.py --workload batch --no-autotune --no-cpu-baseline"
    lines = [
        "# batched ensemble step, 256 domains (sides 64..1024), FP32, default launch "
        "(one workgroup per 32x8 tile)",
        "",
        f"Kernel: `{name}`  (source hash {batch_hash()})",
        "",
        "Commands (from the repository root, on the MI355X host; the copy calibration runs as "
        "for the two-dimensional step summaries):",
        "```",
        f"rocprofv3 --kernel-trace --stats --output-format csv -d {prof}/batch_stats -o run -- {cmd} --steps 100 --warmup 5",
        f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {prof}/batch_pmc_FETCH_SIZE -o run -- {cmd} --steps 5 --warmup 1",
        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {prof}/batch_pmc_WRITE_SIZE -o run -- {cmd} --steps 5 --warmup 1",
        f"python -m paper_2602_14667_amd.profsum batch {prof} profiles",
        "```",
        "",
        "| kernel | calls | avg ns | min ns | max ns |",
        "|---|---|---|---|---|",
    ]
    for k, v in sorted(stats.items(), key=lambda kv: -kv[1]["avg_ns"] * kv[1]["calls"]):
        lines.append(f"| `{k[:90]}` | {v['calls']} | {v['avg_ns']:.0f} | {v['min_ns']:.0f} "
                     f"| {v['max_ns']:.0f} |")
    lines += [
        "",
        f"* nodes per launch: {nodes}; algorithmic bytes per launch: {alg / 1e9:.3f} GB (152 B/node)",
        f"* last {cnt} dispatches (the timed region): average {avg / 1e3:.1f} us -> "
        f"{nodes / avg * 1e3:.0f} MLUPS, {alg / avg:.1f} GB/s algorithmic = "
        f"{alg / avg / 8000 * 100:.1f} % of 8 TB/s",
        f"* HBM traffic per launch (PMC, calibrated): read {rd / 1e9:.3f} GB "
        f"({rd / (alg / 2):.3f}x algorithmic), write {wr / 1e9:.3f} GB ({wr / (alg / 2):.3f}x); "
        f"{(rd + wr) / avg:.1f} GB/s actual",
        f"* calibration: FETCH_SIZE x {fac['FETCH_SIZE']:.4f}, WRITE_SIZE x {fac['WRITE_SIZE']:.4f} "
        f"(plain copy of {COPY_BYTES} B)",
    ]
    with open(os.path.join(out, "batch_step_256domains.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("ok")


def last_dispatches(stats_dir, kernel, count):
    """Average duration (ns) of the last `count` dispatches of the kernel
    whose name contains `kernel` (the timed region of a bench run)."""
    rows = [r for r in _rows(os.path.join(stats_dir, "run_kernel_trace.csv"))
            if kernel in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    rows = rows[-count:]
    durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows]
    return sum(durs) / len(durs), len(durs), rows[-1]["Kernel_Name"] if rows else ""


def stats_summary(stats_dir, out_md, kernel, bytes_per_launch, title, command, last=0):
    stats = kernel_stats(stats_dir)
    bpl = float(bytes_per_launch)
    names = [k for k in stats if kernel in k]
    lines = [f"# {title}", "", "Command (from the repository root, on the MI355X host):", "```",
             command, f"python -m paper_2602_14667_amd.profsum stats {stats_dir} {out_md} "
             f"{kernel} {bytes_per_launch} ...", "```", "",
             "| kernel | calls | avg ns | min ns | max ns |", "|---|---|---|---|---|"]
    for k, v in sorted(stats.items(), key=lambda kv: -kv[1]["avg_ns"] * kv[1]["calls"]):
        lines.append(f"| `{k[:90]}` | {v['calls']} | {v['avg_ns']:.0f} | {v['min_ns']:.0f} "
                     f"| {v['max_ns']:.0f} |")
    lines.append("")
    for k in names:
        avg = stats[k]["avg_ns"]
        lines.append(f"* `{k[:90]}`: average launch {avg / 1e3:.1f} us; {bpl / 1e9:.4f} GB "
                     f"algorithmic per launch -> {bpl / avg:.1f} GB/s = "
                     f"{bpl / avg / 8000 * 100:.1f} % of 8 TB/s")
    if int(last) > 0:
        avg, cnt, name = last_dispatches(stats_dir, kernel, int(last))
        lines.append(f"* last {cnt} dispatches (the timed region) of `{name[:90]}`: average "
                     f"{avg / 1e3:.1f} us -> {bpl / avg:.1f} GB/s = "
                     f"{bpl / avg / 8000 * 100:.1f} % of 8 TB/s")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("ok")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats_summary(*sys.argv[2:9])
    elif sys.argv[1] == "inplace":
        inplace_summary(*sys.argv[2:5])
    elif sys.argv[1] == "step3d":
        step3d_summary(*sys.argv[2:5])
    elif sys.argv[1] == "batch":
        batch_summary(*sys.argv[2:4])
    elif sys.argv[1] == "closure":
        closure_summary(*sys.argv[2:5])
    else:
        main(*sys.argv[1:4])
