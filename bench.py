"""Benchmark of the coupled LB crystal-growth step on one MI355X.

Headline workload: the 3-D forced-convection grid 192 x 128 x 128 (D3Q19 flow + D3Q7 phase field +
D3Q7 solute, inlet/outlet in x, periodic y/z, seed R 12, U0 = U_in = 0.3), binary32, synthetic
seeded input. One step = one coupled time step of all three lattices (one fused kernel); the
timed loop also runs the diagnostics (binary64 reductions + ray-march along 16 directions) every
100 steps. value = whole-job MLUPS (nodes x steps / time).

Each single-grid case is autotuned first (every tiling timed on real steps of a throw-away solver of
the same grid; the timed solver starts on the choice). Also reported: the fused kernel's roofline (algorithmic bytes per launch / HIP-event launch time,
against the 8 TB/s HBM peak), HBM bytes from rocprofv3 counters when profiles/ holds them for the
current kernel source, the binary16-shift variant, the no-flow 3-D grid, and the oracle timed on the
host cores as a CPU baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-tune] [--tune-file PATH]
       python bench.py --profile-run [--tune-file PATH] [--profile-variants PATH]
                                                (short run for rocprofv3: step kernels, batched sweep,
                                                 surrogate MLP, 1 GiB copy)
       python bench.py --summarize-profiles DIR (rocprofv3 csv output -> profiles/*.md, traffic.json)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MEASURE_EVERY = 100
COPY_BYTES_BENCH = 1 << 30


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def bytes_per_lup(p: dict, prec: str) -> int:
    """Algorithmic HBM bytes per lattice update: every population read once and written once,
    plus phi_prev read and written."""
    qs = 5 if p["dim"] == 2 else 7
    qf = (9 if p["dim"] == 2 else 19) if p["flow"] else 0
    rs = 8 if prec == "fp64" else 4
    fs = {"fp64": 8, "fp32": 4, "fp16shift": 2}[prec]
    return 2 * (2 * qs * rs + qf * fs + rs)


def kernel_source_hash() -> str:
    """Hash of the step kernel's code (its headers with the comments and blank space removed), so
    that counter figures taken on other code are not reported."""
    import re
    h = hashlib.sha256()
    for f in ("step.hpp", "lattice.hpp", "mem.hpp", "chmrt.hpp"):
        with open(os.path.join(ROOT, "paper_2206_02145_amd", "csrc", f)) as fh:
            code = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        code = re.sub(r"//[^\n]*", "", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:16]


def counter_traffic(name: str, variant: str | None = None):
    """HBM bytes per launch from committed rocprofv3 counter runs, if taken on this kernel source (and,
    where the run recorded it, on this tiling)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(name)
    if not e or e.get("kernel_source_hash") != kernel_source_hash():
        return None
    if variant is not None and e.get("variant") not in (None, variant):
        return None
    return e.get("bytes_per_launch")


def time_steps(s, steps: int, measure_every: int = 0, dirs=None):
    """Run `steps` steps on the solver's stream between HIP events; returns milliseconds."""
    import torch
    st = s.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    if measure_every:
        s.run(steps, measure_every, dirs)  # diagnostics on the stream, copied back once; synchronises
    else:
        s.step(steps)
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


REPS = 5  # timed blocks per case; the median is reported


def median_ms(fn, reps: int = REPS):
    import statistics
    return statistics.median(fn() for _ in range(reps))


TUNE_LAUNCHES = 20  # timed steps per tiling and round of the autotuner


def tune_grid(p, prec, walls=None):
    """Autotune the step kernel for this grid on a throw-away solver (real steps of every tiling, two
    rounds); the choice goes into the process's tuning cache, so the next solver of the grid starts
    on it."""
    from paper_2206_02145_amd import lbcg
    s = lbcg.Solver(p, prec)
    if walls is not None:
        s.set_walls(walls)
    s.step(2)
    default = s.variants()[0]
    best, us = s.autotune(TUNE_LAUNCHES)
    chosen = s.variants()[best]
    s.close()
    return dict(default=default, chosen=chosen, chosen_us=round(us, 1))


def gpu_case(name, p, prec, steps, warmup, with_measure, walls=None, tune=True):
    import torch

    from paper_2206_02145_amd import lbcg
    from paper_2206_02145_amd import workloads as W
    nodes = p["nx"] * p["ny"] * p["nz"]
    tuning = tune_grid(p, prec, walls) if tune else None
    s = lbcg.Solver(p, prec)
    if walls is not None:
        s.set_walls(walls)
    variant = s.variants()[s.variant]  # the autotuner's choice (else the default tiling)
    dirs = W.directions(16, p["dim"])
    s.step(warmup)
    torch.cuda.synchronize()
    # the fused step kernel alone: launch-to-launch average on its stream (median of REPS blocks)
    ms_kernel = median_ms(lambda: time_steps(s, steps))
    # whole job: steps plus the diagnostics every min(MEASURE_EVERY, steps) steps (median of REPS blocks)
    every = min(MEASURE_EVERY, steps)
    ms_job = median_ms(lambda: time_steps(s, steps, every, dirs)) if with_measure else ms_kernel
    L, mass = s.measure(dirs)
    s.close()
    del s
    torch.cuda.empty_cache()
    bpl = bytes_per_lup(p, prec)
    t_launch = ms_kernel / steps * 1e-3
    achieved = bpl * nodes / t_launch / 1e9
    out = dict(name=name, nodes=nodes, steps=steps, reps=REPS, ms_per_step=ms_job / steps,
               diagnostics_every=every if with_measure else None,
               mlups=nodes * steps / (ms_job * 1e-3) / 1e6,
               kernel_ms=ms_kernel / steps, kernel_mlups=nodes / t_launch / 1e6,
               bytes_per_lup=bpl, achieved_gbs=achieved, frac=achieved / HBM_PEAK_GBS,
               crystal_mean_L=float(L.mean()), nonfinite=mass["nonfinite"], variant=variant, tuning=tuning)
    log(f"{name}: {out['mlups']:.0f} MLUPS (job), kernel {out['kernel_ms']*1e3:.1f} us/step = "
        f"{achieved:.0f} GB/s algorithmic ({out['frac']*100:.1f}% of {HBM_PEAK_GBS:.0f}); {variant}")
    return out


def copy_bandwidth(nbytes: int = COPY_BYTES_BENCH):
    """Device-to-device copy of nbytes (torch copy_, read + write), median of REPS, in GB/s."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)

    def one():
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)
    ms = median_ms(one)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def sweep_case(n: int, steps: int, measure_every: int, plain: bool = True):
    """Batched parametric sweep of n 2-D instances (side, U0, R, u_in drawn from the seeded generator)
    against the same instances run one after another through the single-grid path."""
    import numpy as np
    import torch

    from paper_2206_02145_amd import lbcg
    from paper_2206_02145_amd import workloads as W
    plist = [W.sweep_instance(*d) for d in W.sweep_draws(n)]
    nodes = sum(p["nx"] * p["ny"] for p in plist)
    dirs = W.directions(16)
    # the batch autotuner: every tiling timed on real steps of a throw-away batch of the same
    # instances; the choice is cached, so the timed batch below starts on it
    tb = lbcg.Batch(plist, "fp32")
    names = tb.variants()
    best, best_us, all_us = tb.autotune(20)
    tb.close()
    del tb
    tuning = {nm: round(float(u), 1) for nm, u in zip(names, all_us)}
    log(f"sweep autotuner: {names[best]} ({best_us:.1f} us/step); " +
        ", ".join(f"{k} {v}" for k, v in tuning.items()))
    t0 = time.perf_counter()
    b = lbcg.Batch(plist, "fp32")
    t_create = time.perf_counter() - t0
    tiling = b.variants()[b.variant]
    b.run(measure_every, measure_every, dirs)  # captures the graph (not timed); a separate batch is timed
    b.close()
    del b
    torch.cuda.synchronize()
    b = lbcg.Batch(plist, "fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist_b = b.run(steps, measure_every, dirs, use_graph=True)
    t_batched = time.perf_counter() - t0
    b.close()
    del b
    out = dict(instances=n, steps=steps, measure_every=measure_every, total_nodes=nodes,
               tiling=tiling, tuning_us_per_step=tuning,
               batched_s=t_batched, batched_runs_per_s=n / t_batched,
               batched_mlups=nodes * steps / t_batched / 1e6, create_s=t_create)
    log(f"sweep batched: {n} runs x {steps} steps in {t_batched:.2f} s = {n / t_batched:.1f} runs/s "
        f"({out['batched_mlups']:.0f} MLUPS)")
    if plain:
        t0 = time.perf_counter()
        hist_p = np.zeros_like(hist_b)
        for i, p in enumerate(plist):
            s = lbcg.Solver(p, "fp32")
            for k in range(steps // measure_every):
                s.step(measure_every)
                hist_p[k, i] = s.measure(dirs)[0]
            s.close()
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        diff = float(np.abs(hist_p - hist_b).max())
        out.update(plain_s=t_plain, plain_runs_per_s=n / t_plain, speedup=t_plain / t_batched,
                   max_abs_L_diff_batched_vs_plain=diff)
        log(f"sweep plain: {t_plain:.2f} s = {n / t_plain:.1f} runs/s; batched speedup {t_plain / t_batched:.1f}x, "
            f"max |L batched - L plain| = {diff:.1e}")
    torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, steps: int = 100):
    """The oracle (FP64 C, OpenMP over rows) on the host cores: `steps` coupled steps of the same grid
    after one warm-up step, in MLUPS; and on one core, `steps` steps of a 16-plane z-slab of it (one
    core would take minutes on the whole grid)."""
    from oracle import oracle
    from paper_2206_02145_amd import workloads as W
    oracle.build(force=False)
    s = oracle.Sim(p)
    s.step(1)
    t0 = time.time()
    s.step(steps)
    dt = time.time() - t0
    nodes = p["nx"] * p["ny"] * p["nz"]
    out = dict(value=nodes * steps / dt / 1e6, unit="MLUPS", cores=oracle.num_threads(), kind="oracle",
               cpu_model=cpu_model(), os_cpus=os.cpu_count(),
               sample=f"{steps} coupled steps of the full {p['nx']}x{p['ny']}x{p['nz']} grid after 1 warm-up "
                      f"step ({dt:.1f} s, FP64)")
    del s
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        q = W.scaled(p, p["nx"], p["ny"], 16)
        s1 = oracle.Sim(q)
        s1.step(1)
        t0 = time.time()
        s1.step(steps)
        dt1 = time.time() - t0
    finally:
        oracle.set_num_threads(threads)
    n1 = q["nx"] * q["ny"] * q["nz"]
    out["single_core"] = dict(value=n1 * steps / dt1 / 1e6, unit="MLUPS", cores=1,
                              sample=f"{steps} coupled steps of a {q['nx']}x{q['ny']}x{q['nz']} z-slab of the "
                                     f"same configuration after 1 warm-up step ({dt1:.1f} s, FP64)")
    return out


PROFILE_STEPS = 200  # steps per solver in the profiled run (the first, colder launches weigh little)
COPY_BYTES = 1 << 30


def _kernel_tag(name: str) -> str:
    """Short tag of a demangled kernel name."""
    if "step_single<" in name:
        args = name.split("step_single<", 1)[1].split(">", 1)[0].replace(" ", "")
        parts = args.split(",")
        dim, flow, real, fst = parts[:4]
        prec = {"double": "fp64", "float": "fp32", "__half": "fp16shift"}[fst]
        extra = "".join(f"_{k}" for k, i in (("walls", 10), ("chmrt", 11)) if len(parts) > i and parts[i] == "true")
        return f"step_{dim}d_{'flow' if flow == 'true' else 'noflow'}{extra}_{prec}"
    if "step_batch<" in name:
        parts = name.split("step_batch<", 1)[1].split(">", 1)[0].replace(" ", "").split(",")
        prec = {"double": "fp64", "float": "fp32", "__half": "fp16shift"}[parts[3]]
        return f"step_batch_{parts[0]}d_{'flow' if parts[1] == 'true' else 'noflow'}_{prec}"
    if "gemm_bf16<" in name:
        epi = name.split("gemm_bf16<", 1)[1].split(">", 1)[0].strip()
        return "gemm_bf16_" + {"0": "fwd_hidden", "1": "fwd_out", "2": "bwd_dx", "3": "dw"}.get(epi, epi)
    if "copyBuffer" in name:
        return "copy_1GiB"
    return name.split("(")[0].split("<")[0].replace("void ", "").strip().rsplit("::", 1)[-1]


PROFILE_MLP_STEPS = 50  # surrogate training steps in the profiled run


def profile_workloads():
    """The solvers that `--profile-run` steps, by kernel tag: parameters of one instance (or the list
    of a batch's instances) and the algorithmic bytes of one launch."""
    from paper_2206_02145_amd import workloads as W
    out = {}
    p3, p2 = W.config3(), W.config2()
    for prec in ("fp32", "fp16shift"):
        out[f"step_3d_flow_{prec}"] = bytes_per_lup(p3, prec) * p3["nx"] * p3["ny"] * p3["nz"]
    out["step_3d_flow_chmrt_fp32"] = out["step_3d_flow_fp32"]
    out["step_3d_noflow_fp32"] = bytes_per_lup(p2, "fp32") * p2["nx"] * p2["ny"] * p2["nz"]
    plist = [W.sweep_instance(*d) for d in W.sweep_draws(256)]
    out["step_batch_2d_flow_fp32"] = sum(bytes_per_lup(q, "fp32") * q["nx"] * q["ny"] for q in plist)
    return out


# summary files: name, title, which kernel tags go in it
PROFILE_GROUPS = [
    ("step_3d_flow_c3.md", "fused coupled step, 3-D 192x128x128 with flow (C3)",
     lambda t: t.startswith("step_3d_flow") or t in ("copy_1GiB", "init_kernel", "__amd_rocclr_fillBufferAligned")),
    ("step_3d_noflow_c2.md", "fused coupled step, 3-D 128^3 without flow (C2)",
     lambda t: t.startswith("step_3d_noflow") or t == "copy_1GiB"),
    ("step_batch_sweep_c4.md", "batched sweep, 256 2-D instances with flow, one launch per step (C4), "
     "and the diagnostics kernels of the profiled run",
     lambda t: t.startswith("step_batch") or t in ("copy_1GiB", "raymarch_batch_kernel", "raymarch_kernel",
                                                  "reduce_kernel", "reduce_final")),
    ("mlp_surrogate_c5.md", f"surrogate MLP (C5), {PROFILE_MLP_STEPS} training steps of batch 1024 and one "
     "prediction of 256 runs x 41 times",
     lambda t: t.startswith("gemm_bf16") or t in ("nll_kernel", "bias_grad_kernel", "split_sum_kernel",
                                                  "gather_kernel", "adam_kernel", "to_bf16_kernel")),
]


def summarize_profiles(d: str, out_dir: str = os.path.join(ROOT, "profiles")):
    """Turn the csv of three rocprofv3 runs of `bench.py --profile-run` (kernel trace + stats,
    --pmc FETCH_SIZE, --pmc WRITE_SIZE) into the summaries of PROFILE_GROUPS under profiles/ and
    profiles/traffic.json. Counter values are KiB per dispatch; each is scaled by what the same
    counter reads for the 1 GiB copy (bytes known)."""
    import csv
    import statistics as st

    def rows(sub, fname):
        with open(os.path.join(d, sub, fname)) as fh:
            return list(csv.DictReader(fh))

    stats = {}
    for r in rows("prof_kt", "run_kernel_trace.csv"):
        stats.setdefault(_kernel_tag(r["Kernel_Name"]), []).append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    counters = {}
    for sub, cname in (("prof_fetch", "FETCH_SIZE"), ("prof_write", "WRITE_SIZE")):
        for r in rows(sub, "run_counter_collection.csv"):
            if r["Counter_Name"] != cname:
                continue
            counters.setdefault((_kernel_tag(r["Kernel_Name"]), cname), []).append(float(r["Counter_Value"]))
    # the calibration copy is the largest of the runtime's copy kernels (the others move a few bytes
    # to a few MB): keep the dispatches within half of the largest
    for key, vals in list(counters.items()) + [(("copy_1GiB", "time"), stats.get("copy_1GiB", []))]:
        if key[0] == "copy_1GiB" and vals:
            big = [v for v in vals if v >= 0.5 * max(vals)]
            if key[1] == "time":
                stats["copy_1GiB"] = big
            else:
                counters[key] = big
    # the copy reads and writes 1 GiB: factor = true KiB / counted KiB
    cal = {}
    cal["FETCH_SIZE"] = (COPY_BYTES / 1024) / st.mean(counters[("copy_1GiB", "FETCH_SIZE")])
    cal["WRITE_SIZE"] = (COPY_BYTES / 1024) / st.mean(counters[("copy_1GiB", "WRITE_SIZE")])
    alg_bytes = profile_workloads()
    variants = {}
    vpath = os.path.join(d, "variants.json")
    if os.path.exists(vpath):
        with open(vpath) as fh:
            variants = json.load(fh)
    traffic = {}
    tf = f"--tune-file {d}/tune_cache.txt"
    head = ["Commands (from the repository root, TMPDIR=/tmp; the first is the bench run whose autotuner "
            "choices the profiled runs start on):", "",
             f"    python3 bench.py {tf}",
             f"    rocprofv3 --kernel-trace --stats -f csv -d {d}/prof_kt -o run -- python3 bench.py --profile-run {tf} "
             f"--profile-variants {d}/variants.json",
             f"    rocprofv3 --pmc FETCH_SIZE -f csv -d {d}/prof_fetch -o run -- python3 bench.py --profile-run {tf}",
             f"    rocprofv3 --pmc WRITE_SIZE -f csv -d {d}/prof_write -o run -- python3 bench.py --profile-run {tf}",
             f"    python3 bench.py --summarize-profiles {d}", ""]
    if variants:
        head += ["Profiled tilings: " + "; ".join(f"{k}: {v}" for k, v in sorted(variants.items())), ""]
    head += [
             f"Counter calibration on a 1 GiB device copy: FETCH_SIZE x {cal['FETCH_SIZE']:.3f}, "
             f"WRITE_SIZE x {cal['WRITE_SIZE']:.3f} (true bytes / counted bytes). Algorithmic GB/s: "
             "algorithmic bytes of one launch / its average duration.", "",
             "| kernel | calls | avg us | median us | min us | max us | read MB | write MB | algorithmic MB | measured / algorithmic | GB/s (measured bytes) | GB/s (algorithmic) |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    table = {}
    for tag in sorted(stats):
        ts = stats[tag]
        fe = counters.get((tag, "FETCH_SIZE"))
        wr = counters.get((tag, "WRITE_SIZE"))
        rd_mb = st.mean(fe) * 1024 * cal["FETCH_SIZE"] / 1e6 if fe else float("nan")
        wr_mb = st.mean(wr) * 1024 * cal["WRITE_SIZE"] / 1e6 if wr else float("nan")
        alg = ratio = alg_gbs = ""
        alg_b = alg_bytes.get(tag, 2 * COPY_BYTES if tag == "copy_1GiB" else None)
        if alg_b:
            alg = f"{alg_b / 1e6:.1f}"
            alg_gbs = f"{alg_b / (st.mean(ts) * 1e-6) / 1e9:.0f}"
        if tag in alg_bytes:
            ratio = f"{(rd_mb + wr_mb) * 1e6 / alg_b:.3f}"
            traffic[tag] = {"bytes_per_launch": round((rd_mb + wr_mb) * 1e6),
                            "read_bytes": round(rd_mb * 1e6), "write_bytes": round(wr_mb * 1e6),
                            "avg_us": round(st.mean(ts), 2), "median_us": round(st.median(ts), 2),
                            "kernel_source_hash": kernel_source_hash(),
                            "variant": variants.get(tag)}
        gbs = (rd_mb + wr_mb) * 1e6 / (st.mean(ts) * 1e-6) / 1e9 if fe and wr else float("nan")
        table[tag] = (f"| {tag} | {len(ts)} | {st.mean(ts):.1f} | {st.median(ts):.1f} | {min(ts):.1f} | {max(ts):.1f} | "
                      f"{rd_mb:.1f} | {wr_mb:.1f} | {alg} | {ratio} | {gbs:.0f} | {alg_gbs} |")
    os.makedirs(out_dir, exist_ok=True)
    for fname, title, keep in PROFILE_GROUPS:
        lines = [f"# rocprofv3 summary: {title}", ""] + head + [table[t] for t in sorted(table) if keep(t)]
        with open(os.path.join(out_dir, fname), "w") as fh:
            fh.write("\n".join(lines) + "\n")
        print("\n".join(lines) + "\n")
    with open(os.path.join(out_dir, "traffic.json"), "w") as fh:
        json.dump(traffic, fh, indent=1)


SQ_COUNTERS = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
               "SQ_INSTS_LDS", "SQ_ACTIVE_INST_VALU", "SQ_BUSY_CYCLES"]


def summarize_sq(d: str):
    """Turn the csv of `rocprofv3 --pmc <SQ_COUNTERS> -- bench.py --profile-run` (under d/prof_sq) into
    profiles/step_3d_flow_c3_sq.md: instruction counts per wavefront of the step kernels and the
    share of the kernel time the VALU pipes are busy (wave64 binary32 VALU instructions issue over 4
    cycles on a 16-lane SIMD; 1024 SIMDs at 2.4 GHz; kernel times from profiles/traffic.json)."""
    import csv
    import statistics as st
    per = {}
    with open(os.path.join(d, "prof_sq", "run_counter_collection.csv")) as fh:
        for r in csv.DictReader(fh):
            tag = _kernel_tag(r["Kernel_Name"])
            if not tag.startswith("step_3d_flow"):
                continue
            per.setdefault(tag, {}).setdefault(int(r["Dispatch_Id"]), {}).setdefault(r["Counter_Name"], 0.0)
            per[tag][int(r["Dispatch_Id"])][r["Counter_Name"]] += float(r["Counter_Value"])
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        times = {k: v["avg_us"] for k, v in json.load(fh).items()}
    lines = ["# rocprofv3 SQ counters: fused coupled step, 3-D 192x128x128 with flow (C3)", "",
             "Commands (from the repository root, TMPDIR=/tmp):", "",
             "    rocprofv3 --pmc " + " ".join(SQ_COUNTERS) +
             f" -f csv -d {d}/prof_sq -o run -- python3 bench.py --profile-run --tune-file {d}/tune_cache.txt",
             f"    python3 bench.py --summarize-sq {d}", "",
             "Per wavefront (one wavefront = one 64-node row segment), mean over the dispatches:", "",
             "| kernel | waves | VALU | SALU | VMEM read | VMEM write | LDS | VALU busy (4 cycles / instruction) |",
             "|---|---|---|---|---|---|---|---|"]
    for tag in sorted(per):
        ds = list(per[tag].values())
        m = {c: st.mean(x.get(c, 0.0) for x in ds) for c in SQ_COUNTERS}
        w = m["SQ_WAVES"] or 1.0
        busy = ""
        if tag in times:
            busy = f"{m['SQ_INSTS_VALU'] * 4 / (1024 * times[tag] * 1e-6 * 2.4e9):.0%}"
        lines.append(f"| {tag} | {m['SQ_WAVES']:.0f} | {m['SQ_INSTS_VALU'] / w:.0f} | {m['SQ_INSTS_SALU'] / w:.0f} | "
                     f"{m['SQ_INSTS_VMEM_RD'] / w:.1f} | {m['SQ_INSTS_VMEM_WR'] / w:.1f} | {m['SQ_INSTS_LDS'] / w:.1f} | {busy} |")
    with open(os.path.join(ROOT, "profiles", "step_3d_flow_c3_sq.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-sweep", action="store_true", help="skip the batched-sweep comparison")
    ap.add_argument("--sweep-n", type=int, default=256)
    ap.add_argument("--sweep-steps", type=int, default=4000)
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate study")
    ap.add_argument("--surrogate-train", type=int, default=4096)
    ap.add_argument("--profile-run", action="store_true",
                    help="a short run of the headline kernel and a 1 GiB copy, for rocprofv3")
    ap.add_argument("--no-tune", action="store_true", help="time the default tilings (no autotuning)")
    ap.add_argument("--profile-variants", metavar="PATH",
                    help="with --profile-run: write the tiling profiled for each kernel (JSON)")
    ap.add_argument("--tune-file", metavar="PATH",
                    help="tuning cache file: the autotuner's choices are appended to it, and solvers of a "
                         "grid it already holds start on that choice (with --profile-run: the tilings profiled)")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="summarise rocprofv3 csv output under DIR into profiles/")
    ap.add_argument("--summarize-sq", metavar="DIR", help="summarise the SQ-counter run under DIR/prof_sq")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        return
    if args.summarize_sq:
        summarize_sq(args.summarize_sq)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this solver runs on a "
              f"single MI355X; a multi-GPU run would shard the grid into slabs)", file=sys.stderr)
        sys.exit(2)
    if args.tune_file:  # read by the library at its first use of the tuning cache
        os.environ["LBCG_TUNE_CACHE"] = os.path.abspath(args.tune_file)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    from paper_2206_02145_amd import lbcg
    from paper_2206_02145_amd import workloads as W
    lbcg.lib()

    p3 = W.config3()
    if args.profile_run:
        # every solver starts on the tiling the tuning file holds for its grid (a bench run with the
        # same --tune-file chose it), else on the default; no autotuning here, so that the profile
        # holds only the profiled tilings
        s = lbcg.Solver(p3, "fp32")
        s16 = lbcg.Solver(W.config3(), "fp16shift")
        sm = lbcg.Solver(dict(W.config3(), collision=1, omega_bulk=1.0), "fp32")
        s2 = lbcg.Solver(W.config2(), "fp32")
        bt = lbcg.Batch([W.sweep_instance(*d) for d in W.sweep_draws(256)], "fp32")
        profiled = {"step_3d_flow_fp32": s, "step_3d_flow_fp16shift": s16, "step_3d_flow_chmrt_fp32": sm,
                    "step_3d_noflow_fp32": s2, "step_batch_2d_flow_fp32": bt}
        profiled = {k: x.variants()[x.variant] for k, x in profiled.items()}
        log("profiled tilings: " + json.dumps(profiled))
        if args.profile_variants:
            with open(args.profile_variants, "w") as fh:
                json.dump(profiled, fh, indent=1)
        for x in (s, s16, sm, s2):
            x.step(PROFILE_STEPS)
        torch.cuda.synchronize()
        for x in (s, s16, sm, s2):
            x.close()
        # the batched sweep (one step_batch launch per step, diagnostics every 100 steps, no graph)
        bt.run(PROFILE_STEPS, MEASURE_EVERY, W.directions(16), use_graph=False)
        bt.close()
        # the surrogate MLP on synthetic rows of the sweep's shape: training steps, then a prediction
        import numpy as np
        from paper_2206_02145_amd import surrogate
        rng = np.random.default_rng(5)
        draws = np.array(W.sweep_draws(256), dtype=np.float64)
        t = np.arange(41, dtype=np.float64) * MEASURE_EVERY
        L = np.cumsum(rng.uniform(0.0, 0.1, (256, 41, surrogate.K_DIRS)), axis=1)
        ds = surrogate.Dataset(draws, t, L, np.stack([surrogate.windowed_slopes(t, L[i]) for i in range(256)]), 0.0)
        net = surrogate.Surrogate()
        net.train(ds, steps=PROFILE_MLP_STEPS, batch=1024)
        net.predict(draws, t)
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)  # 1 GiB read + 1 GiB write, the counter calibration
        torch.cuda.synchronize()
        log("profile run done")
        return

    tn = not args.no_tune
    head = gpu_case("3-D flow 192x128x128 fp32", p3, "fp32", args.steps, args.warmup, True, tune=tn)
    f16 = gpu_case("3-D flow 192x128x128 fp16shift", p3, "fp16shift", args.steps, args.warmup, False, tune=tn)
    c2 = gpu_case("3-D no-flow 128^3 fp32", W.config2(), "fp32", args.steps, args.warmup, False, tune=tn)
    pw, mw = W.config3_walls()
    c3w = gpu_case("3-D flow 192x128x128 fp32, walls and a baffle", pw, "fp32", args.steps, args.warmup, False, mw,
                   tune=tn)
    chm = gpu_case("3-D flow 192x128x128 fp32, central-Hermite MRT", dict(p3, collision=1, omega_bulk=1.0), "fp32",
                   args.steps, args.warmup, False, tune=tn)
    # rows of 191 nodes (764 B, stored at a pitch of 256 nodes) and planes of a power-of-two size
    rag = gpu_case("3-D flow 191x128x128 fp32", W.scaled(p3, 191, 128, 128), "fp32", args.steps, args.warmup, False,
                   tune=tn)
    pw2 = gpu_case("3-D flow 256x128x128 fp32", W.scaled(p3, 256, 128, 128), "fp32", args.steps, args.warmup, False,
                   tune=tn)
    sweep = None if args.no_sweep else sweep_case(args.sweep_n, args.sweep_steps, MEASURE_EVERY)
    surr = None
    if not args.no_surrogate:
        from paper_2206_02145_amd import surrogate
        surr = surrogate.run_study(n_train=args.surrogate_train, log=log)
    copy_gbs = copy_bandwidth()
    log(f"1 GiB device copy: {copy_gbs:.0f} GB/s (read + write)")
    cpu = None if args.no_cpu else cpu_baseline(p3)
    if cpu:
        log(f"cpu baseline: {cpu['value']:.2f} MLUPS on {cpu['cores']} threads ({cpu['sample']})")

    traffic = counter_traffic("step_3d_flow_fp32", head["variant"])
    f16["traffic"] = counter_traffic("step_3d_flow_fp16shift", f16["variant"])
    c2["traffic"] = counter_traffic("step_3d_noflow_fp32", c2["variant"])
    rec = {
        "metric": "coupled-LB MLUPS & HBM-roofline %; sweep runs/s batched vs plain at 1e-4 err",
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded tanh seed, uniform supersaturation, inlet flow)",
        "config": {"workload": "3-D coupled phase-field/solute/flow LB, 192x128x128, D3Q7+D3Q7+D3Q19, "
                               "inlet u=0.02 at x-, outlet x+, periodic y/z, seed R=12, U0=U_in=0.3",
                   "nodes": head["nodes"], "diagnostics_every": head["diagnostics_every"],
                   "timed_blocks": REPS, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(head["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(head["frac"], 4),
                     "traffic": traffic,
                     "kernel": "step_single (" + head["variant"] + ")",
                     "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(head["achieved_gbs"] / copy_gbs, 4),
                     "bytes_per_lup": head["bytes_per_lup"], "kernel_us": round(head["kernel_ms"] * 1e3, 2),
                     "tuning": head["tuning"]},
        "cpu_baseline": cpu,
        "sweep": None if sweep is None else {k: (round(v, 4) if isinstance(v, float) else v) for k, v in sweep.items()},
        "surrogate": surr,
        "variants": {
            "fp16shift_flow": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in f16.items()},
            "no_flow_128cube": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in c2.items()},
            "flow_walls_baffle": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in c3w.items()},
            "flow_chmrt": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in chm.items()},
            "flow_191_rows": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rag.items()},
            "flow_256_wide": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in pw2.items()},
        },
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
