"""Benchmark of the Debye-summation hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]

A step is one full profile evaluation (pack -> pair kernel -> FP64 reduce)
of the 50,000-atom double-helix rod on a 200-point q grid over [0, 1] 1/A,
with inputs already resident in HBM.  The headline value is the whole-job
pair.q rate: N(N-1)/2 pairs times the 199 q values with q > 0, per second.

The JSON line also carries
  roofline      the pair kernel's FP32 rate from HIP events recorded on its own
                launch stream: the flops its recurrence performs per pair.q
                (4.5: one FMA and one add to step sin(q r), an add or FMA to
                accumulate) against the MI355X FP32 vector peak (157.3
                TFLOP/s, one wave64 FMA per SIMD every 2 cycles at 2.4 GHz);
                the survey's nominal 10-flop count as frac_nominal;
  cpu_baseline  the FP64 CPU oracle timed on this host on a bounded sample
                (the same molecule, a subset of q values);
  accuracy      max relative error per q against the stored oracle profile;
  batched/grad  the batched and gradient forms against plain launches.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X FP32 vector peak: 256 CU x 4 SIMD x 2.4 GHz x 64 flop per SIMD-cycle,
# i.e. one wave64 FMA (128 flops) every 2 cycles per SIMD, without packed FP32.
PEAK_FP32_TFLOPS = 157.3
SIMDS, CLOCK_HZ, PEAK_CYCLES_PER_WAVE_INSTR = 1024, 2.4e9, 2.0
# Flops the forward recurrence performs per pair*q (what roofline.achieved
# counts): z += d (1), d = fma(-lambda, z, d) (2), and the accumulate, an add
# on even and an FMA on odd q steps (1.5): 4.5 flops in 3 instructions.  The
# VALU counters agree (4.57 executed FP32 flops per pair*q with the set-up).
EXEC_FLOPS_PER_PAIR_Q = 4.5
INSTR_PER_PAIR_Q = 3
# The adjoint: the same two recurrence operations (3 flops) and three FMA
# accumulations (6 flops) per pair*q.
EXEC_FLOPS_PER_PAIR_Q_ADJ = 9.0
# The survey's nominal count (a rotation of 4 FMAs plus an FMA accumulate; 12
# for the adjoint), which this kernel does not execute: reported beside.
NOMINAL_FLOPS_PER_PAIR_Q = 10.0
NOMINAL_FLOPS_PER_PAIR_Q_ADJ = 12.0
# Issue ceilings of the 3-instruction step: at the peak's 2 cycles per
# instruction, and at the 2.3 cycles a microbenchmark of the step's own
# add/add/FMA mix reached on MI355X.
ISSUE_CEILING_PAIR_Q = SIMDS * CLOCK_HZ * 64 / (INSTR_PER_PAIR_Q * PEAK_CYCLES_PER_WAVE_INSTR)
MIX_CYCLES_PER_WAVE_INSTR = 2.3
MIX_CEILING_PAIR_Q = SIMDS * CLOCK_HZ * 64 / (INSTR_PER_PAIR_Q * MIX_CYCLES_PER_WAVE_INSTR)
BASE_SEED_PER_ATOM = 13062258 + 50
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_forward_dna_rod_50k_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "k_forward_dna_rod_50k_valu.txt")
# What the headline pair kernel's code depends on: its template and device
# helpers, and the argument structs and wave size from the internal header
# (the rest of that header and of the .hip files declares or defines other
# kernels, which do not change this one).
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1306_2258_amd", "csrc", f)
                  for f in ("sas_forward_kernel.hpp", "sas_forward.hpp", "sas_device.hpp", "sas_schedule.hpp")]
KERNEL_HEADER = os.path.join(ROOT, "paper_1306_2258_amd", "csrc", "sas_kernels.hpp")
KERNEL_HEADER_PARTS = ("kWave", "StructDesc", "DescView", "Geometry", "ForwardArgs")


def _code_only(text: str) -> str:
    """C++ source without its comments and with whitespace collapsed: what
    the compiler sees (the kernel sources hold no comment markers inside
    string literals)."""
    import re

    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash() -> str:
    import hashlib
    import re

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f) as fh:
            h.update(_code_only(fh.read()).encode())
    with open(KERNEL_HEADER) as fh:
        text = fh.read()
    for name in KERNEL_HEADER_PARTS:
        m = (re.search(r"constexpr int " + name + r" = [^;]*;", text) or
             re.search(r"struct " + name + r" \{.*?\n\};", text, re.S))
        h.update(_code_only(m.group(0) if m else name + " missing").encode())
    return h.hexdigest()[:16]


def stored_counters(path: str, kernel_name: str):
    """key = value lines of a committed --pmc summary, or None when it is
    missing or was taken on different kernel sources or another kernel."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash() or kv.get("kernel") != kernel_name:
        return None
    return kv


def stored_traffic(kernel_name: str):
    """HBM bytes per pair-kernel launch from the committed FETCH/WRITE summary."""
    kv = stored_counters(TRAFFIC_FILE, kernel_name)
    try:
        return float(kv["hbm_bytes_per_launch"]) if kv else None
    except (KeyError, ValueError):
        return None


def stored_valu(kernel_name: str, work: float, kern_ms: float):
    """Executed FP32 rate and VALU issue figures from the committed VALU
    counter summary, scaled to this run's measured kernel time."""
    kv = stored_counters(VALU_FILE, kernel_name)
    if not kv:
        return None
    try:
        flops = float(kv["SQ_INSTS_VALU_FLOPS_FP32"]) * 64.0
        insts = float(kv["SQ_INSTS_VALU"])
    except (KeyError, ValueError):
        return None
    tflops = flops / (kern_ms / 1e3) / 1e12
    out = {"executed_fp32_flops_per_pair_q": flops / work, "executed_fp32_tflops": tflops,
           "frac_of_fp32_peak": tflops / PEAK_FP32_TFLOPS, "valu_insts_per_pair_q": insts * 64.0 / work,
           "cycles_per_valu_inst_per_simd": (kern_ms / 1e3) * 2.4e9 / (insts / 1024.0),
           "source": os.path.relpath(VALU_FILE, ROOT)}
    # GRBM_GUI_ACTIVE counts busy cycles of each of the 8 XCDs: over the
    # kernel's time it gives the clock the chip actually ran at, and the peak
    # scaled to that clock
    try:
        ghz = float(kv["GRBM_GUI_ACTIVE"]) / 8.0 / (kern_ms / 1e3) / 1e9
    except (KeyError, ValueError):
        ghz = None
    if ghz:
        out["effective_clock_ghz"] = ghz
        out["peak_fp32_tflops_at_clock"] = PEAK_FP32_TFLOPS * ghz / 2.4
    return out


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pair_q(n: int, q: np.ndarray) -> float:
    return n * (n - 1) / 2.0 * float(np.count_nonzero(q > 0))


def cpu_baseline(m, budget_q=(50, 100, 150, 199)):
    import oracle

    pick = np.array(budget_q)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.profile(m.coords, m.types, m.table[:, pick], m.q[pick])
    dt = time.perf_counter() - t0
    work = m.n * (m.n - 1) / 2.0 * len(pick)
    cpu = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": work / dt, "unit": "pair*q/s", "cores": threads, "kind": "oracle", "cpu": cpu,
            "sample": f"dna_rod_50k, all {m.n} atoms, {len(pick)} of the 200 q values "
                      f"(indices {list(budget_q)}), FP64, {dt:.1f} s"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="after the steps, copy a buffer of this many bytes (counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2

    import torch

    import paper_1306_2258_amd as sd
    import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    m = W.dna_rod_50k()
    coords = torch.from_numpy(m.coords).to(dev)
    types = torch.from_numpy(m.types).to(dev)
    table = torch.from_numpy(m.table).to(dev)
    ctx = sd.Context(0)
    out = torch.empty(len(m.q), dtype=torch.float64, device=dev)
    log(f"workload dna_rod_50k N={m.n} Nq={len(m.q)}")

    for _ in range(args.warmup):
        sd.debye_profile(coords, types, table, m.q, ctx=ctx, out=out)
    torch.cuda.synchronize()
    ctx.read_timing()
    ctx.enable_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    e0.record()
    t0 = time.perf_counter()
    marks[0].record()
    for k in range(args.steps):
        sd.debye_profile(coords, types, table, m.q, ctx=ctx, out=out)
        marks[k + 1].record()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    per_step = [marks[k].elapsed_time(marks[k + 1]) for k in range(args.steps)]
    ctx.enable_timing(False)
    kt = ctx.read_timing()
    ms_step = ms_total / args.steps
    work = pair_q(m.n, m.q)
    value = work / (ms_step / 1e3)
    kern_ms = kt["forward_ms"] / max(kt["forward_launches"], 1)
    achieved = EXEC_FLOPS_PER_PAIR_Q * work / (kern_ms / 1e3) / 1e12
    bj, qc = ctx.variant()
    launch = ctx.launch()
    kname = f"k_forward_persist<{qc}, {bj}>" if launch == "persistent" else f"k_forward<{qc}, {bj}>"
    if args.copy_probe > 0:
        nbytes = int(args.copy_probe)
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {nbytes} bytes read and written once")
    log(f"{ms_step:.3f} ms/step (wall {wall / args.steps * 1e3:.3f}), pair kernel {kern_ms:.3f} ms, "
        f"{value:.4e} pair*q/s, variant bj={bj} qc={qc}")

    result = {
        "metric": "pair*q sinc evaluations per second (Debye sum, N=50,000 rod, Nq=200)",
        "value": value,
        "unit": "pair*q/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dna_rod_50k", "atoms": m.n, "nq": len(m.q), "q_range": [0.0, 1.0], "types": 5,
                   "pair_q_per_step": work, "variant": {"bj": bj, "qc": qc, "launch": launch}},
        "ms_per_step_median": float(np.median(per_step)) if per_step else None,
        "ms_per_step_min": float(np.min(per_step)) if per_step else None,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": stored_traffic(kname),
                     "kernel": kname, "kernel_ms": kern_ms, "flops_per_pair_q": EXEC_FLOPS_PER_PAIR_Q,
                     "frac_nominal": NOMINAL_FLOPS_PER_PAIR_Q * work / (kern_ms / 1e3) / 1e12 / PEAK_FP32_TFLOPS,
                     "nominal_flops_per_pair_q": NOMINAL_FLOPS_PER_PAIR_Q,
                     "issue_frac": (work / (kern_ms / 1e3)) / ISSUE_CEILING_PAIR_Q,
                     "issue_frac_mix_floor": (work / (kern_ms / 1e3)) / MIX_CEILING_PAIR_Q,
                     "valu_counters": stored_valu(kname, work, kern_ms)},
    }
    vc = result["roofline"]["valu_counters"]
    if vc and vc.get("peak_fp32_tflops_at_clock"):
        result["roofline"]["frac_clock_adjusted"] = achieved / vc["peak_fp32_tflops_at_clock"]

    # accuracy of the timed output against the stored FP64 oracle profile
    gold = os.path.join(ROOT, "tests", "golden", "dna_rod_50k.txt")
    if os.path.exists(gold):
        ref = np.loadtxt(gold)
        got = out.cpu().numpy()
        err = np.abs(got - ref[:, 1]) / ref[:, 1]
        result["accuracy"] = {"max_rel_err": float(err.max()), "argmax_q": float(ref[err.argmax(), 0]),
                              "median_rel_err": float(np.median(err)),
                              "kappa_at_max": float(ref[err.argmax(), 2] / ref[err.argmax(), 1])}
        log(f"max rel err vs oracle {err.max():.3e}")

    if not args.no_extras:
        # end to end from host arrays (the paper's GPU times include transfers):
        # pageable host-to-device copies of coords, types and table, the profile,
        # and I back on the host; median of 5
        e2e = []
        for _ in range(5):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            c_h = torch.from_numpy(m.coords).to(dev)
            t_h = torch.from_numpy(m.types).to(dev)
            f_h = torch.from_numpy(m.table).to(dev)
            sd.debye_profile(c_h, t_h, f_h, m.q, ctx=ctx).cpu()
            e2e.append(time.perf_counter() - t1)
        e2e_s = float(np.median(e2e))
        result["end_to_end"] = {"ms": e2e_s * 1e3, "pair_q_per_s": work / e2e_s,
                                "includes": "host-to-device copies of coords, types and table, the profile, "
                                            "and the copy of I(q) back to the host"}
        try:
            result["batched"] = bench_batched(sd, W, torch, dev)
        except Exception as exc:  # reported, never hides the headline
            result["batched"] = {"error": str(exc)[:200]}
        try:
            result["grad"] = bench_grad(sd, W, torch, dev)
        except Exception as exc:
            result["grad"] = {"error": str(exc)[:200]}
        try:
            result["direct"] = bench_direct(sd, W, torch, dev, ms_step)
        except Exception as exc:
            result["direct"] = {"error": str(exc)[:200]}
        try:
            result["per_atom"] = bench_per_atom(sd, W, torch, dev, ms_step)
        except Exception as exc:
            result["per_atom"] = {"error": str(exc)[:200]}
        try:
            result["grad_table"] = bench_grad_table(sd, torch, dev, coords, types, table, m.q, ms_step)
        except Exception as exc:
            result["grad_table"] = {"error": str(exc)[:200]}
        try:
            result["hybrid"] = bench_hybrid(sd, W, torch, dev)
        except Exception as exc:
            result["hybrid"] = {"error": str(exc)[:200]}

    if not args.no_cpu:
        log("timing the FP64 CPU oracle on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(m)
        log(f"cpu oracle {result['cpu_baseline']['value']:.3e} pair*q/s on {result['cpu_baseline']['cores']} threads")

    print(json.dumps(result), flush=True)
    return 0


def _time(fn, torch, reps=3):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_batched(sd, W, torch, dev):
    """256 globular structures (500..8000 atoms) on a 100-point grid: one
    batched evaluation (plan replay) against 256 plain calls."""
    log("batched: generating the 256-structure ensemble")
    e = W.globular_ensemble()
    coords = torch.from_numpy(e.coords).to(dev)
    types = torch.from_numpy(e.types).to(dev)
    table = torch.from_numpy(e.table).to(dev)
    work = sum(pair_q(int(n), e.q) for n in e.sizes)
    ctx = sd.Context(0)
    ms_batched = _time(lambda: sd.debye_profile_batched(coords, types, e.offsets, table, e.q, ctx=ctx), torch)
    res = {"structures": int(len(e.sizes)), "atoms": int(e.offsets[-1]), "nq": len(e.q), "pair_q": work,
           "ms_batched_call": ms_batched}
    try:
        plan = sd.BatchedPlan(coords, types, e.offsets, table, e.q, ctx=ctx)
        res["ms_plan_replay"] = _time(plan.execute, torch)
        bj, qc = ctx.variant()
        res["plan_variant"] = {"bj": bj, "qc": qc, "launch": ctx.launch()}
        plan.close()
        # the tuned shape with each launch of the pair kernel forced
        ab = {}
        for launch in ("grid", "persistent"):
            actx = sd.Context(0)
            actx.set_variant(bj, qc)
            actx.set_form(launch)
            p2 = sd.BatchedPlan(coords, types, e.offsets, table, e.q, ctx=actx)
            ab[f"ms_{launch}"] = _time(p2.execute, torch)
            p2.close()
        res["plan_launch_ab"] = ab
    except sd.SasError as exc:
        res["plan"] = str(exc)[:120]
    views = [(coords[int(a):int(b)], types[int(a):int(b)]) for a, b in zip(e.offsets[:-1], e.offsets[1:])]
    ctx2 = sd.Context(0)

    def plain():
        for c, t in views:
            sd.debye_profile(c, t, table, e.q, ctx=ctx2)

    res["ms_plain_launches"] = _time(plain, torch, reps=2)
    # the batched result against the plain calls, structure by structure
    batched = sd.debye_profile_batched(coords, types, e.offsets, table, e.q, ctx=ctx)
    diff = 0.0
    for s_idx, (c, t) in enumerate(views):
        p = sd.debye_profile(c, t, table, e.q, ctx=ctx2)
        diff = max(diff, float(((batched[s_idx] - p).abs() / p.abs()).max()))
    res["max_rel_diff_vs_plain"] = diff
    best = min(res.get("ms_plan_replay", ms_batched), ms_batched)
    res["speedup_vs_plain"] = res["ms_plain_launches"] / best
    res["pair_q_per_s"] = work / (best / 1e3)
    log(f"batched {best:.3f} ms vs plain {res['ms_plain_launches']:.3f} ms")
    return res


def bench_direct(sd, W, torch, dev, ms_recurrence):
    """The direct form (one sine per pair and q) on the 50,000-atom rod:
    a 200-point log-spaced grid on [1e-3, 1], and the benchmark's uniform
    grid forced into the direct form (what the recurrence saves)."""
    res = {}
    for label, m, form in (("log_grid_200", W.dna_rod_50k(q=W.log_grid(1e-3, 1.0, 200)), "auto"),
                           ("uniform_grid_200_forced", W.dna_rod_50k(), "direct")):
        coords = torch.from_numpy(m.coords).to(dev)
        types = torch.from_numpy(m.types).to(dev)
        table = torch.from_numpy(m.table).to(dev)
        ctx = sd.Context(0)
        ctx.set_form(form)
        sd.debye_profile(coords, types, table, m.q, ctx=ctx)
        torch.cuda.synchronize()
        ctx.read_timing()
        ctx.enable_timing(True)
        ms = _time(lambda: sd.debye_profile(coords, types, table, m.q, ctx=ctx), torch)
        ctx.enable_timing(False)
        kt = ctx.read_timing()
        kern_ms = kt["forward_ms"] / max(kt["forward_launches"], 1)
        work = pair_q(m.n, m.q)
        res[label] = {"form": ctx.form(), "ms": ms, "kernel_ms": kern_ms, "pair_q_per_s": work / (ms / 1e3),
                      "kernel_pair_q_per_s": work / (kern_ms / 1e3)}
        log(f"direct form {label}: {ms:.3f} ms (pair kernel {kern_ms:.3f} ms)")
    res["recurrence_speedup"] = res["uniform_grid_200_forced"]["ms"] / ms_recurrence
    return res


def bench_per_atom(sd, W, torch, dev, ms_types):
    """The 50,000-atom rod with one table row per atom (T = N = 50,000), on
    the benchmark's 200-point grid: the per-atom form against the type-sorted
    form of the headline."""
    m = W.with_per_atom_factors(W.dna_rod_50k(), BASE_SEED_PER_ATOM)
    coords = torch.from_numpy(m.coords).to(dev)
    types = torch.from_numpy(m.types).to(dev)
    table = torch.from_numpy(m.table).to(dev)
    ctx = sd.Context(0)
    sd.debye_profile(coords, types, table, m.q, ctx=ctx)
    torch.cuda.synchronize()
    ctx.read_timing()
    ctx.enable_timing(True)
    ms = _time(lambda: sd.debye_profile(coords, types, table, m.q, ctx=ctx), torch)
    ctx.enable_timing(False)
    kt = ctx.read_timing()
    kern_ms = kt["forward_ms"] / max(kt["forward_launches"], 1)
    work = pair_q(m.n, m.q)
    bj, qc = ctx.variant()
    log(f"per-atom form (T=N=50,000): {ms:.3f} ms (pair kernel {kern_ms:.3f} ms)")
    out = {"form": ctx.form(), "types": int(m.table.shape[0]), "variant": {"bj": bj, "qc": qc}, "ms": ms,
           "kernel_ms": kern_ms, "pair_q_per_s": work / (ms / 1e3), "slowdown_vs_type_form": ms / ms_types}
    # the table gradient with one row per atom: per-atom sums over the whole
    # square of pairs (twice the profile's pairs), profile returned too
    w = torch.ones(len(m.q), dtype=torch.float64, device=dev)
    sd.debye_grad_table(coords, types, table, m.q, w, with_profile=True, ctx=ctx)
    torch.cuda.synchronize()
    ctx.read_timing()
    ctx.enable_timing(True)
    ms_g = _time(lambda: sd.debye_grad_table(coords, types, table, m.q, w, with_profile=True, ctx=ctx), torch)
    ctx.enable_timing(False)
    kt = ctx.read_timing()
    kern_g = kt["forward_ms"] / max(kt["forward_launches"], 1)
    log(f"per-atom table gradient + profile: {ms_g:.3f} ms (square pair kernel {kern_g:.3f} ms)")
    out["table_grad"] = {"ms_profile_plus_table_grad": ms_g, "kernel_ms": kern_g,
                         "square_pair_q_per_s": 2.0 * work / (kern_g / 1e3), "ratio_vs_profile": ms_g / ms}
    # the coordinate gradient with one row per atom (per-atom adjoint), the
    # profile returned too
    sd.debye_grad(coords, types, table, m.q, w, with_profile=True, ctx=ctx)
    torch.cuda.synchronize()
    ctx.read_timing()
    ctx.enable_timing(True)
    ms_c = _time(lambda: sd.debye_grad(coords, types, table, m.q, w, with_profile=True, ctx=ctx), torch)
    ctx.enable_timing(False)
    kt = ctx.read_timing()
    adj_ms = kt["adjoint_ms"] / max(kt["adjoint_launches"], 1)
    log(f"per-atom coordinate gradient + profile: {ms_c:.3f} ms (adjoint kernel {adj_ms:.3f} ms)")
    out["coord_grad"] = {"ms_profile_plus_grad": ms_c, "adjoint_kernel_ms": adj_ms,
                         "adjoint_pair_q_per_s": work / (adj_ms / 1e3), "ratio_vs_profile": ms_c / ms}
    return out


def bench_grad_table(sd, torch, dev, coords, types, table, q, ms_profile):
    """dL/dtable for the rod's 5-type table on the benchmark's grid (profile
    returned too) against the profile alone."""
    ctx = sd.Context(0)
    w = torch.ones(len(q), dtype=torch.float64, device=dev)
    ms = _time(lambda: sd.debye_grad_table(coords, types, table, q, w, with_profile=True, ctx=ctx), torch)
    log(f"table gradient + profile {ms:.3f} ms vs profile {ms_profile:.3f} ms")
    return {"types": int(table.shape[0]), "ms_profile_plus_table_grad": ms, "ratio": ms / ms_profile}


def bench_hybrid(sd, W, torch, dev):
    """A 50,000-atom globule (R about 51 A) on 200 q in [0, 1]: the hybrid
    (orientation average where cheaper, tol 1e-9) against the direct sum; the
    largest relative difference between the two profiles is the hybrid's
    error (the direct sum is within 1e-7 of the oracle)."""
    m = W.globular(50000)
    coords = torch.from_numpy(m.coords).to(dev)
    types = torch.from_numpy(m.types).to(dev)
    table = torch.from_numpy(m.table).to(dev)
    ctx = sd.Context(0)
    direct = sd.debye_profile(coords, types, table, m.q, ctx=ctx).clone()
    ms_direct = _time(lambda: sd.debye_profile(coords, types, table, m.q, ctx=ctx), torch)
    I, n_o = sd.debye_profile_hybrid(coords, types, table, m.q, tol=1e-9, ctx=ctx)
    ms_hybrid = _time(lambda: sd.debye_profile_hybrid(coords, types, table, m.q, tol=1e-9, ctx=ctx), torch)
    diff = float(((I - direct).abs() / direct.abs()).max())
    log(f"hybrid {ms_hybrid:.3f} ms ({n_o} q averaged) vs direct {ms_direct:.3f} ms, max rel diff {diff:.2e}")
    out = {"atoms": m.n, "nq": len(m.q), "q_averaged": n_o, "ms_direct": ms_direct, "ms_hybrid": ms_hybrid,
           "speedup": ms_direct / ms_hybrid, "max_rel_diff": diff}
    out["split"] = bench_hybrid_split(sd, W, torch, dev, ctx)
    return out


def bench_hybrid_split(sd, W, torch, dev, ctx):
    """A 20,000-atom globule on 200 q in [0, 1], where the automatic hybrid
    averages a low-q prefix and sums the rest directly on a second stream:
    the call against the two parts run alone and against the direct sum of
    every q."""
    m = W.globular(20000, nq=200)
    coords = torch.from_numpy(m.coords).to(dev)
    types = torch.from_numpy(m.types).to(dev)
    table = torch.from_numpy(m.table).to(dev)
    direct = sd.debye_profile(coords, types, table, m.q, ctx=ctx).clone()
    ms_direct = _time(lambda: sd.debye_profile(coords, types, table, m.q, ctx=ctx), torch)
    I, n_o = sd.debye_profile_hybrid(coords, types, table, m.q, tol=1e-9, ctx=ctx)
    ms_hybrid = _time(lambda: sd.debye_profile_hybrid(coords, types, table, m.q, tol=1e-9, ctx=ctx), torch)
    diff = float(((I - direct).abs() / direct.abs()).max())
    res = {"atoms": m.n, "nq": len(m.q), "q_averaged": n_o, "ms_hybrid": ms_hybrid, "ms_direct": ms_direct,
           "max_rel_diff": diff}
    if 0 < n_o < len(m.q):
        qo, qd = np.ascontiguousarray(m.q[:n_o]), np.ascontiguousarray(m.q[n_o:])
        to, td = table[:, :n_o].contiguous(), table[:, n_o:].contiguous()
        res["ms_orient_part_alone"] = _time(
            lambda: sd.debye_profile_hybrid(coords, types, to, qo, tol=1e-9, mode="orient", ctx=ctx), torch)
        res["ms_direct_part_alone"] = _time(lambda: sd.debye_profile(coords, types, td, qd, ctx=ctx), torch)
    log(f"hybrid split: {n_o} of {len(m.q)} q averaged, {ms_hybrid:.3f} ms vs direct {ms_direct:.3f} ms"
        + (f" (parts alone {res['ms_orient_part_alone']:.3f} + {res['ms_direct_part_alone']:.3f} ms)"
           if "ms_orient_part_alone" in res else ""))
    return res


def bench_grad(sd, W, torch, dev):
    """20,000-atom lattice, 100 q: chi^2 against the seeded perturbed copy's
    profile (weights w_m = dchi2/dI_m from the stored oracle profile and
    target), forward + adjoint against the forward alone; the gradient's
    error against the stored oracle gradient at 65 atoms (48 random, the
    rest at block and strip edges)."""
    m = W.lattice_20k()
    coords = torch.from_numpy(m.coords).to(dev)
    types = torch.from_numpy(m.types).to(dev)
    table = torch.from_numpy(m.table).to(dev)
    ctx = sd.Context(0)
    # stored values written by tests/golden/make_golden.py from the oracle
    gold = os.path.join(ROOT, "tests", "golden")
    with open(os.path.join(gold, "lattice_20k_grad.txt")) as fh:
        lines = [ln for ln in fh if not ln.startswith("#")]
    w_h = np.array([float(v) for v in lines[0].split()])
    rows = np.array([[float(v) for v in ln.split()] for ln in lines[1:]])
    atoms, g_ref = rows[:, 0].astype(np.int64), rows[:, 1:4]
    I_ref = np.loadtxt(os.path.join(gold, "lattice_20k.txt"))[:, 1]
    w = torch.from_numpy(w_h).to(dev)
    g, I = sd.debye_grad(coords, types, table, m.q, w, with_profile=True, ctx=ctx)
    g = g.cpu().numpy()[atoms]
    err_I = float(np.max(np.abs(I.cpu().numpy() - I_ref) / I_ref))
    e_norm = float(np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref))
    e_atom = float(np.max(np.linalg.norm(g - g_ref, axis=1)) / np.max(np.linalg.norm(g_ref, axis=1)))
    ms_fwd = _time(lambda: sd.debye_profile(coords, types, table, m.q, ctx=ctx), torch)
    torch.cuda.synchronize()
    ctx.read_timing()
    ctx.enable_timing(True)
    ms_grad = _time(lambda: sd.debye_grad(coords, types, table, m.q, w, with_profile=True, ctx=ctx), torch)
    ctx.enable_timing(False)
    kt = ctx.read_timing()
    adj_ms = kt["adjoint_ms"] / max(kt["adjoint_launches"], 1)
    work = pair_q(m.n, m.q)
    log(f"grad {ms_grad:.3f} ms (adjoint kernel {adj_ms:.3f} ms) vs forward {ms_fwd:.3f} ms; "
        f"gradient error {e_norm:.2e} (norm), {e_atom:.2e} (worst atom)")
    res = {"atoms": m.n, "nq": len(m.q), "ms_forward": ms_fwd, "ms_forward_plus_adjoint": ms_grad,
           "adjoint_kernel_ms": adj_ms, "ratio": ms_grad / ms_fwd,
           "fd_equivalent_speedup": 6 * m.n * ms_fwd / ms_grad,
           "adjoint_tflops": EXEC_FLOPS_PER_PAIR_Q_ADJ * work / (adj_ms / 1e3) / 1e12,
           "adjoint_flops_per_pair_q": EXEC_FLOPS_PER_PAIR_Q_ADJ,
           "adjoint_frac_of_peak": EXEC_FLOPS_PER_PAIR_Q_ADJ * work / (adj_ms / 1e3) / 1e12 / PEAK_FP32_TFLOPS,
           "adjoint_frac_nominal": NOMINAL_FLOPS_PER_PAIR_Q_ADJ * work / (adj_ms / 1e3) / 1e12 / PEAK_FP32_TFLOPS,
           "accuracy": {"target": "seeded perturbed copy, stored oracle profile", "grad_rel_norm_err": e_norm,
                        "grad_worst_atom_err": e_atom, "atoms_checked": int(len(atoms)),
                        "profile_max_rel_err": err_I}}
    # the same lattice on a 100-point log-spaced grid: direct forward + direct adjoint
    ql = W.log_grid(1e-3, 0.5, 100)
    tab_l = torch.from_numpy(W.gaussian_table((10.0,), 2.0, ql)).to(dev)
    fwd_l = sd.debye_profile(coords, types, tab_l, ql, ctx=ctx)
    w_l = 2.0 * (fwd_l - fwd_l * 1.01) / (0.01 * fwd_l * 1.01) ** 2
    ms_fwd_l = _time(lambda: sd.debye_profile(coords, types, tab_l, ql, ctx=ctx), torch)
    ms_grad_l = _time(lambda: sd.debye_grad(coords, types, tab_l, ql, w_l, with_profile=True, ctx=ctx), torch)
    log(f"grad on a log grid {ms_grad_l:.3f} ms vs forward {ms_fwd_l:.3f} ms")
    res["log_grid_100"] = {"ms_forward": ms_fwd_l, "ms_forward_plus_adjoint": ms_grad_l,
                           "ratio": ms_grad_l / ms_fwd_l}
    return res


if __name__ == "__main__":
    sys.exit(main())
