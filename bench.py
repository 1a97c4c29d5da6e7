"""Benchmark: deduplicated new IDB tuples per second of one semi-naive
fixpoint on one MI355X.

Workload (one step = both fixpoints, every step of the hot path):
  * Reach (transitive closure) on an R-MAT graph (a, b, c = 0.57, 0.19,
    0.19), 2^16 nodes, 200,000 distinct edges;
  * same-generation on a random breadth-first tree of 50,000 nodes with
    1-4 children per node.
Inputs are synthetic (workloads/) and in HBM before timing.  Every step
runs both fixpoints on fresh engines carved from one caller-owned arena;
the timed region is hl_run (EDB dedup and index builds, every iteration,
the final empty one).  value = (|Reach| + |SG|) / median step time.  The
same fixpoints on engines kept across runs are reported beside it.

After timing, the outputs are checked for form (sorted, unique, size equal
to the summed deltas); bit-exact parity of these same runs against exact
references (per-source BFS, the closed form of SG on a tree, naive matrix
evaluation of the CSPA-shaped program) is in tests/test_gpu_full.py.

Variants on the same line: the learned position index and the autotuned
settings on the same workload; plain vs learned on the CSPA-shaped program
(2^14 ids), on Reach over a 2^22-node subcritical ER graph and on the
nonlinear closure of that graph; eager buffer management off vs on; sort
and merge of random arity-2 tuples at 1e6..5e8; 4,096 batched Reach
instances against one-at-a-time runs.

Prints one JSON line (see the keys below).  --gpus N > 1 is refused: this
build runs on one GPU.
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

METRIC = "new IDB tuples/sec per fixpoint (learned/batched vs plain HISA), bit-exact"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_engine(program, edb, idb, stream, kernel_timing, learned=False, **kw):
    from paper_2311_02206_amd import Engine
    e = Engine(device=0, stream=stream, kernel_timing=kernel_timing, learned=learned, **kw)
    for name in edb:
        e.declare(name, 2, True)
    for name, ar in idb.items():
        e.declare(name, ar, False)
    for name, rows in edb.items():
        e.load(name, rows)
    e.program(program)
    return e


def well_formed(e, name):
    """The fetched relation is sorted and duplicate-free and its size is the
    sum of the per-iteration deltas (checks on the output alone; bit-exact
    parity at these sizes is in tests/test_gpu_full.py)."""
    R = e.fetch(name)
    key = (R[:, 0].astype(np.uint64) << np.uint64(32)) | R[:, 1].astype(np.uint64)
    return bool(np.all(key[1:] > key[:-1]) and len(R) == sum(e.iteration_counts(name, 0)))


def kernel_digest(path, definitions):
    """SHA-256 of the text that defines a kernel: each named definition
    (from its opening line to its matching closing brace) and every
    compile-time constant of the file."""
    import hashlib
    src = open(path).read()
    parts = [ln for ln in src.splitlines() if ln.lstrip().startswith("constexpr")]
    for d in definitions:
        i = src.find(d)
        if i < 0:
            return None  # the kernel was rewritten since
        j = src.index("{", i)
        depth = 0
        for k in range(j, len(src)):
            depth += {"{": 1, "}": -1}.get(src[k], 0)
            if depth == 0:
                parts.append(src[i:k + 1])
                break
    return hashlib.sha256("\n".join(parts).encode()).hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter passes
    (profiles/<kernel>_traffic.json), or None when there are none or the
    kernel's defining source text has changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if kernel_digest(os.path.join(ROOT, rec["source"]), rec["definitions"]) != rec["source_digest"]:
        return None
    return rec["hbm_bytes_per_launch"]


def host_info():
    """The host the CPU figures were taken on: logical CPUs, the CPUs this
    process may run on, the CPU model and the RAM."""
    model, ram = None, None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
        for ln in open("/proc/meminfo"):
            if ln.startswith("MemTotal"):
                ram = round(int(ln.split()[1]) / 2**20, 1)
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)),
            "cpu_model": model, "ram_gib": ram}


def cpu_baseline(programs, reach_wl):
    """The oracle (single-threaded std::set semi-naive) on a bounded sample of
    the same workload: Reach on R-MAT scale 11 (2,048 nodes, 6,250 edges =
    200,000 / 32) and SG on a 6,250-node tree of the same generator.  Beside
    it: the oracle on the 1,000-node ER Reach configuration at full size,
    and the all-core per-source BFS checker on the full R-MAT Reach input."""
    import oracle
    import workloads
    r = workloads.scaled_rmat(11, 6_250, seed=0xC2A)
    t = workloads.scaled_tree(6_250, seed=0xC2B)
    a = oracle.evaluate(programs["reach"], r["edb"], {"Reach": 2})
    b = oracle.evaluate(programs["sg"], t["edb"], {"SG": 2})
    tuples = len(a.relations["Reach"]) + len(b.relations["SG"])
    secs = a.seconds + b.seconds
    c1 = workloads.reach_er_1000()
    o1 = oracle.evaluate(programs["reach"], c1["edb"], {"Reach": 2})
    threads = min(16, len(os.sched_getaffinity(0)))
    t0 = time.perf_counter()
    total, _ = oracle.reach_bfs_histogram(reach_wl["n_nodes"], reach_wl["edb"]["Edge"],
                                          threads=threads)
    bfs_s = time.perf_counter() - t0
    return {"value": tuples / secs, "unit": "tuples/s", "cores": 1, "kind": "oracle",
            "sample": f"Reach on R-MAT scale 11 (6,250 edges; {len(a.relations['Reach'])} tuples) "
                      f"+ SG on a 6,250-node 1-4-ary tree ({len(b.relations['SG'])} tuples); "
                      f"{secs:.1f} s of fixpoint time",
            "host": host_info(),
            "reach_er_1000_full": {"tuples": len(o1.relations["Reach"]),
                                   "iterations": o1.iterations, "seconds": o1.seconds,
                                   "value": len(o1.relations["Reach"]) / o1.seconds,
                                   "cores": 1},
            "bfs_checker_reach_rmat16_200k": {"tuples": total, "seconds": bfs_s,
                                              "value": total / bfs_s, "cores": threads},
            "table6_host": host_table6()}


TABLE6_SIZES = (1_000_000, 10_000_000, 50_000_000, 100_000_000, 500_000_000)


def host_table6():
    """The host side of the sort / merge / memory microbenchmark: the same
    random 64-bit packed tuples sorted, two sorted halves merged, and a
    fresh buffer of the tuples' size allocated and written, on the host's
    threads (at most 16, the share of host cores that goes with one GPU).
    Repetitions: as many as fit about 2 s per size (at least 1, at most
    100); s_per_100 scales the per-run time to the paper's 100 runs."""
    import oracle
    threads = min(16, len(os.sched_getaffinity(0)))
    rng = np.random.default_rng(6)
    rows = []
    for n in TABLE6_SIZES:
        src = rng.integers(0, 2**64 - 1, size=n, dtype=np.uint64, endpoint=True)
        work = np.empty_like(src)
        st = []
        reps = 1
        while True:
            np.copyto(work, src)
            st.append(oracle.host_sort_u64(work, threads))
            if len(st) >= reps:
                reps = max(1, min(100, int(2.0 / max(st[0], 1e-6))))
                if len(st) >= reps:
                    break
        half = n // 2
        a = work[:half].copy()
        b = np.sort(src[half:2 * half])
        out = np.empty(2 * half, dtype=np.uint64)
        mt = [oracle.host_merge_u64(a, b, out, threads) for _ in range(reps)]
        al = [oracle.host_alloc_init(n * 8, threads) for _ in range(reps)]
        srt, mrg, mem = (float(np.median(x)) for x in (st, mt, al))
        rows.append({"tuples": n, "reps": reps, "sort_ms": round(srt * 1e3, 3),
                     "merge_ms": round(mrg * 1e3, 3), "memory_ms": round(mem * 1e3, 3),
                     "sort_s_per_100": round(srt * 100, 2), "merge_s_per_100": round(mrg * 100, 2),
                     "memory_s_per_100": round(mem * 100, 2)})
        log(f"  host {n}: sort {srt * 1e3:.1f} ms, merge {mrg * 1e3:.1f} ms, "
            f"memory {mem * 1e3:.1f} ms ({reps} reps)")
        del src, work, a, b, out
    return {"threads": threads, "host": host_info(), "rows": rows,
            "note": "64-bit packed tuples; sort: std::sort of one chunk per thread, then "
                    "rounds of merge-path pairwise merges over all threads; memory: malloc "
                    "plus one parallel write of every byte"}


def oracle_timing(programs):
    """The oracle at full size on the two Reach configurations it finishes
    in minutes: the 1,000-node ER graph and the 2^22-node subcritical ER
    graph (about two and a half minutes on one core)."""
    import oracle
    import workloads
    out = {"host": host_info()}
    for name, wl in (("reach_er_1000", workloads.reach_er_1000()),
                     ("reach_er_2p22", workloads.reach_er_2p22())):
        log(f"oracle {name}")
        r = oracle.evaluate(programs["reach"], wl["edb"], {"Reach": 2})
        n = len(r.relations["Reach"])
        out[name] = {"tuples": n, "iterations": r.iterations, "seconds": r.seconds,
                     "value": n / r.seconds, "unit": "tuples/s", "cores": 1}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the learned-index, CSPA and 2^22-node Reach comparisons")
    ap.add_argument("--batched-instances", type=int, default=4096,
                    help="independent Reach instances for the batched variant (0: skip)")
    ap.add_argument("--one-at-a-time-sample", type=int, default=256)
    ap.add_argument("--variant", default="",
                    help="run only this comparison (cspa, reach_er_2p22, nonlinear_er_2p22, "
                         "batched, batched_autotuned, ebm_ablation, nested_join_ablation, "
                         "table6_microbench, oracle_timing) and print its JSON")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="copy this many MiB device-to-device once (a reference kernel of known "
                         "size for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the library has no multi-GPU path); "
              f"got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    programs = {n: open(os.path.join(ROOT, "workloads", "programs", n + ".dl")).read()
                for n in ("reach", "sg")}
    if args.copy_calibration_mb > 0:
        src = torch.ones(args.copy_calibration_mb << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.copy_calibration_mb} MiB device to device")
        del src, dst
    if args.variant:
        steps = max(1, min(args.steps, 3))
        verify = not args.no_verify
        only = {"cspa": lambda: cspa_variant(stream, steps, verify=verify),
                "cspa_rules": lambda: cspa_rules(stream),
                "reach_er_2p22": lambda: er_variant(stream, steps, verify=verify),
                "nonlinear_er_2p22": lambda: nonlinear_variant(stream, steps, verify=verify),
                "batched": lambda: batched_variant(stream, max(1, args.batched_instances),
                                                   args.one_at_a_time_sample, steps,
                                                   programs["reach"], verify=verify),
                "batched_autotuned": lambda: batched_autotuned(
                    stream, max(1, args.batched_instances), steps, programs["reach"]),
                "ebm_ablation": lambda: ebm_ablation(stream, steps),
                "nested_join_ablation": lambda: nested_ablation(stream, steps, verify=verify),
                "table6_microbench": lambda: table6_microbench(stream),
                "oracle_timing": lambda: oracle_timing(programs)}
        if args.variant not in only:
            print(f"unknown variant {args.variant}; one of {sorted(only)}", file=sys.stderr)
            sys.exit(2)
        print(json.dumps({"variant": args.variant, "result": only[args.variant]()}), flush=True)
        return
    log("generating inputs")
    reach_wl = workloads.reach_rmat16()
    sg_wl = workloads.sg_tree_50k()
    specs = {"reach": (programs["reach"], reach_wl["edb"], {"Reach": 2}),
             "sg": (programs["sg"], sg_wl["edb"], {"SG": 2})}
    # the EDB rows are in device memory before any timing; every engine
    # loads them from there (a device-to-device copy, outside the timed run)
    dev_specs = {k: (p, {n: torch.from_numpy(np.ascontiguousarray(rows, dtype=np.uint32)
                                              .view(np.int32)).to("cuda")
                         for n, rows in edb.items()}, idb)
                 for k, (p, edb, idb) in specs.items()}
    torch.cuda.synchronize()

    # 1. Engines kept across runs (eager buffers in their steady state): the
    #    figure beside the headline, and the plain engines the learned and
    #    autotuned variants are compared with.  Timed engines record no
    #    per-kernel events (they cost launch latency).
    engines = {k: make_engine(p, edb, idb, stream, False) for k, (p, edb, idb) in dev_specs.items()}
    for i in range(args.warmup):
        log(f"warmup {i} (reused engines)")
        for e in engines.values():
            e.run()
    reused = {k: [] for k in engines}
    last = {}
    for i in range(args.steps):
        for k, e in engines.items():
            last[k] = e.run()
            reused[k].append(last[k].seconds)
    tuples = sum(last[k].idb_tuples for k in engines)
    reused_med = sum(float(np.median(v)) for v in reused.values())
    peak = max(last[k].peak_bytes for k in engines)
    line_reused = {"value": tuples / reused_med, "ms_per_step": reused_med * 1e3,
                   "per_workload_ms": {k: float(np.median(v)) * 1e3 for k, v in reused.items()},
                   "peak_bytes": {k: last[k].peak_bytes for k in engines}}
    variants = {}
    if not args.no_variants:
        # the same fixpoints with the learned position index in place of the
        # HISA hash probe and the membership search; outputs must be identical
        variants["learned_index"] = learned_variant(stream, dev_specs, args.steps,
                                                    tuples / reused_med, engines,
                                                    verify=not args.no_verify)
        variants["autotuned"] = autotuned_variant(stream, dev_specs, args.steps,
                                                  tuples / reused_med, engines,
                                                  verify=not args.no_verify)
    for e in engines.values():
        e.close()
    engines = {}

    # 2. The headline: every step runs each fixpoint on a fresh engine carved
    #    from one caller-owned arena (a torch tensor), so no run inherits
    #    buffers from an earlier one and no step allocates device memory.
    #    A step's time is the sum of its hl_run wall times; the figure is the
    #    median step.
    arena_bytes = int(peak * 1.25) + (1 << 30)
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    forms = {}

    def fresh_step(check=False):
        out = {}
        for k, (p, edb, idb) in dev_specs.items():
            e = make_engine(p, edb, idb, stream, False, arena=arena)
            try:
                out[k] = e.run()
                if check:
                    forms[k] = well_formed(e, next(iter(idb)))
            finally:
                e.close()
        return out

    for i in range(args.warmup):
        log(f"warmup {i} (fresh engines)")
        fresh_step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    step_s, per = [], {k: [] for k in dev_specs}
    for i in range(args.steps):
        last = fresh_step(check=(i == args.steps - 1) and not args.no_verify)
        step_s.append(sum(r.seconds for r in last.values()))
        for k in dev_specs:
            per[k].append(last[k].seconds)
        log(f"step {i}: " + ", ".join(f"{k} {last[k].seconds * 1e3:.1f} ms" for k in last))
    torch.cuda.synchronize()
    del arena
    torch.cuda.empty_cache()
    med = float(np.median(step_s))
    tuples = sum(last[k].idb_tuples for k in last)
    ms_per_step = med * 1e3
    value = tuples / med
    verified = None if args.no_verify else bool(forms) and all(forms.values())
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(programs, reach_wl)

    line = {
        "metric": METRIC, "value": value, "unit": "tuples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "u32" if all(last[k].key_bytes == 4 for k in last) else "u64",
        "data": "synthetic",
        "config": {"workload": "reach_rmat16_200k+sg_tree_50k", "engine": "plain_hisa",
                   "engines": "fresh per step, carved from a caller-owned arena",
                   "reach_tuples": last["reach"].idb_tuples, "sg_tuples": last["sg"].idb_tuples,
                   "reach_iterations": last["reach"].iterations,
                   "sg_iterations": last["sg"].iterations,
                   "reach_join_outputs": last["reach"].join_outputs,
                   "sg_join_outputs": last["sg"].join_outputs,
                   "reach_candidates": last["reach"].candidates,
                   "sg_candidates": last["sg"].candidates},
        "verified": verified,
        "parity_tests": "tests/test_gpu_full.py (same workloads and engine options: BFS and "
                        "closed-form references, every row and every per-iteration delta)",
        "roofline": None,
        "cpu_baseline": cpu,
        "step_ms": [round(x * 1e3, 3) for x in step_s],
        "per_workload_ms": {k: float(np.median(v)) * 1e3 for k, v in per.items()},
        "phase_ms": {k: last[k].phase_ms for k in last},
        "reused_engine": line_reused,
        "arena_bytes": arena_bytes,
        "kernels": None,
    }
    if variants:
        line["variants"] = variants
    log("kernel-timed pass")
    line["roofline"], line["kernels"] = kernel_pass(stream, dev_specs, runs=2)
    if not args.no_variants:
        for name, fn in (("cspa", cspa_variant), ("reach_er_2p22", er_variant),
                         ("nonlinear_er_2p22", nonlinear_variant)):
            try:
                line["variants"][name] = fn(stream, max(1, min(args.steps, 3)),
                                            verify=not args.no_verify)
            except Exception as exc:  # keep the main line whatever happens here
                line["variants"][name] = {"error": repr(exc)}
    if not args.no_variants:
        for name, fn in (("ebm_ablation", lambda: ebm_ablation(stream, max(1, min(args.steps, 3)))),
                         ("nested_join_ablation",
                          lambda: nested_ablation(stream, max(1, min(args.steps, 3)),
                                                  verify=not args.no_verify)),
                         ("table6_microbench", lambda: table6_microbench(stream))):
            try:
                line["variants"][name] = fn()
            except Exception as exc:  # keep the main line whatever happens here
                line["variants"][name] = {"error": repr(exc)}
    if args.batched_instances > 0:
        try:
            line.setdefault("variants", {})["batched"] = batched_variant(
                stream, args.batched_instances, args.one_at_a_time_sample, max(1, args.steps),
                programs["reach"], verify=not args.no_verify)
        except Exception as exc:  # keep the main line whatever happens here
            line.setdefault("variants", {})["batched"] = {"error": repr(exc)}
    for e in engines.values():
        e.close()
    print(json.dumps(line), flush=True)


def kernel_pass(stream, specs, runs):
    """Per-kernel HIP event timing on separate engines (after one warm-up
    run): the roofline of the kernel with the largest summed launch time and
    the per-kernel totals.  Kept out of the timed steps, whose launches it
    would slow."""
    from paper_2311_02206_amd.hisalog import KERNELS
    engines = {k: make_engine(p, edb, idb, stream, True) for k, (p, edb, idb) in specs.items()}
    try:
        for e in engines.values():
            e.run()
        tot = {kn: [0, 0.0, 0] for kn in KERNELS}
        for _ in range(runs):
            for e in engines.values():
                e.run()
                for kn, (n, ms, b) in e.kernel_stats().items():
                    tot[kn][0] += n
                    tot[kn][1] += ms
                    tot[kn][2] += b
    finally:
        for e in engines.values():
            e.close()
    dom = max(tot, key=lambda kn: tot[kn][1])
    n_l, ms_l, b_l = tot[dom]
    avg_s = ms_l / 1e3 / max(n_l, 1)
    achieved = (b_l / max(n_l, 1)) / avg_s / 1e9 if n_l else 0.0
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom), "launches": n_l,
                "avg_launch_us": round(avg_s * 1e6, 2),
                "algorithmic_bytes_per_launch": int(b_l / max(n_l, 1))}
    kernels = {kn: {"launches": v[0], "ms_per_step": round(v[1] / runs, 3),
                    "GBps": round(v[2] / (v[1] / 1e3) / 1e9, 1) if v[1] else None}
               for kn, v in tot.items()}
    return roofline, kernels


def timed_runs(engines, steps, cold=None):
    """Warm up, then time ``steps`` runs of each engine (hl_run wall time).
    Warm-up repeats (at most three runs) until a run needs no new device
    allocation, so the timed runs measure the steady state of eager buffer
    management; the first run's time goes to ``cold`` (a dict) if given.
    Returns (summed median seconds, per-engine median seconds, last stats)."""
    import torch
    for k, e in engines.items():
        r = e.run()
        if cold is not None:
            cold[k] = r.seconds
        for _ in range(2):
            if r.allocations == 0:
                break
            r = e.run()
    torch.cuda.synchronize()
    runs = {k: [] for k in engines}
    last = {}
    for _ in range(steps):
        for k, e in engines.items():
            last[k] = e.run()
            runs[k].append(last[k].seconds)
    # the median run of each engine: one run that met a device allocation
    # (which the warm-up could not exclude) does not set the figure
    per = {k: float(np.median(v)) for k, v in runs.items()}
    return sum(per.values()), per, last


def identical(a, b, names, verify):
    same = all(a[k].count(n) == b[k].count(n) and
               a[k].iteration_counts(n, 0) == b[k].iteration_counts(n, 0) for k, n in names)
    if verify:
        same = same and all(np.array_equal(a[k].fetch(n), b[k].fetch(n)) for k, n in names)
    return bool(same)


def learned_variant(stream, specs, steps, plain_value, plain_engines, verify=True):
    lengines = {k: make_engine(p, edb, idb, stream, False, learned=True)
                for k, (p, edb, idb) in specs.items()}
    secs, per, last = timed_runs(lengines, steps)
    tuples = sum(r.idb_tuples for r in last.values())
    names = [(k, n) for k, (_, _, idb) in specs.items() for n in idb]
    out = {"value": tuples / secs, "ms_per_step": secs * 1e3, "vs_plain": tuples / secs / plain_value,
           "identical_output": identical(lengines, plain_engines, names, verify),
           "per_workload_ms": {k: v * 1e3 for k, v in per.items()},
           "phase_ms": {k: r.phase_ms for k, r in last.items()}}
    for e in lengines.values():
        e.close()
    return out


def ebm_ablation(stream, steps):
    """Reach with eager buffer management off (exact-size buffers, every
    growth a new allocation and every release a hipFree: the paper's
    "Normal" column of its EBM table) and on, on the 2^22-node ER graph (142
    iterations, long tail) and on R-MAT 2^16."""
    import workloads
    from paper_2311_02206_amd import Engine
    log("ebm ablation")
    prog = open(os.path.join(ROOT, "workloads", "programs", "reach.dl")).read()
    out = {}
    for name, wl in (("reach_er_2p22", workloads.reach_er_2p22()),
                     ("reach_rmat16", workloads.reach_rmat16())):
        row = {}
        for form, ebm in (("normal", False), ("eager", True)):
            e = Engine(device=0, stream=stream, ebm=ebm)
            try:
                e.declare("Edge", 2, True)
                e.declare("Reach", 2, False)
                e.load("Edge", wl["edb"]["Edge"])
                e.program(prog)
                secs, _, last = timed_runs({"x": e}, steps)
                r = last["x"]
                row[form] = {"ms_per_fixpoint": secs * 1e3, "allocations": r.allocations,
                             "peak_bytes": r.peak_bytes, "tuples": r.idb_tuples,
                             "iterations": r.iterations}
            finally:
                e.close()
        row["eager_speedup"] = row["normal"]["ms_per_fixpoint"] / row["eager"]["ms_per_fixpoint"]
        out[name] = row
    return out


def hip_alloc_init_ms(nbytes, stream):
    """Milliseconds to allocate a fresh device buffer of nbytes (hipMalloc,
    which no caching allocator serves) and write every byte once
    (hipMemsetAsync on the stream, then a synchronisation); the buffer is
    freed afterwards, outside the time."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipMemsetAsync.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t,
                                   ctypes.c_void_p]
    hip.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    p = ctypes.c_void_p()
    stream.synchronize()
    t0 = time.perf_counter()
    if hip.hipMalloc(ctypes.byref(p), nbytes) != 0:
        raise MemoryError(f"hipMalloc of {nbytes} bytes failed")
    rc = hip.hipMemsetAsync(p, 0, nbytes, ctypes.c_void_p(stream.cuda_stream))
    rc |= hip.hipStreamSynchronize(ctypes.c_void_p(stream.cuda_stream))
    ms = (time.perf_counter() - t0) * 1e3
    hip.hipFree(p)
    if rc != 0:
        raise RuntimeError("hipMemsetAsync failed")
    return ms


def table6_microbench(stream, reps=100):
    """Sort and merge of random arity-2 tuples (two uniform uint32 columns,
    packed into 64-bit keys, all 64 bits sorted), at the tuple counts of the
    paper's CPU/GPU comparison table, 100 runs each as in the paper.  Merge:
    two sorted halves of N/2 tuples each into one array of N.  Memory: a
    fresh device buffer of the tuples' size allocated and written once (the
    paper's allocation and initialisation column; 10 runs).  Times are per
    run (HIP events around the call on the engine's stream) and, for
    comparison with the table's totals, times 100.  The host side of the
    same table is cpu_baseline.table6_host."""
    import torch
    from paper_2311_02206_amd import Engine
    log("table-6 microbenchmark")
    e = Engine(device=0, stream=stream)
    g = torch.Generator(device="cuda").manual_seed(6)
    rows = []
    try:
        for n in TABLE6_SIZES:
            src = torch.randint(-(1 << 63), (1 << 63) - 1, (n,), dtype=torch.int64,
                                device="cuda", generator=g)
            work = torch.empty_like(src)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            st = []
            for r in range(reps + 1):
                work.copy_(src)
                ev0.record(stream)
                e.sort_keys(work, 64)
                ev1.record(stream)
                ev1.synchronize()
                if r:
                    st.append(ev0.elapsed_time(ev1))
            half = n // 2
            a = work[:half].clone()
            b = src[half:2 * half].clone()
            e.sort_keys(b, 64)
            m = torch.empty(2 * half, dtype=torch.int64, device="cuda")
            mt = []
            for r in range(reps + 1):
                ev0.record(stream)
                e.merge_into(a, b, m)
                ev1.record(stream)
                ev1.synchronize()
                if r:
                    mt.append(ev0.elapsed_time(ev1))
            del m, a, b, work, src
            torch.cuda.empty_cache()
            al = [hip_alloc_init_ms(n * 8, stream) for _ in range(10)]
            srt, mrg, mem = (float(np.median(x)) for x in (st, mt, al))
            rows.append({"tuples": n, "sort_ms": round(srt, 3), "merge_ms": round(mrg, 3),
                         "memory_ms": round(mem, 3),
                         "sort_s_per_100": round(srt / 10, 3), "merge_s_per_100": round(mrg / 10, 3),
                         "memory_s_per_100": round(mem / 10, 3),
                         "sort_GBps": round(3 * 8 * 8 * n / (srt / 1e3) / 1e9, 1),
                         "merge_GBps": round(2 * 8 * 2 * half / (mrg / 1e3) / 1e9, 1)})
            log(f"  {n}: sort {srt:.2f} ms, merge {mrg:.2f} ms, memory {mem:.2f} ms")
    finally:
        e.close()
    return {"reps": reps, "memory_reps": 10, "key_bits": 64, "rows": rows,
            "note": "medians of the runs; sort_GBps counts 8 radix passes of 24 B per key "
                    "(histogram read, scatter read and write); merge_GBps counts one read "
                    "and one write per key; host side: cpu_baseline.table6_host"}


def autotuned_variant(stream, specs, steps, plain_value, plain_engines, verify=True):
    """The same fixpoints after hl_autotune picked each engine's settings
    (probe method and load factor, EBM growth, in-tile dedup); the tuning
    runs are outside the timed steps."""
    log("autotuned variant")
    engines = {k: make_engine(p, edb, idb, stream, False) for k, (p, edb, idb) in specs.items()}
    try:
        chosen = {k: e.autotune(reps=1) for k, e in engines.items()}
        secs, per, last = timed_runs(engines, steps)
        tuples = sum(r.idb_tuples for r in last.values())
        names = [(k, n) for k, (_, _, idb) in specs.items() for n in idb]
        return {"value": tuples / secs, "ms_per_step": secs * 1e3,
                "vs_plain": tuples / secs / plain_value,
                "identical_output": identical(engines, plain_engines, names, verify),
                "per_workload_ms": {k: v * 1e3 for k, v in per.items()},
                "settings": chosen}
    finally:
        for e in engines.values():
            e.close()


LEARNED_FORMS = (("plain", {}), ("learned_index", {"learned": True}))
ALL_FORMS = LEARNED_FORMS + (("fused_graph", {"fused": True, "hip_graph": True}),
                             ("learned_fused_graph", {"learned": True, "fused": True,
                                                      "hip_graph": True}))


def plain_vs_learned(stream, workload, program, edb, idb, steps, verify, extra=None,
                     forms=LEARNED_FORMS):
    """One fixpoint timed on the plain HISA engine and on each other form
    (learned index; fused small iterations from HIP graphs; both); every
    output must be identical to the plain engine's."""
    out = {"workload": workload}
    engines = {}
    try:
        for form, kw in forms:
            e = make_engine(program, edb, idb, stream, False, **kw)
            engines[form] = {"x": e}
            cold = {}
            secs, _, last = timed_runs({"x": e}, steps, cold)
            r = last["x"]
            out[form] = {"value": r.idb_tuples / secs, "unit": "tuples/s",
                         "ms_per_fixpoint": secs * 1e3, "first_run_ms": cold["x"] * 1e3,
                         "allocations_last_run": r.allocations,
                         "tuples": r.idb_tuples,
                         "iterations": r.iterations, "join_outputs": r.join_outputs,
                         "candidates": r.candidates,
                         "key_bytes": r.key_bytes, "peak_bytes": r.peak_bytes,
                         "fused_iterations": r.fused_iterations,
                         "graph_captures": r.graph_captures,
                         "phase_ms": r.phase_ms}
            if verify and not well_formed(e, next(iter(idb))):
                out[form]["well_formed"] = False
        for form, _ in forms[1:]:
            key = "learned_vs_plain" if form == "learned_index" else form + "_vs_plain"
            out[key] = out[form]["value"] / out["plain"]["value"]
        out["identical_output"] = all(identical(engines["plain"], engines[form],
                                                [("x", n) for n in idb], verify)
                                      for form, _ in forms[1:])
        if extra:
            out.update(extra)
    finally:
        for d in engines.values():
            d["x"].close()
    return out


def nonlinear_variant(stream, steps, verify=True):
    """The nonlinear closure T(x,y) :- T(x,z), T(z,y) on the 2^22-node ER
    graph: the growing relation is the join's inner, so its index is
    refreshed after every merge (hash rebuild, or model refit)."""
    import workloads
    log("nonlinear closure variant")
    wl = workloads.reach_er_2p22()
    prog = "T(x, y) :- E(x, y).\nT(x, y) :- T(x, z), T(z, y)."
    return plain_vs_learned(stream, "nonlinear_closure_er_2p22_0.9x", prog,
                            {"E": wl["edb"]["Edge"]}, {"T": 2}, steps, verify)


def nested_ablation(stream, steps, verify=True):
    """Section 5.2 ablation on same-generation over the 50,000-node tree: the
    three-atom rule as a materialised chain of load-balanced binary joins
    (plain) against nested loops, one thread per outer tuple."""
    import workloads
    log("nested join ablation")
    wl = workloads.sg_tree_50k()
    prog = open(os.path.join(ROOT, "workloads", "programs", "sg.dl")).read()
    return plain_vs_learned(stream, "sg_tree_50k", prog, wl["edb"], {"SG": 2}, steps, verify,
                            forms=(("plain", {}), ("nested_joins", {"nested_joins": True})))


def cspa_variant(stream, steps, verify=True):
    """The CSPA-shaped points-to program (10 rules, three mutually recursive
    IDB relations) on Zipf(1.2) pairs over 2^14 ids, literal reading."""
    import workloads
    log("cspa variant")
    wl = workloads.cspa(14)
    prog = open(os.path.join(ROOT, "workloads", "programs", "cspa_shaped.dl")).read()
    return plain_vs_learned(stream, "cspa_shaped_zipf1.2_2p14ids_literal", prog, wl["edb"],
                            {"ValueFlow": 2, "ValueAlias": 2, "MemoryAlias": 2}, steps, verify,
                            {"assign_pairs": len(wl["edb"]["Assign"]),
                             "dereference_pairs": len(wl["edb"]["Dereference"])})


def cspa_rules(stream, scales=(12, 13, 14, 15)):
    """Per-rule join outputs of the CSPA-shaped program (literal reading) as
    the id space doubles: the outputs of each rule's last join and of its
    earlier ones, summed over the run, with the final IDB sizes.  Shows
    which rules drive the growth of the candidates."""
    import workloads
    from paper_2311_02206_amd import Engine
    prog = open(os.path.join(ROOT, "workloads", "programs", "cspa_shaped.dl")).read()
    rules = [ln.strip() for ln in prog.splitlines()
             if ln.strip() and not ln.strip().startswith("//")]
    out = {"rules": rules, "scales": {}}
    for lg in scales:
        log(f"cspa rules: 2^{lg} ids")
        wl = workloads.cspa(lg)
        with Engine(device=0, stream=stream) as e:
            for name in ("Assign", "Dereference"):
                e.declare(name, 2, True)
            for name in ("ValueFlow", "ValueAlias", "MemoryAlias"):
                e.declare(name, 2, False)
            for name, rows in wl["edb"].items():
                e.load(name, rows)
            e.program(prog)
            st = e.run()
            per = e.rule_stats()
            out["scales"][f"2^{lg}"] = {
                "ms": st.seconds * 1e3, "iterations": st.iterations,
                "idb_tuples": st.idb_tuples, "join_outputs": st.join_outputs,
                "per_rule_last_join": [a for a, _ in per],
                "per_rule_earlier_joins": [b for _, b in per],
                "sizes": {n: e.count(n) for n in ("ValueFlow", "ValueAlias", "MemoryAlias")}}
    return out


def er_variant(stream, steps, verify=True):
    """Reach on a subcritical directed ER graph, 2^22 nodes, 0.9 * 2^22 edges
    (long tail of small deltas over a large full relation)."""
    import workloads
    log("reach er 2^22 variant")
    wl = workloads.reach_er_2p22()
    prog = open(os.path.join(ROOT, "workloads", "programs", "reach.dl")).read()
    return plain_vs_learned(stream, "reach_er_2p22_0.9x", prog, wl["edb"], {"Reach": 2},
                            steps, verify, forms=ALL_FORMS)


def batched_autotuned(stream, n_inst, steps, program):
    """The batch after hl_autotune chose its settings (probe method and load
    factor, expand tile, EBM growth, in-tile dedup, fused iterations), timed
    against the engine's defaults with fused iterations from HIP graphs.
    Not part of the default run: the search takes a few minutes."""
    import workloads
    from paper_2311_02206_amd import Engine
    log(f"batched autotune: generating {n_inst} instances")
    nodes, edges = workloads.batched_reach_instances(n_inst, seed=0xC4)
    e = Engine(device=0, stream=stream, ebm_k=1.5, fused=True, hip_graph=True)
    try:
        e.declare("Edge", 2, True)
        e.declare("Reach", 2, False)
        e.batch_layout(nodes)
        e.load_batched("Edge", edges)
        e.program(program)
        for _ in range(4):
            if e.run().allocations == 0:
                break
        before = sorted(e.run().seconds for _ in range(steps))[steps // 2]
        counts = e.iteration_counts("Reach", 0)
        chosen = e.autotune(reps=1)
        for _ in range(4):
            if e.run().allocations == 0:
                break
        runs = [e.run() for _ in range(steps)]
        after = sorted(r.seconds for r in runs)[steps // 2]
        return {"workload": f"batched_reach_{n_inst}_instances", "tuples": runs[-1].idb_tuples,
                "ms_before": before * 1e3, "ms_after": after * 1e3, "speedup": before / after,
                "same_deltas": e.iteration_counts("Reach", 0) == counts, "settings": chosen}
    finally:
        e.close()


def batched_variant(stream, n_inst, sample, steps, program, verify=True):
    """Batched Reach: n_inst independent instances (log-uniform 32..4096 nodes,
    2-4x edges) in one engine, with fused small iterations replayed from HIP
    graphs and without them, against the same instances run one at a time
    (a sample of them, the rate extrapolated per tuple)."""
    import torch
    import workloads
    from paper_2311_02206_amd import Engine
    log(f"batched variant: generating {n_inst} instances")
    nodes, edges = workloads.batched_reach_instances(n_inst, seed=0xC4)
    forms = {}
    e = None
    for form, kw in (("plain", {}), ("fused_graph", {"fused": True, "hip_graph": True})):
        if e is not None:
            e.close()
        e = Engine(device=0, stream=stream, ebm_k=1.5, **kw)
        e.declare("Edge", 2, True)
        e.declare("Reach", 2, False)
        e.batch_layout(nodes)
        e.load_batched("Edge", edges)
        e.program(program)
        for _ in range(4):  # warm-up until the buffers have settled
            if e.run().allocations == 0:
                break
        torch.cuda.synchronize()
        t = 0.0
        for _ in range(steps):
            st = e.run()
            t += st.seconds
        t /= steps
        log(f"batched {form}: {st.idb_tuples} tuples, {st.iterations} iterations, "
            f"{st.fused_iterations} fused, {t * 1e3:.1f} ms")
        forms[form] = {"value": st.idb_tuples / t, "ms_per_fixpoint": t * 1e3,
                       "fused_iterations": st.fused_iterations,
                       "fused_overflows": st.fused_overflows,
                       "graph_captures": st.graph_captures,
                       "allocations_last_run": st.allocations, "peak_bytes": st.peak_bytes,
                       "phase_ms": st.phase_ms,
                       "counts": e.iteration_counts("Reach", 0)}
    # e is the fused engine: its output is checked against one-at-a-time runs
    sample = min(sample, n_inst)
    one_t, one_tuples, same = 0.0, 0, True
    for k in range(sample):
        ek = Engine(device=0, stream=stream)
        ek.declare("Edge", 2, True)
        ek.declare("Reach", 2, False)
        ek.load("Edge", edges[k])
        ek.program(program)
        ek.run()  # warm-up
        sk = ek.run()
        one_t += sk.seconds
        one_tuples += sk.idb_tuples
        if verify and (k < 16 or ek.count("Reach") != e.batch_count("Reach", k)):
            same &= bool(np.array_equal(ek.fetch("Reach"), e.fetch_batched("Reach", k)))
        ek.close()
    value = forms["fused_graph"]["value"]
    one_rate = one_tuples / one_t if one_t > 0 else None
    same_forms = forms["plain"].pop("counts") == forms["fused_graph"].pop("counts")
    out = {"workload": f"batched_reach_{n_inst}_instances", "value": value, "unit": "tuples/s",
           "engine": "batched, fused small iterations from HIP graphs",
           "ms_per_fixpoint": forms["fused_graph"]["ms_per_fixpoint"], "tuples": st.idb_tuples,
           "iterations": st.iterations, "key_bytes": st.key_bytes, "peak_bytes": st.peak_bytes,
           "ebm_k": 1.5, "forms": forms, "forms_same_deltas": bool(same_forms),
           "one_at_a_time": {"value": one_rate, "unit": "tuples/s", "sample_instances": sample,
                             "ms": one_t * 1e3},
           "vs_one_at_a_time": value / one_rate if one_rate else None,
           "sample_identical": bool(same) if verify else None}
    e.close()
    return out


if __name__ == "__main__":
    main()
