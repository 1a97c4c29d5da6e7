"""Benchmark: deduplicated new IDB tuples per second of one semi-naive
fixpoint on one MI355X.

Workload (one step = both fixpoints, every step of the hot path):
  * Reach (transitive closure) on an R-MAT graph (a, b, c = 0.57, 0.19,
    0.19), 2^16 nodes, 200,000 distinct edges;
  * same-generation on a random breadth-first tree of 50,000 nodes with
    1-4 children per node.
Inputs are synthetic (workloads/) and loaded into HBM before timing.  The
timed region is hl_run on both engines (EDB dedup and index builds, every
iteration, the final empty one).  value = (|Reach| + |SG|) / time.

After timing, the outputs are checked bit-exact against independent exact
references: Reach against per-source BFS (tuple count and the per-iteration
delta sizes implied by shortest distances, plus sampled sources row by
row), SG against its closed form on a tree (count, per-iteration deltas,
sampled rows).

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


def make_engine(program, edb, idb, stream, kernel_timing, learned=False):
    from paper_2311_02206_amd import Engine
    e = Engine(device=0, stream=stream, kernel_timing=kernel_timing, learned=learned)
    for name in edb:
        e.declare(name, 2, True)
    for name, ar in idb.items():
        e.declare(name, ar, False)
    for name, rows in edb.items():
        e.load(name, rows)
    e.program(program)
    return e


def verify_reach(e, n_nodes, edges, sources):
    import oracle
    total, hist = oracle.reach_bfs_histogram(n_nodes, edges)
    ok = e.count("Reach") == total
    ok &= e.iteration_counts("Reach", 0) == oracle.reach_deltas_from_histogram(hist)
    R = e.fetch("Reach")
    for s in sources:
        lo, hi = np.searchsorted(R[:, 0], [s, s + 1])
        ok &= np.array_equal(R[lo:hi, 1], oracle.reach_from(n_nodes, edges, s))
    return bool(ok), total


def verify_sg(e, edges, n_sample_rows=2000, seed=0):
    import oracle
    total, deltas = oracle.sg_tree_closed_form(edges)
    ok = e.count("SG") == total and e.iteration_counts("SG", 0) == deltas
    S = e.fetch("SG")
    n = int(edges.max()) + 1
    depth = np.zeros(n, dtype=np.int64)
    parent = np.full(n, -1, dtype=np.int64)
    parent[edges[:, 1]] = edges[:, 0]
    for v in range(1, n):  # breadth-first ids: parents come first
        depth[v] = depth[parent[v]] + 1
    ok &= bool(np.all(S[:, 0] != S[:, 1]))
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(S), size=min(n_sample_rows, len(S)))
    ok &= bool(np.all(depth[S[idx, 0]] == depth[S[idx, 1]]))
    ok &= bool(np.all(np.diff(S[:, 0].astype(np.int64) * (1 << 32) + S[:, 1]) > 0))
    return bool(ok), total


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter passes
    (profiles/<kernel>_traffic.json), or None when there are none or the
    kernel's source has changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["hbm_bytes_per_launch"]


def cpu_baseline(programs):
    """The oracle (single-threaded std::set semi-naive) on a bounded sample of
    the same workload: Reach on R-MAT scale 11 (2,048 nodes, 6,250 edges =
    200,000 / 32) and SG on a 6,250-node tree of the same generator."""
    import oracle
    import workloads
    r = workloads.scaled_rmat(11, 6_250, seed=0xC2A)
    t = workloads.scaled_tree(6_250, seed=0xC2B)
    a = oracle.evaluate(programs["reach"], r["edb"], {"Reach": 2})
    b = oracle.evaluate(programs["sg"], t["edb"], {"SG": 2})
    tuples = len(a.relations["Reach"]) + len(b.relations["SG"])
    secs = a.seconds + b.seconds
    return {"value": tuples / secs, "unit": "tuples/s", "cores": 1, "kind": "oracle",
            "sample": f"Reach on R-MAT scale 11 (6,250 edges; {len(a.relations['Reach'])} tuples) "
                      f"+ SG on a 6,250-node 1-4-ary tree ({len(b.relations['SG'])} tuples); "
                      f"{secs:.1f} s of fixpoint time"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the learned-index run of the same workload")
    ap.add_argument("--batched-instances", type=int, default=4096,
                    help="independent Reach instances for the batched variant (0: skip)")
    ap.add_argument("--one-at-a-time-sample", type=int, default=256)
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="copy this many MiB device-to-device once (a reference kernel of known "
                         "size for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this build has no multi-GPU path); "
              f"got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_2311_02206_amd.hisalog import KERNELS

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
    log("generating inputs")
    reach_wl = workloads.reach_rmat16()
    sg_wl = workloads.sg_tree_50k()
    engines = {
        "reach": make_engine(programs["reach"], reach_wl["edb"], {"Reach": 2}, stream, True),
        "sg": make_engine(programs["sg"], sg_wl["edb"], {"SG": 2}, stream, True),
    }
    torch.cuda.synchronize()

    def step():
        out = {}
        for k, e in engines.items():
            out[k] = e.run()
        return out

    for i in range(args.warmup):
        log(f"warmup {i}")
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    kstats = {k: {kn: [0, 0.0, 0] for kn in KERNELS} for k in engines}
    per = {k: 0.0 for k in engines}
    t0 = time.perf_counter()
    last = None
    for i in range(args.steps):
        last = step()
        for k, e in engines.items():
            per[k] += last[k].seconds
            for kn, (n, ms, b) in e.kernel_stats().items():
                ks = kstats[k][kn]
                ks[0] += n
                ks[1] += ms
                ks[2] += b
        log(f"step {i}: " + ", ".join(f"{k} {last[k].seconds * 1e3:.1f} ms" for k in engines))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tuples = sum(last[k].idb_tuples for k in engines)
    ms_per_step = elapsed / args.steps * 1e3
    value = tuples / (elapsed / args.steps)

    # dominant kernel: the one with the most summed launch time over both
    tot = {kn: (sum(kstats[k][kn][0] for k in engines), sum(kstats[k][kn][1] for k in engines),
                sum(kstats[k][kn][2] for k in engines)) for kn in KERNELS}
    dom = max(tot, key=lambda kn: tot[kn][1])
    n_l, ms_l, b_l = tot[dom]
    avg_s = ms_l / 1e3 / max(n_l, 1)
    achieved = (b_l / max(n_l, 1)) / avg_s / 1e9 if n_l else 0.0
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom), "launches": n_l,
                "avg_launch_us": round(avg_s * 1e6, 2),
                "algorithmic_bytes_per_launch": int(b_l / max(n_l, 1))}

    verified = None
    if not args.no_verify:
        log("verifying against BFS / closed form")
        ok_r, _ = verify_reach(engines["reach"], reach_wl["n_nodes"], reach_wl["edb"]["Edge"],
                               sources=[0, 1, 2, 3, 100, 4095, 20000, 65535])
        ok_s, _ = verify_sg(engines["sg"], sg_wl["edb"]["Edge"])
        verified = bool(ok_r and ok_s)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(programs)

    line = {
        "metric": METRIC, "value": value, "unit": "tuples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "u32" if all(last[k].key_bytes == 4 for k in engines) else "u64",
        "data": "synthetic",
        "config": {"workload": "reach_rmat16_200k+sg_tree_50k", "engine": "plain_hisa",
                   "reach_tuples": last["reach"].idb_tuples, "sg_tuples": last["sg"].idb_tuples,
                   "reach_iterations": last["reach"].iterations,
                   "sg_iterations": last["sg"].iterations,
                   "reach_candidates": last["reach"].candidates,
                   "sg_candidates": last["sg"].candidates},
        "verified": verified,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "per_workload_ms": {k: per[k] / args.steps * 1e3 for k in engines},
        "phase_ms": {k: last[k].phase_ms for k in engines},
        "kernels": {kn: {"launches": v[0], "ms": round(v[1], 3),
                         "GBps": round(v[2] / (v[1] / 1e3) / 1e9, 1) if v[1] else None}
                    for kn, v in tot.items()},
    }
    if not args.no_variants:
        # the same fixpoints with the learned position index in place of the
        # HISA hash probe and the membership search; outputs must be identical
        log("learned-index variant")
        lengines = {
            "reach": make_engine(programs["reach"], reach_wl["edb"], {"Reach": 2}, stream, True,
                                 learned=True),
            "sg": make_engine(programs["sg"], sg_wl["edb"], {"SG": 2}, stream, True,
                              learned=True),
        }
        for e in lengines.values():
            e.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lper = {k: 0.0 for k in lengines}
        lk = {kn: [0, 0.0] for kn in KERNELS}
        lphase = {}
        for i in range(args.steps):
            for k, e in lengines.items():
                r = e.run()
                lper[k] += r.seconds
                lphase[k] = r.phase_ms
                for kn, (n, ms, b) in e.kernel_stats().items():
                    lk[kn][0] += n
                    lk[kn][1] += ms
        torch.cuda.synchronize()
        lel = time.perf_counter() - t0
        same = all(lengines[k].count(n) == engines[k].count(n) and
                   lengines[k].iteration_counts(n, 0) == engines[k].iteration_counts(n, 0)
                   for k, n in (("reach", "Reach"), ("sg", "SG")))
        if not args.no_verify:
            same = same and all(np.array_equal(lengines[k].fetch(n), engines[k].fetch(n))
                                for k, n in (("reach", "Reach"), ("sg", "SG")))
        line["variants"] = {"learned_index": {
            "value": tuples / (lel / args.steps), "ms_per_step": lel / args.steps * 1e3,
            "vs_plain": (tuples / (lel / args.steps)) / value, "identical_output": bool(same),
            "per_workload_ms": {k: lper[k] / args.steps * 1e3 for k in lengines},
            "phase_ms": lphase,
            "kernels_ms": {kn: round(v[1], 3) for kn, v in lk.items()}}}
        for e in lengines.values():
            e.close()
    for e in engines.values():
        e.close()
    engines = {}
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


def batched_variant(stream, n_inst, sample, steps, program, verify=True):
    """Batched Reach: n_inst independent instances (log-uniform 32..4096 nodes,
    2-4x edges) in one engine, against the same instances run one at a time
    (a sample of them, the rate extrapolated per tuple)."""
    import torch
    import workloads
    from paper_2311_02206_amd import Engine
    log(f"batched variant: generating {n_inst} instances")
    nodes, edges = workloads.batched_reach_instances(n_inst, seed=0xC4)
    e = Engine(device=0, stream=stream, ebm_k=1.5)
    e.declare("Edge", 2, True)
    e.declare("Reach", 2, False)
    e.batch_layout(nodes)
    e.load_batched("Edge", edges)
    e.program(program)
    e.run()  # warm-up
    torch.cuda.synchronize()
    t = 0.0
    for _ in range(steps):
        st = e.run()
        t += st.seconds
    t /= steps
    log(f"batched: {st.idb_tuples} tuples, {st.iterations} iterations, {t * 1e3:.1f} ms")
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
    value = st.idb_tuples / t
    one_rate = one_tuples / one_t
    out = {"workload": f"batched_reach_{n_inst}_instances", "value": value, "unit": "tuples/s",
           "ms_per_fixpoint": t * 1e3, "tuples": st.idb_tuples, "iterations": st.iterations,
           "key_bytes": st.key_bytes, "peak_bytes": st.peak_bytes, "ebm_k": 1.5,
           "one_at_a_time": {"value": one_rate, "unit": "tuples/s", "sample_instances": sample,
                             "ms": one_t * 1e3},
           "vs_one_at_a_time": value / one_rate,
           "sample_identical": bool(same) if verify else None}
    e.close()
    return out


if __name__ == "__main__":
    main()
