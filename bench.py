"""Throughput benchmark: exact per-vertex orbit counts (orbits 0..72).

One step = one full call of the HIP path on a device-resident CSR:
validation, degeneracy peeling, orientation, every enumeration kernel,
the orbit equations and the induced transform, ending with device-resident
uint64 counts.  The metric is edges/s = m / (seconds per step).

Default workload: Chung-Lu power-law graph, n = 1,000,000, mean weight 20,
exponent 2.1, weights capped at 50,000, 10^7 endpoint pairs drawn
proportionally to the weights, self-loops and duplicates removed (seed
0x5EED0002).  Synthetic, generated here; it stands in for the paper's
real-world graphs.

Prints one JSON line (rank 0).  Only the ``cpu_baseline`` leg touches the
CPU oracle.
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
WORKLOADS = {
    "chunglu1m": "Chung-Lu n=1M, mean 20, gamma 2.1, w<=50k, 1e7 pairs, seed 0x5EED0002",
    "er2000": "Erdos-Renyi G(n=2000, p=0.005), seed 0x5EED0001",
    "chunglu1m_perm": "Chung-Lu n=1M as above, vertex ids permuted at random (seed 0x5EED0006)",
    "rmat22": "R-MAT scale 22, edge factor 16, (0.57,0.19,0.19,0.05), seed 0x5EED0003",
    "batch100k": ("100,000 small graphs in one batched call: n uniform in [10, 500], even graphs "
                  "Erdos-Renyi with mean degree 6, odd graphs Barabasi-Albert m=3, seed 0x5EED0004"),
}
TRAIN_WORKLOAD = "chunglu250k"


def train_cost_model(orbit, seed=1, iters=1500, batch=4096):
    """Cost-model weights trained on the per-source step counts of a smaller
    graph of the same family (Chung-Lu n=250k, mean 20, gamma 2.1), so the
    timed graph is never seen in training."""
    import torch
    from paper_1911_10616_amd import graphgen as gg
    rp, ci = gg.workload(TRAIN_WORKLOAD)
    n = len(rp) - 1
    feat = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    steps = torch.empty(n, dtype=torch.int64, device="cuda")
    orbit.Counter(rp, ci, 5, features_out=feat, steps_out=steps).run()
    w = orbit.mlp_init(seed=seed)
    loss = orbit.mlp_train(w, feat, steps, iters=iters, batch=batch, lr=3e-3, seed=seed)
    return w, loss


def cpu_baseline(rp, ci, seconds: float, seed: int = 1):
    """The CPU oracle (rooted enumeration) timed on a bounded sample of the
    same graph, scaled to edges/s by extrapolating the time per vertex."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    n = len(rp) - 1
    m = ci.size // 2
    rng = np.random.Generator(np.random.PCG64(seed))
    order = rng.permutation(n).astype(np.uint32)
    budget = 50_000
    done = 0
    complete = 0
    t0 = time.perf_counter()
    batch = threads
    while time.perf_counter() - t0 < seconds and done < n:
        roots = order[done:done + batch]
        _, comp = oracle.rooted_counts(rp, ci, roots, kmax=5, budget=budget, threads=threads)
        done += roots.size
        complete += int(comp.sum())
    el = time.perf_counter() - t0
    per_vertex = el / max(done, 1)
    est_full = per_vertex * n
    return {
        "value": m / est_full,
        "unit": "edges/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{done} uniformly sampled vertices, rooted enumeration of every connected "
                   f"2..5-vertex subset containing the vertex, at most {budget} subsets each "
                   f"({complete} finished within that budget, the rest were cut off, so the "
                   f"extrapolated CPU rate is an upper bound); {el:.1f} s on {threads} threads, "
                   f"scaled by n/{done}"),
    }


def measured_traffic(workload):
    """HBM bytes per k_pairs launch from the committed rocprofv3 counter
    record, if it was taken on this workload and on the current kernel
    source; None otherwise."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_pairs_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def run_batched(args, orbit, gg, rank):
    """Batched mode: one orbit_count_batched call per step over the whole
    batch (autotuned workgroup count and schedule, chosen before the timed
    steps), against the single-graph path on the same disjoint union with
    the static schedule."""
    import torch
    vptr, rp, ci = gg.workload(args.workload)
    n = len(rp) - 1
    m = ci.size // 2
    if args.no_autotune:
        nwg, sched, groups, tune_ms = 1024, 0, 2, 0.0
        bc = orbit.BatchCounter(vptr, rp, ci, k_max=5, num_wg=nwg, groups="wave")
    else:
        bc = orbit.BatchCounter(vptr, rp, ci, k_max=5)
        nwg, sched, groups, tune_ms = bc.autotune((512, 1024, 2048, 4096))
    for _ in range(args.warmup):
        bc.run(timing=True)
    torch.cuda.synchronize()
    phases = {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bc.run(timing=True)
        for nm, ms in orbit.last_phase_times():
            phases[nm] = phases.get(nm, 0.0) + ms
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stats = orbit.last_stats()
    ms_step = 1000.0 * el / args.steps
    phases = {k: v / args.steps for k, v in phases.items()}
    got = bc.out[:n].clone()
    # the same count captured as one HIP graph and replayed
    plan = orbit.Plan(bc)
    plan.launch()
    plan.status()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        plan.launch()
    plan.status()
    graph_ms = 1000.0 * (time.perf_counter() - t2) / args.steps
    graph_same = bool(torch.equal(bc.out[:n], got))
    plan.close()
    del bc
    torch.cuda.empty_cache()
    compare = None
    if not args.no_compare:
        c = orbit.Counter(rp, ci, k_max=5, schedule="static")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out = c.run()
        torch.cuda.synchronize()
        plain_ms = 1000.0 * (time.perf_counter() - t1)
        same = bool(torch.equal(out[:n], got))
        compare = {"path": "single-graph call on the disjoint union, static schedule",
                   "ms_per_step": round(plain_ms, 3), "speedup_of_batched": round(plain_ms / ms_step, 3),
                   "identical_counts": same}
        del c, out
    dom = max((k for k in phases if k in ("pairs", "c5", "c4", "cliques", "clique2_k4terms")),
              key=lambda k: phases[k])
    line = {
        "metric": "edges/s for all <=5-vertex orbit counts (bit-exact), HBM GB/s vs peak",
        "value": round(m * args.steps / el, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "graphs": int(len(vptr) - 1), "n": n,
                   "m": m, "k_max": 5, "orbits": 73,
                   "output": "induced uint64 counts n x 73, concatenated per graph",
                   "autotuned": {"num_wg": nwg, "schedule": ["id", "static", "mlp"][sched],
                                 "groups": ["auto", "workgroup", "wave"][groups],
                                 "gpu_ms": round(tune_ms, 3)}},
        "phases_ms": {k: round(v, 3) for k, v in phases.items()},
        "dominant_phase": dom,
        "work": stats,
    }
    line["graph_replay"] = {"ms_per_step": round(graph_ms, 3), "identical_counts": graph_same}
    if compare is not None:
        line["vs_plain_path"] = compare
    if rank == 0:
        print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chunglu1m", choices=sorted(WORKLOADS))
    ap.add_argument("--schedule", default="mlp", choices=("id", "static", "mlp"),
                    help="order of sources in the per-source kernels")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched workload: 1024 workgroups, id schedule, no tuning runs")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the one-step run with the static schedule")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 4 GiB device-to-device (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 2 * a.numel() * 4, "read_bytes": a.numel() * 4,
                          "write_bytes": b.numel() * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the library counts on one GPU; sharding over several is not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1911_10616_amd import graphgen as gg
    from paper_1911_10616_amd import orbit

    rank = int(os.environ.get("RANK", "0"))
    torch.cuda.set_device(0)
    if args.workload == "batch100k":
        return run_batched(args, orbit, gg, rank)
    rp, ci = gg.workload(args.workload)
    n = len(rp) - 1
    m = ci.size // 2
    w, train_loss = (None, None)
    if args.schedule == "mlp":
        w, train_loss = train_cost_model(orbit)
    counter = orbit.Counter(rp, ci, k_max=5, schedule=args.schedule, mlp_weights=w)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        counter.run(timing=True)
    torch.cuda.synchronize()
    phases = {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        counter.run(timing=True)
        for nm, ms in orbit.last_phase_times():
            phases[nm] = phases.get(nm, 0.0) + ms
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stats = orbit.last_stats()
    ms_step = 1000.0 * el / args.steps
    compare = None
    if not args.no_compare and args.schedule != "static":
        # the plain static-threshold schedule on the same graph, one step
        del counter
        torch.cuda.empty_cache()
        cs = orbit.Counter(rp, ci, k_max=5, schedule="static")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cs.run()
        torch.cuda.synchronize()
        st_ms = 1000.0 * (time.perf_counter() - t1)
        compare = {"schedule": "static", "ms_per_step": round(st_ms, 3),
                   "speedup_of_" + args.schedule: round(st_ms / ms_step, 4)}
        del cs
    value = m * args.steps / el
    phases = {k: v / args.steps for k, v in phases.items()}

    # dominant kernel: the pair sweep over wedges and diamonds.  Algorithmic
    # bytes per launch = 8 B per wedge (its two endpoint ids) + 8 B per
    # diamond (one triangle-list entry), i.e. 8 (W + D).
    dom = "pairs"
    dom_ms = phases.get(dom, float("nan"))
    alg_bytes = 8.0 * (stats["wedges"] + stats["diamonds"])
    achieved = alg_bytes / (dom_ms / 1000.0) / 1e9
    roofline = {"kernel": "k_pairs", "bound": "hbm", "achieved": round(achieved, 3),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                "traffic": measured_traffic(args.workload), "alg_bytes": alg_bytes,
                "avg_ms": round(dom_ms, 3)}

    line = {
        "metric": "edges/s for all <=5-vertex orbit counts (bit-exact), HBM GB/s vs peak",
        "value": round(value, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "n": n, "m": m, "k_max": 5,
                   "orbits": 73, "output": "induced uint64 counts n x 73",
                   "schedule": args.schedule},
        "roofline": roofline,
        "phases_ms": {k: round(v, 3) for k, v in phases.items()},
        "work": stats,
    }
    if compare is not None:
        line["vs_static_schedule"] = compare
    if train_loss is not None:
        line["cost_model"] = {"trained_on": TRAIN_WORKLOAD, "mse_log2_steps": round(train_loss, 4)}
    if not args.no_cpu_baseline and rank == 0:
        line["cpu_baseline"] = cpu_baseline(rp, ci, args.cpu_seconds)
    if rank == 0:
        print(json.dumps(line), flush=True)
    del stream


if __name__ == "__main__":
    main()
