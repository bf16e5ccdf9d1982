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


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(rp, ci, budget: int = 20_000, per_stratum: int = 2, seed: int = 1):
    """The CPU oracle timed on the host cores on a degree-stratified sample
    of the same graph: per degree decile `per_stratum` seeded vertices,
    each enumerated by the oracle's rooted count (every connected 2..5-vertex
    subset containing it) on one thread, up to `budget` subsets; the vertices
    run in parallel on the cores.  The full-graph time is extrapolated
    stratum by stratum (decile size x mean time per sampled vertex) and
    divided by the cores; a vertex cut off at the budget contributes its
    time so far, so with any cut-off the rate is an upper bound.  Also the
    full oracle on the small Erdos-Renyi workload (it finishes there):
    median of 3 runs on one thread and on all the cores."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    from paper_1911_10616_amd import graphgen as gg
    cores = min(16, os.cpu_count() or 1)
    n = len(rp) - 1
    m = ci.size // 2
    d = np.diff(rp.astype(np.int64))
    order = np.argsort(d, kind="stable")
    rng = np.random.Generator(np.random.PCG64(seed))
    strata = np.array_split(order, 10)
    picks = [(s, int(v)) for s, part in enumerate(strata)
             for v in rng.choice(part, size=min(per_stratum, part.size), replace=False)]

    def one(v):
        t = time.perf_counter()
        _, comp = oracle.rooted_counts(rp, ci, [v], kmax=5, budget=budget, threads=1)
        return time.perf_counter() - t, bool(comp[0])
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        res = list(ex.map(one, [v for _, v in picks]))
    wall = time.perf_counter() - t0
    est = 0.0
    per = []
    for s, part in enumerate(strata):
        ts = [r[0] for (ss, _), r in zip(picks, res) if ss == s]
        done = sum(r[1] for (ss, _), r in zip(picks, res) if ss == s)
        est += part.size * (sum(ts) / max(len(ts), 1))
        per.append({"degrees": [int(d[part[0]]), int(d[part[-1]])], "sampled": len(ts),
                    "finished": done, "mean_s": round(sum(ts) / max(len(ts), 1), 4)})
    finished = sum(r[1] for r in res)
    full_s = est / cores
    # the full oracle where it finishes: Erdos-Renyi G(2000, 0.005)
    erp, eci = gg.workload("er2000")
    em = eci.size // 2
    def timed(threads):
        ts = []
        for _ in range(3):
            t = time.perf_counter()
            oracle.induced_counts(erp, eci, threads=threads)
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))
    t1, tc = timed(1), timed(cores)
    return {
        "value": round(m / full_s, 3),
        "unit": "edges/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{len(picks)} vertices, {per_stratum} per degree decile (seeded), each the "
                   f"oracle's rooted enumeration of every connected 2..5-vertex subset containing "
                   f"it, at most {budget:.0e} subsets, one thread per vertex on {cores} cores "
                   f"({wall:.1f} s); {finished} of {len(picks)} finished within the budget, so the "
                   f"rate is an upper bound (a cut-off vertex counts its time so far); full time "
                   f"= sum over deciles of size x mean time, divided by the cores"),
        "cpu_model": _cpu_model(),
        "nproc": os.cpu_count(),
        "coverage": round(finished / len(picks), 3),
        "extrapolated_full_s": round(full_s, 1),
        "strata": per,
        "er2000_full_oracle": {"m": em, "median_s_1_thread": round(t1, 4),
                               f"median_s_{cores}_threads": round(tc, 4),
                               "edges_per_s_1_thread": round(em / t1, 1),
                               f"edges_per_s_{cores}_threads": round(em / tc, 1)},
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
    phases, kernels = {}, {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bc.run(timing=True)
        for nm, ms in orbit.last_phase_times():
            phases[nm] = phases.get(nm, 0.0) + ms
        for nm, ms in orbit.last_kernel_times().items():
            kernels[nm] = kernels.get(nm, 0.0) + ms
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stats = orbit.last_stats()
    ms_step = 1000.0 * el / args.steps
    phases = {k: v / args.steps for k, v in phases.items()}
    kernels = {k: v / args.steps for k, v in kernels.items()}
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
    tk = dict(kernels)
    tk.update({k: phases[k] for k in ("c4", "cliques") if k in phases})
    dom = max(tk, key=lambda k: tk[k])
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
        "kernels_ms": {k: round(v, 3) for k, v in kernels.items()},
        "dominant_kernel": dom,
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
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chunglu1m", choices=sorted(WORKLOADS))
    ap.add_argument("--schedule", default="mlp", choices=("id", "static", "mlp"),
                    help="order of sources in the per-source kernels")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched workload: 1024 workgroups, id schedule, no tuning runs")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the one-step run with the static schedule")
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

    for _ in range(args.warmup):
        counter.run(timing=True)
    torch.cuda.synchronize()
    phases, kernels, step_ms = {}, {}, []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        counter.run(timing=True)
        ph = orbit.last_phase_times()
        step_ms.append(sum(ms for _, ms in ph))
        for nm, ms in ph:
            phases[nm] = phases.get(nm, 0.0) + ms
        for nm, ms in orbit.last_kernel_times().items():
            kernels[nm] = kernels.get(nm, 0.0) + ms
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stats = orbit.last_stats()
    ms_step = 1000.0 * el / args.steps
    value = m * args.steps / el
    phases = {k: v / args.steps for k, v in phases.items()}
    kernels = {k: v / args.steps for k, v in kernels.items()}
    counts = counter.out[:n]
    sums, pats, hist = orbit.voc_summary(counts, 5)
    torch.cuda.synchronize()

    # The dominant kernel: the pair sweep (the undirected 2-hop sweep).
    # Algorithmic bytes per launch, the measurement unit of the 2-hop sweep:
    # 4 B per wedge endpoint, 8 B x sum over vertices of C(d,2) (the wedges
    # W); the diamond walk of its wheel maps (8 B x sum over edges of
    # C(T(e),2)) is reported beside it, not in `achieved`.  The time is
    # the kernel's own, from HIP events on the stream it runs on.
    dom_ms = kernels["pairs"]
    alg_bytes = 8.0 * stats["wedges"]
    achieved = alg_bytes / (dom_ms / 1000.0) / 1e9
    roofline = {"kernel": "k_pairs", "bound": "hbm", "achieved": round(achieved, 3),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                "traffic": measured_traffic(args.workload), "alg_bytes": alg_bytes,
                "alg_bytes_diamonds": 8.0 * stats["diamonds"], "avg_ms": round(dom_ms, 3)}
    # the 5-cycle kernel: 4 B per directed 3-path i <- j <- k -> l
    c5_bytes = 4.0 * stats["paths3"]
    c5_ach = c5_bytes / (kernels["c5"] / 1000.0) / 1e9
    roofline_c5 = {"kernel": "k_c5", "bound": "hbm", "achieved": round(c5_ach, 3),
                   "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(c5_ach / HBM_PEAK_GBS, 6),
                   "alg_bytes": c5_bytes, "avg_ms": round(kernels["c5"], 3)}

    compare = None
    if not args.no_compare and args.schedule != "static":
        # the plain static-threshold schedule on the same graph: the same
        # warm-up, the same number of steps, medians of the per-step GPU times
        k = min(args.steps, 5)
        del counter
        torch.cuda.empty_cache()
        cs = orbit.Counter(rp, ci, k_max=5, schedule="static")
        for _ in range(args.warmup):
            cs.run(timing=True)
        st = []
        for _ in range(k):
            cs.run(timing=True)
            st.append(sum(ms for _, ms in orbit.last_phase_times()))
        torch.cuda.synchronize()
        mine = step_ms[-k:]
        compare = {"schedule": "static", "steps": k,
                   "median_ms": round(float(np.median(st)), 3),
                   "min_max_ms": [round(min(st), 3), round(max(st), 3)],
                   args.schedule + "_median_ms": round(float(np.median(mine)), 3),
                   args.schedule + "_min_max_ms": [round(min(mine), 3), round(max(mine), 3)],
                   "speedup_of_" + args.schedule: round(float(np.median(st) / np.median(mine)), 4)}
        del cs

    voc = {"pattern_copies": {f"H{h}": str(pats[h]) for h in (2, 8, 9, 15, 29)},
           "ccd_orbit17": orbit.ccd(hist[17], n)[::4], "ccd_orbit70": orbit.ccd(hist[70], n)[::4]}

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
                   "schedule": args.schedule, "orbit_groups": "overlapped"},
        "roofline": roofline,
        "roofline_c5": roofline_c5,
        "phases_ms": {k: round(v, 3) for k, v in phases.items()},
        "kernels_ms": {k: round(v, 3) for k, v in kernels.items()},
        "step_gpu_ms_median": round(float(np.median(step_ms)), 3),
        "work": stats,
        "voc": voc,
    }
    if compare is not None:
        line["vs_static_schedule"] = compare
    if train_loss is not None:
        line["cost_model"] = {"trained_on": TRAIN_WORKLOAD, "mse_log2_steps": round(train_loss, 4)}
    if not args.no_cpu_baseline and rank == 0:
        line["cpu_baseline"] = cpu_baseline(rp, ci)
    if rank == 0:
        print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
