"""Benchmark: time-to-exact-OCM and edges/s per iteration on one MI355X.

A step is one complete exact solve (ocm_min / ocm_max through the C ABI):
validation, every policy-iteration phase until convergence, the critical
cycle listing and the tight-edge count, with the CSR already resident in HBM.
The default workload is the 16^6-state product graph (6 automata x 16 local
states, 125.8M edges).  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-exact-OCM & edges/s/iter at 16.7M states; batched/adjoint vs plain"
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_NAMES = {
    "sweep": "k_sweep_tile / k_tiescan_tile<SWEEP> (policy improvement)",
    "tiescan": "k_tiescan_tile (tight-edge count)",
    "cycles": "k_pj_init/round/final (policy-graph cycles)",
    "select": "k_cyc_zero/sum + k_select (minimum-mean cycle)",
    "conn_pull": "k_conn_init/pull (rebuild, pull rounds)",
    "conn_mark": "k_conn_mark (rebuild, push marks)",
    "conn_claim": "k_conn_claim (rebuild, push claims)",
    "reverse": "k_rev_hist/scatter/place (reverse CSR)",
    "values": "k_val_init/round/final (values after a rebuild)",
    "fast": "k_val_init/round/final (values, fast path)",
    "result": "k_cycle_list",
    "validate": "k_validate",
}


# the sources whose digest marks profiles as current (not moved by tests that
# point ROOT at a scratch directory)
SRC_ROOT = ROOT
# profile class -> the kernels whose counters give its traffic: the kernels
# the per-phase profile launches (the device-driven round loops use
# k_round_*, k_val_round_dev and k_pj_round_dev instead).  Each entry is
# (kernel, (template argument index, value) or None): the first sweep is
# k_sweep_tile, the later ones also count tight edges (k_tiescan_tile whose
# second template argument, SWEEP, is true).
KERNEL_SYMBOL = {
    "sweep": [("k_sweep_tile", None), ("k_tiescan_tile", (1, "true"))],
    "tiescan": [("k_tiescan_tile", (1, "false"))],
    "conn_mark": [("k_conn_mark", None)], "conn_claim": [("k_conn_claim", None)],
    "conn_pull": [("k_conn_pull", None)], "values": [("k_val_round", None)],
    "fast": [("k_val_round", None)], "cycles": [("k_pj_round_tagged", None)],
    "reverse": [("k_rev_place", None)],
}


def kernel_key(name):
    """Kernel name without return type, namespace and argument list
    ("k_conn_claim<2, false>")."""
    name = name.replace("void ", "").split("(")[0].strip()
    return name[len("ocm::"):] if name.startswith("ocm::") else name


def template_args(key):
    """Template arguments of a kernel key ("k_x<int, true, 0>" -> ["int", "true", "0"])."""
    if "<" not in key:
        return []
    return [a.strip() for a in key[key.index("<") + 1:key.rindex(">")].split(",")]


def class_kernels(table, cls):
    """Entries of a per-kernel table that belong to the class's kernel."""
    def match(k, base, arg):
        if k.split("<")[0] != base:
            return False
        if arg is None:
            return True
        a = template_args(k)
        return len(a) > arg[0] and a[arg[0]] == arg[1]
    return [v for k, v in table.items()
            if any(match(k, base, arg) for base, arg in KERNEL_SYMBOL.get(cls, []))]


# The sources the single-graph solve is built from (the batched, general and
# multichain files do not change its kernels).
DIGEST_FILES = ("include/ocm.h", "paper_1111_0627_amd/csrc/kernels.h",
                "paper_1111_0627_amd/csrc/device_util.h", "paper_1111_0627_amd/csrc/kernels.hip",
                "paper_1111_0627_amd/csrc/solver.hip", "paper_1111_0627_amd/csrc/batch.hip")


def source_digest():
    """sha256 over the single-graph solve's sources: counters and traces taken
    from another build of its kernels are not used."""
    import hashlib
    h = hashlib.sha256()
    for rel in DIGEST_FILES:
        with open(os.path.join(SRC_ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()


def pmc_file(workload):
    return os.path.join(ROOT, "profiles", f"pmc_{workload}.md")


def load_pmc(workload):
    """Per-kernel HBM counters (KiB per dispatch) and the copy calibration,
    from the JSON block of profiles/pmc_<workload>.md; None if absent or
    taken from other sources."""
    path = pmc_file(workload)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    try:
        blob = text.split("```json", 1)[1].split("```", 1)[0]
        d = json.loads(blob)
    except (IndexError, ValueError):
        return None
    if d.get("source_sha256") != source_digest():
        return None
    return d


def traffic_per_launch(pmc, cls):
    """Calibrated HBM bytes per launch of the class's kernel (averaged over
    its dispatches), or None."""
    if not pmc:
        return None
    ks = class_kernels(pmc["kernels"], cls)
    if not ks:
        return None
    cal = pmc["calibration"]
    d = sum(k["dispatches"] for k in ks)
    kib = sum(k["dispatches"] * (k["fetch_kib"] * cal["fetch_factor"] +
                                 k["write_kib"] * cal["write_factor"]) for k in ks)
    return 1024.0 * kib / d


def load_trace(workload):
    """Per-kernel calls and average duration from the JSON block of
    profiles/<workload>_kernel_trace.md; None if absent or from other sources."""
    path = os.path.join(ROOT, "profiles", f"{workload}_kernel_trace.md")
    if not os.path.exists(path):
        return None
    try:
        d = json.loads(open(path).read().split("```json", 1)[1].split("```", 1)[0])
    except (IndexError, ValueError):
        return None
    return d if d.get("source_sha256") == source_digest() else None


def trace_avg_us(trace, cls):
    """Average duration of the class's kernel in the committed rocprofv3 trace."""
    if not trace:
        return None
    ks = class_kernels(trace["kernels"], cls)
    calls = sum(k["calls"] for k in ks)
    return sum(k["total_ns"] for k in ks) / calls / 1e3 if calls else None


def summarize_trace(db, out, workload, command, note):
    """Writes profiles/<workload>_kernel_trace.md from a rocprofv3
    --kernel-trace database (rocpd SQLite)."""
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), sum(end - start) from kernels group by name").fetchall()
    con.close()
    per = {}
    for name, n, t in rows:
        k = kernel_key(name)
        a = per.setdefault(k, {"calls": 0, "total_ns": 0})
        a["calls"] += n
        a["total_ns"] += t
    tot = sum(v["total_ns"] for v in per.values())
    d = {"workload": workload, "source_sha256": source_digest(), "kernels": per}
    lines = [f"# Kernel trace: {workload}", "", "Command (from the repository root, on one MI355X):",
             "", "```", command, "```", "", note, "",
             "| Kernel | Calls | Total (ms) | Average (us) | Share (%) |", "|---|---:|---:|---:|---:|"]
    for k, v in sorted(per.items(), key=lambda kv: -kv[1]["total_ns"]):
        if v["total_ns"] < 0.001 * tot:
            continue
        lines.append(f"| `{k}` | {v['calls']} | {v['total_ns'] / 1e6:.3f} | "
                     f"{v['total_ns'] / v['calls'] / 1e3:.1f} | {100.0 * v['total_ns'] / tot:.2f} |")
    lines += ["", f"All kernels: {tot / 1e6:.3f} ms. Kernels under 0.1 % of it are left out of the "
              "table (not of the JSON block).", "", "```json", json.dumps(d, indent=1), "```", ""]
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        f.write("\n".join(lines))


def summarize_pmc(fetch_dir, write_dir, out, workload, calib_mb, command):
    """Writes profiles/pmc_<workload>.md from two rocprofv3 --pmc csv runs
    (FETCH_SIZE, then WRITE_SIZE), each holding a device copy of calib_mb MiB."""
    import csv
    import glob

    def load(d, counter):
        per = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                name = r["Kernel_Name"]
                key = "copy" if "copyBuffer" in name else kernel_key(name)
                per.setdefault(key, []).append(float(r["Counter_Value"]))
        return per

    fe, wr = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    copy_kib = calib_mb * 1024.0
    cal = {"copy_bytes": calib_mb << 20, "fetch_kib": max(fe["copy"]), "write_kib": max(wr["copy"])}
    cal["fetch_factor"] = copy_kib / cal["fetch_kib"]
    cal["write_factor"] = copy_kib / cal["write_kib"]
    kernels = {}
    for k in sorted(set(fe) & set(wr)):
        if k == "copy":
            continue
        kernels[k] = {"dispatches": len(fe[k]), "fetch_kib": sum(fe[k]) / len(fe[k]),
                      "write_kib": sum(wr[k]) / len(wr[k])}
    d = {"workload": workload, "source_sha256": source_digest(), "calibration": cal,
         "kernels": kernels}
    lines = [f"# HBM counters per dispatch: {workload}", "",
             "Two `rocprofv3 --pmc` passes over the same run (`FETCH_SIZE`, then `WRITE_SIZE`).",
             f"Each run first copies {calib_mb} MiB on the device; that copy calibrates the counters "
             f"(fetch x{cal['fetch_factor']:.3f}, write x{cal['write_factor']:.3f}).", "",
             "Command (one pass per counter):", "", "```", command, "```", "",
             "| Kernel | Dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | Calibrated MB per dispatch |",
             "|---|---:|---:|---:|---:|"]
    for k, v in kernels.items():
        mb = (v["fetch_kib"] * cal["fetch_factor"] + v["write_kib"] * cal["write_factor"]) / 1024
        lines.append(f"| `{k}` | {v['dispatches']} | {v['fetch_kib']:.0f} | {v['write_kib']:.0f} "
                     f"| {mb:.1f} |")
    lines += ["", "```json", json.dumps(d, indent=1), "```", ""]
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        f.write("\n".join(lines))


def summarize_l2(pmc_dir, out, workload, command):
    """Writes profiles/<workload>_l2_hits.md from a rocprofv3 --pmc
    TCC_HIT_sum TCC_MISS_sum csv run: L2 requests, hit rate and missed lines
    per launch of every kernel."""
    import csv
    import glob
    per = {}
    for f in glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] not in ("TCC_HIT_sum", "TCC_MISS_sum"):
                continue
            k = kernel_key(r["Kernel_Name"])
            a = per.setdefault(k, {"TCC_HIT_sum": [], "TCC_MISS_sum": []})
            a[r["Counter_Name"]].append(float(r["Counter_Value"]))
    rows = []
    for k, v in per.items():
        if not v["TCC_HIT_sum"] or not v["TCC_MISS_sum"]:
            continue
        n = len(v["TCC_HIT_sum"])
        hit = sum(v["TCC_HIT_sum"]) / n
        miss = sum(v["TCC_MISS_sum"]) / len(v["TCC_MISS_sum"])
        rows.append((k, n, hit + miss, hit / (hit + miss) if hit + miss else 0.0, miss * 128 / 1e6))
    rows.sort(key=lambda r: -r[2])
    d = {"workload": workload, "source_sha256": source_digest(),
         "kernels": {r[0]: {"launches": r[1], "requests": r[2], "hit_rate": r[3],
                            "miss_mb": r[4]} for r in rows}}
    lines = [f"# L2 hits and misses per launch, {workload}", "",
             "Command (from the repository root):", "", "```", command, "```", "",
             "L2 requests are counted after the wave's own coalescing (lanes that read one line make "
             "one request). A miss, read or write, moves a 128-byte line.", "",
             "| Kernel | Launches | L2 requests per launch | Hit rate | Misses × 128 B per launch |",
             "|---|---:|---:|---:|---:|"]
    for k, n, req, hr, mb in rows:
        if req < 1e5:
            continue
        lines.append(f"| `{k}` | {n} | {req / 1e6:.2f}M | {hr:.3f} | {mb:.0f} MB |")
    lines += ["", "```json", json.dumps(d, indent=1), "```", ""]
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        f.write("\n".join(lines))


def with_traffic(rf, traffic):
    """Adds the counter-measured HBM bytes per launch and the rate they move
    at (traffic over the live average launch time) beside the algorithmic
    figures."""
    rf["traffic"] = traffic
    if traffic:
        gbs = traffic / (rf["avg_launch_us"] / 1e6) / 1e9
        rf["traffic_gbs"] = gbs
        rf["traffic_frac"] = gbs / PEAK_HBM_GBS
    return rf


def roofline(cls, ms, launches, nbytes):
    """HBM roofline of one kernel class from the library's live hipEvent
    timings and its algorithmic bytes (both summed over the timed steps)."""
    gbs = nbytes / (ms / 1e3) / 1e9 if ms > 0 else 0.0
    return {"kernel": KERNEL_NAMES.get(cls, cls), "bound": "hbm", "achieved": gbs,
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
            "traffic": None, "bytes_per_launch": nbytes / max(launches, 1),
            "avg_launch_us": ms * 1e3 / max(launches, 1)}


def host_cpu():
    """The host's CPU model and logical core count (the oracle uses one)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def cpu_baseline(g, mode, budget_s=30.0):
    """The C oracle (one thread) on the same workload: a full sequential
    policy-iteration solve; edges/s/iter = m * iterations / time."""
    from oracle import native
    t = time.perf_counter()
    sol = native.solve(g.row_ptr, g.col, g.w, mode=mode, tie=False)
    dt = time.perf_counter() - t
    return dict(value=g.m * sol.iterations / dt, unit="edges/s", cores=1, kind="oracle",
                sample=f"one full sequential policy-iteration solve of the same workload "
                       f"({sol.iterations} iterations, {dt:.1f} s, single thread)",
                seconds=round(dt, 2), iterations=sol.iterations, p=sol.p, q=sol.q,
                host=host_cpu())


def cpu_sample(g, mode, budget_s=10.0):
    """The oracle's policy iteration, phase by phase, until it converges or
    the budget is spent (whole iterations): edges/s/iter over what ran."""
    from oracle import native
    st = native.Stepper(g.row_ptr, g.col, g.w, mode=mode)
    t0 = time.perf_counter()
    it, done = 0, False
    while time.perf_counter() - t0 < budget_s:
        ch = st.sweep()
        it += 1
        if it >= 2 and ch == 0:
            done = True
            break
        st.cycles()
        st.select()
        st.connect()
        st.values()
    dt = time.perf_counter() - t0
    return dict(value=g.m * it / dt, unit="edges/s", cores=1, kind="oracle",
                sample=(f"full sequential solve ({it} iterations)" if done else
                        f"the first {it} iterations of the sequential solve (time budget)"),
                seconds=round(dt, 2), iterations_run=it, converged=done)


def bench_multichain(rp, cl, w, mode, steps, ref):
    """The multichain variant (every policy cycle keeps its own gain, no
    rebuild) on the same resident graph: median time to the exact optimum,
    its sweep count, and whether it reaches the same optimum as Alg. 2."""
    from paper_1111_0627_amd import ocm
    import torch
    r = ocm.cycle_mean(rp, cl, w, mode=mode, multichain=True)
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        t = time.perf_counter()
        r = ocm.cycle_mean(rp, cl, w, mode=mode, multichain=True)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1e3)
    return {"time_to_exact_ocm_ms": {"median": float(np.median(ts)), "min": min(ts)},
            "iterations": r.iterations, "jump_rounds": r.jump_rounds,
            "same_optimum": (r.p, r.q) == (ref.p, ref.q)}


def bench_config(name, steps):
    """One single-graph workload: time-to-exact-OCM (median of `steps` after a
    warm-up), iterations, edges/s/iter, the sweep's HBM roofline, and the
    oracle on the host (bounded sample; Karp on the small random graph)."""
    from oracle import native
    from paper_1111_0627_amd import ocm, synth
    import torch
    mode = synth.WORKLOADS[name]["mode"]
    g = synth.workload(name)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    cl = torch.from_numpy(g.col).to(dev)
    w = torch.from_numpy(g.w).to(dev)
    r = ocm.cycle_mean(rp, cl, w, mode=mode)
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        t = time.perf_counter()
        r2 = ocm.cycle_mean(rp, cl, w, mode=mode)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1e3)
        assert (r2.p, r2.q, r2.iterations) == (r.p, r.q, r.iterations)
    med = float(np.median(ts))
    phase = {}
    for _ in range(max(1, steps // 2)):
        rp_ = ocm.cycle_mean(rp, cl, w, mode=mode, profile=True)
        for k, (pms, cnt, nbytes) in rp_.profile.items():
            a = phase.setdefault(k, [0.0, 0, 0.0])
            a[0] += pms
            a[1] += cnt
            a[2] += nbytes
    out = {"n": g.n, "m": g.m, "mode": mode, "iterations": r.iterations,
           "p": r.p, "q": r.q, "cycle_len": r.L, "fast_iters": r.fast_iters,
           "time_to_exact_ocm_ms": {"median": med, "min": min(ts)},
           "edges_per_s_per_iter": g.m * r.iterations / (med / 1e3),
           "roofline_sweep": roofline("sweep", *phase["sweep"])}
    with_traffic(out["roofline_sweep"], traffic_per_launch(load_pmc(name), "sweep"))
    gold = os.path.join(ROOT, "tests", "golden", "workloads.json")
    if os.path.exists(gold):
        with open(gold) as f:
            ex = json.load(f).get(name)
        if ex:
            out["matches_oracle_golden"] = (r.p, r.q, r.cycle_edges.cpu().tolist(), r.iterations) \
                == (ex["p"], ex["q"], ex["cycle"], ex["iterations"])
    out["multichain"] = bench_multichain(rp, cl, w, mode, min(steps, 3), r)
    cb = cpu_sample(g, mode)
    if name == "rand1k":
        t = time.perf_counter()
        kv = native.karp(g.row_ptr, g.col, g.w)
        cb["karp_seconds"] = round(time.perf_counter() - t, 4)
        cb["karp_agrees"] = kv == r.value
    out["cpu_oracle"] = cb
    return out


def batched_cpu_sample(gs, budget_s=12.0):
    """The oracle over a spread sample of the batch's graphs (every k-th),
    scaled to the whole batch by edges x iterations."""
    from oracle import native
    G = len(gs)
    t0 = time.perf_counter()
    done, em = 0, 0
    for k in list(range(0, G, 16)) + list(range(8, G, 16)):
        if time.perf_counter() - t0 > budget_s:
            break
        s = native.solve(gs[k].row_ptr, gs[k].col, gs[k].w, tie=False)
        em += gs[k].m * s.iterations
        done += 1
    dt = time.perf_counter() - t0
    return {"graphs_sampled": done, "seconds": round(dt, 2), "value": em / dt,
            "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"sequential solves of {done} of {G} graphs (every 16th first)"}


def bench_batched(steps: int, full: bool = True):
    """The batched workload: 4,096 random digraphs solved in one batched call
    (ocm_min_batched), against 4,096 sequential single-graph GPU calls.
    full=False (a kernel trace of the batched solves): a cold call and the
    timed ones only."""
    import torch
    from paper_1111_0627_amd import ocm, synth
    t = time.time()
    gs = synth.batch_graphs()
    u, vptr, eptr = synth.disjoint_union(gs)
    log(f"[bench] batch4096: G={len(gs)} N={u.n} M={u.m} generated in {time.time() - t:.1f}s")
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(u.row_ptr).to(dev)
    cl = torch.from_numpy(u.col).to(dev)
    w = torch.from_numpy(u.w).to(dev)
    res = ocm.cycle_mean_batched(rp, cl, w, vptr, eptr)      # cold call
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        t = time.perf_counter()
        r = ocm.cycle_mean_batched(rp, cl, w, vptr, eptr)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t) * 1e3)
    assert (r.p, r.q, r.iterations) == (res.p, res.q, res.iterations)
    if not full:
        return {"workload": "batch4096", "graphs": len(gs), "vertices": u.n, "edges": u.m,
                "steps": steps, "batched_ms": {"median": float(np.median(times)), "min": min(times)}}
    # the same graphs, one plain call each (graphs already resident)
    rps = [rp[int(vptr[k]):int(vptr[k + 1]) + 1] - int(eptr[k]) for k in range(len(gs))]
    plain_ms = 0.0
    agree = 0
    cyc_all = r.cycle_edges.cpu().numpy()
    for k in range(len(gs)):
        e0, e1, v0, v1 = int(eptr[k]), int(eptr[k + 1]), int(vptr[k]), int(vptr[k + 1])
        rk = rps[k].contiguous()
        ck = (cl[e0:e1] - v0).contiguous()
        wk = w[e0:e1]
        torch.cuda.synchronize()
        t = time.perf_counter()
        x = ocm.min_cycle_mean(rk, ck, wk)
        torch.cuda.synchronize()
        plain_ms += (time.perf_counter() - t) * 1e3
        cyc = (cyc_all[r.cycle_ptr[k]:r.cycle_ptr[k + 1]] - int(eptr[k])).tolist()
        agree += (x.p, x.q, x.iterations, x.cycle_edges.cpu().tolist(), x.tie) == \
            (r.p[k], r.q[k], r.iterations[k], cyc, r.tie(k))
    its = np.array(r.iterations)
    med = float(np.median(times))
    gold_ok = None
    gold = os.path.join(ROOT, "tests", "golden", "batch4096.json")
    if os.path.exists(gold):
        with open(gold) as f:
            per = json.load(f)["per_graph"]
        gold_ok = sum(int((r.p[k], r.q[k], r.iterations[k],
                           (cyc_all[r.cycle_ptr[k]:r.cycle_ptr[k + 1]] - int(eptr[k])).tolist(),
                           r.tie(k)) == (e["p"], e["q"], e["iterations"], e["cycle"],
                                         bool(e["tie"])))
                      for k, e in enumerate(per))
    return {"workload": "batch4096", "graphs": len(gs), "vertices": u.n, "edges": u.m,
            "batched_ms": {"median": med, "min": min(times)},
            "plain_calls_total_ms": plain_ms, "speedup_vs_plain_calls": plain_ms / med,
            "graphs_agreeing_with_plain": agree,
            "graphs_matching_oracle_golden": gold_ok,
            "ties_unchecked": int(sum(1 for f in r.flags if f & 2)),
            "iterations": {"min": int(its.min()), "median": float(np.median(its)),
                           "max": int(its.max()), "sum": int(its.sum())},
            "edges_per_s_per_iter": float(sum(g.m * i for g, i in zip(gs, r.iterations)) / (med / 1e3)),
            "cpu_oracle": batched_cpu_sample(gs)}


def bench_small_class(steps: int):
    """Many small graphs (16,384 random digraphs, n log-uniform in [64, 2048],
    deg 1-8 + ring): the batched call with its small-graph class (one graph
    per workgroup in LDS) against the same call with every graph sent
    through the batched loop (OCM_BATCH_SMALL=0, identical results)."""
    import torch
    from paper_1111_0627_amd import ocm, synth
    gs = synth.batch_graphs(G=16384, lo=64, hi=2048, seed=7)
    u, vptr, eptr = synth.disjoint_union(gs)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(u.row_ptr).to(dev)
    cl = torch.from_numpy(u.col).to(dev)
    w = torch.from_numpy(u.w).to(dev)
    out = {"workload": "16384 random digraphs, n log-uniform in [64, 2048], deg 1-8 + ring, "
                       "w int32 in [1,10000]", "graphs": len(gs), "vertices": u.n, "edges": u.m}
    res = {}
    old = os.environ.get("OCM_BATCH_SMALL")
    try:
        for key, flag in (("small_class", "1"), ("loop_only", "0")):
            os.environ["OCM_BATCH_SMALL"] = flag
            r = ocm.cycle_mean_batched(rp, cl, w, vptr, eptr)
            torch.cuda.synchronize()
            ts = []
            for _ in range(steps):
                t = time.perf_counter()
                r = ocm.cycle_mean_batched(rp, cl, w, vptr, eptr)
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t) * 1e3)
            res[key] = r
            out[key + "_ms"] = {"median": float(np.median(ts)), "min": min(ts)}
    finally:
        if old is None:
            os.environ.pop("OCM_BATCH_SMALL", None)
        else:
            os.environ["OCM_BATCH_SMALL"] = old
    a, b = res["small_class"], res["loop_only"]
    out["identical"] = (a.p, a.q, a.iterations, a.cycle_ptr, a.flags, a.status) == \
        (b.p, b.q, b.iterations, b.cycle_ptr, b.flags, b.status) and \
        bool(torch.equal(a.cycle_edges, b.cycle_edges))
    out["speedup"] = out["loop_only_ms"]["median"] / out["small_class_ms"]["median"]
    return out


def bench_adjoint(n_fd: int):
    """The adjoint workload: n = 2^22 random digraph with int64 weights;
    forward through the autograd Function, backward (adjoint scatter), and the
    exact unit finite-difference check on a stratified edge sample."""
    import torch
    from paper_1111_0627_amd import autograd, gradcheck, ocm, synth
    g = synth.workload("rand4m_i64")
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    cl = torch.from_numpy(g.col).to(dev)
    wi = torch.from_numpy(g.w).to(dev)
    wf = wi.to(torch.float64)
    base = ocm.min_cycle_mean(rp, cl, wi, want_policy=True)
    torch.cuda.synchronize()

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t) * 1e3)
        return float(np.median(ts))

    plain = timed(lambda: ocm.min_cycle_mean(rp, cl, wi))

    def fwd_bwd():
        x = wf.clone().requires_grad_(True)
        v = autograd.cycle_mean(x, rp, cl)
        v.backward()
        return x.grad

    def fwd_only():
        with torch.no_grad():
            return autograd.cycle_mean(wf, rp, cl)

    fwd = timed(fwd_only)
    fb = timed(fwd_bwd)
    gout = torch.ones((), dtype=torch.float64, device=dev)
    scat = timed(lambda: ocm.adjoint_scatter(g.m, base.cycle_edges, gout), reps=20)
    grad = fwd_bwd()
    exp = torch.zeros(g.m, dtype=torch.float64, device=dev)
    exp[base.cycle_edges.long()] = 1.0 / len(base.cycle_edges)
    edges = gradcheck.stratified_edges(base.cycle_edges.cpu().numpy(), g.row_ptr, g.m, total=n_fd)
    t = time.perf_counter()
    rep = gradcheck.fd_check(rp, cl, wi, edges, base=base, w_host=g.w)
    fd_s = time.perf_counter() - t
    return {"workload": "rand4m_i64", "n": g.n, "m": g.m, "cycle_len": len(base.cycle_edges),
            "tie": base.tie, "plain_forward_ms": plain, "autograd_forward_ms": fwd,
            "forward_backward_ms": fb, "adjoint_scatter_ms": scat,
            "grad_matches_1_over_C": bool(torch.equal(grad, exp)),
            "fd": {**rep.as_dict(), "edges": len(edges), "seconds": round(fd_s, 2),
                   "note": "each perturbed solve warm-started from the base policy; "
                           "its final no-improvement sweep certifies it"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="product16x6",
                    help="a single-graph workload, or batch4096: the batched solves alone")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-multichain", action="store_true",
                    help="skip the multichain variant's timing on the headline workload")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other single-graph workloads (rand1k, rand1m_max, rand4m_i64, "
                         "hub1m)")
    ap.add_argument("--fd-edges", type=int, default=1000)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before timing, copy one buffer of this many MiB (a plain copy "
                         "kernel of known size, to calibrate HBM byte counters)")
    ap.add_argument("--pmc-summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/pmc_<workload>.md from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--pmc-command", default="", help="command line recorded with --pmc-summarize")
    ap.add_argument("--trace-summarize", metavar="DB",
                    help="write profiles/<workload>_kernel_trace.md from a rocprofv3 "
                         "--kernel-trace database and exit")
    ap.add_argument("--trace-command", default="", help="command line recorded with --trace-summarize")
    ap.add_argument("--l2-summarize", metavar="PMC_DIR",
                    help="write profiles/<workload>_l2_hits.md from a rocprofv3 --pmc "
                         "TCC_HIT_sum TCC_MISS_sum run and exit")
    ap.add_argument("--l2-command", default="", help="command line recorded with --l2-summarize")
    ap.add_argument("--trace-note", default="", help="what the traced run did")
    args = ap.parse_args()
    if args.pmc_summarize:
        summarize_pmc(args.pmc_summarize[0], args.pmc_summarize[1], pmc_file(args.workload),
                      args.workload, args.calib_copy_mb or 1024, args.pmc_command)
        return
    if args.l2_summarize:
        summarize_l2(args.l2_summarize,
                     os.path.join(ROOT, "profiles", f"{args.workload}_l2_hits.md"),
                     args.workload, args.l2_command)
        return
    if args.trace_summarize:
        summarize_trace(args.trace_summarize,
                        os.path.join(ROOT, "profiles", f"{args.workload}_kernel_trace.md"),
                        args.workload, args.trace_command, args.trace_note)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_1111_0627_amd import ocm, synth

    name = args.workload
    if name == "batch4096":   # the batched solves alone (for a kernel trace)
        print(json.dumps(bench_batched(max(1, args.steps), full=False)), flush=True)
        return
    mode = synth.WORKLOADS[name]["mode"]
    t = time.time()
    g = synth.workload(name)
    log(f"[bench] {name}: n={g.n} m={g.m} generated in {time.time() - t:.1f}s")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rp = torch.from_numpy(g.row_ptr).to(dev)
    cl = torch.from_numpy(g.col).to(dev)
    w = torch.from_numpy(g.w).to(dev)
    sw = g.w.dtype.itemsize
    torch.cuda.synchronize()

    if args.calib_copy_mb > 0:
        nb = args.calib_copy_mb << 20
        src = torch.ones(nb // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calib_copy_mb} MiB done")
        del src, dst

    def step(profile):
        return ocm.cycle_mean(rp, cl, w, mode=mode, profile=profile)

    # cold first call (includes workspace allocation)
    t = time.perf_counter()
    res = step(False)
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - t) * 1e3
    log(f"[bench] cold solve {cold_ms:.1f} ms: {res.p}/{res.q} iters={res.iterations} "
        f"|C|={res.L} fast={res.fast_iters}")
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()

    # timed region: K full solves, nothing else on the stream
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(st)
    per_step = []
    results = set()
    for _ in range(args.steps):
        ts = time.perf_counter()
        r = step(False)
        per_step.append((time.perf_counter() - ts) * 1e3)
        results.add((r.p, r.q, r.iterations, r.source, r.L))
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    ms = wall * 1e3 / args.steps

    # the same K solves again with the library's per-launch hipEvents on the
    # solve's stream: per-phase time, launches and algorithmic bytes
    phase = {}
    if not args.no_profile:
        for _ in range(args.steps):
            rp_ = step(True)
            results.add((rp_.p, rp_.q, rp_.iterations, rp_.source, rp_.L))
            for k, (pms, cnt, nbytes) in rp_.profile.items():
                a = phase.setdefault(k, [0.0, 0, 0.0])
                a[0] += pms
                a[1] += cnt
                a[2] += nbytes
    assert len(results) == 1, "solves disagree between steps"
    iters = r.iterations
    value = g.m * iters / (ms / 1e3)

    out = {
        "metric": METRIC, "value": value, "unit": "edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": name, "desc": synth.WORKLOADS[name]["desc"], "n": g.n, "m": g.m,
                   "mode": mode, "iterations": iters, "parallelism": "single GPU"},
        "time_to_exact_ocm_ms": {"median": float(np.median(per_step)), "min": min(per_step),
                                 "cold": cold_ms, "events_total": ev_ms},
        "result": {"p": r.p, "q": r.q, "cycle_len": r.L, "source": r.source,
                   "tight_edges": r.tight_edges, "fast_iters": r.fast_iters,
                   "jump_rounds": r.jump_rounds, "connect_rounds": r.connect_rounds,
                   **r.counters},
    }
    if phase:
        K = args.steps
        out["phase_ms_per_step"] = {k: v[0] / K for k, v in phase.items() if v[1]}
        out["phase_launches_per_step"] = {k: v[1] / K for k, v in phase.items() if v[1]}
        out["phase_gbs"] = {k: v[2] / (v[0] / 1e3) / 1e9 for k, v in phase.items() if v[1] and v[0] > 0}
        dom = max((k for k, v in phase.items() if v[1]), key=lambda k: phase[k][0])
        pmc, trace = load_pmc(name), load_trace(name)
        out["roofline"] = roofline(dom, *phase[dom])
        out["roofline"]["class"] = dom
        with_traffic(out["roofline"], traffic_per_launch(pmc, dom))
        out["roofline"]["trace_avg_launch_us"] = trace_avg_us(trace, dom)
        out["roofline_sweep"] = roofline("sweep", *phase["sweep"])
        with_traffic(out["roofline_sweep"], traffic_per_launch(pmc, "sweep"))
        out["roofline_sweep"]["trace_avg_launch_us"] = trace_avg_us(trace, "sweep")
    if not args.no_multichain:
        log("[bench] multichain variant ...")
        out["multichain"] = bench_multichain(rp, cl, w, mode, args.steps, r)
    if not args.no_configs:
        out["configs"] = {}
        for cname in ("rand1k", "rand1m_max", "rand4m_i64", "hub1m"):
            if cname == name:
                continue
            log(f"[bench] workload {cname} ...")
            out["configs"][cname] = bench_config(cname, max(args.steps, 10))
    if not args.no_adjoint:
        log("[bench] adjoint workload ...")
        out["adjoint"] = bench_adjoint(args.fd_edges)
    if not args.no_batched:
        log("[bench] batched workload ...")
        out["batched"] = bench_batched(max(2, min(args.steps, 5)))
        log("[bench] many small graphs ...")
        out["batched_small"] = bench_small_class(max(2, min(args.steps, 5)))
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle ...")
        cb = cpu_baseline(g, mode)
        cb["agrees_with_gpu"] = (cb["p"], cb["q"], cb["iterations"]) == (r.p, r.q, r.iterations)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
