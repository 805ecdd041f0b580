"""Benchmark of the RAC fixpoint on one MI355X.

A step is one enforcement of the whole hot path over one batch of synthetic
input already resident in HBM. The default workload is the batched-state
configuration: one model-B network (n=1000, d=32, p1=0.8, p2=0.25) and 1024
domain states, each a random partial assignment of 0..20 variables; every
state is run to its arc-consistency fixpoint in one call of
rac_enforce_batch_device (matrix-core path chosen by the autotuner).

Printed (one JSON line): support checks/s of the batched call (value),
fixpoints/s, the same states through the plain per-state loop (1024
sequential rac_enforce calls, each with its own host round trip), the
roofline of the dominant kernel (HIP events around each of its launches),
the CPU oracle timed on a bounded sample of the same states, and secondary
single-instance measurements.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
INT8_PEAK_TOPS = 5000.0        # MI355X dense int8 matrix-core peak, TOP/s

PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "traffic.json")
CSRC = os.path.join(ROOT, "paper_2407_11388_amd", "csrc")


# Sources whose change invalidates the recorded traffic of a kernel.
KERNEL_SOURCES = {"mfma_sweep_kernel": ["mfma.hip", "rac_mfma.h"],
                  "revise_kernel": ["sweep.hip", "rac_internal.h", "rac_host.hip"]}


def _code_only(src: str) -> str:
    """C/C++ source without comments and with whitespace runs collapsed, so
    that a change of comments or layout keeps a kernel's digest."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_digest(kernel: str, read=None) -> str:
    """sha256 over a kernel's sources (code only: comments and whitespace
    runs do not count); measured traffic is only reported while it matches
    the digest recorded with the counters."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        if read is None:
            with open(os.path.join(CSRC, name), encoding="utf-8") as f:
                text = f.read()
        else:
            text = read(name)
        h.update(name.encode() + b"\0" + _code_only(text).encode())
    return h.hexdigest()


def recorded_traffic(name: str):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) of profile
    entry `name`, or None if absent or taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            e = json.load(f)[name]
    except (OSError, KeyError, ValueError):
        return None
    if e.get("sha256") != kernel_digest(e["kernel"]):
        return None
    return e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]


def profile_report(args):
    """Summarises rocprofv3 output (kernel-trace stats plus FETCH_SIZE and
    WRITE_SIZE runs, and the same two counters for a 1 GiB copy) into
    profiles/<name>.txt and the traffic table. CPU only."""
    import csv
    from collections import defaultdict
    name, kernel, trace_dir, fdir, wdir, cfdir, cwdir = args.profile_report

    def counters(d):
        out = defaultdict(list)
        for fn in os.listdir(d):
            if fn.endswith("counter_collection.csv"):
                with open(os.path.join(d, fn)) as f:
                    for r in csv.DictReader(f):
                        out[r["Kernel_Name"].split("(")[0].split("::")[-1]].append(
                            float(r["Counter_Value"]))
        return out

    def stats(d):
        for fn in os.listdir(d):
            if fn.endswith("kernel_stats.csv"):
                with open(os.path.join(d, fn)) as f:
                    return list(csv.DictReader(f))
        return []

    cf, cw = counters(cfdir), counters(cwdir)
    copy_kib = args.copy_bytes / 1024.0
    fscale = copy_kib / cf["__amd_rocclr_copyBuffer"][0]
    wscale = copy_kib / cw["__amd_rocclr_copyBuffer"][0]
    fv, wv = counters(fdir)[kernel], counters(wdir)[kernel]
    top = max(fv)
    if args.profile_top > 0:
        # the N launches that read the most (e.g. the step-1 launch of each of N calls)
        work = sorted(sorted(range(len(fv)), key=lambda i: -fv[i])[:args.profile_top])
    else:
        work = [i for i, v in enumerate(fv) if v > 0.01 * top]   # launches that had work
    fb = sum(fv[i] for i in work) / len(work) * 1024 * fscale
    wb = sum(wv[i] for i in work) / len(work) * 1024 * wscale
    rows = stats(trace_dir)
    lines = [f"# {name}: rocprofv3 summary of {kernel}", ""]
    lines += ["Commands (from the repository root; rocprofv3 run with TMPDIR=/tmp):", ""]
    lines += [f"    {c}" for c in args.profile_command] + [""]
    lines += ["Kernel statistics (--kernel-trace --stats):", "",
              "| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in rows[:10]:
        lines.append(f"| {r['Name'].split('(')[0]} | {r['Calls']} | {float(r['AverageNs'])/1e3:.1f} | "
                     f"{float(r['MinNs'])/1e3:.1f} | {float(r['MaxNs'])/1e3:.1f} | "
                     f"{float(r['Percentage']):.1f} |")
    krow = next((r for r in rows if r["Name"].split("(")[0].endswith(kernel)), None)
    lines += ["", f"HBM traffic of {kernel} (--pmc FETCH_SIZE, then --pmc WRITE_SIZE):", "",
              f"* launches with work: {len(work)} of {len(fv)}",
              f"* FETCH_SIZE per launch: {sum(fv[i] for i in work)/len(work):.0f} KiB raw, x {fscale:.4f} = {fb/1e6:.1f} MB",
              f"* WRITE_SIZE per launch: {sum(wv[i] for i in work)/len(work):.0f} KiB raw, x {wscale:.4f} = {wb/1e6:.1f} MB",
              f"* calibration: a {args.copy_bytes} B device copy reads {cf['__amd_rocclr_copyBuffer'][0]:.0f} KiB "
              f"FETCH_SIZE and {cw['__amd_rocclr_copyBuffer'][0]:.0f} KiB WRITE_SIZE",
              ]
    if krow:
        lines.append(f"* average launch duration (all launches): {float(krow['AverageNs'])/1e3:.1f} us")
    durs = []
    for fn in os.listdir(trace_dir):
        if fn.endswith("kernel_trace.csv"):
            with open(os.path.join(trace_dir, fn)) as f:
                for r in csv.DictReader(f):
                    if r["Kernel_Name"].split("(")[0].endswith(kernel):
                        durs.append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    if args.profile_sq:
        # instruction and cycle counters of the same launches (one --pmc run)
        sq = defaultdict(list)
        for fn in os.listdir(args.profile_sq):
            if fn.endswith("counter_collection.csv"):
                with open(os.path.join(args.profile_sq, fn)) as f:
                    for r in csv.DictReader(f):
                        if r["Kernel_Name"].split("(")[0].endswith(kernel):
                            sq[r["Counter_Name"]].append(float(r["Counter_Value"]))
        if sq:
            lines += ["", f"Instruction counters of {kernel} (--pmc, per launch, median over "
                          f"{len(next(iter(sq.values())))} launches; SQ_INSTS_VALU also counts the "
                          "matrix-core instructions, in more than one unit each):", ""]
            med = {c: sorted(v)[len(v) // 2] for c, v in sq.items()}
            for c in sorted(med):
                lines.append(f"* {c}: {med[c]:.4g}")
            if med.get("SQ_INSTS_MFMA") and med.get("SQ_INSTS_LDS"):
                lines.append(f"* LDS instructions per matrix-core instruction: "
                             f"{med['SQ_INSTS_LDS'] / med['SQ_INSTS_MFMA']:.2f}")
    if durs and args.profile_top > 0:
        busy = sorted(durs)[-args.profile_top:]
        lines.append(f"* average duration of the {len(busy)} longest launches (of {len(durs)}; "
                     f"the launches the traffic above is taken from): {sum(busy) / len(busy) / 1e3:.1f} us")
    elif durs:
        busy = [t for t in durs if t > 0.1 * max(durs)]
        lines.append(f"* average duration of the launches with work ({len(busy)} of {len(durs)}, "
                     f"longer than 10% of the longest): {sum(busy) / len(busy) / 1e3:.1f} us")
    os.makedirs(PROFILES, exist_ok=True)
    with open(os.path.join(PROFILES, name + ".txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    table = {}
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            table = json.load(f)
    table[name] = dict(kernel=kernel, fetch_bytes_per_launch=fb, write_bytes_per_launch=wb,
                       fetch_scale=fscale, write_scale=wscale, launches=len(work),
                       sha256=kernel_digest(kernel))
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
        f.write("\n")
    print("\n".join(lines))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch-states",
                    choices=["batch-states", "uneven-multi", "single-large", "single-mid", "single-small"])
    ap.add_argument("--B", type=int, default=1024)
    ap.add_argument("--plain-states", type=int, default=1024,
                    help="states timed through the plain per-state loop")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--table1", action="store_true",
                    help="only run the Table 1-style MAC-search grid (steps and AC-3 revisions "
                         "per assignment, time per node) and print it as one JSON line")
    ap.add_argument("--table1-out", default="", metavar="PATH",
                    help="with --table1: also write the table as markdown to PATH")
    ap.add_argument("--search-only", action="store_true",
                    help="run only the two batched MAC searches (one JSON line)")
    ap.add_argument("--no-search", action="store_true",
                    help="skip the MAC-search lines in the secondary results")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the 256-instance uneven batch in the secondary results")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES (to calibrate the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--profile-report", nargs=7, default=None,
                    metavar=("NAME", "KERNEL", "TRACE_DIR", "FETCH_DIR", "WRITE_DIR",
                             "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="CPU only: summarise rocprofv3 output into profiles/NAME.txt and "
                         "profiles/traffic.json")
    ap.add_argument("--profile-command", action="append", default=[],
                    help="command line recorded in the profile summary (repeatable)")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--profile-sq", default="", metavar="DIR",
                    help="with --profile-report: a --pmc run of SQ instruction/cycle counters")
    ap.add_argument("--profile-top", type=int, default=0,
                    help="with --profile-report: take traffic and duration from the N launches "
                         "that read the most (0: every launch with work)")
    return ap.parse_args()


def copy_rate(dev, nbytes: int = 1 << 30, reps: int = 5) -> dict:
    """The box's achievable HBM rate: a device-to-device copy of nbytes
    (read plus write bytes per second, best of reps, HIP events), beside the
    8 TB/s specification the fractions are quoted against."""
    import torch
    src = torch.ones(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = 1e9
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    gbs = 2 * nbytes / (best * 1e-3) / 1e9
    del src, dst
    return dict(bytes=nbytes, ms=best, read_write_GBs=gbs, frac_of_spec=gbs / HBM_PEAK_GBS,
                note="torch copy_ on the current stream; read + write bytes")


def algo_row_bytes(inst, path: str = "bits") -> int:
    """Relation bytes a full sweep of one state must read, without layout
    padding: per arc, d rows of ceil(d/32) 32-bit words (bit rows; 8-byte rows
    for 32 < d <= 64), or d*d bytes (int8 rows)."""
    arcs = 2 * int(inst.m)
    if path == "int8":
        return arcs * inst.d * inst.d
    return arcs * inst.d * (4 if inst.d <= 32 else 8)


def host_cpu():
    """The host's CPU model and logical core count (from /proc/cpuinfo)."""
    model, count = "unknown", 0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    count += 1
                    model = line.split(":", 1)[1].strip()
    except OSError:
        pass
    return dict(model=model, logical_cores=count or (os.cpu_count() or 0))


def cpu_baseline_batch(inst, doms, budget_s):
    """The CPU oracle on the first states of the batch until the time budget
    is used (one thread): its Eq. (1) recurrence (the same steps and support
    checks as the GPU path) gives support checks/s and fixpoints/s; AC-3 is
    timed on the same states as well."""
    import oracle

    n, d = inst.n, inst.d
    rel = inst.rel_u8()
    t_rec = t_ac3 = 0.0
    checks = revisions = lookups = 0
    done = 0
    for s in range(doms.shape[0]):
        du8 = oracle.dom_masks_to_u8(doms[s], d)
        t0 = time.perf_counter()
        r = oracle.rac_sync(n, d, inst.edges, rel, du8)
        t_rec += time.perf_counter() - t0
        checks += r["checks"]
        t0 = time.perf_counter()
        _, _, rv, lk = oracle.ac3(n, d, inst.edges, rel, du8)
        t_ac3 += time.perf_counter() - t0
        revisions += rv
        lookups += lk
        done += 1
        if t_rec >= budget_s:
            break
    out = dict(value=checks / t_rec, unit="support checks/s", cores=1, kind="oracle",
               sample=f"oracle Eq. (1) recurrence on the first {done} of {doms.shape[0]} "
                      f"states, one thread, {t_rec:.1f} s",
               fixpoints_per_s=done / t_rec, ac3_fixpoints_per_s=done / t_ac3,
               ac3_revisions_per_state=revisions / max(done, 1),
               ac3_lookups_per_state=lookups / max(done, 1),
               rac_support_checks_per_state=checks / max(done, 1), host=host_cpu())
    # the same oracle on the following states from a pool of threads (the C
    # recurrence runs without the interpreter lock), for about a third of the
    # budget: all host cores (up to 16, the host share of one GPU)
    from concurrent.futures import ThreadPoolExecutor
    threads = max(1, min(16, os.cpu_count() or 1))
    start = done
    t0 = time.perf_counter()

    def one(si):
        du8 = oracle.dom_masks_to_u8(doms[si], d)
        return oracle.rac_sync(n, d, inst.edges, rel, du8)["checks"]

    pool_checks = pool_done = 0
    with ThreadPoolExecutor(max_workers=threads) as ex:
        si = start
        while si < doms.shape[0] and time.perf_counter() - t0 < budget_s / 3:
            chunk = list(range(si, min(doms.shape[0], si + threads)))
            pool_checks += sum(ex.map(one, chunk))
            pool_done += len(chunk)
            si += len(chunk)
    t_pool = time.perf_counter() - t0
    if pool_done:
        out["all_cores"] = dict(threads=threads, value=pool_checks / t_pool,
                                fixpoints_per_s=pool_done / t_pool,
                                sample=f"states {start}..{start + pool_done - 1}, {t_pool:.1f} s")
    return out


def cpu_baseline_single(inst, dom, budget_s):
    import oracle

    n, d = inst.n, inst.d
    rel = inst.rel_u8()
    du8 = oracle.dom_masks_to_u8(dom, d)
    t0 = time.perf_counter()
    reps = 0
    checks = 0
    while True:
        checks = oracle.rac_sync(n, d, inst.edges, rel, du8)["checks"]
        reps += 1
        if time.perf_counter() - t0 >= budget_s or reps >= 5:
            break
    t = (time.perf_counter() - t0) / reps
    t1 = time.perf_counter()
    _, _, revisions, lookups = oracle.ac3(n, d, inst.edges, rel, du8)
    t_ac3 = time.perf_counter() - t1
    return dict(value=checks / t, unit="support checks/s", cores=1, kind="oracle",
                sample=f"oracle Eq. (1) recurrence, one thread, {reps} run(s) of the instance",
                fixpoints_per_s=1.0 / t, ac3_fixpoints_per_s=1.0 / t_ac3,
                ac3_revisions=revisions, ac3_lookups=lookups, rac_support_checks=checks,
                host=host_cpu())


# Open nodes per search round in the bench lines: a sweep (512 .. 8192) on
# both search workloads gains up to 4096 (fewer rounds of the same tree) and
# little beyond.
SEARCH_BATCH = 4096


def search_lines(one_node: bool = True):
    """Batched MAC search (Algorithm 2) on two instances: every child of up to
    SEARCH_BATCH open nodes enforced together per round, against one node per
    round (one_node)."""
    import numpy as np

    from paper_2407_11388_amd import gen, rac
    out = {}
    qe, qr = gen.queens(11)
    mb = gen.model_b(110, 100, 10, 0.1, 0.4)
    for name, (n, d, edges, rel) in (
            ("mac-search queens-11 (all solutions)", (11, 11, qe, qr)),
            ("mac-search model-B n=100 d=10 p1=0.1 p2=0.4 (complete, unsatisfiable)",
             (100, 10, mb.edges, mb.rel_u8()))):
        net = rac.Net.from_u8(n, d, edges, rel)
        root = np.full(n, (1 << d) - 1, dtype=np.uint64)
        line = {}
        for b in (SEARCH_BATCH, 1) if one_node else (SEARCH_BATCH,):
            net.search(root, batch=b, max_nodes=2000 if b == 1 else 0)   # warm-up
            res = None
            for _ in range(3 if b == SEARCH_BATCH else 1):   # the fastest of 3 (batched)
                r, _ = net.search(root, batch=b, max_nodes=0 if b == SEARCH_BATCH else 20000)
                res = r if res is None or r.search_ms < res.search_ms else res
            line[f"batch{b}"] = dict(nodes=int(res.nodes), solutions=int(res.solutions),
                                     failures=int(res.failures), complete=int(res.complete),
                                     rounds=int(res.rounds), ms=res.search_ms,
                                     steps_per_node=res.sweeps / res.nodes,
                                     nodes_per_s=res.nodes / (res.search_ms * 1e-3))
        if one_node:
            line["batched_vs_one_node"] = (line[f"batch{SEARCH_BATCH}"]["nodes_per_s"]
                                           / line["batch1"]["nodes_per_s"])
        out[name] = line
        net.close()
    return out


TABLE1_N = (100, 250, 500, 750, 1000)
TABLE1_DENSITY = (0.1, 0.25, 0.5, 0.75, 1.0)
TABLE1_D, TABLE1_P2 = 10, 0.3


def table1_instance(n: int, p1: float):
    """The model-B instance of one Table 1 grid point (d = 10, p2 = 0.3: the
    paper gives neither its domain size nor its tightness)."""
    from paper_2407_11388_amd import gen
    return gen.model_b(1000 + n + int(round(100 * p1)), n, TABLE1_D, p1, TABLE1_P2)


def table1_grid(gpu_nodes: int = 20000, oracle_cells: float = 4e8):
    """Table 1 on the paper's grid (n in {100, 250, 500, 750, 1000} x density in
    {0.1, 0.25, 0.5, 0.75, 1.0}; its 25 instances are not published, so
    model-B stand-ins with d = 10, p2 = 0.3). Per grid point: the GPU MAC
    search from full domains (batch SEARCH_BATCH, up to `gpu_nodes` nodes,
    checked before each round): recurrence steps per enforcement (an
    enforcement follows every assignment: the paper's #Recurrence) and time
    per node; beside it the oracle's depth-first search on its first nodes
    (as many as take about `oracle_cells` relation-cell visits, between 5 and
    100), run from a pool of host threads: recurrence steps and AC-3
    revisions per enforcement (AC-3 from scratch at every node, an upper
    bound on the incremental AC-3 the paper times)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    import oracle.search as osearch
    from paper_2407_11388_amd import rac

    cells = [(n, p1) for n in TABLE1_N for p1 in TABLE1_DENSITY]

    def oracle_cell(cell):
        n, p1 = cell
        inst = table1_instance(n, p1)
        rel = inst.rel_u8()
        arcs = 2 * int(inst.edges.shape[0])
        nodes = int(max(5, min(100, oracle_cells / max(1, arcs * TABLE1_D * TABLE1_D))))
        t0 = time.perf_counter()
        o = osearch.mac_search(n, TABLE1_D, inst.edges, rel, np.ones((n, TABLE1_D), np.uint8),
                               stop_after=nodes)
        o_s = time.perf_counter() - t0
        return dict(kind="oracle", nodes=o["nodes"], complete=int(o["complete"]),
                    steps_per_node=o["steps"] / o["nodes"],
                    ac3_revisions_per_node=o["revisions"] / o["nodes"],
                    us_per_node=o_s * 1e6 / o["nodes"])

    pool = ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1))
    futs = {c: pool.submit(oracle_cell, c) for c in cells}
    rows = []
    for (n, p1) in cells:
        inst = table1_instance(n, p1)
        net = rac.Net.from_bits(n, TABLE1_D, inst.edges, inst.rel)
        root = np.full(n, (1 << TABLE1_D) - 1, dtype=np.uint64)
        net.search(root, batch=SEARCH_BATCH, max_nodes=2000)   # warm-up
        res, _ = net.search(root, batch=SEARCH_BATCH, max_nodes=gpu_nodes)
        net.close()
        rows.append(dict(
            n=n, p1=p1, d=TABLE1_D, p2=TABLE1_P2, edges=int(inst.edges.shape[0]),
            gpu=dict(nodes=int(res.nodes), complete=int(res.complete), solutions=int(res.solutions),
                     steps_per_node=res.sweeps / res.nodes,
                     us_per_node=res.search_ms * 1e3 / res.nodes)))
        print(f"[table1] n={n} p1={p1}: gpu {rows[-1]['gpu']}", file=sys.stderr, flush=True)
    for r in rows:
        r["cpu_baseline"] = futs[(r["n"], r["p1"])].result()
    pool.shutdown()
    return rows


def table1_markdown(rows, command: str) -> str:
    """Table 1 rows as a short markdown summary."""
    out = ["# Table 1 on the paper's grid: MAC search on model-B stand-ins (d = 10, p2 = 0.3)", "",
           "Command (from the repository root): `" + command + "`", "",
           "Steps = recurrence steps per enforcement (one enforcement per assignment: the paper's "
           "#Recurrence). GPU: batched search (4096 open nodes per round) from full domains, up to "
           "20,000 nodes. Oracle: its depth-first search on its first nodes, AC-3 from scratch at every "
           "node (revisions are an upper bound on an incremental AC-3's).", "",
           "| n | density | edges | GPU nodes | GPU steps / node | µs / node (GPU) | oracle nodes | "
           "oracle steps / node | AC-3 revisions / node | µs / node (oracle) |",
           "|---|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        g, c = r["gpu"], r["cpu_baseline"]
        out.append(f"| {r['n']} | {r['p1']} | {r['edges']} | {g['nodes']}"
                   f"{'' if g['complete'] else ' (capped)'} | {g['steps_per_node']:.3f} | "
                   f"{g['us_per_node']:.2f} | {c['nodes']}{'' if c['complete'] else ' (first)'} | "
                   f"{c['steps_per_node']:.3f} | {c['ac3_revisions_per_node']:.0f} | {c['us_per_node']:.0f} |")
    return "\n".join(out) + "\n"


def main():
    args = parse()
    if args.profile_report:
        profile_report(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the batched "
              "states and instances would shard across GPUs without communication, but the "
              "benchmark runs on, and reports, a single MI355X.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2407_11388_amd import rac
    from paper_2407_11388_amd.gen import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.table1:
        rows = table1_grid()
        print(json.dumps(dict(table1=rows)), flush=True)
        if args.table1_out:
            with open(args.table1_out, "w") as f:
                f.write(table1_markdown(rows, "python bench.py --table1 --table1-out "
                                              "profiles/table1_grid_modelb_d10_p03.md"))
        return
    if args.search_only:
        print(json.dumps(dict(search=search_lines(one_node=False))), flush=True)
        return
    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes=args.copy_calibration)), flush=True)
        return
    out = dict(metric="support checks/s + AC fixpoints/s, batched int8-MFMA vs plain, bit-exact",
               unit="support checks/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               higher_is_better=True, scaling="weak", vs_baseline=None,
               data="synthetic (seeded model-B random CSPs)")

    if args.workload == "batch-states":
        w = workloads.batch_states(B=args.B)
        inst, doms = w.instances[0], w.domains[0]
        B, n, d = doms.shape[0], inst.n, inst.d
        net = rac.Net.from_instance(inst, profile=True)
        d_in = torch.from_numpy(doms.view(np.int64)).to(dev)
        d_out = torch.empty_like(d_in)
        d_it = torch.empty(B, dtype=torch.int32, device=dev)
        d_st = torch.empty(B, dtype=torch.int32, device=dev)
        stream = torch.cuda.current_stream().cuda_stream

        def step():
            net.enforce_batch_device(d_in, d_out, d_it, d_st, stream)

        for _ in range(args.warmup):
            step()
        net.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kms, klaunch, ops = 0.0, 0, 0
        for _ in range(args.steps):
            step()
            net.sync()          # collects the step's per-launch kernel timings
            st = net.stats()
            kms += st.kernel_ms
            klaunch += st.kernel_launches
            ops += st.algo_ops
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        st = net.stats()
        checks = st.support_checks
        iters = d_it.cpu().numpy()
        status = d_st.cpu().numpy()
        path = rac.PATH_NAMES.get(st.path, str(st.path))

        # plain per-state loop: sequential rac_enforce calls on the same states
        P = min(args.plain_states, B)
        net_plain = rac.Net.from_instance(inst, path=rac.PATH_BITS)
        for s in range(min(8, P)):
            net_plain.enforce(doms[s])
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        for s in range(P):
            net_plain.enforce(doms[s])
        tp = (time.perf_counter() - tp0) / P
        net_plain.close()

        # end to end: the host-pointer call, PCIe copies of the domains included
        for _ in range(2):
            net.enforce_batch(doms)
        te0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            net.enforce_batch(doms)
        te = (time.perf_counter() - te0) / reps

        fix_s = B / t
        plain_fix_s = 1.0 / tp
        achieved = ops / (kms * 1e-3) / 1e12 if kms > 0 else None
        out.update(
            value=checks / t, ms_per_step=t * 1e3, dtype="i8",
            config=dict(workload="batch-states: model-B n=1000 d=32 p1=0.8 p2=0.25, "
                                 f"B={B} partial-assignment states (0..20 singletons)",
                        B=B, n=n, d=d, arcs=int(2 * inst.m), path=path,
                        tuned_from=rac.TUNE_SOURCES.get(st.tune_source, str(st.tune_source)),
                        mode="run-to-fixpoint"),
            fixpoints_per_s=fix_s,
            plain_loop=dict(fixpoints_per_s=plain_fix_s, states=P, path="bits",
                            note="sequential rac_enforce calls, host round trip each"),
            batched_vs_plain=fix_s / plain_fix_s,
            end_to_end=dict(ms_per_batch=te * 1e3, fixpoints_per_s=B / te,
                            note="rac_enforce_batch on host buffers: the "
                                 f"{B * n * 8 / 1e6:.0f} MB of domains copied in and out"),
            steps_hist=np.bincount(iters).tolist(), wiped_states=int(status.sum()),
            roofline=dict(kernel="mfma_sweep_kernel", bound="mfma", achieved=achieved,
                          peak=INT8_PEAK_TOPS, unit="TOP/s",
                          frac=(achieved / INT8_PEAK_TOPS) if achieved else None,
                          traffic=recorded_traffic("mfma_sweep_kernel_batch_states"),
                          launches=klaunch,
                          avg_launch_ms=kms / klaunch if klaunch else None,
                          per_unit="2*d*d int8 ops per (arc, active state, step)"),
        )
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline_batch(inst, doms, args.cpu_seconds)
        net.close()
    elif args.workload == "uneven-multi":
        wu = workloads.uneven_multi()
        nets = [rac.Net.from_instance(i, profile=True) for i in wu.instances]
        grp = rac.Group(nets, profile=True)
        flat = np.concatenate(wu.domains).view(np.int64)
        d_in = torch.from_numpy(flat).to(dev)
        d_dom = torch.empty_like(d_in)
        k = len(nets)
        d_it = torch.empty(k, dtype=torch.int32, device=dev)
        d_st = torch.empty(k, dtype=torch.int32, device=dev)
        stream = torch.cuda.current_stream().cuda_stream

        def step():
            d_dom.copy_(d_in)   # the group call works in place
            grp.enforce_device(d_dom, d_it, d_st, stream)
            grp.sync()

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k1, kall, dms = [], 0.0, 0.0
        for _ in range(args.steps):
            step()
            stg = grp.stats()
            k1.append(stg.first_kernel_ms)
            kall += stg.kernel_ms
            dms += stg.device_ms
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        it_u, st_u = d_it.cpu().numpy(), d_st.cpu().numpy()
        algo = sum(algo_row_bytes(i) for i in wu.instances)
        t1 = sum(k1) / len(k1) * 1e-3
        gbs1 = algo / t1 / 1e9
        out.update(value=stg.support_checks / t, ms_per_step=t * 1e3, dtype="u32/u64 bit rows",
                   config=dict(workload=wu.name + ": model-B n~U[20,800] d~U[4,64] "
                                                  "p1~U[0.1,1) p2~U[0.1,0.6)",
                               instances=k, path="bits", mode="run-to-fixpoint"),
                   fixpoints_per_s=k / t, device_ms=dms / args.steps,
                   revise_ms_all_steps=kall / args.steps,
                   steps_max=int(it_u.max()), steps_mean=float(it_u.mean()),
                   wiped_instances=int(st_u.sum()),
                   roofline=dict(kernel="revise_kernel", bound="hbm", achieved=gbs1,
                                 peak=HBM_PEAK_GBS, unit="GB/s", frac=gbs1 / HBM_PEAK_GBS,
                                 traffic=recorded_traffic("revise_kernel_uneven_multi"),
                                 algorithmic_bytes=algo, padded_bytes=int(stg.relation_bytes),
                                 step1_ms=t1 * 1e3,
                                 per_unit="relation rows of every arc of every instance "
                                          "(d rows of ceil(d/32) words), step 1"))
        grp.close()
        for nt in nets:
            nt.close()
    else:
        name = args.workload.replace("-", "_")
        w = getattr(workloads, name)()
        inst, dom = w.instances[0], w.domains[0]
        net = rac.Net.from_instance(inst, profile=True, path=rac.PATH_BITS)
        for _ in range(args.warmup):
            net.enforce(dom)
        kms, k1ms, dms, t_host = 0.0, 0.0, 0.0, 0.0
        for _ in range(args.steps):
            t0 = time.perf_counter()
            net.enforce(dom)
            t_host += time.perf_counter() - t0
            stk = net.stats()
            kms += stk.kernel_ms
            k1ms += stk.first_kernel_ms
            dms += stk.device_ms
        st = net.stats()
        t_call = t_host / args.steps            # one enforcement through the host call
        t_dev = dms / args.steps * 1e-3         # its kernels on the device (all steps)
        t_k1 = k1ms / args.steps * 1e-3         # the revise launch of step 1
        algo = algo_row_bytes(inst)
        gbs = algo / t_k1 / 1e9
        out.update(value=st.support_checks / t_call, ms_per_step=t_call * 1e3,
                   dtype="u32 bit rows",
                   config=dict(workload=w.name, path="bits"),
                   fixpoints_per_s=1.0 / t_call, host_ms_per_call=t_call * 1e3,
                   device_ms_per_call=t_dev * 1e3,
                   device_support_checks_per_s=st.support_checks / t_dev,
                   revise_kernel_support_checks_per_s=st.support_checks / (kms / args.steps * 1e-3),
                   roofline=dict(kernel="revise_kernel", bound="hbm", achieved=gbs,
                                 peak=HBM_PEAK_GBS, unit="GB/s", frac=gbs / HBM_PEAK_GBS,
                                 traffic=recorded_traffic(f"revise_kernel_{args.workload.replace('-', '_')}"),
                                 algorithmic_bytes=algo, padded_bytes=int(st.relation_bytes),
                                 step1_ms=t_k1 * 1e3,
                                 per_unit="relation rows of every arc (d rows of ceil(d/32) words), "
                                          "step 1"))
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline_single(inst, dom, args.cpu_seconds)
        net.close()

    if not args.no_secondary and args.workload == "batch-states":
        sec = {}
        # small and mid single instances: time per fixpoint through the host
        # call on the path the autotuner picks, and on the bit-row path the
        # sweep's bandwidth with warm and (mid) flushed caches
        flush = torch.empty(1 << 30, dtype=torch.uint8, device=dev)

        def host_calls(net, dom, reps=20):
            for _ in range(5):
                net.enforce(dom)
            t_host = 0.0
            for _ in range(reps):
                t0 = time.perf_counter()
                net.enforce(dom)
                t_host += time.perf_counter() - t0
            return t_host / reps

        for wname in ("single_small", "single_mid"):
            ws = getattr(workloads, wname)()
            inst, dom = ws.instances[0], ws.domains[0]
            tuned = rac.Net.from_instance(inst)
            t_auto = host_calls(tuned, dom)
            st_auto = tuned.stats()
            tuned.close()
            net = rac.Net.from_instance(inst, path=rac.PATH_BITS, profile=True)
            t_bits = host_calls(net, dom)
            best = 1e9
            for _ in range(20):
                net.enforce(dom)
                best = min(best, net.stats().kernel_ms)
            stt = net.stats()
            line = dict(us_per_fixpoint_host_call=t_auto * 1e6, fixpoints_per_s=1.0 / t_auto,
                        path=rac.PATH_NAMES[st_auto.path],
                        tuned_from=rac.TUNE_SOURCES[st_auto.tune_source],
                        device_us_per_fixpoint=st_auto.device_ms * 1e3,
                        us_per_fixpoint_host_call_bits=t_bits * 1e6, kernel_ms_bits=best,
                        warm_relation_GBs=algo_row_bytes(inst) / (best * 1e-3) / 1e9,
                        steps=int(stt.sweeps))
            if wname == "single_mid":
                cold = 0.0
                for _ in range(5):
                    flush.fill_(1)      # 1 GiB through L2 and the Infinity Cache
                    torch.cuda.synchronize()
                    net.enforce(dom)
                    cold += net.stats().kernel_ms
                line["cold_relation_GBs"] = algo_row_bytes(inst) / (cold / 5 * 1e-3) / 1e9
            sec[ws.name] = line
            net.close()
        del flush

        wl = workloads.single_large()
        inst, dom = wl.instances[0], wl.domains[0]
        for pname, p in (("bits", rac.PATH_BITS), ("int8", rac.PATH_INT8)):
            net = rac.Net.from_instance(inst, path=p, profile=True)
            for _ in range(3):
                net.enforce(dom)
            best, times = 1e9, []
            for _ in range(10):
                net.enforce(dom)
                times.append(net.stats().kernel_ms)
                best = min(best, times[-1])
            stt = net.stats()
            algo = algo_row_bytes(inst, pname)
            mean = sum(times) / len(times)
            sec[f"single-large n=2000 d=32 p1=0.9 p2=0.2 [{pname}]"] = dict(
                kernel_ms=best, kernel_ms_mean=mean, algorithmic_bytes=algo,
                padded_bytes=int(stt.relation_bytes),
                relation_GBs=algo / (best * 1e-3) / 1e9,
                hbm_frac=algo / (best * 1e-3) / 1e9 / HBM_PEAK_GBS,
                hbm_frac_mean=algo / (mean * 1e-3) / 1e9 / HBM_PEAK_GBS,
                support_checks_per_s=stt.support_checks / (best * 1e-3), steps=int(stt.sweeps))
            net.close()
        if not args.no_uneven:
            wu = workloads.uneven_multi()
            nets = [rac.Net.from_instance(i, profile=True) for i in wu.instances]
            grp = rac.Group(nets, profile=True)
            grp.enforce(wu.domains)
            best, best_dev, best1 = 1e9, 1e9, 1e9
            for _ in range(5):
                _, it_u, st_u = grp.enforce(wu.domains)
                stg = grp.stats()
                best = min(best, stg.kernel_ms)
                best_dev = min(best_dev, stg.device_ms)
                best1 = min(best1, stg.first_kernel_ms)
            algo = sum(algo_row_bytes(i) for i in wu.instances)
            gbs1 = algo / (best1 * 1e-3) / 1e9
            sec["uneven-multi 256 instances (shared step kernels)"] = dict(
                kernel_ms=best, device_ms=best_dev, fixpoints_per_s=len(nets) / (best_dev * 1e-3),
                step1_revise_ms=best1, algorithmic_bytes=algo,
                padded_bytes=int(stg.relation_bytes), step1_relation_GBs=gbs1,
                step1_hbm_frac=gbs1 / HBM_PEAK_GBS,
                support_checks_per_s=stg.support_checks / (best_dev * 1e-3),
                steps_max=int(it_u.max()), steps_mean=float(it_u.mean()),
                wiped_instances=int(st_u.sum()))
            grp.close()
            for nt in nets:
                nt.close()
        if not args.no_search:
            sec.update(search_lines())
        sec["hbm copy (context for the HBM fractions)"] = copy_rate(dev)
        out["secondary"] = sec

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
