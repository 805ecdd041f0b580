"""Builds the autotuner table shipped with librac (rac_tune_gfx950.txt, next
to librac.so): measures, on the GPU, the shapes of the benchmark workloads
and a grid of single-state and batched shapes, and writes the fastest path
and work-item size of each (the same measurement the library runs on the
first call of a shape that is not in its table).

    python -m paper_2407_11388_amd.tune_table OUT.txt
"""
from __future__ import annotations

import os
import sys


def main(out: str) -> None:
    os.environ["RAC_TUNE_CACHE"] = os.path.abspath(out)
    os.environ["RAC_TUNE_TABLE"] = os.devnull   # measure everything, ignore the shipped table
    if os.path.exists(out):
        os.remove(out)
    import numpy as np

    from paper_2407_11388_amd import gen, rac
    from paper_2407_11388_amd.gen import workloads

    measure = dict(tune=rac.TUNE_MEASURE)
    # batched states over a grid of shapes (first, so that the workloads'
    # own measurements below win where a grid shape has the same key)
    for d in (8, 16, 32):
        for n in (64, 256, 1024):
            for p1 in (0.1, 0.5, 1.0):
                for B in (16, 128, 1024):
                    if n * B > 1 << 20:
                        continue
                    inst = gen.model_b(7000 + n + d + int(10 * p1), n, d, p1, 0.25)
                    doms, _ = gen.partial_assign_states(7001 + B, n, d, B, min(20, n))
                    net = rac.Net.from_instance(inst, **measure)
                    net.enforce_batch(doms)
                    print(f"[tune] batch d={d} n={n} p1={p1} B={B}: path {net.stats().path}", flush=True)
                    net.close()
    # single states over a grid of shapes
    for d in (8, 16, 32, 64):
        for n in (64, 256, 1024):
            for p1 in (0.1, 0.5, 1.0):
                inst = gen.model_b(7500 + n + d + int(10 * p1), n, d, p1, 0.25)
                dom = gen.preremove(7501 + n, n, d, (n * d) // 10)
                net = rac.Net.from_instance(inst, **measure)
                net.enforce(dom)
                print(f"[tune] single d={d} n={n} p1={p1}: path {net.stats().path}", flush=True)
                net.close()
    for name in ("single_small", "single_mid", "single_large"):
        w = getattr(workloads, name)()
        net = rac.Net.from_instance(w.instances[0], **measure)
        net.enforce(w.domains[0])
        print(f"[tune] {w.name}: path {net.stats().path}", flush=True)
        net.close()
    w = workloads.uneven_multi()
    for inst, dom in zip(w.instances, w.domains):   # each instance's single-state shape
        net = rac.Net.from_instance(inst, **measure)
        net.enforce(dom)
        net.close()
    print(f"[tune] {w.name}: {len(w.instances)} instances", flush=True)
    w = workloads.batch_states()
    net = rac.Net.from_instance(w.instances[0], **measure)
    net.enforce_batch(w.domains[0])
    print(f"[tune] {w.name}: path {net.stats().path}", flush=True)
    net.close()
    # one entry per key (the last measurement), sorted, under a header
    lines = [ln.rstrip("\n") for ln in open(out) if ln.strip() and not ln.startswith("#")]
    last = {ln.split()[0]: ln for ln in lines}
    head = ["# librac autotuner table, measured on an AMD Instinct MI355X (gfx950) by",
            "#   python -m paper_2407_11388_amd.tune_table rac_tune_gfx950.txt",
            "# key: gfx950/<single|batch>/d<domain size, power of 2>/n<variables, power of 2>/",
            "#      dens<constraint density bucket>/B<states per call, power of 2>",
            "# path: 1 bit rows, 2 int8 rows, 3 matrix cores, 4 fused (one workgroup per state, every",
            "# step in one launch); items: work items of 2^items times the",
            "# default size; handoff: matrix-core states left when the rest moves to the bit rows",
            "# (-1: the default); ms: the measured time per call"]
    with open(out, "w") as f:
        f.write("\n".join(head + [last[k] for k in sorted(last)]) + "\n")
    print(f"[tune] table written to {out}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "rac_tune_gfx950.txt")
