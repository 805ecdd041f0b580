"""The five seeded model-B workloads the library is tested and measured on.

Each stands in for the paper's randomly generated binary CSPs (Section 5.2);
the paper's own 25 instances are not published, so sizes, domain size and
tightness are fixed here. Model-B counts round half up: m = floor(p1*n(n-1)/2 + 1/2)
edges and floor(p2*d^2 + 1/2) forbidden pairs per relation.

  single-small   n=50,   d=10, p1=0.5, p2=0.30, full domains                (seed 1)
  single-mid     n=500,  d=20, p1=1.0, p2=0.35, full minus 1000 values      (seed 2, removals seed 20)
  single-large   n=2000, d=32, p1=0.9, p2=0.20, full domains                (seed 3)
  batch-states   n=1000, d=32, p1=0.8, p2=0.25, 1024 states, each a random
                 partial assignment of 0..20 variables to singletons        (seed 4, states seed 40)
  uneven-multi   256 instances, n~U{20..800}, d~U{4..64}, p1~U[0.1,1),
                 p2~U[0.1,0.6), full domains                                 (seed 5, instance i from
                                                                              substream(5, i))
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import (Instance, full_domains, model_b, partial_assign_states, preremove,
               substream, uneven_params)


@dataclass
class Workload:
    name: str
    instances: List[Instance]
    # per instance: dom[n] (single state) or dom[B, n] (batched states)
    domains: List[np.ndarray]
    params: dict = field(default_factory=dict)


SINGLE_SMALL = dict(seed=1, n=50, d=10, p1=0.5, p2=0.3)
SINGLE_MID = dict(seed=2, n=500, d=20, p1=1.0, p2=0.35, removed=1000, removal_seed=20)
SINGLE_LARGE = dict(seed=3, n=2000, d=32, p1=0.9, p2=0.2)
BATCH_STATES = dict(seed=4, n=1000, d=32, p1=0.8, p2=0.25, B=1024, max_assign=20, state_seed=40)
UNEVEN_MULTI = dict(seed=5, k=256, nmin=20, nmax=800, dmin=4, dmax=64,
                    p1lo=0.1, p1hi=1.0, p2lo=0.1, p2hi=0.6)


def single_small() -> Workload:
    c = SINGLE_SMALL
    inst = model_b(c["seed"], c["n"], c["d"], c["p1"], c["p2"])
    return Workload("single-small n=50 d=10 p1=0.5 p2=0.3", [inst],
                    [full_domains(c["n"], c["d"])], dict(c))


def single_mid() -> Workload:
    c = SINGLE_MID
    inst = model_b(c["seed"], c["n"], c["d"], c["p1"], c["p2"])
    dom = preremove(c["removal_seed"], c["n"], c["d"], c["removed"])
    return Workload("single-mid n=500 d=20 p1=1.0 p2=0.35 (1000 values pre-removed)", [inst],
                    [dom], dict(c))


def single_large() -> Workload:
    c = SINGLE_LARGE
    inst = model_b(c["seed"], c["n"], c["d"], c["p1"], c["p2"])
    return Workload("single-large n=2000 d=32 p1=0.9 p2=0.2", [inst],
                    [full_domains(c["n"], c["d"])], dict(c))


def batch_states(B: Optional[int] = None) -> Workload:
    c = dict(BATCH_STATES)
    if B is not None:
        c["B"] = B
    inst = model_b(c["seed"], c["n"], c["d"], c["p1"], c["p2"])
    dom, _ = partial_assign_states(c["state_seed"], c["n"], c["d"], c["B"], c["max_assign"])
    return Workload(f"batch-states n=1000 d=32 p1=0.8 p2=0.25 B={c['B']}", [inst], [dom], c)


def uneven_multi(k: Optional[int] = None) -> Workload:
    c = dict(UNEVEN_MULTI)
    if k is not None:
        c["k"] = k
    n, d, p1, p2 = uneven_params(c["seed"], c["k"], c["nmin"], c["nmax"], c["dmin"], c["dmax"],
                                 c["p1lo"], c["p1hi"], c["p2lo"], c["p2hi"])
    insts, doms = [], []
    for i in range(c["k"]):
        inst = model_b(substream(c["seed"], i), int(n[i]), int(d[i]), float(p1[i]), float(p2[i]))
        insts.append(inst)
        doms.append(full_domains(int(n[i]), int(d[i])))
    return Workload(f"uneven-multi k={c['k']}", insts, doms, c)
