"""Autotuning of the radius schedule.

The paper starts the radius ladder at a "magic" r_min (taken from PM-LSH): at r_min the
candidate set already reaches beta*n + k, at r_min / c it does not. That radius depends
on the query, so a dataset-level value is chosen from pilot queries: every pilot query
is run from a tiny first radius, the library reports the rounds it needed, and r_min is
set one ladder step below the median terminating radius. A typical query then stops in
its first or second round. Only library calls are made here.
"""
from __future__ import annotations

import numpy as np


def autotune_r_min(index, Q_pilot, k: int, c: float, beta: float, r0: float = 1e-3,
                   precision: str = "fp32") -> float:
    _, _, st = index.query(Q_pilot, k=k, c=c, beta=beta, r_min=r0, stats=True,
                           precision=precision, rescore=4)
    st = st.cpu().numpy()
    ok = st[:, 2] > 0
    if not ok.any():
        raise RuntimeError("pilot queries exhausted the radius ladder; raise r0")
    rounds = st[ok, 0].astype(np.float64)
    med = float(np.median(rounds))
    steps = max(0, int(np.floor(med)) - 2)
    return float(r0 * c ** steps)
