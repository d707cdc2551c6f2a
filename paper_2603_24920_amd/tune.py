"""Radius-schedule autotuning (a thin wrapper over the library's pdet_autotune).

The paper starts the radius ladder at a "magic" r_min (taken from PM-LSH): at r_min the
candidate set already reaches beta*n + k, at r_min / c it does not. That radius depends
on the query, so a dataset-level value is chosen by the library from pilot queries (one
ladder step below their median terminating radius), together with the number of rounds
its batched bound kernel resolves.
"""
from __future__ import annotations


def autotune_r_min(index, Q_pilot, k: int, c: float, beta: float, precision: str = "fp32") -> float:
    """Tune the index on the pilot queries and return the chosen r_min."""
    return index.autotune(Q_pilot, k=k, c=c, beta=beta, precision=precision)["r_min"]
