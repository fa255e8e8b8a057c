"""Constraint-violation metrics (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

constraint_error: for each constraint type k, the batch mean of the Euclidean
norm of that type's residual vector (paper Appendix E, the constraint-error
equation).  max_violation: ||h(u)||_inf per sample, the feasibility bar of the
projected-samples/s metric.  Both re-evaluate h with the oracle's own
definitions.

Parity: the residual definitions are the families' h (pinned there); the
reductions are a mean of 2-norms and a max of absolute values.
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np

from .families import family_of


def max_violation(batch, u_packed, indices=None):
    idx = range(len(batch)) if indices is None else indices
    out = np.zeros(len(batch))
    for s in idx:
        smp = batch.samples[s]
        vo = batch.var_off[s]
        h = family_of(smp).h(np.asarray(u_packed[vo:vo + smp.n], dtype=np.float64))
        out[s] = np.abs(h).max(initial=0.0)
    return out


def constraint_error(batch, u_packed, indices=None):
    idx = list(range(len(batch))) if indices is None else list(indices)
    acc = defaultdict(list)
    for s in idx:
        smp = batch.samples[s]
        vo = batch.var_off[s]
        fam = family_of(smp)
        parts = fam.split(fam.h(np.asarray(u_packed[vo:vo + smp.n], dtype=np.float64)))
        for k, v in parts.items():
            acc[k].append(np.linalg.norm(v))
    return {k: float(np.mean(v)) for k, v in acc.items()}
