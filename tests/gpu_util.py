"""Helpers for the GPU tests: device tensors from numpy relations, plans."""
from __future__ import annotations

import numpy as np


def dev(a):
    import torch
    a = np.ascontiguousarray(np.asarray(a).view(np.int32).reshape(-1, 2))
    return torch.from_numpy(a).to("cuda")


def fixed_plan(mj, ctx, kind, R, S, T, a_domain=0, **fields):
    """Plan with explicit bucket fields (planner 'fixed')."""
    p = mj.Plan()
    for k, v in fields.items():
        setattr(p, k, v)
    return ctx.plan(kind, R, S, T, a_domain, planner="fixed", fixed=p)


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
