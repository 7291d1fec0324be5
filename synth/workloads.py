"""The five named workloads, as seeded recipes.

seed = 201008526 + workload index.

1. er4096   : A n=4096, exactly 8 entries per column, float64 (0,1]; C = A A.
2. rmat20   : R-MAT scale 20, edge factor 16, (a,b,c) = (.57,.19,.19),
              symmetrized, deduplicated, float32 (0,1]; C = A A, HBM budget
              chosen so the batch planner picks 4 column batches.
3. protein2m: Chung-Lu power law (exponent 2.1, mean 50, cap 5000),
              n = 2e6, column-stochastic float32; C = A A with 16
              inner-dimension layers and a 64 GB budget.
4. er262k   : A and B independent, n = 262144, 16 per column, float32
              N(0,1); loss targets N(0,1) on the pattern of C.
5. batch4096: 4096 independent Erdos-Renyi pairs, n_i log-uniform in
              [256, 65536], degrees uniform in [4, 32], float32 (0,1].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import matrices as M

SEED0 = 201008526


@dataclass
class Workload:
    name: str
    index: int
    layers: int = 1
    budget_bytes: int | None = None  # None: computed by the caller's recipe
    target_batches: int | None = None
    dtype: torch.dtype = torch.float32
    params: dict = field(default_factory=dict)

    @property
    def seed(self) -> int:
        return SEED0 + self.index


WORKLOADS = {
    "er4096": Workload("er4096", 1, dtype=torch.float64, params=dict(n=4096, d=8)),
    "rmat20": Workload("rmat20", 2, target_batches=4, params=dict(scale=20, edge_factor=16)),
    "protein2m": Workload("protein2m", 3, layers=16, budget_bytes=64 << 30, params=dict(n=2_000_000)),
    "er262k": Workload("er262k", 4, params=dict(n=262_144, d=16)),
    "batch4096": Workload("batch4096", 5, params=dict(count=4096)),
}


def make_workload(name: str, device="cpu", **over):
    """Inputs (A, B) of a named workload; keyword overrides shrink it for
    tests (e.g. scale=12 for rmat20, n=20000 for protein2m)."""
    w = WORKLOADS[name]
    p = dict(w.params)
    p.update(over)
    s = w.seed
    if name == "er4096":
        A = M.erdos_renyi(p["n"], p["n"], p["d"], s, torch.float64, device)
        return A, A
    if name == "rmat20":
        A = M.rmat(p["scale"], p["edge_factor"], s, dtype=torch.float32, device=device)
        return A, A
    if name == "protein2m":
        A = M.protein_like(p["n"], s, dtype=torch.float32, device=device)
        return A, A
    if name == "er262k":
        A = M.erdos_renyi(p["n"], p["n"], p["d"], s, torch.float32, device, dist="normal")
        B = M.erdos_renyi(p["n"], p["n"], p["d"], s + 7919, torch.float32, device, dist="normal")
        return A, B
    if name == "batch4096":
        spec = M.batch_spec(p["count"], s)
        return spec, [M.batch_instance(spec, i, s, torch.float32, device) for i in range(p["count"])]
    raise KeyError(name)
