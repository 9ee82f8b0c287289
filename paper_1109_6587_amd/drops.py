"""Drops in simple shear between walls, time-stepped on the device.

Each stage of the explicit midpoint rule (Sec. 5):
  1. node normals, node areas and Lap x of the current shape
     (ggem_surface_geometry);
  2. the right-hand side b of Eq. qa for drops with tension 1/Ca
     (ggem_drop_rhs);
  3. GMRES for (I + kappa/4pi D) q = b to the relative residual `tol`, warm
     started from a guess (ggem_fredholm_solve);
  4. the node velocity of Eq. bi_ua (ggem_surface_velocity).
The positions then advance with ggem_advance.  Every step runs in the
library's kernels; this module only orders the calls and keeps the arrays.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import ggem as B


def incidence(tri, n_nodes):
    """Triangles incident to each node as CSR (offsets (n+1,), ids), int32,
    each node's triangles in increasing id order."""
    tri = np.asarray(tri)
    nodes = tri.reshape(-1)
    ids = np.repeat(np.arange(tri.shape[0]), 3)
    order = np.lexsort((ids, nodes))
    off = np.zeros(n_nodes + 1, dtype=np.int64)
    np.add.at(off, nodes + 1, 1)
    return np.cumsum(off).astype(np.int32), ids[order].astype(np.int32)


@dataclass
class SolveRecord:
    step: int
    stage: int
    iters: int
    rel_res: float
    seconds: float


class DropSuspension:
    def __init__(self, case, precision="mixed", restart=20, tol=1e-6, max_iter=300,
                 device="cuda:0"):
        import torch

        self.c = case
        self.dev = torch.device(device)
        self.tol = tol
        self.max_iter = max_iter
        n, m = case.nodes.shape[0], case.tri.shape[0]
        self.plan = B.Plan(case.Lx, case.Lz, case.H, case.alpha, case.Nx, case.Nz, case.Ny,
                           rc=case.rc, precision=precision, max_src=3 * m, max_tgt=n,
                           sync_checks=True)
        self.solver = B.FredholmSolver(self.plan, n, m, restart=restart)
        off, adj = incidence(case.tri, n)
        t = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt,  # noqa: E731
                                                      device=self.dev)
        self.tri = t(case.tri, torch.int32)
        self.off = t(off, torch.int32)
        self.adj = t(adj, torch.int32)
        self.x = t(case.nodes)
        self.q = torch.zeros_like(self.x)
        self.kappa = (case.lam - 1.0) / (case.lam + 1.0)
        self.step_index = 0
        self.records: list[SolveRecord] = []

    def geometry(self, x):
        return self.solver.geometry(x, self.tri, self.off, self.adj)

    def rhs(self, nrm, lap):
        c = self.c
        return self.solver.drop_rhs(nrm, lap, c.lam, c.inv_ca, c.shear)

    def solve(self, x, nrm, b, q0, tol=None, max_iter=None):
        """q from the guess q0 (copied); returns (q, iters, rel_res, seconds)."""
        import torch
        q = q0.clone()
        surf = B.Surface(x, nrm, self.tri, self.kappa)
        torch.cuda.synchronize(self.dev)
        t0 = time.perf_counter()
        it, rr = self.solver.solve(surf, b, q, tol=self.tol if tol is None else tol,
                                   max_iter=self.max_iter if max_iter is None else max_iter)
        torch.cuda.synchronize(self.dev)
        return q, it, rr, time.perf_counter() - t0

    def stage(self, x, q0, stage, hook=None):
        nrm, area, lap = self.geometry(x)
        b = self.rhs(nrm, lap)
        if hook is not None:
            hook.before(x, nrm, lap, b, q0, stage)
        q, it, rr, sec = self.solve(x, nrm, b, q0)
        self.records.append(SolveRecord(self.step_index, stage, it, rr, sec))
        if rr > self.tol:
            raise RuntimeError(f"GMRES stalled at step {self.step_index} stage {stage}: "
                               f"relative residual {rr:.3e} after {it} products")
        if hook is not None:
            hook.after(q)
        u = self.solver.velocity(x, self.tri, q, self.c.shear)
        return u, q

    def step(self, hook=None):
        """One explicit midpoint step; the warm start of each solve is the
        previous stage's density.  `hook.before(x, normals, lap, b, q_prev,
        stage)` and `hook.after(q)` see every solve (e.g. to record it)."""
        dt = self.c.dt
        u1, q1 = self.stage(self.x, self.q, 0, hook)
        xh = self.solver.advance(self.x, u1, 0.5 * dt)
        u2, q2 = self.stage(xh, q1, 1, hook)
        self.solver.advance(self.x, u2, dt, out=self.x)
        self.q = q2
        self.step_index += 1
        self.plan.status()
