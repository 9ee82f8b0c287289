"""Neo-Hookean capsules in simple shear between the walls, time-stepped on
the device (Sec. 4, Sec. 5, Sec. 7.1).

Each stage of the explicit midpoint rule:
  1. node normals, node areas (ggem_surface_geometry);
  2. the membrane traction jump of the current shape
     (ggem_membrane_traction);
  3. the right-hand side b of Eq. qa (ggem_traction_rhs);
  4. q = b when the viscosities match (lambda = 1: the operator of Eq. qa is
     the identity), else GMRES to the relative residual `tol`, warm started
     from the previous stage's density;
  5. the node velocity of Eq. bi_ua.
With discretisation="bi" (the default) steps 4 and 5 use the paper's own
boundary-integral discretisation, element quadrature of the local part and
nodal trapezoid strengths for the global part (ggem_bi_fredholm_solve,
ggem_bi_surface_velocity); with "gauss" they use the three interior Gauss
points per triangle as point sources (ggem_fredholm_solve,
ggem_surface_velocity), the discretisation of the drop workload.
The step dt follows gamma_dot dt = 0.5 Ca h_s^m / a with h_s^m the minimum
node separation (ggem_capsule_separation).  After each step the volume of a
capsule that drifted by more than 1e-4 is corrected (ggem_volume_correct)
and overlaps are removed (ggem_overlap_correct).  Every step runs in the
library's kernels; this module only orders the calls and keeps the arrays.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import ggem as B
from .drops import incidence


@dataclass
class StageRecord:
    step: int
    stage: int
    iters: int
    rel_res: float
    seconds: float


@dataclass
class StepRecord:
    step: int
    dt: float
    h_min: float
    volume_corrections: int
    overlap_sweeps: int
    seconds: float


class CapsuleSuspension:
    def __init__(self, case, precision="mixed", restart=20, tol=1e-6, max_iter=300,
                 vol_tol=1e-4, discretisation="bi", device="cuda:0"):
        import torch

        if discretisation not in ("bi", "gauss"):
            raise ValueError("discretisation must be 'bi' or 'gauss'")
        self.c = case
        self.bi = discretisation == "bi"
        self.dev = torch.device(device)
        self.tol = tol
        self.max_iter = max_iter
        self.vol_tol = vol_tol
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
        self.membrane = B.Membrane(self.solver, case.ncap, self.tri, t(case.ref_nodes), case.G)
        self.rigid = B.RigidParticle(self.plan, n, m, restart=restart) if self.bi else None
        self.v0 = self.membrane.volumes(self.x).clone()
        self.q = torch.zeros_like(self.x)
        self.kappa = (case.lam - 1.0) / (case.lam + 1.0)
        e0, _ = self.membrane.separation(self.x, case.Lx, case.Lz, 1.0)
        self.reach = 1.5 * e0
        self.step_index = 0
        self.stages: list[StageRecord] = []
        self.steps: list[StepRecord] = []

    def min_separation(self):
        """h_s^m: the shortest edge or the smallest gap between capsules."""
        c = self.c
        while True:
            e, g = self.membrane.separation(self.x, c.Lx, c.Lz, self.reach)
            if e <= self.reach:
                return min(e, g)
            self.reach = 1.5 * e

    def time_step(self, h):
        c = self.c
        return 0.5 * c.ca * h / (c.a * c.shear)

    def stage(self, x, q0, stage):
        import torch
        c = self.c
        torch.cuda.synchronize(self.dev)
        t0 = time.perf_counter()
        nrm, _, _ = self.solver.geometry(x, self.tri, self.off, self.adj)
        df = self.membrane.traction(x, self.off, self.adj)
        b = self.solver.traction_rhs(nrm, df, c.lam, c.shear)
        mesh = (x, self.tri, self.off, self.adj)
        if c.lam == 1.0:
            q, it, rr = b, 0, 0.0
        else:
            q = q0.clone()
            if self.bi:
                it, rr = self.rigid.fredholm_solve(*mesh, nrm, self.kappa, b, q, tol=self.tol,
                                                   max_iter=self.max_iter)
            else:
                it, rr = self.solver.solve(B.Surface(x, nrm, self.tri, self.kappa), b, q,
                                           tol=self.tol, max_iter=self.max_iter)
            if rr > self.tol:
                raise RuntimeError(f"GMRES stalled at step {self.step_index} stage {stage}: "
                                   f"relative residual {rr:.3e} after {it} products")
        if self.bi:
            u = self.rigid.surface_velocity(*mesh, q, c.shear)
        else:
            u = self.solver.velocity(x, self.tri, q, c.shear)
        torch.cuda.synchronize(self.dev)
        self.stages.append(StageRecord(self.step_index, stage, it, rr, time.perf_counter() - t0))
        return u, q

    def step(self, dt=None):
        """One explicit midpoint step (dt from the separation rule unless
        given), then the volume and overlap corrections."""
        import torch
        c = self.c
        t0 = time.perf_counter()
        h = self.min_separation()
        dt = self.time_step(h) if dt is None else dt
        u1, q1 = self.stage(self.x, self.q, 0)
        xh = self.solver.advance(self.x, u1, 0.5 * dt)
        u2, q2 = self.stage(xh, q1, 1)
        self.solver.advance(self.x, u2, dt, out=self.x)
        self.q = q2
        nrm, area, _ = self.solver.geometry(self.x, self.tri, self.off, self.adj)
        nv = self.membrane.volume_correct(self.x, nrm, area, self.v0, self.vol_tol)
        sw = self.membrane.overlap_correct(self.x, c.Lx, c.Lz, c.H, c.h_min)
        self.plan.status()
        torch.cuda.synchronize(self.dev)
        self.steps.append(StepRecord(self.step_index, dt, h, nv, sw, time.perf_counter() - t0))
        self.step_index += 1
        return dt

    def close(self):
        if self.rigid is not None:
            self.rigid.close()
        self.membrane.close()
        self.solver.close()
        self.plan.close()
