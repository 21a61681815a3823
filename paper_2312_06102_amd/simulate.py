"""Multi-step N-body runs around the tree build.

The paper measures its construction inside simulations: a leapfrog integrator
over constant timesteps, the tree rebuilt at every step and the force found by
a Barnes-Hut walk with n_crit groups (Sec. 3).  Reordering the particles in
memory by key is optional (Sec. 2.3); the paper reorders at every step for its
timings and suggests doing it only every few steps (Sec. 4).  Between reorders
the particles keep the order of the last reorder, so their keys arrive nearly
sorted.

``Simulation`` runs such a loop entirely through the library's C entry points:
tb_build (auto box, sorted particles kept for the walk), tb_gravity, and the
two particle updates tb_kick_drift and tb_permute.  Every step is

    kick-drift  v += a dt (dt/2 on the first step), x += v dt
    build       the tree of the drifted particles
    reorder     (every `reorder_every` builds) pos, vel, mass and the particle
                ids gathered into the build's key order
    gravity     accelerations and potentials in key order for the next kick

and ``synchronise()`` closes with a half kick so that positions and velocities
refer to the same time.  Per-phase GPU times are taken with events on the
stream the work runs on.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import treebuild as tb

PHASES = ("kick_drift", "build", "reorder", "gravity")


class Simulation:
    def __init__(self, pos, vel, mass, dt: float, n_leaf: int = 10, theta: float = 0.75,
                 n_crit: int = 512, eps: float = 0.0, reorder_every: int = 1,
                 quadrupole: bool = True, curve: str = "morton", device="cuda"):
        if reorder_every < 0:
            raise ValueError("reorder_every must be >= 0 (0: never reorder)")
        self.device = torch.device(device)
        self.pos = torch.as_tensor(np.ascontiguousarray(pos, np.float32), device=self.device)
        self.vel = torch.as_tensor(np.ascontiguousarray(vel, np.float32), device=self.device)
        self.mass = torch.as_tensor(np.ascontiguousarray(mass, np.float32), device=self.device)
        self.n = int(self.pos.shape[0])
        if self.vel.shape != self.pos.shape or self.mass.shape != (self.n,):
            raise ValueError("pos [N,3], vel [N,3] and mass [N] must describe the same particles")
        self.ids = torch.arange(self.n, dtype=torch.int32, device=self.device)
        self.dt, self.theta, self.n_crit, self.eps = float(dt), float(theta), int(n_crit), float(eps)
        self.reorder_every, self.quadrupole = int(reorder_every), bool(quadrupole)
        self.builder = tb.Builder(self.n, n_leaf, "fp64", 0, self.device, sorted_particles=True,
                                  curve=curve)
        # spare arrays: a reorder gathers into them, then the two swap
        self._spare = {k: torch.empty_like(getattr(self, k)) for k in ("pos", "vel", "mass", "ids")}
        self.acc = torch.empty((max(self.n, 1), 4), dtype=torch.float64, device=self.device)
        self.stats = torch.zeros(2, dtype=torch.int64, device=self.device)
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.c_max = max(tb.tb_max_cells(self.n, n_leaf), 1)
        self._gws_bytes = tb.tb_gravity_workspace_bytes(self.c_max)
        self._gws = torch.empty(self._gws_bytes, dtype=torch.uint8, device=self.device)
        self._grav_flags = ((tb.TB_GRAV_QUADRUPOLE if self.quadrupole else 0)
                            | (self.builder.flags & tb.TB_HILBERT))
        self.builds = 0
        self.steps = 0
        self._kick_perm: Optional[torch.Tensor] = None
        self._half_kick_next = True
        self._events = []  # per step: {phase: (start, end)}
        self.interactions = []

    # -- phases ---------------------------------------------------------------
    def _stream(self):
        return torch.cuda.current_stream(self.device)

    def _timed(self, rec, phase, fn):
        s = self._stream()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        rec[phase] = (a, b)

    def _build(self):
        self.builder.launch(self.pos, self.mass, box=None)
        self.builds += 1

    def _reorder(self):
        perm = self.builder.out.perm[:self.n]
        for k in ("pos", "vel", "mass", "ids"):
            tb.permute(perm, getattr(self, k), self._spare[k], self.status)
        for k in ("pos", "vel", "mass", "ids"):
            cur = getattr(self, k)
            setattr(self, k, self._spare[k])
            self._spare[k] = cur

    def _gravity(self):
        o = self.builder.out
        rc = tb.tb_gravity(o.pos_sorted.data_ptr(), o.mass_sorted.data_ptr(), self.n,
                           self.builder._struct, self.c_max, self.theta, self.n_crit, self.eps,
                           self._grav_flags, self.acc.data_ptr(), self.stats.data_ptr(),
                           self._gws.data_ptr(), self._gws_bytes, self._stream().cuda_stream)
        if rc:
            tb._raise(rc, "tb_gravity")

    def _tree_and_forces(self, rec):
        self._timed(rec, "build", self._build)
        if self.reorder_every and (self.builds - 1) % self.reorder_every == 0:
            self._timed(rec, "reorder", self._reorder)
            self._kick_perm = None  # accelerations now follow the particle arrays
        else:
            self._kick_perm = self.builder.out.perm[:self.n]
        self._timed(rec, "gravity", self._gravity)
        self.interactions.append(self.stats.clone())

    def _kick_drift(self, dt_kick, dt_drift):
        tb.kick_drift(self._kick_perm, self.acc, dt_kick, dt_drift, self.pos, self.vel,
                      self.status)

    # -- public ---------------------------------------------------------------
    def step(self, k: int = 1) -> None:
        """Advance k leapfrog steps (asynchronous)."""
        for _ in range(k):
            rec = {}
            if self.builds == 0:
                self._tree_and_forces({})  # forces at the initial positions (not timed)
            dtk = 0.5 * self.dt if self._half_kick_next else self.dt
            self._timed(rec, "kick_drift", lambda: self._kick_drift(dtk, self.dt))
            self._half_kick_next = False
            self._tree_and_forces(rec)
            self._events.append(rec)
            self.steps += 1

    def synchronise(self) -> None:
        """Close with a half kick: velocities at the time of the positions.  The
        next step() starts with a half kick again."""
        if self.builds == 0:
            self._tree_and_forces({})
        if not self._half_kick_next:
            self._kick_drift(0.5 * self.dt, 0.0)
            self._half_kick_next = True
        torch.cuda.synchronize(self.device)
        self.check()

    def check(self) -> None:
        torch.cuda.synchronize(self.device)
        if int(self.status.item()):
            raise tb.TreeBuildError(tb.TB_ERR_INTERNAL, "tb_kick_drift/tb_permute")
        tb._check_status(int(self.builder.out.status.item()), "tb_build/tb_gravity")

    def timings(self) -> dict:
        """Per-phase GPU milliseconds: mean over the steps taken, and per step."""
        torch.cuda.synchronize(self.device)
        per = {p: [] for p in PHASES}
        for rec in self._events:
            for p in PHASES:
                if p in rec:
                    a, b = rec[p]
                    per[p].append(a.elapsed_time(b))
        mean = {p: (float(np.mean(v)) if v else 0.0) for p, v in per.items()}
        mean["reorders"] = len(per["reorder"])
        mean["steps"] = len(self._events)
        return {"mean_ms": mean, "per_step_ms": per}

    def state(self) -> dict:
        """Host copies ordered by particle id: pos, vel, mass, and (from the last
        walk) acceleration and potential."""
        torch.cuda.synchronize(self.device)
        ids = self.ids.cpu().numpy()
        order = np.argsort(ids)
        out = {"pos": self.pos.cpu().numpy()[order], "vel": self.vel.cpu().numpy()[order],
               "mass": self.mass.cpu().numpy()[order]}
        # the walk's outputs are in the key order of the last build
        perm = self.builder.out.perm[:self.n].cpu().numpy()
        acc = self.acc[:self.n].cpu().numpy()
        cur_ids = ids if self._kick_perm is None else ids[perm]
        a = np.empty_like(acc)
        a[cur_ids] = acc
        out["acc"], out["phi"] = a[:, :3], a[:, 3]
        return out

    def energy(self) -> dict:
        """Kinetic, potential (1/2 sum m phi) and total energy; call after
        synchronise()."""
        st = self.state()
        m = st["mass"].astype(np.float64)
        v = st["vel"].astype(np.float64)
        kin = 0.5 * float(np.sum(m * np.einsum("ij,ij->i", v, v)))
        pot = 0.5 * float(np.sum(m * st["phi"]))
        return {"kinetic": kin, "potential": pot, "total": kin + pot}
