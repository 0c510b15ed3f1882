"""Tree/Hermite block-step integration with the force evaluated on the GPU.

The procedure is the paper's tree-Hermite loop (Section 2, steps 1-7):

  1. at every multiple of the tree interval (and at t = 0) the host builds
     the tree, groups and lists and sends particles, nodes and lists;
  2. the host selects the particles due at the next block time;
  4/4a/5. the device predicts particles and nodes and sums each active
     particle's list;
  6. the host corrects the active particles, picks their new block steps and
     sends them back (j-memory update);
  7. time advances.

All particles are synchronised at multiples of the tree interval because
the largest block step equals that interval, so every rebuild happens at an
all-active step, after it has been corrected.
"""
from __future__ import annotations

import contextlib
import math
import types
import time

import numpy as np

from . import binding as B


class Simulation:
    def __init__(self, x, v, m, *, eps2, dt_tree, eta, theta=0.5, n_crit=64, n_leaf=1, precision="mixed",
                 predict_mode="fused", mode="tree", device=0, stream=None, list_headroom=1.5, resident=False,
                 device_tree=False, tree=None, tree_lock=None, device_loop=False):
        if mode not in ("tree", "direct"):
            raise ValueError(mode)
        if device_tree and not (resident and mode == "tree"):
            raise ValueError("the device tree builder serves the resident tree integration")
        if device_loop and not (resident and mode == "tree" and predict_mode == "fused"):
            raise ValueError("the device loop runs the resident tree integration with fused prediction")
        if not (dt_tree > 0 and math.frexp(dt_tree)[0] == 0.5):
            raise ValueError("dt_tree must be a power of two")
        self.x = np.ascontiguousarray(x, np.float64).reshape(-1, 3).copy()
        self.n = self.x.shape[0]
        self.v = np.ascontiguousarray(v, np.float64).reshape(self.n, 3).copy()
        self.m = np.ascontiguousarray(m, np.float64).reshape(self.n).copy()
        self.a = np.zeros((self.n, 3))
        self.j = np.zeros((self.n, 3))
        self.t0 = np.zeros(self.n)
        self.dt = np.zeros(self.n)
        self.ids = np.arange(self.n)
        self.pot = np.zeros(self.n)
        self.eps2, self.dt_tree, self.eta = float(eps2), float(dt_tree), float(eta)
        self.theta, self.n_crit, self.n_leaf = float(theta), int(n_crit), int(n_leaf)
        self.precision, self.predict_mode, self.mode = precision, predict_mode, mode
        self.device, self.stream, self.list_headroom = device, stream, list_headroom
        self.t = 0.0
        self.t_tree = 0.0
        self.ctx = None
        self.tree = None
        self._ectx = None
        self._act_buf = np.empty(self.n, np.int32)
        # resident: the particle state lives on the device between tree rebuilds
        # (scheduler and corrector there); the host arrays are current only after
        # sync_state() and at tree times
        self.resident = bool(resident)
        # resident: rebuild at tree times on the device (ht_state_rebuild), so the
        # state never leaves it; the host path remains the fallback when the tree
        # outgrows the context's capacities
        # (tree, tree_lock: a DeviceTree shared by several simulations and the lock
        # that serialises its use; by default each simulation has its own)
        self.device_tree = bool(device_tree)
        # device_loop: run() queues the block steps up to each tree time on the
        # device with no host round trip between them (ht_dev_run)
        self.device_loop = bool(device_loop)
        self._dtree = tree
        self._own_dtree = tree is None
        self._dtree_lock = tree_lock
        self._perm_pin = None       # pinned landing buffer of a device rebuild's permutation
        self._perm_pending = None   # composite of the permutations not yet applied to the host's m and ids
        self.n_host_rebuilds = 0    # resident rebuilds that went through the host
        self.n_device_rebuilds = 0
        self._pending_dev = None
        self.n_block_steps = 0
        self.n_particle_steps = 0
        self.n_interactions = 0
        self.timers = {"tree": 0.0, "force": 0.0, "host": 0.0, "comm": 0.0}
        self._build_and_send()
        everyone = np.arange(self.n, dtype=np.int32)
        self.ctx.predict(0.0)
        acc, jerk, pot = self._force(everyone)
        self.a, self.j, self.pot = acc, jerk, pot
        self._build_and_send()           # nodes now carry a and jerk; order unchanged
        self.dt = B.initial_steps(self.eta, self.dt_tree, self.a, self.j)
        if self.resident:
            self.ctx.state_enable()
            self.ctx.state_set(self.t0, self.dt, self.m, self.x, self.v, self.a, self.j, self.pot)
        if self.device_tree:
            import torch
            if self._dtree is None:
                self._dtree = B.DeviceTree(n_max=self.n, device=self.device, stream=self.stream)
            self._perm_pin = torch.empty(self.n, dtype=torch.int64, pin_memory=True)
            # one device rebuild now, at t = 0 where every particle is synchronised and
            # already in key order (the same tree, bit for bit), sizes the builder's
            # arrays so that later rebuilds allocate nothing
            self._rebuild_on_device()
            self.n_device_rebuilds = 0

    # ------------------------------------------------------------------ context
    def _make_ctx(self, node_max, group_max, list_max):
        if self.ctx is not None:
            self.ctx.close()
        self.ctx = B.Context(n_max=self.n, node_max=node_max, group_max=group_max, list_max=list_max,
                             active_max=self.n, eps2=self.eps2, precision=self.precision,
                             predict_mode=self.predict_mode, device=self.device, stream=self.stream)
        self._caps = (node_max, group_max, list_max)

    # ------------------------------------------------------------------ step 1
    def _build_and_send(self):
        t_start = time.perf_counter()
        if self.mode == "tree":
            tr = B.HostTree(self.x, self.v, self.a, self.j, self.m, self.n_leaf, self.n_crit, self.theta)
            p = tr.perm
            if not np.array_equal(p, np.arange(self.n)):
                for name in ("x", "v", "a", "j", "m", "t0", "dt", "ids", "pot"):
                    setattr(self, name, np.ascontiguousarray(getattr(self, name)[p]))
            self.tree = tr
            need = (tr.n_node, tr.n_group, tr.n_entries)
        else:
            self.tree = None
            need = (0, 1, 1)
        self.t_tree = self.t
        self.timers["tree"] += time.perf_counter() - t_start
        t_start = time.perf_counter()
        caps = getattr(self, "_caps", None)
        if caps is None or any(n > c for n, c in zip(need, caps)):
            h = self.list_headroom
            self._make_ctx(max(int(need[0] * h), 64), max(int(need[1] * h), 16), max(int(need[2] * h), 1024))
        ctx = self.ctx
        ctx.set_j_particles(self.t0, self.m, self.x, self.v, self.a, self.j)
        if self.mode == "tree":
            tr = self.tree
            ctx.set_nodes(self.t_tree, tr.node_m, tr.node_x, tr.node_v, tr.node_a, tr.node_j)
            ctx.set_interaction_lists(tr.group_first, tr.list_off, tr.entries)
        else:
            ctx.set_nodes(self.t_tree, np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)),
                          np.zeros((0, 3)))
        self.timers["comm"] += time.perf_counter() - t_start

    # ------------------------------------------------------------------ steps 4a/5
    def _force(self, active):
        """Steps 4a and 5 on this simulation's own context (host arrays)."""
        t_start = time.perf_counter()
        if self.mode == "tree":
            out = self.ctx.force(active)
        else:
            out = self.ctx.force_direct(active)
        pairs, _ = self.ctx.last_stats()
        self.n_interactions += pairs
        self.timers["force"] += time.perf_counter() - t_start
        return out

    def next_time(self):
        if self.resident:
            if self._pending_dev is None:
                self._pending_dev = self.ctx.dev_next_block()
            return self._pending_dev[0]
        return float(np.min(self.t0 + self.dt))

    def _apply_perms(self):
        """Device rebuilds reorder the particles on the device; the host's masses
        and identities follow here, when they are needed."""
        p = self._perm_pending
        if p is not None:
            self.m = np.ascontiguousarray(self.m[p])
            self.ids = np.ascontiguousarray(self.ids[p])
            self._perm_pending = None

    def sync_state(self):
        """Resident mode: copy the device state into the host arrays."""
        if self.resident:
            self._apply_perms()
            self.t0, self.dt, self.x, self.v, self.a, self.j, self.pot = self.ctx.state_get(self.n)

    def begin_step(self):
        """Steps 2 and 5 (prediction): pick the next block time and its active
        particles and predict the context there.  Returns (t, active ids)."""
        t_start = time.perf_counter()
        tn, active = B.next_block(self.t0, self.dt, self._act_buf)
        active = active.copy()
        self.timers["host"] += time.perf_counter() - t_start
        self.ctx.predict(tn)
        self._pending = (tn, active)
        return tn, active

    def finish_step(self, acc, jerk, pot):
        """Steps 6 and 7 for the forces of the step begun last: correct, pick
        new steps, and either rebuild (at a tree time; everything re-sent) or
        return the corrected particles as ht_row records for the j-memory."""
        tn, active = self._pending
        self._pending = None
        t_start = time.perf_counter()
        B.correct(active, tn, self.eta, self.dt_tree, self.t0, self.dt, self.x, self.v, self.a, self.j, acc, jerk)
        self.pot[active] = pot
        self.timers["host"] += time.perf_counter() - t_start
        self.t = tn
        self.n_block_steps += 1
        self.n_particle_steps += active.size
        if math.fmod(tn, self.dt_tree) == 0.0:
            if not np.all(self.t0 == tn):
                raise AssertionError("particles not synchronised at a tree time")
            self._build_and_send()
            return None
        return B.make_rows(active, self.t0[active], self.m[active], self.x[active], self.v[active], self.a[active],
                           self.j[active])

    def _step_resident(self):
        if self._pending_dev is None:
            self._pending_dev = self.ctx.dev_next_block()
        tn, active = self._pending_dev
        self._pending_dev = None
        t_start = time.perf_counter()
        if self.mode == "tree":
            self.ctx.dev_step(self.eta, self.dt_tree)
        else:
            self.ctx.dev_step_direct(self.eta, self.dt_tree)
        pairs, _ = self.ctx.last_stats()
        self.n_interactions += pairs
        self.timers["force"] += time.perf_counter() - t_start
        self.t = tn
        self.n_block_steps += 1
        self.n_particle_steps += active.size
        if math.fmod(tn, self.dt_tree) == 0.0 and self.mode == "tree":
            self.rebuild_resident()   # the direct scheme's state needs nothing at tree times
        return tn, active

    def rebuild_resident(self):
        """Resident mode, at a tree time: a new tree and lists, on the device
        (device_tree) or through the host (state back, host builder, state up)."""
        if self.device_tree and self._rebuild_on_device():
            return
        self.n_host_rebuilds += 1
        self.sync_state()
        if not np.all(self.t0 == self.t):
            raise AssertionError("particles not synchronised at a tree time")
        self._build_and_send()
        self.ctx.state_enable()    # the rebuild may have made a larger context
        self.ctx.state_set(self.t0, self.dt, self.m, self.x, self.v, self.a, self.j, self.pot)

    def _rebuild_on_device(self):
        self.ctx.sync()   # the step's kernels end first, so the tree timer holds the rebuild alone
        t_start = time.perf_counter()
        lock = self._dtree_lock if self._dtree_lock is not None else contextlib.nullcontext()
        with lock:
            try:
                perm = self.ctx.state_rebuild(self._dtree, self.n, self.n_leaf, self.n_crit, self.theta, self.t,
                                              out=self._perm_pin.numpy())
            except B.HTError as e:
                if e.code != -2:      # not a capacity shortfall
                    raise
                return False
            M, G, E, _ = self._dtree.sizes()
        # one pending composite, so a long run between syncs holds one array
        self._perm_pending = perm.copy() if self._perm_pending is None else self._perm_pending[perm]
        self.tree = types.SimpleNamespace(n_node=M, n_group=G, n_entries=E)
        self.t_tree = self.t
        self.n_device_rebuilds += 1
        self.timers["tree"] += time.perf_counter() - t_start
        return True

    def step(self):
        """One block step; returns (t, active ids)."""
        if self.resident:
            return self._step_resident()
        tn, active = self.begin_step()
        acc, jerk, pot = self._force(active)
        rows = self.finish_step(acc, jerk, pot)
        if rows is not None:
            t_start = time.perf_counter()
            self.ctx.set_j_particles(rows["t0"], rows["m"], rows["x"], rows["v"], rows["a"], rows["jerk"],
                                     idx=rows["idx"])
            self.timers["comm"] += time.perf_counter() - t_start
        return tn, active

    def run(self, t_end, on_step=None):
        if self.device_loop and on_step is None:
            return self._run_device_loop(t_end)
        while self.next_time() <= t_end:
            tn, act = self.step()
            if on_step is not None:
                on_step(self, tn, act)
        return self

    def _run_device_loop(self, t_end, chunk=32):
        """Block steps up to t_end, queued on the device `chunk` at a time (one
        captured graph each; steps queued past the stop do nothing but still
        cost their launches); the host only rebuilds at tree times."""
        while True:
            t_tree_next = (math.floor(self.t / self.dt_tree) + 1.0) * self.dt_tree
            t_stop = min(t_end, t_tree_next)
            t_start = time.perf_counter()
            k, t_last, psteps = self.ctx.dev_run(self.eta, self.dt_tree, t_stop, chunk)
            self._pending_dev = None
            pairs, _ = self.ctx.last_stats()
            self.n_interactions += pairs
            self.timers["force"] += time.perf_counter() - t_start
            if k == 0:
                return self       # the next block time lies beyond t_end
            self.t = t_last
            self.n_block_steps += k
            self.n_particle_steps += psteps
            if t_last == t_tree_next:
                self.rebuild_resident()

    # ------------------------------------------------------------------ diagnostics
    def energy(self):
        """Total energy at the current (synchronised) time: kinetic on the host,
        potential by direct summation on the GPU in FP64 (Section 3 computes
        the potential energy directly, not with the tree)."""
        self.sync_state()
        if not np.all(self.t0 == self.t):
            raise ValueError("energy needs all particles at the same time")
        if self._ectx is None:
            self._ectx = B.Context(n_max=self.n, node_max=0, group_max=1, list_max=1, active_max=self.n,
                                   eps2=self.eps2, precision="fp64", device=self.device)
        z = np.zeros((self.n, 3))
        self._ectx.set_j_particles(self.t0, self.m, self.x, self.v, z, z)
        self._ectx.predict(self.t)
        _, _, pot = self._ectx.force_direct(np.arange(self.n, dtype=np.int32))
        K = 0.5 * float(np.sum(self.m * np.einsum("ij,ij->i", self.v, self.v)))
        W = 0.5 * float(np.sum(self.m * pot))
        return K + W

    def close(self):
        for c in (self.ctx, self._ectx, self._dtree if self._own_dtree else None):
            if c is not None:
                c.close()
        self.ctx = self._ectx = self._dtree = None
