"""Batched and served tree/Hermite engines: many clusters, one launch per phase.

Each cluster is an independent tree/Hermite simulation (``driver.Simulation``)
with its own j-memory, lists and block times, on one shared stream.  An
engine step advances every resident cluster by one of its own block steps:

  1. one batched j-memory update with all clusters' corrected particles;
  2. each cluster picks its next block time and active set (host) and is
     predicted there;
  3. one batched force launch over all clusters' work items (+ one split
     reduction), results written straight into pinned host memory;
  4. each cluster corrects its particles on the host; clusters at a tree time
     rebuild their tree and lists.

The resident engine can run as a device loop (``device_loop=True``): one
``Engine.step`` call queues up to ``loop_steps`` engine steps (scheduler,
device planner, one force launch and one corrector launch for all clusters
per engine step, captured in HIP graphs) with no host round trip between
them.  A cluster that reaches a tree time stops there; it is rebuilt on its
own stream by a worker thread while later calls run the other clusters, and
sits those calls out until its rebuild is done (the set of clusters in a
call stays the same, so the captured graph is kept).  Each cluster's block
steps, and their bits, are those of the step-by-step engine.

The resident engine can split its clusters into lanes, each with a stream
and a batch object of its own, stepped in turn: while the device works on
one lane's step, the host waits for the next lane's scheduler and plans that
lane, so host planning and device work overlap (one lane by default: every
lane adds its own scheduler upload, synchronisation and launches).

Work plans are per cluster, so a cluster's forces are bit-identical alone and
in any mix (and in any lane).  ``Server`` adds continuous batching: requests for whole cluster
runs arrive over time and are admitted while device memory and batch slots
allow; finished runs leave and free their slots.
"""
from __future__ import annotations

import collections
import concurrent.futures
import ctypes
import dataclasses
import math
import threading
import time

import numpy as np

from . import binding as B
from . import driver
from . import workloads as W


# numpy view of htb_cluster (include/htree_host.h): every field is 8 bytes
_HTB_CLUSTER = np.dtype([("n", np.int64), ("eta", np.float64), ("dt_tree", np.float64)] +
                        [(f, np.uint64) for f in ("t0", "dt", "x", "v", "a", "jerk", "m", "pot", "active")] +
                        [("n_active", np.int64), ("t_next", np.float64)])
assert _HTB_CLUSTER.itemsize == ctypes.sizeof(B.HtbCluster)


@dataclasses.dataclass
class RunSpec:
    """A cluster run: a Plummer model of n particles, `steps` block steps."""

    key: int
    n: int
    seed: int
    steps: int
    theta: float = 0.5
    eta: float = 0.01
    dt_tree: float = 1.0 / 256
    n_crit: int = 256
    eps: float | None = None        # default 4/n
    mass_seed: int | None = None


class Cluster:
    """One cluster run: prepared on the host (initial conditions and the first
    tree, which fix its device footprint), then activated (context, upload,
    first forces) when it becomes resident."""

    def __init__(self, spec: RunSpec, precision: str, stream, device: int = 0, list_headroom: float = 1.5,
                 resident: bool = False, tree=None, tree_lock=None):
        self.spec, self.precision, self.stream, self.device = spec, precision, stream, device
        self.lane = 0            # the engine lane whose stream `stream` is (set by Engine.new_cluster)
        self.resident = resident
        # a shared device tree builder for rebuilds on the device (resident runs it fits)
        self.tree, self.tree_lock = tree, tree_lock
        self.list_headroom = list_headroom
        x, v, m = W.plummer(spec.n, spec.seed)
        if spec.mass_seed is not None:
            m = W.salpeter_masses(spec.n, spec.mass_seed)
        self._ics = (x, v, m)
        z = np.zeros_like(x)
        tr = B.HostTree(x, v, z, z, m, 1, spec.n_crit, spec.theta)
        h = list_headroom
        self.caps = (max(int(tr.n_node * h), 64), max(int(tr.n_group * h), 16), max(int(tr.n_entries * h), 1024))
        # the configuration the context will be created with, and the device bytes it will hold
        self.cfg = context_config(spec.n, *self.caps, precision, device)
        self.reserve = workspace_bytes_of(self.cfg) + (B.state_bytes(self.cfg) if resident else 0)
        self.sim = None
        self.pending = (0, 0)    # (first row, count) of its update rows in the engine's row buffer
        self.steps_done = 0
        self.active_sum = 0
        self._cache = None       # (handle, t0 array, htb_cluster record, active-buffer address, context, arrays)

    def activate(self):
        if self.sim is None:
            spec = self.spec
            eps = spec.eps if spec.eps is not None else 4.0 / spec.n
            x, v, m = self._ics
            self.sim = driver.Simulation(x, v, m, eps2=eps * eps, dt_tree=spec.dt_tree, eta=spec.eta,
                                         theta=spec.theta, n_crit=spec.n_crit, precision=self.precision,
                                         device=self.device, stream=self.stream, list_headroom=self.list_headroom,
                                         resident=self.resident, device_tree=self.tree is not None, tree=self.tree,
                                         tree_lock=self.tree_lock)
            self._ics = None

    @property
    def ctx(self):
        return self.sim.ctx

    @property
    def done(self):
        return self.steps_done >= self.spec.steps

    def footprint(self):
        """Device bytes this run holds (its context workspace, and its state when resident)."""
        if self.sim is None:
            return self.reserve
        ctx = self.sim.ctx
        return ctx.workspace_bytes + (B.state_bytes(ctx.cfg) if self.resident else 0)

    def close(self):
        if self.sim is not None:
            self.sim.close()


def context_config(n, node_max, group_max, list_max, precision="mixed", device=0):
    """The ht_config of a run's context (as driver.Simulation creates it)."""
    return B.HtConfig(device, B.HT_PREC[precision], 0, int(n), int(node_max), int(group_max), int(list_max), int(n),
                      1e-4, None)


def workspace_bytes_of(cfg):
    """ht_workspace_bytes of a context configuration."""
    out = ctypes.c_size_t()
    if B.device_lib().ht_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)) != 0:
        raise ValueError("bad context size")
    return int(out.value)


def workspace_bytes(n, node_max, group_max, list_max, precision="mixed"):
    """ht_workspace_bytes of a context for one run."""
    return workspace_bytes_of(context_config(n, node_max, group_max, list_max, precision))


class Engine:
    """Advances a set of clusters one block step each per engine step."""

    def __init__(self, precision="mixed", device=0, max_clusters=256, max_active=1 << 21, max_items=1 << 20,
                 max_rows=1 << 21, rebuild_workers=4, resident=False, device_tree=False, tree_n_max=0, lanes=None,
                 device_loop=False, loop_steps=32):
        import torch

        # device_loop (resident only): each step() call runs up to loop_steps engine steps on the
        # device (ht_batch_dev_run); tree times are rebuilt between calls
        self.device_loop = bool(device_loop)
        self.loop_steps = int(loop_steps)
        if self.device_loop and not resident:
            raise ValueError("the device loop needs the resident engine")
        if self.device_loop and not (1 <= self.loop_steps <= 4096):
            raise ValueError("loop_steps must be in [1, 4096]")
        self.engine_steps = 0   # engine steps taken (a device-loop call takes several)
        self._loop_view = None  # device loop: (composition generation, clusters, arrays)
        self._loop_gen = 0      # changes when clusters join or leave the device loop

        # resident: each cluster's particle state stays on the device; the block
        # scheduler and the corrector of all clusters run there in batched launches
        self.resident = bool(resident)
        # device_tree (resident only): tree times rebuild on the device with one
        # builder shared by all clusters of up to tree_n_max particles (larger
        # ones rebuild through the host); rebuild workers take turns on it
        self.tree = None
        self.tree_lock = threading.Lock()
        if device_tree:
            if not resident:
                raise ValueError("device rebuilds need the resident engine")
            if tree_n_max < 1:
                raise ValueError("tree_n_max must be positive")
            self._tree_stream = torch.cuda.Stream(device=device)
            self.tree = B.DeviceTree(n_max=int(tree_n_max), device=device, stream=self._tree_stream.cuda_stream)
            self.tree_n_max = int(tree_n_max)
        self.torch = torch
        self.precision, self.device = precision, device
        # lanes (resident only): groups of clusters on streams of their own, stepped out of phase
        self.n_lanes = int(lanes) if lanes is not None else 1
        if self.n_lanes < 1 or (self.n_lanes > 1 and not self.resident):
            raise ValueError("more than one lane needs the resident engine")
        self.streams = [torch.cuda.Stream(device=device) for _ in range(self.n_lanes)]
        # device loop: the clusters' contexts live on a stream of their own, so that a
        # cluster's rebuild runs beside the batch's loop calls
        self._ctx_stream = torch.cuda.Stream(device=device) if self.device_loop else None
        self.batches = [B.Batch(stream=st.cuda_stream, max_clusters=max_clusters, max_items=max_items,
                                max_active=max_active, max_rows=max_rows, device=device) for st in self.streams]
        self.stream, self.batch = self.streams[0], self.batches[0]   # the host-driven engine's one lane
        self._next_lane = 0
        self.max_clusters, self.max_active = max_clusters, max_active
        self.clusters: list[Cluster] = []
        dev = f"cuda:{device}"
        # results of all clusters of a step, cluster k at rows offs[k]..; row slices stay contiguous
        # The force launch writes its results straight into pinned host memory (the host
        # corrects from them next), so an engine step has no device-to-host copy.
        self.h_acc = torch.empty((max_active, 3), dtype=torch.float64, pin_memory=True)
        self.h_jerk = torch.empty((max_active, 3), dtype=torch.float64, pin_memory=True)
        self.h_pot = torch.empty(max_active, dtype=torch.float64, pin_memory=True)
        # corrected particles of every cluster, written by the native corrector, read by the next update
        self._h_rows_t = torch.empty(max_active * B.HT_ROW.itemsize, dtype=torch.uint8, pin_memory=True)
        self.h_rows = self._h_rows_t.numpy().view(B.HT_ROW)
        self._rows_base = np.uint64(self._h_rows_t.data_ptr())
        self.step_ms = []
        self.pairs = 0
        self.equiv_pairs = 0
        self.wall = 0.0
        # where an engine step's time goes: host before the launch, waiting for the device, host after
        self.phase = {"host_begin": 0.0, "device_wait": 0.0, "host_finish": 0.0}
        self.subphase = collections.defaultdict(float)
        # tree rebuilds run beside the engine loop; a rebuilding cluster sits out until it is resident again
        self.pool = concurrent.futures.ThreadPoolExecutor(max_workers=rebuild_workers) if rebuild_workers else None
        self.rebuilding = {}
        # the resident step's per-lane views (cluster lists and their arrays), rebuilt only when the
        # set of stepping clusters changes: a cluster added, removed, finished, or in or out of a rebuild
        self._gen = 0
        self._views_gen = -1
        self._views = []
        self._ptr = (self.h_acc.data_ptr(), self.h_jerk.data_ptr(), self.h_pot.data_ptr())
        self.tuning = None      # (gather_cost, target_items) for every cluster, None = library defaults
        del dev

    def new_cluster(self, spec: RunSpec) -> Cluster:
        shared = self.tree is not None and spec.n <= self.tree_n_max
        lane = self._next_lane                 # lanes in turn, fixed for the cluster's life
        self._next_lane = (lane + 1) % self.n_lanes
        stream = self._ctx_stream if self.device_loop else self.streams[lane]
        c = Cluster(spec, self.precision, stream.cuda_stream, self.device, resident=self.resident,
                    tree=self.tree if shared else None, tree_lock=self.tree_lock if shared else None)
        c.lane = lane
        return c

    def add(self, c: Cluster):
        if len(self.clusters) >= self.max_clusters:
            raise RuntimeError("engine is full")
        c.activate()
        if self.tuning is not None:
            c.ctx.set_tuning(*self.tuning)
        self.clusters.append(c)
        self._gen += 1
        self._loop_gen += 1

    def set_tuning(self, gather_cost: float, target_items: float):
        """Work-plan tuning (ht_set_tuning) for every resident and future cluster."""
        self.tuning = (float(gather_cost), float(target_items))
        self.drain()
        for c in self.clusters:
            c.ctx.set_tuning(*self.tuning)

    def autotune(self, candidates=((12, 64), (12, 256), (12, 1024), (12, 2048), (8, 256), (16, 256), (16, 2048)),
                 steps: int = 6, rounds: int = 2):
        """Pick the work-plan tuning with the least engine wall time per
        interaction on the engine's own clusters.  The wall time holds the
        host's planning (every cluster plans towards its own item target, so a
        batched launch over many clusters needs a far smaller target per
        cluster than one cluster alone) as well as the device's work.  Each
        candidate runs `steps` engine steps per round; rounds interleave the
        candidates so the drift of the step mix averages out.  Advances the
        clusters; returns the choice and the measured ms per 1e9 interactions
        of every candidate."""
        score = {tuple(c): [0.0, 0] for c in candidates}
        for _ in range(rounds):
            for cand in score:
                self.set_tuning(*cand)
                self.step()                         # the first step after a change is not timed
                for st in self.streams:
                    st.synchronize()
                p0, t0 = self.pairs, time.perf_counter()
                for _ in range(steps):
                    self.step()
                for st in self.streams:
                    st.synchronize()
                score[cand][0] += 1e3 * (time.perf_counter() - t0)
                score[cand][1] += self.pairs - p0
        per = {c: 1e9 * v[0] / max(v[1], 1) for c, v in score.items()}
        best = min(per, key=per.get)
        self.set_tuning(*best)
        return best, per

    def set_timing(self, enable=True):
        """Kernel timing of the force launches of every lane."""
        for b in self.batches:
            b.set_timing(enable)

    def kernel_timing(self):
        """(force-kernel ms, launches, pairs) since the last call, over all lanes."""
        ms, launches, pairs = 0.0, 0, 0
        for b in self.batches:
            m_, l_, p_ = b.kernel_timing()
            ms, launches, pairs = ms + m_, launches + l_, pairs + p_
        return ms, launches, pairs

    def _refresh(self, c: Cluster):
        """The cluster's htb_cluster record, context handle and active-buffer
        address, recomputed only when a rebuild replaced its arrays or context."""
        sim = c.sim
        cc = c._cache
        # a rebuild replaces all of a cluster's host arrays at once (and may replace its context)
        if cc is None or cc[1] is not sim.t0 or cc[4] is not sim.ctx:
            arrays = (sim.t0, sim.dt, sim.x, sim.v, sim.a, sim.j, sim.m, sim.pot, sim._act_buf)
            rec = (sim.n, sim.eta, sim.dt_tree) + tuple(a.ctypes.data for a in arrays) + (0, 0.0)
            cc = c._cache = (sim.ctx.handle.value, sim.t0, rec, sim._act_buf.ctypes.data, sim.ctx, arrays)
        return cc

    def _collect_rebuilds(self, wait=False):
        for c, fut in list(self.rebuilding.items()):
            if wait or fut.done():
                fut.result()
                del self.rebuilding[c]
                self._gen += 1

    def step(self):
        """One engine step over all resident clusters; returns the clusters
        that finished their run in this step."""
        t0 = time.perf_counter()
        self._collect_rebuilds()
        if self.device_loop:
            return self._step_loop(t0)
        if self.resident:
            views = self._lane_views()
            if not views:
                if self.rebuilding:
                    self._collect_rebuilds(wait=True)
                return []
            return self._step_resident(views, t0)
        cl = [c for c in self.clusters if not c.done and c not in self.rebuilding]
        if not cl:
            if self.rebuilding:
                self._collect_rebuilds(wait=True)
            return []
        n_cl = len(cl)
        caches = [self._refresh(c) for c in cl]
        view = np.array([cc[2] for cc in caches], dtype=_HTB_CLUSTER)     # the htb_cluster records
        handles = np.fromiter((cc[0] for cc in caches), dtype=np.uint64, count=n_cl)
        act_ptr = np.fromiter((cc[3] for cc in caches), dtype=np.uint64, count=n_cl)
        # 1. j-memory updates from the previous step (one kernel reading pinned rows)
        pend_n = np.fromiter((c.pending[1] for c in cl), dtype=np.int32, count=n_cl)
        sel = np.flatnonzero(pend_n)
        if sel.size:
            pend_off = np.fromiter((c.pending[0] for c in cl), dtype=np.uint64, count=n_cl)
            h = np.ascontiguousarray(handles[sel])
            nr = np.ascontiguousarray(pend_n[sel])
            rp = np.ascontiguousarray(self._rows_base + np.uint64(B.HT_ROW.itemsize) * pend_off[sel])
            # the rows sit in pinned memory that is not rewritten before this step's synchronisation
            self.batch.update_async_raw(sel.size, h.ctypes.data, nr.ctypes.data, rp.ctypes.data, pinned=True)
        ta = time.perf_counter()
        # 2. next block time and active set of every cluster (one native call)
        tb = ta
        B.next_block_many_raw(n_cl, view.ctypes.data)
        tc = time.perf_counter()
        t_next = np.ascontiguousarray(view["t_next"])
        n_act = view["n_active"].astype(np.int64)
        offs = np.zeros(n_cl, dtype=np.int64)
        np.cumsum(n_act[:-1], out=offs[1:])
        total = int(n_act.sum())
        if total > self.max_active:
            raise RuntimeError("active particles over the engine capacity")
        # 3-4. predict every cluster at its own block time, one force launch for all
        B.predict_many_raw(n_cl, handles.ctypes.data, t_next.ctypes.data)
        td = time.perf_counter()
        pa, pj, pp = self._ptr
        uo = offs.astype(np.uint64)
        na32 = n_act.astype(np.int32)
        outs = [np.ascontiguousarray(np.uint64(base) + np.uint64(w) * uo) for base, w in ((pa, 24), (pj, 24), (pp, 8))]
        self.batch.force_async_raw(n_cl, handles.ctypes.data, na32.ctypes.data, act_ptr.ctypes.data,
                                   outs[0].ctypes.data, outs[1].ctypes.data, outs[2].ctypes.data)
        pairs, _ = self.batch.last_stats()
        t1 = time.perf_counter()
        self.stream.synchronize()
        t2 = time.perf_counter()
        # 5. corrector, new steps and update rows of every cluster (one native call)
        rebuild = np.zeros(n_cl, dtype=np.int32)
        B.correct_many_raw(n_cl, view.ctypes.data, offs.ctypes.data, self._ptr[0], self._ptr[1], self._ptr[2],
                           offs.ctypes.data, int(self._rows_base), rebuild.ctypes.data)
        te = time.perf_counter()
        finished = []
        for k, c in enumerate(cl):
            sim = c.sim
            n = int(n_act[k])
            sim.t = float(t_next[k])
            sim.n_block_steps += 1
            sim.n_particle_steps += n
            c.steps_done += 1
            c.active_sum += n
            if rebuild[k]:
                c.pending = (0, 0)          # tree time: new tree, lists, full upload
                if self.pool is not None:
                    self.rebuilding[c] = self.pool.submit(sim._build_and_send)
                else:
                    sim._build_and_send()
            else:
                c.pending = (int(offs[k]), n)
            if c.done:
                finished.append(c)
        t3 = time.perf_counter()
        dt = t3 - t0
        self.phase["host_begin"] += t1 - t0
        self.phase["device_wait"] += t2 - t1
        self.phase["host_finish"] += t3 - t2
        sub = self.subphase
        sub["update"] += ta - t0
        sub["structs"] += tb - ta
        sub["next_block"] += tc - tb
        sub["predict"] += td - tc
        sub["plan_launch"] += t1 - td
        sub["correct"] += te - t2
        sub["bookkeeping"] += t3 - te
        self.step_ms.append(1e3 * dt)
        self.engine_steps += 1
        self.wall += dt
        self.pairs += pairs
        self.equiv_pairs += int(sum(int(n) * (c.sim.n - 1) for c, n in zip(cl, n_act)))
        return finished

    def _lane_views(self):
        """Per lane with stepping clusters: (batch, clusters, context handles,
        eta, dt_tree, N - 1, output buffers), cached until the set changes."""
        if self._views_gen == self._gen:
            return self._views
        cl = [c for c in self.clusters if not c.done and c not in self.rebuilding]
        views = []
        for lane, batch in enumerate(self.batches):
            lc = [c for c in cl if c.lane == lane]
            if not lc:
                continue
            n_cl = len(lc)
            handles = np.fromiter((self._refresh(c)[0] for c in lc), dtype=np.uint64, count=n_cl)
            eta = np.fromiter((c.sim.eta for c in lc), dtype=np.float64, count=n_cl)
            dtt = np.fromiter((c.sim.dt_tree for c in lc), dtype=np.float64, count=n_cl)
            nm1 = np.fromiter((c.sim.n - 1 for c in lc), dtype=np.int64, count=n_cl)
            outs = (np.empty(n_cl), np.empty(n_cl, dtype=np.int64), np.empty(n_cl, dtype=np.uint64))
            views.append((batch, lc, handles, eta, dtt, nm1, outs))
        self._views, self._views_gen = views, self._gen
        return views

    def _step_resident(self, views, t0):
        """Engine step with the clusters' state on the device, lane by lane:
        one batched scheduler (and the lane's one synchronisation), one batched
        force and one batched corrector per lane; the host only plans the work.
        Lanes run on streams of their own, so the device works on one lane
        while the host waits for and plans the next."""
        finished = []
        pairs = 0
        equiv = 0
        t_sync = t_plan = 0.0
        changed = False
        for batch, lc, handles, eta, dtt, nm1, (t_next, n_act, act_ptr) in views:
            ta = time.perf_counter()
            n_cl = len(lc)
            batch.dev_next_block_raw(n_cl, handles.ctypes.data, t_next.ctypes.data, n_act.ctypes.data,
                                     act_ptr.ctypes.data)
            tb = time.perf_counter()
            batch.dev_step_raw(n_cl, handles.ctypes.data, eta.ctypes.data, dtt.ctypes.data)
            pairs += batch.last_stats()[0]
            tc = time.perf_counter()
            equiv += int(np.dot(n_act, nm1))
            for c, t, n in zip(lc, t_next.tolist(), n_act.tolist()):
                sim = c.sim
                sim.t = t
                sim.n_block_steps += 1
                sim.n_particle_steps += n
                c.steps_done += 1
                c.active_sum += n
                if c.steps_done >= c.spec.steps:
                    finished.append(c)
                    changed = True
            for k in np.flatnonzero(np.fmod(t_next, dtt) == 0.0).tolist():   # tree time: rebuild
                c = lc[k]
                changed = True
                if self.pool is not None:
                    self.rebuilding[c] = self.pool.submit(c.sim.rebuild_resident)
                else:
                    c.sim.rebuild_resident()
            t_sync += tb - ta
            t_plan += tc - tb
        if changed:
            self._gen += 1
        t3 = time.perf_counter()
        dt = t3 - t0
        self.phase["host_begin"] += t_sync      # scheduler launches and the lanes' synchronisations
        self.phase["device_wait"] += 0.0
        self.phase["host_finish"] += dt - t_sync   # planning, launches, bookkeeping
        sub = self.subphase
        sub["schedule_sync"] += t_sync
        sub["plan_launch"] += t_plan
        sub["bookkeeping"] += dt - t_sync - t_plan
        self.step_ms.append(1e3 * dt)
        self.engine_steps += 1
        self.wall += dt
        self.pairs += pairs
        self.equiv_pairs += equiv
        return finished

    def _loop_clusters(self):
        """The clusters of the device loop's calls (every unfinished one, also
        while it is being rebuilt) and their fixed arrays, cached until a
        cluster joins or leaves or gets a new context."""
        lv = self._loop_view
        if lv is not None and lv[0] == self._loop_gen:
            return lv[1:]
        lc = [c for c in self.clusters if not c.done]
        handles = np.fromiter((c.sim.ctx.handle.value for c in lc), dtype=np.uint64, count=len(lc))
        eta = np.fromiter((c.sim.eta for c in lc), dtype=np.float64, count=len(lc))
        dtt = np.fromiter((c.sim.dt_tree for c in lc), dtype=np.float64, count=len(lc))
        nm1 = np.fromiter((c.sim.n - 1 for c in lc), dtype=np.int64, count=len(lc))
        self._loop_view = (self._loop_gen, lc, handles, eta, dtt, nm1)
        return self._loop_view[1:]

    def _step_loop(self, t0):
        """Up to loop_steps engine steps on the device.  Every cluster stops at
        its next tree time or at the end of its run; one stopped at a tree time
        is handed to a rebuild worker and sits out the calls until it is done."""
        lc, handles, eta, dtt, nm1 = self._loop_clusters()
        if not lc:
            if self.rebuilding:
                self._collect_rebuilds(wait=True)
            return []
        busy = np.fromiter((c in self.rebuilding for c in lc), dtype=bool, count=len(lc))
        if busy.all():                       # every cluster is being rebuilt: wait for one
            next(iter(self.rebuilding.values())).result()
            self._collect_rebuilds()
            busy = np.fromiter((c in self.rebuilding for c in lc), dtype=bool, count=len(lc))
        t_stop = np.array([(math.floor(c.sim.t / c.sim.dt_tree) + 1.0) * c.sim.dt_tree for c in lc])
        left = np.array([0 if b else c.spec.steps - c.steps_done for c, b in zip(lc, busy)], dtype=np.int32)
        steps, t_last, psteps, pr, step_ms = self.batch.dev_run(handles, eta, dtt, t_stop, left, self.loop_steps)
        finished = []
        changed = False
        for k in np.flatnonzero(steps).tolist():
            c = lc[k]
            sim = c.sim
            sim.t = float(t_last[k])
            sim.n_block_steps += int(steps[k])
            sim.n_particle_steps += int(psteps[k])
            c.steps_done += int(steps[k])
            c.active_sum += int(psteps[k])
            if c.done:
                finished.append(c)
                changed = True
            elif t_last[k] == t_stop[k]:     # tree time: rebuilt beside the next calls
                if self.pool is not None:
                    self.rebuilding[c] = self.pool.submit(self._loop_rebuild, c)
                else:
                    self._loop_rebuild(c)
        if changed:
            self._gen += 1
            self._loop_gen += 1
        dt = time.perf_counter() - t0
        self.phase["device_wait"] += dt
        self.engine_steps += len(step_ms)
        self.step_ms.extend(step_ms.tolist())
        self.wall += dt
        self.pairs += int(pr.sum())
        self.equiv_pairs += int(np.dot(psteps, nm1))
        return finished

    def _loop_rebuild(self, c):
        h = c.sim.ctx.handle.value
        c.sim.rebuild_resident()
        if c.sim.ctx.handle.value != h:      # a larger context (host fallback): the loop's set changed
            self._loop_gen += 1

    def drain(self):
        """Wait for rebuilds in flight."""
        self._collect_rebuilds(wait=True)

    def remove(self, c: Cluster):
        if c in self.rebuilding:
            self.rebuilding.pop(c).result()
        self.clusters.remove(c)
        self._gen += 1
        self._loop_gen += 1

    def close(self):
        self.drain()
        if self.pool is not None:
            self.pool.shutdown(wait=True)
        for c in self.clusters:
            c.close()
        self.clusters = []
        for b in self.batches:
            b.close()
        if self.tree is not None:
            self.tree.close()
            self.tree = None


@dataclasses.dataclass
class Request:
    spec: RunSpec
    arrival: float                 # seconds after the start of the run
    admitted: float = math.nan
    finished: float = math.nan
    cluster: Cluster | None = None
    reserved: int = 0
    rid: int = -1                  # its reservation in the server's pool
    refused: bool = False          # larger than the device-memory budget


class Server:
    """Continuous batching of cluster-run requests on one engine.

    Requests wait in arrival order; the head of the queue is admitted as soon
    as its device-memory reservation fits the budget (ht_cluster_admit on a
    pool of hbm_budget bytes, which also holds the engine's shared tree
    builder) and a batch slot is free (no overtaking, so no request starves).
    A request larger than the whole budget, or one that cannot fit even with
    nothing resident, is refused.  Every engine step advances all resident
    runs; a run leaves the step it finishes and frees its memory.
    """

    def __init__(self, engine: Engine, hbm_budget: int, max_resident: int, keep_finished: bool = False):
        self.engine, self.budget, self.max_resident = engine, int(hbm_budget), int(max_resident)
        self.keep_finished = keep_finished
        self.pool = B.Pool(self.budget, device=engine.device)
        self.resident: list[Request] = []
        self.done: list[Request] = []
        self.refused: list[Request] = []
        self.max_used = 0
        self.max_waiting = 0
        # the shared tree builder's arrays count against the budget (they grow with the largest tree)
        self._tree_id = None
        if engine.tree is not None:
            self._tree_id = self.pool.reserve(engine.tree.device_bytes())
            if self._tree_id is None:
                raise ValueError("the engine's tree builder alone exceeds the device-memory budget")

    @property
    def used(self):
        return self.pool.usage()[0]

    def _track(self):
        if self._tree_id is not None:
            self.pool.resize(self._tree_id, self.engine.tree.device_bytes())
        for r in self.resident:
            grown = r.cluster.footprint()     # a run whose lists outgrew their headroom got a larger context
            if grown != r.reserved:
                self.pool.resize(r.rid, grown)
                r.reserved = grown
        self.max_used = max(self.max_used, self.used)

    def run(self, requests: list[Request], clock=time.perf_counter):
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque[Request] = collections.deque()
        t_start = clock()
        while pending or waiting or self.resident:
            now = clock() - t_start
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            self.max_waiting = max(self.max_waiting, len(waiting))
            while waiting and len(self.resident) < self.max_resident:
                head = waiting[0]
                if head.cluster is None:               # host preparation fixes the footprint
                    head.cluster = self.engine.new_cluster(head.spec)
                try:
                    rid, need = self.pool.admit(head.cluster.cfg, head.cluster.resident)
                except B.HTError as e:                 # larger than the whole budget: never fits
                    if e.code != -2:
                        raise
                    self._refuse(waiting.popleft(), clock() - t_start)
                    continue
                if rid is None:
                    if not self.resident:              # does not fit even with nothing resident
                        self._refuse(waiting.popleft(), clock() - t_start)
                        continue
                    break
                waiting.popleft()
                head.rid, head.reserved = rid, need
                self.engine.add(head.cluster)          # activates: context, upload, first forces
                head.admitted = clock() - t_start
                self.resident.append(head)
            self.max_used = max(self.max_used, self.used)
            if not self.resident:
                if pending:
                    delay = pending[0].arrival - (clock() - t_start)
                    if delay > 0:
                        time.sleep(min(delay, 0.05))
                continue
            finished = self.engine.step()
            self._track()
            now = clock() - t_start
            for c in finished:
                req = next(r for r in self.resident if r.cluster is c)
                req.finished = now
                self.resident.remove(req)
                self.engine.remove(c)
                self.pool.release(req.rid)
                if not self.keep_finished:
                    c.close()
                    req.cluster = None
                self.done.append(req)
        return self.done

    def _refuse(self, req: Request, now: float):
        req.refused = True
        req.finished = now
        if req.cluster is not None:
            req.cluster.close()
            req.cluster = None
        self.refused.append(req)

    def close(self):
        self.pool.close()


def poisson_arrivals(count: int, rate: float, seed: int):
    """Arrival times (seconds) of a Poisson process with the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, count))


def percentile(values, q):
    return float(np.percentile(np.asarray(values, dtype=np.float64), q)) if len(values) else math.nan
