"""Device-resident integration: the block scheduler and the Hermite corrector
on the device (ht_dev_next_block, ht_dev_step) against the host forms."""
import sys

import numpy as np
import pytest

from paper_1602_02832_amd import binding as B
from paper_1602_02832_amd import driver
from paper_1602_02832_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("x", "v", "a", "j", "t0", "dt", "pot")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n", [1, 5, 2047, 2048, 2049, 6000, 300001])
def test_device_scheduler_matches_definition(n):
    """t_next = min(t0 + dt) and the ascending list of particles due then, for
    sizes at and around the scheduler's block boundaries."""
    say(f"device scheduler n={n}")
    rng = np.random.default_rng(n)
    dt = np.ldexp(1.0, -rng.integers(3, 12, n))
    t0 = np.floor(rng.uniform(0, 1, n) / dt) * dt
    x, v, a, j = rng.normal(size=(4, n, 3))
    m = np.full(n, 1.0 / n)
    c = B.Context(n_max=n, node_max=0, group_max=1, list_max=1, active_max=n, eps2=1e-4, precision="mixed")
    c.state_enable()
    c.state_set(t0, dt, m, x, v, a, j)
    tn, act = c.dev_next_block()
    t = t0 + dt
    want = np.flatnonzero(t == t.min())
    assert tn == t.min() and np.array_equal(act, want)
    # a second call on the same state gives the same answer
    tn2, act2 = c.dev_next_block()
    assert tn2 == tn and np.array_equal(act2, act)
    got = c.state_get(n)
    for w, g in zip((t0, dt, x, v, a, j), got):
        assert np.array_equal(w, g)
    # the binding refuses counts and arrays that do not match the state's N
    with pytest.raises(ValueError):
        c.state_get(n - 1)
    with pytest.raises(ValueError):
        c.state_set(t0, dt[:-1], m, x, v, a, j)
    assert all(np.array_equal(w, g) for w, g in zip((t0, dt, x, v, a, j), c.state_get()))
    c.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_resident_integration_equals_host_driven(prec):
    """The same run driven by the host corrector and scheduler, and resident on
    the device, through 16 tree rebuilds: the same bits at the end."""
    c = W.config("plummer2k")
    say(f"resident vs host-driven integration ({prec}) to t={c.t_end}")
    x, v, m = W.make_initial_conditions(c)
    sims = [driver.Simulation(x, v, m, eps2=c.eps2, dt_tree=c.dt_tree, eta=c.eta, theta=c.theta, n_crit=c.n_crit,
                              precision=prec, resident=r) for r in (False, True)]
    for s in sims:
        s.run(c.t_end)
    sims[1].sync_state()
    assert sims[0].n_block_steps == sims[1].n_block_steps and sims[0].t == sims[1].t == c.t_end
    order = [np.argsort(s.ids) for s in sims]
    for f in FIELDS:
        p, q = (getattr(s, f)[o] for s, o in zip(sims, order))
        assert np.array_equal(p, q), f
    e_host, e_dev = sims[0].energy(), sims[1].energy()
    assert e_host == e_dev
    for s in sims:
        s.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_device_rebuilds_equal_host_rebuilds(prec):
    """Resident runs that rebuild on the device (ht_state_rebuild: tree, lists
    and the reordered state never leave it) and through the host builder: the
    same bits after 16 tree times, in the same particle order."""
    c = W.config("plummer2k")
    say(f"device vs host rebuilds ({prec}) to t={c.t_end}")
    x, v, m = W.make_initial_conditions(c)
    sims = [driver.Simulation(x, v, m, eps2=c.eps2, dt_tree=c.dt_tree, eta=c.eta, theta=c.theta, n_crit=c.n_crit,
                              precision=prec, resident=True, device_tree=d) for d in (False, True)]
    for s in sims:
        s.run(c.t_end)
        s.sync_state()
    assert sims[1].n_device_rebuilds >= 16
    assert sims[0].n_block_steps == sims[1].n_block_steps and sims[0].t == sims[1].t == c.t_end
    assert np.array_equal(sims[0].ids, sims[1].ids)
    for f in FIELDS + ("m",):
        assert np.array_equal(getattr(sims[0], f), getattr(sims[1], f)), f
    assert sims[0].energy() == sims[1].energy()
    for s in sims:
        s.close()


def test_device_rebuilds_plummer16k_mixed():
    """The same at 16384 particles (C2's model, n_crit 256) over four tree times."""
    c = W.config("plummer16k")
    t_end = 4 * c.dt_tree
    say(f"device vs host rebuilds plummer16k to t={t_end}")
    x, v, m = W.make_initial_conditions(c)
    sims = [driver.Simulation(x, v, m, eps2=c.eps2, dt_tree=c.dt_tree, eta=c.eta, theta=c.theta, n_crit=c.n_crit,
                              precision="mixed", resident=True, device_tree=d) for d in (False, True)]
    for s in sims:
        s.run(t_end)
        s.sync_state()
    assert sims[1].n_device_rebuilds == 4
    assert np.array_equal(sims[0].ids, sims[1].ids)
    for f in FIELDS + ("m",):
        assert np.array_equal(getattr(sims[0], f), getattr(sims[1], f)), f
    for s in sims:
        s.close()


def test_device_rebuild_falls_back_when_the_tree_outgrows_the_context():
    """With no list headroom, a tree time whose tree outgrows the context (nodes,
    groups or list entries) makes ht_state_rebuild refuse (HT_ERANGE, context
    unchanged) and the driver take the host path with a larger context; the
    run still equals host rebuilds."""
    c = W.config("plummer2k")
    say("device rebuild fallback to the host path")
    x, v, m = W.make_initial_conditions(c)
    sims = [driver.Simulation(x, v, m, eps2=c.eps2, dt_tree=c.dt_tree, eta=c.eta, theta=c.theta, n_crit=c.n_crit,
                              precision="mixed", resident=True, device_tree=d, list_headroom=1.0)
            for d in (False, True)]
    for s in sims:
        s.run(c.t_end)
        s.sync_state()
    dev = sims[1]
    assert dev.n_host_rebuilds >= 1 and dev.n_host_rebuilds + dev.n_device_rebuilds == 16, \
        (dev.n_host_rebuilds, dev.n_device_rebuilds)
    assert np.array_equal(sims[0].ids, dev.ids)
    for f in FIELDS + ("m",):
        assert np.array_equal(getattr(sims[0], f), getattr(dev, f)), f
    for s in sims:
        s.close()


def test_resident_direct_equals_host_driven_direct():
    """The direct Hermite scheme resident on the device (ht_dev_step_direct)
    gives the bits of the host-driven direct run."""
    c = W.config("plummer2k")
    say(f"resident vs host-driven direct scheme to t={c.t_end}")
    x, v, m = W.make_initial_conditions(c)
    sims = [driver.Simulation(x, v, m, eps2=c.eps2, dt_tree=c.dt_tree, eta=c.eta, theta=c.theta, n_crit=c.n_crit,
                              precision="mixed", mode="direct", resident=r) for r in (False, True)]
    for s in sims:
        s.run(c.t_end)
        s.sync_state()
    assert sims[0].n_block_steps == sims[1].n_block_steps and sims[0].t == sims[1].t == c.t_end
    assert np.array_equal(sims[0].ids, sims[1].ids)
    for f in FIELDS:
        assert np.array_equal(getattr(sims[0], f), getattr(sims[1], f)), f
    for s in sims:
        s.close()


@pytest.mark.parametrize("name,t_end", [("plummer2k", None), ("plummer16k", 4.0 / 256)])
def test_device_loop_equals_step_by_step(name, t_end):
    """Block steps queued on the device (ht_dev_run: device scheduler, device
    work planner, force, corrector, no host round trip until each tree time)
    give the bits of the step-by-step resident run, through the rebuilds."""
    c = W.config(name)
    t_end = c.t_end if t_end is None else t_end
    say(f"device loop vs step by step: {name} to t={t_end}")
    x, v, m = W.make_initial_conditions(c)
    sims = [driver.Simulation(x, v, m, eps2=c.eps2, dt_tree=c.dt_tree, eta=c.eta, theta=c.theta, n_crit=c.n_crit,
                              precision="mixed", resident=True, device_tree=True, device_loop=d)
            for d in (False, True)]
    for s in sims:
        s.run(t_end)
        s.sync_state()
    assert sims[0].n_block_steps == sims[1].n_block_steps and sims[0].t == sims[1].t
    assert sims[0].n_particle_steps == sims[1].n_particle_steps
    assert sims[0].n_interactions == sims[1].n_interactions
    assert np.array_equal(sims[0].ids, sims[1].ids)
    for f in FIELDS:
        assert np.array_equal(getattr(sims[0], f), getattr(sims[1], f)), f
    for s in sims:
        s.close()


def test_device_loop_step_cap_stop_time_and_arguments():
    """ht_dev_run's contract: at most max_steps steps per call (chunks of 3 and
    4 give the bits of 7 single steps), the loop ends after the step at t_stop,
    and bad arguments are refused with the state left usable."""
    c = W.config("plummer2k")
    x, v, m = W.make_initial_conditions(c)
    say("device loop: step cap, stop time, arguments")
    mk = lambda: driver.Simulation(x, v, m, eps2=c.eps2, dt_tree=c.dt_tree, eta=c.eta, theta=c.theta,
                                   n_crit=c.n_crit, precision="mixed", resident=True, device_tree=True)
    single, chunked, stopped = mk(), mk(), mk()
    times = []
    for _ in range(7):
        tn, _ = single.step()
        times.append(tn)
    assert times[-1] < c.dt_tree                      # all seven before the first tree time
    far = c.dt_tree - 2.0**-41
    k1, t1, _ = chunked.ctx.dev_run(c.eta, c.dt_tree, far, 3)
    k2, t2, _ = chunked.ctx.dev_run(c.eta, c.dt_tree, far, 4)
    assert (k1, k2) == (3, 4) and (t1, t2) == (times[2], times[6])
    # the stop time: the loop takes the step at t_stop and stops before the next block time
    k3, t3, _ = stopped.ctx.dev_run(c.eta, c.dt_tree, times[4], 1000)
    assert (k3, t3) == (5, times[4])
    # refused calls: nothing runs, and the next good call carries on where the state is
    for args in ((-1.0, c.dt_tree, far, 4), (c.eta, 0.0, far, 4), (c.eta, c.dt_tree, float("nan"), 4),
                 (c.eta, c.dt_tree, far, 0)):
        with pytest.raises(B.HTError) as err:
            stopped.ctx.dev_run(*args)
        assert err.value.code == -1
    stopped.ctx.set_tuning(12.5, 2048)                 # the device planner needs a whole-number gather cost
    with pytest.raises(B.HTError):
        stopped.ctx.dev_run(c.eta, c.dt_tree, far, 4)
    stopped.ctx.set_tuning(12, 2048)
    k4, t4, _ = stopped.ctx.dev_run(c.eta, c.dt_tree, far, 2)
    assert (k4, t4) == (2, times[6])
    chunked.sync_state()
    stopped.sync_state()
    single.sync_state()
    for s in (chunked, stopped):
        for f in FIELDS:
            assert np.array_equal(getattr(s, f), getattr(single, f)), f
    for s in (single, chunked, stopped):
        s.close()
