"""Energy error of GPU-driven tree/Hermite runs against the opening angle, and of
the direct Hermite scheme, from the same initial conditions (Section 3 of
Fukushige & Kawai reports this experiment in its Figs. 5 and 6: energy error
grows with theta, and the tree scheme stays close to the direct one for small
theta).  The paper's parameters are kept (equal masses, eta = 0.01, eps = 1/N,
tree interval 1/64) at a size and span that run in minutes on one GPU.

    python -m paper_1602_02832_amd.energy_study [--n 16384] [--t-end 1.0] [--out file.json]
        [--resident] [--direct-t-end T]

--resident runs the integrations resident on the device (scheduler, force and
corrector there; tree times rebuilt there too).

Prints one JSON object: per run the relative energy error |E(t) - E(0)| / |E(0)|
at every multiple of 1/8 (all particles synchronised there), block steps,
particle steps and wall time.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import driver
from . import workloads as W


def run(x, v, m, *, mode, theta, eps, eta, dt_tree, n_crit, t_end, precision, every=0.125, resident=False):
    res = bool(resident)
    sim = driver.Simulation(x, v, m, eps2=eps * eps, dt_tree=dt_tree, eta=eta, theta=theta, n_crit=n_crit,
                            precision=precision, mode=mode, resident=res, device_tree=res and mode == "tree")
    e0 = sim.energy()
    errs = []
    wall = time.perf_counter()
    t_mark = every
    while t_mark <= t_end + 1e-12:
        sim.run(t_mark)
        errs.append((t_mark, abs((sim.energy() - e0) / e0)))
        print(f"  {mode} theta={theta} t={t_mark:g} dE/E={errs[-1][1]:.3e} steps={sim.n_block_steps}",
              file=sys.stderr, flush=True)
        t_mark += every
    wall = time.perf_counter() - wall
    out = dict(mode=mode, theta=theta if mode == "tree" else None, energy_error=errs,
               block_steps=sim.n_block_steps, particle_steps=sim.n_particle_steps, wall_s=wall,
               resident=res, t_end=t_end)
    sim.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--t-end", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--n-crit", type=int, default=512)
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--thetas", default="0.3,0.5,0.75")
    ap.add_argument("--no-direct", action="store_true")
    ap.add_argument("--out", default="")
    ap.add_argument("--resident", action="store_true", help="runs resident on the device")
    ap.add_argument("--direct-t-end", type=float, default=0.0, help="end of the direct run (default: --t-end)")
    args = ap.parse_args()
    if not (args.t_end > 0 and math.isfinite(args.t_end)):
        raise SystemExit("--t-end must be positive")
    x, v, m = W.plummer(args.n, args.seed)
    common = dict(eps=1.0 / args.n, eta=0.01, dt_tree=1.0 / 64, n_crit=args.n_crit, precision=args.precision)
    runs = []
    for th in (float(t) for t in args.thetas.split(",") if t):
        runs.append(run(x, v, m, mode="tree", theta=th, t_end=args.t_end, resident=args.resident, **common))
    if not args.no_direct:
        runs.append(run(x, v, m, mode="direct", theta=0.0, t_end=args.direct_t_end or args.t_end,
                        resident=args.resident, **common))
    res = dict(n=args.n, seed=args.seed, t_end=args.t_end, eps=1.0 / args.n, eta=0.01, dt_tree=1.0 / 64,
               n_crit=args.n_crit, precision=args.precision, runs=runs)
    text = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text, flush=True)


if __name__ == "__main__":
    main()
