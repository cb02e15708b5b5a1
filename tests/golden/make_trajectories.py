"""Write the stored oracle trajectories that the full-size GPU tests compare against.

Test infrastructure: this script calls only the oracle (``oracle/``) and the seeded inputs
(``rafem_inputs``); nothing here touches the GPU library.  The oracle runs at the
tolerance the parity tests use (PCG to ||r|| <= 1e-13 ||b||, reading of the stopping rule
for the 101^3 workloads), each step warm-started from the previous state.

    python tests/golden/make_trajectories.py c1     # 101^3 hex, 100 coupled steps (~1 h, 1 core)
    python tests/golden/make_trajectories.py c4     # 4 ensemble samples, 3 steps each
    python tests/golden/make_trajectories.py c2     # 161^3 Kuhn tets, 20 coupled steps (~70 min, ~20 GB)

Files (NumPy .npz, no pickled objects):

* ``c1_hex101_trajectory.npz`` -- the coupled 101^3 workload (seed 0) over 100 steps of
  1 s: T and V at 2,000 free nodes (drawn with ``default_rng(2026)``), at steps 1, 10, 20,
  ..., 100, with the 2-norms of the full fields (T, V, T - 37) at those steps and the
  oracle's PCG iteration counts of every step.
* ``c2_tet161_trajectory.npz`` -- the jittered 161^3 Kuhn-tet workload (seed 0) over 20
  steps: T and V at 2,000 free nodes (``default_rng(2029)``) after every step, with the
  full-field norms and the iteration counts.
* ``c4_ensemble_steps.npz`` -- of the 64-sample ensemble (seed 0), the smallest and the
  largest sample and two more drawn with ``default_rng(2027)``: T and V at 2,000 free nodes
  of each (``default_rng(2028 + q)``) after steps 1, 2 and 3, with the full-field norms.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import rafem_inputs as ri  # noqa: E402
from oracle.rafem import Model  # noqa: E402

TOL = 1e-13
C1_FILE = os.path.join(HERE, "c1_hex101_trajectory.npz")
C4_FILE = os.path.join(HERE, "c4_ensemble_steps.npz")
C2_FILE = os.path.join(HERE, "c2_tet161_trajectory.npz")
C1_STEPS = [1] + list(range(10, 101, 10))
N_SAMPLED = 2000


def free_sample(p, seed, count=N_SAMPLED):
    free = np.setdiff1d(np.arange(p.n_nodes), p.dir_ids)
    return np.sort(np.random.default_rng(seed).choice(free, min(count, free.size), replace=False))


def norms(T, V):
    return [np.linalg.norm(T), np.linalg.norm(V), np.linalg.norm(T - 37.0)]


def make_c1(path=C1_FILE):
    p = ri.config1(steps=100)
    nodes = free_sample(p, 2026)
    m = Model(p)
    bio = m.bioheat_system()
    T, V = p.initial_T(), p.initial_V()
    Ts, Vs, nrm, iters = [], [], [], []
    t0 = time.time()
    for k in range(1, 101):
        T, V, info = m.step(T, V, TOL, bioheat=bio)
        iters.append((info.V.iters, info.T.iters))
        if k in C1_STEPS:
            Ts.append(T[nodes])
            Vs.append(V[nodes])
            nrm.append(norms(T, V))
        print(f"c1 step {k}: V {info.V.iters} T {info.T.iters} iterations, "
              f"{time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(path, nodes=nodes, steps=np.array(C1_STEPS), T=np.array(Ts),
                        V=np.array(Vs), norms=np.array(nrm), iters=np.array(iters),
                        tol=np.array(TOL))
    print(f"wrote {path}", flush=True)


def c4_picks(probs):
    sizes = np.array([q.n for q in probs])
    lo, hi = int(np.argmin(sizes)), int(np.argmax(sizes))
    rest = np.setdiff1d(np.arange(len(probs)), [lo, hi])
    two = np.sort(np.random.default_rng(2027).choice(rest, 2, replace=False))
    return [lo, hi] + [int(q) for q in two]


def make_c4(path=C4_FILE):
    probs = ri.config4(steps=3)
    picks = c4_picks(probs)
    out = {"picks": np.array(picks), "tol": np.array(TOL)}
    for q in picks:
        p = probs[q]
        nodes = free_sample(p, 2028 + q)
        states, _ = Model(p).simulate(3, TOL)
        out[f"nodes_{q}"] = nodes
        out[f"T_{q}"] = np.array([T[nodes] for T, _ in states])
        out[f"V_{q}"] = np.array([V[nodes] for _, V in states])
        out[f"norms_{q}"] = np.array([norms(T, V) for T, V in states])
        print(f"c4 sample {q} (n={p.n}) done", flush=True)
    np.savez_compressed(path, **out)
    print(f"wrote {path}", flush=True)


def make_c2(path=C2_FILE):
    p = ri.config2(steps=20)
    nodes = free_sample(p, 2029)
    m = Model(p)
    bio = m.bioheat_system()
    T, V = p.initial_T(), p.initial_V()
    Ts, Vs, nrm, iters = [], [], [], []
    t0 = time.time()
    for k in range(1, 21):
        T, V, info = m.step(T, V, TOL, bioheat=bio)
        iters.append((info.V.iters, info.T.iters))
        Ts.append(T[nodes])
        Vs.append(V[nodes])
        nrm.append(norms(T, V))
        print(f"c2 step {k}: V {info.V.iters} T {info.T.iters} iterations, "
              f"{time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(path, nodes=nodes, steps=np.arange(1, 21), T=np.array(Ts),
                        V=np.array(Vs), norms=np.array(nrm), iters=np.array(iters),
                        tol=np.array(TOL))
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c1", "c4"]
    for w in which:
        {"c1": make_c1, "c4": make_c4, "c2": make_c2}[w]()
