"""Write the stored oracle results that the long GPU parity tests compare with.

Each case runs the FP64 oracle (and nothing else) from a seeded synthetic
droplet for 1000 steps and stores the readout moments (rho, u, T) at sampled
cells: a full plane (2D: a full row) through the droplet centre plus seeded
random cells.  The GPU runs take seconds; the oracle runs take minutes of CPU,
too long for a test, hence the stored values.

  python tests/golden/make_oracle_runs.py [case ...]

Cases (name: lattice, size, droplet radius, T/Tc, steps):
  d3q27_64cube_R10:     D3Q27 64 x 64 x 64, R = 10, T/Tc = 0.8, 1000 steps
  d3q27_128x32x40_R8:   D3Q27 128 x 32 x 40, R = 8, T/Tc = 0.8, 1000 steps
  d2q9_512sq_R40:       D2Q9 512 x 512, R = 40, T/Tc = 0.8, 1000 steps
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import oracle.thermo as TH  # noqa: E402
import synth  # noqa: E402

CASES = {
    "d3q27_64cube_R10": dict(D=3, shape=(64, 64, 64), R=10.0, Tr=0.8, steps=1000, seed=synth.SEED + 20),
    "d3q27_128x32x40_R8": dict(D=3, shape=(40, 32, 128), R=8.0, Tr=0.8, steps=1000, seed=synth.SEED + 21),
    "d2q9_512sq_R40": dict(D=2, shape=(1, 512, 512), R=40.0, Tr=0.8, steps=1000, seed=synth.SEED + 22),
}


def initial_fields(case):
    """The seeded input both sides start from (synth recipes only)."""
    c = CASES[case]
    T0 = c["Tr"] * synth.T_CRIT
    rl, rv, _ = TH.coexistence(T0)
    rho = synth.droplet(c["shape"], c["R"], rl, rv, noise=1e-4, seed=c["seed"])
    return rho, np.full(c["shape"], T0)


def sample_cells(case, n_random=2048):
    """(z, y, x) of the stored cells: the plane (row) through the centre and
    seeded random cells."""
    c = CASES[case]
    nz, ny, nx = c["shape"]
    rng = np.random.default_rng(c["seed"] + 1000)
    if c["D"] == 3:
        yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        plane = np.stack([np.full(yy.size, nz // 2), yy.ravel(), xx.ravel()], 1)
    else:
        plane = np.stack([np.zeros(nx, int), np.full(nx, ny // 2), np.arange(nx)], 1)
    rand = np.stack([rng.integers(0, nz, n_random), rng.integers(0, ny, n_random), rng.integers(0, nx, n_random)], 1)
    return np.concatenate([plane, rand]).astype(np.int64)


def path(case):
    return os.path.join(HERE, f"oracle_{case}.npz")


def run(case):
    c = CASES[case]
    nz, ny, nx = c["shape"]
    rho0, T0 = initial_fields(case)
    L = oracle.Lattice(c["D"], nx, ny, nz)
    L.set_params(**synth.params())
    L.init(rho0, T0)
    t0 = time.time()
    L.step(c["steps"])
    r, u, T, _ = L.moments()
    cells = sample_cells(case)
    z, y, x = cells[:, 0], cells[:, 1], cells[:, 2]
    np.savez_compressed(path(case), cells=cells, rho=r[z, y, x], u=u[:, z, y, x], T=T[z, y, x],
                        steps=c["steps"], shape=np.array(c["shape"]))
    print(f"{case}: {c['steps']} oracle steps in {time.time() - t0:.0f} s -> {path(case)}", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        run(name)
