"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module holds only input recipes: initial density profiles, seeded noise,
the batched-domain table and network initial weights.  It contains none of
the method's arithmetic, so both the CPU oracle and the HIP library can be fed
the very same arrays.

Conventions: scalar fields are float64 arrays of shape (nz, ny, nx) with x
fastest; the default seed is 250800577 and a workload k uses seed + k.
"""
from __future__ import annotations

import math

import numpy as np

SEED = 250800577

# Model parameters of every workload (lattice units, R = 1).  The paper gives
# none; b = 1/3 puts the critical density at 1, RT_c = 0.02 keeps the liquid's
# adiabatic sound speed below 0.5 lattice units down to T/Tc = 0.65, and
# kappa = 0.1 gives interfaces of about 7 (T/Tc = 0.65) to 26 (0.97) cells.
R_GAS = 1.0
B_EXCL = 1.0 / 3.0
T_CRIT = 0.02
A_ATTR = 27.0 * B_EXCL * R_GAS * T_CRIT / 8.0
KAPPA = 0.1
TAU = 1.0
LAMBDA = 1.0
RHO_CRIT = 1.0 / (3.0 * B_EXCL)

# The same fluid with Carnahan-Starling's hard-sphere contact factor in
# Enskog's pressure: round values near the van der Waals critical point above
# (rho_c ~ 1.003, RT_c ~ 0.01995 with eta_c = b rho_c/4 = 0.1304).
B_CS = 0.52
A_CS = 0.0275


def params(kappa: float = KAPPA) -> dict:
    return dict(R=R_GAS, a=A_ATTR, b=B_EXCL, kappa=kappa, tau=TAU, lam=LAMBDA)


def params_cs(kappa: float = KAPPA) -> dict:
    """Parameters of the Carnahan-Starling workloads (eos = "cs")."""
    return dict(R=R_GAS, a=A_CS, b=B_CS, kappa=kappa, tau=TAU, lam=LAMBDA, eos="cs")


def uniform_noise(shape, amplitude, seed):
    """U[-amplitude, amplitude) noise from numpy's PCG64 stream for `seed`."""
    rng = np.random.default_rng(seed)
    return amplitude * rng.uniform(-1.0, 1.0, size=shape)


def splitmix_uniform(n, seed):
    """The counter-based generator the library's initialisers draw from:
    splitmix64 (Steele, Lea & Flood, OOPSLA 2014).  Value c (c = 0 .. n-1) is
    output c + 1 of the stream `seed`: the state seed + (c + 1) gamma,
    gamma = 0x9E3779B97F4A7C15, mixed by z ^= z >> 30, z *= 0xBF58476D1CE4E5B9,
    z ^= z >> 27, z *= 0x94D049BB133111EB, z ^= z >> 31 (all modulo 2^64), and
    taken as a double in [0, 1) from its top 53 bits."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.arange(n, dtype=np.uint64) + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def splitmix_noise(shape, amplitude, seed):
    """U[-amplitude, amplitude) from splitmix_uniform over the cells in
    linear order (x fastest)."""
    n = int(np.prod(shape))
    return (amplitude * (2.0 * splitmix_uniform(n, seed) - 1.0)).reshape(shape)


def _noise(shape, amplitude, seed, rng):
    return (splitmix_noise if rng == "splitmix" else uniform_noise)(shape, amplitude, seed)


def slab(shape, rho_l, rho_v, width=2.0, noise=1e-3, seed=SEED + 1, rng="pcg64", x0=None, x1=None):
    """Flat liquid slab along x between x0 = nx/4 and x1 = 3nx/4 (two interfaces).

    rho = rho_v + (rho_l - rho_v)/2 [tanh((x - x0)/W) - tanh((x - x1)/W)],
    times (1 + noise * U[-1, 1)) with U from numpy's PCG64 (rng = "pcg64") or
    from splitmix_uniform (rng = "splitmix", the library initialisers' noise).
    """
    nz, ny, nx = shape
    x0 = nx / 4.0 if x0 is None else x0
    x1 = 3.0 * nx / 4.0 if x1 is None else x1
    x = np.arange(nx, dtype=np.float64)
    prof = rho_v + 0.5 * (rho_l - rho_v) * (np.tanh((x - x0) / width) - np.tanh((x - x1) / width))
    rho = np.broadcast_to(prof, shape).copy()
    if noise:
        rho *= 1.0 + _noise(shape, noise, seed, rng)
    return rho


def droplet(shape, radius, rho_l, rho_v, width=2.0, noise=1e-4, seed=SEED + 2, centre=None, rng="pcg64"):
    """Droplet of radius R centred at (n-1)/2 on every axis (2D when nz = 1).

    rho = (rho_l + rho_v)/2 - (rho_l - rho_v)/2 tanh((r - R)/W),
    times (1 + noise * U[-1, 1)) (rng as for slab).
    """
    nz, ny, nx = shape
    if centre is None:
        centre = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2
    if nz > 1:
        r2 = r2 + (z - centre[2]) ** 2
    r = np.sqrt(r2)
    rho = 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh((r - radius) / width)
    if noise:
        rho *= 1.0 + _noise(shape, noise, seed, rng)
    return rho


def radius_field(shape, centre=None):
    """Distance of every cell from the droplet centre (same convention as droplet())."""
    nz, ny, nx = shape
    if centre is None:
        centre = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2
    if nz > 1:
        r2 = r2 + (z - centre[2]) ** 2
    return np.sqrt(r2)


def batch_table(n=64, seed=SEED + 3, lo=64, hi=512, tr_lo=0.65, tr_hi=0.97):
    """Uneven batched domains: nx, ny independently round(lo * (hi/lo)^U), U ~ U[0,1);
    even k a slab, odd k a droplet of radius min(nx, ny)/4; T/Tc uniform in
    [tr_lo, tr_hi]; per-domain noise seed seed*1000 + k."""
    rng = np.random.default_rng(seed)
    out = []
    ratio = hi / lo
    for k in range(n):
        nx = int(round(lo * ratio ** rng.uniform()))
        ny = int(round(lo * ratio ** rng.uniform()))
        tr = float(tr_lo + (tr_hi - tr_lo) * rng.uniform())
        kind = "slab" if k % 2 == 0 else "droplet"
        out.append(dict(nx=nx, ny=ny, kind=kind, Tr=tr,
                        R=0.25 * min(nx, ny) if kind == "droplet" else 0.0,
                        seed=seed * 1000 + k))
    return out


def xavier_params(seed=SEED + 5, hidden=64):
    """Glorot-uniform initial weights (zero biases) of the 3-64-64-64-1 network,
    flat in the order W1, b1, W2, b2, W3, b3, W4, b4 (row-major)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in [(3, hidden), (hidden, hidden), (hidden, hidden), (hidden, 1)]:
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-lim, lim, size=(fan_out, fan_in)).reshape(-1))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)
