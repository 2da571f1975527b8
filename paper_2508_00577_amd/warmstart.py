"""Learned warm start for droplet runs.

The solver produces long-run droplet profiles; their radial means become
training samples (T/Tc, R, r/R) -> rho/rho_c for the network, which is
trained on the GPU by the library's own kernels and then seeds new droplets
through evlbm_init_droplet (with the tanh profile as fallback).  The study
compares the number of steps to equilibrium of network-seeded and
tanh-seeded runs and the final density difference between them.

Steps to equilibrium: the plain (tanh-seeded) run is advanced for a long
horizon and its final density field is the reference; a run has reached
equilibrium at the first check (every `check` steps) where its density is
within `tol` (max difference relative to the largest density) of that
reference after aligning the centres of mass.  The same reference judges the
final error of the network-seeded run.  The alignment matters: a droplet in a
periodic box is neutrally stable against translation and wanders by a
fraction of a cell over 1e5 steps, which a pointwise comparison would count as
an error of the profile.  (The thermal relaxation of latent heat across the
domain is slow, so a drift-rate criterion is not met within practical
horizons by either run.)

A periodic box conserves mass and total energy, so two runs can only end in
the same state if they start with the same mass and energy.  The sharp tanh
profile carries excess interface energy that turns into heat; the matched
warm start therefore scales the network's density field to the plain run's
mass and sets its uniform temperature so that the total energy
sum[rho E - a rho^2 + (kappa/2)|grad rho|^2] (global sums of the library)
equals the plain run's.  The unmatched warm start keeps T = Tr Tc.
"""
from __future__ import annotations

import numpy as np

from . import MLP, Lattice, eos_critical


def radial_profile(rho, centre, R, dr=0.5, rmax_factor=3.0):
    """Mean density on radial bins of width dr up to rmax_factor * R around
    centre (2D when rho has one z-plane).  Returns (r_mid, mean) of non-empty bins."""
    nz, ny, nx = rho.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2
    if nz > 1:
        r2 = r2 + (z - centre[2]) ** 2
    r = np.sqrt(r2).ravel()
    rmax = min(rmax_factor * R, 0.5 * min(s for s in rho.shape if s > 1) - 1.0)
    nb = int(rmax / dr)
    idx = np.floor(r / dr).astype(int)
    keep = idx < nb
    sums = np.bincount(idx[keep], weights=rho.ravel()[keep], minlength=nb)
    cnt = np.bincount(idx[keep], minlength=nb)
    ok = cnt > 0
    mids = (np.arange(nb) + 0.5) * dr
    return mids[ok], sums[ok] / cnt[ok]


def centre_of_mass(rho):
    """Centre of mass of the excess density rho - min(rho) (x, y, z order)."""
    w = rho - rho.min()
    nz, ny, nx = rho.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    tot = w.sum()
    return ((w * x).sum() / tot, (w * y).sum() / tot, (w * z).sum() / tot)


def aligned_difference(a, b):
    """max |a - b'| / max |a|, where b' is b translated (periodically, by an
    FFT phase shift) so that its centre of mass coincides with a's: a
    translation-invariant distance between two droplet states."""
    ca, cb = centre_of_mass(a), centre_of_mass(b)
    nz, ny, nx = b.shape
    shift = [(ca[2] - cb[2]) if nz > 1 else 0.0, ca[1] - cb[1], ca[0] - cb[0]]   # z, y, x
    B = np.fft.fftn(b)
    phase = np.ones(b.shape, dtype=complex)
    for ax, (n, d) in enumerate(zip(b.shape, shift)):
        k = np.fft.fftfreq(n)
        sh = [1, 1, 1]
        sh[ax] = n
        phase = phase * np.exp(-2j * np.pi * k * d).reshape(sh)
    bs = np.real(np.fft.ifftn(B * phase))
    return float(np.abs(a - bs).max() / np.abs(a).max())


def run_to_equilibrium(L, max_steps, check=100, tol=1e-7, rho_c=1.0):
    """Step until the equilibrium criterion holds; returns (steps, converged)."""
    prev, _, _ = L.moments()
    umax_prev = np.inf
    steps = 0
    while steps < max_steps:
        L.step(check)
        steps += check
        rho, u, _ = L.moments()
        drift = np.abs(rho - prev).max() / check
        umax = np.abs(u).max()
        if drift < tol * rho_c and umax >= umax_prev * (1 - 1e-3):
            return steps, True
        prev, umax_prev = rho, umax
    return steps, False


def droplet_run(shape, R, Tr, params, steps=None, profile="tanh", mlp=None, storage="f32", max_steps=40000,
                check=100, tol=1e-7, seed=0, noise=0.0):
    nz, ny, nx = shape
    L = Lattice(3 if nz > 1 else 2, nx, ny, nz, storage=storage)
    L.set_params(**params)
    used = L.init_droplet(R, Tr, profile=profile, mlp=mlp, seed=seed, noise=noise)
    if steps is not None:
        L.step(steps)
        return L, used, steps, None
    rho_c = eos_critical(params["R"], params["a"], params["b"], params.get("eos", "vdw"))[0]
    n, conv = run_to_equilibrium(L, max_steps, check, tol, rho_c=rho_c)
    return L, used, n, conv


def training_samples(cases, shape, params, steps, rho_c, seed=0, noise=0.0):
    """(X, Y) from the radial profiles of solver runs: cases = [(R, Tr), ...]."""
    X, Y = [], []
    nz, ny, nx = shape
    centre = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    for k, (R, Tr) in enumerate(cases):
        L, _, _, _ = droplet_run(shape, R, Tr, params, steps=steps, seed=seed + k if noise else 0, noise=noise)
        rho, _, _ = L.moments()
        r, prof = radial_profile(rho, centre, R)
        X.append(np.stack([np.full(r.size, Tr), np.full(r.size, R), r / R], 1))
        Y.append(prof / rho_c)
    return np.concatenate(X), np.concatenate(Y)


def train_network(X, Y, init_params, iters, lr=1e-3):
    net = MLP(init_params)
    hist = net.train(X, Y, iters, lr)
    return net, hist


def network_density(net, shape, R, Tr, rho_c):
    """rho_c y(Tr, R, |x - c|/R) on every cell of a droplet centred in the
    box: the library's network density field, copied to the host."""
    nz, ny, nx = shape
    centre = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    return net.density_field(shape, centre, R, Tr, rho_c).cpu().numpy()


def seed_matched(L, net, R, Tr, params, target):
    """Seed L from the network with the mass and total energy `target` (global
    sums 0 and 5 of a plain-seeded lattice), in the library
    (evlbm_init_droplet_matched).  Returns the temperature used."""
    _, T = L.init_droplet_matched(R, Tr, target[0], target[5], profile="mlp", mlp=net)
    return T


def _first_within(snaps, ref, tol):
    scale = np.abs(ref).max()
    for n, rho in snaps:
        if np.abs(rho - ref).max() < tol * scale:
            return n
    return None


def warm_start_study(net, cases, shape, params, horizon=40000, check=500, tol=2e-2):
    """For each (R, Tr), three seedings of the same droplet: the tanh profile
    ("tanh"), the network profile at T = Tr Tc ("mlp") and the network profile
    with the tanh run's mass and energy ("mlp_matched").  The tanh run's state
    after `horizon` steps is the reference.  Reported per seeding: the initial
    distance to it (aligned_difference), the first checked step within `tol` of
    it (None if never) and the distance at the horizon; and whether the network
    profile passed the fallback checks."""
    out = []
    nz, ny, nx = shape
    for R, Tr in cases:
        runs = {}
        target = None
        used = False
        for prof in ("tanh", "mlp", "mlp_matched"):
            L = Lattice(3 if nz > 1 else 2, nx, ny, nz, storage="f32")
            L.set_params(**params)
            if prof == "mlp_matched":
                seed_matched(L, net, R, Tr, params, target)
            else:
                u = L.init_droplet(R, Tr, profile="mlp" if prof == "mlp" else "tanh",
                                   mlp=net if prof == "mlp" else None)
                used = used or (prof == "mlp" and u)
            if prof == "tanh":
                target = L.global_sums()
            snaps = [(0, L.moments()[0].astype(np.float32))]
            for n in range(check, horizon + 1, check):
                L.step(check)
                snaps.append((n, L.moments()[0].astype(np.float32)))
            runs[prof] = snaps
        ref = runs["tanh"][-1][1].astype(np.float64)
        rec = dict(R=R, Tr=Tr, horizon=horizon, tol=tol, mlp_used=bool(used))
        for prof, snaps in runs.items():
            d = [(n, aligned_difference(ref, r.astype(np.float64))) for n, r in snaps]
            rec["err0_" + prof] = d[0][1]
            rec["steps_" + prof] = next((n for n, e in d if e < tol), None)
            rec["err_end_" + prof] = d[-1][1]
        out.append(rec)
    return out


def _trajectory(L, horizon, check, window=100):
    """Step L to `horizon` and return its density at every `check` steps
    (FP32 host copies, step 0 first) and, at each check, the drift rate
    max |rho_n - rho_(n - window)| / window."""
    rho = L.moments()[0]
    snaps, drift = [(0, rho.astype(np.float32))], []
    n = 0
    while n < horizon:
        L.step(check - window)
        a = L.moments()[0]
        L.step(window)
        n += check
        b = L.moments()[0]
        drift.append((n, float(np.abs(b - a).max() / window)))
        snaps.append((n, b.astype(np.float32)))
    return snaps, drift


def scale_study(net, cases, params, horizon=40000, check=2000, tol=1e-2, drift_tol=1e-7, seed=0, noise=1e-4):
    """The warm start at production sizes.  For each (shape, R, Tr) the plain
    run (tanh profile) and, when the network's profile passes the fallback
    checks, the network run with the plain run's mass and total energy
    (evlbm_init_droplet_matched), both with the same seeded noise, run for
    `horizon` steps with FP32 storage.  Reported per case:
      - mlp_used: False when the case falls back to the tanh profile (then
        the network run is the plain run);
      - steps_eq_plain, steps_eq_mlp: the first check at which the density
        drift rate over 100 steps is below drift_tol rho_c (None: not within
        the horizon);
      - steps_tol_plain, steps_tol_mlp: the first check within `tol` of the
        plain run's state at the horizon (aligned_difference);
      - err0_plain, err0_mlp: the distance from that state at step 0;
        err_end_mlp: at the horizon (the final density error of the network
        run against the plain run).
    A 3D case evaluates the network (trained on 2D profiles) on the 3D radius."""
    rho_c = eos_critical(params["R"], params["a"], params["b"], params.get("eos", "vdw"))[0]
    out = []
    for k, (shape, R, Tr) in enumerate(cases):
        nz, ny, nx = shape
        D = 3 if nz > 1 else 2
        rec = dict(shape=list(shape), R=R, Tr=Tr, horizon=horizon, tol=tol)
        L = Lattice(D, nx, ny, nz, storage="f32")
        L.set_params(**params)
        rec["mlp_used"] = bool(L.init_droplet(R, Tr, profile="mlp", mlp=net, seed=seed + k, noise=noise))
        del L
        L = Lattice(D, nx, ny, nz, storage="f32")
        L.set_params(**params)
        L.init_droplet(R, Tr, profile="tanh", seed=seed + k, noise=noise)
        target = L.global_sums()
        snaps, drift = _trajectory(L, horizon, check)
        del L
        ref = snaps[-1][1].astype(np.float64)
        d = [(n, aligned_difference(ref, r.astype(np.float64))) for n, r in snaps]
        rec["steps_eq_plain"] = next((n for n, v in drift if v < drift_tol * rho_c), None)
        rec["steps_tol_plain"] = next((n for n, e in d if e < tol), None)
        rec["err0_plain"] = d[0][1]
        rec["drift_end_plain"] = drift[-1][1] / rho_c
        if rec["mlp_used"]:
            L = Lattice(D, nx, ny, nz, storage="f32")
            L.set_params(**params)
            _, T = L.init_droplet_matched(R, Tr, target[0], target[5], profile="mlp", mlp=net,
                                          seed=seed + k, noise=noise)
            rec["T_matched_over_T0"] = T / (Tr * eos_critical(params["R"], params["a"], params["b"],
                                                               params.get("eos", "vdw"))[1])
            snaps_m, drift_m = _trajectory(L, horizon, check)
            del L
            dm = [(n, aligned_difference(ref, r.astype(np.float64))) for n, r in snaps_m]
            rec["steps_eq_mlp"] = next((n for n, v in drift_m if v < drift_tol * rho_c), None)
            rec["steps_tol_mlp"] = next((n for n, e in dm if e < tol), None)
            rec["err0_mlp"] = dm[0][1]
            rec["err_end_mlp"] = dm[-1][1]
            rec["drift_end_mlp"] = drift_m[-1][1] / rho_c
        out.append(rec)
    return out
