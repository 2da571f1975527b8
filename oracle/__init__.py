"""FP64 CPU oracle of the Enskog-Vlasov lattice Boltzmann step (test infrastructure).

This package is the correctness reference for the HIP library: a plain, slow,
obviously correct implementation of what the paper (Karlin & Hosseini,
"Practical Kinetic Models for Dense Fluids") defines.  Only the test-suite,
the smoke check and the CPU-baseline leg of the benchmark may import it; the
product never does.  It shares no code with the HIP path.

Modules:
  evo.c      the lattice Boltzmann step (eq. pre_LBM with eq. u_shift,
             T_shift, EVforce1, feq, f_star, correction_u/gamma/q, geq, gstar)
             and the single-cell operator K_lambda (eq. K, def_ustar)
  thermo.py  van der Waals coexistence by Maxwell's equal-area rule and the
             flat-interface surface tension
  mlp.py     the warm-start network (forward, backward, Adam) in FP64
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "evo.c")
_LIB = os.path.join(_HERE, "libevo.so")

EOS_KINDS = {"vdw": 0, "cs": 1}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile evo.c into libevo.so with gcc (plain C11, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c11", "-fPIC",
               "-shared", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.evo_create.restype = ctypes.c_void_p
        L.evo_create.argtypes = [ctypes.c_int] * 4
        L.evo_destroy.argtypes = [ctypes.c_void_p]
        L.evo_Q.argtypes = [ctypes.c_void_p]
        L.evo_N.restype = ctypes.c_long
        L.evo_N.argtypes = [ctypes.c_void_p]
        L.evo_step_count.restype = ctypes.c_long
        L.evo_step_count.argtypes = [ctypes.c_void_p]
        L.evo_set_threads.argtypes = [ctypes.c_int]
        L.evo_get_threads.restype = ctypes.c_int
        L.evo_set_params.argtypes = [ctypes.c_void_p] + [ctypes.c_double] * 7
        L.evo_set_eos.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.evo_set_walls.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.evo_set_prandtl.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.evo_init.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.evo_get_pops.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.evo_set_pops.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.evo_step.argtypes = [ctypes.c_void_p, ctypes.c_long, _dp]
        L.evo_moments.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
        L.evo_corrections.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.evo_global_sums.argtypes = [ctypes.c_void_p, _dp]
        L.evo_psi.restype = ctypes.c_double
        L.evo_psi.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.evo_lattice.argtypes = [ctypes.c_int, _ip, _dp]
        L.evo_product_cell.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
        L.evo_geq_cell.argtypes = [ctypes.c_int, ctypes.c_double, _dp, ctypes.c_double,
                                   ctypes.c_double, _dp]
        L.evo_kop.argtypes = [ctypes.c_int, ctypes.c_double, _dp, ctypes.c_double, _dp,
                              ctypes.c_double, _dp]
        L.evo_stencils.argtypes = [ctypes.c_int] * 4 + [_dp, _dp, _dp]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    lib().evo_set_threads(int(n))


def get_threads() -> int:
    return int(lib().evo_get_threads())


def lattice(D: int):
    """Velocities c[Q,3] (int) and weights w[Q] of D2Q9 (D=2) or D3Q27 (D=3)."""
    c = np.zeros(27 * 3, dtype=np.int32)
    w = np.zeros(27)
    Q = lib().evo_lattice(D, c.ctypes.data_as(_ip), _p(w))
    return c[: 3 * Q].reshape(Q, 3).copy(), w[:Q].copy()


def psi(c: int, xi: float, zeta: float) -> float:
    """Per-axis generating function Psi of eq. phi."""
    return float(lib().evo_psi(int(c), float(xi), float(zeta)))


def product_cell(D, rho, xi, zeta):
    """rho prod_a Psi(c_ia; xi_a, zeta_a) for one cell (eq. feq / eq. f_star)."""
    xi = _f64(list(xi) + [0.0] * (3 - len(xi)))
    zeta = _f64(list(zeta) + [0.0] * (3 - len(zeta)))
    out = np.zeros(9 if D == 2 else 27)
    lib().evo_product_cell(D, float(rho), _p(xi), _p(zeta), _p(out))
    return out


def feq_cell(D, rho, u, theta):
    """f^eq with xi = u, zeta = theta + u^2 (eq. feq with P0/rho = theta)."""
    u = list(u) + [0.0] * (3 - len(u))
    return product_cell(D, rho, u, [theta + x * x for x in u])


def geq_cell(D, rho, u, RT, theta):
    """g^eq(u, RT) with P0/rho = theta (eq. geq)."""
    u = _f64(list(u) + [0.0] * (3 - len(u)))
    out = np.zeros(9 if D == 2 else 27)
    lib().evo_geq_cell(D, float(rho), _p(u), float(RT), float(theta), _p(out))
    return out


def kop(D, rho, u, RT, J, lam):
    """K_lambda(J) of eq. K for one cell with the kinetic lattice Maxwellian."""
    u = _f64(list(u) + [0.0] * (3 - len(u)))
    J = _f64(J)
    out = np.zeros(len(J))
    rc = lib().evo_kop(D, float(rho), _p(u), float(RT), _p(J), float(lam), _p(out))
    if rc != 0:
        raise ValueError("RT* <= 0")
    return out


def stencils(D, shape, phi):
    """Isotropic gradient [D, ...] and Laplacian of a periodic field phi[nz, ny, nx]."""
    nz, ny, nx = shape
    phi = _f64(phi).reshape(-1)
    N = phi.size
    grad = np.zeros(D * N)
    lap = np.zeros(N)
    lib().evo_stencils(D, nx, ny, nz, _p(phi), _p(grad), _p(lap))
    return grad.reshape((D,) + tuple(shape)), lap.reshape(shape)


class Lattice:
    """Oracle lattice: D2Q9 (D=2, nz=1) or D3Q27 (D=3), periodic, FP64.

    Arrays use the layout [nz, ny, nx] (x fastest); vector fields [D, nz, ny, nx];
    populations [Q, nz, ny, nx].
    """

    def __init__(self, D, nx, ny, nz=1):
        self.D, self.nx, self.ny, self.nz = D, nx, ny, nz
        self.shape = (nz, ny, nx)
        self._h = lib().evo_create(D, nx, ny, nz)
        if not self._h:
            raise ValueError("invalid lattice")
        self.Q = lib().evo_Q(self._h)
        self.N = nx * ny * nz

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().evo_destroy(h)
            self._h = None

    def set_params(self, R=1.0, a=0.0, b=0.0, kappa=0.0, tau=1.0, lam=1.0, sphi=-1.0, eos="vdw", Pr=1.0):
        """Model parameters; eos selects the contact factor of Enskog's
        pressure: "vdw" (the paper's van der Waals form) or "cs"
        (Carnahan-Starling); Pr the Prandtl number (tau_g = tau/Pr)."""
        rc = lib().evo_set_params(self._h, R, a, b, kappa, tau, lam, sphi)
        if rc != 0:
            raise ValueError("invalid parameters")
        if lib().evo_set_eos(self._h, EOS_KINDS[eos]) != 0:
            raise ValueError("unknown eos")
        if lib().evo_set_prandtl(self._h, float(Pr)) != 0:
            raise ValueError("Pr must be positive")

    def set_walls(self, Tw, Uw, enable=True):
        """Diffuse walls normal to x at x = -1/2 (at rest) and x = nx - 1/2
        (moving with Uw along y), both at temperature Tw."""
        if lib().evo_set_walls(self._h, 1 if enable else 0, float(Tw), float(Uw)) != 0:
            raise ValueError("walls need nx >= 2 and Tw > 0")

    def init(self, rho, T, u=None):
        rho = _f64(rho).reshape(-1)
        T = _f64(T).reshape(-1)
        u = None if u is None else _f64(u).reshape(-1)
        rc = lib().evo_init(self._h, _p(rho), _p(u), _p(T))
        if rc != 0:
            raise ValueError("non-physical initial state")

    def step(self, n=1, diag=False):
        d = np.zeros((5 + 3 * self.D) * self.N) if diag else None
        rc = lib().evo_step(self._h, int(n), _p(d))
        if rc != 0:
            raise FloatingPointError("non-physical state reached")
        if diag:
            return d.reshape((5 + 3 * self.D,) + self.shape)

    @property
    def step_count(self):
        return int(lib().evo_step_count(self._h))

    def moments(self):
        """(rho, u, T, F) of the readout at the current step."""
        N, D = self.N, self.D
        rho, T = np.zeros(N), np.zeros(N)
        u, F = np.zeros(D * N), np.zeros(D * N)
        lib().evo_moments(self._h, _p(rho), _p(u), _p(T), _p(F))
        s = self.shape
        return rho.reshape(s), u.reshape((D,) + s), T.reshape(s), F.reshape((D,) + s)

    def corrections(self):
        N, D = self.N, self.D
        Phi, qp, Phip = np.zeros(D * N), np.zeros(D * N), np.zeros(N)
        lib().evo_corrections(self._h, _p(Phi), _p(qp), _p(Phip))
        s = self.shape
        return Phi.reshape((D,) + s), qp.reshape((D,) + s), Phip.reshape(s)

    def global_sums(self):
        out = np.zeros(8)
        lib().evo_global_sums(self._h, _p(out))
        return out

    def get_pops(self):
        f = np.zeros(self.Q * self.N)
        g = np.zeros(self.Q * self.N)
        lib().evo_get_pops(self._h, _p(f), _p(g))
        s = (self.Q,) + self.shape
        return f.reshape(s), g.reshape(s)

    def set_pops(self, f, g):
        f = _f64(f).reshape(-1)
        g = _f64(g).reshape(-1)
        assert f.size == self.Q * self.N and g.size == self.Q * self.N
        lib().evo_set_pops(self._h, _p(f), _p(g))


def step_window(D, wf, wg, params, radius=4):
    """One oracle step of a periodic (2*radius+1)-wide window of stored
    populations wf, wg ([Q, W, W, W] in 3D, [Q, 1, W, W] in 2D); returns the
    new populations (f[Q], g[Q]) of the window's centre cell, which are exact
    for the large lattice the window was cut from (see step_sampled)."""
    W = 2 * radius + 1
    L = Lattice(3, W, W, W) if D == 3 else Lattice(2, W, W, 1)
    L.set_params(**params)
    L.set_pops(np.ascontiguousarray(wf, dtype=np.float64), np.ascontiguousarray(wg, dtype=np.float64))
    L.step(1)
    nf, ng = L.get_pops()
    if D == 3:
        return nf[:, radius, radius, radius].copy(), ng[:, radius, radius, radius].copy()
    return nf[:, 0, radius, radius].copy(), ng[:, 0, radius, radius].copy()


def step_sampled(D, f, g, cells, params, radius=4):
    """One oracle step evaluated at selected cells of a large periodic lattice.

    The new populations of a cell depend on the stored populations within
    Chebyshev distance 4 of it (pull: 1, density for the force chain: 3 more),
    so each sample is computed on a periodic (2*radius+1)-wide window around the
    cell; the centre of the window is exact.  f, g: [Q, nz, ny, nx] FP64 arrays;
    cells: iterable of (x, y, z).  Returns (f_new[n, Q], g_new[n, Q]).
    """
    Q, nz, ny, nx = f.shape
    W = 2 * radius + 1
    out_f, out_g = [], []
    for (x, y, z) in cells:
        xs = (np.arange(W) - radius + x) % nx
        ys = (np.arange(W) - radius + y) % ny
        if D == 3:
            zs = (np.arange(W) - radius + z) % nz
            wf = f[:, zs][:, :, ys][:, :, :, xs]
            wg = g[:, zs][:, :, ys][:, :, :, xs]
        else:
            wf = f[:, 0][:, ys][:, :, xs][:, None]
            wg = g[:, 0][:, ys][:, :, xs][:, None]
        nf, ng = step_window(D, wf, wg, params, radius)
        out_f.append(nf)
        out_g.append(ng)
    return np.array(out_f), np.array(out_g)
