"""Python binding of libevlbm, the MI355X (gfx950) Enskog-Vlasov lattice Boltzmann library.

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch provides device memory (output tensors) and streams.  The
names follow include/evlbm.h; errors raise EvlbmError with the library's
message.  The library must have been built (``python -m
paper_2508_00577_amd.build``); nothing here falls back to another
implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libevlbm.so")

D2Q9, D3Q27 = 2, 3
F64, F32, F16DEV, BF16DEV = 0, 1, 2, 3
HOST_F64, DEVICE_F32, DEVICE_F64 = 0, 1, 2
OPT_SPHI, OPT_CHECK_EVERY, OPT_USE_GRAPH, OPT_REREF_EVERY, OPT_PUSH_MOMENTS, OPT_EOS, OPT_PRANDTL = 1, 4, 5, 6, 7, 8, 9
EOS = {"vdw": 0, "cs": 1}  # contact factor of Enskog's pressure: van der Waals, Carnahan-Starling
MEASURE_SLAB, MEASURE_DROPLET = 1, 2
STORAGE = {"f64": F64, "f32": F32, "f16dev": F16DEV, "bf16dev": BF16DEV}
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESTATE", -5: "ENONFINITE", -6: "EIO", -7: "ENONPHYS"}

_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


class EvlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


_lib = None


def lib():
    """Load libevlbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime; load it first so that this library
        # binds to the same runtime (one HIP runtime per process)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2508_00577_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.evlbm_last_error.restype = ctypes.c_char_p
        L.evlbm_version.restype = ctypes.c_char_p
        L.evlbm_create.argtypes = [ctypes.c_int] * 5 + [_vp, ctypes.POINTER(_vp)]
        L.evlbm_destroy.argtypes = [_vp]
        L.evlbm_set_eos.argtypes = [_vp] + [ctypes.c_double] * 4
        L.evlbm_set_relaxation.argtypes = [_vp, ctypes.c_double, ctypes.c_double]
        L.evlbm_set_option.argtypes = [_vp, ctypes.c_int, ctypes.c_double]
        L.evlbm_init_fields.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int]
        L.evlbm_step.argtypes = [_vp, ctypes.c_int64]
        L.evlbm_step_count.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64)]
        L.evlbm_read_moments.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int]
        L.evlbm_global_sums.argtypes = [_vp, _dp]
        L.evlbm_global_sums_noalloc.argtypes = [_vp, _vp]
        L.evlbm_measure.argtypes = [_vp, ctypes.c_int, _dp, _dp]
        L.evlbm_get_populations.argtypes = [_vp, _vp, _vp, ctypes.c_int]
        L.evlbm_set_populations.argtypes = [_vp, _vp, _vp, ctypes.c_int]
        L.evlbm_checkpoint_save.argtypes = [_vp, ctypes.c_char_p]
        L.evlbm_checkpoint_load.argtypes = [_vp, ctypes.c_char_p]
        L.evlbm_synchronize.argtypes = [_vp]
        L.evlbm_population_bytes.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_long)]
        L.evlbm_attach_buffers.argtypes = [_vp, _vp, _vp, ctypes.c_size_t]
        L.evlbm_profile_step.argtypes = [_vp, ctypes.c_int, _dp]
        L.evlbm_eos_coexistence.argtypes = [ctypes.c_int] + [ctypes.c_double] * 4 + [_dp]
        L.evlbm_eos_critical.argtypes = [ctypes.c_int] + [ctypes.c_double] * 3 + [_dp]
        L.evlbm_copy_probe.argtypes = [ctypes.c_double, ctypes.c_int, _dp]
        L.evlbm_batch_create.argtypes = [ctypes.c_int, _vp, ctypes.c_int, _vp, ctypes.POINTER(_vp)]
        L.evlbm_batch_destroy.argtypes = [_vp]
        L.evlbm_batch_set_params.argtypes = [_vp] + [ctypes.c_double] * 7
        L.evlbm_batch_set_option.argtypes = [_vp, ctypes.c_int, ctypes.c_double]
        L.evlbm_batch_init_domain.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp]
        L.evlbm_batch_step.argtypes = [_vp, ctypes.c_int64]
        L.evlbm_batch_read.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp]
        L.evlbm_batch_get_populations.argtypes = [_vp, ctypes.c_int, _vp, _vp]
        L.evlbm_batch_set_tile.argtypes = [_vp, ctypes.c_int]
        L.evlbm_batch_autotune.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _dp]
        _fp = ctypes.POINTER(ctypes.c_float)
        L.evlbm_mlp_create.argtypes = [_vp, ctypes.POINTER(_vp)]
        L.evlbm_mlp_destroy.argtypes = [_vp]
        L.evlbm_mlp_set_params.argtypes = [_vp, _fp, ctypes.c_int]
        L.evlbm_mlp_get_params.argtypes = [_vp, _fp, ctypes.c_int]
        L.evlbm_mlp_forward.argtypes = [_vp, _fp, _fp, ctypes.c_int]
        L.evlbm_mlp_grad.argtypes = [_vp, _fp, _fp, ctypes.c_int, _fp, _fp]
        L.evlbm_mlp_train.argtypes = [_vp, _fp, _fp, ctypes.c_int, ctypes.c_int, ctypes.c_float, _fp]
        L.evlbm_mlp_set_hull.argtypes = [_vp] + [ctypes.c_double] * 4
        L.evlbm_mlp_get_hull.argtypes = [_vp, _dp]
        L.evlbm_init_droplet.argtypes = ([_vp] + [ctypes.c_double] * 5 + [ctypes.c_int, _vp, ctypes.c_double,
                                         ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(ctypes.c_int)])
        L.evlbm_init_slab.argtypes = [_vp] + [ctypes.c_double] * 4 + [ctypes.c_uint64, ctypes.c_double]
        L.evlbm_init_droplet_matched.argtypes = ([_vp] + [ctypes.c_double] * 5 + [ctypes.c_int, _vp, ctypes.c_double,
                                                 ctypes.c_uint64] + [ctypes.c_double] * 3 +
                                                 [ctypes.POINTER(ctypes.c_int), _dp])
        L.evlbm_mlp_density_field.argtypes = [_vp] + [ctypes.c_int] * 3 + [ctypes.c_double] * 6 + [_vp]
        L.evlbm_set_walls.argtypes = [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.evlbm_batch_info.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64)] + [ctypes.POINTER(ctypes.c_int)] * 4
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise EvlbmError(rc, lib().evlbm_last_error().decode())


def _host(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(_vp)
    return ctypes.c_void_p(a.data_ptr())  # torch tensor


def eos_coexistence(T, R=1.0, a=0.0225, b=1.0 / 3.0, eos="vdw"):
    """(rho_l, rho_v, P_coex) of the bulk pressure P_E - a rho^2 at temperature T
    (eos: "vdw" or "cs")."""
    out = np.zeros(3)
    _check(lib().evlbm_eos_coexistence(EOS[eos], R, a, b, T, out.ctypes.data_as(_dp)))
    return tuple(out)


def eos_critical(R=1.0, a=0.0225, b=1.0 / 3.0, eos="vdw"):
    """(rho_c, T_c, P_c) of the bulk pressure P_E - a rho^2 (eos: "vdw" or "cs")."""
    out = np.zeros(3)
    _check(lib().evlbm_eos_critical(EOS[eos], R, a, b, out.ctypes.data_as(_dp)))
    return tuple(out)


def copy_probe(bytes_total=4e9, reps=20):
    """GB/s of a plain streaming copy moving bytes_total per launch (read + write)."""
    out = ctypes.c_double()
    _check(lib().evlbm_copy_probe(float(bytes_total), int(reps), ctypes.byref(out)))
    return out.value


def version():
    return lib().evlbm_version().decode()


class Lattice:
    """One periodic lattice on the GPU: D2Q9 (nz = 1) or D3Q27.

    Fields are indexed [nz, ny, nx] (x fastest); vectors [D, nz, ny, nx].
    `storage` is one of 'f64', 'f32', 'f16dev', 'bf16dev'.  A dedicated torch
    stream is used unless one is given.
    """

    def __init__(self, D, nx, ny, nz=1, storage="f32", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a visible GPU")
        self.D, self.nx, self.ny, self.nz = D, nx, ny, nz
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.Q = 9 if D == 2 else 27
        self.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = _vp()
        _check(lib().evlbm_create(D, nx, ny, nz, self.storage, _vp(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.evlbm_destroy(h)
            self._h = None

    def close(self):
        self.__del__()

    # -- parameters
    def set_eos(self, R=1.0, a=0.0, b=0.0, kappa=0.0):
        _check(lib().evlbm_set_eos(self._h, R, a, b, kappa))

    def set_relaxation(self, tau=1.0, lam=1.0):
        _check(lib().evlbm_set_relaxation(self._h, tau, lam))

    def set_params(self, R=1.0, a=0.0, b=0.0, kappa=0.0, tau=1.0, lam=1.0, sphi=-1.0, eos="vdw", Pr=1.0):
        self.set_eos(R, a, b, kappa)
        self.set_relaxation(tau, lam)
        self.set_option(OPT_SPHI, sphi)
        self.set_option(OPT_EOS, EOS[eos])
        self.set_option(OPT_PRANDTL, Pr)

    def set_option(self, key, value):
        _check(lib().evlbm_set_option(self._h, int(key), float(value)))

    def set_walls(self, Tw, Uw, enable=True):
        """Diffuse walls normal to x: at rest at x = -1/2, moving with Uw along
        y at x = nx - 1/2, both at temperature Tw (evlbm_set_walls)."""
        _check(lib().evlbm_set_walls(self._h, 1 if enable else 0, float(Tw), float(Uw)))

    # -- state
    def init_fields(self, rho, T, u=None):
        """Initialise from host (numpy, FP64) or device (torch, FP32/FP64) fields."""
        if isinstance(rho, np.ndarray):
            rho, T = _host(rho), _host(T)
            u = None if u is None else _host(u)
            where = HOST_F64
        else:
            import torch
            where = DEVICE_F64 if rho.dtype == torch.float64 else DEVICE_F32
            rho, T = rho.contiguous(), T.contiguous()
            u = None if u is None else u.contiguous()
        assert rho.size == self.N if isinstance(rho, np.ndarray) else rho.numel() == self.N
        _check(lib().evlbm_init_fields(self._h, _ptr(rho), _ptr(u), _ptr(T), where))

    def step(self, n=1):
        _check(lib().evlbm_step(self._h, int(n)))

    @property
    def step_count(self):
        v = ctypes.c_int64()
        _check(lib().evlbm_step_count(self._h, ctypes.byref(v)))
        return int(v.value)

    def synchronize(self):
        _check(lib().evlbm_synchronize(self._h))

    def population_bytes(self):
        """(bytes of one population buffer, direction stride in elements)."""
        nb, st = ctypes.c_size_t(), ctypes.c_long()
        _check(lib().evlbm_population_bytes(self._h, ctypes.byref(nb), ctypes.byref(st)))
        return nb.value, st.value

    def attach_buffers(self, a, b):
        """Keep the populations in two caller-owned device tensors (each at
        least population_bytes()[0] bytes); the lattice holds references to
        them so they outlive it."""
        nbytes = min(a.numel() * a.element_size(), b.numel() * b.element_size())
        _check(lib().evlbm_attach_buffers(self._h, _vp(a.data_ptr()), _vp(b.data_ptr()), nbytes))
        # torch's allocator must not hand the memory out again while the
        # lattice's stream may still use it
        a.record_stream(self.stream)
        b.record_stream(self.stream)
        self._attached = (a, b)

    def profile_step(self, nsteps=20):
        """Average kernel durations (ms) of (moments, collide) over nsteps real steps."""
        out = np.zeros(2)
        _check(lib().evlbm_profile_step(self._h, int(nsteps), out.ctypes.data_as(_dp)))
        return float(out[0]), float(out[1])

    def moments(self, device=False, dtype=None):
        """(rho, u, T) of the current state: numpy FP64 (default) or torch tensors."""
        if not device:
            rho = np.zeros(self.shape)
            u = np.zeros((self.D,) + self.shape)
            T = np.zeros(self.shape)
            _check(lib().evlbm_read_moments(self._h, _ptr(rho), _ptr(u), _ptr(T), HOST_F64))
            return rho, u, T
        import torch
        dtype = dtype or torch.float32
        with torch.cuda.stream(self.stream):
            rho = torch.empty(self.shape, dtype=dtype, device="cuda")
            u = torch.empty((self.D,) + self.shape, dtype=dtype, device="cuda")
            T = torch.empty(self.shape, dtype=dtype, device="cuda")
        where = DEVICE_F64 if dtype == torch.float64 else DEVICE_F32
        _check(lib().evlbm_read_moments(self._h, _ptr(rho), _ptr(u), _ptr(T), where))
        # the readout is enqueued on the lattice's stream: order the caller's stream after it
        torch.cuda.current_stream().wait_stream(self.stream)
        return rho, u, T

    def global_sums(self):
        out = np.zeros(8)
        _check(lib().evlbm_global_sums(self._h, out.ctypes.data_as(_dp)))
        return out

    def global_sums_into(self, out):
        """The global sums into a caller-owned device tensor of 8 float64
        values, enqueued on the lattice's stream without any allocation
        (evlbm_global_sums_noalloc; lattices of at most 2^24 cells)."""
        import torch
        if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64 and out.numel() >= 8
                and out.is_contiguous()):
            raise ValueError("out must be a contiguous CUDA float64 tensor of at least 8 values")
        _check(lib().evlbm_global_sums_noalloc(self._h, _vp(out.data_ptr())))
        out.record_stream(self.stream)
        return out

    def measure_slab(self, liquid, vapour1, vapour2):
        g = np.array([liquid[0], liquid[1], vapour1[0], vapour1[1], vapour2[0], vapour2[1]], dtype=np.float64)
        out = np.zeros(8)
        _check(lib().evlbm_measure(self._h, MEASURE_SLAB, g.ctypes.data_as(_dp), out.ctypes.data_as(_dp)))
        return out

    def measure_droplet(self, centre, r_in, r_out):
        c = list(centre) + [0.0] * (3 - len(centre))
        g = np.array(c + [r_in, r_out, 0.0], dtype=np.float64)
        out = np.zeros(8)
        _check(lib().evlbm_measure(self._h, MEASURE_DROPLET, g.ctypes.data_as(_dp), out.ctypes.data_as(_dp)))
        return out

    def get_populations(self, device=False):
        """Decoded populations (f, g), each [Q, nz, ny, nx] FP64: numpy arrays,
        or torch tensors on the lattice's device with device=True."""
        if not device:
            f = np.zeros((self.Q,) + self.shape)
            g = np.zeros((self.Q,) + self.shape)
            _check(lib().evlbm_get_populations(self._h, _ptr(f), _ptr(g), HOST_F64))
            return f, g
        import torch
        with torch.cuda.stream(self.stream):
            f = torch.empty((self.Q,) + self.shape, dtype=torch.float64, device="cuda")
            g = torch.empty((self.Q,) + self.shape, dtype=torch.float64, device="cuda")
        _check(lib().evlbm_get_populations(self._h, _ptr(f), _ptr(g), DEVICE_F64))
        torch.cuda.current_stream().wait_stream(self.stream)
        return f, g

    def set_populations(self, f, g):
        f, g = _host(f), _host(g)
        assert f.size == self.Q * self.N and g.size == self.Q * self.N
        _check(lib().evlbm_set_populations(self._h, _ptr(f), _ptr(g), HOST_F64))

    def _centre(self, centre):
        if centre is None:
            centre = ((self.nx - 1) / 2.0, (self.ny - 1) / 2.0, (self.nz - 1) / 2.0)
        return [float(v) for v in list(centre) + [0.0] * (3 - len(centre))]

    def init_droplet(self, radius, Tr, profile="tanh", mlp=None, centre=None, width=2.0, seed=0, noise=0.0):
        """Droplet at rest at T/Tc = Tr: tanh profile between the coexistence
        densities, or the network's profile (with the tanh fallback), with
        seeded multiplicative noise.  Returns True when the network's profile
        was used."""
        used = ctypes.c_int()
        c = self._centre(centre)
        _check(lib().evlbm_init_droplet(self._h, c[0], c[1], c[2], float(radius), float(Tr),
                                        1 if profile == "mlp" else 0, None if mlp is None else mlp._h, float(width),
                                        int(seed), float(noise), ctypes.byref(used)))
        return bool(used.value)

    def init_droplet_matched(self, radius, Tr, mass, energy, profile="mlp", mlp=None, centre=None, width=2.0,
                             seed=0, noise=0.0):
        """The droplet of init_droplet carrying total mass `mass` and total
        energy `energy` (global sums 0 and 5).  Returns (network used, T)."""
        used = ctypes.c_int()
        T = ctypes.c_double()
        c = self._centre(centre)
        _check(lib().evlbm_init_droplet_matched(self._h, c[0], c[1], c[2], float(radius), float(Tr),
                                                1 if profile == "mlp" else 0, None if mlp is None else mlp._h,
                                                float(width), int(seed), float(noise), float(mass), float(energy),
                                                ctypes.byref(used), ctypes.byref(T)))
        return bool(used.value), T.value

    def init_slab(self, Tr, x0=None, x1=None, width=2.0, seed=0, noise=0.0):
        """Flat liquid slab between x0 and x1 (default nx/4 and 3 nx/4) at rest
        at T/Tc = Tr, with seeded multiplicative noise."""
        x0 = self.nx / 4.0 if x0 is None else x0
        x1 = 3.0 * self.nx / 4.0 if x1 is None else x1
        _check(lib().evlbm_init_slab(self._h, float(x0), float(x1), float(Tr), float(width), int(seed), float(noise)))

    def checkpoint_save(self, path):
        _check(lib().evlbm_checkpoint_save(self._h, str(path).encode()))

    def checkpoint_load(self, path):
        _check(lib().evlbm_checkpoint_load(self._h, str(path).encode()))


TILE_SHAPES = [(64, 4), (64, 16), (128, 2), (64, 8)]  # evlbm_batch_set_tile variants


class Batch:
    """Many periodic D2Q9 domains of uneven sizes advanced together.

    `sizes` is a list of (nx, ny).  Fields of domain k are [1, ny, nx] arrays.
    """

    def __init__(self, sizes, storage="f32", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a visible GPU")
        self.sizes = [(int(a), int(b)) for a, b in sizes]
        self.n = len(self.sizes)
        self.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        desc = (ctypes.c_int * (2 * self.n))(*[v for s in self.sizes for v in s])
        h = _vp()
        _check(lib().evlbm_batch_create(self.n, ctypes.cast(desc, _vp), self.storage, _vp(self.stream.cuda_stream),
                                        ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.evlbm_batch_destroy(h)
            self._h = None

    def set_params(self, R=1.0, a=0.0, b=0.0, kappa=0.0, tau=1.0, lam=1.0, sphi=-1.0, eos="vdw", Pr=1.0):
        _check(lib().evlbm_batch_set_params(self._h, R, a, b, kappa, tau, lam, sphi))
        _check(lib().evlbm_batch_set_option(self._h, OPT_EOS, float(EOS[eos])))
        _check(lib().evlbm_batch_set_option(self._h, OPT_PRANDTL, float(Pr)))

    def init_domain(self, k, rho, T, u=None):
        nx, ny = self.sizes[k]
        rho, T = _host(rho), _host(T)
        assert rho.size == nx * ny and T.size == nx * ny
        u = None if u is None else _host(u)
        _check(lib().evlbm_batch_init_domain(self._h, int(k), _ptr(rho), _ptr(u), _ptr(T)))

    def step(self, n=1):
        _check(lib().evlbm_batch_step(self._h, int(n)))

    def synchronize(self):
        self.stream.synchronize()

    def moments(self, k):
        nx, ny = self.sizes[k]
        rho, T = np.zeros((1, ny, nx)), np.zeros((1, ny, nx))
        u = np.zeros((2, 1, ny, nx))
        _check(lib().evlbm_batch_read(self._h, int(k), _ptr(rho), _ptr(u), _ptr(T)))
        return rho, u, T

    def get_populations(self, k):
        nx, ny = self.sizes[k]
        f, g = np.zeros((9, 1, ny, nx)), np.zeros((9, 1, ny, nx))
        _check(lib().evlbm_batch_get_populations(self._h, int(k), _ptr(f), _ptr(g)))
        return f, g

    def set_tile(self, variant):
        _check(lib().evlbm_batch_set_tile(self._h, int(variant)))

    def info(self):
        cells = ctypes.c_int64()
        nt, v, tx, ty = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().evlbm_batch_info(self._h, ctypes.byref(cells), ctypes.byref(nt), ctypes.byref(v),
                                      ctypes.byref(tx), ctypes.byref(ty)))
        return dict(cells=cells.value, tiles=nt.value, variant=v.value, tile=(tx.value, ty.value))

    def autotune(self, steps=20, cache=None):
        """Pick the fastest tile shape (timed on this batch); with `cache`, a JSON
        file keyed by the domain sizes and storage, reuse a previous choice."""
        import hashlib
        import json
        key = hashlib.sha256(json.dumps([self.storage, self.sizes]).encode()).hexdigest()[:16]
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                table = json.load(fh)
            if key in table:
                self.set_tile(table[key]["variant"])
                return table[key]
        best = ctypes.c_int()
        ms = np.zeros(4)
        _check(lib().evlbm_batch_autotune(self._h, int(steps), ctypes.byref(best), ms.ctypes.data_as(_dp)))
        entry = {"variant": int(best.value), "tile": TILE_SHAPES[best.value], "ms_per_step": ms.tolist()}
        if cache:
            table = {}
            if os.path.exists(cache):
                with open(cache) as fh:
                    table = json.load(fh)
            table[key] = entry
            with open(cache, "w") as fh:
                json.dump(table, fh, indent=1)
        return entry


NPARAM = 8641


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class MLP:
    """The warm-start network on the GPU (forward, gradient, Adam training)."""

    def __init__(self, params=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a visible GPU")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = _vp()
        _check(lib().evlbm_mlp_create(_vp(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        if params is not None:
            self.set_params(params)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.evlbm_mlp_destroy(h)
            self._h = None

    def set_params(self, params):
        p = _f32(params)
        _check(lib().evlbm_mlp_set_params(self._h, _fptr(p), p.size))

    def params(self):
        p = np.zeros(NPARAM, dtype=np.float32)
        _check(lib().evlbm_mlp_get_params(self._h, _fptr(p), NPARAM))
        return p

    def set_hull(self, tr_lo, tr_hi, r_lo, r_hi):
        _check(lib().evlbm_mlp_set_hull(self._h, float(tr_lo), float(tr_hi), float(r_lo), float(r_hi)))

    def hull(self):
        """(tr_lo, tr_hi, r_lo, r_hi): the box of (T/Tc, R) the network is trusted on."""
        out = np.zeros(4)
        _check(lib().evlbm_mlp_get_hull(self._h, out.ctypes.data_as(_dp)))
        return tuple(float(v) for v in out)

    def forward(self, X):
        X = _f32(X).reshape(-1, 3)
        Y = np.zeros(X.shape[0], dtype=np.float32)
        _check(lib().evlbm_mlp_forward(self._h, _fptr(X), _fptr(Y), X.shape[0]))
        return Y

    def grad(self, X, Y):
        X, Y = _f32(X).reshape(-1, 3), _f32(Y)
        g = np.zeros(NPARAM, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        _check(lib().evlbm_mlp_grad(self._h, _fptr(X), _fptr(Y), X.shape[0], _fptr(g), _fptr(loss)))
        return g, float(loss[0])

    def density_field(self, shape, centre, radius, Tr, rho_c=1.0):
        """Device FP64 field rho_c y(T/Tc, R, |x - c|/R) on a [nz, ny, nx]
        lattice (a torch tensor; nz = 1: 2D distance)."""
        import torch
        nz, ny, nx = shape
        c = list(centre) + [0.0] * (3 - len(centre))
        with torch.cuda.stream(self.stream):
            out = torch.empty(shape, dtype=torch.float64, device="cuda")
        _check(lib().evlbm_mlp_density_field(self._h, nx, ny, nz, float(c[0]), float(c[1]), float(c[2]),
                                             float(radius), float(Tr), float(rho_c), _ptr(out)))
        torch.cuda.current_stream().wait_stream(self.stream)
        return out

    def train(self, X, Y, iters, lr=1e-3):
        X, Y = _f32(X).reshape(-1, 3), _f32(Y)
        hist = np.zeros(int(iters), dtype=np.float32)
        _check(lib().evlbm_mlp_train(self._h, _fptr(X), _fptr(Y), X.shape[0], int(iters), float(lr), _fptr(hist)))
        return hist
