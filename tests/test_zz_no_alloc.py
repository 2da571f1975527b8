"""evlbm_global_sums_noalloc through the C ABI against evlbm_global_sums:
two calls in a row, the second on a smaller lattice (the shared device
scratch keeps the first call's partials)."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
ev = pytest.importorskip("paper_2508_00577_amd")


def _lattice(D, shape, storage, seed):
    import oracle.thermo as TH
    nz, ny, nx = shape
    T0 = 0.8 * synth.T_CRIT
    rl, rv, _ = TH.coexistence(T0)
    L = ev.Lattice(D, nx, ny, nz, storage=storage)
    L.set_params(**synth.params())
    L.init_fields(synth.droplet(shape, 0.3 * min(s for s in shape if s > 1), rl, rv, noise=1e-3, seed=seed),
                  np.full(shape, T0))
    L.step(7)
    return L


def test_noalloc_sums_match_global_sums():
    import torch
    lib = ev.lib()
    lib.evlbm_global_sums_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    for D, shape, storage in ((3, (40, 36, 70), "f32"), (2, (1, 23, 57), "f64")):
        L = _lattice(D, shape, storage, synth.SEED + 40 + D)
        ref = L.global_sums()
        out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        rc = lib.evlbm_global_sums_noalloc(L._h, ctypes.c_void_p(out.data_ptr()))
        assert rc == 0, lib.evlbm_last_error()
        L.synchronize()
        got = out.cpu().numpy()
        print(f"D={D} {shape} {storage}: noalloc {got[:3]}, global_sums {ref[:3]}", flush=True)
        assert np.array_equal(got, ref), (got, ref)


def test_noalloc_sums_reject_oversized_lattice():
    lib = ev.lib()
    lib.evlbm_global_sums_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    L = ev.Lattice(3, 512, 256, 129, storage="f32")  # 2^24 + 2^17 cells: beyond the scratch
    L.set_params(**synth.params())
    L.init_fields(np.full((129, 256, 512), 0.5), np.full((129, 256, 512), 0.8 * synth.T_CRIT))
    import torch
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    assert lib.evlbm_global_sums_noalloc(L._h, ctypes.c_void_p(out.data_ptr())) == -1


def test_binding_global_sums_into_matches_global_sums():
    """The binding's Lattice.global_sums_into (the same entry point) fills a
    caller's device tensor with the values of global_sums, and refuses a
    tensor it cannot write."""
    import torch
    L = _lattice(3, (13, 11, 37), "f32", synth.SEED + 47)
    ref = L.global_sums()
    out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    L.global_sums_into(out)
    L.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref)
    with pytest.raises(ValueError):
        L.global_sums_into(torch.zeros(8, dtype=torch.float32, device="cuda"))
