"""The no-allocation entry point mlb_init_mixture_static against
mlb_init_mixture: the same mixtures, stepped the same number of times, give
the same populations (float64 and float32, bit for bit), on two calls in a
row (the second with a smaller lattice), and the host-side rejections."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_static_workspace_size_matches_header():
    from paper_1105_3634_amd import _lib
    src = open(os.path.join(ROOT, "include", "mlb.h")).read()
    m = re.search(r"#define MLB_STATIC_WORKSPACE_BYTES \(\(size_t\)(\d+) << (\d+)\)", src)
    assert m, "MLB_STATIC_WORKSPACE_BYTES not found"
    assert int(m.group(1)) << int(m.group(2)) == _lib.STATIC_WORKSPACE_BYTES


def test_static_rejects_oversize_before_device_work():
    """A mixture whose workspace exceeds the static array is refused with
    MLB_ENOMEM on the host, before any HIP call (this runs without a GPU)."""
    import paper_1105_3634_amd as mlb
    from paper_1105_3634_amd import _lib
    lib = _lib.load()
    m, _, _ = W.config_bulk_diffusion()
    p = mlb.make_params(m, precision=64)
    assert mlb.workspace_bytes(p) > _lib.STATIC_WORKSPACE_BYTES
    h = C.c_void_p()
    st = lib.mlb_init_mixture_static(C.byref(p), None, None, None, C.byref(h))
    assert st == -2, lib.mlb_last_error().decode()
    assert "static" in lib.mlb_last_error().decode()
    assert not h.value
    bad = mlb.make_params(W.Mixture(3, 6, 6, sigma=(2.0, 3.0)))   # stencil reaches the box edge
    assert lib.mlb_init_mixture_static(C.byref(bad), None, None, None, C.byref(h)) == -1


def _cases():
    big = W.Mixture(14, 12, 10, sigma=(2.0, 3.0, 2.5), eps=np.full((3, 3), 0.1), rc_factor=1.5,
                    walls_y=True, wall_ux=(-0.02, 0.03), name="walled ternary with tail")
    nb, ub = W.random_state(big, [0.012, 0.008, 0.006], rel=0.3, u_amp=0.02, seed=31)
    small = W.Mixture(10, 9, 8, sigma=(2.0, 2.5), fext=np.array([[1e-4, 0, 0], [-1e-4, 2e-5, 0]]),
                      name="periodic binary with body force")
    ns, us = W.random_state(small, [0.015, 0.01], rel=0.3, u_amp=0.02, seed=32)
    return [(big, nb, ub), (small, ns, us)]


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [64, 32])
def test_static_matches_caller_workspace(precision):
    import torch
    import paper_1105_3634_amd as mlb
    from paper_1105_3634_amd import _lib
    lib = _lib.load()
    steps = 7
    for m, n0, u0 in _cases():
        print(f"static workspace: {m.name} {m.nx}x{m.ny}x{m.nz} precision {precision}", flush=True)
        ref = mlb.GpuMixture(m, n0, u0, precision=precision, device="cuda:0")
        ref.step(steps)
        f_ref = ref.populations().cpu().numpy()
        ref.close()
        s = mlb.GpuMixture(m, n0, u0, precision=precision, device="cuda:0", static_workspace=True)
        # a second static mixture on the same GPU is refused while the first lives
        h2 = C.c_void_p()
        st = lib.mlb_init_mixture_static(C.byref(s.params), None, None, None, C.byref(h2))
        assert st == -6 and not h2.value, lib.mlb_last_error().decode()
        s.step(3)
        s.step(steps - 3)
        f_s = s.populations().cpu().numpy()
        torch.cuda.synchronize()
        s.close()
        assert f_s.shape == f_ref.shape
        assert np.array_equal(f_s, f_ref), f"max |diff| {np.abs(f_s - f_ref).max():.3e}"
