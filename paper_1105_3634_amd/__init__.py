"""mlb: MI355X-native multicomponent Enskog lattice-Boltzmann step.

Python face of libmlb.so (see include/mlb.h).  PyTorch supplies device
memory and streams; all arithmetic of the step runs in the library's HIP
kernels.  Importing this package does not need a GPU; creating a mixture
does, and fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (MlbError, OPT_NO_GRAPH, OPT_TUNE, opt_tiling, PART_ALL, PART_DISS, PART_EXT, PART_MF, PART_TAIL, Q,
                   SCHEME_CN_J1, SCHEME_FE, TAIL_AUTO, TAIL_DIRECT, TAIL_SPECTRAL)

__all__ = ["GpuMixture", "GpuBatch", "OPT_TUNE", "OPT_NO_GRAPH", "opt_tiling", "make_params", "workspace_bytes", "MlbError", "PART_ALL", "PART_MF", "PART_TAIL",
           "PART_DISS", "PART_EXT", "TAIL_AUTO", "TAIL_DIRECT", "TAIL_SPECTRAL", "SCHEME_CN_J1", "SCHEME_FE"]


def _torch():
    import torch
    return torch


def make_params(mix, precision: int = 32, tail_mode: int = TAIL_AUTO) -> _lib.Params:
    """Fill the C parameter block from a mixture description (any object with
    nx, ny, nz, sigma, tau, kT, rc_factor, walls_y, wall_ux, scheme and the
    eps_matrix() / fext_matrix() accessors; masses from mass_vector() when
    it has one, else 1)."""
    p = _lib.Params()
    p.nx, p.ny, p.nz = int(mix.nx), int(mix.ny), int(mix.nz)
    M = len(mix.sigma)
    p.nspecies = M
    p.precision = int(precision)
    p.scheme = int(getattr(mix, "scheme", SCHEME_CN_J1))
    p.tail_mode = int(tail_mode)
    p.walls_y = 1 if getattr(mix, "walls_y", False) else 0
    p.tau = float(mix.tau)
    p.kT = float(mix.kT)
    eps = np.asarray(mix.eps_matrix(), dtype=np.float64).reshape(M, M)
    fx = np.asarray(mix.fext_matrix(), dtype=np.float64).reshape(M, 3)
    mass = np.asarray(mix.mass_vector(), dtype=np.float64).reshape(M) if hasattr(mix, "mass_vector") else np.ones(M)
    for a in range(M):
        p.mass[a] = float(mass[a])
        p.sigma[a] = float(mix.sigma[a])
        for b in range(M):
            p.eps[a * _lib.MAX_SPECIES + b] = float(eps[a, b])
        for d in range(3):
            p.ext_force[3 * a + d] = float(fx[a, d])
    p.rc_factor = float(getattr(mix, "rc_factor", 2.5))
    wu = getattr(mix, "wall_ux", (0.0, 0.0))
    p.wall_ux[0], p.wall_ux[1] = float(wu[0]), float(wu[1])
    return p


def workspace_bytes(params: _lib.Params) -> int:
    lib = _lib.load()
    n = lib.mlb_workspace_bytes(C.byref(params))
    if n == 0:
        raise MlbError(-1, "mlb_workspace_bytes", lib.mlb_last_error().decode())
    return int(n)


def _stream_handle(stream) -> C.c_void_p:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(int(s.cuda_stream))


class GpuMixture:
    """One mixture on the GPU.  Fields come back as torch tensors on the device."""

    def __init__(self, mix, n0: np.ndarray, u0: np.ndarray, precision: int = 32, tail_mode: int = TAIL_AUTO,
                 device: str = "cuda:0", stream=None, options: int = 0, static_workspace: bool = False):
        """static_workspace: use the library's static device workspace
        (mlb_init_mixture_static) instead of a torch-allocated one; `options`
        must then be 0."""
        torch = _torch()
        self.lib = _lib.load()
        self.mix = mix
        self.params = make_params(mix, precision, tail_mode)
        self.M = len(mix.sigma)
        self.P = self.M * (self.M + 1) // 2
        self.shape = (int(mix.nz), int(mix.ny), int(mix.nx))
        self.N = int(np.prod(self.shape))
        self.device = torch.device(device)
        self.dtype = torch.float64 if precision == 64 else torch.float32
        self.stream = stream
        n0_d = torch.as_tensor(np.ascontiguousarray(n0, dtype=np.float64)).to(self.device)
        u0_d = torch.as_tensor(np.ascontiguousarray(u0, dtype=np.float64)).to(self.device)
        assert n0_d.numel() == self.M * self.N and u0_d.numel() == 3 * self.M * self.N
        h = C.c_void_p()
        if static_workspace:
            assert options == 0, "options are not available with the static workspace"
            with torch.cuda.device(self.device):
                st = self.lib.mlb_init_mixture_static(C.byref(self.params), C.c_void_p(n0_d.data_ptr()),
                                                      C.c_void_p(u0_d.data_ptr()), _stream_handle(stream),
                                                      C.byref(h))
            _lib.check(st, "mlb_init_mixture_static")
            self.h = h
            return
        nbytes = workspace_bytes(self.params)
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self.ws = raw[off:off + nbytes]
        st = self.lib.mlb_init_mixture_ex(C.byref(self.params), C.c_void_p(self.ws.data_ptr()), nbytes,
                                          C.c_void_p(n0_d.data_ptr()), C.c_void_p(u0_d.data_ptr()), int(options),
                                          _stream_handle(stream), C.byref(h))
        _lib.check(st, "mlb_init_mixture_ex")
        self.h = h

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.mlb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --------------------------------------------------------------- driving
    def step(self, nsteps: int = 1) -> None:
        _lib.check(self.lib.mlb_step(self.h, int(nsteps), _stream_handle(self.stream)), "mlb_step")

    def tuning(self):
        """Float32 tiling in use: shape, order, the first gather's thread groups
        per site, shell loop and tile shape, and the time of every tuned
        candidate (mlb_tuning_ex, mlb_tuning_groups, mlb_tuning_gather1_shape)."""
        shape, order, split, groups, g1 = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        ms, gms = (C.c_double * 12)(), C.c_double()
        _lib.check(self.lib.mlb_tuning_ex(self.h, C.byref(shape), C.byref(order), C.byref(split), ms),
                   "mlb_tuning_ex")
        _lib.check(self.lib.mlb_tuning_groups(self.h, C.byref(groups), C.byref(gms)), "mlb_tuning_groups")
        _lib.check(self.lib.mlb_tuning_gather1_shape(self.h, C.byref(g1)), "mlb_tuning_gather1_shape")
        return {"shape": int(shape.value), "order": int(order.value), "gather1_split": int(split.value),
                "gather1_sign_groups": int(groups.value), "gather1_shape": int(g1.value), "trial_ms": list(ms[:]),
                "sign_groups_ms": float(gms.value)}

    def set_graph(self, enable: bool) -> None:
        _lib.check(self.lib.mlb_set_graph(self.h, 1 if enable else 0), "mlb_set_graph")

    @property
    def steps(self) -> int:
        return int(self.lib.mlb_step_count(self.h))

    def set_step_count(self, steps: int) -> None:
        """Resume a checkpoint: the step count saved with the populations."""
        _lib.check(self.lib.mlb_set_step_count(self.h, int(steps)), "mlb_set_step_count")

    def _empty(self, *shape):
        return _torch().empty(shape, dtype=self.dtype, device=self.device)

    def moments(self):
        n = self._empty(self.M, *self.shape)
        j = self._empty(self.M, 3, *self.shape)
        _lib.check(self.lib.mlb_moments(self.h, C.c_void_p(n.data_ptr()), C.c_void_p(j.data_ptr()),
                                        _stream_handle(self.stream)), "mlb_moments")
        return n, j

    def forces(self, parts: int = PART_ALL):
        out = self._empty(self.M, 3, *self.shape)
        _lib.check(self.lib.mlb_forces(self.h, C.c_void_p(out.data_ptr()), int(parts), _stream_handle(self.stream)),
                   "mlb_forces")
        return out

    def fields(self) -> Dict[str, "object"]:
        M, sh = self.M, self.shape
        out = {"n": self._empty(M, *sh), "j": self._empty(M, 3, *sh), "u": self._empty(3, *sh),
               "g": self._empty(self.P, *sh), "vhat": self._empty(M, 3, *sh), "H": self._empty(M, 3, *sh),
               "N": self._empty(M, 3, *sh)}
        ptrs = [C.c_void_p(out[k].data_ptr()) for k in ("n", "j", "u", "g", "vhat", "H", "N")]
        _lib.check(self.lib.mlb_fields(self.h, *ptrs, _stream_handle(self.stream)), "mlb_fields")
        return out

    def populations(self):
        f = self._empty(self.M, Q, *self.shape)
        _lib.check(self.lib.mlb_get_populations(self.h, C.c_void_p(f.data_ptr()), _stream_handle(self.stream)),
                   "mlb_get_populations")
        return f

    def set_populations(self, f) -> None:
        f = f.to(device=self.device, dtype=self.dtype).contiguous()
        assert f.numel() == self.M * Q * self.N
        _lib.check(self.lib.mlb_set_populations(self.h, C.c_void_p(f.data_ptr()), _stream_handle(self.stream)),
                   "mlb_set_populations")
        self._keep = f

    def set_force_profile(self, profile: Optional[np.ndarray]) -> None:
        """Body force per lattice row, [M][3][ny] float64 (added to the uniform
        ext_force), or None to remove it."""
        if profile is None:
            ptr = None
        else:
            prof = np.ascontiguousarray(profile, dtype=np.float64)
            assert prof.shape == (self.M, 3, self.shape[1])
            ptr = prof.ctypes.data_as(C.POINTER(C.c_double))
        _lib.check(self.lib.mlb_set_force_profile(self.h, ptr, _stream_handle(self.stream)), "mlb_set_force_profile")

    # ---------------------------------------------------------------- timing
    def profile_begin(self) -> None:
        _lib.check(self.lib.mlb_profile_begin(self.h), "mlb_profile_begin")

    def profile_end(self) -> Dict[str, tuple]:
        """{pass name: (summed ms, launches)} for the passes run since profile_begin."""
        ms = (C.c_double * _lib.NPASS)()
        cnt = (C.c_int32 * _lib.NPASS)()
        _lib.check(self.lib.mlb_profile_end(self.h, ms, cnt, _stream_handle(self.stream)), "mlb_profile_end")
        return {self.lib.mlb_pass_name(k).decode(): (ms[k], cnt[k]) for k in range(_lib.NPASS)}

    # ------------------------------------------------------- float64 reductions
    def conserved(self):
        mass = (C.c_double * self.M)()
        mom = (C.c_double * (3 * self.M))()
        _lib.check(self.lib.mlb_conserved(self.h, mass, mom, _stream_handle(self.stream)), "mlb_conserved")
        return np.array(mass[:]), np.array(mom[:]).reshape(self.M, 3)

    def record_mode(self, a: int = 0, b: int = 1) -> None:
        _lib.check(self.lib.mlb_record_mode(self.h, a, b, _stream_handle(self.stream)), "mlb_record_mode")

    def record_spread(self, a: int) -> None:
        _lib.check(self.lib.mlb_record_spread(self.h, a, _stream_handle(self.stream)), "mlb_record_spread")

    def reset_series(self) -> None:
        _lib.check(self.lib.mlb_series_reset(self.h, _stream_handle(self.stream)), "mlb_series_reset")

    def fit(self, kind: int = 0, t_min: float = 0.0) -> float:
        out = C.c_double()
        _lib.check(self.lib.mlb_fit_series(self.h, kind, float(t_min), C.byref(out), _stream_handle(self.stream)),
                   "mlb_fit_series")
        return float(out.value)

    def fit_ex(self, kind: int = 0, t_min: float = 0.0) -> Dict[str, float]:
        """The fit with its quality (mlb_fit_series_ex)."""
        out = (C.c_double * 5)()
        _lib.check(self.lib.mlb_fit_series_ex(self.h, kind, float(t_min), out, _stream_handle(self.stream)),
                   "mlb_fit_series_ex")
        return {"D": out[0], "slope": out[1], "samples": int(out[2]), "r2": out[3], "well_conditioned": out[4] == 1.0}

    def series(self):
        cap = int(self.lib.mlb_series_capacity())
        t = (C.c_double * cap)()
        v = (C.c_double * cap)()
        cnt = C.c_int32()
        _lib.check(self.lib.mlb_get_series(self.h, t, v, cap, C.byref(cnt), _stream_handle(self.stream)),
                   "mlb_get_series")
        n = cnt.value
        return np.array(t[:n]), np.array(v[:n])

    # ------------------------------------------------------- learned closure
    def set_closure(self, net: Optional["GpuNet"], check_every: int = 50, tol: float = 1e-2) -> None:
        _lib.check(self.lib.mlb_set_closure(self.h, net.h if net is not None else None, int(check_every), float(tol)),
                   "mlb_set_closure")
        self._net = net

    def closure_stats(self) -> Dict[str, object]:
        checks, fb, err, act = C.c_int64(), C.c_int64(), C.c_double(), C.c_int32()
        _lib.check(self.lib.mlb_closure_stats(self.h, C.byref(checks), C.byref(fb), C.byref(err), C.byref(act)),
                   "mlb_closure_stats")
        steps, failed = C.c_int64(), C.c_int64()
        _lib.check(self.lib.mlb_closure_usage(self.h, C.byref(steps), C.byref(failed)), "mlb_closure_usage")
        return {"checks": int(checks.value), "fallback_step": int(fb.value), "last_err": float(err.value),
                "active": bool(act.value), "net_steps": int(steps.value), "failed_checks": int(failed.value)}

    def closure_sample(self, net: "GpuNet"):
        """(x [14][...], target [6][...]) float32 device tensors for the current state."""
        torch = _torch()
        x = torch.empty((NET_CHANNELS[0],) + self.shape, dtype=torch.float32, device=self.device)
        t = torch.empty((6,) + self.shape, dtype=torch.float32, device=self.device)
        _lib.check(self.lib.mlb_closure_sample(self.h, net.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                               _stream_handle(self.stream)), "mlb_closure_sample")
        return x, t


class GpuBatch:
    """An ensemble of independent mixtures advanced by shared launches."""

    SHAPES = ("16x4x4", "8x8x4", "32x4x2")
    G1_SHAPES = SHAPES + ("4x8x8",)

    def __init__(self, mixes: Sequence, n0s: Sequence[np.ndarray], u0s: Sequence[np.ndarray], precision: int = 32,
                 options: int = 0, device: str = "cuda:0", stream=None):
        torch = _torch()
        self.lib = _lib.load()
        self.count = len(mixes)
        self.params = (_lib.Params * self.count)(*[make_params(m, precision, TAIL_DIRECT) for m in mixes])
        self.mixes = list(mixes)
        self.device = torch.device(device)
        self.dtype = torch.float64 if precision == 64 else torch.float32
        self.stream = stream
        nbytes = self.lib.mlb_batch_workspace_bytes(self.params, self.count)
        if nbytes == 0:
            raise MlbError(-1, "mlb_batch_workspace_bytes", self.lib.mlb_last_error().decode())
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self.ws = raw[off:off + nbytes]
        self._n0 = [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(self.device) for a in n0s]
        self._u0 = [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(self.device) for a in u0s]
        n0p = (C.c_void_p * self.count)(*[t.data_ptr() for t in self._n0])
        u0p = (C.c_void_p * self.count)(*[t.data_ptr() for t in self._u0])
        h = C.c_void_p()
        _lib.check(self.lib.mlb_init_batch(self.params, self.count, C.c_void_p(self.ws.data_ptr()), nbytes, n0p, u0p,
                                           int(options), _stream_handle(stream), C.byref(h)), "mlb_init_batch")
        self.h = h
        self._n0 = self._u0 = None

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.mlb_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, nsteps: int = 1) -> None:
        _lib.check(self.lib.mlb_batch_step(self.h, int(nsteps), _stream_handle(self.stream)), "mlb_batch_step")

    @property
    def steps(self) -> int:
        return int(self.lib.mlb_batch_step_count(self.h))

    def set_step_count(self, steps: int) -> None:
        _lib.check(self.lib.mlb_batch_set_step_count(self.h, int(steps)), "mlb_batch_set_step_count")

    def set_populations(self, k: int, f) -> None:
        M, sh = self._shape(k)
        f = f.to(device=self.device, dtype=self.dtype).contiguous()
        assert tuple(f.shape) == (M, Q) + sh
        _lib.check(self.lib.mlb_batch_set_populations(self.h, int(k), C.c_void_p(f.data_ptr()),
                                                      _stream_handle(self.stream)), "mlb_batch_set_populations")
        self._keep = f

    def _shape(self, k):
        m = self.mixes[k]
        return len(m.sigma), (int(m.nz), int(m.ny), int(m.nx))

    def moments(self, k: int):
        torch = _torch()
        M, sh = self._shape(k)
        n = torch.empty((M,) + sh, dtype=self.dtype, device=self.device)
        j = torch.empty((M, 3) + sh, dtype=self.dtype, device=self.device)
        _lib.check(self.lib.mlb_batch_moments(self.h, k, C.c_void_p(n.data_ptr()), C.c_void_p(j.data_ptr()),
                                              _stream_handle(self.stream)), "mlb_batch_moments")
        return n, j

    def populations(self, k: int):
        torch = _torch()
        M, sh = self._shape(k)
        f = torch.empty((M, Q) + sh, dtype=self.dtype, device=self.device)
        _lib.check(self.lib.mlb_batch_get_populations(self.h, k, C.c_void_p(f.data_ptr()), _stream_handle(self.stream)),
                   "mlb_batch_get_populations")
        return f

    def record_modes(self) -> None:
        _lib.check(self.lib.mlb_batch_record_modes(self.h, _stream_handle(self.stream)), "mlb_batch_record_modes")

    def fit(self, t_min: float = 0.0) -> np.ndarray:
        out = (C.c_double * self.count)()
        _lib.check(self.lib.mlb_batch_fit(self.h, float(t_min), out, _stream_handle(self.stream)), "mlb_batch_fit")
        return np.array(out[:])

    def fit_ex(self, t_min: float = 0.0) -> np.ndarray:
        """[count][5] = (D, slope, samples, R^2, well-conditioned flag) (mlb_batch_fit_ex)."""
        out = (C.c_double * (5 * self.count))()
        _lib.check(self.lib.mlb_batch_fit_ex(self.h, float(t_min), out, _stream_handle(self.stream)),
                   "mlb_batch_fit_ex")
        return np.array(out[:]).reshape(self.count, 5)

    def series(self, system: int):
        """(t, amplitude) of one system's recorded mode series (host arrays)."""
        cap = int(self.lib.mlb_series_capacity())
        t = (C.c_double * cap)()
        v = (C.c_double * cap)()
        cnt = C.c_int32()
        _lib.check(self.lib.mlb_batch_get_series(self.h, int(system), t, v, cap, C.byref(cnt),
                                                 _stream_handle(self.stream)), "mlb_batch_get_series")
        n = cnt.value
        return np.array(t[:n]), np.array(v[:n])

    def tuning(self):
        shape, order, split, groups, g1 = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        ms, gms = (C.c_double * 12)(), C.c_double()
        _lib.check(self.lib.mlb_batch_tuning_ex(self.h, C.byref(shape), C.byref(order), C.byref(split), ms),
                   "mlb_batch_tuning_ex")
        _lib.check(self.lib.mlb_batch_tuning_groups(self.h, C.byref(groups), C.byref(gms)),
                   "mlb_batch_tuning_groups")
        _lib.check(self.lib.mlb_batch_tuning_gather1_shape(self.h, C.byref(g1)), "mlb_batch_tuning_gather1_shape")
        return {"shape": int(shape.value), "order": int(order.value), "gather1_split": int(split.value),
                "gather1_sign_groups": int(groups.value), "gather1_shape": int(g1.value), "trial_ms": list(ms[:]),
                "sign_groups_ms": float(gms.value)}

    def profile_begin(self) -> None:
        _lib.check(self.lib.mlb_batch_profile_begin(self.h), "mlb_batch_profile_begin")

    def profile_end(self) -> Dict[str, tuple]:
        ms = (C.c_double * _lib.NPASS)()
        cnt = (C.c_int32 * _lib.NPASS)()
        _lib.check(self.lib.mlb_batch_profile_end(self.h, ms, cnt, _stream_handle(self.stream)),
                   "mlb_batch_profile_end")
        return {self.lib.mlb_pass_name(k).decode(): (ms[k], cnt[k]) for k in range(_lib.NPASS)}


NET_CHANNELS = (14, 32, 32, 32, 6)


def net_flatten(layers) -> np.ndarray:
    """Parameters as a list of {"W": [Co][Ci][3][3][3], "b": [Co]} -> the flat
    float32 layout of mlb_net_set_params."""
    parts = []
    for L in layers:
        parts.append(np.asarray(L["W"], dtype=np.float32).reshape(-1))
        parts.append(np.asarray(L["b"], dtype=np.float32).reshape(-1))
    return np.ascontiguousarray(np.concatenate(parts))


def net_unflatten(flat: np.ndarray, channels=NET_CHANNELS):
    out, k = [], 0
    for ci, co in zip(channels[:-1], channels[1:]):
        nw = co * ci * 27
        out.append({"W": flat[k:k + nw].reshape(co, ci, 3, 3, 3).copy(), "b": flat[k + nw:k + nw + co].copy()})
        k += nw + co
    return out


class GpuNet:
    """The force-closure network on one grid (nz, ny, nx)."""

    def __init__(self, shape, training: bool = False, device: str = "cuda:0", stream=None):
        torch = _torch()
        self.lib = _lib.load()
        self.shape = tuple(int(v) for v in shape)
        nz, ny, nx = self.shape
        self.N = nx * ny * nz
        self.device = torch.device(device)
        self.stream = stream
        self.nparams = int(self.lib.mlb_net_param_count())
        nbytes = int(self.lib.mlb_net_workspace_bytes(nx, ny, nz, 1 if training else 0))
        if nbytes == 0:
            raise MlbError(-1, "mlb_net_workspace_bytes", self.lib.mlb_last_error().decode())
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self.ws = raw[off:off + nbytes]
        h = C.c_void_p()
        _lib.check(self.lib.mlb_net_create(nx, ny, nz, 1 if training else 0, C.c_void_p(self.ws.data_ptr()), nbytes,
                                           _stream_handle(stream), C.byref(h)), "mlb_net_create")
        self.h = h

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.mlb_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params) -> None:
        flat = params if isinstance(params, np.ndarray) else net_flatten(params)
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        assert flat.size == self.nparams
        _lib.check(self.lib.mlb_net_set_params(self.h, flat.ctypes.data_as(C.POINTER(C.c_float)),
                                               _stream_handle(self.stream)), "mlb_net_set_params")

    def get_params(self, flat: bool = False):
        out = np.empty(self.nparams, dtype=np.float32)
        _lib.check(self.lib.mlb_net_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float)),
                                               _stream_handle(self.stream)), "mlb_net_get_params")
        return out if flat else net_unflatten(out)

    def set_scales(self, n_ref: float, j_ref: float, f_ref: float) -> None:
        _lib.check(self.lib.mlb_net_set_scales(self.h, float(n_ref), float(j_ref), float(f_ref)),
                   "mlb_net_set_scales")
        self.scales = (float(n_ref), float(j_ref), float(f_ref))

    def _dev(self, x, channels):
        torch = _torch()
        x = torch.as_tensor(x).to(device=self.device, dtype=torch.float32).contiguous()
        assert x.numel() == channels * self.N
        return x

    def forward(self, x):
        """x [14][nz][ny][nx] -> y [6][nz][ny][nx] (float32 device tensors)."""
        torch = _torch()
        x = self._dev(x, NET_CHANNELS[0])
        y = torch.empty((6,) + self.shape, dtype=torch.float32, device=self.device)
        _lib.check(self.lib.mlb_net_forward(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                            _stream_handle(self.stream)), "mlb_net_forward")
        return y

    def pool_stats(self, x, t):
        """(mean square of the momentum channels of x over the pool, [mean square
        of each target]) for a pool x [S][14][...], t [S][6][...] (mlb_net_pool_stats)."""
        S = int(x.shape[0])
        assert x.is_contiguous() and t.is_contiguous()
        assert x.numel() == S * NET_CHANNELS[0] * self.N and t.numel() == S * 6 * self.N
        out = (C.c_double * (S + 1))()
        _lib.check(self.lib.mlb_net_pool_stats(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), S, out,
                                               _stream_handle(self.stream)), "mlb_net_pool_stats")
        return float(out[0]), [float(v) for v in out[1:]]

    def pool_rescale(self, x, t, j_div: float, f_div: float) -> None:
        """In place: x's momentum channels / j_div, its gradient channels and t / f_div (mlb_net_pool_rescale)."""
        S = int(x.shape[0])
        assert x.is_contiguous() and t.is_contiguous()
        assert x.numel() == S * NET_CHANNELS[0] * self.N and t.numel() == S * 6 * self.N
        _lib.check(self.lib.mlb_net_pool_rescale(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), S,
                                                 float(j_div), float(f_div), _stream_handle(self.stream)),
                   "mlb_net_pool_rescale")

    def rel_error(self, y, t) -> float:
        """||y - t|| / ||t|| over [6][...] float32 device tensors (mlb_net_rel_error)."""
        y = self._dev(y, 6)
        t = self._dev(t, 6)
        err = C.c_double()
        _lib.check(self.lib.mlb_net_rel_error(self.h, C.c_void_p(y.data_ptr()), C.c_void_p(t.data_ptr()),
                                              C.byref(err), _stream_handle(self.stream)), "mlb_net_rel_error")
        return float(err.value)

    def train_step(self, x, target, lr: float = 1e-3, update: bool = True, want_loss: bool = True,
                   want_grads: bool = False, loss_weight: float = 1.0):
        """One Adam step on loss_weight x MSE; returns (loss before the update or None, gradients or None)."""
        x = self._dev(x, NET_CHANNELS[0])
        t = self._dev(target, 6)
        loss = C.c_double()
        grads = np.empty(self.nparams, dtype=np.float32) if want_grads else None
        _lib.check(self.lib.mlb_net_train_step(
            self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), float(lr), float(loss_weight),
            1 if update else 0,
            C.byref(loss) if want_loss else None,
            grads.ctypes.data_as(C.POINTER(C.c_float)) if want_grads else None,
            _stream_handle(self.stream)), "mlb_net_train_step")
        self._keep = (x, t)
        return (float(loss.value) if want_loss else None), (net_unflatten(grads) if want_grads else None)

    @property
    def adam_steps(self) -> int:
        return int(self.lib.mlb_net_adam_steps(self.h))


__all__ += ["GpuNet", "net_flatten", "net_unflatten", "NET_CHANNELS"]
