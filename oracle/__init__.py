"""FP64 CPU oracle (ctypes wrapper around liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library or its binding.
It shares no code with the GPU path; both take their inputs from the
`workloads` module.

The C library computes the lattice step of the multicomponent kinetic
equation (Sec. 2, eq. evolution) with the self-consistent field of Sec. 3
(eqs. splitforce, potmeanforce, gammaab, tensorgamma, viscousforce); see
mlb_oracle.c for the per-step definition.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

from workloads import MAX_SPECIES, Mixture

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
Q = 19

_lib = None


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("M", C.c_int32),
        ("tau", C.c_double), ("kT", C.c_double),
        ("sigma", C.c_double * MAX_SPECIES),
        ("eps", C.c_double * (MAX_SPECIES * MAX_SPECIES)),
        ("rc_factor", C.c_double),
        ("fext", C.c_double * (MAX_SPECIES * 3)),
        ("walls_y", C.c_int32),
        ("wall_ux", C.c_double * 2),
        ("scheme", C.c_int32),
        ("mass", C.c_double * MAX_SPECIES),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    dp = C.POINTER(C.c_double)
    lib.or_create.restype = C.c_void_p
    lib.or_create.argtypes = [C.POINTER(_Params)]
    lib.or_destroy.argtypes = [C.c_void_p]
    lib.or_init.argtypes = [C.c_void_p, dp, dp, dp]
    lib.or_step.argtypes = [C.c_void_p, dp, dp, C.c_int]
    lib.or_fields.argtypes = [C.c_void_p, dp] + [dp] * 9
    lib.or_collide_site.argtypes = [C.c_void_p, C.c_int, dp, C.c_double, dp, dp, dp, dp]
    lib.or_stencil.restype = C.c_int
    lib.or_stencil.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), dp]
    lib.or_pair_constants.argtypes = [C.c_void_p, C.c_int, C.c_int, dp]
    lib.or_moments.argtypes = [C.c_void_p, dp, dp]
    lib.or_step_ext.argtypes = [C.c_void_p, dp, dp, dp]
    lib.or_set_force_profile.argtypes = [C.c_void_p, dp]
    lib.or_threads.restype = C.c_int
    lib.or_set_threads.argtypes = [C.c_int]
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def threads() -> int:
    return _load().or_threads()


def set_threads(n: int) -> None:
    _load().or_set_threads(int(n))


class Oracle:
    """One mixture on the CPU in FP64."""

    def __init__(self, m: Mixture):
        lib = _load()
        p = _Params()
        p.nx, p.ny, p.nz, p.M = m.nx, m.ny, m.nz, m.M
        p.tau, p.kT = m.tau, m.kT
        for a in range(m.M):
            p.sigma[a] = m.sigma[a]
        e = m.eps_matrix()
        for a in range(m.M):
            for b in range(m.M):
                p.eps[a * MAX_SPECIES + b] = e[a, b]
        p.rc_factor = m.rc_factor
        fx = m.fext_matrix()
        for a in range(m.M):
            for d in range(3):
                p.fext[a * 3 + d] = fx[a, d]
        p.walls_y = 1 if m.walls_y else 0
        p.wall_ux[0], p.wall_ux[1] = m.wall_ux
        p.scheme = m.scheme
        for a, ma in enumerate(m.mass_vector()):
            p.mass[a] = float(ma)
        self._h = lib.or_create(C.byref(p))
        if not self._h:
            raise ValueError("oracle rejected the mixture parameters")
        self.m = m
        self.M, self.N = m.M, m.N
        self.P = m.M * (m.M + 1) // 2

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_destroy(h)
            self._h = None

    def set_force_profile(self, profile: Optional[np.ndarray]) -> None:
        """Body force per lattice row [M][3][ny] added to the uniform one (None removes it)."""
        if profile is None:
            _lib.or_set_force_profile(self._h, None)
            return
        prof = np.ascontiguousarray(profile, dtype=np.float64)
        assert prof.shape == (self.M, 3, self.m.ny)
        _lib.or_set_force_profile(self._h, _ptr(prof))

    # ---------------------------------------------------------------- state
    def init(self, n0: np.ndarray, u0: np.ndarray) -> np.ndarray:
        n0 = np.ascontiguousarray(n0, dtype=np.float64)
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        assert n0.size == self.M * self.N and u0.size == 3 * self.M * self.N
        f = np.zeros((self.M, Q) + self.m.shape())
        _lib.or_init(self._h, _ptr(n0), _ptr(u0), _ptr(f))
        return f

    def step(self, f: np.ndarray, nsteps: int = 1) -> np.ndarray:
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.empty_like(f)
        _lib.or_step(self._h, _ptr(f), _ptr(out), int(nsteps))
        return out

    def densities(self, f: np.ndarray) -> np.ndarray:
        f = np.ascontiguousarray(f, dtype=np.float64)
        n = np.empty((self.M,) + self.m.shape())
        _lib.or_moments(self._h, _ptr(f), _ptr(n))
        return n

    # ---------------------------------------------------- FFT attractive field
    def _tail_spectra(self):
        """FFT of the attractive kernels w_ab placed on the periodic grid
        (the convolution the direct sum evaluates; pinned to it by the tests)."""
        if getattr(self, "_spec", None) is not None:
            return self._spec
        m = self.m
        eps = m.eps_matrix()
        spec = {}
        for a in range(self.M):
            for b in range(a, self.M):
                if eps[a, b] == 0:
                    continue
                e, w = self.stencil("tail", a, b)
                K = np.zeros((3,) + m.shape())
                for sgn in (1, -1):
                    idx = ((sgn * e[:, 2]) % m.nz, (sgn * e[:, 1]) % m.ny, (sgn * e[:, 0]) % m.nx)
                    for d in range(3):
                        np.add.at(K[d], idx, sgn * w[:, d])
                # sum_e w(e) n(r + e) = ifft(conj(fft(w)) fft(n))
                spec[(a, b)] = np.conj(np.fft.rfftn(K, axes=(1, 2, 3)))
        self._spec = spec
        return spec

    def tail_field_fft(self, n: np.ndarray) -> np.ndarray:
        """sum_b (K_ab * n_b) [M][3][N] by FFT, float64."""
        spec = self._tail_spectra()
        m = self.m
        nh = np.fft.rfftn(n, axes=(1, 2, 3))
        out = np.zeros((self.M, 3) + m.shape())
        for a in range(self.M):
            acc = None
            for b in range(self.M):
                key = (min(a, b), max(a, b))
                if key not in spec:
                    continue
                term = spec[key] * nh[b][None]
                acc = term if acc is None else acc + term
            if acc is not None:
                out[a] = np.fft.irfftn(acc, s=m.shape(), axes=(1, 2, 3))
        return out

    def step_fft(self, f: np.ndarray, nsteps: int = 1) -> np.ndarray:
        """Steps with the attractive field by FFT instead of the ordered direct sum."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        for _ in range(int(nsteps)):
            tail = np.ascontiguousarray(self.tail_field_fft(self.densities(f)))
            out = np.empty_like(f)
            _lib.or_step_ext(self._h, _ptr(f), _ptr(out), _ptr(tail))
            f = out
        return f

    def fields(self, f: np.ndarray) -> Dict[str, np.ndarray]:
        f = np.ascontiguousarray(f, dtype=np.float64)
        sh = self.m.shape()
        out = {
            "n": np.empty((self.M,) + sh), "j": np.empty((self.M, 3) + sh),
            "u": np.empty((3,) + sh), "g": np.empty((self.P,) + sh),
            "vhat": np.empty((self.M, 3) + sh), "H": np.empty((self.M, 3) + sh),
            "N": np.empty((self.M, 3) + sh), "parts": np.empty((5, self.M, 3) + sh),
            "gam": np.empty((self.M,) + sh),
        }
        _lib.or_fields(self._h, _ptr(f), *[_ptr(out[k]) for k in
                                            ("n", "j", "u", "g", "vhat", "H", "N", "parts", "gam")])
        p = out.pop("parts")
        out["Nmf"], out["Ntail"], out["Next"], out["Dold"], out["Dnew"] = p
        return out

    def moments(self, f: np.ndarray):
        d = self.fields(f)
        return d["n"], d["j"]

    # ---------------------------------------------------------------- hooks
    def collide_site(self, fi, na, ja, u, Na, species: int = 0) -> np.ndarray:
        """f*_i of one site of `species` (its mass sets the equilibrium's theta)."""
        fi = np.ascontiguousarray(fi, dtype=np.float64)
        ja = np.ascontiguousarray(ja, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        Na = np.ascontiguousarray(Na, dtype=np.float64)
        out = np.empty(Q)
        _lib.or_collide_site(self._h, int(species), _ptr(fi), float(na), _ptr(ja), _ptr(u), _ptr(Na), _ptr(out))
        return out

    def stencil(self, which: str, a: int, b: int = 0):
        code = {"shell": 0, "tail": 1, "ball": 2}[which]
        n = _lib.or_stencil(self._h, code, a, b, None, None)
        e = np.zeros((max(n, 1), 3), dtype=np.int32)
        w = np.zeros((max(n, 1), 3))
        _lib.or_stencil(self._h, code, a, b, e.ctypes.data_as(C.POINTER(C.c_int)), _ptr(w))
        return e[:n].copy(), w[:n].copy()

    def pair_constants(self, a: int, b: int) -> Dict[str, float]:
        out = np.zeros(4)
        _lib.or_pair_constants(self._h, a, b, _ptr(out))
        return {"cm": out[0], "cg": out[1], "ck": out[2], "d": out[3]}


def pair_index(M: int, a: int, b: int) -> int:
    lo, hi = min(a, b), max(a, b)
    return lo * M - (lo * (lo - 1)) // 2 + (hi - lo)
