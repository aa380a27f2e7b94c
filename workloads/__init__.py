"""Seeded synthetic workloads: mixture parameters and initial fields.

This module is shared by the GPU path and the CPU oracle, so it holds no
step arithmetic: only parameter values, lattice sizes and initial density /
velocity arrays drawn from stated seeds.  Every array it returns is float64,
species-major, x fastest:  n0 [M][nz][ny][nx],  u0 [M][3][nz][ny][nx].

Packing fraction convention (hard-sphere mixtures, used to turn the stated
packing into a number density):  xi = (pi/6) sum_c n_c sigma_c^3.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

KT = 1.0 / 3.0          # kT/m = c_s^2 of D3Q19 with unit masses
MAX_SPECIES = 4

SCHEME_CN_J1 = 0        # Crank-Nicolson friction, one Jacobi predictor sweep
SCHEME_FE = 1           # forward Euler (study option; unstable at dense states)


@dataclasses.dataclass
class Mixture:
    """Plain description of one periodic (optionally y-walled) mixture."""
    nx: int
    ny: int
    nz: int
    sigma: Tuple[float, ...]                 # sigma_aa, lattice units
    tau: float = 1.0
    kT: float = KT
    eps: Optional[np.ndarray] = None         # [M][M] attraction depth (0 = off)
    rc_factor: float = 2.5
    fext: Optional[np.ndarray] = None        # [M][3] uniform external force
    walls_y: bool = False
    wall_ux: Tuple[float, float] = (0.0, 0.0)  # x velocity of the y=0 / y=ny-1 wall
    scheme: int = SCHEME_CN_J1
    name: str = ""
    mass: Optional[Tuple[float, ...]] = None  # m_a (None: all 1); kT / m_a is the species' thermal speed^2

    @property
    def M(self) -> int:
        return len(self.sigma)

    def mass_vector(self) -> np.ndarray:
        if self.mass is None:
            return np.ones(self.M)
        return np.asarray(self.mass, dtype=np.float64).reshape(self.M)

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    def eps_matrix(self) -> np.ndarray:
        if self.eps is None:
            return np.zeros((self.M, self.M))
        return np.asarray(self.eps, dtype=np.float64).reshape(self.M, self.M)

    def fext_matrix(self) -> np.ndarray:
        if self.fext is None:
            return np.zeros((self.M, 3))
        return np.asarray(self.fext, dtype=np.float64).reshape(self.M, 3)

    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)


def number_density(packing: float, x: Sequence[float], sigma: Sequence[float]) -> float:
    """Total number density for packing fraction `packing` at mole fractions x."""
    return packing / ((math.pi / 6.0) * sum(xc * s ** 3 for xc, s in zip(x, sigma)))


def _zeros_u(m: Mixture) -> np.ndarray:
    return np.zeros((m.M, 3) + m.shape())


def _fluid_mask(m: Mixture) -> np.ndarray:
    mask = np.ones(m.shape(), dtype=bool)
    if m.walls_y:
        mask[:, 0, :] = False
        mask[:, m.ny - 1, :] = False
    return mask


# ------------------------------------------------------------ initial states
def uniform_state(m: Mixture, n: Sequence[float], u: Optional[np.ndarray] = None):
    """Uniform densities n[a]; optional uniform species velocities u[a][3]."""
    n0 = np.zeros((m.M,) + m.shape())
    for a in range(m.M):
        n0[a] = n[a]
    u0 = _zeros_u(m)
    if u is not None:
        u = np.asarray(u, dtype=np.float64).reshape(m.M, 3)
        for a in range(m.M):
            for d in range(3):
                u0[a, d] = u[a, d]
    n0 *= _fluid_mask(m)
    return n0, u0


def step_state(m: Mixture, n_total: float, x_split: Optional[int] = None):
    """Composition step along x: species 0 left of x_split, species 1 right."""
    xs = m.nx // 2 if x_split is None else x_split
    n0 = np.zeros((m.M,) + m.shape())
    n0[0, :, :, :xs] = n_total
    n0[1, :, :, xs:] = n_total
    return n0 * _fluid_mask(m), _zeros_u(m)


def mode_state(m: Mixture, n_total: float, x1: float, amplitude: float,
               noise: float = 0.0, seed: int = 0, wavelength: Optional[int] = None):
    """Binary composition mode along x: n_0 = n (x1 + A sin kx), n_1 = n (1 - x1 - A sin kx),
    then each density times (1 + noise U(-1,1)), i.i.d. per site and species."""
    L = m.nx if wavelength is None else wavelength
    x = np.arange(m.nx, dtype=np.float64)
    s = np.sin(2.0 * math.pi * x / L)
    n0 = np.zeros((m.M,) + m.shape())
    n0[0] = (n_total * (x1 + amplitude * s))[None, None, :]
    n0[1] = (n_total * ((1.0 - x1) - amplitude * s))[None, None, :]
    if noise > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        n0 *= 1.0 + noise * rng.uniform(-1.0, 1.0, size=n0.shape)
    return n0 * _fluid_mask(m), _zeros_u(m)


def random_state(m: Mixture, n_mean: Sequence[float], rel: float = 0.2, u_amp: float = 0.02,
                 seed: int = 0):
    """Positive random densities around n_mean and random species velocities
    (for per-kernel parity and brute-force checks)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n0 = np.zeros((m.M,) + m.shape())
    for a in range(m.M):
        n0[a] = n_mean[a] * (1.0 + rel * rng.uniform(-1.0, 1.0, size=m.shape()))
    u0 = u_amp * rng.uniform(-1.0, 1.0, size=(m.M, 3) + m.shape())
    mask = _fluid_mask(m)
    return n0 * mask, u0 * mask


def tracer_band_state(m: Mixture, n_total: float, amplitude: float = 0.05, width: float = 8.0):
    """Ternary: species 0:1 equimolar background, tracer species 2 as a Gaussian
    band in x (standard deviation `width`) replacing 0 and 1 proportionally."""
    x = np.arange(m.nx, dtype=np.float64)
    band = amplitude * np.exp(-((x - m.nx / 2) ** 2) / (2.0 * width ** 2))
    n0 = np.zeros((m.M,) + m.shape())
    n0[2] = (n_total * band)[None, None, :]
    n0[0] = (n_total * 0.5 * (1.0 - band))[None, None, :]
    n0[1] = (n_total * 0.5 * (1.0 - band))[None, None, :]
    return n0 * _fluid_mask(m), _zeros_u(m)


# ------------------------------------------------------------------ configs
def config_step_binary(nx=64, ny=12, nz=12) -> Tuple[Mixture, np.ndarray, np.ndarray]:
    """Binary hard spheres, sigma = 2 and 3, total packing 0.2 as a box
    average, composition step along x, zero velocity, tau = 1."""
    m = Mixture(nx, ny, nz, sigma=(2.0, 3.0), tau=1.0, name=f"step_binary_{nx}x{ny}x{nz}")
    n = number_density(0.2, (0.5, 0.5), m.sigma)
    n0, u0 = step_state(m, n)
    return m, n0, u0


def config_bulk_diffusion(nx=128, ny=32, nz=32, seed=2024, noise=0.01) -> Tuple[Mixture, np.ndarray, np.ndarray]:
    """Binary, sigma = 3 and 4.5, packing 0.3, x1 = 0.5, attractive tail
    -eps (sigma/r)^6 with eps/kT = 0.5 and cutoff 2.5 sigma_ab; sinusoidal
    composition mode of amplitude 0.05 plus 1 % seeded uniform noise."""
    eps = np.full((2, 2), 0.5 * KT)
    m = Mixture(nx, ny, nz, sigma=(3.0, 4.5), eps=eps, rc_factor=2.5,
                name=f"bulk_diffusion_{nx}x{ny}x{nz}")
    n = number_density(0.3, (0.5, 0.5), m.sigma)
    n0, u0 = mode_state(m, n, 0.5, 0.05, noise=noise, seed=seed)
    return m, n0, u0


def config_taylor_couette(nx=256, ny=64, nz=16, U=0.05, packing=0.25) -> Tuple[Mixture, np.ndarray, np.ndarray]:
    """Ternary, sigma = 2, 3, 4, packing 0.25 (or `packing`), eps/kT = 0.3
    (cutoff 2.5 sigma), bounce-back walls at y = 0 and ny-1 moving at -U and
    +U, Gaussian tracer band of species 3 (width 8) centred in x."""
    eps = np.full((3, 3), 0.3 * KT)
    m = Mixture(nx, ny, nz, sigma=(2.0, 3.0, 4.0), eps=eps, rc_factor=2.5, walls_y=True,
                wall_ux=(-U, U), name=f"taylor_couette_{nx}x{ny}x{nz}")
    n = number_density(packing, (0.5, 0.5), m.sigma[:2])
    n0, u0 = tracer_band_state(m, n)
    return m, n0, u0


def config_closure_physics(nx=192, ny=64, nz=64, amplitude=0.05) -> Tuple[Mixture, np.ndarray, np.ndarray]:
    """Binary at the step-binary physics (sigma = 2 and 3, packing 0.2, no
    tail) with a composition mode x1 = 0.5 +- 0.05 along x."""
    m = Mixture(nx, ny, nz, sigma=(2.0, 3.0), tau=1.0, name=f"closure_{nx}x{ny}x{nz}")
    n = number_density(0.2, (0.5, 0.5), m.sigma)
    n0, u0 = mode_state(m, n, 0.5, amplitude)
    return m, n0, u0


@dataclasses.dataclass
class EnsembleMember:
    mixture: Mixture
    n0: np.ndarray
    u0: np.ndarray
    x1: float
    packing: float


def config_ensemble(count=64, seed=4242, edges=(32, 48, 64, 96), amplitude=0.05,
                    edge_cap: Optional[int] = None) -> List[EnsembleMember]:
    """Independent periodic binary systems: each box edge drawn from `edges`,
    x1 ~ U[0.1, 0.9], packing ~ U[0.1, 0.35], sigma_11 = 2 and
    sigma_22 = 2 U[1, 2]; a composition mode along x as initial state.
    `edge_cap` (tests only) clips edges to keep systems small."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(count):
        ex, ey, ez = (int(v) for v in rng.choice(np.asarray(edges), size=3))
        x1 = float(rng.uniform(0.1, 0.9))
        xi = float(rng.uniform(0.1, 0.35))
        s2 = 2.0 * float(rng.uniform(1.0, 2.0))
        if edge_cap is not None:
            ex, ey, ez = min(ex, edge_cap), min(ey, edge_cap), min(ez, edge_cap)
        m = Mixture(ex, ey, ez, sigma=(2.0, s2), tau=1.0, name=f"ensemble_{k}")
        n = number_density(xi, (x1, 1.0 - x1), m.sigma)
        n0, u0 = mode_state(m, n, x1, amplitude)
        out.append(EnsembleMember(m, n0, u0, x1, xi))
    return out


# ----------------------------------------------- attractive tails (Sec. 4.1)
def berthelot_eps(w: Sequence[float], sigma: Sequence[float], rc_factor: float = 2.5) -> np.ndarray:
    """Depths eps_ab of the tails U_ab = -eps_ab (sigma_ab / r)^6, sigma_ab < r
    <= rc sigma_ab, whose strengths w_ab = int d^3r U_ab(r) (the w_0 of the
    paper's linear estimate) follow the geometric-mean (Lorentz-Berthelot)
    rule w_ab = sqrt(w_aa w_bb) from the like strengths w[a] (negative:
    attraction).  int U = -(4 pi / 3) eps sigma^3 (1 - rc^-3)."""
    M = len(sigma)
    eps = np.zeros((M, M))
    for a in range(M):
        for b in range(M):
            wab = -math.sqrt(w[a] * w[b])
            sab = 0.5 * (sigma[a] + sigma[b])
            eps[a, b] = -wab / (4.0 * math.pi / 3.0 * sab ** 3 * (1.0 - rc_factor ** -3))
    return eps


def config_tail_study(sigma: float, packing: float, x1: float, w_aa: float = -5.0 * KT,
                      tails: bool = True, nx: Optional[int] = None, amplitude: float = 0.05):
    """Equal-diameter binary at the stated packing and mole fraction x1 with
    Lorentz-Berthelot tails of strengths w_AA and w_BB = w_AA / 2 (the
    attraction of the paper's D(c) study, Sec. 4.1), or none; a composition
    mode along x of wavelength nx.  The cross-section is just wider than the
    tail's reach."""
    rc = 2.5
    reach = int(math.floor(rc * sigma))
    ny = reach + 3
    L = nx if nx is not None else 32 * int(sigma)
    eps = berthelot_eps([w_aa, 0.5 * w_aa], (sigma, sigma), rc) if tails else None
    m = Mixture(L, ny, ny, sigma=(sigma, sigma), eps=eps, rc_factor=rc,
                name=f"tail_study_s{sigma:g}_x{x1:g}_{'lb' if tails else 'hs'}")
    n = number_density(packing, (x1, 1.0 - x1), m.sigma)
    n0, u0 = mode_state(m, n, x1, amplitude)
    return m, n0, u0
