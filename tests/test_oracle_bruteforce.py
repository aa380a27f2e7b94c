"""Brute-force pin of the oracle's non-local sums (no stencil tables).

Every force term is re-evaluated by looping over ALL pairs of lattice sites
(minimum image in the periodic directions), selecting pairs by the distance
rules alone, on grids small enough for O(N^2):
  hard-core mean field         eq. (potmeanforce)
  attractive RPA field         below eq. (potmeanforce)
  drag + viscous pair form     eqs. (gammaab), (tensorgamma), (viscousforce)
  friction rate, predictor, corrector, the BMCSL contact values of
  ball-smoothed packing fractions.
"""
import math

import numpy as np
import pytest

import workloads as W

KT = 1.0 / 3.0
CV = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
               [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
               [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=float)


def _pairs(m):
    z, y, x = np.meshgrid(np.arange(m.nz), np.arange(m.ny), np.arange(m.nx), indexing="ij")
    P = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    E = P[None, :, :] - P[:, None, :]          # E[s, s'] = r' - r
    for d, L in ((0, m.nx), (2, m.nz)):
        E[..., d] = (E[..., d] + L // 2) % L - L // 2
    if not m.walls_y:
        E[..., 1] = (E[..., 1] + m.ny // 2) % m.ny - m.ny // 2
    R2 = (E ** 2).sum(-1)
    return E.astype(float), R2, P


def _ball_count(R):
    k = int(math.ceil(R)) + 1
    g = np.arange(-k, k + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return int(((X ** 2 + Y ** 2 + Z ** 2) <= R * R).sum())


def brute_force(m, f):
    M, N = m.M, m.N
    fl = f.reshape(M, 19, N)
    n = fl.sum(1)
    j = np.einsum("aiN,id->adN", fl, CV)
    E, R2, P = _pairs(m)
    solid = np.zeros(N, bool)
    if m.walls_y:
        solid = (P[:, 1] == 0) | (P[:, 1] == m.ny - 1)
    sig = m.sigma
    # smoothed densities and contact values
    nbar = np.zeros((M, N))
    for c in range(M):
        R = sig[c] / 2
        nbar[c] = ((R2 <= R * R) * n[c][None, :]).sum(1) / _ball_count(R)
    x2 = sum(math.pi / 6 * sig[c] ** 2 * nbar[c] for c in range(M))
    x3 = sum(math.pi / 6 * sig[c] ** 3 * nbar[c] for c in range(M))
    g = {}
    for a in range(M):
        for b in range(M):
            d = sig[a] * sig[b] / (sig[a] + sig[b])
            gab = 1 / (1 - x3) + 3 * d * x2 / (1 - x3) ** 2 + 2 * (d * x2) ** 2 / (1 - x3) ** 3
            g[a, b] = np.where(solid, 0.0, gab)
    with np.errstate(invalid="ignore", divide="ignore"):
        Eh = np.where(R2[..., None] > 0, E / np.sqrt(R2)[..., None], 0.0)
    eps = m.eps_matrix()
    out = {k: np.zeros((M, 3, N)) for k in ("Nmf", "Ntail", "Dold")}
    gam = np.zeros((M, N))
    shells = {}
    for a in range(M):
        for b in range(M):
            sab = 0.5 * (sig[a] + sig[b])
            S = (R2 >= (sab - 0.5) ** 2) & (R2 < (sab + 0.5) ** 2)
            count = S[0].sum() if not m.walls_y else None
            # shell size from a periodic reference (walls truncate rows, not the set)
            k = int(sab) + 2
            gg = np.arange(-k, k + 1)
            X, Y, Z = np.meshgrid(gg, gg, gg, indexing="ij")
            rr = X ** 2 + Y ** 2 + Z ** 2
            count = int(((rr >= (sab - 0.5) ** 2) & (rr < (sab + 0.5) ** 2)).sum())
            what = 4 * math.pi / count
            kap = 2 * sab ** 2 * math.sqrt(2 * 0.5 * KT / math.pi) * what
            G = 0.5 * (g[a, b][:, None] + g[a, b][None, :]) * S
            shells[a, b] = (G, kap)
            out["Nmf"][a] += -KT * sab ** 2 * what * n[a][None, :] * np.einsum("sr,srd->ds", G * n[b][None, :], Eh)
            gam[a] += kap / 3 * (G * n[b][None, :]).sum(1)
            X_ = n[a][:, None, None] * j[b].T[None, :, :] - n[b][None, :, None] * j[a].T[:, None, :]
            proj = (Eh * X_).sum(-1)
            out["Dold"][a] += kap * np.einsum("sr,srd->ds", G * proj, Eh)
            if eps[a, b] != 0:
                T = (R2 > sab ** 2) & (R2 <= (m.rc_factor * sab) ** 2)
                with np.errstate(divide="ignore"):
                    Up = np.where(T, 6 * eps[a, b] * sab ** 6 / np.where(R2 > 0, R2, 1) ** 3.5, 0.0)
                out["Ntail"][a] += n[a][None, :] * np.einsum("sr,srd->ds", Up * n[b][None, :], Eh)
    fx = m.fext_matrix()
    Next = n[:, None, :] * fx[:, :, None]
    Nc = out["Nmf"] + out["Ntail"] + Next
    hg = 0.5 * gam
    with np.errstate(invalid="ignore", divide="ignore"):
        V = np.where(n[:, None, :] > 0, (j + Nc + out["Dold"] + hg[:, None, :] * j)
                     / (n[:, None, :] * (1 + hg[:, None, :])), 0.0)
    H = Nc + 0.5 * out["Dold"]
    Dnew = np.zeros((M, 3, N))
    for a in range(M):
        for b in range(M):
            G, kap = shells[a, b]
            Y_ = V[b].T[None, :, :] - V[a].T[:, None, :]
            proj = (Eh * Y_).sum(-1)
            Dnew[a] += kap * n[a][None, :] * np.einsum("sr,srd->ds", G * n[b][None, :] * proj, Eh)
    Nf = H + 0.5 * Dnew
    for k in ("Nmf", "Ntail", "Dold"):
        out[k][:, :, solid] = 0
    V[:, :, solid] = 0
    H[:, :, solid] = 0
    Dnew[:, :, solid] = 0
    Nf[:, :, solid] = 0
    gam[:, solid] = 0
    sh = (M, 3) + m.shape()
    res = {k: v.reshape(sh) for k, v in out.items()}
    res.update(n=n.reshape((M,) + m.shape()), j=j.reshape(sh), gam=gam.reshape((M,) + m.shape()),
               vhat=V.reshape(sh), H=H.reshape(sh), Dnew=Dnew.reshape(sh), N=Nf.reshape(sh),
               Next=Next.reshape(sh))
    P_ = [(a, b) for a in range(M) for b in range(a, M)]
    res["g"] = np.stack([g[a, b] for a, b in P_]).reshape((len(P_),) + m.shape())
    return res


def _compare(oracle_lib, m, n0, u0, steps=2, rtol=1e-11):
    o = oracle_lib.Oracle(m)
    f = o.step(o.init(n0, u0), steps)    # a few steps so the fields are not the IC
    d = o.fields(f)
    b = brute_force(m, f)
    for k in ("n", "j", "g", "gam", "Nmf", "Ntail", "Next", "Dold", "vhat", "H", "Dnew", "N"):
        scale = max(np.abs(b[k]).max(), 1e-300)
        err = np.abs(d[k] - b[k]).max() / scale
        assert err < rtol, (k, err)


def test_bruteforce_binary_periodic(oracle_lib):
    m = W.Mixture(8, 8, 8, sigma=(2.0, 3.0))
    n0, u0 = W.random_state(m, [0.012, 0.009], rel=0.4, u_amp=0.03, seed=11)
    _compare(oracle_lib, m, n0, u0)


def test_bruteforce_ternary_tail_external(oracle_lib):
    eps = np.array([[0.1, 0.12, 0.08], [0.12, 0.15, 0.05], [0.08, 0.05, 0.2]])
    fx = np.array([[1e-5, 0, 0], [0, -2e-5, 0], [0, 0, 3e-5]])
    m = W.Mixture(12, 12, 12, sigma=(1.5, 2.0, 2.5), eps=eps, rc_factor=2.0, fext=fx)
    n0, u0 = W.random_state(m, [0.03, 0.015, 0.008], rel=0.4, u_amp=0.03, seed=12)
    _compare(oracle_lib, m, n0, u0, steps=1)


def test_bruteforce_walls(oracle_lib):
    m = W.Mixture(8, 9, 8, sigma=(2.0, 3.0), walls_y=True, wall_ux=(-0.03, 0.04))
    n0, u0 = W.random_state(m, [0.012, 0.009], rel=0.4, u_amp=0.03, seed=13)
    _compare(oracle_lib, m, n0, u0)


def test_bruteforce_step_profile_with_empty_species(oracle_lib):
    m, n0, u0 = W.config_step_binary(8, 8, 8)
    _compare(oracle_lib, m, n0, u0, steps=3)


def test_bruteforce_forward_euler(oracle_lib):
    m = W.Mixture(8, 8, 8, sigma=(2.0, 2.5), scheme=W.SCHEME_FE)
    n0, u0 = W.random_state(m, [0.012, 0.009], rel=0.4, u_amp=0.03, seed=14)
    o = oracle_lib.Oracle(m)
    f = o.init(n0, u0)
    d = o.fields(f)
    b = brute_force(m, f)
    ref = b["Nmf"] + b["Ntail"] + b["Next"] + b["Dold"]
    np.testing.assert_allclose(d["N"], ref, rtol=0, atol=1e-11 * np.abs(ref).max())
