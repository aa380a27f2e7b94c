"""Brute-force pin of the oracle's non-local sums (no stencil tables).

Every force term is re-evaluated by looping over ALL pairs of lattice sites
(minimum image in the periodic directions), selecting pairs by the distance
rules alone, on grids small enough for O(N^2):
  hard-core mean field         eq. (potmeanforce)
  attractive RPA field         below eq. (potmeanforce)
  drag + viscous pair form     eqs. (gammaab), (tensorgamma), (viscousforce)
  friction rate, predictor, corrector, the BMCSL contact values of
  ball-smoothed packing fractions.
In a walled box the hard-core sums (balls, shells) also run over the mirror
images of the fluid across the wall planes, which move with the walls; the
attractive field runs over the fluid only.
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
    """Displacements from every target site to every source point.  In a
    periodic box the sources are the sites (minimum image).  In a walled box
    they are the fluid sites plus their mirror images across the wall planes
    y = 1/2 and y = ny - 3/2 (the hard-core stencils' view beyond a wall);
    `img` is 0 for a fluid source, 1 / 2 for an image beyond the y = 0 /
    y = ny - 1 wall, `src` the fluid site a source takes its fields from."""
    z, y, x = np.meshgrid(np.arange(m.nz), np.arange(m.ny), np.arange(m.nx), indexing="ij")
    P = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    N = len(P)
    if m.walls_y:
        fluid = np.flatnonzero((P[:, 1] > 0) & (P[:, 1] < m.ny - 1))
        lo = P[fluid].copy()
        lo[:, 1] = 1 - lo[:, 1]
        hi = P[fluid].copy()
        hi[:, 1] = 2 * m.ny - 3 - hi[:, 1]
        Q = np.concatenate([P[fluid], lo, hi])
        src = np.concatenate([fluid, fluid, fluid])
        img = np.concatenate([np.zeros(len(fluid), int), np.ones(len(fluid), int), 2 * np.ones(len(fluid), int)])
    else:
        Q, src, img = P, np.arange(N), np.zeros(N, int)
    E = Q[None, :, :] - P[:, None, :]          # E[s, q] = r_q - r_s
    for d, L in ((0, m.nx), (2, m.nz)):
        E[..., d] = (E[..., d] + L // 2) % L - L // 2
    if not m.walls_y:
        E[..., 1] = (E[..., 1] + m.ny // 2) % m.ny - m.ny // 2
    R2 = (E ** 2).sum(-1)
    return E.astype(float), R2, P, src, img


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
    E, R2, P, src, img = _pairs(m)
    solid = np.zeros(N, bool)
    if m.walls_y:
        solid = (P[:, 1] == 0) | (P[:, 1] == m.ny - 1)
    sig = m.sigma
    # fields at the sources: an image has its fluid site's density and contact
    # value and the wall's velocity
    ns = n[:, src]
    js = j[:, :, src].copy()
    wall_u = np.zeros((len(src), 3))
    for k, uw in ((1, m.wall_ux[0]), (2, m.wall_ux[1])):
        wall_u[img == k, 0] = uw
    js[:, :, img > 0] = ns[:, None, img > 0] * wall_u.T[None, :, img > 0]
    fluid_src = (img == 0).astype(float)
    # smoothed densities and contact values
    nbar = np.zeros((M, N))
    for c in range(M):
        R = sig[c] / 2
        nbar[c] = ((R2 <= R * R) * ns[c][None, :]).sum(1) / _ball_count(R)
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
            G = 0.5 * (g[a, b][:, None] + g[a, b][src][None, :]) * S
            shells[a, b] = (G, kap)
            out["Nmf"][a] += -KT * sab ** 2 * what * n[a][None, :] * np.einsum("sr,srd->ds", G * ns[b][None, :], Eh)
            gam[a] += kap / 3 * (G * ns[b][None, :]).sum(1)
            X_ = n[a][:, None, None] * js[b].T[None, :, :] - ns[b][None, :, None] * j[a].T[:, None, :]
            proj = (Eh * X_).sum(-1)
            out["Dold"][a] += kap * np.einsum("sr,srd->ds", G * proj, Eh)
            if eps[a, b] != 0:
                # the attractive field sees the fluid only (no images)
                T = (R2 > sab ** 2) & (R2 <= (m.rc_factor * sab) ** 2) & (fluid_src[None, :] > 0)
                with np.errstate(divide="ignore"):
                    Up = np.where(T, 6 * eps[a, b] * sab ** 6 / np.where(R2 > 0, R2, 1) ** 3.5, 0.0)
                out["Ntail"][a] += n[a][None, :] * np.einsum("sr,srd->ds", Up * ns[b][None, :], Eh)
    fx = m.fext_matrix()
    Next = n[:, None, :] * fx[:, :, None]
    Nc = out["Nmf"] + out["Ntail"] + Next
    hg = 0.5 * gam
    with np.errstate(invalid="ignore", divide="ignore"):
        V = np.where(n[:, None, :] > 0, (j + Nc + out["Dold"] + hg[:, None, :] * j)
                     / (n[:, None, :] * (1 + hg[:, None, :])), 0.0)
    H = Nc + 0.5 * out["Dold"]
    Dnew = np.zeros((M, 3, N))
    Vs = V[:, :, src].copy()
    Vs[:, :, img > 0] = wall_u.T[None, :, img > 0]
    for a in range(M):
        for b in range(M):
            G, kap = shells[a, b]
            Y_ = Vs[b].T[None, :, :] - V[a].T[:, None, :]
            proj = (Eh * Y_).sum(-1)
            Dnew[a] += kap * n[a][None, :] * np.einsum("sr,srd->ds", G * ns[b][None, :] * proj, Eh)
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


def test_bruteforce_walls_with_tail(oracle_lib):
    eps = np.array([[0.1, 0.07], [0.07, 0.05]])
    m = W.Mixture(10, 10, 10, sigma=(2.0, 2.5), eps=eps, rc_factor=1.6, walls_y=True, wall_ux=(0.02, -0.05))
    n0, u0 = W.random_state(m, [0.014, 0.009], rel=0.4, u_amp=0.03, seed=15)
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
