"""Pin of the oracle's attractive molecular field against an FFT convolution.

The RPA field below eq. (potmeanforce) is the convolution
  G_ab(r) = - int dr' n_b(r') grad U_ab(r - r'),  U_ab = -eps (sigma_ab/r)^6, r > sigma_ab,
cut at rc sigma_ab; on the lattice it is a circular convolution, which an
FFT computes independently of the oracle's ordered direct sum.
"""
import numpy as np
import pytest

import workloads as W


def _kernel(m, a, b):
    """K[d] on the periodic grid: value at offset e of 6 eps s^6/|e|^7 e_hat_d."""
    sab = 0.5 * (m.sigma[a] + m.sigma[b])
    eps = m.eps_matrix()[a, b]
    K = np.zeros((3,) + m.shape())
    ax = [np.fft.fftfreq(L, 1.0 / L).astype(int) for L in (m.nz, m.ny, m.nx)]
    Z, Y, X = np.meshgrid(*ax, indexing="ij")
    R2 = X ** 2 + Y ** 2 + Z ** 2
    T = (R2 > sab ** 2) & (R2 <= (m.rc_factor * sab) ** 2)
    r = np.sqrt(np.where(R2 > 0, R2, 1))
    mag = np.where(T, 6 * eps * sab ** 6 / r ** 7, 0.0)
    for d, comp in enumerate((X, Y, Z)):
        K[d] = mag * comp / r
    return K


def _tail_fft(m, n):
    out = np.zeros((m.M, 3) + m.shape())
    for a in range(m.M):
        for b in range(m.M):
            if m.eps_matrix()[a, b] == 0:
                continue
            K = _kernel(m, a, b)
            nb = np.fft.fftn(n[b])
            for d in range(3):
                # sum_e K(e) n(r + e) = correlation of n with K
                out[a, d] += n[a] * np.real(np.fft.ifftn(np.conj(np.fft.fftn(K[d])) * nb))
    return out


@pytest.mark.parametrize("shape", [(16, 16, 16), (24, 12, 14)])
def test_tail_matches_fft_convolution(oracle_lib, shape):
    eps = np.array([[0.15, 0.1], [0.1, 0.05]])
    m = W.Mixture(*shape, sigma=(1.5, 2.5), eps=eps, rc_factor=2.2)
    n0, u0 = W.random_state(m, [0.02, 0.01], rel=0.5, u_amp=0.0, seed=21)
    o = oracle_lib.Oracle(m)
    d = o.fields(o.init(n0, u0))
    ref = _tail_fft(m, d["n"])
    err = np.abs(d["Ntail"] - ref).max() / np.abs(ref).max()
    assert err < 1e-12, err


def test_tail_plane_wave_is_odd_and_in_quadrature(oracle_lib):
    # n_b = nbar + delta cos(k x): the field is -delta sin(k x) times a lattice
    # sum and has no cos component (the +-e pairs cancel it exactly)
    m = W.Mixture(20, 12, 12, sigma=(2.0,), eps=np.full((1, 1), 0.2), rc_factor=2.5)
    o = oracle_lib.Oracle(m)
    x = np.arange(20)
    k = 2 * np.pi / 20
    n0 = np.zeros((1,) + m.shape())
    n0[0] = (0.01 + 1e-4 * np.cos(k * x))[None, None, :]
    d = o.fields(o.init(n0, np.zeros((1, 3) + m.shape())))
    e, w = o.stencil("tail", 0, 0)
    lat = 2 * np.sum(w[:, 0] * np.sin(k * e[:, 0]))      # sum over +-e of U' e_x sin(k e_x)
    expect = n0[0] * (-1e-4 * np.sin(k * x) * lat)[None, None, :]
    np.testing.assert_allclose(d["Ntail"][0, 0], expect, rtol=0, atol=1e-13 * np.abs(expect).max())
    assert np.abs(d["Ntail"][0, 1:]).max() < 1e-20


def test_fft_stepping_matches_direct_stepping(oracle_lib):
    """The long-run oracle mode (attractive field by FFT) tracks the ordered
    direct sum to float64 rounding over several steps."""
    m = W.Mixture(16, 14, 12, sigma=(1.5, 2.5), eps=np.array([[0.15, 0.1], [0.1, 0.05]]), rc_factor=2.2)
    n0, u0 = W.random_state(m, [0.02, 0.01], rel=0.5, u_amp=0.01, seed=31)
    o = oracle_lib.Oracle(m)
    f0 = o.init(n0, u0)
    fd = o.step(f0, 5)
    ff = o.step_fft(f0, 5)
    assert np.abs(fd - ff).max() / np.abs(fd).max() < 1e-12


@pytest.mark.parametrize("shape", [(16, 14, 12), (20, 11, 12)])
def test_walled_tail_matches_padded_fft(oracle_lib, shape):
    """With walls in y, points beyond the walls contribute nothing (solid
    layers and out-of-box points hold no density).  The same field is a
    circular convolution on y zero-padded past the tail's reach: the
    oracle's ordered direct sum (walls) against an FFT on the padded grid."""
    eps = np.array([[0.15, 0.1], [0.1, 0.05]])
    m = W.Mixture(*shape, sigma=(1.5, 2.5), eps=eps, rc_factor=2.2, walls_y=True, wall_ux=(0.0, 0.0))
    n0, u0 = W.random_state(m, [0.02, 0.01], rel=0.5, u_amp=0.0, seed=23)
    o = oracle_lib.Oracle(m)
    d = o.fields(o.init(n0, u0))
    n = d["n"]
    assert np.all(n[:, :, 0, :] == 0) and np.all(n[:, :, -1, :] == 0)
    reach = int(np.ceil(m.rc_factor * max(m.sigma)))
    nyp = m.ny + reach
    pm = W.Mixture(m.nx, nyp, m.nz, sigma=m.sigma, eps=eps, rc_factor=m.rc_factor)
    npad = np.zeros((m.M,) + pm.shape())
    npad[:, :, :m.ny, :] = n
    ref = _tail_fft(pm, npad)[:, :, :, :m.ny, :]
    fluid = slice(1, m.ny - 1)
    got = d["Ntail"][:, :, :, fluid, :]
    err = np.abs(got - ref[:, :, :, fluid, :]).max() / np.abs(ref).max()
    assert err < 1e-12, err
