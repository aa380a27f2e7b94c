"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Float64: bit-for-bit equality of every intermediate field and of the
populations after many steps (both sides evaluate the same operations in
the same order, without contraction).
Float32: densities within 1e-5 of the oracle (relative to the field's max
norm) after 100 steps; the float64 error of each case is printed.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("n", "j", "u", "g", "vhat", "H", "N")


def _gpu(m, n0, u0, precision, **kw):
    import paper_1105_3634_amd as mlb
    return mlb.GpuMixture(m, n0, u0, precision=precision, **kw)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _case(name):
    if name == "step_binary":
        return W.config_step_binary()
    if name == "random_binary":
        m = W.Mixture(8, 8, 8, sigma=(2.0, 3.0))
        return (m,) + W.random_state(m, [0.012, 0.009], rel=0.4, u_amp=0.03, seed=11)
    if name == "ternary_tail_ext":
        eps = np.array([[0.1, 0.12, 0.08], [0.12, 0.15, 0.05], [0.08, 0.05, 0.2]])
        fx = np.array([[1e-5, 0, 0], [0, -2e-5, 0], [0, 0, 3e-5]])
        m = W.Mixture(12, 12, 12, sigma=(1.5, 2.0, 2.5), eps=eps, rc_factor=2.0, fext=fx)
        return (m,) + W.random_state(m, [0.03, 0.015, 0.008], rel=0.4, u_amp=0.03, seed=12)
    if name == "walls":
        m = W.Mixture(10, 11, 9, sigma=(2.0, 3.0), walls_y=True, wall_ux=(-0.03, 0.04))
        return (m,) + W.random_state(m, [0.012, 0.009], rel=0.4, u_amp=0.03, seed=13)
    if name == "fe_tau":
        m = W.Mixture(9, 10, 11, sigma=(2.0, 2.5), tau=0.8, scheme=W.SCHEME_FE)
        return (m,) + W.random_state(m, [0.006, 0.004], rel=0.3, u_amp=0.02, seed=14)
    if name == "bulk_small":
        return W.config_bulk_diffusion(32, 24, 24, seed=5)
    if name == "couette_small":
        # the Taylor/Couette physics (ternary, tail 0.3 kT, moving walls) on 48x20x12
        return W.config_taylor_couette(48, 20, 12)
    if name == "single_species":
        # one component with an attractive tail: every mixture sum has one term
        m = W.Mixture(9, 10, 11, sigma=(2.5,), eps=np.array([[0.1]]), rc_factor=2.0)
        return (m,) + W.random_state(m, [0.02], rel=0.4, u_amp=0.03, seed=31)
    if name == "absent_species":
        # a binary whose second species has no particles anywhere
        eps = np.array([[0.1, 0.07], [0.07, 0.05]])
        m = W.Mixture(10, 11, 9, sigma=(2.5, 3.5), eps=eps, rc_factor=2.0)
        n0, u0 = W.random_state(m, [0.02, 0.01], rel=0.4, u_amp=0.03, seed=33)
        n0[1] = 0.0
        u0[1] = 0.0
        return m, n0, u0
    if name == "vacuum_slab":
        # three x planes with no fluid at all: zero total density there
        m = W.Mixture(12, 9, 10, sigma=(2.0, 3.0))
        n0, u0 = W.random_state(m, [0.012, 0.009], rel=0.4, u_amp=0.03, seed=32)
        n0[..., 4:7] = 0.0
        u0[..., 4:7] = 0.0
        return m, n0, u0
    if name == "quaternary_wide":
        # four species up to sigma = 5: shell reach 5, wrapped halos larger
        # than the box in y and z, seven distinct shells
        m = W.Mixture(14, 13, 12, sigma=(2.0, 3.0, 4.0, 5.0))
        return (m,) + W.random_state(m, [0.01, 0.005, 0.002, 0.001], rel=0.3, u_amp=0.02, seed=15)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["step_binary", "random_binary", "ternary_tail_ext", "walls", "fe_tau",
                                  "single_species", "absent_species"])
def test_fp64_fields_bit_exact(oracle_lib, name):
    m, n0, u0 = _case(name)
    print(f"[fp64 fields] case={name} shape={m.shape()} M={m.M}", flush=True)
    o = oracle_lib.Oracle(m)
    f = o.step(o.init(n0, u0), 3)
    ref = o.fields(f)
    g = _gpu(m, n0, u0, 64)
    g.step(3)
    d = g.fields()
    for k in FIELDS:
        got = _np(d[k])
        assert np.array_equal(got, ref[k]), (k, np.abs(got - ref[k]).max())


@pytest.mark.parametrize("name,steps", [("step_binary", 100), ("ternary_tail_ext", 20), ("walls", 40),
                                        ("fe_tau", 30), ("couette_small", 10), ("single_species", 50),
                                        ("absent_species", 30)])
def test_fp64_populations_bit_exact(oracle_lib, name, steps):
    m, n0, u0 = _case(name)
    print(f"[fp64 steps] case={name} shape={m.shape()} steps={steps}", flush=True)
    o = oracle_lib.Oracle(m)
    fo = o.step(o.init(n0, u0), steps)
    g = _gpu(m, n0, u0, 64)
    g.step(steps)
    fg = _np(g.populations())
    assert np.array_equal(fg, fo), np.abs(fg - fo).max()


def _rel_maxnorm(got, ref):
    """Largest per-species error relative to that species' max norm; a species
    with no particles must come out exactly zero (else the error is inf)."""
    out = []
    for a in range(ref.shape[0]):
        diff, scale = np.abs(got[a] - ref[a]).max(), np.abs(ref[a]).max()
        out.append(diff / scale if scale > 0 else (0.0 if diff == 0 else np.inf))
    assert not np.isnan(out).any(), out
    return max(out)


@pytest.mark.parametrize("name,steps", [("step_binary", 100), ("bulk_small", 100), ("walls", 100),
                                        ("fe_tau", 60), ("ternary_tail_ext", 50), ("quaternary_wide", 30),
                                        ("single_species", 100), ("absent_species", 60)])
def test_fp32_densities_within_1e5(oracle_lib, name, steps):
    m, n0, u0 = _case(name)
    print(f"[fp32 densities] case={name} shape={m.shape()} steps={steps}", flush=True)
    o = oracle_lib.Oracle(m)
    fo = o.step(o.init(n0, u0), steps)
    no = o.fields(fo)["n"]
    g32 = _gpu(m, n0, u0, 32)
    g32.step(steps)
    n32 = _np(g32.moments()[0])
    g64 = _gpu(m, n0, u0, 64)
    g64.step(steps)
    n64 = _np(g64.moments()[0])
    e32, e64 = _rel_maxnorm(n32, no), _rel_maxnorm(n64, no)
    print(f"  fp32 rel err {e32:.3e}   fp64 rel err {e64:.3e}", flush=True)
    assert e64 == 0.0
    assert e32 < 1e-5


@pytest.mark.parametrize("name,steps", [("step_binary", 100), ("walls", 100), ("fe_tau", 60),
                                        ("ternary_tail_ext", 50), ("quaternary_wide", 30),
                                        ("single_species", 100), ("absent_species", 60)])
def test_fp32_sign_grouped_gather_within_1e5(oracle_lib, name, steps):
    """The first gather's sign-grouped shell loop (MLB_OPT_GATHER1_SIGN_GROUPS):
    float32 densities against the oracle within 1e-5, and the force parts of
    one step within 2e-6, on the 16x4x4 and 8x8x4 tilings, the latter also
    with the first gather on its own 4x8x8 tiles."""
    import paper_1105_3634_amd as mlb
    m, n0, u0 = _case(name)
    o = oracle_lib.Oracle(m)
    f0 = o.init(n0, u0)
    no = o.fields(o.step(f0, steps))["n"]
    for shape, own in ((0, 0), (1, 0), (1, 1)):
        print(f"[fp32 sign groups] case={name} shape={shape} own={own} steps={steps}", flush=True)
        g = _gpu(m, n0, u0, 32, options=mlb.opt_tiling(shape, 1, 3, 1, own))
        assert g.tuning()["gather1_sign_groups"] == 1
        if name == "ternary_tail_ext":
            ref = o.fields(f0)
            got = _np(g.forces(mlb.PART_ALL))
            e = np.abs(got - ref["N"]).max() / np.abs(ref["N"]).max()
            print(f"  force rel err {e:.3e}", flush=True)
            assert e < 2e-6
        g.step(steps)
        e32 = _rel_maxnorm(_np(g.moments()[0]), no)
        print(f"  fp32 rel err {e32:.3e}", flush=True)
        assert e32 < 1e-5


def test_zero_density_sites(oracle_lib):
    """Sites with no fluid at all (total density zero): the mean velocity there
    is zero, the contact values are those of the empty fluid (1) while the
    smoothing ball holds no fluid, and the fields match the oracle, bit for bit in float64, before the first step and after
    one (the middle plane of the slab is still empty then).  A free vacuum
    interface is not a steady state of the lattice model: the rarefaction
    drives densities negative within a few steps, so only the first steps are
    compared."""
    m, n0, u0 = _case("vacuum_slab")
    o = oracle_lib.Oracle(m)
    f = o.init(n0, u0)
    for steps in (0, 1):
        print(f"[zero density] shape={m.shape()} steps={steps}", flush=True)
        ref = o.fields(f)
        assert not ref["n"][..., 5].any()
        g64 = _gpu(m, n0, u0, 64)
        g32 = _gpu(m, n0, u0, 32)
        g64.step(steps)
        g32.step(steps)
        d64, d32 = g64.fields(), g32.fields()
        for k in FIELDS:
            got = _np(d64[k])
            assert np.array_equal(got, ref[k]), (k, np.abs(got - ref[k]).max())
        for k in ("n", "u", "g", "N"):
            got = _np(d32[k])
            assert np.all(np.isfinite(got)), k
            err = np.abs(got - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-300)
            assert err < 1e-5, (k, err)
        assert not _np(d32["u"])[..., 5].any() and not _np(d64["u"])[..., 5].any()
        if steps == 0:
            # nothing within the smoothing ball of the middle plane yet
            assert np.all(ref["g"][..., 5] == 1.0) and np.all(_np(d32["g"])[..., 5] == 1.0)
        f = o.step(f, 1)


def test_absent_species_reduces_to_single_species():
    """A binary whose second species is empty everywhere evolves species 0
    exactly as the one-species system: float64 populations equal bit for bit
    after 30 steps, float32 densities within 1e-6."""
    import paper_1105_3634_amd as mlb
    m2, n0, u0 = _case("absent_species")
    m1 = W.Mixture(m2.nx, m2.ny, m2.nz, sigma=m2.sigma[:1], eps=m2.eps_matrix()[:1, :1], rc_factor=m2.rc_factor)
    for prec in (64, 32):
        print(f"[absent species] precision={prec}", flush=True)
        g2, g1 = _gpu(m2, n0, u0, prec), _gpu(m1, n0[:1], u0[:1], prec)
        g2.step(30)
        g1.step(30)
        f2, f1 = _np(g2.populations()), _np(g1.populations())
        assert not f2[1].any()
        if prec == 64:
            assert np.array_equal(f2[:1], f1)
        else:
            n2, n1 = _np(g2.moments()[0])[:1], _np(g1.moments()[0])
            err = np.abs(n2 - n1).max() / np.abs(n1).max()
            print(f"  fp32 rel diff {err:.3e}", flush=True)
            assert err < 1e-6


def _spread(n_tracer, nx):
    """Second moment along x, about the box centre, of the y,z-summed density."""
    prof = n_tracer.sum(axis=(0, 1))
    x = np.arange(nx) - 0.5 * nx
    mass = prof.sum()
    mean = (prof * x).sum() / mass
    return (prof * x * x).sum() / mass - mean * mean


def test_spread_record_and_fit_against_oracle(oracle_lib):
    """The tracer-band second moment of Sec. 5.2, recorded on the GPU in float64
    every 10 steps of the walled ternary (moving walls, tail), against the same
    moment of the oracle's densities computed here with numpy; the spread fit
    D = slope(Var, t) / 2 against numpy's least-squares line over the same
    samples (all, then t >= 30)."""
    m, n0, u0 = _case("couette_small")
    tracer, every, samples = m.M - 1, 10, 7
    o = oracle_lib.Oracle(m)
    f = o.init(n0, u0)
    ref = []
    for k in range(samples):
        ref.append(_spread(o.fields(f)["n"][tracer], m.nx))
        if k + 1 < samples:
            f = o.step(f, every)
    ref = np.array(ref)
    t_ref = every * np.arange(samples, dtype=np.float64)
    assert np.ptp(ref) > 1e-3 * ref[0]          # the band does spread
    for prec, tol in ((64, 1e-12), (32, 1e-5)):
        print(f"[spread] case=couette_small precision={prec}", flush=True)
        g = _gpu(m, n0, u0, prec)
        g.reset_series()
        for k in range(samples):
            g.record_spread(tracer)
            if k + 1 < samples:
                g.step(every)
        t, v = g.series()
        assert np.array_equal(t, t_ref)
        err = np.abs(v - ref).max() / np.abs(ref).max()
        print(f"  variance rel err {err:.2e}", flush=True)
        assert err < tol
        for t_min in (0.0, 30.0):
            sel = t >= t_min
            want = 0.5 * np.polyfit(t[sel], (ref if prec == 64 else v)[sel], 1)[0]
            got = g.fit(1, t_min)
            print(f"  t_min={t_min}: D {got:.10f} numpy {want:.10f}", flush=True)
            assert abs(got - want) <= 1e-9 * abs(want)


def test_mode_record_against_oracle(oracle_lib):
    """The composition-mode amplitude of Sec. 5.1, |sum_r (n_0 - n_1)
    exp(-i 2 pi x / nx)|, recorded on the GPU every 10 steps of the bulk
    binary, against numpy's projection of the oracle's densities; the mode
    fit D = -slope(ln A, t) / k^2 against numpy's line over the same
    amplitude window (t from the first sample at or below 0.1 A_first, or
    t_min if earlier, and A >= 1e-6 A_first)."""
    m, n0, u0 = _case("bulk_small")
    every, samples = 10, 7
    k = 2 * np.pi / m.nx
    x = np.arange(m.nx)
    o = oracle_lib.Oracle(m)
    f = o.init(n0, u0)
    ref = []
    for j in range(samples):
        n = o.fields(f)["n"]
        dn = (n[0] - n[1]).sum(axis=(0, 1))
        ref.append(np.hypot((dn * np.cos(k * x)).sum(), (dn * np.sin(k * x)).sum()))
        if j + 1 < samples:
            f = o.step(f, every)
    ref = np.array(ref)
    assert ref[-1] < 0.9 * ref[0]               # the mode decays
    for prec, tol in ((64, 1e-12), (32, 1e-5)):
        print(f"[mode] case=bulk_small precision={prec}", flush=True)
        g = _gpu(m, n0, u0, prec)
        g.reset_series()
        for j in range(samples):
            g.record_mode(0, 1)
            if j + 1 < samples:
                g.step(every)
        t, v = g.series()
        assert np.array_equal(t, every * np.arange(samples, dtype=np.float64))
        err = np.abs(v - ref).max() / ref[0]
        print(f"  amplitude rel err {err:.2e}", flush=True)
        assert err < tol
        for t_min in (0.0, 30.0):
            low = np.flatnonzero(v <= 0.1 * v[0])
            t_lo = min(t_min, t[low[0]]) if low.size else t_min
            sel = (t >= t_lo) & (v >= 1e-6 * v[0])
            want = -np.polyfit(t[sel], np.log((ref if prec == 64 else v)[sel]), 1)[0] / k ** 2
            got = g.fit(0, t_min)
            print(f"  t_min={t_min}: D {got:.10f} numpy {want:.10f}", flush=True)
            assert abs(got - want) <= 1e-9 * abs(want)


def test_fp32_forces_parts(oracle_lib):
    import paper_1105_3634_amd as mlb
    m, n0, u0 = _case("ternary_tail_ext")
    o = oracle_lib.Oracle(m)
    f = o.init(n0, u0)
    ref = o.fields(f)
    for prec, tol in ((64, 0.0), (32, 2e-6)):
        g = _gpu(m, n0, u0, prec)
        for mask, parts in ((mlb.PART_MF, ["Nmf"]), (mlb.PART_TAIL, ["Ntail"]), (mlb.PART_EXT, ["Next"]),
                            (mlb.PART_DISS, ["Dold", "Dnew"]), (mlb.PART_ALL, None)):
            got = _np(g.forces(mask))
            if parts is None:
                want = ref["N"]
            elif parts == ["Dold", "Dnew"]:
                want = 0.5 * ref["Dold"] + 0.5 * ref["Dnew"]
            else:
                want = ref[parts[0]]
            err = np.abs(got - want).max() / max(np.abs(want).max(), 1e-300)
            assert err <= max(tol, 1e-15 if prec == 64 else tol), (prec, mask, err)


def test_conserved_sums_fp64(oracle_lib):
    """Float64 GPU sums of the conserved quantities.  In float64 mass and total
    momentum hold to rounding; in float32 the collision and the pair forces
    cancel only to float32 rounding, so the drift is bounded by
    eps32 * total mass * steps."""
    m, n0, u0 = _case("random_binary")
    o = oracle_lib.Oracle(m)
    d = o.fields(o.init(n0, u0))
    steps = 50
    for prec in (64, 32):
        g = _gpu(m, n0, u0, prec)
        mass0, mom0 = g.conserved()
        g.step(steps)
        mass1, mom1 = g.conserved()
        drift = np.abs(mom1.sum(0) - mom0.sum(0)).max()
        print(f"  precision {prec}: mass drift {np.abs(mass1 / mass0 - 1).max():.2e}, momentum drift {drift:.2e}")
        if prec == 64:
            np.testing.assert_allclose(mass0, d["n"].sum(axis=(1, 2, 3)), rtol=1e-14)
            np.testing.assert_allclose(mass1, mass0, rtol=1e-13)
            assert drift < 1e-15 * m.N
        else:
            np.testing.assert_allclose(mass0, d["n"].sum(axis=(1, 2, 3)), rtol=1e-6)
            np.testing.assert_allclose(mass1, mass0, rtol=2e-6)
            assert drift < 6e-8 * mass0.sum() * steps


@pytest.mark.parametrize("shape,walls", [((16, 16, 16), False), ((24, 12, 14), False), ((15, 13, 17), False),
                                         ((40, 20, 24), False), ((20, 32, 32), False), ((24, 18, 14), True),
                                         ((16, 21, 12), True)])
def test_fp32_spectral_tail_matches_direct_sum(oracle_lib, shape, walls):
    """The MFMA DFT path of the attractive field against the oracle's float64
    direct sum (also checks the matrix-core lane layout: a wrong layout
    scrambles the field).  With walls the transform runs on y zero-padded past
    the tail's reach, so points beyond the walls contribute nothing, as in
    the direct sum."""
    import paper_1105_3634_amd as mlb
    eps = np.array([[0.15, 0.1], [0.1, 0.05]])
    kw = dict(walls_y=True, wall_ux=(-0.02, 0.03)) if walls else {}
    m = W.Mixture(*shape, sigma=(1.5, 2.5), eps=eps, rc_factor=2.2, **kw)
    n0, u0 = W.random_state(m, [0.02, 0.01], rel=0.5, u_amp=0.01, seed=21)
    print(f"[spectral tail] shape={m.shape()} walls={walls}", flush=True)
    o = oracle_lib.Oracle(m)
    ref = o.fields(o.init(n0, u0))
    for mode in (mlb.TAIL_SPECTRAL, mlb.TAIL_DIRECT):
        g = _gpu(m, n0, u0, 32, tail_mode=mode)
        got = _np(g.forces(mlb.PART_TAIL))
        err = np.abs(got - ref["Ntail"]).max() / np.abs(ref["Ntail"]).max()
        print(f"  mode {mode}: rel err {err:.2e}", flush=True)
        assert err < 2e-6, (mode, err)
        tot = _np(g.forces(mlb.PART_ALL))
        err = np.abs(tot - ref["N"]).max() / np.abs(ref["N"]).max()
        assert err < 1e-5, (mode, err)


@pytest.mark.parametrize("name", ["bulk_small", "couette_small"])
def test_fp32_spectral_100_steps(oracle_lib, name):
    import paper_1105_3634_amd as mlb
    m, n0, u0 = _case(name)
    o = oracle_lib.Oracle(m)
    no = o.fields(o.step(o.init(n0, u0), 100))["n"]
    for mode in (mlb.TAIL_SPECTRAL, mlb.TAIL_DIRECT):
        g = _gpu(m, n0, u0, 32, tail_mode=mode)
        g.step(100)
        e = _rel_maxnorm(_np(g.moments()[0]), no)
        print(f"  tail mode {mode}: fp32 density rel err {e:.3e}", flush=True)
        assert e < 1e-5


@pytest.mark.parametrize("name", ["walls", "bulk_small"])
def test_fp32_tilings_agree_bit_for_bit(name):
    """Every tile shape and block order (MLB_OPT_TILING), and the first
    gather on its own 4x8x8 tiles (MLB_OPT_GATHER1_OWN_TILES), sum each
    site's shell lists in the same order, so for one split of the first
    gather's shell lists over thread groups and one form of its shell loop
    the float32 states agree bit for bit; the two splits (2 and 3 groups,
    MLB_OPT_GATHER1_SPLIT) and the plain and sign-grouped loops
    (MLB_OPT_GATHER1_SIGN_GROUPS) add the same terms in different groupings
    and agree to float32 rounding."""
    import paper_1105_3634_amd as mlb
    m, n0, u0 = _case(name)
    refs = {}
    for groups in (0, 1):
        for split in (3, 2):
            for shape in range(3):
                for order in range(2):
                    for own in ((0, 1) if order == 1 else (0,)):
                        print(f"[tilings] case={name} groups={groups} split={split} shape={shape} order={order} "
                              f"own={own}", flush=True)
                        g = _gpu(m, n0, u0, 32, options=mlb.opt_tiling(shape, order, split, groups, own))
                        t = g.tuning()
                        assert (t["shape"], t["order"], t["gather1_split"], t["gather1_sign_groups"],
                                t["gather1_shape"]) == (shape, order, split, groups, 3 if own else shape)
                        g.step(6)
                        n, j = g.moments()
                        got = (_np(n), _np(j))
                        del g
                        key = (groups, split)
                        if key not in refs:
                            refs[key] = got
                            continue
                        ref = refs[key]
                        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), \
                            key + (shape, order, own)
    for a, b in (((0, 2), (0, 3)), ((1, 3), (0, 3)), ((1, 2), (0, 3))):
        e = _rel_maxnorm(refs[a][0], refs[b][0])
        print(f"  {a} vs {b}: density rel diff {e:.2e}", flush=True)
        assert e < 1e-6


def test_handles_of_different_reach_coexist():
    """A live float32 handle with large stencils (bulk diffusion physics,
    sigma 3 and 4.5, spectral tail) keeps stepping exactly as when alone
    after handles with smaller stencils and planes have been created: the
    kernels' LDS limits are never lowered below a live handle's launches."""
    import torch
    m, n0, u0 = _case("bulk_small")
    alone = _gpu(m, n0, u0, 32)
    alone.step(4)
    f_alone = alone.populations().clone()
    del alone
    big = _gpu(m, n0, u0, 32)
    big.step(2)
    ms, ns, us = _case("random_binary")
    small = _gpu(ms, ns, us, 32)
    mc, nc, uc = _case("couette_small")
    other_plane = _gpu(mc, nc, uc, 32)
    small.step(2)
    other_plane.step(2)
    big.step(2)
    torch.cuda.synchronize()
    assert torch.equal(big.populations(), f_alone)
