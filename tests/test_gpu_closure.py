"""GPU parity of the learned force closure.

The network (BF16 weights and activations, float32 accumulation on the
matrix cores) against its float64 oracle (oracle/cnn.py), and the closure
step (moments -> network -> collision + streaming, with exact-force checks
and fallback) against the lattice oracle.

Tolerances follow from the arithmetic.  bfloat16 keeps 8 significant bits,
so one rounding moves a value by at most u = 2^-9 (relative).  The forward
pass rounds the inputs, the weights of the four layers and the three
hidden activations once each (eight roundings, k / sqrt(2) u each way of
counting: 4 sqrt(2) u = 1.1e-2; 5 sqrt(2) u is asserted).  With the inputs
and all weights pre-rounded on the oracle side only the three activation
roundings remain: 3 u = 5.9e-3.  The backward pass adds one rounding of
the gradient per layer (four more, 6 sqrt(2) u = 1.7e-2), hence 2.5e-2 per
gradient tensor.  Adam runs in float32 on float32 master weights:
agreement to a few float32 ulps of the weight plus a few ulps of the step.
"""
import numpy as np
import pytest

import workloads as W
from oracle import cnn

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -9
CIN = cnn.CHANNELS[0]


def bf16(a):
    """Round float values to bfloat16 (nearest even), returned as float64."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def mlb():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_3634_amd as m
    return m


def random_layers(seed, scale_b=0.1):
    rng = np.random.default_rng(seed + 100)
    layers = cnn.init_params(seed=seed)
    for L in layers:
        L["b"] = rng.normal(scale=scale_b, size=L["b"].shape)
    return layers


# (70, 30, 60): 288 tiles of 16 x 8 x 4, more than one per CU, ragged in
# every direction: the persistent blocks walk XCD-contiguous tile ranges
@pytest.mark.parametrize("shape", [(9, 10, 12), (4, 4, 4), (3, 5, 17), (70, 30, 60)])
def test_forward_matches_oracle(mlb, shape):
    print(f"forward parity shape={shape}", flush=True)
    layers = random_layers(7)
    rng = np.random.default_rng(3)
    x = rng.normal(scale=0.7, size=(CIN,) + shape)
    net = mlb.GpuNet(shape)
    net.set_params(layers)
    y = net.forward(x).cpu().numpy().astype(np.float64)
    y_ref, _ = cnn.forward(layers, x)
    assert rel_l2(y, y_ref) < 5 * np.sqrt(2) * U_BF16
    # with the inputs and all weights rounded as the device rounds them
    rounded = [{"W": bf16(L["W"]), "b": np.float32(L["b"]).astype(np.float64)} for L in layers]
    y_r, _ = cnn.forward(rounded, bf16(x))
    assert rel_l2(y, y_r) < 3 * U_BF16
    assert np.max(np.abs(y - y_r)) < 8 * U_BF16 * np.max(np.abs(y_r))


def test_parameter_roundtrip_and_zero_network(mlb):
    shape = (4, 5, 6)
    net = mlb.GpuNet(shape)
    layers = random_layers(11)
    flat = mlb.net_flatten(layers)
    net.set_params(flat)
    back = net.get_params(flat=True)
    np.testing.assert_array_equal(back, flat)
    zero = np.zeros_like(flat)
    net.set_params(zero)
    y = net.forward(np.random.default_rng(0).normal(size=(CIN,) + shape)).cpu().numpy()
    assert np.all(y == 0.0)


def test_gradients_match_oracle(mlb):
    shape = (8, 9, 10)      # 720 sites: three 256-site blocks, the last ragged
    print("gradient parity", flush=True)
    layers = random_layers(5)
    rng = np.random.default_rng(9)
    x = rng.normal(scale=0.7, size=(CIN,) + shape)
    t = rng.normal(scale=0.5, size=(6,) + shape)
    net = mlb.GpuNet(shape, training=True)
    net.set_params(layers)
    loss, grads = net.train_step(x, t, update=False, want_grads=True)
    y_ref, caches = cnn.forward(layers, x)
    loss_ref, gy = cnn.mse(y_ref, t)
    g_ref, _ = cnn.backward(layers, caches, gy)
    assert abs(loss / loss_ref - 1.0) < 4 * np.sqrt(2) * U_BF16
    for l in range(4):
        for key in ("W", "b"):
            e = rel_l2(grads[l][key], g_ref[l][key])
            assert e < 2.5e-2, (l, key, e)
    assert net.adam_steps == 0
    np.testing.assert_array_equal(net.get_params(flat=True), mlb.net_flatten(layers))


def test_adam_two_steps_match_oracle(mlb):
    shape = (6, 6, 7)
    layers = random_layers(2)
    rng = np.random.default_rng(4)
    x = rng.normal(scale=0.7, size=(CIN,) + shape)
    t = rng.normal(scale=0.5, size=(6,) + shape)
    net = mlb.GpuNet(shape, training=True)
    net.set_params(layers)
    p = mlb.net_flatten(layers).astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    lr = 2e-3
    for step in (1, 2):
        _, g = net.train_step(x, t, lr=lr, want_grads=True)
        cnn.adam_step(p, mlb.net_flatten(g).astype(np.float64), m, v, step, lr=lr)
        got = net.get_params(flat=True).astype(np.float64)
        np.testing.assert_allclose(got, p, rtol=4e-7, atol=4e-7 * lr * step)
        p = got.copy()      # continue from the device's float32 weights
    assert net.adam_steps == 2


def test_training_reduces_loss(mlb):
    """A few hundred Adam steps fit a fixed smooth target (the network can
    represent a linear 3x3x3 stencil exactly)."""
    shape = (8, 8, 8)
    rng = np.random.default_rng(1)
    x = rng.normal(scale=0.5, size=(CIN,) + shape)
    Wt = rng.normal(scale=0.1, size=(6, CIN, 3, 3, 3))
    t = cnn.conv3d(x, Wt, np.zeros(6))
    net = mlb.GpuNet(shape, training=True)
    net.set_params(cnn.init_params(seed=0))
    l0, _ = net.train_step(x, t, lr=2e-3)
    for _ in range(300):
        net.train_step(x, t, lr=2e-3, want_loss=False)
    l1, _ = net.train_step(x, t, lr=2e-3)
    assert l1 < 0.05 * l0, (l0, l1)


# ------------------------------------------------------------ closure step
def closure_case(nx=24, ny=12, nz=12):
    return W.config_closure_physics(nx, ny, nz)


def scales(n0):
    n_ref = float(np.mean(n0))
    return n_ref, 1e-3 * n_ref, 1e-4


def test_closure_sample_matches_oracle(mlb, oracle_lib):
    import oracle
    mix, n0, u0 = closure_case()
    o = oracle.Oracle(mix)
    f = o.step(o.init(n0, u0), 3)
    g = mlb.GpuMixture(mix, n0, u0, precision=32)
    g.step(3)
    net = mlb.GpuNet(mix.shape())
    n_ref, j_ref, f_ref = scales(n0)
    net.set_scales(n_ref, j_ref, f_ref)
    x, t = g.closure_sample(net)
    x, t = x.cpu().numpy(), t.cpu().numpy()
    d = o.fields(f)
    # inputs: densities, momenta, lattice pressure gradients c_s^2 (n(r + e_d) - n(r - e_d)) / 2
    # (central differences with periodic wrap, c_s^2 = 1/3) in force units
    grads = [(np.roll(d["n"][a], -1, axis=ax) - np.roll(d["n"][a], 1, axis=ax)) / 6.0 / f_ref
             for a in range(2) for ax in (2, 1, 0)]
    x_ref = np.concatenate([d["n"] / n_ref - 1.0, d["j"][0] / j_ref, d["j"][1] / j_ref, np.stack(grads)])
    t_ref = d["N"].reshape(6, *mix.shape()) / f_ref
    assert np.max(np.abs(x - x_ref)) < 1e-5 * max(1.0, np.max(np.abs(x_ref)))
    assert np.max(np.abs(t - t_ref)) < 1e-4 * np.max(np.abs(t_ref))
    # sampling does not advance or change the state
    assert g.steps == 3
    np.testing.assert_allclose(g.moments()[0].cpu().numpy(), d["n"], rtol=1e-5)


def test_closure_checks_every_step_follow_the_exact_path(mlb, oracle_lib):
    """check_every = 1: every step takes the exact force; the trajectory is
    the plain one (float32 bar) and no fallback happens with tol = inf."""
    import oracle
    mix, n0, u0 = closure_case()
    g = mlb.GpuMixture(mix, n0, u0, precision=32)
    net = mlb.GpuNet(mix.shape())
    net.set_params(random_layers(1))
    net.set_scales(*scales(n0))
    g.set_closure(net, check_every=1, tol=float("inf"))
    g.step(20)
    st = g.closure_stats()
    assert st["checks"] == 20 and st["active"] and st["fallback_step"] == -1 and st["last_err"] > 0
    assert st["net_steps"] == 0 and st["failed_checks"] == 0
    o = oracle.Oracle(mix)
    f = o.step(o.init(n0, u0), 20)
    n_ref = o.densities(f)
    n = g.moments()[0].cpu().numpy()
    assert np.max(np.abs(n - n_ref) / np.abs(n_ref)) < 1e-5


def test_closure_falls_back_when_error_is_large(mlb, oracle_lib):
    import oracle
    mix, n0, u0 = closure_case()
    g = mlb.GpuMixture(mix, n0, u0, precision=32)
    net = mlb.GpuNet(mix.shape())
    net.set_params(random_layers(3))          # untrained: far from the exact force
    net.set_scales(*scales(n0))
    g.set_closure(net, check_every=4, tol=1e-2)
    g.step(13)
    st = g.closure_stats()
    # checks at steps 0, 4, 8, 12 all fail: every step takes the exact force
    assert st["checks"] == 4 and st["failed_checks"] == 4 and st["net_steps"] == 0
    assert st["fallback_step"] == 0 and not st["active"] and st["last_err"] > 1e-2
    o = oracle.Oracle(mix)
    f = o.step(o.init(n0, u0), 13)
    n_ref = o.densities(f)
    n = g.moments()[0].cpu().numpy()
    assert np.max(np.abs(n - n_ref) / np.abs(n_ref)) < 1e-5


def test_closure_network_steps_between_checks(mlb):
    """A check that passes hands the steps up to the next check to the
    network; the next check decides again, and the counters agree with its
    outcome (untrained net: its step-0 error is about 1, below tol = 2)."""
    mix, n0, u0 = closure_case()
    g = mlb.GpuMixture(mix, n0, u0, precision=32)
    net = mlb.GpuNet(mix.shape())
    net.set_params(random_layers(3))
    net.set_scales(*scales(n0))
    g.set_closure(net, check_every=3, tol=2.0)
    g.step(1)
    st = g.closure_stats()
    assert st["checks"] == 1 and st["active"] and st["last_err"] < 2.0 and st["net_steps"] == 0
    g.step(3)                                   # network steps 1 and 2, then the check at step 3
    st = g.closure_stats()
    assert st["checks"] == 2 and st["net_steps"] == 2
    passed = st["last_err"] <= 2.0
    assert st["active"] == passed and st["failed_checks"] == (0 if passed else 1)
    assert st["fallback_step"] == (-1 if passed else 3)


def test_closure_non_finite_network_output_falls_back(mlb, oracle_lib):
    """A network whose output is not finite fails its check even with an
    infinite tolerance, and the run continues on the exact force."""
    import oracle
    mix, n0, u0 = closure_case()
    g = mlb.GpuMixture(mix, n0, u0, precision=32)
    net = mlb.GpuNet(mix.shape())
    layers = random_layers(4)
    layers[3]["b"][0] = np.inf
    net.set_params(layers)
    net.set_scales(*scales(n0))
    g.set_closure(net, check_every=3, tol=float("inf"))
    g.step(7)
    st = g.closure_stats()
    assert st["fallback_step"] == 0 and not st["active"] and not np.isfinite(st["last_err"])
    assert st["checks"] == 3 and st["failed_checks"] == 3 and st["net_steps"] == 0
    o = oracle.Oracle(mix)
    n_ref = o.densities(o.step(o.init(n0, u0), 7))
    n = g.moments()[0].cpu().numpy()
    assert np.max(np.abs(n - n_ref) / np.abs(n_ref)) < 1e-5


C19 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
                [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])


def test_closure_step_is_collision_with_network_force(mlb, oracle_lib):
    """A step between checks: populations after it equal the oracle's
    collision (eq. evolution) with the network's force at every site,
    followed by streaming, from the same pre-step populations."""
    import oracle
    mix, n0, u0 = closure_case(16, 10, 10)
    g = mlb.GpuMixture(mix, n0, u0, precision=32)
    net = mlb.GpuNet(mix.shape())
    net.set_params(random_layers(8, scale_b=0.02))
    n_ref, j_ref, f_ref = scales(n0)
    net.set_scales(n_ref, j_ref, f_ref)
    g.set_closure(net, check_every=1000, tol=float("inf"))
    g.step(1)                                   # step 0 is a check step (exact force)
    f1 = g.populations().cpu().numpy().astype(np.float64)
    x, _ = g.closure_sample(net)
    Nnet = net.forward(x).cpu().numpy().astype(np.float64) * f_ref
    g.step(1)
    f2 = g.populations().cpu().numpy().astype(np.float64)
    st = g.closure_stats()
    assert st["checks"] == 1 and st["active"]
    o = oracle.Oracle(mix)
    d = o.fields(f1)
    nz, ny, nx = mix.shape()
    M = mix.M
    Nnet = Nnet.reshape(M, 3, nz, ny, nx)
    post = np.empty_like(f1)
    for a in range(M):
        for z in range(nz):
            for y in range(ny):
                for xx in range(nx):
                    post[a, :, z, y, xx] = o.collide_site(f1[a, :, z, y, xx], d["n"][a, z, y, xx],
                                                          d["j"][a, :, z, y, xx], d["u"][:, z, y, xx],
                                                          Nnet[a, :, z, y, xx])
    exp = np.empty_like(post)
    for i in range(19):
        exp[:, i] = np.roll(post[:, i], shift=(C19[i, 2], C19[i, 1], C19[i, 0]), axis=(1, 2, 3))
    assert np.max(np.abs(f2 - exp)) < 2e-6 * np.max(np.abs(exp))


def test_closure_graph_replays_match_eager(mlb):
    """Closure steps replayed from the captured graph give the same
    populations as eager launches, across check steps, with eager work
    (samples, moments) between the calls."""
    mix, n0, u0 = closure_case(16, 10, 10)
    runs = []
    for graph in (False, True):
        g = mlb.GpuMixture(mix, n0, u0, precision=32)
        g.set_graph(graph)
        net = mlb.GpuNet(mix.shape())
        net.set_params(random_layers(8, scale_b=0.02))
        net.set_scales(*scales(n0))
        g.set_closure(net, check_every=5, tol=float("inf"))
        snaps = []
        for k in range(4):
            g.step(3)
            g.closure_sample(net)
            snaps.append(g.populations().cpu().numpy())
        runs.append((snaps, g.closure_stats()))
    for a, b in zip(runs[0][0], runs[1][0]):
        np.testing.assert_array_equal(a, b)
    assert runs[0][1] == runs[1][1] and runs[0][1]["checks"] == 3


def test_closure_graph_follows_rescaled_network(mlb):
    """The network's scales are baked into a captured inference graph as
    kernel arguments: after mlb_net_set_scales the replayed network steps must
    use the new scales, as eager steps do (attach, step, rescale, step)."""
    mix, n0, u0 = closure_case(16, 10, 10)
    n_ref, j_ref, f_ref = scales(n0)
    runs = []
    for graph in (False, True):
        g = mlb.GpuMixture(mix, n0, u0, precision=32)
        g.set_graph(graph)
        net = mlb.GpuNet(mix.shape())
        net.set_params(random_layers(8, scale_b=0.02))
        net.set_scales(n_ref, j_ref, f_ref)
        g.set_closure(net, check_every=100, tol=float("inf"))
        g.step(5)                                  # check at 0, then network steps (graph pairs)
        net.set_scales(n_ref, 2.0 * j_ref, 3.0 * f_ref)
        g.step(4)                                  # network steps only
        runs.append(g.populations().cpu().numpy())
    np.testing.assert_array_equal(runs[0], runs[1])


def test_pool_statistics_rescale_and_error(mlb):
    """The training-pool sums, the in-place rescaling and the relative error
    run in the library: against numpy on the same random pool."""
    import torch
    shape = (6, 7, 9)
    net = mlb.GpuNet(shape, training=True)
    N = int(np.prod(shape))
    rng = np.random.default_rng(5)
    S = 300                                           # more than one pass of the library's sample chunks
    x = rng.normal(size=(S, CIN) + shape).astype(np.float32)
    t = (rng.normal(size=(S, 6) + shape) * rng.uniform(0.1, 3.0, size=(S, 1, 1, 1, 1))).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    j_ms, t_ms = net.pool_stats(xd, td)
    x64, t64 = x.astype(np.float64), t.astype(np.float64)
    assert abs(j_ms / np.mean(x64[:, 2:8] ** 2) - 1) < 1e-12
    np.testing.assert_allclose(t_ms, (t64 ** 2).reshape(S, -1).mean(1), rtol=1e-12)
    net.pool_rescale(xd, td, 2.0, 4.0)
    xr, tr = xd.cpu().numpy(), td.cpu().numpy()
    np.testing.assert_array_equal(xr[:, :2], x[:, :2])
    np.testing.assert_allclose(xr[:, 2:8], x[:, 2:8] * np.float32(0.5), rtol=1e-7)
    np.testing.assert_allclose(xr[:, 8:], x[:, 8:] * np.float32(0.25), rtol=1e-7)
    np.testing.assert_allclose(tr, t * np.float32(0.25), rtol=1e-7)
    y = t[0] + rng.normal(scale=0.1, size=t[0].shape).astype(np.float32)
    err = net.rel_error(torch.from_numpy(y).cuda(), torch.from_numpy(t[0]).cuda())
    ref = np.linalg.norm(y.astype(np.float64) - t64[0]) / np.linalg.norm(t64[0])
    assert abs(err / ref - 1) < 1e-12
    assert N > 0


TRAIN_BOX = (192, 12, 12)


def _train_state(amp):
    nx, ny, nz = TRAIN_BOX
    n_tot = W.number_density(0.2, (0.5, 0.5), (2.0, 3.0))

    def make():
        m = W.Mixture(nx, ny, nz, sigma=(2.0, 3.0), tau=1.0, name="closure_train")
        n0, u0 = W.mode_state(m, n_tot, 0.5, amp)
        return m, n0, u0
    return make


@pytest.fixture(scope="module")
def trained(mlb):
    """A network trained as the closure benchmark trains its candidates
    (snapshots of the plain solver every 25 steps over 5000 steps of
    composition modes with amplitudes 0.01 - 0.1 on a 192x12x12 box at the
    step-binary physics, 20 epochs), with network seed 3."""
    from paper_1105_3634_amd.closure_train import init_params, train_closure
    nx, ny, nz = TRAIN_BOX
    net = mlb.GpuNet((nz, ny, nx), training=True)
    net.set_params(init_params(3))
    amps = (0.05, 0.1, 0.04, 0.01, 0.07, 0.03, 0.06, 0.02, 0.08)
    rep = train_closure(net, [_train_state(a) for a in amps], per_state=200, sample_every=25, epochs=20, lr=1e-3,
                        seed=3)
    return net, rep


def test_trained_network_passes_a_check_the_zero_network_fails(mlb, trained):
    """What the trained network gains: it passes the exact-force check on a
    held-out state (amplitude 0.045, after 300 steps) at tolerance 0.2, where
    the network with all parameters zero (a force of zero) fails with error 1."""
    from paper_1105_3634_amd.closure_train import closure_error
    net, rep = trained
    nx, ny, nz = TRAIN_BOX
    m, n0, u0 = _train_state(0.045)()
    g = mlb.GpuMixture(m, n0, u0, precision=32)
    g.step(300)
    err_trained = closure_error(net, g)
    zero = mlb.GpuNet((nz, ny, nx))
    zero.set_scales(*rep.scales)
    err_zero = closure_error(zero, g)
    print(f"  held-out check error: trained {err_trained:.4f}, zero network {err_zero:.4f}", flush=True)
    assert err_zero == pytest.approx(1.0, abs=1e-12)
    assert err_trained < 0.2
    for nt, passes in ((net, True), (zero, False)):
        g2 = mlb.GpuMixture(m, n0, u0, precision=32)
        g2.step(300)
        g2.set_closure(nt, check_every=300, tol=0.2)
        g2.step(1)                                   # checks fall on multiples of check_every: step 300
        st = g2.closure_stats()
        assert st["checks"] == 1 and st["active"] == passes, (st, err_trained)


def test_trained_network_carries_steps_within_the_d12_bar(mlb, trained):
    """The stated accuracy: a checked run (checks every 50 steps, tolerance
    0.1) of 5000 steps on the held-out state puts at least 15 % of the steps
    on the trained network with the fitted D_12 within 2 % of the plain
    run's; the zero network carries none (its runs take the exact force
    throughout)."""
    net, rep = trained

    def run(nt):
        m, n0, u0 = _train_state(0.045)()
        g = mlb.GpuMixture(m, n0, u0, precision=32)
        if nt is not None:
            g.set_closure(nt, check_every=50, tol=0.1)
        for k in range(0, 5001, 10):
            g.record_mode(0, 1)
            if k < 5000:
                g.step(10)
        return g.fit(0, t_min=200), (g.closure_stats()["net_steps"] if nt is not None else 0)

    d_plain, _ = run(None)
    d_net, steps = run(net)
    nx, ny, nz = TRAIN_BOX
    zero = mlb.GpuNet((nz, ny, nx))
    zero.set_scales(*rep.scales)
    d_zero, steps_zero = run(zero)
    print(f"  D_12 plain {d_plain:.5f}, closure {d_net:.5f} ({steps} network steps), zero network "
          f"{d_zero:.5f} ({steps_zero})", flush=True)
    assert steps >= 750 and abs(d_net / d_plain - 1.0) <= 0.02
    assert steps_zero == 0 and d_zero == pytest.approx(d_plain, rel=1e-4)
