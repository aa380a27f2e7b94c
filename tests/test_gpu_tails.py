"""GPU run of the tail-dependence study (Sec. 4.1, eq. berthelot, the D(c)
behaviour the paper shows in its figure of D against concentration): twenty
equal-diameter binaries (sigma 2 and 4, packing 0.3, c = 0.1 .. 0.9, with and
without Lorentz-Berthelot tails w_AA = -5 kT, w_BB = w_AA / 2) advanced as
one float32 batch; each fitted D against the linearised scheme's, and the
tail reduction's shape: below 1, deepest at c = 1/2, shallower at the larger
diameter."""
import numpy as np
import pytest

import workloads as W
from linear_scheme import LinearScheme

pytestmark = pytest.mark.gpu

X1 = (0.1, 0.3, 0.5, 0.7, 0.9)


def study():
    systems = []
    for sigma in (2.0, 4.0):
        for tails in (False, True):
            for x1 in X1:
                systems.append((sigma, tails, x1) + W.config_tail_study(sigma, 0.3, x1, tails=tails))
    return systems


def test_tail_study_batch():
    import paper_1105_3634_amd as mlb
    sys_ = study()
    mixes = [s[3] for s in sys_]
    print(f"[tail study] {len(mixes)} systems, float32 batch", flush=True)
    b = mlb.GpuBatch(mixes, [s[4] for s in sys_], [s[5] for s in sys_], precision=32)
    for t in range(0, 2001, 10):
        b.record_modes()
        if t < 2000:
            b.step(10)
    fits = b.fit_ex(t_min=200)
    D = {}
    for (sigma, tails, x1, m, n0, _), q in zip(sys_, fits):
        nn = np.array([n0[0].mean(), n0[1].mean()])
        lin = LinearScheme((sigma, sigma), nn, eps=m.eps_matrix() if tails else None)
        dl = lin.diffusion(m.nx)
        print(f"  sigma {sigma} tails {tails} c {x1}: D {q[0]:.6f} linear {dl:.6f} r2 {q[3]:.6f}", flush=True)
        assert q[4] == 1.0
        assert abs(q[0] / dl - 1) < 3e-3
        D[(sigma, tails, x1)] = (q[0], dl)
    for sigma in (2.0, 4.0):
        r = np.array([D[(sigma, True, c)][0] / D[(sigma, False, c)][0] for c in X1])
        rl = np.array([D[(sigma, True, c)][1] / D[(sigma, False, c)][1] for c in X1])
        print(f"  sigma {sigma}: ratio {np.round(r, 5)} linear {np.round(rl, 5)}", flush=True)
        assert np.all(np.abs(r - rl) < 1e-3)
        if sigma == 2.0:
            assert np.all(r < 1) and np.argmin(r) == 2
            r2 = r
    assert (1 - r[2]) < 0.5 * (1 - r2[2])
