"""The bound behind the Verlet candidate lists (reading R33): if h is
L-Lipschitz and every particle has moved at most eps h (its h at the build)
since the build, eps = delta / (c L + 2), then a pair within c max(h_i, h_j)
now was within (c + delta) max(h_i, h_j) at the build, so filtering the
candidate lists gives the cut-off lists.  Checked on adversarial and random
configurations (the displacements point the pair together at full length and
h grows along them).  No GPU."""
import numpy as np
import pytest


def _h(x, h0, L, p):
    return h0 + L * np.linalg.norm(x - p, axis=-1)


@pytest.mark.parametrize("c", [2.0, 2.5])
@pytest.mark.parametrize("delta", [0.3, 0.5, 0.8])
@pytest.mark.parametrize("L", [0.0, 0.05, 0.2])
def test_a_pair_within_reach_now_was_a_candidate(c, delta, L):
    rng = np.random.default_rng(int(100 * c + 10 * delta + 1000 * L))
    eps = delta / (c * L + 2.0)
    n = 40_000
    p = np.zeros(3)
    xi = rng.uniform(-1.0, 1.0, (n, 3)) + np.array([3.0, 0.0, 0.0])
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    hi, h0 = _h(xi, 0.05, L, p), 0.05
    # j just outside the candidate reach at the build
    xj = xi.copy()
    for _ in range(100):   # fixed point |xi - xj| = (c + delta) max(h_i, h_j) (a contraction: L (c + delta) < 1)
        hj = _h(xj, h0, L, p)
        xj = xi + u * ((c + delta) * np.maximum(hi, hj) * (1.0 + 1e-9))[:, None]
    hj = _h(xj, h0, L, p)
    rb = np.linalg.norm(xi - xj, axis=1)
    Hb = np.maximum(hi, hj)
    assert np.all(rb >= (c + delta) * Hb)
    # the worst moves: both particles towards each other by eps h, plus random moves
    di = u * (eps * hi)[:, None]
    dj = -u * (eps * hj)[:, None]
    w = rng.normal(size=(n, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    for a, b in ((di, dj), (w * (eps * hi)[:, None], -w * (eps * hj)[:, None])):
        yi, yj = xi + a, xj + b
        r = np.linalg.norm(yi - yj, axis=1)
        H = np.maximum(_h(yi, h0, L, p), _h(yj, h0, L, p))
        # no such pair is within the cut-off now
        assert not np.any(r < c * H * (1.0 - 1e-9))
    # and a larger move does break it: the bound is tight enough to matter
    k = 1.5
    yi, yj = xi + k * di, xj + k * dj
    r = np.linalg.norm(yi - yj, axis=1)
    H = np.maximum(_h(yi, h0, L, p), _h(yj, h0, L, p))
    assert np.any(r < c * H)
