"""Pins of the oracle's field gradient (the H1 error of the experiments' tables) by
central differences of the field itself, at random points, with both partitions
of unity (with the smooth one, points near box faces where several bumps
overlap)."""
import numpy as np
import pytest

import rfm_workloads as W
from oracle import rfm as O


def _random_points(prob, npts, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(prob.lo, prob.hi, size=(npts, prob.dim))
    return x, W.box_of(x, prob.lo, prob.hi, prob.nsub).astype(np.int32)


@pytest.mark.parametrize("name,make", [
    ("2d", lambda: W.config1(nsub=(2, 2), J=30, q=6, test_per_dim=3)),
    ("gray_scott", lambda: W.config2(nsub=(2, 1, 1), J=20, q=4, test_per_dim=2)),
    ("space_time", lambda: W.config4_nohole(nsub=(1, 2, 2), J=20, q=4, test_per_dim=2)),
    ("2d_smooth", lambda: W.config1(nsub=(3, 2), J=30, q=8, pou="b", test_per_dim=3)),
    ("3d_smooth", lambda: W.quasilinear(nsub=(2, 2, 1), J=20, q=5, pou="b", test_per_dim=2)),
])
def test_gradient_matches_central_differences(name, make):
    prob = make()
    u = np.random.default_rng(1).normal(size=prob.n)
    x, ow = _random_points(prob, 200, 3)
    g = O.eval_grad(prob, u, x, ow)
    assert g.shape == (200, prob.ncomp, prob.dim)
    h = 1e-6
    for a in range(prob.dim):
        e = np.zeros(prob.dim)
        e[a] = h
        fd = (O.eval_field(prob, u, x + e, ow) - O.eval_field(prob, u, x - e, ow)) / (2 * h)
        assert np.abs(g[:, :, a] - fd).max() < 1e-7 * np.abs(g).max()


def test_h1_error_of_the_manufactured_solution_fit():
    """The exact-Newton solution of the 2-D workload: its H1 error is small and larger than its L2 error
    (derivatives are harder to represent), and a coefficient vector of zeros has relative H1 error 1."""
    prob = W.config1(nsub=(2, 2), J=120, q=16)
    u, st = O.ipn(prob, opts=O.Opts(mode="exact"))
    e1, e0 = O.rel_h1(prob, u), O.rel_l2(prob, u)
    assert np.all(e1 < 1e-3) and np.all(e1 > e0)
    assert np.allclose(O.rel_h1(prob, np.zeros(prob.n)), 1.0)
