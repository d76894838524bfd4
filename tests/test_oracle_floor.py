"""What relative L2 error the stated discretisations can reach at all.

The error measure (relative L2 of the random-feature field against u* on the
cell-centred test set, one value per component) is minimised over every
coefficient vector by a linear least-squares fit: with the indicator
partition of unity the field on box e is Phi_{e,c} u_{e,c} with coefficients
of its own, so

    min_u ||u_n - u*||^2 = sum_e min_{u_e} ||Phi_{e,c} u_e - u*_e||^2

over the test points of each box, and any subset of boxes gives a lower bound.
No solver (exact Newton, IPN, AMIPN, any precision) can end below it.  The
workloads' target of relL2 <= 1e-6 is therefore out of reach for the features
the Gray-Scott (4x4x4 boxes, J = 300, weights in [-1.5, 1.5]), Helmholtz-with-
holes (8x8x8, J = 250) and space-time Allen-Cahn (4x4x8, J = 400) workloads
state, and within reach for the 2-D workload (2x2 boxes, J = 200).  The boxes
summed below are those with the largest fit residuals (any choice is a valid
bound; this one keeps the test short).

A second test shows where the collocation solve itself ends on one box of the
Gray-Scott workload's size and density (0.25^3, 10^3 points, J = 300 per
component): exact Newton (dense least squares at every step, Sec. 3's
Gauss-Newton definition) stops at relL2 ~1e-4, and 14^3 points do not lower it,
which is the floor the full-size solves reach (1.5e-4, 1.8e-4).
"""
import numpy as np
import pytest

import rfm_workloads as W
from oracle import rfm as O


def best_fit_bound(prob, boxes):
    """Lower bound of the relative L2 error (per component) over all coefficient vectors,
    from the least-squares fits of u* on the test points of the listed boxes."""
    ex = prob.exact(prob.test_x)
    num = np.zeros(prob.ncomp)
    for e in boxes:
        sel = prob.test_owner == e
        assert sel.any()
        for c in range(prob.ncomp):
            phi = O.feature_jet(prob, int(e), c, prob.test_x[sel])[0]
            coef = np.linalg.lstsq(phi, ex[sel, c], rcond=None)[0]
            r = phi @ coef - ex[sel, c]
            num[c] += r @ r
    return np.sqrt(num) / np.linalg.norm(ex, axis=0)


BOUND_CASES = {
    # workload: (generator, boxes summed, bound the sum must exceed per component)
    "gray_scott_4x4x4_J300": (W.config2, [0, 13, 17, 22, 26, 29, 33, 37, 42, 44, 45, 51, 55, 58], 5e-6),
    "allen_cahn_hole_4x4x8_J400": (W.config4, [1, 13, 17, 33, 66, 94, 110, 114], 1.2e-5),
    "helmholtz_holes_8x8x8_J250": (W.config3, [38, 52, 62, 66, 81, 109, 122, 123, 128, 133, 140, 146, 150, 154,
                                               165, 168, 172, 214, 224, 243, 245, 251, 266, 267, 272, 278, 285,
                                               296, 305, 309, 329, 335, 349, 358, 376, 380, 387, 394, 398, 419,
                                               430, 443, 456, 472, 481, 485, 496, 506], 1.3e-6),
}


@pytest.mark.parametrize("name", sorted(BOUND_CASES))
def test_target_error_is_below_what_the_features_can_represent(name):
    gen, boxes, lower = BOUND_CASES[name]
    prob = gen()
    b = best_fit_bound(prob, boxes)
    print(f"{name}: no coefficient vector reaches relL2 below {b}")
    assert np.all(b > lower) and np.all(b > 1e-6)


def test_two_dimensional_workload_can_reach_the_target():
    prob = W.config1()
    b = best_fit_bound(prob, range(4))
    assert np.all(b < 1e-9)
    # and the exact-Newton collocation solve gets there
    u, st = O.ipn(prob, opts=O.Opts(mode="exact"))
    assert st.status == "ok" and O.rel_l2(prob, u)[0] < 1e-6


@pytest.mark.parametrize("lo,q", [((0.0, 0.0, 0.0), 10), ((0.25, 0.25, 0.25), 10), ((0.25, 0.25, 0.25), 14)])
def test_gray_scott_collocation_floor_on_one_box(lo, q):
    lin, poly = W.gray_scott_terms()
    lo = np.asarray(lo)
    prob = W._build("gray_scott_one_box", 3, 2, lo, lo + 0.25, (1, 1, 1), 300, 1.5, q, q,
                    lambda x: W.jet_config2(x, 0.5), lin, poly, seed=0, test_per_dim=16)
    u, st = O.ipn(prob, opts=O.Opts(mode="exact"))
    e = O.rel_l2(prob, u)
    print(f"one box at {lo}, q = {q}: exact Newton IT {st.outer_iters}, relL2 {e}")
    assert st.status == "ok"
    assert np.all(e > 5e-5) and np.all(e < 2e-3)


def test_floor_trajectories_are_rounding_sensitive():
    """The oracle against itself on the coarse unit-ball case: AMIPN restarted from its second iterate and
    from the same iterate perturbed by 1e-13 (relative, entrywise) takes a different number of steps and
    ends 1e-3 apart -- the merit is flat at the floor (||D F|| unchanged to 7 digits from the second step
    on).  Whole-solve trajectories are therefore compared only loosely; the parity bar is per step."""
    prob = W.diffusion_reaction_ball(J=80, q=8, nbdy=600, test_per_dim=3)
    oo = O.Opts(method="amipn", gamma=2.0, lsqr_tol=1e-10, m_max=3)
    u, st = O.amipn(prob, opts=oo)
    assert st.status == "ok"
    r = np.array(st.resnorms[1:])
    assert np.all(np.abs(r - r[0]) < 1e-6 * r[0])
    k = 1
    jac = 1 + sum(st.flags[:k + 1])
    u1 = st.iterates[k]
    up = u1 * (1 + 1e-13 * np.random.default_rng(5).normal(size=u1.size))
    o2 = O.Opts(method="amipn", gamma=2.0, lsqr_tol=1e-10, m_max=3, jac_index0=jac)
    ua, sa = O.amipn(prob, up, o2)
    ub, sb = O.amipn(prob, u1, o2)
    fa = O.eval_field(prob, ua, prob.test_x, prob.test_owner)
    fb = O.eval_field(prob, ub, prob.test_x, prob.test_owner)
    d = np.linalg.norm(fa - fb) / np.linalg.norm(fb)
    print(f"restart from iterate {k + 1}: IT {sa.outer_iters} vs {sb.outer_iters}, fields {d:.2e} apart")
    assert d > 1e-5
