"""FP64 parity of the HIP path with the oracle one Newton step at a time.

A whole solve is not the right unit of comparison: once ||D F|| sits at the
discretisation floor, the stop test (a change of the merit below 1e-10) and
AMIPN's early stop compare quantities that rounding decides, and the merit is so
flat there that iterates 1e-13 apart end 1e-3 apart after a few more steps
(test_oracle_floor.py shows it with the oracle against itself).  So both sides are
started from the same iterate with the same Jacobian index (the sketch's key)
and compared after the same piece of the method:

  * IPN (Alg. 1 steps 2-7): one outer step from every iterate of the oracle's own
    trajectory;
  * AMIPN (Alg. 2): one preconditioner's life, i.e. from every iterate where the
    oracle forms a fresh Jacobian and preconditioner, the outer steps up to and
    including the one that ends with Flag true (or the solve's end).

How closely the two can agree is set by what the method itself determines: a
step is the LSQR solution to tolerance eta, and when the full step is refused
the golden section picks alpha among points whose merits differ by a few ulps
near the floor.  The oracle measures that on itself: the same piece with
another sketch seed (an equally valid run of the method) gives the spread s of
the field and of ||D F||.

  * test_one_step_at_a_time (the solver's settings, eta = 1e-10; IPN steps and
    AMIPN preconditioner lives): the inner-step counts and Flags equal for every
    outer step before the oracle's merit reaches the floor (an outer step that
    moves it by less than tau_rel = 1e-3 relative, the change AMIPN's early stop
    treats as negligible: there whether a line search still finds a decrease is
    a rounding decision), the stall status equal for pieces that
    stay off the floor, and ||D F|| after the last outer step before the floor
    (the piece's end if it stays off it) within the merit bar: 4 s_phi, or
    1e-11 relative to ||D F|| where the piece began plus 1e-13 of ||D F|| at
    the solve's start (the rounding the terms of a small residual carry; they
    are as large as the residual at the start).  A piece wholly on the floor
    has both merits within tau_rel per outer step.  Field differences are
    printed.
  * test_steps_at_tight_tolerance (eta = 1e-14, every IPN step of the oracle's
    trajectory): the new field within max(1e-10, 2 s) of the oracle's
    (relative L2 on the test points).  When either side refused the full step,
    the GPU's field is compared with the oracle's direction taken with the
    GPU's alpha (the golden section's choice among merits equal to rounding is
    not the method's), and the two merits within the merit bar above.  With the LSQR
    truncation out of the way this is the arithmetic of the whole step --
    assembly, row scale, sketch, QR, LSQR, triangular solve, line search,
    update -- against the oracle's: the oracle's two seeds agree to ~1e-14 on
    the well-conditioned cases, so the bar there is 1e-10 flat; on the 2-D
    workload (kappa(D J) = 3e13) the first steps are determined only to ~6e-5.

The sketch is the FP64 Gaussian one (the same Philox stream on both sides).
"""
import sys

import numpy as np
import pytest

import rfm_workloads as W
from oracle import rfm as O

R = None


def setup_module(module):
    global R
    import paper_2510_04170_amd as Rm
    Rm.lib()
    R = Rm


def _announce(msg):
    sys.stdout.write(f"\n[gpu-test] {msg}\n")
    sys.stdout.flush()


CASES = {
    "poisson2d_full": lambda: W.config1(),
    "grayscott_small": lambda: W.config2(nsub=(2, 2, 2), J=40, q=4, test_per_dim=3),
    "helmholtz_cosh_small": lambda: W.helmholtz_cosh(nsub=(2, 2, 1), J=40, q=6, test_per_dim=3),
    "helmholtz_holes_small": lambda: W.config3(nsub=(2, 2, 2), J=40, q=6, test_per_dim=3),
    "allencahn_hole_small": lambda: W.config4(nsub=(2, 2, 2), J=50, q=5, n_t=16, n_theta=12, test_per_dim=3),
    "quasilinear_small": lambda: W.quasilinear(nsub=(2, 2, 1), J=40, q=6, test_per_dim=3),
    "poisson2d_smooth": lambda: W.config1(J=60, q=10, pou="b", test_per_dim=4),
    "grayscott_nonlinear_small": lambda: W.gray_scott_nonlinear(nsub=(2, 1, 1), J=40, q=5, test_per_dim=3),
    # the unit ball at J = 80, q = 8: a coarse discretisation (relL2 ~6e-2) whose merit is flat from the
    # second step on, so whole AMIPN solves of the two sides wander apart along the floor
    "ball_coarse": lambda: W.diffusion_reaction_ball(J=80, q=8, nbdy=600, test_per_dim=3),
    # more than 512 features per box: the register-free assembly and two sketch slabs
    "helmholtz_cosh_wide": lambda: W.helmholtz_cosh(nsub=(2, 1, 1), J=600, q=10, test_per_dim=3),
    # one dimension (single-point faces and interfaces) and one box (no continuity rows)
    "line_1d": lambda: W.line_1d(nsub=(4,), J=16, q=40, R=4.0, test_per_dim=20),
    "grayscott_one_box": lambda: W.config2(nsub=(1, 1, 1), J=40, q=5, test_per_dim=3),
}

GAMMA, ETA, M_MAX = 2.0, 1e-10, 3
# an outer step that changes ||D F|| by less than this (relative) is at the floor: AMIPN's early-stop
# threshold tau_rel, the change the method itself treats as negligible
TAU_FLOOR = 1e-3


def _field(prob, u):
    return O.eval_field(prob, u, prob.test_x, prob.test_owner)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _outer_merits(sg):
    """||D F|| after each outer step of a GPU solve (the merit after the step's last direction)."""
    out, k = [], 0
    for n_in in sg["inner_steps"]:
        k += n_in
        out.append(sg["resnorms"][min(k, len(sg["resnorms"])) - 1])
    return out


def _pieces(st, u0):
    """(start iterate, Jacobian index, first outer step, number of outer steps) of each preconditioner's life."""
    out, k, jac = [], 0, 0
    K = len(st.inner_steps)
    while k < K:
        e = k
        while e < K - 1 and not st.flags[e]:
            e += 1
        out.append((u0 if k == 0 else st.iterates[k - 1], jac, k, e - k + 1))
        jac += 1
        k = e + 1
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("method", ["ipn", "amipn"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_one_step_at_a_time(name, method):
    _announce(f"step parity {name} {method}")
    prob = CASES[name]()
    oo = O.Opts(method=method, gamma=GAMMA, lsqr_tol=ETA, m_max=M_MAX)
    u0 = np.zeros(prob.n)
    _, sto = O.solve(prob, u0, oo)
    phi_0 = float(np.linalg.norm(O.row_scale(O.assemble(prob, u0)[1]) * O.residual(prob, u0)))
    lp = R.from_description(prob)
    worst_phi, compared = 0.0, 0
    try:
        for (us, jac, k0, nout) in _pieces(sto, u0):
            # the oracle's piece is its trajectory's (a restart from us with Jacobian index jac repeats it)
            k1 = k0 + nout
            uo, phi_o = sto.iterates[k1 - 1], sto.resnorms[k1 - 1]
            inner_o, flags_o = sto.inner_steps[k0:k1], sto.flags[k0:k1]
            stall_o = sto.status == "stall" and k1 == len(sto.inner_steps)
            # the same piece with another sketch seed: what the method itself determines
            ua, sa = O.solve(prob, us, O.Opts(method=method, gamma=GAMMA, lsqr_tol=ETA, m_max=M_MAX, seed=7,
                                              jac_index0=jac, max_outer=nout))
            og = R.default_opts(method=R.RFM_AMIPN if method == "amipn" else R.RFM_IPN, sketch_factor=GAMMA,
                                lsqr_tol=ETA, m_max=M_MAX, max_outer=nout, jac_index0=jac)
            ug, sg, rc = lp.solve(us, og)
            phi_start = float(np.linalg.norm(O.row_scale(O.assemble(prob, us)[1]) * O.residual(prob, us)))
            fo = _field(prob, uo)
            ef = _rel(_field(prob, ug), fo)
            spread = _rel(_field(prob, ua), fo)
            er = abs(sg["final_resnorm"] - phi_o) / phi_start
            spread_phi = abs(sa.resnorms[-1] - phi_o) / phi_start
            # outer steps before the oracle's merit reaches the floor
            merits = [phi_start] + list(sto.resnorms[k0:k1])
            fl = next((t for t in range(nout) if abs(merits[t + 1] - merits[t]) < TAU_FLOOR * merits[t]), nout)
            # the merit where the decisions stop being compared: after the last outer step before the floor
            # (the end of the piece if it never reaches it), and at the end of a piece wholly on the floor
            mg = _outer_merits(sg)
            if fl > 0:
                er = abs(mg[fl - 1] - merits[fl]) / phi_start
                if len(sa.resnorms) >= fl:
                    spread_phi = abs(sa.resnorms[fl - 1] - merits[fl]) / phi_start
                bar = max(1e-11 + 1e-13 * phi_0 / phi_start, 4 * spread_phi)
            else:
                bar = TAU_FLOOR * nout
            print(f"  {name} {method} outer steps {k0 + 1}..{k1} (Jacobian {jac}; floor from step "
                  f"{k0 + fl + 1 if fl < nout else '-'}): inner GPU {sg['inner_steps']} oracle {inner_o}, flags GPU "
                  f"{sg['flags']} oracle {flags_o}; alpha GPU {[round(a, 6) for a in sg['alphas']]}; ||DF|| {er:.1e} "
                  f"(bar {bar:.1e}, seed spread {spread_phi:.1e}) of {phi_start:.3e}; field {ef:.2e} (seed spread "
                  f"{spread:.2e})")
            assert sg["inner_steps"][:fl] == inner_o[:fl]
            assert sg["flags"][:fl] == flags_o[:fl]
            if fl == nout:
                assert (rc == R.RFM_ESTALL) == stall_o
            assert er <= bar
            worst_phi, compared = max(worst_phi, er), compared + 1
    finally:
        lp.close()
    print(f"  {name} {method}: {compared} pieces, worst ||DF|| difference {worst_phi:.1e}")


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(CASES))
def test_steps_at_tight_tolerance(name):
    _announce(f"tight step parity {name}")
    prob = CASES[name]()
    eta = 1e-14
    u0 = np.zeros(prob.n)
    _, sto = O.ipn(prob, u0, O.Opts(gamma=GAMMA, lsqr_tol=eta))
    phi_0 = float(np.linalg.norm(O.row_scale(O.assemble(prob, u0)[1]) * O.residual(prob, u0)))
    lp = R.from_description(prob)
    worst = 0.0
    try:
        for k, a_o in enumerate(sto.alphas):
            us = u0 if k == 0 else sto.iterates[k - 1]
            if a_o == 0.0:
                continue  # a refused step: nothing moved
            uo = sto.iterates[k]
            ua, sa = O.ipn(prob, us, O.Opts(gamma=GAMMA, lsqr_tol=eta, max_outer=1, seed=7, jac_index0=k))
            ug, sg, rc = lp.solve(us, R.default_opts(sketch_factor=GAMMA, lsqr_tol=eta, max_outer=1,
                                                     jac_index0=k))
            a_g = sg["alphas"][0]
            fo = _field(prob, uo)
            spread = _rel(_field(prob, ua), fo)
            phi_start = float(np.linalg.norm(O.row_scale(O.assemble(prob, us)[1]) * O.residual(prob, us)))
            if a_o == 1.0 and a_g == 1.0:
                ef = _rel(_field(prob, ug), fo)
                what = "full step"
            else:
                # the oracle's direction with the GPU's step length
                uo_g = us + (a_g / a_o) * (uo - us)
                ef = _rel(_field(prob, ug), _field(prob, uo_g))
                what = f"alpha GPU {a_g:.8f} oracle {a_o:.8f}"
                er = abs(sg["final_resnorm"] - sto.resnorms[k]) / phi_start
                spread_phi = abs(sa.resnorms[-1] - sto.resnorms[k]) / phi_start
                assert er <= max(1e-11 + 1e-13 * phi_0 / phi_start + 1e-9, 4 * spread_phi)
            bar = max(1e-10, 2 * spread)
            print(f"  {name} step {k + 1} ({what}): LSQR GPU {sg['lsqr_iters']} oracle {sto.lsqr_iters[k]}; field "
                  f"{ef:.2e} (seed spread {spread:.1e}, bar {bar:.1e})")
            assert ef <= bar
            worst = max(worst, ef)
    finally:
        lp.close()
    print(f"  {name}: worst field difference {worst:.2e}")
