"""Pins of the oracle's AMIPN control (Alg. 2): inner steps per outer step, the
Flag decisions and the Jacobian evaluations, on problems whose trajectories are
known by hand.

1. F(u) = u^3 with one unknown, from u = 1.  Its Jacobian 3u^2 is exact, so an
   inner step with the Jacobian frozen at the point p is the chord step
   z <- z - z^3 / (3 p^2), and with p = 1 every iterate is z = c_i with
   c_0 = 1, c_{i+1} = c_i - c_i^3 / 3:  1, 2/3, 46/81 = 0.5679, 0.5068,
   0.4634, 0.4303, ...  The map is scale invariant (from z = t c_i with the
   Jacobian at t the iterates are t c_{i+1}, ...), so a fresh Jacobian restarts
   the same sequence scaled by the current iterate.  The row scale is
   100 / (3 p^2) and cancels in the early-stop test
   |F_{i+1} - F_i| < tau |F_0|, i.e. |c_{i+1}^3 - c_i^3| < tau c_{k,0}^3 with
   c_{k,0} the iterate where outer step k began; every full step lowers
   |F| by far more than the factor 1 - 1e-4, so the line search takes alpha = 1.

   * tau = 0.15, m_max = 3.  Outer 1 (Jacobian at 1): the changes of c^3 are
     0.704, 0.113 against 0.15 c_0^3 = 0.15: early stop after 2 steps at
     c_2 = 0.5679, Flag false, the Jacobian kept.  Outer 2 (c_{2}^3 = 0.1832,
     threshold 0.0275): changes 0.0530, 0.0307, 0.0199 -> early stop after 3
     steps (c_5 = 0.4303).  Outer 3 (threshold 0.0119): changes 0.0139, 0.0102
     -> 2 steps (c_7 = 0.3818).  Outer 4, 5 (thresholds 0.0083, 0.0072):
     changes 0.0077, 0.0061, one step each (c_8 = 0.3632, c_9 = 0.3473).  Inner steps [2, 3, 2, 1, 1], Flags all false, one
     Jacobian, u = c_9 = 0.34725791597677 after max_outer = 5.
   * tau = 0.1, m_max = 3.  Outer 1: changes 0.704, 0.113, 0.0530 -> early stop
     at the third step (0.0530 < 0.1), u = c_3 = 0.50685, Jacobian kept.
     Outer 2 (threshold 0.1 c_3^3 = 0.01302): changes 0.0307, 0.0199, 0.0139 ->
     m_max reached, Flag true, a fresh Jacobian at c_6 = 0.40372.  The
     sequence then repeats scaled by c_6: inner steps [3, 3, 3, 3, 3], Flags
     [F, T, F, T, F], three Jacobians (at 1, c_6, c_6^2), and
     u = c_6^2 c_3 = 0.082609328935247.

2. A scripted problem (positions 0, 1, 2, ... with scripted residuals and
   scripted line-search failures) for the rules when a line search finds no
   decrease: it ends the inner loop and forces a fresh preconditioner; with a
   fresh preconditioner and no step taken it ends the solve.

The last test plants mistakes in a copy of the oracle (Flag inverted, the
stall rules weakened, the early-stop threshold taken from the current residual)
and checks that the pins above catch each one.
"""
import importlib.util
import os
import sys

import numpy as np
import pytest

from oracle import rfm as O

ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "rfm.py")


# ---------------------------------------------------------------------------
# F(u) = u^3
# ---------------------------------------------------------------------------

class _Cubic:
    """Stands in for a problem description: one unknown, one residual row."""
    n = 1


def _cubic_assemble(prob, u):
    return np.array([u[0] ** 3]), np.array([[3.0 * u[0] ** 2]])


def _cubic_residual(prob, u):
    return np.array([u[0] ** 3])


def run_cubic(mod, tau, m_max, mode="replica"):
    """AMIPN of module `mod` on F(u) = u^3 from u = 1: (u, stats)."""
    saved = mod.assemble, mod.residual
    mod.assemble, mod.residual = _cubic_assemble, _cubic_residual
    try:
        return mod.amipn(_Cubic(), np.array([1.0]),
                         mod.Opts(method="amipn", mode=mode, m_max=m_max, tau_rel=tau, max_outer=5))
    finally:
        mod.assemble, mod.residual = saved


CUBIC_EXPECTED = {
    # tau: (inner steps per outer step, Flags, Jacobian evaluations, final u)
    0.15: ([2, 3, 2, 1, 1], [False] * 5, 1, 0.34725791597676880),
    0.10: ([3, 3, 3, 3, 3], [False, True, False, True, False], 3, 0.082609328935246720),
}


@pytest.mark.parametrize("mode", ["replica", "exact"])
@pytest.mark.parametrize("tau", sorted(CUBIC_EXPECTED))
def test_amipn_chord_steps_on_a_cubic(tau, mode):
    inner, flags, nj, u_end = CUBIC_EXPECTED[tau]
    u, st = run_cubic(O, tau, 3, mode)
    assert st.inner_steps == inner
    assert st.flags == flags
    assert st.jac_evals == nj
    assert st.outer_iters == 5 and st.status == "maxit"
    assert all(a == 1.0 for a in st.alphas)
    assert abs(u[0] - u_end) < 1e-13 * u_end


# ---------------------------------------------------------------------------
# scripted residuals and line-search failures
# ---------------------------------------------------------------------------

class _Script:
    """u = [position]; a direction is always +1; residual(position) is scripted;
    the line search from position p with the preconditioner of Jacobian index j
    fails when (p, j) is listed, else takes the full step."""
    n = 1

    def __init__(self, F, stalls):
        self.F = {k: np.asarray(v, float) for k, v in F.items()}
        self.stalls = set(stalls)
        self.jac = None
        self.last_pos = None
        self.precond_calls = []


def run_script(mod, script, m_max=3, tau=1e-3):
    def make_precond(prob, u, opts, jac_index):
        prob.precond_calls.append((float(u[0]), jac_index))
        prob.jac = jac_index
        return mod.Precond(DJ=np.eye(1), D=np.ones(2), R=None)

    def residual(prob, z):
        p = float(z[0])
        assert p == round(p), "the scripted line search only evaluates whole steps"
        prob.last_pos = int(round(p))
        return prob.F[prob.last_pos]

    def newton_direction(pc, DF, opts, stats):
        stats.lsqr_iters.append(0)
        return np.ones(1)

    def golden_section(phi, phi0, iters=25, accept=1e-4):
        f1 = phi(1.0)
        start = script.last_pos - 1
        if (start, script.jac) in script.stalls:
            return 0.0, phi0, 1
        return 1.0, f1, 1

    names = ("make_precond", "residual", "newton_direction", "golden_section")
    saved = [getattr(mod, k) for k in names]
    for k, f in zip(names, (make_precond, residual, newton_direction, golden_section)):
        setattr(mod, k, f)
    try:
        u, st = mod.amipn(script, np.array([0.0]), mod.Opts(method="amipn", m_max=m_max, tau_rel=tau,
                                                            outer_tol=1e-10, max_outer=10))
    finally:
        for k, f in zip(names, saved):
            setattr(mod, k, f)
    return u, st


def script_a():
    """m_max = 3, tau = 1e-3.
    Outer 1 (Jacobian 0 at 0): |F| 100 -> 10 -> 5 -> 4, changes 90, 5, 1 >= 0.1: m_max reached,
      Flag true, Jacobian 1 at position 3.
    Outer 2: 4 -> 3.999, change 1e-3 < 4e-3: early stop, Flag false (Jacobian 1 kept); the merit
      changed by 1e-3 > eps, go on.
    Outer 3: the line search from 4 with the kept Jacobian 1 finds no decrease: no step, the
      preconditioner was not fresh, so Flag true and Jacobian 2 at 4 (the unchanged merit does not
      end the solve after a failed line search).
    Outer 4: from 4 with Jacobian 2 to 5, change 5e-11 < 4e-3: early stop; the merit changed by
      5e-11 < eps = 1e-10: converged."""
    F = {0: [100, 0], 1: [10, 0], 2: [5, 0], 3: [4, 0], 4: [3.999, 0], 5: [3.999 - 5e-11, 0]}
    return _Script(F, stalls=[(4, 1)])


def script_b():
    """A line search that fails at the first step of a fresh preconditioner ends the solve."""
    return _Script({0: [1, 0], 1: [0.5, 0]}, stalls=[(0, 0)])


def script_c():
    """A failure after a step was taken (inner step 2 of a fresh preconditioner) does not end the
    solve: Flag true, Jacobian 1 at position 1; then one step to convergence."""
    return _Script({0: [100, 0], 1: [10, 0], 2: [10 - 1e-12, 0]}, stalls=[(1, 0)])


SCRIPT_EXPECTED = {
    # (status, final position, inner steps, Flags, preconditioner calls (position, Jacobian index))
    "a": ("ok", 5.0, [3, 1, 1, 1], [True, False, True, False], [(0.0, 0), (3.0, 1), (4.0, 2)]),
    "b": ("stall", 0.0, [1], [True], [(0.0, 0)]),
    "c": ("ok", 2.0, [2, 1], [True, False], [(0.0, 0), (1.0, 1)]),
}
SCRIPTS = {"a": script_a, "b": script_b, "c": script_c}


def observed(mod, name):
    sc = SCRIPTS[name]()
    u, st = run_script(mod, sc)
    return (st.status, float(u[0]), st.inner_steps, st.flags, sc.precond_calls)


@pytest.mark.parametrize("name", sorted(SCRIPTS))
def test_amipn_stall_and_early_stop_rules(name):
    got = observed(O, name)
    assert got == SCRIPT_EXPECTED[name]


# ---------------------------------------------------------------------------
# the pins catch planted mistakes
# ---------------------------------------------------------------------------

MUTATIONS = {
    # Alg. 2's Flag inverted: an early stop recomputes the preconditioner, reaching m_max keeps it
    "flag_inverted": [("        flag = True\n        stalled = False\n", "        flag = False\n        stalled = False\n"),
                      ("                flag = False\n                Fz = Fn\n",
                       "                flag = True\n                Fz = Fn\n")],
    # a failed line search ends the solve even when the preconditioner was not fresh
    "stall_ignores_freshness": [("if stalled and i == 0 and fresh:", "if stalled and i == 0:")],
    # a failed line search after a step also ends the solve
    "stall_ignores_progress": [("if stalled and i == 0 and fresh:", "if stalled and fresh:")],
    # an unchanged merit after a failed line search counts as convergence
    "stall_counts_as_converged": [("if done and not stalled:", "if done:")],
    # the early stop compared with the current residual instead of the outer step's first one
    "early_stop_reference": [("< opts.tau_rel * F0:", "< opts.tau_rel * float(np.linalg.norm(Fz)):")],
}


def _mutant(name):
    src = open(ORACLE_SRC).read()
    for old, new in MUTATIONS[name]:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    spec = importlib.util.spec_from_loader(f"oracle._mutant_{name}", loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    sys.modules[spec.name] = mod          # dataclasses look their module up while the class is built
    try:
        exec(compile(src, f"{ORACLE_SRC} ({name})", "exec"), mod.__dict__)
    finally:
        del sys.modules[spec.name]
    return mod


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistakes(name):
    mod = _mutant(name)
    caught = []
    for tau, (inner, flags, nj, u_end) in CUBIC_EXPECTED.items():
        u, st = run_cubic(mod, tau, 3)
        if (st.inner_steps, st.flags, st.jac_evals) != (inner, flags, nj) or abs(u[0] - u_end) > 1e-13:
            caught.append(f"cubic tau={tau}")
    for sname in SCRIPTS:
        try:
            got = observed(mod, sname)
        except Exception as e:  # a mutant may also break the script's own assumptions
            got = repr(e)
        if got != SCRIPT_EXPECTED[sname]:
            caught.append(f"script {sname}")
    assert caught, f"mutation {name} passes every AMIPN pin"
