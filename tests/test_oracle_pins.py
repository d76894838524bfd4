"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test targets a mistake that could plausibly sit in the oracle: a dropped
term, a wrong sign, a transposed operand or an off-by-one in the row layout.
"""
import math
import os

import numpy as np
import pytest

import rfm_workloads as W
from oracle import philox as P
from oracle import rfm as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# row layout: counts printed in the paper
# ---------------------------------------------------------------------------

def _golden_rows():
    rows = []
    for line in open(os.path.join(GOLDEN, "row_counts.txt")):
        line = line.split("#")[0].split()
        if line:
            rows.append(line)
    return rows


def _cube_problem(q, J, ncomp, cont_orders, dirichlet_comps, nsub=(2, 2, 2)):
    """(2,2,2) boxes on the unit cube with the paper's uniform grids, built from
    the workload helpers; no data (row counting only)."""
    lo, hi = np.zeros(3), np.ones(3)
    nsub = np.array(nsub)
    nbox = int(np.prod(nsub))
    groups = []
    for e in range(nbox):
        blo, bhi = W.box_bounds(e, lo, hi, nsub)
        groups.append(W.PointGroup(W.KIND_PDE, W.box_grid(blo, bhi, [q] * 3), e))
    for a in range(3):
        for e in range(nbox):
            mi = W.box_multi(e, nsub)
            if mi[a] != 0:
                continue
            mj = list(mi)
            mj[a] = 1
            blo, bhi = W.box_bounds(e, lo, hi, nsub)
            pts = W.face_grid(blo, bhi, a, bhi[a], q)
            for c in range(ncomp):
                groups.append(W.PointGroup(W.KIND_CONTINUITY, pts, e, W.box_index(mj, nsub),
                                           comp=c, cont_order=cont_orders[c]))
    for a in range(3):
        for side in (0, 1):
            for e in range(nbox):
                if W.box_multi(e, nsub)[a] != side:
                    continue
                blo, bhi = W.box_bounds(e, lo, hi, nsub)
                pts = W.face_grid(blo, bhi, a, float(side), q)
                for c in dirichlet_comps:
                    groups.append(W.PointGroup(W.KIND_DIRICHLET, pts, e, comp=c))
    return W.Problem("count", 3, ncomp, lo, hi, nsub, J, np.zeros((nbox, ncomp, 1, 3)),
                     np.zeros((nbox, ncomp, 1)), groups, [], [], lambda x: x, np.zeros((0, 3)),
                     np.zeros(0, np.int32))


@pytest.mark.parametrize("entry", _golden_rows(), ids=lambda r: "-".join(r[:3]))
def test_row_counts_match_paper(entry):
    label, q, J = entry[0], int(entry[1]), int(entry[2])
    if label == "overflow":
        prob = _cube_problem(q, J, 1, [2], [0])
        _, m = O.row_table(prob)
        assert m * prob.n == int(entry[4])
    else:
        prob = _cube_problem(q, J, 3, [2, 2, 1], [0, 1])
        _, m = O.row_table(prob)
        assert (m, prob.n) == (int(entry[4]), int(entry[5]))


def test_config_row_counts():
    p1 = W.config1()
    assert (O.row_table(p1)[1], p1.n) == (1920, 800)
    p2 = W.config2(test_per_dim=2)
    assert (O.row_table(p2)[1], p2.n) == (204800, 38400)


# ---------------------------------------------------------------------------
# Philox and Gaussian entries
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ctr,key", [((0, 0, 0, 0), (0, 0)), ((5, 7, 0, 0), (11, 13)),
                                     ((2**64 - 2, 3, 9, 1), (2**63 + 5, 77))])
def test_philox_matches_numpy_library(ctr, key):
    # numpy's Philox (4x64, 10 rounds) bumps its counter before each block
    bg = np.random.Philox(counter=np.array(ctr, np.uint64), key=np.array(key, np.uint64))
    ref = bg.random_raw(4)
    c1 = list(ctr)
    c1[0] = (c1[0] + 1) % 2**64
    mine = P.philox4x64(np.array([c1], np.uint64), key)[0]
    assert [int(v) for v in mine] == [int(v) for v in ref]


def test_gaussian_moments_and_scaling():
    S = P.sketch_matrix(3, 1, 400, 500)
    g = S.ravel() * math.sqrt(400)
    n = g.size
    assert abs(g.mean()) < 5 / math.sqrt(n)
    assert abs(g.var() - 1) < 6 * math.sqrt(2 / n)
    kurt = np.mean(g ** 4)
    assert abs(kurt - 3) < 0.05
    # E[S^T S] = I: column norms concentrate at 1
    cn = np.linalg.norm(S, axis=0)
    assert abs(cn.mean() - 1) < 0.01
    # entries are random-access by (i, r)
    i = np.array([0, 7, 399, 123])
    r = np.array([0, 3, 499, 250])
    assert np.allclose(P.gaussian_entries(3, 1, i, r) / math.sqrt(400), S[i, r], rtol=0, atol=0)
    # different Jacobian index -> independent matrix
    S2 = P.sketch_matrix(3, 2, 400, 500)
    assert abs(np.corrcoef(S.ravel(), S2.ravel())[0, 1]) < 0.01


# ---------------------------------------------------------------------------
# manufactured data vs finite differences of u*
# ---------------------------------------------------------------------------

def _fd_jet(exact, x, h=1e-4):
    d = x.shape[1]
    val = exact(x)
    grad = np.zeros(val.shape + (d,))
    sec = np.zeros(val.shape + (d,))
    for a in range(d):
        xp, xm = x.copy(), x.copy()
        xp[:, a] += h
        xm[:, a] -= h
        fp, fm = exact(xp), exact(xm)
        grad[..., a] = (fp - fm) / (2 * h)
        sec[..., a] = (fp - 2 * val + fm) / (h * h)
    return val, grad, sec


@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
def test_pde_data_matches_finite_differences(cfg):
    small = [dict(nsub=(2, 2), J=4, q=5), dict(nsub=(2, 2, 2), J=4, q=4),
             dict(nsub=(2, 2, 2), J=4, q=4), dict(nsub=(2, 2, 2), J=4, q=4)][cfg]
    prob = W.make_config(cfg, **small)
    g = prob.groups[1]
    assert g.kind == W.KIND_PDE
    x = g.x
    val, grad, sec = _fd_jet(prob.exact, x)
    for q in range(prob.ncomp):
        f = np.zeros(x.shape[0])
        for (eq, c, coeff, deriv) in prob.lin_terms:
            if eq != q:
                continue
            if deriv == W.D_ID:
                f += coeff * val[:, c]
            elif W.D_X0 <= deriv <= W.D_X3:
                f += coeff * grad[:, c, deriv - 1]
            elif deriv == W.D_LAPLACE:
                f += coeff * sec[:, c].sum(-1)
            elif deriv == W.D_LAPLACE_SPACE:
                f += coeff * sec[:, c, :-1].sum(-1)
        for (eq, coeff, pw) in prob.poly_terms:
            if eq == q:
                f += coeff * np.prod([val[:, c] ** p for c, p in enumerate(pw)], axis=0)
        scale = max(1.0, np.abs(g.data[:, q]).max())
        assert np.abs(f - g.data[:, q]).max() < 2e-5 * scale


def test_helmholtz_closed_form_rhs_is_cube():
    # -Lap u* = kappa^2 u* for the product of sines, so f = u*^3 exactly
    prob = W.config3_nohole(nsub=(2, 2, 2), J=4, q=5)
    g = prob.groups[3]
    ustar = prob.exact(g.x)[:, 0]
    assert np.allclose(g.data[:, 0], ustar ** 3, rtol=1e-12, atol=1e-12)


def test_boundary_data_is_exact_solution():
    prob = W.config2(nsub=(2, 2, 2), J=4, q=4)
    for g in prob.groups:
        if g.kind == W.KIND_DIRICHLET:
            assert np.array_equal(g.data, prob.exact(g.x))


# ---------------------------------------------------------------------------
# features and Jacobian
# ---------------------------------------------------------------------------

def test_feature_derivatives_by_finite_differences():
    prob = W.config2(nsub=(2, 2, 2), J=6, q=3)
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 0.5, size=(7, 3))
    phi, dphi, d2phi = O.feature_jet(prob, 0, 1, x)
    h = 1e-5
    for a in range(3):
        xp, xm = x.copy(), x.copy()
        xp[:, a] += h
        xm[:, a] -= h
        fp, fm = O.feature_jet(prob, 0, 1, xp)[0], O.feature_jet(prob, 0, 1, xm)[0]
        assert np.abs((fp - fm) / (2 * h) - dphi[:, :, a]).max() < 1e-8
        assert np.abs((fp - 2 * phi + fm) / h ** 2 - d2phi[:, :, a]).max() < 1e-4
    # phi is tanh of an affine map of the box-normalised coordinate
    mu, sig = O.box_centre_radius(prob, 0)
    z = ((x - mu) / sig) @ prob.W[0, 1].T + prob.b[0, 1]
    assert np.allclose(phi, np.tanh(z), rtol=0, atol=1e-15)


def _with_neumann(prob):
    """Add a Neumann group (a slanted normal) so every row kind is exercised."""
    rng = np.random.default_rng(5)
    e = 1
    blo, bhi = W.box_bounds(e, prob.lo, prob.hi, prob.nsub)
    x = rng.uniform(blo, bhi, size=(5, prob.dim))
    nrm = rng.normal(size=(5, prob.dim))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    jet = W.jet_of(prob)(x)
    data = np.einsum("pcd,pd->pc", jet[1], nrm)
    prob.groups.append(W.PointGroup(W.KIND_NEUMANN, x, e, normal=nrm, comp=-1, data=data))
    return prob


@pytest.mark.parametrize("cfg", [0, 1, 3])
def test_jacobian_matches_central_differences(cfg):
    small = [dict(nsub=(2, 2), J=5, q=3), dict(nsub=(2, 1, 2), J=4, q=3), dict(nsub=(1, 2, 2), J=4, q=3)][
        [0, 1, 3].index(cfg)]
    prob = _with_neumann(W.make_config(cfg, **small))
    rng = np.random.default_rng(1)
    u = rng.normal(size=prob.n)
    F, J = O.assemble(prob, u)
    assert J.shape == (O.row_table(prob)[1], prob.n)
    Jfd = np.zeros_like(J)
    for j in range(prob.n):
        h = 1e-6 * max(1.0, abs(u[j]))
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        Jfd[:, j] = (O.residual(prob, up) - O.residual(prob, um)) / (2 * h)
    err = np.abs(J - Jfd).max() / np.abs(J).max()
    assert err < 1e-7
    # F is the residual evaluated directly
    assert np.allclose(F, O.residual(prob, u), rtol=0, atol=1e-13 * np.abs(F).max())


def test_linear_rows_do_not_depend_on_u():
    prob = W.config2(nsub=(2, 1, 1), J=4, q=3)
    rng = np.random.default_rng(2)
    _, J1 = O.assemble(prob, rng.normal(size=prob.n))
    _, J2 = O.assemble(prob, rng.normal(size=prob.n))
    npde = sum(O.group_nrows(prob, g) for g in prob.groups if g.kind == W.KIND_PDE)
    assert np.array_equal(J1[npde:], J2[npde:])
    assert not np.allclose(J1[:npde], J2[:npde])


def test_assemble_rows_matches_full():
    prob = W.config2(nsub=(2, 1, 2), J=4, q=3)
    u = np.random.default_rng(3).normal(size=prob.n)
    F, J = O.assemble(prob, u)
    rows = np.array([0, 5, F.size // 2, F.size - 1])
    Fr, Jr = O.assemble_rows(prob, u, rows)
    assert np.array_equal(Fr, F[rows]) and np.array_equal(Jr, J[rows])


# ---------------------------------------------------------------------------
# row scaling, QR, conditioning
# ---------------------------------------------------------------------------

def test_row_scale():
    J = np.array([[1.0, -4.0, 2.0], [0.0, 0.0, 0.0], [1e-8, 0, 3e-9]])
    D = O.row_scale(J, 100.0)
    assert np.allclose(np.abs(D[:, None] * J).max(1), [100, 0, 100])
    assert D[1] == 1.0


def test_qr_r_invariants_and_cholesky_route():
    rng = np.random.default_rng(4)
    B = rng.normal(size=(60, 25)) @ np.diag(np.logspace(0, 3, 25))
    R = O.qr_r(B)
    assert np.all(np.diag(R) > 0)
    assert np.allclose(np.tril(R, -1), 0)
    G = B.T @ B
    assert np.abs(R.T @ R - G).max() < 1e-12 * np.abs(G).max()
    # unique factor: equals the Cholesky factor of B^T B for well-conditioned B
    L = np.linalg.cholesky(G)
    assert np.allclose(R, L.T, rtol=1e-9, atol=1e-9 * np.abs(R).max())


def test_qr_singular_detected():
    B = np.random.default_rng(0).normal(size=(10, 4))
    B[:, 2] = 0
    with pytest.raises(O.SingularPreconditioner):
        O.qr_r(B)


def test_sketch_preconditioning_drops_condition_number():
    """kappa(D J R^-1) is O(1) and independent of kappa(D J) (the bound quoted
    in Sec. 4.1).  For a Gaussian S with s = 2n the singular values of S Q lie
    near the Marchenko-Pastur edges 1 -/+ sqrt(n/s), so those of D J R^-1 lie
    near 1/(1 + sqrt(1/2)) = 0.586 and 1/(1 - sqrt(1/2)) = 3.41 (kappa ~ 5.8)."""
    prob = W.config1(nsub=(2, 2), J=100, q=14)
    u = np.zeros(prob.n)
    F, J = O.assemble(prob, u)
    D = O.row_scale(J)
    DJ = D[:, None] * J
    s = O.sketch_rows(prob.n, 2.0)
    R = O.qr_r(O.sketch(DJ, s, 1, 0))
    sv = np.linalg.svd(DJ, compute_uv=False)
    assert sv[0] / sv[-1] > 1e8
    A = DJ @ np.linalg.inv(R)
    sa = np.linalg.svd(A, compute_uv=False)
    kap = sa[0] / sa[-1]
    assert 3.0 < kap < 10.0
    r = math.sqrt(prob.n / s)
    assert abs(sa[-1] * (1 + r) - 1) < 0.2
    assert abs(sa[0] * (1 - r) - 1) < 0.25


# ---------------------------------------------------------------------------
# LSQR and line search
# ---------------------------------------------------------------------------

def test_lsqr_matches_dense_lstsq():
    rng = np.random.default_rng(7)
    A = rng.normal(size=(80, 30)) @ np.diag(np.linspace(1, 5, 30))
    b = rng.normal(size=80)
    res = O.lsqr(lambda v: A @ v, lambda w: A.T @ w, b, 30, 1e-12, 500)
    x = np.linalg.lstsq(A, b, rcond=None)[0]
    assert res.istop == 2
    assert np.linalg.norm(res.x - x) < 1e-9 * np.linalg.norm(x)
    # consistent system stops by rule 1
    b2 = A @ rng.normal(size=30)
    res2 = O.lsqr(lambda v: A @ v, lambda w: A.T @ w, b2, 30, 1e-12, 500)
    assert res2.istop == 1
    assert np.linalg.norm(A @ res2.x - b2) < 1e-10 * np.linalg.norm(b2)


def test_preconditioned_lsqr_step_matches_lstsq_step():
    prob = W.config1(nsub=(2, 2), J=40, q=10)
    u = np.random.default_rng(8).normal(size=prob.n) * 0.1
    F, J = O.assemble(prob, u)
    D = O.row_scale(J)
    DJ, DF = D[:, None] * J, D * F
    R = O.qr_r(O.sketch(DJ, O.sketch_rows(prob.n, 2.0), 1, 0))
    st = O.Stats()
    pc = O.Precond(DJ, D, R)
    du = O.newton_direction(pc, DF, O.Opts(lsqr_tol=1e-10), st)
    du_ref = np.linalg.lstsq(DJ, -DF, rcond=None)[0]
    assert np.linalg.norm(DJ @ (du - du_ref)) / np.linalg.norm(DF) < 1e-9
    assert 20 < st.lsqr_iters[0] < 150


def test_golden_section_on_unimodal_functions():
    a, f, _ = O.golden_section(lambda t: (t - 0.3) ** 2 + 1.0, 1.09, iters=25)
    assert abs(a - 0.3) < 1e-5 and f < 1.0 + 1e-9
    # decreasing function: the full step is taken at once
    a, f, nev = O.golden_section(lambda t: 2.0 - t, 2.0)
    assert a == 1.0 and nev == 1
    # increasing function: no decrease, no step
    a, f, _ = O.golden_section(lambda t: 1.0 + t, 1.0)
    assert a == 0.0 and f == 1.0
    # minimum at the right end but below the sufficient-decrease factor
    a, f, _ = O.golden_section(lambda t: 1.0 - 1e-6 * t, 1.0)
    assert a > 0.99999


# ---------------------------------------------------------------------------
# Newton solvers
# ---------------------------------------------------------------------------

def test_linear_problem_converges_in_one_full_step():
    """With mu = 0 the Newton step solves the linear least-squares problem exactly."""
    prob = W.config1(nsub=(2, 2), J=40, q=10)
    # drop the cubic term and give the data of -Lap u* only
    prob.poly_terms = []
    for g in prob.groups:
        if g.kind == W.KIND_PDE:
            jet = W.jet_config1(g.x)
            g.data = -jet[2]
    u, st = O.ipn(prob, opts=O.Opts(max_outer=3))
    F, J = O.assemble(prob, np.zeros(prob.n))
    D = O.row_scale(J)
    ref = np.linalg.lstsq(D[:, None] * J, -D * F, rcond=None)[0]
    assert st.alphas[0] == 1.0
    assert np.linalg.norm(D * (J @ (u - ref))) < 1e-8 * np.linalg.norm(D * F)


def test_ipn_and_amipn_reach_manufactured_solution_config1():
    prob = W.config1()
    u, st = O.ipn(prob)
    assert st.status == "ok"
    e_ipn = O.rel_l2(prob, u)
    assert e_ipn[0] < 1e-6
    ua, sta = O.amipn(prob, opts=O.Opts(method="amipn", m_max=5))
    assert sta.status == "ok"
    assert O.rel_l2(prob, ua)[0] < 1e-6
    assert sta.jac_evals <= sta.outer_iters + 1
    assert sta.jac_evals < st.jac_evals
    # the two solvers agree on the field
    fi = O.eval_field(prob, u, prob.test_x, prob.test_owner)
    fa = O.eval_field(prob, ua, prob.test_x, prob.test_owner)
    assert np.linalg.norm(fi - fa) / np.linalg.norm(fi) < 1e-8


def test_exact_and_replica_modes_agree():
    prob = W.config2(nsub=(2, 1, 1), J=30, q=5)
    ur, sr = O.ipn(prob, opts=O.Opts(mode="replica"))
    ue, se = O.ipn(prob, opts=O.Opts(mode="exact"))
    fr = O.eval_field(prob, ur, prob.test_x, prob.test_owner)
    fe = O.eval_field(prob, ue, prob.test_x, prob.test_owner)
    assert np.linalg.norm(fr - fe) / np.linalg.norm(fe) < 1e-7


@pytest.mark.parametrize("cfg,kw,tol", [
    (1, dict(nsub=(1, 1, 1), J=250, q=8), 0.03),      # Gray-Scott pair
    (2, dict(nsub=(1, 1, 1), J=300, q=9), 0.05),      # Helmholtz kappa = 8
    (3, dict(nsub=(2, 2, 2), J=120, q=6), 0.15),      # space-time Allen-Cahn
])
def test_operator_signs_by_manufactured_solution(cfg, kw, tol):
    """The exact-Newton iteration approaches u*; a flipped sign or a dropped
    term in any operator would leave an O(1) error."""
    prob = W.make_config(cfg, **kw)
    u, st = O.ipn(prob, opts=O.Opts(mode="exact"))
    assert st.status == "ok"
    assert np.all(O.rel_l2(prob, u) < tol)


# ---------------------------------------------------------------------------
# geometry with holes
# ---------------------------------------------------------------------------

def test_sphere_holes_geometry():
    p = W.config3(nsub=(2, 2, 2), J=20, q=6, test_per_dim=2)
    c, r = p.params["centres"], p.params["radii"]
    for i in range(len(r)):
        assert 0.15 <= c[i].min() and c[i].max() <= 0.85 and 0.05 <= r[i] <= 0.12
        for j in range(i + 1, len(r)):
            assert np.linalg.norm(c[i] - c[j]) >= r[i] + r[j] + 0.02
    for g in p.groups:
        d = np.linalg.norm(g.x[:, None, :] - c[None], axis=2) - r[None]
        if g.kind == W.KIND_DIRICHLET and np.all(np.abs(d).min(axis=1) < 1e-12):
            # sphere surface points: on one sphere, outside the others, in their owner box
            continue
        assert np.all(d > 0), g.kind
    npde = sum(len(g.x) for g in p.groups if g.kind == W.KIND_PDE)
    assert npde < 8 * 6 ** 3                      # some points fall in the holes
    surf = [g for g in p.groups if g.kind == W.KIND_DIRICHLET and
            np.all(np.abs(np.linalg.norm(g.x[:, None, :] - c[None], axis=2) - r[None]).min(axis=1) < 1e-12)]
    tot = sum(len(g.x) for g in surf)
    assert tot == sum(int(np.ceil(64 * 4 * np.pi * ri ** 2 * 64)) for ri in r)
    for g in surf:
        lo, hi = W.box_bounds(g.owner, p.lo, p.hi, p.nsub)
        assert np.all(g.x >= lo - 1e-12) and np.all(g.x <= hi + 1e-12)
        assert np.allclose(g.data, p.exact(g.x))


def test_moving_hole_neumann_data_by_finite_differences():
    p = W.config4(nsub=(2, 2, 2), J=20, q=5, n_t=8, n_theta=6, test_per_dim=2)
    neu = [g for g in p.groups if g.kind == W.KIND_NEUMANN]
    assert sum(len(g.x) for g in neu) == 8 * 6
    h = 1e-5
    for g in neu:
        c = W.ac_hole_centre(g.x[:, 2])
        assert np.allclose(np.linalg.norm(g.x[:, :2] - c, axis=1), W.AC_HOLE_R)
        # outward normal of the domain points into the hole
        assert np.allclose(g.normal[:, :2], (c - g.x[:, :2]) / W.AC_HOLE_R) and np.all(g.normal[:, 2] == 0)
        fd = (p.exact(g.x + h * g.normal) - p.exact(g.x - h * g.normal)) / (2 * h)
        assert np.allclose(g.data, fd, atol=1e-7)
    for g in p.groups:
        if g.kind in (W.KIND_PDE, W.KIND_CONTINUITY, W.KIND_DIRICHLET):
            assert np.all(np.linalg.norm(g.x[:, :2] - W.ac_hole_centre(g.x[:, 2]), axis=1) > W.AC_HOLE_R)


@pytest.mark.parametrize("make,tol", [
    (lambda: W.config3(nsub=(1, 1, 1), J=300, q=9, test_per_dim=6), 0.05),
    (lambda: W.config4(nsub=(2, 2, 2), J=120, q=6, n_t=24, n_theta=16, test_per_dim=3), 0.15),
])
def test_hole_boundaries_by_manufactured_solution(make, tol):
    """Sphere Dirichlet rows and moving-hole Neumann rows (with their normals) are
    consistent with u*: the exact-Newton iteration approaches it."""
    prob = make()
    u, st = O.ipn(prob, opts=O.Opts(mode="exact"))
    assert st.status == "ok"
    assert np.all(O.rel_l2(prob, u) < tol)


# ---------------------------------------------------------------------------
# count sketch
# ---------------------------------------------------------------------------

def test_count_sketch_structure():
    s, m = 300, 5000
    S = P.count_sketch_matrix(4, 1, s, m)
    # one +-1 per column: S^T S = I exactly
    assert np.array_equal((S != 0).sum(axis=0), np.ones(m))
    assert set(np.unique(S[S != 0])) <= {-1.0, 1.0}
    assert np.array_equal(np.diag(S.T @ S), np.ones(m))
    # buckets and signs are uniform: counts per bucket ~ Poisson(m/s), signs balanced
    cnt = (S != 0).sum(axis=1)
    lam = m / s
    assert abs(cnt.mean() - lam) < 1e-12
    assert abs(cnt.var() - lam) < 6 * lam * np.sqrt(2 / s)
    nz = S[S != 0]
    assert abs(nz.mean()) < 5 / np.sqrt(m)
    # byte-independent check of the hash: word 0 mod s, bit 0 of word 1
    w = P.philox4x64(np.array([[7, 0, 2, 0]], np.uint64), (4, 1))[0]
    h, sig = P.count_sketch_hash(4, 1, np.array([7]), s)
    assert h[0] == int(w[0]) % s and sig[0] == (1.0 if int(w[1]) % 2 == 0 else -1.0)
    # a different Jacobian index rehashes
    S2 = P.count_sketch_matrix(4, 2, s, m)
    assert (np.argmax(S2 != 0, axis=0) != np.argmax(S != 0, axis=0)).mean() > 0.9


def test_count_sketch_preconditions():
    """With s = 3n (the paper's gamma) the count sketch embeds the column space well
    enough that D J R^-1 is well conditioned although D J is not, and LSQR converges."""
    prob = W.config1(nsub=(2, 2), J=100, q=14)
    F, J = O.assemble(prob, np.zeros(prob.n))
    D = O.row_scale(J)
    DJ = D[:, None] * J
    s = O.sketch_rows(prob.n, 3.0)
    R = O.qr_r(P.count_sketch_matrix(1, 0, s, DJ.shape[0]) @ DJ)
    sa = np.linalg.svd(DJ @ np.linalg.inv(R), compute_uv=False)
    sv = np.linalg.svd(DJ, compute_uv=False)
    assert sv[0] / sv[-1] > 1e8
    assert sa[0] / sa[-1] < 100.0
    res = O.lsqr(lambda v: DJ @ O.r_solve(R, v), lambda w: O.rt_solve(R, DJ.T @ w), -D * F, prob.n, 1e-10, 1000)
    assert res.istop in (1, 2)


# ---------------------------------------------------------------------------
# pointwise transcendental terms: Lap u - 100 u + 10 cosh(u) = f (Sec. 6.2, IPN vs AMIPN)
# ---------------------------------------------------------------------------

def test_cosh_data_matches_finite_differences():
    prob = W.helmholtz_cosh(nsub=(2, 2, 2), J=4, q=4)
    g = prob.groups[1]
    assert g.kind == W.KIND_PDE
    val, grad, sec = _fd_jet(prob.exact, g.x)
    f = sec[:, 0].sum(-1) - 100.0 * val[:, 0] + 10.0 * np.cosh(val[:, 0])
    assert np.abs(f - g.data[:, 0]).max() < 2e-5 * max(1.0, np.abs(g.data).max())


@pytest.mark.parametrize("fn", ["cosh", "sinh", "exp"])
def test_pointwise_term_jacobian_matches_central_differences(fn):
    prob = W.helmholtz_cosh(nsub=(2, 1, 2), J=4, q=3)
    prob.fn_terms = [(0, 0, 10.0, fn)]
    u = 0.3 * np.random.default_rng(4).normal(size=prob.n)
    F, J = O.assemble(prob, u)
    Jfd = np.zeros_like(J)
    for j in range(prob.n):
        h = 1e-6
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        Jfd[:, j] = (O.residual(prob, up) - O.residual(prob, um)) / (2 * h)
    assert np.abs(J - Jfd).max() / np.abs(J).max() < 1e-7
    # the term enters F with its sign and coefficient: removing it changes F by exactly 10 f(u_n)
    prob0 = W.helmholtz_cosh(nsub=(2, 1, 2), J=4, q=3)
    prob0.fn_terms = []
    F0 = O.residual(prob0, u)
    un = np.concatenate([O.feature_jet(prob, g.owner, 0, g.x)[0] @ u[O.col_slice(prob, g.owner, 0)]
                         for g in prob.groups if g.kind == W.KIND_PDE])
    npde = un.size
    ref = {"cosh": np.cosh, "sinh": np.sinh, "exp": np.exp}[fn]
    assert np.allclose(F[:npde] - F0[:npde], 10.0 * ref(un), rtol=1e-12, atol=1e-12)
    assert np.array_equal(F[npde:], F0[npde:])


def test_cosh_problem_by_manufactured_solution():
    """The exact-Newton iteration reaches u* of the cosh problem to the discretisation's accuracy."""
    prob = W.helmholtz_cosh(nsub=(1, 1, 1), J=300, q=10, test_per_dim=4)
    u, st = O.ipn(prob, opts=O.Opts(mode="exact"))
    assert st.status == "ok"
    assert np.all(O.rel_l2(prob, u) < 2e-3)


def _flux_divergence(u, x, h=1e-3):
    """-div((1 + u^2) grad u) by central differences of the flux at half steps (a form that does not
    expand the operator into the product terms)."""
    out = np.zeros(x.shape[0])
    u0 = u(x)[:, 0]
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        up, um = u(x + e)[:, 0], u(x - e)[:, 0]
        uhp, uhm = u(x + e / 2)[:, 0], u(x - e / 2)[:, 0]
        out -= ((1 + uhp ** 2) * (up - u0) - (1 + uhm ** 2) * (u0 - um)) / (h * h)
    return out


def test_quasilinear_data_matches_the_flux_form():
    """The data of the quasi-linear benchmark (Sec. 3.2): f = -div((1 + u*^2) grad u*), written out as
    product terms, against central differences of the flux itself; also the jet of u* against central
    differences of u*."""
    prob = W.quasilinear(nsub=(2, 2, 2), J=4, q=5)
    g = prob.groups[1]
    assert g.kind == W.KIND_PDE
    f = _flux_divergence(prob.exact, g.x)
    assert np.abs(f - g.data[:, 0]).max() < 1e-4 * max(1.0, np.abs(g.data).max())
    val, grad, sec = _fd_jet(prob.exact, g.x)
    jv, jg, jl, _ = W.jet_quasilinear(g.x)
    assert np.abs(jv - val).max() < 1e-12
    assert np.abs(jg - grad).max() < 1e-6
    assert np.abs(jl[:, 0] - sec[:, 0].sum(-1)).max() < 1e-4


def test_product_term_jacobian_matches_central_differences():
    """Product terms of field derivatives (u^2 Lap u, u (d_x u)^2, u_x u_y^3 Lap u): the oracle's Jacobian
    rows against central differences of its residual, and each term entering F with its coefficient."""
    prob = W.quasilinear(nsub=(2, 1, 2), J=4, q=3)
    prob.prod_terms = [(0, -1.0, ((0, W.D_ID, 2), (0, W.D_LAPLACE, 1))),
                       (0, -2.0, ((0, W.D_ID, 1), (0, W.D_X0, 2))),
                       (0, 0.5, ((0, W.D_X0, 1), (0, W.D_X1, 3), (0, W.D_LAPLACE, 1)))]
    u = 0.3 * np.random.default_rng(4).normal(size=prob.n)
    F, J = O.assemble(prob, u)
    Jfd = np.zeros_like(J)
    for j in range(prob.n):
        h = 1e-6
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        Jfd[:, j] = (O.residual(prob, up) - O.residual(prob, um)) / (2 * h)
    assert np.abs(J - Jfd).max() / np.abs(J).max() < 1e-7
    # the last term alone: 0.5 u_x u_y^3 Lap u from the feature jets directly
    prob0 = W.quasilinear(nsub=(2, 1, 2), J=4, q=3)
    prob0.prod_terms = prob.prod_terms[:2]
    F0 = O.residual(prob0, u)
    parts = []
    for g in prob.groups:
        if g.kind != W.KIND_PDE:
            continue
        phi, dphi, d2phi = O.feature_jet(prob, g.owner, 0, g.x)
        cu = u[O.col_slice(prob, g.owner, 0)]
        parts.append(0.5 * (dphi[..., 0] @ cu) * (dphi[..., 1] @ cu) ** 3 * (d2phi.sum(-1) @ cu))
    ref = np.concatenate(parts)
    npde = ref.size
    assert np.allclose(F[:npde] - F0[:npde], ref, rtol=1e-11, atol=1e-12)
    assert np.array_equal(F[npde:], F0[npde:])


def test_quasilinear_problem_by_manufactured_solution():
    """The exact-Newton iteration reaches u* of the quasi-linear benchmark to the discretisation's
    accuracy."""
    prob = W.quasilinear(nsub=(1, 1, 1), J=500, q=12, test_per_dim=4)
    u, st = O.ipn(prob, opts=O.Opts(mode="exact"))
    assert st.status == "ok"
    assert np.all(O.rel_l2(prob, u) < 5e-4)


def test_ball_problem_data_and_geometry():
    """The diffusion-reaction problem on the unit ball (Sec. 6.2): its data against central differences of
    the flux (1 + u*^2) grad u* plus u*^3 - u* + e^u*, every collocation and interface point inside the
    ball, the Dirichlet points on the unit sphere and owned by the box that holds them, no rows on the
    cube's faces, and the jet of u* against central differences."""
    prob = W.diffusion_reaction_ball(J=4, q=7, nbdy=500)
    for g in prob.groups:
        r2 = (g.x ** 2).sum(1)
        if g.kind == W.KIND_DIRICHLET:
            assert np.allclose(r2, 1.0, atol=1e-12)
            blo, bhi = W.box_bounds(g.owner, prob.lo, prob.hi, prob.nsub)
            assert np.all((g.x >= blo - 1e-12) & (g.x <= bhi + 1e-12))
        else:
            assert np.all(r2 < 1.0)
    assert sum(g.x.shape[0] for g in prob.groups if g.kind == W.KIND_DIRICHLET) == 500
    g = next(g for g in prob.groups if g.kind == W.KIND_PDE and g.x.shape[0] > 20)
    u = prob.exact(g.x)[:, 0]
    f = _flux_divergence(prob.exact, g.x) + u ** 3 - u + np.exp(u)
    assert np.abs(f - g.data[:, 0]).max() < 1e-4 * max(1.0, np.abs(g.data).max())
    val, grad, sec = _fd_jet(prob.exact, g.x)
    jv, jg, jl, _ = W.jet_ball(g.x)
    assert np.abs(jv - val).max() < 1e-12
    assert np.abs(jg - grad).max() < 1e-6
    assert np.abs(jl[:, 0] - sec[:, 0].sum(-1)).max() < 1e-4


def test_ball_problem_by_manufactured_solution():
    """Exact Newton reaches u* of the ball problem to the discretisation's accuracy (2x2x2 boxes,
    J = 200, q = 10, 2000 sphere points)."""
    prob = W.diffusion_reaction_ball(J=200, q=10, nbdy=2000, test_per_dim=4)
    u, st = O.ipn(prob, opts=O.Opts(mode="exact"))
    assert st.status == "ok"
    assert np.all(O.rel_l2(prob, u) < 5e-3)


def test_gray_scott_nonlinear_data_matches_finite_differences():
    """The paper's Gray-Scott system with D = 1 + u^2, 1 + v^2 (Sec. 6.2): its data (the constant F of
    the first equation carried by the data) against central differences of (u*, v*), and the jet."""
    prob = W.gray_scott_nonlinear(nsub=(2, 2, 2), J=4, q=5)
    g = prob.groups[2]
    assert g.kind == W.KIND_PDE
    val, grad, sec = _fd_jet(prob.exact, g.x)
    u, v = val[:, 0], val[:, 1]
    lu, lv = sec[:, 0].sum(-1), sec[:, 1].sum(-1)
    F, k = W.GS2_F, W.GS2_K
    f1 = (1 + u * u) * lu - u * v * v + F * (1 - u) - F
    f2 = (1 + v * v) * lv + u * v * v - (F + k) * v
    scale = max(1.0, np.abs(g.data).max())
    assert np.abs(f1 - g.data[:, 0]).max() < 2e-5 * scale
    assert np.abs(f2 - g.data[:, 1]).max() < 2e-5 * scale
    jv, jg, jl, _ = W.jet_gray_scott_nonlinear(g.x)
    assert np.abs(jv - val).max() < 1e-12
    assert np.abs(jg - grad).max() < 1e-6
    assert np.abs(jl - sec.sum(-1)).max() < 1e-4


def test_gray_scott_nonlinear_by_manufactured_solution():
    """Exact Newton reaches (u*, v*) of the nonlinear-diffusion Gray-Scott system (one box)."""
    prob = W.gray_scott_nonlinear(nsub=(1, 1, 1), J=300, q=12, test_per_dim=4)
    u, st = O.ipn(prob, opts=O.Opts(mode="exact"))
    assert st.status == "ok"
    assert np.all(O.rel_l2(prob, u) < 5e-3)


# ---------------------------------------------------------------------------
# smooth partition of unity (Sec. 2.2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nsub", [(2, 2), (3, 1), (2, 2, 2)])
def test_smooth_pou_sums_to_one_on_the_domain(nsub):
    """The smooth partition functions sum to 1 everywhere in the domain, the strips along its boundary
    included (where an edge box's bump is flat on the side facing the boundary)."""
    d = len(nsub)
    prob = W.config1(J=4, q=4, pou="b") if d == 2 else W.quasilinear(nsub=nsub, J=4, q=4, pou="b")
    prob.nsub = np.asarray(nsub)
    x = np.random.default_rng(3).uniform(0.0, 1.0, size=(4000, d))
    x[:200, 0] = 0.0
    x[200:400, -1] = 1.0
    s = sum(O.pou_b(prob, e, x)[0] for e in range(int(np.prod(nsub))))
    assert np.abs(s - 1.0).max() < 1e-14


def test_smooth_bump_is_c1_and_its_derivatives():
    """varphi^b: derivatives against central differences away from the band edges; value and first
    derivative continuous across |y| = 3/4 and 5/4 (the second derivative jumps there)."""
    y = np.random.default_rng(4).uniform(-1.5, 1.5, size=5000)
    y = y[np.min(np.abs(np.abs(y)[:, None] - np.array([0.75, 1.25])[None]), axis=1) > 1e-3]
    h = 1e-6
    f, d1, d2 = O.bump_b(y)
    fp, d1p, _ = O.bump_b(y + h)
    fm, d1m, _ = O.bump_b(y - h)
    assert np.abs((fp - fm) / (2 * h) - d1).max() < 1e-7
    assert np.abs((d1p - d1m) / (2 * h) - d2).max() < 1e-5
    for edge in (0.75, 1.25, -0.75, -1.25):
        lo, hi = O.bump_b(np.array([edge - 1e-9])), O.bump_b(np.array([edge + 1e-9]))
        assert abs(lo[0][0] - hi[0][0]) < 1e-8 and abs(lo[1][0] - hi[1][0]) < 1e-7


def test_smooth_pou_field_derivatives_match_central_differences():
    """Gradient and Laplacian of the blended field sum_e psi_e phi_e u_e (product rule in the oracle)
    against central differences of the field itself."""
    prob = W.config1(J=30, q=6, pou="b", test_per_dim=2)
    u = np.random.default_rng(5).normal(size=prob.n)
    x = np.random.default_rng(6).uniform(0.02, 0.98, size=(300, 2))
    own = np.zeros(x.shape[0], np.int32)
    boxes = O.covering_boxes(prob, x)
    grad = sum(O.blended_jet(prob, e, 0, x)[1].transpose(0, 2, 1) @ u[O.col_slice(prob, e, 0)] for e in boxes)
    lap = sum(O.blended_jet(prob, e, 0, x)[2].sum(-1) @ u[O.col_slice(prob, e, 0)] for e in boxes)
    f0 = O.eval_field(prob, u, x, own)[:, 0]
    h, fdl = 1e-4, np.zeros(x.shape[0])
    for a in range(2):
        # first differences with a small step: at the bump's band edges the field's second derivative
        # jumps, so central differences lose their second order there
        hg = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[:, a] += hg
        xm[:, a] -= hg
        gfd = (O.eval_field(prob, u, xp, own)[:, 0] - O.eval_field(prob, u, xm, own)[:, 0]) / (2 * hg)
        assert np.abs(gfd - grad[:, a]).max() < 1e-6 * max(1.0, np.abs(grad).max())
        xp, xm = x.copy(), x.copy()
        xp[:, a] += h
        xm[:, a] -= h
        fp, fm = O.eval_field(prob, u, xp, own)[:, 0], O.eval_field(prob, u, xm, own)[:, 0]
        fdl += (fp - 2 * f0 + fm) / (h * h)
    # the bump's second derivative jumps at |y| = 3/4: compare away from those lines
    far = np.all(np.abs(np.abs((x % 0.5) - 0.25) / 0.25 - 0.75) > 0.01, axis=1)
    assert np.abs(fdl - lap)[far].max() < 1e-3 * max(1.0, np.abs(lap).max())


def test_smooth_pou_jacobian_matches_central_differences():
    """Residual and Jacobian rows with the smooth partition (quasi-linear product terms, Dirichlet rows,
    no continuity rows) against central differences of the residual."""
    prob = W.quasilinear(nsub=(2, 1, 2), J=4, q=3, pou="b")
    assert not any(g.kind == W.KIND_CONTINUITY for g in prob.groups)
    u = 0.3 * np.random.default_rng(4).normal(size=prob.n)
    F, J = O.assemble(prob, u)
    Jfd = np.zeros_like(J)
    for j in range(prob.n):
        h = 1e-6
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        Jfd[:, j] = (O.residual(prob, up) - O.residual(prob, um)) / (2 * h)
    assert np.abs(J - Jfd).max() / np.abs(J).max() < 1e-7


def test_smooth_pou_problem_by_manufactured_solution():
    """Exact Newton with the smooth partition (no continuity rows) reaches u* of the 2-D workload."""
    prob = W.config1(J=200, q=20, pou="b", test_per_dim=10)
    u, st = O.ipn(prob, opts=O.Opts(mode="exact"))
    assert st.status == "ok"
    assert np.all(O.rel_l2(prob, u) < 1e-6)


def test_paper_allen_cahn_moving_hole_data_and_geometry():
    """The paper's space-time Allen-Cahn problem with a moving hole (Sec. 6.3): data against central
    differences of u* (u_t - Lap_xy u + u^3 - u), no collocation point inside the hole, the hole's
    Dirichlet points on its moving circle, and the jet."""
    prob = W.allen_cahn_moving_hole(J=4, q=8)
    for g in prob.groups:
        d = np.linalg.norm(g.x[:, :2] - W.ac2_hole_centre(g.x[:, 2]), axis=1)
        if g.kind == W.KIND_DIRICHLET and np.allclose(d, W.AC2_HOLE_R, atol=1e-12):
            np.testing.assert_allclose(g.data[:, 0], prob.exact(g.x)[:, 0], rtol=0, atol=1e-14)
        else:
            assert np.all(d > W.AC2_HOLE_R)
    g = next(g for g in prob.groups if g.kind == W.KIND_PDE)
    val, grad, sec = _fd_jet(prob.exact, g.x)
    u = val[:, 0]
    f = grad[:, 0, 2] - sec[:, 0, 0] - sec[:, 0, 1] + u ** 3 - u
    assert np.abs(f - g.data[:, 0]).max() < 2e-5 * max(1.0, np.abs(g.data).max())
    jv, jg, jl, jls = W.jet_ac_paper(g.x)
    assert np.abs(jg - grad).max() < 1e-6
    assert np.abs(jls[:, 0] - sec[:, 0, :2].sum(-1)).max() < 1e-4


def test_one_dimensional_workload_by_manufactured_solution():
    """The 1-D workload (single-point faces and interfaces): u*'s derivatives against central differences
    of u* itself, the data f = -u*'' + u*^3 at the PDE points, and exact Newton reaching u*."""
    x = np.linspace(0.05, 0.95, 9)[:, None]
    v, g, lap, _ = W.jet_line(x)
    h = 1e-4
    vp, vm = W.jet_line(x + h)[0], W.jet_line(x - h)[0]
    assert np.allclose((vp - vm) / (2 * h), g[:, :, 0], atol=1e-7)
    assert np.allclose((vp - 2 * v + vm) / h ** 2, lap, atol=1e-5)
    prob = W.line_1d()
    pde = [gr for gr in prob.groups if gr.kind == W.KIND_PDE]
    for gr in pde:
        vv, _, ll, _ = W.jet_line(gr.x)
        assert np.allclose(gr.data, -ll + vv ** 3, rtol=1e-13, atol=1e-13)
    # two end points and three interface points (C0 and C1 rows each): m = 4 * 40 + 2 + 3 * 2
    assert sum(gr.x.shape[0] for gr in prob.groups if gr.kind != W.KIND_PDE) == 2 + 3
    assert O.row_table(prob)[1] == 4 * 40 + 2 + 3 * 2
    # exact Newton gets to the discretisation's floor (4.2e-5), where its line search can end the solve
    u, st = O.ipn(prob, opts=O.Opts(mode="exact"))
    assert st.status in ("ok", "stall") and O.rel_l2(prob, u)[0] < 1e-4
