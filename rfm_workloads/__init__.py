"""Seeded synthetic random-feature-method problems.

This module only *describes* problems: the box partition, the fixed random
feature parameters, the collocation point groups with their data, the PDE
operator as a list of terms, and a manufactured solution with its closed-form
derivatives.  It contains none of the solver's arithmetic (no feature
evaluation, no residual, no Jacobian, no sketch), so it can feed both the GPU
library and the CPU oracle without coupling them.

Problem setting (paper, Sec. 2.1 and Sec. 2.2): P(u) = lambda*L u + mu*N(u) = f
in Omega and B u = g on the boundary; the box Omega_c is split into
non-overlapping boxes, each carrying J tanh features whose weights and biases
are drawn uniformly from [-R, R] and then frozen.  Collocation follows Sec. 5:
uniform grids that include the end points, interface grids that carry C^0 and
C^1 continuity rows, and boundary grids on the outer faces.

Row order.  Every ``PointGroup`` shares one owner box (and one neighbour box
for continuity groups).  Groups are listed in the order
[PDE groups; continuity groups; outer-boundary groups; hole-surface groups],
i.e. F = [R_pde; R_con; R_bdy] of Alg. 3, and a consumer expands each group
into rows ordered (equation or component, continuity order, point).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

# point kinds
KIND_PDE = 0
KIND_DIRICHLET = 1
KIND_NEUMANN = 2
KIND_CONTINUITY = 3

# derivative selectors of a linear term
D_ID = 0                 # the value itself
D_X0, D_X1, D_X2, D_X3 = 1, 2, 3, 4   # first derivative along axis k is 1 + k
D_LAPLACE = 8            # sum of second derivatives over all axes
D_LAPLACE_SPACE = 9      # sum of second derivatives over all axes but the last (time)

# pointwise functions of one field component in a nonlinear term (coeff * f(u_c))
FN_COSH, FN_SINH, FN_EXP = "cosh", "sinh", "exp"
FN_CODES = {FN_COSH: 0, FN_SINH: 1, FN_EXP: 2}
_FN_VALUE = {FN_COSH: np.cosh, FN_SINH: np.sinh, FN_EXP: np.exp}


@dataclass
class PointGroup:
    kind: int
    x: np.ndarray                       # [npts, dim] float64
    owner: int                          # box that owns every point of the group
    neighbor: int = -1                  # second box (continuity groups only)
    normal: Optional[np.ndarray] = None  # [npts, dim] (Neumann, continuity)
    comp: int = -1                      # -1: all components/equations, else one
    cont_order: int = 1                 # continuity groups: 1 -> C0, 2 -> C0 + C1
    data: Optional[np.ndarray] = None   # PDE: [npts, neq]; Dirichlet/Neumann: [npts, ncomp_sel]

    @property
    def npts(self) -> int:
        return int(self.x.shape[0])


@dataclass
class Problem:
    name: str
    dim: int
    ncomp: int
    lo: np.ndarray
    hi: np.ndarray
    nsub: np.ndarray                   # boxes per axis, axis 0 fastest in the box index
    J: int                             # features per box and component
    W: np.ndarray                      # [Mp, ncomp, J, dim]
    b: np.ndarray                      # [Mp, ncomp, J]
    groups: List[PointGroup]
    lin_terms: List[Tuple[int, int, float, int]]            # (eq, comp, coeff, deriv)
    poly_terms: List[Tuple[int, float, Tuple[int, ...]]]    # (eq, coeff, powers per component)
    exact: Callable[[np.ndarray], np.ndarray]               # u*(x) -> [npts, ncomp]
    test_x: np.ndarray                 # [ntest, dim] points for the relative L2 error
    test_owner: np.ndarray             # [ntest] int32
    params: dict = field(default_factory=dict)
    fn_terms: List[Tuple[int, int, float, str]] = field(default_factory=list)  # (eq, comp, coeff, function)
    # (eq, coeff, ((comp, deriv, power), ...)): coeff times the product of derivatives of the field
    prod_terms: List[Tuple[int, float, Tuple[Tuple[int, int, int], ...]]] = field(default_factory=list)
    # partition of unity (Sec. 2.2): "a" indicator of each box (with continuity rows), "b" the smooth
    # tensor-product bump of support 5/4 of each box's half-width (no continuity rows)
    pou: str = "a"

    @property
    def nbox(self) -> int:
        return int(np.prod(self.nsub))

    @property
    def n(self) -> int:
        return self.nbox * self.ncomp * self.J

    @property
    def neq(self) -> int:
        return self.ncomp

    def group_rows(self, g: PointGroup) -> int:
        if g.kind == KIND_PDE:
            return g.npts * (self.neq if g.comp < 0 else 1)
        nc = self.ncomp if g.comp < 0 else 1
        if g.kind == KIND_CONTINUITY:
            return g.npts * nc * g.cont_order
        return g.npts * nc

    @property
    def m(self) -> int:
        return int(sum(self.group_rows(g) for g in self.groups))


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------

def box_index(multi: Sequence[int], nsub: Sequence[int]) -> int:
    e, stride = 0, 1
    for a, i in enumerate(multi):
        e += int(i) * stride
        stride *= int(nsub[a])
    return e


def box_multi(e: int, nsub: Sequence[int]) -> Tuple[int, ...]:
    out = []
    for a in range(len(nsub)):
        out.append(e % int(nsub[a]))
        e //= int(nsub[a])
    return tuple(out)


def box_bounds(e: int, lo, hi, nsub) -> Tuple[np.ndarray, np.ndarray]:
    mi = box_multi(e, nsub)
    h = (np.asarray(hi, float) - np.asarray(lo, float)) / np.asarray(nsub, float)
    blo = np.asarray(lo, float) + np.asarray(mi, float) * h
    return blo, blo + h


def tensor_grid(axes: Sequence[np.ndarray]) -> np.ndarray:
    """Cartesian product of 1-D point sets, first axis varying fastest."""
    mesh = np.meshgrid(*axes[::-1], indexing="ij")
    return np.stack([mm.ravel() for mm in mesh[::-1]], axis=1)


def box_grid(blo, bhi, q: Sequence[int]) -> np.ndarray:
    return tensor_grid([np.linspace(blo[a], bhi[a], q[a]) for a in range(len(q))])


def face_grid(blo, bhi, axis: int, coord: float, qf: int) -> np.ndarray:
    d = len(blo)
    axes = []
    for a in range(d):
        if a == axis:
            axes.append(np.array([coord]))
        else:
            axes.append(np.linspace(blo[a], bhi[a], qf))
    return tensor_grid(axes)


def cell_centres(blo, bhi, per_dim: int) -> np.ndarray:
    axes = []
    for a in range(len(blo)):
        h = (bhi[a] - blo[a]) / per_dim
        axes.append(blo[a] + (np.arange(per_dim) + 0.5) * h)
    return tensor_grid(axes)


def draw_features(seed: int, nbox: int, ncomp: int, J: int, dim: int, R: float):
    """Feature weights then biases, each uniform on [-R, R] (Sec. 2.2)."""
    rng = np.random.default_rng(seed)
    W = rng.uniform(-R, R, size=(nbox, ncomp, J, dim))
    b = rng.uniform(-R, R, size=(nbox, ncomp, J))
    return W, b


# ----------------------------------------------------------------------------
# manufactured solutions: value, gradient, full and spatial Laplacian
# ----------------------------------------------------------------------------

Jet = Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]  # val[n,K], grad[n,K,d], lap[n,K], lap_space[n,K]


def jet_config1(x: np.ndarray) -> Jet:
    X, Y = x[:, 0], x[:, 1]
    pi = math.pi
    sx, sy, cx, cy = np.sin(pi * X), np.sin(pi * Y), np.cos(pi * X), np.cos(pi * Y)
    val = sx * sy + 0.5 * X * Y
    gx = pi * cx * sy + 0.5 * Y
    gy = pi * sx * cy + 0.5 * X
    lap = -2.0 * pi * pi * sx * sy
    return val[:, None], np.stack([gx, gy], 1)[:, None, :], lap[:, None], lap[:, None]


def jet_config2(x: np.ndarray, amp: float = 0.5) -> Jet:
    pi = math.pi
    s = [np.sin(pi * x[:, a]) for a in range(3)]
    c = [np.cos(pi * x[:, a]) for a in range(3)]
    sss = s[0] * s[1] * s[2]
    ccc = c[0] * c[1] * c[2]
    u = 1.0 - amp * sss
    v = 0.25 * ccc
    gu = np.stack([-amp * pi * c[0] * s[1] * s[2], -amp * pi * s[0] * c[1] * s[2], -amp * pi * s[0] * s[1] * c[2]], 1)
    gv = np.stack([-0.25 * pi * s[0] * c[1] * c[2], -0.25 * pi * c[0] * s[1] * c[2], -0.25 * pi * c[0] * c[1] * s[2]], 1)
    lu = 3.0 * pi * pi * amp * sss
    lv = -0.75 * pi * pi * ccc
    val = np.stack([u, v], 1)
    grad = np.stack([gu, gv], 1)
    lap = np.stack([lu, lv], 1)
    return val, grad, lap, lap


def jet_config3(x: np.ndarray, kappa: float = 8.0) -> Jet:
    w = kappa / math.sqrt(3.0)
    s = [np.sin(w * x[:, a]) for a in range(3)]
    c = [np.cos(w * x[:, a]) for a in range(3)]
    val = s[0] * s[1] * s[2]
    grad = np.stack([w * c[0] * s[1] * s[2], w * s[0] * c[1] * s[2], w * s[0] * s[1] * c[2]], 1)
    lap = -3.0 * w * w * val
    return val[:, None], grad[:, None, :], lap[:, None], lap[:, None]


def jet_config4(x: np.ndarray) -> Jet:
    X, Y, T = x[:, 0], x[:, 1], x[:, 2]
    pi = math.pi
    th = np.tanh((X - 0.3 - 0.4 * T) / 0.1)
    sech2 = 1.0 - th * th
    cy, sy = np.cos(pi * Y), np.sin(pi * Y)
    val = th * cy
    gx = 10.0 * sech2 * cy
    gy = -pi * th * sy
    gt = -4.0 * sech2 * cy
    uxx = -200.0 * th * sech2 * cy
    uyy = -pi * pi * th * cy
    utt = 16.0 * (-2.0 * th * sech2) * cy
    lap_space = uxx + uyy
    lap = lap_space + utt
    return val[:, None], np.stack([gx, gy, gt], 1)[:, None, :], lap[:, None], lap_space[:, None]


def _jet_quantity(jet: Jet, c: int, deriv: int) -> np.ndarray:
    val, grad, lap, lap_space = jet
    if deriv == D_ID:
        return val[:, c]
    if D_X0 <= deriv <= D_X3:
        return grad[:, c, deriv - 1]
    if deriv == D_LAPLACE:
        return lap[:, c]
    if deriv == D_LAPLACE_SPACE:
        return lap_space[:, c]
    raise ValueError(deriv)


def apply_operator_to_jet(jet: Jet, lin_terms, poly_terms, neq: int, fn_terms=(), prod_terms=()) -> np.ndarray:
    """Right-hand side f = P(u*) at the points, one column per equation."""
    val = jet[0]
    n = val.shape[0]
    f = np.zeros((n, neq))
    for (q, c, coeff, deriv) in lin_terms:
        f[:, q] += coeff * _jet_quantity(jet, c, deriv)
    for (q, coeff, pw) in poly_terms:
        term = np.ones(n)
        for c, p in enumerate(pw):
            if p:
                term = term * val[:, c] ** p
        f[:, q] += coeff * term
    for (q, c, coeff, fn) in fn_terms:
        f[:, q] += coeff * _FN_VALUE[fn](val[:, c])
    for (q, coeff, facs) in prod_terms:
        term = np.full(n, coeff)
        for (c, deriv, p) in facs:
            term = term * _jet_quantity(jet, c, deriv) ** p
        f[:, q] += term
    return f


# ----------------------------------------------------------------------------
# generic box-partition builder
# ----------------------------------------------------------------------------

def _build(name, dim, ncomp, lo, hi, nsub, J, R, q_int, q_face, jet_fn, lin_terms, poly_terms,
           seed=0, dirichlet_faces=None, test_per_dim=None, inside=None, extra_groups=None,
           params=None, fn_terms=(), prod_terms=(), pou="a"):
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    nsub = np.asarray(nsub, np.int64)
    nbox = int(np.prod(nsub))
    W, b = draw_features(seed, nbox, ncomp, J, dim, R)
    exact = lambda x: jet_fn(x)[0]
    groups: List[PointGroup] = []
    keep = (lambda p: np.ones(p.shape[0], bool)) if inside is None else inside

    # PDE groups, box by box
    for e in range(nbox):
        blo, bhi = box_bounds(e, lo, hi, nsub)
        pts = box_grid(blo, bhi, [q_int] * dim)
        pts = pts[keep(pts)]
        if pts.shape[0] == 0:
            continue
        f = apply_operator_to_jet(jet_fn(pts), lin_terms, poly_terms, ncomp, fn_terms, prod_terms)
        groups.append(PointGroup(KIND_PDE, pts, e, data=f))

    # continuity groups: direction, plane, transverse box (axis 0 fastest); none with the smooth
    # partition of unity, whose blend is already continuously differentiable
    for a in (range(dim) if pou == "a" else ()):
        for p in range(int(nsub[a]) - 1):
            for e in range(nbox):
                mi = box_multi(e, nsub)
                if mi[a] != p:
                    continue
                mj = list(mi)
                mj[a] = p + 1
                e2 = box_index(mj, nsub)
                blo, bhi = box_bounds(e, lo, hi, nsub)
                pts = face_grid(blo, bhi, a, bhi[a], q_face)
                pts = pts[keep(pts)]
                if pts.shape[0] == 0:
                    continue
                nrm = np.zeros_like(pts)
                nrm[:, a] = 1.0
                groups.append(PointGroup(KIND_CONTINUITY, pts, e, neighbor=e2, normal=nrm, comp=-1, cont_order=2))

    # outer faces: x=lo, x=hi, y=lo, y=hi, ...; boxes on the face axis-0 fastest
    faces = dirichlet_faces if dirichlet_faces is not None else [(a, s) for a in range(dim) for s in (0, 1)]
    for (a, side) in faces:
        for e in range(nbox):
            mi = box_multi(e, nsub)
            if mi[a] != (0 if side == 0 else int(nsub[a]) - 1):
                continue
            blo, bhi = box_bounds(e, lo, hi, nsub)
            coord = lo[a] if side == 0 else hi[a]
            pts = face_grid(blo, bhi, a, coord, q_face)
            pts = pts[keep(pts)]
            if pts.shape[0] == 0:
                continue
            g = jet_fn(pts)[0]
            groups.append(PointGroup(KIND_DIRICHLET, pts, e, comp=-1, data=g))

    if extra_groups is not None:
        groups.extend(extra_groups(lo, hi, nsub, jet_fn))

    # relative-L2 test set: cell centres, 2*q_int per axis per box, inside Omega
    tpd = test_per_dim if test_per_dim is not None else 2 * q_int
    tx, to = [], []
    for e in range(nbox):
        blo, bhi = box_bounds(e, lo, hi, nsub)
        pts = cell_centres(blo, bhi, tpd)
        pts = pts[keep(pts)]
        tx.append(pts)
        to.append(np.full(pts.shape[0], e, np.int32))
    return Problem(name=name, dim=dim, ncomp=ncomp, lo=lo, hi=hi, nsub=nsub, J=J, W=W, b=b,
                   groups=groups, lin_terms=list(lin_terms), poly_terms=list(poly_terms),
                   exact=exact, test_x=np.concatenate(tx), test_owner=np.concatenate(to),
                   params=dict(params or {}, seed=seed, R=R, q_int=q_int, q_face=q_face),
                   fn_terms=list(fn_terms), prod_terms=list(prod_terms), pou=pou)


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

def config1(nsub=(2, 2), J=200, q=20, seed=0, R=1.0, test_per_dim=None, pou="a") -> Problem:
    """2-D  -Lap u + u^3 = f on [0,1]^2, u* = sin(pi x) sin(pi y) + x y / 2, Dirichlet."""
    lin = [(0, 0, -1.0, D_LAPLACE)]
    poly = [(0, 1.0, (3,))]
    return _build("poisson_cubic_2d", 2, 1, (0, 0), (1, 1), nsub, J, R, q, q, jet_config1, lin, poly,
                  seed=seed, test_per_dim=test_per_dim, pou=pou)


def jet_line(x: np.ndarray) -> Jet:
    X = x[:, 0]
    pi = math.pi
    val = np.sin(pi * X) + 0.5 * X
    g = pi * np.cos(pi * X) + 0.5
    lap = -pi * pi * np.sin(pi * X)
    return val[:, None], g[:, None, None], lap[:, None], lap[:, None]


def line_1d(nsub=(4,), J=16, q=40, seed=0, R=4.0, test_per_dim=None) -> Problem:
    """1-D  -u'' + u^3 = f on [0, 1], u* = sin(pi x) + x / 2, Dirichlet at both ends: the degenerate
    dimension (faces and interfaces are single points), for edge-case tests."""
    lin = [(0, 0, -1.0, D_LAPLACE)]
    poly = [(0, 1.0, (3,))]
    return _build("poisson_cubic_1d", 1, 1, (0.0,), (1.0,), nsub, J, R, q, q, jet_line, lin, poly,
                  seed=seed, test_per_dim=test_per_dim)


GS_F, GS_K = 0.04, 0.06


def gray_scott_terms(F=GS_F, k=GS_K, Du=1.0, Dv=0.5):
    lin = [(0, 0, -Du, D_LAPLACE), (0, 0, F, D_ID),
           (1, 1, -Dv, D_LAPLACE), (1, 1, F + k, D_ID)]
    # u v^2 enters equation 0 with + and equation 1 with -;  the constant -F of
    # -F(1-u) is carried by the data of equation 0
    poly = [(0, 1.0, (1, 2)), (1, -1.0, (1, 2))]
    return lin, poly


def config2(nsub=(4, 4, 4), J=300, q=10, seed=0, R=1.5, F=GS_F, k=GS_K, amp=0.5,
            test_per_dim=None, pou="a") -> Problem:
    """3-D steady Gray-Scott on the unit cube with a manufactured pair (u*, v*)."""
    lin, poly = gray_scott_terms(F, k)
    jet = lambda x: jet_config2(x, amp)
    return _build("gray_scott_3d", 3, 2, (0, 0, 0), (1, 1, 1), nsub, J, R, q, q, jet, lin, poly,
                  seed=seed, test_per_dim=test_per_dim, params=dict(F=F, k=k, amp=amp), pou=pou)


def config3_nohole(nsub=(8, 8, 8), J=250, q=8, seed=0, R=1.0, test_per_dim=None) -> Problem:
    """3-D nonlinear Helmholtz  -Lap u - kappa^2 u + u^3 = f  (kappa = 8) on the full cube."""
    kap = 8.0
    lin = [(0, 0, -1.0, D_LAPLACE), (0, 0, -kap * kap, D_ID)]
    poly = [(0, 1.0, (3,))]
    return _build("helmholtz_3d", 3, 1, (0, 0, 0), (1, 1, 1), nsub, J, R, q, q, jet_config3, lin, poly,
                  seed=seed, test_per_dim=test_per_dim)


def config4_nohole(nsub=(4, 4, 8), J=400, q=12, seed=0, R=1.0, test_per_dim=None) -> Problem:
    """Space-time Allen-Cahn u_t - 0.01 Lap u - u + u^3 = f on [0,1]^2 x [0,1].

    Time is the last coordinate (Sec. 2.1): the initial condition is a Dirichlet
    face at t = 0 and there is no row at t = 1.
    """
    lin = [(0, 0, 1.0, D_X2), (0, 0, -0.01, D_LAPLACE_SPACE), (0, 0, -1.0, D_ID)]
    poly = [(0, 1.0, (3,))]
    faces = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0)]
    return _build("allen_cahn_st", 3, 1, (0, 0, 0), (1, 1, 1), nsub, J, R, q, q, jet_config4, lin, poly,
                  seed=seed, dirichlet_faces=faces, test_per_dim=test_per_dim)


# Gray-Scott parameter family for the learned initial guess: F, k of the
# reaction terms and the amplitude a of u* = 1 - a sin(pi x) sin(pi y) sin(pi z)
GS_FAMILY = {"F": (0.02, 0.06), "k": (0.04, 0.07), "amp": (0.3, 0.7)}


def gray_scott_family_draw(seed: int) -> tuple:
    """One (F, k, amp) draw, uniform on the family's ranges."""
    rng = np.random.default_rng(seed)
    return tuple(float(rng.uniform(*GS_FAMILY[key])) for key in ("F", "k", "amp"))


def gray_scott_member(F: float, k: float, amp: float, **kw) -> Problem:
    """A member of the family: the Gray-Scott workload with these parameters;
    partition, features and points depend only on kw (not on F, k, amp)."""
    return config2(F=F, k=k, amp=amp, **kw)


def mlp_params(in_dim: int, width: int, depth: int, out_dim: int, seed: int) -> np.ndarray:
    """Seeded network parameters (Glorot-uniform weights, small random biases),
    packed per layer as W [dout][din] row-major then b [dout]; float32."""
    rng = np.random.default_rng(seed)
    d = [in_dim] + [width] * depth + [out_dim]
    parts = []
    for i, o in zip(d[:-1], d[1:]):
        lim = np.sqrt(6.0 / (i + o))
        parts.append(rng.uniform(-lim, lim, size=o * i))
        parts.append(rng.uniform(-0.1, 0.1, size=o))
    return np.concatenate(parts).astype(np.float32)


# ----------------------------------------------------------------------------
# geometry with holes
# ----------------------------------------------------------------------------

def fibonacci_sphere(c, r, npts: int) -> np.ndarray:
    """npts points spread on the sphere |x - c| = r along the golden-angle spiral."""
    k = np.arange(npts) + 0.5
    z = 1.0 - 2.0 * k / npts
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = np.pi * (3.0 - np.sqrt(5.0)) * np.arange(npts)
    return np.asarray(c, float)[None, :] + r * np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def box_of(x: np.ndarray, lo, hi, nsub) -> np.ndarray:
    """Index of the box containing each point (axis 0 fastest; the upper face belongs to the last box)."""
    lo, hi, nsub = np.asarray(lo, float), np.asarray(hi, float), np.asarray(nsub, np.int64)
    idx = np.floor((x - lo) / (hi - lo) * nsub).astype(np.int64)
    idx = np.clip(idx, 0, nsub - 1)
    e = np.zeros(len(x), np.int64)
    for a in range(len(nsub) - 1, -1, -1):
        e = e * nsub[a] + idx[:, a]
    return e


def draw_spheres(n: int, seed: int, lo, hi, nsub, q: int):
    """Centres ~ U(0.15, 0.85)^3, radii ~ U(0.05, 0.12); a draw is rejected when two spheres come
    within 0.02 of each other or a box would keep no collocation point."""
    rng = np.random.default_rng(seed)
    lo, hi, nsub = np.asarray(lo, float), np.asarray(hi, float), np.asarray(nsub, np.int64)
    while True:
        c = rng.uniform(0.15, 0.85, size=(n, 3))
        r = rng.uniform(0.05, 0.12, size=n)
        ok = all(np.linalg.norm(c[i] - c[j]) >= r[i] + r[j] + 0.02 for i in range(n) for j in range(i + 1, n))
        if ok:
            for e in range(int(np.prod(nsub))):
                blo, bhi = box_bounds(e, lo, hi, nsub)
                pts = box_grid(blo, bhi, [q] * 3)
                if not np.any(np.all(np.linalg.norm(pts[:, None, :] - c[None], axis=2) > r[None], axis=1)):
                    ok = False
                    break
        if ok:
            return c, r


def config3(nsub=(8, 8, 8), J=250, q=8, seed=0, R=1.0, holes=4, hole_seed=0, h=None,
            test_per_dim=None) -> Problem:
    """3-D nonlinear Helmholtz on the unit cube minus seeded spherical holes, Dirichlet u* on the
    outer faces and on the sphere surfaces (Fibonacci points, ceil(64 * 4 pi r^2 / h^2) per sphere)."""
    kap = 8.0
    lin = [(0, 0, -1.0, D_LAPLACE), (0, 0, -kap * kap, D_ID)]
    poly = [(0, 1.0, (3,))]
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    c, r = draw_spheres(holes, hole_seed, lo, hi, nsub, q)
    h = h if h is not None else 1.0 / 8.0

    def inside(p):
        return np.all(np.linalg.norm(p[:, None, :] - c[None], axis=2) > r[None], axis=1)

    def spheres(lo_, hi_, nsub_, jet_fn):
        out = []
        for ci, ri in zip(c, r):
            x = fibonacci_sphere(ci, ri, int(np.ceil(64 * 4 * np.pi * ri * ri / (h * h))))
            owner = box_of(x, lo_, hi_, nsub_)
            for e in np.unique(owner):
                pts = x[owner == e]
                out.append(PointGroup(KIND_DIRICHLET, pts, int(e), comp=-1, data=jet_fn(pts)[0]))
        return out

    return _build("helmholtz_3d_holes", 3, 1, lo, hi, nsub, J, R, q, q, jet_config3, lin, poly, seed=seed,
                  test_per_dim=test_per_dim, inside=inside, extra_groups=spheres,
                  params=dict(centres=c, radii=r))


AC_HOLE_R = 0.15


def ac_hole_centre(t):
    t = np.asarray(t, float)
    return np.stack([0.5 + 0.25 * np.cos(2 * np.pi * t), 0.5 + 0.25 * np.sin(2 * np.pi * t)], axis=-1)


def config4(nsub=(4, 4, 8), J=400, q=12, seed=0, R=1.0, n_t=96, n_theta=48, test_per_dim=None) -> Problem:
    """Space-time Allen-Cahn on [0,1]^2 x [0,1] minus a moving disc of radius 0.15 centred at
    (0.5 + 0.25 cos 2 pi t, 0.5 + 0.25 sin 2 pi t): Dirichlet u* on the x, y faces and at t = 0,
    Neumann n . grad u* on the hole (n pointing out of the domain, into the hole), n_t cell-centred
    t levels x n_theta angles."""
    lin = [(0, 0, 1.0, D_X2), (0, 0, -0.01, D_LAPLACE_SPACE), (0, 0, -1.0, D_ID)]
    poly = [(0, 1.0, (3,))]
    faces = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0)]
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)

    def inside(p):
        return np.linalg.norm(p[:, :2] - ac_hole_centre(p[:, 2]), axis=1) > AC_HOLE_R

    def hole(lo_, hi_, nsub_, jet_fn):
        t = (np.arange(n_t) + 0.5) / n_t
        th = 2 * np.pi * np.arange(n_theta) / n_theta
        tt, aa = np.meshgrid(t, th, indexing="ij")
        tt, aa = tt.ravel(), aa.ravel()
        cen = ac_hole_centre(tt)
        dirs = np.stack([np.cos(aa), np.sin(aa)], axis=1)
        x = np.concatenate([cen + AC_HOLE_R * dirs, tt[:, None]], axis=1)
        nrm = np.concatenate([-dirs, np.zeros((len(tt), 1))], axis=1)
        owner = box_of(x, lo_, hi_, nsub_)
        out = []
        for e in np.unique(owner):
            sel = owner == e
            pts, nn = x[sel], nrm[sel]
            g = np.einsum("pcd,pd->pc", jet_fn(pts)[1], nn)
            out.append(PointGroup(KIND_NEUMANN, pts, int(e), normal=nn, comp=-1, data=g))
        return out

    return _build("allen_cahn_st_hole", 3, 1, lo, hi, nsub, J, R, q, q, jet_config4, lin, poly, seed=seed,
                  dirichlet_faces=faces, test_per_dim=test_per_dim, inside=inside, extra_groups=hole)


def jet_ac_paper(x: np.ndarray) -> Jet:
    """u* = 2 sin(x(1 - x)) sin(y(1 - y)) e^(t + 1) (time the last coordinate): value, gradient in
    (x, y, t), Laplacian in (x, y, t) and in (x, y)."""
    X, Y, T = x[:, 0], x[:, 1], x[:, 2]

    def a(s):
        w = s * (1.0 - s)
        return np.sin(w), np.cos(w) * (1.0 - 2.0 * s), -np.sin(w) * (1.0 - 2.0 * s) ** 2 - 2.0 * np.cos(w)

    ax, dax, d2ax = a(X)
    ay, day, d2ay = a(Y)
    et = 2.0 * np.exp(T + 1.0)
    val = ax * ay * et
    grad = np.stack([dax * ay * et, ax * day * et, val], 1)
    lap_space = (d2ax * ay + ax * d2ay) * et
    return val[:, None], grad[:, None, :], (lap_space + val)[:, None], lap_space[:, None]


AC2_HOLE_R = 0.1


def ac2_hole_centre(t):
    t = np.asarray(t, float)
    return np.stack([0.5 + 0.2 * np.cos(np.pi * t), 0.5 + 0.2 * np.sin(np.pi * t)], axis=-1)


def allen_cahn_moving_hole(nsub=(2, 2, 2), J=400, q=20, seed=0, R=1.0, n_t=None, n_theta=None,
                           test_per_dim=None) -> Problem:
    """The paper's space-time Allen-Cahn problem on a domain with a moving hole (Sec. 6.3):
    u_t - Lap u + u^3 - u = f on ([0,1]^2 minus a disc of radius 0.1 centred at
    (0.5 + 0.2 cos(pi t), 0.5 + 0.2 sin(pi t))) x (0, 1], u* = 2 sin(x(1 - x)) sin(y(1 - y)) e^(t+1);
    Dirichlet u* on the x, y faces, at t = 0 and on the hole's boundary (n_t cell-centred t levels x
    n_theta angles, by default q per box along t and 4 q around)."""
    lin = [(0, 0, 1.0, D_X2), (0, 0, -1.0, D_LAPLACE_SPACE), (0, 0, -1.0, D_ID)]
    poly = [(0, 1.0, (3,))]
    faces = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0)]
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    n_t = n_t if n_t is not None else q * int(nsub[2])
    n_theta = n_theta if n_theta is not None else 4 * q

    def inside(p):
        return np.linalg.norm(p[:, :2] - ac2_hole_centre(p[:, 2]), axis=1) > AC2_HOLE_R

    def hole(lo_, hi_, nsub_, jet_fn):
        t = (np.arange(n_t) + 0.5) / n_t
        th = 2 * np.pi * np.arange(n_theta) / n_theta
        tt, aa = np.meshgrid(t, th, indexing="ij")
        tt, aa = tt.ravel(), aa.ravel()
        x = np.concatenate([ac2_hole_centre(tt) + AC2_HOLE_R * np.stack([np.cos(aa), np.sin(aa)], 1), tt[:, None]],
                           axis=1)
        owner = box_of(x, lo_, hi_, nsub_)
        return [PointGroup(KIND_DIRICHLET, x[owner == e], int(e), comp=-1, data=jet_fn(x[owner == e])[0])
                for e in np.unique(owner)]

    return _build("allen_cahn_moving_hole_paper", 3, 1, lo, hi, nsub, J, R, q, q, jet_ac_paper, lin, poly,
                  seed=seed, dirichlet_faces=faces, test_per_dim=test_per_dim, inside=inside, extra_groups=hole)


def make_config(i: int, **kw) -> Problem:
    return [config1, config2, config3_nohole, config4_nohole][i](**kw)


def jet_helmholtz_cosh(x: np.ndarray) -> Jet:
    """u* = (2 + |x|^2) sin(pi x) sin(pi y) sin(pi z), its gradient and Laplacian."""
    pi = math.pi
    s = [np.sin(pi * x[:, a]) for a in range(3)]
    c = [np.cos(pi * x[:, a]) for a in range(3)]
    S = s[0] * s[1] * s[2]
    dS = np.stack([pi * c[0] * s[1] * s[2], pi * s[0] * c[1] * s[2], pi * s[0] * s[1] * c[2]], 1)
    p = 2.0 + (x[:, :3] ** 2).sum(1)
    val = p * S
    grad = 2.0 * x[:, :3] * S[:, None] + p[:, None] * dS
    lap = 6.0 * S + 4.0 * (x[:, :3] * dS).sum(1) - 3.0 * pi * pi * p * S
    return val[:, None], grad[:, None, :], lap[:, None], lap[:, None]


def helmholtz_cosh(nsub=(2, 2, 2), J=400, q=20, seed=0, R=1.0, test_per_dim=None, pou="a") -> Problem:
    """3-D nonlinear Helmholtz with a cosh term on the unit cube (the paper's IPN / AMIPN comparison,
    Sec. 6.2): Lap u - 100 u + 10 cosh(u) = f, u* = (2 + |x|^2) sin(pi x) sin(pi y) sin(pi z),
    Dirichlet u* on the boundary; q^3 collocation points per box, q x q face and interface grids."""
    lin = [(0, 0, 1.0, D_LAPLACE), (0, 0, -100.0, D_ID)]
    fn = [(0, 0, 10.0, FN_COSH)]
    return _build("helmholtz_cosh_3d", 3, 1, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), nsub, J, R, q, q,
                  jet_helmholtz_cosh, lin, [], seed=seed, test_per_dim=test_per_dim, fn_terms=fn, pou=pou)


def jet_quasilinear(x: np.ndarray) -> Jet:
    """u* = (x + y + z) sin(pi x) sin(pi y) cos(pi z), its gradient and Laplacian."""
    pi = math.pi
    sx, sy, sz = (np.sin(pi * x[:, a]) for a in range(3))
    cx, cy, cz = (np.cos(pi * x[:, a]) for a in range(3))
    P = sx * sy * cz
    dP = np.stack([pi * cx * sy * cz, pi * sx * cy * cz, -pi * sx * sy * sz], 1)
    s = x[:, :3].sum(1)
    val = s * P
    grad = P[:, None] + s[:, None] * dP
    lap = -3.0 * pi * pi * s * P + 2.0 * dP.sum(1)
    return val[:, None], grad[:, None, :], lap[:, None], lap[:, None]


def quasilinear_terms():
    """-div((1 + u^2) grad u) = -Lap u - u^2 Lap u - 2 u |grad u|^2: one linear and four product terms."""
    lin = [(0, 0, -1.0, D_LAPLACE)]
    prod = [(0, -1.0, ((0, D_ID, 2), (0, D_LAPLACE, 1)))]
    prod += [(0, -2.0, ((0, D_ID, 1), (0, D_X0 + a, 2))) for a in range(3)]
    return lin, prod


def quasilinear(nsub=(2, 2, 2), J=800, q=20, seed=0, R=1.0, test_per_dim=None, pou="a") -> Problem:
    """3-D quasi-linear elliptic benchmark of the paper (Sec. 3.2 and the AMIPN table of Sec. 6.2):
    -div((1 + u^2) grad u) = f on the unit cube, u* = (x + y + z) sin(pi x) sin(pi y) cos(pi z),
    Dirichlet u* on the boundary; q^3 collocation points per box, q x q face and interface grids."""
    lin, prod = quasilinear_terms()
    return _build("quasilinear_3d", 3, 1, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), nsub, J, R, q, q,
                  jet_quasilinear, lin, [], seed=seed, test_per_dim=test_per_dim, prod_terms=prod, pou=pou)


def jet_ball(x: np.ndarray) -> Jet:
    """u* = (x^2 + y^2 + z^2) sin(pi x) sin(pi y) sin(pi z), its gradient and Laplacian."""
    pi = math.pi
    s = [np.sin(pi * x[:, a]) for a in range(3)]
    c = [np.cos(pi * x[:, a]) for a in range(3)]
    S = s[0] * s[1] * s[2]
    dS = np.stack([pi * c[0] * s[1] * s[2], pi * s[0] * c[1] * s[2], pi * s[0] * s[1] * c[2]], 1)
    p = (x[:, :3] ** 2).sum(1)
    val = p * S
    grad = 2.0 * x[:, :3] * S[:, None] + p[:, None] * dS
    lap = 6.0 * S + 4.0 * (x[:, :3] * dS).sum(1) - 3.0 * pi * pi * p * S
    return val[:, None], grad[:, None, :], lap[:, None], lap[:, None]


def diffusion_reaction_ball(nsub=(2, 2, 2), J=400, q=30, nbdy=30000, seed=0, R=1.0, test_per_dim=None) -> Problem:
    """3-D steady diffusion-reaction on the unit ball (the paper's AMIPN example of Sec. 6.2):
    -div((1 + u^2) grad u) + (u^3 - u) + e^u = f, u* = (x^2 + y^2 + z^2) sin(pi x) sin(pi y) sin(pi z).
    The ball sits in [-1, 1]^3, split into nsub boxes; the q^3 grid points of each box and the q x q
    interface grids are kept where x^2 + y^2 + z^2 < 1; Dirichlet u* at nbdy Fibonacci points of the
    unit sphere, each owned by the box that holds it (no rows on the faces of the cube)."""
    lin, prod = quasilinear_terms()
    lin = lin + [(0, 0, -1.0, D_ID)]
    poly = [(0, 1.0, (3,))]
    fn = [(0, 0, 1.0, FN_EXP)]
    lo, hi = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)

    def inside(p):
        return (p[:, :3] ** 2).sum(1) < 1.0

    def sphere(lo_, hi_, nsub_, jet_fn):
        x = fibonacci_sphere(np.zeros(3), 1.0, nbdy)
        owner = box_of(x, lo_, hi_, nsub_)
        return [PointGroup(KIND_DIRICHLET, x[owner == e], int(e), comp=-1, data=jet_fn(x[owner == e])[0])
                for e in np.unique(owner)]

    return _build("diffusion_reaction_ball", 3, 1, lo, hi, nsub, J, R, q, q, jet_ball, lin, poly, seed=seed,
                  dirichlet_faces=[], test_per_dim=test_per_dim, inside=inside, extra_groups=sphere,
                  fn_terms=fn, prod_terms=prod)


def jet_gray_scott_nonlinear(x: np.ndarray) -> Jet:
    """u* = sin(x(1 - x)) sin(y(1 - y)) e^z and v* = sin(pi x) sin(pi y) sin(pi z): values [P, 2],
    gradients [P, 2, 3] and Laplacians [P, 2]."""
    pi = math.pi
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]

    def a(t):
        w = t * (1.0 - t)
        return np.sin(w), np.cos(w) * (1.0 - 2.0 * t), -np.sin(w) * (1.0 - 2.0 * t) ** 2 - 2.0 * np.cos(w)

    ax, dax, d2ax = a(X)
    ay, day, d2ay = a(Y)
    ez = np.exp(Z)
    u = ax * ay * ez
    gu = np.stack([dax * ay * ez, ax * day * ez, u], 1)
    lu = (d2ax * ay + ax * d2ay + ax * ay) * ez
    s = [np.sin(pi * x[:, k]) for k in range(3)]
    c = [np.cos(pi * x[:, k]) for k in range(3)]
    v = s[0] * s[1] * s[2]
    gv = pi * np.stack([c[0] * s[1] * s[2], s[0] * c[1] * s[2], s[0] * s[1] * c[2]], 1)
    lv = -3.0 * pi * pi * v
    val = np.stack([u, v], 1)
    grad = np.stack([gu, gv], 1)
    lap = np.stack([lu, lv], 1)
    return val, grad, lap, lap


GS2_F, GS2_K = 0.060, 0.062


def gray_scott_nonlinear(nsub=(2, 2, 2), J=400, q=20, seed=0, R=1.0, F=GS2_F, k=GS2_K, test_per_dim=None) -> Problem:
    """The paper's steady Gray-Scott system with solution-dependent diffusion (Sec. 6.2):
    (1 + u^2) Lap u - u v^2 + F (1 - u) = f1, (1 + v^2) Lap v + u v^2 - (F + k) v = f2 on the unit cube,
    u* = sin(x(1 - x)) sin(y(1 - y)) e^z, v* = sin(pi x) sin(pi y) sin(pi z), Dirichlet u*, v*; the
    constant F of the first equation is carried by the data."""
    lin = [(0, 0, 1.0, D_LAPLACE), (0, 0, -F, D_ID), (1, 1, 1.0, D_LAPLACE), (1, 1, -(F + k), D_ID)]
    poly = [(0, -1.0, (1, 2)), (1, 1.0, (1, 2))]
    prod = [(0, 1.0, ((0, D_ID, 2), (0, D_LAPLACE, 1))), (1, 1.0, ((1, D_ID, 2), (1, D_LAPLACE, 1)))]
    return _build("gray_scott_nonlinear_3d", 3, 2, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), nsub, J, R, q, q,
                  jet_gray_scott_nonlinear, lin, poly, seed=seed, test_per_dim=test_per_dim,
                  prod_terms=prod, params=dict(F=F, k=k))


def jet_of(problem: Problem):
    """Closed-form jet of the problem's manufactured solution."""
    name = problem.name
    if name == "allen_cahn_moving_hole_paper":
        return jet_ac_paper
    if name == "gray_scott_nonlinear_3d":
        return jet_gray_scott_nonlinear
    if name == "diffusion_reaction_ball":
        return jet_ball
    if name == "quasilinear_3d":
        return jet_quasilinear
    if name == "helmholtz_cosh_3d":
        return jet_helmholtz_cosh
    if name == "poisson_cubic_2d":
        return jet_config1
    if name == "gray_scott_3d":
        return lambda x: jet_config2(x, problem.params.get("amp", 0.5))
    if name in ("helmholtz_3d", "helmholtz_3d_holes"):
        return jet_config3
    if name in ("allen_cahn_st", "allen_cahn_st_hole"):
        return jet_config4
    raise KeyError(name)
