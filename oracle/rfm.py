"""Plain CPU FP64 oracle of the randomized inexact preconditioned Newton solvers
(IPN, Alg. 1, and AMIPN, Alg. 2) for random-feature-method discretisations.

TEST INFRASTRUCTURE ONLY.  Imported by tests/, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``; the product library never imports, links
or calls anything here, and nothing here imports the product package.

Everything is dense numpy in float64, written for a reader to check against
the paper by eye; there is no blocking, fusion or reordering beyond what each
formula states.  Inputs come from ``rfm_workloads`` (problem description only).

Readings taken where the paper is silent:
 * rows: each point group expands to rows ordered (equation or component,
   continuity order, point); groups keep their listed order, which is
   [PDE; continuity; boundary] as in Alg. 3 step 4;
 * continuity order s uses the s-th derivative along the interface normal
   (eqs. con:1-3), lower box minus upper box;
 * row scale: c / max_j |J_ij| with c = 100 (Sec. 5), a zero row keeps scale 1;
   the scale is recomputed at each Jacobian evaluation and frozen for the
   line searches, stop tests and AMIPN inner steps that use that Jacobian;
 * sketch: Gaussian S with N(0, 1/s) entries from Philox (oracle.philox),
   s = ceil(gamma * n), a fresh key per Jacobian evaluation;
 * R: the R factor of S*D*J with a positive diagonal; a zero or non-finite
   diagonal entry means the preconditioner does not exist;
 * LSQR: Paige-Saunders stopping rules 1 and 2 with atol = btol = eta, no
   condition-number limit, zero start;
 * line search: the full step is accepted when it lowers ||D F|| by the factor
   (1 - 1e-4); otherwise a golden-section search on [0, 1] with a fixed number
   of iterations returns the evaluated step with the smallest ||D F|| (ties to
   the larger step); a step is taken only if it lowers ||D F||;
 * stop test: | ||D F(u_{k+1})|| - ||D F(u_k)|| | < eps under the scale of the
   current Jacobian, or ||D F|| = 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg

from rfm_workloads import (box_multi, KIND_CONTINUITY, KIND_DIRICHLET, KIND_NEUMANN, KIND_PDE, D_ID, D_LAPLACE,
                           D_LAPLACE_SPACE, D_X0, D_X3, Problem, box_bounds)
from . import lowprec, philox

# ---------------------------------------------------------------------------
# features (Sec. 2.2): phi_ij(x) = tanh(k_ij . l_i(x) + b_ij), l_i(x) = (x - mu_i)/sigma_i
# ---------------------------------------------------------------------------


def box_centre_radius(prob: Problem, e: int):
    lo, hi = box_bounds(e, prob.lo, prob.hi, prob.nsub)
    return 0.5 * (lo + hi), 0.5 * (hi - lo)


def feature_jet(prob: Problem, e: int, c: int, x: np.ndarray):
    """Values, gradients and pure second derivatives of the J features of
    (box e, component c) at points x.  Returns phi [n,J], dphi [n,J,d], d2phi [n,J,d].

    With t = tanh(z), z = sum_a w_a (x_a - mu_a)/sigma_a + b:
      d phi / d x_a   = (1 - t^2) w_a / sigma_a
      d2 phi / d x_a^2 = -2 t (1 - t^2) (w_a / sigma_a)^2
    """
    mu, sig = box_centre_radius(prob, e)
    W = prob.W[e, c]            # [J, d]
    b = prob.b[e, c]            # [J]
    l = (x - mu) / sig          # [n, d]
    z = l @ W.T + b             # [n, J]
    t = np.tanh(z)
    dt = 1.0 - t * t
    ws = W / sig                # [J, d]
    dphi = dt[:, :, None] * ws[None, :, :]
    d2phi = (-2.0 * t * dt)[:, :, None] * (ws * ws)[None, :, :]
    return t, dphi, d2phi


# ---------------------------------------------------------------------------
# smooth partition of unity (Sec. 2.2): psi_e(x) = prod_a varphi^b(l_a(x)), l the box's affine map
# to [-1, 1]^d; varphi^b = 1 on |y| <= 3/4, (1 - sin(2 pi |y|)) / 2 on 3/4 <= |y| <= 5/4, 0 beyond
# ---------------------------------------------------------------------------

def bump_b(y: np.ndarray):
    """varphi^b(y) and its first and second derivatives."""
    a = np.abs(y)
    band = (a > 0.75) & (a < 1.25)
    f = np.where(a <= 0.75, 1.0, np.where(band, 0.5 * (1.0 - np.sin(2.0 * np.pi * a)), 0.0))
    d1 = np.where(band, -np.pi * np.cos(2.0 * np.pi * a) * np.sign(y), 0.0)
    d2 = np.where(band, 2.0 * np.pi ** 2 * np.sin(2.0 * np.pi * a), 0.0)
    return f, d1, d2


def pou_b(prob: Problem, e: int, x: np.ndarray):
    """psi_e [n], its gradient [n, d] and pure second derivatives [n, d] at x.  On an axis where the box
    touches the boundary of the domain the bump is 1 on the side facing it, so that the functions sum to
    1 on the whole domain (the tensor-product bumps alone sum to 1/2 on the boundary)."""
    mu, sig = box_centre_radius(prob, e)
    y = (x - mu) / sig
    f, d1, d2 = bump_b(y)
    d = x.shape[1]
    idx = box_multi(e, prob.nsub)
    for a in range(d):
        flat = ((idx[a] == 0) & (y[:, a] < 0)) | ((idx[a] == prob.nsub[a] - 1) & (y[:, a] > 0))
        f[flat, a], d1[flat, a], d2[flat, a] = 1.0, 0.0, 0.0
    psi = np.prod(f, axis=1)
    g = np.zeros_like(x)
    h = np.zeros_like(x)
    for a in range(d):
        others = np.prod(np.delete(f, a, axis=1), axis=1)
        g[:, a] = d1[:, a] / sig[a] * others
        h[:, a] = d2[:, a] / sig[a] ** 2 * others
    return psi, g, h


def in_support_b(prob: Problem, e: int, x: np.ndarray) -> np.ndarray:
    """Points strictly inside the support of psi_e (|l_a(x)| < 5/4 on every axis)."""
    mu, sig = box_centre_radius(prob, e)
    return np.all(np.abs((x - mu) / sig) < 1.25, axis=1)


def blended_jet(prob: Problem, e: int, c: int, x: np.ndarray):
    """psi_e phi of the J features of (e, c): values [n,J], gradients [n,J,d], pure second derivatives
    [n,J,d] by the product rule (d_a (psi phi) = psi d_a phi + phi d_a psi,
    d_aa (psi phi) = psi d_aa phi + 2 d_a psi d_a phi + phi d_aa psi)."""
    phi, dphi, d2phi = feature_jet(prob, e, c, x)
    psi, g, h = pou_b(prob, e, x)
    v = psi[:, None] * phi
    dv = psi[:, None, None] * dphi + phi[:, :, None] * g[:, None, :]
    d2v = psi[:, None, None] * d2phi + 2.0 * g[:, None, :] * dphi + phi[:, :, None] * h[:, None, :]
    return v, dv, d2v


def covering_boxes(prob: Problem, x: np.ndarray) -> List[int]:
    """Boxes whose smooth partition function is non-zero at some of the points x."""
    return [e for e in range(prob.nbox) if in_support_b(prob, e, x).any()]


def apply_deriv(prob: Problem, deriv: int, phi, dphi, d2phi):
    """Linear derivative selector applied to feature (or field) jets."""
    if deriv == D_ID:
        return phi
    if D_X0 <= deriv <= D_X3:
        return dphi[..., deriv - 1]
    if deriv == D_LAPLACE:
        return d2phi.sum(-1)
    if deriv == D_LAPLACE_SPACE:
        return d2phi[..., : prob.dim - 1].sum(-1)
    raise ValueError(deriv)


def col_slice(prob: Problem, e: int, c: int) -> slice:
    """Unknowns are ordered [box][component][feature] (the expansion of Sec. 2.2)."""
    start = (e * prob.ncomp + c) * prob.J
    return slice(start, start + prob.J)


# ---------------------------------------------------------------------------
# residual and Jacobian (Alg. 3 steps 1-4 and the Jacobian that follows it)
# ---------------------------------------------------------------------------


# f and f' of the pointwise terms coeff * f(u_c) (the paper's cosh nonlinearity, Sec. 6.2)
_FN = {"cosh": (np.cosh, np.sinh), "sinh": (np.sinh, np.cosh), "exp": (np.exp, np.exp)}


def _comps(prob: Problem, g) -> List[int]:
    return list(range(prob.ncomp)) if g.comp < 0 else [g.comp]


def _group_F_J_pou_b(prob: Problem, g, u: np.ndarray, with_J: bool):
    """group_F_J with the smooth partition of unity: u_n(x) = sum_e psi_e(x) sum_j phi_ej(x) u_ej over
    the boxes whose support holds x, each of their columns getting psi_e phi (and its derivatives)."""
    if g.kind == KIND_CONTINUITY:
        raise ValueError("no continuity rows with the smooth partition of unity")
    n, x = prob.n, g.x
    boxes = covering_boxes(prob, x)
    jets = {e: [blended_jet(prob, e, c, x) for c in range(prob.ncomp)] for e in boxes}
    coef = {e: [u[col_slice(prob, e, c)] for c in range(prob.ncomp)] for e in boxes}

    def field(c, deriv):
        return sum(apply_deriv(prob, deriv, *jets[e][c]) @ coef[e][c] for e in boxes)

    def add_J(Jq, c, deriv, w):
        for e in boxes:
            Jq[:, col_slice(prob, e, c)] += w[:, None] * apply_deriv(prob, deriv, *jets[e][c])

    Fs, Js = [], []
    if g.kind == KIND_PDE:
        val = [field(c, D_ID) for c in range(prob.ncomp)]
        for q in _comps(prob, g):
            Fq = -g.data[:, q].copy() if g.comp < 0 else -g.data[:, 0].copy()
            Jq = np.zeros((g.npts, n)) if with_J else None
            for (eq, c, coeff, deriv) in prob.lin_terms:
                if eq != q:
                    continue
                Fq += coeff * field(c, deriv)
                if with_J:
                    add_J(Jq, c, deriv, np.full(g.npts, coeff))
            for (eq, coeff, pw) in prob.poly_terms:
                if eq != q:
                    continue
                prod = np.ones(g.npts)
                for c, p in enumerate(pw):
                    prod = prod * val[c] ** p
                Fq += coeff * prod
                if with_J:
                    for c, p in enumerate(pw):
                        if p == 0:
                            continue
                        dprod = p * val[c] ** (p - 1)
                        for c2, p2 in enumerate(pw):
                            if c2 != c:
                                dprod = dprod * val[c2] ** p2
                        add_J(Jq, c, D_ID, coeff * dprod)
            for (eq, c, coeff, fn) in getattr(prob, "fn_terms", ()):
                if eq != q:
                    continue
                f, df = _FN[fn]
                Fq += coeff * f(val[c])
                if with_J:
                    add_J(Jq, c, D_ID, coeff * df(val[c]))
            for (eq, coeff, facs) in getattr(prob, "prod_terms", ()):
                if eq != q:
                    continue
                vk = [field(c, d) for (c, d, p) in facs]
                term = np.full(g.npts, coeff)
                for k, (c, d, p) in enumerate(facs):
                    term = term * vk[k] ** p
                Fq += term
                if with_J:
                    for k, (c, d, p) in enumerate(facs):
                        dk = coeff * p * vk[k] ** (p - 1)
                        for k2, (c2, d2, p2) in enumerate(facs):
                            if k2 != k:
                                dk = dk * vk[k2] ** p2
                        add_J(Jq, c, d, dk)
            Fs.append(Fq)
            Js.append(Jq)
    else:  # Dirichlet or Neumann
        for k, c in enumerate(_comps(prob, g)):
            F = -g.data[:, k].copy()
            Jr = np.zeros((g.npts, n)) if with_J else None
            for e in boxes:
                v, dv, _ = jets[e][c]
                op = v if g.kind == KIND_DIRICHLET else np.einsum("pjd,pd->pj", dv, g.normal)
                F += op @ coef[e][c]
                if with_J:
                    Jr[:, col_slice(prob, e, c)] = op
            Fs.append(F)
            Js.append(Jr)
    return Fs, Js


def group_F_J(prob: Problem, g, u: np.ndarray, with_J: bool = True):
    """Residual rows and dense Jacobian rows [rows, n] of one point group."""
    if getattr(prob, "pou", "a") == "b":
        Fs, Js = _group_F_J_pou_b(prob, g, u, with_J)
        return np.concatenate(Fs), (np.concatenate(Js, axis=0) if with_J else None)
    n = prob.n
    x = g.x
    e = g.owner
    jets = [feature_jet(prob, e, c, x) for c in range(prob.ncomp)]
    Fs, Js = [], []
    if g.kind == KIND_PDE:
        # field values and derivatives u_c(x) = sum_j phi_j(x) u_j (piecewise, owner box only)
        coef = [u[col_slice(prob, e, c)] for c in range(prob.ncomp)]
        val = [jets[c][0] @ coef[c] for c in range(prob.ncomp)]
        for q in _comps(prob, g):
            Fq = -g.data[:, q].copy() if g.comp < 0 else -g.data[:, 0].copy()
            Jq = np.zeros((g.npts, n)) if with_J else None
            for (eq, c, coeff, deriv) in prob.lin_terms:
                if eq != q:
                    continue
                D = apply_deriv(prob, deriv, *jets[c])          # [n, J]
                Fq += coeff * (D @ coef[c])
                if with_J:
                    Jq[:, col_slice(prob, e, c)] += coeff * D
            for (eq, coeff, pw) in prob.poly_terms:
                if eq != q:
                    continue
                prod = np.ones(g.npts)
                for c, p in enumerate(pw):
                    prod = prod * val[c] ** p
                Fq += coeff * prod
                if with_J:
                    for c, p in enumerate(pw):
                        if p == 0:
                            continue
                        dprod = p * val[c] ** (p - 1)
                        for c2, p2 in enumerate(pw):
                            if c2 != c:
                                dprod = dprod * val[c2] ** p2
                        Jq[:, col_slice(prob, e, c)] += (coeff * dprod)[:, None] * jets[c][0]
            # pointwise functions of one component: coeff f(u_c), derivative coeff f'(u_c) phi
            for (eq, c, coeff, fn) in getattr(prob, "fn_terms", ()):
                if eq != q:
                    continue
                f, df = _FN[fn]
                Fq += coeff * f(val[c])
                if with_J:
                    Jq[:, col_slice(prob, e, c)] += (coeff * df(val[c]))[:, None] * jets[c][0]
            # products of field derivatives coeff prod_k (D_k u_{c_k})^{p_k} (a quasi-linear operator
            # written out, e.g. -div((1 + u^2) grad u) = -Lap u - u^2 Lap u - 2 u |grad u|^2); by the
            # product rule the derivative by the coefficients of c_k is
            # coeff p_k (D_k u)^{p_k - 1} (the other factors) D_k phi, summed over the factors
            for (eq, coeff, facs) in getattr(prob, "prod_terms", ()):
                if eq != q:
                    continue
                Dk = [apply_deriv(prob, d, *jets[c]) for (c, d, p) in facs]
                vk = [Dk[k] @ coef[c] for k, (c, d, p) in enumerate(facs)]
                term = np.full(g.npts, coeff)
                for k, (c, d, p) in enumerate(facs):
                    term = term * vk[k] ** p
                Fq += term
                if with_J:
                    for k, (c, d, p) in enumerate(facs):
                        dk = coeff * p * vk[k] ** (p - 1)
                        for k2, (c2, d2, p2) in enumerate(facs):
                            if k2 != k:
                                dk = dk * vk[k2] ** p2
                        Jq[:, col_slice(prob, e, c)] += dk[:, None] * Dk[k]
            Fs.append(Fq)
            Js.append(Jq)
    elif g.kind in (KIND_DIRICHLET, KIND_NEUMANN):
        for k, c in enumerate(_comps(prob, g)):
            phi, dphi, _ = jets[c]
            op = phi if g.kind == KIND_DIRICHLET else np.einsum("pjd,pd->pj", dphi, g.normal)
            Fs.append(op @ u[col_slice(prob, e, c)] - g.data[:, k])
            if with_J:
                Jr = np.zeros((g.npts, n))
                Jr[:, col_slice(prob, e, c)] = op
                Js.append(Jr)
    elif g.kind == KIND_CONTINUITY:
        e2 = g.neighbor
        jets2 = [feature_jet(prob, e2, c, x) for c in range(prob.ncomp)]
        for c in _comps(prob, g):
            for s in range(g.cont_order):
                if s == 0:
                    op1, op2 = jets[c][0], jets2[c][0]
                elif s == 1:
                    op1 = np.einsum("pjd,pd->pj", jets[c][1], g.normal)
                    op2 = np.einsum("pjd,pd->pj", jets2[c][1], g.normal)
                else:
                    raise ValueError("continuity order above C1")
                Fs.append(op1 @ u[col_slice(prob, e, c)] - op2 @ u[col_slice(prob, e2, c)])
                if with_J:
                    Jr = np.zeros((g.npts, n))
                    Jr[:, col_slice(prob, e, c)] = op1
                    Jr[:, col_slice(prob, e2, c)] = -op2
                    Js.append(Jr)
    else:
        raise ValueError(g.kind)
    F = np.concatenate(Fs)
    J = np.concatenate(Js, axis=0) if with_J else None
    return F, J


def residual(prob: Problem, u: np.ndarray) -> np.ndarray:
    """F(u) = [R_pde; R_con; R_bdy] (Alg. 3 step 4)."""
    return np.concatenate([group_F_J(prob, g, u, with_J=False)[0] for g in prob.groups])


def assemble(prob: Problem, u: np.ndarray):
    """Residual F(u) [m] and dense Jacobian J(u) [m, n]."""
    Fs, Js = [], []
    for g in prob.groups:
        F, J = group_F_J(prob, g, u)
        Fs.append(F)
        Js.append(J)
    return np.concatenate(Fs), np.concatenate(Js, axis=0)


def group_nrows(prob: Problem, g) -> int:
    """Rows produced by one point group: one per (equation or component,
    continuity order, point)."""
    nsel = prob.ncomp if g.comp < 0 else 1
    if g.kind == KIND_CONTINUITY:
        return g.npts * nsel * g.cont_order
    return g.npts * nsel


def row_table(prob: Problem):
    """(group index, first row) for every group, in row order, and the total m."""
    out, r = [], 0
    for gi, g in enumerate(prob.groups):
        out.append((gi, r))
        r += group_nrows(prob, g)
    return out, r


def assemble_rows(prob: Problem, u: np.ndarray, rows: np.ndarray):
    """F and dense J restricted to the given global rows (for large problems)."""
    rows = np.asarray(rows, np.int64)
    table, m = row_table(prob)
    starts = np.array([r for _, r in table] + [m])
    F = np.zeros(rows.size)
    J = np.zeros((rows.size, prob.n))
    gidx = np.searchsorted(starts, rows, side="right") - 1
    for gi in np.unique(gidx):
        sel = np.nonzero(gidx == gi)[0]
        Fg, Jg = group_F_J(prob, prob.groups[gi], u)
        loc = rows[sel] - starts[gi]
        F[sel] = Fg[loc]
        J[sel] = Jg[loc]
    return F, J


# ---------------------------------------------------------------------------
# row scaling (Sec. 5, lambda_{k,i} = c / max_j |J_ij|)
# ---------------------------------------------------------------------------


def row_scale(J: np.ndarray, c: float = 100.0) -> np.ndarray:
    mx = np.abs(J).max(axis=1)
    return np.where(mx > 0, c / np.where(mx > 0, mx, 1.0), 1.0)


# ---------------------------------------------------------------------------
# preconditioner: sketch, thin QR (Sec. 4.1, Alg. 1 step 2)
# ---------------------------------------------------------------------------


def sketch_rows(prob_n: int, gamma: float) -> int:
    return int(math.ceil(gamma * prob_n))


def sketch(DJ: np.ndarray, s: int, seed: int, jac_index: int) -> np.ndarray:
    S = philox.sketch_matrix(seed, jac_index, s, DJ.shape[0])
    return S @ DJ


class SingularPreconditioner(RuntimeError):
    pass


def qr_r(B: np.ndarray) -> np.ndarray:
    """R of the thin QR B = Q R with diag(R) > 0 (unique for full column rank)."""
    R = np.linalg.qr(B, mode="r")
    d = np.diag(R)
    if not np.all(np.isfinite(d)) or np.any(d == 0):
        raise SingularPreconditioner("zero or non-finite diagonal in R")
    return np.sign(d)[:, None] * R


def r_solve(R: np.ndarray, y: np.ndarray) -> np.ndarray:
    return scipy.linalg.solve_triangular(R, y, lower=False)


def rt_solve(R: np.ndarray, w: np.ndarray) -> np.ndarray:
    return scipy.linalg.solve_triangular(R, w, lower=False, trans="T")


# ---------------------------------------------------------------------------
# LSQR (Paige and Saunders, ACM TOMS 8(1), 1982), zero start, no damping
# ---------------------------------------------------------------------------


@dataclass
class LsqrResult:
    x: np.ndarray
    iters: int
    istop: int          # 1: rule 1 (residual small), 2: rule 2 (normal-eq. residual small), 0: max iters
    rnorm: float
    arnorm: float


def lsqr(matvec, rmatvec, b: np.ndarray, n: int, tol: float, maxit: int) -> LsqrResult:
    """Golub-Kahan bidiagonalisation with the QR update of the bidiagonal.

    Stops when ||r|| <= tol*||b|| + tol*||A||*||x|| (rule 1) or
    ||A^T r|| <= tol*||A||*||r|| (rule 2); ||A|| is the Frobenius estimate
    sqrt(sum alpha_i^2 + beta_i^2) of the bidiagonal built so far.
    """
    x = np.zeros(n)
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return LsqrResult(x, 0, 1, 0.0, 0.0)
    u = b / beta
    v = rmatvec(u)
    alpha = np.linalg.norm(v)
    if alpha == 0.0:
        return LsqrResult(x, 0, 2, beta, 0.0)
    v = v / alpha
    w = v.copy()
    phibar, rhobar = beta, alpha
    bnorm = beta
    anorm2 = 0.0
    istop, itn = 0, 0
    rnorm, arnorm = beta, alpha * beta
    while itn < maxit:
        itn += 1
        u = matvec(v) - alpha * u
        beta = np.linalg.norm(u)
        if beta > 0:
            u = u / beta
        anorm2 += alpha * alpha + beta * beta
        v = rmatvec(u) - beta * v
        alpha = np.linalg.norm(v)
        if alpha > 0:
            v = v / alpha
        rho = math.hypot(rhobar, beta)
        c, s = rhobar / rho, beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        x = x + (phi / rho) * w
        w = v - (theta / rho) * w
        rnorm = phibar
        arnorm = phibar * alpha * abs(c)
        anorm = math.sqrt(anorm2)
        xnorm = np.linalg.norm(x)
        if rnorm <= tol * bnorm + tol * anorm * xnorm:
            istop = 1
            break
        if arnorm <= tol * anorm * rnorm:
            istop = 2
            break
    return LsqrResult(x, itn, istop, rnorm, arnorm)


# ---------------------------------------------------------------------------
# derivative-free golden-section line search (Alg. 1 step 6, Alg. 2, Remark in Sec. 4)
# ---------------------------------------------------------------------------

GOLD = (math.sqrt(5.0) - 1.0) / 2.0


def golden_section(phi, phi0: float, iters: int = 25, accept: float = 1e-4):
    """Returns (alpha, phi(alpha), evaluations).  alpha = 0 means no decrease found."""
    f1 = phi(1.0)
    nev = 1
    if f1 <= (1.0 - accept) * phi0:
        return 1.0, f1, nev
    best_a, best_f = 1.0, f1

    def consider(a, f):
        nonlocal best_a, best_f
        if f < best_f or (f == best_f and a > best_a):
            best_a, best_f = a, f

    a, b = 0.0, 1.0
    c = b - GOLD * (b - a)
    d = a + GOLD * (b - a)
    fc, fd = phi(c), phi(d)
    nev += 2
    consider(c, fc)
    consider(d, fd)
    for _ in range(iters):
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - GOLD * (b - a)
            fc = phi(c)
            consider(c, fc)
        else:
            a, c, fc = c, d, fd
            d = a + GOLD * (b - a)
            fd = phi(d)
            consider(d, fd)
        nev += 1
    if best_f < phi0:
        return best_a, best_f, nev
    return 0.0, phi0, nev


# ---------------------------------------------------------------------------
# IPN (Alg. 1) and AMIPN (Alg. 2)
# ---------------------------------------------------------------------------


@dataclass
class Opts:
    method: str = "ipn"            # "ipn" | "amipn"
    mode: str = "replica"          # "replica": sketch + QR + LSQR;  "exact": dense lstsq step
    gamma: float = 2.0
    seed: int = 1
    lsqr_tol: float = 1e-10
    lsqr_maxit: int = 500
    outer_tol: float = 1e-10
    max_outer: int = 30
    m_max: int = 3
    tau_rel: float = 1e-3
    row_c: float = 100.0
    gs_iters: int = 25
    sketch_kind: str = "gaussian"  # "gaussian" | "count" (the count sketch of Sec. 4.1, FP64)
    sketch_prec: str = "f64"       # "f64" | "bf16" | "fp8"  (oracle.lowprec)
    sketch_pieces: int = 0         # pieces of D J in the low-precision sketch (0: format default)
    lsqr_prec: str = "f64"         # "f64" | "f32": D J copy used by the LSQR products
    jac_index0: int = 0            # index of the first Jacobian evaluation (the sketch's key word 1)


@dataclass
class Stats:
    outer_iters: int = 0
    jac_evals: int = 0
    lsqr_iters: List[int] = field(default_factory=list)
    alphas: List[float] = field(default_factory=list)
    resnorms: List[float] = field(default_factory=list)
    status: str = "ok"             # ok | maxit | stall | singular
    inner_steps: List[int] = field(default_factory=list)   # directions computed in each outer step
    flags: List[bool] = field(default_factory=list)        # Alg. 2's Flag after each outer step
    iterates: List[np.ndarray] = field(default_factory=list)  # u after each outer step


@dataclass
class Precond:
    """One Jacobian evaluation with its row scale and its preconditioner."""
    DJ: np.ndarray
    D: np.ndarray
    R: Optional[np.ndarray]
    DJ_lsqr: Optional[np.ndarray] = None   # the copy LSQR multiplies by (DJ itself in FP64 mode)


def make_precond(prob: Problem, u: np.ndarray, opts: Opts, jac_index: int) -> Precond:
    F, J = assemble(prob, u)
    D = row_scale(J, opts.row_c)
    DJ = D[:, None] * J
    R = None
    if opts.mode == "replica":
        s = sketch_rows(prob.n, opts.gamma)
        if opts.sketch_kind == "count":
            B = philox.count_sketch_matrix(opts.seed, jac_index, s, DJ.shape[0]) @ DJ
        elif opts.sketch_prec == "f64":
            B = sketch(DJ, s, opts.seed, jac_index)
        else:
            B = lowprec.sketch_lowp(prob, DJ, s, opts.seed, jac_index, opts.sketch_prec, opts.sketch_pieces)
        R = qr_r(B)
    DJl = lowprec.round_f32(DJ) if opts.lsqr_prec == "f32" else DJ
    return Precond(DJ, D, R, DJl)


def newton_direction(pc: Precond, DF: np.ndarray, opts: Opts, stats: Stats) -> np.ndarray:
    """delta u from min ||D F + D J delta u|| (Alg. 1 steps 3-5 / Alg. 2 steps 5-6)."""
    if pc.R is None:
        du = np.linalg.lstsq(pc.DJ, -DF, rcond=None)[0]
        stats.lsqr_iters.append(0)
        return du
    R = pc.R
    A = pc.DJ if pc.DJ_lsqr is None else pc.DJ_lsqr
    res = lsqr(lambda y: A @ r_solve(R, y), lambda w: rt_solve(R, A.T @ w), -DF, R.shape[0],
               opts.lsqr_tol, opts.lsqr_maxit)
    stats.lsqr_iters.append(res.iters)
    return r_solve(R, res.x)


def scaled_norm(prob: Problem, D: np.ndarray, u: np.ndarray) -> float:
    return float(np.linalg.norm(D * residual(prob, u)))


def ipn(prob: Problem, u0: Optional[np.ndarray] = None, opts: Optional[Opts] = None):
    """Alg. 1.  Returns (u, stats)."""
    opts = opts or Opts()
    u = np.zeros(prob.n) if u0 is None else np.array(u0, float)
    st = Stats()
    for k in range(opts.max_outer):
        try:
            pc = make_precond(prob, u, opts, opts.jac_index0 + st.jac_evals)
        except SingularPreconditioner:
            st.status = "singular"
            return u, st
        st.jac_evals += 1
        DF = pc.D * residual(prob, u)
        phi0 = float(np.linalg.norm(DF))
        if phi0 == 0.0:
            break
        du = newton_direction(pc, DF, opts, st)
        alpha, phi1, _ = golden_section(lambda a: scaled_norm(prob, pc.D, u + a * du), phi0, opts.gs_iters)
        st.outer_iters += 1
        st.inner_steps.append(1)
        st.flags.append(True)
        st.alphas.append(alpha)
        if alpha == 0.0:
            st.status = "stall"
            st.resnorms.append(phi0)
            st.iterates.append(u.copy())
            return u, st
        u = u + alpha * du
        st.resnorms.append(phi1)
        st.iterates.append(u.copy())
        if abs(phi1 - phi0) < opts.outer_tol or phi1 == 0.0:
            return u, st
    st.status = "maxit"
    return u, st


def amipn(prob: Problem, u0: Optional[np.ndarray] = None, opts: Optional[Opts] = None):
    """Alg. 2.  One Jacobian and preconditioner per outer step, reused for at most
    m_max inner steps; an early stop keeps the preconditioner for the next outer
    step, reaching m_max recomputes it at the new iterate.

    A line search that finds no decrease ends the inner loop and forces a fresh
    preconditioner; with a fresh one it ends the solve (status "stall")."""
    opts = opts or Opts(method="amipn")
    u = np.zeros(prob.n) if u0 is None else np.array(u0, float)
    st = Stats()
    try:
        pc = make_precond(prob, u, opts, opts.jac_index0)
    except SingularPreconditioner:
        st.status = "singular"
        return u, st
    st.jac_evals = 1
    fresh = True
    for k in range(opts.max_outer):
        z = u.copy()
        Fz = pc.D * residual(prob, z)
        F0 = float(np.linalg.norm(Fz))
        phi_u = F0
        if F0 == 0.0:
            return u, st
        flag = True
        stalled = False
        for i in range(opts.m_max):
            d = newton_direction(pc, Fz, opts, st)
            phiz = float(np.linalg.norm(Fz))
            alpha, phin, _ = golden_section(lambda a: scaled_norm(prob, pc.D, z + a * d), phiz, opts.gs_iters)
            st.alphas.append(alpha)
            if alpha == 0.0:
                stalled = True
                break
            z = z + alpha * d
            Fn = pc.D * residual(prob, z)
            if np.linalg.norm(Fn - Fz) < opts.tau_rel * F0:
                flag = False
                Fz = Fn
                break
            Fz = Fn
        st.outer_iters += 1
        st.inner_steps.append(i + 1)
        if stalled and i == 0 and fresh:
            st.flags.append(True)
            st.status = "stall"
            st.resnorms.append(phi_u)
            st.iterates.append(u.copy())
            return u, st
        if stalled:
            flag = True
        st.flags.append(flag)
        u_new = z
        phi_new = float(np.linalg.norm(pc.D * residual(prob, u_new)))
        st.resnorms.append(phi_new)
        st.iterates.append(u_new.copy())
        done = abs(phi_new - phi_u) < opts.outer_tol or phi_new == 0.0
        u = u_new
        if done and not stalled:
            return u, st
        if flag:
            try:
                pc = make_precond(prob, u, opts, opts.jac_index0 + st.jac_evals)
            except SingularPreconditioner:
                st.status = "singular"
                return u, st
            st.jac_evals += 1
            fresh = True
        else:
            fresh = False
    st.status = "maxit"
    return u, st


def solve(prob: Problem, u0=None, opts: Optional[Opts] = None):
    opts = opts or Opts()
    return (amipn if opts.method == "amipn" else ipn)(prob, u0, opts)


# ---------------------------------------------------------------------------
# field evaluation and error (Sec. 3.2: relative L2 error against u*)
# ---------------------------------------------------------------------------


def eval_field(prob: Problem, u: np.ndarray, x: np.ndarray, owner: np.ndarray) -> np.ndarray:
    """u_n(x) [npts, ncomp]: with the indicator partition of unity the features of the owner box, with
    the smooth one sum_e psi_e phi_e u_e over the boxes whose support holds x."""
    if getattr(prob, "pou", "a") == "b":
        out = np.zeros((x.shape[0], prob.ncomp))
        for e in covering_boxes(prob, x):
            for c in range(prob.ncomp):
                out[:, c] += blended_jet(prob, e, c, x)[0] @ u[col_slice(prob, e, c)]
        return out
    out = np.zeros((x.shape[0], prob.ncomp))
    for e in np.unique(owner):
        sel = np.nonzero(owner == e)[0]
        for c in range(prob.ncomp):
            phi = feature_jet(prob, int(e), c, x[sel])[0]
            out[sel, c] = phi @ u[col_slice(prob, int(e), c)]
    return out


def eval_grad(prob: Problem, u: np.ndarray, x: np.ndarray, owner: np.ndarray) -> np.ndarray:
    """grad u_n(x) [npts, ncomp, d]: the feature gradients (1 - t^2) w_a / sigma_a of the owner box (indicator
    partition), or by the product rule psi_e grad phi + phi grad psi_e summed over the covering boxes."""
    d = prob.dim
    out = np.zeros((x.shape[0], prob.ncomp, d))
    if getattr(prob, "pou", "a") == "b":
        for e in covering_boxes(prob, x):
            for c in range(prob.ncomp):
                dv = blended_jet(prob, e, c, x)[1]                  # [n, J, d]
                out[:, c, :] += np.einsum("njd,j->nd", dv, u[col_slice(prob, e, c)])
        return out
    for e in np.unique(owner):
        sel = np.nonzero(owner == e)[0]
        for c in range(prob.ncomp):
            dphi = feature_jet(prob, int(e), c, x[sel])[1]          # [n, J, d]
            out[sel, c, :] = np.einsum("njd,j->nd", dphi, u[col_slice(prob, int(e), c)])
    return out


def rel_h1(prob: Problem, u: np.ndarray) -> np.ndarray:
    """Per-component relative H1 error on the test points:
    sqrt(sum |u_n - u*|^2 + |grad(u_n - u*)|^2) / sqrt(sum |u*|^2 + |grad u*|^2)."""
    un = eval_field(prob, u, prob.test_x, prob.test_owner)
    gn = eval_grad(prob, u, prob.test_x, prob.test_owner)
    from rfm_workloads import jet_of
    jet = jet_of(prob)(prob.test_x)
    us, gs = jet[0], jet[1]
    num = np.sum((un - us) ** 2, axis=0) + np.sum((gn - gs) ** 2, axis=(0, 2))
    den = np.sum(us ** 2, axis=0) + np.sum(gs ** 2, axis=(0, 2))
    return np.sqrt(num / den)


def rel_l2(prob: Problem, u: np.ndarray) -> np.ndarray:
    """Per-component ||u_n - u*|| / ||u*|| on the problem's test points."""
    un = eval_field(prob, u, prob.test_x, prob.test_owner)
    us = prob.exact(prob.test_x)
    return np.linalg.norm(un - us, axis=0) / np.linalg.norm(us, axis=0)


# ---------------------------------------------------------------------------
# projection of field values onto the feature basis (initial-guess fit)
# ---------------------------------------------------------------------------

def pde_points(prob: Problem):
    """PDE collocation points in row order: (x [npde, d], owner [npde])."""
    xs, ows = [], []
    for g in prob.groups:
        if g.kind == KIND_PDE:
            xs.append(g.x)
            ows.append(np.full(len(g.x), g.owner, np.int32))
    return np.concatenate(xs), np.concatenate(ows)


def feature_matrix_pde(prob: Problem) -> np.ndarray:
    """Phi [npde * ncomp, n]: row (group, component k, point) holds the features
    of (owner box, k) at the point -- the identity operator on the PDE points."""
    rows = []
    for g in prob.groups:
        if g.kind != KIND_PDE:
            continue
        for k in range(prob.ncomp):
            blk = np.zeros((len(g.x), prob.n))
            phi, _, _ = feature_jet(prob, g.owner, k, g.x)
            blk[:, col_slice(prob, g.owner, k)] = phi
            rows.append(blk)
    return np.concatenate(rows)


def project(prob: Problem, values: np.ndarray, c: float = 100.0) -> np.ndarray:
    """argmin_u || D (Phi u - f) || with D = c / max |Phi_row| (values [npde, ncomp])."""
    Phi = feature_matrix_pde(prob)
    f = []
    base = 0
    for g in prob.groups:
        if g.kind != KIND_PDE:
            continue
        n = len(g.x)
        for k in range(prob.ncomp):
            f.append(values[base:base + n, k])
        base += n
    f = np.concatenate(f)
    D = row_scale(Phi, c)
    return np.linalg.lstsq(D[:, None] * Phi, D * f, rcond=None)[0]
