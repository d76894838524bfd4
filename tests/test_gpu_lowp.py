"""Low-precision forms on the GPU against their definitions in the oracle.

  * the fixed-point pieces of D J that the sketch kernels read: chunk
    exponents equal to the oracle's, integer codes within the format's exact
    range, the leading piece equal to the oracle's except where D J sits on a
    rounding tie (the two assemblies differ by ulps), and the pieces together
    within 2^(E - bP - 1) of the oracle's D J;
  * B = S (sum of pieces) / sqrt(s): every matrix-core sum is exact, so B
    matches the oracle's FP64 product to the level of the assembly noise
    (relative L2 <= 1e-11);
  * the preconditioner built from it keeps kappa(D J R^-1) at the FP64 level;
  * LSQR on the FP32 copy of D J: step quality against the dense step, next to
    the oracle's own LSQR on the same FP32 copy;
  * full solves: the error against the oracle's FP64 solve is printed and
    bounded (1e-6 relative on the field), and the error against u* stays at
    the FP64 level.
"""
import math
import sys

import numpy as np
import pytest

import rfm_workloads as W
from oracle import lowprec as L
from oracle import rfm as O

pytestmark = pytest.mark.gpu

R = None


def setup_module(module):
    global R
    import paper_2510_04170_amd as Rm
    Rm.lib()
    R = Rm


CASES = {
    "poisson2d_full": lambda: W.config1(),
    "grayscott_small": lambda: W.config2(nsub=(2, 2, 2), J=40, q=4, test_per_dim=3),
    "allencahn_small": lambda: W.config4_nohole(nsub=(2, 1, 2), J=70, q=4, test_per_dim=3),
    # J = 600 > 512 features per box: 1200-wide continuity rows
    "helmholtz_cosh_wide": lambda: W.helmholtz_cosh(nsub=(2, 1, 1), J=600, q=10, test_per_dim=3),
}

FMTS = {"bf16": 2, "fp8": 3}


def _relerr_l(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _announce(msg):
    sys.stdout.write(f"\n[gpu-test] {msg}\n")
    sys.stdout.flush()


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    _announce(f"low-precision case {request.param}")
    prob = CASES[request.param]()
    lp = R.from_description(prob)
    rng = np.random.default_rng(11)
    u = 0.1 * rng.normal(size=prob.n)
    F, J = O.assemble(prob, u)
    D = O.row_scale(J)
    yield dict(name=request.param, prob=prob, lp=lp, u=u, DF=D * F, DJ=D[:, None] * J)
    lp.close()


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_operand_pieces(case, fmt):
    lp, DJ, prob = case["lp"], case["DJ"], case["prob"]
    lp.stage_assemble(case["u"], 100.0)
    npc = L.DEFAULT_PIECES[fmt]
    bits = L.BITS[fmt]
    lp.stage_sketch(2.0, 1, 0, FMTS[fmt], 0)
    m, n = DJ.shape
    Jb = lp.J
    ops, exps = L.pieces(prob, DJ, fmt, npc)
    bgroups = L.block_groups(prob)
    ties = 0
    for blk in range(n // Jb):
        ns = lp.sketch_operand_slots(blk)
        groups = bgroups[blk]
        assert ns == len(groups)
        got = [lp.get_sketch_operand(p, blk, 0, ns) for p in range(npc)]
        assert np.array_equal(got[0][1], groups)
        for k in range(ns):
            g = groups[k]
            E = got[0][2][k]
            assert np.array_equal(E, exps[blk][k // 4]), (blk, k)
            if g < 0:
                assert not any(gp[0][k].any() for gp in got)
                continue
            rows = 32 * g + np.arange(32)
            ok = rows < m
            ref = np.zeros((32, Jb))
            ref[ok] = DJ[rows[ok], blk * Jb:(blk + 1) * Jb]
            ref = ref.T                                                    # [J][32]
            total = np.zeros_like(ref)
            for p in range(npc):
                unit = np.ldexp(1.0, E - bits * (p + 1))[:, None]
                q = got[p][0][k] / unit
                assert np.array_equal(q, np.round(q)) and np.abs(q).max() <= 2 ** bits, (blk, p, k)
                total += got[p][0][k]
                if p == 0:
                    r0 = np.zeros((32, Jb))
                    r0[ok] = ops[0][rows[ok], blk * Jb:(blk + 1) * Jb]
                    diff = got[0][0][k] != r0.T
                    if diff.any():
                        # only at rounding ties of the first piece: x / unit = n + 1/2 to within noise
                        y = (ref / unit)[diff]
                        assert np.all(np.abs(np.abs(y - np.floor(y)) - 0.5) < 1e-9), (blk, k)
                        ties += int(diff.sum())
            bound = np.ldexp(1.0, E - bits * npc - 1)[:, None] + 1e-12 * 100.0
            assert np.all(np.abs(total - ref) <= bound), (blk, k)
    # The row scale puts each row's largest entry at c = 100 = 12.5 * 2^3, a tie
    # for the first 4-bit FP8 piece: those codes round by the assembly's last ulp.
    print(f"{case['name']} {fmt}: first-piece codes at rounding ties that differ from the oracle's: {ties}")


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_lowp_sketch_matches_definition(case, fmt):
    lp, DJ, prob = case["lp"], case["DJ"], case["prob"]
    lp.stage_assemble(case["u"], 100.0)
    lp.stage_sketch(2.0, 1, 4, FMTS[fmt], 0)
    s = lp.s
    Bg = lp.get_sketch_cols(0, lp.n)
    Bx = L.sketch_lowp(prob, DJ, s, 1, 4, fmt)
    rel = np.linalg.norm(Bg - Bx) / np.linalg.norm(Bx)
    colrel = np.max(np.linalg.norm(Bg - Bx, axis=0) / np.linalg.norm(Bx, axis=0))
    print(f"{case['name']} {fmt}: ||B - B_def|| / ||B_def|| = {rel:.3e}, worst column {colrel:.3e}")
    assert rel < 1e-11
    assert colrel < 1e-10


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_lowp_preconditioner_quality(case, fmt):
    lp, DJ = case["lp"], case["DJ"]
    if DJ.shape[1] > 1500:
        pytest.skip("dense SVD too large")
    lp.stage_assemble(case["u"], 100.0)
    lp.stage_sketch(2.0, 1, 0, FMTS[fmt], 0)
    lp.stage_qr()
    Rg = lp.get_r_cols(0, lp.n)
    sv = np.linalg.svd(DJ @ np.linalg.inv(Rg), compute_uv=False)
    print(f"{case['name']} {fmt}: kappa(D J R^-1) = {sv[0] / sv[-1]:.3f}")
    assert sv[0] / sv[-1] < 12.0


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_streamed_lowp_sketch_gives_the_same_r(case, fmt):
    """The low-precision sketch produced 256 rows per pass into the streamed QR gives the R of the whole
    low-precision sketch."""
    lp = case["lp"]
    lp.stage_assemble(case["u"], 100.0)
    lp.stage_sketch(2.0, 1, 2, FMTS[fmt], 0)
    B = lp.get_sketch_cols(0, lp.n)
    lp.stage_qr()
    Rw = lp.get_r_cols(0, lp.n)
    lp.stage_sketch_qr_streamed(2.0, 1, 2, FMTS[fmt], 0, 256)
    Rs = lp.get_r_cols(0, lp.n)
    assert _relerr_l(Rs, Rw) < max(1e-12, 1e-15 * np.linalg.cond(B))


def test_lsqr_on_fp32_jacobian(case):
    """LSQR on the FP32 copy of D J (products summed in FP64) against the oracle's LSQR on the same rounded
    matrix.  Where u32 kappa(R) <= 1e-2 the FP32 operator is a small perturbation: both converge, within 5
    iterations of each other, to steps whose error against the FP64 least-squares step is within 10x of
    each other.  Where it is larger, rounding D J to FP32 perturbs D J R^-1 by about u32 kappa(D J), so the
    operator is noise in its small singular directions (the solver then falls back to FP64): there both
    sides are measured against the least-squares step of the rounded matrix itself, the problem they
    actually solve, after the same iteration limit."""
    lp, DJ, DF = case["lp"], case["DJ"], case["DF"]
    lp.stage_assemble(case["u"], 100.0)
    lp.stage_sketch(2.0, 1, 0, R.RFM_PREC_F64, 0)
    lp.stage_qr()
    Rg = lp.get_r_cols(0, lp.n)
    kap = np.linalg.cond(Rg)
    usable = 2.0 ** -24 * kap <= 1e-2
    y, it, istop = lp.stage_lsqr(-DF, 1e-10, 500, R.RFM_PREC_F32)
    DJ32 = L.round_f32(DJ)
    ro = O.lsqr(lambda v: DJ32 @ O.r_solve(Rg, v), lambda w: O.rt_solve(Rg, DJ32.T @ w), -DF, lp.n, 1e-10, 500)
    du_g = lp.r_solve(y)
    du_o = O.r_solve(Rg, ro.x)
    A = DJ if usable else DJ32
    du_ls = np.linalg.lstsq(A, -DF, rcond=None)[0]
    nF = np.linalg.norm(DF)
    err_g = np.linalg.norm(A @ (du_g - du_ls)) / nF
    err_o = np.linalg.norm(A @ (du_o - du_ls)) / nF
    print(f"{case['name']} FP32-J LSQR (u32 kappa(R) = {2.0 ** -24 * kap:.1e}): iterations gpu {it} "
          f"(stop {istop}) oracle {ro.iters}; step error vs {'FP64' if usable else 'FP32-matrix'} lstsq: "
          f"gpu {err_g:.3e} oracle {err_o:.3e}")
    if usable:
        assert istop in (1, 2)
        assert abs(it - ro.iters) <= 5
    assert err_g <= max(10 * err_o, 1e-9)


MODES = {
    "bf16_sketch": dict(sketch_prec=2, lsqr_prec=0),
    "fp8_sketch": dict(sketch_prec=3, lsqr_prec=0),
    "bf16_sketch_f32_lsqr": dict(sketch_prec=2, lsqr_prec=1),
    "fp8_sketch_f32_lsqr": dict(sketch_prec=3, lsqr_prec=1),
}

_ref = {}


def _fp64_reference(name, prob):
    if name not in _ref:
        uo, so = O.ipn(prob, opts=O.Opts(gamma=2.0, lsqr_tol=1e-10))
        _ref[name] = (uo, so)
    return _ref[name]


@pytest.mark.parametrize("mode", list(MODES))
def test_mixed_solve_poisson2d(mode):
    _announce(f"mixed-precision solve poisson2d {mode}")
    prob = W.config1()
    lp = R.from_description(prob)
    opts = R.default_opts(sketch_factor=2.0, lsqr_tol=1e-10, **MODES[mode])
    ug, st, rc = lp.solve(None, opts)
    assert rc in (R.RFM_OK, R.RFM_ESTALL), (rc, st)
    if MODES[mode]["lsqr_prec"] == 1:
        # kappa(D J) ~ 3e13 here: the first FP32 step fails and the solve continues in FP64
        assert st["lsqr_fp64_fallback"] == 1
    uo, so = _fp64_reference("poisson2d", prob)
    fg = O.eval_field(prob, ug, prob.test_x, prob.test_owner)
    fo = O.eval_field(prob, uo, prob.test_x, prob.test_owner)
    ex = prob.exact(prob.test_x)
    e_or = np.linalg.norm(fg - fo) / np.linalg.norm(fo)
    e_g = np.linalg.norm(fg - ex) / np.linalg.norm(ex)
    e_o = np.linalg.norm(fo - ex) / np.linalg.norm(ex)
    print(f"poisson2d {mode}: status {rc} IT {st['outer_iters']} NJ {st['jac_evals']} LSQR {st['lsqr_iters']} "
          f"fallback {st['lsqr_fp64_fallback']}; "
          f"field vs FP64 oracle {e_or:.3e}; relL2 vs u* {e_g:.4e} (FP64 oracle {e_o:.4e})")
    assert e_or < 1e-6
    assert e_g < 1.01 * e_o + 1e-9
    lp.close()


@pytest.mark.parametrize("mode", ["bf16_sketch_f32_lsqr", "fp8_sketch"])
def test_mixed_solve_grayscott_small(mode):
    _announce(f"mixed-precision solve grayscott_small {mode}")
    prob = W.config2(nsub=(2, 2, 2), J=40, q=4, test_per_dim=3)
    lp = R.from_description(prob)
    opts = R.default_opts(sketch_factor=2.0, lsqr_tol=1e-10, m_max=5, **MODES[mode])
    ug, st, rc = lp.solve(None, opts)
    assert rc in (R.RFM_OK, R.RFM_ESTALL), (rc, st)
    uo, so = _fp64_reference("grayscott_small", prob)
    fg = O.eval_field(prob, ug, prob.test_x, prob.test_owner)
    fo = O.eval_field(prob, uo, prob.test_x, prob.test_owner)
    e_or = np.linalg.norm(fg - fo) / np.linalg.norm(fo)
    print(f"grayscott_small {mode}: status {rc} IT {st['outer_iters']} LSQR {st['lsqr_iters']} "
          f"fallback {st['lsqr_fp64_fallback']}; "
          f"field vs FP64 oracle {e_or:.3e}")
    assert e_or < 1e-6
    lp.close()


def test_lowp_bad_arguments():
    prob = W.config1(nsub=(2, 2), J=20, q=6)
    lp = R.from_description(prob)
    lp.stage_assemble(np.zeros(lp.n), 100.0)
    with pytest.raises(R.RfmError):
        lp.stage_sketch(2.0, 1, 0, R.RFM_PREC_BF16, 17)
    with pytest.raises(R.RfmError):
        lp.get_sketch_operand(0, 0, 0, 1)          # no low-precision operand formed yet
    lp.stage_sketch(2.0, 1, 0, R.RFM_PREC_BF16, 2)
    with pytest.raises(R.RfmError):
        lp.get_sketch_operand(2, 0, 0, 1)          # piece out of range
    assert lp.sketch_operand_slots(10 ** 6) == -1
    with pytest.raises(R.RfmError):
        lp.solve(None, R.default_opts(lsqr_prec=R.RFM_PREC_BF16))
    lp.close()
