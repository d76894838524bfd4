"""Pins of the oracle's low-precision forms against facts that do not come from
the oracle itself: the bit layouts of BF16 and OCP FP8 E4M3, the normal
distribution function (through math.erf), byte order of the generator words,
and the condition-number drop of Sec. 4.1 that the preconditioner must keep."""
import math
import struct

import numpy as np
import pytest

import rfm_workloads as W
from oracle import lowprec as L
from oracle import philox as P
from oracle import rfm as O


# ---------------------------------------------------------------------------
# rounding to BF16 and E4M3
# ---------------------------------------------------------------------------

def _bf16_neighbours(x):
    """The BF16 values just below and above x, from the float32 bit pattern."""
    f = struct.unpack("<I", struct.pack("<f", np.float32(x)))[0]
    lo = f & 0xFFFF0000
    hi = lo + 0x10000
    dec = lambda b: struct.unpack("<f", struct.pack("<I", b))[0]
    a, b = dec(lo), dec(hi)
    return (a, b) if x >= 0 else (b, a)


def test_bf16_ties_to_even_and_grid():
    # spacing at 1 is 2^-7: 1 + 2^-8 is a tie between 1 (even) and 1 + 2^-7 (odd)
    assert L.round_bf16(1 + 2 ** -8) == 1.0
    # 1 + 3 * 2^-8 ties between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert L.round_bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6
    assert L.round_bf16(-(1 + 3 * 2 ** -8)) == -(1 + 2 ** -6)
    rng = np.random.default_rng(0)
    # values exactly representable in float32 so that the neighbours are exact
    xs = np.float32(rng.normal(size=2000) * 10.0 ** rng.integers(-6, 6, size=2000)).astype(np.float64)
    for x in xs:
        r = float(L.round_bf16(x))
        a, b = _bf16_neighbours(x)
        # r is one of the two neighbours and the nearer one
        assert r in (a, b)
        assert abs(r - x) <= min(abs(a - x), abs(b - x))
        # r has at most 8 significant bits
        assert struct.unpack("<I", struct.pack("<f", r))[0] & 0xFFFF == 0


def test_e4m3_grid_from_the_encoding():
    vals = L.e4m3_values()
    assert vals.max() == 448.0 and vals.min() == -448.0
    assert (vals > 0).sum() == 126          # 7 subnormals + 15 * 8 normals - NaN code, per sign... minus zero
    # every encodable value rounds to itself
    assert np.array_equal(L.round_e4m3(vals), vals)
    # nearest-value rounding, ties to the even code (mantissa bit 0 clear)
    pos = vals[vals >= 0]
    rng = np.random.default_rng(1)
    xs = rng.uniform(-440, 440, size=3000) * 10.0 ** rng.integers(-4, 1, size=3000)
    xs = np.concatenate([xs, (pos[1:] + pos[:-1]) / 2])       # all midpoints
    for x in xs:
        r = float(L.round_e4m3(x))
        d = np.abs(vals - x)
        best = vals[d == d.min()]
        assert r in best
        if len(best) == 2:
            # tie: the neighbour whose mantissa LSB is zero, i.e. r / ulp is even
            e = max(math.frexp(abs(r))[1] - 1, -6) if r != 0 else -6
            assert (abs(r) / 2.0 ** (e - 3)) % 2 == 0
    with pytest.raises(ValueError):
        L.round_e4m3(np.array([500.0]))


# ---------------------------------------------------------------------------
# the table sampler
# ---------------------------------------------------------------------------

def _phi(x):
    return 0.5 * (1.0 + math.erf(x / math.sqrt(2.0)))


@pytest.mark.parametrize("fmt,kmax", [(L.FMT_BF16, 92), (L.FMT_E4M3, 12)])
def test_code_table(fmt, kmax):
    K = L.code_table(fmt)
    ks = L.CODE_SCALE[fmt]
    assert K.shape == (256,)
    assert np.array_equal(K, np.round(K)) and np.abs(K).max() == kmax
    assert np.array_equal(K[::-1], -K)                 # symmetric quantiles
    assert np.all(np.diff(K) >= 0)
    # codes are exact in the operand format (integers up to 256 in BF16, 16 in E4M3)
    if fmt == L.FMT_BF16:
        assert np.array_equal(L.round_bf16(K), K)
    else:
        assert np.array_equal(L.round_e4m3(K), K)
    for b in range(256):
        p = (b + 0.5) / 256
        # K[b] / ks is within 1 / (2 ks) of the quantile q with Phi(q) = p, so
        # Phi(K[b] / ks) is within (largest density between them) / (2 ks) of p
        t = float(K[b]) / ks
        near = max(abs(t) - 0.5 / ks, 0.0)
        dens = math.exp(-0.5 * near * near) / math.sqrt(2 * math.pi)
        assert abs(_phi(t) - p) <= dens * (0.5 / ks) * 1.0001 + 1e-15


def test_sample_bytes_layout_and_moments():
    seed, jac = 7, 2
    i = np.arange(64)
    r = np.full(64, 5)
    b = L.sample_bytes(seed, jac, i, r)
    # independent byte extraction: little-endian bytes of the four 64-bit words
    for q in range(2):
        words = P.philox4x64(np.array([[q, 5, 1, 0]], np.uint64), (seed, jac))[0]
        raw = b"".join(int(w).to_bytes(8, "little") for w in words)
        assert list(b[32 * q:32 * q + 32]) == list(raw)
    S = L.sketch_matrix_codes(3, 1, 300, 400, L.FMT_BF16)
    T = L.code_table(L.FMT_BF16) / L.CODE_SCALE[L.FMT_BF16]
    g = S.ravel()
    n = g.size
    assert abs(g.mean()) < 5 * math.sqrt(np.mean(T ** 2) / n)
    assert abs(g.var() / np.mean(T ** 2) - 1) < 6 * math.sqrt(2 / n)
    # every byte value is used about equally often
    cnt = np.bincount(L.sample_bytes(3, 1, *np.meshgrid(np.arange(300), np.arange(400), indexing="ij")).ravel(),
                      minlength=256)
    assert cnt.min() > 0.8 * n / 256 and cnt.max() < 1.2 * n / 256
    # a different Jacobian index gives an unrelated matrix
    S2 = L.sketch_matrix_codes(3, 2, 300, 400, L.FMT_BF16)
    assert abs(np.corrcoef(g, S2.ravel())[0, 1]) < 0.02


# ---------------------------------------------------------------------------
# pieces
# ---------------------------------------------------------------------------

def _small_problem(cfg=0):
    if cfg == 0:
        prob = W.config1(nsub=(2, 2), J=20, q=6)
    else:
        prob = W.config2(nsub=(2, 1, 1), J=12, q=3, test_per_dim=2)
    u = 0.1 * np.random.default_rng(4).normal(size=prob.n)
    F, J = O.assemble(prob, u)
    D = O.row_scale(J)
    return prob, D[:, None] * J


@pytest.mark.parametrize("cfg", [0, 1])
def test_block_groups_cover_the_numerical_support(cfg):
    prob, DJ = _small_problem(cfg)
    m = DJ.shape[0]
    J = prob.J
    for blk, groups in enumerate(L.block_groups(prob)):
        assert len(groups) % 4 == 0
        real = groups[groups >= 0]
        assert np.all(np.diff(real) > 0)
        nz_rows = np.flatnonzero(np.abs(DJ[:, blk * J:(blk + 1) * J]).max(axis=1) > 0)
        # every row with a non-zero in the block lies in a listed group
        assert set((nz_rows // 32).tolist()) <= set(real.tolist())
        # padding only completes the last chunk
        assert np.all(groups[len(real):] == -1) and len(groups) - len(real) < 4


@pytest.mark.parametrize("fmt", [L.FMT_BF16, L.FMT_E4M3])
@pytest.mark.parametrize("cfg", [0, 1])
def test_fixed_point_pieces(fmt, cfg):
    prob, DJ = _small_problem(cfg)
    m = DJ.shape[0]
    J = prob.J
    b = L.BITS[fmt]
    P = L.DEFAULT_PIECES[fmt]
    ps, exps = L.pieces(prob, DJ, fmt)
    assert len(ps) == P
    total = np.sum(ps, axis=0)
    for blk, groups in enumerate(L.block_groups(prob)):
        cols = slice(blk * J, (blk + 1) * J)
        for h in range(len(groups) // 4):
            rows = L.chunk_rows(groups, h, m)
            X = DJ[rows, cols]
            M = np.abs(X).max(axis=0)
            E = exps[blk][h]
            for j in range(J):
                if M[j] == 0:
                    assert E[j] == 0
                    continue
                # M < 2^E <= 2 M
                assert M[j] < 2.0 ** E[j] <= 2 * M[j]
                left = X[:, j].copy()
                for p in range(P):
                    unit = 2.0 ** (E[j] - b * (p + 1))
                    q = ps[p][rows, blk * J + j] / unit
                    # integer codes within the format's exact integer range
                    assert np.array_equal(q, np.round(q)) and np.abs(q).max() <= 2 ** b
                    # nearest multiple of the unit (within half a unit)
                    assert np.all(np.abs(left - q * unit) <= 0.5 * unit)
                    left = left - q * unit
                assert np.all(np.abs(left) <= 2.0 ** (E[j] - b * P - 1))
    # rows outside a block's chunks are zero in its columns, and the pieces vanish there
    assert np.all(np.abs(DJ - total) <= 2.0 ** (-b * P) * np.abs(DJ).max())


def test_exact_integer_sums():
    """The products the GPU accumulates in FP32 stay exact: the largest chunk
    sum of |codes| * |pieces| fits the 24-bit significand (BF16: integers;
    FP8: three pieces at once on a 2^-8 grid)."""
    assert 128 * 93 * 256 < 2 ** 24
    assert 128 * 12 * (16 + 16 / 16 + 16 / 256) * 2 ** 8 < 2 ** 24
    assert np.abs(L.code_table(L.FMT_BF16)).max() <= 93
    assert np.abs(L.code_table(L.FMT_E4M3)).max() <= 12


# ---------------------------------------------------------------------------
# what the pieces are for: the preconditioner keeps the Sec. 4.1 bound
# ---------------------------------------------------------------------------

def _poisson_small():
    prob = W.config1(nsub=(2, 2), J=100, q=14)
    F, J = O.assemble(prob, np.zeros(prob.n))
    D = O.row_scale(J)
    return prob, D[:, None] * J


@pytest.mark.parametrize("fmt,npc,ok", [(L.FMT_BF16, 6, True), (L.FMT_E4M3, 12, True), (L.FMT_BF16, 1, False)])
def test_lowp_sketch_preconditions(fmt, npc, ok):
    prob, DJ = _poisson_small()
    s = O.sketch_rows(prob.n, 2.0)
    sv = np.linalg.svd(DJ, compute_uv=False)
    assert sv[0] / sv[-1] > 1e8
    R = O.qr_r(L.sketch_lowp(prob, DJ, s, 1, 0, fmt, npc))
    sa = np.linalg.svd(DJ @ np.linalg.inv(R), compute_uv=False)
    kap = sa[0] / sa[-1]
    if ok:
        assert 3.0 < kap < 10.0
    else:
        # one 8-bit piece perturbs D J by ~2^-9 relative: the small singular
        # values are lost and kappa(D J R^-1) grows by orders of magnitude
        assert kap > 1e3


def test_lowp_ipn_matches_fp64_solution():
    prob = W.config1(nsub=(2, 2), J=60, q=10)
    u0, _ = O.ipn(prob, opts=O.Opts())
    f0 = O.eval_field(prob, u0, prob.test_x, prob.test_owner)
    for kw in (dict(sketch_prec="bf16"), dict(sketch_prec="fp8"), dict(sketch_prec="bf16", lsqr_prec="f32")):
        u, st = O.ipn(prob, opts=O.Opts(**kw))
        assert st.status in ("ok", "stall")
        f = O.eval_field(prob, u, prob.test_x, prob.test_owner)
        assert np.linalg.norm(f - f0) / np.linalg.norm(f0) < 1e-6, kw


def test_f32_copy_is_round_to_nearest():
    x = np.array([1 + 2.0 ** -24, 1 + 3 * 2.0 ** -24, -(1 + 3 * 2.0 ** -24), 1e-50])
    y = L.round_f32(x)
    assert list(y) == [1.0, 1 + 2.0 ** -22, -(1 + 2.0 ** -22), 0.0]
