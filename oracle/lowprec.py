"""Low-precision forms of the sketch and of the LSQR products, written out plainly.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the bench's
CPU-baseline leg; never by the product library.

The paper computes in double precision throughout.  The forms below only
change how the preconditioner R is built (Sec. 4.1) and which copy of D J the
inner least-squares iterations multiply by (Alg. 1 step 4); the residual, the
line search and the Newton update stay in FP64.  Each is a definition, so the
GPU path can be compared with it up to FP64 rounding.

Why pieces.  A perturbation E of D J lifts the small singular values of the
sketched matrix to about ||E||; D J R^-1 then has singular values down to
sigma_min(D J) / ||E||.  RFM Jacobians reach kappa ~ 1e13, so the operand
must keep ~40 bits of D J, and the sums must not round at 2^-24 either.
Hence D J is cut into narrow integer pieces on a fixed-point grid, and every
low-precision product is an exact integer sum (no rounding at all in the
FP32 accumulator); the partial results are combined in FP64.

Sketch codes.  Entry S[i, r] (sketch row i, Jacobian row r) is K[b] / k_s,
where b is byte (i mod 32) of the Philox4x64-10 output for counter
(i // 32, r, 1, 0) and key (seed, jac_index) (byte j of the 32 output bytes is
bits 8 (j mod 8) .. 8 (j mod 8) + 7 of 64-bit word j // 8), and K[b] the
integer nearest (ties to even) to k_s Phi^-1((b + 1/2) / 256):
k_s = 32 for BF16 (|K| <= 93), k_s = 4 for FP8 (|K| <= 12).  The entries are
i.i.d., symmetric and bounded (sub-Gaussian), which is all the embedding
argument of Sec. 4.1 needs.

Row chunks.  For each column block (box e, component c) take the 32-row
groups g (rows 32 g .. 32 g + 31) that hold a row whose support includes the
block, in ascending order, padded with empty groups to a multiple of four;
chunk h of the block is groups 4 h .. 4 h + 3 of that list (at most 128
rows).  The support of a row is structural: a PDE row touches every
component of its box, a boundary row its box and component, a continuity row
its component on both boxes.

Pieces.  For column j and chunk h with largest magnitude M > 0 over the
chunk's rows, E = floor(log2 M) + 1 (so M < 2^E); with b bits per piece
(8 for BF16, 4 for FP8) and residual X_0 = D J,
    q_p = round_half_even(X_p / 2^(E - b (p + 1))),
    X_{p+1} = X_p - q_p 2^(E - b (p + 1)),
an integer with |q_p| <= 2^b (exact in BF16 / E4M3).  An all-zero chunk has
E = 0 and zero pieces.  P pieces keep b P bits of the chunk's largest entry.
The sketch is B = S (sum_p q_p 2^(E - b (p + 1))) / sqrt(s); in the GPU every
term S_codes * q_p over a chunk is an integer below 2^22 (BF16: 128 * 93 *
256; FP8: three pieces at once, 2^-8 granularity, 128 * 12 * 17 * 2^8), exact
in FP32.

FP32 LSQR products: D J is rounded once to FP32 (round-to-nearest-even) and
the products J v, J^T w are formed from those values in FP64 arithmetic.
"""
from __future__ import annotations

import math
from typing import List

import numpy as np
from scipy.special import ndtri

from . import philox as P

FMT_BF16 = "bf16"
FMT_E4M3 = "fp8"
DEFAULT_PIECES = {FMT_BF16: 6, FMT_E4M3: 12}
BITS = {FMT_BF16: 8, FMT_E4M3: 4}
CODE_SCALE = {FMT_BF16: 32.0, FMT_E4M3: 4.0}

E4M3_MAX = 448.0


def round_bf16(x) -> np.ndarray:
    """Round-to-nearest-even to 8 significant bits (the BF16 grid; no range limits)."""
    x = np.asarray(x, np.float64)
    m, e = np.frexp(x)                  # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(m * 256.0), e - 8)


def round_e4m3(x) -> np.ndarray:
    """Round-to-nearest-even onto the OCP FP8 E4M3 grid (|x| <= 448 required).

    Normal numbers have 4 significant bits and exponents -6 .. 8; below 2^-6
    the grid is the subnormal step 2^-9."""
    x = np.asarray(x, np.float64)
    if np.any(np.abs(x) > E4M3_MAX):
        raise ValueError("value outside the E4M3 range")
    _, e = np.frexp(x)                  # |x| in [2^(e-1), 2^e)
    quantum = np.ldexp(1.0, np.maximum(e - 1, -6) - 3)
    return np.round(x / quantum) * quantum


def e4m3_values() -> np.ndarray:
    """All finite values of the OCP E4M3 encoding, decoded from the bit fields."""
    vals = []
    for code in range(256):
        s = -1.0 if code & 0x80 else 1.0
        ex = (code >> 3) & 0xF
        mant = code & 0x7
        if ex == 0xF and mant == 0x7:
            continue                    # NaN
        v = mant * 2.0 ** -9 if ex == 0 else (1.0 + mant / 8.0) * 2.0 ** (ex - 7)
        vals.append(s * v)
    return np.array(sorted(set(vals)))


def code_table(fmt: str) -> np.ndarray:
    """K[b] = nearest integer (ties to even) to k_s Phi^-1((b + 1/2) / 256)."""
    return np.round(CODE_SCALE[fmt] * ndtri((np.arange(256) + 0.5) / 256.0))


def sample_bytes(seed: int, jac_index: int, i: np.ndarray, r: np.ndarray) -> np.ndarray:
    """The byte b(i, r) of the table sampler (arrays of the same shape)."""
    i = np.asarray(i, np.int64)
    r = np.asarray(r, np.int64)
    shape = np.broadcast(i, r).shape
    i = np.broadcast_to(i, shape).ravel()
    r = np.broadcast_to(r, shape).ravel()
    ctr = np.zeros((i.size, 4), np.uint64)
    ctr[:, 0] = (i // 32).astype(np.uint64)
    ctr[:, 1] = r.astype(np.uint64)
    ctr[:, 2] = 1
    x = P.philox4x64(ctr, (seed, jac_index))
    j = i % 32
    word = x[np.arange(i.size), j // 8]
    return ((word >> (8 * (j % 8)).astype(np.uint64)) & np.uint64(0xFF)).astype(np.int64).reshape(shape)


def sketch_matrix_codes(seed: int, jac_index: int, s: int, m: int, fmt: str) -> np.ndarray:
    """Dense S in R^{s x m}, S = K[b] / k_s (small problems only)."""
    ii, rr = np.meshgrid(np.arange(s), np.arange(m), indexing="ij")
    return code_table(fmt)[sample_bytes(seed, jac_index, ii, rr)] / CODE_SCALE[fmt]


def block_groups(prob) -> List[np.ndarray]:
    """Per column block e * ncomp + c: the 32-row groups holding a row whose
    structural support includes the block, ascending, padded with -1 to a
    multiple of four."""
    from rfm_workloads import KIND_CONTINUITY, KIND_PDE
    K = prob.ncomp
    nb = int(np.prod(prob.nsub))
    sets = [[] for _ in range(nb * K)]
    r = 0
    for g in prob.groups:
        comps = list(range(K)) if g.comp < 0 else [g.comp]
        if g.kind == KIND_PDE:
            for _ in range(K):               # one row per equation and point
                rows = np.arange(r, r + g.npts)
                r += g.npts
                for c in range(K):
                    sets[g.owner * K + c].append(rows)
        elif g.kind == KIND_CONTINUITY:
            for c in comps:
                rows = np.arange(r, r + g.npts * g.cont_order)
                r += g.npts * g.cont_order
                sets[g.owner * K + c].append(rows)
                sets[g.neighbor * K + c].append(rows)
        else:
            for c in comps:
                rows = np.arange(r, r + g.npts)
                r += g.npts
                sets[g.owner * K + c].append(rows)
    out = []
    for s in sets:
        grp = np.unique(np.concatenate(s) // 32) if s else np.zeros(0, np.int64)
        pad = (-len(grp)) % 4
        out.append(np.concatenate([grp, -np.ones(pad, np.int64)]))
    return out


def chunk_rows(groups: np.ndarray, h: int, m: int) -> np.ndarray:
    """Global rows of chunk h of a block (rows below m of its four groups)."""
    g = groups[4 * h:4 * h + 4]
    g = g[g >= 0]
    rows = (32 * g[:, None] + np.arange(32)[None, :]).ravel()
    return rows[rows < m]


def split_chunk(X: np.ndarray, fmt: str, npieces: int = 0):
    """One chunk (rows x columns) of D J cut into integer pieces per column: returns (pieces, E) with
    pieces[p] = q_p 2^(E - b(p+1)) (q_p integer, nearest with ties to even, taken from what the earlier
    pieces leave) and E = floor(log2 max |X|) + 1 per column (0 for an all-zero column)."""
    npieces = npieces or DEFAULT_PIECES[fmt]
    b = BITS[fmt]
    X = np.array(X, np.float64, copy=True)
    M = np.abs(X).max(axis=0) if X.shape[0] else np.zeros(X.shape[1])
    E = np.where(M > 0, np.frexp(M)[1], 0)          # M = f 2^e, f in [0.5, 1): floor(log2 M) + 1 = e
    out = []
    for p in range(npieces):
        unit = np.ldexp(1.0, E - b * (p + 1))
        piece = np.round(X / unit) * unit
        out.append(piece)
        X = X - piece
    return out, E


def pieces(prob, DJ: np.ndarray, fmt: str, npieces: int = 0):
    """Returns (pieces, exps): pieces[p] is m x n (values q_p 2^(E - b(p+1))),
    exps[e*K + c] is [nchunks, J] (the exponent E of each chunk and column)."""
    npieces = npieces or DEFAULT_PIECES[fmt]
    m, n = DJ.shape
    J = prob.J
    out = [np.zeros_like(DJ) for _ in range(npieces)]
    exps = []
    for blk, groups in enumerate(block_groups(prob)):
        cols = slice(blk * J, (blk + 1) * J)
        nch = len(groups) // 4
        E = np.zeros((nch, J), np.int64)
        for h in range(nch):
            rows = chunk_rows(groups, h, m)
            got, E[h] = split_chunk(DJ[rows, cols], fmt, npieces)
            for p in range(npieces):
                out[p][rows, cols] = got[p]
        exps.append(E)
    return out, exps


def sketch_lowp(prob, DJ: np.ndarray, s: int, seed: int, jac_index: int, fmt: str, npieces: int = 0) -> np.ndarray:
    """B = S (sum of the pieces of D J) / sqrt(s) (FP64 product of exact values)."""
    Jt = np.sum(pieces(prob, DJ, fmt, npieces)[0], axis=0)
    S = sketch_matrix_codes(seed, jac_index, s, DJ.shape[0], fmt)
    return (S @ Jt) / math.sqrt(s)


def round_f32(X: np.ndarray) -> np.ndarray:
    return np.asarray(X, np.float32).astype(np.float64)
