"""Philox4x64-10 counter-based generator and the Gaussian sketch entries.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the bench's
CPU-baseline leg; never by the product library.

Philox is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of a
multiply-xor bijection on a 4x64-bit counter block under a 2x64-bit key that
is bumped by two Weyl constants between rounds.  Written here in plain numpy
uint64 arithmetic (the 128-bit product is assembled from 32-bit halves).

Count sketch (Sec. 4.1 as the paper states it): see count_sketch_hash below.

Gaussian sketch entries (a reading of the sketch S_k of Sec. 4.1, made Gaussian):
S[i, r] for sketch row i and Jacobian row r uses the counter (i // 8, r, 0, 0)
and the key (seed, jac_index).  Each of the four 64-bit outputs x_w is one
Box-Muller pair: with u1 = ((x_w >> 32) + 1) 2^-32 in (0, 1] and
u2 = (x_w mod 2^32) 2^-32 in [0, 1), rows 8q + 2w and 8q + 2w + 1 get
sqrt(-2 ln u1) cos(2 pi u2) and sqrt(-2 ln u1) sin(2 pi u2).  Entries are
scaled by 1/sqrt(s) so that E[S^T S] = I.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def mulhilo64(a: np.ndarray, b: np.uint64):
    """Full 128-bit product of uint64 arrays: returns (hi, lo)."""
    a = np.asarray(a, np.uint64)
    b = np.uint64(b)
    a0, a1 = a & _M32, a >> _S32
    b0, b1 = b & _M32, b >> _S32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> _S32) + (p01 & _M32) + (p10 & _M32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    with np.errstate(over="ignore"):
        lo = a * b
    return hi, lo


def philox4x64(ctr: np.ndarray, key, rounds: int = 10) -> np.ndarray:
    """ctr: [N, 4] uint64, key: (k0, k1).  Returns [N, 4] uint64."""
    c = np.array(ctr, dtype=np.uint64, copy=True).reshape(-1, 4)
    k0 = np.uint64(key[0])
    k1 = np.uint64(key[1])
    x0, x1, x2, x3 = c[:, 0], c[:, 1], c[:, 2], c[:, 3]
    with np.errstate(over="ignore"):
        for rnd in range(rounds):
            if rnd > 0:
                k0 = np.uint64((int(k0) + int(W0)) & 0xFFFFFFFFFFFFFFFF)
                k1 = np.uint64((int(k1) + int(W1)) & 0xFFFFFFFFFFFFFFFF)
            hi0, lo0 = mulhilo64(x0, M0)
            hi1, lo1 = mulhilo64(x2, M1)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return np.stack([x0, x1, x2, x3], axis=1)


def gaussian_octets(seed: int, jac_index: int, q: np.ndarray, r: np.ndarray) -> np.ndarray:
    """N(0,1) entries G[8q + l, r] for l = 0..7, returned as [N, 8]."""
    q = np.asarray(q, np.int64).ravel()
    r = np.asarray(r, np.int64).ravel()
    ctr = np.zeros((q.size, 4), np.uint64)
    ctr[:, 0] = q.astype(np.uint64)
    ctr[:, 1] = r.astype(np.uint64)
    x = philox4x64(ctr, (seed, jac_index))
    out = np.empty((q.size, 8))
    for w in range(4):
        u1 = ((x[:, w] >> np.uint64(32)).astype(np.float64) + 1.0) * 2.0 ** -32
        u2 = (x[:, w] & np.uint64(0xFFFFFFFF)).astype(np.float64) * 2.0 ** -32
        rad = np.sqrt(-2.0 * np.log(u1))
        ang = 2.0 * np.pi * u2
        out[:, 2 * w] = rad * np.cos(ang)
        out[:, 2 * w + 1] = rad * np.sin(ang)
    return out


def gaussian_entries(seed: int, jac_index: int, i: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Unscaled N(0,1) entries G[i, r] for index arrays i, r (same shape)."""
    i = np.asarray(i, np.int64)
    r = np.asarray(r, np.int64)
    shape = np.broadcast(i, r).shape
    i = np.broadcast_to(i, shape).ravel()
    r = np.broadcast_to(r, shape).ravel()
    octs = gaussian_octets(seed, jac_index, i // 8, r)
    return octs[np.arange(i.size), i % 8].reshape(shape)


def sketch_matrix(seed: int, jac_index: int, s: int, m: int) -> np.ndarray:
    """Dense S in R^{s x m} with N(0, 1/s) entries (small problems only)."""
    nq = (s + 7) // 8
    qq, rr = np.meshgrid(np.arange(nq), np.arange(m), indexing="ij")
    octs = gaussian_octets(seed, jac_index, qq, rr).reshape(nq, m, 8)
    G = octs.transpose(0, 2, 1).reshape(8 * nq, m)[:s]
    return G / np.sqrt(s)


# ---------------------------------------------------------------------------
# count sketch (the sketch of Sec. 4.1): one +-1 per column of S
# ---------------------------------------------------------------------------

def count_sketch_hash(seed: int, jac_index: int, r: np.ndarray, s: int):
    """Bucket h(r) in [0, s) and sign sigma(r) of Jacobian row r: Philox4x64-10 at
    counter (r, 0, 2, 0), key (seed, jac_index); h = word 0 mod s, sigma = +1 if bit 0
    of word 1 is clear, else -1."""
    r = np.asarray(r, np.int64).ravel()
    ctr = np.zeros((r.size, 4), np.uint64)
    ctr[:, 0] = r.astype(np.uint64)
    ctr[:, 2] = 2
    x = philox4x64(ctr, (seed, jac_index))
    h = (x[:, 0] % np.uint64(s)).astype(np.int64)
    sig = np.where((x[:, 1] & np.uint64(1)) == 0, 1.0, -1.0)
    return h, sig


def count_sketch_matrix(seed: int, jac_index: int, s: int, m: int) -> np.ndarray:
    """Dense S in R^{s x m}: S[h(r), r] = sigma(r), zero elsewhere (small problems only)."""
    h, sig = count_sketch_hash(seed, jac_index, np.arange(m), s)
    S = np.zeros((s, m))
    S[h, np.arange(m)] = sig
    return S
