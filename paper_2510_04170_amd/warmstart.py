"""Learned initial guess for a parameter family: training data from the
solver itself, training with the library's network kernels, and the
comparison against the zero initial guess.

    python -m paper_2510_04170_amd.warmstart [--train 48] [--test 8] [--steps 6000] [--method ipn|amipn]

prints one JSON object.  Every numerical step runs in the library (solves,
field evaluation, network training and inference, projection); this module
only arranges the calls and the inputs.

The family is the Gray-Scott workload with F ~ U(0.02, 0.06),
k ~ U(0.04, 0.07) and the amplitude a ~ U(0.3, 0.7) of u*.  All members share
partition, features and points, so one problem object serves every member
(its operator and data are replaced per member) and the projection factor is
formed once.  Network inputs are (F, k, a) mapped affinely to [-1, 1] over the
family's ranges (by the library, rfm_warm_inputs) and the point x; outputs the
two field values.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

import rfm_workloads as W

from . import RFM_OK, RFM_ESTALL, RfmMLP, default_opts, from_description

KEYS = ("F", "k", "amp")
# the family's parameter ranges, handed to the library, which encodes each draw onto [-1, 1]
LO = np.array([W.GS_FAMILY[key][0] for key in KEYS])
HI = np.array([W.GS_FAMILY[key][1] for key in KEYS])


class Family:
    """One library problem for all members of the family."""

    def __init__(self, **kw):
        self.kw = kw
        self.base = W.gray_scott_member(0.04, 0.06, 0.5, **kw)
        self.lp = from_description(self.base)
        self.x, self.owner = self.lp.pde_points()

    def close(self):
        self.lp.close()

    def member(self, draw):
        desc = W.gray_scott_member(*draw, **self.kw)
        self.lp.update_from(desc)
        return desc

    def inputs(self, draw) -> np.ndarray:
        return self.lp.warm_inputs(np.asarray(draw, float), LO, HI)


def relerr(lp, desc, u) -> list:
    val = lp.eval(u, desc.test_x, desc.test_owner)
    ex = desc.exact(desc.test_x)
    return (np.linalg.norm(val - ex, axis=0) / np.linalg.norm(ex, axis=0)).tolist()


def collect(fam: Family, draws, opts):
    """Solve each member from the zero guess; samples (inputs, field at the PDE points)."""
    X, Y = [], []
    for d in draws:
        fam.member(d)
        u, st, rc = fam.lp.solve(None, opts)
        if rc not in (RFM_OK, RFM_ESTALL):
            raise RuntimeError(f"training solve failed with status {rc} for {d}")
        X.append(fam.inputs(d))
        Y.append(fam.lp.eval(u, fam.x, fam.owner))
    return np.concatenate(X).astype(np.float32), np.concatenate(Y).astype(np.float32)


def compare(fam: Family, net: RfmMLP, draws, opts):
    """Zero guess against the learned guess on each member; the plain solver decides the final error."""
    rows = []
    for d in draws:
        desc = fam.member(d)
        t0 = time.perf_counter()
        u0, st0, rc0 = fam.lp.solve(None, opts)
        t1 = time.perf_counter()
        uw, info = fam.lp.warm_start(net, np.asarray(d, float), opts, LO, HI)
        t2 = time.perf_counter()
        uw, stw, rcw = fam.lp.solve(uw, opts)
        t3 = time.perf_counter()
        f0 = fam.lp.eval(u0, desc.test_x, desc.test_owner)
        fw = fam.lp.eval(uw, desc.test_x, desc.test_owner)
        rows.append(dict(
            draw=dict(zip(KEYS, d)),
            zero=dict(status=rc0, IT=st0["outer_iters"], NJ=st0["jac_evals"], lsqr=st0["lsqr_iters_total"],
                      seconds=t1 - t0, relL2=relerr(fam.lp, desc, u0)),
            warm=dict(status=rcw, IT=stw["outer_iters"], NJ=stw["jac_evals"], lsqr=stw["lsqr_iters_total"],
                      seconds=t3 - t2, guess_seconds=t2 - t1, relL2=relerr(fam.lp, desc, uw),
                      resnorm_guess=info[0], resnorm_zero=info[1], kept=bool(info[2])),
            field_diff=float(np.linalg.norm(fw - f0) / np.linalg.norm(f0))))
    return rows


def run(n_train=48, n_test=4, steps=6000, batch=4096, lr=3e-3, lr_final=1e-4, width=128, depth=3, sizes=None,
        seed=0, method=0):
    sizes = sizes or dict(nsub=(2, 2, 2), J=60, q=6, test_per_dim=4)
    opts = default_opts(method=method, sketch_factor=2.0, lsqr_tol=1e-10, m_max=5)
    fam = Family(**sizes)
    train_draws = [W.gray_scott_family_draw(100 + i) for i in range(n_train)]
    test_draws = [W.gray_scott_family_draw(1000 + i) for i in range(n_test)]
    net = None
    try:
        t0 = time.perf_counter()
        X, Y = collect(fam, train_draws, opts)
        t1 = time.perf_counter()
        net = RfmMLP(3 + 3, width, depth, 2, seed=seed + 1)
        log = net.train(X, Y, steps=steps, batch=batch, lr=lr, lr_final=lr_final, seed=seed + 7)
        t2 = time.perf_counter()
        rows = compare(fam, net, test_draws, opts)
        n_fam, m_fam = fam.lp.n, fam.lp.m
    finally:
        # release the device memory now rather than at interpreter exit
        if net is not None:
            net.close()
        fam.close()
    mean = lambda key, sub: float(np.mean([r[sub][key] for r in rows]))
    return dict(
        family=dict(sizes={k: list(v) if isinstance(v, tuple) else v for k, v in sizes.items()},
                    n=n_fam, m=m_fam, npde=len(fam.x), train_draws=n_train, test_draws=n_test),
        network=dict(layers=[6] + [width] * depth + [2], steps=steps, batch=batch, lr=lr, lr_final=lr_final,
                     samples=len(X),
                     loss_first=float(log[0]) if len(log) else None, loss_last=float(log[-1]) if len(log) else None),
        seconds=dict(collect=t1 - t0, train=t2 - t1),
        mean=dict(IT_zero=mean("IT", "zero"), IT_warm=mean("IT", "warm"), NJ_zero=mean("NJ", "zero"),
                  NJ_warm=mean("NJ", "warm"), s_zero=mean("seconds", "zero"),
                  s_warm=mean("seconds", "warm") + mean("guess_seconds", "warm")),
        per_draw=rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=48)
    ap.add_argument("--test", type=int, default=8)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--method", choices=["ipn", "amipn"], default="ipn")
    a = ap.parse_args()
    out = run(a.train, a.test, a.steps, a.batch, method=1 if a.method == "amipn" else 0)
    print(json.dumps(out))


if __name__ == "__main__":
    sys.exit(main())
