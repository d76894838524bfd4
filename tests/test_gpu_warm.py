"""Learned initial guess on the GPU against the oracle.

  * network forward and loss gradient: FP32 mode against the FP64 oracle to
    1e-5 (relative L2); BF16 mode against the oracle with the same BF16
    operand rounding to 2e-3 and against the unrounded oracle to 1e-2;
  * Adam: three full-batch steps against the oracle's gradient and update;
  * training lowers the loss on a smooth target;
  * projection: fitted field at the PDE points against the oracle's dense
    least-squares fit to 1e-8;
  * a problem updated to another family member solves like a fresh one;
  * the learned guess against the zero guess on held-out members: the plain
    FP64 solver reaches the same field, in fewer Newton steps on average.
"""
import sys

import numpy as np
import pytest

import rfm_workloads as W
from oracle import mlp as M
from oracle import rfm as O

pytestmark = pytest.mark.gpu

R = None


def setup_module(module):
    global R
    import paper_2510_04170_amd as Rm
    Rm.lib()
    R = Rm


def _announce(msg):
    sys.stdout.write(f"\n[gpu-test] {msg}\n")
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


SHAPES = [(6, 128, 3, 2), (5, 37, 2, 3)]


def _data(in_dim, out_dim, n, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(n, in_dim)).astype(np.float32)
    Y = (np.sin(2 * X[:, :out_dim]) + 0.3 * X[:, -1:] ** 2).astype(np.float32)
    return X, Y


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_and_gradient(shape):
    in_dim, width, depth, out_dim = shape
    _announce(f"network {shape}")
    ds = M.dims(*shape)
    p = W.mlp_params(*shape, seed=11)
    net = R.RfmMLP(*shape, seed=3)
    net.set_params(p)
    assert np.array_equal(net.get_params(), p)
    X, Y = _data(in_dim, out_dim, 300, 12)
    p64 = p.astype(np.float64)
    y_ex, _ = M.forward(p64, ds, X.astype(np.float64))
    y_bf, _ = M.forward(p64, ds, X.astype(np.float64), bf16=True)
    L_ex, g_ex = M.loss_grad(p64, ds, X.astype(np.float64), Y.astype(np.float64))
    L_bf, g_bf = M.loss_grad(p64, ds, X.astype(np.float64), Y.astype(np.float64), bf16=True)

    net.set_precision(R.RFM_PREC_F32)
    yf = net.predict(X)
    Lf, gf = net.loss_grad(X, Y)
    print(f"FP32 mode: forward {_rel(yf, y_ex):.2e}, loss {abs(Lf - L_ex) / L_ex:.2e}, grad {_rel(gf, g_ex):.2e}")
    assert _rel(yf, y_ex) < 1e-5
    assert abs(Lf - L_ex) < 1e-5 * L_ex
    assert _rel(gf, g_ex) < 1e-5

    net.set_precision(R.RFM_PREC_BF16)
    yb = net.predict(X)
    Lb, gb = net.loss_grad(X, Y)
    print(f"BF16 mode: forward vs rounded oracle {_rel(yb, y_bf):.2e}, vs exact {_rel(yb, y_ex):.2e}; "
          f"grad vs rounded oracle {_rel(gb, g_bf):.2e}, vs exact {_rel(gb, g_ex):.2e}")
    assert _rel(yb, y_bf) < 2e-3
    assert _rel(yb, y_ex) < 1e-2
    assert _rel(gb, g_bf) < 2e-3
    assert _rel(gb, g_ex) < 1e-2
    net.close()


def test_adam_steps_match_oracle():
    shape = (6, 32, 2, 2)
    ds = M.dims(*shape)
    p = W.mlp_params(*shape, seed=21)
    X, Y = _data(6, 2, 200, 22)
    net = R.RfmMLP(*shape)
    net.set_precision(R.RFM_PREC_F32)
    net.set_params(p)
    log = net.train(X, Y, steps=3, batch=10 ** 6, lr=1e-2)    # batch covers the data: full, in order
    pg = net.get_params().astype(np.float64)
    po = p.astype(np.float64)
    m = np.zeros_like(po)
    v = np.zeros_like(po)
    moved = np.ones(po.size, bool)
    for t in range(1, 4):
        L, g = M.loss_grad(po, ds, X.astype(np.float64), Y.astype(np.float64))
        assert abs(log[t - 1] - L) < 1e-5 * L
        # an Adam step is about lr * sign(g): components with a gradient at FP32 noise level may go either way
        moved &= np.abs(g) > 1e-4 * np.abs(g).max()
        po, m, v = M.adam(po, m, v, g, t, lr=1e-2)
    d_g, d_o = pg - p, po - p
    print(f"Adam: update difference {np.abs(d_g - d_o)[moved].max():.2e} (lr 1e-2), "
          f"{(~moved).sum()} near-zero-gradient components excluded")
    assert np.abs(d_g - d_o)[moved].max() < 1e-4
    net.close()


def test_training_lowers_the_loss():
    shape = (6, 128, 3, 2)
    X, Y = _data(6, 2, 20000, 31)
    net = R.RfmMLP(*shape, seed=5)
    log = net.train(X, Y, steps=600, batch=2048, lr=2e-3, seed=9)
    print(f"training loss {log[0]:.3e} -> {log[-1]:.3e}")
    assert np.all(np.isfinite(log))
    assert log[-50:].mean() < 0.1 * log[:10].mean()
    net.close()


def _family_problem(draw=(0.04, 0.06, 0.5)):
    return W.gray_scott_member(*draw, nsub=(2, 2, 1), J=30, q=5, test_per_dim=3)


def test_projection_matches_oracle():
    prob = _family_problem()
    lp = R.from_description(prob)
    x, ow = lp.pde_points()
    xo, owo = O.pde_points(prob)
    assert np.array_equal(x, xo) and np.array_equal(ow, owo)
    vals = np.stack([1.0 - 0.5 * np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]),
                     0.25 * np.cos(3 * x[:, 2]) + x[:, 0] * x[:, 1]], axis=1)
    opts = R.default_opts(sketch_factor=2.0, lsqr_tol=1e-12, lsqr_max_iter=1000)
    ug, rn = lp.project(vals, opts)
    uo = O.project(prob, vals)
    Phi = O.feature_matrix_pde(prob)
    e = _rel(Phi @ ug, Phi @ uo)
    print(f"projection: fitted values vs oracle {e:.2e}, residual norm {rn:.3e}")
    assert e < 1e-8
    # second call reuses the factor and gives the same answer for the same values
    ug2, _ = lp.project(vals, opts)
    assert _rel(Phi @ ug2, Phi @ ug) < 1e-12
    lp.close()


def test_update_to_another_member_matches_fresh_problem():
    a, b = (0.03, 0.05, 0.4), (0.055, 0.065, 0.65)
    lp = R.from_description(_family_problem(a))
    pb = _family_problem(b)
    lp.update_from(pb)
    fresh = R.from_description(pb)
    opts = R.default_opts(sketch_factor=2.0, lsqr_tol=1e-10, m_max=5)
    u1, s1, rc1 = lp.solve(None, opts)
    u2, s2, rc2 = fresh.solve(None, opts)
    assert rc1 == rc2 and s1["outer_iters"] == s2["outer_iters"]
    f1 = lp.eval(u1, pb.test_x, pb.test_owner)
    f2 = fresh.eval(u2, pb.test_x, pb.test_owner)
    assert _rel(f1, f2) < 1e-12
    F1, n1 = lp.residual(u1)
    F2, n2 = fresh.residual(u1)
    assert abs(n1 - n2) <= 1e-13 * n2
    lp.close()
    fresh.close()


def test_learned_guess_against_zero_guess():
    _announce("warm-start study (small family)")
    from paper_2510_04170_amd import warmstart as WS
    out = WS.run(n_train=48, n_test=4, steps=6000, batch=4096, lr=3e-3, lr_final=1e-4,
                 sizes=dict(nsub=(2, 2, 2), J=40, q=5, test_per_dim=3))
    mean = out["mean"]
    print(f"warm start: training loss {out['network']['loss_first']:.3e} -> {out['network']['loss_last']:.3e}; "
          f"IT zero {mean['IT_zero']:.2f} warm {mean['IT_warm']:.2f}; NJ zero {mean['NJ_zero']:.2f} "
          f"warm {mean['NJ_warm']:.2f}; s zero {mean['s_zero']:.3f} warm {mean['s_warm']:.3f}")
    for r in out["per_draw"]:
        print(f"  {r['draw']}: zero IT {r['zero']['IT']} warm IT {r['warm']['IT']} kept {r['warm']['kept']} "
              f"|F| guess {r['warm']['resnorm_guess']:.3e} vs zero {r['warm']['resnorm_zero']:.3e}; "
              f"field diff {r['field_diff']:.2e}")
        assert r["zero"]["status"] in (R.RFM_OK, R.RFM_ESTALL) and r["warm"]["status"] in (R.RFM_OK, R.RFM_ESTALL)
        # the plain solver decides the answer: same field either way
        assert r["field_diff"] < 1e-6
        # the learned guess is kept only when it beats the zero vector in the solver's merit ||D0 F||,
        # and on this family it does by a wide margin
        assert r["warm"]["kept"] and r["warm"]["resnorm_guess"] < 0.5 * r["warm"]["resnorm_zero"]
    assert out["network"]["loss_last"] < 0.05 * out["network"]["loss_first"]
    assert mean["NJ_warm"] < mean["NJ_zero"]
