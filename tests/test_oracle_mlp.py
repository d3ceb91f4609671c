"""Pins of the oracle's triplet network: BF16 rounding against torch's
round-to-nearest-even conversion, the forward pass and its gradient against
float64 torch autograd (an independent implementation), central finite
differences, closed-form features, and the limits of the pruning threshold."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2102_08862_amd import synth


def test_bf16_matches_torch():
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 2000), rng.normal(0, 1e4, 2000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9]]).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).float().numpy()
    assert np.array_equal(oracle.bf16(v), ref)
    lib = oracle._load()
    for a in v[:200]:
        assert lib.ora_bf16(float(a)) == float(torch.tensor(a).to(torch.bfloat16).float())


def _torch_forward(m, x, round_act=True):
    w1 = torch.tensor(m.w1, dtype=torch.float64)
    w2 = torch.tensor(m.w2, dtype=torch.float64)
    w3 = torch.tensor(m.w3, dtype=torch.float64)
    b1 = torch.tensor(m.b1, dtype=torch.float64)
    b2 = torch.tensor(m.b2, dtype=torch.float64)
    xx = torch.tensor(x, dtype=torch.float64)
    h1 = torch.relu(xx @ w1.T + b1)
    if round_act:
        h1 = h1.float().to(torch.bfloat16).double()
    h2 = torch.relu(h1 @ w2.T + b2)
    if round_act:
        h2 = h2.float().to(torch.bfloat16).double()
    return h2 @ w3 + m.b3


def _features(n, seed=1):
    rng = np.random.default_rng(seed)
    f = np.zeros((n, 16), np.float32)
    f[:, :12] = rng.normal(0, 1, (n, 12))
    return oracle.bf16(f)


def test_forward_matches_torch_float64():
    m = oracle.MLP.random(3)
    x = _features(500)
    z = oracle.mlp_forward(m, x)
    zt = _torch_forward(m, x).numpy()
    # the BF16 rounding of an activation may flip where FP64 sums differ in
    # their last bits; require near-equality for nearly all
    d = np.abs(z - zt)
    assert (d < 1e-9).mean() > 0.99
    z0 = oracle.mlp_forward(m, x, round_act=False)
    assert np.allclose(z0, _torch_forward(m, x, round_act=False).numpy(), rtol=0, atol=1e-9)


def test_hand_computed_toy_net():
    """w1 routes feature k to hidden k (k < 12), w2 is the identity, w3 sums:
    z = b3 + sum_k relu(relu(x_k + b1_k) + b2_k)."""
    w1 = np.zeros((64, 16), np.float32)
    for k in range(12):
        w1[k, k] = 1.0
    w2 = np.eye(64, dtype=np.float32)
    m = oracle.MLP(w1, np.full(64, 0.5, np.float32), w2, np.full(64, -0.25, np.float32),
                   np.ones(64, np.float32), 0.125)
    x = np.zeros((1, 16), np.float32)
    x[0, :12] = [1, -2, 0.5, 3, -0.75, 0, 2, -1, 0.25, 4, -3, 1.5]
    exp = 0.125 + sum(max(max(v + 0.5, 0) - 0.25, 0) for v in x[0, :12]) + 52 * max(0.5 - 0.25, 0)
    assert oracle.mlp_forward(m, x)[0] == pytest.approx(exp, abs=0)


def test_gradient_matches_torch_autograd_and_finite_differences():
    m = oracle.MLP.random(5)
    x = _features(256, seed=7)
    lab = (np.random.default_rng(8).random(256) < 0.3).astype(np.float32)
    wp = 2.5
    loss, g = oracle.mlp_grad(m, x, lab, w_pos=wp, round_act=False)
    # torch float64 autograd of the same loss
    P = {k: torch.tensor(getattr(m, k), dtype=torch.float64, requires_grad=True) for k in ("w1", "b1", "w2", "b2", "w3")}
    b3 = torch.tensor(m.b3, dtype=torch.float64, requires_grad=True)
    xx = torch.tensor(x, dtype=torch.float64)
    h1 = torch.relu(xx @ P["w1"].T + P["b1"])
    h2 = torch.relu(h1 @ P["w2"].T + P["b2"])
    z = h2 @ P["w3"] + b3
    yt = torch.tensor(lab, dtype=torch.float64)
    lt = torch.nn.functional.binary_cross_entropy_with_logits(z, yt, pos_weight=torch.tensor(wp, dtype=torch.float64))
    lt.backward()
    assert loss == pytest.approx(lt.item(), rel=1e-12)
    for k in ("w1", "b1", "w2", "b2", "w3"):
        assert np.allclose(g[k], P[k].grad.numpy(), rtol=1e-9, atol=1e-12), k
    assert g["b3"] == pytest.approx(b3.grad.item(), rel=1e-9)
    # central finite differences on a few coordinates
    flat = m.flat().astype(np.float64)
    gflat = np.concatenate([g["w1"].ravel(), g["b1"], g["w2"].ravel(), g["b2"], g["w3"], [g["b3"]]])
    rng = np.random.default_rng(9)

    def fd(j, h):
        fp = flat.copy(); fp[j] += h
        fm = flat.copy(); fm[j] -= h
        lp, _ = oracle.mlp_grad(oracle.MLP.from_flat(fp.astype(np.float32)), x, lab, wp, round_act=False)
        lm, _ = oracle.mlp_grad(oracle.MLP.from_flat(fm.astype(np.float32)), x, lab, wp, round_act=False)
        # parameters are stored in FP32: use the actually represented steps
        hp = float(np.float32(fp[j])) - flat[j]
        hm = flat[j] - float(np.float32(fm[j]))
        return (lp - lm) / (hp + hm)

    # a small batch keeps ReLU kinks away from most coordinates
    x, lab = x[:24], lab[:24]
    loss, g = oracle.mlp_grad(m, x, lab, w_pos=wp, round_act=False)
    gflat = np.concatenate([g["w1"].ravel(), g["b1"], g["w2"].ravel(), g["b2"], g["w3"], [g["b3"]]])
    checked = 0
    for j in rng.choice(len(flat), 60, replace=False):
        if j < 64 * 16 and (j % 16) >= 12:
            continue
        a, b = fd(j, 1e-4), fd(j, 2.5e-5)
        if abs(a - b) > 1e-3 * max(1.0, abs(b)):
            continue  # a ReLU kink inside the step: not differentiable there
        assert abs(b - gflat[j]) <= 1e-4 * max(1.0, abs(gflat[j])) + 1e-6, (j, b, gflat[j])
        checked += 1
    assert checked >= 30


def test_features_closed_form(geom):
    x, _ = geom
    xd, xi, xu = float(x[10]), float(x[11]), float(x[12])
    w = np.float32(np.float32(xi - xd) / np.float32(xu - xd))
    c2s = float(np.sqrt(np.float32(0.2)))
    # a straight line y = 0.5 (x - xd) + 1, t = 2 (x - xd): zero residual, zero curvature (up to rounding)
    yd, yi, yu = 1.0, 1.0 + 0.5 * (xi - xd), 1.0 + 0.5 * (xu - xd)
    td, ti, tu = 0.0, 2 * (xi - xd), 2 * (xu - xd)
    f = oracle.mlp_features(yd, td, xd, yi, ti, xi, yu, tu, xu, 1, 1.5, 2.0, float(w), c2s, 5)
    assert abs(f[6]) < 1e-3 and abs(f[7]) < 1e-3 and abs(f[8]) < 1e-2
    assert f[9] == oracle.bf16(np.float32(0.5)) and abs(f[10] - 2.0) < 1e-2
    assert f[4] == 1.0 and f[11] == oracle.bf16(np.float32(5 / 8))
    assert f[5] == oracle.bf16(np.float32(np.float32(xi) / np.float32(245.0)))
    assert (f[12:] == 0).all()
    # a circle of radius 100 through the three points: curvature feature = (1/100)/0.015
    R = 100.0
    pts = []
    for xx in (xd, xi, xu):
        pts.append(R - math.sqrt(R * R - (xx - 150.0) ** 2))
    f = oracle.mlp_features(np.float32(pts[0]), 0.0, xd, np.float32(pts[1]), 0.0, xi, np.float32(pts[2]), 0.0, xu,
                            1, 1.5, 2.0, float(w), c2s, 2)
    assert abs(abs(f[8]) - (1 / R) / 0.015) < 0.05 * (1 / R) / 0.015


def test_threshold_limits(ocfg):
    fr = synth.generate("sector_300", seed=2)
    row, y, t = fr.sector(0)
    m = oracle.MLP.random(1)
    up0, dn0, gap0 = oracle.links(ocfg, row, y, t)
    up, dn, gap, near = oracle.links_pruned(ocfg, row, y, t, m, -1e30)
    assert np.array_equal(up, up0) and np.array_equal(dn, dn0) and np.array_equal(gap, gap0)
    up, dn, gap, near = oracle.links_pruned(ocfg, row, y, t, m, 1e30)
    assert (up == -1).all() and (dn == -1).all()
    # pruned links are a choice among the accepted triplets
    tri, feat = oracle.triplets(ocfg, row, y, t)
    z = oracle.mlp_forward(m, feat)
    th = float(np.median(z))
    up, dn, gap, near = oracle.links_pruned(ocfg, row, y, t, m, th)
    keep = z >= th
    ok = set(map(tuple, tri[keep][:, [0, 1, 2]].tolist()))
    for i in np.nonzero(up >= 0)[0][:2000]:
        assert (dn[i], i, up[i]) in ok


def _torch_adamw(p0, grads, lr, betas, eps, wd):
    """torch.optim.AdamW in float64 with the weights decayed and the biases
    not (two parameter groups), over the given gradient sequence."""
    dm = oracle.decay_mask().astype(bool)
    pw = torch.tensor(p0[dm], dtype=torch.float64, requires_grad=True)
    pb = torch.tensor(p0[~dm], dtype=torch.float64, requires_grad=True)
    opt = torch.optim.AdamW([{"params": [pw], "weight_decay": wd}, {"params": [pb], "weight_decay": 0.0}],
                            lr=lr, betas=betas, eps=eps)
    out = []
    for g in grads:
        pw.grad = torch.tensor(g[dm], dtype=torch.float64)
        pb.grad = torch.tensor(g[~dm], dtype=torch.float64)
        opt.step()
        p = np.empty(len(p0))
        p[dm] = pw.detach().numpy()
        p[~dm] = pb.detach().numpy()
        out.append(p)
    return out


def test_adamw_matches_torch():
    """The oracle's AdamW step against torch.optim.AdamW (float64, CPU) over
    six steps with non-default betas, so that the bias corrections, the
    moment recursions and the step counter all matter; decay on the weights
    only."""
    rng = np.random.default_rng(21)
    p0 = rng.normal(0, 0.5, oracle.MLP_NPARAM)
    grads = [rng.normal(0, 1, oracle.MLP_NPARAM) * rng.choice([1e-3, 1.0, 30.0], oracle.MLP_NPARAM)
             for _ in range(6)]
    hp = dict(lr=1e-2, beta1=0.8, beta2=0.95, eps=1e-6, weight_decay=0.05)
    ref = _torch_adamw(p0, grads, hp["lr"], (hp["beta1"], hp["beta2"]), hp["eps"], hp["weight_decay"])
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for k, g in enumerate(grads):
        oracle.adamw_step(p, m, v, g, k + 1, **hp)
        assert np.allclose(p, ref[k], rtol=1e-12, atol=1e-14), k
    # planted mistakes are caught: a step counter stuck at 1, swapped betas,
    # decay applied to the biases too
    for bad in ("step", "betas", "decay"):
        p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
        kw = dict(hp)
        if bad == "betas":
            kw["beta1"], kw["beta2"] = hp["beta2"], hp["beta1"]
        for k, g in enumerate(grads):
            oracle.adamw_step(p, m, v, g, 1 if bad == "step" else k + 1,
                              decay=np.ones(oracle.MLP_NPARAM, np.uint8) if bad == "decay" else None, **kw)
        assert not np.allclose(p, ref[-1], rtol=1e-6, atol=1e-9), bad
