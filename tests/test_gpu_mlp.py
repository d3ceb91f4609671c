"""GPU tests of the learned triplet pruning: the MFMA inference and training
kernels against the CPU oracle (FP64 with the same BF16 roundings), and the
pruned neighbour finder against the oracle's pruned links."""
import numpy as np
import pytest

import oracle
from paper_2102_08862_amd import synth

from _parity import compare_sector, oracle_cfg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    from paper_2102_08862_amd import tpcca
    assert torch.cuda.is_available()
    tpcca.load_library()
    return tpcca


@pytest.fixture(scope="module")
def x():
    return synth.geometry()[0]


def _feat(n, seed):
    rng = np.random.default_rng(seed)
    f = np.zeros((n, 16), np.float32)
    f[:, :12] = rng.normal(0, 1.5, (n, 12))
    return oracle.bf16(f)


def _to_dev_bf16(f):
    import torch
    bits = (f.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    return torch.from_numpy(bits.view(np.int16).copy()).cuda()


def test_infer_matches_oracle(tp):
    import torch
    m = oracle.MLP.random(11)
    f = _feat(20000, 1)
    trk = tp.Tracker()
    trk.mlp_load(m.flat())
    z = trk.mlp_infer(_to_dev_bf16(f)).cpu().numpy()
    zo = oracle.mlp_forward(m, f)
    bad = np.abs(z - zo) > 1e-3 * (1 + np.abs(zo))
    print("infer: max |dz| %.3g, beyond tolerance %d of %d" % (np.abs(z - zo).max(), bad.sum(), len(z)))
    assert bad.mean() <= 1e-3
    assert np.abs(z - zo).max() < 0.1


def test_grad_matches_oracle(tp):
    import torch
    m = oracle.MLP.random(12)
    n = 4096
    f = _feat(n, 2)
    y = (np.random.default_rng(3).random(n) < 0.2).astype(np.float32)
    trk = tp.Tracker()
    trk.mlp_load(m.flat())
    g, loss = trk.mlp_grad(_to_dev_bf16(f), torch.from_numpy(y).cuda(), pos_weight=3.0)
    g = g.cpu().numpy()
    lo, go = oracle.mlp_grad(m, f, y, w_pos=3.0)
    assert abs(loss.item() - lo) < 1e-3 * max(1.0, abs(lo))
    gflat = np.concatenate([go["w1"].ravel(), go["b1"], go["w2"].ravel(), go["b2"], go["w3"], [go["b3"]]])
    segs = {"w1": (0, 1024), "b1": (1024, 1088), "w2": (1088, 5184), "b2": (5184, 5248), "w3": (5248, 5312),
            "b3": (5312, 5313)}
    for k, (a, b) in segs.items():
        u, v = g[a:b].astype(np.float64), gflat[a:b]
        rel = np.linalg.norm(u - v) / max(np.linalg.norm(v), 1e-30)
        cos = float(u @ v / (np.linalg.norm(u) * np.linalg.norm(v) + 1e-300))
        print("grad %s: rel L2 %.2e cos %.6f" % (k, rel, cos))
        assert rel <= 1e-2 and (cos >= 0.9999 or b - a == 1), k


def test_train_steps_follow_adamw_oracle(tp):
    """Four AdamW steps on four minibatches with non-default betas against
    the FP64 AdamW oracle: each step's gradient is taken from the
    gradient-only call on the same weights and batch (the reduction order is
    fixed, so it is the gradient the update uses); the oracle carries its
    own FP64 moments through the steps, so wrong betas, a wrong bias
    correction or a step counter that does not advance fail from step 2 on."""
    import torch
    m = oracle.MLP.random(13)
    trk = tp.Tracker()
    trk.mlp_load(m.flat())
    hp = dict(lr=2e-3, beta1=0.8, beta2=0.95, eps=1e-7, weight_decay=0.05)
    p = m.flat().astype(np.float64)
    mo, vo = np.zeros_like(p), np.zeros_like(p)
    for k in range(4):
        n = [2048, 1000, 4096, 333][k]
        f = _feat(n, 40 + k)
        y = (np.random.default_rng(50 + k).random(n) < 0.3).astype(np.float32)
        xd, yd = _to_dev_bf16(f), torch.from_numpy(y).cuda()
        g, _ = trk.mlp_grad(xd, yd, pos_weight=2.0)
        g2, _ = trk.mlp_grad(xd, yd, pos_weight=2.0)
        assert torch.equal(g, g2), "gradient is not reproducible"
        trk.mlp_train_step(xd, yd, pos_weight=2.0, **hp)
        p1 = trk.mlp_fetch().astype(np.float64)
        oracle.adamw_step(p, mo, vo, g.cpu().numpy().astype(np.float64), k + 1, **hp)
        exp = p.copy()
        exp[:1024].reshape(64, 16)[:, 12:] = 0
        err = np.abs(p1 - exp)
        print("step %d: max |dp| %.3g" % (k + 1, err.max()))
        assert np.allclose(p1, exp, rtol=1e-5, atol=2e-6), k + 1
        # continue from the device's FP32 parameters (the oracle keeps its moments)
        p = p1.copy()

def test_training_reduces_loss(tp):
    """A separable toy task: label = (feature 0 + feature 6 > 0)."""
    import torch
    n = 8192
    f = _feat(n, 6)
    y = ((f[:, 0] + f[:, 6]) > 0).astype(np.float32)
    trk = tp.Tracker()
    trk.mlp_load(oracle.MLP.random(14).flat())
    xd, yd = _to_dev_bf16(f), torch.from_numpy(y).cuda()
    loss = torch.zeros(1, device="cuda")
    losses = []
    for step in range(300):
        trk.mlp_train_step(xd, yd, lr=3e-3, loss_dev=loss)
        if step % 50 == 0:
            losses.append(loss.item())
    print("losses", losses)
    assert losses[-1] < 0.5 * losses[0]
    z = trk.mlp_infer(xd).cpu().numpy()
    acc = ((z > 0) == (y > 0.5)).mean()
    assert acc > 0.95


def test_pruned_run_triplets_and_links(tp, x):
    fr = synth.generate("sector_300", seed=21)
    row, y, t = fr.sector(0)
    oc = oracle_cfg(x)
    m = oracle.MLP.random(15)
    # theta = -inf: no pruning, links identical to the plain finder
    trk = tp.Tracker(use_mlp=1, mlp_logit_threshold=-1e30)
    trk.set_triplet_pool(True)
    trk.mlp_load(m.flat())
    f = trk.add_frame()
    trk.load_sector(f, 0, row, y, t)
    trk.run(sync=True)
    st = trk.stats()
    assert st["mlp_used"] == 1 and st["n_pool_overflow"] == 0
    compare_sector(trk, f, 0, row, y, t, oc)
    tri, feat, z = trk.triplets(f, 0)
    otri, ofeat = oracle.triplets(oc, row, y, t)
    # the library lists a cluster's triplets of one gap by (down id, up id)
    o = np.lexsort((otri[:, 2], otri[:, 0], otri[:, 3], otri[:, 1]))
    otri, ofeat = otri[o], ofeat[o]
    assert np.array_equal(tri, otri), "triplet identities differ"
    gf = (feat.astype(np.uint32) << 16).view(np.float32)
    assert np.array_equal(gf, ofeat), "triplet features differ"
    zo = oracle.mlp_forward(m, ofeat)
    assert (np.abs(z - zo) > 1e-3 * (1 + np.abs(zo))).mean() <= 1e-3
    # a real threshold: links equal the oracle's except where a triplet sits at the threshold
    th = float(np.median(zo))
    trk2 = tp.Tracker(use_mlp=1, mlp_logit_threshold=th)
    trk2.mlp_load(m.flat())
    g = trk2.add_frame()
    trk2.load_sector(g, 0, row, y, t)
    trk2.run(sync=True)
    up, dn = trk2.links(g, 0)
    oup, odn, ogap, near = oracle.links_pruned(oc, row, y, t, m, th, tol=1e-3 * (1 + abs(th)))
    ok = near == 0
    print("pruned: %d of %d clusters compared, %d pruned triplets" % (ok.sum(), len(ok), trk2.stats()["n_pruned"]))
    assert ok.mean() > 0.99
    assert np.array_equal(up[ok], oup[ok]) and np.array_equal(dn[ok], odn[ok])
    # the same run through the triplet pool gives the same links everywhere
    trk2.set_triplet_pool(True)
    trk2.run(sync=True)
    up2, dn2 = trk2.links(g, 0)
    assert np.array_equal(up, up2) and np.array_equal(dn, dn2)


def _pruned_links(tp, fr, sectors, params, th, pool, **cfg):
    trk = tp.Tracker(use_mlp=1, mlp_logit_threshold=th, **cfg)
    trk.set_triplet_pool(pool)
    trk.mlp_load(params)
    f = trk.load_frame(fr, sectors=sectors)
    trk.run(sync=True)
    st = trk.stats()
    assert st["mlp_used"] == 1 and st["n_pool_overflow"] == 0
    return [trk.links(f, s) for s in sectors], [trk.assignment(f, s) for s in sectors], st


@pytest.mark.parametrize("which", ["random", "trained"])
def test_pruned_search_equals_pool_path(tp, x, which):
    """Scoring inside the search (gap 2 only where no gap-1 triplet
    survives) gives bit-identical links and assignment to scoring every
    triplet from the pool, over a 1 ms slice and at a threshold that prunes
    a large share."""
    from paper_2102_08862_amd import prune_train
    fr = synth.generate("slice_1ms", seed=22)
    secs = [0, 7, 20, 35]
    if which == "trained":
        params, meta = prune_train.load_weights()
        assert params is not None, "trained weights missing"
        th = float(meta["theta"])
    else:
        m = oracle.MLP.random(16)
        params = m.flat()
        th = 0.0
    la, aa, sa = _pruned_links(tp, fr, secs, params, th, False, row_x=x)
    lb, ab, sb = _pruned_links(tp, fr, secs, params, th, True, row_x=x)
    print("%s: scored %d of %d triplets, pruned %d / %d" % (which, sa["n_triplets"], sb["n_triplets"],
                                                           sa["n_pruned"], sb["n_pruned"]))
    assert 0 < sa["n_triplets"] <= sb["n_triplets"] and sa["n_pruned"] > 0
    assert sa["n_links"] == sb["n_links"]
    for (u1, d1), (u2, d2), a1, a2 in zip(la, lb, aa, ab):
        assert np.array_equal(u1, u2) and np.array_equal(d1, d2)
        assert np.array_equal(a1, a2)


def test_pruned_search_dense_tiles(tp, x):
    """Tiles too dense for LDS take the global-memory pruned search: still
    identical to the pool path."""
    rng = np.random.default_rng(12)
    n = 12000
    row = rng.integers(20, 26, n).astype(np.uint8)
    y = (np.round(rng.uniform(-20, 20, n) * 64) / 64).astype(np.float32)
    t = (np.round(rng.uniform(0, 40, n) * 64) / 64).astype(np.float32)
    fr = synth.generate("sector_300", seed=4)
    r0, y0, t0 = fr.sector(0)
    row = np.concatenate([row, r0]); y = np.concatenate([y, y0]); t = np.concatenate([t, t0])
    m = oracle.MLP.random(17)
    res = []
    for pool in (False, True):
        print("case dense pruned, pool %d" % pool, flush=True)
        trk = tp.Tracker(use_mlp=1, mlp_logit_threshold=0.0, row_x=x, pool_per_cluster=64, min_track_hits=3)
        trk.set_triplet_pool(pool)
        trk.mlp_load(m.flat())
        f = trk.add_frame()
        trk.load_sector(f, 0, row, y, t)
        trk.run(sync=True)
        st = trk.stats()
        assert st["n_overflow_tiles"] > 0 and st["n_pool_overflow"] == 0
        res.append((trk.links(f, 0), trk.assignment(f, 0), st))
    ((u1, d1), a1, s1), ((u2, d2), a2, s2) = res
    print("dense: %d overflow tiles, links %d, scored %d of %d" % (s1["n_overflow_tiles"], s1["n_links"],
                                                                  s1["n_triplets"], s2["n_triplets"]))
    assert np.array_equal(u1, u2) and np.array_equal(d1, d2) and np.array_equal(a1, a2)
