"""GPU test of the training-data path of the learned pruning: labels taken
from a pruned run with the threshold at -inf agree with the plain tracker's
chains, and a short training run on them separates the classes."""
import numpy as np
import pytest

from paper_2102_08862_amd import prune_train, synth

pytestmark = pytest.mark.gpu


def test_labels_match_chains_and_training_separates():
    import torch
    from paper_2102_08862_amd import tpcca
    fr = synth.generate("sector_300", seed=31)
    x, _ = synth.geometry()
    trk = tpcca.Tracker(row_x=x)
    trk.mlp_load(prune_train.init_params(1))
    trk.set_pruning(True, -1e30)
    trk.set_triplet_pool(True)
    f = trk.load_frame(fr, sectors=[0])
    trk.run(sync=True)
    xs, ys, n_all, n_pos = prune_train.frame_triplets(trk, f, 1, 1.0, np.random.default_rng(0))
    tr = trk.tracks(f, 0)
    # every interior chain cluster has exactly one positive triplet: its
    # cleaned (down, up) pair, which is its best pair and so was enumerated
    assert n_pos == int((tr["n_clusters"] - 2).sum())
    assert n_all == trk.stats()["n_triplets"] == len(ys)
    print("triplets %d, positive %d" % (n_all, n_pos))
    xd, yd = prune_train.to_device(xs, ys)
    z0 = prune_train.logits(trk, xd)
    hist, pw = prune_train.train(trk, xd, yd, epochs=40, batch=4096, lr=3e-3, every=10 ** 9)
    z = prune_train.logits(trk, xd)
    l0, l1 = prune_train.bce(z0, yd, pw), prune_train.bce(z, yd, pw)
    zp, zn = z[yd > 0.5].cpu().numpy(), z[yd < 0.5].cpu().numpy()
    # rank statistic: probability that a positive outscores a negative
    auc = (np.searchsorted(np.sort(zn), zp).sum()) / (len(zp) * len(zn))
    print("bce %.4f -> %.4f, auc %.4f" % (l0, l1, auc))
    assert l1 < 0.7 * l0 and auc > 0.9


def test_device_samples_match_host_labels():
    """The device sampler with keep = 1 returns every triplet with the same
    label as the host-side labelling; keep < 1 returns a reproducible subset
    of about that share."""
    from paper_2102_08862_amd import tpcca
    fr = synth.generate("sector_300", seed=32)
    x, _ = synth.geometry()
    trk = tpcca.Tracker(row_x=x)
    trk.mlp_load(prune_train.init_params(2))
    trk.set_pruning(True, -1e30)
    trk.set_triplet_pool(True)
    f = trk.load_frame(fr, sectors=[0])
    trk.run(sync=True)
    xs, ys, n_all, n_pos = prune_train.frame_triplets(trk, f, 1, 1.0, np.random.default_rng(0))
    fd, ld = trk.triplet_samples(1.0, 7, n_all + 10)
    assert len(ld) == n_all and int(ld.sum().item()) == n_pos

    def rows(feat, lab):
        a = np.concatenate([feat.view(np.uint16).astype(np.int64), lab[:, None].astype(np.int64)], axis=1)
        return a[np.lexsort(a.T[::-1])]
    assert np.array_equal(rows(fd.cpu().numpy(), ld.cpu().numpy()), rows(xs, ys))
    f1, l1 = trk.triplet_samples(0.25, 9, n_all)
    f2, l2 = trk.triplet_samples(0.25, 9, n_all)
    assert np.array_equal(rows(f1.cpu().numpy(), l1.cpu().numpy()), rows(f2.cpu().numpy(), l2.cpu().numpy()))
    assert abs(len(l1) / n_all - 0.25) < 0.02
