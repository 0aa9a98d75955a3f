"""GPU checks of the error contract: the device check passes on a gfx950,
the non-finite counters of tsne_knn, tsne_kl_grad, tsne_kl_grad_fft and
tsne_optimize count exactly the NaN / infinite coordinates they meet (plain
values planted in the inputs, nothing that can fault), the Python layer
turns a nonzero count into TSNE_ERR_NONFINITE, and the optimiser state
saved to disk resumes the trajectory bit for bit."""
import numpy as np
import pytest
import torch

from helpers import random_graph_P, say, sparse_to_dev, to_dev
from paper_2605_13928_amd import _lib, api, synth, tsne

pytestmark = pytest.mark.gpu


def test_device_is_supported(dev):
    L = _lib.load()
    x = torch.zeros((4, 2), dtype=torch.float32, device=dev)
    # a plain step on the current device: the gfx950 check passes
    _lib.check("tsne_step", L.tsne_step(x.data_ptr(), x.data_ptr(), x.data_ptr(), x.data_ptr(), 4, 200.0, 0.5, 0.2,
                                        0.8, 0.01, None))
    torch.cuda.synchronize()
    assert "gfx950" in torch.cuda.get_device_properties(dev).gcnArchName


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_knn_counts_nonfinite_entries(dev, precision):
    say("knn nonfinite", precision)
    X, _ = synth.make_points("c1", n=700)
    bad = api.nonfinite_counter(dev)
    api.knn(to_dev(X, dev), 30, precision, nonfinite=bad)
    assert int(bad.item()) == 0
    Xb = X.copy()
    rng = np.random.default_rng(3)
    cells = rng.choice(Xb.size, 17, replace=False)
    vals = np.array([np.nan, np.inf, -np.inf] * 6, dtype=np.float32)[:17]
    Xb.reshape(-1)[cells] = vals
    bad.fill_(12345)  # the call zeroes it first
    api.knn(to_dev(Xb, dev), 30, precision, nonfinite=bad)
    assert int(bad.item()) == 17


def test_affinities_raise_on_nonfinite_x(dev):
    w = synth.WORKLOADS["c1"]
    X, _ = synth.make_points(w, n=500)
    X[123, 7] = np.nan
    with pytest.raises(_lib.TsneError) as ei:
        tsne.affinities(to_dev(X, dev), w)
    assert ei.value.status == _lib.TSNE_ERR_NONFINITE


@pytest.mark.parametrize("n", [37, 5000])
def test_klgrad_counts_nonfinite_coordinates(dev, n):
    say("kl_grad nonfinite", n)
    _, _, _, S = random_graph_P(n, 30 if n > 100 else 10, 10.0 if n > 100 else 3.0, 77)
    P = sparse_to_dev(S, dev)
    Y = synth.random_embedding(n, 1.0, 78)
    bad, bad2 = api.nonfinite_counter(dev), api.nonfinite_counter(dev)
    api.kl_grad(to_dev(Y, dev), P, 1.0, nonfinite=bad)
    api.kl_grad_fft(to_dev(Y, dev), P, 1.0, nonfinite=bad2)
    assert int(bad.item()) == 0 and int(bad2.item()) == 0
    Yb = Y.copy()
    Yb[0, 0] = np.nan
    Yb[n - 1, 1] = np.inf
    Yb[n // 2, :] = -np.inf
    api.kl_grad(to_dev(Yb, dev), P, 1.0, nonfinite=bad)
    assert int(bad.item()) == 4
    Yb[n // 2, :] = 0.0
    api.kl_grad_fft(to_dev(Yb, dev), P, 1.0, nonfinite=bad2)
    assert int(bad2.item()) == 2


def test_optimize_counts_nonfinite_positions(dev):
    say("optimize nonfinite")
    n, iters = 3000, 5
    _, _, _, S = random_graph_P(n, 30, 10.0, 79)
    P = sparse_to_dev(S, dev)
    Y = to_dev(synth.random_embedding(n, 0.01, 80), dev)
    st = tsne.State.start(Y)
    tsne.iterate(st, P, synth.WORKLOADS["c1"], iters)
    assert int(st.nonfinite.item()) == 0
    st.check_finite()
    # one NaN coordinate makes Z, hence every gradient and every stepped
    # position, NaN from the first iteration on: 2 n per iteration
    Yb = Y.clone()
    Yb[17, 1] = float("nan")
    sb = tsne.State.start(Yb)
    tsne.iterate(sb, P, synth.WORKLOADS["c1"], iters)
    assert int(sb.nonfinite.item()) == 2 * n * iters
    with pytest.raises(_lib.TsneError) as ei:
        sb.check_finite()
    assert ei.value.status == _lib.TSNE_ERR_NONFINITE


def test_checkpoint_on_disk_resumes_bitwise(dev, tmp_path):
    say("checkpoint resume")
    w = synth.WORKLOADS["c1"]
    X, _ = synth.make_points(w)
    Xd = to_dev(X, dev)
    Y0 = to_dev(synth.make_init(w), dev)
    A = tsne.affinities(Xd, w)
    straight = tsne.iterate(tsne.State.start(Y0), A.P, w, 160, log_every=50)
    # interrupted inside the exaggeration phase, saved, reloaded, continued
    a = tsne.iterate(tsne.State.start(Y0), A.P, w, 70, log_every=50)
    path = str(tmp_path / "state.npz")
    tsne.save_checkpoint(path, a, A.P, w)
    b, Pb, wb = tsne.load_checkpoint(path, dev)
    assert wb == w and b.t == 70 and sorted(b.kl) == [49]
    assert torch.equal(Pb.col, A.P.col) and torch.equal(Pb.val, A.P.val) and torch.equal(Pb.tpos, A.P.tpos)
    tsne.iterate(b, Pb, w, 90, log_every=50)
    assert b.t == straight.t == 160
    for f in ("Y", "update", "gains"):
        assert torch.equal(getattr(b, f), getattr(straight, f)), f
    assert sorted(b.kl) == sorted(straight.kl) == [49, 99, 149]
    assert all(b.kl[t].item() == straight.kl[t].item() for t in b.kl)
    # the run driver: checkpoints every 40 iterations; a second call on the
    # same file resumes there (here: already done) without redoing the affinities
    ck = str(tmp_path / "run.npz")
    _, r1 = tsne.run(Xd, w, Y0, iters=160, checkpoint=ck, checkpoint_every=40)
    assert torch.equal(r1.Y, straight.Y)
    A2, r2 = tsne.run(Xd, w, Y0, iters=160, checkpoint=ck, checkpoint_every=40)
    assert A2 is None and r2.t == 160 and torch.equal(r2.Y, straight.Y)
    # a run cut short at 120 and restarted to 160 ends on the same bits
    ck2 = str(tmp_path / "cut.npz")
    tsne.run(Xd, w, Y0, iters=120, checkpoint=ck2, checkpoint_every=40)
    _, r3 = tsne.run(Xd, w, Y0, iters=160, checkpoint=ck2, checkpoint_every=40)
    assert torch.equal(r3.Y, straight.Y) and torch.equal(r3.gains, straight.gains)
