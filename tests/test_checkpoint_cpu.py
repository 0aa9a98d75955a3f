"""Host-side checks of the on-disk optimiser state (no GPU): the file holds
plain arrays only (loadable with allow_pickle=False), round-trips every field
exactly, and rejects files of another format or with mismatched shapes."""
import numpy as np
import pytest
import torch

from paper_2605_13928_amd import api, synth, tsne


def _state(n=50, t=123):
    g = torch.Generator().manual_seed(5)
    Y = torch.randn((n, 2), generator=g, dtype=torch.float32)
    U = torch.randn((n, 2), generator=g, dtype=torch.float32)
    G = torch.rand((n, 2), generator=g, dtype=torch.float32) + 0.01
    kl = {49: torch.tensor([1.25], dtype=torch.float64), 99: torch.tensor([0.75], dtype=torch.float64)}
    return tsne.State(Y, U, G, torch.empty_like(Y), t, kl)


def _P(n=50):
    idx, _ = synth.random_knn_graph(n, 5, 9)
    row_ptr = np.arange(0, 5 * n + 1, 5, dtype=np.int64)
    col = idx.reshape(-1).astype(np.int32)
    val = np.full(5 * n, 1.0 / (5 * n), dtype=np.float32)
    tpos = np.arange(5 * n, dtype=np.int32)
    return api.SparseP(torch.from_numpy(row_ptr), torch.from_numpy(col), torch.from_numpy(val),
                       torch.from_numpy(tpos), n)


def test_round_trip(tmp_path):
    st, P, w = _state(), _P(), synth.WORKLOADS["c2"]
    path = str(tmp_path / "s.npz")
    tsne.save_checkpoint(path, st, P, w)
    with np.load(path, allow_pickle=False) as f:  # plain arrays only
        assert set(f.files) >= {"format", "t", "Y", "update", "gains", "P_row_ptr", "P_col", "P_val", "workload"}
    b, Pb, wb = tsne.load_checkpoint(path, "cpu")
    assert b.t == 123 and wb == w
    for a in ("Y", "update", "gains"):
        assert torch.equal(getattr(b, a), getattr(st, a))
    assert sorted(b.kl) == [49, 99] and b.kl[49].item() == 1.25 and b.kl[99].item() == 0.75
    for a in ("row_ptr", "col", "val", "tpos"):
        assert torch.equal(getattr(Pb, a), getattr(P, a))
    assert Pb.n == P.n


def test_state_only_and_overwrite(tmp_path):
    path = str(tmp_path / "s.npz")
    tsne.save_checkpoint(path, _state(t=7))
    tsne.save_checkpoint(path, _state(t=8))  # replaced atomically
    b, Pb, wb = tsne.load_checkpoint(path, "cpu")
    assert b.t == 8 and Pb is None and wb is None


def test_rejects_bad_files(tmp_path):
    st = _state()
    p1 = str(tmp_path / "fmt.npz")
    np.savez(p1, format=np.array(99), t=np.array(0), Y=st.Y.numpy(), update=st.update.numpy(),
             gains=st.gains.numpy(), kl_t=np.zeros(0, np.int64), kl_val=np.zeros(0))
    with pytest.raises(ValueError):
        tsne.load_checkpoint(p1, "cpu")
    p2 = str(tmp_path / "shape.npz")
    np.savez(p2, format=np.array(tsne.CHECKPOINT_FORMAT), t=np.array(0), Y=st.Y.numpy(), update=st.update.numpy()[:3],
             gains=st.gains.numpy(), kl_t=np.zeros(0, np.int64), kl_val=np.zeros(0))
    with pytest.raises(ValueError):
        tsne.load_checkpoint(p2, "cpu")
    p3 = str(tmp_path / "P.npz")
    tsne.save_checkpoint(p3, st, _P(n=40))
    with pytest.raises(ValueError):
        tsne.load_checkpoint(p3, "cpu")
