"""The t-SNE run: kNN -> calibrated P -> symmetric P -> iterated gradient + step.

Orchestration only; every stage is one C-ABI call.  The schedule (early
exaggeration 12 with momentum 0.5 for the first 100 iterations, momentum 0.8
afterwards, learning rate 200, gains +0.2 / x0.8 / floor 0.01) follows the
standard optimiser of van der Maaten & Hinton 2008 (Sec. 3.4, Algorithm 1)
with Jacobs-style gains.
"""
from __future__ import annotations

import dataclasses
import json
import os
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api
from .synth import Workload

CHECKPOINT_FORMAT = 1


def schedule(w: Workload, t: int):
    early = t < w.exaggeration_iters
    return (w.exaggeration if early else 1.0), (w.momentum_early if early else w.momentum_late)


@dataclass
class Affinities:
    nbr_idx: torch.Tensor
    nbr_d2: torch.Tensor
    P_cond: torch.Tensor
    beta: torch.Tensor
    converged: torch.Tensor
    n_unconverged: torch.Tensor
    P: api.SparseP


def affinities(X: torch.Tensor, w: Workload, precision: str | None = None, ws: api.Workspace | None = None):
    """kNN, perplexity calibration and symmetrisation on device.  Raises
    TsneError (TSNE_ERR_NONFINITE) when X holds NaN or infinite entries (one
    synchronisation before the symmetrisation, which would otherwise reject
    the incomplete neighbour lists of such rows)."""
    prec = precision or w.knn
    bad = api.nonfinite_counter(X.device)
    idx, d2 = api.knn(X, w.k, prec, n_cand=(w.candidates if prec == "bf16" else None), ws=ws, nonfinite=bad)
    P_cond, beta, conv, nun = api.calibrate_P(d2, w.perplexity)
    api.raise_if_nonfinite(bad, "tsne_knn: X")
    P = api.symmetrize(idx, P_cond, ws=ws)
    return Affinities(idx, d2, P_cond, beta, conv, nun, P)


@dataclass
class State:
    Y: torch.Tensor
    update: torch.Tensor
    gains: torch.Tensor
    grad: torch.Tensor
    t: int = 0
    kl: dict = field(default_factory=dict)
    nonfinite: torch.Tensor | None = None  # int64 [1]: NaN/inf coordinates the last iterate() produced

    @staticmethod
    def start(Y0: torch.Tensor) -> "State":
        Y = Y0.clone().contiguous()
        return State(Y, torch.zeros_like(Y), torch.ones_like(Y), torch.empty_like(Y))

    def check_finite(self):
        """Synchronises and raises TsneError (TSNE_ERR_NONFINITE) if the
        last iterate() produced a NaN or infinite coordinate."""
        api.raise_if_nonfinite(self.nonfinite, f"tsne_optimize up to t = {self.t}")


def save_checkpoint(path: str, state: State, P: api.SparseP | None = None, w: Workload | None = None):
    """Writes the optimiser state (Y, update, gains, t, the logged KL values),
    and optionally P's CSR and the workload, to an .npz file.  Resuming from
    it continues the same trajectory bit for bit (the kernels are
    deterministic and the state is the whole of what an iteration reads).
    Synchronises (copies device tensors to the host); the file is written
    to a temporary name and renamed, so a crash leaves the old one intact."""
    arrs = {
        "format": np.array(CHECKPOINT_FORMAT, dtype=np.int64),
        "t": np.array(state.t, dtype=np.int64),
        "Y": state.Y.detach().cpu().numpy(),
        "update": state.update.detach().cpu().numpy(),
        "gains": state.gains.detach().cpu().numpy(),
        "kl_t": np.array(sorted(state.kl), dtype=np.int64),
        "kl_val": np.array([float(state.kl[t].reshape(-1)[0]) for t in sorted(state.kl)], dtype=np.float64),
    }
    if P is not None:
        arrs.update(P_n=np.array(P.n, dtype=np.int64), P_row_ptr=P.row_ptr.cpu().numpy(), P_col=P.col.cpu().numpy(),
                    P_val=P.val.cpu().numpy())
        if P.tpos is not None:
            arrs["P_tpos"] = P.tpos.cpu().numpy()
    if w is not None:
        arrs["workload"] = np.array(json.dumps(dataclasses.asdict(w)))
    tmp = path + ".tmp.npz"
    np.savez(tmp, **arrs)
    os.replace(tmp, path)


def load_checkpoint(path: str, device) -> tuple[State, api.SparseP | None, Workload | None]:
    """Reads a file written by save_checkpoint (no pickled objects) and puts
    the state (and P, if saved) on `device`."""
    with np.load(path, allow_pickle=False) as f:
        if int(f["format"]) != CHECKPOINT_FORMAT:
            raise ValueError(f"{path}: checkpoint format {int(f['format'])}, expected {CHECKPOINT_FORMAT}")

        def dev(a):
            return torch.from_numpy(np.ascontiguousarray(a)).to(device)

        Y, U, G = dev(f["Y"]), dev(f["update"]), dev(f["gains"])
        if not (Y.dtype == U.dtype == G.dtype == torch.float32 and Y.shape == U.shape == G.shape
                and Y.dim() == 2 and Y.shape[1] == 2):
            raise ValueError(f"{path}: Y, update and gains must be float32 [n, 2]")
        kl = {int(t): torch.tensor([v], dtype=torch.float64, device=device)
              for t, v in zip(f["kl_t"].tolist(), f["kl_val"].tolist())}
        st = State(Y, U, G, torch.empty_like(Y), int(f["t"]), kl)
        P = None
        if "P_row_ptr" in f:
            P = api.SparseP(dev(f["P_row_ptr"]), dev(f["P_col"]), dev(f["P_val"]),
                            dev(f["P_tpos"]) if "P_tpos" in f else None, int(f["P_n"]))
            if P.n != Y.shape[0] or P.row_ptr.shape[0] != P.n + 1:
                raise ValueError(f"{path}: P does not match Y")
        w = Workload(**json.loads(str(f["workload"]))) if "workload" in f else None
    return st, P, w


def iterate(state: State, P: api.SparseP, w: Workload, iters: int, log_every: int = 0,
            ws: api.Workspace | None = None):
    """Run `iters` iterations from state.t in one native call (tsne_optimize);
    KL every log_every iterations lands in state.kl as device scalars."""
    t0, t1 = state.t, state.t + iters
    kl_log = torch.zeros(iters, dtype=torch.float64, device=state.Y.device) if log_every > 0 else None
    if state.nonfinite is None:
        state.nonfinite = api.nonfinite_counter(state.Y.device)
    api.optimize(state.Y, state.update, state.gains, P, t0, t1, w.lr, w.exaggeration, w.exaggeration_iters,
                 w.momentum_early, w.momentum_late, log_every=log_every, kl_log=kl_log, ws=ws,
                 nonfinite=state.nonfinite)
    if kl_log is not None:
        for t in range(t0, t1):
            if (t + 1) % log_every == 0:
                state.kl[t] = kl_log[t - t0:t - t0 + 1]
    state.t = t1
    return state


def iterate_calls(state: State, P: api.SparseP, w: Workload, iters: int, log_every: int = 0,
                  ws: api.Workspace | None = None):
    """The same iterations as separate tsne_kl_grad / tsne_step calls."""
    ws = ws or api.Workspace()
    for _ in range(iters):
        t = state.t
        alpha, mom = schedule(w, t)
        want = log_every > 0 and (t + 1) % log_every == 0
        _, _, kl, _ = api.kl_grad(state.Y, P, alpha, grad=state.grad, want_kl=want, ws=ws)
        if want:
            state.kl[t] = kl
        api.step(state.Y, state.update, state.gains, state.grad, w.lr, mom)
        state.t += 1
    return state


def run(X: torch.Tensor, w: Workload, Y0: torch.Tensor, iters: int | None = None, precision: str | None = None,
        log_every: int = 0, checkpoint: str | None = None, checkpoint_every: int = 0):
    """The whole path.  With `checkpoint` and checkpoint_every > 0 the state
    is saved there every checkpoint_every iterations (and at the end); when
    the file already exists the run resumes from it instead of starting
    over (its P is reused and the affinity stage skipped).  Raises
    TsneError (TSNE_ERR_NONFINITE) if X or the embedding becomes non-finite."""
    ws = api.Workspace()
    total = w.iters if iters is None else iters
    if checkpoint and os.path.exists(checkpoint):
        st, P, _ = load_checkpoint(checkpoint, X.device)
        if P is None:
            raise ValueError(f"{checkpoint} holds no P")
        A = None
    else:
        A = affinities(X, w, precision, ws)
        st, P = State.start(Y0), A.P
    chunk = checkpoint_every if (checkpoint and checkpoint_every > 0) else total
    while st.t < total:
        iterate(st, P, w, min(chunk, total - st.t), log_every, ws)
        st.check_finite()
        if checkpoint and checkpoint_every > 0:
            save_checkpoint(checkpoint, st, P, w)
    return A, st
