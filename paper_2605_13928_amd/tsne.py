"""The t-SNE run: kNN -> calibrated P -> symmetric P -> iterated gradient + step.

Orchestration only; every stage is one C-ABI call.  The schedule (early
exaggeration 12 with momentum 0.5 for the first 100 iterations, momentum 0.8
afterwards, learning rate 200, gains +0.2 / x0.8 / floor 0.01) follows the
standard optimiser of van der Maaten & Hinton 2008 (Sec. 3.4, Algorithm 1)
with Jacobs-style gains.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import api
from .synth import Workload


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
    """kNN, perplexity calibration and symmetrisation on device."""
    prec = precision or w.knn
    idx, d2 = api.knn(X, w.k, prec, n_cand=(w.candidates if prec == "bf16" else None), ws=ws)
    P_cond, beta, conv, nun = api.calibrate_P(d2, w.perplexity)
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

    @staticmethod
    def start(Y0: torch.Tensor) -> "State":
        Y = Y0.clone().contiguous()
        return State(Y, torch.zeros_like(Y), torch.ones_like(Y), torch.empty_like(Y))


def iterate(state: State, P: api.SparseP, w: Workload, iters: int, log_every: int = 0,
            ws: api.Workspace | None = None):
    """Run `iters` iterations from state.t in one native call (tsne_optimize);
    KL every log_every iterations lands in state.kl as device scalars."""
    t0, t1 = state.t, state.t + iters
    kl_log = torch.zeros(iters, dtype=torch.float64, device=state.Y.device) if log_every > 0 else None
    api.optimize(state.Y, state.update, state.gains, P, t0, t1, w.lr, w.exaggeration, w.exaggeration_iters,
                 w.momentum_early, w.momentum_late, log_every=log_every, kl_log=kl_log, ws=ws)
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
        log_every: int = 0):
    ws = api.Workspace()
    A = affinities(X, w, precision, ws)
    st = iterate(State.start(Y0), A.P, w, w.iters if iters is None else iters, log_every, ws)
    return A, st
