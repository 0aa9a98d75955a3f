"""Benchmark of the exact t-SNE hot path on one MI355X.

The headline workload is the full-scale one: 1,000,000 points x 50
dimensions shaped like PCA scores of a cell population, BF16-MFMA kNN
(k = 90, 180 candidates re-ranked in FP32), perplexity 30, then 1000
iterations of the exact all-pairs gradient and the optimiser step.  Inputs
are generated and uploaded before anything is timed.

The one-off affinity stage (kNN, calibration, symmetrisation) runs once and
is timed on its own with HIP events (`affinity_s`, `knn_build_s`).  A timed
step is then a slice of `--slice` consecutive iterations of the schedule
(gradient + step, through tsne_optimize), continuing from where the
previous step stopped: the warmup steps run iterations [0, W s), the timed
ones the next K s, so the early-exaggeration phase and the late phase are
both covered.  For workloads small enough to run whole (n <= 100,000 by
default) a step is instead the whole path: kNN, calibration,
symmetrisation and every iteration.  `value` = ordered pair interactions
evaluated by the gradient over the timed steps / wall time of those steps.
tsne_optimize records HIP events (on the stream the kernels are launched
on) right around launches of the all-pairs repulsion kernel: they give the
dominant kernel's average per-launch time for the roofline.

Outside the timed region: the FP32 exact kNN at the same size (the
BF16-vs-FP32 build comparison and its agreement), the same comparison at
the 200,000-point shape, the CPU-baseline leg (the FP64 oracle timed on a
bounded sample of the same workload, which also yields the error
statistics), the KL autograd timing, the interpolated (FFT) gradient timed
against the exact one, the PCA that produces the embedding's input (200k
cells x 2000 genes, 50 components, 2 power iterations), and UMAP on the
same points (k = 15 neighbour graph, fuzzy union, 200 epochs).  Those legs
run under the resource monitor (0.1 s samples), whose per-leg summary (GPU
activity, VRAM, power, CPU) is the record's `telemetry`.  The CPU-baseline
leg also times the FP64 oracles of the widened rows (interpolated
repulsion, PCA, one UMAP epoch) on bounded samples of the same recipes,
beside the GPU figures (`cpu_baseline.widened_rows`).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5] [--slice S]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak
# the all-pairs kernel's instruction-issue ceiling without packed FP32: 17
# flops per unordered pair over its 10 non-transcendental VALU instructions,
# each one 4-cycle issue slot of a 64-lane wave, the reciprocal running on
# the transcendental unit beside them; 1024 SIMDs, 2.4 GHz
ISSUE_FLOOR_TFLOPS = 17.0 * 64 / (10 * 4) * 1024 * 2.4e9 / 1e12
BF16_PEAK_TFLOPS = 2500.0  # dense
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--slice", type=int, default=None,
                    help="iterations per timed step (default: the whole path for n <= 100000, else 10)")
    ap.add_argument("--knn-fp32-same-n", type=int, default=1,
                    help="also time the FP32 exact kNN at the workload's own size (0: skip)")
    ap.add_argument("--iters", type=int, default=None, help="override the schedule's iteration count")
    ap.add_argument("--knn-compare-n", type=int, default=200_000,
                    help="point count of the BF16-vs-FP32 kNN build comparison (C3 shape)")
    ap.add_argument("--autograd-n", type=int, default=50_000,
                    help="point count of the KL autograd forward/backward timing (0: skip)")
    ap.add_argument("--fft-n", type=int, default=1_000_000,
                    help="point count of the interpolated-vs-exact gradient comparison (C5 shape; 0: skip)")
    ap.add_argument("--pca-n", type=int, default=200_000,
                    help="cells of the PCA timing (tsne_pca, k = 50 of 64, q = 2; 0: skip)")
    ap.add_argument("--pca-g", type=int, default=2000, help="genes of the PCA timing")
    ap.add_argument("--umap-n", type=int, default=1_000_000,
                    help="points of the UMAP timing (c5 shape, k = 15, 200 epochs; 0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-monitor", action="store_true",
                    help="skip the telemetry (GPU activity, VRAM, power per leg) of the legs after the timed region")
    ap.add_argument("--cpu-iters", type=int, default=30)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="launch one device copy of this many MiB first (reference for HBM byte counters)")
    return ap.parse_args()


def source_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


KLGRAD_SOURCES = ["paper_2605_13928_amd/csrc/klgrad.hip", "paper_2605_13928_amd/csrc/klgrad.hpp",
                  "paper_2605_13928_amd/csrc/rep_sym.hpp", "paper_2605_13928_amd/csrc/common.hpp"]


def traffic_from_profile(digest, workload):
    """HBM bytes per launch of the all-pairs kernel from the committed PMC
    summary of this workload, if it was taken on the current kernel source;
    else None."""
    p = os.path.join(ROOT, "profiles", f"rep_sym_{workload}_traffic.txt")
    if not os.path.exists(p):
        return None
    vals = {}
    for line in open(p):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_digest") != digest:
        return None
    try:
        return float(vals["hbm_bytes_per_call"].split()[0])
    except (KeyError, ValueError):
        return None


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2605_13928_amd import api, synth, tsne

    dev = torch.device("cuda:0")
    w = synth.WORKLOADS[args.workload]
    iters = w.iters if args.iters is None else args.iters
    n = w.n
    whole = args.slice is None and n <= 100_000
    sl = iters if whole else (args.slice or 10)
    if not whole and (args.warmup + args.steps) * sl > iters:
        print(json.dumps({"error": f"warmup + steps = {args.warmup + args.steps} slices of {sl} iterations "
                                   f"exceed the schedule's {iters} iterations"}), flush=True)
        sys.exit(2)
    X_np, labels = synth.make_points(w)
    Y0_np = synth.make_init(w)
    X = torch.from_numpy(X_np).to(dev)
    Y0 = torch.from_numpy(Y0_np).to(dev)
    ws = api.Workspace()
    stream = torch.cuda.current_stream(dev)
    if args.copy_calibration_mib:
        # reads and writes exactly MiB * 2^20 bytes each (the MulFunctor elementwise kernel)
        src = torch.ones(args.copy_calibration_mib * (1 << 18), dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    ws_opt = api.Workspace()

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def affinity_stage():
        """kNN, calibration, symmetrisation (one host sync to read nnz)."""
        t = [ev() for _ in range(4)]
        t[0].record(stream)
        idx, d2 = api.knn(X, w.k, w.knn, n_cand=(w.candidates if w.knn == "bf16" else None), ws=ws)
        t[1].record(stream)
        Pc, beta, conv, nun = api.calibrate_P(d2, w.perplexity)
        t[2].record(stream)
        P = api.symmetrize(idx, Pc, want_tpos=False, ws=ws)
        t[3].record(stream)
        return t, P, idx, d2, Pc

    def new_events(count):
        # created (recorded once) up front, so none is created in the timed region
        out = [ev() for _ in range(2 * count)]
        for e in out:
            e.record(stream)
        return out

    if whole:
        # a step is the whole path: affinities, then every iteration
        EVERY = 10  # an event pair around every 10th all-pairs launch (events cost ~5 % of a 20k iteration)
        timed_iters = list(range(0, iters, EVERY))

        def one_step(events):
            t, P, idx, d2, Pc = affinity_stage()
            st = tsne.State.start(Y0)
            t4, t5 = ev(), ev()
            t4.record(stream)
            api.optimize(st.Y, st.update, st.gains, P, 0, iters, w.lr, w.exaggeration, w.exaggeration_iters,
                         w.momentum_early, w.momentum_late, events=events, ws=ws_opt)
            t5.record(stream)
            return (t[0], t[1], t[3], t4, t5), P, idx, d2, Pc

        for _ in range(args.warmup):
            one_step(None)
        torch.cuda.synchronize()
        progress(f"{args.warmup} warmup step(s) done")
        evs_all = []
        for _ in range(args.steps):
            evs = [None] * (2 * iters)
            pairs = new_events(len(timed_iters))
            for q, i in enumerate(timed_iters):
                evs[2 * i], evs[2 * i + 1] = pairs[2 * q], pairs[2 * q + 1]
            evs_all.append(evs)
        marks = []
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for s_ in range(args.steps):
            m, P, idx, d2, Pc = one_step(evs_all[s_])
            marks.append(m)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        grad_ms = np.array([evs_all[s_][2 * i].elapsed_time(evs_all[s_][2 * i + 1])
                            for s_ in range(args.steps) for i in timed_iters])
        knn_s = float(np.median([m[0].elapsed_time(m[1]) for m in marks])) / 1e3
        aff_s = float(np.median([m[0].elapsed_time(m[2]) for m in marks])) / 1e3
        iter_ms = float(np.median([m[3].elapsed_time(m[4]) for m in marks])) / iters
        iters_per_step = iters
        step_desc = "the whole path: kNN, calibration, symmetrisation and all iterations"
    else:
        # the one-off affinity stage, timed once after one untimed run
        affinity_stage()
        torch.cuda.synchronize()
        reps = []
        for _ in range(3):
            t, P, idx, d2, Pc = affinity_stage()
            torch.cuda.synchronize()
            reps.append((t[0].elapsed_time(t[1]), t[1].elapsed_time(t[2]), t[2].elapsed_time(t[3])))
        knn_s, cal_ms, sym_ms = (float(np.median([r[q] for r in reps])) for q in range(3))
        knn_s /= 1e3
        aff_s = knn_s + (cal_ms + sym_ms) / 1e3
        progress(f"affinity stage: kNN {knn_s:.3f} s, calibration {cal_ms:.2f} ms, symmetrisation {sym_ms:.2f} ms")
        st = tsne.State.start(Y0)

        def one_step(events):
            t0_ = st.t
            api.optimize(st.Y, st.update, st.gains, P, t0_, t0_ + sl, w.lr, w.exaggeration, w.exaggeration_iters,
                         w.momentum_early, w.momentum_late, events=events, ws=ws_opt)
            st.t = t0_ + sl

        for _ in range(args.warmup):
            one_step(None)
        torch.cuda.synchronize()
        progress(f"{args.warmup} warmup step(s) of {sl} iterations done (t = {st.t})")
        evs_all = [new_events(sl) for _ in range(args.steps)]
        t_first = st.t
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for s_ in range(args.steps):
            one_step(evs_all[s_])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        grad_ms = np.array([e[2 * i].elapsed_time(e[2 * i + 1]) for e in evs_all for i in range(sl)])
        iter_ms = elapsed * 1e3 / (args.steps * sl)
        iters_per_step = sl
        step_desc = (f"{sl} consecutive iterations of the {iters}-iteration schedule (gradient + step, "
                     f"tsne_optimize); timed steps ran t = {t_first}..{st.t - 1}; the one-off affinity stage "
                     f"(kNN, calibration, symmetrisation) is timed separately in affinity_s")
    progress(f"{args.steps} timed step(s): {elapsed:.3f} s")

    pairs_per_step = float(n) * float(n - 1) * iters_per_step
    value = pairs_per_step * args.steps / elapsed
    grad_ms_mean = float(grad_ms.mean())
    flops_per_call = api.KLGRAD_FLOPS_PER_ORDERED_PAIR * float(n) * float(n - 1)
    achieved_tflops = flops_per_call / (grad_ms_mean * 1e-3) / 1e12
    digest = source_digest(KLGRAD_SOURCES)
    traffic = traffic_from_profile(digest, args.workload)

    # --- telemetry of the legs below (outside the timed region) -----------
    mon = None
    if not args.no_monitor:
        from paper_2605_13928_amd import monitor as _monitor

        mon = _monitor.Monitor(period=0.1, device=dev.index or 0)  # CSV files in a fresh temporary directory

    def phase(name):
        if mon is not None:
            mon.timestamp(name)

    # --- BF16-MFMA vs FP32 kNN build, outside the timed region -------------
    phase("knn_compare")

    def p_diff(PA, PB, nn):
        """L1 of PA - PB over the union pattern and the largest relative
        difference over common entries (on the device)."""
        def keys(P):
            rows = torch.repeat_interleave(torch.arange(nn, device=dev), P.row_ptr[1:] - P.row_ptr[:-1])
            return rows * nn + P.col.long()
        ka, kb = keys(PA), keys(PB)
        kk = torch.cat([ka, kb])
        vv = torch.cat([PA.val.double(), -PB.val.double()])
        uk, inv = torch.unique(kk, return_inverse=True)
        acc = torch.zeros(uk.numel(), dtype=torch.float64, device=dev).index_add_(0, inv, vv)
        cnt = torch.zeros(uk.numel(), dtype=torch.int32, device=dev).index_add_(
            0, inv, torch.ones_like(inv, dtype=torch.int32))
        l1 = float(acc.abs().sum())
        va = torch.zeros(uk.numel(), dtype=torch.float64, device=dev).index_add_(0, inv[:ka.numel()],
                                                                               PA.val.double())
        common = cnt == 2
        rel = float((acc[common].abs() / va[common]).max()) if bool(common.any()) else 0.0
        return l1, rel

    def knn_compare(Xc, nn, reps32, reps16, wsk, label):
        def time_knn(prec, reps):
            out = None
            ts = []
            for r in range(reps + 1):
                a_, b_ = ev(), ev()
                a_.record(stream)
                out = api.knn(Xc, 90, prec, n_cand=(180 if prec == "bf16" else None), ws=wsk)
                b_.record(stream)
                torch.cuda.synchronize()
                if r > 0:
                    ts.append(a_.elapsed_time(b_) / 1e3)
            return float(np.median(ts)), out

        t32, (i32, d32) = time_knn("fp32", reps32)
        t16, (i16, d16) = time_knn("bf16", reps16)
        a32 = torch.sort(i32.long(), 1).values
        a16 = torch.sort(i16.long(), 1).values
        hits = 0
        for r0 in range(0, nn, 100_000):
            pos = torch.searchsorted(a32[r0:r0 + 100_000], a16[r0:r0 + 100_000]).clamp(max=89)
            hits += int((torch.gather(a32[r0:r0 + 100_000], 1, pos) == a16[r0:r0 + 100_000]).sum())
        same_rows = (a16 == a32).all(1)
        P32 = api.symmetrize(i32, api.calibrate_P(d32, 30.0)[0], want_tpos=False, ws=wsk)
        P16 = api.symmetrize(i16, api.calibrate_P(d16, 30.0)[0], want_tpos=False, ws=wsk)
        l1, prel = p_diff(P16, P32, nn)
        dsame = None
        if bool(same_rows.any()):
            d32s, d16s = d32[same_rows].double(), d16[same_rows].double()
            dsame = float(((d16s - d32s).abs() / d32s.clamp(min=1e-30)).max())
        # the dense formulation's MFMA work; both paths skip the tiles their
        # box test rules out, so this is an equivalent rate, not executed work
        dense_flops = 2.0 * nn * nn * 64
        progress(f"kNN comparison at n={nn} done")
        return {"n": nn, "workload": label, "k": 90, "n_cand": 180, "fp32_exact_s": t32, "bf16_mfma_rerank_s": t16,
                "speedup": t32 / t16, "bf16_vs_fp32_set_agreement": hits / (nn * 90.0),
                "bf16_vs_fp32_rows_identical": float(same_rows.double().mean()),
                "bf16_vs_fp32_d2_max_rel_identical_rows": dsame,
                "bf16_vs_fp32_P_L1": l1, "bf16_vs_fp32_P_max_rel_common": prel,
                "bf16_dense_equivalent_tflops": dense_flops / t16 / 1e12}

    knn_cmp = {"in_workload_s": knn_s, "precision": w.knn}
    if w.knn == "bf16" and args.knn_fp32_same_n:
        knn_cmp.update(knn_compare(X, n, 1, 3, ws, f"{w.name} (the benchmark's own points)"))
    ncmp = args.knn_compare_n
    if ncmp:
        Xc_np, _ = synth.make_points("c3", n=ncmp)
        Xc = torch.from_numpy(Xc_np).to(dev)
        knn_cmp["c3_shape"] = knn_compare(Xc, ncmp, 3, 5, api.Workspace(), "c3 shape (30 equal clusters)")
        del Xc

    phase("autograd")
    # --- differentiation form (KL autograd) at the 50k-point shape ----------
    diff = {}
    if args.autograd_n:
        from paper_2605_13928_amd.autograd import kl_divergence

        wd = synth.WORKLOADS["c4"]
        nd = args.autograd_n
        Xd = torch.from_numpy(synth.make_points(wd, n=nd)[0]).to(dev)
        wsd = api.Workspace()
        idd, d2d = api.knn(Xd, wd.k, "fp32", ws=wsd)
        Pd = api.symmetrize(idd, api.calibrate_P(d2d, wd.perplexity)[0], want_tpos=True, ws=wsd)
        Yd = torch.from_numpy(synth.make_init(wd, n=nd)).to(dev).requires_grad_(True)
        vd = Pd.val.clone().requires_grad_(True)
        fw, bw = [], []
        for r in range(6):
            Yd.grad = None
            vd.grad = None
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            c = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            C = kl_divergence(Yd, vd, Pd)
            b.record(stream)
            C.backward()
            c.record(stream)
            torch.cuda.synchronize()
            if r > 0:
                fw.append(a.elapsed_time(b))
                bw.append(b.elapsed_time(c))
        pairs_d = float(nd) * (nd - 1)
        diff = {"n": nd, "nnz": int(Pd.nnz), "forward_ms": float(np.median(fw)), "backward_ms": float(np.median(bw)),
                "forward_pairs_per_s": pairs_d / (np.median(fw) * 1e-3),
                "backward_pairs_per_s": pairs_d / (np.median(bw) * 1e-3), "KL": float(C.item())}
        del Xd, Yd, vd, Pd, idd, d2d
        progress(f"autograd timing at n={nd} done")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            out = fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts)), out

    # --- interpolated repulsion (tsne_kl_grad_fft) against the exact pass ---
    phase("interpolated_gradient")
    interp = {}
    if args.fft_n:
        wf = synth.WORKLOADS["c5"]
        nf = args.fft_n
        Xf = torch.from_numpy(synth.make_points(wf, n=nf)[0]).to(dev)
        wsf = api.Workspace()
        idf, d2f = api.knn(Xf, wf.k, "bf16", n_cand=wf.candidates, ws=wsf)
        Pf = api.symmetrize(idf, api.calibrate_P(d2f, wf.perplexity)[0], ws=wsf)
        del Xf, idf, d2f
        wse, wsi = api.Workspace(), api.Workspace()

        def compare_at(Yf):
            te, (ge, Ze, _, _) = timed(lambda: api.kl_grad(Yf, Pf, 1.0, want_Z=True, ws=wse), 3)
            tf, (gf, Zf, _) = timed(lambda: api.kl_grad_fft(Yf, Pf, 1.0, want_Z=True, ws=wsi), 10)
            return {"exact_ms": te, "interpolated_ms": tf, "speedup": te / tf,
                    "grad_rel_err_vs_exact": float(torch.linalg.norm(gf - ge) / torch.linalg.norm(ge)),
                    "Z_rel_err_vs_exact": abs(Zf.item() - Ze.item()) / Ze.item()}

        # the state of a run: 500 iterations of the interpolated optimiser
        # (the c5 schedule) from the standard start, where P-neighbours sit
        # close together in the embedding
        late_iters = 500
        st_f = tsne.State.start(torch.from_numpy(synth.make_init(wf, n=nf)).to(dev))
        for t in range(late_iters):
            alpha, mom = tsne.schedule(wf, t)
            api.kl_grad_fft(st_f.Y, Pf, alpha, grad=st_f.grad, ws=wsi)
            api.step(st_f.Y, st_f.update, st_f.gains, st_f.grad, wf.lr, mom)
        torch.cuda.synchronize()
        interp = {"n": nf, "nnz": int(Pf.nnz),
                  "embedding": f"the state after {late_iters} iterations of the interpolated optimiser "
                               f"(c5 schedule, standard start)",
                  "n_interp": 3, "min_boxes": 50, "max_box_width": 1.0, "max_fft": 2048}
        interp.update(compare_at(st_f.Y))
        std = 30.0  # a spread random embedding of the same scale, no structure
        Yr = torch.from_numpy(synth.random_embedding(nf, std, 4242)).to(dev)
        interp["random_embedding"] = dict(embedding=f"N(0, {std:g}^2 I), float32, seed 4242", **compare_at(Yr))
        del st_f, Yr, Pf, wse, wsi, wsf
        progress(f"interpolated gradient at n={nf} done")

    # --- PCA (tsne_pca): randomized truncated SVD of a cells x genes matrix ---
    phase("pca")
    pca = {}
    if args.pca_n:
        npc, gpc, kpc, qpc = args.pca_n, args.pca_g, 50, 2
        Xp = torch.from_numpy(synth.make_expression(npc, gpc, 2024)).to(dev)
        Om = torch.from_numpy(synth.make_omega(gpc, 2025)).to(dev)
        wsp = api.Workspace()
        tp, (sc, comp, sv, mu) = timed(lambda: api.pca(Xp, kpc, Om, qpc, ws=wsp), 5)
        passes = 2 + 2 * qpc  # X products: the range finder, 2 per power iteration, B
        flops = passes * 2.0 * npc * gpc * api.PCA_SUBSPACE
        # checks that need no oracle: orthonormal components, and the scores
        # equal to the centred rows projected on them (FP64, a sample of rows)
        cd = comp.double()
        orth_err = float((cd @ cd.T - torch.eye(kpc, dtype=torch.float64, device=dev)).abs().max())
        rows = torch.from_numpy(np.random.default_rng(11).choice(npc, 2000, replace=False)).to(dev)
        proj = (Xp[rows].double() - mu.double()) @ cd.T
        proj_err = float(torch.linalg.norm(sc[rows].double() - proj) / torch.linalg.norm(proj))
        pca = {"n": npc, "g": gpc, "k": kpc, "q": qpc, "subspace": api.PCA_SUBSPACE,
               "data": "make_expression: 64 latent programmes, singular values 100 to 1, noise 0.05, offset 2",
               "ms": tp, "x_passes": passes, "x_product_tflops": flops / (tp * 1e-3) / 1e12,
               "x_read_tb_s": passes * npc * gpc * 4 / (tp * 1e-3) / 1e12,
               "components_orthonormality_max_err": orth_err, "scores_projection_rel_err": proj_err,
               "singular_values_head": [float(v) for v in sv[:5].cpu()]}
        del Xp, Om, sc, comp, sv, mu, wsp
        progress(f"pca at {npc} x {gpc} done")

    # --- UMAP on the c5 points: kNN (k = 15), weights, union, layout -------
    phase("umap")
    umap = {}
    if args.umap_n:
        nu, ku, n_ep, neg = args.umap_n, 15, 200, 5
        Xu, labu = synth.make_points("c5", n=nu)
        Xu = torch.from_numpy(Xu).to(dev)
        wsu = api.Workspace()
        a_u, b_u = api.umap_fit_ab(0.5)
        runs = []
        for rep in range(2):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
            ev[0].record(stream)
            idu, d2u = api.knn(Xu, ku, "bf16", n_cand=2 * ku, ws=wsu)
            ev[1].record(stream)
            _, _, wu = api.umap_weights(d2u)
            ev[2].record(stream)
            Gu = api.umap_fuzzy_union(idu, wu, ws=wsu)  # reads nnz back (one sync)
            ev[3].record(stream)
            Yu = torch.from_numpy(synth.umap_init(nu, 3)).to(dev)
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t0.record(stream)
            api.umap_layout(Yu, Gu, a_u, b_u, n_ep, 1.0, neg, seed=1, ws=wsu)
            ev[4].record(stream)
            torch.cuda.synchronize()
            runs.append((ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3]),
                         t0.elapsed_time(ev[4])))
        kn, wt, un, lay = (float(np.median([r[q] for r in runs])) for q in range(4))
        r_u = Gu.val / Gu.val.max()
        sampled = float(torch.floor(float(n_ep) * r_u).sum().item())  # entries sampled over all epochs
        inter = sampled * (1 + neg)
        # structure check without the oracle: 10-NN label purity in the
        # embedding on 2000 sampled points
        rows = torch.from_numpy(np.random.default_rng(12).choice(nu, 2000, replace=False)).to(dev)
        dd = torch.cdist(Yu[rows].double(), Yu.double())
        dd[torch.arange(2000, device=dev), rows] = float("inf")
        nn10 = torch.topk(dd, 10, largest=False).indices.cpu().numpy()
        lab_t = labu[rows.cpu().numpy()]
        purity = float((labu[nn10] == lab_t[:, None]).mean())
        umap = {"n": nu, "k": ku, "knn": "bf16 + fp32 re-rank of 2k", "nnz": int(Gu.nnz), "n_epochs": n_ep,
                "neg_rate": neg, "min_dist": 0.5, "a": a_u, "b": b_u, "init": "uniform [-10, 10]^2, seed 3",
                "knn_ms": kn, "weights_ms": wt, "union_ms": un, "layout_ms": lay, "ms_per_epoch": lay / n_ep,
                "total_ms": kn + wt + un + lay, "sampled_entries": sampled,
                "pair_interactions_per_s": inter / (lay * 1e-3), "label_purity_10nn_sample": purity}
        del Xu, idu, d2u, wu, Gu, Yu, wsu, dd
        progress(f"umap at {nu} done")

    phase("cpu_baseline")
    # --- CPU baseline: the FP64 oracle on a bounded sample ------------------
    cpu = None
    errors = {}
    # GPU-side error statistics that need no oracle: entropy at the returned
    # beta recomputed in FP64 from the GPU's own distances, and sum P.
    beta = api.calibrate_P(d2, w.perplexity)[1].cpu().numpy().astype(np.float64)
    dd = d2.cpu().numpy().astype(np.float64)
    s_ = dd - dd.min(1, keepdims=True)
    e_ = np.exp(-beta[:, None] * s_)
    H = np.log(e_.sum(1)) + beta * (e_ * s_).sum(1) / e_.sum(1)
    errors["perplexity_H_max_abs_err_nats"] = float(np.abs(H - np.log(w.perplexity)).max())
    errors["P_sum_abs_err"] = float(abs(P.val.double().sum().item() - 1.0))
    if not args.no_cpu_baseline:
        import oracle

        thr = oracle.num_threads()
        big = n > 100_000
        qrows = (np.random.default_rng(7).choice(n, 1000, replace=False).astype(np.int64) if big
                 else np.arange(0, n, 10, dtype=np.int64))
        t0 = time.perf_counter()
        oi, od = oracle.knn(X_np, w.k, rows=qrows)
        t_knn = (time.perf_counter() - t0) * (n / qrows.size)
        gi, gd = synth.random_knn_graph(n, w.k, w.data_seed)  # full-size seeded graph for the linear stages
        t0 = time.perf_counter()
        Pc_o, _, _, _ = oracle.calibrate(gd, w.perplexity, tol=1e-5)
        S_o = oracle.symmetrize(gi, Pc_o)
        t_ps = time.perf_counter() - t0
        Sg = oracle.CSR(S_o.row_ptr, S_o.col, S_o.val.astype(np.float32).astype(np.float64))
        Y = Y0_np.astype(np.float64)
        if big:
            # the full FP64 gradient is O(n^2) per iteration: time per-row parts
            # (Z_i, repulsion, attraction; O(n) each) on sampled rows and scale
            grows = np.random.default_rng(8).choice(n, 256, replace=False).astype(np.int64)
            t0 = time.perf_counter()
            oracle.grad_rows(Y, grows, Sg)
            t_it = (time.perf_counter() - t0) * (n / grows.size)
            it_desc = (f"per-row gradient parts (Z_i, repulsion, attraction) on {grows.size} of {n} rows (time "
                       f"x{n // grows.size}) per iteration")
        else:
            U = np.zeros_like(Y)
            G = np.ones_like(Y)
            t0 = time.perf_counter()
            for t in range(args.cpu_iters):
                a, m = oracle.tsne_schedule(t, w.exaggeration, w.exaggeration_iters, w.momentum_early,
                                            w.momentum_late)
                g, _, _ = oracle.kl_grad(Y, Sg, a, want_kl=False)
                oracle.step(Y, U, G, g, w.lr, m)
            t_it = (time.perf_counter() - t0) / args.cpu_iters
            it_desc = f"{args.cpu_iters} of {iters} gradient+step iterations (time x{iters / args.cpu_iters:g})"
        t_run = t_knn + t_ps + t_it * iters
        t_step = t_run if whole else t_it * iters_per_step
        progress("CPU baseline timed")
        cpu = {"value": pairs_per_step / t_step, "unit": "pair interactions/s", "cores": thr, "kind": "oracle",
               "sample": (f"FP64 oracle, {thr} threads: exact kNN on {qrows.size} of {n} query rows (time x"
                          f"{n / qrows.size:g}); calibration + symmetrisation of a full-size seeded k={w.k} graph; "
                          f"{it_desc}; host {platform.processor() or platform.machine()}; value = the step's "
                          f"pair interactions / the oracle's extrapolated time for the same step "
                          f"({'the whole path' if whole else f'{iters_per_step} iterations'})"),
               "s_per_step_extrapolated": t_step, "s_per_run_extrapolated": t_run}
        # the oracles of the widened rows beside their GPU legs (bounded
        # samples, seeded synthetic inputs of the same recipes)
        nxt = {}
        if interp:
            from oracle import interp as o_interp

            Yi = synth.random_embedding(interp["n"], 30.0, 4242).astype(np.float64)
            t0 = time.perf_counter()
            o_interp.repulsion(Yi)
            nxt["interpolated_repulsion"] = {
                "oracle_s": time.perf_counter() - t0,
                "gpu_ms_whole_call": interp["random_embedding"]["interpolated_ms"],
                "sample": f"oracle/interp.py repulsion and Z by the same scheme (FP64 NumPy) at the leg's full "
                          f"{interp['n']} points on its random embedding; the GPU figure (same embedding) also "
                          f"holds the exact CSR attraction"}
            del Yi
        if pca:
            from oracle import pca as o_pca

            Xo = synth.make_expression(pca["n"], pca["g"], 2024).astype(np.float64)
            Omo = synth.make_omega(pca["g"], 2025).astype(np.float64)
            t0 = time.perf_counter()
            o_pca.randomized_pca(Xo, pca["k"], Omo, pca["q"])
            nxt["pca"] = {"oracle_s": time.perf_counter() - t0, "gpu_ms": pca["ms"],
                          "sample": f"oracle/pca.py (FP64 NumPy) at the leg's full {pca['n']} x {pca['g']}, q = {pca['q']}"}
            del Xo, Omo
        if umap:
            from oracle import umap as o_umap

            nu_o = 100_000
            io, _ = synth.random_knn_graph(nu_o, umap["k"], 21)
            rp_o, col_o, val_o = o_umap.fuzzy_union(io, np.random.default_rng(21).random((nu_o, umap["k"])), nu_o)
            Yo_u = synth.umap_init(nu_o, 22).astype(np.float64)
            t0 = time.perf_counter()
            o_umap.layout_epoch(Yo_u, rp_o, col_o, val_o.astype(np.float32), umap["n_epochs"] // 2, umap["n_epochs"],
                                umap["a"], umap["b"], 1.0, umap["neg_rate"], 5)
            t_ep = time.perf_counter() - t0
            nxt["umap_epoch"] = {
                "oracle_s": t_ep, "oracle_s_scaled_to_leg": t_ep * umap["nnz"] / col_o.size,
                "gpu_ms_per_epoch": umap["ms_per_epoch"],
                "sample": f"oracle/umap.py, one mid-schedule epoch (FP64 NumPy) on a seeded {nu_o}-point k = "
                          f"{umap['k']} graph (nnz {col_o.size}), scaled by stored entries to the leg's graph "
                          f"(nnz {umap['nnz']})"}
        if nxt:
            cpu["widened_rows"] = nxt
            progress("CPU baselines of the widened rows timed")
        # errors vs FP64 from identical inputs
        g_idx = idx.cpu().numpy()[qrows]
        errors["knn_set_agreement_sampled_rows"] = float(
            np.mean([len(set(p) & set(q)) / w.k for p, q in zip(g_idx.tolist(), oi.tolist())]))
        ddq = d2.cpu().numpy()[qrows].astype(np.float64)
        same = g_idx == oi
        errors["knn_d2_max_rel_on_agreeing_slots"] = float(
            np.max(np.abs(ddq[same] - od[same]) / np.maximum(od[same], 1e-30)))
        Pd = api.SparseP(torch.from_numpy(Sg.row_ptr).to(dev), torch.from_numpy(Sg.col).to(dev),
                         torch.from_numpy(Sg.val.astype(np.float32)).to(dev), None, n)
        for ystd, a in ((0.01, 12.0), (20.0, 1.0)):
            Yt = synth.random_embedding(n, ystd, 99)
            if big:
                # sampled rows: the oracle's per-row parts with the GPU's Z,
                # which is checked through its per-row sums on the same rows
                gg, Zg, _, Zr = api.kl_grad(torch.from_numpy(Yt).to(dev), Pd, a, want_Z=True, want_Zrow=True)
                er = np.random.default_rng(9).choice(n, 256, replace=False).astype(np.int64)
                Zo_r, Ro, Ao = oracle.grad_rows(Yt.astype(np.float64), er, Sg)
                go = 4.0 * (a * Ao - Ro / Zg.item())
                gg = gg.cpu().numpy().astype(np.float64)[er]
                errors[f"Zrow_rel_max_ystd{ystd:g}_sampled"] = float(
                    np.max(np.abs(Zr.cpu().numpy()[er] - Zo_r) / Zo_r))
                errors[f"Z_sum_of_rows_rel_ystd{ystd:g}"] = abs(float(Zr.sum()) - Zg.item()) / Zg.item()
                tag = "_sampled"
            else:
                gg, Zg, klg, _ = api.kl_grad(torch.from_numpy(Yt).to(dev), Pd, a, want_Z=True, want_kl=True)
                go, Zo, klo = oracle.kl_grad(Yt.astype(np.float64), Sg, a)
                gg = gg.cpu().numpy().astype(np.float64)
                errors[f"Z_rel_ystd{ystd:g}"] = abs(Zg.item() - Zo) / Zo
                errors[f"KL_rel_ystd{ystd:g}"] = abs(klg.item() - klo) / abs(klo)
                tag = ""
            errors[f"grad_rel_norm_ystd{ystd:g}{tag}"] = float(np.linalg.norm(gg - go) / np.linalg.norm(go))
            errors[f"grad_max_entry_rel_ystd{ystd:g}{tag}"] = float(np.abs(gg - go).max() / np.abs(go).max())
        errors["sample"] = ("kNN: the GPU lists of the benchmark's own run on the oracle's sampled query rows; "
                            "gradient: the oracle's P of a seeded random k-regular graph, seeded embeddings"
                            + ("; 256 sampled rows against the oracle's per-row parts" if big else ""))

    telemetry = None
    if mon is not None:
        ses = mon.stop()
        keep = ("duration_s", "samples", "mean_gfx_pct", "max_gfx_pct", "max_hip_used_bytes", "mean_power_w",
                "max_power_w", "max_temp_hotspot_c", "mean_proc_cpu_pct", "max_proc_rss_bytes")
        telemetry = {"period_s": 0.1, "gpu_sampled": bool(np.isfinite(ses.data["gfx_pct"]).any()),
                     "sample_us_median": float(np.median(ses.data["sample_us"])) if ses.t.size else None,
                     "steps": {r["name"]: {k: (None if isinstance(r[k], float) and not np.isfinite(r[k]) else r[k])
                                           for k in keep} for r in ses.steps if r["name"] != "start"}}

    roofline = {"bound": "alu", "achieved": achieved_tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved_tflops / FP32_PEAK_TFLOPS, "traffic": traffic,
                "kernel": "rep_sym_kernel (all-pairs Student-t repulsion and Z of tsne_kl_grad)",
                "flops_per_call": flops_per_call, "ms_per_call": grad_ms_mean,
                "flops_per_ordered_pair": api.KLGRAD_FLOPS_PER_ORDERED_PAIR, "source_digest": digest,
                "issue_floor": {"tflops": ISSUE_FLOOR_TFLOPS, "frac": achieved_tflops / ISSUE_FLOOR_TFLOPS,
                                "basis": "10 non-transcendental VALU instructions per unordered pair, one 4-cycle "
                                         "issue slot of a wave each, the reciprocal on the transcendental unit beside "
                                         "them, at 2.4 GHz on 1024 SIMDs, 17 flops per pair; packed FP32 is not used"}}
    rec = {
        "metric": "KL-grad pair interactions/s + kNN build s, BF16-MFMA vs FP32 at stated error",
        "value": value,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: exact t-SNE, N={n} x {w.d}, {w.clusters}-cluster mixture "
                               f"({w.weights} weights{', PCA-like spectrum' if w.shape == 'pca' else ''}), "
                               f"perplexity {w.perplexity:g}, k={w.k}, {w.knn} kNN"
                               f"{f' (n_cand {w.candidates})' if w.knn == 'bf16' else ''}, {iters} iterations",
                   "n": n, "d": w.d, "k": w.k, "perplexity": w.perplexity, "iters": iters, "knn": w.knn,
                   "step": step_desc, "iterations_per_step": iters_per_step},
        "repulsion_pairs_per_s": float(n) * (n - 1) / (grad_ms_mean * 1e-3),
        "iteration_ms": iter_ms,
        "iteration_pairs_per_s": float(n) * (n - 1) / (iter_ms * 1e-3),
        "affinity_s": aff_s,
        "run_s_estimate": {"value": aff_s + iters * iter_ms / 1e3,
                           "what": f"the whole {iters}-iteration run: the measured affinity stage plus {iters} x "
                                   f"the measured per-iteration time"},
        "knn_build_s": knn_cmp,
        "kl_autograd": diff,
        "interpolated_gradient": interp,
        "pca": pca,
        "umap": umap,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "telemetry": telemetry,
        "errors_vs_fp64": errors,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
