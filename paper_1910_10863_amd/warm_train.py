"""Learned warm start (not in the paper): data generation by the method's own
solves, training of the MLP, and the evaluation against the cold start.

Host orchestration over the library's calls (warm.py binds them): solves,
modal analysis, features, target statistics and standardisation, forward /
backward / Adam, the validation shrink, BF16 inference and the start-vector
synthesis all run in libpfmbem.so.  This module orders the calls, picks the
learning rate of each Adam step (cosine decay) and gathers the shuffled
training rows with torch indexing.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import Dict

import numpy as np

from . import pfm
from .warm import MLP, N_MODES, SIZES, features, modes_analyse, modes_synthesise


def block_problem(r: float, rho_ratio: float, c_ratio: float, B: int, **kw) -> "pfm.Problem":
    import workloads as W
    wl = W.warm_start_block(r, rho_ratio, c_ratio)
    opts = dict(max_batch=B, restart=100, max_iter=2000, wood_margin=1e-3)
    opts.update(kw)
    return pfm.Problem.from_workload(wl, **opts)


@dataclass
class Dataset:
    x: "object"           # float32 [n, 5] network inputs
    t: "object"           # float32 [n, 2048] modal coefficients
    draws: np.ndarray     # [n, 5]
    iters: np.ndarray     # cold-start iterations of each solve
    seconds: float


def generate(groups: np.ndarray, thetas: np.ndarray, K: int = N_MODES, log=None) -> Dataset:
    """Solve every draw (cold start, residual 1e-8) and record its modes.
    groups [G, 4] = (ka, r, rho ratio, c ratio), thetas [G, B]."""
    import torch
    xs, ts, ds, its = [], [], [], []
    t0 = time.perf_counter()
    for g in range(groups.shape[0]):
        ka, r, rr, cr = (float(v) for v in groups[g])
        th = thetas[g]
        prob = block_problem(r, rr, cr, th.size)
        try:
            prob.set_batch(ka, th)
        except pfm.PfmError as e:
            if e.code == 5:          # Wood anomaly: no data
                prob.close()
                continue
            raise
        x, infos = prob.solve_batch()
        ok = [i for i, inf in enumerate(infos) if inf["status"] == 0]
        vec = modes_analyse(prob, K, th, x)
        draws = np.stack([[ka, th[i], r, rr, cr] for i in range(th.size)])
        ds.append(draws[ok])
        ts.append(vec[ok])
        its.extend(infos[i]["iters"] for i in ok)
        prob.close()
        if log and (g + 1) % max(1, groups.shape[0] // 10) == 0:
            log(f"generate: {g + 1}/{groups.shape[0]} groups, {time.perf_counter() - t0:.1f} s")
    draws = np.concatenate(ds)
    d = torch.tensor(draws, dtype=torch.float64, device="cuda")
    return Dataset(features(d), torch.cat(ts), draws, np.array(its), time.perf_counter() - t0)


def train(data: Dataset, epochs: int = 100, batch: int = 256, lr: float = 1e-3, lr_end: float = 1e-5,
          seed: int = 1, log=None, sizes=SIZES, val_frac: float = 0.1) -> "MLP":
    """Adam on the standardised targets, cosine learning-rate decay; the
    standardisation is folded into the last layer at the end.  Then every
    output is shrunk towards zero by s = max(0, 1 - E[(y - t)^2] / E[t^2])
    measured on a held-back validation split: modes the network cannot
    predict are left out of the start vector (a mode missing from the start
    vector costs GMRES less than a mode with a wrong value)."""
    import torch
    n_all = data.x.shape[0]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    order = torch.randperm(n_all, device="cuda", generator=gen)
    n_val = int(round(val_frac * n_all)) if n_all >= 20 else 0
    vi, ti = order[:n_val], order[n_val:]
    xv, tv = data.x[vi].contiguous(), data.t[vi].contiguous()
    x_tr, t_tr = data.x[ti].contiguous(), data.t[ti].contiguous()
    n = x_tr.shape[0]
    batch = min(batch, n)
    net = MLP(sizes, max_batch=max(batch, n_val, 4), seed=seed)
    mean, std = net.target_stats(t_tr)
    tz = net.standardise(t_tr, mean, std)
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    t = 0
    yb = torch.empty((batch, sizes[-1]), dtype=torch.float32, device="cuda")
    losses = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=gen)
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            xb = x_tr[idx].contiguous()
            tb = tz[idx].contiguous()
            net.forward(xb, yb)
            want = s == steps_per_epoch - 1
            loss = net.backward_mse(tb, want_loss=want)
            t += 1
            cur = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * t / total))
            net.adam(cur, t)
            if want:
                losses.append(loss)
        if log and (ep + 1) % max(1, epochs // 10) == 0:
            log(f"train: epoch {ep + 1}/{epochs} loss {losses[-1]:.4e} {time.perf_counter() - t0:.1f} s")
    net.scale_output(std, mean)
    net.shrink = None
    if n_val > 0:
        net.shrink, net.val_rel_err = net.validation_shrink(xv, tv)
    net.to_bf16()
    net.losses = losses
    net.train_seconds = time.perf_counter() - t0
    return net


def evaluate(net: "MLP", groups: np.ndarray, thetas: np.ndarray, K: int = N_MODES, tols=(1e-8,),
             log=None, precond: bool = False) -> Dict:
    """Cold start against the BF16 prediction used two ways on the same draws:
    as the start vector (with fallback to zero) and as the augmentation of
    the first GMRES cycle, at each GMRES tolerance in `tols`, all three with
    plain GMRES or (precond) GMRES right-preconditioned by the fibres'
    free-space self blocks.  Returns, per tolerance, iteration counts and
    times (inference included), and the start residuals of the predictions."""
    import torch
    out = {"tolerances": {}}
    r0 = []
    for tol in tols:
        it = {"cold": [], "start": [], "augment": []}
        tm = {"cold": 0.0, "start": 0.0, "augment": 0.0}
        fb = 0
        for g in range(groups.shape[0]):
            ka, r, rr, cr = (float(v) for v in groups[g])
            th = thetas[g]
            prob = block_problem(r, rr, cr, th.size, tol=tol, precond=precond)
            try:
                prob.set_batch(ka, th)
            except pfm.PfmError as e:
                if e.code == 5:
                    prob.close()
                    continue
                raise
            draws = torch.tensor([[ka, th[i], r, rr, cr] for i in range(th.size)], dtype=torch.float64,
                                 device="cuda")
            res = {}
            for mode in ("cold", "start", "augment"):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if mode == "cold":
                    _, inf = prob.solve_batch()
                else:
                    x0 = modes_synthesise(prob, K, th, net.infer_bf16(features(draws)))
                    _, inf = prob.solve_batch(x0=x0, fallback=mode == "start", augment=mode == "augment")
                torch.cuda.synchronize()
                tm[mode] += time.perf_counter() - t0
                res[mode] = inf
            if tol == tols[0]:
                b = prob.rhs_batch()
                res0 = torch.linalg.vector_norm(b - prob.matvec_batch(x0), dim=1) / torch.linalg.vector_norm(b, dim=1)
                r0.extend(float(v) for v in res0)
            for i in range(th.size):
                if any(res[mo][i]["status"] != 0 for mo in res):
                    continue
                for mo in res:
                    it[mo].append(res[mo][i]["iters"])
                fb += res["start"][i]["fallback"]
            prob.close()
        c = np.array(it["cold"])
        rec = {"n": int(c.size), "cold_mean_iters": float(c.mean()), "cold_seconds": tm["cold"]}
        for mo in ("start", "augment"):
            w = np.array(it[mo])
            rec[mo] = {"mean_iters": float(w.mean()), "iters_saved_frac": float(1 - w.sum() / c.sum()),
                       "seconds_incl_inference": tm[mo], "worse_than_cold": int(np.sum(w > c)),
                       "better_than_cold": int(np.sum(w < c))}
        rec["start"]["fallbacks"] = int(fb)
        out["tolerances"][f"{tol:.0e}"] = rec
        if log:
            log(f"evaluate tol {tol:.0e}: {rec}")
    out["median_start_residual"] = float(np.median(r0)) if r0 else None
    return out
