"""Autotuner of the batched sweep: leaf size (the P2P tile: rows of one
near-field workgroup and columns of its block stream) and expansion order p.

For a geometry and the angles of a batch it builds one handle per candidate,
measures the relative error of the batched apply against a p = 40 reference
apply on the same random densities at the largest frequency of the sweep
(the FMM truncation error grows with k), and times the per-frequency setup
(pfm_set_batch) and the batched apply with HIP events.  Among the candidates
whose error meets the target it picks the one with the smallest modelled
cost per frequency,

    cost = t_setup + iters * t_apply,

with iters the expected GMRES iterations per frequency.  Every measurement
runs through the C library; this module only orders the candidates.
"""
from __future__ import annotations

import hashlib
import json
import os
from dataclasses import asdict, dataclass, field
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

LEAF_CANDIDATES = (16, 32, 64)
P_CANDIDATES = (12, 16, 20, 24, 32)
REF_P = 40


@dataclass
class Trial:
    leaf_max: int
    p: int
    err: float
    t_setup_ms: float
    t_apply_ms: float
    cost_ms: float
    ok: bool


@dataclass
class Choice:
    leaf_max: int
    p: int
    err: float
    cost_ms: float
    trials: List[Trial] = field(default_factory=list)

    def to_json(self) -> dict:
        d = asdict(self)
        return d


def select(trials: Sequence[Trial]) -> Trial:
    """The accurate trial of least cost; ties go to the larger p (more margin).
    Raises when no trial meets the error target."""
    good = [t for t in trials if t.ok]
    if not good:
        raise RuntimeError("no candidate meets the error target; allow larger p or a looser target")
    return min(good, key=lambda t: (t.cost_ms, -t.p))


def cost(t_setup_ms: float, t_apply_ms: float, iters: float) -> float:
    return t_setup_ms + iters * t_apply_ms


def _key(geom: dict, ka: float, thetas: Sequence[float], target: float, cands) -> str:
    blob = json.dumps({"g": geom, "ka": ka, "th": list(map(float, thetas)), "t": target, "c": cands},
                      sort_keys=True, default=lambda a: list(map(float, a)))
    return hashlib.sha256(blob.encode()).hexdigest()[:16]


def autotune(geom: dict, ka_max: float, thetas: Sequence[float], target_err: float = 1e-10,
             leaves: Iterable[int] = LEAF_CANDIDATES, ps: Iterable[int] = P_CANDIDATES,
             iters: float = 30.0, reps: int = 20, seed: int = 17, cache: Optional[str] = None,
             measure: Optional[Callable[[int, int], Tuple[float, float, float]]] = None) -> Choice:
    """Pick (leaf_max, p) for a batched sweep.

    geom: keyword arguments of pfm.Problem without the tuning options
    (lattice, a, M_L, M_H, n_elem, radii, rho_fiber, c_fiber, rho_matrix,
    c_matrix, and optionally eta, mac, g_far).  measure(leaf, p) -> (err,
    t_setup_ms, t_apply_ms) replaces the GPU measurement (tests).
    The result is stored in / read from the JSON file `cache` when given."""
    leaves = tuple(int(x) for x in leaves)
    ps = tuple(int(x) for x in ps)
    key = _key(geom, ka_max, thetas, target_err, [leaves, ps, iters])
    if cache and os.path.exists(cache):
        with open(cache) as f:
            db = json.load(f)
        if key in db:
            d = db[key]
            return Choice(d["leaf_max"], d["p"], d["err"], d["cost_ms"],
                          [Trial(**t) for t in d.get("trials", [])])
    if measure is None:
        measure = _gpu_measure(geom, ka_max, thetas, reps, seed)
    trials = []
    for leaf in leaves:
        for p in sorted(ps):
            err, ts, ta = measure(leaf, p)
            ok = err <= target_err
            trials.append(Trial(leaf, p, err, ts, ta, cost(ts, ta, iters), ok))
            if ok:
                break          # larger p at this leaf size is only slower
    best = select(trials)
    ch = Choice(best.leaf_max, best.p, best.err, best.cost_ms, trials)
    if cache:
        db = {}
        if os.path.exists(cache):
            with open(cache) as f:
                db = json.load(f)
        db[key] = ch.to_json()
        with open(cache, "w") as f:
            json.dump(db, f, indent=1)
    return ch


def autotune_bands(geom: dict, kas: Sequence[float], thetas: Sequence[float], n_bands: int = 4,
                   target_err: float = 1e-10, leaves: Iterable[int] = LEAF_CANDIDATES,
                   ps: Iterable[int] = P_CANDIDATES, iters: float = 30.0, reps: int = 10,
                   measure_factory=None) -> List[Tuple[List[float], Choice]]:
    """Frequency-adaptive expansion order (the closing remark of Sec. 4: p
    must grow with the frequency): the sorted frequencies are cut into
    n_bands consecutive bands of nearly equal count, and each band gets the
    (leaf_max, p) that autotune picks at its own largest frequency.  Returns
    [(frequencies of the band, choice)].  measure_factory(ka) -> measure
    replaces the GPU measurement (tests)."""
    ks = sorted(float(k) for k in kas)
    n_bands = max(1, min(n_bands, len(ks)))
    edges = [round(i * len(ks) / n_bands) for i in range(n_bands + 1)]
    out = []
    for b in range(n_bands):
        band = ks[edges[b]:edges[b + 1]]
        if not band:
            continue
        meas = measure_factory(band[-1]) if measure_factory else None
        ch = autotune(geom, band[-1], thetas, target_err=target_err, leaves=leaves, ps=ps, iters=iters,
                      reps=reps, measure=meas)
        out.append((band, ch))
    return out


def _gpu_measure(geom: dict, ka: float, thetas: Sequence[float], reps: int, seed: int):
    import numpy as np
    import torch

    from . import pfm

    B = len(thetas)
    ref_cache: Dict[int, torch.Tensor] = {}
    rng = np.random.default_rng(seed)

    def handle(leaf, p):
        return pfm.Problem(**geom, p=p, leaf_max=leaf, max_batch=B)

    psi_holder = {}

    def densities(n):
        if "psi" not in psi_holder:
            z = rng.standard_normal((B, n)) + 1j * rng.standard_normal((B, n))
            psi_holder["psi"] = torch.tensor(z, device="cuda")
        return psi_holder["psi"]

    def reference(leaf):
        # the reference uses the same leaf size so that only p differs
        if leaf not in ref_cache:
            h = handle(leaf, REF_P)
            h.set_batch(ka, thetas)
            ref_cache[leaf] = h.matvec_batch(densities(h.n)).clone()
            h.close()
        return ref_cache[leaf]

    def measure(leaf, p):
        ref = reference(leaf)
        h = handle(leaf, p)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        h.set_batch(ka, thetas)                 # first setup (plan-time effects)
        torch.cuda.synchronize()
        e0.record()
        h.set_batch(ka, thetas)
        e1.record()
        torch.cuda.synchronize()
        t_setup = e0.elapsed_time(e1)
        psi = densities(h.n)
        y = h.matvec_batch(psi)
        err = float(torch.max(torch.linalg.vector_norm(y - ref, dim=1) / torch.linalg.vector_norm(ref, dim=1)))
        for _ in range(3):
            h.matvec_batch(psi, y)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            h.matvec_batch(psi, y)
        e1.record()
        torch.cuda.synchronize()
        t_apply = e0.elapsed_time(e1) / reps
        h.close()
        return err, t_setup, t_apply

    return measure


def geometry_of(wl) -> dict:
    """pfm.Problem geometry/material keywords of a workload."""
    return dict(lattice=wl.lattice, a=wl.a, M_L=wl.M_L, M_H=wl.M_H, n_elem=wl.n_elem, radii=wl.radii,
                rho_fiber=wl.rho_fiber, c_fiber=wl.c_fiber, rho_matrix=wl.rho_matrix, c_matrix=wl.c_matrix,
                eta=wl.eta, shape=wl.shape)
