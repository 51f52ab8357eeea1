"""ctypes binding of the learned warm start (include/pfmwarm.h), plus the
host-side orchestration of its data generation, training and evaluation.

Every arithmetic step runs in libpfmbem.so: features, the MLP forward /
backward / Adam steps in FP32, BF16 inference on the matrix cores, the modal
analysis of solved densities and the synthesis of start vectors, and the
GMRES solves themselves.  PyTorch holds the device memory; besides that it
only shuffles and gathers training rows and computes the mean and spread of
the training targets (the standardisation that is folded into the last
layer afterwards).
"""
from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import pfm

EXPORTS = ["pfm_mlp_create", "pfm_mlp_destroy", "pfm_mlp_set_stream", "pfm_mlp_n_params", "pfm_mlp_buffers",
           "pfm_mlp_get_params", "pfm_mlp_set_params", "pfm_mlp_get_grads", "pfm_mlp_scale_output",
           "pfm_mlp_forward", "pfm_mlp_backward_mse", "pfm_mlp_adam", "pfm_mlp_to_bf16", "pfm_mlp_infer_bf16",
           "pfm_warm_features", "pfm_modes_analyse", "pfm_modes_synthesise"]

SIZES = (5, 256, 256, 256, 2048)      # (ka, theta, r, rho ratio, c ratio) -> 16 fibres x 2 x 32 modes x re/im
N_MODES = 32

_bound = False


def lib():
    global _bound
    L = pfm.lib()
    if _bound:
        return L
    P = ctypes.c_void_p
    fp = ctypes.c_void_p
    L.pfm_mlp_create.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int, ctypes.c_ulonglong,
                                 ctypes.POINTER(P)]
    L.pfm_mlp_destroy.argtypes = [P]
    L.pfm_mlp_destroy.restype = None
    L.pfm_mlp_set_stream.argtypes = [P, P]
    L.pfm_mlp_n_params.argtypes = [P]
    L.pfm_mlp_n_params.restype = ctypes.c_longlong
    L.pfm_mlp_buffers.argtypes = [P, ctypes.POINTER(fp), ctypes.POINTER(fp)]
    L.pfm_mlp_get_params.argtypes = [P, fp]
    L.pfm_mlp_set_params.argtypes = [P, fp]
    L.pfm_mlp_get_grads.argtypes = [P, fp]
    L.pfm_mlp_scale_output.argtypes = [P, fp, fp]
    L.pfm_mlp_forward.argtypes = [P, fp, ctypes.c_int, fp]
    L.pfm_mlp_backward_mse.argtypes = [P, fp, ctypes.c_int, ctypes.POINTER(ctypes.c_float)]
    L.pfm_mlp_adam.argtypes = [P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int]
    L.pfm_mlp_to_bf16.argtypes = [P]
    L.pfm_mlp_infer_bf16.argtypes = [P, fp, ctypes.c_int, fp]
    L.pfm_warm_features.argtypes = [fp, ctypes.c_int, fp, P]
    dp = ctypes.POINTER(ctypes.c_double)
    L.pfm_modes_analyse.argtypes = [P, ctypes.c_int, ctypes.c_int, dp, fp, fp]
    L.pfm_modes_synthesise.argtypes = [P, ctypes.c_int, ctypes.c_int, dp, fp, fp]
    _bound = True
    return L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _check(code, what):
    if code != 0:
        raise pfm.PfmError(code, what)


class MLP:
    """The warm-start network (FP32 parameters on the device)."""

    def __init__(self, sizes: Sequence[int] = SIZES, max_batch: int = 1024, seed: int = 1):
        import torch
        L = lib()
        self._L = L
        self.sizes = tuple(int(s) for s in sizes)
        self.max_batch = max_batch
        arr = (ctypes.c_int * len(self.sizes))(*self.sizes)
        self._h = ctypes.c_void_p()
        _check(L.pfm_mlp_create(arr, len(self.sizes) - 1, max_batch, seed, ctypes.byref(self._h)), "pfm_mlp_create")
        self.n_params = L.pfm_mlp_n_params(self._h)
        _check(L.pfm_mlp_set_stream(self._h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), "stream")

    def close(self):
        if self._h:
            self._L.pfm_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        import torch
        p = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(self._L.pfm_mlp_get_params(self._h, _ptr(p)), "get_params")
        return p

    def set_params(self, p):
        _check(self._L.pfm_mlp_set_params(self._h, _ptr(p.contiguous())), "set_params")

    def grads(self):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(self._L.pfm_mlp_get_grads(self._h, _ptr(g)), "get_grads")
        return g

    def forward(self, x, out=None):
        import torch
        y = out if out is not None else torch.empty((x.shape[0], self.sizes[-1]), dtype=torch.float32, device="cuda")
        _check(self._L.pfm_mlp_forward(self._h, _ptr(x), x.shape[0], _ptr(y)), "forward")
        return y

    def backward_mse(self, t, want_loss: bool = False) -> Optional[float]:
        loss = ctypes.c_float()
        _check(self._L.pfm_mlp_backward_mse(self._h, _ptr(t), t.shape[0], ctypes.byref(loss) if want_loss else None),
               "backward")
        return loss.value if want_loss else None

    def adam(self, lr: float, t: int, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        _check(self._L.pfm_mlp_adam(self._h, lr, b1, b2, eps, t), "adam")

    def scale_output(self, scale, shift):
        _check(self._L.pfm_mlp_scale_output(self._h, _ptr(scale), _ptr(shift)), "scale_output")

    def to_bf16(self):
        _check(self._L.pfm_mlp_to_bf16(self._h), "to_bf16")

    def infer_bf16(self, x, out=None):
        import torch
        y = out if out is not None else torch.empty((x.shape[0], self.sizes[-1]), dtype=torch.float32, device="cuda")
        _check(self._L.pfm_mlp_infer_bf16(self._h, _ptr(x), x.shape[0], _ptr(y)), "infer_bf16")
        return y


def features(draws):
    """draws: float64 CUDA tensor [B, 5] -> float32 [B, 5] network inputs."""
    import torch
    L = lib()
    x = torch.empty(draws.shape, dtype=torch.float32, device="cuda")
    _check(L.pfm_warm_features(_ptr(draws), draws.shape[0], _ptr(x),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), "features")
    return x


def modes_analyse(prob: "pfm.Problem", K: int, thetas, psi):
    import torch
    L = lib()
    th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64).reshape(-1))
    B = th.size
    vec = torch.empty((B, 4 * prob.M * K), dtype=torch.float32, device="cuda")
    _check(L.pfm_modes_analyse(prob._h, K, B, th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(psi),
                               _ptr(vec)), "modes_analyse")
    return vec


def modes_synthesise(prob: "pfm.Problem", K: int, thetas, vec):
    import torch
    L = lib()
    th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64).reshape(-1))
    B = th.size
    psi = torch.empty((B, prob.n), dtype=torch.complex128, device="cuda")
    _check(L.pfm_modes_synthesise(prob._h, K, B, th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  _ptr(vec.contiguous()), _ptr(psi)), "modes_synthesise")
    return psi


# ---------------------------------------------------------------------------
# data generation, training, evaluation
# ---------------------------------------------------------------------------
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
    mean = t_tr.mean(dim=0)
    std = t_tr.std(dim=0).clamp_min(1e-6)
    tz = ((t_tr - mean) / std).contiguous()
    net = MLP(sizes, max_batch=max(batch, n_val, 1), seed=seed)
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
    net.scale_output(std.contiguous(), mean.contiguous())
    net.shrink = None
    if n_val > 0:
        yv = net.forward(xv)
        mse = ((yv - tv) ** 2).mean(dim=0)
        pw = (tv ** 2).mean(dim=0).clamp_min(1e-30)
        shrink = (1.0 - mse / pw).clamp(min=0.0, max=1.0).contiguous()
        net.scale_output(shrink, torch.zeros_like(shrink))
        net.shrink = shrink
        net.val_rel_err = float(torch.sqrt(((net.forward(xv) - tv) ** 2).sum() / (tv ** 2).sum()))
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
