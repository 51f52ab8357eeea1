"""Learned warm start on the GPU against the CPU oracle: MLP forward and
gradients, Adam, BF16 inference on the matrix cores, features, modal
transforms; and what the trained network gains over the cold start."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def warm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_10863_amd import warm as w
    w.lib()
    return w


warm_train = pytest.importorskip("paper_1910_10863_amd.warm_train")


def test_target_stats_standardise_and_shrink(warm):
    """The library's statistics of training targets (mean, standard deviation
    with n - 1) and the validation shrink s_o = clamp(1 - sum (y - t)^2 /
    sum t^2, 0, 1), folded into the last layer, against numpy in FP64."""
    rng = np.random.default_rng(8)
    sizes = (5, 32, 48)
    n = 40
    net = warm.MLP(sizes, max_batch=n, seed=5)
    t = (rng.standard_normal((n, 48)) * rng.uniform(0.1, 3.0, 48) + rng.uniform(-1, 1, 48)).astype(np.float32)
    tt = torch.tensor(t, device="cuda")
    mean, std = net.target_stats(tt)
    assert np.allclose(mean.cpu().numpy(), t.astype(np.float64).mean(0), rtol=1e-6, atol=1e-6)
    assert np.allclose(std.cpu().numpy(), t.astype(np.float64).std(0, ddof=1), rtol=1e-6)
    z = net.standardise(tt, mean, std).cpu().numpy()
    ref = (t - mean.cpu().numpy()) / std.cpu().numpy()
    assert np.max(np.abs(z - ref)) < 1e-5
    x = rng.uniform(-1, 1, (n, 5)).astype(np.float32)
    xt = torch.tensor(x, device="cuda")
    y = net.forward(xt).cpu().numpy().astype(np.float64)
    shrink, err = net.validation_shrink(xt, tt)
    tv = t.astype(np.float64)
    s_ref = np.clip(1 - ((y - tv) ** 2).sum(0) / np.maximum((tv ** 2).sum(0), 1e-30), 0, 1)
    assert np.allclose(shrink.cpu().numpy(), s_ref, rtol=1e-5, atol=1e-6)
    e_ref = np.sqrt(((s_ref * y - tv) ** 2).sum() / (tv ** 2).sum())
    assert abs(err - e_ref) < 1e-5 * e_ref
    y2 = net.forward(xt).cpu().numpy()
    assert np.allclose(y2, s_ref * y, rtol=1e-4, atol=1e-5)


def _flat(params):
    return np.concatenate([np.concatenate([Wm.ravel(), b]) for Wm, b in params])


def _net_with_oracle_params(warm, sizes, batch, seed):
    from oracle import warmstart as ws
    params = ws.init_params(sizes, seed)
    net = warm.MLP(sizes, max_batch=batch, seed=3)
    net.set_params(torch.tensor(_flat(params), dtype=torch.float32, device="cuda"))
    # the oracle works on the FP32-rounded parameters the GPU holds
    p32 = [(Wm.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for Wm, b in params]
    return net, p32


@pytest.mark.parametrize("sizes,batch", [((5, 32, 32, 24), 37), ((5, 256, 256, 256, 2048), 64)])
def test_forward_and_gradients_vs_oracle(warm, sizes, batch):
    from oracle import warmstart as ws
    rng = np.random.default_rng(8)
    X = rng.uniform(-1, 1, (batch, sizes[0])).astype(np.float32)
    T = rng.standard_normal((batch, sizes[-1])).astype(np.float32)
    net, p32 = _net_with_oracle_params(warm, sizes, batch, 5)
    y = net.forward(torch.tensor(X, device="cuda")).cpu().numpy()
    loss = net.backward_mse(torch.tensor(T, device="cuda"), want_loss=True)
    g = net.grads().cpu().numpy()
    yo = ws.forward(p32, X.astype(np.float64))[-1]
    lo, go = ws.mse_and_grads(p32, X.astype(np.float64), T.astype(np.float64))
    gof = _flat(go)
    ey = np.max(np.abs(y - yo)) / np.max(np.abs(yo))
    eg = np.max(np.abs(g - gof)) / np.max(np.abs(gof))
    _say("mlp", sizes, "forward err", ey, "grad err", eg, "loss", loss, lo)
    assert ey < 2e-6
    assert eg < 2e-5
    assert abs(loss - lo) < 1e-5 * lo


def test_adam_steps_vs_oracle(warm):
    from oracle import warmstart as ws
    sizes, batch = (5, 16, 12), 20
    rng = np.random.default_rng(9)
    X = rng.uniform(-1, 1, (batch, 5)).astype(np.float32)
    T = rng.standard_normal((batch, 12)).astype(np.float32)
    net, p32 = _net_with_oracle_params(warm, sizes, batch, 6)
    p = _flat(p32)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in (1, 2, 3):
        net.forward(torch.tensor(X, device="cuda"))
        net.backward_mse(torch.tensor(T, device="cuda"))
        g = net.grads().cpu().numpy().astype(np.float64)
        net.adam(1e-2, t)
        p, m, v = ws.adam(p, g, m, v, t, lr=1e-2)
        got = net.params().cpu().numpy()
        assert np.max(np.abs(got - p)) < 1e-6, t
        # continue the oracle from the GPU's parameters (FP32 state)
        p = got.astype(np.float64)


def _bf16(a):
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_inference_vs_oracle_rounding(warm):
    """The MFMA layer equals the definition with bf16-rounded weights and
    inputs (FP32 accumulation order aside) and stays close to FP32."""
    sizes, batch = (5, 256, 256, 256, 2048), 45
    rng = np.random.default_rng(10)
    X = rng.uniform(-1, 1, (batch, 5)).astype(np.float32)
    net, p32 = _net_with_oracle_params(warm, sizes, batch, 7)
    net.to_bf16()
    xt = torch.tensor(X, device="cuda")
    yb = net.infer_bf16(xt).cpu().numpy()
    yf = net.forward(xt).cpu().numpy()
    h = X.astype(np.float64)
    for li, (Wm, b) in enumerate(p32):
        z = _bf16(h) @ _bf16(Wm).T + b
        h = np.tanh(z) if li < len(p32) - 1 else z
        h = h.astype(np.float32).astype(np.float64)
    e_ref = np.max(np.abs(yb - h)) / np.max(np.abs(h))
    e_f32 = np.max(np.abs(yb - yf)) / np.max(np.abs(yf))
    _say("bf16 vs rounded oracle", e_ref, "vs fp32", e_f32)
    assert e_ref < 1e-3
    assert e_f32 < 3e-2


def test_scale_output_folds_affine_map(warm):
    sizes, batch = (5, 16, 8), 9
    net = warm.MLP(sizes, max_batch=batch, seed=4)
    x = torch.rand((batch, 5), device="cuda") * 2 - 1
    y0 = net.forward(x).clone()
    sc = torch.linspace(0.5, 2.0, 8, device="cuda")
    sh = torch.linspace(-1.0, 1.0, 8, device="cuda")
    net.scale_output(sc, sh)
    y1 = net.forward(x)
    assert torch.max(torch.abs(y1 - (y0 * sc + sh))).item() < 1e-5


def test_features_vs_oracle(warm):
    from oracle import warmstart as ws
    d = W.warm_start_draws(50, 3)
    x = warm.features(torch.tensor(d, device="cuda")).cpu().numpy()
    assert np.max(np.abs(x - ws.features(d))) < 1e-6


def test_modes_vs_oracle(warm):
    from oracle import warmstart as ws
    from paper_1910_10863_amd import pfm
    wl = W.warm_start_block(0.3, 10.0, 1.2)
    prob = pfm.Problem.from_workload(wl, max_batch=3)
    th = [0.1, 0.7, 1.3]
    prob.set_batch(3.0, th)
    psi = np.stack([W.random_density(prob.n, 30 + b) for b in range(3)])
    K = 32
    vec = warm.modes_analyse(prob, K, th, torch.tensor(psi, device="cuda")).cpu().numpy()
    from oracle import geometry as geo
    cen = geo.fibre_centres(wl.lattice, wl.a, wl.M_L, wl.M_H)[0]
    for b in range(3):
        ref = ws.modes_to_vector(ws.density_modes(psi[b], wl.M, wl.n_elem, K, 3.0, th[b], cen))
        assert np.max(np.abs(vec[b] - ref)) < 1e-6 * np.max(np.abs(ref)), b
    back = warm.modes_synthesise(prob, K, th, torch.tensor(vec, device="cuda")).cpu().numpy()
    for b in range(3):
        ref = ws.modes_density(ws.vector_to_modes(vec[b].astype(np.float64), wl.M, K), wl.M, wl.n_elem, K, 3.0,
                               th[b], cen)
        assert np.max(np.abs(back[b] - ref)) < 1e-12 * np.max(np.abs(ref)), b


def test_bad_start_falls_back_to_cold(warm):
    prob = warm_train.block_problem(0.3, 10.0, 1.1, 2)
    prob.set_batch(2.5, [0.2, 0.9])
    xc, ic = prob.solve_batch()
    x0 = xc.clone()
    x0[1] = 1e3 * torch.randn_like(x0[1])          # member 1: a start far worse than zero
    xw, iw = prob.solve_batch(x0=x0, fallback=True)
    assert iw[0]["fallback"] == 0 and iw[0]["iters"] == 0
    assert iw[1]["fallback"] == 1 and iw[1]["iters"] == ic[1]["iters"]
    assert torch.allclose(xw[1], xc[1], rtol=0, atol=1e-12 * float(torch.max(torch.abs(xc[1]))))


def test_augmented_cycle_never_loses_to_cold(warm):
    """Augmentation with the exact solution converges at once; with a
    random vector it takes no more iterations than the cold start."""
    prob = warm_train.block_problem(0.3, 10.0, 1.1, 3)
    prob.set_batch(2.5, [0.2, 0.9, 1.3])
    xc, ic = prob.solve_batch()
    xa, ia = prob.solve_batch(x0=xc, augment=True)
    assert all(i["iters"] <= 1 and i["status"] == 0 for i in ia), ia
    xr, ir = prob.solve_batch(x0=torch.randn_like(xc), augment=True)
    for c, r in zip(ic, ir):
        assert r["status"] == 0 and r["iters"] <= c["iters"] + 1, (c, r)
    # every solution agrees with the cold one to the tolerance the residual allows
    assert float(torch.max(torch.linalg.vector_norm(xr - xc, dim=1) / torch.linalg.vector_norm(xc, dim=1))) < 1e-6


def test_trained_network_gain(warm):
    """Train on solves from a narrow parameter box and evaluate on held-out
    draws of the same box.  The BF16 prediction starts GMRES at a residual of
    a few percent; to a residual of 1e-4 it saves iterations.  To 1e-8 a
    start vector with an error of about one percent spread over all modes and
    fibres costs GMRES more than it saves (the cold Krylov space of the smooth
    incident field converges superlinearly), so there the prediction is used
    to augment the first cycle, which never needs more iterations than the
    cold start."""

    def groups(n, seed):
        r = np.random.default_rng(seed)
        g = np.stack([r.uniform(1.0, 2.0, n), r.uniform(0.25, 0.3, n), r.uniform(10.0, 14.0, n),
                      r.uniform(0.9, 1.1, n)], axis=1)
        th = r.uniform(0.0, 0.6, (n, 8))
        return g, th

    g_tr, t_tr = groups(60, 1)
    data = warm_train.generate(g_tr, t_tr)
    _say("generated", data.x.shape[0], "solves in", data.seconds, "s; mean cold iters", data.iters.mean())
    net = warm_train.train(data, epochs=300, batch=64, lr=2e-3, seed=2)
    _say("loss", net.losses[0], "->", net.losses[-1], "in", net.train_seconds, "s")
    assert net.losses[-1] < 0.1 * net.losses[0]
    g_te, t_te = groups(4, 99)
    res = warm_train.evaluate(net, g_te, t_te, tols=(1e-4, 1e-8))
    _say("evaluation", res)
    assert res["median_start_residual"] < 0.1
    loose, tight = res["tolerances"]["1e-04"], res["tolerances"]["1e-08"]
    assert loose["n"] >= 24 and tight["n"] >= 24
    assert loose["start"]["mean_iters"] < 0.9 * loose["cold_mean_iters"]
    assert tight["augment"]["worse_than_cold"] == 0
