"""GPU parity of the surrogate's BF16-MFMA kernels against the FP64 NumPy
reference on identical BF16 operands: forward predictions, per-layer
gradients and Adam updates (relative L2 <= 1e-3 per tensor; the GPU
accumulates in FP32, and a BF16 rounding of a value that lies within its FP32
error of a rounding boundary may go either way)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _make(torch_mod, n_in, n_out, width, depth, batch, ensemble=1, seed=3, weight_decay=0.0):
    from oracle.mlp_oracle import MLPOracle, bf16
    from paper_1707_09073_amd import gfmc
    net = gfmc.SurrogateNet(n_in, n_out, width=width, depth=depth, ensemble=ensemble, max_batch=batch, seed=seed,
                            weight_decay=weight_decay)
    rng = np.random.default_rng(seed)
    xm, xs = rng.normal(size=n_in), rng.uniform(0.5, 2.0, n_in)
    ym, ys = rng.normal(size=n_out), rng.uniform(0.5, 2.0, n_out)
    net.sg_set_normalization(xm, xs, ym, ys)
    oracles = []
    for e in range(ensemble):
        Ws, bs = [], []
        for l in range(depth + 1):
            W, b = net.sg_get_params(e, l)
            Ws.append(bf16(W))
            bs.append(b.astype(np.float64))
        oracles.append(MLPOracle(Ws, bs, xm, xs, ym, ys, n_in))
    x = (xm + xs * rng.normal(size=(batch, n_in))).astype(np.float32)
    y = (ym + ys * rng.normal(size=(batch, n_out))).astype(np.float32)
    return net, oracles, x, y


def test_forward_and_gradients_match_oracle(torch_mod):
    torch = torch_mod
    # several 128-wide tiles in every dimension, ragged edges (300, 200, 257)
    net, (o,), x, y = _make(torch, n_in=300, n_out=257, width=384, depth=2, batch=200)
    _say("surrogate small: forward/backward vs oracle")
    xd = torch.tensor(x, device="cuda")
    yd = torch.tensor(y, device="cuda")
    out = torch.empty((200, 257), device="cuda", dtype=torch.float32)
    net.sg_forward(0, xd, out)
    torch.cuda.synchronize()
    pred_o, _ = o.forward(x)
    assert _rel(out.cpu().numpy(), pred_o) <= 1e-3
    loss = net.sg_backward(0, xd, yd)
    loss_o, dW_o, db_o, _ = o.loss_and_grads(x, y)
    assert loss == pytest.approx(loss_o, rel=1e-4)
    for l in range(3):
        dW, db = net.sg_get_grads(0, l)
        if l == 0:
            dW, dWo = dW[:300], dW_o[0][:300]
        else:
            dWo = dW_o[l]
        assert _rel(dW, dWo) <= 1e-3, (l, _rel(dW, dWo))
        assert _rel(db, db_o[l]) <= 1e-3, (l, _rel(db, db_o[l]))


@pytest.mark.parametrize("wd", [0.0, 0.5])
def test_adam_step_matches_oracle(torch_mod, wd):
    torch = torch_mod
    from oracle.mlp_oracle import adam_step
    net, (o,), x, y = _make(torch, n_in=100, n_out=140, width=256, depth=1, batch=64, weight_decay=wd)
    W0 = [net.sg_get_params(0, l)[0].astype(np.float64) for l in range(2)]
    xd, yd = torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda")
    net.sg_train_step(0, xd, yd, lr=1e-3)
    _, dW_o, _, _ = o.loss_and_grads(x, y)
    for l in range(2):
        W1 = net.sg_get_params(0, l)[0].astype(np.float64)
        rows = slice(0, 100) if l == 0 else slice(None)
        want, _, _ = adam_step(W0[l][rows], 0.0, 0.0, dW_o[l][rows], 1, 1e-3, wd=wd)
        diff = np.abs(W1[rows] - want)
        # step 1 of Adam moves every weight by ~lr * sign(g): only signs of
        # near-zero gradients may disagree
        assert diff.max() <= 2.0e-3 + 1e-6
        assert np.mean(diff <= 1e-6) >= 0.99


def test_full_size_forward(torch_mod):
    """The surrogate's real shape: 1803 -> 1024 x 4 (GELU) -> 3600."""
    torch = torch_mod
    net, (o,), x, _ = _make(torch, n_in=1803, n_out=3600, width=1024, depth=4, batch=64, seed=11)
    _say("surrogate full size forward")
    xd = torch.tensor(x, device="cuda")
    out = torch.empty((64, 3600), device="cuda", dtype=torch.float32)
    net.sg_forward(0, xd, out)
    torch.cuda.synchronize()
    pred_o, _ = o.forward(x)
    assert _rel(out.cpu().numpy(), pred_o) <= 1e-3


def test_training_reduces_loss_and_ensemble_predicts(torch_mod):
    torch = torch_mod
    from paper_1707_09073_amd import gfmc
    rng = np.random.default_rng(7)
    n_in, n_out, n = 40, 60, 256
    x = rng.normal(size=(n, n_in)).astype(np.float32)
    A = rng.normal(size=(n_in, n_out)) / np.sqrt(n_in)
    y = np.tanh(x @ A).astype(np.float32) * 3.0 + 1.0
    net = gfmc.SurrogateNet(n_in, n_out, width=256, depth=2, ensemble=3, max_batch=n, seed=5)
    net.sg_set_normalization(x.mean(0), x.std(0), y.mean(0), y.std(0))
    xd, yd = torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda")
    first = [net.sg_backward(e, xd, yd) for e in range(3)]
    for it in range(300):
        for e in range(3):
            net.sg_train_step(e, xd, yd, lr=2e-3, want_loss=False)
    last = [net.sg_backward(e, xd, yd) for e in range(3)]
    assert all(l < f / 20 for f, l in zip(first, last)), (first, last)
    mean = torch.empty((n, n_out), device="cuda"); std = torch.empty((n, n_out), device="cuda")
    net.sg_predict(xd, mean, std)
    torch.cuda.synchronize()
    m = mean.cpu().numpy()
    assert np.linalg.norm(m - y) / np.linalg.norm(y) < 0.1
    # the ensemble mean equals the mean of the members' de-normalised forwards
    outs = []
    for e in range(3):
        o = torch.empty((n, n_out), device="cuda")
        net.sg_forward(e, xd, o)
        outs.append(o.cpu().numpy() * y.std(0) + y.mean(0))
    torch.cuda.synchronize()
    assert np.allclose(m, np.mean(outs, axis=0), rtol=1e-4, atol=1e-4)
    assert np.allclose(std.cpu().numpy(), np.std(outs, axis=0, ddof=1), rtol=1e-3, atol=1e-4)


@pytest.mark.parametrize("shape", [
    # ragged widths (not multiples of the 512-column GEMV block), 3 members
    dict(n_in=300, n_out=257, width=384, depth=2, ensemble=3, seed=13),
    # the surrogate's real shape: 1803 -> 1024 x 4 (GELU) -> 3600, 4 members
    dict(n_in=1803, n_out=3600, width=1024, depth=4, ensemble=4, seed=17),
])
def test_small_batch_predict_matches_oracle_and_gemm_path(torch_mod, shape):
    """sg_predict at batch <= 8 takes the split-K GEMV path; its ensemble mean
    and spread match the oracle's, and the rows agree with the MFMA path."""
    torch = torch_mod
    n_out, E = shape["n_out"], shape["ensemble"]
    net, oracles, x, _ = _make(torch, shape["n_in"], n_out, shape["width"], shape["depth"], batch=16,
                               ensemble=E, seed=shape["seed"])
    _say(f"surrogate small-batch predict {shape}")
    ym, ys = net._norm[2].astype(np.float64), net._norm[3].astype(np.float64)
    outs = np.stack([o.forward(x)[0] * ys + ym for o in oracles])
    mean_o, std_o = outs.mean(0), outs.std(0, ddof=1)
    xd = torch.tensor(x, device="cuda")
    big_m = torch.empty((16, n_out), device="cuda"); big_s = torch.empty_like(big_m)
    net.sg_predict(xd, big_m, big_s)  # batch 16: MFMA path
    big_m, big_s = big_m.cpu().numpy(), big_s.cpu().numpy()
    for lo, hi in [(0, 1), (1, 3), (3, 7), (7, 15), (15, 16)]:
        m = torch.empty((hi - lo, n_out), device="cuda"); s = torch.empty_like(m)
        net.sg_predict(xd[lo:hi].contiguous(), m, s)
        m, s = m.cpu().numpy(), s.cpu().numpy()
        assert _rel(m, mean_o[lo:hi]) <= 1e-3, (lo, hi, _rel(m, mean_o[lo:hi]))
        assert _rel(s, std_o[lo:hi]) <= 2e-2, (lo, hi, _rel(s, std_o[lo:hi]))
        assert _rel(m, big_m[lo:hi]) <= 1e-3
        assert _rel(s, big_s[lo:hi]) <= 2e-2


@pytest.mark.parametrize("width,n_out,batch", [(1024, 3600, 4096), (2048, 600, 4096), (1024, 3600, 3999)])
def test_large_batch_output_layer_matches_oracle(torch_mod, width, n_out, batch):
    """Batches of about 4096 through 1803 -> width -> n_out, in the forward
    products and the backward products of the training step.  Width 1024:
    the output layer has 16 x 15 tiles of 256 x 256 (16-wavefront
    workgroups), the input layer 32 x 8 tiles of 128 x 128 (one per compute
    unit, three LDS stages); batch 3999 leaves the last row of tiles ragged
    and the K slabs of the 1803-wide input a ragged tail.  Width 2048: the
    input layer has 32 x 16 tiles of 128 x 128 (two stages), the 600-wide
    output layer takes the register-staged kernel."""
    torch = torch_mod
    net, (o,), x, y = _make(torch, n_in=1803, n_out=n_out, width=width, depth=1, batch=batch, seed=23)
    _say(f"surrogate batch {batch}, width {width}, {n_out} outputs: forward and gradients vs oracle")
    xd, yd = torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda")
    out = torch.empty((batch, n_out), device="cuda", dtype=torch.float32)
    net.sg_forward(0, xd, out)
    torch.cuda.synchronize()
    loss_o, dW_o, db_o, pred_o = o.loss_and_grads(x, y)
    assert _rel(out.cpu().numpy(), pred_o) <= 1e-3
    loss = net.sg_backward(0, xd, yd)
    assert loss == pytest.approx(loss_o, rel=1e-4)
    first = [net.sg_get_grads(0, l) for l in range(2)]
    for l in range(2):
        dW, db = first[l]
        dWo = dW_o[l][:1803] if l == 0 else dW_o[l]
        dW = dW[:1803] if l == 0 else dW
        assert _rel(dW, dWo) <= 1e-3, (l, _rel(dW, dWo))
        assert _rel(db, db_o[l]) <= 1e-3, (l, _rel(db, db_o[l]))
    # the split products and column sums are added in a fixed order: a second
    # backward on the same inputs gives the same bits
    assert net.sg_backward(0, xd, yd) == loss
    for l in range(2):
        dW, db = net.sg_get_grads(0, l)
        assert np.array_equal(dW, first[l][0]) and np.array_equal(db, first[l][1]), l


def test_predict_or_mc_answers_from_surrogate_or_monte_carlo(torch_mod):
    """sg_predict_or_mc on a 37 x 2 x 5 device grid, against the oracle: each
    member's forward by the MLP oracle on the same BF16 weights, the
    ensemble mean and spread, the decoded maps and the predicted error by the
    oracle's decode.  Within tolerance and the training box the surrogate
    answers with those maps (1e-3, the BF16 bar; the spread, a difference of
    members, to 2e-2).  Outside the box, or beyond the tolerance: the Monte
    Carlo of the given context, equal to the same runs through the mc_*
    calls.  A missing context, one of another grid, or one set up for
    another bias point is refused when the Monte Carlo is needed."""
    from oracle.mlp_oracle import MLPOracle, bf16, decode_maps, ensemble_mean_spread, predicted_error
    from paper_1707_09073_amd import gfmc, workloads as W
    torch = torch_mod
    cells, L = (37, 2, 5), (370.0, 40.0, 100.0)
    nc = cells[0] * cells[1] * cells[2]
    cfg = W.device_config(n_particles=7777, precision="fp32", Vds=3.0, Vgs=-1.0, n_cells=cells, L_nm=L)
    K = cfg["substeps"]
    n_in, n_out, E = 3 + nc, 2 * nc + 2, 3
    net = gfmc.SurrogateNet(n_in, n_out, width=64, depth=2, ensemble=E, max_batch=8, seed=5)
    # normalisation centred away from the queried point, so that the members'
    # different weights give different answers
    xm = np.concatenate([[-0.5, 4.0, 17.5], 290.0 + 5.0 * np.sin(np.arange(nc))])
    xs = np.concatenate([[1.0, 2.0, 0.5], np.full(nc, 20.0)])
    ym = np.zeros(n_out)
    ym[-2:] = [10.0, 20.0]  # log-norms of the two maps
    ys = np.full(n_out, 0.05)
    ys[-2:] = 0.1
    net.sg_set_normalization(xm, xs, ym, ys)
    # the features of the context's bias point: Vgs, Vds, log10 doping (cm^-3), T per subcell
    x = np.concatenate([[cfg["Vgs"], cfg["Vds"], np.log10(cfg["N_D_m3"] * 1e-6)], np.full(nc, cfg["T0_K"])])
    x = x.astype(np.float32)
    _say("predict_or_mc: surrogate answer vs the oracle")
    members = []
    for e in range(E):
        Ws, bs = zip(*[net.sg_get_params(e, l) for l in range(3)])
        o = MLPOracle([bf16(w) for w in Ws], [b.astype(np.float64) for b in bs], xm, xs, ym, ys, n_in)
        members.append(o.forward(x[None])[0] * net._norm[3].astype(np.float64) + net._norm[2].astype(np.float64))
    mean_o, spread_o = ensemble_mean_spread(np.stack(members))
    calib = 1.7
    maps_o = decode_maps(mean_o, nc)[0]
    perr_o = predicted_error(mean_o, spread_o, nc, calib)[0]
    maps, perr, used = net.sg_predict_or_mc(x, calib, tol=1e30)
    assert not used
    assert _rel(maps[:nc], maps_o[:nc]) <= 1e-3 and _rel(maps[nc:], maps_o[nc:]) <= 1e-3
    assert perr == pytest.approx(perr_o, rel=2e-2)
    # and exactly the decoding of sg_predict's own mean and spread
    xd = torch.tensor(x[None], device="cuda")
    m = torch.empty((1, n_out), device="cuda")
    sd = torch.empty_like(m)
    net.sg_predict(xd, m, sd)
    m, sd = m.cpu().numpy().astype(np.float64), sd.cpu().numpy().astype(np.float64)
    assert _rel(maps, decode_maps(m, nc)[0]) <= 1e-6
    assert perr == pytest.approx(predicted_error(m, sd, nc, calib)[0], rel=1e-5)
    _say("predict_or_mc: outside the training box")
    ens, ref = gfmc.Ensemble(cfg), gfmc.Ensemble(cfg)
    assert ens.mc_get_ncell() == nc
    box = (x + 1.0, x + 2.0)  # every feature lies below the box
    maps, _, used = net.sg_predict_or_mc(x, calib, tol=1e30, ens=ens, warm_substeps=5 * K, window_substeps=5 * K,
                                         box=box)
    assert used
    ref.mc_step(5 * K)
    ref.mc_tally(0, reset_window=True)
    ref.mc_step(5 * K)
    r = ref.mc_maps(0)
    assert np.array_equal(maps[:nc], r["heat_Wm3"]) and np.array_equal(maps[nc:], r["density_m3"])
    _say("predict_or_mc: beyond the tolerance")
    maps, perr, used = net.sg_predict_or_mc(x, calib, tol=0.0, ens=ens, warm_substeps=0, window_substeps=3 * K)
    assert used and perr > 0.0
    ref.mc_tally(0, reset_window=True)
    ref.mc_step(3 * K)
    r = ref.mc_maps(0)
    assert np.array_equal(maps[:nc], r["heat_Wm3"]) and np.array_equal(maps[nc:], r["density_m3"])
    _say("predict_or_mc: refused contexts")
    with pytest.raises(gfmc.MCError):
        net.sg_predict_or_mc(x, calib, tol=0.0)
    other = gfmc.Ensemble(W.device_config(n_particles=4000, precision="fp32", n_cells=(20, 2, 2),
                                          L_nm=(200.0, 20.0, 20.0)))
    with pytest.raises(gfmc.MCError):
        net.sg_predict_or_mc(x, calib, tol=0.0, ens=other, window_substeps=K)
    wrong_bias = gfmc.Ensemble(dict(cfg, Vds=4.0))
    with pytest.raises(gfmc.MCError):
        net.sg_predict_or_mc(x, calib, tol=0.0, ens=wrong_bias, window_substeps=K)
    with pytest.raises(gfmc.MCError):
        net.sg_predict_or_mc(x, calib, tol=0.0, ens=ens, instance=1, window_substeps=K)
    T = np.full(nc, 300.0)
    T[5] = 310.0
    hot = gfmc.Ensemble(dict(cfg, T_cells=T))
    with pytest.raises(gfmc.MCError):
        net.sg_predict_or_mc(x, calib, tol=0.0, ens=hot, window_substeps=K)
    for e in (ens, ref, other, wrong_bias, hot):
        e.close()
    net.close()
