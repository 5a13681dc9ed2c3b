"""The allocation-free small-batch predictor against sg_predict, through the
C ABI: the same ensemble mean and spread (the split sums may run in another
order), on two calls in a row, the second with a smaller batch, and against
the MLP oracle on the same BF16 weights."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def test_static_scratch_predict_equals_workspace_predict():
    import torch
    assert torch.cuda.is_available()
    from oracle.mlp_oracle import MLPOracle, bf16
    from paper_1707_09073_amd import gfmc
    n_in, n_out, width, depth, E = 1803, 3602, 1024, 4, 4
    net = gfmc.SurrogateNet(n_in, n_out, width=width, depth=depth, ensemble=E, max_batch=16, seed=29)
    rng = np.random.default_rng(29)
    xm, xs = rng.normal(size=n_in), rng.uniform(0.5, 2.0, n_in)
    ym, ys = rng.normal(size=n_out), rng.uniform(0.5, 2.0, n_out)
    net.sg_set_normalization(xm, xs, ym, ys)
    members = []
    for e in range(E):
        Ws, bs = zip(*[net.sg_get_params(e, l) for l in range(depth + 1)])
        members.append(MLPOracle([bf16(w) for w in Ws], [b.astype(np.float64) for b in bs], xm, xs, ym, ys, n_in))
    for batch, seed in ((8, 1), (3, 2)):
        _say(f"static-scratch predict: batch {batch}")
        x = (xm + xs * np.random.default_rng(seed).normal(size=(batch, n_in))).astype(np.float32)
        xd = torch.tensor(x, device="cuda")
        m_ws, s_ws = torch.empty((batch, n_out), device="cuda"), torch.empty((batch, n_out), device="cuda")
        m_st, s_st = torch.full_like(m_ws, np.nan), torch.full_like(s_ws, np.nan)
        net.sg_predict(xd, m_ws, s_ws)
        net.sg_predict_static(xd, m_st, s_st)
        torch.cuda.synchronize()
        m_ws, s_ws, m_st, s_st = (t.cpu().numpy() for t in (m_ws, s_ws, m_st, s_st))
        assert np.all(np.isfinite(m_st)) and np.all(np.isfinite(s_st))
        assert _rel(m_st, m_ws) <= 1e-3, _rel(m_st, m_ws)
        assert _rel(s_st, s_ws) <= 2e-2, _rel(s_st, s_ws)
        outs = np.stack([o.forward(x)[0] * ys.astype(np.float32) + ym.astype(np.float32) for o in members])
        assert _rel(m_st, outs.mean(0)) <= 1e-3
        assert _rel(s_st, outs.std(0, ddof=1)) <= 2e-2
    # more rows than the small-batch path takes: refused, nothing launched
    x = torch.zeros((9, n_in), device="cuda")
    out = torch.empty((9, n_out), device="cuda")
    with pytest.raises(gfmc.MCError):
        net.sg_predict_static(x, out, out)
    net.close()
