"""Host logic of the surrogate runtime (no GPU): the target encoding (unit
shape and log-norm per map) inverts exactly, its predicted-error estimate
behaves as a relative error, and the input features follow the recipe."""
import math

import numpy as np

from paper_1707_09073_amd import surrogate as S
from paper_1707_09073_amd import workloads as W


def test_encode_decode_round_trip():
    rng = np.random.default_rng(0)
    Y = np.concatenate([rng.normal(size=(5, S.N_CELL)) * 1e17, rng.uniform(1e22, 1e25, (5, S.N_CELL))], axis=1)
    T = S.encode(Y)
    assert T.shape == (5, S.N_ENC)
    for k in range(2):
        sl = slice(k * S.N_CELL, (k + 1) * S.N_CELL)
        assert np.allclose(np.linalg.norm(T[:, sl], axis=1), 1.0, rtol=1e-14)
    assert np.allclose(S.decode(T), Y, rtol=1e-12, atol=0)


def test_encoded_spread_is_a_relative_error():
    rng = np.random.default_rng(1)
    T = S.encode(rng.uniform(1.0, 2.0, (4, 2 * S.N_CELL)))
    # no spread -> no predicted error
    assert np.all(S.encoded_spread(T, np.zeros_like(T)) == 0.0)
    # a log-norm spread of 0.03 alone is a 3% relative error
    sd = np.zeros_like(T)
    sd[:, 2 * S.N_CELL] = 0.03
    assert np.allclose(S.encoded_spread(T, sd), 0.03)
    # a shape spread of 1% of the shape norm is a 1% error; both combine in quadrature
    sd[:, :S.N_CELL] = 0.01 * T[:, :S.N_CELL]
    assert np.allclose(S.encoded_spread(T, sd), math.hypot(0.01, 0.03))


def test_rel_l2_and_features():
    ref = np.ones((2, 2 * S.N_CELL))
    pred = ref.copy()
    pred[0, :S.N_CELL] *= 1.02
    e = S.rel_l2(pred, ref)
    assert np.allclose(e[0], [0.02, 0.0]) and np.allclose(e[1], 0.0)
    cfg = W.surrogate_inputs(1, seed=5)[0]
    f = S.features(cfg)
    assert f.shape == (3 + S.N_CELL,)
    assert f[0] == np.float32(cfg["Vgs"]) and f[1] == np.float32(cfg["Vds"])
    assert math.isclose(f[2], math.log10(cfg["N_D_m3"] * 1e-6), rel_tol=1e-6)
    assert np.allclose(f[3:], cfg["T_cells"], rtol=1e-6)


def test_host_decode_and_spread_equal_the_oracle():
    """The batched runtime decodes maps and predicted errors on the host;
    both equal the oracle's definitions (the ones the library's one-query
    entry point follows)."""
    from oracle.mlp_oracle import decode_maps, predicted_error
    rng = np.random.default_rng(4)
    mean = S.encode(rng.uniform(1.0, 5.0, (6, 2 * S.N_CELL)) * np.array([[1e12] * S.N_CELL + [1e24] * S.N_CELL]))
    spread = np.abs(rng.normal(0.0, 0.01, mean.shape))
    assert np.allclose(S.decode(mean), decode_maps(mean, S.N_CELL), rtol=1e-13, atol=0)
    assert np.allclose(S.encoded_spread(mean, spread), predicted_error(mean, spread, S.N_CELL, 1.0), rtol=1e-13)
