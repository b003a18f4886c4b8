"""Pins of the FP64 reference of the learned view scorer (oracle/surrogate.py): bfloat16
rounding against torch's conversion, im2col against scipy's correlation and its adjoint
identity, and the FP64 backward pass against central finite differences."""
import numpy as np
import pytest
import torch
from scipy.signal import correlate2d

from oracle import surrogate as S


def random_params(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    shapes = [(co, ci * 9) for ci, co in S.CONV] + [(S.WIDTH, S.WIDTH), (1, S.WIDTH)]
    w = [rng.normal(0, scale * (2.0 / s[1]) ** 0.5, s) for s in shapes]
    b = [rng.normal(0, 0.05, s[0]) for s in shapes]
    return w, b


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 1, 10000), rng.normal(0, 1e-3, 1000) * 1e3, [1.0, 1 + 2 ** -9, 1 + 3 * 2 ** -9]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16(x), ref)
    assert S.bf16(np.array([1 + 2 ** -9]))[0] == 1.0            # tie to even
    assert S.bf16(np.array([1 + 3 * 2 ** -9]))[0] == 1 + 2 ** -7  # tie to even (up)


def test_im2col_matches_correlation_and_adjoint():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(3, 2, 11, 14))
    k = rng.normal(size=(3, 9))
    col = S.im2col(x)
    y = (k.reshape(1, -1) @ col).reshape(2, S.out_size(11), S.out_size(14))
    for bi in range(2):
        ref = sum(correlate2d(np.pad(x[c, bi], 1), k[c].reshape(3, 3), mode="valid") for c in range(3))[::2, ::2]
        assert np.allclose(y[bi], ref, atol=1e-12)
    d = rng.normal(size=col.shape)
    assert abs(np.sum(col * d) - np.sum(x * S.col2im(d, 3, 2, 11, 14))) < 1e-9


def test_backward_matches_finite_differences_fp64():
    w, b = random_params(3)
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, (4, 2, S.IN_H, S.IN_W))
    c = rng.normal(size=2)
    pred, cache = S.forward(w, b, x, bf=False)
    gw, gb = S.backward(w, cache, c, bf=False)
    checked = 0
    for l in range(6):
        for _ in range(4):
            i = tuple(rng.integers(0, s) for s in w[l].shape)
            h = 1e-6
            w[l][i] += h
            lp = c @ S.forward(w, b, x, bf=False)[0]
            w[l][i] -= 2 * h
            lm = c @ S.forward(w, b, x, bf=False)[0]
            w[l][i] += h
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gw[l][i]) <= 1e-6 * max(1.0, abs(fd)), (l, i, fd, gw[l][i])
            checked += 1
        j = int(rng.integers(0, b[l].shape[0]))
        b[l][j] += 1e-6
        lp = c @ S.forward(w, b, x, bf=False)[0]
        b[l][j] -= 2e-6
        lm = c @ S.forward(w, b, x, bf=False)[0]
        b[l][j] += 1e-6
        assert abs((lp - lm) / 2e-6 - gb[l][j]) <= 1e-6 * max(1.0, abs(gb[l][j]))
    assert checked == 24


def test_mse_gradient():
    p, t = np.array([1.0, 2.0, 4.0]), np.array([0.0, 2.0, 1.0])
    loss, d = S.mse(p, t)
    assert loss == pytest.approx(10.0 / 3.0)
    assert np.allclose(d, [2.0 / 3.0, 0.0, 2.0])
