"""Pins for the U-Net oracle (CPU): each primitive against an independent
definition or an exact identity, the whole backward pass against central
differences, Adam against its first-step closed form, and the bfloat16
rounding against torch's conversion."""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import unet


def _rng(s=0):
    return np.random.default_rng(s)


def test_conv3_matches_scipy_correlate_channel_by_channel():
    r = _rng(1)
    X = r.standard_normal((5, 6, 7, 3))
    W = r.standard_normal((27, 3, 2))
    Y = unet.conv3(X, W)
    for co in range(2):
        ref = sum(ndi.correlate(X[..., ci], W[:, ci, co].reshape(3, 3, 3), mode="constant", cval=0.0)
                  for ci in range(3))
        assert np.abs(Y[..., co] - ref).max() < 1e-12


def test_conv3_gradients_are_the_adjoints():
    r = _rng(2)
    X = r.standard_normal((4, 5, 6, 3))
    W = r.standard_normal((27, 3, 4))
    dY = r.standard_normal((4, 5, 6, 4))
    lhs = (unet.conv3(X, W) * dY).sum()
    assert abs(lhs - (X * unet.conv3_dgrad(dY, W)).sum()) < 1e-10 * abs(lhs)
    assert abs(lhs - (W * unet.conv3_wgrad(X, dY)).sum()) < 1e-10 * abs(lhs)
    # a single tap picks one neighbour: identity kernel at the centre
    Wc = np.zeros((27, 3, 3))
    Wc[13] = np.eye(3)
    assert np.array_equal(unet.conv3(X, Wc), X)
    # tap 0 is the offset (-1, -1, -1)
    W0 = np.zeros((27, 3, 3))
    W0[0] = np.eye(3)
    Y = unet.conv3(X, W0)
    assert np.array_equal(Y[1:, 1:, 1:], X[:-1, :-1, :-1]) and not Y[0].any()


def test_pool_and_upsample_are_adjoint_and_consistent():
    r = _rng(3)
    X = r.standard_normal((4, 6, 8, 2))
    P = r.standard_normal((2, 3, 4, 2))
    assert abs((unet.pool2(X) * P).sum() - (X * unet.pool2_bwd(P)).sum()) < 1e-12
    assert abs((unet.up2(P) * X).sum() - (P * unet.up2_bwd(X)).sum()) < 1e-12
    assert np.allclose(unet.pool2(unet.up2(P)), P)
    assert np.allclose(unet.pool2(np.full((4, 4, 4, 1), 3.0)), 3.0)


def _params(seed, scale=0.3):
    r = _rng(seed)
    W = [r.standard_normal((27, ci, co)) * scale / np.sqrt(27 * ci) * np.sqrt(2) for ci, co in unet.layer_shapes()]
    return {"W": W, "w_out": r.standard_normal(unet.CH[0]) * 0.3}


def _loss(params, X, T, mask):
    out, _ = unet.forward(params, X)
    return unet.mse(out, T, mask)[0]


def test_backward_matches_central_differences():
    r = _rng(4)
    params = _params(5)
    X = np.zeros((8, 8, 8, unet.IN_CH))
    X[..., :2] = r.standard_normal((8, 8, 8, 2))
    T = r.standard_normal((8, 8, 8))
    mask = np.ones((8, 8, 8))
    mask[:, :, 6:] = 0.0
    out, cache = unet.forward(params, X)
    L, dout = unet.mse(out, T, mask)
    g = unet.backward(cache, dout)
    # directional derivative along a random direction in weight space
    d = {"W": [r.standard_normal(w.shape) for w in params["W"]], "w_out": r.standard_normal(unet.CH[0])}
    gd = sum((a * b).sum() for a, b in zip(g["W"], d["W"])) + (g["w_out"] * d["w_out"]).sum()
    eps = 1e-6

    def moved(s):
        return {"W": [w + s * eps * dw for w, dw in zip(params["W"], d["W"])],
                "w_out": params["w_out"] + s * eps * d["w_out"]}

    fd = (_loss(moved(1), X, T, mask) - _loss(moved(-1), X, T, mask)) / (2 * eps)
    assert abs(fd - gd) <= 1e-6 * abs(gd), (fd, gd)
    # single weights of the first and of a skip-consuming layer
    for k, idx in ((0, (13, 1, 3)), (12, (4, 40, 7)), (6, (0, 5, 9))):
        p2 = {"W": [w.copy() for w in params["W"]], "w_out": params["w_out"]}
        p2["W"][k][idx] += eps
        lp = _loss(p2, X, T, mask)
        p2["W"][k][idx] -= 2 * eps
        lm = _loss(p2, X, T, mask)
        assert abs((lp - lm) / (2 * eps) - g["W"][k][idx]) <= 1e-5 * max(1e-8, abs(g["W"][k][idx])) + 1e-10


def test_adam_first_step_moves_by_lr_times_sign():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    w1, m, v = unet.adam(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(w1, w - 0.01 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding_matches_torch_and_ties_to_even():
    torch = pytest.importorskip("torch")
    r = _rng(6)
    x = np.concatenate([r.standard_normal(10000) * 10.0 ** r.integers(-6, 6, 10000),
                        [1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -0.0, 0.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(unet.bf16(x), ref)
    assert unet.bf16(1.0 + 2.0 ** -8) == 1.0               # tie -> even
    assert unet.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie -> even (up)
