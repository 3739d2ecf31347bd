"""Oracle for the learned preconditioner's 3D U-Net: forward pass, backward
pass (input and weight gradients), mean-squared-error loss and one Adam
step, in FP64 numpy by direct definition.

TEST INFRASTRUCTURE ONLY (see oracle/mesh.py): imported by tests/ and by
nothing on the product path.

The paper does not contain this network; it is the learned preconditioner
added to the pressure solve (CG with a preconditioner that is a trained
network, used in flexible CG).  The definitions written out here:

* voxel grids are channels-last arrays X[z, y, x, c];
* conv3(X, W), W[t, ci, co] with taps t = 9 (dz+1) + 3 (dy+1) + (dx+1) over
  the offsets (dz, dy, dx) in {-1, 0, 1}^3:
      Y[z, y, x, co] = sum_t sum_ci X[z+dz, y+dy, x+dx, ci] W[t, ci, co],
  zero outside the grid (same padding), no bias;
* relu(a) = max(a, 0); pool2 = mean over 2x2x2 blocks; up2 = nearest
  neighbour (each voxel copied to its 2x2x2 children);
* the network: two conv3+relu per level on the way down (channels 16, 32,
  48, 64 on four levels), pool2 between levels; on the way up up2, then the
  concatenation [upsampled, skip] of the channels, then two conv3+relu;
  finally a 1x1x1 convolution to one channel (weights w_out[16]);
* loss L = (1/|mask|) sum_mask (out - target)^2;
* Adam: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
  w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).

Optional bf16 storage emulation (store="bf16"): values are rounded to
bfloat16 (round to nearest, ties to even) where the GPU network stores them:
network input, the 3x3x3 weights, every stored activation and activation
gradient (the final 1x1x1 weights stay unrounded).
Arithmetic itself stays FP64.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
IN_CH = 8        # input channels as stored (2 used: coefficient, residual)
CH = (16, 32, 48, 64)


def bf16(a):
    """Round FP64 values to the nearest bfloat16 (ties to even), as FP64."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _st(a, store):
    return bf16(a) if store == "bf16" else a


def shift(X, dz, dy, dx):
    """S[z, y, x] = X[z+dz, y+dy, x+dx], zero where that lies outside."""
    S = np.zeros_like(X)
    D, H, W = X.shape[:3]

    def rng(d, n):
        return (max(0, -d), min(n, n - d))

    (z0, z1), (y0, y1), (x0, x1) = rng(dz, D), rng(dy, H), rng(dx, W)
    S[z0:z1, y0:y1, x0:x1] = X[z0 + dz:z1 + dz, y0 + dy:y1 + dy, x0 + dx:x1 + dx]
    return S


def conv3(X, W):
    Y = np.zeros(X.shape[:3] + (W.shape[2],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        Y += shift(X, dz, dy, dx) @ W[t]
    return Y


def conv3_dgrad(dY, W):
    """Gradient with respect to X of sum(conv3(X, W) * dY)."""
    dX = np.zeros(dY.shape[:3] + (W.shape[1],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        dX += shift(dY, -dz, -dy, -dx) @ W[t].T
    return dX


def conv3_wgrad(X, dY):
    """Gradient with respect to W of sum(conv3(X, W) * dY)."""
    ci, co = X.shape[3], dY.shape[3]
    dW = np.zeros((27, ci, co))
    Yf = dY.reshape(-1, co)
    for t, (dz, dy, dx) in enumerate(TAPS):
        dW[t] = shift(X, dz, dy, dx).reshape(-1, ci).T @ Yf
    return dW


def relu(a):
    return np.maximum(a, 0.0)


def pool2(X):
    D, H, W, C = X.shape
    return X.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(1, 3, 5))


def pool2_bwd(dP):
    return np.repeat(np.repeat(np.repeat(dP, 2, 0), 2, 1), 2, 2) / 8.0


def up2(X):
    return np.repeat(np.repeat(np.repeat(X, 2, 0), 2, 1), 2, 2)


def up2_bwd(dU):
    D, H, W, C = dU.shape
    return dU.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


def layer_shapes():
    """(ci, co) of the fourteen 3x3x3 convolutions in order."""
    c0, c1, c2, c3 = CH
    return [(IN_CH, c0), (c0, c0), (c0, c1), (c1, c1), (c1, c2), (c2, c2), (c2, c3), (c3, c3),
            (c3 + c2, c2), (c2, c2), (c2 + c1, c1), (c1, c1), (c1 + c0, c0), (c0, c0)]


def forward(params, X, store=None):
    """params: {"W": [14 arrays (27, ci, co)], "w_out": (16,)}; X (D, H, W, 8).
    Returns the one-channel output (D, H, W) and the cache for backward."""
    Ws = [_st(w, store) for w in params["W"]]
    wo = np.asarray(params["w_out"], dtype=np.float64)  # kept in FP32 on the GPU
    X = _st(X, store)
    c = {"X": X}
    a = X
    skips = []
    k = 0
    for lev in range(4):
        for _ in range(2):
            c[f"in{k}"] = a
            a = _st(relu(conv3(a, Ws[k])), store)
            c[f"a{k}"] = a
            k += 1
        if lev < 3:
            skips.append(a)
            a = _st(pool2(a), store)
    for lev in (2, 1, 0):
        a = np.concatenate([up2(a), skips[lev]], axis=3)
        for _ in range(2):
            c[f"in{k}"] = a
            a = _st(relu(conv3(a, Ws[k])), store)
            c[f"a{k}"] = a
            k += 1
    out = a @ wo
    c["Ws"], c["wo"], c["last"] = Ws, wo, a
    return out, c


def backward(c, dout, store=None):
    """Gradients of sum(out * dout) with respect to the weights."""
    Ws, wo = c["Ws"], c["wo"]
    g_out = c["last"].reshape(-1, CH[0]).T @ dout.reshape(-1)
    da = _st(dout[..., None] * wo[None, None, None, :], store)
    gW = [None] * 14
    dskip = {}
    k = 13
    for lev in (0, 1, 2):
        for _ in range(2):
            dy = _st(da * (c[f"a{k}"] > 0), store)
            gW[k] = conv3_wgrad(c[f"in{k}"], dy)
            da = _st(conv3_dgrad(dy, Ws[k]), store)
            k -= 1
        cu = da.shape[3] - (CH[lev])
        dskip[lev] = da[..., cu:]
        da = _st(up2_bwd(da[..., :cu]), store)
    for lev in (3, 2, 1, 0):
        for j in range(2):
            dy = _st(da * (c[f"a{k}"] > 0), store)
            gW[k] = conv3_wgrad(c[f"in{k}"], dy)
            if k > 0:
                da = _st(conv3_dgrad(dy, Ws[k]), store)
            k -= 1
        if lev > 0:
            # into the skip output of the level above: its own gradient from
            # the concatenation plus the pooled path
            da = _st(dskip[lev - 1] + pool2_bwd(da), store)
    return {"W": gW, "w_out": g_out}


def mse(out, target, mask):
    d = (out - target) * mask
    n = mask.sum()
    return float((d * d).sum() / n), 2.0 * d / n


def adam(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
