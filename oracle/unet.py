"""Plain FP64 numpy reference of the learned correction network (test infrastructure only).

The network is not in the paper: it is the learned form of the preconditioner, a small
convolutional U-Net applied after the mean-value block solve A_0^{-1} (Section 5) inside
flexible GMRES.  What it computes is fixed here by plain definitions, in NHWC layout
(image rows, columns, channels; channels fastest):

  conv3(X, W, b)[y, x, o] = b[o] + Σ_{dy, dx ∈ {-1,0,1}} Σ_c W[o, dy+1, dx+1, c] X[y+dy, x+dx, c]
                            (cross-correlation, zero padding outside the image)
  conv1(X, W, b)[y, x, o] = b[o] + Σ_c W[o, 0, 0, c] X[y, x, c]
  relu(z) = max(z, 0);  pool(X) = mean of 2×2 blocks;  up(X) = nearest 2× upsampling
  concat(U, S) = channels of U followed by the channels of S

  U-Net, channel widths (32, 64, 128), H and W divisible by 4:
    s0 = relu(conv3(relu(conv3(x, enc0a)), enc0b))                 H   × W   × 32
    s1 = relu(conv3(relu(conv3(pool(s0), enc1a)), enc1b))          H/2 × W/2 × 64
    bt = relu(conv3(relu(conv3(pool(s1), bota)), botb))            H/4 × W/4 × 128
    d1 = relu(conv3(relu(conv3(concat(up(bt), s1), dec1a)), dec1b))  H/2 × W/2 × 64
    d0 = relu(conv3(relu(conv3(concat(up(d1), s0), dec0a)), dec0b))  H × W × 32
    y  = conv1(d0, head)                                           H × W × c_out
  loss(y, t) = mean((y - t)²) over all H·W·c_out entries.

Parameters are flattened layer by layer in the order of LAYERS, each as W (shape
[c_out, k, k, c_in], C order) followed by b [c_out].  Adam follows Kingma & Ba (2015):
m ← β1 m + (1-β1) g, v ← β2 v + (1-β2) g², θ ← θ - lr m̂ / (sqrt(v̂) + ε) with the bias
corrections m̂ = m / (1-β1^t), v̂ = v / (1-β2^t).

The mapping between an SG vector (Q PC blocks of an n×n grid, complex) and the network
tensors: input channels 2q, 2q+1 = Re, Im of block q scaled by sqrt(Q·n²)/||r||, then the
s+1 coefficient fields k_l / k̄; the grid is zero-padded to H = W = ceil(n/4)·4.  Output
channels 2q, 2q+1 are Re, Im of the correction of block q in units of
||A_0^{-1} r|| / sqrt(Q·n²).

Storage precision.  The network keeps its input, its convolution weights and every
stored activation and activation gradient in bfloat16 (8-bit exponent, 8-bit significand,
round to nearest even), with biases, the head output, accumulation and parameter
gradients in higher precision.  ``forward`` and ``loss_and_grad`` take an optional
rounding function applied at exactly those storage points (``bf16_round``); without it
they are the exact FP64 definitions.

Parity unpinned against the paper (no network exists there); pinned by the tests
against library correlation, adjoint identities, central finite differences, the
closed-form first Adam step, and exact bfloat16 values.
"""
from __future__ import annotations

import numpy as np

WIDTHS = (32, 64, 128)


def layers(c_in: int, c_out: int):
    """(name, kernel size, input channels, output channels) of every layer, in order."""
    w0, w1, w2 = WIDTHS
    return [
        ("enc0a", 3, c_in, w0), ("enc0b", 3, w0, w0),
        ("enc1a", 3, w0, w1), ("enc1b", 3, w1, w1),
        ("bota", 3, w1, w2), ("botb", 3, w2, w2),
        ("dec1a", 3, w2 + w1, w1), ("dec1b", 3, w1, w1),
        ("dec0a", 3, w1 + w0, w0), ("dec0b", 3, w0, w0),
        ("head", 1, w0, c_out),
    ]


def num_params(c_in: int, c_out: int) -> int:
    return sum(co * k * k * ci + co for _, k, ci, co in layers(c_in, c_out))


def unflatten(theta: np.ndarray, c_in: int, c_out: int) -> dict:
    out, off = {}, 0
    for name, k, ci, co in layers(c_in, c_out):
        nw = co * k * k * ci
        out[name] = (theta[off:off + nw].reshape(co, k, k, ci), theta[off + nw:off + nw + co])
        off += nw + co
    assert off == theta.size
    return out


def flatten(grads: dict, c_in: int, c_out: int) -> np.ndarray:
    parts = []
    for name, _, _, _ in layers(c_in, c_out):
        gw, gb = grads[name]
        parts += [gw.ravel(), gb.ravel()]
    return np.concatenate(parts)


# ---- building blocks and their adjoints ------------------------------------------------

def conv(X: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Cross-correlation with zero padding (k = 1 or 3), plus bias."""
    H, Wd, _ = X.shape
    co, k, _, _ = W.shape
    r = k // 2
    Xp = np.pad(X, ((r, r), (r, r), (0, 0)))
    Y = np.broadcast_to(b, (H, Wd, co)).astype(np.float64).copy()
    for i in range(k):
        for j in range(k):
            Y += Xp[i:i + H, j:j + Wd, :] @ W[:, i, j, :].T
    return Y


def conv_backward(X: np.ndarray, W: np.ndarray, dY: np.ndarray):
    """Gradients of Σ dY·conv(X, W, b) with respect to X, W and b."""
    H, Wd, _ = X.shape
    co, k, _, ci = W.shape
    r = k // 2
    Xp = np.pad(X, ((r, r), (r, r), (0, 0)))
    dXp = np.zeros_like(Xp)
    dW = np.zeros_like(W)
    for i in range(k):
        for j in range(k):
            dXp[i:i + H, j:j + Wd, :] += dY @ W[:, i, j, :]
            dW[:, i, j, :] = np.einsum("yxo,yxc->oc", dY, Xp[i:i + H, j:j + Wd, :])
    db = dY.sum(axis=(0, 1))
    return dXp[r:r + H, r:r + Wd, :], dW, db


def pool(X: np.ndarray) -> np.ndarray:
    H, W, C = X.shape
    return X.reshape(H // 2, 2, W // 2, 2, C).mean(axis=(1, 3))


def pool_backward(dY: np.ndarray) -> np.ndarray:
    return np.repeat(np.repeat(dY, 2, axis=0), 2, axis=1) / 4.0


def up(X: np.ndarray) -> np.ndarray:
    return np.repeat(np.repeat(X, 2, axis=0), 2, axis=1)


def up_backward(dY: np.ndarray) -> np.ndarray:
    H, W, C = dY.shape
    return dY.reshape(H // 2, 2, W // 2, 2, C).sum(axis=(1, 3))


def relu(z):
    return np.maximum(z, 0.0)


def bf16_round(a) -> np.ndarray:
    """Nearest bfloat16 value (ties to even) of each entry, returned as float64: the float32
    value of the entry with its 16 low significand bits rounded away."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _identity(a):
    return a


# ---- the network ------------------------------------------------------------------------

def forward(theta: np.ndarray, x: np.ndarray, c_out: int, keep: bool = False, rnd=None):
    """Network output for one NHWC input; with keep=True also the intermediate tensors.
    rnd: rounding applied to the input, the weights and every stored activation."""
    rnd = rnd or _identity
    P = {k: (rnd(w), b) for k, (w, b) in unflatten(theta, x.shape[2], c_out).items()}
    t = {"x": rnd(x)}

    def cr(name, inp):
        return rnd(relu(conv(inp, *P[name])))

    t["e0a"] = cr("enc0a", t["x"])
    t["s0"] = cr("enc0b", t["e0a"])
    t["p0"] = rnd(pool(t["s0"]))
    t["e1a"] = cr("enc1a", t["p0"])
    t["s1"] = cr("enc1b", t["e1a"])
    t["p1"] = rnd(pool(t["s1"]))
    t["ba"] = cr("bota", t["p1"])
    t["bt"] = cr("botb", t["ba"])
    t["c1"] = np.concatenate([up(t["bt"]), t["s1"]], axis=2)
    t["d1a"] = cr("dec1a", t["c1"])
    t["d1"] = cr("dec1b", t["d1a"])
    t["c0"] = np.concatenate([up(t["d1"]), t["s0"]], axis=2)
    t["d0a"] = cr("dec0a", t["c0"])
    t["d0"] = cr("dec0b", t["d0a"])
    t["y"] = conv(t["d0"], *P["head"])
    t["P"] = P
    return (t["y"], t) if keep else t["y"]


def loss(y: np.ndarray, target: np.ndarray) -> float:
    return float(np.mean((y - target) ** 2))


def loss_and_grad(theta: np.ndarray, x: np.ndarray, target: np.ndarray, rnd=None):
    """Loss and its gradient with respect to theta (flat) and to the input x.  rnd: rounding
    of the forward pass (see ``forward``) and of every stored activation gradient."""
    rnd = rnd or _identity
    c_in, c_out = x.shape[2], target.shape[2]
    y, t = forward(theta, x, c_out, keep=True, rnd=rnd)
    P = t["P"]
    L = loss(y, target)
    g = {}
    dy = rnd(2.0 * (y - target) / y.size)

    def back(name, inp, out, dout):
        # out = relu(conv(inp)) except for the head (no activation)
        dz = dout if name == "head" else dout * (out > 0)
        dx, dw, db = conv_backward(inp, P[name][0], dz)
        g[name] = (dw, db)
        return dx

    dd0 = rnd(back("head", t["d0"], None, dy))
    dd0a = rnd(back("dec0b", t["d0a"], t["d0"], dd0))
    dc0 = rnd(back("dec0a", t["c0"], t["d0a"], dd0a))
    w1 = WIDTHS[1]
    dd1 = rnd(up_backward(dc0[:, :, :w1]))
    ds0 = dc0[:, :, w1:].copy()
    dd1a = rnd(back("dec1b", t["d1a"], t["d1"], dd1))
    dc1 = rnd(back("dec1a", t["c1"], t["d1a"], dd1a))
    w2 = WIDTHS[2]
    dbt = rnd(up_backward(dc1[:, :, :w2]))
    ds1 = dc1[:, :, w2:].copy()
    dba = rnd(back("botb", t["ba"], t["bt"], dbt))
    dp1 = rnd(back("bota", t["p1"], t["ba"], dba))
    ds1 = rnd(ds1 + pool_backward(dp1))
    de1a = rnd(back("enc1b", t["e1a"], t["s1"], ds1))
    dp0 = rnd(back("enc1a", t["p0"], t["e1a"], de1a))
    ds0 = rnd(ds0 + pool_backward(dp0))
    de0a = rnd(back("enc0b", t["e0a"], t["s0"], ds0))
    dx = back("enc0a", t["x"], t["e0a"], de0a)
    return L, flatten(g, c_in, c_out), dx


def adam_step(theta, m, v, grad, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step number t >= 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def he_init(c_in: int, c_out: int, rng: np.random.Generator) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; the head is scaled by 0.1."""
    parts = []
    for name, k, ci, co in layers(c_in, c_out):
        std = np.sqrt(2.0 / (k * k * ci)) * (0.1 if name == "head" else 1.0)
        parts += [rng.standard_normal(co * k * k * ci) * std, np.zeros(co)]
    return np.concatenate(parts)


# ---- SG vector ↔ network tensors -------------------------------------------------------

def padded_size(n: int) -> int:
    return (n + 3) // 4 * 4


def pack_input(r: np.ndarray, k_fields: np.ndarray, kbar: float, Q: int, n: int) -> np.ndarray:
    """NHWC input of a residual r (Q·n² complex, blocks of n×n with x fastest)."""
    H = padded_size(n)
    s1 = k_fields.shape[0]
    R = np.asarray(r).reshape(Q, n, n) * (np.sqrt(Q * n * n) / np.linalg.norm(r))
    x = np.zeros((H, H, 2 * Q + s1))
    x[:n, :n, 0:2 * Q:2] = np.moveaxis(R.real, 0, 2)
    x[:n, :n, 1:2 * Q:2] = np.moveaxis(R.imag, 0, 2)
    x[:n, :n, 2 * Q:] = np.moveaxis(np.asarray(k_fields).reshape(s1, n, n) / kbar, 0, 2)
    return x


def unpack_output(y: np.ndarray, scale: float, Q: int, n: int) -> np.ndarray:
    """SG vector (Q·n² complex) of the network output, times scale / sqrt(Q·n²)."""
    c = (y[:n, :n, 0:2 * Q:2] + 1j * y[:n, :n, 1:2 * Q:2]) * (scale / np.sqrt(Q * n * n))
    return np.moveaxis(c, 2, 0).reshape(-1)


def pack_target(c: np.ndarray, scale: float, Q: int, n: int) -> np.ndarray:
    """NHWC target of a correction c (SG vector) in units of scale / sqrt(Q·n²)."""
    H = padded_size(n)
    C = np.asarray(c).reshape(Q, n, n) * (np.sqrt(Q * n * n) / scale)
    t = np.zeros((H, H, 2 * Q))
    t[:n, :n, 0::2] = np.moveaxis(C.real, 0, 2)
    t[:n, :n, 1::2] = np.moveaxis(C.imag, 0, 2)
    return t
