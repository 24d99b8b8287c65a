"""Reference U-Net for the learned warm start (plain NumPy, float64).

Test infrastructure (oracle); see the package docstring.  The network is not
part of the paper: it predicts a start field for the Basic Scheme (Sec. 4).
This module writes its forward and backward passes out directly, layer by
layer, for checking the GPU kernels:

* 3x3x3 convolution with periodic padding, out[p] = sum_t W_t in[p + d_t] + b,
  taps t = 9 (dz+1) + 3 (dy+1) + (dx+1); 1x1 convolution for the head;
* ReLU, 2x2x2 average pooling, nearest x2 upsampling, channel concatenation;
* mean squared error over the first 36 head channels.

Parameters are one flat vector: every layer's weights [t][co][ci] in layer
order, then every layer's biases.  ``emulate_bf16`` rounds weights and every
stored activation / activation gradient to bfloat16 at the points where the
GPU stores them, so that both sides take the same rounding decisions.
"""
from __future__ import annotations

import numpy as np

LAYERS = [(32, 32, 3), (32, 32, 3), (32, 64, 3), (64, 64, 3), (64, 128, 3), (128, 128, 3),
          (192, 64, 3), (64, 64, 3), (96, 32, 3), (32, 32, 3), (32, 64, 1)]
E1A, E1B, E2A, E2B, E3A, E3B, D2A, D2B, D1A, D1B, HEAD = range(11)


def bf16(x):
    """Round float64 values to the nearest bfloat16 (ties to even) via float32."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def param_layout():
    offs, off = [], 0
    for cin, cout, ks in LAYERS:
        offs.append(off)
        off += ks ** 3 * cin * cout
    boffs = []
    for cin, cout, ks in LAYERS:
        boffs.append(off)
        off += cout
    return offs, boffs, off


def unpack(params):
    offs, boffs, n = param_layout()
    p = np.asarray(params, dtype=np.float64)
    assert p.size == n
    Ws, bs = [], []
    for (cin, cout, ks), o, bo in zip(LAYERS, offs, boffs):
        Ws.append(p[o:o + ks ** 3 * cin * cout].reshape(ks ** 3, cout, cin))
        bs.append(p[bo:bo + cout])
    return Ws, bs


def _taps(ks):
    c = ks // 2
    return [(t // (ks * ks) - c, (t // ks) % ks - c, t % ks - c) for t in range(ks ** 3)]


def conv(x, W, b, ks):
    """x (D,H,W,Cin) -> (D,H,W,Cout), periodic padding."""
    out = np.zeros(x.shape[:3] + (W.shape[1],))
    for t, (dz, dy, dx) in enumerate(_taps(ks)):
        xs = np.roll(x, shift=(-dz, -dy, -dx), axis=(0, 1, 2))   # xs[p] = x[p + d]
        out += xs @ W[t].T
    return out + b


def conv_bwd(x, W, ks, dout):
    """Gradients of conv: (dx, dW, db)."""
    dW = np.zeros_like(W)
    dx = np.zeros(x.shape)
    for t, (dz, dy, dxx) in enumerate(_taps(ks)):
        xs = np.roll(x, shift=(-dz, -dy, -dxx), axis=(0, 1, 2))
        dW[t] = np.einsum("zyxo,zyxi->oi", dout, xs)
        dxs = dout @ W[t]                                          # grad wrt xs
        dx += np.roll(dxs, shift=(dz, dy, dxx), axis=(0, 1, 2))    # back to x's indexing
    db = dout.sum(axis=(0, 1, 2))
    return dx, dW, db


def pool(x):
    D, H, W, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(1, 3, 5))


def pool_bwd(d):
    return np.repeat(np.repeat(np.repeat(d, 2, 0), 2, 1), 2, 2) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def up_bwd(d):
    D, H, W, C = d.shape
    return d.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


def forward_backward(phase, target, params, emulate_bf16=False, need_grads=True):
    """Loss and (optionally) flat parameter gradients for one sample.

    phase: (n^3,) 0/1; target: (n^3, 36).  Returns (loss, grads or None, head (n^3, 64)).
    """
    rb = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    Ws, bs = unpack(params)
    Wr = [rb(W) for W in Ws]
    n = round(len(phase) ** (1 / 3))
    x0 = np.zeros((n, n, n, 32))
    x0[..., 0] = np.asarray(phase, dtype=np.float64).reshape(n, n, n)
    x0 = rb(x0)

    def lay(l, x, relu=True):
        y = conv(x, Wr[l], bs[l], LAYERS[l][2])
        return rb(np.maximum(y, 0.0)) if relu else y

    e1a = lay(E1A, x0)
    e1b = lay(E1B, e1a)
    p1 = rb(pool(e1b))
    e2a = lay(E2A, p1)
    e2b = lay(E2B, e2a)
    p2 = rb(pool(e2b))
    e3a = lay(E3A, p2)
    e3b = lay(E3B, e3a)
    cat2 = np.concatenate([up(e3b), e2b], axis=-1)
    d2a = lay(D2A, cat2)
    d2b = lay(D2B, d2a)
    cat1 = np.concatenate([up(d2b), e1b], axis=-1)
    d1a = lay(D1A, cat1)
    d1b = lay(D1B, d1a)
    y = lay(HEAD, d1b, relu=False)
    V = n ** 3
    T = np.asarray(target, dtype=np.float64).reshape(n, n, n, 36)
    diff = y[..., :36] - T
    loss = float(np.sum(diff ** 2) / (V * 36))
    if not need_grads:
        return loss, None, y.reshape(V, 64)
    gW = [None] * 11
    gb = [None] * 11
    dy = np.zeros_like(y)
    dy[..., :36] = 2.0 * diff / (V * 36)
    dy = rb(dy)

    def back(l, x, dpre, want_dx=True):
        dx, gW[l], gb[l] = conv_bwd(x, Wr[l], LAYERS[l][2], dpre)
        return rb(dx) if want_dx else None

    mask = lambda g, a: g * (a > 0)
    g_d1b = mask(back(HEAD, d1b, dy), d1b)
    g_d1a = mask(back(D1B, d1a, g_d1b), d1a)
    g_cat1 = back(D1A, cat1, g_d1a)
    g_d2b = mask(rb(up_bwd(g_cat1[..., :64])), d2b)
    g_d2a = mask(back(D2B, d2a, g_d2b), d2a)
    g_cat2 = back(D2A, cat2, g_d2a)
    g_e3b = mask(rb(up_bwd(g_cat2[..., :128])), e3b)
    g_e3a = mask(back(E3B, e3a, g_e3b), e3a)
    g_p2 = back(E3A, p2, g_e3a)
    g_e2b = mask(rb(g_cat2[..., 128:] + pool_bwd(g_p2)), e2b)
    g_e2a = mask(back(E2B, e2a, g_e2b), e2a)
    g_p1 = back(E2A, p1, g_e2a)
    g_e1b = mask(rb(g_cat1[..., 64:] + pool_bwd(g_p1)), e1b)
    g_e1a = mask(back(E1B, e1a, g_e1b), e1a)
    back(E1A, x0, g_e1a, want_dx=False)
    grads = np.concatenate([g.reshape(-1) for g in gW] + [g for g in gb])
    return loss, grads, y.reshape(V, 64)
