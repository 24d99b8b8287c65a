"""Pins for the reference U-Net (oracle/unet.py), independent of its own code.

* convolution: single-channel slices against scipy.ndimage.correlate with
  periodic ('wrap') boundaries, and the delta-weight / constant-field cases;
* pooling and upsampling: closed forms (mean preservation, adjointness);
* backward pass: central finite differences of the loss in float64;
* bf16 rounding: exactly representable values, ties to even.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

from lsh_inputs import unet_init_params
from oracle import unet


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def test_conv_matches_scipy_wrap_correlation():
    rng = _rng(1)
    n, cin, cout = 5, 3, 2
    x = rng.standard_normal((n, n, n, cin))
    W = rng.standard_normal((27, cout, cin))
    b = rng.standard_normal(cout)
    out = unet.conv(x, W, b, 3)
    for co in range(cout):
        ref = np.full((n, n, n), b[co])
        for ci in range(cin):
            # kernel k[dz+1, dy+1, dx+1] = W[t][co][ci]; correlate: out[p] = sum_j k[j] x[p + j - 1]
            k = W[:, co, ci].reshape(3, 3, 3)
            ref += ndi.correlate(x[..., ci], k, mode="wrap")
        np.testing.assert_allclose(out[..., co], ref, rtol=1e-12, atol=1e-12)


def test_conv_delta_weight_is_a_shift_and_constant_field():
    rng = _rng(2)
    n = 4
    x = rng.standard_normal((n, n, n, 1))
    for t, (dz, dy, dx) in enumerate([(-1, 0, 1), (1, 1, -1), (0, -1, 0)]):
        W = np.zeros((27, 1, 1))
        W[9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)] = 1.0
        out = unet.conv(x, W, np.zeros(1), 3)
        for z in range(n):
            for y in range(n):
                for xx in range(n):
                    assert out[z, y, xx, 0] == x[(z + dz) % n, (y + dy) % n, (xx + dx) % n, 0]
    W = rng.standard_normal((27, 2, 3))
    c = np.ones((n, n, n, 3)) * np.array([1.0, -2.0, 0.5])
    out = unet.conv(c, W, np.zeros(2), 3)
    np.testing.assert_allclose(out, np.broadcast_to(W.sum(axis=0) @ np.array([1.0, -2.0, 0.5]), out.shape),
                               rtol=1e-12)


def test_pool_up_closed_forms():
    rng = _rng(3)
    x = rng.standard_normal((4, 4, 4, 2))
    p = unet.pool(x)
    assert p.shape == (2, 2, 2, 2)
    np.testing.assert_allclose(p[1, 0, 1], x[2:4, 0:2, 2:4].mean(axis=(0, 1, 2)))
    np.testing.assert_allclose(p.mean(axis=(0, 1, 2)), x.mean(axis=(0, 1, 2)))
    u = unet.up(p)
    np.testing.assert_array_equal(u[3, 1, 2], p[1, 0, 1])
    # adjointness <up(a), b> = <a, up_bwd(b)>, <pool(a), b> = <a, pool_bwd(b)>
    a = rng.standard_normal((2, 2, 2, 2))
    bb = rng.standard_normal((4, 4, 4, 2))
    assert np.isclose(np.sum(unet.up(a) * bb), np.sum(a * unet.up_bwd(bb)))
    assert np.isclose(np.sum(unet.pool(bb) * a), np.sum(bb * unet.pool_bwd(a)))


def test_bf16_rounding():
    v = np.array([1.0, -2.5, 0.0, 3.0 * 2.0 ** -10])
    np.testing.assert_array_equal(unet.bf16(v), v)
    one = 1.0
    ulp = 2.0 ** -7
    # halfway cases round to even mantissa
    assert unet.bf16(one + ulp / 2) == one
    assert unet.bf16(one + 3 * ulp / 2) == one + 2 * ulp
    assert unet.bf16(one + ulp / 2 + 2.0 ** -20) == one + ulp
    x = _rng(4).standard_normal(1000)
    r = unet.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 * (1 + 1e-12))


def test_param_layout_matches_layer_table():
    offs, boffs, n = unet.param_layout()
    assert n == sum(ks ** 3 * ci * co + co for ci, co, ks in unet.LAYERS)
    p = unet_init_params(5, unet.LAYERS)
    assert p.size == n and p.dtype == np.float32
    assert np.all(p[boffs[0]:] == 0.0)


@pytest.fixture(scope="module")
def small_problem():
    rng = _rng(7)
    n = 8
    phase = (rng.random(n ** 3) < 0.3).astype(np.uint8)
    target = rng.standard_normal((n ** 3, 36)) * 0.1
    # a non-trivial bias keeps ReLUs away from exact zeros of the zero-bias init
    params = unet_init_params(11, unet.LAYERS).astype(np.float64)
    _, boffs, _ = unet.param_layout()
    params[boffs[0]:] = rng.standard_normal(params.size - boffs[0]) * 0.05
    return phase, target, params


def test_backward_matches_finite_differences(small_problem):
    phase, target, params = small_problem
    loss, g, _ = unet.forward_backward(phase, target, params)
    offs, boffs, _ = unet.param_layout()
    rng = _rng(8)
    picks = []
    for l, (cin, cout, ks) in enumerate(unet.LAYERS):
        picks += list(offs[l] + rng.integers(0, ks ** 3 * cin * cout, 2))
        picks.append(boffs[l] + int(rng.integers(0, cout)))
    h = 1e-5
    for i in picks:
        pp = params.copy()
        pp[i] += h
        lp = unet.forward_backward(phase, target, pp, need_grads=False)[0]
        pp[i] -= 2 * h
        lm = unet.forward_backward(phase, target, pp, need_grads=False)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-9 + 1e-4 * abs(g[i]), (i, fd, g[i])
    assert loss > 0


def test_input_gradient_direction(small_problem):
    """A small step against the gradient lowers the loss (first-order descent)."""
    phase, target, params = small_problem
    loss, g, _ = unet.forward_backward(phase, target, params)
    step = 1e-5 / np.linalg.norm(g)
    l2 = unet.forward_backward(phase, target, params - step * g, need_grads=False)[0]
    assert l2 < loss
    assert np.isclose(loss - l2, step * np.dot(g, g), rtol=1e-2)
