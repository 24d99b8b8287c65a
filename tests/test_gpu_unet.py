"""GPU parity of the U-Net warm start kernels (MFMA bf16) against the reference
network (oracle/unet.py, float64 with bf16 rounding at the points where the GPU
stores bf16).

Tolerance: relative L2 error 2e-2 on the head output, the loss and every
layer's weight and bias gradient.  Both sides round the same stored values to
bf16, but the GPU accumulates in float32 in another order, so a value near a
rounding boundary can round the other way (one bf16 ulp, 2^-8 relative), and
such flips propagate; 2e-2 is a few ulps of bf16.
"""
import numpy as np
import pytest

import lsh_inputs as li
from oracle import unet

pytestmark = pytest.mark.gpu
TOL = 2e-2


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def sample(seed, n):
    rng = np.random.Generator(np.random.PCG64(seed))
    c, r = li.rsa_spheres(seed, 1.0 / n, 0.3, rmin=1.5, rmax=3.0)
    phase = li.spheres_phase_grid(n, c, r)
    target = (rng.standard_normal((n ** 3, 36)) * 0.05 + 0.1 * phase[:, None]).astype(np.float32)
    params = li.unet_init_params(seed + 1, unet.LAYERS)
    _, boffs, _ = unet.param_layout()
    params[boffs[0]:] = (rng.standard_normal(params.size - boffs[0]) * 0.05).astype(np.float32)
    return phase, target, params


def to_dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("n", [8, 16])
def test_forward_and_gradients_match_oracle(lib, n):
    import torch
    phase, target, params = sample(100 + n, n)
    net = lib.UNet(params)
    print(f"unet parity n={n}", flush=True)
    net.zero_grad()
    loss = net.train_step(to_dev(phase, torch.uint8), to_dev(target, torch.float32), n, 0.0)
    head = net.head(n).cpu().numpy()
    g = net.grads()
    oloss, og, ohead = unet.forward_backward(phase, target, params, emulate_bf16=True)
    assert rel(head, ohead) < TOL
    assert abs(loss - oloss) / oloss < TOL
    offs, boffs, _ = unet.param_layout()
    for l, (cin, cout, ks) in enumerate(unet.LAYERS):
        sw = slice(offs[l], offs[l] + ks ** 3 * cin * cout)
        sb = slice(boffs[l], boffs[l] + cout)
        assert rel(g[sw], og[sw]) < TOL, (l, rel(g[sw], og[sw]))
        assert rel(g[sb], og[sb]) < TOL, (l, rel(g[sb], og[sb]))
    # the parameters themselves are untouched by lr = 0
    np.testing.assert_array_equal(net.params(), params)


def test_gradients_accumulate_until_cleared(lib):
    import torch
    n = 8
    phase, target, params = sample(7, n)
    net = lib.UNet(params)
    ph, tg = to_dev(phase, torch.uint8), to_dev(target, torch.float32)
    net.zero_grad()
    net.train_step(ph, tg, n, 0.0)
    g1 = net.grads()
    net.train_step(ph, tg, n, 0.0)
    g2 = net.grads()
    assert rel(g2, 2 * g1) < 1e-5
    net.zero_grad()
    net.train_step(ph, tg, n, 0.0)
    assert rel(net.grads(), g1) < 1e-5


def test_adam_training_lowers_the_loss(lib):
    import torch
    n = 16
    phase, target, params = sample(21, n)
    net = lib.UNet(params)
    ph, tg = to_dev(phase, torch.uint8), to_dev(target, torch.float32)
    losses = [net.train_step(ph, tg, n, 1e-3) for _ in range(60)]
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0], losses[::10]
    # Adam's first step moves each weight by about lr against its gradient's sign
    net2 = lib.UNet(params)
    net2.zero_grad()
    net2.train_step(ph, tg, n, 0.0)
    g = net2.grads()
    net2.zero_grad()
    net2.train_step(ph, tg, n, 1e-3)
    dp = net2.params() - params
    big = np.abs(g) > 1e-5          # Adam's eps (1e-8) is then below 1e-3 of |g|
    assert big.sum() > 1000
    np.testing.assert_allclose(dp[big], -1e-3 * np.sign(g[big]), rtol=2e-3, atol=1e-6)


@pytest.mark.parametrize("n", [16, 32])
def test_predict_contracts_unit_load_channels(lib, n):
    """lsh_unet_predict forms the head (1x1 convolution) and its contraction
    with the loads in one kernel and stores no head.  Its output equals the
    contraction of the head that a training step's forward pass stores (the
    same convolution sums, FP64 contraction) at 1e-12, and at 16^3 that head is
    the oracle network's."""
    import torch
    phase, target, params = sample(33, n)
    net = lib.UNet(params)
    ph = to_dev(phase, torch.uint8)
    rng = np.random.Generator(np.random.PCG64(3))
    eps = np.vstack([np.eye(6), rng.standard_normal((3, 6))])
    print(f"unet predict n={n}", flush=True)
    E = net.predict(ph, n, eps).cpu().numpy()            # (9, 6, V)
    with pytest.raises(lib.LshError):
        net.head(n)                                       # a prediction leaves no head behind
    net.train_step(ph, to_dev(np.zeros((n ** 3, 36)), torch.float32), n, 0.0)
    y = net.head(n).cpu().numpy().astype(np.float64)      # (V, 64)
    fields = y[:, :36].reshape(-1, 6, 6)                  # [p][load j][Mandel c]
    scale = np.array([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])
    ref = np.einsum("lj,pjc->lcp", eps, fields) * scale[None, :, None]
    np.testing.assert_allclose(E, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    if n == 16:
        # the prediction is the forward pass of the oracle network
        _, _, ohead = unet.forward_backward(phase, np.zeros((n ** 3, 36)), params, emulate_bf16=True,
                                            need_grads=False)
        assert rel(y, ohead) < TOL


def test_pack_target_voigt_to_mandel(lib):
    import torch
    n = 8
    V = n ** 3
    rng = np.random.Generator(np.random.PCG64(4))
    E6 = rng.standard_normal((6, 6, V))
    T = lib.UNet.pack_target(to_dev(E6, torch.float64), n).cpu().numpy()
    scale = np.array([1, 1, 1, 1 / np.sqrt(2), 1 / np.sqrt(2), 1 / np.sqrt(2)])
    ref = (E6 * scale[None, :, None]).transpose(2, 0, 1).reshape(V, 36)
    np.testing.assert_allclose(T, ref.astype(np.float32), rtol=1e-7, atol=0)


def test_workspace_too_small_is_rejected(lib):
    import ctypes
    import torch
    n = 8
    phase, target, params = sample(5, n)
    net = lib.UNet(params)
    nb = ctypes.c_size_t()
    assert lib._lib.lsh_unet_act_bytes(net._h, n, 1, ctypes.byref(nb)) == 0
    small = torch.empty(nb.value // 2, dtype=torch.uint8, device="cuda")
    ph, tg = to_dev(phase, torch.uint8), to_dev(target, torch.float32)
    loss = ctypes.c_double()
    rc = lib._lib.lsh_unet_train_step(net._h, ctypes.c_void_p(ph.data_ptr()), ctypes.c_void_p(tg.data_ptr()), n,
                                      0.0, ctypes.c_void_p(small.data_ptr()), small.numel(), None, ctypes.byref(loss))
    assert lib.STATUS.get(rc) == "LSH_EWORKSPACE"
