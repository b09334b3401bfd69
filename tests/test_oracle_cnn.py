"""Pins for the oracle of the learned stage's CNN: the convolution against
PyTorch's CPU conv2d with circular padding (a library routine), gradients
against central finite differences, and Adam's first step against its
closed form (a step of lr along -sign(g))."""
import numpy as np
import pytest

from oracle import cnn


def test_conv_matches_torch_circular_conv2d():
    torch = pytest.importorskip("torch")
    F = torch.nn.functional
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 9, 7))
    w = rng.standard_normal((4, 3, 3, 3))
    xt = F.pad(torch.from_numpy(x), (1, 1, 1, 1), mode="circular")
    ref = F.conv2d(xt, torch.from_numpy(w)).numpy()
    np.testing.assert_allclose(cnn.conv_forward(x, w), ref, atol=1e-12)


def fd_check(fun, x, grad, eps=1e-6, samples=12, seed=1):
    rng = np.random.default_rng(seed)
    for _ in range(samples):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp = x.copy(); xp[idx] += eps
        xm = x.copy(); xm[idx] -= eps
        fd = (fun(xp) - fun(xm)) / (2 * eps)
        assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, grad[idx])


def test_conv_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 3, 6, 5))
    w = rng.standard_normal((4, 3, 3, 3))
    gy = rng.standard_normal((2, 4, 6, 5))
    f_x = lambda xx: float(np.sum(cnn.conv_forward(xx, w) * gy))
    f_w = lambda ww: float(np.sum(cnn.conv_forward(x, ww) * gy))
    fd_check(f_x, x, cnn.conv_backward_data(gy, w))
    fd_check(f_w, w, cnn.conv_backward_weight(gy, x))


def test_network_gradient_matches_finite_differences():
    ws = cnn.init_weights(3, channels=(2, 4, 4, 2))
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 2, 8, 8))
    t = rng.standard_normal((2, 2, 8, 8))

    def L(ws_):
        y, _, _ = cnn.forward(ws_, x)
        return cnn.loss(y, t)

    y, acts, pre = cnn.forward(ws, x)
    grads = cnn.backward(ws, acts, pre, cnn.loss_grad(y, t))
    for li in range(len(ws)):
        def f(wl, li=li):
            w2 = list(ws); w2[li] = wl
            return L(w2)
        fd_check(f, ws[li], grads[li], samples=6, seed=li)


def test_adam_first_step_is_lr_sign_step():
    w = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -4.0, 1e-3])]
    opt = cnn.Adam([(3,)], lr=1e-2)
    out = opt.step(w, g)[0]
    np.testing.assert_allclose(out, w[0] - 1e-2 * np.sign(g[0]), rtol=0, atol=1e-7)


def test_channel_packing_round_trip():
    rng = np.random.default_rng(5)
    v = rng.standard_normal((3, 4, 4)) + 1j * rng.standard_normal((3, 4, 4))
    np.testing.assert_array_equal(cnn.from_channels(cnn.to_channels(v)), v)
