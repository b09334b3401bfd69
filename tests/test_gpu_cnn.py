"""The learned-stage network on the GPU against the FP64 oracle (oracle/cnn.py).

Forward output, loss and every weight gradient are compared per tensor.
fp32 path (fp32 storage and MFMA, FP32 accumulation): relative error <= 1e-5.
bf16 path: weights, activations and back-propagated gradients are rounded to
bf16 (unit roundoff u = 2^-9) once per layer and direction, products
accumulate in FP32.  The gradient of layer l of an L-layer network has passed
through 2 (L - l) - 1 such roundings (forward activations of layers >= l, the
loss gradient and the backward passes above l), so its tolerance is
4 (2 (L - l) - 1) u: 8.6e-2 for the first layer, 7.8e-3 for the last; the
forward output, which passes L roundings, and the loss get 4 L u = 4.7e-2.
The Adam step is checked against the oracle's Adam applied to the same
gradients, and training must fit a map a 3 x 3 network can represent.
"""
import numpy as np
import pytest

from oracle import cnn as ocnn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -9
L = len(ocnn.CHANNELS) - 1
TOL = {"f32": 1e-5, "bf16": 4 * L * U_BF16}


def grad_tol(dtype, layer):
    return 1e-5 if dtype == "f32" else 4 * (2 * (L - layer) - 1) * U_BF16


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def data():
    rng = np.random.default_rng(5)
    n, B = 32, 3
    x = rng.standard_normal((B, n, n)) + 1j * rng.standard_normal((B, n, n))
    t = rng.standard_normal((B, n, n)) + 1j * rng.standard_normal((B, n, n))
    ws = ocnn.init_weights(11)
    return n, x, t, ws


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_forward_matches_oracle(data, dtype):
    from paper_1409_0297_amd import CNN
    n, x, t, ws = data
    net = CNN(n, dtype=dtype, max_batch=4)
    net.set_weights(ws)
    y = net.forward(x).cpu().numpy().reshape(x.shape)
    net.close()
    yo, _, _ = ocnn.forward(ws, ocnn.to_channels(x))
    e = rel(y, ocnn.from_channels(yo))
    assert e <= TOL[dtype], (dtype, e)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_loss_and_gradients_match_oracle(data, dtype):
    from paper_1409_0297_amd import CNN
    n, x, t, ws = data
    net = CNN(n, dtype=dtype, max_batch=4)
    net.set_weights(ws)
    loss, grads = net.loss_grad(x, t, want_grads=True)
    net.close()
    X, T = ocnn.to_channels(x), ocnn.to_channels(t)
    yo, acts, pre = ocnn.forward(ws, X)
    lo = ocnn.loss(yo, T)
    go = ocnn.backward(ws, acts, pre, ocnn.loss_grad(yo, T))
    errs = [rel(g, r) for g, r in zip(grads, go)]
    print(dtype, "loss", loss, lo, "gradient errors", errs)
    assert abs(loss - lo) <= TOL[dtype] * lo, (loss, lo)
    for li, e in enumerate(errs):
        assert e <= grad_tol(dtype, li), (dtype, li, errs)


def test_adam_step_matches_oracle(data):
    from paper_1409_0297_amd import CNN
    n, x, t, ws = data
    net = CNN(n, dtype="f32", max_batch=4)
    net.set_weights(ws)
    opt = ocnn.Adam([w.shape for w in ws], lr=1e-3)
    cur = [w.astype(np.float32).astype(np.float64) for w in ws]
    for _ in range(3):
        _, g = net.loss_grad(x, t, want_grads=True)
        net.adam_step(1e-3)
        cur = opt.step(cur, [gi.astype(np.float64) for gi in g])
    got = net.get_weights()
    net.close()
    for a, b in zip(got, cur):
        assert rel(a, b) <= 1e-6


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_training_fits_a_representable_map(dtype):
    """Target = the input shifted by one grid step (a single tap of a 3 x 3
    filter, representable through ReLU pairs): Adam must cut the loss 10x."""
    from paper_1409_0297_amd import CNN
    rng = np.random.default_rng(9)
    n, B = 32, 8
    x = rng.standard_normal((B, n, n)) + 1j * rng.standard_normal((B, n, n))
    t = np.roll(x, 1, axis=2)
    net = CNN(n, dtype=dtype, max_batch=B)
    net.set_weights(ocnn.init_weights(3))
    first = net.loss_grad(x, t)
    for _ in range(300):
        net.loss_grad(x, t)
        net.adam_step(3e-3)
    last = net.loss_grad(x, t)
    net.close()
    assert last <= 0.1 * first, (dtype, first, last)


def test_learned_stage_trains_on_krylov_pairs_and_keeps_the_solution():
    """Train on (v_j, M v_j) pairs of a random-media family (n = 64,
    omega = 2 pi 8, 8 bumps), attach to solves of unseen media: every solve
    still converges to the plain solve's solution, the network lowers its
    training loss, and the acceptance counts add up.  The measured gain (accepted
    steps, preconditioner applications saved, time) is printed; on this family
    the network, which sees only v and not the medium, approximates P^{-1} Q
    poorly and saves at most a step per solve."""
    from paper_1409_0297_amd import CNN, learned
    V, Z = learned.training_pairs(64, 8, 8.0, 8, 0.05, range(100, 130))
    net = CNN(64, dtype="bf16", max_batch=16)
    net.set_weights(ocnn.init_weights(1))
    first = net.loss_grad(V[:16], Z[:16])
    hist = learned.train(net, V, Z, epochs=15, batch=16, lr=1e-3)
    assert hist[-1] < first, (first, hist)
    rows = learned.evaluate(net, 64, 8, 8.0, 8, 0.05, [500, 501], rho=0.9)
    net.close()
    for r in rows:
        print(r)
        assert r["code"] == 0 and r["relres"] <= 1e-10
        assert r["diff"] <= 1e-8
        assert r["iters_learned"] >= r["accepted"] and r["rejected"] >= 0
        assert r["precond_applies_learned"] == r["iters_learned"] - r["accepted"]
