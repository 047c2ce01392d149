"""GPU parity of the MLP cost model's training and inference kernels against the
FP64 CPU oracle (same initial parameters, same data, same step order).
Tolerance: FP32 against FP64, relative 1e-4 for losses and gradients."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1706_10086_amd as mg  # noqa: E402
from oracle import mlp as omlp  # noqa: E402


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mg.lib()
    return torch.device("cuda:0")


def problem(I, H, O, B, seed):
    theta = mlp_init = omlp.he_uniform_init(I, H, O, seed)
    theta = (mlp_init + 0.05 * synth.uniform_pm1(mlp_init.shape, seed + 5)).astype(np.float32)
    X = synth.uniform_pm1((B, I), seed + 1).astype(np.float32)
    T = (0.5 + 0.5 * synth.uniform_pm1((B, O), seed + 2)).astype(np.float32)
    M = (synth.unit(seed + 3, B * O) < 0.6).astype(np.float32).reshape(B, O)
    return theta, X, T, M


def to_dev(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


@pytest.mark.parametrize("I,H,O,B", [(6, 5, 4, 7), (6, 64, 19, 300), (6, 64, 19, 3000), (6, 8, 70, 130),
                                     (6, 64, 250, 6000), (3, 100, 129, 1000)])
def test_loss_and_gradient_match_oracle(dev, I, H, O, B):
    say(f"mlp grad I={I} H={H} O={O} B={B}")
    theta, X, T, M = problem(I, H, O, B, 10 + B)
    net = mg.MLP(I, H, O, theta)
    net.set_data(to_dev(X, dev), to_dev(T, dev), to_dev(M, dev))
    L, g = net.loss_grad()
    Lr, gr = omlp.loss_and_grad(theta.astype(np.float64), X, T, M, I, H, O)
    say(f"  loss gpu {L:.7g} oracle {Lr:.7g}")
    assert abs(L - Lr) <= 1e-4 * abs(Lr)
    assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr)
    assert np.all(np.abs(g - gr) <= 1e-4 * np.abs(gr).max() + 1e-6)
    net.destroy()


def test_adam_steps_track_the_oracle(dev):
    I, H, O, B = 6, 64, 19, 500
    say("mlp adam 20 steps vs oracle")
    theta, X, T, M = problem(I, H, O, B, 77)
    net = mg.MLP(I, H, O, theta)
    net.set_data(to_dev(X, dev), to_dev(T, dev), to_dev(M, dev))
    net.train(20, lr=1e-3)
    got = net.get_params().astype(np.float64)
    th = theta.astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for t in range(1, 21):
        _, g = omlp.loss_and_grad(th, X, T, M, I, H, O)
        th, m, v = omlp.adam_step(th, g, m, v, t, lr=1e-3)
    moved = np.linalg.norm(th - theta)
    say(f"  param distance {np.linalg.norm(got - th):.3e} (moved {moved:.3e})")
    assert np.linalg.norm(got - th) <= 2e-3 * moved
    net.destroy()


def test_training_reduces_loss_and_is_deterministic(dev):
    I, H, O, B = 6, 64, 19, 2000
    say("mlp training determinism")
    theta, X, T, M = problem(I, H, O, B, 91)
    outs = []
    for _ in range(2):
        net = mg.MLP(I, H, O, theta)
        net.set_data(to_dev(X, dev), to_dev(T, dev), to_dev(M, dev))
        L0, _ = net.loss_grad()
        L = net.train(300, lr=3e-3)
        outs.append(net.get_params())
        net.destroy()
        assert L < 0.5 * L0
    assert np.array_equal(outs[0], outs[1])


def test_forward_and_masked_argmax(dev):
    I, H, O, B = 6, 64, 19, 1000
    say("mlp forward / predict")
    theta, X, T, M = problem(I, H, O, B, 5)
    M[7] = 0.0           # a row with no allowed output
    net = mg.MLP(I, H, O, theta)
    Y = net.forward(to_dev(X, dev)).cpu().numpy()
    Yr, _ = omlp.forward(theta.astype(np.float64), X, I, H, O)
    assert np.max(np.abs(Y - Yr)) <= 1e-5 * (np.max(np.abs(Yr)) + 1)
    idx = net.predict(to_dev(X, dev), to_dev(M, dev)).cpu().numpy()
    assert idx[7] == -1
    ref = omlp.masked_argmax(Y.astype(np.float64), M)
    assert np.array_equal(idx, ref)
    # against the FP64 network: the chosen output is within rounding of the best
    for r in range(B):
        if r == 7:
            continue
        allowed = M[r] != 0
        assert allowed[idx[r]]
        assert Yr[r, idx[r]] >= Yr[r][allowed].max() - 1e-5
    net.destroy()
