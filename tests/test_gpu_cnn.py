"""GPU tests of the learned-initialiser network (include/vam_cnn.h): MFMA
forward, loss and gradients against the plain FP64 CPU network, within a
bound that the reference's BF16 error model sets before the GPU runs;
determinism, the Adam update, and learning a fixed filter."""
import sys

import numpy as np
import pytest

import synth
from oracle import cnn as ocnn

torch = pytest.importorskip("torch")
import paper_2211_03516_amd as vam

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relL2(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300))


def _setup(L, C, H, W, n, seed, s0=0.05, s1=2.0):
    rng = synth.SplitMix64(seed)
    p = synth.cnninit.he_init(L, C, seed=seed, zero_last=False)
    x = rng.uniform(n * 2 * H * W).reshape(n, 2, H, W) * np.array([20.0, 0.5]).reshape(1, 2, 1, 1)
    t = x[:, 1] + 0.3 * (rng.uniform(n * H * W).reshape(n, H, W) - 0.5)
    return p, x, t, (s0, s1)


# Bound on the GPU's deviation from the plain FP64 network: LAMBDA times the
# root-mean-square error that the BF16 error model of oracle.cnn predicts
# for this network and input (independent relative errors, uniform on
# [-2^-8, 2^-8], at every value the library stores in BF16).  An error that
# is a sum of many such independent terms exceeds three times its RMS with
# small probability; the model is computed on the CPU from the FP64
# network alone.
LAMBDA = 3.0


@pytest.mark.parametrize("L,C,H,W,n", [(6, 64, 24, 40, 3), (3, 16, 17, 15, 32), (2, 8, 8, 4, 1)])
def test_cnn_matches_oracle(L, C, H, W, n):
    p, x, t, (s0, s1) = _setup(L, C, H, W, n, seed=L * 100 + C)
    p64 = p.astype(np.float64)
    xf, tf = x.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64)
    model = ocnn.rounding_model(p64, xf, tf, L, C, s0, s1, draws=8, seed=L * 100 + C)
    say("cnn L %d C %d %dx%d n %d; BF16 error model: out %.2e loss %.2e grads %s"
        % (L, C, H, W, n, model["out"], model["loss"], np.array2string(model["grads"], precision=2)))
    net = vam.Cnn(L, C, H, W, max_batch=n, in_scale=(s0, s1))
    net.set_params(p)
    assert np.array_equal(net.get_params(), p)
    xd = torch.from_numpy(x).float().to(DEV)
    td = torch.from_numpy(t).float().to(DEV)
    y = net.forward(xd).cpu().numpy()
    loss = net.loss_grad(xd, td)
    g = net.grads().astype(np.float64)
    # the plain FP64 network; compare the network's own contribution
    # z / s1 = y - x1
    y_ref, _ = ocnn.forward(p64, xf, L, C, s0, s1)
    loss_ref, g_ref = ocnn.loss_grad(p64, xf, tf, L, C, s0, s1)
    e_y = relL2(y - xf[:, 1], y_ref - xf[:, 1])
    e_l = abs(loss - loss_ref) / loss_ref
    e_g = np.array([relL2(g[s], g_ref[s]) for s in ocnn.layer_slices(L, C)])
    # diagnostic only: the same network with BF16 rounding emulated at the
    # storage points
    y_em, _ = ocnn.forward(p64, xf, L, C, s0, s1, bf16=True)
    _, g_em = ocnn.loss_grad(p64, xf, tf, L, C, s0, s1, bf16=True)
    say("  vs FP64: out %.2e loss %.2e grads %s; vs BF16 emulation: out %.2e grads %.2e"
        % (e_y, e_l, np.array2string(e_g, precision=2), relL2(y - xf[:, 1], y_em - xf[:, 1]),
           relL2(g, g_em)))
    assert e_y <= LAMBDA * model["out"]
    assert e_l <= LAMBDA * model["loss"]
    assert np.all(e_g <= LAMBDA * model["grads"])
    net.close()


def test_cnn_deterministic_and_adam():
    L, C, H, W, n = 4, 32, 16, 16, 4
    p, x, t, sc = _setup(L, C, H, W, n, seed=9)
    net = vam.Cnn(L, C, H, W, max_batch=n, in_scale=sc)
    net.set_params(p)
    xd = torch.from_numpy(x).float().to(DEV)
    td = torch.from_numpy(t).float().to(DEV)
    l1 = net.loss_grad(xd, td)
    g1 = net.grads()
    l2 = net.loss_grad(xd, td)
    g2 = net.grads()
    assert l1 == l2 and np.array_equal(g1, g2)
    # two Adam steps against the update written out in FP64
    b1, b2, eps, lr = 0.9, 0.999, 1e-8, 1e-3
    w = p.astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for step in (1, 2):
        net.loss_grad(xd, td, want_loss=False)
        g = net.grads().astype(np.float64)
        net.adam_step(lr, b1, b2, eps)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        w = w - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
        got = net.get_params().astype(np.float64)
        assert np.abs(got - w).max() <= 1e-6 * max(1.0, np.abs(w).max())
    net.close()


def test_cnn_learns_a_fixed_filter():
    # target: x1 plus a 3x3 box blur of x0 / 40 -- within reach of one layer
    L, C, H, W, n = 3, 16, 32, 32, 8
    rng = synth.SplitMix64(77)
    x = rng.uniform(n * 2 * H * W).reshape(n, 2, H, W)
    x0 = torch.from_numpy(x[:, :1])
    blur = torch.nn.functional.conv2d(x0, torch.full((1, 1, 3, 3), 1.0 / 9, dtype=torch.float64), padding=1)
    t = x[:, 1] + blur[:, 0].numpy() / 40.0
    net = vam.Cnn(L, C, H, W, max_batch=n, in_scale=(1.0, 1.0))
    net.set_params(synth.cnninit.he_init(L, C, seed=3))
    xd = torch.from_numpy(x).float().to(DEV)
    td = torch.from_numpy(t).float().to(DEV)
    first = net.loss_grad(xd, td)
    for it in range(300):
        net.adam_step(3e-3)
        last = net.loss_grad(xd, td)
    say("fixed filter: loss %.3e -> %.3e" % (first, last))
    assert last < first / 20
    net.close()
