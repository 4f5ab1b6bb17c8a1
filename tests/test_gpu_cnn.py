"""GPU tests of the learned-initialiser network (include/vam_cnn.h): MFMA
forward, loss and gradients against the CPU reference with the same BF16
rounding points, determinism, the Adam update, and learning a fixed filter."""
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


@pytest.mark.parametrize("L,C,H,W,n", [(6, 64, 24, 40, 3), (3, 16, 17, 15, 32), (2, 8, 8, 4, 1)])
def test_cnn_matches_oracle(L, C, H, W, n):
    p, x, t, (s0, s1) = _setup(L, C, H, W, n, seed=L * 100 + C)
    say("cnn L %d C %d %dx%d n %d" % (L, C, H, W, n))
    net = vam.Cnn(L, C, H, W, max_batch=n, in_scale=(s0, s1))
    net.set_params(p)
    assert np.array_equal(net.get_params(), p)
    p64 = p.astype(np.float64)
    xd = torch.from_numpy(x).float().to(DEV)
    td = torch.from_numpy(t).float().to(DEV)
    xf, tf = x.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64)
    y = net.forward(xd).cpu().numpy()
    y_ref, _ = ocnn.forward(p64, xf, L, C, s0, s1, bf16=True)
    # compare the network's own contribution z / s1 = y - x1
    e_y = relL2(y - xf[:, 1], y_ref - xf[:, 1])
    loss = net.loss_grad(xd, td)
    g = net.grads().astype(np.float64)
    loss_ref, g_ref = ocnn.loss_grad(p64, xf, tf, L, C, s0, s1, bf16=True)
    e_l = abs(loss - loss_ref) / loss_ref
    e_g = relL2(g, g_ref)
    # per layer
    off, worst = 0, 0.0
    for ci, co in ocnn.layer_shapes(L, C):
        k = co * 9 * ci + co
        worst = max(worst, relL2(g[off:off + k], g_ref[off:off + k]))
        off += k
    _, g_exact = ocnn.loss_grad(p64, xf, tf, L, C, s0, s1, bf16=False)
    say("  forward %.2e  loss %.2e  grads %.2e (worst layer %.2e); BF16 storage vs FP64: grads %.2e"
        % (e_y, e_l, e_g, worst, relL2(g, g_exact)))
    # Bound: both sides round to BF16 at the same points, but FP32 (GPU) and
    # FP64 (reference) sums differ by ~1e-6 relative, which moves a fraction
    # ~2e-6 / 2^-7 ~ 3e-4 of the stored values across a BF16 rounding
    # boundary; each such flip is one BF16 ulp (2^-7 relative), ~1.5e-4
    # rel-L2 per layer, compounding over up to six layers.
    assert e_y <= 3e-3 and e_l <= 1e-4 and worst <= 3e-3
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
