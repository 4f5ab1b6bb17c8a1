"""Pins of the learned-initialiser network's CPU reference (oracle.cnn):
direct-sum convolutions and gradients, a centre-tap kernel, the residual
identity of an untrained network and central finite differences."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import synth
from oracle import cnn


def test_conv_matches_direct_sum():
    rng = synth.SplitMix64(101)
    a = rng.uniform(2 * 3 * 5 * 6).reshape(2, 3, 5, 6) - 0.5
    w = rng.uniform(4 * 3 * 9).reshape(4, 3, 3, 3) - 0.5
    b = rng.uniform(4) - 0.5
    got = F.conv2d(torch.from_numpy(a), torch.from_numpy(w), torch.from_numpy(b), padding=1).numpy()
    assert np.allclose(got, cnn.conv3x3_loops(a, w, b), rtol=1e-12, atol=1e-12)


def test_conv_gradients_match_direct_sums():
    rng = synth.SplitMix64(102)
    a = rng.uniform(2 * 3 * 4 * 5).reshape(2, 3, 4, 5) - 0.5
    w = rng.uniform(4 * 3 * 9).reshape(4, 3, 3, 3) - 0.5
    g = rng.uniform(2 * 4 * 4 * 5).reshape(2, 4, 4, 5) - 0.5
    dw_ref, da_ref = cnn.conv3x3_grads_loops(a, w, g)
    dw = torch.nn.grad.conv2d_weight(torch.from_numpy(a), w.shape, torch.from_numpy(g), padding=1).numpy()
    da = torch.nn.grad.conv2d_input(a.shape, torch.from_numpy(w), torch.from_numpy(g), padding=1).numpy()
    assert np.allclose(dw, dw_ref, rtol=1e-12, atol=1e-12)
    assert np.allclose(da, da_ref, rtol=1e-12, atol=1e-12)


def test_centre_tap_kernel_and_untrained_residual():
    # a network whose hidden layers pass channel 1 through (centre tap,
    # identity across channels) and whose last layer reads it with weight
    # -1/2: z = -s1 x1 / 2, y = x1 + z / s1 = x1 / 2 for x1 >= 0
    L, C, s0, s1 = 3, 8, 0.5, 2.0
    shapes = cnn.layer_shapes(L, C)
    parts = []
    for l, (ci, co) in enumerate(shapes):
        w = np.zeros((co, 3, 3, ci))
        if l < L - 1:
            for o in range(min(ci, co)):
                w[o, 1, 1, o] = 1.0
        else:
            w[0, 1, 1, 1] = -0.5
        parts += [w.reshape(-1), np.zeros(co)]
    params = np.concatenate(parts)
    rng = synth.SplitMix64(103)
    x = rng.uniform(3 * 2 * 6 * 7).reshape(3, 2, 6, 7)
    y, _ = cnn.forward(params, x, L, C, s0, s1, bf16=False)
    assert np.allclose(y, x[:, 1] / 2.0, rtol=1e-14, atol=1e-14)
    # zero last layer: the network returns its residual input
    p0 = synth.cnninit.he_init(L, C, seed=5)
    y0, _ = cnn.forward(p0, x, L, C, s0, s1, bf16=False)
    assert np.array_equal(y0, x[:, 1])


@pytest.mark.parametrize("bf16", [False])
def test_backward_matches_central_differences(bf16):
    L, C, s0, s1 = 3, 8, 0.7, 1.3
    rng = synth.SplitMix64(104)
    params = (rng.uniform(synth.cnninit.param_count(L, C)) - 0.5) * 0.6
    x = rng.uniform(2 * 2 * 5 * 6).reshape(2, 2, 5, 6)
    t = rng.uniform(2 * 5 * 6).reshape(2, 5, 6)
    loss, grad = cnn.loss_grad(params, x, t, L, C, s0, s1, bf16=bf16)
    idx = (np.arange(40) * 7919) % params.size
    h = 1e-6
    fd = []
    for i in idx:
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        lp, _ = cnn.loss_grad(pp, x, t, L, C, s0, s1, bf16=bf16)
        lm, _ = cnn.loss_grad(pm, x, t, L, C, s0, s1, bf16=bf16)
        fd.append((lp - lm) / (2 * h))
    fd = np.array(fd)
    assert np.abs(grad[idx] - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())
    assert np.abs(fd).max() > 1e-3       # the sampled parameters matter


def test_rounding_model_matches_its_closed_form_on_one_layer():
    # One convolution from two input channels, z = conv(a, w) + b, with the
    # inputs a and the weights w stored.  To first order in u,
    # dz_p = sum_{c,k} w_ck a_{c,p+k} (d_w,ck + d_a,c,p+k), and every d in
    # that sum is a different independent U[-u, u] variable (variance
    # u^2 / 3), so E|dz|^2 = 2 (u^2 / 3) sum_p sum_{c,k} (w_ck a_{c,p+k})^2,
    # i.e. conv(a^2, w^2) summed.  The model's RMS over many draws must
    # reproduce it; perturbing only one of the two stores, or a variance
    # other than u^2 / 3, would miss it by a factor of sqrt(2) or more.
    L, C, s0, s1 = 1, 4, 0.8, 1.7
    rng = synth.SplitMix64(105)
    params = rng.uniform(synth.cnninit.param_count(L, C)) - 0.5
    x = rng.uniform(3 * 2 * 9 * 11).reshape(3, 2, 9, 11)
    t = rng.uniform(3 * 9 * 11).reshape(3, 9, 11)
    (w, b), = cnn.unpack(params, L, C)
    xt = torch.from_numpy(x)
    a = torch.stack([s0 * xt[:, 0], s1 * xt[:, 1]], dim=1)
    z = F.conv2d(a, w, b, padding=1)
    e2 = 2.0 * cnn.U_BF16 ** 2 / 3.0 * float(F.conv2d(a * a, w * w, padding=1).sum())
    want = np.sqrt(e2) / float(z.norm())
    got = cnn.rounding_model(params, x, t, L, C, s0, s1, draws=400, seed=3)["out"]
    assert abs(got / want - 1.0) < 0.05, (got, want)
