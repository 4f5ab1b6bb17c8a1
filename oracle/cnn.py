"""Plain CPU reference of the learned-initialiser network (test
infrastructure: only tests, the smoke check and the benchmark's CPU leg use
it).

The network is not in the paper; it replaces the paper's filtered
parallel-beam starting point (Sec. 2.3) by a learned one.  Definition, per
image with inputs x0 (parallel-beam projection) and x1 (filtered start):
    a_0 = (s0 x0, s1 x1)
    a_l = relu(conv3x3(a_{l-1}, W_l) + b_l)      l = 1 .. L-1
    z   = conv3x3(a_{L-1}, W_L) + b_L            (one output channel)
    y   = x1 + z / s1
    loss = mean over pixels of (s1 y - s1 t)^2
conv3x3 is a cross-correlation with zero padding 1.  Everything is FP64
(torch CPU).  With bf16=True the values are rounded to bfloat16 (nearest
even) where the GPU library stores them in that format: the inputs a_0, the
weights, every hidden activation, the output gradient and every hidden
gradient.  The backward pass is written out layer by layer (weight and
input gradients of a convolution from torch's convolution-gradient
routines) so that those rounding points sit where the library has them.

Pins (tests): a brute-force loop convolution and its two gradients on tiny
inputs, a centre-tap kernel reproducing its input, and central finite
differences of the loss against this backward pass.
"""
import numpy as np
import torch
import torch.nn.functional as F



def layer_shapes(layers, channels):
    return [(2 if l == 0 else channels, 1 if l == layers - 1 else channels) for l in range(layers)]


def unpack(params, layers, channels):
    """[(W [c_out][c_in][3][3], b [c_out])] as FP64 tensors."""
    out, off = [], 0
    p = np.asarray(params, dtype=np.float64)
    for ci, co in layer_shapes(layers, channels):
        w = p[off:off + co * 9 * ci].reshape(co, 3, 3, ci)
        off += co * 9 * ci
        b = p[off:off + co]
        off += co
        out.append((torch.from_numpy(np.ascontiguousarray(w.transpose(0, 3, 1, 2))), torch.from_numpy(b.copy())))
    assert off == p.size
    return out


def pack(grads):
    """Flat array in the library's layout from [(dW [c_out][c_in][3][3], db)]."""
    parts = []
    for dw, db in grads:
        parts.append(dw.permute(0, 2, 3, 1).reshape(-1).numpy())
        parts.append(db.numpy())
    return np.concatenate(parts)


def _r(x, on):
    return x.to(torch.bfloat16).to(torch.float64) if on else x


def forward(params, x, layers, channels, s0, s1, bf16=True):
    """y [n][H][W] and the cache of the backward pass; x [n][2][H][W]."""
    P = unpack(params, layers, channels)
    x = torch.as_tensor(np.asarray(x, dtype=np.float64))
    a = _r(torch.stack([s0 * x[:, 0], s1 * x[:, 1]], dim=1), bf16)
    acts = [a]
    z = None
    for l, (w, b) in enumerate(P):
        z = F.conv2d(a, _r(w, bf16), b, padding=1)
        if l < len(P) - 1:
            a = _r(torch.relu(z), bf16)
            acts.append(a)
    y = x[:, 1] + z[:, 0] / s1
    return y.numpy(), (P, acts, z, x)


def loss_grad(params, x, t, layers, channels, s0, s1, bf16=True):
    """(loss, flat gradient in the library's layout)."""
    _, (P, acts, z, xt) = forward(params, x, layers, channels, s0, s1, bf16)
    t = torch.as_tensor(np.asarray(t, dtype=np.float64))
    r = z[:, 0] + s1 * xt[:, 1] - s1 * t
    npix = r.numel()
    loss = float((r * r).sum() / npix)
    g = torch.zeros_like(z)
    g[:, 0] = 2.0 * r / npix
    g = _r(g, bf16)
    grads = [None] * len(P)
    for l in range(len(P) - 1, -1, -1):
        w, _ = P[l]
        a = acts[l]
        dw = torch.nn.grad.conv2d_weight(a, w.shape, g, padding=1)
        db = g.sum(dim=(0, 2, 3))
        grads[l] = (dw, db)
        if l == 0:
            break
        da = torch.nn.grad.conv2d_input(a.shape, _r(w, bf16), g, padding=1)
        g = _r(da * (a > 0), bf16)
    return loss, pack(grads)


# ---------------------------------------------------------------- pins ----

def conv3x3_loops(a, w, b):
    """Direct sum of the definition (tiny inputs only): a [n][ci][H][W],
    w [co][ci][3][3], zero padding 1."""
    n, ci, H, W = a.shape
    co = w.shape[0]
    out = np.zeros((n, co, H, W))
    for i in range(n):
        for o in range(co):
            for y in range(H):
                for x in range(W):
                    s = b[o]
                    for c in range(ci):
                        for dy in range(3):
                            for dx in range(3):
                                yy, xx = y + dy - 1, x + dx - 1
                                if 0 <= yy < H and 0 <= xx < W:
                                    s += a[i, c, yy, xx] * w[o, c, dy, dx]
                    out[i, o, y, x] = s
    return out


def conv3x3_grads_loops(a, w, g):
    """Weight and input gradients of sum(conv3x3(a, w) * g) by direct sums."""
    n, ci, H, W = a.shape
    co = w.shape[0]
    dw = np.zeros_like(w)
    da = np.zeros_like(a)
    for i in range(n):
        for o in range(co):
            for y in range(H):
                for x in range(W):
                    for c in range(ci):
                        for dy in range(3):
                            for dx in range(3):
                                yy, xx = y + dy - 1, x + dx - 1
                                if 0 <= yy < H and 0 <= xx < W:
                                    dw[o, c, dy, dx] += a[i, c, yy, xx] * g[i, o, y, x]
                                    da[i, c, yy, xx] += w[o, c, dy, dx] * g[i, o, y, x]
    return dw, da
