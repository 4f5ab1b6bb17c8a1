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
(torch CPU) by default: that plain network is the reference the GPU
library is held to.  The storage points of the network are the values a
BF16 implementation keeps in that format: the inputs a_0, the weights,
every hidden activation, the output gradient and every hidden gradient.
`bf16` selects the map applied there: none (default), rounding to bfloat16
(nearest even; a diagnostic emulation), or a callable (the error model
below).  The backward pass is written out layer by layer (weight and input
gradients of a convolution from torch's convolution-gradient routines) so
that the storage points sit between the layers' products.

Pins (tests): a brute-force loop convolution and its two gradients on tiny
inputs, a centre-tap kernel reproducing its input, and central finite
differences of the loss against this backward pass.

Error model of BF16 storage (`rounding_model`).  A value stored in bfloat16
with round-to-nearest is x (1 + d), |d| <= u = 2^-8.  Following the
probabilistic rounding-error analysis of Higham and Mary (SIAM J. Sci.
Comput. 41, 2019), the d of different stored values are modelled as
independent, mean zero and uniform on [-u, u]; each stored value (every
weight once, every activation and gradient element once) gets its own d.
The FP64 network is run with such perturbations at every storage point and
the relative L2 deviations of the output, the loss and each layer's
gradient from the unperturbed FP64 network are averaged in quadrature over
a few draws.  This gives, before any GPU result is seen, the expected size
of the error that storing those values in BF16 causes; FP32 accumulation
adds ~sqrt(576) 2^-24 ~ 1e-6, negligible beside it.
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


U_BF16 = 2.0 ** -8   # unit roundoff of bfloat16 (8 significant bits)


def _store(bf16):
    """The map applied at every storage point: identity (plain FP64), BF16
    round-to-nearest-even (bf16=True), or a callable."""
    if callable(bf16):
        return bf16
    if bf16:
        return lambda x: x.to(torch.bfloat16).to(torch.float64)
    return lambda x: x


def _forward(P, x, s0, s1, st):
    """Forward pass with the weights already stored; st is the storage map
    of the activations."""
    a = st(torch.stack([s0 * x[:, 0], s1 * x[:, 1]], dim=1))
    acts = [a]
    z = None
    for l, (w, b) in enumerate(P):
        z = F.conv2d(a, w, b, padding=1)
        if l < len(P) - 1:
            a = st(torch.relu(z))
            acts.append(a)
    return acts, z


def forward(params, x, layers, channels, s0, s1, bf16=False):
    """y [n][H][W] and the cache of the backward pass; x [n][2][H][W]."""
    st = _store(bf16)
    P = [(st(w), b) for w, b in unpack(params, layers, channels)]
    x = torch.as_tensor(np.asarray(x, dtype=np.float64))
    acts, z = _forward(P, x, s0, s1, st)
    y = x[:, 1] + z[:, 0] / s1
    return y.numpy(), (P, acts, z, x)


def loss_grad(params, x, t, layers, channels, s0, s1, bf16=False):
    """(loss, flat gradient in the library's layout)."""
    st = _store(bf16)
    _, (P, acts, z, xt) = forward(params, x, layers, channels, s0, s1, st)
    t = torch.as_tensor(np.asarray(t, dtype=np.float64))
    r = z[:, 0] + s1 * xt[:, 1] - s1 * t
    npix = r.numel()
    loss = float((r * r).sum() / npix)
    g = torch.zeros_like(z)
    g[:, 0] = 2.0 * r / npix
    g = st(g)
    grads = [None] * len(P)
    for l in range(len(P) - 1, -1, -1):
        w, _ = P[l]
        a = acts[l]
        dw = torch.nn.grad.conv2d_weight(a, w.shape, g, padding=1)
        db = g.sum(dim=(0, 2, 3))
        grads[l] = (dw, db)
        if l == 0:
            break
        da = torch.nn.grad.conv2d_input(a.shape, w, g, padding=1)
        g = st(da * (a > 0))
    return loss, pack(grads)


def layer_slices(layers, channels):
    """Slices of the flat parameter (or gradient) vector, one per layer."""
    out, off = [], 0
    for ci, co in layer_shapes(layers, channels):
        k = co * 9 * ci + co
        out.append(slice(off, off + k))
        off += k
    return out


def perturbation(u, gen):
    """Storage map of the error model: x (1 + d), d ~ U[-u, u] drawn
    independently for every element each time a value is stored."""
    def st(x):
        d = (torch.rand(x.shape, generator=gen, dtype=torch.float64) * 2.0 - 1.0) * u
        return x * (1.0 + d)
    return st


def rounding_model(params, x, t, layers, channels, s0, s1, draws=8, seed=0, u=U_BF16):
    """Expected relative errors of BF16 storage under the error model above:
    dict with 'out' (rel-L2 of z / s1 = y - x1), 'loss' (relative) and
    'grads' (rel-L2 per layer), each the root mean square over `draws`
    perturbed FP64 runs against the plain FP64 network."""
    x = np.asarray(x, dtype=np.float64)
    y0, _ = forward(params, x, layers, channels, s0, s1, bf16=False)
    l0, g0 = loss_grad(params, x, t, layers, channels, s0, s1, bf16=False)
    z0 = y0 - x[:, 1]
    sl = layer_slices(layers, channels)
    gen = torch.Generator().manual_seed(int(seed))
    eo, el, eg = [], [], []
    for _ in range(draws):
        st = perturbation(u, gen)
        P = [(st(w), b) for w, b in unpack(params, layers, channels)]
        xt = torch.as_tensor(x)
        acts, z = _forward(P, xt, s0, s1, st)
        zp = (z[:, 0] / s1).numpy()
        eo.append(np.linalg.norm(zp - z0) / np.linalg.norm(z0))
        # loss and gradients of the perturbed network, with the gradient
        # storage points perturbed too
        lp, gp = loss_grad(params, x, t, layers, channels, s0, s1, bf16=st)
        el.append(abs(lp - l0) / abs(l0))
        eg.append([np.linalg.norm(gp[s] - g0[s]) / np.linalg.norm(g0[s]) for s in sl])
    rms = lambda v: np.sqrt(np.mean(np.square(np.asarray(v)), axis=0))
    return {"out": float(rms(eo)), "loss": float(rms(el)), "grads": rms(eg)}


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
