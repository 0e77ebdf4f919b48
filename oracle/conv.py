"""Plain FP64 reference of the 3-D convolution network used for the learned
initial guess (test infrastructure only; shares nothing with the GPU code).

Tensors are channels-last: x[n, z, y, x, c].  Weights w[o, d, c] with the tap
index d = dx + 3 dy + 9 dz, dx, dy, dz in {0, 1, 2}.  Three tap patterns:

  s1 (stride 1, zero padding 1):   out[p] = sum_d,c w[o,d,c] x[p + d - 1]
  s2 (stride 2, zero padding 1):   out[p] = sum_d,c w[o,d,c] x[2p + d - 1]
  t2 (transposed stride 2):        out[P] = sum_d,c w[o,d,c] x[(P + 1 - d) / 2]
                                   (only where P + 1 - d is even)
with the offsets applied per axis and out-of-range input positions reading 0.
Grid sizes: s1 keeps G, s2 maps G -> (G-1)/2 + 1, t2 maps G -> 2(G-1) + 1.

Each function is the definition written out (a loop over the 27 taps with
array slicing); input and weight gradients are their own definitions too,
checked against central finite differences in tests/test_conv_oracle.py.
"""
import numpy as np

MODES = ("s1", "s2", "t2")


def out_size(G, mode):
    return {"s1": G, "s2": (G - 1) // 2 + 1, "t2": 2 * (G - 1) + 1}[mode]


def taps():
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                yield dx + 3 * dy + 9 * dz, (dz, dy, dx)


def _src_index(P, d, G_in, mode):
    """Input index along one axis for output indices P and tap offset d (0..2),
    and a validity mask."""
    if mode == "s1":
        i = P + d - 1
        ok = (i >= 0) & (i < G_in)
    elif mode == "s2":
        i = 2 * P + d - 1
        ok = (i >= 0) & (i < G_in)
    else:
        t = P + 1 - d
        ok = (t % 2 == 0) & (t >= 0) & (t // 2 < G_in)
        i = t // 2
    return np.where(ok, i, 0), ok


def gather(x, d3, mode, G_out):
    """x[n, src(z), src(y), src(x), c] for tap offsets d3 = (dz, dy, dx), zero where invalid."""
    G_in = x.shape[1]
    P = np.arange(G_out)
    (iz, oz), (iy, oy), (ix, ox) = (_src_index(P, d, G_in, mode) for d in d3)
    g = x[:, iz][:, :, iy][:, :, :, ix]
    mask = oz[:, None, None] & oy[None, :, None] & ox[None, None, :]
    return g * mask[None, :, :, :, None]


def conv3d(x, w, mode, bias=None):
    """out[n, p, o] = sum_{d, c} w[o, d, c] x[n, src(p, d), c] (+ bias[o])."""
    G_out = out_size(x.shape[1], mode)
    out = np.zeros(x.shape[:1] + (G_out,) * 3 + (w.shape[0],))
    for d, d3 in taps():
        out += gather(x, d3, mode, G_out) @ w[:, d, :].T
    if bias is not None:
        out += bias
    return out


def conv3d_weight_grad(gy, x, mode):
    """dL/dw[o, d, c] = sum_{n, p} gy[n, p, o] x[n, src(p, d), c]."""
    G_out = gy.shape[1]
    dw = np.zeros((gy.shape[-1], 27, x.shape[-1]))
    gyf = gy.reshape(-1, gy.shape[-1])
    for d, d3 in taps():
        dw[:, d, :] = gyf.T @ gather(x, d3, mode, G_out).reshape(-1, x.shape[-1])
    return dw


def conv3d_input_grad(gy, w, mode, G_in):
    """dL/dx[n, q, c] = sum over (p, d) with src(p, d) = q of w[o, d, c] gy[n, p, o],
    accumulated by scattering every tap's contribution back to its source
    (taps in order; one scatter of all valid output points per tap)."""
    n, G_out = gy.shape[0], gy.shape[1]
    gx = np.zeros((n, G_in, G_in, G_in, w.shape[2]))
    P = np.arange(G_out)
    for d, (dz, dy, dx) in taps():
        contrib = gy @ w[:, d, :]  # [n, p, c]
        (iz, oz), (iy, oy), (ix, ox) = (_src_index(P, dd, G_in, mode) for dd in (dz, dy, dx))
        a, b, c = np.nonzero(oz)[0], np.nonzero(oy)[0], np.nonzero(ox)[0]
        src = np.ix_(iz[a], iy[b], ix[c])
        np.add.at(gx, (slice(None),) + src, contrib[:, a][:, :, b][:, :, :, c])
    return gx


def adam_step(p, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1), all in FP32:
    m = beta1 m + (1 - beta1) g; v = beta2 v + (1 - beta2) g^2;
    m_hat = m / (1 - beta1^t); v_hat = v / (1 - beta2^t);
    p = p - lr m_hat / (sqrt(v_hat) + eps), t = 1, 2, ... the step number.
    Returns the new (p, m, v)."""
    f = np.float32
    p, m, v, g = (np.asarray(a, dtype=np.float32) for a in (p, m, v, g))
    b1, b2 = f(beta1), f(beta2)
    m = b1 * m + (f(1) - b1) * g
    v = b2 * v + (f(1) - b2) * (g * g)
    m_hat = m / (f(1) - b1 ** t)
    v_hat = v / (f(1) - b2 ** t)
    p = p - f(lr) * m_hat / (np.sqrt(v_hat) + f(eps))
    return p, m, v


def bf16(a):
    """Round to bfloat16 (round to nearest even on the FP32 bit pattern)."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- the network

# (Cin, Cout, mode, relu, skip source layer or None); layer outputs feed the next layer
LAYERS = [
    (8, 16, "s1", True, None),     # 0  G
    (16, 16, "s1", True, None),    # 1  G        -> skip s0
    (16, 32, "s2", True, None),    # 2  G/2
    (32, 32, "s1", True, None),    # 3           -> skip s1
    (32, 64, "s2", True, None),    # 4  G/4
    (64, 64, "s1", True, None),    # 5           -> skip s2
    (64, 128, "s2", True, None),   # 6  G/8
    (128, 128, "s1", True, None),  # 7
    (128, 64, "t2", True, 5),      # 8  G/4, + s2 before the ReLU
    (64, 64, "s1", True, None),    # 9
    (64, 32, "t2", True, 3),       # 10 G/2, + s1
    (32, 32, "s1", True, None),    # 11
    (32, 16, "t2", True, 1),       # 12 G, + s0
    (16, 8, "s1", False, None),    # 13 G, channel 0 is the prediction
]


def net_input(g, mask):
    """Channels: 0 boundary value (0 inside), 1 boundary mask, 2..7 zero."""
    x = np.zeros(g.shape + (8,))
    x[..., 0] = np.where(mask, g, 0.0)
    x[..., 1] = mask
    return x


def net_forward(params, x, round_bf16=False):
    """params: list of (w[o, 27, c], b[o]).  Returns the list of layer outputs.
    With round_bf16 the stored activations and the weights are rounded to
    bfloat16 (FP32 accumulation is emulated by FP64, a tighter reference)."""
    R = bf16 if round_bf16 else (lambda a: a)
    acts = []
    h = R(x)
    for li, (cin, cout, mode, relu, skip) in enumerate(LAYERS):
        w, b = params[li]
        pre = conv3d(h, R(w), mode, b)
        if skip is not None:
            pre = pre + acts[skip]
        out = np.maximum(pre, 0.0) if relu else pre
        h = R(out) if li < len(LAYERS) - 1 else out
        acts.append(h)
    return acts


def _a_times(diff, interior, apply_a):
    """A e per sample (node order x fastest, as the grid's C order), kept on
    interior nodes."""
    return np.stack([apply_a(d.ravel()).reshape(d.shape) for d in diff]) * interior


def net_loss(params, x, target, interior, round_bf16=False, apply_a=None):
    """Mean squared error of channel 0 over interior nodes; with apply_a (a
    function returning A v for a node vector v) the energy norm e^T A e of the
    interior error e instead, per interior node."""
    acts = net_forward(params, x, round_bf16)
    pred = acts[-1][..., 0]
    diff = (pred - target) * interior
    if apply_a is None:
        return float(np.sum(diff ** 2) / np.sum(interior)), acts
    return float(np.sum(diff * _a_times(diff, interior, apply_a)) / np.sum(interior)), acts


def net_grads_bf16(params, x, target, interior, apply_a=None, rounded=True):
    """The gradient of net_loss as a bfloat16 network computes it: weights,
    input and stored activations in bfloat16 (net_forward with round_bf16),
    the output gradient 2 e / count (or 2 A e / count) rounded to bfloat16,
    every layer's output gradient stored in bfloat16 (a skip connection's
    share added first, then the input gradient of the next layer, the sum
    rounded once), sums taken exactly (FP64 standing in for FP32
    accumulation).  The ReLU masks come from the stored activations.
    rounded=False drops every rounding, which leaves the FP64 chain rule.
    Returns ([(dw, db)], [(sum |gy| |x|, sum |gy|)]) per layer: the
    gradient and the sums of absolute terms behind each entry."""
    R = bf16 if rounded else (lambda a: a)
    pb = [(R(w), b) for w, b in params]
    xb = R(x)
    acts = net_forward(pb, xb, round_bf16=rounded)
    count = float(np.sum(interior))
    diff = (acts[-1][..., 0] - target) * interior
    g_out = np.zeros_like(acts[-1])
    g_out[..., 0] = R(2.0 * (diff if apply_a is None else _a_times(diff, interior, apply_a)) / count)
    grads, sc = [None] * len(LAYERS), [None] * len(LAYERS)
    g_act = {len(LAYERS) - 1: g_out}
    for li in range(len(LAYERS) - 1, -1, -1):
        cin, cout, mode, relu, skip = LAYERS[li]
        gy = g_act.pop(li)
        if relu:
            gy = gy * (acts[li] > 0)
        h_in = acts[li - 1] if li > 0 else xb
        grads[li] = (conv3d_weight_grad(gy, h_in, mode), gy.reshape(-1, cout).sum(axis=0))
        sc[li] = (conv3d_weight_grad(np.abs(gy), np.abs(h_in), mode), np.abs(gy).reshape(-1, cout).sum(axis=0))
        if skip is not None:
            g_act[skip] = R(g_act.get(skip, 0.0) + gy)
        if li > 0:
            g_act[li - 1] = R(conv3d_input_grad(gy, pb[li][0], mode, h_in.shape[1]) + g_act.get(li - 1, 0.0))
    return grads, sc


def net_grads(params, x, target, interior, apply_a=None, scales=False):
    """Gradient of net_loss (FP64) by the chain rule through conv3d_input_grad /
    conv3d_weight_grad; returns [(dw, db)] per layer.  For the energy norm the
    output gradient is 2 A e (A symmetric).  With scales, also returns per
    layer the sums of absolute terms behind each entry, (sum |gy| |x|, sum |gy|),
    the scale that rounding errors of the summed terms are relative to."""
    acts = net_forward(params, x)
    count = float(np.sum(interior))
    g_out = np.zeros_like(acts[-1])
    diff = (acts[-1][..., 0] - target) * interior
    g_out[..., 0] = 2.0 * (diff if apply_a is None else _a_times(diff, interior, apply_a)) / count
    grads = [None] * len(LAYERS)
    sc = [None] * len(LAYERS)
    g_act = {len(LAYERS) - 1: g_out}
    for li in range(len(LAYERS) - 1, -1, -1):
        cin, cout, mode, relu, skip = LAYERS[li]
        gy = g_act.pop(li)
        if relu:
            gy = gy * (acts[li] > 0)
        h_in = acts[li - 1] if li > 0 else x
        w, _ = params[li]
        grads[li] = (conv3d_weight_grad(gy, h_in, mode), gy.reshape(-1, cout).sum(axis=0))
        if scales:
            sc[li] = (conv3d_weight_grad(np.abs(gy), np.abs(h_in), mode), np.abs(gy).reshape(-1, cout).sum(axis=0))
        if skip is not None:
            g_act[skip] = g_act.get(skip, 0.0) + gy
        if li > 0:
            g_act[li - 1] = g_act.get(li - 1, 0.0) + conv3d_input_grad(gy, w, mode, h_in.shape[1])
    return (grads, sc) if scales else grads
