"""GPU parity of the BF16 matrix-core convolutions and the learned-guess
network against the FP64 conv oracle (oracle/conv.py).

Inputs and weights are rounded to bfloat16 on the host first, so the oracle
sees exactly the operands the matrix cores multiply; the GPU accumulates in
FP32:
  conv forward   |y32 - ref| <= 1e-5 * sum |w| |x| (+ the bf16 store: 2^-8 |ref|)
  weight grad    |dw - ref|  <= 1e-5 * sum |gy| |x| over the reduction
  input grad     |gx32 - ref| <= 1e-5 * sum |w| |gy| (+ 2^-8 |ref| for the
                 bf16 store), s1 / s2 / t2 at the network's channel counts and
                 grids, 65^3 and 33^3 included, with and without accumulation
  network        the whole-network gradient against the bfloat16-emulated
                 chain rule (oracle/conv.net_grads_bf16: the GPU's rounding
                 points, exact sums).  With every ReLU pre-activation at
                 least 1 from the kink (half the masks zero), every entry:
                 |g - ref| <= 1e-2 * sum of the entry's absolute terms, and
                 the prediction likewise.  With He initialisation, where
                 rounding can flip a ReLU mask (which changes whole terms),
                 per layer rel. L2 <= 0.2, cosine >= 0.98, per tap <= 0.3
  Adam           three FP32 steps against oracle/conv.adam_step, every
                 parameter within 1e-6 (|p| + lr t)
"""
import numpy as np
import pytest
import torch

from oracle import conv

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1505_08023_amd.mfe import Context
    c = Context(0)
    yield c
    c.close()


def to_bf16_tensor(a, device):
    return torch.tensor(np.asarray(a, np.float32), device=device).to(torch.bfloat16)


CASES = [("s1", 9, 8, 16), ("s1", 9, 16, 16), ("s1", 5, 128, 128), ("s2", 17, 16, 32), ("s2", 9, 64, 128),
         ("t2", 9, 32, 16), ("t2", 5, 128, 64), ("s1", 9, 16, 8)]
# small grids split the reduction over several workgroups (summed in a fixed
# order afterwards); these larger ones run unsplit with the wider wave tiles
LARGE = [("s1", 65, 8, 16, 1), ("s1", 33, 16, 32, 2), ("t2", 33, 32, 16, 1)]


@pytest.mark.parametrize("mode,G,cin,cout,batch", [c + (2,) for c in CASES] + LARGE)
def test_conv_forward(ctx, mode, G, cin, cout, batch):
    from paper_1505_08023_amd.mfe import conv3d
    rng = np.random.default_rng(hash((mode, G, cin, cout)) % 2 ** 32)
    x = conv.bf16(rng.standard_normal((batch, G, G, G, cin)))
    w = conv.bf16(rng.standard_normal((cout, 27, cin)) / np.sqrt(27 * cin))
    b = rng.standard_normal(cout).astype(np.float32)
    xg = to_bf16_tensor(x, ctx.device)
    y, y32 = conv3d(ctx, mode, xg, w, b, relu=False, out32=True)
    ref = conv.conv3d(x, w, mode, b.astype(np.float64))
    scale = conv.conv3d(np.abs(x), np.abs(w), mode) + np.abs(b)
    y32 = y32.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(y32 - ref) <= 1e-5 * scale + 1e-6)
    yb = y.float().cpu().numpy().astype(np.float64)
    assert np.all(np.abs(yb - ref) <= 2 ** -8 * np.abs(ref) + 1e-5 * scale + 1e-6)
    # ReLU epilogue
    yr = conv3d(ctx, mode, xg, w, b, relu=True).float().cpu().numpy()
    assert np.all(np.abs(yr - np.maximum(yb, 0)) <= 1e-6 + 2 ** -8 * np.abs(yb))


@pytest.mark.parametrize("mode,G,cin,cout", CASES)
def test_conv_weight_gradient(ctx, mode, G, cin, cout):
    from paper_1505_08023_amd.mfe import conv3d_wgrad
    rng = np.random.default_rng(7 + hash((mode, G, cin, cout)) % 2 ** 30)
    x = conv.bf16(rng.standard_normal((2, G, G, G, cin)))
    Go = conv.out_size(G, mode)
    gy = conv.bf16(rng.standard_normal((2, Go, Go, Go, cout)))
    dw = conv3d_wgrad(ctx, mode, to_bf16_tensor(x, ctx.device), to_bf16_tensor(gy, ctx.device)).astype(np.float64)
    ref = conv.conv3d_weight_grad(gy, x, mode)
    scale = conv.conv3d_weight_grad(np.abs(gy), np.abs(x), mode)
    assert np.all(np.abs(dw - ref) <= 1e-5 * scale + 1e-6)


# (mode, G_in, cin, cout, batch) of the forward convolution whose input
# gradient is formed: the small split-reduction cases and the network's own
# layers at G = 65 (batch 1: the unsplit paths and the LDS stride-1 path)
DGRAD = [c + (2,) for c in CASES] + [("s1", 65, 16, 16, 1), ("s2", 65, 16, 32, 1), ("t2", 33, 32, 16, 1),
                                      ("s1", 65, 16, 8, 1), ("s1", 33, 32, 32, 1), ("s2", 33, 32, 64, 1),
                                      ("t2", 17, 64, 32, 1), ("t2", 9, 128, 64, 1)]


@pytest.mark.parametrize("accumulate", [False, True])
@pytest.mark.parametrize("mode,G,cin,cout,batch", DGRAD)
def test_conv_input_gradient(ctx, mode, G, cin, cout, batch, accumulate):
    from paper_1505_08023_amd.mfe import conv3d_dgrad
    print("dgrad", mode, G, cin, cout, batch, accumulate, flush=True)
    rng = np.random.default_rng(11 + hash((mode, G, cin, cout)) % 2 ** 30)
    Go = conv.out_size(G, mode)
    gy = conv.bf16(rng.standard_normal((batch, Go, Go, Go, cout)))
    w = conv.bf16(rng.standard_normal((cout, 27, cin)) / np.sqrt(27 * cin))
    ref = conv.conv3d_input_grad(gy, w, mode, G)
    scale = conv.conv3d_input_grad(np.abs(gy), np.abs(w), mode, G)
    gx0 = None
    if accumulate:
        prev = conv.bf16(rng.standard_normal((batch, G, G, G, cin)))
        ref = ref + prev
        scale = scale + np.abs(prev)
        gx0 = to_bf16_tensor(prev, ctx.device)
    gx, gx32 = conv3d_dgrad(ctx, mode, to_bf16_tensor(gy, ctx.device), w, G, gx=gx0, accumulate=accumulate,
                            out32=True)
    g32 = gx32.cpu().numpy().astype(np.float64)
    err = np.abs(g32 - ref)
    print("dgrad worst |d| / scale", float(np.max(err / (scale + 1e-30))))
    assert np.all(err <= 1e-5 * scale + 1e-6)
    gb = gx.float().cpu().numpy().astype(np.float64)
    assert np.all(np.abs(gb - ref) <= 2 ** -8 * np.abs(ref) + 1e-5 * scale + 1e-6)


def test_adam_steps_match_oracle(ctx):
    """Three Adam steps on the GPU's FP32 master weights, with gradients set
    through mfe_net_set_grad, against oracle/conv.adam_step: the standard
    hyper-parameters, then a large eps and no first-moment memory."""
    from paper_1505_08023_amd.mfe import Net
    net = Net(ctx, 9, 1)
    rng = np.random.default_rng(21)
    n = net.nparams
    for lr, b1, b2, eps in ((1e-3, 0.9, 0.999, 1e-8), (0.05, 0.0, 0.99, 0.5)):
        p = rng.standard_normal(n).astype(np.float32)
        net.set_params(p)
        m, v = np.zeros(n, np.float32), np.zeros(n, np.float32)
        for t in range(1, 4):
            g = (rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 1, n)).astype(np.float32)
            net.set_grad(g)
            net.adam_step(lr, b1, b2, eps)
            p, m, v = conv.adam_step(p, m, v, g, t, lr, b1, b2, eps)
            got = net.get_params()
            err = np.abs(got.astype(np.float64) - p)
            assert np.all(err <= 1e-6 * (np.abs(p) + lr * t)), (t, float(err.max()))
    net.close()


def he_params(rng, scale=1.0):
    return [(rng.standard_normal((co, 27, ci)) * scale * np.sqrt(2.0 / (27 * ci)), rng.standard_normal(co) * 0.01)
            for ci, co, *_ in conv.LAYERS]


def flatten(params):
    return np.concatenate([np.concatenate([w.ravel(), b]) for w, b in params]).astype(np.float32)


def unflatten(flat):
    out, q = [], 0
    for ci, co, *_ in conv.LAYERS:
        w = flat[q:q + co * 27 * ci].reshape(co, 27, ci)
        q += co * 27 * ci
        b = flat[q:q + co]
        q += co
        out.append((w.astype(np.float64), b.astype(np.float64)))
    return out


def boundary_mask(G):
    m = np.zeros((G, G, G), bool)
    m[0], m[-1], m[:, 0], m[:, -1], m[:, :, 0], m[:, :, -1] = (True,) * 6
    return m


def test_network_parameters_roundtrip(ctx):
    from paper_1505_08023_amd.mfe import Net
    net = Net(ctx, 17, 2)
    p = flatten(he_params(np.random.default_rng(0)))
    assert net.nparams == p.size
    net.set_params(p)
    assert np.array_equal(net.get_params(), p)
    net.close()


def margin_params(rng):
    """Weights at a tenth of the He scale, biases +4 on even and -4 on odd
    output channels of every ReLU layer (0 on the linear last layer): every
    pre-activation then stays at least 1 away from the ReLU's kink (checked
    on the oracle's forward pass), so no rounding difference can move a ReLU
    mask, while half of the masks are zero."""
    out = []
    for ci, co, mode, relu, skip in conv.LAYERS:
        b = np.where(np.arange(co) % 2 == 0, 4.0, -4.0) if relu else np.zeros(co)
        out.append((rng.standard_normal((co, 27, ci)) * 0.1 * np.sqrt(2.0 / (27 * ci)), b))
    return out


def pre_activations(pb, x):
    """The bfloat16 forward pass of the oracle, returning every layer's value
    before its ReLU."""
    pre, acts, h = [], [], conv.bf16(x)
    for li, (cin, cout, mode, relu, skip) in enumerate(conv.LAYERS):
        w, b = pb[li]
        z = conv.conv3d(h, w, mode, b) + (acts[skip] if skip is not None else 0.0)
        pre.append(z)
        h = conv.bf16(np.maximum(z, 0.0)) if relu else z
        acts.append(h)
    return pre


def check_prediction(pred, pb, x, ref_pred):
    """Every predicted value within 1e-2 of the sum of the absolute terms of
    the last layer's output."""
    acts_abs = conv.net_forward(pb, x, round_bf16=True)
    h = np.abs(acts_abs[-2])
    w, b = pb[-1]
    scale = conv.conv3d(h, np.abs(w), "s1", np.abs(b))[..., 0]
    err = np.abs(pred - ref_pred)
    print("prediction worst |d| / scale", float(np.max(err / scale)))
    assert np.all(err <= 1e-2 * scale)


def check_gradient_entries(got, ref, scales, what):
    """Per entry |g - ref| <= 1e-2 * (sum of its absolute terms); an entry
    whose terms all vanish must be exactly 0."""
    for li, ((gw, gb), (rw, rb), (sw, sb)) in enumerate(zip(got, ref, scales)):
        ew, eb = np.abs(gw - rw), np.abs(gb - rb)
        worst = max(float(np.max(ew / (sw + 1e-300))), float(np.max(eb / (sb + 1e-300))))
        print(what, "layer", li, "worst |d| / absolute sum", worst)
        assert np.all(ew <= 1e-2 * sw) and np.all(eb <= 1e-2 * sb), (what, li, worst)


def check_gradient_groups(got, ref, what):
    """The general regime, where rounding can move ReLU masks: per layer
    relative L2 <= 0.2 and cosine >= 0.98, and per tap d (all o, c) relative
    L2 <= 0.3, so a mistake confined to one tap of one layer still fails."""
    for li, ((gw, gb), (rw, rb)) in enumerate(zip(got, ref)):
        a, r = np.concatenate([gw.ravel(), gb]), np.concatenate([rw.ravel(), rb])
        err = np.linalg.norm(a - r) / np.linalg.norm(r)
        cos = float(a @ r / (np.linalg.norm(a) * np.linalg.norm(r)))
        d = (gw - rw).transpose(1, 0, 2).reshape(27, -1)
        tap = np.linalg.norm(d, axis=1) / np.linalg.norm(rw.transpose(1, 0, 2).reshape(27, -1), axis=1)
        print(what, "layer", li, "rel L2", err, "cos", cos, "worst tap", float(tap.max()))
        assert err <= 0.2 and cos >= 0.98 and np.all(tap <= 0.3), (what, li, err, cos, float(tap.max()))


def network_case(rng, G, B, params):
    mask = boundary_mask(G)
    g = rng.uniform(0, 1, (B, G, G, G))
    target = rng.uniform(0, 1, (B, G, G, G))
    x = np.stack([conv.net_input(g[i], mask) for i in range(B)])
    interior = np.broadcast_to(~mask, (B, G, G, G)).astype(float)
    return g, target, x, interior


@pytest.mark.parametrize("regime", ["margin", "general"])
def test_network_forward_and_gradient(ctx, regime):
    """The squared-error loss and its gradient through the whole network
    against the bfloat16-emulated oracle (the GPU's rounding points).  In the
    margin regime (no ReLU mask within reach of rounding) the prediction and
    every gradient entry meet the 1e-2 bar of the sum of their absolute
    terms; measured worst 3e-3, in the deepest layers.  In the general regime
    (He initialisation) rounding moves a few ReLU masks, each of which
    changes whole terms, so there the bar is per layer and per tap."""
    from paper_1505_08023_amd.mfe import Net
    G, B = 17, 2
    rng = np.random.default_rng(1)
    params = unflatten(flatten(margin_params(rng) if regime == "margin" else he_params(rng)))
    pb = [(conv.bf16(w), b) for w, b in params]  # the GPU multiplies bf16 weights
    g, target, x, interior = network_case(rng, G, B, params)
    if regime == "margin":
        for (cin, cout, mode, relu, skip), z in zip(conv.LAYERS, pre_activations(pb, x)):
            if relu:
                assert z[..., 0::2].min() >= 1.0 and z[..., 1::2].max() <= -1.0
    net = Net(ctx, G, B)
    net.set_params(flatten(params))
    gt = torch.tensor(g.reshape(-1), device=ctx.device)
    tt = torch.tensor(target.reshape(-1), device=ctx.device)
    pred = net.forward(gt).cpu().numpy().reshape(B, G, G, G)
    acts = conv.net_forward(pb, x, round_bf16=True)
    check_prediction(pred, pb, x, acts[-1][..., 0])
    loss, grad = net.loss_grad(gt, tt, want_grad=True)
    ref_loss, _ = conv.net_loss(pb, x, target, interior, round_bf16=True)
    assert abs(loss - ref_loss) <= 0.02 * ref_loss
    ref_grads, scales = conv.net_grads_bf16(params, x, target, interior)
    if regime == "margin":
        check_gradient_entries(unflatten(grad), ref_grads, scales, "mse")
    else:
        check_gradient_groups(unflatten(grad), ref_grads, "mse")
    net.close()


@pytest.mark.parametrize("regime", ["margin", "general"])
def test_network_energy_loss_gradient(ctx, regime):
    """The energy-norm loss e^T A e / count (A the 16^3 stiffness matrix,
    applied by the library's SpMV) and the gradient through the network
    against the bfloat16-emulated oracle gradient, with both formats, under
    the two regimes of test_network_forward_and_gradient."""
    import oracle
    from paper_1505_08023_amd.mfe import Net, Problem
    G, B = 17, 2
    rng = np.random.default_rng(7)
    params = unflatten(flatten(margin_params(rng) if regime == "margin" else he_params(rng)))
    pb = [(conv.bf16(w), b) for w, b in params]
    g, target, x, interior = network_case(rng, G, B, params)
    A = oracle.assemble(G - 1, G - 1, G - 1)
    apply_a = lambda v: oracle.csr_spmv(A, v)
    prob = Problem.mesh(ctx, G - 1, G - 1, G - 1)
    net = Net(ctx, G, B)
    net.set_params(flatten(params))
    gt = torch.tensor(g.reshape(-1), device=ctx.device)
    tt = torch.tensor(target.reshape(-1), device=ctx.device)
    ref_loss, _ = conv.net_loss(pb, x, target, interior, round_bf16=True, apply_a=apply_a)
    ref_grads, ref_scales = conv.net_grads_bf16(params, x, target, interior, apply_a=apply_a)
    losses = {}
    for fmt in ("bcrs13", "csr"):
        loss, grad = net.loss_grad(gt, tt, want_grad=True, energy=prob, fmt=fmt)
        losses[fmt] = loss
        assert abs(loss - ref_loss) <= 0.02 * ref_loss, (fmt, loss, ref_loss)
        if regime == "margin":
            check_gradient_entries(unflatten(grad), ref_grads, ref_scales, "energy " + fmt)
        else:
            check_gradient_groups(unflatten(grad), ref_grads, "energy " + fmt)
    assert abs(losses["csr"] - losses["bcrs13"]) <= 1e-12 * losses["csr"]
    # the mesh must be the network's grid
    other = Problem.mesh(ctx, 8, 8, 8)
    with pytest.raises(RuntimeError):
        net.loss_grad(gt, tt, energy=other)
    other.close()
    prob.close()
    net.close()


def test_network_graph_replays(ctx):
    """The forward and backward passes replay captured graphs: alternating
    inputs, with other device work in between, reproduce every result
    bitwise, and a different input gives a different result."""
    from paper_1505_08023_amd.mfe import Net
    G, B = 17, 2
    rng = np.random.default_rng(5)
    net = Net(ctx, G, B)
    net.set_params(flatten(he_params(rng)))
    gs = [torch.tensor(rng.uniform(0, 1, B * G ** 3), device=ctx.device) for _ in range(2)]
    tt = torch.tensor(rng.uniform(0, 1, B * G ** 3), device=ctx.device)
    first = []
    for rep in range(3):
        for i, g in enumerate(gs):
            pred = net.forward(g).cpu().numpy()
            loss, grad = net.loss_grad(g, tt, want_grad=True)
            junk = torch.randn(1 << 20, device=ctx.device)  # eager work between replays
            junk.mul_(2.0).sum().item()
            if rep == 0:
                first.append((pred, loss, grad))
            else:
                assert np.array_equal(pred, first[i][0]) and loss == first[i][1]
                assert np.array_equal(grad, first[i][2])
    assert not np.array_equal(first[0][0], first[1][0])
    net.close()


def test_network_training_reduces_loss(ctx):
    from paper_1505_08023_amd.mfe import Net
    G, B = 17, 4
    rng = np.random.default_rng(2)
    net = Net(ctx, G, B)
    net.set_params(flatten(he_params(rng)))
    # a smooth target that depends on the boundary data: the average face value
    g = rng.uniform(0, 1, (B, G, G, G))
    target = np.repeat(g.reshape(B, -1).mean(axis=1), G ** 3)
    gt = torch.tensor(g.reshape(-1), device=ctx.device)
    tt = torch.tensor(target, device=ctx.device)
    losses = []
    for _ in range(60):
        losses.append(net.loss_grad(gt, tt))
        net.adam_step(1e-3)
    assert losses[-1] < 0.2 * losses[0], losses[::10]
    # predict_x0 keeps the boundary values exactly
    x0 = net.predict_x0(gt[:G ** 3].contiguous()).cpu().numpy().reshape(G, G, G)
    m = boundary_mask(G)
    assert np.array_equal(x0[m], g[0][m])
    net.close()


def test_trained_network_reduces_cg_iterations(ctx):
    """The shipped 64^3 network against the method without it, on held-out
    boundary data: CG (FP64, and FP32-inner / FP64-refinement) from the
    network's guess reaches the same 1e-8 tolerance in fewer iterations than
    from x0 = 0, and every guess is kept (its residual is below ||b||)."""
    import os
    from paper_1505_08023_amd import learned
    from paper_1505_08023_amd.mfe import Net
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    params, meta = learned.load(os.path.join(root, "paper_1505_08023_amd", "weights", "net64.npz"))
    net = Net(ctx, 65, 1)
    net.set_params(params)
    seeds = list(range(learned.HELD_OUT_BASE + 900, learned.HELD_OUT_BASE + 904))
    ev = learned.evaluate(ctx, net, 64, seeds)
    print({k: v for k, v in ev.items() if k != "rows"})
    assert ev["guesses_used"] == len(seeds) and ev["guesses_used_mixed"] == len(seeds)
    assert ev["worst_res_learned"] <= 1e-8 and ev["worst_res_learned_mixed"] <= 1e-8
    assert ev["mean_its_learned"] <= 0.85 * ev["mean_its_plain"]
    assert ev["mean_its_learned_mixed"] < ev["mean_its_mixed"]
    # and than from the trivial guess that is exact on the boundary only
    assert ev["mean_its_learned"] < ev["mean_its_boundary_start"] <= ev["mean_its_plain"]
    assert ev["mean_guess_rel_res"] < 1e-2
    net.close()
