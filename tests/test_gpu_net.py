"""GPU parity of the BF16 matrix-core convolutions and the learned-guess
network against the FP64 conv oracle (oracle/conv.py).

Inputs and weights are rounded to bfloat16 on the host first, so the oracle
sees exactly the operands the matrix cores multiply; the GPU accumulates in
FP32:
  conv forward   |y32 - ref| <= 1e-5 * sum |w| |x| (+ the bf16 store: 2^-8 |ref|)
  weight grad    |dw - ref|  <= 1e-5 * sum |gy| |x| over the reduction
  network        the whole-network gradient against the FP64 chain rule on
                 the same parameters: per layer relative L2 error <= 0.1 and
                 cosine >= 0.99 (activations and gradients are stored in
                 bfloat16 on the GPU, 2^-8 relative per value)
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


def test_network_forward_and_gradient(ctx):
    from paper_1505_08023_amd.mfe import Net
    G, B = 17, 2
    rng = np.random.default_rng(1)
    params = unflatten(flatten(he_params(rng)))
    pb = [(conv.bf16(w), b) for w, b in params]  # the GPU multiplies bf16 weights
    mask = boundary_mask(G)
    g = rng.uniform(0, 1, (B, G, G, G))
    target = rng.uniform(0, 1, (B, G, G, G))
    x = np.stack([conv.net_input(g[i], mask) for i in range(B)])
    interior = np.broadcast_to(~mask, (B, G, G, G)).astype(float)
    net = Net(ctx, G, B)
    net.set_params(flatten(params))
    gt = torch.tensor(g.reshape(-1), device=ctx.device)
    tt = torch.tensor(target.reshape(-1), device=ctx.device)
    pred = net.forward(gt).cpu().numpy().reshape(B, G, G, G)
    acts = conv.net_forward(pb, x, round_bf16=True)
    ref_pred = acts[-1][..., 0]
    rel = np.linalg.norm(pred - ref_pred) / np.linalg.norm(ref_pred)
    assert rel <= 0.02, rel
    loss, grad = net.loss_grad(gt, tt, want_grad=True)
    ref_loss, _ = conv.net_loss(pb, x, target, interior, round_bf16=True)
    assert abs(loss - ref_loss) <= 0.02 * ref_loss
    ref_grads = conv.net_grads(pb, x, target, interior)
    got = unflatten(grad)
    for li, ((gw, gb), (rw, rb)) in enumerate(zip(got, ref_grads)):
        a = np.concatenate([gw.ravel(), gb])
        r = np.concatenate([rw.ravel(), rb])
        err = np.linalg.norm(a - r) / np.linalg.norm(r)
        cos = float(a @ r / (np.linalg.norm(a) * np.linalg.norm(r)))
        print("layer", li, "rel err", err, "cos", cos)
        assert err <= 0.1 and cos >= 0.99, (li, err, cos)
    net.close()


def test_network_energy_loss_gradient(ctx):
    """The energy-norm loss e^T A e / count (A the 16^3 stiffness matrix,
    applied by the library's SpMV) and the gradient through the network,
    against the FP64 oracle on the same bf16 parameters, with both formats.
    The output gradient 2 A e is a second difference of the error, and its
    products with the smooth activations cancel more than those of the
    squared error's 2 e do (the sums come out 1.3-2.5 times smaller against
    the sums of their absolute terms), so each layer's error is bounded
    against those absolute sums: ||dw - ref|| <= 0.1 ||sum |gy| |x| || (the
    squared-error test's 10 % taken against the scale of the terms rather than
    of their sum), with the same cosine >= 0.99.  A dropped factor 2 errs by
    0.12-0.27 of that scale and a sign or operand mistake fails the cosine."""
    import oracle
    from paper_1505_08023_amd.mfe import Net, Problem
    G, B = 17, 2
    rng = np.random.default_rng(7)
    params = unflatten(flatten(he_params(rng)))
    pb = [(conv.bf16(w), b) for w, b in params]
    mask = boundary_mask(G)
    g = rng.uniform(0, 1, (B, G, G, G))
    target = rng.uniform(0, 1, (B, G, G, G))
    x = np.stack([conv.net_input(g[i], mask) for i in range(B)])
    interior = np.broadcast_to(~mask, (B, G, G, G)).astype(float)
    A = oracle.assemble(G - 1, G - 1, G - 1)
    apply_a = lambda v: oracle.csr_spmv(A, v)
    prob = Problem.mesh(ctx, G - 1, G - 1, G - 1)
    net = Net(ctx, G, B)
    net.set_params(flatten(params))
    gt = torch.tensor(g.reshape(-1), device=ctx.device)
    tt = torch.tensor(target.reshape(-1), device=ctx.device)
    ref_loss, _ = conv.net_loss(pb, x, target, interior, round_bf16=True, apply_a=apply_a)
    ref_grads, ref_scales = conv.net_grads(pb, x, target, interior, apply_a=apply_a, scales=True)
    losses = {}
    for fmt in ("bcrs13", "csr"):
        loss, grad = net.loss_grad(gt, tt, want_grad=True, energy=prob, fmt=fmt)
        losses[fmt] = loss
        assert abs(loss - ref_loss) <= 0.02 * ref_loss, (fmt, loss, ref_loss)
        for li, ((gw, gb), (rw, rb), (sw, sb)) in enumerate(zip(unflatten(grad), ref_grads, ref_scales)):
            a = np.concatenate([gw.ravel(), gb])
            r = np.concatenate([rw.ravel(), rb])
            sc = np.concatenate([sw.ravel(), sb])
            err = np.linalg.norm(a - r) / np.linalg.norm(sc)
            cos = float(a @ r / (np.linalg.norm(a) * np.linalg.norm(r)))
            print(fmt, "layer", li, "error / absolute sums", err, "rel err", np.linalg.norm(a - r) / np.linalg.norm(r),
                  "cos", cos)
            assert err <= 0.1 and cos >= 0.99, (fmt, li, err, cos)
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
    assert ev["mean_guess_rel_res"] < 1e-2
    net.close()
