"""Pins of the FP64 convolution oracle (oracle/conv.py): forward against a
brute-force loop over output points, input and weight gradients against
central finite differences, and the network gradient likewise."""
import itertools

import numpy as np
import pytest

from oracle import conv


def brute(x, w, mode):
    n, G = x.shape[0], x.shape[1]
    Go = conv.out_size(G, mode)
    out = np.zeros((n, Go, Go, Go, w.shape[0]))
    for b, pz, py, px in itertools.product(range(n), range(Go), range(Go), range(Go)):
        for dz, dy, dx in itertools.product(range(3), repeat=3):
            src = []
            for P, d in ((pz, dz), (py, dy), (px, dx)):
                if mode == "s1":
                    src.append(P + d - 1)
                elif mode == "s2":
                    src.append(2 * P + d - 1)
                else:
                    t = P + 1 - d
                    src.append(t // 2 if t % 2 == 0 else -1)
            if all(0 <= s < G for s in src):
                out[b, pz, py, px] += w[:, dx + 3 * dy + 9 * dz, :] @ x[b, src[0], src[1], src[2]]
    return out


@pytest.mark.parametrize("mode,G", [("s1", 4), ("s2", 5), ("t2", 3)])
def test_forward_against_brute_force(mode, G):
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, G, G, G, 3))
    w = rng.standard_normal((4, 27, 3))
    assert np.allclose(conv.conv3d(x, w, mode), brute(x, w, mode), atol=1e-12)


def test_sizes():
    assert [conv.out_size(65, "s2"), conv.out_size(33, "s2"), conv.out_size(17, "s2")] == [33, 17, 9]
    assert [conv.out_size(9, "t2"), conv.out_size(17, "t2"), conv.out_size(33, "t2")] == [17, 33, 65]


@pytest.mark.parametrize("mode,G", [("s1", 4), ("s2", 5), ("t2", 3)])
def test_gradients_against_finite_differences(mode, G):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, G, G, G, 2))
    w = rng.standard_normal((3, 27, 2))
    Go = conv.out_size(G, mode)
    gy = rng.standard_normal((1, Go, Go, Go, 3))

    def L(xx, ww):
        return float(np.sum(conv.conv3d(xx, ww, mode) * gy))

    gx = conv.conv3d_input_grad(gy, w, mode, G)
    gw = conv.conv3d_weight_grad(gy, x, mode)
    eps = 1e-6
    for idx in [tuple(rng.integers(0, s) for s in x.shape) for _ in range(12)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        fd = (L(xp, w) - L(xm, w)) / (2 * eps)
        assert abs(fd - gx[idx]) <= 1e-7 * max(1.0, abs(fd))
    for idx in [tuple(rng.integers(0, s) for s in w.shape) for _ in range(12)]:
        wp, wm = w.copy(), w.copy()
        wp[idx] += eps
        wm[idx] -= eps
        fd = (L(x, wp) - L(x, wm)) / (2 * eps)
        assert abs(fd - gw[idx]) <= 1e-7 * max(1.0, abs(fd))


def test_adjoint_identities():
    """<conv(x, w), y> = <x, input_grad(y, w)> for each tap pattern."""
    rng = np.random.default_rng(2)
    for mode, G in (("s1", 5), ("s2", 7), ("t2", 4)):
        x = rng.standard_normal((1, G, G, G, 2))
        w = rng.standard_normal((3, 27, 2))
        Go = conv.out_size(G, mode)
        y = rng.standard_normal((1, Go, Go, Go, 3))
        lhs = np.sum(conv.conv3d(x, w, mode) * y)
        rhs = np.sum(x * conv.conv3d_input_grad(y, w, mode, G))
        assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def small_params(rng, scale=0.3):
    return [(rng.standard_normal((co, 27, ci)) * scale / np.sqrt(27 * ci), rng.standard_normal(co) * 0.05)
            for ci, co, *_ in conv.LAYERS]


def test_network_gradient_against_finite_differences():
    rng = np.random.default_rng(3)
    G = 9
    params = small_params(rng, scale=1.0)
    mask = np.zeros((G, G, G), bool)
    mask[0], mask[-1], mask[:, 0], mask[:, -1], mask[:, :, 0], mask[:, :, -1] = (True,) * 6
    g = rng.uniform(0, 1, (G, G, G))
    x = conv.net_input(g, mask)[None]
    target = rng.uniform(0, 1, (1, G, G, G))
    interior = (~mask)[None].astype(float)
    grads = conv.net_grads(params, x, target, interior)
    eps = 1e-6
    for li in (0, 4, 8, 12, 13):
        w, b = params[li]
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in w.shape)
            wp = [(ww.copy(), bb) for ww, bb in params]
            wm = [(ww.copy(), bb) for ww, bb in params]
            wp[li][0][idx] += eps
            wm[li][0][idx] -= eps
            fd = (conv.net_loss(wp, x, target, interior)[0] - conv.net_loss(wm, x, target, interior)[0]) / (2 * eps)
            assert abs(fd - grads[li][0][idx]) <= 1e-6 * max(1e-3, abs(fd)), (li, idx)
        o = int(rng.integers(0, b.shape[0]))
        bp = [(ww, bb.copy()) for ww, bb in params]
        bm = [(ww, bb.copy()) for ww, bb in params]
        bp[li][1][o] += eps
        bm[li][1][o] -= eps
        fd = (conv.net_loss(bp, x, target, interior)[0] - conv.net_loss(bm, x, target, interior)[0]) / (2 * eps)
        assert abs(fd - grads[li][1][o]) <= 1e-6 * max(1e-3, abs(fd))


def test_energy_loss_gradient_against_finite_differences():
    """The energy-norm loss e^T A e (A the assembled 8^3 stiffness matrix of
    the oracle) through the whole network: its chain-rule gradient, whose
    output term 2 A e rests on the symmetry of A, against central differences."""
    import oracle
    rng = np.random.default_rng(4)
    G = 9
    A = oracle.assemble(G - 1, G - 1, G - 1)
    apply_a = lambda v: oracle.csr_spmv(A, v)
    params = small_params(rng, scale=1.0)
    mask = np.zeros((G, G, G), bool)
    mask[0], mask[-1], mask[:, 0], mask[:, -1], mask[:, :, 0], mask[:, :, -1] = (True,) * 6
    g = rng.uniform(0, 1, (G, G, G))
    x = conv.net_input(g, mask)[None]
    target = rng.uniform(0, 1, (1, G, G, G))
    interior = (~mask)[None].astype(float)
    loss = conv.net_loss(params, x, target, interior, apply_a=apply_a)[0]
    assert loss > 0.0
    grads = conv.net_grads(params, x, target, interior, apply_a=apply_a)
    eps = 1e-6
    for li in (0, 8, 13):
        w, b = params[li]
        for _ in range(2):
            idx = tuple(rng.integers(0, s) for s in w.shape)
            wp = [(ww.copy(), bb) for ww, bb in params]
            wm = [(ww.copy(), bb) for ww, bb in params]
            wp[li][0][idx] += eps
            wm[li][0][idx] -= eps
            fd = (conv.net_loss(wp, x, target, interior, apply_a=apply_a)[0]
                  - conv.net_loss(wm, x, target, interior, apply_a=apply_a)[0]) / (2 * eps)
            assert abs(fd - grads[li][0][idx]) <= 1e-6 * max(1e-3, abs(fd)), (li, idx)
        o = int(rng.integers(0, b.shape[0]))
        bp = [(ww, bb.copy()) for ww, bb in params]
        bm = [(ww, bb.copy()) for ww, bb in params]
        bp[li][1][o] += eps
        bm[li][1][o] -= eps
        fd = (conv.net_loss(bp, x, target, interior, apply_a=apply_a)[0]
              - conv.net_loss(bm, x, target, interior, apply_a=apply_a)[0]) / (2 * eps)
        assert abs(fd - grads[li][1][o]) <= 1e-6 * max(1e-3, abs(fd))


def test_bf16_rounding():
    # spacing 2^-7 at 1: 1 + 2^-8 is a tie (to the even 1.0), 1 + 3 2^-8 a tie (to the even 1 + 2^-6)
    v = np.array([1.0, 1.00390625, 1.001953125, -3.14159, 1e-20, 65504.0, 1.01171875])
    r = conv.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 and r[6] == 1.015625
    assert abs(r[3] + 3.140625) < 1e-12
    assert np.all(np.abs(r - v) <= np.abs(v) * 2 ** -8 + 1e-38)


def test_adam_constant_gradient_closed_form():
    """Adam from m = v = 0 with a constant gradient g: m_t = (1 - beta1^t) g
    and v_t = (1 - beta2^t) g^2, so the bias-corrected moments are g and g^2
    and every step moves p by -lr g / (|g| + eps), exactly in real
    arithmetic.  A large eps (0.5) separates eps outside the square root
    from eps inside it; a missing bias correction, swapped betas or a wrong
    sign change the step."""
    rng = np.random.default_rng(3)
    g = rng.standard_normal(1000).astype(np.float32)
    p0 = rng.standard_normal(1000).astype(np.float32)
    lr, eps = 0.01, 0.5
    p, m, v = p0, np.zeros(1000, np.float32), np.zeros(1000, np.float32)
    for t in range(1, 6):
        p, m, v = conv.adam_step(p, m, v, g, t, lr, 0.9, 0.999, eps)
        expect = p0.astype(np.float64) - t * lr * g / (np.abs(g) + eps)
        assert np.all(np.abs(p - expect) <= 1e-6 * (np.abs(expect) + t * lr)), t
    assert p.dtype == np.float32


def test_adam_without_moment_memory_is_a_scaled_sign_step():
    """With beta1 = beta2 = 0 nothing is remembered: each step moves p by
    -lr g_t / (|g_t| + eps) for that step's own gradient."""
    rng = np.random.default_rng(4)
    p = rng.standard_normal(500).astype(np.float32)
    m, v = np.zeros(500, np.float32), np.zeros(500, np.float32)
    lr, eps = 0.1, 0.25
    for t in range(1, 4):
        g = rng.standard_normal(500).astype(np.float32)
        expect = p.astype(np.float64) - lr * g / (np.abs(g) + eps)
        p, m, v = conv.adam_step(p, m, v, g, t, lr, 0.0, 0.0, eps)
        assert np.all(np.abs(p - expect) <= 1e-6 * (np.abs(expect) + lr))


@pytest.mark.parametrize("energy", [False, True])
def test_bf16_network_gradient_structure_and_closeness(energy):
    """The bfloat16-emulated network gradient (net_grads_bf16): with its
    roundings dropped it is the FP64 chain rule (net_grads, pinned by finite
    differences above) to rounding, so its skip shares, ReLU masks and
    accumulation order are those of the definition; with them it stays
    within 15 % relative L2 and cosine 0.99 of the FP64 gradient on the same
    bf16 weights (bfloat16 activations move some ReLU masks), and every
    entry is bounded by its sum of absolute terms."""
    import oracle
    rng = np.random.default_rng(6)
    G = 9
    params = [(rng.standard_normal((co, 27, ci)) * np.sqrt(2.0 / (27 * ci)), rng.standard_normal(co) * 0.01)
              for ci, co, *_ in conv.LAYERS]
    pb = [(conv.bf16(w), b) for w, b in params]
    mask = np.zeros((G, G, G), bool)
    mask[0], mask[-1], mask[:, 0], mask[:, -1], mask[:, :, 0], mask[:, :, -1] = (True,) * 6
    g = rng.uniform(0, 1, (2, G, G, G))
    target = rng.uniform(0, 1, (2, G, G, G))
    x = np.stack([conv.net_input(g[i], mask) for i in range(2)])
    interior = np.broadcast_to(~mask, (2, G, G, G)).astype(float)
    apply_a = None
    if energy:
        A = oracle.assemble(G - 1, G - 1, G - 1)
        apply_a = lambda v: oracle.csr_spmv(A, v)
    exact = conv.net_grads(params, x, target, interior, apply_a=apply_a)
    plain, _ = conv.net_grads_bf16(params, x, target, interior, apply_a=apply_a, rounded=False)
    for (gw, gb), (rw, rb) in zip(plain, exact):
        assert np.allclose(gw, rw, rtol=1e-12, atol=1e-14 * np.abs(rw).max())
        assert np.allclose(gb, rb, rtol=1e-12, atol=1e-14 * np.abs(rb).max())
    ref = conv.net_grads(pb, x, target, interior, apply_a=apply_a)
    got, scales = conv.net_grads_bf16(params, x, target, interior, apply_a=apply_a)
    for li, ((gw, gb), (rw, rb)) in enumerate(zip(got, ref)):
        a, r = np.concatenate([gw.ravel(), gb]), np.concatenate([rw.ravel(), rb])
        err = np.linalg.norm(a - r) / np.linalg.norm(r)
        cos = float(a @ r / (np.linalg.norm(a) * np.linalg.norm(r)))
        assert err <= 0.15 and cos >= 0.99, (li, err, cos)
    for (gw, gb), (sw, sb) in zip(got, scales):
        assert np.all(np.abs(gw) <= sw * (1 + 1e-12)) and np.all(np.abs(gb) <= sb * (1 + 1e-12))
