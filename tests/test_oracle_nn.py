"""Pins for the learned-initialisation oracle (oracle/nn.py).

Independent references: PyTorch CPU float64 convolution and autograd,
PyTorch's bfloat16 cast and Adam, adjointness identities, and central
finite differences of the whole network loss.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import nn  # noqa: E402


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a))


def test_bf16_matches_torch_cast():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-8, 8, 10000),
                        [0.0, -0.0, 1.0, 65504.0, 1e-40, 3.0e38]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(nn.bf16(x), ref)


def test_conv3x3_matches_torch():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 7, 9, 5))
    w = rng.standard_normal((6, 3, 3, 5))
    b = rng.standard_normal(6)
    ref = torch.nn.functional.conv2d(_t(x).permute(0, 3, 1, 2), _t(w).permute(0, 3, 1, 2), _t(b), padding=1)
    np.testing.assert_allclose(nn.conv3x3(x, w, b), ref.permute(0, 2, 3, 1).numpy(), atol=1e-12)


def test_conv3x3_gradients_match_autograd():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 6, 5, 4))
    w = rng.standard_normal((3, 3, 3, 4))
    dy = rng.standard_normal((2, 6, 5, 3))
    xt = _t(x).permute(0, 3, 1, 2).requires_grad_(True)
    wt = _t(w).permute(0, 3, 1, 2).requires_grad_(True)
    bt = torch.zeros(3, dtype=torch.float64, requires_grad=True)
    y = torch.nn.functional.conv2d(xt, wt, bt, padding=1)
    y.backward(_t(dy).permute(0, 3, 1, 2))
    np.testing.assert_allclose(nn.conv3x3_grad_input(dy, w), xt.grad.permute(0, 2, 3, 1).numpy(), atol=1e-12)
    dw, db = nn.conv3x3_grad_weight(x, dy)
    np.testing.assert_allclose(dw, wt.grad.permute(0, 2, 3, 1).numpy(), atol=1e-12)
    np.testing.assert_allclose(db, bt.grad.numpy(), atol=1e-12)


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 8, 6, 3))
    y = rng.standard_normal((1, 4, 3, 3))
    assert np.sum(nn.avgpool2(x) * y) == pytest.approx(np.sum(x * nn.avgpool2_grad(y)), rel=1e-12)
    assert np.sum(nn.upsample2(y) * x) == pytest.approx(np.sum(y * nn.upsample2_grad(x)), rel=1e-12)


def test_loss_invariant_to_global_phase_and_zero_when_exact():
    rng = np.random.default_rng(4)
    psi = rng.uniform(-np.pi, np.pi, (1, 4, 4))
    amp = rng.random((1, 4, 4))
    out = np.stack([np.cos(psi + 0.7), np.sin(psi + 0.7)], axis=-1) * 3.0
    loss, _ = nn.phase_loss(out, psi, amp)
    assert abs(loss) < 1e-12


def test_batch_loss_is_mean_of_image_losses():
    rng = np.random.default_rng(7)
    out = rng.standard_normal((2, 5, 6, 2))
    psi = rng.uniform(-np.pi, np.pi, (2, 5, 6))
    amp = rng.random((2, 5, 6))
    lb, gb = nn.phase_loss(out, psi, amp)
    l0, g0 = nn.phase_loss(out[:1], psi[:1], amp[:1])
    l1, g1 = nn.phase_loss(out[1:], psi[1:], amp[1:])
    assert lb == pytest.approx(0.5 * (l0 + l1), rel=1e-14)
    np.testing.assert_allclose(gb, 0.5 * np.concatenate([g0, g1]), rtol=1e-13, atol=1e-16)
    # a separate global phase per image leaves the loss at zero
    ph = np.array([0.3, -2.0])[:, None, None]
    exact = np.stack([np.cos(psi + ph), np.sin(psi + ph)], axis=-1) * 2.0
    assert abs(nn.phase_loss(exact, psi, amp)[0]) < 1e-12


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(5)
    enc = (3, 4, 5)
    p = nn.init_params(rng, enc)
    x = rng.random((2, 8, 8, 1))
    psi = rng.uniform(-np.pi, np.pi, (2, 8, 8))
    amp = rng.random((2, 8, 8)) + 0.1
    out, cache = nn.forward(p, x, enc)
    loss, dout = nn.phase_loss(out, psi, amp)
    g = nn.backward(p, cache, dout, enc)
    h = 1e-6
    for name in ["e0a.w", "e1b.w", "e2a.b", "d0a.w", "d1b.w", "head.w", "head.b"]:
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = nn.phase_loss(nn.forward(p, x, enc)[0], psi, amp)
            flat[idx] = old - h
            lm, _ = nn.phase_loss(nn.forward(p, x, enc)[0], psi, amp)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (name, idx, fd, an)


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    p = {"a": rng.standard_normal(5)}
    m = {"a": np.zeros(5)}
    v = {"a": np.zeros(5)}
    pt = torch.nn.Parameter(_t(p["a"].copy()))
    opt = torch.optim.Adam([pt], lr=1e-2)
    for t in range(1, 4):
        g = rng.standard_normal(5)
        nn.adam_step(p, {"a": g}, m, v, t, lr=1e-2)
        opt.zero_grad()
        pt.grad = _t(g)
        opt.step()
    np.testing.assert_allclose(p["a"], pt.detach().numpy(), rtol=1e-12, atol=1e-12)


def test_normalise_input_unit_rms():
    rng = np.random.default_rng(8)
    T = rng.random((3, 6, 10)) * np.array([1.0, 5.0, 0.01])[:, None, None]
    x = nn.normalise_input(T)
    assert x.shape == (3, 6, 10, 1)
    np.testing.assert_allclose(np.mean(x[..., 0] ** 2, axis=(1, 2)), 1.0, rtol=1e-13)
    np.testing.assert_allclose(x[1, ..., 0] / x[1, 0, 0, 0], T[1] / T[1, 0, 0], rtol=1e-13)


def test_quadratic_phase_values():
    ny, nx = 8, 16
    psi = nn.quadratic_phase(ny, nx)
    for v, u in [(0, 0), (4, 8), (7, 3), (1, 15)]:
        ref = 2 * np.pi * ((u - 8) ** 2 / 16 + (v - 4) ** 2 / 8)
        assert np.exp(1j * psi[v, u]) == pytest.approx(np.exp(1j * ref), abs=1e-12)
    assert psi[4, 8] == 0.0


def test_replay_phase_levels_recovers_consistent_hologram():
    # If the replay phase is that of a quantised hologram whose replay
    # amplitude is the target, the inverse transform returns that hologram.
    from oracle import hologram, slm
    rng = np.random.default_rng(9)
    L = 8
    lev = rng.integers(0, L, (16, 16))
    R = hologram.forward(slm.level_phasor(lev, L))
    got, g = nn.replay_phase_levels(np.abs(R), R * 3.7, L)
    np.testing.assert_array_equal(got, lev)
    np.testing.assert_allclose(g, slm.level_phasor(lev, L), atol=1e-12)


def test_replay_phase_levels_quadratic_residual():
    # a residual phase about the quadratic phase plus add_quadratic is the
    # same start as the full phase
    rng = np.random.default_rng(10)
    T = rng.random((16, 32))
    psi = rng.uniform(-np.pi, np.pi, (16, 32))
    full, g1 = nn.replay_phase_levels(T, np.exp(1j * psi), 8)
    res, g2 = nn.replay_phase_levels(T, np.exp(1j * (psi - nn.quadratic_phase(16, 32))), 8, add_quadratic=True)
    np.testing.assert_allclose(g2, g1, atol=1e-12)
    q, _ = nn.replay_phase_levels(T, None, 8, add_quadratic=True)
    q2, _ = nn.replay_phase_levels(T, np.exp(1j * nn.quadratic_phase(16, 32)), 8)
    np.testing.assert_array_equal(q, q2)
