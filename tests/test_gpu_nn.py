"""GPU parity of the learned-initialisation network against the FP64 oracle.

Both sides multiply identical bfloat16 operands; the GPU accumulates in FP32,
the oracle exactly in FP64, and both round stored activations to bfloat16
(ties to even).  Tolerances follow from that:
  * a bf16 result may land on either neighbour of the exact value, so it is
    within 2^-8 relative of it (plus a tiny absolute term for FP32
    accumulation near zero);
  * pooling, upsampling and their adjoints add at most four bf16 values,
    which FP32 does exactly: they are compared bit for bit;
  * FP32 results (weight gradients, loss gradient) are within 1e-4 of the
    largest entry of the FP64 value;
  * whole-network outputs and gradients, where bf16 rounding flips
    propagate through later layers, within 2e-3 and 1e-2 relative L2.
"""
import numpy as np
import pytest

import synth
from oracle import nn, slm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2008_12214_amd as hg  # noqa: E402

DEV = "cuda:0"
BF16_REL = 2.0 ** -8


def say(*a):
    print("[gpu-nn]", *a, flush=True)


def bf(a):
    """numpy -> bf16 device tensor (round to nearest even)."""
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV).to(torch.bfloat16)


def f32(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64) if t.dtype == torch.bfloat16 else t.cpu().numpy()


def assert_bf16_close(gpu, ref, what):
    gpu, ref = np.asarray(gpu, np.float64), np.asarray(ref, np.float64)
    tol = BF16_REL * np.abs(ref) + 1e-6 * max(np.max(np.abs(ref)), 1e-30)
    bad = np.abs(gpu - ref) > tol
    changed = np.mean(gpu != nn.bf16(ref))
    say(f"{what}: max err/|ref| {np.max(np.abs(gpu - ref) / (np.abs(ref) + 1e-30)):.2e}, "
        f"bf16 neighbour flips {changed:.2e}")
    assert not bad.any(), f"{what}: {int(bad.sum())} elements outside one bf16 step, first at {np.argwhere(bad)[0]}"


def rng_bf(rng, shape, scale=1.0):
    return nn.bf16(rng.standard_normal(shape) * scale)


CONV_CASES = [  # n, h, w, cin, cout, bias/relu, mask
    # direct-gather kernel (width not a multiple of 16, or cin not of 8)
    (2, 16, 24, 16, 16, True, False),
    (1, 7, 9, 1, 16, True, False),     # first layer: one input channel
    (2, 5, 7, 1, 16, False, True),
    (1, 7, 9, 3, 16, True, False),     # 63 pixels: ragged tail, scalar gather
    (2, 12, 20, 48, 48, False, True),  # three 16-channel groups per wave
    (1, 8, 8, 128, 128, True, False),
    (1, 9, 13, 192, 64, False, False),
    (3, 5, 6, 32, 96, True, True),
    # LDS-tiled kernel: full and partial row/column tiles, every tile shape
    (2, 9, 64, 16, 16, True, False),    # 4 x 64 tiles, ragged last tile row
    (1, 6, 48, 48, 48, False, True),    # 32-wide tiles, partial last column tile
    (2, 5, 128, 96, 32, True, False),   # 2 x 64 tiles
    (1, 4, 32, 192, 64, True, True),    # 2 x 32 tiles
    (1, 3, 16, 128, 128, False, False),  # 4 x 16 tiles
    (1, 7, 80, 64, 64, True, False),
    # channel-chunked kernel (Cin % 32 == 0, width >= 64): 4 x 64 tiles, every
    # output-channel block count, several chunks, ragged tiles, masks
    (1, 6, 64, 192, 64, True, True),
    (2, 9, 130, 32, 48, False, False),
    (1, 4, 64, 64, 16, True, False),
    (1, 5, 96, 128, 32, True, True),
    (1, 5, 72, 48, 16, True, True),     # a half chunk (16 channels) after a whole one
]


@pytest.mark.parametrize("n,h,w,cin,cout,affine,masked", CONV_CASES)
def test_conv3x3_forward(n, h, w, cin, cout, affine, masked):
    say("conv3x3", n, h, w, cin, cout, affine, masked)
    rng = np.random.default_rng(cin * 1000 + cout)
    x = rng_bf(rng, (n, h, w, cin))
    wt = rng.standard_normal((cout, 3, 3, cin)) / np.sqrt(9 * cin)
    b = rng.standard_normal(cout).astype(np.float32).astype(np.float64) if affine else None
    mask = rng_bf(rng, (n, h, w, cout)) if masked else None
    wg = hg.hg_nn_pack_weights(f32(wt))
    y = hg.hg_nn_conv3x3(bf(x), wg, cout, bias=f32(b) if affine else None,
                         mask=bf(mask) if masked else None, relu=affine)
    ref = nn.conv3x3(x, nn.bf16(wt), b)
    if affine:
        ref = nn.relu(ref)
    if masked:
        ref = ref * (mask > 0)
    assert_bf16_close(host(y), ref, "conv3x3")


@pytest.mark.parametrize("n,h,w,cin,cout", [(2, 10, 12, 16, 32), (1, 6, 7, 48, 16), (2, 4, 8, 128, 64),
                                            (2, 6, 64, 48, 16), (1, 5, 32, 192, 64), (1, 5, 64, 16, 64),
                                            (1, 4, 128, 32, 96)])
def test_conv3x3_data_gradient(n, h, w, cin, cout):
    say("conv3x3 data gradient", n, h, w, cin, cout)
    rng = np.random.default_rng(7 + cin)
    dy = rng_bf(rng, (n, h, w, cout))
    wt = rng.standard_normal((cout, 3, 3, cin)) / np.sqrt(9 * cin)
    mask = rng_bf(rng, (n, h, w, cin))
    wg = hg.hg_nn_pack_weights(f32(wt), flip=True)
    dx = hg.hg_nn_conv3x3(bf(dy), wg, cin, mask=bf(mask))
    ref = nn.conv3x3_grad_input(dy, nn.bf16(wt)) * (mask > 0)
    assert_bf16_close(host(dx), ref, "conv3x3 data gradient")


@pytest.mark.parametrize("n,h,w,cin,cout", [(2, 16, 24, 16, 16), (1, 7, 9, 1, 16), (2, 12, 20, 48, 48),
                                            (1, 8, 8, 128, 128), (4, 64, 64, 16, 32),
                                            # odd heights, partial 64-wide tiles, several images
                                            (3, 7, 70, 32, 64), (2, 9, 130, 64, 16)])
def test_conv3x3_weight_gradient(n, h, w, cin, cout):
    say("conv3x3 weight gradient", n, h, w, cin, cout)
    rng = np.random.default_rng(11 + cout)
    x = rng_bf(rng, (n, h, w, cin))
    dy = rng_bf(rng, (n, h, w, cout))
    dw, db = hg.hg_nn_conv3x3_wgrad(bf(x), bf(dy))
    rdw, rdb = nn.conv3x3_grad_weight(x, dy)
    for g, r, what in ((host(dw), rdw, "dw"), (host(db), rdb, "db")):
        err = np.max(np.abs(g - r)) / np.max(np.abs(r))
        say(f"  {what}: max err / max |ref| = {err:.2e}")
        assert err < 1e-4, what


@pytest.mark.parametrize("c1,c2", [(32, 16), (20, 12)])  # 16-byte and scalar kernels
def test_pool_upsample_and_adjoints_bit_exact(c1, c2):
    say("pool / upsample / adjoints", c1, c2)
    rng = np.random.default_rng(21)
    n, h, w = 2, 12, 20
    x = rng_bf(rng, (n, h, w, c2))
    np.testing.assert_array_equal(host(hg.hg_nn_avgpool2(bf(x))), nn.bf16(nn.avgpool2(x)))
    dy = rng_bf(rng, (n, h // 2, w // 2, c2))
    dskip = rng_bf(rng, (n, h, w, c2))
    mask = rng_bf(rng, (n, h, w, c2))
    got = host(hg.hg_nn_avgpool2_backward(bf(dy), bf(dskip), bf(mask)))
    np.testing.assert_array_equal(got, nn.bf16(nn.avgpool2_grad(dy) + dskip) * (mask > 0))
    np.testing.assert_array_equal(host(hg.hg_nn_avgpool2_backward(bf(dy))), nn.bf16(nn.avgpool2_grad(dy)))
    lo = rng_bf(rng, (n, h // 2, w // 2, c1))
    np.testing.assert_array_equal(host(hg.hg_nn_upsample_concat(bf(lo), bf(x))),
                                  np.concatenate([nn.upsample2(lo), x], axis=3))
    dcat = rng_bf(rng, (n, h, w, c1 + c2))
    mlo = rng_bf(rng, (n, h // 2, w // 2, c1))
    dlo, dsk = hg.hg_nn_upsample_concat_backward(bf(dcat), c1, mask_lo=bf(mlo))
    np.testing.assert_array_equal(host(dlo), nn.bf16(nn.upsample2_grad(dcat[..., :c1])) * (mlo > 0))
    np.testing.assert_array_equal(host(dsk), dcat[..., c1:])


@pytest.mark.parametrize("c", [16, 12])  # 16-channel kernels and the generic ones
def test_head_loss_and_head_backward(c):
    say("head / loss / head backward", c)
    rng = np.random.default_rng(31)
    n, h, w = 3, 16, 8
    x = nn.bf16(np.maximum(rng.standard_normal((n, h, w, c)), 0))
    wt = rng.standard_normal((2, 1, 1, c)) * 0.3
    b = np.array([0.5, -0.25])
    out = hg.hg_nn_head(bf(x), f32(wt[:, 0, 0, :]), f32(b))
    ref_out = x @ nn.bf16(wt)[:, 0, 0, :].T + b
    got_out = host(out)
    assert np.max(np.abs(got_out - ref_out)) < 1e-5 * np.max(np.abs(ref_out))
    psi = rng.uniform(-np.pi, np.pi, (n, h, w))
    amp = rng.random((n, h, w)).astype(np.float32).astype(np.float64)
    label = (np.exp(1j * psi) * rng.uniform(0.5, 2.0, (n, h, w))).astype(np.complex64)
    dout, loss = hg.hg_nn_phase_loss(out, torch.from_numpy(label).to(DEV), f32(amp))
    # the oracle sees the GPU's own head output and the label's float32 phase
    rl, rd = nn.phase_loss(got_out.astype(np.float64), np.angle(label.astype(np.complex128)), amp)
    gl, gd = host(loss), host(dout)
    say(f"  loss gpu {np.mean(gl):.8f} oracle {rl:.8f}")
    assert abs(np.mean(gl) - rl) < 1e-5
    assert np.max(np.abs(gd - rd)) < 1e-4 * np.max(np.abs(rd))
    dx, dwb = hg.hg_nn_head_backward(dout, f32(wt[:, 0, 0, :]), bf(x))
    rdx = (gd.astype(np.float64) @ nn.bf16(wt)[:, 0, 0, :]) * (x > 0)
    assert_bf16_close(host(dx), rdx, "head data gradient")
    rdw = gd.reshape(-1, 2).T.astype(np.float64) @ x.reshape(-1, c)
    rdb = gd.reshape(-1, 2).sum(axis=0)
    g = host(dwb)
    assert np.max(np.abs(g[:2 * c] - rdw.ravel())) < 1e-4 * np.max(np.abs(rdw))
    assert np.max(np.abs(g[2 * c:] - rdb)) < 1e-4 * max(np.max(np.abs(rdb)), 1e-3)


def _flat(p):
    return np.concatenate([np.concatenate([p[name + ".w"].ravel(), p[name + ".b"].ravel()])
                           for name, _, _ in nn.layer_shapes()])


def _unflat(v):
    g, off = {}, 0
    for name, ci, co in nn.layer_shapes():
        k = 1 if name == "head" else 3
        nw = co * k * k * ci
        g[name + ".w"] = v[off:off + nw].reshape(co, k, k, ci)
        off += nw
        g[name + ".b"] = v[off:off + co]
        off += co
    assert off == v.size
    return g


def test_param_layout_matches_oracle():
    assert hg.hg_nn_param_count() == _flat(nn.init_params(np.random.default_rng(0))).size


@pytest.mark.parametrize("n,h,w", [(2, 32, 48), (1, 64, 64)])
def test_network_forward_backward(n, h, w):
    say("network forward/backward", n, h, w)
    rng = np.random.default_rng(41 + h)
    p = nn.init_params(rng)
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    T = np.stack([synth.gaussian_target(max(h, w), seed=5 + i)[:h, :w] for i in range(n)]).astype(np.float32)
    psi = rng.uniform(-np.pi, np.pi, (n, h, w))
    label = np.exp(1j * psi).astype(np.complex64)
    params = f32(_flat(p))
    ws = hg.hg_nn_workspace(n, h, w, DEV)
    out = hg.hg_nn_forward(params, f32(T), ws)
    grads, loss = hg.hg_nn_backward(params, out, torch.from_numpy(label).to(DEV), f32(T), ws)
    x = nn.normalise_input(T.astype(np.float64))
    ref_out, cache = nn.forward(p, x, round_bf16=True)
    got_out = host(out)
    e = np.linalg.norm(got_out - ref_out) / np.linalg.norm(ref_out)
    say(f"  head output rel L2 {e:.2e}")
    assert e < 2e-3
    # backward from the GPU's own head output so both sides see the same dout
    rl, dout = nn.phase_loss(got_out.astype(np.float64), np.angle(label.astype(np.complex128)),
                             T.astype(np.float64))
    assert abs(float(np.mean(host(loss))) - rl) < 1e-5
    ref_g = nn.backward(p, cache, dout, round_bf16=True)
    got_g = _unflat(host(grads).astype(np.float64))
    worst = 0.0
    for k in ref_g:
        r = np.asarray(ref_g[k], np.float64)
        err = np.linalg.norm(got_g[k] - r) / max(np.linalg.norm(r), 1e-30)
        worst = max(worst, err)
        assert err < 1e-2, (k, err)
    say(f"  worst gradient rel L2 {worst:.2e}")


def test_adam_matches_oracle():
    say("adam")
    rng = np.random.default_rng(51)
    n = 1000
    p = {"a": rng.standard_normal(n).astype(np.float32).astype(np.float64)}
    m = {"a": np.zeros(n)}
    v = {"a": np.zeros(n)}
    tp, tm, tv = f32(p["a"]), f32(m["a"]), f32(v["a"])
    for t in range(1, 6):
        g = rng.standard_normal(n).astype(np.float32).astype(np.float64)
        nn.adam_step(p, {"a": g}, m, v, t, lr=1e-2)
        hg.hg_nn_adam(tp, f32(g), tm, tv, t, lr=1e-2)
    np.testing.assert_allclose(host(tp), p["a"], rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("mode", ["phasor", "quadratic", "residual"])
def test_replay_phase_init_levels(mode):
    say("replay-phase start levels, mode =", mode)
    rng = np.random.default_rng(61)
    b, ny, nx, L = 2, 64, 128, 8
    T = np.stack([synth.gaussian_target(128, seed=9 + i)[:ny, :nx] for i in range(b)]).astype(np.float32)
    ph = (rng.standard_normal((b, ny, nx)) + 1j * rng.standard_normal((b, ny, nx))).astype(np.complex64)
    if mode == "quadratic":
        lev = hg.hg_replay_phase_init(f32(T), L)
    elif mode == "phasor":
        lev = hg.hg_replay_phase_init(f32(T), L, phasor=torch.from_numpy(ph).to(DEV))
    else:
        lev = hg.hg_replay_phase_init(f32(T), L, phasor=torch.from_numpy(ph).to(DEV), add_quadratic=True)
    got = host(lev)
    for i in range(b):
        ref, g = nn.replay_phase_levels(T[i].astype(np.float64), None if mode == "quadratic" else ph[i], L,
                                        add_quadratic=mode != "phasor")
        mism = got[i].astype(np.int64) != ref
        margin = slm.boundary_margin(g, L)
        # FP32 transform error relative to the local |g|: exempt pixels near a
        # decision boundary (angular margin below 1e-3 rad) and report them
        bad = mism & (margin >= 1e-3)
        say(f"  image {i}: {int(mism.sum())} mismatches, {int((mism & (margin < 1e-3)).sum())} exempt")
        assert not bad.any()


def test_quadratic_phase_apply():
    say("quadratic phase apply")
    rng = np.random.default_rng(65)
    f = (rng.standard_normal((2, 64, 256)) + 1j * rng.standard_normal((2, 64, 256))).astype(np.complex64)
    q = np.exp(1j * nn.quadratic_phase(64, 256))
    for sign in (1, -1):
        got = host(hg.hg_quadratic_phase_apply(torch.from_numpy(f).to(DEV), sign))
        ref = f.astype(np.complex128) * (q if sign > 0 else np.conj(q))
        assert np.max(np.abs(got - ref)) < 1e-5 * np.max(np.abs(ref))


def test_batched_gs_with_start_levels_and_replay():
    say("batched GS with start levels and replay output")
    rng = np.random.default_rng(71)
    n, L, iters = 128, 8, 5
    Ts = [f32(synth.gaussian_target(n, seed=20 + i)) for i in range(3)]
    inits = [torch.from_numpy(rng.integers(0, L, (n, n)).astype(np.uint8)).to(DEV) for _ in range(3)]
    levs, nms, reps = hg.hg_gs_batched(Ts, iters, L, init_levels=inits, want_replay=True)
    for i in range(3):
        out = hg.hg_gs(Ts[i], iters, L, init_levels=inits[i], want_replay=True)
        np.testing.assert_array_equal(host(levs[i]), host(out["levels"]))
        np.testing.assert_allclose(host(nms[i]), host(out["nmse"]), rtol=1e-9)
        np.testing.assert_allclose(host(reps[i]), host(out["replay"]), rtol=0, atol=1e-5)
