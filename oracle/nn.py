"""Learned-initialisation network in FP64 (oracle; test infrastructure).

The paper has no learned component; this is the layer-local reference for the
network that predicts an initial phase from the target (a project
addition).  Everything is float64 on NHWC arrays (batch, height, width,
channels).  Wherever the GPU stores bfloat16 operands, ``bf16`` rounds to the
nearest bfloat16 (ties to even) so both sides multiply identical values.

Network reading (U-Net encoder-decoder):
  encoder  level l = 0..3 with 16, 32, 64, 128 channels: two 3x3 convolutions
           (zero padding 1) with bias and ReLU, then 2x2 average pooling
           (not after level 3);
  decoder  levels 2, 1, 0: nearest 2x upsampling, concatenation with the
           encoder output of that level (upsampled channels first), two 3x3
           convolutions with ReLU;
  head     1x1 convolution to 2 channels (a, b); the predicted replay-plane
           phase is arg(a + i b).
Weights are OHWI: w[co][ky][kx][ci]; conv(x)[n,y,x,co] =
  bias[co] + sum_{ky,kx,ci} x[n, y+ky-1, x+kx-1, ci] w[co,ky,kx,ci].
Loss (global-phase invariant, per image): 1 - |sum_p a_p z_p conj(e^{i psi_p})| /
sum_p a_p with z_p = (a + i b)/|a + i b| and a_p the target amplitude,
averaged over the images of a batch.
"""
import numpy as np

from . import hologram as _holo
from . import slm as _slm

ENC = (16, 32, 64, 128)


def bf16(x):
    """Round float values to the nearest bfloat16 (ties to even); returns float64."""
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(x32), np.nan, out)


def _pad(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))


def conv3x3(x, w, bias=None):
    """3x3 convolution, zero padding 1 (the definition above, summed tap by tap)."""
    x = np.asarray(x, np.float64)
    n, h, wd, ci = x.shape
    co = w.shape[0]
    xp = _pad(x)
    y = np.zeros((n, h, wd, co))
    for ky in range(3):
        for kx in range(3):
            y += xp[:, ky:ky + h, kx:kx + wd, :] @ w[:, ky, kx, :].T
    if bias is not None:
        y += bias
    return y


def conv3x3_grad_input(dy, w):
    """d loss / d x of conv3x3 given d loss / d y."""
    n, h, wd, co = dy.shape
    ci = w.shape[3]
    dxp = np.zeros((n, h + 2, wd + 2, ci))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + h, kx:kx + wd, :] += dy @ w[:, ky, kx, :]
    return dxp[:, 1:-1, 1:-1, :]


def conv3x3_grad_weight(x, dy):
    """d loss / d w (OHWI) and d loss / d bias of conv3x3."""
    n, h, wd, ci = x.shape
    co = dy.shape[3]
    xp = _pad(x)
    dw = np.zeros((co, 3, 3, ci))
    dyf = dy.reshape(-1, co)
    for ky in range(3):
        for kx in range(3):
            dw[:, ky, kx, :] = dyf.T @ xp[:, ky:ky + h, kx:kx + wd, :].reshape(-1, ci)
    return dw, dyf.sum(axis=0)


def relu(x):
    return np.maximum(x, 0.0)


def avgpool2(x):
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def avgpool2_grad(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) * 0.25


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_grad(dy):
    n, h, w, c = dy.shape
    return dy.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


def layer_shapes(enc=ENC):
    """(name, cin, cout) of every 3x3 layer in order, then the head."""
    shapes = []
    cin = 1
    for l, c in enumerate(enc):
        shapes += [(f"e{l}a", cin, c), (f"e{l}b", c, c)]
        cin = c
    for l in range(len(enc) - 2, -1, -1):
        c = enc[l]
        shapes += [(f"d{l}a", cin + c, c), (f"d{l}b", c, c)]
        cin = c
    shapes.append(("head", cin, 2))
    return shapes


def init_params(rng, enc=ENC):
    """He-normal 3x3 weights (OHWI) with bias 0.01; 1x1 head with bias (1, 0) so
    the predicted phasor a + i b starts away from 0, where its phase is undefined."""
    p = {}
    for name, ci, co in layer_shapes(enc):
        if name == "head":
            p[name + ".w"] = rng.standard_normal((co, 1, 1, ci)) * np.sqrt(1.0 / ci)
            p[name + ".b"] = np.array([1.0, 0.0])
        else:
            p[name + ".w"] = rng.standard_normal((co, 3, 3, ci)) * np.sqrt(2.0 / (9 * ci))
            p[name + ".b"] = np.full(co, 0.01)
    return p


def forward(p, x, enc=ENC, round_bf16=False):
    """Network forward pass.  Returns (head output [n,h,w,2], cache for backward).

    round_bf16 rounds weights and every stored activation to bfloat16 as the
    GPU does (accumulation stays exact float64).
    """
    q = (lambda a: bf16(a)) if round_bf16 else (lambda a: a)
    cache = {"x": q(x)}
    h = cache["x"]
    skips = []
    for l in range(len(enc)):
        for s in "ab":
            name = f"e{l}{s}"
            cache[name + ".in"] = h
            h = q(relu(conv3x3(h, q(p[name + ".w"]), p[name + ".b"])))
            cache[name + ".out"] = h
        if l < len(enc) - 1:
            skips.append(h)
            h = q(avgpool2(h))
    for l in range(len(enc) - 2, -1, -1):
        h = np.concatenate([upsample2(h), skips[l]], axis=3)
        for s in "ab":
            name = f"d{l}{s}"
            cache[name + ".in"] = h
            h = q(relu(conv3x3(h, q(p[name + ".w"]), p[name + ".b"])))
            cache[name + ".out"] = h
    cache["head.in"] = h
    out = h @ q(p["head.w"])[:, 0, 0, :].T + p["head.b"]
    return out, cache


def phase_loss(out, psi, amp):
    """Global-phase-invariant loss and its gradient with respect to out.

    Each image n has its own free global phase, so its loss is
    l_n = 1 - |S_n| / W_n with S_n = sum_p amp z conj(e^{i psi}) and
    W_n = sum_p amp over that image; the batch loss is the mean of l_n.
    Arrays carry the batch as their leading axis.
    """
    a, b = out[..., 0], out[..., 1]
    nb = a.shape[0]
    axes = tuple(range(1, a.ndim))
    r = np.sqrt(a * a + b * b) + 1e-12
    z = (a + 1j * b) / r
    y = np.exp(1j * psi)
    S = np.sum(amp * z * np.conj(y), axis=axes)
    W = np.sum(amp, axis=axes)
    loss = float(np.mean(1.0 - np.abs(S) / W))
    # Near the current point |S_n| = Re(conj(s_hat_n) S_n) with s_hat_n = S_n/|S_n|,
    # so d l_n/d(a, b) = -Re(conj(s_hat_n) amp conj(y) dz/d(a, b)) / W_n.
    shp = (nb,) + (1,) * (a.ndim - 1)
    s_hat = (S / (np.abs(S) + 1e-300)).reshape(shp)
    c = amp * np.conj(s_hat) * np.conj(y)
    # z = (a + ib)/r: dz/da = 1/r - a(a+ib)/r^3, dz/db = i/r - b(a+ib)/r^3
    dz_da = 1.0 / r - a * (a + 1j * b) / r ** 3
    dz_db = 1j / r - b * (a + 1j * b) / r ** 3
    scale = (W * nb).reshape(shp)
    ga = -np.real(c * dz_da) / scale
    gb = -np.real(c * dz_db) / scale
    return loss, np.stack([ga, gb], axis=-1)


def backward(p, cache, dout, enc=ENC, round_bf16=False):
    """Gradients of all parameters given d loss / d head output."""
    q = (lambda a: bf16(a)) if round_bf16 else (lambda a: a)
    g = {}
    hin = cache["head.in"]
    g["head.w"] = (dout.reshape(-1, 2).T @ hin.reshape(-1, hin.shape[3]))[:, None, None, :]
    g["head.b"] = dout.reshape(-1, 2).sum(axis=0)
    dh = q(dout @ q(p["head.w"])[:, 0, 0, :])
    skip_grads = {}
    for l in range(0, len(enc) - 1):
        for s in "ba":
            name = f"d{l}{s}"
            dz = dh * (cache[name + ".out"] > 0)
            g[name + ".w"], g[name + ".b"] = conv3x3_grad_weight(cache[name + ".in"], dz)
            dh = q(conv3x3_grad_input(dz, q(p[name + ".w"])))
        cup = cache[f"d{l}a.in"].shape[3] - enc[l]
        skip_grads[l] = dh[..., cup:]
        dh = q(upsample2_grad(dh[..., :cup]))
    for l in range(len(enc) - 1, -1, -1):
        if l < len(enc) - 1:
            dh = q(avgpool2_grad(dh) + skip_grads[l])
        for s in "ba":
            name = f"e{l}{s}"
            dz = dh * (cache[name + ".out"] > 0)
            g[name + ".w"], g[name + ".b"] = conv3x3_grad_weight(cache[name + ".in"], dz)
            dh = q(conv3x3_grad_input(dz, q(p[name + ".w"])))
    return g


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) of every parameter in place; t starts at 1."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def normalise_input(T):
    """Network input: each target image scaled to unit rms, sum T^2 = H W
    (the same automatic scaling the hologram loops apply); shape [n, h, w, 1]."""
    T = np.asarray(T, np.float64)
    n = T.shape[0]
    hw = T[0].size
    s = np.sqrt(hw / np.sum(T.reshape(n, -1) ** 2, axis=1))
    return (T * s.reshape((n,) + (1,) * (T.ndim - 1)))[..., None]


def quadratic_phase(ny, nx):
    """Deterministic replay-plane start phase for label generation:
    psi0[v][u] = 2 pi ((u - nx/2)^2 / nx + (v - ny/2)^2 / ny), centred indices."""
    u = np.arange(nx) - nx // 2
    v = np.arange(ny) - ny // 2
    return 2.0 * np.pi * ((u[None, :] ** 2 % nx) / nx + (v[:, None] ** 2 % ny) / ny)


def replay_phase_levels(T, phasor, L, add_quadratic=False):
    """SLM start levels from a replay-plane phase: P_L(IDFT(T e^{i psi})),
    psi = arg(phasor) (+ quadratic_phase when add_quadratic).

    phasor is a complex centred array or None (a zero entry, or None, counts
    as phase 0).  Returns (levels, g) with g the field before projection."""
    T = np.asarray(T, np.float64)
    if phasor is None:
        unit = np.ones(T.shape, np.complex128)
    else:
        y = np.asarray(phasor, np.complex128)
        mag = np.abs(y)
        unit = np.where(mag > 0, y / np.where(mag > 0, mag, 1.0), 1.0 + 0j)
    if add_quadratic:
        unit = unit * np.exp(1j * quadratic_phase(*T.shape))
    g = _holo.backward(T * unit)
    _, levels = _slm.project(g, L)
    return levels, g
