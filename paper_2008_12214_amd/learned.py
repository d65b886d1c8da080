"""Learned initialisation: label generation, training and time-to-NMSE evaluation.

The iterative algorithms of the paper start from a random phase
("Iterative Fourier Transform Algorithms" section).  Here a network
predicts the replay-plane phase of a target, the SLM start levels are the
projection of the inverse transform of T e^{i psi}, and a few GS iterations
refine them; plain GS from a random phase stays the reference and the arbiter
of NMSE.  Every step runs in the library's kernels (hg_gs_batched,
hg_replay_phase_init, hg_nn_forward / hg_nn_backward / hg_nn_adam); this
module only sequences the calls and holds the tensors.

    python -m paper_2008_12214_amd.learned --train 4096 --epochs 4 --eval 64

Labels: replay-plane phase after `label_iters` GS iterations (8 levels) from
the quadratic replay-plane start phase psi0, so a label is a function of its
target alone.  The network predicts the residual phase about psi0 (a
translation-equivariant network cannot produce the position-dependent psi0
itself), so its start is psi0 + arg(a + ib) and an all-zero correction is
the quadratic start.  Loss: per-image global-phase-invariant phase error
weighted by the target amplitude.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import _binding as B

# (name, cin, cout) of the fixed network, parameter-vector order
LAYERS = []
_enc = (16, 32, 64, 128)
_cin = 1
for _l, _c in enumerate(_enc):
    LAYERS += [(f"e{_l}a", _cin, _c), (f"e{_l}b", _c, _c)]
    _cin = _c
for _l in range(len(_enc) - 2, -1, -1):
    LAYERS += [(f"d{_l}a", _cin + _enc[_l], _enc[_l]), (f"d{_l}b", _enc[_l], _enc[_l])]
    _cin = _enc[_l]
LAYERS.append(("head", _cin, 2))


def _torch():
    import torch
    return torch


def log(*a):
    print("[learned]", *a, file=sys.stderr, flush=True)


def init_params(seed, device="cuda", head_scale=0.01):
    """He-normal 3x3 weights (bias 0.01); a 1x1 head with small weights and bias
    (1, 0), so the untrained network predicts a near-zero residual phase."""
    torch = _torch()
    rng = np.random.default_rng(seed)
    parts = []
    for name, ci, co in LAYERS:
        if name == "head":
            parts += [rng.standard_normal(co * ci) * head_scale * math.sqrt(1.0 / ci), np.array([1.0, 0.0])]
        else:
            parts += [rng.standard_normal(co * 9 * ci) * math.sqrt(2.0 / (9 * ci)), np.full(co, 0.01)]
    v = np.concatenate(parts).astype(np.float32)
    assert v.size == B.hg_nn_param_count()
    return torch.from_numpy(v).to(device)


WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet512_l8.npy")


def load_params(path=WEIGHTS, device="cuda"):
    """Trained parameters (float32 vector in the library's layout); the default
    file was trained on 20000 512^2 Gaussian-sum targets with 8 phase levels."""
    torch = _torch()
    v = np.load(path, allow_pickle=False).astype(np.float32)
    if v.size != B.hg_nn_param_count():
        raise ValueError(f"{path}: {v.size} parameters, the network has {B.hg_nn_param_count()}")
    return torch.from_numpy(v).to(device)


def learned_start(params, targets, levels=8, workspace=None):
    """SLM start levels from the network: psi0 + arg(network output) for targets [B, n, n]."""
    ws = workspace if workspace is not None else B.hg_nn_workspace(*targets.shape, targets.device)
    out = B.hg_nn_forward(params, targets, ws)
    return B.hg_replay_phase_init(targets, levels, phasor=out, add_quadratic=True)


def make_targets(n, seeds, device="cuda"):
    """Gaussian-sum targets [len(seeds), n, n] float32 on the device."""
    import synth
    torch = _torch()
    out = torch.empty((len(seeds), n, n), dtype=torch.float32, device=device)
    for i, s in enumerate(seeds):
        out[i].copy_(torch.from_numpy(synth.gaussian_target(n, seed=int(s))))
    return out


def make_labels(targets, levels=8, iters=200, chunk=256):
    """Residual replay-plane phasors R e^{-i psi0} (complex64) after `iters` GS
    iterations from the quadratic start, and each run's final NMSE."""
    torch = _torch()
    labels = torch.empty(targets.shape, dtype=torch.complex64, device=targets.device)
    finals = []
    for s in range(0, targets.shape[0], chunk):
        T = targets[s:s + chunk]
        lev0 = B.hg_replay_phase_init(T, levels)
        _, nm, rep = B.hg_gs_batched(list(T), iters, levels, init_levels=list(lev0), want_replay=True)
        res = torch.stack(rep)
        B.hg_quadratic_phase_apply(res, -1)
        labels[s:s + chunk].copy_(res)
        finals.append(torch.stack([x[-1] for x in nm]))
    return labels, torch.cat(finals)


def phase_loss(out, labels, amp):
    """Per-image loss of a head output against residual labels (library kernel)."""
    _, loss = B.hg_nn_phase_loss(out, labels, amp)
    return loss


def train(targets, labels, epochs, batch=16, lr=2e-3, seed=0, params=None, report_s=20.0):
    """Adam with cosine decay; returns (params, per-step mean losses)."""
    torch = _torch()
    dev = targets.device
    n_img, h, w = targets.shape
    params = init_params(seed, dev) if params is None else params
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    ws = B.hg_nn_workspace(batch, h, w, dev)
    g = torch.Generator().manual_seed(seed)
    steps_per_epoch = n_img // batch
    total = epochs * steps_per_epoch
    losses = []
    step = 0
    t0 = last = time.time()
    for ep in range(epochs):
        perm = torch.randperm(n_img, generator=g).to(dev)
        for i in range(steps_per_epoch):
            idx = perm[i * batch:(i + 1) * batch]
            T = targets.index_select(0, idx).contiguous()
            lab = labels.index_select(0, idx).contiguous()
            out = B.hg_nn_forward(params, T, ws)
            grads, loss = B.hg_nn_backward(params, out, lab, T, ws)
            step += 1
            rate = lr * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / total))
            B.hg_nn_adam(params, grads, m, v, step, lr=rate)
            losses.append(loss.mean())
            if time.time() - last > report_s:
                last = time.time()
                log(f"epoch {ep} step {step}/{total} loss {float(losses[-1]):.4f} "
                    f"({(time.time() - t0) / step * 1e3:.1f} ms/step)")
    torch.cuda.synchronize()
    return params, torch.stack(losses).cpu().numpy()


def _time(fn, reps=3):
    """Median device time (ms) of fn() on the current stream, after one warm-up call."""
    torch = _torch()
    fn()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def evaluate(params, targets, levels=8, refine=10, gs_iters=200, seed=7, untrained=None):
    """Time-to-NMSE of the learned start against plain GS from a Philox random phase.

    All paths run batched over the evaluation targets.  Plain GS: per-problem
    NMSE curves over gs_iters iterations and its time model t(k) = a + b k
    (measured at two iteration counts).  Learned path: network forward,
    start levels, `refine` GS iterations, timed as one sequence.  For each
    target, k* is the first GS iteration whose NMSE is at or below the
    learned path's final NMSE; the gain is t_GS(k*) / t_learned.
    """
    torch = _torch()
    K, h, w = targets.shape
    dev = targets.device
    T = list(targets)
    seeds = [seed] * K
    _, nm_gs = B.hg_gs_batched(T, gs_iters, levels, seeds=seeds)
    curves = torch.stack(nm_gs).cpu().numpy()            # [K, gs_iters + 1]
    k1, k2 = 10, 60
    t1 = _time(lambda: B.hg_gs_batched(T, k1, levels, seeds=seeds))
    t2 = _time(lambda: B.hg_gs_batched(T, k2, levels, seeds=seeds))
    slope = (t2 - t1) / (k2 - k1)
    icpt = t1 - slope * k1

    ws = B.hg_nn_workspace(K, h, w, dev)

    def learned(p):
        out = B.hg_nn_forward(p, targets, ws)
        lev0 = B.hg_replay_phase_init(targets, levels, phasor=out, add_quadratic=True)
        return B.hg_gs_batched(T, refine, levels, init_levels=list(lev0))

    def quadratic():
        lev0 = B.hg_replay_phase_init(targets, levels)
        return B.hg_gs_batched(T, refine, levels, init_levels=list(lev0))

    # GS from the quadratic start: the stronger reference for the network
    t_qinit = _time(lambda: B.hg_replay_phase_init(targets, levels))
    lev_q = B.hg_replay_phase_init(targets, levels)
    _, nm_q = B.hg_gs_batched(T, gs_iters, levels, init_levels=list(lev_q))
    curves_q = torch.stack(nm_q).cpu().numpy()

    res = {"targets": K, "size": h, "levels": levels, "refine_iters": refine, "gs_iters": gs_iters,
           "gs_ms_per_iter_batch": slope, "gs_ms_setup_batch": icpt,
           "gs_nmse_median_at": {str(k): float(np.median(curves[:, k])) for k in (10, 50, 100, gs_iters)}}
    t_fwd = _time(lambda: B.hg_nn_forward(params, targets, ws))
    res["forward_ms_batch"] = t_fwd
    res["quadratic_init_ms_batch"] = t_qinit
    res["quadratic_gs_nmse_median_at"] = {str(k): float(np.median(curves_q[:, k])) for k in (10, 50, 100, gs_iters)}
    # how well the phase itself is predicted: network vs zero residual (the quadratic start)
    labels, _ = make_labels(targets, levels)
    out = B.hg_nn_forward(params, targets, ws)
    flat = torch.zeros_like(out)
    flat[..., 0] = 1.0
    res["label_loss_network"] = float(phase_loss(out, labels, targets).mean())
    res["label_loss_quadratic"] = float(phase_loss(flat, labels, targets).mean())
    log(f"held-out label loss: network {res['label_loss_network']:.4f}, "
        f"quadratic start {res['label_loss_quadratic']:.4f}")
    variants = [("learned", lambda: learned(params)), ("quadratic_only", quadratic)]
    if untrained is not None:
        variants.append(("untrained_net", lambda: learned(untrained)))
    for name, fn in variants:
        _, nm = fn()
        final = torch.stack([x[-1] for x in nm]).cpu().numpy()
        t_path = _time(fn)
        kstar, gain = [], []
        for i in range(K):
            hit = np.nonzero(curves[i] <= final[i])[0]
            if hit.size:
                k = int(hit[0])
                kstar.append(k)
                gain.append((icpt + slope * k) / t_path)
            else:
                kstar.append(None)
                gain.append((icpt + slope * gs_iters) / t_path)  # lower bound: GS never got there
        reached = [k is not None for k in kstar]
        kq, gain_q = [], []
        for i in range(K):
            hit = np.nonzero(curves_q[i] <= final[i])[0]
            k = int(hit[0]) if hit.size else gs_iters
            kq.append(k if hit.size else None)
            gain_q.append((t_qinit + icpt + slope * k) / t_path)
        res[name] = {
            "path_ms_batch": t_path,
            "final_nmse_median": float(np.median(final)),
            "gs_final_nmse_median": float(np.median(curves[:, -1])),
            "kstar_median": float(np.median([k for k in kstar if k is not None])) if any(reached) else None,
            "gs_reached_fraction": float(np.mean(reached)),
            "time_gain_median": float(np.median(gain)),
            "win_fraction": float(np.mean(np.array(gain) > 1.0)),
            "quadratic_gs_kstar_median": float(np.median([k for k in kq if k is not None]))
            if any(k is not None for k in kq) else None,
            "quadratic_gs_reached_fraction": float(np.mean([k is not None for k in kq])),
            "time_gain_vs_quadratic_gs_median": float(np.median(gain_q)),
        }
        log(name, json.dumps(res[name]))
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--levels", type=int, default=8)
    ap.add_argument("--train", type=int, default=4096, help="training targets (seeds 100000..)")
    ap.add_argument("--eval", type=int, default=64, help="held-out targets (seeds 900000..)")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--label-iters", type=int, default=200)
    ap.add_argument("--refine", type=int, default=10)
    ap.add_argument("--save", default=None, help="write the trained parameters (.npy)")
    ap.add_argument("--load", default=None, help="skip training and load parameters (.npy)")
    ap.add_argument("--out", default=None, help="write the evaluation as JSON")
    ap.add_argument("--profile", type=int, default=0,
                    help="only run 3 forward + backward passes of the shipped network on this many targets "
                         "(for a kernel trace) and print their times")
    a = ap.parse_args(argv)
    torch = _torch()
    dev = torch.device("cuda:0")
    n = a.size
    if a.profile:
        params = load_params(device=dev)
        T = make_targets(n, range(900000, 900000 + a.profile), dev)
        labels, _ = make_labels(T, a.levels, 20)
        ws = B.hg_nn_workspace(a.profile, n, n, dev)
        fwd = _time(lambda: B.hg_nn_forward(params, T, ws))
        out = B.hg_nn_forward(params, T, ws)
        bwd = _time(lambda: B.hg_nn_backward(params, out, labels, T, ws))
        print(json.dumps({"batch": a.profile, "size": n, "forward_ms": fwd, "backward_ms": bwd,
                          "forward_us_per_image": fwd / a.profile * 1e3}), flush=True)
        return
    t0 = time.time()
    res = {}
    if a.load:
        params = torch.from_numpy(np.load(a.load).astype(np.float32)).to(dev)
    else:
        log(f"targets: {a.train} at {n}^2")
        tr = make_targets(n, range(100000, 100000 + a.train), dev)
        log(f"labels: {a.label_iters} GS iterations, {a.levels} levels ({time.time() - t0:.1f} s)")
        t1 = time.time()
        labels, final = make_labels(tr, a.levels, a.label_iters)
        torch.cuda.synchronize()
        res["label_s"] = time.time() - t1
        res["label_nmse_median"] = float(final.median())
        log(f"labels done in {res['label_s']:.1f} s, median final NMSE {res['label_nmse_median']:.4f}")
        t1 = time.time()
        params, losses = train(tr, labels, a.epochs, a.batch, a.lr)
        res["train_s"] = time.time() - t1
        res["train_steps"] = int(losses.size)
        res["train_ms_per_image"] = res["train_s"] * 1e3 / (losses.size * a.batch)
        res["loss_first"] = float(np.mean(losses[:20]))
        res["loss_last"] = float(np.mean(losses[-20:]))
        log(f"trained {losses.size} steps in {res['train_s']:.1f} s; loss {res['loss_first']:.4f} -> "
            f"{res['loss_last']:.4f}")
        del tr, labels
        if a.save:
            np.save(a.save, params.cpu().numpy())
    ev = make_targets(n, range(900000, 900000 + a.eval), dev)
    res["eval"] = evaluate(params, ev, a.levels, a.refine, untrained=init_params(12345, dev, head_scale=1.0))
    res["total_s"] = time.time() - t0
    line = json.dumps(res)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
