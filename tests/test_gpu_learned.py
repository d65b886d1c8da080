"""What the trained network gains (GPU).

The committed weights were trained on the GPU with the library's own
forward / backward kernels (20000 Gaussian-sum targets at 512^2, 8 phase
levels).  On held-out targets the network's start must beat the same start
without the network (the quadratic replay phase it is a residual on): a
lower phase loss against the GS-converged replay phase, and a lower NMSE
after the same 10 GS iterations.  Plain GS from a random phase must not
reach that NMSE in the same 10 iterations.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2008_12214_amd as hg  # noqa: E402
from paper_2008_12214_amd import learned  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print("[gpu-learned]", *a, flush=True)


def test_trained_network_beats_its_start_without_it():
    n, K, levels, refine = 512, 8, 8, 10
    say("held-out targets", K, "at", n)
    T = learned.make_targets(n, range(900100, 900100 + K), DEV)
    params = learned.load_params(device=DEV)
    labels, _ = learned.make_labels(T, levels, iters=200)
    ws = hg.hg_nn_workspace(K, n, n, DEV)
    out = hg.hg_nn_forward(params, T, ws)
    flat = torch.zeros_like(out)
    flat[..., 0] = 1.0
    loss_net = float(learned.phase_loss(out, labels, T).mean())
    loss_quad = float(learned.phase_loss(flat, labels, T).mean())
    say(f"phase loss: network {loss_net:.4f}, quadratic start {loss_quad:.4f}")
    assert loss_net < loss_quad - 0.005

    def final_nmse(start):
        _, nm = hg.hg_gs_batched(list(T), refine, levels, init_levels=list(start))
        return np.array([float(x[-1]) for x in nm])

    nm_net = final_nmse(learned.learned_start(params, T, levels, ws))
    nm_quad = final_nmse(hg.hg_replay_phase_init(T, levels))
    _, nm_rand = hg.hg_gs_batched(list(T), refine, levels, seeds=[7] * K)
    nm_rand = np.array([float(x[-1]) for x in nm_rand])
    say(f"NMSE after {refine} GS: network {np.median(nm_net):.4f}, quadratic {np.median(nm_quad):.4f}, "
        f"random {np.median(nm_rand):.4f}")
    assert np.median(nm_net) < np.median(nm_quad)
    assert np.all(nm_net < nm_rand)


def test_learned_start_time_gain():
    """Wall-time gain of the learned start (network forward, start levels, 10
    GS iterations) over plain GS from a random phase, as the time plain GS
    needs to reach the same NMSE (200 iterations when it never does, a lower
    bound).  The gain over GS from the quadratic start alone, which is the
    network's own ablation, is measured and printed.  The network forward
    costs tens of microseconds per image, against about 2 us per GS iteration
    at 512^2.  It saves about two iterations over the quadratic start, so
    that gain stays below 1."""
    K = 16
    T = learned.make_targets(512, range(900200, 900200 + K), DEV)
    params = learned.load_params(device=DEV)
    res = learned.evaluate(params, T, levels=8, refine=10)
    g = res["learned"]
    say(f"learned start: median NMSE {g['final_nmse_median']:.4f}, time gain over plain GS "
        f"{g['time_gain_median']:.2f} (plain GS reached it on {g['gs_reached_fraction']:.2f} of the targets), "
        f"over quadratic-start GS {g['time_gain_vs_quadratic_gs_median']:.2f}; "
        f"forward {res['forward_ms_batch'] / K * 1e3:.1f} us per image")
    assert g["time_gain_median"] >= 1.5
    assert g["win_fraction"] >= 0.75
