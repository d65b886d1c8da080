"""Column-pass kernels for GS / weighted GS (and adaptive OSPR) at batch scale (GPU).

Three kinds run these passes (hg_set_column_kernel): one column tile per
workgroup (the default), a persistent software-pipelined pass for batches
of at least 2048 column tiles (8 problems of 1024^2, 32 of 512^2), and the
classic one-tile kernels.  For each of the first two, in the 1024^2 x 32
weighted binary configuration the benchmark times and in the 1024^2 and
512^2 Fresnel 8-level classes of the uneven batch: the first iteration in
lock-step against the FP64 oracle on sampled problems, and a 4-iteration
batch against the same problems called one by one through the classic
kernels (the kernels round differently, so NMSE agrees to the parity
tolerance and levels up to rare flips at decision boundaries).
"""
import numpy as np
import pytest

import synth
from oracle import hologram, metrics, slm
from parity import NMSE_TOL, exempt_bounds, level_check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2008_12214_amd as hg  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print("[gpu-pipeline]", *a, flush=True)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


CASES = [
    # n, batch, weighted, levels, fresnel   (the first is the benchmark's configuration)
    (1024, 32, True, 2, False),
    (1024, 8, False, 8, True),
    (512, 32, False, 8, True),
]


def _problem(n, b, L, fresnel):
    T = synth.gaussian_target(n, seed=2, batch_item=b)
    start = np.random.default_rng(1000 + b).integers(0, L, (n, n)).astype(np.uint8)
    optics = (synth.WAVELENGTH_M, synth.PITCH_M, synth.fresnel_z(4, b)) if fresnel else (0.0, 0.0, 0.0)
    return T, start, optics


KINDS = {"tile": hg.COLUMN_TILE, "persistent": hg.COLUMN_PERSISTENT}


def _with_kind(kind, fn):
    hg.hg_set_column_kernel(kind)
    try:
        return fn()
    finally:
        hg.hg_set_column_kernel(hg.COLUMN_TILE)


def _batched(n, B, weighted, L, fresnel, iters, kind):
    probs = [_problem(n, b, L, fresnel) for b in range(B)]

    def run():
        lv, nm = hg.hg_gs_batched([dev(p[0]) for p in probs], iters, L, weighted=weighted,
                                  init_levels=[dev(p[1]) for p in probs], optics=[p[2] for p in probs])
        return [host(x) for x in lv], [host(x) for x in nm]
    lv, nm = _with_kind(kind, run)
    return probs, lv, nm


@pytest.mark.parametrize("kind", sorted(KINDS))
@pytest.mark.parametrize("n,B,weighted,L,fresnel", CASES)
def test_batch_column_pass_first_iteration_lockstep(n, B, weighted, L, fresnel, kind):
    say("lock-step", kind, n, B, "wgs" if weighted else "gs", L, "fresnel" if fresnel else "fourier")
    probs, lv, nm = _batched(n, B, weighted, L, fresnel, 1, KINDS[kind])
    for b in (0, B - 1):
        T, start, optics = probs[b]
        ref = hologram.gs(T, 1, L, init_levels=start.astype(np.int64), weighted=weighted,
                          optics=optics if fresnel else None)
        bad, ex = level_check(lv[b], ref["levels"], ref["g"], L, where=f"problem {b}")
        assert bad == 0, f"problem {b}: {bad} non-exempt level mismatches"
        err = np.max(np.abs(nm[b] - ref["nmse"]) / ref["nmse"])
        assert err < NMSE_TOL, (b, err)
        say(f"  problem {b}: nmse rel err {err:.2e}, exempt flips {ex}")


@pytest.mark.parametrize("kind", sorted(KINDS))
@pytest.mark.parametrize("n,B,weighted,L,fresnel", CASES)
def test_batch_column_pass_matches_classic_single_calls(n, B, weighted, L, fresnel, kind):
    """After one iteration the batch kernel and the classic kernel called on
    one problem agree on every level up to the exempt-flip bound and on the
    NMSE to the parity tolerance.  Over four free-running iterations a single
    boundary flip legitimately changes the trajectory, so the level
    differences and NMSE gap after four are reported, not gated (each kernel
    is held to the oracle in lock-step elsewhere)."""
    say("batch vs classic single calls", kind, n, B, "wgs" if weighted else "gs", L)
    for K in (1, 4):
        probs, lv, nm = _batched(n, B, weighted, L, fresnel, K, KINDS[kind])
        for b in (0, B // 2, B - 1):
            T, start, (lam, p, z) = probs[b]
            call = hg.hg_wgs if weighted else hg.hg_gs
            o = _with_kind(hg.COLUMN_CLASSIC, lambda: call(dev(T), K, L, init_levels=dev(start), wavelength_m=lam,
                                                             pitch_m=p, z_m=z))
            nm1, lv1 = host(o["nmse"]), host(o["levels"])
            err = np.max(np.abs(nm[b] - nm1) / nm1)
            nflip = int(np.sum(lv[b] != lv1))
            say(f"  {K} iteration(s), problem {b}: nmse rel diff {err:.2e}, level differences {nflip}")
            if K == 1:
                assert err < NMSE_TOL, (b, err)
                assert nflip <= exempt_bounds(lv1.size, L)[0], (b, nflip)
            else:
                assert nm[b][-1] < nm[b][0]


# ---------------------------------------------------------------------------
# OSPR column passes at 1024^2 (the batched OSPR benchmark's class)
# ---------------------------------------------------------------------------
OSPR_KINDS = {"tile": hg.COLUMN_TILE, "classic": hg.COLUMN_CLASSIC}


def _ospr_batch(kind, Ts, sub, seeds):
    def run():
        lv, nm, ac = hg.hg_ospr_batched([dev(T) for T in Ts], sub, True, seeds=seeds, want_accum=True)
        return [host(x) for x in lv], [host(x) for x in nm], [host(x) for x in ac]
    return _with_kind(kind, run)


@pytest.mark.parametrize("kind", sorted(OSPR_KINDS))
def test_ospr_1024_batch_lockstep(kind):
    """Adaptive OSPR, 3 problems of 1024^2, 5 subframes: every subframe of
    the first and last problem in lock-step with the oracle (continuing from
    the GPU's own binary subframes), the accumulated intensity to the field
    tolerance."""
    say("ospr 1024 lock-step", kind)
    n, B, sub = 1024, 3, 5
    Ts = [synth.gaussian_target(n, seed=3, batch_item=b) for b in range(B)]
    seeds = [70 + b for b in range(B)]
    lv, nm, ac = _ospr_batch(OSPR_KINDS[kind], Ts, sub, seeds)
    for b in (0, B - 1):
        T = hologram.prepare_target(Ts[b], 2)
        A = np.zeros_like(T)
        lev = lv[b].astype(np.int64)
        for i in range(sub):
            k, g, _, _ = hologram.ospr_subframe(T, A, i + 1, True, seed=seeds[b], batch_item=b)
            bad, _ = level_check(lev[i], k, g, 2, where=f"problem {b} subframe {i + 1}")
            assert bad == 0, (b, i, bad)
            h = np.where(lev[i] == 1, -1.0, 1.0)
            A = A + np.abs(hologram.forward(h)) ** 2
            e = metrics.nmse(T, np.sqrt(A / (i + 1)))
            assert abs(nm[b][i] - e) / e < NMSE_TOL, (b, i, nm[b][i], e)
        rel = np.linalg.norm(ac[b] - A) / np.linalg.norm(A)
        assert rel < 1e-4, (b, rel)
        say(f"  problem {b}: final nmse {nm[b][-1]:.4f}, accum rel {rel:.2e}")


def test_ospr_1024_tile_matches_classic():
    """The tile and classic OSPR column kernels on the same batch: NMSE to the
    parity tolerance, levels up to rare decision-boundary flips."""
    say("ospr 1024 tile vs classic")
    n, B, sub = 1024, 4, 8
    Ts = [synth.gaussian_target(n, seed=5, batch_item=b) for b in range(B)]
    seeds = [90 + b for b in range(B)]
    lt, nt, at = _ospr_batch(hg.COLUMN_TILE, Ts, sub, seeds)
    lc, nc, acc = _ospr_batch(hg.COLUMN_CLASSIC, Ts, sub, seeds)
    for b in range(B):
        err = np.max(np.abs(nt[b] - nc[b]) / nc[b])
        flips = float(np.mean(lt[b] != lc[b]))
        say(f"  problem {b}: nmse rel diff {err:.2e}, level differences {flips:.2e}")
        assert err < NMSE_TOL, (b, err)
        assert flips < 1e-3, (b, flips)
