"""Autotuned launch configurations and the general-L projection (GPU).

hg_autotune times the compiled column tiles and row groupings of one size and
batch class and installs the fastest; calls made with the tuned configuration
must still match the FP64 oracle in lock-step.  The row pass's general level
path (L outside {0, 2, 4, 8}: the arctangent and a per-workgroup level table,
the multi-level projection of Listing 1 at full circle) runs in lock-step at
L = 3, 16 and 256 on a square and a rectangular grid.
"""
import numpy as np
import pytest

import synth
from oracle import hologram, slm
from parity import FIELD_TOL, NMSE_TOL, level_check, rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2008_12214_amd as hg  # noqa: E402

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return abs(float(a) - float(b)) / abs(float(b))


def _lockstep_batched(Ts, L, weighted, seeds, iters, check):
    """Iterations 1..iters of problems `check` of one batched call, each
    against the oracle's step from the state the call reached before it."""
    B = len(Ts)
    tg = [dev(t) for t in Ts]
    n0, n1 = Ts[0].shape
    prev = {}
    for k in range(1, iters + 1):
        wts = [torch.ones((n0, n1), dtype=torch.float32, device=DEV) for _ in range(B)] if weighted else None
        lv, nm = hg.hg_gs_batched(tg, k, L, seeds=seeds, weighted=weighted, weights=wts)
        for b in check:
            lev_k, nm_k = host(lv[b]).astype(np.int64), host(nm[b])
            w_k = host(wts[b]).astype(np.float64) if weighted else None
            T = hologram.prepare_target(Ts[b], L)
            if k == 1:
                ref = hologram.gs(Ts[b], 1, L, seed=seeds[b], batch_item=b, weighted=weighted)
                r_lev, r_g, r_nm, r_w = ref["levels"], ref["g"], ref["nmse"][0], ref["weights"]
            else:
                lev_p, w_p = prev[b]
                st = hologram.gs_step(T, L, slm.level_phasor(lev_p, L), weighted=weighted, w_prev=w_p,
                                      next_nmse=False)
                r_lev, r_g, r_nm, r_w = st["levels"], st["g"], st["nmse"], st["weights"]
            where = f"problem {b} iteration {k}"
            bad, _ = level_check(lev_k, r_lev, r_g, L, where=where)
            assert bad == 0, f"{where}: {bad} non-exempt level mismatches"
            assert _rel(nm_k[k - 1], r_nm) < NMSE_TOL, (where, nm_k[k - 1], r_nm)
            if weighted:
                assert rel_l2(w_k, r_w) < FIELD_TOL, where
            prev[b] = (lev_k, w_k)
    return nm


@pytest.mark.parametrize("ny,nx,B,L,weighted", [(1024, 1024, 32, 2, True), (512, 512, 1, 8, False)])
def test_autotuned_configuration_is_compiled_and_keeps_parity(ny, nx, B, L, weighted):
    say(f"autotune {ny}x{nx} batch {B}")
    default = hg.hg_get_launch_config(ny, nx, B)
    try:
        c, r = hg.hg_autotune(ny, nx, B, device=DEV)
        say(f"  default (column tile, rows per group) {default}, tuned ({c}, {r})")
        assert (c, r) == hg.hg_get_launch_config(ny, nx, B)
        assert c in (2, 4, 8, 16) and r in (1, 2, 4, 8, 16, 32, 64)
        Ts = [synth.gaussian_target(nx, seed=21, batch_item=b, ny=ny) for b in range(B)]
        seeds = [40 + b for b in range(B)]
        check = sorted({0, B - 1})
        nm_t = _lockstep_batched(Ts, L, weighted, seeds, 2, check)
        # the same call in the default configuration agrees to rounding
        hg.hg_set_launch_config(ny, nx, B, 0, 0)
        _, nm_d = hg.hg_gs_batched([dev(t) for t in Ts], 2, L, seeds=seeds, weighted=weighted)
        for b in check:
            a, d = host(nm_t[b]), host(nm_d[b])
            assert np.max(np.abs(a[:2] - d[:2]) / d[:2]) < NMSE_TOL, (b, a, d)
    finally:
        hg.hg_set_launch_config(ny, nx, B, 0, 0)


@pytest.mark.parametrize("ny,nx", [(256, 256), (512, 1024)])
@pytest.mark.parametrize("L", [3, 16, 256])
def test_general_levels_lockstep(ny, nx, L):
    """Three iterations of 8-problem batches (the multi-launch row and column
    passes) at L = 3, 16 and 256; problems 0 and 7 in lock-step."""
    say(f"general-L lock-step {ny}x{nx} L={L}")
    B = 8
    Ts = [synth.gaussian_target(nx, seed=22, batch_item=b, ny=ny) for b in range(B)]
    _lockstep_batched(Ts, L, False, [60 + b for b in range(B)], 3, [0, B - 1])
