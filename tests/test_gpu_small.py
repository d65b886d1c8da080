"""Single-launch path for small holograms (GPU).

Problems whose sides are 64 or 128 run a whole call in one workgroup with
the field in LDS.  Its agreement with the FP64 oracle is checked in lock-step
by the parity tests (the 64^2 cases there, and the rectangular, Fresnel and
weighted small cases, run through it).  Here: a K-iteration call equals K
chained single-iteration calls bit for bit (the iteration loop, the weight
carry and the last-iteration outputs), a batched call equals the same
problems called one by one, and the two launch paths agree to the parity
tolerance.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2008_12214_amd as hg  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print("[gpu-small]", *a, flush=True)


def host(t):
    torch.cuda.synchronize()
    return None if t is None else t.cpu().numpy()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


OPTICS = dict(wavelength_m=synth.WAVELENGTH_M, pitch_m=synth.PITCH_M, z_m=0.12)


@pytest.mark.parametrize("ny,nx,weighted,L,fresnel", [
    (64, 64, False, 8, False), (64, 128, True, 2, False), (128, 64, False, 4, True),
    (128, 128, True, 8, True), (128, 128, False, 0, True)])
def test_full_call_equals_chained_iterations(ny, nx, weighted, L, fresnel):
    say(ny, nx, "wgs" if weighted else "gs", f"L={L}", "fresnel" if fresnel else "fourier")
    assert hg.hg_get_launch_config(ny, nx)  # sizes are supported
    T = dev(synth.gaussian_target(nx, seed=ny + L, ny=ny))
    opt = OPTICS if fresnel else {}
    K = 6
    w_full = dev(np.random.default_rng(9).uniform(0.5, 2.0, (ny, nx)).astype(np.float32)) if weighted else None
    w_chain = w_full.clone() if weighted else None
    call = hg.hg_wgs if weighted else hg.hg_gs
    extra = (lambda w: dict(weights=w)) if weighted else (lambda w: {})
    full = call(T, K, L, seed=5, want_field=True, want_replay=True, **extra(w_full), **opt)
    lev, fld, nms = None, None, []
    for _ in range(K):
        o = call(T, 1, L, seed=5, init_levels=lev, init_field=fld if L == 0 else None, want_field=True,
                 want_replay=True, **extra(w_chain), **opt)
        if L >= 2:
            lev = o["levels"].clone()
        fld = o["field"].clone()
        nms.append(host(o["nmse"]))
    if L >= 2:
        np.testing.assert_array_equal(host(full["levels"]), host(lev))
    np.testing.assert_array_equal(host(full["field"]), host(fld))
    np.testing.assert_array_equal(host(full["replay"]), host(o["replay"]))
    if weighted:
        np.testing.assert_array_equal(host(w_full), host(w_chain))
    # nmse[k] of the full call and nmse[1] of chained call k sum the same
    # replay (bit-identical above) in the iteration branch and the final
    # branch, which the compiler may contract into FMAs differently
    np.testing.assert_allclose(host(full["nmse"])[1:], np.array([n[1] for n in nms]), rtol=1e-6, atol=0)


def test_batched_equals_single_calls():
    say("batched small classes vs single calls (given start levels)")
    sizes = [(64, 64)] * 12 + [(64, 128)] * 3 + [(128, 128)] * 3
    rng = np.random.default_rng(3)
    targets = [dev(synth.gaussian_target(nx, seed=4, batch_item=i, ny=ny)) for i, (ny, nx) in enumerate(sizes)]
    starts = [dev(rng.integers(0, 8, (ny, nx)).astype(np.uint8)) for (ny, nx) in sizes]
    # one kind of propagation per size class (a Fourier problem in a Fresnel
    # class is modulated through a unit chirp instead of a sign flip)
    optics = [(0.0, 0.0, 0.0) if s == (64, 128) else (synth.WAVELENGTH_M, synth.PITCH_M, synth.fresnel_z(4, i))
              for i, s in enumerate(sizes)]
    lv, nm = hg.hg_gs_batched(targets, 9, 8, init_levels=starts, optics=optics)
    for i in range(len(sizes)):
        lam, p, z = optics[i]
        o = hg.hg_gs(targets[i], 9, 8, init_levels=starts[i], wavelength_m=lam, pitch_m=p, z_m=z)
        np.testing.assert_array_equal(host(lv[i]), host(o["levels"]), err_msg=str(i))
        np.testing.assert_array_equal(host(nm[i]), host(o["nmse"]), err_msg=str(i))


@pytest.mark.parametrize("ny,nx,weighted,L,fresnel", [(64, 64, False, 8, False), (128, 128, True, 2, True)])
def test_single_launch_close_to_pipeline(ny, nx, weighted, L, fresnel):
    """Both launch paths from the same start levels: the first iteration's
    NMSE (before any projection can differ) agrees to 1e-6, the trajectory's
    NMSE to the parity tolerance; at most a few levels differ (a level flips
    where the two kernels' rounding straddles a decision boundary)."""
    say("single launch vs pipeline", ny, nx, L)
    T = dev(synth.gaussian_target(nx, seed=7, ny=ny))
    start = dev(np.random.default_rng(1).integers(0, L, (ny, nx)).astype(np.uint8))
    opt = OPTICS if fresnel else {}
    call = hg.hg_wgs if weighted else hg.hg_gs
    out = []
    for fused in (1, 0):
        hg.hg_set_small_fused(fused)
        try:
            o = call(T, 3, L, init_levels=start, **opt)
            out.append((host(o["levels"]), host(o["nmse"])))
        finally:
            hg.hg_set_small_fused(1)
    (la, na), (lb, nb) = out
    assert abs(na[0] - nb[0]) / nb[0] < 1e-6
    assert np.max(np.abs(na - nb) / nb) < 1e-4
    assert np.mean(la != lb) < 1e-3
