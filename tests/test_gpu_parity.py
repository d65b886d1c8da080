"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances: complex fields and NMSE within 1e-4 relative (L2 for fields).
Quantised levels must match exactly except at pixels whose oracle phase lies
within 1e-5 rad of a decision boundary or whose field is zero to FP32
precision (|g| below 1e-6 of its rms); those are counted and reported.
Quantised runs are checked in lock-step: each step starts both sides from
the GPU's own state (levels, weights, accumulated intensity), because a
single legitimate near-threshold flip changes the rest of a free-running
trajectory.  Continuous-phase runs are compared free-running.
"""
import numpy as np
import pytest

import synth
from oracle import hologram, philox, slm, metrics
from parity import FIELD_TOL, NMSE_TOL, level_check, rel_l2, rel_max, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2008_12214_amd as hg  # noqa: E402

DEV = "cuda:0"


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# ---------------------------------------------------------------------------
# Philox and propagation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,item,tag,axis", [(1, 0, 1, 1), (0xDEADBEEF12345678, 7, 0x100 + 3, 0),
                                                 (5, 2, 0x100 + 24, 1)])
def test_philox_phases_bit_exact(seed, item, tag, axis):
    say("philox", seed, item, tag, axis)
    ny, nx = 64, 256
    z = host(hg.hg_random_phase(seed, item, tag, axis, ny, nx, device=DEV)).astype(np.complex128)
    u_gpu = np.round(np.mod(np.angle(z) / (2 * np.pi), 1.0) * 2 ** 24).astype(np.int64) % (1 << 24)
    words = philox.line_words(seed, tag, ny, nx, axis, batch_item=item)
    u_ref = (words >> np.uint64(40)).astype(np.int64)
    np.testing.assert_array_equal(u_gpu, u_ref)
    np.testing.assert_allclose(np.abs(z), 1.0, atol=1e-6)


@pytest.mark.parametrize("ny,nx,z", [(64, 128, 0.0), (256, 64, 0.0), (128, 128, 0.05), (1024, 1024, 0.0),
                                     (512, 1024, 0.3)])
def test_propagate_matches_oracle(ny, nx, z):
    say("propagate", ny, nx, z)
    rng = np.random.default_rng(ny + nx)
    f = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex64)
    lam, p = synth.WAVELENGTH_M, synth.PITCH_M
    R = host(hg.hg_fresnel_propagate(dev(f), lam, p, z, +1))
    R_ref = hologram.fresnel_propagate(f, lam, p, z, +1)
    assert rel_l2(R, R_ref) < FIELD_TOL
    b = host(hg.hg_fresnel_propagate(dev(R_ref.astype(np.complex64)), lam, p, z, -1))
    assert rel_l2(b, hologram.fresnel_propagate(R_ref.astype(np.complex64), lam, p, z, -1)) < FIELD_TOL


def test_propagate_4096_properties():
    say("propagate 4096^2")
    n = 4096
    rng = np.random.default_rng(5)
    f = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(np.complex64)
    F = hg.hg_fresnel_propagate(dev(f), 0, 0, 0, +1)
    back = host(hg.hg_fresnel_propagate(F, 0, 0, 0, -1))
    Fh = host(F).astype(np.complex128)
    assert rel_l2(back, f) < FIELD_TOL
    assert abs(np.sum(np.abs(Fh) ** 2) / np.sum(np.abs(f.astype(np.complex128)) ** 2) - 1) < 1e-5
    # sampled outputs computed one by one from Eq. fouriertrans2d5c (centred)
    y = np.arange(n)[:, None]
    x = np.arange(n)[None, :]
    for (vc, uc) in [(0, 0), (n // 2, n // 2), (17, 4000), (3001, 5)]:
        v, u = vc - n // 2, uc - n // 2
        ph = -2 * np.pi * (((u * x) % n) / n + ((v * y) % n) / n)
        ref = np.sum(f * np.exp(1j * ph)) / n
        assert abs(Fh[vc, uc] - ref) < 1e-4 * np.sqrt(np.mean(np.abs(Fh) ** 2)) * 10


# ---------------------------------------------------------------------------
# continuous-phase GS, free-running
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ny,nx,iters,optics", [(64, 64, 50, None), (128, 256, 20, None),
                                                (256, 128, 10, (532e-9, 8e-6, 0.1)), (1024, 1024, 5, None),
                                                (128, 128, 10, (532e-9, 8e-6, 0.15)), (512, 1024, 4, None),
                                                (1024, 256, 4, (532e-9, 8e-6, 0.2))])
def test_gs_continuous_free_running(ny, nx, iters, optics):
    """Free-running: NMSE of every iteration; fields while the trajectories
    have not yet drifted apart (zero-amplitude target regions leave the
    phase there unconstrained, so rounding differences grow slowly)."""
    say("gs L=0", ny, nx, iters, optics)
    T = synth.uniform_target(ny, nx, seed=1) if ny == nx == 64 else synth.gaussian_target(nx, seed=2, ny=ny)
    lam, p, z = optics if optics else (0.0, 0.0, 0.0)
    out = hg.hg_gs(dev(T), iters, 0, seed=1, wavelength_m=lam, pitch_m=p, z_m=z)
    ref = hologram.gs(T, iters, 0, seed=1, optics=optics)
    nm = host(out["nmse"])
    say("  nmse gpu/ref final", nm[-1], ref["nmse"][-1])
    assert rel_max(nm, ref["nmse"]) < NMSE_TOL
    k = min(iters, 5)
    out = hg.hg_gs(dev(T), k, 0, seed=1, wavelength_m=lam, pitch_m=p, z_m=z, want_field=True, want_replay=True)
    ref = hologram.gs(T, k, 0, seed=1, optics=optics)
    assert rel_l2(host(out["field"]), ref["field"]) < FIELD_TOL
    assert rel_l2(host(out["replay"]), ref["replay"]) < FIELD_TOL


@pytest.mark.parametrize("ny,nx,steps,optics", [(128, 256, 20, None), (256, 128, 10, (532e-9, 8e-6, 0.1))])
def test_gs_continuous_lockstep(ny, nx, steps, optics):
    say("gs L=0 lock-step", ny, nx, steps, optics)
    T = synth.gaussian_target(nx, seed=2, ny=ny)
    lam, p, z = optics if optics else (0.0, 0.0, 0.0)
    f = None
    for k in range(steps):
        out = hg.hg_gs(dev(T), 1, 0, seed=1, init_field=None if f is None else dev(f.astype(np.complex64)),
                       wavelength_m=lam, pitch_m=p, z_m=z, want_field=True, want_replay=True)
        ref = hologram.gs(T, 1, 0, seed=1, init_field=f, optics=optics)
        gf = host(out["field"])
        assert rel_l2(gf, ref["field"]) < FIELD_TOL, k
        assert rel_l2(host(out["replay"]), ref["replay"]) < FIELD_TOL, k
        assert rel_max(host(out["nmse"]), ref["nmse"]) < NMSE_TOL, k
        f = gf.astype(np.complex128)


# ---------------------------------------------------------------------------
# quantised GS / WGS, lock-step
# ---------------------------------------------------------------------------
def _lockstep(T, L, steps, weighted, seed=1, optics=None, start=None):
    """Run `steps` lock-step iterations; returns (max nmse err, total exempt)."""
    ny, nx = T.shape
    lam, p, z = optics if optics else (0.0, 0.0, 0.0)
    lev, w = start if start is not None else (None, None)
    worst, exempt_total = 0.0, 0
    for k in range(steps):
        kw = dict(seed=seed, wavelength_m=lam, pitch_m=p, z_m=z,
                  init_levels=None if lev is None else dev(lev.astype(np.uint8)))
        if weighted:
            wt = None if w is None else dev(w.astype(np.float32))
            out = hg.hg_wgs(dev(T), 1, L, weights=wt if wt is not None else dev(np.ones((ny, nx), np.float32)),
                            **kw)
        else:
            out = hg.hg_gs(dev(T), 1, L, **kw)
        ref = hologram.gs(T, 1, L, seed=seed, init_levels=lev, weighted=weighted,
                          weights=None if w is None else w, optics=optics)
        g_lev = host(out["levels"])
        bad, ex = level_check(g_lev, ref["levels"], ref["g"], L, where=f"step {k}")
        exempt_total += ex
        assert bad == 0, f"step {k}: {bad} non-exempt level mismatches ({ex} exempt)"
        e = rel_max(host(out["nmse"]), ref["nmse"])
        worst = max(worst, e)
        assert e < NMSE_TOL, f"step {k}: nmse rel err {e}"
        if weighted:
            gw = host(out["weights"])
            assert rel_l2(gw, ref["weights"]) < FIELD_TOL, f"step {k}: weights"
            w = gw.astype(np.float64)
        lev = g_lev.astype(np.int64)
    return worst, exempt_total, (lev, w)


def test_gs_8level_64_lockstep_50():
    say("gs L=8 64^2 lock-step x50")
    T = synth.uniform_target(64, 64, seed=1)
    worst, ex, _ = _lockstep(T, 8, 50, weighted=False)
    say(f"  worst nmse rel err {worst:.2e}, exempt level flips {ex}")


def test_wgs_binary_256_lockstep_30():
    say("wgs L=2 256^2 lock-step x30")
    T = synth.gaussian_target(256, seed=2)
    worst, ex, _ = _lockstep(T, 2, 30, weighted=True)
    say(f"  worst nmse rel err {worst:.2e}, exempt level flips {ex}")


def test_gs_fresnel_lockstep():
    say("gs L=8 fresnel 256^2 lock-step x5")
    T = synth.gaussian_target(256, seed=4)
    _lockstep(T, 8, 5, weighted=False, optics=(532e-9, 8e-6, synth.fresnel_z(4, 0)))


@pytest.mark.parametrize("ny,nx,weighted,L,optics", [(256, 512, False, 4, None), (512, 256, True, 4, (532e-9, 8e-6, 0.15)),
                                                    (512, 512, False, 8, None)])
def test_four_and_eight_levels_lockstep(ny, nx, weighted, L, optics):
    """Four and eight levels through the multi-launch pipeline, whose row pass
    decides these level sets by quadrant comparisons instead of an angle."""
    say("row-pass L=4/8 lock-step", ny, nx, "wgs" if weighted else "gs", L, optics)
    T = synth.gaussian_target(nx, seed=6, ny=ny)
    worst, ex, _ = _lockstep(T, L, 4, weighted=weighted, optics=optics)
    say(f"  worst nmse rel err {worst:.2e}, exempt level flips {ex}")


@pytest.mark.parametrize("ny,nx,weighted,L,optics", [
    (64, 128, True, 2, None), (128, 64, False, 4, (532e-9, 8e-6, 0.12)),
    (128, 128, True, 8, (532e-9, 8e-6, 0.2)), (128, 128, False, 3, None)])
def test_small_single_launch_lockstep(ny, nx, weighted, L, optics):
    """Sizes that run whole in the single-launch small-problem kernel."""
    say("small single launch lock-step", ny, nx, "wgs" if weighted else "gs", L, optics)
    T = synth.gaussian_target(nx, seed=5, ny=ny)
    worst, ex, _ = _lockstep(T, L, 4, weighted=weighted, optics=optics)
    say(f"  worst nmse rel err {worst:.2e}, exempt level flips {ex}")


# ---------------------------------------------------------------------------
# Liu-Taghizadeh: growing target square, amplitude free outside it
# ---------------------------------------------------------------------------
def _lt_lockstep(T, L, r0, dr, steps, optics=None):
    lam, p, z = optics if optics else (0.0, 0.0, 0.0)
    lev, worst, exempt = None, 0.0, 0
    for k in range(steps):
        r = r0 + k * dr  # iteration k + 1 of the schedule, as a single iteration
        out = hg.hg_lt(dev(T), 1, L, r, 0, seed=1, init_levels=None if lev is None else dev(lev.astype(np.uint8)),
                       wavelength_m=lam, pitch_m=p, z_m=z)
        ref = hologram.gs(T, 1, L, seed=1, init_levels=lev, optics=optics, lt=(r, 0))
        g_lev = host(out["levels"])
        bad, ex = level_check(g_lev, ref["levels"], ref["g"], L)
        exempt += ex
        assert bad == 0, f"step {k}: {bad} non-exempt level mismatches"
        e = rel_max(host(out["nmse"]), ref["nmse"])
        worst = max(worst, e)
        assert e < NMSE_TOL, f"step {k}: nmse rel err {e}"
        lev = g_lev.astype(np.int64)
    return worst, exempt


@pytest.mark.parametrize("n,L,r0,dr,steps,optics", [(256, 8, 40, 16, 6, None),
                                                    (1024, 2, 200, 100, 2, (532e-9, 8e-6, 0.3))])
def test_lt_lockstep(n, L, r0, dr, steps, optics):
    say("Liu-Taghizadeh lock-step", n, L, r0, dr, steps, optics)
    T = synth.gaussian_target(n, seed=8)
    worst, ex = _lt_lockstep(T, L, r0, dr, steps, optics)
    say(f"  worst nmse rel err {worst:.2e}, exempt level flips {ex}")


def test_lt_continuous_free_running():
    say("Liu-Taghizadeh L=0 free-running 128x256")
    T = synth.gaussian_target(256, seed=9, ny=128)
    out = hg.hg_lt(dev(T), 8, 0, 20, 12, seed=1, want_field=True)
    ref = hologram.gs(T, 8, 0, seed=1, lt=(20, 12))
    assert rel_max(host(out["nmse"]), ref["nmse"]) < NMSE_TOL
    out = hg.hg_lt(dev(T), 3, 0, 20, 12, seed=1, want_field=True, want_replay=True)
    ref = hologram.gs(T, 3, 0, seed=1, lt=(20, 12))
    assert rel_l2(host(out["field"]), ref["field"]) < FIELD_TOL
    assert rel_l2(host(out["replay"]), ref["replay"]) < FIELD_TOL


def test_lt_call_equals_chained_iterations_and_batch():
    say("Liu-Taghizadeh: 6 iterations == 6 chained single iterations == batched")
    T = synth.gaussian_target(256, seed=10)
    full = hg.hg_lt(dev(T), 6, 8, 30, 20, seed=5)
    lev, nms = None, []
    for k in range(6):
        o = hg.hg_lt(dev(T), 1, 8, 30 + 20 * k, 0, seed=5, init_levels=lev)
        lev = o["levels"].clone()
        nms.append(host(o["nmse"]))
    np.testing.assert_array_equal(host(full["levels"]), host(lev))
    assert rel_max(host(full["nmse"])[1:], np.array([n[1] for n in nms])) < 1e-8
    # a batch mixing Liu-Taghizadeh and plain GS problems of one size
    Ts = [dev(synth.gaussian_target(256, seed=10 + i)) for i in range(4)]
    starts = [dev(np.random.default_rng(i).integers(0, 8, (256, 256)).astype(np.uint8)) for i in range(4)]
    lts = [(30, 20), None, (0, 64), None]
    lv, nm = hg.hg_gs_batched(Ts, 6, 8, init_levels=starts, lt=lts)
    for i in range(4):
        if lts[i] is None:
            o = hg.hg_gs(Ts[i], 6, 8, init_levels=starts[i])
        else:
            o = hg.hg_lt(Ts[i], 6, 8, lts[i][0], lts[i][1], init_levels=starts[i])
        np.testing.assert_array_equal(host(lv[i]), host(o["levels"]), err_msg=str(i))
        assert rel_max(host(nm[i]), host(o["nmse"])) < 1e-8


@pytest.mark.parametrize("rpb", [2, 4])
def test_gs_fresnel_2048_rows(rpb):
    """2048-wide rows span two waves: a 4-row group staged through LDS with
    one exchange buffer per row (4 rows per workgroup) or two double-buffered
    rows (2).  One lock-step iteration against the oracle, then a 3-iteration
    call (whose earlier iterations take the projection path that writes
    nothing) gives the levels of 3 chained single iterations bit for bit."""
    say(f"gs L=8 fresnel 2048^2, {rpb} rows per workgroup")
    saved = hg.hg_get_launch_config(2048, 2048, 1)
    hg.hg_set_launch_config(2048, 2048, 1, saved[0], rpb)
    try:
        T = synth.gaussian_target(2048, seed=4)
        lam, p, z = optics = (532e-9, 8e-6, synth.fresnel_z(4, 0))
        _, ex, _ = _lockstep(T, 8, 1, weighted=False, optics=optics)
        full = hg.hg_gs(dev(T), 3, 8, seed=5, wavelength_m=lam, pitch_m=p, z_m=z)
        lev, nms = None, []
        for _ in range(3):
            o = hg.hg_gs(dev(T), 1, 8, seed=5, init_levels=lev, wavelength_m=lam, pitch_m=p, z_m=z)
            lev = o["levels"].clone()
            nms.append(host(o["nmse"]))
        np.testing.assert_array_equal(host(full["levels"]), host(lev))
        # a chained call's value comes from the finishing column launch, the
        # full call's from the next iteration's: the same sums in another order
        assert rel_max(host(full["nmse"])[1:], np.array([n[1] for n in nms])) < 1e-8
        say(f"  exempt level flips {ex}")
    finally:
        hg.hg_set_launch_config(2048, 2048, 1, *saved)


@pytest.mark.parametrize("weighted,L", [(True, 2), (False, 8)])
def test_sparse_target_lockstep(weighted, L):
    """A target of a few isolated points at 1024^2: most column tiles miss its
    support (they read no target), the others meet it on one or two rows.
    Two iterations in lock-step with the FP64 oracle."""
    say("sparse target 1024^2 lock-step", "wgs" if weighted else "gs", L)
    rng = np.random.default_rng(21)
    T = np.zeros((1024, 1024))
    ys, xs = rng.integers(0, 1024, 6), rng.integers(0, 1024, 6)
    T[ys, xs] = rng.uniform(0.5, 1.0, 6)
    worst, ex, _ = _lockstep(T.astype(np.float32), L, 2, weighted=weighted)
    say(f"  worst nmse rel err {worst:.2e}, exempt level flips {ex}")


def test_wgs_binary_4096_lockstep():
    """The largest supported plane (4096^2, two columns per tile, one row per
    workgroup): one weighted binary iteration in lock-step with the FP64
    oracle, every level and the NMSE values."""
    say("wgs binary 4096^2 lock-step")
    T = synth.gaussian_target(4096, seed=9)
    worst, ex, _ = _lockstep(T, 2, 1, weighted=True)
    say(f"  nmse rel err {worst:.2e}, exempt level flips {ex}")


def test_wgs_binary_1024_full_size_sampled():
    """Headline workload (1024^2, binary, weighted, 100 iterations): lock-step
    on iterations 1-3, then the single 100-iteration call the bench times
    continues from there and its last steps are checked in lock-step."""
    say("wgs L=2 1024^2 sampled lock-step")
    T = synth.gaussian_target(1024, seed=2)
    _, ex0, state = _lockstep(T, 2, 3, weighted=True)
    lev, w = state
    wt = dev(w.astype(np.float32))
    out = hg.hg_wgs(dev(T), 94, 2, init_levels=dev(lev.astype(np.uint8)), weights=wt)
    lev2, w2 = host(out["levels"]).astype(np.int64), host(wt).astype(np.float64)
    nm = host(out["nmse"])
    assert np.all(np.isfinite(nm)) and nm[-1] < nm[0]
    _, ex1, _ = _lockstep(T, 2, 3, weighted=True, start=(lev2, w2))
    say(f"  exempt level flips {ex0 + ex1}, nmse after 97 it {nm[-1]:.4f}")


def test_multi_iteration_call_equals_chained_steps():
    say("resume: 6 iterations == 6 chained single iterations")
    T = synth.gaussian_target(256, seed=3)
    w_full = dev(np.ones((256, 256), np.float32))
    full = hg.hg_wgs(dev(T), 6, 8, seed=5, weights=w_full)
    lev, w = None, dev(np.ones((256, 256), np.float32))
    nms = []
    for k in range(6):
        o = hg.hg_wgs(dev(T), 1, 8, seed=5, init_levels=lev, weights=w)
        lev = o["levels"].clone()
        nms.append(host(o["nmse"]))
    np.testing.assert_array_equal(host(full["levels"]), host(lev))
    np.testing.assert_array_equal(host(w_full), host(w))
    np.testing.assert_array_equal(host(full["nmse"])[1:], np.array([n[1] for n in nms]))


# ---------------------------------------------------------------------------
# OSPR, lock-step on the accumulated intensity
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ny,nx,subframes,adaptive,cfg", [
    (128, 128, 8, False, None),
    (512, 512, 24, True, None),     # small batch at 512: 8 elements per thread in both passes
    (512, 1024, 4, True, None),     # 8-element columns, 16-element rows
    (512, 512, 4, True, (8, 8)),    # the 16-element tiles, set explicitly
])
def test_ospr_lockstep(ny, nx, subframes, adaptive, cfg):
    say("ospr", ny, nx, subframes, adaptive, cfg)
    T_raw = synth.gaussian_target(nx, seed=3, ny=ny)
    if cfg is not None:
        hg.hg_set_launch_config(ny, nx, 1, *cfg)
    try:
        out = hg.hg_ospr(dev(T_raw), subframes, adaptive, seed=3, want_accum=True)
    finally:
        if cfg is not None:
            hg.hg_set_launch_config(ny, nx, 1, 0, 0)
    lev = host(out["levels"]).astype(np.int64)
    nm = host(out["nmse"])
    T = hologram.prepare_target(T_raw, 2)
    A = np.zeros_like(T)
    ex_total = 0
    for i in range(subframes):
        k, g, A_ref, e_ref = hologram.ospr_subframe(T, A, i + 1, adaptive, seed=3)
        bad, ex = level_check(lev[i], k, g, 2)
        ex_total += ex
        assert bad == 0, f"subframe {i + 1}: {bad} non-exempt mismatches"
        # continue from the GPU's own subframe (lock-step on the state A)
        h = np.where(lev[i] == 1, -1.0, 1.0)
        A = A + np.abs(hologram.forward(h)) ** 2
        e = metrics.nmse(T, np.sqrt(A / (i + 1)))
        assert abs(nm[i] - e) / e < NMSE_TOL, (i, nm[i], e)
    assert rel_l2(host(out["accum"]), A) < FIELD_TOL
    say(f"  exempt flips {ex_total}, final nmse {nm[-1]:.4f}")


def test_ospr_batched_lockstep_and_single_call():
    """Many OSPR problems of two sizes in one call: sampled problems in lock-step
    with the oracle (each draws its subframe phases with its own Philox item),
    and problem 0 equals the single-problem call bit for bit."""
    say("ospr batched")
    sizes = [(256, 256)] * 3 + [(512, 256)] * 2
    seeds = [31 + i for i in range(len(sizes))]
    Ts = [synth.gaussian_target(nx, seed=3, batch_item=i, ny=ny) for i, (ny, nx) in enumerate(sizes)]
    sub = 6
    lv, nm, ac = hg.hg_ospr_batched([dev(T) for T in Ts], sub, True, seeds=seeds, want_accum=True)
    for i in (0, 4):
        T = hologram.prepare_target(Ts[i], 2)
        A = np.zeros_like(T)
        lev = host(lv[i]).astype(np.int64)
        nmi = host(nm[i])
        for n in range(sub):
            k, g, _, _ = hologram.ospr_subframe(T, A, n + 1, True, seed=seeds[i], batch_item=i)
            bad, _ = level_check(lev[n], k, g, 2)
            assert bad == 0, (i, n, bad)
            h = np.where(lev[n] == 1, -1.0, 1.0)
            A = A + np.abs(hologram.forward(h)) ** 2
            e = metrics.nmse(T, np.sqrt(A / (n + 1)))
            assert abs(nmi[n] - e) / e < NMSE_TOL, (i, n, nmi[n], e)
        assert rel_l2(host(ac[i]), A) < FIELD_TOL
    one = hg.hg_ospr(dev(Ts[0]), sub, True, seed=seeds[0], want_accum=True)
    np.testing.assert_array_equal(host(one["levels"]), host(lv[0]))
    np.testing.assert_array_equal(host(one["nmse"]), host(nm[0]))


# ---------------------------------------------------------------------------
# batched uneven problems
# ---------------------------------------------------------------------------
def test_batched_uneven_first_step_and_continuous():
    say("batched uneven")
    sizes = [64, 128, 64, 256, 128]
    seeds = [11, 12, 13, 14, 15]
    optics = [(synth.WAVELENGTH_M, synth.PITCH_M, synth.fresnel_z(4, i)) for i in range(len(sizes))]
    optics[2] = (0.0, 0.0, 0.0)  # one Fourier problem inside a Fresnel class
    targets = [synth.gaussian_target(n, seed=4, batch_item=i) for i, n in enumerate(sizes)]
    lv, nm = hg.hg_gs_batched([dev(t) for t in targets], 1, 8, seeds=seeds, optics=optics)
    for i, T in enumerate(targets):
        opt = optics[i] if optics[i][2] > 0 else None
        ref = hologram.gs(T, 1, 8, seed=seeds[i], optics=opt, batch_item=i)
        bad, ex = level_check(host(lv[i]), ref["levels"], ref["g"], 8)
        assert bad == 0, (i, bad)
        assert rel_max(host(nm[i]), ref["nmse"]) < NMSE_TOL
    lv, nm = hg.hg_gs_batched([dev(t) for t in targets], 6, 0, seeds=seeds, optics=optics)
    for i, T in enumerate(targets):
        opt = optics[i] if optics[i][2] > 0 else None
        ref = hologram.gs(T, 6, 0, seed=seeds[i], optics=opt, batch_item=i)
        assert rel_max(host(nm[i]), ref["nmse"]) < NMSE_TOL
