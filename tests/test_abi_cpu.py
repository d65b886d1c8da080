"""C-ABI checks that need no GPU: exported symbols, status strings, workspace
queries and host-side argument validation (which runs before any HIP call)."""
import ctypes
import os
import re

import pytest

import paper_2008_12214_amd as hg
from conftest import ROOT

L = hg.lib()
FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: validation fails first


def test_every_declared_symbol_is_exported():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            hdr = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"\b(hg_[a-z0-9_]+)\s*\(", hdr))
    assert {"hg_gs", "hg_wgs", "hg_ospr", "hg_fresnel_propagate", "hg_gs_batched", "hg_nn_forward",
            "hg_nn_backward", "hg_nn_adam", "hg_replay_phase_init", "hg_nn_conv3x3"} <= names
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    for s in range(6):
        assert hg.hg_status_string(s) != "unknown status"
    assert hg.hg_status_string(99) == "unknown status"


def test_numeric_status_argument_checks():
    """hg_numeric_status validates its workspace before any HIP call."""
    assert L.hg_numeric_status(None, None) == hg.HG_ERR_INVALID_ARG
    assert "NULL" in hg.hg_last_error()
    assert L.hg_numeric_status(ctypes.c_void_p(0x10010), None) == hg.HG_ERR_INVALID_ARG
    assert "aligned" in hg.hg_last_error()


def test_workspace_queries():
    g = hg.hg_workspace_size(hg.HG_OP_GS, 1024, 1024, 100)
    w = hg.hg_workspace_size(hg.HG_OP_WGS, 1024, 1024, 100)
    o = hg.hg_workspace_size(hg.HG_OP_OSPR, 512, 512, 24)
    assert g >= 1024 * 1024 * 12 and w >= g + 1024 * 1024 * 4 and o >= 512 * 512 * 16
    assert hg.hg_workspace_size(hg.HG_OP_GS, 1000, 1024, 10) == 0
    assert hg.hg_workspace_size(hg.HG_OP_GS, 32, 32, 10) == 0
    assert hg.hg_workspace_size(hg.HG_OP_GS, 8192, 64, 10) == 0
    assert hg.hg_workspace_size(hg.HG_OP_GS, 64, 64, 0) == 0
    assert hg.hg_workspace_size(99, 64, 64, 1) == 0
    assert hg.hg_workspace_size(hg.HG_OP_PROPAGATE, 64, 4096, 0) > 0


def _gs(target=FAKE, ny=64, nx=64, iters=5, levels=8, levels_out=FAKE, ws=FAKE, wsb=1 << 30, init_levels=None,
        z=0.0, lam=0.0, pitch=0.0):
    return L.hg_gs(target, ny, nx, iters, levels, 1, init_levels, None, lam, pitch, z, levels_out, None, None,
                   None, ws, wsb, None)


@pytest.mark.parametrize("kw,status", [
    (dict(ny=100), hg.HG_ERR_UNSUPPORTED_SIZE),
    (dict(nx=32), hg.HG_ERR_UNSUPPORTED_SIZE),
    (dict(nx=8192), hg.HG_ERR_UNSUPPORTED_SIZE),
    (dict(target=None), hg.HG_ERR_INVALID_ARG),
    (dict(iters=0), hg.HG_ERR_INVALID_ARG),
    (dict(levels=1), hg.HG_ERR_INVALID_ARG),
    (dict(levels=257), hg.HG_ERR_INVALID_ARG),
    (dict(levels_out=None), hg.HG_ERR_INVALID_ARG),
    (dict(levels=0, init_levels=FAKE), hg.HG_ERR_INVALID_ARG),
    (dict(z=0.1, lam=0.0, pitch=8e-6), hg.HG_ERR_INVALID_ARG),
    (dict(ws=None), hg.HG_ERR_WORKSPACE),
    (dict(ws=ctypes.c_void_p(0x10010)), hg.HG_ERR_WORKSPACE),
    (dict(wsb=1024), hg.HG_ERR_WORKSPACE),
])
def test_gs_validation(kw, status):
    assert _gs(**kw) == status
    assert hg.hg_last_error() != ""


def test_wgs_ospr_propagate_batched_validation():
    assert L.hg_wgs(FAKE, 64, 64, 0, 2, 1, None, None, 0.0, 0.0, 0.0, FAKE, None, None, None, None, FAKE, 1 << 30,
                    None) == hg.HG_ERR_INVALID_ARG
    assert L.hg_ospr(FAKE, 64, 64, 4, 1, 1, None, None, None, FAKE, 1 << 30, None) == hg.HG_ERR_INVALID_ARG
    assert L.hg_ospr(FAKE, 64, 64, 4, 1, 1, FAKE, None, None, FAKE, 16, None) == hg.HG_ERR_WORKSPACE
    assert L.hg_fresnel_propagate(FAKE, FAKE, 64, 64, 0.0, 0.0, 0.0, 0, FAKE, 1 << 30, None) == hg.HG_ERR_INVALID_ARG
    assert L.hg_fresnel_propagate(None, FAKE, 64, 64, 0.0, 0.0, 0.0, 1, FAKE, 1 << 30, None) == hg.HG_ERR_INVALID_ARG
    assert L.hg_random_phase(1, 0, 1, 1, 48, 64, FAKE, None) == hg.HG_ERR_UNSUPPORTED_SIZE
    assert L.hg_random_phase(1, 0, 1, 2, 64, 64, FAKE, None) == hg.HG_ERR_INVALID_ARG
    assert L.hg_gs_batched(None, 0, 0, FAKE, 1 << 30, None) == hg.HG_ERR_INVALID_ARG
    probs = (hg._binding.hg_problem * 2)()
    probs[0] = hg._binding.hg_problem(64, 64, 8, 3, 1, 0, 0, 0, 0x10000, 0x10000, None)
    probs[1] = hg._binding.hg_problem(128, 64, 8, 3, 1, 0, 0, 0, 0x10000, None, None)
    assert L.hg_gs_batched(probs, 2, 0, FAKE, 1 << 30, None) == hg.HG_ERR_INVALID_ARG
    assert "problem 1" in hg.hg_last_error()
    probs[1] = hg._binding.hg_problem(128, 64, 8, 3, 1, 0, 0, 0, 0x10000, 0x10000, None)
    need = L.hg_gs_batched_workspace_size(probs, 2)
    assert need > L.hg_workspace_size(hg.HG_OP_WGS, 64, 64, 3)
    assert L.hg_gs_batched(probs, 2, 0, FAKE, need - 256, None) == hg.HG_ERR_WORKSPACE


# ---------------------------------------------------------------------------
# learned initialisation: shape checks and workspace queries (host only)
# ---------------------------------------------------------------------------
def test_nn_param_count_and_workspace_queries():
    assert hg.hg_nn_param_count() == 487026
    assert hg.hg_nn_workspace_size(1, 12, 16) == 0       # not a multiple of 8
    assert hg.hg_nn_workspace_size(0, 64, 64) == 0
    a = hg.hg_nn_workspace_size(1, 64, 64)
    b = hg.hg_nn_workspace_size(4, 64, 64)
    assert a > 64 * 64 * 400 and b - a > 3 * 64 * 64 * 400
    assert L.hg_nn_wgrad_workspace_size(1, 8, 8, 16, 24) == 0  # cout not a multiple of 16
    assert L.hg_nn_kpad(9) == 32 and L.hg_nn_kpad(144) == 160 and L.hg_nn_kpad(288) == 288
    assert L.hg_replay_phase_init_workspace_size(2, 64, 128) >= 2 * 64 * 128 * 8
    assert L.hg_replay_phase_init_workspace_size(1, 100, 128) == 0


@pytest.mark.parametrize("args,status", [
    (dict(h=12), hg.HG_ERR_UNSUPPORTED_SIZE),
    (dict(batch=0), hg.HG_ERR_UNSUPPORTED_SIZE),
    (dict(params=None), hg.HG_ERR_INVALID_ARG),
    (dict(ws=None), hg.HG_ERR_WORKSPACE),
    (dict(wsb=1024), hg.HG_ERR_WORKSPACE),
])
def test_nn_forward_validation(args, status):
    a = dict(params=FAKE, target=FAKE, batch=1, h=64, w=64, out=FAKE, ws=FAKE, wsb=1 << 40)
    a.update(args)
    st = L.hg_nn_forward(a["params"], a["target"], a["batch"], a["h"], a["w"], a["out"], a["ws"], a["wsb"], None)
    assert st == status, hg.hg_last_error()
    assert hg.hg_last_error()


def test_nn_layer_validation():
    assert L.hg_nn_conv3x3(FAKE, FAKE, None, None, FAKE, 1, 8, 8, 16, 24, 0, None) == hg.HG_ERR_INVALID_ARG
    assert L.hg_nn_conv3x3(None, FAKE, None, None, FAKE, 1, 8, 8, 16, 16, 0, None) == hg.HG_ERR_INVALID_ARG
    assert L.hg_nn_avgpool2(FAKE, FAKE, 1, 7, 8, 4, None) == hg.HG_ERR_INVALID_ARG
    assert L.hg_nn_adam(FAKE, FAKE, FAKE, FAKE, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None) == hg.HG_ERR_INVALID_ARG
    assert L.hg_replay_phase_init(None, FAKE, 1, 64, 64, 1, 1, FAKE, FAKE, 1 << 30, None) == hg.HG_ERR_INVALID_ARG
    assert L.hg_replay_phase_init(None, FAKE, 1, 64, 48, 8, 1, FAKE, FAKE, 1 << 30, None) == \
        hg.HG_ERR_UNSUPPORTED_SIZE
    assert L.hg_quadratic_phase_apply(FAKE, 1, 64, 64, 0, None) == hg.HG_ERR_INVALID_ARG
    assert L.hg_nn_conv3x3_wgrad(FAKE, FAKE, FAKE, FAKE, 1, 8, 8, 16, 272, FAKE, 1 << 30, None) == \
        hg.HG_ERR_INVALID_ARG  # more than 256 output channels


def test_committed_network_weights_match_the_layout():
    import numpy as np
    from paper_2008_12214_amd import learned
    v = np.load(learned.WEIGHTS, allow_pickle=False)
    assert v.dtype == np.float32 and v.shape == (hg.hg_nn_param_count(),)
    assert np.isfinite(v).all()


def test_lt_validation():
    """Liu-Taghizadeh arguments are checked on the host before any launch."""
    args = lambda r0, dr, lev=FAKE: (FAKE, 64, 64, 3, 8, 1, None, None, 0.0, 0.0, 0.0, r0, dr, lev, None, None, None,
                                     FAKE, 1 << 30, None)
    assert L.hg_lt(*args(-1, 2)) == hg.HG_ERR_INVALID_ARG
    assert "lt_r0" in hg.hg_last_error()
    assert L.hg_lt(*args(4, -2)) == hg.HG_ERR_INVALID_ARG
    assert L.hg_lt(*args(4, 2, None)) == hg.HG_ERR_INVALID_ARG  # levels_out required at 8 levels
    probs = (hg._binding.hg_problem * 1)()
    probs[0] = hg._binding.hg_problem(64, 64, 8, 3, 1, 0, 0, 0, 0x10000, 0x10000, None)
    probs[0].lt, probs[0].lt_r0, probs[0].lt_dr = 1, 8, 4
    assert L.hg_gs_batched(probs, 1, 1, FAKE, 1 << 30, None) == hg.HG_ERR_INVALID_ARG  # not weighted
    assert "weighted" in hg.hg_last_error()
    probs[0].lt_r0 = -3
    assert L.hg_gs_batched(probs, 1, 0, FAKE, 1 << 30, None) == hg.HG_ERR_INVALID_ARG


def test_roi_validation():
    """A region of interest runs with plain GS: weighted or Liu-Taghizadeh
    problems that carry one are rejected on the host before any launch."""
    probs = (hg._binding.hg_problem * 1)()
    probs[0] = hg._binding.hg_problem(64, 64, 2, 3, 1, 0, 0, 0, 0x10000, 0x10000, None)
    probs[0].roi = 0x10000
    assert L.hg_gs_batched(probs, 1, 1, FAKE, 1 << 30, None) == hg.HG_ERR_INVALID_ARG  # weighted
    assert "region of interest" in hg.hg_last_error()
    probs[0].lt, probs[0].lt_r0, probs[0].lt_dr = 1, 8, 4
    assert L.hg_gs_batched(probs, 1, 0, FAKE, 1 << 30, None) == hg.HG_ERR_INVALID_ARG  # LT
    assert "region of interest" in hg.hg_last_error()
    # the struct ends with the mask pointer, as in include/hologen.h
    assert hg._binding.hg_problem.roi.offset == ctypes.sizeof(hg._binding.hg_problem) - ctypes.sizeof(ctypes.c_void_p)


def test_ospr_batched_validation():
    P = hg._binding.hg_ospr_problem
    probs = (P * 2)()
    probs[0] = P(64, 64, 1, 0x10000, 0x10000, None, None)
    probs[1] = P(64, 48, 1, 0x10000, 0x10000, None, None)
    assert L.hg_ospr_batched_workspace_size(probs, 2, 4) == 0
    assert L.hg_ospr_batched(probs, 2, 4, 1, FAKE, 1 << 30, None) == hg.HG_ERR_UNSUPPORTED_SIZE
    assert "problem 1" in hg.hg_last_error()
    probs[1] = P(128, 64, 1, 0x10000, None, None, None)
    assert L.hg_ospr_batched(probs, 2, 4, 1, FAKE, 1 << 30, None) == hg.HG_ERR_INVALID_ARG  # levels_out
    probs[1] = P(128, 64, 1, 0x10000, 0x10000, None, None)
    need = L.hg_ospr_batched_workspace_size(probs, 2, 4)
    assert need >= L.hg_workspace_size(hg.HG_OP_OSPR, 64, 64, 4) + L.hg_workspace_size(hg.HG_OP_OSPR, 128, 64, 4)
    assert L.hg_ospr_batched(probs, 2, 4, 1, FAKE, need - 256, None) == hg.HG_ERR_WORKSPACE
    assert L.hg_ospr_batched(probs, 2, 0, 1, FAKE, 1 << 30, None) == hg.HG_ERR_INVALID_ARG  # subframes



def test_static_scratch_variant_rejects_oversize_before_any_hip_call():
    """hg_wgs_static checks its arguments and the static scratch's capacity on
    the host: a 2048^2 problem needs more than HG_STATIC_SCRATCH_BYTES."""
    def call(ny=64, nx=64, iters=5, levels=2, target=FAKE, levels_out=FAKE):
        return L.hg_wgs_static(target, ny, nx, iters, levels, 1, None, None, 0.0, 0.0, 0.0, levels_out, None, None,
                               None, None, None)
    need = hg.hg_workspace_size(hg.HG_OP_WGS, 2048, 2048, 100)
    assert need > hg.HG_STATIC_SCRATCH_BYTES
    assert call(ny=2048, nx=2048, iters=100) == hg.HG_ERR_WORKSPACE
    assert "static scratch" in hg.hg_last_error()
    assert hg.hg_workspace_size(hg.HG_OP_WGS, 1024, 1024, 100) <= hg.HG_STATIC_SCRATCH_BYTES
    assert call(ny=100) == hg.HG_ERR_UNSUPPORTED_SIZE
    assert call(target=None) == hg.HG_ERR_INVALID_ARG
    assert call(levels_out=None) == hg.HG_ERR_INVALID_ARG


def test_amplitude_slm_argument_checks():
    """slm_levels = L | HG_SLM_AMPLITUDE needs 2 <= L <= 256 and is not
    accepted by Liu-Taghizadeh; the checks run on the host."""
    A = hg.HG_SLM_AMPLITUDE
    assert _gs(levels=A) == hg.HG_ERR_INVALID_ARG
    assert _gs(levels=A | 1) == hg.HG_ERR_INVALID_ARG
    assert _gs(levels=A | 257) == hg.HG_ERR_INVALID_ARG
    assert _gs(levels=A | 4, levels_out=None) == hg.HG_ERR_INVALID_ARG
    assert L.hg_lt(FAKE, 64, 64, 5, A | 2, 1, None, None, 0.0, 0.0, 0.0, 4, 1, FAKE, None, None, None, FAKE,
                   1 << 30, None) == hg.HG_ERR_INVALID_ARG
    assert "phase SLMs" in hg.hg_last_error()


def test_search_argument_checks():
    """hg_search validates sizes, levels, algorithm and sweeps on the host."""
    def call(ny=16, nx=16, levels=2, algo=0, sweeps=5, t0=0.0, alpha=1.0, init=FAKE, ws=FAKE, wsb=1 << 30):
        return L.hg_search(FAKE, 2, ny, nx, levels, algo, sweeps, t0, alpha, 1, init, FAKE, FAKE, None, ws, wsb, None)
    assert hg.hg_search_workspace_size(16, 16, 2) == 2 * 16 * 16 * 8
    assert hg.hg_search_workspace_size(128, 16, 2) == 0
    assert call(ny=128) == hg.HG_ERR_UNSUPPORTED_SIZE
    assert call(nx=12) == hg.HG_ERR_UNSUPPORTED_SIZE
    assert call(levels=1) == hg.HG_ERR_INVALID_ARG
    assert call(algo=7) == hg.HG_ERR_INVALID_ARG
    assert call(sweeps=0) == hg.HG_ERR_INVALID_ARG
    assert call(init=None) == hg.HG_ERR_INVALID_ARG
    assert call(algo=1, t0=-1.0) == hg.HG_ERR_INVALID_ARG
    assert call(algo=1, alpha=0.0) == hg.HG_ERR_INVALID_ARG
    assert call(ws=None) == hg.HG_ERR_WORKSPACE
    assert call(wsb=100) == hg.HG_ERR_WORKSPACE


def test_batch_chunk_setting():
    """hg_set_batch_chunk stores the chunk size process-wide and rejects sizes
    beyond 1 TiB; 0 (whole size classes) is accepted."""
    old = hg.hg_get_batch_chunk()
    try:
        hg.hg_set_batch_chunk(0)
        assert hg.hg_get_batch_chunk() == 0
        hg.hg_set_batch_chunk(3 << 20)
        assert hg.hg_get_batch_chunk() == 3 << 20
        assert L.hg_set_batch_chunk(ctypes.c_size_t((1 << 40) + 1)) == hg.HG_ERR_INVALID_ARG
        assert "1 TiB" in hg.hg_last_error()
        assert hg.hg_get_batch_chunk() == 3 << 20
    finally:
        hg.hg_set_batch_chunk(old)
