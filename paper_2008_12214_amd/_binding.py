"""ctypes binding of include/hologen.h and include/hologen_nn.h (argument marshalling only).

Each ``hg_*`` function here has the name and meaning of the C entry point.
Tensors must live on the GPU the library runs on; outputs and the
workspace are allocated with torch on the target tensor's device, and the
call is enqueued on torch's current stream of that device (or ``stream``).
"""
import ctypes
import os

HG_OK, HG_ERR_INVALID_ARG, HG_ERR_UNSUPPORTED_SIZE, HG_ERR_WORKSPACE, HG_ERR_HIP, HG_ERR_NUMERIC = range(6)
HG_OP_GS, HG_OP_WGS, HG_OP_OSPR, HG_OP_PROPAGATE = 1, 2, 3, 4

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libhologen.so")

_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_u64 = ctypes.c_uint64
_sz = ctypes.c_size_t


class HologenError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hologen status {status}: {msg}")
        self.status = status


class hg_kernel_times(ctypes.Structure):
    _fields_ = [("col_ms", _d), ("row_ms", _d), ("setup_ms", _d),
                ("col_launches", ctypes.c_longlong), ("row_launches", ctypes.c_longlong),
                ("setup_launches", ctypes.c_longlong)]


class hg_problem(ctypes.Structure):
    _fields_ = [("ny", _i), ("nx", _i), ("slm_levels", _i), ("iters", _i), ("seed", _u64),
                ("wavelength_m", _d), ("pitch_m", _d), ("z_m", _d),
                ("target", _vp), ("levels_out", _vp), ("nmse_out", _vp),
                ("init_levels", _vp), ("replay_out", _vp),
                ("lt", _i), ("lt_r0", _i), ("lt_dr", _i), ("reserved_", _i), ("weights", _vp), ("roi", _vp)]


class hg_ospr_problem(ctypes.Structure):
    _fields_ = [("ny", _i), ("nx", _i), ("seed", _u64), ("target", _vp), ("levels_out", _vp),
                ("nmse_out", _vp), ("accum_out", _vp)]


_LIB = None


def lib():
    """Load the in-tree HIP library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(lib_path):
            raise ImportError(f"{lib_path} is missing: run __graft_entry__.build() "
                              "(python -m paper_2008_12214_amd.build) first")
        # PyTorch-ROCm carries its own HIP runtime with the same SONAME as the
        # system one.  Loading torch first makes the library bind to that
        # runtime, so both share one device context and torch's streams are
        # valid handles here.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(lib_path)
        L.hg_workspace_size.restype = _sz
        L.hg_workspace_size.argtypes = [_i, _i, _i, _i]
        L.hg_gs.restype = _i
        L.hg_gs.argtypes = [_vp, _i, _i, _i, _i, _u64, _vp, _vp, _d, _d, _d, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
        L.hg_wgs.restype = _i
        L.hg_wgs.argtypes = [_vp, _i, _i, _i, _i, _u64, _vp, _vp, _d, _d, _d, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                             _vp]
        L.hg_wgs_static.restype = _i
        L.hg_wgs_static.argtypes = [_vp, _i, _i, _i, _i, _u64, _vp, _vp, _d, _d, _d, _vp, _vp, _vp, _vp, _vp, _vp]
        L.hg_search_workspace_size.restype = _sz
        L.hg_search_workspace_size.argtypes = [_i, _i, _i]
        L.hg_search.restype = _i
        L.hg_search.argtypes = [_vp, _i, _i, _i, _i, _i, _i, _d, _d, _u64, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
        L.hg_gs_step.restype = _i
        L.hg_gs_step.argtypes = [_vp, _i, _i, _i, _i, _vp, _vp, _d, _d, _d, _i, _vp, _vp, _vp, _vp, _vp, _vp,
                                 _vp, _sz, _vp]
        L.hg_lt.restype = _i
        L.hg_lt.argtypes = [_vp, _i, _i, _i, _i, _u64, _vp, _vp, _d, _d, _d, _i, _i, _vp, _vp, _vp, _vp, _vp, _sz,
                            _vp]
        L.hg_ospr.restype = _i
        L.hg_ospr.argtypes = [_vp, _i, _i, _i, _i, _u64, _vp, _vp, _vp, _vp, _sz, _vp]
        L.hg_ospr_batched_workspace_size.restype = _sz
        L.hg_ospr_batched_workspace_size.argtypes = [ctypes.POINTER(hg_ospr_problem), _i, _i]
        L.hg_ospr_batched.restype = _i
        L.hg_ospr_batched.argtypes = [ctypes.POINTER(hg_ospr_problem), _i, _i, _i, _vp, _sz, _vp]
        L.hg_fresnel_propagate.restype = _i
        L.hg_fresnel_propagate.argtypes = [_vp, _vp, _i, _i, _d, _d, _d, _i, _vp, _sz, _vp]
        L.hg_random_phase.restype = _i
        L.hg_random_phase.argtypes = [_u64, ctypes.c_uint32, ctypes.c_uint32, _i, _i, _i, _vp, _vp]
        L.hg_gs_batched_workspace_size.restype = _sz
        L.hg_gs_batched_workspace_size.argtypes = [ctypes.POINTER(hg_problem), _i]
        L.hg_gs_batched.restype = _i
        L.hg_gs_batched.argtypes = [ctypes.POINTER(hg_problem), _i, _i, _vp, _sz, _vp]
        L.hg_autotune_workspace_size.restype = _sz
        L.hg_autotune_workspace_size.argtypes = [_i, _i, _i]
        L.hg_autotune.restype = _i
        L.hg_autotune.argtypes = [_i, _i, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), _vp, _sz, _vp]
        L.hg_set_launch_config.restype = _i
        L.hg_set_launch_config.argtypes = [_i, _i, _i, _i, _i]
        L.hg_set_small_fused.restype = _i
        L.hg_set_small_fused.argtypes = [_i]
        L.hg_set_column_kernel.restype = _i
        L.hg_set_column_kernel.argtypes = [_i]
        L.hg_set_batch_chunk.restype = _i
        L.hg_set_batch_chunk.argtypes = [ctypes.c_size_t]
        L.hg_get_batch_chunk.restype = ctypes.c_size_t
        L.hg_get_batch_chunk.argtypes = []
        L.hg_get_launch_config.restype = _i
        L.hg_get_launch_config.argtypes = [_i, _i, _i, ctypes.POINTER(_i), ctypes.POINTER(_i)]
        L.hg_timing_enable.restype = None
        L.hg_timing_enable.argtypes = [_i]
        L.hg_timing_read.restype = _i
        L.hg_timing_read.argtypes = [ctypes.POINTER(hg_kernel_times)]
        L.hg_numeric_status.restype = _i
        L.hg_numeric_status.argtypes = [_vp, _vp]
        L.hg_status_string.restype = ctypes.c_char_p
        L.hg_status_string.argtypes = [_i]
        L.hg_last_error.restype = ctypes.c_char_p
        L.hg_last_error.argtypes = []
        _declare_nn(L)
        _LIB = L
    return _LIB


def hg_status_string(status):
    return lib().hg_status_string(status).decode()


def hg_last_error():
    return lib().hg_last_error().decode()


def _check(status):
    if status != HG_OK:
        raise HologenError(status, hg_last_error() or hg_status_string(status))


def hg_numeric_status(workspace, stream=None):
    """Raise HologenError(HG_ERR_NUMERIC) if the last call that used `workspace`
    (a torch uint8 device tensor passed as workspace=...) saw non-finite NMSE sums."""
    _check(lib().hg_numeric_status(_ptr(workspace), _stream(workspace.device, stream)))


def hg_autotune(ny, nx, batch=1, device="cuda", stream=None):
    """Time the compiled tile schedules for (ny, nx, batch); returns (col_tile, rows_per_group)."""
    torch = _torch()
    dev = torch.device(device)
    ws = _workspace(int(lib().hg_autotune_workspace_size(ny, nx, batch)), dev, None)
    c, r = _i(0), _i(0)
    _check(lib().hg_autotune(ny, nx, batch, ctypes.byref(c), ctypes.byref(r), _ptr(ws), ws.numel(),
                             _stream(dev, stream)))
    return c.value, r.value


def hg_set_launch_config(ny, nx, batch, col_tile, rows_per_group):
    _check(lib().hg_set_launch_config(ny, nx, batch, col_tile, rows_per_group))


COLUMN_TILE, COLUMN_PERSISTENT, COLUMN_CLASSIC = 0, 1, 2


def hg_set_column_kernel(kind):
    """Column-pass kernel kind: COLUMN_TILE (default), COLUMN_PERSISTENT or COLUMN_CLASSIC."""
    _check(lib().hg_set_column_kernel(int(kind)))


def hg_set_batch_chunk(field_bytes):
    """Field bytes per chunk of a batched GS call (0: each size class whole)."""
    _check(lib().hg_set_batch_chunk(int(field_bytes)))


def hg_get_batch_chunk():
    """Current field bytes per chunk of a batched GS call."""
    return int(lib().hg_get_batch_chunk())


def hg_set_small_fused(enable):
    """Single-launch path for small problems (each side 64 or 128): on (default) or off."""
    _check(lib().hg_set_small_fused(int(bool(enable))))


def hg_get_launch_config(ny, nx, batch=1):
    c, r = _i(0), _i(0)
    _check(lib().hg_get_launch_config(ny, nx, batch, ctypes.byref(c), ctypes.byref(r)))
    return c.value, r.value


def hg_timing_enable(on=True):
    lib().hg_timing_enable(int(bool(on)))


def hg_timing_read():
    """Summed device ms and launch counts per category since the last read."""
    t = hg_kernel_times()
    _check(lib().hg_timing_read(ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in hg_kernel_times._fields_}


def hg_workspace_size(op, ny, nx, iters=1):
    return int(lib().hg_workspace_size(op, ny, nx, iters))


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(dev, stream):
    torch = _torch()
    s = torch.cuda.current_stream(dev) if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_tensor(t, dtype, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous {dtype} of shape {tuple(shape)}")
    return t


def _workspace(nbytes, dev, workspace):
    torch = _torch()
    if workspace is None:
        workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
    return workspace


def _gs_call(weighted, target, iters, slm_levels, seed, init_levels, init_field, wavelength_m, pitch_m, z_m,
             weights, want_field, want_replay, stream, workspace, lt=None, static_scratch=False):
    torch = _torch()
    ny, nx = target.shape
    _dev_tensor(target, torch.float32, (ny, nx), "target")
    dev = target.device
    if init_levels is not None:
        _dev_tensor(init_levels, torch.uint8, (ny, nx), "init_levels")
    if init_field is not None:
        _dev_tensor(init_field, torch.complex64, (ny, nx), "init_field")
    if weights is not None:
        _dev_tensor(weights, torch.float32, (ny, nx), "weights")
    op = HG_OP_WGS if weighted else HG_OP_GS
    ws = None if static_scratch else _workspace(hg_workspace_size(op, ny, nx, iters), dev, workspace)
    levels = torch.empty((ny, nx), dtype=torch.uint8, device=dev) if slm_levels >= 2 else None
    nmse = torch.empty(iters + 1, dtype=torch.float64, device=dev)
    field = torch.empty((ny, nx), dtype=torch.complex64, device=dev) if want_field else None
    replay = torch.empty((ny, nx), dtype=torch.complex64, device=dev) if want_replay else None
    args = [_ptr(target), ny, nx, iters, slm_levels, seed & (2**64 - 1), _ptr(init_levels), _ptr(init_field),
            float(wavelength_m), float(pitch_m), float(z_m)]
    if lt is not None:
        args += [int(lt[0]), int(lt[1])]
    args += [_ptr(levels), _ptr(field), _ptr(replay), _ptr(nmse)]
    if weighted:
        args.append(_ptr(weights))
    if static_scratch:
        args.append(_stream(dev, stream))
        fn = lib().hg_wgs_static
    else:
        args += [_ptr(ws), ws.numel(), _stream(dev, stream)]
        fn = lib().hg_lt if lt is not None else (lib().hg_wgs if weighted else lib().hg_gs)
    _check(fn(*args))
    return dict(levels=levels, nmse=nmse, field=field, replay=replay, weights=weights)


def hg_gs(target, iters, slm_levels, seed=0, init_levels=None, init_field=None, wavelength_m=0.0, pitch_m=0.0,
          z_m=0.0, want_field=False, want_replay=False, stream=None, workspace=None):
    """Gerchberg-Saxton on the GPU; returns dict(levels, nmse, field, replay)."""
    return _gs_call(False, target, iters, slm_levels, seed, init_levels, init_field, wavelength_m, pitch_m, z_m,
                    None, want_field, want_replay, stream, workspace)


def hg_wgs(target, iters, slm_levels, seed=0, init_levels=None, init_field=None, wavelength_m=0.0, pitch_m=0.0,
           z_m=0.0, weights=None, want_field=False, want_replay=False, stream=None, workspace=None):
    """Weighted GS on the GPU; `weights` (float32, centred) is read and updated in place."""
    return _gs_call(True, target, iters, slm_levels, seed, init_levels, init_field, wavelength_m, pitch_m, z_m,
                    weights, want_field, want_replay, stream, workspace)


def hg_wgs_static(target, iters, slm_levels, seed=0, init_levels=None, init_field=None, wavelength_m=0.0,
                  pitch_m=0.0, z_m=0.0, weights=None, want_field=False, want_replay=False, stream=None):
    """hg_wgs without a workspace: the library's static per-GPU scratch
    (at most HG_STATIC_SCRATCH_BYTES; calls overlapping on one GPU race)."""
    return _gs_call(True, target, iters, slm_levels, seed, init_levels, init_field, wavelength_m, pitch_m, z_m,
                    weights, want_field, want_replay, stream, None, static_scratch=True)


HG_STATIC_SCRATCH_BYTES = 32 << 20
# slm_levels flag: an amplitude SLM with the L transmissions k / (L - 1)
HG_SLM_AMPLITUDE = 0x10000
# slm_levels flag: the field between passes held as two binary16 values (ny in 256..1024)
HG_FIELD_FP16 = 0x20000


HG_SEARCH_DS, HG_SEARCH_SA = 0, 1


def hg_search_workspace_size(ny, nx, batch):
    return int(lib().hg_search_workspace_size(ny, nx, batch))


def hg_search(targets, slm_levels, algorithm, max_sweeps, init_levels, t0=0.0, alpha=1.0, seed=0, stream=None,
              workspace=None):
    """Direct search or simulated annealing over a batch of holograms of one
    size: targets [B, ny, nx] float32, init_levels [B, ny, nx] uint8 (CUDA).
    Returns dict(levels [B, ny, nx], error [B, max_sweeps + 1], sweeps [B])."""
    torch = _torch()
    B, ny, nx = targets.shape
    _dev_tensor(targets, torch.float32, (B, ny, nx), "targets")
    _dev_tensor(init_levels, torch.uint8, (B, ny, nx), "init_levels")
    dev = targets.device
    ws = _workspace(int(lib().hg_search_workspace_size(ny, nx, B)), dev, workspace)
    levels = torch.empty((B, ny, nx), dtype=torch.uint8, device=dev)
    err = torch.empty((B, max_sweeps + 1), dtype=torch.float64, device=dev)
    sweeps = torch.empty(B, dtype=torch.int32, device=dev)
    _check(lib().hg_search(_ptr(targets), B, ny, nx, int(slm_levels), int(algorithm), int(max_sweeps), float(t0),
                           float(alpha), seed & (2**64 - 1), _ptr(init_levels), _ptr(levels), _ptr(err),
                           _ptr(sweeps), _ptr(ws), ws.numel(), _stream(dev, stream)))
    return dict(levels=levels, error=err, sweeps=sweeps)


def hg_gs_step(target, slm_levels, levels_in=None, field_in=None, weights=None, lt_radius=-1, wavelength_m=0.0,
               pitch_m=0.0, z_m=0.0, stream=None, workspace=None):
    """One GS (weights None) or weighted GS iteration from a given state.

    Returns dict(replay=R_k before the constraint, g=field before projection,
    levels, field=f_k, nmse=[NMSE of R_k, NMSE of f_k's replay], weights=w_k
    (the `weights` tensor, updated in place)).
    """
    torch = _torch()
    ny, nx = target.shape
    _dev_tensor(target, torch.float32, (ny, nx), "target")
    dev = target.device
    if levels_in is not None:
        _dev_tensor(levels_in, torch.uint8, (ny, nx), "levels_in")
    if field_in is not None:
        _dev_tensor(field_in, torch.complex64, (ny, nx), "field_in")
    weighted = weights is not None
    if weighted:
        _dev_tensor(weights, torch.float32, (ny, nx), "weights")
    op = HG_OP_WGS if weighted else HG_OP_GS
    ws = _workspace(hg_workspace_size(op, ny, nx, 1), dev, workspace)
    c64 = dict(dtype=torch.complex64, device=dev)
    r, g, f = torch.empty((ny, nx), **c64), torch.empty((ny, nx), **c64), torch.empty((ny, nx), **c64)
    levels = torch.empty((ny, nx), dtype=torch.uint8, device=dev) if slm_levels >= 2 else None
    nmse = torch.empty(2, dtype=torch.float64, device=dev)
    _check(lib().hg_gs_step(_ptr(target), ny, nx, slm_levels, int(weighted), _ptr(levels_in), _ptr(field_in),
                            float(wavelength_m), float(pitch_m), float(z_m), int(lt_radius), _ptr(weights),
                            _ptr(r), _ptr(g), _ptr(levels), _ptr(f), _ptr(nmse), _ptr(ws), ws.numel(),
                            _stream(dev, stream)))
    return dict(replay=r, g=g, levels=levels, field=f, nmse=nmse, weights=weights)


def hg_lt(target, iters, slm_levels, lt_r0, lt_dr, seed=0, init_levels=None, init_field=None, wavelength_m=0.0,
          pitch_m=0.0, z_m=0.0, want_field=False, want_replay=False, stream=None, workspace=None):
    """Liu-Taghizadeh on the GPU (target square of radius lt_r0 + (k-1) lt_dr pixels at
    iteration k); returns dict(levels, nmse, field, replay)."""
    return _gs_call(False, target, iters, slm_levels, seed, init_levels, init_field, wavelength_m, pitch_m, z_m,
                    None, want_field, want_replay, stream, workspace, lt=(lt_r0, lt_dr))


def hg_ospr(target, subframes, adaptive, seed=0, want_accum=False, stream=None, workspace=None):
    """OSPR / adaptive OSPR; returns dict(levels [subframes, ny, nx], nmse, accum)."""
    torch = _torch()
    ny, nx = target.shape
    _dev_tensor(target, torch.float32, (ny, nx), "target")
    dev = target.device
    ws = _workspace(hg_workspace_size(HG_OP_OSPR, ny, nx, subframes), dev, workspace)
    levels = torch.empty((subframes, ny, nx), dtype=torch.uint8, device=dev)
    nmse = torch.empty(subframes, dtype=torch.float64, device=dev)
    accum = torch.empty((ny, nx), dtype=torch.float32, device=dev) if want_accum else None
    _check(lib().hg_ospr(_ptr(target), ny, nx, subframes, int(bool(adaptive)), seed & (2**64 - 1), _ptr(levels),
                         _ptr(nmse), _ptr(accum), _ptr(ws), ws.numel(), _stream(dev, stream)))
    return dict(levels=levels, nmse=nmse, accum=accum)


def hg_ospr_batched(targets, subframes, adaptive, seeds=None, want_accum=False, stream=None, workspace=None):
    """Many OSPR / adaptive OSPR problems (possibly of different sizes) in one call;
    returns (levels, nmse, accum) lists (accum entries None unless want_accum)."""
    torch = _torch()
    dev = targets[0].device
    arr = (hg_ospr_problem * len(targets))()
    levels, nmses, accs = [], [], []
    for i, t in enumerate(targets):
        ny, nx = t.shape
        _dev_tensor(t, torch.float32, (ny, nx), f"targets[{i}]")
        lv = torch.empty((subframes, ny, nx), dtype=torch.uint8, device=dev)
        nm = torch.empty(subframes, dtype=torch.float64, device=dev)
        ac = torch.empty((ny, nx), dtype=torch.float32, device=dev) if want_accum else None
        arr[i] = hg_ospr_problem(ny, nx, (seeds[i] if seeds is not None else 0) & (2**64 - 1), t.data_ptr(),
                                 lv.data_ptr(), nm.data_ptr(), ac.data_ptr() if ac is not None else None)
        levels.append(lv)
        nmses.append(nm)
        accs.append(ac)
    nbytes = int(lib().hg_ospr_batched_workspace_size(arr, len(targets), subframes))
    ws = _workspace(nbytes, dev, workspace)
    _check(lib().hg_ospr_batched(arr, len(targets), subframes, int(bool(adaptive)), _ptr(ws), ws.numel(),
                                 _stream(dev, stream)))
    return levels, nmses, accs


def hg_fresnel_propagate(field, wavelength_m=0.0, pitch_m=0.0, z_m=0.0, direction=1, out=None, stream=None,
                         workspace=None):
    """Unitary Fourier/Fresnel propagation of a complex64 field; returns `out`."""
    torch = _torch()
    ny, nx = field.shape
    _dev_tensor(field, torch.complex64, (ny, nx), "field")
    dev = field.device
    if out is None:
        out = torch.empty_like(field)
    ws = _workspace(hg_workspace_size(HG_OP_PROPAGATE, ny, nx, 1), dev, workspace)
    _check(lib().hg_fresnel_propagate(_ptr(field), _ptr(out), ny, nx, float(wavelength_m), float(pitch_m),
                                      float(z_m), int(direction), _ptr(ws), ws.numel(), _stream(dev, stream)))
    return out


def hg_random_phase(seed, item, tag, axis, ny, nx, device="cuda", stream=None):
    """The library's Philox phasor field exp(2 pi i u24) for (seed, item, tag) on lines along `axis`."""
    torch = _torch()
    dev = torch.device(device)
    out = torch.empty((ny, nx), dtype=torch.complex64, device=dev)
    _check(lib().hg_random_phase(seed & (2**64 - 1), item, tag, axis, ny, nx, _ptr(out), _stream(dev, stream)))
    return out


def _problem_array(problems):
    arr = (hg_problem * len(problems))()
    for i, p in enumerate(problems):
        arr[i] = hg_problem(p["ny"], p["nx"], p["slm_levels"], p["iters"], p.get("seed", 0) & (2**64 - 1),
                            p.get("wavelength_m", 0.0), p.get("pitch_m", 0.0), p.get("z_m", 0.0),
                            p["target"].data_ptr() if p.get("target") is not None else None,
                            p["levels_out"].data_ptr() if p.get("levels_out") is not None else None,
                            p["nmse_out"].data_ptr() if p.get("nmse_out") is not None else None,
                            p["init_levels"].data_ptr() if p.get("init_levels") is not None else None,
                            p["replay_out"].data_ptr() if p.get("replay_out") is not None else None)
        lt = p.get("lt")
        if lt is not None:
            arr[i].lt, arr[i].lt_r0, arr[i].lt_dr = 1, int(lt[0]), int(lt[1])
        if p.get("weights") is not None:
            arr[i].weights = p["weights"].data_ptr()
        if p.get("roi") is not None:
            arr[i].roi = p["roi"].data_ptr()
    return arr


def hg_gs_batched_workspace_size(problems):
    arr = _problem_array(problems)
    return int(lib().hg_gs_batched_workspace_size(arr, len(problems)))


def hg_gs_batched(targets, iters, slm_levels, seeds=None, optics=None, weighted=False, init_levels=None,
                  want_replay=False, stream=None, workspace=None, lt=None, weights=None, roi=None):
    """Many GS problems (possibly of different sizes) in one call.

    targets: list of float32 CUDA tensors; slm_levels: one value for every
    problem or a list of one per problem (levels, with HG_SLM_AMPLITUDE or-ed
    in for an amplitude SLM); optics: optional list of
    (wavelength_m, pitch_m, z_m) per problem; init_levels: optional list of
    uint8 start levels (entries may be None); weights: optional list of
    float32 weight tensors (weighted calls read w_0 and write w_K in place;
    entries may be None); roi: optional list of uint8 region-of-interest
    masks (centred, nonzero = controlled; entries may be None).  Returns
    (levels, nmse) lists, plus the list of final centred replays when
    want_replay.
    """
    torch = _torch()
    dev = targets[0].device
    probs, levels, nmses, replays = [], [], [], []
    per = list(slm_levels) if isinstance(slm_levels, (list, tuple)) else [slm_levels] * len(targets)
    for i, t in enumerate(targets):
        ny, nx = t.shape
        _dev_tensor(t, torch.float32, (ny, nx), f"targets[{i}]")
        lv = torch.empty((ny, nx), dtype=torch.uint8, device=dev) if per[i] >= 2 else None
        nm = torch.empty(iters + 1, dtype=torch.float64, device=dev)
        rp = torch.empty((ny, nx), dtype=torch.complex64, device=dev) if want_replay else None
        il = init_levels[i] if init_levels is not None else None
        if il is not None:
            _dev_tensor(il, torch.uint8, (ny, nx), f"init_levels[{i}]")
        wt = weights[i] if weights is not None else None
        if wt is not None:
            _dev_tensor(wt, torch.float32, (ny, nx), f"weights[{i}]")
        rm = roi[i] if roi is not None else None
        if rm is not None:
            _dev_tensor(rm, torch.uint8, (ny, nx), f"roi[{i}]")
        lam, pit, z = optics[i] if optics is not None else (0.0, 0.0, 0.0)
        probs.append(dict(ny=ny, nx=nx, slm_levels=per[i], iters=iters,
                          seed=(seeds[i] if seeds is not None else 0), wavelength_m=lam, pitch_m=pit, z_m=z,
                          target=t, levels_out=lv, nmse_out=nm, init_levels=il, replay_out=rp,
                          lt=(lt[i] if lt is not None else None), weights=wt, roi=rm))
        levels.append(lv)
        nmses.append(nm)
        replays.append(rp)
    arr = _problem_array(probs)
    nbytes = int(lib().hg_gs_batched_workspace_size(arr, len(probs)))
    ws = _workspace(nbytes, dev, workspace)
    _check(lib().hg_gs_batched(arr, len(probs), int(bool(weighted)), _ptr(ws), ws.numel(), _stream(dev, stream)))
    return (levels, nmses, replays) if want_replay else (levels, nmses)


# ---------------------------------------------------------------------------
# learned initialisation (include/hologen_nn.h)
# ---------------------------------------------------------------------------
_l = ctypes.c_long


def _declare_nn(L):
    sig = {
        "hg_nn_param_count": (_l, []),
        "hg_nn_workspace_size": (_sz, [_i, _i, _i]),
        "hg_nn_forward": (_i, [_vp, _vp, _i, _i, _i, _vp, _vp, _sz, _vp]),
        "hg_nn_backward": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _vp, _vp, _vp, _sz, _vp]),
        "hg_nn_adam": (_i, [_vp, _vp, _vp, _vp, _l, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                            ctypes.c_float, _i, _vp]),
        "hg_replay_phase_init_workspace_size": (_sz, [_i, _i, _i]),
        "hg_replay_phase_init": (_i, [_vp, _vp, _i, _i, _i, _i, _i, _vp, _vp, _sz, _vp]),
        "hg_quadratic_phase_apply": (_i, [_vp, _i, _i, _i, _i, _vp]),
        "hg_nn_kpad": (_i, [_i]),
        "hg_nn_pack_weights": (_i, [_vp, _vp, _i, _i, _i, _vp]),
        "hg_nn_conv3x3": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _i, _vp]),
        "hg_nn_wgrad_workspace_size": (_sz, [_i, _i, _i, _i, _i]),
        "hg_nn_conv3x3_wgrad": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _vp, _sz, _vp]),
        "hg_nn_avgpool2": (_i, [_vp, _vp, _i, _i, _i, _i, _vp]),
        "hg_nn_avgpool2_backward": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _i, _vp]),
        "hg_nn_upsample_concat": (_i, [_vp, _vp, _vp, _i, _i, _i, _i, _i, _vp]),
        "hg_nn_upsample_concat_backward": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _vp]),
        "hg_nn_head": (_i, [_vp, _vp, _vp, _vp, _l, _i, _vp]),
        "hg_nn_head_workspace_size": (_sz, [_i]),
        "hg_nn_head_backward": (_i, [_vp, _vp, _vp, _vp, _vp, _l, _i, _vp, _sz, _vp]),
        "hg_nn_loss_workspace_size": (_sz, [_i]),
        "hg_nn_phase_loss": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _l, _vp, _sz, _vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _need(t, dtype, name, ndim=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous() or (ndim is not None and t.dim() != ndim):
        raise ValueError(f"{name} must be a contiguous {dtype} tensor" + (f" with {ndim} dims" if ndim else ""))
    return t


def hg_nn_param_count():
    return int(lib().hg_nn_param_count())


def hg_nn_workspace_size(batch, h, w):
    return int(lib().hg_nn_workspace_size(batch, h, w))


def hg_nn_workspace(batch, h, w, device="cuda"):
    """A workspace tensor for hg_nn_forward / hg_nn_backward at this shape."""
    torch = _torch()
    n = hg_nn_workspace_size(batch, h, w)
    if n == 0:
        raise HologenError(HG_ERR_UNSUPPORTED_SIZE, "network shape unsupported (h, w multiples of 8)")
    return torch.empty(n, dtype=torch.uint8, device=torch.device(device))


def hg_nn_forward(params, target, workspace, out=None, stream=None):
    """Head output [B, H, W, 2] float32 for targets [B, H, W]; activations stay in `workspace`."""
    torch = _torch()
    _need(params, torch.float32, "params", 1)
    _need(target, torch.float32, "target", 3)
    b, h, w = target.shape
    dev = target.device
    if out is None:
        out = torch.empty((b, h, w, 2), dtype=torch.float32, device=dev)
    _need(out, torch.float32, "out", 4)
    _check(lib().hg_nn_forward(_ptr(params), _ptr(target), b, h, w, _ptr(out), _ptr(workspace), workspace.numel(),
                               _stream(dev, stream)))
    return out


def hg_nn_backward(params, out, label, amp, workspace, grads=None, stream=None):
    """(grads, per-image loss) of the phase loss; follows hg_nn_forward on the same workspace."""
    torch = _torch()
    _need(params, torch.float32, "params", 1)
    _need(out, torch.float32, "out", 4)
    _need(label, torch.complex64, "label", 3)
    _need(amp, torch.float32, "amp", 3)
    b, h, w = amp.shape
    dev = amp.device
    if grads is None:
        grads = torch.empty_like(params)
    loss = torch.empty(b, dtype=torch.float32, device=dev)
    _check(lib().hg_nn_backward(_ptr(params), _ptr(out), _ptr(label), _ptr(amp), b, h, w, _ptr(grads), _ptr(loss),
                                _ptr(workspace), workspace.numel(), _stream(dev, stream)))
    return grads, loss


def hg_nn_adam(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    torch = _torch()
    for t, n in ((params, "params"), (grads, "grads"), (m, "m"), (v, "v")):
        _need(t, torch.float32, n)
    _check(lib().hg_nn_adam(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), params.numel(), lr, beta1, beta2, eps,
                            int(step), _stream(params.device, stream)))


def hg_replay_phase_init(target, slm_levels, phasor=None, add_quadratic=None, stream=None):
    """SLM start levels P_L(IDFT(T e^{i psi})) for targets [B, ny, nx].

    psi = arg(phasor) (+ the quadratic phase when add_quadratic); phasor None
    with add_quadratic left unset selects the quadratic phase alone."""
    torch = _torch()
    _need(target, torch.float32, "target", 3)
    b, ny, nx = target.shape
    dev = target.device
    if add_quadratic is None:
        add_quadratic = phasor is None
    if phasor is not None:
        if phasor.dtype == torch.float32 and phasor.dim() == 4 and phasor.shape[-1] == 2:
            _need(phasor, torch.float32, "phasor", 4)
        else:
            _need(phasor, torch.complex64, "phasor", 3)
    levels = torch.empty((b, ny, nx), dtype=torch.uint8, device=dev)
    n = int(lib().hg_replay_phase_init_workspace_size(b, ny, nx))
    ws = _workspace(n, dev, None)
    _check(lib().hg_replay_phase_init(_ptr(phasor), _ptr(target), b, ny, nx, slm_levels, int(bool(add_quadratic)),
                                      _ptr(levels), _ptr(ws), ws.numel(), _stream(dev, stream)))
    return levels


def hg_quadratic_phase_apply(field, sign, stream=None):
    """In place: field [B, ny, nx] complex64 (centred) *= exp(sign i psi0)."""
    torch = _torch()
    _need(field, torch.complex64, "field", 3)
    b, ny, nx = field.shape
    _check(lib().hg_quadratic_phase_apply(_ptr(field), b, ny, nx, int(sign), _stream(field.device, stream)))
    return field


def hg_nn_pack_weights(w, flip=False, stream=None):
    """bf16 GEMM operand from OHWI float32 weights [cout, 3, 3, cin]."""
    torch = _torch()
    _need(w, torch.float32, "w", 4)
    cout, _, _, cin = w.shape
    rows, k = (cin, 9 * cout) if flip else (cout, 9 * cin)
    wg = torch.empty((rows, int(lib().hg_nn_kpad(k))), dtype=torch.bfloat16, device=w.device)
    _check(lib().hg_nn_pack_weights(_ptr(w), _ptr(wg), cout, cin, int(bool(flip)), _stream(w.device, stream)))
    return wg


def hg_nn_conv3x3(x, wg, cout, bias=None, mask=None, relu=False, stream=None):
    torch = _torch()
    _need(x, torch.bfloat16, "x", 4)
    n, h, w, cin = x.shape
    y = torch.empty((n, h, w, cout), dtype=torch.bfloat16, device=x.device)
    _check(lib().hg_nn_conv3x3(_ptr(x), _ptr(wg), _ptr(bias), _ptr(mask), _ptr(y), n, h, w, cin, cout,
                               int(bool(relu)), _stream(x.device, stream)))
    return y


def hg_nn_conv3x3_wgrad(x, dy, stream=None):
    torch = _torch()
    _need(x, torch.bfloat16, "x", 4)
    _need(dy, torch.bfloat16, "dy", 4)
    n, h, w, cin = x.shape
    cout = dy.shape[3]
    dw = torch.empty((cout, 3, 3, cin), dtype=torch.float32, device=x.device)
    db = torch.empty(cout, dtype=torch.float32, device=x.device)
    ws = _workspace(int(lib().hg_nn_wgrad_workspace_size(n, h, w, cin, cout)), x.device, None)
    _check(lib().hg_nn_conv3x3_wgrad(_ptr(x), _ptr(dy), _ptr(dw), _ptr(db), n, h, w, cin, cout, _ptr(ws),
                                     ws.numel(), _stream(x.device, stream)))
    return dw, db


def hg_nn_avgpool2(x, stream=None):
    torch = _torch()
    _need(x, torch.bfloat16, "x", 4)
    n, h, w, c = x.shape
    y = torch.empty((n, h // 2, w // 2, c), dtype=torch.bfloat16, device=x.device)
    _check(lib().hg_nn_avgpool2(_ptr(x), _ptr(y), n, h, w, c, _stream(x.device, stream)))
    return y


def hg_nn_avgpool2_backward(dy, dskip=None, mask=None, stream=None):
    torch = _torch()
    _need(dy, torch.bfloat16, "dy", 4)
    n, h2, w2, c = dy.shape
    dx = torch.empty((n, 2 * h2, 2 * w2, c), dtype=torch.bfloat16, device=dy.device)
    _check(lib().hg_nn_avgpool2_backward(_ptr(dy), _ptr(dskip), _ptr(mask), _ptr(dx), n, 2 * h2, 2 * w2, c,
                                         _stream(dy.device, stream)))
    return dx


def hg_nn_upsample_concat(lo, skip, stream=None):
    torch = _torch()
    _need(lo, torch.bfloat16, "lo", 4)
    _need(skip, torch.bfloat16, "skip", 4)
    n, h, w, c2 = skip.shape
    c1 = lo.shape[3]
    out = torch.empty((n, h, w, c1 + c2), dtype=torch.bfloat16, device=lo.device)
    _check(lib().hg_nn_upsample_concat(_ptr(lo), _ptr(skip), _ptr(out), n, h, w, c1, c2, _stream(lo.device, stream)))
    return out


def hg_nn_upsample_concat_backward(dout, c1, mask_lo=None, stream=None):
    torch = _torch()
    _need(dout, torch.bfloat16, "dout", 4)
    n, h, w, c = dout.shape
    c2 = c - c1
    dlo = torch.empty((n, h // 2, w // 2, c1), dtype=torch.bfloat16, device=dout.device)
    dskip = torch.empty((n, h, w, c2), dtype=torch.bfloat16, device=dout.device)
    _check(lib().hg_nn_upsample_concat_backward(_ptr(dout), _ptr(mask_lo), _ptr(dlo), _ptr(dskip), n, h, w, c1, c2,
                                                _stream(dout.device, stream)))
    return dlo, dskip


def hg_nn_head(x, w, b, stream=None):
    torch = _torch()
    _need(x, torch.bfloat16, "x")
    c = x.shape[-1]
    pixels = x.numel() // c
    out = torch.empty(tuple(x.shape[:-1]) + (2,), dtype=torch.float32, device=x.device)
    _check(lib().hg_nn_head(_ptr(x), _ptr(w), _ptr(b), _ptr(out), pixels, c, _stream(x.device, stream)))
    return out


def hg_nn_head_backward(dout, w, x, stream=None):
    """(dx, dwb): dwb = weight gradient [2, c] flattened, then bias gradient [2]."""
    torch = _torch()
    _need(x, torch.bfloat16, "x")
    c = x.shape[-1]
    pixels = x.numel() // c
    dx = torch.empty_like(x)
    dwb = torch.empty(2 * c + 2, dtype=torch.float32, device=x.device)
    ws = _workspace(int(lib().hg_nn_head_workspace_size(c)), x.device, None)
    _check(lib().hg_nn_head_backward(_ptr(dout), _ptr(w), _ptr(x), _ptr(dx), _ptr(dwb), pixels, c, _ptr(ws),
                                     ws.numel(), _stream(x.device, stream)))
    return dx, dwb


def hg_nn_phase_loss(out, label, amp, stream=None):
    """(dout, per-image loss) of the phase loss for head output out [B, ..., 2]."""
    torch = _torch()
    _need(out, torch.float32, "out")
    _need(label, torch.complex64, "label")
    _need(amp, torch.float32, "amp")
    b = amp.shape[0]
    hw = amp.numel() // b
    dout = torch.empty_like(out)
    loss = torch.empty(b, dtype=torch.float32, device=out.device)
    ws = _workspace(int(lib().hg_nn_loss_workspace_size(b)), out.device, None)
    _check(lib().hg_nn_phase_loss(_ptr(out), _ptr(label), _ptr(amp), _ptr(dout), _ptr(loss), b, hw, _ptr(ws),
                                  ws.numel(), _stream(out.device, stream)))
    return dout, loss
