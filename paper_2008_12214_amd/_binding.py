"""ctypes binding of include/hologen.h (argument marshalling only).

Each ``hg_*`` function here has the name and meaning of the C entry point.
Tensors must live on the GPU the library runs on; outputs and the
workspace are allocated with torch on the target tensor's device, and the
call is enqueued on torch's current stream of that device (or ``stream``).
"""
import ctypes
import os

HG_OK, HG_ERR_INVALID_ARG, HG_ERR_UNSUPPORTED_SIZE, HG_ERR_WORKSPACE, HG_ERR_HIP = range(5)
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
                ("target", _vp), ("levels_out", _vp), ("nmse_out", _vp)]


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
        L.hg_ospr.restype = _i
        L.hg_ospr.argtypes = [_vp, _i, _i, _i, _i, _u64, _vp, _vp, _vp, _vp, _sz, _vp]
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
        L.hg_get_launch_config.restype = _i
        L.hg_get_launch_config.argtypes = [_i, _i, _i, ctypes.POINTER(_i), ctypes.POINTER(_i)]
        L.hg_timing_enable.restype = None
        L.hg_timing_enable.argtypes = [_i]
        L.hg_timing_read.restype = _i
        L.hg_timing_read.argtypes = [ctypes.POINTER(hg_kernel_times)]
        L.hg_status_string.restype = ctypes.c_char_p
        L.hg_status_string.argtypes = [_i]
        L.hg_last_error.restype = ctypes.c_char_p
        L.hg_last_error.argtypes = []
        _LIB = L
    return _LIB


def hg_status_string(status):
    return lib().hg_status_string(status).decode()


def hg_last_error():
    return lib().hg_last_error().decode()


def _check(status):
    if status != HG_OK:
        raise HologenError(status, hg_last_error() or hg_status_string(status))


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
             weights, want_field, want_replay, stream, workspace):
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
    nbytes = hg_workspace_size(op, ny, nx, iters)
    ws = _workspace(nbytes, dev, workspace)
    levels = torch.empty((ny, nx), dtype=torch.uint8, device=dev) if slm_levels >= 2 else None
    nmse = torch.empty(iters + 1, dtype=torch.float64, device=dev)
    field = torch.empty((ny, nx), dtype=torch.complex64, device=dev) if want_field else None
    replay = torch.empty((ny, nx), dtype=torch.complex64, device=dev) if want_replay else None
    args = [_ptr(target), ny, nx, iters, slm_levels, seed & (2**64 - 1), _ptr(init_levels), _ptr(init_field),
            float(wavelength_m), float(pitch_m), float(z_m), _ptr(levels), _ptr(field), _ptr(replay), _ptr(nmse)]
    if weighted:
        args.append(_ptr(weights))
    args += [_ptr(ws), ws.numel(), _stream(dev, stream)]
    _check((lib().hg_wgs if weighted else lib().hg_gs)(*args))
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
                            p["nmse_out"].data_ptr() if p.get("nmse_out") is not None else None)
    return arr


def hg_gs_batched_workspace_size(problems):
    arr = _problem_array(problems)
    return int(lib().hg_gs_batched_workspace_size(arr, len(problems)))


def hg_gs_batched(targets, iters, slm_levels, seeds=None, optics=None, weighted=False, stream=None,
                  workspace=None):
    """Many GS problems (possibly of different sizes) in one call.

    targets: list of float32 CUDA tensors; optics: optional list of
    (wavelength_m, pitch_m, z_m) per problem.  Returns (levels, nmse) lists.
    """
    torch = _torch()
    dev = targets[0].device
    probs, levels, nmses = [], [], []
    for i, t in enumerate(targets):
        ny, nx = t.shape
        _dev_tensor(t, torch.float32, (ny, nx), f"targets[{i}]")
        lv = torch.empty((ny, nx), dtype=torch.uint8, device=dev) if slm_levels >= 2 else None
        nm = torch.empty(iters + 1, dtype=torch.float64, device=dev)
        lam, pit, z = optics[i] if optics is not None else (0.0, 0.0, 0.0)
        probs.append(dict(ny=ny, nx=nx, slm_levels=slm_levels, iters=iters,
                          seed=(seeds[i] if seeds is not None else 0), wavelength_m=lam, pitch_m=pit, z_m=z,
                          target=t, levels_out=lv, nmse_out=nm))
        levels.append(lv)
        nmses.append(nm)
    arr = _problem_array(probs)
    nbytes = int(lib().hg_gs_batched_workspace_size(arr, len(probs)))
    ws = _workspace(nbytes, dev, workspace)
    _check(lib().hg_gs_batched(arr, len(probs), int(bool(weighted)), _ptr(ws), ws.numel(), _stream(dev, stream)))
    return levels, nmses
