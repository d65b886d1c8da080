"""Benchmark of the weighted-GS hot path on one MI355X.

Workload: weighted Gerchberg-Saxton, binary-phase SLM, 1024x1024 complex64,
100 iterations per hologram, target = sum of 32 Gaussians in the central
512x512 window (seeded synthetic stand-in for the paper's images).  A step
is one complete hg_gs_batched call (set-up, 100 iterations, NMSE finisher)
over a batch of B such holograms already resident in HBM; the default
B = 32 makes the working set (~0.9 GB) exceed the 256 MB Infinity Cache so
the figure is an HBM figure.  value = B * 100 * steps / seconds
(hologram-iterations per second).

Prints one JSON line.  The roofline object reports the column pass (the
kernel that moves the most bytes per launch), timed with hipEvents on the
launch stream during a second, instrumented pass over the same steps.  The
cpu_baseline leg times the FP64 oracle on this host on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GS iter/s at 1024^2 c64 (%HBM peak); time-to-NMSE learned-init vs plain GS"
HBM_PEAK_GBS = 8000.0
N = 1024
LEVELS = 2
# algorithmic HBM bytes per pixel: weighted column pass = field r+w (16) +
# target r (4) and weights r+w (8) on the target support only (the target is
# zero elsewhere, which the set-up pass records per tile, and weights there
# are never used), i.e. 16 + 12 * support fraction; its final launch (NMSE
# only) = field r (8) + target r (4); row pass = field r+w (16), + levels w
# (1) on the last.
COL_FIELD_BYTES, COL_SUPPORT_BYTES, COL_FINAL_BYTES, ROW_BYTES = 16, 12, 12, 16
ITERS = 100


def support_of(T, binary):
    """Fraction of pixels where the prepared target is nonzero (binary: T or its mirror, after symmetrisation)."""
    import numpy as np
    if binary:
        n0, n1 = T.shape
        mir = T[(-np.arange(n0)) % n0][:, (-np.arange(n1)) % n1]
        return float(np.mean((T > 0) | (mir > 0)))
    return float(np.mean(T > 0))


def kernel_source_hash():
    """sha256 of the HIP sources: ties a committed traffic measurement to the kernels it was taken on."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2008_12214_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".inc")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def committed_traffic(batch):
    """HBM bytes per column-pass launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel sources and launches of this many problems; else None."""
    path = os.path.join(ROOT, "profiles", "wgs1024_colpass_traffic.json")
    try:
        t = json.load(open(path))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash() or t.get("problems_per_launch") != batch:
        return None
    return t.get("hbm_bytes_per_launch")


def copy_calibration(nbytes=1 << 30, reps=5):
    """A plain device copy of known size, for calibrating the FETCH_SIZE/WRITE_SIZE counters."""
    import torch
    dev = torch.device("cuda:0")
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize(dev)
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}), flush=True)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(budget_s=20.0):
    """FP64 oracle weighted GS on one 1024^2 target: iterations per second."""
    import numpy as np
    import synth
    from oracle import hologram
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    T = synth.gaussian_target(N, seed=2)
    t0 = time.perf_counter()
    hologram.gs(T, 1, LEVELS, seed=1, weighted=True)
    t1 = time.perf_counter() - t0  # one iteration + final evaluation
    k = int(max(2, min(50, budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    hologram.gs(T, k, LEVELS, seed=1, weighted=True)
    dt = time.perf_counter() - t0
    return {"value": k / dt, "unit": "iter/s", "cores": int(cores), "kind": "oracle",
            "sample": f"one 1024x1024 binary weighted-GS hologram, {k} iterations (+1 final "
                      f"evaluation), FP64 DFT-matrix oracle, {dt:.1f} s"}


def oracle_scaling(sizes=(64, 512, 1024, 2048)):
    """Seconds per weighted binary GS iteration of the FP64 oracle at several
    grid sizes, on every BLAS thread of this host and on one: context for the
    cpu_baseline figure (one iteration per size and thread count, after a
    warm-up iteration at the smaller sizes)."""
    import platform
    import numpy as np
    import synth
    from oracle import hologram
    from threadpoolctl import threadpool_info, threadpool_limits
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    out = {"cpu_model": model, "logical_cpus": os.cpu_count(), "blas_threads": threads, "per_iteration_s": {}}
    for n in sizes:
        T = hologram.prepare_target(synth.gaussian_target(n, seed=2), 2)
        f = np.exp(2j * np.pi * np.random.default_rng(1).random((n, n)))
        w = np.ones((n, n))
        row = {}
        for label, limit in (("all_threads", None), ("one_thread", 1)):
            with threadpool_limits(limits=limit):
                if n <= 1024:
                    hologram.gs_step(T, 2, f, weighted=True, w_prev=w, next_nmse=False)
                t0 = time.perf_counter()
                hologram.gs_step(T, 2, f, weighted=True, w_prev=w, next_nmse=False)
                row[label] = round(time.perf_counter() - t0, 4)
        out["per_iteration_s"][f"{n}x{n}"] = row
        log(f"oracle {n}^2: {row}")
    return out


def learned_time_to_nmse(n_eval=64):
    """The learned start (trained weights shipped with the package) against
    plain GS from a random phase and against GS from the quadratic start, on
    held-out 512^2 targets with 8 levels: the time-to-NMSE half of the
    metric.  Returns a compact summary (medians over the targets)."""
    import torch
    from paper_2008_12214_amd import learned
    dev = torch.device("cuda:0")
    params = learned.load_params(device=dev)
    targets = learned.make_targets(512, range(900000, 900000 + n_eval), device=dev)
    r = learned.evaluate(params, targets, levels=8, refine=10, gs_iters=200)
    L, Q = r["learned"], r["quadratic_only"]
    return {"workload": f"learned start + 10 GS, 512x512, 8 levels, {n_eval} held-out targets",
            "learned_final_nmse_median": round(L["final_nmse_median"], 5),
            "plain_gs_nmse_median_at_200": round(r["gs_nmse_median_at"]["200"], 5),
            "plain_gs_reached_fraction": L["gs_reached_fraction"],
            "time_gain_vs_plain_gs_median": round(L["time_gain_median"], 3),
            "time_gain_vs_plain_gs_is_lower_bound": L["gs_reached_fraction"] < 1.0,
            "time_gain_vs_quadratic_start_gs_median": round(L["time_gain_vs_quadratic_gs_median"], 3),
            "quadratic_only_final_nmse_median": round(Q["final_nmse_median"], 5),
            "quadratic_only_time_gain_vs_plain_gs_median": round(Q["time_gain_median"], 3),
            "network_forward_us_per_image": round(r["forward_ms_batch"] / n_eval * 1e3, 2),
            "gs_us_per_hologram_iteration": round(r["gs_ms_per_iter_batch"] / n_eval * 1e3, 3)}


def torchfft_context(B, iters=10):
    """Context only, not the product: the weighted binary GS loop of the default
    workload written as unfused torch ops on the same GPU (torch.fft = rocFFT,
    complex64): two library 2D FFTs plus element-wise and reduction kernels per
    iteration.  Returns hologram-iterations per second."""
    import torch
    import synth
    dev = torch.device("cuda:0")
    T = torch.stack([torch.from_numpy(synth.gaussian_target(N, seed=2, batch_item=b)) for b in range(B)]).to(dev)
    T = T * torch.sqrt(N * N / (T * T).sum(dim=(1, 2), keepdim=True))
    f = torch.exp(2j * torch.pi * torch.rand((B, N, N), device=dev)).to(torch.complex64)
    w = torch.ones_like(T)
    om = T > 0

    def step(f, w):
        R = torch.fft.fft2(f, norm="ortho")
        A = R.abs()
        _ = (T * A).sum(dim=(1, 2)), (A * A).sum(dim=(1, 2))  # NMSE sums
        m = (w * om).sum(dim=(1, 2), keepdim=True) / om.sum(dim=(1, 2), keepdim=True)
        ratio = torch.clamp(T, min=0.1) / torch.clamp(A, min=0.1)
        w = torch.where(om, torch.clamp(w * ratio / m, 1e-6, 1e6) ** 0.7, w)
        Rp = w * T * R / torch.clamp(A, min=1e-30)
        g = torch.fft.ifft2(Rp, norm="ortho")
        return torch.where(g.real < 0, -1.0, 1.0).to(torch.complex64), w

    for _ in range(2):
        f, w = step(f, w)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(iters):
        f, w = step(f, w)
    torch.cuda.synchronize(dev)
    return B * iters / (time.perf_counter() - t0)


def search_workload(args):
    """Holographic search: 256 binary holograms of 64 x 64 pixels, direct
    search from random levels until a sweep keeps no change (at most 40
    sweeps), one call.  value = pixel trials per second (one trial = one
    proposed level change, whose error change sums over all 4096 replay
    pixels)."""
    import numpy as np
    import torch
    import synth
    import paper_2008_12214_amd as hg
    dev = torch.device("cuda:0")
    B, n, L, max_sw = 256, 64, 2, 40
    T = torch.from_numpy(np.stack([synth.gaussian_target(n, seed=61, batch_item=b) for b in range(B)])).to(dev)
    init = torch.from_numpy(np.random.default_rng(7).integers(0, L, (B, n, n)).astype(np.uint8)).to(dev)
    ws = torch.empty(hg.hg_search_workspace_size(n, n, B), dtype=torch.uint8, device=dev)
    out = hg.hg_search(T, L, hg.HG_SEARCH_DS, max_sw, init, workspace=ws)  # warm-up
    torch.cuda.synchronize(dev)
    times = []
    for _ in range(max(1, args.steps)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        out = hg.hg_search(T, L, hg.HG_SEARCH_DS, max_sw, init, workspace=ws)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b) * 1e-3)
    med = sorted(times)[len(times) // 2]
    sweeps = out["sweeps"].cpu().numpy()
    trials = int(np.sum(sweeps)) * n * n * (L - 1)
    flops_per_trial = 22 * n * n  # per replay pixel: kernel and change products, modulus, error terms
    achieved = trials * flops_per_trial / med / 1e12
    err = out["error"].cpu().numpy()
    log(f"search: {trials} trials in {med * 1e3:.1f} ms, {trials / med:.3e} trials/s")
    res = {"metric": "pixel trials/s (holographic direct search)", "value": round(trials / med, 1),
           "unit": "trials/s", "n_gpus": 1, "steps": len(times), "warmup": 1,
           "ms_per_step": round(med * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "direct_search_binary_64x64_x256", "batch": B, "grid": [n, n], "slm_levels": L,
                      "max_sweeps": max_sw, "start": "uniform random levels"},
           "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": 157.3, "unit": "TFLOP/s",
                        "frac": round(achieved / 157.3, 4), "traffic": None,
                        "kernel": "k_search<64,64> (one workgroup per hologram, sequential trials)",
                        "flop_per_trial": flops_per_trial},
           "cpu_baseline": None,
           "extra": {"sweeps_median": float(np.median(sweeps)), "us_per_trial_per_hologram": round(
               med / (np.max(sweeps) * n * n * (L - 1)) * 1e6, 3),
               "error_median_start": float(np.median(err[:, 0])),
               "error_median_final": float(np.median(err[np.arange(B), sweeps]))}}
    print(json.dumps(res), flush=True)


def other_workload(args):
    """The non-headline workloads, one JSON line each.  The timed region is K
    replays of a HIP graph holding one whole library call (set-up, every
    iteration or subframe, NMSE finisher); the eager rate of the same call
    and per-kernel hipEvent times of an instrumented eager pass are reported
    beside it."""
    import ctypes
    import torch
    import synth
    import paper_2008_12214_amd as hg
    from paper_2008_12214_amd._binding import hg_problem

    dev = torch.device("cuda:0")
    lib = hg.lib()
    wl = args.workload

    def cur_stream():
        return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)

    def check(st):
        if st != 0:
            raise RuntimeError(hg.hg_last_error())

    if wl == "gs64":
        n, iters, levels = 64, 50, 8
        T = torch.from_numpy(synth.uniform_target(n, n, seed=1)).to(dev)
        lv = torch.empty((n, n), dtype=torch.uint8, device=dev)
        nm = torch.empty(iters + 1, dtype=torch.float64, device=dev)
        nb = lib.hg_workspace_size(hg.HG_OP_GS, n, n, iters)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)

        def step():
            check(lib.hg_gs(ctypes.c_void_p(T.data_ptr()), n, n, iters, levels, 1, None, None, 0.0, 0.0, 0.0,
                            ctypes.c_void_p(lv.data_ptr()), None, None, ctypes.c_void_p(nm.data_ptr()),
                            ctypes.c_void_p(ws.data_ptr()), nb, cur_stream()))
        px, units, unit = n * n, iters, "iter/s"
        bytes_col = px * (iters * 20 + 12)
        bytes_row = px * (8 + iters * 16 + 1)
        config = {"workload": "gs_8level_64x64_50it", "grid": [n, n], "iters": iters, "slm_levels": levels,
                  "target": "sqrt of uniform intensity"}
        kernel = "single-launch small-problem kernel k_small<64,64> (multi-launch: column pass k_col<64>)"
    elif wl == "ospr512":
        n, sub = 512, 24
        T = torch.from_numpy(synth.gaussian_target(n, seed=3)).to(dev)
        lv = torch.empty((sub, n, n), dtype=torch.uint8, device=dev)
        nm = torch.empty(sub, dtype=torch.float64, device=dev)
        nb = lib.hg_workspace_size(hg.HG_OP_OSPR, n, n, sub)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)

        def step():
            check(lib.hg_ospr(ctypes.c_void_p(T.data_ptr()), n, n, sub, 1, 3, ctypes.c_void_p(lv.data_ptr()),
                              ctypes.c_void_p(nm.data_ptr()), None, ctypes.c_void_p(ws.data_ptr()), nb,
                              cur_stream()))
        px, units, unit = n * n, sub, "subframes/s"
        # column launches: first (T r 4 omega, field w 8), subframes 2..N (field r+w 16, T 4 omega,
        # accumulator r+w 8; no read for subframe 2), final (field r 8, T 4 omega); T is read on its
        # support only (omega: support fraction of the symmetrised binary target); row: field r+w 16
        # + levels w 1
        om = support_of(T.cpu().numpy(), True)
        bytes_col = px * (8 + 24 * (sub - 1) - 4 + 8 + 4 * om * (sub + 1))
        bytes_row = px * 17 * sub
        config = {"workload": "adaptive_ospr_binary_512x512_24sf", "grid": [n, n], "subframes": sub,
                  "slm_levels": 2, "target": "gaussian sum, 32 blobs, central window"}
        kernel = "column pass of adaptive OSPR (4-column tiles, 8 elements per thread, k_colq_ospr<512,4,COL_OSPR,8>)"
    elif wl == "ospr1024x32":
        n, B, sub = 1024, 32, 24
        tg = [torch.from_numpy(synth.gaussian_target(n, seed=3, batch_item=b)).to(dev) for b in range(B)]
        lv = [torch.empty((sub, n, n), dtype=torch.uint8, device=dev) for _ in range(B)]
        nm = [torch.empty(sub, dtype=torch.float64, device=dev) for _ in range(B)]
        P = hg._binding.hg_ospr_problem
        arr = (P * B)()
        for b in range(B):
            arr[b] = P(n, n, 3, tg[b].data_ptr(), lv[b].data_ptr(), nm[b].data_ptr(), None)
        nb = lib.hg_ospr_batched_workspace_size(arr, B, sub)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)

        def step():
            check(lib.hg_ospr_batched(arr, B, sub, 1, ctypes.c_void_p(ws.data_ptr()), nb, cur_stream()))
        px, units, unit = n * n * B, sub * B, "subframes/s"
        om = sum(support_of(x.cpu().numpy(), True) for x in tg) / B  # as for ospr512
        bytes_col = px * (8 + 24 * (sub - 1) - 4 + 8 + 4 * om * (sub + 1))
        bytes_row = px * 17 * sub
        config = {"workload": "adaptive_ospr_binary_1024x1024_24sf_x32", "batch": B, "grid": [n, n],
                  "subframes": sub, "slm_levels": 2, "target": "gaussian sum, 32 blobs, central window"}
        kernel = "column pass of adaptive OSPR (one tile per workgroup, k_colq_ospr<1024,4,COL_OSPR>)"
    elif wl == "lt1024":
        n, B, iters, levels = 1024, 32, 100, 2
        tnp = [synth.gaussian_target(n, seed=2, batch_item=b) for b in range(B)]
        tg = [torch.from_numpy(a).to(dev) for a in tnp]
        lv = [torch.empty((n, n), dtype=torch.uint8, device=dev) for _ in range(B)]
        nm = [torch.empty(iters + 1, dtype=torch.float64, device=dev) for _ in range(B)]
        arr = (hg_problem * B)()
        for b in range(B):
            arr[b] = hg_problem(n, n, levels, iters, 1, 0.0, 0.0, 0.0, tg[b].data_ptr(), lv[b].data_ptr(),
                                nm[b].data_ptr())
            arr[b].lt, arr[b].lt_r0, arr[b].lt_dr = 1, 256, 4
        nb = lib.hg_gs_batched_workspace_size(arr, B)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)

        def step():
            check(lib.hg_gs_batched(arr, B, 0, ctypes.c_void_p(ws.data_ptr()), nb, cur_stream()))
        px = n * n * B
        units, unit = iters * B, "iter/s"
        # tile column kernel: field r+w 16 + target 4 on its support (binary: symmetrised)
        om = sum(support_of(a, True) for a in tnp) / B
        bytes_col = px * (iters * (16 + 4 * om) + 12)
        bytes_row = px * (8 + iters * 16 + 1)
        config = {"workload": "lt_binary_1024x1024_100it", "batch": B, "grid": [n, n], "iters": iters,
                  "slm_levels": levels, "lt_r0": 256, "lt_dr": 4, "target": "gaussian sum, 32 blobs, central window"}
        kernel = "column pass of Liu-Taghizadeh (one tile per workgroup, k_colq<1024,4,COL_GS>)"
    elif wl == "wgs1024f16":
        n, B, iters = 1024, 32, 100
        levels = 2 | hg.HG_FIELD_FP16  # the headline batch with the field held as binary16 pairs
        tnp = [synth.gaussian_target(n, seed=2, batch_item=b) for b in range(B)]
        tg = [torch.from_numpy(a).to(dev) for a in tnp]
        lv = [torch.empty((n, n), dtype=torch.uint8, device=dev) for _ in range(B)]
        nm = [torch.empty(iters + 1, dtype=torch.float64, device=dev) for _ in range(B)]
        arr = (hg_problem * B)()
        for b in range(B):
            arr[b] = hg_problem(n, n, levels, iters, 1, 0.0, 0.0, 0.0, tg[b].data_ptr(), lv[b].data_ptr(),
                                nm[b].data_ptr())
        nb = lib.hg_gs_batched_workspace_size(arr, B)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)

        def step():
            check(lib.hg_gs_batched(arr, B, 1, ctypes.c_void_p(ws.data_ptr()), nb, cur_stream()))
        px = n * n * B
        units, unit = iters * B, "iter/s"
        # 16-bit field: weighted column pass field r+w 8 + 12 omega B/px, final
        # pass field 4 + target 4 (wave kernel, target everywhere), rows 8
        om = sum(support_of(a, True) for a in tnp) / B
        bytes_col = px * (iters * (8 + 12 * om) + 8)
        bytes_row = px * (4 + iters * 8 + 1)
        config = {"workload": "wgs_binary_1024x1024_100it_field16", "batch": B, "grid": [n, n], "iters": iters,
                  "slm_levels": 2, "field_storage": "binary16 pairs",
                  "target": "gaussian sum, 32 blobs, central window"}
        kernel = "column pass of weighted GS, 16-bit field (k_colq<1024,4,COL_WGS,16,false,true>)"
    elif wl == "amp1024":
        n, B, iters = 1024, 32, 100
        levels = 2 | hg.HG_SLM_AMPLITUDE  # binary amplitude SLM, transmissions {0, 1}
        tnp = [synth.gaussian_target(n, seed=2, batch_item=b) for b in range(B)]
        tg = [torch.from_numpy(a).to(dev) for a in tnp]
        lv = [torch.empty((n, n), dtype=torch.uint8, device=dev) for _ in range(B)]
        nm = [torch.empty(iters + 1, dtype=torch.float64, device=dev) for _ in range(B)]
        arr = (hg_problem * B)()
        for b in range(B):
            arr[b] = hg_problem(n, n, levels, iters, 1, 0.0, 0.0, 0.0, tg[b].data_ptr(), lv[b].data_ptr(),
                                nm[b].data_ptr())
        nb = lib.hg_gs_batched_workspace_size(arr, B)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)

        def step():
            check(lib.hg_gs_batched(arr, B, 1, ctypes.c_void_p(ws.data_ptr()), nb, cur_stream()))
        px = n * n * B
        units, unit = iters * B, "iter/s"
        # as the headline: weighted column pass 16 + 12 omega B/px (target
        # symmetrised, as for every amplitude SLM), final pass 12, rows 16
        om = sum(support_of(a, True) for a in tnp) / B
        bytes_col = px * (iters * (16 + 12 * om) + 12)
        bytes_row = px * (8 + iters * 16 + 1)
        config = {"workload": "wgs_binary_amplitude_1024x1024_100it", "batch": B, "grid": [n, n], "iters": iters,
                  "slm": "binary amplitude {0, 1}", "target": "gaussian sum, 32 blobs, central window"}
        kernel = "column pass of weighted GS (one tile per workgroup, k_colq<1024,4,COL_WGS>)"
    else:
        sizes = synth.batch_mix()
        iters, levels = 50, 8
        B = len(sizes)
        tnp = [synth.gaussian_target(s, seed=4, batch_item=b) for b, s in enumerate(sizes)]
        tg = [torch.from_numpy(a).to(dev) for a in tnp]
        lv = [torch.empty((s, s), dtype=torch.uint8, device=dev) for s in sizes]
        nm = [torch.empty(iters + 1, dtype=torch.float64, device=dev) for _ in sizes]
        arr = (hg_problem * B)()
        for b, s in enumerate(sizes):
            arr[b] = hg_problem(s, s, levels, iters, 1000 + b, synth.WAVELENGTH_M, synth.PITCH_M,
                                synth.fresnel_z(4, b), tg[b].data_ptr(), lv[b].data_ptr(), nm[b].data_ptr())
        nb = lib.hg_gs_batched_workspace_size(arr, B)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)

        def step():
            check(lib.hg_gs_batched(arr, B, 0, ctypes.c_void_p(ws.data_ptr()), nb, cur_stream()))
        px = sum(s * s for s in sizes)
        units, unit = iters, "batch-iter/s"
        # 512^2 and 1024^2 run the tile column kernel (target read on its
        # support only: 16 + 4 omega B/px); 256^2 and 2048^2 the classic
        # kernels (target read everywhere: 20 B/px)
        per_iter = sum(s * s * ((16 + 4 * support_of(tnp[b], False)) if s in (512, 1024) else 20)
                       for b, s in enumerate(sizes))
        bytes_col = iters * per_iter + 12 * px
        bytes_row = px * (8 + iters * 16 + 1)
        config = {"workload": "batched_uneven_fresnel_8level_50it", "problems": B,
                  "sizes": {str(s): sizes.count(s) for s in sorted(set(sizes))}, "pixels": px, "iters": iters,
                  "slm_levels": levels, "wavelength_m": synth.WAVELENGTH_M, "pitch_m": synth.PITCH_M,
                  "z_m": "uniform [0.1, 0.5]"}
        kernel = "column pass of Fresnel GS, all size classes (k_colq / k_col)"

    log(f"{wl}: warmup {args.warmup}, steps {args.steps}")
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize(dev)
    k = args.steps
    t0 = time.perf_counter()
    for _ in range(k):
        step()
    torch.cuda.synchronize(dev)
    eager = (time.perf_counter() - t0) / k

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for _ in range(max(1, args.warmup)):
        g.replay()
    torch.cuda.synchronize(dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        g.replay()
        b.record()
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    per = sorted(a.elapsed_time(b) * 1e-3 for a, b in ev)
    med = per[len(per) // 2]

    multi = None
    if wl == "gs64":
        # the same call through the multi-launch pipeline, for comparison
        hg.hg_set_small_fused(0)
        step()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(k):
            step()
        torch.cuda.synchronize(dev)
        multi = (time.perf_counter() - t0) / k
        hg.hg_set_small_fused(1)

    hg.hg_timing_enable(True)
    hg.hg_timing_read()
    step()
    torch.cuda.synchronize(dev)
    kt = hg.hg_timing_read()
    hg.hg_timing_enable(False)
    call_gbs = (bytes_col + bytes_row) / med / 1e9
    if kt["row_launches"] == 0:
        # single-launch small-problem kernel: the field never leaves LDS, so
        # the call is a latency figure, not an HBM one
        fused_us = kt["col_ms"] / kt["col_launches"] * 1e3
        log(f"graph median {med * 1e3:.4f} ms/call, eager {eager * 1e3:.4f} ms/call; single launch {fused_us:.1f} us")
        roof = None
        row = None
        kernel_us = {"single_launch_us": round(fused_us, 2)}
    else:
        col_gbs = bytes_col / (kt["col_ms"] * 1e-3) / 1e9
        row_gbs = bytes_row / (kt["row_ms"] * 1e-3) / 1e9
        log(f"graph median {med * 1e3:.3f} ms/call, eager {eager * 1e3:.3f} ms/call; column {col_gbs:.0f} GB/s, "
            f"row {row_gbs:.0f} GB/s, whole call {call_gbs:.0f} GB/s")
        roof = {"bound": "hbm", "achieved": round(col_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(col_gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": kernel,
                "bytes_per_launch": int(bytes_col / kt["col_launches"]),
                "avg_launch_us": round(kt["col_ms"] / kt["col_launches"] * 1e3, 2)}
        row = {"avg_launch_us": round(kt["row_ms"] / kt["row_launches"] * 1e3, 2), "achieved_GBs": round(row_gbs, 1)}
        kernel_us = None
    out = {
        "metric": f"{unit} ({wl})", "value": round(units / med, 1), "unit": unit, "n_gpus": 1, "steps": k,
        "warmup": args.warmup, "ms_per_step": round(wall / k * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": config,
        "roofline": roof,
        "cpu_baseline": None,
        "extra": {"graph_median_ms_per_call": round(med * 1e3, 4), "eager_ms_per_call": round(eager * 1e3, 4),
                  "eager_value": round(units / eager, 1), "row_pass": row, "kernel": kernel_us,
                  "multi_launch_eager_ms_per_call": None if multi is None else round(multi * 1e3, 4),
                  "whole_call_algorithmic_GBs": round(call_gbs, 1),
                  "setup_ms": round(kt.get("setup_ms", 0.0), 4)},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-b1", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-start time-to-NMSE leg")
    ap.add_argument("--iters", type=int, default=100,
                    help="iterations per hologram (100 is the workload; fewer only for short profiles)")
    ap.add_argument("--workload", default="wgs1024",
                    choices=["wgs1024", "gs64", "ospr512", "ospr1024x32", "uneven", "lt1024", "amp1024",
                             "wgs1024f16", "search64"],
                    help="wgs1024 (default): the headline batch; gs64: one 64^2 8-level GS, latency; "
                         "ospr512: adaptive binary OSPR, 512^2, 24 subframes; uneven: 256 Fresnel problems "
                         "of four sizes, 8 levels, 50 iterations; lt1024: 32 binary Liu-Taghizadeh problems "
                         "of 1024^2, 100 iterations, region radius 256 + 4 per iteration; ospr1024x32: 32 "
                         "adaptive binary OSPR problems of 1024^2, 24 subframes, in one call; amp1024: the "
                         "headline batch on a binary amplitude SLM; wgs1024f16: the headline batch with 16-bit "
                         "field storage; search64: direct search on 256 binary 64^2 holograms")
    ap.add_argument("--context", action="store_true",
                    help="also time the same loop as unfused torch.fft (rocFFT) ops, for context")
    ap.add_argument("--oracle-scaling", action="store_true",
                    help="only time the FP64 oracle per iteration at 64^2..2048^2 on all BLAS threads and on one")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.oracle_scaling:
        print(json.dumps({"oracle_scaling": oracle_scaling()}), flush=True)
        return
    global ITERS
    ITERS = args.iters
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "search64":
        search_workload(args)
        return
    if args.workload != "wgs1024":
        other_workload(args)
        return

    import ctypes
    import torch
    import synth
    import paper_2008_12214_amd as hg
    from paper_2008_12214_amd._binding import hg_problem

    dev = torch.device("cuda:0")
    lib = hg.lib()

    def support_fraction(B):
        """Fraction of pixels on the binary-symmetrised target support, over the batch."""
        import numpy as np
        tot = 0.0
        for b in range(B):
            T = synth.gaussian_target(N, seed=2, batch_item=b)
            mir = T[(-np.arange(N)) % N][:, (-np.arange(N)) % N]
            tot += float(np.mean((T > 0) | (mir > 0)))
        return tot / B

    def setup(B):
        targets = [torch.from_numpy(synth.gaussian_target(N, seed=2, batch_item=b)).to(dev) for b in range(B)]
        levels = [torch.empty((N, N), dtype=torch.uint8, device=dev) for _ in range(B)]
        nmse = [torch.empty(ITERS + 1, dtype=torch.float64, device=dev) for _ in range(B)]
        arr = (hg_problem * B)()
        for b in range(B):
            arr[b] = hg_problem(N, N, LEVELS, ITERS, 1, 0.0, 0.0, 0.0, targets[b].data_ptr(),
                                levels[b].data_ptr(), nmse[b].data_ptr())
        nbytes = lib.hg_gs_batched_workspace_size(arr, B)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        stream = torch.cuda.current_stream(dev)
        sp = ctypes.c_void_p(stream.cuda_stream)

        def step():
            st = lib.hg_gs_batched(arr, B, 1, ctypes.c_void_p(ws.data_ptr()), nbytes, sp)
            if st != 0:
                raise RuntimeError(hg.hg_last_error())
        return step, (targets, levels, nmse, ws, arr)

    def timed(step, k):
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(k):
            step()
        torch.cuda.synchronize(dev)
        return time.perf_counter() - t0

    B = args.batch
    log(f"batch {B} x {N}^2 weighted GS, {ITERS} iterations, warmup {args.warmup}, steps {args.steps}")
    step, keep = setup(B)
    for _ in range(args.warmup):
        step()
    dt = timed(step, args.steps)
    value = B * ITERS * args.steps / dt
    log(f"timed {dt:.3f} s -> {value:.1f} hologram-iterations/s")
    nm_final = float(keep[2][0][-1].item())

    # instrumented pass: per-kernel device time with hipEvents on the launch stream
    hg.hg_timing_enable(True)
    hg.hg_timing_read()
    timed(step, args.steps)
    kt = hg.hg_timing_read()
    hg.hg_timing_enable(False)
    px = N * N * B
    omega = support_fraction(B)
    col_px_bytes = COL_FIELD_BYTES + COL_SUPPORT_BYTES * omega
    col_bytes = args.steps * (ITERS * col_px_bytes + COL_FINAL_BYTES) * px
    # row launches: one initial pass (writes the field, 8 B/px) + ITERS passes
    row_bytes = args.steps * (8 + ITERS * ROW_BYTES + 1) * px
    # the call runs in chunks of problems whose field planes fit the chunk size
    chunk = hg.hg_get_batch_chunk()
    per_launch = B if chunk == 0 else max(1, min(B, chunk // (N * N * 8)))
    col_avg_ms = kt["col_ms"] / kt["col_launches"]
    row_avg_ms = kt["row_ms"] / kt["row_launches"]
    col_gbs = col_bytes / (kt["col_ms"] * 1e-3) / 1e9
    row_gbs = row_bytes / (kt["row_ms"] * 1e-3) / 1e9
    iter_gbs = (ITERS * (col_px_bytes + ROW_BYTES)) * px * args.steps / dt / 1e9
    log(f"column pass avg {col_avg_ms * 1e3:.1f} us ({col_gbs:.0f} GB/s), row pass avg {row_avg_ms * 1e3:.1f} us "
        f"({row_gbs:.0f} GB/s)")
    del step, keep
    torch.cuda.empty_cache()

    b1 = None
    if not args.no_b1:
        step1, keep1 = setup(1)
        for _ in range(args.warmup):
            step1()
        k1 = max(args.steps, 10)
        dt1 = timed(step1, k1)
        b1 = {"iter_per_s": ITERS * k1 / dt1, "us_per_iteration": dt1 / (k1 * ITERS) * 1e6,
              "algorithmic_GBs": (col_px_bytes + ROW_BYTES) * N * N * ITERS * k1 / dt1 / 1e9}
        log(f"B=1: {b1['iter_per_s']:.0f} iter/s, {b1['us_per_iteration']:.1f} us/iteration")
        del step1, keep1

    ctx = None
    if args.context:
        log("context: unfused torch.fft (rocFFT) loop")
        ctx = {"kind": "unfused torch.fft (rocFFT) + torch element-wise ops, same GPU, not the product",
               "iter_per_s": round(torchfft_context(B), 1)}
        log(f"torch.fft loop {ctx['iter_per_s']:.0f} hologram-iterations/s")
        torch.cuda.empty_cache()

    learned_summary = None
    if not args.no_learned:
        log("learned start: time to NMSE")
        try:
            learned_summary = learned_time_to_nmse()
        except Exception as e:  # reported, not fatal: the headline line is still printed
            learned_summary = {"error": f"{type(e).__name__}: {e}"}
        log(f"learned start: {learned_summary}")
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline()
        log(f"oracle {cpu['value']:.3f} iter/s on {cpu['cores']} threads")

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"wgs_binary_{N}x{N}_{ITERS}it", "batch": B, "grid": [N, N], "iters": ITERS,
                   "slm_levels": LEVELS, "target": "gaussian sum, 32 blobs, central window"},
        "roofline": {"bound": "hbm", "achieved": round(col_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(col_gbs / HBM_PEAK_GBS, 4), "traffic": committed_traffic(per_launch),
                     "kernel": "column pass of weighted GS (one tile per workgroup, k_colq<1024,4,COL_WGS>)",
                     "bytes_per_launch": int(col_bytes / kt["col_launches"]),
                     "bytes_per_px": round(col_px_bytes, 3), "support_fraction": round(omega, 4),
                     "avg_launch_us": round(col_avg_ms * 1e3, 2), "problems_per_launch": per_launch,
                     "chunk_field_bytes": chunk},
        "cpu_baseline": cpu,
        "extra": {"row_pass": {"avg_launch_us": round(row_avg_ms * 1e3, 2), "achieved_GBs": round(row_gbs, 1)},
                  "whole_iteration_algorithmic_GBs": round(iter_gbs, 1),
                  "whole_iteration_frac": round(iter_gbs / HBM_PEAK_GBS, 4),
                  "per_hologram_iter_per_s": round(value / B, 1), "b1": b1, "library_context": ctx,
                  "final_nmse_item0": nm_final, "learned_init": learned_summary},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
