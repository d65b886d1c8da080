"""HIP graph capture of whole library calls (GPU).

A call enqueues only kernels on the caller's stream (no allocation, copy,
memset or host synchronisation), so a torch-captured graph of it replays
the same work.  Each replay is checked, bit for bit, against the eager
call, with eager work on the outputs between replays (they are cleared).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2008_12214_amd as hg  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print("[gpu-graph]", *a, flush=True)


def _check_replays(run, outputs_of, reps=3):
    ref = {k: v.clone() for k, v in outputs_of(run()).items()}
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        captured = outputs_of(run())
    for rep in range(reps):
        for v in captured.values():
            v.zero_()
        scratch = torch.randn(1 << 20, device=DEV).sum()  # unrelated eager work
        g.replay()
        torch.cuda.synchronize()
        for k, v in captured.items():
            assert torch.equal(v, ref[k]), (rep, k)
        del scratch
    return ref


def test_gs_64_8level_graph_replays():
    say("GS 64^2, 8 levels, 50 iterations")
    T = torch.from_numpy(synth.uniform_target(64, 64, seed=1)).to(DEV)
    ws = torch.empty(hg.hg_workspace_size(hg.HG_OP_GS, 64, 64, 50), dtype=torch.uint8, device=DEV)
    ref = _check_replays(lambda: hg.hg_gs(T, 50, 8, seed=1, workspace=ws),
                         lambda o: {"levels": o["levels"], "nmse": o["nmse"]})
    assert np.isfinite(ref["nmse"].cpu().numpy()).all()


def test_wgs_binary_256_graph_replays():
    say("weighted GS 256^2, binary, 20 iterations, caller weights")
    T = torch.from_numpy(synth.gaussian_target(256, seed=2)).to(DEV)
    w = torch.ones((256, 256), dtype=torch.float32, device=DEV)
    ws = torch.empty(hg.hg_workspace_size(hg.HG_OP_WGS, 256, 256, 20), dtype=torch.uint8, device=DEV)

    def run():
        w.fill_(1.0)
        return hg.hg_wgs(T, 20, 2, seed=3, weights=w, workspace=ws)
    _check_replays(run, lambda o: {"levels": o["levels"], "nmse": o["nmse"], "weights": w})


def test_ospr_adaptive_512_graph_replays():
    say("adaptive OSPR 512^2, 8 subframes")
    T = torch.from_numpy(synth.gaussian_target(512, seed=3)).to(DEV)
    ws = torch.empty(hg.hg_workspace_size(hg.HG_OP_OSPR, 512, 512, 8), dtype=torch.uint8, device=DEV)
    _check_replays(lambda: hg.hg_ospr(T, 8, True, seed=5, workspace=ws),
                   lambda o: {"levels": o["levels"], "nmse": o["nmse"]})
