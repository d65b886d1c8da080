"""Batched GS in chunks (GPU).

hg_gs_batched runs each size class in chunks of problems whose field planes
fit a byte budget, one chunk after another.  Every problem keeps its own
Philox item and its own fixed-order sums, so levels, NMSE histories, weights
and replays must be bit-identical for every chunk size, including a chunk of
one problem and no chunking at all.  The mixed batch spans several size
classes (Fourier and Fresnel, 8-level and binary, 16-bit field storage) with
class sizes that the chunk sizes do not divide, and a class of 64 problems of
256^2, whose column pass runs the persistent pipelined kernel (at least 2048
column tiles per launch) for the whole class and so for each of its chunks.
"""
import numpy as np
import pytest

import synth
from parity import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2008_12214_amd as hg  # noqa: E402

DEV = "cuda:0"


@pytest.fixture
def restore_chunk():
    old = hg.hg_get_batch_chunk()
    yield
    hg.hg_set_batch_chunk(old)


def _mixed():
    shapes = [(256, 256)] * 5 + [(512, 256)] * 3 + [(1024, 1024)] * 3
    Ts = [synth.gaussian_target(nx, seed=11, batch_item=i, ny=ny) for i, (ny, nx) in enumerate(shapes)]
    levels = [8 if i % 2 else 2 for i in range(len(shapes))]
    optics = [(5.32e-7, 8e-6, 0.3) if i % 3 == 0 else (0.0, 0.0, 0.0) for i in range(len(shapes))]
    return Ts, levels, optics


def _run(Ts, levels, optics, weighted, iters):
    tg = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.float32)).to(DEV) for t in Ts]
    wts = [torch.ones(t.shape, dtype=torch.float32, device=DEV) for t in Ts] if weighted else None
    lv, nm, rp = hg.hg_gs_batched(tg, iters, levels, seeds=[5] * len(Ts), optics=optics, weighted=weighted,
                                  weights=wts, want_replay=True)
    torch.cuda.synchronize()
    return ([x.cpu() for x in lv], [x.cpu() for x in nm], [x.cpu() for x in rp],
            [x.cpu() for x in wts] if weighted else None)


@pytest.mark.parametrize("weighted", [False, True])
def test_chunked_batch_is_bit_identical(weighted, restore_chunk):
    Ts, levels, optics = _mixed()
    iters = 6
    hg.hg_set_batch_chunk(0)
    ref = _run(Ts, levels, optics, weighted, iters)
    # 1 MiB: two 256^2 problems, one 512x256 problem, one 1024^2 problem per
    # chunk; 20 MiB: two 1024^2 problems, the small classes whole
    for chunk in (1 << 20, 20 << 20, 128 << 20):
        say(f"chunk {chunk >> 20} MiB, weighted {weighted}")
        hg.hg_set_batch_chunk(chunk)
        got = _run(Ts, levels, optics, weighted, iters)
        for part, (a, b) in enumerate(zip(ref, got)):
            if a is None:
                continue
            for i, (x, y) in enumerate(zip(a, b)):
                assert torch.equal(x, y), f"chunk {chunk}: output {part} of problem {i} differs"


def test_chunked_field16_batch_is_bit_identical(restore_chunk):
    Ts = [synth.gaussian_target(256, seed=3, batch_item=i) for i in range(5)]
    L = 2 | hg.HG_FIELD_FP16
    hg.hg_set_batch_chunk(0)
    ref = _run(Ts, [L] * 5, None, True, 5)
    hg.hg_set_batch_chunk(2 * 256 * 256 * 4)  # two problems of 4-byte elements per chunk
    got = _run(Ts, [L] * 5, None, True, 5)
    for part, (a, b) in enumerate(zip(ref, got)):
        for i, (x, y) in enumerate(zip(a, b)):
            assert torch.equal(x, y), f"output {part} of problem {i} differs"


def test_chunks_keep_the_class_kernel(restore_chunk):
    Ts = [synth.gaussian_target(256, seed=4, batch_item=i) for i in range(64)]
    hg.hg_set_batch_chunk(0)
    ref = _run(Ts, [2] * 64, None, True, 4)
    hg.hg_set_batch_chunk(3 * 256 * 256 * 8)  # three problems per chunk, 22 chunks
    got = _run(Ts, [2] * 64, None, True, 4)
    for part, (a, b) in enumerate(zip(ref, got)):
        for i, (x, y) in enumerate(zip(a, b)):
            assert torch.equal(x, y), f"output {part} of problem {i} differs"


def test_chunked_ospr_batch_is_bit_identical(restore_chunk):
    """Batched adaptive OSPR in chunks (counted by field planes, as for GS):
    subframe levels, NMSE and the accumulated intensity equal those of the
    whole call.  The 512^2 class of
    three problems keeps its small-batch kernels in every chunk."""
    shapes = [512] * 3 + [256] * 4
    Ts = [torch.from_numpy(synth.gaussian_target(n, seed=6, batch_item=i)).to(DEV) for i, n in enumerate(shapes)]
    out = {}
    for chunk in (0, 512 * 512 * 8, 2 * 256 * 256 * 8):
        say(f"OSPR chunk {chunk} bytes")
        hg.hg_set_batch_chunk(chunk)
        lv, nm, ac = hg.hg_ospr_batched(Ts, 6, True, seeds=[9] * len(Ts), want_accum=True)
        torch.cuda.synchronize()
        out[chunk] = [x.cpu() for x in lv + nm + ac]
    for chunk, got in out.items():
        for i, (x, y) in enumerate(zip(out[0], got)):
            assert torch.equal(x, y), f"chunk {chunk}: output {i} differs"
