"""Non-finite inputs through the C ABI (GPU): a NaN in the target or in the
caller's weights makes every NMSE the finisher reports NaN, in every
column-pass kernel (the single-launch small kernel, the tile kernel, the
classic kernels), and hg_numeric_status reports HG_ERR_NUMERIC; the next
clean call with the same workspace reports HG_OK."""
import numpy as np
import pytest

import synth
from parity import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2008_12214_amd as hg  # noqa: E402

DEV = "cuda:0"


def _ws(op, n, iters):
    return torch.empty(hg.hg_workspace_size(op, n, n, iters), dtype=torch.uint8, device=DEV)


@pytest.mark.parametrize("n,kind", [(64, hg.COLUMN_TILE), (1024, hg.COLUMN_TILE), (1024, hg.COLUMN_CLASSIC),
                                    (2048, hg.COLUMN_TILE)])
def test_nan_target_gives_nan_nmse_and_numeric_status(n, kind):
    say("NaN target", n, kind)
    T = synth.gaussian_target(n, seed=2)
    bad = T.copy()
    bad[n // 2 + 3, n // 2 - 5] = np.nan  # inside the support
    ws = _ws(hg.HG_OP_WGS, n, 3)
    hg.hg_set_column_kernel(kind)
    try:
        out = hg.hg_wgs(torch.from_numpy(bad).to(DEV), 3, 2, seed=1, workspace=ws)
        nm = out["nmse"].cpu().numpy()
        assert np.all(np.isnan(nm)), nm
        with pytest.raises(hg.HologenError) as e:
            hg.hg_numeric_status(ws)
        assert e.value.status == hg.HG_ERR_NUMERIC
        out = hg.hg_wgs(torch.from_numpy(T).to(DEV), 3, 2, seed=1, workspace=ws)
        hg.hg_numeric_status(ws)  # clean call: no error
        assert np.all(np.isfinite(out["nmse"].cpu().numpy()))
    finally:
        hg.hg_set_column_kernel(hg.COLUMN_TILE)


def test_nan_weight_and_batched_status():
    say("NaN weight; batched call status")
    n = 256
    T = synth.gaussian_target(n, seed=3)
    w = np.ones((n, n), np.float32)
    w[n // 2, n // 2] = np.nan
    ws = _ws(hg.HG_OP_WGS, n, 2)
    out = hg.hg_wgs(torch.from_numpy(T).to(DEV), 2, 8, seed=1, weights=torch.from_numpy(w).to(DEV), workspace=ws)
    assert np.isnan(out["nmse"].cpu().numpy()[-1])
    with pytest.raises(hg.HologenError):
        hg.hg_numeric_status(ws)
    # a batched call: the NaN problem sits in the second size class
    Ts = [torch.from_numpy(synth.gaussian_target(m, seed=4, batch_item=i)).to(DEV) for i, m in enumerate((128, 256))]
    Tb = Ts[1].clone()
    Tb[5, 7] = float("nan")
    wsb = torch.empty(64 << 20, dtype=torch.uint8, device=DEV)
    lv, nm = hg.hg_gs_batched([Ts[0], Tb], 2, 4, workspace=wsb)
    assert np.all(np.isfinite(nm[0].cpu().numpy())) and np.all(np.isnan(nm[1].cpu().numpy()))
    with pytest.raises(hg.HologenError):
        hg.hg_numeric_status(wsb)
    hg.hg_gs_batched([Ts[0], Ts[1]], 2, 4, workspace=wsb)
    hg.hg_numeric_status(wsb)
