"""The mixed-precision workload at full size (N = 262144 points in d = 28,
i.i.d. normal; kernel exp(-r/4); leaf 256; tol 1e-4; rank <= 256; HSS;
W: N x 1024), in the launch configuration the benchmark times, against the
oracle's own compression and tree walk on sampled columns (column j of Y
depends only on column j of W):
  * FP64: <= 1e-10 relative (Frobenius), elementwise within 1e-12 max|Y|;
  * near and far blocks computed from the points and skeletons, on a store
    loaded without them: the same FP64 bar;
  * split BF16 (near, far and leaf-basis products; FP64 transfers): within
    the workload's compression tolerance 1e-4;
  * FP32: 2e-5 against the oracle on the FP32-rounded columns (FP32 rounding
    of blocks and W, FP32 accumulation over contractions up to 512).
The oracle compresses this matrix in one to two minutes on the host cores."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle.oracle import OracleH2
from tests.helpers import rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(900)
def test_c4_full_size_sampled_columns():
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_1812_07152_amd as hmx
    w = wl.C4
    X = wl.gen_points(w)
    _say("[c4] oracle compression (N=262144, d=28, HSS, rank <= 256)")
    H = OracleH2.from_workload(w, X)
    W = wl.gen_w(w)
    cols = np.random.default_rng(44).choice(w.Q, 4, replace=False)
    Wc = np.ascontiguousarray(W[:, cols])
    _say("[c4] oracle tree walk on 4 columns")
    Yref = H.eval(Wc)
    Yref32 = H.eval(np.ascontiguousarray(Wc.astype(np.float32).astype(np.float64)))
    tol_el = 1e-12 * np.abs(Yref).max()

    M = hmx.hm_load_compressed_mem(H, 0, hmx.precbit(hmx.HM_PREC_FP64) | hmx.precbit(hmx.HM_PREC_BF16X3)
                                   | hmx.precbit(hmx.HM_PREC_FP32))
    Wd = torch.from_numpy(W).cuda()
    Yd = torch.full_like(Wd, float("nan"))
    _say("[c4] gpu FP64 eval Q=1024")
    hmx.hm_eval(M, Wd, Yd)
    hmx.hm_check(M)
    Y = Yd[:, torch.from_numpy(cols).cuda()].cpu().numpy()
    err = rel(Y, Yref)
    _say(f"[c4] FP64 rel err vs oracle {err:.3e}")
    assert err <= 1e-10
    np.testing.assert_allclose(Y, Yref, rtol=0, atol=tol_el)

    _say("[c4] gpu split-BF16 eval Q=1024")
    hmx.hm_eval(M, Wd, Yd, prec=hmx.HM_PREC_BF16X3)
    hmx.hm_check(M)
    err = rel(Yd[:, torch.from_numpy(cols).cuda()].cpu().numpy(), Yref)
    _say(f"[c4] split-BF16 rel err vs oracle {err:.3e}")
    assert err <= w.tol

    _say("[c4] gpu FP32 eval Q=1024")
    W32 = Wd.float()
    Y32 = torch.full_like(W32, float("nan"))
    hmx.hm_eval(M, W32, Y32)
    hmx.hm_check(M)
    err = rel(Y32[:, torch.from_numpy(cols).cuda()].double().cpu().numpy(), Yref32)
    _say(f"[c4] FP32 rel err vs oracle {err:.3e}")
    assert err <= 2e-5
    del M, W32, Y32

    _say("[c4] gpu FP64 with near and far blocks from the points")
    Mp = hmx.hm_load_compressed_mem(H, 0, hmx.precbit(hmx.HM_PREC_FP64) | hmx.HM_LOAD_NO_NEAR_BLOCKS
                                    | hmx.HM_LOAD_NO_FAR_BLOCKS)
    hmx.hm_set_points(Mp, X, w.kernel, w.h)
    hmx.hm_eval(Mp, Wd, Yd, flags=hmx.HM_NEAR_FROM_POINTS | hmx.HM_FAR_FROM_POINTS)
    hmx.hm_check(Mp)
    Y = Yd[:, torch.from_numpy(cols).cuda()].cpu().numpy()
    err = rel(Y, Yref)
    _say(f"[c4] from points rel err vs oracle {err:.3e}")
    assert err <= 1e-10
    np.testing.assert_allclose(Y, Yref, rtol=0, atol=tol_el)
