"""Batched form: several matrices of uneven size, rank and width in one
persistent launch (hm_batch_*), checked against the oracle and against the
same matrices evaluated one by one with hm_eval."""
import numpy as np
import pytest

import workloads as wl
from oracle.oracle import OracleH2
from tests.helpers import rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SPECS = [
    wl.small("b0", N=700, d=3, m=32, Q=5, seed=11),
    wl.small("b1", N=1500, d=8, points="mixture", m=48, h=1.0, Q=17, seed=12),
    wl.small("b2", N=3000, d=3, m=64, Q=64, h=0.4, seed=13),
    wl.small("b3", N=2048, d=3, m=40, adm=wl.ADM_HSS, kernel=wl.KERNEL_LAPLACE, h=2.0, rmax=40, Q=100, seed=14),
    wl.small("b4", N=4096, d=8, points="mixture", m=64, h=1.2, Q=300, seed=15),
    # leaves of 100 points and ranks 76..91: the 80-, 96- and 112-row tiles
    # of FP32 256-column launches (b1 and b2 take the 48-row ones)
    wl.small("b5", N=1600, d=3, m=128, h=0.5, tol=1e-9, rmax=128, Q=260, seed=16),
]


@pytest.fixture(scope="module")
def setup():
    import paper_1812_07152_amd as hmx
    Hs = [OracleH2.from_workload(w, wl.gen_points(w)) for w in SPECS]
    both = hmx.precbit(hmx.HM_PREC_FP64) | hmx.precbit(hmx.HM_PREC_FP32)
    Ms = [hmx.hm_load_compressed_mem(H, 0, both) for H in Hs]
    return hmx, Hs, Ms


def _inputs(dtype, seed_off=0):
    Ws = [torch.from_numpy(wl.gen_w(w, seed=w.w_seed + seed_off)).to("cuda", dtype) for w in SPECS]
    Ys = [torch.full_like(W, float("nan")) for W in Ws]
    return Ws, Ys


@pytest.mark.parametrize("flags", [0, 1, 2], ids=["graph", "autotune", "no_graph"])
def test_batched_fp64_matches_oracle_and_solo(setup, flags):
    hmx, Hs, Ms = setup
    B = hmx.hm_batch_create(Ms, [w.Q for w in SPECS], flags=flags)
    info = hmx.hm_batch_info(B)
    assert info["n"] == len(SPECS) and info["n_tasks"] > 0
    if flags == 1:
        assert sum(v > 0 for v in info["tuned_ms"].values()) >= 2
    for rep in range(3):  # replays of the captured graph with fresh inputs
        Ws, Ys = _inputs(torch.float64, seed_off=rep)
        hmx.hm_batch_eval(B, Ws, Ys)
        hmx.hm_batch_check(B)
        for H, W, Y, M in zip(Hs, Ws, Ys, Ms):
            Wn = W.cpu().numpy()
            Yb = Y.cpu().numpy()
            ref = H.eval(Wn)
            assert rel(Yb, ref) <= 1e-10
            Ys_ = torch.empty_like(W)
            hmx.hm_eval(M, W, Ys_)
            torch.cuda.synchronize()
            np.testing.assert_allclose(Yb, Ys_.cpu().numpy(), rtol=0, atol=1e-13 * np.abs(ref).max())


def test_eval_batched_one_shot_fp32(setup):
    hmx, Hs, Ms = setup
    Ws, Ys = _inputs(torch.float32)
    hmx.hm_eval_batched(Ms, Ws, Ys)
    torch.cuda.synchronize()
    for H, W, Y in zip(Hs, Ws, Ys):
        ref = H.eval(W.double().cpu().numpy())
        assert rel(Y.double().cpu().numpy(), ref) <= 5e-6


def test_batch_rejects_bad_arguments(setup):
    hmx, Hs, Ms = setup
    with pytest.raises(hmx.HMError):
        hmx.hm_batch_create(Ms, [0] * len(Ms))
    with pytest.raises(hmx.HMError):
        hmx.hm_batch_create(Ms, [4] * len(Ms), dtype=hmx.HM_F32, prec=hmx.HM_PREC_FP64)
    B = hmx.hm_batch_create(Ms[:2], [4, 4])
    Ws = [torch.zeros(H.N, 4, dtype=torch.float64, device="cuda") for H in Hs[:2]]
    with pytest.raises(ValueError):
        hmx.hm_batch_eval(B, Ws, [torch.zeros(10, 4, dtype=torch.float64, device="cuda")] * 2)


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_batched_256_column_tile_narrow_last_tiles(setup, dtype):
    """HM_BATCH_TILE(256): the widths 5, 17, 64, 100, 300 and 260 end in tiles
    of 16, 32, 64, 128, 64 and 16 columns (300 = 256 + 44); FP64 to the parity bar
    and FP32 to its bar against the oracle, and each matrix as hm_eval
    computes it alone (128-column tiles: the same products per column)."""
    hmx, Hs, Ms = setup
    f64 = dtype == "fp64"
    tdt = torch.float64 if f64 else torch.float32
    B = hmx.hm_batch_create(Ms, [w.Q for w in SPECS], dtype=hmx.HM_F64 if f64 else hmx.HM_F32,
                            flags=hmx.HM_BATCH_TILE(256))
    assert hmx.hm_batch_info(B)["column_tile"] == 256
    for rep in range(2):
        Ws, Ys = _inputs(tdt, seed_off=10 + rep)
        hmx.hm_batch_eval(B, Ws, Ys)
        hmx.hm_batch_check(B)
        for H, W, Y, M in zip(Hs, Ws, Ys, Ms):
            Wn = W.double().cpu().numpy()
            Yb = Y.double().cpu().numpy()
            ref = H.eval(Wn)
            assert rel(Yb, ref) <= (1e-10 if f64 else 5e-6)
            Ys_ = torch.empty_like(W)
            hmx.hm_eval(M, W, Ys_)
            torch.cuda.synchronize()
            np.testing.assert_allclose(Yb, Ys_.double().cpu().numpy(), rtol=0,
                                       atol=(1e-13 if f64 else 1e-6) * np.abs(ref).max())


def test_batched_tile_flag_refusals(setup):
    hmx, Hs, Ms = setup
    Q = [w.Q for w in SPECS]
    for bad in (hmx.HM_BATCH_TILE(48), hmx.HM_BATCH_TILE(512), hmx.HM_BATCH_TILE(128) | hmx.HM_BATCH_AUTOTUNE):
        with pytest.raises(hmx.HMError):
            hmx.hm_batch_create(Ms, Q, flags=bad)
