"""Serving form: resident matrices, non-blocking submit/poll, continuous
batching.  Each result must be bitwise the same alone and in a concurrent mix
(and match the oracle), the mix must coalesce requests into fewer sweeps, and
a request beyond the HBM budget is refused while the server keeps serving."""
import time

import numpy as np
import pytest

import workloads as wl
from oracle.oracle import OracleH2
from tests.helpers import rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SPECS = [
    wl.small("s0", N=900, d=3, m=32, seed=21),
    wl.small("s1", N=2500, d=8, points="mixture", m=50, h=1.0, seed=22),
    wl.small("s2", N=1800, d=3, m=60, adm=wl.ADM_HSS, kernel=wl.KERNEL_LAPLACE, h=2.0, rmax=60, seed=23),
]


@pytest.fixture(scope="module")
def setup():
    import paper_1812_07152_amd as hmx
    Hs = [OracleH2.from_workload(w, wl.gen_points(w)) for w in SPECS]
    Ms = [hmx.hm_load_compressed_mem(H, 0, hmx.precbit(hmx.HM_PREC_FP64)) for H in Hs]
    return hmx, Hs, Ms


@pytest.fixture(scope="module")
def setup32(setup):
    hmx, Hs, _ = setup
    return hmx, Hs, [hmx.hm_load_compressed_mem(H, 0, hmx.precbit(hmx.HM_PREC_FP32)) for H in Hs]


def wait_all(hmx, S, tickets, deadline_s=60.0):
    lat = {}
    t0 = time.time()
    while len(lat) < len(tickets):
        assert time.time() - t0 < deadline_s, "requests did not complete in time"
        for t in tickets:
            if t in lat:
                continue
            done, l = hmx.hm_poll(S, t)
            if done:
                lat[t] = l
        time.sleep(0.0005)
    return [lat[t] for t in tickets]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_alone_equals_mix_and_oracle(setup, setup32, dtype):
    """Each result bitwise the same alone and in a concurrent mix, and against
    the FP64 oracle: <= 1e-10 in FP64; in FP32 <= 5e-6 against the oracle on
    the FP32-rounded W (FP32 rounding of the blocks and W, accumulated in FP32:
    the bar of the plain FP32 path)."""
    hmx, Hs, Ms = setup if dtype == "f64" else setup32
    f64 = dtype == "f64"
    S = hmx.hm_server_create(0, hbm_budget=1 << 30, max_slots=3, dtype=hmx.HM_F64 if f64 else hmx.HM_F32)
    ids = [hmx.hm_server_add(S, M) for M in Ms]
    rng = np.random.default_rng(5)
    reqs = [(int(rng.integers(0, len(Ms))), int(rng.integers(1, 65))) for _ in range(30)]
    tdt = torch.float64 if f64 else torch.float32
    Ws = [torch.from_numpy(rng.standard_normal((Hs[m].N, q))).to("cuda", tdt) for m, q in reqs]
    # alone: one request at a time
    alone = []
    for (m, q), W in zip(reqs, Ws):
        Y = torch.full_like(W, float("nan"))
        wait_all(hmx, S, [hmx.hm_submit(S, ids[m], W, Y)])
        alone.append(Y.cpu().numpy())
    before = hmx.hm_server_stats(S)
    # mix: everything at once
    Ys = [torch.full_like(W, float("nan")) for W in Ws]
    tickets = [hmx.hm_submit(S, ids[m], W, Y) for (m, q), W, Y in zip(reqs, Ws, Ys)]
    lats = wait_all(hmx, S, tickets)
    after = hmx.hm_server_stats(S)
    assert after["completed"] - before["completed"] == len(reqs) and after["failed"] == 0
    assert after["sweeps"] - before["sweeps"] < len(reqs), "the mix was not coalesced"
    assert all(l > 0 for l in lats)
    for (m, q), W, Y, Ya in zip(reqs, Ws, Ys, alone):
        Ym = Y.cpu().numpy()
        assert np.array_equal(Ym, Ya), "result differs alone vs in the mix"
        err = rel(Ym.astype(np.float64), Hs[m].eval(W.double().cpu().numpy()))
        assert err <= (1e-10 if f64 else 5e-6), err
    hmx.hm_server_destroy(S)


def test_sweeps_overlap_and_mid_sweep_admission(setup):
    """Continuous batching: several sweeps (also of one matrix) are on the
    device at once, and a request submitted while sweeps of its matrix run is
    admitted and correct."""
    hmx, Hs, Ms = setup
    S = hmx.hm_server_create(0, hbm_budget=1 << 30, max_slots=3, dtype=hmx.HM_F64)
    ids = [hmx.hm_server_add(S, M) for M in Ms]
    rng = np.random.default_rng(6)
    H = Hs[1]
    # six 512-column requests on one matrix: at most two fit one sweep
    Ws = [torch.from_numpy(rng.standard_normal((H.N, 512))).cuda() for _ in range(6)]
    Ys = [torch.full_like(W, float("nan")) for W in Ws]
    tickets = [hmx.hm_submit(S, ids[1], W, Y) for W, Y in zip(Ws, Ys)]
    mid = hmx.hm_server_stats(S)["inflight"]
    Wm = torch.from_numpy(rng.standard_normal((H.N, 7))).cuda()
    Ym = torch.full_like(Wm, float("nan"))
    tickets.append(hmx.hm_submit(S, ids[1], Wm, Ym))
    wait_all(hmx, S, tickets)
    st = hmx.hm_server_stats(S)
    print(f"[serving] inflight when the extra request came: {mid}, peak inflight {st['peak_inflight']}, "
          f"sweeps {st['sweeps']}", flush=True)
    assert st["failed"] == 0 and st["completed"] == 7
    assert st["peak_inflight"] >= 2, "sweeps never overlapped on the device"
    for W, Y in zip(Ws + [Wm], Ys + [Ym]):
        assert rel(Y.cpu().numpy(), H.eval(W.cpu().numpy())) <= 1e-10
    hmx.hm_server_destroy(S)


def test_submit_is_ordered_after_the_callers_stream(setup):
    """W is written by work still queued on the caller's stream when the
    request is submitted (no host synchronization): the sweep must wait for
    it (hm_submit records an event on that stream)."""
    hmx, Hs, Ms = setup
    S = hmx.hm_server_create(0, hbm_budget=1 << 30, max_slots=2, dtype=hmx.HM_F64)
    mid = hmx.hm_server_add(S, Ms[0])
    H = Hs[0]
    src = torch.from_numpy(np.random.default_rng(7).standard_normal((H.N, 16))).cuda()
    side = torch.cuda.Stream()
    big = torch.randn(4096, 4096, device="cuda", dtype=torch.float64)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        for _ in range(4):                 # keep the stream busy for a while
            big = big @ big * 1e-3
        W = torch.zeros_like(src)
        W.copy_(src)                       # W is ready only after the products
        Y = torch.full_like(src, float("nan"))
        t = hmx.hm_submit(S, mid, W, Y, stream=side)
    wait_all(hmx, S, [t])
    assert rel(Y.cpu().numpy(), H.eval(src.cpu().numpy())) <= 1e-10
    hmx.hm_server_destroy(S)


def test_budget_refusal_keeps_serving(setup):
    hmx, Hs, Ms = setup
    H = Hs[1]
    # budget fits a 4-column sweep of matrix 1 but not a 512-column request
    budget = 2 * H.N * 8 * 8
    S = hmx.hm_server_create(0, hbm_budget=budget, max_slots=2, dtype=hmx.HM_F64)
    mid = hmx.hm_server_add(S, Ms[1])
    big = torch.zeros(H.N, 512, dtype=torch.float64, device="cuda")
    with pytest.raises(hmx.HMError) as e:
        hmx.hm_submit(S, mid, big, torch.empty_like(big))
    assert e.value.status == -5  # HM_ERR_BUSY
    W = torch.from_numpy(np.random.default_rng(1).standard_normal((H.N, 4))).cuda()
    Y = torch.empty_like(W)
    t = hmx.hm_submit(S, mid, W, Y)
    wait_all(hmx, S, [t])
    assert rel(Y.cpu().numpy(), H.eval(W.cpu().numpy())) <= 1e-10
    with pytest.raises(hmx.HMError):   # retired ticket
        hmx.hm_poll(S, t)
    with pytest.raises(hmx.HMError):   # unknown matrix
        hmx.hm_submit(S, 7, W, Y)
    hmx.hm_server_destroy(S)
