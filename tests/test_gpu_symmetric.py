"""Symmetric storage (HM_LOAD_SYMMETRIC; the kernel matrix is symmetric,
Section 1, so B_ba = B_ab^T and D_ba = D_ab^T): every far and near block of an
unordered pair is stored once and the other product reads it transposed.

Against the full store, on the same representation: results bitwise equal
(the same products in the same order) for FP64 under both launch styles,
FP32 and split BF16, and within the FP64 parity bar of the oracle; the FP64
and FP32 stores hold about half the bytes.  Structures cover leaves and
ranks above one 128-row tile (mirror rows read from a second row tile),
HSS, 8-point leaves, the two-means budget structure, a single node and a
ragged case; the headline workload at full size; a representation that is
not symmetric is refused."""
import sys
import types

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


@pytest.fixture(scope="module")
def hmx():
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_1812_07152_amd as hmx
    return hmx


CASES = {
    "c1": wl.C1,
    "ragged": wl.small("ragged", N=777, d=2, m=20, Q=3),
    "mix8": wl.small("mix8", N=3000, d=8, points="mixture", m=50, h=1.0, Q=37),
    "hss_lap": wl.small("hss_lap", N=2500, d=3, m=70, adm=wl.ADM_HSS, kernel=wl.KERNEL_LAPLACE,
                        h=2.0, rmax=70, Q=20),
    "tall": wl.small("tall", N=4096, d=28, points="normal", m=256, adm=wl.ADM_HSS,
                     kernel=wl.KERNEL_LAPLACE, h=4.0, tol=1e-4, rmax=200, Q=40),
    "deep_small_leaves": wl.small("deep", N=2048, d=3, m=8, Q=4, rmax=8),
    "tm_budget": wl.small("tm_budget", N=3000, d=8, points="mixture", m=50, h=1.0, adm=wl.ADM_BUDGET,
                          budget=0.1, part=wl.PART_TWO_MEANS, Q=24),
    "single_node": wl.small("single_node", N=100, d=3, m=128, Q=5),
}


def _evals(hmx, M, W, flags=0):
    """FP64 (task graph and per-level launches), FP32 and split BF16 results."""
    out = {}
    Wd = torch.from_numpy(W).cuda()
    for name, prec, dt, fl in (("fp64", hmx.HM_PREC_FP64, torch.float64, 0),
                               ("fp64_level", hmx.HM_PREC_FP64, torch.float64, hmx.HM_LEVEL_LAUNCHES),
                               ("fp32", hmx.HM_PREC_FP32, torch.float32, 0),
                               ("fp32_level", hmx.HM_PREC_FP32, torch.float32, hmx.HM_LEVEL_LAUNCHES),
                               ("bf16x3", hmx.HM_PREC_BF16X3, torch.float64, 0)):
        Wx = Wd.to(dt)
        Y = torch.full_like(Wx, float("nan"))
        hmx.hm_eval(M, Wx, Y, prec=prec, flags=flags | fl)
        hmx.hm_check(M)
        out[name] = Y.cpu().numpy()
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_symmetric_store_equals_full_store(hmx, name):
    w = CASES[name]
    X = wl.gen_points(w)
    H = OracleH2.from_workload(w, X)
    mask = hmx.precbit(hmx.HM_PREC_FP64) | hmx.precbit(hmx.HM_PREC_FP32) | hmx.precbit(hmx.HM_PREC_BF16X3)
    _say(f"[sym] case={name} N={w.N}")
    Mf = hmx.hm_load_compressed_mem(H, 0, mask)
    Ms = hmx.hm_load_compressed_mem(H, 0, mask | hmx.HM_LOAD_SYMMETRIC)
    inf, ins = hmx.hm_info(Mf), hmx.hm_info(Ms)
    assert (inf["E_D"], inf["E_B"], inf["flops_per_col"]) == (ins["E_D"], ins["E_B"], ins["flops_per_col"])
    if H.n_near + H.n_far > 1:
        assert ins["bytes_fp64"] < inf["bytes_fp64"]
    _say(f"[sym] case={name}: FP64 store {inf['bytes_fp64'] / 1e6:.2f} MB -> {ins['bytes_fp64'] / 1e6:.2f} MB")
    W = wl.gen_w(w, Q=max(w.Q, 24))
    Yf, Ys = _evals(hmx, Mf, W), _evals(hmx, Ms, W)
    for k in Yf:
        assert np.array_equal(Yf[k], Ys[k]), k
    Yref = H.eval(W)
    assert rel(Ys["fp64"], Yref) <= 1e-10
    np.testing.assert_allclose(Ys["fp64"], Yref, rtol=0, atol=1e-12 * max(1.0, np.abs(Yref).max()))
    assert rel(Ys["fp32"].astype(np.float64), Yref) <= 5e-6 + 1e-6  # FP32 rounding of W as well


def test_symmetric_store_q_shapes_and_tree_order(hmx):
    w = CASES["tall"]
    H = OracleH2.from_workload(w, wl.gen_points(w))
    M = hmx.hm_load_compressed_mem(H, 0, hmx.precbit(hmx.HM_PREC_FP64) | hmx.HM_LOAD_SYMMETRIC)
    for Q in (1, 17, 130, 300):
        W = wl.gen_w(w, Q=Q, seed=500 + Q)
        Wd = torch.from_numpy(W).cuda()
        Y = torch.full_like(Wd, float("nan"))
        hmx.hm_eval(M, Wd, Y)
        hmx.hm_check(M)
        assert rel(Y.cpu().numpy(), H.eval(W)) <= 1e-10, Q
    W = wl.gen_w(w)
    Wt = torch.from_numpy(W[H.perm]).cuda()
    Yt = torch.empty_like(Wt)
    hmx.hm_eval(M, Wt, Yt, flags=hmx.HM_TREE_ORDER)
    hmx.hm_check(M)
    assert rel(Yt.cpu().numpy(), H.eval(W)[H.perm]) <= 1e-10


def test_symmetric_store_rejects_asymmetric_representation(hmx):
    w = CASES["mix8"]
    H = OracleH2.from_workload(w, wl.gen_points(w))
    bad = types.SimpleNamespace(**{k: getattr(H, k) for k in (
        "N", "d", "n_nodes", "perm", "start", "size", "parent", "left", "right", "level", "rank", "basis_off",
        "basis", "far_ptr", "far_col", "far_off", "B", "near_ptr", "near_col", "near_off", "skel_ptr", "skel")})
    bad.params = H.params
    D = np.array(H.D)
    # one entry of an off-diagonal near block, not of its mirror
    a, b, e = next((a, b, e) for a, b, e in H.near_pairs() if a != b)
    D[int(H.near_off[e])] += 1e-3
    bad.D = D
    with pytest.raises(hmx.HMError):
        hmx.hm_load_compressed_mem(bad, 0, hmx.precbit(hmx.HM_PREC_FP64) | hmx.HM_LOAD_SYMMETRIC)
    hmx.hm_load_compressed_mem(bad, 0, hmx.precbit(hmx.HM_PREC_FP64))  # the full store takes it as is


def test_symmetric_store_batched_and_served(hmx):
    """The batched launch and the server run the mirror products too."""
    names = ("c1", "mix8", "tall")
    Hs, Ms, Mf, Ws = [], [], [], []
    for n in names:
        w = CASES[n]
        H = OracleH2.from_workload(w, wl.gen_points(w))
        Hs.append(H)
        Mf.append(hmx.hm_load_compressed_mem(H, 0, hmx.precbit(hmx.HM_PREC_FP32)))
        Ms.append(hmx.hm_load_compressed_mem(H, 0, hmx.precbit(hmx.HM_PREC_FP32) | hmx.HM_LOAD_SYMMETRIC))
        Ws.append(torch.from_numpy(wl.gen_w(w, Q=16 + 8 * len(Ws))).to("cuda", torch.float32))
    Yf = [torch.empty_like(W) for W in Ws]
    Ys = [torch.empty_like(W) for W in Ws]
    hmx.hm_eval_batched(Mf, Ws, Yf)
    hmx.hm_eval_batched(Ms, Ws, Ys)
    torch.cuda.synchronize()
    for a, b in zip(Yf, Ys):
        assert torch.equal(a, b)
    srv = hmx.hm_server_create(0, 2 << 30, 2, hmx.HM_F32, hmx.HM_PREC_FP32)
    ids = [hmx.hm_server_add(srv, M) for M in Ms]
    outs = [torch.full_like(W, float("nan")) for W in Ws]
    tickets = [hmx.hm_submit(srv, i, W, Y) for i, W, Y in zip(ids, Ws, outs)]
    import time
    deadline = time.time() + 60
    pending = set(tickets)
    while pending and time.time() < deadline:
        for t in list(pending):
            if hmx.hm_poll(srv, t)[0]:
                pending.discard(t)
        time.sleep(0.001)
    assert not pending, "requests did not complete"
    for a, b in zip(outs, Yf):
        assert torch.equal(a, b)
    hmx.hm_server_destroy(srv)


@pytest.mark.timeout(900)
def test_symmetric_store_full_size_headline(hmx):
    """N = 65536, d = 8, Q = 256 in the benchmark's configuration: the FP64
    store about halves and the result is bitwise that of the full store."""
    w = wl.C2
    X = wl.gen_points(w)
    _say("[sym c2] compression (host inspector)")
    R = hmx.hm_compress(X, kernel=w.kernel, h=w.h, leaf_size=w.m, tol=w.tol, max_rank=w.rmax,
                        admissibility=w.adm, tau=w.tau, sample_rows=w.sample_rows, seed=w.sample_seed)
    Mf = hmx.hm_load_compressed_mem(R, 0)
    Ms = hmx.hm_load_compressed_mem(R, 0, hmx.precbit(hmx.HM_PREC_FP64) | hmx.HM_LOAD_SYMMETRIC)
    bf, bs = hmx.hm_info(Mf)["bytes_fp64"], hmx.hm_info(Ms)["bytes_fp64"]
    _say(f"[sym c2] FP64 store {bf / 1e9:.2f} GB -> {bs / 1e9:.2f} GB")
    assert bs < 0.56 * bf
    W = torch.from_numpy(wl.gen_w(w)).cuda()
    Yf, Ys = torch.empty_like(W), torch.empty_like(W)
    hmx.hm_eval(Mf, W, Yf)
    hmx.hm_eval(Ms, W, Ys)
    hmx.hm_check(Ms)
    assert torch.equal(Yf, Ys)


@pytest.mark.parametrize("name", ["mix8", "tall", "tm_budget"])
def test_symmetric_store_with_blocks_from_points(hmx, name):
    """A symmetric store evaluated with blocks made from the points: near
    blocks from the points with the far blocks read from the store (mirrors
    among them), and far blocks from the skeletons with the near blocks read
    from the store; each bitwise equal to the full store's evaluation with
    the same flags, and within the FP64 parity bar of the oracle."""
    w = CASES[name]
    X = wl.gen_points(w)
    H = OracleH2.from_workload(w, X)
    Mf = hmx.hm_load_compressed_mem(H, 0)
    Ms = hmx.hm_load_compressed_mem(H, 0, hmx.precbit(hmx.HM_PREC_FP64) | hmx.HM_LOAD_SYMMETRIC)
    for M in (Mf, Ms):
        hmx.hm_set_points(M, X, w.kernel, w.h)
    W = wl.gen_w(w, Q=max(w.Q, 24))
    Yref = H.eval(W)
    Wd = torch.from_numpy(W).cuda()
    for flags in (hmx.HM_NEAR_FROM_POINTS, hmx.HM_FAR_FROM_POINTS):
        _say(f"[sym] case={name} points flags={flags}")
        out = []
        for M in (Mf, Ms):
            Y = torch.full_like(Wd, float("nan"))
            hmx.hm_eval(M, Wd, Y, flags=flags)
            hmx.hm_check(M)
            out.append(Y.cpu().numpy())
        assert np.array_equal(out[0], out[1]), flags
        assert rel(out[1], Yref) <= 1e-10
