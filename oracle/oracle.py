"""Python face of the CPU FP64 oracle (hm_oracle.c) for Y = K~ W.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  It shares no code
with the GPU path.  Parity unpinned against the paper's own outputs: the paper
prints no numeric worked example; every pin is built from definitions,
invariants, brute force and textbook routines (see tests/test_oracle_*.py).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"oracle library missing: build it with oracle/build.py ({_LIB_PATH})")
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_build.restype = ctypes.c_void_p
        L.orc_build.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                ctypes.c_double, ctypes.c_int64, ctypes.c_uint64]
        L.orc_build_ex.restype = ctypes.c_void_p
        L.orc_build_ex.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_double, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int,
                                   ctypes.c_double]
        L.orc_split_centers.restype = ctypes.c_int
        L.orc_split_centers.argtypes = [ctypes.c_void_p, ctypes.c_int, _f64p]
        L.orc_free.argtypes = [ctypes.c_void_p]
        L.orc_sizes.argtypes = [ctypes.c_void_p, _i64p]
        L.orc_ptrs.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_eval.restype = ctypes.c_int
        L.orc_eval.argtypes = [ctypes.c_void_p, _f64p, ctypes.c_int64, _f64p,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_dense_ktilde.argtypes = [ctypes.c_void_p, _f64p]
        L.orc_exact_rows.argtypes = [ctypes.c_void_p, _i64p, ctypes.c_int64, _f64p,
                                     ctypes.c_int64, _f64p]
        L.orc_pqr_id_public.restype = ctypes.c_int
        L.orc_pqr_id_public.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_int, _i32p, _i32p, _f64p, _f64p]
        L.orc_points.restype = ctypes.c_void_p
        L.orc_points.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.orc_row_sample_public.restype = ctypes.c_int64
        L.orc_row_sample_public.argtypes = [ctypes.c_void_p, ctypes.c_int, _i64p, ctypes.c_int64]
        L.orc_write.restype = ctypes.c_int
        L.orc_write.argtypes = [ctypes.c_void_p, ctypes.c_char_p]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def pqr_id(A: np.ndarray, tol: float, rmax: int):
    """Pivoted-QR ID of one block (rows x cols).  Returns (k, piv, Tcoef, rdiag, capped)
    with A[:, piv[:k]] @ [I, Tcoef] ~= A[:, piv]."""
    A = np.asarray(A, dtype=np.float64)
    mr, nc = A.shape
    Ac = np.asfortranarray(A).copy(order="F")
    k = np.zeros(1, np.int32)
    piv = np.zeros(max(nc, 1), np.int32)
    T = np.zeros(max(nc * nc, 1), np.float64)
    rd = np.zeros(nc + 1, np.float64)
    capped = lib().orc_pqr_id_public(_p(Ac, _f64p), mr, nc, tol, rmax, _p(k, _i32p), _p(piv, _i32p),
                                     _p(T, _f64p), _p(rd, _f64p))
    kk = int(k[0])
    return kk, piv[:nc].copy(), T[: kk * (nc - kk)].reshape(kk, nc - kk).copy(), rd[: kk + 1].copy(), bool(capped)


def exact_rows(X: np.ndarray, kernel: int, h: float, rows, W: np.ndarray) -> np.ndarray:
    """(K W)[rows, :] from the kernel's definition, for points X (original
    order), without compressing anything."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    H = lib().orc_points(_p(X, _f64p), X.shape[0], X.shape[1], int(kernel), float(h))
    if not H:
        raise ValueError("oracle rejected the points")
    try:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        W = np.ascontiguousarray(W, dtype=np.float64)
        out = np.zeros((len(rows), W.shape[1]), np.float64)
        lib().orc_exact_rows(ctypes.c_void_p(H), _p(rows, _i64p), len(rows), _p(W, _f64p), W.shape[1],
                             _p(out, _f64p))
        return out
    finally:
        lib().orc_free(ctypes.c_void_p(H))


class OracleH2:
    """Compressed H^2 representation built by the oracle, with its arrays copied out."""

    def __init__(self, X: np.ndarray, *, kernel: int, h: float, m: int, tol: float, rmax: int,
                 adm: int, tau: float, sample_rows: int = 4096, sample_seed: int = 7,
                 part: int = 0, budget: float = 0.0):
        X = np.ascontiguousarray(X, dtype=np.float64)
        N, d = X.shape
        self.params = dict(kernel=kernel, h=h, m=m, tol=tol, rmax=rmax, adm=adm, tau=tau,
                           sample_rows=sample_rows, sample_seed=sample_seed, part=part, budget=budget)
        self._h = lib().orc_build_ex(_p(X, _f64p), N, d, kernel, h, m, tol, rmax, adm, tau,
                                     sample_rows, sample_seed, part, budget)
        if not self._h:
            raise ValueError("oracle rejected the inputs")
        s = np.zeros(10, np.int64)
        lib().orc_sizes(self._h, _p(s, _i64p))
        self.N, self.d, self.L, self.n_nodes = int(s[0]), int(s[1]), int(s[2]), int(s[3])
        n_far, n_near, bl, Bl, Dl, sl = (int(v) for v in s[4:10])
        self.n_far, self.n_near = n_far, n_near
        n = self.n_nodes
        p = (ctypes.c_void_p * 23)()
        lib().orc_ptrs(self._h, p)

        def view(i, ctype, count, shape=None):
            # zero-copy view of oracle-owned memory; valid while self lives
            if count == 0:
                return np.zeros(0 if shape is None else shape, np.ctypeslib.as_ctypes_type(ctype))
            a = np.ctypeslib.as_array((np.ctypeslib.as_ctypes_type(ctype) * count).from_address(p[i]))
            return a if shape is None else a.reshape(shape)

        i64, i32, f64 = np.int64, np.int32, np.float64
        self.perm = view(0, i64, self.N)
        self.start, self.size = view(1, i64, n), view(2, i64, n)
        self.parent, self.left, self.right = view(3, i32, n), view(4, i32, n), view(5, i32, n)
        self.level, self.rank, self.cap_hit = view(6, i32, n), view(7, i32, n), view(8, i32, n)
        self.basis_off, self.basis = view(9, i64, n), view(10, f64, bl)
        self.far_ptr, self.far_col = view(11, i64, n + 1), view(12, i32, n_far)
        self.far_off, self.B = view(13, i64, n_far), view(14, f64, Bl)
        self.near_ptr, self.near_col = view(15, i64, n + 1), view(16, i32, n_near)
        self.near_off, self.D = view(17, i64, n_near), view(18, f64, Dl)
        self.skel_ptr, self.skel = view(19, i64, n + 1), view(20, i64, sl)
        self.centroid, self.radius = view(21, f64, n * self.d, (n, self.d)), view(22, f64, n)

    @classmethod
    def from_workload(cls, w, X: np.ndarray) -> "OracleH2":
        return cls(X, kernel=w.kernel, h=w.h, m=w.m, tol=w.tol, rmax=w.rmax, adm=w.adm, tau=w.tau,
                   sample_rows=w.sample_rows, sample_seed=w.sample_seed, part=w.part, budget=w.budget)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    # -- structure helpers -------------------------------------------------
    def is_leaf(self, a: int) -> bool:
        return self.left[a] < 0

    def ncols(self, a: int) -> int:
        if self.is_leaf(a):
            return int(self.size[a])
        return int(self.rank[self.left[a]] + self.rank[self.right[a]])

    def basis_of(self, a: int) -> np.ndarray:
        k, c = int(self.rank[a]), self.ncols(a)
        o = int(self.basis_off[a])
        return self.basis[o:o + k * c].reshape(k, c)

    def far_pairs(self):
        for a in range(self.n_nodes):
            for e in range(self.far_ptr[a], self.far_ptr[a + 1]):
                yield a, int(self.far_col[e]), int(e)

    def near_pairs(self):
        for a in range(self.n_nodes):
            for e in range(self.near_ptr[a], self.near_ptr[a + 1]):
                yield a, int(self.near_col[e]), int(e)

    def B_block(self, e: int, a: int, b: int) -> np.ndarray:
        ka, kb = int(self.rank[a]), int(self.rank[b])
        o = int(self.far_off[e])
        return self.B[o:o + ka * kb].reshape(ka, kb)

    def D_block(self, e: int, a: int, b: int) -> np.ndarray:
        sa, sb = int(self.size[a]), int(self.size[b])
        o = int(self.near_off[e])
        return self.D[o:o + sa * sb].reshape(sa, sb)

    def stats(self) -> dict:
        """Entry counts and algorithmic flops per column of W:
        flops = 2 Q (2 E_V + 2 E_T + E_B + E_D)."""
        leaf = self.left < 0
        E_V = int(np.sum(self.rank[leaf].astype(np.int64) * self.size[leaf]))
        E_T = int(sum(int(self.rank[a]) * self.ncols(a) for a in range(self.n_nodes) if not leaf[a]))
        E_B = len(self.B)
        E_D = len(self.D)
        return dict(N=self.N, L=self.L, n_nodes=self.n_nodes, n_far=self.n_far, n_near=self.n_near,
                    E_V=E_V, E_T=E_T, E_B=E_B, E_D=E_D,
                    flops_per_col=2 * (2 * E_V + 2 * E_T + E_B + E_D),
                    max_rank=int(self.rank.max()), cap_hits=int(self.cap_hit.sum()),
                    ranks_by_level=[self.rank[self.level == l].tolist() for l in range(self.L + 1)])

    # -- evaluation --------------------------------------------------------
    def node_offsets(self, Q: int) -> np.ndarray:
        """Offsets of each node's k x Q block in the node-major dumps."""
        off = np.zeros(self.n_nodes + 1, np.int64)
        off[1:] = np.cumsum(self.rank.astype(np.int64) * Q)
        return off

    def eval(self, W: np.ndarray, dump: bool = False):
        W = np.ascontiguousarray(W, dtype=np.float64)
        assert W.shape[0] == self.N
        Q = W.shape[1]
        Y = np.empty((self.N, Q), np.float64)
        if not dump:
            rc = lib().orc_eval(self._h, _p(W, _f64p), Q, _p(Y, _f64p), None, None, None, None)
            assert rc == 0
            return Y
        tot = int(self.rank.astype(np.int64).sum()) * Q
        what = np.zeros(max(tot, 1), np.float64)
        yhat = np.zeros(max(tot, 1), np.float64)
        yn = np.zeros((self.N, Q), np.float64)
        yf = np.zeros((self.N, Q), np.float64)
        rc = lib().orc_eval(self._h, _p(W, _f64p), Q, _p(Y, _f64p),
                            what.ctypes.data_as(ctypes.c_void_p), yhat.ctypes.data_as(ctypes.c_void_p),
                            yn.ctypes.data_as(ctypes.c_void_p), yf.ctypes.data_as(ctypes.c_void_p))
        assert rc == 0
        return Y, dict(what=what[:tot], yhat=yhat[:tot], ynear=yn, yfar=yf)

    def dense_ktilde(self) -> np.ndarray:
        Kt = np.zeros((self.N, self.N), np.float64)
        lib().orc_dense_ktilde(self._h, _p(Kt, _f64p))
        return Kt

    def exact_rows(self, rows, W: np.ndarray) -> np.ndarray:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        W = np.ascontiguousarray(W, dtype=np.float64)
        out = np.zeros((len(rows), W.shape[1]), np.float64)
        lib().orc_exact_rows(self._h, _p(rows, _i64p), len(rows), _p(W, _f64p), W.shape[1],
                             _p(out, _f64p))
        return out

    def split_centers(self, a: int):
        """(c1, c2): the two means of node a's two-means split, or None."""
        out = np.zeros(2 * self.d, np.float64)
        if not lib().orc_split_centers(self._h, int(a), _p(out, _f64p)):
            return None
        return out[:self.d].copy(), out[self.d:].copy()

    def row_sample(self, a: int) -> np.ndarray:
        """Rows (tree positions, ascending) of the ID of node a."""
        out = np.zeros(max(self.N, 1), np.int64)
        n = lib().orc_row_sample_public(self._h, int(a), _p(out, _i64p), len(out))
        if n < 0:
            raise ValueError("bad node")
        return out[:n].copy()

    def write(self, path: str) -> None:
        rc = lib().orc_write(self._h, os.fsencode(path))
        if rc != 0:
            raise OSError(f"oracle could not write {path}")
