"""Shared test helpers: dense kernel matrices straight from the definition and
a test-side reader of the HMC1 compressed-representation file.  Neither
calls the oracle or the GPU library."""
from __future__ import annotations

import numpy as np

import workloads as wl


def dense_kernel(X: np.ndarray, kernel: int, h: float, Y: np.ndarray | None = None) -> np.ndarray:
    """K(i,j) = kernel(x_i, y_j) computed with numpy broadcasting (Section 1 of the paper)."""
    Y = X if Y is None else Y
    diff = X[:, None, :] - Y[None, :, :]
    r2 = np.einsum("ijk,ijk->ij", diff, diff)
    if kernel == wl.KERNEL_GAUSSIAN:
        return np.exp(-r2 / (2.0 * h * h))
    return np.exp(-np.sqrt(r2) / h)


def rel(a: np.ndarray, b: np.ndarray) -> float:
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def read_hmc1(path: str) -> dict:
    """Parse an HMC1 file with numpy (independent of the library's loader)."""
    raw = open(path, "rb").read()
    hdr = raw[:128]
    assert hdr[:4] == b"HMC1"
    u32 = lambda o: int(np.frombuffer(hdr, np.uint32, 1, o)[0])
    i32 = lambda o: int(np.frombuffer(hdr, np.int32, 1, o)[0])
    i64 = lambda o: int(np.frombuffer(hdr, np.int64, 1, o)[0])
    f64 = lambda o: float(np.frombuffer(hdr, np.float64, 1, o)[0])
    out = dict(version=u32(4), N=i64(8), d=i64(16), n_nodes=i32(24), L=i32(28), flags=u32(32),
               kernel=i32(36), h=f64(40), tol=f64(48), tau=f64(56), rmax=i32(64), m=i32(68),
               n_far=i64(72), n_near=i64(80), basis_len=i64(88), B_len=i64(96), D_len=i64(104),
               skel_len=i64(112))
    off = 128
    n = out["n_nodes"]

    def take(name, dt, count):
        nonlocal off
        a = np.frombuffer(raw, dt, count, off)
        off += a.nbytes
        out[name] = a

    take("perm", np.int64, out["N"])
    take("start", np.int64, n)
    take("size", np.int64, n)
    for k in ("parent", "left", "right", "level", "rank"):
        take(k, np.int32, n)
    take("basis_off", np.int64, n)
    take("basis", np.float64, out["basis_len"])
    take("far_ptr", np.int64, n + 1)
    take("far_col", np.int32, out["n_far"])
    take("far_off", np.int64, out["n_far"])
    take("B", np.float64, out["B_len"])
    take("near_ptr", np.int64, n + 1)
    take("near_col", np.int32, out["n_near"])
    take("near_off", np.int64, out["n_near"])
    take("D", np.float64, out["D_len"])
    take("skel_ptr", np.int64, n + 1)
    take("skel", np.int64, out["skel_len"])
    assert off == len(raw), (off, len(raw))
    return out
