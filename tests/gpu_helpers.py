"""Shared helpers for the GPU tests: host <-> device copies in the column-major
layout of the C interface.  No arithmetic of the method lives here."""
import numpy as np
import torch

_NP2T = {np.dtype(np.float32): torch.float32, np.dtype(np.float64): torch.float64,
         np.dtype(np.complex64): torch.complex64, np.dtype(np.complex128): torch.complex128}


def to_dev(a: np.ndarray, dtype=None) -> torch.Tensor:
    a = np.asarray(a)
    if dtype is not None:
        a = a.astype(dtype)
    flat = np.ascontiguousarray(a.ravel(order="F"))
    return torch.from_numpy(flat).to("cuda")


def from_dev(t: torch.Tensor, shape) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().reshape(shape, order="F")


def relerr(a, b) -> float:
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


def reconstruct(U, S, V, ranks):
    """Transform-domain faces U_f diag(S_f) V_f^H from factor arrays
    U (m, kmax, nf), S (kmax, nf), V (p, kmax, nf) -- plain products for
    comparing outputs, not part of either implementation."""
    m, kmax, nf = U.shape
    p = V.shape[0]
    out = np.zeros((m, p, nf), dtype=np.result_type(U, V, np.float64), order="F")
    for f in range(nf):
        k = int(ranks[f])
        out[:, :, f] = (U[:, :k, f] * S[:k, f]) @ np.conj(V[:, :k, f]).T
    return out
