"""Seeded synthetic inputs for the t-SVDM path.

This module only draws random numbers and assembles the input matrices the
workloads are defined by (Kronecker sums, Gaussian factors, Gaussian noise,
Gaussian test matrices).  It holds none of the method's arithmetic: no
transform, no SVD, no truncation, no apply.  Both the oracle-side tests and the
HIP-side tests/benchmark take their inputs from here; where a workload is
specified in the transform domain, each side builds the spatial tensor with its
own code from the factors returned here.

All arrays are float64, tensors are (m, p, n3) in Fortran order (element
(a, b, t) at a + m*b + m*p*t).  Seeds: numpy PCG64 with 2105011700 + workload
index, so every run draws the same numbers.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 2105011700


def rng(index: int, salt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([SEED_BASE + index, salt]))


def gaussian(g: np.random.Generator, shape) -> np.ndarray:
    return np.asfortranarray(g.standard_normal(shape))


def orthonormal_stack(g: np.random.Generator, rows: int, cols: int, count: int) -> np.ndarray:
    """count independent rows x cols matrices with orthonormal columns (Q factor
    of a Gaussian matrix, signs fixed so that diag(R) > 0); shape (rows, cols, count)."""
    G = g.standard_normal((count, rows, cols))
    Q, R = np.linalg.qr(G)
    sgn = np.sign(np.diagonal(R, axis1=1, axis2=2))
    sgn[sgn == 0] = 1.0
    Q = Q * sgn[:, None, :]
    return np.asfortranarray(np.transpose(Q, (1, 2, 0)))


def kron_sum(B: np.ndarray, C: np.ndarray) -> np.ndarray:
    """sum_i B[i] kron C[i]."""
    return np.asfortranarray(sum(np.kron(B[i], C[i]) for i in range(B.shape[0])))


def add_relative_noise(g: np.random.Generator, A: np.ndarray, rel: float) -> np.ndarray:
    """A + N with N = G * (rel * ||A||_F / ||G||_F), G iid N(0,1)."""
    G = g.standard_normal(A.shape)
    return np.asfortranarray(A + G * (rel * np.linalg.norm(A) / np.linalg.norm(G)))


# ---------------------------------------------------------------- workloads
def kronecker_sum_matrix(terms: int = 4, size: int = 32, noise: float = 1e-8, index: int = 0,
                         salt: int = 0):
    """Plain FP64 workload: A = sum_{i<terms} B_i kron C_i + noise, with
    B_i, C_i in R^{size x size} iid N(0,1).  Blocking l = q = m = n = size."""
    g = rng(index, salt)
    B = g.standard_normal((terms, size, size))
    C = g.standard_normal((terms, size, size))
    A = add_relative_noise(g, kron_sum(B, C), noise)
    return dict(A=A, B=B, C=C, ell=size, q=size, m=size, n=size, terms=terms, noise=noise)


def known_rank_factors(m: int = 512, p: int = 512, n3: int = 256, k: int = 32,
                       decay: float = 1.0 / 8.0, oversample: int = 8, index: int = 1,
                       salt: int = 0, omega_cols: int | None = None):
    """Transform-domain factors of a tensor of M-rank k: for every face f,
    Xhat_f = U_f diag(sigma) V_f^T with U_f (m x k), V_f (p x k) orthonormal
    and sigma_j = 10^(-decay * j), j = 1..k.  Also the Gaussian test matrix
    Omega (p x (k + oversample)) the randomized range finder draws."""
    g = rng(index, salt)
    U = orthonormal_stack(g, m, k, n3)
    V = orthonormal_stack(g, p, k, n3)
    sigma = 10.0 ** (-decay * np.arange(1, k + 1))
    ell = omega_cols if omega_cols is not None else k + oversample
    Omega = gaussian(g, (p, ell))
    return dict(U=U, V=V, sigma=sigma, Omega=Omega, m=m, p=p, n3=n3, k=k, ell=ell)


def uneven_batch(count: int = 256, lo: int = 16, hi: int = 64, rmin: int = 2, rmax: int = 16,
                 noise: float = 1e-6, index: int = 2, salt: int = 0, form: bool = True):
    """Independent Kronecker-sum matrices sum_{i<r} B_i kron C_i with square
    factors of sizes s_B, s_C = round(exp(U(ln lo, ln hi))) and r uniform in
    {rmin..rmax}, iid N(0,1) entries, plus relative noise.  With form=False
    only the factors are returned (no A; noise must be 0)."""
    if not form and noise:
        raise ValueError("noise needs the formed matrix")
    g = rng(index, salt)
    out = []
    for _ in range(count):
        sB = int(round(np.exp(g.uniform(np.log(lo), np.log(hi)))))
        sC = int(round(np.exp(g.uniform(np.log(lo), np.log(hi)))))
        r = int(g.integers(rmin, rmax + 1))
        B = g.standard_normal((r, sB, sB))
        C = g.standard_normal((r, sC, sC))
        rec = dict(B=B, C=C, sB=sB, sC=sC, r=r, ell=sB, q=sB, m=sC, n=sC)
        if form:
            A = kron_sum(B, C)
            rec["A"] = add_relative_noise(g, A, noise) if noise else A
        out.append(rec)
    return out


def decay_profiles(count: int, k: int = 32, lo: float = 1.0 / 16.0, hi: float = 0.5,
                   index: int = 3, salt: int = 0):
    """Per-face singular-value decay rates rho ~ U[lo, hi]; sigma_j = 10^(-rho j)."""
    g = rng(index, salt)
    rho = g.uniform(lo, hi, size=count)
    return rho


def apply_factors(m: int = 64, ell: int = 64, q: int = 64, n: int = 64, k: int = 16,
                  nrhs: int = 1024, decay: float = 1.0 / 8.0, index: int = 4, salt: int = 0):
    """Apply workload: spatial-domain factors U (m x k x n), V (p x k x n) with
    p = ell*q, iid N(0,1), singular values sigma_j = 10^(-decay j) on every
    transform-domain face, and right-hand sides X ((q*n) x nrhs) iid N(0,1)."""
    g = rng(index, salt)
    p = ell * q
    U = gaussian(g, (m, k, n))
    V = gaussian(g, (p, k, n))
    sigma = 10.0 ** (-decay * np.arange(1, k + 1))
    X = gaussian(g, (q * n, nrhs))
    return dict(U=U, V=V, sigma=sigma, X=X, m=m, ell=ell, q=q, n=n, p=p, k=k, nrhs=nrhs)


def decay_faces_device(rho, m: int = 512, p: int = 512, k: int = 32, index: int = 3, salt: int = 0,
                       device: str = "cuda"):
    """Transform-domain faces Xhat_f = U_f diag(10^(-rho_f j)) V_f^T, j = 1..k,
    with U_f (m x k), V_f (p x k) the Q factors of iid N(0,1) matrices drawn on
    the device (torch generator seeded from (index, salt)); FP64 products,
    stored FP32 as a flat column-major (m, p, nf) buffer."""
    import torch

    nf = len(rho)
    gen = torch.Generator(device=device).manual_seed(SEED_BASE * 1000 + index * 100003 + salt)
    U = torch.linalg.qr(torch.randn(nf, m, k, generator=gen, device=device, dtype=torch.float64)).Q
    V = torch.linalg.qr(torch.randn(nf, p, k, generator=gen, device=device, dtype=torch.float64)).Q
    j = torch.arange(1, k + 1, device=device, dtype=torch.float64)
    sig = 10.0 ** (-torch.as_tensor(rho, device=device, dtype=torch.float64)[:, None] * j)
    # [f, b, a] = sum_r V[f, b, r] sig[f, r] U[f, a, r]: column-major (m, p) faces
    X = torch.bmm((V * sig[:, None, :]).contiguous(), U.transpose(1, 2).contiguous())
    return X.reshape(-1).to(torch.float32).contiguous(), sig.cpu().numpy()


def spacetime_covariance(N: int = 1351, T: int = 30, index: int = 9, salt: int = 0,
                         length: float = 90.0, tscale: float = 0.5):
    """Blocks of a space-time covariance matrix (the input of Sec. 6.2): N
    points x_j drawn uniformly on a longitude/latitude box (degrees; a
    stand-in for the land-mass grid points), T equidistant times in [0, 1],
    and the T distinct N x N blocks C_i[j, k] = phi(|x_j - x_k|, |t_1 - t_i|)
    of the symmetric block-Toeplitz matrix, phi(r, tau) = exp(-((r/90)^2 +
    (tau/0.5)^2)) (Euclidean distance in degrees).  Returns the blocks stacked
    N x N x T (float64, Fortran order), the points and the times."""
    g = rng(index, salt)
    pts = np.stack([g.uniform(-180.0, 180.0, N), g.uniform(-60.0, 80.0, N)], axis=1)
    times = np.linspace(0.0, 1.0, T)
    d = np.sqrt(np.sum((pts[:, None, :] - pts[None, :, :]) ** 2, axis=2))
    blocks = np.empty((N, N, T), order="F")
    for i in range(T):
        blocks[:, :, i] = np.exp(-((d / length) ** 2 + (abs(times[0] - times[i]) / tscale) ** 2))
    return blocks, pts, times
