"""Oracle for the t-SVDM path: plain, slow, obviously-correct double precision.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, links or calls anything in ``oracle/``; only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` do.  The
oracle shares no code with the HIP path.

Conventions
-----------
* Third-order tensors are numpy arrays of shape (m, p, n3) in Fortran order:
  element (a, b, t) sits at a + m*b + m*p*t, so frontal faces X[:, :, t] are
  contiguous and a tube X[a, b, :] has stride m*p.
* All arithmetic is float64 / complex128.  Library primitives (matmul,
  Cholesky, triangular solve) serve as steps; the facewise SVD is the
  hand-written one-sided Jacobi in ``jacobi.c``.

Paper passages followed (Kilmer & Saibaba, "Structured matrix approximations
via tensor decompositions"):
* frontal slices, twist/sq, the mode-3 unfolding and the mode-i product
  (Sec. 2.1, eq. mode3unfold): the transform X x_3 M multiplies every tube by M;
* the block-matrix/tensor maps T_E and M_E and the Kronecker-sum form
  struct_E (Sec. 3, eq. kronsum), with the generic blocking of the remark after
  Lemma lem:tenapprox (p = l*q, E_jk = e_j e_k^T, eta = 1);
* Algorithm alg:strategy (Sec. 3.1): map, compress, map back; Lemma
  lem:tenapprox: the matrix error equals the tensor error in Frobenius norm.
The transform-domain algebra (M-product, t-SVDM, transforms) is not defined in
the paper; it is the standard linear algebra written out below, function by
function.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build(force=False)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        for name in ("oracle_svd_faces_d", "oracle_svd_faces_z"):
            fn = getattr(lib, name)
            fn.restype = None
            fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, ip,
                           ctypes.c_int, ctypes.c_double]
        _LIB = lib
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# --------------------------------------------------------------------------
# Facewise SVD (one-sided Jacobi, jacobi.c)
# --------------------------------------------------------------------------
JACOBI_TOL = 1e-15
JACOBI_MAX_SWEEPS = 60


def svd_faces(F: np.ndarray, max_sweeps: int = JACOBI_MAX_SWEEPS, tol: float = JACOBI_TOL):
    """Thin SVD of every face F[:, :, f] (shape (r, c, nf), any dtype).

    Returns U (r, ns, nf), s (ns, nf), V (c, ns, nf), sweeps (nf,), with
    F[:, :, f] = U[:, :, f] @ diag(s[:, f]) @ V[:, :, f]^H and s sorted
    decreasing.  sweeps[f] = -1 if the sweep cap was reached.
    """
    if F.ndim == 2:
        F = F[:, :, None]
    r, c, nf = F.shape
    ns = min(r, c)
    cplx = np.iscomplexobj(F)
    dt = np.complex128 if cplx else np.float64
    A = np.asfortranarray(F, dtype=dt)
    U = np.zeros((r, ns, nf), dtype=dt, order="F")
    V = np.zeros((c, ns, nf), dtype=dt, order="F")
    s = np.zeros((ns, nf), dtype=np.float64, order="F")
    sw = np.zeros(nf, dtype=np.int32)
    if nf and ns:
        fn = _lib().oracle_svd_faces_z if cplx else _lib().oracle_svd_faces_d
        fn(r, c, nf, _ptr(A), _ptr(U), _ptr(s), _ptr(V),
           sw.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), max_sweeps, tol)
    return U, s, V, sw


# --------------------------------------------------------------------------
# Sec. 3: block matrix <-> tensor maps (generic and structured E)
# --------------------------------------------------------------------------
def tensor_from_blockmat(A: np.ndarray, ell: int, q: int, m: int, n: int) -> np.ndarray:
    """T_E[A] for the generic blocking (no repeated blocks).

    A is (ell*m) x (q*n) with ell x q blocks of size m x n.  With p = ell*q and
    E_b = e_j e_k^T for b = j + ell*k (blocks enumerated column by column, the
    column-unwrapping order of vec in Sec. 2.1), eta_b = 1, the lateral slice
    b of the tensor is twist(A_jk) (Sec. 3, definition of T_E), i.e.
    X[a, b, t] = A[j*m + a, k*n + t].
    """
    A = np.asarray(A)
    assert A.shape == (ell * m, q * n)
    X = np.zeros((m, ell * q, n), dtype=A.dtype, order="F")
    for k in range(q):
        for j in range(ell):
            X[:, j + ell * k, :] = A[j * m:(j + 1) * m, k * n:(k + 1) * n]
    return X


def blockmat_from_tensor(X: np.ndarray, ell: int, q: int) -> np.ndarray:
    """M_E[X] = sum_b E_b kron sq(X[:, b, :]) for the generic blocking (Sec. 3)."""
    m, p, n = X.shape
    assert p == ell * q
    A = np.zeros((ell * m, q * n), dtype=X.dtype, order="F")
    for k in range(q):
        for j in range(ell):
            A[j * m:(j + 1) * m, k * n:(k + 1) * n] = X[:, j + ell * k, :]
    return A


def placement_generic(ell: int, q: int):
    """The tuple E of the generic blocking: E_b = e_j e_k^T, b = j + ell*k."""
    E = []
    for k in range(q):
        for j in range(ell):
            Eb = np.zeros((ell, q))
            Eb[j, k] = 1.0
            E.append(Eb)
    return E


def kron_sum_faces(B: np.ndarray, C: np.ndarray, M: np.ndarray, faces) -> np.ndarray:
    """Transform-domain faces of X = T_E[A], A = sum_r B_r kron C_r, for the
    generic blocking with square B_r (l x l, so q = l) and square C_r (m x m,
    so n = m), without forming A.

    Block (j, k) of A is sum_r B_r[j, k] C_r, so X(a, j + l*k, t) =
    sum_r B_r[j, k] C_r[a, t] (Sec. 3, T_E) and the mode-3 product gives
    Xhat_f[a, b] = sum_r (C_r M^T)[a, f] vec(B_r)[b] (column-major vec):
    every face has rank at most r.  B: (r, l, l), C: (r, m, m).  Returns an
    (m, l*l, len(faces)) array."""
    B = np.asarray(B, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    r, l, _ = B.shape
    m = C.shape[1]
    # vec(B_r)[j + l*k] = B_r[j, k]: column-major unwrapping
    vecB = np.stack([B[i].reshape(-1, order="F") for i in range(r)])
    CM = np.einsum("rat,ft->raf", C, M)  # (C_r M^T)[a, f]
    out = np.empty((m, l * l, len(faces)), order="F")
    for i, f in enumerate(faces):
        out[:, :, i] = CM[:, :, f].T @ vecB
    return out


def struct_kron(E, blocks) -> np.ndarray:
    """struct(A) = sum_k E_k kron B_k (eq. kronsum with B_k = sqrt(eta_k) A_k)."""
    return sum(np.kron(Ek, Bk) for Ek, Bk in zip(E, blocks))


def tensor_from_blockmat_E(A: np.ndarray, E, m: int, n: int) -> np.ndarray:
    """T_E[A] for a general placement tuple E (Sec. 3).

    E_k has entries 1/sqrt(eta_k) where the distinct block A_k occurs; the
    lateral slice k of the tensor is sqrt(eta_k) twist(A_k).  A_k is read from
    the first position where E_k is non-zero.
    """
    p = len(E)
    X = np.zeros((m, p, n), dtype=A.dtype, order="F")
    for k, Ek in enumerate(E):
        nz = np.argwhere(Ek != 0)
        eta = len(nz)
        i, j = nz[0]
        X[:, k, :] = np.sqrt(eta) * A[i * m:(i + 1) * m, j * n:(j + 1) * n]
    return X


def blockmat_from_tensor_E(X: np.ndarray, E) -> np.ndarray:
    """M_E[X] = sum_k E_k kron sq(X[:, k, :]) for a general placement tuple (Sec. 3)."""
    return struct_kron(E, [X[:, k, :] for k in range(X.shape[1])])


# --------------------------------------------------------------------------
# Explicit transform matrices and the mode-3 product
# --------------------------------------------------------------------------
def dct2_matrix(n: int) -> np.ndarray:
    """Orthonormal DCT-II: M[f, t] = a_f cos(pi (2t+1) f / (2n)),
    a_0 = sqrt(1/n), a_f = sqrt(2/n) for f >= 1 (0-based f, t)."""
    f = np.arange(n)[:, None]
    t = np.arange(n)[None, :]
    # cos is 4n-periodic in the integer (2t+1)f; reducing it first keeps the
    # argument small and the entries accurate to a few ulps
    M = np.cos(np.pi * (((2 * t + 1) * f) % (4 * n)) / (2.0 * n))
    M[0, :] *= np.sqrt(1.0 / n)
    M[1:, :] *= np.sqrt(2.0 / n)
    return M


def dft_matrix(n: int) -> np.ndarray:
    """Unitary DFT: M[f, t] = n^{-1/2} exp(-2 pi i f t / n) (0-based)."""
    f = np.arange(n)[:, None]
    t = np.arange(n)[None, :]
    return np.exp(-2j * np.pi * ((f * t) % n) / n) / np.sqrt(n)


def m_inverse(M: np.ndarray) -> np.ndarray:
    """Inverse of an orthogonal / unitary transform: M^H."""
    return M.conj().T


def mode3(X: np.ndarray, M: np.ndarray) -> np.ndarray:
    """X x_3 M: every tube X[a, b, :] is multiplied by M (Sec. 2.1: the mode-i
    product is U A_(i); for i = 3 the columns of the unfolding are the tubes).

    Xh[a, b, f] = sum_t M[f, t] X[a, b, t].
    """
    m, p, n = X.shape
    assert M.shape[1] == n
    tubes = X.reshape(m * p, n, order="F")            # row i = tube of (a, b)
    out = tubes @ M.T                                   # row i = (M @ tube)^T
    return np.asfortranarray(out.reshape(m, p, M.shape[0], order="F"))


def inverse_mode3(Xh: np.ndarray, M: np.ndarray) -> np.ndarray:
    return mode3(Xh, m_inverse(M))


# --------------------------------------------------------------------------
# M-product algebra (facewise in the transform domain)
# --------------------------------------------------------------------------
def mprod(A: np.ndarray, B: np.ndarray, M: np.ndarray) -> np.ndarray:
    """C = A *_M B: transform both, multiply matching faces, transform back."""
    Ah, Bh = mode3(A, M), mode3(B, M)
    Ch = np.zeros((Ah.shape[0], Bh.shape[1], Ah.shape[2]), dtype=np.result_type(Ah, Bh),
                  order="F")
    for f in range(Ah.shape[2]):
        Ch[:, :, f] = Ah[:, :, f] @ Bh[:, :, f]
    return inverse_mode3(Ch, M)


def ttranspose(A: np.ndarray, M: np.ndarray) -> np.ndarray:
    """Conjugate transpose under *_M: the transform-domain faces are conj-transposed."""
    Ah = mode3(A, M)
    Th = np.asfortranarray(np.conj(np.transpose(Ah, (1, 0, 2))))
    return inverse_mode3(Th, M)


# --------------------------------------------------------------------------
# Truncation rules and the truncated t-SVDM
# --------------------------------------------------------------------------
def rank_fixed(s: np.ndarray, k: int) -> int:
    return int(min(k, s.shape[0]))


def rank_energy(s: np.ndarray, fro2: float, tau: float, kmax: int | None = None) -> int:
    """Smallest k with sum_{j>k} s_j^2 <= tau^2 * ||face||_F^2 (per face)."""
    ns = s.shape[0]
    cap = ns if kmax is None else min(kmax, ns)
    tail = np.concatenate([np.cumsum((s ** 2)[::-1])[::-1], [0.0]])  # tail[k] = sum_{j>=k}
    bound = tau * tau * fro2
    for k in range(cap + 1):
        if tail[k] <= bound:
            return k
    return cap


def hermitian_pairs(n3: int):
    """For the unitary DFT of a real tensor, face n3-f is the conjugate of face f."""
    return [(f, (n3 - f) % n3) for f in range(n3 // 2 + 1)]


def tsvdm_truncate_faces(Xh: np.ndarray, mode: str = "fixed", k: int = 1, tau: float = 0.0,
                         real_dft: bool = False):
    """Facewise truncated SVD in the transform domain.

    For every face f: SVD by one-sided Jacobi, rank k_f by the rule, keep the
    leading k_f triplets.  Returns dict with U, s, V (full thin factors), ranks,
    fro2 (squared face norms) and That (the truncated faces).

    real_dft: the faces come from the unitary DFT of a real tensor; faces
    f > n3/2 are then taken as the conjugates of faces n3 - f (same singular
    values and rank), so that the result transforms back to a real tensor.
    """
    m, p, nf = Xh.shape
    if real_dft:
        half = nf // 2 + 1
        U, s, V, sw = svd_faces(Xh[:, :, :half])
        Uf = np.zeros((m, U.shape[1], nf), dtype=U.dtype, order="F")
        Vf = np.zeros((p, V.shape[1], nf), dtype=V.dtype, order="F")
        sf = np.zeros((s.shape[0], nf), order="F")
        swf = np.zeros(nf, dtype=np.int32)
        for f in range(nf):
            g = f if f < half else nf - f
            conj = f >= half
            Uf[:, :, f] = np.conj(U[:, :, g]) if conj else U[:, :, g]
            Vf[:, :, f] = np.conj(V[:, :, g]) if conj else V[:, :, g]
            sf[:, f] = s[:, g]
            swf[f] = sw[g]
        U, s, V, sw = Uf, sf, Vf, swf
    else:
        U, s, V, sw = svd_faces(Xh)
    fro2 = np.array([np.sum(np.abs(Xh[:, :, f]) ** 2) for f in range(nf)])
    if real_dft:  # the mirrored face must use the same norm as its partner
        for f in range(nf // 2 + 1, nf):
            fro2[f] = fro2[nf - f]
    ranks = np.zeros(nf, dtype=np.int32)
    for f in range(nf):
        if mode == "fixed":
            ranks[f] = rank_fixed(s[:, f], k)
        elif mode == "energy":
            ranks[f] = rank_energy(s[:, f], fro2[f], tau, kmax=k if k > 0 else None)
        else:
            raise ValueError(mode)
    That = np.zeros_like(Xh, dtype=U.dtype)
    for f in range(nf):
        kf = ranks[f]
        That[:, :, f] = (U[:, :kf, f] * s[:kf, f]) @ np.conj(V[:, :kf, f]).T
    return dict(U=U, s=s, V=V, ranks=ranks, fro2=fro2, That=That, sweeps=sw)


def tsvdm(X: np.ndarray, M: np.ndarray, mode: str = "fixed", k: int = 1, tau: float = 0.0):
    """Truncated t-SVDM of a real tensor: transform, facewise truncation,
    inverse transform.  Returns dict with Xh, the facewise result and T (the
    approximation in the original domain, real part for real input)."""
    Xh = mode3(np.asarray(X, dtype=np.float64), M)
    real_dft = np.iscomplexobj(M)
    res = tsvdm_truncate_faces(Xh, mode, k, tau, real_dft=real_dft)
    T = inverse_mode3(res["That"], M)
    if real_dft:
        T = np.real(T)
    res["Xh"] = Xh
    res["T"] = np.asfortranarray(T)
    return res


def truncation_error(s: np.ndarray, ranks: np.ndarray) -> float:
    """sqrt of the discarded energy, sum_f sum_{j > k_f} s_{f,j}^2."""
    return float(np.sqrt(sum(np.sum(s[ranks[f]:, f] ** 2) for f in range(s.shape[1]))))


# --------------------------------------------------------------------------
# Randomized facewise range finder (double precision reference)
# --------------------------------------------------------------------------
def cholqr(Y: np.ndarray):
    """One Cholesky-QR step: G = Y^H Y = R^H R, Q = Y R^{-1}."""
    import scipy.linalg as sla
    G = np.conj(Y).T @ Y
    R = np.linalg.cholesky(G).conj().T          # upper triangular
    Q = sla.solve_triangular(R, Y.T, trans="T", lower=False).T if not np.iscomplexobj(Y) \
        else Y @ np.linalg.inv(R)
    return Q, R


def cholqr2(Y: np.ndarray):
    """CholeskyQR2 (Fukaya, Nakatsukasa, Yanagisawa, Yamamoto 2014)."""
    Q1, R1 = cholqr(Y)
    Q, R2 = cholqr(Q1)
    return Q, R2 @ R1


def shifted_cholqr3(Y: np.ndarray):
    """Shifted CholeskyQR3 (Fukaya, Kannan, Nakatsukasa, Yamada, Yanagisawa
    2020): a first Cholesky-QR on Y^H Y + s I with
    s = 11 (m n + n (n+1)) u ||Y||_F^2, then CholeskyQR2."""
    import scipy.linalg as sla
    mrows, n = Y.shape
    u = np.finfo(np.float64).eps / 2
    s = 11.0 * (mrows * n + n * (n + 1)) * u * np.sum(np.abs(Y) ** 2)
    G = np.conj(Y).T @ Y + s * np.eye(n)
    R1 = np.linalg.cholesky(G).conj().T
    Q1 = Y @ np.linalg.inv(R1)
    Q, R2 = cholqr2(Q1)
    return Q, R2 @ R1


def householder_qr(Y: np.ndarray):
    """Thin Householder QR (numpy): an orthonormal basis of the columns of Y,
    also when Y is rank deficient (its extra columns then span arbitrary
    directions orthogonal to the range, which the projection B = Q^H F maps
    to zero rows)."""
    Q, R = np.linalg.qr(Y)
    return Q, R


def randomized_face(F: np.ndarray, Omega: np.ndarray, power_iters: int = 1,
                    qr=householder_qr):
    """Randomized range finder with power iteration, then the small SVD
    (Halko, Martinsson, Tropp 2011, Algs. 4.4 and 5.1), all in float64.  The
    range finder only needs an orthonormal basis of each sketch; the default
    is Householder QR, which, unlike Cholesky-based QR, also holds when a
    sketch is exactly rank deficient (inputs of exact rank below ell):

      Y = F Omega; Q = qr(Y)
      repeat power_iters times: Z = F^H Q; Qz = qr(Z); Y = F Qz; Q = qr(Y)
      B = Q^H F; B = U_B diag(s) V^H; U = Q U_B.
    Returns U, s, V (thin, ell columns) and the basis Q.
    """
    Y = F @ Omega
    Q, _ = qr(Y)
    for _ in range(power_iters):
        Z = np.conj(F).T @ Q
        Qz, _ = qr(Z)
        Y = F @ Qz
        Q, _ = qr(Y)
    B = np.conj(Q).T @ F
    UB, s, V, _ = svd_faces(B[:, :, None])
    return Q @ UB[:, :, 0], s[:, 0], V[:, :, 0], Q


def randomized_tsvdm_faces(Xh: np.ndarray, Omega: np.ndarray, k: int, power_iters: int = 1,
                           mode: str = "fixed", tau: float = 0.0):
    """Randomized facewise truncation of a transform-domain tensor (real, or
    complex faces as the DFT gives) with one shared real Gaussian test matrix
    Omega (p x ell); for complex faces the adjoint in the range finder is the
    conjugate transpose and the norms are sums of |x|^2.

    Rank rule on the small SVD: fixed k, or the smallest k <= the cap k with
    ||F||^2 - sum_{j<=k} s_j^2 <= tau^2 ||F||^2 (the left side is the squared
    error of the rank-k result because Q has orthonormal columns), the cap
    when no such k exists.  cert[f] is
    the error ||F - T_f||_F of the kept approximation, formed explicitly."""
    m, p, nf = Xh.shape
    ell = Omega.shape[1]
    dt = np.complex128 if np.iscomplexobj(Xh) else np.float64
    U = np.zeros((m, ell, nf), dtype=dt, order="F")
    V = np.zeros((p, ell, nf), dtype=dt, order="F")
    s = np.zeros((ell, nf), order="F")
    ranks = np.zeros(nf, dtype=np.int32)
    cert = np.zeros(nf)
    That = np.zeros_like(Xh, dtype=dt)
    for f in range(nf):
        F = Xh[:, :, f]
        Uf, sf, Vf, _ = randomized_face(F, Omega, power_iters)
        ns = sf.shape[0]
        U[:, :ns, f], s[:ns, f], V[:, :ns, f] = Uf, sf, Vf
        fro2 = float(np.sum(np.abs(F) ** 2))
        if mode == "fixed":
            kf = min(k, ns)
        else:
            # smallest k <= the cap meeting tau; the cap itself when none does
            kf = min(k, ns)
            for kk in range(min(k, ns) + 1):
                if fro2 - np.sum(sf[:kk] ** 2) <= tau * tau * fro2:
                    kf = kk
                    break
        ranks[f] = kf
        That[:, :, f] = (Uf[:, :kf] * sf[:kf]) @ np.conj(Vf[:, :kf]).T
        cert[f] = np.sqrt(max(np.sum(np.abs(F - That[:, :, f]) ** 2), 0.0))
    return dict(U=U, s=s, V=V, ranks=ranks, cert=cert, That=That)


# --------------------------------------------------------------------------
# Applying the structured approximation  A_hat = M_E[T]  to vectors
# --------------------------------------------------------------------------
def dense_apply(Ahat: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = A_hat x with the dense matrix formed explicitly."""
    return Ahat @ x


def approx_from_factors(U: np.ndarray, s: np.ndarray, V: np.ndarray, ranks: np.ndarray,
                        M: np.ndarray) -> np.ndarray:
    """T = That x_3 M^{-1} from transform-domain factors (all n3 faces):
    That_f = U_f diag(s_f) V_f^H with the leading ranks[f] triplets."""
    m, _, nf = U.shape
    p = V.shape[0]
    That = np.zeros((m, p, nf), dtype=np.result_type(U, V), order="F")
    for f in range(nf):
        kf = ranks[f]
        That[:, :, f] = (U[:, :kf, f] * s[:kf, f]) @ np.conj(V[:, :kf, f]).T
    T = inverse_mode3(That, M)
    return T


def expand_hermitian(Uh: np.ndarray, s: np.ndarray, Vh: np.ndarray, ranks: np.ndarray, n3: int):
    """Full set of n3 DFT faces from the first n3//2+1 of a real tensor."""
    half = n3 // 2 + 1
    m, kk, _ = Uh.shape
    p = Vh.shape[0]
    U = np.zeros((m, kk, n3), dtype=np.complex128, order="F")
    V = np.zeros((p, kk, n3), dtype=np.complex128, order="F")
    S = np.zeros((kk, n3), order="F")
    R = np.zeros(n3, dtype=np.int32)
    for f in range(n3):
        g = f if f < half else n3 - f
        U[:, :, f] = Uh[:, :, g] if f < half else np.conj(Uh[:, :, g])
        V[:, :, f] = Vh[:, :, g] if f < half else np.conj(Vh[:, :, g])
        S[:, f] = s[:, g]
        R[f] = ranks[g]
    return U, S, V, R


# --------------------------------------------------------------------------
# Unfoldings, mode products and HOSVD factors (Sec. 2.1, Sec. 2.4); the
# mode-2 compression of Sec. 6.3
# --------------------------------------------------------------------------
def unfold(X: np.ndarray, mode: int) -> np.ndarray:
    """The mode-i unfolding of Sec. 2.1 for a (m, p, n) tensor:
    mode 1: [X_1, X_2, .., X_n] (m x pn, X_t the frontal slices);
    mode 2: [X_1^T, X_2^T, .., X_n^T] (p x mn);
    mode 3: [sq(X_{:,1,:})^T, .., sq(X_{:,p,:})^T] (n x mp, eq. mode3unfold)."""
    m, p, n = X.shape
    if mode == 1:
        return np.hstack([X[:, :, t] for t in range(n)])
    if mode == 2:
        return np.hstack([X[:, :, t].T for t in range(n)])
    if mode == 3:
        return np.hstack([X[:, b, :].T for b in range(p)])
    raise ValueError("mode must be 1, 2 or 3")


def fold(Am: np.ndarray, mode: int, shape) -> np.ndarray:
    """Inverse of unfold for a tensor of the given shape (m, p, n)."""
    m, p, n = shape
    X = np.zeros(shape, dtype=Am.dtype, order="F")
    if mode == 1:
        for t in range(n):
            X[:, :, t] = Am[:, t * p:(t + 1) * p]
    elif mode == 2:
        for t in range(n):
            X[:, :, t] = Am[:, t * m:(t + 1) * m].T
    elif mode == 3:
        for b in range(p):
            X[:, b, :] = Am[:, b * m:(b + 1) * m].T
    else:
        raise ValueError("mode must be 1, 2 or 3")
    return X


def mode_product(X: np.ndarray, U: np.ndarray, mode: int) -> np.ndarray:
    """X x_i U = fold(U X_(i)) (Sec. 2.1 definition of the mode-i product)."""
    shape = list(X.shape)
    shape[mode - 1] = U.shape[0]
    return fold(U @ unfold(X, mode), mode, tuple(shape))


def sign_fix(W: np.ndarray) -> np.ndarray:
    """Columns of W with their largest-magnitude entry made positive (the
    first such entry on ties): a deterministic choice among the sign-equivalent
    singular vectors."""
    W = np.array(W, dtype=np.float64, copy=True)
    for j in range(W.shape[1]):
        i = int(np.argmax(np.abs(W[:, j])))
        if W[i, j] < 0:
            W[:, j] = -W[:, j]
    return W


def hosvd_factor(X: np.ndarray, mode: int, r: int | None = None):
    """HOSVD factor of one mode (Sec. 2.4): the leading r left singular
    vectors of the mode unfolding (library SVD), sign-fixed, and all the
    singular values of the unfolding."""
    Um, s, _ = np.linalg.svd(unfold(X, mode), full_matrices=False)
    r = Um.shape[1] if r is None else r
    return sign_fix(Um[:, :r]), s


def mode3_transform_matrix(X: np.ndarray) -> np.ndarray:
    """The data-driven orthogonal transform M = W^T, W the full mode-3 HOSVD
    factor of X (n x n): X x_3 M is the mode-3 core of the HOSVD, and face f of
    it carries the energy s_f^2 of the unfolding."""
    W, _ = hosvd_factor(X, 3)
    assert W.shape[0] == W.shape[1], "needs n <= m p"
    return W.T


def mode2_compress(X: np.ndarray, r: int):
    """The mode-2 compression of Sec. 6.3: V the leading r left singular
    vectors of X_(2) (p x r), core G = X x_2 V^T (m x r x n) and the
    approximation T = G x_2 V; the error ||X - T||_F equals the root of the
    discarded squared singular values of X_(2) (Eckart-Young on the
    unfolding, V having orthonormal columns)."""
    V, s = hosvd_factor(X, 2, r)
    G = mode_product(X, V.T, 2)
    T = mode_product(G, V, 2)
    return dict(V=V, G=G, T=T, s=s)


def kron_terms_mode2(V: np.ndarray, G: np.ndarray, E):
    """Kronecker terms of the mode-2 compressed tensor (Sec. 6.3, Thm
    thm:tuckerkron with U = I, W = I): C_j = struct(v_{kj})_{k=1..p}
    (l x q) and D_j = sq(G_{:,j,:}) (m x n), so M_E[G x_2 V] = sum_j C_j kron D_j."""
    r = V.shape[1]
    C = [struct_kron(E, [np.array([[V[k, j]]]) for k in range(V.shape[0])]) for j in range(r)]
    D = [G[:, j, :] for j in range(r)]
    return C, D


def kron_terms_tsvdm(U: np.ndarray, s: np.ndarray, V: np.ndarray, ranks: np.ndarray, M: np.ndarray, E):
    """Kronecker terms of the truncated t-SVDM (the analogue of Thm
    thm:tuckerkron for the t-SVDM; derived): with T = That x_3 M^{-1} and That_f
    = sum_r s_fr U_f[:, r] V_f[:, r]^H, lateral slice b of T is
        sq(T_{:, b, :}) = sum_{f, r} conj(V_f[b, r]) s_fr U_f[:, r] (M^{-1}[:, f])^T,
    so M_E[T] = sum_{f, r} struct(conj V_f[:, r]) kron D_fr with
    D_fr = s_fr U_f[:, r] (M^{-1}[:, f])^T (a rank-one m x n matrix) and
    struct(v) = sum_b E_b v_b (Sec. 3, eq. kronsum).  Factors of all n faces
    (full spectrum); returns the lists C, D."""
    Minv = m_inverse(M)
    C, D = [], []
    for f in range(U.shape[2]):
        for r in range(int(ranks[f])):
            C.append(struct_kron(E, [np.array([[np.conj(V[b, r, f])]]) for b in range(V.shape[0])]))
            D.append(s[r, f] * np.outer(U[:, r, f], Minv[:, f]))
    return C, D


def spsd_two_sided(X: np.ndarray, U: np.ndarray):
    """The two-sided compression of Sec. 5.1 for a tensor X = T_E[A] of a
    symmetric block matrix (m x p x m): G = X x_1 U^T x_3 U^T and
    T = G x_1 U x_3 U."""
    G = mode_product(mode_product(X, U.T, 1), U.T, 3)
    T = mode_product(mode_product(G, U, 1), U, 3)
    return G, T


def spsd_factor(X: np.ndarray, r: int) -> np.ndarray:
    """U of Sec. 5.1: the dominant r left singular vectors of the mode-1
    unfolding (which has the mode-3 unfolding's range for a symmetric block
    matrix)."""
    U, _ = hosvd_factor(X, 1, r)
    return U
