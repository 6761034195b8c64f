"""GPU parity of the truncated t-SVDM as a Kronecker sum (the t-SVDM analogue
of Thm thm:tuckerkron) and as an M-product operator Y = T *_M X, against the
oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import from_dev, reconstruct, relerr, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2105_01170_amd import api  # noqa: E402
from paper_2105_01170_amd import tsvdm as C  # noqa: E402


def _E_list(block_of, ell, q, p):
    E = [np.zeros((ell, q)) for _ in range(p)]
    eta = np.bincount([v for v in block_of if v >= 0], minlength=p)
    for j in range(q):
        for i in range(ell):
            k = block_of[i + ell * j]
            if k >= 0:
                E[k][i, j] = 1.0 / np.sqrt(eta[k])
    return E


def _truncated(m, p, n, kind, k, dtype, salt):
    """The GPU's truncated t-SVDM of a random tensor and the original-domain
    tensor T of its returned factors (formed on the host, FP64)."""
    g = synth.rng(8, salt)
    X = np.asfortranarray(g.standard_normal((m, p, n)))
    M = oracle.dct2_matrix(n) if kind == C.M_DCT2 else oracle.dft_matrix(n)
    if dtype == "f64":
        xh = api.transform(to_dev(X), m, p, n, kind, +1)
        nf = n // 2 + 1 if kind == C.M_DFT else n
        tdt = torch.complex128 if kind == C.M_DFT else torch.float64
        F = api.Truncator(m, p, nf, tdt, k=k, precision=C.PREC_F64, kmax=k)(xh)
    else:
        xh = api.transform(to_dev(X, np.float32), m, p, n, kind, +1)
        nf = n
        omega = to_dev(synth.gaussian(g, (p, k + 4)), np.float32)
        F = api.Truncator(m, p, nf, torch.float32, k=k, precision=C.PREC_MIXED, oversample=4, power_iters=1,
                          omega=omega)(xh)
    kmax = F.kmax
    U = from_dev(F.U, (m, kmax, nf))
    S = from_dev(F.S, (kmax, nf))
    V = from_dev(F.V, (p, kmax, nf))
    ranks = from_dev(F.ranks, (nf,))
    if kind == C.M_DFT:
        Uf, Sf, Vf, Rf = oracle.expand_hermitian(U, S, V, ranks, n)
        T = np.real(oracle.approx_from_factors(Uf, Sf, Vf, Rf, M))
    else:
        T = oracle.inverse_mode3(reconstruct(U.astype(np.float64), S, V.astype(np.float64), ranks), M)
    return F, T, M, X


@pytest.mark.parametrize("kind,dtype", [(C.M_DCT2, "f64"), (C.M_DFT, "f64"), (C.M_DCT2, "f32")])
@pytest.mark.parametrize("structure", [C.PLACE_GENERIC, C.PLACE_TOEPLITZ])
def test_kronecker_terms_sum_to_the_structured_approximation(kind, dtype, structure):
    """sum_j C_j kron D_j = M_E[T] for the returned factors; every D_j has rank
    one (two for the DFT's real and imaginary parts) and every C_j the
    placement's structure."""
    ell = q = 4
    m, n, k = 12, 8, 3
    block_of, p = C.tsvdm_block_structure(structure, ell, q, 0)
    F, T, M, _ = _truncated(m, p, n, kind, k, dtype, 10 + structure + kind)
    pl = api.Placement(ell, q, block_of, p) if structure != C.PLACE_GENERIC else None
    Cd, Dd, nt = api.kron_terms(F, kind, n, ell, q, placement=pl)
    Cs = from_dev(Cd, (ell * q * nt,)).reshape((ell, q, nt), order="F").astype(np.float64)
    Ds = from_dev(Dd, (m * n * nt,)).reshape((m, n, nt), order="F").astype(np.float64)
    E = _E_list(block_of, ell, q, p)
    want = oracle.blockmat_from_tensor_E(T, E)
    got = sum(np.kron(Cs[:, :, j], Ds[:, :, j]) for j in range(nt))
    tol = 1e-11 if dtype == "f64" else 1e-5
    assert relerr(got, want) < tol
    # D_j = s u (M^{-1}[:, f])^T has rank one; for the DFT the real and the
    # imaginary part of a complex rank-one matrix each have rank at most two
    rk = 2 if kind == C.M_DFT else 1
    for j in range(nt):
        Dj = Ds[:, :, j]
        if np.any(Dj):
            sv = np.linalg.svd(Dj, compute_uv=False)
            assert sv[rk] <= 1e-6 * sv[0]
    if structure == C.PLACE_TOEPLITZ:  # a Toeplitz placement gives Toeplitz C_j
        for j in range(nt):
            Cj = Cs[:, :, j]
            for d in range(-q + 1, ell):
                diag = np.diagonal(Cj, -d)
                np.testing.assert_allclose(diag, diag[0], atol=1e-14 * max(np.abs(Cj).max(), 1e-300))


@pytest.mark.parametrize("kind,dtype", [(C.M_DCT2, "f64"), (C.M_DFT, "f64"), (C.M_DCT2, "f32")])
@pytest.mark.parametrize("s", [1, 70])
def test_mprod_operator_against_oracle(kind, dtype, s):
    """Y = T *_M X with the GPU's factors against the oracle's M-product of T
    and X (pinned by the block-circulant definition for the DFT)."""
    m, p, n, k = 20, 36, 16, 5
    F, T, M, _ = _truncated(m, p, n, kind, k, dtype, 20 + kind + s)
    g = synth.rng(8, 99 + s)
    X = np.asfortranarray(g.standard_normal((p, s, n)))
    npdt = np.float64 if dtype == "f64" else np.float32
    Y = from_dev(api.mprod(F, kind, n, to_dev(X, npdt), s), (m, s, n)).astype(np.float64)
    ref = np.real(oracle.mprod(T, X.astype(npdt).astype(np.float64), M))
    tol = 1e-11 if dtype == "f64" else 2e-5
    assert relerr(Y, ref) < tol


def test_mprod_operator_bcirc_shape():
    """The other reading of the 4096^2 apply: T (64 x 64 x 64, rank 16 per
    face, DFT) as a block-circulant operator on X (64 x 96 x 64); against the
    oracle's M-product."""
    m = p = n = 64
    k, s = 16, 96
    g = synth.rng(8, 7)
    U = np.asfortranarray(g.standard_normal((m, k, n)))
    V = np.asfortranarray(g.standard_normal((p, k, n)))
    sig = 10.0 ** (-np.arange(1, k + 1) / 8.0)
    Th = np.zeros((m, p, n), dtype=complex, order="F")
    M = oracle.dft_matrix(n)
    Uh, Vh = oracle.mode3(U, M), oracle.mode3(V, M)
    for f in range(n):
        Th[:, :, f] = (Uh[:, :, f] * sig) @ np.conj(Vh[:, :, f]).T
    T = np.real(oracle.inverse_mode3(Th, M))
    xh = api.transform(to_dev(T), m, p, n, C.M_DFT, +1)
    nf = n // 2 + 1
    F = api.Truncator(m, p, nf, torch.complex128, k=k, precision=C.PREC_F64, kmax=k)(xh)
    X = np.asfortranarray(g.standard_normal((p, s, n)))
    Y = from_dev(api.mprod(F, C.M_DFT, n, to_dev(X), s), (m, s, n))
    ref = np.real(oracle.mprod(T, X, M))
    assert relerr(Y, ref) < 1e-10
