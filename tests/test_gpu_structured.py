"""GPU parity of the structured placements (Sec. 3): T_E and M_E for the
block-diagonal, block-banded, block-Toeplitz, block-Hankel and generic
structures against the oracle's maps, bit for bit; the t-SVDM of a
structured matrix and the structured apply against the oracle's dense
product."""
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
    """The tuple E of Sec. 3 from the block map: E_k = 1/sqrt(eta_k) at the
    positions of distinct block k."""
    E = [np.zeros((ell, q)) for _ in range(p)]
    eta = np.zeros(p, dtype=int)
    for v in block_of:
        if v >= 0:
            eta[v] += 1
    for j in range(q):
        for i in range(ell):
            k = block_of[i + ell * j]
            if k >= 0:
                E[k][i, j] = 1.0 / np.sqrt(eta[k])
    return E, eta


def _structured_matrix(block_of, ell, q, p, m, n, g):
    """A block matrix with the given block map and iid N(0,1) distinct blocks."""
    blocks = [g.standard_normal((m, n)) for _ in range(p)]
    A = np.zeros((ell * m, q * n), order="F")
    for j in range(q):
        for i in range(ell):
            k = block_of[i + ell * j]
            if k >= 0:
                A[i * m:(i + 1) * m, j * n:(j + 1) * n] = blocks[k]
    return A


CASES = [(C.PLACE_GENERIC, 3, 4, 0), (C.PLACE_DIAGONAL, 4, 4, 0), (C.PLACE_BANDED, 5, 5, 1),
         (C.PLACE_BANDED_SYM, 6, 6, 2), (C.PLACE_TOEPLITZ, 5, 4, 0), (C.PLACE_TOEPLITZ_SYM, 5, 5, 0),
         (C.PLACE_HANKEL, 4, 6, 0)]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_structured_maps_equal_oracle(case, dtype):
    """T_E[A] (a padded leading dimension) and M_E of the result equal the
    oracle's maps bit for bit; M_E[T_E[A]] = A; eta is the occurrence count."""
    kind, ell, q, b = case
    m, n = 7, 5
    pl = api.Placement.structure(kind, ell, q, b)
    p = pl.p
    E, eta = _E_list(pl.block_of, ell, q, p)
    assert pl.eta() == list(eta)
    g = np.random.default_rng(100 + kind)
    A = _structured_matrix(pl.block_of, ell, q, p, m, n, g).astype(dtype)
    lda = ell * m + 3
    Apad = np.zeros((lda, q * n), dtype=dtype, order="F")
    Apad[:ell * m] = A
    X = from_dev(pl.tensor_from_blockmat(to_dev(Apad), m, n, lda=lda), (m, p, n))
    Xo = oracle.tensor_from_blockmat_E(A, E, m, n)
    assert X.dtype == Xo.dtype and np.array_equal(X, Xo)
    A2 = from_dev(pl.blockmat_from_tensor(to_dev(X), m, n), (ell * m, q * n))
    Ao = oracle.blockmat_from_tensor_E(Xo.astype(np.float64), E)
    assert np.array_equal(A2, Ao.astype(dtype))
    tol = 1e-15 if dtype == np.float64 else 1e-7
    np.testing.assert_allclose(A2, A, rtol=tol, atol=0)


def _low_rank_structured(kind, ell, q, b, m, n, rank, noise, salt):
    """X0 = sum of `rank` outer products u_r o v_r o w_r plus relative noise
    (m x p x n), and A = M_E[X0] (the oracle's map): a structured matrix whose
    tensor has low tubal rank."""
    block_of, p = C.tsvdm_block_structure(kind, ell, q, b)
    E, _ = _E_list(block_of, ell, q, p)
    g = synth.rng(5, salt)
    X0 = np.zeros((m, p, n))
    for _ in range(rank):
        X0 += np.einsum("a,b,t->abt", g.standard_normal(m), g.standard_normal(p), g.standard_normal(n))
    X0 = synth.add_relative_noise(g, X0, noise)
    A = oracle.blockmat_from_tensor_E(X0, E)
    return np.asfortranarray(A), block_of, p, E


@pytest.mark.parametrize("kind,b", [(C.PLACE_TOEPLITZ, 0), (C.PLACE_BANDED, 2)])
def test_structured_tsvdm_pipeline_and_apply_f64(kind, b):
    """Algorithm alg:strategy on a structured matrix, on the GPU: T_E, DCT-II,
    plain FP64 truncation to the tensor's rank, and the structured apply
    y = M_E[T] x; against the oracle's t-SVDM of T_E[A] and its dense
    product, and Lemma lem:tenapprox on the GPU's result."""
    ell = q = 12
    m, n, k = 16, 16, 3
    A, block_of, p, E = _low_rank_structured(kind, ell, q, b, m, n, k, 1e-9, 10 + kind)
    pl = api.Placement(ell, q, block_of, p)
    xd = pl.tensor_from_blockmat(to_dev(A), m, n)
    xh = api.transform(xd, m, p, n, C.M_DCT2, +1)
    tr = api.Truncator(m, p, n, torch.float64, k=k, precision=C.PREC_F64)
    F = tr(xh)
    U, S, V = from_dev(F.U, (m, k, n)), from_dev(F.S, (k, n)), from_dev(F.V, (p, k, n))
    ranks = from_dev(F.ranks, (n,))
    M = oracle.dct2_matrix(n)
    X = oracle.tensor_from_blockmat_E(A, E, m, n)
    ref = oracle.tsvdm(X, M, "fixed", k)
    That = reconstruct(U, S, V, ranks)
    assert relerr(That, ref["That"]) < 1e-10
    T = oracle.inverse_mode3(That, M)
    Ahat = oracle.blockmat_from_tensor_E(T, E)
    assert np.linalg.norm(A - Ahat) == pytest.approx(np.linalg.norm(X - T), rel=1e-9)  # Lemma lem:tenapprox
    assert relerr(Ahat, A) < 1e-8
    x = synth.gaussian(synth.rng(5, 99), (q * n, 9))
    y = from_dev(pl.apply(F, C.M_DCT2, n, to_dev(x)), (ell * m, 9))
    Aref = oracle.blockmat_from_tensor_E(ref["T"], E)
    y_ref = oracle.dense_apply(Aref, x)
    assert relerr(y, y_ref) < 1e-10


@pytest.mark.parametrize("kind,b", [(C.PLACE_TOEPLITZ, 0), (C.PLACE_HANKEL, 0), (C.PLACE_BANDED_SYM, 1)])
def test_structured_apply_dft_complex_f64(kind, b):
    """The structured apply with the DFT (complex factors of the stored half
    spectrum, plain FP64 truncation) against the oracle's dense product."""
    ell, q, m, n, k = 6, 6, 10, 8, 2
    A, block_of, p, E = _low_rank_structured(kind, ell, q, b, m, n, k, 1e-3, 20 + kind)
    pl = api.Placement(ell, q, block_of, p)
    xd = pl.tensor_from_blockmat(to_dev(A), m, n)
    xh = api.transform(xd, m, p, n, C.M_DFT, +1)
    half = n // 2 + 1
    tr = api.Truncator(m, p, half, torch.complex128, k=k, precision=C.PREC_F64, kmax=k)
    F = tr(xh)
    X = oracle.tensor_from_blockmat_E(A, E, m, n)
    ref = oracle.tsvdm(X, oracle.dft_matrix(n), "fixed", k)
    Aref = np.real(oracle.blockmat_from_tensor_E(ref["T"], E))
    x = synth.gaussian(synth.rng(5, 98), (q * n, 7))
    y = from_dev(pl.apply(F, C.M_DFT, n, to_dev(x)), (ell * m, 7))
    assert relerr(y, oracle.dense_apply(Aref, x)) < 1e-10


@pytest.mark.parametrize("kind,b", [(C.PLACE_TOEPLITZ, 0), (C.PLACE_BANDED, 1), (C.PLACE_DIAGONAL, 0)])
def test_structured_mixed_truncation_and_apply_f32(kind, b):
    """FP32 storage: T_E, DCT-II, the mixed-precision truncation and the
    structured apply on FP32 matrix cores (zero blocks included), against
    the oracle's exact truncation and dense product at 1e-4."""
    ell = q = 8
    m, n, k = 24, 16, 4
    A, block_of, p, E = _low_rank_structured(kind, ell, q, b, m, n, k, 1e-8, 30 + kind)
    os_ = min(8, min(m, p) - k)  # the block-diagonal tensor has only p = 8 lateral slices
    pl = api.Placement(ell, q, block_of, p)
    A32 = A.astype(np.float32)
    xd = pl.tensor_from_blockmat(to_dev(A32), m, n)
    xh = api.transform(xd, m, p, n, C.M_DCT2, +1)
    omega = to_dev(synth.gaussian(synth.rng(5, 97), (p, k + os_)), np.float32)
    tr = api.Truncator(m, p, n, torch.float32, k=k, precision=C.PREC_MIXED, oversample=os_, power_iters=1,
                       omega=omega)
    F = tr(xh)
    X = oracle.tensor_from_blockmat_E(A32.astype(np.float64), E, m, n)
    ref = oracle.tsvdm(X, oracle.dct2_matrix(n), "fixed", k)
    Fk = F.kmax
    U = from_dev(F.U, (m, Fk, n)).astype(np.float64)
    S = from_dev(F.S, (Fk, n))
    V = from_dev(F.V, (p, Fk, n)).astype(np.float64)
    assert relerr(reconstruct(U, S, V, from_dev(F.ranks, (n,))), ref["That"]) < 1e-4
    x = synth.gaussian(synth.rng(5, 96), (q * n, 70))
    y = from_dev(pl.apply(F, C.M_DCT2, n, to_dev(x, np.float32)), (ell * m, 70))
    Aref = oracle.blockmat_from_tensor_E(ref["T"], E)
    assert relerr(y, oracle.dense_apply(Aref, x)) < 1e-4


def test_generic_placement_apply_equals_generic_apply():
    """With the generic structure (every block distinct, eta = 1) the
    structured apply gives the generic tsvdm_apply's result bit for bit."""
    ell, q, m, n, k = 4, 5, 12, 8, 3
    g = np.random.default_rng(41)
    A = np.asfortranarray(g.standard_normal((ell * m, q * n)))
    pl = api.Placement.structure(C.PLACE_GENERIC, ell, q)
    p = ell * q
    xd = pl.tensor_from_blockmat(to_dev(A), m, n)
    xh = api.transform(xd, m, p, n, C.M_DCT2, +1)
    F = api.Truncator(m, p, n, torch.float64, k=k, precision=C.PREC_F64)(xh)
    x = to_dev(g.standard_normal((q * n, 5)))
    y1 = pl.apply(F, C.M_DCT2, n, x)
    y2 = api.apply(F, C.M_DCT2, n, ell, q, x)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
