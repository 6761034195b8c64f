"""GPU parity of the data-driven transforms (Sec. 2.4: the mode-3 HOSVD factor
as M) and of the mode-2 compression of Sec. 6.3 against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import from_dev, reconstruct, relerr, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2105_01170_amd import api  # noqa: E402
from paper_2105_01170_amd import tsvdm as C  # noqa: E402


@pytest.mark.parametrize("shape", [(9, 7, 5), (33, 20, 64), (70, 3, 17)])
@pytest.mark.parametrize("mode", [2, 3])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_mode_gram_equals_unfolding_gram(shape, mode, dtype):
    m, p, n = shape
    if (p if mode == 2 else n) > 64:
        pytest.skip("order above 64")
    X = np.asfortranarray(np.random.default_rng(sum(shape) + mode).standard_normal(shape)).astype(dtype)
    G = from_dev(api.mode_gram(to_dev(X), m, p, n, mode), ((p if mode == 2 else n),) * 2)
    Um = oracle.unfold(X.astype(np.float64), mode)
    np.testing.assert_allclose(G, Um @ Um.T, rtol=1e-12, atol=1e-12 * np.max(np.abs(Um @ Um.T)))


@pytest.mark.parametrize("N", [1, 5, 16, 37, 64])
def test_sym_eig_against_library(N):
    g = np.random.default_rng(N)
    Q = np.linalg.qr(g.standard_normal((N, N)))[0]
    lam = np.sort(g.uniform(0.1, 3.0, N) * np.logspace(0, -6, N))[::-1]
    G = np.asfortranarray((Q * lam) @ Q.T)
    lg, Wg = api.sym_eig(to_dev(G), N)
    lg, Wg = from_dev(lg, (N,)), from_dev(Wg, (N, N))
    w, V = np.linalg.eigh(G)
    order = np.argsort(-w, kind="stable")
    np.testing.assert_allclose(lg, w[order], rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(Wg, oracle.sign_fix(V[:, order]), atol=1e-9)
    np.testing.assert_allclose(Wg.T @ Wg, np.eye(N), atol=1e-13)


def _tubes_in_subspace(m, p, n, r, salt, noise=1e-9):
    """X = sum_i a_i o b_i o w_i with w_i random (not sparse in any fixed
    transform) plus relative noise."""
    g = synth.rng(6, salt)
    X = np.zeros((m, p, n))
    for i in range(r):
        X += 10.0 ** (-0.5 * i) * np.einsum("a,b,t->abt", g.standard_normal(m), g.standard_normal(p),
                                           g.standard_normal(n))
    return np.asfortranarray(synth.add_relative_noise(g, X, noise))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_mode3_transform_matches_oracle_and_concentrates_energy(dtype):
    """M = W^T from the GPU's mode-3 Gram equals the oracle's sign-fixed HOSVD
    factor; sv are the singular values of X_(3); the GPU transform with this M
    puts the energy sv_f^2 into face f (closed form)."""
    m, p, n = 24, 30, 20
    X = _tubes_in_subspace(m, p, n, 6, 1, noise=1e-3).astype(dtype)
    Xd = to_dev(X)
    M, sv = api.mode3_transform(Xd, m, p, n)
    M = from_dev(M, (n, n))
    sv = from_dev(sv, (n,))
    Mo = oracle.mode3_transform_matrix(X.astype(np.float64))
    _, so = oracle.hosvd_factor(X.astype(np.float64), 3)
    np.testing.assert_allclose(sv, so, rtol=1e-10, atol=1e-12 * so[0])
    # rows of M for the six well-separated singular values agree entry by entry;
    # the trailing rows span the noise subspace (close singular values, so
    # individual vectors are ill-determined): compare its projector
    np.testing.assert_allclose(M[:6], Mo[:6], atol=1e-9)
    np.testing.assert_allclose(M[6:].T @ M[6:], Mo[6:].T @ Mo[6:], atol=1e-9)
    np.testing.assert_allclose(M @ M.T, np.eye(n), atol=1e-13)
    xh = api.transform(Xd, m, p, n, C.M_DENSE, +1, M=to_dev(M))
    energy = np.sum(from_dev(xh, (m, p, n)).astype(np.float64) ** 2, axis=(0, 1))
    tol = 1e-10 if dtype == np.float64 else 1e-5
    np.testing.assert_allclose(energy, sv ** 2, rtol=tol, atol=tol * sv[0] ** 2)


def test_tsvdm_with_data_driven_transform_against_oracle_and_dct():
    """t-SVDM with M = the mode-3 HOSVD factor (GPU: Gram, Jacobi, dense
    transform, plain FP64 truncation, energy rule) against the oracle's
    t-SVDM with its own HOSVD factor: the same ranks and the same truncated
    tensor in the original domain (M rows agree up to the sign convention,
    which the facewise SVD absorbs), and the energy compaction of the HOSVD
    factor against the DCT-II."""
    m, p, n, tau = 20, 18, 16, 1e-3
    X = _tubes_in_subspace(m, p, n, 5, 2)
    Xd = to_dev(X)
    Md, _ = api.mode3_transform(Xd, m, p, n)
    xh = api.transform(Xd, m, p, n, C.M_DENSE, +1, M=Md)
    tr = api.Truncator(m, p, n, torch.float64, rank_mode=C.RANK_ENERGY, k=0, tau=tau, precision=C.PREC_F64)
    F = tr(xh)
    kmax = F.kmax
    U, S, V = from_dev(F.U, (m, kmax, n)), from_dev(F.S, (kmax, n)), from_dev(F.V, (p, kmax, n))
    ranks = from_dev(F.ranks, (n,))
    Mg = from_dev(Md, (n, n))
    T = oracle.inverse_mode3(reconstruct(U, S, V, ranks), Mg)
    Mo = oracle.mode3_transform_matrix(X)
    ref = oracle.tsvdm(X, Mo, "energy", 0, tau)
    assert np.array_equal(ranks, ref["ranks"])
    assert relerr(T, ref["T"]) < 1e-9
    # energy compaction: the first faces of X x_3 M hold the largest energy any
    # orthogonal M can put there (Eckart-Young on X_(3)); with tubes in a
    # 5-dimensional random subspace, five faces hold all but the noise, while
    # the DCT-II spreads the energy over every face
    e_dd = np.sum(from_dev(xh, (m, p, n)) ** 2, axis=(0, 1))
    e_dct = np.sum(oracle.mode3(X, oracle.dct2_matrix(n)) ** 2, axis=(0, 1))
    assert np.sum(e_dd[:5]) / np.sum(e_dd) > 1 - 1e-12
    assert np.sum(np.sort(e_dct)[::-1][:5]) / np.sum(e_dct) < 0.99


def _block_tridiagonal_tridiagonal_blocks(ell, m, R, salt):
    """A block-tridiagonal matrix (every block in the band distinct, p = 3l - 2)
    whose blocks are tridiagonal: A_k = sum_{i<R} c_{k,i} T_i with random
    tridiagonal m x m matrices T_i and coefficients decaying as 10^-i, so the
    mode-2 unfolding of T_E[A] has rapidly decaying singular values (the
    property the SuiteSparse matrices of Sec. 6.3 are compressed by).  The
    decay 10^(-i/2) keeps the leading eigenvectors well separated."""
    g = synth.rng(7, salt)
    Ts = []
    for _ in range(R):
        Ti = np.diag(g.standard_normal(m)) + np.diag(g.standard_normal(m - 1), 1) + np.diag(g.standard_normal(m - 1), -1)
        Ts.append(Ti)
    block_of, p = C.tsvdm_block_structure(C.PLACE_BANDED, ell, ell, 1)
    blocks = [sum(g.standard_normal() * 10.0 ** (-0.5 * i) * Ts[i] for i in range(R)) for _ in range(p)]
    A = np.zeros((ell * m, ell * m), order="F")
    for j in range(ell):
        for i in range(ell):
            k = block_of[i + ell * j]
            if k >= 0:
                A[i * m:(i + 1) * m, j * m:(j + 1) * m] = blocks[k]
    return A, block_of, p


def test_mode2_compression_of_a_block_tridiagonal_matrix():
    """Sec. 6.3 on the GPU: X = T_E[A] (block-tridiagonal placement, p = 3l - 2
    = 64), V from the mode-2 Gram (leading r eigenvectors), G = X x_2 V^T,
    T = G x_2 V, A_hat = M_E[T] and the Kronecker terms C_j = M_E of v_j
    (a block with m = n = 1), D_j = sq(G_{:,j,:}); against the oracle's
    compression: the error is the root of the discarded eigenvalues, the
    D_j stay tridiagonal, and the compression ratio (p r + nnz(G)) / nnz(A)
    of Table tab:kronsum is computed."""
    ell, m, R, r = 22, 16, 8, 6
    A, block_of, p = _block_tridiagonal_tridiagonal_blocks(ell, m, R, 3)
    assert p == 3 * ell - 2 == 64
    pl = api.Placement(ell, ell, block_of, p)
    X = pl.tensor_from_blockmat(to_dev(A), m, m)
    G2 = api.mode_gram(X, m, p, m, 2)
    lam, W = api.sym_eig(G2, p)
    Vd = W[:p * r].clone()  # leading r eigenvectors, p x r column major
    Gc = api.mode2_product(X, m, p, m, Vd, p, r, +1)
    T = api.mode2_product(Gc, m, r, m, Vd, p, r, -1)
    Ahat = from_dev(pl.blockmat_from_tensor(T, m, m), (ell * m, ell * m))
    lam = from_dev(lam, (p,))
    E = []
    eta = np.zeros(p, dtype=int)
    for v in block_of:
        if v >= 0:
            eta[v] += 1
    for k in range(p):
        Ek = np.zeros((ell, ell))
        for j in range(ell):
            for i in range(ell):
                if block_of[i + ell * j] == k:
                    Ek[i, j] = 1.0 / np.sqrt(eta[k])
        E.append(Ek)
    Xh = oracle.tensor_from_blockmat_E(A, E, m, m)
    ref = oracle.mode2_compress(Xh, r)
    V = from_dev(Vd, (p, r))
    np.testing.assert_allclose(V, ref["V"], atol=1e-9)
    np.testing.assert_allclose(lam, np.concatenate([ref["s"] ** 2, np.zeros(p - len(ref["s"]))]),
                               rtol=1e-9, atol=1e-12 * lam[0])
    Aref = oracle.blockmat_from_tensor_E(ref["T"], E)
    assert relerr(Ahat, Aref) < 1e-10
    err = np.linalg.norm(A - Ahat)
    assert err == pytest.approx(np.sqrt(max(np.sum(lam[r:]), 0.0)), rel=1e-6)
    assert err / np.linalg.norm(A) < 3e-3
    Gh = from_dev(Gc, (m, r, m))
    C_terms, D_terms = [], []
    for j in range(r):
        Cj = from_dev(pl.blockmat_from_tensor(Vd[j * p:(j + 1) * p].contiguous(), 1, 1), (ell, ell))
        C_terms.append(Cj)
        D_terms.append(Gh[:, j, :])
    Co, Do = oracle.kron_terms_mode2(ref["V"], ref["G"], E)
    for j in range(r):
        np.testing.assert_allclose(C_terms[j], Co[j], atol=1e-9)
        np.testing.assert_allclose(D_terms[j], Do[j], atol=1e-9 * np.max(np.abs(Do[j])))
        band = np.abs(np.subtract.outer(np.arange(m), np.arange(m))) > 1
        assert np.max(np.abs(D_terms[j][band])) <= 1e-12 * np.max(np.abs(D_terms[j]))
    Akron = sum(np.kron(Cj, Dj) for Cj, Dj in zip(C_terms, D_terms))
    assert relerr(Akron, Ahat) < 1e-12
    nnzG = sum(int(np.count_nonzero(D)) for D in D_terms)
    ratio = (p * r + nnzG) / np.count_nonzero(A)
    # every D_j and every block tridiagonal: (p r + r (3m - 2)) / (p (3m - 2))
    assert nnzG == r * (3 * m - 2) and np.count_nonzero(A) == p * (3 * m - 2)
    assert ratio == pytest.approx((p * r + r * (3 * m - 2)) / (p * (3 * m - 2)))
