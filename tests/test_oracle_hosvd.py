"""Pins of the oracle's unfoldings, mode products, HOSVD factors and the
mode-2 compression (Sec. 2.1, Sec. 2.4, Sec. 6.3), no GPU."""
import numpy as np
import pytest

import oracle


def _rand(shape, seed):
    return np.asfortranarray(np.random.default_rng(seed).standard_normal(shape))


def test_mode_products_are_the_facewise_textbook_products():
    """X x_1 U multiplies every frontal face on the left, X x_2 V on the right
    by V^T, and X x_3 M is the explicit per-tube transform (three independent
    formulas for the three unfoldings of Sec. 2.1)."""
    m, p, n = 4, 5, 3
    X = _rand((m, p, n), 1)
    U, V, M = _rand((6, m), 2), _rand((2, p), 3), _rand((n, n), 4)
    Y1 = oracle.mode_product(X, U, 1)
    Y2 = oracle.mode_product(X, V, 2)
    for t in range(n):
        np.testing.assert_allclose(Y1[:, :, t], U @ X[:, :, t], rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(Y2[:, :, t], X[:, :, t] @ V.T, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(oracle.mode_product(X, M, 3), oracle.mode3(X, M), rtol=1e-13, atol=1e-13)
    for mode in (1, 2, 3):
        assert np.array_equal(oracle.fold(oracle.unfold(X, mode), mode, X.shape), X)
    assert oracle.unfold(X, 1).shape == (m, p * n)
    assert oracle.unfold(X, 2).shape == (p, m * n)
    assert oracle.unfold(X, 3).shape == (n, m * p)


def _tucker(ranks, dims, seed):
    g = np.random.default_rng(seed)
    G = np.asfortranarray(g.standard_normal(ranks))
    U = np.linalg.qr(g.standard_normal((dims[0], ranks[0])))[0]
    V = np.linalg.qr(g.standard_normal((dims[1], ranks[1])))[0]
    W = np.linalg.qr(g.standard_normal((dims[2], ranks[2])))[0]
    X = oracle.mode_product(oracle.mode_product(oracle.mode_product(G, U, 1), V, 2), W, 3)
    return X, G, U, V, W


def test_mode3_unfolding_of_a_tucker_tensor():
    """eq. mode3flatkron: X_(3) = W G_(3) (V^T kron U^T), and eq. klatslice:
    sq(X_{:,k,:}) = U (sum_j v_kj sq(G_{:,j,:})) W^T."""
    X, G, U, V, W = _tucker((2, 3, 2), (5, 4, 6), 5)
    lhs = oracle.unfold(X, 3)
    rhs = W @ oracle.unfold(G, 3) @ np.kron(V.T, U.T)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-13)
    for k in range(X.shape[1]):
        S = sum(V[k, j] * G[:, j, :] for j in range(G.shape[1]))
        np.testing.assert_allclose(X[:, k, :], U @ S @ W.T, rtol=1e-12, atol=1e-13)


def test_hosvd_recovers_a_tucker_tensor_and_mode3_transform_energies():
    """HOSVD (Sec. 2.4) with the multilinear ranks reproduces a Tucker tensor;
    the data-driven transform M = W^T is orthogonal and puts the energy s_f^2
    of the mode-3 unfolding into face f (a decreasing profile)."""
    X, *_ = _tucker((2, 3, 3), (6, 5, 4), 6)
    U, _ = oracle.hosvd_factor(X, 1, 2)
    V, _ = oracle.hosvd_factor(X, 2, 3)
    W, _ = oracle.hosvd_factor(X, 3, 3)
    core = oracle.mode_product(oracle.mode_product(oracle.mode_product(X, U.T, 1), V.T, 2), W.T, 3)
    Y = oracle.mode_product(oracle.mode_product(oracle.mode_product(core, U, 1), V, 2), W, 3)
    np.testing.assert_allclose(Y, X, rtol=1e-12, atol=1e-12)
    Z = _rand((7, 5, 6), 7)
    M = oracle.mode3_transform_matrix(Z)
    np.testing.assert_allclose(M @ M.T, np.eye(6), atol=1e-13)
    _, s = oracle.hosvd_factor(Z, 3)
    Zh = oracle.mode3(Z, M)
    energy = np.sum(Zh ** 2, axis=(0, 1))
    np.testing.assert_allclose(energy, s ** 2, rtol=1e-12)
    assert np.all(np.diff(energy) <= 0)
    # sign convention: the largest-magnitude entry of every row of M is positive
    for f in range(6):
        assert M[f, np.argmax(np.abs(M[f]))] > 0


def test_mode2_compression_error_and_kronecker_terms():
    """Sec. 6.3: G = X x_2 V^T with V from X_(2); the error of T = G x_2 V is the
    root of the discarded squared singular values of X_(2) (Eckart-Young),
    and M_E[T] = sum_j C_j kron D_j with C_j = struct(v_{kj}) (block
    tridiagonal for the tridiagonal placement) and D_j = sq(G_{:,j,:})
    (Thm thm:tuckerkron with U = I, W = I)."""
    ell, m = 5, 3
    # block-tridiagonal placement, every block in the band distinct: p = 3l - 2
    occ = [(i, j) for j in range(ell) for i in range(ell) if abs(i - j) <= 1]
    p = len(occ)
    assert p == 3 * ell - 2
    E = []
    for (i, j) in occ:
        Ek = np.zeros((ell, ell))
        Ek[i, j] = 1.0
        E.append(Ek)
    X = _rand((m, p, m), 8)
    r = 4
    res = oracle.mode2_compress(X, r)
    err = np.linalg.norm(X - res["T"])
    assert err == pytest.approx(np.sqrt(np.sum(res["s"][r:] ** 2)), rel=1e-10)
    np.testing.assert_allclose(res["V"].T @ res["V"], np.eye(r), atol=1e-13)
    C, D = oracle.kron_terms_mode2(res["V"], res["G"], E)
    Ahat = sum(np.kron(Cj, Dj) for Cj, Dj in zip(C, D))
    np.testing.assert_allclose(Ahat, oracle.blockmat_from_tensor_E(res["T"], E), rtol=1e-12, atol=1e-13)
    for Cj in C:
        for i in range(ell):
            for j in range(ell):
                if abs(i - j) > 1:
                    assert Cj[i, j] == 0.0
    # full mode-2 rank: exact
    full = oracle.mode2_compress(X, p)
    np.testing.assert_allclose(full["T"], X, atol=1e-12)


@pytest.mark.parametrize("kind", ["dct", "dft"])
def test_kronecker_terms_of_the_tsvdm(kind):
    """M_E[T] of a truncated t-SVDM equals the sum of the Kronecker terms
    struct(conj v_fr) kron s_fr u_fr (M^{-1}[:, f])^T (generic placement and a
    block-Toeplitz placement); each D_fr has rank one."""
    ell, q, m, n, k = 3, 3, 4, 6, 2
    M = oracle.dct2_matrix(n) if kind == "dct" else oracle.dft_matrix(n)
    Ed = np.diag(np.ones(ell - 1), -1)
    toep = [np.linalg.matrix_power(Ed, j) / np.sqrt(ell - j) for j in range(ell)] + \
        [np.linalg.matrix_power(Ed.T, j) / np.sqrt(ell - j) for j in range(1, ell)]
    for E in (oracle.placement_generic(ell, q), toep):
        p = len(E)
        X = _rand((m, p, n), 11 + p)
        res = oracle.tsvdm(X, M, "fixed", k)
        Uf, sf, Vf = [], [], []
        for f in range(n):
            u, sv, vh = np.linalg.svd(res["Xh"][:, :, f], full_matrices=False)
            Uf.append(u[:, :k])
            sf.append(sv[:k])
            Vf.append(np.conj(vh[:k]).T)
        U, s, V = np.stack(Uf, 2), np.stack(sf, 1), np.stack(Vf, 2)
        C, D = oracle.kron_terms_tsvdm(U, s, V, np.full(n, k), M, E)
        assert len(C) == n * k
        total = sum(np.kron(Cj, Dj) for Cj, Dj in zip(C, D))
        want = oracle.blockmat_from_tensor_E(res["T"], E)
        np.testing.assert_allclose(total, want, atol=1e-12)
        if kind == "dft":
            assert np.max(np.abs(np.imag(total))) < 1e-12
        for Dj in D:
            assert np.linalg.matrix_rank(Dj, tol=1e-12 * max(np.abs(Dj).max(), 1e-300)) <= 1


def test_spsd_two_sided_compression_pins():
    """Sec. 5.1 on a small symmetric block-Toeplitz covariance (Sec. 6.2's
    kernel): the mode-1 and mode-3 unfoldings of T_E[C] have the same range;
    M_E[G x_1 U x_3 U] = (I kron P) C (I kron P) with P = U U^T; the
    approximation stays positive semidefinite; tr = T tr(U^T C_1 U)."""
    import synth
    N, T, r = 12, 5, 4
    blocks, _, _ = synth.spacetime_covariance(N, T, salt=3)
    # symmetric block-Toeplitz placement: block (i, j) is C_{|i-j|}, eta_k = 2(T-k) (T for k = 0)
    E = []
    for k in range(T):
        Ek = np.zeros((T, T))
        for i in range(T):
            for j in range(T):
                if abs(i - j) == k:
                    Ek[i, j] = 1.0
        E.append(Ek / np.linalg.norm(Ek))
    eta = [np.count_nonzero(Ek) for Ek in E]
    Cmat = oracle.struct_kron(E, [np.sqrt(e) * blocks[:, :, k] for k, e in enumerate(eta)])
    assert np.allclose(Cmat, Cmat.T) and np.min(np.linalg.eigvalsh(Cmat)) > -1e-10
    X = oracle.tensor_from_blockmat_E(Cmat, E, N, N)
    W1, _ = oracle.hosvd_factor(X, 1)
    W3, _ = oracle.hosvd_factor(X, 3)
    np.testing.assert_allclose(W1 @ W1.T, W3 @ W3.T, atol=1e-10)
    U = oracle.spsd_factor(X, r)
    G, Tt = oracle.spsd_two_sided(X, U)
    Chat = oracle.blockmat_from_tensor_E(Tt, E)
    P = U @ U.T
    IP = np.kron(np.eye(T), P)
    np.testing.assert_allclose(Chat, IP @ Cmat @ IP, atol=1e-12)
    assert np.min(np.linalg.eigvalsh(Chat)) > -1e-12
    assert np.trace(Chat) == pytest.approx(T * np.trace(U.T @ blocks[:, :, 0] @ U), rel=1e-12)
    assert np.trace(Cmat) == pytest.approx(N * T, rel=1e-14)
