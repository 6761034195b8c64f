"""Pins for the oracle: checks against what the paper and the mathematics fix,
never against the oracle's own formulas retyped.  CPU only (not marked gpu).

Each test names the passage or the independent fact it rests on.
"""
import os

import numpy as np
import pytest
import scipy.fft

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand(shape, seed, cplx=False):
    g = np.random.default_rng(seed)
    a = g.standard_normal(shape)
    if cplx:
        a = a + 1j * g.standard_normal(shape)
    return np.asfortranarray(a)


def _load(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


# ------------------------------------------------------------ transforms
@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 8, 32, 64, 256])
def test_dct2_matrix_matches_library_dct(n):
    """Explicit DCT-II matrix against scipy's orthonormal DCT-II (library)."""
    x = _rand((n, 5), n)
    ref = scipy.fft.dct(x, type=2, norm="ortho", axis=0)
    assert np.max(np.abs(oracle.dct2_matrix(n) @ x - ref)) < 1e-13


def test_dct2_golden_closed_form():
    """Length-4 orthonormal DCT-II against its exact trigonometric values."""
    assert np.max(np.abs(oracle.dct2_matrix(4) - _load("dct2_n4.txt"))) < 1e-15


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 33, 64])
def test_dft_matrix_matches_library_fft(n):
    x = _rand((n, 4), n + 100, cplx=True)
    ref = np.fft.fft(x, axis=0, norm="ortho")
    assert np.max(np.abs(oracle.dft_matrix(n) @ x - ref)) < 1e-13


@pytest.mark.parametrize("kind", ["dct", "dft"])
def test_mode3_matches_library_transform_along_tubes(kind):
    """X x_3 M applies M to every tube (Sec. 2.1 mode-i product); compared with
    the library transform along axis 2, which also pins the reshapes."""
    X = _rand((5, 7, 16), 3)
    if kind == "dct":
        got = oracle.mode3(X, oracle.dct2_matrix(16))
        ref = scipy.fft.dct(X, type=2, norm="ortho", axis=2)
    else:
        got = oracle.mode3(X, oracle.dft_matrix(16))
        ref = np.fft.fft(X, axis=2, norm="ortho")
    assert np.max(np.abs(got - ref)) < 1e-13


@pytest.mark.parametrize("kind", ["dct", "dft", "orth"])
def test_transform_is_frobenius_isometry_and_invertible(kind):
    """vec(X x_3 M) = (M kron I) vec X and Kronecker products of orthogonal
    matrices are orthogonal (Sec. 2.2, properties 1 and 3), so the norm is kept."""
    n = 12
    if kind == "dct":
        M = oracle.dct2_matrix(n)
    elif kind == "dft":
        M = oracle.dft_matrix(n)
    else:
        M, _ = np.linalg.qr(_rand((n, n), 9))
    X = _rand((6, 4, n), 4)
    Xh = oracle.mode3(X, M)
    assert abs(np.linalg.norm(Xh) - np.linalg.norm(X)) < 1e-13 * np.linalg.norm(X)
    assert np.max(np.abs(oracle.inverse_mode3(Xh, M) - X)) < 1e-13


# ------------------------------------------------------------ Jacobi SVD
@pytest.mark.parametrize("shape", [(9, 4), (4, 9), (6, 6), (1, 5), (5, 1), (33, 17)])
@pytest.mark.parametrize("cplx", [False, True])
def test_jacobi_svd_against_library(shape, cplx):
    A = _rand(shape, 11, cplx)
    U, s, V, sw = oracle.svd_faces(A)
    U, s, V = U[:, :, 0], s[:, 0], V[:, :, 0]
    assert sw[0] > 0
    ref = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(s - ref)) < 1e-12 * ref[0]
    assert np.all(np.diff(s) <= 0)
    assert np.max(np.abs((U * s) @ V.conj().T - A)) < 1e-13 * np.linalg.norm(A)
    ns = min(shape)
    assert np.max(np.abs(U.conj().T @ U - np.eye(ns))) < 1e-13
    assert np.max(np.abs(V.conj().T @ V - np.eye(ns))) < 1e-13


def test_jacobi_svd_rank_deficient_and_graded():
    """Rank-deficient input: trailing singular values are rounding-level; a
    graded spectrum down to 1e-12 is resolved to high relative accuracy."""
    g = np.random.default_rng(5)
    Qa, _ = np.linalg.qr(g.standard_normal((20, 8)))
    Qb, _ = np.linalg.qr(g.standard_normal((12, 8)))
    sig = 10.0 ** -np.arange(8.0) * np.array([1, 1, 1, 1, 1, 1, 1, 0.0])
    A = (Qa * sig) @ Qb.T
    _, s, _, _ = oracle.svd_faces(A)
    assert np.max(np.abs(s[:7, 0] - sig[:7]) / sig[:7]) < 1e-9
    assert np.all(s[7:, 0] < 1e-14)


# ------------------------------------------------------------ Sec. 3 maps
def test_block_maps_roundtrip_bit_exact():
    """M_E[T_E[A]] = A (Sec. 3), exactly, for the generic blocking."""
    ell, q, m, n = 3, 4, 5, 2
    A = _rand((ell * m, q * n), 1)
    X = oracle.tensor_from_blockmat(A, ell, q, m, n)
    assert X.shape == (m, ell * q, n)
    assert np.array_equal(oracle.blockmat_from_tensor(X, ell, q), A)
    # generic E as a Kronecker sum, eq. kronsum: struct(A) = A
    E = oracle.placement_generic(ell, q)
    assert np.array_equal(oracle.struct_kron(E, [X[:, b, :] for b in range(ell * q)]), A)
    # Frobenius norm is preserved (Lemma lem:tenapprox with a zero approximation)
    assert np.linalg.norm(X) == pytest.approx(np.linalg.norm(A), rel=1e-15)


def test_paper_block_tridiagonal_example_golden():
    """Sec. 3 block-banded example: 4 x 4 blocks, p = 7 distinct blocks,
    ||E_k||_F = 1 (eq. fnormw), struct(A) = A (eq. kronsum), and the error
    transfer of Lemma lem:tenapprox for an arbitrary tensor perturbation."""
    occ = _load("block_tridiagonal_4x4.txt").astype(int)
    ell = 4
    p = occ[:, 0].max()
    assert p == 7 == 2 * ell - 1
    m, n = 3, 2
    g = np.random.default_rng(7)
    blocks = [g.standard_normal((m, n)) for _ in range(p)]
    A = np.zeros((ell * m, ell * n))
    for k, i, j in occ:
        A[(i - 1) * m:i * m, (j - 1) * n:j * n] = blocks[k - 1]
    E = []
    for k in range(1, p + 1):
        rows = occ[occ[:, 0] == k]
        Ek = np.zeros((ell, ell))
        for _, i, j in rows:
            Ek[i - 1, j - 1] = 1.0 / np.sqrt(len(rows))
        E.append(Ek)
    for Ek in E:
        assert np.linalg.norm(Ek) == pytest.approx(1.0, abs=1e-15)
    eta = [int(np.count_nonzero(Ek)) for Ek in E]
    assert np.max(np.abs(oracle.struct_kron(E, [np.sqrt(e) * B for e, B in zip(eta, blocks)]) - A)) < 1e-14
    X = oracle.tensor_from_blockmat_E(A, E, m, n)
    assert np.max(np.abs(oracle.blockmat_from_tensor_E(X, E) - A)) < 1e-14
    T = X + 1e-3 * g.standard_normal(X.shape)
    lhs = np.linalg.norm(A - oracle.blockmat_from_tensor_E(T, E))
    assert lhs == pytest.approx(np.linalg.norm(X - T), rel=1e-12)


def test_block_toeplitz_placement():
    """Sec. 3 block-Toeplitz example: 2l-1 distinct blocks from powers of the
    down/up shift matrices with weights 1/sqrt(l - j); struct(A) = A and
    ||E_k||_F = 1."""
    ell, m, n = 5, 2, 3
    g = np.random.default_rng(8)
    blocks = [g.standard_normal((m, n)) for _ in range(2 * ell - 1)]
    Ed = np.diag(np.ones(ell - 1), -1)
    E, Bs = [], []
    for j in range(ell):               # A_1..A_l on the main and lower diagonals
        E.append(np.linalg.matrix_power(Ed, j) / np.sqrt(ell - j))
        Bs.append(blocks[j])
    for j in range(1, ell):            # A_{l+1}..A_{2l-1} on the upper diagonals
        E.append(np.linalg.matrix_power(Ed.T, j) / np.sqrt(ell - j))
        Bs.append(blocks[ell - 1 + j])
    A = np.zeros((ell * m, ell * n))
    for i in range(ell):
        for jj in range(ell):
            d = i - jj
            A[i * m:(i + 1) * m, jj * n:(jj + 1) * n] = blocks[d] if d >= 0 else blocks[ell - 1 - d]
    for Ek in E:
        assert np.linalg.norm(Ek) == pytest.approx(1.0, abs=1e-15)
    eta = [int(np.count_nonzero(Ek)) for Ek in E]
    assert np.max(np.abs(oracle.struct_kron(E, [np.sqrt(e) * B for e, B in zip(eta, Bs)]) - A)) < 1e-14
    X = oracle.tensor_from_blockmat_E(A, E, m, n)
    assert np.max(np.abs(oracle.blockmat_from_tensor_E(X, E) - A)) < 1e-14


# ------------------------------------------------------------ t-SVDM
def _dct_known_rank(m, p, n3, k, seed):
    g = np.random.default_rng(seed)
    Xh = np.zeros((m, p, n3), order="F")
    sig = np.zeros((k, n3))
    for f in range(n3):
        Ua, _ = np.linalg.qr(g.standard_normal((m, k)))
        Va, _ = np.linalg.qr(g.standard_normal((p, k)))
        sig[:, f] = np.sort(g.uniform(0.5, 2.0, k))[::-1]
        Xh[:, :, f] = (Ua * sig[:, f]) @ Va.T
    # spatial tensor built with the library inverse DCT, not the oracle's matrix
    X = scipy.fft.idct(Xh, type=2, norm="ortho", axis=2)
    return np.asfortranarray(X), sig


def test_exact_rank_recovery_and_truncation_error():
    """Known M-rank k: truncation at k recovers X; truncation at k-1 discards
    exactly the k-th singular value of every face (Eckart-Young per face plus
    the isometry of the transform)."""
    m, p, n3, k = 9, 7, 8, 3
    X, sig = _dct_known_rank(m, p, n3, k, 21)
    M = oracle.dct2_matrix(n3)
    r = oracle.tsvdm(X, M, "fixed", k)
    assert np.max(np.abs(r["T"] - X)) < 1e-12
    r2 = oracle.tsvdm(X, M, "fixed", k - 1)
    err = np.linalg.norm(r2["T"] - X)
    assert err == pytest.approx(np.sqrt(np.sum(sig[k - 1, :] ** 2)), rel=1e-12)


@pytest.mark.parametrize("kind", ["dct", "dft"])
def test_truncation_error_equals_discarded_library_singular_values(kind):
    """||X - T||_F^2 = sum over faces of the discarded squared singular values,
    with the singular values taken from the library SVD of the library-
    transformed faces; and the same error at matrix level (Lemma lem:tenapprox)."""
    ell, q, m, n = 3, 2, 4, 6
    A = _rand((ell * m, q * n), 31)
    X = oracle.tensor_from_blockmat(A, ell, q, m, n)
    M = oracle.dct2_matrix(n) if kind == "dct" else oracle.dft_matrix(n)
    r = oracle.tsvdm(X, M, "fixed", 2)
    Xh_lib = scipy.fft.dct(X, type=2, norm="ortho", axis=2) if kind == "dct" else \
        np.fft.fft(X, axis=2, norm="ortho")
    tail = 0.0
    for f in range(n):
        s = np.linalg.svd(Xh_lib[:, :, f], compute_uv=False)
        tail += np.sum(s[2:] ** 2)
    err_t = np.linalg.norm(X - r["T"])
    assert err_t == pytest.approx(np.sqrt(tail), rel=1e-11)
    Ahat = oracle.blockmat_from_tensor(r["T"], ell, q)
    assert np.linalg.norm(A - Ahat) == pytest.approx(err_t, rel=1e-12)
    if kind == "dft":
        assert np.isrealobj(r["T"])


def test_energy_rule_meets_tolerance_and_is_minimal():
    m, p, n3 = 8, 10, 4
    X = _rand((m, p, n3), 41)
    M = oracle.dct2_matrix(n3)
    tau = 0.3
    r = oracle.tsvdm(X, M, "energy", 0, tau)
    Xh = scipy.fft.dct(X, type=2, norm="ortho", axis=2)
    for f in range(n3):
        s = np.linalg.svd(Xh[:, :, f], compute_uv=False)
        fro2 = np.sum(Xh[:, :, f] ** 2)
        kf = r["ranks"][f]
        assert np.sum(s[kf:] ** 2) <= tau ** 2 * fro2
        if kf > 0:
            assert np.sum(s[kf - 1:] ** 2) > tau ** 2 * fro2


def test_identity_transform_is_facewise_svd():
    """M = I: the t-SVDM is the truncated SVD of each frontal slice."""
    X = _rand((6, 5, 3), 51)
    r = oracle.tsvdm(X, np.eye(3), "fixed", 2)
    for t in range(3):
        U, s, Vt = np.linalg.svd(X[:, :, t])
        assert np.max(np.abs(r["T"][:, :, t] - (U[:, :2] * s[:2]) @ Vt[:2])) < 1e-13


def test_single_face_is_plain_truncated_svd():
    X = _rand((7, 9, 1), 52)
    r = oracle.tsvdm(X, oracle.dct2_matrix(1), "fixed", 3)
    U, s, Vt = np.linalg.svd(X[:, :, 0])
    assert np.max(np.abs(r["T"][:, :, 0] - (U[:, :3] * s[:3]) @ Vt[:3])) < 1e-13


def test_mprod_dft_equals_block_circulant_brute_force():
    """With the unitary DFT as M, A *_M B = n^{-1/2} fold(bcirc(A) unfold(B)),
    bcirc written out by its definition (block (i, j) = A_{(i-j) mod n})."""
    m, k, p, n = 3, 4, 2, 5
    A = _rand((m, k, n), 61)
    B = _rand((k, p, n), 62)
    bc = np.zeros((m * n, k * n))
    for i in range(n):
        for j in range(n):
            bc[i * m:(i + 1) * m, j * k:(j + 1) * k] = A[:, :, (i - j) % n]
    ub = np.concatenate([B[:, :, t] for t in range(n)], axis=0)
    cb = bc @ ub
    ref = np.stack([cb[t * m:(t + 1) * m] for t in range(n)], axis=2) / np.sqrt(n)
    got = oracle.mprod(A, B, oracle.dft_matrix(n))
    assert np.max(np.abs(got - ref)) < 1e-13


def test_mprod_golden_n2():
    a, b, c = _load("tprod_n2.txt")
    got = oracle.mprod(a.reshape(1, 1, 2), b.reshape(1, 1, 2), oracle.dft_matrix(2))
    assert np.max(np.abs(got.ravel() - c / np.sqrt(2))) < 1e-14


def test_tsvdm_factorisation_under_mprod():
    """X = U *_M S *_M V^H from the full facewise SVD (no truncation)."""
    X = _rand((4, 3, 6), 71)
    M = oracle.dct2_matrix(6)
    Xh = oracle.mode3(X, M)
    U, s, V, _ = oracle.svd_faces(Xh)
    S = np.zeros((3, 3, 6))
    for f in range(6):
        S[:, :, f] = np.diag(s[:, f])
    Ut = oracle.inverse_mode3(U, M)
    St = oracle.inverse_mode3(S, M)
    Vt = oracle.inverse_mode3(V, M)
    Y = oracle.mprod(oracle.mprod(Ut, St, M), oracle.ttranspose(Vt, M), M)
    assert np.max(np.abs(Y - X)) < 1e-13


def test_kronecker_sum_workload_has_rank_terms_faces():
    """A = sum_{i<=4} B_i kron C_i maps to a tensor whose transform-domain
    faces have rank <= 4 (face f is sum_i (C_i M^T)[:, f] vec(B_i)^T, Sec. 2.2
    property 1); truncation to rank 4 recovers A to the noise level."""
    w = synth.kronecker_sum_matrix(terms=4, size=8, noise=1e-8)
    X = oracle.tensor_from_blockmat(w["A"], w["ell"], w["q"], w["m"], w["n"])
    M = oracle.dct2_matrix(w["n"])
    r = oracle.tsvdm(X, M, "fixed", 4)
    rel = np.linalg.norm(w["A"] - oracle.blockmat_from_tensor(r["T"], w["ell"], w["q"])) / \
        np.linalg.norm(w["A"])
    assert rel < 1e-8          # the noise has relative size 1e-8
    assert rel > 1e-10         # ... and most of it is discarded
    assert np.all(r["s"][4, :] < 1e-7 * r["s"][0, :])


def test_kronecker_apply_identity():
    """vec(C X B^T) = (B kron C) vec(X) (Sec. 2.2 property 1): the dense apply
    of a Kronecker-sum matrix rebuilt through T_E / M_E."""
    g = np.random.default_rng(81)
    B = g.standard_normal((3, 4, 4))
    C = g.standard_normal((3, 5, 5))
    A = synth.kron_sum(B, C)
    X = oracle.tensor_from_blockmat(A, 4, 4, 5, 5)
    Ahat = oracle.blockmat_from_tensor(X, 4, 4)
    Xr = g.standard_normal((5, 4))
    y = oracle.dense_apply(Ahat, Xr.reshape(-1, order="F"))
    ref = sum(C[i] @ Xr @ B[i].T for i in range(3)).reshape(-1, order="F")
    assert np.max(np.abs(y - ref)) < 1e-12


# ------------------------------------------------------------ randomized
def test_cholqr2_orthogonal_and_exact():
    Y = _rand((200, 12), 91)
    Q, R = oracle.cholqr2(Y)
    assert np.max(np.abs(Q.T @ Q - np.eye(12))) < 1e-14
    assert np.max(np.abs(Q @ R - Y)) < 1e-13 * np.linalg.norm(Y)
    assert np.allclose(R, np.triu(R))


def test_shifted_cholqr3_survives_ill_conditioning():
    """cond(Y) ~ 1e11: plain Cholesky-QR loses orthogonality, the shifted
    variant returns an orthonormal basis of the same range."""
    g = np.random.default_rng(92)
    Qa, _ = np.linalg.qr(g.standard_normal((300, 10)))
    Qb, _ = np.linalg.qr(g.standard_normal((10, 10)))
    Y = (Qa * np.logspace(0, -11, 10)) @ Qb
    Q, R = oracle.shifted_cholqr3(Y)
    assert np.max(np.abs(Q.T @ Q - np.eye(10))) < 1e-13
    assert np.max(np.abs(Q @ R - Y)) < 1e-13


def test_randomized_reference_reproduces_exact_rank_truncation():
    """Exact M-rank k input with ell > k: the range finder captures the range
    exactly, so the randomized result equals the deterministic truncation."""
    m, p, n3, k = 40, 30, 4, 5
    X, _ = _dct_known_rank(m, p, n3, k, 93)
    M = oracle.dct2_matrix(n3)
    Xh = oracle.mode3(X, M)
    Omega = _rand((p, k + 4), 94)
    rr = oracle.randomized_tsvdm_faces(Xh, Omega, k, power_iters=1)
    det = oracle.tsvdm_truncate_faces(Xh, "fixed", k)
    assert np.max(np.abs(rr["That"] - det["That"])) < 1e-11
    assert np.all(rr["cert"] < 1e-11)
    # truncating below the rank: certificate = discarded singular value
    rr2 = oracle.randomized_tsvdm_faces(Xh, Omega, k - 1, power_iters=1)
    assert np.allclose(rr2["cert"], det["s"][k - 1, :], rtol=1e-9)


def test_hermitian_half_faces_conjugate():
    """Faces f and n3 - f of the unitary DFT of a real tensor are conjugate,
    so they share singular values and rank."""
    X = _rand((4, 5, 7), 95)
    Xh = oracle.mode3(X, oracle.dft_matrix(7))
    for f in range(1, 7):
        assert np.max(np.abs(Xh[:, :, f] - np.conj(Xh[:, :, 7 - f]))) < 1e-14


# ------------------------------------------------------------------ Kronecker-sum faces
def test_kron_sum_faces_match_the_map_and_transform():
    """Closed form of the transform-domain faces of T_E[sum_r B_r kron C_r]
    against the definition: form A, map it with T_E (generic blocking, Sec. 3)
    and multiply every tube by M; every face has rank <= r."""
    g = np.random.default_rng(11)
    r, ell, m = 3, 4, 6
    B = g.standard_normal((r, ell, ell))
    C = g.standard_normal((r, m, m))
    A = sum(np.kron(B[i], C[i]) for i in range(r))
    M = oracle.dct2_matrix(m)
    Xh = oracle.mode3(oracle.tensor_from_blockmat(A, ell, ell, m, m), M)
    faces = [0, 2, 5]
    F = oracle.kron_sum_faces(B, C, M, faces)
    for i, f in enumerate(faces):
        np.testing.assert_allclose(F[:, :, i], Xh[:, :, f], atol=1e-12 * np.abs(Xh).max())
        assert np.linalg.matrix_rank(F[:, :, i], tol=1e-10 * np.linalg.norm(F[:, :, i])) <= r


# ------------------------------------------------------------ randomized energy rule
def _faces_with_spectra(m, p, spectra, seed):
    """Faces U_f diag(s_f) V_f^T with U_f, V_f the Q factors (numpy QR) of
    Gaussian matrices, so the singular values of face f are exactly s_f."""
    g = np.random.default_rng(seed)
    Xh = np.zeros((m, p, len(spectra)), order="F")
    for f, s in enumerate(spectra):
        Ua, _ = np.linalg.qr(g.standard_normal((m, len(s))))
        Va, _ = np.linalg.qr(g.standard_normal((p, len(s))))
        Xh[:, :, f] = (Ua * s) @ Va.T
    return Xh


def _geometric_crossing(rho, tau, r):
    """For s_j = 10^(-rho j), j = 1..r (q = 10^(-2 rho)): the discarded energy
    after k terms is sum_{j=k+1..r} q^j = q (q^k - q^r) / (1 - q) and the total
    q (1 - q^r) / (1 - q), so the energy rule holds iff
    q^k <= tau^2 + (1 - tau^2) q^r, i.e. k >= x = log(tau^2 + (1 - tau^2) q^r) / log q.
    Returns (ceil(x), x): the crossing rank in closed form, and x itself (its
    distance from the integers is the margin of the rank decision)."""
    q = 10.0 ** (-2.0 * rho)
    x = np.log(tau ** 2 + (1.0 - tau ** 2) * q ** r) / np.log(q)
    return int(np.ceil(x)), x


def test_randomized_energy_rule_exact_rank_closed_form():
    """Faces of exact rank 12 <= the sketch width 16, geometric spectra: the
    randomized reference (same Omega for every face, one power iteration)
    captures the range exactly, so its energy rule must return the
    closed-form crossing rank of each spectrum, and its certificate the
    discarded singular values (Eckart-Young); the margin of every decision is
    at least a fifth of a rank step (x at least 0.2 from an integer)."""
    m, p, r, ell, tau = 60, 48, 12, 16, 1e-3
    rhos = [0.25, 0.35, 0.45, 0.7, 0.9, 1.3]
    spectra = [10.0 ** (-rho * np.arange(1, r + 1)) for rho in rhos]
    want = []
    for rho in rhos:
        k, x = _geometric_crossing(rho, tau, r)
        assert min(x - np.floor(x), np.ceil(x) - x) >= 0.2 or k == r
        want.append(min(k, r))
    assert len(set(want)) >= 5
    Xh = _faces_with_spectra(m, p, spectra, 301)
    Omega = _rand((p, ell), 302)
    rr = oracle.randomized_tsvdm_faces(Xh, Omega, ell, power_iters=1, mode="energy", tau=tau)
    assert list(rr["ranks"]) == want
    for f, s in enumerate(spectra):
        tail = np.sqrt(np.sum(s[want[f]:] ** 2))
        assert rr["cert"][f] == pytest.approx(tail, rel=1e-6, abs=1e-13)
        assert rr["cert"][f] <= tau * np.linalg.norm(s)
    # a rank cap below the crossing rank returns the cap
    rc = oracle.randomized_tsvdm_faces(Xh, Omega, 4, power_iters=1, mode="energy", tau=tau)
    assert list(rc["ranks"]) == [min(w, 4) for w in want]


@pytest.mark.parametrize("tau", [2e-3, 5e-4, 2e-4])
def test_randomized_energy_rule_rank_beyond_sketch(tau):
    """Rank 40 > sketch width 20 with s_j = 10^(-j/4): the discarded energy
    includes the 20 directions the sketch never sees, so a rule that forgot
    them, or an off-by-one in the tail, returns another rank than the closed
    form; with one power iteration the leading Ritz values are accurate to
    far below the decision margins (checked here to be at least 15% of the
    threshold)."""
    m, p, r, ell, cap, rho = 70, 64, 40, 20, 16, 0.25
    k, x = _geometric_crossing(rho, tau, r)
    assert min(x - np.floor(x), np.ceil(x) - x) >= 0.15 and k <= cap
    s = 10.0 ** (-rho * np.arange(1, r + 1))
    Xh = _faces_with_spectra(m, p, [s, s], 311)
    Omega = _rand((p, ell), 312)
    rr = oracle.randomized_tsvdm_faces(Xh, Omega, cap, power_iters=1, mode="energy", tau=tau)
    assert list(rr["ranks"]) == [k, k]
    tail = np.sqrt(np.sum(s[k:] ** 2))
    np.testing.assert_allclose(rr["cert"], tail, rtol=1e-3)


def test_geometric_crossing_matches_a_direct_count():
    """The closed form used above against counting the tail term by term."""
    for rho in (0.1, 0.25, 0.4, 0.7):
        for tau in (1e-2, 3e-3, 1e-4):
            s2 = 10.0 ** (-2 * rho * np.arange(1, 33))
            k, x = _geometric_crossing(rho, tau, 32)
            if min(x - np.floor(x), np.ceil(x) - x) < 1e-6:
                continue
            ks = [kk for kk in range(33) if s2[kk:].sum() <= tau ** 2 * s2.sum()]
            assert ks[0] == k


# ------------------------------------------------------------ factors -> tensor
@pytest.mark.parametrize("n", [7, 8])
def test_hermitian_expansion_and_reconstruction_from_library_svd(n):
    """Half of the DFT faces of a real tensor (numpy FFT), their thin SVD by
    numpy, expanded to all n faces by conjugation and mapped back by
    approx_from_factors: with every triplet kept the real input returns and
    the imaginary part vanishes (a missing conjugation leaves it non-zero);
    truncated to 2 triplets the error equals the discarded singular values of
    all n library faces (Eckart-Young per face, isometry of the unitary DFT)."""
    m, p = 5, 6
    X = _rand((m, p, n), 321)
    Xh = np.fft.fft(X, axis=2, norm="ortho")
    half = n // 2 + 1
    r = min(m, p)
    U = np.zeros((m, r, half), dtype=complex, order="F")
    V = np.zeros((p, r, half), dtype=complex, order="F")
    S = np.zeros((r, half), order="F")
    for f in range(half):
        u, s, vh = np.linalg.svd(Xh[:, :, f], full_matrices=False)
        U[:, :, f], S[:, f], V[:, :, f] = u, s, vh.conj().T
    M = oracle.dft_matrix(n)
    Uf, Sf, Vf, Rf = oracle.expand_hermitian(U, S, V, np.full(half, r), n)
    T = oracle.approx_from_factors(Uf, Sf, Vf, Rf, M)
    assert np.max(np.abs(np.imag(T))) < 1e-13
    assert np.max(np.abs(np.real(T) - X)) < 1e-13
    Uf, Sf, Vf, Rf = oracle.expand_hermitian(U, S, V, np.full(half, 2), n)
    T2 = oracle.approx_from_factors(Uf, Sf, Vf, Rf, M)
    assert np.max(np.abs(np.imag(T2))) < 1e-13
    tail = sum(np.sum(np.linalg.svd(Xh[:, :, f], compute_uv=False)[2:] ** 2) for f in range(n))
    assert np.linalg.norm(np.real(T2) - X) == pytest.approx(np.sqrt(tail), rel=1e-12)


def test_approx_from_factors_dct_full_rank_returns_input():
    """DCT-II: library DCT of the tensor, numpy SVD of every face, all
    triplets kept, then approx_from_factors returns the input."""
    m, p, n = 6, 4, 5
    X = _rand((m, p, n), 331)
    Xh = scipy.fft.dct(X, type=2, norm="ortho", axis=2)
    U = np.zeros((m, 4, n), order="F")
    V = np.zeros((p, 4, n), order="F")
    S = np.zeros((4, n), order="F")
    for f in range(n):
        u, s, vh = np.linalg.svd(Xh[:, :, f], full_matrices=False)
        U[:, :, f], S[:, f], V[:, :, f] = u, s, vh.T
    T = oracle.approx_from_factors(U, S, V, np.full(n, 4), oracle.dct2_matrix(n))
    assert np.max(np.abs(T - X)) < 1e-13


# ------------------------------------------------------------ randomized, complex faces
def _complex_faces_with_spectra(m, p, spectra, seed):
    """Complex faces U_f diag(s_f) V_f^H with U_f, V_f the Q factors (numpy QR)
    of complex Gaussian matrices: the singular values of face f are exactly
    s_f, and the face is not the complexification of a real one."""
    g = np.random.default_rng(seed)
    Xh = np.zeros((m, p, len(spectra)), dtype=np.complex128, order="F")
    for f, s in enumerate(spectra):
        r = len(s)
        Ua, _ = np.linalg.qr(g.standard_normal((m, r)) + 1j * g.standard_normal((m, r)))
        Va, _ = np.linalg.qr(g.standard_normal((p, r)) + 1j * g.standard_normal((p, r)))
        Xh[:, :, f] = (Ua * s) @ np.conj(Va).T
    return Xh


@pytest.mark.parametrize("shape", [(50, 36), (30, 44)])
def test_randomized_complex_faces_exact_rank_and_eckart_young(shape):
    """Complex faces of exact rank 9 with a real Gaussian Omega of width 14:
    the range finder captures the range exactly (a real test matrix spans the
    complex range of a generic complex face), so truncation at 9 returns the
    face, the returned singular values are the constructed ones, and
    truncation at 6 leaves the discarded singular values as the error
    (Eckart-Young).  Dropping the conjugate of the adjoint anywhere in the
    range finder or the reconstruction fails all three."""
    m, p = shape
    r = 9
    spectra = [np.linspace(3.0, 0.5, r), 10.0 ** (-0.3 * np.arange(r))]
    Xh = _complex_faces_with_spectra(m, p, spectra, 331)
    Omega = _rand((p, r + 5), 332)
    rr = oracle.randomized_tsvdm_faces(Xh, Omega, r, power_iters=1)
    assert np.max(np.abs(rr["That"] - Xh)) < 1e-11 * np.abs(Xh).max()
    assert np.all(rr["cert"] < 1e-11)
    for f, s in enumerate(spectra):
        np.testing.assert_allclose(rr["s"][:r, f], s, rtol=1e-12)
        U, V = rr["U"][:, :r, f], rr["V"][:, :r, f]
        assert np.max(np.abs(np.conj(U).T @ U - np.eye(r))) < 1e-12
        assert np.max(np.abs(np.conj(V).T @ V - np.eye(r))) < 1e-12
    rr6 = oracle.randomized_tsvdm_faces(Xh, Omega, 6, power_iters=0)
    for f, s in enumerate(spectra):
        assert rr6["cert"][f] == pytest.approx(np.sqrt(np.sum(s[6:] ** 2)), rel=1e-9)


def test_randomized_complex_energy_rule_closed_form():
    """The energy rule on complex faces of exact rank 12 (sketch width 16):
    each rank is the closed-form crossing of its geometric spectrum, as for
    real faces; the phases of the singular vectors do not enter."""
    m, p, r, ell, tau = 60, 48, 12, 16, 1e-3
    rhos = [0.25, 0.35, 0.45, 0.7, 0.9]
    spectra = [10.0 ** (-rho * np.arange(1, r + 1)) for rho in rhos]
    want = []
    for rho in rhos:
        k, x = _geometric_crossing(rho, tau, r)
        assert min(x - np.floor(x), np.ceil(x) - x) >= 0.2 or k == r
        want.append(min(k, r))
    Xh = _complex_faces_with_spectra(m, p, spectra, 333)
    Omega = _rand((p, ell), 334)
    rr = oracle.randomized_tsvdm_faces(Xh, Omega, ell, power_iters=1, mode="energy", tau=tau)
    assert list(rr["ranks"]) == want
    for f, s in enumerate(spectra):
        assert rr["cert"][f] == pytest.approx(np.sqrt(np.sum(s[want[f]:] ** 2)), rel=1e-6, abs=1e-13)


def test_randomized_dft_half_spectrum_error_identity():
    """Randomized truncation of the stored half spectrum of a real tensor's
    unitary DFT, expanded to all faces by conjugation and transformed back:
    the result is real and its error equals sqrt(sum_f w_f cert_f^2) with
    w_f = 2 for the faces whose conjugate is not stored (unitarity of M and
    Lemma lem:tenapprox)."""
    m, p, n3, k = 24, 20, 6, 5
    X = _rand((m, p, n3), 335)
    M = oracle.dft_matrix(n3)
    Xh = oracle.mode3(X, M)
    half = n3 // 2 + 1
    Omega = _rand((p, k + 4), 336)
    rr = oracle.randomized_tsvdm_faces(np.asfortranarray(Xh[:, :, :half]), Omega, k, power_iters=1)
    U, s, V, ranks = oracle.expand_hermitian(rr["U"], rr["s"], rr["V"], rr["ranks"], n3)
    T = oracle.approx_from_factors(U, s, V, ranks, M)
    assert np.max(np.abs(np.imag(T))) < 1e-12
    w = np.array([1.0 if f in (0, n3 // 2) else 2.0 for f in range(half)])
    err = np.linalg.norm((X - np.real(T)).ravel())
    assert err == pytest.approx(np.sqrt(np.sum(w * rr["cert"] ** 2)), rel=1e-10)


def test_randomized_complex_power_iteration_accuracy():
    """Complex faces of rank 40 with s_j = 10^(-j/4) and a sketch of width 20:
    one power iteration makes the leading ten Ritz values exact to ~1e-15
    relative (the gap to s_21 enters to the sixth power, 10^(-16.5) for
    j = 10), while a sketch without a correct power step is off by ~1e-5
    (second power).  So the returned singular values pin the adjoint step
    (the conjugate transpose) of the complex power iteration."""
    m, p, r, ell = 70, 64, 40, 20
    s = 10.0 ** (-0.25 * np.arange(1, r + 1))
    Xh = _complex_faces_with_spectra(m, p, [s, s], 337)
    Omega = _rand((p, ell), 338)
    rr = oracle.randomized_tsvdm_faces(Xh, Omega, ell, power_iters=1)
    for f in range(2):
        np.testing.assert_allclose(rr["s"][:10, f], s[:10], rtol=1e-9)
    r0 = oracle.randomized_tsvdm_faces(Xh, Omega, ell, power_iters=0)
    assert np.max(np.abs(r0["s"][:10, 0] / s[:10] - 1.0)) > 1e-8  # the power step matters here
