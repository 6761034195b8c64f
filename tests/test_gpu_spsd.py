"""GPU parity of the SPSD-preserving two-sided compression (Sec. 5.1) on a
synthetic space-time covariance (Sec. 6.2) against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import from_dev, relerr, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2105_01170_amd import api  # noqa: E402
from paper_2105_01170_amd import tsvdm as C  # noqa: E402


def _E_sym_toeplitz(T):
    E = []
    for k in range(T):
        Ek = np.zeros((T, T))
        for i in range(T):
            for j in range(T):
                if abs(i - j) == k:
                    Ek[i, j] = 1.0
        E.append(Ek / np.linalg.norm(Ek))
    return E


def _gpu_spsd(blocks, N, T, r, salt):
    """T_E from the distinct blocks (symmetric block-Toeplitz placement), U
    from the mixed-precision truncation of the mode-1 unfolding (X's memory
    read as one N x (T N) face), and the two-sided core."""
    pl = api.Placement.structure(C.PLACE_TOEPLITZ_SYM, T, T)
    assert pl.p == T
    b64 = to_dev(blocks)
    X64 = pl.tensor_from_blocks(b64, N, N)
    X32 = pl.tensor_from_blocks(to_dev(blocks, np.float32), N, N)
    omega = to_dev(synth.gaussian(synth.rng(9, 100 + salt), (T * N, r + 8)), np.float32)
    tr = api.Truncator(N, T * N, 1, torch.float32, k=r, precision=C.PREC_MIXED, oversample=8, power_iters=1,
                       omega=omega)
    F = tr(X32)
    U = F.U[:N * r]
    G = api.two_sided(X64, N, T, U, r)
    return pl, X64, U, G


def test_spsd_two_sided_against_oracle():
    N, T, r = 150, 10, 16
    blocks, _, _ = synth.spacetime_covariance(N, T, salt=1)
    pl, X64, U, G = _gpu_spsd(blocks, N, T, r, 1)
    Uh = from_dev(U, (N, r)).astype(np.float64)
    E = _E_sym_toeplitz(T)
    eta = [np.count_nonzero(Ek) for Ek in E]
    Cmat = oracle.struct_kron(E, [np.sqrt(e) * blocks[:, :, k] for k, e in enumerate(eta)])
    X = from_dev(X64, (N, T, N))
    np.testing.assert_allclose(X, oracle.tensor_from_blockmat_E(Cmat, E, N, N), rtol=1e-15, atol=0)
    Go, To = oracle.spsd_two_sided(X, Uh)
    np.testing.assert_allclose(from_dev(G, (r, T, r)), Go, rtol=1e-11, atol=1e-12 * np.abs(Go).max())
    Tg = api.two_sided_inverse(G, N, T, U, r)
    Chat = from_dev(pl.blockmat_from_tensor(Tg, N, N), (N * T, N * T))
    P = Uh @ Uh.T
    IP = np.kron(np.eye(T), P)
    assert relerr(Chat, IP @ Cmat @ IP) < 1e-11
    lam = np.linalg.eigvalsh((Chat + Chat.T) / 2)
    assert lam[0] > -1e-10 * lam[-1]  # positive semidefinite, as (I kron P) C (I kron P)
    # the trace metric of Sec. 6.2 against the oracle's own (exact SVD) factor
    tr_c = N * T
    rel_gpu = abs(tr_c - T * np.trace(Uh.T @ blocks[:, :, 0] @ Uh)) / tr_c
    Uo = oracle.spsd_factor(oracle.tensor_from_blockmat_E(Cmat, E, N, N), r)
    rel_o = abs(tr_c - T * np.trace(Uo.T @ blocks[:, :, 0] @ Uo)) / tr_c
    assert rel_gpu == pytest.approx(rel_o, rel=1e-2)
    # tr((I kron P) C (I kron P)) = T tr(U^T U U^T C_1 U): T tr(U^T C_1 U) when U
    # has orthonormal columns (here to the FP32 rounding of U)
    UtU = Uh.T @ Uh
    assert np.trace(Chat) == pytest.approx(T * np.trace(UtU @ Uh.T @ blocks[:, :, 0] @ Uh), rel=1e-11)
    assert np.trace(Chat) == pytest.approx(T * np.trace(Uh.T @ blocks[:, :, 0] @ Uh), rel=1e-6)
