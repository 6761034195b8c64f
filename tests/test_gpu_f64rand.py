"""GPU parity of the FP64 randomized truncation (PREC_F64_RAND: the mixed
path's range finder with every product in FP64) against the oracle's FP64
randomized truncation with the same Gaussian test matrix, at the 1e-10
relative tolerance of the FP64 path."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import from_dev, reconstruct, relerr, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2105_01170_amd import api  # noqa: E402
from paper_2105_01170_amd import tsvdm as C  # noqa: E402


def _factors(F, nf):
    m, p, k = F.m, F.p, F.kmax
    return dict(U=from_dev(F.U, (m, k, nf)), S=from_dev(F.S, (k, nf)), V=from_dev(F.V, (p, k, nf)),
                ranks=from_dev(F.ranks, (nf,)), cert=from_dev(F.cert, (nf,)), fro=from_dev(F.fro, (nf,)),
                info=from_dev(F.info, (nf,)))


def _faces(m, p, rhos, r, salt, noise=0.0):
    """Faces U_f diag(10^(-rho_f j)) V_f^T (j = 1..r) plus optional Gaussian
    noise of relative size `noise`, FP64."""
    g = synth.rng(5, salt)
    nf = len(rhos)
    U = synth.orthonormal_stack(g, m, r, nf)
    V = synth.orthonormal_stack(g, p, r, nf)
    Xh = np.zeros((m, p, nf), order="F")
    for f, rho in enumerate(rhos):
        Xh[:, :, f] = (U[:, :, f] * 10.0 ** (-rho * np.arange(1, r + 1))) @ V[:, :, f].T
        if noise:
            E = g.standard_normal((m, p))
            Xh[:, :, f] += noise * np.linalg.norm(Xh[:, :, f]) / np.linalg.norm(E) * E
    return Xh


def _run(Xh, k, os_, q, mode=C.RANK_FIXED, tau=0.0, certify=1, salt=0):
    m, p, nf = Xh.shape
    Omega = synth.gaussian(synth.rng(6, salt), (p, k + os_)).astype(np.float32)
    tr = api.Truncator(m, p, nf, torch.float64, rank_mode=mode, k=k, tau=tau, precision=C.PREC_F64_RAND,
                       oversample=os_, power_iters=q, certify=certify, omega=to_dev(Omega))
    got = _factors(tr(to_dev(Xh)), nf)
    return got, Omega.astype(np.float64)


@pytest.mark.parametrize("shape,k,os_,q", [((512, 512), 32, 8, 1), ((130, 96), 10, 4, 1), ((1100, 75), 20, 8, 1),
                                           ((96, 200), 50, 10, 0), ((64, 64), 3, 2, 1)])
def test_f64rand_fixed_matches_oracle_randomized(shape, k, os_, q):
    """FIXED rank: the truncation equals the oracle's FP64 randomized one with
    the same Omega to 1e-10 (relative Frobenius), singular values to 1e-12
    ||X_f||, U orthonormal to 1e-12, and the certificate is the error of the
    returned factors to 1e-9.  The faces decay slowly enough (sigma_j =
    10^(-rho j), rho <= 1/12) that the sketch's condition number stays below
    ~1e5, so two correct FP64 evaluations of the same randomized truncation
    agree to ~1e-11.  Shapes: the 512 x 512 headline faces (width 48), m not
    a multiple of 4 (width 16), 1100 rows (three 512-row Cholesky-QR chunks)
    with p = 75 (a ragged column block), width 64 without power iteration, a
    tiny sketch."""
    m, p = shape
    Xh = _faces(m, p, [1 / 12, 1 / 16, 1 / 20, 1 / 24, 1 / 32], min(m, p, 60), salt=m + p)
    got, Om = _run(Xh, k, os_, q, salt=k)
    nf = Xh.shape[2]
    rnd = oracle.randomized_tsvdm_faces(Xh, Om, k, q)
    assert np.array_equal(got["ranks"], rnd["ranks"]) and np.all(got["info"] == 0)
    That = reconstruct(got["U"], got["S"], got["V"], got["ranks"])
    assert relerr(That, rnd["That"]) < 1e-10
    for f in range(nf):
        fro = np.linalg.norm(Xh[:, :, f])
        np.testing.assert_allclose(got["S"][:k, f], rnd["s"][:k, f], rtol=0, atol=1e-12 * fro)
        Uf = got["U"][:, :k, f]
        assert np.abs(Uf.T @ Uf - np.eye(k)).max() < 1e-12
    true = np.array([np.linalg.norm(Xh[:, :, f] - That[:, :, f]) for f in range(nf)])
    np.testing.assert_allclose(got["cert"], true, rtol=1e-9, atol=1e-15 * np.max(got["fro"]))
    np.testing.assert_allclose(got["fro"], np.sqrt(np.sum(Xh ** 2, axis=(0, 1))), rtol=1e-14)


def test_f64rand_fast_decay_and_noise_floor():
    """Faces whose spectrum falls below a noise floor of 1e-7 ||X_f|| well
    before the rank (sigma_j = 10^(-j/4), 10^(-j/3)): no Cholesky breakdown,
    and the truncation is as good as the oracle's (the rank-32 truncation
    reaches into the noise, where the two differ by rounding, so the errors
    are compared, not the factors)."""
    m = p = 512
    k, os_ = 32, 8
    Xh = _faces(m, p, [1 / 4, 1 / 3, 1 / 2], 60, salt=17, noise=1e-7)
    got, Om = _run(Xh, k, os_, 1, salt=18)
    assert np.all(got["info"] == 0)
    rnd = oracle.randomized_tsvdm_faces(Xh, Om, k, 1)
    That = reconstruct(got["U"], got["S"], got["V"], got["ranks"])
    for f in range(Xh.shape[2]):
        err = np.linalg.norm(Xh[:, :, f] - That[:, :, f])
        assert err <= 1.01 * rnd["cert"][f]
        np.testing.assert_allclose(got["cert"][f], err, rtol=1e-9)


def test_f64rand_energy_ranks_equal_oracle():
    """ENERGY rule: the ranks equal, bit for bit, those of the oracle's FP64
    randomized truncation with the same Omega, on faces whose discarded energy
    stays clear of tau^2 ||X_f||^2 at every rank; without certify the
    certificate is the estimate sqrt(||X_f||^2 - sum_{j<=k} s_j^2), equal to
    the oracle's explicit error to the rounding of that difference."""
    m, p, k, os_, tau = 160, 144, 40, 8, 2e-6
    rhos = [1 / 16, 1 / 12, 1 / 8, 1 / 6, 1 / 4, 1 / 3, 1 / 2, 0.7]
    Xh = _faces(m, p, rhos, 48, salt=3)
    sig = [10.0 ** (-rho * np.arange(1, 49)) for rho in rhos]
    for s in sig:  # margin: no rank within 1e-2 of the threshold
        fro2 = np.sum(s * s)
        tails = np.array([np.sum(s[j:] ** 2) for j in range(len(s) + 1)])
        assert np.all(np.abs(tails - tau * tau * fro2) > 1e-2 * tau * tau * fro2)
    got, Om = _run(Xh, k, os_, 1, mode=C.RANK_ENERGY, tau=tau, certify=0, salt=7)
    rnd = oracle.randomized_tsvdm_faces(Xh, Om, k, 1, mode="energy", tau=tau)
    assert np.array_equal(got["ranks"], rnd["ranks"])
    assert np.all((got["info"] == 0) | ((got["info"] == 4) & (got["ranks"] == k)))
    # the estimate is a difference of squares: cert^2 ~ tau^2 ||X_f||^2 carries
    # rounding of ~1e-15 ||X_f||^2, i.e. ~1e-3 relative at tau = 2e-6
    np.testing.assert_allclose(got["cert"], rnd["cert"], rtol=1e-2)
    # the fast-decaying faces (rho up to 0.7) have sketches whose condition
    # number reaches 1/u, so two correct FP64 evaluations agree to ~1e-9 here
    # (1e-10 holds for the well-conditioned sketches of the FIXED test)
    That = reconstruct(got["U"], got["S"], got["V"], got["ranks"])
    assert relerr(That, rnd["That"]) < 2e-9


def test_f64rand_zero_and_nonfinite_faces():
    """A zero face gets rank 0, zero factors, certificate 0 and info 2 (the
    range finder's Cholesky breaks down); a face holding a NaN info 3; the
    other faces are unchanged, bit for bit."""
    m, p, k = 96, 80, 8
    Xh = _faces(m, p, [1 / 3, 1 / 2, 1 / 4, 0.4], 24, salt=9)
    good, _ = _run(Xh, k, 8, 1, mode=C.RANK_ENERGY, tau=1e-3, salt=1)
    bad = Xh.copy(order="F")
    bad[:, :, 1] = 0.0
    bad[5, 7, 2] = np.nan
    got, _ = _run(bad, k, 8, 1, mode=C.RANK_ENERGY, tau=1e-3, salt=1)
    for f in (0, 3):
        for key in ("U", "S", "V", "ranks", "cert", "fro", "info"):
            assert np.array_equal(np.take(got[key], f, axis=-1), np.take(good[key], f, axis=-1)), (f, key)
    assert got["ranks"][1] == 0 and got["cert"][1] == 0.0 and got["info"][1] == 2
    assert not np.any(got["U"][:, :, 1]) and not np.any(got["V"][:, :, 1])
    assert got["info"][2] == 3


def test_f64rand_headline_tensor_against_exact_truncation():
    """The headline construction on a 16-face slab (512 x 512 faces of M-rank 32,
    sigma_j = 10^(-j/8), DCT-II, FP64 throughout): the FP64 randomized
    truncation with k = 32, width 40, one power iteration recovers the exact
    rank-32 truncation of the oracle's facewise SVD to 1e-10."""
    m, p, n3, k, os_ = 512, 512, 16, 32, 8
    fac = synth.known_rank_factors(m=m, p=p, n3=n3, k=k, oversample=os_, salt=41)
    Xh = np.zeros((m, p, n3), order="F")
    for f in range(n3):
        Xh[:, :, f] = (fac["U"][:, :, f] * fac["sigma"]) @ fac["V"][:, :, f].T
    M = oracle.dct2_matrix(n3)
    X = oracle.inverse_mode3(Xh, M)
    xh = api.transform(to_dev(X), m, p, n3, C.M_DCT2, +1)
    tr = api.Truncator(m, p, n3, torch.float64, k=k, precision=C.PREC_F64_RAND, oversample=os_, power_iters=1,
                       omega=to_dev(fac["Omega"].astype(np.float32)))
    got = _factors(tr(xh), n3)
    assert np.all(got["ranks"] == k) and np.all(got["info"] == 0)
    That = reconstruct(got["U"], got["S"], got["V"], got["ranks"])
    sample = [0, 5, 15]
    ex = oracle.tsvdm_truncate_faces(np.asfortranarray(Xh[:, :, sample]), "fixed", k)
    assert relerr(That[:, :, sample], ex["That"]) < 1e-10
    assert np.max(got["cert"] / got["fro"]) < 1e-12


@pytest.mark.parametrize("mode", [C.RANK_FIXED, C.RANK_ENERGY])
def test_f64rand_two_face_groups_equal_separate_calls(mode):
    """40 FP64 faces of 512 x 840 (137.6 MB, past the 128 MiB from which the
    faces run in two groups, the second half on a side stream): every output
    equals, bit for bit, two separate calls on the first and last 20 faces
    (one group each)."""
    nf, m, p = 40, 512, 840
    assert 8 * m * p * nf >= 128 << 20 > 8 * m * p * (nf // 2)
    rhos = [0.05 + 0.01 * f for f in range(nf)]
    Xh = _faces(m, p, rhos, 40, salt=91, noise=1e-9)
    tau = 1e-3 if mode == C.RANK_ENERGY else 0.0
    got, _ = _run(Xh, 12, 8, 1, mode=mode, tau=tau, salt=92)
    half = nf // 2
    parts = [_run(np.asfortranarray(Xh[:, :, lo:lo + half]), 12, 8, 1, mode=mode, tau=tau, salt=92)[0]
             for lo in (0, half)]
    for key in ("U", "S", "V", "ranks", "cert", "fro", "info"):
        joined = np.concatenate([parts[0][key], parts[1][key]], axis=-1)
        assert np.array_equal(got[key], joined), key
    if mode == C.RANK_ENERGY:
        assert len(np.unique(got["ranks"])) > 1
