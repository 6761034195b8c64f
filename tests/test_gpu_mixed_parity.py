"""GPU parity of the mixed-precision truncation against the oracle at the
headline shape (512 x 512 faces, k = 32, ell = 40) and of its energy-rule
ranks, bit for bit, against the oracle's randomized reference with the same
Gaussian test matrix."""
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
    return dict(U=from_dev(F.U, (m, k, nf)).astype(np.float64), S=from_dev(F.S, (k, nf)),
                V=from_dev(F.V, (p, k, nf)).astype(np.float64), ranks=from_dev(F.ranks, (nf,)),
                cert=from_dev(F.cert, (nf,)), fro=from_dev(F.fro, (nf,)), info=from_dev(F.info, (nf,)))


def _decaying_faces(m, p, rhos, r, salt):
    """Transform-domain faces U_f diag(10^(-rho_f j)) V_f^T, j = 1..r, rounded to
    FP32 (input assembly); also the designed singular values."""
    g = synth.rng(1, salt)
    nf = len(rhos)
    U = synth.orthonormal_stack(g, m, r, nf)
    V = synth.orthonormal_stack(g, p, r, nf)
    sig = np.array([10.0 ** (-rho * np.arange(1, r + 1)) for rho in rhos])  # (nf, r)
    Xh = np.zeros((m, p, nf), order="F")
    for f in range(nf):
        Xh[:, :, f] = (U[:, :, f] * sig[f]) @ V[:, :, f].T
    return Xh.astype(np.float32), sig


def _energy_margin_ok(sig, tau, cap, rel_margin=1e-2):
    """Every face's discarded energy at every k <= cap stays rel_margin * tau^2
    ||X_f||^2 away from the threshold (so rounding cannot move the rank)."""
    for s in sig:
        fro2 = np.sum(s * s)
        for k in range(min(cap, len(s)) + 1):
            tail = np.sum(s[k:] ** 2)
            if abs(tail - tau * tau * fro2) < rel_margin * tau * tau * fro2:
                return False
    return True


@pytest.mark.parametrize("shape", [(160, 144), (130, 96)])
def test_mixed_energy_ranks_equal_oracle_randomized(shape):
    """ENERGY rule: the mixed path's per-face ranks equal, bit for bit, the
    ranks of the oracle's FP64 randomized truncation with the same Omega, and
    the exact energy ranks of the oracle's facewise SVD, on inputs whose
    discarded energy stays 1e-2 tau^2 ||X_f||^2 clear of the threshold.
    (160, 144): 16-byte load path; (130, 96): m not a multiple of 4."""
    m, p = shape
    rhos = [1 / 16, 1 / 12, 1 / 8, 1 / 6, 1 / 4, 1 / 3, 1 / 2, 0.7, 0.09, 0.11, 0.15, 0.2]
    r, cap, os_ = 30, 32, 8
    Xh32, sig = _decaying_faces(m, p, rhos, r, salt=11 + m)
    taus = [1e-2, 5e-3, 3e-3, 1e-3, 5e-4, 2e-4]
    taus = [t for t in taus if _energy_margin_ok(sig, t, cap)]
    assert len(taus) >= 2
    g = synth.rng(1, 500 + m)
    Omega = synth.gaussian(g, (p, cap + os_)).astype(np.float32)
    nf = len(rhos)
    Xh64 = Xh32.astype(np.float64)
    xd, od = to_dev(Xh32), to_dev(Omega)
    for tau in taus:
        tr = api.Truncator(m, p, nf, torch.float32, rank_mode=C.RANK_ENERGY, k=cap, tau=tau,
                           precision=C.PREC_MIXED, oversample=os_, power_iters=1, omega=od)
        got = _factors(tr(xd), nf)
        rnd = oracle.randomized_tsvdm_faces(Xh64, Omega.astype(np.float64), cap, 1, mode="energy",
                                            tau=tau)
        exact = oracle.tsvdm_truncate_faces(Xh64, "energy", cap, tau)
        assert np.array_equal(got["ranks"], rnd["ranks"]), (tau, got["ranks"], rnd["ranks"])
        assert np.array_equal(got["ranks"], exact["ranks"]), (tau, got["ranks"], exact["ranks"])
        assert np.all(got["info"] == 0)
        That = reconstruct(got["U"], got["S"], got["V"], got["ranks"])
        assert relerr(That, rnd["That"]) < 1e-4
        true = np.array([np.linalg.norm(Xh64[:, :, f] - That[:, :, f]) for f in range(nf)])
        assert np.all(true <= tau * got["fro"])
        # the certificate is the error of the returned factors
        np.testing.assert_allclose(got["cert"], true, rtol=1e-9, atol=1e-14 * np.max(got["fro"]))


def test_energy_cap_miss_sets_info4():
    """ENERGY with a cap below the rank the tolerance needs: the cap is
    returned and info = 4, in the mixed and in the plain FP64 path; faces that
    meet tau within the cap keep info = 0 (the oracle's ranks)."""
    m, p = 96, 80
    rhos = [1 / 16, 1 / 2, 1 / 20, 0.8]
    Xh32, sig = _decaying_faces(m, p, rhos, 24, salt=77)
    nf, cap, tau = len(rhos), 8, 1e-3
    Xh64 = Xh32.astype(np.float64)
    exact = oracle.tsvdm_truncate_faces(Xh64, "energy", min(m, p), tau)
    need = exact["ranks"]
    assert np.any(need > cap) and np.any(need <= cap)
    g = synth.rng(1, 78)
    Omega = synth.gaussian(g, (p, cap + 8)).astype(np.float32)
    tr = api.Truncator(m, p, nf, torch.float32, rank_mode=C.RANK_ENERGY, k=cap, tau=tau,
                       precision=C.PREC_MIXED, oversample=8, power_iters=1, omega=to_dev(Omega))
    got = _factors(tr(to_dev(Xh32)), nf)
    want = np.minimum(need, cap)
    assert np.array_equal(got["ranks"], want)
    assert np.array_equal(got["info"], np.where(need > cap, 4, 0))
    trp = api.Truncator(m, p, nf, torch.float64, rank_mode=C.RANK_ENERGY, k=cap, tau=tau,
                        precision=C.PREC_F64, kmax=cap)
    gp = _factors(trp(to_dev(Xh64)), nf)
    assert np.array_equal(gp["ranks"], want)
    assert np.array_equal(gp["info"], np.where(need > cap, 4, 0))


def test_mixed_headline_shape_512_k32_ell40():
    """The headline configuration on a 16-face slab: 512 x 512 faces of M-rank
    32 with sigma_j = 10^(-j/8), built in the transform domain, mapped back
    with the oracle's explicit inverse DCT-II and stored FP32; on the GPU the
    forward transform and the mixed truncation with k = 32, oversampling 8
    (ell = 40, padded width 48, eight 64-row blocks per face), one power
    iteration, FIXED rank.  Compared element by element with the oracle's
    exact facewise truncation (sampled faces) and with its FP64 randomized
    truncation with the same Omega (all faces), at 1e-4."""
    m, p, n3, k, os_ = 512, 512, 16, 32, 8
    fac = synth.known_rank_factors(m=m, p=p, n3=n3, k=k, oversample=os_, salt=31)
    Xh = np.zeros((m, p, n3), order="F")
    for f in range(n3):
        Xh[:, :, f] = (fac["U"][:, :, f] * fac["sigma"]) @ fac["V"][:, :, f].T
    M = oracle.dct2_matrix(n3)
    X = oracle.inverse_mode3(Xh, M).astype(np.float32)
    Omega = fac["Omega"].astype(np.float32)
    xh = api.transform(to_dev(X), m, p, n3, C.M_DCT2, +1)
    tr = api.Truncator(m, p, n3, torch.float32, k=k, precision=C.PREC_MIXED, oversample=os_,
                       power_iters=1, omega=to_dev(Omega))
    got = _factors(tr(xh), n3)
    assert np.all(got["ranks"] == k) and np.all(got["info"] == 0)
    Xh64 = oracle.mode3(X.astype(np.float64), M)
    That = reconstruct(got["U"], got["S"], got["V"], got["ranks"])
    rnd = oracle.randomized_tsvdm_faces(Xh64, Omega.astype(np.float64), k, 1)
    assert np.array_equal(rnd["ranks"], got["ranks"])
    assert relerr(That, rnd["That"]) < 1e-4
    sample = [0, 7, 15]
    ex = oracle.tsvdm_truncate_faces(np.asfortranarray(Xh64[:, :, sample]), "fixed", k)
    assert relerr(That[:, :, sample], ex["That"]) < 1e-4
    # Weyl: |s_j(A) - s_j(B)| <= ||A - B||_2, so the singular values are compared
    # on the scale of ||Xhat_f||, not relative to each (small) s_j
    for i, f in enumerate(sample):
        np.testing.assert_allclose(got["S"][:k, f], ex["s"][:k, i], rtol=0, atol=1e-6 * got["fro"][f])
    np.testing.assert_allclose(got["fro"], np.sqrt(np.sum(Xh64 ** 2, axis=(0, 1))), rtol=1e-6)
    # the certificate is the error of the returned factors against the FP32
    # transform-domain tensor they were computed from, evaluated in FP64
    xg = from_dev(xh, (m, p, n3)).astype(np.float64)
    true = np.array([np.linalg.norm(xg[:, :, f] - That[:, :, f]) for f in range(n3)])
    np.testing.assert_allclose(got["cert"], true, rtol=1e-9, atol=1e-14 * np.max(got["fro"]))
    assert np.max(got["cert"] / got["fro"]) < 1e-5


@pytest.mark.parametrize("precision", [C.PREC_MIXED, C.PREC_F64])
def test_zero_and_nonfinite_faces(precision):
    """An all-zero face and a face holding a NaN, between ordinary faces, ENERGY
    rule: the zero face gets rank 0, ||X_f|| = 0, certificate 0 and zero
    factors (mixed path: info = 2, the range finder's Cholesky breaks down on
    a zero sketch; FP64 path: info = 0); the NaN face info = 3; the ordinary
    faces come out bit for bit as in a run without the degenerate faces."""
    m, p, cap, tau = 96, 80, 16, 1e-3
    Xh32, _ = _decaying_faces(m, p, [1 / 3, 1 / 2, 1 / 4, 0.4], 24, salt=91)
    nf = Xh32.shape[2]
    bad = Xh32.copy(order="F")
    bad[:, :, 1] = 0.0
    bad[5, 7, 2] = np.nan
    if precision == C.PREC_MIXED:
        dt, npdt, kw = torch.float32, np.float32, dict(oversample=8, power_iters=1)
        Omega = synth.gaussian(synth.rng(1, 92), (p, cap + 8)).astype(np.float32)
        kw["omega"] = to_dev(Omega)
    else:
        dt, npdt, kw = torch.float64, np.float64, dict(kmax=cap)
    tr = api.Truncator(m, p, nf, dt, rank_mode=C.RANK_ENERGY, k=cap, tau=tau, precision=precision, **kw)
    good = _factors(tr(to_dev(Xh32.astype(npdt))), nf)
    got = _factors(tr(to_dev(bad.astype(npdt))), nf)
    assert np.all(good["info"] == 0)
    for f in (0, 3):
        for key in ("U", "S", "V", "ranks", "cert", "fro", "info"):
            a, b = np.take(got[key], f, axis=-1), np.take(good[key], f, axis=-1)
            assert np.array_equal(a, b), (f, key)
    assert got["ranks"][1] == 0 and got["fro"][1] == 0.0 and got["cert"][1] == 0.0
    assert not np.any(got["U"][:, :, 1]) and not np.any(got["S"][:, 1]) and not np.any(got["V"][:, :, 1])
    assert got["info"][1] == (2 if precision == C.PREC_MIXED else 0)
    assert got["info"][2] == 3 and not np.isfinite(got["fro"][2])


def test_mixed_rows_over_several_qr_chunks():
    """m = 1100 rows: the Cholesky-QR passes over the sketch and the final
    basis take three chunks of 512 rows, the last one ragged (76 rows), with
    the second pass re-reading Q from memory; p = 300.  FIXED k = 20,
    oversampling 8, one power iteration: ranks and the truncation equal the
    oracle's FP64 randomized truncation with the same Omega, at 1e-4."""
    m, p, k, os_ = 1100, 300, 20, 8
    Xh32, _ = _decaying_faces(m, p, [1 / 10, 1 / 6, 1 / 4], 40, salt=93)
    nf = Xh32.shape[2]
    Omega = synth.gaussian(synth.rng(1, 94), (p, k + os_)).astype(np.float32)
    tr = api.Truncator(m, p, nf, torch.float32, k=k, precision=C.PREC_MIXED, oversample=os_, power_iters=1,
                       omega=to_dev(Omega))
    got = _factors(tr(to_dev(Xh32)), nf)
    assert np.all(got["ranks"] == k) and np.all(got["info"] == 0)
    Xh64 = Xh32.astype(np.float64)
    rnd = oracle.randomized_tsvdm_faces(Xh64, Omega.astype(np.float64), k, 1)
    That = reconstruct(got["U"], got["S"], got["V"], got["ranks"])
    assert relerr(That, rnd["That"]) < 1e-4
    # orthonormal columns of U to FP32 accuracy
    for f in range(nf):
        Uf = got["U"][:, :k, f]
        assert np.abs(Uf.T @ Uf - np.eye(k)).max() < 1e-5
    true = np.array([np.linalg.norm(Xh64[:, :, f] - That[:, :, f]) for f in range(nf)])
    np.testing.assert_allclose(got["cert"], true, rtol=1e-9, atol=1e-14 * np.max(got["fro"]))



def test_certificate_of_few_wide_faces_split_over_columns():
    """Two 130 x 9000 faces: 6 row blocks in all, so the certificate pass
    splits each face's columns over 32 ranges (a workgroup each) and sums
    the partials in order.  The certificate still equals the error of the
    returned factors against the faces (FP64 on the host), and the
    truncation agrees with the oracle's randomized one at 1e-4."""
    m, p, k, os_ = 130, 9000, 12, 8
    Xh32, _ = _decaying_faces(m, p, [1 / 4, 1 / 6], 40, salt=95)
    nf = Xh32.shape[2]
    Omega = synth.gaussian(synth.rng(1, 96), (p, k + os_)).astype(np.float32)
    tr = api.Truncator(m, p, nf, torch.float32, k=k, precision=C.PREC_MIXED, oversample=os_, power_iters=1,
                       omega=to_dev(Omega))
    got = _factors(tr(to_dev(Xh32)), nf)
    assert np.all(got["ranks"] == k) and np.all(got["info"] == 0)
    Xh64 = Xh32.astype(np.float64)
    That = reconstruct(got["U"], got["S"], got["V"], got["ranks"])
    true = np.array([np.linalg.norm(Xh64[:, :, f] - That[:, :, f]) for f in range(nf)])
    np.testing.assert_allclose(got["cert"], true, rtol=1e-9, atol=1e-14 * np.max(got["fro"]))
    rnd = oracle.randomized_tsvdm_faces(Xh64, Omega.astype(np.float64), k, 1)
    assert relerr(That, rnd["That"]) < 1e-4


def test_few_wide_faces_split_passes_with_vector_loads():
    """Three 128 x 6000 faces (m a multiple of 4: 16-byte loads): 6 row
    blocks in all, so the X W passes split every block's columns over
    workgroups (partial products summed by the reduction kernel), each face's
    blocks run on three XCDs, and the one-pass Cholesky-QR of the 6000-row Z
    spreads its chunks over workgroups.  The certificate equals the error of
    the returned factors and the truncation agrees with the oracle's
    randomized one (same Omega) at 1e-4."""
    m, p, k, os_ = 128, 6000, 10, 6
    Xh32, _ = _decaying_faces(m, p, [1 / 4, 1 / 5, 1 / 7], 40, salt=97)
    nf = Xh32.shape[2]
    Omega = synth.gaussian(synth.rng(1, 98), (p, k + os_)).astype(np.float32)
    tr = api.Truncator(m, p, nf, torch.float32, k=k, precision=C.PREC_MIXED, oversample=os_, power_iters=1,
                       omega=to_dev(Omega))
    got = _factors(tr(to_dev(Xh32)), nf)
    assert np.all(got["ranks"] == k) and np.all(got["info"] == 0)
    Xh64 = Xh32.astype(np.float64)
    np.testing.assert_allclose(got["fro"], [np.linalg.norm(Xh64[:, :, f]) for f in range(nf)], rtol=1e-6)
    That = reconstruct(got["U"], got["S"], got["V"], got["ranks"])
    true = np.array([np.linalg.norm(Xh64[:, :, f] - That[:, :, f]) for f in range(nf)])
    np.testing.assert_allclose(got["cert"], true, rtol=1e-9, atol=1e-14 * np.max(got["fro"]))
    rnd = oracle.randomized_tsvdm_faces(Xh64, Omega.astype(np.float64), k, 1)
    assert relerr(That, rnd["That"]) < 1e-4
