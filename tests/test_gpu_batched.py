"""GPU parity of the batched truncation (tsvdm_batched_*) against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import from_dev, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2105_01170_amd import api  # noqa: E402
from paper_2105_01170_amd import tsvdm as C  # noqa: E402

TAU = 1e-4


def _kron_tensors(count, lo, hi, rmin, rmax, noise, salt):
    """(Xhat in FP32 as float64, shape) of T_E[A] x_3 DCT-II for uneven Kronecker sums."""
    out = []
    for w in synth.uneven_batch(count=count, lo=lo, hi=hi, rmin=rmin, rmax=rmax, noise=noise,
                                salt=salt):
        X = oracle.tensor_from_blockmat(w["A"], w["ell"], w["q"], w["m"], w["n"])
        xh = oracle.mode3(X, oracle.dct2_matrix(w["n"]))
        out.append(np.asfortranarray(xh.astype(np.float32).astype(np.float64)))
    return out


def _run(xhs, **kw):
    xd = [to_dev(x, np.float32) for x in xhs]
    bt = api.BatchedTruncator(xd, [x.shape for x in xhs], **kw)
    F = bt()
    torch.cuda.synchronize()
    return bt, xd, F


def _host(F, shape):
    m, p, nf = shape
    k = F.kmax
    return (from_dev(F.U, (m, k, nf)), from_dev(F.S, (k, nf)), from_dev(F.V, (p, k, nf)),
            from_dev(F.ranks, (nf,)), from_dev(F.cert, (nf,)), from_dev(F.fro, (nf,)),
            from_dev(F.info, (nf,)))


def _check_face(xf, U, S, V, r, cert, fro, ref_s, ref_r, ref_T, fro2, mode):
    """Rank, singular values, reconstruction and certificate of one face."""
    assert r == ref_r
    # eigenvalues of R R^T differ from those of X X^T by at most trace(S) <= 1e-3 tau^2 ||X||^2
    tol2 = (2e-3 * TAU * TAU if mode == "energy" else 1e-13) * fro2
    np.testing.assert_array_less(np.abs(S[:r] ** 2 - ref_s[:r] ** 2), tol2 + 1e-9 * ref_s[:r] ** 2 + 1e-300)
    T = (U[:, :r] * S[:r]) @ V[:, :r].T
    nrm = np.sqrt(fro2)
    assert np.linalg.norm(T - ref_T) <= 3e-6 * nrm + 1e-30
    disc2 = float(np.sum(ref_s[r:] ** 2))
    assert cert ** 2 >= disc2 * (1 - 1e-9) - 1e-13 * fro2
    assert cert ** 2 <= disc2 + tol2 + 1e-12 * fro2
    assert np.linalg.norm(xf - T) <= cert + 3e-6 * nrm
    assert fro == pytest.approx(nrm, rel=1e-12, abs=1e-300)
    if r:
        np.testing.assert_allclose(U[:, :r].T @ U[:, :r], np.eye(r), atol=2e-6)


@pytest.mark.parametrize("mode", ["energy", "fixed"])
def test_uneven_kronecker_batch_matches_oracle(mode):
    xhs = _kron_tensors(10, 6, 20, 2, 6, 1e-6, salt=1)
    k = 8 if mode == "energy" else 3
    bt, _, Fs = _run(xhs, rank_mode=C.RANK_ENERGY if mode == "energy" else C.RANK_FIXED, k=k,
                     tau=TAU if mode == "energy" else 0.5, kmax=8)
    for xh, F in zip(xhs, Fs):
        U, S, V, ranks, cert, fro, info = _host(F, xh.shape)
        ref = oracle.tsvdm_truncate_faces(xh, mode, k, TAU)
        assert np.all(info == 0)
        for f in range(xh.shape[2]):
            _check_face(xh[:, :, f], U[:, :, f], S[:, f], V[:, :, f], ranks[f], cert[f], fro[f],
                        ref["s"][:, f], ref["ranks"][f], ref["That"][:, :, f], ref["fro2"][f], mode)


def test_energy_faces_needing_more_than_16_pivots():
    """Faces with singular values 10^(-i/3.3): the energy rule keeps 14 of them
    (the discarded energy at ranks 13 and 14 is 1.32 and 0.33 times the bound,
    clear of it), but the pivoted Cholesky stops only after about 19 pivots
    (its trace tolerance is 1e-3 tau^2), so these faces take the 32-pivot
    pass, in one batch with Kronecker faces that finish within 16; all match
    the oracle."""
    g = np.random.default_rng(11)
    m, p, nf = 40, 50, 3
    graded = np.empty((m, p, nf))
    sig = 10.0 ** (-np.arange(m) / 3.3)
    for f in range(nf):
        q1, _ = np.linalg.qr(g.standard_normal((m, m)))
        q2, _ = np.linalg.qr(g.standard_normal((p, m)))
        graded[:, :, f] = (q1 * sig) @ q2.T
    xhs = [np.asfortranarray(graded.astype(np.float32).astype(np.float64))] + _kron_tensors(3, 6, 20, 2, 6, 1e-6,
                                                                                          salt=4)
    bt, _, Fs = _run(xhs, rank_mode=C.RANK_ENERGY, k=16, tau=TAU, kmax=16)
    for i, (xh, F) in enumerate(zip(xhs, Fs)):
        U, S, V, ranks, cert, fro, info = _host(F, xh.shape)
        ref = oracle.tsvdm_truncate_faces(xh, "energy", 16, TAU)
        assert np.all(info == 0)
        if i == 0:
            assert np.all(ranks == 14)
        for f in range(xh.shape[2]):
            _check_face(xh[:, :, f], U[:, :, f], S[:, f], V[:, :, f], ranks[f], cert[f], fro[f],
                        ref["s"][:, f], ref["ranks"][f], ref["That"][:, :, f], ref["fro2"][f], "energy")


def test_fixed_rank_above_16():
    """FIXED rank 20 with kmax 24 (the V kernel for ranks above 16): random
    faces of at most 32 rows, so the pivoted Cholesky is exact and the
    factors match the oracle's truncated SVD."""
    g = np.random.default_rng(13)
    xhs = [np.asfortranarray(g.standard_normal(sh).astype(np.float32).astype(np.float64))
           for sh in [(30, 50, 2), (21, 37, 3), (32, 20, 1)]]
    bt, _, Fs = _run(xhs, rank_mode=C.RANK_FIXED, k=20, tau=0.5, kmax=24)
    for xh, F in zip(xhs, Fs):
        U, S, V, ranks, cert, fro, info = _host(F, xh.shape)
        ref = oracle.tsvdm_truncate_faces(xh, "fixed", 20, TAU)
        assert np.all(info == 0) and np.all(ranks == 20)
        assert np.all(U[:, 20:, :] == 0) and np.all(V[:, 20:, :] == 0)
        for f in range(xh.shape[2]):
            _check_face(xh[:, :, f], U[:, :, f], S[:, f], V[:, :, f], ranks[f], cert[f], fro[f],
                        ref["s"][:, f], ref["ranks"][f], ref["That"][:, :, f], ref["fro2"][f], "fixed")


def test_edge_faces_single_row_zero_face_and_cap():
    """A one-row tensor, an all-zero face, a tensor of 64-row faces of full
    rank (the energy target cannot be met within the cap: rank = cap, flag 4,
    and the certificate still bounds the error of the returned factors)."""
    g = np.random.default_rng(5)
    one_row = np.asfortranarray(g.standard_normal((1, 50, 3)))
    zero = np.zeros((8, 30, 2), order="F")
    zero[:, :, 1] = g.standard_normal((8, 30))
    full = np.asfortranarray(g.standard_normal((64, 70, 2)))
    xhs = [x.astype(np.float32).astype(np.float64) for x in (one_row, zero, full)]
    bt, _, Fs = _run(xhs, rank_mode=C.RANK_ENERGY, k=16, tau=TAU, kmax=16)
    U, S, V, ranks, cert, fro, info = _host(Fs[0], xhs[0].shape)
    assert np.all(ranks == 1) and np.all(info == 0)
    for f in range(3):
        T = (U[:, :1, f] * S[:1, f]) @ V[:, :1, f].T
        assert np.linalg.norm(T - xhs[0][:, :, f]) <= 3e-6 * np.linalg.norm(xhs[0][:, :, f])
    U, S, V, ranks, cert, fro, info = _host(Fs[1], xhs[1].shape)
    assert ranks[0] == 0 and cert[0] == 0.0 and fro[0] == 0.0 and info[0] == 0
    assert np.all(U[:, :, 0] == 0) and np.all(V[:, :, 0] == 0) and np.all(S[:, 0] == 0)
    assert ranks[1] == 8
    U, S, V, ranks, cert, fro, info = _host(Fs[2], xhs[2].shape)
    assert np.all(ranks == 16) and np.all(info == 4)
    for f in range(2):
        xf = xhs[2][:, :, f]
        T = (U[:, :16, f] * S[:16, f]) @ V[:, :16, f].T
        true = np.linalg.norm(xf - T)
        assert true <= cert[f] * (1 + 1e-6) + 3e-6 * np.linalg.norm(xf)
        assert cert[f] > TAU * np.linalg.norm(xf)


def test_graph_capture_replays_and_autotune_match_eager(tmp_path):
    """The launch sequence captured in a graph gives, on every replay (with
    eager work and synchronisation in between), exactly the eager result; the
    autotuned configuration gives exactly the same result too (the per-face
    arithmetic does not depend on the launch configuration)."""
    xhs = _kron_tensors(6, 8, 24, 2, 5, 1e-6, salt=2)
    bt, xd, Fs = _run(xhs, rank_mode=C.RANK_ENERGY, k=8, tau=TAU, kmax=8)
    ref = [[t.clone() for t in (F.U, F.S, F.V, F.ranks, F.cert)] for F in Fs]
    cfg0 = bt.config()
    assert cfg0[3] in (0, 1)
    cfg = bt.autotune()
    torch.cuda.synchronize()
    assert cfg[3] == 1 and cfg[0] in (1, 2, 4) and cfg[1] in (16, 32) and cfg[2] in (1, 2, 4)
    for F, r in zip(Fs, ref):
        for a, b in zip((F.U, F.S, F.V, F.ranks, F.cert), r):
            assert torch.equal(a, b)
    # a second plan over the same shapes starts from the tuned configuration
    bt2 = api.BatchedTruncator(xd, [x.shape for x in xhs], rank_mode=C.RANK_ENERGY, k=8, tau=TAU,
                               kmax=8)
    assert bt2.config() == cfg
    # the table survives the process through its file: cleared, a new plan is
    # untuned; loaded back, a new plan starts tuned with the same configuration
    tune = tmp_path / "tune.txt"
    C.tsvdm_autotune_save(tune)
    C.tsvdm_autotune_clear()
    bt3 = api.BatchedTruncator(xd, [x.shape for x in xhs], rank_mode=C.RANK_ENERGY, k=8, tau=TAU, kmax=8)
    assert bt3.config()[3] == 0
    assert C.tsvdm_autotune_load(tune) >= 1
    bt4 = api.BatchedTruncator(xd, [x.shape for x in xhs], rank_mode=C.RANK_ENERGY, k=8, tau=TAU, kmax=8)
    assert bt4.config() == cfg
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bt(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        bt()
    for rep in range(3):
        for F in Fs:
            for t in (F.U, F.S, F.V, F.cert):
                t.fill_(-7.0)
            F.ranks.fill_(-7)
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for F, r in zip(Fs, ref):
            for a, b in zip((F.U, F.S, F.V, F.ranks, F.cert), r):
                assert torch.equal(a, b), f"replay {rep}"


def _device_kron_tensor(w, dev):
    """T_E[sum_r B_r kron C_r] x_3 DCT-II on the device: the matrix is formed
    with torch.kron (FP32) and mapped and transformed by the library."""
    B = torch.from_numpy(w["B"]).to(dev, torch.float32)
    Cc = torch.from_numpy(w["C"]).to(dev, torch.float32)
    A = torch.zeros(w["sB"] * w["sC"], w["sB"] * w["sC"], device=dev)
    for i in range(w["r"]):
        A += torch.kron(B[i], Cc[i])
    Acm = A.t().contiguous().reshape(-1)  # column major
    m, ell = w["sC"], w["sB"]
    view = C.tsvdm_tensor_from_blockmat(Acm.data_ptr(), ell * m, C.F32, ell, ell, m, m)
    xh = api.transform(Acm, m, ell * ell, m, C.M_DCT2, +1, view=view)
    return xh


def test_full_size_uneven_batch_sampled_faces():
    """The 256-matrix uneven batch (factor sizes log-uniform in [16, 64], 2..16
    terms, about 8.9k faces of 16..64 x 256..4096), energy rule tau = 1e-4:
    every rank equals the number of terms r (each face is a sum of r rank-one
    terms), and sampled faces match the oracle's closed-form faces."""
    mats = synth.uneven_batch(count=256, noise=0.0, form=False)
    dev = "cuda"
    xd = [_device_kron_tensor(w, dev) for w in mats]
    shapes = [(w["sC"], w["sB"] ** 2, w["sC"]) for w in mats]
    bt = api.BatchedTruncator(xd, shapes, rank_mode=C.RANK_ENERGY, k=16, tau=TAU, kmax=16)
    Fs = bt()
    torch.cuda.synchronize()
    nfaces = sum(s[2] for s in shapes)
    assert 8000 < nfaces < 10000
    odd = []
    for i, (w, F) in enumerate(zip(mats, Fs)):
        ranks = F.ranks.cpu().numpy()
        info = F.info.cpu().numpy()
        assert np.all(info == 0)
        assert np.all(ranks <= min(w["r"], w["sC"]))
        odd += [(i, int(f)) for f in np.nonzero(ranks != min(w["r"], w["sC"]))[0]]
    # a face whose r-th singular value falls below tau ||face|| has a lower
    # rank: those (rare) faces must match the oracle's rank exactly
    assert len(odd) < 50
    for i, f in odd:
        w = mats[i]
        xf = oracle.kron_sum_faces(w["B"], w["C"], oracle.dct2_matrix(w["sC"]), [f])[:, :, 0]
        s_ref = np.linalg.svd(xf, compute_uv=False)
        assert int(Fs[i].ranks[f].item()) == oracle.rank_energy(s_ref, float(np.sum(xf ** 2)), TAU, 16)
    g = np.random.default_rng(7)
    big = int(np.argmax([s[0] * s[1] for s in shapes]))
    picks = [(big, 0), (big, shapes[big][2] - 1)] + [(int(i), int(g.integers(shapes[i][2])))
                                                     for i in g.choice(256, 10, replace=False)]
    for i, f in picks:
        w, F, (m, p, nf) = mats[i], Fs[i], shapes[i]
        xf = oracle.kron_sum_faces(w["B"], w["C"], oracle.dct2_matrix(m), [f])[:, :, 0]
        s_ref = np.linalg.svd(xf, compute_uv=False)
        k = int(F.ranks[f].item())
        U = from_dev(F.U, (m, 16, nf))[:, :k, f]
        S = from_dev(F.S, (16, nf))[:k, f]
        V = from_dev(F.V, (p, 16, nf))[:, :k, f]
        nrm = np.linalg.norm(xf)
        np.testing.assert_allclose(S, s_ref[:k], atol=2e-6 * nrm)
        assert np.linalg.norm(xf - (U * S) @ V.T) <= 1e-5 * nrm
        assert float(F.cert[f].item()) <= 1e-5 * nrm
