"""GPU checks of the learned-width truncation (tsvdm_truncate_learned):
certified errors, parity of sampled faces with the oracle's exact truncation,
the certificate fallback, and training of the predictor on library labels."""
import numpy as np
import pytest

import oracle
from oracle import mlp
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2105_01170_amd import api, learned  # noqa: E402
from paper_2105_01170_amd import tsvdm as C  # noqa: E402

M = P = 128
TAU = 1e-4


def _omega():
    g = np.random.default_rng(21)
    return torch.from_numpy(np.asfortranarray(g.standard_normal((P, 40))).astype(np.float32)
                            .ravel(order="F")).to("cuda")


def _faces(n, salt, lo=1 / 16, hi=1 / 2):
    rho = synth.decay_profiles(n, lo=lo, hi=hi, index=3, salt=salt)
    xh, sig = synth.decay_faces_device(rho, M, P, 32, index=3, salt=salt)
    return xh, sig


def _host(F, nf):
    k = F.kmax
    U = F.U.cpu().numpy().reshape((M, k, nf), order="F")
    S = F.S.cpu().numpy().reshape((k, nf), order="F")
    V = F.V.cpu().numpy().reshape((P, k, nf), order="F")
    return U, S, V


def _constant_predictor(width_out, rank_out=0.3):
    """Zero weights, output bias (rank_out, width_out): every face gets the same
    width and rank cap (rank 0.3 -> 10, within the width-16 cap of 13)."""
    theta = np.zeros(mlp.NPARAMS)
    mlp.unpack(theta)["b3"][...] = [rank_out, width_out]
    return api.RankPredictor(torch.from_numpy(theta))


def _check_batch(xh, F, widths, nf, sample):
    cert = F.cert.cpu().numpy()
    fro = F.fro.cpu().numpy()
    assert np.all(cert <= TAU * fro * (1 + 1e-12))
    assert set(np.unique(widths)) <= {16, 32, 40}
    U, S, V = _host(F, nf)
    ranks = F.ranks.cpu().numpy()
    X = xh.cpu().numpy().astype(np.float64).reshape((M, P, nf), order="F")
    for f in sample:
        xf = X[:, :, f]
        ref = oracle.tsvdm_truncate_faces(xf[:, :, None], "energy", 32, TAU)
        k = ranks[f]
        T = (U[:, :k, f] * S[:k, f]) @ V[:, :k, f].T
        true = np.linalg.norm(xf - T)
        assert true <= cert[f] * (1 + 1e-3) + 1e-6 * fro[f]
        # the randomized truncation keeps at least the optimal rank, not many more
        assert ref["ranks"][0] <= k <= ref["ranks"][0] + 3
        np.testing.assert_allclose(S[:k, f][:ref["ranks"][0]], ref["s"][:ref["ranks"][0], 0],
                                   rtol=1e-3, atol=1e-6 * fro[f])


def test_fallback_restores_the_tolerance():
    """A predictor that always answers width 16, on slowly decaying faces (the
    energy rank exceeds the width-16 cap of 13): every face fails its
    certificate there and is truncated again with width 40."""
    nf = 64
    xh, _ = _faces(nf, salt=1, lo=1 / 16, hi=1 / 12)
    pred = _constant_predictor(0.1)
    lt = api.LearnedTruncator(M, P, nf, _omega(), tau=TAU)
    F = lt(xh, pred)
    widths = lt.widths.cpu().numpy()
    assert np.all(widths == 40)
    _check_batch(xh, F, widths, nf, range(0, nf, 9))


def test_trained_predictor_widths_and_parity():
    """Train on library labels of 4096 faces, truncate 256 held-out faces:
    the certified error meets tau everywhere and sampled faces agree with the
    oracle's exact truncation."""
    om = _omega()
    feats, tg = [], []
    for b in range(16):
        xh, _ = _faces(256, salt=100 + b)
        feats.append(api.rank_features(xh, M, P, 256, om))
        rank, width = learned.labels(xh, M, P, 256, om, TAU)
        tg.append(learned.targets(rank, width))
    feats = torch.cat(feats)
    tg = torch.cat(tg)
    pred = api.RankPredictor(torch.from_numpy(mlp.init_params(np.random.default_rng(4))))
    hist = learned.train(pred, feats, tg, epochs=25, batch=512, lr=2e-3)
    assert hist[-1] < 0.2 * hist[0]
    xh, _ = _faces(256, salt=999)
    lt = api.LearnedTruncator(M, P, 256, om, tau=TAU)
    F = lt(xh, pred)
    widths = lt.widths.cpu().numpy()
    assert len(np.unique(widths)) >= 2  # the widths follow the faces
    _check_batch(xh, F, widths, 256, range(0, 256, 23))


def test_narrow_faces_take_the_narrow_width():
    """Fast decay (rho in [0.4, 0.5], energy rank <= 10): a width-16 answer
    holds for every face (no fallback), and the result is timed against the
    fixed width 40 on the same faces (printed)."""
    nf = 256
    xh, _ = _faces(nf, salt=7, lo=0.4, hi=0.5)
    om = _omega()
    pred = _constant_predictor(0.1)
    lt = api.LearnedTruncator(M, P, nf, om, tau=TAU)
    F = lt(xh, pred)
    widths = lt.widths.cpu().numpy()
    assert np.all(widths == 16)
    _check_batch(xh, F, widths, nf, range(0, nf, 31))
    fixed = api.Truncator(M, P, nf, torch.float32, rank_mode=C.RANK_ENERGY, k=32, tau=TAU,
                          precision=C.PREC_MIXED, oversample=8, power_iters=1, omega=om, kmax=32)
    times = {}
    for name, fn in (("fixed40", lambda: fixed(xh)), ("learned", lambda: lt(xh, pred))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            fn()
        e1.record()
        torch.cuda.synchronize()
        times[name] = e0.elapsed_time(e1) / 5
    print("narrow faces, ms per batch:", times)


def test_predicted_rank_moves_the_bucket_and_caps_the_rank():
    """The predicted rank takes part in the choice: a width-16 answer with a
    predicted rank of 20 (above the width-16 cap of 13) puts every face in the
    width-32 bucket, and the energy rule's cap becomes min(26, 20 + 2) = 22:
    on slowly decaying faces (energy rank above 22) every face misses there
    and falls back to width 40 with cap 32, meeting tau."""
    nf = 64
    xh, _ = _faces(nf, salt=3, lo=1 / 16, hi=1 / 14)
    lt = api.LearnedTruncator(M, P, nf, _omega(), tau=TAU)
    pred = _constant_predictor(0.1, rank_out=20 / 32)
    F = lt(xh, pred)
    assert np.all(lt.widths.cpu().numpy() == 40)
    _check_batch(xh, F, lt.widths.cpu().numpy(), nf, range(0, nf, 13))
    # faces of fast decay stay in the width-32 bucket, ranks within the cap 22
    xh2, _ = _faces(nf, salt=4, lo=0.25, hi=0.3)
    F2 = lt(xh2, pred)
    w2 = lt.widths.cpu().numpy()
    assert np.all(w2 == 32) and np.all(F2.ranks.cpu().numpy() <= 22)
    _check_batch(xh2, F2, w2, nf, range(0, nf, 13))


def test_learned_truncation_graph_replays_match_eager():
    """The learned truncation launches kernels only (bucket sizes stay on the
    device, buckets on internal streams joined by events): captured in a
    graph, every replay (with eager work and synchronization between) gives
    the eager result bit for bit, fallback faces included."""
    nf = 128
    xh_a, _ = _faces(nf // 2, salt=21, lo=0.4, hi=0.5)       # width 16 holds
    xh_b, _ = _faces(nf // 2, salt=22, lo=1 / 16, hi=1 / 12)  # fall back to width 40
    xh = torch.cat([xh_a, xh_b]).contiguous()
    lt = api.LearnedTruncator(M, P, nf, _omega(), tau=TAU)
    pred = _constant_predictor(0.1)
    F = lt(xh, pred)
    torch.cuda.synchronize()
    outs = (F.U, F.S, F.V, F.ranks, F.cert, F.fro, F.info, lt.widths)
    ref = [t.clone() for t in outs]
    w = lt.widths.cpu().numpy()
    assert np.all(w[: nf // 2] == 16) and np.all(w[nf // 2:] == 40)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        lt(xh, pred, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        lt(xh, pred)
    for rep in range(3):
        for t in outs:
            t.fill_(-7)
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert torch.equal(a, b), rep
        del junk


def test_library_rank_labels_equal_the_closed_form():
    """The rank labels the library produces for training (the width-40
    truncation's energy rank, cap 32) equal, face by face, the exact energy
    rank of the prescribed spectrum sigma_j = 10^(-rho j), j = 1..32 (the
    oracle's rank_label, itself pinned to the closed form of the geometric
    tail), on every face whose discarded energy stays 1e-2 tau^2 ||X_f||^2
    clear of the threshold at every k (most of the 256 faces)."""
    nf = 256
    xh, sig = _faces(nf, salt=41)
    rank, _ = learned.labels(xh, M, P, nf, _omega(), TAU)
    rank = rank.cpu().numpy()
    want = np.array([mlp.rank_label(s, TAU) for s in sig])
    clear = np.array([all(abs(np.sum(s[k:] ** 2) - TAU * TAU * np.sum(s * s)) >= 1e-2 * TAU * TAU * np.sum(s * s)
                          for k in range(33)) for s in sig])
    assert clear.sum() >= 200
    assert np.array_equal(rank[clear], want[clear]), np.nonzero(rank[clear] != want[clear])
    assert len(np.unique(want[clear])) >= 10  # the labels span the range of ranks
