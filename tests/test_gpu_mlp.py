"""GPU parity of the rank predictor kernels (tsvdm_mlp_*, tsvdm_rank_features)
against the oracle MLP with the same half-precision roundings."""
import struct
import zlib

import numpy as np
import pytest

import oracle
from oracle import mlp
import synth
from tests.gpu_helpers import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2105_01170_amd import api  # noqa: E402
from paper_2105_01170_amd import tsvdm as C  # noqa: E402


def _params(seed):
    g = np.random.default_rng(seed)
    theta = mlp.init_params(g)
    P = mlp.unpack(theta)
    for b in ("b1", "b2", "b3"):
        P[b][...] = g.uniform(-0.3, 0.3, P[b].shape)
    return theta


def _inputs(seed, n):
    g = np.random.default_rng(seed)
    # feature-like inputs: log10 ratios of a decreasing profile, in [-16, 0]
    X = -np.sort(g.uniform(0, 16, size=(n, 32)), axis=1)
    X[:, 0] = 0.0
    T = g.uniform(0, 1, size=(n, 2))
    return X, T


def _half(a):
    return a.astype(np.float16).astype(np.float64)


@pytest.mark.parametrize("n", [1, 200, 1000])
def test_forward_matches_oracle(n):
    theta = _params(1)
    X, _ = _inputs(2, n)
    pr = api.RankPredictor(torch.from_numpy(theta))
    y = pr.forward(torch.from_numpy(X).to("cuda", torch.float16)).cpu().numpy()
    ref, _ = mlp.forward(_half(theta), X, fp16=True)
    # half rounding of an activation may land on the other neighbour when the
    # FP32 and FP64 sums straddle a rounding boundary: a few half ulps
    scale = np.abs(ref).max()
    assert np.abs(y - ref).max() <= 4e-3 * scale


@pytest.mark.parametrize("n", [37, 128, 1024])
def test_gradient_and_loss_match_oracle(n):
    theta = _params(3)
    X, T = _inputs(4, n)
    pr = api.RankPredictor(torch.from_numpy(theta))
    g = pr.gradient(torch.from_numpy(X).to("cuda", torch.float16),
                    torch.from_numpy(T).to("cuda", torch.float32)).cpu().numpy()
    L, ref = mlp.backward(_half(theta), X, T, fp16=True)
    assert np.abs(g - ref).max() <= 5e-3 * np.abs(ref).max()
    assert float(pr.loss.item()) == pytest.approx(L, rel=5e-3)


def test_adam_step_matches_oracle():
    """One step from zero moments: w32 moves by -lr g / (|g| + eps); the half
    copy follows the master weights."""
    theta = _params(5)
    X, T = _inputs(6, 512)
    pr = api.RankPredictor(torch.from_numpy(theta))
    x16 = torch.from_numpy(X).to("cuda", torch.float16)
    t32 = torch.from_numpy(T).to("cuda", torch.float32)
    g = pr.gradient(x16, t32).cpu().numpy().astype(np.float64)
    pr.train_step(x16, t32, lr=1e-3)
    w = pr.w32.cpu().numpy().astype(np.float64)
    th32 = theta.astype(np.float32).astype(np.float64)
    ref, _, _ = mlp.adam_step(th32, np.zeros_like(g), np.zeros_like(g), g, 1, lr=1e-3)
    np.testing.assert_allclose(w, ref, atol=1e-6)
    np.testing.assert_array_equal(pr.w16.cpu().numpy(), pr.w32.cpu().numpy().astype(np.float16))


def test_rank_features_match_sketch_singular_values():
    """Features of faces with a known decay: log10(s_j / s_1) of the exact
    singular values of the same (BF16-product) sketch, to the BF16 level."""
    m, p, nf = 96, 80, 6
    fac = synth.known_rank_factors(m=m, p=p, n3=nf, k=32, decay=1.0 / 8.0, oversample=8, salt=3)
    Xh = np.zeros((m, p, nf), order="F")
    for f in range(nf):
        Xh[:, :, f] = (fac["U"][:, :, f] * fac["sigma"]) @ fac["V"][:, :, f].T
    Om = fac["Omega"]
    feats = api.rank_features(to_dev(Xh, np.float32), m, p, nf, to_dev(Om, np.float32)).cpu().numpy()
    for f in range(nf):
        s = np.linalg.svd(Xh[:, :, f].astype(np.float32).astype(np.float64) @ Om[:, :32].astype(np.float32),
                          compute_uv=False)
        ref = mlp.features(s)[0]
        # BF16 operands: relative error ~2^-8 on the sketch; the leading ratios
        # are accurate to a few 1e-3 in log10, the smallest ones less so
        np.testing.assert_allclose(feats[f, :16].astype(np.float64), ref[:16], atol=2e-2)
        assert np.all(np.diff(feats[f].astype(np.float64)) <= 1e-3)


def test_checkpoint_round_trip_corruption_and_resume(tmp_path):
    """Saving after a few Adam steps and loading into a fresh predictor restores
    weights, moments and step exactly; training on from the checkpoint gives
    the same weights as training on without it; a flipped byte, a truncated
    file and a foreign file are rejected."""
    theta = _params(7)
    X, T = _inputs(8, 256)
    x16 = torch.from_numpy(X).to("cuda", torch.float16)
    t32 = torch.from_numpy(T).to("cuda", torch.float32)
    a = api.RankPredictor(torch.from_numpy(theta))
    for _ in range(3):
        a.train_step(x16, t32, lr=1e-3)
    path = tmp_path / "pred.ckpt"
    a.save(path)
    saved_w32 = a.w32.cpu().numpy()
    b = api.RankPredictor(torch.zeros(C.tsvdm_mlp_nparams())).load(path)
    assert b.step == 3
    for name in ("w16", "w32", "m", "v"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name
    for _ in range(2):
        a.train_step(x16, t32, lr=1e-3)
        b.train_step(x16, t32, lr=1e-3)
    assert a.step == b.step == 5
    assert torch.equal(a.w32, b.w32) and torch.equal(a.m, b.m) and torch.equal(a.v, b.v)

    raw = bytearray(path.read_bytes())
    nbytes = 24 + C.tsvdm_mlp_nparams() * 14 + 4
    assert len(raw) == nbytes and raw[:8] == b"TSVDMMLP"
    # the documented layout: header fields, then the CRC-32 (IEEE 802.3) of all preceding bytes
    assert struct.unpack_from("<IIiI", raw, 8) == (1, C.tsvdm_mlp_nparams(), 3, 0)
    assert zlib.crc32(bytes(raw[:-4])) == struct.unpack_from("<I", raw, nbytes - 4)[0]
    n = C.tsvdm_mlp_nparams()
    w32 = np.frombuffer(bytes(raw[24 + 2 * n:24 + 6 * n]), dtype="<f4")
    np.testing.assert_array_equal(w32, saved_w32)
    c = api.RankPredictor(torch.from_numpy(theta))
    before = c.w32.clone()
    bad = tmp_path / "bad.ckpt"
    raw[1000] ^= 0x10
    bad.write_bytes(bytes(raw))
    with pytest.raises(C.TsvdmError, match="CRC"):
        c.load(bad)
    bad.write_bytes(path.read_bytes()[:-100])
    with pytest.raises(C.TsvdmError, match="bytes"):
        c.load(bad)
    bad.write_bytes(b"not a checkpoint" * 10)
    with pytest.raises(C.TsvdmError, match="not a predictor checkpoint"):
        c.load(bad)
    assert c.step == 0 and torch.equal(c.w32, before)  # nothing written on failure
