"""GPU parity of tsvdm_transform against the oracle's explicit per-tube product."""
import numpy as np
import pytest

import oracle
from tests.gpu_helpers import from_dev, relerr, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2105_01170_amd import api  # noqa: E402
from paper_2105_01170_amd import tsvdm as C  # noqa: E402

# (m, p, n3): several tiles and a ragged tail of tubes; power-of-two lengths use
# the FFT kernel, others the direct kernel
SHAPES = [(5, 7, 8), (33, 17, 16), (64, 40, 32), (9, 11, 256), (3, 5, 1024), (7, 13, 12),
          (6, 5, 31), (4, 3, 1), (2, 3, 2), (17, 9, 100),
          # whole tiles with 16-byte rows: the vector load/store path
          (8, 16, 2), (16, 8, 1024), (32, 32, 64),
          # register-tiled direct product for lengths 33..64
          (9, 14, 45), (3, 300, 63)]
TOL = {np.float32: 3e-6, np.float64: 1e-12}


def _M(kind, n):
    return oracle.dct2_matrix(n) if kind == C.M_DCT2 else oracle.dft_matrix(n)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", [C.M_DCT2, C.M_DFT])
def test_forward_and_inverse(kind, shape, dt):
    m, p, n = shape
    g = np.random.default_rng(hash((kind, shape)) % 2**32)
    X = np.asfortranarray(g.standard_normal((m, p, n))).astype(dt)
    M = _M(kind, n)
    ref = oracle.mode3(X.astype(np.float64), M)
    if kind == C.M_DFT:
        ref = ref[:, :, : n // 2 + 1]
    xd = to_dev(X)
    yd = api.transform(xd, m, p, n, kind, +1)
    got = from_dev(yd, ref.shape)
    assert relerr(got, ref) < TOL[dt], relerr(got, ref)
    # inverse of the oracle's spectrum returns the original tensor
    back = api.transform(to_dev(ref.astype(got.dtype)), m, p, n, kind, -1)
    assert relerr(from_dev(back, X.shape), X.astype(np.float64)) < TOL[dt]


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_dense_orthogonal_M(dt):
    m, p, n = 11, 6, 24
    g = np.random.default_rng(3)
    M, _ = np.linalg.qr(g.standard_normal((n, n)))
    X = np.asfortranarray(g.standard_normal((m, p, n))).astype(dt)
    Md = to_dev(M, np.float64)
    y = api.transform(to_dev(X), m, p, n, C.M_DENSE, +1, M=Md)
    ref = oracle.mode3(X.astype(np.float64), M)
    assert relerr(from_dev(y, ref.shape), ref) < TOL[dt]
    back = api.transform(y, m, p, n, C.M_DENSE, -1, M=Md)
    assert relerr(from_dev(back, X.shape), X.astype(np.float64)) < TOL[dt]


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("ell,q,m,n", [(3, 5, 7, 16), (3, 5, 7, 21), (8, 6, 13, 37)])
def test_blockmat_view_zero_copy(dt, ell, q, m, n):
    """T_E[A] read in place through the strided view (Sec. 3 map, generic E):
    a power-of-two length (FFT) and two others (matrix-core direct product,
    the last over two chunks of tubes with a ragged tail)."""
    lda = ell * m + 3  # padded leading dimension
    g = np.random.default_rng(4)
    Afull = np.asfortranarray(g.standard_normal((lda, q * n))).astype(dt)
    A = Afull[: ell * m]
    Ad = to_dev(Afull)
    view = C.tsvdm_tensor_from_blockmat(Ad.data_ptr(), lda, C.F32 if dt == np.float32 else C.F64,
                                        ell, q, m, n)
    y = api.transform(Ad, m, ell * q, n, C.M_DCT2, +1, view=view)
    ref = oracle.mode3(oracle.tensor_from_blockmat(A.astype(np.float64), ell, q, m, n),
                       oracle.dct2_matrix(n))
    assert relerr(from_dev(y, ref.shape), ref) < TOL[dt]


def test_large_tile_count_dct256_fp32():
    """Launch shape of the 512 x 512 x 256 workload on a slab: 64 x 512 x 256."""
    m, p, n = 64, 512, 256
    g = np.random.default_rng(5)
    X = np.asfortranarray(g.standard_normal((m, p, n))).astype(np.float32)
    y = api.transform(to_dev(X), m, p, n, C.M_DCT2, +1)
    ref = oracle.mode3(X.astype(np.float64), oracle.dct2_matrix(n))
    assert relerr(from_dev(y, ref.shape), ref) < TOL[np.float32]


def test_empty_tensor_is_noop():
    x = torch.zeros(1, dtype=torch.float32, device="cuda")
    out = torch.full((1,), 7.0, dtype=torch.float32, device="cuda")
    t_in = C.dense_tensor(x.data_ptr(), 0, 5, 8, C.F32)
    t_out = C.dense_tensor(out.data_ptr(), 0, 5, 8, C.F32)
    C.tsvdm_transform(C.mdesc(C.M_DCT2, 8), 1, t_in, t_out, 0)
    torch.cuda.synchronize()
    assert out.item() == 7.0


@pytest.mark.parametrize("direction", [1, -1])
def test_batched_transform_matches_single_and_oracle(direction):
    """tsvdm_transform_batched over an uneven set (lengths in both direct
    classes, FP32 and FP64, a dense M, a strided T_E view, and tensors it
    launches one by one: DFT and n3 > 64) against tsvdm_transform and the
    oracle; replays from a captured graph give the same bits."""
    g = np.random.default_rng(7)
    Q, _ = np.linalg.qr(g.standard_normal((20, 20)))
    specs = [  # (m, p, n3, kind, dtype)
        (5, 7, 12, C.M_DCT2, np.float32), (33, 17, 31, C.M_DCT2, np.float32),
        (9, 14, 45, C.M_DCT2, np.float32), (3, 300, 63, C.M_DCT2, np.float64),
        (16, 8, 64, C.M_DCT2, np.float32), (6, 5, 20, C.M_DENSE, np.float64),
        (4, 5, 8, C.M_DFT, np.float32), (17, 9, 100, C.M_DCT2, np.float32),
        (2, 3, 1, C.M_DCT2, np.float32)]
    xs, outs, shapes, kinds, Ms, refs, views = [], [], [], [], [], [], []
    for (m, p, n3, kind, dt) in specs:
        if kind == C.M_DFT and direction < 0:
            Xh = (g.standard_normal((m, p, n3 // 2 + 1)) + 1j * g.standard_normal((m, p, n3 // 2 + 1)))
            X = np.asfortranarray(Xh.astype(np.complex64))
        else:
            X = np.asfortranarray(g.standard_normal((m, p, n3))).astype(dt)
        Md = to_dev(np.asfortranarray(Q), np.float64) if kind == C.M_DENSE else None
        xd = to_dev(X)
        single = api.transform(xd, m, p, n3, kind, direction, M=Md)
        xs.append(xd)
        outs.append(torch.empty_like(single))
        shapes.append((m, p, n3))
        kinds.append(kind)
        Ms.append(Md)
        refs.append(single)
        views.append(None)
    # a strided T_E view as one more input (forward and inverse read it the same way)
    ell, q, m, n = 3, 5, 7, 16
    A = np.asfortranarray(g.standard_normal((ell * m, q * n))).astype(np.float32)
    Ad = to_dev(A)
    view = C.tsvdm_tensor_from_blockmat(Ad.data_ptr(), ell * m, C.F32, ell, q, m, n)
    xs.append(Ad)
    single = api.transform(Ad, m, ell * q, n, C.M_DCT2, direction, view=view)
    outs.append(torch.empty_like(single))
    shapes.append((m, ell * q, n))
    kinds.append(C.M_DCT2)
    Ms.append(None)
    refs.append(single)
    views.append(view)
    bt = api.BatchedTransform(xs, outs, shapes, kinds, direction, Ms=Ms, views=views)
    bt()
    torch.cuda.synchronize()
    first = [o.clone() for o in outs]
    for i, (o, r, (m, p, n3), kind) in enumerate(zip(outs, refs, shapes, kinds)):
        pow2 = n3 >= 2 and (n3 & (n3 - 1)) == 0
        if kind != C.M_DFT and n3 <= 64 and pow2:
            # the batch uses the direct product where tsvdm_transform uses its FFT
            assert relerr(o.cpu().numpy(), r.cpu().numpy()) < (3e-6 if o.dtype == torch.float32 else 1e-12), i
        else:
            assert torch.equal(o, r), i
    # against the oracle's explicit product
    for i, ((m, p, n3, kind, dt), o) in enumerate(zip(specs, outs)):
        x = xs[i].cpu().numpy()
        if kind == C.M_DFT:
            continue  # covered by test_forward_and_inverse
        M = Q if kind == C.M_DENSE else oracle.dct2_matrix(n3)
        X = x.reshape((m, p, n3), order="F").astype(np.float64)
        ref = oracle.mode3(X, M if direction > 0 else M.T)
        assert relerr(from_dev(o, ref.shape), ref) < TOL[dt], i
    # replays of a captured graph reproduce the eager result
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        bt(stream=s)
    for _ in range(3):
        for o in outs:
            o.zero_()
        graph.replay()
        torch.cuda.synchronize()
        for o, f in zip(outs, first):
            assert torch.equal(o, f)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("direction", [1, -1])
def test_batched_direct_dct_every_length(dt, direction):
    """The batched plan transforms every tensor with n3 <= 64 by the direct
    product (the DCT-II as two half-size products over its even/odd symmetry),
    powers of two included: every length 1..64, each tensor over two chunks of
    tubes with a ragged tail, against the oracle's DCT-II matrix (forward) or
    its transpose (inverse)."""
    g = np.random.default_rng(17)
    m, p = 23, 41  # 943 tubes: two 512-tube chunks, the second partial
    xs, outs, shapes, Xs = [], [], [], []
    for n in range(1, 65):
        X = np.asfortranarray(g.standard_normal((m, p, n))).astype(dt)
        xd = to_dev(X)
        xs.append(xd)
        outs.append(torch.empty_like(xd))
        shapes.append((m, p, n))
        Xs.append(X)
    bt = api.BatchedTransform(xs, outs, shapes, [C.M_DCT2] * len(shapes), direction)
    bt()
    torch.cuda.synchronize()
    for X, o, (m_, p_, n) in zip(Xs, outs, shapes):
        M = oracle.dct2_matrix(n)
        ref = oracle.mode3(X.astype(np.float64), M if direction > 0 else np.ascontiguousarray(M.T))
        err = relerr(from_dev(o, ref.shape), ref)
        assert err < TOL[dt], (n, err)
