"""PyTorch-facing helpers around the C ABI.

PyTorch supplies device memory and the stream; every computation is a call
into libtsvdm.so through :mod:`.tsvdm`.  Tensors are flat device buffers in
the column-major layout of the C interface: a third-order (m, p, n3) tensor
has element (a, b, t) at a + m*b + m*p*t.  Complex data uses torch's complex
dtypes (interleaved re/im, as the C interface expects).
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import tsvdm as C

_TORCH_DT = {C.F64: torch.float64, C.F32: torch.float32, C.C64: torch.complex64,
             C.C128: torch.complex128}
_CODE = {v: k for k, v in _TORCH_DT.items()}


def dtype_code(t: torch.Tensor) -> int:
    return _CODE[t.dtype]


def _stream(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _mdesc(kind: int, n3: int, M: torch.Tensor | None):
    if kind == C.M_DENSE:
        if M is None or M.dtype != torch.float64 or not M.is_cuda:
            raise ValueError("dense M must be a float64 CUDA tensor (n3 x n3, column major)")
        return C.mdesc(kind, n3, M.data_ptr())
    return C.mdesc(kind, n3)


def transform(x: torch.Tensor, m: int, p: int, n3: int, kind: int, direction: int = 1,
              M: torch.Tensor | None = None, out: torch.Tensor | None = None, view=None,
              stream=None) -> torch.Tensor:
    """x (dense (m, p, nf_in) or the strided `view` descriptor over x) x_3 M^{+-1}."""
    real_in = not x.is_complex()
    if kind == C.M_DFT:
        nf_out = n3 // 2 + 1 if direction > 0 else n3
        if direction > 0:
            odt = torch.complex64 if x.dtype == torch.float32 else torch.complex128
        else:
            odt = torch.float32 if x.dtype == torch.complex64 else torch.float64
    else:
        nf_out = n3
        odt = x.dtype
    nf_in = n3 if (kind != C.M_DFT or direction > 0) else n3 // 2 + 1
    if out is None:
        out = torch.empty(m * p * nf_out, dtype=odt, device=x.device)
    tin = view if view is not None else C.dense_tensor(x.data_ptr(), m, p, nf_in, dtype_code(x))
    tout = C.dense_tensor(out.data_ptr(), m, p, nf_out, dtype_code(out))
    C.tsvdm_transform(_mdesc(kind, n3, M), direction, tin, tout, _stream(stream))
    del real_in
    return out


@dataclass
class Factors:
    m: int
    p: int
    nf: int
    kmax: int
    U: torch.Tensor
    S: torch.Tensor
    V: torch.Tensor
    ranks: torch.Tensor
    cert: torch.Tensor
    fro: torch.Tensor
    info: torch.Tensor

    def desc(self) -> C.TsvdmFactors:
        return C.factors(self.m, self.p, self.nf, self.kmax, dtype_code(self.U),
                         self.U.data_ptr(), self.S.data_ptr(), self.V.data_ptr(),
                         self.ranks.data_ptr(), self.cert.data_ptr(), self.fro.data_ptr(),
                         self.info.data_ptr())


def empty_factors(m, p, nf, kmax, dtype, device="cuda") -> Factors:
    return Factors(m, p, nf, kmax,
                   torch.zeros(m * kmax * nf, dtype=dtype, device=device),
                   torch.zeros(kmax * nf, dtype=torch.float64, device=device),
                   torch.zeros(p * kmax * nf, dtype=dtype, device=device),
                   torch.zeros(nf, dtype=torch.int32, device=device),
                   torch.zeros(nf, dtype=torch.float64, device=device),
                   torch.zeros(nf, dtype=torch.float64, device=device),
                   torch.zeros(nf, dtype=torch.int32, device=device))


class Truncator:
    """Holds the options, the workspace and the output factors of repeated
    tsvdm_truncate calls on tensors of one shape."""

    def __init__(self, m, p, nf, dtype, *, rank_mode=C.RANK_FIXED, k=1, tau=0.0,
                 precision=C.PREC_F64, oversample=0, power_iters=0, max_sweeps=0, certify=1,
                 omega: torch.Tensor | None = None, kmax=None, device="cuda"):
        self.omega = omega
        self.opts = C.truncate_opts(rank_mode, k, tau, precision, oversample, power_iters,
                                    max_sweeps, certify, omega.data_ptr() if omega is not None else 0)
        self.m, self.p, self.nf, self.dtype = m, p, nf, dtype
        probe = C.dense_tensor(0, m, p, nf, _CODE[dtype])
        self.ws_bytes = C.tsvdm_truncate_workspace_size(probe, self.opts)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)
        if kmax is None:
            ns = min(m, p)
            kmax = min(k if k > 0 else ns, ns)
            if precision != C.PREC_F64:
                kmax = min(kmax, k + oversample)
        if precision == C.PREC_MIXED:  # FP32 factors, complex for complex faces
            fdt = torch.complex64 if dtype == torch.complex64 else torch.float32
        else:
            fdt = dtype
        self.F = empty_factors(m, p, nf, max(kmax, 1), fdt, device)

    def __call__(self, xhat: torch.Tensor, stream=None) -> Factors:
        X = C.dense_tensor(xhat.data_ptr(), self.m, self.p, self.nf, dtype_code(xhat))
        C.tsvdm_truncate(X, self.opts, self.F.desc(), self.ws.data_ptr(), self.ws_bytes,
                         _stream(stream))
        return self.F


class BatchedTransform:
    """Mode-3 transforms of many tensors in few launches (tsvdm_transform_plan_*):
    ins[i] is the input (a dense device buffer of shape (m, p, n3) or, with
    views[i], any strided descriptor over it), outs[i] a dense output buffer,
    M[i] = (kind, n3, dense M or None).  Creating the object uploads the work
    list once; calling launches the batch asynchronously (safe to capture)."""

    def __init__(self, ins: list, outs: list, shapes: list, kinds: list, direction: int = 1,
                 Ms: list | None = None, views: list | None = None, device="cuda"):
        self.keep = (ins, outs, Ms)
        Ms = Ms if Ms is not None else [None] * len(ins)
        self.md = [_mdesc(k, n3, M) for k, (m, p, n3), M in zip(kinds, shapes, Ms)]
        def faces(kind, n3):  # (input faces, output faces), as for transform()
            if kind != C.M_DFT:
                return n3, n3
            return (n3, n3 // 2 + 1) if direction > 0 else (n3 // 2 + 1, n3)

        self.tin, self.tout = [], []
        for i, (x, y, (m, p, n3), k) in enumerate(zip(ins, outs, shapes, kinds)):
            fi, fo = faces(k, n3)
            self.tin.append(views[i] if views is not None and views[i] is not None else
                            C.dense_tensor(x.data_ptr(), m, p, fi, dtype_code(x)))
            self.tout.append(C.dense_tensor(y.data_ptr(), m, p, fo, dtype_code(y)))
        self.ws_bytes = C.tsvdm_transform_batched_workspace_size(self.md, self.tin)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)
        self.plan = C.tsvdm_transform_plan_create(self.md, direction, self.tin, self.tout, self.ws.data_ptr(),
                                                  self.ws_bytes)

    def __call__(self, stream=None):
        C.tsvdm_transform_batched(self.plan, _stream(stream))

    def __del__(self):
        plan = getattr(self, "plan", None)
        if plan:
            C.tsvdm_transform_plan_destroy(plan)
            self.plan = None


class BatchedTruncator:
    """Facewise truncation of an uneven batch (tsvdm_batched_*): the tensors
    xhats[i] are dense FP32 (m_i, p_i, nf_i) device buffers with m_i <= 64.
    Allocates the factors of every tensor and the workspace, creates the plan
    (one synchronous upload); calling launches the batch asynchronously (safe
    to capture in a CUDA/HIP graph)."""

    def __init__(self, xhats: list, shapes: list, *, rank_mode=C.RANK_ENERGY, k=16, tau=1e-4,
                 max_sweeps=0, kmax=None, device="cuda"):
        self.xhats = xhats
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.opts = C.truncate_opts(rank_mode, k, tau, C.PREC_F64, 0, 0, max_sweeps, 1, 0)
        kmax = k if kmax is None else kmax
        self.Xd = [C.dense_tensor(x.data_ptr(), m, p, nf, C.F32)
                   for x, (m, p, nf) in zip(xhats, self.shapes)]
        self.F = [empty_factors(m, p, nf, kmax, torch.float32, device) for (m, p, nf) in self.shapes]
        self.ws_bytes = C.tsvdm_batched_workspace_size(self.Xd)
        if self.ws_bytes == 0:
            raise C.TsvdmError(C.EINVAL, C.tsvdm_last_error())
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.plan = C.tsvdm_batched_plan_create(self.Xd, self.opts, [f.desc() for f in self.F],
                                                self.ws.data_ptr(), self.ws_bytes)

    def __call__(self, stream=None) -> list:
        C.tsvdm_truncate_batched(self.plan, _stream(stream))
        return self.F

    def autotune(self, stream=None) -> list:
        C.tsvdm_batched_autotune(self.plan, _stream(stream))
        return C.tsvdm_batched_config(self.plan)

    def config(self) -> list:
        return C.tsvdm_batched_config(self.plan)

    def set_config(self, cfg) -> None:
        C.tsvdm_batched_set_config(self.plan, cfg)

    def __del__(self):
        plan = getattr(self, "plan", None)
        if plan:
            C.tsvdm_batched_plan_destroy(plan)
            self.plan = None


class RankPredictor:
    """The rank/sketch-width predictor (tsvdm_mlp_*): FP32 master weights, the
    half copy the kernels read, Adam moments, and the training workspace."""

    def __init__(self, theta: torch.Tensor, device="cuda"):
        n = C.tsvdm_mlp_nparams()
        theta = theta.to(device=device, dtype=torch.float32).contiguous()
        if theta.numel() != n:
            raise ValueError(f"expected {n} parameters, got {theta.numel()}")
        self.w32 = theta.clone()
        self.w16 = torch.empty(n, dtype=torch.float16, device=device)
        self.m = torch.zeros(n, dtype=torch.float32, device=device)
        self.v = torch.zeros(n, dtype=torch.float32, device=device)
        self.step = 0
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self._ws = None
        C.tsvdm_f32_to_f16(self.w32.data_ptr(), self.w16.data_ptr(), n, _stream(None))

    def _workspace(self, n):
        need = C.tsvdm_mlp_train_workspace_size(n)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.w32.device)
        return self._ws

    def forward(self, x16: torch.Tensor, stream=None) -> torch.Tensor:
        n = x16.shape[0]
        y = torch.empty(n, 2, dtype=torch.float32, device=x16.device)
        C.tsvdm_mlp_forward(self.w16.data_ptr(), x16.data_ptr(), n, y.data_ptr(), _stream(stream))
        return y

    def gradient(self, x16: torch.Tensor, target: torch.Tensor, stream=None) -> torch.Tensor:
        n = x16.shape[0]
        ws = self._workspace(n)
        g = torch.empty(C.tsvdm_mlp_nparams(), dtype=torch.float32, device=x16.device)
        C.tsvdm_mlp_gradient(self.w16.data_ptr(), x16.data_ptr(), target.data_ptr(), n, g.data_ptr(),
                             self.loss.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream))
        return g

    def train_step(self, x16: torch.Tensor, target: torch.Tensor, lr=1e-3, stream=None):
        n = x16.shape[0]
        ws = self._workspace(n)
        self.step += 1
        C.tsvdm_mlp_train_step(self.w32.data_ptr(), self.w16.data_ptr(), self.m.data_ptr(),
                               self.v.data_ptr(), self.step, lr, x16.data_ptr(), target.data_ptr(), n,
                               self.loss.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream))
        return self.loss

    def save(self, path: str):
        """Write the training state (weights, Adam moments, step) to a checksummed file."""
        torch.cuda.synchronize(self.w32.device)
        C.tsvdm_mlp_save(str(path), self.w16.data_ptr(), self.w32.data_ptr(), self.m.data_ptr(),
                         self.v.data_ptr(), self.step)

    def load(self, path: str):
        """Restore the state written by save(); raises on a corrupt or foreign file."""
        torch.cuda.synchronize(self.w32.device)
        self.step = C.tsvdm_mlp_load(str(path), self.w16.data_ptr(), self.w32.data_ptr(), self.m.data_ptr(),
                                     self.v.data_ptr())
        return self


def rank_features(xhat: torch.Tensor, m: int, p: int, nf: int, omega: torch.Tensor,
                  stream=None) -> torch.Tensor:
    """(nf, 32) half features of every face (tsvdm_rank_features)."""
    X = C.dense_tensor(xhat.data_ptr(), m, p, nf, C.F32)
    need = C.tsvdm_rank_features_workspace_size(X)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=xhat.device)
    out = torch.empty(nf, 32, dtype=torch.float16, device=xhat.device)
    C.tsvdm_rank_features(X, omega.data_ptr(), out.data_ptr(), ws.data_ptr(), need, _stream(stream))
    return out


class LearnedTruncator:
    """tsvdm_truncate_learned on tensors of one shape: workspace, factors
    (kmax 32) and the per-face widths."""

    def __init__(self, m, p, nf, omega: torch.Tensor, tau=1e-4, power_iters=1, device="cuda"):
        self.m, self.p, self.nf = m, p, nf
        self.omega = omega
        self.opts = C.truncate_opts(C.RANK_ENERGY, 32, tau, C.PREC_MIXED, 8, power_iters, 0, 1,
                                    omega.data_ptr())
        X = C.dense_tensor(0, m, p, nf, C.F32)
        self.ws_bytes = C.tsvdm_truncate_learned_workspace_size(X)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)
        self.F = empty_factors(m, p, nf, 32, torch.float32, device)
        self.widths = torch.zeros(nf, dtype=torch.int32, device=device)

    def __call__(self, xhat: torch.Tensor, predictor: RankPredictor, stream=None) -> Factors:
        X = C.dense_tensor(xhat.data_ptr(), self.m, self.p, self.nf, C.F32)
        C.tsvdm_truncate_learned(X, self.opts, predictor.w16.data_ptr(), self.F.desc(),
                                 self.widths.data_ptr(), self.ws.data_ptr(), self.ws_bytes,
                                 _stream(stream))
        return self.F


def apply(F: Factors, kind: int, n3: int, ell: int, q: int, x: torch.Tensor, ldx: int | None = None,
          compute: int | None = None, M: torch.Tensor | None = None, y: torch.Tensor | None = None,
          ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """y = M_E[T] x for the factors F; x is (q*n3) x nrhs column major (flat)."""
    if compute is None:
        compute = C.F64 if F.U.dtype in (torch.float64, torch.complex128) else C.F32
    rdt = torch.float64 if compute == C.F64 else torch.float32
    rows_x = q * n3
    ldx = ldx or rows_x
    nrhs = x.numel() // ldx
    md = _mdesc(kind, n3, M)
    desc = F.desc()
    need = C.tsvdm_apply_workspace_size(md, desc, ell, q, nrhs, compute)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    if y is None:
        y = torch.empty(ell * F.m * nrhs, dtype=rdt, device=x.device)
    C.tsvdm_apply(md, desc, ell, q, nrhs, x.data_ptr(), ldx, y.data_ptr(), ell * F.m, compute,
                  ws.data_ptr(), need, _stream(stream))
    return y


class Placement:
    """A structured placement (Sec. 3): the block map of an ell x q block grid
    with p distinct blocks (block_of[i + ell*j] = k or -1), its device table
    in a torch-owned workspace, and the maps T_E, M_E and the structured apply
    through the C interface."""

    def __init__(self, ell: int, q: int, block_of, p: int | None = None, device="cuda"):
        block_of = [int(v) for v in block_of]
        self.ell, self.q = ell, q
        self.p = p if p is not None else max(block_of) + 1
        need = C.tsvdm_placement_workspace_size(ell, q, self.p)
        self.ws = torch.empty(max(need, 1), dtype=torch.uint8, device=device)
        self.handle = C.tsvdm_placement_create(ell, q, self.p, block_of, self.ws.data_ptr(), need)
        self.block_of = block_of

    @classmethod
    def structure(cls, kind: int, ell: int, q: int, b: int = 0, device="cuda"):
        block_of, p = C.tsvdm_block_structure(kind, ell, q, b)
        return cls(ell, q, block_of, p, device)

    def eta(self) -> list:
        return C.tsvdm_placement_eta(self.handle, self.p)

    def tensor_from_blockmat(self, A: torch.Tensor, m: int, n: int, lda: int | None = None,
                             out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """X = T_E[A] (dense m x p x n) from the column-major block matrix A (flat)."""
        lda = lda or self.ell * m
        if out is None:
            out = torch.empty(m * self.p * n, dtype=A.dtype, device=A.device)
        C.tsvdm_tensor_from_blockmat_E(self.handle, A.data_ptr(), lda, dtype_code(A), m, n, out.data_ptr(),
                                       _stream(stream))
        return out

    def tensor_from_blocks(self, blocks: torch.Tensor, m: int, n: int, out: torch.Tensor | None = None,
                           stream=None) -> torch.Tensor:
        """X = T_E from the distinct blocks stacked m x n x p (flat, column major)."""
        if out is None:
            out = torch.empty(m * self.p * n, dtype=blocks.dtype, device=blocks.device)
        C.tsvdm_tensor_from_blocks_E(self.handle, blocks.data_ptr(), dtype_code(blocks), m, n, out.data_ptr(),
                                     _stream(stream))
        return out

    def blockmat_from_tensor(self, X: torch.Tensor, m: int, n: int, out: torch.Tensor | None = None,
                             stream=None) -> torch.Tensor:
        """A = M_E[X] ((ell m) x (q n), flat column major) from the dense m x p x n tensor X."""
        if out is None:
            out = torch.empty(self.ell * m * self.q * n, dtype=X.dtype, device=X.device)
        C.tsvdm_blockmat_from_tensor_E(self.handle, X.data_ptr(), dtype_code(X), m, n, out.data_ptr(),
                                       self.ell * m, _stream(stream))
        return out

    def apply(self, F: Factors, kind: int, n3: int, x: torch.Tensor, compute: int | None = None,
              M: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """y = M_E[T] x for the factors F of the structured tensor (F.p == p)."""
        if compute is None:
            compute = C.F64 if F.U.dtype in (torch.float64, torch.complex128) else C.F32
        rdt = torch.float64 if compute == C.F64 else torch.float32
        ldx = self.q * n3
        nrhs = x.numel() // ldx
        md = _mdesc(kind, n3, M)
        desc = F.desc()
        need = C.tsvdm_apply_E_workspace_size(self.handle, md, desc, nrhs, compute)
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
        y = torch.empty(self.ell * F.m * nrhs, dtype=rdt, device=x.device)
        C.tsvdm_apply_E(self.handle, md, desc, nrhs, x.data_ptr(), ldx, y.data_ptr(), self.ell * F.m, compute,
                        ws.data_ptr(), need, _stream(stream))
        return y

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            C.tsvdm_placement_destroy(h)
            self.handle = None


def mode_gram(x: torch.Tensor, m: int, p: int, n3: int, mode: int, stream=None) -> torch.Tensor:
    """G = X_(mode) X_(mode)^T (FP64, column major flat) of the dense tensor x."""
    X = C.dense_tensor(x.data_ptr(), m, p, n3, dtype_code(x))
    N = n3 if mode == 3 else p
    need = C.tsvdm_mode_gram_workspace_size(X, mode)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    G = torch.empty(N * N, dtype=torch.float64, device=x.device)
    C.tsvdm_mode_gram(X, mode, G.data_ptr(), ws.data_ptr(), need, _stream(stream))
    return G


def sym_eig(G: torch.Tensor, N: int, stream=None):
    """(lam decreasing, W column major flat) of the symmetric N x N FP64 matrix G."""
    lam = torch.empty(N, dtype=torch.float64, device=G.device)
    W = torch.empty(N * N, dtype=torch.float64, device=G.device)
    C.tsvdm_sym_eig(G.data_ptr(), N, lam.data_ptr(), W.data_ptr(), _stream(stream))
    return lam, W


def mode3_transform(x: torch.Tensor, m: int, p: int, n3: int, stream=None):
    """(M = W^T, the singular values of X_(3)): the mode-3 HOSVD factor as a dense transform."""
    X = C.dense_tensor(x.data_ptr(), m, p, n3, dtype_code(x))
    need = C.tsvdm_mode3_transform_workspace_size(X)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    M = torch.empty(n3 * n3, dtype=torch.float64, device=x.device)
    sv = torch.empty(n3, dtype=torch.float64, device=x.device)
    C.tsvdm_mode3_transform(X, M.data_ptr(), sv.data_ptr(), ws.data_ptr(), need, _stream(stream))
    return M, sv


def mode2_product(x: torch.Tensor, m: int, p: int, n3: int, V: torch.Tensor, pv: int, r: int, direction: int,
                  stream=None) -> torch.Tensor:
    """x (m x p x n3) x_2 V^T (direction +1, p == pv) or x_2 V (direction -1, p == r)."""
    X = C.dense_tensor(x.data_ptr(), m, p, n3, dtype_code(x))
    pout = r if direction == 1 else pv
    out = torch.empty(m * pout * n3, dtype=x.dtype, device=x.device)
    C.tsvdm_mode2_product(X, V.data_ptr(), pv, r, direction, out.data_ptr(), _stream(stream))
    return out


def kron_terms(F: Factors, kind: int, n3: int, ell: int = 0, q: int = 0, placement: Placement | None = None,
               M: torch.Tensor | None = None, stream=None):
    """(C, D, nterms): the Kronecker terms of the truncated t-SVDM, C flat
    (ell*q*nterms), D flat (m*n3*nterms), column major per term."""
    md = _mdesc(kind, n3, M)
    desc = F.desc()
    nt = C.tsvdm_kron_terms_count(md, desc)
    if placement is not None:
        ell, q = placement.ell, placement.q
    rdt = torch.float64 if F.U.dtype in (torch.float64, torch.complex128) else torch.float32
    Cout = torch.empty(max(ell * q * nt, 1), dtype=rdt, device=F.U.device)
    Dout = torch.empty(max(F.m * n3 * nt, 1), dtype=rdt, device=F.U.device)
    C.tsvdm_kron_terms(md, desc, placement.handle if placement is not None else 0, ell, q, Cout.data_ptr(),
                       Dout.data_ptr(), _stream(stream))
    return Cout, Dout, nt


def mprod(F: Factors, kind: int, n3: int, x: torch.Tensor, s: int, M: torch.Tensor | None = None,
          stream=None) -> torch.Tensor:
    """Y = T *_M X for X (p x s x n3, flat column major) with the truncated t-SVDM F."""
    md = _mdesc(kind, n3, M)
    desc = F.desc()
    X = C.dense_tensor(x.data_ptr(), F.p, s, n3, dtype_code(x))
    y = torch.empty(F.m * s * n3, dtype=x.dtype, device=x.device)
    Y = C.dense_tensor(y.data_ptr(), F.m, s, n3, dtype_code(y))
    need = C.tsvdm_mprod_workspace_size(md, desc, s)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    C.tsvdm_mprod(md, desc, X, Y, ws.data_ptr(), need, _stream(stream))
    return y


def two_sided(x: torch.Tensor, m: int, p: int, U: torch.Tensor, r: int, stream=None) -> torch.Tensor:
    """G = X x_1 U^T x_3 U^T (r x p x r, FP64 flat) of the dense m x p x m tensor x."""
    X = C.dense_tensor(x.data_ptr(), m, p, m, dtype_code(x))
    need = C.tsvdm_two_sided_workspace_size(X, r)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    G = torch.empty(r * p * r, dtype=torch.float64, device=x.device)
    C.tsvdm_two_sided(X, U.data_ptr(), dtype_code(U), r, 1, G.data_ptr(), ws.data_ptr(), need, _stream(stream))
    return G


def two_sided_inverse(G: torch.Tensor, m: int, p: int, U: torch.Tensor, r: int, dtype=torch.float64,
                      stream=None) -> torch.Tensor:
    """T = G x_1 U x_3 U (m x p x m, flat)."""
    out = torch.empty(m * p * m, dtype=dtype, device=G.device)
    X = C.dense_tensor(out.data_ptr(), m, p, m, dtype_code(out))
    C.tsvdm_two_sided(X, U.data_ptr(), dtype_code(U), r, -1, G.data_ptr(), 0, 0, _stream(stream))
    return out
