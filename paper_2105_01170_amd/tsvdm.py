"""Thin ctypes binding of the t-SVDM C ABI (include/tsvdm.h).

The functions here carry the C entry points' names and only marshal
arguments: every step of the computation runs in the HIP library
``libtsvdm.so``.  Device memory and streams come from the caller (PyTorch
tensors in the helpers below).  If the library is not built, loading it
raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsvdm.so")

# status / dtype / transform / rank / precision codes (tsvdm.h)
OK, EINVAL, EUNSUPPORTED, EWORKSPACE, EDEVICE = 0, 1, 2, 3, 4
F64, F32, BF16, C64, C128 = 0, 1, 2, 3, 4
M_DCT2, M_DFT, M_DENSE = 0, 1, 2
RANK_FIXED, RANK_ENERGY = 0, 1
PREC_F64, PREC_MIXED, PREC_F64_RAND = 0, 1, 2
(PLACE_GENERIC, PLACE_DIAGONAL, PLACE_BANDED, PLACE_BANDED_SYM, PLACE_TOEPLITZ, PLACE_TOEPLITZ_SYM,
 PLACE_HANKEL) = range(7)


class TsvdmMdesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("n3", ctypes.c_int64),
                ("M", ctypes.c_void_p)]


class TsvdmTensor(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("p", ctypes.c_int64), ("n3", ctypes.c_int64),
                ("s_a", ctypes.c_int64), ("s_b", ctypes.c_int64), ("s_t", ctypes.c_int64),
                ("bsplit", ctypes.c_int64), ("s_bk", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32), ("data", ctypes.c_void_p)]


class TsvdmTruncateOpts(ctypes.Structure):
    _fields_ = [("rank_mode", ctypes.c_int32), ("k", ctypes.c_int32), ("tau", ctypes.c_double),
                ("precision", ctypes.c_int32), ("oversample", ctypes.c_int32),
                ("power_iters", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("certify", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("omega", ctypes.c_void_p)]


class TsvdmFactors(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("p", ctypes.c_int64), ("nf", ctypes.c_int64),
                ("kmax", ctypes.c_int64), ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("U", ctypes.c_void_p), ("S", ctypes.c_void_p), ("V", ctypes.c_void_p),
                ("ranks", ctypes.c_void_p), ("cert", ctypes.c_void_p), ("fro", ctypes.c_void_p),
                ("info", ctypes.c_void_p)]


EXPORTS = ["tsvdm_version", "tsvdm_last_error", "tsvdm_tensor_from_blockmat",
           "tsvdm_check_orthogonal", "tsvdm_transform", "tsvdm_truncate_workspace_size",
           "tsvdm_truncate", "tsvdm_apply_workspace_size", "tsvdm_apply", "tsvdm_timing_enable",
           "tsvdm_timing_count", "tsvdm_timing_get", "tsvdm_batched_workspace_size",
           "tsvdm_batched_plan_create", "tsvdm_truncate_batched", "tsvdm_batched_autotune",
           "tsvdm_batched_config", "tsvdm_batched_set_config", "tsvdm_batched_plan_destroy", "tsvdm_mlp_nparams",
           "tsvdm_mlp_forward", "tsvdm_mlp_train_workspace_size", "tsvdm_mlp_gradient",
           "tsvdm_mlp_train_step", "tsvdm_f32_to_f16", "tsvdm_rank_features_workspace_size",
           "tsvdm_rank_features", "tsvdm_truncate_learned_workspace_size", "tsvdm_truncate_learned",
           "tsvdm_transform_batched_workspace_size", "tsvdm_transform_plan_create",
           "tsvdm_transform_batched", "tsvdm_transform_plan_destroy", "tsvdm_truncate_noalloc",
           "tsvdm_noalloc_scratch_bytes", "tsvdm_block_structure", "tsvdm_placement_workspace_size",
           "tsvdm_placement_create", "tsvdm_placement_eta", "tsvdm_placement_destroy",
           "tsvdm_tensor_from_blockmat_E", "tsvdm_blockmat_from_tensor_E", "tsvdm_apply_E_workspace_size",
           "tsvdm_apply_E", "tsvdm_mode_gram_workspace_size", "tsvdm_mode_gram", "tsvdm_sym_eig",
           "tsvdm_mode3_transform_workspace_size", "tsvdm_mode3_transform", "tsvdm_mode2_product",
           "tsvdm_kron_terms_count", "tsvdm_kron_terms", "tsvdm_mprod_workspace_size", "tsvdm_mprod",
           "tsvdm_tensor_from_blocks_E", "tsvdm_two_sided_workspace_size", "tsvdm_two_sided", "tsvdm_mlp_save",
           "tsvdm_mlp_load", "tsvdm_autotune_save", "tsvdm_autotune_load", "tsvdm_autotune_clear"]

_LIB = None


def lib():
    """Load libtsvdm.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.tsvdm_version.restype = i32
        L.tsvdm_version.argtypes = []
        L.tsvdm_last_error.restype = ctypes.c_char_p
        L.tsvdm_last_error.argtypes = []
        L.tsvdm_tensor_from_blockmat.restype = i32
        L.tsvdm_tensor_from_blockmat.argtypes = [vp, i64, i32, i64, i64, i64, i64, P(TsvdmTensor)]
        L.tsvdm_check_orthogonal.restype = i32
        L.tsvdm_check_orthogonal.argtypes = [vp, i64, ctypes.c_double]
        L.tsvdm_transform.restype = i32
        L.tsvdm_transform.argtypes = [P(TsvdmMdesc), i32, P(TsvdmTensor), P(TsvdmTensor), vp]
        L.tsvdm_transform_batched_workspace_size.restype = sz
        L.tsvdm_transform_batched_workspace_size.argtypes = [i32, P(TsvdmMdesc), P(TsvdmTensor)]
        L.tsvdm_transform_plan_create.restype = i32
        L.tsvdm_transform_plan_create.argtypes = [i32, P(TsvdmMdesc), i32, P(TsvdmTensor), P(TsvdmTensor), vp,
                                                  sz, P(vp)]
        L.tsvdm_transform_batched.restype = i32
        L.tsvdm_transform_batched.argtypes = [vp, vp]
        L.tsvdm_transform_plan_destroy.restype = None
        L.tsvdm_transform_plan_destroy.argtypes = [vp]
        L.tsvdm_truncate_workspace_size.restype = sz
        L.tsvdm_truncate_workspace_size.argtypes = [P(TsvdmTensor), P(TsvdmTruncateOpts)]
        L.tsvdm_truncate.restype = i32
        L.tsvdm_truncate.argtypes = [P(TsvdmTensor), P(TsvdmTruncateOpts), P(TsvdmFactors), vp, sz, vp]
        L.tsvdm_apply_workspace_size.restype = sz
        L.tsvdm_truncate_noalloc.argtypes = [P(TsvdmTensor), P(TsvdmTruncateOpts), P(TsvdmFactors), vp]
        L.tsvdm_truncate_noalloc.restype = i32
        L.tsvdm_noalloc_scratch_bytes.argtypes = []
        L.tsvdm_noalloc_scratch_bytes.restype = sz
        L.tsvdm_block_structure.argtypes = [i32, i64, i64, i64, vp, P(i64)]
        L.tsvdm_block_structure.restype = i32
        L.tsvdm_placement_workspace_size.argtypes = [i64, i64, i64]
        L.tsvdm_placement_workspace_size.restype = sz
        L.tsvdm_placement_create.argtypes = [i64, i64, i64, vp, vp, sz, P(vp)]
        L.tsvdm_placement_create.restype = i32
        L.tsvdm_placement_eta.argtypes = [vp, vp]
        L.tsvdm_placement_eta.restype = i32
        L.tsvdm_placement_destroy.argtypes = [vp]
        L.tsvdm_placement_destroy.restype = None
        L.tsvdm_tensor_from_blockmat_E.argtypes = [vp, vp, i64, i32, i64, i64, vp, vp]
        L.tsvdm_tensor_from_blockmat_E.restype = i32
        L.tsvdm_blockmat_from_tensor_E.argtypes = [vp, vp, i32, i64, i64, vp, i64, vp]
        L.tsvdm_blockmat_from_tensor_E.restype = i32
        L.tsvdm_apply_E_workspace_size.argtypes = [vp, P(TsvdmMdesc), P(TsvdmFactors), i64, i32]
        L.tsvdm_apply_E_workspace_size.restype = sz
        L.tsvdm_apply_E.argtypes = [vp, P(TsvdmMdesc), P(TsvdmFactors), i64, vp, i64, vp, i64, i32, vp, sz, vp]
        L.tsvdm_apply_E.restype = i32
        L.tsvdm_mode_gram_workspace_size.argtypes = [P(TsvdmTensor), i32]
        L.tsvdm_mode_gram_workspace_size.restype = sz
        L.tsvdm_mode_gram.argtypes = [P(TsvdmTensor), i32, vp, vp, sz, vp]
        L.tsvdm_mode_gram.restype = i32
        L.tsvdm_sym_eig.argtypes = [vp, i64, vp, vp, vp]
        L.tsvdm_sym_eig.restype = i32
        L.tsvdm_mode3_transform_workspace_size.argtypes = [P(TsvdmTensor)]
        L.tsvdm_mode3_transform_workspace_size.restype = sz
        L.tsvdm_mode3_transform.argtypes = [P(TsvdmTensor), vp, vp, vp, sz, vp]
        L.tsvdm_mode3_transform.restype = i32
        L.tsvdm_mode2_product.argtypes = [P(TsvdmTensor), vp, i64, i64, i32, vp, vp]
        L.tsvdm_mode2_product.restype = i32
        L.tsvdm_kron_terms_count.argtypes = [P(TsvdmMdesc), P(TsvdmFactors)]
        L.tsvdm_kron_terms_count.restype = i64
        L.tsvdm_kron_terms.argtypes = [P(TsvdmMdesc), P(TsvdmFactors), vp, i64, i64, vp, vp, vp]
        L.tsvdm_kron_terms.restype = i32
        L.tsvdm_mprod_workspace_size.argtypes = [P(TsvdmMdesc), P(TsvdmFactors), i64]
        L.tsvdm_mprod_workspace_size.restype = sz
        L.tsvdm_mprod.argtypes = [P(TsvdmMdesc), P(TsvdmFactors), P(TsvdmTensor), P(TsvdmTensor), vp, sz, vp]
        L.tsvdm_mprod.restype = i32
        L.tsvdm_tensor_from_blocks_E.argtypes = [vp, vp, i32, i64, i64, vp, vp]
        L.tsvdm_tensor_from_blocks_E.restype = i32
        L.tsvdm_two_sided_workspace_size.argtypes = [P(TsvdmTensor), i64]
        L.tsvdm_two_sided_workspace_size.restype = sz
        L.tsvdm_two_sided.argtypes = [P(TsvdmTensor), vp, i32, i64, i32, vp, vp, sz, vp]
        L.tsvdm_two_sided.restype = i32
        L.tsvdm_autotune_save.argtypes = [ctypes.c_char_p]
        L.tsvdm_autotune_save.restype = i32
        L.tsvdm_autotune_load.argtypes = [ctypes.c_char_p, P(i32)]
        L.tsvdm_autotune_load.restype = i32
        L.tsvdm_autotune_clear.argtypes = []
        L.tsvdm_autotune_clear.restype = None
        L.tsvdm_mlp_save.argtypes = [ctypes.c_char_p, vp, vp, vp, vp, i32]
        L.tsvdm_mlp_save.restype = i32
        L.tsvdm_mlp_load.argtypes = [ctypes.c_char_p, vp, vp, vp, vp, P(i32)]
        L.tsvdm_mlp_load.restype = i32
        L.tsvdm_apply_workspace_size.argtypes = [P(TsvdmMdesc), P(TsvdmFactors), i64, i64, i64, i32]
        L.tsvdm_apply.restype = i32
        L.tsvdm_apply.argtypes = [P(TsvdmMdesc), P(TsvdmFactors), i64, i64, i64, vp, i64, vp, i64,
                                  i32, vp, sz, vp]
        L.tsvdm_timing_enable.restype = i32
        L.tsvdm_timing_enable.argtypes = [i32]
        L.tsvdm_timing_count.restype = i32
        L.tsvdm_timing_count.argtypes = []
        L.tsvdm_timing_get.restype = i32
        L.tsvdm_timing_get.argtypes = [i32, P(ctypes.c_char_p), P(i32), P(ctypes.c_double)]
        L.tsvdm_batched_workspace_size.restype = sz
        L.tsvdm_batched_workspace_size.argtypes = [i32, P(TsvdmTensor)]
        L.tsvdm_batched_plan_create.restype = i32
        L.tsvdm_batched_plan_create.argtypes = [i32, P(TsvdmTensor), P(TsvdmTruncateOpts),
                                                P(TsvdmFactors), vp, sz, P(vp)]
        L.tsvdm_truncate_batched.restype = i32
        L.tsvdm_truncate_batched.argtypes = [vp, vp]
        L.tsvdm_batched_autotune.restype = i32
        L.tsvdm_batched_autotune.argtypes = [vp, vp]
        L.tsvdm_batched_config.restype = i32
        L.tsvdm_batched_config.argtypes = [vp, P(i32)]
        L.tsvdm_batched_set_config.restype = i32
        L.tsvdm_batched_set_config.argtypes = [vp, P(i32)]
        L.tsvdm_batched_plan_destroy.restype = None
        L.tsvdm_batched_plan_destroy.argtypes = [vp]
        L.tsvdm_mlp_nparams.restype = i64
        L.tsvdm_mlp_nparams.argtypes = []
        L.tsvdm_mlp_forward.restype = i32
        L.tsvdm_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
        L.tsvdm_mlp_train_workspace_size.restype = sz
        L.tsvdm_mlp_train_workspace_size.argtypes = [i64]
        L.tsvdm_mlp_gradient.restype = i32
        L.tsvdm_mlp_gradient.argtypes = [vp, vp, vp, i64, vp, vp, vp, sz, vp]
        L.tsvdm_mlp_train_step.restype = i32
        L.tsvdm_mlp_train_step.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, vp, vp, i64, vp, vp, sz, vp]
        L.tsvdm_f32_to_f16.restype = i32
        L.tsvdm_f32_to_f16.argtypes = [vp, vp, i64, vp]
        L.tsvdm_rank_features_workspace_size.restype = sz
        L.tsvdm_rank_features_workspace_size.argtypes = [P(TsvdmTensor)]
        L.tsvdm_rank_features.restype = i32
        L.tsvdm_rank_features.argtypes = [P(TsvdmTensor), vp, vp, vp, sz, vp]
        L.tsvdm_truncate_learned_workspace_size.restype = sz
        L.tsvdm_truncate_learned_workspace_size.argtypes = [P(TsvdmTensor)]
        L.tsvdm_truncate_learned.restype = i32
        L.tsvdm_truncate_learned.argtypes = [P(TsvdmTensor), P(TsvdmTruncateOpts), vp, P(TsvdmFactors), vp,
                                             vp, sz, vp]
        _LIB = L
    return _LIB


class TsvdmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tsvdm status {status}: {msg}")
        self.status = status


def _check(st):
    if st != OK:
        raise TsvdmError(st, lib().tsvdm_last_error().decode())
    return st


# ------------------------------------------------------------ C entry points
def tsvdm_version() -> int:
    return lib().tsvdm_version()


def tsvdm_last_error() -> str:
    return lib().tsvdm_last_error().decode()


def tsvdm_tensor_from_blockmat(A_ptr: int, lda: int, dtype: int, ell: int, q: int, m: int,
                               n: int) -> TsvdmTensor:
    out = TsvdmTensor()
    _check(lib().tsvdm_tensor_from_blockmat(A_ptr, lda, dtype, ell, q, m, n, ctypes.byref(out)))
    return out


def tsvdm_check_orthogonal(M_host_ptr: int, n3: int, tol: float) -> int:
    return lib().tsvdm_check_orthogonal(M_host_ptr, n3, tol)


def tsvdm_transform(M: TsvdmMdesc, direction: int, inp: TsvdmTensor, out: TsvdmTensor,
                    stream: int = 0):
    _check(lib().tsvdm_transform(ctypes.byref(M), direction, ctypes.byref(inp), ctypes.byref(out),
                                 stream))


def tsvdm_truncate_workspace_size(X: TsvdmTensor, opts: TsvdmTruncateOpts) -> int:
    return lib().tsvdm_truncate_workspace_size(ctypes.byref(X), ctypes.byref(opts))


def tsvdm_truncate(X: TsvdmTensor, opts: TsvdmTruncateOpts, F: TsvdmFactors, ws_ptr: int,
                   ws_bytes: int, stream: int = 0):
    _check(lib().tsvdm_truncate(ctypes.byref(X), ctypes.byref(opts), ctypes.byref(F), ws_ptr,
                                ws_bytes, stream))


def tsvdm_truncate_noalloc(X: TsvdmTensor, opts: TsvdmTruncateOpts, F: TsvdmFactors, stream: int = 0):
    _check(lib().tsvdm_truncate_noalloc(ctypes.byref(X), ctypes.byref(opts), ctypes.byref(F), stream))


def tsvdm_noalloc_scratch_bytes() -> int:
    return lib().tsvdm_noalloc_scratch_bytes()


def tsvdm_block_structure(kind: int, ell: int, q: int, b: int = 0):
    """(block_of as a list of ell*q ints, column major over the block grid; p)."""
    arr = (ctypes.c_int32 * (ell * q))()
    p = ctypes.c_int64(0)
    _check(lib().tsvdm_block_structure(kind, ell, q, b, arr, ctypes.byref(p)))
    return list(arr), p.value


def tsvdm_placement_workspace_size(ell: int, q: int, p: int) -> int:
    return lib().tsvdm_placement_workspace_size(ell, q, p)


def tsvdm_placement_create(ell: int, q: int, p: int, block_of, ws_ptr: int, ws_bytes: int) -> int:
    arr = (ctypes.c_int32 * (ell * q))(*block_of)
    h = ctypes.c_void_p(0)
    _check(lib().tsvdm_placement_create(ell, q, p, arr, ws_ptr, ws_bytes, ctypes.byref(h)))
    return h.value


def tsvdm_placement_eta(pl: int, p: int) -> list:
    arr = (ctypes.c_int32 * p)()
    _check(lib().tsvdm_placement_eta(pl, arr))
    return list(arr)


def tsvdm_placement_destroy(pl: int):
    lib().tsvdm_placement_destroy(pl)


def tsvdm_tensor_from_blockmat_E(pl: int, A_ptr: int, lda: int, dtype: int, m: int, n: int, X_ptr: int,
                                 stream: int = 0):
    _check(lib().tsvdm_tensor_from_blockmat_E(pl, A_ptr, lda, dtype, m, n, X_ptr, stream))


def tsvdm_blockmat_from_tensor_E(pl: int, X_ptr: int, dtype: int, m: int, n: int, A_ptr: int, lda: int,
                                 stream: int = 0):
    _check(lib().tsvdm_blockmat_from_tensor_E(pl, X_ptr, dtype, m, n, A_ptr, lda, stream))


def tsvdm_apply_E_workspace_size(pl: int, M: TsvdmMdesc, F: TsvdmFactors, nrhs: int, compute: int) -> int:
    return lib().tsvdm_apply_E_workspace_size(pl, ctypes.byref(M), ctypes.byref(F), nrhs, compute)


def tsvdm_apply_E(pl: int, M: TsvdmMdesc, F: TsvdmFactors, nrhs: int, x_ptr: int, ldx: int, y_ptr: int,
                  ldy: int, compute: int, ws_ptr: int, ws_bytes: int, stream: int = 0):
    _check(lib().tsvdm_apply_E(pl, ctypes.byref(M), ctypes.byref(F), nrhs, x_ptr, ldx, y_ptr, ldy, compute,
                               ws_ptr, ws_bytes, stream))


def tsvdm_mode_gram_workspace_size(X: TsvdmTensor, mode: int) -> int:
    return lib().tsvdm_mode_gram_workspace_size(ctypes.byref(X), mode)


def tsvdm_mode_gram(X: TsvdmTensor, mode: int, G_ptr: int, ws_ptr: int, ws_bytes: int, stream: int = 0):
    _check(lib().tsvdm_mode_gram(ctypes.byref(X), mode, G_ptr, ws_ptr, ws_bytes, stream))


def tsvdm_sym_eig(G_ptr: int, N: int, lam_ptr: int, W_ptr: int, stream: int = 0):
    _check(lib().tsvdm_sym_eig(G_ptr, N, lam_ptr, W_ptr, stream))


def tsvdm_mode3_transform_workspace_size(X: TsvdmTensor) -> int:
    return lib().tsvdm_mode3_transform_workspace_size(ctypes.byref(X))


def tsvdm_mode3_transform(X: TsvdmTensor, M_ptr: int, sv_ptr: int, ws_ptr: int, ws_bytes: int, stream: int = 0):
    _check(lib().tsvdm_mode3_transform(ctypes.byref(X), M_ptr, sv_ptr, ws_ptr, ws_bytes, stream))


def tsvdm_mode2_product(X: TsvdmTensor, V_ptr: int, pv: int, r: int, direction: int, out_ptr: int,
                        stream: int = 0):
    _check(lib().tsvdm_mode2_product(ctypes.byref(X), V_ptr, pv, r, direction, out_ptr, stream))


def tsvdm_kron_terms_count(M: TsvdmMdesc, F: TsvdmFactors) -> int:
    return lib().tsvdm_kron_terms_count(ctypes.byref(M), ctypes.byref(F))


def tsvdm_kron_terms(M: TsvdmMdesc, F: TsvdmFactors, pl: int, ell: int, q: int, C_ptr: int, D_ptr: int,
                     stream: int = 0):
    _check(lib().tsvdm_kron_terms(ctypes.byref(M), ctypes.byref(F), pl or None, ell, q, C_ptr, D_ptr, stream))


def tsvdm_mprod_workspace_size(M: TsvdmMdesc, F: TsvdmFactors, s: int) -> int:
    return lib().tsvdm_mprod_workspace_size(ctypes.byref(M), ctypes.byref(F), s)


def tsvdm_mprod(M: TsvdmMdesc, F: TsvdmFactors, X: TsvdmTensor, Y: TsvdmTensor, ws_ptr: int, ws_bytes: int,
                stream: int = 0):
    _check(lib().tsvdm_mprod(ctypes.byref(M), ctypes.byref(F), ctypes.byref(X), ctypes.byref(Y), ws_ptr, ws_bytes,
                             stream))


def tsvdm_tensor_from_blocks_E(pl: int, blocks_ptr: int, dtype: int, m: int, n: int, X_ptr: int, stream: int = 0):
    _check(lib().tsvdm_tensor_from_blocks_E(pl, blocks_ptr, dtype, m, n, X_ptr, stream))


def tsvdm_two_sided_workspace_size(X: TsvdmTensor, r: int) -> int:
    return lib().tsvdm_two_sided_workspace_size(ctypes.byref(X), r)


def tsvdm_two_sided(X: TsvdmTensor, U_ptr: int, udtype: int, r: int, direction: int, G_ptr: int, ws_ptr: int,
                    ws_bytes: int, stream: int = 0):
    _check(lib().tsvdm_two_sided(ctypes.byref(X), U_ptr, udtype, r, direction, G_ptr, ws_ptr, ws_bytes, stream))


def tsvdm_autotune_save(path: str):
    _check(lib().tsvdm_autotune_save(str(path).encode()))


def tsvdm_autotune_load(path: str) -> int:
    n = ctypes.c_int32(0)
    _check(lib().tsvdm_autotune_load(str(path).encode(), ctypes.byref(n)))
    return n.value


def tsvdm_autotune_clear():
    lib().tsvdm_autotune_clear()


def tsvdm_mlp_save(path: str, w16: int, w32: int, m: int, v: int, step: int):
    _check(lib().tsvdm_mlp_save(path.encode(), w16, w32, m, v, step))


def tsvdm_mlp_load(path: str, w16: int, w32: int, m: int, v: int) -> int:
    step = ctypes.c_int32(0)
    _check(lib().tsvdm_mlp_load(path.encode(), w16, w32, m, v, ctypes.byref(step)))
    return step.value


def tsvdm_apply_workspace_size(M: TsvdmMdesc, F: TsvdmFactors, ell: int, q: int, nrhs: int,
                               compute: int) -> int:
    return lib().tsvdm_apply_workspace_size(ctypes.byref(M), ctypes.byref(F), ell, q, nrhs, compute)


def tsvdm_apply(M: TsvdmMdesc, F: TsvdmFactors, ell: int, q: int, nrhs: int, x_ptr: int, ldx: int,
                y_ptr: int, ldy: int, compute: int, ws_ptr: int, ws_bytes: int, stream: int = 0):
    _check(lib().tsvdm_apply(ctypes.byref(M), ctypes.byref(F), ell, q, nrhs, x_ptr, ldx, y_ptr,
                             ldy, compute, ws_ptr, ws_bytes, stream))


def _array(ctype, items):
    arr = (ctype * len(items))()
    for i, it in enumerate(items):
        arr[i] = it
    return arr


def tsvdm_transform_batched_workspace_size(Ms: list, ins: list) -> int:
    if len(Ms) != len(ins):
        raise ValueError("one M descriptor per tensor")
    return lib().tsvdm_transform_batched_workspace_size(len(ins), _array(TsvdmMdesc, Ms),
                                                        _array(TsvdmTensor, ins))


def tsvdm_transform_plan_create(Ms: list, direction: int, ins: list, outs: list, ws_ptr: int,
                                ws_bytes: int) -> int:
    """Returns the opaque host plan handle (an address)."""
    if not (len(Ms) == len(ins) == len(outs)):
        raise ValueError("one M descriptor and one output per tensor")
    h = ctypes.c_void_p()
    _check(lib().tsvdm_transform_plan_create(len(ins), _array(TsvdmMdesc, Ms), direction,
                                             _array(TsvdmTensor, ins), _array(TsvdmTensor, outs), ws_ptr,
                                             ws_bytes, ctypes.byref(h)))
    return h.value


def tsvdm_transform_batched(plan: int, stream: int = 0):
    _check(lib().tsvdm_transform_batched(plan, stream))


def tsvdm_transform_plan_destroy(plan: int):
    lib().tsvdm_transform_plan_destroy(plan)


def tsvdm_batched_workspace_size(Xs: list) -> int:
    return lib().tsvdm_batched_workspace_size(len(Xs), _array(TsvdmTensor, Xs))


def tsvdm_batched_plan_create(Xs: list, opts: TsvdmTruncateOpts, Fs: list, ws_ptr: int,
                              ws_bytes: int) -> int:
    """Returns the opaque host plan handle (an address)."""
    if len(Xs) != len(Fs):
        raise ValueError("one factors descriptor per tensor")
    h = ctypes.c_void_p()
    _check(lib().tsvdm_batched_plan_create(len(Xs), _array(TsvdmTensor, Xs), ctypes.byref(opts),
                                           _array(TsvdmFactors, Fs), ws_ptr, ws_bytes,
                                           ctypes.byref(h)))
    return h.value


def tsvdm_truncate_batched(plan: int, stream: int = 0):
    _check(lib().tsvdm_truncate_batched(plan, stream))


def tsvdm_batched_autotune(plan: int, stream: int = 0):
    _check(lib().tsvdm_batched_autotune(plan, stream))


def tsvdm_batched_config(plan: int) -> list:
    cfg = (ctypes.c_int32 * 4)()
    _check(lib().tsvdm_batched_config(plan, cfg))
    return list(cfg)


def tsvdm_batched_set_config(plan: int, cfg) -> None:
    arr = (ctypes.c_int32 * 4)(*[int(v) for v in list(cfg)[:3]], 0)
    _check(lib().tsvdm_batched_set_config(plan, arr))


def tsvdm_batched_plan_destroy(plan: int):
    lib().tsvdm_batched_plan_destroy(plan)


def tsvdm_mlp_nparams() -> int:
    return lib().tsvdm_mlp_nparams()


def tsvdm_mlp_forward(w16: int, x: int, n: int, y: int, stream: int = 0):
    _check(lib().tsvdm_mlp_forward(w16, x, n, y, stream))


def tsvdm_mlp_train_workspace_size(n: int) -> int:
    return lib().tsvdm_mlp_train_workspace_size(n)


def tsvdm_mlp_gradient(w16: int, x: int, target: int, n: int, grad: int, loss: int, ws: int,
                       ws_bytes: int, stream: int = 0):
    _check(lib().tsvdm_mlp_gradient(w16, x, target, n, grad, loss or None, ws, ws_bytes, stream))


def tsvdm_mlp_train_step(w32: int, w16: int, m: int, v: int, step: int, lr: float, x: int,
                         target: int, n: int, loss: int, ws: int, ws_bytes: int, stream: int = 0):
    _check(lib().tsvdm_mlp_train_step(w32, w16, m, v, step, lr, x, target, n, loss or None, ws,
                                      ws_bytes, stream))


def tsvdm_f32_to_f16(a: int, b: int, n: int, stream: int = 0):
    _check(lib().tsvdm_f32_to_f16(a, b, n, stream))


def tsvdm_rank_features_workspace_size(X: TsvdmTensor) -> int:
    return lib().tsvdm_rank_features_workspace_size(ctypes.byref(X))


def tsvdm_rank_features(X: TsvdmTensor, omega: int, features: int, ws: int, ws_bytes: int,
                        stream: int = 0):
    _check(lib().tsvdm_rank_features(ctypes.byref(X), omega, features, ws, ws_bytes, stream))


def tsvdm_truncate_learned_workspace_size(X: TsvdmTensor) -> int:
    return lib().tsvdm_truncate_learned_workspace_size(ctypes.byref(X))


def tsvdm_truncate_learned(X: TsvdmTensor, opts: TsvdmTruncateOpts, w16: int, F: TsvdmFactors,
                           widths: int, ws: int, ws_bytes: int, stream: int = 0):
    _check(lib().tsvdm_truncate_learned(ctypes.byref(X), ctypes.byref(opts), w16, ctypes.byref(F),
                                        widths, ws, ws_bytes, stream))


def tsvdm_timing_enable(on: bool):
    _check(lib().tsvdm_timing_enable(1 if on else 0))


def tsvdm_timing_count() -> int:
    return lib().tsvdm_timing_count()


def tsvdm_timing_get(i: int):
    name = ctypes.c_char_p()
    n = ctypes.c_int32()
    ms = ctypes.c_double()
    _check(lib().tsvdm_timing_get(i, ctypes.byref(name), ctypes.byref(n), ctypes.byref(ms)))
    return name.value.decode(), n.value, ms.value


def timing_table() -> dict:
    """{kernel name: (launches, total ms)} of the current timing window."""
    return {name: (n, ms) for name, n, ms in (tsvdm_timing_get(i) for i in range(tsvdm_timing_count()))}


# ------------------------------------------------------------ descriptors
def mdesc(kind: int, n3: int, M_ptr: int = 0) -> TsvdmMdesc:
    return TsvdmMdesc(kind, 0, n3, M_ptr or None)


def dense_tensor(ptr: int, m: int, p: int, n3: int, dtype: int) -> TsvdmTensor:
    """Descriptor of a dense column-major (m, p, n3) tensor at device address ptr."""
    return TsvdmTensor(m, p, n3, 1, m, m * p, 0, 0, dtype, 0, ptr)


def truncate_opts(rank_mode=RANK_FIXED, k=1, tau=0.0, precision=PREC_F64, oversample=0,
                  power_iters=0, max_sweeps=0, certify=1, omega_ptr=0) -> TsvdmTruncateOpts:
    return TsvdmTruncateOpts(rank_mode, k, tau, precision, oversample, power_iters, max_sweeps,
                             certify, 0, omega_ptr or None)


def factors(m, p, nf, kmax, dtype, U, S, V, ranks, cert=0, fro=0, info=0) -> TsvdmFactors:
    return TsvdmFactors(m, p, nf, kmax, dtype, 0, U, S, V, ranks, cert or None, fro or None,
                        info or None)
