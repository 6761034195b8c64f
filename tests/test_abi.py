"""C-ABI checks that need no GPU: symbols, struct layouts, host-side validation."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2105_01170_amd import tsvdm as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsvdm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tsvdm_[A-Za-z0-9_]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = C.lib()
    declared = _declared_functions()
    assert set(declared) == set(C.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
    assert C.tsvdm_version() >> 16 == 1


def test_struct_layout_matches_c_compiler(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "tsvdm.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("sizeof tsvdm_mdesc %zu\n", sizeof(tsvdm_mdesc));
  printf("sizeof tsvdm_tensor %zu\n", sizeof(tsvdm_tensor));
  printf("sizeof tsvdm_truncate_opts %zu\n", sizeof(tsvdm_truncate_opts));
  printf("sizeof tsvdm_factors %zu\n", sizeof(tsvdm_factors));
  P(tsvdm_mdesc, M); P(tsvdm_tensor, bsplit); P(tsvdm_tensor, dtype); P(tsvdm_tensor, data);
  P(tsvdm_truncate_opts, tau); P(tsvdm_truncate_opts, certify); P(tsvdm_truncate_opts, omega);
  P(tsvdm_factors, dtype); P(tsvdm_factors, U); P(tsvdm_factors, info);
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True,
                                                              text=True, check=True).stdout.split("\n") if line)
    out = {k: int(v) for k, v in out.items()}
    assert out["sizeof tsvdm_mdesc"] == ctypes.sizeof(C.TsvdmMdesc)
    assert out["sizeof tsvdm_tensor"] == ctypes.sizeof(C.TsvdmTensor)
    assert out["sizeof tsvdm_truncate_opts"] == ctypes.sizeof(C.TsvdmTruncateOpts)
    assert out["sizeof tsvdm_factors"] == ctypes.sizeof(C.TsvdmFactors)
    for key, val in out.items():
        if key.startswith("sizeof"):
            continue
        struct, field = key.split(".")
        cls = {"tsvdm_mdesc": C.TsvdmMdesc, "tsvdm_tensor": C.TsvdmTensor,
               "tsvdm_truncate_opts": C.TsvdmTruncateOpts, "tsvdm_factors": C.TsvdmFactors}[struct]
        assert getattr(cls, field).offset == val, key


def test_blockmat_view_strides():
    """T_E[A] view: X(a, j + ell*k, t) = A(j*m + a, k*n + t) with lda."""
    v = C.tsvdm_tensor_from_blockmat(0x1000, 50, C.F64, 3, 4, 7, 5)
    assert (v.m, v.p, v.n3) == (7, 12, 5)
    ell, lda, m, n = 3, 50, 7, 5
    for a, j, k, t in [(0, 0, 0, 0), (6, 2, 3, 4), (3, 1, 2, 0)]:
        b = j + ell * k
        addr = a * v.s_a + (b % v.bsplit) * v.s_b + (b // v.bsplit) * v.s_bk + t * v.s_t
        assert addr == (j * m + a) + lda * (k * n + t)


def test_blockmat_view_rejects_bad_arguments():
    with pytest.raises(C.TsvdmError) as e:
        C.tsvdm_tensor_from_blockmat(0x1000, 10, C.F64, 3, 4, 7, 5)  # lda < ell*m
    assert e.value.status == C.EINVAL
    with pytest.raises(C.TsvdmError):
        C.tsvdm_tensor_from_blockmat(0x1000, 50, C.C64, 3, 4, 7, 5)
    with pytest.raises(C.TsvdmError):
        C.tsvdm_tensor_from_blockmat(0, 50, C.F64, 3, 4, 7, 5)


def test_check_orthogonal_host():
    Q, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((9, 9)))
    Qf = np.asfortranarray(Q)
    assert C.tsvdm_check_orthogonal(Qf.ctypes.data, 9, 1e-12) == C.OK
    Qf[0, 0] += 1e-6
    assert C.tsvdm_check_orthogonal(Qf.ctypes.data, 9, 1e-12) == C.EINVAL
    assert "not orthogonal" in C.tsvdm_last_error()


def _t(m, p, n3, dt, ptr=0x1000):
    return C.dense_tensor(ptr, m, p, n3, dt)


@pytest.mark.parametrize("case", [
    dict(M=(C.M_DFT, 8), d=1, i=(4, 5, 8, C.F32), o=(4, 5, 8, C.C64)),      # out must have 5 faces
    dict(M=(C.M_DFT, 8), d=1, i=(4, 5, 8, C.F32), o=(4, 5, 5, C.F32)),      # out must be complex
    dict(M=(C.M_DCT2, 8), d=1, i=(4, 5, 8, C.F32), o=(4, 5, 8, C.F64)),     # precision mismatch
    dict(M=(C.M_DCT2, 8), d=2, i=(4, 5, 8, C.F32), o=(4, 5, 8, C.F32)),     # direction
    dict(M=(C.M_DCT2, 8), d=1, i=(4, 5, 8, C.F32), o=(4, 6, 8, C.F32)),     # p mismatch
    dict(M=(C.M_DENSE, 8), d=1, i=(4, 5, 8, C.F32), o=(4, 5, 8, C.F32)),    # dense without M
    dict(M=(C.M_DCT2, 4096), d=1, i=(4, 5, 4096, C.F32), o=(4, 5, 4096, C.F32)),  # too long
])
def test_transform_validation(case):
    M = C.mdesc(*case["M"])
    tin = _t(*case["i"], ptr=0x1000)
    tout = _t(*case["o"], ptr=0x9000)
    with pytest.raises(C.TsvdmError) as e:
        C.tsvdm_transform(M, case["d"], tin, tout, 0)
    assert e.value.status in (C.EINVAL, C.EUNSUPPORTED)
    assert C.tsvdm_last_error()


def test_transform_rejects_strided_output_and_aliasing():
    M = C.mdesc(C.M_DCT2, 8)
    tin = _t(4, 5, 8, C.F32, 0x1000)
    tout = _t(4, 5, 8, C.F32, 0x9000)
    tout.s_t = 999
    with pytest.raises(C.TsvdmError):
        C.tsvdm_transform(M, 1, tin, tout, 0)
    with pytest.raises(C.TsvdmError):
        C.tsvdm_transform(M, 1, tin, _t(4, 5, 8, C.F32, 0x1000), 0)


def test_truncate_validation_and_workspace():
    X = _t(64, 48, 4, C.F32)
    o = C.truncate_opts(C.RANK_FIXED, 8, 0.0, C.PREC_MIXED, 8, 1, 0, 1, 0x2000)
    ws = C.tsvdm_truncate_workspace_size(X, o)
    assert ws > 0
    F = C.factors(64, 48, 4, 8, C.F32, 0x3000, 0x4000, 0x5000, 0x6000)
    with pytest.raises(C.TsvdmError) as e:       # workspace too small
        C.tsvdm_truncate(X, o, F, 0x7000, ws - 1, 0)
    assert e.value.status == C.EWORKSPACE
    bad = [
        C.truncate_opts(C.RANK_FIXED, 8, 0.0, C.PREC_MIXED, 8, 1, 0, 1, 0),        # no omega
        C.truncate_opts(C.RANK_FIXED, 60, 0.0, C.PREC_MIXED, 8, 1, 0, 1, 0x2000),  # ell > 64
        C.truncate_opts(C.RANK_FIXED, 8, 0.0, C.PREC_MIXED, 8, 2, 0, 1, 0x2000),   # power iters
        C.truncate_opts(C.RANK_FIXED, 8, 0.0, C.PREC_F64, 0, 0, 0, 1, 0),          # F32 data, F64 path
        C.truncate_opts(7, 8, 0.0, C.PREC_MIXED, 8, 1, 0, 1, 0x2000),              # rank mode
        C.truncate_opts(C.RANK_ENERGY, 8, -1.0, C.PREC_MIXED, 8, 1, 0, 1, 0x2000),  # tau < 0
    ]
    # the size query reads shapes only: a missing omega is an error of the call,
    # not of the query
    assert C.tsvdm_truncate_workspace_size(X, bad[0]) == ws
    assert C.tsvdm_truncate_workspace_size(C.dense_tensor(0, 64, 48, 4, C.F32), o) == ws
    for i, ob in enumerate(bad):
        if i > 0:
            assert C.tsvdm_truncate_workspace_size(X, ob) == 0
        with pytest.raises(C.TsvdmError):
            C.tsvdm_truncate(X, ob, F, 0x7000, ws, 0)
    # factor shape and kmax checks
    with pytest.raises(C.TsvdmError):
        C.tsvdm_truncate(X, o, C.factors(64, 48, 5, 8, C.F32, 1, 2, 3, 4), 0x7000, ws, 0)
    with pytest.raises(C.TsvdmError):
        C.tsvdm_truncate(X, o, C.factors(64, 48, 4, 7, C.F32, 1, 2, 3, 4), 0x7000, ws, 0)
    with pytest.raises(C.TsvdmError):
        C.tsvdm_truncate(X, o, C.factors(64, 48, 4, 8, C.F64, 1, 2, 3, 4), 0x7000, ws, 0)


def test_apply_validation():
    M = C.mdesc(C.M_DFT, 8)
    F = C.factors(6, 12, 5, 3, C.C64, 1, 2, 3, 4)
    assert C.tsvdm_apply_workspace_size(M, F, 3, 4, 10, C.F32) > 0
    with pytest.raises(C.TsvdmError):  # p != ell*q
        C.tsvdm_apply(M, F, 3, 5, 10, 0x1000, 32, 0x2000, 18, C.F32, 0x3000, 1 << 20, 0)
    with pytest.raises(C.TsvdmError):  # real factors with the DFT
        C.tsvdm_apply(M, C.factors(6, 12, 5, 3, C.F32, 1, 2, 3, 4), 3, 4, 10, 0x1000, 32, 0x2000,
                      18, C.F32, 0x3000, 1 << 20, 0)
    with pytest.raises(C.TsvdmError):  # nf must be n3/2+1
        C.tsvdm_apply(M, C.factors(6, 12, 8, 3, C.C64, 1, 2, 3, 4), 3, 4, 10, 0x1000, 32, 0x2000,
                      18, C.F32, 0x3000, 1 << 20, 0)
    with pytest.raises(C.TsvdmError):  # ldx too small
        C.tsvdm_apply(M, F, 3, 4, 10, 0x1000, 31, 0x2000, 18, C.F32, 0x3000, 1 << 20, 0)
    with pytest.raises(C.TsvdmError) as e:  # workspace
        C.tsvdm_apply(M, F, 3, 4, 10, 0x1000, 32, 0x2000, 18, C.F32, 0x3000, 1, 0)
    assert e.value.status == C.EWORKSPACE
    with pytest.raises(C.TsvdmError):  # compute precision vs factors
        C.tsvdm_apply(M, F, 3, 4, 10, 0x1000, 32, 0x2000, 18, C.F64, 0x3000, 1 << 20, 0)


def test_batched_validation_and_workspace():
    """Shape, dtype, stride, option and workspace errors of the batched entry
    points are reported before any device work (no GPU needed)."""
    Xs = [_t(16, 256, 16, C.F32, 0x1000), _t(40, 900, 40, C.F32, 0x2000)]
    ws = C.tsvdm_batched_workspace_size(Xs)
    # face table + FP64 Gram of every face + queue counters
    assert ws >= 16 * 16 * 16 * 8 + 40 * 40 * 40 * 8
    Fs = [C.factors(16, 256, 16, 16, C.F32, 0x3000, 0x4000, 0x5000, 0x6000),
          C.factors(40, 900, 40, 16, C.F32, 0x3000, 0x4000, 0x5000, 0x6000)]
    o = C.truncate_opts(C.RANK_ENERGY, 16, 1e-4)
    with pytest.raises(C.TsvdmError) as e:        # workspace too small
        C.tsvdm_batched_plan_create(Xs, o, Fs, 0x7000, ws - 1)
    assert e.value.status == C.EWORKSPACE
    bad_tensors = [
        [_t(65, 256, 16, C.F32)],                  # more than 64 rows
        [_t(16, 256, 16, C.F64)],                  # FP32 only
        [_t(0, 256, 16, C.F32)],                   # empty face
    ]
    for Xb in bad_tensors:
        assert C.tsvdm_batched_workspace_size(Xb) == 0
        with pytest.raises(C.TsvdmError) as e:
            C.tsvdm_batched_plan_create(Xb, o, Fs[:1], 0x7000, 1 << 30)
        assert e.value.status == C.EINVAL
    strided = _t(16, 256, 16, C.F32)
    strided.s_t += 1
    assert C.tsvdm_batched_workspace_size([strided]) == 0
    bad_opts = [C.truncate_opts(C.RANK_ENERGY, 0, 1e-4), C.truncate_opts(C.RANK_ENERGY, 33, 1e-4),
                C.truncate_opts(C.RANK_ENERGY, 16, 0.0), C.truncate_opts(7, 16, 1e-4)]
    for ob in bad_opts:
        with pytest.raises(C.TsvdmError) as e:
            C.tsvdm_batched_plan_create(Xs, ob, Fs, 0x7000, ws)
        assert e.value.status == C.EINVAL
    # factors that do not match their tensor, or kmax below the rank cap
    Fbad = [C.factors(16, 255, 16, 16, C.F32, 0x3000, 0x4000, 0x5000, 0x6000), Fs[1]]
    with pytest.raises(C.TsvdmError):
        C.tsvdm_batched_plan_create(Xs, o, Fbad, 0x7000, ws)
    Fbad = [C.factors(16, 256, 16, 8, C.F32, 0x3000, 0x4000, 0x5000, 0x6000), Fs[1]]
    with pytest.raises(C.TsvdmError):
        C.tsvdm_batched_plan_create(Xs, o, Fbad, 0x7000, ws)
    with pytest.raises(C.TsvdmError):
        C.tsvdm_truncate_batched(0, 0)
    C.tsvdm_batched_plan_destroy(0)


def test_transform_batched_validation_and_workspace():
    """Batched transform plans: workspace sizing, and argument errors (naming
    the tensor) before any device work."""
    Ms = [C.mdesc(C.M_DCT2, 12), C.mdesc(C.M_DCT2, 45), C.mdesc(C.M_DFT, 8), C.mdesc(C.M_DCT2, 100)]
    ins = [_t(5, 7, 12, C.F32, 0x1000), _t(9, 14, 45, C.F32, 0x2000), _t(4, 5, 8, C.F32, 0x3000),
           _t(3, 4, 100, C.F32, 0x4000)]
    outs = [_t(5, 7, 12, C.F32, 0x5000), _t(9, 14, 45, C.F32, 0x6000), _t(4, 5, 5, C.C64, 0x7000),
            _t(3, 4, 100, C.F32, 0x8000)]
    ws = C.tsvdm_transform_batched_workspace_size(Ms, ins)
    # descriptors of all four tensors, then work items (tensor, tile): one tile
    # of 35 tubes (n3 <= 32 class) and two of 126 tubes (n3 <= 64 class)
    assert ws >= 256 + 2 * 256
    with pytest.raises(C.TsvdmError) as e:
        C.tsvdm_transform_plan_create(Ms, 1, ins, outs, 0x9000, ws - 1)
    assert e.value.status == C.EWORKSPACE
    bad = list(outs)
    bad[1] = _t(9, 14, 45, C.F64, 0x6000)  # precision differs from the input
    with pytest.raises(C.TsvdmError) as e:
        C.tsvdm_transform_plan_create(Ms, 1, ins, bad, 0x9000, ws)
    assert e.value.status == C.EINVAL
    assert "tensor 1" in C.tsvdm_last_error()
    with pytest.raises(C.TsvdmError) as e:
        C.tsvdm_transform_plan_create(Ms, 2, ins, outs, 0x9000, ws)  # direction
    assert e.value.status == C.EINVAL
    assert C.tsvdm_transform_batched_workspace_size([C.mdesc(7, 8)], ins[:1]) == 0
    # an empty batch needs no workspace and launches nothing
    assert C.tsvdm_transform_batched_workspace_size([], []) == 0
    plan = C.tsvdm_transform_plan_create([], 1, [], [], 0, 0)
    C.tsvdm_transform_plan_destroy(plan)


def test_batched_set_config_rejects_null_plan():
    arr = (ctypes.c_int32 * 4)(2, 16, 2, 0)
    assert C.lib().tsvdm_batched_set_config(None, arr) == C.EINVAL


# ------------------------------------------------------------ Sec. 3 placements (host code)
def _occurrences(block_of, ell, q):
    occ = {}
    for j in range(q):
        for i in range(ell):
            k = block_of[i + ell * j]
            if k >= 0:
                occ.setdefault(k, []).append((i, j))
    return occ


def test_block_structure_paper_block_tridiagonal_example():
    """BANDED_SYM with b = 1 on 4 x 4 blocks is the block-tridiagonal display of
    Sec. 3 (tests/golden/block_tridiagonal_4x4.txt): p = 7 and the same
    occurrences of every distinct block."""
    block_of, p = C.tsvdm_block_structure(C.PLACE_BANDED_SYM, 4, 4, 1)
    assert p == 7
    rows = np.loadtxt(os.path.join(ROOT, "tests", "golden", "block_tridiagonal_4x4.txt"), dtype=int)
    want = {}
    for k, i, j in rows:
        want.setdefault(k - 1, set()).add((i - 1, j - 1))
    got = {k: set(v) for k, v in _occurrences(block_of, 4, 4).items()}
    assert got == want


@pytest.mark.parametrize("ell,b", [(4, 1), (7, 1), (7, 2), (9, 3)])
def test_block_structure_banded_counts_match_the_paper(ell, b):
    """Sec. 3 block-banded example: p = l(2b+1) - b(b+1) distinct blocks when
    block-non-symmetric, p = l(b+1) - b(b+1)/2 when block-symmetric (l = ell
    blocks per side, b the block semibandwidth); for b = 1 these are 3l - 2 and
    2l - 1.  Every block in the band is covered, none outside."""
    bo, p = C.tsvdm_block_structure(C.PLACE_BANDED, ell, ell, b)
    assert p == ell * (2 * b + 1) - b * (b + 1)
    bs, ps = C.tsvdm_block_structure(C.PLACE_BANDED_SYM, ell, ell, b)
    assert ps == ell * (b + 1) - b * (b + 1) // 2
    if b == 1:
        assert (p, ps) == (3 * ell - 2, 2 * ell - 1)
    for j in range(ell):
        for i in range(ell):
            inside = abs(i - j) <= b
            assert (bo[i + ell * j] >= 0) == inside and (bs[i + ell * j] >= 0) == inside
    assert sorted(set(v for v in bo if v >= 0)) == list(range(p))
    # block-non-symmetric: every block in the band distinct; symmetric: (i, j) ~ (j, i)
    assert all(len(v) == 1 for v in _occurrences(bo, ell, ell).values())
    for j in range(ell):
        for i in range(ell):
            assert bs[i + ell * j] == bs[j + ell * i]


def test_block_structure_toeplitz_hankel_diagonal():
    """ex:btoep: 2l - 1 distinct blocks, the d-th lower diagonal repeated l - d
    times (weights 1/sqrt(l - d)); Hankel: constant anti-diagonals; the
    block-diagonal example: p = l; generic: p = l q, b = i + l j."""
    ell = 5
    bt, p = C.tsvdm_block_structure(C.PLACE_TOEPLITZ, ell, ell)
    assert p == 2 * ell - 1
    occ = _occurrences(bt, ell, ell)
    for d in range(ell):
        assert sorted(occ[d]) == sorted((i, i - d) for i in range(d, ell))
    for d in range(1, ell):
        assert sorted(occ[ell - 1 + d]) == sorted((i, i + d) for i in range(ell - d))
    bh, ph = C.tsvdm_block_structure(C.PLACE_HANKEL, 3, 4)
    assert ph == 6 and all(bh[i + 3 * j] == i + j for i in range(3) for j in range(4))
    bd, pd = C.tsvdm_block_structure(C.PLACE_DIAGONAL, 4, 4)
    assert pd == 4 and bd == [0, -1, -1, -1, -1, 1, -1, -1, -1, -1, 2, -1, -1, -1, -1, 3]
    bg, pg = C.tsvdm_block_structure(C.PLACE_GENERIC, 3, 2)
    assert pg == 6 and bg == list(range(6))
    bts, pts = C.tsvdm_block_structure(C.PLACE_TOEPLITZ_SYM, 4, 3)
    assert pts == 4 and all(bts[i + 4 * j] == abs(i - j) for i in range(4) for j in range(3))
    with pytest.raises(C.TsvdmError):
        C.tsvdm_block_structure(C.PLACE_DIAGONAL, 3, 4)
    with pytest.raises(C.TsvdmError):
        C.tsvdm_block_structure(99, 3, 4)


def test_autotune_table_file_round_trip_and_rejection(tmp_path):
    """The autotune table file: entries loaded from a file are saved back
    unchanged (sorted by key); a bad header, an out-of-range configuration or
    trailing junk is rejected with the line and merges nothing."""
    C.tsvdm_autotune_clear()
    src = tmp_path / "tune.txt"
    src.write_text("tsvdm-autotune 1\n0000010000132040 2 32 4\n00000100000f1030 1 16 1\n")
    assert C.tsvdm_autotune_load(src) == 2
    out = tmp_path / "out.txt"
    C.tsvdm_autotune_save(out)
    assert out.read_text() == "tsvdm-autotune 1\n00000100000f1030 1 16 1\n0000010000132040 2 32 4\n"
    assert not (tmp_path / "out.txt.tmp").exists()
    for body, msg in [("tsvdm-autotune 2\n", "not a version 1"),
                      ("tsvdm-autotune 1\n0000000000000001 2 24 4\n", "line 2"),
                      ("tsvdm-autotune 1\n0000000000000001 2 16 4\n0000000000000002 2 16 4 x\n", "line 3"),
                      ("tsvdm-autotune 1\n0000000000000003 0 16 4\n", "line 2")]:
        bad = tmp_path / "bad.txt"
        bad.write_text(body)
        with pytest.raises(C.TsvdmError, match=msg):
            C.tsvdm_autotune_load(bad)
    C.tsvdm_autotune_save(out)  # the failed loads merged nothing
    assert out.read_text().count("\n") == 3
    with pytest.raises(C.TsvdmError, match="cannot open"):
        C.tsvdm_autotune_load(tmp_path / "missing.txt")
    C.tsvdm_autotune_clear()
    C.tsvdm_autotune_save(out)
    assert out.read_text() == "tsvdm-autotune 1\n"


def test_truncate_complex_mixed_validation_and_workspace():
    """PREC_MIXED on complex (C64) faces: a workspace of its own size, C64
    factors required, sketch width at most 48, no allocation-free variant;
    C128 faces are refused (FP64 data belongs to the FP64 paths)."""
    X = _t(64, 48, 5, C.C64)
    o = C.truncate_opts(C.RANK_FIXED, 8, 0.0, C.PREC_MIXED, 8, 1, 0, 1, 0x2000)
    ws = C.tsvdm_truncate_workspace_size(X, o)
    assert ws > C.tsvdm_truncate_workspace_size(_t(64, 48, 5, C.F32), o) > 0
    F = C.factors(64, 48, 5, 8, C.C64, 0x3000, 0x4000, 0x5000, 0x6000)
    with pytest.raises(C.TsvdmError) as e:
        C.tsvdm_truncate(X, o, F, 0x7000, ws - 1, 0)
    assert e.value.status == C.EWORKSPACE
    with pytest.raises(C.TsvdmError):            # real factors for complex faces
        C.tsvdm_truncate(X, o, C.factors(64, 48, 5, 8, C.F32, 1, 2, 3, 4), 0x7000, ws, 0)
    wide = C.truncate_opts(C.RANK_FIXED, 41, 0.0, C.PREC_MIXED, 8, 1, 0, 1, 0x2000)  # ell 49
    Xw = _t(64, 64, 5, C.C64)
    assert C.tsvdm_truncate_workspace_size(Xw, wide) == 0
    with pytest.raises(C.TsvdmError) as e:
        C.tsvdm_truncate(Xw, wide, C.factors(64, 64, 5, 41, C.C64, 1, 2, 3, 4), 0x7000, 1 << 30, 0)
    assert e.value.status == C.EUNSUPPORTED
    assert C.tsvdm_truncate_workspace_size(_t(64, 48, 5, C.C128), o) == 0
    with pytest.raises(C.TsvdmError) as e:
        C.tsvdm_truncate_noalloc(X, o, F, 0)
    assert e.value.status == C.EUNSUPPORTED
