/*
 * tsvdm.h -- C ABI of the MI355X (gfx950) t-SVDM library.
 *
 * The library computes, on one GPU, the data-parallel core of the tensor-based
 * structured matrix approximation of Kilmer & Saibaba ("Structured matrix
 * approximations via tensor decompositions"), Algorithm alg:strategy (Sec. 3.1)
 * with a transform-domain truncated tensor SVD as the tensor compression of
 * step 3 (the paper admits any tensor approximation there, remarks of Sec. 3):
 *
 *   A  --T_E-->  X = T_E[A]  --x3 M-->  Xhat  --facewise truncated SVD-->
 *   (Uhat_f, S_f, Vhat_f)_f  --apply-->  y = M_E[T] x.
 *
 * Conventions shared by every entry point
 *  - Every data pointer is a DEVICE pointer owned by the caller; the library
 *    never allocates or frees device memory.  Scratch space is the caller's
 *    `workspace` of the size the matching *_workspace_size call returns.
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL = the
 *    null stream) and is asynchronous; results are valid after the caller
 *    synchronises the stream.
 *  - Column-major storage.  A third-order tensor of dims (m, p, n3) stores
 *    element (a, b, t) at a*s_a + b*s_b + t*s_t (dense: 1, m, m*p).  Frontal
 *    slices (faces) are the m x p matrices X(:, :, t) (Sec. 2.1).
 *  - Complex values (C64, C128) are interleaved (re, im) pairs.
 *  - Status: argument errors (null pointers, shapes, strides, dtypes, sizes,
 *    workspace) are detected on the host before anything is launched and are
 *    returned synchronously; tsvdm_last_error() then holds a message.  Errors
 *    found on the device (non-convergence, breakdown, non-finite input) are
 *    reported per face in tsvdm_factors.info after the stream is synchronised.
 *  - No C++ exception crosses this interface.  Calls are thread-safe as long
 *    as concurrent calls use distinct outputs and workspaces.
 */
#ifndef TSVDM_H
#define TSVDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tsvdm_status;
enum {
    TSVDM_OK = 0,
    TSVDM_EINVAL = 1,        /* bad argument (null pointer, shape, stride, size) */
    TSVDM_EUNSUPPORTED = 2,  /* valid but not implemented combination */
    TSVDM_EWORKSPACE = 3,    /* workspace missing or smaller than required */
    TSVDM_EDEVICE = 4        /* a HIP runtime call failed (launch, device query) */
};

/* element types */
enum {
    TSVDM_F64 = 0,
    TSVDM_F32 = 1,
    TSVDM_BF16 = 2,
    TSVDM_C64 = 3,   /* complex float  */
    TSVDM_C128 = 4   /* complex double */
};

/* the transform M applied along mode 3 (every tube) */
enum {
    TSVDM_M_DCT2 = 0,   /* orthonormal DCT-II: M[f,t] = a_f cos(pi (2t+1) f / (2 n3)) */
    TSVDM_M_DFT = 1,    /* unitary DFT: M[f,t] = n3^{-1/2} exp(-2 pi i f t / n3)      */
    TSVDM_M_DENSE = 2   /* caller-supplied real orthogonal n3 x n3 matrix             */
};

typedef struct {
    int32_t kind;      /* TSVDM_M_* */
    int32_t reserved;
    int64_t n3;        /* transform length (tube length in the original domain) */
    const double *M;   /* TSVDM_M_DENSE only: device pointer, n3 x n3, column major,
                          FP64.  Must be orthogonal (inverse = transpose); see
                          tsvdm_check_orthogonal. Ignored otherwise. */
} tsvdm_mdesc;

/* A strided third-order tensor.  The lateral index b may be split as
 * b = j + bsplit * k (0 <= j < bsplit): its address term is then
 * j*s_b + k*s_bk.  bsplit = 0 means no split (address term b*s_b).
 * The split expresses the zero-copy view T_E[A] of a block matrix. */
typedef struct {
    int64_t m, p, n3;
    int64_t s_a, s_b, s_t;
    int64_t bsplit, s_bk;
    int32_t dtype;     /* TSVDM_F32/F64/C64/C128 */
    int32_t reserved;
    void *data;        /* device pointer */
} tsvdm_tensor;

/* Rank selection for the facewise truncation */
enum {
    TSVDM_RANK_FIXED = 0,   /* k_f = min(k, min(m,p))                                  */
    TSVDM_RANK_ENERGY = 1   /* k_f = smallest k <= kcap with
                               sum_{j>k} s_{f,j}^2 <= tau^2 ||Xhat_f||_F^2            */
};

/* Arithmetic of the facewise truncation */
enum {
    TSVDM_PREC_F64 = 0,     /* plain: full facewise SVD by one-sided Jacobi in FP64     */
    TSVDM_PREC_MIXED = 1,   /* randomized range finder: BF16 sketch and first power
                               half-step, split-BF16 (FP32-accurate) final half-step
                               and projection, FP64 orthogonalisation and core SVD;
                               real (F32) or complex (C64) faces                      */
    TSVDM_PREC_F64_RAND = 2 /* the same randomized range finder with every product in
                               FP64 (FP64 MFMA) on an FP64 Xhat: FP64 accuracy of the
                               sketched truncation, for real M                        */
};

typedef struct {
    int32_t rank_mode;     /* TSVDM_RANK_* */
    int32_t k;             /* FIXED: the rank.  ENERGY: cap on the rank (<= kmax)   */
    double tau;            /* ENERGY: relative tolerance per face                   */
    int32_t precision;     /* TSVDM_PREC_* */
    int32_t oversample;    /* MIXED, F64_RAND: sketch width ell = k + oversample
                              (ell <= 64)                                            */
    int32_t power_iters;   /* MIXED, F64_RAND: 0 or 1 power iterations              */
    int32_t max_sweeps;    /* Jacobi sweep cap, 0 = default (60 plain, 30 core)     */
    int32_t certify;       /* MIXED, F64_RAND: 1 = cert by an explicit residual pass */
    int32_t reserved;
    const float *omega;    /* MIXED, F64_RAND: device, p x ell Gaussian test matrix, column
                              major FP32 (the random draws of the range finder)     */
} tsvdm_truncate_opts;

/* Transform-domain factors: face f holds Uhat_f (m x kmax), S_f (kmax),
 * Vhat_f (p x kmax); only the leading ranks[f] columns are meaningful, the
 * rest are zero.  nf = n3 for real transforms, n3/2+1 for the DFT of a real
 * tensor (the other faces are the conjugates). */
typedef struct {
    int64_t m, p, nf, kmax;
    int32_t dtype;     /* of U and V: F32 or F64 (real M); C64 or C128 (DFT) */
    int32_t reserved;
    void *U;           /* m x kmax x nf  */
    double *S;         /* kmax x nf, singular values, decreasing per face       */
    void *V;           /* p x kmax x nf  */
    int32_t *ranks;    /* nf */
    double *cert;      /* nf or NULL: the certificate ||Xhat_f - Uhat_f S_f Vhat_f^H||_F
                          of the returned factors.  PREC_F64: the discarded
                          singular values of the full SVD.  PREC_MIXED with
                          certify: evaluated after the factors are stored, from
                          the stored values (FP64 products and sums), so it is
                          the error of the factors the caller receives to within
                          ~1e-15 ||Xhat_f||_F; without certify: -1 (FIXED) or
                          the estimate the energy rule used (ENERGY).
                          PREC_F64_RAND: with certify as for MIXED; without,
                          the estimate sqrt(||Xhat_f||^2 - sum_{j<=k} s_j^2) */
    double *fro;       /* nf or NULL: ||Xhat_f||_F                               */
    int32_t *info;     /* nf or NULL: 0 ok, 1 Jacobi sweep cap reached,
                          2 Cholesky breakdown in the range finder, 3 non-finite,
                          4 ENERGY: no rank up to the cap meets tau (the cap is
                          returned).  When several apply, the larger code of
                          1..3 wins over 4 */
} tsvdm_factors;

/* Library version, (major << 16) | minor. */
int32_t tsvdm_version(void);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *tsvdm_last_error(void);

/* Zero-copy view X = T_E[A] of a column-major block matrix A ((ell*m) x (q*n),
 * leading dimension lda >= ell*m) for the generic placement of the remark
 * after Lemma lem:tenapprox (Sec. 3): p = ell*q distinct blocks, E_b = e_j e_k^T
 * with b = j + ell*k, eta = 1, so X(a, b, t) = A(j*m + a, k*n + t).
 * Fills *out; copies nothing.  dtype is TSVDM_F32 or TSVDM_F64. */
tsvdm_status tsvdm_tensor_from_blockmat(const void *A, int64_t lda, int32_t dtype, int64_t ell,
                                        int64_t q, int64_t m, int64_t n, tsvdm_tensor *out);

/* ---------------------------------------------------------------- structured placements
 * Sec. 3 (block matrix to tensor mapping) for a block matrix A ((ell m) x
 * (q n), ell x q blocks of m x n) whose blocks repeat: p distinct blocks A_k,
 * block (i, j) of A equal to A_{k(i,j)}, or a zero block (k = -1).  E_k holds
 * 1/sqrt(eta_k) at the eta_k positions of A_k (||E_k||_F = 1, eq. fnormw), and
 *   T_E[A](:, k, :) = sqrt(eta_k) twist(A_k)            (X is m x p x n),
 *   M_E[X] = sum_k E_k kron sq(X(:, k, :)),
 * so block (i, j) of M_E[X] is X(:, k(i,j), :) / sqrt(eta_k).  The block map is
 * an int32 HOST array block_of[i + ell j] (column major over the block grid,
 * 0-based).  Step 1 of Algorithm alg:strategy (determine E and A) for the
 * structures of the examples of Sec. 3: */
enum {
    TSVDM_PLACE_GENERIC = 0,       /* k = i + ell j, p = ell q (every block distinct)        */
    TSVDM_PLACE_DIAGONAL = 1,      /* block-diagonal example: k = i on the diagonal, p = ell */
    TSVDM_PLACE_BANDED = 2,        /* block-banded example, |i - j| <= b, every block in the
                                      band distinct, numbered column by column              */
    TSVDM_PLACE_BANDED_SYM = 3,    /* block-banded with (i, j) and (j, i) equal, numbered
                                      column by column over i <= j (ell == q)                */
    TSVDM_PLACE_TOEPLITZ = 4,      /* block-Toeplitz (example ex:btoep): k = i - j on the main
                                      and lower diagonals, ell - 1 + (j - i) above, p = ell+q-1 */
    TSVDM_PLACE_TOEPLITZ_SYM = 5,  /* block-Toeplitz with equal blocks on diagonals +-d:
                                      k = |i - j|, p = max(ell, q)                           */
    TSVDM_PLACE_HANKEL = 6         /* block-Hankel: k = i + j, p = ell + q - 1               */
};

/* Fills the host array block_of (ell*q entries) for `kind` (b: the block
 * semibandwidth of the banded kinds, ignored otherwise) and *p. */
tsvdm_status tsvdm_block_structure(int32_t kind, int64_t ell, int64_t q, int64_t b, int32_t *block_of,
                                   int64_t *p);

/* A placement: validation of block_of (entries in -1..p-1, every k occurring),
 * eta_k, a representative block of each k (the first in row-major block
 * order) and the weights sqrt(eta_k), 1/sqrt(eta_k) (IEEE double on the host),
 * uploaded (synchronous copy) into the caller's device workspace of
 * tsvdm_placement_workspace_size bytes, which must stay allocated while the
 * placement is used.  *pl is a host object released with
 * tsvdm_placement_destroy. */
typedef struct tsvdm_placement_s tsvdm_placement;
size_t tsvdm_placement_workspace_size(int64_t ell, int64_t q, int64_t p);
tsvdm_status tsvdm_placement_create(int64_t ell, int64_t q, int64_t p, const int32_t *block_of, void *workspace,
                                    size_t workspace_bytes, tsvdm_placement **pl);
/* eta (host, p entries): the occurrence counts. */
tsvdm_status tsvdm_placement_eta(const tsvdm_placement *pl, int32_t *eta);
void tsvdm_placement_destroy(tsvdm_placement *pl);

/* X = T_E[A]: A (device, column major, lda >= ell m) -> X (device, dense
 * m x p x n), dtype F32 or F64 (the weight product in FP64, then rounded to
 * the dtype).  Asynchronous on stream. */
tsvdm_status tsvdm_tensor_from_blockmat_E(const tsvdm_placement *pl, const void *A, int64_t lda, int32_t dtype,
                                          int64_t m, int64_t n, void *X, void *stream);

/* A = M_E[X]: X (device, dense m x p x n) -> A (device, (ell m) x (q n),
 * lda >= ell m; zero blocks written as zeros).  Asynchronous on stream. */
tsvdm_status tsvdm_blockmat_from_tensor_E(const tsvdm_placement *pl, const void *X, int32_t dtype, int64_t m,
                                          int64_t n, void *A, int64_t lda, void *stream);

/* X = T_E from the tuple of distinct blocks (the definition of Sec. 3,
 * T_E[A](:, k, :) = sqrt(eta_k) twist(A_k)): blocks (device) holds A_k at
 * blocks + m n k (m x n each, column major, the p blocks stacked), X (device,
 * dense m x p x n).  For matrices too large to form: only the p distinct blocks
 * are read.  Asynchronous. */
tsvdm_status tsvdm_tensor_from_blocks_E(const tsvdm_placement *pl, const void *blocks, int32_t dtype, int64_t m,
                                        int64_t n, void *X, void *stream);

/* y = M_E[T] x for the structured placement (T = That x_3 M^{-1}, That_f =
 * Uhat_f S_f Vhat_f^H from F, whose lateral size F->p is the placement's p):
 * the factors of the generic placement, Vg_f(i + ell j, r) = Vhat_f(k(i,j), r)
 * / sqrt(eta_k) (zero for zero blocks), are formed in the workspace and the
 * generic tsvdm_apply runs on them (same arguments, precisions and limits). */
size_t tsvdm_apply_E_workspace_size(const tsvdm_placement *pl, const tsvdm_mdesc *M, const tsvdm_factors *F,
                                    int64_t nrhs, int32_t compute);
tsvdm_status tsvdm_apply_E(const tsvdm_placement *pl, const tsvdm_mdesc *M, const tsvdm_factors *F, int64_t nrhs,
                           const void *x, int64_t ldx, void *y, int64_t ldy, int32_t compute, void *workspace,
                           size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------- data-driven transforms
 * Unfoldings of Sec. 2.1 for a dense real tensor X (m x p x n3, F32 or F64):
 * X_(3) (n3 x mp, row t = frontal face t, eq. mode3unfold) and X_(2) (p x mn,
 * row b = lateral slice b).  FP64 results throughout. */

/* G = X_(mode) X_(mode)^T for mode 3 (n3 x n3: inner products of the frontal
 * faces) or mode 2 (p x p: sum over faces of X_t^T X_t), order at most 64;
 * G device, column major.  Fixed workgroup count, partials summed in order
 * (deterministic).  Asynchronous on stream. */
size_t tsvdm_mode_gram_workspace_size(const tsvdm_tensor *X, int32_t mode);
tsvdm_status tsvdm_mode_gram(const tsvdm_tensor *X, int32_t mode, double *G, void *workspace, size_t workspace_bytes,
                             void *stream);

/* Eigendecomposition of a symmetric N x N FP64 matrix G (device, column major,
 * N <= 64) by the cyclic Jacobi solver in one workgroup: lam (N, device)
 * decreasing, W (N x N, device, column major) the eigenvectors, each with its
 * largest-magnitude entry positive (the first such entry on ties). */
tsvdm_status tsvdm_sym_eig(const double *G, int64_t N, double *lam, double *W, void *stream);

/* The mode-3 HOSVD factor (Sec. 2.4) as the transform: with W the left singular
 * vectors of X_(3) (eigenvectors of the mode-3 Gram, sign-fixed as above), M =
 * W^T (n3 x n3, device, column major, FP64) for TSVDM_M_DENSE, so that face f
 * of X x_3 M carries the energy sv[f]^2 of the unfolding; sv (n3, device, may
 * be NULL): the singular values of X_(3), decreasing.  n3 <= 64.  The Jacobi
 * solver stops rotating pairs below 1e-15 of the Gram's trace: eigenvalues
 * are exact to that absolute level, and rows of M for eigenvalues within it
 * of each other or of zero are some orthonormal basis of their subspace. */
size_t tsvdm_mode3_transform_workspace_size(const tsvdm_tensor *X);
tsvdm_status tsvdm_mode3_transform(const tsvdm_tensor *X, double *M, double *sv, void *workspace,
                                   size_t workspace_bytes, void *stream);

/* Mode-2 products of Sec. 6.3 with V (pv x r, device, column major, FP64):
 * direction +1: out = X x_2 V^T (X m x pv x n3 -> out m x r x n3, the core G);
 * direction -1: out = X x_2 V   (X m x r x n3 -> out m x pv x n3, T = G x_2 V).
 * out dense with X's dtype; FP64 accumulation.  Asynchronous on stream. */
tsvdm_status tsvdm_mode2_product(const tsvdm_tensor *X, const double *V, int64_t pv, int64_t r, int32_t direction,
                                 void *out, void *stream);

/* ---------------------------------------------------------------- the t-SVDM as a Kronecker sum and an operator
 * Kronecker terms of the truncated t-SVDM (the t-SVDM analogue of Thm
 * thm:tuckerkron; derived from T = That x_3 M^{-1}): M_E[T] = sum_j C_j kron D_j,
 *   C_j = struct(conj v_fr) = sum_b E_b conj(Vhat_f[b, r])   (ell x q; it keeps the
 *         block structure of the placement),
 *   D_j = S_f[r] Uhat_f[:, r] (M^{-1}[:, f])^T               (m x n3, rank one).
 * Real M: term j = f kmax + r.  DFT (stored half spectrum): each stored complex
 * triplet gives two real terms, 2 (f kmax + r) + {0, 1}: (Re C, w_f Re D) and
 * (Im C, -w_f Im D), w_f = 2 except faces 0 and n3/2, whose sum over the stored
 * faces is the real M_E[T] (Re D and Im D have rank at most two).  Terms with r >= ranks[f] are zero.  C (device):
 * ell*q*nterms, D (device): m*n3*nterms, column major, the factors' real type.
 * pl = NULL: the generic placement with ell*q = F->p.  Asynchronous. */
int64_t tsvdm_kron_terms_count(const tsvdm_mdesc *M, const tsvdm_factors *F);
tsvdm_status tsvdm_kron_terms(const tsvdm_mdesc *M, const tsvdm_factors *F, const tsvdm_placement *pl, int64_t ell,
                              int64_t q, void *C, void *D, void *stream);

/* The truncated t-SVDM as an M-product operator: Y = T *_M X for X (p x s x n3,
 * original domain, real, the factors' precision, any view tsvdm_transform
 * accepts), Y (m x s x n3, dense): Xhat = X x_3 M, Yhat_f = Uhat_f diag(S_f)
 * Vhat_f^H Xhat_f on every stored face, Y = Yhat x_3 M^{-1} (the product is
 * facewise in the transform domain).  kmax <= 64.  Asynchronous. */
size_t tsvdm_mprod_workspace_size(const tsvdm_mdesc *M, const tsvdm_factors *F, int64_t s);
tsvdm_status tsvdm_mprod(const tsvdm_mdesc *M, const tsvdm_factors *F, const tsvdm_tensor *X, tsvdm_tensor *Y,
                         void *workspace, size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------- SPSD-preserving compression
 * Sec. 5.1: for a symmetric positive semidefinite block matrix (ell = q, m = n)
 * the mode-1 and mode-3 unfoldings of X = T_E[A] (m x p x m) share their range
 * and one factor U (m x r, orthonormal columns, e.g. the dominant left singular
 * vectors of X_(1), which is X's memory read as one m x (p m) face) compresses
 * both: direction +1: G = X x_1 U^T x_3 U^T, G(:, b, :) = U^T sq(X(:, b, :)) U
 * (G device FP64, r x p x r); direction -1: X = G x_1 U x_3 U (X is the output).
 * M_E of the reconstruction is (I kron U U^T) A (I kron U U^T), positive
 * semidefinite whenever A is.  U: F32 or F64 (udtype), r <= 64.  FP64
 * accumulation.  Asynchronous. */
size_t tsvdm_two_sided_workspace_size(const tsvdm_tensor *X, int64_t r);
tsvdm_status tsvdm_two_sided(const tsvdm_tensor *X, const void *U, int32_t udtype, int64_t r, int32_t direction,
                             double *G, void *workspace, size_t workspace_bytes, void *stream);

/* Host-side check that the n3 x n3 column-major HOST matrix M is orthogonal:
 * max |M^T M - I| <= tol.  Returns TSVDM_OK or TSVDM_EINVAL. */
tsvdm_status tsvdm_check_orthogonal(const double *M_host, int64_t n3, double tol);

/* Mode-3 transform of every tube (Sec. 2.1: X x_3 M multiplies each tube by M).
 *   direction = +1: out = in x_3 M;   direction = -1: out = in x_3 M^{-1}.
 * DCT2 / DENSE: in and out are real (F32 or F64, same type), n3 faces each.
 * DFT, direction +1: real in (n3 faces) -> complex out (C64/C128) holding
 *   faces 0..n3/2 (out->n3 = n3/2 + 1).
 * DFT, direction -1: complex in holding faces 0..n3/2 -> real out (n3 faces);
 *   the remaining faces are taken as conjugates, imaginary parts of faces 0
 *   and n3/2 are ignored.
 * `in` may be any strided view (e.g. from tsvdm_tensor_from_blockmat); `out`
 * must be dense (strides 1, m, m*p) and must not overlap `in`.
 * Power-of-two n3 (2..1024) uses an FFT in LDS; other lengths and DENSE use
 * a direct per-tube product. */
tsvdm_status tsvdm_transform(const tsvdm_mdesc *M, int32_t direction, const tsvdm_tensor *in,
                             tsvdm_tensor *out, void *stream);

/* Batched mode-3 transform of nmat independent tensors (Sec. 2.1 for each;
 * the inputs of the uneven batch below): out[i] = in[i] x_3 M[i]^(+-1), every
 * (M[i], in[i], out[i]) as for tsvdm_transform, one direction for all.  The
 * tensors whose M is DCT2 or DENSE with n3 <= 64 (and whose view and output
 * span less than 2 GiB) are transformed by the direct per-tube product:
 * workgroup w takes chunk w of a work list of 512-tube chunks of all of them,
 * in one launch per precision for the DCT2 tensors (the DCT-II as two
 * half-size products over its even/odd symmetry) and one per precision and
 * length class (n3 in 1..16, 17..32, 33..48, 49..64) for the DENSE ones.  The
 * other tensors (DFT, n3 > 64, larger spans) are launched one by one, as
 * tsvdm_transform would.  Results equal tsvdm_transform's bit for bit
 * where it too uses the direct product (n3 not a power of two, or DENSE); for
 * a power-of-two n3 <= 64, where tsvdm_transform uses its FFT, they agree to
 * rounding.
 *
 * Usage: size the workspace, create a plan (validation, one synchronous
 * upload of the tensor descriptors and the work list into the workspace),
 * then launch with tsvdm_transform_batched as often as needed (asynchronous;
 * no allocation, no host-device copy: safe under stream capture).  The plan
 * keeps the device pointers and M descriptors it was created with; the
 * workspace must stay allocated and untouched while the plan is used. */
typedef struct tsvdm_transform_plan_s tsvdm_transform_plan;

/* Workspace bytes for the batch (host arrays M[nmat], in[nmat]; shapes and M
 * kinds only).  0 if the arguments are invalid or nothing needs a table. */
size_t tsvdm_transform_batched_workspace_size(int32_t nmat, const tsvdm_mdesc *M, const tsvdm_tensor *in);

/* Validates every tensor (errors name the tensor index), builds the work
 * list and uploads it into the caller's workspace (synchronous copy).  *plan
 * is a host object released with tsvdm_transform_plan_destroy. */
tsvdm_status tsvdm_transform_plan_create(int32_t nmat, const tsvdm_mdesc *M, int32_t direction,
                                         const tsvdm_tensor *in, const tsvdm_tensor *out, void *workspace,
                                         size_t workspace_bytes, tsvdm_transform_plan **plan);

/* Launches the batch on `stream` (asynchronous). */
tsvdm_status tsvdm_transform_batched(const tsvdm_transform_plan *plan, void *stream);

/* Releases the host plan (the workspace stays the caller's). NULL is allowed. */
void tsvdm_transform_plan_destroy(tsvdm_transform_plan *plan);

/* Workspace bytes tsvdm_truncate needs for this input and options (only the
 * shapes are read: data and omega may be NULL).  0 if the arguments are invalid. */
size_t tsvdm_truncate_workspace_size(const tsvdm_tensor *Xhat, const tsvdm_truncate_opts *opts);

/* Facewise truncated SVD of a dense transform-domain tensor Xhat (the output
 * of tsvdm_transform): for every face f, Xhat_f ~ Uhat_f diag(S_f) Vhat_f^H
 * with rank ranks[f] chosen by opts->rank_mode.  Together with the inverse
 * transform this is the truncated t-SVDM, step 3 of Algorithm alg:strategy.
 *   PREC_F64:   Xhat FP64 or C128; factors F64 / C128; full SVD per face.
 *   PREC_MIXED: Xhat FP32 (real M); factors F32; randomized range finder
 *               with the caller's Gaussian omega, power iteration, FP64
 *               shifted Cholesky-QR, FP64 core SVD.  ENERGY decides each
 *               rank from the estimate ||Xhat_f - Q B||^2 + sum_{j>k} s_j(B)^2
 *               (Q the basis, B = Q^H Xhat_f; a residual pass with the
 *               projection).  With opts->certify, a pass after the factors
 *               computes cert from the stored factors (see tsvdm_factors).
 *               Xhat C64 (the stored half spectrum of the DFT of a real
 *               tensor, or any complex faces): factors C64, the same steps in
 *               complex arithmetic with the real omega (adjoints are
 *               conjugate transposes, the QR Hermitian, the core a Hermitian
 *               eigensolver), sketch width k + oversample up to 48, m up to
 *               32768.  From 32 faces on, half of them run on a stream the
 *               library creates per device (as tsvdm_truncate_learned's),
 *               joined back to `stream` with events; under stream capture
 *               that happens only if an earlier call created it (else one
 *               stream, same results).  Complex truncations issued at once
 *               from several host threads on one device must be serialized.
 *   PREC_F64_RAND: Xhat FP64 (real M); factors F64; the PREC_MIXED steps
 *               with every product in FP64 (FP64 MFMA, FP64 panels), the
 *               residual ||Xhat_f - Q B||^2 taken as ||Xhat_f||^2 - ||B||^2;
 *               finite data below 1e100 in magnitude.
 * out->kmax >= the largest rank that can be returned (k for FIXED, the cap
 * for ENERGY).  The error of the approximation in the original domain is
 * sqrt(sum_f w_f cert_f^2) (w_f = 1, or 2 for DFT faces 0 < f < n3/2). */
tsvdm_status tsvdm_truncate(const tsvdm_tensor *Xhat, const tsvdm_truncate_opts *opts,
                            tsvdm_factors *out, void *workspace, size_t workspace_bytes,
                            void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * tsvdm_truncate with PREC_MIXED on a real F32 Xhat and no workspace
 * argument.  Its scratch is a static device array of tsvdm_noalloc_scratch_bytes() bytes (32 MiB), one
 * per GPU the library runs on, held until the process ends; the call itself
 * allocates nothing.  The faces are processed in consecutive groups whose
 * workspace fits the array (the results equal tsvdm_truncate's bit for bit).
 * Returns TSVDM_EWORKSPACE if a single face needs more scratch than the array
 * holds, TSVDM_EUNSUPPORTED for other precisions and complex faces; other
 * arguments as for
 * tsvdm_truncate.  Every call on one GPU uses that GPU's one array: calls
 * that overlap on the same GPU (other streams, other threads) race and give
 * wrong results; serialise them.  Nothing needs clearing between calls (every
 * scratch value is written before it is read). */
tsvdm_status tsvdm_truncate_noalloc(const tsvdm_tensor *Xhat, const tsvdm_truncate_opts *opts,
                                    tsvdm_factors *out, void *stream);

/* Size of the static scratch array of tsvdm_truncate_noalloc, in bytes. */
size_t tsvdm_noalloc_scratch_bytes(void);

/* Workspace bytes tsvdm_apply needs: the transformed right-hand sides and,
 * for compute = F32 or BF16, a copy of Vhat with the rows j + ell*k of each
 * block row j contiguous in k. */
size_t tsvdm_apply_workspace_size(const tsvdm_mdesc *M, const tsvdm_factors *F, int64_t ell,
                                  int64_t q, int64_t nrhs, int32_t compute);

/* y = A_hat x with A_hat = M_E[T] (Sec. 3, map M_E, generic placement with
 * p = ell*q) and T = That x_3 M^{-1}, That_f = Uhat_f diag(S_f) Vhat_f^H from
 * the factors F (only the leading ranks[f] triplets).  A_hat is never formed:
 *   xt_k = tube transform of the k-th block row of x by conj(M),
 *   Z_f[r, j, c] = sum_k conj(Vhat_f[j + ell*k, r]) xt_k[f, c],
 *   y_j[:, c] = sum_f Uhat_f diag(S_f) Z_f[:, j, c].
 * x: (q*n3) x nrhs, column major (ldx), y: (ell*m) x nrhs (ldy), both real of
 * the compute type's precision: FP32 for compute = F32 (or BF16), FP64 for
 * compute = F64.  Factor precision must match (F32/C64 or F64/C128).
 * F32 runs the per-face products on FP32 matrix cores, BF16 on BF16 matrix
 * cores (operands, and Z between the two products, rounded to BF16; FP32
 * accumulation), F64 on FP64 matrix cores, when every per-face buffer is
 * under 2 GiB; otherwise on the vector units (BF16 then rounds the operands
 * only).  Asynchronous on stream; launches kernels only. */
tsvdm_status tsvdm_apply(const tsvdm_mdesc *M, const tsvdm_factors *F, int64_t ell, int64_t q,
                         int64_t nrhs, const void *x, int64_t ldx, void *y, int64_t ldy,
                         int32_t compute, void *workspace, size_t workspace_bytes, void *stream);

/* Per-kernel timing (diagnostics).  While enabled, every kernel launch the
 * library makes is bracketed by two HIP events recorded on the launch
 * stream, so one kernel inside a multi-kernel call can be timed on its own
 * stream.  Enabling starts a fresh window.  Costs one flag test per launch
 * when disabled (the default).  Host-side only; not thread-safe with
 * respect to enabling/reading while other threads launch. */
tsvdm_status tsvdm_timing_enable(int32_t on);

/* Waits for the recorded events, reduces them per kernel name and returns
 * the number of distinct names. */
int32_t tsvdm_timing_count(void);

/* Name, number of launches and summed milliseconds of entry i (0-based, after
 * tsvdm_timing_count).  The name stays valid until the next enable or count. */
tsvdm_status tsvdm_timing_get(int32_t i, const char **name, int32_t *launches, double *total_ms);

/* ---------------------------------------------------------------- batches
 * Facewise truncation of an uneven batch: nmat dense transform-domain tensors
 * Xhat[i] (FP32, m_i x p_i x nf_i, each face with m_i <= 64 rows, at most 2^28
 * elements per face and p_i < 2^24), each with
 * its own factors F[i] (F32 U and V, kmax_i columns).  This is the truncation
 * step of Algorithm alg:strategy for many independent inputs at once (e.g.
 * the Kronecker-sum matrices of Sec. 3 mapped by T_E and transformed).
 *
 * Per face, with X = Xhat_f (m x p):
 *   1. G = X X^T in FP64 (every product of FP32 values is exact in FP64);
 *   2. rank-revealing pivoted Cholesky P G P^T = R^T R + S, stopped when
 *      trace(S) <= 1e-3 tau^2 trace(G) (ENERGY) or 1e-15 trace(G) (FIXED), or
 *      after 32 steps; Jacobi eigensolver of R R^T;
 *   3. rank k_f by opts->rank_mode, with the discarded energy counted as
 *      sum_{j>k} lambda_j(R R^T) + trace(S), an upper bound on the exact
 *      discarded energy; cert_f = its square root;
 *   4. U = P^T R^T U_H diag(sigma)^{-1} (orthonormal), V = X^T U diag(sigma)^{-1}.
 * The result is the truncated SVD of the face up to trace(S).
 *
 * Usage: size the workspace, create a plan (host work and one synchronous
 * upload of the face table into the workspace), optionally autotune it, then
 * launch with tsvdm_truncate_batched as often as needed (asynchronous; no
 * allocation, no host-device copy: safe under stream capture).  The plan
 * keeps the device pointers it was created with. */
typedef struct tsvdm_batched_plan_s tsvdm_batched_plan;

/* Workspace bytes for the batch (shapes only). 0 if the arguments are invalid. */
size_t tsvdm_batched_workspace_size(int32_t nmat, const tsvdm_tensor *Xhat);

/* Validates the batch (host arrays Xhat[nmat], F[nmat] of device pointers),
 * orders the faces by cost (largest first) and writes the face table into the
 * caller's workspace (synchronous copy).  opts: rank_mode, k (FIXED rank or
 * ENERGY cap, <= F[i].kmax and <= 32), tau, max_sweeps; the other fields are
 * ignored.  *plan is a host object released with tsvdm_batched_plan_destroy. */
tsvdm_status tsvdm_batched_plan_create(int32_t nmat, const tsvdm_tensor *Xhat,
                                       const tsvdm_truncate_opts *opts, const tsvdm_factors *F,
                                       void *workspace, size_t workspace_bytes,
                                       tsvdm_batched_plan **plan);

/* Launches the batch on `stream`: a queue reset, the persistent Gram kernel,
 * the per-face core, the persistent V kernel.  Outputs as for tsvdm_truncate. */
tsvdm_status tsvdm_truncate_batched(const tsvdm_batched_plan *plan, void *stream);

/* Times the candidate launch configurations of the two persistent kernels on
 * this plan (it runs the batch several times on `stream` and synchronizes),
 * keeps the fastest in the plan and in a process-wide table keyed by the
 * batch signature, which later plans of the same signature start from. */
tsvdm_status tsvdm_batched_autotune(tsvdm_batched_plan *plan, void *stream);

/* The plan's configuration: cfg[0] Gram workgroups (of four wavefronts, one
 * face each at a time) per CU, cfg[1] Gram columns per prefetch step (16 or
 * 32), cfg[2] V workgroups per CU, cfg[3] 1 if it came from the autotuner
 * (here or through the table). */
tsvdm_status tsvdm_batched_config(const tsvdm_batched_plan *plan, int32_t cfg[4]);

/* Sets the plan's launch configuration (cfg[0..2] as above; cfg[3] ignored,
 * the result reads as not tuned).  1 <= cfg[0], cfg[2] <= 16, cfg[1] 16 or
 * 32, else TSVDM_EINVAL and the plan is unchanged.  The results do not depend
 * on the configuration. */
tsvdm_status tsvdm_batched_set_config(tsvdm_batched_plan *plan, const int32_t cfg[4]);

/* Releases the host plan (the workspace stays the caller's). NULL is allowed. */
void tsvdm_batched_plan_destroy(tsvdm_batched_plan *plan);

/* Persistent autotune table.  The process-wide table of tuned configurations
 * (filled by tsvdm_batched_autotune, keyed by the batch signature and the
 * device's CU count) is written to / merged from a text file:
 *   line 1 "tsvdm-autotune 1", then one line per entry:
 *   "<key, 16 hex digits> <cfg[0]> <cfg[1]> <cfg[2]>".
 * Save writes a temporary file and renames it over `path`.  Load validates the
 * whole file (header, ranges as for tsvdm_batched_set_config) before merging
 * any entry (TSVDM_EINVAL with the line otherwise); *n_entries (may be NULL)
 * receives the number merged.  Plans created afterwards start from a matching
 * entry and read as tuned.  Clear empties the table.  Host-only, thread-safe. */
tsvdm_status tsvdm_autotune_save(const char *path);
tsvdm_status tsvdm_autotune_load(const char *path, int32_t *n_entries);
void tsvdm_autotune_clear(void);

/* ---------------------------------------------------------------- rank predictor
 * A multilayer perceptron 32 -> 64 -> 64 -> 2 (ReLU hidden layers, linear
 * output) that predicts, per transform-domain face, (k/32, l/48): the rank and
 * the sketch width of the randomized truncation (step 3 of Algorithm
 * alg:strategy), from the features log10(s_j / s_1), j = 1..32, of a 32-column
 * sketch of the face (tsvdm_rank_features).  Half precision weights, inputs
 * and hidden activations; FP32 accumulation.
 * Parameters, flat (6402 values): W1 (64 x 32, row major), b1 (64),
 * W2 (64 x 64), b2 (64), W3 (2 x 64), b3 (2).  Half buffers hold IEEE binary16
 * bit patterns.  All pointers are device pointers owned by the caller. */

/* Number of parameters (6402). */
int64_t tsvdm_mlp_nparams(void);

/* y (n x 2, FP32, row major) = MLP(x) for the n x 32 half inputs x (row major). */
tsvdm_status tsvdm_mlp_forward(const uint16_t *w16, const uint16_t *x, int64_t n, float *y,
                               void *stream);

/* Workspace bytes for tsvdm_mlp_gradient / tsvdm_mlp_train_step on n samples. */
size_t tsvdm_mlp_train_workspace_size(int64_t n);

/* grad (6402, FP32) of loss = sum_s |MLP(x_s) - t_s|^2 / (2n) at the half
 * weights w16 (forward as tsvdm_mlp_forward, backward in FP32); *loss (device,
 * may be NULL) receives the loss.  target: n x 2 FP32, row major. */
tsvdm_status tsvdm_mlp_gradient(const uint16_t *w16, const uint16_t *x, const float *target, int64_t n,
                                float *grad, float *loss, void *workspace, size_t workspace_bytes,
                                void *stream);

/* One training step on the batch (x, target): the gradient at w16, then Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias correction for step >= 1) on the FP32
 * master weights w32 with moments m, v; w16 is refreshed from w32. */
tsvdm_status tsvdm_mlp_train_step(float *w32, uint16_t *w16, float *m, float *v, int32_t step, float lr,
                                  const uint16_t *x, const float *target, int64_t n, float *loss,
                                  void *workspace, size_t workspace_bytes, void *stream);

/* Checkpoint of the predictor's training state (resume a training run): a
 * versioned little-endian binary file, header {magic "TSVDMMLP", uint32 version
 * = 1, uint32 nparams, int32 step, uint32 0}, then the half weights w16, the
 * FP32 master weights w32 and the Adam moments m, v (nparams values each), then
 * the CRC-32 (IEEE 802.3) of all preceding bytes.  The buffers are device (or
 * host) pointers, copied synchronously.  Load validates magic, version,
 * parameter count, length and CRC (TSVDM_EINVAL with a message otherwise)
 * before writing anything. */
tsvdm_status tsvdm_mlp_save(const char *path, const uint16_t *w16, const float *w32, const float *m, const float *v,
                            int32_t step);
tsvdm_status tsvdm_mlp_load(const char *path, uint16_t *w16, float *w32, float *m, float *v, int32_t *step);

/* b[i] = a[i] rounded to half (nearest even), i < n. */
tsvdm_status tsvdm_f32_to_f16(const float *a, uint16_t *b, int64_t n, void *stream);

/* Workspace bytes for tsvdm_rank_features (shapes only); 0 if invalid. */
size_t tsvdm_rank_features_workspace_size(const tsvdm_tensor *Xhat);

/* Predictor inputs of every face of the dense FP32 transform-domain tensor
 * Xhat (m >= 32, p >= 40): the singular values s of the sketch
 * Y = Xhat_f omega[:, :32] (BF16 products, FP32 accumulation; FP64 Gram and
 * Jacobi eigenvalues), features[f][j] = log10(s_j / s_1) (0 when s_1 = 0, at
 * least -30), j < 32, as halves (nf x 32, row major).  omega: p x 32 or wider
 * (the first 32 columns are used), column major FP32. */
tsvdm_status tsvdm_rank_features(const tsvdm_tensor *Xhat, const float *omega, uint16_t *features,
                                 void *workspace, size_t workspace_bytes, void *stream);

/* Workspace bytes for tsvdm_truncate_learned (shapes only); 0 if invalid. */
size_t tsvdm_truncate_learned_workspace_size(const tsvdm_tensor *Xhat);

/* Mixed-precision truncation (as tsvdm_truncate with PREC_MIXED and the
 * energy rule) whose rank cap and sketch width are chosen per face by the
 * predictor w16 (the learned part of step 3 of Algorithm alg:strategy):
 * features, prediction (k/32, l/48) -> kh = ceil(32 k) in 1..32, lw =
 * ceil(48 l) + 1; the face takes the first bucket (width 16, 32, 40 with rank
 * caps 13, 26, 32) whose width is at least lw and cap at least kh, and the
 * energy rule's cap min(bucket cap, kh + 2).  The feature sketch
 * Xhat_f omega[:, :32] is the first sketch of the width-16 and width-32
 * buckets.  Faces whose certified error then exceeds tau ||Xhat_f|| (and did
 * not already run at width 40 with cap 32) are truncated again there.  widths
 * (nf, device) receives each face's final width.  opts: ENERGY, tau, omega
 * (p x 40), power_iters, max_sweeps.  out->kmax >= 32; cert and fro are
 * required.  Launches kernels only (bucket sizes stay on the device): it can be
 * captured in a graph.  The three buckets run on three streams the library
 * creates per device on first use (so the first call on a device must not be
 * under stream capture; it returns an error if it is) and joins back to
 * `stream` with events; learned truncations issued at once from several host
 * threads on one device share those streams and must be serialized by the
 * caller. */
tsvdm_status tsvdm_truncate_learned(const tsvdm_tensor *Xhat, const tsvdm_truncate_opts *opts,
                                    const uint16_t *w16, tsvdm_factors *out, int32_t *widths,
                                    void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TSVDM_H */
