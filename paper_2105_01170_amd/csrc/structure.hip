// Structured placements of a block matrix (Sec. 3, block matrix to tensor
// mapping): A ((ell m) x (q n)) with ell x q blocks of size m x n, p distinct
// blocks A_k, block (i, j) equal to A_{k(i,j)} or zero (k = -1).  E_k holds
// 1/sqrt(eta_k) where A_k occurs (eta_k occurrences, so ||E_k||_F = 1, eq.
// fnormw); the maps are
//   T_E[A](:, k, :) = sqrt(eta_k) twist(A_k),
//   M_E[X] = sum_k E_k kron sq(X(:, k, :)),
// so block (i, j) of M_E[X] is X(:, k(i,j), :) / sqrt(eta_k) (zero if k = -1),
// and M_E[T_E[A]] = A for a matrix with that structure.
//
// The placement is a host plan with a small device table in the caller's
// workspace: the block map k(i, j), a representative block of every k (the
// first occurrence in row-major block order: smallest block row, then
// column) and the weights sqrt(eta_k), 1/sqrt(eta_k) (formed on the host in
// IEEE double precision).  T_E is a gather kernel into a dense m x p x n
// tensor (p is at most ell q, usually far smaller for a structured matrix);
// M_E a scatter into the block matrix.  The structured apply forms, per
// stored face, the factor V of the generic placement,
//   Vg[i + ell j, r] = Vhat[k(i,j), r] / sqrt(eta_k)   (zero if k = -1),
// so that M_E[T] = M_Eg[Tg] with Tg = That_g x_3 M^{-1}, That_g,f = Uhat_f
// S_f Vg_f^H, and runs the generic fused apply on it.
#include "common.h"

#include <math.h>

#include <vector>

using namespace tsvdm;

struct tsvdm_placement_s {
    int64_t ell, q, p;
    std::vector<int32_t> eta;  // host copy of the occurrence counts
    int32_t *blk;              // device: k(i, j) at i + ell j
    int32_t *rep;              // device: representative block (i_k, j_k) at 2k, 2k+1
    double *w, *winv;          // device: sqrt(eta_k), 1 / sqrt(eta_k)
};

namespace {

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t table_bytes(int64_t ell, int64_t q, int64_t p) {
    return al256(sizeof(int32_t) * (size_t)(ell * q)) + al256(sizeof(int32_t) * 2 * (size_t)p) +
           2 * al256(sizeof(double) * (size_t)p);
}

// X(a, k, t) = w_k A(i_k m + a, j_k n + t); one thread per element, a fastest
template <typename T>
__global__ void k_tensor_from_blockmat_E(const T *__restrict__ A, int64_t lda, int64_t m, int64_t n, int64_t p,
                                         const int32_t *__restrict__ rep, const double *__restrict__ w,
                                         T *__restrict__ X) {
    const int64_t tot = m * p * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = e % m, kt = e / m, k = kt % p, t = kt / p;
        const int64_t i = rep[2 * k], j = rep[2 * k + 1];
        X[e] = (T)(w[k] * (double)A[(i * m + a) + lda * (j * n + t)]);
    }
}

// A(i m + a, j n + t) = X(a, k(i,j), t) / sqrt(eta_k), or 0; one thread per
// element of the (ell m) x (q n) block matrix, rows fastest
template <typename T>
__global__ void k_blockmat_from_tensor_E(const T *__restrict__ X, int64_t m, int64_t n, int64_t p, int64_t ell,
                                         int64_t q, const int32_t *__restrict__ blk,
                                         const double *__restrict__ winv, T *__restrict__ A, int64_t lda) {
    const int64_t rows = ell * m, tot = rows * q * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e % rows, c = e / rows;
        const int64_t i = r / m, a = r % m, j = c / n, t = c % n;
        const int k = blk[i + ell * j];
        A[r + lda * c] = k >= 0 ? (T)(winv[k] * (double)X[a + m * k + m * p * t]) : T(0);
    }
}

// Vg(i + ell j, r, f) = V(k(i,j), r, f) / sqrt(eta_k) or 0, E real components
// per element (1 real, 2 complex)
template <typename T, int E>
__global__ void k_vgather_E(const T *__restrict__ V, int64_t p, int64_t ell, int64_t q, int64_t kmax, int64_t nf,
                            const int32_t *__restrict__ blk, const double *__restrict__ winv, T *__restrict__ Vg) {
    const int64_t pg = ell * q, tot = pg * kmax * nf;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = e % pg, rf = e / pg;
        const int k = blk[b];
#pragma unroll
        for (int c = 0; c < E; ++c)
            Vg[E * e + c] = k >= 0 ? (T)(winv[k] * (double)V[E * (k + p * rf) + c]) : T(0);
    }
}

unsigned grid_of(int64_t tot) {
    const int64_t g = (tot + 255) / 256;
    return (unsigned)(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

#define FAILS(code, ...)        \
    do {                        \
        set_error(__VA_ARGS__); \
        return (code);          \
    } while (0)

}  // namespace

extern "C" {

tsvdm_status tsvdm_block_structure(int32_t kind, int64_t ell, int64_t q, int64_t b, int32_t *block_of,
                                   int64_t *p_out) {
    if (!block_of || !p_out) FAILS(TSVDM_EINVAL, "block_of and p are required");
    if (ell < 1 || q < 1 || ell * q > (int64_t)1 << 30) FAILS(TSVDM_EINVAL, "block grid %lld x %lld", (long long)ell, (long long)q);
    int64_t p = 0;
    auto at = [&](int64_t i, int64_t j) -> int32_t & { return block_of[i + ell * j]; };
    for (int64_t e = 0; e < ell * q; ++e) block_of[e] = -1;
    switch (kind) {
        case TSVDM_PLACE_GENERIC:  // k = i + ell j
            for (int64_t j = 0; j < q; ++j)
                for (int64_t i = 0; i < ell; ++i) at(i, j) = (int32_t)p++;
            break;
        case TSVDM_PLACE_DIAGONAL:
            if (ell != q) FAILS(TSVDM_EINVAL, "a block-diagonal placement needs ell == q");
            for (int64_t i = 0; i < ell; ++i) at(i, i) = (int32_t)p++;
            break;
        case TSVDM_PLACE_BANDED:  // |i - j| <= b, every block distinct, column by column
            if (b < 0) FAILS(TSVDM_EINVAL, "block semibandwidth must be >= 0");
            for (int64_t j = 0; j < q; ++j)
                for (int64_t i = 0; i < ell; ++i)
                    if (i - j <= b && j - i <= b) at(i, j) = (int32_t)p++;
            break;
        case TSVDM_PLACE_BANDED_SYM:  // (i, j) and (j, i) share, numbered over i <= j column by column
            if (b < 0) FAILS(TSVDM_EINVAL, "block semibandwidth must be >= 0");
            if (ell != q) FAILS(TSVDM_EINVAL, "a block-symmetric placement needs ell == q");
            for (int64_t j = 0; j < q; ++j)
                for (int64_t i = 0; i <= j; ++i)
                    if (j - i <= b) {
                        at(i, j) = (int32_t)p;
                        at(j, i) = (int32_t)p;
                        ++p;
                    }
            break;
        case TSVDM_PLACE_TOEPLITZ:  // main and lower diagonals 0..ell-1, then upper 1..q-1
            for (int64_t j = 0; j < q; ++j)
                for (int64_t i = 0; i < ell; ++i) at(i, j) = (int32_t)(i >= j ? i - j : ell - 1 + (j - i));
            p = ell + q - 1;
            break;
        case TSVDM_PLACE_TOEPLITZ_SYM:  // k = |i - j|
            for (int64_t j = 0; j < q; ++j)
                for (int64_t i = 0; i < ell; ++i) at(i, j) = (int32_t)(i >= j ? i - j : j - i);
            p = ell > q ? ell : q;
            break;
        case TSVDM_PLACE_HANKEL:  // k = i + j
            for (int64_t j = 0; j < q; ++j)
                for (int64_t i = 0; i < ell; ++i) at(i, j) = (int32_t)(i + j);
            p = ell + q - 1;
            break;
        default:
            FAILS(TSVDM_EINVAL, "unknown block structure %d", kind);
    }
    *p_out = p;
    return TSVDM_OK;
}

size_t tsvdm_placement_workspace_size(int64_t ell, int64_t q, int64_t p) {
    if (ell < 1 || q < 1 || p < 1 || p > ell * q) return 0;
    return table_bytes(ell, q, p);
}

tsvdm_status tsvdm_placement_create(int64_t ell, int64_t q, int64_t p, const int32_t *block_of, void *workspace,
                                    size_t workspace_bytes, tsvdm_placement **out) {
    if (!out) FAILS(TSVDM_EINVAL, "out is NULL");
    *out = nullptr;
    if (ell < 1 || q < 1 || ell * q > (int64_t)1 << 30) FAILS(TSVDM_EINVAL, "block grid %lld x %lld", (long long)ell, (long long)q);
    if (p < 1 || p > ell * q) FAILS(TSVDM_EINVAL, "p = %lld must be in 1..ell*q", (long long)p);
    if (!block_of) FAILS(TSVDM_EINVAL, "block_of is NULL");
    const size_t need = table_bytes(ell, q, p);
    if (!workspace || workspace_bytes < need)
        FAILS(TSVDM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    std::vector<int32_t> eta(p, 0), rep(2 * p, -1);
    // representatives in row-major block order: smallest block row, then column
    for (int64_t i = 0; i < ell; ++i)
        for (int64_t j = 0; j < q; ++j) {
            const int32_t k = block_of[i + ell * j];
            if (k < -1 || k >= p) FAILS(TSVDM_EINVAL, "block_of[%lld] = %d outside -1..p-1", (long long)(i + ell * j), k);
            if (k < 0) continue;
            if (eta[k]++ == 0) {
                rep[2 * k] = (int32_t)i;
                rep[2 * k + 1] = (int32_t)j;
            }
        }
    std::vector<double> w(p), winv(p);
    for (int64_t k = 0; k < p; ++k) {
        if (eta[k] == 0) FAILS(TSVDM_EINVAL, "distinct block %lld occurs nowhere", (long long)k);
        w[k] = std::sqrt((double)eta[k]);
        winv[k] = 1.0 / w[k];
    }
    char *base = reinterpret_cast<char *>(workspace);
    auto *pl = new tsvdm_placement_s;
    pl->ell = ell;
    pl->q = q;
    pl->p = p;
    pl->eta = eta;
    size_t off = 0;
    pl->blk = reinterpret_cast<int32_t *>(base + off);
    off += al256(sizeof(int32_t) * (size_t)(ell * q));
    pl->rep = reinterpret_cast<int32_t *>(base + off);
    off += al256(sizeof(int32_t) * 2 * (size_t)p);
    pl->w = reinterpret_cast<double *>(base + off);
    off += al256(sizeof(double) * (size_t)p);
    pl->winv = reinterpret_cast<double *>(base + off);
    hipError_t e = hipMemcpy(pl->blk, block_of, sizeof(int32_t) * (size_t)(ell * q), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(pl->rep, rep.data(), sizeof(int32_t) * 2 * (size_t)p, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(pl->w, w.data(), sizeof(double) * (size_t)p, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(pl->winv, winv.data(), sizeof(double) * (size_t)p, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete pl;
        return hip_check(e, "tsvdm_placement_create: table upload");
    }
    *out = pl;
    return TSVDM_OK;
}

tsvdm_status tsvdm_placement_eta(const tsvdm_placement *pl, int32_t *eta) {
    if (!pl || !eta) FAILS(TSVDM_EINVAL, "placement and eta are required");
    for (int64_t k = 0; k < pl->p; ++k) eta[k] = pl->eta[k];
    return TSVDM_OK;
}

void tsvdm_placement_destroy(tsvdm_placement *pl) { delete pl; }

tsvdm_status tsvdm_tensor_from_blockmat_E(const tsvdm_placement *pl, const void *A, int64_t lda, int32_t dtype,
                                          int64_t m, int64_t n, void *X, void *stream) {
    if (!pl || !A || !X) FAILS(TSVDM_EINVAL, "placement, A and X are required");
    if (m < 1 || n < 1) FAILS(TSVDM_EINVAL, "block size %lld x %lld", (long long)m, (long long)n);
    if (lda < pl->ell * m) FAILS(TSVDM_EINVAL, "lda (%lld) < ell*m (%lld)", (long long)lda, (long long)(pl->ell * m));
    if (dtype != TSVDM_F32 && dtype != TSVDM_F64) FAILS(TSVDM_EINVAL, "dtype must be F32 or F64");
    hipStream_t s = (hipStream_t)stream;
    const int64_t tot = m * pl->p * n;
    if (dtype == TSVDM_F64)
        TSVDM_LAUNCH("tensor_from_blockmat_E", k_tensor_from_blockmat_E<double>, dim3(grid_of(tot)), dim3(256), 0, s,
                     reinterpret_cast<const double *>(A), lda, m, n, pl->p, (const int32_t *)pl->rep,
                     (const double *)pl->w, reinterpret_cast<double *>(X));
    else
        TSVDM_LAUNCH("tensor_from_blockmat_E", k_tensor_from_blockmat_E<float>, dim3(grid_of(tot)), dim3(256), 0, s,
                     reinterpret_cast<const float *>(A), lda, m, n, pl->p, (const int32_t *)pl->rep,
                     (const double *)pl->w, reinterpret_cast<float *>(X));
    TSVDM_LAUNCH_CHECK("tensor_from_blockmat_E");
    return TSVDM_OK;
}

tsvdm_status tsvdm_blockmat_from_tensor_E(const tsvdm_placement *pl, const void *X, int32_t dtype, int64_t m,
                                          int64_t n, void *A, int64_t lda, void *stream) {
    if (!pl || !A || !X) FAILS(TSVDM_EINVAL, "placement, X and A are required");
    if (m < 1 || n < 1) FAILS(TSVDM_EINVAL, "block size %lld x %lld", (long long)m, (long long)n);
    if (lda < pl->ell * m) FAILS(TSVDM_EINVAL, "lda (%lld) < ell*m (%lld)", (long long)lda, (long long)(pl->ell * m));
    if (dtype != TSVDM_F32 && dtype != TSVDM_F64) FAILS(TSVDM_EINVAL, "dtype must be F32 or F64");
    hipStream_t s = (hipStream_t)stream;
    const int64_t tot = pl->ell * m * pl->q * n;
    if (dtype == TSVDM_F64)
        TSVDM_LAUNCH("blockmat_from_tensor_E", k_blockmat_from_tensor_E<double>, dim3(grid_of(tot)), dim3(256), 0, s,
                     reinterpret_cast<const double *>(X), m, n, pl->p, pl->ell, pl->q, (const int32_t *)pl->blk,
                     (const double *)pl->winv, reinterpret_cast<double *>(A), lda);
    else
        TSVDM_LAUNCH("blockmat_from_tensor_E", k_blockmat_from_tensor_E<float>, dim3(grid_of(tot)), dim3(256), 0, s,
                     reinterpret_cast<const float *>(X), m, n, pl->p, pl->ell, pl->q, (const int32_t *)pl->blk,
                     (const double *)pl->winv, reinterpret_cast<float *>(A), lda);
    TSVDM_LAUNCH_CHECK("blockmat_from_tensor_E");
    return TSVDM_OK;
}

// the generic-placement factors the structured apply runs on
static void generic_factors(const tsvdm_placement *pl, const tsvdm_factors *F, void *Vg, tsvdm_factors *G) {
    *G = *F;
    G->p = pl->ell * pl->q;
    G->V = Vg;
}

static size_t elem_bytes(int32_t dtype) {
    return dtype == TSVDM_F32 ? 4 : dtype == TSVDM_F64 || dtype == TSVDM_C64 ? 8 : 16;
}

size_t tsvdm_apply_E_workspace_size(const tsvdm_placement *pl, const tsvdm_mdesc *M, const tsvdm_factors *F,
                                    int64_t nrhs, int32_t compute) {
    if (!pl || !M || !F || F->p != pl->p) return 0;
    const size_t vg = al256(elem_bytes(F->dtype) * (size_t)(pl->ell * pl->q) * F->kmax * F->nf);
    tsvdm_factors G;
    generic_factors(pl, F, reinterpret_cast<void *>(256), &G);
    const size_t ap = tsvdm_apply_workspace_size(M, &G, pl->ell, pl->q, nrhs, compute);
    return ap ? vg + ap : 0;
}

tsvdm_status tsvdm_apply_E(const tsvdm_placement *pl, const tsvdm_mdesc *M, const tsvdm_factors *F, int64_t nrhs,
                           const void *x, int64_t ldx, void *y, int64_t ldy, int32_t compute, void *workspace,
                           size_t workspace_bytes, void *stream) {
    if (!pl || !M || !F) FAILS(TSVDM_EINVAL, "placement, M and F are required");
    if (F->p != pl->p) FAILS(TSVDM_EINVAL, "factor p (%lld) != the placement's p (%lld)", (long long)F->p, (long long)pl->p);
    if (!F->V) FAILS(TSVDM_EINVAL, "factor pointers must be set");
    const size_t need = tsvdm_apply_E_workspace_size(pl, M, F, nrhs, compute);
    if (need == 0) {
        tsvdm_factors G;
        generic_factors(pl, F, reinterpret_cast<void *>(256), &G);
        tsvdm_apply_workspace_size(M, &G, pl->ell, pl->q, nrhs, compute);  // sets the message
        return TSVDM_EINVAL;
    }
    if (!workspace || workspace_bytes < need)
        FAILS(TSVDM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    hipStream_t s = (hipStream_t)stream;
    char *base = reinterpret_cast<char *>(workspace);
    const size_t vg = al256(elem_bytes(F->dtype) * (size_t)(pl->ell * pl->q) * F->kmax * F->nf);
    const int64_t tot = pl->ell * pl->q * F->kmax * F->nf;
    switch (F->dtype) {
        case TSVDM_F32:
            TSVDM_LAUNCH("apply_E_vgather", (k_vgather_E<float, 1>), dim3(grid_of(tot)), dim3(256), 0, s,
                         reinterpret_cast<const float *>(F->V), F->p, pl->ell, pl->q, F->kmax, F->nf,
                         (const int32_t *)pl->blk, (const double *)pl->winv, reinterpret_cast<float *>(base));
            break;
        case TSVDM_F64:
            TSVDM_LAUNCH("apply_E_vgather", (k_vgather_E<double, 1>), dim3(grid_of(tot)), dim3(256), 0, s,
                         reinterpret_cast<const double *>(F->V), F->p, pl->ell, pl->q, F->kmax, F->nf,
                         (const int32_t *)pl->blk, (const double *)pl->winv, reinterpret_cast<double *>(base));
            break;
        case TSVDM_C64:
            TSVDM_LAUNCH("apply_E_vgather", (k_vgather_E<float, 2>), dim3(grid_of(tot)), dim3(256), 0, s,
                         reinterpret_cast<const float *>(F->V), F->p, pl->ell, pl->q, F->kmax, F->nf,
                         (const int32_t *)pl->blk, (const double *)pl->winv, reinterpret_cast<float *>(base));
            break;
        default:
            TSVDM_LAUNCH("apply_E_vgather", (k_vgather_E<double, 2>), dim3(grid_of(tot)), dim3(256), 0, s,
                         reinterpret_cast<const double *>(F->V), F->p, pl->ell, pl->q, F->kmax, F->nf,
                         (const int32_t *)pl->blk, (const double *)pl->winv, reinterpret_cast<double *>(base));
            break;
    }
    TSVDM_LAUNCH_CHECK("apply_E_vgather");
    tsvdm_factors G;
    generic_factors(pl, F, base, &G);
    return tsvdm_apply(M, &G, pl->ell, pl->q, nrhs, x, ldx, y, ldy, compute, base + vg, workspace_bytes - vg,
                       stream);
}

}  // extern "C"

namespace tsvdm {
void placement_tables(const tsvdm_placement *pl, int64_t *ell, int64_t *q, int64_t *p, const int32_t **blk,
                      const double **winv) {
    *ell = pl->ell;
    *q = pl->q;
    *p = pl->p;
    *blk = pl->blk;
    *winv = pl->winv;
}
}  // namespace tsvdm

namespace {
// X(a, k, t) = sqrt(eta_k) B(a, t, k) from the distinct blocks stacked m x n x p:
// a workgroup copies whole columns kt = k + p t of X (one division per column,
// contiguous loads and stores), grid-stride over the p n columns
template <typename T>
__global__ __launch_bounds__(256) void k_tensor_from_blocks_E(const T *__restrict__ B, int64_t m, int64_t n,
                                                              int64_t p, const double *__restrict__ w,
                                                              T *__restrict__ X) {
    const int64_t ncol = p * n;
    for (int64_t kt = blockIdx.x; kt < ncol; kt += gridDim.x) {
        const int64_t k = kt % p, t = kt / p;
        const double wk = w[k];
        const T *src = B + m * t + m * n * k;
        T *dst = X + m * kt;
        for (int64_t a = threadIdx.x; a < m; a += 256) dst[a] = (T)(wk * (double)src[a]);
    }
}
inline unsigned columns_grid(int64_t ncol) { return (unsigned)(ncol < 1 ? 1 : ncol < (1 << 20) ? ncol : (1 << 20)); }
}  // namespace

extern "C" tsvdm_status tsvdm_tensor_from_blocks_E(const tsvdm_placement *pl, const void *blocks, int32_t dtype,
                                                   int64_t m, int64_t n, void *X, void *stream) {
    if (!pl || !blocks || !X) FAILS(TSVDM_EINVAL, "placement, blocks and X are required");
    if (m < 1 || n < 1) FAILS(TSVDM_EINVAL, "block size %lld x %lld", (long long)m, (long long)n);
    if (dtype != TSVDM_F32 && dtype != TSVDM_F64) FAILS(TSVDM_EINVAL, "dtype must be F32 or F64");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == TSVDM_F64)
        TSVDM_LAUNCH("tensor_from_blocks_E", k_tensor_from_blocks_E<double>, dim3(columns_grid(pl->p * n)), dim3(256), 0, s,
                     reinterpret_cast<const double *>(blocks), m, n, pl->p, (const double *)pl->w,
                     reinterpret_cast<double *>(X));
    else
        TSVDM_LAUNCH("tensor_from_blocks_E", k_tensor_from_blocks_E<float>, dim3(columns_grid(pl->p * n)), dim3(256), 0, s,
                     reinterpret_cast<const float *>(blocks), m, n, pl->p, (const double *)pl->w,
                     reinterpret_cast<float *>(X));
    TSVDM_LAUNCH_CHECK("tensor_from_blocks_E");
    return TSVDM_OK;
}
