// Two-sided compression that preserves positive semidefiniteness (Sec. 5.1).
//
// For a symmetric positive semidefinite block matrix A (ell = q, m = n) the
// mode-1 and mode-3 unfoldings of X = T_E[A] (m x p x m) have the same range,
// so one factor U (m x r) compresses both modes:
//   G = X x_1 U^T x_3 U^T,  G(:, b, :) = U^T sq(X(:, b, :)) U   (r x p x r),
//   T = G x_1 U x_3 U,      T(:, b, :) = U G(:, b, :) U^T        (m x p x m),
// and M_E[T] = (I kron P) A (I kron P) with P = U U^T, a congruence of A, so it
// stays SPSD for any U.  U is the caller's (the dominant left singular vectors
// of the mode-1 unfolding, e.g. from tsvdm_truncate of X_(1), which is X's own
// memory read as one m x (p m) face).
//
// Forward: one workgroup per (b, 64 columns t of the slice): W = U^T S(:, t..)
// (r x 64) over 64-row chunks of S = sq(X(:, b, :)) (leading dimension m p)
// staged in LDS with the matching rows of U, then the partial U^T S U =
// W U(t.., :) of those columns; partials summed in order by a second kernel.
// Inverse: one workgroup per (b, 64 rows, 64 columns): H = G_b U(t.., :)^T
// (r x 64), then U(a.., :) H.  FP64 accumulation throughout.
#include "common.h"

using namespace tsvdm;

namespace {

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int ST = 256;

typedef double f64x4_t __attribute__((ext_vector_type(4)));

// Workgroup (column chunk t0 of 64, slice b): W = U^T S[:, t0 .. t0+63] (r x 64,
// S = sq(X(:, b, :))) by FP64 MFMA 16x16x4 over 64-row LDS chunks of U and S
// (wavefront w: column tile w, every row tile of U^T), then the partial
// W U[t0 .. t0+63, :] (r x r) on the vector units.  Rows past m are staged as
// zeros, so the tail chunk needs no special case.
template <typename TX, typename TU>
__global__ __launch_bounds__(ST) void k_two_sided_fwd(const TX *__restrict__ X, int64_t m, int64_t p,
                                                      const TU *__restrict__ U, int r, double *__restrict__ part) {
    __shared__ double us[64 * 65];  // us[a * 65 + i] = U(a0 + a, i); later U(t0 + c, j)
    __shared__ double xs[64 * 65];  // xs[a * 65 + c] = S(a0 + a, t0 + c)
    __shared__ double ws[64 * 65];  // ws[i * 65 + c] = W(i, c)
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t b = blockIdx.y, t0 = (int64_t)blockIdx.x * 64;
    const int64_t lds = m * p;  // leading dimension of S = sq(X(:, b, :))
    const TX *S = X + m * b;
    const int nti = (r + 15) / 16;
    f64x4_t acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = f64x4_t{0, 0, 0, 0};
    for (int64_t a0 = 0; a0 < m; a0 += 64) {
        __syncthreads();
        {
            // element tid + q ST of the chunk: row tid % 64, column tid / 64 + 4 q.
            // Every load is issued before any is used (the fence keeps the
            // conversions after them; without it each load waited for the
            // last); loading the next chunk during the products was slower
            constexpr int PER = 64 * 64 / ST;
            TX xr[PER];
            TU ur[PER];
            const int aa = tid & 63;
            const bool oka = a0 + aa < m;
            const TX *sp = S + (oka ? a0 + aa : 0);
            const TU *up = U + (oka ? a0 + aa : 0);
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int cc = (tid >> 6) + 4 * q;
                const bool okx = oka && t0 + cc < m, oku = oka && cc < r;
                xr[q] = sp[lds * (okx ? t0 + cc : 0)];
                ur[q] = up[(int64_t)m * (oku ? cc : 0)];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int cc = (tid >> 6) + 4 * q;
                const bool okx = oka && t0 + cc < m, oku = oka && cc < r;
                xs[aa * 65 + cc] = okx ? (double)xr[q] : 0.0;
                us[aa * 65 + cc] = oku ? (double)ur[q] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            const int a = 4 * kk + (lane >> 4);
            const double bv = xs[a * 65 + 16 * wave + (lane & 15)];  // B[k][c] = S(a, c)
#pragma unroll
            for (int ti = 0; ti < 4; ++ti)
                if (ti < nti)  // A[i][k] = U(a, i)
                    acc[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(us[a * 65 + 16 * ti + (lane & 15)], bv, acc[ti],
                                                                   0, 0, 0);
        }
    }
    __syncthreads();
    // FP64 16x16x4 output: row lane/16 + 4v, column lane%16 of the tile
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
        if (ti < nti)
#pragma unroll
            for (int v = 0; v < 4; ++v) ws[(16 * ti + (lane >> 4) + 4 * v) * 65 + 16 * wave + (lane & 15)] = acc[ti][v];
    for (int e = tid; e < 64 * 64; e += ST) {  // U rows t0 .. t0+63
        const int cc = e % 64, j = e / 64;
        us[cc * 65 + j] = t0 + cc < m && j < r ? (double)U[(t0 + cc) + m * j] : 0.0;
    }
    __syncthreads();
    // partial(i, j) = sum_c W(i, c) U(t0 + c, j); thread e covers entries e, e + ST, ..
    double *P = part + ((int64_t)b * gridDim.x + blockIdx.x) * r * r;
    for (int e = tid; e < r * r; e += ST) {
        const int i = e % r, j = e / r;
        double s = 0.0;
        for (int c = 0; c < 64; ++c) s = fma(ws[i * 65 + c], us[c * 65 + j], s);
        P[e] = s;
    }
}

// G(i, b, j) = ordered sum over the column chunks of the partials
__global__ void k_two_sided_reduce(const double *__restrict__ part, int nchunks, int r, int64_t p,
                                   double *__restrict__ G) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)r * r * p) return;
    const int64_t ij = e % ((int64_t)r * r), b = e / ((int64_t)r * r);
    const int i = (int)(ij % r), j = (int)(ij / r);
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[((int64_t)b * nchunks + c) * r * r + ij];
    G[i + (int64_t)r * b + (int64_t)r * p * j] = s;  // G is r x p x r
}

// T(a, b, t) = sum_{i, j} U(a, i) G(i, b, j) U(t, j); workgroup (64 a, 64 t, b)
template <typename TX, typename TU>
__global__ __launch_bounds__(ST) void k_two_sided_inv(const double *__restrict__ G, int64_t m, int64_t p,
                                                      const TU *__restrict__ U, int r, TX *__restrict__ T) {
    __shared__ double gs[64 * 65];  // gs[i * 65 + j] = G(i, b, j)
    __shared__ double hs[64 * 65];  // hs[i * 65 + c] = H(i, c) = sum_j G(i, j) U(t0 + c, j)
    __shared__ double ua[64 * 65];  // ua[a * 65 + i] = U(a0 + a, i)
    const int tid = threadIdx.x, cl = tid & 63, g = tid >> 6;
    const int64_t a0 = (int64_t)blockIdx.x * 64, t0 = (int64_t)blockIdx.y * 64, b = blockIdx.z;
    for (int e = tid; e < 64 * 64; e += ST) {
        const int i = e % 64, j = e / 64;
        gs[i * 65 + j] = i < r && j < r ? G[i + (int64_t)r * b + (int64_t)r * p * j] : 0.0;
        ua[i * 65 + j] = a0 + i < m && j < r ? (double)U[(a0 + i) + m * j] : 0.0;
    }
    __syncthreads();
    // H(i, c) for c = cl, i = g + 4 u
    {
        const bool okc = t0 + cl < m;
        double h[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) h[u] = 0.0;
        for (int j = 0; j < r; ++j) {
            const double ut = okc ? (double)U[(t0 + cl) + m * j] : 0.0;
#pragma unroll
            for (int u = 0; u < 16; ++u) h[u] = fma(gs[(g + 4 * u) * 65 + j], ut, h[u]);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) hs[(g + 4 * u) * 65 + cl] = h[u];
    }
    __syncthreads();
    // T(a0 + a, b, t0 + c): thread (a = cl, c = g + 4 v)
    const int64_t a = a0 + cl;
    for (int v = 0; v < 16; ++v) {
        const int64_t t = t0 + g + 4 * v;
        double s = 0.0;
        for (int i = 0; i < r; ++i) s = fma(ua[cl * 65 + i], hs[i * 65 + g + 4 * v], s);
        if (a < m && t < m) T[a + m * b + m * p * t] = (TX)s;
    }
}

#define FAILP(code, ...)        \
    do {                        \
        set_error(__VA_ARGS__); \
        return (code);          \
    } while (0)

tsvdm_status check_two_sided(const tsvdm_tensor *X, const void *U, int32_t udtype, int64_t r) {
    if (!X || !X->data || !U) FAILP(TSVDM_EINVAL, "X (with data) and U are required");
    if (X->dtype != TSVDM_F32 && X->dtype != TSVDM_F64) FAILP(TSVDM_EINVAL, "X must be real F32 or F64");
    if (udtype != TSVDM_F32 && udtype != TSVDM_F64) FAILP(TSVDM_EINVAL, "U must be real F32 or F64");
    if (X->s_a != 1 || X->s_b != X->m || X->s_t != X->m * X->p || X->bsplit != 0) FAILP(TSVDM_EINVAL, "X must be dense");
    if (X->n3 != X->m) FAILP(TSVDM_EINVAL, "two-sided compression needs an m x p x m tensor (m = n)");
    if (r < 1 || r > 64 || r > X->m) FAILP(TSVDM_EUNSUPPORTED, "rank r = %lld must be in 1..min(64, m)", (long long)r);
    if (X->p > 65535 || (X->m + 63) / 64 > 65535) FAILP(TSVDM_EUNSUPPORTED, "shape beyond the launch grid");
    return TSVDM_OK;
}

}  // namespace

extern "C" {

size_t tsvdm_two_sided_workspace_size(const tsvdm_tensor *X, int64_t r) {
    if (!X || r < 1 || X->m < 1 || X->p < 1) return 0;
    const int64_t nch = (X->m + 63) / 64;
    return al256(sizeof(double) * (size_t)(X->p * nch * r * r));
}

tsvdm_status tsvdm_two_sided(const tsvdm_tensor *X, const void *U, int32_t udtype, int64_t r, int32_t direction,
                             double *G, void *workspace, size_t workspace_bytes, void *stream) {
    tsvdm_status st = check_two_sided(X, U, udtype, r);
    if (st != TSVDM_OK) return st;
    if (!G) FAILP(TSVDM_EINVAL, "G is NULL");
    hipStream_t s = (hipStream_t)stream;
    const int64_t m = X->m, p = X->p, nch = (m + 63) / 64;
    const bool xd = X->dtype == TSVDM_F64, ud = udtype == TSVDM_F64;
    if (direction == 1) {
        const size_t need = tsvdm_two_sided_workspace_size(X, r);
        if (!workspace || workspace_bytes < need)
            FAILP(TSVDM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
        double *part = reinterpret_cast<double *>(workspace);
        const dim3 grid((unsigned)nch, (unsigned)p);
#define TSVDM_TS(TXT, TUT)                                                                                 \
    TSVDM_LAUNCH("two_sided", (k_two_sided_fwd<TXT, TUT>), grid, dim3(ST), 0, s,                           \
                 reinterpret_cast<const TXT *>(X->data), m, p, reinterpret_cast<const TUT *>(U), (int)r, part)
        if (xd) {
            if (ud) TSVDM_TS(double, double);
            else TSVDM_TS(double, float);
        } else {
            if (ud) TSVDM_TS(float, double);
            else TSVDM_TS(float, float);
        }
#undef TSVDM_TS
        const int64_t tot = r * r * p;
        TSVDM_LAUNCH("two_sided_reduce", k_two_sided_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     (const double *)part, (int)nch, (int)r, p, G);
    } else if (direction == -1) {
        // G is the input (r x p x r), X the output tensor
        const dim3 grid((unsigned)nch, (unsigned)nch, (unsigned)p);
#define TSVDM_TI(TXT, TUT)                                                                                 \
    TSVDM_LAUNCH("two_sided_inv", (k_two_sided_inv<TXT, TUT>), grid, dim3(ST), 0, s, (const double *)G, m, p, \
                 reinterpret_cast<const TUT *>(U), (int)r, reinterpret_cast<TXT *>(X->data))
        if (xd) {
            if (ud) TSVDM_TI(double, double);
            else TSVDM_TI(double, float);
        } else {
            if (ud) TSVDM_TI(float, double);
            else TSVDM_TI(float, float);
        }
#undef TSVDM_TI
    } else {
        FAILP(TSVDM_EINVAL, "direction must be +1 or -1");
    }
    TSVDM_LAUNCH_CHECK("two-sided compression");
    return TSVDM_OK;
}

}  // extern "C"
