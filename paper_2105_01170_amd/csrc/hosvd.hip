// Data-driven orthogonal transforms and the mode-2 compression (Sec. 2.4,
// HOSVD; Sec. 6.3).
//
//  * Mode Gram: G = X_(3) X_(3)^T (n3 x n3; entry (s, t) is the inner product
//    of frontal faces s and t, eq. mode3unfold) or G = X_(2) X_(2)^T (p x p;
//    the sum over faces of X_t^T X_t), in FP64 from FP32 or FP64 data.  A
//    persistent kernel: workgroup w walks element chunks w, w + G, .. of the
//    unfolding's rows, staging 64 elements of every row in LDS; thread
//    (bi, bj) accumulates the 4 x 4 block of rows 4 bi.., 4 bj.. (bi <= bj) in
//    registers; the per-workgroup partials are summed in order by a second
//    kernel (the result does not depend on the number of workgroups' timing,
//    only on the grid size, which is fixed by the shape).
//  * Symmetric eigensolver (N <= 64): the cyclic Jacobi solver of the core
//    SVD in one workgroup, eigenvalues in decreasing order, each eigenvector
//    with its largest-magnitude entry positive (first such entry on ties).
//  * Mode-3 transform: M = W^T with W the eigenvectors of the mode-3 Gram,
//    i.e. the left singular vectors of X_(3): the mode-3 HOSVD factor as the
//    orthogonal M of the transform (face f of X x_3 M then carries the energy
//    s_f^2 of the unfolding).
//  * Mode-2 product: out = X x_2 K for K = V^T (compression G = X x_2 V^T) or
//    K = V (reconstruction T = G x_2 V), facewise products with FP64
//    accumulation.
#include "common.h"
#include "jacobi_dev.h"

#include <math.h>

using namespace tsvdm;

namespace {

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int GT = 256, CH = 64;  // threads; elements per chunk
constexpr int GRAM_WG = 512;      // workgroups of the Gram kernel (fixed, so the partials are summed in a fixed order)

// element e of row j of the mode-`mode` unfolding of a dense m x p x n3 tensor
struct UnfoldView {
    int64_t m, p, n3;
    int mode;
    __device__ __forceinline__ int64_t addr(int64_t j, int64_t e) const {
        if (mode == 3) return e + m * p * j;   // face j, element e = a + m b
        const int64_t a = e % m, t = e / m;    // lateral slice j, element e = a + m t
        return a + m * j + m * p * t;
    }
    __host__ __device__ int64_t rows() const { return mode == 3 ? n3 : p; }
    __host__ __device__ int64_t cols() const { return mode == 3 ? m * p : m * n3; }
};

template <int NP, typename T>
__global__ __launch_bounds__(GT) void k_mode_gram(const T *__restrict__ X, UnfoldView v, double *__restrict__ part) {
    constexpr int NB = NP / 4, NBLK = NB * (NB + 1) / 2, LDX = CH + 1;
    __shared__ double xs[NP * LDX];
    const int tid = threadIdx.x;
    const int N = (int)v.rows();
    const int64_t E = v.cols(), nch = (E + CH - 1) / CH;
    int bi = 0, bj = 0;
    const bool own = tid < NBLK;
    {
        int rem = own ? tid : 0;
        while (rem >= NB - bi) {
            rem -= NB - bi;
            ++bi;
        }
        bj = bi + rem;
    }
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) acc[u][w] = 0.0;
    const int el = tid % CH, j0 = tid / CH;  // this thread's element and first row of the staging
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const int64_t e = c * CH + el;
        __syncthreads();
        {
            // all of the thread's loads issued before any is stored (the fence
            // keeps the conversions and LDS stores after them)
            constexpr int PJ = NP * CH / GT;
            T xv[PJ];
#pragma unroll
            for (int i = 0; i < PJ; ++i) {
                const int j = j0 + i * (GT / CH);
                xv[i] = X[j < N && e < E ? v.addr(j, e) : 0];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < PJ; ++i) {
                const int j = j0 + i * (GT / CH);
                xs[j * LDX + el] = j < N && e < E ? (double)xv[i] : 0.0;
            }
        }
        __syncthreads();
        if (own) {
#pragma unroll 4
            for (int k = 0; k < CH; ++k) {
                double a[4], b[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[u] = xs[(4 * bi + u) * LDX + k];
                    b[u] = xs[(4 * bj + u) * LDX + k];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int w = 0; w < 4; ++w) acc[u][w] = fma(a[u], b[w], acc[u][w]);
            }
        }
    }
    if (own) {
        double *P = part + (int64_t)blockIdx.x * NP * NP;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int w = 0; w < 4; ++w) P[(4 * bi + u) * NP + 4 * bj + w] = acc[u][w];
    }
}

// G (N x N, column major) = sum of the partials' upper blocks, mirrored.
// Workgroup: 16 entries, each summed by 16 threads over the partials
// q, q + 16, .. (independent loads in flight), then the 16 sums of an entry
// added in a fixed order: the result is the same on every run.
constexpr int RE = 16, RQ = 16;
template <int NP>
__global__ __launch_bounds__(RE * RQ) void k_gram_reduce(const double *__restrict__ part, int nparts, int N,
                                                         double *__restrict__ G) {
    __shared__ double red[RQ][RE];
    const int el = threadIdx.x % RE, q = threadIdx.x / RE;
    const int e = blockIdx.x * RE + el;
    double s = 0.0;
    if (e < N * N) {
        int i = e % N, j = e / N;
        if (i / 4 > j / 4) {  // lower block: the mirror of an upper one
            const int t = i;
            i = j;
            j = t;
        }
        const double *src = part + i * NP + j;
        int w = q;
        for (; w + 3 * RQ < nparts; w += 4 * RQ) {
            const double a = src[(int64_t)w * NP * NP], b = src[(int64_t)(w + RQ) * NP * NP];
            const double c = src[(int64_t)(w + 2 * RQ) * NP * NP], d = src[(int64_t)(w + 3 * RQ) * NP * NP];
            s += (a + b) + (c + d);
        }
        for (; w < nparts; w += RQ) s += src[(int64_t)w * NP * NP];
    }
    red[q][el] = s;
    __syncthreads();
    if (q == 0 && e < N * N) {
        double t = 0.0;
        for (int u = 0; u < RQ; ++u) t += red[u][el];
        G[e] = t;
    }
}

constexpr int ET = 1024;
// Eigendecomposition of the symmetric N x N matrix G (column major, FP64):
// lam[j] decreasing, W[:, j] the eigenvectors (largest-magnitude entry
// positive), and, when Mt is set, Mt = W^T (column major).
template <int LP>
__global__ __launch_bounds__(ET) void k_sym_eig(const double *__restrict__ G, int N, int max_sweeps, double jtol,
                                                double *__restrict__ lam, double *__restrict__ W,
                                                double *__restrict__ Mt, int32_t *__restrict__ info) {
    constexpr int LD = jacobi_ld<LP>(), LDE = jacobi_ld<LP>(), NPM = LP / 2;
    __shared__ __align__(16) double Gb[2][LP * LD];
    __shared__ __align__(16) double Eb[2][LP * LDE];
    __shared__ __align__(16) double2 cs[2][NPM];
    __shared__ double lv[LP];
    __shared__ int perm[LP];
    __shared__ int rflag[3];
    __shared__ double sgn[LP];
    const int tid = threadIdx.x;
    for (int e = tid; e < LP * LD; e += ET) Gb[0][e] = 0.0;
    for (int e = tid; e < LP * LDE; e += ET) Eb[0][e] = Eb[1][e] = 0.0;
    __syncthreads();
    for (int e = tid; e < N * N; e += ET) {
        const int i = e % N, j = e / N;
        Gb[0][i * LD + j] = G[e];
    }
    if (tid < N) Eb[0][tid * LDE + tid] = 1.0;
    if (tid < 3) rflag[tid] = 0;
    __syncthreads();
    // absolute rotation threshold jtol times the trace (0: the relative test
    // alone, every eigenpair to full relative accuracy).  For a transform
    // basis of a positive semidefinite Gram, 1e-15 leaves the eigenvectors of
    // eigenvalues at the rounding level of the largest unresolved, which on
    // low-rank data took most of the sweeps
    if (tid < 64) {
        double t = 0.0;
        for (int c = tid; c < N; c += 64) t += fabs(Gb[0][c * LD + c]);
        t = wave_sum(t);
        if (tid == 0) lv[0] = t;
    }
    __syncthreads();
    const double atol = jtol * lv[0];
    __syncthreads();
    int conv = 0, dslot;
    const double *Gf, *Ef;
    jacobi_eig<LP, ET>(Gb[0], Gb[1], Eb[0], Eb[1], &cs[0][0], rflag, N, atol, max_sweeps, conv, Gf, Ef, dslot);
    if (tid < N) {
        const int sl = jacobi_slot(tid, dslot);
        lv[tid] = Gf[sl * LD + sl];
    }
    __syncthreads();
    if (tid < N) {
        int pos = 0;
        const double li = lv[tid];
        for (int j = 0; j < N; ++j) pos += sorts_before(lv[j], j, li, tid);
        perm[pos] = tid;
    }
    __syncthreads();
    if (tid < N) {  // sign of eigenvector tid (in sorted order)
        const int sl = jacobi_slot(perm[tid], dslot);
        double best = -1.0, v = 0.0;
        for (int r = 0; r < N; ++r) {
            const double x = Ef[sl * LDE + r];
            if (fabs(x) > best) {
                best = fabs(x);
                v = x;
            }
        }
        sgn[tid] = v < 0.0 ? -1.0 : 1.0;
        lam[tid] = lv[perm[tid]];
    }
    __syncthreads();
    for (int e = tid; e < N * N; e += ET) {
        const int r = e % N, j = e / N;
        const double x = sgn[j] * Ef[jacobi_slot(perm[j], dslot) * LDE + r];
        W[r + (int64_t)N * j] = x;
        if (Mt) Mt[j + (int64_t)N * r] = x;
    }
    if (tid == 0 && info) *info = conv || N <= 1 ? 0 : 1;
}

// s = sqrt(max(lam, 0))
__global__ void k_sqrt_pos(const double *__restrict__ lam, int N, double *__restrict__ s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) s[i] = sqrt(fmax(lam[i], 0.0));
}

// out(a, c, t) = sum_b in(a, b, t) K(b, c), K(b, c) = Kp[b * skb + c * skc];
// workgroup: rows a0..a0+63, columns c0..c0+63 of face t; thread (a, group g)
// accumulates columns c0 + 16 g .. +15 in FP64; K staged in LDS 64 b at a time
template <typename T>
__global__ __launch_bounds__(GT) void k_mode2(const T *__restrict__ in, int64_t m, int64_t pin, int64_t n3,
                                              const double *__restrict__ Kp, int64_t skb, int64_t skc, int64_t pout,
                                              T *__restrict__ out) {
    __shared__ double ks[64 * 65];  // ks[b * 65 + c]
    const int tid = threadIdx.x, al = tid & 63, g = tid >> 6;
    const int64_t a = (int64_t)blockIdx.x * 64 + al, t = blockIdx.y, c0 = (int64_t)blockIdx.z * 64;
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    const T *In = in + m * pin * t;
    for (int64_t b0 = 0; b0 < pin; b0 += 64) {
        __syncthreads();
        for (int e = tid; e < 64 * 64; e += GT) {
            const int bb = e % 64, cc = e / 64;
            const bool ok = b0 + bb < pin && c0 + cc < pout;
            ks[bb * 65 + cc] = ok ? Kp[(b0 + bb) * skb + (c0 + cc) * skc] : 0.0;
        }
        __syncthreads();
        const int64_t nb = pin - b0 < 64 ? pin - b0 : 64;
        for (int bb = 0; bb < nb; ++bb) {
            const double x = a < m ? (double)In[a + m * (b0 + bb)] : 0.0;
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u] = fma(x, ks[bb * 65 + 16 * g + u], acc[u]);
        }
    }
    if (a < m) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int64_t c = c0 + 16 * g + u;
            if (c < pout) out[a + m * c + m * pout * t] = (T)acc[u];
        }
    }
}

int padded(int64_t n) { return n <= 16 ? 16 : n <= 32 ? 32 : n <= 48 ? 48 : 64; }

#define FAILH(code, ...)        \
    do {                        \
        set_error(__VA_ARGS__); \
        return (code);          \
    } while (0)

bool dense_real(const tsvdm_tensor *X) {
    return X && X->data && (X->dtype == TSVDM_F32 || X->dtype == TSVDM_F64) && X->s_a == 1 && X->s_b == X->m &&
           X->s_t == X->m * X->p && X->bsplit == 0 && X->m >= 1 && X->p >= 1 && X->n3 >= 1;
}

size_t gram_ws(int64_t N) { return al256(sizeof(double) * (size_t)GRAM_WG * padded(N) * padded(N)); }

tsvdm_status launch_gram(const tsvdm_tensor *X, int mode, double *G, void *ws, hipStream_t s) {
    UnfoldView v{X->m, X->p, X->n3, mode};
    const int64_t N = v.rows();
    const int NP = padded(N);
    double *part = reinterpret_cast<double *>(ws);
#define TSVDM_GRAM(NPV)                                                                                     \
    do {                                                                                                    \
        if (X->dtype == TSVDM_F64)                                                                          \
            TSVDM_LAUNCH("mode_gram", (k_mode_gram<NPV, double>), dim3(GRAM_WG), dim3(GT), 0, s,            \
                         reinterpret_cast<const double *>(X->data), v, part);                               \
        else                                                                                                \
            TSVDM_LAUNCH("mode_gram", (k_mode_gram<NPV, float>), dim3(GRAM_WG), dim3(GT), 0, s,             \
                         reinterpret_cast<const float *>(X->data), v, part);                                \
        TSVDM_LAUNCH("mode_gram_reduce", (k_gram_reduce<NPV>), dim3((unsigned)((N * N + RE - 1) / RE)),           \
                     dim3(RE * RQ), 0, s, (const double *)part, GRAM_WG, (int)N, G);                        \
    } while (0)
    switch (NP) {
        case 16: TSVDM_GRAM(16); break;
        case 32: TSVDM_GRAM(32); break;
        case 48: TSVDM_GRAM(48); break;
        default: TSVDM_GRAM(64); break;
    }
#undef TSVDM_GRAM
    TSVDM_LAUNCH_CHECK("mode gram");
    return TSVDM_OK;
}

tsvdm_status launch_eig(const double *G, int64_t N, double *lam, double *W, double *Mt, double jtol, hipStream_t s) {
#define TSVDM_EIG(LPV)                                                                                         \
    TSVDM_LAUNCH("sym_eig", (k_sym_eig<LPV>), dim3(1), dim3(ET), 0, s, G, (int)N, 60, jtol, lam, W, Mt,         \
                 (int32_t *)nullptr)
    switch (padded(N)) {
        case 16: TSVDM_EIG(16); break;
        case 32: TSVDM_EIG(32); break;
        case 48: TSVDM_EIG(48); break;
        default: TSVDM_EIG(64); break;
    }
#undef TSVDM_EIG
    TSVDM_LAUNCH_CHECK("sym eig");
    return TSVDM_OK;
}

}  // namespace

extern "C" {

size_t tsvdm_mode_gram_workspace_size(const tsvdm_tensor *X, int32_t mode) {
    if (!X || (mode != 2 && mode != 3)) return 0;
    const int64_t N = mode == 3 ? X->n3 : X->p;
    if (N < 1 || N > 64) return 0;
    return gram_ws(N);
}

tsvdm_status tsvdm_mode_gram(const tsvdm_tensor *X, int32_t mode, double *G, void *workspace, size_t workspace_bytes,
                             void *stream) {
    if (!dense_real(X)) FAILH(TSVDM_EINVAL, "X must be a dense real F32/F64 tensor with data");
    if (mode != 2 && mode != 3) FAILH(TSVDM_EINVAL, "mode must be 2 or 3");
    if (!G) FAILH(TSVDM_EINVAL, "G is NULL");
    const int64_t N = mode == 3 ? X->n3 : X->p;
    if (N > 64) FAILH(TSVDM_EUNSUPPORTED, "mode-%d Gram of order %lld: at most 64", mode, (long long)N);
    const size_t need = gram_ws(N);
    if (!workspace || workspace_bytes < need)
        FAILH(TSVDM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    return launch_gram(X, mode, G, workspace, (hipStream_t)stream);
}

tsvdm_status tsvdm_sym_eig(const double *G, int64_t N, double *lam, double *W, void *stream) {
    if (!G || !lam || !W) FAILH(TSVDM_EINVAL, "G, lam and W are required");
    if (N < 1 || N > 64) FAILH(TSVDM_EUNSUPPORTED, "order %lld: 1..64", (long long)N);
    return launch_eig(G, N, lam, W, nullptr, 0.0, (hipStream_t)stream);
}

size_t tsvdm_mode3_transform_workspace_size(const tsvdm_tensor *X) {
    if (!X || X->n3 < 1 || X->n3 > 64) return 0;
    const int64_t N = X->n3;
    return gram_ws(N) + 3 * al256(sizeof(double) * (size_t)(N * N));
}

tsvdm_status tsvdm_mode3_transform(const tsvdm_tensor *X, double *M, double *sv, void *workspace,
                                   size_t workspace_bytes, void *stream) {
    if (!dense_real(X)) FAILH(TSVDM_EINVAL, "X must be a dense real F32/F64 tensor with data");
    if (!M) FAILH(TSVDM_EINVAL, "M is NULL");
    const int64_t N = X->n3;
    if (N > 64) FAILH(TSVDM_EUNSUPPORTED, "the mode-3 transform supports n3 <= 64");
    const size_t need = tsvdm_mode3_transform_workspace_size(X);
    if (!workspace || workspace_bytes < need)
        FAILH(TSVDM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    hipStream_t s = (hipStream_t)stream;
    char *base = reinterpret_cast<char *>(workspace);
    double *G = reinterpret_cast<double *>(base + gram_ws(N));
    double *W = G + al256(sizeof(double) * (size_t)(N * N)) / sizeof(double);
    double *lam = W + al256(sizeof(double) * (size_t)(N * N)) / sizeof(double);
    tsvdm_status st = launch_gram(X, 3, G, workspace, s);
    if (st != TSVDM_OK) return st;
    st = launch_eig(G, N, lam, W, M, 1e-15, s);
    if (st != TSVDM_OK) return st;
    if (sv) {
        TSVDM_LAUNCH("sqrt_pos", k_sqrt_pos, dim3(1), dim3(64), 0, s, (const double *)lam, (int)N, sv);
        TSVDM_LAUNCH_CHECK("mode3 transform");
    }
    return TSVDM_OK;
}

tsvdm_status tsvdm_mode2_product(const tsvdm_tensor *X, const double *V, int64_t pv, int64_t r, int32_t direction,
                                 void *out, void *stream) {
    if (!dense_real(X)) FAILH(TSVDM_EINVAL, "X must be a dense real F32/F64 tensor with data");
    if (!V || !out) FAILH(TSVDM_EINVAL, "V and out are required");
    if (pv < 1 || r < 1) FAILH(TSVDM_EINVAL, "V must be pv x r with pv, r >= 1");
    if (direction != 1 && direction != -1) FAILH(TSVDM_EINVAL, "direction must be +1 or -1");
    int64_t pin, pout, skb, skc;
    if (direction == 1) {  // out = X x_2 V^T: K(b, c) = V(b, c)
        if (X->p != pv) FAILH(TSVDM_EINVAL, "X has %lld lateral slices, V has %lld rows", (long long)X->p, (long long)pv);
        pin = pv;
        pout = r;
        skb = 1;
        skc = pv;
    } else {  // out = X x_2 V: K(j, b) = V(b, j)
        if (X->p != r) FAILH(TSVDM_EINVAL, "X has %lld lateral slices, V has %lld columns", (long long)X->p, (long long)r);
        pin = r;
        pout = pv;
        skb = pv;
        skc = 1;
    }
    if (X->n3 > 65535 || (X->m + 63) / 64 > 0x7fffffff || (pout + 63) / 64 > 65535)
        FAILH(TSVDM_EUNSUPPORTED, "mode-2 product: shape beyond the launch grid");
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid((unsigned)((X->m + 63) / 64), (unsigned)X->n3, (unsigned)((pout + 63) / 64));
    if (X->dtype == TSVDM_F64)
        TSVDM_LAUNCH("mode2_product", k_mode2<double>, grid, dim3(GT), 0, s, reinterpret_cast<const double *>(X->data),
                     X->m, pin, X->n3, V, skb, skc, pout, reinterpret_cast<double *>(out));
    else
        TSVDM_LAUNCH("mode2_product", k_mode2<float>, grid, dim3(GT), 0, s, reinterpret_cast<const float *>(X->data),
                     X->m, pin, X->n3, V, skb, skc, pout, reinterpret_cast<float *>(out));
    TSVDM_LAUNCH_CHECK("mode2 product");
    return TSVDM_OK;
}

}  // extern "C"
