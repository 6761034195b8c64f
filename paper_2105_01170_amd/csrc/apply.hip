// y = A_hat x for the structured approximation A_hat = M_E[T] (Sec. 3, map
// M_E, generic placement p = ell*q, block (j, k) of A_hat = sq(T(:, j+ell*k, :))),
// T = That x_3 M^{-1}, That_f = Uhat_f diag(S_f) Vhat_f^H.  A_hat is never formed.
//
// With x split into q blocks x_k of n3 rows:
//   y_j(a, c) = sum_k sum_t T(a, j+ell*k, t) x_k(t, c)
//             = sum_f sum_k That(a, j+ell*k, f) xt_k(f, c),   xt_k = conj(M) x_k,
// because T(a,b,t) = sum_f conj(M(f,t)) That(a,b,f) for orthogonal/unitary M.
// So:  (1) transform every RHS tube x_k(:, c) (one launch of the tube
// transform); (2) for each output tile (64 rows a of block row j, 64 columns
// c) and each face f:  Z_f(r, c) = sum_k conj(Vhat_f(j+ell*k, r)) xt_k(f, c)
// kept in LDS, then  y += sum_r Uhat_f(a, r) S_f(r) Z_f(r, c).
// For the DFT of real data only faces 0..n3/2 are stored; faces f and n3-f
// contribute conjugate terms, so the sum over all faces is
// sum_{stored f} w_f Re(term_f), w_f = 2 except f = 0 and f = n3/2.
#include "common.h"

using namespace tsvdm;

namespace {

constexpr int AT = 256;

template <typename T>
struct Elem {  // real or complex element helpers for the apply kernel
};

__device__ __forceinline__ float rbf(float x) { return bf2f(f2bf(x)); }

template <typename T, bool CPLX, bool BF>
__global__ __launch_bounds__(AT) void k_apply(const T *__restrict__ U, const double *__restrict__ S,
                                              const T *__restrict__ V, const int32_t *__restrict__ ranks,
                                              int64_t m, int64_t p, int64_t kmax, int nf, int n3,
                                              int64_t ell, int64_t q, const T *__restrict__ xt,
                                              int64_t nrhs, T *__restrict__ y, int64_t ldy, int KQ) {
    // tile: rows a0..a0+63 of block row j, columns c0..c0+63
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int E = CPLX ? 2 : 1;
    const int kcap = (int)(kmax < 64 ? kmax : 64);
    T *us = reinterpret_cast<T *>(smem);          // [64][kcap] x E   (U S)
    T *zs = us + 64 * kcap * E;                   // [kcap][64] x E   Z
    T *vs = zs + kcap * 64 * E;                   // [KQ][kcap] x E   Vhat rows j + ell*k
    T *xs = vs + KQ * kcap * E;                   // [KQ][64]  x E    xt
    const int64_t mtiles = (m + 63) / 64;
    const int64_t j = blockIdx.x / mtiles, a0 = (blockIdx.x % mtiles) * 64, c0 = (int64_t)blockIdx.y * 64;
    const int tid = threadIdx.x;
    const int ta = tid & 63;  // output row within the tile
    T acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = T(0);
    for (int f = 0; f < nf; ++f) {
        const int kf = ranks[f] < kcap ? ranks[f] : kcap;
        if (kf == 0) continue;
        const T wgt = (CPLX && !(f == 0 || 2 * f == n3)) ? T(2) : T(1);
        __syncthreads();
        for (int e = tid; e < 64 * kf; e += AT) {
            int a = e % 64, r = e / 64;
            bool ok = a0 + a < m;
            double s = S[(int64_t)f * kmax + r];
            for (int c = 0; c < E; ++c) {
                T u = ok ? U[((int64_t)f * m * kmax + (a0 + a) + m * r) * E + c] : T(0);
                T v = (T)((double)u * s);
                us[(a * kcap + r) * E + c] = BF ? rbf(v) : v;
            }
        }
        for (int e = tid; e < kf * 64; e += AT) {
            for (int c = 0; c < E; ++c) zs[e * E + c] = T(0);
        }
        for (int k0 = 0; k0 < q; k0 += KQ) {
            const int kq = (int)((q - k0) < KQ ? (q - k0) : KQ);
            __syncthreads();
            for (int e = tid; e < kq * kf; e += AT) {
                int kk = e % kq, r = e / kq;
                int64_t b = j + ell * (k0 + kk);
                for (int c = 0; c < E; ++c) {
                    T v = V[((int64_t)f * p * kmax + b + p * r) * E + c];
                    vs[(kk * kcap + r) * E + c] = BF ? rbf(v) : v;
                }
            }
            for (int e = tid; e < kq * 64; e += AT) {
                int kk = e % kq, cc = e / kq;
                bool ok = c0 + cc < nrhs;
                int64_t idx = (k0 + kk) + q * (c0 + cc) + q * nrhs * f;
                for (int c = 0; c < E; ++c) {
                    T v = ok ? xt[idx * E + c] : T(0);
                    xs[(kk * 64 + cc) * E + c] = BF ? rbf(v) : v;
                }
            }
            __syncthreads();
            // Z(r, c) += sum_k conj(V(k, r)) conj(xt(k, c))  [complex: conj of the
            // forward DFT gives xt = conj(M) x];  real: V(k, r) xt(k, c)
            for (int e = tid; e < kf * 64; e += AT) {
                int cc = e % 64, r = e / 64;
                T zr = zs[e * E], zi = CPLX ? zs[e * E + 1] : T(0);
                for (int kk = 0; kk < kq; ++kk) {
                    T vr = vs[(kk * kcap + r) * E], xr = xs[(kk * 64 + cc) * E];
                    if (CPLX) {
                        T vi = vs[(kk * kcap + r) * E + 1], xi = xs[(kk * 64 + cc) * E + 1];
                        // conj(v) conj(x) = conj(v x)
                        zr += vr * xr - vi * xi;
                        zi -= vr * xi + vi * xr;
                    } else {
                        zr += vr * xr;
                    }
                }
                zs[e * E] = zr;
                if (CPLX) zs[e * E + 1] = zi;
            }
        }
        __syncthreads();
        // y(a, c) += w Re(sum_r (U S)(a, r) Z(r, c))
        for (int i = 0; i < 16; ++i) {
            int cc = (tid >> 6) + 4 * i;
            T sr = T(0);
            for (int r = 0; r < kf; ++r) {
                T ur = us[(ta * kcap + r) * E], zr = zs[(r * 64 + cc) * E];
                if (CPLX) {
                    T ui = us[(ta * kcap + r) * E + 1], zi = zs[(r * 64 + cc) * E + 1];
                    sr += ur * zr - ui * zi;
                } else {
                    sr += ur * zr;
                }
            }
            acc[i] += wgt * sr;
        }
    }
    if (a0 + ta < m) {
        for (int i = 0; i < 16; ++i) {
            int64_t cc = c0 + (tid >> 6) + 4 * i;
            if (cc < nrhs) y[(j * m + a0 + ta) + ldy * cc] = acc[i];
        }
    }
}

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

namespace tsvdm {

size_t apply_workspace(const tsvdm_mdesc *M, const tsvdm_factors *F, int64_t ell, int64_t q,
                       int64_t nrhs, int32_t compute) {
    (void)ell;
    const bool cplx = M->kind == TSVDM_M_DFT;
    const size_t es = (compute == TSVDM_F64 ? 8 : 4) * (cplx ? 2 : 1);
    return al256(es * (size_t)q * nrhs * F->nf);
}

tsvdm_status launch_apply(const tsvdm_mdesc *M, const tsvdm_factors *F, int64_t ell, int64_t q,
                          int64_t nrhs, const void *x, int64_t ldx, void *y, int64_t ldy,
                          int32_t compute, void *ws, hipStream_t s) {
    const bool cplx = M->kind == TSVDM_M_DFT;
    const bool dbl = compute == TSVDM_F64;
    const int64_t n3 = M->n3, nf = F->nf;
    // (1) RHS tubes: element (k, c, t) of the view is x[k*n3 + t + ldx*c]
    tsvdm_tensor in{}, out{};
    in.m = q; in.p = nrhs; in.n3 = n3;
    in.s_a = n3; in.s_b = ldx; in.s_t = 1; in.bsplit = 0; in.s_bk = 0;
    in.dtype = dbl ? TSVDM_F64 : TSVDM_F32;
    in.data = const_cast<void *>(x);
    out.m = q; out.p = nrhs; out.n3 = nf;
    out.s_a = 1; out.s_b = q; out.s_t = q * nrhs; out.bsplit = 0; out.s_bk = 0;
    out.dtype = cplx ? (dbl ? TSVDM_C128 : TSVDM_C64) : in.dtype;
    out.data = ws;
    tsvdm_status st = launch_transform(M, 1, &in, &out, s);
    if (st != TSVDM_OK) return st;
    // (2) fused contraction
    const int kcap = (int)(F->kmax < 64 ? F->kmax : 64);
    if (F->kmax > 64) {
        set_error("tsvdm_apply: kmax > 64 is not supported");
        return TSVDM_EUNSUPPORTED;
    }
    const size_t es = (dbl ? 8 : 4) * (cplx ? 2 : 1);
    int KQ = 64;
    auto lds_of = [&](int kq) { return es * ((size_t)64 * kcap * 2 + (size_t)kq * kcap + (size_t)kq * 64); };
    while (KQ > 8 && lds_of(KQ) > 60 * 1024) KQ >>= 1;
    const size_t lds = lds_of(KQ);
    if (lds > 160 * 1024) {
        set_error("tsvdm_apply: tile does not fit in LDS (kmax too large for this precision)");
        return TSVDM_EUNSUPPORTED;
    }
    const int64_t mtiles = (F->m + 63) / 64;
    dim3 grid((unsigned)(mtiles * ell), (unsigned)((nrhs + 63) / 64));
#define TSVDM_APPLY(T, C, B)                                                                        \
    do {                                                                                            \
        if (lds > 65536) {                                                                          \
            hipError_t e_ = hipFuncSetAttribute(reinterpret_cast<const void *>(k_apply<T, C, B>),    \
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
            if (e_ != hipSuccess) return hip_check(e_, "hipFuncSetAttribute(apply)");              \
        }                                                                                           \
        TSVDM_LAUNCH("apply_fused", (k_apply<T, C, B>), grid, dim3(AT), lds, s,                              \
                           reinterpret_cast<const T *>(F->U), F->S, reinterpret_cast<const T *>(F->V), \
                           F->ranks, F->m, F->p, F->kmax, (int)nf, (int)n3, ell, q,                 \
                           reinterpret_cast<const T *>(ws), nrhs, reinterpret_cast<T *>(y), ldy, KQ); \
    } while (0)
    if (dbl) {
        if (cplx) TSVDM_APPLY(double, true, false);
        else TSVDM_APPLY(double, false, false);
    } else if (compute == TSVDM_BF16) {
        if (cplx) TSVDM_APPLY(float, true, true);
        else TSVDM_APPLY(float, false, true);
    } else {
        if (cplx) TSVDM_APPLY(float, true, false);
        else TSVDM_APPLY(float, false, false);
    }
#undef TSVDM_APPLY
    TSVDM_LAUNCH_CHECK("k_apply");
    return TSVDM_OK;
}

}  // namespace tsvdm
