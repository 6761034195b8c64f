// The truncated t-SVDM as an operator and as a Kronecker sum.
//
//  * Kronecker terms (the t-SVDM analogue of Thm thm:tuckerkron; derived):
//    with T = That x_3 M^{-1} and That_f = sum_r s_fr u_fr v_fr^H, lateral
//    slice b of T is sum_{f,r} conj(v_fr[b]) s_fr u_fr (M^{-1}[:, f])^T, so
//      M_E[T] = sum_{f,r} C_fr kron D_fr,
//      C_fr = struct(conj v_fr) = sum_b E_b conj(v_fr[b])  (l x q, the block
//             structure of A: zero blocks stay zero, repeated blocks repeat),
//      D_fr = s_fr u_fr (M^{-1}[:, f])^T                 (m x n3, rank one).
//    For the DFT of real data only faces 0..n3/2 are stored; a stored face f
//    and its conjugate n3 - f add up to w_f Re(C kron D) = w_f (Re C kron Re D
//    - Im C kron Im D), w_f = 2 except f = 0 and f = n3/2, so each stored
//    complex triplet gives two real terms.  One workgroup per term.
//  * The M-product operator: Y = That *_M X for X (p x s x n3, original
//    domain): Xhat = X x_3 M, Yhat_f = Uhat_f diag(S_f) Vhat_f^H Xhat_f, Y =
//    Yhat x_3 M^{-1} (the product is facewise in the transform domain).  The
//    facewise products: one workgroup per (face, 64 columns of X), Z = Vhat^H
//    Xhat (k x 64) accumulated over 32-row chunks staged in LDS, then
//    Yhat = Uhat (S Z) over 32-row chunks of Uhat.
#include "common.h"

#include <math.h>

using namespace tsvdm;

namespace {

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// M^{-1}[t, f] for the real transforms: M^T (DCT-II formula, or a dense M)
__device__ __forceinline__ double minv_real(int kind, const double *Md, int n3, int t, int f) {
    if (kind == TSVDM_M_DENSE) return Md[f + (int64_t)n3 * t];
    const double a = f == 0 ? sqrt(1.0 / n3) : sqrt(2.0 / n3);
    return a * cospi((double)((2 * t + 1) * f) / (2.0 * n3));
}

// Real: term j = f * kmax + r.  Complex (DFT): terms 2 (f * kmax + r) + {0, 1}.
// C: (l x q) x nterms, D: (m x n3) x nterms, column major, the factors' real type.
template <typename T, bool CPLX>
__global__ __launch_bounds__(256) void k_kron_terms(const T *__restrict__ U, const double *__restrict__ S,
                                                    const T *__restrict__ V, const int32_t *__restrict__ ranks,
                                                    int64_t m, int64_t p, int64_t kmax, int n3, int kind,
                                                    const double *__restrict__ Md, int64_t ell, int64_t q,
                                                    const int32_t *__restrict__ blk, const double *__restrict__ winv,
                                                    T *__restrict__ Cout, T *__restrict__ Dout) {
    constexpr int E = CPLX ? 2 : 1;
    const int64_t term = blockIdx.x;
    const int64_t fr = CPLX ? term / 2 : term;
    const int part = CPLX ? (int)(term & 1) : 0;  // 0: real parts, 1: imaginary parts
    const int f = (int)(fr / kmax), r = (int)(fr % kmax);
    const bool live = r < ranks[f];
    T *Cj = Cout + term * ell * q;
    T *Dj = Dout + term * m * n3;
    const T *Vf = V + (int64_t)E * p * kmax * f;
    const T *Uf = U + (int64_t)E * m * kmax * f;
    for (int64_t e = threadIdx.x; e < ell * q; e += blockDim.x) {
        const int k = blk ? blk[e] : (int)e;
        double c = 0.0;
        if (live && k >= 0) {
            const double w = blk ? winv[k] : 1.0;
            // conj(v): real part v_re, imaginary part -v_im
            c = part == 0 ? w * (double)Vf[E * (k + p * r)] : -w * (double)Vf[E * (k + p * r) + 1];
        }
        Cj[e] = (T)c;
    }
    const double s = live ? S[(int64_t)kmax * f + r] : 0.0;
    const double wt = CPLX && !(f == 0 || 2 * f == n3) ? 2.0 : 1.0;
    for (int64_t e = threadIdx.x; e < m * n3; e += blockDim.x) {
        const int64_t a = e % m;
        const int t = (int)(e / m);
        double d = 0.0;
        if (live) {
            if (CPLX) {
                // M^{-1}[t, f] = conj(M[f, t]) = n3^{-1/2} exp(+2 pi i f t / n3)
                double sn, cs;
                sincospi(2.0 * (double)((int64_t)f * t % n3) / n3, &sn, &cs);
                const double g = 1.0 / sqrt((double)n3);
                const double ur = (double)Uf[E * (a + m * r)], ui = (double)Uf[E * (a + m * r) + 1];
                const double dr = s * g * (ur * cs - ui * sn), di = s * g * (ur * sn + ui * cs);
                d = part == 0 ? wt * dr : -wt * di;
            } else {
                d = s * (double)Uf[a + m * r] * minv_real(kind, Md, n3, t, f);
            }
        }
        Dj[e] = (T)d;
    }
}

// complex helpers on (re, im) pairs held as two scalars
template <typename T>
struct Acc {
    T re, im;
};

// Yhat_f(:, c0..c0+63) = Uhat_f diag(S_f) Vhat_f^H Xhat_f(:, c0..c0+63).
// Xhat p x s x nf, Yhat m x s x nf (interleaved complex when CPLX).  Thread
// (column c = tid % 64, group g = tid / 64) accumulates ranks g, g+4, .. of Z
// (k <= 64: at most 16 per thread), then rows a of Yhat for its column.
template <typename T, bool CPLX>
__global__ __launch_bounds__(256) void k_mprod_faces(const T *__restrict__ U, const double *__restrict__ S,
                                                     const T *__restrict__ V, const int32_t *__restrict__ ranks,
                                                     int64_t m, int64_t p, int64_t kmax, int64_t s,
                                                     const T *__restrict__ Xh, T *__restrict__ Yh) {
    constexpr int E = CPLX ? 2 : 1, BC = 32;  // rows per staged chunk
    __shared__ T vs[BC * 65 * E];  // vs[(b * 65 + r) * E]: Vhat rows of the chunk (later Uhat rows)
    __shared__ T xs[BC * 65 * E];  // xs[(b * 65 + c) * E]: Xhat rows of the chunk
    __shared__ T zs[64 * 65 * E];  // zs[(r * 65 + c) * E]: S Z
    const int tid = threadIdx.x, cl = tid & 63, g = tid >> 6;
    const int f = blockIdx.y;
    const int64_t c0 = (int64_t)blockIdx.x * 64, c = c0 + cl;
    const int kf = (int)(ranks[f] < kmax ? ranks[f] : kmax), kc = kf < 64 ? kf : 64;
    const T *Vf = V + (int64_t)E * p * kmax * f;
    const T *Uf = U + (int64_t)E * m * kmax * f;
    const T *Xf = Xh + (int64_t)E * p * s * f;
    T *Yf = Yh + (int64_t)E * m * s * f;
    Acc<T> z[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) z[u] = Acc<T>{T(0), T(0)};
    // staging: element tid + 256 i of a chunk is row tid % BC, column tid / BC
    // + 8 i; all of a thread's loads are issued before any is used (the fence
    // keeps the selects and LDS stores after them)
    constexpr int PER = BC * 64 / 256;
    const int sb = tid % BC, sc = tid / BC;
    for (int64_t b0 = 0; b0 < p; b0 += BC) {
        __syncthreads();
        {
            T vv[PER * E], xv[PER * E];
            const int64_t b = b0 + sb;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int cc = sc + 8 * i;
                const bool okv = b < p && cc < kc, okx = b < p && c0 + cc < s;
#pragma unroll
                for (int q = 0; q < E; ++q) {
                    vv[i * E + q] = Vf[okv ? E * (b + p * cc) + q : 0];
                    xv[i * E + q] = Xf[okx ? E * (b + p * (c0 + cc)) + q : 0];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int cc = sc + 8 * i;
                const bool okv = b < p && cc < kc, okx = b < p && c0 + cc < s;
#pragma unroll
                for (int q = 0; q < E; ++q) {
                    vs[(sb * 65 + cc) * E + q] = okv ? vv[i * E + q] : T(0);
                    xs[(sb * 65 + cc) * E + q] = okx ? xv[i * E + q] : T(0);
                }
            }
        }
        __syncthreads();
        const int nb = (int)(p - b0 < BC ? p - b0 : BC);
        for (int bb = 0; bb < nb; ++bb) {
            const T xr = xs[(bb * 65 + cl) * E], xi = CPLX ? xs[(bb * 65 + cl) * E + 1] : T(0);
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int r = g + 4 * u;
                if (r >= kc) break;
                const T vr = vs[(bb * 65 + r) * E], vi = CPLX ? vs[(bb * 65 + r) * E + 1] : T(0);
                // conj(v) x
                z[u].re += vr * xr + (CPLX ? vi * xi : T(0));
                if (CPLX) z[u].im += vr * xi - vi * xr;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int r = g + 4 * u;
        if (r < 64) {
            const T sv = r < kc ? (T)S[(int64_t)kmax * f + r] : T(0);
            zs[(r * 65 + cl) * E] = sv * z[u].re;
            if (CPLX) zs[(r * 65 + cl) * E + 1] = sv * z[u].im;
        }
    }
    for (int64_t a0 = 0; a0 < m; a0 += BC) {
        __syncthreads();
        {
            T uv[PER * E];
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int rr = sc + 8 * i;
                const bool ok = a0 + sb < m && rr < kc;
#pragma unroll
                for (int q = 0; q < E; ++q) uv[i * E + q] = Uf[ok ? E * (a0 + sb + m * rr) + q : 0];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int rr = sc + 8 * i;
                const bool ok = a0 + sb < m && rr < kc;
#pragma unroll
                for (int q = 0; q < E; ++q) vs[(sb * 65 + rr) * E + q] = ok ? uv[i * E + q] : T(0);
            }
        }
        __syncthreads();
        // thread: column cl, rows a0 + g + 4 i
        for (int i = 0; i < BC / 4; ++i) {
            const int aa = g + 4 * i;
            if (a0 + aa >= m) break;
            T yr = 0, yi = 0;
            for (int r = 0; r < kc; ++r) {
                const T ur = vs[(aa * 65 + r) * E], zr = zs[(r * 65 + cl) * E];
                if (CPLX) {
                    const T ui = vs[(aa * 65 + r) * E + 1], zi = zs[(r * 65 + cl) * E + 1];
                    yr += ur * zr - ui * zi;
                    yi += ur * zi + ui * zr;
                } else {
                    yr += ur * zr;
                }
            }
            if (c < s) {
                Yf[E * (a0 + aa + m * c)] = yr;
                if (CPLX) Yf[E * (a0 + aa + m * c) + 1] = yi;
            }
        }
    }
}

#define FAILM(code, ...)        \
    do {                        \
        set_error(__VA_ARGS__); \
        return (code);          \
    } while (0)

bool cplx_of(int32_t d) { return d == TSVDM_C64 || d == TSVDM_C128; }
bool dbl_of(int32_t d) { return d == TSVDM_F64 || d == TSVDM_C128; }

tsvdm_status check_factors_for(const tsvdm_mdesc *M, const tsvdm_factors *F) {
    if (!M || !F) FAILM(TSVDM_EINVAL, "M and F are required");
    if (M->kind < TSVDM_M_DCT2 || M->kind > TSVDM_M_DENSE) FAILM(TSVDM_EINVAL, "unknown M kind");
    if (M->n3 < 1 || M->n3 > 1024) FAILM(TSVDM_EUNSUPPORTED, "transform length must be in 1..1024");
    if (M->kind == TSVDM_M_DENSE && !M->M) FAILM(TSVDM_EINVAL, "dense M requires M->M");
    const int64_t nf = M->kind == TSVDM_M_DFT ? M->n3 / 2 + 1 : M->n3;
    if (F->nf != nf) FAILM(TSVDM_EINVAL, "factor nf (%lld) != %lld", (long long)F->nf, (long long)nf);
    if ((M->kind == TSVDM_M_DFT) != cplx_of(F->dtype))
        FAILM(TSVDM_EINVAL, "factor dtype does not match the transform (complex iff DFT)");
    if (F->kmax < 1 || F->m < 1 || F->p < 1) FAILM(TSVDM_EINVAL, "factor m, p and kmax must be >= 1");
    if (!F->U || !F->S || !F->V || !F->ranks) FAILM(TSVDM_EINVAL, "factor pointers must be set");
    return TSVDM_OK;
}

}  // namespace

extern "C" {

int64_t tsvdm_kron_terms_count(const tsvdm_mdesc *M, const tsvdm_factors *F) {
    if (!M || !F) return 0;
    return F->nf * F->kmax * (M->kind == TSVDM_M_DFT ? 2 : 1);
}

tsvdm_status tsvdm_kron_terms(const tsvdm_mdesc *M, const tsvdm_factors *F, const tsvdm_placement *pl, int64_t ell,
                              int64_t q, void *C, void *D, void *stream) {
    tsvdm_status st = check_factors_for(M, F);
    if (st != TSVDM_OK) return st;
    if (!C || !D) FAILM(TSVDM_EINVAL, "C and D are required");
    const int32_t *blk = nullptr;
    const double *winv = nullptr;
    if (pl) {
        int64_t pp;
        placement_tables(pl, &ell, &q, &pp, &blk, &winv);
        if (pp != F->p) FAILM(TSVDM_EINVAL, "factor p (%lld) != the placement's p (%lld)", (long long)F->p, (long long)pp);
    } else if (ell < 1 || q < 1 || ell * q != F->p) {
        FAILM(TSVDM_EINVAL, "generic placement: ell*q (%lld) must equal the factor p (%lld)", (long long)(ell * q),
              (long long)F->p);
    }
    const int64_t nterms = tsvdm_kron_terms_count(M, F);
    if (nterms > 0x7fffffff) FAILM(TSVDM_EUNSUPPORTED, "too many terms");
    hipStream_t s = (hipStream_t)stream;
    const int n3 = (int)M->n3;
#define TSVDM_KRON(T, CX)                                                                                           \
    TSVDM_LAUNCH("kron_terms", (k_kron_terms<T, CX>), dim3((unsigned)nterms), dim3(256), 0, s,                     \
                 reinterpret_cast<const T *>(F->U), F->S, reinterpret_cast<const T *>(F->V), F->ranks, F->m, F->p,    \
                 F->kmax, n3, M->kind, M->M, ell, q, blk, winv, reinterpret_cast<T *>(C), reinterpret_cast<T *>(D))
    if (dbl_of(F->dtype)) {
        if (cplx_of(F->dtype)) TSVDM_KRON(double, true);
        else TSVDM_KRON(double, false);
    } else {
        if (cplx_of(F->dtype)) TSVDM_KRON(float, true);
        else TSVDM_KRON(float, false);
    }
#undef TSVDM_KRON
    TSVDM_LAUNCH_CHECK("kron terms");
    return TSVDM_OK;
}

size_t tsvdm_mprod_workspace_size(const tsvdm_mdesc *M, const tsvdm_factors *F, int64_t s) {
    if (check_factors_for(M, F) != TSVDM_OK || s < 0) return 0;
    const size_t es = (dbl_of(F->dtype) ? 8 : 4) * (cplx_of(F->dtype) ? 2 : 1);
    return al256(es * (size_t)F->p * s * F->nf) + al256(es * (size_t)F->m * s * F->nf);
}

tsvdm_status tsvdm_mprod(const tsvdm_mdesc *M, const tsvdm_factors *F, const tsvdm_tensor *X, tsvdm_tensor *Y,
                         void *workspace, size_t workspace_bytes, void *stream) {
    tsvdm_status st = check_factors_for(M, F);
    if (st != TSVDM_OK) return st;
    if (!X || !Y || !X->data || !Y->data) FAILM(TSVDM_EINVAL, "X and Y with data are required");
    if (F->kmax > 64) FAILM(TSVDM_EUNSUPPORTED, "tsvdm_mprod: kmax up to 64");
    const int32_t real_t = dbl_of(F->dtype) ? TSVDM_F64 : TSVDM_F32;
    if (X->dtype != real_t || Y->dtype != real_t)
        FAILM(TSVDM_EINVAL, "X and Y must be real with the factors' precision");
    if (X->m != F->p || X->n3 != M->n3) FAILM(TSVDM_EINVAL, "X must be p x s x n3 (p = %lld, n3 = %lld)",
                                              (long long)F->p, (long long)M->n3);
    const int64_t s = X->p;
    if (Y->m != F->m || Y->p != s || Y->n3 != M->n3) FAILM(TSVDM_EINVAL, "Y must be m x s x n3");
    if (Y->s_a != 1 || Y->s_b != Y->m || Y->s_t != Y->m * Y->p || Y->bsplit != 0) FAILM(TSVDM_EINVAL, "Y must be dense");
    if ((s + 63) / 64 > 0x7fffffff || F->nf > 65535) FAILM(TSVDM_EUNSUPPORTED, "shape beyond the launch grid");
    const size_t need = tsvdm_mprod_workspace_size(M, F, s);
    if (!workspace || workspace_bytes < need)
        FAILM(TSVDM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    if (s == 0) return TSVDM_OK;
    hipStream_t hs = (hipStream_t)stream;
    const bool cx = cplx_of(F->dtype), dbl = dbl_of(F->dtype);
    const size_t es = (dbl ? 8 : 4) * (cx ? 2 : 1);
    char *base = reinterpret_cast<char *>(workspace);
    void *xh = base, *yh = base + al256(es * (size_t)F->p * s * F->nf);
    // Xhat = X x_3 M
    tsvdm_tensor th{};
    th.m = F->p;
    th.p = s;
    th.n3 = F->nf;
    th.s_a = 1;
    th.s_b = F->p;
    th.s_t = F->p * s;
    th.dtype = cx ? (dbl ? TSVDM_C128 : TSVDM_C64) : real_t;
    th.data = xh;
    st = tsvdm_transform(M, +1, X, &th, stream);  // validates X
    if (st != TSVDM_OK) return st;
    const dim3 grid((unsigned)((s + 63) / 64), (unsigned)F->nf);
#define TSVDM_MPROD(T, CX)                                                                                      \
    TSVDM_LAUNCH("mprod_faces", (k_mprod_faces<T, CX>), grid, dim3(256), 0, hs, reinterpret_cast<const T *>(F->U), \
                 F->S, reinterpret_cast<const T *>(F->V), F->ranks, F->m, F->p, F->kmax, s,                     \
                 reinterpret_cast<const T *>(xh), reinterpret_cast<T *>(yh))
    if (dbl) {
        if (cx) TSVDM_MPROD(double, true);
        else TSVDM_MPROD(double, false);
    } else {
        if (cx) TSVDM_MPROD(float, true);
        else TSVDM_MPROD(float, false);
    }
#undef TSVDM_MPROD
    TSVDM_LAUNCH_CHECK("mprod faces");
    // Y = Yhat x_3 M^{-1}
    tsvdm_tensor yt = th;
    yt.m = F->m;
    yt.s_b = F->m;
    yt.s_t = F->m * s;
    yt.data = yh;
    return tsvdm_transform(M, -1, &yt, Y, stream);
}

}  // extern "C"
