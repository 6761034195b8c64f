// Plain FP64 facewise truncated SVD (PREC_F64): one-sided Jacobi.
//
// For every face of the transform-domain tensor, the n = min(m, p) vectors of
// the smaller side (columns of the face if m >= p, else columns of its
// conjugate transpose), each of length L = max(m, p), are orthogonalised by
// plane rotations chosen from their 2x2 Gram matrix (Hestenes' method).  One
// workgroup of 16 wavefronts owns one face; pairs are scheduled by the
// round-robin ordering so that the n/2 rotations of a round touch disjoint
// vectors and run on different wavefronts at once.  A sweep with no rotation
// ends the face.  Singular values are the vector norms; the left/right
// vectors are the normalised vectors and the accumulated rotations.
// Truncation then keeps the leading k_f triplets by the fixed or energy rule.
// Bound: FP64 ALU and L2 bandwidth (the face is re-read every round).
#include "common.h"

#include <math.h>

using namespace tsvdm;

namespace {

constexpr int JT = 1024;  // threads per workgroup (16 wavefronts)
constexpr int JW = JT / 64;

__device__ __forceinline__ double cj(double x) { return x; }
__device__ __forceinline__ cx<double> cj(cx<double> x) { return {x.re, -x.im}; }
__device__ __forceinline__ double abs2(double x) { return x * x; }
__device__ __forceinline__ double abs2(cx<double> x) { return x.re * x.re + x.im * x.im; }
__device__ __forceinline__ double mul(double a, double b) { return a * b; }
__device__ __forceinline__ cx<double> mul(cx<double> a, cx<double> b) { return cmul(a, b); }
__device__ __forceinline__ double scale(double a, double s) { return a * s; }
__device__ __forceinline__ cx<double> scale(cx<double> a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ double axpby(double c, double x, double s, double y) { return c * x + s * y; }
__device__ __forceinline__ cx<double> axpby(double c, cx<double> x, double s, cx<double> y) {
    return {c * x.re + s * y.re, c * x.im + s * y.im};
}
template <typename T> __device__ __forceinline__ T zero();
template <> __device__ __forceinline__ double zero<double>() { return 0.0; }
template <> __device__ __forceinline__ cx<double> zero<cx<double>>() { return {0.0, 0.0}; }
template <typename T> __device__ __forceinline__ T one();
template <> __device__ __forceinline__ double one<double>() { return 1.0; }
template <> __device__ __forceinline__ cx<double> one<cx<double>>() { return {1.0, 0.0}; }

__device__ __forceinline__ double wsum(double v) { return wave_sum(v); }

// copy face f into the working vectors W (L x n), V = I (n x n), ||face||^2
template <typename T>
__global__ __launch_bounds__(JT) void k_jac_prepare(const T *__restrict__ X, int64_t m, int64_t p,
                                                    T *__restrict__ W, T *__restrict__ V,
                                                    double *__restrict__ fro2) {
    __shared__ double part[JW];
    const int64_t f = blockIdx.x;
    const bool tall = m >= p;
    const int64_t L = tall ? m : p, n = tall ? p : m;
    const T *F = X + f * m * p;
    T *Wf = W + f * L * n;
    T *Vf = V + f * n * n;
    double acc = 0.0;
    for (int64_t e = threadIdx.x; e < m * p; e += JT) {
        // e enumerates W: vector j = e / L, element t = e % L
        int64_t j = e / L, t = e % L;
        T v = tall ? F[t + m * j] : cj(F[j + m * t]);
        Wf[e] = v;
        acc += abs2(v);
    }
    for (int64_t e = threadIdx.x; e < n * n; e += JT) Vf[e] = (e % n == e / n) ? one<T>() : zero<T>();
    acc = wsum(acc);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < JW; ++w) s += part[w];
        fro2[f] = s;
    }
}

// pair k of round r in the round-robin ordering of ne (even) players
__device__ __forceinline__ void rr_pair(int r, int k, int ne, int &a, int &b) {
    if (k == 0) {
        a = r;
        b = ne - 1;
    } else {
        a = (r + k) % (ne - 1);
        b = (r - k + (ne - 1)) % (ne - 1);
    }
    if (a > b) { int t = a; a = b; b = t; }
}

template <typename T>
__global__ __launch_bounds__(JT) void k_jac_sweeps(int64_t m, int64_t p, T *__restrict__ W,
                                                   T *__restrict__ V, int max_sweeps, double tol,
                                                   int *__restrict__ sweeps_used) {
    __shared__ int rotated;
    const int64_t f = blockIdx.x;
    const bool tall = m >= p;
    const int L = (int)(tall ? m : p), n = (int)(tall ? p : m);
    T *Wf = W + (int64_t)f * L * n;
    T *Vf = V + (int64_t)f * n * n;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ne = n + (n & 1);
    int sweep = 0, done = 0;
    for (sweep = 1; sweep <= max_sweeps && n > 1; ++sweep) {
        if (threadIdx.x == 0) rotated = 0;
        __syncthreads();
        for (int r = 0; r < ne - 1; ++r) {
            for (int k = wave; k < ne / 2; k += JW) {
                int a, b;
                rr_pair(r, k, ne, a, b);
                if (b >= n) continue;
                T *wa = Wf + (int64_t)a * L, *wb = Wf + (int64_t)b * L;
                double al = 0.0, be = 0.0;
                T ga = zero<T>();
                for (int t = lane; t < L; t += 64) {
                    T x = wa[t], y = wb[t];
                    al += abs2(x);
                    be += abs2(y);
                    T pr = mul(cj(x), y);
                    ga = axpby(1.0, ga, 1.0, pr);
                }
                al = wsum(al);
                be = wsum(be);
                double agr, agi = 0.0;
                if constexpr (sizeof(T) == sizeof(double)) {
                    agr = wsum((double)*reinterpret_cast<double *>(&ga));
                } else {
                    cx<double> g2 = *reinterpret_cast<cx<double> *>(&ga);
                    agr = wsum(g2.re);
                    agi = wsum(g2.im);
                }
                double ag = sqrt(agr * agr + agi * agi);
                if (ag == 0.0 || ag <= tol * sqrt(al * be)) continue;
                // angle zeroing the off-diagonal of [[al, |g|], [|g|, be]]
                double zeta = (be - al) / (2.0 * ag);
                double tn = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + tn * tn), sn = cs * tn;
                T ph;  // exp(-i phi): makes the pair's Gram entry real
                if constexpr (sizeof(T) == sizeof(double)) {
                    *reinterpret_cast<double *>(&ph) = agr > 0 ? 1.0 : -1.0;
                } else {
                    *reinterpret_cast<cx<double> *>(&ph) = cx<double>{agr / ag, -agi / ag};
                }
                for (int t = lane; t < L; t += 64) {
                    T x = wa[t], y = mul(wb[t], ph);
                    wa[t] = axpby(cs, x, -sn, y);
                    wb[t] = axpby(sn, x, cs, y);
                }
                T *va = Vf + (int64_t)a * n, *vb = Vf + (int64_t)b * n;
                for (int t = lane; t < n; t += 64) {
                    T x = va[t], y = mul(vb[t], ph);
                    va[t] = axpby(cs, x, -sn, y);
                    vb[t] = axpby(sn, x, cs, y);
                }
                if (lane == 0) rotated = 1;
            }
            __syncthreads();
        }
        if (!rotated) {
            done = 1;
            break;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) sweeps_used[f] = (done || n <= 1) ? (n <= 1 ? 1 : sweep) : -1;
}

template <typename T>
__global__ __launch_bounds__(JT) void k_jac_finish(int64_t m, int64_t p, int64_t kmax,
                                                   const T *__restrict__ W, const T *__restrict__ V,
                                                   const double *__restrict__ fro2,
                                                   const int *__restrict__ sweeps_used, int mode,
                                                   int kfix, double tau, T *__restrict__ Uo,
                                                   double *__restrict__ So, T *__restrict__ Vo,
                                                   int32_t *__restrict__ ranks,
                                                   double *__restrict__ cert, double *__restrict__ fro,
                                                   int32_t *__restrict__ info) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t f = blockIdx.x;
    const bool tall = m >= p;
    const int L = (int)(tall ? m : p), n = (int)(tall ? p : m);
    double *nrm = reinterpret_cast<double *>(smem);       // [n]
    int *perm = reinterpret_cast<int *>(nrm + n);          // [n] perm[r] = vector of rank r
    __shared__ int kf_s;
    __shared__ double cert_s;
    const T *Wf = W + (int64_t)f * L * n;
    const T *Vf = V + (int64_t)f * n * n;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int j = wave; j < n; j += JW) {
        double acc = 0.0;
        for (int t = lane; t < L; t += 64) acc += abs2(Wf[(int64_t)j * L + t]);
        acc = wsum(acc);
        if (lane == 0) nrm[j] = sqrt(acc);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += JT) {  // stable descending order
        int pos = 0;
        double si = nrm[i];
        for (int j = 0; j < n; ++j) pos += sorts_before(nrm[j], j, si, i);
        perm[pos] = i;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int kf, miss = 0;
        const int cap = (int)(kmax < n ? kmax : n);
        if (mode == TSVDM_RANK_FIXED) {
            kf = kfix < n ? kfix : n;
        } else {
            int kc = kfix > 0 && kfix < cap ? kfix : cap;
            double bound = tau * tau * fro2[f], tail = 0.0;
            for (int j = 0; j < n; ++j) tail += nrm[perm[j]] * nrm[perm[j]];
            kf = -1;
            for (int k = 0; k <= kc; ++k) {
                if (tail <= bound) { kf = k; break; }
                if (k < n) tail -= nrm[perm[k]] * nrm[perm[k]];
            }
            if (kf < 0) {  // the tolerance is not met within the cap
                kf = kc;
                miss = 1;
            }
        }
        double disc = 0.0;
        for (int j = n - 1; j >= kf; --j) disc += nrm[perm[j]] * nrm[perm[j]];
        kf_s = kf;
        cert_s = sqrt(disc);
        ranks[f] = kf;
        if (cert) cert[f] = sqrt(disc);
        if (fro) fro[f] = sqrt(fro2[f]);
        if (info) info[f] = !isfinite(fro2[f]) ? 3 : sweeps_used[f] < 0 ? 1 : miss ? 4 : 0;
    }
    __syncthreads();
    const int kf = kf_s;
    for (int r = threadIdx.x; r < kmax; r += JT) So[f * kmax + r] = r < kf ? nrm[perm[r]] : 0.0;
    // U: m x kmax, V: p x kmax
    for (int64_t e = threadIdx.x; e < m * kmax; e += JT) {
        int r = (int)(e / m), i = (int)(e % m);
        T v = zero<T>();
        if (r < kf) {
            int j = perm[r];
            if (tall) {
                double s = nrm[j];
                v = s > 0 ? scale(Wf[(int64_t)j * L + i], 1.0 / s) : zero<T>();
            } else {
                v = Vf[(int64_t)j * n + i];
            }
        }
        Uo[f * m * kmax + e] = v;
    }
    for (int64_t e = threadIdx.x; e < p * kmax; e += JT) {
        int r = (int)(e / p), i = (int)(e % p);
        T v = zero<T>();
        if (r < kf) {
            int j = perm[r];
            if (tall) {
                v = Vf[(int64_t)j * n + i];
            } else {
                double s = nrm[j];
                v = s > 0 ? scale(Wf[(int64_t)j * L + i], 1.0 / s) : zero<T>();
            }
        }
        Vo[f * p * kmax + e] = v;
    }
    (void)cert_s;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <typename T>
tsvdm_status run_jacobi(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, tsvdm_factors *F,
                        void *ws, hipStream_t s) {
    const int64_t m = X->m, p = X->p, nf = X->n3;
    const int64_t L = m >= p ? m : p, n = m >= p ? p : m;
    char *w = reinterpret_cast<char *>(ws);
    T *W = reinterpret_cast<T *>(w);
    w += align256(sizeof(T) * nf * L * n);
    T *V = reinterpret_cast<T *>(w);
    w += align256(sizeof(T) * nf * n * n);
    double *fro2 = reinterpret_cast<double *>(w);
    w += align256(sizeof(double) * nf);
    int *sw = reinterpret_cast<int *>(w);
    const int maxsw = o->max_sweeps > 0 ? o->max_sweeps : 60;
    TSVDM_LAUNCH("jacobi_prepare", k_jac_prepare<T>, dim3((unsigned)nf), dim3(JT), 0, s,
                       reinterpret_cast<const T *>(X->data), m, p, W, V, fro2);
    TSVDM_LAUNCH_CHECK("k_jac_prepare");
    TSVDM_LAUNCH("jacobi_sweeps", k_jac_sweeps<T>, dim3((unsigned)nf), dim3(JT), 0, s, m, p, W, V, maxsw,
                       1e-15, sw);
    TSVDM_LAUNCH_CHECK("k_jac_sweeps");
    size_t lds = (sizeof(double) + sizeof(int)) * (size_t)n;
    TSVDM_LAUNCH("jacobi_finish", k_jac_finish<T>, dim3((unsigned)nf), dim3(JT), lds, s, m, p, F->kmax, W, V,
                       fro2, sw, o->rank_mode, o->k, o->tau, reinterpret_cast<T *>(F->U), F->S,
                       reinterpret_cast<T *>(F->V), F->ranks, F->cert, F->fro, F->info);
    TSVDM_LAUNCH_CHECK("k_jac_finish");
    return TSVDM_OK;
}

}  // namespace

namespace tsvdm {

size_t jacobi_workspace(int64_t m, int64_t p, int64_t nf, bool cplx) {
    const int64_t L = m >= p ? m : p, n = m >= p ? p : m;
    const size_t es = cplx ? 16 : 8;
    return align256(es * nf * L * n) + align256(es * nf * n * n) + align256(8 * nf) +
           align256(4 * nf);
}

tsvdm_status launch_jacobi_truncate(const tsvdm_tensor *X, const tsvdm_truncate_opts *o,
                                    tsvdm_factors *F, void *ws, hipStream_t s) {
    const int64_t n = X->m < X->p ? X->m : X->p;
    if (n > 4096) {
        set_error("PREC_F64: min(m, p) = %lld exceeds 4096", (long long)n);
        return TSVDM_EUNSUPPORTED;
    }
    if (X->dtype == TSVDM_C128) return run_jacobi<cx<double>>(X, o, F, ws, s);
    return run_jacobi<double>(X, o, F, ws, s);
}

}  // namespace tsvdm
