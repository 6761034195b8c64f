// Mixed-precision randomized facewise truncated SVD (PREC_MIXED).
//
// For every face X_f (m x p, FP32) of the transform-domain tensor, with the
// caller's Gaussian test matrix Omega (p x ell, ell = k + oversample):
//
//   Y  = X Omega            BF16 MFMA, FP32 accumulation        (pass 1, + ||X||^2)
//   Q  = qr(Y)              FP64 shifted Cholesky-QR3
//   Z  = X^T Q              BF16 MFMA                            (pass 2)
//   Qz = qr(Z)              FP64 shifted Cholesky-QR3
//   Y' = X Qz               split-BF16 MFMA (hi*hi + hi*lo + lo*hi), FP32-accurate (pass 3)
//   Q  = qr(Y')             FP64 shifted Cholesky-QR3
//   B^T = X^T Q             split-BF16 MFMA                      (pass 4)
//   B B^T = U_B L U_B^T     FP64 Gram + cyclic Jacobi eigensolver, s = sqrt(L)
//   Uhat = Q U_B, Vhat = B^T U_B / s, truncated to k_f
//   cert = ||X - Uhat S Vhat^T||_F  (explicit residual pass 5, FP64 sums)
//
// This is the randomized range finder with power iteration of Halko,
// Martinsson & Tropp (2011), applied face by face.  Only the first sketch
// and the first power half-step run in plain BF16: the range they find is
// refined by the FP32-accurate last half-step, so BF16 rounding of the data
// does not limit the accuracy (the last half-step maps any basis that sees
// the dominant right subspace onto the exact dominant left subspace).
//
// The passes over X are HBM-bound skinny GEMMs (N = ell <= 64); every
// workgroup stages a 64-row (or 64-column) slab of one face through LDS,
// converting FP32 to BF16 on the way, and the four wavefronts each drive
// 16 x 16 MFMA tiles.  The small FP64 steps use one workgroup per face.
#include "common.h"

#include <math.h>

using namespace tsvdm;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int GT = 256;  // threads per workgroup
enum { PROD_BF16 = 0, PROD_SPLIT = 1 };

__device__ __forceinline__ void split_bf16(float x, uint16_t &hi, uint16_t &lo) {
    hi = f2bf(x);
    lo = f2bf(x - bf2f(hi));
}

__device__ __forceinline__ f32x4 mfma(const u16x8 &a, const u16x8 &b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// ---------------------------------------------------------------- Y = X W
// Grid (ceil(m/64), nf).  Workgroup: rows a0..a0+63 of face f, all LP
// columns of the result; K = p in chunks of 32.  W (p x nw used columns,
// leading dim ldw) is per face (stride w_stride) or shared (w_stride = 0).
// Both the X slab and the W chunk are converted to BF16 (hi, and lo for the
// split product) once per workgroup and staged in LDS with K contiguous, so
// each lane's MFMA operand is one 16-byte LDS read.
template <int LP, int PROD>
__global__ __launch_bounds__(GT) void k_xw(const float *__restrict__ X, int m, int p,
                                           const float *__restrict__ W, int64_t w_stride, int ldw,
                                           int nw, float *__restrict__ Y,
                                           double *__restrict__ fro_part) {
    constexpr int KC = 32, LDK = KC + 8;  // LDS row pitch (bf16 elements)
    constexpr int NB = LP / 16;
    constexpr bool SPL = PROD == PROD_SPLIT;
    __shared__ __align__(16) uint16_t xh[64 * LDK];
    __shared__ __align__(16) uint16_t xl[SPL ? 64 * LDK : 8];
    __shared__ __align__(16) uint16_t wh[LP * LDK];
    __shared__ __align__(16) uint16_t wl[SPL ? LP * LDK : 8];
    __shared__ double red[GT / 64];
    const int f = blockIdx.y, a0 = blockIdx.x * 64;
    const float *Xf = X + (int64_t)f * m * p;
    const float *Wf = W + (int64_t)f * w_stride;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = tid & 63, kg = tid >> 6;  // X load mapping: row, 8-column group
    f32x4 acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = f32x4{0, 0, 0, 0};
    double fro = 0.0;
    const bool rok = a0 + lr < m;
    for (int b0 = 0; b0 < p; b0 += KC) {
        u16x8 h, l;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            int b = b0 + 8 * kg + v;
            float x = (rok && b < p) ? Xf[(a0 + lr) + (int64_t)m * b] : 0.0f;
            fro += (double)x * (double)x;
            uint16_t hh, ll;
            split_bf16(x, hh, ll);
            h[v] = hh;
            l[v] = ll;
        }
        *reinterpret_cast<u16x8 *>(&xh[lr * LDK + 8 * kg]) = h;
        if (SPL) *reinterpret_cast<u16x8 *>(&xl[lr * LDK + 8 * kg]) = l;
        for (int e = tid; e < KC * LP; e += GT) {
            int k = e % KC, c = e / KC, b = b0 + k;
            float w = (c < nw && b < p) ? Wf[b + (int64_t)ldw * c] : 0.0f;
            uint16_t hh, ll;
            split_bf16(w, hh, ll);
            wh[c * LDK + k] = hh;
            if (SPL) wl[c * LDK + k] = ll;
        }
        __syncthreads();
        const int ar = 16 * wave + (lane & 15), kq = 8 * (lane >> 4);
        u16x8 Ah = *reinterpret_cast<const u16x8 *>(&xh[ar * LDK + kq]);
        u16x8 Al;
        if (SPL) Al = *reinterpret_cast<const u16x8 *>(&xl[ar * LDK + kq]);
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int c = 16 * j + (lane & 15);
            u16x8 Bh = *reinterpret_cast<const u16x8 *>(&wh[c * LDK + kq]);
            acc[j] = mfma(Ah, Bh, acc[j]);
            if (SPL) {
                u16x8 Bl = *reinterpret_cast<const u16x8 *>(&wl[c * LDK + kq]);
                acc[j] = mfma(Ah, Bl, acc[j]);
                acc[j] = mfma(Al, Bh, acc[j]);
            }
        }
        __syncthreads();
    }
    float *Yf = Y + (int64_t)f * m * LP;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int c = 16 * j + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int r = a0 + 16 * wave + 4 * (lane >> 4) + v;
            if (r < m) Yf[r + (int64_t)m * c] = acc[j][v];
        }
    }
    if (fro_part) {
        fro = wave_sum(fro);
        if (lane == 0) red[wave] = fro;
        __syncthreads();
        if (tid == 0) fro_part[(int64_t)f * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

// ---------------------------------------------------------------- Z = X^T W
// Grid (ceil(p/64), nf).  Workgroup: output rows b0..b0+63 (columns of the
// face), K = m in chunks of 64.  W is m x nw (leading dim ldw), per face.
template <int LP, int PROD>
__global__ __launch_bounds__(GT) void k_xtw(const float *__restrict__ X, int m, int p,
                                            const float *__restrict__ W, int64_t w_stride, int ldw,
                                            int nw, float *__restrict__ Z) {
    constexpr int KC = 64, LDK = KC + 8;
    constexpr int NB = LP / 16;
    constexpr bool SPL = PROD == PROD_SPLIT;
    __shared__ __align__(16) uint16_t xh[64 * LDK];
    __shared__ __align__(16) uint16_t xl[SPL ? 64 * LDK : 8];
    __shared__ __align__(16) uint16_t wh[LP * LDK];
    __shared__ __align__(16) uint16_t wl[SPL ? LP * LDK : 8];
    const int f = blockIdx.y, b0 = blockIdx.x * 64;
    const float *Xf = X + (int64_t)f * m * p;
    const float *Wf = W + (int64_t)f * w_stride;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int q4 = tid & 15, cj0 = tid >> 4;  // X load mapping: 4 rows, column
    f32x4 acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = f32x4{0, 0, 0, 0};
    for (int a0 = 0; a0 < m; a0 += KC) {
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int cj = cj0 + 16 * it, b = b0 + cj;
            uint16_t hh[4], ll[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int a = a0 + 4 * q4 + v;
                float x = (b < p && a < m) ? Xf[a + (int64_t)m * b] : 0.0f;
                split_bf16(x, hh[v], ll[v]);
            }
            uint2 ph, pl;
            ph.x = hh[0] | ((uint32_t)hh[1] << 16);
            ph.y = hh[2] | ((uint32_t)hh[3] << 16);
            pl.x = ll[0] | ((uint32_t)ll[1] << 16);
            pl.y = ll[2] | ((uint32_t)ll[3] << 16);
            *reinterpret_cast<uint2 *>(&xh[cj * LDK + 4 * q4]) = ph;
            if (SPL) *reinterpret_cast<uint2 *>(&xl[cj * LDK + 4 * q4]) = pl;
        }
        for (int e = tid; e < KC * LP; e += GT) {
            int k = e % KC, c = e / KC, a = a0 + k;
            float w = (c < nw && a < m) ? Wf[a + (int64_t)ldw * c] : 0.0f;
            uint16_t hh, ll;
            split_bf16(w, hh, ll);
            wh[c * LDK + k] = hh;
            if (SPL) wl[c * LDK + k] = ll;
        }
        __syncthreads();
        const int br = 16 * wave + (lane & 15);
#pragma unroll
        for (int kk = 0; kk < KC / 32; ++kk) {
            const int kq = 32 * kk + 8 * (lane >> 4);
            u16x8 Ah = *reinterpret_cast<const u16x8 *>(&xh[br * LDK + kq]);
            u16x8 Al;
            if (SPL) Al = *reinterpret_cast<const u16x8 *>(&xl[br * LDK + kq]);
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int c = 16 * j + (lane & 15);
                u16x8 Bh = *reinterpret_cast<const u16x8 *>(&wh[c * LDK + kq]);
                acc[j] = mfma(Ah, Bh, acc[j]);
                if (SPL) {
                    u16x8 Bl = *reinterpret_cast<const u16x8 *>(&wl[c * LDK + kq]);
                    acc[j] = mfma(Ah, Bl, acc[j]);
                    acc[j] = mfma(Al, Bh, acc[j]);
                }
            }
        }
        __syncthreads();
    }
    float *Zf = Z + (int64_t)f * p * LP;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int c = 16 * j + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int r = b0 + 16 * wave + 4 * (lane >> 4) + v;
            if (r < p) Zf[r + (int64_t)p * c] = acc[j][v];
        }
    }
}

// ---------------------------------------------------------------- FP64 Gram
// G = S^T S for the rows x LP panel S (leading dim rows) of FP32 values,
// accumulated in FP64 (products of two FP32 values are exact in FP64).
// Result in LDS G[LP][LP+1].  Every thread owns a BS x BS block (BS = LP/16).
template <int LP>
__device__ void gram64(const float *__restrict__ S, int rows, double *G, float *stage) {
    constexpr int BS = LP / 16, RC = 64;
    const int tid = threadIdx.x, bi = (tid >> 4) * BS, bj = (tid & 15) * BS;
    double acc[BS][BS];
#pragma unroll
    for (int i = 0; i < BS; ++i)
#pragma unroll
        for (int j = 0; j < BS; ++j) acc[i][j] = 0.0;
    for (int r0 = 0; r0 < rows; r0 += RC) {
        for (int e = tid; e < RC * LP; e += GT) {
            int r = e % RC, c = e / RC;
            stage[r * (LP + 1) + c] = r0 + r < rows ? S[(r0 + r) + (int64_t)rows * c] : 0.0f;
        }
        __syncthreads();
        for (int r = 0; r < RC; ++r) {
            double a[BS], b[BS];
#pragma unroll
            for (int i = 0; i < BS; ++i) a[i] = stage[r * (LP + 1) + bi + i];
#pragma unroll
            for (int j = 0; j < BS; ++j) b[j] = stage[r * (LP + 1) + bj + j];
#pragma unroll
            for (int i = 0; i < BS; ++i)
#pragma unroll
                for (int j = 0; j < BS; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < BS; ++i)
#pragma unroll
        for (int j = 0; j < BS; ++j) G[(bi + i) * (LP + 1) + bj + j] = acc[i][j];
    __syncthreads();
}

// ---------------------------------------------------------------- Cholesky-QR
// Q = S R^{-1} with G + shift I = R^T R, repeated `passes` times, the first
// one shifted if `shift_first` (Fukaya et al. 2020, shift
// 11 (rows*ell + ell(ell+1)) u ||S||_F^2).  One workgroup per face; columns
// ell..LP-1 of the panel are zero on input and output.
template <int LP>
__global__ __launch_bounds__(GT) void k_cholqr(const float *__restrict__ Sin, int rows, int ell,
                                               float *__restrict__ Qout, int passes, int shift_first,
                                               int32_t *__restrict__ qr_info) {
    constexpr int CH = GT;  // rows per triangular-solve chunk (one per thread)
    __shared__ double G[LP * (LP + 1)];
    __shared__ float chunk[CH * (LP + 1)];  // also the Gram staging area
    __shared__ double rinv[LP];
    __shared__ int bad;
    const int f = blockIdx.x, tid = threadIdx.x;
    const float *S = Sin + (int64_t)f * rows * LP;
    float *Q = Qout + (int64_t)f * rows * LP;
    if (tid == 0) bad = 0;
    for (int pass = 0; pass < passes; ++pass) {
        const float *src = pass == 0 ? S : Q;
        gram64<LP>(src, rows, G, chunk);
        if (tid == 0) {
            double tr = 0.0;
            for (int c = 0; c < ell; ++c) tr += G[c * (LP + 1) + c];
            double sh = 0.0;
            if (pass == 0 && shift_first)
                sh = 11.0 * ((double)rows * ell + (double)ell * (ell + 1)) * 0x1p-53 * tr;
            for (int c = 0; c < ell; ++c) G[c * (LP + 1) + c] += sh;
            for (int c = ell; c < LP; ++c) {
                for (int j = 0; j < LP; ++j) G[c * (LP + 1) + j] = G[j * (LP + 1) + c] = 0.0;
                G[c * (LP + 1) + c] = 1.0;
            }
        }
        __syncthreads();
        // right-looking Cholesky: row j of R = row j of G scaled by 1/sqrt(pivot)
        for (int j = 0; j < LP; ++j) {
            double piv = G[j * (LP + 1) + j];
            bool ok = piv > 0.0 && isfinite(piv);
            double d = ok ? sqrt(piv) : 1.0;
            // trailing update uses the unscaled row j (only rows i > j change)
            for (int e = tid; e < (LP - j - 1) * (LP - j - 1); e += GT) {
                int i = j + 1 + e / (LP - j - 1), c = j + 1 + e % (LP - j - 1);
                if (c >= i && ok) G[i * (LP + 1) + c] -= G[j * (LP + 1) + i] * G[j * (LP + 1) + c] / piv;
            }
            __syncthreads();
            for (int c = j + 1 + tid; c < LP; c += GT) G[j * (LP + 1) + c] = ok ? G[j * (LP + 1) + c] / d : 0.0;
            if (tid == 0) {
                G[j * (LP + 1) + j] = d;
                rinv[j] = 1.0 / d;
                if (!ok) bad = 1;
            }
            __syncthreads();
        }
        // forward substitution q R = s, one row per thread, in place in LDS;
        // the solved entries are stored as FP32 (the precision of Q), every
        // dot product is accumulated in FP64
        for (int r0 = 0; r0 < rows; r0 += CH) {
            const int nr = rows - r0 < CH ? rows - r0 : CH;
            for (int e = tid; e < CH * LP; e += GT) {
                int r = e % CH, c = e / CH;
                chunk[r * (LP + 1) + c] = r < nr ? src[(r0 + r) + (int64_t)rows * c] : 0.0f;
            }
            __syncthreads();
            float *row = chunk + tid * (LP + 1);
            for (int c = 0; c < ell; ++c) {
                double v = (double)row[c];
                for (int j = 0; j < c; ++j) v -= (double)row[j] * G[j * (LP + 1) + c];
                row[c] = (float)(v * rinv[c]);
            }
            for (int c = ell; c < LP; ++c) row[c] = 0.0f;
            __syncthreads();
            for (int e = tid; e < CH * LP; e += GT) {
                int r = e % CH, c = e / CH;
                if (r < nr) Q[(r0 + r) + (int64_t)rows * c] = chunk[r * (LP + 1) + c];
            }
            __syncthreads();
        }
    }
    if (tid == 0 && bad) qr_info[f] = 2;
}

// ---------------------------------------------------------------- core SVD
// B B^T from B^T (p x LP): FP64 Gram, cyclic Jacobi eigensolver with the
// round-robin ordering, eigenvalues sorted decreasing, rank rule.
template <int LP>
__global__ __launch_bounds__(GT) void k_core(const float *__restrict__ Bt, int p, int ell,
                                             const double *__restrict__ fro_part, int nparts,
                                             int mode, int kfix, double tau, int max_sweeps,
                                             double *__restrict__ UB, double *__restrict__ sig,
                                             int *__restrict__ perm_out, int *__restrict__ kf_out,
                                             double *__restrict__ fro2_out,
                                             int32_t *__restrict__ jinfo) {
    constexpr int EB = sizeof(double) * LP * (LP + 1), SB = sizeof(float) * 64 * (LP + 1);
    __shared__ double G[LP * (LP + 1)];
    __shared__ __align__(16) unsigned char eraw[EB > SB ? EB : SB];
    double *E = reinterpret_cast<double *>(eraw);  // eigenvectors, column c = vector c
    float *stage = reinterpret_cast<float *>(eraw);  // Gram staging, used before E
    __shared__ double cs[LP / 2][2];
    __shared__ int rot;
    __shared__ double lam[LP];
    __shared__ int perm[LP];
    const int f = blockIdx.x, tid = threadIdx.x;
    __shared__ double trace;
    gram64<LP>(Bt + (int64_t)f * p * LP, p, G, stage);
    if (tid == 0) {
        double t = 0.0;
        for (int c = 0; c < ell; ++c) t += G[c * (LP + 1) + c];
        trace = t;
    }
    for (int e = tid; e < LP * LP; e += GT) E[(e / LP) * (LP + 1) + e % LP] = (e / LP == e % LP) ? 1.0 : 0.0;
    const int ne = ell + (ell & 1);
    int sweep = 0, conv = 0;
    __syncthreads();
    for (sweep = 1; sweep <= max_sweeps && ell > 1; ++sweep) {
        if (tid == 0) rot = 0;
        __syncthreads();
        for (int r = 0; r < ne - 1; ++r) {
            if (tid < ne / 2) {
                int a, b, k = tid;
                if (k == 0) { a = r; b = ne - 1; }
                else { a = (r + k) % (ne - 1); b = (r - k + (ne - 1)) % (ne - 1); }
                if (a > b) { int t = a; a = b; b = t; }
                double c = 1.0, s = 0.0;
                if (b < ell) {
                    double app = G[a * (LP + 1) + a], aqq = G[b * (LP + 1) + b], apq = G[a * (LP + 1) + b];
                    // relative test (high relative accuracy for well separated pairs) and an
                    // absolute floor at the rounding level of the Gram matrix
                    if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && fabs(apq) > 1e-15 * trace) {
                        double zeta = (aqq - app) / (2.0 * apq);
                        double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = c * t;
                        rot = 1;
                    }
                }
                cs[k][0] = c;
                cs[k][1] = s;
            }
            __syncthreads();
            // rows: (row_a, row_b) <- (c row_a - s row_b, s row_a + c row_b)
            for (int e = tid; e < (ne / 2) * ell; e += GT) {
                int k = e / ell, col = e % ell, a, b;
                if (k == 0) { a = r; b = ne - 1; }
                else { a = (r + k) % (ne - 1); b = (r - k + (ne - 1)) % (ne - 1); }
                if (a > b) { int t = a; a = b; b = t; }
                if (b >= ell) continue;
                double c = cs[k][0], s = cs[k][1];
                double x = G[a * (LP + 1) + col], y = G[b * (LP + 1) + col];
                G[a * (LP + 1) + col] = c * x - s * y;
                G[b * (LP + 1) + col] = s * x + c * y;
            }
            __syncthreads();
            // columns of G and of E
            for (int e = tid; e < (ne / 2) * ell; e += GT) {
                int k = e / ell, row = e % ell, a, b;
                if (k == 0) { a = r; b = ne - 1; }
                else { a = (r + k) % (ne - 1); b = (r - k + (ne - 1)) % (ne - 1); }
                if (a > b) { int t = a; a = b; b = t; }
                if (b >= ell) continue;
                double c = cs[k][0], s = cs[k][1];
                double x = G[row * (LP + 1) + a], y = G[row * (LP + 1) + b];
                G[row * (LP + 1) + a] = c * x - s * y;
                G[row * (LP + 1) + b] = s * x + c * y;
                x = E[row * (LP + 1) + a];
                y = E[row * (LP + 1) + b];
                E[row * (LP + 1) + a] = c * x - s * y;
                E[row * (LP + 1) + b] = s * x + c * y;
            }
            __syncthreads();
        }
        if (!rot) { conv = 1; break; }
        __syncthreads();
    }
    if (tid < ell) lam[tid] = fmax(G[tid * (LP + 1) + tid], 0.0);
    __syncthreads();
    if (tid < ell) {
        int pos = 0;
        double li = lam[tid];
        for (int j = 0; j < ell; ++j) pos += (lam[j] > li) || (lam[j] == li && j < tid);
        perm[pos] = tid;
    }
    __syncthreads();
    if (tid == 0) {
        double fro2 = 0.0;
        for (int i = 0; i < nparts; ++i) fro2 += fro_part[(int64_t)f * nparts + i];
        int kf;
        if (mode == TSVDM_RANK_FIXED) {
            kf = kfix < ell ? kfix : ell;
        } else {
            int cap = kfix > 0 && kfix < ell ? kfix : ell;
            double tail = 0.0, bound = tau * tau * fro2;
            for (int j = 0; j < ell; ++j) tail += lam[j];
            kf = cap;
            for (int k = 0; k <= cap; ++k) {
                if (tail <= bound) { kf = k; break; }
                if (k < ell) tail -= lam[perm[k]];
            }
        }
        kf_out[f] = kf;
        fro2_out[f] = fro2;
        jinfo[f] = (conv || ell <= 1) ? 0 : 1;
    }
    for (int r = tid; r < LP; r += GT) {
        int j = r < ell ? perm[r] : r;
        sig[(int64_t)f * LP + r] = r < ell ? sqrt(lam[j]) : 0.0;
        perm_out[(int64_t)f * LP + r] = j;
    }
    for (int e = tid; e < LP * LP; e += GT)
        UB[(int64_t)f * LP * LP + e] = E[(e % LP) * (LP + 1) + e / LP];  // column major, col = e/LP
}

// ---------------------------------------------------------------- factors
// Uhat[:, r] = Q U_B[:, perm[r]],  Vhat[:, r] = B^T U_B[:, perm[r]] / s_r  (r < k_f)
template <int LP>
__global__ __launch_bounds__(GT) void k_factors(const float *__restrict__ Q, const float *__restrict__ Bt,
                                                int m, int p, int ell, int64_t kmax,
                                                const double *__restrict__ UB,
                                                const double *__restrict__ sig,
                                                const int *__restrict__ perm,
                                                const int *__restrict__ kf_in,
                                                const double *__restrict__ fro2,
                                                const int32_t *__restrict__ qr_info,
                                                const int32_t *__restrict__ jinfo,
                                                float *__restrict__ Uo, double *__restrict__ So,
                                                float *__restrict__ Vo, int32_t *__restrict__ ranks,
                                                double *__restrict__ fro, int32_t *__restrict__ info) {
    __shared__ double ub[LP * LP];  // ub[c * LP + r] = U_B[c, perm[r]] (and / s_r for V)
    __shared__ double ubv[LP * LP];
    const int f = blockIdx.y, tid = threadIdx.x;
    const int kf = kf_in[f];
    for (int e = tid; e < LP * LP; e += GT) {
        int c = e / LP, r = e % LP;
        double u = 0.0, v = 0.0;
        if (r < kf && c < ell) {
            int j = perm[(int64_t)f * LP + r];
            double s = sig[(int64_t)f * LP + r];
            u = UB[(int64_t)f * LP * LP + c + (int64_t)LP * j];
            v = s > 0.0 ? u / s : 0.0;
        }
        ub[e] = u;
        ubv[e] = v;
    }
    __syncthreads();
    const int row = blockIdx.x * GT + tid;
    if (row < m) {
        const float *Qf = Q + (int64_t)f * m * LP;
        double qv[LP];
#pragma unroll
        for (int c = 0; c < LP; ++c) qv[c] = Qf[row + (int64_t)m * c];
        for (int r = 0; r < kmax; ++r) {
            double acc = 0.0;
            if (r < kf) {
#pragma unroll
                for (int c = 0; c < LP; ++c) acc += qv[c] * ub[c * LP + (r < LP ? r : 0)];
            }
            Uo[(int64_t)f * m * kmax + row + (int64_t)m * r] = (float)acc;
        }
    }
    if (row < p) {
        const float *Bf = Bt + (int64_t)f * p * LP;
        double bv[LP];
#pragma unroll
        for (int c = 0; c < LP; ++c) bv[c] = Bf[row + (int64_t)p * c];
        for (int r = 0; r < kmax; ++r) {
            double acc = 0.0;
            if (r < kf) {
#pragma unroll
                for (int c = 0; c < LP; ++c) acc += bv[c] * ubv[c * LP + (r < LP ? r : 0)];
            }
            Vo[(int64_t)f * p * kmax + row + (int64_t)p * r] = (float)acc;
        }
    }
    if (blockIdx.x == 0) {
        for (int r = tid; r < kmax; r += GT) So[(int64_t)f * kmax + r] = r < kf ? sig[(int64_t)f * LP + r] : 0.0;
        if (tid == 0) {
            ranks[f] = kf;
            if (fro) fro[f] = sqrt(fro2[f]);
            if (info) {
                int code = 0;
                if (jinfo[f]) code = 1;
                if (qr_info[f]) code = 2;
                if (!isfinite(fro2[f])) code = 3;
                info[f] = code;
            }
        }
    }
}

// ---------------------------------------------------------------- certificate
// partial sums of (X - Uhat S Vhat^T)^2 over 64-row slabs, FP64 accumulation
__global__ __launch_bounds__(GT) void k_resid(const float *__restrict__ X, int m, int p,
                                              const float *__restrict__ U, const double *__restrict__ S,
                                              const float *__restrict__ V, int64_t kmax,
                                              const int32_t *__restrict__ ranks,
                                              double *__restrict__ part) {
    __shared__ float us[64 * 65];
    __shared__ float vs[64 * 65];
    __shared__ double red[GT / 64];
    const int f = blockIdx.y, a0 = blockIdx.x * 64, tid = threadIdx.x;
    const int kf = ranks[f] < 64 ? ranks[f] : 64;
    const float *Xf = X + (int64_t)f * m * p;
    const float *Uf = U + (int64_t)f * m * kmax;
    const float *Vf = V + (int64_t)f * p * kmax;
    for (int e = tid; e < 64 * 64; e += GT) {
        int r = e % 64, j = e / 64;
        us[r * 65 + j] = (j < kf && a0 + r < m) ? (float)(Uf[(a0 + r) + (int64_t)m * j] * S[(int64_t)f * kmax + j]) : 0.0f;
    }
    double acc = 0.0;
    const int r = tid & 63;
    for (int b0 = 0; b0 < p; b0 += 64) {
        __syncthreads();
        for (int e = tid; e < 64 * 64; e += GT) {
            int c = e % 64, j = e / 64;
            vs[c * 65 + j] = (j < kf && b0 + c < p) ? Vf[(b0 + c) + (int64_t)p * j] : 0.0f;
        }
        __syncthreads();
        for (int c = tid >> 6; c < 64; c += GT / 64) {
            if (a0 + r >= m || b0 + c >= p) continue;
            float pr = 0.0f;
            for (int j = 0; j < kf; ++j) pr = fmaf(us[r * 65 + j], vs[c * 65 + j], pr);
            double d = (double)Xf[(a0 + r) + (int64_t)m * (b0 + c)] - (double)pr;
            acc += d * d;
        }
    }
    acc = wave_sum(acc);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) part[(int64_t)f * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_cert(const double *__restrict__ part, int nparts, int nf, double *__restrict__ cert) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += part[(int64_t)f * nparts + i];
    cert[f] = sqrt(s);
}

__global__ void k_fill(double *__restrict__ x, int n, double v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ void k_zero_i32(int32_t *__restrict__ x, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0;
}

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct MixedWs {
    float *Y, *Qm, *Z, *Qp;
    double *fro_part, *res_part, *UB, *sig, *fro2;
    int *perm, *kf;
    int32_t *qr_info, *jinfo;
};

size_t carve(char *base, int64_t m, int64_t p, int64_t nf, int LP, MixedWs *w) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *ptr = base ? base + off : nullptr;
        off += al256(bytes);
        return ptr;
    };
    const int64_t mparts = (m + 63) / 64;
    MixedWs t;
    t.Y = (float *)take(sizeof(float) * nf * m * LP);
    t.Qm = (float *)take(sizeof(float) * nf * m * LP);
    t.Z = (float *)take(sizeof(float) * nf * p * LP);
    t.Qp = (float *)take(sizeof(float) * nf * p * LP);
    t.fro_part = (double *)take(sizeof(double) * nf * mparts);
    t.res_part = (double *)take(sizeof(double) * nf * mparts);
    t.UB = (double *)take(sizeof(double) * nf * LP * LP);
    t.sig = (double *)take(sizeof(double) * nf * LP);
    t.fro2 = (double *)take(sizeof(double) * nf);
    t.perm = (int *)take(sizeof(int) * nf * LP);
    t.kf = (int *)take(sizeof(int) * nf);
    t.qr_info = (int32_t *)take(sizeof(int32_t) * nf);
    t.jinfo = (int32_t *)take(sizeof(int32_t) * nf);
    if (w) *w = t;
    return off;
}

template <int LP>
tsvdm_status run_mixed(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, tsvdm_factors *F,
                       void *wsp, hipStream_t s) {
    const int m = (int)X->m, p = (int)X->p, nf = (int)X->n3, ell = o->k + o->oversample;
    MixedWs w;
    carve(reinterpret_cast<char *>(wsp), m, p, nf, LP, &w);
    const float *Xd = reinterpret_cast<const float *>(X->data);
    const dim3 gm((m + 63) / 64, nf), gp((p + 63) / 64, nf);
    const int mparts = (m + 63) / 64;
    hipLaunchKernelGGL(k_zero_i32, dim3((nf + 255) / 256), dim3(256), 0, s, w.qr_info, nf);
    // pass 1: sketch
    hipLaunchKernelGGL((k_xw<LP, PROD_BF16>), gm, dim3(GT), 0, s, Xd, m, p, o->omega, (int64_t)0, p, ell,
                       w.Y, w.fro_part);
    hipLaunchKernelGGL((k_cholqr<LP>), dim3(nf), dim3(GT), 0, s, w.Y, m, ell, w.Qm, 3, 1, w.qr_info);
    const float *Qsrc = w.Qm;
    if (o->power_iters > 0) {
        // pass 2: Z = X^T Q
        hipLaunchKernelGGL((k_xtw<LP, PROD_BF16>), gp, dim3(GT), 0, s, Xd, m, p, w.Qm, (int64_t)m * LP, m,
                           LP, w.Z);
        hipLaunchKernelGGL((k_cholqr<LP>), dim3(nf), dim3(GT), 0, s, w.Z, p, ell, w.Qp, 3, 1, w.qr_info);
        // pass 3: Y' = X Qz, FP32-accurate
        hipLaunchKernelGGL((k_xw<LP, PROD_SPLIT>), gm, dim3(GT), 0, s, Xd, m, p, w.Qp, (int64_t)p * LP, p,
                           LP, w.Y, (double *)nullptr);
        hipLaunchKernelGGL((k_cholqr<LP>), dim3(nf), dim3(GT), 0, s, w.Y, m, ell, w.Qm, 3, 1, w.qr_info);
    }
    // pass 4: B^T = X^T Q, FP32-accurate
    hipLaunchKernelGGL((k_xtw<LP, PROD_SPLIT>), gp, dim3(GT), 0, s, Xd, m, p, Qsrc, (int64_t)m * LP, m, LP,
                       w.Z);
    const int msw = o->max_sweeps > 0 ? o->max_sweeps : 30;
    hipLaunchKernelGGL((k_core<LP>), dim3(nf), dim3(GT), 0, s, w.Z, p, ell, w.fro_part, mparts,
                       o->rank_mode, o->k, o->tau, msw, w.UB, w.sig, w.perm, w.kf, w.fro2, w.jinfo);
    const int rows = m > p ? m : p;
    hipLaunchKernelGGL((k_factors<LP>), dim3((rows + GT - 1) / GT, nf), dim3(GT), 0, s, Qsrc, w.Z, m, p,
                       ell, F->kmax, w.UB, w.sig, w.perm, w.kf, w.fro2, w.qr_info, w.jinfo,
                       reinterpret_cast<float *>(F->U), F->S, reinterpret_cast<float *>(F->V), F->ranks,
                       F->fro, F->info);
    if (F->cert) {
        if (o->certify) {
            hipLaunchKernelGGL(k_resid, gm, dim3(GT), 0, s, Xd, m, p,
                               reinterpret_cast<const float *>(F->U), F->S,
                               reinterpret_cast<const float *>(F->V), F->kmax, F->ranks, w.res_part);
            hipLaunchKernelGGL(k_cert, dim3((nf + 255) / 256), dim3(256), 0, s, w.res_part, mparts, nf,
                               F->cert);
        } else {
            hipLaunchKernelGGL(k_fill, dim3((nf + 255) / 256), dim3(256), 0, s, F->cert, nf, -1.0);
        }
    }
    TSVDM_LAUNCH_CHECK("mixed truncate");
    return TSVDM_OK;
}

}  // namespace

namespace tsvdm {

static int padded(int ell) { return ell <= 16 ? 16 : ell <= 32 ? 32 : ell <= 48 ? 48 : 64; }

size_t mixed_workspace(int64_t m, int64_t p, int64_t nf, int ell) {
    return carve(nullptr, m, p, nf, padded(ell), nullptr);
}

tsvdm_status launch_mixed_truncate(const tsvdm_tensor *X, const tsvdm_truncate_opts *o,
                                   tsvdm_factors *F, void *ws, hipStream_t s) {
    if (X->m > 65536 || X->p > 65536 || X->n3 > 65535) {
        set_error("PREC_MIXED: face dims up to 65536 and up to 65535 faces");
        return TSVDM_EUNSUPPORTED;
    }
    switch (padded(o->k + o->oversample)) {
        case 16: return run_mixed<16>(X, o, F, ws, s);
        case 32: return run_mixed<32>(X, o, F, ws, s);
        case 48: return run_mixed<48>(X, o, F, ws, s);
        default: return run_mixed<64>(X, o, F, ws, s);
    }
}

}  // namespace tsvdm
