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

// ---------------------------------------------------------------- matrix cores
// The same contraction on FP32 16x16x4 MFMAs (FP32 and BF16-rounded operands).
// k_apply_mfma reads its operands straight from memory and serves ranks 33..64;
// k_apply_lds below (ranks up to 32) stages them in LDS first.
// Workgroup: block row j, rows a0 .. a0+63 of it and 64 columns; wavefront w
// owns columns c0 + 16 w .. + 15 and all 64 rows.  Per stored face f:
//   Z(r, c) = sum_k conj(V(j + l k, r)) conj(xt(k, c))  (real M: no conj)
// in registers, 16 ranks per block (NRB blocks), over steps of 16 k: lane
// (l16, kl) = (lane % 16, lane / 16) holds xt(16 kk + 4 kl + t, c0 + 16 w + l16),
// t = 0..3, from one contiguous load, and MFMA step t takes entry t as its B
// operand, so the A operand (lane l16 = rank) takes V at the same k, read
// from a copy Vp whose rows j + l k of block row j are contiguous in k.  Then
//   y(a, c) += w_f Re(sum_r (U S)(a, r) Z(r, c))
// with Z straight from the accumulators: the FP32 16x16x4 output holds rank
// 4 kl + v of the block in entry v, so step s of the second product takes
// entry s as its B operand and (U S)(a, 16 rb + 4 kl + s) as its A operand.
// Complex products: Zr = Vr Xr - Vi Xi and nZi = Vr Xi + Vi Xr (= -Im Z), the
// latter as (Vr + Vi)(Xr + Xi) - Vr Xr - Vi Xi (three real products, Gauss),
// so Re(US Z) = USr Zr + USi nZi.  Elements that do not exist (k >= q, r >= rank,
// a >= m, c >= nrhs) load as zero through the 2^31 offset of a buffer
// resource per face (each under 2 GiB, checked on the host) or a select.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
constexpr uint32_t kMiss = 0x80000000u;

__device__ __forceinline__ uint32_t miss_if(bool bad) { return bad ? kMiss : 0u; }

// BF16 compute: four FP32 16x16x4 steps t = 0..3 of a lane take operands at
// k = 4 kl + t, which is the lane's operand of one BF16 16x16x16 MFMA (a lane
// holds k = 4 (lane/16) .. + 3 of its row, or column), with the same output
// layout; so each group of four FP32 MFMAs becomes one on BF16 operands
// (rounded to nearest even; V, x~ and U S are BF16 values already).
typedef short s16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ s16x4 pk4(float a, float b, float c, float d) {
    return s16x4{(short)f2bf(a), (short)f2bf(b), (short)f2bf(c), (short)f2bf(d)};
}
__device__ __forceinline__ f32x4 mfma_bf4(const s16x4 &a, const s16x4 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Vp_f(k + q j, r) = Vhat_f(j + l k, r): the rows a block row j takes, made
// contiguous in k (one thread per element of E floats, read in order)
template <int E>
__global__ __launch_bounds__(256) void k_vrelayout(const float *__restrict__ V, float *__restrict__ Vp, int64_t p,
                                                   int64_t ell, int64_t q, int64_t total) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= total) return;
    const int64_t col = i / p, b = i - col * p;  // col = r + kmax f
    const int64_t j = b % ell, k = b / ell;
    const int64_t o = col * p + k + q * j;
#pragma unroll
    for (int e = 0; e < E; ++e) Vp[o * E + e] = V[i * E + e];
}

template <bool CPLX, bool BF, int NRB>
__global__ __launch_bounds__(AT) void k_apply_mfma(const float *__restrict__ U, const double *__restrict__ S,
                                                   const float *__restrict__ Vp, const int32_t *__restrict__ ranks,
                                                   int m, int p, int kmax, int nf, int n3, int ell, int q,
                                                   const float *__restrict__ xt, int nrhs, float *__restrict__ y,
                                                   int64_t ldy) {
    constexpr int E = CPLX ? 2 : 1;
    const int kcap = kmax < 16 * NRB ? kmax : 16 * NRB;
    const int mtiles = (m + 63) >> 6;
    const int j = blockIdx.x / mtiles, a0 = (blockIdx.x % mtiles) * 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int l16 = lane & 15, kl = lane >> 4;
    const int c = blockIdx.y * 64 + 16 * w + l16;
    const bool cok = c < nrhs;
    const int nkk = (q + 15) >> 4;
    f32x4 acc[4];
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) acc[ab] = f32x4{0, 0, 0, 0};
    for (int f = 0; f < nf; ++f) {
        int kf = ranks[f];
        kf = kf < kcap ? kf : kcap;
        if (kf <= 0) continue;
        const float wgt = (CPLX && !(f == 0 || 2 * f == n3)) ? 2.0f : 1.0f;
        const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float *>(xt) + (int64_t)f * q * nrhs * E, 0, q * nrhs * E * 4, 0x00020000);
        const __amdgpu_buffer_rsrc_t rv = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float *>(Vp) + (int64_t)f * p * kmax * E, 0, p * kmax * E * 4, 0x00020000);
        const __amdgpu_buffer_rsrc_t ru = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float *>(U) + (int64_t)f * m * kmax * E, 0, m * kmax * E * 4, 0x00020000);
        // complex: zr, zi and z3 collect Vr Xr, Vi Xi and (Vr + Vi)(Xr + Xi)
        // (three real products per complex one); Zr and nZi are formed after
        // the k loop
        f32x4 zr[NRB], zi[NRB], z3[NRB];
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) zr[rb] = zi[rb] = z3[rb] = f32x4{0, 0, 0, 0};
        for (int kk = 0; kk < nkk; ++kk) {
            const int k0 = 16 * kk + 4 * kl;
            // B operand: xt(k0 .. k0+3, c)
            const uint32_t xo = (((uint32_t)k0 + (uint32_t)q * (uint32_t)c) * (4u * E)) | miss_if(!cok || k0 >= q);
            float xr[4], xi[4];
            if (CPLX) {
                const u32x4 x01 = __builtin_amdgcn_raw_buffer_load_b128(rx, (int)xo, 0, 0);
                const u32x4 x23 = __builtin_amdgcn_raw_buffer_load_b128(rx, (int)(xo + 16u), 0, 0);
                const uint32_t e0 = x01.x, e1 = x01.y, e2 = x01.z, e3 = x01.w;
                const uint32_t e4 = x23.x, e5 = x23.y, e6 = x23.z, e7 = x23.w;
                xr[0] = __uint_as_float(e0); xi[0] = __uint_as_float(e1);
                xr[1] = __uint_as_float(e2); xi[1] = __uint_as_float(e3);
                xr[2] = __uint_as_float(e4); xi[2] = __uint_as_float(e5);
                xr[3] = __uint_as_float(e6); xi[3] = __uint_as_float(e7);
            } else {
                const u32x4 x03 = __builtin_amdgcn_raw_buffer_load_b128(rx, (int)xo, 0, 0);
                const uint32_t e0 = x03.x, e1 = x03.y, e2 = x03.z, e3 = x03.w;
                xr[0] = __uint_as_float(e0); xr[1] = __uint_as_float(e1);
                xr[2] = __uint_as_float(e2); xr[3] = __uint_as_float(e3);
                xi[0] = xi[1] = xi[2] = xi[3] = 0.0f;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const bool kin = k0 + t < q;  // a partial last group reads the next column
                xr[t] = kin ? (BF ? rbf(xr[t]) : xr[t]) : 0.0f;
                xi[t] = kin ? (BF ? rbf(xi[t]) : xi[t]) : 0.0f;
            }
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb) {
                const int r = 16 * rb + l16;
                // A operand: Vp(k0 .. k0+3 + q j, r), zero past the rank or q
                const uint32_t vo =
                    (((uint32_t)k0 + (uint32_t)q * (uint32_t)j + (uint32_t)p * (uint32_t)r) * (4u * E)) |
                    miss_if(r >= kf || k0 >= q);
                float vra[4], via[4];
                if (CPLX) {
                    const u32x4 v01 = __builtin_amdgcn_raw_buffer_load_b128(rv, (int)vo, 0, 0);
                    const uint32_t g0 = v01.x, g1 = v01.y, g2 = v01.z, g3 = v01.w;
                    const u32x4 v23 = __builtin_amdgcn_raw_buffer_load_b128(rv, (int)(vo + 16u), 0, 0);
                    const uint32_t g4 = v23.x, g5 = v23.y, g6 = v23.z, g7 = v23.w;
                    vra[0] = __uint_as_float(g0); via[0] = __uint_as_float(g1);
                    vra[1] = __uint_as_float(g2); via[1] = __uint_as_float(g3);
                    vra[2] = __uint_as_float(g4); via[2] = __uint_as_float(g5);
                    vra[3] = __uint_as_float(g6); via[3] = __uint_as_float(g7);
                } else {
                    const u32x4 v03 = __builtin_amdgcn_raw_buffer_load_b128(rv, (int)vo, 0, 0);
                    const uint32_t g0 = v03.x, g1 = v03.y, g2 = v03.z, g3 = v03.w;
                    vra[0] = __uint_as_float(g0); vra[1] = __uint_as_float(g1);
                    vra[2] = __uint_as_float(g2); vra[3] = __uint_as_float(g3);
                    via[0] = via[1] = via[2] = via[3] = 0.0f;
                }
                float vrt[4], vit[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    // a partial last group reads the next block row's rows
                    const bool kin = k0 + t < q;
                    vrt[t] = kin ? vra[t] : 0.0f;
                    vit[t] = kin ? via[t] : 0.0f;
                    if (BF) {
                        vrt[t] = rbf(vrt[t]);
                        vit[t] = rbf(vit[t]);
                    }
                }
                if constexpr (BF) {
                    zr[rb] = mfma_bf4(pk4(vrt[0], vrt[1], vrt[2], vrt[3]), pk4(xr[0], xr[1], xr[2], xr[3]), zr[rb]);
                    if (CPLX) {
                        zi[rb] = mfma_bf4(pk4(vit[0], vit[1], vit[2], vit[3]), pk4(xi[0], xi[1], xi[2], xi[3]), zi[rb]);
                        z3[rb] = mfma_bf4(pk4(vrt[0] + vit[0], vrt[1] + vit[1], vrt[2] + vit[2], vrt[3] + vit[3]),
                                          pk4(xr[0] + xi[0], xr[1] + xi[1], xr[2] + xi[2], xr[3] + xi[3]), z3[rb]);
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        zr[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(vrt[t], xr[t], zr[rb], 0, 0, 0);
                        if (CPLX) {
                            zi[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(vit[t], xi[t], zi[rb], 0, 0, 0);
                            z3[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(vrt[t] + vit[t], xr[t] + xi[t], z3[rb], 0, 0, 0);
                        }
                    }
                }
            }
        }
        if (CPLX) {
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb) {
                const f32x4 p1 = zr[rb], p2 = zi[rb];
                zr[rb] = p1 - p2;          // Vr Xr - Vi Xi
                zi[rb] = z3[rb] - p1 - p2; // Vr Xi + Vi Xr = -Im Z
            }
        }
        // y += w Re(U S Z): A operand (U S)(a0 + 16 ab + l16, 16 rb + 4 kl + s)
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) {
            float bu[4][4], bv[4][4];  // BF16 compute: (U S w) of the four steps, per ab
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int r = 16 * rb + 4 * kl + s;
                const bool rin = r < kf;
                const double sr = rin ? S[(int64_t)f * kmax + r] : 0.0;
                const float bzr = zr[rb][s];
                const float bzi = zi[rb][s];
#pragma unroll
                for (int ab = 0; ab < 4; ++ab) {
                    const int a = a0 + 16 * ab + l16;
                    const uint32_t uo = (((uint32_t)a + (uint32_t)m * (uint32_t)r) * (4u * E)) | miss_if(!rin || a >= m);
                    float ur, ui = 0.0f;
                    if (CPLX) {
                        const u32x2 u2 = __builtin_amdgcn_raw_buffer_load_b64(ru, (int)uo, 0, 0);
                        const uint32_t g0 = u2.x, g1 = u2.y;
                        ur = __uint_as_float(g0);
                        ui = __uint_as_float(g1);
                    } else {
                        ur = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ru, (int)uo, 0, 0));
                    }
                    // (U S) rounded as stored by the plain kernel, then the
                    // exact conjugate-pair weight
                    float usr = (float)((double)ur * sr), usi = (float)((double)ui * sr);
                    if (BF) {
                        usr = rbf(usr);
                        usi = rbf(usi);
                        bu[ab][s] = usr * wgt;
                        bv[ab][s] = usi * wgt;
                    } else {
                        acc[ab] = __builtin_amdgcn_mfma_f32_16x16x4f32(usr * wgt, bzr, acc[ab], 0, 0, 0);
                        if (CPLX) acc[ab] = __builtin_amdgcn_mfma_f32_16x16x4f32(usi * wgt, bzi, acc[ab], 0, 0, 0);
                    }
                }
            }
            if constexpr (BF) {
                const float z0 = zr[rb][0], z1 = zr[rb][1], z2 = zr[rb][2], z3v = zr[rb][3];
                const float w0 = zi[rb][0], w1 = zi[rb][1], w2 = zi[rb][2], w3 = zi[rb][3];
#pragma unroll
                for (int ab = 0; ab < 4; ++ab) {
                    acc[ab] = mfma_bf4(pk4(bu[ab][0], bu[ab][1], bu[ab][2], bu[ab][3]), pk4(z0, z1, z2, z3v), acc[ab]);
                    if (CPLX)
                        acc[ab] = mfma_bf4(pk4(bv[ab][0], bv[ab][1], bv[ab][2], bv[ab][3]), pk4(w0, w1, w2, w3), acc[ab]);
                }
            }
        }
    }
    // FP32 16x16x4 output: row 4 kl + v of block ab, column l16
    if (cok) {
#pragma unroll
        for (int ab = 0; ab < 4; ++ab)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = a0 + 16 * ab + 4 * kl + v;
                if (a < m) y[((int64_t)j * m + a) + ldy * c] = acc[ab][v];
            }
    }
}

// Ranks <= 32: the same products with the workgroup's operands staged in LDS.
// Per face and chunk of 32 k, the 256 threads copy x~ (64 columns), the 16 NRB
// rank rows of Vp and, on the first chunk, U S w (64 rows, rounded as the
// plain kernel rounds it) with 16-byte loads, consecutive lanes on
// consecutive 16-byte pieces of one column or row; elements that do not
// exist are stored as zero.  Columns of x~ and rows of Vp are padded by 16
// bytes (no bank conflicts for the 16-byte operand reads).  The four
// wavefronts then read their MFMA operands from LDS in the layout above.
// The global loads of the next stage (face, chunk) are issued before the
// current stage's products.
template <bool CPLX, bool BF, int NRB>
__global__ __launch_bounds__(AT) void k_apply_lds(const float *__restrict__ U, const double *__restrict__ S,
                                                  const float *__restrict__ Vp, const int32_t *__restrict__ ranks,
                                                  int m, int p, int kmax, int nf, int n3, int ell, int q,
                                                  const float *__restrict__ xt, int nrhs, float *__restrict__ y,
                                                  int64_t ldy) {
    constexpr int E = CPLX ? 2 : 1;
    constexpr int KC = 32;              // k per chunk
    constexpr int XS = KC * E + 4;      // floats per staged column of x~ or row of Vp
    constexpr int RK = 16 * NRB;        // ranks held
    constexpr int US = RK * E + 4;      // floats per staged row of U S
    constexpr int KPC = 4 / E;          // k (or rows a) per 16-byte piece
    constexpr int CH = KC / KPC;        // pieces per column
    __shared__ __align__(16) float xs[64 * XS];
    __shared__ __align__(16) float vs[RK * XS];
    __shared__ __align__(16) float us[64 * US];
    const int kcap = kmax < RK ? kmax : RK;
    const int mtiles = (m + 63) >> 6;
    const int j = blockIdx.x / mtiles, a0 = (blockIdx.x % mtiles) * 64;
    const int c0 = blockIdx.y * 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int l16 = lane & 15, kl = lane >> 4;
    constexpr int NXU = (64 * CH + AT - 1) / AT;         // staging loads per thread: x~
    constexpr int NVU = (RK * CH + AT - 1) / AT;         // Vp
    constexpr int NUU = (RK * (64 / KPC) + AT - 1) / AT; // U
    f32x4 acc[4];
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) acc[ab] = f32x4{0, 0, 0, 0};
    auto face_rank = [&](int f) {
        const int r = ranks[f];
        return r < kcap ? r : kcap;
    };
    auto next_face = [&](int f) {  // first face from f on with a nonzero rank
        while (f < nf && face_rank(f) <= 0) ++f;
        return f;
    };
    // one stage = one face and chunk of k; its global loads go to registers
    // one stage ahead, so that they are in flight during the previous stage's
    // products
    u32x4 gx[NXU], gv[NVU], gu[NUU];
    double gs[NUU];
    auto load_stage = [&](int f, int kc0) {
        const int kf = face_rank(f);
        const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float *>(xt) + (int64_t)f * q * nrhs * E, 0, q * nrhs * E * 4, 0x00020000);
        const __amdgpu_buffer_rsrc_t rv = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float *>(Vp) + (int64_t)f * p * kmax * E, 0, p * kmax * E * 4, 0x00020000);
        const __amdgpu_buffer_rsrc_t ru = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float *>(U) + (int64_t)f * m * kmax * E, 0, m * kmax * E * 4, 0x00020000);
#pragma unroll
        for (int u = 0; u < NXU; ++u) {
            const int g = u * AT + tid, cc = g / CH, h = g % CH;
            const int k = kc0 + KPC * h, c = c0 + cc;
            const uint32_t xo = (((uint32_t)k + (uint32_t)q * (uint32_t)c) * (4u * E)) |
                                miss_if(g >= 64 * CH || c >= nrhs || k >= q);
            gx[u] = __builtin_amdgcn_raw_buffer_load_b128(rx, (int)xo, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < NVU; ++u) {
            const int g = u * AT + tid, r = g / CH, h = g % CH;
            const int k = kc0 + KPC * h;
            const uint32_t vo = (((uint32_t)k + (uint32_t)q * (uint32_t)j + (uint32_t)p * (uint32_t)r) * (4u * E)) |
                                miss_if(g >= RK * CH || r >= kf || k >= q);
            gv[u] = __builtin_amdgcn_raw_buffer_load_b128(rv, (int)vo, 0, 0);
        }
        if (kc0 == 0) {
#pragma unroll
            for (int u = 0; u < NUU; ++u) {
                const int g = u * AT + tid, r = g / (64 / KPC), h = g % (64 / KPC);
                const int a = a0 + KPC * h;
                const bool rin = g < RK * (64 / KPC) && r < kf;
                const uint32_t uo = (((uint32_t)a + (uint32_t)m * (uint32_t)r) * (4u * E)) | miss_if(!rin || a >= m);
                gu[u] = __builtin_amdgcn_raw_buffer_load_b128(ru, (int)uo, 0, 0);
                gs[u] = rin ? S[(int64_t)f * kmax + r] : 0.0;
            }
        }
    };
    // the registers of a stage into LDS; entries that do not exist as zero
    auto put = [&](float *dst, const u32x4 &v, int k) {
        const uint32_t e0 = v.x, e1 = v.y, e2 = v.z, e3 = v.w;
        float4 o;
        // a piece across q reads the next column or row: its entries past q are zeroed
        o.x = __uint_as_float(e0);
        o.y = (CPLX ? k : k + 1) < q ? __uint_as_float(e1) : 0.0f;
        o.z = (CPLX ? k + 1 : k + 2) < q ? __uint_as_float(e2) : 0.0f;
        o.w = (CPLX ? k + 1 : k + 3) < q ? __uint_as_float(e3) : 0.0f;
        if (BF) {
            o.x = rbf(o.x);
            o.y = rbf(o.y);
            o.z = rbf(o.z);
            o.w = rbf(o.w);
        }
        *reinterpret_cast<float4 *>(dst) = o;
    };
    auto store_stage = [&](int f, int kc0) {
        const float wgt = (CPLX && !(f == 0 || 2 * f == n3)) ? 2.0f : 1.0f;
#pragma unroll
        for (int u = 0; u < NXU; ++u) {
            const int g = u * AT + tid, cc = g / CH, h = g % CH;
            if (g < 64 * CH) put(&xs[cc * XS + KPC * h * E], gx[u], kc0 + KPC * h);
        }
#pragma unroll
        for (int u = 0; u < NVU; ++u) {
            const int g = u * AT + tid, r = g / CH, h = g % CH;
            if (g < RK * CH) put(&vs[r * XS + KPC * h * E], gv[u], kc0 + KPC * h);
        }
        if (kc0 == 0) {
            // U S w, transposed to rows a
#pragma unroll
            for (int u = 0; u < NUU; ++u) {
                const int g = u * AT + tid, r = g / (64 / KPC), h = g % (64 / KPC);
                if (g >= RK * (64 / KPC)) continue;
                const int a = a0 + KPC * h;
                const uint32_t e[4] = {gu[u].x, gu[u].y, gu[u].z, gu[u].w};
#pragma unroll
                for (int i = 0; i < KPC; ++i) {
                    const bool ain = a + i < m;  // the next rank's rows past m
#pragma unroll
                    for (int ee = 0; ee < E; ++ee) {
                        float x = ain ? (float)((double)__uint_as_float(e[i * E + ee]) * gs[u]) : 0.0f;
                        if (BF) x = rbf(x);
                        us[(KPC * h + i) * US + r * E + ee] = x * wgt;
                    }
                }
            }
        }
    };
    f32x4 zr[NRB], zi[NRB], z3[NRB];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) zr[rb] = zi[rb] = z3[rb] = f32x4{0, 0, 0, 0};
    int f = next_face(0), kc0 = 0;
    if (f < nf) load_stage(f, 0);
    while (f < nf) {
        __syncthreads();  // the previous stage's operands are consumed
        store_stage(f, kc0);
        __syncthreads();
        int fn = f, kn = kc0 + KC;
        if (kn >= q) {
            fn = next_face(f + 1);
            kn = 0;
        }
        if (fn < nf) load_stage(fn, kn);
        // Z += conj(V^T x~) over this chunk's k, in steps of 16
        const int nkk = (q - kc0 < KC ? q - kc0 + 15 : KC) >> 4;
        for (int kk = 0; kk < nkk; ++kk) {
            const float *xp = &xs[(16 * w + l16) * XS + (16 * kk + 4 * kl) * E];
            float xr[4], xi[4];
            if (CPLX) {
                const float4 xa = *reinterpret_cast<const float4 *>(xp);
                const float4 xb = *reinterpret_cast<const float4 *>(xp + 4);
                xr[0] = xa.x; xi[0] = xa.y; xr[1] = xa.z; xi[1] = xa.w;
                xr[2] = xb.x; xi[2] = xb.y; xr[3] = xb.z; xi[3] = xb.w;
            } else {
                const float4 xa = *reinterpret_cast<const float4 *>(xp);
                xr[0] = xa.x; xr[1] = xa.y; xr[2] = xa.z; xr[3] = xa.w;
                xi[0] = xi[1] = xi[2] = xi[3] = 0.0f;
            }
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb) {
                const float *vp = &vs[(16 * rb + l16) * XS + (16 * kk + 4 * kl) * E];
                float vr[4], vi[4];
                if (CPLX) {
                    const float4 va = *reinterpret_cast<const float4 *>(vp);
                    const float4 vb = *reinterpret_cast<const float4 *>(vp + 4);
                    vr[0] = va.x; vi[0] = va.y; vr[1] = va.z; vi[1] = va.w;
                    vr[2] = vb.x; vi[2] = vb.y; vr[3] = vb.z; vi[3] = vb.w;
                } else {
                    const float4 va = *reinterpret_cast<const float4 *>(vp);
                    vr[0] = va.x; vr[1] = va.y; vr[2] = va.z; vr[3] = va.w;
                    vi[0] = vi[1] = vi[2] = vi[3] = 0.0f;
                }
                if constexpr (BF) {
                    zr[rb] = mfma_bf4(pk4(vr[0], vr[1], vr[2], vr[3]), pk4(xr[0], xr[1], xr[2], xr[3]), zr[rb]);
                    if (CPLX) {
                        zi[rb] = mfma_bf4(pk4(vi[0], vi[1], vi[2], vi[3]), pk4(xi[0], xi[1], xi[2], xi[3]), zi[rb]);
                        z3[rb] = mfma_bf4(pk4(vr[0] + vi[0], vr[1] + vi[1], vr[2] + vi[2], vr[3] + vi[3]),
                                          pk4(xr[0] + xi[0], xr[1] + xi[1], xr[2] + xi[2], xr[3] + xi[3]), z3[rb]);
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        zr[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(vr[t], xr[t], zr[rb], 0, 0, 0);
                        if (CPLX) {
                            zi[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(vi[t], xi[t], zi[rb], 0, 0, 0);
                            z3[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(vr[t] + vi[t], xr[t] + xi[t], z3[rb], 0, 0, 0);
                        }
                    }
                }
            }
        }
        if (kc0 + KC >= q) {
            // the face is complete: y += Re(U S w Z)
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb) {
                if (CPLX) {
                    const f32x4 p1 = zr[rb], p2 = zi[rb];
                    zr[rb] = p1 - p2;           // Vr Xr - Vi Xi
                    zi[rb] = z3[rb] - p1 - p2;  // Vr Xi + Vi Xr = -Im Z
                }
#pragma unroll
                for (int ab = 0; ab < 4; ++ab) {
                    const float *up = &us[(16 * ab + l16) * US + (16 * rb + 4 * kl) * E];
                    float ur[4], ui[4];
                    if (CPLX) {
                        const float4 ua = *reinterpret_cast<const float4 *>(up);
                        const float4 ub = *reinterpret_cast<const float4 *>(up + 4);
                        ur[0] = ua.x; ui[0] = ua.y; ur[1] = ua.z; ui[1] = ua.w;
                        ur[2] = ub.x; ui[2] = ub.y; ur[3] = ub.z; ui[3] = ub.w;
                    } else {
                        const float4 ua = *reinterpret_cast<const float4 *>(up);
                        ur[0] = ua.x; ur[1] = ua.y; ur[2] = ua.z; ur[3] = ua.w;
                        ui[0] = ui[1] = ui[2] = ui[3] = 0.0f;
                    }
                    if constexpr (BF) {
                        const float z0 = zr[rb][0], z1 = zr[rb][1], z2 = zr[rb][2], z3v = zr[rb][3];
                        acc[ab] = mfma_bf4(pk4(ur[0], ur[1], ur[2], ur[3]), pk4(z0, z1, z2, z3v), acc[ab]);
                        if (CPLX) {
                            const float w0 = zi[rb][0], w1 = zi[rb][1], w2 = zi[rb][2], w3 = zi[rb][3];
                            acc[ab] = mfma_bf4(pk4(ui[0], ui[1], ui[2], ui[3]), pk4(w0, w1, w2, w3), acc[ab]);
                        }
                    } else {
#pragma unroll
                        for (int sx = 0; sx < 4; ++sx) {
                            const float bzr = zr[rb][sx];
                            const float bzi = zi[rb][sx];
                            acc[ab] = __builtin_amdgcn_mfma_f32_16x16x4f32(ur[sx], bzr, acc[ab], 0, 0, 0);
                            if (CPLX) acc[ab] = __builtin_amdgcn_mfma_f32_16x16x4f32(ui[sx], bzi, acc[ab], 0, 0, 0);
                        }
                    }
                }
                zr[rb] = zi[rb] = z3[rb] = f32x4{0, 0, 0, 0};
            }
        }
        f = fn;
        kc0 = kn;
    }
    const int c = c0 + 16 * w + l16;
    if (c < nrhs) {
#pragma unroll
        for (int ab = 0; ab < 4; ++ab)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = a0 + 16 * ab + 4 * kl + v;
                if (a < m) y[((int64_t)j * m + a) + ldy * c] = acc[ab][v];
            }
    }
}

// FP64 compute on FP64 matrix cores: the contraction of k_apply_lds with FP64
// operands and the FP64 16x16x4 MFMA (A[i][k]: lane%16 = i, lane/16 = k;
// B[k][j]: lane/16 = k, lane%16 = j; result row lane/16 + 4v, column lane%16).
// Workgroup: block row j, rows a0 .. a0+63, 64 columns; wavefront w owns
// columns c0 + 16 w .. + 15.  Per face and chunk of 16 k the workgroup stages
// x~ (64 columns), the NRB*16 rank rows of Vp and, on the first chunk, U S w
// (64 rows) in LDS with 16-byte loads (one complex, or two real, values);
// instruction kk of a chunk takes k = 4 kk + lane/16.  Z stays in the
// accumulators: entry v of lane (l16, kl) is Z(16 rb + kl + 4 v, l16), which
// is the B operand of step v of the second product, whose A operand is
// (U S w)(a, 16 rb + kl + 4 v).  Complex products by three real ones, as in
// the FP32 kernel.  Elements that do not exist load as zero (2^31 offset of a
// buffer resource per face, each under 2 GiB, checked on the host).
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <bool CPLX, int NRB>
__global__ __launch_bounds__(AT) void k_apply_f64(const double *__restrict__ U, const double *__restrict__ S,
                                                  const double *__restrict__ Vp, const int32_t *__restrict__ ranks,
                                                  int m, int p, int kmax, int nf, int n3, int ell, int q,
                                                  const double *__restrict__ xt, int nrhs, double *__restrict__ y,
                                                  int64_t ldy) {
    constexpr int E = CPLX ? 2 : 1;
    constexpr int KC = 16;              // k per chunk
    constexpr int XS = KC * E + 2;      // doubles per staged column of x~ or row of Vp
    constexpr int RK = 16 * NRB;        // ranks held
    constexpr int US = RK * E + 2;      // doubles per staged row of U S
    constexpr int KPC = 2 / E;          // k (or rows a) per 16-byte piece
    constexpr int CH = KC / KPC;        // pieces per column
    __shared__ __align__(16) double xs[64 * XS];
    __shared__ __align__(16) double vs[RK * XS];
    __shared__ __align__(16) double us[64 * US];
    const int kcap = kmax < RK ? kmax : RK;
    const int mtiles = (m + 63) >> 6;
    const int j = blockIdx.x / mtiles, a0 = (blockIdx.x % mtiles) * 64;
    const int c0 = blockIdx.y * 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int l16 = lane & 15, kl = lane >> 4;
    constexpr int NXU = (64 * CH + AT - 1) / AT;
    constexpr int NVU = (RK * CH + AT - 1) / AT;
    constexpr int NUU = (RK * (64 / KPC) + AT - 1) / AT;
    f64x4 acc[4];
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) acc[ab] = f64x4{0, 0, 0, 0};
    auto face_rank = [&](int f) {
        const int r = ranks[f];
        return r < kcap ? r : kcap;
    };
    auto next_face = [&](int f) {
        while (f < nf && face_rank(f) <= 0) ++f;
        return f;
    };
    u32x4 gx[NXU], gv[NVU], gu[NUU];
    double gs[NUU];
    auto load_stage = [&](int f, int kc0) {
        const int kf = face_rank(f);
        const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<double *>(xt) + (int64_t)f * q * nrhs * E, 0, q * nrhs * E * 8, 0x00020000);
        const __amdgpu_buffer_rsrc_t rv = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<double *>(Vp) + (int64_t)f * p * kmax * E, 0, p * kmax * E * 8, 0x00020000);
        const __amdgpu_buffer_rsrc_t ru = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<double *>(U) + (int64_t)f * m * kmax * E, 0, m * kmax * E * 8, 0x00020000);
#pragma unroll
        for (int u = 0; u < NXU; ++u) {
            const int g = u * AT + tid, cc = g / CH, hh = g % CH;
            const int k = kc0 + KPC * hh, c = c0 + cc;
            const uint32_t xo = (((uint32_t)k + (uint32_t)q * (uint32_t)c) * (8u * E)) |
                                miss_if(g >= 64 * CH || c >= nrhs || k >= q);
            gx[u] = __builtin_amdgcn_raw_buffer_load_b128(rx, (int)xo, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < NVU; ++u) {
            const int g = u * AT + tid, r = g / CH, hh = g % CH;
            const int k = kc0 + KPC * hh;
            const uint32_t vo = (((uint32_t)k + (uint32_t)q * (uint32_t)j + (uint32_t)p * (uint32_t)r) * (8u * E)) |
                                miss_if(g >= RK * CH || r >= kf || k >= q);
            gv[u] = __builtin_amdgcn_raw_buffer_load_b128(rv, (int)vo, 0, 0);
        }
        if (kc0 == 0) {
#pragma unroll
            for (int u = 0; u < NUU; ++u) {
                const int g = u * AT + tid, r = g / (64 / KPC), hh = g % (64 / KPC);
                const int a = a0 + KPC * hh;
                const bool rin = g < RK * (64 / KPC) && r < kf;
                const uint32_t uo = (((uint32_t)a + (uint32_t)m * (uint32_t)r) * (8u * E)) | miss_if(!rin || a >= m);
                gu[u] = __builtin_amdgcn_raw_buffer_load_b128(ru, (int)uo, 0, 0);
                gs[u] = rin ? S[(int64_t)f * kmax + r] : 0.0;
            }
        }
    };
    // a 16-byte piece as two doubles; a real piece across q reads the next
    // column or row: its second entry past q is zeroed
    auto put = [&](double *dst, const u32x4 &v, int k) {
        const uint32_t e0 = v.x, e1 = v.y, e2 = v.z, e3 = v.w;
        const double d0 = __hiloint2double((int)e1, (int)e0);
        double d1 = __hiloint2double((int)e3, (int)e2);
        if (!CPLX && k + 1 >= q) d1 = 0.0;
        *reinterpret_cast<double2 *>(dst) = double2{d0, d1};
    };
    auto store_stage = [&](int f, int kc0) {
        const double wgt = (CPLX && !(f == 0 || 2 * f == n3)) ? 2.0 : 1.0;
#pragma unroll
        for (int u = 0; u < NXU; ++u) {
            const int g = u * AT + tid, cc = g / CH, hh = g % CH;
            if (g < 64 * CH) put(&xs[cc * XS + KPC * hh * E], gx[u], kc0 + KPC * hh);
        }
#pragma unroll
        for (int u = 0; u < NVU; ++u) {
            const int g = u * AT + tid, r = g / CH, hh = g % CH;
            if (g < RK * CH) put(&vs[r * XS + KPC * hh * E], gv[u], kc0 + KPC * hh);
        }
        if (kc0 == 0) {
#pragma unroll
            for (int u = 0; u < NUU; ++u) {
                const int g = u * AT + tid, r = g / (64 / KPC), hh = g % (64 / KPC);
                if (g >= RK * (64 / KPC)) continue;
                const int a = a0 + KPC * hh;
                const uint32_t e0 = gu[u].x, e1 = gu[u].y, e2 = gu[u].z, e3 = gu[u].w;
                const double d[2] = {__hiloint2double((int)e1, (int)e0), __hiloint2double((int)e3, (int)e2)};
#pragma unroll
                for (int i = 0; i < KPC; ++i) {
                    const bool ain = a + i < m;
#pragma unroll
                    for (int ee = 0; ee < E; ++ee)
                        us[(KPC * hh + i) * US + r * E + ee] = ain ? d[i * E + ee] * gs[u] * wgt : 0.0;
                }
            }
        }
    };
    f64x4 zr[NRB], zi[NRB], z3[NRB];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) zr[rb] = zi[rb] = z3[rb] = f64x4{0, 0, 0, 0};
    int f = next_face(0), kc0 = 0;
    if (f < nf) load_stage(f, 0);
    while (f < nf) {
        __syncthreads();  // the previous stage's operands are consumed
        store_stage(f, kc0);
        __syncthreads();
        int fn = f, kn = kc0 + KC;
        if (kn >= q) {
            fn = next_face(f + 1);
            kn = 0;
        }
        if (fn < nf) load_stage(fn, kn);
        const int nkk = (q - kc0 < KC ? q - kc0 + 3 : KC) >> 2;
        for (int kk = 0; kk < nkk; ++kk) {
            const double *xp = &xs[(16 * w + l16) * XS + (4 * kk + kl) * E];
            const double xr = xp[0], xi = CPLX ? xp[1] : 0.0;
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb) {
                const double *vp = &vs[(16 * rb + l16) * XS + (4 * kk + kl) * E];
                const double vr = vp[0], vi = CPLX ? vp[1] : 0.0;
                zr[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(vr, xr, zr[rb], 0, 0, 0);
                if (CPLX) {
                    zi[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(vi, xi, zi[rb], 0, 0, 0);
                    z3[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(vr + vi, xr + xi, z3[rb], 0, 0, 0);
                }
            }
        }
        if (kc0 + KC >= q) {
            // the face is complete: y += Re(U S w Z)
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb) {
                if (CPLX) {
                    const f64x4 p1 = zr[rb], p2 = zi[rb];
                    zr[rb] = p1 - p2;           // Vr Xr - Vi Xi
                    zi[rb] = z3[rb] - p1 - p2;  // Vr Xi + Vi Xr = -Im Z
                }
#pragma unroll
                for (int ab = 0; ab < 4; ++ab) {
#pragma unroll
                    for (int sx = 0; sx < 4; ++sx) {
                        const double *up = &us[(16 * ab + l16) * US + (16 * rb + kl + 4 * sx) * E];
                        const double bzr = zr[rb][sx];
                        acc[ab] = __builtin_amdgcn_mfma_f64_16x16x4f64(up[0], bzr, acc[ab], 0, 0, 0);
                        if (CPLX) {
                            const double bzi = zi[rb][sx];
                            acc[ab] = __builtin_amdgcn_mfma_f64_16x16x4f64(up[1], bzi, acc[ab], 0, 0, 0);
                        }
                    }
                }
                zr[rb] = zi[rb] = z3[rb] = f64x4{0, 0, 0, 0};
            }
        }
        f = fn;
        kc0 = kn;
    }
    const int c = c0 + 16 * w + l16;
    if (c < nrhs) {
#pragma unroll
        for (int ab = 0; ab < 4; ++ab)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = a0 + 16 * ab + kl + 4 * v;
                if (a < m) y[((int64_t)j * m + a) + ldy * c] = acc[ab][v];
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
    // the transformed right-hand sides and the relaid-out V
    return al256(es * (size_t)q * nrhs * F->nf) + al256(es * (size_t)F->p * F->kmax * F->nf);
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
    // FP32 and BF16: the matrix-core kernel, when every per-face buffer and
    // every offset it forms (64 past the last column, row and rank included)
    // stays below 2 GiB
    const int64_t E = cplx ? 2 : 1, lim = int64_t(1) << 31;
    const bool mfma_fits = !dbl && (int64_t)q * (nrhs + 64) * 4 * E + 64 < lim &&
                           ((int64_t)q * (ell + 1) + 16 + F->p * (int64_t)64) * 4 * E + 64 < lim &&
                           (F->m + 64 + F->m * (int64_t)64) * 4 * E < lim && F->p * F->kmax * 4 * E < lim &&
                           mtiles * ell < lim;
    // FP64: the FP64 matrix-core kernel under the same 2 GiB conditions on
    // 8-byte elements
    const bool mfma64_fits = dbl && (int64_t)q * (nrhs + 64) * 8 * E + 64 < lim &&
                             ((int64_t)q * (ell + 1) + 16 + F->p * (int64_t)64) * 8 * E + 64 < lim &&
                             (F->m + 64 + F->m * (int64_t)64) * 8 * E < lim && F->p * F->kmax * 8 * E < lim &&
                             mtiles * ell < lim;
    if (mfma64_fits) {
        const int nrb = (kcap + 15) / 16;
        double *Vp = reinterpret_cast<double *>(reinterpret_cast<char *>(ws) + al256(es * (size_t)q * nrhs * nf));
        const int64_t tot = F->p * F->kmax * nf;
        if (tot > 0) {
            // the relayout moves whole elements: 4 (complex) or 2 (real) floats each
            const dim3 gr((unsigned)((tot + 255) / 256));
            if (cplx)
                TSVDM_LAUNCH("apply_v_relayout", k_vrelayout<4>, gr, dim3(256), 0, s,
                             reinterpret_cast<const float *>(F->V), reinterpret_cast<float *>(Vp), F->p, ell, q, tot);
            else
                TSVDM_LAUNCH("apply_v_relayout", k_vrelayout<2>, gr, dim3(256), 0, s,
                             reinterpret_cast<const float *>(F->V), reinterpret_cast<float *>(Vp), F->p, ell, q, tot);
        }
#define TSVDM_APPLY64(C, NRB)                                                                                 \
    TSVDM_LAUNCH("apply_fused", (k_apply_f64<C, NRB>), grid, dim3(AT), 0, s,                                   \
                 reinterpret_cast<const double *>(F->U), F->S, (const double *)Vp, F->ranks, (int)F->m, (int)F->p, \
                 (int)F->kmax, (int)nf, (int)n3, (int)ell, (int)q, reinterpret_cast<const double *>(ws), (int)nrhs, \
                 reinterpret_cast<double *>(y), ldy)
#define TSVDM_APPLY64_NRB(C)                          \
    do {                                              \
        switch (nrb) {                                \
            case 1: TSVDM_APPLY64(C, 1); break;       \
            case 2: TSVDM_APPLY64(C, 2); break;       \
            case 3: TSVDM_APPLY64(C, 3); break;       \
            default: TSVDM_APPLY64(C, 4); break;      \
        }                                             \
    } while (0)
        if (cplx) TSVDM_APPLY64_NRB(true);
        else TSVDM_APPLY64_NRB(false);
#undef TSVDM_APPLY64_NRB
#undef TSVDM_APPLY64
        TSVDM_LAUNCH_CHECK("k_apply_f64");
        return TSVDM_OK;
    }
    if (mfma_fits) {
        const int nrb = (kcap + 15) / 16;
        float *Vp = reinterpret_cast<float *>(reinterpret_cast<char *>(ws) + al256(es * (size_t)q * nrhs * nf));
        const int64_t tot = F->p * F->kmax * nf;
        if (tot > 0) {
            const dim3 gr((unsigned)((tot + 255) / 256));
            if (cplx)
                TSVDM_LAUNCH("apply_v_relayout", k_vrelayout<2>, gr, dim3(256), 0, s,
                             reinterpret_cast<const float *>(F->V), Vp, F->p, ell, q, tot);
            else
                TSVDM_LAUNCH("apply_v_relayout", k_vrelayout<1>, gr, dim3(256), 0, s,
                             reinterpret_cast<const float *>(F->V), Vp, F->p, ell, q, tot);
        }
#define TSVDM_APPLY_MFMA(C, B, NRB)                                                                        \
    TSVDM_LAUNCH("apply_fused", (k_apply_mfma<C, B, NRB>), grid, dim3(AT), 0, s,                             \
                 reinterpret_cast<const float *>(F->U), F->S, Vp, F->ranks,                                  \
                 (int)F->m, (int)F->p, (int)F->kmax, (int)nf, (int)n3, (int)ell, (int)q,                    \
                 reinterpret_cast<const float *>(ws), (int)nrhs, reinterpret_cast<float *>(y), ldy)
#define TSVDM_APPLY_NRB(C, B)                         \
    do {                                              \
        switch (nrb) {                                \
            case 1: TSVDM_APPLY_MFMA(C, B, 1); break; \
            case 2: TSVDM_APPLY_MFMA(C, B, 2); break; \
            case 3: TSVDM_APPLY_MFMA(C, B, 3); break; \
            default: TSVDM_APPLY_MFMA(C, B, 4); break; \
        }                                             \
    } while (0)
        const bool bf = compute == TSVDM_BF16;
        if (nrb <= 2) {
#define TSVDM_APPLY_LDS1(C, B, NRB)                                                                          \
    TSVDM_LAUNCH("apply_fused", (k_apply_lds<C, B, NRB>), grid, dim3(AT), 0, s,                              \
                 reinterpret_cast<const float *>(F->U), F->S, Vp, F->ranks, (int)F->m, (int)F->p, (int)F->kmax, \
                 (int)nf, (int)n3, (int)ell, (int)q, reinterpret_cast<const float *>(ws), (int)nrhs,          \
                 reinterpret_cast<float *>(y), ldy)
#define TSVDM_APPLY_LDS(C, B)                     \
    do {                                          \
        if (nrb == 1) TSVDM_APPLY_LDS1(C, B, 1);  \
        else TSVDM_APPLY_LDS1(C, B, 2);           \
    } while (0)
            if (cplx) {
                if (bf) TSVDM_APPLY_LDS(true, true);
                else TSVDM_APPLY_LDS(true, false);
            } else {
                if (bf) TSVDM_APPLY_LDS(false, true);
                else TSVDM_APPLY_LDS(false, false);
            }
#undef TSVDM_APPLY_LDS
#undef TSVDM_APPLY_LDS1
        } else if (cplx) {
            if (bf) TSVDM_APPLY_NRB(true, true);
            else TSVDM_APPLY_NRB(true, false);
        } else {
            if (bf) TSVDM_APPLY_NRB(false, true);
            else TSVDM_APPLY_NRB(false, false);
        }
#undef TSVDM_APPLY_NRB
#undef TSVDM_APPLY_MFMA
        TSVDM_LAUNCH_CHECK("k_apply_mfma");
        return TSVDM_OK;
    }
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
