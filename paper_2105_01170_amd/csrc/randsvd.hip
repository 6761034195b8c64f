// Mixed-precision randomized facewise truncated SVD (PREC_MIXED).
//
// For every face X_f (m x p, FP32) of the transform-domain tensor, with the
// caller's Gaussian test matrix Omega (p x ell, ell = k + oversample):
//
//   Y  = X Omega          BF16 MFMA, FP32 accumulation          (pass 1, + ||X||^2)
//   Q  = orth(Y)          one shifted Cholesky-QR step          (Gram: FP32 partials)
//   Z  = X^T Q            BF16 MFMA                              (pass 2)
//   Qz = orth(Z)          one shifted Cholesky-QR step          (Gram: FP32 partials)
//   Y' = X Qz             split-BF16 MFMA (hi*hi + hi*lo + lo*hi), FP32-accurate (pass 3)
//   Q  = qr(Y')           FP64 shifted Cholesky-QR2 (FP64 Gram by MFMA)
//   B^T = X^T Q           split-BF16 MFMA                        (pass 4)
//   r2 = ||X - Q B||^2    FP32 MFMA product, FP64 sums           (pass 5)
//   B B^T = U_B L U_B^T   FP64 Gram (MFMA) + cyclic Jacobi eigensolver, s = sqrt(L)
//   Uhat = Q U_B, Vhat = B^T U_B / s, truncated to k_f;  cert^2 = r2 + sum_{j>k_f} L_j
//
// This is the randomized range finder with power iteration of Halko,
// Martinsson & Tropp (2011), applied face by face.  Only the first sketch
// and the first power half-step run in plain BF16, and their bases only
// need the right span: one Cholesky-QR step with a shift at the rounding
// level of the FP32 Gram matrix (Fukaya et al. 2020) bounds cond(Q) and keeps
// the span exact.  The last half-step is FP32-accurate, so BF16 rounding of
// the data does not limit the result; its basis is made orthonormal in FP64.
//
// The passes over X are HBM-bound skinny GEMMs (N = ell <= 64).  Every
// workgroup streams a 64-row (or 64-column) slab of one face, converts it to
// BF16 in registers, stages it in LDS, and the four wavefronts drive 16x16
// MFMA tiles; the next slab's loads are issued before the current slab's
// MFMAs.  The small FP64 steps use one workgroup per face.
#include "common.h"
#include "jacobi_dev.h"

#include <math.h>

#include <algorithm>
#include <mutex>

using namespace tsvdm;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int GT = 256;  // threads per workgroup
enum { PROD_BF16 = 0, PROD_SPLIT = 1 };
// most column ranges per 64-row block (the certificate pass, the X W passes);
// the certificate partials hold that many per block
constexpr int kResidSplitMax = 32;

// (x0, x1) -> packed BF16 pairs hi = RNE(x), lo = RNE(x - hi) (x - hi is
// exact in FP32), element 0 in the low half; the hardware packed conversion
__device__ __forceinline__ void split2(float x0, float x1, uint32_t &hi, uint32_t &lo) {
    const f32x2 v = {x0, x1};
    const bf16x2 h = __builtin_convertvector(v, bf16x2);
    const bf16x2 l = __builtin_convertvector(v - __builtin_convertvector(h, f32x2), bf16x2);
    hi = __builtin_bit_cast(uint32_t, h);
    lo = __builtin_bit_cast(uint32_t, l);
}

__device__ __forceinline__ f32x4 mfma(const u16x8 &a, const u16x8 &b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// ---------------------------------------------------------------- Gram partials
// Gram partials: the upper 16x16 tiles of the LP x LP block Gram (tile t in
// row-major order over the upper triangle), each row major, packed one after
// another; one partial per LP*LP doubles of the workspace.
template <int LP>
constexpr int gram_tiles() {
    return (LP / 16) * (LP / 16 + 1) / 2;
}

// G (LDS, pitch ldg) = ordered sum over pp of the nparts packed partials of
// face f, both triangles.  All loads of a block of 8 partials are issued
// before any is summed (clamped addresses, zero-selected, no branches).
// lps: the width the partials were written for (LP, or 32 when LP = 16: the
// 16 x 16 Gram is the first packed tile of a width-32 partial).  pstride,
// fparts: the nparts summed are every pstride-th of the face's fparts
// partials (group sums of k_gram_group), fparts < 0 meaning nparts.
template <int LP, int NTH>
__device__ __forceinline__ void load_gram_partials(const double *__restrict__ gpart, int f, int nparts,
                                                   double *G, int ldg, int lps = LP, int pstride = 1,
                                                   int fparts = -1) {
    constexpr int NT = LP / 16, NE2 = gram_tiles<LP>() * 128;
    constexpr int E2 = (NE2 + NTH - 1) / NTH, PB = 8;
    const int S2 = lps * lps / 2;
    const int tid = threadIdx.x;
    const double2 *g2 =
        reinterpret_cast<const double2 *>(gpart + (int64_t)f * (fparts < 0 ? nparts : fparts) * lps * lps);
    double2 acc[E2];
#pragma unroll
    for (int q = 0; q < E2; ++q) acc[q] = double2{0.0, 0.0};
    for (int p0 = 0; p0 < nparts; p0 += PB) {
        double2 v[E2][PB];
#pragma unroll
        for (int q = 0; q < E2; ++q)
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                const int e2 = tid + q * NTH, pp = p0 + u;
                const bool in = e2 < NE2 && pp < nparts;
                const double2 t = g2[(int64_t)(pp < nparts ? pp : nparts - 1) * pstride * S2 + (e2 < NE2 ? e2 : 0)];
                v[q][u] = in ? t : double2{0.0, 0.0};
            }
#pragma unroll
        for (int q = 0; q < E2; ++q)
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                acc[q].x += v[q][u].x;
                acc[q].y += v[q][u].y;
            }
    }
#pragma unroll
    for (int q = 0; q < E2; ++q) {
        const int e2 = tid + q * NTH;
        if (e2 < NE2) {
            const int t = (2 * e2) >> 8, r = ((2 * e2) >> 4) & 15, c = (2 * e2) & 15;
            int ti = 0, tt = t;
            while (tt >= NT - ti) {
                tt -= NT - ti;
                ++ti;
            }
            const int tj = ti + tt, i = 16 * ti + r, j = 16 * tj + c;
            G[i * ldg + j] = acc[q].x;
            G[i * ldg + j + 1] = acc[q].y;
            if (ti != tj) {
                G[j * ldg + i] = acc[q].x;
                G[(j + 1) * ldg + i] = acc[q].y;
            }
        }
    }
}

// ---------------------------------------------------------------- XCD map
// Workgroups are dispatched round-robin over the 8 XCDs (workgroup L runs on
// XCD L % 8, each with its own L2).  For a pass whose nb blocks of a face all
// read the same per-face operand, give those blocks consecutive slots on one
// XCD, so the operand is fetched into that L2 once instead of eight times.
// With fewer than 8 faces a face's blocks are cut into g = ceil(8 / nf)
// consecutive runs, each on its own XCD (else a single face would run on one
// XCD of eight).  The grid is ceil(nb / g) times nf g rounded up to a
// multiple of 8 (xcd_grid); workgroups past the faces or past a face's last
// block get f = nf and exit at once.
__host__ __device__ __forceinline__ int xcd_runs(int nf) { return nf >= 8 || nf < 1 ? 1 : (nf + 7) / nf; }
__device__ __forceinline__ void xcd_map(int L, int nb, int nf, int &b, int &f) {
    const int g = xcd_runs(nf), nbv = (nb + g - 1) / g;
    const int x = L & 7, s = L >> 3;
    const int vf = (s / nbv) * 8 + x;  // run vf % g of face vf / g
    b = (vf % g) * nbv + s % nbv;
    f = vf / g;
    if (b >= nb) f = nf;
}
inline unsigned xcd_grid(int nb, int nf) {
    const int g = xcd_runs(nf), nbv = (nb + g - 1) / g;
    return (unsigned)nbv * (unsigned)((nf * g + 7) / 8 * 8);
}

// ---------------------------------------------------------------- staging
// Rows r0..r0+RC-1 of the rows x LP column-major panel S into
// st[r*(LP+1) + c] (zeros past the last row).  All loads of a thread are
// issued before any LDS store, so they are in flight together.
template <int LP, int RC>
__device__ __forceinline__ void stage_panel(const float *__restrict__ S, int rows, int r0, float *st) {
    constexpr int PER = RC * LP / GT;
    static_assert(RC * LP % GT == 0, "panel size");
    float v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * GT, r = e % RC, c = e / RC;
        v[q] = r0 + r < rows ? S[(r0 + r) + (int64_t)rows * c] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * GT, r = e % RC, c = e / RC;
        st[r * (LP + 1) + c] = v[q];
    }
}

// As stage_panel, with 16-byte loads of four consecutive rows: rows a multiple
// of 4 and S 16-byte aligned (checked by the caller).
template <int LP, int RC>
__device__ __forceinline__ void stage_panel4(const float *__restrict__ S, int rows, int r0, float *st) {
    constexpr int PER = RC * LP / (4 * GT);
    static_assert(RC * LP % (4 * GT) == 0, "panel size");
    f32x4 v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * GT, r = 4 * (e % (RC / 4)), c = e / (RC / 4);
        const bool ok = r0 + r < rows;  // then r0 + r + 3 < rows
        const f32x4 x = *reinterpret_cast<const f32x4 *>(S + (ok ? (r0 + r) + (int64_t)rows * c : 0));
        v[q] = ok ? x : f32x4{0, 0, 0, 0};
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + q * GT, r = 4 * (e % (RC / 4)), c = e / (RC / 4);
#pragma unroll
        for (int u = 0; u < 4; ++u) st[(r + u) * (LP + 1) + c] = v[q][u];
    }
}

// upper 16x16 tile t (row-major over the upper triangle) -> tile coordinates
template <int NT>
__device__ __forceinline__ void tile_ij(int t, int &ti, int &tj) {
    ti = 0;
    while (t >= NT - ti) {
        t -= NT - ti;
        ++ti;
    }
    tj = ti + t;
}

// Write the 16x16 accumulator tile (ti, tj) of a symmetric LP x LP matrix
// and its mirror image.  Output layout of the 16x16x4 MFMAs (column
// lane%16 in both): FP32 holds row 4*(lane/16) + v in slot v, FP64 holds row
// lane/16 + 4*v.  Diagonal tiles write only their upper half and mirror it,
// so every entry has exactly one writer.
template <bool F64, typename T, typename V4>
__device__ __forceinline__ void put_sym_tile(T *G, int ld, int ti, int tj, const V4 &acc, int lane) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int ir = F64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
        const int i = 16 * ti + ir, j = 16 * tj + (lane & 15);
        if (ti < tj || i <= j) {
            G[i * ld + j] = acc[v];
            G[j * ld + i] = acc[v];
        }
    }
}

// FP64 Gram of the 64 x LP block held in the four wavefronts' MFMA
// accumulators (row 16*wave + 4*(lane/16) + v, column 16*j + lane%16), by FP64
// MFMA on the upper tiles (products of FP32 values are exact in FP64), written
// to `out` as packed upper tiles (gram_tiles).  Every tile is split into two
// halves of 32 rows, so the 2 * gram_tiles items spread evenly over the four
// wavefronts; the second half's sum goes through `red` (LDS, 256 doubles per
// tile, written after every read of ys, so it may overlap ys) to the
// first's.  The FP64 16x16x4 output (row lane/16 + 4v, column lane%16) at
// index 64v + lane is the tile in row-major order, so the stores are
// contiguous.  `ys` holds 64*(LP+1) floats.  Ends with a barrier.
template <int LP>
__device__ void block_gram_f64(const f32x4 (&acc)[LP / 16], double *__restrict__ out, float *ys, double *red) {
    constexpr int NT = LP / 16, NTILE = gram_tiles<LP>(), IPW = (2 * NTILE + 3) / 4;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            ys[(16 * wave + 4 * (lane >> 4) + v) * (LP + 1) + 16 * j + (lane & 15)] = acc[j][v];
    __syncthreads();
    f64x4 g[IPW];
#pragma unroll
    for (int u = 0; u < IPW; ++u) {
        g[u] = f64x4{0, 0, 0, 0};
        const int it = wave + 4 * u;
        if (it >= 2 * NTILE) continue;
        int ti, tj;
        tile_ij<NT>(it >> 1, ti, tj);
        const int r0 = 32 * (it & 1);
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            const int r = r0 + 4 * kk + (lane >> 4);
            g[u] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)ys[r * (LP + 1) + 16 * ti + (lane & 15)],
                                                        (double)ys[r * (LP + 1) + 16 * tj + (lane & 15)], g[u],
                                                        0, 0, 0);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < IPW; ++u) {
        const int it = wave + 4 * u;
        if (it < 2 * NTILE && (it & 1)) {
#pragma unroll
            for (int v = 0; v < 4; ++v) red[(it >> 1) * 256 + 64 * v + lane] = g[u][v];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < IPW; ++u) {
        const int it = wave + 4 * u;
        if (it >= 2 * NTILE || (it & 1)) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v)
            out[(it >> 1) * 256 + 64 * v + lane] = g[u][v] + red[(it >> 1) * 256 + 64 * v + lane];
    }
    __syncthreads();
}

// ---------------------------------------------------------------- Y = X W
// Grid (ceil(m/64), nf).  Workgroup: rows a0..a0+63 of face f, all LP
// columns of the result; K = p in chunks of 32.  W (p x nw used columns,
// leading dim ldw) is per face (stride w_stride) or shared (w_stride = 0).
// The X slab and the W chunk are converted to BF16 (hi, and lo for the
// split product) and staged in LDS with K contiguous, so each lane's MFMA
// operand is one 16-byte LDS read; the next chunk is loaded into registers
// while the current one is multiplied.  A lane loads a 4 x 4 block of the
// chunk (four consecutive rows of four adjacent columns).  VEC: m is a
// multiple of 4, X is 16-byte aligned and a face spans less than 4 GiB
// (checked by the caller), so each column of the block is one 16-byte load
// at a 32-bit offset from the face.  Loads go to clamped addresses; bit masks
// mark the valid values and are applied when the chunk is converted, so no
// instruction waits on a load that is still in flight.
template <int LP, int PROD, bool GRAM, bool VEC>
__global__ __launch_bounds__(GT) void k_xw(const float *__restrict__ X, int m, int p, int nf,
                                           const float *__restrict__ W, int64_t w_stride, int ldw,
                                           int nw, float *__restrict__ Y,
                                           double *__restrict__ fro_part,
                                           double *__restrict__ gram_part,
    const int32_t *__restrict__ fmap, int ksplit = 1, float *__restrict__ ypart = nullptr,
    double *__restrict__ frop = nullptr) {
    constexpr int KC = 64, LDK = KC + 8;  // LDS row pitch (bf16 elements)
    constexpr int NB = LP / 16, WPT = KC * LP / GT;
    constexpr bool SPL = PROD == PROD_SPLIT;
    __shared__ __align__(16) uint16_t xh[64 * LDK];
    __shared__ __align__(16) uint16_t xl[SPL ? 64 * LDK : 8];
    __shared__ __align__(16) uint16_t wh[LP * LDK];
    __shared__ __align__(16) uint16_t wl[SPL ? LP * LDK : 8];
    // Gram staging; afterwards the Gram's half-tile sums (as doubles)
    constexpr int YS = 64 * (LP + 1) > 512 * gram_tiles<LP>() ? 64 * (LP + 1) : 512 * gram_tiles<LP>();
    __shared__ __align__(16) float ys[GRAM ? YS : 1];
    __shared__ double red[GT / 64];
    const int nb = (m + 63) / 64;
    int bx, f;
    xcd_map(blockIdx.x, nb * ksplit, nf, bx, f);
    if (f >= nf) return;  // a padding face of the grid
    if (fmap && fmap[f] < 0) return;  // an unused slot of a face list sized on the device
    const int blk = bx / ksplit, sp = bx - blk * ksplit;
    const int a0 = blk * 64;
    // the workgroup's columns c0 .. pe-1: range sp of ksplit over the chunks
    const int cps = ((p + KC - 1) / KC + ksplit - 1) / ksplit;
    const int c0 = min(p, sp * cps * KC), pe = min(p, (sp + 1) * cps * KC);
    const float *Xf = X + (int64_t)(fmap ? fmap[f] : f) * m * p;
    const float *Wf = W + (int64_t)f * w_stride;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int rq = tid & 15, cg = tid >> 4;  // X load mapping: rows 4rq.., columns 4cg..
    f32x4 acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = f32x4{0, 0, 0, 0};
    double fro = 0.0;
    const int arow = a0 + 4 * rq;
    const char *Xb = reinterpret_cast<const char *>(Xf), *Wb = reinterpret_cast<const char *>(Wf);
    float xr[16], wr[WPT];  // xr[4 * it + v] = X[arow + v][b0 + 4cg + it]
    uint32_t xm = 0, wm = 0;
    auto load = [&](int b0) {
        xm = 0;
        wm = 0;
        if constexpr (VEC) {  // arow < m implies arow + 3 < m
#pragma unroll
            for (int it = 0; it < 4; ++it) {
                const int b = b0 + 4 * cg + it;
                const bool ok = b < pe && arow < m;
                const uint32_t off = ok ? 4u * ((uint32_t)arow + (uint32_t)m * (uint32_t)b) : 0u;
                const f32x4 x = *reinterpret_cast<const f32x4 *>(Xb + off);
#pragma unroll
                for (int v = 0; v < 4; ++v) xr[4 * it + v] = x[v];
                xm |= ok ? 0xFu << (4 * it) : 0u;
            }
        } else {
            // one row per lane, 16 columns per wavefront: every load is 64
            // consecutive rows of one column
            const int a = a0 + lane;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int b = b0 + 16 * wave + i;
                const bool ok = b < pe && a < m;
                xr[i] = Xf[ok ? a + (int64_t)m * b : 0];
                xm |= (uint32_t)ok << i;
            }
        }
        if constexpr (VEC) {  // four consecutive rows of W (p, ldw multiples of 4)
#pragma unroll
            for (int q = 0; q < WPT / 4; ++q) {
                const int e = tid + q * GT, k4 = e % (KC / 4), c = e / (KC / 4), b = b0 + 4 * k4;
                const bool ok = c < nw && b < pe;
                const f32x4 x = *reinterpret_cast<const f32x4 *>(
                    Wb + (ok ? 4u * ((uint32_t)b + (uint32_t)ldw * (uint32_t)c) : 0u));
#pragma unroll
                for (int v = 0; v < 4; ++v) wr[4 * q + v] = x[v];
                wm |= ok ? 0xFu << (4 * q) : 0u;
            }
        } else {
#pragma unroll
            for (int q = 0; q < WPT; ++q) {
                const int e = tid + q * GT, k = e % KC, c = e / KC, b = b0 + k;
                const bool ok = c < nw && b < pe;
                wr[q] = *reinterpret_cast<const float *>(Wb + (ok ? 4u * ((uint32_t)b + (uint32_t)ldw * (uint32_t)c) : 0u));
                wm |= (uint32_t)ok << q;
            }
        }
    };
    load(c0);
    for (int b0 = c0; b0 < pe; b0 += KC) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            // VEC: row 4rq + v, columns 4cg .. 4cg+3; else row lane, columns
            // 16 wave + 4v .. 16 wave + 4v + 3
            float x[4];
#pragma unroll
            for (int it = 0; it < 4; ++it) {
                const int q = VEC ? 4 * it + v : 4 * v + it;
                x[it] = (xm >> q) & 1u ? xr[q] : 0.0f;
                fro += (double)x[it] * (double)x[it];
            }
            uint2 h, l;
            split2(x[0], x[1], h.x, l.x);
            split2(x[2], x[3], h.y, l.y);
            const int at = VEC ? (4 * rq + v) * LDK + 4 * cg : lane * LDK + 16 * wave + 4 * v;
            *reinterpret_cast<uint2 *>(&xh[at]) = h;
            if (SPL) *reinterpret_cast<uint2 *>(&xl[at]) = l;
        }
        if constexpr (VEC) {
#pragma unroll
            for (int q = 0; q < WPT / 4; ++q) {  // rows 4k4 .. 4k4+3 of column c
                const int e = tid + q * GT, k4 = e % (KC / 4), c = e / (KC / 4);
                float w4[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) w4[v] = (wm >> (4 * q + v)) & 1u ? wr[4 * q + v] : 0.0f;
                uint2 h, l;
                split2(w4[0], w4[1], h.x, l.x);
                split2(w4[2], w4[3], h.y, l.y);
                *reinterpret_cast<uint2 *>(&wh[c * LDK + 4 * k4]) = h;
                if (SPL) *reinterpret_cast<uint2 *>(&wl[c * LDK + 4 * k4]) = l;
            }
        } else {
#pragma unroll
            for (int q = 0; q < WPT; q += 2) {
                const int e0 = tid + q * GT, e1 = e0 + GT;
                uint32_t hh, ll;
                split2((wm >> q) & 1u ? wr[q] : 0.0f, (wm >> (q + 1)) & 1u ? wr[q + 1] : 0.0f, hh, ll);
                wh[(e0 / KC) * LDK + e0 % KC] = (uint16_t)hh;
                wh[(e1 / KC) * LDK + e1 % KC] = (uint16_t)(hh >> 16);
                if (SPL) {
                    wl[(e0 / KC) * LDK + e0 % KC] = (uint16_t)ll;
                    wl[(e1 / KC) * LDK + e1 % KC] = (uint16_t)(ll >> 16);
                }
            }
        }
        __syncthreads();
        if (b0 + KC < pe) load(b0 + KC);  // next chunk in flight during the MFMAs
        const int ar = 16 * wave + (lane & 15);
#pragma unroll
        for (int kk = 0; kk < KC / 32; ++kk) {
            const int kq = 32 * kk + 8 * (lane >> 4);
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
        }
        __syncthreads();
    }
    if (ksplit > 1) {
        // a partial product: into panel sp of the face's ypart (stride p LP
        // per face, ksplit m <= p), ||X||^2 of the columns into frop; k_ysum
        // sums them and forms the Gram partials
        float *Pf = ypart + (int64_t)f * p * LP + (int64_t)sp * m * LP;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int c = 16 * j + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = a0 + 16 * wave + 4 * (lane >> 4) + v;
                if (r < m) Pf[r + (int64_t)m * c] = acc[j][v];
            }
        }
        if (fro_part) {
            fro = wave_sum(fro);
            if (lane == 0) red[wave] = fro;
            __syncthreads();
            if (tid == 0)
                frop[(int64_t)f * nb * kResidSplitMax + blk * ksplit + sp] = red[0] + red[1] + red[2] + red[3];
        }
        return;
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
    if (GRAM) block_gram_f64<LP>(acc, gram_part + ((int64_t)f * nb + blk) * LP * LP, ys, reinterpret_cast<double *>(ys));
    if (fro_part) {
        fro = wave_sum(fro);
        if (lane == 0) red[wave] = fro;
        __syncthreads();
        if (tid == 0) fro_part[(int64_t)f * nb + blk] = red[0] + red[1] + red[2] + red[3];
    }
}

// The ksplit partial products of k_xw summed in order (grid (ceil(m/64), nf),
// XCD-aware): Y, the FP64 Gram partials of its 64-row blocks and, with
// fro_part, ||X||^2 per block from the partial sums in frop.
template <int LP>
__global__ __launch_bounds__(GT) void k_ysum(const float *__restrict__ ypart, int m, int p, int nf, int ksplit,
                                             float *__restrict__ Y, double *__restrict__ gram_part,
                                             const double *__restrict__ frop, double *__restrict__ fro_part,
                                             const int32_t *__restrict__ fmap) {
    constexpr int NB = LP / 16;
    constexpr int YS = 64 * (LP + 1) > 512 * gram_tiles<LP>() ? 64 * (LP + 1) : 512 * gram_tiles<LP>();
    __shared__ __align__(16) float ys[YS];
    const int nb = (m + 63) / 64;
    int blk, f;
    xcd_map(blockIdx.x, nb, nf, blk, f);
    if (f >= nf) return;  // a padding face of the grid
    if (fmap && fmap[f] < 0) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, a0 = blk * 64;
    const float *Pf = ypart + (int64_t)f * p * LP;
    float *Yf = Y + (int64_t)f * m * LP;
    // the sums in row order (a lane per row: every load 64 consecutive rows
    // of a column), staged in LDS as ys[r * (LP+1) + c]
    // (four partials of all of a thread's columns in flight at once; every
    // sum in the order of the partials)
    constexpr int PER = 64 * LP / GT;
    const int r = a0 + lane;
    const bool rok = r < m;
    const float *src = Pf + (rok ? r : 0);
    const int64_t pst = (int64_t)m * LP;
    float t[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) t[u] = 0.0f;
    int q = 0;
    for (; q + 4 <= ksplit; q += 4) {
        float v[4][PER];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int u = 0; u < PER; ++u) v[i][u] = src[(q + i) * pst + (int64_t)m * (wave + 4 * u)];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int u = 0; u < PER; ++u) t[u] += v[i][u];
    }
    for (; q < ksplit; ++q) {
        float v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) v[u] = src[q * pst + (int64_t)m * (wave + 4 * u)];
#pragma unroll
        for (int u = 0; u < PER; ++u) t[u] += v[u];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int c = wave + 4 * u;
        if (rok) Yf[r + (int64_t)m * c] = t[u];
        ys[lane * (LP + 1) + c] = rok ? t[u] : 0.0f;
    }
    __syncthreads();
    // the MFMA output layout block_gram_f64 takes: row 16 wave + 4 (lane/16) + v,
    // column 16 j + lane % 16
    f32x4 acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[j][v] = ys[(16 * wave + 4 * (lane >> 4) + v) * (LP + 1) + 16 * j + (lane & 15)];
    __syncthreads();
    block_gram_f64<LP>(acc, gram_part + ((int64_t)f * nb + blk) * LP * LP, ys, reinterpret_cast<double *>(ys));
    if (fro_part && tid == 0) {
        double t = 0.0;
        for (int q = 0; q < ksplit; ++q) t += frop[(int64_t)f * nb * kResidSplitMax + blk * ksplit + q];
        fro_part[(int64_t)f * nb + blk] = t;
    }
}

// ---------------------------------------------------------------- Z = X^T W
// Grid (ceil(p/64), nf).  Workgroup: output rows b0..b0+63 (columns of the
// face), K = m in chunks of 64.  W is m x nw (leading dim ldw), per face.
// RES (with GRAM, W = Q with ldw = m, the projection B^T = X^T Q): the
// workgroup then also sums ||X[:, b0:b0+64] - Q B[:, b0:b0+64]||_F^2 into
// res_part[f * nb + blk], computed directly (not by cancellation): Q B by
// FP32 MFMA from the block of B^T it has just formed, differences and squares
// in FP64.  It reads the X block a second time, last chunk first, so the
// chunks it read most recently come from cache.  Together with the discarded
// eigenvalues of B B^T this is the error of the truncated result.
// VEC: m is a multiple of 4, X is 16-byte aligned and a face spans less than
// 4 GiB (checked by the caller), so the four consecutive rows a lane reads
// are one 16-byte load at a 32-bit offset from the face.  Loads go to
// clamped addresses; bit masks mark the valid values and are applied when
// the values are used, so no instruction waits on a load still in flight.
template <int LP, int PROD, bool GRAM, bool RES, bool VEC>
__global__ __launch_bounds__(GT) void k_xtw(const float *__restrict__ X, int m, int p, int nf,
                                            const float *__restrict__ W, int64_t w_stride, int ldw,
                                            int nw, float *__restrict__ Z,
                                            double *__restrict__ gram_part,
                                            double *__restrict__ res_part,
    const int32_t *__restrict__ fmap) {
    constexpr int KC = 64, LDK = KC + 8;
    constexpr int NB = LP / 16, WPT = KC * LP / GT;
    constexpr bool SPL = PROD == PROD_SPLIT;
    static_assert(!RES || GRAM, "the residual takes B^T from the Gram staging");
    // LDS: the BF16 operands of the main loop; the residual stages the FP32
    // Q chunk (64 x (LP+1)) in the same bytes afterwards
    constexpr int XS = 64 * LDK, WS = LP * LDK;  // uint16 elements, multiples of 8
    // and, after the loop, the Gram's half-tile sums (GRB bytes)
    constexpr int MAINB = (SPL ? 2 : 1) * (XS + WS) * 2, QSB = RES ? 64 * (LP + 1) * 4 : 0;
    constexpr int GRB = GRAM ? 2048 * gram_tiles<LP>() : 0, SB0 = MAINB > QSB ? MAINB : QSB;
    __shared__ __align__(16) uint16_t smem[(SB0 > GRB ? SB0 : GRB) / 2];
    __shared__ float ys[GRAM ? 64 * (LP + 1) : 1];
    __shared__ double red[RES ? GT / 64 : 1];
    uint16_t *xh = smem, *wh = smem + XS;
    uint16_t *xl = SPL ? smem + XS + WS : xh, *wl = SPL ? smem + 2 * XS + WS : wh;
    const int nb = (p + 63) / 64;
    int blk, f;
    xcd_map(blockIdx.x, nb, nf, blk, f);
    if (f >= nf) return;  // a padding face of the grid
    if (fmap && fmap[f] < 0) return;  // an unused slot of a face list sized on the device
    const int b0 = blk * 64;
    const float *Xf = X + (int64_t)(fmap ? fmap[f] : f) * m * p;
    const float *Wf = W + (int64_t)f * w_stride;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int q4 = tid & 15, cj0 = tid >> 4;  // X load mapping: 4 rows, column
    f32x4 acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = f32x4{0, 0, 0, 0};
    const char *Xb = reinterpret_cast<const char *>(Xf), *Wb = reinterpret_cast<const char *>(Wf);
    float xr[16], wr[WPT];
    uint32_t xm = 0, wm = 0;
    auto load = [&](int a0) {
        xm = 0;
        wm = 0;
        if constexpr (VEC) {  // a < m implies a + 3 < m
            const int a = a0 + 4 * q4;
#pragma unroll
            for (int it = 0; it < 4; ++it) {
                const int b = b0 + cj0 + 16 * it;
                const bool ok = b < p && a < m;
                const uint32_t off = ok ? 4u * ((uint32_t)a + (uint32_t)m * (uint32_t)b) : 0u;
                const f32x4 x = *reinterpret_cast<const f32x4 *>(Xb + off);
#pragma unroll
                for (int v = 0; v < 4; ++v) xr[4 * it + v] = x[v];
                xm |= ok ? 0xFu << (4 * it) : 0u;
            }
        } else {
            // one row per lane, 16 columns per wavefront: every load is 64
            // consecutive rows of one column
            const int a = a0 + lane;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int b = b0 + 16 * wave + i;
                const bool ok = b < p && a < m;
                xr[i] = Xf[ok ? a + (int64_t)m * b : 0];
                xm |= (uint32_t)ok << i;
            }
        }
        if constexpr (VEC) {  // four consecutive rows of W (m, ldw multiples of 4)
#pragma unroll
            for (int q = 0; q < WPT / 4; ++q) {
                const int e = tid + q * GT, k4 = e % (KC / 4), c = e / (KC / 4), aw = a0 + 4 * k4;
                const bool ok = c < nw && aw < m;
                const f32x4 x = *reinterpret_cast<const f32x4 *>(
                    Wb + (ok ? 4u * ((uint32_t)aw + (uint32_t)ldw * (uint32_t)c) : 0u));
#pragma unroll
                for (int v = 0; v < 4; ++v) wr[4 * q + v] = x[v];
                wm |= ok ? 0xFu << (4 * q) : 0u;
            }
        } else {
#pragma unroll
            for (int q = 0; q < WPT; ++q) {
                const int e = tid + q * GT, k = e % KC, c = e / KC, aw = a0 + k;
                const bool ok = c < nw && aw < m;
                wr[q] = *reinterpret_cast<const float *>(Wb + (ok ? 4u * ((uint32_t)aw + (uint32_t)ldw * (uint32_t)c) : 0u));
                wm |= (uint32_t)ok << q;
            }
        }
    };
    load(0);
    for (int a0 = 0; a0 < m; a0 += KC) {
        if constexpr (VEC) {
#pragma unroll
            for (int it = 0; it < 4; ++it) {
                const int cj = cj0 + 16 * it;
                float x[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) x[v] = (xm >> (4 * it + v)) & 1u ? xr[4 * it + v] : 0.0f;
                uint2 ph, pl;
                split2(x[0], x[1], ph.x, pl.x);
                split2(x[2], x[3], ph.y, pl.y);
                *reinterpret_cast<uint2 *>(&xh[cj * LDK + 4 * q4]) = ph;
                if (SPL) *reinterpret_cast<uint2 *>(&xl[cj * LDK + 4 * q4]) = pl;
            }
        } else {  // row a0 + lane of columns 16 wave + i
#pragma unroll
            for (int i = 0; i < 16; i += 2) {
                uint32_t hh, ll;
                split2((xm >> i) & 1u ? xr[i] : 0.0f, (xm >> (i + 1)) & 1u ? xr[i + 1] : 0.0f, hh, ll);
                const int cj = 16 * wave + i;
                xh[cj * LDK + lane] = (uint16_t)hh;
                xh[(cj + 1) * LDK + lane] = (uint16_t)(hh >> 16);
                if (SPL) {
                    xl[cj * LDK + lane] = (uint16_t)ll;
                    xl[(cj + 1) * LDK + lane] = (uint16_t)(ll >> 16);
                }
            }
        }
        if constexpr (VEC) {
#pragma unroll
            for (int q = 0; q < WPT / 4; ++q) {  // rows 4k4 .. 4k4+3 of column c
                const int e = tid + q * GT, k4 = e % (KC / 4), c = e / (KC / 4);
                float w4[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) w4[v] = (wm >> (4 * q + v)) & 1u ? wr[4 * q + v] : 0.0f;
                uint2 h, l;
                split2(w4[0], w4[1], h.x, l.x);
                split2(w4[2], w4[3], h.y, l.y);
                *reinterpret_cast<uint2 *>(&wh[c * LDK + 4 * k4]) = h;
                if (SPL) *reinterpret_cast<uint2 *>(&wl[c * LDK + 4 * k4]) = l;
            }
        } else {
#pragma unroll
            for (int q = 0; q < WPT; q += 2) {
                const int e0 = tid + q * GT, e1 = e0 + GT;
                uint32_t hh, ll;
                split2((wm >> q) & 1u ? wr[q] : 0.0f, (wm >> (q + 1)) & 1u ? wr[q + 1] : 0.0f, hh, ll);
                wh[(e0 / KC) * LDK + e0 % KC] = (uint16_t)hh;
                wh[(e1 / KC) * LDK + e1 % KC] = (uint16_t)(hh >> 16);
                if (SPL) {
                    wl[(e0 / KC) * LDK + e0 % KC] = (uint16_t)ll;
                    wl[(e1 / KC) * LDK + e1 % KC] = (uint16_t)(ll >> 16);
                }
            }
        }
        __syncthreads();
        if (a0 + KC < m) load(a0 + KC);  // next chunk in flight during the MFMAs
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
    if (GRAM)
        block_gram_f64<LP>(acc, gram_part + ((int64_t)f * nb + blk) * LP * LP, ys, reinterpret_cast<double *>(smem));
    if (RES) {
        // ys[b * (LP+1) + c] = B^T[b0 + b][c] (rows past p are zero): the
        // B operands of the 16x16x4 MFMA (k = lane/16, column lane%16)
        constexpr int LD = LP + 1, KK = LP / 4;
        float *qs = reinterpret_cast<float *>(smem);
        // X values of the MFMA output positions: rows a = a0 + 16*wave +
        // 4*(lane/16) + v (four consecutive rows), columns b = b0 + 16t + lane%16
        auto rload = [&](int a0, f32x4(&xv)[4], uint32_t &msk) {
            const int a = a0 + 16 * wave + 4 * (lane >> 4);
            msk = 0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int b = b0 + 16 * t + (lane & 15);
                const bool bok = b < p;
                if constexpr (VEC) {
                    const bool ok = bok && a < m;
                    const uint32_t off = ok ? 4u * ((uint32_t)a + (uint32_t)m * (uint32_t)b) : 0u;
                    xv[t] = *reinterpret_cast<const f32x4 *>(Xb + off);
                    msk |= ok ? 0xFu << (4 * t) : 0u;
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const bool ok = bok && a + v < m;
                        xv[t][v] = Xf[ok ? a + v + (int64_t)m * b : 0];
                        msk |= (uint32_t)ok << (4 * t + v);
                    }
                }
            }
        };
        const int nch = (m + KC - 1) / KC;
        double racc = 0.0;
        f32x4 xv[4], xn[4];
        uint32_t vm, nm = 0;
        rload((nch - 1) * KC, xv, vm);
        for (int ci = nch - 1; ci >= 0; --ci) {
            const int a0 = ci * KC;
            if constexpr (VEC) stage_panel4<LP, 64>(Wf, m, a0, qs);
            else stage_panel<LP, 64>(Wf, m, a0, qs);
            __syncthreads();
            if (ci > 0) rload(a0 - KC, xn, nm);  // next chunk in flight during the MFMAs
            f32x4 pr[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) pr[t] = f32x4{0, 0, 0, 0};
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                if (4 * kk >= nw) break;  // columns past ell of Q are zero
                const float av = qs[(16 * wave + (lane & 15)) * LD + 4 * kk + (lane >> 4)];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float bv = ys[(16 * t + (lane & 15)) * LD + 4 * kk + (lane >> 4)];
                    pr[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, pr[t], 0, 0, 0);
                }
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float x = (vm >> (4 * t + v)) & 1u ? xv[t][v] : 0.0f;
                    const double d = (double)x - (double)pr[t][v];
                    racc += d * d;
                }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < 4; ++t) xv[t] = xn[t];
            vm = nm;
        }
        racc = wave_sum(racc);
        if (lane == 0) red[wave] = racc;
        __syncthreads();
        if (tid == 0) res_part[(int64_t)f * nb + blk] = red[0] + red[1] + red[2] + red[3];
    }
}

// ---------------------------------------------------------------- FP64 passes
// The passes of the FP64 randomized truncation (PREC_F64_RAND): the same
// products as above on FP64 data, by FP64 MFMA 16x16x4 (A[i][k]: lane%16 = i,
// lane/16 = k; B[k][j]: lane/16 = k, lane%16 = j; result row lane/16 + 4v,
// column lane%16), FP64 accumulation.  Workgroups as above (64 rows, or 64
// columns, of one face; all LP result columns), K in chunks of 32 staged in
// LDS, the next chunk's loads issued before the current chunk's products.
// Loads: consecutive lanes read consecutive rows of one column (512 bytes per
// wavefront and instruction), addresses clamped, invalid values zeroed.

// FP64 Gram of the 64 x LP block held in the four wavefronts' FP64
// accumulators (row 16*wave + lane/16 + 4v, column 16*j + lane%16), packed
// upper tiles as block_gram_f64 writes them.  ys: 64 * (LP + 1) doubles.
template <int LP>
__device__ void block_gram_f64d(const f64x4 (&acc)[LP / 16], double *__restrict__ out, double *ys, double *red) {
    constexpr int NT = LP / 16, NTILE = gram_tiles<LP>(), IPW = (2 * NTILE + 3) / 4;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) ys[(16 * wave + (lane >> 4) + 4 * v) * (LP + 1) + 16 * j + (lane & 15)] = acc[j][v];
    __syncthreads();
    f64x4 g[IPW];
#pragma unroll
    for (int u = 0; u < IPW; ++u) {
        g[u] = f64x4{0, 0, 0, 0};
        const int it = wave + 4 * u;
        if (it >= 2 * NTILE) continue;
        int ti, tj;
        tile_ij<NT>(it >> 1, ti, tj);
        const int r0 = 32 * (it & 1);
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            const int r = r0 + 4 * kk + (lane >> 4);
            g[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ys[r * (LP + 1) + 16 * ti + (lane & 15)],
                                                        ys[r * (LP + 1) + 16 * tj + (lane & 15)], g[u], 0, 0, 0);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < IPW; ++u) {
        const int it = wave + 4 * u;
        if (it < 2 * NTILE && (it & 1)) {
#pragma unroll
            for (int v = 0; v < 4; ++v) red[(it >> 1) * 256 + 64 * v + lane] = g[u][v];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < IPW; ++u) {
        const int it = wave + 4 * u;
        if (it >= 2 * NTILE || (it & 1)) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v)
            out[(it >> 1) * 256 + 64 * v + lane] = g[u][v] + red[(it >> 1) * 256 + 64 * v + lane];
    }
    __syncthreads();
}

template <int LP>
constexpr int gram64_lds() {  // doubles for the Gram staging and its tile halves
    return 64 * (LP + 1) > 256 * gram_tiles<LP>() ? 64 * (LP + 1) : 256 * gram_tiles<LP>();
}

// Y = X W: grid (ceil(m/64) * nf) through xcd_map.  W (p x nw used columns,
// leading dim ldw, FP32 or FP64) per face (stride w_stride) or shared.
template <int LP, typename TW, bool GRAM>
__global__ __launch_bounds__(GT) void k_xw64(const double *__restrict__ X, int m, int p, int nf,
                                             const TW *__restrict__ W, int64_t w_stride, int ldw, int nw,
                                             double *__restrict__ Y, double *__restrict__ fro_part,
                                             double *__restrict__ gram_part) {
    constexpr int KC = 32, XL = KC + 1, WL = LP + 1, NB = LP / 16, WPT = KC * LP / GT;
    __shared__ double xs[64 * XL];  // xs[r * XL + k] = X[a0 + r][b0 + k]
    __shared__ double ws[KC * WL];  // ws[k * WL + c] = W[b0 + k][c]
    __shared__ double ys[GRAM ? gram64_lds<LP>() : 1];
    __shared__ double red[GT / 64];
    const int nb = (m + 63) / 64;
    int blk, f;
    xcd_map(blockIdx.x, nb, nf, blk, f);
    if (f >= nf) return;  // a padding face of the grid
    const int a0 = blk * 64, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const double *Xf = X + (int64_t)f * m * p;
    const TW *Wf = W + (int64_t)f * w_stride;
    const int xr_ = tid & 63, xc0 = tid >> 6;  // X loads: row a0 + xr_, columns xc0 + 4i
    const bool rok = a0 + xr_ < m;
    double xv[KC / 4], wv[WPT];
    auto load = [&](int b0) {
#pragma unroll
        for (int i = 0; i < KC / 4; ++i) {
            const int b = b0 + xc0 + 4 * i;
            const bool ok = rok && b < p;
            const double v = Xf[ok ? (a0 + xr_) + (int64_t)m * b : 0];
            xv[i] = ok ? v : 0.0;
        }
#pragma unroll
        for (int q = 0; q < WPT; ++q) {
            const int e = tid + q * GT, k = e % KC, c = e / KC, b = b0 + k;
            const bool ok = c < nw && b < p;
            const double v = (double)Wf[ok ? b + (int64_t)ldw * c : 0];
            wv[q] = ok ? v : 0.0;
        }
    };
    f64x4 acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = f64x4{0, 0, 0, 0};
    double fro = 0.0;
    load(0);
    for (int b0 = 0; b0 < p; b0 += KC) {
#pragma unroll
        for (int i = 0; i < KC / 4; ++i) {
            xs[xr_ * XL + xc0 + 4 * i] = xv[i];
            fro += xv[i] * xv[i];
        }
#pragma unroll
        for (int q = 0; q < WPT; ++q) {
            const int e = tid + q * GT;
            ws[(e % KC) * WL + e / KC] = wv[q];
        }
        __syncthreads();
        if (b0 + KC < p) load(b0 + KC);
        const int ar = 16 * wave + (lane & 15);
#pragma unroll
        for (int kk = 0; kk < KC / 4; ++kk) {
            const int k = 4 * kk + (lane >> 4);
            const double a = xs[ar * XL + k];
#pragma unroll
            for (int j = 0; j < NB; ++j)
                acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, ws[k * WL + 16 * j + (lane & 15)], acc[j], 0, 0, 0);
        }
        __syncthreads();
    }
    double *Yf = Y + (int64_t)f * m * LP;
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = a0 + 16 * wave + (lane >> 4) + 4 * v;
            if (r < m) Yf[r + (int64_t)m * (16 * j + (lane & 15))] = acc[j][v];
        }
    if (GRAM) block_gram_f64d<LP>(acc, gram_part + ((int64_t)f * nb + blk) * LP * LP, ys, ys);
    if (fro_part) {
        fro = wave_sum(fro);
        if (lane == 0) red[wave] = fro;
        __syncthreads();
        if (tid == 0) fro_part[(int64_t)f * nb + blk] = red[0] + red[1] + red[2] + red[3];
    }
}

// Z = X^T W: grid (ceil(p/64) * nf) through xcd_map; workgroup: columns
// b0 .. b0+63 of X (rows of Z), K = m.  W (m x nw, leading dim ldw, FP64)
// per face (stride w_stride).
template <int LP, bool GRAM>
__global__ __launch_bounds__(GT) void k_xtw64(const double *__restrict__ X, int m, int p, int nf,
                                              const double *__restrict__ W, int64_t w_stride, int ldw, int nw,
                                              double *__restrict__ Z, double *__restrict__ gram_part) {
    constexpr int KC = 32, XL = KC + 1, WL = LP + 1, NB = LP / 16, WPT = KC * LP / GT;
    __shared__ double xs[64 * XL];  // xs[c * XL + k] = X[a0 + k][b0 + c]
    __shared__ double ws[KC * WL];  // ws[k * WL + j] = W[a0 + k][j]
    __shared__ double ys[GRAM ? gram64_lds<LP>() : 1];
    const int nb = (p + 63) / 64;
    int blk, f;
    xcd_map(blockIdx.x, nb, nf, blk, f);
    if (f >= nf) return;  // a padding face of the grid
    const int b0 = blk * 64, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const double *Xf = X + (int64_t)f * m * p;
    const double *Wf = W + (int64_t)f * w_stride;
    const int xk = tid & 31, xc0 = tid >> 5;  // X loads: row a0 + xk, columns b0 + xc0 + 8i
    double xv[8], wv[WPT];
    auto load = [&](int a0) {
        const bool kok = a0 + xk < m;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int b = b0 + xc0 + 8 * i;
            const bool ok = kok && b < p;
            const double v = Xf[ok ? (a0 + xk) + (int64_t)m * b : 0];
            xv[i] = ok ? v : 0.0;
        }
#pragma unroll
        for (int q = 0; q < WPT; ++q) {
            const int e = tid + q * GT, k = e % KC, c = e / KC, a = a0 + k;
            const bool ok = c < nw && a < m;
            const double v = Wf[ok ? a + (int64_t)ldw * c : 0];
            wv[q] = ok ? v : 0.0;
        }
    };
    f64x4 acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = f64x4{0, 0, 0, 0};
    load(0);
    for (int a0 = 0; a0 < m; a0 += KC) {
#pragma unroll
        for (int i = 0; i < 8; ++i) xs[(xc0 + 8 * i) * XL + xk] = xv[i];
#pragma unroll
        for (int q = 0; q < WPT; ++q) {
            const int e = tid + q * GT;
            ws[(e % KC) * WL + e / KC] = wv[q];
        }
        __syncthreads();
        if (a0 + KC < m) load(a0 + KC);
        const int cr = 16 * wave + (lane & 15);
#pragma unroll
        for (int kk = 0; kk < KC / 4; ++kk) {
            const int k = 4 * kk + (lane >> 4);
            const double a = xs[cr * XL + k];
#pragma unroll
            for (int j = 0; j < NB; ++j)
                acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, ws[k * WL + 16 * j + (lane & 15)], acc[j], 0, 0, 0);
        }
        __syncthreads();
    }
    double *Zf = Z + (int64_t)f * p * LP;
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = b0 + 16 * wave + (lane >> 4) + 4 * v;
            if (r < p) Zf[r + (int64_t)p * (16 * j + (lane & 15))] = acc[j][v];
        }
    if (GRAM) block_gram_f64d<LP>(acc, gram_part + ((int64_t)f * nb + blk) * LP * LP, ys, ys);
}

// ---------------------------------------------------------------- Gram groups
// In place: partial g*grp of face f becomes the ordered sum of that face's
// partials g*grp .. g*grp+grp-1 (grid (groups x element blocks, nf); a
// thread per packed element and group, eight loads in flight), so a
// Cholesky-QR whose rows are spread over many workgroups (cholqr_row_groups)
// sums a few group sums in each of them instead of every partial.
template <int LP>
__global__ __launch_bounds__(256) void k_gram_group(double *__restrict__ gpart, int nparts, int grp,
                                                    const int32_t *__restrict__ fmap) {
    constexpr int NE2 = gram_tiles<LP>() * 128, NBK = (NE2 + 255) / 256, S2 = LP * LP / 2;
    const int f = blockIdx.y;
    if (fmap && fmap[f] < 0) return;
    const int g = blockIdx.x / NBK, e2 = (blockIdx.x % NBK) * 256 + threadIdx.x;
    const int p0 = g * grp, p1 = p0 + grp < nparts ? p0 + grp : nparts;
    if (e2 >= NE2 || p0 >= nparts) return;
    double2 *g2 = reinterpret_cast<double2 *>(gpart + (int64_t)f * nparts * LP * LP);
    double2 acc = double2{0.0, 0.0};
    for (int pp = p0; pp < p1; pp += 8) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = pp + u < p1 ? pp + u : p1 - 1;
            const double2 t = g2[(int64_t)q * S2 + e2];
            v[u] = pp + u < p1 ? t : double2{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            acc.x += v[u].x;
            acc.y += v[u].y;
        }
    }
    g2[(int64_t)p0 * S2 + e2] = acc;
}
template <int LP>
inline unsigned gram_group_blocks(int nparts, int grp) {
    constexpr int NE2 = gram_tiles<LP>() * 128;
    return (unsigned)(((nparts + grp - 1) / grp) * ((NE2 + 255) / 256));
}

// ---------------------------------------------------------------- Cholesky-QR
// Orthonormal basis Q (rows x LP, FP32, columns >= ell zero) of the rows x ell
// panel S by shifted Cholesky-QR (Fukaya et al. 2020): G = S^T S (+ shift on
// the first pass), R = chol(G), Q = S R^{-1}; `passes` = 2 repeats the step on
// Q (Cholesky-QR2).  One workgroup per face, QT threads, one row per thread:
//  * the first Gram is the sum of the per-64-row-block partials written by the
//    GEMM pass that produced S (all loads of a block of 8 partials in flight);
//  * the Cholesky factorisation is right-looking with one barrier per column,
//    every thread loading its operands of a step before it writes any;
//  * the triangular solve runs in registers, fully unrolled, with R^T read by
//    LDS broadcast; the row is solved in FP64 and stored as FP32;
//  * the Gram of the first pass's Q, for the second pass, comes from those FP32
//    rows staged in LDS (FP64 MFMA), so the second pass reads nothing from HBM
//    when the panel fits in one chunk of QT rows.
// With one pass the rows are independent once R is known: gridDim.y
// workgroups per face (cholqr_row_groups) each form the same R and solve the
// chunks blockIdx.y, blockIdx.y + gridDim.y, ..  (a few tall panels on many
// CUs; every row as with one workgroup).  Two passes need gridDim.y = 1.
constexpr int QT = 512;

// Workgroups per face for a one-pass Cholesky-QR of nf panels of `rows` rows:
// about 256 in all, at most one per chunk of QT rows.
inline unsigned cholqr_row_groups(int64_t rows, int64_t nf) {
    const int64_t nch = (rows + QT - 1) / QT, want = nf > 0 ? 256 / nf : 1;
    const int64_t g = want < nch ? want : nch;
    return g < 1 ? 1u : (unsigned)g;
}

// T: the panel's element type (FP32 in the mixed path, FP64 in the FP64
// randomized path, which stages fewer rows per LDS pass).
// fmap: face list (an entry < 0 is an unused slot); src_global: the panel and
// its Gram partials are indexed by the listed face and written for width
// src_lp (a sketch taken once for all faces, whose first columns this
// width-LP basis reuses), the output by the list position.
template <int LP, typename T = float>
__global__ __launch_bounds__(QT) void k_cholqr(const T *__restrict__ Sin, int rows, int ell,
                                               T *__restrict__ Qout, int passes,
                                               const double *__restrict__ gpart, int nparts,
                                               int32_t *__restrict__ qr_info, int first,
                                               const int32_t *__restrict__ fmap = nullptr, int src_global = 0,
                                               int src_lp = LP, int pgroup = 1) {
    constexpr bool D = sizeof(T) == 8;
    constexpr int LDG = LP + 1, LDR = LP + 2, LDS_ = LP + 1;
    // rows staged per LDS round for the second pass's Gram: a quarter of the
    // chunk keeps the kernel's LDS near 60 KB at width 48, so GEMM workgroups
    // of another face group can share the CU with it
    constexpr int HR = D ? (LP <= 32 ? QT / 2 : QT / 4) : QT / 4;
    constexpr int NT = LP / 16, NTILE = NT * (NT + 1) / 2, TPW = (NTILE + 7) / 8;
    __shared__ double G[LP * LDG];
    __shared__ __align__(16) double Rt[LP * LDR];  // Rt[c * LDR + j] = R[j][c]
    __shared__ double rinv[LP];
    __shared__ T st[HR * LDS_];  // rows of the chunk (or part of it) for the Gram
    __shared__ double trace_s;
    __shared__ int bad;
    const int f = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (fmap && fmap[f] < 0) return;  // an unused slot of a face list sized on the device
    const int fs = src_global ? fmap[f] : f, slp = src_global ? src_lp : LP;
    const T *S = Sin + (int64_t)fs * rows * slp;
    T *Q = Qout + (int64_t)f * rows * LP;
    if (tid == 0) bad = 0;

    // ---- first Gram: ordered sum of the partials (of their group sums, pgroup > 1)
    if (pgroup > 1) load_gram_partials<LP, QT>(gpart, fs, (nparts + pgroup - 1) / pgroup, G, LDG, slp, pgroup, nparts);
    else load_gram_partials<LP, QT>(gpart, fs, nparts, G, LDG, slp);
    __syncthreads();

    const int nch = (rows + QT - 1) / QT;
    T x[LP];
    for (int pass = 0; pass < passes; ++pass) {
        // ---- the rounding level of the Gram, 11 (rows*ell + ell(ell+1)) u tr(G)
        // (u = 2^-53): the first pass adds it to the diagonal as the shift;
        // later passes, on a basis the shifted pass has already equilibrated,
        // take a pivot at or below it as a numerically dependent direction
        // and drop it (zero column of Q, no flag) instead of dividing by it
        if (wave == 0) {
            double t = 0.0;
            for (int c = lane; c < ell; c += 64) t += G[c * LDG + c];
            t = wave_sum(t);
            if (lane == 0) trace_s = t;
        }
        __syncthreads();
        const double level = 11.0 * ((double)rows * ell + (double)ell * (ell + 1)) * 0x1p-53 * trace_s;
        const double pfloor = pass == 0 ? 0.0 : level;
        if (pass == 0) {
            if (tid < ell) G[tid * LDG + tid] += level;
            __syncthreads();
        }
        // ---- Cholesky of the leading ell x ell block.  Step j subtracts the
        // outer product of row j over the pivot from the rows below; row j of
        // the trailing matrix is final after step j, so the rows of R
        // (row j / sqrt(pivot j)) are formed afterwards, all at once.  The
        // upper entries (i, c) are numbered by decreasing row, so the entries
        // a step updates (i > j) are a prefix of the numbering: wavefronts
        // past it skip the step, the others read their operands branch free.
        {
            constexpr int NU = LP * (LP + 1) / 2, UPT = (NU + QT - 1) / QT;
            int ei[UPT], ec[UPT];
#pragma unroll
            for (int u = 0; u < UPT; ++u) {
                // entry e: rows ell-1, ell-2, .. 0, each with columns i .. ell-1
                int rem = tid + u * QT, i = ell - 1;
                while (i >= 0 && rem >= ell - i) {
                    rem -= ell - i;
                    --i;
                }
                ei[u] = i;  // -1: no entry
                ec[u] = i >= 0 ? i + rem : 0;
            }
            for (int j = 0; j < ell; ++j) {
                const int cnt = (ell - j - 1) * (ell - j) / 2;  // entries with i > j
                const double piv = G[j * LDG + j];
                const double ipv = piv > pfloor && isfinite(piv) ? recip(piv) : 0.0;
#pragma unroll
                for (int u = 0; u < UPT; ++u) {
                    if (u * QT + (tid & ~63) >= cnt) break;  // whole wavefront past the prefix
                    const bool act = tid + u * QT < cnt;
                    const int i = act ? ei[u] : j, c = act ? ec[u] : j;
                    const double gji = G[j * LDG + i], gjc = G[j * LDG + c], gic = G[i * LDG + c];
                    const double l = gji * ipv;
                    if (act) G[i * LDG + c] = gic - l * gjc;
                }
                __syncthreads();
            }
            // R[j][c] = G[j][c] / sqrt(G[j][j]), c >= j.  A pivot at or below
            // the floor of a later pass drops direction j (rinv 0: a zero
            // column, skipped by the elimination above); a non-positive pivot
            // of the shifted pass (a zero or non-finite panel) gives a unit
            // row and the flag
            for (int e = tid; e < ell * ell; e += QT) {
                const int j = e / ell, c = e % ell;
                if (c < j) continue;
                const double piv = G[j * LDG + j];
                const bool fin = isfinite(piv), ok = fin && piv > pfloor, drop = fin && !ok && pass > 0;
                const double d = ok ? sqrt(piv) : 1.0;
                Rt[c * LDR + j] = ok ? G[j * LDG + c] / d : (c == j ? 1.0 : 0.0);
                if (c == j) {
                    rinv[j] = drop ? 0.0 : 1.0 / d;
                    if (!ok && !drop) bad = 1;
                }
            }
            __syncthreads();
        }
        // ---- Q = S R^{-1}, chunks of QT rows; Gram of the result for the next pass
        const bool again = pass + 1 < passes;
        f64x4 gacc[TPW];
#pragma unroll
        for (int t = 0; t < TPW; ++t) gacc[t] = f64x4{0, 0, 0, 0};
        for (int ch = blockIdx.y; ch < nch; ch += gridDim.y) {
            const int row = ch * QT + tid;
            if (pass == 0 || nch > 1) {
                const T *src = (pass == 0 ? S : Q) + (row < rows ? row : rows - 1);
#pragma unroll
                for (int c = 0; c < LP; ++c) x[c] = src[(int64_t)rows * c];
                if (row >= rows) {
#pragma unroll
                    for (int c = 0; c < LP; ++c) x[c] = (T)0;
                }
            }
            double qd[LP];
#pragma unroll
            for (int c = 0; c < LP; ++c) {
                if (c < ell) {
                    double v0 = (double)x[c], v1 = 0.0, v2 = 0.0, v3 = 0.0;
                    const double *rc = Rt + c * LDR;
#pragma unroll
                    for (int j = 0; j + 3 < c; j += 4) {
                        const double2 r01 = *reinterpret_cast<const double2 *>(rc + j);
                        const double2 r23 = *reinterpret_cast<const double2 *>(rc + j + 2);
                        v0 -= qd[j] * r01.x;
                        v1 -= qd[j + 1] * r01.y;
                        v2 -= qd[j + 2] * r23.x;
                        v3 -= qd[j + 3] * r23.y;
                    }
#pragma unroll
                    for (int j = c & ~3; j < c; ++j) v0 -= qd[j] * rc[j];
                    qd[c] = ((v0 + v1) + (v2 + v3)) * rinv[c];
                } else {
                    qd[c] = 0.0;
                }
                x[c] = (T)qd[c];
            }
            if (row < rows) {
#pragma unroll
                for (int c = 0; c < LP; ++c) Q[row + (int64_t)rows * c] = x[c];
            }
            if (again) {
#pragma unroll
                for (int h = 0; h < QT / HR; ++h) {
                    if (tid / HR == h) {
                        const int r = tid % HR;
#pragma unroll
                        for (int c = 0; c < LP; ++c) st[r * LDS_ + c] = x[c];
                    }
                    __syncthreads();
#pragma unroll
                    for (int t = 0; t < TPW; ++t) {
                        const int idx = wave + 8 * t;
                        if (idx >= NTILE) continue;
                        int ti, tj;
                        tile_ij<NT>(idx, ti, tj);
#pragma unroll 4
                        for (int kk = 0; kk < HR / 4; ++kk) {
                            const int r = 4 * kk + (lane >> 4);
                            const double a = st[r * LDS_ + 16 * ti + (lane & 15)];
                            const double b = st[r * LDS_ + 16 * tj + (lane & 15)];
                            gacc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, gacc[t], 0, 0, 0);
                        }
                    }
                    __syncthreads();
                }
            }
        }
        if (again) {
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int idx = wave + 8 * t;
                if (idx >= NTILE) continue;
                int ti, tj;
                tile_ij<NT>(idx, ti, tj);
                put_sym_tile<true>(G, LDG, ti, tj, gacc[t], lane);
            }
            __syncthreads();
        }
    }
    // the first Cholesky-QR of a truncation sets the flag, later ones raise it
    if (tid == 0 && blockIdx.y == 0) {
        if (first) qr_info[f] = bad ? 2 : 0;
        else if (bad) qr_info[f] = 2;
    }
}

// ---------------------------------------------------------------- core SVD
// B B^T (sum of the projection's FP64 per-block Gram partials), its
// eigenvalues and eigenvectors by the cyclic Jacobi solver of jacobi_dev.h.
// Entries of B B^T are below 2^300 (squares of FP32 data summed over at most
// 2^16 rows), so the rotation arithmetic cannot overflow.
// Eigenvalues sorted decreasing, rank rule, certificate
//   cert^2 = ||X - Q B||^2 + sum_{j > k_f} lambda_j
// (the error of Q U_B[:, :k] U_B[:, :k]^T B, since Q has orthonormal columns).
// The energy rule takes the smallest k whose certified error meets tau.
// nres < 0 (FP64 data): ||X - Q B||^2 is taken as ||X||^2 - sum_j lambda_j,
// accurate to ~1e-16 ||X||^2, far below any tolerance tau^2 ||X||^2 in use.
// jtol: the Jacobi solver's absolute threshold over the trace.  The sums
// above use the diagonal of the rotated matrix, E^T (B B^T) E, and equal
// ||B - E_k E_k^T B||^2 for the orthogonal E the solver returns whether or
// not it has converged, so the threshold moves no certificate.
constexpr double kJacobiTolMixed = 1e-12;  // B carries ~1e-5 relative error
template <int LP>
__global__ __launch_bounds__(QT) void k_core(const double *__restrict__ gpart, int nparts, int ell,
                                             const double *__restrict__ fro_part, int nfro,
                                             const double *__restrict__ res_part, int nres,
                                             int mode, int kfix, double tau, int max_sweeps, double jtol,
                                             double *__restrict__ UB, double *__restrict__ sig,
                                             int *__restrict__ perm_out, int *__restrict__ kf_out,
                                             double *__restrict__ fro2_out, double *__restrict__ cert,
                                             int32_t *__restrict__ jinfo,
    const int32_t *__restrict__ fmap, const int32_t *__restrict__ kcap_face = nullptr, int pgroup = 1) {
    constexpr int LD = jacobi_ld<LP>(), LDE = jacobi_ld<LP>(), NPM = LP / 2;
    __shared__ __align__(16) double Gb[2][LP * LD];
    __shared__ __align__(16) double Eb[2][LP * LDE];  // eigenvectors transposed: E[c * LDE + r]
    __shared__ __align__(16) double2 cs[2][NPM];      // rotations, by round parity
    __shared__ double lam[LP];
    __shared__ int perm[LP];
    __shared__ double trace_s;
    __shared__ int rflag[3];
    const int f = blockIdx.x, tid = threadIdx.x;
    if (fmap && fmap[f] < 0) return;  // an unused slot of a face list sized on the device
    for (int e = tid; e < LP * LD; e += QT) Gb[0][e] = 0.0;
    for (int e = tid; e < LP * LDE; e += QT) Eb[0][e] = Eb[1][e] = 0.0;
    __syncthreads();
    // Gram into the leading block (the padded rows and columns of the
    // partials are zero), identity eigenvectors
    // (of their group sums, pgroup > 1: k_gram_group)
    if (pgroup > 1) load_gram_partials<LP, QT>(gpart, f, (nparts + pgroup - 1) / pgroup, Gb[0], LD, LP, pgroup, nparts);
    else load_gram_partials<LP, QT>(gpart, f, nparts, Gb[0], LD);
    if (tid < ell) Eb[0][tid * LDE + tid] = 1.0;
    if (tid < 3) rflag[tid] = 0;
    __syncthreads();
    if (tid < 64) {
        double t = 0.0;
        for (int c = tid; c < ell; c += 64) t += Gb[0][c * LD + c];
        t = wave_sum(t);
        if (tid == 0) trace_s = t;
    }
    __syncthreads();
    const double trace = trace_s;

    int conv = 0;
    const double *G, *E;
    int dslot;
    jacobi_eig<LP, QT>(Gb[0], Gb[1], Eb[0], Eb[1], &cs[0][0], rflag, ell, jtol * trace, max_sweeps, conv, G, E,
                       dslot);
    if (tid < ell) {
        const int sl = jacobi_slot(tid, dslot);
        lam[tid] = fmax(G[sl * LD + sl], 0.0);
    }
    __syncthreads();
    if (tid < ell) {
        int pos = 0;
        double li = lam[tid];
        for (int j = 0; j < ell; ++j) pos += (lam[j] > li) || (lam[j] == li && j < tid);
        perm[pos] = tid;
    }
    __syncthreads();
    if (tid == 0) {
        double fro2 = 0.0, res = 0.0;
        for (int i = 0; i < nfro; ++i) fro2 += fro_part[(int64_t)f * nfro + i];
        for (int i = 0; i < nres; ++i) res += res_part[(int64_t)f * nres + i];
        if (nres < 0) {  // FP64 data: ||X - Q B||^2 = ||X||^2 - ||B||^2 (Q orthonormal)
            double b2 = 0.0;
            for (int j = 0; j < ell; ++j) b2 += lam[j];
            res = fmax(fro2 - b2, 0.0);
        }
        int kf, miss = 0;
        if (mode == TSVDM_RANK_FIXED) {
            kf = kfix < ell ? kfix : ell;
        } else {
            int cap = kfix > 0 && kfix < ell ? kfix : ell;
            if (kcap_face) {  // a per-face cap (the predicted rank), at least 1
                const int kc = kcap_face[fmap ? fmap[f] : f];
                cap = kc < 1 ? 1 : kc < cap ? kc : cap;
            }
            double tail = res, bound = tau * tau * fro2;
            for (int j = 0; j < ell; ++j) tail += lam[j];
            kf = -1;
            for (int k = 0; k <= cap; ++k) {
                if (tail <= bound) { kf = k; break; }
                if (k < ell) tail -= lam[perm[k]];
            }
            if (kf < 0) {  // the tolerance is not met within the cap
                kf = cap;
                miss = 1;
            }
        }
        double disc = 0.0;
        for (int j = ell - 1; j >= kf; --j) disc += lam[perm[j]];
        kf_out[f] = kf;
        fro2_out[f] = fro2;
        if (cert) cert[fmap ? fmap[f] : f] = nres != 0 ? sqrt(res + disc) : -1.0;
        // bit 0: sweep cap reached; bit 2: energy target missed at the cap
        jinfo[f] = ((conv || ell <= 1) ? 0 : 1) | (miss ? 4 : 0);
    }
    for (int r = tid; r < LP; r += QT) {
        int j = r < ell ? perm[r] : r;
        sig[(int64_t)f * LP + r] = r < ell ? sqrt(lam[j]) : 0.0;
        perm_out[(int64_t)f * LP + r] = j;
    }
    for (int e = tid; e < LP * LP; e += QT)
        UB[(int64_t)f * LP * LP + e] = e / LP < ell ? E[jacobi_slot(e / LP, dslot) * LDE + e % LP] : 0.0;  // col e/LP
}

// ---------------------------------------------------------------- factors
// Uhat[:, r] = Q U_B[:, perm[r]],  Vhat[:, r] = B^T U_B[:, perm[r]] / s_r  (r < k_f;
// zero for k_f <= r < kmax).  Grid (ceil(m/64) + ceil(p/64), nf): the first
// ceil(m/64) blocks of a face make 64 rows of Uhat each, the others rows of
// Vhat.  A wavefront makes 16 rows by FP32 MFMA 16x16x4 on the transposed
// product (U_B^T Q^T), so that a lane's four results are consecutive rows; the
// inputs Q and B^T are FP32 and U_B is rounded to FP32, which adds an error of
// the order of the FP32 rounding of the inputs themselves.
template <typename T>
struct Acc4;
template <>
struct Acc4<float> {
    typedef f32x4 type;
};
template <>
struct Acc4<double> {
    typedef f64x4 type;
};

// T: element type of Q, B^T and the factors (FP32 mixed, FP64 randomized);
// FP64 uses the FP64 MFMA, whose output holds row lane/16 + 4v.
template <int LP, typename T = float>
__global__ __launch_bounds__(GT) void k_factors(const T *__restrict__ Q, const T *__restrict__ Bt,
                                                int m, int p, int ell, int64_t kmax,
                                                const double *__restrict__ UB,
                                                const double *__restrict__ sig,
                                                const int *__restrict__ perm,
                                                const int *__restrict__ kf_in,
                                                const double *__restrict__ fro2,
                                                const int32_t *__restrict__ qr_info,
                                                const int32_t *__restrict__ jinfo,
                                                T *__restrict__ Uo, double *__restrict__ So,
                                                T *__restrict__ Vo, int32_t *__restrict__ ranks,
                                                double *__restrict__ fro, int32_t *__restrict__ info,
    const int32_t *__restrict__ fmap) {
    constexpr int LU = LP + 1, NT = LP / 16;
    constexpr bool D = sizeof(T) == 8;
    typedef typename Acc4<T>::type V4;
    __shared__ T ubs[LP * LU];  // ubs[r * LU + c] = U_B[c, perm[r]] (/ s_r for V), zero for r >= k_f
    const int f = blockIdx.y, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int fd = fmap ? fmap[f] : f;
    if (fd < 0) return;  // an unused slot of a face list sized on the device
    const int kf = kf_in[f], nbu = (m + 63) / 64;
    const bool isv = (int)blockIdx.x >= nbu;
    const int blk = isv ? blockIdx.x - nbu : blockIdx.x, rows = isv ? p : m;
    const T *S = isv ? Bt + (int64_t)f * p * LP : Q + (int64_t)f * m * LP;  // rows x LP, column major
    T *O = isv ? Vo + (int64_t)fd * p * kmax : Uo + (int64_t)fd * m * kmax;
    for (int e = tid; e < LP * LP; e += GT) {
        const int r = e / LP, c = e % LP;
        T u = (T)0;
        if (r < kf && c < ell) {
            const double v = UB[(int64_t)f * LP * LP + c + (int64_t)LP * perm[(int64_t)f * LP + r]];
            const double s = sig[(int64_t)f * LP + r];
            u = (T)(isv ? (s > 0.0 ? v / s : 0.0) : v);
        }
        ubs[r * LU + c] = u;
    }
    __syncthreads();
    const int kc = kf < kmax ? kf : (int)kmax;       // columns with values
    const int nt = (kc + 15) / 16;                   // their 16-column tiles
    const int row0 = blk * 64 + 16 * wave, jr = row0 + (lane & 15), kl = lane >> 4;
    const bool rok = jr < rows;
    V4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = V4{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < LP / 4; ++kk) {
        if (4 * kk >= ell) break;  // columns past ell of U_B^T are zero
        const T x = S[rok ? jr + (int64_t)rows * (4 * kk + kl) : 0];
        const T bq = rok ? x : (T)0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t >= nt) break;
            const T a = ubs[(16 * t + (lane & 15)) * LU + 4 * kk + kl];
            if constexpr (D) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bq, acc[t], 0, 0, 0);
            else acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bq, acc[t], 0, 0, 0);
        }
    }
    // result (r = 16t + 4*(lane/16) + v for FP32, 16t + lane/16 + 4v for FP64;
    // row = row0 + lane%16)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (t >= nt) break;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 16 * t + (D ? kl + 4 * v : 4 * kl + v);
            if (rok && r < kmax) O[jr + (int64_t)rows * r] = acc[t][v];
        }
    }
    // zero columns past the computed tiles
    const int64_t zc = kmax - 16 * nt;
    for (int64_t e = tid; e < 64 * zc; e += GT) {
        const int row = blk * 64 + (int)(e % 64);
        if (row < rows) O[row + (int64_t)rows * (16 * nt + e / 64)] = (T)0;
    }
    if (blockIdx.x == 0) {
        for (int r = tid; r < kmax; r += GT) So[(int64_t)fd * kmax + r] = r < kf ? sig[(int64_t)f * LP + r] : 0.0;
        if (tid == 0) {
            ranks[fd] = kf;
            if (fro) fro[fd] = sqrt(fro2[f]);
            if (info) {
                int code = (jinfo[f] & 4) ? 4 : 0;
                if (jinfo[f] & 1) code = 1;
                if (qr_info[f]) code = 2;
                if (!isfinite(fro2[f])) code = 3;
                info[fd] = code;
            }
        }
    }
}

// ---------------------------------------------------------------- certificate
// Error of the returned factors: res_part[f * nb + blk] = the squared
// Frobenius norm of rows a0 .. a0+63 of Xhat_f - Uhat_f diag(S_f) Vhat_f^T,
// with Uhat, S, Vhat the values just stored (the first ranks[f] <= KP
// triplets).  The product is formed by FP64 MFMA 16x16x4 (A = rows of Uhat,
// exact in FP64; B = S_r times rows of Vhat, one rounding of the FP64
// product; FP64 accumulation), the differences and squares in FP64, so the
// sum is the exact error of the stored factors to a relative ~1e-15 of
// ||Xhat_f||^2.  Grid (ceil(m/64) * nf) through xcd_map; the workgroup walks
// the face's columns in chunks of 64: the X chunk (64 x 64 FP32, 16-byte
// loads of four rows when VEC) and the Vhat chunk (KP x 64) staged in LDS,
// the next chunk's loads issued before the current chunk's products (the
// S_r scaling of W is applied as the operand is read).  Wavefront w owns rows a0 + 16w .. +15 and four 16-column output tiles
// (independent accumulators); the FP64 output layout (row lane/16 + 4v,
// column lane%16) picks the X values from LDS.
// T: element type of X and the factors (FP32 mixed, FP64 randomized).
// CPLX: complex faces and factors, X read as the real 2m x p matrix X' of its
// interleaved storage (m is then 2m): (Uhat S Vhat^H)' = [Uhat' | (-i Uhat)']
// times [S Re Vhat | S Im Vhat]^T, the two column sets interleaved (column 2r
// and 2r+1 for triplet r), so the kernel runs unchanged on 2 ranks[f] columns.
// nsplit: the face's columns split into that many ranges, one workgroup per
// (64-row block, range), partial r = blk * nsplit + range (in that order, so
// the ordered sum of a face's partials is fixed); more than one only where the
// faces times row blocks leave most CUs idle (resid_splits).
template <int KP, bool VEC, typename T, bool CPLX>
__device__ __forceinline__ void resid_body(const T *__restrict__ X, int m, int p, int nf,
                                           const T *__restrict__ U, const double *__restrict__ S,
                                           const T *__restrict__ V, int64_t kmax,
                                           const int32_t *__restrict__ ranks, double *__restrict__ res_part,
                                           const int32_t *__restrict__ fmap, int nsplit) {
    constexpr int NS = KP / 4, XP = 66, VPT = KP / 4;  // V loads per thread per chunk
    __shared__ T xs[64 * XP];    // xs[c * XP + r] = X[a0 + r][b0 + c]
    constexpr int WP = 80;  // rows 4 apart fall 16 banks apart
    __shared__ T ws[KP * WP];    // ws[r * WP + c] = V[b0 + c][r]
    __shared__ double ss[KP];        // S_r
    __shared__ double red[GT / 64];
    const int nb = ((m + 63) / 64) * nsplit;
    int blkx, f;
    xcd_map(blockIdx.x, nb, nf, blkx, f);
    if (f >= nf) return;  // a padding face of the grid
    const int fd = fmap ? fmap[f] : f;
    if (fd < 0) return;  // an unused slot of a face list sized on the device
    const int blk = blkx / nsplit, sp = blkx % nsplit;
    const int cps = ((p + 63) / 64 + nsplit - 1) / nsplit;  // 64-column chunks per range
    const int c0 = sp * cps * 64, c1 = (sp + 1) * cps * 64 < p ? (sp + 1) * cps * 64 : p;
    const int a0 = blk * 64;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int rk = CPLX ? 2 * ranks[fd] : ranks[fd];
    const int kf = rk < KP ? rk : KP, ns = (kf + 3) / 4;
    const T *Xf = X + (int64_t)fd * m * p;
    const T *Uf = U + (int64_t)fd * m * kmax;
    const T *Vf = V + (int64_t)fd * (CPLX ? 2 * p : p) * kmax;
    const double *Sf = S + (int64_t)fd * kmax;
    double ua[NS];  // A operands: Uhat[a0 + 16 wave + lane%16][4 s + lane/16]
    {
        // all loads first, then (after the fence) their conversions
        const int row = a0 + 16 * wave + (lane & 15);
        T uraw[NS];
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            const int r = 4 * st + (lane >> 4);
            const bool ok = row < m && r < kf;
            int64_t idx;
            if constexpr (CPLX) {  // row 2i + a of X'; column 2r' + b
                const int rc = r >> 1, a = row & 1;
                idx = (r & 1) == 0 ? row + (int64_t)m * rc : a == 0 ? row + 1 + (int64_t)m * rc : row - 1 + (int64_t)m * rc;
            } else {
                idx = row + (int64_t)m * r;
            }
            uraw[st] = Uf[ok ? idx : 0];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            const int r = 4 * st + (lane >> 4);
            const bool ok = row < m && r < kf;
            const bool neg = CPLX && (r & 1) == 1 && (row & 1) == 1;
            ua[st] = ok ? (neg ? -(double)uraw[st] : (double)uraw[st]) : 0.0;
        }
    }
    const int xq = tid & 15, xc = tid >> 4, vc = tid & 63, vr0 = tid >> 6;
    if (tid < KP) ss[tid] = tid < kf ? Sf[CPLX ? tid >> 1 : tid] : 0.0;
    // chunk loads: X rows a0 + 4 (tid%16) .. +3 of columns b0 + tid/16 + 16 it
    // (VEC), else row a0 + lane of columns b0 + 16 wave .. +15 (every load 64
    // consecutive rows of a column); V row b0 + tid%64 of ranks tid/64 + 4 q
    T xr[16], vr[VPT];
    auto load = [&](int b0) {
        if constexpr (!VEC) {
            const int a = a0 + lane;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int b = b0 + 16 * wave + i;
                const bool ok = b < p && a < m;
                const T v = Xf[ok ? a + (int64_t)m * b : 0];
                xr[i] = ok ? v : (T)0;
            }
        }
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int b = b0 + xc + 16 * it, a = a0 + 4 * xq;
            if constexpr (VEC) {
                const bool ok = b < p && a < m;  // then a + 3 < m
                const T *src = Xf + (ok ? a + (int64_t)m * b : 0);
                if constexpr (sizeof(T) == 8) {
                    const double2 v0 = *reinterpret_cast<const double2 *>(src);
                    const double2 v1 = *reinterpret_cast<const double2 *>(src + 2);
                    xr[4 * it + 0] = ok ? v0.x : 0.0;
                    xr[4 * it + 1] = ok ? v0.y : 0.0;
                    xr[4 * it + 2] = ok ? v1.x : 0.0;
                    xr[4 * it + 3] = ok ? v1.y : 0.0;
                } else {
                    // the last read of Xhat in a truncation: non-temporal
                    const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(src));
#pragma unroll
                    for (int u = 0; u < 4; ++u) xr[4 * it + u] = ok ? v[u] : 0.0f;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int r = vr0 + 4 * q, b = b0 + vc;
            const bool ok = r < kf && b < p;
            const int64_t vo = CPLX ? 2 * (int64_t)b + (r & 1) + 2 * (int64_t)p * (r >> 1) : b + (int64_t)p * r;
            const T v = Vf[ok ? vo : 0];
            vr[q] = ok ? v : (T)0;
        }
    };
    double racc = 0.0;
    if (c0 < c1) load(c0);
    for (int b0 = c0; b0 < c1; b0 += 64) {
        if constexpr (VEC) {
#pragma unroll
            for (int it = 0; it < 4; ++it)
#pragma unroll
                for (int u = 0; u < 4; ++u) xs[(xc + 16 * it) * XP + 4 * xq + u] = xr[4 * it + u];
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) xs[(16 * wave + i) * XP + lane] = xr[i];
        }
#pragma unroll
        for (int q = 0; q < VPT; ++q) ws[(vr0 + 4 * q) * WP + vc] = vr[q];
        __syncthreads();
        if (b0 + 64 < c1) load(b0 + 64);  // next chunk in flight during the products
        f64x4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = f64x4{0, 0, 0, 0};
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            if (st >= ns) break;
            const int r = 4 * st + (lane >> 4);
            const double sr = ss[r];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[st], sr * (double)ws[r * WP + 16 * t + (lane & 15)],
                                                           acc[t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double d = (double)xs[(16 * t + (lane & 15)) * XP + 16 * wave + (lane >> 4) + 4 * v] - acc[t][v];
                racc += d * d;
            }
        __syncthreads();
    }
    racc = wave_sum(racc);
    if (lane == 0) red[wave] = racc;
    __syncthreads();
    if (tid == 0) res_part[(int64_t)f * nb + blkx] = red[0] + red[1] + red[2] + red[3];
}

// Real faces: four wavefronts per SIMD (at most 128 registers).
template <int KP, bool VEC, typename T = float>
__global__ __launch_bounds__(GT) __attribute__((amdgpu_waves_per_eu(4))) void k_resid(
    const T *__restrict__ X, int m, int p, int nf, const T *__restrict__ U, const double *__restrict__ S,
    const T *__restrict__ V, int64_t kmax, const int32_t *__restrict__ ranks, double *__restrict__ res_part,
    const int32_t *__restrict__ fmap, int nsplit) {
    resid_body<KP, VEC, T, false>(X, m, p, nf, U, S, V, kmax, ranks, res_part, fmap, nsplit);
}

// Complex faces (2 ranks[f] real columns).  The same register cap: at width
// 64 it spills a few registers, and that costs less than the occupancy the
// uncapped kernel loses (measured 256 against 342 us on the 129 stored faces
// of the 512 x 512 x 256 DFT workload).
template <int KP, bool VEC>
__global__ __launch_bounds__(GT) __attribute__((amdgpu_waves_per_eu(4))) void k_resid_c(const float *__restrict__ X, int m, int p, int nf,
                                                const float *__restrict__ U, const double *__restrict__ S,
                                                const float *__restrict__ V, int64_t kmax,
                                                const int32_t *__restrict__ ranks, double *__restrict__ res_part) {
    resid_body<KP, VEC, float, true>(X, m, p, nf, U, S, V, kmax, ranks, res_part, nullptr, 1);
}

// cert[f] = sqrt of the ordered sum of face f's residual partials
__global__ void k_cert(const double *__restrict__ res_part, int nparts, int nf, double *__restrict__ cert,
                       const int32_t *__restrict__ fmap) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf || (fmap && fmap[f] < 0)) return;
    double r = 0.0;
    for (int i = 0; i < nparts; ++i) r += res_part[(int64_t)f * nparts + i];
    cert[fmap ? fmap[f] : f] = sqrt(r);
}

// ---------------------------------------------------------------- complex faces
// The mixed path on complex faces (the stored half spectrum of the DFT of a
// real tensor) runs its passes over X with the real GEMM kernels above.  A
// complex m x p face stored interleaved is the real 2m x p matrix X' whose
// rows 2i and 2i+1 hold the real and imaginary parts of row i; for a complex
// panel Q write Q' for the same view and (iQ)' for that of i Q.  Then
//   X' Omega                 = (X Omega)'                  (Omega real)
//   X'^T [Q' | (iQ)']        = [Re X^H Q | -Im X^H Q]
//   X' [Re Z | Im Z]         = P,  X Z = (P[2i, :l] - P[2i+1, l:]) + i (P[2i+1, :l] + P[2i, l:])
//   X'^T [Q' | (iQ)'] with the Gram partials and the residual of the
//   projection gives B^H = X^H Q in that layout, the Gram of its 2l real
//   columns and ||X' - [Q' | (iQ)'] [Re B^H | -Im B^H]^T||^2 = ||X - Q B||^2,
// so every pass reads X once, at twice the real width.  The per-face kernels
// below take and give panels in these layouts:
//   CIN_IL   S = (X Omega)' (2 rows x LP)
//   CIN_COMB S = P (2 rows x 2LP), combined as above
//   CIN_PC   S = [Re Z | -Im Z] (rows x 2LP)
//   COUT_RL  Q as [Q' | (iQ)'] (2 rows x 2LP), the operand of X'^T
//   COUT_PL  Q as [Re Q | Im Q] (rows x 2LP), the operand of X'
// Columns from ell to LP of each half are zero.
enum { CIN_IL = 0, CIN_COMB = 1, CIN_PC = 2 };
enum { COUT_RL = 0, COUT_PL = 1 };
constexpr int CQT = 512;

// Gram partials of a complex panel in one of the input layouts: rows
// blk*CGR .. +CGR-1 of face f as the real rows [Re y | Im y] (2LP wide; the
// combine of CIN_COMB and the sign of CIN_PC applied as they are staged),
// their 2LP x 2LP real Gram by FP64 MFMA 16x16x4 (products of FP32 values are
// exact), written as packed upper tiles (gram_tiles<2LP>) at
// gpart[(f * nblk + blk) * 4 LP^2].  With W = [Re Y | Im Y] the complex Gram
// is Y^H Y = W11 + W22 + i (W12 - W12^T).  Grid (ceil(rows/CGR), nf),
// GT threads; spreads the first Gram of every Cholesky-QR over several
// workgroups per face.
constexpr int CGR = 128;
template <int LP, int IN>
__global__ __launch_bounds__(GT) void k_cgram(const float *__restrict__ Sin, int rows, int ell,
                                              double *__restrict__ gpart) {
    constexpr int L2 = 2 * LP, LDS_ = L2 + 1, NT = L2 / 16, NTILE = NT * (NT + 1) / 2, TPW = (NTILE + 3) / 4;
    constexpr int PER = CGR * LP / GT;  // (row, column) pairs per thread
    __shared__ float st[CGR * LDS_];
    const int blk = blockIdx.x, f = blockIdx.y, nblk = gridDim.x, tid = threadIdx.x, wave = tid >> 6,
              lane = tid & 63;
    const int64_t R2 = 2 * (int64_t)rows;
    const float *S = Sin + (int64_t)f * (IN == CIN_IL ? R2 * LP : IN == CIN_COMB ? R2 * L2 : (int64_t)rows * L2);
    const int r0 = blk * CGR;
    float re[PER], im[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {  // pair e: row e % CGR, column e / CGR (consecutive rows per lane)
        const int e = tid + q * GT, r = e % CGR, c = e / CGR, row = r0 + r;
        const int rw = row < rows ? row : rows - 1;
        float a, b;
        if constexpr (IN == CIN_IL) {
            const float2 v = *reinterpret_cast<const float2 *>(S + 2 * (int64_t)rw + R2 * c);
            a = v.x;
            b = v.y;
        } else if constexpr (IN == CIN_COMB) {
            const float2 u = *reinterpret_cast<const float2 *>(S + 2 * (int64_t)rw + R2 * c);
            const float2 v = *reinterpret_cast<const float2 *>(S + 2 * (int64_t)rw + R2 * (LP + c));
            a = u.x - v.y;
            b = u.y + v.x;
        } else {
            a = S[rw + (int64_t)rows * c];
            b = -S[rw + (int64_t)rows * (LP + c)];
        }
        const bool ok = row < rows && c < ell;
        re[q] = ok ? a : 0.0f;
        im[q] = ok ? b : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = tid + q * GT, r = e % CGR, c = e / CGR;
        st[r * LDS_ + c] = re[q];
        st[r * LDS_ + LP + c] = im[q];
    }
    __syncthreads();
    f64x4 g[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) g[t] = f64x4{0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int idx = wave + 4 * t;
        if (idx >= NTILE) continue;
        int ti, tj;
        tile_ij<NT>(idx, ti, tj);
#pragma unroll 4
        for (int kk = 0; kk < CGR / 4; ++kk) {
            const int r = 4 * kk + (lane >> 4);
            g[t] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)st[r * LDS_ + 16 * ti + (lane & 15)],
                                                        (double)st[r * LDS_ + 16 * tj + (lane & 15)], g[t], 0, 0, 0);
        }
    }
    double *out = gpart + ((int64_t)f * nblk + blk) * L2 * L2;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int idx = wave + 4 * t;
        if (idx >= NTILE) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) out[idx * 256 + 64 * v + lane] = g[t][v];
    }
}

// Complex Cholesky-QR: G = Y^H Y (+ shift on the first pass) = R^H R, R upper
// triangular with a real positive diagonal, Q = Y R^{-1}; `passes` = 2 repeats
// the step on Q.  One workgroup per face, one row per thread in chunks of CQT
// rows.  The first Gram is the ordered sum of the nparts partials k_cgram
// wrote; the second pass's is formed here from the solved rows (staged in LDS
// as FP32 [Re | Im], FP64 MFMA over the 2LP x 2LP real Gram W^T W of
// W = [Re Y | Im Y]); both become Y^H Y = W11 + W22 + i (W12 - W12^T).  Shift, dropping rule and flag as in
// k_cholqr; the triangular solve is in FP64 in registers, in place in the
// row's own array (the row value of column c is needed only when q[c] is
// formed), the result stored as FP32 and its rounded rows are what the next
// pass's Gram sees.
template <int LP, int IN, int OUT>
__global__ __launch_bounds__(CQT) void k_cholqr_c(const float *__restrict__ Sin, int rows, int ell,
                                                  float *__restrict__ Qout, int passes,
                                                  int32_t *__restrict__ qr_info, int first,
                                                  const double *__restrict__ gpart, int nparts) {
    constexpr int L2 = 2 * LP, LDG = LP + 1, LDR = LP + 1, LDS_ = L2 + 1, HR = 128;
    constexpr int NW = CQT / 64, NT = L2 / 16, NH = LP / 16, NTILE = NT * (NT + 1) / 2;
    constexpr int TPW = (NTILE + NW - 1) / NW;
    __shared__ __align__(16) double2 G[LP * LDG];
    __shared__ __align__(16) double2 Rt[LP * LDR];  // Rt[c * LDR + j] = R[j][c]
    __shared__ double rinv[LP];
    __shared__ float st[HR * LDS_];
    __shared__ double trace_s;
    __shared__ int bad;
    const int f = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t R2 = 2 * (int64_t)rows;
    const float *S = Sin + (int64_t)f * (IN == CIN_IL ? R2 * LP : IN == CIN_COMB ? R2 * L2 : (int64_t)rows * L2);
    float *Q = Qout + (int64_t)f * (OUT == COUT_RL ? R2 * L2 : (int64_t)rows * L2);
    if (tid == 0) bad = 0;
    const int nch = (rows + CQT - 1) / CQT;
    double2 q[LP];  // the thread's row: input values, then the solved row
    // row `row` of the input panel, or (own) of this kernel's output
    // Eight columns at a time, their raw values all loaded before any is
    // converted (the fence keeps the conversions after the loads; converted as
    // loaded, each load waited for the last).  The input and this kernel's
    // output share a layout up to the sign of CIN_PC and the second operand
    // of CIN_COMB (loaded from the input and ignored for the own rows).
    static_assert((IN == CIN_PC) == (OUT == COUT_PL), "layouts");
    auto load_row = [&](int row, bool own) {
        const int rw = row < rows ? row : rows - 1;
        const float *base = own ? Q : S;
        constexpr int CB = 8;
        static_assert(LP % CB == 0, "column groups");
#pragma unroll
        for (int c0 = 0; c0 < LP; c0 += CB) {
            float2 u[CB], v[CB];
#pragma unroll
            for (int i = 0; i < CB; ++i) {
                const int c = c0 + i;
                if constexpr (IN == CIN_PC) {
                    u[i] = float2{base[rw + (int64_t)rows * c], base[rw + (int64_t)rows * (LP + c)]};
                } else {
                    u[i] = *reinterpret_cast<const float2 *>(base + 2 * (int64_t)rw + R2 * c);
                    if constexpr (IN == CIN_COMB)
                        v[i] = *reinterpret_cast<const float2 *>(S + 2 * (int64_t)rw + R2 * (LP + c));
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < CB; ++i) {
                const int c = c0 + i;
                float a = u[i].x, b = u[i].y;
                if constexpr (IN == CIN_PC) {
                    if (!own) b = -b;
                } else if constexpr (IN == CIN_COMB) {
                    if (!own) {
                        a = u[i].x - v[i].y;
                        b = u[i].y + v[i].x;
                    }
                }
                const bool ok = row < rows && c < ell;
                q[c] = double2{ok ? (double)a : 0.0, ok ? (double)b : 0.0};
            }
        }
    };
    // the rows of every thread through LDS into the 2LP x 2LP Gram tiles
    auto accumulate = [&](f64x4(&g)[TPW]) {
#pragma unroll
        for (int hh = 0; hh < CQT / HR; ++hh) {
            if (tid / HR == hh) {
                const int r = tid % HR;
#pragma unroll
                for (int c = 0; c < LP; ++c) {
                    st[r * LDS_ + c] = (float)q[c].x;
                    st[r * LDS_ + LP + c] = (float)q[c].y;
                }
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int idx = wave + NW * t;
                if (idx >= NTILE) continue;
                int ti, tj;
                tile_ij<NT>(idx, ti, tj);
#pragma unroll 4
                for (int kk = 0; kk < HR / 4; ++kk) {
                    const int r = 4 * kk + (lane >> 4);
                    g[t] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)st[r * LDS_ + 16 * ti + (lane & 15)],
                                                                (double)st[r * LDS_ + 16 * tj + (lane & 15)], g[t],
                                                                0, 0, 0);
                }
            }
            __syncthreads();
        }
    };
    // Gram tiles -> complex G: Re from W11 and W22, Im from W12 (set, then
    // its transpose subtracted); FP64 MFMA output row lane/16 + 4v
    auto to_complex = [&](const f64x4(&g)[TPW]) {
#pragma unroll
        for (int ph = 0; ph < 2; ++ph) {
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int idx = wave + NW * t;
                if (idx >= NTILE) continue;
                int ti, tj;
                tile_ij<NT>(idx, ti, tj);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 16 * ti + (lane >> 4) + 4 * v, j = 16 * tj + (lane & 15);
                    const double x = g[t][v];
                    if (tj < NH) {  // W11
                        if (ph == 0 && (ti < tj || i <= j)) {
                            G[i * LDG + j].x = x;
                            G[j * LDG + i].x = x;
                        }
                    } else if (ti >= NH) {  // W22
                        const int a = i - LP, b = j - LP;
                        if (ph == 1 && (ti < tj || a <= b)) {
                            G[a * LDG + b].x += x;
                            if (a != b) G[b * LDG + a].x += x;
                        }
                    } else {  // W12
                        if (ph == 0) G[i * LDG + (j - LP)].y = x;
                        else G[(j - LP) * LDG + i].y -= x;
                    }
                }
            }
            __syncthreads();
        }
    };

    // ---- first Gram: ordered sum of the partials, then W11 and W12 set and
    // W22 and -W12^T added (two phases, every entry has one writer in each)
    {
        constexpr int NE2 = NTILE * 128, E2 = (NE2 + CQT - 1) / CQT, PB = 4;
        const double2 *g2 = reinterpret_cast<const double2 *>(gpart + (int64_t)f * nparts * L2 * L2);
        double2 acc[E2];
#pragma unroll
        for (int u = 0; u < E2; ++u) acc[u] = double2{0.0, 0.0};
        for (int p0 = 0; p0 < nparts; p0 += PB) {
            double2 v[E2][PB];
#pragma unroll
            for (int u = 0; u < E2; ++u)
#pragma unroll
                for (int b = 0; b < PB; ++b) {
                    const int e2 = tid + u * CQT, pp = p0 + b;
                    const bool in = e2 < NE2 && pp < nparts;
                    const double2 t = g2[(int64_t)(pp < nparts ? pp : nparts - 1) * (L2 * L2 / 2) + (e2 < NE2 ? e2 : 0)];
                    v[u][b] = in ? t : double2{0.0, 0.0};
                }
#pragma unroll
            for (int u = 0; u < E2; ++u)
#pragma unroll
                for (int b = 0; b < PB; ++b) {
                    acc[u].x += v[u][b].x;
                    acc[u].y += v[u][b].y;
                }
        }
#pragma unroll
        for (int ph = 0; ph < 2; ++ph) {
#pragma unroll
            for (int u = 0; u < E2; ++u) {
                const int e2 = tid + u * CQT;
                if (e2 >= NE2) continue;
                const int t = (2 * e2) >> 8, r = ((2 * e2) >> 4) & 15, c = (2 * e2) & 15;
                int ti, tj;
                tile_ij<NT>(t, ti, tj);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int i = 16 * ti + r, j = 16 * tj + c + h;
                    const double x = h ? acc[u].y : acc[u].x;
                    if (tj < NH) {  // W11 (the tile holds both triangles of a diagonal tile)
                        if (ph == 0) {
                            G[i * LDG + j].x = x;
                            if (ti != tj) G[j * LDG + i].x = x;
                        }
                    } else if (ti >= NH) {  // W22
                        if (ph == 1) {
                            G[(i - LP) * LDG + (j - LP)].x += x;
                            if (ti != tj) G[(j - LP) * LDG + (i - LP)].x += x;
                        }
                    } else {  // W12
                        if (ph == 0) G[i * LDG + (j - LP)].y = x;
                        else G[(j - LP) * LDG + i].y -= x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int pass = 0; pass < passes; ++pass) {
        if (wave == 0) {
            double t = 0.0;
            for (int c = lane; c < ell; c += 64) t += G[c * LDG + c].x;
            t = wave_sum(t);
            if (lane == 0) trace_s = t;
        }
        __syncthreads();
        const double level = 11.0 * ((double)rows * ell + (double)ell * (ell + 1)) * 0x1p-53 * trace_s;
        const double pfloor = pass == 0 ? 0.0 : level;
        if (pass == 0) {
            if (tid < ell) G[tid * LDG + tid].x += level;
            __syncthreads();
        }
        // ---- right-looking Cholesky, upper entries numbered by decreasing row
        // (see k_cholqr): G[i][c] -= conj(G[j][i]) G[j][c] / G[j][j]
        {
            constexpr int NU = LP * (LP + 1) / 2, UPT = (NU + CQT - 1) / CQT;
            int ei[UPT], ec[UPT];
#pragma unroll
            for (int u = 0; u < UPT; ++u) {
                int rem = tid + u * CQT, i = ell - 1;
                while (i >= 0 && rem >= ell - i) {
                    rem -= ell - i;
                    --i;
                }
                ei[u] = i;
                ec[u] = i >= 0 ? i + rem : 0;
            }
            for (int j = 0; j < ell; ++j) {
                const int cnt = (ell - j - 1) * (ell - j) / 2;
                const double piv = G[j * LDG + j].x;
                const double ipv = piv > pfloor && isfinite(piv) ? recip(piv) : 0.0;
#pragma unroll
                for (int u = 0; u < UPT; ++u) {
                    if (u * CQT + (tid & ~63) >= cnt) break;
                    const bool act = tid + u * CQT < cnt;
                    const int i = act ? ei[u] : j, c = act ? ec[u] : j;
                    const double2 gji = G[j * LDG + i], gjc = G[j * LDG + c], gic = G[i * LDG + c];
                    const double2 l = cmulc(gji, gjc);
                    if (act) G[i * LDG + c] = double2{gic.x - l.x * ipv, gic.y - l.y * ipv};
                }
                __syncthreads();
            }
            for (int e = tid; e < ell * ell; e += CQT) {
                const int j = e / ell, c = e % ell;
                if (c < j) continue;
                const double piv = G[j * LDG + j].x;
                const bool fin = isfinite(piv), ok = fin && piv > pfloor, drop = fin && !ok && pass > 0;
                const double d = ok ? sqrt(piv) : 1.0, id = 1.0 / d;
                const double2 gjc = G[j * LDG + c];
                Rt[c * LDR + j] = c == j ? double2{d, 0.0} : ok ? double2{gjc.x * id, gjc.y * id} : double2{0.0, 0.0};
                if (c == j) {
                    rinv[j] = drop ? 0.0 : id;
                    if (!ok && !drop) bad = 1;
                }
            }
            __syncthreads();
        }
        // ---- Q = Y R^{-1} row by row: q[c] = (y[c] - sum_{j<c} q[j] R[j][c]) / R[c][c]
        const bool again = pass + 1 < passes;
        f64x4 g[TPW];
#pragma unroll
        for (int t = 0; t < TPW; ++t) g[t] = f64x4{0, 0, 0, 0};
        for (int ch = 0; ch < nch; ++ch) {
            const int row = ch * CQT + tid;
            load_row(row, pass > 0);
#pragma unroll
            for (int c = 0; c < LP; ++c) {
                if (c < ell) {
                    double2 v0 = q[c], v1{0.0, 0.0};
                    const double2 *rc = Rt + c * LDR;
#pragma unroll
                    for (int j = 0; j + 1 < c; j += 2) {
                        const double2 r0 = rc[j], r1 = rc[j + 1];
                        const double2 p0 = cmul(q[j], r0), p1 = cmul(q[j + 1], r1);
                        v0.x -= p0.x;
                        v0.y -= p0.y;
                        v1.x -= p1.x;
                        v1.y -= p1.y;
                    }
                    if (c & 1) {
                        const double2 p0 = cmul(q[c - 1], rc[c - 1]);
                        v0.x -= p0.x;
                        v0.y -= p0.y;
                    }
                    const double ri = rinv[c];
                    q[c] = double2{(v0.x + v1.x) * ri, (v0.y + v1.y) * ri};
                } else {
                    q[c] = double2{0.0, 0.0};
                }
            }
            if (row < rows) {
#pragma unroll
                for (int c = 0; c < LP; ++c) {
                    const float a = (float)q[c].x, b = (float)q[c].y;
                    if constexpr (OUT == COUT_RL) {
                        *reinterpret_cast<float2 *>(Q + 2 * (int64_t)row + R2 * c) = float2{a, b};
                        *reinterpret_cast<float2 *>(Q + 2 * (int64_t)row + R2 * (LP + c)) = float2{-b, a};
                    } else {
                        Q[row + (int64_t)rows * c] = a;
                        Q[row + (int64_t)rows * (LP + c)] = b;
                    }
                }
            }
            if (again) accumulate(g);
        }
        if (again) to_complex(g);
    }
    if (tid == 0) {
        if (first) qr_info[f] = bad ? 2 : 0;
        else if (bad) qr_info[f] = 2;
    }
}

// Complex core: H = B B^H = (B^H)^H B^H, formed from the Gram partials of the
// projection's [Re B^H | -Im B^H] (width 2LP, staged in the eigenvector
// buffers): H = W11 + W22 + i (W21 - W12); its eigenpairs by the Hermitian
// Jacobi solver; sorting, rank rule, certificate and outputs as k_core (U_B
// complex, column j at UB[f][j], LP entries).
template <int LP>
__global__ __launch_bounds__(QT) void k_core_c(const double *__restrict__ gpart, int nparts, int ell,
                                               const double *__restrict__ fro_part, int nfro,
                                               const double *__restrict__ res_part, int nres, int mode, int kfix,
                                               double tau, int max_sweeps, double jtol, double2 *__restrict__ UB,
                                               double *__restrict__ sig, int *__restrict__ perm_out,
                                               int *__restrict__ kf_out, double *__restrict__ fro2_out,
                                               double *__restrict__ cert, int32_t *__restrict__ jinfo) {
    constexpr int L2 = 2 * LP, LD = jacobi_ldc<LP>(), NPM = LP / 2, LDW = L2 + 1;
    __shared__ __align__(16) double2 Gb[2][LP * LD];
    __shared__ __align__(16) double2 Eb[2][LP * LD];
    __shared__ double2 cs[2][NPM], ph[2][NPM];
    __shared__ double lam[LP];
    __shared__ int perm[LP];
    __shared__ double trace_s;
    __shared__ int rflag[3];
    static_assert(L2 * LDW * sizeof(double) <= sizeof(Eb), "the real Gram fits in the eigenvector buffers");
    const int f = blockIdx.x, tid = threadIdx.x;
    double *W = reinterpret_cast<double *>(&Eb[0][0]);
    load_gram_partials<L2, QT>(gpart, f, nparts, W, LDW);
    __syncthreads();
    for (int e = tid; e < LP * LD; e += QT) {
        const int a = e / LD, b = e % LD;
        double2 v{0.0, 0.0};
        if (b < LP) {
            v.x = W[a * LDW + b] + W[(LP + a) * LDW + LP + b];
            v.y = a == b ? 0.0 : W[(LP + a) * LDW + b] - W[a * LDW + LP + b];
        }
        Gb[0][e] = v;
    }
    __syncthreads();
    for (int e = tid; e < LP * LD; e += QT) Eb[0][e] = Eb[1][e] = double2{0.0, 0.0};
    __syncthreads();
    if (tid < ell) Eb[0][tid * LD + tid] = double2{1.0, 0.0};
    if (tid < 3) rflag[tid] = 0;
    if (tid < 64) {
        double t = 0.0;
        for (int c = tid; c < ell; c += 64) t += Gb[0][c * LD + c].x;
        t = wave_sum(t);
        if (tid == 0) trace_s = t;
    }
    __syncthreads();
    const double trace = trace_s;
    int conv = 0, dslot;
    const double2 *G, *E;
    jacobi_eig_c<LP, QT>(Gb[0], Gb[1], Eb[0], Eb[1], &cs[0][0], &ph[0][0], rflag, ell, jtol * trace, max_sweeps,
                         conv, G, E, dslot);
    if (tid < ell) {
        const int sl = jacobi_slot(tid, dslot);
        lam[tid] = fmax(G[sl * LD + sl].x, 0.0);
    }
    __syncthreads();
    if (tid < ell) {
        int pos = 0;
        double li = lam[tid];
        for (int j = 0; j < ell; ++j) pos += (lam[j] > li) || (lam[j] == li && j < tid);
        perm[pos] = tid;
    }
    __syncthreads();
    if (tid == 0) {
        double fro2 = 0.0, res = 0.0;
        for (int i = 0; i < nfro; ++i) fro2 += fro_part[(int64_t)f * nfro + i];
        for (int i = 0; i < nres; ++i) res += res_part[(int64_t)f * nres + i];
        int kf, miss = 0;
        if (mode == TSVDM_RANK_FIXED) {
            kf = kfix < ell ? kfix : ell;
        } else {
            const int cap = kfix > 0 && kfix < ell ? kfix : ell;
            double tail = res, bound = tau * tau * fro2;
            for (int j = 0; j < ell; ++j) tail += lam[j];
            kf = -1;
            for (int k = 0; k <= cap; ++k) {
                if (tail <= bound) {
                    kf = k;
                    break;
                }
                if (k < ell) tail -= lam[perm[k]];
            }
            if (kf < 0) {
                kf = cap;
                miss = 1;
            }
        }
        double disc = 0.0;
        for (int j = ell - 1; j >= kf; --j) disc += lam[perm[j]];
        kf_out[f] = kf;
        fro2_out[f] = fro2;
        if (cert) cert[f] = nres != 0 ? sqrt(res + disc) : -1.0;
        jinfo[f] = ((conv || ell <= 1) ? 0 : 1) | (miss ? 4 : 0);
    }
    for (int r = tid; r < LP; r += QT) {
        int j = r < ell ? perm[r] : r;
        sig[(int64_t)f * LP + r] = r < ell ? sqrt(lam[j]) : 0.0;
        perm_out[(int64_t)f * LP + r] = j;
    }
    for (int e = tid; e < LP * LP; e += QT)
        UB[(int64_t)f * LP * LP + e] =
            e / LP < ell ? E[jacobi_slot(e / LP, dslot) * LD + e % LP] : double2{0.0, 0.0};
}

// Complex factors: Uhat = Q U_B[:, perm], Vhat = B^H U_B[:, perm] / s, from
// the layouts above by FP32 MFMA 16x16x4 (the structure of k_factors):
//   Uhat' = [Q' | (iQ)'] [Re U_B; Im U_B]                    (rows 2m)
//   Re Vhat = [Re B^H | -Im B^H] [Re U_B; Im U_B] / s,
//   Im Vhat = [Re B^H | -Im B^H] [Im U_B; -Re U_B] / s       (rows p)
// Output columns r of Uhat; for Vhat, output column 2r + b is part b of
// complex column r, stored interleaved.  Uo, Vo: C64 factors, face stride
// m kmax and p kmax complex values.  Grid (ceil(2m/64) + ceil(p/64), nf).
template <int LP>
__global__ __launch_bounds__(GT) void k_factors_c(const float *__restrict__ Qr, const float *__restrict__ Btr, int m,
                                                  int p, int ell, int64_t kmax, const double2 *__restrict__ UB,
                                                  const double *__restrict__ sig, const int *__restrict__ perm,
                                                  const int *__restrict__ kf_in, const double *__restrict__ fro2,
                                                  const int32_t *__restrict__ qr_info,
                                                  const int32_t *__restrict__ jinfo, float *__restrict__ Uo,
                                                  double *__restrict__ So, float *__restrict__ Vo,
                                                  int32_t *__restrict__ ranks, double *__restrict__ fro,
                                                  int32_t *__restrict__ info) {
    constexpr int L2 = 2 * LP, LU = L2 + 1, NT = L2 / 16;
    __shared__ float ubs[L2 * LU];
    const int f = blockIdx.y, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int kf = kf_in[f], m2 = 2 * m, nbu = (m2 + 63) / 64;
    const bool isv = (int)blockIdx.x >= nbu;
    const int blk = isv ? blockIdx.x - nbu : blockIdx.x, rows = isv ? p : m2;
    const float *S = isv ? Btr + (int64_t)f * p * L2 : Qr + (int64_t)f * m2 * L2;
    const int kc = kf < kmax ? kf : (int)kmax;
    for (int e = tid; e < L2 * L2; e += GT) {
        const int r = e / L2, c = e % L2, cc = c < LP ? c : c - LP, rk = isv ? r >> 1 : r;
        float u = 0.0f;
        if (rk < kc && cc < ell) {
            const double2 v = UB[(int64_t)f * LP * LP + cc + (int64_t)LP * perm[(int64_t)f * LP + rk]];
            if (!isv) {
                u = (float)(c < LP ? v.x : v.y);
            } else {
                const double sv = sig[(int64_t)f * LP + rk], is = sv > 0.0 ? 1.0 / sv : 0.0;
                const double val = (r & 1) == 0 ? (c < LP ? v.x : v.y) : (c < LP ? v.y : -v.x);
                u = (float)(val * is);
            }
        }
        ubs[r * LU + c] = u;
    }
    __syncthreads();
    const int ncol = isv ? 2 * kc : kc, nt = (ncol + 15) / 16;
    const int row0 = blk * 64 + 16 * wave, jr = row0 + (lane & 15), kl = lane >> 4;
    const bool rok = jr < rows;
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < L2 / 4; ++kk) {
        if ((4 * kk) % LP >= ell) continue;  // zero columns of both halves
        const float x = S[rok ? jr + (int64_t)rows * (4 * kk + kl) : 0];
        const float bq = rok ? x : 0.0f;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t >= nt) break;
            const float a = ubs[(16 * t + (lane & 15)) * LU + 4 * kk + kl];
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bq, acc[t], 0, 0, 0);
        }
    }
    float *Uf = Uo + (int64_t)f * m2 * kmax;
    float *Vf = Vo + (int64_t)f * 2 * p * kmax;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (t >= nt) break;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int e = 16 * t + 4 * kl + v;
            if (!rok) continue;
            if (!isv) {
                if (e < kmax) Uf[jr + (int64_t)m2 * e] = acc[t][v];
            } else if ((e >> 1) < kmax) {
                Vf[2 * (int64_t)jr + (e & 1) + 2 * (int64_t)p * (e >> 1)] = acc[t][v];
            }
        }
    }
    // zero the columns past the computed tiles
    const int done = isv ? 8 * nt : 16 * nt;
    const int64_t zc = kmax - done;
    for (int64_t e = tid; e < 64 * zc; e += GT) {
        const int row = blk * 64 + (int)(e % 64);
        const int64_t col = done + e / 64;
        if (row >= rows) continue;
        if (!isv) Uf[row + (int64_t)m2 * col] = 0.0f;
        else *reinterpret_cast<float2 *>(Vf + 2 * (int64_t)row + 2 * (int64_t)p * col) = float2{0.0f, 0.0f};
    }
    if (blockIdx.x == 0) {
        for (int r = tid; r < kmax; r += GT) So[(int64_t)f * kmax + r] = r < kf ? sig[(int64_t)f * LP + r] : 0.0;
        if (tid == 0) {
            ranks[f] = kf;
            if (fro) fro[f] = sqrt(fro2[f]);
            if (info) {
                int code = (jinfo[f] & 4) ? 4 : 0;
                if (jinfo[f] & 1) code = 1;
                if (qr_info[f]) code = 2;
                if (!isfinite(fro2[f])) code = 3;
                info[f] = code;
            }
        }
    }
}

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct MixedWs {
    float *Y, *Qm, *Z, *Qp;
    double *gram_m, *gram_p, *fro_part, *res_part, *cert_part, *UB, *sig, *fro2;
    int *perm, *kf;
    int32_t *qr_info, *jinfo;
};

// Column ranges of the certificate pass per face (resid_body): more than one
// only when the faces' 64-row blocks alone would leave most of the 256 CUs
// idle (a few wide faces); then about 512 workgroups in all.
inline int resid_splits(int64_t nf, int64_t mparts, int64_t p) {
    const int64_t chunks = (p + 63) / 64, blocks = nf * mparts;
    if (blocks >= 256 || blocks < 1) return 1;
    int64_t sp = (512 + blocks - 1) / blocks;
    if (sp > kResidSplitMax) sp = kResidSplitMax;
    if (sp > chunks) sp = chunks;
    return sp < 1 ? 1 : (int)sp;
}

// Column ranges of the X W passes (k_xw, ksplit) for the same reason, with
// the partial products kept in the face's Z panel (p x LP, idle during those
// passes), so at most p / m of them; from the whole tensor's face count, so
// that face groups give the same bits.
inline int xw_splits(int64_t nf, int64_t mparts, int64_t m, int64_t p) {
    int64_t sp = resid_splits(nf, mparts, p);
    const int64_t cap = m > 0 ? p / m : 1;
    if (sp > cap) sp = cap;
    return sp < 1 ? 1 : (int)sp;
}

// esz: bytes per element of the panels Y, Q, Z, Qz (4 mixed, 8 FP64 randomized);
// gm_parts: Gram partials per face in gram_m (-1: one per 64 rows of X, the
// passes' partials; the complex path keeps the k_cgram partials there)
size_t carve(char *base, int64_t m, int64_t p, int64_t nf, int LP, MixedWs *w, int esz = 4, int64_t gm_parts = -1) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *ptr = base ? base + off : nullptr;
        off += al256(bytes);
        return ptr;
    };
    const int64_t mparts = (m + 63) / 64, pparts = (p + 63) / 64;
    MixedWs t;
    t.Y = (float *)take((size_t)esz * nf * m * LP);
    t.Qm = (float *)take((size_t)esz * nf * m * LP);
    t.Z = (float *)take((size_t)esz * nf * p * LP);
    t.Qp = (float *)take((size_t)esz * nf * p * LP);
    t.gram_m = (double *)take(sizeof(double) * nf * (gm_parts < 0 ? mparts : gm_parts) * LP * LP);
    t.gram_p = (double *)take(sizeof(double) * nf * pparts * LP * LP);
    t.fro_part = (double *)take(sizeof(double) * nf * mparts);
    t.res_part = (double *)take(sizeof(double) * nf * pparts);
    t.cert_part = (double *)take(sizeof(double) * nf * mparts * kResidSplitMax);
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

// ---------------------------------------------------------------- learned rank
// features[f][j] = log10(s_j / s_1) (0 when s_1 = 0, at least -30) of the
// singular values s (decreasing, LP per face) of the face's sketch, as halves
__global__ void k_rank_features(const double *__restrict__ sig, int LPs, int nf,
                                _Float16 *__restrict__ feat) {
    const int f = blockIdx.x, j = threadIdx.x;
    if (f >= nf || j >= 32) return;
    const double s1 = sig[(int64_t)f * LPs], sj = sig[(int64_t)f * LPs + j];
    double v = 0.0;
    if (s1 > 0.0) v = sj > 0.0 ? log10(sj / s1) : -30.0;
    feat[(int64_t)f * 32 + j] = (_Float16)fmax(v, -30.0);
}

// Widths of the learned truncation from the predictor's (k/32, l/48): the
// predicted rank kh = ceil(32 k/32) (1..32) and width lw = ceil(48 l/48) + 1;
// a face takes the first bucket (width 16, 32, 40 with rank caps 13, 26, 32)
// whose width is at least lw and whose cap is at least kh, and the energy
// rule's cap min(bucket cap, kh + 2).  Stable partition of the faces into the
// three lists (lists[b * nf + i], unused slots -1), counts[b]; widths[f] and
// caps[f] record each face's choice.  One workgroup.
__global__ __launch_bounds__(1024) void k_width_partition(const float *__restrict__ y, int nf,
                                                          int32_t *__restrict__ lists,
                                                          int32_t *__restrict__ counts,
                                                          int32_t *__restrict__ widths,
                                                          int32_t *__restrict__ caps) {
    __shared__ int base[3];
    __shared__ int wsum[3][16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < 3) base[tid] = 0;
    __syncthreads();
    for (int f0 = 0; f0 < nf; f0 += 1024) {
        const int f = f0 + tid;
        int b = -1;
        if (f < nf) {
            // NaN or out-of-range predictions end in a valid bucket (the
            // certificate's fallback catches a wrong choice)
            const float kr = ceilf(y[2 * f] * 32.0f), lr = ceilf(y[2 * f + 1] * 48.0f) + 1.0f;
            const int kh = kr >= 1.0f && kr <= 32.0f ? (int)kr : kr > 32.0f ? 32 : 1;
            const int lw = lr >= 1.0f && lr <= 48.0f ? (int)lr : lr > 48.0f ? 48 : 1;
            b = lw <= 16 && kh <= 13 ? 0 : lw <= 32 && kh <= 26 ? 1 : 2;
            const int bc = b == 0 ? 13 : b == 1 ? 26 : 32;
            widths[f] = b == 0 ? 16 : b == 1 ? 32 : 40;
            caps[f] = kh + 2 < bc ? kh + 2 : bc;
        }
        for (int c = 0; c < 3; ++c) {
            const unsigned long long mask = __ballot(b == c);
            const int before = __popcll(mask & ((1ull << lane) - 1ull));
            if (lane == 0) wsum[c][wave] = __popcll(mask);
            __syncthreads();
            int off = base[c];
            for (int w = 0; w < wave; ++w) off += wsum[c][w];
            if (b == c) lists[c * nf + off + before] = f;
            __syncthreads();
            if (tid == 0) {
                int t = 0;
                for (int w = 0; w < 16; ++w) t += wsum[c][w];
                base[c] += t;
            }
            __syncthreads();
        }
    }
    for (int c = 0; c < 3; ++c)
        for (int i = base[c] + tid; i < nf; i += 1024) lists[c * nf + i] = -1;
    if (tid < 3) counts[tid] = base[tid];
}

// Stable list of the faces whose certified error exceeds tau ||Xhat_f|| and
// that did not already run at the full width with the full cap: they are
// truncated again with width 40 and cap 32.  Unused slots -1.
__global__ __launch_bounds__(1024) void k_fallback_list(const double *__restrict__ cert,
                                                        const double *__restrict__ fro, double tau, int nf,
                                                        int32_t *__restrict__ widths,
                                                        const int32_t *__restrict__ caps,
                                                        int32_t *__restrict__ list, int32_t *__restrict__ count) {
    __shared__ int base;
    __shared__ int wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) base = 0;
    __syncthreads();
    for (int f0 = 0; f0 < nf; f0 += 1024) {
        const int f = f0 + tid;
        const bool bad = f < nf && (widths[f] < 40 || caps[f] < 32) && !(cert[f] <= tau * fro[f]);
        const unsigned long long mask = __ballot(bad);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wave] = __popcll(mask);
        __syncthreads();
        int off = base;
        for (int w = 0; w < wave; ++w) off += wsum[w];
        if (bad) {
            list[off + before] = f;
            widths[f] = 40;
        }
        __syncthreads();
        if (tid == 0) {
            int t = 0;
            for (int w = 0; w < 16; ++w) t += wsum[w];
            base += t;
        }
        __syncthreads();
    }
    for (int i = base + tid; i < nf; i += 1024) list[i] = -1;
    if (tid == 0) *count = base;
}

// Faces [f0, f0 + nfg) through the whole path on stream s.  Every kernel
// below works face by face, so the pointers are offset to the first face of
// the range and the kernels see a tensor of nfg faces.

// The GEMM passes' 16-byte loads of four consecutive rows at 32-bit offsets
// from the face: m and p multiples of 4 (every face start of X, and every
// row block of a W with leading dimension m or p, is then as aligned as its
// base), X 16-byte aligned, a face below 4 GiB.  The workspace panels are
// 256-byte aligned; Omega is checked where it is used.
bool vec_loads_ok(const float *X, int m, int p) {
    return m % 4 == 0 && p % 4 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0 &&
           (int64_t)m * p < (int64_t)1 << 30;
}
// Three streams and four events per device, created on first use and kept
// until the process ends: the three width buckets of a learned truncation run
// concurrently (their FP64 steps are latency-bound, one workgroup per face).
// Default priority.  Learned truncations issued from several host threads at
// once on one device share them and must be serialized by the caller.
struct SideStreams {
    hipStream_t s[3];
    hipEvent_t ev[4];
};
std::mutex g_side_mu;
SideStreams *g_side[64];

tsvdm_status side_streams(SideStreams **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_check(e, "side streams: device");
    if (dev < 0 || dev >= 64) {
        set_error("side streams: device index %d beyond 64", dev);
        return TSVDM_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_side_mu);
    if (!g_side[dev]) {
        SideStreams t{};
        for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&t.s[i], hipStreamNonBlocking);
        for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&t.ev[i], hipEventDisableTiming);
        if (e != hipSuccess) return hip_check(e, "side streams: create");
        g_side[dev] = new SideStreams(t);
    }
    *out = g_side[dev];
    return TSVDM_OK;
}

// wf0: the face of the workspace w0 the group starts at (f0 when w0 was carved
// for the whole tensor, 0 when it was carved for the group alone).
// fmap: the group's faces (entries < 0: unused slots of a list sized on the
// device; every kernel's workgroups for them exit at once).  src: a sketch
// X Omega[:, :32] with its width-32 Gram partials, taken once for all faces
// (indexed by face); a group of width 16 or 32 then starts from its first
// columns instead of a sketch pass.  kcap_face: per-face energy-rule caps.
// mark: recorded on s once the group's first pass over X (the sketch) has been
// enqueued (the start of a second group on another stream).
template <int LP>
tsvdm_status run_group(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, tsvdm_factors *F,
                       const MixedWs &w0, int f0, int nfg, hipStream_t s,
                       const int32_t *fmap = nullptr, int wf0 = -1, const MixedWs *src = nullptr,
                       const int32_t *kcap_face = nullptr, hipEvent_t mark = nullptr) {
    const int m = (int)X->m, p = (int)X->p, ell = o->k + o->oversample;
    const int mparts = (m + 63) / 64, pparts = (p + 63) / 64;
    const int64_t kmax = F->kmax;
    MixedWs w = w0;
    const int64_t g0 = wf0 < 0 ? f0 : wf0;
    w.Y += g0 * m * LP;
    w.Qm += g0 * m * LP;
    w.Z += g0 * p * LP;
    w.Qp += g0 * p * LP;
    w.gram_m += g0 * mparts * LP * LP;
    w.gram_p += g0 * pparts * LP * LP;
    w.fro_part += g0 * mparts;
    w.res_part += g0 * pparts;
    w.cert_part += g0 * mparts * kResidSplitMax;
    w.UB += g0 * LP * LP;
    w.sig += g0 * LP;
    w.fro2 += g0;
    w.perm += g0 * LP;
    w.kf += g0;
    w.qr_info += g0;
    w.jinfo += g0;
    const float *Xd = reinterpret_cast<const float *>(X->data) + (int64_t)f0 * m * p;
    float *Uo = reinterpret_cast<float *>(F->U) + (int64_t)f0 * m * kmax;
    float *Vo = reinterpret_cast<float *>(F->V) + (int64_t)f0 * p * kmax;
    double *So = F->S + (int64_t)f0 * kmax;
    int32_t *ranks = F->ranks + f0;
    double *cert = F->cert ? F->cert + f0 : nullptr;
    double *fro = F->fro ? F->fro + f0 : nullptr;
    int32_t *info = F->info ? F->info + f0 : nullptr;
    const int nf = nfg;
    const dim3 gm(xcd_grid(mparts, nf)), gp(xcd_grid(pparts, nf));
    const bool power = o->power_iters > 0;
    // the energy rule needs the sketch residual ||X - Q B||^2 before the rank
    // is chosen (an estimate of the error, computed with the projection); the
    // certificate is the error of the returned factors, computed after them
    const bool resid = o->rank_mode == TSVDM_RANK_ENERGY;
    const bool exact = o->certify && cert;
    const bool v4 = vec_loads_ok(Xd, m, p) && reinterpret_cast<uintptr_t>(w.Y) % 16 == 0;
    const double *gm_c = w.gram_m, *gp_c = w.gram_p;
    // the X W passes of a few wide faces: xsp column ranges per 64-row block,
    // partial products in Z and the partial ||X||^2 in cert_part (both idle
    // then), summed by k_ysum
    const int xsp = xw_splits(X->n3, mparts, m, p);
    const dim3 gx(xcd_grid(mparts * xsp, nf));
    float *xyp = xsp > 1 ? w.Z : nullptr;
    double *xfp = xsp > 1 ? w.cert_part : nullptr;
#define TSVDM_YSUM(NAME, FRO)                                                                               \
    do {                                                                                                    \
        if (xsp > 1)                                                                                        \
            TSVDM_LAUNCH(NAME, (k_ysum<LP>), gm, dim3(GT), 0, s, (const float *)w.Z, m, p, nf, xsp, w.Y,      \
                         w.gram_m, (const double *)w.cert_part, FRO, fmap);                                 \
    } while (0)
#define TSVDM_SKETCH()                                                                                      \
    do {                                                                                                    \
        if (v4 && reinterpret_cast<uintptr_t>(o->omega) % 16 == 0)                                          \
            TSVDM_LAUNCH("sketch_xw_bf16", (k_xw<LP, PROD_BF16, true, true>), gx, dim3(GT), 0, s, Xd, m, p, nf, \
                         o->omega, (int64_t)0, p, ell, w.Y, w.fro_part, w.gram_m, fmap, xsp, xyp, xfp);      \
        else                                                                                                \
            TSVDM_LAUNCH("sketch_xw_bf16", (k_xw<LP, PROD_BF16, true, false>), gx, dim3(GT), 0, s, Xd, m, p,    \
                         nf, o->omega, (int64_t)0, p, ell, w.Y, w.fro_part, w.gram_m, fmap, xsp, xyp, xfp);  \
        TSVDM_YSUM("sketch_reduce", w.fro_part);                                                            \
    } while (0)
#define TSVDM_MARK()                                                                                        \
    do {                                                                                                    \
        if (mark) {                                                                                         \
            hipError_t e_ = hipEventRecord(mark, s);                                                        \
            if (e_ != hipSuccess) return hip_check(e_, "mixed truncate: group mark");                       \
        }                                                                                                   \
    } while (0)
    const bool reuse = power && src && LP <= 32 && ell <= 32;
    if (power) {
        if (reuse) {
            // the sketch's first ell columns were taken once for all faces
            TSVDM_LAUNCH("cholqr_sketch", (k_cholqr<LP>), dim3(nf, cholqr_row_groups(m, nf)), dim3(QT), 0, s,
                         (const float *)src->Y, m, ell, w.Qm, 1, (const double *)src->gram_m, mparts, w.qr_info, 1,
                         fmap, 1, 32);
            TSVDM_MARK();
        } else {
            // pass 1: sketch Y = X Omega (BF16), ||X||^2, Gram partials of Y
            TSVDM_SKETCH();
            TSVDM_MARK();
            // basis of the sketch: one shifted Cholesky-QR step (its span is what
            // the power step needs)
            TSVDM_LAUNCH("cholqr_sketch", (k_cholqr<LP>), dim3(nf, cholqr_row_groups(m, nf)), dim3(QT), 0, s,
                         (const float *)w.Y, m, ell, w.Qm, 1, gm_c, mparts, w.qr_info, 1, fmap);
        }
        // pass 2: Z = X^T Q (BF16) and its Gram partials; basis of Z
        if (v4)
            TSVDM_LAUNCH("power_xtw_bf16", (k_xtw<LP, PROD_BF16, true, false, true>), gp, dim3(GT), 0, s, Xd, m,
                         p, nf, (const float *)w.Qm, (int64_t)m * LP, m, ell, w.Z, w.gram_p, (double *)nullptr, fmap);
        else
            TSVDM_LAUNCH("power_xtw_bf16", (k_xtw<LP, PROD_BF16, true, false, false>), gp, dim3(GT), 0, s, Xd, m,
                         p, nf, (const float *)w.Qm, (int64_t)m * LP, m, ell, w.Z, w.gram_p, (double *)nullptr, fmap);
        // many partials and rows spread over workgroups: group sums first
        const unsigned zrg = cholqr_row_groups(p, nf);
        const int zgp = zrg > 1 && pparts > 64 ? 32 : 1;
        if (zgp > 1)
            TSVDM_LAUNCH("gram_group_z", (k_gram_group<LP>), dim3(gram_group_blocks<LP>(pparts, zgp), nf), dim3(256),
                         0, s, w.gram_p, pparts, zgp, fmap);
        TSVDM_LAUNCH("cholqr_power_z", (k_cholqr<LP>), dim3(nf, zrg), dim3(QT), 0, s, (const float *)w.Z, p, ell,
                     w.Qp, 1, gp_c, pparts, w.qr_info, 0, fmap, 0, LP, zgp);
        // pass 3: Y' = X Qz, FP32-accurate (split BF16), and its Gram partials
        // (and ||X||^2 when the sketch pass was skipped)
        double *fp3 = reuse ? w.fro_part : (double *)nullptr;
        if (v4)
            TSVDM_LAUNCH("power_xw_split", (k_xw<LP, PROD_SPLIT, true, true>), gx, dim3(GT), 0, s, Xd, m, p, nf,
                         (const float *)w.Qp, (int64_t)p * LP, p, ell, w.Y, fp3, w.gram_m, fmap, xsp, xyp, xfp);
        else
            TSVDM_LAUNCH("power_xw_split", (k_xw<LP, PROD_SPLIT, true, false>), gx, dim3(GT), 0, s, Xd, m, p, nf,
                         (const float *)w.Qp, (int64_t)p * LP, p, ell, w.Y, fp3, w.gram_m, fmap, xsp, xyp, xfp);
        TSVDM_YSUM("power_xw_reduce", fp3);
    } else {
        TSVDM_SKETCH();
        TSVDM_MARK();
    }
#undef TSVDM_MARK
#undef TSVDM_SKETCH
#undef TSVDM_YSUM
    // final basis: FP64 shifted Cholesky-QR2 (first Gram from the partials)
    TSVDM_LAUNCH("cholqr_final", (k_cholqr<LP>), dim3(nf), dim3(QT), 0, s, (const float *)w.Y, m, ell, w.Qm,
                 2, gm_c, mparts, w.qr_info, power ? 0 : 1, fmap);
    // pass 4: B^T = X^T Q, FP32-accurate, the Gram partials of B^T and, for
    // the energy rule, ||X - Q B||^2 per 64-column block
#define TSVDM_PROJECT(NAME, RES, V, RP)                                                                    \
    TSVDM_LAUNCH(NAME, (k_xtw<LP, PROD_SPLIT, true, RES, V>), gp, dim3(GT), 0, s, Xd, m, p, nf,             \
                 (const float *)w.Qm, (int64_t)m * LP, m, ell, w.Z, w.gram_p, RP, fmap)
    if (resid) {
        if (v4) TSVDM_PROJECT("project_resid_split", true, true, w.res_part);
        else TSVDM_PROJECT("project_resid_split", true, false, w.res_part);
    } else {
        if (v4) TSVDM_PROJECT("project_xtw_split", false, true, (double *)nullptr);
        else TSVDM_PROJECT("project_xtw_split", false, false, (double *)nullptr);
    }
#undef TSVDM_PROJECT
    const int msw = o->max_sweeps > 0 ? o->max_sweeps : 30;
    // a face of many column blocks: group sums of its Gram partials first
    const int cgp = pparts > 64 ? 32 : 1;
    if (cgp > 1)
        TSVDM_LAUNCH("gram_group_b", (k_gram_group<LP>), dim3(gram_group_blocks<LP>(pparts, cgp), nf), dim3(256), 0,
                     s, w.gram_p, pparts, cgp, fmap);
    TSVDM_LAUNCH("core_gram_eig", (k_core<LP>), dim3(nf), dim3(QT), 0, s, gp_c, pparts, ell,
                 (const double *)w.fro_part, mparts, (const double *)w.res_part, resid ? pparts : 0,
                 o->rank_mode, o->k, o->tau, msw, kJacobiTolMixed, w.UB, w.sig, w.perm, w.kf, w.fro2,
                 exact ? (double *)nullptr : cert, w.jinfo, fmap, kcap_face, cgp);
    TSVDM_LAUNCH("factors", (k_factors<LP>), dim3((unsigned)(mparts + pparts), nf), dim3(GT), 0, s,
                 (const float *)w.Qm, (const float *)w.Z, m, p, ell, kmax, w.UB, w.sig, w.perm, w.kf,
                 w.fro2, w.qr_info, w.jinfo, Uo, So, Vo, ranks, fro, info, fmap);
    if (exact) {
        // the certificate: ||Xhat_f - Uhat_f S_f Vhat_f^T||_F of the stored factors
        // ranks are at most min(kmax, ell): the W staging is sized for that
        const int kcap = (int)(kmax < ell ? kmax : ell);
        const bool xv = m % 4 == 0 && reinterpret_cast<uintptr_t>(Xd) % 16 == 0;
        // from the whole tensor's face count, so that face groups (the
        // allocation-free entry point, the learned buckets) sum every face's
        // partials in the same order as one call on all faces
        const int nsp = resid_splits(X->n3, mparts, p);
        const dim3 gr(xcd_grid(mparts * nsp, nf));
#define TSVDM_RESID(KP)                                                                                        \
    do {                                                                                                      \
        if (xv)                                                                                               \
            TSVDM_LAUNCH("resid_factors", (k_resid<KP, true>), gr, dim3(GT), 0, s, Xd, m, p, nf,              \
                         (const float *)Uo, (const double *)So, (const float *)Vo, kmax, (const int32_t *)ranks, \
                         w.cert_part, fmap, nsp);                                                             \
        else                                                                                                  \
            TSVDM_LAUNCH("resid_factors", (k_resid<KP, false>), gr, dim3(GT), 0, s, Xd, m, p, nf,             \
                         (const float *)Uo, (const double *)So, (const float *)Vo, kmax, (const int32_t *)ranks, \
                         w.cert_part, fmap, nsp);                                                             \
    } while (0)
        if (kcap <= 16) TSVDM_RESID(16);
        else if (kcap <= 32) TSVDM_RESID(32);
        else if (kcap <= 48) TSVDM_RESID(48);
        else TSVDM_RESID(64);
#undef TSVDM_RESID
        TSVDM_LAUNCH("cert", k_cert, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s,
                     (const double *)w.cert_part, mparts * nsp, nf, cert, fmap);
    }
    TSVDM_LAUNCH_CHECK("mixed truncate");
    return TSVDM_OK;
}

bool side_streams_created(SideStreams **out);

// Whether a randomized truncation runs its faces in two groups (below): at
// least 32 faces and 128 MiB of face data.  The second group starts one
// sketch pass late, and the split pays only when the passes over X it hides
// under the other group's per-face FP64 kernels are long: 256 faces of 512^2
// FP32 (256 MiB) ran 4-5% faster in two groups, 64 such faces 2% slower and
// 127 faces of 64^2 6% slower.
inline bool split_pays(int64_t nf, int64_t bytes) { return nf >= 32 && bytes >= ((int64_t)128 << 20); }

// Two face groups, as for complex faces (run_cplx): the second half of the
// faces runs on a side stream, started once the first half's sketch pass has
// finished, so that each group's latency-bound per-face FP64 kernels (one
// workgroup per face) run beside the other group's passes over X; the
// caller's stream then waits for the side stream.  One group unless
// split_pays, or when s is being captured and the side streams do not exist
// yet.  The workspace is carved for the whole tensor and every group uses its
// faces' part of it; the results do not depend on the grouping.
template <int LP>
tsvdm_status run_mixed(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, tsvdm_factors *F,
                       void *wsp, hipStream_t s) {
    MixedWs w;
    carve(reinterpret_cast<char *>(wsp), X->m, X->p, X->n3, LP, &w);
    const int nf = (int)X->n3;
    SideStreams *ss = nullptr;
    bool split = split_pays(nf, 4 * X->m * X->p * X->n3);
    if (split) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        hipError_t e = hipStreamIsCapturing(s, &cs);
        if (e != hipSuccess) return hip_check(e, "mixed truncate: capture status");
        split = cs == hipStreamCaptureStatusNone ? side_streams(&ss) == TSVDM_OK : side_streams_created(&ss);
    }
    if (!split) return run_group<LP>(X, o, F, w, 0, nf, s);
    const int g0 = (nf + 1) / 2;
    tsvdm_status st = run_group<LP>(X, o, F, w, 0, g0, s, nullptr, -1, nullptr, nullptr, ss->ev[2]);
    if (st != TSVDM_OK) return st;
    hipStream_t sb = ss->s[0];
    hipError_t e = hipStreamWaitEvent(sb, ss->ev[2], 0);
    if (e != hipSuccess) return hip_check(e, "mixed truncate: fork");
    if ((st = run_group<LP>(X, o, F, w, g0, nf - g0, sb)) != TSVDM_OK) return st;
    if ((e = hipEventRecord(ss->ev[3], sb)) != hipSuccess) return hip_check(e, "mixed truncate: join");
    if ((e = hipStreamWaitEvent(s, ss->ev[3], 0)) != hipSuccess) return hip_check(e, "mixed truncate: join");
    return TSVDM_OK;
}

// ---------------------------------------------------------------- complex faces
// PREC_MIXED on complex faces (C64 Xhat, C64 factors): the steps of run_group
// with the layouts of the complex kernels above, for faces [f0, f0 + nfg) of
// the workspace w0 carved for the whole tensor (every kernel works face by
// face, so the pointers are offset to the group's first face; each panel by
// its per-face stride in the carve, which is at least what every kernel
// writes per face).  LP: the padded complex width; the passes run at 2LP real
// columns over the 2m x p real view of each face.  mark: recorded on s after
// the group's sketch pass (or null).
template <int LP>
tsvdm_status run_cplx_group(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, tsvdm_factors *F,
                            const MixedWs &w0, int f0, int nfg, hipStream_t s, hipEvent_t mark) {
    constexpr int L2 = 2 * LP;
    const int m = (int)X->m, p = (int)X->p, nf = nfg, ell = o->k + o->oversample, m2 = 2 * m;
    const int mparts = (m2 + 63) / 64, pparts = (p + 63) / 64;
    const int64_t kmax = F->kmax;
    const int cg = (std::max(m, p) + CGR - 1) / CGR;  // Gram partials per face
    MixedWs w = w0;
    const int64_t g0 = f0;
    w.Y += g0 * m2 * L2;
    w.Qm += g0 * m2 * L2;
    w.Z += g0 * p * L2;
    w.Qp += g0 * p * L2;
    w.gram_m += g0 * cg * L2 * L2;
    w.gram_p += g0 * pparts * L2 * L2;
    w.fro_part += g0 * mparts;
    w.res_part += g0 * pparts;
    w.cert_part += g0 * mparts * kResidSplitMax;
    w.UB += g0 * L2 * L2;
    w.sig += g0 * L2;
    w.fro2 += g0;
    w.perm += g0 * L2;
    w.kf += g0;
    w.qr_info += g0;
    w.jinfo += g0;
    const float *Xd = reinterpret_cast<const float *>(X->data) + g0 * m2 * p;
    float *Uo = reinterpret_cast<float *>(F->U) + g0 * m2 * kmax;
    float *Vo = reinterpret_cast<float *>(F->V) + g0 * 2 * p * kmax;
    double *So = F->S + g0 * kmax;
    int32_t *ranks = F->ranks + g0;
    double *cert = F->cert ? F->cert + g0 : nullptr;
    double *fro = F->fro ? F->fro + g0 : nullptr;
    int32_t *info = F->info ? F->info + g0 : nullptr;
    const dim3 gm(xcd_grid(mparts, nf)), gp(xcd_grid(pparts, nf));
    const bool power = o->power_iters > 0;
    const bool resid = o->rank_mode == TSVDM_RANK_ENERGY;
    const bool exact = o->certify && cert;
    const bool v4 = vec_loads_ok(Xd, m2, p);
    // pass 1: (X Omega)' (BF16) and ||X||^2
    if (v4 && reinterpret_cast<uintptr_t>(o->omega) % 16 == 0)
        TSVDM_LAUNCH("c_sketch_xw_bf16", (k_xw<LP, PROD_BF16, false, true>), gm, dim3(GT), 0, s, Xd, m2, p, nf,
                     o->omega, (int64_t)0, p, ell, w.Y, w.fro_part, (double *)nullptr, (const int32_t *)nullptr);
    else
        TSVDM_LAUNCH("c_sketch_xw_bf16", (k_xw<LP, PROD_BF16, false, false>), gm, dim3(GT), 0, s, Xd, m2, p, nf,
                     o->omega, (int64_t)0, p, ell, w.Y, w.fro_part, (double *)nullptr, (const int32_t *)nullptr);
    if (mark) {
        hipError_t e = hipEventRecord(mark, s);
        if (e != hipSuccess) return hip_check(e, "complex truncate: mark");
    }
    if (power) {
        TSVDM_LAUNCH("c_gram_sketch", (k_cgram<LP, CIN_IL>), dim3((m + CGR - 1) / CGR, nf), dim3(GT), 0, s,
                     (const float *)w.Y, m, ell, w.gram_m);
        TSVDM_LAUNCH("c_cholqr_sketch", (k_cholqr_c<LP, CIN_IL, COUT_RL>), dim3(nf), dim3(CQT), 0, s,
                     (const float *)w.Y, m, ell, w.Qm, 1, w.qr_info, 1, (const double *)w.gram_m,
                     (m + CGR - 1) / CGR);
        // pass 2: [Re Z | -Im Z] = X'^T [Q' | (iQ)'] (BF16), Z = X^H Q
        if (v4)
            TSVDM_LAUNCH("c_power_xtw_bf16", (k_xtw<L2, PROD_BF16, false, false, true>), gp, dim3(GT), 0, s, Xd,
                         m2, p, nf, (const float *)w.Qm, (int64_t)m2 * L2, m2, L2, w.Z, (double *)nullptr,
                         (double *)nullptr, (const int32_t *)nullptr);
        else
            TSVDM_LAUNCH("c_power_xtw_bf16", (k_xtw<L2, PROD_BF16, false, false, false>), gp, dim3(GT), 0, s, Xd,
                         m2, p, nf, (const float *)w.Qm, (int64_t)m2 * L2, m2, L2, w.Z, (double *)nullptr,
                         (double *)nullptr, (const int32_t *)nullptr);
        TSVDM_LAUNCH("c_gram_power_z", (k_cgram<LP, CIN_PC>), dim3((p + CGR - 1) / CGR, nf), dim3(GT), 0, s,
                     (const float *)w.Z, p, ell, w.gram_m);
        TSVDM_LAUNCH("c_cholqr_power_z", (k_cholqr_c<LP, CIN_PC, COUT_PL>), dim3(nf), dim3(CQT), 0, s,
                     (const float *)w.Z, p, ell, w.Qp, 1, w.qr_info, 0, (const double *)w.gram_m,
                     (p + CGR - 1) / CGR);
        // pass 3: P = X' [Re Qz | Im Qz] (split BF16); X Qz is combined from P
        if (v4)
            TSVDM_LAUNCH("c_power_xw_split", (k_xw<L2, PROD_SPLIT, false, true>), gm, dim3(GT), 0, s, Xd, m2, p,
                         nf, (const float *)w.Qp, (int64_t)p * L2, p, L2, w.Y, (double *)nullptr, (double *)nullptr,
                         (const int32_t *)nullptr);
        else
            TSVDM_LAUNCH("c_power_xw_split", (k_xw<L2, PROD_SPLIT, false, false>), gm, dim3(GT), 0, s, Xd, m2, p,
                         nf, (const float *)w.Qp, (int64_t)p * L2, p, L2, w.Y, (double *)nullptr, (double *)nullptr,
                         (const int32_t *)nullptr);
        TSVDM_LAUNCH("c_gram_final", (k_cgram<LP, CIN_COMB>), dim3((m + CGR - 1) / CGR, nf), dim3(GT), 0, s,
                     (const float *)w.Y, m, ell, w.gram_m);
        TSVDM_LAUNCH("c_cholqr_final", (k_cholqr_c<LP, CIN_COMB, COUT_RL>), dim3(nf), dim3(CQT), 0, s,
                     (const float *)w.Y, m, ell, w.Qm, 2, w.qr_info, 0, (const double *)w.gram_m,
                     (m + CGR - 1) / CGR);
    } else {
        TSVDM_LAUNCH("c_gram_final", (k_cgram<LP, CIN_IL>), dim3((m + CGR - 1) / CGR, nf), dim3(GT), 0, s,
                     (const float *)w.Y, m, ell, w.gram_m);
        TSVDM_LAUNCH("c_cholqr_final", (k_cholqr_c<LP, CIN_IL, COUT_RL>), dim3(nf), dim3(CQT), 0, s,
                     (const float *)w.Y, m, ell, w.Qm, 2, w.qr_info, 1, (const double *)w.gram_m,
                     (m + CGR - 1) / CGR);
    }
    // pass 4: [Re B^H | -Im B^H] = X'^T [Q' | (iQ)'] (split BF16), its Gram
    // partials and, for the energy rule, ||X - Q B||^2 per 64-column block
#define TSVDM_CPROJECT(NAME, RES, V, RP)                                                                   \
    TSVDM_LAUNCH(NAME, (k_xtw<L2, PROD_SPLIT, true, RES, V>), gp, dim3(GT), 0, s, Xd, m2, p, nf,            \
                 (const float *)w.Qm, (int64_t)m2 * L2, m2, L2, w.Z, w.gram_p, RP, (const int32_t *)nullptr)
    if (resid) {
        if (v4) TSVDM_CPROJECT("c_project_resid_split", true, true, w.res_part);
        else TSVDM_CPROJECT("c_project_resid_split", true, false, w.res_part);
    } else {
        if (v4) TSVDM_CPROJECT("c_project_xtw_split", false, true, (double *)nullptr);
        else TSVDM_CPROJECT("c_project_xtw_split", false, false, (double *)nullptr);
    }
#undef TSVDM_CPROJECT
    const int msw = o->max_sweeps > 0 ? o->max_sweeps : 30;
    double2 *UB = reinterpret_cast<double2 *>(w.UB);
    TSVDM_LAUNCH("c_core_gram_eig", (k_core_c<LP>), dim3(nf), dim3(QT), 0, s, (const double *)w.gram_p, pparts,
                 ell, (const double *)w.fro_part, mparts, (const double *)w.res_part, resid ? pparts : 0,
                 o->rank_mode, o->k, o->tau, msw, kJacobiTolMixed, UB, w.sig, w.perm, w.kf, w.fro2,
                 exact ? (double *)nullptr : cert, w.jinfo);
    TSVDM_LAUNCH("c_factors", (k_factors_c<LP>), dim3((unsigned)((m2 + 63) / 64 + pparts), nf), dim3(GT), 0, s,
                 (const float *)w.Qm, (const float *)w.Z, m, p, ell, kmax, (const double2 *)UB, (const double *)w.sig,
                 (const int *)w.perm, (const int *)w.kf, (const double *)w.fro2, (const int32_t *)w.qr_info,
                 (const int32_t *)w.jinfo, Uo, So, Vo, ranks, fro, info);
    if (exact) {
        // the certificate of the stored complex factors: 2 ranks[f] real columns
        const int kcap = (int)(kmax < ell ? kmax : ell);
        const bool xv = m2 % 4 == 0 && reinterpret_cast<uintptr_t>(Xd) % 16 == 0;
#define TSVDM_CRESID(KP)                                                                                       \
    do {                                                                                                      \
        if (xv)                                                                                               \
            TSVDM_LAUNCH("c_resid_factors", (k_resid_c<KP, true>), gm, dim3(GT), 0, s, Xd, m2, p, nf,         \
                         (const float *)Uo, (const double *)So, (const float *)Vo, kmax,                      \
                         (const int32_t *)ranks, w.cert_part);                                                \
        else                                                                                                  \
            TSVDM_LAUNCH("c_resid_factors", (k_resid_c<KP, false>), gm, dim3(GT), 0, s, Xd, m2, p, nf,        \
                         (const float *)Uo, (const double *)So, (const float *)Vo, kmax,                      \
                         (const int32_t *)ranks, w.cert_part);                                                \
    } while (0)
        if (kcap <= 16) TSVDM_CRESID(32);
        else if (kcap <= 32) TSVDM_CRESID(64);
        else TSVDM_CRESID(96);
#undef TSVDM_CRESID
        TSVDM_LAUNCH("c_cert", k_cert, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s,
                     (const double *)w.cert_part, mparts, nf, cert, (const int32_t *)nullptr);
    }
    TSVDM_LAUNCH_CHECK("mixed truncate (complex)");
    return TSVDM_OK;
}

// The side streams of this device if they already exist (none are created:
// the caller may be capturing a graph).
bool side_streams_created(SideStreams **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
    std::lock_guard<std::mutex> lk(g_side_mu);
    *out = g_side[dev];
    return *out != nullptr;
}

// Two face groups: with one workgroup per face, the per-face FP64 kernels of
// a group leave most CUs idle, so the second group runs on a side stream,
// started once the first group's sketch pass has finished, and its passes
// over X fill those CUs (and the other way round); the caller's stream then
// waits for it.  One group unless split_pays, or when the side streams do not
// exist yet and s is being captured (creating them would break the capture).
// The results do not depend on the grouping: every kernel works face by face.
template <int LP>
tsvdm_status run_cplx(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, tsvdm_factors *F, void *wsp,
                      hipStream_t s) {
    const int m = (int)X->m, p = (int)X->p, nf = (int)X->n3;
    MixedWs w;
    carve(reinterpret_cast<char *>(wsp), 2 * m, p, nf, 2 * LP, &w, 4, (std::max(m, p) + CGR - 1) / CGR);
    SideStreams *ss = nullptr;
    bool split = split_pays(nf, 8 * X->m * X->p * X->n3);
    if (split) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        hipError_t e = hipStreamIsCapturing(s, &cs);
        if (e != hipSuccess) return hip_check(e, "complex truncate: capture status");
        split = cs == hipStreamCaptureStatusNone ? side_streams(&ss) == TSVDM_OK : side_streams_created(&ss);
    }
    if (!split) return run_cplx_group<LP>(X, o, F, w, 0, nf, s, nullptr);
    const int g0 = (nf + 1) / 2;
    tsvdm_status st = run_cplx_group<LP>(X, o, F, w, 0, g0, s, ss->ev[0]);
    if (st != TSVDM_OK) return st;
    hipStream_t sb = ss->s[0];
    hipError_t e = hipStreamWaitEvent(sb, ss->ev[0], 0);
    if (e != hipSuccess) return hip_check(e, "complex truncate: fork");
    if ((st = run_cplx_group<LP>(X, o, F, w, g0, nf - g0, sb, nullptr)) != TSVDM_OK) return st;
    if ((e = hipEventRecord(ss->ev[1], sb)) != hipSuccess) return hip_check(e, "complex truncate: join");
    if ((e = hipStreamWaitEvent(s, ss->ev[1], 0)) != hipSuccess) return hip_check(e, "complex truncate: join");
    return TSVDM_OK;
}

// ---------------------------------------------------------------- FP64 randomized
// PREC_F64_RAND: the randomized range finder of the mixed path with every
// product in FP64 (FP64 MFMA) on an FP64 Xhat: Y = X Omega, Q = qr(Y),
// Z = X^T Q, Qz = qr(Z), Y = X Qz, Q = qr(Y) (each shifted Cholesky-QR2),
// B^T = X^T Q, core eigensolver of B B^T, factors, and the certificate of the
// stored factors as in the mixed path (or, without certify, the estimate
// sqrt(||X||^2 - sum_{j<=k} lambda_j)).
constexpr double kJacobiTolF64 = 1e-15;
// The faces f0 .. f0+nfg-1 (the workspace w0 carved for the whole tensor);
// mark as in run_group.
template <int LP>
tsvdm_status run_f64rand_group(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, tsvdm_factors *F,
                               const MixedWs &w0, int f0, int nfg, hipStream_t s, hipEvent_t mark) {
    const int m = (int)X->m, p = (int)X->p, nf = nfg, ell = o->k + o->oversample;
    const int mparts = (m + 63) / 64, pparts = (p + 63) / 64;
    const int64_t kmax = F->kmax, g0 = f0;
    MixedWs w = w0;
    double *Y = reinterpret_cast<double *>(w.Y) + g0 * m * LP, *Qm = reinterpret_cast<double *>(w.Qm) + g0 * m * LP;
    double *Z = reinterpret_cast<double *>(w.Z) + g0 * p * LP, *Qp = reinterpret_cast<double *>(w.Qp) + g0 * p * LP;
    w.gram_m += g0 * mparts * LP * LP;
    w.gram_p += g0 * pparts * LP * LP;
    w.fro_part += g0 * mparts;
    w.cert_part += g0 * mparts * kResidSplitMax;
    w.UB += g0 * LP * LP;
    w.sig += g0 * LP;
    w.fro2 += g0;
    w.perm += g0 * LP;
    w.kf += g0;
    w.qr_info += g0;
    w.jinfo += g0;
    const double *Xd = reinterpret_cast<const double *>(X->data) + g0 * m * p;
    double *Uo = reinterpret_cast<double *>(F->U) + g0 * m * kmax, *Vo = reinterpret_cast<double *>(F->V) + g0 * p * kmax;
    double *So = F->S + g0 * kmax;
    int32_t *ranks = F->ranks + g0;
    double *cert = F->cert ? F->cert + g0 : nullptr;
    double *fro = F->fro ? F->fro + g0 : nullptr;
    int32_t *info = F->info ? F->info + g0 : nullptr;
    const dim3 gm(xcd_grid(mparts, nf)), gp(xcd_grid(pparts, nf));
    const bool power = o->power_iters > 0;
    const bool exact = o->certify && cert;
    TSVDM_LAUNCH("f64_sketch_xw", (k_xw64<LP, float, true>), gm, dim3(GT), 0, s, Xd, m, p, nf, o->omega,
                 (int64_t)0, p, ell, Y, w.fro_part, w.gram_m);
    if (mark) {
        hipError_t e = hipEventRecord(mark, s);
        if (e != hipSuccess) return hip_check(e, "FP64 randomized truncate: group mark");
    }
    if (power) {
        // both intermediate bases are made orthonormal (two passes): a single
        // shifted pass leaves columns of norm ~sqrt(shift) along directions
        // below the shift, and on FP64 data (no FP32 rounding floor) two such
        // steps in a row push the final sketch's condition number past 1/u
        TSVDM_LAUNCH("f64_cholqr_sketch", (k_cholqr<LP, double>), dim3(nf), dim3(QT), 0, s, (const double *)Y, m,
                     ell, Qm, 2, (const double *)w.gram_m, mparts, w.qr_info, 1);
        TSVDM_LAUNCH("f64_power_xtw", (k_xtw64<LP, true>), gp, dim3(GT), 0, s, Xd, m, p, nf, (const double *)Qm,
                     (int64_t)m * LP, m, ell, Z, w.gram_p);
        TSVDM_LAUNCH("f64_cholqr_power_z", (k_cholqr<LP, double>), dim3(nf), dim3(QT), 0, s, (const double *)Z,
                     p, ell, Qp, 2, (const double *)w.gram_p, pparts, w.qr_info, 0);
        TSVDM_LAUNCH("f64_power_xw", (k_xw64<LP, double, true>), gm, dim3(GT), 0, s, Xd, m, p, nf,
                     (const double *)Qp, (int64_t)p * LP, p, ell, Y, (double *)nullptr, w.gram_m);
    }
    TSVDM_LAUNCH("f64_cholqr_final", (k_cholqr<LP, double>), dim3(nf), dim3(QT), 0, s, (const double *)Y, m, ell,
                 Qm, 2, (const double *)w.gram_m, mparts, w.qr_info, power ? 0 : 1);
    TSVDM_LAUNCH("f64_project_xtw", (k_xtw64<LP, true>), gp, dim3(GT), 0, s, Xd, m, p, nf, (const double *)Qm,
                 (int64_t)m * LP, m, ell, Z, w.gram_p);
    const int msw = o->max_sweeps > 0 ? o->max_sweeps : 30;
    TSVDM_LAUNCH("f64_core_gram_eig", (k_core<LP>), dim3(nf), dim3(QT), 0, s, (const double *)w.gram_p, pparts,
                 ell, (const double *)w.fro_part, mparts, (const double *)nullptr, -1, o->rank_mode, o->k, o->tau,
                 msw, kJacobiTolF64, w.UB, w.sig, w.perm, w.kf, w.fro2, exact ? (double *)nullptr : cert,
                 w.jinfo, (const int32_t *)nullptr);
    TSVDM_LAUNCH("f64_factors", (k_factors<LP, double>), dim3((unsigned)(mparts + pparts), nf), dim3(GT), 0, s,
                 (const double *)Qm, (const double *)Z, m, p, ell, kmax, w.UB, w.sig, w.perm, w.kf, w.fro2,
                 w.qr_info, w.jinfo, Uo, So, Vo, ranks, fro, info, (const int32_t *)nullptr);
    if (exact) {
        const int kcap = (int)(kmax < ell ? kmax : ell);
        const bool xv = m % 4 == 0 && reinterpret_cast<uintptr_t>(Xd) % 16 == 0;
#define TSVDM_RESID64(KP)                                                                                       \
    do {                                                                                                        \
        if (xv)                                                                                                 \
            TSVDM_LAUNCH("f64_resid_factors", (k_resid<KP, true, double>), gm, dim3(GT), 0, s, Xd, m, p, nf,    \
                         (const double *)Uo, (const double *)So, (const double *)Vo, kmax,                      \
                         (const int32_t *)ranks, w.cert_part, (const int32_t *)nullptr, 1);                    \
        else                                                                                                    \
            TSVDM_LAUNCH("f64_resid_factors", (k_resid<KP, false, double>), gm, dim3(GT), 0, s, Xd, m, p, nf,   \
                         (const double *)Uo, (const double *)So, (const double *)Vo, kmax,                      \
                         (const int32_t *)ranks, w.cert_part, (const int32_t *)nullptr, 1);                    \
    } while (0)
        if (kcap <= 16) TSVDM_RESID64(16);
        else if (kcap <= 32) TSVDM_RESID64(32);
        else if (kcap <= 48) TSVDM_RESID64(48);
        else TSVDM_RESID64(64);
#undef TSVDM_RESID64
        TSVDM_LAUNCH("f64_cert", k_cert, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s,
                     (const double *)w.cert_part, mparts, nf, cert, (const int32_t *)nullptr);
    }
    TSVDM_LAUNCH_CHECK("FP64 randomized truncate");
    return TSVDM_OK;
}

// Two face groups on two streams, as in run_mixed (the same conditions).
template <int LP>
tsvdm_status run_f64rand(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, tsvdm_factors *F, void *wsp,
                         hipStream_t s) {
    MixedWs w;
    carve(reinterpret_cast<char *>(wsp), X->m, X->p, X->n3, LP, &w, 8);
    const int nf = (int)X->n3;
    SideStreams *ss = nullptr;
    bool split = split_pays(nf, 8 * X->m * X->p * X->n3);
    if (split) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        hipError_t e = hipStreamIsCapturing(s, &cs);
        if (e != hipSuccess) return hip_check(e, "FP64 randomized truncate: capture status");
        split = cs == hipStreamCaptureStatusNone ? side_streams(&ss) == TSVDM_OK : side_streams_created(&ss);
    }
    if (!split) return run_f64rand_group<LP>(X, o, F, w, 0, nf, s, nullptr);
    const int g0 = (nf + 1) / 2;
    tsvdm_status st = run_f64rand_group<LP>(X, o, F, w, 0, g0, s, ss->ev[2]);
    if (st != TSVDM_OK) return st;
    hipStream_t sb = ss->s[0];
    hipError_t e = hipStreamWaitEvent(sb, ss->ev[2], 0);
    if (e != hipSuccess) return hip_check(e, "FP64 randomized truncate: fork");
    if ((st = run_f64rand_group<LP>(X, o, F, w, g0, nf - g0, sb, nullptr)) != TSVDM_OK) return st;
    if ((e = hipEventRecord(ss->ev[3], sb)) != hipSuccess) return hip_check(e, "FP64 randomized truncate: join");
    if ((e = hipStreamWaitEvent(s, ss->ev[3], 0)) != hipSuccess) return hip_check(e, "FP64 randomized truncate: join");
    return TSVDM_OK;
}

// ---------------------------------------------------------------- no allocation
// Scratch of tsvdm_truncate_noalloc: one copy per GPU (each device holds its
// own instance of this array at its own address), kept until the process
// ends.  Host code never uses the name `scratch` as an address: it is a
// host-side stand-in; the device address comes from hipGetSymbolAddress.
constexpr size_t kNoallocScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

// Device address of the current device's scratch array (looked up once per device).
tsvdm_status noalloc_scratch(void **ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_check(e, "noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("noalloc: device %d beyond the %d devices the scratch table holds", dev, kMaxDevices);
        return TSVDM_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_check(e, "noalloc: hipGetSymbolAddress(scratch)");
        if (!p) {
            set_error("noalloc: no device address for the scratch array");
            return TSVDM_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return TSVDM_OK;
}

// The faces in groups whose workspace fits the scratch array, one run_group
// each, with the workspace carved for the group alone.
template <int LP>
tsvdm_status run_mixed_noalloc(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, tsvdm_factors *F,
                               hipStream_t s) {
    const int64_t m = X->m, p = X->p, nf = X->n3;
    const size_t one = carve(nullptr, m, p, 1, LP, nullptr);
    if (one > kNoallocScratchBytes) {
        set_error("noalloc: one %lld x %lld face needs %zu bytes of scratch, the static scratch holds %zu",
                  (long long)m, (long long)p, one, kNoallocScratchBytes);
        return TSVDM_EWORKSPACE;
    }
    int64_t g = (int64_t)(kNoallocScratchBytes / one);
    if (g > nf) g = nf;
    while (g > 1 && carve(nullptr, m, p, g, LP, nullptr) > kNoallocScratchBytes) --g;
    void *base = nullptr;
    tsvdm_status st = noalloc_scratch(&base);
    if (st != TSVDM_OK) return st;
    for (int64_t f0 = 0; f0 < nf; f0 += g) {
        const int64_t n = nf - f0 < g ? nf - f0 : g;
        MixedWs w;
        carve(reinterpret_cast<char *>(base), m, p, n, LP, &w);
        st = run_group<LP>(X, o, F, w, (int)f0, (int)n, s, nullptr, 0);
        if (st != TSVDM_OK) return st;
    }
    return TSVDM_OK;
}

}  // namespace

namespace tsvdm {

static int padded(int ell) { return ell <= 16 ? 16 : ell <= 32 ? 32 : ell <= 48 ? 48 : 64; }

size_t mixed_workspace(int64_t m, int64_t p, int64_t nf, int ell, bool cplx) {
    if (cplx) return carve(nullptr, 2 * m, p, nf, 2 * padded(ell), nullptr, 4, (std::max(m, p) + CGR - 1) / CGR);
    return carve(nullptr, m, p, nf, padded(ell), nullptr);
}

tsvdm_status launch_mixed_truncate(const tsvdm_tensor *X, const tsvdm_truncate_opts *o,
                                   tsvdm_factors *F, void *ws, hipStream_t s) {
    if (X->m > 65536 || X->p > 65536 || X->n3 > 65535) {
        set_error("PREC_MIXED: face dims up to 65536 and up to 65535 faces");
        return TSVDM_EUNSUPPORTED;
    }
    if (X->dtype == TSVDM_C64) {
        if (X->m > 32768) {
            set_error("PREC_MIXED on complex faces: m up to 32768");
            return TSVDM_EUNSUPPORTED;
        }
        switch (padded(o->k + o->oversample)) {
            case 16: return run_cplx<16>(X, o, F, ws, s);
            case 32: return run_cplx<32>(X, o, F, ws, s);
            default: return run_cplx<48>(X, o, F, ws, s);
        }
    }
    switch (padded(o->k + o->oversample)) {
        case 16: return run_mixed<16>(X, o, F, ws, s);
        case 32: return run_mixed<32>(X, o, F, ws, s);
        case 48: return run_mixed<48>(X, o, F, ws, s);
        default: return run_mixed<64>(X, o, F, ws, s);
    }
}

size_t f64rand_workspace(int64_t m, int64_t p, int64_t nf, int ell) {
    return carve(nullptr, m, p, nf, padded(ell), nullptr, 8);
}

tsvdm_status launch_f64rand_truncate(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, tsvdm_factors *F,
                                     void *ws, hipStream_t s) {
    if (X->m > 65536 || X->p > 65536 || X->n3 > 65535) {
        set_error("PREC_F64_RAND: face dims up to 65536 and up to 65535 faces");
        return TSVDM_EUNSUPPORTED;
    }
    switch (padded(o->k + o->oversample)) {
        case 16: return run_f64rand<16>(X, o, F, ws, s);
        case 32: return run_f64rand<32>(X, o, F, ws, s);
        case 48: return run_f64rand<48>(X, o, F, ws, s);
        default: return run_f64rand<64>(X, o, F, ws, s);
    }
}

tsvdm_status launch_mixed_truncate_noalloc(const tsvdm_tensor *X, const tsvdm_truncate_opts *o,
                                           tsvdm_factors *F, hipStream_t s) {
    if (X->m > 65536 || X->p > 65536 || X->n3 > 65535) {
        set_error("PREC_MIXED: face dims up to 65536 and up to 65535 faces");
        return TSVDM_EUNSUPPORTED;
    }
    switch (padded(o->k + o->oversample)) {
        case 16: return run_mixed_noalloc<16>(X, o, F, s);
        case 32: return run_mixed_noalloc<32>(X, o, F, s);
        case 48: return run_mixed_noalloc<48>(X, o, F, s);
        default: return run_mixed_noalloc<64>(X, o, F, s);
    }
}

size_t noalloc_scratch_bytes() { return kNoallocScratchBytes; }

// ---------------------------------------------------------------- learned rank
// Features: sketch Y = Xhat_f Omega[:, :32] (BF16, the first pass of the
// mixed path), Gram of Y, its eigenvalues by the Jacobi core, s_j = sqrt.
size_t features_workspace(int64_t m, int64_t p, int64_t nf) {
    return carve(nullptr, m, p, nf, 32, nullptr);
}

tsvdm_status launch_rank_features(const tsvdm_tensor *X, const float *omega, uint16_t *features, void *ws,
                                  hipStream_t s) {
    const int m = (int)X->m, p = (int)X->p, nf = (int)X->n3;
    if (nf == 0) return TSVDM_OK;
    MixedWs w;
    carve(reinterpret_cast<char *>(ws), m, p, nf, 32, &w);
    const int mparts = (m + 63) / 64;
    const float *Xd = reinterpret_cast<const float *>(X->data);
    const dim3 gm(xcd_grid(mparts, nf));
    if (vec_loads_ok(Xd, m, p) && reinterpret_cast<uintptr_t>(omega) % 16 == 0)
        TSVDM_LAUNCH("features_sketch", (k_xw<32, PROD_BF16, true, true>), gm, dim3(GT), 0, s, Xd, m, p, nf,
                     omega, (int64_t)0, p, 32, w.Y, w.fro_part, w.gram_m, (const int32_t *)nullptr);
    else
        TSVDM_LAUNCH("features_sketch", (k_xw<32, PROD_BF16, true, false>), gm, dim3(GT), 0, s, Xd, m, p, nf,
                     omega, (int64_t)0, p, 32, w.Y, w.fro_part, w.gram_m, (const int32_t *)nullptr);
    TSVDM_LAUNCH("features_eig", (k_core<32>), dim3(nf), dim3(QT), 0, s, (const double *)w.gram_m, mparts, 32,
                 (const double *)w.fro_part, mparts, (const double *)nullptr, 0, (int)TSVDM_RANK_FIXED, 32, 0.0,
                 30, 1e-15, w.UB, w.sig, w.perm, w.kf, w.fro2, (double *)nullptr, w.jinfo, (const int32_t *)nullptr);
    TSVDM_LAUNCH("features_log", k_rank_features, dim3(nf), dim3(32), 0, s, (const double *)w.sig, 32, nf,
                 reinterpret_cast<_Float16 *>(features));
    TSVDM_LAUNCH_CHECK("rank features");
    return TSVDM_OK;
}

namespace {
struct LearnedWs {
    uint16_t *feat;
    float *y;
    int32_t *lists, *counts, *fb_list, *caps;
    char *feat_ws, *bucket_ws[3];
};

constexpr int kBucketLP[3] = {16, 32, 48};

size_t learned_carve(char *base, int64_t m, int64_t p, int64_t nf, LearnedWs *w) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *ptr = base ? base + off : nullptr;
        off += al256(bytes);
        return ptr;
    };
    LearnedWs t;
    t.feat = (uint16_t *)take(sizeof(uint16_t) * 32 * nf);
    t.y = (float *)take(sizeof(float) * 2 * nf);
    t.lists = (int32_t *)take(sizeof(int32_t) * 3 * nf);
    t.counts = (int32_t *)take(sizeof(int32_t) * 8);
    t.fb_list = (int32_t *)take(sizeof(int32_t) * nf);
    t.caps = (int32_t *)take(sizeof(int32_t) * nf);
    t.feat_ws = take(features_workspace(m, p, nf));
    for (int b = 0; b < 3; ++b) t.bucket_ws[b] = take(carve(nullptr, m, p, nf, kBucketLP[b], nullptr));
    if (w) *w = t;
    return off;
}

}  // namespace

size_t learned_workspace(int64_t m, int64_t p, int64_t nf) { return learned_carve(nullptr, m, p, nf, nullptr); }

// Launches only (no host synchronization, no allocation after the first call
// on a device): capturable in a graph.  The feature sketch X Omega[:, :32]
// and its Gram partials serve twice: the features, and the first sketch of the
// width-16 and width-32 buckets.  Each bucket runs over a face list sized on
// the device (grids for all nf faces, unused slots exit at once) on its own
// stream; the fallback list then reruns, on the caller's stream, the faces
// whose certificate misses tau.
tsvdm_status launch_learned_truncate(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, const uint16_t *w16,
                                     tsvdm_factors *F, int32_t *widths, void *ws, hipStream_t s) {
    const int m = (int)X->m, p = (int)X->p, nf = (int)X->n3;
    if (nf == 0) return TSVDM_OK;
    LearnedWs w;
    learned_carve(reinterpret_cast<char *>(ws), m, p, nf, &w);
    tsvdm_status st = launch_rank_features(X, o->omega, w.feat, w.feat_ws, s);
    if (st != TSVDM_OK) return st;
    st = launch_mlp_forward(w16, w.feat, nf, w.y, s);
    if (st != TSVDM_OK) return st;
    TSVDM_LAUNCH("width_partition", k_width_partition, dim3(1), dim3(1024), 0, s, (const float *)w.y, nf,
                 w.lists, w.counts, widths, w.caps);
    TSVDM_LAUNCH_CHECK("width partition");
    SideStreams *ss = nullptr;
    if ((st = side_streams(&ss)) != TSVDM_OK) return st;
    hipError_t e = hipEventRecord(ss->ev[0], s);
    if (e != hipSuccess) return hip_check(e, "learned truncate: fork");
    MixedWs fw;  // the feature pass's sketch and Gram partials, indexed by face
    carve(w.feat_ws, m, p, nf, 32, &fw);
    // per width: (rank cap, oversampling) with ell = cap + oversampling
    const int caps[3] = {13, 26, 32}, overs[3] = {3, 6, 8};
    for (int b = 0; b < 3; ++b) {
        hipStream_t sb = ss->s[b];
        if ((e = hipStreamWaitEvent(sb, ss->ev[0], 0)) != hipSuccess) return hip_check(e, "learned truncate: wait");
        tsvdm_truncate_opts ob = *o;
        ob.rank_mode = TSVDM_RANK_ENERGY;
        ob.k = caps[b] < (int)F->kmax ? caps[b] : (int)F->kmax;
        ob.oversample = caps[b] + overs[b] - ob.k;
        ob.certify = 1;
        MixedWs tw;
        carve(w.bucket_ws[b], m, p, nf, kBucketLP[b], &tw);
        const int32_t *list = w.lists + (int64_t)b * nf;
        const MixedWs *src = b < 2 ? &fw : nullptr;
        if (b == 0) st = run_group<16>(X, &ob, F, tw, 0, nf, sb, list, -1, src, w.caps);
        else if (b == 1) st = run_group<32>(X, &ob, F, tw, 0, nf, sb, list, -1, src, w.caps);
        else st = run_group<48>(X, &ob, F, tw, 0, nf, sb, list, -1, src, w.caps);
        if (st != TSVDM_OK) return st;
        if ((e = hipEventRecord(ss->ev[1 + b], sb)) != hipSuccess) return hip_check(e, "learned truncate: join");
        if ((e = hipStreamWaitEvent(s, ss->ev[1 + b], 0)) != hipSuccess) return hip_check(e, "learned truncate: join");
    }
    // faces whose certificate misses tau: again with the full width and cap
    TSVDM_LAUNCH("fallback_list", k_fallback_list, dim3(1), dim3(1024), 0, s, (const double *)F->cert,
                 (const double *)F->fro, o->tau, nf, widths, (const int32_t *)w.caps, w.fb_list, w.counts + 3);
    TSVDM_LAUNCH_CHECK("fallback list");
    tsvdm_truncate_opts ob = *o;
    ob.rank_mode = TSVDM_RANK_ENERGY;
    ob.k = 32 < (int)F->kmax ? 32 : (int)F->kmax;
    ob.oversample = 40 - ob.k;
    ob.certify = 1;
    MixedWs tw;
    carve(w.bucket_ws[2], m, p, nf, 48, &tw);
    return run_group<48>(X, &ob, F, tw, 0, nf, s, w.fb_list);
}

}  // namespace tsvdm
