// Mode-3 transform of every tube: Xhat = X x_3 M (or x_3 M^{-1}).
//
// The mode-3 product multiplies each tube X(a, b, :) by M (mode-i product and
// mode-3 unfolding, Sec. 2.1).  Two implementations:
//
//  * k_fft_tubes: power-of-two tube length N (2..1024).  A tile of 2*TP
//    consecutive tubes (consecutive linear index i = a + m*b, so every load
//    and store of one time step is a contiguous run) is staged in LDS, two
//    real tubes packed into one complex sequence, and transformed by an
//    in-place radix-4/radix-2 decimation-in-time FFT.  The orthonormal DCT-II
//    uses Makhoul's reordering (even samples ascending, odd samples
//    descending) and a quarter-wave post-twiddle; its inverse runs the same
//    steps backwards.  The unitary DFT of real tubes keeps the Hermitian half
//    (faces 0..N/2).  Bound: HBM (about 2.5 log2 N flop per element).
//
//  * k_dense_tubes: any length up to 1024 and caller-supplied dense M.  The
//    tile is staged in LDS and every output is a direct sum over the tube;
//    DCT/DFT coefficients come from an LDS cosine table.
#include "common.h"

#include <math.h>

using namespace tsvdm;

namespace {

constexpr int NT = 256;

enum { KIND_DCT = 0, KIND_DFT = 1 };

__device__ __forceinline__ int bitrev(int x, int bits) {
    return (int)(__brev((unsigned)x) >> (32 - bits));
}

// position of sample t in Makhoul's reordered sequence
__device__ __forceinline__ int makhoul(int t, int N) { return (t & 1) ? (N - 1 - (t >> 1)) : (t >> 1); }

template <typename T>
__device__ __forceinline__ T dct_alpha(int f, int N) {
    return f == 0 ? (T)sqrt(1.0 / N) : (T)sqrt(2.0 / N);
}

// VEC: the input (forward) and output are dense with every tile full and 16-byte
// aligned rows, so a thread moves 16 bytes per load/store (4 FP32 or 2 FP64
// tubes of one time step) and issues all of its tile loads at once.
template <typename T, int KIND, int DIR, bool VEC>
__global__ __launch_bounds__(NT) void k_fft_tubes(const void *__restrict__ in, View iv,
                                                  void *__restrict__ out, int64_t ntubes,
                                                  int64_t mp, int logn, int logtp) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = 1 << logn, H = N >> 1, TP = 1 << logtp, TT = 2 * TP, logtt = logtp + 1;
    cx<T> *buf = reinterpret_cast<cx<T> *>(smem);  // [N][TP]
    cx<T> *tw = buf + N * TP;                        // [N/2]  exp(-+2 pi i j / N)
    cx<T> *wq = tw + H;                              // [N]    exp(-i pi f / (2N))
    int64_t *base = reinterpret_cast<int64_t *>(wq + N);  // [2TP]
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * TT;
    constexpr int UNR = 16;
    constexpr int VW = 16 / sizeof(T);  // elements per 16-byte vector
    typedef T vec_t __attribute__((ext_vector_type(VW)));
    // vector path, forward: the tile (at most 32 KiB, so at most 2048 vectors,
    // VMAX a thread) is loaded before the twiddles are computed, which then
    // overlap the loads' latency.  The input is read once: non-temporal loads
    // leave the caches (and the MALL) to the transformed tensor the next pass
    // reads (measured on 512 x 512 x 256: transform 124.6 -> 121.3 us, the
    // following sketch pass 74.4 -> 70.4 us)
    constexpr int VMAX = 2048 / NT;
    const int lvpr = logtt - (VW == 4 ? 2 : 1), vpr = 1 << lvpr, vtotal = vpr * N;
    vec_t vfirst[VMAX];
    if constexpr (DIR > 0 && VEC) {
        const T *X = reinterpret_cast<const T *>(in) + i0;
#pragma unroll
        for (int q = 0; q < VMAX; ++q) {
            const int w = tid + q * NT;
            const int u4 = w & (vpr - 1), t = w >> lvpr;
            if (w < vtotal)
                vfirst[q] = __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(X + u4 * VW + (int64_t)t * iv.s_t));
        }
    }

    for (int j = tid; j < H; j += NT) {
        double s, c;
        sincospi(2.0 * j / N, &s, &c);
        tw[j] = {(T)c, (T)(DIR > 0 ? -s : s)};
    }
    if (KIND == KIND_DCT) {
        for (int f = tid; f < N; f += NT) {
            double s, c;
            sincospi((double)f / (2.0 * N), &s, &c);
            wq[f] = {(T)c, (T)(-s)};
        }
    }
    for (int u = tid; u < TT; u += NT) base[u] = (i0 + u < ntubes) ? iv.tube_base(i0 + u) : -1;
    __syncthreads();

    // ---------------------------------------------------------------- load
    // Every thread issues a batch of UNR independent loads before it touches
    // LDS, so that many loads are in flight per wavefront.
    if constexpr (DIR > 0 && VEC) {
#pragma unroll
        for (int q = 0; q < VMAX; ++q) {
            const int w = tid + q * NT;
            if (w >= vtotal) break;
            const int u4 = w & (vpr - 1), t = w >> lvpr;
            const int n = KIND == KIND_DCT ? makhoul(t, N) : t;
            cx<T> *rowp = &buf[bitrev(n, logn) * TP];
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                const int u = u4 * VW + e;
                reinterpret_cast<T *>(&rowp[u & (TP - 1)])[u >= TP] = vfirst[q][e];
            }
        }
    } else if (DIR > 0) {  // real tubes in; tube u < TP -> real part, u >= TP -> imaginary part
        const T *X = reinterpret_cast<const T *>(in);
        const int total = TT * N;
        for (int w0 = tid; w0 < total; w0 += NT * UNR) {
            T vals[UNR];
#pragma unroll
            for (int q = 0; q < UNR; ++q) {
                const int w = w0 + q * NT;
                const int u = w & (TT - 1), t = w >> logtt;
                const int64_t b = w < total ? base[u] : -1;
                vals[q] = b >= 0 ? X[b + (int64_t)t * iv.s_t] : T(0);
            }
#pragma unroll
            for (int q = 0; q < UNR; ++q) {
                const int w = w0 + q * NT;
                if (w >= total) break;
                const int u = w & (TT - 1), t = w >> logtt;
                const int n = KIND == KIND_DCT ? makhoul(t, N) : t;
                T *slot = reinterpret_cast<T *>(&buf[bitrev(n, logn) * TP + (u & (TP - 1))]);
                slot[u >= TP] = vals[q];
            }
        }
    } else if (KIND == KIND_DFT) {  // Hermitian half spectra in (faces 0..N/2)
        const cx<T> *X = reinterpret_cast<const cx<T> *>(in);
#pragma unroll 4
        for (int w = tid; w < TP * (H + 1); w += NT) {
            int c = w & (TP - 1), f = w >> logtp;
            int64_t bx = base[c], by = base[c + TP];
            cx<T> a = bx >= 0 ? X[bx + (int64_t)f * iv.s_t] : cx<T>{0, 0};
            cx<T> b = by >= 0 ? X[by + (int64_t)f * iv.s_t] : cx<T>{0, 0};
            if (f == 0 || f == H) { a.im = 0; b.im = 0; }
            // Z = Sx + i Sy over the full spectrum, with S[N-f] = conj(S[f])
            buf[bitrev(f, logn) * TP + c] = {a.re - b.im, a.im + b.re};
            if (f > 0 && f < H) buf[bitrev(N - f, logn) * TP + c] = {a.re + b.im, b.re - a.im};
        }
    } else {  // inverse DCT-II: rebuild the FFT of Makhoul's sequence
        const T *X = reinterpret_cast<const T *>(in);
        const T rs0 = (T)sqrt((double)N), rs1 = (T)sqrt(N / 2.0);  // 1 / alpha_f
#pragma unroll 4
        for (int w = tid; w < TP * (H + 1); w += NT) {
            int c = w & (TP - 1), f = w >> logtp, g = N - f;
            int64_t bx = base[c], by = base[c + TP];
            T sf = f == 0 ? rs0 : rs1;
            T ax = bx >= 0 ? X[bx + (int64_t)f * iv.s_t] * sf : T(0);
            T ay = by >= 0 ? X[by + (int64_t)f * iv.s_t] * sf : T(0);
            T bxv = (f > 0 && bx >= 0) ? X[bx + (int64_t)g * iv.s_t] * rs1 : T(0);
            T byv = (f > 0 && by >= 0) ? X[by + (int64_t)g * iv.s_t] * rs1 : T(0);
            // V[f] = exp(i pi f/(2N)) (C[f] - i C[N-f]),  Z = Vx + i Vy
            cx<T> wc = cconj(wq[f]);
            cx<T> vx = cmul(wc, cx<T>{ax, -bxv}), vy = cmul(wc, cx<T>{ay, -byv});
            buf[bitrev(f, logn) * TP + c] = {vx.re - vy.im, vx.im + vy.re};
            if (f > 0 && f < H) {
                cx<T> wg = cconj(wq[g]);
                cx<T> ux = cmul(wg, cx<T>{bxv, -ax}), uy = cmul(wg, cx<T>{byv, -ay});
                buf[bitrev(g, logn) * TP + c] = {ux.re - uy.im, ux.im + uy.re};
            }
        }
    }
    __syncthreads();

    // ---------------------------------------------------------------- FFT
    int s = 0;
    if (logn & 1) {  // one radix-2 stage (h = 1)
        for (int w = tid; w < TP * H; w += NT) {
            int c = w & (TP - 1), qi = w >> logtp;
            int i0r = qi << 1, i1r = i0r + 1;
            cx<T> a = buf[i0r * TP + c], b = buf[i1r * TP + c];
            buf[i0r * TP + c] = cadd(a, b);
            buf[i1r * TP + c] = csub(a, b);
        }
        s = 1;
        __syncthreads();
    }
    for (; s < logn; s += 2) {  // radix-4: stages s and s+1 together
        const int h = 1 << s;
        for (int w = tid; w < TP * (N >> 2); w += NT) {
            int c = w & (TP - 1), qi = w >> logtp;
            int pos = qi & (h - 1), grp = qi >> s;
            int r0 = (grp << (s + 2)) + pos;
            cx<T> x0 = buf[r0 * TP + c], x1 = buf[(r0 + h) * TP + c];
            cx<T> x2 = buf[(r0 + 2 * h) * TP + c], x3 = buf[(r0 + 3 * h) * TP + c];
            cx<T> wa = tw[pos << (logn - s - 1)];
            cx<T> wb = tw[pos << (logn - s - 2)];
            cx<T> wc = tw[(pos + h) << (logn - s - 2)];
            cx<T> t1 = cmul(x1, wa), t3 = cmul(x3, wa);
            cx<T> a0 = cadd(x0, t1), a1 = csub(x0, t1), a2 = cadd(x2, t3), a3 = csub(x2, t3);
            cx<T> u2 = cmul(a2, wb), u3 = cmul(a3, wc);
            buf[r0 * TP + c] = cadd(a0, u2);
            buf[(r0 + 2 * h) * TP + c] = csub(a0, u2);
            buf[(r0 + h) * TP + c] = cadd(a1, u3);
            buf[(r0 + 3 * h) * TP + c] = csub(a1, u3);
        }
        __syncthreads();
    }

    // ---------------------------------------------------------------- store
    if (DIR > 0 && KIND == KIND_DCT) {
        T *Y = reinterpret_cast<T *>(out);
        const T al0 = (T)sqrt(1.0 / N), al1 = (T)sqrt(2.0 / N);
        auto dct_val = [&](int u, int f) -> T {
            const int c = u & (TP - 1);
            cx<T> Z = buf[f * TP + c], Zr = buf[((N - f) & (N - 1)) * TP + c];
            cx<T> V = u < TP ? cx<T>{(Z.re + Zr.re) * T(0.5), (Z.im - Zr.im) * T(0.5)}
                             : cx<T>{(Z.im + Zr.im) * T(0.5), (Zr.re - Z.re) * T(0.5)};
            cx<T> W = wq[f];
            return (W.re * V.re - W.im * V.im) * (f == 0 ? al0 : al1);
        };
        if (VEC) {
            const int lvpr = logtt - (VW == 4 ? 2 : 1), vpr = 1 << lvpr;
#pragma unroll 4
            for (int w = tid; w < vpr * N; w += NT) {
                const int u4 = w & (vpr - 1), f = w >> lvpr;
                vec_t v;
#pragma unroll
                for (int e = 0; e < VW; ++e) v[e] = dct_val(u4 * VW + e, f);
                *reinterpret_cast<vec_t *>(Y + i0 + u4 * VW + mp * f) = v;
            }
        } else {
#pragma unroll 8
            for (int w = tid; w < TT * N; w += NT) {
                int u = w & (TT - 1), f = w >> logtt;
                T val = dct_val(u, f);
                if (i0 + u < ntubes) Y[(i0 + u) + mp * f] = val;
            }
        }
    } else if (DIR > 0) {  // DFT, faces 0..N/2
        cx<T> *Y = reinterpret_cast<cx<T> *>(out);
        const T sc = (T)(0.5 / sqrt((double)N));
#pragma unroll 8
        for (int w = tid; w < TT * (H + 1); w += NT) {
            int u = w & (TT - 1), f = w >> logtt, c = u & (TP - 1);
            cx<T> Z = buf[f * TP + c], Zr = buf[((N - f) & (N - 1)) * TP + c];
            cx<T> V = u < TP ? cx<T>{(Z.re + Zr.re) * sc, (Z.im - Zr.im) * sc}
                             : cx<T>{(Z.im + Zr.im) * sc, (Zr.re - Z.re) * sc};
            if (i0 + u < ntubes) Y[(i0 + u) + mp * f] = V;
        }
    } else {
        T *Y = reinterpret_cast<T *>(out);
        const T sc = KIND == KIND_DFT ? (T)(1.0 / sqrt((double)N)) : (T)(1.0 / N);
        auto inv_val = [&](int u, int t) -> T {
            int n = KIND == KIND_DCT ? makhoul(t, N) : t;
            cx<T> Z = buf[n * TP + (u & (TP - 1))];
            return (u < TP ? Z.re : Z.im) * sc;
        };
        if (VEC) {
            const int lvpr = logtt - (VW == 4 ? 2 : 1), vpr = 1 << lvpr;
#pragma unroll 4
            for (int w = tid; w < vpr * N; w += NT) {
                const int u4 = w & (vpr - 1), t = w >> lvpr;
                vec_t v;
#pragma unroll
                for (int e = 0; e < VW; ++e) v[e] = inv_val(u4 * VW + e, t);
                *reinterpret_cast<vec_t *>(Y + i0 + u4 * VW + mp * t) = v;
            }
        } else {
#pragma unroll 8
            for (int w = tid; w < TT * N; w += NT) {
                int u = w & (TT - 1), t = w >> logtt;
                T val = inv_val(u, t);
                if (i0 + u < ntubes) Y[(i0 + u) + mp * t] = val;
            }
        }
    }
}

// ---------------------------------------------------------------- dense
enum { DENSE_DCT_FWD = 0, DENSE_DCT_INV, DENSE_M_FWD, DENSE_M_INV, DENSE_DFT_FWD, DENSE_DFT_INV };

template <typename T, int CASE>
__global__ __launch_bounds__(NT) void k_dense_tubes(const void *__restrict__ in, View iv,
                                                    void *__restrict__ out, int64_t ntubes,
                                                    int64_t mp, int N, int nf_in, int nf_out,
                                                    int TB, const double *__restrict__ Md) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr bool CIN = CASE == DENSE_DFT_INV;
    constexpr bool COUT = CASE == DENSE_DFT_FWD;
    constexpr bool TAB = CASE == DENSE_DCT_FWD || CASE == DENSE_DCT_INV || CASE == DENSE_DFT_FWD ||
                         CASE == DENSE_DFT_INV;
    double *ctab = reinterpret_cast<double *>(smem);  // [4N] cos(pi j / (2N))
    T *xs = reinterpret_cast<T *>(smem + (TAB ? sizeof(double) * 4 * N : 0));  // [nf_in][TB](x2)
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * TB;
    if (TAB)
        for (int j = tid; j < 4 * N; j += NT) ctab[j] = cospi((double)j / (2.0 * N));
    const int E = CIN ? 2 : 1;
    for (int w = tid; w < TB * nf_in; w += NT) {
        int u = w % TB, t = w / TB;
        bool ok = i0 + u < ntubes;
        int64_t b = ok ? iv.tube_base(i0 + u) + (int64_t)t * iv.s_t : 0;
        if (CIN) {
            const T *X = reinterpret_cast<const T *>(in);
            xs[(t * TB + u) * 2 + 0] = ok ? X[2 * b] : T(0);
            xs[(t * TB + u) * 2 + 1] = ok ? X[2 * b + 1] : T(0);
        } else {
            const T *X = reinterpret_cast<const T *>(in);
            xs[t * TB + u] = ok ? X[b] : T(0);
        }
    }
    __syncthreads();
    const int u = tid % TB, ng = NT / TB;
    const int fourN = 4 * N;
    const double rsn = 1.0 / sqrt((double)N);
    for (int o = tid / TB; o < nf_out; o += ng) {
        double acc = 0.0, acci = 0.0;
        for (int j = 0; j < nf_in; ++j) {
            if (CASE == DENSE_DCT_FWD || CASE == DENSE_DCT_INV) {
                int f = CASE == DENSE_DCT_FWD ? o : j, t = CASE == DENSE_DCT_FWD ? j : o;
                double a = f == 0 ? sqrt(1.0 / N) : sqrt(2.0 / N);
                acc += a * ctab[((2 * t + 1) * f) % fourN] * (double)xs[j * TB + u];
            } else if (CASE == DENSE_M_FWD) {
                acc += Md[o + (int64_t)N * j] * (double)xs[j * TB + u];
            } else if (CASE == DENSE_M_INV) {
                acc += Md[j + (int64_t)N * o] * (double)xs[j * TB + u];
            } else if (CASE == DENSE_DFT_FWD) {
                int r = (int)(((int64_t)o * j) % N);
                double c = ctab[4 * r], sn = ctab[(4 * r - N + fourN) % fourN];
                double x = (double)xs[j * TB + u];
                acc += c * x;
                acci -= sn * x;
            } else {  // DENSE_DFT_INV: faces j = 0..nf_in-1 of a Hermitian spectrum
                int r = (int)(((int64_t)j * o) % N);
                double c = ctab[4 * r], sn = ctab[(4 * r - N + fourN) % fourN];
                double wgt = (j == 0 || 2 * j == N) ? 1.0 : 2.0;
                acc += wgt * (c * (double)xs[(j * TB + u) * 2] - sn * (double)xs[(j * TB + u) * 2 + 1]);
            }
        }
        if (i0 + u < ntubes) {
            if (COUT) {
                T *Y = reinterpret_cast<T *>(out);
                Y[2 * ((i0 + u) + mp * o)] = (T)(acc * rsn);
                Y[2 * ((i0 + u) + mp * o) + 1] = (T)(acci * rsn);
            } else {
                T *Y = reinterpret_cast<T *>(out);
                Y[(i0 + u) + mp * o] = (T)(CASE == DENSE_DFT_INV ? acc * rsn : acc);
            }
        }
    }
    (void)E;
}

// Real M, n3 <= NMAX (16, 32, 48 or 64; n3 > NMAX - 16): the transform of
// the tubes is the product Y = M X (n3 x n3 times n3 x tubes) on the matrix
// cores.  A workgroup takes a chunk of kDirectChunk consecutive tubes of one
// tensor: it writes M (or M^T for INV) into LDS once, zero-padded to NMAX x
// NMAX, then each wavefront forms 16 C tubes at a time with 16x16x4 MFMAs
// (FP32 data in FP32, FP64 in FP64): the B operand (time step 4kk + lane/16 of
// tube lane%16) is loaded from the input straight into registers, the A
// operand (16 output rows by 4 time steps) comes from LDS.  After M is
// written there is no further barrier: the wavefronts stream through the
// chunk independently and many workgroups share a CU, so their loads,
// products and stores overlap.  DCT-II coefficients come from a table of
// cos(pi j / (2 n3)), j < 4 n3.
//
// Loads and stores go through buffer resources (base address and byte size
// of the input view and of the output in scalar registers, a 32-bit byte
// offset per lane, the offset of a group of time steps or output rows as a
// scalar offset).  The host guarantees that both byte spans, including
// NMAX time steps or rows, are below 2^31 (direct_span).  A lane whose
// element does not exist (time step or output row past n3, tube past the
// chunk) is given the offset 2^31: at or beyond the resource size whether or
// not the scalar offset is added, so the load returns zero and the store is
// dropped, with no select on a loaded value.
constexpr uint32_t kOffNone = 0x80000000u;

template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

template <typename T>
__device__ __forceinline__ void bstore(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(uint32_t __attribute__((ext_vector_type(2))), v),
                                              r, (int)voff, (int)soff, 0);
}

template <typename T, int NMAX, bool INV>
__device__ __forceinline__ void direct_chunk(const T *__restrict__ in, const View &iv, uint32_t in_bytes,
                                             T *__restrict__ out, uint32_t out_bytes, int64_t ntubes, int64_t mp,
                                             int N, const double *__restrict__ Md, bool dense, int64_t c0) {
    constexpr int G = NT / 64;                      // threads per row while M is written
    constexpr int LDM = NMAX + 4;                   // row pitch of M (4-lane groups hit distinct banks)
    constexpr int NTI = NMAX / 16, NK = NMAX / 4;   // output row blocks, time-step groups
    constexpr int C = sizeof(T) == 4 ? 2 : 1;       // 16-tube column blocks per wavefront step
    constexpr int NB = kDirectChunk / (16 * C * G); // steps of a wavefront per chunk
    static_assert(NB % 2 == 0, "steps are taken in pairs");
    constexpr uint32_t SZ = sizeof(T);
    __shared__ __align__(16) T Ms[NMAX * LDM];
    __shared__ double ctab[4 * NMAX];
    typedef T v4 __attribute__((ext_vector_type(4)));
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, kl = lane >> 4, l16 = lane & 15;
    const __amdgpu_buffer_rsrc_t rin = __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(in), 0, (int)in_bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rout = __builtin_amdgcn_make_buffer_rsrc(out, 0, (int)out_bytes, 0x00020000);
    const int64_t cend = c0 + kDirectChunk < ntubes ? c0 + kDirectChunk : ntubes;
    const uint32_t st_b = (uint32_t)iv.s_t * SZ;    // byte stride of one time step
    const uint32_t mp_b = (uint32_t)mp * SZ;        // byte stride of one output face
    // output rows of a lane: FP32 4*(lane/16) + v, FP64 lane/16 + 4v (+16 ti)
    const uint32_t orow = sizeof(T) == 4 ? 4 * kl : kl;
    const View32 v32 = make_view32(iv);  // tube offsets without 64-bit division
    // B operands of step s of this wavefront (tubes b0 + 16c + lane%16, time
    // step 4 kk + lane/16); tubes past the chunk read tube c0; only the last
    // four groups can reach past n3 (n3 > NMAX - 16)
    auto load_step = [&](T (&bx)[C][NK], int st) {
        const int64_t b0 = c0 + 16 * C * (wave + G * st);
        uint32_t vin[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int64_t i = b0 + l16 + 16 * c;
            vin[c] = v32.tube_base((uint32_t)(i < cend ? i : c0)) * SZ + (uint32_t)kl * st_b;
        }
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) {
            const uint32_t soff = (uint32_t)(4 * kk) * st_b;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const uint32_t vo = (kk >= NK - 4 && 4 * kk + kl >= N) ? kOffNone : vin[c];
                bx[c][kk] = bload<T>(rin, vo, soff);
            }
        }
    };
    // the first step's loads are in flight while M is written
    T xa[C][NK], xb[C][NK];
    load_step(xa, 0);
    if (!dense)
        for (int j = tid; j < 4 * N; j += NT) ctab[j] = cospi((double)j / (2.0 * N));
    for (int e = tid; e < NMAX * LDM; e += NT) Ms[e] = T(0);
    __syncthreads();
    // Ms[o * LDM + j]: coefficient of input j in output o.  Thread (o, g)
    // fills row o at columns j = g, g+G, ...; the cosine table index
    // (2t+1) f mod 4N advances by a fixed step along the row (no divisions).
    {
        const int o = tid % 64, g = tid / 64;
        if (o < N) {
            const int fourN = 4 * N;
            if (dense) {
                for (int j = g; j < N; j += G)
                    Ms[o * LDM + j] = (T)(INV ? Md[j + (int64_t)N * o] : Md[o + (int64_t)N * j]);
            } else {
                const double a0c = sqrt(1.0 / N), a1c = sqrt(2.0 / N);
                // forward: M[o][j], index (2j+1) o; inverse: M[j][o], index (2o+1) j
                int idx = INV ? ((2 * o + 1) * g) % fourN : ((2 * g + 1) * o) % fourN;
                const int step = INV ? (G * (2 * o + 1)) % fourN : (2 * G * o) % fourN;
                for (int j = g; j < N; j += G) {
                    const double a = (INV ? j : o) == 0 ? a0c : a1c;
                    Ms[o * LDM + j] = (T)(a * ctab[idx]);
                    idx += step;
                    if (idx >= fourN) idx -= fourN;
                }
            }
        }
    }
    __syncthreads();
    auto mma_store = [&](const T (&bx)[C][NK], int st) {
        const int64_t b0 = c0 + 16 * C * (wave + G * st);
        // M is read from LDS in every step: an opaque zero offset keeps the
        // compiler from merging the reads of all steps into registers held
        // across the chunk (64 more registers, fewer wavefronts per SIMD)
        int zoff;
        asm volatile("s_mov_b32 %0, 0" : "=s"(zoff));
        const T *Mz = Ms + zoff;
        v4 acc[C][NTI];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int ti = 0; ti < NTI; ++ti) acc[c][ti] = v4{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < NK; ++kk)
#pragma unroll
            for (int ti = 0; ti < NTI; ++ti) {
                const T am = Mz[(16 * ti + l16) * LDM + 4 * kk + kl];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    if constexpr (sizeof(T) == 4)
                        acc[c][ti] = __builtin_amdgcn_mfma_f32_16x16x4f32(am, bx[c][kk], acc[c][ti], 0, 0, 0);
                    else
                        acc[c][ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(am, bx[c][kk], acc[c][ti], 0, 0, 0);
                }
            }
        // rows below NMAX - 16 exist for every n3 of the class; the last block
        // drops rows past n3
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int64_t i = b0 + l16 + 16 * c;
            const uint32_t vout = i < cend ? (uint32_t)i * SZ + orow * mp_b : kOffNone;
#pragma unroll
            for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const uint32_t r0 = 16 * ti + (sizeof(T) == 4 ? v : 4 * v);  // row of lane group 0
                    const uint32_t vo = (ti == NTI - 1 && (int)(r0 + orow) >= N) ? kOffNone : vout;
                    bstore<T>(acc[c][ti][v], rout, vo, r0 * mp_b);
                }
        }
    };
    // steps in pairs through two register buffers; a wavefront's steps past
    // the end of a short chunk read tube c0 and store nothing
#pragma unroll
    for (int st = 0; st < NB; st += 2) {
        load_step(xb, st + 1);
        mma_store(xa, st);
        if (st + 2 < NB) load_step(xa, st + 2);
        mma_store(xb, st + 1);
    }
}

// DCT-II variant of direct_chunk: the even/odd symmetry of the orthonormal
// DCT-II, M[o][N-1-t] = (-1)^o M[o][t], splits each tube's product into two
// half-size ones (half the matrix-core work).  With H = ceil(N/2):
//  forward: u[t] = x[t] + x[N-1-t], w[t] = x[t] - x[N-1-t] (t < H; for odd N
//    the middle sample has no partner, which reads as zero), then
//    out[2o'] = sum_t M[2o'][t] u[t] and out[2o'+1] = sum_t M[2o'+1][t] w[t];
//  inverse: A[t] = sum_o' M[2o'][t] y[2o'], B[t] = sum_o' M[2o'+1][t] y[2o'+1]
//    (t < H), then out[t] = A[t] + B[t] and out[N-1-t] = A[t] - B[t]
//    (the odd-N middle row only once; its odd coefficients are zero).
// LDS holds the two half matrices (rows by depth, zero-padded to HM = NMAX/2
// deep and to whole 16-row blocks); the rest is as in direct_chunk.
template <typename T, int NMAX, bool INV>
__device__ __forceinline__ void direct_chunk_dct(const T *__restrict__ in, const View &iv, uint32_t in_bytes,
                                                 T *__restrict__ out, uint32_t out_bytes, int64_t ntubes,
                                                 int64_t mp, int N, int64_t c0) {
    constexpr int G = NT / 64;
    constexpr int HM = NMAX / 2;                    // depth of each half product (a multiple of 4)
    constexpr int NTH = (HM + 15) / 16;             // 16-row output blocks of each half product
    constexpr int LDH = HM + 4;                     // row pitch of the half matrices
    constexpr int NKH = HM / 4;                     // time-step groups of each half product
    constexpr int C = sizeof(T) == 4 ? 2 : 1;
    constexpr int NB = kDirectChunk / (16 * C * G);
    static_assert(NB % 2 == 0, "steps are taken in pairs");
    constexpr uint32_t SZ = sizeof(T);
    __shared__ __align__(16) T Me[16 * NTH * LDH];
    __shared__ __align__(16) T Mo[16 * NTH * LDH];
    __shared__ double ctab[4 * NMAX];
    typedef T v4 __attribute__((ext_vector_type(4)));
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, kl = lane >> 4, l16 = lane & 15;
    const __amdgpu_buffer_rsrc_t rin = __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(in), 0, (int)in_bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rout = __builtin_amdgcn_make_buffer_rsrc(out, 0, (int)out_bytes, 0x00020000);
    const int64_t cend = c0 + kDirectChunk < ntubes ? c0 + kDirectChunk : ntubes;
    const int H = (N + 1) / 2;
    const uint32_t st_b = (uint32_t)iv.s_t * SZ;
    const uint32_t mp_b = (uint32_t)mp * SZ;
    const uint32_t orow = sizeof(T) == 4 ? 4 * kl : kl;  // output row of lane group (+ v or 4v)
    const View32 v32 = make_view32(iv);  // tube offsets without 64-bit division
    // the lane's two operands of group kk: forward x[t], x[N-1-t]; inverse
    // y[2o'], y[2o'+1] (t, o' = 4 kk + lane/16); zero past the tube.  The
    // group's part of the offset (4 kk steps) is uniform: a scalar offset for
    // x[t] and y[2o'], y[2o'+1], one subtraction for the mirrored x[N-1-t].
    const uint32_t lrow = INV ? 2 * kl : kl;  // the lane's first time step in a group
    auto load_step = [&](T (&xa)[C][NKH], T (&xb)[C][NKH], int st) {
        const int64_t b0 = c0 + 16 * C * (wave + G * st);
        uint32_t va[C], vb[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int64_t i = b0 + l16 + 16 * c;
            const uint32_t vin = v32.tube_base((uint32_t)(i < cend ? i : c0)) * SZ;
            va[c] = vin + lrow * st_b;
            vb[c] = INV ? va[c] + st_b : vin + (uint32_t)(N - 1 - kl) * st_b;
        }
#pragma unroll
        for (int kk = 0; kk < NKH; ++kk) {
            const int t = 4 * kk + kl;
            bool oka, okb;
            if (INV) {
                oka = 2 * t < N;
                okb = 2 * t + 1 < N;
            } else {
                oka = t < H;
                okb = N - 1 - t > t;
            }
            const uint32_t sa = (uint32_t)((INV ? 8 : 4) * kk) * st_b;  // uniform
#pragma unroll
            for (int c = 0; c < C; ++c) {
                xa[c][kk] = bload<T>(rin, oka ? va[c] : kOffNone, sa);
                if (INV)
                    xb[c][kk] = bload<T>(rin, okb ? vb[c] : kOffNone, sa);
                else
                    xb[c][kk] = bload<T>(rin, okb ? vb[c] - sa : kOffNone, 0);
            }
        }
    };
    T xa0[C][NKH], xb0[C][NKH], xa1[C][NKH], xb1[C][NKH];
    load_step(xa0, xb0, 0);
    for (int j = tid; j < 4 * N; j += NT) ctab[j] = cospi((double)j / (2.0 * N));
    for (int e = tid; e < 16 * NTH * LDH; e += NT) {
        Me[e] = T(0);
        Mo[e] = T(0);
    }
    __syncthreads();
    {
        // entry (row r, depth k) of each half matrix: forward Me = M[2k'][..],
        // rows o' and depth t; inverse rows t and depth o'
        const double a0c = sqrt(1.0 / N), a1c = sqrt(2.0 / N);
        for (int e = tid; e < 2 * H * H; e += NT) {
            const int half = e / (H * H), rr = (e % (H * H)) / H, kk = e % H;
            const int o = INV ? 2 * kk + half : 2 * rr + half;  // DCT frequency
            const int t = INV ? rr : kk;                        // sample
            if (o >= N) continue;
            const double v = (o == 0 ? a0c : a1c) * ctab[((2 * t + 1) * o) % (4 * N)];
            (half ? Mo : Me)[rr * LDH + kk] = (T)v;
        }
    }
    __syncthreads();
    auto mma_store = [&](const T (&xa)[C][NKH], const T (&xb)[C][NKH], int st) {
        const int64_t b0 = c0 + 16 * C * (wave + G * st);
        int zoff;
        asm volatile("s_mov_b32 %0, 0" : "=s"(zoff));
        const T *Mez = Me + zoff, *Moz = Mo + zoff;
        v4 ae[C][NTH], ao[C][NTH];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int ti = 0; ti < NTH; ++ti) ae[c][ti] = ao[c][ti] = v4{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < NKH; ++kk) {
            T be[C], bo[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (INV) {
                    be[c] = xa[c][kk];
                    bo[c] = xb[c][kk];
                } else {
                    be[c] = xa[c][kk] + xb[c][kk];
                    bo[c] = xa[c][kk] - xb[c][kk];
                }
            }
#pragma unroll
            for (int ti = 0; ti < NTH; ++ti) {
                const T me = Mez[(16 * ti + l16) * LDH + 4 * kk + kl];
                const T mo = Moz[(16 * ti + l16) * LDH + 4 * kk + kl];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    if constexpr (sizeof(T) == 4) {
                        ae[c][ti] = __builtin_amdgcn_mfma_f32_16x16x4f32(me, be[c], ae[c][ti], 0, 0, 0);
                        ao[c][ti] = __builtin_amdgcn_mfma_f32_16x16x4f32(mo, bo[c], ao[c][ti], 0, 0, 0);
                    } else {
                        ae[c][ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(me, be[c], ae[c][ti], 0, 0, 0);
                        ao[c][ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(mo, bo[c], ao[c][ti], 0, 0, 0);
                    }
                }
            }
        }
        // stores: the lane's part of the offset once per column block, the
        // row block's part (16 ti + v rows) as a scalar offset; only the last
        // row block can pass n3 and checks its rows
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int64_t i = b0 + l16 + 16 * c;
            const uint32_t vi = i < cend ? (uint32_t)i * SZ : kOffNone;
            const uint32_t v1 = vi + (INV ? orow : 2 * orow) * mp_b;          // rows r or 2r
            const uint32_t v2 = INV ? vi + (uint32_t)(N - 1 - (int)orow) * mp_b  // rows N-1-r
                                    : v1 + mp_b;                               // rows 2r+1
#pragma unroll
            for (int ti = 0; ti < NTH; ++ti)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const uint32_t ru = 16 * ti + (sizeof(T) == 4 ? v : 4 * v);  // uniform part of r
                    const int r = (int)(ru + orow);
                    const T e = ae[c][ti][v], od = ao[c][ti][v];
                    const bool last = ti == NTH - 1;
                    if (INV) {
                        // rows r (A + B) and N-1-r (A - B), r < H; the middle row of odd N once
                        const bool ok1 = !last || r < H, ok2 = N - 1 - r > r;
                        bstore<T>(e + od, rout, ok1 ? v1 : kOffNone, ru * mp_b);
                        bstore<T>(e - od, rout, ok2 ? v2 - ru * mp_b : kOffNone, 0);
                    } else {
                        // rows 2r (even product) and 2r + 1 (odd product)
                        const bool ok1 = !last || 2 * r < N, ok2 = !last || 2 * r + 1 < N;
                        bstore<T>(e, rout, ok1 ? v1 : kOffNone, 2 * ru * mp_b);
                        bstore<T>(od, rout, ok2 ? v2 : kOffNone, 2 * ru * mp_b);
                    }
                }
        }
    };
#pragma unroll
    for (int st = 0; st < NB; st += 2) {
        load_step(xa1, xb1, st + 1);
        mma_store(xa0, xb0, st);
        if (st + 2 < NB) load_step(xa0, xb0, st + 2);
        mma_store(xa1, xb1, st + 1);
    }
}

template <typename T, int NMAX, bool INV, bool DENSE>
__global__ __launch_bounds__(NT) void k_direct_small(const T *__restrict__ in, View iv, uint32_t in_bytes,
                                                     T *__restrict__ out, uint32_t out_bytes, int64_t ntubes,
                                                     int64_t mp, int N, const double *__restrict__ Md) {
    if constexpr (DENSE)
        direct_chunk<T, NMAX, INV>(in, iv, in_bytes, out, out_bytes, ntubes, mp, N, Md, true,
                                   (int64_t)blockIdx.x * kDirectChunk);
    else
        direct_chunk_dct<T, NMAX, INV>(in, iv, in_bytes, out, out_bytes, ntubes, mp, N,
                                       (int64_t)blockIdx.x * kDirectChunk);
}

// Batched direct product: workgroup w transforms chunk items[w].chunk of the
// tensor described by desc[items[w].d] (tensors of one precision and one
// length class, NMAX - 16 < n3 <= NMAX).
// Batched DCT-II: one launch for every length class (the class of each work
// item from its tensor's n3), so the classes share one tail; the plan lists
// the items largest class first.
template <typename T, bool INV>
__global__ __launch_bounds__(NT) void k_direct_batched_dct(const DirectDesc *__restrict__ desc,
                                                           const DirectItem *__restrict__ items) {
    const DirectItem it = items[blockIdx.x];
    const DirectDesc &d = desc[it.d];
    const T *in = reinterpret_cast<const T *>(d.in);
    T *out = reinterpret_cast<T *>(d.out);
    const int64_t c0 = (int64_t)it.chunk * kDirectChunk;
    switch (direct_class(d.N)) {
        case 16: direct_chunk_dct<T, 16, INV>(in, d.iv, d.in_bytes, out, d.out_bytes, d.ntubes, d.mp, d.N, c0); break;
        case 32: direct_chunk_dct<T, 32, INV>(in, d.iv, d.in_bytes, out, d.out_bytes, d.ntubes, d.mp, d.N, c0); break;
        case 48: direct_chunk_dct<T, 48, INV>(in, d.iv, d.in_bytes, out, d.out_bytes, d.ntubes, d.mp, d.N, c0); break;
        default: direct_chunk_dct<T, 64, INV>(in, d.iv, d.in_bytes, out, d.out_bytes, d.ntubes, d.mp, d.N, c0); break;
    }
}

template <typename T, int NMAX, bool INV, bool DENSE>
__global__ __launch_bounds__(NT) void k_direct_batched(const DirectDesc *__restrict__ desc,
                                                       const DirectItem *__restrict__ items) {
    const DirectItem it = items[blockIdx.x];
    const DirectDesc &d = desc[it.d];
    if constexpr (DENSE)
        direct_chunk<T, NMAX, INV>(reinterpret_cast<const T *>(d.in), d.iv, d.in_bytes,
                                   reinterpret_cast<T *>(d.out), d.out_bytes, d.ntubes, d.mp, d.N, d.Md, true,
                                   (int64_t)it.chunk * kDirectChunk);
    else
        direct_chunk_dct<T, NMAX, INV>(reinterpret_cast<const T *>(d.in), d.iv, d.in_bytes,
                                       reinterpret_cast<T *>(d.out), d.out_bytes, d.ntubes, d.mp, d.N,
                                       (int64_t)it.chunk * kDirectChunk);
}

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename T>
tsvdm_status run_fft(int kind, int dir, const tsvdm_tensor *in, tsvdm_tensor *out, int N,
                     hipStream_t s) {
    int logn = 0;
    while ((1 << logn) < N) ++logn;
    const int64_t ntubes = in->m * in->p, mp = ntubes;
    // tile of 2*TP tubes: at most 32 KiB of LDS for the spectra, so that four
    // or more workgroups share a CU and their load, FFT and store phases
    // overlap (measured: 64 KiB tiles 162 us, 32 KiB 132 us, 16 KiB 159 us
    // for 512 x 512 x 256 FP32; the 16 KiB tile reads 64-byte runs per face)
    int TP = 64;
    while (TP > 1 && (size_t)N * TP * sizeof(cx<T>) > 32768) TP >>= 1;
    int logtp = 0;
    while ((1 << logtp) < TP) ++logtp;
    const size_t lds = sizeof(cx<T>) * ((size_t)N * TP + N / 2 + N) + sizeof(int64_t) * 2 * TP;
    const int64_t grid = (ntubes + 2 * TP - 1) / (2 * TP);
    if (grid == 0) return TSVDM_OK;
    View iv = make_view(*in);
    // vector fast path: all tiles full, 16-byte aligned rows in and out; dense
    // input for the forward direction
    const int vw = 16 / (int)sizeof(T);
    const bool dense_in = in->s_a == 1 && in->s_b == in->m && in->bsplit == 0;
    const bool vec = ntubes % (2 * TP) == 0 && mp % vw == 0 && 2 * TP >= vw &&
                     ((uintptr_t)out->data % 16) == 0 &&
                     (dir < 0 || (dense_in && in->s_t % vw == 0 && ((uintptr_t)in->data % 16) == 0));
    hipError_t e = hipSuccess;
#define TSVDM_FFT_LAUNCH(KD, DR)                                                                \
    do {                                                                                         \
        auto kern = vec ? k_fft_tubes<T, KD, DR, true> : k_fft_tubes<T, KD, DR, false>;          \
        e = allow_lds(kern, lds);                                                                \
        if (e != hipSuccess) return hip_check(e, "hipFuncSetAttribute(fft)");                   \
        TSVDM_LAUNCH("transform_fft", kern, dim3((unsigned)grid), dim3(NT), lds, s, in->data, iv,   \
                     out->data, ntubes, mp, logn, logtp);                                                \
    } while (0)
    if (kind == KIND_DCT && dir > 0) TSVDM_FFT_LAUNCH(KIND_DCT, 1);
    else if (kind == KIND_DCT) TSVDM_FFT_LAUNCH(KIND_DCT, -1);
    else if (dir > 0) TSVDM_FFT_LAUNCH(KIND_DFT, 1);
    else TSVDM_FFT_LAUNCH(KIND_DFT, -1);
#undef TSVDM_FFT_LAUNCH
    TSVDM_LAUNCH_CHECK("k_fft_tubes");
    return TSVDM_OK;
}

template <typename T>
tsvdm_status run_dense(int kind, int dir, const tsvdm_mdesc *M, const tsvdm_tensor *in,
                       tsvdm_tensor *out, int N, hipStream_t s) {
    const int64_t ntubes = in->m * in->p, mp = ntubes;
    const int nf_in = (int)in->n3, nf_out = (int)out->n3;
    const bool tab = kind != TSVDM_M_DENSE;
    const bool cin = kind == TSVDM_M_DFT && dir < 0;
    const size_t esz = sizeof(T) * (cin ? 2 : 1);
    const size_t tabb = tab ? sizeof(double) * 4 * N : 0;
    int TB = 64;
    while (TB > 1 && tabb + (size_t)nf_in * TB * esz > 96 * 1024) TB >>= 1;
    const size_t lds = tabb + (size_t)nf_in * TB * esz;
    const int64_t grid = (ntubes + TB - 1) / TB;
    if (grid == 0) return TSVDM_OK;
    View iv = make_view(*in);
    hipError_t e = hipSuccess;
#define TSVDM_DENSE_LAUNCH(CS)                                                                  \
    do {                                                                                         \
        auto kern = k_dense_tubes<T, CS>;                                                        \
        e = allow_lds(kern, lds);                                                                \
        if (e != hipSuccess) return hip_check(e, "hipFuncSetAttribute(dense)");                 \
        TSVDM_LAUNCH("transform_direct", kern, dim3((unsigned)grid), dim3(NT), lds, s, in->data, iv, \
                     out->data, ntubes, mp, N, nf_in, nf_out, TB, M->M);                             \
    } while (0)
    uint32_t in_bytes = 0, out_bytes = 0;
    if (kind != TSVDM_M_DFT && N <= 64 && direct_span(*in, N, sizeof(T), &in_bytes, &out_bytes)) {
        const int64_t g2 = (ntubes + kDirectChunk - 1) / kDirectChunk;
        const double *Md = M->M;
#define TSVDM_SMALL_LAUNCH(NM, INV, DN)                                                          \
    TSVDM_LAUNCH("transform_direct", (k_direct_small<T, NM, INV, DN>), dim3((unsigned)g2), dim3(NT), 0, s, \
                 reinterpret_cast<const T *>(in->data), iv, in_bytes, reinterpret_cast<T *>(out->data), out_bytes, \
                 ntubes, mp, N, Md)
#define TSVDM_SMALL_CLASS(NM)                                                                                 \
    do {                                                                                                      \
        if (dir > 0) { if (dn) TSVDM_SMALL_LAUNCH(NM, false, true); else TSVDM_SMALL_LAUNCH(NM, false, false); } \
        else { if (dn) TSVDM_SMALL_LAUNCH(NM, true, true); else TSVDM_SMALL_LAUNCH(NM, true, false); }          \
    } while (0)
        const bool dn = kind == TSVDM_M_DENSE;
        switch (direct_class(N)) {
            case 16: TSVDM_SMALL_CLASS(16); break;
            case 32: TSVDM_SMALL_CLASS(32); break;
            case 48: TSVDM_SMALL_CLASS(48); break;
            default: TSVDM_SMALL_CLASS(64); break;
        }
#undef TSVDM_SMALL_CLASS
#undef TSVDM_SMALL_LAUNCH
        TSVDM_LAUNCH_CHECK("k_direct_small");
        return TSVDM_OK;
    }
    if (kind == TSVDM_M_DCT2) {
        if (dir > 0) TSVDM_DENSE_LAUNCH(DENSE_DCT_FWD);
        else TSVDM_DENSE_LAUNCH(DENSE_DCT_INV);
    } else if (kind == TSVDM_M_DENSE) {
        if (dir > 0) TSVDM_DENSE_LAUNCH(DENSE_M_FWD);
        else TSVDM_DENSE_LAUNCH(DENSE_M_INV);
    } else {
        if (dir > 0) TSVDM_DENSE_LAUNCH(DENSE_DFT_FWD);
        else TSVDM_DENSE_LAUNCH(DENSE_DFT_INV);
    }
#undef TSVDM_DENSE_LAUNCH
    TSVDM_LAUNCH_CHECK("k_dense_tubes");
    return TSVDM_OK;
}

}  // namespace

namespace tsvdm {

tsvdm_status launch_direct_batched(const DirectDesc *desc, const TransformGroup &g, int direction,
                                   hipStream_t s) {
    if (g.count == 0) return TSVDM_OK;
    const dim3 grid((unsigned)g.count);
#define TSVDM_DB(T, NM, INV)                                                                          \
    do {                                                                                                  \
        if (g.dense)                                                                                      \
            TSVDM_LAUNCH("transform_direct_batched", (k_direct_batched<T, NM, INV, true>), grid, dim3(NT), 0, \
                         s, desc, g.items);                                                               \
        else                                                                                              \
            TSVDM_LAUNCH("transform_direct_batched", (k_direct_batched<T, NM, INV, false>), grid, dim3(NT), 0, \
                         s, desc, g.items);                                                               \
    } while (0)
#define TSVDM_DB_CLASS(T)                                                                   \
    do {                                                                                    \
        switch (g.nmax) {                                                                   \
            case 16: if (direction > 0) TSVDM_DB(T, 16, false); else TSVDM_DB(T, 16, true); break; \
            case 32: if (direction > 0) TSVDM_DB(T, 32, false); else TSVDM_DB(T, 32, true); break; \
            case 48: if (direction > 0) TSVDM_DB(T, 48, false); else TSVDM_DB(T, 48, true); break; \
            default: if (direction > 0) TSVDM_DB(T, 64, false); else TSVDM_DB(T, 64, true); break; \
        }                                                                                   \
    } while (0)
    if (!g.dense) {  // DCT-II: every length class in one launch
        if (g.dbl) {
            if (direction > 0)
                TSVDM_LAUNCH("transform_direct_batched", (k_direct_batched_dct<double, false>), grid, dim3(NT), 0, s,
                             desc, g.items);
            else
                TSVDM_LAUNCH("transform_direct_batched", (k_direct_batched_dct<double, true>), grid, dim3(NT), 0, s,
                             desc, g.items);
        } else {
            if (direction > 0)
                TSVDM_LAUNCH("transform_direct_batched", (k_direct_batched_dct<float, false>), grid, dim3(NT), 0, s,
                             desc, g.items);
            else
                TSVDM_LAUNCH("transform_direct_batched", (k_direct_batched_dct<float, true>), grid, dim3(NT), 0, s,
                             desc, g.items);
        }
    } else if (g.dbl) {
        TSVDM_DB_CLASS(double);
    } else {
        TSVDM_DB_CLASS(float);
    }
#undef TSVDM_DB_CLASS
#undef TSVDM_DB
    TSVDM_LAUNCH_CHECK("k_direct_batched");
    return TSVDM_OK;
}

tsvdm_status launch_transform(const tsvdm_mdesc *M, int direction, const tsvdm_tensor *in,
                              tsvdm_tensor *out, hipStream_t s) {
    const int N = (int)M->n3;
    const bool pow2 = N >= 2 && (N & (N - 1)) == 0;
    const bool dbl = in->dtype == TSVDM_F64 || in->dtype == TSVDM_C128;
    if (M->kind != TSVDM_M_DENSE && pow2) {
        int kind = M->kind == TSVDM_M_DCT2 ? KIND_DCT : KIND_DFT;
        return dbl ? run_fft<double>(kind, direction, in, out, N, s)
                   : run_fft<float>(kind, direction, in, out, N, s);
    }
    return dbl ? run_dense<double>(M->kind, direction, M, in, out, N, s)
               : run_dense<float>(M->kind, direction, M, in, out, N, s);
}

}  // namespace tsvdm
