// Internal helpers shared by the HIP sources of the t-SVDM library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tsvdm.h"

namespace tsvdm {

// ---------------------------------------------------------------- complex
template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.re, -a.im}; }

// ---------------------------------------------------------------- bf16
// Round-to-nearest-even float -> bf16 bit pattern (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// ---------------------------------------------------------------- views
// Strided third-order tensor view with an optionally split lateral index
// (b = j + bsplit*k), the zero-copy form of T_E[A].
struct View {
    int64_t m, p, n3, s_a, s_b, s_t, bsplit, s_bk;
    __host__ __device__ __forceinline__ int64_t tube_base(int64_t i) const {
        int64_t a = i % m, b = i / m;
        if (bsplit > 0) return a * s_a + (b % bsplit) * s_b + (b / bsplit) * s_bk;
        return a * s_a + b * s_b;
    }
};

// Division of 32-bit n < 2^31 by an invariant d >= 1 (Granlund and Montgomery,
// "Division by invariant integers using multiplication", 1994): with
// l = ceil(log2 d) and mul = floor(2^32 (2^l - d) / d) + 1 (< 2^32),
// floor(n / d) = (mulhi(mul, n) + n) >> l, the sum below 2^32 since n < 2^31.
struct UDiv {
    uint32_t d, mul, sh;
};
__host__ __device__ inline UDiv make_udiv(uint32_t d) {
    uint32_t l = 0;
    while (l < 31 && (1u << l) < d) ++l;
    const uint64_t mul = ((((uint64_t)1 << l) - d) << 32) / d + 1;
    return UDiv{d, (uint32_t)mul, l};
}
__device__ __forceinline__ uint32_t udiv(uint32_t n, const UDiv &u) {
    return (__umulhi(u.mul, n) + n) >> u.sh;
}

// A View whose element offsets are below 2^31 (direct_span), with the tube
// index split by invariant-divisor multiplication instead of 64-bit division.
struct View32 {
    UDiv m, bs;  // bs.d = 0: no block split
    uint32_t s_a, s_b, s_bk;
    __device__ __forceinline__ uint32_t tube_base(uint32_t i) const {
        const uint32_t b = udiv(i, m), a = i - b * m.d;
        if (bs.d == 0) return a * s_a + b * s_b;
        const uint32_t k = udiv(b, bs);
        return a * s_a + (b - k * bs.d) * s_b + k * s_bk;
    }
};
__device__ __forceinline__ View32 make_view32(const View &v) {
    View32 w;
    w.m = make_udiv((uint32_t)v.m);
    w.bs = v.bsplit > 0 ? make_udiv((uint32_t)v.bsplit) : UDiv{0, 0, 0};
    w.s_a = (uint32_t)v.s_a;
    w.s_b = (uint32_t)v.s_b;
    w.s_bk = (uint32_t)v.s_bk;
    return w;
}

// Direct (matrix-core) transform of tubes of length n3 <= 64: one workgroup
// per chunk of kDirectChunk consecutive tubes; the length class is
// direct_class(n3), the multiple of 16 at or above n3.
constexpr int kDirectChunk = 512;
__host__ __device__ constexpr int direct_class(int64_t n3) { return (int)(16 * ((n3 + 15) / 16)); }

// Byte spans of the input view and of the dense output of the direct
// transform, false unless both, counted up to direct_class(n3) time steps and
// output faces, are below 2^31 with non-negative strides (the direct kernels
// address both through buffer resources with 32-bit offsets).
inline bool direct_span(const tsvdm_tensor &in, int64_t n3, size_t esz, uint32_t *in_bytes,
                        uint32_t *out_bytes) {
    const int64_t lim = (int64_t)1 << 31;
    if (in.m <= 0 || in.p <= 0 || n3 <= 0) return false;
    if (in.s_a < 0 || in.s_b < 0 || in.s_t < 0 || in.s_bk < 0) return false;
    const int64_t nm = direct_class(n3);
    // largest element offset of a tube start, then of its last (padded) step
    int64_t base = (in.m - 1) * in.s_a;
    if (in.bsplit > 0) {
        const int64_t bs = in.bsplit < in.p ? in.bsplit : in.p;
        base += (bs - 1) * in.s_b + ((in.p - 1) / in.bsplit) * in.s_bk;
    } else {
        base += (in.p - 1) * in.s_b;
    }
    const double in_b = ((double)base + (double)nm * (double)in.s_t + 1.0) * (double)esz;
    const double out_b = (double)in.m * (double)in.p * (double)nm * (double)esz;
    if (!(in_b < (double)lim) || !(out_b < (double)lim)) return false;
    *in_bytes = (uint32_t)(((double)base + (double)(n3 - 1) * (double)in.s_t + 1.0) * (double)esz);
    *out_bytes = (uint32_t)((double)in.m * (double)in.p * (double)n3 * (double)esz);
    return true;
}

// Batched direct transform: one descriptor per tensor and one work item per
// chunk of kDirectChunk tubes (device arrays in the plan's workspace).
struct DirectDesc {
    const void *in;
    void *out;
    View iv;
    int64_t ntubes, mp;
    const double *Md;  // dense M (device), or null for the DCT-II
    int32_t N, dense;
    uint32_t in_bytes, out_bytes;  // direct_span
};
struct DirectItem {
    int32_t d, chunk;
};
// chunks of one precision and one length class (nmax = direct_class(N)), one launch
struct TransformGroup {
    bool dbl, dense;
    int nmax;
    const DirectItem *items;
    int64_t count;
};

inline View make_view(const tsvdm_tensor &t) {
    View v;
    v.m = t.m; v.p = t.p; v.n3 = t.n3;
    v.s_a = t.s_a; v.s_b = t.s_b; v.s_t = t.s_t;
    v.bsplit = t.bsplit; v.s_bk = t.s_bk;
    return v;
}

// Wave-level sum (64 lanes) via cross-lane shuffles.
// Strict total order for a descending sort by value with NaN last and ties
// broken by index: the rank sum_j sorts_before(v[j], j, v[i], i) of entry i is
// then a permutation of 0..n-1 whatever the values (a NaN input cannot leave
// a slot of the permutation unwritten).
__device__ __forceinline__ bool sorts_before(double a, int i, double b, int j) {
    const bool na = a != a, nb = b != b;
    if (na || nb) return nb && (!na || i < j);
    return a > b || (a == b && i < j);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace tsvdm

// ---------------------------------------------------------------- host side
namespace tsvdm {
void set_error(const char *fmt, ...);
tsvdm_status hip_check(hipError_t e, const char *what);

// launchers implemented in the .hip files
tsvdm_status launch_transform(const tsvdm_mdesc *M, int direction, const tsvdm_tensor *in,
                              tsvdm_tensor *out, hipStream_t s);
tsvdm_status launch_direct_batched(const DirectDesc *desc, const TransformGroup &g, int direction,
                                   hipStream_t s);
size_t jacobi_workspace(int64_t m, int64_t p, int64_t nf, bool cplx);
tsvdm_status launch_jacobi_truncate(const tsvdm_tensor *X, const tsvdm_truncate_opts *o,
                                    tsvdm_factors *F, void *ws, hipStream_t s);
size_t mixed_workspace(int64_t m, int64_t p, int64_t nf, int ell, bool cplx = false);
size_t f64rand_workspace(int64_t m, int64_t p, int64_t nf, int ell);
tsvdm_status launch_f64rand_truncate(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, tsvdm_factors *F,
                                     void *ws, hipStream_t s);
tsvdm_status launch_mixed_truncate(const tsvdm_tensor *X, const tsvdm_truncate_opts *o,
                                   tsvdm_factors *F, void *ws, hipStream_t s);
tsvdm_status launch_mixed_truncate_noalloc(const tsvdm_tensor *X, const tsvdm_truncate_opts *o,
                                           tsvdm_factors *F, hipStream_t s);
size_t noalloc_scratch_bytes();
// the device tables of a structured placement (structure.hip)
void placement_tables(const tsvdm_placement *pl, int64_t *ell, int64_t *q, int64_t *p, const int32_t **blk,
                      const double **winv);
tsvdm_status launch_mlp_forward(const uint16_t *w16, const uint16_t *x, int64_t n, float *y, hipStream_t s);
size_t features_workspace(int64_t m, int64_t p, int64_t nf);
tsvdm_status launch_rank_features(const tsvdm_tensor *X, const float *omega, uint16_t *features, void *ws,
                                  hipStream_t s);
size_t learned_workspace(int64_t m, int64_t p, int64_t nf);
tsvdm_status launch_learned_truncate(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, const uint16_t *w16,
                                     tsvdm_factors *F, int32_t *widths, void *ws, hipStream_t s);
size_t apply_workspace(const tsvdm_mdesc *M, const tsvdm_factors *F, int64_t ell, int64_t q,
                       int64_t nrhs, int32_t compute);
tsvdm_status launch_apply(const tsvdm_mdesc *M, const tsvdm_factors *F, int64_t ell, int64_t q,
                          int64_t nrhs, const void *x, int64_t ldx, void *y, int64_t ldy,
                          int32_t compute, void *ws, hipStream_t s);
}  // namespace tsvdm

namespace tsvdm {
extern bool g_trace;
void trace_begin(const char *name, hipStream_t s);
void trace_end(hipStream_t s);
}  // namespace tsvdm

// Launch with optional per-kernel event timing (tsvdm_timing_enable).
#define TSVDM_LAUNCH(name, kernel, grid, block, lds, stream, ...)              \
    do {                                                                      \
        if (::tsvdm::g_trace) ::tsvdm::trace_begin(name, stream);            \
        hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);   \
        if (::tsvdm::g_trace) ::tsvdm::trace_end(stream);                    \
    } while (0)

#define TSVDM_LAUNCH_CHECK(what)                                      \
    do {                                                              \
        hipError_t e_ = hipGetLastError();                            \
        if (e_ != hipSuccess) return ::tsvdm::hip_check(e_, what);    \
    } while (0)
