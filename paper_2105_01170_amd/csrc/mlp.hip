// Learned rank predictor: a multilayer perceptron 32 -> 64 -> 64 -> 2 (ReLU
// hidden layers, linear output) in half precision with FP32 accumulation,
// trained with mean-squared error and Adam on FP32 master weights.
//
// Parameters, flat: W1 (64 x 32, row major), b1 (64), W2 (64 x 64), b2 (64),
// W3 (2 x 64), b3 (2): 6402 values.  Inputs are rows of 32 halves.
//  * k_mlp_fwd: one sample per wavefront (a hidden unit per lane), weights
//    in LDS, packed-half dot products (two half products summed into an FP32
//    accumulator); the hidden activations are rounded to half as they are
//    stored.
//  * k_mlp_grad: a block of 128 samples: the same forward pass, the backward
//    pass per sample in FP32, then the block's gradient as small products over
//    its samples (dZ^T A), written as one partial per block (deterministic).
//  * k_mlp_reduce: sums the partials in block order; k_mlp_adam applies Adam
//    (bias-corrected) to the master weights and refreshes the half copy.
#include "common.h"

#include <stdio.h>
#include <string.h>

#include <vector>

using namespace tsvdm;

namespace {

constexpr int NIN = 32, NH = 64, NOUT = 2;
constexpr int OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NOUT * NH, NPAR = OB3 + NOUT;
static_assert(NPAR == 6402, "parameter count");
constexpr int FT = 256;    // threads per block (forward)
constexpr int GS = 128;    // samples per gradient block
constexpr int GT = 256;    // threads per gradient block

typedef _Float16 half_t;
typedef half_t half2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float dot2(half2_t a, half2_t b, float c) {
    return __builtin_amdgcn_fdot2(a, b, c, false);
}

// forward of one sample: x (32 halves) -> a1, a2 (64 halves each), y (2)
// with the weights in LDS (halves, same flat layout)
__device__ __forceinline__ void mlp_sample(const half_t *w, const half_t *x, half_t *a1, half_t *a2,
                                           float *y, float *z1, float *z2) {
    const half2_t *x2 = reinterpret_cast<const half2_t *>(x);
    half2_t xv[NIN / 2];
#pragma unroll
    for (int i = 0; i < NIN / 2; ++i) xv[i] = x2[i];
    for (int u = 0; u < NH; ++u) {
        const half2_t *row = reinterpret_cast<const half2_t *>(w + OW1 + u * NIN);
        float acc = (float)w[OB1 + u];
#pragma unroll
        for (int i = 0; i < NIN / 2; ++i) acc = dot2(row[i], xv[i], acc);
        if (z1) z1[u] = acc;
        a1[u] = (half_t)fmaxf(acc, 0.0f);
    }
    const half2_t *h2 = reinterpret_cast<const half2_t *>(a1);
    for (int u = 0; u < NH; ++u) {
        const half2_t *row = reinterpret_cast<const half2_t *>(w + OW2 + u * NH);
        float acc = (float)w[OB2 + u];
#pragma unroll
        for (int i = 0; i < NH / 2; ++i) acc = dot2(row[i], h2[i], acc);
        if (z2) z2[u] = acc;
        a2[u] = (half_t)fmaxf(acc, 0.0f);
    }
    const half2_t *g2 = reinterpret_cast<const half2_t *>(a2);
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
        const half2_t *row = reinterpret_cast<const half2_t *>(w + OW3 + o * NH);
        float acc = (float)w[OB3 + o];
#pragma unroll
        for (int i = 0; i < NH / 2; ++i) acc = dot2(row[i], g2[i], acc);
        y[o] = acc;
    }
}

// One sample per wavefront: lane u forms hidden unit u of both layers (the
// same packed-half dot-product chain over its weight row as mlp_sample, so
// the results are the same bits), the activations pass between the layers
// through LDS, lanes 0 and 1 form the two outputs.  Four wavefronts per
// workgroup, each taking samples wave, wave + 4 * gridDim.x, ...
__global__ __launch_bounds__(FT) void k_mlp_fwd(const half_t *__restrict__ w16, const half_t *__restrict__ X,
                                                int64_t n, float *__restrict__ Y) {
    __shared__ __align__(16) half_t w[NPAR + 2];
    __shared__ __align__(16) half_t xs[FT / 64][NIN];
    __shared__ __align__(16) half_t hs[FT / 64][2][NH];
    for (int e = threadIdx.x; e < NPAR; e += FT) w[e] = w16[e];
    const int wave = threadIdx.x >> 6, u = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (FT / 64);
    const int64_t iters = (n + nw - 1) / nw;  // the same count in every wavefront
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t s = (it * gridDim.x + blockIdx.x) * (FT / 64) + wave;
        const bool ok = s < n;
        if (u < NIN) xs[wave][u] = ok ? X[s * NIN + u] : (half_t)0.0f;
        __syncthreads();
        {
            const half2_t *row = reinterpret_cast<const half2_t *>(w + OW1 + u * NIN);
            const half2_t *x2 = reinterpret_cast<const half2_t *>(xs[wave]);
            float acc = (float)w[OB1 + u];
#pragma unroll
            for (int i = 0; i < NIN / 2; ++i) acc = dot2(row[i], x2[i], acc);
            hs[wave][0][u] = (half_t)fmaxf(acc, 0.0f);
        }
        __syncthreads();
        {
            const half2_t *row = reinterpret_cast<const half2_t *>(w + OW2 + u * NH);
            const half2_t *h2 = reinterpret_cast<const half2_t *>(hs[wave][0]);
            float acc = (float)w[OB2 + u];
#pragma unroll
            for (int i = 0; i < NH / 2; ++i) acc = dot2(row[i], h2[i], acc);
            hs[wave][1][u] = (half_t)fmaxf(acc, 0.0f);
        }
        __syncthreads();
        if (u < NOUT && ok) {
            const half2_t *row = reinterpret_cast<const half2_t *>(w + OW3 + u * NH);
            const half2_t *g2 = reinterpret_cast<const half2_t *>(hs[wave][1]);
            float acc = (float)w[OB3 + u];
#pragma unroll
            for (int i = 0; i < NH / 2; ++i) acc = dot2(row[i], g2[i], acc);
            Y[s * NOUT + u] = acc;
        }
        __syncthreads();
    }
}

// Block b: samples [b*GS, min(n, (b+1)*GS)).  part[b * (NPAR + 1) + ...]:
// the block's gradient of loss = sum_s |y_s - t_s|^2 / (2 n), then its loss.
__global__ __launch_bounds__(GT) void k_mlp_grad(const half_t *__restrict__ w16, const half_t *__restrict__ X,
                                                 const float *__restrict__ Tg, int64_t n,
                                                 float *__restrict__ part) {
    __shared__ __align__(16) half_t w[NPAR + 2];
    __shared__ __align__(16) half_t xs[GS * NIN];
    __shared__ __align__(16) half_t a1s[GS * NH];
    __shared__ __align__(16) half_t a2s[GS * NH];
    __shared__ float dz1[GS * (NH + 1)];
    __shared__ float dz2[GS * (NH + 1)];
    __shared__ float dys[GS * NOUT];
    __shared__ float lsum[GT];
    const int tid = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * GS;
    const int ns = (int)(n - s0 < GS ? n - s0 : GS);
    for (int e = tid; e < NPAR; e += GT) w[e] = w16[e];
    for (int e = tid; e < GS * NIN; e += GT) {
        const int s = e / NIN;
        xs[e] = s < ns ? X[s0 * NIN + e] : (half_t)0.0f;
    }
    __syncthreads();
    float l = 0.0f;
    if (tid < GS) {
        const int s = tid;
        float z1[NH], z2[NH], y[NOUT];
        half_t *a1 = a1s + s * NH, *a2 = a2s + s * NH;
        mlp_sample(w, xs + s * NIN, a1, a2, y, z1, z2);
        float dy[NOUT];
        const float inv_n = 1.0f / (float)n;
#pragma unroll
        for (int o = 0; o < NOUT; ++o) {
            const float d = s < ns ? y[o] - Tg[(s0 + s) * NOUT + o] : 0.0f;
            l += 0.5f * d * d;
            dy[o] = d * inv_n;
            dys[s * NOUT + o] = dy[o];
        }
        // da2 = W3^T dy, dz2 = da2 (z2 > 0)
        for (int v = 0; v < NH; ++v) {
            float da = 0.0f;
#pragma unroll
            for (int o = 0; o < NOUT; ++o) da += (float)w[OW3 + o * NH + v] * dy[o];
            dz2[s * (NH + 1) + v] = z2[v] > 0.0f ? da : 0.0f;
        }
        // da1 = W2^T dz2, dz1 = da1 (z1 > 0)
        for (int u = 0; u < NH; ++u) {
            float da = 0.0f;
            for (int v = 0; v < NH; ++v) da += (float)w[OW2 + v * NH + u] * dz2[s * (NH + 1) + v];
            dz1[s * (NH + 1) + u] = z1[u] > 0.0f ? da : 0.0f;
        }
    }
    lsum[tid] = l;
    __syncthreads();
    // block gradient: G = dZ^T A over the block's samples (rows past ns are zero)
    float *pg = part + (int64_t)blockIdx.x * (NPAR + 1);
    for (int e = tid; e < NPAR; e += GT) {
        float acc = 0.0f;
        if (e < OB1) {  // W1[u][i] = sum_s dz1[s][u] x[s][i]
            const int u = e / NIN, i = e % NIN;
            for (int s = 0; s < GS; ++s) acc += dz1[s * (NH + 1) + u] * (float)xs[s * NIN + i];
        } else if (e < OW2) {
            const int u = e - OB1;
            for (int s = 0; s < GS; ++s) acc += dz1[s * (NH + 1) + u];
        } else if (e < OB2) {
            const int u = (e - OW2) / NH, v = (e - OW2) % NH;
            for (int s = 0; s < GS; ++s) acc += dz2[s * (NH + 1) + u] * (float)a1s[s * NH + v];
        } else if (e < OW3) {
            const int u = e - OB2;
            for (int s = 0; s < GS; ++s) acc += dz2[s * (NH + 1) + u];
        } else if (e < OB3) {
            const int o = (e - OW3) / NH, v = (e - OW3) % NH;
            for (int s = 0; s < GS; ++s) acc += dys[s * NOUT + o] * (float)a2s[s * NH + v];
        } else {
            const int o = e - OB3;
            for (int s = 0; s < GS; ++s) acc += dys[s * NOUT + o];
        }
        pg[e] = acc;
    }
    if (tid == 0) {
        float t = 0.0f;
        for (int i = 0; i < GT; ++i) t += lsum[i];
        pg[NPAR] = t / (float)n;
    }
}

// grad[e] = sum_b part[b][e] in block order (e = NPAR: the loss)
__global__ void k_mlp_reduce(const float *__restrict__ part, int nblk, float *__restrict__ grad,
                             float *__restrict__ loss) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e > NPAR) return;
    float acc = 0.0f;
    for (int b = 0; b < nblk; ++b) acc += part[(int64_t)b * (NPAR + 1) + e];
    if (e < NPAR) grad[e] = acc;
    else if (loss) *loss = acc;
}

__global__ void k_mlp_adam(float *__restrict__ w32, half_t *__restrict__ w16, float *__restrict__ m,
                           float *__restrict__ v, const float *__restrict__ grad, float lr, float c1,
                           float c2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NPAR) return;
    const float g = grad[e];
    const float mm = 0.9f * m[e] + 0.1f * g;
    const float vv = 0.999f * v[e] + 0.001f * g * g;
    m[e] = mm;
    v[e] = vv;
    const float wn = w32[e] - lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
    w32[e] = wn;
    w16[e] = (half_t)wn;
}

__global__ void k_f32_to_f16(const float *__restrict__ a, half_t *__restrict__ b, int n) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) b[e] = (half_t)a[e];
}

size_t grad_ws(int64_t n) {
    const int64_t nblk = (n + GS - 1) / GS;
    return (size_t)(nblk * (NPAR + 1) + NPAR + 64) * sizeof(float);
}

tsvdm_status run_grad(const uint16_t *w16, const uint16_t *x, const float *t, int64_t n, float *grad,
                      float *loss, void *ws, hipStream_t s) {
    const int64_t nblk = (n + GS - 1) / GS;
    float *part = reinterpret_cast<float *>(ws);
    TSVDM_LAUNCH("mlp_grad", k_mlp_grad, dim3((unsigned)nblk), dim3(GT), 0, s,
                 reinterpret_cast<const half_t *>(w16), reinterpret_cast<const half_t *>(x), t, n, part);
    TSVDM_LAUNCH("mlp_reduce", k_mlp_reduce, dim3((NPAR + 1 + 255) / 256), dim3(256), 0, s,
                 (const float *)part, (int)nblk, grad, loss);
    TSVDM_LAUNCH_CHECK("mlp gradient");
    return TSVDM_OK;
}

bool check_n(int64_t n, const char *who) {
    if (n < 1 || n > (int64_t(1) << 26)) {
        set_error("%s: n must be in 1..2^26 (got %lld)", who, (long long)n);
        return false;
    }
    return true;
}

}  // namespace

namespace tsvdm {
tsvdm_status launch_mlp_forward(const uint16_t *w16, const uint16_t *x, int64_t n, float *y, hipStream_t s) {
    const int64_t blocks = (n + FT / 64 - 1) / (FT / 64);
    TSVDM_LAUNCH("mlp_forward", k_mlp_fwd, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(FT), 0, s,
                 reinterpret_cast<const half_t *>(w16), reinterpret_cast<const half_t *>(x), n, y);
    TSVDM_LAUNCH_CHECK("mlp_forward");
    return TSVDM_OK;
}
}  // namespace tsvdm

namespace {
// CRC-32 of the IEEE 802.3 polynomial (reflected, 0xEDB88320), bit by bit
uint32_t crc32_update(uint32_t crc, const unsigned char *p, size_t n) {
    for (size_t i = 0; i < n; ++i) {
        crc ^= p[i];
        for (int b = 0; b < 8; ++b) crc = (crc >> 1) ^ (0xEDB88320u & (0u - (crc & 1u)));
    }
    return crc;
}

constexpr char kMagic[8] = {'T', 'S', 'V', 'D', 'M', 'M', 'L', 'P'};
constexpr uint32_t kVersion = 1;

struct CkptHeader {
    char magic[8];
    uint32_t version, nparams;
    int32_t step;
    uint32_t reserved;
};
static_assert(sizeof(CkptHeader) == 24, "checkpoint header layout");
}  // namespace

extern "C" {

int64_t tsvdm_mlp_nparams(void) { return NPAR; }

tsvdm_status tsvdm_mlp_save(const char *path, const uint16_t *w16, const float *w32, const float *m, const float *v,
                            int32_t step) {
    if (!path || !w16 || !w32 || !m || !v) {
        set_error("mlp_save: NULL argument");
        return TSVDM_EINVAL;
    }
    std::vector<unsigned char> buf(sizeof(CkptHeader) + NPAR * (2 + 3 * 4) + 4);
    CkptHeader h{};
    memcpy(h.magic, kMagic, 8);
    h.version = kVersion;
    h.nparams = NPAR;
    h.step = step;
    memcpy(buf.data(), &h, sizeof(h));
    size_t off = sizeof(h);
    hipError_t e = hipMemcpy(buf.data() + off, w16, NPAR * 2, hipMemcpyDefault);
    off += NPAR * 2;
    const float *src[3] = {w32, m, v};
    for (int i = 0; i < 3 && e == hipSuccess; ++i) {
        e = hipMemcpy(buf.data() + off, src[i], NPAR * 4, hipMemcpyDefault);
        off += NPAR * 4;
    }
    if (e != hipSuccess) return hip_check(e, "mlp_save: copy to host");
    const uint32_t crc = crc32_update(0xFFFFFFFFu, buf.data(), off) ^ 0xFFFFFFFFu;
    memcpy(buf.data() + off, &crc, 4);
    FILE *f = fopen(path, "wb");
    if (!f) {
        set_error("mlp_save: cannot open %s", path);
        return TSVDM_EINVAL;
    }
    const size_t wrote = fwrite(buf.data(), 1, buf.size(), f);
    const int closed = fclose(f);
    if (wrote != buf.size() || closed != 0) {
        set_error("mlp_save: short write to %s", path);
        return TSVDM_EINVAL;
    }
    return TSVDM_OK;
}

tsvdm_status tsvdm_mlp_load(const char *path, uint16_t *w16, float *w32, float *m, float *v, int32_t *step) {
    if (!path || !w16 || !w32 || !m || !v || !step) {
        set_error("mlp_load: NULL argument");
        return TSVDM_EINVAL;
    }
    const size_t total = sizeof(CkptHeader) + NPAR * (2 + 3 * 4) + 4;
    std::vector<unsigned char> buf(total + 1);
    FILE *f = fopen(path, "rb");
    if (!f) {
        set_error("mlp_load: cannot open %s", path);
        return TSVDM_EINVAL;
    }
    const size_t got = fread(buf.data(), 1, buf.size(), f);
    fclose(f);
    CkptHeader h{};
    if (got >= sizeof(h)) memcpy(&h, buf.data(), sizeof(h));
    if (got < sizeof(h) || memcmp(h.magic, kMagic, 8) != 0) {
        set_error("mlp_load: %s is not a predictor checkpoint", path);
        return TSVDM_EINVAL;
    }
    if (h.version != kVersion || h.nparams != (uint32_t)NPAR) {
        set_error("mlp_load: checkpoint version %u with %u parameters; expected version %u with %d", h.version,
                  h.nparams, kVersion, NPAR);
        return TSVDM_EINVAL;
    }
    if (got != total) {
        set_error("mlp_load: %s has %zu bytes, expected %zu", path, got, total);
        return TSVDM_EINVAL;
    }
    uint32_t crc;
    memcpy(&crc, buf.data() + total - 4, 4);
    if ((crc32_update(0xFFFFFFFFu, buf.data(), total - 4) ^ 0xFFFFFFFFu) != crc) {
        set_error("mlp_load: CRC mismatch in %s", path);
        return TSVDM_EINVAL;
    }
    size_t off = sizeof(h);
    hipError_t e = hipMemcpy(w16, buf.data() + off, NPAR * 2, hipMemcpyDefault);
    off += NPAR * 2;
    float *dst[3] = {w32, m, v};
    for (int i = 0; i < 3 && e == hipSuccess; ++i) {
        e = hipMemcpy(dst[i], buf.data() + off, NPAR * 4, hipMemcpyDefault);
        off += NPAR * 4;
    }
    if (e != hipSuccess) return hip_check(e, "mlp_load: copy to the device");
    *step = h.step;
    return TSVDM_OK;
}

size_t tsvdm_mlp_train_workspace_size(int64_t n) {
    if (n < 1 || n > (int64_t(1) << 26)) return 0;
    return grad_ws(n);
}

tsvdm_status tsvdm_mlp_forward(const uint16_t *w16, const uint16_t *x, int64_t n, float *y, void *stream) {
    if (!w16 || !x || !y) {
        set_error("mlp_forward: NULL argument");
        return TSVDM_EINVAL;
    }
    if (!check_n(n, "mlp_forward")) return TSVDM_EINVAL;
    return launch_mlp_forward(w16, x, n, y, (hipStream_t)stream);
}

tsvdm_status tsvdm_mlp_gradient(const uint16_t *w16, const uint16_t *x, const float *target, int64_t n,
                                float *grad, float *loss, void *ws, size_t ws_bytes, void *stream) {
    if (!w16 || !x || !target || !grad || !ws) {
        set_error("mlp_gradient: NULL argument");
        return TSVDM_EINVAL;
    }
    if (!check_n(n, "mlp_gradient")) return TSVDM_EINVAL;
    if (ws_bytes < grad_ws(n)) {
        set_error("mlp_gradient: workspace of %zu bytes needed, %zu given", grad_ws(n), ws_bytes);
        return TSVDM_EWORKSPACE;
    }
    return run_grad(w16, x, target, n, grad, loss, ws, (hipStream_t)stream);
}

tsvdm_status tsvdm_mlp_train_step(float *w32, uint16_t *w16, float *m, float *v, int32_t step, float lr,
                                  const uint16_t *x, const float *target, int64_t n, float *loss, void *ws,
                                  size_t ws_bytes, void *stream) {
    if (!w32 || !w16 || !m || !v || !x || !target || !ws) {
        set_error("mlp_train_step: NULL argument");
        return TSVDM_EINVAL;
    }
    if (!check_n(n, "mlp_train_step")) return TSVDM_EINVAL;
    if (step < 1 || !(lr > 0.0f)) {
        set_error("mlp_train_step: step >= 1 and lr > 0 required");
        return TSVDM_EINVAL;
    }
    if (ws_bytes < grad_ws(n)) {
        set_error("mlp_train_step: workspace of %zu bytes needed, %zu given", grad_ws(n), ws_bytes);
        return TSVDM_EWORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t nblk = (n + GS - 1) / GS;
    float *grad = reinterpret_cast<float *>(ws) + nblk * (NPAR + 1);
    tsvdm_status st = run_grad(w16, x, target, n, grad, loss, ws, s);
    if (st != TSVDM_OK) return st;
    const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
    TSVDM_LAUNCH("mlp_adam", k_mlp_adam, dim3((NPAR + 255) / 256), dim3(256), 0, s, w32,
                 reinterpret_cast<half_t *>(w16), m, v, (const float *)grad, lr, c1, c2);
    TSVDM_LAUNCH_CHECK("mlp_train_step");
    return TSVDM_OK;
}

tsvdm_status tsvdm_f32_to_f16(const float *a, uint16_t *b, int64_t n, void *stream) {
    if (!a || !b || n < 0 || n > (int64_t(1) << 30)) {
        set_error("f32_to_f16: bad arguments");
        return TSVDM_EINVAL;
    }
    if (n == 0) return TSVDM_OK;
    TSVDM_LAUNCH("f32_to_f16", k_f32_to_f16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                 (hipStream_t)stream, a, reinterpret_cast<half_t *>(b), (int)n);
    TSVDM_LAUNCH_CHECK("f32_to_f16");
    return TSVDM_OK;
}

}  // extern "C"
