// Host side of the C ABI: argument validation, workspace sizing, dispatch.
// Every check runs before anything is enqueued; a failed check returns a
// status and leaves a message for tsvdm_last_error().
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <vector>

#include <algorithm>

#include "common.h"

namespace tsvdm {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

tsvdm_status hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return TSVDM_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return TSVDM_EDEVICE;
}

}  // namespace tsvdm

using namespace tsvdm;

#define FAIL(code, ...)            \
    do {                           \
        set_error(__VA_ARGS__);    \
        return (code);             \
    } while (0)

static bool is_real(int32_t d) { return d == TSVDM_F32 || d == TSVDM_F64; }
static bool is_cplx(int32_t d) { return d == TSVDM_C64 || d == TSVDM_C128; }
static bool is_double(int32_t d) { return d == TSVDM_F64 || d == TSVDM_C128; }
static bool is_dense(const tsvdm_tensor &t) {
    return t.s_a == 1 && t.s_b == t.m && t.s_t == t.m * t.p && t.bsplit == 0;
}

static tsvdm_status check_tensor(const tsvdm_tensor *t, const char *name, bool need_data = true) {
    if (!t) FAIL(TSVDM_EINVAL, "%s is NULL", name);
    if (t->m < 0 || t->p < 0 || t->n3 < 0) FAIL(TSVDM_EINVAL, "%s has a negative dimension", name);
    if (t->dtype < TSVDM_F64 || t->dtype > TSVDM_C128 || t->dtype == TSVDM_BF16)
        FAIL(TSVDM_EINVAL, "%s has unsupported dtype %d", name, t->dtype);
    if (need_data && t->m * t->p * t->n3 > 0 && !t->data) FAIL(TSVDM_EINVAL, "%s->data is NULL", name);
    if (t->bsplit < 0) FAIL(TSVDM_EINVAL, "%s->bsplit is negative", name);
    if (t->bsplit > 0 && t->p % t->bsplit != 0)
        FAIL(TSVDM_EINVAL, "%s->bsplit (%lld) does not divide p (%lld)", name, (long long)t->bsplit,
             (long long)t->p);
    return TSVDM_OK;
}

// ---- batched transform plan (host object)
struct tsvdm_transform_plan_s {
    int32_t direction = 1;
    const DirectDesc *desc = nullptr;
    std::vector<TransformGroup> groups;  // batched direct launches
    std::vector<int32_t> rest;           // tensors launched one by one
    std::vector<tsvdm_mdesc> M;
    std::vector<tsvdm_tensor> in, out;
};

static size_t al256h(size_t x) { return (x + 255) & ~(size_t)255; }

// group of tensor i in the batched direct launches: DCT-II 4*double (every
// length class in one launch), dense M 8 + 4*double + length class index
// (classes of 16); or -1 for a tensor launched by itself (DFT, N > 64, a view
// or output spanning 2 GiB or more, negative strides) or an empty one
constexpr int kTGroups = 16;
static int tgroup(const tsvdm_mdesc &M, const tsvdm_tensor &in) {
    if (M.kind == TSVDM_M_DFT || M.n3 > 64 || in.m * in.p == 0) return -1;
    const bool dbl = in.dtype == TSVDM_F64;
    uint32_t ib = 0, ob = 0;
    if (!direct_span(in, M.n3, dbl ? 8 : 4, &ib, &ob)) return -1;
    if (M.kind != TSVDM_M_DENSE) return 4 * (dbl ? 1 : 0);
    return 8 + 4 * (dbl ? 1 : 0) + direct_class(M.n3) / 16 - 1;
}

static int64_t tchunks(const tsvdm_tensor &in) { return (in.m * in.p + kDirectChunk - 1) / kDirectChunk; }

// workspace layout: descriptors, then the work items of groups 0..kTGroups-1
static size_t tplan_layout(int32_t nmat, const tsvdm_mdesc *M, const tsvdm_tensor *in,
                           int64_t cnt[kTGroups], size_t off[kTGroups + 1]) {
    for (int g = 0; g < kTGroups; ++g) cnt[g] = 0;
    for (int32_t i = 0; i < nmat; ++i) {
        const int g = tgroup(M[i], in[i]);
        if (g >= 0) cnt[g] += tchunks(in[i]);
    }
    off[0] = al256h(sizeof(DirectDesc) * (size_t)nmat);
    for (int g = 0; g < kTGroups; ++g) off[g + 1] = off[g] + al256h(sizeof(DirectItem) * (size_t)cnt[g]);
    return off[kTGroups];
}

static tsvdm_status check_transform(const tsvdm_mdesc *M, int32_t direction, const tsvdm_tensor *in,
                                    const tsvdm_tensor *out, bool need_data = true) {
    if (!M) FAIL(TSVDM_EINVAL, "M is NULL");
    if (M->kind < TSVDM_M_DCT2 || M->kind > TSVDM_M_DENSE) FAIL(TSVDM_EINVAL, "unknown M kind %d", M->kind);
    if (M->n3 < 1) FAIL(TSVDM_EINVAL, "M->n3 must be >= 1");
    if (M->n3 > 1024) FAIL(TSVDM_EUNSUPPORTED, "transform length %lld > 1024", (long long)M->n3);
    if (M->kind == TSVDM_M_DENSE && !M->M) FAIL(TSVDM_EINVAL, "dense M requires M->M");
    if (direction != 1 && direction != -1) FAIL(TSVDM_EINVAL, "direction must be +1 or -1");
    tsvdm_status st;
    if ((st = check_tensor(in, "in", need_data)) != TSVDM_OK) return st;
    if ((st = check_tensor(out, "out", need_data)) != TSVDM_OK) return st;
    if (!is_dense(*out)) FAIL(TSVDM_EINVAL, "out must be dense (strides 1, m, m*p)");
    if (in->m != out->m || in->p != out->p) FAIL(TSVDM_EINVAL, "in and out differ in m or p");
    if (is_double(in->dtype) != is_double(out->dtype)) FAIL(TSVDM_EINVAL, "in and out differ in precision");
    const int64_t n3 = M->n3, half = n3 / 2 + 1;
    if (M->kind == TSVDM_M_DFT) {
        if (direction > 0) {
            if (!is_real(in->dtype) || !is_cplx(out->dtype))
                FAIL(TSVDM_EINVAL, "forward DFT maps a real tensor to a complex one");
            if (in->n3 != n3 || out->n3 != half)
                FAIL(TSVDM_EINVAL, "forward DFT: in->n3 must be %lld and out->n3 %lld", (long long)n3,
                     (long long)half);
        } else {
            if (!is_cplx(in->dtype) || !is_real(out->dtype))
                FAIL(TSVDM_EINVAL, "inverse DFT maps a complex half spectrum to a real tensor");
            if (in->n3 != half || out->n3 != n3)
                FAIL(TSVDM_EINVAL, "inverse DFT: in->n3 must be %lld and out->n3 %lld", (long long)half,
                     (long long)n3);
        }
    } else {
        if (!is_real(in->dtype) || in->dtype != out->dtype)
            FAIL(TSVDM_EINVAL, "DCT-II / dense M map real tensors to real tensors of the same type");
        if (in->n3 != n3 || out->n3 != n3) FAIL(TSVDM_EINVAL, "tube length differs from M->n3");
    }
    if (need_data && in->data == out->data && in->m * in->p > 0) FAIL(TSVDM_EINVAL, "in and out must not alias");
    return TSVDM_OK;
}

extern "C" {

int32_t tsvdm_version(void) { return (1 << 16) | 0; }

const char *tsvdm_last_error(void) { return g_err; }

tsvdm_status tsvdm_tensor_from_blockmat(const void *A, int64_t lda, int32_t dtype, int64_t ell,
                                        int64_t q, int64_t m, int64_t n, tsvdm_tensor *out) {
    if (!out) FAIL(TSVDM_EINVAL, "out is NULL");
    if (ell <= 0 || q <= 0 || m <= 0 || n <= 0) FAIL(TSVDM_EINVAL, "block sizes must be positive");
    if (lda < ell * m) FAIL(TSVDM_EINVAL, "lda (%lld) < ell*m (%lld)", (long long)lda, (long long)(ell * m));
    if (!is_real(dtype)) FAIL(TSVDM_EINVAL, "block matrix dtype must be F32 or F64");
    if (!A) FAIL(TSVDM_EINVAL, "A is NULL");
    // X(a, j + ell*k, t) = A(j*m + a, k*n + t) = A[a + m*j + lda*n*k + lda*t]
    out->m = m;
    out->p = ell * q;
    out->n3 = n;
    out->s_a = 1;
    out->s_b = m;
    out->s_t = lda;
    out->bsplit = ell;
    out->s_bk = lda * n;
    out->dtype = dtype;
    out->reserved = 0;
    out->data = const_cast<void *>(A);
    return TSVDM_OK;
}

tsvdm_status tsvdm_check_orthogonal(const double *M, int64_t n3, double tol) {
    if (!M || n3 <= 0) FAIL(TSVDM_EINVAL, "M is NULL or n3 <= 0");
    for (int64_t i = 0; i < n3; ++i)
        for (int64_t j = 0; j < n3; ++j) {
            double acc = 0.0;
            for (int64_t t = 0; t < n3; ++t) acc += M[t + n3 * i] * M[t + n3 * j];
            double d = std::fabs(acc - (i == j ? 1.0 : 0.0));
            if (!(d <= tol))
                FAIL(TSVDM_EINVAL, "M is not orthogonal: |M^T M - I|(%lld,%lld) = %g", (long long)i,
                     (long long)j, d);
        }
    return TSVDM_OK;
}

tsvdm_status tsvdm_transform(const tsvdm_mdesc *M, int32_t direction, const tsvdm_tensor *in,
                             tsvdm_tensor *out, void *stream) {
    tsvdm_status st = check_transform(M, direction, in, out);
    if (st != TSVDM_OK) return st;
    if (in->m * in->p == 0) return TSVDM_OK;
    return launch_transform(M, direction, in, out, (hipStream_t)stream);
}

size_t tsvdm_transform_batched_workspace_size(int32_t nmat, const tsvdm_mdesc *M, const tsvdm_tensor *in) {
    if (nmat < 0 || (nmat > 0 && (!M || !in))) return 0;
    for (int32_t i = 0; i < nmat; ++i)
        if (M[i].kind < TSVDM_M_DCT2 || M[i].kind > TSVDM_M_DENSE || M[i].n3 < 1 || in[i].m < 0 || in[i].p < 0)
            return 0;
    int64_t cnt[kTGroups];
    size_t off[kTGroups + 1];
    return tplan_layout(nmat, M, in, cnt, off);
}

tsvdm_status tsvdm_transform_plan_create(int32_t nmat, const tsvdm_mdesc *M, int32_t direction,
                                         const tsvdm_tensor *in, const tsvdm_tensor *out, void *workspace,
                                         size_t workspace_bytes, tsvdm_transform_plan **plan) {
    if (!plan) FAIL(TSVDM_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (nmat < 0) FAIL(TSVDM_EINVAL, "nmat must be >= 0");
    if (nmat > 0 && (!M || !in || !out)) FAIL(TSVDM_EINVAL, "M, in and out must not be NULL");
    for (int32_t i = 0; i < nmat; ++i) {
        tsvdm_status st = check_transform(&M[i], direction, &in[i], &out[i]);
        if (st != TSVDM_OK) {
            char msg[512];
            snprintf(msg, sizeof(msg), "tensor %d: %s", (int)i, tsvdm_last_error());
            FAIL(st, "%s", msg);
        }
        if (tchunks(in[i]) > INT32_MAX) FAIL(TSVDM_EUNSUPPORTED, "tensor %d has too many tubes", (int)i);
    }
    int64_t cnt[kTGroups];
    size_t off[kTGroups + 1];
    const size_t need = tplan_layout(nmat, M, in, cnt, off);
    if (need > 0 && !workspace) FAIL(TSVDM_EWORKSPACE, "workspace is NULL");
    if (workspace_bytes < need)
        FAIL(TSVDM_EWORKSPACE, "workspace too small: %zu < %zu bytes", workspace_bytes, need);
    std::vector<unsigned char> h(need, 0);
    DirectDesc *desc = reinterpret_cast<DirectDesc *>(h.data());
    int64_t fill[kTGroups] = {};
    auto *plan_obj = new tsvdm_transform_plan_s;
    plan_obj->direction = direction;
    for (int32_t i = 0; i < nmat; ++i) {
        const int g = tgroup(M[i], in[i]);
        if (g < 0) {
            if (in[i].m * in[i].p > 0) plan_obj->rest.push_back(i);
            continue;
        }
        DirectDesc &d = desc[i];
        d.in = in[i].data;
        d.out = out[i].data;
        d.iv = make_view(in[i]);
        d.ntubes = in[i].m * in[i].p;
        d.mp = d.ntubes;
        d.Md = M[i].kind == TSVDM_M_DENSE ? M[i].M : nullptr;
        d.N = (int32_t)M[i].n3;
        d.dense = M[i].kind == TSVDM_M_DENSE ? 1 : 0;
        direct_span(in[i], M[i].n3, (g & 4) ? 8 : 4, &d.in_bytes, &d.out_bytes);
        DirectItem *items = reinterpret_cast<DirectItem *>(h.data() + off[g]);
        const int64_t nt = tchunks(in[i]);
        for (int64_t t = 0; t < nt; ++t) items[fill[g]++] = DirectItem{i, (int32_t)t};
    }
    // the DCT groups hold every length class: largest class first, so the
    // launch ends on the cheapest chunks
    for (int g = 0; g < kTGroups; ++g) {
        if ((g & 8) || cnt[g] == 0) continue;
        DirectItem *items = reinterpret_cast<DirectItem *>(h.data() + off[g]);
        std::stable_sort(items, items + cnt[g], [&](const DirectItem &a, const DirectItem &b) {
            return direct_class(desc[a.d].N) > direct_class(desc[b.d].N);
        });
    }
    if (need > 0) {
        const hipError_t e = hipMemcpy(workspace, h.data(), need, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            delete plan_obj;
            return hip_check(e, "hipMemcpy(transform plan)");
        }
    }
    unsigned char *ws = reinterpret_cast<unsigned char *>(workspace);
    plan_obj->desc = reinterpret_cast<const DirectDesc *>(ws);
    for (int g = 0; g < kTGroups; ++g)
        if (cnt[g] > 0)
            plan_obj->groups.push_back(
                TransformGroup{(g & 4) != 0, (g & 8) != 0, (g & 8) ? 16 * (g % 4 + 1) : 0, reinterpret_cast<const DirectItem *>(ws + off[g]), cnt[g]});
    plan_obj->M.assign(M, M + nmat);
    plan_obj->in.assign(in, in + nmat);
    plan_obj->out.assign(out, out + nmat);
    *plan = plan_obj;
    return TSVDM_OK;
}

tsvdm_status tsvdm_transform_batched(const tsvdm_transform_plan *plan, void *stream) {
    if (!plan) FAIL(TSVDM_EINVAL, "plan is NULL");
    const hipStream_t s = (hipStream_t)stream;
    for (const TransformGroup &g : plan->groups) {
        tsvdm_status st = launch_direct_batched(plan->desc, g, plan->direction, s);
        if (st != TSVDM_OK) return st;
    }
    for (int32_t i : plan->rest) {
        tsvdm_tensor o = plan->out[i];
        tsvdm_status st = launch_transform(&plan->M[i], plan->direction, &plan->in[i], &o, s);
        if (st != TSVDM_OK) return st;
    }
    return TSVDM_OK;
}

void tsvdm_transform_plan_destroy(tsvdm_transform_plan *plan) { delete plan; }

// need_data = false for the workspace query, which looks at shapes only
static tsvdm_status check_truncate(const tsvdm_tensor *X, const tsvdm_truncate_opts *o,
                                   bool need_data = true) {
    tsvdm_status st;
    if ((st = check_tensor(X, "Xhat", need_data)) != TSVDM_OK) return st;
    if (!is_dense(*X)) FAIL(TSVDM_EINVAL, "Xhat must be dense (strides 1, m, m*p)");
    if (!o) FAIL(TSVDM_EINVAL, "opts is NULL");
    if (o->rank_mode != TSVDM_RANK_FIXED && o->rank_mode != TSVDM_RANK_ENERGY)
        FAIL(TSVDM_EUNSUPPORTED, "rank mode %d", o->rank_mode);
    if (o->k < 0) FAIL(TSVDM_EINVAL, "k must be >= 0");
    if (o->rank_mode == TSVDM_RANK_ENERGY && !(o->tau >= 0.0)) FAIL(TSVDM_EINVAL, "tau must be >= 0");
    if (o->max_sweeps < 0) FAIL(TSVDM_EINVAL, "max_sweeps must be >= 0");
    if (o->precision == TSVDM_PREC_F64) {
        if (!is_double(X->dtype)) FAIL(TSVDM_EINVAL, "PREC_F64 needs an F64 or C128 Xhat");
    } else if (o->precision == TSVDM_PREC_MIXED || o->precision == TSVDM_PREC_F64_RAND) {
        if (o->precision == TSVDM_PREC_MIXED && X->dtype != TSVDM_F32 && X->dtype != TSVDM_C64)
            FAIL(TSVDM_EUNSUPPORTED, "PREC_MIXED needs an F32 or C64 Xhat");
        if (o->precision == TSVDM_PREC_F64_RAND && X->dtype != TSVDM_F64)
            FAIL(TSVDM_EUNSUPPORTED, "PREC_F64_RAND needs a real F64 Xhat");
        if (o->oversample < 0) FAIL(TSVDM_EINVAL, "oversample must be >= 0");
        if (o->power_iters < 0 || o->power_iters > 1) FAIL(TSVDM_EUNSUPPORTED, "power_iters must be 0 or 1");
        int ell = o->k + o->oversample;
        if (ell < 1 || ell > 64) FAIL(TSVDM_EUNSUPPORTED, "sketch width k+oversample = %d not in 1..64", ell);
        if (is_cplx(X->dtype) && ell > 48)
            FAIL(TSVDM_EUNSUPPORTED, "sketch width k+oversample = %d not in 1..48 for complex faces", ell);
        if (ell > X->m || ell > X->p)
            FAIL(TSVDM_EINVAL, "sketch width %d exceeds min(m, p) = %lld", ell,
                 (long long)(X->m < X->p ? X->m : X->p));
        if (need_data && !o->omega) FAIL(TSVDM_EINVAL, "the randomized truncation needs the test matrix omega");
    } else {
        FAIL(TSVDM_EINVAL, "unknown precision %d", o->precision);
    }
    return TSVDM_OK;
}

size_t tsvdm_truncate_workspace_size(const tsvdm_tensor *X, const tsvdm_truncate_opts *o) {
    if (check_truncate(X, o, false) != TSVDM_OK) return 0;
    if (o->precision == TSVDM_PREC_F64) return jacobi_workspace(X->m, X->p, X->n3, is_cplx(X->dtype));
    if (o->precision == TSVDM_PREC_F64_RAND) return f64rand_workspace(X->m, X->p, X->n3, o->k + o->oversample);
    return mixed_workspace(X->m, X->p, X->n3, o->k + o->oversample, is_cplx(X->dtype));
}

// the factors of a truncation of X with options o
static tsvdm_status check_truncate_out(const tsvdm_tensor *X, const tsvdm_truncate_opts *o,
                                       const tsvdm_factors *F) {
    if (!F) FAIL(TSVDM_EINVAL, "out is NULL");
    if (F->m != X->m || F->p != X->p || F->nf != X->n3)
        FAIL(TSVDM_EINVAL, "factor dims (%lld, %lld, %lld) differ from Xhat (%lld, %lld, %lld)",
             (long long)F->m, (long long)F->p, (long long)F->nf, (long long)X->m, (long long)X->p,
             (long long)X->n3);
    const int64_t ns = X->m < X->p ? X->m : X->p;
    int64_t need = o->k;
    if (o->rank_mode == TSVDM_RANK_ENERGY && o->k == 0) need = ns;
    if (need > ns) need = ns;
    if (o->precision != TSVDM_PREC_F64 && need > o->k + o->oversample) need = o->k + o->oversample;
    if (F->kmax < need || F->kmax < 1)
        FAIL(TSVDM_EINVAL, "out->kmax (%lld) < largest possible rank (%lld)", (long long)F->kmax, (long long)need);
    const int32_t want = o->precision == TSVDM_PREC_MIXED ? (X->dtype == TSVDM_C64 ? TSVDM_C64 : TSVDM_F32) : X->dtype;
    if (F->dtype != want) FAIL(TSVDM_EINVAL, "factor dtype %d, expected %d", F->dtype, want);
    if (X->m * X->p * X->n3 > 0 && (!F->U || !F->S || !F->V || !F->ranks))
        FAIL(TSVDM_EINVAL, "factor pointers U, S, V, ranks must be set");
    return TSVDM_OK;
}

tsvdm_status tsvdm_truncate(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, tsvdm_factors *F,
                            void *ws, size_t ws_bytes, void *stream) {
    tsvdm_status st;
    if ((st = check_truncate(X, o)) != TSVDM_OK) return st;
    if ((st = check_truncate_out(X, o, F)) != TSVDM_OK) return st;
    size_t need_ws = tsvdm_truncate_workspace_size(X, o);
    if (need_ws > 0 && (!ws || ws_bytes < need_ws))
        FAIL(TSVDM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need_ws, ws_bytes);
    if (X->n3 == 0) return TSVDM_OK;
    if (o->precision == TSVDM_PREC_F64) return launch_jacobi_truncate(X, o, F, ws, (hipStream_t)stream);
    if (o->precision == TSVDM_PREC_F64_RAND) return launch_f64rand_truncate(X, o, F, ws, (hipStream_t)stream);
    return launch_mixed_truncate(X, o, F, ws, (hipStream_t)stream);
}

tsvdm_status tsvdm_truncate_noalloc(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, tsvdm_factors *F,
                                    void *stream) {
    tsvdm_status st;
    if ((st = check_truncate(X, o)) != TSVDM_OK) return st;
    if (o->precision != TSVDM_PREC_MIXED) FAIL(TSVDM_EUNSUPPORTED, "tsvdm_truncate_noalloc: PREC_MIXED only");
    if (X->dtype != TSVDM_F32) FAIL(TSVDM_EUNSUPPORTED, "tsvdm_truncate_noalloc: a real F32 Xhat only");
    if ((st = check_truncate_out(X, o, F)) != TSVDM_OK) return st;
    if (X->n3 == 0) return TSVDM_OK;
    return launch_mixed_truncate_noalloc(X, o, F, (hipStream_t)stream);
}

size_t tsvdm_noalloc_scratch_bytes(void) { return noalloc_scratch_bytes(); }

// ---------------------------------------------------------------- learned rank
static tsvdm_status check_features(const tsvdm_tensor *X, bool need_data) {
    tsvdm_status st;
    if ((st = check_tensor(X, "Xhat", need_data)) != TSVDM_OK) return st;
    if (!is_dense(*X)) FAIL(TSVDM_EINVAL, "Xhat must be dense (strides 1, m, m*p)");
    if (X->dtype != TSVDM_F32) FAIL(TSVDM_EUNSUPPORTED, "the sketch features need a real F32 Xhat");
    if (X->m < 32 || X->p < 40) FAIL(TSVDM_EUNSUPPORTED, "faces need m >= 32 and p >= 40");
    if (X->m > 65536 || X->p > 65536 || X->n3 > 65535)
        FAIL(TSVDM_EUNSUPPORTED, "face dims up to 65536 and up to 65535 faces");
    return TSVDM_OK;
}

size_t tsvdm_rank_features_workspace_size(const tsvdm_tensor *X) {
    if (check_features(X, false) != TSVDM_OK) return 0;
    return features_workspace(X->m, X->p, X->n3);
}

tsvdm_status tsvdm_rank_features(const tsvdm_tensor *X, const float *omega, uint16_t *features, void *ws,
                                 size_t ws_bytes, void *stream) {
    tsvdm_status st;
    if ((st = check_features(X, true)) != TSVDM_OK) return st;
    if (!omega || !features) FAIL(TSVDM_EINVAL, "omega and features are required");
    const size_t need = features_workspace(X->m, X->p, X->n3);
    if (!ws || ws_bytes < need) FAIL(TSVDM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    return launch_rank_features(X, omega, features, ws, (hipStream_t)stream);
}

size_t tsvdm_truncate_learned_workspace_size(const tsvdm_tensor *X) {
    if (check_features(X, false) != TSVDM_OK) return 0;
    return learned_workspace(X->m, X->p, X->n3);
}

tsvdm_status tsvdm_truncate_learned(const tsvdm_tensor *X, const tsvdm_truncate_opts *o, const uint16_t *w16,
                                    tsvdm_factors *F, int32_t *widths, void *ws, size_t ws_bytes,
                                    void *stream) {
    tsvdm_status st;
    if ((st = check_features(X, true)) != TSVDM_OK) return st;
    if (!o || !w16 || !F || !widths) FAIL(TSVDM_EINVAL, "opts, w16, out and widths are required");
    if (o->rank_mode != TSVDM_RANK_ENERGY || !(o->tau > 0.0 && o->tau < 1.0))
        FAIL(TSVDM_EINVAL, "the learned truncation uses the energy rule with 0 < tau < 1");
    if (!o->omega) FAIL(TSVDM_EINVAL, "omega (p x 40) is required");
    if (o->power_iters < 0 || o->power_iters > 1) FAIL(TSVDM_EUNSUPPORTED, "power_iters must be 0 or 1");
    if (o->max_sweeps < 0) FAIL(TSVDM_EINVAL, "max_sweeps must be >= 0");
    if (F->m != X->m || F->p != X->p || F->nf != X->n3 || F->dtype != TSVDM_F32 || F->kmax < 32)
        FAIL(TSVDM_EINVAL, "factors must be F32 with the dims of Xhat and kmax >= 32");
    if (!F->U || !F->S || !F->V || !F->ranks || !F->cert || !F->fro)
        FAIL(TSVDM_EINVAL, "factor pointers U, S, V, ranks, cert, fro must be set");
    const size_t need = learned_workspace(X->m, X->p, X->n3);
    if (!ws || ws_bytes < need) FAIL(TSVDM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    if (X->n3 == 0) return TSVDM_OK;
    return launch_learned_truncate(X, o, w16, F, widths, ws, (hipStream_t)stream);
}

static tsvdm_status check_apply(const tsvdm_mdesc *M, const tsvdm_factors *F, int64_t ell, int64_t q,
                                int64_t nrhs, int32_t compute) {
    if (!M || !F) FAIL(TSVDM_EINVAL, "M or F is NULL");
    if (M->kind < TSVDM_M_DCT2 || M->kind > TSVDM_M_DENSE) FAIL(TSVDM_EINVAL, "unknown M kind");
    if (M->n3 < 1 || M->n3 > 1024) FAIL(TSVDM_EUNSUPPORTED, "transform length must be in 1..1024");
    if (M->kind == TSVDM_M_DENSE && !M->M) FAIL(TSVDM_EINVAL, "dense M requires M->M");
    if (ell <= 0 || q <= 0 || nrhs < 0) FAIL(TSVDM_EINVAL, "ell, q must be > 0 and nrhs >= 0");
    if (F->p != ell * q) FAIL(TSVDM_EINVAL, "factor p (%lld) != ell*q (%lld)", (long long)F->p, (long long)(ell * q));
    const int64_t nf = M->kind == TSVDM_M_DFT ? M->n3 / 2 + 1 : M->n3;
    if (F->nf != nf) FAIL(TSVDM_EINVAL, "factor nf (%lld) != %lld", (long long)F->nf, (long long)nf);
    if (F->kmax < 1 || F->m < 1) FAIL(TSVDM_EINVAL, "factor m and kmax must be >= 1");
    if (M->kind == TSVDM_M_DFT ? !is_cplx(F->dtype) : !is_real(F->dtype))
        FAIL(TSVDM_EINVAL, "factor dtype does not match the transform (complex iff DFT)");
    if (compute != TSVDM_F32 && compute != TSVDM_F64 && compute != TSVDM_BF16)
        FAIL(TSVDM_EINVAL, "compute must be F32, F64 or BF16");
    if ((compute == TSVDM_F64) != is_double(F->dtype))
        FAIL(TSVDM_EINVAL, "compute precision must match the factor precision");
    if (!F->U || !F->S || !F->V || !F->ranks) FAIL(TSVDM_EINVAL, "factor pointers must be set");
    return TSVDM_OK;
}

size_t tsvdm_apply_workspace_size(const tsvdm_mdesc *M, const tsvdm_factors *F, int64_t ell, int64_t q,
                                  int64_t nrhs, int32_t compute) {
    if (check_apply(M, F, ell, q, nrhs, compute) != TSVDM_OK) return 0;
    return apply_workspace(M, F, ell, q, nrhs, compute);
}

tsvdm_status tsvdm_apply(const tsvdm_mdesc *M, const tsvdm_factors *F, int64_t ell, int64_t q,
                         int64_t nrhs, const void *x, int64_t ldx, void *y, int64_t ldy,
                         int32_t compute, void *ws, size_t ws_bytes, void *stream) {
    tsvdm_status st;
    if ((st = check_apply(M, F, ell, q, nrhs, compute)) != TSVDM_OK) return st;
    if (nrhs == 0) return TSVDM_OK;
    if (!x || !y) FAIL(TSVDM_EINVAL, "x or y is NULL");
    if (ldx < q * M->n3) FAIL(TSVDM_EINVAL, "ldx < q*n3");
    if (ldy < ell * F->m) FAIL(TSVDM_EINVAL, "ldy < ell*m");
    size_t need = apply_workspace(M, F, ell, q, nrhs, compute);
    if (need > 0 && (!ws || ws_bytes < need))
        FAIL(TSVDM_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    return launch_apply(M, F, ell, q, nrhs, x, ldx, y, ldy, compute, ws, (hipStream_t)stream);
}

}  // extern "C"
