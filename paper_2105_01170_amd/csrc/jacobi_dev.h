// Device helpers shared by the FP64 eigensolvers of the truncation kernels:
// refined hardware reciprocals, the symmetric Schur 2x2 rotation, the
// round-robin slot permutation and a cyclic Jacobi eigensolver for a
// workgroup.
#pragma once

#include "common.h"

namespace tsvdm {

// 1/a for a > 0 normal: hardware reciprocal refined by two Newton steps
// (error within an ulp or two; used for Cholesky multipliers, where that is
// below the rounding of the update itself)
__device__ __forceinline__ double recip(double a) {
    double r = __builtin_amdgcn_rcp(a);
    double e = fma(-a, r, 1.0);
    r = fma(r, e, r);
    e = fma(-a, r, 1.0);
    return fma(r, e, r);
}

// 1/sqrt(a) for a > 0 normal: hardware estimate refined by two Newton steps
__device__ __forceinline__ double rsqrt_nr(double a) {
    double y = __builtin_amdgcn_rsq(a);
    double e = fma(-a * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-a * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// a pair rotates when its off-diagonal entry is not negligible: relative to
// the diagonal pair (1e-15) and above the absolute threshold atol (the
// caller's choice, a multiple of the trace)
__device__ __forceinline__ bool jneeds(double app, double aqq, double apq, double atol) {
    return apq * apq > 1e-30 * fabs(app * aqq) && fabs(apq) > atol;
}

// rotation (c, s) of a pair from its entries app, aqq, apq: the smaller of
// the two angles that annihilate apq, by the half-angle formulas
//   h = sqrt(d^2 + e^2),  c = sqrt((1 + |d|/h) / 2),  s = +-|e| / (2 h c)
// (d = aqq - app, e = 2 apq; no cancellation, c^2 + s^2 = 1 up to rounding);
// identity (and false) for a padding pair or a pair that need not rotate.
// Branch free, so that the caller's loads are all issued up front.
__device__ __forceinline__ bool jrot(double app, double aqq, double apq, bool valid, double atol,
                                     double &c, double &s) {
    const bool go = valid && jneeds(app, aqq, apq, atol);
    const double d = aqq - app, e = 2.0 * apq;
    const double y = rsqrt_nr(go ? fma(d, d, e * e) : 1.0);  // 1 / h
    const double c2 = fma(0.5 * fabs(d), y, 0.5);          // cos^2 of the angle
    const double z = rsqrt_nr(c2);                          // 1 / c
    const double sa = 0.5 * fabs(e) * y * z;
    const bool pos = d == 0.0 || ((d > 0.0) == (e > 0.0));
    c = go ? c2 * z : 1.0;
    s = go ? (pos ? sa : -sa) : 0.0;
    return go;
}

// Pitch (doubles) of the matrix and eigenvector buffers of jacobi_eig: even,
// so that rows of a pair of slots start 16-byte aligned.
template <int LP>
constexpr int jacobi_ld() {
    return LP + 2;
}

// Slot permutation of the round-robin (circle) ordering on ne = 2h slots,
// pair k in slots (2k, 2k+1): slot 0 stays; the top row 2, 4, .., 2h-2 moves
// one place right, its last entry to 2h-1; the bottom row 2h-1, .., 3, 1
// moves one place left, slot 1 to slot 2.  After ne-1 rounds every pair of
// entries has shared a slot pair once.
__device__ __forceinline__ int rr_next(int s, int h) {
    if (s == 0 || h == 1) return s;
    const int k = s >> 1;
    if ((s & 1) == 0) return k <= h - 2 ? s + 2 : 2 * h - 1;
    return k >= 1 ? s - 2 : 2;
}

// Cyclic Jacobi eigensolver of the symmetric n x n matrix in G0 (LDS, pitch
// jacobi_ld<LP>(), upper triangle i <= j used) with the round-robin ordering,
// run on slots: in every round pair k occupies slots (2k, 2k+1), and after the
// round every entry moves to the slots rr_next gives, which is the same
// permutation in every round.  So every work item reads and writes fixed
// addresses for the whole solve.  Two barriers per round:
//  A. thread k < ne/2 (ne = n rounded up to even) forms the rotation (c, s)
//     of pair k from its diagonal block and stores it in cs (one record set
//     per round parity, cs[2][LP/2]); meanwhile the eigenvector columns take
//     the previous round's rotations and move to their next slots (E0/E1
//     transposed, E[c * LDE + r] = entry r of the eigenvector in slot c, the
//     identity on the first n slots of E0 on entry);
//  B. every 2x2 block (pair p rows, pair q columns, p <= q) of the current
//     buffer becomes J_p^T B J_q and is written to its next slots in the
//     other buffer.
// The last round's rotations reach the eigenvectors after the loop.  Before
// every sweep all pairs are tested with the rotation criterion (jneeds, with
// the absolute threshold atol); when none would rotate the iteration ends
// (conv = 1).  At most max_sweeps sweeps.
// rflag[3]: zero on entry.  Entries past ne of G0 and E0 zero; G1, E1 any.
// NTH threads take part (the whole workgroup); ends with a barrier.  On
// return Gout holds the final matrix (its diagonal the eigenvalues, in slot
// order) and Eout the eigenvectors in the same slot order; for odd n, dslot
// is the slot of the zero padding entry (its eigenvalue and eigenvector are
// zero), else -1.  The n real eigenpairs are in the other ne slots.
template <int LP, int NTH>
__device__ void jacobi_eig(double *G0, double *G1, double *E0, double *E1, double2 *cs, int *rflag, int n,
                           double atol, int max_sweeps, int &conv, const double *&Gout, const double *&Eout,
                           int &dslot) {
    constexpr int LD = jacobi_ld<LP>(), LDE = jacobi_ld<LP>(), NPM = LP / 2;
    constexpr int IPT = (NPM * (NPM + 1) / 2 + (LP / 4) * NPM + NTH - 1) / NTH;  // items per thread
    const int tid = threadIdx.x, lane = tid & 63;
    const int ne = n + (n & 1), h = ne / 2, n1 = ne - 1;
    auto up = [&](int i, int j) -> int { return i <= j ? i * LD + j : j * LD + i; };
    // this thread's items, fixed for all rounds: G block (pp <= qq) or E block
    // (rows 4*i1 .. 4*i1+3, pair i2), with their source and destination offsets
    const int ng = h * (h + 1) / 2, nq = (ne + 3) / 4, nitems = ng + nq * h;
    int ik[IPT], i1[IPT], i2[IPT], src[IPT], d0[IPT], d1[IPT], d2[IPT], d3[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
        const int it = tid + u * NTH;
        ik[u] = it < ng ? 0 : it < nitems ? 1 : 2;
        i1[u] = i2[u] = src[u] = d0[u] = d1[u] = d2[u] = d3[u] = 0;
        if (ik[u] == 0) {
            int pp = 0, rem = it;
            while (rem >= h - pp) {
                rem -= h - pp;
                ++pp;
            }
            const int qq = pp + rem;
            i1[u] = pp;
            i2[u] = qq;
            src[u] = 2 * pp * LD + 2 * qq;
            const int a = rr_next(2 * pp, h), b = rr_next(2 * pp + 1, h);
            const int c = rr_next(2 * qq, h), d = rr_next(2 * qq + 1, h);
            d0[u] = up(a, c);
            d1[u] = up(a, d);
            d2[u] = up(b, c);
            d3[u] = up(b, d);
        } else if (ik[u] == 1) {
            const int k = (it - ng) % h, r0 = 4 * ((it - ng) / h);
            i1[u] = r0;
            i2[u] = k;
            src[u] = 2 * k * LDE + r0;
            d0[u] = rr_next(2 * k, h) * LDE + r0;
            d1[u] = rr_next(2 * k + 1, h) * LDE + r0;
        }
    }
    double *Gc = G0, *Gn = G1, *Ec = E0, *En = E1;
    // eigenvector block item: the rotations of record set par
    auto e_item = [&](int u, int par) {
        const double2 *pc = reinterpret_cast<const double2 *>(Ec + src[u]);
        const double2 *pd = reinterpret_cast<const double2 *>(Ec + src[u] + LDE);
        const double2 rt = cs[par * NPM + i2[u]];
        const double2 x0 = pc[0], x1 = pc[1], y0 = pd[0], y1 = pd[1];
        double2 *qc = reinterpret_cast<double2 *>(En + d0[u]);
        double2 *qd = reinterpret_cast<double2 *>(En + d1[u]);
        qc[0] = double2{rt.x * x0.x - rt.y * y0.x, rt.x * x0.y - rt.y * y0.y};
        qc[1] = double2{rt.x * x1.x - rt.y * y1.x, rt.x * x1.y - rt.y * y1.y};
        qd[0] = double2{rt.y * x0.x + rt.x * y0.x, rt.y * x0.y + rt.x * y0.y};
        qd[1] = double2{rt.y * x1.x + rt.x * y1.x, rt.y * x1.y + rt.x * y1.y};
    };

    int rr = 0;  // rounds over all sweeps
    conv = 0;
    for (int sweep = 1;; ++sweep) {
        // convergence test over the upper triangle of the slots; flag fl,
        // cleared two tests ahead (every thread has read it by then)
        const int fl = sweep % 3;
        {
            bool need = false;
            for (int e = tid; e < ne * ne; e += NTH) {
                const int i = e / ne, j = e - i * ne;
                if (i < j) need |= jneeds(Gc[i * LD + i], Gc[j * LD + j], Gc[i * LD + j], atol);
            }
            if (__any(need) && lane == 0) rflag[fl] = 1;
            __syncthreads();
            if (tid == 0) rflag[(sweep + 2) % 3] = 0;
            if (rflag[fl] == 0) {
                conv = 1;
                break;
            }
        }
        if (sweep > max_sweeps) break;
        for (int r = 0; r < n1; ++r, ++rr) {
            const int par = rr & 1;
            // ---- A: rotations; eigenvectors of the previous round
            if (tid < h) {
                const double2 g = *reinterpret_cast<const double2 *>(Gc + 2 * tid * (LD + 1));
                const double aqq = Gc[(2 * tid + 1) * (LD + 1)];
                double c, s;
                jrot(g.x, aqq, g.y, true, atol, c, s);
                cs[par * NPM + tid] = double2{c, s};
            }
            if (rr > 0) {
#pragma unroll
                for (int u = 0; u < IPT; ++u)
                    if (ik[u] == 1) e_item(u, par ^ 1);
            }
            __syncthreads();
            if (rr > 0) {
                double *t = Ec;
                Ec = En;
                En = t;
            }
            // ---- B: blocks to their next slots
#pragma unroll
            for (int u = 0; u < IPT; ++u) {
                if (ik[u] != 0) continue;
                const double2 r0 = *reinterpret_cast<const double2 *>(Gc + src[u]);
                const double2 r1 = *reinterpret_cast<const double2 *>(Gc + src[u] + LD);
                const double2 rp = cs[par * NPM + i1[u]], rq = cs[par * NPM + i2[u]];
                const bool dg = i1[u] == i2[u];
                // diagonal block: (b, a) is not stored; it equals (a, b)
                const double m00 = r0.x, m01 = r0.y, m10 = dg ? r0.y : r1.x, m11 = r1.y;
                const double cp = rp.x, sp = rp.y, cq = rq.x, sq = rq.y;
                // rows: (a, b) <- (cp a - sp b, sp a + cp b); then the columns
                const double t00 = cp * m00 - sp * m10, t01 = cp * m01 - sp * m11;
                const double t10 = sp * m00 + cp * m10, t11 = sp * m01 + cp * m11;
                Gn[d0[u]] = cq * t00 - sq * t01;
                Gn[d1[u]] = sq * t00 + cq * t01;
                if (!dg) Gn[d2[u]] = cq * t10 - sq * t11;
                Gn[d3[u]] = sq * t10 + cq * t11;
            }
            __syncthreads();
            double *t = Gc;
            Gc = Gn;
            Gn = t;
        }
    }
    // the eigenvectors take the last round's rotations
    if (rr > 0) {
#pragma unroll
        for (int u = 0; u < IPT; ++u)
            if (ik[u] == 1) e_item(u, (rr - 1) & 1);
        __syncthreads();
        Ec = En;
    }
    __syncthreads();
    Gout = Gc;
    Eout = Ec;
    // the padding entry starts in slot ne-1 and moves once per round; the
    // permutation has period ne-1 on the moving slots
    dslot = -1;
    if (n & 1) {
        int sl = ne - 1;
        for (int k = 0, nr = n1 > 0 ? rr % n1 : 0; k < nr; ++k) sl = rr_next(sl, h);
        dslot = sl;
    }
}

// Slot of the j-th real eigenpair (j < n) given the padding slot of jacobi_eig.
__device__ __forceinline__ int jacobi_slot(int j, int dslot) { return dslot >= 0 && j >= dslot ? j + 1 : j; }

// ---------------------------------------------------------------- Hermitian
// Complex arithmetic on (re, im) pairs.
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// conj(a) * b
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
    return double2{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}

// Rotation of the Hermitian pair [[app, apq], [conj(apq), aqq]]: with
// w = apq / |apq| the phase diag(1, conj(w)) turns the pair into the real
// symmetric [[app, |apq|], [|apq|, aqq]], and the real rotation (c, s) of
// jrot annihilates that; the unitary is U = diag(1, conj(w)) [[c, s], [-s, c]].
// Same test as jneeds on |apq|, in squares.  Identity (c = 1, s = 0, w = 1)
// when the pair need not rotate.  Branch free.
__device__ __forceinline__ bool jrot_c(double app, double aqq, double2 apq, double atol, double &c, double &s,
                                       double2 &w) {
    const double a2 = apq.x * apq.x + apq.y * apq.y;
    const bool go = a2 > 1e-30 * fabs(app * aqq) && a2 > atol * atol;
    const double ih = rsqrt_nr(go ? a2 : 1.0);  // 1 / |apq|
    const double h = a2 * ih;                   // |apq|
    w = go ? double2{apq.x * ih, apq.y * ih} : double2{1.0, 0.0};
    const double d = aqq - app, e = 2.0 * h;
    const double y = rsqrt_nr(go ? fma(d, d, e * e) : 1.0);
    const double c2 = fma(0.5 * fabs(d), y, 0.5);
    const double z = rsqrt_nr(c2);
    const double sa = 0.5 * e * y * z;
    c = go ? c2 * z : 1.0;
    s = go ? (d >= 0.0 ? sa : -sa) : 0.0;
    return go;
}

// Pitch (complex entries) of the buffers of jacobi_eig_c.
template <int LP>
constexpr int jacobi_ldc() {
    return LP + 1;
}

// Cyclic Jacobi eigensolver of the Hermitian n x n matrix in G0 (LDS, complex
// entries, pitch jacobi_ldc<LP>(), upper triangle i <= j used, the diagonal
// real), on the slot scheme of jacobi_eig: the same round-robin ordering,
// the same two barriers per round and fixed addresses for every work item.
// A pair's record is (c, s) in cs and the phase w in ph; block (P rows, Q
// columns) becomes U_P^H B U_Q.  Because only the upper triangle is stored,
// an entry whose destination slots (i, j) have i > j is stored conjugated at
// (j, i); the lower entry of a diagonal block is the conjugate of its upper
// one.  E0/E1 hold the eigenvectors transposed (E[c * LDC + r] = entry r of
// the eigenvector in slot c), the identity on the first n slots of E0 on
// entry; entries past ne of G0 and E0 zero.  Returns like jacobi_eig: Gout's
// diagonal (real parts) the eigenvalues in slot order, Eout the eigenvectors,
// dslot the padding slot for odd n.  Ends with a barrier.
template <int LP, int NTH>
__device__ void jacobi_eig_c(double2 *G0, double2 *G1, double2 *E0, double2 *E1, double2 *cs, double2 *ph,
                             int *rflag, int n, double atol, int max_sweeps, int &conv, const double2 *&Gout,
                             const double2 *&Eout, int &dslot) {
    constexpr int LD = jacobi_ldc<LP>(), NPM = LP / 2;
    constexpr int IPT = (NPM * (NPM + 1) / 2 + (LP / 4) * NPM + NTH - 1) / NTH;
    const int tid = threadIdx.x, lane = tid & 63;
    const int ne = n + (n & 1), h = ne / 2, n1 = ne - 1;
    // destination of slot entry (i, j): its upper position, and whether the
    // value goes there conjugated
    auto up = [&](int i, int j, int &cj) -> int {
        cj = i > j;
        return i <= j ? i * LD + j : j * LD + i;
    };
    const int ng = h * (h + 1) / 2, nq = (ne + 3) / 4, nitems = ng + nq * h;
    int ik[IPT], i1[IPT], i2[IPT], src[IPT], d0[IPT], d1[IPT], d2[IPT], d3[IPT], cjm[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
        const int it = tid + u * NTH;
        ik[u] = it < ng ? 0 : it < nitems ? 1 : 2;
        i1[u] = i2[u] = src[u] = d0[u] = d1[u] = d2[u] = d3[u] = cjm[u] = 0;
        if (ik[u] == 0) {
            int pp = 0, rem = it;
            while (rem >= h - pp) {
                rem -= h - pp;
                ++pp;
            }
            const int qq = pp + rem;
            i1[u] = pp;
            i2[u] = qq;
            src[u] = 2 * pp * LD + 2 * qq;
            const int a = rr_next(2 * pp, h), b = rr_next(2 * pp + 1, h);
            const int c = rr_next(2 * qq, h), d = rr_next(2 * qq + 1, h);
            int c0, c1, c2, c3;
            d0[u] = up(a, c, c0);
            d1[u] = up(a, d, c1);
            d2[u] = up(b, c, c2);
            d3[u] = up(b, d, c3);
            cjm[u] = c0 | (c1 << 1) | (c2 << 2) | (c3 << 3);
        } else if (ik[u] == 1) {
            const int k = (it - ng) % h, r0 = 4 * ((it - ng) / h);
            i1[u] = r0;
            i2[u] = k;
            src[u] = 2 * k * LD + r0;
            d0[u] = rr_next(2 * k, h) * LD + r0;
            d1[u] = rr_next(2 * k + 1, h) * LD + r0;
        }
    }
    double2 *Gc = G0, *Gn = G1, *Ec = E0, *En = E1;
    // eigenvector block item: E_p <- c E_p - s conj(w) E_q, E_q <- s E_p + c conj(w) E_q
    auto e_item = [&](int u, int par) {
        const double2 rt = cs[par * NPM + i2[u]], w = ph[par * NPM + i2[u]];
        double2 x[4], y[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            x[v] = Ec[src[u] + v];
            y[v] = Ec[src[u] + LD + v];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double2 wy = cmulc(w, y[v]);
            En[d0[u] + v] = double2{rt.x * x[v].x - rt.y * wy.x, rt.x * x[v].y - rt.y * wy.y};
            En[d1[u] + v] = double2{rt.y * x[v].x + rt.x * wy.x, rt.y * x[v].y + rt.x * wy.y};
        }
    };
    auto put = [&](int d, int cj, double2 v) { Gn[d] = cj ? double2{v.x, -v.y} : v; };

    int rr = 0;
    conv = 0;
    for (int sweep = 1;; ++sweep) {
        const int fl = sweep % 3;
        {
            bool need = false;
            for (int e = tid; e < ne * ne; e += NTH) {
                const int i = e / ne, j = e - i * ne;
                if (i < j) {
                    const double2 g = Gc[i * LD + j];
                    const double a2 = g.x * g.x + g.y * g.y, app = Gc[i * LD + i].x, aqq = Gc[j * LD + j].x;
                    need |= a2 > 1e-30 * fabs(app * aqq) && a2 > atol * atol;
                }
            }
            if (__any(need) && lane == 0) rflag[fl] = 1;
            __syncthreads();
            if (tid == 0) rflag[(sweep + 2) % 3] = 0;
            if (rflag[fl] == 0) {
                conv = 1;
                break;
            }
        }
        if (sweep > max_sweeps) break;
        for (int r = 0; r < n1; ++r, ++rr) {
            const int par = rr & 1;
            if (tid < h) {
                const double app = Gc[2 * tid * (LD + 1)].x, aqq = Gc[(2 * tid + 1) * (LD + 1)].x;
                const double2 apq = Gc[2 * tid * (LD + 1) + 1];
                double c, s;
                double2 w;
                jrot_c(app, aqq, apq, atol, c, s, w);
                cs[par * NPM + tid] = double2{c, s};
                ph[par * NPM + tid] = w;
            }
            if (rr > 0) {
#pragma unroll
                for (int u = 0; u < IPT; ++u)
                    if (ik[u] == 1) e_item(u, par ^ 1);
            }
            __syncthreads();
            if (rr > 0) {
                double2 *t = Ec;
                Ec = En;
                En = t;
            }
#pragma unroll
            for (int u = 0; u < IPT; ++u) {
                if (ik[u] != 0) continue;
                const bool dg = i1[u] == i2[u];
                const double2 m00 = Gc[src[u]], m01 = Gc[src[u] + 1];
                const double2 m10 = dg ? double2{m01.x, -m01.y} : Gc[src[u] + LD], m11 = Gc[src[u] + LD + 1];
                const double2 rp = cs[par * NPM + i1[u]], rq = cs[par * NPM + i2[u]];
                const double2 wp = ph[par * NPM + i1[u]], wq = ph[par * NPM + i2[u]];
                const double cp = rp.x, sp = rp.y, cq = rq.x, sq = rq.y;
                // rows: (r0, r1) <- (cp r0 - sp w_p r1, sp r0 + cp w_p r1)
                const double2 u0 = cmul(wp, m10), u1 = cmul(wp, m11);
                const double2 t00{cp * m00.x - sp * u0.x, cp * m00.y - sp * u0.y};
                const double2 t01{cp * m01.x - sp * u1.x, cp * m01.y - sp * u1.y};
                const double2 t10{sp * m00.x + cp * u0.x, sp * m00.y + cp * u0.y};
                const double2 t11{sp * m01.x + cp * u1.x, sp * m01.y + cp * u1.y};
                // columns: (k0, k1) <- (cq k0 - sq conj(w_q) k1, sq k0 + cq conj(w_q) k1)
                const double2 v0 = cmulc(wq, t01), v1 = cmulc(wq, t11);
                double2 b00{cq * t00.x - sq * v0.x, cq * t00.y - sq * v0.y};
                const double2 b01{sq * t00.x + cq * v0.x, sq * t00.y + cq * v0.y};
                const double2 b10{cq * t10.x - sq * v1.x, cq * t10.y - sq * v1.y};
                double2 b11{sq * t10.x + cq * v1.x, sq * t10.y + cq * v1.y};
                if (dg) {  // diagonal entries of a Hermitian matrix are real
                    b00.y = 0.0;
                    b11.y = 0.0;
                }
                const int cj = cjm[u];
                put(d0[u], cj & 1, b00);
                put(d1[u], (cj >> 1) & 1, b01);
                if (!dg) put(d2[u], (cj >> 2) & 1, b10);
                put(d3[u], (cj >> 3) & 1, b11);
            }
            __syncthreads();
            double2 *t = Gc;
            Gc = Gn;
            Gn = t;
        }
    }
    if (rr > 0) {
#pragma unroll
        for (int u = 0; u < IPT; ++u)
            if (ik[u] == 1) e_item(u, (rr - 1) & 1);
        __syncthreads();
        Ec = En;
    }
    __syncthreads();
    Gout = Gc;
    Eout = Ec;
    dslot = -1;
    if (n & 1) {
        int sl = ne - 1;
        for (int k = 0, nr = n1 > 0 ? rr % n1 : 0; k < nr; ++k) sl = rr_next(sl, h);
        dslot = sl;
    }
}

}  // namespace tsvdm
