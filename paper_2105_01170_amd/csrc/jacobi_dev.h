// Device helpers shared by the FP64 eigensolvers of the truncation kernels:
// refined hardware reciprocals, the round-robin pair ordering, the symmetric
// Schur 2x2 rotation and a cyclic Jacobi eigensolver for a workgroup.
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

__device__ __forceinline__ void rr_pair(int r, int k, int n1, int &a, int &b) {
    if (k == 0) {
        a = r;
        b = n1;
    } else {
        a = r + k;
        if (a >= n1) a -= n1;
        b = r - k;
        if (b < 0) b += n1;
    }
    if (a > b) {
        const int t = a;
        a = b;
        b = t;
    }
}

// a pair rotates when its off-diagonal entry is not negligible, relative to
// the diagonal pair and at the rounding level of the trace
__device__ __forceinline__ bool jneeds(double app, double aqq, double apq, double trace) {
    return apq * apq > 1e-30 * fabs(app * aqq) && fabs(apq) > 1e-15 * trace;
}

// rotation (c, s) of a pair from its entries app, aqq, apq: the smaller of
// the two angles that annihilate apq, by the half-angle formulas
//   h = sqrt(d^2 + e^2),  c = sqrt((1 + |d|/h) / 2),  s = +-|e| / (2 h c)
// (d = aqq - app, e = 2 apq; no cancellation, c^2 + s^2 = 1 up to rounding);
// identity (and false) for a padding pair or a pair that need not rotate.
// Branch free, so that the caller's loads are all issued up front.
__device__ __forceinline__ bool jrot(double app, double aqq, double apq, bool valid, double trace,
                                     double &c, double &s) {
    const bool go = valid && jneeds(app, aqq, apq, trace);
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

// Cyclic Jacobi eigensolver of the symmetric n x n matrix in G (LDS, pitch
// LP+1; only the upper triangle i <= j is read or written) with the
// round-robin ordering: in round r the ne/2 disjoint pairs (ne = n rounded up
// to even) are (r, ne-1) and ((r+k) mod (ne-1), (r-k) mod (ne-1)),
// k = 1..ne/2-1.  Two barriers per round:
//  A. thread k < ne/2 forms the rotation (c, s) of pair k from the current
//     diagonal pair and off-diagonal entry and stores it in cs (one record set
//     per round parity, cs[2][LP/2]); meanwhile the eigenvector columns take
//     the previous round's rotations (Et, transposed: Et[c*(LP+2) + r] =
//     E[r][c], the identity on entry, rows in quads);
//  B. every 2x2 block (pair p rows, pair q columns, p <= q) becomes
//     J_p^T B J_q from its four stored entries and the two rotations.
// Every entry of the upper triangle belongs to exactly one block, so the
// blocks update in place.  The last round's rotations reach the eigenvectors
// after the loop.  rflag[3]: zero on entry.  Before every sweep all pairs are
// tested with the rotation criterion; when none would rotate the iteration
// ends (conv = 1) -- the same result as a sweep without rotations, at the
// cost of one parallel pass.  At most max_sweeps sweeps.  NTH threads take
// part (the whole workgroup).  Returns G (its diagonal is the eigenvalues).
// Ends with a barrier.  G1 is not used (kept for the callers' layout).
template <int LP, int NTH>
__device__ const double *jacobi_eig(double *G, double *G1, double *Et, double2 *cs, int *rflag,
                                    int n, double trace, int max_sweeps, int &conv) {
    constexpr int LD = LP + 1, LDE = LP + 2, NPM = LP / 2;
    constexpr int IPT = (NPM * (NPM + 1) / 2 + (LP / 4) * NPM + NTH - 1) / NTH;  // items per thread
    (void)G1;
    const int tid = threadIdx.x, lane = tid & 63;
    const int ne = n + (n & 1), np = ne / 2, n1 = ne - 1;
    // this thread's items, fixed for all rounds: G block (pp <= qq) or E block
    // (rows 4*i1 .. 4*i1+3, pair i2)
    const int ng = np * (np + 1) / 2, nq = (ne + 3) / 4, nitems = ng + nq * np;
    int ik[IPT], i1[IPT], i2[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
        const int it = tid + u * NTH;
        ik[u] = it < ng ? 0 : it < nitems ? 1 : 2;
        if (ik[u] == 0) {
            int pp = 0, rem = it;
            while (rem >= np - pp) {
                rem -= np - pp;
                ++pp;
            }
            i1[u] = pp;
            i2[u] = pp + rem;
        } else if (ik[u] == 1) {
            i1[u] = (it - ng) / np;
            i2[u] = (it - ng) % np;
        } else {
            i1[u] = i2[u] = 0;
        }
    }
    auto up = [&](int i, int j) -> int { return i <= j ? i * LD + j : j * LD + i; };
    // eigenvector block item: the rotations of round r (record set par)
    auto e_item = [&](int u, int r, int par) {
        int c2, d;
        rr_pair(r, i2[u], n1, c2, d);
        const int r0 = 4 * i1[u];
        double2 *pc = reinterpret_cast<double2 *>(Et + c2 * LDE + r0);
        double2 *pd = reinterpret_cast<double2 *>(Et + d * LDE + r0);
        const double2 rt = cs[par * NPM + i2[u]];
        const double2 x0 = pc[0], x1 = pc[1], y0 = pd[0], y1 = pd[1];
        pc[0] = double2{rt.x * x0.x - rt.y * y0.x, rt.x * x0.y - rt.y * y0.y};
        pc[1] = double2{rt.x * x1.x - rt.y * y1.x, rt.x * x1.y - rt.y * y1.y};
        pd[0] = double2{rt.y * x0.x + rt.x * y0.x, rt.y * x0.y + rt.x * y0.y};
        pd[1] = double2{rt.y * x1.x + rt.x * y1.x, rt.y * x1.y + rt.x * y1.y};
    };

    int sweep = 0, rr = 0, rprev = 0;  // rr counts rounds over all sweeps
    conv = 0;
    for (sweep = 1;; ++sweep) {
        // convergence test over the upper triangle; flag fl, cleared two
        // tests ahead (every thread has read it by the next test's barrier)
        const int fl = sweep % 3;
        {
            bool need = false;
            for (int e = tid; e < n * n; e += NTH) {
                const int i = e / n, j = e - i * n;
                if (i < j) need |= jneeds(G[i * LD + i], G[j * LD + j], G[i * LD + j], trace);
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
            if (tid < np) {
                int a, b;
                rr_pair(r, tid, n1, a, b);
                double c, s;
                jrot(G[a * LD + a], G[b * LD + b], G[a * LD + b], b < n, trace, c, s);
                cs[par * NPM + tid] = double2{c, s};
            }
            if (rr > 0) {
#pragma unroll
                for (int u = 0; u < IPT; ++u)
                    if (ik[u] == 1) e_item(u, rprev, par ^ 1);
            }
            __syncthreads();
            // ---- B: blocks
#pragma unroll
            for (int u = 0; u < IPT; ++u) {
                if (ik[u] == 0) {
                    int a, b, c2, d;
                    rr_pair(r, i1[u], n1, a, b);
                    rr_pair(r, i2[u], n1, c2, d);
                    const double2 rp = cs[par * NPM + i1[u]], rq = cs[par * NPM + i2[u]];
                    const int p00 = up(a, c2), p01 = up(a, d), p10 = up(b, c2), p11 = up(b, d);
                    const double m00 = G[p00], m01 = G[p01], m10 = G[p10], m11 = G[p11];
                    const double cp = rp.x, sp = rp.y, cq = rq.x, sq = rq.y;
                    // rows: (a, b) <- (cp a - sp b, sp a + cp b); then the columns
                    const double t00 = cp * m00 - sp * m10, t01 = cp * m01 - sp * m11;
                    const double t10 = sp * m00 + cp * m10, t11 = sp * m01 + cp * m11;
                    const double n00 = cq * t00 - sq * t01, n01 = sq * t00 + cq * t01;
                    const double n11 = sq * t10 + cq * t11;
                    if (i2[u] != i1[u]) {
                        G[p00] = n00;
                        G[p01] = n01;
                        G[p10] = cq * t10 - sq * t11;
                        G[p11] = n11;
                    } else {  // diagonal block: entries (a,a), (a,b), (b,b)
                        G[p00] = n00;
                        G[p01] = n01;
                        G[p11] = n11;
                    }
                }
            }
            __syncthreads();
            rprev = r;
        }
    }
    // the eigenvectors take the last round's rotations
    if (rr > 0) {
#pragma unroll
        for (int u = 0; u < IPT; ++u)
            if (ik[u] == 1) e_item(u, rprev, (rr - 1) & 1);
    }
    __syncthreads();
    return G;
}

}  // namespace tsvdm
