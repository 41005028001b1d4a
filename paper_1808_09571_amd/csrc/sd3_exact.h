// Exact orientation signs and the exact closed triangle/triangle intersection
// test, for the rare pairs that the FP64 filter cannot settle.
//
// Exact arithmetic uses floating-point expansions (sums of non-overlapping
// doubles, Priest / Shewchuk): a difference of two doubles is exactly a
// two-term expansion (Two-Diff), a product of two doubles is exactly two
// doubles (Two-Product through a fused multiply-add), and a double is added
// to an expansion exactly by the Grow-Expansion sweep of Two-Sums.  The sign
// of an expansion is the sign of its largest component.  Requires every
// nonzero |coordinate| in [2^-256, 2^256] (no underflow or overflow).
#pragma once
#include "sd3_common.h"

#pragma clang fp contract(off)

namespace sd3 {
namespace ex {

__device__ __forceinline__ void two_sum(double a, double b, double &x, double &y) {
    x = a + b;
    double bv = x - a;
    double av = x - bv;
    y = (a - av) + (b - bv);
}

__device__ __forceinline__ void two_diff(double a, double b, double &x, double &y) {
    x = a - b;
    double bv = a - x;
    double av = x + bv;
    y = (a - av) + (bv - b);
}

__device__ __forceinline__ void two_prod(double a, double b, double &x, double &y) {
    x = a * b;
    y = fma(a, b, -x);
}

// h <- e + b for a non-overlapping expansion e sorted by increasing magnitude
// (h may alias e; capacity n + 1).  Zero components are dropped; a zero sum
// is the single component 0.
__device__ __forceinline__ int grow(double *e, int n, double b) {
    double q = b;
    int m = 0;
    for (int i = 0; i < n; i++) {
        double s, t;
        two_sum(q, e[i], s, t);
        q = s;
        if (t != 0.0) e[m++] = t;
    }
    if (q != 0.0 || m == 0) e[m++] = q;
    return m;
}

// acc <- acc + e * f (all expansions); returns the new length of acc.
__device__ __forceinline__ int add_product(double *acc, int na, const double *e, int ne,
                                           const double *f, int nf) {
    for (int i = 0; i < ne; i++)
        for (int j = 0; j < nf; j++) {
            double x, y;
            two_prod(e[i], f[j], x, y);
            na = grow(acc, na, y);
            na = grow(acc, na, x);
        }
    return na;
}

__device__ __forceinline__ int sign_of(const double *e, int n) {
    double top = e[n - 1];
    return top > 0.0 ? 1 : (top < 0.0 ? -1 : 0);
}

// b - a as an expansion of at most two components
__device__ __forceinline__ int diff2(double b, double a, double *out) {
    double x, y;
    two_diff(b, a, x, y);
    int n = 0;
    if (y != 0.0) out[n++] = y;
    out[n++] = x;
    return n;
}

// exact sign of ((b-a) x (c-a)) . (d-a)
__device__ __noinline__ int orient3d_exact(const double *a, const double *b, const double *c,
                                           const double *d) {
    double u[3][2], v[3][2], w[3][2];
    int nu[3], nv[3], nw[3];
    for (int k = 0; k < 3; k++) {
        nu[k] = diff2(b[k], a[k], u[k]);
        nv[k] = diff2(c[k], a[k], v[k]);
        nw[k] = diff2(d[k], a[k], w[k]);
    }
    double det[216];  // 1 + 3 * (17 * 2 * 2) components at most
    int nd = 1;
    det[0] = 0.0;
    for (int k = 0; k < 3; k++) {
        int j = (k + 1) % 3, l = (k + 2) % 3;
        // minor_k = u_j v_l - u_l v_j
        double m[24];  // 1 + 2 * (2 * 2 * 2) components at most
        int nm = 1;
        m[0] = 0.0;
        nm = add_product(m, nm, u[j], nu[j], v[l], nv[l]);
        double neg[2];
        for (int i = 0; i < nu[l]; i++) neg[i] = -u[l][i];
        nm = add_product(m, nm, neg, nu[l], v[j], nv[j]);
        nd = add_product(det, nd, m, nm, w[k], nw[k]);
    }
    return sign_of(det, nd);
}

// exact sign of (b-a) x (c-a) in the plane
__device__ __noinline__ int orient2d_exact(const double *a, const double *b, const double *c) {
    double u[2][2], v[2][2];
    int nu[2], nv[2];
    for (int k = 0; k < 2; k++) {
        nu[k] = diff2(b[k], a[k], u[k]);
        nv[k] = diff2(c[k], a[k], v[k]);
    }
    double det[24];
    int nd = 1;
    det[0] = 0.0;
    nd = add_product(det, nd, u[0], nu[0], v[1], nv[1]);
    double neg[2];
    for (int i = 0; i < nu[1]; i++) neg[i] = -u[1][i];
    nd = add_product(det, nd, neg, nu[1], v[0], nv[0]);
    return sign_of(det, nd);
}

__device__ __forceinline__ void proj2(const double *p, int k, double *o) {
    o[0] = p[(k + 1) % 3];
    o[1] = p[(k + 2) % 3];
}

// r lies on the closed segment [p, q] given that the three are collinear
__device__ __forceinline__ bool between2(const double *p, const double *q, const double *r) {
    return fmin(p[0], q[0]) <= r[0] && r[0] <= fmax(p[0], q[0]) && fmin(p[1], q[1]) <= r[1] &&
           r[1] <= fmax(p[1], q[1]);
}

__device__ bool seg_seg_2d(const double *p, const double *q, const double *r, const double *s) {
    int o1 = orient2d_exact(p, q, r), o2 = orient2d_exact(p, q, s);
    int o3 = orient2d_exact(r, s, p), o4 = orient2d_exact(r, s, q);
    if (o1 * o2 < 0 && o3 * o4 < 0) return true;
    return (o1 == 0 && between2(p, q, r)) || (o2 == 0 && between2(p, q, s)) ||
           (o3 == 0 && between2(r, s, p)) || (o4 == 0 && between2(r, s, q));
}

// point in a closed non-degenerate 2D triangle
__device__ bool point_in_tri_2d(const double *p, const double *a, const double *b,
                                const double *c) {
    int s0 = orient2d_exact(a, b, p), s1 = orient2d_exact(b, c, p), s2 = orient2d_exact(c, a, p);
    return (s0 >= 0 && s1 >= 0 && s2 >= 0) || (s0 <= 0 && s1 <= 0 && s2 <= 0);
}

// 2D closed segment vs closed non-degenerate triangle
__device__ bool seg_tri_2d(const double *p, const double *q, const double *t) {
    const double *a = t, *b = t + 2, *c = t + 4;
    return seg_seg_2d(p, q, a, b) || seg_seg_2d(p, q, b, c) || seg_seg_2d(p, q, c, a) ||
           point_in_tri_2d(p, a, b, c);
}

// a coordinate axis whose drop keeps triangle T non-degenerate, -1 if none
__device__ int faithful_axis(const double *T) {
    for (int k = 0; k < 3; k++) {
        double a[2], b[2], c[2];
        proj2(T, k, a);
        proj2(T + 3, k, b);
        proj2(T + 6, k, c);
        if (orient2d_exact(a, b, c) != 0) return k;
    }
    return -1;
}

// closed segments in 3D: coplanar, and meeting in all three projections (a
// projection keeps shared points shared, and one of them is injective on the
// common plane or line)
__device__ bool seg_seg_3d(const double *p, const double *q, const double *r, const double *s) {
    if (orient3d_exact(p, q, r, s) != 0) return false;
    for (int k = 0; k < 3; k++) {
        double P[2], Q[2], R[2], S[2];
        proj2(p, k, P);
        proj2(q, k, Q);
        proj2(r, k, R);
        proj2(s, k, S);
        if (!seg_seg_2d(P, Q, R, S)) return false;
    }
    return true;
}

// closed segment vs closed non-degenerate triangle T with faithful axis kT;
// op/oq = orient3d(T, p), orient3d(T, q)
__device__ bool seg_tri_3d(const double *p, const double *q, const double *T, int kT, int op,
                           int oq) {
    if (op * oq > 0) return false;
    if (op == 0 && oq == 0) {
        double P[2], Q[2], t2[6];
        proj2(p, kT, P);
        proj2(q, kT, Q);
        for (int i = 0; i < 3; i++) proj2(T + 3 * i, kT, t2 + 2 * i);
        return seg_tri_2d(P, Q, t2);
    }
    int s0 = orient3d_exact(p, q, T, T + 3);
    int s1 = orient3d_exact(p, q, T + 3, T + 6);
    int s2 = orient3d_exact(p, q, T + 6, T);
    return (s0 >= 0 && s1 >= 0 && s2 >= 0) || (s0 <= 0 && s1 <= 0 && s2 <= 0);
}

// edges of P (degenerate or not) against non-degenerate T
__device__ bool edges_vs_tri(const double *P, const double *T, int kT) {
    int o[3];
    for (int i = 0; i < 3; i++) o[i] = orient3d_exact(T, T + 3, T + 6, P + 3 * i);
    for (int i = 0; i < 3; i++) {
        int j = (i + 1) % 3;
        if (seg_tri_3d(P + 3 * i, P + 3 * j, T, kT, o[i], o[j])) return true;
    }
    return false;
}

// Exact: do closed triangles A and B share a point?  Two closed triangles meet
// iff an edge of one meets the other (a degenerate triangle is the union of
// its edges); coplanar pairs are decided in a projection that keeps B
// non-degenerate.
__device__ bool tri_tri_exact(const double *A, const double *B) {
    int kA = faithful_axis(A), kB = faithful_axis(B);
    if (kA < 0 && kB < 0) {
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++)
                if (seg_seg_3d(A + 3 * i, A + 3 * ((i + 1) % 3), B + 3 * j, B + 3 * ((j + 1) % 3)))
                    return true;
        return false;
    }
    if (kA < 0) return edges_vs_tri(A, B, kB);
    if (kB < 0) return edges_vs_tri(B, A, kA);
    int sa[3];
    for (int i = 0; i < 3; i++) sa[i] = orient3d_exact(B, B + 3, B + 6, A + 3 * i);
    if ((sa[0] > 0 && sa[1] > 0 && sa[2] > 0) || (sa[0] < 0 && sa[1] < 0 && sa[2] < 0))
        return false;
    if (sa[0] == 0 && sa[1] == 0 && sa[2] == 0) {  // coplanar
        double a2[6], b2[6];
        for (int i = 0; i < 3; i++) {
            proj2(A + 3 * i, kB, a2 + 2 * i);
            proj2(B + 3 * i, kB, b2 + 2 * i);
        }
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++)
                if (seg_seg_2d(a2 + 2 * i, a2 + 2 * ((i + 1) % 3), b2 + 2 * j,
                               b2 + 2 * ((j + 1) % 3)))
                    return true;
        return point_in_tri_2d(a2, b2, b2 + 2, b2 + 4) || point_in_tri_2d(b2, a2, a2 + 2, a2 + 4);
    }
    for (int i = 0; i < 3; i++) {
        int j = (i + 1) % 3;
        if (seg_tri_3d(A + 3 * i, A + 3 * j, B, kB, sa[i], sa[j])) return true;
    }
    return edges_vs_tri(B, A, kA);
}

}  // namespace ex
}  // namespace sd3

#pragma clang fp contract(fast)
