// FP64 triangle-pair distance with a disjointness certificate and a filtered
// intersection test.  The plain FP64 kernel and the FP64 rescue pass both call
// this code, with floating-point contraction disabled and every fused
// multiply-add written out, so both produce the same bits for the same pair.
#pragma once
#include "sd3_common.h"

#pragma clang fp contract(off)

namespace sd3 {

// Per-triangle data, stored as 30 fields read through a strided reference so
// that the same routine serves LDS tiles (stride K) and private copies
// (stride 1).
enum : int {
    F_V = 0,    // v0 v1 v2 (9)
    F_E = 9,    // e_k = v_{k+1} - v_k (9)
    F_EE = 18,  // |e_k|^2 (3)
    F_IE = 21,  // 1/|e_k|^2, 0 for a zero-length edge (3)
    F_G1 = 24,  // dual basis of (v1 - v0, v2 - v0): beta1 = g1 . (p - v0) (3)
    F_G2 = 27,  // beta2 = g2 . (p - v0) (3)
    F_NTRI64 = 30,
    F_LO = 30,  // FP32 tiles only: triangle bounding box (3 + 3)
    F_HI = 33,
    F_NTRI32 = 36,
};

template <typename T>
struct TriRef {
    T *p;
    int stride;
    __device__ __forceinline__ T operator[](int f) const { return p[f * stride]; }
    __device__ __forceinline__ T &at(int f) const { return p[f * stride]; }
};

__device__ __forceinline__ double dot3d(double ax, double ay, double az, double bx, double by,
                                        double bz) {
    return fma(az, bz, fma(ay, by, ax * bx));
}

__device__ __forceinline__ double clamp01d(double x) { return fmin(fmax(x, 0.0), 1.0); }

// Fill the derived fields from the vertices v (the values of fields 0..8,
// held in registers).
__device__ __forceinline__ void tri_derive64(TriRef<double> t, const double (&v)[9]) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
        int n = (k + 1) % 3;
        double ex = v[3 * n] - v[3 * k], ey = v[3 * n + 1] - v[3 * k + 1],
               ez = v[3 * n + 2] - v[3 * k + 2];
        t.at(F_E + 3 * k) = ex;
        t.at(F_E + 3 * k + 1) = ey;
        t.at(F_E + 3 * k + 2) = ez;
        double ee = dot3d(ex, ey, ez, ex, ey, ez);
        t.at(F_EE + k) = ee;
        t.at(F_IE + k) = ee > 0.0 ? 1.0 / ee : 0.0;
    }
    // E0 = v1 - v0, E1 = v2 - v0
    double E0x = v[3] - v[0], E0y = v[4] - v[1], E0z = v[5] - v[2];
    double E1x = v[6] - v[0], E1y = v[7] - v[1], E1z = v[8] - v[2];
    double a = dot3d(E0x, E0y, E0z, E0x, E0y, E0z);
    double b = dot3d(E0x, E0y, E0z, E1x, E1y, E1z);
    double c = dot3d(E1x, E1y, E1z, E1x, E1y, E1z);
    double nx = E0y * E1z - E0z * E1y, ny = E0z * E1x - E0x * E1z, nz = E0x * E1y - E0y * E1x;
    double nn = dot3d(nx, ny, nz, nx, ny, nz);  // = a c - b^2 without cancellation
    double inn = nn > 0.0 ? 1.0 / nn : 0.0;
    t.at(F_G1 + 0) = (c * E0x - b * E1x) * inn;
    t.at(F_G1 + 1) = (c * E0y - b * E1y) * inn;
    t.at(F_G1 + 2) = (c * E0z - b * E1z) * inn;
    t.at(F_G2 + 0) = (a * E1x - b * E0x) * inn;
    t.at(F_G2 + 1) = (a * E1y - b * E0y) * inn;
    t.at(F_G2 + 2) = (a * E1z - b * E0z) * inn;
}

// The same from v0 v1 v2 as stored in fields 0..8.
__device__ __forceinline__ void tri_prep64(TriRef<double> t) {
    double v[9];
#pragma unroll
    for (int i = 0; i < 9; i++) v[i] = t[F_V + i];
    tri_derive64(t, v);
}

// Filtered orient3d: sign of ((b-a) x (c-a)) . (d-a), or 2 when the FP64
// evaluation cannot prove a strict sign.  Every elementary triple product
// passes through at most 8 roundings (3 differences, 2 products, 1 minor
// difference, 2 sums), so 10 u * (sum of |triple products|) bounds the error.
__device__ __forceinline__ int orient3d_f64(const double *a, const double *b, const double *c,
                                            const double *d) {
    double ux = b[0] - a[0], uy = b[1] - a[1], uz = b[2] - a[2];
    double vx = c[0] - a[0], vy = c[1] - a[1], vz = c[2] - a[2];
    double wx = d[0] - a[0], wy = d[1] - a[1], wz = d[2] - a[2];
    double p1 = uy * vz, p2 = uz * vy, p3 = uz * vx, p4 = ux * vz, p5 = ux * vy, p6 = uy * vx;
    double det = (p1 - p2) * wx + (p3 - p4) * wy + (p5 - p6) * wz;
    double perm = (fabs(p1) + fabs(p2)) * fabs(wx) + (fabs(p3) + fabs(p4)) * fabs(wy) +
                  (fabs(p5) + fabs(p6)) * fabs(wz);
    double bound = 10.0 * U64 * perm;
    if (det > bound) return 1;
    if (det < -bound) return -1;
    return 2;
}

// Closed triangles A, B (9 doubles each): 1 = they meet, 0 = disjoint,
// 2 = undecided (a vertex on or near the other plane, coplanar input, or a
// crossing line passing near a triangle edge -- left to exact arithmetic).
// For non-coplanar triangles with every vertex strictly off the other plane,
// the triangles meet iff an edge of one crosses the other: the crossing point
// of a straddling edge is in the closed triangle iff the line through the
// edge passes on the same side of all three directed triangle edges (Eq. 4's
// u, v >= 0, u + v <= 1 in sign form).
__device__ __noinline__ int tri_tri_filtered64(const double *A, const double *B) {
    int sa[3], sb[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        sa[i] = orient3d_f64(B, B + 3, B + 6, A + 3 * i);
        if (sa[i] == 2) return 2;
    }
    if (sa[0] == sa[1] && sa[1] == sa[2]) return 0;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        sb[i] = orient3d_f64(A, A + 3, A + 6, B + 3 * i);
        if (sb[i] == 2) return 2;
    }
    if (sb[0] == sb[1] && sb[1] == sb[2]) return 0;
    for (int pass = 0; pass < 2; pass++) {
        const double *P = pass ? B : A;
        const double *T = pass ? A : B;
        const int *s = pass ? sb : sa;
        for (int i = 0; i < 3; i++) {
            int j = (i + 1) % 3;
            if (s[i] == s[j]) continue;
            int o0 = orient3d_f64(P + 3 * i, P + 3 * j, T, T + 3);
            int o1 = orient3d_f64(P + 3 * i, P + 3 * j, T + 3, T + 6);
            int o2 = orient3d_f64(P + 3 * i, P + 3 * j, T + 6, T);
            if (o0 == 2 || o1 == 2 || o2 == 2) return 2;
            if (o0 == o1 && o1 == o2) return 1;
        }
    }
    return 0;
}

struct Pair64 {
    double d2;   // squared distance (0 when the pair is certified to meet)
    int status;  // 0 disjoint, 1 meet, 2 undecided (d2 = distance if disjoint)
};

// Distance between closed triangles A and B: the minimum of the 9 edge/edge
// distances (clamped minimisation of |r + s u - t v|^2 over [0,1]^2, Sec.
// 3.2.2 item (i) and Eq. 3) and the 6 vertex/face distances (item (iii):
// foot of the perpendicular inside the face).  Every candidate is the length
// of a vector between two points of the triangles (feasible parameters), all
// vectors formed from coordinate differences first.  Disjointness is then
// certified by the separating plane normal to the best vector; otherwise the
// filtered intersection test decides.
__device__ __forceinline__ Pair64 pair64(TriRef<double> A, TriRef<double> B) {
    double best = __builtin_inf();
    double bx = 0.0, by = 0.0, bz = 0.0;  // best vector, from the B point to the A point
#pragma unroll
    for (int k = 0; k < 3; k++) {
        double ux = A[F_E + 3 * k], uy = A[F_E + 3 * k + 1], uz = A[F_E + 3 * k + 2];
        double a = A[F_EE + k], ia = A[F_IE + k];
#pragma unroll
        for (int l = 0; l < 3; l++) {
            double vx = B[F_E + 3 * l], vy = B[F_E + 3 * l + 1], vz = B[F_E + 3 * l + 2];
            double c = B[F_EE + l], ic = B[F_IE + l];
            double rx = A[F_V + 3 * k] - B[F_V + 3 * l];
            double ry = A[F_V + 3 * k + 1] - B[F_V + 3 * l + 1];
            double rz = A[F_V + 3 * k + 2] - B[F_V + 3 * l + 2];
            double bb = dot3d(ux, uy, uz, vx, vy, vz);
            double d = dot3d(ux, uy, uz, rx, ry, rz);
            double e = dot3d(vx, vy, vz, rx, ry, rz);
            double D = fma(a, c, -(bb * bb));
            // s from the line/line solution, t projected for that s, then s
            // projected again for the clamped t (exactly the clamped
            // minimiser when t is interior; covers zero-length edges)
            double s = 0.0;
            if (D > 0.0) s = clamp01d(fma(bb, e, -(c * d)) / D);
            double t = clamp01d(fma(bb, s, e) * ic);
            s = clamp01d(fma(bb, t, -d) * ia);
            double wx = fma(-t, vx, fma(s, ux, rx));
            double wy = fma(-t, vy, fma(s, uy, ry));
            double wz = fma(-t, vz, fma(s, uz, rz));
            double q = dot3d(wx, wy, wz, wx, wy, wz);
            if (q < best) {
                best = q;
                bx = wx;
                by = wy;
                bz = wz;
            }
        }
    }
#pragma unroll
    for (int side = 0; side < 2; side++) {
        TriRef<double> P = side ? B : A;  // vertex owner
        TriRef<double> F = side ? A : B;  // face owner
        double e0x = F[F_E], e0y = F[F_E + 1], e0z = F[F_E + 2];
        double e2x = F[F_E + 6], e2y = F[F_E + 7], e2z = F[F_E + 8];
#pragma unroll
        for (int i = 0; i < 3; i++) {
            double wx = P[F_V + 3 * i] - F[F_V], wy = P[F_V + 3 * i + 1] - F[F_V + 1],
                   wz = P[F_V + 3 * i + 2] - F[F_V + 2];
            double b1 = dot3d(F[F_G1], F[F_G1 + 1], F[F_G1 + 2], wx, wy, wz);
            double b2 = dot3d(F[F_G2], F[F_G2 + 1], F[F_G2 + 2], wx, wy, wz);
            if (b1 >= 0.0 && b2 >= 0.0 && b1 + b2 <= 1.0) {
                // foot = v0 + b1 (v1 - v0) + b2 (v2 - v0) = v0 + b1 e0 - b2 e2
                double qx = fma(b2, e2x, fma(-b1, e0x, wx));
                double qy = fma(b2, e2y, fma(-b1, e0y, wy));
                double qz = fma(b2, e2z, fma(-b1, e0z, wz));
                double q = dot3d(qx, qy, qz, qx, qy, qz);
                if (q < best) {
                    best = q;
                    double sg = side ? -1.0 : 1.0;
                    bx = sg * qx;
                    by = sg * qy;
                    bz = sg * qz;
                }
            }
        }
    }
    // Certificate: along n = best vector, min over vertex pairs of n.(a_k - b_l)
    // minus its rounding error (< 7 u |n| Mr) > 0 proves a separating plane.
    double sep = __builtin_inf(), mr = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
        for (int l = 0; l < 3; l++) {
            double rx = A[F_V + 3 * k] - B[F_V + 3 * l];
            double ry = A[F_V + 3 * k + 1] - B[F_V + 3 * l + 1];
            double rz = A[F_V + 3 * k + 2] - B[F_V + 3 * l + 2];
            sep = fmin(sep, dot3d(bx, by, bz, rx, ry, rz));
            mr = fmax(mr, fmax(fabs(rx), fmax(fabs(ry), fabs(rz))));
        }
    double cb = 16.0 * SQRT3 * U64 * mr;
    if (best > 0.0 && sep > 0.0 && sep * sep > (cb * cb) * best) return {best, 0};
    double va[9], vb[9];
#pragma unroll
    for (int i = 0; i < 9; i++) {
        va[i] = A[F_V + i];
        vb[i] = B[F_V + i];
    }
    int f = tri_tri_filtered64(va, vb);
    if (f == 1) return {0.0, 1};
    return {best, f == 0 ? 0 : 2};
}

}  // namespace sd3

#pragma clang fp contract(fast)
