// FP32 triangle-pair test with forward error bounds.
//
// The two triangles are FP32 copies expressed in one tile's frame (the other
// tile shifted into it): every real vertex lies within eps_c (a per-tile-pair
// bound) of its FP32 copy, so
// distances between the real triangles and between the copies differ by at
// most eps_c.  On the copies, every candidate is the vector between two
// feasible points (clamped edge parameters, or a face foot whose barycentric
// weights passed the inside test), so its length is an upper bound up to the
// rounding of the vector itself; and the separation of the two triangles
// along the best vector is a lower bound up to the rounding of nine dot
// products.  Neither bound depends on how accurately the clamped parameters
// were computed, so the approximate reciprocal (v_rcp_f32) is used freely.
#pragma once
#include "sd3_pair64.h"

namespace sd3 {

__device__ __forceinline__ float clamp01f(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }

// Fill the derived fields (edges, squared lengths and their reciprocals, face
// dual basis, bounding box) of an FP32 triangle from its vertices v (the
// values of fields 0..8, held in registers).
__device__ __forceinline__ void tri_derive32(TriRef<float> t, const float (&v)[9]) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
        int n = (k + 1) % 3;
        float ex = v[3 * n] - v[3 * k], ey = v[3 * n + 1] - v[3 * k + 1], ez = v[3 * n + 2] - v[3 * k + 2];
        t.at(F_E + 3 * k) = ex;
        t.at(F_E + 3 * k + 1) = ey;
        t.at(F_E + 3 * k + 2) = ez;
        float ee = ex * ex + ey * ey + ez * ez;
        t.at(F_EE + k) = ee;
        t.at(F_IE + k) = ee > 0.0f ? __builtin_amdgcn_rcpf(ee) : 0.0f;
    }
    float E0x = v[3] - v[0], E0y = v[4] - v[1], E0z = v[5] - v[2];
    float E1x = v[6] - v[0], E1y = v[7] - v[1], E1z = v[8] - v[2];
    float a = E0x * E0x + E0y * E0y + E0z * E0z;
    float b = E0x * E1x + E0y * E1y + E0z * E1z;
    float c = E1x * E1x + E1y * E1y + E1z * E1z;
    float nx = E0y * E1z - E0z * E1y, ny = E0z * E1x - E0x * E1z, nz = E0x * E1y - E0y * E1x;
    float nn = nx * nx + ny * ny + nz * nz;
    float inn = nn > 0.0f ? __builtin_amdgcn_rcpf(nn) : 0.0f;
    t.at(F_G1 + 0) = (c * E0x - b * E1x) * inn;
    t.at(F_G1 + 1) = (c * E0y - b * E1y) * inn;
    t.at(F_G1 + 2) = (c * E0z - b * E1z) * inn;
    t.at(F_G2 + 0) = (a * E1x - b * E0x) * inn;
    t.at(F_G2 + 1) = (a * E1y - b * E0y) * inn;
    t.at(F_G2 + 2) = (a * E1z - b * E0z) * inn;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        t.at(F_LO + k) = fminf(v[k], fminf(v[3 + k], v[6 + k]));
        t.at(F_HI + k) = fmaxf(v[k], fmaxf(v[3 + k], v[6 + k]));
    }
}

// The same from fields 0..8 as stored.
__device__ __forceinline__ void tri_prep32(TriRef<float> t) {
    float v[9];
#pragma unroll
    for (int i = 0; i < 9; i++) v[i] = t[F_V + i];
    tri_derive32(t, v);
}

struct Pair32 {
    float d2;  // squared length of the best candidate vector
    float lb;  // certified lower bound of the real pair distance (-inf: may touch)
};

// elb: per-tile-pair bound of the lower-bound error (rounding of the nine
// separation dot products and of the final quotient, plus eps_c).
__device__ __forceinline__ Pair32 pair32(TriRef<float> A, TriRef<float> B, float elb) {
    float best = __builtin_inff();
    float bx = 0.0f, by = 0.0f, bz = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        float ux = A[F_E + 3 * k], uy = A[F_E + 3 * k + 1], uz = A[F_E + 3 * k + 2];
        float a = A[F_EE + k], ia = A[F_IE + k];
#pragma unroll
        for (int l = 0; l < 3; l++) {
            float vx = B[F_E + 3 * l], vy = B[F_E + 3 * l + 1], vz = B[F_E + 3 * l + 2];
            float c = B[F_EE + l], ic = B[F_IE + l];
            float rx = A[F_V + 3 * k] - B[F_V + 3 * l];
            float ry = A[F_V + 3 * k + 1] - B[F_V + 3 * l + 1];
            float rz = A[F_V + 3 * k + 2] - B[F_V + 3 * l + 2];
            float bb = ux * vx + uy * vy + uz * vz;
            float d = ux * rx + uy * ry + uz * rz;
            float e = vx * rx + vy * ry + vz * rz;
            float D = a * c - bb * bb;
            float s = D > 0.0f ? clamp01f((bb * e - c * d) * __builtin_amdgcn_rcpf(D)) : 0.0f;
            float t = clamp01f((bb * s + e) * ic);
            s = clamp01f((bb * t - d) * ia);
            float wx = rx + s * ux - t * vx;
            float wy = ry + s * uy - t * vy;
            float wz = rz + s * uz - t * vz;
            float q = wx * wx + wy * wy + wz * wz;
            bool better = q < best;
            best = better ? q : best;
            bx = better ? wx : bx;
            by = better ? wy : by;
            bz = better ? wz : bz;
        }
    }
#pragma unroll
    for (int side = 0; side < 2; side++) {
        TriRef<float> P = side ? B : A;
        TriRef<float> F = side ? A : B;
        float e0x = F[F_E], e0y = F[F_E + 1], e0z = F[F_E + 2];
        float e2x = F[F_E + 6], e2y = F[F_E + 7], e2z = F[F_E + 8];
        float sg = side ? -1.0f : 1.0f;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            float wx = P[F_V + 3 * i] - F[F_V], wy = P[F_V + 3 * i + 1] - F[F_V + 1],
                  wz = P[F_V + 3 * i + 2] - F[F_V + 2];
            float b1 = F[F_G1] * wx + F[F_G1 + 1] * wy + F[F_G1 + 2] * wz;
            float b2 = F[F_G2] * wx + F[F_G2 + 1] * wy + F[F_G2 + 2] * wz;
            float qx = wx - b1 * e0x + b2 * e2x;
            float qy = wy - b1 * e0y + b2 * e2y;
            float qz = wz - b1 * e0z + b2 * e2z;
            float q = qx * qx + qy * qy + qz * qz;
            bool better = b1 >= 0.0f && b2 >= 0.0f && b1 + b2 <= 1.0f && q < best;
            best = better ? q : best;
            bx = better ? sg * qx : bx;
            by = better ? sg * qy : by;
            bz = better ? sg * qz : bz;
        }
    }
    float sep = __builtin_inff();
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
        for (int l = 0; l < 3; l++) {
            float rx = A[F_V + 3 * k] - B[F_V + 3 * l];
            float ry = A[F_V + 3 * k + 1] - B[F_V + 3 * l + 1];
            float rz = A[F_V + 3 * k + 2] - B[F_V + 3 * l + 2];
            sep = fminf(sep, bx * rx + by * ry + bz * rz);
        }
    float lb = best > 0.0f ? sep * __builtin_amdgcn_rsqf(best) - elb : -__builtin_inff();
    return {best, lb};
}

// Signed volume ((b-a) x (c-a)) . (d-a) in FP32 (error bounded per tile pair).
__device__ __forceinline__ float orient3d_f32(float ax, float ay, float az, float bx, float by,
                                              float bz, float cx, float cy, float cz, float dx,
                                              float dy, float dz) {
    float ux = bx - ax, uy = by - ay, uz = bz - az;
    float vx = cx - ax, vy = cy - ay, vz = cz - az;
    float wx = dx - ax, wy = dy - ay, wz = dz - az;
    return (uy * vz - uz * vy) * wx + (uz * vx - ux * vz) * wy + (ux * vy - uy * vx) * wz;
}

// Certified FP32 intersection classification of a pair whose boxes overlap:
// 0 = certainly disjoint (one triangle strictly on one side of the other's
// plane by more than eo), 1 = certainly meeting (an edge strictly crosses the
// other triangle's plane and the line strictly passes inside all three edges,
// Eq. 4 with margins), 2 = not settled.
// eo bounds the error of every orientation value of the pair: all points lie
// in the pair's bounding box of extent Ms, so each of the 6 elementary triple
// products is at most Ms^3 and passes through at most 8 FP32 roundings
// (48 u Ms^3 < 64 u Ms^3), and moving the 4 points by at most eps each moves
// the determinant by at most 18 eps Ms^2 + O(eps^2 Ms).
__device__ __forceinline__ int isect32(TriRef<float> A, TriRef<float> B, float eps_c) {
    float ms = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; k++)
        ms = fmaxf(ms, fmaxf(A[F_HI + k], B[F_HI + k]) - fminf(A[F_LO + k], B[F_LO + k]));
    ms *= 1.0f + 0x1p-20f;
    const float eo = (24.0f * eps_c * ms * ms + 24.0f * eps_c * eps_c * ms +
                      8.0f * eps_c * eps_c * eps_c + 64.0f * 0x1p-24f * ms * ms * ms) *
                     (1.0f + 0x1p-16f);
    float o[2][3];
#pragma unroll
    for (int side = 0; side < 2; side++) {
        TriRef<float> P = side ? B : A;
        TriRef<float> T = side ? A : B;
#pragma unroll
        for (int i = 0; i < 3; i++)
            o[side][i] = orient3d_f32(T[0], T[1], T[2], T[3], T[4], T[5], T[6], T[7], T[8],
                                      P[3 * i], P[3 * i + 1], P[3 * i + 2]);
        if ((o[side][0] > eo && o[side][1] > eo && o[side][2] > eo) ||
            (o[side][0] < -eo && o[side][1] < -eo && o[side][2] < -eo))
            return 0;
    }
#pragma unroll
    for (int side = 0; side < 2; side++) {
        TriRef<float> P = side ? B : A;
        TriRef<float> T = side ? A : B;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            int j = (i + 1) % 3;
            float oi = o[side][i], oj = o[side][j];
            if (!((oi > eo && oj < -eo) || (oi < -eo && oj > eo))) continue;
            float px = P[3 * i], py = P[3 * i + 1], pz = P[3 * i + 2];
            float qx = P[3 * j], qy = P[3 * j + 1], qz = P[3 * j + 2];
            float s0 = orient3d_f32(px, py, pz, qx, qy, qz, T[0], T[1], T[2], T[3], T[4], T[5]);
            float s1 = orient3d_f32(px, py, pz, qx, qy, qz, T[3], T[4], T[5], T[6], T[7], T[8]);
            float s2 = orient3d_f32(px, py, pz, qx, qy, qz, T[6], T[7], T[8], T[0], T[1], T[2]);
            if ((s0 > eo && s1 > eo && s2 > eo) || (s0 < -eo && s1 < -eo && s2 < -eo)) return 1;
        }
    }
    return 2;
}

}  // namespace sd3
