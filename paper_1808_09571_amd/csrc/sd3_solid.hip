// Solid semantics (opts.semantics = SD3_SOLID): each row's mesh is read as
// the boundary of a solid (the paper's ore bodies are closed meshes, Sec. 4),
// so a mesh nested inside the other's solid meets it, at distance 0.  For
// surfaces that do not meet, the solids meet iff a point of one surface lies
// inside the other solid; one vertex per side decides it for connected closed
// meshes.
//
// Point in solid by ray parity, exactly: the segment from the point p to a far
// point q crosses the closed mesh an odd number of times iff p is inside.  A
// crossing with triangle (a, b, c) is decided by exact orientation signs
// (FP64 filter, then expansions): p and q strictly on opposite sides of the
// plane, and the line pq strictly on one side of all three directed edges
// (Eq. 4's u, v >= 0, u + v <= 1 with every inequality strict).  A zero sign
// (the segment through an edge or a vertex, or q on a plane) makes the
// direction degenerate: the query is run again with the next direction of a
// fixed list.  p on a plane is no crossing unless p lies in the closed
// triangle (then the surfaces meet and the row is already settled).
#include <algorithm>

#include "sd3_kernels.h"
#include "sd3_pair64.h"
#include "sd3_exact.h"

namespace sd3 {

// ray directions tried in turn (the first along +z, the others generic)
__constant__ double kSolidDir[SOLID_DIRS][3] = {
    {0.0, 0.0, 1.0},
    {0.3713906763541037, 0.5570860145311556, 0.7427813527082074},
    {-0.6139406135149205, 0.2364129372436342, 0.7531236829418232},
    {0.1118033988749895, -0.8944271909999159, 0.4330127018922193},
    {-0.2672612419124244, -0.5345224838248488, -0.8017837257372732},
    {0.7071067811865476, 0.1414213562373095, -0.6928203230275509},
    {-0.8660254037844386, 0.4082482904638630, 0.2886751345948129},
    {0.5298129428260175, -0.2119251771304070, -0.8212100613803272},
};

__device__ __forceinline__ int orient_sign(const double *a, const double *b, const double *c,
                                           const double *d) {
    const int f = orient3d_f64(a, b, c, d);
    return f != 2 ? f : ex::orient3d_exact(a, b, c, d);
}

// zero-area triangle, exactly: (b - a) x (c - a) = 0 in every coordinate plane
__device__ bool solid_degenerate(const double *a, const double *b, const double *c) {
    for (int k = 0; k < 3; k++) {
        double pa[2], pb[2], pc[2];
        ex::proj2(a, k, pa);
        ex::proj2(b, k, pb);
        ex::proj2(c, k, pc);
        if (ex::orient2d_exact(pa, pb, pc) != 0) return false;
    }
    return true;
}

// 0: no crossing, 1: crossing, 2: degenerate direction, 4: p in the triangle
__device__ int ray_cross(const double *p, const double *q, const double *a, const double *b,
                         const double *c) {
    const int sq = orient_sign(a, b, c, q);
    const int sp = orient_sign(a, b, c, p);
    if (sq == 0) return solid_degenerate(a, b, c) ? 0 : 2;
    if (sp == 0) {
        double P[9] = {p[0], p[1], p[2], p[0], p[1], p[2], p[0], p[1], p[2]};
        double T[9] = {a[0], a[1], a[2], b[0], b[1], b[2], c[0], c[1], c[2]};
        return ex::tri_tri_exact(P, T) ? 4 : 0;
    }
    if (sp == sq) return 0;
    const int o1 = orient_sign(p, q, a, b);
    const int o2 = orient_sign(p, q, b, c);
    const int o3 = orient_sign(p, q, c, a);
    if (o1 == 0 || o2 == 0 || o3 == 0) return 2;
    return (o1 == o2 && o2 == o3) ? 1 : 0;
}

__device__ __forceinline__ void solid_vertex(const double *X, int64_t nvr, const int32_t *tri, int64_t t,
                                             int k, double *out) {
    const int32_t v = tri[3 * t + k];
    const int64_t vi = (v >= 0 && (int64_t)v < nvr) ? v : 0;
    for (int c = 0; c < 3; c++) out[c] = X[3 * vi + c];
}

// One block per query (row g, side s: the first vertex of side s's row
// against side 1 - s's triangles; direction dir[query]).  res bits: 1 inside
// (odd crossings), 2 degenerate direction, 4 on the other surface.
__global__ __launch_bounds__(256) void k_inside(SolidSide A, SolidSide B, const RowState *rows,
                                                const int32_t *queries, int64_t nq, const uint8_t *dir,
                                                uint8_t *res) {
    __shared__ double red[6][4];
    __shared__ int flags[4];
    for (int64_t qi = blockIdx.x; qi < nq; qi += gridDim.x) {
        const int32_t code = queries[qi];
        const int64_t g = code >> 1;
        const int side = code & 1;
        const SolidSide &P = side ? B : A;  // the point's side
        const SolidSide &M = side ? A : B;  // the solid's side
        const int64_t pt0 = P.t_off[g], pt1 = P.t_off[g + 1];
        const int64_t mt0 = M.t_off[g], mt1 = M.t_off[g + 1];
        if (rows[g].hit || pt1 == pt0 || mt1 == mt0) {
            if (threadIdx.x == 0) res[code] = 0;
            continue;
        }
        double p[3];
        solid_vertex(P.xyz + 3 * P.v_off[g], P.v_off[g + 1] - P.v_off[g], P.tri, pt0, 0, p);
        const double *X = M.xyz + 3 * M.v_off[g];
        const int64_t nvr = M.v_off[g + 1] - M.v_off[g];
        // the solid's box, then a far point beyond it along the direction
        double lo[3] = {p[0], p[1], p[2]}, hi[3] = {p[0], p[1], p[2]};
        for (int64_t t = mt0 + threadIdx.x; t < mt1; t += blockDim.x)
            for (int k = 0; k < 3; k++) {
                double v[3];
                solid_vertex(X, nvr, M.tri, t, k, v);
                for (int c = 0; c < 3; c++) {
                    lo[c] = fmin(lo[c], v[c]);
                    hi[c] = fmax(hi[c], v[c]);
                }
            }
        for (int c = 0; c < 3; c++) {
            lo[c] = wave_min(lo[c]);
            hi[c] = wave_max(hi[c]);
        }
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0)
            for (int c = 0; c < 3; c++) {
                red[c][w] = lo[c];
                red[3 + c][w] = hi[c];
            }
        if (threadIdx.x < 4) flags[threadIdx.x] = 0;
        __syncthreads();
        double ext = 0.0;
        for (int c = 0; c < 3; c++) {
            double l = red[c][0], h = red[3 + c][0];
            for (int k = 1; k < (int)(blockDim.x >> 6); k++) {
                l = fmin(l, red[c][k]);
                h = fmax(h, red[3 + c][k]);
            }
            ext = fmax(ext, h - l);
        }
        const double *d = kSolidDir[dir[code] % SOLID_DIRS];
        const double L = 2.0 * ext + 1.0;
        const double q[3] = {p[0] + L * d[0], p[1] + L * d[1], p[2] + L * d[2]};
        int cross = 0, deg = 0, on = 0;
        for (int64_t t = mt0 + threadIdx.x; t < mt1; t += blockDim.x) {
            double a[3], b[3], c[3];
            solid_vertex(X, nvr, M.tri, t, 0, a);
            solid_vertex(X, nvr, M.tri, t, 1, b);
            solid_vertex(X, nvr, M.tri, t, 2, c);
            const int r = ray_cross(p, q, a, b, c);
            cross ^= r & 1;
            deg |= (r >> 1) & 1;
            on |= (r >> 2) & 1;
        }
        if (cross) atomicXor(&flags[0], 1);
        if (deg) atomicOr(&flags[1], 1);
        if (on) atomicOr(&flags[2], 1);
        __syncthreads();
        if (threadIdx.x == 0) res[code] = (uint8_t)(flags[0] | (flags[1] << 1) | (flags[2] << 2));
        __syncthreads();
    }
}

// Rows whose solids meet without surface contact: distance 0, hit 1.
__global__ void k_solid_apply(const uint8_t *res, int64_t G, double *dist, uint8_t *hit,
                              const RowState *rows, Lists L, const uint32_t *vflags) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= G || call_failed(L, vflags) || rows[g].hit) return;
    const uint8_t a = res[2 * g], b = res[2 * g + 1];
    if (((a | b) & 1) || ((a | b) & 4)) {
        if (dist) dist[g] = 0.0;
        if (hit) hit[g] = 1;
    }
}

void launch_inside(const SolidSide &A, const SolidSide &B, const RowState *rows, const int32_t *queries,
                   int64_t nq, const uint8_t *dir, uint8_t *res, int grid, hipStream_t s) {
    if (nq > 0)
        hipLaunchKernelGGL(k_inside, dim3((unsigned)std::min<int64_t>(nq, grid)), dim3(256), 0, s, A, B, rows,
                           queries, nq, dir, res);
}

void launch_solid_apply(const uint8_t *res, int64_t G, double *dist, uint8_t *hit, const RowState *rows,
                        Lists &L, const uint32_t *vflags, hipStream_t s) {
    if (G > 0)
        hipLaunchKernelGGL(k_solid_apply, dim3((unsigned)((G + 255) / 256)), dim3(256), 0, s, res, G, dist, hit,
                           rows, L, vflags);
}

}  // namespace sd3
