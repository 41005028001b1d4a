// 3D volume of each row (Sec. 3.2.1): by the divergence theorem with the
// field F = p / 3 the volume is a sum over the faces (Eq. 1), and on a
// counter-clockwise triangle u v w the face term is u . n / 6 with
// n = (v - u) x (w - u) (Eq. 2).
//
// HBM-bound: per triangle 12 bytes of indices and three 24-byte vertex
// gathers, one term, and a sum.  Each term is formed in double-double
// arithmetic (the differences v - u and w - u are exact two-term values, the
// products carry their rounding error through fused multiply-adds), and the
// terms are summed in double-double, so the result keeps about 100 bits of the
// terms' magnitude before the final rounding: far below 1e-12 relative unless
// the faces' terms cancel by more than 2^50 (a closed mesh about 10^5 of its
// own sizes away from the origin).
//
// Work items are (row, chunk of VOL_CHUNK consecutive triangles of that row),
// listed on the host; a block reduces its chunk to one double-double partial;
// a second kernel adds each row's partials in chunk order and writes the
// volume, so the result does not depend on scheduling.
#include <algorithm>

#include "sd3_kernels.h"

#pragma clang fp contract(off)

namespace sd3 {

struct DD {
    double hi, lo;
};

__device__ __forceinline__ DD dd_two_sum(double a, double b) {
    const double s = a + b;
    const double bv = s - a;
    const double av = s - bv;
    return {s, (a - av) + (b - bv)};
}

__device__ __forceinline__ DD dd_fast(double hi, double lo) {
    const double s = hi + lo;
    return {s, lo - (s - hi)};
}

__device__ __forceinline__ DD dd_add(DD a, DD b) {
    DD s = dd_two_sum(a.hi, b.hi);
    DD t = dd_two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = dd_fast(s.hi, s.lo);
    s.lo += t.lo;
    return dd_fast(s.hi, s.lo);
}

__device__ __forceinline__ DD dd_neg(DD a) { return {-a.hi, -a.lo}; }

__device__ __forceinline__ DD dd_mul(DD a, DD b) {
    const double p = a.hi * b.hi;
    double e = fma(a.hi, b.hi, -p);
    e = fma(a.hi, b.lo, e);
    e = fma(a.lo, b.hi, e);
    return dd_fast(p, e);
}

__device__ __forceinline__ DD dd_mul_d(double a, DD b) {
    const double p = a * b.hi;
    double e = fma(a, b.hi, -p);
    e = fma(a, b.lo, e);
    return dd_fast(p, e);
}

// exact difference a - b as a double-double
__device__ __forceinline__ DD dd_diff(double a, double b) {
    const double s = a - b;
    const double bv = a - s;
    const double av = s + bv;
    return {s, (a - av) + (bv - b)};
}

__device__ __forceinline__ DD dd_shfl_xor(DD v, int o) { return {__shfl_xor(v.hi, o), __shfl_xor(v.lo, o)}; }

// u . ((v - u) x (w - u)) for triangle t of its row (vertex indices clamped
// into the row; an index outside it sets `bad`).
__device__ __forceinline__ DD vol_term(const double *X, int64_t nvr, const int32_t *tri, int64_t t,
                                       uint32_t &bad) {
    double p[3][3];
    for (int k = 0; k < 3; k++) {
        const int32_t v = tri[3 * t + k];
        const bool ok = v >= 0 && (int64_t)v < nvr;
        bad |= ok ? 0u : V_INDEX;
        const int64_t vi = ok ? v : 0;
        for (int c = 0; c < 3; c++) p[k][c] = X[3 * vi + c];
    }
    DD a[3], b[3];
    for (int c = 0; c < 3; c++) {
        a[c] = dd_diff(p[1][c], p[0][c]);
        b[c] = dd_diff(p[2][c], p[0][c]);
    }
    DD s = {0.0, 0.0};
    for (int c = 0; c < 3; c++) {
        const int j = (c + 1) % 3, l = (c + 2) % 3;
        const DD n = dd_add(dd_mul(a[j], b[l]), dd_neg(dd_mul(a[l], b[j])));
        s = dd_add(s, dd_mul_d(p[0][c], n));
    }
    return s;
}

constexpr int VOL_CHUNK = 4096;  // triangles per work item
constexpr int VOL_WG = 256;

// item: [row, first triangle of the chunk (global index)] in wrow/wfirst
__global__ __launch_bounds__(VOL_WG) void k_vol_partial(const double *xyz, const int32_t *tri,
                                                        const int64_t *v_off, const int64_t *t_off,
                                                        const int32_t *wrow, const int64_t *wfirst,
                                                        int64_t nitems, DD *part, uint32_t *flags) {
    __shared__ DD red[VOL_WG / 64];
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int64_t g = wrow[it];
        const int64_t t0 = wfirst[it], t1 = min(t_off[g + 1], t0 + (int64_t)VOL_CHUNK);
        const double *X = xyz + 3 * v_off[g];
        const int64_t nvr = v_off[g + 1] - v_off[g];
        DD s = {0.0, 0.0};
        uint32_t bad = 0;
        for (int64_t t = t0 + threadIdx.x; t < t1; t += VOL_WG) s = dd_add(s, vol_term(X, nvr, tri, t, bad));
        for (int o = 32; o > 0; o >>= 1) s = dd_add(s, dd_shfl_xor(s, o));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        if (bad) atomicOr(flags, bad);
        __syncthreads();
        if (threadIdx.x == 0) {
            DD r = red[0];
            for (int w = 1; w < VOL_WG / 64; w++) r = dd_add(r, red[w]);
            part[it] = r;
        }
        __syncthreads();
    }
}

// Coordinates of every vertex (the same checks as the distance operators).
__global__ __launch_bounds__(256) void k_vol_validate(const double *xyz, int64_t nv, uint32_t *flags) {
    uint32_t f = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 3 * nv;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double x = fabs(xyz[i]);
        if (!(x <= 1.7976931348623157e308)) f |= V_NONFINITE;
        else if (x != 0.0 && (x < 0x1p-256 || x > 0x1p256)) f |= V_RANGE;
    }
    if (f) atomicOr(flags, f);
}

// Row g: its partials (items witem[g] .. witem[g+1] - 1) in order, / 6.
__global__ void k_vol_rows(const DD *part, const int64_t *witem, int64_t G, double *vol,
                           const uint32_t *flags) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= G || *flags) return;
    DD s = {0.0, 0.0};
    for (int64_t i = witem[g]; i < witem[g + 1]; i++) s = dd_add(s, part[i]);
    // (hi + lo) / 6 rounded once more: hi / 6 plus the remainder's share
    const double q = s.hi / 6.0;
    const double r = fma(-q, 6.0, s.hi);  // exact remainder of hi - 6 q
    vol[g] = q + (r + s.lo) / 6.0;
}

__global__ void k_vol_clear(uint32_t *flags) {
    if (threadIdx.x == 0) *flags = 0;
}

void launch_volume(const double *xyz, int64_t nv, const int32_t *tri, const int64_t *v_off,
                   const int64_t *t_off, const int32_t *wrow, const int64_t *wfirst, int64_t nitems,
                   const int64_t *witem, int64_t G, void *part, double *vol, uint32_t *flags, int grid,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_vol_clear, dim3(1), dim3(64), 0, s, flags);
    const unsigned vg = (unsigned)std::min<int64_t>(std::max<int64_t>((3 * nv + 255) / 256, 1), 4096);
    if (nv > 0) hipLaunchKernelGGL(k_vol_validate, dim3(vg), dim3(256), 0, s, xyz, nv, flags);
    if (nitems > 0)
        hipLaunchKernelGGL(k_vol_partial, dim3((unsigned)std::min<int64_t>(nitems, grid)), dim3(VOL_WG), 0, s,
                           xyz, tri, v_off, t_off, wrow, wfirst, nitems, (DD *)part, flags);
    if (G > 0)
        hipLaunchKernelGGL(k_vol_rows, dim3((unsigned)((G + 255) / 256)), dim3(256), 0, s, (const DD *)part,
                           witem, G, vol, flags);
}

int volume_chunk() { return VOL_CHUNK; }

}  // namespace sd3
