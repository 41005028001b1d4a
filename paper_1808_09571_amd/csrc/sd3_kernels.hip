// sd3 kernels for gfx950: validation, spatial sort and tiling, tile-pair
// bounds and work queue, the triangle-pair passes (FP32 with error bounds,
// FP64), the FP64 rescue pass, exact arithmetic, and the final reduction.
#include <type_traits>

#include "sd3_kernels.h"
#include "sd3_pair64.h"
#include "sd3_pair32.h"
#include "sd3_exact.h"

static_assert(sd3::C_NCOUNTERS <= 256, "the first block clears every counter");

namespace sd3 {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
// Row g with off[g] <= i < off[g+1] (off non-decreasing, off[0] <= i < off[G]).
__device__ __forceinline__ int64_t find_row(const int64_t *off, int64_t G, int64_t i) {
    int64_t lo = 0, hi = G;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// The same row found by a whole wave for a wave-uniform i: each round the 64
// lanes probe 64 evenly spaced offsets of the remaining range and the count
// of probes at or below i narrows it 64-fold (two dependent loads for 4096
// rows instead of twelve).  Every lane of the wave must take part.
__device__ __forceinline__ int64_t wave_find_row(const int64_t *off, int64_t G, int64_t i) {
    int64_t lo = 0, hi = G;
    while (hi - lo > 1) {
        const int64_t step = (hi - lo + 63) >> 6;
        const int64_t p = lo + (int64_t)(lane_id() + 1) * step;
        const int c = __popcll(__ballot(p < hi && off[p] <= i));
        hi = min(hi, lo + (int64_t)(c + 1) * step);
        lo += (int64_t)c * step;
    }
    return lo;
}

// Workgroups are dealt to the GPU's 8 XCDs (each with its own L2) in turn:
// block b runs on XCD b % 8.  The logical block of b gives each XCD one
// contiguous range [x q + min(x, r), ...) of the nb blocks (q = nb / 8,
// r = nb % 8), so that neighbouring blocks -- the same row's data -- share an
// L2 instead of being fetched into all eight.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
    const unsigned x = b & 7u, k = b >> 3, q = nb >> 3, r = nb & 7u;
    return x * q + min(x, r) + k;
}

// LDS written by some lanes of a wave and read by others: the wave's LDS
// operations complete in issue order, so keeping the compiler from moving
// them across this point is all that is needed (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Vertex index of corner k of triangle t, local to its row of nvr vertices.
// An index outside the row reads vertex 0 instead: kernels that run before the
// validation flags are read (graph replays) never address memory outside the
// row, and the flags keep such a call from writing results.
__device__ __forceinline__ int64_t corner(const int32_t *tri, int64_t t, int k, int64_t nvr) {
    int32_t v = tri[3 * t + k];
    return (v >= 0 && (int64_t)v < nvr) ? (int64_t)v : 0;
}

__device__ __forceinline__ unsigned long long load_acq(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_acq32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

static inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    return (unsigned)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------------------
// a1: validation of device-resident inputs
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t coord_flags(double v) {
    double x = fabs(v);
    if (!(x <= 1.7976931348623157e308)) return V_NONFINITE;
    if (x != 0.0 && (x < 0x1p-256 || x > 0x1p256)) return V_RANGE;
    return 0u;
}

// Every triangle index of both sides must lie inside its row.  Blocks own
// contiguous ranges of VT_ITEMS triangles of one side (A's blocks first);
// one wave search finds the row of a block's first triangle and each thread
// walks forward from it.
constexpr int VT_ITEMS = 4096;

struct TriSide {
    const int32_t *tri;
    int64_t nt;
    const int64_t *v_off, *t_off;
    unsigned nblk;
};

// Starts row g's state from both (merged) row boxes.
__device__ void row_init_vals(RowState *rows, int64_t g, const unsigned long long *bA,
                              const unsigned long long *bB);

// Triangle blocks of the validation launch (blk counts A's blocks, then B's):
// every index load of the block's VT_ITEMS triangles is issued before the
// first check; each thread then walks its items' rows forward from the
// block's first row, keeping the current row's end and vertex count, so
// items in the same row need no further load.
__device__ void validate_tris(const TriSide &A, const TriSide &B, int64_t G, unsigned blk,
                              uint32_t *flags) {
    __shared__ int64_t g0s;
    const bool sa = blk < A.nblk;
    const TriSide &S = sa ? A : B;
    const int64_t t0 = (int64_t)(sa ? blk : blk - A.nblk) * VT_ITEMS;
    const int64_t t1 = min(S.nt, t0 + VT_ITEMS);
    constexpr int PER = VT_ITEMS / 256;
    int32_t tv[PER][3];
#pragma unroll
    for (int r = 0; r < PER; r++) {
        const int64_t t = min(t0 + threadIdx.x + 256 * r, t1 - 1);
#pragma unroll
        for (int k = 0; k < 3; k++) tv[r][k] = S.tri[3 * t + k];
    }
    if (threadIdx.x < 64) {
        const int64_t g0 = wave_find_row(S.t_off, G, t0);
        if (threadIdx.x == 0) g0s = g0;
    }
    __syncthreads();
    int64_t g = g0s;
    int64_t end = S.t_off[g + 1], nvr = S.v_off[g + 1] - S.v_off[g];
    uint32_t f = 0;
#pragma unroll
    for (int r = 0; r < PER; r++) {
        const int64_t t = t0 + threadIdx.x + 256 * r;
        if (t >= t1) break;
        while (end <= t) {
            g++;
            end = S.t_off[g + 1];
            nvr = S.v_off[g + 1] - S.v_off[g];
        }
        for (int k = 0; k < 3; k++)
            if (tv[r][k] < 0 || tv[r][k] >= nvr) f = V_INDEX;
    }
    if (f) atomicOr(flags + (sa ? 0 : 1), f);
}

// ---------------------------------------------------------------------------
// a2: row boxes, Morton keys, radix sort, tiles
// ---------------------------------------------------------------------------
// The first kernel of a call: clears the device scalars 0-11 (queue, rescue,
// exact, seed, work items, exact blocks done), the validation flags of both
// sides, the counters, the row boxes of both sides and the kept-triangle
// counts of a culling call.
__global__ void k_prep_init(unsigned int *sc, uint32_t *flags, unsigned long long *counters,
                            unsigned long long *boxA, unsigned long long *boxB, int64_t nbox,
                            int32_t *kc, int64_t nkc) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < 12) sc[i] = 0u;
    if (i < 2) flags[i] = 0u;
    if (i < C_NCOUNTERS) counters[i] = 0ull;
    if (i < nbox) {
        unsigned long long v = (i % 6) < 3 ? ~0ull : 0ull;
        boxA[i] = v;
        boxB[i] = v;
    }
    if (i < nkc) kc[i] = 0;
}

// Rows of the vertex chunks of a block's contiguous range: the row of vertex
// i walked forward from row g (off[g] <= i; g and i wave-uniform), a few
// steps (rows usually span many chunks), else a wave search.
__device__ __forceinline__ int64_t walk_row(const int64_t *off, int64_t G, int64_t g, int64_t i) {
    for (int k = 0; k < 4; k++) {
        if (off[g + 1] > i) return g;
        g++;
    }
    return wave_find_row(off, G, i);
}

// The row of consecutive chunks' vertices, walked forward (wave-uniform):
// the current row and the offset where it ends, so that a chunk inside one
// row needs no load.
struct RowCursor {
    int64_t g, end;
    __device__ void start(const int64_t *off, int64_t G, int64_t i) {
        g = wave_find_row(off, G, i);
        end = off[g + 1];
    }
    // row of vertex i (at or after the current row's start)
    __device__ int64_t at(const int64_t *off, int64_t G, int64_t i) {
        if (i >= end) {
            g = walk_row(off, G, g, i);
            end = off[g + 1];
        }
        return g;
    }
};

// Row of one lane's vertex i of a chunk whose rows are g0..g1.
__device__ __forceinline__ int64_t lane_row(const int64_t *off, int64_t G, int64_t g0, int64_t g1,
                                            int64_t i) {
    if (g1 - g0 >= 16) return find_row(off, G, i);
    int64_t g = g0;
    while (off[g + 1] <= i) g++;
    return g;
}

// Row bounding boxes of all vertices.  Each block owns a contiguous range of
// vertices and keeps running per-thread min/max (FP64) while its chunks stay
// inside one row; it reduces over the block and issues one atomic per
// component (on the order-preserving bits) only when the row changes (rows
// are contiguous), so large rows cost a few atomics per block instead of one
// per wave.
__device__ void rowbox_flush(int64_t g, double *lo, double *hi, unsigned long long (*red)[6],
                             unsigned long long *box) {
    for (int k = 0; k < 3; k++) {
        const double a = wave_min(lo[k]), b = wave_max(hi[k]);
        if (lane_id() == 0) {
            red[threadIdx.x >> 6][k] = ordered_bits(a);
            red[threadIdx.x >> 6][3 + k] = ordered_bits(b);
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        int k = threadIdx.x;
        unsigned long long v = red[0][k];
        for (int w = 1; w < 4; w++) v = k < 3 ? min(v, red[w][k]) : max(v, red[w][k]);
        if (k < 3) {
            if (v < box[g * 6 + k]) atomicMin(&box[g * 6 + k], v);
        } else {
            if (v > box[g * 6 + k]) atomicMax(&box[g * 6 + k], v);
        }
    }
    __syncthreads();
    for (int k = 0; k < 3; k++) {
        lo[k] = __builtin_inf();
        hi[k] = -__builtin_inf();
    }
}

// A chunk that crosses rows: each wave reduces per row it touches (a wave's
// lanes hold consecutive vertices, so a few rows at most) and issues one
// atomic per row and component; a wave over more than four rows (rows of a
// few vertices) lets every lane issue its own.
__device__ void rowbox_split(const double (&x)[3], bool valid, int64_t g, unsigned long long *box) {
    const int64_t gl = valid ? g : INT64_MAX, gh = valid ? g : -1;
    const int64_t w0 = wave_min(gl), w1 = wave_max(gh);
    if (w1 < 0) return;
    if (w1 - w0 > 3) {
        if (valid)
            for (int k = 0; k < 3; k++) {
                const unsigned long long v = ordered_bits(x[k]);
                atomicMin(&box[g * 6 + k], v);
                atomicMax(&box[g * 6 + 3 + k], v);
            }
        return;
    }
    for (int64_t r = w0; r <= w1; r++) {
        const bool in = valid && g == r;
        if (!__ballot(in)) continue;
        for (int k = 0; k < 3; k++) {
            const double a = wave_min(in ? x[k] : __builtin_inf());
            const double b = wave_max(in ? x[k] : -__builtin_inf());
            if (lane_id() == 0) {
                atomicMin(&box[r * 6 + k], ordered_bits(a));
                atomicMax(&box[r * 6 + 3 + k], ordered_bits(b));
            }
        }
    }
}

struct XyzSide {
    const double *xyz;
    int64_t nv;
    const int64_t *v_off;
    unsigned long long *box;
    unsigned nblk;
    int rep;  // box replicas: block b reduces into replica b % rep
};

// The same pass checks every coordinate (finite, magnitude range).
__device__ void rowbox_side(const XyzSide &S, int64_t G, unsigned blk, uint32_t *flag) {
    __shared__ unsigned long long red[4][6];
    unsigned long long *box = S.box + (int64_t)(blk % (unsigned)S.rep) * G * 6;
    const int64_t nv = S.nv;
    int64_t per = ((nv + S.nblk - 1) / S.nblk + 255) / 256 * 256;
    int64_t b0 = blk * per, b1 = min(nv, b0 + per);
    double lo[3], hi[3];
    for (int k = 0; k < 3; k++) {
        lo[k] = __builtin_inf();
        hi[k] = -__builtin_inf();
    }
    uint32_t f = 0;
    int64_t cur = -1;
    // the rows of each chunk's first and last vertex, walked forward (rows
    // are contiguous and usually span many chunks); each chunk's coordinates
    // are loaded while the previous chunk is reduced
    RowCursor rc{0, 0};
    double xn[3] = {0.0, 0.0, 0.0};
    if (b0 < b1) {
        rc.start(S.v_off, G, b0);
        if (b0 + threadIdx.x < b1)
            for (int k = 0; k < 3; k++) xn[k] = S.xyz[3 * (b0 + threadIdx.x) + k];
    }
    for (int64_t base = b0; base < b1; base += 256) {
        int64_t last = min(base + 255, b1 - 1);
        const int64_t g0 = rc.at(S.v_off, G, base);
        const int64_t g1 = rc.at(S.v_off, G, last);
        int64_t i = base + threadIdx.x;
        bool valid = i <= last;
        const double x[3] = {xn[0], xn[1], xn[2]};
        if (i + 256 < b1)
            for (int k = 0; k < 3; k++) xn[k] = S.xyz[3 * (i + 256) + k];
        if (valid)
            for (int k = 0; k < 3; k++) f |= coord_flags(x[k]);
        if (g0 == g1) {
            if (g0 != cur) {
                if (cur >= 0) rowbox_flush(cur, lo, hi, red, box);
                cur = g0;
            }
            if (valid)
                for (int k = 0; k < 3; k++) {
                    lo[k] = fmin(lo[k], x[k]);
                    hi[k] = fmax(hi[k], x[k]);
                }
        } else {
            if (cur >= 0) rowbox_flush(cur, lo, hi, red, box);
            cur = -1;
            rowbox_split(x, valid, valid ? lane_row(S.v_off, G, g0, g1, i) : -1, box);
        }
    }
    if (cur >= 0) rowbox_flush(cur, lo, hi, red, box);
    if (f) atomicOr(flag, f);
}

// Blocks [0, A.nblk) take side A's vertices, then B's vertices.
__global__ __launch_bounds__(256) void k_rowbox(XyzSide A, XyzSide B, int64_t G, uint32_t *flags) {
    if (blockIdx.x < A.nblk) rowbox_side(A, G, blockIdx.x, flags);
    else rowbox_side(B, G, blockIdx.x - A.nblk, flags + 1);
}

// The triangles of both sides (A's blocks first); a launch of its own, so
// that the vertex pass keeps its few registers.
__global__ __launch_bounds__(256) void k_validate_tris(TriSide TA, TriSide TB, int64_t G, uint32_t *flags) {
    validate_tris(TA, TB, G, blockIdx.x, flags);
}

static unsigned rowbox_blocks(int64_t nv) {
    if (nv <= 0) return 0;
    unsigned g = grid_for(nv, 1024);
    return g > 8192 ? 8192 : g;
}

int rowbox_replicas(int64_t nv, int64_t G) {
    if (G <= 0) return 1;
    const int64_t per_row = rowbox_blocks(nv) / G;
    return (int)std::max<int64_t>(1, std::min<int64_t>(16, per_row / 16));
}

void launch_validate_rowbox(SideBufs &A, SideBufs &B, PrepBufs &P, uint32_t *flags, Lists &L,
                            hipStream_t s, bool indices) {
    const int64_t G = A.G;
    const int64_t nbox = (int64_t)A.boxrep * G * 6;
    const int64_t nkc = P.kc ? 2 * G : 0;
    // (one block at least: C_NCOUNTERS <= 256)
    const int64_t nz = std::max<int64_t>(256, std::max(nbox, nkc));
    hipLaunchKernelGGL(k_prep_init, dim3(grid_for(nz, 256)), dim3(256), 0, s, L.qcount, flags, L.counters,
                       A.rowbox, B.rowbox, nbox, P.kc, nkc);
    XyzSide xa{A.xyz, A.nv, A.v_off, A.rowbox, rowbox_blocks(A.nv), A.boxrep};
    XyzSide xb{B.xyz, B.nv, B.v_off, B.rowbox, rowbox_blocks(B.nv), B.boxrep};
    // (without `indices` the key kernel checks the triangle indices)
    TriSide ta{A.tri, A.nt, A.v_off, A.t_off, indices ? grid_for(A.nt, VT_ITEMS) : 0u};
    TriSide tb{B.tri, B.nt, B.v_off, B.t_off, indices ? grid_for(B.nt, VT_ITEMS) : 0u};
    if (xa.nblk + xb.nblk > 0)
        hipLaunchKernelGGL(k_rowbox, dim3(xa.nblk + xb.nblk), dim3(256), 0, s, xa, xb, G, flags);
    if (ta.nblk + tb.nblk > 0)
        hipLaunchKernelGGL(k_validate_tris, dim3(ta.nblk + tb.nblk), dim3(256), 0, s, ta, tb, G, flags);
}

__device__ __forceinline__ uint32_t spread10(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// key = the top mbits of the 30-bit Morton code of the triangle's first
// vertex, quantised on cubic cells of the row box (the largest extent / 1024
// on every axis, so a flat surface spends its bits on its two long axes);
// value = triangle index within its side.  Both sides in one launch (A's
// triangles, then B's); the sort keeps every item within its row.

// Row g's box component k (ordered bits) merged over the rep replicas.
__device__ __forceinline__ unsigned long long merged_box(const unsigned long long *box, int rep,
                                                         int64_t G, int64_t g, int k) {
    unsigned long long v = box[g * 6 + k];
    for (int r = 1; r < rep; r++) {
        const unsigned long long w = box[(int64_t)r * G * 6 + g * 6 + k];
        v = k < 3 ? min(v, w) : max(v, w);
    }
    return v;
}

// Cells of a row: the origin (box minimum) and the scale mapping the largest
// extent onto 1024 cells, from the six ordered-bit box components.
__device__ __forceinline__ double row_cells(const unsigned long long *b, double lo[3]) {
    double ext = 0.0;
    for (int k = 0; k < 3; k++) {
        lo[k] = from_ordered_bits(b[k]);
        ext = fmax(ext, from_ordered_bits(b[3 + k]) - lo[k]);
    }
    return ext > 0.0 ? 1024.0 / ext : 0.0;
}

// 30-bit Morton code of point p on those cells.
__device__ __forceinline__ uint32_t morton_code(const double *p, const double *lo, double sc) {
    uint32_t q[3];
    for (int k = 0; k < 3; k++) {
        const double f = (p[k] - lo[k]) * sc;
        const int qi = (int)f;
        q[k] = (uint32_t)(qi < 0 ? 0 : (qi > 1023 ? 1023 : qi));
    }
    return spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2);
}

struct MortonSide {
    const double *xyz;
    const int32_t *tri;
    int64_t nt;
    const int64_t *v_off, *t_off;
    const unsigned long long *box;
    const uint32_t *vcode;  // per-vertex codes (VC keys)
    int32_t *kc;            // kept triangles per row (culling VC keys), else nullptr
    const uint8_t *oc;      // per-vertex outcodes (culling), else nullptr
};

// Per-vertex Morton codes for large sorts: the key kernel then gathers a
// 4-byte code per triangle instead of a 24-byte vertex (a sixth of the lines
// when a row's vertex order is far from its triangle order) and no row box.
// Blocks own contiguous vertex ranges as in the row-box pass; a wave merges a
// row's box once while its chunks stay inside that row.
struct VcodeSide {
    const double *xyz;
    int64_t nv;
    const int64_t *v_off;
    const unsigned long long *box;
    uint32_t *code;
    unsigned nblk;
    const unsigned long long *obox;  // the other side's row boxes (culling), else nullptr
    const double *cub;               // per row: how far beyond that box a triangle is
                                     // still kept (distance calls), else nullptr (0)
    uint8_t *oc;                     // the outcodes again, one byte per vertex (culling):
                                     // the key kernel gathers two per triangle from this
                                     // array, a quarter of the codes' footprint
};

// The other side's row box (six ordered-bit components) widened by e >= 0 on
// every side and then by 2^-50 (|bound| + e), far more than the rounding of
// the two operations (2^-53 of that each), so that a point outside it is
// farther than e from the box along that axis.
__device__ __forceinline__ void cull_box(const unsigned long long *ob, double e, double lo[3], double hi[3]) {
    for (int k = 0; k < 3; k++) {
        lo[k] = from_ordered_bits(ob[k]);
        hi[k] = from_ordered_bits(ob[3 + k]);
        if (e > 0.0) {
            lo[k] = (lo[k] - e) - 0x1p-50 * (fabs(lo[k]) + e);
            hi[k] = (hi[k] + e) + 0x1p-50 * (fabs(hi[k]) + e);
        }
    }
}

// Outcode of point p against that box: bit 2k set when coordinate k lies
// below it, bit 2k + 1 when above.  A triangle whose three vertices share a
// set bit lies entirely beyond one of the box's planes (exact comparisons of
// the stored coordinates), so it is farther than e from every point of the
// other side.
__device__ __forceinline__ uint32_t outcode(const double *p, const double *lo, const double *hi) {
    uint32_t oc = 0;
    for (int k = 0; k < 3; k++) {
        oc |= (p[k] < lo[k] ? 1u : 0u) << (2 * k);
        oc |= (p[k] > hi[k] ? 1u : 0u) << (2 * k + 1);
    }
    return oc;
}

// Cull distance of each row for a distance call: the smallest distance
// between corners of 64 evenly spaced triangles of each side (two surface
// points bound the row distance from above), rounded up, plus a margin far
// above the FP64 rounding of any pair distance in the row (2^-30 of the row
// extent and of the bound; the pruning margin is 2^-36 of both), so that a
// triangle culled by it could not hold the FP64 minimum.  One wave per row.
struct UbSide {
    const double *xyz;
    const int32_t *tri;
    const int64_t *v_off, *t_off;
    const unsigned long long *box;
};

__global__ __launch_bounds__(256) void k_row_ub(UbSide A, UbSide B, int64_t G, int rep, double *cub) {
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= G) return;  // (wave-uniform)
    const int lane = lane_id();
    const int64_t ta = A.t_off[g], na = A.t_off[g + 1] - ta, tb = B.t_off[g], nb = B.t_off[g + 1] - tb;
    if (na == 0 || nb == 0) {
        if (lane == 0) cub[g] = __builtin_inf();
        return;
    }
    const int64_t va = A.v_off[g], vb = B.v_off[g];
    const double *pa = A.xyz + 3 * (va + corner(A.tri, ta + (lane * na) / 64, 0, A.v_off[g + 1] - va));
    const double *pb = B.xyz + 3 * (vb + corner(B.tri, tb + (lane * nb) / 64, 0, B.v_off[g + 1] - vb));
    const double p0 = pa[0], p1 = pa[1], p2 = pa[2];
    const double q0 = pb[0], q1 = pb[1], q2 = pb[2];
    double m = __builtin_inf();
    for (int j = 0; j < 64; j++) {
        const double d0 = p0 - __shfl(q0, j), d1 = p1 - __shfl(q1, j), d2 = p2 - __shfl(q2, j);
        m = fmin(m, d0 * d0 + d1 * d1 + d2 * d2);
    }
    m = wave_min(m);
    double ext2 = 0.0;
    for (int k = 0; k < 3; k++) {
        const double lo = fmin(from_ordered_bits(merged_box(A.box, rep, G, g, k)),
                               from_ordered_bits(merged_box(B.box, rep, G, g, k)));
        const double hi = fmax(from_ordered_bits(merged_box(A.box, rep, G, g, 3 + k)),
                               from_ordered_bits(merged_box(B.box, rep, G, g, 3 + k)));
        ext2 += (hi - lo) * (hi - lo);
    }
    const double ub = sqrt(m) * (1.0 + 8.0 * U64);
    if (lane == 0) cub[g] = ub + 0x1p-30 * (sqrt(ext2) * 1.01 + ub);
}

template <bool CULL>
__device__ void vcode_side(const VcodeSide &S, int64_t G, int rep, unsigned blk) {
    const int lane = lane_id();
    const int64_t nv = S.nv;
    const int64_t per = ((nv + S.nblk - 1) / S.nblk + 255) / 256 * 256;
    const int64_t b0 = blk * per, b1 = min(nv, b0 + per);
    int64_t cg = -1;  // row whose cells are held (wave-uniform)
    double clo[3] = {0.0, 0.0, 0.0}, csc = 0.0;
    double olo[3] = {0.0, 0.0, 0.0}, ohi[3] = {0.0, 0.0, 0.0};  // the row's cull box
    RowCursor rc{0, 0};
    double pn[3] = {0.0, 0.0, 0.0};  // the next chunk's coordinates, in flight
    if (b0 < b1) {
        rc.start(S.v_off, G, b0);
        if (b0 + threadIdx.x < b1)
            for (int k = 0; k < 3; k++) pn[k] = S.xyz[3 * (b0 + threadIdx.x) + k];
    }
    for (int64_t base = b0; base < b1; base += 256) {
        const int64_t last = min(base + 255, b1 - 1);
        const int64_t g0 = rc.at(S.v_off, G, base);
        const int64_t g1 = rc.at(S.v_off, G, last);
        const int64_t i = base + threadIdx.x;
        const bool valid = i <= last;
        const double p[3] = {pn[0], pn[1], pn[2]};
        if (i + 256 < b1)
            for (int k = 0; k < 3; k++) pn[k] = S.xyz[3 * (i + 256) + k];
        // a culling call keeps the vertex's outcode against the other side's
        // row box in the code's low 6 bits (keys use its top 24 bits at most)
        if (g0 == g1) {
            if (g0 != cg) {
                const unsigned long long m = lane < 6 ? merged_box(S.box, rep, G, g0, lane)
                                                      : (CULL && lane < 12 ? merged_box(S.obox, rep, G, g0, lane - 6) : 0ull);
                unsigned long long b[6];
                for (int k = 0; k < 6; k++) b[k] = __shfl(m, k);
                if (CULL) {
                    unsigned long long ob[6];
                    for (int k = 0; k < 6; k++) ob[k] = __shfl(m, 6 + k);
                    cull_box(ob, S.cub ? S.cub[g0] : 0.0, olo, ohi);
                }
                csc = row_cells(b, clo);
                cg = g0;
            }
            if (valid && CULL) {
                const uint32_t oc = outcode(p, olo, ohi);
                S.code[i] = (morton_code(p, clo, csc) & ~63u) | oc;
                S.oc[i] = (uint8_t)oc;
            } else if (valid) {
                S.code[i] = morton_code(p, clo, csc);
            }
        } else if (valid) {
            const int64_t g = lane_row(S.v_off, G, g0, g1, i);
            unsigned long long b[6];
            for (int k = 0; k < 6; k++) b[k] = merged_box(S.box, rep, G, g, k);
            double lo[3];
            const double sc = row_cells(b, lo);
            uint32_t code = morton_code(p, lo, sc);
            if (CULL) {
                unsigned long long ob[6];
                for (int k = 0; k < 6; k++) ob[k] = merged_box(S.obox, rep, G, g, k);
                double bl[3], bh[3];
                cull_box(ob, S.cub ? S.cub[g] : 0.0, bl, bh);
                const uint32_t oc = outcode(p, bl, bh);
                code = (code & ~63u) | oc;
                S.oc[i] = (uint8_t)oc;
            }
            S.code[i] = code;
        }
    }
}

// CULL: a culling call (the sides' other-box pointers are set).
template <bool CULL>
__global__ __launch_bounds__(256) void k_vcode(VcodeSide A, VcodeSide B, int64_t G, int rep) {
    if (blockIdx.x < A.nblk) vcode_side<CULL>(A, G, rep, blockIdx.x);
    else vcode_side<CULL>(B, G, rep, blockIdx.x - A.nblk);
}

// Sort block b's entry from the side's row offsets, the row found by `find`
// (a wave search or a thread's own binary search).
template <typename Find>
__device__ __forceinline__ SBlock sort_block_entry(const SortSeg &S, int64_t b, Find find) {
    SBlock k;
    k.side = b >= S.nbA ? 1 : 0;
    const int64_t bl = k.side ? b - S.nbA : b;
    const int64_t *sb = k.side ? S.sbB : S.sbA;
    const int64_t *to = k.side ? S.toffB : S.toffA;
    k.g = find(sb, bl);
    const int64_t s0 = sb[k.g], s1 = sb[k.g + 1];
    const int64_t j = bl - s0;
    k.t0 = to[k.g] + j * S.rsi;
    k.n = (int)min((int64_t)S.rsi, to[k.g + 1] - k.t0);
    k.i0 = (k.side ? S.ntA : 0) + k.t0;
    k.hstride = (int)(s1 - s0);
    k.hbase = 256 * ((k.side ? S.nbA : 0) + s0) + j;
    k.loc = (int32_t)(j * S.rsi);
    return k;
}

// Sort block b of the row-segmented sort (every lane of the wave calls this;
// b wave-uniform): from the table when the call built one, else by a wave
// search of the row offsets.
__device__ __forceinline__ SBlock sort_block(const SortSeg &S, int64_t b) {
    if (S.tab) return S.tab[b];
    return sort_block_entry(S, b, [&](const int64_t *sb, int64_t bl) { return wave_find_row(sb, S.G, bl); });
}

// The table: one thread per sort block, each with its own binary search.
__global__ __launch_bounds__(256) void k_sort_table(SortSeg S) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= S.nb) return;
    S.tab[b] = sort_block_entry(S, b, [&](const int64_t *sb, int64_t bl) { return find_row(sb, S.G, bl); });
}

// One block of 1024 threads per sort block of RS_ITEMS keys (all in one row),
// so that the histogram of the sort's first digit is counted here.  Each
// thread takes RS_ITEMS / 1024 items and issues all their index loads, then
// all their vertex (VC: code) loads, before any store.  Without per-vertex
// codes the block's row box is merged once, by each wave, while those loads
// are in flight.
// The same launch starts every row's state from the merged row boxes (one
// wave per row).  LOC: values are the triangle's index within its row (else
// within its side).
template <int RS_ITEMS, bool VC, bool LOC>
__global__ __launch_bounds__(1024) void k_morton(MortonSide A, MortonSide B, SortSeg S, int mbits,
                                                 uint32_t *keys, int32_t *vals, uint32_t *hist,
                                                 int rep, int64_t G, RowState *rows, uint32_t *flags) {
    constexpr int PER = RS_ITEMS / 1024;
    __shared__ uint32_t h[256];
    __shared__ unsigned long long rb[16][12];   // per wave: the merged boxes of the row it starts
    const int lane = lane_id();
    {
        // the grid's last waves start the rows
        const int64_t nwv = ((int64_t)gridDim.x * blockDim.x) >> 6;
        const int64_t wv = nwv - 1 - (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
        unsigned long long *m = rb[threadIdx.x >> 6];
        for (int64_t g = wv; g < G; g += nwv) {
            if (lane < 12) m[lane] = merged_box(lane < 6 ? A.box : B.box, rep, G, g, lane % 6);
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) row_init_vals(rows, g, m, m + 6);
            __builtin_amdgcn_wave_barrier();
        }
    }
    if ((int64_t)blockIdx.x >= S.nb) return;  // the one block of a call with no items
    const int64_t bl = xcd_block(blockIdx.x, gridDim.x);
    const SBlock k = sort_block(S, bl);
    const MortonSide &M = k.side ? B : A;
    __shared__ uint32_t nkeep;  // the block's kept triangles (culling)
    __shared__ uint32_t wk[PER][16];  // kept items per round and wave (culling)
    if (threadIdx.x < 256) h[threadIdx.x] = 0;
    if (threadIdx.x == 0) nkeep = 0;
    const int64_t vb = M.v_off[k.g];
    const int64_t nvr = M.v_off[k.g + 1] - vb;
    int64_t vi[PER];
    bool ok[PER];
    int32_t tv[PER][3];
#pragma unroll
    for (int r = 0; r < PER; r++) {
        const int j = r * 1024 + (int)threadIdx.x;
        ok[r] = j < k.n;
        const int64_t t = k.t0 + (ok[r] ? j : 0);
#pragma unroll
        for (int c = 0; c < 3; c++) tv[r][c] = M.tri[3 * t + c];
    }
    // every triangle index must lie inside its row (the three indices share
    // the cache lines the first one is read from); an invalid first index
    // reads vertex 0 of the row, and the flag keeps the call from writing
    // results
    uint32_t bad = 0;
#pragma unroll
    for (int r = 0; r < PER; r++) {
#pragma unroll
        for (int c = 0; c < 3; c++) bad |= ok[r] && (tv[r][c] < 0 || (int64_t)tv[r][c] >= nvr);
        vi[r] = vb + ((tv[r][0] >= 0 && (int64_t)tv[r][0] < nvr) ? (int64_t)tv[r][0] : 0);
    }
    if (__ballot(bad) && lane == 0) atomicOr(flags + k.side, V_INDEX);
    // the key point is the triangle's first vertex (keys only order work).
    // A culling call also reads the other two vertices' outcodes: a triangle
    // whose box misses the other side's row box cannot meet that side, gets
    // the largest key (kept ones are held below it) and is not counted, so
    // the row's kept triangles come first in its sorted range.
    double cen[VC ? 1 : PER][3];
    uint32_t code[PER];
    bool cut[PER];
#pragma unroll
    for (int r = 0; r < PER; r++) {
        cut[r] = false;
        if (VC) {
            code[r] = ok[r] ? M.vcode[vi[r]] : 0u;
        } else {
#pragma unroll
            for (int c = 0; c < 3; c++) cen[VC ? 0 : r][c] = ok[r] ? M.xyz[3 * vi[r] + c] : 0.0;
        }
    }
    // (the other two codes only where the first vertex lies outside: a zero
    // outcode keeps the triangle whatever the others are)
    if (VC && M.kc) {
#pragma unroll
        for (int r = 0; r < PER; r++) {
            if (ok[r] && (code[r] & 63u) != 0u) {
                const int32_t v1 = tv[r][1], v2 = tv[r][2];
                const uint32_t o1 = M.oc[vb + ((v1 >= 0 && (int64_t)v1 < nvr) ? (int64_t)v1 : 0)];
                const uint32_t o2 = M.oc[vb + ((v2 >= 0 && (int64_t)v2 < nvr) ? (int64_t)v2 : 0)];
                cut[r] = (code[r] & o1 & o2 & 63u) != 0u;
            }
        }
    }
    double lo[3] = {0.0, 0.0, 0.0}, sc = 0.0;
    if (!VC) {
        const unsigned long long mb = lane < 6 ? merged_box(M.box, rep, G, k.g, lane) : 0ull;
        unsigned long long b[6];
        for (int c = 0; c < 6; c++) b[c] = __shfl(mb, c);
        sc = row_cells(b, lo);
    }
    // a culling call writes the block's kept items first, in item order, at
    // the kept items before them (a ballot per round and wave, one barrier);
    // the first sort pass reads only those, the culled ones being counted in
    // digit 255
    int32_t at[PER];
#pragma unroll
    for (int r = 0; r < PER; r++) at[r] = r * 1024 + (int)threadIdx.x;
    if (VC && M.kc) {
        const int w = (int)(threadIdx.x >> 6);
        unsigned long long bal[PER];
#pragma unroll
        for (int r = 0; r < PER; r++) {
            bal[r] = __ballot(ok[r] && !cut[r]);
            if (lane == 0) wk[r][w] = (uint32_t)__popcll(bal[r]);
        }
        __syncthreads();
        uint32_t run = 0;
#pragma unroll
        for (int r = 0; r < PER; r++) {
            uint32_t before = 0, tot = 0;
            for (int q = 0; q < 16; q++) {
                const uint32_t c = wk[r][q];
                before += q < w ? c : 0u;
                tot += c;
            }
            at[r] = (int32_t)(run + before + (uint32_t)__popcll(bal[r] & lanes_below()));
            run += tot;
        }
        if (threadIdx.x == 0) {
            nkeep = run;
            S.bn[bl] = (int32_t)run;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; r++) {
        if (!ok[r] || cut[r]) continue;  // (culled items are counted below, not written)
        const int j = r * 1024 + (int)threadIdx.x;
        if (!VC) code[r] = morton_code(cen[VC ? 0 : r], lo, sc);
        uint32_t key = code[r] >> (30 - mbits);
        if (VC && M.kc) {
            // kept keys hold no 255 digit (each byte capped at 254), so that
            // every pass places the culled items (all digits 255, counted,
            // never written) at the end of the row
            uint32_t kk = 0;
            for (int sh = 0; sh < mbits; sh += 8) kk |= min((key >> sh) & 255u, 254u) << sh;
            key = kk;
        }
        keys[k.i0 + at[r]] = key;
        vals[k.i0 + at[r]] = (int32_t)(LOC ? k.loc + j : k.t0 + j);
        atomicAdd(&h[key & 255u], 1u);
    }
    if (VC && M.kc) {
        // culled items all fall in digit 255: one LDS atomic per wave
        uint32_t ncut = 0;
#pragma unroll
        for (int r = 0; r < PER; r++) ncut += (uint32_t)__popcll(__ballot(ok[r] && cut[r]));
        if (lane == 0 && ncut) atomicAdd(&h[255], ncut);
    }
    __syncthreads();
    if (threadIdx.x < 256) hist[k.hbase + (int64_t)threadIdx.x * k.hstride] = h[threadIdx.x];
    if (VC && M.kc && threadIdx.x == 0 && nkeep) atomicAdd(M.kc + k.g, (int32_t)nkeep);
}

// Stable LSD radix sort, 8-bit digits, within rows.  Blocks of 256 threads
// own one sort block (up to RS_ITEMS consecutive items of one row); per pass:
// digit histogram per block (the first pass's comes from the key kernel), one
// exclusive scan over (row, digit, block), and a stable scatter that ranks
// equal digits inside a wave with ballots.

// Items of sort block k that a pass after the first reads: all of them, or
// in a culling call the part of the block inside its row's kept prefix (the
// first pass put the kept items first, the culled ones, all digits 255, at
// the row's end, where no later pass reads or writes them).
__device__ __forceinline__ int kept_in_block(const SortSeg &S, const SBlock &k) {
    if (!S.kc) return k.n;
    const int64_t kept = (int64_t)S.kc[(k.side ? S.G : 0) + k.g] - (int64_t)k.loc;
    return (int)max((int64_t)0, min((int64_t)k.n, kept));
}

template <int RS_ITEMS>
__global__ void k_hist(const uint32_t *keys, SortSeg S, int shift, uint32_t *hist) {
    constexpr int PER = RS_ITEMS / 256;
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    const SBlock k = sort_block(S, xcd_block(blockIdx.x, gridDim.x));
    // every load first, at clamped indices (n >= 1 here), so that the thread
    // waits for one memory latency rather than one per item
    // (a culling call: this pass reads the row's kept prefix only; the
    // block's other items, culled, all have digit 255 and are counted there
    // without being read)
    const int nv = kept_in_block(S, k);
    uint32_t kv[PER];
#pragma unroll
    for (int r = 0; r < PER; r++) kv[r] = keys[k.i0 + max(0, min(r * 256 + (int)threadIdx.x, nv - 1))];
    __syncthreads();
    // items of digit 255 (the culled items of a culling call, all in one
    // digit) are counted per wave: one LDS atomic instead of one per item on
    // a single address
    uint32_t n255 = threadIdx.x == 0 ? (uint32_t)(k.n - nv) : 0u;
#pragma unroll
    for (int r = 0; r < PER; r++) {
        const bool in = r * 256 + (int)threadIdx.x < nv;
        const uint32_t dg = (kv[r] >> shift) & 255;
        n255 += (uint32_t)__popcll(__ballot(in && dg == 255u));
        if (in && dg != 255u) atomicAdd(&h[dg], 1u);
    }
    if (lane_id() == 0 && n255) atomicAdd(&h[255], n255);
    __syncthreads();
    hist[k.hbase + (int64_t)threadIdx.x * k.hstride] = h[threadIdx.x];
}

// Exclusive scan of the (row, digit, block) histogram in chunks of 4096 entries:
// k_scan_local scans each chunk in LDS and records the chunk total, k_scan_top
// scans the chunk totals; the scatter adds both parts.
constexpr int SCAN_CHUNK = 4096;

// Inclusive prefix sum over the wave on DPP lane moves (every lane active):
// shifts by 1, 2, 4 and 8 lanes within each row of 16 (lanes with no source
// add 0), then the broadcasts of lane 15 to the next row and of lane 31 to
// the upper half.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

__global__ __launch_bounds__(1024) void k_scan_local(uint32_t *a, int64_t total, uint32_t *part) {
    __shared__ uint32_t wsum[16];
    int64_t c0 = (int64_t)blockIdx.x * SCAN_CHUNK;
    int tid = threadIdx.x;
    uint32_t v[4], s = 0;
    for (int k = 0; k < 4; k++) {
        int64_t i = c0 + 4 * tid + k;
        v[k] = i < total ? a[i] : 0u;
        s += v[k];
    }
    uint32_t inc = wave_incl_scan(s);
    if (lane_id() == 63) wsum[tid >> 6] = inc;
    __syncthreads();
    uint32_t wbase = 0;
    for (int w = 0; w < (tid >> 6); w++) wbase += wsum[w];
    uint32_t run = wbase + inc - s;
    for (int k = 0; k < 4; k++) {
        int64_t i = c0 + 4 * tid + k;
        if (i < total) a[i] = run;
        run += v[k];
    }
    if (tid == 1023) part[blockIdx.x] = wbase + inc;
}

__global__ __launch_bounds__(64) void k_scan_top(uint32_t *part, int64_t n) {
    uint32_t carry = 0;
    for (int64_t b = 0; b < n; b += 64) {
        int64_t i = b + lane_id();
        uint32_t v = i < n ? part[i] : 0u;
        uint32_t inc = wave_incl_scan(v);
        if (i < n) part[i] = carry + inc - v;
        carry += __shfl(inc, 63);
    }
}

// Stable scatter of one radix pass.  Wave w of a block ranks the block's
// quarter [w*Q, (w+1)*Q) in rounds of 64 items (8 ballots find the lanes with
// the same digit); per-wave running digit counts live in LDS, so ranking
// needs no block-wide barrier.  The block then places its items in LDS in
// digit order and writes each digit's run to consecutive global addresses.
// With at most 256 scan chunks the block scans the chunk totals itself
// (ncraw > 0: part holds raw totals), which saves the top-level scan launch.
// MODE 0: key and value in, key and value out (kout == nullptr: the last
// pass's keys, which nothing reads, are not written); MODE 1: key and value
// in, one word out (the next digit above the 24-bit value); MODE 2: words in
// and out (the digit is the top byte).
template <int RS_ITEMS, int MODE>
__global__ __launch_bounds__(256) void k_scatter(const uint32_t *kin, const int32_t *vin, uint32_t *kout,
                                                 int32_t *vout, SortSeg S, int shift,
                                                 const uint32_t *hist, const uint32_t *part, int ncraw,
                                                 int later) {
    using KT = uint32_t;
    constexpr int Q = RS_ITEMS / 4;   // items per wave
    constexpr int R = Q / 64;         // rounds per wave
    __shared__ uint32_t wc[4][256];   // per-wave digit counts, then per-wave offsets
    __shared__ uint32_t gbase[256];   // global position of the block's first item of each digit
    __shared__ uint32_t loff[256];    // block-local position of each digit's first item
    // staged items in digit order: MODE 0 keys and values, MODE 1 the output
    // words and each item's digit (a byte), MODE 2 words
    __shared__ KT skey[RS_ITEMS];
    constexpr bool V = MODE < 2;  // separate values in
    __shared__ int32_t sval[MODE == 0 ? RS_ITEMS : 1];
    __shared__ uint8_t sdig[MODE == 1 ? RS_ITEMS : 1];
    const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const SBlock sbk = sort_block(S, blk);
    const int64_t b0 = sbk.i0;
    // items of this block: [b0, n); in a culling call the kept ones only
    // (first in the block for the first pass, first in the row after it; the
    // culled ones keep their reserved places, digit 255 at the row's end,
    // unwritten)
    const int nvalid = later ? kept_in_block(S, sbk) : (S.bn ? S.bn[blk] : sbk.n);
    const int64_t n = b0 + nvalid;
    if (ncraw > 0) {
        // exclusive scan of the raw chunk totals (one per thread) into loff
        __shared__ uint32_t csum[4];
        uint32_t v = tid < ncraw ? part[tid] : 0u;
        uint32_t inc = wave_incl_scan(v);
        if (lane == 63) csum[w] = inc;
        __syncthreads();
        uint32_t pre = inc - v;
        for (int k = 0; k < w; k++) pre += csum[k];
        loff[tid] = pre;
        __syncthreads();
        int64_t e = sbk.hbase + (int64_t)tid * sbk.hstride;
        gbase[tid] = hist[e] + loff[e / SCAN_CHUNK];
        __syncthreads();
    } else {
        int64_t e = sbk.hbase + (int64_t)tid * sbk.hstride;
        gbase[tid] = hist[e] + part[e / SCAN_CHUNK];
    }
    for (int k = 0; k < 4; k++) wc[k][tid] = 0;
    __syncthreads();
    KT key[R];
    int32_t val[R];
    uint32_t rk[R];
    // issue every load of this thread before ranking (one memory latency)
#pragma unroll
    for (int r = 0; r < R; r++) {
        int64_t i = b0 + w * Q + r * 64 + lane;
        key[r] = i < n ? kin[i] : (KT)0;
        if (V) val[r] = i < n ? vin[i] : 0;
    }
    for (int r = 0; r < R; r++) {
        int64_t i = b0 + w * Q + r * 64 + lane;
        bool valid = i < n;
        uint32_t d = (uint32_t)((key[r] >> shift) & 255);
        unsigned long long peers = __ballot(valid);
        for (int bit = 0; bit < 8; bit++) {
            unsigned long long m = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? m : ~m;
        }
        uint32_t before = valid ? wc[w][d] : 0u;
        __builtin_amdgcn_wave_barrier();
        uint32_t rank = (uint32_t)__popcll(peers & lanes_below());
        rk[r] = valid ? before + rank : 0xffffffffu;
        if (valid && rank == 0) wc[w][d] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // digit totals -> block-local offsets (thread = digit), then per-wave offsets
    {
        uint32_t c0 = wc[0][tid], c1 = wc[1][tid], c2 = wc[2][tid], c3 = wc[3][tid];
        uint32_t tot = c0 + c1 + c2 + c3;
        uint32_t inc = wave_incl_scan(tot);
        __shared__ uint32_t wsum[4];
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t pre = inc - tot;
        for (int k = 0; k < w; k++) pre += wsum[k];
        loff[tid] = pre;
        wc[0][tid] = pre;
        wc[1][tid] = pre + c0;
        wc[2][tid] = pre + c0 + c1;
        wc[3][tid] = pre + c0 + c1 + c2;
    }
    __syncthreads();
    for (int r = 0; r < R; r++) {
        if (rk[r] == 0xffffffffu) continue;
        uint32_t d = (uint32_t)((key[r] >> shift) & 255);
        uint32_t slot = wc[w][d] + rk[r];
        if (MODE == 1) {
            skey[slot] = ((key[r] >> (shift + 8)) & 255u) << 24 | (uint32_t)val[r];
            sdig[slot] = (uint8_t)d;
        } else {
            skey[slot] = key[r];
            if (MODE == 0) sval[slot] = val[r];
        }
    }
    __syncthreads();
    for (int j = tid; j < nvalid; j += 256) {
        const KT k = skey[j];
        const uint32_t d = MODE == 1 ? (uint32_t)sdig[j] : (uint32_t)((k >> shift) & 255);
        const uint32_t pos = gbase[d] + (uint32_t)j - loff[d];
        if (MODE == 0) {
            if (kout) kout[pos] = k;
            vout[pos] = sval[j];
        } else {
            kout[pos] = k;
        }
    }
}

// Sort (keys[0], vals[0]) within rows by K's key bits; result in keys[res]
// (narrow sorts: words) or vals[res].  The first pass's histogram is already
// in `hist` (from the key kernel).
template <int RS_ITEMS>
static int radix_sort(uint32_t **keys, int32_t **vals, uint32_t *hist, uint32_t *part, const SortSeg &S,
                      const SortKey &K, hipStream_t s, KernelEvents *kev) {
    int cur = 0;
    if (S.nb == 0) return cur;
    const int nb = (int)S.nb;
    int64_t total = (int64_t)nb * 256;
    int nchunk = (int)((total + SCAN_CHUNK - 1) / SCAN_CHUNK);
    for (int p = 0; p < K.passes; p++) {
        const bool last = p == K.passes - 1;
        const int mode = !K.narrow ? 0 : last ? 2 : p == K.passes - 2 ? 1 : 0;
        const int shift = mode == 2 ? 24 : 8 * p;
        if (p > 0)
            hipLaunchKernelGGL((k_hist<RS_ITEMS>), dim3(nb), dim3(256), 0, s, keys[cur], S, shift, hist);
        hipLaunchKernelGGL(k_scan_local, dim3(nchunk), dim3(1024), 0, s, hist, total, part);
        const bool inline_top = nchunk <= 256;
        if (!inline_top)
            hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(64), 0, s, part, (int64_t)nchunk);
        if (kev) kev->begin(KE_SCATTER, s);
        const int ncr = inline_top ? nchunk : 0;
        const int later = p > 0 ? 1 : 0;
        if (mode == 2)
            hipLaunchKernelGGL((k_scatter<RS_ITEMS, 2>), dim3(nb), dim3(256), 0, s, keys[cur], nullptr,
                               keys[cur ^ 1], nullptr, S, shift, hist, part, ncr, later);
        else if (mode == 1)
            hipLaunchKernelGGL((k_scatter<RS_ITEMS, 1>), dim3(nb), dim3(256), 0, s, keys[cur], vals[cur],
                               keys[cur ^ 1], nullptr, S, shift, hist, part, ncr, later);
        else
            hipLaunchKernelGGL((k_scatter<RS_ITEMS, 0>), dim3(nb), dim3(256), 0, s, keys[cur], vals[cur],
                               last ? nullptr : keys[cur ^ 1], vals[cur ^ 1], S, shift, hist, part, ncr, later);
        if (kev) kev->end(KE_SCATTER, s);
        cur ^= 1;
    }
    return cur;
}

// The largest |x - o| (rounded to FP64) over a tile's coordinates x, from
// its box: rounding is monotone, so along each axis the largest offset is
// attained at the box's low or high end, and the value equals the maximum
// over the vertices themselves.
__device__ __forceinline__ double box_offset_max(const double (&lo)[3], const double (&hi)[3],
                                                 const double (&o)[3]) {
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++) m = fmax(m, fmax(hi[k] - o[k], o[k] - lo[k]));
    return m;
}

// Tiles: gather each tile's triangles in sorted order and write the slot
// triangle ids and the tile metadata (box, origin, storage error bound).  The
// coordinate copies of a large call are written later, for queued tiles only
// (most tiles of a large call are never queued); a small call, whose time is
// a chain of short launches, writes them here.
constexpr int64_t LAZY_COPY_MIN_TILES = 16384;

static bool lazy_copies(const SideBufs &A, const SideBufs &B) {
    return A.NT + B.NT >= LAZY_COPY_MIN_TILES;
}

struct TileJob {
    const double *xyz;
    const int32_t *tri;
    const int64_t *v_off, *t_off, *tile_off;
    int64_t G, NT;
    int tk;
    const int32_t *sorted;  // sorted items: triangle index within the side, or
                            // (packed) digit << 24 | index within the row
    int packed;
    int32_t *ids;  // triangle of each slot
    TileMeta *meta;
    uint32_t *mat;  // 0: no copies yet, 1: written here
    float *t32;     // copies written here (small calls), else nullptr
    double *t64;
    const int32_t *kc;  // triangles kept per row (a culling call: the first kc[g] of the
                        // row's sorted range; the metadata build only), else nullptr
};

// Lane l of the wave owns slots l and l + 64 (the second only for tk = 128);
// slots past the tile's last triangle repeat it, and slots past tk are not
// written.
template <bool TWO>
__device__ void tile_one(const TileJob &J, int64_t t) {
    const int lane = lane_id(), tk = J.tk;
    const int64_t g = wave_find_row(J.tile_off, J.G, t);
    const int64_t i = t - J.tile_off[g];
    const int64_t ntr = J.t_off[g + 1] - J.t_off[g];
    const int n = (int)min((int64_t)tk, ntr - i * tk);
    const double *X = J.xyz + 3 * J.v_off[g];
    const int64_t nvr = J.v_off[g + 1] - J.v_off[g];
    double v[2][9];
    double lo[3], hi[3], o[3];
    for (int k = 0; k < 3; k++) {
        lo[k] = __builtin_inf();
        hi[k] = -__builtin_inf();
    }
    // all loads of both slots first (one chain of memory latency); the loops
    // are unrolled so that the arrays stay in registers
    const bool two = TWO;
    int64_t tri_id[2] = {0, 0}, vi[2][3];
#pragma unroll
    for (int r = 0; r < 2; r++)
        if (r == 0 || two) {
            const int32_t w = J.sorted[J.t_off[g] + i * tk + min(lane + 64 * r, n - 1)];
            tri_id[r] = J.packed ? J.t_off[g] + (w & 0xffffff) : w;
        }
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int k = 0; k < 3; k++) vi[r][k] = (r == 0 || two) ? corner(J.tri, tri_id[r], k, nvr) : 0;
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const double *p = X + 3 * vi[r][k];
            v[r][3 * k] = (r == 0 || two) ? p[0] : 0.0;
            v[r][3 * k + 1] = (r == 0 || two) ? p[1] : 0.0;
            v[r][3 * k + 2] = (r == 0 || two) ? p[2] : 0.0;
        }
#pragma unroll
    for (int r = 0; r < 2; r++) {
        const int j = lane + 64 * r;
        if (j < tk) {
            J.ids[t * tk + j] = (int32_t)tri_id[r];
            for (int k = 0; k < 3; k++) {
                lo[k] = fmin(lo[k], fmin(v[r][k], fmin(v[r][3 + k], v[r][6 + k])));
                hi[k] = fmax(hi[k], fmax(v[r][k], fmax(v[r][3 + k], v[r][6 + k])));
            }
        }
    }
    for (int k = 0; k < 3; k++) {
        lo[k] = wave_min(lo[k]);
        hi[k] = wave_max(hi[k]);
        o[k] = (double)(float)(0.5 * lo[k] + 0.5 * hi[k]);
    }
    // rad = the largest magnitude of the tile's FP32 offsets from the origin,
    // (float)(x - o): rounding to FP32 is monotone and odd, so it is the
    // largest FP64 offset magnitude rounded once
    const double rad = (double)(float)box_offset_max(lo, hi, o);
    if (J.t32 || J.t64) {
#pragma unroll
        for (int r = 0; r < 2; r++) {
            const int j = lane + 64 * r;
            if (j >= tk) continue;
#pragma unroll
            for (int c = 0; c < 9; c++) {
                const int64_t at = (t * 9 + c) * tk + j;
                if (J.t32)
                    J.t32[at] = (float)(v[r][c] - o[c % 3]);
                else
                    J.t64[at] = v[r][c];
            }
        }
    }
    // Storage error of a coordinate: d = x - o is rounded to FP64 (relative
    // 2^-53) and then to FP32 (relative 2^-24, or 2^-150 absolute in the
    // subnormal range), so |f - d| <= (2^-24 + 2^-52) |d| + 2^-149 with
    // |d| <= rad (1 + 2^-22); a vertex (three coordinates) is within sqrt(3)
    // times that of its copy.
    const double err = 1.7321 * ((0x1p-24 + 0x1p-52) * rad * (1.0 + 0x1p-22) + 0x1p-149);
    if (lane == 0) {
        TileMeta m;
        for (int k = 0; k < 3; k++) {
            m.o[k] = o[k];
            m.lo[k] = lo[k];
            m.hi[k] = hi[k];
            m.rep[k] = v[0][k];
        }
        m.eps = (float)(err * (1.0 + 0x1p-20));
        m.rad = (float)rad;
        m.row = (int32_t)g;
        m.n = n;
        J.meta[t] = m;
        J.mat[t] = (J.t32 || J.t64) ? 1u : 0u;
    }
}

// Both sides in one launch, one wave per tile: waves [0, NT_A) build A's
// tiles, the rest B's.
template <bool TWO>
__global__ void k_tiles(TileJob A, TileJob B) {
    int64_t t = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (t < A.NT) tile_one<TWO>(A, t);
    else if (t - A.NT < B.NT) tile_one<TWO>(B, t - A.NT);
}

// The tile build of a large call (no copies): the tile's box, origin and
// radius need each of its vertices once, and a tile's triangles share most of
// them (about 40 distinct vertices for 64 triangles), so only the distinct
// vertices are gathered.  The slots' corner indices go into a hash table in
// LDS (linear probing, compare-and-swap from an empty key), the occupied
// entries are numbered with ballots, and each lane loads some of the distinct
// vertices: one 24-byte gather per distinct vertex instead of one per corner.
// The build is bound by vector instructions, most of them in the FP64
// min/max reductions of the box, so a wave builds M consecutive tiles of one
// side at once, lanes [m S, (m + 1) S) (S = 64 / M) working on tile m with
// TK / S slots each: one reduction over groups of S lanes serves all M tiles
// (a wave-wide reduction per tile cost twice the instructions).
constexpr uint32_t HASH_EMPTY = 0xffffffffu;
constexpr int TILE_META_M64 = 4;   // tiles per wave of the metadata build, 64-triangle tiles
constexpr int TILE_META_M128 = 2;  // and 128-triangle tiles

template <int TK, int M>
__device__ void tile_meta_group(const TileJob &J, int64_t t0, uint32_t *hk, int32_t *uv) {
    constexpr int S = 64 / M;         // lanes per tile
    constexpr int SL = TK / S;        // slots per lane
    constexpr int HS = 4 * TK;        // table entries per tile (at most 3 TK keys)
    constexpr int HB = TK == 32 ? 7 : (TK == 64 ? 8 : 9);  // log2(HS)
    constexpr int US = 3 * TK;        // distinct-vertex list per tile
    static_assert(M * S == 64 && SL * S == TK, "tile groups fill the wave");
    const int lane = lane_id();
    const int m = lane / S, sl = lane % S;
    // lanes of this lane's tile (contiguous), and those of them below it
    const unsigned long long gm = (S == 64 ? ~0ull : ((1ull << S) - 1ull)) << (m * S);
    const unsigned long long gbelow = gm & lanes_below();
    // rows: consecutive tiles mostly share one; search again only past its end
    int64_t g[M];
    g[0] = wave_find_row(J.tile_off, J.G, t0);
#pragma unroll
    for (int q = 1; q < M; q++) {
        g[q] = g[q - 1];
        if (t0 + q < J.NT && t0 + q >= J.tile_off[g[q] + 1]) g[q] = wave_find_row(J.tile_off, J.G, t0 + q);
    }
    // this lane's tile; one past the side's end (the last wave of a side)
    // repeats tile t0's loads and writes nothing
    const bool on = t0 + m < J.NT;
    int64_t gl = g[0];
#pragma unroll
    for (int q = 1; q < M; q++) gl = m == q ? g[q] : gl;
    if (!on) gl = g[0];
    const int64_t tl = on ? t0 + m : t0;
    const int64_t i = tl - J.tile_off[gl];
    const int64_t tlo = J.t_off[gl];
    // a culling call's tiles hold the row's kept triangles only; a tile past
    // them is empty (n = 0: it takes the row's first triangle, a real one,
    // builds an empty box and is never a candidate; the sorted range past
    // the kept items is not written)
    const int64_t nrow = J.kc ? (int64_t)J.kc[gl] : J.t_off[gl + 1] - tlo;
    const int n = (int)max((int64_t)0, min((int64_t)TK, nrow - i * TK));
    const bool live = on && n > 0;
    const int64_t pos = tlo + i * TK;
    const int64_t vb = J.v_off[gl];
    const int64_t nvr = J.v_off[gl + 1] - vb;
    const double *X = J.xyz + 3 * vb;
    // a wave whose tiles are all empty (the kept triangles lead each row, so
    // most waves past them hold no live tile) writes their metadata only:
    // the empty box and, as the representative, corner 0 of the first slot
    if (!__any(live)) {
        if (on && sl == S - 1) {
            const double *rv = X + 3 * corner(J.tri, tlo, 0, nvr);
            TileMeta mt;
            for (int k = 0; k < 3; k++) {
                mt.o[k] = 0.0;
                mt.lo[k] = __builtin_inf();
                mt.hi[k] = -__builtin_inf();
                mt.rep[k] = rv[k];
            }
            mt.eps = 0.0f;
            mt.rad = 0.0f;
            mt.row = (int32_t)gl;
            mt.n = 0;
            J.meta[tl] = mt;
            J.mat[tl] = 0u;
        }
        return;
    }
    int64_t tri_id[SL];
    uint32_t c[SL][3];
#pragma unroll
    for (int r = 0; r < SL; r++) {
        tri_id[r] = tlo;
        if (n > 0) {
            const int32_t w = J.sorted[pos + min(sl + S * r, n - 1)];
            tri_id[r] = J.packed ? tlo + (w & 0xffffff) : w;
        }
    }
#pragma unroll
    for (int q = 0; q < M * HS / 64; q++) hk[q * 64 + lane] = HASH_EMPTY;
#pragma unroll
    for (int r = 0; r < SL; r++)
#pragma unroll
        for (int k = 0; k < 3; k++) c[r][k] = (uint32_t)corner(J.tri, tri_id[r], k, nvr);
    // (an empty tile's slots are never read)
    if (live)
#pragma unroll
        for (int r = 0; r < SL; r++) J.ids[tl * TK + sl + S * r] = (int32_t)tri_id[r];
    wave_lds_sync();
    // insert every slot's corners into the tile's table; a table holds at
    // most 3/4 of its size in keys, so every probe ends
    uint32_t *ht = hk + m * HS;
    if (live)
#pragma unroll
        for (int r = 0; r < SL; r++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const uint32_t key = c[r][k];
                uint32_t h = (key * 2654435761u) >> (32 - HB);
                for (;;) {
                    const uint32_t old = atomicCAS(&ht[h], HASH_EMPTY, key);
                    if (old == HASH_EMPTY || old == key) break;
                    h = (h + 1) & (HS - 1);
                }
            }
    wave_lds_sync();
    // number the tile's distinct vertices in table order (at least one for a
    // tile that exists, none for one past the end)
    int32_t *ul = uv + m * US;
    int nu = 0;
#pragma unroll
    for (int q = 0; q < HS / S; q++) {
        const uint32_t key = ht[q * S + sl];
        const bool occ = key != HASH_EMPTY;
        const unsigned long long b = __ballot(occ);
        if (occ) ul[nu + __popcll(b & gbelow)] = (int32_t)key;
        nu += __popcll(b & gm);
    }
    wave_lds_sync();
    // gather them: lane sl of round q holds distinct vertex S q + sl of its
    // tile (rounds up to the largest count among the wave's tiles)
    int nmax = 0;
#pragma unroll
    for (int q = 0; q < M; q++) nmax = max(nmax, __builtin_amdgcn_readlane(nu, q * S));
    double lo[3], hi[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        lo[k] = __builtin_inf();
        hi[k] = -__builtin_inf();
    }
    for (int q = 0; q * S < nmax; q++) {  // (wave-uniform)
        const int u = q * S + sl;
        const bool in = u < nu;
        const double *pv = X + 3 * (int64_t)(in ? (uint32_t)ul[u] : c[0][0]);
        const double p0 = pv[0], p1 = pv[1], p2 = pv[2];
        lo[0] = in ? fmin(lo[0], p0) : lo[0];
        lo[1] = in ? fmin(lo[1], p1) : lo[1];
        lo[2] = in ? fmin(lo[2], p2) : lo[2];
        hi[0] = in ? fmax(hi[0], p0) : hi[0];
        hi[1] = in ? fmax(hi[1], p1) : hi[1];
        hi[2] = in ? fmax(hi[2], p2) : hi[2];
    }
    // the representative vertex: corner 0 of slot 0 (the tile's first lane),
    // as in the copying build
    const uint32_t c0 = (uint32_t)__shfl((int)c[0][0], m * S);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        lo[k] = group_min<S>(lo[k]);
        hi[k] = group_max<S>(hi[k]);
    }
    // the tile's last lane holds its box and writes its metadata (an empty
    // tile: the empty box, origin 0, radius and error 0)
    if (on && sl == S - 1) {
        double o[3] = {0.0, 0.0, 0.0};
        if (live)
            for (int k = 0; k < 3; k++) o[k] = (double)(float)(0.5 * lo[k] + 0.5 * hi[k]);
        // rad as in the copying build: the largest FP64 offset magnitude
        // rounded once to FP32 (the same set of coordinates)
        const double rad = live ? (double)(float)box_offset_max(lo, hi, o) : 0.0;
        const double err = live ? 1.7321 * ((0x1p-24 + 0x1p-52) * rad * (1.0 + 0x1p-22) + 0x1p-149) : 0.0;
        const double *rv = X + 3 * (int64_t)c0;
        TileMeta mt;
        for (int k = 0; k < 3; k++) {
            mt.o[k] = o[k];
            mt.lo[k] = lo[k];
            mt.hi[k] = hi[k];
            mt.rep[k] = rv[k];
        }
        mt.eps = (float)(err * (1.0 + 0x1p-20));
        mt.rad = (float)rad;
        mt.row = (int32_t)gl;
        mt.n = n;
        J.meta[tl] = mt;
        J.mat[tl] = 0u;
    }
}

// One wave per M tiles: waves [0, ceil(NT_A / M)) build A's tiles, the rest B's.
template <int TK, int M>
__global__ __launch_bounds__(256) void k_tiles_meta(TileJob A, TileJob B) {
    __shared__ uint32_t hk[4][M * 4 * TK];
    __shared__ int32_t uv[4][M * 3 * TK];
    const int w = threadIdx.x >> 6;
    const int64_t v = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 4 + w;
    const int64_t wa = (A.NT + M - 1) / M;
    if (v < wa) tile_meta_group<TK, M>(A, v * M, hk[w], uv[w]);
    else if ((v - wa) * M < B.NT) tile_meta_group<TK, M>(B, (v - wa) * M, hk[w], uv[w]);
}

template <int TK, int M>
static void launch_tiles_meta(const TileJob &ja, const TileJob &jb, hipStream_t s) {
    const int64_t waves = (ja.NT + M - 1) / M + (jb.NT + M - 1) / M;
    hipLaunchKernelGGL((k_tiles_meta<TK, M>), dim3(grid_for(waves, 4)), dim3(256), 0, s, ja, jb);
}

// Both sides are sorted in one sequence of launches (each row's items stay in
// the row's range).  Two 8-bit passes (16 Morton bits) while no row has more
// than 2^18 triangles, else three (24 bits): the key only orders work, and
// 16 bits already keep the tiles of such rows compact (the 4096-row batch
// evaluates about 1% more tile pairs than with 24 bits and saves a pass),
// while rows of millions of triangles need the finer cells (the 4M-triangle
// TIN against the 1M-triangle blob evaluates 258 tile pairs instead of 2
// with 16 bits).
SortKey sort_key(int64_t max_row_items) {
    SortKey K;
    K.passes = max_row_items <= ((int64_t)1 << 18) ? 2 : 3;
    K.mbits = 8 * K.passes;
    K.narrow = max_row_items <= ((int64_t)1 << 24);
    return K;
}

// Keys and the sort with RSI items per sort block (P.seg.rsi).
template <int RSI>
static int sort_items(SideBufs &A, SideBufs &B, PrepBufs &P, const SortKey &K, RowState *rows,
                      hipStream_t s, KernelEvents *kev) {
    // large sorts take their keys from per-vertex codes (P.vcode is then set)
    constexpr bool VC = RSI > RS_ITEMS;
    // culling (P.kc) comes with per-vertex codes only
    int32_t *kc = VC ? P.kc : nullptr;
    MortonSide ma{A.xyz, A.tri, A.nt, A.v_off, A.t_off, A.rowbox, P.vcode, kc, kc ? P.oc : nullptr};
    MortonSide mb{B.xyz, B.tri, B.nt, B.v_off, B.t_off, B.rowbox, VC ? P.vcode + A.nv : nullptr,
                  kc ? kc + A.G : nullptr, kc ? P.oc + A.nv : nullptr};
    if (VC) {
        const double *cub = kc ? P.cub : nullptr;
        VcodeSide ca{A.xyz, A.nv, A.v_off, A.rowbox, P.vcode, rowbox_blocks(A.nv), kc ? B.rowbox : nullptr, cub,
                     kc ? P.oc : nullptr};
        VcodeSide cb{B.xyz, B.nv, B.v_off, B.rowbox, P.vcode + A.nv, rowbox_blocks(B.nv), kc ? A.rowbox : nullptr, cub,
                     kc ? P.oc + A.nv : nullptr};
        if (cub && A.G > 0)
            hipLaunchKernelGGL(k_row_ub, dim3(grid_for(A.G, 4)), dim3(256), 0, s,
                               UbSide{A.xyz, A.tri, A.v_off, A.t_off, A.rowbox},
                               UbSide{B.xyz, B.tri, B.v_off, B.t_off, B.rowbox}, A.G, A.boxrep, P.cub);
        if (ca.nblk + cb.nblk > 0 && kc)
            hipLaunchKernelGGL(k_vcode<true>, dim3(ca.nblk + cb.nblk), dim3(256), 0, s, ca, cb, A.G, A.boxrep);
        else if (ca.nblk + cb.nblk > 0)
            hipLaunchKernelGGL(k_vcode<false>, dim3(ca.nblk + cb.nblk), dim3(256), 0, s, ca, cb, A.G, A.boxrep);
    }
    if (P.seg.tab && P.seg.nb > 0)
        hipLaunchKernelGGL(k_sort_table, dim3(grid_for(P.seg.nb, 256)), dim3(256), 0, s, P.seg);
    // at least one block: the key kernel also starts the row states
    const int grid = P.seg.nb > 0 ? (int)P.seg.nb : 1;
    if (K.narrow)
        hipLaunchKernelGGL((k_morton<RSI, VC, true>), dim3(grid), dim3(1024), 0, s, ma, mb, P.seg, K.mbits,
                           P.keys[0], P.vals[0], P.hist, A.boxrep, A.G, rows, P.flags);
    else
        hipLaunchKernelGGL((k_morton<RSI, VC, false>), dim3(grid), dim3(1024), 0, s, ma, mb, P.seg, K.mbits,
                           P.keys[0], P.vals[0], P.hist, A.boxrep, A.G, rows, P.flags);
    return radix_sort<RSI>(P.keys, P.vals, P.hist, P.part, P.seg, K, s, kev);
}

void launch_prep(SideBufs &A, SideBufs &B, PrepBufs &P, const SortKey &K, RowState *rows,
                 hipStream_t s, KernelEvents *kev) {
    if (A.G == 0) return;
    // smaller sort blocks shorten each block's serial ranking on small sorts;
    // larger ones write longer contiguous runs on big sorts (and take their
    // keys from the per-vertex code buffer)
    const int cur = P.seg.rsi == RS_ITEMS ? sort_items<RS_ITEMS>(A, B, P, K, rows, s, kev)
                                          : sort_items<2 * RS_ITEMS>(A, B, P, K, rows, s, kev);
    if (kev) kev->begin(KE_TILES, s);
    if (A.NT + B.NT > 0) {
        const int32_t *sorted = K.narrow ? (const int32_t *)P.keys[cur] : P.vals[cur];
        const int pk = K.narrow ? 1 : 0;
        const bool lazy = lazy_copies(A, B);
        // (a culling call is a large sort, so its copies are lazy)
        TileJob ja{A.xyz, A.tri, A.v_off, A.t_off, A.tile_off, A.G, A.NT, A.tk, sorted, pk, A.ids,
                   A.meta, A.mat, lazy ? nullptr : A.t32, lazy ? nullptr : A.t64, P.kc};
        TileJob jb{B.xyz, B.tri, B.v_off, B.t_off, B.tile_off, B.G, B.NT, B.tk, sorted + A.nt, pk,
                   B.ids, B.meta, B.mat, lazy ? nullptr : B.t32, lazy ? nullptr : B.t64,
                   P.kc ? P.kc + A.G : nullptr};
        // one slot per lane below 128-triangle tiles: fewer registers, more
        // waves in flight for the gathers
        const dim3 grid(grid_for(A.NT + B.NT, 4));
        if (lazy) {
            // the metadata build: tiles per wave by tile size
            if (A.tk == 128) launch_tiles_meta<128, TILE_META_M128>(ja, jb, s);
            else if (A.tk == 64) launch_tiles_meta<64, TILE_META_M64>(ja, jb, s);
            else launch_tiles_meta<32, 4>(ja, jb, s);
        } else if (A.tk > 64) {
            hipLaunchKernelGGL(k_tiles<true>, grid, dim3(256), 0, s, ja, jb);
        } else {
            hipLaunchKernelGGL(k_tiles<false>, grid, dim3(256), 0, s, ja, jb);
        }
    }
    if (kev) kev->end(KE_TILES, s);
}

// Coordinate copies of the queued tiles.  Lane l of wave w takes queue
// entries (64 k + l) W + w (W waves), so that a short queue spreads over many
// waves; a lane claims each of its entry's two tiles by swapping its word to
// 1, and the wave then writes the tiles whose claim returned 0, NG at a time
// with the loads of all NG in flight together: slot ids, corner indices and
// FP64 vertices gathered as in the tile build, written as FP32 offsets from
// the tile's origin (PREC 0: the same values the tile's box and error bound
// were computed from) or as the FP64 coordinates (PREC 1).
struct MatSide {
    const double *xyz;
    const int32_t *tri;
    const int64_t *v_off;
    const int32_t *ids;
    const TileMeta *meta;
    float *t32;
    double *t64;
    uint32_t *mat;
};

// Up to NG tiles of one side taken from the wave's claim mask m (cleared as
// they are taken); lane l's claimed tile is tl.
template <int PREC, int TK, int NG>
__device__ void mat_group(const MatSide &S, unsigned long long &m, int tl) {
    constexpr int R = TK > 64 ? 2 : 1;
    const int lane = lane_id();
    int t[NG];
#pragma unroll
    for (int i = 0; i < NG; i++) {
        t[i] = -1;
        if (m) {
            t[i] = __builtin_amdgcn_readlane(tl, __ffsll((long long)m) - 1);
            m &= m - 1;
        }
    }
    int64_t vb[NG], id[NG][R];
    int32_t vi[NG][R][3];
    double v[NG][R][9];
#pragma unroll
    for (int i = 0; i < NG; i++) {
        vb[i] = 0;
        if (t[i] < 0) continue;
#pragma unroll
        for (int r = 0; r < R; r++) id[i][r] = S.ids[(int64_t)t[i] * TK + min(lane + 64 * r, TK - 1)];
    }
#pragma unroll
    for (int i = 0; i < NG; i++) {
        if (t[i] < 0) continue;
        const int64_t g = S.meta[t[i]].row;
        vb[i] = S.v_off[g];
        const int64_t nvr = S.v_off[g + 1] - vb[i];
#pragma unroll
        for (int r = 0; r < R; r++)
#pragma unroll
            for (int k = 0; k < 3; k++) vi[i][r][k] = (int32_t)corner(S.tri, id[i][r], k, nvr);
    }
#pragma unroll
    for (int i = 0; i < NG; i++) {
        if (t[i] < 0) continue;
        const double *X = S.xyz + 3 * vb[i];
#pragma unroll
        for (int r = 0; r < R; r++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const double *p = X + 3 * (int64_t)vi[i][r][k];
                v[i][r][3 * k] = p[0];
                v[i][r][3 * k + 1] = p[1];
                v[i][r][3 * k + 2] = p[2];
            }
    }
#pragma unroll
    for (int i = 0; i < NG; i++) {
        if (t[i] < 0) continue;
        const TileMeta &mt = S.meta[t[i]];
        const double o[3] = {mt.o[0], mt.o[1], mt.o[2]};
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int j = lane + 64 * r;
            if (j >= TK) continue;
#pragma unroll
            for (int c = 0; c < 9; c++) {
                const int64_t at = ((int64_t)t[i] * 9 + c) * TK + j;
                if (PREC == 0)
                    S.t32[at] = (float)(v[i][r][c] - o[c % 3]);
                else
                    S.t64[at] = v[i][r][c];
            }
        }
    }
}

template <int PREC, int TK>
__global__ __launch_bounds__(256) void k_materialize(MatSide A, MatSide B, Lists L) {
    constexpr int NG = TK > 64 ? 2 : 4;
    const int64_t n = min(*L.qcount, L.qcap);
    const int lane = lane_id();
    const int64_t W = (int64_t)gridDim.x * 4, w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    for (int64_t k = 0; k * 64 * W + w < n; k++) {
        const int64_t e = (k * 64 + lane) * W + w;
        int ta = -1, tb = -1;
        if (e < n) {
            const int2 q = L.queue[e];
            ta = q.x;
            tb = q.y;
        }
        // a plain read first: most tiles of a busy queue were claimed already
        const bool ca = ta >= 0 && A.mat[ta] == 0u && atomicExch(&A.mat[ta], 1u) == 0u;
        const bool cb = tb >= 0 && B.mat[tb] == 0u && atomicExch(&B.mat[tb], 1u) == 0u;
        unsigned long long ma = __ballot(ca), mb = __ballot(cb);
        if ((ma | mb) && lane == 0)
            atomicAdd(&L.counters[C_COPIED], (unsigned long long)(__popcll(ma) + __popcll(mb)));
        while (ma) mat_group<PREC, TK, NG>(A, ma, ta);
        while (mb) mat_group<PREC, TK, NG>(B, mb, tb);
    }
}

void launch_materialize(SideBufs &A, SideBufs &B, const Lists &L, int prec, int grid, hipStream_t s) {
    if (A.NT == 0 || B.NT == 0 || !lazy_copies(A, B)) return;
    const MatSide ma{A.xyz, A.tri, A.v_off, A.ids, A.meta, A.t32, A.t64, A.mat};
    const MatSide mb{B.xyz, B.tri, B.v_off, B.ids, B.meta, B.t32, B.t64, B.mat};
    const dim3 gr(grid), bl(256);
#define SD3_MAT(P, T) hipLaunchKernelGGL((k_materialize<P, T>), gr, bl, 0, s, ma, mb, L)
    if (prec == 0) {
        if (A.tk == 128) SD3_MAT(0, 128);
        else if (A.tk == 64) SD3_MAT(0, 64);
        else SD3_MAT(0, 32);
    } else {
        if (A.tk == 128) SD3_MAT(1, 128);
        else if (A.tk == 64) SD3_MAT(1, 64);
        else SD3_MAT(1, 32);
    }
#undef SD3_MAT
}

// ---------------------------------------------------------------------------
// row state
// ---------------------------------------------------------------------------
// Row state from the two row boxes (6 ordered-bit values each).
__device__ void row_init_vals(RowState *rows, int64_t g, const unsigned long long *bA,
                              const unsigned long long *bB) {
    RowState r;
    r.ub = double_to_bits(__builtin_inf());
    r.d2 = double_to_bits(__builtin_inf());
    r.hit = 0;
    r.seed_q = -1;
    r.best = ~0ull;
    r.scale = 0.0;
    double ext2 = 0.0;
    bool ok = bA[0] != ~0ull && bB[0] != ~0ull;
    if (ok) {
        for (int k = 0; k < 3; k++) {
            double lo = fmin(from_ordered_bits(bA[k]), from_ordered_bits(bB[k]));
            double hi = fmax(from_ordered_bits(bA[3 + k]), from_ordered_bits(bB[3 + k]));
            ext2 += (hi - lo) * (hi - lo);
        }
    }
    r.margin_scale = 0x1p-36 * sqrt(ext2) * 1.01;
    rows[g] = r;
}


// ---------------------------------------------------------------------------
// a3: tile-pair bounds and the work queue
// ---------------------------------------------------------------------------
// A work item is (row, block of 64 A tiles, chunk of 256 B tiles); the A
// tiles' boxes sit in LDS and each thread walks them against its B tile.
struct WorkItem {
    int64_t g, a0, na, b;
    bool bvalid;
};

__device__ __forceinline__ WorkItem decode_item(const int64_t *wi_off, int64_t G, int64_t wi,
                                                const int64_t *tA, const int64_t *tB) {
    WorkItem w;
    w.g = find_row(wi_off, G, wi);
    int64_t local = wi - wi_off[w.g];
    int64_t nA = tA[w.g + 1] - tA[w.g], nB = tB[w.g + 1] - tB[w.g];
    int64_t nbc = (nB + 255) / 256;
    int64_t ab = local / nbc, bc = local % nbc;
    w.a0 = tA[w.g] + ab * 64;
    w.na = min((int64_t)64, nA - ab * 64);
    int64_t bl = bc * 256 + threadIdx.x;
    w.bvalid = bl < nB;
    w.b = tB[w.g] + (w.bvalid ? bl : 0);
    return w;
}

__device__ __forceinline__ double box_gap2(const double *alo, const double *ahi, const double *blo,
                                           const double *bhi) {
    double s = 0.0;
    for (int k = 0; k < 3; k++) {
        double gp = fmax(0.0, fmax(blo[k] - ahi[k], alo[k] - bhi[k]));
        s += gp * gp;
    }
    return s;
}

// Boxes of tile groups: 64 consecutive tiles of a row on the A side (one work
// item's A block), 256 on the B side (one work item's B chunk).
__device__ void group_box(const TileMeta *meta, const int64_t *tile_off, const int64_t *grp_off,
                          int64_t G, int gs, GroupBox *out, int64_t gid) {
    __shared__ double red[4][6];
    int64_t g = find_row(grp_off, G, gid);
    int64_t t0 = tile_off[g] + (gid - grp_off[g]) * gs;
    int64_t t1 = min(t0 + gs, tile_off[g + 1]);
    int64_t t = t0 + threadIdx.x;
    bool valid = threadIdx.x < gs && t < t1;
    double lo[3], hi[3];
    for (int k = 0; k < 3; k++) {
        lo[k] = valid ? meta[t].lo[k] : __builtin_inf();
        hi[k] = valid ? meta[t].hi[k] : -__builtin_inf();
        lo[k] = wave_min(lo[k]);
        hi[k] = wave_max(hi[k]);
    }
    if (lane_id() == 0)
        for (int k = 0; k < 3; k++) {
            red[threadIdx.x >> 6][k] = lo[k];
            red[threadIdx.x >> 6][3 + k] = hi[k];
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        GroupBox b;
        for (int k = 0; k < 3; k++) {
            b.lo[k] = fmin(fmin(red[0][k], red[1][k]), fmin(red[2][k], red[3][k]));
            b.hi[k] = fmax(fmax(red[0][3 + k], red[1][3 + k]), fmax(red[2][3 + k], red[3][3 + k]));
            b.rep[k] = meta[t0].rep[k];
        }
        out[gid] = b;
    }
}

// Blocks [0, nblkA) build A's block boxes, the rest B's chunk boxes.
__global__ __launch_bounds__(256) void k_group_boxes(const TileMeta *mA, const int64_t *tA,
                                                     const int64_t *blkA, int64_t nblkA,
                                                     const TileMeta *mB, const int64_t *tB,
                                                     const int64_t *chkB, int64_t G,
                                                     GroupBox *gA, GroupBox *gB) {
    if ((int64_t)blockIdx.x < nblkA) group_box(mA, tA, blkA, G, 64, gA, blockIdx.x);
    else group_box(mB, tB, chkB, G, 256, gB, blockIdx.x - nblkA);
}

void launch_group_boxes(const SideBufs &A, const SideBufs &B, const QueueGeo &Q, int64_t nblkA,
                        int64_t nchkB, hipStream_t s) {
    if (nblkA + nchkB > 0)
        hipLaunchKernelGGL(k_group_boxes, dim3((unsigned)(nblkA + nchkB)), dim3(256), 0, s, A.meta,
                           A.tile_off, Q.blkA, nblkA, B.meta, B.tile_off, Q.chkB, A.G, Q.gA, Q.gB);
}

// Per work item: box lower bound of its (A block, B chunk) pair, kept for the
// tile-level kernels, and the distance between two real vertices (an upper
// bound of the row distance).
__global__ void k_wi_seed(const GroupBox *gA, const GroupBox *gB, const int64_t *blkA,
                          const int64_t *chkB, const int64_t *tA, const int64_t *tB,
                          const int64_t *wi_off, int64_t G, int64_t n_wi, RowState *rows,
                          float *wi_lb, int update_ub) {
    int64_t wi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    // lanes past the end stay in the wave for the reduction below; lane 0 of
    // a wave is past the end only when the whole wave is
    if (__shfl((int)(wi < n_wi), 0) == 0) return;
    const bool valid = wi < n_wi;
    int64_t g = -1;
    double u = __builtin_inf();
    if (valid) {
        g = find_row(wi_off, G, wi);
        int64_t local = wi - wi_off[g];
        int64_t nB = tB[g + 1] - tB[g];
        int64_t nbc = (nB + 255) / 256;
        const GroupBox &a = gA[blkA[g] + local / nbc];
        const GroupBox &b = gB[chkB[g] + local % nbc];
        double g2 = box_gap2(a.lo, a.hi, b.lo, b.hi);
        wi_lb[wi] = (float)(sqrt(g2) * (1.0 - 8.0 * U64) * (1.0 - 0x1p-20));
        double dx = a.rep[0] - b.rep[0], dy = a.rep[1] - b.rep[1], dz = a.rep[2] - b.rep[2];
        u = sqrt(dx * dx + dy * dy + dz * dz) * (1.0 + 8.0 * U64);
    }
    if (!update_ub) return;
    const int64_t g0 = __shfl(g, 0);
    if (__all(!valid || g == g0)) {
        // one row for the whole wave: one atomic instead of 64
        u = wave_min(u);
        if (lane_id() == 0 && u < bits_to_double(load_acq(&rows[g0].ub))) atomic_min_pos(&rows[g0].ub, u);
    } else if (valid && u < bits_to_double(load_acq(&rows[g].ub))) {
        atomic_min_pos(&rows[g].ub, u);
    }
}

// The work items whose group bound may still hold the row minimum (distance:
// lower bound <= ub + m; intersects: overlapping groups), compacted: in the
// tile-level kernels that follow, the useful workgroups come first and every
// other one exits after one load instead of a row search (used with many
// rows, where that search is long).
__device__ __forceinline__ void row_scale(RowState *rows, int64_t g);

// With scale_rows, the same launch also sets every row's feature length scale.
__global__ void k_wi_compact(const float *wi_lb, const int64_t *wi_off, int64_t G, int64_t n_wi,
                             const RowState *rows, int mode, int32_t *list, unsigned int *count,
                             RowState *scale_rows) {
    int64_t wi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (scale_rows && wi < G) row_scale(scale_rows, wi);
    bool keep = false;
    if (wi < n_wi) {
        int64_t g = find_row(wi_off, G, wi);
        double lb = (double)wi_lb[wi];
        if (mode == 1) {
            keep = lb <= 0.0;
        } else {
            const RowState &R = rows[g];
            double ub = bits_to_double(R.ub);
            keep = lb <= ub + row_margin(R, ub);
        }
    }
    unsigned long long m = __ballot(keep);
    if (m == 0) return;
    unsigned int base = 0;
    if (lane_id() == 0) base = atomicAdd(count, (unsigned int)__popcll(m));
    base = __shfl(base, 0);
    if (keep) list[base + __popcll(m & lanes_below())] = (int32_t)wi;
}

// True when the whole work item can be skipped.  The row bound is read by
// thread 0 only and broadcast through LDS: other workgroups lower it
// concurrently, and every thread of the block must take the same branch.
__device__ __forceinline__ bool wi_pruned(const float *wi_lb, int64_t wi, const RowState &R,
                                          int mode) {
    __shared__ int flag;
    if (threadIdx.x == 0) {
        double lb = (double)wi_lb[wi];
        if (mode == 1) {
            flag = lb > 0.0;
        } else {
            double ub = bits_to_double(load_acq(&R.ub));
            flag = lb > ub + row_margin(R, ub);
        }
    }
    __syncthreads();
    return flag != 0;
}

// Upper bound seed: the distance between two real vertices bounds the row
// distance from above.  Over the compacted list (wlist) or every work item.
__global__ __launch_bounds__(256) void k_ub_seed(const TileMeta *mA, const TileMeta *mB,
                                                 const int64_t *tA, const int64_t *tB,
                                                 const int64_t *wi_off, int64_t G,
                                                 RowState *rows, const float *wi_lb,
                                                 const int32_t *wlist, const unsigned int *wcount) {
    __shared__ double rep[64][3];
    int64_t wi = blockIdx.x;  // without a list: one block per work item
    if (wlist) {
        if (blockIdx.x >= *wcount) return;
        wi = wlist[blockIdx.x];
    }
    WorkItem w = decode_item(wi_off, G, wi, tA, tB);
    if (wi_pruned(wi_lb, wi, rows[w.g], 0)) return;
    if (threadIdx.x < w.na)
        for (int k = 0; k < 3; k++) rep[threadIdx.x][k] = mA[w.a0 + threadIdx.x].rep[k];
    __syncthreads();
    double best = __builtin_inf();
    if (w.bvalid) {
        double bp[3];
        for (int k = 0; k < 3; k++) bp[k] = mB[w.b].rep[k];
        for (int a = 0; a < w.na; a++) {
            double dx = rep[a][0] - bp[0], dy = rep[a][1] - bp[1], dz = rep[a][2] - bp[2];
            best = fmin(best, dx * dx + dy * dy + dz * dz);
        }
    }
    __shared__ double wred[4];
    best = wave_min(best);
    if (lane_id() == 0) wred[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        best = fmin(fmin(wred[0], wred[1]), fmin(wred[2], wred[3]));
        if (best < __builtin_inf()) {
            double u = sqrt(best) * (1.0 + 8.0 * U64);
            if (u < bits_to_double(load_acq(&rows[w.g].ub))) atomic_min_pos(&rows[w.g].ub, u);
        }
    }
}

// Keep the tile pairs that may hold the minimum (distance: box lower bound
// <= ub + m) or a contact (intersects: closed boxes overlap).
__device__ __forceinline__ uint32_t float_order_bits(float f) {
    uint32_t b = __float_as_uint(f);
    return (b >> 31) ? ~b : (b | 0x80000000u);
}

// Tile-pair box filter of one work item (thread = B tile, loop over the A
// block's tiles) into the queue.  With RANK 1 the same launch also chooses
// each row's seed: the kept entry with the smallest box bound, combined per
// wave and published with one atomicMin per wave on the row's choice (ordered
// bound bits << 32 | queue index).
template <int RANK>
__global__ __launch_bounds__(256) void k_filter(const TileMeta *mA, const TileMeta *mB,
                                                const int64_t *tA, const int64_t *tB,
                                                const int64_t *wi_off, int64_t G, int64_t wi0,
                                                RowState *rows, int mode, int2 *queue,
                                                float *qlb, unsigned int *qcount,
                                                unsigned int qcap, const float *wi_lb,
                                                const int32_t *wlist, const unsigned int *wcount,
                                                RowState *scale_rows) {
    __shared__ double box[64][6];
    // block 0 of the first uncompacted pass also sets the rows' feature scale
    if (scale_rows && blockIdx.x == 0)
        for (int64_t g = threadIdx.x; g < G; g += blockDim.x) row_scale(scale_rows, g);
    int64_t wi;
    if (wlist) {
        if (blockIdx.x >= *wcount) return;
        wi = wlist[blockIdx.x];
    } else {
        wi = wi0 + blockIdx.x;
    }
    WorkItem w = decode_item(wi_off, G, wi, tA, tB);
    if (wi_pruned(wi_lb, wi, rows[w.g], mode)) return;
    if (threadIdx.x < w.na)
        for (int k = 0; k < 3; k++) {
            box[threadIdx.x][k] = mA[w.a0 + threadIdx.x].lo[k];
            box[threadIdx.x][3 + k] = mA[w.a0 + threadIdx.x].hi[k];
        }
    __syncthreads();
    double blo[3], bhi[3];
    for (int k = 0; k < 3; k++) {
        blo[k] = mB[w.b].lo[k];
        bhi[k] = mB[w.b].hi[k];
    }
    const RowState &R = rows[w.g];
    double ub = bits_to_double(R.ub);  // final after the seed kernels (previous launch)
    double lim = ub + row_margin(R, ub);
    // keep iff sqrt(g2) (1 - 8u) <= lim; compared squared with slack, the square
    // root is taken only for kept pairs
    double lim2 = lim * lim * (1.0 + 32.0 * U64);
    bool hit = R.hit != 0;
    unsigned long long best = ~0ull;  // this wave's seed candidate
    // groups of FG A tiles share one queue claim (their entries keep the
    // per-tile order, a-major then lane)
    constexpr int FG = 8;
    for (int a0 = 0; a0 < w.na; a0 += FG) {
        float lbf[FG];
        unsigned long long m[FG];
        unsigned int tot = 0;
#pragma unroll
        for (int j = 0; j < FG; j++) {
            const int a = a0 + j;
            bool keep = false;
            lbf[j] = 0.0f;
            if (a < w.na && w.bvalid && !hit) {
                double g2 = box_gap2(box[a], box[a] + 3, blo, bhi);
                if (mode == 0) {
                    keep = g2 <= lim2;
                    if (keep) lbf[j] = (float)(sqrt(g2) * (1.0 - 8.0 * U64) * (1.0 - 0x1p-20));
                } else {
                    keep = g2 == 0.0 && box[a][0] <= bhi[0] && blo[0] <= box[a][3] &&
                           box[a][1] <= bhi[1] && blo[1] <= box[a][4] && box[a][2] <= bhi[2] &&
                           blo[2] <= box[a][5];
                }
            }
            m[j] = __ballot(keep);
            tot += (unsigned int)__popcll(m[j]);
        }
        if (tot == 0) continue;
        unsigned int basei = 0;
        if (lane_id() == 0) basei = atomicAdd(qcount, tot);
        basei = __builtin_amdgcn_readfirstlane(basei);
#pragma unroll
        for (int j = 0; j < FG; j++) {
            const bool keep = (m[j] >> lane_id()) & 1ull;
            const unsigned int idx = basei + (unsigned int)__popcll(m[j] & lanes_below());
            basei += (unsigned int)__popcll(m[j]);
            if (keep && idx < qcap) {
                queue[idx] = make_int2((int)(w.a0 + a0 + j), (int)w.b);
                qlb[idx] = lbf[j];
            }
            if (RANK == 1 && keep && idx < qcap)
                best = min(best, ((unsigned long long)float_order_bits(lbf[j]) << 32) | idx);
        }
    }
    if (RANK == 1) {
        best = wave_min(best);
        if (lane_id() == 0 && best != ~0ull && best < rows[w.g].best) atomicMin(&rows[w.g].best, best);
    }
}

template <int RANK>
static void launch_filter(const SideBufs &A, const SideBufs &B, const QueueGeo &Q, int64_t n_wi,
                          int64_t wi_begin, RowState *rows, Lists &L, int mode, hipStream_t s) {
    const unsigned nb = (unsigned)n_wi;
    if (Q.compact) {
        // single pass over all work items: compact the survivors of the group
        // bound first (the count is read on the device)
        const int64_t nthreads = mode == 0 && n_wi < A.G ? A.G : n_wi;
        hipLaunchKernelGGL(k_wi_compact, dim3(grid_for(nthreads, 256)), dim3(256), 0, s, Q.wi_lb,
                           Q.wi_off, A.G, n_wi, rows, mode, Q.wlist, Q.wcount + 1,
                           mode == 0 ? rows : (RowState *)nullptr);
        hipLaunchKernelGGL(k_filter<RANK>, dim3(nb), dim3(256), 0, s, A.meta, B.meta, A.tile_off,
                           B.tile_off, Q.wi_off, A.G, (int64_t)0, rows, mode, L.queue, L.qlb,
                           L.qcount, L.qcap, Q.wi_lb, Q.wlist, Q.wcount + 1,
                           (RowState *)nullptr);
    } else {
        hipLaunchKernelGGL(k_filter<RANK>, dim3(nb), dim3(256), 0, s, A.meta, B.meta, A.tile_off,
                           B.tile_off, Q.wi_off, A.G, wi_begin, rows, mode, L.queue, L.qlb,
                           L.qcount, L.qcap, Q.wi_lb, (const int32_t *)nullptr,
                           (const unsigned int *)nullptr,
                           mode == 0 && wi_begin == 0 ? rows : (RowState *)nullptr);
    }
}

void launch_queue(const SideBufs &A, const SideBufs &B, const QueueGeo &Q, int64_t n_wi,
                  int64_t wi_begin, RowState *rows, Lists &L, int what, hipStream_t s, int rank) {
    if (n_wi <= 0) return;
    const unsigned nb = (unsigned)n_wi;
    if (what == Q_SEED || what == Q_GROUPS) {
        hipLaunchKernelGGL(k_wi_seed, dim3(grid_for(n_wi, 256)), dim3(256), 0, s, Q.gA, Q.gB, Q.blkA,
                           Q.chkB, A.tile_off, B.tile_off, Q.wi_off, A.G, n_wi, rows, Q.wi_lb,
                           what == Q_SEED ? 1 : 0);
        if (what == Q_SEED && Q.compact) {
            hipLaunchKernelGGL(k_wi_compact, dim3(grid_for(n_wi, 256)), dim3(256), 0, s, Q.wi_lb,
                               Q.wi_off, A.G, n_wi, rows, 0, Q.wlist, Q.wcount, (RowState *)nullptr);
            hipLaunchKernelGGL(k_ub_seed, dim3(nb), dim3(256), 0, s, A.meta, B.meta, A.tile_off,
                               B.tile_off, Q.wi_off, A.G, rows, Q.wi_lb, Q.wlist, Q.wcount);
        } else if (what == Q_SEED) {
            hipLaunchKernelGGL(k_ub_seed, dim3(nb), dim3(256), 0, s, A.meta, B.meta, A.tile_off,
                               B.tile_off, Q.wi_off, A.G, rows, Q.wi_lb, (const int32_t *)nullptr,
                               (const unsigned int *)nullptr);
        }
        return;
    }
    const int mode = what == Q_FILTER_DIST ? 0 : 1;
    if (rank == 1) launch_filter<1>(A, B, Q, n_wi, wi_begin, rows, L, mode, s);
    else launch_filter<0>(A, B, Q, n_wi, wi_begin, rows, L, mode, s);
}

// ---------------------------------------------------------------------------
// a4-a7: triangle-pair passes over the queue (persistent workgroups)
// ---------------------------------------------------------------------------
// Per-tile-pair constants of the FP32 pass (see sd3_pair32.h for the model)
// for tile a shifted into tile b's frame (the pair pass calls it with its B
// tile as a, so that its A tile's staged copy is kept across consecutive
// entries of the same A tile; the model is symmetric in the two tiles
// otherwise); eps_c bounds how far the real
// triangles are from their FP32 copies; eu / elb bound the evaluation error of
// the upper / lower bounds; eo bounds the error of FP32 orientation values.
struct TP32 {
    float sh[3];
    float eu, elb, eps_f, box_tol;
    double eps_c;
};

__device__ __forceinline__ TP32 tp32_consts(const TileMeta &a, const TileMeta &b) {
    TP32 c;
    double dinf = 0.0;
    for (int k = 0; k < 3; k++) {
        double d = a.o[k] - b.o[k];
        c.sh[k] = (float)d;
        dinf = fmax(dinf, fabs(d));
    }
    double Ra = a.rad, Rb = b.rad;
    double MA = (Ra + dinf) * (1.0 + 2.0 * U32) + 1e-30;
    double epsA = a.eps + SQRT3 * (U32 * (Ra + 2.01 * dinf) + 2.0 * U64 * dinf);
    double eps_c = (epsA + b.eps) * (1.0 + 1e-6);
    double Mr = MA + Rb;
    double Mw = Mr + 4.0 * fmax(Ra + 2.0 * U32 * MA, Rb);
    c.eps_c = eps_c;
    c.eu = (float)((8.0 * SQRT3 * U32 * Mw + eps_c) * (1.0 + 1e-5));
    c.elb = (float)((16.0 * SQRT3 * U32 * Mr + eps_c) * (1.0 + 1e-5));
    c.eps_f = (float)(eps_c * (1.0 + 1e-5));
    c.box_tol = (float)((eps_c + 4.0 * U32 * Mr) * (1.0 + 1e-5));
    return c;
}

// Ranker features of a tile pair, length-normalised by the row scale (the
// vertex-pair upper bound after seeding) and compressed with log2(1 + x):
// box lower bound, the two tiles' box extents, box-centre distance, and the
// two real triangle counts (in units of 64 triangles).
__device__ __forceinline__ void tp_features(const TileMeta &a, const TileMeta &b, double scale,
                                            float lbf, float *f) {
    double s = scale > 0.0 ? 1.0 / scale : 1.0;
    double c2 = 0.0;
    f[0] = log2f(1.0f + (float)(lbf * s));
    for (int k = 0; k < 3; k++) {
        f[1 + k] = log2f(1.0f + (float)((a.hi[k] - a.lo[k]) * s));
        f[4 + k] = log2f(1.0f + (float)((b.hi[k] - b.lo[k]) * s));
        double d = 0.5 * (a.lo[k] + a.hi[k]) - 0.5 * (b.lo[k] + b.hi[k]);
        c2 += d * d;
    }
    f[7] = log2f(1.0f + (float)(sqrt(c2) * s));
    f[8] = (float)a.n * (1.0f / 64.0f);
    f[9] = (float)b.n * (1.0f / 64.0f);
}

// Training target: log2 of the tile pair's smallest candidate distance (or a
// lower bound of it when no triangle pair was tested), in row-scale units.
__device__ __forceinline__ float tp_target(double outcome, double scale) {
    double s = scale > 0.0 ? 1.0 / scale : 1.0;
    return log2f((float)(outcome * s) + 0x1p-10f);
}

__device__ __forceinline__ void log_tile_pair(const Lists &L, const TileMeta &a, const TileMeta &b,
                                              double scale, float lbf, double outcome, int row) {
    unsigned long long i = atomicAdd(L.log_count, 1ull);
    if (i >= L.log_cap) return;
    float f[MLP_IN];
    tp_features(a, b, scale, lbf, f);
    float *r = L.log + i * LOG_STRIDE;
    for (int k = 0; k < MLP_IN; k++) r[k] = f[k];
    r[MLP_IN] = tp_target(outcome, scale);
    r[MLP_IN + 1] = __int_as_float(row);
}

// Squared gap of two boxes, without contraction, so that the value is a
// monotone function of the bounds: a group-box pair that fails a threshold
// contains no triangle-box pair that passes it.
template <typename T>
__device__ __forceinline__ T gap2_boxes(const T (&alo)[3], const T (&ahi)[3], const T (&blo)[3],
                                        const T (&bhi)[3]) {
#pragma clang fp contract(off)
    T g2 = 0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        T gp = fmax(fmax(blo[k] - ahi[k], alo[k] - bhi[k]), (T)0);
        g2 += gp * gp;
    }
    return g2;
}

template <typename T>
__device__ __forceinline__ bool overlap_boxes(const T (&alo)[3], const T (&ahi)[3], const T (&blo)[3],
                                              const T (&bhi)[3], T tol) {
    bool keep = true;
#pragma unroll
    for (int k = 0; k < 3; k++) keep = keep && blo[k] - ahi[k] <= tol && alo[k] - bhi[k] <= tol;
    return keep;
}

// A lower bound rounded down to its upper 16 bits (negative bounds become 0:
// such pairs are rescued whatever the upper bound).
__device__ __forceinline__ uint32_t lb_down16(float lb) {
    return __float_as_uint(fmaxf(lb, 0.0f)) >> 16;
}

// Append to a global list with one atomic per wave (divergence-safe).
template <typename T>
__device__ __forceinline__ void global_push(bool keep, const T &item, T *arr, unsigned int *count,
                                            unsigned int cap) {
    unsigned long long act = __ballot(1);
    unsigned long long m = __ballot(keep);
    if (m == 0) return;
    int leader = __ffsll((long long)act) - 1;
    unsigned int base = 0;
    if (lane_id() == leader) base = atomicAdd(count, (unsigned int)__popcll(m));
    base = __shfl(base, leader);
    if (keep) {
        unsigned int idx = base + (unsigned int)__popcll(m & lanes_below());
        if (idx < cap) arr[idx] = item;
    }
}


constexpr int QB = 16;      // most queue entries a wave claims at once
constexpr int RING = 128;   // LDS ring of triangle pairs awaiting their test (two batches)
constexpr int TLCAP = 192;  // FP32 pairs awaiting the rescue decision of their tile pair
constexpr unsigned RCHUNK = 128;  // rescue-list slots a wave claims at once

// Lane i's value in every lane (i wave-uniform): v_readlane into a scalar.
__device__ __forceinline__ int rl_i(int v, int i) { return __builtin_amdgcn_readlane(v, i); }
__device__ __forceinline__ float rl_f(float v, int i) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), i));
}
__device__ __forceinline__ unsigned long long rl_u64(unsigned long long b, int i) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, i);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), i);
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ double rl_d(double v, int i) {
    return __longlong_as_double((long long)rl_u64((unsigned long long)__double_as_longlong(v), i));
}


// A wave's share of the rescue list: it claims RCHUNK slots with one atomic
// and fills them in order, so that most appends need no global atomic (and no
// wait on one).  Slots left unused when the wave finishes are written with
// ta = -1, which the rescue kernels skip; the list's count is the number of
// slots claimed (an overflow is still detected from it).
struct RescueChunk {
    unsigned base = 0, left = 0;  // wave-uniform
    // every lane of the wave calls this (keep may be false)
    __device__ __forceinline__ void push(bool keep, const Rescue &item, const Lists &L) {
        const unsigned long long m = __ballot(keep);
        if (m == 0) return;
        const unsigned n = (unsigned)__popcll(m);
        const unsigned pos = (unsigned)__popcll(m & lanes_below());
        unsigned idx;
        if (n <= left) {
            idx = base + pos;
            base += n;
            left -= n;
        } else {
            unsigned nb = 0;
            if (lane_id() == 0) nb = atomicAdd(L.rcount, RCHUNK);
            nb = (unsigned)__builtin_amdgcn_readfirstlane((int)nb);
            idx = pos < left ? base + pos : nb + (pos - left);
            base = nb + (n - left);
            left = RCHUNK - (n - left);
        }
        if (keep && idx < L.rcap) L.rescue[idx] = item;
    }
    __device__ __forceinline__ void close(const Lists &L) {
        for (unsigned j = (unsigned)lane_id(); j < left; j += 64)
            if (base + j < L.rcap) L.rescue[base + j] = Rescue{-1, -1, 0u, 0.0f};
    }
};

// One claimed queue entry, held in the registers of the lane of its index in
// the wave's batch: its tiles, row and counts, the row's state when the batch
// was gathered (a stale upper bound is still an upper bound: it only prunes
// less), and the FP32 constants of the tile pair.
struct Entry {
    int ta, tb, g, na, nb, seed_q, hit;
    float lbf;
    double ub, msc;  // row upper bound and margin scale
    float sh0, sh1, sh2, eu, elb, eps_f, box_tol;
    double eps_c;
};

// Gathers entry q0 + lane of the batch into lane `lane`'s registers (lanes at
// and beyond the batch size keep ta = -1).  In the seed pass entry g is row
// g's chosen queue entry.  Returns 1 in the lanes whose two tiles name
// different rows (an inconsistency the caller counts; never expected).
template <int PREC, int MODE>
__device__ __forceinline__ int wave_gather(Entry &E, const Lists &L, unsigned qcount,
                                           const TileMeta *mA, const TileMeta *mB,
                                           RowState *rows, unsigned q0, unsigned qb) {
    const int lane = lane_id();
    E.ta = -1;
    E.tb = -1;
    E.hit = 0;
    E.seed_q = -1;
    int bad = 0;
    if ((unsigned)lane < qb && q0 + lane < qcount) {
        unsigned q = q0 + lane;
        bool have = true;
        if (L.seed_pass) {
            const unsigned long long best = rows[q].best;
            have = best != ~0ull;
            q = (unsigned)(best & 0xffffffffu);
            rows[q0 + lane].seed_q = have ? (int)q : -1;
        }
        if (have) {
            const int2 e = L.queue[q];
            const float lb = L.qlb[q];
            const TileMeta a = mA[e.x], b = mB[e.y];
            const RowState R = rows[a.row];
            bad = a.row != b.row;
            E.ta = e.x;
            E.tb = e.y;
            E.g = a.row;
            E.na = a.n;
            E.nb = b.n;
            E.lbf = lb;
            E.hit = (int)R.hit;
            E.seed_q = R.seed_q;
            E.ub = bits_to_double(R.ub);
            E.msc = R.margin_scale;
            if (PREC == 0) {
                // B is shifted into A's frame, so that A's staged copy serves
                // every consecutive entry of the same A tile
                const TP32 c = tp32_consts(b, a);
                E.sh0 = c.sh[0];
                E.sh1 = c.sh[1];
                E.sh2 = c.sh[2];
                E.eu = c.eu;
                E.elb = c.elb;
                E.eps_f = c.eps_f;
                E.box_tol = c.box_tol;
                E.eps_c = c.eps_c;
            }
        }
    }
    return bad;
}

// Upper bound of the row distance from the smallest FP32 candidate dm of a
// tile pair (see sd3_pair32.h), rounded up once more for the FP64 compare.
__device__ __forceinline__ double fp32_upper(float dm, float eu) {
    const double U = sqrt((double)dm) * (1.0 + 4.0 * U32) + (double)eu;
    return U * (1.0 + 4.0 * U64);
}

// One wave per tile pair.  Each wave claims batches of up to QB queue
// entries (its first batch is its static share, later ones come from the
// shared head, claimed one batch ahead so the atomic's latency overlaps the
// current batch), gathers them into its lanes' registers, and evaluates them
// one by one.  The global loads of the next live entry's two tiles (and of
// its row's current upper bound) are issued as soon as the current entry is
// staged, so they travel while the current entry is culled and tested.  Per
// entry: both tiles staged into the wave's own LDS (FP32 copies, the B tile
// shifted into the A tile's frame, or FP64; the A tile is kept when the
// previous entry staged the same one), a cull of 8 x 8 slot-group boxes, then of
// triangle boxes, with the surviving triangle pairs compacted by ballots into
// an LDS ring and tested 64 at a time, one pair per lane.  Distance: the wave
// lowers the row bound with one atomic whose result it does not wait for,
// and rescues the FP32 pairs whose certified lower bound does not exceed the
// smaller of the row bound read at staging and its own upper bound (plus
// margin); intersects: certified hits set the row flag, undecided pairs go
// to the rescue (FP32) or exact (FP64) list.  Nothing is shared between
// waves but the queue head, the rows' state and the lists, so there is no
// workgroup barrier.
template <int PREC, int MODE, int TK>
__global__ __launch_bounds__(64) void k_pairs(const float *t32A, const double *t64A,
                                              const TileMeta *mA, const float *t32B,
                                              const double *t64B, const TileMeta *mB,
                                              RowState *rows, Lists L) {
    static_assert(tile_size_ok(TK), "tile size");
    constexpr int NF = F_NTRI32;
    constexpr int NG = TK / 8, NGP = NG * NG;
    constexpr int NS = 2 * TK / 64;  // staging slots per lane: [A slots | B slots]
    constexpr bool TESTED_LIST = PREC == 0 && MODE == 0;
    using Tt = typename std::conditional<PREC == 0, float, double>::type;
    // the staged tiles, slot-major: a slot's NF fields are contiguous, so a
    // triangle's fields are read with 16-byte LDS loads
    __shared__ __attribute__((aligned(16))) Tt sA[NF * TK];
    __shared__ __attribute__((aligned(16))) Tt sB[NF * TK];
    __shared__ Tt gbox[2][NG][6];  // [side][group][lo xyz, hi xyz]
    __shared__ uint32_t glist[NGP];
    __shared__ uint32_t ring[RING];
    __shared__ uint32_t tl[TESTED_LIST ? TLCAP : 1];
    const int lane = lane_id();
    const unsigned long long below = lanes_below();
    const unsigned qcount = L.seed_pass ? (unsigned)L.nrows : min(*L.qcount, L.qcap);
    const unsigned nwave = gridDim.x;
    // entries per claim: 1 for short queues (every wave starts at once), up
    // to QB for long ones (one atomic and one gather per batch)
    const unsigned qb = max(1u, min((unsigned)QB, qcount / (nwave * 4u)));
    unsigned long long n_eval = 0, n_boxed = 0, n_tested = 0, n_resc = 0, n_exact = 0, n_bad = 0;
    RescueChunk rch;
    int staged_a = -1;  // the A tile whose copy is in sA (wave-uniform)
    unsigned claim = blockIdx.x;
    for (;;) {
        const unsigned q0 = claim * qb;
        if (q0 >= qcount) break;
        Entry E;
        n_bad += wave_gather<PREC, MODE>(E, L, qcount, mA, mB, rows, q0, qb);
        unsigned nxt = 0;
        if (lane == 0) nxt = nwave + atomicAdd(L.qhead, 1u);
        const int bn = (int)min(qb, qcount - q0);
        // entry i is evaluated unless its row has no seed choice, already
        // meets, was seeded with it, or its box bound exceeds the row bound
        // (plus margin) gathered with the batch (wave-uniform)
        auto live = [&](int i) __attribute__((always_inline)) {
            if (rl_i(E.ta, i) < 0 || rl_i(E.hit, i)) return false;
            if (!L.seed_pass && (int)(q0 + (unsigned)i) == rl_i(E.seed_q, i)) return false;
            if (MODE == 0) {
                const double ub = rl_d(E.ub, i), msc = rl_d(E.msc, i);
                if ((double)rl_f(E.lbf, i) > ub + msc + 1.4551915228366852e-11 * ub) return false;
            }
            return true;
        };
        // raw tile data of the entry staged next (its A tile only when that
        // is not the one staged already), and its row's upper bound
        Tt raw[NS][9];
        unsigned long long raw_ub = ~0ull;
        int pf = -1;
        bool raw_keepA = false;
        auto load_raw = [&](int j) __attribute__((always_inline)) {
            const int ja = rl_i(E.ta, j), jb = rl_i(E.tb, j);
            raw_keepA = ja == staged_a;
#pragma unroll
            for (int s = 0; s < NS; s++) {
                const int sl = s * 64 + lane;
                const bool onB = sl >= TK;
                if (!onB && raw_keepA) continue;
                const int jj = onB ? sl - TK : sl;
                const Tt *src = PREC == 0 ? (const Tt *)(onB ? t32B + (int64_t)jb * 9 * TK : t32A + (int64_t)ja * 9 * TK)
                                          : (const Tt *)(onB ? t64B + (int64_t)jb * 9 * TK : t64A + (int64_t)ja * 9 * TK);
#pragma unroll
                for (int c = 0; c < 9; c++) raw[s][c] = src[c * TK + jj];
            }
            if (MODE == 0) raw_ub = rows[rl_i(E.g, j)].ub;
            pf = j;
        };
        int i = 0;
        while (i < bn && !live(i)) i++;
        for (; i < bn;) {
            if (pf != i) load_raw(i);
            const int ta = rl_i(E.ta, i), tb = rl_i(E.tb, i), g = rl_i(E.g, i);
            const int na = rl_i(E.na, i), nb = rl_i(E.nb, i);
            const float lbf = rl_f(E.lbf, i);
            const double msc = rl_d(E.msc, i);
            n_eval++;
            float sh[3] = {0.0f, 0.0f, 0.0f}, eu = 0.0f, elb = 0.0f, eps_f = 0.0f, box_tol = 0.0f;
            double eps_c = 0.0;
            if (PREC == 0) {
                sh[0] = rl_f(E.sh0, i);
                sh[1] = rl_f(E.sh1, i);
                sh[2] = rl_f(E.sh2, i);
                eu = rl_f(E.eu, i);
                elb = rl_f(E.elb, i);
                eps_f = rl_f(E.eps_f, i);
                box_tol = rl_f(E.box_tol, i);
                eps_c = rl_d(E.eps_c, i);
            }
            // stage both tiles from the raw registers: slot s of [A slots |
            // B slots], 64 at a time; each group of 8 consecutive slots (8
            // lanes) reduces its box.  An A tile that is already staged (the
            // previous entry's) is kept: A stays in its own frame and B is
            // shifted into it
            const bool keepA = raw_keepA;
            staged_a = ta;
#pragma unroll
            for (int s = 0; s < NS; s++) {
                const int sl = s * 64 + lane;
                const bool onB = sl >= TK;
                if (!onB && keepA) continue;
                const int j = onB ? sl - TK : sl;
                Tt *dst = onB ? sB : sA;
                // the vertices in registers: stored, and every derived field
                // and the triangle box computed from them (no LDS read back)
                Tt v[9];
                if (PREC == 0) {
                    const float sx = onB ? sh[0] : 0.0f, sy = onB ? sh[1] : 0.0f, sz = onB ? sh[2] : 0.0f;
#pragma unroll
                    for (int c = 0; c < 9; c++) v[c] = (Tt)raw[s][c] + (Tt)(c % 3 == 0 ? sx : c % 3 == 1 ? sy : sz);
                } else {
#pragma unroll
                    for (int c = 0; c < 9; c++) v[c] = raw[s][c];
                }
#pragma unroll
                for (int c = 0; c < 9; c++) dst[j * NF + c] = v[c];
                Tt bx[6];
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    bx[k] = fmin(v[k], fmin(v[3 + k], v[6 + k]));
                    bx[3 + k] = fmax(v[k], fmax(v[3 + k], v[6 + k]));
                }
                if constexpr (PREC == 0) {
                    tri_derive32(TriRef<float>{(float *)dst + j * NF, 1}, v);
                } else {
                    tri_derive64(TriRef<double>{(double *)dst + j * NF, 1}, v);
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        dst[j * NF + F_LO + k] = bx[k];
                        dst[j * NF + F_HI + k] = bx[3 + k];
                    }
                }
                if constexpr (PREC == 0) {
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        bx[k] = group8_min(bx[k]);
                        bx[3 + k] = group8_max(bx[3 + k]);
                    }
                } else {
#pragma unroll
                    for (int o = 1; o < 8; o <<= 1)
#pragma unroll
                        for (int k = 0; k < 3; k++) {
                            bx[k] = fmin(bx[k], __shfl_xor(bx[k], o));
                            bx[3 + k] = fmax(bx[3 + k], __shfl_xor(bx[3 + k], o));
                        }
                }
                if ((j & 7) == 0)
#pragma unroll
                    for (int k = 0; k < 6; k++) gbox[onB ? 1 : 0][j >> 3][k] = bx[k];
            }
            // the row bound now: the batch's, or the one read with the tiles
            double ub = rl_d(E.ub, i);
            if (MODE == 0) ub = fmin(ub, bits_to_double(rl_u64(raw_ub, 0)));
            // the next live entry's loads travel while this one is worked
            // (FP32 tiles; the FP64 copies would take twice the registers)
            int nx = i + 1;
            while (nx < bn && !live(nx)) nx++;
            if (PREC == 0 && nx < bn) load_raw(nx);
            float T2f = 0.0f;
            double T2d = 0.0;
            if (MODE == 0) {
                const double m = msc + 1.4551915228366852e-11 * ub;
                if (PREC == 0) {
                    const double T = (ub + m + eps_c) / (1.0 - 4.0 * U32);
                    const double T2 = T * T * (1.0 + 16.0 * U32);
                    T2f = T2 < 3.0e38 ? (float)(T2 * (1.0 + 0x1p-20)) : __builtin_inff();
                } else {
                    const double T = (ub + m) * (1.0 + 8.0 * U64);
                    T2d = T * T;
                }
            }
            wave_lds_sync();
            // group-box pairs, compacted into glist
            unsigned gcnt = 0;
#pragma unroll
            for (int p0 = 0; p0 < NGP; p0 += 64) {
                const int p = p0 + lane, ga = p / NG, gb = p % NG;
                bool keep = p < NGP && ga * 8 < na && gb * 8 < nb;
                if (keep) {
                    const Tt alo[3] = {gbox[0][ga][0], gbox[0][ga][1], gbox[0][ga][2]};
                    const Tt ahi[3] = {gbox[0][ga][3], gbox[0][ga][4], gbox[0][ga][5]};
                    const Tt blo[3] = {gbox[1][gb][0], gbox[1][gb][1], gbox[1][gb][2]};
                    const Tt bhi[3] = {gbox[1][gb][3], gbox[1][gb][4], gbox[1][gb][5]};
                    if (MODE == 0) {
                        const Tt g2 = gap2_boxes(alo, ahi, blo, bhi);
                        keep = PREC == 0 ? (float)g2 <= T2f : (double)g2 <= T2d;
                    } else {
                        keep = overlap_boxes(alo, ahi, blo, bhi, PREC == 0 ? (Tt)box_tol : (Tt)0);
                    }
                }
                const unsigned long long mk = __ballot(keep);
                if (keep) glist[gcnt + __popcll(mk & below)] = (uint32_t)(ga | (gb << 8));
                gcnt += (unsigned)__popcll(mk);
            }
            wave_lds_sync();
            n_boxed += (unsigned long long)NGP + 64ull * gcnt;
            // the pairs of each surviving group pair (lane -> (a, b)) through
            // their triangle-box test into the ring; full batches of 64 are
            // tested at once
            Tt tmin = (Tt)__builtin_inf();
            unsigned rc = 0, rd = 0, tc = 0;
            auto rescue_tested = [&](double lim) __attribute__((always_inline)) {
                // every lane runs every round (the chunk state stays uniform)
                for (unsigned k0 = 0; k0 < tc; k0 += 64) {
                    const unsigned k = k0 + (unsigned)lane;
                    const uint32_t x = k < tc ? tl[k] : 0u;
                    const float lb = __uint_as_float((x >> 16) << 16);
                    const bool resc = k < tc && (double)lb <= lim;
                    rch.push(resc, Rescue{ta, tb, (uint32_t)((x & 255) | (((x >> 8) & 255) << 16)), lb}, L);
                    n_resc += resc;
                }
            };
            auto test_batch = [&](unsigned n) __attribute__((always_inline)) {
                const bool on = (unsigned)lane < n;
                uint32_t e = on ? ring[(rd + lane) & (RING - 1)] : 0u;
                const int a = e & 255, b = (e >> 8) & 255;
                if (PREC == 0) {
                    TriRef<float> TA{(float *)sA + a * NF, 1}, TB{(float *)sB + b * NF, 1};
                    if (MODE == 0) {
                        uint32_t te = 0;
                        if (on) {
                            const Pair32 r = pair32(TA, TB, elb);
                            tmin = fmin(tmin, (Tt)r.d2);
                            te = (uint32_t)(a | (b << 8)) | (lb_down16(r.lb) << 16);
                        }
                        if (tc + n > (unsigned)TLCAP) {
                            // the tested list is full: decide its pairs now
                            // against the row bound lowered by this tile
                            // pair's own minimum so far (a larger limit than
                            // the final one: it only rescues more)
                            const float dm = wave_min((float)tmin);
                            const double lim0 = dm < __builtin_inff() ? fmin(ub, fp32_upper(dm, eu)) : ub;
                            wave_lds_sync();
                            rescue_tested(lim0 + msc + 1.4551915228366852e-11 * lim0);
                            tc = 0;
                            wave_lds_sync();
                        }
                        if (on) tl[tc + lane] = te;
                        tc += n;
                    } else {
                        int c = 0;
                        if (on) {
                            c = isect32(TA, TB, eps_f);
                            // not settled by planes and crossings: a certified
                            // separating plane along the closest direction
                            // still proves the pair disjoint
                            if (c == 2 && pair32(TA, TB, elb).lb > 0.0f) c = 0;
                        }
                        if (__ballot(c == 1) && lane == 0) atomicOr(&rows[g].hit, 1u);
                        Rescue it{ta, tb, (uint32_t)(a | (b << 16)), 0.0f};
                        rch.push(c == 2, it, L);
                        n_resc += c == 2;
                    }
                } else {
                    TriRef<double> TA{(double *)sA + a * NF, 1}, TB{(double *)sB + b * NF, 1};
                    // distance and intersects both use the full FP64 pair test:
                    // its separating-plane certificate settles the disjoint
                    // pairs whose orientation signs are exact zeros
                    int st = 0;
                    double d2 = 0.0;
                    if (on) {
                        const Pair64 r = pair64(TA, TB);
                        st = r.status;
                        d2 = r.d2;
                        if (MODE == 0) tmin = fmin(tmin, (Tt)r.d2);
                    }
                    if (__ballot(st == 1) && lane == 0) atomicOr(&rows[g].hit, 1u);
                    ExactItem it{ta, tb, (uint32_t)(a | (b << 16)), 0, d2};
                    global_push(st == 2, it, L.exact, L.xcount, L.xcap);
                    n_exact += st == 2;
                }
                rd += n;
            };
            for (unsigned gi = 0; gi < gcnt; gi++) {
                const uint32_t ge = glist[gi];
                const int a = (int)(ge & 255) * 8 + (lane >> 3);
                const int b = (int)((ge >> 8) & 255) * 8 + (lane & 7);
                bool keep = a < na && b < nb;
                const Tt *pa = sA + a * NF, *pb = sB + b * NF;
                const Tt alo[3] = {pa[F_LO], pa[F_LO + 1], pa[F_LO + 2]};
                const Tt ahi[3] = {pa[F_HI], pa[F_HI + 1], pa[F_HI + 2]};
                const Tt blo[3] = {pb[F_LO], pb[F_LO + 1], pb[F_LO + 2]};
                const Tt bhi[3] = {pb[F_HI], pb[F_HI + 1], pb[F_HI + 2]};
                if (MODE == 0) {
                    const Tt g2 = gap2_boxes(alo, ahi, blo, bhi);
                    keep = keep && (PREC == 0 ? (float)g2 <= T2f : (double)g2 <= T2d);
                } else {
                    keep = keep && overlap_boxes(alo, ahi, blo, bhi, PREC == 0 ? (Tt)box_tol : (Tt)0);
                }
                const unsigned long long mk = __ballot(keep);
                if (keep) ring[(rc + __popcll(mk & below)) & (RING - 1)] = (uint32_t)(a | (b << 8));
                rc += (unsigned)__popcll(mk);
                if (rc - rd >= 64) {
                    wave_lds_sync();
                    test_batch(64);
                }
            }
            if (rc > rd) {
                wave_lds_sync();
                test_batch(rc - rd);
            }
            n_tested += rc;
            if (MODE == 0) {
                const Tt dm = wave_min(tmin);
                if (PREC == 0) {
                    // the row bound from this tile pair's own minimum goes out
                    // with an atomic that is not waited for; the rescue limit
                    // is the smaller of that minimum's bound and the row bound
                    // read with the tiles (every other result it can miss
                    // only makes the limit larger: more pairs are rescued,
                    // and the rescue kernel filters them again)
                    double ub_now = ub;
                    if ((float)dm < __builtin_inff()) {
                        const double U = fp32_upper((float)dm, eu);
                        if (lane == 0) atomicMin(&rows[g].ub, double_to_bits(U));
                        ub_now = fmin(ub_now, U);
                    }
                    const double lim = ub_now + msc + 1.4551915228366852e-11 * ub_now;
                    wave_lds_sync();
                    rescue_tested(lim);
                } else if (lane == 0 && (double)dm < __builtin_inf()) {
                    atomic_min_pos(&rows[g].d2, (double)dm);
                    atomic_min_pos(&rows[g].ub, sqrt((double)dm));
                }
                if (L.log && lane == 0) {
                    // smallest tested candidate distance, else the cull
                    // threshold (every untested pair lies beyond it)
                    const double T2 = PREC == 0 ? (double)T2f : T2d;
                    const double out = sqrt(fmin((double)dm, T2));
                    log_tile_pair(L, mA[ta], mB[tb], rows[g].scale, lbf, out, g);
                }
            }
            wave_lds_sync();  // LDS reads of this tile pair before the next staging
            i = nx;
        }
        if (MODE == 0 && L.log) {
            // entries pruned at dequeue: their box bound is the logged
            // (lower-bound) outcome
            for (int k = 0; k < bn; k++)
                if (rl_i(E.ta, k) >= 0 && !rl_i(E.hit, k) && !live(k) &&
                    (L.seed_pass || (int)(q0 + (unsigned)k) != rl_i(E.seed_q, k)) && lane == 0) {
                    const int kg = rl_i(E.g, k);
                    log_tile_pair(L, mA[rl_i(E.ta, k)], mB[rl_i(E.tb, k)], rows[kg].scale, rl_f(E.lbf, k),
                                  rl_f(E.lbf, k), kg);
                }
        }
        claim = (unsigned)__builtin_amdgcn_readfirstlane((int)nxt);
    }
    rch.close(L);
    n_resc = wave_sum(n_resc);
    n_exact = wave_sum(n_exact);
    n_bad = wave_sum(n_bad);
    if (lane == 0) {
        if (n_eval) atomicAdd(&L.counters[C_TP_EVAL], n_eval);
        if (n_boxed) atomicAdd(&L.counters[C_TRI_BOXED], n_boxed);
        if (n_tested) atomicAdd(&L.counters[PREC == 0 ? C_TRI32 : C_TRI64], n_tested);
        if (n_resc) atomicAdd(&L.counters[C_RESCUED], n_resc);
        if (n_exact) atomicAdd(&L.counters[C_EXACT], n_exact);
        if (n_bad) atomicAdd(&L.counters[C_SKEW], n_bad);
    }
}


template <int P, int M>
static int occupancy_tk(int tk) {
    int n = 0;
    hipError_t e = tk == 32    ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_pairs<P, M, 32>, 64, 0)
                   : tk == 64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_pairs<P, M, 64>, 64, 0)
                              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_pairs<P, M, 128>, 64, 0);
    return e == hipSuccess && n >= 1 ? n : 1;
}

int pairs_blocks_per_cu(int precision, int mode, int tk) {
    if (precision == 0) return mode == 0 ? occupancy_tk<0, 0>(tk) : occupancy_tk<0, 1>(tk);
    return mode == 0 ? occupancy_tk<1, 0>(tk) : occupancy_tk<1, 1>(tk);
}

template <int P, int M>
static void launch_pairs_tk(const SideBufs &A, const SideBufs &B, RowState *rows, Lists &L, int grid,
                            hipStream_t s) {
#define SD3_LAUNCH_PAIRS(T)                                                                          \
    hipLaunchKernelGGL((k_pairs<P, M, T>), dim3(grid), dim3(64), 0, s, A.t32, A.t64, A.meta, B.t32, \
                       B.t64, B.meta, rows, L)
    if (A.tk == 32) SD3_LAUNCH_PAIRS(32);
    else if (A.tk == 64) SD3_LAUNCH_PAIRS(64);
    else SD3_LAUNCH_PAIRS(128);
#undef SD3_LAUNCH_PAIRS
}

void launch_pairs(const SideBufs &A, const SideBufs &B, RowState *rows, Lists &L, int precision,
                  int mode, int grid, hipStream_t s) {
    if (precision == 0 && mode == 0) launch_pairs_tk<0, 0>(A, B, rows, L, grid, s);
    else if (precision == 0) launch_pairs_tk<0, 1>(A, B, rows, L, grid, s);
    else if (mode == 0) launch_pairs_tk<1, 0>(A, B, rows, L, grid, s);
    else launch_pairs_tk<1, 1>(A, B, rows, L, grid, s);
}

// ---------------------------------------------------------------------------
// a5: FP64 rescue of the pairs the FP32 bounds did not settle
// ---------------------------------------------------------------------------
// FP64 vertices of one tile slot: from the tile's exact copies when they
// exist (plain FP64 path), else gathered through the slot's triangle id from
// the inputs (the same values, so both give identical results).
struct TriSrc {
    const double *t64;
    const int32_t *ids;
    const double *xyz;
    const int32_t *tri;
    const int64_t *v_off;
    const TileMeta *meta;
    int tk;
};

static TriSrc tri_src(const SideBufs &S) { return {S.t64, S.ids, S.xyz, S.tri, S.v_off, S.meta, S.tk}; }

__device__ __forceinline__ void load_tri64(const TriSrc &S, int tile, int slot, double *out) {
    if (S.t64) {
#pragma unroll
        for (int c = 0; c < 9; c++) out[c] = S.t64[((int64_t)tile * 9 + c) * S.tk + slot];
        return;
    }
    const int64_t id = S.ids[(int64_t)tile * S.tk + slot];
    const int64_t g = S.meta[tile].row;
    const double *X = S.xyz + 3 * S.v_off[g];
    const int64_t nvr = S.v_off[g + 1] - S.v_off[g];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const double *p = X + 3 * corner(S.tri, id, k, nvr);
        out[3 * k] = p[0];
        out[3 * k + 1] = p[1];
        out[3 * k + 2] = p[2];
    }
}

// FP64 re-evaluation of rescue entries first, first + step, ... (every lane
// of a wave calls this: the counters are summed per wave).
template <int MODE>
__device__ void rescue_items(const TriSrc &SA, const TriSrc &SB, RowState *rows, const Lists &L,
                             unsigned first, unsigned step) {
    const TileMeta *mA = SA.meta;
    const unsigned n = min(*L.rcount, L.rcap);
    unsigned long long n64 = 0, nex = 0;
    for (unsigned i = first; i < n; i += step) {
        Rescue e = L.rescue[i];
        if (e.ta < 0) continue;  // an unused slot of a wave's claimed chunk
        int a = e.slots & 0xffff, b = e.slots >> 16;
        // the vertices depend on the entry alone: their loads go out beside
        // the row state's, not after its checks
        double ta[F_NTRI64], tb[F_NTRI64];
        load_tri64(SA, e.ta, a, ta);
        load_tri64(SB, e.tb, b, tb);
        int g = mA[e.ta].row;
        RowState *R = rows + g;
        if (load_acq32(&R->hit)) continue;
        if (MODE == 0) {
            double ub = bits_to_double(load_acq(&R->ub));
            if ((double)e.lb > ub + row_margin(*R, ub)) continue;
            tri_prep64(TriRef<double>{ta, 1});
            tri_prep64(TriRef<double>{tb, 1});
            Pair64 r = pair64(TriRef<double>{ta, 1}, TriRef<double>{tb, 1});
            n64++;
            if (r.status == 1) {
                atomicOr(&R->hit, 1u);
                atomic_min_pos(&R->d2, 0.0);
            } else {
                atomic_min_pos(&R->d2, r.d2);
                if (r.status == 2) {
                    ExactItem it{e.ta, e.tb, e.slots, 0, r.d2};
                    unsigned j = atomicAdd(L.xcount, 1u);
                    if (j < L.xcap) L.exact[j] = it;
                    nex++;
                }
            }
        } else {
            tri_prep64(TriRef<double>{ta, 1});
            tri_prep64(TriRef<double>{tb, 1});
            int f = pair64(TriRef<double>{ta, 1}, TriRef<double>{tb, 1}).status;
            n64++;
            if (f == 1) atomicOr(&R->hit, 1u);
            else if (f == 2) {
                ExactItem it{e.ta, e.tb, e.slots, 0, 0.0};
                unsigned j = atomicAdd(L.xcount, 1u);
                if (j < L.xcap) L.exact[j] = it;
                nex++;
            }
        }
    }
    n64 = wave_sum(n64);
    nex = wave_sum(nex);
    if (lane_id() == 0) {
        if (n64) atomicAdd(&L.counters[C_TRI64], n64);
        if (nex) atomicAdd(&L.counters[C_EXACT], nex);
    }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_rescue(TriSrc SA, TriSrc SB, RowState *rows, Lists L) {
    rescue_items<MODE>(SA, SB, rows, L, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

void launch_rescue(const SideBufs &A, const SideBufs &B, RowState *rows, Lists &L, int mode,
                   int grid, hipStream_t s) {
    if (mode == 0)
        hipLaunchKernelGGL(k_rescue<0>, dim3(grid), dim3(256), 0, s, tri_src(A), tri_src(B), rows, L);
    else
        hipLaunchKernelGGL(k_rescue<1>, dim3(grid), dim3(256), 0, s, tri_src(A), tri_src(B), rows, L);
}

// ---------------------------------------------------------------------------
// exact arithmetic for the pairs the FP64 filter left undecided
// ---------------------------------------------------------------------------
__device__ __forceinline__ void finalize_row(const RowState *rows, int64_t g, double *dist,
                                             uint8_t *hit) {
    bool h = rows[g].hit != 0;
    if (dist) dist[g] = h ? 0.0 : sqrt(bits_to_double(rows[g].d2));
    if (hit) hit[g] = h ? 1 : 0;
}

// Exact arithmetic for the listed pairs, items first, first + step, ...
__device__ void exact_items(const TriSrc &SA, const TriSrc &SB, RowState *rows, const Lists &L,
                            int mode, unsigned first, unsigned step) {
    const TileMeta *mA = SA.meta;
    const unsigned n = min(*L.xcount, L.xcap);
    for (unsigned i = first; i < n; i += step) {
        ExactItem e = L.exact[i];
        double va[9], vb[9];
        load_tri64(SA, e.ta, e.slots & 0xffff, va);
        load_tri64(SB, e.tb, e.slots >> 16, vb);
        RowState *R = rows + mA[e.ta].row;
        if (load_acq32(&R->hit)) continue;
        if (ex::tri_tri_exact(va, vb)) {
            atomicOr(&R->hit, 1u);
            atomic_min_pos(&R->d2, 0.0);
        } else if (mode == 0) {
            atomic_min_pos(&R->d2, e.d2);
        }
    }
}

// True in the last block of the grid to reach this point; every other
// block's memory updates are then visible to it (fence before the counter).
__device__ __forceinline__ bool last_block_done(unsigned int *done) {
    __shared__ int last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (last) __threadfence();
    return last != 0;
}

// The results of rows [0, fin_rows), unless the call failed on the device.
__device__ __forceinline__ void finalize_rows(const RowState *rows, int64_t fin_rows, double *dist,
                                              uint8_t *hit, const Lists &L, const uint32_t *vflags) {
    if (call_failed(L, vflags)) return;
    for (int64_t g = threadIdx.x; g < fin_rows; g += blockDim.x) finalize_row(rows, g, dist, hit);
}

// With fin_rows > 0 the last block to finish also writes the results.
__global__ __launch_bounds__(64) void k_exact(TriSrc SA, TriSrc SB, RowState *rows, Lists L,
                                              int mode, int64_t fin_rows, double *dist,
                                              uint8_t *hit, const uint32_t *vflags) {
    exact_items(SA, SB, rows, L, mode, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
    if (fin_rows <= 0) return;
    if (last_block_done(L.xdone)) finalize_rows(rows, fin_rows, dist, hit, L, vflags);
}

void launch_exact(const SideBufs &A, const SideBufs &B, RowState *rows, Lists &L, int mode,
                  int grid, hipStream_t s, int64_t fin_rows, double *dist, uint8_t *hit,
                  const uint32_t *vflags) {
    hipLaunchKernelGGL(k_exact, dim3(grid), dim3(64), 0, s, tri_src(A), tri_src(B), rows, L, mode,
                       fin_rows, dist, hit, vflags);
}

// Rescue, exact arithmetic and results in one launch: every block re-evaluates
// its share of the rescue list in FP64; the last block to finish (when no
// more items can be added) takes every exact item and writes the results.
template <int MODE>
__global__ __launch_bounds__(256) void k_resolve(TriSrc SA, TriSrc SB, RowState *rows, Lists L,
                                                 int64_t fin_rows, double *dist, uint8_t *hit,
                                                 const uint32_t *vflags) {
    rescue_items<MODE>(SA, SB, rows, L, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
    if (!last_block_done(L.xdone)) return;
    exact_items(SA, SB, rows, L, MODE, threadIdx.x, blockDim.x);
    if (fin_rows > 0) {
        // this block's own exact updates, then fresh row states
        __syncthreads();
        __threadfence();
        finalize_rows(rows, fin_rows, dist, hit, L, vflags);
    }
}

void launch_resolve(const SideBufs &A, const SideBufs &B, RowState *rows, Lists &L, int mode,
                    int grid, hipStream_t s, int64_t fin_rows, double *dist, uint8_t *hit,
                    const uint32_t *vflags) {
    if (mode == 0)
        hipLaunchKernelGGL(k_resolve<0>, dim3(grid), dim3(256), 0, s, tri_src(A), tri_src(B), rows, L,
                           fin_rows, dist, hit, vflags);
    else
        hipLaunchKernelGGL(k_resolve<1>, dim3(grid), dim3(256), 0, s, tri_src(A), tri_src(B), rows, L,
                           fin_rows, dist, hit, vflags);
}

// ---------------------------------------------------------------------------
// seed round: rank the queued tile pairs, evaluate each row's best first
// ---------------------------------------------------------------------------
// Feature length scale of a row: its upper bound after seeding, else its extent.
__device__ __forceinline__ void row_scale(RowState *rows, int64_t g) {
    double ub = bits_to_double(rows[g].ub);
    double ext = rows[g].margin_scale * 0x1p36;
    rows[g].scale = (ub > 0.0 && ub < __builtin_inf()) ? ub : (ext > 0.0 ? ext : 1.0);
}


// The ranker on the matrix cores: a wave scores 16 tile pairs at a time,
// each layer a chain of FP32 MFMAs (v_mfma_f32_16x16x4_f32: D[16 x 16] +=
// A[16 x 4] B[4 x 16]; lane l holds A[l % 16][l / 16], B[l / 16][l % 16] and
// D[4 (l / 16) + r][l % 16], r = 0..3), so that every weight read from LDS
// serves 16 pairs.  Rows of A are the 16 pairs, B is the layer's transposed
// weights, one 16-column tile of the 64 hidden units per accumulator.
typedef float mfx4 __attribute__((ext_vector_type(4)));

constexpr int MLP_K1 = 12;       // first layer's inputs, padded to 3 steps of 4
constexpr int MLP_HP = MLP_H + 4;  // padded activation rows in LDS
// Weights in LDS in the order the B operands are read: layer L, K-step s,
// column tile c, lane l holds W_L[16 c + l % 16][4 s + l / 16] at
// [(s * 4 + c) * 64 + l] (one contiguous 256-byte read per MFMA).
struct alignas(16) MlpLds {
    float w1[(MLP_K1 / 4) * 4 * 64];
    float w2[(MLP_H / 4) * 4 * 64];
    float w3[(MLP_H / 4) * 4 * 64];
    float bias[3 * MLP_H + MLP_H + 1];  // b1 b2 b3 w4 b4
};
// Per wave: the 16 pairs' features and one layer's activations.
struct MlpWave {
    float x[16][MLP_K1];
    float h[16][MLP_HP];
};
static_assert(MLP_H == 64, "four 16-column tiles per layer");

// Weights into LDS by a 256-thread block (the B-operand order above).
__device__ void mlp_stage(MlpLds &M, const float *W) {
    const int t = threadIdx.x;
    for (int i = t; i < (MLP_K1 / 4) * 4 * 64; i += 256) {
        const int l = i & 63, c = (i >> 6) & 3, st = i >> 8;
        const int row = 16 * c + (l & 15), k = 4 * st + (l >> 4);
        M.w1[i] = k < MLP_IN ? W[MLP_W1 + row * MLP_IN + k] : 0.0f;
    }
    for (int i = t; i < (MLP_H / 4) * 4 * 64; i += 256) {
        const int l = i & 63, c = (i >> 6) & 3, st = i >> 8;
        const int row = 16 * c + (l & 15), k = 4 * st + (l >> 4);
        M.w2[i] = W[MLP_W2 + row * MLP_H + k];
        M.w3[i] = W[MLP_W3 + row * MLP_H + k];
    }
    if (t < MLP_H) {
        M.bias[t] = W[MLP_B1 + t];
        M.bias[MLP_H + t] = W[MLP_B2 + t];
        M.bias[2 * MLP_H + t] = W[MLP_B3 + t];
        M.bias[3 * MLP_H + t] = W[MLP_W4 + t];
    }
    if (t == 0) M.bias[4 * MLP_H] = W[MLP_B4];
}

// One layer: acc[c] = A B_c over `steps` K-steps, A read from rows a[16][*]
// (lane l takes a[l % 16][4 s + l / 16]), B from the staged weights.
template <int STEPS, int AS>
__device__ __forceinline__ void mlp_layer(const float *w, const float (*a)[AS], mfx4 (&acc)[4]) {
    const int lane = lane_id();
#pragma unroll
    for (int c = 0; c < 4; c++) acc[c] = mfx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int st = 0; st < STEPS; st++) {
        const float av = a[lane & 15][4 * st + (lane >> 4)];
#pragma unroll
        for (int c = 0; c < 4; c++)
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, w[(st * 4 + c) * 64 + lane], acc[c], 0, 0, 0);
    }
}

// Bias, ReLU and the activations back to LDS in row order (h[pair][unit]).
__device__ __forceinline__ void mlp_store(const mfx4 (&acc)[4], const float *bias, float (*h)[MLP_HP]) {
    const int lane = lane_id();
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const int j = 16 * c + (lane & 15);
        const float b = bias[j];
#pragma unroll
        for (int r = 0; r < 4; r++) h[4 * (lane >> 4) + r][j] = fmaxf(acc[c][r] + b, 0.0f);
    }
}

// Scores of the 16 pairs whose features are in Wv.x (rows past the batch
// hold zeros); lane i < 16 returns pair i's score.  The whole wave takes part.
__device__ float mlp_scores16(const MlpLds &M, MlpWave &Wv) {
    const int lane = lane_id();
    mfx4 acc[4];
    wave_lds_sync();
    mlp_layer<MLP_K1 / 4, MLP_K1>(M.w1, Wv.x, acc);
    mlp_store(acc, M.bias, Wv.h);
    wave_lds_sync();
    mlp_layer<MLP_H / 4, MLP_HP>(M.w2, Wv.h, acc);
    wave_lds_sync();  // every read of h before it is overwritten
    mlp_store(acc, M.bias + MLP_H, Wv.h);
    wave_lds_sync();
    mlp_layer<MLP_H / 4, MLP_HP>(M.w3, Wv.h, acc);
    // output: b4 + sum_j w4[j] relu(h3[i][j]); lane l holds rows 4 (l / 16) + r
    float p[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const int j = 16 * c + (lane & 15);
        const float b = M.bias[2 * MLP_H + j], w = M.bias[3 * MLP_H + j];
#pragma unroll
        for (int r = 0; r < 4; r++) p[r] += w * fmaxf(acc[c][r] + b, 0.0f);
    }
#pragma unroll
    for (int r = 0; r < 4; r++)
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) p[r] += __shfl_xor(p[r], o);
    // pair i = 4 g + r sits in lanes 16 g .. 16 g + 15, register r
    const int src = 16 * ((lane & 15) >> 2);
    float sc = 0.0f;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const float v = __shfl(p[r], src);
        if ((lane & 3) == r) sc = v;
    }
    return sc + M.bias[4 * MLP_H];
}

// Learned seed choice: each wave takes 16 consecutive queued tile pairs at a
// time; lanes 0-15 gather one pair's features each, the wave scores them on
// the matrix cores, and each pair's lane keeps its row's lowest (ordered
// score bits << 32 | queue index) with atomicMin.
__global__ __launch_bounds__(256) void k_rank(const TileMeta *mA, const TileMeta *mB, RowState *rows,
                                              Lists L, const float *W) {
    __shared__ MlpLds M;
    __shared__ MlpWave Wv[4];
    const unsigned n = min(*L.qcount, L.qcap);
    const unsigned nw = gridDim.x * 4u;
    if ((unsigned)blockIdx.x * 64u >= n) return;  // no pair for this block: skip the weights
    mlp_stage(M, W);
    __syncthreads();
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    MlpWave &V = Wv[wv];
    for (unsigned q0 = (blockIdx.x * 4u + wv) * 16u; q0 < n; q0 += nw * 16u) {
        const unsigned q = q0 + (unsigned)lane;
        const bool mine = lane < 16 && q < n;
        int row = 0;
        float f[MLP_IN];
        for (int k = 0; k < MLP_IN; k++) f[k] = 0.0f;
        if (mine) {
            const int2 e = L.queue[q];
            const TileMeta &a = mA[e.x];
            row = a.row;
            tp_features(a, mB[e.y], rows[row].scale, L.qlb[q], f);
        }
        if (lane < 16)
            for (int k = 0; k < MLP_K1; k++) V.x[lane][k] = k < MLP_IN ? f[k] : 0.0f;
        const float sc = mlp_scores16(M, V);
        if (mine) {
            const unsigned long long key = ((unsigned long long)float_order_bits(sc) << 32) | q;
            if (key < rows[row].best) atomicMin(&rows[row].best, key);
        }
        wave_lds_sync();  // the features are read before the next batch's
    }
}

void launch_rank(const SideBufs &A, const SideBufs &B, RowState *rows, Lists &L,
                 const float *ranker, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_rank, dim3(grid), dim3(256), 0, s, A.meta, B.meta, rows, L, ranker);
}

// The seed round's scorer on given feature rows (x: [n][MLP_IN]): the same
// LDS weight layout and the same 16-pair matrix-core evaluation as k_rank,
// so its outputs are exactly the scores k_rank ranks by.
__global__ __launch_bounds__(256) void k_rank_score(const float *W, const float *x, int64_t n,
                                                    float *y) {
    __shared__ MlpLds M;
    __shared__ MlpWave Wv[4];
    if ((int64_t)blockIdx.x * 64 >= n) return;
    mlp_stage(M, W);
    __syncthreads();
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    MlpWave &V = Wv[wv];
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t i0 = ((int64_t)blockIdx.x * 4 + wv) * 16; i0 < n; i0 += nw * 16) {
        const int64_t i = i0 + lane;
        if (lane < 16)
            for (int k = 0; k < MLP_K1; k++) V.x[lane][k] = (k < MLP_IN && i < n) ? x[i * MLP_IN + k] : 0.0f;
        const float sc = mlp_scores16(M, V);
        if (lane < 16 && i < n) y[i] = sc;
        wave_lds_sync();
    }
}

void launch_rank_score(const float *W, const float *x, int64_t n, float *y, int grid,
                       hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_rank_score, dim3(grid), dim3(256), 0, s, W, x, n, y);
}

// Before each later queue pass's filter: no row has a seed choice yet, and
// the seed pass's head is reset.
__global__ void k_seed_reset(RowState *rows, int64_t G, unsigned int *seedhead) {
    int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g == 0) *seedhead = 0;
    if (g >= G) return;
    rows[g].best = ~0ull;
    rows[g].seed_q = -1;
}

void launch_seed_reset(RowState *rows, int64_t G, unsigned int *seedhead, hipStream_t s) {
    hipLaunchKernelGGL(k_seed_reset, dim3(grid_for(G > 0 ? G : 1, 256)), dim3(256), 0, s, rows, G,
                       seedhead);
}

// ---------------------------------------------------------------------------
// final reduction
// ---------------------------------------------------------------------------
// Writes the results unless the call failed on the device: a validation flag
// is set or a work list overflowed (its count passed its capacity), in which
// case the outputs stay untouched and the host reports the error.
__global__ void k_finalize(const RowState *rows, int64_t G, double *dist, uint8_t *hit, Lists L,
                           const uint32_t *vflags) {
    int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= G) return;
    if (call_failed(L, vflags)) return;
    finalize_row(rows, g, dist, hit);
}

void launch_finalize(const RowState *rows, int64_t G, double *dist, uint8_t *hit, Lists &L,
                     const uint32_t *vflags, hipStream_t s) {
    if (G > 0)
        hipLaunchKernelGGL(k_finalize, dim3(grid_for(G, 256)), dim3(256), 0, s, rows, G, dist, hit, L,
                           vflags);
}

// Between queue passes: the finished pass's count goes to the candidate
// counter (an overflow is remembered) before the queue is emptied.
__global__ void k_reset_queue(Lists L) {
    if (threadIdx.x == 0) {
        unsigned int q = *L.qcount;
        L.counters[C_TP_CAND] += q;
        if (q > L.qcap) L.counters[C_QUEUE_OVF] += 1;
        *L.qcount = 0;
        *L.qhead = 0;
    }
}

void launch_reset_queue(Lists &L, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, s, L);
}


}  // namespace sd3
