// Segments and points against one triangle mesh: the paper's measured
// workload (Sec. 4: drill-hole line segments against an ore-body mesh), with
// the three operators of Sec. 3.2.2 / 3.2.3 -- distance (items (i)-(iii):
// segment/segment, segment/surface, point/surface, then the minimum),
// intersects (Eq. 4 crossings with closed constraints) and the distance
// threshold filter (distance <= r, "filtering drill holes based on their
// distance").
//
// A segment P0 P1 is the degenerate triangle (P0, P1, P1) and a point the
// triangle (P, P, P): the FP64 triangle-pair routine and the exact
// intersection test of the mesh path apply unchanged (a zero-area triangle
// is the union of its edges), so the values are those sd3_distance returns
// for the same inputs.
//
// Layout: the mesh is prepared once per call into an AoS array of FP64
// triangles (30 derived fields + box, 36 doubles) and boxes of consecutive
// 64-triangle tiles.  One wave owns 64 segments (one per lane, staged into
// LDS as degenerate triangles); it walks the mesh tiles, culls each tile by
// box against every live lane, then each triangle box against each lane, and
// compacts the surviving (segment, triangle) pairs with ballots into an LDS
// ring that is tested 64 pairs at a time, one pair per lane.  Per-segment
// state (best squared distance, flags) lives in LDS and is updated with LDS
// atomics.
#include <algorithm>

#include "sd3_kernels.h"
#include "sd3_pair64.h"
#include "sd3_exact.h"

namespace sd3 {

constexpr int MESH_TK = 64;   // triangles per mesh tile
constexpr int SEED_PTS = 256; // mesh vertices a segment's first upper bound is taken over
constexpr int SEG_NF = 36;    // prepared mesh triangle: F_NTRI64 fields + box
constexpr int SEG_RING = 128;

// Validation of the segment coordinates (flags[0]) and of the mesh
// (coordinates and indices, flags[1]); every flag word starts at 0.
__global__ __launch_bounds__(256) void k_seg_validate(const double *seg, int64_t n, const double *xyz,
                                                      int64_t nv, const int32_t *tri, int64_t nt,
                                                      uint32_t *flags) {
    uint32_t fs = 0, fm = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 6 * n; i += stride) {
        const double x = fabs(seg[i]);
        if (!(x <= 1.7976931348623157e308)) fs |= V_NONFINITE;
        else if (x != 0.0 && (x < 0x1p-256 || x > 0x1p256)) fs |= V_RANGE;
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 3 * nv; i += stride) {
        const double x = fabs(xyz[i]);
        if (!(x <= 1.7976931348623157e308)) fm |= V_NONFINITE;
        else if (x != 0.0 && (x < 0x1p-256 || x > 0x1p256)) fm |= V_RANGE;
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 3 * nt; i += stride) {
        const int32_t v = tri[i];
        if (v < 0 || (int64_t)v >= nv) fm |= V_INDEX;
    }
    if (fs) atomicOr(&flags[0], fs);
    if (fm) atomicOr(&flags[1], fm);
}

// Prepared mesh: triangle t's 30 FP64 fields and its box, and the box of
// each tile of 64 consecutive triangles (one wave per tile; indices are
// clamped into the mesh so that invalid contents never address other memory).
__global__ __launch_bounds__(64) void k_seg_mesh(const double *xyz, int64_t nv, const int32_t *tri,
                                                 int64_t nt, double *P, double *tbox) {
    const int64_t tile = blockIdx.x;
    const int64_t t = tile * MESH_TK + threadIdx.x;
    double lo[3] = {__builtin_inf(), __builtin_inf(), __builtin_inf()};
    double hi[3] = {-__builtin_inf(), -__builtin_inf(), -__builtin_inf()};
    if (t < nt) {
        double *q = P + t * SEG_NF;
        for (int k = 0; k < 3; k++) {
            int32_t v = tri[3 * t + k];
            const int64_t vi = (v >= 0 && (int64_t)v < nv) ? v : 0;
            for (int c = 0; c < 3; c++) q[F_V + 3 * k + c] = xyz[3 * vi + c];
        }
        tri_prep64(TriRef<double>{q, 1});
        for (int c = 0; c < 3; c++) {
            lo[c] = fmin(q[F_V + c], fmin(q[F_V + 3 + c], q[F_V + 6 + c]));
            hi[c] = fmax(q[F_V + c], fmax(q[F_V + 3 + c], q[F_V + 6 + c]));
            q[F_NTRI64 + c] = lo[c];
            q[F_NTRI64 + 3 + c] = hi[c];
        }
    }
    for (int c = 0; c < 3; c++) {
        lo[c] = wave_min(lo[c]);
        hi[c] = wave_max(hi[c]);
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; c++) {
            tbox[tile * 6 + c] = lo[c];
            tbox[tile * 6 + 3 + c] = hi[c];
        }
}

// Box of the whole mesh from its tile boxes (one block).
__global__ __launch_bounds__(64) void k_seg_meshbox(const double *tbox, int64_t ntiles, double *mbox) {
    double lo[3] = {__builtin_inf(), __builtin_inf(), __builtin_inf()};
    double hi[3] = {-__builtin_inf(), -__builtin_inf(), -__builtin_inf()};
    for (int64_t t = threadIdx.x; t < ntiles; t += 64)
        for (int c = 0; c < 3; c++) {
            lo[c] = fmin(lo[c], tbox[t * 6 + c]);
            hi[c] = fmax(hi[c], tbox[t * 6 + 3 + c]);
        }
    for (int c = 0; c < 3; c++) {
        lo[c] = wave_min(lo[c]);
        hi[c] = wave_max(hi[c]);
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; c++) {
            // an empty mesh leaves a box that adds nothing to the extent
            mbox[c] = ntiles > 0 ? lo[c] : 0.0;
            mbox[3 + c] = ntiles > 0 ? hi[c] : 0.0;
        }
}

// The exact closed test for a pair the FP64 filter left undecided (rare; a
// call keeps its registers out of the common path).
__device__ __attribute__((noinline)) bool seg_pair_exact(const double *va, const double *vb) {
    return ex::tri_tri_exact(va, vb);
}

__device__ __forceinline__ double seg_gap2(const double *alo, const double *ahi, const double *blo,
                                           const double *bhi) {
#pragma clang fp contract(off)
    double g2 = 0.0;
    for (int k = 0; k < 3; k++) {
        const double gp = fmax(fmax(blo[k] - ahi[k], alo[k] - bhi[k]), 0.0);
        g2 += gp * gp;
    }
    return g2;
}

// Squared cull threshold of a segment with upper bound ub (distance: the best
// so far; threshold filter: r): a triangle whose box gap exceeds it is
// farther than ub by more than the margin m, which exceeds twice the FP64
// error of any pair distance of the segment (m scales with the extent of the
// segment and the mesh, as the row margin of the mesh path).
__device__ __forceinline__ double seg_cull2(double ub, double msc) {
    if (!(ub < __builtin_inf())) return __builtin_inf();
    const double T = (ub + msc + 1.4551915228366852e-11 * ub) * (1.0 + 8.0 * U64);
    return T * T;
}

// MODE 0: distance (dist[i], hit[i] optional); 1: intersects (hit[i]);
// 2: within r (hit[i] = distance <= r).  cnt[0..2]: triangle boxes compared,
// full pair tests, exact tests (summed per wave).
template <int MODE>
__global__ __launch_bounds__(64) void k_segs(const double *seg, int64_t n, const double *P, int64_t nt,
                                             const double *tbox, const double *mbox, double r,
                                             double *dist, uint8_t *hit, const uint32_t *flags,
                                             unsigned long long *cnt) {
    __shared__ double sS[F_NTRI64 * 64];          // the wave's segments, stride 64
    __shared__ unsigned long long best[64];       // squared distance bits
    __shared__ uint32_t done[64];                 // hit (MODE 0, 1) or within (MODE 2)
    __shared__ uint32_t ring[SEG_RING];
    if (flags[0] | flags[1]) return;  // invalid contents: outputs stay untouched
    const int lane = lane_id();
    const unsigned long long below = lanes_below();
    const int64_t ntiles = (nt + MESH_TK - 1) / MESH_TK;
    unsigned long long n_box = 0, n_full = 0, n_ex = 0;
    for (int64_t base = (int64_t)blockIdx.x * 64; base < n; base += (int64_t)gridDim.x * 64) {
        const int64_t i = base + lane;
        const bool mine = i < n;
        double lo[3], hi[3];
        double p[3], q[3];
        {
            for (int c = 0; c < 3; c++) {
                p[c] = mine ? seg[6 * i + c] : 0.0;
                q[c] = mine ? seg[6 * i + 3 + c] : 0.0;
            }
            TriRef<double> S{sS + lane, 64};
            for (int c = 0; c < 3; c++) {
                S.at(F_V + c) = p[c];
                S.at(F_V + 3 + c) = q[c];
                S.at(F_V + 6 + c) = q[c];
                lo[c] = fmin(p[c], q[c]);
                hi[c] = fmax(p[c], q[c]);
            }
            tri_prep64(S);
        }
        // margin scale: 2^-36 of the extent of the segment and the mesh
        double ext = 0.0;
        for (int c = 0; c < 3; c++) ext = fmax(ext, fmax(hi[c], mbox[3 + c]) - fmin(lo[c], mbox[c]));
        const double msc = 1.4551915228366852e-11 * ext;
        best[lane] = double_to_bits(__builtin_inf());
        done[lane] = mine ? 0u : 1u;
        // distance: a first upper bound, the distance from the nearer endpoint
        // to the nearest of up to SEED_PTS mesh vertices (first vertices of
        // evenly spaced triangles; wave-uniform loads), so that the cull is
        // tight from the first tile on.  Any segment point and mesh point
        // bound the distance from above; the returned value still comes from
        // the pair routine alone.
        double ub = __builtin_inf();
        if (MODE == 0 && nt > 0) {
            const int64_t ns = min((int64_t)SEED_PTS, nt);
            double u2 = __builtin_inf();
#pragma unroll 16
            for (int64_t k = 0; k < ns; k++) {
                const double *v = P + ((k * nt) / ns) * SEG_NF + F_V;
                double a2 = 0.0, b2 = 0.0;
                for (int c = 0; c < 3; c++) {
                    const double da = p[c] - v[c], db = q[c] - v[c];
                    a2 += da * da;
                    b2 += db * db;
                }
                u2 = fmin(u2, fmin(a2, b2));
            }
            ub = sqrt(u2) * (1.0 + 4.0 * U64);
        }
        unsigned rc = 0, rd = 0;
        // test ring entries rd .. rd + cnt - 1, one per lane
        auto test_batch = [&](unsigned cntb) __attribute__((always_inline)) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const bool on = (unsigned)lane < cntb;
            const uint32_t e = on ? ring[(rd + lane) & (SEG_RING - 1)] : 0u;
            const int slot = (int)(e & 63);
            const int64_t t = (int64_t)(e >> 6);
            if (on && !done[slot]) {
                TriRef<double> A{sS + slot, 64};
                TriRef<double> B{const_cast<double *>(P) + t * SEG_NF, 1};
                const Pair64 pr = pair64(A, B);
                int st = pr.status;
                n_full++;
                if (st == 2) {
                    double va[9], vb[9];
                    for (int k = 0; k < 9; k++) {
                        va[k] = A[F_V + k];
                        vb[k] = B[F_V + k];
                    }
                    st = seg_pair_exact(va, vb) ? 1 : 0;
                    n_ex++;
                }
                if (st == 1) {
                    if (MODE == 0) {
                        atomicOr(&done[slot], 1u);
                        atomicMin(&best[slot], 0ull);
                    } else {
                        atomicOr(&done[slot], 1u);
                    }
                } else if (MODE == 0) {
                    atomicMin(&best[slot], double_to_bits(pr.d2));
                } else if (MODE == 2 && sqrt(pr.d2) <= r) {
                    atomicOr(&done[slot], 1u);
                }
            }
            rd += cntb;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        for (int64_t tl = 0; tl < ntiles; tl++) {
            // this lane's cull threshold now (the best so far in LDS)
            double T2 = 0.0;
            if (MODE == 0) T2 = seg_cull2(fmin(ub, sqrt(bits_to_double(best[lane]))), msc);
            if (MODE == 2) T2 = seg_cull2(r, msc);
            const bool live = done[lane] == 0;  // out-of-range lanes start done
            const double *tb = tbox + tl * 6;
            const double blo[3] = {tb[0], tb[1], tb[2]}, bhi[3] = {tb[3], tb[4], tb[5]};
            const double g2 = seg_gap2(lo, hi, blo, bhi);
            const bool tile_in = live && (MODE == 1 ? g2 == 0.0 : g2 <= T2);
            if (__ballot(tile_in) == 0) continue;
            const int64_t t0 = tl * MESH_TK, t1 = min(nt, t0 + (int64_t)MESH_TK);
            for (int64_t t = t0; t < t1; t++) {
                const double *q = P + t * SEG_NF + F_NTRI64;  // wave-uniform: scalar loads
                const double tlo[3] = {q[0], q[1], q[2]}, thi[3] = {q[3], q[4], q[5]};
                const double h2 = seg_gap2(lo, hi, tlo, thi);
                const bool keep = tile_in && (MODE == 1 ? h2 == 0.0 : h2 <= T2);
                n_box += tile_in;
                const unsigned long long mk = __ballot(keep);
                if (keep) ring[(rc + __popcll(mk & below)) & (SEG_RING - 1)] = (uint32_t)lane | ((uint32_t)t << 6);
                rc += (unsigned)__popcll(mk);
                if (rc - rd >= 64) test_batch(64);
            }
            if (rc > rd) test_batch(rc - rd);
        }
        if (mine) {
            if (MODE == 0) {
                const bool h = done[lane] != 0;
                dist[i] = h ? 0.0 : sqrt(bits_to_double(best[lane]));
                if (hit) hit[i] = h ? 1 : 0;
            } else {
                hit[i] = done[lane] ? 1 : 0;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    n_box = wave_sum(n_box);
    n_full = wave_sum(n_full);
    n_ex = wave_sum(n_ex);
    if (lane == 0) {
        if (n_box) atomicAdd(&cnt[0], n_box);
        if (n_full) atomicAdd(&cnt[1], n_full);
        if (n_ex) atomicAdd(&cnt[2], n_ex);
    }
}

__global__ void k_seg_clear(uint32_t *flags, unsigned long long *cnt) {
    if (threadIdx.x < 2) flags[threadIdx.x] = 0;
    if (threadIdx.x < 4) cnt[threadIdx.x] = 0;
}

void launch_seg_validate(const double *seg, int64_t n, const double *xyz, int64_t nv, const int32_t *tri,
                         int64_t nt, uint32_t *flags, unsigned long long *cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_seg_clear, dim3(1), dim3(64), 0, s, flags, cnt);
    const int64_t work = std::max<int64_t>(6 * n, std::max<int64_t>(3 * nv, 3 * nt));
    const unsigned grid = (unsigned)std::min<int64_t>(std::max<int64_t>((work + 255) / 256, 1), 4096);
    hipLaunchKernelGGL(k_seg_validate, dim3(grid), dim3(256), 0, s, seg, n, xyz, nv, tri, nt, flags);
}

void launch_seg_mesh(const double *xyz, int64_t nv, const int32_t *tri, int64_t nt, double *P,
                     double *tbox, double *mbox, hipStream_t s) {
    const int64_t ntiles = (nt + MESH_TK - 1) / MESH_TK;
    if (ntiles > 0)
        hipLaunchKernelGGL(k_seg_mesh, dim3((unsigned)ntiles), dim3(64), 0, s, xyz, nv, tri, nt, P, tbox);
    hipLaunchKernelGGL(k_seg_meshbox, dim3(1), dim3(64), 0, s, tbox, ntiles, mbox);
}

int seg_blocks_per_cu(int mode) {
    int b = 0;
    hipError_t e = mode == 0   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_segs<0>, 64, 0)
                   : mode == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_segs<1>, 64, 0)
                               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_segs<2>, 64, 0);
    return e == hipSuccess && b > 0 ? b : 1;
}

void launch_segs(int mode, const double *seg, int64_t n, const double *P, int64_t nt, const double *tbox,
                 const double *mbox, double r, double *dist, uint8_t *hit, const uint32_t *flags,
                 unsigned long long *cnt, int grid, hipStream_t s) {
    if (n <= 0) return;
    const unsigned g = (unsigned)std::min<int64_t>(grid, (n + 63) / 64);
    if (mode == 0)
        hipLaunchKernelGGL(k_segs<0>, dim3(g), dim3(64), 0, s, seg, n, P, nt, tbox, mbox, r, dist, hit,
                           flags, cnt);
    else if (mode == 1)
        hipLaunchKernelGGL(k_segs<1>, dim3(g), dim3(64), 0, s, seg, n, P, nt, tbox, mbox, r, dist, hit,
                           flags, cnt);
    else
        hipLaunchKernelGGL(k_segs<2>, dim3(g), dim3(64), 0, s, seg, n, P, nt, tbox, mbox, r, dist, hit,
                           flags, cnt);
}

}  // namespace sd3
