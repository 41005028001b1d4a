// Shared device/host definitions of the sd3 GPU path (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sd3 {

// Triangles per tile (TK): 32, 64 (default) or 128, chosen per call.  A tile
// is built by one wave, and a tile pair is TK*TK triangle-pair tests.
constexpr int TK_DEFAULT = 64;
constexpr int TK_MAX = 128;
__host__ __device__ constexpr bool tile_size_ok(int tk) { return tk == 32 || tk == 64 || tk == 128; }
constexpr int WG = 256;  // threads per workgroup of the block-wide kernels

constexpr double U64 = 1.1102230246251565e-16;  // 2^-53
constexpr double U32 = 5.9604644775390625e-08;  // 2^-24
constexpr double SQRT3 = 1.7320508075688772;

// Per-tile metadata.  Vertex coordinates are stored twice: exact FP64 copies
// (t64) and FP32 offsets from the tile origin (t32).
struct TileMeta {
    double o[3];    // origin; an FP32-representable point near the box centre
    double lo[3];   // exact bounding box of the tile's vertices
    double hi[3];
    double rep[3];  // one vertex of the tile (exact), for cheap upper bounds
    float eps;      // Euclidean bound of |t32 vertex - (vertex - o)|
    float rad;      // max |t32 coordinate| over the tile
    int32_t row;    // batch row of the tile
    int32_t n;      // real triangles (slots >= n repeat slot n - 1)
};

// Rescue list entry: a triangle pair whose FP32 bounds did not settle it.
struct Rescue {
    int32_t ta, tb;   // global tile ids (A side, B side)
    uint32_t slots;   // slot in ta | slot in tb << 16
    float lb;         // certified lower bound of the pair distance
};

// Exact list entry: a pair whose FP64 filtered predicates were undecided.
struct ExactItem {
    int32_t ta, tb;
    uint32_t slots;
    int32_t pad;
    double d2;        // FP64 squared distance if the pair turns out disjoint
};

// Row state (one per geometry pair).  Non-negative doubles compare like their
// bit patterns, so unsigned 64-bit atomicMin is a floating-point min.
struct RowState {
    unsigned long long ub;    // upper bound of the row distance (double bits)
    unsigned long long d2;    // min FP64 squared distance found (double bits)
    uint32_t hit;             // 1 once an intersecting pair is certified
    int32_t seed_q;           // queue index evaluated in the seed round, -1 if none
    double margin_scale;      // 2^-36 * (row extent); margin m(ub) = scale + 2^-36 ub
    unsigned long long best;  // seed choice: ordered score bits << 32 | queue index
    double scale;             // feature length scale (upper bound after seeding)
};

// Tile-pair ranker: a 10 -> 64 -> 64 -> 64 -> 1 ReLU MLP in FP32, parameters packed
// as W1[64][10] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] w4[64] b4.
constexpr int MLP_IN = 10;
constexpr int MLP_H = 64;
constexpr int MLP_W1 = 0;
constexpr int MLP_B1 = MLP_W1 + MLP_H * MLP_IN;
constexpr int MLP_W2 = MLP_B1 + MLP_H;
constexpr int MLP_B2 = MLP_W2 + MLP_H * MLP_H;
constexpr int MLP_W3 = MLP_B2 + MLP_H;
constexpr int MLP_B3 = MLP_W3 + MLP_H * MLP_H;
constexpr int MLP_W4 = MLP_B3 + MLP_H;
constexpr int MLP_B4 = MLP_W4 + MLP_H;
constexpr int MLP_NPARAM = MLP_B4 + 1;  // 9089
constexpr int LOG_STRIDE = 12;           // features[10], target, row

__device__ __forceinline__ double bits_to_double(unsigned long long b) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ unsigned long long double_to_bits(double d) { return (unsigned long long)__double_as_longlong(d); }

__device__ __forceinline__ void atomic_min_pos(unsigned long long *p, double v) {
    atomicMin(p, double_to_bits(v));
}

// Order-preserving map of any double to an unsigned 64-bit key.
__device__ __forceinline__ unsigned long long ordered_bits(double d) {
    unsigned long long b = double_to_bits(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_ordered_bits(unsigned long long k) {
    unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return bits_to_double(b);
}

// Wave-wide (64 lanes) reductions.
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o);
        v = w < v ? w : v;
    }
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    return v;
}
// Floating-point specialisations on DPP lane moves (no LDS crossbar): swaps
// within quads (lanes 1,0,3,2 and 2,3,0,1), mirrors within half rows and
// rows, then the broadcasts of lane 15 to the next row and of lane 31 to the
// upper half, which leave the wave's extremum in lane 63; it is read back
// into a scalar.  Lanes a row mask leaves out keep the identity.  Every lane
// of the wave must be active (all callers are convergent); the values
// reduced here are never NaN for valid input.
namespace dpp {
constexpr int QUAD_1032 = 0xB1, QUAD_2301 = 0x4E, ROW_HALF_MIRROR = 0x141, ROW_MIRROR = 0x140,
              ROW_BCAST15 = 0x142, ROW_BCAST31 = 0x143;

// A DPP move of each lane's value; lanes outside the row mask keep ident.
// Moves over all rows (quad swaps, mirrors: every lane has a source) need no
// old value, which saves setting it.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ int mov32(int v, int ident) {
    if constexpr (ROWS == 0xf) return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, false);
    else return __builtin_amdgcn_update_dpp(ident, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float movf(float v, float ident) {
    return __int_as_float(mov32<CTRL, ROWS>(__float_as_int(v), __float_as_int(ident)));
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double movd(double v, double ident) {
    const long long b = __double_as_longlong(v), i = __double_as_longlong(ident);
    const int lo = mov32<CTRL, ROWS>((int)b, (int)i);
    const int hi = mov32<CTRL, ROWS>((int)(b >> 32), (int)(i >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane63(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane63(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
}  // namespace dpp

template <>
__device__ __forceinline__ double wave_min<double>(double v) {
    const double I = __builtin_inf();
    v = fmin(v, dpp::movd<dpp::QUAD_1032>(v, I));
    v = fmin(v, dpp::movd<dpp::QUAD_2301>(v, I));
    v = fmin(v, dpp::movd<dpp::ROW_HALF_MIRROR>(v, I));
    v = fmin(v, dpp::movd<dpp::ROW_MIRROR>(v, I));
    v = fmin(v, dpp::movd<dpp::ROW_BCAST15, 0xa>(v, I));
    v = fmin(v, dpp::movd<dpp::ROW_BCAST31, 0xc>(v, I));
    return dpp::lane63(v);
}
template <>
__device__ __forceinline__ double wave_max<double>(double v) {
    const double I = -__builtin_inf();
    v = fmax(v, dpp::movd<dpp::QUAD_1032>(v, I));
    v = fmax(v, dpp::movd<dpp::QUAD_2301>(v, I));
    v = fmax(v, dpp::movd<dpp::ROW_HALF_MIRROR>(v, I));
    v = fmax(v, dpp::movd<dpp::ROW_MIRROR>(v, I));
    v = fmax(v, dpp::movd<dpp::ROW_BCAST15, 0xa>(v, I));
    v = fmax(v, dpp::movd<dpp::ROW_BCAST31, 0xc>(v, I));
    return dpp::lane63(v);
}
template <>
__device__ __forceinline__ float wave_min<float>(float v) {
    const float I = __builtin_inff();
    v = fminf(v, dpp::movf<dpp::QUAD_1032>(v, I));
    v = fminf(v, dpp::movf<dpp::QUAD_2301>(v, I));
    v = fminf(v, dpp::movf<dpp::ROW_HALF_MIRROR>(v, I));
    v = fminf(v, dpp::movf<dpp::ROW_MIRROR>(v, I));
    v = fminf(v, dpp::movf<dpp::ROW_BCAST15, 0xa>(v, I));
    v = fminf(v, dpp::movf<dpp::ROW_BCAST31, 0xc>(v, I));
    return dpp::lane63(v);
}
template <>
__device__ __forceinline__ float wave_max<float>(float v) {
    const float I = -__builtin_inff();
    v = fmaxf(v, dpp::movf<dpp::QUAD_1032>(v, I));
    v = fmaxf(v, dpp::movf<dpp::QUAD_2301>(v, I));
    v = fmaxf(v, dpp::movf<dpp::ROW_HALF_MIRROR>(v, I));
    v = fmaxf(v, dpp::movf<dpp::ROW_MIRROR>(v, I));
    v = fmaxf(v, dpp::movf<dpp::ROW_BCAST15, 0xa>(v, I));
    v = fmaxf(v, dpp::movf<dpp::ROW_BCAST31, 0xc>(v, I));
    return dpp::lane63(v);
}
// Minimum / maximum over each aligned group of 8 lanes, in every lane of the
// group (quad swaps, then the half-row mirror joins the two quads).
__device__ __forceinline__ float group8_min(float v) {
    const float I = __builtin_inff();
    v = fminf(v, dpp::movf<dpp::QUAD_1032>(v, I));
    v = fminf(v, dpp::movf<dpp::QUAD_2301>(v, I));
    return fminf(v, dpp::movf<dpp::ROW_HALF_MIRROR>(v, I));
}
__device__ __forceinline__ float group8_max(float v) {
    const float I = -__builtin_inff();
    v = fmaxf(v, dpp::movf<dpp::QUAD_1032>(v, I));
    v = fmaxf(v, dpp::movf<dpp::QUAD_2301>(v, I));
    return fmaxf(v, dpp::movf<dpp::ROW_HALF_MIRROR>(v, I));
}
// Minimum / maximum over each aligned group of S lanes (S = 16, 32 or 64),
// left in the group's last lane (and, for S = 16, in every lane of it): the
// steps of the wave reduction that stay inside the group.
template <int S>
__device__ __forceinline__ double group_min(double v) {
    static_assert(S == 16 || S == 32 || S == 64, "group of 16, 32 or 64 lanes");
    const double I = __builtin_inf();
    v = fmin(v, dpp::movd<dpp::QUAD_1032>(v, I));
    v = fmin(v, dpp::movd<dpp::QUAD_2301>(v, I));
    v = fmin(v, dpp::movd<dpp::ROW_HALF_MIRROR>(v, I));
    v = fmin(v, dpp::movd<dpp::ROW_MIRROR>(v, I));
    if constexpr (S >= 32) v = fmin(v, dpp::movd<dpp::ROW_BCAST15, 0xa>(v, I));
    if constexpr (S == 64) v = fmin(v, dpp::movd<dpp::ROW_BCAST31, 0xc>(v, I));
    return v;
}
template <int S>
__device__ __forceinline__ double group_max(double v) {
    static_assert(S == 16 || S == 32 || S == 64, "group of 16, 32 or 64 lanes");
    const double I = -__builtin_inf();
    v = fmax(v, dpp::movd<dpp::QUAD_1032>(v, I));
    v = fmax(v, dpp::movd<dpp::QUAD_2301>(v, I));
    v = fmax(v, dpp::movd<dpp::ROW_HALF_MIRROR>(v, I));
    v = fmax(v, dpp::movd<dpp::ROW_MIRROR>(v, I));
    if constexpr (S >= 32) v = fmax(v, dpp::movd<dpp::ROW_BCAST15, 0xa>(v, I));
    if constexpr (S == 64) v = fmax(v, dpp::movd<dpp::ROW_BCAST31, 0xc>(v, I));
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }
__device__ __forceinline__ unsigned long long lanes_below() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Pruning margin m(ub): far above twice the FP64 rounding error of any pair
// distance in the row (errors scale with the row extent), so a pair skipped
// because its lower bound exceeds ub + m can never hold the FP64 minimum.
__device__ __forceinline__ double row_margin(const RowState &r, double ub) {
    return r.margin_scale + 1.4551915228366852e-11 * ub;  // 2^-36
}

}  // namespace sd3
