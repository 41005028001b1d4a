// sd3 C-ABI: argument checks, device buffers and the pipeline of one call.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/sd3.h"
#include "sd3_kernels.h"
#include "sd3_mlp.h"

using namespace sd3;

// Allocation-free calls (sd3_distance_noalloc): every device buffer of such a
// call is carved from this array.  Each GPU the library runs on holds its own
// copy (at its own address) until the process ends; every allocation-free
// call on one GPU shares it, so such calls must not overlap on a GPU.  Host
// code never passes `scratch` itself to a kernel or a copy (on the host it is
// only a stand-in for the symbol): it uses the per-device address that
// hipGetSymbolAddress returns at set-up (scratch_on_device).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES] = {};

// The device address of `scratch` on HIP device `device`, resolved once per
// device with that device current (the caller's current device is restored).
hipError_t scratch_on_device(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        e = hipSetDevice(device);
        if (e != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t e2 = hipSetDevice(prev);
        if (e != hipSuccess) return e;
        if (e2 != hipSuccess) return e2;
        if (!p) return hipErrorInvalidSymbol;
        scratch_ptr[device] = p;
    }
    *out = scratch_ptr[device];
    return hipSuccess;
}

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

void release(DevBuf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

struct SideState {
    DevBuf xyz, tri, rowbox, t32, t64, ids, meta, mat;
};

constexpr unsigned int QUEUE_BUDGET = 1u << 29;   // tile pairs per queue pass (12 B each)
constexpr unsigned int QUEUE_MIN = 64u * 256u;    // one work item's tile pairs
constexpr unsigned int RESCUE_CAP = 1u << 24;     // FP32 pairs sent to FP64
constexpr unsigned int EXACT_CAP = 1u << 22;      // pairs sent to exact arithmetic
constexpr unsigned int EXACT_CAP_MAX = 1u << 26;  // largest exact list an eager call grows to
// Calls without allocation (sd3_distance_noalloc): every buffer is carved
// from one static device array; smaller work lists, longer queues run in
// more passes.
constexpr unsigned int NOALLOC_QUEUE = 1u << 21;
constexpr unsigned int NOALLOC_RESCUE = 1u << 20;
constexpr unsigned int NOALLOC_EXACT = 1u << 18;
// offset arrays of G + 1 staged per call: v_off, t_off and tile offsets of
// both sides, work items, A blocks, B chunks, sort blocks of both sides
constexpr int N_OFFSETS = 11;
constexpr int64_t NOALLOC_MAX_ROWS = 4096;  // bounds the pinned staging below
// pinned host staging allocated at context creation, enough for the offsets
// (9 arrays of G + 1) and the solid-semantics queries of NOALLOC_MAX_ROWS rows
constexpr size_t NOALLOC_HOST_BYTES = sizeof(int64_t) * N_OFFSETS * (NOALLOC_MAX_ROWS + 1) + 12 * NOALLOC_MAX_ROWS + 4096;

// The buffers of a call outgrew the static scratch (bytes needed so far).
struct ScratchFull {
    size_t need;
};

void *ensure(DevBuf &b, size_t bytes);

// Device work space of one call: a context owns one, and every graph owns its
// own, so that replays never share buffers with eager calls.
struct Workspace {
    SideState side[2];
    DevBuf rows, queue, qlb, rescue, exact, scalars, out_d;
    DevBuf keys0, keys1, vals0, vals1, hist, part, vcode, kc, cub, oc, bn, small, grpA, grpB, wi_lb, wlist, sorttab;
    DevBuf seg_in, seg_mesh, seg_out;  // segment calls: staged inputs, prepared mesh, outputs
    DevBuf vol_items, vol_part;        // volume calls: work items, partial sums
    DevBuf solid;                      // solid semantics: queries, directions, results
    // work-list capacities (a call's options may lower them)
    int64_t queue_budget = QUEUE_BUDGET;
    unsigned int rescue_cap = RESCUE_CAP, exact_cap = EXACT_CAP;
    // static scratch mode: buffers are carved from [arena, arena + arena_cap)
    // in call order and never freed; the DevBufs stay empty
    char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    bool arena_full = false;
    void *buf(DevBuf &b, size_t bytes) {
        if (!arena) return ensure(b, bytes);
        if (bytes == 0) bytes = 256;
        const size_t off = (arena_used + 255) & ~(size_t)255;
        arena_used = off + bytes;
        if (arena_used > arena_cap) {
            // keep counting (the error reports the whole need); nothing is
            // launched or copied before the plan checks arena_full
            arena_full = true;
            return arena;
        }
        return arena + off;
    }
    void release_all() {
        for (auto &sd : side) {
            DevBuf *bs[] = {&sd.xyz, &sd.tri, &sd.rowbox, &sd.t32, &sd.t64, &sd.ids, &sd.meta, &sd.mat};
            for (DevBuf *b : bs) release(*b);
        }
        DevBuf *bs[] = {&rows, &queue, &qlb, &rescue, &exact, &scalars, &out_d, &keys0, &keys1,
                        &vals0, &vals1, &hist, &part, &vcode, &kc, &cub, &oc, &bn, &small, &grpA, &grpB, &wi_lb,
                        &wlist, &sorttab, &seg_in, &seg_mesh, &seg_out, &vol_items, &vol_part, &solid};
        for (DevBuf *b : bs) release(*b);
    }
};

struct Plan {
    int64_t G = 0;
    int tk = TK_DEFAULT;                // triangles per tile
    std::vector<int64_t> tileA, tileB;  // [G+1] tile offsets
    std::vector<int64_t> wi;            // [G+1] work-item offsets
    std::vector<int64_t> blkA, chkB;    // [G+1] A-block (64 tiles) / B-chunk (256 tiles) offsets
    std::vector<int64_t> sbA, sbB;      // [G+1] sort blocks of each row (rsi items each)
    int rsi = RS_ITEMS;                 // items per sort block
    int64_t max_row = 0;                // most triangles in one row of either side
    int64_t potential = 0;              // sum of tilesA * tilesB
};

}  // namespace

struct sd3_ctx {
    int device = 0;
    int cus = 0;
    std::string err;
    Workspace ws;
    Workspace sws;        // allocation-free calls: carved from the device's `scratch`
    DevBuf mlp;           // ranker training scratch
    void *pin = nullptr;  // pinned host staging: offsets up, counters down
    size_t pin_cap = 0;
    int pairs_grid[2][2][3] = {};         // [precision][mode][tile size 32/64/128]
    int seg_grid[3] = {};                 // segment kernels, per operator
    std::map<uint64_t, int> tuned;        // workload key -> tile size (sd3_autotune)
    hipEvent_t ev[8] = {};
    KernelEvents *kev = nullptr;  // created on the first timed call
    // a second stream (default priority) and two events that fork the
    // learned ranking off a call's stream beside the tile copies and join it
    // back (graph capture records the fork as two parallel branches)
    hipStream_t side = nullptr;
    hipEvent_t fork[2] = {};
};

namespace {

constexpr int64_t RESOLVE_MAX_ROWS = 64;           // FP64 rescue inside the exact launch
constexpr int64_t CULL_MIN_ROWS = 64;              // pre-cull of large sorts above this many rows
constexpr int64_t COMPACT_MIN_ROWS = 64;           // compacted work lists above this
// device scalars: [0] queue count [1] queue head [2] rescue count [3] rescue
// head [4] exact count [7] seed pass head [8] [9] work-item counts [11] exact
// blocks done [12] [13] validation flags of a and b; the counters follow at
// byte 64
constexpr size_t SCALAR_BYTES = 64 + sizeof(unsigned long long) * C_NCOUNTERS;

struct HipError {
    hipError_t e;
    const char *what;
};

void check(hipError_t e, const char *what) {
    if (e != hipSuccess) throw HipError{e, what};
}

void *ensure(DevBuf &b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (b.cap >= bytes) return b.p;
    if (b.p) check(hipFree(b.p), "hipFree");
    b.p = nullptr;
    b.cap = 0;
    size_t want = bytes + bytes / 4;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        e = hipMalloc(&b.p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw HipError{hipErrorOutOfMemory, "hipMalloc"};
        }
        want = bytes;
    }
    b.cap = want;
    return b.p;
}

// Pinned host staging of `bytes` (+ a 512-byte readback area at the end).
char *ensure_pinned(sd3_ctx *ctx, size_t bytes) {
    bytes += 512;
    if (ctx->pin_cap < bytes) {
        if (ctx->pin) check(hipHostFree(ctx->pin), "hipHostFree");
        ctx->pin = nullptr;
        ctx->pin_cap = 0;
        size_t want = bytes + bytes / 4 + 4096;
        check(hipHostMalloc(&ctx->pin, want, hipHostMallocDefault), "hipHostMalloc");
        ctx->pin_cap = want;
    }
    return (char *)ctx->pin;
}

char *readback_area(sd3_ctx *ctx) { return (char *)ctx->pin + ctx->pin_cap - 512; }

// Pinned staging for a call on workspace `ws`: an allocation-free call only
// uses what the context allocated at creation (its row limit keeps `bytes`
// within it).
char *staging(sd3_ctx *ctx, const Workspace &ws, size_t bytes) {
    if (ws.arena && bytes + 512 > ctx->pin_cap) throw HipError{hipErrorOutOfMemory, "static host staging"};
    return ensure_pinned(ctx, bytes);
}

sd3_status fail(sd3_ctx *ctx, sd3_status s, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return s;
}

// Host-side structural checks shared by every entry point.
sd3_status check_geoms(const sd3_geoms *g, std::string &msg) {
    if (!g) {
        msg = "geometry batch is NULL";
        return SD3_E_INVALID_ARG;
    }
    if (g->count < 0) {
        msg = "count < 0";
        return SD3_E_INVALID_ARG;
    }
    if (g->mem != SD3_MEM_HOST && g->mem != SD3_MEM_DEVICE) {
        msg = "unknown memory kind";
        return SD3_E_INVALID_ARG;
    }
    if (!g->v_off || !g->t_off) {
        msg = "offsets are NULL";
        return SD3_E_INVALID_ARG;
    }
    if (g->v_off[0] != 0 || g->t_off[0] != 0) {
        msg = "offsets must start at 0";
        return SD3_E_INVALID_ARG;
    }
    for (int64_t i = 0; i < g->count; i++) {
        if (g->v_off[i + 1] < g->v_off[i] || g->t_off[i + 1] < g->t_off[i]) {
            msg = "offsets decrease at row " + std::to_string(i);
            return SD3_E_INVALID_ARG;
        }
    }
    int64_t nv = g->v_off[g->count], nt = g->t_off[g->count];
    if (nt > INT32_MAX - 1 || nv > ((int64_t)1 << 40)) {
        msg = "batch too large (at most 2^31 - 2 triangles)";
        return SD3_E_INVALID_ARG;
    }
    if ((nv > 0 && !g->xyz) || (nt > 0 && !g->tri)) {
        msg = "xyz or tri is NULL";
        return SD3_E_INVALID_ARG;
    }
    for (int64_t i = 0; i < g->count; i++) {
        if (g->t_off[i + 1] > g->t_off[i] && g->v_off[i + 1] == g->v_off[i]) {
            msg = "row " + std::to_string(i) + " has triangles but no vertices";
            return SD3_E_INDEX_RANGE;
        }
    }
    return SD3_OK;
}

sd3_status check_host_data(const sd3_geoms *g, std::string &msg) {
    int64_t nv = g->v_off[g->count];
    for (int64_t i = 0; i < nv * 3; i++) {
        double x = std::fabs(g->xyz[i]);
        if (!(x <= 1.7976931348623157e308)) {
            msg = "non-finite coordinate at vertex " + std::to_string(i / 3);
            return SD3_E_NONFINITE;
        }
        if (x != 0.0 && (x < 0x1p-256 || x > 0x1p256)) {
            msg = "coordinate magnitude outside [2^-256, 2^256] at vertex " + std::to_string(i / 3);
            return SD3_E_RANGE;
        }
    }
    for (int64_t r = 0; r < g->count; r++) {
        int64_t nvr = g->v_off[r + 1] - g->v_off[r];
        for (int64_t t = g->t_off[r]; t < g->t_off[r + 1]; t++)
            for (int k = 0; k < 3; k++) {
                int32_t v = g->tri[3 * t + k];
                if (v < 0 || v >= nvr) {
                    msg = "triangle " + std::to_string(t) + " indexes vertex " + std::to_string(v) +
                          " outside row " + std::to_string(r);
                    return SD3_E_INDEX_RANGE;
                }
            }
    }
    return SD3_OK;
}

int64_t tiles_of(int64_t nt, int tk) { return (nt + tk - 1) / tk; }

int tk_index(int tk) { return tk == 32 ? 0 : (tk == 64 ? 1 : 2); }

int ilog2(uint64_t x) {
    int r = 0;
    while (x > 1) {
        x >>= 1;
        r++;
    }
    return r;
}

// Workload class of the autotuner: operator, precision, order, and the
// binary magnitudes of the row count and of the mean triangles per row.
uint64_t workload_key(const sd3_opts &o, int mode, const sd3_geoms *a, const sd3_geoms *b) {
    int64_t G = a->count;
    int64_t tri = a->t_off[G] + b->t_off[G];
    int64_t mean = G > 0 ? tri / G : 0;
    return (uint64_t)mode | ((uint64_t)o.precision << 2) | ((uint64_t)o.order << 4) |
           ((uint64_t)ilog2((uint64_t)G + 1) << 8) | ((uint64_t)ilog2((uint64_t)mean + 1) << 16);
}

int choose_tile(const sd3_ctx *ctx, const sd3_opts &o, int mode, const sd3_geoms *a,
                const sd3_geoms *b) {
    if (o.tile != SD3_TILE_AUTO) return o.tile;
    auto it = ctx->tuned.find(workload_key(o, mode, a, b));
    return it != ctx->tuned.end() ? it->second : TK_DEFAULT;
}

// Argument checks of the two operators and of graph creation.
sd3_status check_call(sd3_ctx *ctx, const sd3_geoms *a, const sd3_geoms *b, const double *dist,
                      const uint8_t *hit, const sd3_opts *opts_in, int mode, sd3_opts &opts) {
    std::string msg;
    sd3_status st = check_geoms(a, msg);
    if (st == SD3_OK) st = check_geoms(b, msg);
    if (st != SD3_OK) return fail(ctx, st, msg);
    if (a->count != b->count) return fail(ctx, SD3_E_INVALID_ARG, "batches differ in count");
    if (a->mem != b->mem) return fail(ctx, SD3_E_INVALID_ARG, "batches differ in memory kind");
    if ((mode == 0 && !dist) || (mode == 1 && !hit))
        return fail(ctx, SD3_E_INVALID_ARG, "output pointer is NULL");
    sd3_default_opts(&opts);
    if (opts_in) opts = *opts_in;
    if (opts.precision != SD3_PREC_FP32_RESCUE && opts.precision != SD3_PREC_FP64)
        return fail(ctx, SD3_E_INVALID_ARG, "unknown precision");
    if (opts.order != SD3_ORDER_BOUND && opts.order != SD3_ORDER_NONE &&
        opts.order != SD3_ORDER_LEARNED)
        return fail(ctx, SD3_E_INVALID_ARG, "unknown order");
    if (opts.order == SD3_ORDER_LEARNED && !opts.ranker)
        return fail(ctx, SD3_E_INVALID_ARG, "SD3_ORDER_LEARNED needs opts.ranker");
    if (opts.tile != SD3_TILE_AUTO && !tile_size_ok(opts.tile))
        return fail(ctx, SD3_E_INVALID_ARG, "tile must be 0, 32, 64 or 128");
    if (opts.queue_cap < 0) return fail(ctx, SD3_E_INVALID_ARG, "queue_cap < 0");
    if (opts.rescue_cap < 0 || opts.exact_cap < 0 || opts.rescue_cap > INT32_MAX || opts.exact_cap > INT32_MAX)
        return fail(ctx, SD3_E_INVALID_ARG, "rescue_cap / exact_cap outside [0, 2^31)");
    if (opts.semantics != SD3_SURFACE && opts.semantics != SD3_SOLID)
        return fail(ctx, SD3_E_INVALID_ARG, "unknown semantics");
    if (opts.log && (opts.log_cap < 0 || a->mem != SD3_MEM_DEVICE))
        return fail(ctx, SD3_E_INVALID_ARG, "log needs a device buffer and log_cap >= 0");
    if (a->mem == SD3_MEM_HOST) {
        st = check_host_data(a, msg);
        if (st == SD3_OK) st = check_host_data(b, msg);
        if (st != SD3_OK) return fail(ctx, st, msg);
    }
    return SD3_OK;
}

// Phase events (opts.timing): ev[0] at the start, ev[k+1] at the end of phase k.
struct PhaseClock {
    sd3_ctx *ctx;
    hipStream_t s;
    bool on;
    void mark(int k) {
        if (!on) return;
        if (!ctx->ev[k]) check(hipEventCreate(&ctx->ev[k]), "hipEventCreate");
        check(hipEventRecord(ctx->ev[k], s), "hipEventRecord");
    }
    void read(double *ms) {
        for (int k = 0; k < 7; k++) {
            float f = 0.0f;
            if (on) check(hipEventElapsedTime(&f, ctx->ev[k], ctx->ev[k + 1]), "hipEventElapsedTime");
            ms[k] = f;
        }
    }
};

// One planned call: host plan and the device views of its work space.
struct Call {
    int mode = 0;
    sd3_opts opts{};
    Plan P;
    SideBufs A{}, B{};
    PrepBufs PB{};
    QueueGeo Q{};
    Lists L{};
    RowState *rows = nullptr;
    unsigned int *sc = nullptr;  // device scalars + counters (SCALAR_BYTES)
    uint32_t *flags = nullptr;   // sc + 12: validation flags of a, b
    int64_t n_wi = 0, per_pass = 0;
    int passes = 0;
    bool seed = false;
    int grid_pairs = 0;
    double *dd = nullptr;  // device outputs
    uint8_t *hd = nullptr;
};

// Upload (host inputs) or reference (device inputs) one side and size its
// buffers.  No kernel reads the data here.
void setup_side(Workspace &ws, int which, const sd3_geoms *g, int64_t NT, int tk, bool fp64,
                const int64_t *d_offs, SideBufs &S, hipStream_t s) {
    SideState &st = ws.side[which];
    int64_t G = g->count, nv = g->v_off[G], nt = g->t_off[G];
    S.G = G;
    S.nv = nv;
    S.nt = nt;
    S.NT = NT;
    S.tk = tk;
    if (g->mem == SD3_MEM_HOST) {
        double *x = (double *)ws.buf(st.xyz, sizeof(double) * 3 * nv);
        int32_t *t = (int32_t *)ws.buf(st.tri, sizeof(int32_t) * 3 * nt);
        // (a static scratch already too small stops before any copy)
        if (ws.arena_full) throw ScratchFull{ws.arena_used};
        if (nv) check(hipMemcpyAsync(x, g->xyz, sizeof(double) * 3 * nv, hipMemcpyHostToDevice, s), "H2D xyz");
        if (nt) check(hipMemcpyAsync(t, g->tri, sizeof(int32_t) * 3 * nt, hipMemcpyHostToDevice, s), "H2D tri");
        S.xyz = x;
        S.tri = t;
    } else {
        S.xyz = g->xyz;
        S.tri = g->tri;
    }
    S.v_off = d_offs;
    S.t_off = d_offs + (G + 1);
    S.tile_off = d_offs + 2 * (G + 1);
    // replicas of the row boxes spread the reduction atomics of many blocks
    // over one row; both sides use the count for the larger one (set by the
    // caller), room for the most any side can ask for is kept here
    S.boxrep = rowbox_replicas(nv, G);
    const int64_t rep_room = std::max<int64_t>(rowbox_replicas((int64_t)1 << 40, G), 1);
    S.rowbox = (unsigned long long *)ws.buf(st.rowbox, sizeof(unsigned long long) * 6 * rep_room *
                                                           (G > 0 ? G : 1));
    // FP32 tile copies for the FP32 path, FP64 copies for the plain FP64
    // pass (both written only for queued tiles); the triangle id of each
    // slot for both (the FP32 path gathers FP64 vertices for its few rescues)
    S.t32 = fp64 ? nullptr : (float *)ws.buf(st.t32, sizeof(float) * 9 * tk * S.NT);
    S.t64 = fp64 ? (double *)ws.buf(st.t64, sizeof(double) * 9 * tk * S.NT) : nullptr;
    S.ids = (int32_t *)ws.buf(st.ids, sizeof(int32_t) * tk * S.NT);
    S.meta = (TileMeta *)ws.buf(st.meta, sizeof(TileMeta) * S.NT);
    S.mat = (uint32_t *)ws.buf(st.mat, sizeof(uint32_t) * S.NT);
}

// Plans a call: tiles and work items per row, buffer sizes in `ws`, offsets
// (and host inputs) staged on stream s.  Launches no kernel.
void plan_call(sd3_ctx *ctx, Workspace &ws, const sd3_geoms *a, const sd3_geoms *b,
               const sd3_opts &opts, int mode, int tk, double *dist, uint8_t *hit, Call &C,
               hipStream_t s) {
    const int64_t G = a->count;
    C.mode = mode;
    C.opts = opts;
    Plan &P = C.P;
    P.G = G;
    P.tk = tk;
    P.potential = 0;
    P.tileA.assign(G + 1, 0);
    P.tileB.assign(G + 1, 0);
    P.wi.assign(G + 1, 0);
    P.blkA.assign(G + 1, 0);
    P.chkB.assign(G + 1, 0);
    for (int64_t g = 0; g < G; g++) {
        int64_t na = tiles_of(a->t_off[g + 1] - a->t_off[g], tk);
        int64_t nb = tiles_of(b->t_off[g + 1] - b->t_off[g], tk);
        P.tileA[g + 1] = P.tileA[g] + na;
        P.tileB[g + 1] = P.tileB[g] + nb;
        P.blkA[g + 1] = P.blkA[g] + (na + 63) / 64;
        P.chkB[g + 1] = P.chkB[g] + (nb + 255) / 256;
        // a row with an empty side has no work items
        P.wi[g + 1] = P.wi[g] + (na > 0 && nb > 0 ? ((na + 63) / 64) * ((nb + 255) / 256) : 0);
        P.potential += na * nb;
    }
    // sort blocks: each row's items in blocks of rsi (larger blocks for large
    // sorts)
    {
        const int64_t n = a->t_off[G] + b->t_off[G];
        P.rsi = n <= SMALL_SORT ? RS_ITEMS : 2 * RS_ITEMS;
        P.sbA.assign(G + 1, 0);
        P.sbB.assign(G + 1, 0);
        P.max_row = 0;
        for (int64_t g = 0; g < G; g++) {
            const int64_t na = a->t_off[g + 1] - a->t_off[g], nb = b->t_off[g + 1] - b->t_off[g];
            P.sbA[g + 1] = P.sbA[g] + (na + P.rsi - 1) / P.rsi;
            P.sbB[g + 1] = P.sbB[g] + (nb + P.rsi - 1) / P.rsi;
            P.max_row = std::max(P.max_row, std::max(na, nb));
        }
    }
    // all offsets in one pinned staging copy: [A v_off | A t_off | A tiles |
    // B v_off | B t_off | B tiles | work items | A blocks | B chunks | A sort
    // blocks | B sort blocks]
    const int64_t G1 = G + 1;
    int64_t *hs = (int64_t *)staging(ctx, ws, sizeof(int64_t) * N_OFFSETS * G1);
    memcpy(hs, a->v_off, sizeof(int64_t) * G1);
    memcpy(hs + G1, a->t_off, sizeof(int64_t) * G1);
    memcpy(hs + 2 * G1, P.tileA.data(), sizeof(int64_t) * G1);
    memcpy(hs + 3 * G1, b->v_off, sizeof(int64_t) * G1);
    memcpy(hs + 4 * G1, b->t_off, sizeof(int64_t) * G1);
    memcpy(hs + 5 * G1, P.tileB.data(), sizeof(int64_t) * G1);
    memcpy(hs + 6 * G1, P.wi.data(), sizeof(int64_t) * G1);
    memcpy(hs + 7 * G1, P.blkA.data(), sizeof(int64_t) * G1);
    memcpy(hs + 8 * G1, P.chkB.data(), sizeof(int64_t) * G1);
    memcpy(hs + 9 * G1, P.sbA.data(), sizeof(int64_t) * G1);
    memcpy(hs + 10 * G1, P.sbB.data(), sizeof(int64_t) * G1);
    int64_t *ds = (int64_t *)ws.buf(ws.small, sizeof(int64_t) * N_OFFSETS * G1);
    const bool fp64 = opts.precision == SD3_PREC_FP64;
    setup_side(ws, 0, a, P.tileA[G], tk, fp64, ds, C.A, s);
    setup_side(ws, 1, b, P.tileB[G], tk, fp64, ds + 3 * G1, C.B, s);
    C.A.boxrep = C.B.boxrep = std::max(C.A.boxrep, C.B.boxrep);
    {
        int64_t n = C.A.nt + C.B.nt;
        const int64_t nb = P.sbA[G] + P.sbB[G];
        C.PB.keys[0] = (uint32_t *)ws.buf(ws.keys0, sizeof(uint32_t) * n);
        C.PB.keys[1] = (uint32_t *)ws.buf(ws.keys1, sizeof(uint32_t) * n);
        C.PB.vals[0] = (int32_t *)ws.buf(ws.vals0, sizeof(int32_t) * n);
        C.PB.vals[1] = (int32_t *)ws.buf(ws.vals1, sizeof(int32_t) * n);
        C.PB.hist = (uint32_t *)ws.buf(ws.hist, sizeof(uint32_t) * 256 * (nb + 1));
        C.PB.part = (uint32_t *)ws.buf(ws.part, sizeof(uint32_t) * (256 * (nb + 1) / 4096 + 2));
        C.PB.vcode = P.rsi > RS_ITEMS ? (uint32_t *)ws.buf(ws.vcode, sizeof(uint32_t) * (C.A.nv + C.B.nv))
                                      : nullptr;
        // a large sort of many rows builds tiles of the triangles whose boxes
        // meet the other side's row box only (intersects), or come within the
        // row's cull distance of it (distance; not in allocation-free calls,
        // whose static scratch keeps its size).  A call of a few rows is a
        // short chain of launches whose tile build is small: the cull's extra
        // loads cost it more than they save (the 4M-triangle TIN against the
        // 1M-triangle blob: 0.435 -> 0.509 ms per distance call)
        const bool cull = C.PB.vcode && G > CULL_MIN_ROWS && (mode == 1 || (mode == 0 && !ws.arena));
        C.PB.kc = cull ? (int32_t *)ws.buf(ws.kc, sizeof(int32_t) * 2 * G) : nullptr;
        C.PB.cub = cull && mode == 0 ? (double *)ws.buf(ws.cub, sizeof(double) * G) : nullptr;
        C.PB.oc = cull ? (uint8_t *)ws.buf(ws.oc, (size_t)(C.A.nv + C.B.nv)) : nullptr;
        C.PB.seg = SortSeg{ds + 9 * G1, ds + 10 * G1, C.A.t_off, C.B.t_off, G, C.A.nt, P.sbA[G], nb, P.rsi,
                           G >= SORT_TABLE_MIN_ROWS ? (SBlock *)ws.buf(ws.sorttab, sizeof(SBlock) * (nb + 1))
                                                    : nullptr,
                           C.PB.kc, cull ? (int32_t *)ws.buf(ws.bn, sizeof(int32_t) * (nb + 1)) : nullptr};
    }
    QueueGeo &Q = C.Q;
    Q.wi_off = ds + 6 * G1;
    Q.blkA = ds + 7 * G1;
    Q.chkB = ds + 8 * G1;
    Q.gA = (GroupBox *)ws.buf(ws.grpA, sizeof(GroupBox) * (P.blkA[G] + 1));
    Q.gB = (GroupBox *)ws.buf(ws.grpB, sizeof(GroupBox) * (P.chkB[G] + 1));
    Q.wi_lb = (float *)ws.buf(ws.wi_lb, sizeof(float) * (P.wi[G] + 1));
    Q.wlist = (int32_t *)ws.buf(ws.wlist, sizeof(int32_t) * (P.wi[G] + 1));
    C.rows = (RowState *)ws.buf(ws.rows, sizeof(RowState) * (G > 0 ? G : 1));

    Lists &L = C.L;
    const int64_t budget = opts.queue_cap > 0 ? std::min<int64_t>(std::max<int64_t>(opts.queue_cap, QUEUE_MIN),
                                                                  ws.queue_budget)
                                              : ws.queue_budget;
    unsigned int qcap = (unsigned int)std::min<int64_t>(std::max<int64_t>(P.potential, 1), budget);
    L.queue = (int2 *)ws.buf(ws.queue, sizeof(int2) * qcap);
    L.qlb = (float *)ws.buf(ws.qlb, sizeof(float) * qcap);
    L.qcap = qcap;
    // work-list capacities: the workspace's, or smaller ones from the options
    // (an exact list that overflowed is enlarged through them on a re-run)
    const int64_t xmax = ws.arena ? (int64_t)NOALLOC_EXACT : (int64_t)EXACT_CAP_MAX;
    L.rcap = opts.rescue_cap > 0 ? (unsigned int)std::min<int64_t>(opts.rescue_cap, ws.rescue_cap) : ws.rescue_cap;
    L.xcap = (unsigned int)std::min<int64_t>(opts.exact_cap > 0 ? opts.exact_cap : ws.exact_cap, xmax);
    L.rescue = (Rescue *)ws.buf(ws.rescue, sizeof(Rescue) * L.rcap);
    L.exact = (ExactItem *)ws.buf(ws.exact, sizeof(ExactItem) * L.xcap);
    unsigned int *sc = (unsigned int *)ws.buf(ws.scalars, SCALAR_BYTES);
    C.sc = sc;
    C.flags = sc + 12;
    C.PB.flags = C.flags;
    L.qcount = sc;
    L.qhead = sc + 1;
    L.rcount = sc + 2;
    L.rhead = sc + 3;
    L.xcount = sc + 4;
    L.counters = (unsigned long long *)(sc + 16);
    Q.wcount = sc + 8;  // [8] seeding, [9] filtering
    L.seed_pass = 0;
    L.log = mode == 0 ? opts.log : nullptr;
    L.log_cap = (unsigned long long)opts.log_cap;
    L.log_count = L.counters + C_LOGGED;
    L.xdone = sc + 11;
    L.nrows = G;

    const int prec = opts.precision == SD3_PREC_FP64 ? 1 : 0;
    int &gp = ctx->pairs_grid[prec][mode][tk_index(tk)];
    if (gp == 0) gp = ctx->cus * pairs_blocks_per_cu(prec, mode, tk);
    C.grid_pairs = gp;
    // the queue holds at most qcap tile pairs: split the work items into
    // passes whose potential tile pairs fit
    C.n_wi = P.wi[G];
    C.per_pass = P.potential <= (int64_t)qcap ? std::max<int64_t>(C.n_wi, 1)
                                              : std::max<int64_t>(1, qcap / QUEUE_MIN);
    C.passes = (int)((C.n_wi + C.per_pass - 1) / C.per_pass);
    // compacted work lists spare the later kernels' blocks a row search; with
    // few rows that search is short and every block checks its own item
    Q.compact = C.n_wi <= C.per_pass && G > COMPACT_MIN_ROWS ? 1 : 0;
    C.seed = mode == 0 && opts.order != SD3_ORDER_NONE && C.n_wi > 0;
    if (a->mem == SD3_MEM_DEVICE) {
        C.dd = dist;
        C.hd = hit;
    } else {
        char *ob = (char *)ws.buf(ws.out_d, (sizeof(double) + 8) * (G > 0 ? G : 1));
        C.dd = dist ? (double *)ob : nullptr;
        C.hd = hit ? (uint8_t *)(ob + sizeof(double) * G) : nullptr;
    }
    // every buffer is placed: stage the offsets (a static scratch too small
    // for the call stops here, before anything is copied or launched)
    if (ws.arena_full) throw ScratchFull{ws.arena_used};
    check(hipMemcpyAsync(ds, hs, sizeof(int64_t) * N_OFFSETS * G1, hipMemcpyHostToDevice, s), "H2D offsets");
}

// Device validation (flags in the scalar block) fused with the row boxes: the
// first kernels of every call (host inputs were also checked on the host).
// Without `indices` the triangle indices are checked by the key kernel: every
// kernel clamps an index into its row before any gather, and the final kernel
// writes no result while a flag is set.
void enqueue_validate(Call &C, hipStream_t s, bool indices) {
    launch_validate_rowbox(C.A, C.B, C.PB, C.flags, C.L, s, indices);
}

// Every kernel of the call after validation, in stream order, with no host
// synchronisation (graph capture records exactly this).
void enqueue_pipeline(sd3_ctx *ctx, Call &C, hipStream_t s, PhaseClock *clk, KernelEvents *kev) {
    auto mark = [&](int k) {
        if (clk) clk->mark(k);
    };
    SideBufs &A = C.A, &B = C.B;
    QueueGeo &Q = C.Q;
    Lists &L = C.L;
    const int64_t G = C.P.G;
    const int mode = C.mode;
    const int prec = C.opts.precision == SD3_PREC_FP64 ? 1 : 0;
    launch_prep(A, B, C.PB, sort_key(C.P.max_row), C.rows, s, kev);
    launch_group_boxes(A, B, Q, C.P.blkA[G], C.P.chkB[G], s);
    mark(2);
    launch_queue(A, B, Q, C.n_wi, 0, C.rows, L, mode == 0 ? Q_SEED : Q_GROUPS, s, 0);
    // (the rows' feature scale is set by the work-item compaction, else by the
    // first pass's filter)
    // seed round of each pass (distance): the filter (box bound) or the
    // ranker records each row's best-ranked queued tile pair, and a pass of
    // the tile-pair kernel over the rows' choices evaluates them first
    const bool learned = C.seed && C.opts.order == SD3_ORDER_LEARNED;
    const int rank = C.seed && !learned ? 1 : 0;
    Lists LS = L;
    LS.qhead = C.sc + 7;
    LS.seed_pass = 1;
    for (int64_t w0 = 0; w0 < C.n_wi; w0 += C.per_pass) {
        int64_t nw = std::min(C.per_pass, C.n_wi - w0);
        if (w0 > 0) {
            launch_reset_queue(L, s);
            if (C.seed) launch_seed_reset(C.rows, G, LS.qhead, s);
        }
        if (kev) kev->begin(KE_FILTER, s);
        launch_queue(A, B, Q, nw, w0, C.rows, L, mode == 0 ? Q_FILTER_DIST : Q_FILTER_HIT, s, rank);
        if (kev) kev->end(KE_FILTER, s);
        if (learned && G > RESOLVE_MAX_ROWS) {
            // the ranking and the tile copies read the queue and write disjoint
            // state: in calls of many rows the ranking runs on the side stream
            // beside the copies (a call of a few rows, a short chain of
            // launches, gains nothing from the join)
            check(hipEventRecord(ctx->fork[0], s), "hipEventRecord");
            check(hipStreamWaitEvent(ctx->side, ctx->fork[0], 0), "hipStreamWaitEvent");
            launch_rank(A, B, C.rows, L, C.opts.ranker, ctx->cus * 2, ctx->side);
            check(hipEventRecord(ctx->fork[1], ctx->side), "hipEventRecord");
            launch_materialize(A, B, L, prec, ctx->cus * 16, s);
            check(hipStreamWaitEvent(s, ctx->fork[1], 0), "hipStreamWaitEvent");
        } else {
            launch_materialize(A, B, L, prec, ctx->cus * 16, s);
            if (learned) launch_rank(A, B, C.rows, L, C.opts.ranker, ctx->cus * 2, s);
        }
        // at most one seed per row
        if (C.seed) launch_pairs(A, B, C.rows, LS, prec, mode, (int)std::min<int64_t>(C.grid_pairs, G), s);
        if (w0 == 0) mark(3);
        if (kev) kev->begin(KE_PAIRS, s);
        launch_pairs(A, B, C.rows, L, prec, mode, C.grid_pairs, s);
        if (kev) kev->end(KE_PAIRS, s);
    }
    if (C.n_wi == 0) mark(3);
    mark(4);
    // up to 65536 rows the exact kernel's last block also writes the results;
    // with few rows (a short rescue list) the FP64 rescue shares that launch
    const int64_t fin_rows = G <= 65536 ? G : 0;
    if (prec == 0 && G <= RESOLVE_MAX_ROWS) {
        launch_resolve(A, B, C.rows, L, mode, 64, s, fin_rows, C.dd, C.hd, C.flags);
        mark(5);
        mark(6);
        return;
    }
    if (prec == 0) launch_rescue(A, B, C.rows, L, mode, ctx->cus * 4, s);
    mark(5);
    launch_exact(A, B, C.rows, L, mode, 64, s, fin_rows, C.dd, C.hd, C.flags);
    mark(6);
    if (fin_rows == 0) launch_finalize(C.rows, G, C.dd, C.hd, L, C.flags, s);
}

sd3_status flags_status(sd3_ctx *ctx, const unsigned int *sc_h) {
    uint32_t f = sc_h[12] | sc_h[13];
    if (f & V_NONFINITE) return fail(ctx, SD3_E_NONFINITE, "non-finite coordinate");
    if (f & V_RANGE) return fail(ctx, SD3_E_RANGE, "coordinate magnitude outside [2^-256, 2^256]");
    if (f & V_INDEX) return fail(ctx, SD3_E_INDEX_RANGE, "triangle index outside its row");
    return SD3_OK;
}

// Status of a finished call from its scalars and counters (read back).
sd3_status call_status(sd3_ctx *ctx, const Call &C, const unsigned int *sc_h,
                       const unsigned long long *cnt_h) {
    sd3_status st = flags_status(ctx, sc_h);
    if (st != SD3_OK) return st;
    if (sc_h[0] > C.L.qcap || cnt_h[C_QUEUE_OVF] != 0) return fail(ctx, SD3_E_CAPACITY, "tile-pair queue overflow");
    if (sc_h[2] > C.L.rcap) return fail(ctx, SD3_E_CAPACITY, "rescue list overflow");
    if (sc_h[4] > C.L.xcap) return fail(ctx, SD3_E_CAPACITY, "exact list overflow");
    return SD3_OK;
}

void fill_counts(const Call &C, const unsigned int *sc_h, const unsigned long long *cnt_h,
                 sd3_stats *stats) {
    memset(stats, 0, sizeof(*stats));
    stats->tile_pairs_total = C.P.potential;
    stats->tile_pairs_candidate = (int64_t)(cnt_h[C_TP_CAND] + sc_h[0]);
    stats->tile_pairs_evaluated = (int64_t)cnt_h[C_TP_EVAL];
    stats->tri_pairs_boxed = (int64_t)cnt_h[C_TRI_BOXED];
    stats->tri_pairs_fp32 = (int64_t)cnt_h[C_TRI32];
    stats->tri_pairs_fp64 = (int64_t)cnt_h[C_TRI64];
    stats->rescued = (int64_t)cnt_h[C_RESCUED];
    stats->exact = (int64_t)cnt_h[C_EXACT];
    stats->logged = (int64_t)cnt_h[C_LOGGED];
    stats->sort_items = C.A.nt + C.B.nt;
    const SortKey K = sort_key(C.P.max_row);
    stats->sort_item_bytes = K.scatter_bytes();
    stats->sort_passes = K.passes;
    stats->tile = C.P.tk;
    stats->queue_passes = C.passes;
    stats->queue_skew = (int64_t)cnt_h[C_SKEW];
    stats->tiles_copied = (int64_t)cnt_h[C_COPIED];
}

sd3_status device_error(sd3_ctx *ctx, const HipError &e) {
    (void)hipGetLastError();
    if (e.e == hipErrorOutOfMemory) return fail(ctx, SD3_E_NOMEM, std::string(e.what) + ": out of device memory");
    return fail(ctx, SD3_E_DEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
}

// Solid semantics after the surface results are in: point-in-solid queries
// for both sides of every row (rows already meeting return at once), again
// with the next ray direction for those whose direction was degenerate, then
// the rows whose solids meet get distance 0 and hit 1.  Host buffers: the
// context's pinned staging (the static scratch's for allocation-free calls).
void solid_pass(sd3_ctx *ctx, Workspace &ws, Call &C, hipStream_t s, char *host, size_t host_cap) {
    const int64_t G = C.P.G, nq = 2 * G;
    if (G == 0) return;
    uint8_t *res = (uint8_t *)ws.buf(ws.solid, (size_t)nq * 6 + 64);
    uint8_t *dir = res + nq;
    int32_t *queries = (int32_t *)(((uintptr_t)(dir + nq) + 3) & ~(uintptr_t)3);
    if (ws.arena_full) throw ScratchFull{ws.arena_used};
    if ((size_t)nq * 6 + 64 > host_cap) throw HipError{hipErrorOutOfMemory, "solid staging"};
    int32_t *hq = (int32_t *)host;
    uint8_t *hdir = (uint8_t *)(hq + nq);
    uint8_t *hres = hdir + nq;
    for (int64_t i = 0; i < nq; i++) {
        hq[i] = (int32_t)i;
        hdir[i] = 0;
    }
    const SolidSide A{C.A.xyz, C.A.tri, C.A.v_off, C.A.t_off};
    const SolidSide B{C.B.xyz, C.B.tri, C.B.v_off, C.B.t_off};
    int64_t n = nq;
    for (int round = 0; round < SOLID_DIRS && n > 0; round++) {
        check(hipMemcpyAsync(dir, hdir, nq, hipMemcpyHostToDevice, s), "H2D directions");
        check(hipMemcpyAsync(queries, hq, sizeof(int32_t) * n, hipMemcpyHostToDevice, s), "H2D queries");
        launch_inside(A, B, C.rows, queries, n, dir, res, ctx->cus * 4, s);
        check(hipMemcpyAsync(hres, res, nq, hipMemcpyDeviceToHost, s), "D2H inside");
        check(hipStreamSynchronize(s), "sync");
        int64_t m = 0;
        for (int64_t k = 0; k < n; k++) {
            const int32_t code = hq[k];
            if (hres[code] & 2) {
                hdir[code]++;
                hq[m++] = code;
            }
        }
        n = m;
    }
    if (n > 0) throw HipError{hipErrorUnknown, "no generic ray direction for a point-in-solid query"};
    launch_solid_apply(res, G, C.dd, C.hd, C.rows, C.L, C.flags, s);
}

// What a finished call's scalars say about its work lists.
enum Overflow { OVF_NONE = 0, OVF_RESCUE = 1, OVF_EXACT = 2, OVF_OTHER = 3 };
Overflow overflow_kind(const Call &C, const unsigned int *sc_h, const unsigned long long *cnt_h) {
    if (sc_h[0] > C.L.qcap || cnt_h[C_QUEUE_OVF] != 0) return OVF_OTHER;
    if (sc_h[2] > C.L.rcap) return OVF_RESCUE;
    if (sc_h[4] > C.L.xcap) return OVF_EXACT;
    return OVF_NONE;
}

// One call on workspace `ws` (the context's own, or its static scratch).
// When a work list overflows, the call is computed again instead of failing:
// a full rescue list (FP32 pairs the bounds did not settle) by the plain FP64
// pass, which needs no rescue list and gives the same bits; a full exact list
// with a list four times longer (up to the workspace's limit).  `depth`
// counts those re-runs.
sd3_status run(sd3_ctx *ctx, Workspace &ws, const sd3_geoms *a, const sd3_geoms *b, double *dist,
               uint8_t *hit, const sd3_opts *opts_in, sd3_stats *stats, void *stream, int mode,
               int depth = 0) {
    auto t0 = std::chrono::steady_clock::now();
    if (!ctx) return SD3_E_INVALID_ARG;
    ctx->err.clear();
    sd3_opts opts;
    sd3_status st = check_call(ctx, a, b, dist, hit, opts_in, mode, opts);
    if (st != SD3_OK) return st;
    const bool stat = ws.arena != nullptr;
    const int tk = choose_tile(ctx, opts, mode, a, b);
    hipStream_t s = (hipStream_t)stream;
    Overflow ovf = OVF_NONE;
    int64_t xcap_used = 0;
    try {
        check(hipSetDevice(ctx->device), "hipSetDevice");
        PhaseClock clk{ctx, s, opts.timing != 0};
        clk.mark(0);
        Call C;
        if (stat) {
            ws.arena_used = 0;
            ws.arena_full = false;
        }
        plan_call(ctx, ws, a, b, opts, mode, tk, dist, hit, C, s);
        char *rb = readback_area(ctx);
        const unsigned int *sc_h = (const unsigned int *)rb;
        const unsigned long long *cnt_h = (const unsigned long long *)(rb + 64);
        alignas(16) char rbcopy[SCALAR_BYTES];
        // device inputs are validated by the call's kernels (coordinates
        // first, indices by the key kernel); the flags are read with the
        // counters at the end, and a flagged call writes no result
        enqueue_validate(C, s, false);
        clk.mark(1);
        KernelEvents *kev = nullptr;
        if (opts.timing) {
            if (!ctx->kev) {
                ctx->kev = new KernelEvents();
                for (auto &row : ctx->kev->ev)
                    for (auto &e : row) check(hipEventCreate(&e), "hipEventCreate");
            }
            kev = ctx->kev;
            for (int c = 0; c < KE_CLASSES; c++) kev->n[c] = 0;
        }
        enqueue_pipeline(ctx, C, s, &clk, kev);
        if (a->mem == SD3_MEM_DEVICE) clk.mark(7);
        // scalars and counters: an error leaves the outputs untouched (the
        // final kernel did not write them)
        check(hipMemcpyAsync(rb, C.sc, SCALAR_BYTES, hipMemcpyDeviceToHost, s), "D2H counters");
        check(hipStreamSynchronize(s), "sync");
        check(hipGetLastError(), "kernel launch");
        st = flags_status(ctx, sc_h);
        if (st != SD3_OK) return st;
        ovf = overflow_kind(C, sc_h, cnt_h);
        xcap_used = C.L.xcap;
        if (ovf == OVF_NONE && opts.semantics == SD3_SOLID) {
            // the staging below may move the pinned buffer the scalars were
            // read into: keep a copy of them
            memcpy(rbcopy, rb, SCALAR_BYTES);
            sc_h = (const unsigned int *)rbcopy;
            cnt_h = (const unsigned long long *)(rbcopy + 64);
            const size_t hb = (size_t)C.P.G * 12 + 64;
            solid_pass(ctx, ws, C, s, staging(ctx, ws, hb), hb);
            check(hipGetLastError(), "kernel launch");
        }
        if (ovf == OVF_NONE) {
            const int64_t G = C.P.G;
            if (a->mem == SD3_MEM_HOST && G > 0) {
                if (dist) check(hipMemcpyAsync(dist, C.dd, sizeof(double) * G, hipMemcpyDeviceToHost, s), "D2H dist");
                if (hit) check(hipMemcpyAsync(hit, C.hd, G, hipMemcpyDeviceToHost, s), "D2H hit");
                clk.mark(7);
                check(hipStreamSynchronize(s), "sync");
            } else if (a->mem == SD3_MEM_HOST) {
                clk.mark(7);
                check(hipStreamSynchronize(s), "sync");
            }
            if (stats) {
                fill_counts(C, sc_h, cnt_h, stats);
                stats->fallback = depth;
                stats->ms_total =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                clk.read(stats->ms_phase);
                if (kev)
                    for (int c = 0; c < KE_CLASSES; c++) {
                        double ms = 0.0;
                        for (int i = 0; i < std::min(kev->n[c], 16); i++) {
                            float f = 0.0f;
                            check(hipEventElapsedTime(&f, kev->ev[c][2 * i], kev->ev[c][2 * i + 1]), "elapsed");
                            ms += f;
                        }
                        stats->ms_kernel[c] = ms;
                        stats->n_kernel[c] = std::min(kev->n[c], 16);
                    }
            }
            return SD3_OK;
        }
    } catch (const HipError &e) {
        return device_error(ctx, e);
    } catch (const ScratchFull &f) {
        return fail(ctx, SD3_E_CAPACITY, "the call needs at least " + std::to_string(f.need) +
                                             " bytes of static scratch; the limit is " +
                                             std::to_string(ws.arena_cap));
    } catch (const std::bad_alloc &) {
        return fail(ctx, SD3_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ctx, SD3_E_DEVICE, "unexpected error");
    }
    // a work list overflowed: compute the call again (the outputs are untouched)
    sd3_opts again = opts;
    if (ovf == OVF_RESCUE && opts.precision == SD3_PREC_FP32_RESCUE && depth < 4) {
        again.precision = SD3_PREC_FP64;
        again.tile = tk;
        return run(ctx, ws, a, b, dist, hit, &again, stats, stream, mode, depth + 1);
    }
    const int64_t xmax = stat ? (int64_t)NOALLOC_EXACT : (int64_t)EXACT_CAP_MAX;
    if (ovf == OVF_EXACT && xcap_used < xmax && depth < 8) {
        again.exact_cap = std::min<int64_t>(xcap_used * 4, xmax);
        again.tile = tk;
        return run(ctx, ws, a, b, dist, hit, &again, stats, stream, mode, depth + 1);
    }
    return fail(ctx, SD3_E_CAPACITY, ovf == OVF_RESCUE  ? "rescue list overflow"
                                     : ovf == OVF_EXACT ? "exact list overflow"
                                                        : "tile-pair queue overflow");
}

}  // namespace

struct sd3_graph {
    sd3_ctx *ctx = nullptr;
    Workspace ws;
    Call C;
    hipStream_t cs = nullptr;  // capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *pin = nullptr;  // pinned readback of scalars and counters
};

namespace {

MlpScratch mlp_scratch(sd3_ctx *ctx, int64_t n) {
    int64_t m = n > 0 ? n : 1;
    float *b = (float *)ensure(ctx->mlp, sizeof(float) * (6 * MLP_H + 2) * m);
    MlpScratch s;
    s.h1 = b;
    s.h2 = b + MLP_H * m;
    s.h3 = b + 2 * MLP_H * m;
    s.d1 = b + 3 * MLP_H * m;
    s.d2 = b + 4 * MLP_H * m;
    s.d3 = b + 5 * MLP_H * m;
    s.y = b + 6 * MLP_H * m;
    s.dy = s.y + m;
    return s;
}

template <typename F>
sd3_status guarded(sd3_ctx *ctx, F f) {
    try {
        check(hipSetDevice(ctx->device), "hipSetDevice");
        f();
        check(hipGetLastError(), "kernel launch");
    } catch (const HipError &e) {
        (void)hipGetLastError();
        if (e.e == hipErrorOutOfMemory) return fail(ctx, SD3_E_NOMEM, "out of device memory");
        return fail(ctx, SD3_E_DEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
    } catch (...) {
        return fail(ctx, SD3_E_DEVICE, "unexpected error");
    }
    return SD3_OK;
}

}  // namespace

extern "C" {

void sd3_default_opts(sd3_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->precision = SD3_PREC_FP32_RESCUE;
    o->order = SD3_ORDER_BOUND;
}

sd3_status sd3_create(sd3_ctx **out, int device) {
    if (!out) return SD3_E_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return SD3_E_NO_DEVICE;
    }
    if (device < 0 || device >= n) return SD3_E_NO_DEVICE;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return SD3_E_DEVICE;
    if (strncmp(p.gcnArchName, "gfx950", 6) != 0) return SD3_E_NO_DEVICE;
    // set-up of allocation-free calls: the device's copy of `scratch` and
    // pinned staging for their offsets
    void *sp = nullptr;
    if (scratch_on_device(device, &sp) != hipSuccess) {
        (void)hipGetLastError();
        return SD3_E_DEVICE;
    }
    sd3_ctx *c = new (std::nothrow) sd3_ctx();
    if (!c) return SD3_E_NOMEM;
    c->device = device;
    c->cus = p.multiProcessorCount;
    c->sws.arena = (char *)sp;
    c->sws.arena_cap = NOALLOC_SCRATCH_BYTES;
    c->sws.queue_budget = NOALLOC_QUEUE;
    c->sws.rescue_cap = NOALLOC_RESCUE;
    c->sws.exact_cap = NOALLOC_EXACT;
    try {
        ensure_pinned(c, NOALLOC_HOST_BYTES);
        check(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking), "hipStreamCreate");
        for (hipEvent_t &e : c->fork) check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    } catch (const HipError &) {
        (void)hipGetLastError();
        for (hipEvent_t &e : c->fork)
            if (e) (void)hipEventDestroy(e);
        if (c->side) (void)hipStreamDestroy(c->side);
        if (c->pin) (void)hipHostFree(c->pin);
        delete c;
        return SD3_E_NOMEM;
    }
    *out = c;
    return SD3_OK;
}

sd3_status sd3_destroy(sd3_ctx *ctx) {
    if (!ctx) return SD3_OK;
    (void)hipSetDevice(ctx->device);
    ctx->ws.release_all();
    release(ctx->mlp);
    for (hipEvent_t &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t &e : ctx->fork)
        if (e) (void)hipEventDestroy(e);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->pin) (void)hipHostFree(ctx->pin);
    if (ctx->kev) {
        for (auto &row : ctx->kev->ev)
            for (auto &e : row)
                if (e) (void)hipEventDestroy(e);
        delete ctx->kev;
    }
    delete ctx;
    return SD3_OK;
}

sd3_status sd3_distance(sd3_ctx *ctx, const sd3_geoms *a, const sd3_geoms *b, double *dist,
                        uint8_t *hit, const sd3_opts *opts, sd3_stats *stats, void *stream) {
    return ctx ? run(ctx, ctx->ws, a, b, dist, hit, opts, stats, stream, 0) : SD3_E_INVALID_ARG;
}

sd3_status sd3_distance_noalloc(sd3_ctx *ctx, const sd3_geoms *a, const sd3_geoms *b, double *dist,
                                uint8_t *hit, const sd3_opts *opts, sd3_stats *stats, void *stream) {
    if (!ctx) return SD3_E_INVALID_ARG;
    ctx->err.clear();
    if (opts && opts->timing)
        return fail(ctx, SD3_E_INVALID_ARG, "timing is not available without allocation (it needs HIP events)");
    if (a && b && (a->count > NOALLOC_MAX_ROWS || b->count > NOALLOC_MAX_ROWS))
        return fail(ctx, SD3_E_CAPACITY, "allocation-free calls take at most " +
                                             std::to_string(NOALLOC_MAX_ROWS) + " rows");
    return run(ctx, ctx->sws, a, b, dist, hit, opts, stats, stream, 0);
}

sd3_status sd3_intersects(sd3_ctx *ctx, const sd3_geoms *a, const sd3_geoms *b, uint8_t *hit,
                          const sd3_opts *opts, sd3_stats *stats, void *stream) {
    return ctx ? run(ctx, ctx->ws, a, b, nullptr, hit, opts, stats, stream, 1) : SD3_E_INVALID_ARG;
}

sd3_status sd3_segments(sd3_ctx *ctx, int32_t op, const double *seg, int64_t n, int32_t seg_mem,
                        const sd3_geoms *mesh, double r, double *dist, uint8_t *flag, sd3_stats *stats,
                        void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (!ctx) return SD3_E_INVALID_ARG;
    ctx->err.clear();
    std::string msg;
    sd3_status st = check_geoms(mesh, msg);
    if (st != SD3_OK) return fail(ctx, st, msg);
    if (mesh->count != 1) return fail(ctx, SD3_E_INVALID_ARG, "the mesh must be a batch of one row");
    if (op != SD3_SEG_DISTANCE && op != SD3_SEG_INTERSECTS && op != SD3_SEG_WITHIN)
        return fail(ctx, SD3_E_INVALID_ARG, "unknown segment operator");
    if (n < 0 || (n > 0 && !seg)) return fail(ctx, SD3_E_INVALID_ARG, "segments are NULL or n < 0");
    if (seg_mem != mesh->mem) return fail(ctx, SD3_E_INVALID_ARG, "segments and mesh differ in memory kind");
    if ((op == SD3_SEG_DISTANCE && !dist) || (op != SD3_SEG_DISTANCE && !flag))
        return fail(ctx, SD3_E_INVALID_ARG, "output pointer is NULL");
    if (op == SD3_SEG_WITHIN && !(r >= 0.0 && r <= 1.7976931348623157e308))
        return fail(ctx, SD3_E_INVALID_ARG, "r must be finite and >= 0");
    const int64_t nv = mesh->v_off[1], nt = mesh->t_off[1];
    if (nt >= ((int64_t)1 << 25)) return fail(ctx, SD3_E_INVALID_ARG, "mesh too large (at most 2^25 - 1 triangles)");
    if (seg_mem == SD3_MEM_HOST) {
        st = check_host_data(mesh, msg);
        if (st != SD3_OK) return fail(ctx, st, msg);
        for (int64_t i = 0; i < 6 * n; i++) {
            const double x = std::fabs(seg[i]);
            if (!(x <= 1.7976931348623157e308))
                return fail(ctx, SD3_E_NONFINITE, "non-finite coordinate in segment " + std::to_string(i / 6));
            if (x != 0.0 && (x < 0x1p-256 || x > 0x1p256))
                return fail(ctx, SD3_E_RANGE, "coordinate magnitude outside [2^-256, 2^256] in segment " +
                                                  std::to_string(i / 6));
        }
    }
    hipStream_t s = (hipStream_t)stream;
    Workspace &ws = ctx->ws;
    const int mode = op == SD3_SEG_DISTANCE ? 0 : (op == SD3_SEG_INTERSECTS ? 1 : 2);
    try {
        check(hipSetDevice(ctx->device), "hipSetDevice");
        const double *dseg = seg;
        const double *xyz = mesh->xyz;
        const int32_t *tri = mesh->tri;
        if (seg_mem == SD3_MEM_HOST) {
            char *in = (char *)ensure(ws.seg_in, sizeof(double) * (6 * n + 3 * nv) + sizeof(int32_t) * 3 * nt + 64);
            double *ds = (double *)in;
            double *dx = ds + 6 * n;
            int32_t *dt = (int32_t *)(dx + 3 * nv);
            if (n) check(hipMemcpyAsync(ds, seg, sizeof(double) * 6 * n, hipMemcpyHostToDevice, s), "H2D segments");
            if (nv) check(hipMemcpyAsync(dx, xyz, sizeof(double) * 3 * nv, hipMemcpyHostToDevice, s), "H2D mesh xyz");
            if (nt) check(hipMemcpyAsync(dt, tri, sizeof(int32_t) * 3 * nt, hipMemcpyHostToDevice, s), "H2D mesh tri");
            dseg = ds;
            xyz = dx;
            tri = dt;
        }
        const int64_t ntiles = (nt + SEG_MESH_TILE - 1) / SEG_MESH_TILE;
        double *P = (double *)ensure(ws.seg_mesh, sizeof(double) * (SEG_MESH_FIELDS * nt + 6 * ntiles + 6) + 64);
        double *tbox = P + SEG_MESH_FIELDS * nt;
        double *mbox = tbox + 6 * ntiles;
        unsigned int *sc = (unsigned int *)ensure(ws.scalars, SCALAR_BYTES);
        uint32_t *flags = (uint32_t *)sc;
        unsigned long long *cnt = (unsigned long long *)(sc + 16);
        double *odist = dist;
        uint8_t *oflag = flag;
        if (seg_mem == SD3_MEM_HOST) {
            char *o = (char *)ensure(ws.seg_out, (sizeof(double) + 1) * (n > 0 ? n : 1) + 64);
            odist = dist ? (double *)o : nullptr;
            oflag = flag ? (uint8_t *)(o + sizeof(double) * (n > 0 ? n : 1)) : nullptr;
        }
        launch_seg_validate(dseg, n, xyz, nv, tri, nt, flags, cnt, s);
        ensure_pinned(ctx, 0);
        char *rb = readback_area(ctx);
        if (seg_mem == SD3_MEM_DEVICE) {
            // device inputs are validated before any kernel reads them
            check(hipMemcpyAsync(rb, sc, 64, hipMemcpyDeviceToHost, s), "D2H flags");
            check(hipStreamSynchronize(s), "sync");
            const uint32_t f = ((const uint32_t *)rb)[0] | ((const uint32_t *)rb)[1];
            if (f & V_NONFINITE) return fail(ctx, SD3_E_NONFINITE, "non-finite coordinate");
            if (f & V_RANGE) return fail(ctx, SD3_E_RANGE, "coordinate magnitude outside [2^-256, 2^256]");
            if (f & V_INDEX) return fail(ctx, SD3_E_INDEX_RANGE, "triangle index outside the mesh");
        }
        launch_seg_mesh(xyz, nv, tri, nt, P, tbox, mbox, s);
        int &gp = ctx->seg_grid[mode];
        if (gp == 0) gp = ctx->cus * seg_blocks_per_cu(mode);
        launch_segs(mode, dseg, n, P, nt, tbox, mbox, r, mode == 0 ? odist : nullptr, oflag, flags, cnt, gp, s);
        check(hipGetLastError(), "kernel launch");
        check(hipMemcpyAsync(rb, sc, SCALAR_BYTES, hipMemcpyDeviceToHost, s), "D2H counters");
        if (seg_mem == SD3_MEM_HOST && n > 0) {
            if (dist) check(hipMemcpyAsync(dist, odist, sizeof(double) * n, hipMemcpyDeviceToHost, s), "D2H dist");
            if (flag) check(hipMemcpyAsync(flag, oflag, n, hipMemcpyDeviceToHost, s), "D2H flags");
        }
        check(hipStreamSynchronize(s), "sync");
        const unsigned long long *cnt_h = (const unsigned long long *)(rb + 64);
        if (stats) {
            memset(stats, 0, sizeof(*stats));
            stats->tile_pairs_total = ntiles * ((n + 63) / 64);
            stats->tri_pairs_boxed = (int64_t)cnt_h[0];
            stats->tri_pairs_fp64 = (int64_t)cnt_h[1];
            stats->exact = (int64_t)cnt_h[2];
            stats->tile = SEG_MESH_TILE;
            stats->ms_total =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
    } catch (const HipError &e) {
        return device_error(ctx, e);
    } catch (const std::bad_alloc &) {
        return fail(ctx, SD3_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ctx, SD3_E_DEVICE, "unexpected error");
    }
    return SD3_OK;
}

sd3_status sd3_volume(sd3_ctx *ctx, const sd3_geoms *g, double *vol, sd3_stats *stats, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (!ctx) return SD3_E_INVALID_ARG;
    ctx->err.clear();
    std::string msg;
    sd3_status st = check_geoms(g, msg);
    if (st != SD3_OK) return fail(ctx, st, msg);
    if (!vol) return fail(ctx, SD3_E_INVALID_ARG, "output pointer is NULL");
    if (g->mem == SD3_MEM_HOST) {
        st = check_host_data(g, msg);
        if (st != SD3_OK) return fail(ctx, st, msg);
    }
    const int64_t G = g->count, nv = g->v_off[G], nt = g->t_off[G];
    const int64_t CH = volume_chunk();
    hipStream_t s = (hipStream_t)stream;
    Workspace &ws = ctx->ws;
    try {
        check(hipSetDevice(ctx->device), "hipSetDevice");
        // work items: (row, chunk) with the rows' offsets, staged in one copy:
        // [v_off | t_off | item offsets (G+1) | first triangle of each item |
        //  row of each item (int32)]
        int64_t nitems = 0;
        for (int64_t r = 0; r < G; r++) nitems += (g->t_off[r + 1] - g->t_off[r] + CH - 1) / CH;
        const size_t bytes = sizeof(int64_t) * (3 * (G + 1) + nitems) + sizeof(int32_t) * (nitems + 1);
        char *hs = ensure_pinned(ctx, bytes);
        int64_t *h_voff = (int64_t *)hs, *h_toff = h_voff + (G + 1), *h_witem = h_toff + (G + 1);
        int64_t *h_wfirst = h_witem + (G + 1);
        int32_t *h_wrow = (int32_t *)(h_wfirst + nitems);
        memcpy(h_voff, g->v_off, sizeof(int64_t) * (G + 1));
        memcpy(h_toff, g->t_off, sizeof(int64_t) * (G + 1));
        int64_t it = 0;
        for (int64_t r = 0; r < G; r++) {
            h_witem[r] = it;
            for (int64_t t = g->t_off[r]; t < g->t_off[r + 1]; t += CH) {
                h_wfirst[it] = t;
                h_wrow[it] = (int32_t)r;
                it++;
            }
        }
        h_witem[G] = it;
        char *ds = (char *)ensure(ws.vol_items, bytes + 64);
        check(hipMemcpyAsync(ds, hs, bytes, hipMemcpyHostToDevice, s), "H2D volume items");
        const int64_t *d_voff = (const int64_t *)ds, *d_toff = d_voff + (G + 1), *d_witem = d_toff + (G + 1);
        const int64_t *d_wfirst = d_witem + (G + 1);
        const int32_t *d_wrow = (const int32_t *)(d_wfirst + nitems);
        const double *xyz = g->xyz;
        const int32_t *tri = g->tri;
        if (g->mem == SD3_MEM_HOST) {
            SideState &sd = ws.side[0];
            double *x = (double *)ensure(sd.xyz, sizeof(double) * 3 * nv);
            int32_t *t = (int32_t *)ensure(sd.tri, sizeof(int32_t) * 3 * nt);
            // (a static scratch already too small stops before any copy)
        if (ws.arena_full) throw ScratchFull{ws.arena_used};
        if (nv) check(hipMemcpyAsync(x, g->xyz, sizeof(double) * 3 * nv, hipMemcpyHostToDevice, s), "H2D xyz");
            if (nt) check(hipMemcpyAsync(t, g->tri, sizeof(int32_t) * 3 * nt, hipMemcpyHostToDevice, s), "H2D tri");
            xyz = x;
            tri = t;
        }
        void *part = ensure(ws.vol_part, 16 * (size_t)(nitems > 0 ? nitems : 1) + sizeof(double) * (G > 0 ? G : 1));
        double *dvol = g->mem == SD3_MEM_HOST ? (double *)((char *)part + 16 * (size_t)(nitems > 0 ? nitems : 1))
                                              : vol;
        unsigned int *sc = (unsigned int *)ensure(ws.scalars, SCALAR_BYTES);
        launch_volume(xyz, nv, tri, d_voff, d_toff, d_wrow, d_wfirst, nitems, d_witem, G, part, dvol,
                      (uint32_t *)sc, ctx->cus * 8, s);
        check(hipGetLastError(), "kernel launch");
        char *rb = readback_area(ctx);
        check(hipMemcpyAsync(rb, sc, 4, hipMemcpyDeviceToHost, s), "D2H flags");
        check(hipStreamSynchronize(s), "sync");
        const uint32_t f = *(const uint32_t *)rb;
        if (f & V_NONFINITE) return fail(ctx, SD3_E_NONFINITE, "non-finite coordinate");
        if (f & V_RANGE) return fail(ctx, SD3_E_RANGE, "coordinate magnitude outside [2^-256, 2^256]");
        if (f & V_INDEX) return fail(ctx, SD3_E_INDEX_RANGE, "triangle index outside its row");
        if (g->mem == SD3_MEM_HOST && G > 0) {
            check(hipMemcpyAsync(vol, dvol, sizeof(double) * G, hipMemcpyDeviceToHost, s), "D2H volume");
            check(hipStreamSynchronize(s), "sync");
        }
        if (stats) {
            memset(stats, 0, sizeof(*stats));
            stats->sort_items = nt;
            stats->ms_total =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
    } catch (const HipError &e) {
        return device_error(ctx, e);
    } catch (const std::bad_alloc &) {
        return fail(ctx, SD3_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ctx, SD3_E_DEVICE, "unexpected error");
    }
    return SD3_OK;
}

sd3_status sd3_graph_create(sd3_ctx *ctx, int32_t kind, const sd3_geoms *a, const sd3_geoms *b,
                            double *dist, uint8_t *hit, const sd3_opts *opts_in, sd3_graph **out) {
    if (!ctx || !out) return SD3_E_INVALID_ARG;
    *out = nullptr;
    ctx->err.clear();
    if (kind != SD3_KIND_DISTANCE && kind != SD3_KIND_INTERSECTS)
        return fail(ctx, SD3_E_INVALID_ARG, "unknown kind");
    const int mode = kind == SD3_KIND_DISTANCE ? 0 : 1;
    if (mode == 1) dist = nullptr;
    sd3_opts opts;
    sd3_status st = check_call(ctx, a, b, dist, hit, opts_in, mode, opts);
    if (st != SD3_OK) return st;
    if (a->mem != SD3_MEM_DEVICE) return fail(ctx, SD3_E_INVALID_ARG, "graphs need device-resident batches");
    if (opts.timing || opts.log) return fail(ctx, SD3_E_INVALID_ARG, "graphs support neither timing nor log");
    if (opts.semantics != SD3_SURFACE) return fail(ctx, SD3_E_INVALID_ARG, "graphs support surface semantics only");
    const int tk = choose_tile(ctx, opts, mode, a, b);
    sd3_graph *g = new (std::nothrow) sd3_graph();
    if (!g) return fail(ctx, SD3_E_NOMEM, "host allocation failed");
    g->ctx = ctx;
    bool capturing = false;
    try {
        check(hipSetDevice(ctx->device), "hipSetDevice");
        check(hipStreamCreateWithFlags(&g->cs, hipStreamNonBlocking), "hipStreamCreate");
        check(hipHostMalloc(&g->pin, SCALAR_BYTES, hipHostMallocDefault), "hipHostMalloc");
        plan_call(ctx, g->ws, a, b, opts, mode, tk, dist, hit, g->C, g->cs);
        // validate the current contents once, before anything reads them
        enqueue_validate(g->C, g->cs, true);
        check(hipMemcpyAsync(g->pin, g->C.sc, 64, hipMemcpyDeviceToHost, g->cs), "D2H flags");
        check(hipStreamSynchronize(g->cs), "sync");
        st = flags_status(ctx, (const unsigned int *)g->pin);
        if (st == SD3_OK) {
            check(hipStreamBeginCapture(g->cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            capturing = true;
            enqueue_validate(g->C, g->cs, false);
            enqueue_pipeline(ctx, g->C, g->cs, nullptr, nullptr);
            capturing = false;
            check(hipStreamEndCapture(g->cs, &g->graph), "hipStreamEndCapture");
            check(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        }
    } catch (const HipError &e) {
        if (capturing) {
            hipGraph_t dead = nullptr;
            (void)hipStreamEndCapture(g->cs, &dead);
            if (dead) (void)hipGraphDestroy(dead);
        }
        st = device_error(ctx, e);
    } catch (const std::bad_alloc &) {
        st = fail(ctx, SD3_E_NOMEM, "host allocation failed");
    } catch (...) {
        st = fail(ctx, SD3_E_DEVICE, "unexpected error");
    }
    if (st != SD3_OK) {
        std::string keep = ctx->err;
        sd3_graph_destroy(g);
        ctx->err = keep;
        return st;
    }
    *out = g;
    return SD3_OK;
}

sd3_status sd3_graph_launch(sd3_graph *g, void *stream) {
    if (!g || !g->exec) return SD3_E_INVALID_ARG;
    sd3_ctx *ctx = g->ctx;
    try {
        check(hipSetDevice(ctx->device), "hipSetDevice");
        check(hipGraphLaunch(g->exec, (hipStream_t)stream), "hipGraphLaunch");
    } catch (const HipError &e) {
        return device_error(ctx, e);
    }
    return SD3_OK;
}

sd3_status sd3_graph_result(sd3_graph *g, sd3_stats *stats, void *stream) {
    if (!g || !g->exec) return SD3_E_INVALID_ARG;
    sd3_ctx *ctx = g->ctx;
    ctx->err.clear();
    const unsigned int *sc_h = (const unsigned int *)g->pin;
    const unsigned long long *cnt_h = (const unsigned long long *)((char *)g->pin + 64);
    try {
        check(hipSetDevice(ctx->device), "hipSetDevice");
        hipStream_t s = (hipStream_t)stream;
        check(hipMemcpyAsync(g->pin, g->C.sc, SCALAR_BYTES, hipMemcpyDeviceToHost, s), "D2H counters");
        check(hipStreamSynchronize(s), "sync");
    } catch (const HipError &e) {
        return device_error(ctx, e);
    }
    sd3_status st = call_status(ctx, g->C, sc_h, cnt_h);
    if (st != SD3_OK) return st;
    if (stats) fill_counts(g->C, sc_h, cnt_h, stats);
    return SD3_OK;
}

sd3_status sd3_graph_destroy(sd3_graph *g) {
    if (!g) return SD3_OK;
    (void)hipSetDevice(g->ctx->device);
    if (g->cs) (void)hipStreamSynchronize(g->cs);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->cs) (void)hipStreamDestroy(g->cs);
    if (g->pin) (void)hipHostFree(g->pin);
    g->ws.release_all();
    delete g;
    return SD3_OK;
}

sd3_status sd3_autotune(sd3_ctx *ctx, int32_t kind, const sd3_geoms *a, const sd3_geoms *b,
                        const sd3_opts *opts_in, int32_t reps, sd3_tune_report *report,
                        void *stream) {
    if (!ctx) return SD3_E_INVALID_ARG;
    ctx->err.clear();
    if (kind != SD3_KIND_DISTANCE && kind != SD3_KIND_INTERSECTS)
        return fail(ctx, SD3_E_INVALID_ARG, "unknown kind");
    if (reps < 1) return fail(ctx, SD3_E_INVALID_ARG, "reps < 1");
    const int mode = kind == SD3_KIND_DISTANCE ? 0 : 1;
    sd3_opts opts;
    sd3_default_opts(&opts);
    if (opts_in) opts = *opts_in;
    opts.timing = 0;
    opts.log = nullptr;
    std::string msg;
    sd3_status st = check_geoms(a, msg);
    if (st == SD3_OK) st = check_geoms(b, msg);
    if (st != SD3_OK) return fail(ctx, st, msg);
    if (a->count != b->count) return fail(ctx, SD3_E_INVALID_ARG, "batches differ in count");
    const int64_t G = a->count;
    // scratch outputs of the tuning calls
    std::vector<double> hd_dist;
    std::vector<uint8_t> hd_hit;
    double *dist = nullptr;
    uint8_t *hit = nullptr;
    DevBuf dev_out;
    try {
        if (a->mem == SD3_MEM_DEVICE) {
            check(hipSetDevice(ctx->device), "hipSetDevice");
            char *o = (char *)ensure(dev_out, (sizeof(double) + 1) * (G > 0 ? G : 1));
            dist = (double *)o;
            hit = (uint8_t *)(o + sizeof(double) * (G > 0 ? G : 1));
        } else {
            hd_dist.resize(G > 0 ? G : 1);
            hd_hit.resize(G > 0 ? G : 1);
            dist = hd_dist.data();
            hit = hd_hit.data();
        }
    } catch (const HipError &e) {
        return device_error(ctx, e);
    }
    const int cand[3] = {32, 64, 128};
    sd3_tune_report rep{};
    // one untimed call per size, then `reps` rounds that time the sizes in
    // turn (drift of the clock or of the device affects every size alike)
    std::vector<double> ms[3];
    for (int r = 0; r <= reps && st == SD3_OK; r++) {
        for (int c = 0; c < 3 && st == SD3_OK; c++) {
            opts.tile = cand[c];
            auto t0 = std::chrono::steady_clock::now();
            st = run(ctx, ctx->ws, a, b, mode == 0 ? dist : nullptr, hit, &opts, nullptr, stream, mode);
            auto t1 = std::chrono::steady_clock::now();
            if (r > 0) ms[c].push_back(std::chrono::duration<double, std::milli>(t1 - t0).count());
        }
    }
    if (dev_out.p) release(dev_out);
    if (st != SD3_OK) return st;
    double best_ms = 0.0;
    for (int c = 0; c < 3; c++) {
        std::sort(ms[c].begin(), ms[c].end());
        rep.tile[c] = cand[c];
        rep.ms[c] = ms[c][ms[c].size() / 2];
        rep.n = c + 1;
        if (c == 0 || rep.ms[c] < best_ms) {
            best_ms = rep.ms[c];
            rep.best = cand[c];
        }
    }
    opts.tile = SD3_TILE_AUTO;
    ctx->tuned[workload_key(opts, mode, a, b)] = rep.best;
    if (report) *report = rep;
    return SD3_OK;
}

sd3_status sd3_mlp_forward(sd3_ctx *ctx, const float *params, const float *x, int64_t n, float *y,
                           void *stream) {
    if (!ctx) return SD3_E_INVALID_ARG;
    if (!params || n < 0 || (n > 0 && (!x || !y))) return fail(ctx, SD3_E_INVALID_ARG, "bad MLP arguments");
    return guarded(ctx, [&] {
        MlpScratch s = mlp_scratch(ctx, n);
        mlp_forward(params, x, n, s, y, (hipStream_t)stream);
    });
}

sd3_status sd3_mlp_score(sd3_ctx *ctx, const float *params, const float *x, int64_t n, float *y,
                         void *stream) {
    if (!ctx) return SD3_E_INVALID_ARG;
    if (!params || n < 0 || (n > 0 && (!x || !y))) return fail(ctx, SD3_E_INVALID_ARG, "bad MLP arguments");
    return guarded(ctx, [&] {
        const int64_t waves = (n + 3) / 4;
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(waves, (int64_t)ctx->cus * 2));
        launch_rank_score(params, x, n, y, grid, (hipStream_t)stream);
    });
}

sd3_status sd3_mlp_loss_grad(sd3_ctx *ctx, const float *params, const float *x, const float *t,
                             int64_t n, float *loss, float *grad, void *stream) {
    if (!ctx) return SD3_E_INVALID_ARG;
    if (!params || !loss || !grad || n < 0 || (n > 0 && (!x || !t)))
        return fail(ctx, SD3_E_INVALID_ARG, "bad MLP arguments");
    return guarded(ctx, [&] {
        MlpScratch s = mlp_scratch(ctx, n);
        mlp_loss_grad(params, x, t, n, s, loss, grad, (hipStream_t)stream);
    });
}

sd3_status sd3_adam_step(sd3_ctx *ctx, float *p, const float *g, float *m, float *v, int64_t count,
                         int32_t step, float lr, float beta1, float beta2, float eps, void *stream) {
    if (!ctx) return SD3_E_INVALID_ARG;
    if (!p || !g || !m || !v || count < 0 || step < 1)
        return fail(ctx, SD3_E_INVALID_ARG, "bad Adam arguments");
    return guarded(ctx, [&] { adam_step(p, g, m, v, count, step, lr, beta1, beta2, eps, (hipStream_t)stream); });
}

sd3_status sd3_validate(const sd3_geoms *g) {
    std::string msg;
    sd3_status s = check_geoms(g, msg);
    if (s != SD3_OK) return s;
    if (g->mem != SD3_MEM_HOST) return SD3_E_INVALID_ARG;
    return check_host_data(g, msg);
}

const char *sd3_status_string(sd3_status s) {
    switch (s) {
        case SD3_OK: return "ok";
        case SD3_E_INVALID_ARG: return "invalid argument";
        case SD3_E_INDEX_RANGE: return "triangle index out of range";
        case SD3_E_NONFINITE: return "non-finite coordinate";
        case SD3_E_RANGE: return "coordinate magnitude outside [2^-256, 2^256]";
        case SD3_E_NOMEM: return "out of memory";
        case SD3_E_DEVICE: return "device error";
        case SD3_E_NO_DEVICE: return "no gfx950 device";
        case SD3_E_CAPACITY: return "internal work list overflow";
    }
    return "unknown status";
}

const char *sd3_last_error(const sd3_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

}  // extern "C"
