// sd3 C-ABI: argument checks, device buffers and the pipeline of one call.
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/sd3.h"
#include "sd3_kernels.h"
#include "sd3_mlp.h"

using namespace sd3;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

struct SideState {
    DevBuf xyz, tri, v_off, t_off, tile_off, rowbox, t32, t64, meta;
};

struct Plan {
    int64_t G = 0;
    std::vector<int64_t> tileA, tileB;  // [G+1] tile offsets
    std::vector<int64_t> wi;            // [G+1] work-item offsets
    std::vector<int64_t> blkA, chkB;    // [G+1] A-block (64 tiles) / B-chunk (256 tiles) offsets
    int64_t potential = 0;              // sum of tilesA * tilesB
};

}  // namespace

struct sd3_ctx {
    int device = 0;
    int cus = 0;
    std::string err;
    SideState side[2];
    DevBuf rows, wi_off, queue, qlb, rescue, exact, counters, scalars, flags, out_d, out_h;
    DevBuf keys0, keys1, vals0, vals1, hist, part, small, grpA, grpB, wi_lb, seedq, seedlb;
    DevBuf mlp;    // ranker training scratch
    DevBuf wlist;  // compacted work items
    void *pin = nullptr;  // pinned host staging: offsets up, counters down
    size_t pin_cap = 0;
    int pairs_grid[2][2] = {{0, 0}, {0, 0}};
    hipEvent_t ev[8] = {};
    KernelEvents *kev = nullptr;  // created on the first timed call
};

namespace {

constexpr unsigned int QUEUE_BUDGET = 1u << 27;   // tile pairs per queue pass
constexpr unsigned int RESCUE_CAP = 1u << 24;     // FP32 pairs sent to FP64
constexpr unsigned int EXACT_CAP = 1u << 22;      // pairs sent to exact arithmetic

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

void release(DevBuf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
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

int64_t tiles_of(int64_t nt) { return (nt + K - 1) / K; }

// Upload (host inputs) or reference (device inputs) one side and size its
// buffers.  Offsets were staged already.  No kernel reads the data before it
// has been validated.
void setup_side(sd3_ctx *ctx, int which, const sd3_geoms *g, int64_t NT, const int64_t *d_offs,
                SideBufs &S, hipStream_t s) {
    SideState &st = ctx->side[which];
    int64_t G = g->count, nv = g->v_off[G], nt = g->t_off[G];
    S.G = G;
    S.nv = nv;
    S.nt = nt;
    S.NT = NT;
    if (g->mem == SD3_MEM_HOST) {
        double *x = (double *)ensure(st.xyz, sizeof(double) * 3 * nv);
        int32_t *t = (int32_t *)ensure(st.tri, sizeof(int32_t) * 3 * nt);
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
    S.rowbox = (unsigned long long *)ensure(st.rowbox, sizeof(unsigned long long) * 6 * (G > 0 ? G : 1));
    S.t32 = (float *)ensure(st.t32, sizeof(float) * 9 * K * S.NT);
    S.t64 = (double *)ensure(st.t64, sizeof(double) * 9 * K * S.NT);
    S.meta = (TileMeta *)ensure(st.meta, sizeof(TileMeta) * S.NT);
}

// Morton key bits: 30 for the code plus enough to keep rows apart.
int key_bits(int64_t G) {
    int rowbits = 0;
    while (((int64_t)1 << rowbits) < G) rowbits++;
    return 30 + rowbits;
}

// Validate device-resident data on the device (one synchronisation).
sd3_status validate_device(sd3_ctx *ctx, const sd3_geoms *a, const SideBufs &A,
                           const sd3_geoms *b, const SideBufs &B, hipStream_t s) {
    uint32_t *flags = (uint32_t *)ensure(ctx->flags, 256);
    check(hipMemsetAsync(flags, 0, 2 * sizeof(uint32_t), s), "memset flags");
    launch_validate(a->xyz, A.nv, a->tri, A.nt, A.v_off, A.t_off, A.G, flags, s);
    launch_validate(b->xyz, B.nv, b->tri, B.nt, B.v_off, B.t_off, B.G, flags + 1, s);
    uint32_t *h = (uint32_t *)readback_area(ctx);
    check(hipMemcpyAsync(h, flags, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s), "D2H flags");
    check(hipStreamSynchronize(s), "sync");
    uint32_t f = h[0] | h[1];
    if (f & V_NONFINITE) return fail(ctx, SD3_E_NONFINITE, "non-finite coordinate");
    if (f & V_RANGE) return fail(ctx, SD3_E_RANGE, "coordinate magnitude outside [2^-256, 2^256]");
    if (f & V_INDEX) return fail(ctx, SD3_E_INDEX_RANGE, "triangle index outside its row");
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

sd3_status run(sd3_ctx *ctx, const sd3_geoms *a, const sd3_geoms *b, double *dist, uint8_t *hit,
               const sd3_opts *opts_in, sd3_stats *stats, void *stream, int mode) {
    auto t0 = std::chrono::steady_clock::now();
    if (!ctx) return SD3_E_INVALID_ARG;
    ctx->err.clear();
    std::string msg;
    sd3_status st = check_geoms(a, msg);
    if (st == SD3_OK) st = check_geoms(b, msg);
    if (st != SD3_OK) return fail(ctx, st, msg);
    if (a->count != b->count) return fail(ctx, SD3_E_INVALID_ARG, "batches differ in count");
    if (a->mem != b->mem) return fail(ctx, SD3_E_INVALID_ARG, "batches differ in memory kind");
    if ((mode == 0 && !dist) || (mode == 1 && !hit))
        return fail(ctx, SD3_E_INVALID_ARG, "output pointer is NULL");
    sd3_opts opts;
    sd3_default_opts(&opts);
    if (opts_in) opts = *opts_in;
    if (opts.precision != SD3_PREC_FP32_RESCUE && opts.precision != SD3_PREC_FP64)
        return fail(ctx, SD3_E_INVALID_ARG, "unknown precision");
    if (opts.order != SD3_ORDER_BOUND && opts.order != SD3_ORDER_NONE &&
        opts.order != SD3_ORDER_LEARNED)
        return fail(ctx, SD3_E_INVALID_ARG, "unknown order");
    if (opts.order == SD3_ORDER_LEARNED && !opts.ranker)
        return fail(ctx, SD3_E_INVALID_ARG, "SD3_ORDER_LEARNED needs opts.ranker");
    if (opts.log && (opts.log_cap < 0 || a->mem != SD3_MEM_DEVICE))
        return fail(ctx, SD3_E_INVALID_ARG, "log needs a device buffer and log_cap >= 0");
    if (a->mem == SD3_MEM_HOST) {
        st = check_host_data(a, msg);
        if (st == SD3_OK) st = check_host_data(b, msg);
        if (st != SD3_OK) return fail(ctx, st, msg);
    }
    const int64_t G = a->count;
    hipStream_t s = (hipStream_t)stream;
    try {
        check(hipSetDevice(ctx->device), "hipSetDevice");
        // plan: tiles per row and queue work items
        Plan P;
        P.G = G;
        P.tileA.assign(G + 1, 0);
        P.tileB.assign(G + 1, 0);
        P.wi.assign(G + 1, 0);
        P.blkA.assign(G + 1, 0);
        P.chkB.assign(G + 1, 0);
        for (int64_t g = 0; g < G; g++) {
            int64_t na = tiles_of(a->t_off[g + 1] - a->t_off[g]);
            int64_t nb = tiles_of(b->t_off[g + 1] - b->t_off[g]);
            P.tileA[g + 1] = P.tileA[g] + na;
            P.tileB[g + 1] = P.tileB[g] + nb;
            P.blkA[g + 1] = P.blkA[g] + (na + 63) / 64;
            P.chkB[g + 1] = P.chkB[g] + (nb + 255) / 256;
            // a row with an empty side has no work items
            P.wi[g + 1] = P.wi[g] + (na > 0 && nb > 0 ? ((na + 63) / 64) * ((nb + 255) / 256) : 0);
            P.potential += na * nb;
        }
        PhaseClock clk{ctx, s, opts.timing != 0};
        clk.mark(0);
        // all offsets in one pinned staging copy: [A v_off | A t_off | A tiles |
        // B v_off | B t_off | B tiles | work items | A blocks | B chunks]
        const int64_t G1 = G + 1;
        int64_t *hs = (int64_t *)ensure_pinned(ctx, sizeof(int64_t) * 9 * G1);
        memcpy(hs, a->v_off, sizeof(int64_t) * G1);
        memcpy(hs + G1, a->t_off, sizeof(int64_t) * G1);
        memcpy(hs + 2 * G1, P.tileA.data(), sizeof(int64_t) * G1);
        memcpy(hs + 3 * G1, b->v_off, sizeof(int64_t) * G1);
        memcpy(hs + 4 * G1, b->t_off, sizeof(int64_t) * G1);
        memcpy(hs + 5 * G1, P.tileB.data(), sizeof(int64_t) * G1);
        memcpy(hs + 6 * G1, P.wi.data(), sizeof(int64_t) * G1);
        memcpy(hs + 7 * G1, P.blkA.data(), sizeof(int64_t) * G1);
        memcpy(hs + 8 * G1, P.chkB.data(), sizeof(int64_t) * G1);
        int64_t *ds = (int64_t *)ensure(ctx->small, sizeof(int64_t) * 9 * G1);
        check(hipMemcpyAsync(ds, hs, sizeof(int64_t) * 9 * G1, hipMemcpyHostToDevice, s), "H2D offsets");
        SideBufs A{}, B{};
        setup_side(ctx, 0, a, P.tileA[G], ds, A, s);
        setup_side(ctx, 1, b, P.tileB[G], ds + 3 * G1, B, s);
        if (a->mem == SD3_MEM_DEVICE) {
            st = validate_device(ctx, a, A, b, B, s);
            if (st != SD3_OK) return st;
        }
        clk.mark(1);
        PrepBufs PB{};
        {
            int64_t n = A.nt + B.nt;
            int64_t nb = (n + 4095) / 4096 + 1;
            PB.keys[0] = (uint64_t *)ensure(ctx->keys0, sizeof(uint64_t) * n);
            PB.keys[1] = (uint64_t *)ensure(ctx->keys1, sizeof(uint64_t) * n);
            PB.vals[0] = (int32_t *)ensure(ctx->vals0, sizeof(int32_t) * n);
            PB.vals[1] = (int32_t *)ensure(ctx->vals1, sizeof(int32_t) * n);
            PB.hist = (uint32_t *)ensure(ctx->hist, sizeof(uint32_t) * 256 * nb);
            PB.part = (uint32_t *)ensure(ctx->part, sizeof(uint32_t) * (256 * nb / 4096 + 2));
        }
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
        launch_prep(A, B, PB, key_bits(G), s, kev);
        QueueGeo Q{};
        Q.wi_off = ds + 6 * G1;
        Q.blkA = ds + 7 * G1;
        Q.chkB = ds + 8 * G1;
        Q.gA = (GroupBox *)ensure(ctx->grpA, sizeof(GroupBox) * (P.blkA[G] + 1));
        Q.gB = (GroupBox *)ensure(ctx->grpB, sizeof(GroupBox) * (P.chkB[G] + 1));
        Q.wi_lb = (float *)ensure(ctx->wi_lb, sizeof(float) * (P.wi[G] + 1));
        Q.wlist = (int32_t *)ensure(ctx->wlist, sizeof(int32_t) * (P.wi[G] + 1));
        launch_group_boxes(A, Q.blkA, P.blkA[G], 64, Q.gA, s);
        launch_group_boxes(B, Q.chkB, P.chkB[G], 256, Q.gB, s);
        RowState *rows = (RowState *)ensure(ctx->rows, sizeof(RowState) * (G > 0 ? G : 1));
        launch_rows_init(rows, G, A.rowbox, B.rowbox, s);

        Lists L{};
        unsigned int qcap = (unsigned int)std::min<int64_t>(std::max<int64_t>(P.potential, 1), QUEUE_BUDGET);
        L.queue = (int2 *)ensure(ctx->queue, sizeof(int2) * qcap);
        L.qlb = (float *)ensure(ctx->qlb, sizeof(float) * qcap);
        L.qcap = qcap;
        L.rescue = (Rescue *)ensure(ctx->rescue, sizeof(Rescue) * RESCUE_CAP);
        L.rcap = RESCUE_CAP;
        L.exact = (ExactItem *)ensure(ctx->exact, sizeof(ExactItem) * EXACT_CAP);
        L.xcap = EXACT_CAP;
        // device scalars (64 B) followed by the counters, read back in one copy
        unsigned int *sc = (unsigned int *)ensure(ctx->scalars, 64 + sizeof(unsigned long long) * C_NCOUNTERS);
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
        launch_reset_lists(L, s);
        clk.mark(2);
        const int prec = opts.precision == SD3_PREC_FP64 ? 1 : 0;
        int &gp = ctx->pairs_grid[prec][mode];
        if (gp == 0) gp = ctx->cus * pairs_blocks_per_cu(prec, mode);
        const int grid_pairs = gp;
        // the queue holds at most qcap tile pairs: split the work items into
        // passes whose potential tile pairs fit
        int64_t n_wi = P.wi[G];
        int64_t per_pass = P.potential <= (int64_t)qcap ? std::max<int64_t>(n_wi, 1)
                                                        : std::max<int64_t>(1, qcap / (64 * 256));
        launch_queue(A, B, Q, n_wi, 0, rows, L, mode == 0 ? Q_SEED : Q_GROUPS, s);
        std::vector<unsigned long long> cand_total(1, 0);
        if (mode == 0) launch_row_scale(rows, G, s);
        // seed round: single queue pass, distance only
        const bool seed = mode == 0 && opts.order != SD3_ORDER_NONE && n_wi <= per_pass;
        Q.compact = n_wi <= per_pass ? 1 : 0;
        for (int64_t w0 = 0; w0 < n_wi; w0 += per_pass) {
            int64_t nw = std::min(per_pass, n_wi - w0);
            if (w0 > 0) launch_reset_queue(L, s);
            if (kev) kev->begin(KE_FILTER, s);
            launch_queue(A, B, Q, nw, w0, rows, L, mode == 0 ? Q_FILTER_DIST : Q_FILTER_HIT, s);
            if (kev) kev->end(KE_FILTER, s);
            if (seed) {
                int2 *sq = (int2 *)ensure(ctx->seedq, sizeof(int2) * (G + 1));
                float *sl = (float *)ensure(ctx->seedlb, sizeof(float) * (G + 1));
                launch_rank(A, B, rows, L, opts.order == SD3_ORDER_LEARNED ? opts.ranker : nullptr,
                            ctx->cus * 2, s);
                Lists LS = L;
                LS.queue = sq;
                LS.qlb = sl;
                LS.qcount = sc + 6;
                LS.qhead = sc + 7;
                LS.qcap = (unsigned int)(G > 0 ? G : 1);
                LS.seed_pass = 1;
                launch_seed_build(rows, G, L, sq, sl, LS.qcount, s);
                launch_pairs(A, B, rows, LS, prec, mode, grid_pairs, s);
            }
            if (w0 == 0) clk.mark(3);
            if (kev) kev->begin(KE_PAIRS, s);
            launch_pairs(A, B, rows, L, prec, mode, grid_pairs, s);
            if (kev) kev->end(KE_PAIRS, s);
            if (n_wi > per_pass) {
                unsigned int *qh = (unsigned int *)readback_area(ctx);
                check(hipMemcpyAsync(qh, L.qcount, sizeof(unsigned int), hipMemcpyDeviceToHost, s), "D2H qcount");
                check(hipStreamSynchronize(s), "sync");
                unsigned int qc = *qh;
                if (qc > qcap) return fail(ctx, SD3_E_CAPACITY, "tile-pair queue overflow");
                cand_total[0] += qc;
            }
        }
        if (n_wi == 0) clk.mark(3);
        clk.mark(4);
        if (prec == 0) launch_rescue(A, B, rows, L, mode, ctx->cus * 4, s);
        clk.mark(5);
        launch_exact(A, B, rows, L, mode, 64, s);
        clk.mark(6);
        // counters first: an overflow is reported before any output is written
        char *rb = readback_area(ctx);
        check(hipMemcpyAsync(rb, sc, 64 + sizeof(unsigned long long) * C_NCOUNTERS, hipMemcpyDeviceToHost, s),
              "D2H counters");
        const unsigned int *sc_h = (const unsigned int *)rb;
        const unsigned long long *cnt_h = (const unsigned long long *)(rb + 64);
        check(hipStreamSynchronize(s), "sync");
        check(hipGetLastError(), "kernel launch");
        if (n_wi <= per_pass) {
            if (sc_h[0] > qcap) return fail(ctx, SD3_E_CAPACITY, "tile-pair queue overflow");
            cand_total[0] = sc_h[0];
        }
        if (sc_h[2] > L.rcap) return fail(ctx, SD3_E_CAPACITY, "rescue list overflow");
        if (sc_h[4] > L.xcap) return fail(ctx, SD3_E_CAPACITY, "exact list overflow");
        // outputs
        double *dd = nullptr;
        uint8_t *hd = nullptr;
        if (a->mem == SD3_MEM_DEVICE) {
            dd = dist;
            hd = hit;
        } else {
            char *ob = (char *)ensure(ctx->out_d, (sizeof(double) + 8) * (G > 0 ? G : 1));
            dd = dist ? (double *)ob : nullptr;
            hd = hit ? (uint8_t *)(ob + sizeof(double) * G) : nullptr;
        }
        launch_finalize(rows, G, dd, hd, s);
        if (a->mem == SD3_MEM_HOST && G > 0) {
            if (dist) check(hipMemcpyAsync(dist, dd, sizeof(double) * G, hipMemcpyDeviceToHost, s), "D2H dist");
            if (hit) check(hipMemcpyAsync(hit, hd, G, hipMemcpyDeviceToHost, s), "D2H hit");
        }
        clk.mark(7);
        check(hipStreamSynchronize(s), "sync");
        if (getenv("SD3_DEBUG_ROWS") && G > 0) {
            std::vector<RowState> rh(std::min<int64_t>(G, 4));
            check(hipMemcpy(rh.data(), rows, sizeof(RowState) * rh.size(), hipMemcpyDeviceToHost), "D2H rows");
            for (size_t g = 0; g < rh.size(); g++) {
                double ub, d2;
                memcpy(&ub, &rh[g].ub, 8);
                memcpy(&d2, &rh[g].d2, 8);
                fprintf(stderr, "sd3 row %zu: ub %.17g d2 %.17g hit %u seed_q %d margin %.3g scale %.17g\n", g,
                        ub, d2, rh[g].hit, rh[g].seed_q, rh[g].margin_scale, rh[g].scale);
            }
        }
        if (stats) {
            memset(stats, 0, sizeof(*stats));
            stats->tile_pairs_total = P.potential;
            stats->tile_pairs_candidate = (int64_t)cand_total[0];
            stats->tile_pairs_evaluated = (int64_t)cnt_h[C_TP_EVAL];
            stats->tri_pairs_boxed = (int64_t)cnt_h[C_TRI_BOXED];
            stats->tri_pairs_fp32 = (int64_t)cnt_h[C_TRI32];
            stats->tri_pairs_fp64 = (int64_t)cnt_h[C_TRI64];
            stats->rescued = (int64_t)cnt_h[C_RESCUED];
            stats->exact = (int64_t)cnt_h[C_EXACT];
            stats->logged = (int64_t)cnt_h[C_LOGGED];
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
            stats->sort_items = A.nt + B.nt;
            stats->sort_key_bytes = key_bits(G) + 1 <= 32 ? 4 : 8;
            stats->sort_passes = (key_bits(G) + 1 + 7) / 8;
        }
    } catch (const HipError &e) {
        (void)hipGetLastError();
        if (e.e == hipErrorOutOfMemory) return fail(ctx, SD3_E_NOMEM, std::string(e.what) + ": out of device memory");
        return fail(ctx, SD3_E_DEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
    } catch (const std::bad_alloc &) {
        return fail(ctx, SD3_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ctx, SD3_E_DEVICE, "unexpected error");
    }
    return SD3_OK;
}

}  // namespace

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
    sd3_ctx *c = new (std::nothrow) sd3_ctx();
    if (!c) return SD3_E_NOMEM;
    c->device = device;
    c->cus = p.multiProcessorCount;
    *out = c;
    return SD3_OK;
}

sd3_status sd3_destroy(sd3_ctx *ctx) {
    if (!ctx) return SD3_OK;
    (void)hipSetDevice(ctx->device);
    for (auto &sd : ctx->side) {
        DevBuf *bs[] = {&sd.xyz, &sd.tri, &sd.v_off, &sd.t_off, &sd.tile_off, &sd.rowbox,
                        &sd.t32, &sd.t64, &sd.meta};
        for (DevBuf *b : bs) release(*b);
    }
    DevBuf *bs[] = {&ctx->rows, &ctx->wi_off, &ctx->queue, &ctx->qlb, &ctx->rescue, &ctx->exact,
                    &ctx->counters, &ctx->scalars, &ctx->flags, &ctx->out_d, &ctx->out_h,
                    &ctx->keys0, &ctx->keys1, &ctx->vals0, &ctx->vals1, &ctx->hist, &ctx->part,
                    &ctx->grpA, &ctx->grpB, &ctx->wi_lb, &ctx->seedq, &ctx->seedlb, &ctx->mlp,
                    &ctx->wlist};
    for (DevBuf *b : bs) release(*b);
    for (hipEvent_t &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    release(ctx->small);
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
    return run(ctx, a, b, dist, hit, opts, stats, stream, 0);
}

sd3_status sd3_intersects(sd3_ctx *ctx, const sd3_geoms *a, const sd3_geoms *b, uint8_t *hit,
                          const sd3_opts *opts, sd3_stats *stats, void *stream) {
    return run(ctx, a, b, nullptr, hit, opts, stats, stream, 1);
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
