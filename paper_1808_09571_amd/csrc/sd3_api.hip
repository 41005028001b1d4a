// sd3 C-ABI: argument checks, device buffers and the pipeline of one call.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/sd3.h"
#include "sd3_kernels.h"

using namespace sd3;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

struct SideState {
    DevBuf xyz, tri, v_off, t_off, tile_off, rowbox, keys0, keys1, vals0, vals1, hist, t32, t64, meta;
};

struct Plan {
    int64_t G = 0;
    std::vector<int64_t> tileA, tileB;  // [G+1] tile offsets
    std::vector<int64_t> wi;            // [G+1] work-item offsets
    int64_t potential = 0;              // sum of tilesA * tilesB
};

}  // namespace

struct sd3_ctx {
    int device = 0;
    int cus = 0;
    std::string err;
    SideState side[2];
    DevBuf rows, wi_off, queue, qlb, rescue, exact, counters, scalars, flags, out_d, out_h;
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
// buffers.  No kernel reads the data before it has been validated.
void setup_side(sd3_ctx *ctx, int which, const sd3_geoms *g, const std::vector<int64_t> &tile_off,
                  SideBufs &S, hipStream_t s) {
    SideState &st = ctx->side[which];
    int64_t G = g->count, nv = g->v_off[G], nt = g->t_off[G];
    S.G = G;
    S.nv = nv;
    S.nt = nt;
    S.NT = tile_off[G];
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
    int64_t *vo = (int64_t *)ensure(st.v_off, sizeof(int64_t) * (G + 1));
    int64_t *to = (int64_t *)ensure(st.t_off, sizeof(int64_t) * (G + 1));
    int64_t *tf = (int64_t *)ensure(st.tile_off, sizeof(int64_t) * (G + 1));
    check(hipMemcpyAsync(vo, g->v_off, sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s), "H2D v_off");
    check(hipMemcpyAsync(to, g->t_off, sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s), "H2D t_off");
    check(hipMemcpyAsync(tf, tile_off.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s), "H2D tiles");
    S.v_off = vo;
    S.t_off = to;
    S.tile_off = tf;
    S.rowbox = (unsigned long long *)ensure(st.rowbox, sizeof(unsigned long long) * 6 * (G > 0 ? G : 1));
    S.keys[0] = (uint64_t *)ensure(st.keys0, sizeof(uint64_t) * nt);
    S.keys[1] = (uint64_t *)ensure(st.keys1, sizeof(uint64_t) * nt);
    S.vals[0] = (int32_t *)ensure(st.vals0, sizeof(int32_t) * nt);
    S.vals[1] = (int32_t *)ensure(st.vals1, sizeof(int32_t) * nt);
    S.hist = (uint32_t *)ensure(st.hist, sizeof(uint32_t) * 256 * ((nt + 4095) / 4096 + 1));
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
sd3_status validate_device(sd3_ctx *ctx, const sd3_geoms *g, const SideBufs &S, hipStream_t s) {
    uint32_t *flags = (uint32_t *)ensure(ctx->flags, 256);
    check(hipMemsetAsync(flags, 0, sizeof(uint32_t), s), "memset flags");
    launch_validate(g->xyz, S.nv, g->tri, S.nt, S.v_off, S.t_off, S.G, flags, s);
    uint32_t h = 0;
    check(hipMemcpyAsync(&h, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "D2H flags");
    check(hipStreamSynchronize(s), "sync");
    if (h & V_NONFINITE) return fail(ctx, SD3_E_NONFINITE, "non-finite coordinate");
    if (h & V_RANGE) return fail(ctx, SD3_E_RANGE, "coordinate magnitude outside [2^-256, 2^256]");
    if (h & V_INDEX) return fail(ctx, SD3_E_INDEX_RANGE, "triangle index outside its row");
    return SD3_OK;
}

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
    if (opts.order != SD3_ORDER_BOUND && opts.order != SD3_ORDER_NONE)
        return fail(ctx, SD3_E_INVALID_ARG, "unknown order");
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
        for (int64_t g = 0; g < G; g++) {
            int64_t na = tiles_of(a->t_off[g + 1] - a->t_off[g]);
            int64_t nb = tiles_of(b->t_off[g + 1] - b->t_off[g]);
            P.tileA[g + 1] = P.tileA[g] + na;
            P.tileB[g + 1] = P.tileB[g] + nb;
            P.wi[g + 1] = P.wi[g] + ((na + 63) / 64) * ((nb + 255) / 256);
            P.potential += na * nb;
        }
        SideBufs A{}, B{};
        setup_side(ctx, 0, a, P.tileA, A, s);
        setup_side(ctx, 1, b, P.tileB, B, s);
        if (a->mem == SD3_MEM_DEVICE) {
            st = validate_device(ctx, a, A, s);
            if (st == SD3_OK) st = validate_device(ctx, b, B, s);
            if (st != SD3_OK) return st;
        }
        launch_prep(A, key_bits(G), s);
        launch_prep(B, key_bits(G), s);
        RowState *rows = (RowState *)ensure(ctx->rows, sizeof(RowState) * (G > 0 ? G : 1));
        launch_rows_init(rows, G, A.rowbox, B.rowbox, s);
        int64_t *wi = (int64_t *)ensure(ctx->wi_off, sizeof(int64_t) * (G + 1));
        check(hipMemcpyAsync(wi, P.wi.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s), "H2D wi");
        Lists L{};
        unsigned int qcap = (unsigned int)std::min<int64_t>(std::max<int64_t>(P.potential, 1), QUEUE_BUDGET);
        L.queue = (int2 *)ensure(ctx->queue, sizeof(int2) * qcap);
        L.qlb = (float *)ensure(ctx->qlb, sizeof(float) * qcap);
        L.qcap = qcap;
        L.rescue = (Rescue *)ensure(ctx->rescue, sizeof(Rescue) * RESCUE_CAP);
        L.rcap = RESCUE_CAP;
        L.exact = (ExactItem *)ensure(ctx->exact, sizeof(ExactItem) * EXACT_CAP);
        L.xcap = EXACT_CAP;
        unsigned int *sc = (unsigned int *)ensure(ctx->scalars, 64);
        L.qcount = sc;
        L.qhead = sc + 1;
        L.rcount = sc + 2;
        L.rhead = sc + 3;
        L.xcount = sc + 4;
        L.counters = (unsigned long long *)ensure(ctx->counters, sizeof(unsigned long long) * C_NCOUNTERS);
        launch_reset_lists(L, s);
        const int prec = opts.precision == SD3_PREC_FP64 ? 1 : 0;
        const int grid_pairs = ctx->cus * 8;
        // the queue holds at most qcap tile pairs: split the work items into
        // passes whose potential tile pairs fit
        int64_t n_wi = P.wi[G];
        int64_t per_pass = P.potential <= (int64_t)qcap ? std::max<int64_t>(n_wi, 1)
                                                        : std::max<int64_t>(1, qcap / (64 * 256));
        if (mode == 0) launch_queue(A, B, wi, n_wi, 0, rows, L, Q_SEED, s);
        std::vector<unsigned long long> cand_total(1, 0);
        for (int64_t w0 = 0; w0 < n_wi; w0 += per_pass) {
            int64_t nw = std::min(per_pass, n_wi - w0);
            if (w0 > 0) launch_reset_queue(L, s);
            launch_queue(A, B, wi, nw, w0, rows, L, mode == 0 ? Q_FILTER_DIST : Q_FILTER_HIT, s);
            launch_pairs(A, B, rows, L, prec, mode, grid_pairs, s);
            if (n_wi > per_pass) {
                unsigned int qc = 0;
                check(hipMemcpyAsync(&qc, L.qcount, sizeof(unsigned int), hipMemcpyDeviceToHost, s), "D2H qcount");
                check(hipStreamSynchronize(s), "sync");
                if (qc > qcap) return fail(ctx, SD3_E_CAPACITY, "tile-pair queue overflow");
                cand_total[0] += qc;
            }
        }
        if (prec == 0) launch_rescue(A, B, rows, L, mode, ctx->cus * 4, s);
        launch_exact(A, B, rows, L, mode, ctx->cus * 4, s);
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
        unsigned int sc_h[5];
        unsigned long long cnt_h[C_NCOUNTERS];
        check(hipMemcpyAsync(sc_h, sc, sizeof(sc_h), hipMemcpyDeviceToHost, s), "D2H scalars");
        check(hipMemcpyAsync(cnt_h, L.counters, sizeof(cnt_h), hipMemcpyDeviceToHost, s), "D2H counters");
        check(hipStreamSynchronize(s), "sync");
        check(hipGetLastError(), "kernel launch");
        if (n_wi <= per_pass) {
            if (sc_h[0] > qcap) return fail(ctx, SD3_E_CAPACITY, "tile-pair queue overflow");
            cand_total[0] = sc_h[0];
        }
        if (sc_h[2] > L.rcap) return fail(ctx, SD3_E_CAPACITY, "rescue list overflow");
        if (sc_h[4] > L.xcap) return fail(ctx, SD3_E_CAPACITY, "exact list overflow");
        if (a->mem == SD3_MEM_HOST && G > 0) {
            if (dist) check(hipMemcpyAsync(dist, dd, sizeof(double) * G, hipMemcpyDeviceToHost, s), "D2H dist");
            if (hit) check(hipMemcpyAsync(hit, hd, G, hipMemcpyDeviceToHost, s), "D2H hit");
            check(hipStreamSynchronize(s), "sync");
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
            stats->ms_total =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
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
        DevBuf *bs[] = {&sd.xyz, &sd.tri, &sd.v_off, &sd.t_off, &sd.tile_off, &sd.rowbox, &sd.keys0,
                        &sd.keys1, &sd.vals0, &sd.vals1, &sd.hist, &sd.t32, &sd.t64, &sd.meta};
        for (DevBuf *b : bs) release(*b);
    }
    DevBuf *bs[] = {&ctx->rows, &ctx->wi_off, &ctx->queue, &ctx->qlb, &ctx->rescue, &ctx->exact,
                    &ctx->counters, &ctx->scalars, &ctx->flags, &ctx->out_d, &ctx->out_h};
    for (DevBuf *b : bs) release(*b);
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
