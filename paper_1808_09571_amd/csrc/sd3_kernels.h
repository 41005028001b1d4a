// Host-side launch wrappers of the sd3 kernels (defined in sd3_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sd3_common.h"

namespace sd3 {

// Per-side prepared data (all device pointers).
struct SideBufs {
    const double *xyz;
    const int32_t *tri;
    const int64_t *v_off;     // [G+1]
    const int64_t *t_off;     // [G+1]
    const int64_t *tile_off;  // [G+1]
    int64_t G, nv, nt, NT;
    int tk;                      // triangles per tile
    int boxrep;                  // replicas of the row boxes (spread the reduction atomics)
    unsigned long long *rowbox;  // [boxrep][G*6] ordered bits: lo xyz (min), hi xyz (max);
                                 // replica 0 holds the merged box after validation
    float *t32;                  // [NT*9*tk]: tile t, coordinate c, slot j at (t*9+c)*tk+j
                                 // (FP32 path), or nullptr
    double *t64;                 // [NT*9*tk] exact copies (plain FP64 path), or nullptr
    int32_t *ids;                // [NT*tk] triangle of each slot
    TileMeta *meta;              // [NT]
    uint32_t *mat;               // [NT] 0 until the tile's copies (t32 or t64) are written
                                 // (large calls: only tiles of queued tile pairs get them)
};

// Optional HIP-event brackets around selected kernel launches (timing mode):
// per kernel class, up to 16 (begin, end) pairs per call.
enum : int { KE_SCATTER = 0, KE_TILES = 1, KE_FILTER = 2, KE_PAIRS = 3, KE_CLASSES = 4 };
struct KernelEvents {
    hipEvent_t ev[KE_CLASSES][32];
    int n[KE_CLASSES];
    void begin(int c, hipStream_t s) {
        if (n[c] < 16) (void)hipEventRecord(ev[c][2 * n[c]], s);
    }
    void end(int c, hipStream_t s) {
        if (n[c] < 16) (void)hipEventRecord(ev[c][2 * n[c] + 1], s);
        n[c]++;
    }
};

// Radix-sort items per block (each block's per-digit histogram is one row of
// the scanned (digit, block) table): RS_ITEMS for sorts of up to SMALL_SORT
// keys, twice that above; buffers are sized for RS_ITEMS.  Larger sorts also
// take their keys from per-vertex Morton codes.
constexpr int RS_ITEMS = 2048;
constexpr int64_t SMALL_SORT = (int64_t)1 << 22;

// Sort blocks: each row of each side is cut into blocks of `rsi` items (a
// row's last block may be shorter, an empty row has none); A's blocks come
// first.  A block's per-digit histogram goes to its row's region of the
// histogram table, laid out [row][digit][block of the row] with A's rows
// before B's, so one exclusive scan of the whole table gives every (row,
// digit, block) its place in the sorted order: the sort orders items within
// their row and never moves them across rows, and the keys hold Morton bits
// only.
// One sort block: its side, row, first item (both sides' items numbered A
// then B) and first triangle of the side, length, and where its digit counts
// go in the histogram table (digit d at hbase + d * hstride).
struct SBlock {
    int64_t i0, t0, g, hbase;
    int32_t n, hstride, side;
    int32_t loc;  // index of the block's first item within its row
};
struct SortSeg {
    const int64_t *sbA, *sbB;      // [G+1] first sort block of each row (B's counted from nbA)
    const int64_t *toffA, *toffB;  // [G+1] triangle offsets
    int64_t G, ntA, nbA, nb;       // rows, A's items, A's blocks, all blocks
    int rsi;                       // items per block
    SBlock *tab;                   // [nb] every block's entry (calls of many rows), or nullptr:
                                   // each block then finds its own
    const int32_t *kc;             // [2G] kept items per row of a culling call, else nullptr:
                                   // after the first pass they lead each row's range and
                                   // later passes read and place only them
    int32_t *bn;                   // [nb] kept items per sort block of a culling call (the key
                                   // kernel writes them first in the block), else nullptr
};
// Calls of at least this many rows build the sort-block table first.
constexpr int64_t SORT_TABLE_MIN_ROWS = 64;

// Sort buffers shared by both sides (device).
struct PrepBufs {
    uint32_t *keys[2];  // [ntA + ntB] ping-pong
    int32_t *vals[2];
    uint32_t *hist;     // [256 * blocks]
    uint32_t *part;     // [chunks]
    uint32_t *vcode;    // [nvA + nvB] Morton code of every vertex, or nullptr (keys
                        // then quantise each first vertex themselves)
    int32_t *kc;        // [2G] triangles kept per row (A rows, then B rows) when a
                        // call culls by the other side's row box (large sorts
                        // only), else nullptr
    uint8_t *oc;        // [nvA + nvB] every vertex's outcode (culling calls), else nullptr
    double *cub;        // [G] a distance call's cull distance per row (an upper
                        // bound of the row distance plus a margin), else nullptr
                        // (intersects culls by the box itself)
    SortSeg seg;
    uint32_t *flags;    // [2] validation flags of A and B (the key kernel checks indices)
};

// Counters (device, unsigned long long[16]).
enum Counter : int {
    C_TP_CAND = 0,
    C_TP_EVAL = 1,
    C_TRI_BOXED = 2,
    C_TRI32 = 3,
    C_TRI64 = 4,
    C_RESCUED = 5,
    C_EXACT = 6,
    C_QUEUE_OVF = 7,
    C_RESCUE_OVF = 8,
    C_EXACT_OVF = 9,
    C_LOGGED = 10,
    C_SKEW = 11,  // waves that found the block's queue entry changed under them
    C_COPIED = 12,  // tiles whose coordinate copies were written
    C_NCOUNTERS = 16,
};

// Queue / work lists (device).
struct Lists {
    int2 *queue;
    float *qlb;
    unsigned int *qcount;   // [1]
    unsigned int *qhead;    // [1]
    unsigned int qcap;
    Rescue *rescue;
    unsigned int *rcount;
    unsigned int *rhead;
    unsigned int rcap;
    ExactItem *exact;
    unsigned int *xcount;
    unsigned int xcap;
    unsigned long long *counters;  // [C_NCOUNTERS]
    int seed_pass;                 // 1: entries are the rows' seed choices (RowState::best)
    int64_t nrows;                 // rows (entries of a seed pass)
    float *log;                    // training log (device) or nullptr
    unsigned long long log_cap;
    unsigned long long *log_count;
    unsigned int *xdone;           // blocks of the exact kernel that finished
};

// Validation flags.
enum : uint32_t { V_NONFINITE = 1, V_RANGE = 2, V_INDEX = 4 };

// A call failed on the device when either side's validation flags are set or
// a work list overflowed (queue: this pass or an earlier one).
__device__ __forceinline__ bool call_failed(const Lists &L, const uint32_t *vflags) {
    return (vflags && (vflags[0] | vflags[1]) != 0) || *L.qcount > L.qcap ||
           L.counters[C_QUEUE_OVF] != 0 || *L.rcount > L.rcap || *L.xcount > L.xcap;
}


// Validation of both sides (flags[0] for A, flags[1] for B) fused with the
// row bounding boxes (one read of xyz): clears the flags, boxes, work-list
// scalars and counters, checks every coordinate, reduces the row boxes (into
// A.boxrep replicas) and, with `indices`, checks every triangle index (a
// call's pipeline leaves that to the key kernel, which reads the indices
// anyway).
void launch_validate_rowbox(SideBufs &A, SideBufs &B, PrepBufs &P, uint32_t *flags, Lists &L,
                            hipStream_t s, bool indices);
// Replicas of the row boxes for rows of nv vertices on the larger side: at
// most 16, one unless a row spans at least 32 reduction blocks.
int rowbox_replicas(int64_t nv, int64_t G);
// Sort items: the Morton prefix (mbits = 8 * passes bits, one 8-bit radix
// pass per byte) with the triangle's index.  Narrow (no row has more than
// 2^24 triangles): the index is the triangle's within its row, and the pass
// before the last writes each item as one 32-bit word, the last digit above
// the 24-bit index, which the last pass moves alone (4 bytes per item instead
// of a key and a value); else a 32-bit key and a 32-bit value, the index
// within the side, throughout.
struct SortKey {
    int mbits, passes;
    bool narrow;
    int bits() const { return mbits; }
    // bytes an item moves through the scatter passes: 16 per full pass
    // (key and value read and written), 12 for the last full pass (no keys
    // written) or the narrowing pass (one word written), 8 for a word pass
    int scatter_bytes() const { return narrow ? 16 * (passes - 2) + 12 + 8 : 16 * (passes - 1) + 12; }
};
SortKey sort_key(int64_t max_row_items);
// Morton keys of both sides (the same launch starts the row states from the
// merged row boxes), the radix sort and the tiles.
void launch_prep(SideBufs &A, SideBufs &B, PrepBufs &P, const SortKey &K, RowState *rows,
                 hipStream_t s, KernelEvents *kev);
// The FP32 (prec 0) or FP64 copies of every tile named by a queued tile pair
// that has none yet (the tile build of a large call writes only metadata and
// slot ids; a small call's tile build writes every copy, and this launches
// nothing).
void launch_materialize(SideBufs &A, SideBufs &B, const Lists &L, int prec, int grid, hipStream_t s);

// Group boxes (A block of 64 tiles / B chunk of 256 tiles of one row).
struct GroupBox {
    double lo[3], hi[3], rep[3];
};

// Queue geometry (device): work-item offsets, group offsets and boxes, and the
// per-work-item group lower bound.
struct QueueGeo {
    const int64_t *wi_off;  // [G+1]
    const int64_t *blkA;    // [G+1] A-block offsets
    const int64_t *chkB;    // [G+1] B-chunk offsets
    GroupBox *gA, *gB;
    float *wi_lb;           // [n_wi]
    int32_t *wlist;         // [n_wi] compacted work items
    unsigned int *wcount;   // [2] device counts (seeding, filtering); zeroed per call
    int compact;            // compacted work lists (single queue pass over many rows)
};

// Group boxes of both sides in one launch: A blocks of 64 tiles, B chunks of
// 256 tiles.
void launch_group_boxes(const SideBufs &A, const SideBufs &B, const QueueGeo &Q, int64_t nblkA,
                        int64_t nchkB, hipStream_t s);

// Q_SEED: group bounds and upper bounds from vertex pairs (distance);
// Q_GROUPS: group bounds only (intersects); Q_FILTER_DIST: keep tile pairs with
// box lower bound <= ub + m; Q_FILTER_HIT: keep overlapping boxes.
enum : int { Q_SEED = 0, Q_GROUPS = 1, Q_FILTER_DIST = 2, Q_FILTER_HIT = 3 };
// rank (filter passes of sd3_distance): 1 chooses each row's seed by box bound
// in the filter's own launch, 0 does not.
void launch_queue(const SideBufs &A, const SideBufs &B, const QueueGeo &Q, int64_t n_wi,
                  int64_t wi_begin, RowState *rows, Lists &L, int what, hipStream_t s, int rank);
// Learned seed choice: scores every queued tile pair with the ranker MLP
// (weights `ranker`) and keeps each row's lowest score in the row state.
void launch_rank(const SideBufs &A, const SideBufs &B, RowState *rows, Lists &L,
                 const float *ranker, int grid, hipStream_t s);
// The learned seed round's scorer applied to feature rows x [n][MLP_IN] -> y [n]
// (the device function k_rank uses).
void launch_rank_score(const float *W, const float *x, int64_t n, float *y, int grid,
                       hipStream_t s);
int pairs_blocks_per_cu(int precision, int mode, int tk);
void launch_pairs(const SideBufs &A, const SideBufs &B, RowState *rows, Lists &L, int precision,
                  int mode, int grid, hipStream_t s);
void launch_rescue(const SideBufs &A, const SideBufs &B, RowState *rows, Lists &L, int mode,
                   int grid, hipStream_t s);
// With fin_rows > 0 the last block of the exact kernel also writes the
// results (as launch_finalize), which saves a launch.
void launch_exact(const SideBufs &A, const SideBufs &B, RowState *rows, Lists &L, int mode,
                  int grid, hipStream_t s, int64_t fin_rows, double *dist, uint8_t *hit,
                  const uint32_t *vflags);
// Rescue, exact arithmetic and (fin_rows > 0) the results in one launch, for
// calls whose rescue list is short (few rows).
void launch_resolve(const SideBufs &A, const SideBufs &B, RowState *rows, Lists &L, int mode,
                    int grid, hipStream_t s, int64_t fin_rows, double *dist, uint8_t *hit,
                    const uint32_t *vflags);
// Seed round: the filter (box bound) or the ranker records each row's
// best-ranked queued tile pair in the row state; a pass of the tile-pair
// kernel in seed mode (Lists::seed_pass) evaluates those before the main pass.
void launch_seed_reset(RowState *rows, int64_t G, unsigned int *seedhead, hipStream_t s);
void launch_finalize(const RowState *rows, int64_t G, double *dist, uint8_t *hit, Lists &L,
                     const uint32_t *vflags, hipStream_t s);
void launch_reset_queue(Lists &L, hipStream_t s);

// Solid semantics (sd3_solid.hip): point-in-solid queries by exact ray
// parity.  Query code 2 g + s: the first vertex of side s's row g against
// side 1 - s's row g; dir[code] selects the ray direction; res[code] bits:
// 1 inside, 2 degenerate direction (run again with another), 4 on the surface.
constexpr int SOLID_DIRS = 8;
struct SolidSide {
    const double *xyz;
    const int32_t *tri;
    const int64_t *v_off, *t_off;  // [G+1] device
};
void launch_inside(const SolidSide &A, const SolidSide &B, const RowState *rows, const int32_t *queries,
                   int64_t nq, const uint8_t *dir, uint8_t *res, int grid, hipStream_t s);
// rows whose solids meet (res) get distance 0 and hit 1 (unless the call failed)
void launch_solid_apply(const uint8_t *res, int64_t G, double *dist, uint8_t *hit, const RowState *rows,
                        Lists &L, const uint32_t *vflags, hipStream_t s);

// Volume of each row (sd3_volume.hip): work items are (row, chunk of
// volume_chunk() triangles); part holds 16 bytes per item; flags[0] takes the
// validation bits.
int volume_chunk();
void launch_volume(const double *xyz, int64_t nv, const int32_t *tri, const int64_t *v_off,
                   const int64_t *t_off, const int32_t *wrow, const int64_t *wfirst, int64_t nitems,
                   const int64_t *witem, int64_t G, void *part, double *vol, uint32_t *flags, int grid,
                   hipStream_t s);

// Segments / points against one mesh (sd3_segments.hip).  Mesh preparation:
// P [nt][36] FP64 triangles (30 derived fields, box), tile boxes [ceil(nt/64)][6]
// and the mesh box mbox[6].  flags[0] (segments) and flags[1] (mesh) take the
// validation bits; cnt[0..2]: box tests, full pair tests, exact tests.
constexpr int SEG_MESH_TILE = 64;
constexpr int SEG_MESH_FIELDS = 36;
void launch_seg_validate(const double *seg, int64_t n, const double *xyz, int64_t nv, const int32_t *tri,
                         int64_t nt, uint32_t *flags, unsigned long long *cnt, hipStream_t s);
void launch_seg_mesh(const double *xyz, int64_t nv, const int32_t *tri, int64_t nt, double *P,
                     double *tbox, double *mbox, hipStream_t s);
int seg_blocks_per_cu(int mode);
// mode 0: dist (+ hit if non-null), 1: hit = intersects, 2: hit = distance <= r
void launch_segs(int mode, const double *seg, int64_t n, const double *P, int64_t nt, const double *tbox,
                 const double *mbox, double r, double *dist, uint8_t *hit, const uint32_t *flags,
                 unsigned long long *cnt, int grid, hipStream_t s);

}  // namespace sd3
