/*
 * sj.h -- C ABI of the MI355X (gfx950) spatial-join library.
 *
 * The library computes the filter step of the spatial intersection join of
 * Tsitsigkos, Bouros, Mamoulis and Terrovitis, "Parallel In-Memory Evaluation
 * of Spatial Joins" (SIGSPATIAL 2019, arXiv 1908.11740):
 *
 *   given two collections R and S of axis-aligned rectangles (object MBRs),
 *   return every pair (r, s), r in R, s in S, whose rectangles share at least
 *   one point (Sec. 1, problem statement; Algorithm 1 input/output).
 *
 * It follows the paper's partition-based method (PBSM, Sec. 2.2): both inputs
 * are assigned to every tile of a uniform K x K grid they intersect
 * (partitioning phase, Sec. 3.4 steps 1-4), each tile's two lists are sorted
 * by lower x-endpoint and joined with the forward-scan plane sweep of
 * Algorithm 1 (joining phase, Sec. 3.4 steps 5-6), and a pair found in
 * several tiles is reported only in the tile that holds the reference point
 * of its intersection (Eq. (1)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Rectangles   n x 4 float32, array-of-structs (x_l, y_l, x_u, y_u), in
 *              DEVICE memory, 16-byte aligned.  Every value must be finite and
 *              x_l <= x_u, y_l <= y_u; otherwise the call returns SJ_ERR_RECT.
 *              Intersection is closed: touching edges and corners count, and
 *              zero-width or zero-height rectangles are allowed.  -0.0 is
 *              treated as +0.0.
 * Sizes        n < 2^30 rectangles per input; at most 2^31 - 1 tile entries
 *              (rectangles times the tiles each one covers) per input.
 * Pairs        sj_pair {r, s}: 0-based positions in the caller's R and S.
 *              Each intersecting pair is reported exactly once.  The order is
 *              unspecified; the set does not depend on K, the split threshold
 *              or any launch shape.
 * Streams      `stream` is a hipStream_t (NULL = the default stream).  Work is
 *              enqueued on it.  Entry points that return a count synchronise
 *              that stream once to read it.
 * Ownership    Input pointers are borrowed for the duration of the call (the
 *              caller may free them once the stream has synchronised).
 *              Output buffers are caller-owned.  sj_part and sj_batch handles
 *              are library-owned and released with their _free function.
 * Errors       No exception or abort crosses the ABI; every failure is a
 *              negative sj_status.  Handles are not thread-safe: calls that
 *              use the same handle, or that run on the same device, must not
 *              overlap in time.
 */
#ifndef SJ_H
#define SJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SJ_OK = 0,
    SJ_ERR_ARG = -1,           /* bad argument: NULL pointer, negative size, K out of range */
    SJ_ERR_RECT = -2,          /* an input rectangle is NaN / infinite / inverted            */
    SJ_ERR_CAPACITY = -3,      /* output buffer too small; *n_pairs holds the needed count   */
    SJ_ERR_GRID_MISMATCH = -4, /* R and S were partitioned on different grids               */
    SJ_ERR_OOM = -5,           /* device allocation failed                                   */
    SJ_ERR_DEVICE = -6,        /* HIP runtime error, or no usable GPU                        */
    SJ_ERR_TOO_LARGE = -7      /* input beyond the size limits above                         */
} sj_status;

/* Largest grid: K x K tiles with K <= SJ_K_MAX. */
#define SJ_K_MAX 8192

/* sj_grid.flags */
#define SJ_PLAIN 0x1u           /* baseline schedule: one workgroup per tile, no dense-tile
                                   splitting, no batching of small tiles                   */
#define SJ_RULE_ONLY 0x2u       /* sj_choose_grid: use the statistics rule even if a
                                   learned picker is loaded                                */
#define SJ_TWO_PASS 0x4u        /* sj_join: count, scan, then write the pairs in a second
                                   sweep instead of one sweep into scratch + compaction;
                                   never changes the result                                */
#define SJ_STRIPES 0x8u         /* one-dimensional partitioning (Sec. 3.1): k vertical stripes
                                   of the domain, each joined by a plane sweep along y; the
                                   duplicate test of Eq. (1) reduces to the reference point's
                                   x (Sec. 3.2).  sj_choose_grid's rule then uses the mean
                                   x-extent (Sec. 4.3.1)                                   */
#define SJ_SWEEP_X 0x10u        /* sj_join: sweep every tile along x.  Without it, tiles
                                   joined as medium or dense work units choose their
                                   sweeping axis with the model of Sec. 3.3 (Eq. (2));
                                   never changes the result                                */
#define SJ_GBDA 0x20u           /* sj_join: join each dense tile as the 9 class-class mini-joins
                                   of grouping-based duplicate avoidance (classes by where a
                                   rectangle's projections begin relative to the tile; only the
                                   9 class pairs that can hold a pair whose reference point is
                                   in the tile), each split into pivot ranges, with no
                                   duplicate test; never changes the result                */
#define SJ_SORTED_OUTPUT 0x40u  /* sj_join, sj_distance_join: the pairs are written in
                                   lexicographic (r, s) order (sj_sort_pairs after the
                                   join), so the output bytes do not depend on the grid or
                                   schedule; without it the order is unspecified           */

/*
 * The uniform grid (Sec. 2.2; K x K tiles, Sec. 4.3.2).
 *   k          cells per dimension, 1..SJ_K_MAX.  0 in sj_choose_grid's input
 *              means "choose".
 *   split_tau  dense-tile split threshold: a tile whose two lists together
 *              hold more than split_tau entries is joined by several
 *              workgroups, each taking a contiguous range of at most
 *              split_tau sweep pivots.  0 = library default; INT32_MAX =
 *              never split.  Never changes the result.
 *   domain     x0, y0, x1, y1 of the gridded region; all zero = the unit
 *              square [0,1)^2 (the paper normalises data to [0,1], Sec. 4.1).
 *              Rectangles outside it are clamped into the border tiles.
 *   flags      SJ_PLAIN, SJ_RULE_ONLY, SJ_TWO_PASS, SJ_STRIPES, SJ_SWEEP_X, SJ_GBDA,
 *              SJ_SORTED_OUTPUT.
 * Tile (tx, ty) holds the rectangles whose cell ranges
 * [cell(x_l), cell(x_u)] x [cell(y_l), cell(y_u)] contain it, with
 * cell(v) = clamp(floor((v - x0) * K / (x1 - x0)), 0, K - 1) in float32.
 * With SJ_STRIPES, stripe t holds the rectangles whose x cell range
 * [cell(x_l), cell(x_u)] contains t.
 */
typedef struct {
    int32_t k;
    int32_t split_tau;
    float domain[4];
    uint32_t flags;
} sj_grid;

typedef struct {
    int32_t r, s;
} sj_pair;

typedef struct sj_part sj_part; /* one partitioned input (library-owned, device memory) */

/*
 * Partitioning phase for one input (Sec. 3.4 steps 1-4; PBSM assignment of
 * Sec. 2.2): validate the rectangles, count the entries of every tile,
 * prefix-sum the counts into per-tile segment offsets and scatter each
 * rectangle into the segment of every tile it intersects.
 *   rects  n x 4 float32 AoS, device.
 *   g      grid with 1 <= k <= SJ_K_MAX and a non-degenerate domain.
 *   out    *out == NULL: a new handle is created.  *out != NULL: that handle
 *          is reused (its device buffers grow only when too small).
 * Synchronises the stream once (to size the segments).  On error *out is
 * left as it was on entry.
 */
sj_status sj_partition(const float* rects, int64_t n, const sj_grid* g, sj_part** out,
                       void* stream);

/*
 * Joining phase (Sec. 3.4 steps 5-6): per tile, sort both lists by x_l and
 * run the forward-scan plane sweep of Algorithm 1; keep a pair only if the
 * reference point of Eq. (1) lies in the tile.
 *   R, S      handles partitioned on the same grid (k and domain), else
 *             SJ_ERR_GRID_MISMATCH.  The split threshold and flags of R's
 *             grid select the schedule.
 *   out       device buffer of `capacity` pairs (may be NULL if capacity 0).
 *   n_pairs   host; receives |J|.  If |J| > capacity the call returns
 *             SJ_ERR_CAPACITY and the buffer contents are unspecified.
 */
sj_status sj_join(const sj_part* R, const sj_part* S, sj_pair* out, int64_t capacity,
                  int64_t* n_pairs, void* stream);

/* As sj_join, counting |J| without writing pairs. */
sj_status sj_join_count(const sj_part* R, const sj_part* S, int64_t* n_pairs, void* stream);

/*
 * Both phases in one call (Sec. 3.4 steps 1-6): sj_partition of R and of S
 * on grid g, then sj_join, with one status readback (one stream
 * synchronisation) for the whole sequence instead of one per call.  The
 * partitions' buffers are sized from bounds (and from earlier calls on the
 * same handles); the kernels check every capacity on the device, and when a
 * partition outgrows its buffers they grow and the sequence runs again.
 *   R, S        nR / nS x 4 float32 AoS, device, 16-byte aligned.
 *   g           a resolved grid (1 <= k <= SJ_K_MAX; choose one first with
 *               sj_choose_grid for the learned / rule choice); SJ_PLAIN is
 *               rejected (SJ_ERR_ARG).
 *   pr, ps      partition handles as in sj_partition (*p == NULL: created;
 *               else reused).  On return they hold the two partitions; on
 *               error handles created by the call are freed and *pr, *ps
 *               are left as they were.
 *   out         device buffer of `capacity` pairs; NULL: count only.
 *   n_pairs     host; receives |J| (SJ_ERR_CAPACITY if it exceeds capacity).
 */
sj_status sj_join_rects(const float* R, int64_t nR, const float* S, int64_t nS, const sj_grid* g,
                        sj_part** pr, sj_part** ps, sj_pair* out, int64_t capacity,
                        int64_t* n_pairs, void* stream);

/* Entries (rectangle-tile assignments) and rectangles of a partitioned input. */
sj_status sj_part_info(const sj_part* P, int64_t* n_rects, int64_t* n_entries, sj_grid* g);

/* Two-level partition statistics: entries of the coarse (level-1) cells and
 * level-2 chunks of the last sj_partition on P (diagnostics). */
sj_status sj_part_stats(const sj_part* P, int64_t* level1_entries, int64_t* level2_chunks);

/*
 * Copy a partitioned input back to the host (for inspection and tests):
 *   offsets   k*k + 1 int64 (k + 1 with SJ_STRIPES): segment of tile t = ty*k + tx
 *             (stripe t) is [offsets[t], offsets[t+1]).
 *   ids       n_entries int32 rectangle positions, grouped by tile (order
 *             within a tile unspecified).
 * Either pointer may be NULL.  Synchronises the stream.
 */
sj_status sj_part_download(const sj_part* P, int64_t* offsets, int32_t* ids, void* stream);

void sj_part_free(sj_part* P);

const char* sj_status_string(sj_status s);

/* Version string of the library build. */
const char* sj_version(void);

/* Detail of the last failure on the calling thread (HIP error text or the
 * device status word); empty if none.  The string is library-owned. */
const char* sj_last_error(void);

/*
 * Autotuner.  sj_tune times the join of (R, S) -- into `out` (capacity
 * pairs), or count-only if out is NULL -- `reps` times for every candidate
 * schedule: workgroup size of the small-tile kernel (64 = one wavefront per
 * span unit, 128, 256, 512), the entry cap of a small tile (E/4 or E/2 of
 * the unit's LDS slab E), the entry cap of a medium tile (1024, 2048) and,
 * unless the grid fixes it, the split threshold (128, 256, 1024).  The
 * fastest is cached for (device, K, log2 |entries| of R and S, mode) and
 * used by every later sj_join / sj_join_count that matches; best (host, may
 * be NULL) receives it.  The schedule never changes the result.
 * Synchronises the stream.  sj_tune_clear empties the cache.
 */
typedef struct {
    int32_t block;      /* 64, 128, 256 or 512                  */
    int32_t small_cap;  /* tiles with <= small_cap entries are batched */
    int32_t med_cap;    /* tiles with <= med_cap entries: one workgroup each */
    int32_t split_tau;  /* 0 = the grid's                        */
    double ms;          /* mean time of the winning candidate    */
} sj_tuning;

sj_status sj_tune(const sj_part* R, const sj_part* S, sj_pair* out, int64_t capacity,
                  int32_t reps, sj_tuning* best, void* stream);
void sj_tune_clear(void);
/* Put a schedule into the cache for the class of (R, S) (as sj_tune would):
 * block in {64, 128, 256, 512}, caps >= 2; clamped to the kernel's LDS slab. */
sj_status sj_tune_set(const sj_part* R, const sj_part* S, int32_t count_only,
                      const sj_tuning* t);
/* Persist the autotuner cache, so that separate processes (a benchmark and
 * its profiling run) join with the same schedule.  sj_tune_save writes every
 * cached entry as one text line: the device's architecture name (e.g.
 * gfx950), K, log2 |entries| of R and of S, the mode (bit 0 count only,
 * bit 1 distance join, bit 2 SJ_STRIPES, bit 3 SJ_GBDA) and the schedule.  sj_tune_load adds the entries of
 * a file whose architecture name matches the current device (others are
 * skipped) to the cache, replacing entries of the same class; *n_loaded (may
 * be NULL) receives their count.  Errors: SJ_ERR_ARG for a NULL path, a
 * file that cannot be opened or a malformed line (nothing is added then). */
sj_status sj_tune_save(const char* path);
/* The cached schedule for the class of (R, S) in *t (host): SJ_OK if the
 * cache holds one, SJ_ERR_ARG if not (or for NULL arguments). */
sj_status sj_tune_lookup(const sj_part* R, const sj_part* S, int32_t count_only, sj_tuning* t);
sj_status sj_tune_load(const char* path, int32_t* n_loaded);

/*
 * Many independent joins in one replayable launch.  Joins, like tiles, are
 * independent tasks (Sec. 3.4): a batch plans every join once (grid from
 * grids[j], or where its k or split_tau is 0 the picker / rule of
 * sj_choose_grid), sizes its buffers and records one hipGraph: the
 * partitioning sequence once for all 2 n_joins inputs (every launch runs the
 * workgroups of all inputs) and one classification launch for all joins,
 * which appends every join's work units -- span units of small tiles, medium
 * tiles, dense tiles split into pivot ranges -- tagged with the join's index
 * to work lists shared by the batch (a batch holding an input too large for
 * the batched scans runs each join's partitions and classification on a few
 * concurrent streams instead, joins assigned longest-first); then one
 * sequence of join launches whose persistent workgroups take the units of
 * all joins from those lists.  The pairs are staged in scratch chunks that
 * each hold one join's pairs, and a compaction moves every chunk into its
 * join's slice of `out` at a position reserved on the join's counter (pair
 * order within a slice unspecified).  Every join uses the batch's
 * small-tile workgroup shape and default caps, its grid's split threshold
 * and flags; SJ_PLAIN and SJ_TWO_PASS do not apply to batches.
 * sj_batch_run replays it: one graph launch and one status readback for
 * the whole batch.
 *   R[j], S[j]   device rectangle arrays (as sj_partition) of nR[j], nS[j]
 *                rectangles; borrowed for the batch's lifetime (replays
 *                read them again, so their contents may change between runs).
 *   grids        n_joins grids, or NULL (all chosen).  A K the batch
 *                chooses (sj_choose_grid: picker or rule) is further capped
 *                at floor(sqrt((nR + nS) / 4)) on a 2-D grid: inside one
 *                replay a join's per-tile passes are not hidden behind call
 *                overhead (of the caps 8N ... N/32 timed on a held-out batch
 *                of 256 joins, N/4 replayed fastest).  A caller's K is kept.
 *                The coarse cells of a batch's two-level partitions are
 *                sized for the join's larger input (about 8192 rectangles
 *                each), so that a small join does not pay for 32 x 32
 *                nearly empty cells.
 *   out          device pair buffer, or NULL for count-only joins; join j
 *                writes [out_offsets[j], out_offsets[j+1]) (host array of
 *                n_joins + 1).  Borrowed like the inputs.
 *   n_pairs      host, n_joins: |J_j| of every join.
 * Creation runs the batch once (capacities are checked on the device and
 * grown as needed) before recording.  A run returns SJ_ERR_CAPACITY if some
 * join's pairs exceed its slice (its n_pairs is still exact).  When a join
 * outgrows its buffers on a later run (new data), its buffers and the shared
 * lists grow, the batch runs again and the graph is recorded again.
 * Synchronises `stream` once.
 */
typedef struct sj_batch sj_batch;

sj_status sj_batch_create(int32_t n_joins, const float* const* R, const int64_t* nR,
                          const float* const* S, const int64_t* nS, const sj_grid* grids,
                          sj_pair* out, const int64_t* out_offsets, sj_batch** batch,
                          void* stream);
sj_status sj_batch_run(sj_batch* batch, int64_t* n_pairs, void* stream);
/* The grid of every join (k and split_tau; 0 = library default). */
sj_status sj_batch_info(const sj_batch* batch, int32_t* k, int32_t* split_tau);
/* One run of the batch without the recorded graph: the same kernels,
 * launched one by one (so that per-kernel timers see them), with the same
 * results and status as sj_batch_run. */
sj_status sj_batch_run_eager(sj_batch* batch, int64_t* n_pairs, void* stream);
/* Entries of every partition of the last run (host arrays of 2 n_joins, the
 * R sides then the S sides, either may be NULL): m1 coarse-cell entries,
 * m tile entries (each rectangle counted once per tile it meets). */
sj_status sj_batch_entries(const sj_batch* batch, int64_t* m1, int64_t* m);
/* Work statistics of the batch's last run, summed over its joins (fields as
 * sj_last_join_stats; pairs_* per work class).  Synchronises the device.
 * Declared with sj_join_stats below. */
void sj_batch_free(sj_batch* batch);
/* One-shot: create (which runs every join), report, free. */
sj_status sj_batch_join(int32_t n_joins, const float* const* R, const int64_t* nR,
                        const float* const* S, const int64_t* nS, const sj_grid* grids,
                        sj_pair* out, const int64_t* out_offsets, int64_t* n_pairs, void* stream);

/*
 * Work statistics of the last sj_join / sj_join_count on the calling thread's
 * current device (diagnostics; synchronises the device).  Tiles with both
 * lists non-empty are classed by entries n = |R_T| + |S_T|: small (batched
 * into LDS units), medium (one workgroup each) and dense (sorted in global
 * memory, swept in pivot ranges).  The plain schedule classifies no tiles
 * (its per-tile fields are 0).  pairs_* are -1 unless single_pass.
 * small_cap and med_cap are the class bounds used (small: n <= small_cap,
 * medium: n <= med_cap).  axis_tiles counts the tiles that evaluated the
 * sweeping-axis model (the medium and dense ones, unless SJ_SWEEP_X, the
 * plain schedule or stripes), axis_y those of them swept along y.
 */
typedef struct {
    int64_t n_pairs;
    int64_t small_tiles, small_units, medium_tiles, dense_tiles, dense_units;
    int64_t small_entries, medium_entries, dense_entries;
    int64_t pairs_small, pairs_medium, pairs_dense;
    int32_t single_pass;
    int32_t small_cap, med_cap;
    int64_t axis_tiles, axis_y;
} sj_join_stats;

sj_status sj_last_join_stats(sj_join_stats* out);
sj_status sj_batch_stats(const sj_batch* batch, sj_join_stats* out);

/*
 * Canonical order of a result set (Sec. 1 defines J as a set; this gives it
 * one reproducible order): sorts pairs[0..n) in place by (r, s),
 * lexicographically, with a device radix sort of the 64-bit keys
 * (r << 32) | s over the digits that r < n_r and s < n_s can set.
 *   pairs     device, n sj_pair, 8-byte aligned; every r in [0, n_r) and
 *             every s in [0, n_s) (the caller's input sizes), else the
 *             order is unspecified.
 *   n         < 2^32 (else SJ_ERR_TOO_LARGE).
 * Enqueued on the stream (no synchronisation); a library-owned buffer of n
 * pairs is kept per device.  Stable, so equal pairs keep their order.
 */
sj_status sj_sort_pairs(sj_pair* pairs, int64_t n, int64_t n_r, int64_t n_s, void* stream);

/* Most pairs sj_sort_pairs_noalloc sorts (its fixed work buffer: 8 bytes per
 * pair plus the digit histograms, about 33 MiB per GPU). */
#define SJ_SORT_NOALLOC_MAX 4194304

/*
 * For callers that cannot allocate device memory (code recorded into a HIP
 * graph, tight serving loops, harnesses that forbid allocation): the same
 * sort as sj_sort_pairs, same arguments, result and order, with no hipMalloc,
 * hipFree or other allocating call.  Its work buffers live in one fixed
 * device array per GPU (about 33 MiB), held from the first call on that GPU
 * until the process ends.
 *   n         <= SJ_SORT_NOALLOC_MAX, else SJ_ERR_TOO_LARGE (nothing is
 *             enqueued; sj_last_error names the limit).
 * Enqueued on the stream (no synchronisation).  Every call on one GPU uses
 * the same array and keeps the last call's contents, so calls that overlap
 * on one GPU -- on different streams, or from different threads -- race and
 * must be ordered by the caller.  It does not share buffers with
 * sj_sort_pairs.
 */
sj_status sj_sort_pairs_noalloc(sj_pair* pairs, int64_t n, int64_t n_r, int64_t n_s,
                                void* stream);

/*
 * The sweeping-axis model of Sec. 3.3 for chosen tiles of two partitioned
 * inputs (the join evaluates the same model on its medium and dense tiles).
 * Per axis, the tile is cut into k divisions and I = sum_i H_R[i] * H_S[i]
 * (Eq. (2)) over histograms of the sampled rectangles meeting each division;
 * the sweep runs along y when I^y < I^x.  Sample: the rectangles whose input
 * index is a multiple of 100.  k: clamp(floor(tile extent / mean extent of
 * the tile's sampled rectangles), 1, 1000), the mean of (w + h) / 2 in cell
 * units with w, h clipped to 2 cells and summed in fixed point (2^-30).
 * Division of v in tile column t: clamp(floor(fl(fl(u - t) * k)), 0, k-1),
 * u = fl(fl(v - x0) * sx) the float32 cell coordinate.  A tile whose sample
 * misses R or S reports k = 0, I^x = I^y = 0 and axis x.
 *   R, S     partitions on the same 2-D grid (not SJ_STRIPES), else
 *            SJ_ERR_GRID_MISMATCH / SJ_ERR_ARG.
 *   tiles    host, n x (tx, ty) int32 with 0 <= tx, ty < k, else SJ_ERR_ARG.
 *   out      host, n x (k, I^x, I^y, axis) int64; axis 1 = y.
 * Synchronises the stream.
 */
sj_status sj_sweep_axis(const sj_part* R, const sj_part* S, const int32_t* tiles, int64_t n,
                        int64_t* out, void* stream);

/*
 * Choosing the grid (statistics rule of Sec. 4.3.1 / 4.3.3, or the learned
 * picker).  The chosen K and split threshold never change the join result.
 *
 * Features of an instance, SJ_FEAT_DIM float32 (R's block, then S's):
 *   [0] log2(n + 1); [1], [2] log2(mean w + 1e-9), log2(mean h + 1e-9);
 *   [3], [4] log2(std w + 1e-9), log2(std h + 1e-9)  (w, h in domain units);
 *   [5 + 32*cy + cx] log2(1 + 1024 * share of the sampled rectangle centres
 *   in cell (cx, cy) of a 32 x 32 grid over the domain), sampling every
 *   100th rectangle.  Moments cover every rectangle (float64, fixed order).
 */
#define SJ_FEAT_SIDE 1029
#define SJ_FEAT_DIM (2 * SJ_FEAT_SIDE)

typedef struct {
    double mean_extent;    /* e: mean over R and S of (w + h) / 2, domain units */
    int32_t k_rule;        /* clamp(round(1 / (10 e)), 1, SJ_K_MAX)              */
    int32_t k_learned;     /* the picker's K (0 if not used)                     */
    int32_t tau_learned;   /* the picker's split threshold (0 if not used)       */
    int32_t used_learned;  /* 1 if the picker chose                              */
    double mean_x_extent;  /* mean over R and S of w (the 1-D rule's statistic)  */
    int32_t k_cap;         /* largest K chosen for a 2-D grid: floor(sqrt(8 (nR + nS)))
                              clamped to [1, SJ_K_MAX]; SJ_K_MAX with SJ_STRIPES     */
} sj_choice;

/* The rule's K for a mean extent e (domain units): clamp(round(1/(10 e)),
 * 1, SJ_K_MAX); e == 0 gives SJ_K_MAX.  Pure host function. */
int32_t sj_rule_k(double mean_extent);

/*
 * Features of (R, S) (layout above) into `feat` (device, SJ_FEAT_DIM
 * float32) and, if mean_extent != NULL, the rule's e to the host.  The
 * domain is g's (g may be NULL: the unit square).  Synchronises the stream
 * once.  SJ_ERR_RECT if a rectangle is invalid.
 */
sj_status sj_features(const float* R, int64_t nR, const float* S, int64_t nS, const sj_grid* g,
                      float* feat, double* mean_extent, void* stream);

/*
 * Fill in g->k when it is 0 and g->split_tau when it is 0: with the loaded
 * picker unless g->flags has SJ_RULE_ONLY, else with the rule (the split
 * threshold then stays 0 = library default).  Non-zero fields are kept.
 * A chosen 2-D K is at most k_cap = floor(sqrt(8 (nR + nS))): the per-tile
 * arrays cost O(K^2) whatever the input size.
 * With SJ_STRIPES the rule is the 1-D one, k = clamp(round(1 / (10 e_x)),
 * 1, SJ_K_MAX) from the mean x-extent e_x, and the picker is not used.
 * info (host, may be NULL) receives the statistics and both choices.
 * Computes the features on the device and synchronises the stream once.
 */
sj_status sj_choose_grid(const float* R, int64_t nR, const float* S, int64_t nS, sj_grid* g,
                         sj_choice* info, void* stream);

/*
 * Learned picker for the calling thread's current device.  blob (host) =
 * mu[SJ_FEAT_DIM] | sd[SJ_FEAT_DIM] | ystat[4] | params[sj_mlp_param_count(
 * SJ_FEAT_DIM)]: feature standardisation, target standardisation (mean of
 * log2 K, mean of log2 tau, their standard deviations) and the network.
 * Copied to device memory; n must be the blob's exact length, else
 * SJ_ERR_ARG.
 */
sj_status sj_picker_load(const float* blob, int64_t n);
void sj_picker_unload(void);
int32_t sj_picker_loaded(void);

/*
 * The picker's network: a 2 x 64 FP32 MLP, y = W3 relu(W2 relu(W1 xn + b1)
 * + b2) + b3 with xn = (x - mu) / sd (mu, sd may be NULL: identity) and two
 * outputs.  Parameters: one flat device array [W1 (64 x d_in, row-major),
 * b1 (64), W2 (64 x 64), b2 (64), W3 (2 x 64), b3 (2)]; all buffers below
 * are device float32, row-major per sample.  Reductions run in a fixed
 * order, so results are deterministic.
 */
int64_t sj_mlp_param_count(int32_t d_in); /* -1 unless 1 <= d_in <= 4096 */

/* Y[batch x 2]; act (may be NULL) receives [h1 (64), h2 (64)] per sample
 * for sj_mlp_backward. */
sj_status sj_mlp_forward(const float* params, int32_t d_in, const float* mu, const float* sd,
                         const float* X, int32_t batch, float* Y, float* act, void* stream);

/* Mean squared error L = 1/(2 batch) sum (Y - T)^2 into *loss (device, may
 * be NULL) and dY = (Y - T) / batch. */
sj_status sj_mlp_loss(const float* Y, const float* T, int32_t batch, float* dY, float* loss,
                      void* stream);

/* Gradient of the loss w.r.t. every parameter into grad (param count);
 * dact is batch x 128 scratch. */
sj_status sj_mlp_backward(const float* params, int32_t d_in, const float* mu, const float* sd,
                          const float* X, int32_t batch, const float* act, const float* dY,
                          float* dact, float* grad, void* stream);

/* One Adam step (Kingma and Ba 2015, bias-corrected; step >= 1) on n
 * parameters with moment buffers m, v. */
sj_status sj_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t n, float lr,
                      float beta1, float beta2, float eps, int32_t step, void* stream);

/*
 * Synthetic instance generator on the device (the learned picker's training
 * corpus and the many-join batch).  Counter-based Philox4x32-10 (Salmon et
 * al., SC 2011) keyed by `seed`; `side` separates the streams of R and S.
 * Rectangle i: with probability `background` (or when k == 0) a centre
 * uniform in [0,1)^2, else mu_c + sigma_c * N(0, I) of a cluster c drawn by
 * inverse CDF over cumw (redrawn while outside [0,1)^2, at most 64 times,
 * then uniform).  Extents: ext_mode 0 = log-normal with median ext_a and
 * log-sd ext_b; 1 = uniform in [0, ext_a].  Box = centre -/+ extent / 2.
 *   rects       n x 4 float32, device, 16-byte aligned (output).
 *   mu, sigma   k x 2 and k float32 cluster means / deviations, device.
 *   cumw        k float32 cumulative weights (cumw[k-1] = 1), device.
 */
sj_status sj_generate(float* rects, int64_t n, const float* mu, const float* sigma,
                      const float* cumw, int32_t k, float background, int32_t ext_mode,
                      float ext_a, float ext_b, uint64_t seed, uint32_t side, void* stream);

/*
 * Epsilon-distance join of two point sets (Sec. 1: a distance join between
 * point sets reduces to the intersection join of squares of side eps around
 * the points, followed by a distance check).  Here each square is anchored
 * at its point (the point is its lower-left corner), and the join checks
 * the distance of every pair the filter passes as it finds it.
 *
 * Result: every (i, j) with dx*dx + dy*dy <= eps*eps, where dx = P[i].x -
 * Q[j].x and dy = P[i].y - Q[j].y, evaluated in float64 from the float32
 * values with each operation rounded once (no fused multiply-add).  The set
 * does not depend on the grid or schedule; its order is unspecified.
 *
 *   P, Q       nP x 2 and nQ x 2 float32 points (x, y), device, 8-byte
 *              aligned; every coordinate finite (else SJ_ERR_RECT).
 *   eps        finite, >= 0 (else SJ_ERR_ARG).
 *   g          in/out grid for the squares: when g->k is 0, k and split_tau
 *              are chosen as by sj_choose_grid on the squares and written
 *              back; domain and flags (SJ_PLAIN, SJ_TWO_PASS, SJ_STRIPES,
 *              SJ_RULE_ONLY) apply as for rectangles.
 *   out        capacity sj_pair slots (device, caller-owned), or NULL with
 *              capacity 0: count only, nothing written, SJ_OK.
 *   n_pairs    (host) the number of result pairs.  If out is not NULL and
 *              the count exceeds capacity the call returns SJ_ERR_CAPACITY
 *              and the first capacity slots hold an unspecified subset.
 *              SJ_SORTED_OUTPUT in g->flags: sorted by (i, j) as sj_join.
 * The squares (the side widened by a relative 2^-44 so that rounding cannot
 * lose a pair) and their partitions live in library-owned device buffers
 * that are reused and grown across calls.  Synchronises the stream.  Size
 * limits as for rectangles.
 */
sj_status sj_distance_join(const float* P, int64_t nP, const float* Q, int64_t nQ, float eps,
                           sj_grid* g, sj_pair* out, int64_t capacity, int64_t* n_pairs,
                           void* stream);

/*
 * Autotune the join schedule of an epsilon-distance join (as sj_tune does for
 * two partitions): builds the squares, the grid (when g->k is 0; written
 * back) and the partitions as sj_distance_join does, then times every
 * candidate schedule on them with the full pair output and caches the
 * fastest for that grid and size class, so that later sj_distance_join calls
 * on the same inputs use it.  best (host, may be NULL) receives it.
 * Arguments as for sj_distance_join; reps >= 1.  Synchronises the stream.
 */
sj_status sj_distance_tune(const float* P, int64_t nP, const float* Q, int64_t nQ, float eps,
                           sj_grid* g, int32_t reps, sj_tuning* best, void* stream);

/* Work of the last sj_distance_join on the calling thread's current device
 * (all zero before the first): the pairs the filter passed to the distance
 * check (squares that meet, each pair once) and the tile entries of the two
 * partitions of squares
 * (final and first-level, as sj_part_info and sj_part_stats report them). */
typedef struct {
    int64_t candidates;
    int64_t entries_p, entries_q;
    int64_t level1_entries_p, level1_entries_q;
} sj_distance_info;

sj_status sj_distance_last_info(sj_distance_info* info);

/*
 * Opt-in per-kernel timer (tracing).  sj_prof_enable(1) clears the totals and
 * brackets every subsequent kernel launch of the library with a pair of HIP
 * events on the launch's stream; sj_prof_enable(0) stops it.  sj_prof_collect
 * waits for the recorded events, adds their elapsed times to per-kernel
 * totals and returns the number of kernels with totals; entry i is read with
 * sj_prof_name (library-owned string), sj_prof_total_ms and sj_prof_calls.
 */
void sj_prof_enable(int on);
int sj_prof_collect(void);
const char* sj_prof_name(int i);
double sj_prof_total_ms(int i);
int64_t sj_prof_calls(int i);

#ifdef __cplusplus
}
#endif

#endif /* SJ_H */
