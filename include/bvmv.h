/*
 * bvmv: binary adjacency-matrix x vector products computed directly on a
 * Boldi-Vigna-style compressed graph, and the PageRank power method driven by
 * them, on AMD Instinct MI355X (gfx950).
 *
 * The operation (Francisco, Gagie, Ladra, Navarro, "Exploiting
 * Computation-Friendly Graph Compression Methods for Adjacency-Matrix
 * Multiplication", arXiv 1708.07271):
 *   - A is the n x n binary adjacency matrix, row i = the list L_i of node i;
 *     y = A x^T, y_i = sum_{j in L_i} x_j (Section "Introduction").
 *   - Row i is stored against a reference row r_i < i within a window W
 *     (Section "Our Approach"); with A' = rows v_i - v_{r_i} and
 *     w_i = v_{r_i} . x^T, A x^T = A' x^T + w^T (the Proposition), so
 *     y_i = y_{r_i} + sum_j A'_ij x_j reuses the reference row's sum.
 *   - PageRank: p_t = a p_0 + (1 - a) p_{t-1} M, M = D^{-1} A (Section
 *     "PageRank", Eq. (1)); the left product is taken as a right product with
 *     the transposed matrix (Section "Experimental Evaluation").
 *
 * Conventions for every entry point:
 *   - Vectors passed as `const void*` / `void*` are DEVICE pointers owned by
 *     the caller, of the element type the precision selects (double for
 *     BVMV_F64, float otherwise), contiguous unless a leading dimension is
 *     given.  Multi-vector arguments are column-major: element (v, c) of an
 *     n x k block lives at c * ld + v, so each right-hand side is one
 *     contiguous vector.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue work
 *     on it and return without synchronising, except where stated.
 *   - Return value: a bvmv_status.  On a negative status the outputs are
 *     unspecified and bvmv_last_error() returns a message (thread-local).
 *     No exception crosses this interface.
 *   - The library owns every handle it returns until the matching free call.
 */
#ifndef BVMV_H
#define BVMV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bvmv_graph bvmv_graph;
typedef struct bvmv_csr bvmv_csr;

typedef enum {
  BVMV_OK = 0,
  BVMV_NOT_CONVERGED = 1,   /* PageRank hit max_iter; outputs are still written */
  BVMV_EINVAL = -1,         /* bad argument (null pointer, size, option out of range) */
  BVMV_EFORMAT = -2,        /* malformed or truncated bitstream */
  BVMV_ENOMEM = -3,         /* host or device allocation failed, or over the memory budget */
  BVMV_EDEVICE = -4         /* HIP runtime error */
} bvmv_status;

typedef enum {
  BVMV_F64 = 0,       /* double vectors, double accumulation */
  BVMV_F32 = 1,       /* float vectors, float accumulation along reuse chains */
  BVMV_F32_COMP = 2   /* float vectors, two-sum compensated (hi, lo) accumulation */
} bvmv_prec;

/* Layout and tuning options of bvmv_load.  Zero fields take defaults. */
typedef struct {
  int device;            /* HIP device ordinal */
  int tile_rows;         /* rows per tile (one wavefront each, up to 2 rows a lane): 8..128 (0 = 64) */
  int window_cap;        /* max x-window columns staged in LDS per tile: 64..8191 (0 = 256).  A block
                            holds four tiles' windows at 16 bytes a column plus about 2 KiB a tile,
                            so a layout whose widest window does not fit the device's LDS per block
                            is refused at load with BVMV_EINVAL (160 KiB: about 2400 columns) */
  int stage_bytes;       /* max entry-stream bytes of one tile; a new tile starts before a tile's
                            streams would exceed it: 512..16384 (0 = 4096) */
  int long_row_bytes;    /* rows whose entries would take more stream bytes than this are summed by
                            the whole wave from their own array (0 = stage_bytes/2) */
  int interval_mode;     /* 0 = interval sums from a per-tile prefix of x, P[s+len] - P[s] (default);
                            1 = intervals summed entry by entry from the staged x window */
  int autotune;          /* 1 = build and time candidate layouts at load (tile_rows, window_cap and
                            stage_bytes among six settings, FP32 two-sum product, 20 launches
                            each) and keep the fastest; the choice is remembered for the rest
                            of the process per size bucket (floor(log2 n), mean degree).  The
                            options' tile_rows, window_cap, stage_bytes, long_row_bytes are then
                            ignored.  The decoded lists stay on the host (as with keep_lists,
                            without the export), so that bvmv_group can lay the graph out again */
  int keep_lists;        /* 1 = keep the decoded lists on the host (export, CSR baseline) */
  int nthreads;          /* host decode / layout threads (0 = hardware concurrency, max 16) */
  uint64_t device_mem_budget;  /* bytes; 0 = unlimited.  Layout larger than this -> BVMV_ENOMEM */
} bvmv_load_opts;

/* Decode a bitstream and build the device layout.
 * bitstream: HOST pointer to nbytes bytes in the project's BV-style format
 *   (list referencing within a window, copy/skip blocks, intervals,
 *   gap-coded residuals; Section "Our Approach").  Copied; the caller may
 *   free it on return.
 * opts: may be NULL (defaults).  out: receives the handle.
 * Errors: BVMV_EFORMAT for a malformed stream, BVMV_EINVAL for bad options,
 *   BVMV_ENOMEM, BVMV_EDEVICE.  Synchronous. */
int bvmv_load(const void* bitstream, size_t nbytes, const bvmv_load_opts* opts, bvmv_graph** out);

/* y = A x (Section "Our Approach": y_i = y_{r_i} + sum_j A'_ij x_j, plus
 * interval sums and residual entries).  x, y: device vectors of n elements
 * (double for BVMV_F64, float otherwise); overlapping x and y give
 * BVMV_EINVAL.  Deterministic: the same inputs give bit-identical y.
 * Accuracy, per entry, relative to the exactly rounded sum: BVMV_F64 1e-12;
 * BVMV_F32_COMP 1e-5 (the FP32 bar); BVMV_F32 is an uncompensated mode that
 * does NOT meet 1e-5: its error grows with the reference-chain depth and the
 * magnitude of the window's prefix sums (tested to 1e-3). */
int bvmv_multiply(bvmv_graph* g, const void* x, void* y, int prec, void* stream);

/* y = x A, the left product (Section "PageRank" multiplies the row vector
 * p by M), computed on the loaded rows without the transposed graph: with
 * R the references (R_ik = 1 iff r_i = k), A = (I - R)^{-1} A', so
 * x A = c A' with c_k = x_k + the sum of c_i over the rows i that reference
 * k (Proposition of Section "Our Approach", read backwards).  Per tile, c
 * is resolved level by level from the deepest, A' is read column-wise
 * (interval entries as a difference array over the window), and each tile
 * writes its window's contribution; a second launch sums, for every column,
 * the contributions of the tiles whose window covers it and the entries
 * outside the windows, in a fixed order.  x, y: device vectors of n
 * elements (double for BVMV_F64, float otherwise), not overlapping.
 * Deterministic.  A single graph (not a group).  The first call builds the
 * column-wise layout (host work and device allocations, kept with the
 * graph); products on one graph must not overlap in time (they share its
 * buffers). */
int bvmv_multiply_left(bvmv_graph* g, const void* x, void* y, int prec, void* stream);

/* Y = A X for k right-hand sides at once (the product of the Proposition of
 * Section "Our Approach" applied to each column; Section "PageRank" needs one
 * per personalized start vector p_0): every tile of the layout is decoded
 * once and multiplies the k columns one after another.  X, Y: column-major
 * n x k blocks with leading dimension ld >= n (elements).  1 <= k <= 64.
 * prec: BVMV_F32 or BVMV_F32_COMP (float) or BVMV_F64 (double).  Column c of
 * Y is bit-identical to bvmv_multiply of column c of X.  Overlapping blocks
 * give BVMV_EINVAL. */
int bvmv_multiply_batch(bvmv_graph* g, const void* X, void* Y, int k, int64_t ld, int prec, void* stream);

typedef struct bvmv_mlp bvmv_mlp;  /* the warm-restart network (declared with its entry points below) */

/* PageRank options.  damping = beta, the weight of following links (the
 * paper's teleport probability a is 1 - beta).  Iteration stops at the first
 * t with ||p_t - p_{t-1}||_1 < tol (accumulated in double), or at max_iter. */
typedef struct {
  double damping;   /* 0 <= damping < 1.  0 means the default 0.85 unless exact_zero_damping = 1,
                       which takes damping = 0 literally (then p = teleport after one step) */
  double tol;       /* > 0 (0 = default 1e-6) */
  int max_iter;     /* > 0 (0 = default 1000) */
  int prec;         /* BVMV_F32_COMP (default), BVMV_F32 or BVMV_F64 */
  int chunk;        /* iterations per captured HIP graph replay (0 = default 16) */
  int exact_zero_damping;  /* 1 = use damping exactly as given, even 0 */
  int fallback_check;      /* 1 (k = 1, single graph, start given): run one iteration from
                              `start` and one from the teleport vector, and keep `start` only
                              if its residual is the smaller; the probes are not counted */
  const bvmv_mlp* mlp;     /* non-NULL: learned warm restarts with this network (k = 1, uniform
                              teleport, no start vector; a single graph or a group whose
                              members share R; see the learned section below) */
  int restart_every;       /* K >= 3: a restart after every K iterations (0 = default 10) */
  int max_restarts;        /* restarts to try (0 = default 2); the first rejected one ends them */
} bvmv_pr_opts;

typedef struct {
  int iters;          /* iterations run (the t at which the stopping test held); an accepted
                         restart's probe iteration is one of them */
  int converged;      /* 1 if residual < tol */
  double residual;    /* ||p_t - p_{t-1}||_1 of the last iteration */
  int used_start;     /* 1: started from `start`; 0: from the teleport vector (no start, or
                         the fallback check rejected it) */
  int products;       /* matrix products run: iters + rejected restart probes */
  int restarts_accepted, restarts_rejected;
} bvmv_pr_result;

/* PageRank by the power method, Eq. (1), on the loaded rows read as IN-LINK
 * lists: row v lists every u with an edge u -> v (the transposed matrix, as
 * the paper does), so the out-degree d_u is the number of rows listing u.
 * Per iteration: delta = sum of p_u over d_u = 0 (double); z_u = p_u / d_u;
 * y = B z (the compressed product); p'_v = (1-beta) v_v + beta (y_v + delta v_v);
 * residual = ||p' - p||_1 (double).  Dangling mass goes to the teleport vector.
 * teleport: device n x k column-major (ld = n) of the prec's element type, each
 *   column a probability vector; NULL = uniform 1/n for every column (on a
 *   group: each member graph gets its own uniform vector).
 * start: device n x k start vectors; NULL = the teleport vector.
 * p_out: device n x k result.  res: HOST array of k results (for a group:
 *   one per member graph).  k = number of personalized right-hand sides.
 * Synchronises `stream` once per replayed chunk to read the residuals.
 * Returns BVMV_NOT_CONVERGED (with outputs written) if some column did not
 * converge within max_iter. */
int bvmv_pagerank(bvmv_graph* g, const bvmv_pr_opts* opts, const void* teleport, const void* start,
                  void* p_out, int k, bvmv_pr_result* res, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): bvmv_pagerank of
 * a single graph (not a group) for one right-hand side, with the same
 * arguments and results (k = 1), that allocates nothing.  Its working set
 * (the two iterates, their z = p / d, the block partials and the state) lives
 * in a fixed array of BVMV_NOALLOC_SCRATCH_BYTES of device memory that the
 * library holds on every device it runs on until the process ends; the
 * caller passes inputs and outputs as for bvmv_pagerank.
 * Limit: 4 * n * (element size) + 16 * (tiles / 4 + 1) bytes (each part
 * rounded up to 256) plus 256 must fit in the array: n up to about 2^21 in
 * the float modes and 2^20 in BVMV_F64 at the default layout; a larger graph
 * gives BVMV_EINVAL before any device work.  Options: opts->mlp and
 * opts->fallback_check must be 0 (BVMV_EINVAL otherwise).
 * Iterations are launched directly (no captured graph), `chunk` at a time;
 * after each chunk the state is read back with a synchronising copy into host
 * stack memory.  Results are bit-identical to bvmv_pagerank's.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (every word a call reads it has written first): calls that
 * overlap on one GPU (concurrent streams or threads) race and give wrong
 * results; serialise them. */
#define BVMV_NOALLOC_SCRATCH_BYTES (33u << 20)
int bvmv_pagerank_noalloc(bvmv_graph* g, const bvmv_pr_opts* opts, const void* teleport, const void* start,
                          void* p_out, bvmv_pr_result* res, void* stream);

/* Ragged batch: the block-diagonal union of `count` loaded graphs as one
 * handle.  Member i occupies rows/columns [offsets[i], offsets[i+1]).
 * bvmv_multiply on a group multiplies every member at once; bvmv_pagerank
 * runs every member's PageRank (own uniform teleport, own stopping test) in
 * one launch sequence.  The members stay valid and owned by the caller.
 * Members laid out differently (autotuned one by one, or loaded with other
 * options) share one layout in the group when every member still holds its
 * decoded lists (autotune or keep_lists): each of the members' layouts is
 * timed over the whole group (FP32 two-sum product, 10 launches) and the
 * fastest is used for all; a member's rows may then be summed in another
 * order than in its own handle.  Otherwise the members' own layouts are
 * joined as they are. */
int bvmv_group(bvmv_graph* const* graphs, int count, bvmv_graph** out);
/* offsets: HOST array of count+1 row offsets of a group's members. */
int bvmv_group_offsets(const bvmv_graph* group, int64_t* offsets, int* count);

typedef struct {
  int64_t n, m;             /* nodes, edges (nonzeros of A) */
  int64_t m_prime;          /* nonzeros of A' with the paper's fallback rule (keep v_i when
                               |v_i - v_{r_i}| >= |v_i|) and the stream's references */
  int64_t units;            /* work units of the device layout: entries + 1 per reused row */
  int64_t diff_rows, direct_rows, long_rows;
  int64_t escapes;          /* entries outside their tile's x window */
  int64_t ntiles;
  int64_t layout_bytes;     /* device bytes of the layout (tiles, row info, entry streams, long rows) */
  int64_t stream_bytes;     /* size of the input bitstream */
  int64_t n_singles, n_wide, n_intervals;  /* entries of the three per-tile streams */
  int W, R, Lmin, zeta_k;
  int tile_rows, window_cap, stage_bytes, long_row_bytes, interval_mode;
  int max_level;            /* deepest reuse level in the layout (<= R) */
  int ngraphs;              /* 1, or the member count of a group */
  int autotuned;            /* 0: layout from the options; 1: chosen by timing candidate layouts at
                               load (for a group: one of its members' layouts, timed over the
                               whole group); 2: the autotuner's earlier choice for this size
                               bucket */
} bvmv_info;
int bvmv_get_info(const bvmv_graph* g, bvmv_info* out);

/* Decoded lists of a graph loaded with keep_lists = 1, into HOST buffers:
 * rowptr[n+1] (uint64), col[m] (uint32, each row strictly increasing). */
int bvmv_export_csr(const bvmv_graph* g, uint64_t* rowptr, uint32_t* col);

/* deg = A 1 by integer reuse on the device (deg_i = deg_{r_i} - skipped +
 * added entries).  deg: device int32[n]. */
int bvmv_degrees(bvmv_graph* g, int32_t* deg, void* stream);

/* Host-only decode (no device needed).  Call with rowptr = col = refs = NULL
 * to get n and m, then again with buffers of n+1, m and n elements.
 * refs[i] = i - r_i (0 = no reference). */
int bvmv_decode(const void* bitstream, size_t nbytes, int nthreads, uint64_t* rowptr, uint32_t* col,
                uint8_t* refs, int64_t* n, int64_t* m);

/* Plain CSR baseline built the same way (row tiles, LDS-staged column ids,
 * whole-block long rows).  From a graph loaded with keep_lists = 1, or from
 * host CSR arrays (copied; the caller keeps them): rowptr holds n + 1
 * offsets, rowptr[0] = 0 and nondecreasing; col holds rowptr[n] column ids
 * below n, in any order within a row (a repeated id counts twice); col may
 * be NULL when rowptr[n] = 0.  BVMV_EINVAL, before any device work, for
 * n < 1 or n >= 2^32 - 1, a null pointer, offsets that start elsewhere or
 * decrease, or a column id out of range. */
int bvmv_csr_create(const bvmv_graph* g, bvmv_csr** out);
int bvmv_csr_create_host(int64_t n, const uint64_t* rowptr, const uint32_t* col, int device, bvmv_csr** out);
int bvmv_csr_multiply(bvmv_csr* c, const void* x, void* y, int prec, void* stream);
/* PageRank with the CSR product, same semantics as bvmv_pagerank, k = 1. */
int bvmv_csr_pagerank(bvmv_csr* c, const bvmv_pr_opts* opts, const void* teleport, const void* start,
                      void* p_out, bvmv_pr_result* res, void* stream);
int64_t bvmv_csr_bytes(const bvmv_csr* c);
void bvmv_csr_free(bvmv_csr* c);

/* Column blocks (Section "Final Remarks": splitting the matrix into
 * submatrices of consecutive columns, so that a row's reference need not
 * match the whole row).  Each block A_b (rows restricted to a column range)
 * is loaded as a graph of its own with bvmv_load: same n, its own references
 * and tiles.  bvmv_colblocks_multiply computes y = sum_b A_b x: the first
 * block stores y, each later one adds its rows' sums to y (in the vector
 * type, after the block's own accumulation), in block order, so the result
 * is deterministic.  The blocks stay owned by the caller and must outlive the
 * handle.  BVMV_EINVAL for a null pointer, a group, or blocks of different n
 * or device.  Only products are defined on the handle. */
typedef struct bvmv_colblocks bvmv_colblocks;
int bvmv_colblocks_create(bvmv_graph* const* blocks, int count, bvmv_colblocks** out);
int bvmv_colblocks_multiply(bvmv_colblocks* c, const void* x, void* y, int prec, void* stream);
void bvmv_colblocks_free(bvmv_colblocks* c);

/* ---------------------------------------------------------------------------
 * Biclique format (Section "Final Remarks", after Hernandez and Navarro's
 * biclique extraction): the edges of G split into bicliques (S_r, C_r) --
 * every node of S_r points to every node of C_r, |S_r| |C_r| edges stored as
 * the |S_r| + |C_r| ids of the two sets -- plus residual edges.  The product
 * takes c_r = sum_{j in C_r} x_j for every biclique, then
 * y_i = sum_{r : i in S_r} c_r + sum_{j : (i, j) residual} x_j, in time
 * proportional to the stored ids.
 * ------------------------------------------------------------------------- */
typedef struct bvmv_biclique bvmv_biclique;

/* Build the device layout of a biclique decomposition of an n-node graph.
 * All arrays are HOST arrays, copied (the caller keeps them):
 *   sptr[nbic+1], sidx: S_r = sidx[sptr[r] .. sptr[r+1]);
 *   cptr[nbic+1], cidx: C_r = cidx[cptr[r] .. cptr[r+1]);
 *   rptr[n+1], rcol: residual edges (i, j), j in rcol[rptr[i] .. rptr[i+1]).
 * Every set and residual row strictly increasing with ids below n; offsets
 * start at 0 and do not decrease; empty sets are allowed.  The bicliques and
 * the residual must partition the edges (no edge listed twice).
 * Errors: BVMV_EINVAL (null pointers, n < 1, n + nbic >= 2^32 - 1, more than
 * 2^32 - 1 stored ids or edges), BVMV_EFORMAT (unsorted or out-of-range
 * ids, bad offsets, an edge listed twice), BVMV_ENOMEM, BVMV_EDEVICE.
 * Synchronous.  The layout holds a device array of the nbic sums c_r, so
 * products on one handle must not overlap in time (one stream at a time). */
int bvmv_biclique_load(int64_t n, int64_t nbic, const uint64_t* sptr, const uint32_t* sidx, const uint64_t* cptr,
                       const uint32_t* cidx, const uint64_t* rptr, const uint32_t* rcol, int device,
                       bvmv_biclique** out);
/* y = A x on the biclique layout (two launches on `stream`: the sums c_r,
 * then the rows).  x, y: device vectors of n elements (double for BVMV_F64,
 * float otherwise), not overlapping.  Row partials accumulate as in
 * bvmv_multiply (double in BVMV_F64 and BVMV_F32_COMP); c_r is stored in the
 * vector type.  Deterministic. */
int bvmv_biclique_multiply(bvmv_biclique* b, const void* x, void* y, int prec, void* stream);
typedef struct {
  int64_t n, m;         /* nodes, edges of the graph the decomposition represents */
  int64_t nbic;         /* bicliques */
  int64_t s_ids, c_ids; /* stored ids: sum |S_r|, sum |C_r| */
  int64_t residual;     /* residual edges */
  int64_t words;        /* s_ids + c_ids + residual (the paper's compressed size in words) */
  int64_t layout_bytes; /* device bytes of the two passes' ids, offsets and tiles */
} bvmv_biclique_info;
int bvmv_biclique_get_info(const bvmv_biclique* b, bvmv_biclique_info* out);
void bvmv_biclique_free(bvmv_biclique* b);

/* Host interpretation of the device layout that bvmv_load would build from
 * this bitstream and options, in double precision: y = A x with x and y HOST
 * arrays of n doubles.  A test aid for the layout builder (no device
 * needed); no other entry point uses it.  stats (may be NULL) receives 9
 * values: tiles, units, differential rows, direct rows, long rows, escapes,
 * layout bytes, m', deepest level.  BVMV_EINVAL if the layout is
 * inconsistent. */
int bvmv_layout_selfcheck(const void* bitstream, size_t nbytes, const bvmv_load_opts* opts, const double* x,
                          double* y, int64_t* stats);

/* Host interpretation of the left product's column-wise layout
 * (bvmv_multiply_left), in double precision: y = x A with x and y HOST
 * arrays of n doubles.  A test aid (no device needed); BVMV_EINVAL if the
 * layout is inconsistent. */
int bvmv_left_selfcheck(const void* bitstream, size_t nbytes, const bvmv_load_opts* opts, const double* x,
                        double* y);

/* ---------------------------------------------------------------------------
 * Learned PageRank warm restarts (not in the paper; its PageRank starts from
 * the uniform vector, Section "Experimental Evaluation").  Every K iterations
 * of Eq. (1) a small MLP maps 12 inputs per node v to s_v, its estimate of
 * the remaining correction t_v = n (p*_v - p_K(v)) / delta in units of the
 * last step, delta = ||p_K - p_{K-1}||_1; the restart vector is
 * p'_v = max(p_K(v) + s_v delta / n, p_K(v) / 1000) / sum.  One iteration from
 * p' gives its residual r'; p' is kept only if r' < damping * delta (the L1
 * contraction bounds the plain method's next residual by damping * delta),
 * otherwise the run goes on from p_K and no further restart is tried.  The
 * fixed point does not depend on the restarts: the stopping test and its
 * error bound are the plain method's.
 * On a group every member is restarted at the same phase boundary, and only
 * while every member is still iterating; each member keeps or rejects its
 * restart by its own probe (a rejecting member goes on from its p_K with the
 * state it had), and after any rejection no member is restarted again.  With
 * one restart (max_restarts = 1) each member's result is bit-identical to
 * its run alone.
 * Inputs of node v (rows read as in-link lists):
 *   0 log1p(in-degree)   1 log1p(out-degree d)   2 reference-chain depth / R
 *   3 [d = 0]   4 log1p(intervals of the row)   5 log1p(residuals of the row)
 *   6 log1p(mean out-degree of the in-neighbours)
 *   7 log1p(mean in-degree of the in-neighbours)
 *   8 log(n p_K)   9 n (p_K - p_{K-1}) / delta   10 n (p_{K-1} - p_{K-2}) / delta
 *   11 n (p_{K-2} - p_{K-3}) / delta
 * ------------------------------------------------------------------------- */
/* Input rows F (device, n x 12 node-major FP32) must start on a 16-byte
 * boundary: the kernels move each row's inputs as 16-byte vectors.  A
 * misaligned F gives BVMV_EINVAL. */
#define BVMV_NFEAT 12        /* inputs per node */
#define BVMV_MLP_PARAMS 5057 /* W1 (64x12), b1 (64), W2 (64x64), b2 (64), w3 (64), b3 (1), row-major (out, in) */

/* The structural inputs 0..7 of every node into columns 0..7 of F (device,
 * n x 12 node-major FP32); columns 8..11 are left as they are.  Uses the
 * degree pass and two products; uploads the row coding statistics once per
 * graph.  Single graph only.  Synchronous. */
int bvmv_features(bvmv_graph* g, float* F, void* stream);

/* A training sample of g: K >= 3 plain iterations from the uniform vector
 * (prec as for bvmv_pagerank), then all 12 inputs into F (device n x 12) and,
 * if p_star (device, n of the prec's type) is given, the target
 * t = n (p_star - p_K) / delta into T (device n floats).  delta: HOST double
 * or NULL.  BVMV_EINVAL if the run converges within K iterations (delta would
 * be below tol).  Single graph only.  Synchronous. */
int bvmv_restart_sample(bvmv_graph* g, int K, int prec, const void* p_star, float* F, float* T, double* delta,
                        void* stream);

/* A network on `device` with the given FP32 master parameters (HOST array of
 * BVMV_MLP_PARAMS); weights are used as BF16 copies, biases as FP32; Adam
 * state zero.  Synchronous. */
int bvmv_mlp_create(int device, const float* params, bvmv_mlp** out);
/* HOST copy of the FP32 master parameters.  Synchronous. */
int bvmv_mlp_params(const bvmv_mlp* m, float* params);
/* s = network(F) for n rows: F device n x 12, s device n floats.  GEMM
 * operands BF16 (round to nearest even), FP32 accumulation; biases, GELU and
 * the output layer FP32. */
int bvmv_mlp_forward(bvmv_mlp* m, const float* F, int64_t n, float* s, void* stream);
/* Gradient of the mean squared error (1/n) sum (s_i - target_i)^2 over n <= 2^20
 * rows: grad device, BVMV_MLP_PARAMS + 1 floats (the gradient, then the loss). */
int bvmv_mlp_gradient(bvmv_mlp* m, const float* F, const float* target, int64_t n, float* grad, void* stream);
/* One training step: the gradient on (F, target), then Adam (b1 = 0.9,
 * b2 = 0.999, eps = 1e-8) with learning rate lr.  loss: device float or NULL. */
int bvmv_mlp_train_step(bvmv_mlp* m, const float* F, const float* target, int64_t n, float lr, float* loss,
                        void* stream);
void bvmv_mlp_free(bvmv_mlp* m);

void bvmv_free(bvmv_graph* g);
const char* bvmv_last_error(void);
/* Library version string. */
const char* bvmv_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BVMV_H */
