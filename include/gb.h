/*
 * gb.h -- C ABI of libgb: graph-partitioned SP2 density matrices on one MI355X.
 *
 * The calls follow the paper's statement of the problem (Niklasson et al., "Graph-based
 * linear scaling electronic structure theory"): from a sparse symmetric Hamiltonian H in a
 * local basis, a threshold tau and an occupation n_occ, build the data-dependency graph S
 * (Eq. 2; any graph is allowed, obs. viii), split it into cores with halos (Eq. 6 and
 * obs. vi), expand every subgraph's dense principal submatrix with the same recursive SP2
 * sequence (the zero-temperature expansion after Eq. 7) and assemble the core columns into
 * D (obs. i).
 *
 * Conventions shared by every call
 *   - Matrix and index pointers are DEVICE pointers unless marked (host).
 *   - `stream` is a hipStream_t (NULL = the null stream); every call is ordered on it.
 *   - Return value: GB_OK or a negative gb_status; gb_last_error() then holds a message
 *     (thread-local, valid until the next failing call on the same thread).
 *   - Argument checks (null pointers, sizes, ranges, NaN) run on the host before any device
 *     work and return GB_EINVAL or GB_ESHAPE; HIP failures return GB_EHIP.
 *   - No call keeps a pointer to caller memory after it returns.  Handles (graph, partition)
 *     own their device memory until *_destroy; destroying NULL is a no-op.
 *   - Floating point on the graph, bounds and gather steps is evaluated in a fixed
 *     (canonical) order with separately rounded products and sums, so index results are
 *     reproducible bit for bit on any device and agree with a sequential CPU evaluation.
 */
#ifndef GB_H
#define GB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gb_status;
#define GB_OK 0
#define GB_EINVAL (-1)        /* invalid argument value or null pointer               */
#define GB_ENOMEM (-2)        /* device allocation failed                              */
#define GB_EHIP (-3)          /* a HIP runtime call or kernel launch failed            */
#define GB_ESHAPE (-4)        /* an output array is too small / sizes are inconsistent */
#define GB_EUNSUPPORTED (-5)  /* valid request outside what this build implements      */

/* The dense batch buffers of gb_density / gb_foe_density are cached between calls (per device
 * and per concurrent call, grown when a call needs more), so a loop of calls does not
 * reallocate them; so are the host buffers of the multilevel partitioner (its coarse graphs
 * and the pinned copy of the graph it reads).  gb_trim frees the cached buffers of every call
 * that has returned. */
gb_status gb_trim(void);

/* Kernel-variant table of the autotuner (the tile edge, and for FP64 / FP32 the LDS staging,
 * chosen per 256-wide size bucket of padded subgraph sizes by timing each variant once; see
 * gb_sp2_opts.tile_policy).  gb_tune_save writes the table of this process as JSON to `path`
 * (tagged with the library's source hash and the device: "libgb-tune-1" format); gb_tune_load
 * merges such a file into it, so a later process skips the timing runs.  A file written by
 * another build of the library or on another device, or malformed, is GB_EINVAL and leaves the
 * table unchanged.  With the environment variable GB_TUNE_FILE set, the library reads that
 * file at its first tuning (ignoring it if unusable) and rewrites it after every new entry.
 * n_entries (may be NULL) receives the number of entries written / read.  Host only. */
gb_status gb_tune_save(const char* path, int32_t* n_entries);
gb_status gb_tune_load(const char* path, int32_t* n_entries);

/* Rate this device sustains, measured by the library's own kernels (the measured denominators
 * of the squaring kernels' rooflines, beside the datasheet figures): kind 0 / 1 / 2 / 3 = dense
 * matrix-core TFLOP/s in FP64 (16x16x4), FP32 (16x16x4), bf16 (16x16x32) or fp16 (16x16x32)
 * from eight independent accumulation chains per wave on register operands over 8 workgroups
 * per CU (no memory traffic); kind 5 / 6 = bf16 / fp16 on the 32x32x16 instruction; kind 4 =
 * HBM GB/s (bytes read + written) of a 2 GiB streaming copy.  One warm-up launch, then five timed.  clock_mhz (host, may be NULL) receives the mean
 * core clock of the last MFMA launch's workgroups (core cycles over constant-rate wall-clock
 * ticks; 0 for kind 4): the clock the matrix cores ran at under that load.  GB_EINVAL for an
 * unknown kind or a NULL rate.  Synchronises `stream`. */
gb_status gb_peak_rate(int32_t kind, void* stream, double* rate, double* clock_mhz);

/* Library version string (static storage). */
const char* gb_version(void);
/* Message for the last failing call on this thread ("" if none). */
const char* gb_last_error(void);

/*
 * Device memory hook.  By default every buffer the library needs (handles, batch buffers,
 * scratch) comes from the device's stream-ordered pool (hipMallocAsync / hipFreeAsync, with
 * the pool's release threshold raised so freed memory stays cached).  gb_set_allocator
 * replaces that for every later allocation in the process: alloc(bytes, stream, ctx) returns
 * device memory usable in stream order on `stream` (NULL on failure: the call then fails with
 * GB_ENOMEM), free(ptr, stream, ctx) returns it.  Each buffer is freed through the allocator
 * that made it, so the hook may be changed while handles are alive; it must stay valid (and
 * ctx alive) until every buffer it made is freed.  gb_set_allocator(NULL, NULL, NULL)
 * restores the default; exactly one of alloc/free NULL is GB_EINVAL.  Not thread-safe with
 * respect to concurrent library calls.
 */
typedef void* (*gb_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*gb_free_fn)(void* ptr, void* stream, void* ctx);
gb_status gb_set_allocator(gb_alloc_fn alloc, gb_free_fn free_fn, void* ctx);

/*
 * Row-major ELLPACK matrix: `n` rows, `width` slots per row.  Row i occupies
 * col[i*width .. i*width+width-1] / val[...]: valid entries first with strictly ascending
 * column indices in [0, n), then padding col = -1, val = 0.0.
 * For H (input): symmetric in pattern and value, diagonal entry present in every row.
 * For D (output): COLUMN-ELLPACK -- row i of the arrays holds column i of D (the paper
 * assembles D column by column and D is not symmetric, obs. i): col = global row indices
 * ascending, val = D[row, i].
 */
typedef struct {
  int32_t n;
  int32_t width;
  int32_t* col;
  double* val;
} gb_ell;

/*
 * a1. Gershgorin bounds of H (the SP2 start map X0 = (e_max I - H)/(e_max - e_min) needs a
 * spectral enclosure; the global bounds also enclose every principal submatrix).
 *   e_min = min_i (h_ii - R_i), e_max = max_i (h_ii + R_i), R_i = sum_{j != i} |h_ij| summed
 *   sequentially in ascending column order.  Results written to host doubles.
 * Synchronises `stream`.
 */
gb_status gb_spectral_bounds(const gb_ell* H, void* stream, double* emin, double* emax);
/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): gb_spectral_bounds without any allocation.  The
 * per-workgroup partials and the result live in a fixed device array of the library
 * (3 x 1024 + 3 doubles, 24 KB, held on every GPU the library runs on until the process ends);
 * the call makes no hipMalloc, hipFree or other allocating call.  Rows are grid-strided over at
 * most 1024 workgroups, so any n is accepted and the array never needs more room.  Same
 * e_min / e_max bit for bit as gb_spectral_bounds (min and max are exact).  Every call on one GPU
 * shares that GPU's array (each workgroup writes its own partial before the final pass reads
 * it, so nothing has to start at zero): calls that overlap on one GPU, from several streams or
 * threads, race and must be serialised by the caller.  Synchronises `stream`.  Errors as
 * gb_spectral_bounds (GB_EINVAL for NULL arguments or an H holding NaN or Inf).
 */
gb_status gb_spectral_bounds_noalloc(const gb_ell* H, void* stream, double* emin, double* emax);

/* Graph rules (Eq. 2, Eq. 8, obs. viii).  Every rule adds all self-loops (T^(0) = I puts
 * vertex i in its own subgraph, Eqs. 5-6) and the result is symmetric. */
typedef enum {
  /* S = {(i,j): j two hops from i in pattern(H), |(X0^2)_ij| >= tau}; (X0^2)_ij is summed
   * over k ascending with separate rounding (no fused multiply-add).  aux unused. */
  GB_GRAPH_X2 = 0,
  /* S = {(i,j): |aux_ij| >= tau} (aux = H if NULL); aux symmetric ELL. */
  GB_GRAPH_PATTERN = 1,
  /* Adaptive MD graph: {|Dprev_ij| >= tau_aux} united with X2(H, tau), symmetrised; aux is
   * the previous D in column-ELL form. */
  GB_GRAPH_DPREV = 2,
  /* Eq. 8 with eps = 0: paths of length two in pattern(H) U {|Dprev_ij| >= tau_aux}
   * (symmetrised); tau unused.  Dense in 3D systems: intended for small n. */
  GB_GRAPH_DPREV_SYMBOLIC = 3
} gb_graph_mode;

typedef struct gb_graph_s gb_graph_t;

/*
 * a2. Build the data-dependency graph.  `aux`: see gb_graph_mode.  tau, tau_aux >= 0.
 * On success *out owns a device CSR (row_ptr int32 [n+1], col int32 [nnz], rows sorted
 * ascending, no duplicates).  Synchronises `stream` once (to size the CSR).
 */
gb_status gb_build_graph(const gb_ell* H, const gb_ell* aux, double tau, double tau_aux,
                         int32_t mode, void* stream, gb_graph_t** out);
/*
 * Divide-and-conquer comparison graph (the cutoff-radius halos the paper compares with, Fig. 5):
 * orbital o of site a is vertex a * orbs_per_site + o; (i, j) is an edge iff the minimum-image
 * distance between their sites in the periodic cube of edge `box` is below r_cut (same site
 * included).  Canonical distance, per axis d = x_b - x_a, d = d - box * rint(d / box), then
 * r2 = (dx*dx + dy*dy) + dz*dz, edge iff r2 < r_cut*r_cut.  pos: device [n_sites][3] FP64.
 * Partitioned with gb_partition, its halos are every orbital within r_cut of a core site.
 * GB_EINVAL for n_sites < 1, orbs_per_site < 1, r_cut <= 0 or box < 2 r_cut.  Synchronises once.
 */
gb_status gb_build_graph_rcut(const double* pos, int32_t n_sites, int32_t orbs_per_site,
                              double box, double r_cut, void* stream, gb_graph_t** out);
/* Sizes of a graph (host outputs). */
gb_status gb_graph_info(const gb_graph_t* g, int32_t* n, int64_t* nnz);
/* Copy the CSR into caller device buffers row_ptr [n+1] and col [nnz]. */
gb_status gb_graph_copy(const gb_graph_t* g, int32_t* row_ptr, int32_t* col, void* stream);
/* Device views of the CSR (valid until gb_graph_destroy; the caller must not write them). */
gb_status gb_graph_view(const gb_graph_t* g, int32_t* n, int64_t* nnz, const int32_t** row_ptr,
                        const int32_t** col);
void gb_graph_destroy(gb_graph_t* g);

/* Core selection (obs. vi-vii: a core may be any set of vertices, a "community"). */
typedef enum {
  GB_PART_BLOCK = 0, /* cores = consecutive runs of core_size vertices in vertex order      */
  GB_PART_BFS = 1,   /* the same runs cut from a Cuthill-McKee order of the graph: start at  *
                      * the unvisited vertex of smallest (degree, index), append unvisited   *
                      * neighbours by (degree, index); each core's vertices then ascending   */
  GB_PART_MULTILEVEL = 2 /* communities of at most core_size vertices from a multilevel     *
                      * partitioner (the paper takes its communities from one) aimed at the  *
                      * cost sum_s (|core| + |halo|)^3 and independent of vertex order; see  *
                      * gb_partition_host.  Runs on the host (the graph is copied back).     */
} gb_part_method;

typedef struct gb_partition_s gb_partition_t;

/*
 * a3 + a4. Partition the graph into cores and build every core's subgraph (Eq. 6): the core
 * vertices ascending, then the halo -- every vertex outside the core adjacent to it --
 * ascending.  Synchronises `stream` once (to size the subgraph lists).
 */
gb_status gb_partition(const gb_graph_t* g, int32_t core_size, int32_t method, void* stream,
                       gb_partition_t** out);
/*
 * Host: the cores GB_PART_MULTILEVEL chooses for a host CSR graph (row_ptr [n+1], col [nnz],
 * symmetric; self loops ignored).  Edges are weighted by the number of common closed
 * neighbours of their ends; heavy-edge matching coarsens the graph (pairs up to core_size/4
 * vertices, a fixed pseudo-random visiting order: vertices sorted by SplitMix64 of
 * (level << 32 | v)) until no pair can be matched; parts of at most core_size vertices are
 * grown on the coarsest graph (seeds in breadth-first order, each part taking the unassigned
 * neighbour most strongly tied to it) and projected back to the input graph.  All choices
 * have fixed tie-breaks, so the cores are a function of the graph.  Outputs (host,
 * caller-owned): *n_cores; core_ptr
 * [n_cores + 1] (room for n + 1); core_vtx [n] (each core ascending, cores in ascending order
 * of their smallest vertex); *cost = sum_s (|core| + |halo|)^3 (any of cost may be NULL).
 * GB_EINVAL for NULL arrays, n < 1 or core_size < 1.
 */
gb_status gb_partition_host(int32_t n, const int32_t* row_ptr, const int32_t* col,
                            int32_t core_size, int32_t* n_cores, int32_t* core_ptr,
                            int32_t* core_vtx, int64_t* cost);
/*
 * On-the-fly update (MD): the cores of `prev` (a partition of a graph on the same vertices,
 * e.g. the previous step's) carried to graph g, renumbered as gb_partition_host emits cores,
 * and their subgraphs on g as in gb_partition.  No edge weights or coarsening are computed, so
 * the cost is that of building the halos.  GB_ESHAPE if prev covers a different vertex count.
 */
gb_status gb_partition_update(const gb_graph_t* g, const gb_partition_t* prev, void* stream,
                              gb_partition_t** out);
/* Host form of gb_partition_update on a host CSR graph: prev_core_ptr [prev_n_cores + 1] and
 * prev_core_vtx [n] (every vertex exactly once); outputs as gb_partition_host (the cost on the
 * new graph). */
gb_status gb_partition_update_host(int32_t n, const int32_t* row_ptr, const int32_t* col,
                                   int32_t prev_n_cores, const int32_t* prev_core_ptr,
                                   const int32_t* prev_core_vtx, int32_t* n_cores,
                                   int32_t* core_ptr, int32_t* core_vtx, int64_t* cost);
/* n_sub subgraphs, the largest has max_sub vertices, total = sum of sizes (host outputs). */
gb_status gb_partition_info(const gb_partition_t* p, int32_t* n_sub, int32_t* max_sub,
                            int64_t* total);
/* Copy core_ptr [n_sub+1], sub_ptr [n_sub+1] and sub_idx [total] into caller device buffers
 * (any may be NULL to skip it). */
gb_status gb_partition_copy(const gb_partition_t* p, int32_t* core_ptr, int32_t* sub_ptr,
                            int32_t* sub_idx, void* stream);
/* Device views of core_ptr [n_sub+1], sub_ptr [n_sub+1] and sub_idx [total] (valid until
 * gb_partition_destroy; read-only).  Any output pointer may be NULL. */
gb_status gb_partition_view(const gb_partition_t* p, int32_t* n_sub, int32_t* max_sub,
                            const int32_t** core_ptr, const int32_t** sub_ptr,
                            const int32_t** sub_idx);
void gb_partition_destroy(gb_partition_t* p);

/* Arithmetic of the squaring loop. */
/* Low-precision variants square an FP32 iterate, keep the traces and the branch decision in
 * FP64, stop the low-precision loop when |t1 - t2| <= 1e-5 n / 1024 or when it stops
 * decreasing, and finish with FP64 refinement (McWeeny by default). */
typedef enum {
  GB_FP64 = 0,          /* every square in FP64 on the matrix cores                         */
  GB_FP32_REFINE = 1,   /* squares on FP32 MFMA (FP32 accumulate), then FP64 refinement      */
  GB_BF16_REFINE = 2,   /* squares on BF16 MFMA from one bf16 plane (FP32 accumulate)        */
  GB_BF16X3_REFINE = 3, /* two bf16 planes hi + lo, three products (about 16 bits)           */
  GB_BF16X6_REFINE = 4, /* three bf16 planes, six products (about FP32 precision)            */
  GB_FP16X3_REFINE = 5  /* two fp16 planes of 2^14 X (hi, lo), three products (about 22 bits) */
} gb_precision;

typedef struct {
  int32_t precision;         /* gb_precision; default GB_FP64                                */
  int32_t n_refine;          /* low precision: at most this many FP64 refinement steps       *
                              * (0 = 8 McWeeny steps / 16 SP2 steps)                          */
  int32_t refine_kind;       /* low precision: 0 = McWeeny X <- 3X^2 - 2X^3 on the core rows  *
                              * that D keeps (one or two steps, p or p(p), by products of the *
                              * k core rows with X; 2 n^2 k flops each), accepted if the FP64 *
                              * stop test holds on them, else as 2;                           *
                              * 1 = FP64 SP2 steps until it holds, the first by the trace     *
                              * rule, then alternating X^2 / 2X - X^2 (replayed from          *
                              * branch_in when that extends past the low-precision loop);     *
                              * 2 = McWeeny steps on whole blocks until the stop test holds   */
  int32_t n_fp64_first;      /* low precision: run the first SP2 steps in FP64 (default 0)   */
  int32_t max_iter;          /* default 100 when 0                                           */
  double idem_tol;           /* stop when |Tr X - Tr X^2| <= idem_tol; 0 = 1e-10 * n / 1024   */
  const gb_partition_t* partition; /* NULL: build X2(threshold) + BLOCK(core_size) inside    */
  int32_t core_size;         /* used when partition == NULL; default 32                      */
  const uint8_t* branch_in;  /* (host) replay this branch sequence instead of choosing it    */
  int32_t n_branch_in;       /* at most 127 (the stats record 128 steps)                     */
  double emin, emax;         /* spectral bounds; both 0 = Gershgorin                          */
  int32_t keep_tape;         /* 1: keep SP2 checkpoints for gb_density_vjp (GB_FP64 only)    */
  int32_t tape_stride;       /* checkpoint every tape_stride-th iterate; 0 = 4               */
  int32_t launch_mode;       /* 0 (default): device-driven loop -- one batched squaring     *
                              *    launch per step over every subgraph; the stop flag, step   *
                              *    counter, branch and step records stay on the device, every *
                              *    launch reads the branch there and returns at once after    *
                              *    the stop, so the host enqueues 32 steps (then 8 at a time) *
                              *    without waiting for any decision;                          *
                              * 1: one launch per subgraph per step, decided on the host     *
                              *    (the baseline);                                            *
                              * 2: as 0 with two steps captured in a hipGraph and replayed;   *
                              * 3: batched launches, every decision read back by the host.    *
                              * keep_tape and refine_kind 1 run their steps as in 3.          */
  int32_t tile_policy;       /* kernel variant of the squares: 0 = split squares autotuned   *
                              * per 256-wide size bucket (timed once per process or read from *
                              * the tuning table), FP64 / FP32 squares on policy 5 (the       *
                              * fastest measured in every bucket); 1 = 128-edge tiles, 2 =    *
                              * 64-edge; FP64 / FP32 squares                                   *
                              * also 4 = 64-edge with three LDS stages, 5 = 64-edge with      *
                              * register-staged loads; GB_FP16X3_REFINE also 6 / 7 = 128- /   *
                              * 64-edge tiles with the split under the products (two LDS      *
                              * buffers; bit-identical to 1 / 2).  Values a precision has no   *
                              * kernel for are taken as 0, as 3 is by all.                    */
  int32_t tile_order;        /* 0: each subgraph's tiles on one XCD (L2 reuse); 1: as listed */
  int32_t check_idem;        /* 1: also compute stats.idem_max, max |X^2 - X| over the core   *
                              *    columns (one more square of the core tiles, or nine slab  *
                              *    products after the core-row refinement); 0 (default): the  *
                              *    FP64 trace stop test alone, stats.idem_max = NaN           */
  void* workspace;           /* caller-owned device memory for the batch buffers and X0     *
                              * (256-byte aligned, at least gb_density_workspace bytes; needs *
                              * a partition); NULL: buffers cached by the library (gb_trim)   */
  size_t workspace_bytes;
} gb_sp2_opts;

typedef struct {
  int32_t iters;             /* SP2 updates applied                                          */
  int32_t converged;         /* 1 if the stop rule fired (or the replay ended idempotent)    */
  int32_t n_sub, max_sub;
  uint8_t branch[128];       /* branch of each update: 0 = X^2, 1 = 2X - X^2                  */
  double trace;              /* Tr D (sum of the assembled diagonal)                         */
  double idem;               /* |Tr X - Tr X^2| at the stop                                  */
  double idem_max;           /* max over core columns of |X^2 - X| after the loop            */
  double emin, emax;
  double min_margin;         /* smallest | |t2-n| - |2t1-t2-n| | over chosen branches        */
  double t1[128], t2[128];   /* core traces of X and X^2 at each square                      */
  float ms_bounds, ms_graph, ms_part, ms_gather, ms_sp2, ms_refine, ms_scatter, ms_total;
  float ms_square;           /* summed device time of the FP64 SP2 steps (mode 0, 1)         */
  int32_t n_square;          /* number of FP64 SP2 steps, one fused square+update launch each */
  float ms_square_lo;        /* the same for the low-precision squaring launches             */
  int32_t n_square_lo;
  int32_t n_tile64;          /* subgraphs squared with 64-edge tiles                         */
  int32_t n_refine_done;     /* McWeeny steps applied                                        */
  int32_t planes_db;         /* split loops: 1-3 bf16 planes, 4 = two fp16 planes; 0 otherwise */
  int32_t n_stage3;          /* subgraphs squared with the three-stage 64-edge kernel         */
  int32_t n_regstage;        /* subgraphs squared with the register-staged 64-edge kernel     */
  double square_flops;       /* algorithmic flops of one square launch: sum_s 2 n_s^3        */
  double square_flops_exec;  /* matrix-core flops one launch executes: every active wave's    *
                              * block over the padded size (upper tiles, padding; times the   *
                              * plane products for split squares, applied by the caller)      */
  struct gb_tape_s* tape;    /* with keep_tape: the recorded expansion (free: gb_tape_destroy) */
  int32_t n_near_tie;        /* trace-rule decisions whose margin is within the rounding of   *
                              * the summed traces (64 ulp of |t1| + |t2| + n_occ): another     *
                              * summation order could have taken the other branch             */
  int32_t n_split_il;        /* fp16 split loops: subgraphs squared with the split under the  *
                              * products (tile policies 6 / 7, or the tuner's choice)          */
} gb_sp2_stats;

typedef struct gb_tape_s gb_tape_t;

/*
 * a5-a12. Density matrix D = P_tau(X0) of the partitioned SP2 expansion (Eq. 6 with the SP2
 * recursion), assembled into caller-owned column-ELL D (D->n = H->n, D->width >= max_sub;
 * slots beyond a column's subgraph size are padding).
 *   Loop: square every subgraph block; t1, t2 = sums of the core diagonals of X and X^2 over
 *   all subgraphs (FP64); stop if |t1 - t2| <= idem_tol (D is the current X); otherwise
 *   X <- X^2 if |t2 - n_occ| < |2 t1 - t2 - n_occ|, else X <- 2X - X^2, for every subgraph.
 * Non-convergence is not an error (stats->converged = 0).  stats may be NULL.
 * Synchronisation (launch modes 0 and 2): `stream` is waited for once to read the spectral
 * bounds, once when the squaring loop has stopped (once more per 8 steps beyond the first 32),
 * once after the low-precision refinement check, and at the end; modes 1 and 3 also wait once
 * per SP2 step.  Without a partition the graph and partition steps add one wait each.
 * GB_EINVAL if H holds NaN or Inf (checked on the Gershgorin pass, also with given bounds).
 * GB_ESHAPE if D->width < max_sub (stats->max_sub then holds the needed width), or if the
 * caller's workspace is smaller than gb_density_workspace returns.
 */
gb_status gb_density(const gb_ell* H, int32_t n_occ, double threshold, const gb_sp2_opts* opts,
                     gb_ell* D, gb_sp2_stats* stats, void* stream);

/*
 * Bytes of caller-owned workspace gb_density needs with these options on opts->partition (the
 * dense batch buffers of the partition's subgraphs, padded to multiples of 64, in the loop's
 * precision and FP64, the core-row refinement slabs and X0 on H's pattern; statement of the
 * problem: D from H through the subgraph expansions).  Host only; H's arrays are not read
 * (only H->n and H->width).  GB_EINVAL without a partition.  Handles, the tape and small
 * per-call arrays (offsets, tile lists, partial traces) still come from the allocator.
 */
gb_status gb_density_workspace(const gb_ell* H, const gb_sp2_opts* opts, size_t* bytes);

/*
 * a14. Adjoint of the expansion recorded by gb_density(keep_tape = 1): given dL/dD on D's
 * column-ELL pattern (G_D: n x width with the same layout as the D that call produced; only
 * G_D->val is read), write dL/dH per ELL slot of H into G_H->val.  G_H->col must be H's column
 * array (the pattern is read from it; G_H->width = H's width).  Observables are traces with D
 * (<A> = Tr[D A], SP2 paragraph after Eq. 7); the derivative runs the recursion backwards with
 * the graph, partition, spectral bounds and branch sequence held fixed:
 *   X <- X^2:       Gbar <- Gbar X + X Gbar;      X <- 2X - X^2:  Gbar <- 2 Gbar - (Gbar X + X Gbar)
 * seeded with the symmetric part of dL/dD on each block's core columns, and
 * dL/dh = -Gbar_0 / (e_max - e_min) summed over every subgraph holding both vertices (ascending
 * subgraph order, deterministic).  The result is the symmetric per-slot gradient: perturbing
 * H_ij and H_ji together by h changes L by h (G_ij + G_ji).  Segments between checkpoints are
 * recomputed forward.  Synchronises `stream`.  The tape stays valid until gb_tape_destroy.
 */
gb_status gb_density_vjp(const gb_tape_t* tape, const gb_ell* G_D, gb_ell* G_H, void* stream);
void gb_tape_destroy(gb_tape_t* tape);

/*
 * Finite-temperature density matrix by the Chebyshev Fermi-operator expansion (Eq. 7, with
 * the terms built by the recurrence of Eq. 5 and evaluated per subgraph as in Eq. 6):
 *   D = [exp(beta (H - mu)) + 1]^-1 ~ sum_{n=0..order} c_n T_n(Ht),
 *   Ht = (2H - (e_max + e_min) I)/(e_max - e_min),  T_0 = I, T_1 = Ht,
 *   T_{n+1} = 2 Ht T_n - T_{n-1}, formed as Ht T_n + (Ht T_n)^T - T_{n-1} (one batched FP64
 *   general product per term over every subgraph, then an explicit symmetrisation),
 * c_n by K-node Chebyshev-Gauss quadrature (gb_chebyshev_fermi).  Graph and partition as for
 * gb_density (X2 graph at `threshold` + block cores of core_size unless a partition is given).
 * With mu = NaN the chemical potential is chosen so that the summed core traces
 * sum_n c_n(mu) t_n (t_n = sum over subgraphs of the core diagonal of T_n) equal n_occ
 * (gb_foe_solve_mu); the recurrence then runs twice (traces, then the sum).
 * D as for gb_density (caller-owned column-ELL, D->width >= max_sub).  Synchronises `stream`.
 */
typedef struct {
  double beta;               /* inverse temperature (1 / energy unit of H), > 0               */
  double mu;                 /* chemical potential, or NaN: solved for n_occ                   */
  int32_t order;             /* highest Chebyshev degree M >= 1                                */
  int32_t n_nodes;           /* quadrature nodes K for the coefficients; 0 = max(4(M+1), 1024) */
  const gb_partition_t* partition; /* NULL: build X2(threshold) + BLOCK(core_size) inside      */
  int32_t core_size;         /* used when partition == NULL; default 32                       */
  double emin, emax;         /* spectral bounds; both 0 = Gershgorin                           */
  int32_t tile_policy;       /* accepted for symmetry with gb_sp2_opts; the general product    *
                              * always uses 128-edge tiles                                     */
  int32_t tile_order;        /* as in gb_sp2_opts                                              */
  double* traces;            /* (host) NULL, or order + 1 doubles receiving the summed core    *
                              * traces t_n (reuse them with gb_foe_solve_mu for other n_occ)  */
} gb_foe_opts;

typedef struct {
  double mu;                 /* the chemical potential used                                    */
  double trace;              /* sum_n c_n t_n (the summed core traces of the expansion)       */
  double coef_tail;          /* |c_order| + |c_order-1| (size of the last terms kept)          */
  double emin, emax;
  int32_t n_sub, max_sub, passes;
  float ms_bounds, ms_graph, ms_part, ms_gather, ms_terms, ms_scatter, ms_total;
  float ms_product;          /* summed device time of the product launches                    */
  int32_t n_product;         /* number of product launches                                     */
  double product_flops;      /* flops of one product launch: sum_s 2 n_s^3                    */
} gb_foe_stats;

gb_status gb_foe_density(const gb_ell* H, int32_t n_occ, double threshold, const gb_foe_opts* opts,
                         gb_ell* D, gb_foe_stats* stats, void* stream);

/* Host: the coefficients c_0 .. c_order of the Fermi function on [e_min, e_max] (mapped to
 * [-1, 1]) by K-node Chebyshev-Gauss quadrature, theta_k = pi (k + 1/2) / K:
 *   c_n = (2 - delta_n0) / K sum_k f(e(cos theta_k)) cos(n theta_k),
 *   e(x) = (e_max + e_min)/2 + x (e_max - e_min)/2,  f(e) = 1 / (1 + exp(beta (e - mu))).
 * n_nodes = 0 takes max(4 (order + 1), 1024).  coef: host array of order + 1 doubles. */
gb_status gb_chebyshev_fermi(double emin, double emax, double beta, double mu, int32_t order,
                             int32_t n_nodes, double* coef);
/* Host: mu in [e_min, e_max] with sum_n c_n(mu) traces[n] = n_occ (bisection to the last
 * representable bracket); GB_EINVAL if n_occ is outside the range the traces allow. */
gb_status gb_foe_solve_mu(const double* traces, int32_t order, double emin, double emax,
                          double beta, double n_occ, int32_t n_nodes, double* mu);

/* Host: the pre-determined SP2 branch sequence for a HOMO/LUMO pair (MD section: the whole
 * sequence of a step fixed in advance from the previous step's gap, so the subgraph expansions
 * exchange no traces).  With u = 1 - (e_max - e_homo)/(e_max - e_min) and
 * v = (e_max - e_lumo)/(e_max - e_min) (the distances of the two X0 images from 1 and 0), each
 * step is X^2 (0) when v > u, else 2X - X^2 (1), applied to both (X^2: v <- v^2,
 * u <- 2u - u^2; 2X - X^2: u <- u^2, v <- 2v - v^2), until both are <= delta.  out: host array
 * of max_len bytes; *len receives the length.  Replay it with gb_sp2_opts.branch_in.
 * GB_EINVAL unless e_min < e_homo < e_lumo < e_max and delta > 0; GB_ESHAPE if max_len steps
 * do not reach delta. */
gb_status gb_sp2_sequence(double emin, double emax, double e_homo, double e_lumo, double delta,
                          int32_t max_len, uint8_t* out, int32_t* len);

/* Host: HOMO/LUMO estimates from the core traces of an SP2 expansion (MD section: the next
 * step's sequence comes from the gap estimated during the previous step, after Rubensson and
 * Niklasson's interior-eigenvalue estimates).  Uses only the traces the trace rule computes:
 * t1[i] = Tr X_i and t2[i] = Tr X_i^2 for i = 0 .. n_branch (gb_sp2_stats.t1 / t2 with
 * n_branch = iters), branch[i] the update after iterate i.  With A = t1 - t2, B = t1 - n_occ,
 * L = (A + B)/2 and U = (A - B)/2 are, to fourth order, the sums over the unoccupied
 * eigenvalues of g(x) = x - x^2/2 (right after a step 2X - X^2) and over the occupied ones of
 * g(1 - x) (right after a step X^2).  From the latest such iterate whose sum exceeds `floor`:
 * the bound g^-1(L + U^2/2) is at least the LUMO image, so lumo_bound <= e_lumo (and likewise
 * homo_bound >= e_homo); from the latest pair of such iterates with a squaring of that side
 * between them, the ratio of their sums solved for one level by bisection gives lumo_ratio
 * >= e_lumo and homo_ratio <= e_homo.  Images are mapped back to X0 through the inverse branch
 * maps, which shrinks their relative error at every square root.  The bracket holds to fourth
 * order in the distances and to the rounding of the traces; a sequence from the bounds
 * (gb_sp2_sequence) is long enough for the spectrum the traces came from.
 * floor <= 0 takes max(10 (|t1 - n_occ| + |t1 - t2|) at the last iterate, 1e-12 n_occ).
 * GB_EINVAL for NULL pointers, n_branch < 1, emax <= emin, a branch other than 0/1, or when a
 * side has no usable iterate above the floor (an expansion that did not converge). */
typedef struct {
  double homo_bound, lumo_bound;   /* homo_bound >= e_homo, lumo_bound <= e_lumo              */
  double homo_ratio, lumo_ratio;   /* homo_ratio <= e_homo, lumo_ratio >= e_lumo              */
  double floor;                    /* the noise floor used                                     */
  int32_t homo_iter[3], lumo_iter[3];  /* iterates used: bound, ratio pair (i, j)            */
} gb_gap_estimate;

gb_status gb_sp2_estimate_gap(const double* t1, const double* t2, const uint8_t* branch,
                              int32_t n_branch, double n_occ, double emin, double emax,
                              double floor, gb_gap_estimate* out);

#ifdef __cplusplus
}
#endif

#endif /* GB_H */
