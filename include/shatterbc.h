/*
 * shatterbc -- exact betweenness centrality on AMD Instinct MI355X (gfx950)
 * with the shattering and compression method of Sariyuce, Saule, Kaya and
 * Catalyurek, "Shattering and Compressing Networks for Centrality Analysis".
 *
 * Problem (Section 2): an undirected, unweighted, loop-free graph G=(V,E) in
 * compressed row storage with 32-bit indices (Section 4).  Output: for every
 * vertex v, bc[v] = sum over ordered pairs s != v != t of sigma_st(v)/sigma_st
 * (Eq. (1), Section 2.1), unnormalised.  SBC_UNORDERED halves it (unordered
 * pairs); the halving is exact in binary64.
 *
 * Conventions for every call:
 *   - Return value: SBC_OK (0) or a negative sbc_status.  Nothing throws across
 *     this interface.  sbc_last_error() gives a message for the calling thread.
 *   - Host buffers are owned by the caller; the library copies what it needs
 *     before returning and keeps no caller pointer.
 *   - Device memory the library allocates is owned by the object that
 *     allocated it and freed by the matching *_destroy call.
 *   - "host" / "device" on a pointer says where it must point.
 *   - The compute path runs only on the GPU; without a usable gfx950 device
 *     every compute call returns SBC_E_NO_DEVICE (there is no CPU fallback).
 *     Graph creation and preprocessing are host-only and work without a GPU.
 */
#ifndef SHATTERBC_H
#define SHATTERBC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sbc_status;
#define SBC_OK 0
#define SBC_E_INVALID_ARG (-1)     /* NULL pointer, bad size, bad mode or option */
#define SBC_E_NOT_SYMMETRIC (-2)   /* an arc u->v without v->u */
#define SBC_E_SELF_LOOP (-3)       /* arc v->v (the paper assumes loop-free graphs, Section 2) */
#define SBC_E_DUP_EDGE (-4)        /* the same arc twice in one row */
#define SBC_E_INDEX_RANGE (-5)     /* a column index outside [0, n) */
#define SBC_E_TOO_LARGE (-6)       /* 2^31 or more arcs / packed vertices */
#define SBC_E_OOM (-7)             /* host or device allocation failed, or over the memory budget */
#define SBC_E_DEVICE (-8)          /* a HIP runtime call failed */
#define SBC_E_SIGMA_OVERFLOW (-9)  /* a path count exceeded the binary64 range */
#define SBC_E_CANCELLED (-10)
#define SBC_E_NOT_READY (-11)      /* job not finished yet (sbc_job_poll) */
#define SBC_E_NO_DEVICE (-12)      /* no usable gfx950 GPU */

/* sbc_graph_create flags */
#define SBC_SANITIZE 1u /* symmetrise, drop self loops and duplicate arcs instead of failing */

/* run modes (bit flags) */
#define SBC_PLAIN 0u         /* Algorithm 1 on the whole graph, no preprocessing */
#define SBC_COMPRESSED 1u    /* preprocess (default "odai" unless the graph was preprocessed) */
#define SBC_UNORDERED 2u     /* report unordered-pair scores (Eq. (1) halved) */
/* Bit-reproducible result: every work item (a piece and up to 64 of its
 * sources) accumulates its dependencies (Eq. (3), Algorithm 2's accumulation
 * step) into an area of its own, and the areas of a piece are summed in the
 * order of its sources afterwards, so no sum depends on the order in which
 * the device schedules items.  The same graph, mode and context parameters
 * then give the same bits on every run, alone or served beside other jobs.
 * Costs one double per (item, piece vertex) of device memory, and small
 * pieces run on the 64-source batch kernel instead of the small-piece kernel
 * (whose waves add into shared sums in no fixed order), with every entry
 * pulled by a whole wave. */
#define SBC_DETERMINISTIC 4u

typedef struct sbc_context_s* sbc_context;
typedef struct sbc_graph_s* sbc_graph;
typedef struct sbc_plan_s* sbc_plan;
typedef struct sbc_server_s* sbc_server;
typedef struct sbc_job_s* sbc_job;

/* Preprocessing statistics (Section 3; Section 4.2 names the letters). */
typedef struct {
  int64_t n, m;             /* input vertices and undirected edges */
  int64_t components;       /* connected components of the input */
  int64_t stripped;         /* degree-1 vertices removed (Section 3.3.1) */
  int64_t blocks;           /* biconnected components (Sections 3.2.1, 3.4) */
  int64_t bridges;          /* two-vertex blocks, done in closed form (Section 3.2.2) */
  int64_t twin_classes;     /* identical-vertex classes with >= 2 members (Section 3.3.3) */
  int64_t twins_merged;     /* vertices removed by merging */
  int64_t tiny_pieces;      /* pieces of <= 2 vertices after merging, closed form */
  int64_t pieces;           /* pieces left for the GPU */
  int64_t piece_vertices;   /* sum of piece vertex counts */
  int64_t piece_arcs;       /* sum of piece arc counts (2 x edges) */
  double work_teps;         /* sum over pieces of vertices x edges */
  double ms_degree1, ms_shatter, ms_twins, ms_pack; /* host wall time per stage */
  int64_t side_vertices;    /* side vertices removed (Section 3.3.2) */
  int64_t side_pieces;      /* side pieces: blocks whose side vertices run Algorithm 3 */
} sbc_prep_stats;

/* Statistics of one execution. */
typedef struct {
  double ms_device;          /* device time from first to last kernel of the run (HIP events) */
  double ms_traverse;        /* device time of the traversal kernels (forward + backward sweeps) */
  double ms_mapback;         /* device time of the Eq. (5) gather */
  double ms_host;            /* host wall time of the call */
  double teps;               /* sources x edges traversed, summed over pieces */
  double algo_bytes;         /* streaming-model bytes: per (source, piece) 8*arcs + 56*vertices */
  int64_t items;             /* work items drained from the device queue */
  int64_t batched_sources;   /* sources run by the 64-lane multi-source kernels (batch and team) */
  int64_t lds_sources;       /* sources run by the small-piece kernel (state in LDS) */
  int64_t global_sources;    /* always 0 (no other traversal kernel) */
  int32_t overflow;          /* device flags of the run (nonzero: a check failed or a path count overflowed) */
  /* Per traversal kernel class: 0 small pieces, one source per wavefront (LDS),
   * 2 64-source batches (one workgroup per batch), 3 the same for deep pieces
   * (a launch of its own), 4 64-source batches run by teams of workgroups (one
   * team per XCD); 1 is not used and stays 0.
   * Device time of the class's persistent launch, its streaming-model bytes,
   * and its sources x edges. */
  double ms_class[5];
  double bytes_class[5];
  double teps_class[5];
  int32_t grid_class[5];      /* resident workgroups of the launch */
  int32_t items_class[5];     /* work items of the launch */
} sbc_run_stats;

const char* sbc_status_string(sbc_status s);
/* Message of the calling thread's last failing call ("" if none). */
const char* sbc_last_error(void);
/* Library version string. */
const char* sbc_version(void);

/* ---------------------------------------------------------------- context */

/* Bind to GPU `device` (HIP ordinal).  Checks that it is gfx950.
 * Errors: SBC_E_NO_DEVICE, SBC_E_DEVICE, SBC_E_INVALID_ARG (out NULL). */
sbc_status sbc_context_create(int device, sbc_context* out);
sbc_status sbc_context_destroy(sbc_context ctx);

/* Tuning knobs, by name.  Known keys:
 *   "wave_max_vertices"  largest piece run by the small-piece kernel (default
 *                        256, at most 4096; 0: never): one source per
 *                        wavefront, the piece's CSR and every source's levels,
 *                        path counts and dependencies in LDS.  Pieces whose
 *                        arcs do not fit 64 KB of LDS go to the batch kernel
 *   "wave_wg_waves"      wavefronts per small-piece workgroup (4 or 8)
 *   "wave_sources_per_item" sources per small-piece work item (1..64)
 *   "batch_wg_waves"     wavefronts per workgroup of the multi-source kernel (4, 8, 16)
 *   "batch_waves_per_eu" occupancy target of the multi-source kernel: 0 (compiler default), 6 or 8 waves per SIMD
 *   "slots"              resident workgroups per traversal kernel (0 = auto)
 *   "cluster_sources"    batch source order: 0 piece order, 1 breadth-first balls,
 *                        2 (default) vertices grouped by a common neighbour of
 *                        degree >= 32 first, then balls
 *   "batch_pairs"        the batch kernel pulls entries with at most 32 arcs and
 *                        at most this many of the batch's sources as (entry,
 *                        source) pairs, one per lane (default 16, 0..64; 0: one
 *                        wave per entry always)
 *   "batch_compact"      1 (default): the batch kernel keeps an entry's path counts and
 *                        coefficients together, one value per lane the entry holds,
 *                        so a pull of a few-lane entry reads one sector; 0: one
 *                        64-value row per vertex (the team kernel's layout)
 *   "deep_min_levels"    pieces whose breadth-first depth from their highest-degree
 *                        vertex exceeds this (default 64; 0: never) run on the
 *                        batch kernel in a launch of their own (class 3)
 *   "deep_wg_waves"      wavefronts per workgroup of that launch (4, 8, 16; default 16)
 *   "deep_waves_per_eu"  its occupancy target: 0 (default), 6 or 8
 *   "mem_budget_mb"      traversal-state budget of a plan (0: 60% of free memory)
 *   "profile_phases"     1: plans keep per-phase timers of the batch and team kernels
 *   "order_plain"        1: plain plans run on the graph renumbered breadth-first
 *                        from its highest-degree vertex (Section 4.1)
 *   "team_min_vertices"  smallest piece run by the team kernel (0: never): all
 *                        workgroups of one XCD share one 64-source batch
 *   "team_count"         teams of the team kernel (default 64; a multiple of 8
 *                        puts team_count/8 teams on each of the 8 XCDs)
 *   "team_wg_waves"      wavefronts per workgroup of the team kernel (4, 8, 16; default 16)
 *   "team_waves_per_eu"  occupancy target of the team kernel: 0 or 8
 *   "team_local_fences"  1 (default): a team whose workgroups all run on one XCD
 *                        synchronises through that XCD's L2 (L1 invalidation
 *                        only); 0: agent-scope fences always
 *   "team_cooperative"   1 (default): the team kernel is launched cooperatively (the
 *                        runtime starts it only when every workgroup is
 *                        resident); 0: an ordinary launch of the same grid,
 *                        whose bounded join barrier turns a workgroup that
 *                        never starts into SBC_E_DEVICE (for tools that do not
 *                        handle cooperative launches)
 *   "team_split_arcs"    team kernel: rows with more arcs are pulled in slices
 *                        of 256 arcs spread over the team (default 2048)
 *   "team_max_levels"    pieces whose breadth-first depth from their highest-degree
 *                        vertex exceeds this stay on the one-workgroup batch
 *                        kernel (0: no limit)
 *   "far_wg_waves"       wavefronts per workgroup of the farness kernel (4, 8, 16; default 16)
 *   "server_order"       serving: 1 (default) least estimated work first, 0 oldest first
 *   "server_max_wait_ms" serving: a job waiting longer is taken first (default 30000)
 *   "sample_items"       tuning only (0: off): plans run an evenly spaced sample of
 *                        the work items -- at most this many of the kernel class
 *                        with the most items, and the same fraction of every
 *                        other class (at least one) -- so the result covers
 *                        only those items' sources
 *   "team_spin_ms"       bound of one team barrier wait; a longer wait aborts
 *                        the launch with SBC_E_DEVICE instead of hanging
 *                        (0: no waiting at all, which aborts any team of more
 *                        than one workgroup: a test of the abort path)
 * Read-only (get only): "cus" compute units, "lds_limit_bytes" LDS per workgroup.
 * Errors: SBC_E_INVALID_ARG for an unknown key or out-of-range value. */
sbc_status sbc_context_set_param(sbc_context ctx, const char* key, int64_t value);
sbc_status sbc_context_get_param(sbc_context ctx, const char* key, int64_t* value);
/* Name of the bound device (e.g. "AMD Instinct MI355X"), NUL-terminated, at most len bytes. */
sbc_status sbc_context_device_name(sbc_context ctx, char* buf, size_t len);

/* ------------------------------------------------------------------ graph */

/* Copy a CSR graph: row_ptr[n+1] and col[row_ptr[n]] (host), each undirected
 * edge present as both arcs, no self loops, no duplicates (unless
 * SBC_SANITIZE).  Host-only; needs no GPU.
 * Errors: SBC_E_INVALID_ARG, SBC_E_INDEX_RANGE, SBC_E_SELF_LOOP,
 * SBC_E_DUP_EDGE, SBC_E_NOT_SYMMETRIC, SBC_E_TOO_LARGE, SBC_E_OOM. */
sbc_status sbc_graph_create(int32_t n, const int32_t* row_ptr, const int32_t* col, uint32_t flags,
                            sbc_graph* out);
sbc_status sbc_graph_destroy(sbc_graph g);
/* n and the number of arcs (2 x edges) of the stored graph. */
sbc_status sbc_graph_info(sbc_graph g, int32_t* n, int64_t* arcs);

/* Shatter and compress (Section 3), host-only.  ops holds letters applied in
 * this order: 'o' orders each piece's vertices breadth-first from its
 * highest-degree vertex (the ordering of Section 4.1, applied per piece after
 * the other steps), 'd' degree-1 vertices (Section 3.3.1), 'a' articulation
 * vertices via biconnected components, bridges included ('b' is accepted as
 * the same step; Sections 3.2.1, 3.2.2, 3.4), 's' side vertices -- degree 1
 * to 4, neighbours pairwise adjacent (Sections 3.3.2, 3.4) -- removed one
 * after another from each piece, each leaving an Algorithm 3 search on the
 * piece as it was (a side piece), 'i' identical vertices (Section 3.3.3) of
 * equal reach, 'u' identical vertices whatever their reach (a generalisation
 * the paper leaves out: the class's traversal starts every member's
 * dependency at the members' mean reach minus one and the host adds each
 * member's difference from the mean, and the terms for pairs between members,
 * to that member alone; 'u' includes 'i').
 * "" keeps every connected component whole.  st may be NULL.
 * Errors: SBC_E_INVALID_ARG for an unknown letter, SBC_E_TOO_LARGE. */
sbc_status sbc_graph_preprocess(sbc_graph g, const char* ops, sbc_prep_stats* st);

/* Sizes of the preprocessed problem: pieces P, piece vertices V, piece arcs A,
 * map entries M (original vertex -> piece vertex links). */
sbc_status sbc_graph_export_sizes(sbc_graph g, int64_t* P, int64_t* V, int64_t* A, int64_t* M);
/* Copy the preprocessed problem out (host buffers sized by export_sizes; any
 * may be NULL to skip it):
 *   vtx_off[P+1]   piece p owns piece vertices [vtx_off[p], vtx_off[p+1])
 *   row[V+1]       absolute arc offsets; col[A] local (piece-relative) ids
 *   reach[V], ident[V]   Section 3.2 / 3.3.3 attributes of a piece vertex:
 *                  ident = the identical vertices it stands for, reach = their
 *                  reaches summed (ident x the common reach when they are equal)
 *   corr[V]        per-member terms added to each piece vertex's bc'
 *   bcx[n]         per-original-vertex terms closed in form on the host
 *   map_off[n+1], map_idx[M]   original v -> piece vertices (Eq. (5))
 * bc[v] = bcx[v] + sum over j in map of (bc'[map_idx[j]] + corr[map_idx[j]]). */
sbc_status sbc_graph_export(sbc_graph g, int32_t* vtx_off, int32_t* row, int32_t* col, int32_t* reach,
                            int32_t* ident, double* corr, double* bcx, int32_t* map_off, int32_t* map_idx);
/* nside[P] (host): 0 for a piece of Algorithm 2 (every vertex a source), or
 * k > 0 for a side piece: a piece as it was before its side vertices were
 * removed, those being its local ids 0..k-1 in removal order; its only
 * sources are those k vertices, and source i runs Algorithm 3 (Section
 * 3.3.2) on the piece without side vertices 0..i-1, adding
 * reach[i]*delta[w] + reach[i]*(delta[w] - (reach[w]-1)) to every other
 * vertex w still there.  Its bc' enters Eq. (5) like any piece's.
 * Errors: SBC_E_INVALID_ARG (NULL, or not preprocessed). */
sbc_status sbc_graph_export_side(sbc_graph g, int32_t* nside);

/* ------------------------------------------------------------------- plan */

/* Upload the problem of `mode` (SBC_PLAIN or SBC_COMPRESSED; SBC_COMPRESSED on
 * a graph not yet preprocessed runs "odai" first) to the device, build the
 * work queue and allocate traversal state.  The plan keeps everything
 * resident, so repeated executions touch no host memory.
 * Errors: SBC_E_NO_DEVICE, SBC_E_OOM, SBC_E_DEVICE, SBC_E_INVALID_ARG. */
sbc_status sbc_plan_create(sbc_context ctx, sbc_graph g, uint32_t mode, sbc_plan* out);
sbc_status sbc_plan_destroy(sbc_plan p);
/* Run the whole path (every source of every piece, forward and backward
 * sweeps, accumulation, Eq. (5) gather) on `stream` (a hipStream_t, NULL =
 * the plan's own stream) and write bc (n doubles, device memory, or NULL to
 * keep it inside the plan).  Asynchronous: returns after enqueueing; the
 * output is valid once the stream reaches this point.
 * Errors: SBC_E_DEVICE. */
sbc_status sbc_plan_execute(sbc_plan p, double* bc_dev, void* stream);
/* Wait for the last execution and return its statistics (and
 * SBC_E_SIGMA_OVERFLOW if a path count overflowed). */
sbc_status sbc_plan_sync(sbc_plan p, sbc_run_stats* st);
/* Copy the plan's own result (n doubles) to host memory (waits). */
sbc_status sbc_plan_result(sbc_plan p, double* bc_host);
/* Phase timers of the last execution of the 64-source batch and team kernels, kept
 * when the context parameter "profile_phases" was 1 at plan creation (the
 * paper splits its times into a BFS phase and a back-propagation phase,
 * Section 4.2).  out[0..7]: mean milliseconds per resident workgroup spent
 * taking items, discovering the next level (forward), counting paths
 * (forward), counting paths of split long rows, retiring frontiers, in the
 * backward sweep, in split long rows of the backward sweep, and restoring
 * state; out[8..10]: items, levels and (vertex, level) entries processed;
 * out[11]: mean milliseconds per workgroup waiting at team barriers.
 * count is the length of out (at most 12 values are written).
 * Errors: SBC_E_INVALID_ARG if profiling was off for this plan. */
sbc_status sbc_plan_phase_profile(sbc_plan p, double* out, int32_t count);
/* Team layout of the last execution's team kernel (pieces from
 * "team_min_vertices" on): for team t < min(cap, *nteams), sizes[t] workgroups
 * and xcc_masks[t] the set of XCDs (bit x for hardware XCC id x) they ran on.
 * *nteams is 0 when the plan has no team pieces.  Waits for the execution.
 * Errors: SBC_E_INVALID_ARG (NULL outputs, or not executed yet). */
sbc_status sbc_plan_team_layout(sbc_plan p, int32_t* sizes, int32_t* xcc_masks, int32_t cap, int32_t* nteams);
/* Capture one execution into a HIP graph and replay it on later executes
 * (enable = 1) or go back to direct launches (enable = 0). */
sbc_status sbc_plan_use_graph(sbc_plan p, int enable);

/* --------------------------------------------------------- one-shot calls */

/* Plan, execute, copy back and destroy: bc_host[n] (host).  st may be NULL. */
sbc_status sbc_betweenness(sbc_context ctx, sbc_graph g, uint32_t mode, double* bc_host, sbc_run_stats* st);
/* Same with the result left in device memory bc_dev[n] on `stream`;
 * synchronises the stream before returning. */
sbc_status sbc_betweenness_device(sbc_context ctx, sbc_graph g, uint32_t mode, double* bc_dev, void* stream,
                                  sbc_run_stats* st);
/* Algorithm 1 restricted to the listed sources (plain graph, ordered pairs):
 * bc_host[v] = sum over s in sources of delta_s(v).  Sources must be distinct.
 * Errors: SBC_E_INVALID_ARG, SBC_E_INDEX_RANGE. */
sbc_status sbc_betweenness_sources(sbc_context ctx, sbc_graph g, int64_t nsrc, const int32_t* sources,
                                   double* bc_host, sbc_run_stats* st);

/* Algorithm 2 with identical-vertex weights (Sections 3.2.1, 3.3.3) on one
 * attributed piece given in host CSR form (local ids, symmetric, loop-free):
 * bc_host[v] = sum over sources s of ident[s]*reach[s]*delta_s(v), v != s,
 * where sigma counts paths through v != s with weight ident[v] and delta
 * starts at reach[v]-1.  reach/ident may be NULL (all ones).  `kernel` forces
 * one traversal kernel: 0 automatic, 3 64-lane multi-source, 4 64-lane
 * multi-source run by teams of workgroups, 5 small-piece kernel (one source
 * per wavefront, everything in LDS).  1 and 2 name one-source-per-workgroup
 * kernels this library does not have (SBC_E_INVALID_ARG).
 * Errors: SBC_E_INVALID_ARG (shape, or a piece too large for the forced kernel). */
sbc_status sbc_piece_bc(sbc_context ctx, int32_t n, const int32_t* row_ptr, const int32_t* col,
                        const int32_t* reach, const int32_t* ident, int kernel, double* bc_host,
                        sbc_run_stats* st);

/* Verification of the traversal's per-source state (Algorithm 1's BFS phase,
 * Section 2.1, and its back propagation, Eq. (3), in the weighted form of
 * Algorithm 2 with ident, Sections 3.2.1 and 3.3.3) on the same attributed
 * piece form as sbc_piece_bc.  The sources sources[0..nsrc) (distinct, in
 * [0, n)) run through traversal kernel `kernel` (0 automatic, 3 batch, 4 team,
 * 5 small-piece), built with a step that also writes each source's state;
 * the bc' arithmetic is the same code the other calls run.  Row k of each
 * output (host, nsrc x n values, any may be NULL) belongs to sources[k]:
 *   dist[k*n + v]   BFS level of v from sources[k], -1 when unreachable
 *   sigma[k*n + v]  shortest-path count (ident-weighted through v != source)
 *   delta[k*n + v]  dependency of v (0 at the source itself and where
 *                   unreachable)
 * Errors: SBC_E_INVALID_ARG (shape, kernel, nsrc outside 1..n, duplicate
 * sources, a piece too large for the forced kernel), SBC_E_INDEX_RANGE (a
 * source outside [0, n)), SBC_E_TOO_LARGE (nsrc x n >= 2^31). */
sbc_status sbc_sources_state(sbc_context ctx, int32_t n, const int32_t* row_ptr, const int32_t* col,
                             const int32_t* reach, const int32_t* ident, int32_t nsrc, const int32_t* sources,
                             int kernel, int32_t* dist, double* sigma, double* delta);

/* sbc_sources_state for the single source s with the automatic kernel choice:
 * dist[n], sigma[n], delta[n] (host).  Any output may be NULL.
 * Errors: as sbc_sources_state; SBC_E_INDEX_RANGE when s is outside [0, n). */
sbc_status sbc_single_source(sbc_context ctx, int32_t n, const int32_t* row_ptr, const int32_t* col,
                             const int32_t* reach, const int32_t* ident, int32_t s, int32_t* dist,
                             double* sigma, double* delta);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the result
 * of sbc_piece_bc (bc' of one attributed piece, all sources, ordered pairs)
 * from inputs already in device memory, with no device allocation.
 *   n              piece vertices, 1..SBC_NOALLOC_MAX_VERTICES
 *   arcs           entries of col_dev (2 x edges)
 *   row_ptr_dev    device, n+1 int32 arc offsets (row_ptr_dev[0] = 0)
 *   col_dev        device, arcs int32 local neighbour ids (symmetric, loop-free)
 *   reach_dev, ident_dev  device, n int32 each (>= 1, reach x ident < 2^31),
 *                  or NULL for all ones (a value out of range is reported in
 *                  flags_dev)
 *   bc_dev         device, n doubles: receives bc'
 *   flags_dev      device, one int32 (or NULL): the run's device check flags,
 *                  0 when every check passed and every work item finished
 *   stream         hipStream_t (NULL = the null stream)
 * Asynchronous: only kernel launches are enqueued on `stream`; the output and
 * flags are valid once the stream reaches this point.  The 64-source batch
 * kernel's traversal state, work items and control words live in one static
 * device array of SBC_NOALLOC_SCRATCH_MB MiB per GPU, which the library holds
 * from the first call on a GPU until the process ends; every call on that GPU
 * shares it, so calls that overlap on one GPU (concurrent streams or threads)
 * race and give wrong results.  The CSR is read as given (row offsets within
 * [0, arcs], neighbour ids within [0, n) are checked on the device and
 * reported in flags_dev).
 * Errors: SBC_E_INVALID_ARG (NULL argument, n < 1, arcs < 0), SBC_E_TOO_LARGE
 * (n > SBC_NOALLOC_MAX_VERTICES, or the piece's state does not fit the
 * array), SBC_E_DEVICE (a launch failed). */
#define SBC_NOALLOC_MAX_VERTICES 65536
#define SBC_NOALLOC_SCRATCH_MB 256
sbc_status sbc_piece_bc_noalloc(sbc_context ctx, int32_t n, int32_t arcs, const int32_t* row_ptr_dev,
                                const int32_t* col_dev, const int32_t* reach_dev, const int32_t* ident_dev,
                                double* bc_dev, int32_t* flags_dev, void* stream);

/* Streaming copy of `bytes` (rounded down to 16) between two device buffers
 * the library allocates, `reps` times after one warm-up: *gbps = (read +
 * write bytes) / time.  It measures the bandwidth a plain streaming kernel
 * reaches on this device, and gives a kernel of known traffic
 * (copy_kernel) for scaling hardware byte counters.
 * Errors: SBC_E_INVALID_ARG, SBC_E_OOM, SBC_E_DEVICE. */
sbc_status sbc_copy_bandwidth(sbc_context ctx, size_t bytes, int reps, double* gbps);

/* ---------------------------------------------------- farness and closeness
 *
 * Closeness centrality on the same shattered pieces: the paper builds its
 * shattering for betweenness and names closeness as the next measure to
 * carry it to (Sections 1 and 5), without formulas.  The farness of v is the
 * sum of hop distances from v to every vertex of its connected component; the
 * closeness is (component size - 1) / farness (0 for an isolated vertex).
 * All values are exact (int64).
 *
 * The host strips degree-1 vertices (Section 3.3.1) and shatters at
 * articulation vertices (Section 3.2.1; bridges as two-vertex blocks,
 * Section 3.2.2), with the reach of every copy as for betweenness.  The
 * device computes, for every vertex v of every piece B of 3 or more
 * vertices, W_B(v) = sum over w in B of reach_B(w) * d_B(v, w) (64 sources
 * per work item, breadth-first only); the host then passes once up and once
 * down the block-cut tree and the stripped trees:
 *   farness(v) = W_B(v) + farness(t) - W_B(t)   for v in B below its top t,
 *   farness(u) = farness(v) + R - 2 s            for u stripped from v with a
 *                                                subtree of s vertices,
 * the search root's farness being the sum, over what hangs from it, of the
 * W and distance sums accumulated on the way up. */
typedef struct sbc_far_s* sbc_far;

typedef struct {
  int64_t n, components;
  int64_t stripped;        /* degree-1 vertices removed */
  int64_t blocks, bridges; /* blocks of the stripped graph; two-vertex ones among them */
  int64_t pieces;          /* blocks of >= 3 vertices (or whole components without 'a'): device pieces */
  int64_t piece_vertices, piece_arcs;
  double ms_prep;
} sbc_far_stats;

typedef struct {
  double ms_kernel;        /* device time of the farness kernel */
  double ms_device_total;  /* uploads, kernel and downloads */
  double ms_finish;        /* host pass over the block-cut tree */
  double ms_total;
  double teps;             /* sum over pieces of n_p * m_p, per second of kernel time */
  int64_t items, grid, waves;
  int32_t flags;           /* device flags (0 on success) */
} sbc_far_run_stats;

/* Prepare graph g for farness with preprocessing `ops`: any of 'o'
 * (breadth-first order per piece, Section 4.1), 'd' (degree-1), 'a'
 * (articulation shattering); "" keeps each component whole.  Host only; the
 * graph may be used or destroyed afterwards (nothing refers to it).
 * Errors: SBC_E_INVALID_ARG (NULL, or a letter other than o, d, a), SBC_E_OOM. */
sbc_status sbc_far_create(sbc_graph g, const char* ops, sbc_far* out, sbc_far_stats* st);
sbc_status sbc_far_destroy(sbc_far f);
/* Sizes of the device pieces: P, V = sum of n_p, A = sum of arcs. */
sbc_status sbc_far_info(sbc_far f, int32_t* pieces, int64_t* vertices, int64_t* arcs);
/* Copies the device pieces to host buffers (any may be NULL): vtx_off[P+1],
 * row[V+1] (absolute arc offsets), col[A] (piece-local ids), reach[V] and
 * orig[V] (the original vertex of each piece vertex). */
sbc_status sbc_far_export(sbc_far f, int32_t* vtx_off, int32_t* row, int32_t* col, int32_t* reach, int32_t* orig);
/* Host pass only: farness[n] (and closeness[n] unless NULL) from the per-piece
 * sums piece_sums[V] (W_B of every piece vertex, in export order), however
 * they were computed.  Needs no GPU. */
sbc_status sbc_far_finish(sbc_far f, const int64_t* piece_sums, int64_t* farness, double* closeness);
/* The whole computation: device sums (written to piece_sums[V] unless NULL),
 * then the host pass.  Outputs are host buffers.
 * Errors: SBC_E_DEVICE (launch failure, or a device range check),
 * SBC_E_OOM, SBC_E_TOO_LARGE. */
sbc_status sbc_far_run(sbc_context ctx, sbc_far f, int64_t* piece_sums, int64_t* farness, double* closeness,
                       sbc_far_run_stats* st);

/* ---------------------------------------------------------------- serving */

/* A continuously batching request loop on one GPU.  Jobs are admitted while
 * their device footprint fits in hbm_budget_bytes (0 = 80% of free memory)
 * and a slot is free; admitted jobs run concurrently on `slots` streams, so a
 * job that arrives while others run starts as soon as a slot and memory free
 * up.  The budget is allocated at creation, divided among the slots as
 * device arenas (plus 64 MiB of pinned staging memory per slot): a job's
 * device buffers come from its slot's arena and its copies run
 * asynchronously on the slot's stream, so no job allocates or frees device
 * memory (a job whose state does not fit its slot's arena fails with
 * SBC_E_OOM).
 * A free slot takes the waiting job with the least estimated work
 * (n x arcs x (1 + breadth-first depth / 16)), or the oldest job once it has
 * waited server_max_wait_ms; context parameter server_order = 0 takes the
 * oldest job always.
 * Errors: SBC_E_INVALID_ARG, SBC_E_DEVICE. */
sbc_status sbc_server_create(sbc_context ctx, int slots, size_t hbm_budget_bytes, sbc_server* out);
/* Drains every submitted job, then stops the loop and frees the server. */
sbc_status sbc_server_destroy(sbc_server s);

typedef struct {
  double submit_to_start_ms;  /* waiting for admission */
  double start_to_done_ms;    /* preprocessing + device work + copy back */
  double latency_ms;          /* submit to result on the host */
  double teps;                /* sources x edges of the job */
  int64_t footprint_bytes;    /* device bytes the job held */
} sbc_job_stats;

/* Queue a betweenness job on graph g (which must outlive the job and must
 * not be used by another call until the job is released).  Thread-safe. */
sbc_status sbc_server_submit(sbc_server s, sbc_graph g, uint32_t mode, sbc_job* out);
/* *done = 1 when the job has finished (successfully or not). */
sbc_status sbc_job_poll(sbc_job j, int* done);
/* Block until the job finishes; copy bc (n doubles, host) and its stats
 * (either may be NULL).  Returns the job's own status. */
sbc_status sbc_job_wait(sbc_job j, double* bc_host, sbc_job_stats* st);
sbc_status sbc_job_release(sbc_job j);

#ifdef __cplusplus
}
#endif

#endif /* SHATTERBC_H */
