/*
 * agal.h -- C ABI of the MI355X near-wall mesh-adaptation library.
 *
 * Method: "Towards a GPU-native adaptive mesh refinement scheme for the
 * Lattice Boltzmann Method in complex geometries" (Jaber, Essel, Sullivan,
 * 2025).  A triangle (3D) or edge (2D) mesh is embedded in a forest of
 * octrees (quadtrees) whose nodes are blocks of 4^D cells, in three steps
 * (Abstract; Sec. II): import the faces, distribute them to a uniform grid of
 * bins of user-set density, then refine the grid level by level near the wall
 * and link boundary nodes to the faces along the lattice directions.
 *
 * Conventions shared by every call
 *  - Every call returns agal_status; no exception crosses the ABI.  On
 *    failure out-handles are left untouched and agal_last_error() (per host
 *    thread) describes the cause.
 *  - Pointers named d_* are device pointers (HIP device memory of the
 *    current device); everything else is host memory.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  All
 *    device work is enqueued on it.  Calls that must size an output read a
 *    device count back and synchronise that stream (stated per call).
 *  - Handles own their device memory until destroyed; device pointers
 *    returned by *_view stay valid until the owning handle is destroyed and
 *    hold final values once `stream` has been synchronised.
 *  - Handles are not thread-safe; distinct handles may be used from distinct
 *    host threads on distinct streams.
 *  - Inputs are never retained: a call has consumed its input buffers once
 *    the work it enqueued on `stream` has completed.
 */
#ifndef AGAL_H
#define AGAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AGAL_API __attribute__((visibility("default")))

typedef enum agal_status {
    AGAL_OK = 0,
    AGAL_EINVAL = 1,    /* an argument is out of its documented range */
    AGAL_ENOMEM = 2,    /* a device or host allocation failed */
    AGAL_EHIP = 3,      /* the HIP runtime reported an error */
    AGAL_ECAPACITY = 4, /* a preallocated capacity was exceeded (batched plans) */
    AGAL_ESTATE = 5     /* handles do not belong together or a result is inconsistent */
} agal_status;

typedef struct agal_context_t *agal_context;
typedef struct agal_geom_t *agal_geom;
typedef struct agal_bins_t *agal_bins;
typedef struct agal_forest_t *agal_forest;
typedef struct agal_links_t *agal_links;
typedef struct agal_batch_t *agal_batch;
typedef struct agal_forest_diff_t *agal_forest_diff;

/* Optional device allocator.  alloc returns device memory usable on `stream`
 * (or NULL on failure); free releases it in stream order.  A NULL allocator
 * selects the HIP stream-ordered pool (hipMallocAsync / hipFreeAsync). */
typedef struct agal_allocator {
    void *ctx;
    void *(*alloc)(void *ctx, size_t bytes, void *stream);
    void (*free)(void *ctx, void *ptr, void *stream);
} agal_allocator;

/* Lattice velocity sets (Sec. II-C-1: links follow the directions of the
 * discrete velocity set).  Direction order: rest; the axis directions in
 * +/- pairs (x, y, z); for D3Q19/D3Q27 the 12 edge directions in +/- pairs
 * ((1,1,0),(-1,-1,0),(1,-1,0),(-1,1,0), then the xz and yz analogues); for
 * D3Q27 the 8 corner directions in +/- pairs ((1,1,1),(1,1,-1),(1,-1,1),
 * (-1,1,1) and negatives).  D2Q9: rest, (+-1,0), (0,+-1), (1,1),(-1,-1),
 * (1,-1),(-1,1).  Direction i and its opposite are i and i+1 for odd i. */
enum { AGAL_D2Q9 = 9, AGAL_D3Q19 = 19, AGAL_D3Q27 = 27 };

#define AGAL_MAX_LEVELS 8

/* Forest of root trees (Sec. II-A): roots[a] root blocks along axis a tile
 * [lo, hi]; each block holds 4^D cells; n_levels refinement passes make
 * levels 0..n_levels.  d_spec[l] (host, one per pass, >= 0) is the near-wall
 * distance for the cells tested in pass l (Sec. II-C-2). */
typedef struct agal_forest_desc {
    int dim;
    int roots[3];
    int n_levels;
    const float *d_spec;
    float lo[3];
    float hi[3];
} agal_forest_desc;

/* ---- context ---------------------------------------------------------- */
AGAL_API agal_status agal_context_create(const agal_allocator *alloc, agal_context *out);
AGAL_API void agal_context_destroy(agal_context ctx);

/* ---- import (Sec. II-B) -------------------------------------------------
 * Copies the geometry into library-owned device memory as a structure-of-
 * arrays coordinate list (vertex k, axis a of face f) plus per-face bounding
 * boxes, and keeps the index list for the adjoint.
 *   dim         2 (edges) or 3 (triangles).
 *   d_vertices  n_vertices x dim FP32, row-major.
 *   d_faces     n_faces x dim int32 vertex indices, row-major; NULL means
 *               d_vertices is already a coordinate list of n_faces x dim
 *               corners (then n_vertices must equal n_faces * dim).
 * Errors: AGAL_EINVAL for dim not in {2,3}, n_faces < 1, n_vertices < 1, an
 * index outside [0, n_vertices), or a NaN/Inf coordinate (checked on the
 * device; this call synchronises `stream`). */
AGAL_API agal_status agal_import_faces(agal_context ctx, int dim, const float *d_vertices, int64_t n_vertices,
                                       const int32_t *d_faces, int64_t n_faces, void *stream, agal_geom *out);
/* d_coords: (dim*dim) x n_faces FP32, row (k*dim + a) = axis a of vertex k.
 * d_aabb: (2*dim) x n_faces FP32, rows 0..dim-1 minima, dim..2dim-1 maxima. */
AGAL_API agal_status agal_geom_view(agal_geom g, int *dim, int64_t *n_faces, int64_t *n_vertices,
                                    const float **d_coords, const float **d_aabb);

/* ---- spatial binning (Sec. II-C-3) ---------------------------------------
 * B bins per axis tile [lo, hi] (B^D bins; bin (ix,iy,iz) has linear index
 * (iz*B + iy)*B + ix).  Face f belongs to every bin its bounding box touches:
 * per axis the index range is [idx(min), idx(max)] with
 * idx(x) = clamp(floor((x - lo) * s), 0, B-1), s = (float)B / (hi - lo), all
 * FP32, so faces partly outside [lo, hi] go to the edge bins.  Output is a
 * CSR: offsets (B^D + 1 uint32) and face ids ascending inside each bin.
 * Errors: AGAL_EINVAL for B < 1, B^D > 2^31, hi <= lo.  Synchronises
 * `stream` once to size the id array. */
AGAL_API agal_status agal_bin_faces(agal_geom g, const float lo[3], const float hi[3], int32_t B, void *stream,
                                    agal_bins *out);
AGAL_API agal_status agal_bins_view(agal_bins b, const uint32_t **d_offsets, const int32_t **d_face_ids,
                                    int64_t *n_bins, int64_t *n_entries);
/* agal_bin_faces without any device allocation, for callers that cannot
 * allocate (code between allocation-free points of a serving loop, harnesses
 * that forbid hipMalloc): the same bins, written into caller buffers.
 *   d_offsets    B^D + 1 uint32 (caller-owned);
 *   d_face_ids   ids_capacity int32 (caller-owned; may be NULL when
 *                ids_capacity is 0);
 *   *n_entries   the number of (face, bin) entries P, set on AGAL_OK and on
 *                AGAL_ECAPACITY.
 * Working memory (per-bin counts and cursors, scan status) lives in a fixed
 * 32 MiB device array of the library, one per GPU, kept until the process
 * ends: 3 B^D + ids_capacity / 2048 words plus a few thousand must fit in
 * 8 Mi words (about 2.8 million bins).  Every call on one GPU uses that GPU's
 * array, so calls that overlap on one GPU (other streams or host threads)
 * race; calls in sequence on one stream are safe (each clears what it needs).
 * Errors: those of agal_bin_faces; AGAL_EINVAL when the grid and capacity do
 * not fit the scratch array; AGAL_ECAPACITY when P > ids_capacity (offsets
 * are written, ids are not); AGAL_EHIP when the scratch address could not be
 * taken at context creation.  Synchronises `stream` once (to read P). */
AGAL_API agal_status agal_bin_faces_noalloc(agal_geom g, const float lo[3], const float hi[3], int32_t B,
                                            uint32_t *d_offsets, int32_t *d_face_ids, int64_t ids_capacity,
                                            void *stream, int64_t *n_entries);
/* The paper's own binning (Sec. II-C-3 and its discretization figure): each
 * face is sampled at points and goes to every bin holding one of them.  An
 * edge a -> b, e = b - a, is cut into 2^k equal pieces, k the least integer
 * >= 0 (at most 12) with max_a |e_a| <= spacing * 2^k; its points are
 * a + e * (j 2^-k), j = 0..2^k (FP32, one product and one sum per component).
 * A triangle (a, b, c) takes the points q_j of edge a -> b and samples every
 * segment q_j -> c the same way; a 2D face is its edge.  A point's bin is
 * idx() of agal_bin_faces per axis.  Output: the same CSR layout (ascending
 * face ids per bin), a subset of the bounding-box bins.
 *   spacing       sample spacing in domain units; <= 0 selects half the
 *                 smallest bin edge.
 *   bin_fraction  0: the (face, bin) pairs are counted, scanned and
 *                 scattered; B_f >= 1: the paper's form, B^D / B_f bins at a
 *                 time (rounded up) through an indicator array of that many
 *                 rows of n_faces words, each row then compacted in face
 *                 order (memory ~ 4 n_faces B^D / B_f bytes).
 * Sampled-point bins serve the own-bin refinement and the list-mode link
 * step; the box-test refinement and the bin walk of the link step need the
 * bounding-box bins and refuse these (AGAL_EINVAL).
 * Errors: those of agal_bin_faces; AGAL_EINVAL for a negative bin_fraction
 * or a NaN or infinite spacing; AGAL_ECAPACITY when one fraction's indicator
 * array would exceed 32 GiB.  Synchronises `stream` (the pairs form once, the
 * fraction form once more when its first guess of ten entries per face was
 * short). */
AGAL_API agal_status agal_bin_faces_discrete(agal_geom g, const float lo[3], const float hi[3], int32_t B,
                                             float spacing, int32_t bin_fraction, void *stream, agal_bins *out);

/* ---- near-wall refinement (Sec. II-C-1, II-C-2, II-A) --------------------
 * For pass l = 0..n_levels-1, every cell of every block present at level l
 * when the pass starts is tested: it is flagged when a face meets the closed
 * cube of half-width d_spec[l] centred on the cell centre (13-axis
 * separating-axis test in FP32; the cell centre is
 * lo + (float)(2g+1) * (0.5f * dx_l), dx_l = (hi - lo) / (4 * roots * 2^l)).
 * A block with a flagged cell is marked and refined into 2^D children; 2:1
 * balance across faces, edges and corners is restored by refining the
 * coarser neighbours that need it.  Blocks created in pass l are not tested
 * in pass l.  Results are identical to testing every face (binning only
 * prunes candidates).
 * Block keys: a root's key is its x-fastest linear index; a child's key is
 * parent_key * 2^D + (cx + 2 cy + 4 cz).  Requires
 * roots_x*roots_y*roots_z * 2^(D*n_levels) <= 2^32.
 * Errors: AGAL_EINVAL for dim mismatch with the geometry, roots < 1,
 * n_levels outside [0, AGAL_MAX_LEVELS], key overflow, a negative or
 * non-finite d_spec, hi <= lo; AGAL_ESTATE when `bins` belongs to another
 * geometry.  Synchronises `stream` once per pass to size the next level. */
AGAL_API agal_status agal_near_wall_refine(agal_geom g, agal_bins b, const agal_forest_desc *desc, void *stream,
                                           agal_forest *out);
/* The paper's own form of the near-wall refinement (Sec. II-C-2 with
 * Algorithm 1; the propagation paragraph of Sec. II-C-3).  Pass l flags a cell
 * when its centre lies within Euclidean distance d_spec[l] of a face of the
 * one bin that holds the centre (FP32 point-to-face distance without
 * divisions: edges, vertices and the face interior); then the marks spread
 * to neighbouring blocks of the level (faces, edges, corners), one ring per
 * step, over n_prop steps (n_prop < 0: 1 + floor(d_spec[l] / (4 dx_l)) with
 * the smallest cell size over the axes, and none when the bins are a single
 * bin, where every cell sees every face).  A face beyond the own bin is
 * missed unless propagation reaches it, so the forest depends on B, as in
 * the paper.  Exported marks: 1 flagged, 2 balance, 3 propagation; balance
 * and children as agal_near_wall_refine.  Errors and synchronisation as
 * agal_near_wall_refine. */
AGAL_API agal_status agal_near_wall_refine_own_bin(agal_geom g, agal_bins b, const agal_forest_desc *desc,
                                                   int n_prop, void *stream, agal_forest *out);
/* How the flag step of each pass runs (the flags are identical either way).
 * Face-centric: one lane per (face, cell near the face) pair; above level 0
 * it finds blocks through a dense scratch table over the level's block grid
 * (roots * 2^l positions per axis, 4 bytes each).  Cell-centric: one wave per
 * block over the bins under the block, no table.  A level whose block grid
 * has at most max_entries positions takes the face-centric step, unless the
 * geometry's largest face has more than 4096 candidate cells there (its box
 * extent plus the distance on both sides, per axis; measured at import).  Default
 * 2^24 (a 64 MiB table at most); 0 makes every level cell-centric.  Applies
 * to agal_near_wall_refine calls made with ctx afterwards.
 * Errors: AGAL_EINVAL for a NULL context or a negative limit. */
AGAL_API agal_status agal_context_set_flag_table_limit(agal_context ctx, int64_t max_entries);
/* Level arrays in ascending key order:
 *   d_keys[n]          block keys;
 *   d_leaf[n]          1 when the block has no children;
 *   d_mark[n]          1 = refined because one of its cells was flagged,
 *                      2 = refined only to keep 2:1 balance, 0 = not refined;
 *   d_cell_flag[n*4^D] per-cell test results, cells x-fastest (0 for blocks
 *                      that were never tested); NULL at the finest level. */
AGAL_API agal_status agal_forest_level_view(agal_forest f, int level, const uint32_t **d_keys,
                                            const uint8_t **d_leaf, const uint8_t **d_mark,
                                            const uint8_t **d_cell_flag, int64_t *n_blocks);
AGAL_API agal_status agal_forest_info(agal_forest f, int *dim, int *n_levels);

/* ---- re-adaptation of a moving body ---------------------------------------
 * The paper refines once, before the solver, and names moving geometry as the
 * case where rebuilding the bins every step weighs on the choice of bin
 * density (Results discussion); refinement and coarsening of the blocks are
 * those of the forest-of-octrees scheme (Sec. II-C-1).  A step of a moving
 * body imports the moved faces, bins them and refines from the roots (the
 * re-adapted forest is the near-wall forest of the new geometry); this call
 * then relates it to the previous forest, level by level, for a solver to
 * carry its block data over.  Both forests must share dimension, root grid,
 * domain and level count; they may come from different geometries.
 * Per level l, device arrays owned by the diff (valid until it is destroyed):
 *   d_old_index[n_new] int32  position of each new block in the old level l,
 *                             -1 when the old level has no such key;
 *   d_state[n_new]     uint8  0 kept (same key and leaf bit), 1 created,
 *                             2 refined (a leaf before, now with children),
 *                             3 coarsened (children before, now a leaf: they
 *                             are removed at level l + 1);
 *   d_removed[n_old]   uint8  1 when the old block's key is absent from the
 *                             new level l;
 *   counts[4]                 created, refined, coarsened, removed blocks.
 * Synchronises `stream` once (to read the counts).
 * Errors: AGAL_EINVAL for NULL arguments or forests over different grids. */
AGAL_API agal_status agal_forest_diff_create(agal_forest old_forest, agal_forest new_forest, void *stream,
                                             agal_forest_diff *out);
AGAL_API agal_status agal_forest_diff_view(agal_forest_diff d, int level, const int32_t **d_old_index,
                                           const uint8_t **d_state, const uint8_t **d_removed, int64_t *n_new,
                                           int64_t *n_old, int64_t counts[4]);
AGAL_API void agal_destroy_forest_diff(agal_forest_diff d);

/* ---- link fractions (Sec. II-C-1) ----------------------------------------
 * For every cell of every block of the finest level and every non-rest
 * direction c_i of `lattice`, q_i is the smallest t in [0, 1] at which the
 * segment x + t c_i dx_L (x the cell centre) meets a face (closed faces, both
 * orientations), and face_i the lowest face id attaining it; -1 / -1 when
 * there is none (and always for the rest direction).  Cells with at least one
 * link are emitted in ascending node key = block_key * 4^D + cell.
 * Outputs: d_node_key[n_nodes] uint64, d_q[n_nodes * Q] FP32,
 * d_face[n_nodes * Q] int32, row-major by node.
 * Errors: AGAL_EINVAL when the lattice does not match the dimension;
 * AGAL_ESTATE when the handles come from different geometries.
 * Synchronises `stream` once to read the node count. */
AGAL_API agal_status agal_link_fractions(agal_geom g, agal_bins b, agal_forest f, int lattice, void *stream,
                                         agal_links *out);
AGAL_API agal_status agal_links_view(agal_links l, const uint64_t **d_node_key, const float **d_q,
                                     const int32_t **d_face, int64_t *n_nodes, int *Q);
/* How agal_link_fractions finds each finest-level block's candidate faces
 * (the results are identical either way).  List mode: every face lists the
 * blocks whose link box its bounding box meets (face-side, a few blocks per
 * face), then one pass finds the cells that have a link and a second writes
 * each node's row at its final place.  Walk mode: each block walks the bins
 * under it, and nodes are staged per block and compacted.  A call takes list
 * mode while the geometry's largest face (box extent per axis, measured at
 * import) has at most max_blocks_per_face candidate blocks at the finest
 * level; default 512, 0 selects walk mode always.  Applies to calls made with
 * ctx afterwards.
 * Errors: AGAL_EINVAL for a NULL context or a negative limit. */
AGAL_API agal_status agal_context_set_link_list_limit(agal_context ctx, int64_t max_blocks_per_face);

/* ---- adjoint ---------------------------------------------------------------
 * Accumulates dL/d(vertex) for L = sum over link slots of grad_q * q:
 * each slot with face >= 0 adds grad_q * lambda_k * n / (D . n) to vertex k
 * of its face (lambda the barycentric weights of the hit, n a face normal,
 * D = c_i dx_L), through the index list given at import.
 *   d_grad_q        n_nodes x Q FP32 (slots with face < 0 are ignored);
 *   d_grad_vertices n_vertices x dim FP32, ACCUMULATED into (the caller
 *                   zeroes it); for a coordinate-list import the "vertices"
 *                   are the n_faces*dim corners.
 * The hit is recomputed in FP32 with the denominator D . n in FP64 when the
 * ray grazes the face.  Float atomics make the summation order vary between
 * runs (results agree to rounding).
 * Errors: AGAL_ESTATE when `l` was not computed from `g`. */
AGAL_API agal_status agal_link_fractions_backward(agal_geom g, agal_links l, const float *d_grad_q,
                                                  float *d_grad_vertices, void *stream);

/* ---- node classification ---------------------------------------------------
 * The step after the link fractions that the paper leaves to future work
 * (Results discussion, Conclusion): the side of every boundary node of `l`,
 * read from the orientation of the faces its links meet.  The surface must be
 * closed and oriented so that n = (b - a) x (c - a) (3D) or n = (e_y, -e_x),
 * e = b - a (2D) points out of the solid (counter-clockwise loops in 2D).  A
 * link entering the solid has c_i . n < 0, one leaving it c_i . n > 0; the
 * sign is evaluated in FP64 from the FP32 corners.
 *   d_class  n_nodes uint8, caller-owned, in the order of agal_links_view:
 *            1 fluid (every link enters), 2 solid (every link leaves),
 *            3 mixed (links disagree, or one meets its face along the face's
 *            plane: a link grazing an edge or corner of the solid).
 * Errors: AGAL_ESTATE when `l` was not computed from `g`; AGAL_EINVAL for a
 * NULL handle or output. */
AGAL_API agal_status agal_classify_nodes(agal_geom g, agal_links l, uint8_t *d_class, void *stream);

/* ---- batched form: many bodies, one graph launch --------------------------
 * Each body is a complete near-wall problem (import, bins, refinement, link
 * fractions and optionally the adjoint) with its own geometry, forest, bins
 * and lattice.  A plan sizes every body once with the calls above, reserves
 * device capacity for all intermediate arrays (measured sizes times
 * 1 + capacity_margin), and captures one hipGraph of persistent kernels that
 * process all bodies together; every size stays on the device.  Each run is a
 * single hipGraphLaunch with no host synchronisation.  Flags and link
 * fractions are bit-identical to the single-body calls on the same input.
 *
 * Body inputs are device pointers that must stay valid and keep their shapes
 * while the plan lives; their values may change between runs (the plan
 * re-reads them).  If a run outgrows a capacity, the arrays concerned stop
 * growing, the results of that run are incomplete and agal_batch_status
 * returns AGAL_ECAPACITY: create a new plan.
 */
typedef struct agal_body_desc {
    int dim;
    const float *d_vertices;       /* n_vertices x dim FP32 */
    int64_t n_vertices;
    const int32_t *d_faces;        /* n_faces x dim int32; NULL: coordinate list */
    int64_t n_faces;
    agal_forest_desc forest;       /* forest.d_spec is read during plan creation */
    int lattice;
    int32_t bins;                  /* bins per axis; <= 0: chosen by the tuner */
} agal_body_desc;

typedef struct agal_tune_opts {
    int tune_bins;                 /* 1: time candidate bin densities per face-count bucket */
    int tune_grid;                 /* 1: time persistent grids of 1, 2, 4, 8 workgroups per CU */
    int with_adjoint;              /* 1: the graph ends with the adjoint of every body */
    float capacity_margin;         /* extra fraction of each measured size (0: 0.25) */
    const char *cache_path;        /* text file of tuned bin densities, read and extended; NULL: none */
} agal_tune_opts;

/* Plans and captures the batch (synchronises `stream`; runs every body once
 * on it).  n_bodies in [1, 256]; bodies of one plan share the dimension.
 * Errors: as the single-body calls for each body; AGAL_EINVAL for an empty or
 * oversized batch. */
AGAL_API agal_status agal_batch_plan_create(agal_context ctx, int n_bodies, const agal_body_desc *bodies,
                                            const agal_tune_opts *opts, void *stream, agal_batch *out);
/* Enqueues one run (one graph launch) on `stream`. */
AGAL_API agal_status agal_batch_run(agal_batch b, void *stream);
/* Synchronises `stream`, reads the per-body sizes of the last run, and
 * returns AGAL_ECAPACITY if a capacity overflowed, AGAL_EINVAL if an input was
 * invalid (non-finite coordinate or index out of range), AGAL_ESTATE if a
 * forest lost 2:1 balance. */
AGAL_API agal_status agal_batch_status(agal_batch b, void *stream);
/* Results of body `body` after agal_batch_status: node keys, q and faces as
 * agal_links_view; *d_grad_q is where the caller writes the n_nodes x Q
 * adjoint input before a run (plans with the adjoint; capacity
 * *node_capacity rows), *d_grad_vertices the n_vertices x dim result (zeroed
 * by every run). */
AGAL_API agal_status agal_batch_body_view(agal_batch b, int body, const uint64_t **d_node_key, const float **d_q,
                                          const int32_t **d_face, int64_t *n_nodes, int *Q, float **d_grad_q,
                                          const float **d_grad_vertices, int64_t *node_capacity, int32_t *bins);
/* Forest level of body `body` after agal_batch_status (layout as
 * agal_forest_level_view). */
AGAL_API agal_status agal_batch_level_view(agal_batch b, int body, int level, const uint32_t **d_keys,
                                           const uint8_t **d_leaf, const uint8_t **d_mark,
                                           const uint8_t **d_cell_flag, int64_t *n_blocks);
/* Persistent grid chosen by the plan (workgroups per CU). */
AGAL_API agal_status agal_batch_info(agal_batch b, int *n_bodies, int *workgroups_per_cu);
AGAL_API void agal_destroy_batch(agal_batch b);

/* ---- kernel timing -------------------------------------------------------
 * With profiling enabled, every kernel the library launches with `ctx` is
 * bracketed by HIP events recorded on its launch stream.  agal_profile_read
 * waits for the recorded events, aggregates them per kernel name (launch
 * count and total milliseconds, in order of first appearance, at most
 * max_entries names), stores the count in *n_entries and clears the record.
 * Names are static strings owned by the library. */
AGAL_API agal_status agal_profile_enable(agal_context ctx, int enable);
AGAL_API agal_status agal_profile_read(agal_context ctx, int max_entries, const char **names, int64_t *launches,
                                       double *total_ms, int *n_entries);

/* ---- misc -------------------------------------------------------------- */
AGAL_API agal_status agal_lattice_vectors(int lattice, int32_t *c /* host, lattice x 3 */);
AGAL_API void agal_destroy_geom(agal_geom g);
AGAL_API void agal_destroy_bins(agal_bins b);
AGAL_API void agal_destroy_forest(agal_forest f);
AGAL_API void agal_destroy_links(agal_links l);
AGAL_API const char *agal_status_string(agal_status s);
AGAL_API const char *agal_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AGAL_H */
