/*
 * trimap: triangular-domain GPU kernels driven by the block-space map
 * lambda(omega), for AMD Instinct MI355X (gfx950).  C ABI.
 *
 * Method: C. A. Navarro, B. Bustos, N. Hitschfeld, "A Non-linear GPU Thread
 * Map for Triangular Domains" (arXiv 1609.01490).
 *
 * Conventions common to every entry point
 * ---------------------------------------
 *  - Every function returns a tri_status; nothing aborts or exits.  On error
 *    tri_last_error() returns a message for the calling thread.
 *  - Pointers named dev_* / x / y / c / cur / nxt / out / ws are DEVICE
 *    pointers owned by the caller; the library never frees them and never
 *    allocates device memory inside a launch call.  Host pointers are named
 *    explicitly (host_*).
 *  - `stream` is a hipStream_t passed as void* (NULL: the null stream).  All
 *    launches are asynchronous and ordered on that stream.
 *  - Matrices are row-major with a leading dimension `ld` in ELEMENTS.
 *  - Triangular domain of side n: cells (i, j) with 0 <= j <= i < n
 *    (include_diag = 1) or 0 <= j < i < n (include_diag = 0).
 *  - A plan is immutable after creation (apart from its cache of stencil
 *    graphs, guarded by a lock); concurrent launches of one plan on
 *    different streams are safe.
 */
#ifndef TRIMAP_H
#define TRIMAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TRI_OK = 0,
    TRI_E_INVAL = 1,       /* bad argument: null pointer, bad enum, ld < n, misalignment */
    TRI_E_RANGE = 2,       /* sizes beyond the index or grid limits */
    TRI_E_NOMEM = 3,       /* host allocation failed, or workspace too small */
    TRI_E_HIP = 4,         /* a HIP runtime call failed (message kept) */
    TRI_E_UNSUPPORTED = 5  /* valid request the library does not implement */
} tri_status;

/* Parallel-space maps (Section 4.2 of the paper; lambda: Section 3.1). */
typedef enum {
    TRI_MAP_BB = 0,     /* bounding box: m x m blocks, upper blocks discarded   */
    TRI_MAP_RB = 1,     /* rectangular box: the triangle folded to a rectangle  */
    TRI_MAP_REC = 2,    /* recursive partition (m a power of two)               */
    TRI_MAP_UTM = 3,    /* upper-triangular map, thread space (Avril et al.)    */
    TRI_MAP_LAMBDA = 4  /* lambda(omega): exactly m(m+1)/2 blocks (Eq. eq_gmap) */
} tri_map;

/* Plan flags (bit set). */
enum {
    TRI_FLAG_XCD_SWIZZLE = 1u, /* lambda: give each XCD a contiguous range of omega   */
    TRI_FLAG_SQRT_RSQ = 2u,    /* lambda: sqrt(x) as x * rsq(x) (the paper's lambda_R) */
    TRI_FLAG_SQRT_F64 = 4u,    /* lambda: FP64 square root                             */
    TRI_FLAG_ORDER_REVERSE = 8u, /* lambda: dispatch omega from T-1 down to 0            */
    TRI_FLAG_ORDER_PAIRS = 16u,  /* lambda: alternate omega from the front and the back  */
    TRI_FLAG_LIFE_TEMPORAL = 32u, /* stencil: several generations per launch (wider halo) */
    TRI_FLAG_SQRT_NEWTON = 64u,  /* lambda: bit-trick rsqrt + 3 Newton steps (lambda_N)  */
    /* lambda, for the square-root study only: the paper's inexact row
     * floor(sqrt(1/4 + 2 omega) + 1e-4 - 1/2) without the integer
     * correction, with the square root the other SQRT flags select.  Wrong
     * for some omega (tiles missed or repeated; never outside the domain). */
    TRI_FLAG_SQRT_EPS = 128u
};

/* Plan flags, bits 8..11: the number of consecutive tiles of the map that one
 * workgroup walks in the kernels that take strips (the distance map's MFMA
 * modes, the fp32 elementwise kernel at tiles 16 and 32 with 16-byte rows,
 * the bit-sliced Life kernel at tile 64 with 16-byte rows):
 * TRI_FLAG_STRIP(k) asks for G = 2^k tiles (k = 0..5, G = 1..32); none of
 * these bits set: G chosen from the tile count in the distance map, one
 * tile per workgroup elsewhere.  Kernels without strips ignore them. */
#define TRI_FLAG_STRIP_MASK 0xF00u
#define TRI_FLAG_STRIP(k) ((uint32_t)((k) + 1) << 8)
/* Plan flag for the same kernels under lambda: strips aligned to tile rows
 * (strip c of tile row i holds the row's tiles c G .. c G + G - 1) and
 * taken column by column (strip c of every row before strip c + 1), so that
 * the workgroups running together share their column tiles.  Without it a
 * strip is G consecutive omega in row order (it may cross a row end). */
#define TRI_FLAG_STRIP_COLS 0x1000u
/* Plan flag for the same kernels under lambda: strips aligned to tile rows
 * as with TRI_FLAG_STRIP_COLS, taken row by row (every strip of tile row i
 * before row i + 1), so that each strip's first tile column is a multiple
 * of G.  TRI_FLAG_STRIP_COLS takes precedence. */
#define TRI_FLAG_STRIP_ALIGN 0x2000u
/* Plan flag for the distance map's matrix-core modes (up to 128
 * dimensions): the pipelined kernel, one workgroup per CU, the column
 * operands of two tiles in LDS and each tile's stores interleaved with the
 * next tile's products. */
#define TRI_FLAG_EDM_PIPE 0x4000u
/* Plan flag for the elementwise strip kernels (tiles 16 and 32, strips of
 * G >= 4 tiles): two-row bands.  A strip holds G / 2 columns of two
 * consecutive tile rows (lambda) or grid rows (BB, RB, REC), so that a
 * workgroup meets each 2 x 2 block of tiles at once; every tile is still
 * located by the map on its own (under lambda, tile (2p + r, c) is omega
 * T_{2p+r} + c).  TRI_FLAG_STRIP_COLS and TRI_FLAG_STRIP_ALIGN take
 * precedence.  The distance map and the stencil reject it. */
#define TRI_FLAG_STRIP_BAND 0x8000u
/* Plan flag for the bit-sliced Life strips (tile 64, 16-byte rows), in
 * both forms (one generation with the paper's 1-cell halo, and with
 * TRI_FLAG_LIFE_TEMPORAL up to 16 generations with a 16-cell halo): a wave
 * moves tiles 2 j and 2 j + 1 of its strip as one window two tiles wide
 * when they are neighbours in a tile row (every row segment a whole
 * 128-byte line; the temporal window's halo shares the edge words with the
 * tiles), each tile still located by the map on its own; any other tile
 * in a window of its own, of which only that tile is written back.
 * Section 5's shared-memory test; the pairing is a scheduling choice
 * outside the paper. */
#define TRI_FLAG_LIFE_WIDE 0x10000u

/* Elementwise bodies. */
enum {
    /* C[i][j] = (A[i] XOR B[j]) + i*j, uint32 wrap-around; x = A (uint32[n]),
     * y = B (uint32[n]), c = C (int32 n x ld).  Dummy-kernel role, Sections 4.1 and 5. */
    TRI_OP_XORMUL_I32 = 0,
    /* C[i][j] = fl(fl(a * X[i][j]) + Y[j][i]), two binary32 roundings, no
     * fused multiply-add; x = X, y = Y, c = C (float n x ld each). */
    TRI_OP_AXPYT_F32 = 1,
    /* Euclidean distance of four features, the global-memory distance test
     * of Section 5: x = P (float[n][4], 16-byte aligned), y unused (may be
     * NULL), c = C (float n x ld).  With p = P[i], q = P[j] and every step
     * rounded to binary32 (no fused multiply-add):
     * C[i][j] = sqrt(((dx*dx + dy*dy) + dz*dz) + dw*dw), d. = p. - q.,
     * with a correctly rounded square root; C[i][i] = 0. */
    TRI_OP_EDM4_F32 = 2
};

/* Distance-map arithmetic. */
enum {
    TRI_EDM_FP32 = 0,   /* direct sum of squared differences in FP32                */
    TRI_EDM_BF16X3 = 1, /* centred split-BF16 Gram on MFMA (hi*hi + hi*lo + lo*hi)  */
    TRI_EDM_BF16 = 2    /* centred single-BF16 Gram on MFMA (faster, less accurate) */
};

typedef struct tri_plan tri_plan;

typedef struct {
    int64_t n;             /* side of the domain                                     */
    int64_t tile;          /* rho: tile side in cells                                */
    int64_t m;             /* tiles per side = ceil(n_eff / rho), n_eff = n or n-1    */
    int64_t tiles;         /* m (m + 1) / 2                                          */
    int64_t grid_x;        /* launch grid in blocks                                  */
    int64_t grid_y;
    int64_t grid_blocks;   /* grid_x * grid_y                                        */
    int64_t wasted_blocks; /* blocks of the grid that map to no tile                 */
    int64_t elements;      /* cells of the domain: n(n+1)/2 or n(n-1)/2              */
    int64_t dump_entries;  /* entries written by tri_map_dump                         */
    int32_t map;
    int32_t include_diag;
    uint32_t flags;
    int32_t reserved;
} tri_plan_info;

/* Create a plan for a triangular domain of side n (0 <= n < 2^31) tiled in
 * rho x rho tiles, rho in {8, 16, 32, 64}, under one of the five maps.
 * Tile space (Section 3.1): m = ceil(n_eff / rho) tiles per side with
 * n_eff = n (include_diag = 1) or n - 1 (include_diag = 0: the strict lower
 * triangle is handled as the diagonal-including triangle of side n - 1
 * shifted down one row, which is Eq. eq_theorem_nodiag at rho = 1).
 * Grids: BB m x m; lambda 1-D of m(m+1)/2 blocks; RB m x (m+1)/2 (m odd) or
 * (m+1) x m/2 (m even); REC m/2 x (m+1), m a power of two, else
 * TRI_E_UNSUPPORTED; UTM one thread per cell (thread space).
 * *out receives a host object freed by tri_plan_destroy. */
tri_status tri_map_plan(tri_plan **out, int64_t n, int tile, int map, int include_diag,
                        uint32_t flags);
tri_status tri_plan_destroy(tri_plan *plan);
tri_status tri_plan_query(const tri_plan *plan, tri_plan_info *info);

/* Test hook: write the map itself.  Tile maps: for grid block
 * b = by * grid_x + bx, dev_out[2b], dev_out[2b+1] = its tile (bi, bj) or
 * (-1, -1) when discarded.  UTM: for thread k < elements, the cell (i, j).
 * dev_out holds 2 * dump_entries int64. */
tri_status tri_map_dump(const tri_plan *plan, int64_t *dev_out, void *stream);

/* Test hook: lambda(omega) (include_diag = 1, Eq. eq_gmap) or its variant
 * without diagonal (Eq. eq_theorem_nodiag), evaluated by the device code for
 * count arbitrary omega < 2^60 from dev_omega (uint64); writes
 * dev_out[2t], dev_out[2t+1] = (i, j).  flags selects the square root
 * (TRI_FLAG_SQRT_*). */
tri_status tri_lambda_eval(const uint64_t *dev_omega, int64_t count, int include_diag,
                           uint32_t flags, int64_t *dev_out, void *stream);

/* Apply an elementwise body to every cell of the plan's domain
 * (include_diag must be 1).  Cells j > i and rows >= n are never written.
 * Requirements: ld >= n; for TRI_OP_AXPYT_F32 x, y, c all n x ld with the
 * same ld; for TRI_OP_XORMUL_I32 x, y hold n uint32 and c is n x ld int32;
 * for TRI_OP_EDM4_F32 x holds n 16-byte-aligned points of four floats.
 * Rows are accessed 16 bytes at a time when ld % 4 == 0 and the matrix
 * pointers are 16-byte aligned, one element at a time otherwise.
 * `a` is used by TRI_OP_AXPYT_F32 only. */
tri_status tri_launch_elementwise(const tri_plan *plan, int op, const void *x, const void *y,
                                  void *c, int64_t ld, float a, void *stream);

/* The dummy kernel of the square-root study (Section 4.1): every cell
 * (i, j) of the plan's domain (any map, tile 8 to 64, with or without the
 * diagonal) forms its coordinates through the map and computes i + j; cells
 * with i + j == target store that sum to sink[0] (device int32).  A target
 * no cell reaches (e.g. -1) writes nothing, so the launch costs the
 * dispatch, the map (TRI_FLAG_SQRT_* variants included) and the per-cell
 * test alone. */
tri_status tri_launch_dummy(const tri_plan *plan, int32_t target, int32_t *sink, void *stream);

/* ---- Tetrahedral domains (Section 6) ------------------------------------- */

/* A plan for the tetrahedron of n points tiled in rho^3 tiles (rho in {8,
 * 16, 32, 64}): tiles (i, j, k), 0 <= i <= j <= k < m, m = ceil(n_eff / rho),
 * Tet(m) = m(m+1)(m+2)/6 of them.  strict = 1 covers the triples
 * a > b > c of n points (the non-strict tetrahedron of side n_eff = n - 2,
 * shifted: (a, b, c) = (k + 2, j + 1, i) per point), strict = 0 the triples
 * a >= b >= c (n_eff = n).  map: TRI_MAP_LAMBDA (1-D grid of Tet(m) blocks;
 * block omega's layer k is the largest with Tet(k) <= omega, from a cube
 * root and an exact integer correction, the rest of omega through the 2-D
 * lambda) or TRI_MAP_BB (m x m x m grid, blocks with i <= j <= k kept;
 * m <= 65535).  flags: 0 (FP32 roots below 2^32) or TRI_FLAG_SQRT_F64 (FP64
 * roots).  n < 2^21.  Freed by tri_tet_destroy. */
typedef struct tri_tet tri_tet;
tri_status tri_tet_plan(tri_tet **out, int64_t n, int tile, int map, int strict, uint32_t flags);
tri_status tri_tet_destroy(tri_tet *plan);
/* Tiles Tet(m), launched grid blocks, and triples in the domain (any
 * pointer may be NULL). */
tri_status tri_tet_query(const tri_tet *plan, int64_t *tiles, int64_t *grid_blocks, int64_t *cells);

/* Test hook: for grid block b (b = (bz gy + by) gx + bx), dev_out[3b..3b+2]
 * = its tile (i, j, k), or -1 three times when the block is discarded. */
tri_status tri_tet_dump(const tri_tet *plan, int64_t *dev_out, void *stream);

/* Test hook: the tetrahedral lambda of count arbitrary omega < 2^62
 * (uint64) into dev_out[3t..3t+2] = (i, j, k); flags as for the plan. */
tri_status tri_lambda3_eval(const uint64_t *dev_omega, int64_t count, uint32_t flags,
                            int64_t *dev_out, void *stream);

/* A triplet kernel over the strict tetrahedron: triangles of the neighbour
 * graph of n points (rows (x, y, z, unused) of `points`, FP32, 16-byte
 * aligned).  Points a and b are neighbours when, in binary32 without fused
 * multiply-add, ((dx^2 + dy^2) + dz^2) < r2 with d. = a. - b.  Every triple
 * a > b > c of mutual neighbours is a triangle: counts[v] (int32[n]) gets the
 * number of triangles with vertex v, *total (uint64, 8-byte aligned) their
 * number; the call clears both first.  The plan must be strict. */
tri_status tri_triangles(const tri_tet *plan, const float *points, float r2, int32_t *counts,
                         unsigned long long *total, void *stream);

/* The dummy kernel on the tetrahedron: each triple (a, b, c) of the plan's
 * domain forms its indices through the map and computes a + b + c; triples
 * with a + b + c == target store it to sink[0] (device int32). */
tri_status tri_tet_dummy(const tri_tet *plan, int32_t target, int32_t *sink, void *stream);

/* Game of Life B3/S23 on the lower triangle (include_diag must be 1): the
 * cellular automaton on a triangular domain that the Introduction (Section
 * 1) names among the problems the map serves, run with the shared-memory
 * tile pattern of the collision test of Section 5 (each tile and its halo
 * staged on chip).  The
 * tile maps stage each tile with a one-cell halo in LDS; UTM (thread space)
 * has no 2-D block, so its threads read their eight neighbours from global
 * memory (and it has no temporal blocking).  cur and nxt
 * are uint8 n x ld grids whose domain cells hold 0 or 1; cells above the
 * diagonal are treated as dead whatever they hold, and are never written.
 * Runs `steps` synchronous generations, reading cur and writing nxt, then
 * the other way round: the result is in cur when steps is even, in nxt when
 * odd.  Requires ld % 4 == 0, ld >= n, 4-byte aligned pointers, steps >= 0.
 * With TRI_FLAG_LIFE_TEMPORAL in the plan (tiles 16, 32, 64; no graph) one
 * launch advances up to four generations from a tile staged with a 4-cell
 * halo (up to sixteen with a 16-cell halo for 64 x 64 tiles on grids of at
 * least 512 tiles whose ld is a multiple of 16 and whose buffers are
 * 16-byte aligned), the number of launches keeping the parity of `steps`.
 * Tile 64 with ld a multiple of 16 and 16-byte aligned buffers also runs
 * bit-sliced without the flag (same results).  Otherwise
 * each generation is one kernel launch; when use_graph is non-zero the
 * generations are built once into a hipGraph of kernel nodes for this
 * (cur, nxt, ld, steps), kept with the plan and replayed by every later call
 * with the same arguments (the graph is freed by tri_plan_destroy, which must
 * then not race with launches still in flight). */
tri_status tri_launch_stencil(const tri_plan *plan, uint8_t *cur, uint8_t *nxt, int64_t ld,
                              int steps, int use_graph, void *stream);

/* Euclidean distance map (the EDM test of Section 5): for the plan's strict
 * lower triangle (include_diag must be 0; any tile map but UTM), writes
 * d(i, j) = sqrt(sum_k (x_ik - x_jk)^2) in FP32 to out[i(i-1)/2 + j] (the
 * condensed strict lower triangle, n(n-1)/2 floats; n(n-1)/2 < 2^32).  x is
 * n x d FP32 (1 <= d <= 4096), leading dimension ldx >= d, 4-byte aligned.
 * mode is a TRI_EDM_* value:
 *  - TRI_EDM_FP32: plan tile 16, 32, 64 or 128; no workspace (ws may be NULL).
 *  - TRI_EDM_BF16X3 / TRI_EDM_BF16: plan tile 128; `out` 16-byte aligned
 *    (rows are written as 16-byte vectors); ws a device buffer of at least
 *    tri_edm_workspace_size() bytes, 256-byte aligned, else TRI_E_NOMEM /
 *    TRI_E_INVAL.  Distances whose Gram-based square is below fixup_thr
 *    (>= 0) are recomputed directly in FP32 from x.
 * tri_edm_workspace_size returns the workspace bytes for (plan, d, mode),
 * 0 for TRI_EDM_FP32, and TRI_E_UNSUPPORTED when the plan's tile does not
 * fit the mode. */
tri_status tri_edm_workspace_size(const tri_plan *plan, int64_t d, int mode, size_t *bytes);
tri_status tri_edm(const tri_plan *plan, const float *x, int64_t d, int64_t ldx, float *out,
                   int mode, float fixup_thr, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): tri_edm
 * with the MFMA modes' workspace taken from a scratch array the library
 * holds on each GPU it runs on (TRI_EDM_NOALLOC_SCRATCH_BYTES, kept until
 * the process ends).  Same arguments, kernels and results as tri_edm;
 * TRI_EDM_FP32 needs no workspace and runs as tri_edm does.  A request
 * whose workspace (tri_edm_workspace_size) exceeds the scratch returns
 * TRI_E_RANGE and launches nothing (with d = 128 that is n above about
 * 32000 points).  The call allocates nothing, on the device or the host
 * heap; the first call on a device looks up that device's scratch address.
 * Every call on one GPU shares that GPU's scratch and nothing in it needs
 * to start cleared: calls that overlap in time on one GPU (other streams,
 * other threads) race and must be serialised by the caller. */
#define TRI_EDM_NOALLOC_SCRATCH_BYTES (16u << 20)
tri_status tri_edm_noalloc(const tri_plan *plan, const float *x, int64_t d, int64_t ldx,
                           float *out, int mode, float fixup_thr, void *stream);

/* Collision detection of n spheres (the shared-memory test of Section 5).
 * The plan covers the strict lower triangle (include_diag must be 0); any
 * map, tile 8, 16, 32, 64 or 128 (tile maps stage both blocks of spheres in
 * LDS; UTM reads them from global memory per pair).  spheres is n x 4 FP32
 * rows (x, y, z, r), 16-byte aligned; dim is 3, or 1 (only x and r are
 * read).  Spheres a and b overlap when, in binary32 without fused
 * multiply-add, s < (r_a + r_b)^2 with s = dx^2 (+ dy^2) (+ dz^2) summed left
 * to right (d. = a. - b.); touching spheres (equality) and NaN coordinates
 * do not overlap.  counts (int32[n], device, 4-byte aligned) is cleared by
 * the call and then receives, for every sphere, the number of other spheres
 * it overlaps.  Stream-ordered, no host synchronisation, no allocation. */
tri_status tri_collide(const tri_plan *plan, const float *spheres, int dim, int32_t *counts,
                       void *stream);

/* ------------------------------------------------------------------------
 * Batched uneven domains in one persistent launch per generation.
 *
 * Instance k (0 <= k < count) is a distance map (TRI_KIND_EDM: strict lower
 * triangle of n_k points in d_k dimensions, FP32 direct arithmetic, edm_tile
 * in {16, 32, 64}) or a Game of Life (TRI_KIND_LIFE: lower triangle of side
 * n_k, life_tile in {8, 16, 32, 64}, life_steps generations).  Each instance
 * contributes m_k (m_k + 1) / 2 tiles (Section 3.1); a global work item g is
 * located by the exclusive prefix sum of these counts and mapped to its tile
 * by lambda(g - P_k) (Eq. eq_gmap).  Persistent workgroups take items from an
 * atomic counter; generation s of the Life instances is one kernel, so the
 * whole batch is one hipGraph (a counter-reset node, then one node per
 * generation; distance-map items run in generation 0).  Results equal the
 * per-instance kernels bit for bit.
 * ------------------------------------------------------------------------ */
typedef struct tri_batch tri_batch;

enum { TRI_KIND_EDM = 0, TRI_KIND_LIFE = 1 };

/* How tri_batch_launch runs the batch. */
enum {
    TRI_BATCH_GRAPH = 0,        /* one hipGraphLaunch of the instantiated graph       */
    TRI_BATCH_STREAM = 1,       /* the same persistent kernels launched on the stream */
    TRI_BATCH_PER_INSTANCE = 2  /* one launch per instance and generation (baseline)  */
};

typedef struct {
    int32_t count;
    int32_t life_instances;
    int32_t edm_tile;
    int32_t life_tile;
    int32_t life_steps;
    int32_t persistent_workgroups;
    int32_t graph_nodes;                 /* kernel nodes after the counter reset   */
    int32_t reserved;
    int64_t items_generation0;          /* tiles in generation 0                  */
    int64_t items_per_later_generation; /* Life tiles in each later generation    */
} tri_batch_info;

/* Plan a batch from host arrays kind[count], n[count], d[count] (d ignored
 * for Life).  flags: 0 or TRI_FLAG_LIFE_TEMPORAL (life_tile >= 16: each node
 * advances the Life instances by up to four generations, as in
 * tri_launch_stencil; the number of nodes keeps the parity of life_steps).
 * Needs the device that will run it to be current: it queries the CU count
 * and occupancy and allocates the plan's own device arrays (prefix sums,
 * instance descriptors, counters).  n_k < 2^20; at most 2^31 tiles per
 * generation. */
tri_status tri_batch_plan(tri_batch **out, int32_t count, const int32_t *host_kind,
                          const int64_t *host_n, const int64_t *host_d, int edm_tile,
                          int life_tile, int life_steps, uint32_t flags);

/* Bind the instances' device buffers (host arrays of device pointers):
 * distance map k: a[k] = x (n_k x d_k FP32, leading dimension ld[k] >= d_k),
 * b[k] = condensed output (n_k (n_k - 1) / 2 FP32); Life k: a[k] = the grid
 * holding generation 0 on entry, b[k] = the other grid (both uint8, row
 * pitch ld[k] >= n_k, a multiple of 4).  After an even number of
 * generations the Life result is in a[k], after an odd number in b[k].
 * When the plan has life_tile 64 with TRI_FLAG_LIFE_TEMPORAL and every Life
 * grid has a pitch that is a multiple of 16 and 16-byte aligned buffers,
 * the bound kernel moves Life tiles bit-sliced, one per wave, with 16-byte
 * row loads and stores (same results).  Copies the descriptors to the
 * device (synchronously) and builds and instantiates the graph.  Rebinding
 * replaces both. */
tri_status tri_batch_bind(tri_batch *b, void *const *host_a, void *const *host_b,
                          const int64_t *host_ld);

/* Run the bound batch on `stream` (how = TRI_BATCH_*).  Launches of one
 * batch plan share its counters: calls that overlap in time race. */
tri_status tri_batch_launch(tri_batch *b, int how, void *stream);
tri_status tri_batch_query(const tri_batch *b, tri_batch_info *info);
tri_status tri_batch_destroy(tri_batch *b);

/* Autotune the tiles of a batch: plans, binds and times (one warm-up, then
 * `reps` graph launches with HIP events on `stream`) every edm_tile in
 * {16, 32, 64} with every life_tile in {8, 16, 32, 64} (one generation per
 * node) and in {16, 32, 64} with TRI_FLAG_LIFE_TEMPORAL, on the given
 * instances and buffers (arguments as for tri_batch_plan and tri_batch_bind),
 * and returns the fastest choice (best_flags may be NULL) and its time per
 * launch.  The buffers are used for real: distance-map outputs are
 * rewritten and the Life grids advance by (reps + 1) * life_steps
 * generations per candidate. */
tri_status tri_batch_autotune(int32_t count, const int32_t *host_kind, const int64_t *host_n,
                              const int64_t *host_d, int life_steps, void *const *host_a,
                              void *const *host_b, const int64_t *host_ld, int reps, void *stream,
                              int *best_edm_tile, int *best_life_tile, uint32_t *best_flags,
                              float *best_ms);

/* ------------------------------------------------------------------------
 * Autotuner: tile size and map for a workload and problem size.  Not part
 * of the paper's method (its Section 5 compares the maps at fixed sizes);
 * a tool of this library that picks among the paper's maps on this GPU.
 *
 * tri_autotune times every candidate (tiles 8/16/32/64 — plus 128 for the
 * fp32 elementwise body, 16/32/64/128 for the FP32 distance map, 128 for the
 * MFMA one — times maps BB, RB, REC (when
 * m is a power of two) and lambda, the latter plain, with
 * TRI_FLAG_XCD_SWIZZLE, TRI_FLAG_ORDER_REVERSE, TRI_FLAG_ORDER_PAIRS and
 * swizzle + pairs, plus UTM for the elementwise bodies and Life) on this
 * GPU: one warm-up and `reps` timed calls, each between two HIP events on
 * `stream`, ranked by the median of the calls, on scratch buffers of the
 * problem's size that it allocates and frees itself (so it is not for graph
 * capture): zeroed, except the distance maps' coordinates, uniform in
 * [0, 1) (all-equal points would time the near-duplicate recompute of every
 * pair).  d is the dimension of the distance maps; for Life it is the
 * number of generations of one timed call (0: 32), so that a caller ranks
 * the candidates on the schedule it runs.  Life candidates include
 * TRI_FLAG_LIFE_TEMPORAL for BB and lambda at tiles 16..64 (lambda plain,
 * swizzled, or swizzled in the pairs order); Life times are reported per
 * generation.  The fastest candidate goes to *best and into a process-wide
 * cache keyed by GPU architecture, CU count, workload, floor(log2 n) and d
 * (distance maps and Life); with
 * use_cache non-zero a cached entry is returned without timing.  When `all`
 * is non-NULL up to all_cap timed candidates are written there and their
 * number to *all_count.
 * ------------------------------------------------------------------------ */
enum {
    TRI_TUNE_ELEMENTWISE_F32 = 0,
    TRI_TUNE_ELEMENTWISE_I32 = 1,
    TRI_TUNE_LIFE = 2,
    TRI_TUNE_EDM_FP32 = 3,
    TRI_TUNE_EDM_BF16X3 = 4
};

typedef struct {
    int32_t tile;
    int32_t map;
    uint32_t flags;
    float ms; /* mean time of one call (Life: one generation) */
} tri_tune_choice;

tri_status tri_autotune(int workload, int64_t n, int64_t d, int reps, int use_cache, void *stream,
                        tri_tune_choice *best, tri_tune_choice *all, int32_t all_cap,
                        int32_t *all_count);
/* Save / load / clear the tuning cache (a small JSON file, one entry per
 * line: arch, cus, workload, bucket, d, tile, map, flags, ms). */
tri_status tri_tune_cache_save(const char *path);
tri_status tri_tune_cache_load(const char *path);
tri_status tri_tune_cache_clear(void);

/* Measurement probe: c[k] = a[k] + b[k] for k < count (FP32, count a
 * multiple of 4, 16-byte aligned device buffers), streamed with 16-byte
 * non-temporal loads and stores by a grid-stride kernel: the bandwidth a
 * plain kernel with the elementwise body's mix (two reads, one write)
 * reaches on this GPU. */
tri_status tri_stream_add(float *c, const float *a, const float *b, int64_t count, void *stream);

/* Measurement probe sweep: one streaming kernel over count FP32 (a multiple
 * of 4, 16-byte aligned device buffers) with a chosen access mix, to find
 * the bandwidth a plain kernel of each mix reaches on this GPU:
 *   kind 0  read a (each workgroup's sum feeds a store to c that no run
 *           takes),
 *   kind 1  c = a + b (two reads, one write: the fp32 elementwise mix),
 *   kind 2  fill c (write only; a and b unused),
 *   kind 3  c = a (one read, one write).
 * c holds count floats for every kind.  Each thread keeps `unroll` (1, 2, 4 or 8) 16-byte vectors per read stream
 * in flight; workgroups of `threads` (64 .. 1024, a power of two) walk the
 * buffers in chunks of threads * unroll vectors, grid-stride; `workgroups`
 * caps the grid (0: one chunk per workgroup, no loop); `nontemporal`
 * selects non-temporal loads and stores. */
tri_status tri_stream_probe(int kind, int unroll, int threads, int nontemporal,
                            int64_t workgroups, float *c, const float *a, const float *b,
                            int64_t count, void *stream);

/* Human-readable name of a status, and the last error message of the
 * calling thread ("" if none). */
const char *tri_status_str(tri_status st);
const char *tri_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TRIMAP_H */
