/*
 * trimap oracle: a plain, slow, obviously correct CPU implementation of what
 * the triangular-domain hot path computes.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file.  It is used by tests/, by the smoke check of the
 * package entry module, and by the CPU-baseline leg of bench.py.  It shares
 * no code, header, table or constant generator with the HIP library.
 *
 * Source: C. A. Navarro, B. Bustos, N. Hitschfeld, "A Non-linear GPU Thread
 * Map for Triangular Domains" (arXiv 1609.01490).  Each function cites the
 * section / equation it follows.  Readings of passages the paper leaves
 * silent, garbled or inconsistent are marked READING and are listed in the
 * design notes of the repository.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared -o liboracle.so
 *        trimap_oracle.c -lm
 * (-ffp-contract=off: single-precision expressions below are evaluated as
 *  written, one IEEE-754 binary32 rounding per operation, no fused ops.)
 *
 * Parity status: every function here is pinned by a CPU test against values
 * fixed by the paper or by mathematics (worked example, closed forms,
 * bijectivity by brute force, textbook Life patterns, library routines).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Integer square root                                                       */
/* ------------------------------------------------------------------------ */

/* floor(sqrt(x)) by binary search on r with r*r <= x.  Written with a
 * division so that no intermediate overflows 64 bits. */
uint64_t orc_isqrt(uint64_t x)
{
    uint64_t lo = 0, hi = 0xFFFFFFFFull; /* sqrt(2^64-1) < 2^32 */
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo + 1) / 2; /* mid >= 1 */
        if (mid <= x / mid)
            lo = mid; /* mid*mid <= x */
        else
            hi = mid - 1;
    }
    return lo;
}

/* ------------------------------------------------------------------------ */
/* The block-space map lambda(omega)  (Section 3.1)                           */
/* ------------------------------------------------------------------------ */

/* Theorem / Eq. eq_gmap: block omega of the row-major numbering of the lower
 * triangle including the diagonal (Eq. eq_matrix_indexing) lies in row
 *   i = floor( sqrt(1/4 + 2 omega) - 1/2 ),   column j = omega - i(i+1)/2.
 * sqrt(1/4 + 2w) - 1/2 = (sqrt(8w+1) - 1)/2, and floor((s-1)/2) equals
 * floor((floor(s)-1)/2), so i is obtained exactly from the integer square
 * root of 8w+1.  Valid for omega < 2^60. */
void orc_lambda(uint64_t omega, int64_t *i, int64_t *j)
{
    uint64_t s = orc_isqrt(8ull * omega + 1ull);
    uint64_t r = (s - 1ull) / 2ull;
    *i = (int64_t)r;
    *j = (int64_t)(omega - r * (r + 1ull) / 2ull);
}

/* Eq. eq_theorem_nodiag: the variant without the diagonal.  Row
 *   i = floor( sqrt(1/4 + 2 omega) + 1/2 ) = floor((sqrt(8w+1)+1)/2).
 * READING: the printed column omega - i(i+1)/2 is negative for omega = 0
 * (it would give (1,-1)); the numbering of the strict lower triangle starts
 * row i at i(i-1)/2, so the column is j = omega - i(i-1)/2. */
void orc_lambda_nodiag(uint64_t omega, int64_t *i, int64_t *j)
{
    uint64_t s = orc_isqrt(8ull * omega + 1ull);
    uint64_t r = (s + 1ull) / 2ull;
    *i = (int64_t)r;
    *j = (int64_t)(omega - r * (r - 1ull) / 2ull);
}

/* ------------------------------------------------------------------------ */
/* Parallel-space maps on a tile grid  (Sections 3.1 and 4.2)                 */
/* ------------------------------------------------------------------------ */
/* Tile space: m tiles per side, tiles (bi, bj) with 0 <= bj <= bi < m.
 * Each map is a grid (gw x gh blocks, block id b = by*gw + bx) and a function
 * from grid block to tile, or "no tile" (-1, -1) for a discarded block.     */

enum { ORC_BB = 0, ORC_RB = 1, ORC_REC = 2, ORC_UTM = 3, ORC_LAMBDA = 4 };

static int is_pow2(int64_t m) { return m > 0 && (m & (m - 1)) == 0; }

/* Grid shape of a tile-space map.  Returns 0, or -1 when the map does not
 * apply (REC needs m a power of two; UTM is a thread-space map). */
int orc_map_grid(int map, int64_t m, int64_t *gw, int64_t *gh)
{
    if (m < 1)
        return -1;
    switch (map) {
    case ORC_BB: /* Section 4.2: an m x m box of blocks */
        *gw = m;
        *gh = m;
        return 0;
    case ORC_LAMBDA: /* Section 3.1: exactly m(m+1)/2 blocks, one dimension */
        *gw = m * (m + 1) / 2;
        *gh = 1;
        return 0;
    case ORC_RB: /* Section 4.2, rectangular box */
        if (m % 2) {
            *gw = m;
            *gh = (m + 1) / 2;
        } else {
            *gw = m + 1;
            *gh = m / 2;
        }
        return 0;
    case ORC_REC: /* Section 4.2, recursive partition; m = 2^k */
        if (!is_pow2(m))
            return -1;
        if (m == 1) {
            *gw = 1;
            *gh = 1;
        } else {
            *gw = m / 2;
            *gh = m + 1;
        }
        return 0;
    default:
        return -1;
    }
}

/* Tile of grid block (bx, by) under a tile-space map; (-1,-1) if the block
 * is discarded.
 *
 * BB (Section 4.2): identity, kept iff the block lies on or below the
 *   diagonal.  READING: the printed block test "B_i > B_j" would discard the
 *   diagonal blocks that the following sentence then filters per thread, so
 *   the block test is B_i >= B_j.
 *
 * RB (Section 4.2): the triangle is folded into a rectangle: the part of the
 *   grid on/above the diagonal is the rotated far end of the triangle.
 *   READING: the printed "j = n - i - 1" is constant along a row; the
 *   rotation it describes is j = n - t_x - 1.  For odd m the grid is
 *   m x (m+1)/2: below the diagonal (bx < by) a block maps to row by-1, on
 *   or above it to (m-1-by, m-1-bx).  For even m the rectangle is
 *   (m+1) x m/2: bx <= by maps to (by, bx), otherwise to (m-1-by, bx-by-1).
 *
 * REC (Section 4.2, after Ries et al.): READING (the paper defers the layout
 *   to Ries et al.): for m = 2^k the strictly-lower part is a set of squares,
 *   level l holding m/(2s) squares of side s = 2^(l-1); square q of that
 *   level covers rows q*2s+s .. q*2s+2s-1 and columns q*2s .. q*2s+s-1.
 *   Level l occupies s consecutive grid rows of width m/2 (grid row
 *   by = s-1+r holds row r of every square of the level), so the k levels
 *   fill m-1 rows; the m diagonal tiles, the extra pass of the paper, are two
 *   more rows of the same grid.
 *
 * LAMBDA (Eq. eq_gmap): block omega = bx maps to lambda(omega).            */
void orc_map_tile(int map, int64_t m, int64_t bx, int64_t by, int64_t *ti, int64_t *tj)
{
    *ti = -1;
    *tj = -1;
    switch (map) {
    case ORC_BB:
        if (bx <= by) {
            *ti = by;
            *tj = bx;
        }
        return;
    case ORC_LAMBDA:
        orc_lambda((uint64_t)bx, ti, tj);
        return;
    case ORC_RB:
        if (m % 2) {
            if (bx < by) {
                *ti = by - 1;
                *tj = bx;
            } else {
                *ti = m - 1 - by;
                *tj = m - 1 - bx;
            }
        } else {
            if (bx <= by) {
                *ti = by;
                *tj = bx;
            } else {
                *ti = m - 1 - by;
                *tj = bx - by - 1;
            }
        }
        return;
    case ORC_REC: {
        if (m == 1) {
            *ti = 0;
            *tj = 0;
            return;
        }
        if (by >= m - 1) { /* the diagonal pass */
            int64_t t = (by - (m - 1)) * (m / 2) + bx;
            *ti = t;
            *tj = t;
            return;
        }
        /* level: s = largest power of two with s - 1 <= by, i.e. s <= by+1 */
        int64_t s = 1;
        while (2 * s <= by + 1)
            s *= 2;
        int64_t r = by - (s - 1);
        int64_t q = bx / s, c = bx % s;
        *ti = q * 2 * s + s + r;
        *tj = q * 2 * s + c;
        return;
    }
    default:
        return;
    }
}

/* Dump the whole grid of a tile-space map: out[2*b], out[2*b+1] = tile of
 * block b = by*gw + bx, or -1,-1.  Returns the number of blocks, or -1. */
int64_t orc_map_dump(int map, int64_t m, int64_t *out)
{
    int64_t gw, gh;
    if (orc_map_grid(map, m, &gw, &gh))
        return -1;
    for (int64_t by = 0; by < gh; ++by)
        for (int64_t bx = 0; bx < gw; ++bx) {
            int64_t b = by * gw + bx;
            orc_map_tile(map, m, bx, by, &out[2 * b], &out[2 * b + 1]);
        }
    return gw * gh;
}

/* UTM, the thread-space map of Avril et al. (Section 4.2): thread k of a
 * problem of size N owns the k-th pair (a, b), 1 <= a < b <= N, in
 * lexicographic order (the formula printed in the paper enumerates exactly
 * this order).  Row a starts at the count of pairs in rows 1..a-1, which is
 * (a-1)(2N-a)/2; a is found by a plain linear scan over rows. */
int orc_utm_pair(int64_t N, int64_t k, int64_t *a, int64_t *b)
{
    int64_t start = 0;
    for (int64_t r = 1; r < N; ++r) {
        int64_t len = N - r; /* pairs (r, r+1..N) */
        if (k < start + len) {
            *a = r;
            *b = r + 1 + (k - start);
            return 0;
        }
        start += len;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Triangular elementwise bodies                                             */
/* ------------------------------------------------------------------------ */

/* Integer body: for every cell (i, j) with 0 <= j <= i < n,
 *   C[i][j] = (A[i] XOR B[j]) + i*j   in uint32 arithmetic (mod 2^32).
 * Rows r0..r1-1 are computed into out (row r at out + (r-r0)*ldo); cells
 * j > i of out are not written.  The dummy-kernel role of Sections 4.1 and 5, with
 * a real per-cell write. */
void orc_c0(int64_t n, const uint32_t *A, const uint32_t *B, int64_t r0, int64_t r1,
            int32_t *out, int64_t ldo)
{
    for (int64_t i = r0; i < r1 && i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            uint32_t v = (A[i] ^ B[j]) + (uint32_t)((uint64_t)i * (uint64_t)j);
            out[(i - r0) * ldo + j] = (int32_t)v;
        }
}

/* Single-precision body: for every cell with 0 <= j <= i < n,
 *   C[i][j] = fl( fl(a * X[i][j]) + Y[j][i] )
 * two binary32 round-to-nearest-even operations, multiply then add, no
 * fusion.  X and Y are n x n row-major with leading dimension ld.  Rows
 * r0..r1-1 are written to out (leading dimension ldo). */
void orc_c1(int64_t n, float a, const float *X, const float *Y, int64_t ld, int64_t r0,
            int64_t r1, float *out, int64_t ldo)
{
    for (int64_t i = r0; i < r1 && i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            float t = a * X[i * ld + j];
            float c = t + Y[j * ld + i];
            out[(i - r0) * ldo + j] = c;
        }
}

/* ------------------------------------------------------------------------ */
/* Game of Life on a lower-triangular domain                                 */
/* ------------------------------------------------------------------------ */

/* Conway's rule B3/S23 (Gardner's column, cited in Section 1 as cellular
 * automata on triangular domains).  Domain: cells (i, j), 0 <= j <= i < n.
 * All cells outside the domain (j > i, or outside the n x n square) are dead
 * at every step.  Update is synchronous.
 *
 * The simulation runs on the window rows r0..r0+h-1, columns c0..c0+w-1 of
 * the grid `in` (n rows, leading dimension ld; only domain cells are read,
 * they hold 0 or 1).  Cells outside the window are also treated as dead, so
 * the result is exact for the whole domain when the window covers it, and
 * exact at least `steps` cells inside the window's border otherwise (the
 * light cone of a cell after s steps has radius s).  out is h x w (leading
 * dimension ldo); its cells outside the domain are set to 0. */
int orc_gol(int64_t n, const uint8_t *in, int64_t ld, int64_t r0, int64_t c0, int64_t h,
            int64_t w, int steps, uint8_t *out, int64_t ldo)
{
    int64_t H = h + 2, W = w + 2; /* one dead frame around the window */
    uint8_t *cur = (uint8_t *)calloc((size_t)(H * W), 1);
    uint8_t *nxt = (uint8_t *)calloc((size_t)(H * W), 1);
    uint8_t *dom = (uint8_t *)calloc((size_t)(H * W), 1);
    if (!cur || !nxt || !dom) {
        free(cur);
        free(nxt);
        free(dom);
        return -1;
    }
    for (int64_t r = 0; r < h; ++r)
        for (int64_t c = 0; c < w; ++c) {
            int64_t i = r0 + r, j = c0 + c;
            int inside = (i >= 0 && i < n && j >= 0 && j <= i);
            dom[(r + 1) * W + (c + 1)] = (uint8_t)inside;
            if (inside)
                cur[(r + 1) * W + (c + 1)] = in[i * ld + j] ? 1 : 0;
        }
    for (int s = 0; s < steps; ++s) {
        for (int64_t r = 1; r <= h; ++r)
            for (int64_t c = 1; c <= w; ++c) {
                int64_t p = r * W + c;
                if (!dom[p]) {
                    nxt[p] = 0;
                    continue;
                }
                int cnt = 0;
                for (int dr = -1; dr <= 1; ++dr)
                    for (int dc = -1; dc <= 1; ++dc)
                        if (dr || dc)
                            cnt += cur[p + dr * W + dc];
                int alive = cur[p];
                nxt[p] = (uint8_t)((cnt == 3) || (alive && cnt == 2));
            }
        uint8_t *t = cur;
        cur = nxt;
        nxt = t;
    }
    for (int64_t r = 0; r < h; ++r)
        for (int64_t c = 0; c < w; ++c)
            out[r * ldo + c] = cur[(r + 1) * W + (c + 1)];
    free(cur);
    free(nxt);
    free(dom);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Euclidean distance map  (Section 5, the EDM test)                         */
/* ------------------------------------------------------------------------ */

/* d(i, j) = sqrt( sum_k (x_ik - x_jk)^2 ) for the strict lower triangle
 * j < i (the map without diagonal, Eq. eq_theorem_nodiag), evaluated in
 * binary64 from binary32 coordinates.  For each requested row r = rows[t],
 * the r distances d(r, 0..r-1) are appended to out; with rows = 0..n-1 the
 * output is the condensed strict lower triangle, entry (i, j) at
 * i(i-1)/2 + j.  X is n x d, leading dimension ldx. */
void orc_edm_rows(int64_t n, int64_t d, const float *X, int64_t ldx, const int64_t *rows,
                  int64_t nrows, double *out)
{
    int64_t o = 0;
    for (int64_t t = 0; t < nrows; ++t) {
        int64_t i = rows[t];
        if (i < 0 || i >= n)
            continue;
        for (int64_t j = 0; j < i; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < d; ++k) {
                double diff = (double)X[i * ldx + k] - (double)X[j * ldx + k];
                acc += diff * diff;
            }
            out[o++] = sqrt(acc);
        }
    }
}

/* Four-feature distance map, the global-memory test of Section 5: every
 * point carries (x, y, z, w).  The paper gives the formula (Section 5, the
 * EDM paragraph) without fixing a precision; here it is one binary32
 * expression with a fixed order, so that any conforming evaluation is
 * bit-identical: d. = p. - q. rounded, squares rounded, the sum
 * ((dx^2 + dy^2) + dz^2) + dw^2 rounded left to right, then the correctly
 * rounded sqrtf.  P is n x 4 (row-major, no padding).  Rows r0..r1-1 of the
 * lower triangle with diagonal (j <= i) are written to out, leading
 * dimension ldo; cells j > i of out are left as they are. */
void orc_edm4(int64_t n, const float *P, int64_t r0, int64_t r1, float *out, int64_t ldo)
{
    for (int64_t i = r0; i < r1 && i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            float dx = P[4 * i + 0] - P[4 * j + 0];
            float dy = P[4 * i + 1] - P[4 * j + 1];
            float dz = P[4 * i + 2] - P[4 * j + 2];
            float dw = P[4 * i + 3] - P[4 * j + 3];
            float sx = dx * dx, sy = dy * dy, sz = dz * dz, sw = dw * dw;
            float s = sx + sy;
            s = s + sz;
            s = s + sw;
            out[(i - r0) * ldo + j] = sqrtf(s);
        }
}

/* ------------------------------------------------------------------------ */
/* Collision detection of spheres (Section 5, the shared-memory test)       */
/* ------------------------------------------------------------------------ */

/* Spheres k = 0..n-1 are rows (x, y, z, r) of S (n x 4).  In dim = 3 two
 * spheres overlap when the squared distance of their centres is below the
 * square of the sum of their radii; in dim = 1 only x is a coordinate.  The
 * paper does not fix the arithmetic; here it is binary32 with a fixed order
 * (differences, squares, sum left to right, r_a + r_b, its square) and a
 * strict comparison, so that touching spheres do not count.  The test is
 * symmetric in (a, b): a - b is exactly -(b - a). */
static int orc_overlap(int dim, const float *a, const float *b)
{
    float dx = a[0] - b[0];
    float s = dx * dx;
    if (dim == 3) {
        float dy = a[1] - b[1];
        float dz = a[2] - b[2];
        float sy = dy * dy, sz = dz * dz;
        s = s + sy;
        s = s + sz;
    }
    float rr = a[3] + b[3];
    float t = rr * rr;
    return s < t;
}

/* counts[k] = number of spheres other than k that overlap sphere k: every
 * pair j < i of the strict lower triangle is tested once and counted for
 * both spheres. */
void orc_collide(int64_t n, int dim, const float *S, int32_t *counts)
{
    for (int64_t k = 0; k < n; ++k)
        counts[k] = 0;
    for (int64_t i = 1; i < n; ++i)
        for (int64_t j = 0; j < i; ++j)
            if (orc_overlap(dim, S + 4 * i, S + 4 * j)) {
                counts[i]++;
                counts[j]++;
            }
}

/* The count of one sphere k alone (same pairs, same test). */
int32_t orc_collide_one(int64_t n, int dim, const float *S, int64_t k)
{
    int32_t c = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == k)
            continue;
        const int64_t hi = j > k ? j : k, lo = j > k ? k : j;
        c += orc_overlap(dim, S + 4 * hi, S + 4 * lo);
    }
    return c;
}

/* ------------------------------------------------------------------------ */
/* Tetrahedral block map (Section 6, the extension to 3-D)                    */
/* ------------------------------------------------------------------------ */

/* Tetrahedral number Tet(k) = k(k+1)(k+2)/6: the number of blocks in layers
 * 0..k-1, layer k being a triangle of (k+1)(k+2)/2 blocks (Section 6). */
uint64_t orc_tet(uint64_t k)
{
    return k * (k + 1ull) / 2ull * (k + 2ull) / 3ull;
}

/* The 3-D lambda: block omega lies in layer k, the largest k with
 * Tet(k) <= omega (the integer part of the real root of the cubic of
 * Section 6, found here by an integer binary search, which is exact); within
 * the layer omega_2D = omega - Tet(k) is mapped by the 2-D lambda to row j
 * and column i.  Result (i, j, k) with 0 <= i <= j <= k. */
void orc_lambda3(uint64_t omega, int64_t *i, int64_t *j, int64_t *k)
{
    uint64_t lo = 0, hi = 3100000ull; /* Tet(3.1e6) > 2^62; k(k+1)/2 (k+2) < 2^64 */
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo + 1) / 2;
        if (orc_tet(mid) <= omega)
            lo = mid;
        else
            hi = mid - 1;
    }
    *k = (int64_t)lo;
    orc_lambda(omega - orc_tet(lo), j, i);
}

/* Bounding box of the tetrahedron: an m x m x m grid, block (bx, by, bz)
 * (id = (bz m + by) m + bx) kept iff bx <= by <= bz, as tile (i, j, k) =
 * (bx, by, bz).  Writes 3 entries per grid block, -1 for discarded ones;
 * returns the number of blocks. */
int64_t orc_bb3_dump(int64_t m, int64_t *out)
{
    int64_t b = 0;
    for (int64_t bz = 0; bz < m; ++bz)
        for (int64_t by = 0; by < m; ++by)
            for (int64_t bx = 0; bx < m; ++bx, ++b) {
                int keep = bx <= by && by <= bz;
                out[3 * b + 0] = keep ? bx : -1;
                out[3 * b + 1] = keep ? by : -1;
                out[3 * b + 2] = keep ? bz : -1;
            }
    return b;
}

/* ------------------------------------------------------------------------ */
/* Triangles of the neighbour graph (a triplet kernel on the tetrahedron)    */
/* ------------------------------------------------------------------------ */

/* Points are rows (x, y, z, w) of P (n x 4; w unused).  Points a and b are
 * neighbours when their squared distance, in binary32 without fused
 * multiply-add, ((dx^2 + dy^2) + dz^2) with d. = a. - b., is below r2
 * (strict).  The test is symmetric: a - b is exactly -(b - a). */
static int orc_near(const float *a, const float *b, float r2)
{
    float dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    float sx = dx * dx, sy = dy * dy, sz = dz * dz;
    float s = sx + sy;
    s = s + sz;
    return s < r2;
}

/* Every triple a > b > c of mutual neighbours is one triangle: counts[v]
 * receives the number of triangles with vertex v, *total their number. */
void orc_triangles(int64_t n, const float *P, float r2, int32_t *counts, uint64_t *total)
{
    uint64_t t = 0;
    for (int64_t v = 0; v < n; ++v)
        counts[v] = 0;
    for (int64_t a = 2; a < n; ++a)
        for (int64_t b = 1; b < a; ++b) {
            if (!orc_near(P + 4 * a, P + 4 * b, r2))
                continue;
            for (int64_t c = 0; c < b; ++c)
                if (orc_near(P + 4 * a, P + 4 * c, r2) && orc_near(P + 4 * b, P + 4 * c, r2)) {
                    counts[a]++;
                    counts[b]++;
                    counts[c]++;
                    t++;
                }
        }
    *total = t;
}

/* The triangle count of one vertex v alone: pairs u > w of neighbours of v
 * that are neighbours of each other.  nb is scratch for n indices. */
int32_t orc_triangles_one(int64_t n, const float *P, float r2, int64_t v, int64_t *nb)
{
    int64_t d = 0;
    for (int64_t u = 0; u < n; ++u)
        if (u != v && orc_near(P + 4 * (u > v ? u : v), P + 4 * (u > v ? v : u), r2))
            nb[d++] = u;
    int32_t c = 0;
    for (int64_t x = 1; x < d; ++x)
        for (int64_t y = 0; y < x; ++y)
            c += orc_near(P + 4 * nb[x], P + 4 * nb[y], r2);
    return c;
}

/* ------------------------------------------------------------------------ */
/* Batched work queue over per-instance lambda numberings                    */
/* ------------------------------------------------------------------------ */

/* Instances k = 0..count-1 own blocks[k] consecutive global work items,
 * numbered in instance order.  Item g belongs to the unique instance k with
 * start_k <= g < start_k + blocks[k], and is that instance's block
 * omega = g - start_k, whose tile is lambda(omega) (Eq. eq_gmap).  Plain
 * linear scan.  Returns 0, or -1 if g is past the last item. */
int orc_queue_locate(int64_t count, const int64_t *blocks, int64_t g, int64_t *k,
                     int64_t *omega)
{
    int64_t start = 0;
    for (int64_t t = 0; t < count; ++t) {
        if (g < start + blocks[t]) {
            *k = t;
            *omega = g - start;
            return 0;
        }
        start += blocks[t];
    }
    return -1;
}
