// Device side of the parallel-space maps: grid block -> tile (bi, bj) of the
// lower triangle of an m x m tile grid (0 <= bj <= bi < m), and the
// thread-space UTM map.  Each map is a self-contained function with no side
// effects (the Conclusions, Section 7, make this point for lambda).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "trimap.h"

namespace trimap {

// Uniform description of the tile grid handed to every tile kernel.
struct TileGrid {
    int32_t m;       // tiles per side
    uint32_t flags;  // TRI_FLAG_*, plus kLambda24
    uint64_t T;      // tiles, m (m + 1) / 2
};

// Internal TileGrid flags: lambda launched as a 1-D grid of exactly T < 2^24
// blocks with the default root and order (the swizzle allowed), or as a
// 2-D grid of 2^16-block rows over T < 2^32 blocks with no flags, so the map
// can take a 32-bit path.
constexpr uint32_t kLambda24 = 1u << 31;
constexpr uint32_t kLambda32 = 1u << 30;

// ---------------------------------------------------------------------------
// lambda(omega), Eq. eq_gmap: row i = floor((sqrt(8 omega + 1) - 1) / 2),
// column j = omega - i (i + 1) / 2.
//
// The square root is taken in floating point and the row is then corrected
// by one integer step so that T_i <= omega < T_{i+1} (T_i = i (i + 1) / 2).
// For omega < 2^32 the FP32 estimate is within 0.05 of the true row (8w+1 is
// rounded twice to 24 bits, the hardware square root adds at most a few
// units in the last place, and the row is below 2^16.5), so one step makes
// it exact; that is why no epsilon is added as in the paper's lambda_N and
// lambda_R.  omega >= 2^32 always takes the FP64 root.
// ---------------------------------------------------------------------------
// Square root of the lambda_N variant (Section 4.1): reciprocal square root
// from the integer bit trick of the fast inverse square root (initial
// constant 0x5f3759df, Lomont's analysis), three Newton-Raphson steps
// y <- y (3/2 - (x/2) y^2), then sqrt(x) = x y.
__device__ __forceinline__ float sqrt_newton3(float x)
{
    float y = __uint_as_float(0x5f3759dfu - (__float_as_uint(x) >> 1));
    const float h = 0.5f * x;
#pragma unroll
    for (int k = 0; k < 3; ++k) y = y * (1.5f - h * y * y);
    return x * y;
}

__device__ __forceinline__ float sqrt_variant(float x, uint32_t flags)
{
    if (flags & TRI_FLAG_SQRT_RSQ) return x * __builtin_amdgcn_rsqf(x);
    if (flags & TRI_FLAG_SQRT_NEWTON) return sqrt_newton3(x);
    return __builtin_amdgcn_sqrtf(x);
}

// The paper's inexact form (Section 4.1): i = floor(sqrt(1/4 + 2 omega) + eps
// - 1/2) with eps = 1e-4 and no integer correction.  Kept for the square-root
// study only: it is wrong for some omega, so kernels may miss or repeat tiles.
__device__ __forceinline__ uint32_t lambda_row_eps(uint64_t w, uint32_t flags)
{
    const float s = sqrt_variant(0.25f + 2.0f * (float)(uint32_t)w, flags) + 1e-4f;
    const float r = s - 0.5f;
    return r < 0.f ? 0u : (uint32_t)r;
}

__device__ __forceinline__ uint32_t lambda_row(uint64_t w, uint32_t flags)
{
    int32_t r;
    if ((flags & TRI_FLAG_SQRT_F64) || (w >> 32)) {
        double s = __builtin_sqrt(8.0 * (double)w + 1.0);
        r = (int32_t)((s - 1.0) * 0.5);
    } else {
        if (flags & TRI_FLAG_SQRT_EPS) return lambda_row_eps(w, flags);
        float x = __builtin_fmaf(8.0f, (float)(uint32_t)w, 1.0f);
        float s = sqrt_variant(x, flags);
        r = (int32_t)((s - 1.0f) * 0.5f);
    }
    uint32_t i = r < 0 ? 0u : (uint32_t)r;
    uint64_t t = (uint64_t)i * (i + 1) / 2;  // first block of row i
    if (t > w)
        --i;
    else if (t + i + 1 <= w)
        ++i;
    return i;
}

__device__ __forceinline__ void lambda_tile(uint64_t w, uint32_t flags, int32_t &bi, int32_t &bj)
{
    uint32_t i = lambda_row(w, flags);
    bi = (int32_t)i;
    bj = (int32_t)(w - (uint64_t)i * (i + 1) / 2);
}

// The same map for w < 2^24 (a 1-D grid) in 32-bit arithmetic: 8w + 1 is
// rounded once to 24 bits, the root is off by far less than one row, and
// rows stay below 2^12.5, so T_i and the one-step correction fit in 32 bits.
// The map is wave-uniform: a handful of scalar instructions per wave after
// the square root (the scalar unit is shared by the CU's waves, so its
// instruction count, not the root, is what the map costs).
__device__ __forceinline__ void lambda_tile_24(uint32_t w, int32_t &bi, int32_t &bj)
{
    const float x = __builtin_fmaf(8.0f, (float)w, 1.0f);
    uint32_t i = (uint32_t)((__builtin_amdgcn_sqrtf(x) - 1.0f) * 0.5f);
    uint32_t t = i * (i + 1) / 2;
    if (t > w) {
        --i;
        t -= i + 1;
    } else if (t + i + 1 <= w) {
        t += i + 1;
        ++i;
    }
    bi = (int32_t)i;
    bj = (int32_t)(w - t);
}

// The same for w < 2^32: 8w + 1 is rounded twice to 24 bits and the root is
// still within one row (rows stay below 2^16.5).  T_i < 2^32 is formed
// from the even factor of i (i + 1) so that no product overflows, and the
// upward step compares w - T_i with the row length.
__device__ __forceinline__ void lambda_tile_32(uint32_t w, int32_t &bi, int32_t &bj)
{
    const float x = __builtin_fmaf(8.0f, (float)w, 1.0f);
    uint32_t i = (uint32_t)((__builtin_amdgcn_sqrtf(x) - 1.0f) * 0.5f);
    uint32_t t = (i & 1u) ? i * ((i + 1) >> 1) : (i >> 1) * (i + 1);
    if (t > w) {
        --i;
        t -= i + 1;
    } else if (w - t >= i + 1) {
        t += i + 1;
        ++i;
    }
    bi = (int32_t)i;
    bj = (int32_t)(w - t);
}

// Give each of the 8 XCDs a contiguous range of omega.  Workgroups are
// dispatched to XCDs round-robin by linear id; block L runs on XCD L mod 8.
// With G = 8q + r blocks, XCD x holds q + (x < r) blocks, so its range starts
// at x q + min(x, r).  A bijection of [0, G).
__device__ __forceinline__ uint64_t xcd_swizzle(uint64_t L, uint64_t G)
{
    uint64_t x = L & 7, l = L >> 3, q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + l;
}

// Order in which the workgroups of a lambda grid visit omega: a bijection
// of [0, T) applied to the (possibly swizzled) block number L < T.  Reverse
// starts with the longest tile rows; pairs alternates a block from the front
// with one from the back, so short and long tile rows run together.
__device__ __forceinline__ uint64_t dispatch_order(uint64_t L, uint64_t T, uint32_t flags)
{
    if (flags & TRI_FLAG_ORDER_REVERSE) return T - 1 - L;
    if (flags & TRI_FLAG_ORDER_PAIRS) return (L & 1) ? T - 1 - (L >> 1) : (L >> 1);
    return L;
}

enum { MAP_BB = TRI_MAP_BB, MAP_RB = TRI_MAP_RB, MAP_REC = TRI_MAP_REC,
       MAP_UTM = TRI_MAP_UTM, MAP_LAMBDA = TRI_MAP_LAMBDA };

// Tile of this workgroup under a tile-space map, or false when the block is
// discarded.  BB, RB and REC use a 2-D grid (blockIdx.x = column); lambda a
// 1-D grid (2-D only when the tile count exceeds one grid dimension).
// The 2-D tile maps at an explicit grid position (bx, by): BB, RB and REC.
template <int MAP>
__device__ __forceinline__ bool tile_at_xy(const TileGrid &g, int32_t bx, int32_t by, int32_t &bi,
                                           int32_t &bj)
{
    if constexpr (MAP == MAP_BB) {
        // Section 4.2: the block test (on or below the diagonal) comes before
        // any thread coordinate is formed.
        if (bx > by) return false;
        bi = by;
        bj = bx;
        return true;
    } else if constexpr (MAP == MAP_RB) {
        const int32_t m = g.m;
        if (m & 1) {
            if (bx < by) { bi = by - 1; bj = bx; }
            else { bi = m - 1 - by; bj = m - 1 - bx; }
        } else {
            if (bx <= by) { bi = by; bj = bx; }
            else { bi = m - 1 - by; bj = bx - by - 1; }
        }
        return true;
    } else if constexpr (MAP == MAP_REC) {
        const int32_t m = g.m;
        if (m == 1) { bi = bj = 0; return true; }
        if (by >= m - 1) {  // the diagonal pass: two grid rows of m/2 tiles
            bi = bj = (by - (m - 1)) * (m >> 1) + bx;
            return true;
        }
        const int32_t lg = 31 - __builtin_clz((uint32_t)(by + 1));  // level: side s = 2^lg
        const int32_t s = 1 << lg;
        const int32_t r = by - (s - 1);
        const int32_t q = bx >> lg, c = bx & (s - 1);
        bi = q * 2 * s + s + r;
        bj = q * 2 * s + c;
        return true;
    }
    return false;
}

template <int MAP>
__device__ __forceinline__ bool tile_of_block_raw(const TileGrid &g, int32_t &bi, int32_t &bj)
{
    if constexpr (MAP != MAP_LAMBDA) {
        return tile_at_xy<MAP>(g, (int32_t)blockIdx.x, (int32_t)blockIdx.y, bi, bj);
    } else {
        if (g.flags & kLambda24) {
            // 1-D grid of exactly T < 2^24 blocks, default root and order
            uint32_t L = blockIdx.x;
            if (g.flags & TRI_FLAG_XCD_SWIZZLE) {
                const uint32_t x = L & 7, l = L >> 3, G = (uint32_t)g.T, q = G >> 3, r = G & 7;
                L = x * q + (x < r ? x : r) + l;
            }
            lambda_tile_24(L, bi, bj);
            return true;
        }
        if (g.flags & kLambda32) {
            // 2-D grid of 2^16-block rows, T < 2^32, default root and order
            const uint32_t L = (blockIdx.y << 16) + blockIdx.x;
            if (L >= (uint32_t)g.T) return false;
            lambda_tile_32(L, bi, bj);
            return true;
        }
        uint64_t L = (uint64_t)blockIdx.y * gridDim.x + blockIdx.x;
        if (g.flags & TRI_FLAG_XCD_SWIZZLE)
            L = xcd_swizzle(L, (uint64_t)gridDim.x * gridDim.y);
        if (L >= g.T) return false;
        lambda_tile(dispatch_order(L, g.T, g.flags), g.flags, bi, bj);
        return true;
    }
}

// Same, plus a range check (0 <= bj <= bi < m) so that no kernel can address
// memory outside the domain's rows whatever a map returns.
template <int MAP>
__device__ __forceinline__ bool tile_of_block(const TileGrid &g, int32_t &bi, int32_t &bj)
{
    if (!tile_of_block_raw<MAP>(g, bi, bj)) return false;
    return (uint32_t)bi < (uint32_t)g.m && (uint32_t)bj <= (uint32_t)bi;
}

// ---------------------------------------------------------------------------
// Strips: a workgroup walks G tiles of the map, so that one dispatch serves
// several tiles and the tiles of a strip, which mostly share their tile row,
// reuse what the workgroup has staged.  The tiles are taken in groups of
// K G consecutive tile numbers (omega under lambda; grid columns of one
// grid row, blockIdx.y, under BB, RB and REC) shared by K consecutive
// workgroups: workgroup k of a group takes numbers k, k + K, k + 2K, ...,
// so at each step the group's K workgroups work on K adjacent tiles (with
// the XCD swizzle, on one XCD and one L2).  The dispatch order and swizzle
// of lambda act on workgroups.  Every tile is still mapped on its own.
// ---------------------------------------------------------------------------
//
// Column-major strips (TRI_FLAG_STRIP_COLS, lambda, K = 1): the strips are
// aligned to tile rows (strip c of row i holds omega T_i + c G .. up to the
// row's end) and workgroup s takes them column by column: strip column c
// (rows c G .. m - 1, m - c G strips) before c + 1.  With the XCD swizzle
// the workgroups resident on one XCD then walk the same columns of many
// rows, so a kernel that stages column operands per tile finds them in L2.
// Strip s lies in column c with P(c) <= s < P(c + 1), P(c) = c m - G c (c -
// 1) / 2 (the strips of the columns before c): the root of the quadratic,
// corrected by integer steps, as lambda finds its row.
//
// Row-major aligned strips (TRI_FLAG_STRIP_ALIGN, lambda, K = 1): the same
// row-aligned strips taken row by row (every strip of row i before row
// i + 1), so that each strip starts at a multiple of G tiles in its row.
// Row i has ceil((i + 1) / G) strips, so the rows a G .. a G + G - 1 have
// a + 1 each and G a (a + 1) / 2 strips lie before row a G: strip s is in
// row group a = floor((sqrt(8 s / G + 1) - 1) / 2) (lambda on s / G, with
// the integer correction), row a G + o / (a + 1), strip o mod (a + 1), for
// o = s - G a (a + 1) / 2.
//
// Two-row bands (TRI_FLAG_STRIP_BAND, K = 1, G >= 4): a strip holds G / 2
// columns of two consecutive tile rows (lambda) or grid rows (BB, RB,
// REC), and its tile k lies in row 2 p + (k & 1), column c0 + (k >> 1), so
// that tiles 4 q .. 4 q + 3 form a 2 x 2 block.  Under lambda the bands
// are row pairs p (rows 2 p, 2 p + 1, columns 0 .. 2 p + 1), cut at
// multiples of H = G / 2 columns: pair p has ceil((p + 1) / Q) strips, Q =
// H / 2, which is the aligned order above with rows read as row pairs and
// G as Q; the two tiles of column c are omega T_2p + c and T_2p+1 + c,
// each mapped by lambda on its own.
// ---------------------------------------------------------------------------
struct StripGrid {
    uint32_t strips;  // lambda: workgroups in the launch (gridDim.x)
    int32_t G;        // tiles per workgroup
    int32_t K;        // workgroups per group
    int32_t gx;       // BB / RB / REC: columns of the map's grid
    int32_t gy;       // BB / RB / REC: rows of the map's grid
};

__host__ __device__ __forceinline__ uint64_t strip_cols_prefix(uint32_t c, uint32_t m, uint32_t G)
{
    return c ? (uint64_t)c * m - (uint64_t)G * c * (c - 1) / 2 : 0;
}

// First omega of column-major strip s (s below the strip count).
__device__ __forceinline__ uint32_t strip_cols_first(uint32_t s, uint32_t m, uint32_t G)
{
    const double a = (double)m + 0.5 * (double)G;
    const double disc = a * a - 2.0 * (double)G * (double)s;
    const double c0 = (a - __builtin_sqrt(disc > 0.0 ? disc : 0.0)) / (double)G;
    uint32_t c = c0 > 0.0 ? (uint32_t)c0 : 0u;
    while (c > 0 && strip_cols_prefix(c, m, G) > s) --c;
    while (strip_cols_prefix(c + 1, m, G) <= s) ++c;
    const uint32_t i = c * G + (uint32_t)(s - strip_cols_prefix(c, m, G));
    return (uint32_t)((uint64_t)i * (i + 1) / 2) + c * G;
}

// Strips of the row-major aligned order before row i.
__host__ __device__ __forceinline__ uint64_t strip_align_prefix(uint32_t i, uint32_t G)
{
    const uint64_t a = i / G, b = i % G;
    return (uint64_t)G * a * (a + 1) / 2 + b * (a + 1);
}

// First omega of row-major aligned strip s (s below the strip count).
__device__ __forceinline__ uint32_t strip_align_first(uint32_t s, uint32_t G)
{
    const double x = 8.0 * (double)s / (double)G + 1.0;
    uint64_t a = (uint64_t)((__builtin_sqrt(x) - 1.0) * 0.5);
    while (a > 0 && (uint64_t)G * a * (a + 1) / 2 > s) --a;
    while ((uint64_t)G * (a + 1) * (a + 2) / 2 <= s) ++a;
    const uint64_t o = s - (uint64_t)G * a * (a + 1) / 2;
    const uint64_t i = a * G + o / (a + 1), c = o % (a + 1);
    return (uint32_t)(i * (i + 1) / 2 + c * G);
}

// First omega of two-row band strip s under lambda (s below the strip
// count, G >= 4): the omega of the band's top-left tile, row 2 p, column
// c H.
__device__ __forceinline__ uint32_t strip_band_first(uint32_t s, uint32_t G)
{
    const uint32_t H = G / 2, Q = G / 4;
    const double x = 8.0 * (double)s / (double)Q + 1.0;
    uint64_t a = (uint64_t)((__builtin_sqrt(x) - 1.0) * 0.5);
    while (a > 0 && (uint64_t)Q * a * (a + 1) / 2 > s) --a;
    while ((uint64_t)Q * (a + 1) * (a + 2) / 2 <= s) ++a;
    const uint64_t o = s - (uint64_t)Q * a * (a + 1) / 2;
    const uint64_t pr = a * Q + o / (a + 1), c = o % (a + 1);
    return (uint32_t)(pr * (2 * pr + 1) + c * H);
}

// True when a plan's flags select the two-row band order (the column-major
// and row-major aligned orders take precedence).
__host__ __device__ __forceinline__ bool strip_band(uint32_t flags)
{
    return (flags & TRI_FLAG_STRIP_BAND) && !(flags & (TRI_FLAG_STRIP_COLS | TRI_FLAG_STRIP_ALIGN));
}

// Launch grid of a strip kernel for a plan's map, tile grid (m tiles a side,
// flags) and map grid (gx, gy).  The two-row band order needs G >= 4.
__host__ __forceinline__ StripGrid strip_grid(int map, int32_t m, uint32_t flags, uint64_t T,
                                              uint32_t gx, uint32_t gy, int32_t G, int32_t K,
                                              dim3 &grid)
{
    StripGrid s{0u, G, K, (int32_t)gx, (int32_t)gy};
    const uint64_t span = (uint64_t)G * (uint64_t)K;  // tile numbers per group
    if (map == TRI_MAP_LAMBDA && (flags & TRI_FLAG_STRIP_COLS)) {
        s.K = 1;
        s.strips = (uint32_t)strip_cols_prefix((uint32_t)((m + G - 1) / G), (uint32_t)m, (uint32_t)G);
        grid = dim3(s.strips, 1);
    } else if (map == TRI_MAP_LAMBDA && (flags & TRI_FLAG_STRIP_ALIGN)) {
        s.K = 1;
        s.strips = (uint32_t)strip_align_prefix((uint32_t)m, (uint32_t)G);
        grid = dim3(s.strips, 1);
    } else if (strip_band(flags) && map == TRI_MAP_LAMBDA) {
        s.K = 1;
        s.strips = (uint32_t)strip_align_prefix((uint32_t)((m + 1) / 2), (uint32_t)(G / 4));
        grid = dim3(s.strips, 1);
    } else if (strip_band(flags)) {
        s.K = 1;
        const uint32_t H = (uint32_t)G / 2;
        grid = dim3((gx + H - 1) / H, (gy + 1) / 2);
    } else if (map == TRI_MAP_LAMBDA) {
        s.strips = (uint32_t)((T + span - 1) / span * (uint64_t)K);
        grid = dim3(s.strips, 1);
    } else {
        grid = dim3((uint32_t)((gx + span - 1) / span * (uint64_t)K), gy);
    }
    return s;
}

// First tile number of this workgroup's strip; its tile t is first + t K.
template <int MAP>
__device__ __forceinline__ uint32_t strip_first(const TileGrid &g, const StripGrid &sg)
{
    uint32_t L = blockIdx.x;
    if constexpr (MAP == MAP_LAMBDA) {
        const uint32_t ns = sg.strips;
        if (g.flags & TRI_FLAG_XCD_SWIZZLE) {
            const uint32_t x = L & 7, q = ns >> 3, r = ns & 7;
            L = x * q + (x < r ? x : r) + (L >> 3);
        }
        // the orders act on whole groups
        const uint32_t K = (uint32_t)sg.K, ng = ns / K, grp = L / K, k = L % K;
        uint32_t G2 = grp;
        if (g.flags & TRI_FLAG_ORDER_REVERSE) G2 = ng - 1 - grp;
        else if (g.flags & TRI_FLAG_ORDER_PAIRS) G2 = (grp & 1) ? ng - 1 - (grp >> 1) : (grp >> 1);
        if (g.flags & TRI_FLAG_STRIP_COLS) return strip_cols_first(G2, (uint32_t)g.m, (uint32_t)sg.G);
        if (g.flags & TRI_FLAG_STRIP_ALIGN) return strip_align_first(G2, (uint32_t)sg.G);
        if (g.flags & TRI_FLAG_STRIP_BAND) return strip_band_first(G2, (uint32_t)sg.G);
        return G2 * K * (uint32_t)sg.G + k;
    } else {
        if (strip_band(g.flags)) return L * (uint32_t)(sg.G / 2);
        const uint32_t K = (uint32_t)sg.K;
        return (L / K) * K * (uint32_t)sg.G + L % K;
    }
}

// Tile t of the strip starting at `first`, or false when it maps to no tile
// (beyond the grid, or a bounding-box block above the diagonal).  Lambda
// takes its 32-bit exact form (strip kernels need fewer than 2^32 tiles).
template <int MAP>
__device__ __forceinline__ bool strip_tile(const TileGrid &g, const StripGrid &sg, uint32_t first,
                                           int k, int32_t &bi, int32_t &bj)
{
    if constexpr (MAP == MAP_LAMBDA) {
        uint64_t w = first + (uint64_t)k * (uint32_t)sg.K;
        int kc = k;  // the tile's column offset within its strip
        if (strip_band(g.flags)) {
            // column c0 + k / 2 of row 2 p + (k & 1): T_2p+1 = T_2p + 2 p + 1
            int32_t r0, c0;
            if (g.T <= (1ull << 24)) lambda_tile_24(first, r0, c0);
            else lambda_tile_32(first, r0, c0);
            kc = k >> 1;
            w = first + (uint64_t)kc + (uint64_t)(k & 1) * (uint32_t)(r0 + 1);
        }
        if (w >= g.T) return false;
        if (g.T <= (1ull << 24)) lambda_tile_24((uint32_t)w, bi, bj);
        else lambda_tile_32((uint32_t)w, bi, bj);
        // an aligned strip ends with its row: tile k of the strip has
        // column bj0 + kc >= kc, the next row's tiles columns below kc
        if ((g.flags & (TRI_FLAG_STRIP_COLS | TRI_FLAG_STRIP_ALIGN | TRI_FLAG_STRIP_BAND)) && bj < kc)
            return false;
    } else {
        int32_t bx = (int32_t)first + k * sg.K, by = (int32_t)blockIdx.y;
        if (strip_band(g.flags)) {
            bx = (int32_t)first + (k >> 1);
            by = 2 * by + (k & 1);
            if (by >= sg.gy) return false;
        }
        if (bx >= sg.gx) return false;
        if (!tile_at_xy<MAP>(g, bx, by, bi, bj)) return false;
    }
    return (uint32_t)bi < (uint32_t)g.m && (uint32_t)bj <= (uint32_t)bi;
}

// First tile index >= k of the strip that maps to a tile (G if none).
template <int MAP>
__device__ __forceinline__ int strip_next(const TileGrid &g, const StripGrid &sg, uint32_t first,
                                          int k, int32_t &bi, int32_t &bj)
{
    for (; k < sg.G; ++k)
        if (strip_tile<MAP>(g, sg, first, k, bi, bj)) return k;
    return sg.G;
}

// Tiles per strip asked for by a plan's TRI_FLAG_STRIP bits (0: none).
__host__ __device__ __forceinline__ int32_t strip_flag_len(uint32_t flags)
{
    const uint32_t v = (flags & TRI_FLAG_STRIP_MASK) >> 8;
    return v ? (1 << (v - 1)) : 0;
}

// ---------------------------------------------------------------------------
// UTM (Section 4.2, Avril et al.): thread k of a problem of size N owns the
// k-th pair (a, b), 1 <= a < b <= N, in lexicographic order:
//   a = floor((2N + 1 - sqrt(4N^2 - 4N - 8k + 1)) / 2),
//   b = a + 1 + k - (a - 1)(2N - a) / 2.
// The root is taken in FP32 and a is corrected by integer steps against
// the row starts S(a) = (a - 1)(2N - a) / 2, which removes the accuracy limit
// of the original (k <= 1e8).  A lower-triangle cell is then
//   (i, j) = (N - 1 - a, N - b)   with N = side + 1,
// which enumerates 0 <= j <= i < side (consecutive k: consecutive j).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void utm_cell(uint64_t k, int64_t side, int32_t &i, int32_t &j)
{
    const int64_t N = side + 1;
    const double Dd = 4.0 * (double)N * (double)N - 4.0 * (double)N - 8.0 * (double)k + 1.0;
    const float s = __builtin_amdgcn_sqrtf((float)Dd);
    int64_t a = (int64_t)(((double)(2 * N + 1) - (double)s) * 0.5);
    a = a < 1 ? 1 : (a > N - 1 ? N - 1 : a);
    auto S = [N](int64_t aa) { return (aa - 1) * (2 * N - aa) / 2; };
    // S is strictly increasing on [1, N), so both loops end; for the sizes
    // a 32-bit grid can reach they run at most once.
    while (a > 1 && S(a) > (int64_t)k) --a;
    while (a < N - 1 && S(a + 1) <= (int64_t)k) ++a;
    const int64_t b = a + 1 + (int64_t)k - S(a);
    i = (int32_t)(N - 1 - a);
    j = (int32_t)(N - b);
}

}  // namespace trimap
