// Triangular elementwise kernels: one workgroup per tile rho x rho, the tile
// chosen by a parallel-space map (block-space mapping, Section 3.1: the
// block coordinate is mapped, each thread adds its offset inside the block).
//
//  * AXPYT_F32: C[i][j] = fl(fl(a X[i][j]) + Y[j][i]) for j <= i.  The mirror
//    tile of Y is read row-major (coalesced) and transposed through LDS.
//  * XORMUL_I32: C[i][j] = (A[i] xor B[j]) + i j (mod 2^32), the dummy
//    kernel of Sections 4.1 and 5 with a real per-cell store.
//  * EDM4_F32: C[i][j] = |P_i - P_j| for four features per point, the
//    global-memory distance test of Section 5: both points come straight
//    from global memory (they stay in L1/L2), nothing is staged in LDS.
//
// All are HBM-bound: 12 B (axpyt) or 4 B (xormul, edm4) of algorithmic
// traffic per cell.  Rows move as 16-byte vectors; stores are non-temporal (the output
// is not re-read).  UTM (thread space) has no tile and gets its own scalar
// kernel, reading Y[j][i] straight from memory as the map implies.
#include <type_traits>

#include "common.hpp"
#include "maps.hpp"

namespace trimap {

TileGrid plan_tile_grid(const tri_plan *p);

typedef float f4 __attribute__((ext_vector_type(4)));
typedef int i4 __attribute__((ext_vector_type(4)));

struct ElemArgs {
    TileGrid g;
    int32_t n;
    int64_t ld;
    const void *x;
    const void *y;
    void *c;
    float a;
};

// threads per workgroup and elements per vector for a tile size
template <int TILE, bool VECTOR>
struct ElemShape {
    static constexpr int VEC = (VECTOR && TILE >= 16) ? 4 : 1;
    static constexpr int NT_RAW = TILE * TILE / VEC;
    // tile 128 takes 512 threads: its 66 KB transpose buffer holds the CU to
    // two workgroups, so the extra waves are what keeps more loads in flight
    static constexpr int NT_MAX = TILE >= 128 ? 512 : 256;
    static constexpr int NT = NT_RAW > NT_MAX ? NT_MAX : NT_RAW;
    static constexpr int VPR = TILE / VEC;    // vectors per row
    static constexpr int RPP = NT / VPR;      // rows per pass
    static constexpr int PASSES = TILE / RPP;
    static_assert(RPP * PASSES == TILE, "tile shape");
};

template <int MAP, int TILE, bool VECTOR>
__global__ void __launch_bounds__((ElemShape<TILE, VECTOR>::NT)) k_axpyt(ElemArgs p)
{
    using S = ElemShape<TILE, VECTOR>;
    int32_t bi, bj;
    if (!tile_of_block<MAP>(p.g, bi, bj)) return;

    __shared__ float ys[TILE][TILE + 1];
    const int tr = threadIdx.x / S::VPR;
    const int tc = (threadIdx.x % S::VPR) * S::VEC;
    const int32_t n = p.n;
    const int64_t ld = p.ld;
    const int32_t i0 = bi * TILE, j0 = bj * TILE;
    const float *X = (const float *)p.x;
    const float *Y = (const float *)p.y;
    float *C = (float *)p.c;
    const float a = p.a;
    // every cell of the tile is in the domain
    const bool full = (bj < bi) && (i0 + TILE <= n);

    // Every load is unconditional, so that all of them are in flight at once
    // (a load under a condition is waited for where the branches rejoin).
    // On tiles that cross the diagonal or the last row the addresses are
    // clamped into the n x ld matrices; the values read there belong to
    // cells that are never stored.  X first, then the mirror tile of Y
    // (rows j0.., columns i0..; Y[j][i] lands in ys[j-j0][i-i0]).
    using V = typename std::conditional<S::VEC == 4, f4, float>::type;
    const int32_t cmax = (int32_t)(ld - S::VEC);  // last column start of a vector
    V xv[S::PASSES], yv[S::PASSES];
#pragma unroll
    for (int ps = 0; ps < S::PASSES; ++ps) {
        const int r = tr + ps * S::RPP;
        int32_t i = i0 + r, jc = j0 + tc;
        if (!full) {
            i = i < n ? i : n - 1;
            jc = jc < cmax ? jc : cmax;
        }
        xv[ps] = __builtin_nontemporal_load((const V *)(X + (int64_t)i * ld + jc));
    }
#pragma unroll
    for (int ps = 0; ps < S::PASSES; ++ps) {
        const int r = tr + ps * S::RPP;
        int32_t jr = j0 + r, ic = i0 + tc;
        if (!full) {
            jr = jr < n ? jr : n - 1;
            ic = ic < cmax ? ic : cmax;
        }
        yv[ps] = __builtin_nontemporal_load((const V *)(Y + (int64_t)jr * ld + ic));
    }
#pragma unroll
    for (int ps = 0; ps < S::PASSES; ++ps) {
        const int r = tr + ps * S::RPP;
        if constexpr (S::VEC == 4) {
            ys[r][tc + 0] = yv[ps].x;
            ys[r][tc + 1] = yv[ps].y;
            ys[r][tc + 2] = yv[ps].z;
            ys[r][tc + 3] = yv[ps].w;
        } else {
            ys[r][tc] = yv[ps];
        }
    }
    __syncthreads();

#pragma unroll
    for (int ps = 0; ps < S::PASSES; ++ps) {
        const int r = tr + ps * S::RPP;
        const int32_t i = i0 + r, jc = j0 + tc;
        if (!full && (i >= n || jc > i)) continue;
        float *crow = C + (int64_t)i * ld + jc;
        if constexpr (S::VEC == 4) {
            const f4 x4 = xv[ps];
            f4 o;
            o.x = __fadd_rn(__fmul_rn(a, x4.x), ys[tc + 0][r]);
            o.y = __fadd_rn(__fmul_rn(a, x4.y), ys[tc + 1][r]);
            o.z = __fadd_rn(__fmul_rn(a, x4.z), ys[tc + 2][r]);
            o.w = __fadd_rn(__fmul_rn(a, x4.w), ys[tc + 3][r]);
            if (full || jc + 3 <= i) {
                __builtin_nontemporal_store(o, (f4 *)crow);
            } else {  // the vector straddles the diagonal
                crow[0] = o.x;
                if (jc + 1 <= i) crow[1] = o.y;
                if (jc + 2 <= i) crow[2] = o.z;
            }
        } else {
            __builtin_nontemporal_store(__fadd_rn(__fmul_rn(a, xv[ps]), ys[tc][r]), crow);
        }
    }
}

// Strip form of AXPYT for tiles 16 and 32 (plans with TRI_FLAG_STRIP): a
// workgroup of four waves walks G consecutive tiles of the map (strip_first
// and strip_tile; every tile still mapped on its own), wave w taking tiles
// w, w + 4, w + 8, ... of the strip, so that the four waves work on adjacent
// tiles and one dispatch serves G tiles instead of one.  A wave moves a
// whole tile by itself: 16-byte vectors, rows per pass 64 / (TILE / 4), and
// its own transpose buffer in LDS (the LDS operations of one wave execute in
// order, so a wave needs no barrier between its tiles).  The loads of the
// wave's next tile are issued before the current tile's transpose and
// stores.  Same arithmetic and operation order as k_axpyt.
template <int MAP, int TILE>
__global__ void __launch_bounds__(256) k_axpyt_strip(ElemArgs p, StripGrid sg)
{
    constexpr int VPR = TILE / 4, RPP = 64 / VPR, PASSES = TILE / RPP;
    static_assert(RPP * PASSES == TILE, "tile shape");
    __shared__ float ysh[4][TILE][TILE + 1];
    const int l = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float (*ys)[TILE + 1] = ysh[w];
    const int tr = l / VPR, tc = (l % VPR) * 4;
    const int32_t n = p.n;
    const int64_t ld = p.ld;
    const float *X = (const float *)p.x;
    const float *Y = (const float *)p.y;
    float *C = (float *)p.c;
    const float a = p.a;
    const int32_t cmax = (int32_t)(ld - 4);  // last column start of a vector
    const uint32_t first = strip_first<MAP>(p.g, sg);

    // the wave's next tile at or after strip index k (k >= G: none)
    auto next = [&](int k, int32_t &bi, int32_t &bj) {
        for (; k < sg.G; k += 4)
            if (strip_tile<MAP>(p.g, sg, first, k, bi, bj)) break;
        bi = __builtin_amdgcn_readfirstlane(bi);
        bj = __builtin_amdgcn_readfirstlane(bj);
        return k;
    };
    f4 xv[PASSES], yv[PASSES];
    // every load unconditional; addresses clamped into the matrices on
    // tiles that cross the diagonal or the last row (values never stored)
    auto load = [&](int32_t bi, int32_t bj) {
        const int32_t i0 = bi * TILE, j0 = bj * TILE;
        const bool full = (bj < bi) && (i0 + TILE <= n);
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int r = tr + ps * RPP;
            int32_t i = i0 + r, jc = j0 + tc;
            if (!full) {
                i = i < n ? i : n - 1;
                jc = jc < cmax ? jc : cmax;
            }
            xv[ps] = __builtin_nontemporal_load((const f4 *)(X + (int64_t)i * ld + jc));
        }
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int r = tr + ps * RPP;
            int32_t jr = j0 + r, ic = i0 + tc;
            if (!full) {
                jr = jr < n ? jr : n - 1;
                ic = ic < cmax ? ic : cmax;
            }
            yv[ps] = __builtin_nontemporal_load((const f4 *)(Y + (int64_t)jr * ld + ic));
        }
    };

    int32_t bi = 0, bj = 0;
    int k = next(w, bi, bj);
    if (k >= sg.G) return;
    load(bi, bj);
    while (k < sg.G) {
        // this tile's operands into the transpose buffer and registers
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int r = tr + ps * RPP;
            ys[r][tc + 0] = yv[ps].x;
            ys[r][tc + 1] = yv[ps].y;
            ys[r][tc + 2] = yv[ps].z;
            ys[r][tc + 3] = yv[ps].w;
        }
        f4 xc[PASSES];
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) xc[ps] = xv[ps];
        const int32_t i0 = bi * TILE, j0 = bj * TILE;
        const bool full = (bj < bi) && (i0 + TILE <= n);
        // the next tile's loads, in flight during this tile's stores
        int32_t nbi = 0, nbj = 0;
        const int nk = next(k + 4, nbi, nbj);
        if (nk < sg.G) load(nbi, nbj);
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int r = tr + ps * RPP;
            const int32_t i = i0 + r, jc = j0 + tc;
            if (!full && (i >= n || jc > i)) continue;
            float *crow = C + (int64_t)i * ld + jc;
            f4 o;
            o.x = __fadd_rn(__fmul_rn(a, xc[ps].x), ys[tc + 0][r]);
            o.y = __fadd_rn(__fmul_rn(a, xc[ps].y), ys[tc + 1][r]);
            o.z = __fadd_rn(__fmul_rn(a, xc[ps].z), ys[tc + 2][r]);
            o.w = __fadd_rn(__fmul_rn(a, xc[ps].w), ys[tc + 3][r]);
            if (full || jc + 3 <= i) {
                __builtin_nontemporal_store(o, (f4 *)crow);
            } else {  // the vector straddles the diagonal
                crow[0] = o.x;
                if (jc + 1 <= i) crow[1] = o.y;
                if (jc + 2 <= i) crow[2] = o.z;
            }
        }
        k = nk;
        bi = nbi;
        bj = nbj;
    }
}

// Tile 16 in strips: a wave moves two tiles at once, one per half-wave
// (tiles 2 j and 2 j + 1 of the strip, j = w, w + 4, ...), so that where the
// two are neighbours in a tile row (the usual case) every load and store
// instruction covers whole 128-byte lines: 8 rows x 64 bytes of each tile.
// Each half-wave maps its tile on its own; a half whose tile is missing
// (past the strip or the grid) loads tile (0, 0) and stores nothing.
template <int MAP>
__global__ void __launch_bounds__(256) k_axpyt_strip_pairs(ElemArgs p, StripGrid sg)
{
    constexpr int TILE = 16, RPP = 8, PASSES = 2;
    __shared__ float ysh[8][TILE][TILE + 1];
    const int l = threadIdx.x & 63, h = l >> 5, hl = l & 31;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float (*ys)[TILE + 1] = ysh[2 * w + h];
    const int tr = hl / 4, tc = (hl % 4) * 4;
    const int32_t n = p.n;
    const int64_t ld = p.ld;
    const float *X = (const float *)p.x;
    const float *Y = (const float *)p.y;
    float *C = (float *)p.c;
    const float a = p.a;
    const int32_t cmax = (int32_t)(ld - 4);
    const uint32_t first = strip_first<MAP>(p.g, sg);

    // this half's tile of pair j (false: none)
    auto tile = [&](int j, int32_t &bi, int32_t &bj) {
        const int k = 2 * j + h;
        const bool v = k < sg.G && strip_tile<MAP>(p.g, sg, first, k, bi, bj);
        if (!v) bi = bj = 0;
        return v;
    };
    f4 xv[PASSES], yv[PASSES];
    auto load = [&](int32_t bi, int32_t bj) {
        const int32_t i0 = bi * TILE, j0 = bj * TILE;
        const bool full = (bj < bi) && (i0 + TILE <= n);
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int r = tr + ps * RPP;
            int32_t i = i0 + r, jc = j0 + tc;
            if (!full) {
                i = i < n ? i : n - 1;
                jc = jc < cmax ? jc : cmax;
            }
            xv[ps] = __builtin_nontemporal_load((const f4 *)(X + (int64_t)i * ld + jc));
        }
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int r = tr + ps * RPP;
            int32_t jr = j0 + r, ic = i0 + tc;
            if (!full) {
                jr = jr < n ? jr : n - 1;
                ic = ic < cmax ? ic : cmax;
            }
            yv[ps] = __builtin_nontemporal_load((const f4 *)(Y + (int64_t)jr * ld + ic));
        }
    };

    int j = w;
    int32_t bi = 0, bj = 0;
    bool v = tile(j, bi, bj);
    load(bi, bj);
    while (2 * j < sg.G) {
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int r = tr + ps * RPP;
            ys[r][tc + 0] = yv[ps].x;
            ys[r][tc + 1] = yv[ps].y;
            ys[r][tc + 2] = yv[ps].z;
            ys[r][tc + 3] = yv[ps].w;
        }
        f4 xc[PASSES];
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) xc[ps] = xv[ps];
        const int32_t i0 = bi * TILE, j0 = bj * TILE;
        const bool full = v && (bj < bi) && (i0 + TILE <= n);
        const bool cv = v;
        // the next pair's loads, in flight during this pair's stores
        int32_t nbi = 0, nbj = 0;
        const int nj = j + 4;
        const bool nv = tile(nj, nbi, nbj);
        if (2 * nj < sg.G) load(nbi, nbj);
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int r = tr + ps * RPP;
            const int32_t i = i0 + r, jc = j0 + tc;
            if (!cv || (!full && (i >= n || jc > i))) continue;
            float *crow = C + (int64_t)i * ld + jc;
            f4 o;
            o.x = __fadd_rn(__fmul_rn(a, xc[ps].x), ys[tc + 0][r]);
            o.y = __fadd_rn(__fmul_rn(a, xc[ps].y), ys[tc + 1][r]);
            o.z = __fadd_rn(__fmul_rn(a, xc[ps].z), ys[tc + 2][r]);
            o.w = __fadd_rn(__fmul_rn(a, xc[ps].w), ys[tc + 3][r]);
            if (full || jc + 3 <= i) {
                __builtin_nontemporal_store(o, (f4 *)crow);
            } else {  // the vector straddles the diagonal
                crow[0] = o.x;
                if (jc + 1 <= i) crow[1] = o.y;
                if (jc + 2 <= i) crow[2] = o.z;
            }
        }
        j = nj;
        v = nv;
        bi = nbi;
        bj = nbj;
    }
}

// Tile 16 in two-row band strips (TRI_FLAG_STRIP_BAND): a wave moves a
// 2 x 2 block of tiles at once (tiles 4 q .. 4 q + 3 of the strip, rows
// 2 p and 2 p + 1, columns c and c + 1, q = w, w + 4, ...), each of the
// four located by the map on its own.  Within the block every row of X and
// C is a whole 128-byte line across two tiles, and so is every row of the
// mirror block of Y across the two tile rows; the block moves as one
// 32 x 32 transpose through the wave's LDS buffer.  Tile (r, c) of the
// block is tile 4 q + 2 c + r; a lane's 16-byte vector at block row R,
// column C belongs to tile (R / 16, C / 16) for X and C and to tile
// (C / 16, R / 16) for Y, whose rows are the tiles' columns.  A missing
// tile (above the diagonal, past the last row or the strip) loads from
// tile (0, 0) and stores nothing.  Same arithmetic and operation order as
// k_axpyt.
template <int MAP>
__global__ void __launch_bounds__(256) k_axpyt_strip_quads(ElemArgs p, StripGrid sg)
{
    constexpr int TILE = 16, BLK = 32, VPR = BLK / 4, RPP = 64 / VPR, PASSES = BLK / RPP;
    __shared__ float ysh[4][BLK][BLK + 1];
    const int l = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float (*ys)[BLK + 1] = ysh[w];
    const int tr = l / VPR, tc = (l % VPR) * 4;  // block row (pass 0), block column
    const int lc = tc / TILE, tcl = tc % TILE;    // the lane's tile column, column in it
    const int32_t n = p.n;
    const int64_t ld = p.ld;
    const float *X = (const float *)p.x;
    const float *Y = (const float *)p.y;
    float *C = (float *)p.c;
    const float a = p.a;
    const int32_t cmax = (int32_t)(ld - 4);
    const uint32_t first = strip_first<MAP>(p.g, sg);

    struct Quad {
        int32_t bi[2][2], bj[2][2];  // [r][c]
        bool v[2][2];
    };
    auto locate = [&](int q, Quad &Q) {
        bool any = false;
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int k = 4 * q + 2 * c + r;
                int32_t bi = 0, bj = 0;
                bool v = k < sg.G && strip_tile<MAP>(p.g, sg, first, k, bi, bj);
                if (!v) bi = bj = 0;
                Q.bi[r][c] = __builtin_amdgcn_readfirstlane(bi);
                Q.bj[r][c] = __builtin_amdgcn_readfirstlane(bj);
                Q.v[r][c] = v;
                any = any || v;
            }
        return any;
    };
    f4 xv[PASSES], yv[PASSES];
    auto load = [&](const Quad &Q) {
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int R = tr + ps * RPP, rt = R / TILE, rl = R % TILE;
            // X: tile (rt, lc), row rl, columns tcl ..
            const int32_t bi = lc ? Q.bi[rt][1] : Q.bi[rt][0];
            const int32_t bj = lc ? Q.bj[rt][1] : Q.bj[rt][0];
            const bool full = (bj < bi) && (bi * TILE + TILE <= n);
            int32_t i = bi * TILE + rl, jc = bj * TILE + tcl;
            if (!full) {
                i = i < n ? i : n - 1;
                jc = jc < cmax ? jc : cmax;
            }
            xv[ps] = __builtin_nontemporal_load((const f4 *)(X + (int64_t)i * ld + jc));
        }
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int R = tr + ps * RPP, rt = R / TILE, rl = R % TILE;
            // Y: the mirror of tile (lc, rt): Y row bj * 16 + rl, columns bi * 16 + tcl ..
            const int32_t bi = rt ? Q.bi[lc][1] : Q.bi[lc][0];
            const int32_t bj = rt ? Q.bj[lc][1] : Q.bj[lc][0];
            const bool full = (bj < bi) && (bi * TILE + TILE <= n);
            int32_t jr = bj * TILE + rl, ic = bi * TILE + tcl;
            if (!full) {
                jr = jr < n ? jr : n - 1;
                ic = ic < cmax ? ic : cmax;
            }
            yv[ps] = __builtin_nontemporal_load((const f4 *)(Y + (int64_t)jr * ld + ic));
        }
    };

    int q = w;
    Quad Q;
    bool v = locate(q, Q);
    while (4 * q < sg.G && !v) v = locate(q += 4, Q);
    if (4 * q >= sg.G) return;
    load(Q);
    while (4 * q < sg.G) {
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int R = tr + ps * RPP;
            ys[R][tc + 0] = yv[ps].x;
            ys[R][tc + 1] = yv[ps].y;
            ys[R][tc + 2] = yv[ps].z;
            ys[R][tc + 3] = yv[ps].w;
        }
        f4 xc[PASSES];
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) xc[ps] = xv[ps];
        const Quad cq = Q;
        // the next block's loads, in flight during this block's stores
        int nq = q + 4;
        bool nv = false;
        while (4 * nq < sg.G && !(nv = locate(nq, Q))) nq += 4;
        if (4 * nq < sg.G) load(Q);
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int R = tr + ps * RPP, rt = R / TILE, rl = R % TILE;
            const int32_t bi = lc ? cq.bi[rt][1] : cq.bi[rt][0];
            const int32_t bj = lc ? cq.bj[rt][1] : cq.bj[rt][0];
            const bool tv = lc ? cq.v[rt][1] : cq.v[rt][0];
            const bool full = tv && (bj < bi) && (bi * TILE + TILE <= n);
            const int32_t i = bi * TILE + rl, jc = bj * TILE + tcl;
            if (!tv || (!full && (i >= n || jc > i))) continue;
            float *crow = C + (int64_t)i * ld + jc;
            f4 o;
            o.x = __fadd_rn(__fmul_rn(a, xc[ps].x), ys[tc + 0][R]);
            o.y = __fadd_rn(__fmul_rn(a, xc[ps].y), ys[tc + 1][R]);
            o.z = __fadd_rn(__fmul_rn(a, xc[ps].z), ys[tc + 2][R]);
            o.w = __fadd_rn(__fmul_rn(a, xc[ps].w), ys[tc + 3][R]);
            if (full || jc + 3 <= i) {
                __builtin_nontemporal_store(o, (f4 *)crow);
            } else {  // the vector straddles the diagonal
                crow[0] = o.x;
                if (jc + 1 <= i) crow[1] = o.y;
                if (jc + 2 <= i) crow[2] = o.z;
            }
        }
        q = nq;
        (void)nv;
    }
}

template <int MAP, int TILE, bool VECTOR>
__global__ void __launch_bounds__((ElemShape<TILE, VECTOR>::NT)) k_xormul(ElemArgs p)
{
    using S = ElemShape<TILE, VECTOR>;
    int32_t bi, bj;
    if (!tile_of_block<MAP>(p.g, bi, bj)) return;

    const int tr = threadIdx.x / S::VPR;
    const int tc = (threadIdx.x % S::VPR) * S::VEC;
    const int32_t n = p.n;
    const int64_t ld = p.ld;
    const int32_t i0 = bi * TILE, j0 = bj * TILE;
    const uint32_t *A = (const uint32_t *)p.x;
    const uint32_t *B = (const uint32_t *)p.y;
    int32_t *C = (int32_t *)p.c;
    const bool full = (bj < bi) && (i0 + TILE <= n);

#pragma unroll
    for (int ps = 0; ps < S::PASSES; ++ps) {
        const int r = tr + ps * S::RPP;
        const int32_t i = i0 + r, jc = j0 + tc;
        if (!full && (i >= n || jc > i)) continue;
        const uint32_t ai = A[i];
        int32_t *crow = C + (int64_t)i * ld + jc;
        if constexpr (S::VEC == 4) {
            // B[jc .. jc+3]: jc + 3 may pass n on the last tile row, so read
            // element by element there (B holds exactly n values)
            uint32_t b0 = B[jc], b1 = 0, b2 = 0, b3 = 0;
            if (full || jc + 3 < n) { b1 = B[jc + 1]; b2 = B[jc + 2]; b3 = B[jc + 3]; }
            else {
                if (jc + 1 < n) b1 = B[jc + 1];
                if (jc + 2 < n) b2 = B[jc + 2];
            }
            const uint32_t ui = (uint32_t)i;
            i4 o;
            o.x = (int32_t)((ai ^ b0) + ui * (uint32_t)(jc + 0));
            o.y = (int32_t)((ai ^ b1) + ui * (uint32_t)(jc + 1));
            o.z = (int32_t)((ai ^ b2) + ui * (uint32_t)(jc + 2));
            o.w = (int32_t)((ai ^ b3) + ui * (uint32_t)(jc + 3));
            if (full || jc + 3 <= i) {
                __builtin_nontemporal_store(o, (i4 *)crow);
            } else {
                crow[0] = o.x;
                if (jc + 1 <= i) crow[1] = o.y;
                if (jc + 2 <= i) crow[2] = o.z;
            }
        } else {
            const uint32_t v = (ai ^ B[jc]) + (uint32_t)i * (uint32_t)jc;
            __builtin_nontemporal_store((int32_t)v, crow);
        }
    }
}

// |P_i - P_j| with a fixed operation order: differences, squares, the sum
// ((dx^2 + dy^2) + dz^2) + dw^2, each rounded to binary32, then a correctly
// rounded square root.
__device__ __forceinline__ float dist4(f4 a, f4 b)
{
    const float dx = __fsub_rn(a.x, b.x), dy = __fsub_rn(a.y, b.y);
    const float dz = __fsub_rn(a.z, b.z), dw = __fsub_rn(a.w, b.w);
    float s = __fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy));
    s = __fadd_rn(s, __fmul_rn(dz, dz));
    s = __fadd_rn(s, __fmul_rn(dw, dw));
    return __builtin_sqrtf(s);
}

template <int MAP, int TILE, bool VECTOR>
__global__ void __launch_bounds__((ElemShape<TILE, VECTOR>::NT)) k_edm4(ElemArgs p)
{
    using S = ElemShape<TILE, VECTOR>;
    int32_t bi, bj;
    if (!tile_of_block<MAP>(p.g, bi, bj)) return;

    const int tr = threadIdx.x / S::VPR;
    const int tc = (threadIdx.x % S::VPR) * S::VEC;
    const int32_t n = p.n;
    const int64_t ld = p.ld;
    const int32_t i0 = bi * TILE, j0 = bj * TILE;
    const f4 *P = (const f4 *)p.x;
    float *C = (float *)p.c;
    const bool full = (bj < bi) && (i0 + TILE <= n);

    // the lane's column points (the same for all its rows), read once from
    // global memory; past n - 1 (the ragged last tile) clamped and unused
    const int32_t jc = j0 + tc;
    f4 pj[S::VEC];
#pragma unroll
    for (int v = 0; v < S::VEC; ++v) pj[v] = P[jc + v < n ? jc + v : n - 1];

#pragma unroll
    for (int ps = 0; ps < S::PASSES; ++ps) {
        const int r = tr + ps * S::RPP;
        const int32_t i = i0 + r;
        if (!full && (i >= n || jc > i)) continue;
        const f4 pi = P[i];
        float *crow = C + (int64_t)i * ld + jc;
        if constexpr (S::VEC == 4) {
            f4 o;
            o.x = dist4(pi, pj[0]);
            o.y = dist4(pi, pj[1]);
            o.z = dist4(pi, pj[2]);
            o.w = dist4(pi, pj[3]);
            if (full || jc + 3 <= i) {
                __builtin_nontemporal_store(o, (f4 *)crow);
            } else {  // the vector straddles the diagonal
                crow[0] = o.x;
                if (jc + 1 <= i) crow[1] = o.y;
                if (jc + 2 <= i) crow[2] = o.z;
            }
        } else {
            __builtin_nontemporal_store(dist4(pi, pj[0]), crow);
        }
    }
}

// UTM: thread k owns cell utm_cell(k); no tile, no LDS.
template <int OP>
__global__ void __launch_bounds__(kUtmThreads) k_elem_utm(ElemArgs p, int64_t elements)
{
    const uint64_t k = ((uint64_t)blockIdx.y * gridDim.x + blockIdx.x) * kUtmThreads + threadIdx.x;
    if (k >= (uint64_t)elements) return;
    int32_t i, j;
    utm_cell(k, p.n, i, j);
    if ((uint32_t)i >= (uint32_t)p.n || (uint32_t)j > (uint32_t)i) return;
    const int64_t ld = p.ld;
    if constexpr (OP == TRI_OP_AXPYT_F32) {
        const float *X = (const float *)p.x;
        const float *Y = (const float *)p.y;
        ((float *)p.c)[(int64_t)i * ld + j] =
            __fadd_rn(__fmul_rn(p.a, X[(int64_t)i * ld + j]), Y[(int64_t)j * ld + i]);
    } else if constexpr (OP == TRI_OP_EDM4_F32) {
        const f4 *P = (const f4 *)p.x;
        ((float *)p.c)[(int64_t)i * ld + j] = dist4(P[i], P[j]);
    } else {
        const uint32_t *A = (const uint32_t *)p.x;
        const uint32_t *B = (const uint32_t *)p.y;
        ((int32_t *)p.c)[(int64_t)i * ld + j] =
            (int32_t)((A[i] ^ B[j]) + (uint32_t)i * (uint32_t)j);
    }
}

template <int OP, int MAP, int TILE, bool VECTOR>
static void launch_tile(const tri_plan *p, const ElemArgs &args, hipStream_t s)
{
    const dim3 grid(p->gx, p->gy);
    constexpr int NT = ElemShape<TILE, VECTOR>::NT;
    if constexpr (OP == TRI_OP_AXPYT_F32)
        k_axpyt<MAP, TILE, VECTOR><<<grid, NT, 0, s>>>(args);
    else if constexpr (OP == TRI_OP_EDM4_F32)
        k_edm4<MAP, TILE, VECTOR><<<grid, NT, 0, s>>>(args);
    else
        k_xormul<MAP, TILE, VECTOR><<<grid, NT, 0, s>>>(args);
}

template <int OP, int MAP, bool VECTOR>
static bool dispatch_tile(const tri_plan *p, const ElemArgs &args, hipStream_t s)
{
    switch (p->tile) {
    case 8: launch_tile<OP, MAP, 8, VECTOR>(p, args, s); return true;
    case 16: launch_tile<OP, MAP, 16, VECTOR>(p, args, s); return true;
    case 32: launch_tile<OP, MAP, 32, VECTOR>(p, args, s); return true;
    case 64: launch_tile<OP, MAP, 64, VECTOR>(p, args, s); return true;
    case 128: launch_tile<OP, MAP, 128, VECTOR>(p, args, s); return true;
    }
    return false;
}

template <int MAP, int TILE>
static void launch_axpyt_strip(const tri_plan *p, const ElemArgs &args, hipStream_t s)
{
    dim3 grid;
    const StripGrid sg = strip_grid(MAP, args.g.m, args.g.flags, args.g.T, p->gx, p->gy,
                                    strip_flag_len(p->flags), 1, grid);
    if constexpr (TILE == 16) {
        if (strip_band(p->flags)) k_axpyt_strip_quads<MAP><<<grid, 256, 0, s>>>(args, sg);
        else k_axpyt_strip_pairs<MAP><<<grid, 256, 0, s>>>(args, sg);
    } else
        k_axpyt_strip<MAP, TILE><<<grid, 256, 0, s>>>(args, sg);
}

template <int MAP>
static bool dispatch_axpyt_strip(const tri_plan *p, const ElemArgs &args, hipStream_t s)
{
    if (p->tile == 16) launch_axpyt_strip<MAP, 16>(p, args, s);
    else if (p->tile == 32) launch_axpyt_strip<MAP, 32>(p, args, s);
    else return false;
    return true;
}

template <int OP, bool VECTOR>
static bool dispatch_map(const tri_plan *p, const ElemArgs &args, hipStream_t s)
{
    // strips of tiles 16 and 32 (16-byte vectors, tile maps)
    if constexpr (OP == TRI_OP_AXPYT_F32 && VECTOR) {
        if ((p->tile == 16 || p->tile == 32) && strip_flag_len(p->flags) && p->map != TRI_MAP_UTM) {
            switch (p->map) {
            case TRI_MAP_BB: return dispatch_axpyt_strip<MAP_BB>(p, args, s);
            case TRI_MAP_RB: return dispatch_axpyt_strip<MAP_RB>(p, args, s);
            case TRI_MAP_REC: return dispatch_axpyt_strip<MAP_REC>(p, args, s);
            case TRI_MAP_LAMBDA: return dispatch_axpyt_strip<MAP_LAMBDA>(p, args, s);
            }
        }
    }
    switch (p->map) {
    case TRI_MAP_BB: return dispatch_tile<OP, MAP_BB, VECTOR>(p, args, s);
    case TRI_MAP_RB: return dispatch_tile<OP, MAP_RB, VECTOR>(p, args, s);
    case TRI_MAP_REC: return dispatch_tile<OP, MAP_REC, VECTOR>(p, args, s);
    case TRI_MAP_LAMBDA: return dispatch_tile<OP, MAP_LAMBDA, VECTOR>(p, args, s);
    case TRI_MAP_UTM:
        k_elem_utm<OP><<<dim3(p->gx, p->gy), kUtmThreads, 0, s>>>(args, p->elements);
        return true;
    }
    return false;
}

}  // namespace trimap

using namespace trimap;

extern "C" tri_status tri_launch_elementwise(const tri_plan *p, int op, const void *x,
                                             const void *y, void *c, int64_t ld, float a,
                                             void *stream)
{
    clear_error();
    if (!p) return fail(TRI_E_INVAL, "tri_launch_elementwise: plan is NULL");
    if (op != TRI_OP_XORMUL_I32 && op != TRI_OP_AXPYT_F32 && op != TRI_OP_EDM4_F32)
        return fail(TRI_E_INVAL, "tri_launch_elementwise: op = %d", op);
    if (!p->diag)
        return fail(TRI_E_UNSUPPORTED, "tri_launch_elementwise: needs include_diag = 1");
    if (p->tile > 128)
        return fail(TRI_E_UNSUPPORTED, "tri_launch_elementwise: tile %d > 128", p->tile);
    if (p->n == 0) return TRI_OK;
    if (!x || (!y && op != TRI_OP_EDM4_F32) || !c)
        return fail(TRI_E_INVAL, "tri_launch_elementwise: NULL buffer");
    if (ld < p->n) return fail(TRI_E_INVAL, "tri_launch_elementwise: ld %lld < n %lld",
                               (long long)ld, (long long)p->n);
    if (strip_band(p->flags) && strip_flag_len(p->flags) && strip_flag_len(p->flags) < 4)
        return fail(TRI_E_INVAL, "tri_launch_elementwise: two-row band strips need G >= 4 tiles");
    const uintptr_t cx = (uintptr_t)c, xx = (uintptr_t)x, yx = (uintptr_t)y;
    if ((cx | xx | yx) & 3) return fail(TRI_E_INVAL, "tri_launch_elementwise: unaligned buffer");
    if (op == TRI_OP_EDM4_F32 && (xx & 15))
        return fail(TRI_E_INVAL, "tri_launch_elementwise: EDM4 points need 16-byte alignment");
    bool vector = (ld % 4 == 0) && ((cx & 15) == 0);
    if (op == TRI_OP_AXPYT_F32) vector = vector && ((xx & 15) == 0) && ((yx & 15) == 0);

    ElemArgs args{plan_tile_grid(p), (int32_t)p->n, ld, x, y, c, a};
    hipStream_t s = (hipStream_t)stream;
    bool ok;
    if (op == TRI_OP_AXPYT_F32)
        ok = vector ? dispatch_map<TRI_OP_AXPYT_F32, true>(p, args, s)
                    : dispatch_map<TRI_OP_AXPYT_F32, false>(p, args, s);
    else if (op == TRI_OP_EDM4_F32)
        ok = vector ? dispatch_map<TRI_OP_EDM4_F32, true>(p, args, s)
                    : dispatch_map<TRI_OP_EDM4_F32, false>(p, args, s);
    else
        ok = vector ? dispatch_map<TRI_OP_XORMUL_I32, true>(p, args, s)
                    : dispatch_map<TRI_OP_XORMUL_I32, false>(p, args, s);
    if (!ok) return fail(TRI_E_UNSUPPORTED, "tri_launch_elementwise: tile %d", p->tile);
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}
