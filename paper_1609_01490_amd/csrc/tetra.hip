// The tetrahedral extension of the block-space map (Section 6) and a triplet
// kernel over it.
//
// Tile space: m = ceil(n_eff / rho) tiles per side, tiles (i, j, k) with
// 0 <= i <= j <= k < m, Tet(m) = m (m + 1) (m + 2) / 6 of them.  Layer k is
// the triangle of tiles (i, j), i <= j <= k, numbered as in two dimensions;
// block omega lies in the layer k with Tet(k) <= omega < Tet(k + 1), the
// integer part of the real root of x^3 + 3x^2 + 2x - 6 omega = 0.  The
// paper evaluates that root in closed form; here u = k + 1 solves
// u^3 - u = 6 Tet(k), so cbrt(6 omega) is a close estimate of u, taken in
// FP32 (v_log_f32 / v_exp_f32) or FP64, and two bounded integer steps make
// k exact, as the 2-D map does with its square root.  The rest of omega goes
// through the 2-D lambda.
//
// The bounding box is an m x m x m grid whose blocks with i <= j <= k are
// kept (Section 6: about 5/6 of them are discarded for large m).
//
// Strict triples a > b > c of n points are the non-strict tetrahedron of
// side n - 2 shifted: (a, b, c) = (k + 2, j + 1, i), as the strict triangle
// is the non-strict one of side n - 1 shifted by one row.
#include <new>
#include <type_traits>

#include "common.hpp"
#include "maps.hpp"

struct tri_tet {
    int64_t n;       // points
    int64_t ne;      // side of the non-strict tetrahedron that is tiled
    int32_t strict;  // 1: triples a > b > c; 0: a >= b >= c
    int32_t tile;
    int32_t map;     // TRI_MAP_BB or TRI_MAP_LAMBDA
    uint32_t flags;
    int64_t m;       // tiles per side
    uint64_t T;      // tiles, Tet(m)
    uint64_t cells;  // triples in the domain
    uint32_t gx, gy, gz;
    int64_t blocks;
};

namespace trimap {

struct TetGrid {
    int32_t m;
    uint32_t flags;
    uint64_t T;
};

__device__ __forceinline__ uint64_t tet_number(uint64_t k) { return k * (k + 1) / 2 * (k + 2) / 3; }

// Layer of block w: the largest k with Tet(k) <= w.
__device__ __forceinline__ uint32_t lambda3_layer(uint64_t w, uint32_t flags)
{
    int64_t k;
    if ((flags & TRI_FLAG_SQRT_F64) || (w >> 32)) {
        k = (int64_t)::cbrt(6.0 * (double)w) - 1;
    } else {
        const float x = 6.0f * (float)(uint32_t)w;
        const float u = x > 0.f ? __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 3.0f))
                                : 0.f;
        k = (int64_t)u - 1;
    }
    if (k < 0) k = 0;
    // The estimate is within one layer for every w below 2^62; the loops
    // run at most twice and end for any start since Tet is increasing.
    while (k > 0 && tet_number((uint64_t)k) > w) --k;
    while (tet_number((uint64_t)k + 1) <= w) ++k;
    return (uint32_t)k;
}

__device__ __forceinline__ void lambda3_tile(uint64_t w, uint32_t flags, int32_t &i, int32_t &j,
                                             int32_t &k)
{
    const uint32_t kk = lambda3_layer(w, flags);
    const uint64_t w2 = w - tet_number(kk);
    const uint32_t r = lambda_row(w2, flags & TRI_FLAG_SQRT_F64);
    k = (int32_t)kk;
    j = (int32_t)r;
    i = (int32_t)(w2 - (uint64_t)r * (r + 1) / 2);
}

// The same map for w < 2^24 (a 1-D grid, FP32 roots) in 32-bit arithmetic:
// there k <= 470, so Tet(k + 1) and the layer's 2-D numbering fit in 32 bits.
__device__ __forceinline__ uint32_t tet32(uint32_t k) { return k * (k + 1) / 2 * (k + 2) / 3; }

__device__ __forceinline__ void lambda3_tile_24(uint32_t w, int32_t &i, int32_t &j, int32_t &k)
{
    const float x = 6.0f * (float)w;
    const float u = x > 0.f ? __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 3.0f)) : 0.f;
    int32_t kk = (int32_t)u - 1;
    if (kk < 0) kk = 0;
    while (kk > 0 && tet32((uint32_t)kk) > w) --kk;
    while (tet32((uint32_t)kk + 1) <= w) ++kk;
    k = kk;
    lambda_tile_24(w - tet32((uint32_t)kk), j, i);
}

template <int MAP>
__device__ __forceinline__ bool tet_of_block_raw(const TetGrid &g, int32_t &i, int32_t &j,
                                                 int32_t &k)
{
    if constexpr (MAP == MAP_BB) {
        i = (int32_t)blockIdx.x;
        j = (int32_t)blockIdx.y;
        k = (int32_t)blockIdx.z;
        return i <= j && j <= k;
    } else {
        if (g.flags & kLambda24) {  // 1-D grid of exactly T < 2^24 blocks
            lambda3_tile_24(blockIdx.x, i, j, k);
            return true;
        }
        const uint64_t L = (uint64_t)blockIdx.y * gridDim.x + blockIdx.x;
        if (L >= g.T) return false;
        lambda3_tile(L, g.flags, i, j, k);
        return true;
    }
}

template <int MAP>
__device__ __forceinline__ bool tet_of_block(const TetGrid &g, int32_t &i, int32_t &j, int32_t &k)
{
    if (!tet_of_block_raw<MAP>(g, i, j, k)) return false;
    return (uint32_t)k < (uint32_t)g.m && (uint32_t)j <= (uint32_t)k && (uint32_t)i <= (uint32_t)j;
}

static TetGrid tet_grid(const tri_tet *p)
{
    uint32_t f = p->flags;
    if (p->map == TRI_MAP_LAMBDA && f == 0 && p->gy == 1 && (uint64_t)p->gx == p->T &&
        p->T <= (1ull << 24))
        f |= kLambda24;
    return TetGrid{(int32_t)p->m, f, p->T};
}

// ---------------------------------------------------------------------------
// test hooks
// ---------------------------------------------------------------------------
template <int MAP>
__global__ void __launch_bounds__(64) k_tet_dump(TetGrid g, int64_t *out)
{
    if (threadIdx.x != 0) return;
    const uint64_t b = ((uint64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    int32_t i, j, k;
    const bool keep = tet_of_block_raw<MAP>(g, i, j, k);
    out[3 * b + 0] = keep ? i : -1;
    out[3 * b + 1] = keep ? j : -1;
    out[3 * b + 2] = keep ? k : -1;
}

__global__ void __launch_bounds__(256) k_lambda3_eval(const uint64_t *omega, int64_t count,
                                                      uint32_t flags, int64_t *out)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= count) return;
    int32_t i, j, k;
    lambda3_tile(omega[t], flags, i, j, k);
    out[3 * t + 0] = i;
    out[3 * t + 1] = j;
    out[3 * t + 2] = k;
}

// ---------------------------------------------------------------------------
// triangles of the neighbour graph
// ---------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));

struct TriArgs {
    TetGrid g;
    int32_t n;
    const f4 *p;        // (x, y, z, unused) per point
    float r2;
    int32_t *counts;
    unsigned long long *total;
};

// Squared distance below r2, binary32 without fused multiply-add, fixed order.
__device__ __forceinline__ bool near3(f4 a, f4 b, float r2)
{
    const float dx = __fsub_rn(a.x, b.x), dy = __fsub_rn(a.y, b.y), dz = __fsub_rn(a.z, b.z);
    float s = __fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy));
    s = __fadd_rn(s, __fmul_rn(dz, dz));
    return s < r2;
}

// Tile (i, j, k) holds the points a = 2 + k rho + ta, b = 1 + j rho + tb and
// c = i rho + tc (strict triples; the non-strict domain has no offsets).
// The three neighbour relations between the tiles' points are formed once
// as bit masks (one wave ballot gives 64 / rho rows), so a pair (a, b) of
// neighbours finds all its triangles with one AND and a population count:
// rho^2 distance tests per relation instead of rho^3 per triple.
template <int TILE>
struct TriShape {
    static constexpr int NT = TILE == 8 ? 64 : 256;  // one wave holds the 64 pairs of rho = 8
};

template <int MAP, int TILE>
__global__ void __launch_bounds__((TriShape<TILE>::NT)) k_triangles(TriArgs p, int32_t strict)
{
    static_assert(TILE == 8 || TILE == 16 || TILE == 32 || TILE == 64, "mask width");
    constexpr int NT = TriShape<TILE>::NT;
    using M = typename std::conditional<TILE == 64, uint64_t, uint32_t>::type;  // a row of a relation
    int32_t ti, tj, tk;
    if (!tet_of_block<MAP>(p.g, ti, tj, tk)) return;

    __shared__ f4 pts[3][TILE];          // 0: a (tile k), 1: b (tile j), 2: c (tile i)
    __shared__ M mask[3][TILE];          // 0: a-b over b, 1: a-c over c, 2: b-c over c
    const int32_t n = p.n;
    const int32_t a0 = 2 * strict + tk * TILE, b0 = strict + tj * TILE, c0 = ti * TILE;
    const float nan = __builtin_nanf("");
    const int t = threadIdx.x;
    if (t < 3 * TILE) {
        const int s = t / TILE, q = t % TILE;
        const int32_t idx = (s == 0 ? a0 : (s == 1 ? b0 : c0)) + q;
        pts[s][q] = idx < n ? p.p[idx] : f4{nan, nan, nan, nan};
    }
    __syncthreads();

    // masks: relation s pairs rows of set r(s) with columns of set c(s); a
    // lane keeps its column point in registers through a relation's rows
    constexpr int RPB = 64 / TILE;     // rows per ballot
    constexpr int BPR = TILE / RPB;    // ballots per relation
    constexpr int NW = NT / 64;        // waves
    const int w = t >> 6, l = t & 63;
    const int col = l % TILE;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int rs = s == 2 ? 1 : 0, cs = s == 0 ? 1 : 2;
        const f4 pc = pts[cs][col];
        for (int k = w; k < BPR; k += NW) {
            const int row = k * RPB + l / TILE;
            const bool hit = near3(pts[rs][row], pc, p.r2);
            const uint64_t bal = __ballot(hit);
            if (l % TILE == 0) {
                if constexpr (TILE == 64)
                    mask[s][row] = bal;
                else
                    mask[s][row] = (M)((bal >> (l - l % TILE)) & ((1ull << TILE) - 1ull));
            }
        }
    }
    __syncthreads();

    // pairs (a, b): TILE^2 of them, over the NT threads
    const bool same_kj = (tk == tj), same_ji = (tj == ti);
    for (int q = t; q < TILE * TILE; q += NT) {
        const int ta = q / TILE, tb = q % TILE;
        // a > b: always across tiles, within one tile index iff ta >= tb
        // (a = tb + 2 + ..., b = tb + 1 + ... on the shifted tetrahedron)
        if (same_kj && ta < tb) continue;
        if (!((mask[0][ta] >> tb) & 1u)) continue;
        M m = mask[1][ta] & mask[2][tb];
        if (same_ji) m &= (tb == TILE - 1) ? ~(M)0 : (((M)2 << tb) - 1);  // c <= b in the tile
        if (!m) continue;
        const int c = __builtin_popcountll((uint64_t)m);
        atomicAdd(&p.counts[a0 + ta], c);
        atomicAdd(&p.counts[b0 + tb], c);
        atomicAdd(p.total, (unsigned long long)c);
        while (m) {
            const int tc = __builtin_ctzll((uint64_t)m);
            m &= m - 1;
            atomicAdd(&p.counts[c0 + tc], 1);
        }
    }
}

__global__ void __launch_bounds__(256) k_tri_clear(int32_t *v, int64_t count,
                                                   unsigned long long *total)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q < count) v[q] = 0;
    if (q == 0) *total = 0;
}

template <int MAP>
static bool triangles_tile(const tri_tet *p, const TriArgs &a, hipStream_t s)
{
    const dim3 grid(p->gx, p->gy, p->gz);
    const int32_t st = p->strict;
    switch (p->tile) {
    case 8: k_triangles<MAP, 8><<<grid, TriShape<8>::NT, 0, s>>>(a, st); return true;
    case 16: k_triangles<MAP, 16><<<grid, TriShape<16>::NT, 0, s>>>(a, st); return true;
    case 32: k_triangles<MAP, 32><<<grid, TriShape<32>::NT, 0, s>>>(a, st); return true;
    case 64: k_triangles<MAP, 64><<<grid, TriShape<64>::NT, 0, s>>>(a, st); return true;
    }
    return false;
}

// ---------------------------------------------------------------------------
// dummy kernel (the map alone)
// ---------------------------------------------------------------------------
template <int MAP, int TILE>
__global__ void __launch_bounds__(256) k_tet_dummy(TetGrid g, int32_t n, int32_t strict,
                                                   int32_t target, int32_t *sink)
{
    constexpr int CELLS = TILE * TILE * TILE;
    int32_t ti, tj, tk;
    if (!tet_of_block<MAP>(g, ti, tj, tk)) return;
    for (int q = threadIdx.x; q < CELLS; q += 256) {
        const int32_t c = ti * TILE + q % TILE;
        const int32_t b = strict + tj * TILE + (q / TILE) % TILE;
        const int32_t a = 2 * strict + tk * TILE + q / (TILE * TILE);
        // in the domain: a < n and a >= b >= c shifted
        if (a < n && b - strict <= a - 2 * strict && c <= b - strict &&
            (int64_t)a + b + c == target)
            sink[0] = a + b + c;
    }
}

}  // namespace trimap

using namespace trimap;

extern "C" {

tri_status tri_tet_plan(tri_tet **out, int64_t n, int tile, int map, int strict, uint32_t flags)
{
    clear_error();
    if (!out) return fail(TRI_E_INVAL, "tri_tet_plan: out is NULL");
    *out = nullptr;
    if (n < 0) return fail(TRI_E_INVAL, "tri_tet_plan: n = %lld < 0", (long long)n);
    if (n >= (1ll << 21)) return fail(TRI_E_RANGE, "tri_tet_plan: n = %lld >= 2^21", (long long)n);
    if (tile != 8 && tile != 16 && tile != 32 && tile != 64)
        return fail(TRI_E_INVAL, "tri_tet_plan: tile = %d not in {8,16,32,64}", tile);
    if (map != TRI_MAP_BB && map != TRI_MAP_LAMBDA)
        return fail(TRI_E_UNSUPPORTED, "tri_tet_plan: map = %d (BB or lambda)", map);
    if (strict != 0 && strict != 1) return fail(TRI_E_INVAL, "tri_tet_plan: strict = %d", strict);
    if (flags & ~(uint32_t)TRI_FLAG_SQRT_F64)
        return fail(TRI_E_INVAL, "tri_tet_plan: unknown flags 0x%x", flags);
    tri_tet p{};
    p.n = n;
    p.strict = strict;
    p.ne = strict ? (n > 2 ? n - 2 : 0) : n;
    p.tile = tile;
    p.map = map;
    p.flags = flags;
    p.m = (p.ne + tile - 1) / tile;
    const uint64_t m = (uint64_t)p.m;
    p.T = m * (m + 1) / 2 * (m + 2) / 3;
    const uint64_t ne = (uint64_t)p.ne;
    p.cells = ne * (ne + 1) / 2 * (ne + 2) / 3;
    if (map == TRI_MAP_BB) {
        if (m > 65535) return fail(TRI_E_RANGE, "tri_tet_plan: BB grid side %llu > 65535",
                                   (unsigned long long)m);
        p.gx = p.gy = p.gz = (uint32_t)(m ? m : 0);
        p.blocks = (int64_t)(m * m * m);
    } else {
        if (p.T <= (1ull << 24)) {
            p.gx = (uint32_t)p.T;
            p.gy = 1;
        } else {
            p.gx = 1u << 16;
            const uint64_t y = (p.T + p.gx - 1) / p.gx;
            if (y > kMaxGridY) return fail(TRI_E_RANGE, "tri_tet_plan: %llu tiles exceed the grid",
                                           (unsigned long long)p.T);
            p.gy = (uint32_t)y;
        }
        p.gz = 1;
        p.blocks = (int64_t)p.gx * p.gy;
        if (p.T == 0) {
            p.gx = p.gy = p.gz = 0;
            p.blocks = 0;
        }
    }
    tri_tet *h = new (std::nothrow) tri_tet(p);
    if (!h) return fail(TRI_E_NOMEM, "tri_tet_plan: out of host memory");
    *out = h;
    return TRI_OK;
}

tri_status tri_tet_destroy(tri_tet *p)
{
    clear_error();
    delete p;
    return TRI_OK;
}

tri_status tri_tet_query(const tri_tet *p, int64_t *tiles, int64_t *grid_blocks, int64_t *cells)
{
    clear_error();
    if (!p) return fail(TRI_E_INVAL, "tri_tet_query: plan is NULL");
    if (tiles) *tiles = (int64_t)p->T;
    if (grid_blocks) *grid_blocks = p->blocks;
    if (cells) *cells = (int64_t)p->cells;
    return TRI_OK;
}

tri_status tri_tet_dump(const tri_tet *p, int64_t *dev_out, void *stream)
{
    clear_error();
    if (!p || !dev_out) return fail(TRI_E_INVAL, "tri_tet_dump: NULL argument");
    if (p->blocks == 0) return TRI_OK;
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid(p->gx, p->gy, p->gz);
    if (p->map == TRI_MAP_BB) k_tet_dump<MAP_BB><<<grid, 64, 0, s>>>(tet_grid(p), dev_out);
    else k_tet_dump<MAP_LAMBDA><<<grid, 64, 0, s>>>(tet_grid(p), dev_out);
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}

tri_status tri_lambda3_eval(const uint64_t *dev_omega, int64_t count, uint32_t flags,
                            int64_t *dev_out, void *stream)
{
    clear_error();
    if (count < 0 || (count && (!dev_omega || !dev_out)))
        return fail(TRI_E_INVAL, "tri_lambda3_eval: bad arguments");
    if (flags & ~(uint32_t)TRI_FLAG_SQRT_F64)
        return fail(TRI_E_INVAL, "tri_lambda3_eval: unknown flags 0x%x", flags);
    if (count == 0) return TRI_OK;
    const int64_t blocks = (count + 255) / 256;
    if (blocks > (int64_t)kMaxWorkItems / 256) return fail(TRI_E_RANGE, "tri_lambda3_eval: count");
    k_lambda3_eval<<<dim3((uint32_t)blocks), 256, 0, (hipStream_t)stream>>>(dev_omega, count, flags,
                                                                            dev_out);
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}

tri_status tri_triangles(const tri_tet *p, const float *points, float r2, int32_t *counts,
                         unsigned long long *total, void *stream)
{
    clear_error();
    if (!p) return fail(TRI_E_INVAL, "tri_triangles: plan is NULL");
    if (!p->strict) return fail(TRI_E_INVAL, "tri_triangles: the plan must be strict");
    if (p->n == 0) return TRI_OK;
    if (!points || !counts || !total) return fail(TRI_E_INVAL, "tri_triangles: NULL buffer");
    if (((uintptr_t)points & 15) || ((uintptr_t)counts & 3) || ((uintptr_t)total & 7))
        return fail(TRI_E_INVAL, "tri_triangles: misaligned buffer");
    hipStream_t s = (hipStream_t)stream;
    k_tri_clear<<<dim3((uint32_t)((p->n + 255) / 256)), 256, 0, s>>>(counts, p->n, total);
    TRI_HIP(hipGetLastError());
    if (p->blocks == 0) return TRI_OK;
    TriArgs a{tet_grid(p), (int32_t)p->n, (const f4 *)points, r2, counts, total};
    const bool ok = p->map == TRI_MAP_BB ? triangles_tile<MAP_BB>(p, a, s)
                                         : triangles_tile<MAP_LAMBDA>(p, a, s);
    if (!ok) return fail(TRI_E_UNSUPPORTED, "tri_triangles: tile %d", p->tile);
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}

tri_status tri_tet_dummy(const tri_tet *p, int32_t target, int32_t *sink, void *stream)
{
    clear_error();
    if (!p) return fail(TRI_E_INVAL, "tri_tet_dummy: plan is NULL");
    if (!sink || ((uintptr_t)sink & 3)) return fail(TRI_E_INVAL, "tri_tet_dummy: sink");
    if (p->blocks == 0) return TRI_OK;
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid(p->gx, p->gy, p->gz);
    const TetGrid g = tet_grid(p);
    const int32_t n = (int32_t)p->n, st = p->strict;
#define TET_DUMMY(MAP, T) k_tet_dummy<MAP, T><<<grid, 256, 0, s>>>(g, n, st, target, sink)
    if (p->map == TRI_MAP_BB) {
        if (p->tile == 8) TET_DUMMY(MAP_BB, 8);
        else if (p->tile == 16) TET_DUMMY(MAP_BB, 16);
        else if (p->tile == 32) TET_DUMMY(MAP_BB, 32);
        else TET_DUMMY(MAP_BB, 64);
    } else {
        if (p->tile == 8) TET_DUMMY(MAP_LAMBDA, 8);
        else if (p->tile == 16) TET_DUMMY(MAP_LAMBDA, 16);
        else if (p->tile == 32) TET_DUMMY(MAP_LAMBDA, 32);
        else TET_DUMMY(MAP_LAMBDA, 64);
    }
#undef TET_DUMMY
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}

}  // extern "C"
