// Collision detection of n spheres (the shared-memory test of Section 5):
// every pair j < i of the strict lower triangle is tested once and, when the
// spheres overlap, counted for both of them.
//
// Tile maps (BB, RB, REC, lambda): tile (bi, bj) of the strict plan covers
// spheres 1 + bi rho .. (rows) against bj rho .. (columns).  Both blocks of
// spheres are staged in LDS (the shared-memory pattern the test is about);
// each lane keeps RB row spheres in registers and walks CB column spheres
// read from LDS (16 consecutive lanes read 16 consecutive spheres, lanes of
// other rows the same ones: broadcast).  Rows past n are staged as NaN so
// that they never overlap; only diagonal tiles test j < i per pair.
//
// UTM works in thread space: one lane per pair, both spheres read from
// global memory, no LDS (the map cannot form 2-D blocks).
//
// Overlaps are rare (a few per sphere), so a hit goes straight to two
// global atomic increments; the pair test itself bounds the kernel:
// 11 vector ALU operations per pair in 3-D, 5 in 1-D (plus one scalar OR).
#include "common.hpp"
#include "maps.hpp"

namespace trimap {

TileGrid plan_tile_grid(const tri_plan *p);

typedef float f4 __attribute__((ext_vector_type(4)));

struct CollideArgs {
    TileGrid g;
    int32_t n;
    const f4 *s;       // (x, y, z, r) per sphere
    int32_t *counts;
};

// Squared centre distance below the squared radius sum, binary32 with a
// fixed order (no fused multiply-add), strict comparison.
template <int DIM>
__device__ __forceinline__ bool overlap(f4 a, f4 b)
{
    const float dx = __fsub_rn(a.x, b.x);
    float s = __fmul_rn(dx, dx);
    if constexpr (DIM == 3) {
        const float dy = __fsub_rn(a.y, b.y), dz = __fsub_rn(a.z, b.z);
        s = __fadd_rn(s, __fmul_rn(dy, dy));
        s = __fadd_rn(s, __fmul_rn(dz, dz));
    }
    const float rr = __fadd_rn(a.w, b.w);
    return s < __fmul_rn(rr, rr);
}

template <int TILE>
struct CollideShape {
    static constexpr int NT = TILE * TILE < 256 ? TILE * TILE : 256;
    static constexpr int TX = TILE < 16 ? TILE : 16;  // lanes along columns
    static constexpr int TY = NT / TX;                // lanes along rows
    static constexpr int RB = TILE / TY;              // rows per lane
    static constexpr int CB = TILE / TX;              // columns per lane
    static_assert(RB * TY == TILE && CB * TX == TILE, "collide tile");
};

template <int MAP, int TILE, int DIM>
__global__ void __launch_bounds__((CollideShape<TILE>::NT)) k_collide(CollideArgs p)
{
    using S = CollideShape<TILE>;
    int32_t bi, bj;
    if (!tile_of_block<MAP>(p.g, bi, bj)) return;

    __shared__ f4 rows[TILE];
    __shared__ f4 cols[TILE];
    const int32_t n = p.n;
    const int32_t i0 = 1 + bi * TILE, j0 = bj * TILE;
    const float nan = __builtin_nanf("");
    for (int t = threadIdx.x; t < 2 * TILE; t += S::NT) {
        const int32_t k = t < TILE ? i0 + t : j0 + (t - TILE);
        const f4 v = k < n ? p.s[k] : f4{nan, nan, nan, nan};
        if (t < TILE) rows[t] = v;
        else cols[t - TILE] = v;
    }
    __syncthreads();

    const int ty = threadIdx.x / S::TX, tx = threadIdx.x % S::TX;
    f4 ri[S::RB];
#pragma unroll
    for (int a = 0; a < S::RB; ++a) ri[a] = rows[ty + S::TY * a];
    // First pass: only whether any pair of this lane overlaps (one lane-mask
    // OR per pair); overlaps are rare, so the second pass, which recounts
    // them with the diagonal test and the atomics, seldom runs.
    bool any = false;
#pragma unroll
    for (int b = 0; b < S::CB; ++b) {
        const f4 cj = cols[tx + S::TX * b];
#pragma unroll
        for (int a = 0; a < S::RB; ++a) any |= overlap<DIM>(ri[a], cj);
    }
    if (!any) return;
    const bool diag = (bi == bj);
#pragma unroll
    for (int b = 0; b < S::CB; ++b) {
        const int c = tx + S::TX * b;
        const f4 cj = cols[c];
#pragma unroll
        for (int a = 0; a < S::RB; ++a) {
            const int r = ty + S::TY * a;
            // j = j0 + c < i = 1 + j0 + r on a diagonal tile iff c <= r
            if (overlap<DIM>(ri[a], cj) && (!diag || c <= r)) {
                atomicAdd(&p.counts[i0 + r], 1);
                atomicAdd(&p.counts[j0 + c], 1);
            }
        }
    }
}

template <int DIM>
__global__ void __launch_bounds__(kUtmThreads) k_collide_utm(CollideArgs p, int64_t side,
                                                             int64_t pairs)
{
    const uint64_t k = ((uint64_t)blockIdx.y * gridDim.x + blockIdx.x) * kUtmThreads + threadIdx.x;
    if (k >= (uint64_t)pairs) return;
    int32_t i, j;
    utm_cell(k, side, i, j);
    i += 1;  // strict triangle of side n = diagonal-including triangle of side n - 1, shifted
    if ((uint32_t)i >= (uint32_t)p.n || (uint32_t)j >= (uint32_t)i) return;
    if (overlap<DIM>(p.s[i], p.s[j])) {
        atomicAdd(&p.counts[i], 1);
        atomicAdd(&p.counts[j], 1);
    }
}

__global__ void __launch_bounds__(256) k_zero_i32(int32_t *v, int64_t count)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < count) v[k] = 0;
}

template <int MAP, int DIM>
static bool collide_tile(const tri_plan *p, const CollideArgs &a, hipStream_t s)
{
    const dim3 grid(p->gx, p->gy);
    switch (p->tile) {
    case 8: k_collide<MAP, 8, DIM><<<grid, CollideShape<8>::NT, 0, s>>>(a); return true;
    case 16: k_collide<MAP, 16, DIM><<<grid, CollideShape<16>::NT, 0, s>>>(a); return true;
    case 32: k_collide<MAP, 32, DIM><<<grid, CollideShape<32>::NT, 0, s>>>(a); return true;
    case 64: k_collide<MAP, 64, DIM><<<grid, CollideShape<64>::NT, 0, s>>>(a); return true;
    case 128: k_collide<MAP, 128, DIM><<<grid, CollideShape<128>::NT, 0, s>>>(a); return true;
    }
    return false;
}

template <int DIM>
static bool collide_map(const tri_plan *p, const CollideArgs &a, hipStream_t s)
{
    switch (p->map) {
    case TRI_MAP_BB: return collide_tile<MAP_BB, DIM>(p, a, s);
    case TRI_MAP_RB: return collide_tile<MAP_RB, DIM>(p, a, s);
    case TRI_MAP_REC: return collide_tile<MAP_REC, DIM>(p, a, s);
    case TRI_MAP_LAMBDA: return collide_tile<MAP_LAMBDA, DIM>(p, a, s);
    case TRI_MAP_UTM:
        k_collide_utm<DIM><<<dim3(p->gx, p->gy), kUtmThreads, 0, s>>>(a, p->ne, p->elements);
        return true;
    }
    return false;
}

}  // namespace trimap

using namespace trimap;

extern "C" tri_status tri_collide(const tri_plan *p, const float *spheres, int dim,
                                  int32_t *counts, void *stream)
{
    clear_error();
    if (!p) return fail(TRI_E_INVAL, "tri_collide: plan is NULL");
    if (p->diag) return fail(TRI_E_INVAL, "tri_collide: the plan must exclude the diagonal");
    if (dim != 1 && dim != 3) return fail(TRI_E_INVAL, "tri_collide: dim = %d", dim);
    if (p->tile > 128) return fail(TRI_E_UNSUPPORTED, "tri_collide: tile %d > 128", p->tile);
    if (p->n == 0) return TRI_OK;
    if (!spheres || !counts) return fail(TRI_E_INVAL, "tri_collide: NULL buffer");
    if ((uintptr_t)spheres & 15)
        return fail(TRI_E_INVAL, "tri_collide: spheres need 16-byte alignment");
    if ((uintptr_t)counts & 3) return fail(TRI_E_INVAL, "tri_collide: unaligned counts");
    hipStream_t s = (hipStream_t)stream;
    k_zero_i32<<<dim3((uint32_t)((p->n + 255) / 256)), 256, 0, s>>>(counts, p->n);
    TRI_HIP(hipGetLastError());
    if (p->n < 2) return TRI_OK;
    CollideArgs a{plan_tile_grid(p), (int32_t)p->n, (const f4 *)spheres, counts};
    const bool ok = dim == 3 ? collide_map<3>(p, a, s) : collide_map<1>(p, a, s);
    if (!ok) return fail(TRI_E_UNSUPPORTED, "tri_collide: tile %d", p->tile);
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}
