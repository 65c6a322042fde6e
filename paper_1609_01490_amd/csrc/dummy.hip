// The dummy kernel of the square-root study (Section 4.1): every cell (i, j)
// of the plan's domain forms its coordinates through the map and computes
// i + j; only cells whose sum equals a target store it.  With a target no
// cell reaches, nothing is written and the kernel costs the dispatch, the
// map and the per-cell test alone, which is what the paper's improvement
// factors compare (its version stores every sum to one fixed address; on
// this hardware those stores would serialise on one L2 channel and hide the
// map's cost).
#include "common.hpp"
#include "maps.hpp"

namespace trimap {

TileGrid plan_tile_grid(const tri_plan *p);

struct DummyArgs {
    TileGrid g;
    int32_t n;
    int32_t row_off;  // 1 for the strict triangle
    int32_t target;
    int32_t *sink;
};

template <int TILE>
struct DummyShape {
    static constexpr int NT = TILE * TILE < 256 ? TILE * TILE : 256;
    static constexpr int PASSES = TILE * TILE / NT;
};

template <int MAP, int TILE>
__global__ void __launch_bounds__((DummyShape<TILE>::NT)) k_dummy(DummyArgs p)
{
    using S = DummyShape<TILE>;
    int32_t bi, bj;
    if (!tile_of_block<MAP>(p.g, bi, bj)) return;
#pragma unroll
    for (int ps = 0; ps < S::PASSES; ++ps) {
        const int t = threadIdx.x + ps * S::NT;
        const int32_t i = p.row_off + bi * TILE + t / TILE;
        const int32_t j = bj * TILE + t % TILE;
        if (i < p.n && j < i + 1 - p.row_off && (int64_t)i + j == p.target) p.sink[0] = i + j;
    }
}

__global__ void __launch_bounds__(kUtmThreads) k_dummy_utm(DummyArgs p, int64_t side,
                                                           int64_t cells)
{
    const uint64_t k = ((uint64_t)blockIdx.y * gridDim.x + blockIdx.x) * kUtmThreads + threadIdx.x;
    if (k >= (uint64_t)cells) return;
    int32_t i, j;
    utm_cell(k, side, i, j);
    i += p.row_off;
    if (i < p.n && j < i + 1 - p.row_off && (int64_t)i + j == p.target) p.sink[0] = i + j;
}

// The lambda map of the square-root study in one 32-bit shape for every
// root (1-D grid of exactly T < 2^24 blocks), so that the variants differ
// only in how the root is taken: v_sqrt_f32 (lambda_X), x v_rsq_f32
// (lambda_R), bit trick + 3 Newton steps (lambda_N), FP64; each either with
// the exact one-step integer correction or, with EPS, as the paper's
// floor(sqrt(1/4 + 2 omega) + 1e-4 - 1/2) with no correction (wrong tiles
// are then dropped by the range check).
enum { ROOT_SQRT = 0, ROOT_RSQ = 1, ROOT_NEWTON = 2, ROOT_F64 = 3 };

template <int ROOT>
__device__ __forceinline__ float study_root(float x)
{
    if constexpr (ROOT == ROOT_RSQ) return x * __builtin_amdgcn_rsqf(x);
    else if constexpr (ROOT == ROOT_NEWTON) return sqrt_newton3(x);
    else return __builtin_amdgcn_sqrtf(x);
}

template <int ROOT, bool EPS>
__device__ __forceinline__ bool study_lambda(uint32_t w, int32_t m, int32_t &bi, int32_t &bj)
{
    uint32_t i;
    if constexpr (EPS) {
        const float r = study_root<ROOT>(0.25f + 2.0f * (float)w) + 1e-4f - 0.5f;
        i = r < 0.f ? 0u : (uint32_t)r;
        bi = (int32_t)i;
        bj = (int32_t)(w - i * (i + 1) / 2);
    } else {
        if constexpr (ROOT == ROOT_F64)
            i = (uint32_t)((__builtin_sqrt(8.0 * (double)w + 1.0) - 1.0) * 0.5);
        else
            i = (uint32_t)((study_root<ROOT>(__builtin_fmaf(8.0f, (float)w, 1.0f)) - 1.0f) * 0.5f);
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
    return (uint32_t)bi < (uint32_t)m && (uint32_t)bj <= (uint32_t)bi;
}

template <int TILE, int ROOT, bool EPS>
__global__ void __launch_bounds__((DummyShape<TILE>::NT)) k_dummy_study(DummyArgs p)
{
    using S = DummyShape<TILE>;
    uint32_t L = blockIdx.x;
    if (p.g.flags & TRI_FLAG_XCD_SWIZZLE) {
        const uint32_t x = L & 7, l = L >> 3, G = (uint32_t)p.g.T, q = G >> 3, r = G & 7;
        L = x * q + (x < r ? x : r) + l;
    }
    int32_t bi, bj;
    if (!study_lambda<ROOT, EPS>(L, p.g.m, bi, bj)) return;
#pragma unroll
    for (int ps = 0; ps < S::PASSES; ++ps) {
        const int t = threadIdx.x + ps * S::NT;
        const int32_t i = p.row_off + bi * TILE + t / TILE;
        const int32_t j = bj * TILE + t % TILE;
        if (i < p.n && j < i + 1 - p.row_off && (int64_t)i + j == p.target) p.sink[0] = i + j;
    }
}

template <int ROOT, bool EPS>
static bool dummy_study_tile(const tri_plan *p, const DummyArgs &a, hipStream_t s)
{
    const dim3 grid(p->gx);
    switch (p->tile) {
    case 8: k_dummy_study<8, ROOT, EPS><<<grid, DummyShape<8>::NT, 0, s>>>(a); return true;
    case 16: k_dummy_study<16, ROOT, EPS><<<grid, DummyShape<16>::NT, 0, s>>>(a); return true;
    case 32: k_dummy_study<32, ROOT, EPS><<<grid, DummyShape<32>::NT, 0, s>>>(a); return true;
    case 64: k_dummy_study<64, ROOT, EPS><<<grid, DummyShape<64>::NT, 0, s>>>(a); return true;
    }
    return false;
}

// The study shape applies to lambda plans launched as a 1-D grid of exactly
// T < 2^24 blocks whose flags select only a root, the epsilon form and the
// swizzle; false if the plan does not qualify.
static bool dummy_study(const tri_plan *p, const DummyArgs &a, hipStream_t s, bool &ok)
{
    const uint32_t f = p->flags;
    const uint32_t allowed = TRI_FLAG_XCD_SWIZZLE | TRI_FLAG_SQRT_RSQ | TRI_FLAG_SQRT_NEWTON |
                             TRI_FLAG_SQRT_F64 | TRI_FLAG_SQRT_EPS;
    if (p->map != TRI_MAP_LAMBDA || p->gy != 1 || (uint64_t)p->gx != (uint64_t)p->T ||
        p->T > (1ll << 24) || (f & ~allowed))
        return false;
    const bool eps = f & TRI_FLAG_SQRT_EPS;
    const int root = (f & TRI_FLAG_SQRT_RSQ)      ? ROOT_RSQ
                     : (f & TRI_FLAG_SQRT_NEWTON) ? ROOT_NEWTON
                     : (f & TRI_FLAG_SQRT_F64)    ? ROOT_F64
                                                  : ROOT_SQRT;
    if (eps && root == ROOT_F64) return false;  // not one of the paper's forms
    if (eps) {
        ok = root == ROOT_RSQ      ? dummy_study_tile<ROOT_RSQ, true>(p, a, s)
             : root == ROOT_NEWTON ? dummy_study_tile<ROOT_NEWTON, true>(p, a, s)
                                   : dummy_study_tile<ROOT_SQRT, true>(p, a, s);
    } else {
        ok = root == ROOT_RSQ      ? dummy_study_tile<ROOT_RSQ, false>(p, a, s)
             : root == ROOT_NEWTON ? dummy_study_tile<ROOT_NEWTON, false>(p, a, s)
             : root == ROOT_F64    ? dummy_study_tile<ROOT_F64, false>(p, a, s)
                                   : dummy_study_tile<ROOT_SQRT, false>(p, a, s);
    }
    return true;
}

template <int MAP>
static bool dummy_tile(const tri_plan *p, const DummyArgs &a, hipStream_t s)
{
    const dim3 grid(p->gx, p->gy);
    switch (p->tile) {
    case 8: k_dummy<MAP, 8><<<grid, DummyShape<8>::NT, 0, s>>>(a); return true;
    case 16: k_dummy<MAP, 16><<<grid, DummyShape<16>::NT, 0, s>>>(a); return true;
    case 32: k_dummy<MAP, 32><<<grid, DummyShape<32>::NT, 0, s>>>(a); return true;
    case 64: k_dummy<MAP, 64><<<grid, DummyShape<64>::NT, 0, s>>>(a); return true;
    }
    return false;
}

}  // namespace trimap

using namespace trimap;

extern "C" tri_status tri_launch_dummy(const tri_plan *p, int32_t target, int32_t *sink,
                                       void *stream)
{
    clear_error();
    if (!p) return fail(TRI_E_INVAL, "tri_launch_dummy: plan is NULL");
    if (p->tile > 64) return fail(TRI_E_UNSUPPORTED, "tri_launch_dummy: tile %d > 64", p->tile);
    if (!sink || ((uintptr_t)sink & 3)) return fail(TRI_E_INVAL, "tri_launch_dummy: sink");
    if (p->elements == 0) return TRI_OK;
    DummyArgs a{plan_tile_grid(p), (int32_t)p->n, p->row_off, target, sink};
    hipStream_t s = (hipStream_t)stream;
    bool ok = true;
    switch (p->map) {
    case TRI_MAP_BB: ok = dummy_tile<MAP_BB>(p, a, s); break;
    case TRI_MAP_RB: ok = dummy_tile<MAP_RB>(p, a, s); break;
    case TRI_MAP_REC: ok = dummy_tile<MAP_REC>(p, a, s); break;
    case TRI_MAP_LAMBDA:
        if (!dummy_study(p, a, s, ok)) ok = dummy_tile<MAP_LAMBDA>(p, a, s);
        break;
    case TRI_MAP_UTM:
        k_dummy_utm<<<dim3(p->gx, p->gy), kUtmThreads, 0, s>>>(a, p->ne, p->elements);
        break;
    }
    if (!ok) return fail(TRI_E_UNSUPPORTED, "tri_launch_dummy: tile %d", p->tile);
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}
