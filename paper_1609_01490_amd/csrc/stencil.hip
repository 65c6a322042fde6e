// Game of Life (B3/S23) on the lower-triangular domain: the shared-memory
// neighbourhood case of the paper (Section 5, where lambda keeps the 2-D
// thread block and therefore the tile with its halo).
//
// One workgroup per rho x rho tile; the tile body (life_tile_body) stages the
// tile plus a one-cell halo in LDS as 32-bit words of four cells ((rho + 2)
// rows x (rho/4 + 2) words: the halo columns come in as whole words) and
// updates it with byte-sliced (SWAR) arithmetic, four cells per 32-bit
// operation.  Cells outside the domain (j > i, outside the n x n square) are
// zeroed as they are loaded and never stored, so the upper triangle is never
// touched.
#include <mutex>
#include <vector>

#include "bodies.hpp"
#include "common.hpp"
#include "maps.hpp"

namespace trimap {

TileGrid plan_tile_grid(const tri_plan *p);

struct LifeArgs {
    TileGrid g;
    LifeTile t;
};

// threads per workgroup of the one-launch-per-step kernel
template <int TILE>
constexpr int life_threads() { return TILE == 8 ? 16 : (TILE == 64 ? 256 : 64); }

template <int MAP, int TILE>
__global__ void __launch_bounds__(life_threads<TILE>()) k_life(LifeArgs p)
{
    constexpr int NT = life_threads<TILE>();
    int32_t bi, bj;
    if (!tile_of_block<MAP>(p.g, bi, bj)) return;
    __shared__ uint32_t L[LifeShape<TILE, NT>::LDS_WORDS];
    life_tile_body<TILE, NT>(p.t, bi, bj, L);
}

// UTM (thread space): thread k owns the cell utm_cell(k) and reads its eight
// neighbours straight from global memory; there is no tile to stage a halo
// in, so this is the global-memory variant of the update.
__global__ void __launch_bounds__(kUtmThreads) k_life_utm(LifeArgs p)
{
    const LifeTile &t = p.t;
    const int64_t cells = (int64_t)t.n * (t.n + 1) / 2;
    const uint64_t k = ((uint64_t)blockIdx.y * gridDim.x + blockIdx.x) * kUtmThreads + threadIdx.x;
    if (k >= (uint64_t)cells) return;
    int32_t i, j;
    utm_cell(k, t.n, i, j);
    if ((uint32_t)i >= (uint32_t)t.n || (uint32_t)j > (uint32_t)i) return;
    int cnt = 0;
#pragma unroll
    for (int di = -1; di <= 1; ++di)
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj) {
            if (di == 0 && dj == 0) continue;
            const int32_t r = i + di, c = j + dj;
            if (r >= 0 && r < t.n && c >= 0 && c <= r) cnt += t.cur[(int64_t)r * t.ld + c];
        }
    const uint8_t alive = t.cur[(int64_t)i * t.ld + j];
    t.nxt[(int64_t)i * t.ld + j] = (uint8_t)(cnt == 3 || (alive && cnt == 2));
}

template <int MAP>
static bool life_tile(const tri_plan *p, const LifeArgs &a, hipStream_t s);

template <int MAP, int TILE>
__global__ void __launch_bounds__(256) k_life_multi(LifeArgs p, int gens)
{
    int32_t bi, bj;
    if (!tile_of_block<MAP>(p.g, bi, bj)) return;
    __shared__ uint32_t buf[2 * LifeMultiShape<TILE>::WORDS];
    life_multi_tile_body<TILE>(p.t, bi, bj, gens, buf);
}

// 64 x 64 tiles, bit-sliced, one wave per tile; VEC: 16-byte row loads and
// stores (ld a multiple of 16, 16-byte aligned grids) and up to KH
// (kLifeBitsStencilGen by default) generations, else up to kLifeMaxGen
template <int MAP, bool VEC, int KH = (VEC ? kLifeBitsStencilGen : kLifeMaxGen)>
__global__ void __launch_bounds__(64) k_life_bits(LifeArgs p, int gens)
{
    int32_t bi, bj;
    if (!tile_of_block<MAP>(p.g, bi, bj)) return;
    __shared__ __attribute__((aligned(16))) uint32_t buf[2 * LifeBitsShape<KH>::WORDS];
    life_bits_wave_body<VEC, KH>(p.t, bi, bj, gens, buf);
}

// Strips (plans with TRI_FLAG_STRIP): a workgroup of four waves walks G
// consecutive tiles of the map, wave w taking tiles w, w + 4, ... of the
// strip, each with its own LDS buffers (the wave body needs no workgroup
// barrier), so that one dispatch serves G tiles.  KH = 1: one generation
// with the 1-cell halo; else up to KH generations.
template <int MAP, int KH>
__global__ void __launch_bounds__(256) k_life_bits_strip(LifeArgs p, int gens, StripGrid sg)
{
    __shared__ __attribute__((aligned(16))) uint32_t buf[4][2 * LifeBitsShape<KH>::WORDS];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t first = strip_first<MAP>(p.g, sg);
    for (int k = w; k < sg.G; k += 4) {
        int32_t bi, bj;
        if (!strip_tile<MAP>(p.g, sg, first, k, bi, bj)) continue;
        bi = __builtin_amdgcn_readfirstlane(bi);
        bj = __builtin_amdgcn_readfirstlane(bj);
        life_bits_wave_body<true, KH>(p.t, bi, bj, gens, buf[w]);
    }
}

// Strips with TRI_FLAG_LIFE_WIDE: wave w takes tiles 2 j and 2 j + 1 of the
// strip (j = w, w + 4, ...) together, as one window two tiles wide, when
// they are neighbours in a tile row (each still located by the map on its
// own), and otherwise each in a window of its own whose second half is not
// written back (one body, so that the registers are those of the paired
// body alone).  KH = 1: one generation with the 1-cell halo; else up to
// KH = 16 generations.
template <int MAP, int KH>
__global__ void __launch_bounds__(256) k_life_bits_strip_wide(LifeArgs p, int gens, StripGrid sg)
{
    static_assert(KH == 1 || KH == LifeBits16Pair::K, "halo");
    constexpr int WW = KH == 1 ? LifeBits1Pair::WORDS : LifeBits16Pair::WORDS;
    __shared__ __attribute__((aligned(16))) uint32_t buf[4][WW];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t first = strip_first<MAP>(p.g, sg);
    for (int j = w; 2 * j < sg.G; j += 4) {
        int32_t ai = 0, aj = 0, ci = 0, cj = 0;
        const bool va = __builtin_amdgcn_readfirstlane(
            (int)strip_tile<MAP>(p.g, sg, first, 2 * j, ai, aj));
        const bool vc = __builtin_amdgcn_readfirstlane(
            (int)(2 * j + 1 < sg.G && strip_tile<MAP>(p.g, sg, first, 2 * j + 1, ci, cj)));
        ai = __builtin_amdgcn_readfirstlane(ai);
        aj = __builtin_amdgcn_readfirstlane(aj);
        ci = __builtin_amdgcn_readfirstlane(ci);
        cj = __builtin_amdgcn_readfirstlane(cj);
        // up to two windows: the pair, or each valid tile alone
        const bool pair = va && vc && ci == ai && cj == aj + 1;
        const int nw = pair ? 1 : (int)va + (int)vc;
        for (int u = 0; u < nw; ++u) {
            const bool first = u == 0 && va;
            const int32_t bi = first ? ai : ci, bj = first ? aj : cj;
            if constexpr (KH == 1) life_bits1_pair_body(p.t, bi, bj, pair, buf[w]);
            else life_bits16_pair_body(p.t, bi, bj, pair, gens, buf[w]);
        }
    }
}

// One generation of 64 x 64 tiles with the 1-cell halo of the paper's tiles,
// bit-sliced, one wave per tile, 16-byte row moves
template <int MAP>
__global__ void __launch_bounds__(64) k_life_bits1(LifeArgs p)
{
    int32_t bi, bj;
    if (!tile_of_block<MAP>(p.g, bi, bj)) return;
    __shared__ __attribute__((aligned(16))) uint32_t buf[2 * LifeBitsShape<1>::WORDS];
    life_bits_wave_body<true, 1>(p.t, bi, bj, 1, buf);
}

// whether the bit-sliced kernel may move rows as 16-byte vectors
static bool life_vec16(const LifeTile &t)
{
    return t.ld % 16 == 0 && (((uintptr_t)t.cur | (uintptr_t)t.nxt) & 15) == 0;
}

// strip walk and launch grid of a plan's strip kernels
static StripGrid life_strip_grid(const tri_plan *p, const TileGrid &g, dim3 &grid)
{
    return strip_grid(p->map, g.m, g.flags, g.T, p->gx, p->gy, strip_flag_len(p->flags), 1, grid);
}

// strips take the bit-sliced kernels only (tile 64, 16-byte rows)
static bool life_strips(const tri_plan *p, const LifeTile &t)
{
    return p->map != TRI_MAP_UTM && p->tile == 64 && strip_flag_len(p->flags) && life_vec16(t);
}

// One generation of a plan's tiles (64 x 64 tiles with 16-byte rows:
// bit-sliced)
template <int MAP>
static bool life_tile(const tri_plan *p, const LifeArgs &a, hipStream_t s)
{
    const dim3 grid(p->gx, p->gy);
    switch (p->tile) {
    case 8: k_life<MAP, 8><<<grid, life_threads<8>(), 0, s>>>(a); return true;
    case 16: k_life<MAP, 16><<<grid, life_threads<16>(), 0, s>>>(a); return true;
    case 32: k_life<MAP, 32><<<grid, life_threads<32>(), 0, s>>>(a); return true;
    case 64:
        if (life_vec16(a.t) && strip_flag_len(p->flags)) {
            dim3 sgrid;
            const StripGrid sg = life_strip_grid(p, a.g, sgrid);
            if (p->flags & TRI_FLAG_LIFE_WIDE)
                k_life_bits_strip_wide<MAP, 1><<<sgrid, 256, 0, s>>>(a, 1, sg);
            else
                k_life_bits_strip<MAP, 1><<<sgrid, 256, 0, s>>>(a, 1, sg);
        } else if (life_vec16(a.t)) {
            k_life_bits1<MAP><<<grid, 64, 0, s>>>(a);
        } else {
            k_life<MAP, 64><<<grid, life_threads<64>(), 0, s>>>(a);
        }
        return true;
    }
    return false;
}

// 64 x 64 tiles take the bit-sliced one-wave kernel on grids of at least
// this many tiles, the byte-sliced 256-thread one below (measured, 20
// generations: with 16-byte rows the bit-sliced kernel wins from n = 2048,
// 0.055 vs 0.061 ms, to n = 8192, 0.151 vs 0.332 ms, and ties at n = 1024;
// moving rows byte by byte it wins only at n = 16384)
constexpr uint64_t kLifeBitsMinTiles = 16384;
constexpr uint64_t kLifeBitsMinTilesVec = 512;

template <int MAP>
static bool life_multi_kernel_tile(int tile, uint64_t tiles, bool vec, const void *&fn,
                                   int &threads, int &maxgen)
{
    threads = 256;
    maxgen = kLifeMaxGen;
    switch (tile) {
    case 16: fn = (const void *)k_life_multi<MAP, 16>; return true;
    case 32: fn = (const void *)k_life_multi<MAP, 32>; return true;
    case 64:
        if (tiles >= (vec ? kLifeBitsMinTilesVec : kLifeBitsMinTiles)) {
            fn = vec ? (const void *)k_life_bits<MAP, true> : (const void *)k_life_bits<MAP, false>;
            threads = 64;
            if (vec) maxgen = kLifeBitsStencilGen;
        } else {
            fn = (const void *)k_life_multi<MAP, 64>;
        }
        return true;
    }
    return false;
}

template <int MAP>
static const void *life_strip_kernel(int kh, bool wide)
{
    if (wide)
        return kh == 1 ? (const void *)k_life_bits_strip_wide<MAP, 1>
                       : (const void *)k_life_bits_strip_wide<MAP, kLifeBitsStencilGen>;
    return kh == 1 ? (const void *)k_life_bits_strip<MAP, 1>
                   : (const void *)k_life_bits_strip<MAP, kLifeBitsStencilGen>;
}

// the strip kernel of a plan (kh = 1: one generation; else the temporal one)
static const void *life_strip_fn(const tri_plan *p, int kh)
{
    const bool wide = (p->flags & TRI_FLAG_LIFE_WIDE) != 0;
    switch (p->map) {
    case TRI_MAP_BB: return life_strip_kernel<MAP_BB>(kh, wide);
    case TRI_MAP_RB: return life_strip_kernel<MAP_RB>(kh, wide);
    case TRI_MAP_REC: return life_strip_kernel<MAP_REC>(kh, wide);
    case TRI_MAP_LAMBDA: return life_strip_kernel<MAP_LAMBDA>(kh, wide);
    }
    return nullptr;
}

static bool life_multi_kernel(const tri_plan *p, bool vec, const void *&fn, int &threads,
                              int &maxgen)
{
    const uint64_t T = (uint64_t)p->T;
    switch (p->map) {
    case TRI_MAP_BB: return life_multi_kernel_tile<MAP_BB>(p->tile, T, vec, fn, threads, maxgen);
    case TRI_MAP_RB: return life_multi_kernel_tile<MAP_RB>(p->tile, T, vec, fn, threads, maxgen);
    case TRI_MAP_REC: return life_multi_kernel_tile<MAP_REC>(p->tile, T, vec, fn, threads, maxgen);
    case TRI_MAP_LAMBDA:
        return life_multi_kernel_tile<MAP_LAMBDA>(p->tile, T, vec, fn, threads, maxgen);
    }
    return false;
}

// Generations of each launch for `steps` generations, at most maxgen each,
// with as many launches as the parity of steps allows (the result lands in
// cur for even steps, in nxt for odd).
std::vector<int> life_multi_schedule(int steps, int maxgen)
{
    int L = (steps + maxgen - 1) / maxgen;
    if ((L & 1) != (steps & 1)) ++L;
    std::vector<int> g(L, steps / L);
    for (int k = 0; k < steps % L; ++k) ++g[k];
    return g;
}

// One temporal-blocking launch of one domain under lambda (batched
// per-instance mode); false for an unsupported tile.
bool launch_life_multi_lambda(int tile, const TileGrid &g, const LifeTile &t, int gens,
                              hipStream_t s)
{
    LifeArgs a{g, t};
    uint32_t gx, gy;
    if (g.T <= (1ull << 24)) { gx = (uint32_t)g.T; gy = 1; }
    else { gx = 1u << 16; gy = (uint32_t)((g.T + gx - 1) / gx); }
    const dim3 grid(gx, gy);
    if (gens > kLifeMaxGen && tile != 64) return false;
    if (gens > kLifeBitsStencilGen) return false;
    switch (tile) {
    case 16: k_life_multi<MAP_LAMBDA, 16><<<grid, 256, 0, s>>>(a, gens); return true;
    case 32: k_life_multi<MAP_LAMBDA, 32><<<grid, 256, 0, s>>>(a, gens); return true;
    case 64:
        // the bit-sliced kernel with 16-byte rows: the shallower halo where
        // it suffices (the batch's launches advance up to kLifeBitsMaxGen)
        if (gens > kLifeMaxGen) {  // only the bit-sliced kernel with 16-byte rows goes beyond 4
            if (!life_vec16(t)) return false;
            if (gens <= kLifeBitsMaxGen)
                k_life_bits<MAP_LAMBDA, true, kLifeBitsMaxGen><<<grid, 64, 0, s>>>(a, gens);
            else
                k_life_bits<MAP_LAMBDA, true><<<grid, 64, 0, s>>>(a, gens);
        } else if (life_vec16(t) && g.T >= kLifeBitsMinTilesVec)
            k_life_bits<MAP_LAMBDA, true, kLifeBitsMaxGen><<<grid, 64, 0, s>>>(a, gens);
        else if (!life_vec16(t) && g.T >= kLifeBitsMinTiles)
            k_life_bits<MAP_LAMBDA, false><<<grid, 64, 0, s>>>(a, gens);
        else k_life_multi<MAP_LAMBDA, 64><<<grid, 256, 0, s>>>(a, gens);
        return true;
    }
    return false;
}

// kernel address and block size of the one-step kernel of a plan
template <int MAP>
static bool life_kernel_tile(int tile, bool vec, const void *&fn, int &threads)
{
    switch (tile) {
    case 8: fn = (const void *)k_life<MAP, 8>; threads = life_threads<8>(); return true;
    case 16: fn = (const void *)k_life<MAP, 16>; threads = life_threads<16>(); return true;
    case 32: fn = (const void *)k_life<MAP, 32>; threads = life_threads<32>(); return true;
    case 64:
        if (vec) { fn = (const void *)k_life_bits1<MAP>; threads = 64; }
        else { fn = (const void *)k_life<MAP, 64>; threads = life_threads<64>(); }
        return true;
    }
    return false;
}

static bool life_kernel(const tri_plan *p, bool vec, const void *&fn, int &threads)
{
    switch (p->map) {
    case TRI_MAP_UTM: fn = (const void *)k_life_utm; threads = kUtmThreads; return true;
    case TRI_MAP_BB: return life_kernel_tile<MAP_BB>(p->tile, vec, fn, threads);
    case TRI_MAP_RB: return life_kernel_tile<MAP_RB>(p->tile, vec, fn, threads);
    case TRI_MAP_REC: return life_kernel_tile<MAP_REC>(p->tile, vec, fn, threads);
    case TRI_MAP_LAMBDA: return life_kernel_tile<MAP_LAMBDA>(p->tile, vec, fn, threads);
    }
    return false;
}

static bool life_step(const tri_plan *p, const LifeArgs &a, hipStream_t s)
{
    switch (p->map) {
    case TRI_MAP_UTM:
        k_life_utm<<<dim3(p->gx, p->gy), kUtmThreads, 0, s>>>(a);
        return true;
    case TRI_MAP_BB: return life_tile<MAP_BB>(p, a, s);
    case TRI_MAP_RB: return life_tile<MAP_RB>(p, a, s);
    case TRI_MAP_REC: return life_tile<MAP_REC>(p, a, s);
    case TRI_MAP_LAMBDA: return life_tile<MAP_LAMBDA>(p, a, s);
    }
    return false;
}

// One Life generation of one domain under lambda (batched per-instance
// mode); false for an unsupported tile.
bool launch_life_lambda(int tile, const TileGrid &g, const LifeTile &t, hipStream_t s)
{
    LifeArgs a{g, t};
    uint32_t gx, gy;
    if (g.T <= (1ull << 24)) { gx = (uint32_t)g.T; gy = 1; }
    else { gx = 1u << 16; gy = (uint32_t)((g.T + gx - 1) / gx); }
    const dim3 grid(gx, gy);
    switch (tile) {
    case 8: k_life<MAP_LAMBDA, 8><<<grid, life_threads<8>(), 0, s>>>(a); return true;
    case 16: k_life<MAP_LAMBDA, 16><<<grid, life_threads<16>(), 0, s>>>(a); return true;
    case 32: k_life<MAP_LAMBDA, 32><<<grid, life_threads<32>(), 0, s>>>(a); return true;
    case 64:
        if (life_vec16(t)) k_life_bits1<MAP_LAMBDA><<<grid, 64, 0, s>>>(a);
        else k_life<MAP_LAMBDA, 64><<<grid, life_threads<64>(), 0, s>>>(a);
        return true;
    }
    return false;
}

// The generations of one (plan, buffers, steps) as an instantiated graph of
// kernel nodes, built on first use and kept with the plan until
// tri_plan_destroy.
static tri_status life_graph(const tri_plan *p, const LifeArgs &a0, int steps,
                             hipGraphExec_t &exec)
{
    const PlanGraphKey key{(const void *)a0.t.cur, (const void *)a0.t.nxt, a0.t.ld, steps};
    std::lock_guard<std::mutex> lk(p->graphs->mu);
    auto it = p->graphs->execs.find(key);
    if (it != p->graphs->execs.end()) {
        exec = it->second;
        return TRI_OK;
    }
    const void *fn = nullptr;
    int threads = 0;
    if (!life_kernel(p, life_vec16(a0.t), fn, threads))
        return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: tile");
    dim3 grid(p->gx, p->gy);
    StripGrid sg{};
    int one = 1;
    const bool strips = life_strips(p, a0.t);
    if (strips) {
        fn = life_strip_fn(p, 1);
        threads = 256;
        sg = life_strip_grid(p, a0.g, grid);
    }
    hipGraph_t g = nullptr;
    TRI_HIP(hipGraphCreate(&g, 0));
    hipGraphNode_t prev = nullptr;
    hipError_t e = hipSuccess;
    for (int k = 0; k < steps && e == hipSuccess; ++k) {
        LifeArgs a = a0;
        a.t.cur = (k & 1) ? a0.t.nxt : a0.t.cur;
        a.t.nxt = (k & 1) ? (uint8_t *)a0.t.cur : a0.t.nxt;
        void *args1[] = {&a};
        void *args3[] = {&a, &one, &sg};
        hipKernelNodeParams np{};
        np.func = (void *)fn;
        np.gridDim = grid;
        np.blockDim = dim3(threads);
        np.sharedMemBytes = 0;
        np.kernelParams = strips ? args3 : args1;
        np.extra = nullptr;
        hipGraphNode_t node;
        e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &np);
        prev = node;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "tri_launch_stencil: graph");
    p->graphs->execs[key] = exec;
    return TRI_OK;
}

}  // namespace trimap

using namespace trimap;

extern "C" tri_status tri_launch_stencil(const tri_plan *p, uint8_t *cur, uint8_t *nxt,
                                         int64_t ld, int steps, int use_graph, void *stream)
{
    clear_error();
    if (!p) return fail(TRI_E_INVAL, "tri_launch_stencil: plan is NULL");
    if (!p->diag) return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: needs include_diag = 1");
    if (p->map != TRI_MAP_UTM && p->tile > 64)
        return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: tile %d > 64", p->tile);
    if (p->map == TRI_MAP_UTM && (p->flags & TRI_FLAG_LIFE_TEMPORAL))
        return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: UTM has no tile for temporal blocking");
    if (p->flags & TRI_FLAG_STRIP_BAND)
        return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: two-row band strips are for the elementwise kernels");
        if (steps < 0) return fail(TRI_E_INVAL, "tri_launch_stencil: steps < 0");
    if (p->n == 0 || steps == 0) return TRI_OK;
    if (!cur || !nxt || cur == nxt) return fail(TRI_E_INVAL, "tri_launch_stencil: bad buffers");
    if (ld < p->n || ld % 4) return fail(TRI_E_INVAL, "tri_launch_stencil: ld must be >= n and a multiple of 4");
    if (((uintptr_t)cur | (uintptr_t)nxt) & 3)
        return fail(TRI_E_INVAL, "tri_launch_stencil: buffers must be 4-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    LifeArgs a{plan_tile_grid(p), LifeTile{(int32_t)p->n, ld, cur, nxt}};
    if (p->flags & TRI_FLAG_LIFE_TEMPORAL) {
        if (use_graph)
            return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: graphs of the temporal kernel are not built");
        const void *fn = nullptr;
        int threads = 256, maxgen = kLifeMaxGen;
        if (!life_multi_kernel(p, life_vec16(a.t), fn, threads, maxgen))
            return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: temporal blocking needs tile 16, 32 or 64");
        dim3 grid(p->gx, p->gy);
        StripGrid sg{};
        const bool strips = life_strips(p, a.t);
        if (strips) {
            fn = life_strip_fn(p, kLifeBitsStencilGen);
            threads = 256;
            maxgen = kLifeBitsStencilGen;
            sg = life_strip_grid(p, a.g, grid);
        }
        const std::vector<int> sched = life_multi_schedule(steps, maxgen);
        for (size_t k = 0; k < sched.size(); ++k) {
            a.t.cur = (k & 1) ? nxt : cur;
            a.t.nxt = (k & 1) ? cur : nxt;
            int gens = sched[k];
            void *args[] = {&a, &gens, &sg};
            TRI_HIP(hipLaunchKernel(fn, grid, dim3(threads), args, 0, s));
        }
        return TRI_OK;
    }
    if (use_graph) {
        hipGraphExec_t exec = nullptr;
        tri_status st = life_graph(p, a, steps, exec);
        if (st != TRI_OK) return st;
        TRI_HIP(hipGraphLaunch(exec, s));
        return TRI_OK;
    }
    for (int k = 0; k < steps; ++k) {
        a.t.cur = (k & 1) ? nxt : cur;
        a.t.nxt = (k & 1) ? cur : nxt;
        if (!life_step(p, a, s)) return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: tile");
        TRI_HIP(hipGetLastError());
    }
    return TRI_OK;
}
