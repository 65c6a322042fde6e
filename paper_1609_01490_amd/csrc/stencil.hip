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

template <int MAP>
static bool life_tile(const tri_plan *p, const LifeArgs &a, hipStream_t s)
{
    const dim3 grid(p->gx, p->gy);
    switch (p->tile) {
    case 8: k_life<MAP, 8><<<grid, life_threads<8>(), 0, s>>>(a); return true;
    case 16: k_life<MAP, 16><<<grid, life_threads<16>(), 0, s>>>(a); return true;
    case 32: k_life<MAP, 32><<<grid, life_threads<32>(), 0, s>>>(a); return true;
    case 64: k_life<MAP, 64><<<grid, life_threads<64>(), 0, s>>>(a); return true;
    }
    return false;
}

// ---------------------------------------------------------------------------
// Temporal blocking (TRI_FLAG_LIFE_TEMPORAL): one launch advances up to
// kLifeMaxGen generations.  The workgroup stages its tile with a halo of
// kLifeMaxGen cells (rows) and one word (4 cells) on each side, runs the
// generations in LDS, and writes only the tile: after g generations every
// cell at least g cells inside the staged window is exact (the light cone of
// a cell grows by one per generation), so the tile is exact after up to four.
// Cells outside the domain are forced dead after every generation, as the
// rule requires.  HBM traffic per generation falls from one read and one
// write of the tile to (1 + halo) / g reads and 1 / g writes.
// ---------------------------------------------------------------------------
constexpr int kLifeMaxGen = 4;

template <int TILE>
struct LifeMultiShape {
    static constexpr int NT = 256;
    static constexpr int W = TILE / 4 + 2;        // words per staged row
    static constexpr int R = TILE + 2 * kLifeMaxGen;  // staged rows
    static constexpr int PW = W + 2;              // padded LDS row (zero border)
    static constexpr int PR = R + 2;
    static constexpr int STRIPS = NT / W;         // strips of rows per word column
    static constexpr int SH = (R + STRIPS - 1) / STRIPS;
    static constexpr int WORDS = PR * PW;
};

// domain mask of the staged word at row gi, column gj (4-aligned): bytes of
// cells 0 <= gj + b <= gi < n
__device__ __forceinline__ uint32_t life_window_mask(int32_t gi, int32_t gj, int32_t n)
{
    if (gi < 0 || gi >= n || gj < 0) return 0u;
    return life_domain_mask(gi, gj);
}

template <int MAP, int TILE>
__global__ void __launch_bounds__(256) k_life_multi(LifeArgs p, int gens)
{
    using S = LifeMultiShape<TILE>;
    int32_t bi, bj;
    if (!tile_of_block<MAP>(p.g, bi, bj)) return;
    __shared__ uint32_t buf[2][S::WORDS];
    const int32_t n = p.t.n;
    const int64_t ld = p.t.ld;
    const int32_t i0 = bi * TILE, j0 = bj * TILE;
    const int K = kLifeMaxGen;

    // stage rows i0-K .. i0+TILE+K-1, words at columns j0-4 .. j0+TILE, with
    // a zero border around the window
    for (int idx = threadIdx.x; idx < S::WORDS; idx += S::NT) {
        const int pr = idx / S::PW, pw = idx % S::PW;
        uint32_t v = 0;
        if (pr >= 1 && pr <= S::R && pw >= 1 && pw <= S::W) {
            const int32_t gi = i0 - K + (pr - 1);
            const int32_t gj = j0 - 4 + 4 * (pw - 1);
            const uint32_t m = life_window_mask(gi, gj, n);
            if (m) v = *(const uint32_t *)(p.t.cur + (int64_t)gi * ld + gj) & m;
        }
        buf[0][idx] = v;
        buf[1][idx] = 0;
    }
    __syncthreads();

    const int w = threadIdx.x % S::W;      // word column of this thread
    const int st = threadIdx.x / S::W;     // strip
    const bool active = st < S::STRIPS;
    const int r0 = st * S::SH;             // first staged row of the strip
    const int32_t gj = j0 - 4 + 4 * w;
    int cur = 0;
    for (int g = 0; g < gens; ++g) {
        const uint32_t *A = buf[cur];
        uint32_t *B = buf[cur ^ 1];
        if (active) {
            auto L = [A](int r, int c) { return A[(r + 1) * S::PW + (c + 1)]; };
            uint32_t hprev = life_hsum3(L(r0 - 1, w - 1), L(r0 - 1, w), L(r0 - 1, w + 1));
            uint32_t hcur = life_hsum3(L(r0, w - 1), L(r0, w), L(r0, w + 1));
            for (int k = 0; k < S::SH; ++k) {
                const int r = r0 + k;
                if (r >= S::R) break;
                const uint32_t hnext = life_hsum3(L(r + 1, w - 1), L(r + 1, w), L(r + 1, w + 1));
                const uint32_t self = L(r, w);
                const uint32_t s9 = hprev + hcur + hnext;
                uint32_t nv = life_zero_bytes(s9 ^ 0x03030303u) |
                              (life_zero_bytes(s9 ^ 0x04040404u) & self);
                nv &= life_window_mask(i0 - K + r, gj, n);  // dead outside the domain
                B[(r + 1) * S::PW + (w + 1)] = nv;
                hprev = hcur;
                hcur = hnext;
            }
        }
        __syncthreads();
        cur ^= 1;
    }

    // the tile: staged rows K .. K+TILE-1, words 1 .. TILE/4
    const uint32_t *A = buf[cur];
    for (int idx = threadIdx.x; idx < TILE * (TILE / 4); idx += S::NT) {
        const int tr = idx / (TILE / 4), tw = idx % (TILE / 4);
        const int32_t gi = i0 + tr, gjw = j0 + 4 * tw;
        const uint32_t v = A[(K + tr + 1) * S::PW + (tw + 1 + 1)];
        if (gi < n && gjw + 3 <= gi) {
            *(uint32_t *)(p.t.nxt + (int64_t)gi * ld + gjw) = v;
        } else if (gi < n && gjw <= gi) {  // the word holding the diagonal cell
            uint8_t *q = p.t.nxt + (int64_t)gi * ld + gjw;
            for (int b = 0; b <= gi - gjw; ++b) q[b] = (uint8_t)(v >> (8 * b));
        }
    }
}

template <int MAP>
static bool life_multi_kernel_tile(int tile, const void *&fn)
{
    switch (tile) {
    case 16: fn = (const void *)k_life_multi<MAP, 16>; return true;
    case 32: fn = (const void *)k_life_multi<MAP, 32>; return true;
    case 64: fn = (const void *)k_life_multi<MAP, 64>; return true;
    }
    return false;
}

static bool life_multi_kernel(const tri_plan *p, const void *&fn)
{
    switch (p->map) {
    case TRI_MAP_BB: return life_multi_kernel_tile<MAP_BB>(p->tile, fn);
    case TRI_MAP_RB: return life_multi_kernel_tile<MAP_RB>(p->tile, fn);
    case TRI_MAP_REC: return life_multi_kernel_tile<MAP_REC>(p->tile, fn);
    case TRI_MAP_LAMBDA: return life_multi_kernel_tile<MAP_LAMBDA>(p->tile, fn);
    }
    return false;
}

// Generations per launch for a run of `steps` generations, at most
// kLifeMaxGen each, with a number of launches of the same parity as steps
// (the result then lands in the buffer the one-step path would leave it in).
static std::vector<int> life_multi_schedule(int steps)
{
    int L = (steps + kLifeMaxGen - 1) / kLifeMaxGen;
    if ((L & 1) != (steps & 1)) ++L;
    std::vector<int> g(L, steps / L);
    for (int k = 0; k < steps % L; ++k) ++g[k];
    return g;
}

// kernel address and block size of the one-step kernel of a plan
template <int MAP>
static bool life_kernel_tile(int tile, const void *&fn, int &threads)
{
    switch (tile) {
    case 8: fn = (const void *)k_life<MAP, 8>; threads = life_threads<8>(); return true;
    case 16: fn = (const void *)k_life<MAP, 16>; threads = life_threads<16>(); return true;
    case 32: fn = (const void *)k_life<MAP, 32>; threads = life_threads<32>(); return true;
    case 64: fn = (const void *)k_life<MAP, 64>; threads = life_threads<64>(); return true;
    }
    return false;
}

static bool life_kernel(const tri_plan *p, const void *&fn, int &threads)
{
    switch (p->map) {
    case TRI_MAP_BB: return life_kernel_tile<MAP_BB>(p->tile, fn, threads);
    case TRI_MAP_RB: return life_kernel_tile<MAP_RB>(p->tile, fn, threads);
    case TRI_MAP_REC: return life_kernel_tile<MAP_REC>(p->tile, fn, threads);
    case TRI_MAP_LAMBDA: return life_kernel_tile<MAP_LAMBDA>(p->tile, fn, threads);
    }
    return false;
}

static bool life_step(const tri_plan *p, const LifeArgs &a, hipStream_t s)
{
    switch (p->map) {
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
    case 64: k_life<MAP_LAMBDA, 64><<<grid, life_threads<64>(), 0, s>>>(a); return true;
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
    if (!life_kernel(p, fn, threads)) return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: tile");
    hipGraph_t g = nullptr;
    TRI_HIP(hipGraphCreate(&g, 0));
    hipGraphNode_t prev = nullptr;
    hipError_t e = hipSuccess;
    for (int k = 0; k < steps && e == hipSuccess; ++k) {
        LifeArgs a = a0;
        a.t.cur = (k & 1) ? a0.t.nxt : a0.t.cur;
        a.t.nxt = (k & 1) ? (uint8_t *)a0.t.cur : a0.t.nxt;
        void *args[] = {&a};
        hipKernelNodeParams np{};
        np.func = (void *)fn;
        np.gridDim = dim3(p->gx, p->gy);
        np.blockDim = dim3(threads);
        np.sharedMemBytes = 0;
        np.kernelParams = args;
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
    if (p->map == TRI_MAP_UTM)
        return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: UTM has no tile to stage a halo in");
    if (p->tile > 64) return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: tile %d > 64", p->tile);
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
        if (!life_multi_kernel(p, fn))
            return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: temporal blocking needs tile 16, 32 or 64");
        const std::vector<int> sched = life_multi_schedule(steps);
        for (size_t k = 0; k < sched.size(); ++k) {
            a.t.cur = (k & 1) ? nxt : cur;
            a.t.nxt = (k & 1) ? cur : nxt;
            int gens = sched[k];
            void *args[] = {&a, &gens};
            TRI_HIP(hipLaunchKernel(fn, dim3(p->gx, p->gy), dim3(256), args, 0, s));
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
