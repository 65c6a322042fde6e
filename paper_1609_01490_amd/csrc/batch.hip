// Batched triangular domains of uneven size in one persistent launch per
// generation, driven by a work queue over per-instance lambda numberings.
//
// Instance k owns B_k = m_k (m_k + 1) / 2 tiles (Section 3.1, block count of
// lambda).  The exclusive prefix P_k of the B_k numbers all tiles of all
// instances as one global range, so a work item g belongs to the instance k
// with P_k <= g < P_{k+1} and is that instance's block omega = g - P_k,
// whose tile is lambda(omega) (Eq. eq_gmap).  The prefix array grows with the
// number of instances, not with n, which keeps the paper's rule that a map
// uses no table growing with the problem size (Section 4.2).
//
// Persistent workgroups take items from an atomic counter until the range is
// exhausted, so small and large instances share the machine without one
// launch per instance.  Distance-map instances are independent tiles
// (generation 0 only); Game-of-Life instances need a grid-wide dependency
// between generations, so each generation is one node of a hipGraph (one
// persistent kernel per node, each with its own counter), and a small kernel
// node at the head of the graph clears the counters (no memset node).
#include <algorithm>
#include <new>
#include <vector>

#include "bodies.hpp"
#include "common.hpp"
#include "maps.hpp"

struct tri_batch;

namespace trimap {

bool launch_edm_f32_lambda(int tile, const TileGrid &g, const EdmTile &t, hipStream_t s);
bool launch_life_lambda(int tile, const TileGrid &g, const LifeTile &t, hipStream_t s);
bool launch_life_multi_lambda(int tile, const TileGrid &g, const LifeTile &t, int gens,
                              hipStream_t s);
std::vector<int> life_multi_schedule(int steps, int maxgen);

struct BatchDesc {
    int32_t kind;  // TRI_KIND_*
    int32_t n;
    int32_t d;
    int32_t pad;   // kDescVec16: a Life grid whose rows move as 16-byte vectors
    int64_t ld;    // distance map: ldx; Life: row pitch in bytes
    void *a;       // distance map: x; Life: grid of even generations
    void *b;       // distance map: out; Life: grid of odd generations
};

constexpr int32_t kDescVec16 = 1;  // ld % 16 == 0 and 16-byte aligned grids
constexpr int32_t kDescEdmVec4 = 2;  // distance map: coordinates staged as 16-byte vectors

struct BatchStepArgs {
    const BatchDesc *desc;
    const int64_t *prefix;  // count + 1 entries, prefix[0] = 0, prefix[count] = total
    const int32_t *idx;     // queue position -> instance (Life-only queues); null = identity
    int32_t count;
    int32_t step;           // node of the graph (Life buffers alternate per node)
    int32_t gens;           // Life generations in this node (0: the one-step body)
    int64_t total;
    uint32_t *head;         // this generation's counter
};

constexpr int kBatchThreads = 256;
// generations per node of the bit-sliced Life body in the batch (its halo)
constexpr int kBatchBitsGen = kLifeBitsStencilGen;
constexpr int kPrefixLds = 1024;  // prefix entries kept in LDS (else searched in memory)

template <int TL>
constexpr int life_multi_bytes() { return TL >= 16 ? 2 * LifeMultiShape<(TL >= 16 ? TL : 16)>::WORDS * 4 : 0; }

template <int TE, int TL>
struct BatchLds {
    static constexpr int EDM_BYTES = EdmF32Shape<TE>::LDS_FLOATS * 4;
    static constexpr int LIFE_BYTES = LifeShape<TL, kBatchThreads>::LDS_WORDS * 4;
    static constexpr int MULTI_BYTES = life_multi_bytes<TL>();
    // 64 x 64 Life tiles with several generations: one bit-sliced window of
    // two tiles per wave
    static constexpr int BITS_BYTES =
        TL == 64 ? kBatchThreads / 64 * LifeBits16Pair::WORDS * 4 : 0;
    static constexpr int B1 = EDM_BYTES > LIFE_BYTES ? EDM_BYTES : LIFE_BYTES;
    static constexpr int B2 = B1 > MULTI_BYTES ? B1 : MULTI_BYTES;
    static constexpr int BYTES = B2 > BITS_BYTES ? B2 : BITS_BYTES;
};

// Items are taken kChunk at a time (one atomic per chunk) and the next
// chunk is claimed as soon as the current one starts, so the atomic's
// round trip overlaps the work.  Consecutive items usually belong to the
// same instance: its range and descriptor are kept until an item leaves it.
constexpr int kChunk = 4;

// A workgroup-uniform 64-bit value read from LDS, made wave-uniform for the
// compiler (a value loaded from LDS counts as divergent, and so would every
// index, tile coordinate and branch derived from it)
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Every item through a workgroup-wide body (byte-sliced Life); four waves
// per SIMD bound the registers at 128 with no spills, and the grid is sized
// from the occupancy this gives.
template <int TE, int TL>
__global__ void __launch_bounds__(kBatchThreads, 4) k_batch_step(BatchStepArgs a)
{
    __shared__ __attribute__((aligned(16))) unsigned char body_lds[BatchLds<TE, TL>::BYTES];
    __shared__ int64_t pfx[kPrefixLds];
    __shared__ int64_t slot;

    const bool in_lds = a.count + 1 <= kPrefixLds;
    if (in_lds)
        for (int k = threadIdx.x; k <= a.count; k += kBatchThreads) pfx[k] = a.prefix[k];
    uint32_t next = 0;  // thread 0: first item of the chunk claimed ahead
    if (threadIdx.x == 0) next = atomicAdd(a.head, (uint32_t)kChunk);

    int64_t lo_g = 0, hi_g = 0;  // item range of the cached instance
    BatchDesc D{};
    for (;;) {
        __syncthreads();  // the previous item is done with the LDS and with slot
        if (threadIdx.x == 0) {
            slot = (int64_t)next;
            if ((int64_t)next < a.total) next = atomicAdd(a.head, (uint32_t)kChunk);
        }
        __syncthreads();
        const int64_t g0 = uniform64(slot);
        if (g0 >= a.total) return;  // uniform over the workgroup
        for (int c = 0; c < kChunk; ++c) {
            const int64_t g = g0 + c;
            if (g >= a.total) break;
            if (g < lo_g || g >= hi_g) {
                // instance: the largest q with prefix[q] <= g
                int lo = 0, hi = a.count;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    const int64_t pm = in_lds ? pfx[mid] : a.prefix[mid];
                    if (pm <= g) lo = mid;
                    else hi = mid;
                }
                lo = __builtin_amdgcn_readfirstlane(lo);  // uniform over the workgroup
                lo_g = uniform64(in_lds ? pfx[lo] : a.prefix[lo]);
                hi_g = uniform64(in_lds ? pfx[lo + 1] : a.prefix[lo + 1]);
                D = a.desc[a.idx ? __builtin_amdgcn_readfirstlane(a.idx[lo]) : lo];
            }
            if (c > 0) __syncthreads();  // LDS reuse between items of a chunk
            int32_t bi, bj;
            lambda_tile((uint64_t)(g - lo_g), 0u, bi, bj);
            bi = __builtin_amdgcn_readfirstlane(bi);
            bj = __builtin_amdgcn_readfirstlane(bj);
            if (D.kind == TRI_KIND_EDM) {
                const EdmTile t{D.n, D.d, D.ld, (const float *)D.a, (float *)D.b};
                if (D.pad & kDescEdmVec4)
                    edm_f32_tile_body<TE, kEdmStageVec4>(t, bi, bj, (float *)body_lds);
                else
                    edm_f32_tile_body<TE, kEdmStageLoop>(t, bi, bj, (float *)body_lds);
            } else {
                const bool even = (a.step & 1) == 0;
                const LifeTile t{D.n, D.ld, (const uint8_t *)(even ? D.a : D.b),
                                 (uint8_t *)(even ? D.b : D.a)};
                bool done = false;
                if constexpr (TL >= 16) {
                    if (a.gens > 0) {
                        life_multi_tile_body<TL, true>(t, bi, bj, a.gens, (uint32_t *)body_lds);
                        done = true;
                    }
                }
                if (!done) life_tile_body<TL, kBatchThreads, false>(t, bi, bj, (uint32_t *)body_lds);
            }
        }
    }
}

// 64 x 64 Life tiles, every Life grid of the batch with 16-byte rows, and
// nodes of several generations (temporal plans): items are taken
// kChunkBits at a time.  The workgroup first runs the chunk's distance
// items one after the other, then each wave takes two consecutive items,
// 2 w and 2 w + 1, through the bit-sliced window of two tiles: as one
// window when they are neighbours in a tile row of one instance (as
// consecutive lambda blocks mostly are), else each in a window of its own
// with the second half not written back.  One call site per body keeps the
// registers at those of the larger body.  VEC4: every distance instance
// stages its coordinates as 16-byte vectors (chosen at bind time, so that
// the kernel holds one distance body).
constexpr int kChunkBits = 2 * kBatchThreads / 64;

template <int TE, bool VEC4>
__global__ void __launch_bounds__(kBatchThreads, 4) k_batch_step_bits(BatchStepArgs a)
{
    constexpr int EDM_BYTES = EdmF32Shape<TE>::LDS_FLOATS * 4;
    constexpr int PAIR_BYTES = kBatchThreads / 64 * LifeBits16Pair::WORDS * 4;
    static_assert(kBatchBitsGen == LifeBits16Pair::K, "halo of the paired window");
    __shared__ __attribute__((aligned(16)))
    unsigned char body_lds[EDM_BYTES > PAIR_BYTES ? EDM_BYTES : PAIR_BYTES];
    __shared__ int64_t pfx[kPrefixLds];
    __shared__ int64_t slot;

    const bool in_lds = a.count + 1 <= kPrefixLds;
    if (in_lds)
        for (int k = threadIdx.x; k <= a.count; k += kBatchThreads) pfx[k] = a.prefix[k];
    uint32_t next = 0;  // thread 0: first item of the chunk claimed ahead
    if (threadIdx.x == 0) next = atomicAdd(a.head, (uint32_t)kChunkBits);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint32_t *wl = (uint32_t *)body_lds + wv * LifeBits16Pair::WORDS;

    // the instance of item g (wave-uniform): the largest q with prefix[q] <= g
    const auto locate = [&](int64_t g, int64_t &lo_g, int64_t &hi_g, BatchDesc &D) {
        int lo = 0, hi = a.count;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            const int64_t pm = in_lds ? pfx[mid] : a.prefix[mid];
            if (pm <= g) lo = mid;
            else hi = mid;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        lo_g = uniform64(in_lds ? pfx[lo] : a.prefix[lo]);
        hi_g = uniform64(in_lds ? pfx[lo + 1] : a.prefix[lo + 1]);
        D = a.desc[a.idx ? __builtin_amdgcn_readfirstlane(a.idx[lo]) : lo];
    };
    int64_t lo_g = 0, hi_g = 0;  // item range of the cached instance
    BatchDesc D{};
    for (;;) {
        __syncthreads();  // the previous chunk is done with the LDS and with slot
        if (threadIdx.x == 0) {
            slot = (int64_t)next;
            if ((int64_t)next < a.total) next = atomicAdd(a.head, (uint32_t)kChunkBits);
        }
        __syncthreads();
        const int64_t g0 = uniform64(slot);
        if (g0 >= a.total) return;  // uniform over the workgroup
        // the chunk's distance items, the whole workgroup each
        bool used = false;
        for (int c = 0; c < kChunkBits; ++c) {
            const int64_t g = g0 + c;
            if (g >= a.total) break;
            if (g < lo_g || g >= hi_g) locate(g, lo_g, hi_g, D);
            if (D.kind != TRI_KIND_EDM) continue;
            if (used) __syncthreads();  // LDS reuse between items
            used = true;
            int32_t bi, bj;
            lambda_tile((uint64_t)(g - lo_g), 0u, bi, bj);
            bi = __builtin_amdgcn_readfirstlane(bi);
            bj = __builtin_amdgcn_readfirstlane(bj);
            const EdmTile t{D.n, D.d, D.ld, (const float *)D.a, (float *)D.b};
            edm_f32_tile_body<TE, VEC4 ? kEdmStageVec4 : kEdmStageLoop>(t, bi, bj, (float *)body_lds);
        }
        if (used) __syncthreads();  // the windows below reuse the LDS
        // the chunk's Life items: wave w takes items 2 w and 2 w + 1
        bool life[2];
        int32_t ti[2], tj[2];
        int64_t tl[2];
        BatchDesc TD[2];
        int64_t l0 = 0, h0 = 0;  // the instance range of item 2 w
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int64_t g = g0 + 2 * wv + e;
            life[e] = false;
            ti[e] = tj[e] = 0;
            tl[e] = -1;
            if (g < a.total) {
                int64_t l, h;
                if (e == 1 && g < h0) {  // in the instance of item 2 w (g - 1 < total, so l0 is set)
                    l = l0;
                    TD[1] = TD[0];
                } else {
                    locate(g, l, h, TD[e]);
                    if (e == 0) {
                        l0 = l;
                        h0 = h;
                    }
                }
                if (TD[e].kind == TRI_KIND_LIFE) {
                    life[e] = true;
                    tl[e] = l;
                    lambda_tile((uint64_t)(g - l), 0u, ti[e], tj[e]);
                    ti[e] = __builtin_amdgcn_readfirstlane(ti[e]);
                    tj[e] = __builtin_amdgcn_readfirstlane(tj[e]);
                }
            }
        }
        const bool pair = life[0] && life[1] && tl[0] == tl[1] && ti[1] == ti[0] && tj[1] == tj[0] + 1;
        const int nw = pair ? 1 : (int)life[0] + (int)life[1];
        const bool even = (a.step & 1) == 0;
        for (int u = 0; u < nw; ++u) {
            const int e = (u == 0 && life[0]) ? 0 : 1;
            const BatchDesc &W = TD[e];
            const LifeTile t{W.n, W.ld, (const uint8_t *)(even ? W.a : W.b),
                             (uint8_t *)(even ? W.b : W.a)};
            life_bits16_pair_body(t, ti[e], tj[e], pair, a.gens, wl);
        }
    }
}

__global__ void k_batch_reset(uint32_t *heads, int32_t count)
{
    for (int k = threadIdx.x; k < count; k += blockDim.x) heads[k] = 0u;
}

typedef void (*StepKernel)(BatchStepArgs);

template <int TE>
static StepKernel step_kernel_te(int tl, bool bits, bool vec4)
{
    switch (tl) {
    case 8: return k_batch_step<TE, 8>;
    case 16: return k_batch_step<TE, 16>;
    case 32: return k_batch_step<TE, 32>;
    case 64:
        if (!bits) return k_batch_step<TE, 64>;
        return vec4 ? k_batch_step_bits<TE, true> : k_batch_step_bits<TE, false>;
    }
    return nullptr;
}

// bits: the bit-sliced variant (tile 64 only; null otherwise), vec4: its
// form for batches whose distance instances all stage 16-byte vectors
static StepKernel step_kernel(int te, int tl, bool bits = false, bool vec4 = false)
{
    if (bits && tl != 64) return nullptr;
    switch (te) {
    case 16: return step_kernel_te<16>(tl, bits, vec4);
    case 32: return step_kernel_te<32>(tl, bits, vec4);
    case 64: return step_kernel_te<64>(tl, bits, vec4);
    }
    return nullptr;
}

}  // namespace trimap

using namespace trimap;

struct tri_batch {
    int32_t count = 0, edm_tile = 0, life_tile = 0, steps = 0;
    bool temporal = false;
    std::vector<int> sched;             // Life generations per node (temporal)
    std::vector<int32_t> kind;
    std::vector<int64_t> n, d, tiles;   // tiles: lambda blocks of each instance
    std::vector<int64_t> prefix0;       // every instance (generation 0)
    std::vector<int64_t> prefix1;       // Life instances (generations >= 1)
    std::vector<int32_t> idx1;
    std::vector<BatchDesc> desc;        // host copy (per-instance mode)
    int device = 0;
    uint32_t grid = 0;                  // persistent workgroups
    StepKernel kernel = nullptr;        // the kernel bound (one of the two below)
    StepKernel kernel_bytes = nullptr;  // Life tiles byte-sliced
    StepKernel kernel_bits = nullptr;   // 64 x 64 Life tiles bit-sliced (or null)
    uint32_t grid_bytes = 0, grid_bits = 0;
    // device memory owned by the plan
    BatchDesc *d_desc = nullptr;
    int64_t *d_prefix0 = nullptr, *d_prefix1 = nullptr;
    int32_t *d_idx1 = nullptr;
    uint32_t *d_heads = nullptr;
    bool bound = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void batch_free(tri_batch *b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    (void)hipFree(b->d_desc);
    (void)hipFree(b->d_prefix0);
    (void)hipFree(b->d_prefix1);
    (void)hipFree(b->d_idx1);
    (void)hipFree(b->d_heads);
    delete b;
}

static int batch_nodes(const tri_batch *b)
{
    return b->temporal ? std::max<int>(1, (int)b->sched.size()) : std::max(1, b->steps);
}

static BatchStepArgs step_args(const tri_batch *b, int s)
{
    BatchStepArgs a{};
    a.desc = b->d_desc;
    a.step = s;
    a.gens = (b->temporal && s < (int)b->sched.size()) ? b->sched[s] : 0;
    a.head = b->d_heads + s;
    if (s == 0) {
        a.prefix = b->d_prefix0;
        a.idx = nullptr;
        a.count = b->count;
        a.total = b->prefix0.back();
    } else {
        a.prefix = b->d_prefix1;
        a.idx = b->d_idx1;
        a.count = (int32_t)b->idx1.size();
        a.total = b->prefix1.back();
    }
    return a;
}

// the persistent launches: counter reset, then one kernel per generation
static tri_status batch_enqueue(const tri_batch *b, hipStream_t s)
{
    const int S = batch_nodes(b);
    k_batch_reset<<<1, 256, 0, s>>>(b->d_heads, S);
    TRI_HIP(hipGetLastError());
    for (int k = 0; k < S; ++k) {
        BatchStepArgs a = step_args(b, k);
        if (a.total == 0) continue;
        hipLaunchKernelGGL(b->kernel, dim3(b->grid), dim3(kBatchThreads), 0, s, a);
        TRI_HIP(hipGetLastError());
    }
    return TRI_OK;
}

static tri_status batch_build_graph(tri_batch *b)
{
    const int S = batch_nodes(b);
    TRI_HIP(hipGraphCreate(&b->graph, 0));
    hipGraphNode_t prev = nullptr;
    {
        hipKernelNodeParams np{};
        uint32_t *heads = b->d_heads;
        int32_t cnt = S;
        void *args[] = {&heads, &cnt};
        np.func = (void *)k_batch_reset;
        np.gridDim = dim3(1);
        np.blockDim = dim3(256);
        np.sharedMemBytes = 0;
        np.kernelParams = args;
        np.extra = nullptr;
        TRI_HIP(hipGraphAddKernelNode(&prev, b->graph, nullptr, 0, &np));
    }
    for (int k = 0; k < S; ++k) {
        BatchStepArgs a = step_args(b, k);
        if (a.total == 0) continue;
        hipKernelNodeParams np{};
        void *args[] = {&a};
        np.func = (void *)b->kernel;
        np.gridDim = dim3(b->grid);
        np.blockDim = dim3(kBatchThreads);
        np.sharedMemBytes = 0;
        np.kernelParams = args;
        np.extra = nullptr;
        hipGraphNode_t node;
        TRI_HIP(hipGraphAddKernelNode(&node, b->graph, &prev, 1, &np));
        prev = node;
    }
    TRI_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return TRI_OK;
}

extern "C" {

tri_status tri_batch_plan(tri_batch **out, int32_t count, const int32_t *host_kind,
                          const int64_t *host_n, const int64_t *host_d, int edm_tile,
                          int life_tile, int life_steps, uint32_t flags)
{
    clear_error();
    if (!out) return fail(TRI_E_INVAL, "tri_batch_plan: out is NULL");
    *out = nullptr;
    if (count < 1 || !host_kind || !host_n || !host_d)
        return fail(TRI_E_INVAL, "tri_batch_plan: need count >= 1 and host arrays");
    if (edm_tile != 16 && edm_tile != 32 && edm_tile != 64)
        return fail(TRI_E_INVAL, "tri_batch_plan: edm_tile %d not in {16,32,64}", edm_tile);
    if (life_tile != 8 && life_tile != 16 && life_tile != 32 && life_tile != 64)
        return fail(TRI_E_INVAL, "tri_batch_plan: life_tile %d not in {8,16,32,64}", life_tile);
    if (life_steps < 0 || life_steps > 4096)
        return fail(TRI_E_INVAL, "tri_batch_plan: life_steps %d not in [0, 4096]", life_steps);
    if (flags & ~(uint32_t)TRI_FLAG_LIFE_TEMPORAL)
        return fail(TRI_E_INVAL, "tri_batch_plan: unknown flags 0x%x", flags);
    if ((flags & TRI_FLAG_LIFE_TEMPORAL) && life_tile < 16)
        return fail(TRI_E_UNSUPPORTED, "tri_batch_plan: temporal blocking needs life_tile >= 16");

    tri_batch *b = new (std::nothrow) tri_batch();
    if (!b) return fail(TRI_E_NOMEM, "tri_batch_plan: out of host memory");
    b->count = count;
    b->edm_tile = edm_tile;
    b->life_tile = life_tile;
    b->steps = life_steps;
    b->temporal = (flags & TRI_FLAG_LIFE_TEMPORAL) != 0;
    if (b->temporal && life_steps > 0) b->sched = life_multi_schedule(life_steps, kLifeMaxGen);
    b->kernel = b->kernel_bytes = step_kernel(edm_tile, life_tile);
    b->kernel_bits = step_kernel(edm_tile, life_tile, true);
    b->prefix0.push_back(0);
    b->prefix1.push_back(0);
    for (int32_t k = 0; k < count; ++k) {
        const int32_t kd = host_kind[k];
        const int64_t nk = host_n[k], dk = host_d[k];
        if (kd != TRI_KIND_EDM && kd != TRI_KIND_LIFE) {
            batch_free(b);
            return fail(TRI_E_INVAL, "tri_batch_plan: kind[%d] = %d", k, kd);
        }
        if (nk < 1 || nk >= (1ll << 20)) {
            batch_free(b);
            return fail(TRI_E_RANGE, "tri_batch_plan: n[%d] = %lld not in [1, 2^20)", k, (long long)nk);
        }
        if (kd == TRI_KIND_EDM && (dk < 1 || dk > 4096)) {
            batch_free(b);
            return fail(TRI_E_RANGE, "tri_batch_plan: d[%d] = %lld not in [1, 4096]", k, (long long)dk);
        }
        const int64_t ne = kd == TRI_KIND_EDM ? nk - 1 : nk;
        const int tile = kd == TRI_KIND_EDM ? edm_tile : life_tile;
        const int64_t m = (ne + tile - 1) / tile;
        const int64_t T = m * (m + 1) / 2;
        b->kind.push_back(kd);
        b->n.push_back(nk);
        b->d.push_back(dk);
        b->tiles.push_back(T);
        // generation 0 holds every distance-map tile and the Life tiles of
        // the first generation (none when no generation is asked for)
        b->prefix0.push_back(b->prefix0.back() + ((kd == TRI_KIND_LIFE && life_steps == 0) ? 0 : T));
        if (kd == TRI_KIND_LIFE) {
            b->prefix1.push_back(b->prefix1.back() + T);
            b->idx1.push_back(k);
        }
    }
    if (b->prefix0.back() >= (1ll << 31)) {
        batch_free(b);
        return fail(TRI_E_RANGE, "tri_batch_plan: more than 2^31 tiles in one generation");
    }

    hipError_t e = hipGetDevice(&b->device);
    int cus = 0, per_cu = 0, per_cu_bits = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)b->kernel_bytes,
                                                         kBatchThreads, 0);
    if (e == hipSuccess && b->kernel_bits)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_bits, (const void *)b->kernel_bits,
                                                         kBatchThreads, 0);
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "tri_batch_plan: device query");
    }
    b->grid = b->grid_bytes = (uint32_t)std::max(1, cus * std::max(1, per_cu));
    b->grid_bits = (uint32_t)std::max(1, cus * std::max(1, per_cu_bits));

    const size_t nl = b->idx1.size();
    const int S = batch_nodes(b);
    e = hipMalloc(&b->d_desc, sizeof(BatchDesc) * count);
    if (e == hipSuccess) e = hipMalloc(&b->d_prefix0, sizeof(int64_t) * (count + 1));
    if (e == hipSuccess) e = hipMalloc(&b->d_prefix1, sizeof(int64_t) * (nl + 1));
    if (e == hipSuccess && nl) e = hipMalloc(&b->d_idx1, sizeof(int32_t) * nl);
    if (e == hipSuccess) e = hipMalloc(&b->d_heads, sizeof(uint32_t) * S);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_prefix0, b->prefix0.data(), sizeof(int64_t) * (count + 1),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_prefix1, b->prefix1.data(), sizeof(int64_t) * (nl + 1),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && nl)
        e = hipMemcpy(b->d_idx1, b->idx1.data(), sizeof(int32_t) * nl, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "tri_batch_plan: device allocation");
    }
    *out = b;
    return TRI_OK;
}

tri_status tri_batch_bind(tri_batch *b, void *const *host_a, void *const *host_b,
                          const int64_t *host_ld)
{
    clear_error();
    if (!b || !host_a || !host_b || !host_ld) return fail(TRI_E_INVAL, "tri_batch_bind: NULL argument");
    std::vector<BatchDesc> desc(b->count);
    for (int32_t k = 0; k < b->count; ++k) {
        BatchDesc &D = desc[k];
        D.kind = b->kind[k];
        D.n = (int32_t)b->n[k];
        D.d = (int32_t)b->d[k];
        D.pad = 0;
        D.ld = host_ld[k];
        D.a = host_a[k];
        D.b = host_b[k];
        if (!D.a || !D.b || D.a == D.b)
            return fail(TRI_E_INVAL, "tri_batch_bind: buffers of instance %d", k);
        if (D.kind == TRI_KIND_EDM) {
            if (D.ld < D.d || (((uintptr_t)D.a | (uintptr_t)D.b) & 3))
                return fail(TRI_E_INVAL, "tri_batch_bind: instance %d: ldx < d or unaligned", k);
            // 16-byte staging loads where every row starts on 16 bytes and
            // the byte offsets fit 32 bits (as for the single FP32 kernel)
            if (D.d % 4 == 0 && D.ld % 4 == 0 && ((uintptr_t)D.a & 15) == 0 &&
                (uint64_t)D.n * (uint64_t)D.ld * 4 < (1ull << 31))
                D.pad = kDescEdmVec4;
        } else {
            if (D.ld < D.n || D.ld % 4 || (((uintptr_t)D.a | (uintptr_t)D.b) & 3))
                return fail(TRI_E_INVAL,
                            "tri_batch_bind: instance %d: ld must be >= n, a multiple of 4", k);
            if (D.ld % 16 == 0 && (((uintptr_t)D.a | (uintptr_t)D.b) & 15) == 0) D.pad = kDescVec16;
        }
    }
    TRI_HIP(hipMemcpy(b->d_desc, desc.data(), sizeof(BatchDesc) * b->count,
                      hipMemcpyHostToDevice));
    b->desc = desc;
    // the bit-sliced kernel when every Life grid has 16-byte rows and the
    // nodes advance several generations
    bool bits = b->kernel_bits != nullptr && b->temporal;
    bool vec4 = true;  // every distance instance stages 16-byte vectors
    for (const BatchDesc &D : desc) {
        if (D.kind == TRI_KIND_LIFE && !(D.pad & kDescVec16)) bits = false;
        if (D.kind == TRI_KIND_EDM && !(D.pad & kDescEdmVec4)) vec4 = false;
    }
    // (the two forms of the bit-sliced kernel have the same launch bound and
    // LDS, so the same persistent grid)
    b->kernel = bits ? (vec4 ? step_kernel(b->edm_tile, b->life_tile, true, true) : b->kernel_bits)
                     : b->kernel_bytes;
    b->grid = bits ? b->grid_bits : b->grid_bytes;
    // the bit-sliced kernel advances up to kBatchBitsGen generations per
    // node (fewer nodes than the plan's schedule, whose counters it reuses)
    if (b->temporal && b->steps > 0)
        b->sched = life_multi_schedule(b->steps, bits ? kBatchBitsGen : kLifeMaxGen);
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    tri_status st = batch_build_graph(b);
    if (st != TRI_OK) return st;
    b->bound = true;
    return TRI_OK;
}

tri_status tri_batch_launch(tri_batch *b, int how, void *stream)
{
    clear_error();
    if (!b) return fail(TRI_E_INVAL, "tri_batch_launch: plan is NULL");
    if (!b->bound) return fail(TRI_E_INVAL, "tri_batch_launch: call tri_batch_bind first");
    hipStream_t s = (hipStream_t)stream;
    switch (how) {
    case TRI_BATCH_GRAPH:
        TRI_HIP(hipGraphLaunch(b->exec, s));
        return TRI_OK;
    case TRI_BATCH_STREAM:
        return batch_enqueue(b, s);
    case TRI_BATCH_PER_INSTANCE: {
        // the same tile bodies, one launch per instance and generation
        for (int32_t k = 0; k < b->count; ++k) {
            const BatchDesc &D = b->desc[k];
            const int64_t ne = D.kind == TRI_KIND_EDM ? D.n - 1 : D.n;
            const int tile = D.kind == TRI_KIND_EDM ? b->edm_tile : b->life_tile;
            const int64_t m = (ne + tile - 1) / tile;
            const TileGrid g{(int32_t)m, 0u, (uint64_t)b->tiles[k]};
            if (b->tiles[k] == 0) continue;
            if (D.kind == TRI_KIND_EDM) {
                const EdmTile t{D.n, D.d, D.ld, (const float *)D.a, (float *)D.b};
                if (!launch_edm_f32_lambda(tile, g, t, s))
                    return fail(TRI_E_UNSUPPORTED, "tri_batch_launch: distance instance %d", k);
                TRI_HIP(hipGetLastError());
            } else {
                const int nodes = b->temporal ? (int)b->sched.size() : b->steps;
                for (int st = 0; st < nodes; ++st) {
                    const bool even = (st & 1) == 0;
                    const LifeTile t{D.n, D.ld, (const uint8_t *)(even ? D.a : D.b),
                                     (uint8_t *)(even ? D.b : D.a)};
                    const bool ok = b->temporal ? launch_life_multi_lambda(tile, g, t, b->sched[st], s)
                                                : launch_life_lambda(tile, g, t, s);
                    if (!ok)
                        return fail(TRI_E_UNSUPPORTED, "tri_batch_launch: Life instance %d", k);
                    TRI_HIP(hipGetLastError());
                }
            }
        }
        return TRI_OK;
    }
    }
    return fail(TRI_E_INVAL, "tri_batch_launch: how = %d", how);
}

tri_status tri_batch_query(const tri_batch *b, tri_batch_info *info)
{
    clear_error();
    if (!b || !info) return fail(TRI_E_INVAL, "tri_batch_query: NULL argument");
    info->count = b->count;
    info->life_instances = (int32_t)b->idx1.size();
    info->edm_tile = b->edm_tile;
    info->life_tile = b->life_tile;
    info->life_steps = b->steps;
    info->graph_nodes = batch_nodes(b);
    info->persistent_workgroups = (int32_t)b->grid;
    info->items_generation0 = b->prefix0.back();
    info->items_per_later_generation = b->prefix1.back();
    return TRI_OK;
}

tri_status tri_batch_autotune(int32_t count, const int32_t *host_kind, const int64_t *host_n,
                              const int64_t *host_d, int life_steps, void *const *host_a,
                              void *const *host_b, const int64_t *host_ld, int reps, void *stream,
                              int *best_edm_tile, int *best_life_tile, uint32_t *best_flags,
                              float *best_ms)
{
    clear_error();
    if (!best_edm_tile || !best_life_tile) return fail(TRI_E_INVAL, "tri_batch_autotune: NULL output");
    if (reps < 1) reps = 1;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    TRI_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he, "tri_batch_autotune: event");
    }
    const int edm_tiles[] = {16, 32, 64}, life_tiles[] = {8, 16, 32, 64};
    float best = -1.f;
    tri_status st = TRI_OK;
    for (int te : edm_tiles) {
        for (int cand = 0; cand < 7; ++cand) {
            // life tiles 8..64 one generation per node, then 16..64 temporal
            const int tl = cand < 4 ? life_tiles[cand] : life_tiles[cand - 3];
            const uint32_t fl = cand < 4 ? 0u : (uint32_t)TRI_FLAG_LIFE_TEMPORAL;
            tri_batch *b = nullptr;
            st = tri_batch_plan(&b, count, host_kind, host_n, host_d, te, tl, life_steps, fl);
            if (st != TRI_OK) break;
            st = tri_batch_bind(b, host_a, host_b, host_ld);
            if (st == TRI_OK) st = tri_batch_launch(b, TRI_BATCH_GRAPH, stream);  // warm-up
            if (st == TRI_OK) he = hipEventRecord(e0, s);
            for (int r = 0; r < reps && st == TRI_OK && he == hipSuccess; ++r)
                st = tri_batch_launch(b, TRI_BATCH_GRAPH, stream);
            if (st == TRI_OK && he == hipSuccess) he = hipEventRecord(e1, s);
            if (st == TRI_OK && he == hipSuccess) he = hipEventSynchronize(e1);
            float ms = 0.f;
            if (st == TRI_OK && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            tri_batch_destroy(b);
            if (he != hipSuccess) st = hip_fail(he, "tri_batch_autotune: timing");
            if (st != TRI_OK) break;
            ms /= (float)reps;
            if (best < 0.f || ms < best) {
                best = ms;
                *best_edm_tile = te;
                *best_life_tile = tl;
                if (best_flags) *best_flags = fl;
            }
        }
        if (st != TRI_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != TRI_OK) return st;
    if (best_ms) *best_ms = best;
    return TRI_OK;
}

tri_status tri_batch_destroy(tri_batch *b)
{
    clear_error();
    batch_free(b);
    return TRI_OK;
}

}  // extern "C"
