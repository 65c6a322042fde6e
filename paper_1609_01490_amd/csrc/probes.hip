// Measurement probes: a STREAM-style add (c = a + b over 16-byte vectors, two
// reads and one write per element, the same mix as the fp32 elementwise
// body) that gives the HBM bandwidth a plain streaming kernel reaches on this
// GPU, the ceiling the triangular kernels are compared with.
#include "common.hpp"

namespace trimap {

typedef float f4p __attribute__((ext_vector_type(4)));

// Each workgroup streams a contiguous block of 4 x 256 vectors: every
// thread issues its four loads of a and of b before the first add.
constexpr int kStreamUnroll = 4;

__global__ void __launch_bounds__(256) k_stream_add(f4p *c, const f4p *a, const f4p *b,
                                                    uint64_t nvec)
{
    const uint64_t base = (uint64_t)blockIdx.x * (256 * kStreamUnroll) + threadIdx.x;
    f4p x[kStreamUnroll], y[kStreamUnroll];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
        const uint64_t k = base + 256 * u;
        if (k < nvec) {
            x[u] = __builtin_nontemporal_load(a + k);
            y[u] = __builtin_nontemporal_load(b + k);
        }
    }
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
        const uint64_t k = base + 256 * u;
        if (k < nvec) __builtin_nontemporal_store(x[u] + y[u], c + k);
    }
}

// Bandwidth probes for the roofline comparisons: one kernel shape with the
// access mix a template parameter.  Each thread moves 16-byte vectors,
// UNROLL of them per stream in flight before the first is used; workgroups
// walk the buffers in chunks of blockDim.x * UNROLL vectors (grid-stride, so
// that a grid of a few workgroups per CU streams the whole buffer as
// persistent workgroups, and a grid of one chunk per workgroup does not
// loop).  NT: non-temporal loads and stores.
enum { kProbeRead = 0, kProbeAdd = 1, kProbeFill = 2, kProbeCopy = 3 };

template <int KIND, int UNROLL, bool NT>
__global__ void __launch_bounds__(1024) k_probe(f4p *c, const f4p *a, const f4p *b, uint64_t nvec,
                                                float target)
{
    const uint64_t chunk = (uint64_t)blockDim.x * UNROLL;
    f4p acc = {0.f, 0.f, 0.f, 0.f};
    for (uint64_t base = (uint64_t)blockIdx.x * chunk + threadIdx.x; base < nvec;
         base += (uint64_t)gridDim.x * chunk) {
        f4p x[UNROLL], y[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const uint64_t k = base + (uint64_t)blockDim.x * u;
            if (k < nvec) {
                if (KIND != kProbeFill) x[u] = NT ? __builtin_nontemporal_load(a + k) : a[k];
                if (KIND == kProbeAdd) y[u] = NT ? __builtin_nontemporal_load(b + k) : b[k];
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const uint64_t k = base + (uint64_t)blockDim.x * u;
            if (k >= nvec) continue;
            if (KIND == kProbeRead) {
                acc += x[u];
            } else {
                f4p v;
                if (KIND == kProbeAdd) v = x[u] + y[u];
                else if (KIND == kProbeCopy) v = x[u];
                else v = f4p{target, target, target, target};
                if (NT) __builtin_nontemporal_store(v, c + k);
                else c[k] = v;
            }
        }
    }
    // the read probe keeps its loads live through a store no run takes
    // (target is chosen so that no sum equals it)
    if (KIND == kProbeRead && acc.x + acc.y + acc.z + acc.w == target)
        c[blockIdx.x] = acc;
}

template <int KIND, int UNROLL>
static void probe_launch(bool nt, dim3 grid, int threads, f4p *c, const f4p *a, const f4p *b,
                         uint64_t nvec, hipStream_t s)
{
    if (nt)
        k_probe<KIND, UNROLL, true><<<grid, threads, 0, s>>>(c, a, b, nvec, -1.f);
    else
        k_probe<KIND, UNROLL, false><<<grid, threads, 0, s>>>(c, a, b, nvec, -1.f);
}

template <int KIND>
static bool probe_unroll(int unroll, bool nt, dim3 grid, int threads, f4p *c, const f4p *a,
                         const f4p *b, uint64_t nvec, hipStream_t s)
{
    switch (unroll) {
    case 1: probe_launch<KIND, 1>(nt, grid, threads, c, a, b, nvec, s); return true;
    case 2: probe_launch<KIND, 2>(nt, grid, threads, c, a, b, nvec, s); return true;
    case 4: probe_launch<KIND, 4>(nt, grid, threads, c, a, b, nvec, s); return true;
    case 8: probe_launch<KIND, 8>(nt, grid, threads, c, a, b, nvec, s); return true;
    }
    return false;
}

}  // namespace trimap

using namespace trimap;

extern "C" tri_status tri_stream_probe(int kind, int unroll, int threads, int nontemporal,
                                       int64_t workgroups, float *c, const float *a,
                                       const float *b, int64_t count, void *stream)
{
    clear_error();
    if (kind < kProbeRead || kind > kProbeCopy) return fail(TRI_E_INVAL, "tri_stream_probe: kind");
    if (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8)
        return fail(TRI_E_INVAL, "tri_stream_probe: unroll must be 1, 2, 4 or 8");
    if (threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024)
        return fail(TRI_E_INVAL, "tri_stream_probe: threads must be 64 .. 1024, a power of two");
    if (count < 0 || workgroups < 0) return fail(TRI_E_INVAL, "tri_stream_probe: negative size");
    const bool need_a = kind != kProbeFill, need_b = kind == kProbeAdd;
    if (count > 0 && (!c || (need_a && !a) || (need_b && !b)))
        return fail(TRI_E_INVAL, "tri_stream_probe: NULL buffer");
    if (count % 4 || (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15))
        return fail(TRI_E_INVAL, "tri_stream_probe: count must be a multiple of 4 and buffers "
                                 "16-byte aligned");
    if (count == 0) return TRI_OK;
    const uint64_t nvec = (uint64_t)count / 4;
    const uint64_t chunk = (uint64_t)threads * unroll;
    uint64_t blocks = (nvec + chunk - 1) / chunk;
    if (workgroups > 0 && (uint64_t)workgroups < blocks) blocks = (uint64_t)workgroups;
    if (blocks > kMaxWorkItems / (uint64_t)threads)
        return fail(TRI_E_RANGE, "tri_stream_probe: count too large");
    const dim3 grid((uint32_t)blocks);
    hipStream_t s = (hipStream_t)stream;
    const bool nt = nontemporal != 0;
    f4p *cv = (f4p *)c;
    const f4p *av = (const f4p *)a, *bv = (const f4p *)b;
    switch (kind) {
    case kProbeRead: probe_unroll<kProbeRead>(unroll, nt, grid, threads, cv, av, bv, nvec, s); break;
    case kProbeAdd: probe_unroll<kProbeAdd>(unroll, nt, grid, threads, cv, av, bv, nvec, s); break;
    case kProbeFill: probe_unroll<kProbeFill>(unroll, nt, grid, threads, cv, av, bv, nvec, s); break;
    case kProbeCopy: probe_unroll<kProbeCopy>(unroll, nt, grid, threads, cv, av, bv, nvec, s); break;
    }
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}

extern "C" tri_status tri_stream_add(float *c, const float *a, const float *b, int64_t count,
                                     void *stream)
{
    clear_error();
    if (count < 0 || (count > 0 && (!a || !b || !c)))
        return fail(TRI_E_INVAL, "tri_stream_add: bad arguments");
    if (count % 4 || (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15))
        return fail(TRI_E_INVAL, "tri_stream_add: count must be a multiple of 4 and buffers 16-byte aligned");
    if (count == 0) return TRI_OK;
    const uint64_t nvec = (uint64_t)count / 4;
    const uint64_t blocks = (nvec + 256 * kStreamUnroll - 1) / (256 * kStreamUnroll);
    if (blocks > kMaxWorkItems / 256) return fail(TRI_E_RANGE, "tri_stream_add: count too large");
    k_stream_add<<<dim3((uint32_t)blocks), 256, 0, (hipStream_t)stream>>>((f4p *)c, (const f4p *)a,
                                                                          (const f4p *)b, nvec);
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}
