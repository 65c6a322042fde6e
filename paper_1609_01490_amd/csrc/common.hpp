// Internal declarations shared by the trimap translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "trimap.h"

#include <map>
#include <mutex>
#include <tuple>

// Instantiated graphs a plan has built (one per buffers / step count), owned
// by the plan and destroyed with it.
struct PlanGraphKey {
    const void *cur;
    const void *nxt;
    int64_t ld;
    int steps;
    bool operator<(const PlanGraphKey &o) const
    {
        return std::tie(cur, nxt, ld, steps) < std::tie(o.cur, o.nxt, o.ld, o.steps);
    }
};

struct PlanGraphs {
    std::mutex mu;
    std::map<PlanGraphKey, hipGraphExec_t> execs;
};

// A plan: tile space of a triangular domain under one map (Section 3.1).
// The strict lower triangle of side n is stored as the diagonal-including
// triangle of side n - 1 shifted down one row (row_off = 1).
struct tri_plan {
    int64_t n;        // side of the domain
    int64_t ne;       // side of the diagonal-including triangle that is tiled
    int32_t row_off;  // 0, or 1 for the strict lower triangle
    int32_t tile;     // rho
    int32_t map;      // tri_map
    int32_t diag;     // include_diag
    uint32_t flags;   // TRI_FLAG_*
    int64_t m;        // tiles per side
    int64_t T;        // tiles = m (m + 1) / 2
    int64_t elements; // cells of the domain
    // launch grid of the map, in blocks (UTM: blocks of kUtmThreads threads)
    uint32_t gx, gy;
    int64_t blocks;
    PlanGraphs *graphs;  // graph cache (the only mutable part of a plan)
};

namespace trimap {

constexpr int kUtmThreads = 256;
constexpr uint64_t kMaxWorkItems = 0xFFFFFFFFull;  // per grid dimension
constexpr uint32_t kMaxGridY = 65535u;

tri_status fail(tri_status st, const char *fmt, ...);
tri_status hip_fail(hipError_t e, const char *what);
void clear_error();

}  // namespace trimap

#define TRI_HIP(call)                                          \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return trimap::hip_fail(e_, #call); \
    } while (0)
