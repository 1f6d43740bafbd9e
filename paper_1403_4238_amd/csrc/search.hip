// findBestPatch on gfx950, one search per launch: every work-group stages
// and scores one tile (see search_tile.h) and writes the tile's minimum key
// to the partials; the commit kernel reduces them.  k_search_direct is the
// same search without LDS staging, the paper's kernel without local memory
// (Alg. 1 as against Alg. 2), kept for that comparison.
#include <hip/hip_ext.h>

#include "search_tile.h"

namespace inpaint {

namespace {

using tile::ScalarTarget;
using tile::TileGeom;

// Minimum over the work-group of the wave minima, written to out[t].
__device__ __forceinline__ void write_tile_min(uint64_t best, int t, uint64_t *__restrict__ out, uint64_t *red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t b = red[0];
#pragma unroll
        for (int w = 1; w < kSearchWaves; ++w) b = red[w] < b ? red[w] : b;
        out[t] = b;
    }
}

// Stages and scores one tile and writes its minimum key to out[t].  `live`
// (uniform) is false when the fill loop has nothing pending: the tile is then
// staged but neither scored nor written.
template <int R, int NY, bool ISECT = false>
__device__ __forceinline__ void search_tile(const JobDev &d, const TargetStage *tg, bool live, int rx0, int ry0,
                                            int rx1, int ry1, int ntx, int t, uint64_t *__restrict__ out,
                                            uint32_t *lds, uint64_t *red) {
    int tx0, ty0;
    tile::tile_origin<R, NY>(rx0, ry0, ntx, t, &tx0, &ty0);
    const uint32_t vmask = tile::stage_tile<R, NY, ISECT>(d, tx0, ty0, rx1, ry1, lds);
    // one barrier publishes the LDS tile and tells whether any candidate of
    // the tile is valid
    if (!__syncthreads_or(live && vmask != 0)) {
        if (threadIdx.x == 0 && live) out[t] = ~0ull;
        return;
    }
    const ScalarTarget view{(tile::ConstTarget *)tg};
    write_tile_min(tile::wave_min_u64(tile::score_tile<R, NY, ScalarTarget, ISECT>(d, view, tx0, ty0, vmask, lds)),
                   t, out, red);
}

// Consecutive work-groups are dispatched round-robin over the 8 XCDs; remap
// so that each XCD scores one contiguous band of tiles and keeps that band
// of the image resident in its own L2 across searches.
__device__ __forceinline__ int xcd_band_tile(int bid, int grid) {
    const int per = grid >> 3;
    return (bid & 7) * per + (bid >> 3);
}

template <int R, int NY, bool ISECT>
__global__ __launch_bounds__(kSearchWaves * 64) void k_search(JobDev d, int query, int rx0, int ry0,
                                                              int rx1, int ry1, int ntx, int ntiles) {
    using G = TileGeom<R, NY>;
    __shared__ __attribute__((aligned(16))) uint32_t lds[G::LDS_WORDS];
    __shared__ uint64_t red[kSearchWaves];
    const int t = xcd_band_tile((int)blockIdx.x, (int)gridDim.x);
    if (t >= ntiles) return;
    // The state is read here but tested only after the tile loads are
    // issued, so its latency overlaps theirs.
    bool live = true;
    if (!query) {
        const IterState *st = d.st;
        live = !(st->done || st->error || !st->pending || st->iter >= st->iter_limit);
    }
    search_tile<R, NY, ISECT>(d, query ? d.qtgt : d.tgt, live, rx0, ry0, rx1, ry1, ntx, t, d.partials, lds, red);
}

// One tile scored straight from the padded plane (no LDS tile); otherwise
// as k_search.
template <int R, int NY, bool ISECT>
__global__ __launch_bounds__(kSearchWaves * 64) void k_search_direct(JobDev d, int query, int rx0, int ry0,
                                                                     int rx1, int ry1, int ntx, int ntiles) {
    __shared__ uint64_t red[kSearchWaves];
    const int t = xcd_band_tile((int)blockIdx.x, (int)gridDim.x);
    if (t >= ntiles) return;
    bool live = true;
    if (!query) {
        const IterState *st = d.st;
        live = !(st->done || st->error || !st->pending || st->iter >= st->iter_limit);
    }
    int tx0, ty0;
    tile::tile_origin<R, NY>(rx0, ry0, ntx, t, &tx0, &ty0);
    const uint32_t vmask = tile::tile_valid<R, NY, ISECT>(d, tx0, ty0, rx1, ry1);
    if (!__syncthreads_or(live && vmask != 0)) {
        if (threadIdx.x == 0 && live) d.partials[t] = ~0ull;
        return;
    }
    const ScalarTarget view{(tile::ConstTarget *)(query ? d.qtgt : d.tgt)};
    write_tile_min(tile::wave_min_u64(tile::score_direct<R, NY, ScalarTarget, ISECT>(d, view, tx0, ty0, vmask)), t,
                   d.partials, red);
}

// Persistent form over many images: work-groups stride over a static list of
// (image slot, tile) items; finished images cost one state read per item.
template <int R, int NY>
__global__ __launch_bounds__(kSearchWaves * 64) void k_search_batched(const JobDev *slots,
                                                                      const WorkItem *items,
                                                                      const int32_t *nitems) {
    using G = TileGeom<R, NY>;
    __shared__ __attribute__((aligned(16))) uint32_t lds[G::LDS_WORDS];
    __shared__ uint64_t red[kSearchWaves];
    const int n = *nitems;
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const WorkItem w = items[it];
        const JobDev &d = slots[w.slot];
        const IterState *st = d.st;
        const bool live = st && !st->done && !st->error && st->pending && st->iter < st->iter_limit;
        if (live)
            search_tile<R, NY>(d, d.tgt, true, d.rx0, d.ry0, d.rx1, d.ry1, d.ntx, w.tile, d.partials, lds, red);
        __syncthreads();
    }
}

template <int R, int NY, bool DIRECT>
hipError_t launch_search_t(const JobDev &d, bool query, int rx0, int ry0, int rx1, int ry1, int ntx,
                           int nty, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
    const int ntiles = ntx * nty;
    if (ntiles <= 0) return hipSuccess;
    const int grid = (ntiles + 7) / 8 * 8;
    auto kernel = DIRECT ? (d.isect ? k_search_direct<R, NY, true> : k_search_direct<R, NY, false>)
                         : (d.isect ? k_search<R, NY, true> : k_search<R, NY, false>);
    if (start) {
        // The runtime stamps these events with the kernel's own begin / end.
        hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(kSearchWaves * 64), 0, s, start, stop, 0, d,
                              query ? 1 : 0, rx0, ry0, rx1, ry1, ntx, ntiles);
    } else {
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(kSearchWaves * 64), 0, s, d, query ? 1 : 0, rx0, ry0, rx1,
                           ry1, ntx, ntiles);
    }
    return hipGetLastError();
}

template <int R, bool DIRECT = false>
hipError_t launch_search_r(const JobDev &d, bool query, int rx0, int ry0, int rx1, int ry1, int tile_rows,
                           int ntx, int nty, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    switch (tile_rows) {
        case 4: return launch_search_t<R, 4, DIRECT>(d, query, rx0, ry0, rx1, ry1, ntx, nty, s, e0, e1);
        case 8: return launch_search_t<R, 8, DIRECT>(d, query, rx0, ry0, rx1, ry1, ntx, nty, s, e0, e1);
        case 16: return launch_search_t<R, 16, DIRECT>(d, query, rx0, ry0, rx1, ry1, ntx, nty, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

template <int R>
hipError_t launch_search_batched_r(const JobDev *slots, const WorkItem *items, const int32_t *nitems,
                                   int tile_rows, int grid, hipStream_t s) {
    const dim3 g(grid), b(kSearchWaves * 64);
    switch (tile_rows) {
        case 4: hipLaunchKernelGGL((k_search_batched<R, 4>), g, b, 0, s, slots, items, nitems); break;
        case 8: hipLaunchKernelGGL((k_search_batched<R, 8>), g, b, 0, s, slots, items, nitems); break;
        case 16: hipLaunchKernelGGL((k_search_batched<R, 16>), g, b, 0, s, slots, items, nitems); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_search(const JobDev &d, bool query, int r, int rx0, int ry0, int rx1, int ry1,
                         int tile_rows, int ntx, int nty, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    switch (r) {
        case 1: return launch_search_r<1>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        case 2: return launch_search_r<2>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        case 3: return launch_search_r<3>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        case 4: return launch_search_r<4>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        case 5: return launch_search_r<5>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        case 6: return launch_search_r<6>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        case 7: return launch_search_r<7>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        case 8: return launch_search_r<8>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_search_direct(const JobDev &d, bool query, int r, int rx0, int ry0, int rx1, int ry1,
                                int tile_rows, int ntx, int nty, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    switch (r) {
        case 1: return launch_search_r<1, true>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        case 2: return launch_search_r<2, true>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        case 3: return launch_search_r<3, true>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        case 4: return launch_search_r<4, true>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        case 5: return launch_search_r<5, true>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        case 6: return launch_search_r<6, true>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        case 7: return launch_search_r<7, true>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        case 8: return launch_search_r<8, true>(d, query, rx0, ry0, rx1, ry1, tile_rows, ntx, nty, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_search_batched(const JobDev *slots, const WorkItem *items, const int32_t *nitems, int r,
                                 int tile_rows, int grid, hipStream_t s) {
    switch (r) {
        case 1: return launch_search_batched_r<1>(slots, items, nitems, tile_rows, grid, s);
        case 2: return launch_search_batched_r<2>(slots, items, nitems, tile_rows, grid, s);
        case 3: return launch_search_batched_r<3>(slots, items, nitems, tile_rows, grid, s);
        case 4: return launch_search_batched_r<4>(slots, items, nitems, tile_rows, grid, s);
        case 5: return launch_search_batched_r<5>(slots, items, nitems, tile_rows, grid, s);
        case 6: return launch_search_batched_r<6>(slots, items, nitems, tile_rows, grid, s);
        case 7: return launch_search_batched_r<7>(slots, items, nitems, tile_rows, grid, s);
        case 8: return launch_search_batched_r<8>(slots, items, nitems, tile_rows, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace inpaint
