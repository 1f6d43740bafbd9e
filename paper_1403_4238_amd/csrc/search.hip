// findBestPatch on gfx950: masked-SSD exemplar search with a fused argmin.
//
// For every valid candidate centre c of the search rectangle (whole patch in
// the image and in the original known region) the kernel evaluates
//     SSD(c) = sum over known target offsets o of sum over R,G,B of
//              (t(o) - I(c + o))^2                            (Eq. 4)
// exactly in 32-bit integers, as T2 - 2 X(c) + S(c) with
//     X(c) = sum_o m(o) <t(o), I(c+o)>,   S(c) = sum_o m(o) |I(c+o)|^2,
// where <.,.> is the dot product of two RGBX words (X = 0 in the target).
// Each known (offset, candidate) pair costs two v_dot4_u32_u8: one for the
// cross term and one (shared per source pixel) for the square.
//
// Work decomposition: a work-group of 4 waves owns a 64-column x (4*NY)-row
// tile of candidate centres.  The source pixels of the tile plus its r-pixel
// halo are staged once in LDS as RGBX words.  Lane l of wave w handles the
// column x0 + l and NY consecutive rows; for each dx it loads the NY + 2r
// source words of its column once and reuses each for every (dy, candidate)
// pair that needs it.  The known-offset mask is uniform across the wave, so
// masked offsets are skipped with scalar branches and cost nothing.  Scores
// are reduced to one key (ssd << 32 | raster index) per tile: the minimum key
// is the (ssd, index)-lexicographic minimum, i.e. ties go to the lowest
// raster index.  No SSD array is ever written.
#include <hip/hip_ext.h>

#include "inpaint_dev.h"

namespace inpaint {

namespace {

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

// The target patch is read-only for the whole search and uniform across the
// wave; reading it through the constant address space lets the compiler use
// scalar loads into SGPRs instead of a vector memory round trip per offset.
typedef const __attribute__((address_space(4))) TargetStage ConstTarget;

template <int R, int NY>
struct TileGeom {
    static constexpr int P = 2 * R + 1;
    static constexpr int TH = kSearchWaves * NY;
    static constexpr int LW = kTileW + 2 * R;
    static constexpr int LH = TH + 2 * R;
    static constexpr int LDS_WORDS = LW * LH;
};

// Scores one tile and writes its minimum key to out[tile].
template <int R, int NY>
__device__ __forceinline__ void search_tile(const JobDev &d, const TargetStage *tg_generic,
                                            int rx0, int ry0, int rx1, int ry1, int ntx, int tile,
                                            uint64_t *__restrict__ out, uint32_t *lds,
                                            uint64_t *red) {
    using G = TileGeom<R, NY>;
    ConstTarget *tg = (ConstTarget *)tg_generic;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tx0 = rx0 + (tile % ntx) * kTileW;
    const int ty0 = ry0 + (tile / ntx) * G::TH;
    const int W = d.W, H = d.H;
    const int x = tx0 + lane;
    const int yb = ty0 + wave * NY;

    // Validity of this thread's candidates and the tile staging (the tile
    // plus its halo: rows ty0-R .., columns tx0-R ..) are loaded together;
    // one barrier then publishes the LDS tile and tells whether any
    // candidate of the tile is valid.
    uint32_t vmask = 0;
    if (x < rx1) {
#pragma unroll
        for (int i = 0; i < NY; ++i) {
            const int y = yb + i;
            if (y < ry1 && d.vrad[(int64_t)y * W + x] >= R) vmask |= 1u << i;
        }
    }
    for (int i = tid; i < G::LDS_WORDS; i += kSearchWaves * 64) {
        const int ly = i / G::LW, lx = i - ly * G::LW;
        const int gx = tx0 - R + lx, gy = ty0 - R + ly;
        uint32_t v = 0;
        if ((unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H) v = d.img[(int64_t)gy * W + gx];
        lds[i] = v;
    }
    if (!__syncthreads_or(vmask != 0)) {
        if (tid == 0) out[tile] = ~0ull;
        return;
    }

    uint32_t A[NY], B[NY];
#pragma unroll
    for (int i = 0; i < NY; ++i) {
        A[i] = 0;
        B[i] = 0;
    }
    uint32_t mb[(G::P * G::P + 31) / 32];
#pragma unroll
    for (int w = 0; w < (G::P * G::P + 31) / 32; ++w) mb[w] = tg->mbits[w];
    const uint32_t *colp = lds + wave * NY * G::LW + lane;
#pragma unroll
    for (int dxi = 0; dxi < G::P; ++dxi) {
        // This column's target words, loaded unconditionally (scalar loads).
        uint32_t tcol[G::P];
#pragma unroll
        for (int dyi = 0; dyi < G::P; ++dyi) tcol[dyi] = tg->tpix[dxi * G::P + dyi];
        uint32_t col[NY + 2 * R], sq[NY + 2 * R];
#pragma unroll
        for (int j = 0; j < NY + 2 * R; ++j) {
            col[j] = colp[j * G::LW + dxi];
            sq[j] = __builtin_amdgcn_udot4(col[j], col[j], 0u, false);
        }
#pragma unroll
        for (int dyi = 0; dyi < G::P; ++dyi) {
            const int slot = dxi * G::P + dyi;
            if (mb[slot >> 5] & (1u << (slot & 31))) {
                const uint32_t t = tcol[dyi];
#pragma unroll
                for (int i = 0; i < NY; ++i) {
                    A[i] = __builtin_amdgcn_udot4(t, col[i + dyi], A[i], false);
                    B[i] += sq[i + dyi];
                }
            }
        }
    }

    const uint32_t t2 = tg->t2;
    uint64_t best = ~0ull;
#pragma unroll
    for (int i = 0; i < NY; ++i) {
        if (vmask & (1u << i)) {
            const uint32_t ssd = t2 - 2u * A[i] + B[i];
            const uint64_t key = ((uint64_t)ssd << 32) | (uint32_t)((yb + i) * W + x);
            best = key < best ? key : best;
        }
    }
    best = wave_min_u64(best);
    if (lane == 0) red[wave] = best;
    __syncthreads();
    if (tid == 0) {
        uint64_t b = red[0];
#pragma unroll
        for (int w = 1; w < kSearchWaves; ++w) b = red[w] < b ? red[w] : b;
        out[tile] = b;
    }
}

// Consecutive work-groups are dispatched round-robin over the 8 XCDs; remap
// so that each XCD scores one contiguous band of tiles and keeps that band
// of the image resident in its own L2 across searches.
__device__ __forceinline__ int xcd_band_tile(int bid, int grid) {
    const int per = grid >> 3;
    return (bid & 7) * per + (bid >> 3);
}

template <int R, int NY>
__global__ __launch_bounds__(kSearchWaves * 64) void k_search(JobDev d, int query, int rx0, int ry0,
                                                              int rx1, int ry1, int ntx, int ntiles) {
    using G = TileGeom<R, NY>;
    __shared__ uint32_t lds[G::LDS_WORDS];
    __shared__ uint64_t red[kSearchWaves];
    if (!query) {
        const IterState *st = d.st;
        if (st->done || st->error || !st->pending || st->iter >= st->iter_limit) return;
    }
    const int tile = xcd_band_tile((int)blockIdx.x, (int)gridDim.x);
    if (tile >= ntiles) return;
    search_tile<R, NY>(d, query ? d.qtgt : d.tgt, rx0, ry0, rx1, ry1, ntx, tile, d.partials, lds, red);
}

// Persistent form over many images: work-groups stride over a static list of
// (image slot, tile) items; finished images cost one state read per item.
template <int R, int NY>
__global__ __launch_bounds__(kSearchWaves * 64) void k_search_batched(const JobDev *slots,
                                                                      const WorkItem *items,
                                                                      const int32_t *nitems) {
    using G = TileGeom<R, NY>;
    __shared__ uint32_t lds[G::LDS_WORDS];
    __shared__ uint64_t red[kSearchWaves];
    const int n = *nitems;
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const WorkItem w = items[it];
        const JobDev &d = slots[w.slot];
        const IterState *st = d.st;
        const bool live = st && !st->done && !st->error && st->pending && st->iter < st->iter_limit;
        if (live)
            search_tile<R, NY>(d, d.tgt, d.rx0, d.ry0, d.rx1, d.ry1, d.ntx, w.tile, d.partials, lds, red);
        __syncthreads();
    }
}

template <int R, int NY>
hipError_t launch_search_t(const JobDev &d, bool query, int rx0, int ry0, int rx1, int ry1, int ntx,
                           int nty, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
    const int ntiles = ntx * nty;
    if (ntiles <= 0) return hipSuccess;
    const int grid = (ntiles + 7) / 8 * 8;
    if (start) {
        // The runtime stamps these events with the kernel's own begin / end.
        hipExtLaunchKernelGGL((k_search<R, NY>), dim3(grid), dim3(kSearchWaves * 64), 0, s, start, stop, 0, d,
                              query ? 1 : 0, rx0, ry0, rx1, ry1, ntx, ntiles);
    } else {
        hipLaunchKernelGGL((k_search<R, NY>), dim3(grid), dim3(kSearchWaves * 64), 0, s, d, query ? 1 : 0, rx0,
                           ry0, rx1, ry1, ntx, ntiles);
    }
    return hipGetLastError();
}

template <int R>
hipError_t launch_search_r(const JobDev &d, bool query, int rx0, int ry0, int rx1, int ry1, int tile_rows,
                           int ntx, int nty, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    switch (tile_rows) {
        case 4: return launch_search_t<R, 4>(d, query, rx0, ry0, rx1, ry1, ntx, nty, s, e0, e1);
        case 8: return launch_search_t<R, 8>(d, query, rx0, ry0, rx1, ry1, ntx, nty, s, e0, e1);
        case 16: return launch_search_t<R, 16>(d, query, rx0, ry0, rx1, ry1, ntx, nty, s, e0, e1);
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
