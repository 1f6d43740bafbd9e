// findBestPatch on the gfx950 matrix cores: the masked SSD (Eq. 4) as exact
// int8 MFMA arithmetic with int32 accumulation.
//
// In the offset-by-128 domain (t' = t - 128, s' = s - 128, which leaves every
// difference unchanged) the masked SSD of candidate c is
//     SSD(c) = T2' - 2 X'(c) + S'(c),
//     X'(c) = sum_o m(o) <t'(o), s'(c+o)>          (cross term)
//     S'(c) = sum_o m(o) |s'(c+o)|^2                (masked square term)
// with T2' = sum_o m(o) |t'(o)|^2 a per-target constant.  All operands are
// int8 and all sums fit in int32, so the result is exact.
//
// A wave owns 16x16 candidate tiles.  For each patch row dy, the cross term of
// a tile is a 16 x 96 by 96 x 16 product: the A rows are the 16 candidate rows
// shifted by dy, each holding 24 consecutive source pixels (RGBX bytes); B is
// the banded Toeplitz matrix of the target's row dy, B[(x, ch)][n] =
// m t'(x - n - r, dy, ch) for 0 <= x - n <= 2r.  That is two
// v_mfma_i32_16x16x64_i8 per dy.  The square term uses the same banded mask
// against per-pixel planes of the low and high byte of |s'|^2 (two more
// MFMAs).  The B operands depend only on the target: each work-group builds
// them as shifted tables in LDS from the 1.3 KB staged target (words and
// known mask) and every wave reads one patch row's operands at a time; the
// A fragments are 16-byte LDS reads from the staged tile.
//
// The planes are static (candidate windows lie in the original known
// region, which never changes) and zero-padded, and the tiling starts on a
// column that puts every staged window on an 8-pixel boundary: a tile is
// staged with unconditional 16-byte loads, issued together with the
// candidates' validity radii and the staged target before the first wait.
#include <hip/hip_ext.h>

#include "search_mfma_tile.h"

namespace inpaint {

namespace {

using namespace mtile;

template <int R>
struct MfmaLds {
    MfmaTile<R> tile;
    FragTables<R> ft;
    uint64_t red[kSearchWaves];
};

// Pass 1 of the B-operand tables from a staged target (words and known mask
// in column-major slot order); the caller's barrier publishes it.
template <int R>
__device__ __forceinline__ void build_patch_from(const TargetStage *tg, FragTables<R> *ft) {
    build_patch<R>(
        ft, [&](int sl) { return tg->tpix[sl]; }, [&](int sl) { return (tg->mbits[sl >> 5] >> (sl & 31)) & 1u; });
}

// Stages and scores tile t against the target whose B-operand tables are
// built here from its 1.3 KB stage (build = true) or are already in L.ft
// (the previous tile of this work-group had the same target).
template <int R>
__device__ __forceinline__ void search_tile_mfma(const JobDev &d, const TargetStage *tg, bool build, bool live,
                                                 int rx0, int ry0, int rx1, int ry1, int ntx, int t, uint64_t *out,
                                                 MfmaLds<R> &L) {
    int tx0, ty0;
    tile_origin<R>(rx0, ry0, ntx, t, &tx0, &ty0);
    if (build) build_patch_from<R>(tg, &L.ft);   // its loads in flight with the tile's
    const uint32_t vmask = stage_tile<R>(d, tx0, ty0, rx0, rx1, ry1, L.tile);
    // one barrier publishes the tile (and pass 1) and tells whether any
    // candidate is valid
    if (!__syncthreads_or(live && vmask != 0)) {
        if (build) {
            build_tables<R>(&L.ft);   // (every thread reaches this branch: keeps the tables whole)
            __syncthreads();
        }
        if (threadIdx.x == 0 && live) out[t] = ~0ull;
        return;
    }
    if (build) {
        build_tables<R>(&L.ft);
        __syncthreads();
    }
    const uint64_t best = tile::wave_min_u64(score_tile_rows<R>(d, &L.ft, tx0, ty0, vmask, L.tile));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) L.red[wave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t m = L.red[0];
#pragma unroll
        for (int w = 1; w < kSearchWaves; ++w) m = L.red[w] < m ? L.red[w] : m;
        out[t] = m;
    }
}

__device__ __forceinline__ int xcd_band_tile(int bid, int grid) {
    const int per = grid >> 3;
    return (bid & 7) * per + (bid >> 3);
}

template <int R>
__global__ __launch_bounds__(kSearchWaves * 64) void k_search_mfma(JobDev d, int query, int rx0, int ry0, int rx1,
                                                                   int ry1, int ntx, int ntiles) {
    __shared__ MfmaLds<R> L;
    const int tile = xcd_band_tile((int)blockIdx.x, (int)gridDim.x);
    if (tile >= ntiles) return;
    // read now, tested after the tile loads are issued
    bool live = true;
    if (!query) {
        const IterState *st = d.st;
        live = !(st->done || st->error || !st->pending || st->iter >= st->iter_limit);
    }
    search_tile_mfma<R>(d, query ? d.qtgt : d.tgt, true, live, rx0, ry0, rx1, ry1, ntx, tile, d.partials, L);
}

// Persistent form over many images (the batch's graph form): work-groups
// take runs of a static list of (image slot, tile) items; each image's B
// tables come from its staged target.
template <int R>
__global__ __launch_bounds__(kSearchWaves * 64) void k_search_batched_mfma(const JobDev *slots,
                                                                           const WorkItem *items,
                                                                           const int32_t *nitems) {
    __shared__ MfmaLds<R> L;
    const int n = *nitems;
    // each work-group takes a contiguous run of the (slot-ordered) items, so
    // consecutive tiles mostly share a target and its B tables are built
    // once per run of that slot
    const int per = (n + (int)gridDim.x - 1) / (int)gridDim.x;
    const int i0 = (int)blockIdx.x * per, i1 = min(n, i0 + per);
    int built = -1;   // slot whose target's tables are in L.ft
    for (int it = i0; it < i1; ++it) {
        const WorkItem w = items[it];
        const JobDev &d = slots[w.slot];
        const IterState *st = d.st;
        const bool live = st && !st->done && !st->error && st->pending && st->iter < st->iter_limit;
        if (live) {
            search_tile_mfma<R>(d, d.tgt, built != w.slot, true, d.rx0, d.ry0, d.rx1, d.ry1, d.ntx, w.tile,
                                d.partials, L);
            built = w.slot;
        }
        __syncthreads();
    }
}

template <int R>
hipError_t launch_mfma_t(const JobDev &d, bool query, int rx0, int ry0, int rx1, int ry1, int ntx, int nty,
                         hipStream_t s, hipEvent_t start, hipEvent_t stop) {
    const int ntiles = ntx * nty;
    if (ntiles <= 0) return hipSuccess;
    const int grid = (ntiles + 7) / 8 * 8;
    if (start)
        hipExtLaunchKernelGGL((k_search_mfma<R>), dim3(grid), dim3(kSearchWaves * 64), 0, s, start, stop, 0, d,
                              query ? 1 : 0, rx0, ry0, rx1, ry1, ntx, ntiles);
    else
        hipLaunchKernelGGL((k_search_mfma<R>), dim3(grid), dim3(kSearchWaves * 64), 0, s, d, query ? 1 : 0, rx0,
                           ry0, rx1, ry1, ntx, ntiles);
    return hipGetLastError();
}

// Static source planes of the MFMA search in the padded layout, from the
// original image: offset RGBX words and the |s'|^2 byte pair (zero outside
// the image).  Only original known pixels are ever read by a valid
// candidate, and those never change.
__global__ __launch_bounds__(256) void k_mfma_planes(JobDev d) {
    const int pitch = d.pitch;
    const int64_t n = (int64_t)pitch * padded_rows(d.H);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = (int)(i % pitch) - kPadL, y = (int)(i / pitch) - kPadT;
    uint32_t w = 0;
    uint16_t q = 0;
    if (x >= 0 && x < d.W && y >= 0 && y < d.H) {
        const uint32_t v = d.img[(int64_t)y * d.W + x];
        w = v ^ 0x80808080u;
        q = sq_bytes(v);
    }
    d.srcw[i] = w;
    d.srcq[i] = q;
}

}  // namespace

hipError_t launch_mfma_planes(const JobDev &d, hipStream_t s) {
    const int64_t n = (int64_t)d.pitch * padded_rows(d.H);
    hipLaunchKernelGGL(k_mfma_planes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d);
    return hipGetLastError();
}

bool mfma_supported(int r) { return r >= 1 && r <= kMfmaMaxRadius; }

hipError_t launch_search_batched_mfma(const JobDev *slots, const WorkItem *items, const int32_t *nitems, int r,
                                      int grid, hipStream_t s) {
#define CALL(R) hipLaunchKernelGGL(k_search_batched_mfma<R>, dim3(grid), dim3(kSearchWaves * 64), 0, s, slots, items, nitems)
    switch (r) {
        case 1: CALL(1); break;
        case 2: CALL(2); break;
        case 3: CALL(3); break;
        case 4: CALL(4); break;
        case 5: CALL(5); break;
        case 6: CALL(6); break;
        default: return hipErrorInvalidValue;
    }
#undef CALL
    return hipGetLastError();
}

hipError_t launch_search_mfma(const JobDev &d, bool query, int r, int rx0, int ry0, int rx1, int ry1, int ntx, int nty,
                              hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    switch (r) {
        case 1: return launch_mfma_t<1>(d, query, rx0, ry0, rx1, ry1, ntx, nty, s, e0, e1);
        case 2: return launch_mfma_t<2>(d, query, rx0, ry0, rx1, ry1, ntx, nty, s, e0, e1);
        case 3: return launch_mfma_t<3>(d, query, rx0, ry0, rx1, ry1, ntx, nty, s, e0, e1);
        case 4: return launch_mfma_t<4>(d, query, rx0, ry0, rx1, ry1, ntx, nty, s, e0, e1);
        case 5: return launch_mfma_t<5>(d, query, rx0, ry0, rx1, ry1, ntx, nty, s, e0, e1);
        case 6: return launch_mfma_t<6>(d, query, rx0, ry0, rx1, ry1, ntx, nty, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace inpaint
