// findBestPatch on gfx950: masked-SSD exemplar search with a fused argmin.
//
// For every valid candidate centre c of the search rectangle (whole patch in
// the image and in the original known region) the kernel evaluates
//     SSD(c) = sum over known target offsets o of sum over R,G,B of
//              (t(o) - I(c + o))^2                            (Eq. 4)
// exactly in 32-bit integers, as T2 - 2 X(c) + S(c) with
//     X(c) = sum_o m(o) <t(o), I(c+o)>,   S(c) = sum_o m(o) |I(c+o)|^2,
// where <.,.> is the dot product of two RGBX words (X = 0 in the target).
// The cross term costs one v_dot4_u32_u8 per (known offset, candidate).  The
// square term is taken from running sums down each patch column: with
// Q_j = sum_{j' < j} |s_j'|^2 over the source words a lane holds for one
// column, a run of known offsets dy = a..b adds Q_{i+b+1} - Q_{i+a} to
// candidate row i, so S costs two adds per (column run, candidate) instead of
// one per known offset, and the Q_j take one dot4-accumulate each.
//
// Work decomposition: a work-group of 4 waves owns a 64-column x (4*NY)-row
// tile of candidate centres.  Candidate windows lie in the original known
// region, whose pixels never change, so the search reads a static copy of
// the image in a zero-padded plane: the tile plus its r-pixel halo is staged
// into LDS with unconditional 16-byte loads, all issued before the first
// wait, together with the validity radii of the candidates.  Lane l of wave
// w handles column x0 + l and NY consecutive rows; for each dx it reads the
// NY + 2r source words of its column once and reuses each for every
// (dy, candidate) pair that needs it.  The masks are uniform across the
// wave, so masked offsets are skipped with scalar branches and cost nothing.
// Scores are reduced to one key (ssd << 32 | raster index) per tile: the
// minimum key is the (ssd, index)-lexicographic minimum, i.e. ties go to the
// lowest raster index.  No SSD array is ever written.
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
    static constexpr int NJ = NY + 2 * R;                       // source rows per lane and column
    static constexpr int LW = (kTileW + 2 * R + 3 + 3) / 4 * 4;  // staged words per row, from a 16-byte boundary
    static constexpr int LQ = LW / 4;
    static constexpr int LH = TH + 2 * R;
    static constexpr int NQ = LQ * LH;                           // 16-byte quads per staged tile
    static constexpr int QIT = (NQ + kSearchWaves * 64 - 1) / (kSearchWaves * 64);
    static constexpr int LDS_WORDS = LW * LH;
    static constexpr int MW = (P * P + 31) / 32;
};

// Scores one tile and writes its minimum key to out[tile].  `live` (uniform)
// is false when the fill loop has nothing pending: the tile is then staged
// but neither scored nor written.
template <int R, int NY>
__device__ __forceinline__ void search_tile(const JobDev &d, const TargetStage *tg_generic, bool live,
                                            int rx0, int ry0, int rx1, int ry1, int ntx, int tile,
                                            uint64_t *__restrict__ out, uint32_t *lds, uint64_t *red) {
    using G = TileGeom<R, NY>;
    ConstTarget *tg = (ConstTarget *)tg_generic;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tx0 = rx0 + (tile % ntx) * kTileW;
    const int ty0 = ry0 + (tile / ntx) * G::TH;
    const int W = d.W, pitch = d.pitch;
    const int x = tx0 + lane;
    const int yb = ty0 + wave * NY;

    // ---- issue every load of the tile before any wait: the staged window
    // (padded rows ty0 - R + kPadT .., columns from the 16-byte boundary at
    // or below tx0 - R + kPadL) and the validity radii of this lane's rows.
    const int gx0 = tx0 - R + kPadL;
    const int sh = gx0 & 3;
    const uint4 *src4 = (const uint4 *)(d.srcp + (int64_t)(ty0 - R + kPadT) * pitch + (gx0 - sh));
    const int qpitch = pitch >> 2;
    uint4 q[G::QIT];
#pragma unroll
    for (int k = 0; k < G::QIT; ++k) {
        const int qi = min(tid + k * kSearchWaves * 64, G::NQ - 1);
        const int ly = qi / G::LQ, lq = qi - ly * G::LQ;
        q[k] = src4[ly * qpitch + lq];
    }
    const uint8_t *vr = d.vradp + (int64_t)(yb + kPadT) * pitch + (x + kPadL);
    uint32_t v[NY];
#pragma unroll
    for (int i = 0; i < NY; ++i) v[i] = vr[i * pitch];

    // ---- publish: one barrier makes the LDS tile visible and tells whether
    // any candidate of the tile is valid.
    uint4 *lds4 = (uint4 *)lds;
#pragma unroll
    for (int k = 0; k < G::QIT; ++k) lds4[min(tid + k * kSearchWaves * 64, G::NQ - 1)] = q[k];
    uint32_t vmask = 0;
#pragma unroll
    for (int i = 0; i < NY; ++i)
        if (x < rx1 && yb + i < ry1 && v[i] >= (uint32_t)R) vmask |= 1u << i;
    if (!__syncthreads_or(live && vmask != 0)) {
        if (tid == 0 && live) out[tile] = ~0ull;
        return;
    }

    uint32_t A[NY], S[NY];
#pragma unroll
    for (int i = 0; i < NY; ++i) {
        A[i] = 0;
        S[i] = 0;
    }
    uint32_t mb[G::MW], sb[G::MW], eb[G::MW];
#pragma unroll
    for (int w = 0; w < G::MW; ++w) {
        mb[w] = tg->mbits[w];
        sb[w] = tg->sbits[w];
        eb[w] = tg->ebits[w];
    }
    const uint32_t *colp = lds + wave * NY * G::LW + lane + sh;
#pragma unroll
    for (int dxi = 0; dxi < G::P; ++dxi) {
        // This column's target words, loaded unconditionally (scalar loads).
        uint32_t tcol[G::P];
#pragma unroll
        for (int dyi = 0; dyi < G::P; ++dyi) tcol[dyi] = tg->tpix[dxi * G::P + dyi];
        uint32_t col[G::NJ], pre[G::NJ + 1];
        pre[0] = 0;
#pragma unroll
        for (int j = 0; j < G::NJ; ++j) {
            col[j] = colp[j * G::LW + dxi];
            pre[j + 1] = __builtin_amdgcn_udot4(col[j], col[j], pre[j], false);
        }
#pragma unroll
        for (int dyi = 0; dyi < G::P; ++dyi) {
            const int slot = dxi * G::P + dyi;
            const uint32_t bit = 1u << (slot & 31);
            if (mb[slot >> 5] & bit) {
                const uint32_t t = tcol[dyi];
#pragma unroll
                for (int i = 0; i < NY; ++i) A[i] = __builtin_amdgcn_udot4(t, col[i + dyi], A[i], false);
            }
            // The empty volatile asm keeps these blocks behind their scalar
            // branches (instead of being speculated into selects).
            if (sb[slot >> 5] & bit) {
                asm volatile("");
#pragma unroll
                for (int i = 0; i < NY; ++i) S[i] -= pre[i + dyi];
            }
            if (eb[slot >> 5] & bit) {
                asm volatile("");
#pragma unroll
                for (int i = 0; i < NY; ++i) S[i] += pre[i + dyi + 1];
            }
        }
    }

    const uint32_t t2 = tg->t2;
    uint64_t best = ~0ull;
#pragma unroll
    for (int i = 0; i < NY; ++i) {
        if (vmask & (1u << i)) {
            const uint32_t ssd = t2 - 2u * A[i] + S[i];
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
    __shared__ __attribute__((aligned(16))) uint32_t lds[G::LDS_WORDS];
    __shared__ uint64_t red[kSearchWaves];
    const int tile = xcd_band_tile((int)blockIdx.x, (int)gridDim.x);
    if (tile >= ntiles) return;
    // The state is read here but tested only after the tile loads are
    // issued, so its latency overlaps theirs.
    bool live = true;
    if (!query) {
        const IterState *st = d.st;
        live = !(st->done || st->error || !st->pending || st->iter >= st->iter_limit);
    }
    search_tile<R, NY>(d, query ? d.qtgt : d.tgt, live, rx0, ry0, rx1, ry1, ntx, tile, d.partials, lds, red);
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
