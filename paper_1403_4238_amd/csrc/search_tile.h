// Exemplar-search tile (findBestPatch on gfx950): staging of a candidate
// tile and its masked-SSD scoring, shared by the one-search-per-launch
// kernels and the persistent fill kernel.
//
// For every valid candidate centre c of the search rectangle (whole patch in
// the image and in the original known region) the SSD of Eq. 4 is evaluated
// exactly in 32-bit integers as T2 - 2 X(c) + S(c) with
//     X(c) = sum_o m(o) <t(o), I(c+o)>,   S(c) = sum_o m(o) |I(c+o)|^2,
// where <.,.> is the dot product of two RGBX words (X = 0 in the target).
// The cross term costs one v_dot4_u32_u8 per (known offset, candidate).  The
// square term is taken from running sums down each patch column: with
// Q_j = sum_{j' < j} |s_j'|^2 over the source words a lane holds for one
// column, a run of known offsets dy = a..b adds Q_{i+b+1} - Q_{i+a} to
// candidate row i, so S costs two adds per (column run, candidate) instead of
// one per known offset, and the Q_j take one dot4-accumulate each.
//
// A work-group of 4 waves owns a 64-column x (4*NY)-row tile of candidate
// centres.  Candidate windows lie in the original known region, whose pixels
// never change, so the search reads a static copy of the image in a
// zero-padded plane: the tile plus its r-pixel halo is staged into LDS with
// unconditional 16-byte loads, all issued before the first wait, together
// with the validity radii of the candidates.  Lane l of wave w handles
// column x0 + l and NY consecutive rows; for each dx it reads the NY + 2r
// source words of its column once and reuses each for every (dy, candidate)
// pair that needs it.  The masks are uniform across the wave, so masked
// offsets are skipped with scalar branches and cost nothing.  (score_direct
// runs the same scoring reading the plane in device memory instead of the
// LDS tile, for the comparison with a search without local memory.)  Scores reduce
// to keys (ssd << 32 | raster index): the minimum key is the
// (ssd, index)-lexicographic minimum, i.e. ties go to the lowest raster
// index.  No SSD array is ever written.
#pragma once

#include "inpaint_dev.h"

namespace inpaint {

// ---- wave-wide folds on DPP lane moves (VALU only: no LDS round trip per
// step as with shuffles).  Rows of 16 lanes fold by row_shr 1, 2, 4 and 8,
// which leaves each row's fold in its lane 15; row_bcast 15 then folds row
// 2 into lane 63 (and row 0 into lane 31), and row_bcast 31 folds lane 31
// into lane 63, which readlane hands to every lane.  A lane whose source
// lies outside the wave or before the start of its row reads 0, so every
// fold here is one with identity 0 (values are re-encoded where needed);
// no identity registers are tied to the moves.  Lanes other than 63 end with
// partial folds.  Every lane of the wave must be active.
namespace dpp {
constexpr int kShr1 = 0x111, kShr2 = 0x112, kShr4 = 0x114, kShr8 = 0x118, kBcast15 = 0x142, kBcast31 = 0x143;

template <int CTRL>
__device__ __forceinline__ uint32_t mov(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, true);
}
template <int CTRL>
__device__ __forceinline__ uint64_t mov(uint64_t v) {
    return (uint64_t)mov<CTRL>((uint32_t)v) | (uint64_t)mov<CTRL>((uint32_t)(v >> 32)) << 32;
}
__device__ __forceinline__ uint32_t lane63(uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, 63); }
__device__ __forceinline__ uint64_t lane63(uint64_t v) { return (uint64_t)lane63((uint32_t)v) | (uint64_t)lane63((uint32_t)(v >> 32)) << 32; }

// Row folds: lane 15 of each 16-lane row ends with its row's fold.
template <class T, class Op>
__device__ __forceinline__ T fold_rows(T v, Op op) {
    v = op(v, mov<kShr1>(v));
    v = op(v, mov<kShr2>(v));
    v = op(v, mov<kShr4>(v));
    v = op(v, mov<kShr8>(v));
    return v;
}
// Wave fold, in every lane.
template <class T, class Op>
__device__ __forceinline__ T fold_wave(T v, Op op) {
    v = fold_rows(v, op);
    v = op(v, mov<kBcast15>(v));
    v = op(v, mov<kBcast31>(v));
    return lane63(v);
}
__device__ __forceinline__ uint64_t min_u64(uint64_t v) {   // as the maximum of the complements
    return ~fold_wave(~v, [](uint64_t a, uint64_t b) { return b > a ? b : a; });
}
__device__ __forceinline__ uint32_t sum_u32(uint32_t v) {
    return fold_wave(v, [](uint32_t a, uint32_t b) { return a + b; });
}
__device__ __forceinline__ uint32_t or_u32(uint32_t v) {
    return fold_wave(v, [](uint32_t a, uint32_t b) { return a | b; });
}
}  // namespace dpp

namespace tile {

// The target patch is read-only for a whole search and uniform across the
// wave; reading it through the constant address space lets the compiler use
// scalar loads into SGPRs instead of a vector memory round trip per offset.
// (Only valid while the target cannot change during the dispatch.)
typedef const __attribute__((address_space(4))) TargetStage ConstTarget;

struct ScalarTarget {
    ConstTarget *tg;
    __device__ uint32_t pix(int slot) const { return tg->tpix[slot]; }
    __device__ uint32_t known(int w) const { return tg->mbits[w]; }
    __device__ uint32_t starts(int w) const { return tg->sbits[w]; }
    __device__ uint32_t ends(int w) const { return tg->ebits[w]; }
    __device__ uint32_t t2() const { return tg->t2; }
};

// A copy of the target in LDS, for kernels that search several targets in
// one dispatch: words are read back with broadcast LDS loads, mask words are
// moved to SGPRs so the offset loop still branches on scalars.
struct TargetLds {
    uint32_t tpix[kMaxOffsets + 15];
    uint32_t mbits[16], sbits[16], ebits[16];
    uint32_t t2, pad[3];
};

struct LdsTarget {
    const TargetLds *t;
    __device__ uint32_t pix(int slot) const { return t->tpix[slot]; }
    __device__ uint32_t known(int w) const { return __builtin_amdgcn_readfirstlane(t->mbits[w]); }
    __device__ uint32_t starts(int w) const { return __builtin_amdgcn_readfirstlane(t->sbits[w]); }
    __device__ uint32_t ends(int w) const { return __builtin_amdgcn_readfirstlane(t->ebits[w]); }
    __device__ uint32_t t2() const { return __builtin_amdgcn_readfirstlane(t->t2); }
};

// Copies the staged target of radius R into LDS (whole work-group; the
// caller publishes it with a barrier).
template <int R>
__device__ __forceinline__ void load_target(const TargetStage *tg, TargetLds *t) {
    constexpr int P = 2 * R + 1, MW = (P * P + 31) / 32;
    for (int i = threadIdx.x; i < P * P; i += blockDim.x) t->tpix[i] = tg->tpix[i];
    if (threadIdx.x < MW) {
        t->mbits[threadIdx.x] = tg->mbits[threadIdx.x];
        t->sbits[threadIdx.x] = tg->sbits[threadIdx.x];
        t->ebits[threadIdx.x] = tg->ebits[threadIdx.x];
    }
    if (threadIdx.x == 0) t->t2 = tg->t2;
}

// Smallest validity-plane value of a candidate centre: the patch radius
// (its whole window is source) or, with INTERSECT scoring, 1 (the centre
// itself is a source pixel).
template <int R, bool ISECT>
__device__ __forceinline__ constexpr uint32_t valid_min() {
    return ISECT ? 1u : (uint32_t)R;
}

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

// Tile origin of tile index `tile` in a rect starting at (rx0, ry0).
template <int R, int NY>
__device__ __forceinline__ void tile_origin(int rx0, int ry0, int ntx, int tile, int *tx0, int *ty0) {
    *tx0 = rx0 + (tile % ntx) * kTileW;
    *ty0 = ry0 + (tile / ntx) * TileGeom<R, NY>::TH;
}

// Issues every load of the tile at (tx0, ty0) before any wait -- the staged
// window (padded rows ty0 - R + kPadT .., columns from the 16-byte boundary
// at or below tx0 - R + kPadL) and the validity radii of this lane's rows --
// then writes the window to LDS.  Returns this thread's candidate validity
// bits (bit i: row i of its column); the caller publishes the LDS tile with
// a barrier.
template <int R, int NY, bool ISECT = false>
__device__ __forceinline__ uint32_t stage_tile(const JobDev &d, int tx0, int ty0, int rx1, int ry1, uint32_t *lds) {
    using G = TileGeom<R, NY>;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int pitch = d.pitch;
    const int x = tx0 + lane, yb = ty0 + wave * NY;
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

    uint4 *lds4 = (uint4 *)lds;
#pragma unroll
    for (int k = 0; k < G::QIT; ++k) lds4[min(tid + k * kSearchWaves * 64, G::NQ - 1)] = q[k];
    uint32_t vmask = 0;
#pragma unroll
    for (int i = 0; i < NY; ++i)
        if (x < rx1 && yb + i < ry1 && v[i] >= valid_min<R, ISECT>()) vmask |= 1u << i;
    return vmask;
}

// Validity bits of this thread's candidates (bit i: row i of its column) for
// the tile at (tx0, ty0), without staging the tile.
template <int R, int NY, bool ISECT = false>
__device__ __forceinline__ uint32_t tile_valid(const JobDev &d, int tx0, int ty0, int rx1, int ry1) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = tx0 + lane, yb = ty0 + wave * NY;
    const uint8_t *vr = d.vradp + (int64_t)(yb + kPadT) * d.pitch + (x + kPadL);
    uint32_t v[NY];
#pragma unroll
    for (int i = 0; i < NY; ++i) v[i] = vr[i * d.pitch];
    uint32_t vmask = 0;
#pragma unroll
    for (int i = 0; i < NY; ++i)
        if (x < rx1 && yb + i < ry1 && v[i] >= valid_min<R, ISECT>()) vmask |= 1u << i;
    return vmask;
}

// Scores this thread's candidates against target view T and returns their
// minimum key (~0 if none is valid).  `colp` points at the source word of
// this lane's column for offset (-R, -R) of its first candidate row;
// consecutive rows are `stride` words apart.
//
// With INTERSECT scoring an offset counts only where the source pixel is a
// source pixel too, flagged by the 4th byte of its word (1, else the word is
// 0).  The cross and square terms need no change, because non-source words
// are zero (the flag byte is masked out of the square term).  The target
// term becomes per candidate: the sum of |t|^2 times the flag over the
// target's known offsets.
template <int R, int NY, bool ISECT, class T>
__device__ __forceinline__ uint64_t score_cols(const JobDev &d, const T &tg, int tx0, int ty0, uint32_t vmask,
                                               const uint32_t *colp, int stride) {
    using G = TileGeom<R, NY>;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int W = d.W;
    const int x = tx0 + lane, yb = ty0 + wave * NY;

    uint32_t A[NY], S[NY], T2[NY];
#pragma unroll
    for (int i = 0; i < NY; ++i) {
        A[i] = 0;
        S[i] = 0;
        T2[i] = 0;
    }
    uint32_t mb[G::MW], sb[G::MW], eb[G::MW];
#pragma unroll
    for (int w = 0; w < G::MW; ++w) {
        mb[w] = tg.known(w);
        sb[w] = tg.starts(w);
        eb[w] = tg.ends(w);
    }
#pragma unroll
    for (int dxi = 0; dxi < G::P; ++dxi) {
        // This column's target words, loaded unconditionally.
        uint32_t tcol[G::P];
#pragma unroll
        for (int dyi = 0; dyi < G::P; ++dyi) tcol[dyi] = tg.pix(dxi * G::P + dyi);
        uint32_t col[G::NJ], pre[G::NJ + 1];
        pre[0] = 0;
#pragma unroll
        for (int j = 0; j < G::NJ; ++j) {
            col[j] = colp[j * stride + dxi];
            const uint32_t c3 = ISECT ? (col[j] & 0x00ffffffu) : col[j];
            pre[j + 1] = __builtin_amdgcn_udot4(c3, c3, pre[j], false);
        }
#pragma unroll
        for (int dyi = 0; dyi < G::P; ++dyi) {
            const int slot = dxi * G::P + dyi;
            const uint32_t bit = 1u << (slot & 31);
            if (mb[slot >> 5] & bit) {
                const uint32_t t = tcol[dyi];
#pragma unroll
                for (int i = 0; i < NY; ++i) A[i] = __builtin_amdgcn_udot4(t, col[i + dyi], A[i], false);
                if (ISECT) {
                    const uint32_t tsq = __builtin_amdgcn_udot4(t, t, 0u, false);
#pragma unroll
                    for (int i = 0; i < NY; ++i) T2[i] += (col[i + dyi] >> 24) * tsq;
                }
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

    const uint32_t t2 = tg.t2();
    uint64_t best = ~0ull;
#pragma unroll
    for (int i = 0; i < NY; ++i) {
        if (vmask & (1u << i)) {
            const uint32_t ssd = (ISECT ? T2[i] : t2) - 2u * A[i] + S[i];
            const uint64_t key = ((uint64_t)ssd << 32) | (uint32_t)((yb + i) * W + x);
            best = key < best ? key : best;
        }
    }
    return best;
}

// Scores a tile staged in LDS by stage_tile.
template <int R, int NY, class T, bool ISECT = false>
__device__ __forceinline__ uint64_t score_tile(const JobDev &d, const T &tg, int tx0, int ty0, uint32_t vmask,
                                               const uint32_t *lds) {
    using G = TileGeom<R, NY>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sh = (tx0 - R + kPadL) & 3;
    return score_cols<R, NY, ISECT>(d, tg, tx0, ty0, vmask, lds + wave * NY * G::LW + lane + sh, G::LW);
}

// Scores the tile straight from the padded source plane in device memory
// (through the vector caches), with no LDS staging.  The words read are a
// subset of the window stage_tile loads, so the plane's padding covers them.
template <int R, int NY, class T, bool ISECT = false>
__device__ __forceinline__ uint64_t score_direct(const JobDev &d, const T &tg, int tx0, int ty0, uint32_t vmask) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = tx0 + lane, yb = ty0 + wave * NY;
    const uint32_t *colp = d.srcp + (int64_t)(yb - R + kPadT) * d.pitch + (x - R + kPadL);
    return score_cols<R, NY, ISECT>(d, tg, tx0, ty0, vmask, colp, d.pitch);
}

// Minimum over the wave.  (Kept out of score_tile: inlined there it makes
// the register allocator copy the square-term accumulators at every branch.)
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) { return dpp::min_u64(v); }

}  // namespace tile
}  // namespace inpaint
