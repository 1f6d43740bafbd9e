// Exact int8-MFMA exemplar-search tile on gfx950 (see search_mfma.hip for
// the arithmetic): staging of a 64 x 64 candidate tile, the B operands of a
// target, and the scoring loop, shared by the one-search-per-launch kernel
// and the persistent fill kernel.
#pragma once

#include "search_tile.h"

namespace inpaint {
namespace mtile {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kMfmaTilesPerWave = 4;                       // 16-row tiles stacked per wave
constexpr int kMfmaTileH = 16 * kMfmaTilesPerWave;          // 64 rows
constexpr int kMfmaStrideA = 100;                           // words per staged row (100 % 32 == 4)
constexpr int kMfmaStrideQ = 272;                           // bytes per |s'|^2 row (68 words, 68 % 32 == 4)

template <int R>
struct MfmaGeom {
    static constexpr int P = 2 * R + 1;
    static constexpr int ROWS = kMfmaTileH + 2 * R;
    static constexpr int COLS = kTileW + 2 * R;                 // staged columns that meet nonzero B entries
    static constexpr int QA = (COLS + 3) / 4;                   // 16-byte quads per row: RGBX words
    static constexpr int QQ = (2 * COLS + 15) / 16;             // 16-byte quads per row: |s'|^2 byte pairs
    static constexpr int NA = ROWS * QA, NQ = ROWS * QQ;
    static constexpr int AIT = (NA + kSearchWaves * 64 - 1) / (kSearchWaves * 64);
    static constexpr int QIT = (NQ + kSearchWaves * 64 - 1) / (kSearchWaves * 64);
};

// |s'|^2 of an RGBX word, split into (low byte - 128, high byte - 128) int8s
// packed as a 16-bit value (low byte first).
__device__ __forceinline__ uint16_t sq_bytes(uint32_t w) {
    const int r = (int)(w & 255) - 128, g = (int)((w >> 8) & 255) - 128, b = (int)((w >> 16) & 255) - 128;
    const int q = r * r + g * g + b * b;              // 0 .. 49152
    const int lo = (q & 255) - 128, hi = (q >> 8) - 128;
    return (uint16_t)((uint8_t)lo | ((uint32_t)(uint8_t)hi << 8));
}

template <int R>
struct MfmaTile {
    alignas(16) uint32_t a[MfmaGeom<R>::ROWS * kMfmaStrideA];      // RGBX ^ 0x80808080
    alignas(16) uint8_t q[MfmaGeom<R>::ROWS * kMfmaStrideQ + 32];  // (lo', hi') per pixel
};

// Per-target tables a work-group builds in LDS, from which every wave reads
// its B operands with a few aligned LDS loads.  With T(dy, x) the target
// word (RGB ^ 0x808080) at patch column x of row dy where known, 0 elsewhere
// (also outside 0 <= x < P), and M(dy, x) its 0/1 known flag:
// tc[s][dy][i] = T(dy, i - 16 - s), so the four words lane (n, g) needs,
// T(dy, 16 h + 4 g - n + j), start 16-byte aligned in copy s = n mod 4;
// lw[dy][i] = M(dy, i - 16) | M(dy, i - 15) << 16.  Built in two passes:
// the patch itself into tm / km (one slot per thread, with the per-wave
// partial sums of T2', k and the row mask), then the shifted tables.
template <int R>
struct FragTables {
    static constexpr int P = 2 * R + 1;
    alignas(16) uint32_t tc[4][P][48];
    uint32_t lw[P][48];
    uint32_t tm[P][P];   // T(dy, x)
    uint8_t km[P][P];    // M(dy, x)
    int t2p[kSearchWaves], k[kSearchWaves];
    uint32_t rowmask[kSearchWaves];
};

// Pass 1, from the staged words (column-major slots x * P + dy) and the
// known mask; `word(slot)` and `known(slot)` read them wherever they are.
template <int R, class Word, class Known>
__device__ __forceinline__ void build_patch(FragTables<R> *ft, Word word, Known known) {
    constexpr int P = 2 * R + 1;
    int t2 = 0, kk = 0;
    uint32_t rows = 0;
    for (int sl = threadIdx.x; sl < P * P; sl += blockDim.x) {
        const int x = sl / P, dy = sl - x * P;
        const bool kn = known(sl);
        const uint32_t w = kn ? word(sl) : 0u;
        ft->tm[dy][x] = kn ? (w ^ 0x00808080u) : 0u;
        ft->km[dy][x] = kn ? 1 : 0;
        if (kn) {
            const int a = (int)(w & 255) - 128, b = (int)((w >> 8) & 255) - 128, c = (int)((w >> 16) & 255) - 128;
            t2 += a * a + b * b + c * c;
            kk += 1;
            rows |= 1u << dy;
        }
    }
    t2 = (int)dpp::sum_u32((uint32_t)t2);   // exact: 32-bit wrap-around sums
    kk = (int)dpp::sum_u32((uint32_t)kk);
    rows = dpp::or_u32(rows);
    if ((threadIdx.x & 63) == 0) {
        ft->t2p[threadIdx.x >> 6] = t2;
        ft->k[threadIdx.x >> 6] = kk;
        ft->rowmask[threadIdx.x >> 6] = rows;
    }
}

// Pass 2, after a barrier that publishes pass 1.
template <int R>
__device__ __forceinline__ void build_tables(FragTables<R> *ft) {
    constexpr int P = 2 * R + 1, NT = 4 * P * 48, NL = P * 48, T = kSearchWaves * 64;
#pragma unroll
    for (int it = 0; it < (NT + T - 1) / T; ++it) {
        const int e = threadIdx.x + it * T;
        if (e < NT) {
            const int s = e / (P * 48), r = e - s * (P * 48), dy = r / 48, i = r - dy * 48;
            const int x = i - 16 - s;
            ft->tc[s][dy][i] = (x >= 0 && x < P) ? ft->tm[dy][x] : 0u;
        }
    }
#pragma unroll
    for (int it = 0; it < (NL + T - 1) / T; ++it) {
        const int e = threadIdx.x + it * T;
        if (e < NL) {
            const int dy = e / 48, i = e - dy * 48, x = i - 16;
            const uint32_t m0 = (x >= 0 && x < P) ? ft->km[dy][x] : 0u;
            const uint32_t m1 = (x + 1 >= 0 && x + 1 < P) ? ft->km[dy][x + 1] : 0u;
            ft->lw[dy][i] = m0 | (m1 << 16);
        }
    }
}

// First tile column and row of tile `tile` of the MFMA tiling of the rect.
template <int R>
__device__ __forceinline__ void tile_origin(int rx0, int ry0, int ntx, int tile, int *tx0, int *ty0) {
    *tx0 = mfma_tile_x0(rx0, R) + (tile % ntx) * kTileW;
    *ty0 = ry0 + (tile / ntx) * kMfmaTileH;
}

// Issues every load of the tile at (tx0, ty0) -- staged window (padded rows
// ty0 - R + kPadT .., columns tx0 - R + kPadL .., a multiple of 8) and the
// validity radii of this lane's candidates (rows 16 t + 4 g + i of the tile,
// column tx0 + 16 wave + n) -- then writes the window to LDS.  Returns the
// lane's validity bits (bit 4 t + i); the caller publishes with a barrier.
template <int R>
__device__ __forceinline__ uint32_t stage_tile(const JobDev &d, int tx0, int ty0, int rx0, int rx1, int ry1,
                                               MfmaTile<R> &L) {
    using G = MfmaGeom<R>;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, g = lane >> 4;
    const int pitch = d.pitch;
    const int cx = tx0 + 16 * wave + n;
    const int64_t org = (int64_t)(ty0 - R + kPadT) * pitch + (tx0 - R + kPadL);
    const uint4 *wa = (const uint4 *)(d.srcw + org);
    const uint4 *wq = (const uint4 *)(d.srcq + org);
    uint4 va[G::AIT], vq[G::QIT];
#pragma unroll
    for (int k = 0; k < G::AIT; ++k) {
        const int i = min(tid + k * kSearchWaves * 64, G::NA - 1);
        const int ly = i / G::QA, lq = i - ly * G::QA;
        va[k] = wa[ly * (pitch >> 2) + lq];
    }
#pragma unroll
    for (int k = 0; k < G::QIT; ++k) {
        const int i = min(tid + k * kSearchWaves * 64, G::NQ - 1);
        const int ly = i / G::QQ, lq = i - ly * G::QQ;
        vq[k] = wq[ly * (pitch >> 3) + lq];
    }
    const uint8_t *vr = d.vradp + (int64_t)(ty0 + 4 * g + kPadT) * pitch + (cx + kPadL);
    uint32_t vv[kMfmaTilesPerWave * 4];
#pragma unroll
    for (int t = 0; t < kMfmaTilesPerWave; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) vv[4 * t + i] = vr[(16 * t + i) * pitch];

#pragma unroll
    for (int k = 0; k < G::AIT; ++k) {
        const int i = min(tid + k * kSearchWaves * 64, G::NA - 1);
        const int ly = i / G::QA, lq = i - ly * G::QA;
        *(uint4 *)&L.a[ly * kMfmaStrideA + 4 * lq] = va[k];
    }
#pragma unroll
    for (int k = 0; k < G::QIT; ++k) {
        const int i = min(tid + k * kSearchWaves * 64, G::NQ - 1);
        const int ly = i / G::QQ, lq = i - ly * G::QQ;
        *(uint4 *)&L.q[ly * kMfmaStrideQ + 16 * lq] = vq[k];
    }
    uint32_t vmask = 0;
    const bool colok = cx >= rx0 && cx < rx1;
#pragma unroll
    for (int t = 0; t < kMfmaTilesPerWave; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int y = ty0 + 16 * t + 4 * g + i;
            if (colok && y < ry1 && vv[4 * t + i] >= (uint32_t)R) vmask |= 1u << (4 * t + i);
        }
    return vmask;
}

// Scores this lane's candidates of a staged tile and returns their minimum
// key (~0 if none is valid).  The B operands are read from the per-target
// tables in LDS one patch row at a time (rows outer, the four 16-row blocks
// inner): only one row's B operands and the 16 accumulators are live, so
// the register budget does not grow with the patch size, and the 16
// independent accumulation chains keep the matrix cores busy.
template <int R>
__device__ __forceinline__ uint64_t score_tile_rows(const JobDev &d, const FragTables<R> *ft, int tx0, int ty0,
                                                    uint32_t vmask, const MfmaTile<R> &L) {
    constexpr int P = 2 * R + 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4, s4 = n & 3;
    const int W = d.W, cx = tx0 + 16 * wave + n;
    int t2 = 0, kk = 0;
#pragma unroll
    for (int w = 0; w < kSearchWaves; ++w) {
        t2 += ft->t2p[w];
        kk += ft->k[w];
    }
    t2 = __builtin_amdgcn_readfirstlane(t2);
    kk = __builtin_amdgcn_readfirstlane(kk);
    v4i c0[kMfmaTilesPerWave], c1[kMfmaTilesPerWave], cl[kMfmaTilesPerWave], ch[kMfmaTilesPerWave];
#pragma unroll
    for (int t = 0; t < kMfmaTilesPerWave; ++t) {
        c0[t] = v4i{0, 0, 0, 0};
        c1[t] = v4i{0, 0, 0, 0};
        cl[t] = v4i{0, 0, 0, 0};
        ch[t] = v4i{0, 0, 0, 0};
    }
    const int base = n * kMfmaStrideA + 16 * wave + 4 * g;
    const int qbase = n * kMfmaStrideQ + 32 * wave + 16 * g;
#pragma unroll
    for (int dy = 0; dy < P; ++dy) {
        const v4i b0 = *(const v4i *)&ft->tc[s4][dy][4 * g + 16 - 4 * (n >> 2)];
        const v4i b1 = *(const v4i *)&ft->tc[s4][dy][16 + 4 * g + 16 - 4 * (n >> 2)];
        v4i bl, bh;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t w = ft->lw[dy][8 * g + 2 * j - n + 16];
            bl[j] = (int)w;
            bh[j] = (int)(w << 8);
        }
#pragma unroll
        for (int t = 0; t < kMfmaTilesPerWave; ++t) {
            const int row = (16 * t + dy);
            const v4i a0 = *(const v4i *)&L.a[base + row * kMfmaStrideA];
            const v4i a1 = *(const v4i *)&L.a[base + row * kMfmaStrideA + 16];
            const v4i aq = *(const v4i *)&L.q[qbase + row * kMfmaStrideQ];
            c0[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a0, b0, c0[t], 0, 0, 0);
            c1[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1, b1, c1[t], 0, 0, 0);
            cl[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(aq, bl, cl[t], 0, 0, 0);
            ch[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(aq, bh, ch[t], 0, 0, 0);
        }
    }
    uint64_t best = ~0ull;
#pragma unroll
    for (int t = 0; t < kMfmaTilesPerWave; ++t) {
        // C lane (n, g) holds rows 4g + i of column n.
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (vmask & (1u << (4 * t + i))) {
                const int s2 = 256 * (ch[t][i] + 128 * kk) + cl[t][i] + 128 * kk;
                const uint32_t ssd = (uint32_t)(t2 - 2 * (c0[t][i] + c1[t][i]) + s2);
                const int y = ty0 + 16 * t + 4 * g + i;
                const uint64_t key = ((uint64_t)ssd << 32) | (uint32_t)(y * W + cx);
                best = key < best ? key : best;
            }
        }
    }
    return best;
}

}  // namespace mtile
}  // namespace inpaint
