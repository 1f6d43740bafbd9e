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
// MFMAs).  The B fragments depend only on the target: the commit kernel
// builds them once per target in the register layout, each wave loads them
// with coalesced 16-byte reads and keeps them in registers; the A fragments
// are 16-byte LDS reads from the staged tile.
//
// The planes are static (candidate windows lie in the original known
// region, which never changes) and zero-padded, and the tiling starts on a
// column that puts every staged window on an 8-pixel boundary: a tile is
// staged with unconditional 16-byte loads, issued together with the
// candidates' validity radii and the B fragments before the first wait.
#include <hip/hip_ext.h>

#include "inpaint_dev.h"

namespace inpaint {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kMfmaTilesPerWave = 4;                       // 16-row tiles stacked per wave
constexpr int kMfmaTileH = 16 * kMfmaTilesPerWave;          // 64 rows: the SIMT tiling with 16 rows per thread
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

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

// |s'|^2 of an RGBX word, split into (low byte - 128, high byte - 128) int8s
// packed as a 16-bit value (low byte first).
__device__ __forceinline__ uint16_t sq_bytes(uint32_t w) {
    const int r = (int)(w & 255) - 128, g = (int)((w >> 8) & 255) - 128, b = (int)((w >> 16) & 255) - 128;
    const int q = r * r + g * g + b * b;              // 0 .. 49152
    const int lo = (q & 255) - 128, hi = (q >> 8) - 128;
    return (uint16_t)((uint8_t)lo | ((uint32_t)(uint8_t)hi << 8));
}

template <int R>
struct MfmaLds {
    alignas(16) uint32_t a[MfmaGeom<R>::ROWS * kMfmaStrideA];   // RGBX ^ 0x80808080
    alignas(16) uint8_t q[MfmaGeom<R>::ROWS * kMfmaStrideQ + 32];  // (lo', hi') per pixel
    uint64_t red[kSearchWaves];
};

template <int R>
__device__ __forceinline__ void search_tile_mfma(const JobDev &d, const MfmaFrags *frag, bool live, int rx0, int ry0,
                                                 int rx1, int ry1, int ntx, int tile, uint64_t *out, MfmaLds<R> &L) {
    using G = MfmaGeom<R>;
    constexpr int P = G::P;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, g = lane >> 4;
    const int tx0 = mfma_tile_x0(rx0, R) + (tile % ntx) * kTileW;
    const int ty0 = ry0 + (tile / ntx) * kMfmaTileH;
    const int W = d.W, pitch = d.pitch;
    const int cx = tx0 + 16 * wave + n;   // this lane's candidate column

    // ---- issue: staged window (padded rows ty0 - R + kPadT .., columns
    // tx0 - R + kPadL .., a multiple of 8), validity radii of this lane's
    // candidates (rows 16 t + 4 g + i of the tile) and the B fragments.
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
    const MfmaFrags *fr = frag;
    v4i bc[P][2], bh[P], bl[P];
#pragma unroll
    for (int dy = 0; dy < P; ++dy) {
        bc[dy][0] = *(const v4i *)fr->c[dy][0][lane];
        bc[dy][1] = *(const v4i *)fr->c[dy][1][lane];
        bl[dy] = *(const v4i *)fr->l[dy][lane];
        bh[dy] = *(const v4i *)fr->h[dy][lane];
    }

    // ---- publish the tile; one barrier also tells whether any candidate
    // of the tile is valid.
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
    if (!__syncthreads_or(live && vmask != 0)) {
        if (tid == 0 && live) out[tile] = ~0ull;
        return;
    }

    const int t2 = fr->t2p, kk = fr->k;
    const uint32_t rowmask = fr->rowmask;

    uint64_t best = ~0ull;
#pragma unroll
    for (int t = 0; t < kMfmaTilesPerWave; ++t) {
        // four independent accumulation chains keep the MFMA pipeline busy
        v4i c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0}, ch = {0, 0, 0, 0}, cl = {0, 0, 0, 0};
#pragma unroll
        for (int dy = 0; dy < P; ++dy) {
            if (!((rowmask >> dy) & 1u)) continue;   // uniform: patch row without a known pixel
            const int ly = 16 * t + n + dy;                   // A row = candidate row n of the tile
            const v4i a0 = *(const v4i *)&L.a[ly * kMfmaStrideA + 16 * wave + 4 * g];
            const v4i a1 = *(const v4i *)&L.a[ly * kMfmaStrideA + 16 * wave + 16 + 4 * g];
            const v4i aq = *(const v4i *)&L.q[ly * kMfmaStrideQ + 32 * wave + 16 * g];
            c0 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a0, bc[dy][0], c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1, bc[dy][1], c1, 0, 0, 0);
            cl = __builtin_amdgcn_mfma_i32_16x16x64_i8(aq, bl[dy], cl, 0, 0, 0);
            ch = __builtin_amdgcn_mfma_i32_16x16x64_i8(aq, bh[dy], ch, 0, 0, 0);
        }
        // C lane (n, g) holds rows 4g + i of column n.
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (vmask & (1u << (4 * t + i))) {
                const int s2 = 256 * (ch[i] + 128 * kk) + cl[i] + 128 * kk;
                const uint32_t ssd = (uint32_t)(t2 - 2 * (c0[i] + c1[i]) + s2);
                const int y = ty0 + 16 * t + 4 * g + i;
                const uint64_t key = ((uint64_t)ssd << 32) | (uint32_t)(y * W + cx);
                best = key < best ? key : best;
            }
        }
    }
    best = wave_min_u64(best);
    if (lane == 0) L.red[wave] = best;
    __syncthreads();
    if (tid == 0) {
        uint64_t b = L.red[0];
#pragma unroll
        for (int w = 1; w < kSearchWaves; ++w) b = L.red[w] < b ? L.red[w] : b;
        out[tile] = b;
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
    search_tile_mfma<R>(d, query ? d.qfrag : d.frag, live, rx0, ry0, rx1, ry1, ntx, tile, d.partials, L);
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
