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
#include <hip/hip_ext.h>

#include "inpaint_dev.h"

namespace inpaint {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kMfmaTilesPerWave = 4;                       // 16-row tiles stacked per wave
constexpr int kMfmaTileH = 16 * kMfmaTilesPerWave;          // 64 rows: the SIMT tiling with 16 rows per thread
constexpr int kMfmaCols = 80;                               // staged columns (64 + halo, rounded)
constexpr int kMfmaStrideA = 100;                           // words per staged row (100 % 32 == 4)
constexpr int kMfmaStrideQ = 272;                           // bytes per |s'|^2 row (68 words, 68 % 32 == 4)

template <int R>
struct MfmaGeom {
    static constexpr int P = 2 * R + 1;
    static constexpr int ROWS = kMfmaTileH + 2 * R;
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
    uint32_t a[MfmaGeom<R>::ROWS * kMfmaStrideA];            // RGBX ^ 0x80808080
    uint8_t q[MfmaGeom<R>::ROWS * kMfmaStrideQ + 32];         // (lo', hi') per pixel
    uint64_t red[kSearchWaves];
};

template <int R>
__device__ __forceinline__ void search_tile_mfma(const JobDev &d, const MfmaFrags *frag, int rx0, int ry0, int rx1,
                                                 int ry1, int ntx, int tile, uint64_t *out, MfmaLds<R> &L) {
    using G = MfmaGeom<R>;
    constexpr int P = G::P;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, g = lane >> 4;
    const int tx0 = rx0 + (tile % ntx) * kTileW;
    const int ty0 = ry0 + (tile / ntx) * kMfmaTileH;
    const int W = d.W, H = d.H;
    const int cx = tx0 + 16 * wave + n;   // this lane's candidate column

    // Validity of this lane's candidates: rows 16 t + 4 g + i of the tile.
    uint32_t vmask = 0;
    if (cx < rx1) {
#pragma unroll
        for (int t = 0; t < kMfmaTilesPerWave; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int y = ty0 + 16 * t + 4 * g + i;
                if (y < ry1 && d.vrad[(int64_t)y * W + cx] >= R) vmask |= 1u << (4 * t + i);
            }
    }
    // Stage the source tile (+ halo) as offset words and |s'|^2 bytes.
    // Columns past 64 + 2R are read by the MFMA fragments but meet zero B
    // entries, so they are left unstaged.
    constexpr int COLS = kTileW + 2 * R;
    for (int i = tid; i < G::ROWS * COLS; i += kSearchWaves * 64) {
        const int ly = i / COLS, lx = i - ly * COLS;
        const int gx = tx0 - R + lx, gy = ty0 - R + ly;
        uint32_t v = 0x80808080u;
        uint16_t q = 0;
        if ((unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H) {
            const int64_t gi = (int64_t)gy * W + gx;
            v = d.srcw[gi];
            q = d.srcq[gi];
        }
        L.a[ly * kMfmaStrideA + lx] = v;
        *(uint16_t *)&L.q[ly * kMfmaStrideQ + 2 * lx] = q;
    }
    if (!__syncthreads_or(vmask != 0)) {
        if (tid == 0) out[tile] = ~0ull;
        return;
    }

    // B operands of this target, built once per target by the commit
    // kernel in the MFMA register layout: 16 contiguous bytes per lane.
    const MfmaFrags *fr = frag;
    v4i bc[P][2], bh[P], bl[P];
#pragma unroll
    for (int dy = 0; dy < P; ++dy) {
        bc[dy][0] = *(const v4i *)fr->c[dy][0][lane];
        bc[dy][1] = *(const v4i *)fr->c[dy][1][lane];
        bl[dy] = *(const v4i *)fr->l[dy][lane];
        bh[dy] = *(const v4i *)fr->h[dy][lane];
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
    if (!query) {
        const IterState *st = d.st;
        if (st->done || st->error || !st->pending || st->iter >= st->iter_limit) return;
    }
    const int tile = xcd_band_tile((int)blockIdx.x, (int)gridDim.x);
    if (tile >= ntiles) return;
    search_tile_mfma<R>(d, query ? d.qfrag : d.frag, rx0, ry0, rx1, ry1, ntx, tile, d.partials, L);
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

// Static source planes of the MFMA search, from the original image: offset
// RGBX words and the |s'|^2 byte pair.  Only original known pixels are ever
// read by a valid candidate, and those never change.
__global__ __launch_bounds__(256) void k_mfma_planes(JobDev d) {
    const int64_t n = (int64_t)d.W * d.H;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t v = d.img[i];
    d.srcw[i] = v ^ 0x80808080u;
    d.srcq[i] = sq_bytes(v);
}

}  // namespace

hipError_t launch_mfma_planes(const JobDev &d, hipStream_t s) {
    const int64_t n = (int64_t)d.W * d.H;
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
