// Initialisation, fill-front / priority, selection, target staging and the
// copy / confidence update of exemplar-based object removal on gfx950.
//
// Everything here except the exemplar search (search.hip) is latency-bound
// work on at most a few thousand pixels per iteration, so the per-iteration
// part runs as ONE work-group of 256 threads per image ("commit" kernel):
//   reduce the search partials -> copy the source patch -> stage the
//   neighbourhood of the patch in LDS -> refresh the priorities there ->
//   refresh the affected block maxima -> argmax -> stage the next target.
//
// Priorities are binary64 and must match a plain sequential CPU evaluation
// bit for bit, so this file is compiled with FP contraction off and every
// sum runs in the fixed raster order of the patch offsets.  The same
// templated routine evaluates a priority from global memory (initialisation)
// and from the LDS copy of the neighbourhood (per iteration).
#pragma clang fp contract(off)

#include "search_mfma_tile.h"

namespace inpaint {

namespace {

// Neighbourhood the commit kernel stages around the target: the refresh
// window reaches 2r+1 from it, a priority reads its patch (r) and gradients
// one pixel further, so 3r+2.
template <int R>
struct Stage {
    static constexpr int half = 3 * R + 2;
    static constexpr int side = 2 * half + 1;
    static constexpr int n = side * side;
};

__device__ __forceinline__ bool in_img(const JobDev &d, int x, int y) {
    return (unsigned)x < (unsigned)d.W && (unsigned)y < (unsigned)d.H;
}

// ---- pixel views: what a priority evaluation reads -------------------------

// Straight from global memory.
// Column and row of a raster index (0 <= i < W * H < 2^31, so a 32-bit
// unsigned division, much shorter than a 64-bit one).
__device__ __forceinline__ int col_of(int64_t i, int W) { return (int)((uint32_t)i % (uint32_t)W); }
__device__ __forceinline__ int row_of(int64_t i, int W) { return (int)((uint32_t)i / (uint32_t)W); }

struct GlobalView {
    const JobDev &d;
    __device__ bool known(int x, int y) const { return in_img(d, x, y) && d.hole[(int64_t)y * d.W + x] == 0; }
    // hole indicator with out-of-image pixels counted as hole (the normal)
    __device__ int hole_or_out(int x, int y) const {
        return (!in_img(d, x, y) || d.hole[(int64_t)y * d.W + x]) ? 1 : 0;
    }
    __device__ double conf(int x, int y) const { return d.conf[(int64_t)y * d.W + x]; }
    // C of a known pixel, +0.0 for any other
    __device__ double conf_known(int x, int y) const { return known(x, y) ? conf(x, y) : 0.0; }
    // Central-difference gradient of the gray image at a known pixel whose
    // four neighbours are known: returns gx^2 + gy^2, or -1 otherwise.
    __device__ int grad(int x, int y, int *gx, int *gy) const {
        if (!known(x, y) || !known(x + 1, y) || !known(x - 1, y) || !known(x, y + 1) || !known(x, y - 1))
            return -1;
        const uint8_t *g = d.gray;
        const int W = d.W;
        *gx = (int)g[(int64_t)y * W + x + 1] - (int)g[(int64_t)y * W + x - 1];
        *gy = (int)g[(int64_t)(y + 1) * W + x] - (int)g[(int64_t)(y - 1) * W + x];
        return *gx * *gx + *gy * *gy;
    }
};

// The LDS copy of a square neighbourhood: status 0 known, 1 hole, 2 outside
// the image; confidences of known pixels (+0.0 for the others); gradients
// precomputed per pixel.
template <int R>
struct LdsStage {
    static constexpr int WIN = 4 * R + 3;          // refresh window side
    static constexpr int NBA = (WIN + 6) / 8 + 1;  // 8x8 blocks it can touch per axis
    uint8_t st[Stage<R>::n];
    uint8_t gray[Stage<R>::n];
    double conf[Stage<R>::n];
    uint32_t img[Stage<R>::n];
    int mag[Stage<R>::n];
    int gxy[Stage<R>::n];   // gx in the low 16 bits, gy in the high 16 (signed)
    int64_t bkey[NBA * NBA * 64];   // priority keys of the blocks the window touches
    double2 wcd[WIN * WIN];         // (C, D) of the window pixels
    int16_t front[WIN * WIN];       // window pixels on the front (window-local index)
    int nfront;
    double fsum[64];                // per front pixel of a round: confidence sum
    int fbest[4][64], fbxy[4][64];  // and the best gradient of parts of the patch rows
};

template <int R>
struct LdsView {
    const LdsStage<R> &s;
    int ox, oy;
    static constexpr int side = Stage<R>::side;
    __device__ int at(int x, int y) const { return (y - oy) * side + (x - ox); }
    __device__ bool known(int x, int y) const { return s.st[at(x, y)] == 0; }
    __device__ int hole_or_out(int x, int y) const { return s.st[at(x, y)] != 0 ? 1 : 0; }
    // C of a known pixel, +0.0 for any other (the staged array holds +0.0
    // for pixels that are not known).
    __device__ double conf_known(int x, int y) const { return s.conf[at(x, y)]; }
    __device__ int grad(int x, int y, int *gx, int *gy) const {
        const int i = at(x, y);
        const int v = s.gxy[i];
        *gx = (int)(int16_t)(v & 0xffff);
        *gy = v >> 16;
        return s.mag[i];
    }
};

// Fill front: a hole pixel with at least one in-image 4-neighbour known.
// (x, y) is always inside the image here.
__device__ __forceinline__ bool on_front(const GlobalView &v, int x, int y) {
    if (v.hole_or_out(x, y) == 0) return false;
    return v.known(x + 1, y) || v.known(x - 1, y) || v.known(x, y + 1) || v.known(x, y - 1);
}

// The same test on the LDS copy, with all five reads unconditional.
template <int R>
__device__ __forceinline__ bool on_front(const LdsView<R> &v, int x, int y) {
    const int i = v.at(x, y);
    const uint8_t *st = v.s.st;
    const int c = st[i], e = st[i + 1], w = st[i - 1], n = st[i - LdsView<R>::side], so = st[i + LdsView<R>::side];
    return c == 1 && (e == 0 || w == 0 || n == 0 || so == 0);
}

// Eq. 2.  Confidence: sum of C over the known pixels of the patch, in raster
// order of the offsets, divided by the constant patch area P*P.  Data term:
// the isophote (-gy, gx)/2 at the known pixel of the patch with the largest
// central-difference gradient of the gray image (all four neighbours known;
// first in raster order on ties), dotted with the unit normal of the front
// (central differences of the hole indicator), absolute value, over 255.
// Unknown offsets add +0.0, which leaves the running sum bit-identical (it
// starts at +0.0 and only non-negative values are added), so the loop needs
// no branches and unrolls fully.
template <int R, class V>
__device__ void priority_terms(const V &v, int px, int py, double norm1, double norm2, double *C, double *D) {
    constexpr int P = 2 * R + 1;
    // Unrolled a few rows at a time: enough independent LDS reads in flight
    // without running out of registers (a fully unrolled 9x9 spills).
    constexpr int kRows = R <= 2 ? P : (R <= 4 ? 3 : 1);
    double sum = 0.0;
#pragma unroll kRows
    for (int dy = -R; dy <= R; ++dy)
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) sum = sum + v.conf_known(px + dx, py + dy);
    *C = sum / (double)(P * P);

    int gx = 0, gy = 0, best = -1;
#pragma unroll kRows
    for (int dy = -R; dy <= R; ++dy)
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) {
            int ax = 0, ay = 0;
            const int mag = v.grad(px + dx, py + dy, &ax, &ay);
            const bool take = mag > best;
            best = take ? mag : best;
            gx = take ? ax : gx;
            gy = take ? ay : gy;
        }
    const int nx = v.hole_or_out(px + 1, py) - v.hole_or_out(px - 1, py);
    const int ny = v.hole_or_out(px, py + 1) - v.hole_or_out(px, py - 1);
    const int kn = nx * nx + ny * ny;
    if (kn == 0) {
        *D = 0.0;
    } else {
        int a = gx * ny - gy * nx;
        if (a < 0) a = -a;
        *D = (0.5 * (double)a) / (kn == 1 ? norm1 : norm2);
    }
}

// The confidence sum of Eq. 2 at (px, py) on the LDS neighbourhood, in
// raster order as priority_terms adds it (rows read one ahead of the adds).
template <int R>
__device__ double conf_sum_lds(const LdsView<R> &v, int px, int py) {
    constexpr int P = 2 * R + 1, side = LdsView<R>::side;
    const double *cf = v.s.conf + v.at(px - R, py - R);
    double c0[P], c1[P];
#pragma unroll
    for (int dx = 0; dx < P; ++dx) c0[dx] = cf[dx];
    double sum = 0.0;
#pragma unroll 1
    for (int dy = 0; dy < P; ++dy) {
        // the row after the last one is still inside the staged square
#pragma unroll
        for (int dx = 0; dx < P; ++dx) c1[dx] = cf[(dy + 1) * side + dx];
#pragma unroll
        for (int dx = 0; dx < P; ++dx) sum = sum + c0[dx];
#pragma unroll
        for (int dx = 0; dx < P; ++dx) c0[dx] = c1[dx];
    }
    return sum;
}

// The largest gradient magnitude of the patch rows dy0 .. dy1 - 1 (offsets
// from the top row) at (px, py), first in raster order on ties: *best (-1 if
// none) and its packed gradient *bxy.
template <int R>
__device__ void grad_best_lds(const LdsView<R> &v, int px, int py, int dy0, int dy1, int *best, int *bxy) {
    constexpr int P = 2 * R + 1, side = LdsView<R>::side;
    const int base = v.at(px - R, py - R) + dy0 * side;
    const int *mg = v.s.mag + base;
    const int *gp = v.s.gxy + base;
    int m0[P], m1[P], g0[P], g1[P];
#pragma unroll
    for (int dx = 0; dx < P; ++dx) {
        m0[dx] = mg[dx];
        g0[dx] = gp[dx];
    }
    int b = -1, bg = 0;
#pragma unroll 1
    for (int dy = dy0; dy < dy1; ++dy) {
#pragma unroll
        for (int dx = 0; dx < P; ++dx) {
            m1[dx] = mg[(dy - dy0 + 1) * side + dx];
            g1[dx] = gp[(dy - dy0 + 1) * side + dx];
        }
#pragma unroll
        for (int dx = 0; dx < P; ++dx) {
            const bool take = m0[dx] > b;
            b = take ? m0[dx] : b;
            bg = take ? g0[dx] : bg;
        }
#pragma unroll
        for (int dx = 0; dx < P; ++dx) {
            m0[dx] = m1[dx];
            g0[dx] = g1[dx];
        }
    }
    *best = b;
    *bxy = bg;
}

// D of Eq. 2 from the chosen packed gradient and the normal at (px, py),
// as priority_terms computes it.
template <int R>
__device__ double data_term_lds(const LdsView<R> &v, int px, int py, int bxy, double norm1, double norm2) {
    const int gx = (int)(int16_t)(bxy & 0xffff), gy = bxy >> 16;
    const int nx = v.hole_or_out(px + 1, py) - v.hole_or_out(px - 1, py);
    const int ny = v.hole_or_out(px, py + 1) - v.hole_or_out(px, py - 1);
    const int kn = nx * nx + ny * ny;
    if (kn == 0) return 0.0;
    int a = gx * ny - gy * nx;
    if (a < 0) a = -a;
    return (0.5 * (double)a) / (kn == 1 ? norm1 : norm2);
}

// (C, D) of a pixel: C = -1 marks "not on the front".
template <int R, class V>
__device__ double2 pixel_terms(const V &v, const JobDev &d, int x, int y) {
    double2 cd = make_double2(-1.0, 0.0);
    if (on_front(v, x, y)) priority_terms<R>(v, x, y, d.norm1, d.norm2, &cd.x, &cd.y);
    return cd;
}

// Priority key from cached terms: bits of P = C * D (Eq. 1), -1 off the front.
// Non-negative doubles order like their bit patterns.
__device__ __forceinline__ int64_t key_of(double2 cd) {
    return cd.x < 0.0 ? -1 : __double_as_longlong(cd.x * cd.y);
}

// ---- work-group reductions (blockDim.x a multiple of 64, <= 1024) ----

__device__ __forceinline__ bool better(int64_t ka, int64_t ia, int64_t kb, int64_t ib) {
    return ka > kb || (ka == kb && ia < ib);
}

// (key, index) pairs, the greater key winning and equal keys going to the
// lower index: a strict total order, so every fold order gives the same pair.
// For the DPP folds a pair is encoded as (key + 1, INT64_MAX - index), which
// maps the identity (-1, INT64_MAX) to (0, 0) and the order to the
// lexicographic order of the two unsigned words (keys are -1 or the bits of
// a non-negative double, indices non-negative).
struct KeyIdx {
    uint64_t k, i;
};
__device__ __forceinline__ KeyIdx key_idx_max(KeyIdx a, KeyIdx b) {
    return (b.k > a.k || (b.k == a.k && b.i > a.i)) ? b : a;
}
template <int CTRL>
__device__ __forceinline__ KeyIdx key_idx_mov(KeyIdx v) {
    return {dpp::mov<CTRL>(v.k), dpp::mov<CTRL>(v.i)};
}
__device__ __forceinline__ KeyIdx key_idx_enc(int64_t key, int64_t idx) {
    return {(uint64_t)(key + 1), (uint64_t)(INT64_MAX - idx)};
}
__device__ __forceinline__ void key_idx_dec(KeyIdx v, int64_t &key, int64_t &idx) {
    key = (int64_t)v.k - 1;
    idx = INT64_MAX - (int64_t)v.i;
}
__device__ __forceinline__ KeyIdx row_argmax_enc(KeyIdx v) {
    v = key_idx_max(v, key_idx_mov<dpp::kShr1>(v));
    v = key_idx_max(v, key_idx_mov<dpp::kShr2>(v));
    v = key_idx_max(v, key_idx_mov<dpp::kShr4>(v));
    v = key_idx_max(v, key_idx_mov<dpp::kShr8>(v));
    return v;
}
// Lane 15 of each 16-lane row ends with the row's maximum.
__device__ __forceinline__ void row_argmax(int64_t &key, int64_t &idx) {
    key_idx_dec(row_argmax_enc(key_idx_enc(key, idx)), key, idx);
}
// The wave's maximum, in every lane (all lanes active).
__device__ __forceinline__ void wave_argmax(int64_t &key, int64_t &idx) {
    KeyIdx v = row_argmax_enc(key_idx_enc(key, idx));
    v = key_idx_max(v, key_idx_mov<dpp::kBcast15>(v));
    v = key_idx_max(v, key_idx_mov<dpp::kBcast31>(v));
    key_idx_dec({dpp::lane63(v.k), dpp::lane63(v.i)}, key, idx);
}

// Work-group folds: each wave folds on DPP, lane 0 posts the wave's result,
// then every thread folds the posted results itself (no second wave pass).
// The closing barrier lets the caller reuse the scratch words.
__device__ void block_argmax(int64_t &key, int64_t &idx, int64_t *sk, int64_t *si) {
    wave_argmax(key, idx);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) {
        sk[w] = key;
        si[w] = idx;
    }
    __syncthreads();
    key = sk[0];
    idx = si[0];
    for (int q = 1; q < nw; ++q)
        if (better(sk[q], si[q], key, idx)) {
            key = sk[q];
            idx = si[q];
        }
    __syncthreads();
}

__device__ uint64_t block_min_u64(uint64_t v, uint64_t *sh) {
    v = dpp::min_u64(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    v = sh[0];
    for (int q = 1; q < nw; ++q) v = sh[q] < v ? sh[q] : v;
    __syncthreads();
    return v;
}

// State of the fill loop at the start of an iteration.
struct Snap {
    int64_t iter, limit, remaining, p;
    double C, D, Pr;
    int32_t done, err, pending, k;
};

__device__ __forceinline__ Snap load_snap(const IterState *st, const TargetStage *tg) {
    Snap v;
    v.iter = st->iter;
    v.limit = st->iter_limit;
    v.remaining = st->remaining;
    v.p = st->p_idx;
    v.C = st->C;
    v.D = st->D;
    v.Pr = st->Pr;
    v.done = st->done;
    v.err = st->error;
    v.pending = st->pending;
    v.k = tg->k;
    return v;
}

struct Scratch {
    Snap snap;           // loop state broadcast by thread 0
    int64_t k[16];
    int64_t i[16];
    uint64_t u[16];
    uint32_t mbits[16];
    uint32_t sbits[16];
    uint32_t ebits[16];
    int64_t bmk[64], bmi[64];        // maxima of the blocks a refresh touched
    uint32_t tp[kMaxOffsets + 15];   // the staged target words (column-major slots)
};

// Persistent fill: writes the target just staged (s.tp and the mask words,
// published by the staging barriers) into every record of the handshake,
// go words excluded.
__device__ void write_records(FillSync *sy, const Scratch &s, int P, int kk, uint32_t t2) {
    const int n = P * P, mw = (n + 31) / 32;
    for (int i = threadIdx.x; i < kGoCopies * n; i += blockDim.x) {
        const int c = i / n, t = i - c * n;
        sy->rec[c].tpix[t] = s.tp[t];
    }
    for (int i = threadIdx.x; i < kGoCopies * mw; i += blockDim.x) {
        const int c = i / mw, w = i - c * mw;
        sy->rec[c].mbits[w] = s.mbits[w];
        sy->rec[c].sbits[w] = s.sbits[w];
        sy->rec[c].ebits[w] = s.ebits[w];
    }
    if (threadIdx.x < kGoCopies) {
        sy->rec[threadIdx.x].t2 = t2;
        sy->rec[threadIdx.x].k = (uint32_t)kk;
    }
}

// The same from a target staged by an earlier dispatch.
__device__ void write_records(FillSync *sy, const TargetStage *tg, int P) {
    const int n = P * P, mw = (n + 31) / 32;
    for (int i = threadIdx.x; i < kGoCopies * n; i += blockDim.x) {
        const int c = i / n, t = i - c * n;
        sy->rec[c].tpix[t] = tg->tpix[t];
    }
    for (int i = threadIdx.x; i < kGoCopies * mw; i += blockDim.x) {
        const int c = i / mw, w = i - c * mw;
        sy->rec[c].mbits[w] = tg->mbits[w];
        sy->rec[c].sbits[w] = tg->sbits[w];
        sy->rec[c].ebits[w] = tg->ebits[w];
    }
    if (threadIdx.x < kGoCopies) {
        sy->rec[threadIdx.x].t2 = tg->t2;
        sy->rec[threadIdx.x].k = (uint32_t)tg->k;
    }
}

// Records of the MFMA (lean) form carry their own freshness: each word is
// the target word (RGB) with a 7-bit tag of the fill iteration it belongs
// to in bits 24-30 and its known flag in bit 31.  Consecutive iterations of
// a job have different tags, and every word of a record is rewritten each
// iteration, so a word that carries the expected tag is that iteration's.
__device__ __forceinline__ uint32_t rec_tag(int64_t iter) { return (uint32_t)(iter % 127) + 1u; }
__device__ __forceinline__ uint32_t lean_word(uint32_t pix, bool known, uint32_t tag) {
    return (pix & 0x00ffffffu) | (tag << 24) | (known ? 0x80000000u : 0u);
}

// The lean records from a target staged by an earlier dispatch.
__device__ void write_records_lean(FillSync *sy, const TargetStage *tg, int P, uint32_t tag) {
    const int n = P * P;
    for (int i = threadIdx.x; i < kGoCopies * n; i += blockDim.x) {
        const int c = i / n, t = i - c * n;
        sy->rec[c].tpix[t] = lean_word(tg->tpix[t], (tg->mbits[t >> 5] >> (t & 31)) & 1u, tag);
    }
}

// One wave recomputes the maximum of the 8x8 priority block (bx, by).
__device__ void refresh_block_wave(const JobDev &d, int bx, int by) {
    const int lane = threadIdx.x & 63;
    const int x = bx * kBlock + (lane & (kBlock - 1)), y = by * kBlock + lane / kBlock;
    int64_t key = -1, idx = INT64_MAX;
    if (in_img(d, x, y)) {
        idx = (int64_t)y * d.W + x;
        key = key_of(d.pcd[idx]);
    }
    wave_argmax(key, idx);
    if (lane == 0) {
        d.blk[by * d.nbw + bx].key = key;
        d.blk[by * d.nbw + bx].idx = idx;
    }
}

// Stages the target patch at (tx, ty) with radius r into *tg: known mask,
// RGBX words and T2 = sum of squared known target values, in column-major
// slot order (dx + r) * P + (dy + r).
// Column-run bits of mask word w (of mw) of a P x P patch in column-major
// slot order: a known slot starts a run when the slot above it in its column
// is unknown or outside the patch, and ends one when the slot below is.
__device__ __forceinline__ void run_bits(const uint32_t *mbits, int w, int mw, int P, uint32_t *sb, uint32_t *eb) {
    const uint32_t m = mbits[w];
    const uint32_t up = (m << 1) | (w > 0 ? mbits[w - 1] >> 31 : 0u);        // slot - 1 known
    const uint32_t dn = (m >> 1) | (w + 1 < mw ? mbits[w + 1] << 31 : 0u);   // slot + 1 known
    uint32_t cs = 0, ce = 0;   // slots at the top / bottom of their column
    const int base = 32 * w;
    for (int c = (base + P - 1) / P * P; c < base + 32; c += P) cs |= 1u << (c - base);
    for (int c = (base + P) / P * P - 1; c < base + 32; c += P) ce |= 1u << (c - base);
    *sb = m & (cs | ~up);
    *eb = m & (ce | ~dn);
}

// Target staging core: slot(t, &pix) says whether patch slot t (column-major,
// (dx + r) * P + (dy + r)) is known and gives its RGB word.  One pass over
// the slots writes the words and takes the known mask with a wave ballot per
// 64 slots (no atomics), then one barrier; the column-run bits follow from
// the mask words: a known slot starts a run when the slot above it in its
// column is unknown or outside the patch, and ends one when the slot below
// is.  Returns the known count k; T2 = sum of squared known values.
template <class F>
__device__ int stage_slots(int r, int tx, int ty, TargetStage *tg, Scratch &s, FillSync *recs,
                           F slot) {
    const int P = 2 * r + 1, n = P * P, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t t2 = 0;
    for (int base = 0; base < n; base += blockDim.x) {
        const int t = base + threadIdx.x;
        uint32_t pix = 0;
        const bool kn = t < n && slot(t, &pix);
        if (t < n) {
            tg->tpix[t] = pix;
            s.tp[t] = pix;
        }
        if (kn) {
            const uint32_t R = pix & 255, G = (pix >> 8) & 255, B = (pix >> 16) & 255;
            t2 += R * R + G * G + B * B;
        }
        const uint64_t bal = __ballot(kn);
        const int w0 = (base >> 5) + 2 * wave;
        if (lane == 0 && w0 < 16) {
            s.mbits[w0] = (uint32_t)bal;
            if (w0 + 1 < 16) s.mbits[w0 + 1] = (uint32_t)(bal >> 32);
        }
    }
    t2 = dpp::sum_u32(t2);
    if (lane == 0) s.u[wave] = t2;
    __syncthreads();
    const int mw = (n + 31) / 32, nw = blockDim.x >> 6;
    uint32_t T2 = 0;
    for (int w = 0; w < nw; ++w) T2 += (uint32_t)s.u[w];
    int kk = 0;
    for (int w = 0; w < mw; ++w) kk += __popc(s.mbits[w]);
    if ((int)threadIdx.x < mw) {
        const int w = threadIdx.x;
        uint32_t sb, eb;
        run_bits(s.mbits, w, mw, P, &sb, &eb);
        s.sbits[w] = sb;
        s.ebits[w] = eb;
        tg->mbits[w] = s.mbits[w];
        tg->sbits[w] = sb;
        tg->ebits[w] = eb;
    }
    if (threadIdx.x == 0) {
        tg->tx = tx;
        tg->ty = ty;
        tg->r = r;
        tg->k = kk;
        tg->t2 = T2;
    }
    if (recs) {
        __syncthreads();   // s.sbits / s.ebits
        write_records(recs, s, P, kk, T2);
    }
    return kk;
}

__device__ int stage_target(const JobDev &d, int tx, int ty, int r, TargetStage *tg, Scratch &s,
                            FillSync *recs = nullptr) {
    const int P = 2 * r + 1;
    const GlobalView v{d};
    return stage_slots(r, tx, ty, tg, s, recs, [&](int t, uint32_t *pix) {
        const int x = tx + t / P - r, y = ty + t % P - r;
        if (!v.known(x, y)) return false;
        *pix = d.img[(int64_t)y * d.W + x] & 0x00ffffffu;
        return true;
    });
}

// Persistent fill with the MFMA search: stages only what its search groups
// read -- the words with their known flags, tagged for iteration `tag` (see
// lean_word) -- into every record, and the words and the known mask into the
// target (the words straight from the slot pass, no barrier in between).  T2 and the
// column-run bits of the target follow once, for the last target staged in a
// dispatch (finish_stage).  Returns k.
template <class F>
__device__ int stage_slots_lean(int r, int tx, int ty, TargetStage *tg, Scratch &s, FillSync *recs, uint32_t tag,
                                F slot) {
    const int P = 2 * r + 1, n = P * P, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int base = 0; base < n; base += blockDim.x) {
        const int t = base + threadIdx.x;
        uint32_t pix = 0;
        const bool kn = t < n && slot(t, &pix);
        if (t < n) {
            tg->tpix[t] = pix;
            s.tp[t] = pix;
            const uint32_t w = lean_word(pix, kn, tag);
#pragma unroll
            for (int c = 0; c < kGoCopies; ++c) recs->rec[c].tpix[t] = w;
        }
        const uint64_t bal = __ballot(kn);
        const int w0 = (base >> 5) + 2 * wave;
        if (lane == 0 && w0 < 16) {
            s.mbits[w0] = (uint32_t)bal;
            if (w0 + 1 < 16) s.mbits[w0 + 1] = (uint32_t)(bal >> 32);
        }
    }
    __syncthreads();
    const int mw = (n + 31) / 32;
    int kk = 0;
    for (int w = 0; w < mw; ++w) kk += __popc(s.mbits[w]);
    if ((int)threadIdx.x < mw) tg->mbits[threadIdx.x] = s.mbits[threadIdx.x];
    if (threadIdx.x == 0) {
        tg->tx = tx;
        tg->ty = ty;
        tg->r = r;
        tg->k = kk;
    }
    return kk;
}

// Completes the target that stage_slots_lean left in s.tp / s.mbits: T2 and
// the column-run bits.
__device__ void finish_stage(int r, TargetStage *tg, Scratch &s) {
    const int P = 2 * r + 1, n = P * P, mw = (n + 31) / 32, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t t2 = 0;
    for (int t = threadIdx.x; t < n; t += blockDim.x)
        if ((s.mbits[t >> 5] >> (t & 31)) & 1u) {
            const uint32_t pix = s.tp[t], R = pix & 255, G = (pix >> 8) & 255, B = (pix >> 16) & 255;
            t2 += R * R + G * G + B * B;
        }
    t2 = dpp::sum_u32(t2);
    if (lane == 0) s.u[wave] = t2;
    __syncthreads();
    if ((int)threadIdx.x < mw) {
        uint32_t sb, eb;
        run_bits(s.mbits, threadIdx.x, mw, P, &sb, &eb);
        tg->sbits[threadIdx.x] = sb;
        tg->ebits[threadIdx.x] = eb;
    }
    if (threadIdx.x == 0) {
        uint32_t T2 = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) T2 += (uint32_t)s.u[w];
        tg->t2 = T2;
    }
}

// Argmax over the priority blocks, then stages the winner as the next target.
__device__ void select_and_stage(const JobDev &d, Scratch &s) {
    int64_t key = -1, idx = INT64_MAX;
    const int bw = d.pbx1 - d.pbx0, nb = bw * (d.pby1 - d.pby0);
    for (int t = threadIdx.x; t < nb; t += blockDim.x) {
        const BlockBest b = d.blk[(d.pby0 + t / bw) * d.nbw + d.pbx0 + t % bw];
        if (better(b.key, b.idx, key, idx)) {
            key = b.key;
            idx = b.idx;
        }
    }
    block_argmax(key, idx, s.k, s.i);
    IterState *st = d.st;
    if (key < 0) {
        // No front pixel although the hole is not empty: cannot happen for a
        // valid state; flag it instead of looping.
        if (threadIdx.x == 0) st->error = INPAINT_DEVICE;
        return;
    }
    const int px = col_of(idx, d.W), py = row_of(idx, d.W);
    stage_target(d, px, py, d.r, d.tgt, s);
    if (threadIdx.x == 0) {
        const double2 cd = d.pcd[idx];
        st->p_idx = idx;
        st->C = cd.x;
        st->D = cd.y;
        st->Pr = cd.x * cd.y;
        st->pending = 1;
    }
}

// Geometry of one refresh: the window of pixels whose priority can change
// (within 2r+1 of the filled target, clipped to the image) and the 8x8
// blocks it touches.
struct Refresh {
    int wx0, wx1, wy0, wy1;   // window
    int abx0, aby0, nabx, naby;
};

template <int R>
__device__ Refresh refresh_geometry(const JobDev &d, int px, int py) {
    constexpr int reach = 2 * R + 1;
    Refresh g;
    g.wx0 = max(px - reach, 0);
    g.wx1 = min(px + reach + 1, d.W);
    g.wy0 = max(py - reach, 0);
    g.wy1 = min(py + reach + 1, d.H);
    g.abx0 = g.wx0 / kBlock;
    g.aby0 = g.wy0 / kBlock;
    g.nabx = (g.wx1 - 1) / kBlock - g.abx0 + 1;
    g.naby = (g.wy1 - 1) / kBlock - g.aby0 + 1;
    return g;
}

// Gradients of the LDS neighbourhood on the stage-local square [lo, hi)^2
// (1 <= lo, hi <= side - 1): the central-difference gradient of the gray
// image at known pixels whose four neighbours are known (magnitude and
// packed components), magnitude -1 elsewhere.
template <int R>
__device__ void grad_pass(LdsStage<R> &L, int lo, int hi) {
    constexpr int side = Stage<R>::side;
    const int w = hi - lo, n = w * w;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int i = (lo + t / w) * side + lo + t % w;
        int mag = -1, gxy = 0;
        if (L.st[i] == 0 && L.st[i + 1] == 0 && L.st[i - 1] == 0 && L.st[i + side] == 0 && L.st[i - side] == 0) {
            const int gx = (int)L.gray[i + 1] - (int)L.gray[i - 1];
            const int gy = (int)L.gray[i + side] - (int)L.gray[i - side];
            mag = gx * gx + gy * gy;
            gxy = (gx & 0xffff) | (gy << 16);
        }
        L.mag[i] = mag;
        L.gxy[i] = gxy;
    }
}

// Re-evaluates the priorities of the refresh window from the LDS copy of the
// neighbourhood (already updated by the copy): gradients once per pixel, then
// each front pixel's (C, D).  New terms go to global memory (for later
// iterations) and to LDS; then one wave per touched block recomputes its
// maximum, writes it, and folds it into the thread's running argmax.
// Block maxima of the refreshed window: 16 threads per touched block, 4 keys
// each, then a 16-lane reduction ((key, index) pairs are totally ordered, so
// any reduction order gives the same maximum); the block's first thread
// writes it to global memory and to s.bmk / s.bmi.
template <int R>
__device__ void block_maxima(const JobDev &d, const Refresh &g, LdsStage<R> &L, Scratch &s) {
    const int sub = threadIdx.x & 15, nb = g.nabx * g.naby;
    for (int b0 = 0; b0 < nb; b0 += blockDim.x >> 4) {
        const int b = b0 + (threadIdx.x >> 4);
        const int bx = g.abx0 + b % g.nabx, by = g.aby0 + b / g.nabx;
        int64_t bk = -1, bi = INT64_MAX;
        if (b < nb) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int e = sub + 16 * j;
                const int x = bx * kBlock + (e & 7), y = by * kBlock + (e >> 3);
                const int64_t k = in_img(d, x, y) ? L.bkey[b * 64 + e] : -1;
                const int64_t i = in_img(d, x, y) ? (int64_t)y * d.W + x : INT64_MAX;
                if (better(k, i, bk, bi)) {
                    bk = k;
                    bi = i;
                }
            }
        }
        row_argmax(bk, bi);   // the block's 16 threads are one DPP row
        if (b < nb && sub == 15) {
            d.blk[by * d.nbw + bx].key = bk;
            d.blk[by * d.nbw + bx].idx = bi;
            s.bmk[b] = bk;
            s.bmi[b] = bi;
        }
    }
}

// Front pixels of the refresh window go to a compact list so the costly
// evaluations fill whole waves (L.nfront must be 0 before; the caller's
// barrier publishes the list).  Pixels off the front already carry (C, D) =
// (-1, 0) in global memory and key -1 in LDS: a hole pixel off the front has
// never been on it (the front only gains hole pixels), a known one was set
// when it was filled (the copy) or at initialisation.
template <int R>
__device__ void list_front(int px, int py, const Refresh &g, LdsStage<R> &L) {
    using S = Stage<R>;
    const LdsView<R> v{L, px - S::half, py - S::half};
    const int ww = g.wx1 - g.wx0, nwin = ww * (g.wy1 - g.wy0);
    constexpr int WIN = LdsStage<R>::WIN;
    for (int t = threadIdx.x; t < nwin; t += blockDim.x) {
        const int x = g.wx0 + t % ww, y = g.wy0 + t / ww;
        const int wi = (y - (py - 2 * R - 1)) * WIN + (x - (px - 2 * R - 1));
        if (on_front(v, x, y)) L.front[atomicAdd(&L.nfront, 1)] = (int16_t)wi;
    }
}

// The search-independent half of a commit, run by the persistent committer
// while the search is still going: which pixels the copy fills (the hole
// pixels of the target patch) and the confidence they take (C of the
// target) do not depend on the source patch chosen.  So it marks them filled
// (hole map, confidence, off the front), lists the new front of the refresh
// window, and computes each front pixel's confidence term into L.wcd[wi].x.
// The raster-order FP64 sums are the same ones the full refresh computes.
// Only the copied colours, the gradients near the patch and the data terms
// wait for the search.  fb gets the patch slots to copy (bit t: dx = t % P
// - r, dy = t / P - r).  Only for the original source region with whole-patch
// scoring: there the candidate set never changes and context creation
// rejects an empty one, so the search always returns a source patch.
template <int R>
__device__ void precommit(const JobDev &d, const Snap &v, const Refresh &g, LdsStage<R> &L, uint32_t *fb) {
    using S = Stage<R>;
    constexpr int P = 2 * R + 1;
    const int W = d.W;
    const int px = col_of(v.p, W), py = row_of(v.p, W);
    if (threadIdx.x < kMaskWords) fb[threadIdx.x] = 0;
    if (threadIdx.x == 0) L.nfront = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < P * P; t += blockDim.x) {
        const int dx = t % P - R, dy = t / P - R;
        const int li = (dy + S::half) * S::side + (dx + S::half);
        if (L.st[li] == 1) {
            atomicOr(&fb[t >> 5], 1u << (t & 31));
            const int x = px + dx, y = py + dy;
            const int64_t dst = (int64_t)y * W + x;
            d.conf[dst] = v.C;
            d.hole[dst] = 0;
            d.pcd[dst] = make_double2(-1.0, 0.0);
            L.st[li] = 0;
            L.conf[li] = v.C;
            L.bkey[((y / kBlock - g.aby0) * g.nabx + (x / kBlock - g.abx0)) * 64 + (y & 7) * 8 + (x & 7)] = -1;
        }
    }
    __syncthreads();
    list_front<R>(px, py, g, L);
    __syncthreads();
    const LdsView<R> lv{L, px - S::half, py - S::half};
    constexpr int WIN = LdsStage<R>::WIN;
    const int nfront = L.nfront;
    for (int f = threadIdx.x; f < nfront; f += blockDim.x) {
        const int wi = L.front[f];
        const int x = px - 2 * R - 1 + wi % WIN, y = py - 2 * R - 1 + wi / WIN;
        L.wcd[wi].x = conf_sum_lds<R>(lv, x, y) / (double)(P * P);
    }
}

// Data terms of the listed front pixels (their C already in L.wcd[wi].x),
// in rounds of 64: wave w searches the gradient maxima of the w-th quarter
// of the patch rows; the quarters combine in row order, a later one winning
// only when strictly larger (the first-in-raster-order tie rule).
template <int R>
__device__ void refresh_data_terms(const JobDev &d, int px, int py, const Refresh &g, LdsStage<R> &L) {
    using S = Stage<R>;
    constexpr int P = 2 * R + 1, WIN = LdsStage<R>::WIN;
    const LdsView<R> v{L, px - S::half, py - S::half};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nfront = L.nfront;
    for (int f0 = 0; f0 < nfront; f0 += 64) {
        const int f = f0 + lane;
        if (f < nfront) {
            const int wi = L.front[f];
            const int x = px - 2 * R - 1 + wi % WIN, y = py - 2 * R - 1 + wi / WIN;
            int b, bg;
            grad_best_lds<R>(v, x, y, wave * P / 4, (wave + 1) * P / 4, &b, &bg);
            L.fbest[wave][lane] = b;
            L.fbxy[wave][lane] = bg;
        }
        __syncthreads();
        if (f < nfront && wave == 0) {
            const int wi = L.front[f];
            const int x = px - 2 * R - 1 + wi % WIN, y = py - 2 * R - 1 + wi / WIN;
            int best = L.fbest[0][lane], bxy = L.fbxy[0][lane];
#pragma unroll
            for (int q = 1; q < 4; ++q)
                if (L.fbest[q][lane] > best) {
                    best = L.fbest[q][lane];
                    bxy = L.fbxy[q][lane];
                }
            double2 cd;
            cd.x = L.wcd[wi].x;
            cd.y = data_term_lds<R>(v, x, y, bxy, d.norm1, d.norm2);
            d.pcd[(int64_t)y * d.W + x] = cd;
            L.wcd[wi] = cd;
            const int b = (y / kBlock - g.aby0) * g.nabx + (x / kBlock - g.abx0);
            L.bkey[b * 64 + (y & 7) * 8 + (x & 7)] = key_of(cd);
        }
        __syncthreads();
    }
}

template <int R, bool PRE = false>
__device__ void refresh_near(const JobDev &d, int px, int py, const Refresh &g, LdsStage<R> &L, Scratch &s) {
    using S = Stage<R>;
    const int ox = px - S::half, oy = py - S::half;
    const LdsView<R> v{L, ox, oy};
    if (!PRE && threadIdx.x == 0) L.nfront = 0;
    // The copy changed gradients only within one pixel of the patch; the
    // rest of the square was evaluated before it (grad_pass on the whole).
    __syncthreads();   // the copied pixels
    grad_pass<R>(L, S::half - R - 1, S::half + R + 2);
    __syncthreads();
    if (PRE) {
        // precommit listed the front and put each front pixel's C in
        // L.wcd[wi].x; only D needs the copied gray values.
        refresh_data_terms<R>(d, px, py, g, L);
        block_maxima<R>(d, g, L, s);
        return;
    }
    list_front<R>(px, py, g, L);
    __syncthreads();
    constexpr int WIN = LdsStage<R>::WIN;
    const int nfront = L.nfront;
    // Rounds of 64 front pixels.  The confidence sum (a serial FP64 chain)
    // runs in wave 0 and the gradient search in waves 2 (top rows) and 3
    // (bottom rows), one front pixel per lane, so each lane reads about a
    // third of a patch's LDS words.  The bottom half's best wins only when
    // strictly larger, which keeps the first-in-raster-order tie rule.
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int f0 = 0; f0 < nfront; f0 += 64) {
        const int f = f0 + lane;
        if (f < nfront && wave != 1) {
            const int wi = L.front[f];
            const int x = px - 2 * R - 1 + wi % WIN, y = py - 2 * R - 1 + wi / WIN;
            if (wave == 0) {
                L.fsum[lane] = conf_sum_lds<R>(v, x, y);
            } else {
                const int h = wave - 2;
                int b, bg;
                grad_best_lds<R>(v, x, y, h ? R + 1 : 0, h ? 2 * R + 1 : R + 1, &b, &bg);
                L.fbest[h][lane] = b;
                L.fbxy[h][lane] = bg;
            }
        }
        __syncthreads();
        if (f < nfront && wave == 0) {
            const int wi = L.front[f];
            const int x = px - 2 * R - 1 + wi % WIN, y = py - 2 * R - 1 + wi / WIN;
            const int bxy = L.fbest[1][lane] > L.fbest[0][lane] ? L.fbxy[1][lane] : L.fbxy[0][lane];
            double2 cd;
            cd.x = L.fsum[lane] / (double)((2 * R + 1) * (2 * R + 1));
            cd.y = data_term_lds<R>(v, x, y, bxy, d.norm1, d.norm2);
            d.pcd[(int64_t)y * d.W + x] = cd;
            L.wcd[wi] = cd;
            const int b = (y / kBlock - g.aby0) * g.nabx + (x / kBlock - g.abx0);
            L.bkey[b * 64 + (y & 7) * 8 + (x & 7)] = key_of(cd);
        }
        __syncthreads();
    }
    block_maxima<R>(d, g, L, s);
}

// Stages the next target (nx, ny) from the LDS neighbourhood of the filled
// target (px, py); valid when the whole patch lies inside it.
template <int R>
__device__ __forceinline__ int stage_target_lds(const LdsStage<R> &L, int px, int py, int tx, int ty, TargetStage *tg,
                                                Scratch &s, FillSync *recs = nullptr) {
    using S = Stage<R>;
    constexpr int P = 2 * R + 1;
    return stage_slots(R, tx, ty, tg, s, recs, [&](int t, uint32_t *pix) {
        const int i = (ty + t % P - R - py + S::half) * S::side + (tx + t / P - R - px + S::half);
        if (L.st[i] != 0) return false;
        *pix = L.img[i] & 0x00ffffffu;
        return true;
    });
}

}  // namespace

// ----------------------------------------------------------------- kernels

__global__ void k_init_info(InitInfo *info, uint32_t nonce) {
    info->hole_count = 0;
    info->bad = 0;
    info->bx0 = INT32_MAX;
    info->by0 = INT32_MAX;
    info->bx1 = INT32_MIN;
    info->by1 = INT32_MIN;
    info->valid_count = 0;
    info->nonce = nonce;
    info->seal = 0;
    info->blocks = 0;
}

__global__ void k_seal(InitInfo *info, uint32_t nonce) { info->seal = nonce; }

// Initialisation: zero the hole pixels, RGBX image, integer BT.601 gray
// (299 R + 587 G + 114 B + 500) div 1000, hole map, confidence 1 / 0, hole
// count and bounding box.
__global__ __launch_bounds__(256) void k_init_pixels(JobDev d, const uint8_t *rgb, int ch,
                                                     const uint8_t *mask) {
    const int64_t n = (int64_t)d.W * d.H;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    __shared__ int s_cnt, s_x0, s_y0, s_x1, s_y1;
    if (threadIdx.x == 0) {
        s_cnt = 0;
        s_x0 = INT32_MAX;
        s_y0 = INT32_MAX;
        s_x1 = INT32_MIN;
        s_y1 = INT32_MIN;
    }
    __syncthreads();
    if (i < n) {
        const int x = col_of(i, d.W), y = row_of(i, d.W);
        const bool h = mask[i] != 0;
        const uint32_t R = h ? 0 : rgb[i * ch], G = h ? 0 : rgb[i * ch + 1],
                       B = h ? 0 : rgb[i * ch + 2];
        d.img[i] = R | (G << 8) | (B << 16);
        d.gray[i] = (uint8_t)((299 * R + 587 * G + 114 * B + 500) / 1000);
        d.hole[i] = h ? 1 : 0;
        d.hole0[i] = h ? 1 : 0;
        d.conf[i] = h ? 0.0 : 1.0;
        if (h) {
            atomicAdd(&s_cnt, 1);
            atomicMin(&s_x0, x);
            atomicMin(&s_y0, y);
            atomicMax(&s_x1, x + 1);
            atomicMax(&s_y1, y + 1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt > 0) {
        atomicAdd((unsigned long long *)&d.info->hole_count, (unsigned long long)s_cnt);
        atomicMin(&d.info->bx0, s_x0);
        atomicMin(&d.info->by0, s_y0);
        atomicMax(&d.info->bx1, s_x1);
        atomicMax(&d.info->by1, s_y1);
    }
    if (threadIdx.x == 0) atomicAdd(&d.info->blocks, 1u);
}

// ---- checkpoint import (resume / iterative editing) ------------------------

// Counts the pixels of a checkpoint that fail its checks: a hole pixel
// outside the original hole, or a filled pixel of the original hole whose
// confidence is not in [0, 1] (NaN included).  Writes nothing else.
__global__ __launch_bounds__(256) void k_import_check(JobDev d, const uint8_t *hole, const double *conf) {
    const int64_t n = (int64_t)d.W * d.H;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (i < n) {
        const bool h = hole[i] != 0, h0 = d.hole0[i] != 0;
        const double c = conf[i];
        bad = (h && !h0) || (h0 && !h && !(c >= 0.0 && c <= 1.0));
    }
    if (bad) atomicAdd((unsigned long long *)&d.info->bad, 1ull);
    if (threadIdx.x == 0) atomicAdd(&d.info->blocks, 1u);
}

// Overlays a checked checkpoint on the original-hole pixels: those still in
// its hole become hole again (zeroed), the others take its colour, the gray
// value of that colour and its confidence.  Other pixels keep their values.
__global__ __launch_bounds__(256) void k_import_apply(JobDev d, const uint8_t *rgb, int ch, const uint8_t *hole,
                                                      const double *conf) {
    const int64_t n = (int64_t)d.W * d.H;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    __shared__ int s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    if (i < n && d.hole0[i]) {
        const bool h = hole[i] != 0;
        const uint32_t R = h ? 0 : rgb[i * ch], G = h ? 0 : rgb[i * ch + 1], B = h ? 0 : rgb[i * ch + 2];
        d.img[i] = R | (G << 8) | (B << 16);
        d.gray[i] = (uint8_t)((299 * R + 587 * G + 114 * B + 500) / 1000);
        d.hole[i] = h ? 1 : 0;
        d.conf[i] = h ? 0.0 : conf[i];
        if (h) atomicAdd(&s_cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt > 0) atomicAdd((unsigned long long *)&d.info->hole_count, (unsigned long long)s_cnt);
    if (threadIdx.x == 0) atomicAdd(&d.info->blocks, 1u);
}

__global__ void k_import_reset(InitInfo *info, uint32_t nonce) {
    info->hole_count = 0;
    info->bad = 0;
    info->nonce = nonce;
    info->seal = 0;
    info->blocks = 0;
}

// Horizontal distance (capped at 10) from each pixel to the nearest hole or
// out-of-image pixel of its row.
__global__ __launch_bounds__(256) void k_init_hdist(JobDev d, uint8_t *hdist) {
    const int64_t n = (int64_t)d.W * d.H;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = col_of(i, d.W), y = row_of(i, d.W);
    int h = 10;
    for (int dx = 0; dx < 10; ++dx) {
        const int xl = x - dx, xr = x + dx;
        if (xl < 0 || xr >= d.W || d.hole[(int64_t)y * d.W + xl] || d.hole[(int64_t)y * d.W + xr]) {
            h = dx;
            break;
        }
    }
    hdist[i] = (uint8_t)h;
}

// vrad = (Chebyshev distance to the nearest hole or out-of-image pixel) - 1,
// clamped to [0, 8]: the patch of radius r at a centre lies inside the image
// and the original known region iff vrad >= r.
__global__ __launch_bounds__(256) void k_init_vrad(JobDev d, const uint8_t *hdist) {
    const int64_t n = (int64_t)d.W * d.H;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = col_of(i, d.W), y = row_of(i, d.W);
    int dist = 10;
    for (int dy = -9; dy <= 9; ++dy) {
        const int yy = y + dy, ady = dy < 0 ? -dy : dy;
        const int h = (yy < 0 || yy >= d.H) ? 0 : hdist[(int64_t)yy * d.W + x];
        const int m = ady > h ? ady : h;
        dist = m < dist ? m : dist;
    }
    int v = dist - 1;
    v = v < 0 ? 0 : (v > kMaxRadius ? kMaxRadius : v);
    d.vrad[i] = (uint8_t)v;
}

// Search planes: the original image (hole pixels zero) and vrad in the
// zero-padded layout the search stages from.  With INTERSECT scoring the 4th
// byte of a source pixel's word is 1 and the validity plane only flags
// source pixels (a candidate centre needs to be one).
__global__ __launch_bounds__(256) void k_init_padded(JobDev d) {
    const int pitch = d.pitch;
    const int64_t n = (int64_t)pitch * padded_rows(d.H);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = (int)(i % pitch) - kPadL, y = (int)(i / pitch) - kPadT;
    uint32_t pix = 0;
    uint8_t vr = 0;
    if (x >= 0 && x < d.W && y >= 0 && y < d.H) {
        pix = d.img[(int64_t)y * d.W + x];
        vr = d.vrad[(int64_t)y * d.W + x];
        if (d.isect) {
            const bool src = d.hole[(int64_t)y * d.W + x] == 0;
            pix |= src ? 1u << 24 : 0u;
            vr = src ? 1 : 0;
        }
    }
    d.srcp[i] = pix;
    d.vradp[i] = vr;
}

// Number of valid source centres in the search rectangle.
__global__ __launch_bounds__(256) void k_count_valid(JobDev d) {
    const int rw = d.rx1 - d.rx0;
    const int64_t n = (int64_t)rw * (d.ry1 - d.ry0);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    __shared__ int s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    if (i < n) {
        const int x = d.rx0 + (int)(i % rw), y = d.ry0 + (int)(i / rw);
        const int64_t j = (int64_t)y * d.W + x;
        if (d.isect ? d.hole[j] == 0 : d.vrad[j] >= d.r) atomicAdd(&s_cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt)
        atomicAdd((unsigned long long *)&d.info->valid_count, (unsigned long long)s_cnt);
}

// Priority terms and block maxima of every block of the priority range; one
// wave per 8x8 block.
template <int R>
__global__ __launch_bounds__(256) void k_prio_init(JobDev d) {
    const int bw = d.pbx1 - d.pbx0, nb = bw * (d.pby1 - d.pby0);
    const int b = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (b >= nb) return;
    const int bx = d.pbx0 + b % bw, by = d.pby0 + b / bw;
    const int lane = threadIdx.x & 63;
    const int x = bx * kBlock + (lane & (kBlock - 1)), y = by * kBlock + lane / kBlock;
    const GlobalView v{d};
    if (in_img(d, x, y)) d.pcd[(int64_t)y * d.W + x] = pixel_terms<R>(v, d, x, y);
    refresh_block_wave(d, bx, by);   // same wave: its own writes are visible
}

// Issues every global load the commit needs that does not depend on the
// search result -- the target's neighbourhood, the cached keys of the touched
// blocks, the block maxima of the priority range and the search partials --
// before consuming any of them, so together they cost about one memory round
// trip.  Leaves the neighbourhood and the block keys in LDS, the running
// argmax over the untouched blocks in (key, idx), and returns the minimum
// search key of this thread's partials.
// BW: priority-block loads per thread issued with the first batch (the whole
// range of a hole up to BW * 256 blocks); TB: loads in flight per round trip
// for the rest.
template <int R, bool PARTIALS, int TB = 8, int BW = 4>
__device__ uint64_t gather(const JobDev &d, int px, int py, const Refresh &g, LdsStage<R> &L, int64_t &key,
                           int64_t &idx) {
    using S = Stage<R>;
    constexpr int T = kCommitThreads;
    constexpr int NIT = (S::n + T - 1) / T;
    constexpr int KIT = (LdsStage<R>::NBA * LdsStage<R>::NBA * 64 + T - 1) / T;
    constexpr int BIT = PARTIALS ? 16 : BW, PIT = PARTIALS ? 8 : 0;
    const int ox = px - S::half, oy = py - S::half;
    const int nkeys = g.nabx * g.naby * 64;
    const int bw = d.pbx1 - d.pbx0, nb = bw * (d.pby1 - d.pby0);
    const int ntiles = d.ntx * d.nty;
    const int tid = threadIdx.x;

    uint8_t h[NIT], gv[NIT];
    double c[NIT];
    uint32_t im[NIT];
    double2 cd[KIT];
    BlockBest bb[BIT];
    uint64_t pv[PIT > 0 ? PIT : 1];
    // ---- issue (all unconditional, from clamped addresses)
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
        const int t = min(tid + k * T, S::n - 1);
        const int x = min(max(ox + t % S::side, 0), d.W - 1), y = min(max(oy + t / S::side, 0), d.H - 1);
        const int64_t i = (int64_t)y * d.W + x;
        h[k] = d.hole[i];
        gv[k] = d.gray[i];
        c[k] = d.conf[i];
        im[k] = d.img[i];
    }
#pragma unroll
    for (int k = 0; k < KIT; ++k) {
        const int t = min(tid + k * T, nkeys - 1);
        const int b = t >> 6, lane = t & 63;
        const int x = min((g.abx0 + b % g.nabx) * kBlock + (lane & 7), d.W - 1);
        const int y = min((g.aby0 + b / g.nabx) * kBlock + (lane >> 3), d.H - 1);
        cd[k] = d.pcd[(int64_t)y * d.W + x];
    }
#pragma unroll
    for (int k = 0; k < BIT; ++k) {
        const int t = min(tid + k * T, nb - 1);
        bb[k] = d.blk[(d.pby0 + t / bw) * d.nbw + d.pbx0 + t % bw];
    }
#pragma unroll
    for (int k = 0; k < PIT; ++k) pv[k] = d.partials[min(tid + k * T, ntiles - 1)];
    (void)pv;

    // ---- consume
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
        const int t = tid + k * T;
        if (t < S::n) {
            const int x = ox + t % S::side, y = oy + t / S::side;
            const bool in = in_img(d, x, y);
            L.st[t] = !in ? 2 : (h[k] ? 1 : 0);
            L.gray[t] = gv[k];
            L.conf[t] = (in && !h[k]) ? c[k] : 0.0;   // C of known pixels, +0.0 elsewhere
            L.img[t] = im[k];
        }
    }
#pragma unroll
    for (int k = 0; k < KIT; ++k) {
        const int t = tid + k * T;
        if (t < nkeys) {
            const int b = t >> 6, lane = t & 63;
            const int x = (g.abx0 + b % g.nabx) * kBlock + (lane & 7), y = (g.aby0 + b / g.nabx) * kBlock + (lane >> 3);
            L.bkey[t] = in_img(d, x, y) ? key_of(cd[k]) : -1;
        }
    }
    auto take_block = [&](int t, const BlockBest &b) {
        const int bx = d.pbx0 + t % bw, by = d.pby0 + t / bw;
        const bool touched = bx >= g.abx0 && bx < g.abx0 + g.nabx && by >= g.aby0 && by < g.aby0 + g.naby;
        if (t < nb && !touched && better(b.key, b.idx, key, idx)) {
            key = b.key;
            idx = b.idx;
        }
    };
#pragma unroll
    for (int k = 0; k < BIT; ++k) take_block(tid + k * T, bb[k]);
    uint64_t best = ~0ull;
#pragma unroll
    for (int k = 0; k < PIT; ++k) best = pv[k] < best ? pv[k] : best;   // clamped repeats are harmless

    // ---- tails of large holes / rectangles, TB loads in flight per round
    // trip (the arrays above are dead by now, so their registers are free);
    // the argmax is order-independent (a strict total order)
    for (int t0 = tid + BIT * T; t0 < nb; t0 += TB * T) {
        BlockBest tb[TB];
#pragma unroll
        for (int q = 0; q < TB; ++q) {
            const int t = min(t0 + q * T, nb - 1);
            tb[q] = d.blk[(d.pby0 + t / bw) * d.nbw + d.pbx0 + t % bw];
        }
#pragma unroll
        for (int q = 0; q < TB; ++q) take_block(t0 + q * T, tb[q]);   // t >= nb is skipped there
    }
    if (PARTIALS) {
        for (int t0 = tid + PIT * T; t0 < ntiles; t0 += TB * T) {
            uint64_t tp[TB];
#pragma unroll
            for (int q = 0; q < TB; ++q) tp[q] = d.partials[min(t0 + q * T, ntiles - 1)];
#pragma unroll
            for (int q = 0; q < TB; ++q) best = tp[q] < best ? tp[q] : best;   // clamped repeats are harmless
        }
    }
    return best;
}

// A copy of one target patch in LDS (slot order as stage_target), with its
// centre's raster index (-1: none).
template <int R>
struct PatchCopy {
    uint32_t pix[(2 * R + 1) * (2 * R + 1)];
    uint8_t known[(2 * R + 1) * (2 * R + 1)];
    int64_t idx;
};

// The patch at raster index idx in registers: load_patch() issues the loads
// (hole byte and word together, from clamped addresses) without waiting for
// them, so they stay in flight across other work; store_patch() then writes
// the copy to *c (idx < 0: none; whole group, the caller's next barrier
// publishes it).
template <int R>
struct PatchLoad {
    static constexpr int P = 2 * R + 1, N = (P * P + kCommitThreads - 1) / kCommitThreads;
    uint32_t pix[N];
    uint8_t hole[N];
};

template <int R>
__device__ __forceinline__ PatchLoad<R> load_patch(const JobDev &d, int64_t idx) {
    constexpr int P = 2 * R + 1;
    PatchLoad<R> f{};
    if (idx < 0) return f;
    const int tx = col_of(idx, d.W), ty = row_of(idx, d.W);
#pragma unroll
    for (int j = 0; j < PatchLoad<R>::N; ++j) {
        const int t = min((int)threadIdx.x + j * kCommitThreads, P * P - 1);
        const int x = min(max(tx + t / P - R, 0), d.W - 1), y = min(max(ty + t % P - R, 0), d.H - 1);
        const int64_t i = (int64_t)y * d.W + x;
        f.hole[j] = d.hole[i];
        f.pix[j] = d.img[i];
    }
    return f;
}

template <int R>
__device__ __forceinline__ void store_patch(const JobDev &d, int64_t idx, const PatchLoad<R> &f, PatchCopy<R> *c) {
    constexpr int P = 2 * R + 1;
    if (threadIdx.x == 0) c->idx = idx;
    if (idx < 0) return;
    const int tx = col_of(idx, d.W), ty = row_of(idx, d.W);
#pragma unroll
    for (int j = 0; j < PatchLoad<R>::N; ++j) {
        const int t = (int)threadIdx.x + j * kCommitThreads;
        if (t < P * P) {
            const int x = tx + t / P - R, y = ty + t % P - R;
            const bool kn = in_img(d, x, y) && f.hole[j] == 0;
            c->known[t] = kn ? 1 : 0;
            c->pix[t] = kn ? f.pix[j] & 0x00ffffffu : 0u;
        }
    }
}

// What the stream-form commit reports about its copy: the target and the
// number of pixels filled (nf counts them under INTERSECT scoring).
struct CommitNote {
    int64_t p;
    int32_t filled;
    int32_t nf;
};

// CURRENT source policy: the pixels this iteration filled become source
// pixels.  Writes their words into the padded source plane and brings the
// validity planes up to date around the patch: the horizontal distances of
// the patch rows, then the validity radii of every centre whose radius can
// have changed (as k_init_hdist / k_init_vrad compute them).  The hole map
// changed only inside the patch, which the LDS neighbourhood holds; every
// other pixel is read from device memory, unchanged since earlier launches.
template <int R, bool ISECT>
__device__ void add_filled_sources(const JobDev &d, const LdsStage<R> &L, int px, int py) {
    constexpr int P = 2 * R + 1, half = Stage<R>::half, side = Stage<R>::side;
    constexpr int HW = 2 * R + 19;   // columns px - R - 9 .. px + R + 9
    const int W = d.W, H = d.H, pitch = d.pitch;
    auto known = [&](int x, int y) -> bool {
        if ((unsigned)x >= (unsigned)W || (unsigned)y >= (unsigned)H) return false;
        const int lx = x - px + half, ly = y - py + half;
        if ((unsigned)lx < (unsigned)side && (unsigned)ly < (unsigned)side) return L.st[ly * side + lx] == 0;
        return d.hole[(int64_t)y * W + x] == 0;
    };
    // the patch's known pixels (rewriting the unchanged ones is harmless)
    for (int t = threadIdx.x; t < P * P; t += blockDim.x) {
        const int x = px + t % P - R, y = py + t / P - R;
        if (!known(x, y)) continue;
        const int64_t pi = (int64_t)(y + kPadT) * pitch + (x + kPadL);
        d.srcp[pi] = L.img[(y - py + half) * side + (x - px + half)] | (ISECT ? 1u << 24 : 0u);
        if (ISECT) d.vradp[pi] = 1;
    }
    if (ISECT) return;   // INTERSECT candidates only need their centre to be a source pixel
    __shared__ uint8_t hrow[P * HW];
    for (int t = threadIdx.x; t < P * HW; t += blockDim.x) {
        const int x = px - R - 9 + t % HW, y = py - R + t / HW;
        uint8_t h = 0;
        if ((unsigned)x < (unsigned)W && (unsigned)y < (unsigned)H) {
            int hh = 10;
            for (int dx = 0; dx < 10; ++dx)
                if (!known(x - dx, y) || !known(x + dx, y)) {
                    hh = dx;
                    break;
                }
            h = (uint8_t)hh;
            d.hdist[(int64_t)y * W + x] = h;
        }
        hrow[t] = h;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < HW * HW; t += blockDim.x) {
        const int x = px - R - 9 + t % HW, y = py - R - 9 + t / HW;
        if ((unsigned)x >= (unsigned)W || (unsigned)y >= (unsigned)H) continue;
        int dist = 10;
        for (int dy = -9; dy <= 9; ++dy) {
            const int yy = y + dy, ady = dy < 0 ? -dy : dy;
            int h;
            if (yy < 0 || yy >= H) h = 0;
            else if (yy >= py - R && yy <= py + R) h = hrow[(yy - py + R) * HW + (x - px + R + 9)];
            else h = d.hdist[(int64_t)yy * W + x];
            const int m = ady > h ? ady : h;
            dist = m < dist ? m : dist;
        }
        int v = dist - 1;
        v = v < 0 ? 0 : (v > kMaxRadius ? kMaxRadius : v);
        d.vrad[(int64_t)y * W + x] = (uint8_t)v;
        d.vradp[(int64_t)(y + kPadT) * pitch + (x + kPadL)] = (uint8_t)v;
    }
}

// The part of a fill iteration that needs the search result `best`: copy the
// source patch into the target's hole pixels (they take the target's
// confidence), log, refresh priorities near the patch, select and stage the
// next target.  (key, idx) is the running argmax over the untouched blocks
// from gather(), whose LDS neighbourhood it consumes.  Thread 0 writes the
// new loop state to *out; the caller publishes it with a barrier.
//
// After the copy everything runs out of LDS; the next target is staged from
// LDS when its patch lies inside the staged neighbourhood (the common case:
// the front moves locally).  (key0, idx0) is the argmax over the blocks the
// refresh does not touch (block-uniform).
//
// PRE: precommit() already marked the patch's hole pixels filled (fb lists
// them), listed the new front and computed its confidence terms; only the
// colours are copied here.
template <int R, bool ISECT = false, bool PRE = false, bool LEAN = false>
__device__ void commit_finish(const JobDev &d, Scratch &s, LdsStage<R> &L, const Snap &v, uint64_t best,
                              const Refresh &g, int64_t key0, int64_t idx0, Snap *out, FillSync *recs = nullptr,
                              CommitNote *note = nullptr, const PatchCopy<R> *far = nullptr,
                              const uint32_t *fb = nullptr) {
    IterState *st = d.st;
    constexpr int P = 2 * R + 1;
    const int W = d.W;
    const int px = col_of(v.p, W), py = row_of(v.p, W);
    Snap n = v;
    if (best == ~0ull) {
        if (threadIdx.x == 0) {
            st->error = INPAINT_NO_CANDIDATE;
            n.err = INPAINT_NO_CANDIDATE;
            *out = n;
        }
        return;
    }

    // ---- copy the source patch
    const int64_t q = (int64_t)(best & 0xffffffffu);
    const uint32_t ssd = (uint32_t)(best >> 32);
    const int qx = col_of(q, W), qy = row_of(q, W);
    // the hole pixels of the target patch: its in-image pixels minus the known k
    // (with INTERSECT scoring only those whose source pixel is a source pixel
    // are filled, counted as they are copied)
    int64_t filled = (int64_t)(min(px + R + 1, W) - max(px - R, 0)) * (min(py + R + 1, d.H) - max(py - R, 0)) - v.k;
    if (ISECT) {
        if (threadIdx.x == 0) note->nf = 0;
        __syncthreads();
    }
    for (int t = threadIdx.x; t < P * P; t += blockDim.x) {
        const int dx = t % P - R, dy = t / P - R;
        const int li = (dy + Stage<R>::half) * Stage<R>::side + (dx + Stage<R>::half);
        if (PRE) {
            if ((fb[t >> 5] >> (t & 31)) & 1) {
                const int64_t dst = (int64_t)(py + dy) * W + (px + dx), src = (int64_t)(qy + dy) * W + (qx + dx);
                const uint32_t pix = d.img[src];
                const uint8_t gv = d.gray[src];
                d.img[dst] = pix;
                d.gray[dst] = gv;
                L.img[li] = pix;
                L.gray[li] = gv;
            }
        } else if (L.st[li] == 1) {
            if (ISECT) {
                // the flag byte of the source word, read before any of this
                // copy's writes (the padded plane covers R pixels around the image)
                const uint32_t sw = d.srcp[(int64_t)(qy + dy + kPadT) * d.pitch + (qx + dx + kPadL)];
                if ((sw >> 24) == 0) continue;
                atomicAdd(&note->nf, 1);
            }
            const int64_t dst = (int64_t)(py + dy) * W + (px + dx), src = (int64_t)(qy + dy) * W + (qx + dx);
            const uint32_t pix = d.img[src];
            const uint8_t gv = d.gray[src];
            d.img[dst] = pix;
            d.gray[dst] = gv;
            d.conf[dst] = v.C;
            d.hole[dst] = 0;
            L.st[li] = 0;
            L.img[li] = pix;
            L.gray[li] = gv;
            L.conf[li] = v.C;
            // off the front from now on
            const int x = px + dx, y = py + dy;
            d.pcd[dst] = make_double2(-1.0, 0.0);
            L.bkey[((y / kBlock - g.aby0) * g.nabx + (x / kBlock - g.abx0)) * 64 + (y & 7) * 8 + (x & 7)] = -1;
        }
    }
    if (ISECT) {
        __syncthreads();
        filled = note->nf;
    }
    if (note && threadIdx.x == 0) {
        note->p = v.p;
        note->filled = (int32_t)filled;
    }
    const int64_t remaining = v.remaining - filled;
    if (threadIdx.x == 0) {
        StepRec rec;
        rec.target_index = v.p;
        rec.source_index = q;
        rec.ssd = ssd;
        rec.known_k = v.k;
        rec.n_filled = (int32_t)filled;
        rec.reserved = 0;
        rec.priority = v.Pr;
        rec.confidence = v.C;
        rec.data_term = v.D;
        rec.remaining = remaining;
        if (v.iter < d.log_cap) d.log[v.iter] = rec;
        st->last = rec;
        st->remaining = remaining;
        st->iter = v.iter + 1;
        st->pending = 0;
        if (remaining == 0) st->done = 1;
        n.iter = v.iter + 1;
        n.remaining = remaining;
        n.pending = 0;
        n.done = remaining == 0 ? 1 : 0;
    }
    if (remaining == 0) {
        if (threadIdx.x == 0) *out = n;
        return;
    }

    // ---- priorities near the patch, block maxima, argmax: wave 0 reduces
    // the touched blocks' maxima and (key0, idx0)
    refresh_near<R, PRE>(d, px, py, g, L, s);
    __syncthreads();
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x, nb = g.nabx * g.naby;
        int64_t k2 = lane < nb ? s.bmk[lane] : (lane == 63 ? key0 : -1);
        int64_t i2 = lane < nb ? s.bmi[lane] : (lane == 63 ? idx0 : INT64_MAX);
        wave_argmax(k2, i2);
        if (lane == 0) {
            s.k[0] = k2;
            s.i[0] = i2;
        }
    }
    __syncthreads();
    const int64_t key = s.k[0], idx = s.i[0];
    if (key < 0) {
        // No front pixel although the hole is not empty: cannot happen for a
        // valid state; flag it instead of looping.
        if (threadIdx.x == 0) {
            st->error = INPAINT_DEVICE;
            n.err = INPAINT_DEVICE;
            *out = n;
        }
        return;
    }

    // ---- stage the next target
    const int tx = col_of(idx, W), ty = row_of(idx, W);
    const int adx = abs(tx - px), ady = abs(ty - py);
    int kk;
    if (LEAN) {
        // (the same three sources of the patch as below)
        using S = Stage<R>;
        constexpr int P = 2 * R + 1;
        if (adx <= 2 * R + 2 && ady <= 2 * R + 2) {
            kk = stage_slots_lean(R, tx, ty, d.tgt, s, recs, rec_tag(v.iter + 1), [&](int t, uint32_t *pix) {
                const int i = (ty + t % P - R - py + S::half) * S::side + (tx + t / P - R - px + S::half);
                if (L.st[i] != 0) return false;
                *pix = L.img[i] & 0x00ffffffu;
                return true;
            });
        } else if (far && far->idx == idx) {
            kk = stage_slots_lean(R, tx, ty, d.tgt, s, recs, rec_tag(v.iter + 1), [&](int t, uint32_t *pix) {
                *pix = far->pix[t];
                return far->known[t] != 0;
            });
        } else {
            const GlobalView gv{d};
            kk = stage_slots_lean(R, tx, ty, d.tgt, s, recs, rec_tag(v.iter + 1), [&](int t, uint32_t *pix) {
                const int x = tx + t / P - R, y = ty + t % P - R;
                if (!gv.known(x, y)) return false;
                *pix = d.img[(int64_t)y * d.W + x] & 0x00ffffffu;
                return true;
            });
        }
    } else if (adx <= 2 * R + 2 && ady <= 2 * R + 2) {
        kk = stage_target_lds<R>(L, px, py, tx, ty, d.tgt, s, recs);
    } else if (far && far->idx == idx) {
        // the best pixel of the untouched blocks, copied before this
        // iteration's search ended: its patch is at least 2r + 2 pixels from
        // the filled one, so the copy did not change it
        kk = stage_slots(R, tx, ty, d.tgt, s, recs, [&](int t, uint32_t *pix) {
            *pix = far->pix[t];
            return far->known[t] != 0;
        });
    } else {
        kk = stage_target(d, tx, ty, R, d.tgt, s, recs);
    }
    if (threadIdx.x == 0) {
        double2 cd;
        if (adx <= 2 * R + 1 && ady <= 2 * R + 1)
            cd = L.wcd[(ty - (py - 2 * R - 1)) * LdsStage<R>::WIN + (tx - (px - 2 * R - 1))];
        else
            cd = d.pcd[idx];
        st->p_idx = idx;
        st->C = cd.x;
        st->D = cd.y;
        st->Pr = cd.x * cd.y;
        st->pending = 1;
        n.p = idx;
        n.C = cd.x;
        n.D = cd.y;
        n.Pr = cd.x * cd.y;
        n.pending = 1;
        n.k = kk;
        *out = n;
    }
}

// One fill iteration after the search: reduce the search partials and
// finish.  With no staged target (right after create) it only selects and
// stages.  Latency is the cost here, so every global load that does not
// depend on the search result is issued at once up front (gather).
template <int R, bool ISECT = false>
__device__ void commit_body(const JobDev &d, Scratch &s, LdsStage<R> &L, CommitNote *note = nullptr) {
    const Snap v = load_snap(d.st, d.tgt);
    if (v.done || v.err) return;
    if (!v.pending) {
        select_and_stage(d, s);
        return;
    }
    if (v.iter >= v.limit) return;
    const int px = col_of(v.p, d.W), py = row_of(v.p, d.W);
    const Refresh g = refresh_geometry<R>(d, px, py);
    int64_t key = -1, idx = INT64_MAX;
    uint64_t best = gather<R, true>(d, px, py, g, L, key, idx);
    best = block_min_u64(best, s.u);   // its barriers also publish the LDS stores
    grad_pass<R>(L, 1, Stage<R>::side - 1);
    block_argmax(key, idx, s.k, s.i);
    commit_finish<R, ISECT>(d, s, L, v, best, g, key, idx, &s.snap, nullptr, note);
}

// ---- persistent fill: one dispatch runs many iterations ------------------
//
// Work-group 0 commits; work-group 1 + t owns search tile t for the whole
// dispatch, staged in LDS once (its source pixels never change).  Per
// iteration k: the committer publishes go = (epoch, k + 1) once target k is
// staged; every search group copies the target to LDS, scores its tile and
// writes its minimum key, tagged with k, to its own slot; meanwhile the committer
// issues the search-independent loads of the commit (gather).  When every
// slot carries iteration k's tag it reduces the keys and finishes the
// iteration.  go carries the launch epoch, so values left by an earlier
// dispatch never match.  Every wait is bounded: a search group gives up
// after kSpinLimit polls; the committer then flags a device error and
// publishes stop, and every group exits.

constexpr uint32_t kSpinLimit = 1u << 22;

// Go words: the launch epoch in the high half; in the low half either stop
// (all ones) or k + 1 (k < 2^25 - 1, the dispatch's iteration) in bits 0-24
// with the record tag of that iteration (lean records; 0 otherwise) in bits
// 25-31.
constexpr uint32_t kGoK = (1u << 25) - 1;
__device__ __forceinline__ uint64_t go_word(uint32_t epoch, uint32_t k1, uint32_t tag = 0) {
    return ((uint64_t)epoch << 32) | (tag << 25) | k1;
}
__device__ __forceinline__ uint64_t go_stop(uint32_t epoch) { return ((uint64_t)epoch << 32) | 0xffffffffu; }
__device__ __forceinline__ bool go_is(uint64_t v, uint32_t epoch, uint32_t k1) {
    return (v >> 32) == epoch && (uint32_t)v != 0xffffffffu && (v & kGoK) == k1;
}
__device__ __forceinline__ uint32_t go_tag(uint64_t v) { return (uint32_t)(v >> 25) & 0x7fu; }

// Thread 0 of search group t: 1 once target k is staged, 0 on stop or time-out.
//
// Ordering of the record reads after the go word (hardware, not the language
// memory model): the committer writes the record, waits for its stores
// (s_waitcnt) and releases the go word at agent scope, which writes the L2
// back first.  Here the go word is polled with relaxed agent-scope loads;
// the caller's barrier follows the matching load's completion, and every
// record word is then read with an agent-scope load too, which is coherent
// at device scope (it does not hit a stale copy in the CU's L1 or an XCD's
// L2).  So the reads observe the record.  An agent-scope acquire fence
// after the match would make this a language-level guarantee, but on gfx950
// it invalidates caches for every search group on every iteration: it was
// measured to slow the 1080p removal from 49.2 ms to 61.4 ms.  (The MFMA
// form does not depend on this order: its lean records tag every word with
// the iteration, and its search groups check the tag of each word they use
// and read stale words again.)
__device__ int wait_go(const FillSync *sy, int t, uint32_t epoch, uint32_t k) {
    const uint64_t stop = go_stop(epoch);
    const uint64_t *g = &sy->rec[t % kGoCopies].go;
    for (uint32_t spin = 0; spin < kSpinLimit; ++spin) {
        const uint64_t v = __hip_atomic_load(g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (go_is(v, epoch, k + 1)) return 1;
        if (v == stop) return 0;
        __builtin_amdgcn_s_sleep(1);
    }
    return 0;
}

// Committer (all threads, after a barrier): writes every copy of the go word.
__device__ __forceinline__ void publish_go(FillSync *sy, uint64_t word) {
    if (threadIdx.x < kGoCopies)
        __hip_atomic_store(&sy->rec[threadIdx.x].go, word, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t slot_tag(uint32_t k) { return k % 255u + 1u; }

__device__ __forceinline__ uint64_t slot_word(uint64_t key, uint32_t tag) {
    if (key == ~0ull) return (~0ull << 8) | tag;
    const uint64_t ssd = key >> 32, idx = key & 0xffffffffu;
    return (ssd << (kSlotIndexBits + 8)) | (idx << 8) | tag;
}

// Committer (all threads): waits until every search slot carries `tag`, then
// returns the minimum search key (block-wide, ~0 if no tile had a valid
// candidate), or sets *ok = 0 on time-out.  Each slot word is self-contained,
// so plain device-scope loads suffice (no acquire, no cache invalidation).
__device__ uint64_t collect_slots(const uint64_t *fs, int ntiles, uint32_t tag, Scratch &s, int *ok) {
    constexpr int T = kCommitThreads;
    const int per = (ntiles + T - 1) / T;           // slots of this thread: tid + T j
    uint32_t pend = 0;
    for (int j = 0; j < per && j < 32; ++j)
        if ((int)threadIdx.x + T * j < ntiles) pend |= 1u << j;
    uint64_t best = ~0ull;   // minimum of (word >> 8)
    // Each thread polls its own slots (no barrier per round), so the last
    // report is seen one load latency after it lands.
    for (uint32_t spin = 0; pend && spin < kSpinLimit; ++spin) {
        for (uint32_t m = pend; m; m &= m - 1) {
            const int j = __builtin_ctz(m);
            const uint64_t w = __hip_atomic_load(&fs[threadIdx.x + T * j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((w & 255u) == tag) {
                pend &= ~(1u << j);
                best = (w >> 8) < best ? (w >> 8) : best;
            }
        }
        if (pend) __builtin_amdgcn_s_sleep(1);
    }
    const int done = !__syncthreads_or(pend != 0);
    *ok = done;
    if (!done) return ~0ull;
    // (each slot word is the whole report: nothing else of the search
    // groups is read, so no acquire is needed here)
    best = block_min_u64(best, s.u);
    const uint64_t ssd = best >> kSlotIndexBits, idx = best & ((1ull << kSlotIndexBits) - 1);
    if (ssd == (1ull << 26) - 1) return ~0ull;
    return (ssd << 32) | idx;
}

template <int R>
struct CommitLds {
    Scratch s;
    LdsStage<R> L;
    PatchCopy<R> far;   // the untouched blocks' best pixel: the usual far next target
    uint32_t fill[kMaskWords];   // the target patch's hole pixels (precommit)
};

template <int R, int NY>
struct SearchLds {
    __attribute__((aligned(16))) uint32_t tile[tile::TileGeom<R, NY>::LDS_WORDS];
    tile::TargetLds tgt;
    uint64_t red[kSearchWaves];
    int32_t flag;
};

template <int R, int NY>
union FillLds {
    CommitLds<R> c;
    SearchLds<R, NY> s;
};

// TB, BW: gather()'s load batching (smaller under a tighter register budget);
// LEAN: the search groups read only the words and the known mask of a record.
template <int R, int TB, int BW, bool LEAN>
__device__ void fill_commit(const JobDev &d0, int ntiles, int n_iters, uint32_t epoch, CommitLds<R> &C) {
    Scratch &s = C.s;
    LdsStage<R> &L = C.L;
    // (Every MFMA search builds its B-operand tables from the staged words
    // and known mask.)  d is used in place: a copy of it would live in
    // scratch memory when d0 is not a kernel argument.
    const JobDev &d = d0;
    bool staged = false;
    FillSync *sy = d.sync;
    if (threadIdx.x == 0) s.snap = load_snap(d.st, d.tgt);
    __syncthreads();
    Snap v = s.snap;
    if (!v.done && !v.err && !v.pending) {   // nothing staged yet
        select_and_stage(d, s);
        __syncthreads();
        if (threadIdx.x == 0) s.snap = load_snap(d.st, d.tgt);   // this thread's own writes
        __syncthreads();
        v = s.snap;
    }
    if (!v.done && !v.err && v.pending) {
        if (LEAN)
            write_records_lean(sy, d.tgt, 2 * R + 1, rec_tag(v.iter));
        else
            write_records(sy, d.tgt, 2 * R + 1);
    }
    for (int i = threadIdx.x; i < ntiles; i += blockDim.x)
        __hip_atomic_store(&d.fslot[i], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool fresh = false;   // s.snap holds the state commit_finish left
    for (uint32_t k = 0;; ++k) {
        // Every wave's writes (records, state, slot resets) reach this
        // XCD's L2; then wave 0's release of go writes the L2 back, so they
        // reach device scope before go does.  (Nothing this group reads is
        // written by another group except through device-scope loads, so no
        // acquire is needed.)  The barrier also publishes s.snap.
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (fresh) v = s.snap;
        fresh = false;
        const bool stop = v.done || v.err || !v.pending || v.iter >= v.limit || (int)k >= n_iters;
        publish_go(sy, stop ? go_stop(epoch) : go_word(epoch, k + 1, LEAN ? rec_tag(v.iter) : 0u));
        if (stop) break;

        // search-independent loads of the commit, overlapping the search
        const int px = col_of(v.p, d.W), py = row_of(v.p, d.W);
        const Refresh g = refresh_geometry<R>(d, px, py);
        int64_t key = -1, idx = INT64_MAX;
        gather<R, false, TB, BW>(d, px, py, g, L, key, idx);
        block_argmax(key, idx, s.k, s.i);   // its barriers also publish the neighbourhood
        // the untouched blocks' best pixel wins whenever the next target is
        // far: copy its patch while the search still runs, its loads in
        // flight during the precommit
        const int64_t far_idx = key >= 0 ? idx : -1;
        const PatchLoad<R> far = load_patch<R>(d, far_idx);
        precommit<R>(d, v, g, L, C.fill);
        // (after the precommit marked the patch known: the gradients within
        // one pixel of the patch are recomputed after the copy anyway)
        grad_pass<R>(L, 1, Stage<R>::side - 1);
        store_patch<R>(d, far_idx, far, &C.far);

        // (its barriers also publish the gathered LDS neighbourhood)
        int ok = 0;
        const uint64_t best = collect_slots(d.fslot, ntiles, slot_tag(k), s, &ok);
        if (!ok) {
            if (threadIdx.x == 0) d.st->error = INPAINT_DEVICE;
            v.err = INPAINT_DEVICE;
            continue;      // publishes stop
        }
        commit_finish<R, false, true, LEAN>(d, s, L, v, best, g, key, idx, &s.snap, sy, nullptr, &C.far, C.fill);
        fresh = true;
        staged = true;
    }
    // s.tp / s.mbits hold the last target staged here
    if (LEAN && staged && v.pending && !v.done && !v.err) {
        finish_stage(R, d.tgt, s);
        __syncthreads();
    }
}

// Copies record `rec` (published by the go word just observed) into LDS,
// each word with an agent-scope load (see wait_go for the ordering).
template <int R>
__device__ __forceinline__ void load_record(const FillRec *rec, tile::TargetLds *t) {
    constexpr int P = 2 * R + 1, MW = (P * P + 31) / 32;
    for (int i = threadIdx.x; i < P * P; i += blockDim.x)
        t->tpix[i] = __hip_atomic_load(&rec->tpix[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x < MW) {
        t->mbits[threadIdx.x] = __hip_atomic_load(&rec->mbits[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t->sbits[threadIdx.x] = __hip_atomic_load(&rec->sbits[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t->ebits[threadIdx.x] = __hip_atomic_load(&rec->ebits[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x == 0) t->t2 = __hip_atomic_load(&rec->t2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int R, int NY>
__device__ void fill_search(const JobDev &d, int ntiles, uint32_t epoch, SearchLds<R, NY> &S) {
    // The tile stays in this group's LDS for the whole dispatch, so the
    // order of tiles over the XCDs does not matter here.
    const int t = (int)blockIdx.x - 1;
    int tx0, ty0;
    tile::tile_origin<R, NY>(d.rx0, d.ry0, d.ntx, t, &tx0, &ty0);
    const uint32_t vmask = tile::stage_tile<R, NY>(d, tx0, ty0, d.rx1, d.ry1, S.tile);
    const bool anyv = __syncthreads_or(vmask != 0);
    FillSync *sy = d.sync;
    for (uint32_t k = 0;; ++k) {
        if (threadIdx.x == 0) S.flag = wait_go(sy, t, epoch, k);
        __syncthreads();
        if (!S.flag) break;
        uint64_t best = ~0ull;
        if (anyv) {
            load_record<R>(&sy->rec[t % kGoCopies], &S.tgt);
            __syncthreads();
            const tile::LdsTarget view{&S.tgt};
            best = tile::wave_min_u64(tile::score_tile<R, NY>(d, view, tx0, ty0, vmask, S.tile));
            if ((threadIdx.x & 63) == 0) S.red[threadIdx.x >> 6] = best;
            __syncthreads();
            if (threadIdx.x == 0)
                for (int w = 0; w < kSearchWaves; ++w) best = S.red[w] < best ? S.red[w] : best;
        }
        if (threadIdx.x == 0)
            __hip_atomic_store(&d.fslot[t], slot_word(best, slot_tag(k)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
    }
}

template <int R>
struct SearchLdsMfma {
    mtile::MfmaTile<R> tile;
    mtile::FragTables<R> ft;
    uint64_t red[kSearchWaves];
    int32_t flag;
    uint32_t tag;
};

template <int R>
union FillLdsMfma {
    CommitLds<R> c;
    SearchLdsMfma<R> s;
};

// Search group of the MFMA form: one 64 x 64 tile of the MFMA tiling, staged
// once; per target it builds the B-operand tables in LDS from the record and
// scores the tile on the matrix cores.
template <int R>
__device__ void fill_search_mfma(const JobDev &d, uint32_t epoch, SearchLdsMfma<R> &S) {
    const int t = (int)blockIdx.x - 1;
    int tx0, ty0;
    mtile::tile_origin<R>(d.rx0, d.ry0, d.ntx, t, &tx0, &ty0);
    const uint32_t vmask = mtile::stage_tile<R>(d, tx0, ty0, d.rx0, d.rx1, d.ry1, S.tile);
    const bool anyv = __syncthreads_or(vmask != 0);
    FillSync *sy = d.sync;
    const FillRec *rec = &sy->rec[t % kGoCopies];
    constexpr int N = (2 * R + 1) * (2 * R + 1);
    static_assert(N <= kSearchWaves * 64, "one record word per thread");
    for (uint32_t k = 0;; ++k) {
        // Each poll reads the go word (thread 0) and this group's record
        // words (thread i: word i) together, so the target arrives with the
        // go word instead of one memory round trip after it.  Once go shows
        // iteration k, a word counts only with the tag go carries; stale
        // words (the previous iteration's) are read again.
        uint32_t w = 0;
        uint32_t spin = 0;
        for (;; ++spin) {
            uint64_t gv = 0;
            if (threadIdx.x == 0) gv = __hip_atomic_load(&rec->go, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (anyv && (int)threadIdx.x < N)
                w = __hip_atomic_load(&rec->tpix[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (threadIdx.x == 0) {
                // 1: go for iteration k (its tag in S.tag), 0: stop or time-out, -1: not yet
                S.flag = go_is(gv, epoch, k + 1) ? 1 : (gv == go_stop(epoch) ? 0 : -1);
                if (spin >= kSpinLimit) S.flag = 0;
                S.tag = go_tag(gv);
            }
            __syncthreads();
            const int f = S.flag;
            if (f == 1 && __syncthreads_and(!anyv || (int)threadIdx.x >= N || ((w >> 24) & 0x7fu) == S.tag)) break;
            if (f == 0) break;
            if (f == -1) __builtin_amdgcn_s_sleep(1);
            __syncthreads();   // thread 0 rewrites S.flag only after everyone read it
        }
        if (S.flag == 0) break;
        uint64_t best = ~0ull;
        if (anyv) {
            // the target from the record words into the patch tables, then
            // the shifted tables
            mtile::build_patch<R>(
                &S.ft, [&](int) { return w & 0x00ffffffu; }, [&](int) { return w >> 31; });
            __syncthreads();
            mtile::build_tables<R>(&S.ft);
            __syncthreads();
            best = tile::wave_min_u64(mtile::score_tile_rows<R>(d, &S.ft, tx0, ty0, vmask, S.tile));
            if ((threadIdx.x & 63) == 0) S.red[threadIdx.x >> 6] = best;
            __syncthreads();
            if (threadIdx.x == 0)
                for (int w = 0; w < kSearchWaves; ++w) best = S.red[w] < best ? S.red[w] : best;
        }
        if (threadIdx.x == 0)
            __hip_atomic_store(&d.fslot[t], slot_word(best, slot_tag(k)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
    }
}

// gather()'s load batching of the MFMA committer: smaller batches for the
// larger patches keep it within the register budget of two work-groups per
// CU (no spills).
template <int R>
struct MfmaCommitBatch {
    static constexpr int TB = R <= 4 ? 8 : (R == 5 ? 4 : 2);
    static constexpr int BW = R <= 4 ? 12 : (R == 5 ? 6 : 4);
};

template <int R>
__global__ __launch_bounds__(kCommitThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_fill_mfma(JobDev d, int ntiles, int n_iters, uint32_t epoch) {
    __shared__ FillLdsMfma<R> lds;
    if (blockIdx.x == 0)
        fill_commit<R, MfmaCommitBatch<R>::TB, MfmaCommitBatch<R>::BW, true>(d, ntiles, n_iters, epoch, lds.c);
    else
        fill_search_mfma<R>(d, epoch, lds.s);
}

template <int R>
__global__ __launch_bounds__(kCommitThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_fill(JobDev d, int ntiles, int n_iters, uint32_t epoch) {
    __shared__ FillLds<R, kFillTileRows> lds;
    if (blockIdx.x == 0)
        fill_commit<R, 2, 4, false>(d, ntiles, n_iters, epoch, lds.c);
    else
        fill_search<R, kFillTileRows>(d, ntiles, epoch, lds.s);
}

// ---- batched persistent fill: many jobs in one dispatch -----------------
//
// Work-groups [0, n_commit) each commit one job (fill_commit, exactly as in
// the single-job kernels, on that job's own records and slot words).  Every
// other work-group is a search group owning a list of (job, tile) items; a
// job's tiles are spread over many groups and a group's items come from
// many jobs.  Wave 0 keeps one item per lane -- its job, tile and the job
// iteration it scores next -- and polls all its items' go words at once.
// The group then serves one ready item, taken round-robin: stage the tile
// unless it is the one already in LDS, read the job's record, score, and
// write the job's slot word of that tile.  So a search group never waits on
// one job while another has work for it, and a job's iteration is scored by
// whichever groups are free.  A group with a single item keeps its tile in
// LDS for the whole dispatch, as the single-job kernels do.  Every wait is
// bounded as there: committers time out on their slots and publish stop; a
// search group gives up after kSpinLimit empty polls in a row.

struct MultiPick {
    int32_t pick;       // item to serve, -1: none ready
    int32_t all_done;   // every item's job published stop
    int32_t slot, tile;
    uint32_t k;
    uint32_t tag;       // record tag the item's go word carries
};

// Wave 0: polls the go words of this group's items (lane i: item i) and
// publishes the next ready item after `rot` (round-robin) in *pk.  my_k is
// the job iteration lane i's item scores next; it advances for the item
// picked.  The caller's barrier publishes *pk.
__device__ __forceinline__ void multi_poll(const uint64_t *my_go, int my_slot, int my_tile, uint32_t &my_k,
                                           bool &my_done, int rot, uint32_t epoch, MultiPick *pk) {
    const int lane = threadIdx.x & 63;
    bool ready = false;
    uint64_t v = 0;
    if (!my_done) {
        v = __hip_atomic_load(my_go, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ready = go_is(v, epoch, my_k + 1);
        my_done = v == go_stop(epoch);
    }
    const uint64_t rb = __ballot(ready), db = __ballot(my_done);
    const uint64_t hi = rb & (~0ull << rot);
    // (the record reads that follow are ordered after the go load as in
    // wait_go: agent-scope loads issued after it completed)
    const int pick = hi ? __builtin_ctzll(hi) : (rb ? __builtin_ctzll(rb) : -1);
    if (lane == 0) {
        pk->pick = pick;
        pk->all_done = db == ~0ull;
    }
    if (lane == pick) {
        pk->slot = my_slot;
        pk->tile = my_tile;
        pk->k = my_k;
        pk->tag = go_tag(v);
        my_k += 1;
    }
}

// Scores item (job d, tile t) for iteration k of the MFMA form and reports
// in the job's slot word.  restage: the tile in LDS is not this item's.
template <int R>
__device__ __forceinline__ void multi_serve_mfma(const JobDev &d, int t, uint32_t k, uint32_t tag, bool restage,
                                                 SearchLdsMfma<R> &S, uint32_t &vmask, bool &anyv) {
    int tx0, ty0;
    mtile::tile_origin<R>(d.rx0, d.ry0, d.ntx, t, &tx0, &ty0);
    if (restage) {
        vmask = mtile::stage_tile<R>(d, tx0, ty0, d.rx0, d.rx1, d.ry1, S.tile);
        anyv = __syncthreads_or(vmask != 0);
    }
    uint64_t best = ~0ull;
    if (anyv) {
        // the record words of iteration k: read until every one carries the
        // go word's tag (bounded; on a time-out no slot word is written, and
        // the committer's bounded wait reports the device error)
        const FillRec *rec = &d.sync->rec[t % kGoCopies];
        constexpr int N = (2 * R + 1) * (2 * R + 1);
        static_assert(N <= kSearchWaves * 64, "one record word per thread");
        uint32_t w = 0;
        for (uint32_t spin = 0;; ++spin) {
            if ((int)threadIdx.x < N)
                w = __hip_atomic_load(&rec->tpix[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__syncthreads_and((int)threadIdx.x >= N || ((w >> 24) & 0x7fu) == tag)) break;
            if (spin >= kSpinLimit) return;
        }
        mtile::build_patch<R>(
            &S.ft, [&](int) { return w & 0x00ffffffu; }, [&](int) { return w >> 31; });
        __syncthreads();
        mtile::build_tables<R>(&S.ft);
        __syncthreads();
        best = tile::wave_min_u64(mtile::score_tile_rows<R>(d, &S.ft, tx0, ty0, vmask, S.tile));
        if ((threadIdx.x & 63) == 0) S.red[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int w = 0; w < kSearchWaves; ++w) best = S.red[w] < best ? S.red[w] : best;
    }
    if (threadIdx.x == 0)
        __hip_atomic_store(&d.fslot[t], slot_word(best, slot_tag(k)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The same for the SIMT form.
template <int R>
__device__ __forceinline__ void multi_serve_simt(const JobDev &d, int t, uint32_t k, bool restage,
                                 SearchLds<R, kFillTileRows> &S, uint32_t &vmask, bool &anyv) {
    constexpr int NY = kFillTileRows;
    int tx0, ty0;
    tile::tile_origin<R, NY>(d.rx0, d.ry0, d.ntx, t, &tx0, &ty0);
    if (restage) {
        vmask = tile::stage_tile<R, NY>(d, tx0, ty0, d.rx1, d.ry1, S.tile);
        anyv = __syncthreads_or(vmask != 0);
    }
    uint64_t best = ~0ull;
    if (anyv) {
        load_record<R>(&d.sync->rec[t % kGoCopies], &S.tgt);
        __syncthreads();
        const tile::LdsTarget view{&S.tgt};
        best = tile::wave_min_u64(tile::score_tile<R, NY>(d, view, tx0, ty0, vmask, S.tile));
        if ((threadIdx.x & 63) == 0) S.red[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int w = 0; w < kSearchWaves; ++w) best = S.red[w] < best ? S.red[w] : best;
    }
    if (threadIdx.x == 0)
        __hip_atomic_store(&d.fslot[t], slot_word(best, slot_tag(k)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Search group w of a batched dispatch; serve(d, tile, k, tag, restage,
// vmask, anyv) scores one item (tag: the record tag its go word carried).
template <class Serve>
__device__ __forceinline__ void multi_search(const MultiPlan &m, int w, uint32_t epoch, MultiPick *pk, Serve serve) {
    const int i0 = m.first[w], ni = m.first[w + 1] - i0;   // 0 <= ni <= kMultiMaxItems (host-checked)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int my_slot = 0, my_tile = 0;
    uint32_t my_k = 0;
    bool my_done = true;
    const uint64_t *my_go = nullptr;   // go word of the record this lane's item reads
    if (wave == 0 && lane < ni) {
        const WorkItem it = m.items[i0 + lane];
        my_slot = it.slot;
        my_tile = it.tile;
        my_go = &m.slots[my_slot].sync->rec[my_tile % kGoCopies].go;
        my_done = false;
    }
    uint32_t vmask = 0;
    bool anyv = false;
    int staged = -1;   // item whose tile is in LDS
    int rot = 0;
    for (uint32_t spin = 0; spin < kSpinLimit;) {
        if (wave == 0) multi_poll(my_go, my_slot, my_tile, my_k, my_done, rot, epoch, pk);
        __syncthreads();
        const int pick = pk->pick;
        if (pick < 0) {
            if (pk->all_done) break;
            ++spin;
            __builtin_amdgcn_s_sleep(1);
            __syncthreads();   // wave 0 rewrites *pk only after everyone read it
            continue;
        }
        spin = 0;
        rot = pick + 1 < ni ? pick + 1 : 0;
        // (by value: the fields the search reads become scalar registers)
        const JobDev d = m.slots[pk->slot];
        serve(d, pk->tile, pk->k, pk->tag, staged != pick, vmask, anyv);
        staged = pick;
        __syncthreads();
    }
}

template <int R>
__global__ __launch_bounds__(kCommitThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_fill_multi_mfma(
    MultiPlan m, int n_iters, uint32_t epoch) {
    __shared__ FillLdsMfma<R> lds;
    __shared__ MultiPick pk;
    if ((int)blockIdx.x < m.n_commit) {
        // by value: held through a reference to device memory, the job's
        // fields would stay live in vector registers (and spill)
        const JobDev d = m.slots[m.commit[blockIdx.x]];
        fill_commit<R, MfmaCommitBatch<R>::TB, MfmaCommitBatch<R>::BW, true>(d, d.ntx * d.nty, n_iters, epoch,
                                                                             lds.c);
        return;
    }
    multi_search(m, (int)blockIdx.x - m.n_commit, epoch, &pk,
                 [&](const JobDev &d, int t, uint32_t k, uint32_t tag, bool restage, uint32_t &vmask, bool &anyv)
                     __attribute__((always_inline)) { multi_serve_mfma<R>(d, t, k, tag, restage, lds.s, vmask, anyv); });
}

template <int R>
__global__ __launch_bounds__(kCommitThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_fill_multi(
    MultiPlan m, int n_iters, uint32_t epoch) {
    __shared__ FillLds<R, kFillTileRows> lds;
    __shared__ MultiPick pk;
    if ((int)blockIdx.x < m.n_commit) {
        const JobDev d = m.slots[m.commit[blockIdx.x]];   // by value, see k_fill_multi_mfma
        fill_commit<R, 2, 4, false>(d, d.ntx * d.nty, n_iters, epoch, lds.c);
        return;
    }
    multi_search(m, (int)blockIdx.x - m.n_commit, epoch, &pk,
                 [&](const JobDev &d, int t, uint32_t k, uint32_t, bool restage, uint32_t &vmask, bool &anyv)
                     __attribute__((always_inline)) {
                     multi_serve_simt<R>(d, t, k, restage, lds.s, vmask, anyv);
                 });
}

// The MFMA form for jobs of several radii in one dispatch: the LDS of the
// largest radius; each committer takes its job's radius, and each search
// group the radius of its items (the plan gives a search group items of one
// radius only), so every work-group runs the per-radius code of its own
// radius for the whole dispatch.
union MixLdsMfma {
    FillLdsMfma<1> r1;
    FillLdsMfma<2> r2;
    FillLdsMfma<3> r3;
    FillLdsMfma<4> r4;
    FillLdsMfma<5> r5;
};
static_assert(kMultiMixMaxR == 5, "MixLdsMfma holds radii 1..5");

template <int R>
__device__ __forceinline__ void mixed_role(const MultiPlan &m, int n_iters, uint32_t epoch, FillLdsMfma<R> &lds,
                                           MultiPick *pk) {
    if ((int)blockIdx.x < m.n_commit) {
        const JobDev d = m.slots[m.commit[blockIdx.x]];   // by value, see k_fill_multi_mfma
        fill_commit<R, MfmaCommitBatch<R>::TB, MfmaCommitBatch<R>::BW, true>(d, d.ntx * d.nty, n_iters, epoch,
                                                                             lds.c);
        return;
    }
    multi_search(m, (int)blockIdx.x - m.n_commit, epoch, pk,
                 [&](const JobDev &d, int t, uint32_t k, uint32_t tag, bool restage, uint32_t &vmask, bool &anyv)
                     __attribute__((always_inline)) { multi_serve_mfma<R>(d, t, k, tag, restage, lds.s, vmask, anyv); });
}

__global__ __launch_bounds__(kCommitThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_fill_multi_mfma_mixed(
    MultiPlan m, int n_iters, uint32_t epoch) {
    __shared__ MixLdsMfma lds;
    __shared__ MultiPick pk;
    // this work-group's radius: its job's, or its first item's (a search
    // group without items has nothing to serve)
    int r = 0;
    if ((int)blockIdx.x < m.n_commit) {
        r = m.slots[m.commit[blockIdx.x]].r;
    } else {
        const int w = (int)blockIdx.x - m.n_commit;
        if (m.first[w + 1] > m.first[w]) r = m.slots[m.items[m.first[w]].slot].r;
    }
    switch (r) {
        case 1: mixed_role<1>(m, n_iters, epoch, lds.r1, &pk); break;
        case 2: mixed_role<2>(m, n_iters, epoch, lds.r2, &pk); break;
        case 3: mixed_role<3>(m, n_iters, epoch, lds.r3, &pk); break;
        case 4: mixed_role<4>(m, n_iters, epoch, lds.r4, &pk); break;
        case 5: mixed_role<5>(m, n_iters, epoch, lds.r5, &pk); break;
        default: break;   // no items; the host plan holds only radii 1 .. 5
    }
}

template <int R, bool ISECT>
__global__ __launch_bounds__(kCommitThreads) void k_commit(JobDev d) {
    __shared__ Scratch s;
    __shared__ LdsStage<R> L;
    __shared__ CommitNote note;
    if (threadIdx.x == 0) note.filled = 0;
    commit_body<R, ISECT>(d, s, L, &note);
    if (d.policy == INPAINT_SOURCE_CURRENT) {
        __syncthreads();
        if (note.filled > 0) add_filled_sources<R, ISECT>(d, L, col_of(note.p, d.W), row_of(note.p, d.W));
    }
}

// One work-group per listed slot (all with patch radius R); the list length
// is read from device memory so the slot list can change between graph
// replays without re-capture.
template <int R>
__global__ __launch_bounds__(kCommitThreads) void k_commit_batched(const JobDev *slots, const int32_t *ids,
                                                                   const int32_t *n) {
    __shared__ Scratch s;
    __shared__ LdsStage<R> L;
    if ((int)blockIdx.x >= *n) return;
    const JobDev d = slots[ids[blockIdx.x]];
    if (d.st == nullptr) return;   // empty slot
    commit_body<R>(d, s, L);
}

__global__ __launch_bounds__(kCommitThreads) void k_stage_query(JobDev d, int tx, int ty, int r) {
    __shared__ Scratch s;
    stage_target(d, tx, ty, r, d.qtgt, s);
}

__global__ __launch_bounds__(kCommitThreads) void k_reduce_partials(const uint64_t *partials, int n,
                                                                   uint64_t *out) {
    __shared__ uint64_t sh[16];
    uint64_t best = ~0ull;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const uint64_t v = partials[t];
        best = v < best ? v : best;
    }
    best = block_min_u64(best, sh);
    if (threadIdx.x == 0) *out = best;
}

// Number of attached images that are still unfinished and error-free, and
// each slot's state (0 empty, 1 running, 2 finished, 3 error).
__global__ void k_count_active(const JobDev *slots, int nslots, int64_t *out, int32_t *status) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < nslots; i += blockDim.x) {
        const IterState *st = slots[i].st;
        int v = 0;
        if (st) v = st->error ? 3 : (st->done ? 2 : 1);
        if (v == 1) atomicAdd(&cnt, 1);
        status[i] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) *out = cnt;
}

// ---------------------------------------------------------------- launchers

static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

uint32_t init_pixel_blocks(const JobDev &d) { return blocks_for((int64_t)d.W * d.H, 256); }

hipError_t launch_seal(const JobDev &d, uint32_t nonce, hipStream_t s) {
    hipLaunchKernelGGL(k_seal, dim3(1), dim3(1), 0, s, d.info, nonce);
    return hipGetLastError();
}

hipError_t launch_init(const JobDev &d, const uint8_t *stage_rgb, int channels,
                       const uint8_t *stage_mask, uint8_t *hdist, uint32_t nonce, hipStream_t s) {
    const int64_t n = (int64_t)d.W * d.H;
    hipLaunchKernelGGL(k_init_info, dim3(1), dim3(1), 0, s, d.info, nonce);
    hipLaunchKernelGGL(k_init_pixels, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, stage_rgb,
                       channels, stage_mask);
    hipLaunchKernelGGL(k_init_hdist, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, hdist);
    hipLaunchKernelGGL(k_init_vrad, dim3(blocks_for(n, 256)), dim3(256), 0, s, d,
                       (const uint8_t *)hdist);
    const int64_t np = (int64_t)d.pitch * padded_rows(d.H);
    hipLaunchKernelGGL(k_init_padded, dim3(blocks_for(np, 256)), dim3(256), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_import_check(const JobDev &d, const uint8_t *hole, const double *conf, uint32_t nonce,
                               hipStream_t s) {
    const int64_t n = (int64_t)d.W * d.H;
    hipLaunchKernelGGL(k_import_reset, dim3(1), dim3(1), 0, s, d.info, nonce);
    hipLaunchKernelGGL(k_import_check, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, hole, conf);
    return hipGetLastError();
}

hipError_t launch_import_apply(const JobDev &d, const uint8_t *rgb, int channels, const uint8_t *hole,
                               const double *conf, uint8_t *hdist, uint32_t nonce, hipStream_t s) {
    const int64_t n = (int64_t)d.W * d.H;
    hipLaunchKernelGGL(k_import_reset, dim3(1), dim3(1), 0, s, d.info, nonce);
    hipLaunchKernelGGL(k_import_apply, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, rgb, channels, hole, conf);
    if (d.policy == INPAINT_SOURCE_CURRENT) {
        // the source region is the current known region: rebuild its planes
        hipLaunchKernelGGL(k_init_hdist, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, hdist);
        hipLaunchKernelGGL(k_init_vrad, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, (const uint8_t *)hdist);
        const int64_t np = (int64_t)d.pitch * padded_rows(d.H);
        hipLaunchKernelGGL(k_init_padded, dim3(blocks_for(np, 256)), dim3(256), 0, s, d);
    }
    return hipGetLastError();
}

hipError_t launch_count_valid(const JobDev &d, hipStream_t s) {
    const int64_t n = (int64_t)(d.rx1 - d.rx0) * (d.ry1 - d.ry0);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_valid, dim3(blocks_for(n, 256)), dim3(256), 0, s, d);
    return hipGetLastError();
}

#define INPAINT_RADIUS_SWITCH(r, CALL) \
    switch (r) {                          \
        case 1: CALL(1); break;           \
        case 2: CALL(2); break;           \
        case 3: CALL(3); break;           \
        case 4: CALL(4); break;           \
        case 5: CALL(5); break;           \
        case 6: CALL(6); break;           \
        case 7: CALL(7); break;           \
        case 8: CALL(8); break;           \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_prio_init(const JobDev &d, hipStream_t s) {
    const int nb = (d.pbx1 - d.pbx0) * (d.pby1 - d.pby0);
#define CALL(R) hipLaunchKernelGGL(k_prio_init<R>, dim3((nb + 3) / 4), dim3(256), 0, s, d)
    INPAINT_RADIUS_SWITCH(d.r, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_commit(const JobDev &d, hipStream_t s) {
#define CALL(R)                                                                            \
    if (d.isect) hipLaunchKernelGGL((k_commit<R, true>), dim3(1), dim3(kCommitThreads), 0, s, d); \
    else hipLaunchKernelGGL((k_commit<R, false>), dim3(1), dim3(kCommitThreads), 0, s, d)
    INPAINT_RADIUS_SWITCH(d.r, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_commit_batched(const JobDev *slots, const int32_t *ids, const int32_t *n, int grid, int r,
                                 hipStream_t s) {
    if (grid <= 0) return hipSuccess;
#define CALL(R) hipLaunchKernelGGL(k_commit_batched<R>, dim3(grid), dim3(kCommitThreads), 0, s, slots, ids, n)
    INPAINT_RADIUS_SWITCH(r, CALL)
#undef CALL
    return hipGetLastError();
}

static const void *fill_kernel(int r, bool mfma) {
    if (mfma) {
        switch (r) {
            case 1: return (const void *)k_fill_mfma<1>;
            case 2: return (const void *)k_fill_mfma<2>;
            case 3: return (const void *)k_fill_mfma<3>;
            case 4: return (const void *)k_fill_mfma<4>;
            case 5: return (const void *)k_fill_mfma<5>;
            case 6: return (const void *)k_fill_mfma<6>;
            default: return nullptr;
        }
    }
    switch (r) {
        case 1: return (const void *)k_fill<1>;
        case 2: return (const void *)k_fill<2>;
        case 3: return (const void *)k_fill<3>;
        case 4: return (const void *)k_fill<4>;
        case 5: return (const void *)k_fill<5>;
        case 6: return (const void *)k_fill<6>;
        case 7: return (const void *)k_fill<7>;
        case 8: return (const void *)k_fill<8>;
        default: return nullptr;
    }
}

hipError_t fill_blocks_per_cu(int r, bool mfma, int *blocks) {
    const void *f = fill_kernel(r, mfma);
    if (!f) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, f, kCommitThreads, 0);
}

int fill_grid(int ntiles) { return 1 + ntiles; }

hipError_t launch_fill(const JobDev &d, int ntiles, int n_iters, uint32_t epoch, hipStream_t s) {
    const void *f = fill_kernel(d.r, d.mfma != 0);
    if (!f) return hipErrorInvalidValue;
    JobDev dd = d;
    void *args[] = {&dd, &ntiles, &n_iters, &epoch};
    return hipLaunchKernel(f, dim3(fill_grid(ntiles)), dim3(kCommitThreads), args, 0, s);
}

static const void *fill_multi_kernel(bool mfma, int r) {
    if (mfma) {
        switch (r) {
            case kMultiMixed: return (const void *)k_fill_multi_mfma_mixed;
            case 1: return (const void *)k_fill_multi_mfma<1>;
            case 2: return (const void *)k_fill_multi_mfma<2>;
            case 3: return (const void *)k_fill_multi_mfma<3>;
            case 4: return (const void *)k_fill_multi_mfma<4>;
            case 5: return (const void *)k_fill_multi_mfma<5>;
            case 6: return (const void *)k_fill_multi_mfma<6>;
            default: return nullptr;
        }
    }
    switch (r) {
        case 1: return (const void *)k_fill_multi<1>;
        case 2: return (const void *)k_fill_multi<2>;
        case 3: return (const void *)k_fill_multi<3>;
        case 4: return (const void *)k_fill_multi<4>;
        case 5: return (const void *)k_fill_multi<5>;
        case 6: return (const void *)k_fill_multi<6>;
        case 7: return (const void *)k_fill_multi<7>;
        case 8: return (const void *)k_fill_multi<8>;
        default: return nullptr;
    }
}

hipError_t multi_blocks_per_cu(bool mfma, int r, int *blocks) {
    const void *f = fill_multi_kernel(mfma, r);
    if (!f) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, f, kCommitThreads, 0);
}

hipError_t launch_fill_multi(const MultiPlan &m, bool mfma, int r, int grid, int n_iters, uint32_t epoch,
                             hipStream_t s) {
    const void *f = fill_multi_kernel(mfma, r);
    if (!f || grid <= m.n_commit) return hipErrorInvalidValue;
    MultiPlan mm = m;
    void *args[] = {&mm, &n_iters, &epoch};
    return hipLaunchKernel(f, dim3(grid), dim3(kCommitThreads), args, 0, s);
}

hipError_t launch_stage_query(const JobDev &d, int tx, int ty, int r, hipStream_t s) {
    hipLaunchKernelGGL(k_stage_query, dim3(1), dim3(kCommitThreads), 0, s, d, tx, ty, r);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const JobDev &d, int ntiles, uint64_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kCommitThreads), 0, s,
                       (const uint64_t *)d.partials, ntiles, out);
    return hipGetLastError();
}

hipError_t launch_count_active(const JobDev *slots, int nslots, int64_t *out, int32_t *status, hipStream_t s) {
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, s, slots, nslots, out, status);
    return hipGetLastError();
}

}  // namespace inpaint
