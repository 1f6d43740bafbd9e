// Initialisation, fill-front / priority, selection, target staging and the
// copy / confidence update of exemplar-based object removal on gfx950.
//
// Everything here except the exemplar search (search.hip) is latency-bound
// work on at most a few thousand pixels per iteration, so the per-iteration
// part runs as ONE work-group of 1024 threads per image ("commit" kernel):
//   reduce the search partials -> copy the source patch -> refresh the
//   priorities near the filled patch -> argmax -> stage the next target.
//
// Priorities are binary64 and must match a plain sequential CPU evaluation
// bit for bit, so this file is compiled with FP contraction off and every
// sum runs in the fixed raster order of the patch offsets.
#pragma clang fp contract(off)

#include "inpaint_dev.h"

namespace inpaint {

namespace {

__device__ __forceinline__ bool in_img(const JobDev &d, int x, int y) {
    return (unsigned)x < (unsigned)d.W && (unsigned)y < (unsigned)d.H;
}

// Known = inside the image and not in the current hole.
__device__ __forceinline__ bool known_px(const JobDev &d, int x, int y) {
    return in_img(d, x, y) && d.hole[(int64_t)y * d.W + x] == 0;
}

// Hole indicator with out-of-image pixels counted as hole (normal estimate).
__device__ __forceinline__ int hole_or_out(const JobDev &d, int x, int y) {
    return (!in_img(d, x, y) || d.hole[(int64_t)y * d.W + x]) ? 1 : 0;
}

// Fill front: a hole pixel with at least one in-image 4-neighbour known.
__device__ __forceinline__ bool on_front(const JobDev &d, int x, int y) {
    if (!in_img(d, x, y) || d.hole[(int64_t)y * d.W + x] == 0) return false;
    return known_px(d, x + 1, y) || known_px(d, x - 1, y) || known_px(d, x, y + 1) ||
           known_px(d, x, y - 1);
}

// Eq. 2.  Confidence: sum of C over the known pixels of the patch, in raster
// order of the offsets, divided by the constant patch area P*P.  Data term:
// the isophote (-gy, gx)/2 at the known pixel of the patch with the largest
// central-difference gradient of the gray image (all four neighbours known;
// first in raster order on ties), dotted with the unit normal of the front
// (central differences of the hole indicator), absolute value, over 255.
__device__ void priority_terms(const JobDev &d, int px, int py, double *C, double *D) {
    const int r = d.r, P = 2 * r + 1, W = d.W;
    double sum = 0.0;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
            const int x = px + dx, y = py + dy;
            if (known_px(d, x, y)) sum = sum + d.conf[(int64_t)y * W + x];
        }
    *C = sum / (double)(P * P);

    int gx = 0, gy = 0, best = -1;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
            const int x = px + dx, y = py + dy;
            if (!known_px(d, x, y) || !known_px(d, x + 1, y) || !known_px(d, x - 1, y) ||
                !known_px(d, x, y + 1) || !known_px(d, x, y - 1))
                continue;
            const uint8_t *g = d.gray;
            const int ax = (int)g[(int64_t)y * W + x + 1] - (int)g[(int64_t)y * W + x - 1];
            const int ay = (int)g[(int64_t)(y + 1) * W + x] - (int)g[(int64_t)(y - 1) * W + x];
            const int mag = ax * ax + ay * ay;
            if (mag > best) {
                best = mag;
                gx = ax;
                gy = ay;
            }
        }
    const int nx = hole_or_out(d, px + 1, py) - hole_or_out(d, px - 1, py);
    const int ny = hole_or_out(d, px, py + 1) - hole_or_out(d, px, py - 1);
    const int kn = nx * nx + ny * ny;
    if (kn == 0) {
        *D = 0.0;
    } else {
        int a = gx * ny - gy * nx;
        if (a < 0) a = -a;
        *D = (0.5 * (double)a) / (kn == 1 ? d.norm1 : d.norm2);
    }
}

// Priority key of a pixel: bits of P = C * D (Eq. 1) on the front, else -1.
// Non-negative doubles order like their bit patterns.
__device__ int64_t pixel_key(const JobDev &d, int x, int y) {
    if (!on_front(d, x, y)) return -1;
    double C, D;
    priority_terms(d, x, y, &C, &D);
    return __double_as_longlong(C * D);
}

// ---- work-group reductions (blockDim.x a multiple of 64, <= 1024) ----

__device__ __forceinline__ bool better(int64_t ka, int64_t ia, int64_t kb, int64_t ib) {
    return ka > kb || (ka == kb && ia < ib);
}

__device__ void block_argmax(int64_t &key, int64_t &idx, int64_t *sk, int64_t *si) {
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t k2 = __shfl_xor(key, off);
        const int64_t i2 = __shfl_xor(idx, off);
        if (better(k2, i2, key, idx)) {
            key = k2;
            idx = i2;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) {
        sk[w] = key;
        si[w] = idx;
    }
    __syncthreads();
    if (w == 0) {
        key = lane < nw ? sk[lane] : -1;
        idx = lane < nw ? si[lane] : INT64_MAX;
        for (int off = 32; off > 0; off >>= 1) {
            const int64_t k2 = __shfl_xor(key, off);
            const int64_t i2 = __shfl_xor(idx, off);
            if (better(k2, i2, key, idx)) {
                key = k2;
                idx = i2;
            }
        }
        if (lane == 0) {
            sk[0] = key;
            si[0] = idx;
        }
    }
    __syncthreads();
    key = sk[0];
    idx = si[0];
    __syncthreads();
}

__device__ uint64_t block_min_u64(uint64_t v, uint64_t *sh) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    if (w == 0) {
        v = lane < nw ? sh[lane] : ~0ull;
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t o = __shfl_xor(v, off);
            v = o < v ? o : v;
        }
        if (lane == 0) sh[0] = v;
    }
    __syncthreads();
    v = sh[0];
    __syncthreads();
    return v;
}

__device__ int64_t block_sum_i64(int64_t v, int64_t *sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    if (w == 0) {
        v = lane < nw ? sh[lane] : 0;
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) sh[0] = v;
    }
    __syncthreads();
    v = sh[0];
    __syncthreads();
    return v;
}

struct Scratch {
    int64_t k[16];
    int64_t i[16];
    uint64_t u[16];
    uint32_t mbits[16];
    int64_t bcast[8];
};

// Recomputes the priority-block maximum of block (bx, by).
__device__ void refresh_block(const JobDev &d, int bx, int by, Scratch &s) {
    const int x = bx * kBlock + (int)(threadIdx.x & (kBlock - 1));
    const int y = by * kBlock + (int)(threadIdx.x / kBlock);
    int64_t key = -1, idx = INT64_MAX;
    if (threadIdx.x < kBlock * kBlock && in_img(d, x, y)) {
        idx = (int64_t)y * d.W + x;
        key = d.pkey[idx];
    }
    block_argmax(key, idx, s.k, s.i);
    if (threadIdx.x == 0) {
        d.blk[by * d.nbw + bx].key = key;
        d.blk[by * d.nbw + bx].idx = idx;
    }
}

// Stages the target patch at (tx, ty) with radius r into *tg: known mask,
// RGBX words, k and T2 = sum of squared known target values.
__device__ void stage_target(const JobDev &d, int tx, int ty, int r, TargetStage *tg, Scratch &s) {
    const int P = 2 * r + 1;
    if (threadIdx.x < 16) s.mbits[threadIdx.x] = 0;
    __syncthreads();
    int64_t kk = 0, t2 = 0;
    for (int t = threadIdx.x; t < kMaxOffsets + 15; t += blockDim.x) {
        uint32_t pix = 0;
        if (t < P * P) {
            const int dx = t % P - r, dy = t / P - r;
            const int x = tx + dx, y = ty + dy;
            if (known_px(d, x, y)) {
                pix = d.img[(int64_t)y * d.W + x] & 0x00ffffffu;
                const int R = pix & 255, G = (pix >> 8) & 255, B = (pix >> 16) & 255;
                kk += 1;
                t2 += R * R + G * G + B * B;
                atomicOr(&s.mbits[t >> 5], 1u << (t & 31));
            }
        }
        tg->tpix[t] = pix;
    }
    kk = block_sum_i64(kk, s.k);
    t2 = block_sum_i64(t2, s.k);
    if (threadIdx.x < 16) tg->mbits[threadIdx.x] = s.mbits[threadIdx.x];
    if (threadIdx.x == 0) {
        tg->tx = tx;
        tg->ty = ty;
        tg->r = r;
        tg->k = (int32_t)kk;
        tg->t2 = (uint32_t)t2;
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
    const int px = (int)(idx % d.W), py = (int)(idx / d.W);
    stage_target(d, px, py, d.r, d.tgt, s);
    if (threadIdx.x == 0) {
        double C, D;
        priority_terms(d, px, py, &C, &D);
        st->p_idx = idx;
        st->C = C;
        st->D = D;
        st->Pr = C * D;
        st->pending = 1;
    }
}

}  // namespace

// ----------------------------------------------------------------- kernels

__global__ void k_init_info(InitInfo *info) {
    info->hole_count = 0;
    info->bx0 = INT32_MAX;
    info->by0 = INT32_MAX;
    info->bx1 = INT32_MIN;
    info->by1 = INT32_MIN;
    info->valid_count = 0;
}

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
        const int x = (int)(i % d.W), y = (int)(i / d.W);
        const bool h = mask[i] != 0;
        const uint32_t R = h ? 0 : rgb[i * ch], G = h ? 0 : rgb[i * ch + 1],
                       B = h ? 0 : rgb[i * ch + 2];
        d.img[i] = R | (G << 8) | (B << 16);
        d.gray[i] = (uint8_t)((299 * R + 587 * G + 114 * B + 500) / 1000);
        d.hole[i] = h ? 1 : 0;
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
}

// Horizontal distance (capped at 10) from each pixel to the nearest hole or
// out-of-image pixel of its row.
__global__ __launch_bounds__(256) void k_init_hdist(JobDev d, uint8_t *hdist) {
    const int64_t n = (int64_t)d.W * d.H;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = (int)(i % d.W), y = (int)(i / d.W);
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
    const int x = (int)(i % d.W), y = (int)(i / d.W);
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
        if (d.vrad[(int64_t)y * d.W + x] >= d.r) atomicAdd(&s_cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt)
        atomicAdd((unsigned long long *)&d.info->valid_count, (unsigned long long)s_cnt);
}

// Priority keys and block maxima of every block of the priority range.
__global__ __launch_bounds__(1024) void k_prio_init(JobDev d) {
    __shared__ Scratch s;
    const int bw = d.pbx1 - d.pbx0;
    const int bx = d.pbx0 + (int)blockIdx.x % bw, by = d.pby0 + (int)blockIdx.x / bw;
    const int x = bx * kBlock + (int)(threadIdx.x & (kBlock - 1));
    const int y = by * kBlock + (int)(threadIdx.x / kBlock);
    if (in_img(d, x, y)) d.pkey[(int64_t)y * d.W + x] = pixel_key(d, x, y);
    __syncthreads();
    refresh_block(d, bx, by, s);
}

// One fill iteration after the search: reduce the search partials, copy the
// source patch into the target's hole pixels (they take the target's
// confidence), log, refresh priorities near the patch, select and stage the
// next target.  With no staged target it only selects and stages.
__device__ void commit_body(const JobDev &d, Scratch &s) {
    IterState *st = d.st;
    if (st->done || st->error) return;
    if (st->pending) {
        if (st->iter >= st->iter_limit) return;
        const int ntiles = d.ntx * d.nty;
        uint64_t best = ~0ull;
        for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
            const uint64_t v = d.partials[t];
            best = v < best ? v : best;
        }
        best = block_min_u64(best, s.u);
        if (best == ~0ull) {
            if (threadIdx.x == 0) st->error = INPAINT_NO_CANDIDATE;
            return;
        }
        const int64_t q = (int64_t)(best & 0xffffffffu);
        const uint32_t ssd = (uint32_t)(best >> 32);
        const int64_t p = st->p_idx;
        const double C = st->C;
        const int W = d.W, r = d.r, P = 2 * r + 1;
        const int px = (int)(p % W), py = (int)(p / W), qx = (int)(q % W), qy = (int)(q / W);
        int64_t filled = 0;
        if (threadIdx.x < P * P) {
            const int dx = (int)threadIdx.x % P - r, dy = (int)threadIdx.x / P - r;
            const int x = px + dx, y = py + dy;
            if (in_img(d, x, y) && d.hole[(int64_t)y * W + x]) {
                const int64_t dst = (int64_t)y * W + x, src = (int64_t)(qy + dy) * W + (qx + dx);
                d.img[dst] = d.img[src];
                d.gray[dst] = d.gray[src];
                d.conf[dst] = C;
                d.hole[dst] = 0;
                filled = 1;
            }
        }
        filled = block_sum_i64(filled, s.k);
        const int64_t remaining = st->remaining - filled;
        __syncthreads();
        if (threadIdx.x == 0) {
            StepRec rec;
            rec.target_index = p;
            rec.source_index = q;
            rec.ssd = ssd;
            rec.known_k = d.tgt->k;
            rec.n_filled = (int32_t)filled;
            rec.reserved = 0;
            rec.priority = st->Pr;
            rec.confidence = C;
            rec.data_term = st->D;
            rec.remaining = remaining;
            const int64_t it = st->iter;
            if (it < d.log_cap) d.log[it] = rec;
            st->last = rec;
            st->remaining = remaining;
            st->iter = it + 1;
            st->pending = 0;
            if (remaining == 0) st->done = 1;
        }
        if (remaining == 0) return;
        // Priorities can change only within 2r+1 (Chebyshev) of the target:
        // that is where the hole, the confidences and the gray values read
        // by a priority evaluation changed.
        const int reach = 2 * r + 1;
        const int wx0 = max(px - reach, 0), wx1 = min(px + reach + 1, d.W);
        const int wy0 = max(py - reach, 0), wy1 = min(py + reach + 1, d.H);
        const int ww = wx1 - wx0, nwin = ww * (wy1 - wy0);
        __syncthreads();
        for (int t = threadIdx.x; t < nwin; t += blockDim.x) {
            const int x = wx0 + t % ww, y = wy0 + t / ww;
            d.pkey[(int64_t)y * W + x] = pixel_key(d, x, y);
        }
        __syncthreads();
        for (int by = wy0 / kBlock; by <= (wy1 - 1) / kBlock; ++by)
            for (int bx = wx0 / kBlock; bx <= (wx1 - 1) / kBlock; ++bx) refresh_block(d, bx, by, s);
        __syncthreads();
    }
    select_and_stage(d, s);
}

__global__ __launch_bounds__(kCommitThreads) void k_commit(JobDev d) {
    __shared__ Scratch s;
    commit_body(d, s);
}

__global__ __launch_bounds__(kCommitThreads) void k_commit_batched(const JobDev *slots, int nslots) {
    __shared__ Scratch s;
    if ((int)blockIdx.x >= nslots) return;
    const JobDev d = slots[blockIdx.x];
    if (d.st == nullptr) return;   // empty slot
    commit_body(d, s);
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

// ---------------------------------------------------------------- launchers

static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_init(const JobDev &d, const uint8_t *stage_rgb, int channels,
                       const uint8_t *stage_mask, uint8_t *hdist, hipStream_t s) {
    const int64_t n = (int64_t)d.W * d.H;
    hipLaunchKernelGGL(k_init_info, dim3(1), dim3(1), 0, s, d.info);
    hipLaunchKernelGGL(k_init_pixels, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, stage_rgb,
                       channels, stage_mask);
    hipLaunchKernelGGL(k_init_hdist, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, hdist);
    hipLaunchKernelGGL(k_init_vrad, dim3(blocks_for(n, 256)), dim3(256), 0, s, d,
                       (const uint8_t *)hdist);
    return hipGetLastError();
}

hipError_t launch_count_valid(const JobDev &d, hipStream_t s) {
    const int64_t n = (int64_t)(d.rx1 - d.rx0) * (d.ry1 - d.ry0);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_valid, dim3(blocks_for(n, 256)), dim3(256), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_prio_init(const JobDev &d, hipStream_t s) {
    const int nb = (d.pbx1 - d.pbx0) * (d.pby1 - d.pby0);
    hipLaunchKernelGGL(k_prio_init, dim3(nb), dim3(1024), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_commit(const JobDev &d, hipStream_t s) {
    hipLaunchKernelGGL(k_commit, dim3(1), dim3(kCommitThreads), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_commit_batched(const JobDev *slots, int nslots, hipStream_t s) {
    hipLaunchKernelGGL(k_commit_batched, dim3(nslots), dim3(kCommitThreads), 0, s, slots, nslots);
    return hipGetLastError();
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

}  // namespace inpaint

namespace inpaint {

// Number of attached images that are still unfinished and error-free.
__global__ void k_count_active(const JobDev *slots, int nslots, int64_t *out) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < nslots; i += blockDim.x) {
        const IterState *st = slots[i].st;
        if (st && !st->done && !st->error) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) *out = cnt;
}

hipError_t launch_count_active(const JobDev *slots, int nslots, int64_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, s, slots, nslots, out);
    return hipGetLastError();
}

}  // namespace inpaint
