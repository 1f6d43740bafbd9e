// Host runtime of libinpaint.so: the C ABI of include/inpaint.h.
//
// A context owns no device memory of its own: every device buffer of a job is
// carved out of the caller's workspace (a torch tensor in the Python
// binding), so the caller's allocator and a serving loop's admission see the
// exact footprint.  Device work runs on the caller's stream.  The only
// allocations the library makes are small pinned host mirrors of the
// iteration state, and, for a batch, its slot table and work lists.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <vector>

#include "inpaint.h"
#include "inpaint_dev.h"

using namespace inpaint;

static_assert(sizeof(InitInfo) <= 64, "InitInfo is read back through the 64-byte pinned key buffer");

namespace {

thread_local std::string g_create_error;

constexpr uint64_t kAlign = 256;
constexpr int kDefaultTileRows = 8;
constexpr int kMaxGroups = 4096;   // work-groups of a persistent dispatch (co-resident: <= 4 per CU)

uint64_t align_up(uint64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Per-call values the init, count and import kernel sequences write into
// InitInfo (never 0, which is what a fresh workspace holds).
std::atomic<uint32_t> g_nonce{0};
uint32_t next_nonce() {
    uint32_t v;
    do v = (g_nonce.fetch_add(1) + 1) * 2654435761u;
    while (v == 0);
    return v;
}

// Persistent dispatches (k_fill*, k_fill_multi*) need every work-group of
// their grid resident at once: their groups wait on one another, and the
// host sizes the grid from the occupancy API for an otherwise idle device.
// Kernels of other streams running beside such a dispatch hold resources
// its late groups need; while new ones keep arriving those groups can wait
// past the dispatch's bounded waits (a device error), and with cooperative
// launches results were seen to go wrong as well.  So a persistent dispatch
// runs alone: it holds this lock exclusively from its launch until the host
// has seen it end, and every other call of the library that puts work on the
// device holds it shared until that work has ended (each such call
// synchronises its stream before it returns).  Calls that do not run a
// persistent dispatch still overlap one another freely.
std::shared_mutex g_device_mu;
typedef std::shared_lock<std::shared_mutex> SharedDevice;
typedef std::unique_lock<std::shared_mutex> ExclusiveDevice;

// Launch epochs of persistent dispatches, unique in the process: a job's
// records and slot words may hold values from any earlier dispatch that ran
// it (alone or in a batch), and only the current epoch's go words count.
std::atomic<uint32_t> g_epoch{0};
uint32_t next_epoch() {
    uint32_t v;
    do v = g_epoch.fetch_add(1) + 1;
    while (v == 0);
    return v;
}

// Whether the kernel sequence stamped with `nonce` ran to its end: its first
// kernel wrote the nonce, its last one the seal, and (blocks != 0) every
// work-group of its pixel pass finished.  When it did not, what InitInfo
// holds says nothing about the caller's input.
bool sealed(const InitInfo &info, uint32_t nonce, uint32_t blocks) {
    return info.nonce == nonce && info.seal == nonce && (blocks == 0 || info.blocks == blocks);
}

// Host rows to a packed device buffer.  A 2D copy from pageable memory moves
// every row separately (one transfer per row), so packed rows go as one copy.
static hipError_t upload_rows(void *dst, size_t row_bytes, const void *src, size_t stride, int rows,
                              hipStream_t s) {
    if (stride == row_bytes) return hipMemcpyAsync(dst, src, row_bytes * rows, hipMemcpyHostToDevice, s);
    return hipMemcpy2DAsync(dst, row_bytes, src, stride, row_bytes, rows, hipMemcpyHostToDevice, s);
}

// The nonzero bytes of a caller's W x H mask and their bounding box
// (half-open).  Create and import compare the device's count (and box) of
// the uploaded mask with these, so a pass that read anything but the
// caller's bytes is reported as a device failure instead of being run.
struct MaskStats {
    int64_t count = 0;
    int x0 = INT32_MAX, y0 = INT32_MAX, x1 = INT32_MIN, y1 = INT32_MIN;
};
static MaskStats mask_stats(const uint8_t *m, int stride, int W, int H) {
    MaskStats r;
    for (int y = 0; y < H; ++y) {
        const uint8_t *row = m + (int64_t)y * stride;
        int first = -1, last = -1;
        int64_t c = 0;
        for (int x = 0; x < W; ++x)
            if (row[x]) {
                if (first < 0) first = x;
                last = x;
                ++c;
            }
        if (c == 0) continue;
        r.count += c;
        r.x0 = std::min(r.x0, first);
        r.x1 = std::max(r.x1, last + 1);
        r.y0 = std::min(r.y0, y);
        r.y1 = y + 1;
    }
    return r;
}

struct Layout {
    uint64_t img, gray, hole, hole0, vrad, conf, pcd, blk, partials, tgt, qtgt, srcw, srcq, srcp, vradp, hdist, st,
        sync, fslot, info, key, mplan, log, total;
    int64_t log_cap;
    int max_tiles;
};

bool tile_rows_ok(int t) { return t == 4 || t == 8 || t == 16; }

int64_t log_capacity(int W, int H, const inpaint_params &p) {
    return p.log_capacity < 0 ? (int64_t)W * H : (int64_t)p.log_capacity;
}

Layout make_layout(int W, int H, const inpaint_params &p) {
    Layout L{};
    const uint64_t n = (uint64_t)W * H;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = align_up(off + std::max<uint64_t>(bytes, 1));
        return o;
    };
    L.img = take(4 * n);
    L.gray = take(n);
    L.hole = take(n);
    L.hole0 = take(n);
    L.vrad = take(n);
    L.conf = take(8 * n);
    L.pcd = take(16 * n);  // also the upload staging area during create (<= 6n bytes)
    const uint64_t nblk = (uint64_t)((W + kBlock - 1) / kBlock) * ((H + kBlock - 1) / kBlock);
    L.blk = take(sizeof(BlockBest) * nblk);
    // (+7: the MFMA tiling may start up to 7 columns left of the rect)
    L.max_tiles = ((W + 7 + kTileW - 1) / kTileW) * ((H + search_tile_h(4) - 1) / search_tile_h(4));
    L.partials = take(8ull * L.max_tiles);
    L.tgt = take(sizeof(TargetStage));
    L.qtgt = take(sizeof(TargetStage));
    const bool mfma = p.path == INPAINT_PATH_MFMA;
    const uint64_t np = (uint64_t)padded_pitch(W) * padded_rows(H);
    L.srcw = mfma ? take(4 * np) : 0;
    L.srcq = mfma ? take(2 * np) : 0;
    L.srcp = take(4 * np);
    L.vradp = take(np);
    // the CURRENT source policy with WHOLE scoring keeps its row distances
    const bool keep_hdist = p.source_policy == INPAINT_SOURCE_CURRENT && p.scoring == INPAINT_SCORE_WHOLE;
    L.hdist = keep_hdist ? take(n) : 0;
    L.st = take(sizeof(IterState));
    L.sync = take(sizeof(FillSync));
    L.fslot = take(8 * (uint64_t)L.max_tiles);
    L.info = take(sizeof(InitInfo));
    L.key = take(8);
    // one-job plan of the batched persistent dispatch (images whose tiles
    // outnumber the co-resident work-groups): slot, committer id, items, first
    L.mplan = take(sizeof(JobDev) + 256 + sizeof(WorkItem) * (uint64_t)L.max_tiles + 4ull * (kMaxGroups + 1));
    L.log_cap = log_capacity(W, H, p);
    L.log = take(sizeof(StepRec) * (uint64_t)L.log_cap);
    L.total = off;
    return L;
}

const char *status_name(int32_t s) {
    switch (s) {
        case INPAINT_OK: return "ok";
        case INPAINT_DONE: return "done";
        case INPAINT_INVALID_ARGUMENT: return "invalid argument";
        case INPAINT_NO_CANDIDATE: return "no valid source centre in the search rectangle";
        case INPAINT_OUT_OF_MEMORY: return "out of memory";
        case INPAINT_DEVICE: return "device error";
        default: return "unknown status";
    }
}

// Alpha-window axis (Eq. 6): the object spans [b0, b1) on an axis of length n;
// the window is round_half_up((1 + 2 alpha) * w) wide, the extra split with the
// smaller half on the low side, clipped to [0, n).
void alpha_axis(int b0, int b1, int n, int an, int ad, int *lo, int *hi) {
    const int64_t w = b1 - b0;
    const int64_t num = w * (ad + 2 * (int64_t)an);
    const int64_t total = (2 * num + ad) / (2 * (int64_t)ad);
    const int64_t extra = total - w;
    const int64_t e_lo = extra / 2, e_hi = extra - e_lo;
    *lo = (int)std::max<int64_t>(0, b0 - e_lo);
    *hi = (int)std::min<int64_t>(n, b1 + e_hi);
}

}  // namespace

struct inpaint_ctx {
    JobDev d{};
    inpaint_params p{};
    Layout L{};
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    int device = 0;           // device current at create (the workspace's)
    uint8_t *ws = nullptr;
    int64_t hole0 = 0;
    int64_t candidates = 0;
    inpaint_rect rect{};      // image-clipped search rect (reported)
    bool mfma = false;        // search on the matrix cores
    bool direct = false;      // SIMT search without LDS staging
    int32_t run_form = INPAINT_FORM_PLAIN;   // form inpaint_run uses
    bool multi = false;       // persistent form through the batched dispatch (tiles > co-resident groups)
    int multi_grid = 0;       // its grid
    MultiPlan mplan{};        // its one-job plan (in the workspace)
    int32_t sticky = 0;
    std::string err;
    IterState *h_state = nullptr;   // pinned mirror of the device state
    uint64_t *h_key = nullptr;      // pinned
    hipGraphExec_t graph = nullptr;
    int graph_n = 0;
    inpaint_batch *batch = nullptr;
    // search-kernel timing (inpaint_profile_search)
    bool prof = false;
    std::vector<hipEvent_t> ev0, ev1;   // one pair per iteration of a replay
    double prof_ms = 0.0;
    int64_t prof_n = 0;

    int32_t fail(int32_t st, const std::string &msg) {
        err = msg;
        return st;
    }
    int32_t hip_fail(hipError_t e, const char *what) {
        sticky = INPAINT_DEVICE;
        err = std::string(what) + ": " + hipGetErrorString(e);
        return INPAINT_DEVICE;
    }
    // Reads the device iteration state into the pinned mirror (synchronous).
    hipError_t pull_state() {
        hipError_t e = hipMemcpyAsync(h_state, d.st, sizeof(IterState), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        return e;
    }
    hipError_t set_limit(int64_t limit) {
        h_state->iter_limit = limit;
        return hipMemcpyAsync(&d.st->iter_limit, &h_state->iter_limit, sizeof(int64_t),
                              hipMemcpyHostToDevice, stream);
    }
};

#define HIP_OR_FAIL(ctx, expr, what)                  \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return (ctx)->hip_fail(e_, what); \
    } while (0)

extern "C" {

const char *inpaint_status_string(int32_t status) { return status_name(status); }

const char *inpaint_last_error(const inpaint_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

static int32_t check_params(int32_t W, int32_t H, const inpaint_params *p, std::string *why) {
    if (!p) {
        *why = "params is NULL";
        return INPAINT_INVALID_ARGUMENT;
    }
    if (p->patch_radius < 1 || p->patch_radius > kMaxRadius) {
        *why = "patch_radius must be in 1..8";
        return INPAINT_INVALID_ARGUMENT;
    }
    const int P = 2 * p->patch_radius + 1;
    if (W < P || H < P) {
        *why = "image smaller than the patch";
        return INPAINT_INVALID_ARGUMENT;
    }
    if ((int64_t)W * H >= (1ll << 31)) {
        *why = "image has 2^31 pixels or more";
        return INPAINT_INVALID_ARGUMENT;
    }
    if (p->search_mode < INPAINT_SEARCH_FULL || p->search_mode > INPAINT_SEARCH_RECT) {
        *why = "unknown search_mode";
        return INPAINT_INVALID_ARGUMENT;
    }
    if (p->search_mode == INPAINT_SEARCH_ALPHA && (p->alpha_num < 0 || p->alpha_den <= 0)) {
        *why = "alpha must be a non-negative rational with positive denominator";
        return INPAINT_INVALID_ARGUMENT;
    }
    if (p->search_mode == INPAINT_SEARCH_RECT && (p->rect.x0 > p->rect.x1 || p->rect.y0 > p->rect.y1)) {
        *why = "search rect has x0 > x1 or y0 > y1";
        return INPAINT_INVALID_ARGUMENT;
    }
    if (p->path < INPAINT_PATH_AUTO || p->path > INPAINT_PATH_SIMT_DIRECT) {
        *why = "unknown path";
        return INPAINT_INVALID_ARGUMENT;
    }
    if (p->form < INPAINT_FORM_PLAIN || p->form > INPAINT_FORM_PERSISTENT) {
        *why = "unknown form";
        return INPAINT_INVALID_ARGUMENT;
    }
    if (p->form != INPAINT_FORM_PLAIN && (p->iters_per_check < 1 || p->iters_per_check > kMaxDispatchIters)) {
        *why = "iters_per_check must be in 1 .. 33554430 in the stream, graph and persistent forms";
        return INPAINT_INVALID_ARGUMENT;
    }
    if (p->log_capacity < -1) {
        *why = "log_capacity must be >= -1";
        return INPAINT_INVALID_ARGUMENT;
    }
    if (p->tile_rows != 0 && !tile_rows_ok(p->tile_rows)) {
        *why = "tile_rows must be 0, 4, 8 or 16";
        return INPAINT_INVALID_ARGUMENT;
    }
    if (p->path == INPAINT_PATH_MFMA && !mfma_supported(p->patch_radius)) {
        *why = "the int8-MFMA search supports patch radius 1..6";
        return INPAINT_INVALID_ARGUMENT;
    }
    if (p->source_policy < INPAINT_SOURCE_ORIGINAL || p->source_policy > INPAINT_SOURCE_CURRENT) {
        *why = "unknown source_policy";
        return INPAINT_INVALID_ARGUMENT;
    }
    if (p->scoring < INPAINT_SCORE_WHOLE || p->scoring > INPAINT_SCORE_INTERSECT) {
        *why = "unknown scoring";
        return INPAINT_INVALID_ARGUMENT;
    }
    if (p->path == INPAINT_PATH_MFMA && (p->source_policy != INPAINT_SOURCE_ORIGINAL || p->scoring != INPAINT_SCORE_WHOLE)) {
        *why = "the int8-MFMA search supports only the default candidate domain";
        return INPAINT_INVALID_ARGUMENT;
    }
    if (p->path == INPAINT_PATH_MFMA && p->tile_rows != 0 && p->tile_rows != kMfmaTileRows) {
        *why = "the int8-MFMA search uses tile_rows 16";
        return INPAINT_INVALID_ARGUMENT;
    }
    for (int i = 0; i < 1; ++i)
        if (p->reserved[i] != 0) {
            *why = "reserved fields must be zero";
            return INPAINT_INVALID_ARGUMENT;
        }
    return INPAINT_OK;
}

// Whether the persistent fill with one tile per search work-group can run
// this job: the SIMT search with its tile shape or the MFMA search, and
// every work-group of the dispatch co-resident.
static bool persistent_fits(const inpaint_ctx *c) {
    const JobDev &d = c->d;
    const int ntiles = d.ntx * d.nty;
    // (the committer scans at most 32 slots per thread)
    if (c->direct || c->d.policy != INPAINT_SOURCE_ORIGINAL || c->d.isect) return false;
    if ((!c->mfma && d.tile_rows != kFillTileRows) || ntiles <= 0 || ntiles > 32 * kCommitThreads) return false;
    if ((int64_t)d.W * d.H > (1ll << kSlotIndexBits)) return false;   // slot word index field
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    if (fill_blocks_per_cu(d.r, c->mfma, &per_cu) != hipSuccess) return false;
    return (int64_t)fill_grid(ntiles) <= (int64_t)per_cu * cus;
}

// Search items of the batched persistent dispatch spread round-robin over
// n_search groups: item i goes to group i % n_search, so a job's tiles land
// on different groups.  Writes items grouped by search group and the CSR
// offsets first[0..n_search].
static void spread_items(const std::vector<WorkItem> &all, int n_search, std::vector<WorkItem> *items,
                         std::vector<int32_t> *first) {
    first->assign(n_search + 1, 0);
    for (size_t i = 0; i < all.size(); ++i) (*first)[i % n_search + 1] += 1;
    for (int w = 0; w < n_search; ++w) (*first)[w + 1] += (*first)[w];
    items->resize(all.size());
    std::vector<int32_t> pos(first->begin(), first->end() - 1);
    for (size_t i = 0; i < all.size(); ++i) (*items)[pos[i % n_search]++] = all[i];
}

// spread_items for a dispatch whose jobs have several radii: every search
// group gets items of one radius only.  The groups are shared out among the
// radii in proportion to their items (each radius at least one; every item
// its own group when all fit), then each radius spreads its items over its
// groups.  radius[i]: the radius of all[i]'s job.  Returns false when there
// are more radii than groups.
static bool spread_items_by_radius(const std::vector<WorkItem> &all, const std::vector<int> &radius, int n_search,
                                   std::vector<WorkItem> *items, std::vector<int32_t> *first) {
    std::map<int, std::vector<WorkItem>> by_r;
    for (size_t i = 0; i < all.size(); ++i) by_r[radius[i]].push_back(all[i]);
    const int nr = (int)by_r.size();
    if (nr > n_search) return false;
    std::vector<int> groups;
    if ((int64_t)all.size() <= n_search) {
        for (auto &kv : by_r) groups.push_back((int)kv.second.size());
    } else {
        // largest remainders after a floor of max(1, proportional share)
        std::vector<std::pair<double, int>> rem;
        int used = 0, k = 0;
        for (auto &kv : by_r) {
            const double share = (double)n_search * kv.second.size() / all.size();
            const int g = std::max(1, (int)share);
            groups.push_back(g);
            used += g;
            rem.push_back({share - g, k++});
        }
        std::sort(rem.begin(), rem.end(), [](const auto &x, const auto &y) {
            return x.first > y.first || (x.first == y.first && x.second < y.second);
        });
        for (size_t q = 0; used < n_search; q = (q + 1) % rem.size(), ++used) groups[rem[q].second] += 1;
        while (used > n_search) {   // the floors of 1 overshot: take from the largest
            const int big = (int)(std::max_element(groups.begin(), groups.end()) - groups.begin());
            groups[big] -= 1;
            used -= 1;
        }
    }
    items->clear();
    first->assign(1, 0);
    int k = 0;
    for (auto &kv : by_r) {
        std::vector<WorkItem> its;
        std::vector<int32_t> fst;
        spread_items(kv.second, groups[k++], &its, &fst);
        const int32_t base = first->back();
        for (size_t w = 1; w < fst.size(); ++w) first->push_back(base + fst[w]);
        items->insert(items->end(), its.begin(), its.end());
    }
    while ((int)first->size() < n_search + 1) first->push_back(first->back());   // idle groups
    return true;
}

// Co-resident work-groups of the batched persistent kernel on this device.
static int multi_capacity(bool mfma, int r) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (multi_blocks_per_cu(mfma, r, &per_cu) != hipSuccess) return 0;
    return std::min(per_cu * cus, kMaxGroups);
}

// The persistent form for a job whose tiles outnumber the co-resident
// work-groups: the batched dispatch with this one job, its tiles spread over
// every other co-resident group.  Builds and uploads the plan into the
// workspace.  Returns false when that does not fit either.
static bool setup_multi(inpaint_ctx *c) {
    const JobDev &d = c->d;
    const int ntiles = d.ntx * d.nty;
    if (c->direct || d.policy != INPAINT_SOURCE_ORIGINAL || d.isect) return false;
    if (!c->mfma && d.tile_rows != kFillTileRows) return false;
    if (ntiles <= 0 || ntiles > 32 * kCommitThreads || ntiles > c->L.max_tiles) return false;
    if ((int64_t)d.W * d.H > (1ll << kSlotIndexBits)) return false;
    const int cap = multi_capacity(c->mfma, d.r);
    const int n_search = cap - 1;
    if (n_search < 1 || ntiles > (int64_t)n_search * kMultiMaxItems) return false;
    std::vector<WorkItem> all(ntiles), items;
    std::vector<int32_t> first;
    for (int t = 0; t < ntiles; ++t) all[t] = WorkItem{0, t};
    spread_items(all, n_search, &items, &first);
    uint8_t *base = c->ws + c->L.mplan;
    JobDev *slot = (JobDev *)base;
    int32_t *commit = (int32_t *)(base + sizeof(JobDev));
    WorkItem *ditems = (WorkItem *)(base + sizeof(JobDev) + 256);
    int32_t *dfirst = (int32_t *)(base + sizeof(JobDev) + 256 + sizeof(WorkItem) * (uint64_t)c->L.max_tiles);
    const int32_t zero = 0;
    hipError_t e = hipMemcpy(slot, &d, sizeof(JobDev), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(commit, &zero, 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ditems, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dfirst, first.data(), 4 * first.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return false;
    c->mplan = MultiPlan{slot, commit, ditems, dfirst, 1};
    c->multi_grid = 1 + n_search;
    c->multi = true;
    return true;
}

int32_t inpaint_workspace_bytes(int32_t W, int32_t H, const inpaint_params *p, uint64_t *bytes) {
    std::string why;
    const int32_t st = check_params(W, H, p, &why);
    if (st != INPAINT_OK) return st;
    if (!bytes) return INPAINT_INVALID_ARGUMENT;
    *bytes = make_layout(W, H, *p).total;
    return INPAINT_OK;
}

// Kernel rectangle of candidate centres: the image-clipped rect further
// clipped to [r, W - r) x [r, H - r), outside of which no centre is valid.
// (INTERSECT scoring passes r = 0: its windows may leave the image.)
static void kernel_rect(int W, int H, int r, const inpaint_rect &img_rect, int *k) {
    k[0] = std::max(img_rect.x0, r);
    k[1] = std::max(img_rect.y0, r);
    k[2] = std::min(img_rect.x1, W - r);
    k[3] = std::min(img_rect.y1, H - r);
}

// Search tiles over the kernel rect; mfma_r > 0 selects the MFMA tiling of
// that radius (64 x 64 tiles from an aligned first column).
static void set_tiles(JobDev &d, int tile_rows, int mfma_r = 0) {
    d.tile_rows = tile_rows;
    const int rw = std::max(d.rx1 - d.rx0, 0), rh = std::max(d.ry1 - d.ry0, 0);
    const int tx0 = mfma_r > 0 ? mfma_tile_x0(d.rx0, mfma_r) : d.rx0;
    d.ntx = (std::max(d.rx1 - tx0, 0) + kTileW - 1) / kTileW;
    d.nty = (rh + search_tile_h(tile_rows) - 1) / search_tile_h(tile_rows);
    if (rw == 0 || rh == 0) d.ntx = d.nty = 0;
}

static int32_t create_fail(inpaint_ctx *c, int32_t st, const std::string &msg) {
    g_create_error = msg;
    if (c) {
        if (c->stream) hipStreamSynchronize(c->stream);
        if (c->h_state) hipHostFree(c->h_state);
        if (c->h_key) hipHostFree(c->h_key);
        if (c->cap_stream) hipStreamDestroy(c->cap_stream);
        delete c;
    }
    return st;
}

int32_t inpaint_create(const inpaint_image *img, const uint8_t *mask, int32_t mask_stride,
                       const inpaint_params *p, void *d_workspace, uint64_t ws_bytes, void *hip_stream,
                       inpaint_ctx **out) {
    SharedDevice lock(g_device_mu);
    g_create_error.clear();
    if (!img || !img->data || !mask || !out || !d_workspace)
        return create_fail(nullptr, INPAINT_INVALID_ARGUMENT, "NULL argument");
    const int W = img->width, H = img->height, ch = img->channels;
    std::string why;
    int32_t st = check_params(W, H, p, &why);
    if (st != INPAINT_OK) return create_fail(nullptr, st, why);
    if (ch != 3 && ch != 4) return create_fail(nullptr, INPAINT_INVALID_ARGUMENT, "channels must be 3 or 4");
    if (img->stride_bytes < W * ch || mask_stride < W)
        return create_fail(nullptr, INPAINT_INVALID_ARGUMENT, "row stride smaller than the row");
    if (((uintptr_t)d_workspace) % kAlign != 0)
        return create_fail(nullptr, INPAINT_INVALID_ARGUMENT, "workspace not 256-byte aligned");
    const Layout L = make_layout(W, H, *p);
    if (ws_bytes < L.total) return create_fail(nullptr, INPAINT_OUT_OF_MEMORY, "workspace too small");
    const MaskStats hm = mask_stats(mask, mask_stride, W, H);
    if (hm.count == 0) return create_fail(nullptr, INPAINT_INVALID_ARGUMENT, "mask is empty");
    if (hm.count >= (int64_t)W * H) return create_fail(nullptr, INPAINT_INVALID_ARGUMENT, "mask covers the whole image");

    inpaint_ctx *c = new (std::nothrow) inpaint_ctx();
    if (!c) return create_fail(nullptr, INPAINT_OUT_OF_MEMORY, "host allocation failed");
    c->p = *p;
    c->L = L;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (uint8_t *)d_workspace;
    if (hipHostMalloc((void **)&c->h_state, sizeof(IterState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->h_key, 64, hipHostMallocDefault) != hipSuccess)
        return create_fail(c, INPAINT_OUT_OF_MEMORY, "pinned host allocation failed");
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return create_fail(c, INPAINT_DEVICE, "stream creation failed");
    if (hipGetDevice(&c->device) != hipSuccess) return create_fail(c, INPAINT_DEVICE, "no current device");
    // Device address of the allocation-free query's scratch array on this
    // device (taken once per device; a failure only disables that query).
    static_scratch_setup(c->device);

    JobDev &d = c->d;
    uint8_t *ws = c->ws;
    d.img = (uint32_t *)(ws + L.img);
    d.gray = ws + L.gray;
    d.hole = ws + L.hole;
    d.hole0 = ws + L.hole0;
    d.vrad = ws + L.vrad;
    d.conf = (double *)(ws + L.conf);
    d.pcd = (double2 *)(ws + L.pcd);
    d.blk = (BlockBest *)(ws + L.blk);
    d.partials = (uint64_t *)(ws + L.partials);
    d.tgt = (TargetStage *)(ws + L.tgt);
    d.qtgt = (TargetStage *)(ws + L.qtgt);
    d.mfma = p->path == INPAINT_PATH_MFMA ? 1 : 0;
    d.srcw = d.mfma ? (uint32_t *)(ws + L.srcw) : nullptr;
    d.srcq = d.mfma ? (uint16_t *)(ws + L.srcq) : nullptr;
    d.srcp = (uint32_t *)(ws + L.srcp);
    d.vradp = ws + L.vradp;
    d.hdist = L.hdist ? ws + L.hdist : nullptr;
    d.policy = p->source_policy;
    d.isect = p->scoring == INPAINT_SCORE_INTERSECT ? 1 : 0;
    d.pitch = padded_pitch(W);
    d.st = (IterState *)(ws + L.st);
    d.sync = (FillSync *)(ws + L.sync);
    d.fslot = (uint64_t *)(ws + L.fslot);
    d.info = (InitInfo *)(ws + L.info);
    d.log = (StepRec *)(ws + L.log);
    d.W = W;
    d.H = H;
    d.r = p->patch_radius;
    d.log_cap = (int32_t)std::min<int64_t>(L.log_cap, INT32_MAX);
    d.nbw = (W + kBlock - 1) / kBlock;
    d.norm1 = 255.0;
    d.norm2 = std::sqrt(2.0) * 255.0;

    // Upload: compact RGB(A) rows and the mask into the staging area (the
    // priority-term plane, unused until the priorities are initialised).
    const uint64_t n = (uint64_t)W * H;
    uint8_t *stage_rgb = (uint8_t *)d.pcd;
    uint8_t *stage_mask = stage_rgb + 4 * n;
    uint8_t *hdist = d.hdist ? d.hdist : stage_mask + n;
    hipStream_t s = c->stream;
    hipError_t e = upload_rows(stage_rgb, (size_t)W * ch, img->data, img->stride_bytes, H, s);
    if (e == hipSuccess) e = upload_rows(stage_mask, W, mask, mask_stride, H, s);
    const uint32_t nonce = next_nonce();
    if (e == hipSuccess) e = launch_init(d, stage_rgb, ch, stage_mask, hdist, nonce, s);
    if (e == hipSuccess && d.mfma) e = launch_mfma_planes(d, s);
    if (e == hipSuccess) e = launch_seal(d, nonce, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->h_key, d.info, sizeof(InitInfo), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return create_fail(c, INPAINT_DEVICE, std::string("init: ") + hipGetErrorString(e));
    InitInfo info;
    std::memcpy(&info, c->h_key, sizeof(info));
    if (!sealed(info, nonce, init_pixel_blocks(d)))
        return create_fail(c, INPAINT_DEVICE, "init kernels did not run to completion (no error was reported)");
    if (info.hole_count != hm.count || info.bx0 != hm.x0 || info.bx1 != hm.x1 || info.by0 != hm.y0 ||
        info.by1 != hm.y1)
        return create_fail(c, INPAINT_DEVICE, "the initialisation read a mask other than the caller's "
                                              "(its upload had not landed)");
    c->hole0 = info.hole_count;

    // Search rectangle.
    inpaint_rect R{0, 0, W, H};
    if (p->search_mode == INPAINT_SEARCH_ALPHA) {
        alpha_axis(info.bx0, info.bx1, W, p->alpha_num, p->alpha_den, &R.x0, &R.x1);
        alpha_axis(info.by0, info.by1, H, p->alpha_num, p->alpha_den, &R.y0, &R.y1);
    } else if (p->search_mode == INPAINT_SEARCH_RECT) {
        R.x0 = std::max(p->rect.x0, 0);
        R.y0 = std::max(p->rect.y0, 0);
        R.x1 = std::min(p->rect.x1, W);
        R.y1 = std::min(p->rect.y1, H);
    }
    c->rect = R;
    int k[4];
    kernel_rect(W, H, d.isect ? 0 : d.r, R, k);
    d.rx0 = k[0];
    d.ry0 = k[1];
    d.rx1 = std::max(k[2], k[0]);
    d.ry1 = std::max(k[3], k[1]);
    c->mfma = p->path == INPAINT_PATH_MFMA;
    c->direct = p->path == INPAINT_PATH_SIMT_DIRECT;
    set_tiles(d, c->mfma ? kMfmaTileRows : (p->tile_rows ? p->tile_rows : kDefaultTileRows), c->mfma ? d.r : 0);

    // Priority blocks: the hole's bbox grown by 2r+1 (how far a fill can
    // change a priority), in 32x32 blocks.
    const int reach = 2 * d.r + 1;
    d.pbx0 = std::max(info.bx0 - reach, 0) / kBlock;
    d.pby0 = std::max(info.by0 - reach, 0) / kBlock;
    d.pbx1 = (std::min(info.bx1 + reach, W) + kBlock - 1) / kBlock;
    d.pby1 = (std::min(info.by1 + reach, H) + kBlock - 1) / kBlock;

    const uint32_t nonce2 = next_nonce();
    e = launch_count_valid(d, s);
    if (e == hipSuccess) e = launch_seal(d, nonce2, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->h_key, d.info, sizeof(InitInfo), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return create_fail(c, INPAINT_DEVICE, std::string("count: ") + hipGetErrorString(e));
    std::memcpy(&info, c->h_key, sizeof(info));
    if (info.seal != nonce2)
        return create_fail(c, INPAINT_DEVICE, "the candidate count did not run to completion (no error was reported)");
    if (info.valid_count <= 0)
        return create_fail(c, INPAINT_INVALID_ARGUMENT, "no valid source centre in the search rectangle");
    c->candidates = info.valid_count;

    IterState &h = *c->h_state;
    std::memset(&h, 0, sizeof(h));
    h.remaining = c->hole0;
    h.iter = 0;
    h.iter_limit = INT64_MAX;
    e = hipMemcpyAsync(d.st, &h, sizeof(IterState), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(d.sync, 0, sizeof(FillSync), s);
    if (e == hipSuccess) e = hipMemsetAsync(d.fslot, 0, 8 * (size_t)L.max_tiles, s);
    if (e == hipSuccess) e = launch_prio_init(d, s);
    if (e == hipSuccess) e = launch_commit(d, s);  // selects and stages the first target
    if (e == hipSuccess) e = c->pull_state();
    if (e != hipSuccess) return create_fail(c, INPAINT_DEVICE, std::string("first select: ") + hipGetErrorString(e));
    if (c->h_state->error) return create_fail(c, INPAINT_DEVICE, "device error during the first selection");
    if (!c->h_state->pending && !c->h_state->done)
        return create_fail(c, INPAINT_DEVICE, "the first selection did not run (no error was reported)");
    c->run_form = p->form;
    if (p->form == INPAINT_FORM_PERSISTENT && !persistent_fits(c) && !setup_multi(c))
        c->run_form = INPAINT_FORM_STREAM;
    *out = c;
    return INPAINT_OK;
}

int32_t inpaint_search_info(const inpaint_ctx *ctx, inpaint_rect *rect, int64_t *candidates) {
    if (!ctx) return INPAINT_INVALID_ARGUMENT;
    if (rect) *rect = ctx->rect;
    if (candidates) *candidates = ctx->candidates;
    return INPAINT_OK;
}

int32_t inpaint_find_exemplar(inpaint_ctx *ctx, int32_t tx, int32_t ty, int32_t r, inpaint_rect rect,
                              int64_t *source_index, uint32_t *ssd) {
    SharedDevice lock(g_device_mu);
    if (!ctx) return INPAINT_INVALID_ARGUMENT;
    if (ctx->sticky) return ctx->sticky;
    const JobDev &d = ctx->d;
    if (!source_index || !ssd) return ctx->fail(INPAINT_INVALID_ARGUMENT, "NULL output");
    if (tx < 0 || ty < 0 || tx >= d.W || ty >= d.H) return ctx->fail(INPAINT_INVALID_ARGUMENT, "target outside the image");
    if (r < 1 || r > kMaxRadius) return ctx->fail(INPAINT_INVALID_ARGUMENT, "patch_radius must be in 1..8");
    if (rect.x0 > rect.x1 || rect.y0 > rect.y1) return ctx->fail(INPAINT_INVALID_ARGUMENT, "x0 > x1 or y0 > y1");
    inpaint_rect R{std::max(rect.x0, 0), std::max(rect.y0, 0), std::min(rect.x1, d.W), std::min(rect.y1, d.H)};
    int k[4];
    kernel_rect(d.W, d.H, d.isect ? 0 : r, R, k);
    if (k[2] <= k[0] || k[3] <= k[1]) return ctx->fail(INPAINT_NO_CANDIDATE, "no valid centre in the rect");
    JobDev q = d;
    q.rx0 = k[0];
    q.ry0 = k[1];
    q.rx1 = k[2];
    q.ry1 = k[3];
    set_tiles(q, d.tile_rows, ctx->mfma && mfma_supported(r) ? r : 0);
    hipStream_t s = ctx->stream;
    uint64_t *dkey = (uint64_t *)(ctx->ws + ctx->L.key);
    HIP_OR_FAIL(ctx, launch_stage_query(q, tx, ty, r, s), "stage");
    if (ctx->mfma && mfma_supported(r))
        HIP_OR_FAIL(ctx, launch_search_mfma(q, true, r, q.rx0, q.ry0, q.rx1, q.ry1, q.ntx, q.nty, s), "search");
    else if (ctx->direct)
        HIP_OR_FAIL(ctx, launch_search_direct(q, true, r, q.rx0, q.ry0, q.rx1, q.ry1, q.tile_rows, q.ntx, q.nty, s),
                    "search");
    else
        HIP_OR_FAIL(ctx, launch_search(q, true, r, q.rx0, q.ry0, q.rx1, q.ry1, q.tile_rows, q.ntx, q.nty, s), "search");
    HIP_OR_FAIL(ctx, launch_reduce_partials(q, q.ntx * q.nty, dkey, s), "reduce");
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->h_key, dkey, 8, hipMemcpyDeviceToHost, s), "copy");
    HIP_OR_FAIL(ctx, hipStreamSynchronize(s), "sync");
    const uint64_t key = ctx->h_key[0];
    if (key == ~0ull) return ctx->fail(INPAINT_NO_CANDIDATE, "no valid centre in the rect");
    *source_index = (int64_t)(key & 0xffffffffu);
    *ssd = (uint32_t)(key >> 32);
    return INPAINT_OK;
}

// inpaint_find_exemplar with its scratch (target stage, MFMA operands, tile
// partials, key) in the static device array instead of the workspace.
int32_t inpaint_find_exemplar_static(inpaint_ctx *ctx, int32_t tx, int32_t ty, int32_t r, inpaint_rect rect,
                                     int64_t *source_index, uint32_t *ssd) {
    SharedDevice lock(g_device_mu);
    if (!ctx) return INPAINT_INVALID_ARGUMENT;
    if (ctx->sticky) return ctx->sticky;
    const JobDev &d = ctx->d;
    if (!source_index || !ssd) return ctx->fail(INPAINT_INVALID_ARGUMENT, "NULL output");
    if (tx < 0 || ty < 0 || tx >= d.W || ty >= d.H) return ctx->fail(INPAINT_INVALID_ARGUMENT, "target outside the image");
    if (r < 1 || r > kMaxRadius) return ctx->fail(INPAINT_INVALID_ARGUMENT, "patch_radius must be in 1..8");
    if (rect.x0 > rect.x1 || rect.y0 > rect.y1) return ctx->fail(INPAINT_INVALID_ARGUMENT, "x0 > x1 or y0 > y1");
    inpaint_rect R{std::max(rect.x0, 0), std::max(rect.y0, 0), std::min(rect.x1, d.W), std::min(rect.y1, d.H)};
    int k[4];
    kernel_rect(d.W, d.H, d.isect ? 0 : r, R, k);
    if (k[2] <= k[0] || k[3] <= k[1]) return ctx->fail(INPAINT_NO_CANDIDATE, "no valid centre in the rect");
    uint8_t *base = (uint8_t *)static_scratch(ctx->device);
    if (!base) return ctx->fail(INPAINT_DEVICE, "the static scratch array has no device address on this device");
    JobDev q = d;
    q.rx0 = k[0];
    q.ry0 = k[1];
    q.rx1 = k[2];
    q.ry1 = k[3];
    const bool mfma = ctx->mfma && mfma_supported(r);
    set_tiles(q, d.tile_rows, mfma ? r : 0);
    if ((int64_t)q.ntx * q.nty > kStaticMaxTiles)
        return ctx->fail(INPAINT_INVALID_ARGUMENT, "search rect needs more than " + std::to_string(kStaticMaxTiles) +
                                                       " search tiles (the static scratch limit)");
    q.qtgt = (TargetStage *)(base + kStaticStageOff);
    q.partials = (uint64_t *)(base + kStaticPartialsOff);
    uint64_t *dkey = (uint64_t *)(base + kStaticKeyOff);
    hipStream_t s = ctx->stream;
    HIP_OR_FAIL(ctx, launch_stage_query(q, tx, ty, r, s), "stage");
    if (mfma)
        HIP_OR_FAIL(ctx, launch_search_mfma(q, true, r, q.rx0, q.ry0, q.rx1, q.ry1, q.ntx, q.nty, s), "search");
    else if (ctx->direct)
        HIP_OR_FAIL(ctx, launch_search_direct(q, true, r, q.rx0, q.ry0, q.rx1, q.ry1, q.tile_rows, q.ntx, q.nty, s),
                    "search");
    else
        HIP_OR_FAIL(ctx, launch_search(q, true, r, q.rx0, q.ry0, q.rx1, q.ry1, q.tile_rows, q.ntx, q.nty, s), "search");
    HIP_OR_FAIL(ctx, launch_reduce_partials(q, q.ntx * q.nty, dkey, s), "reduce");
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->h_key, dkey, 8, hipMemcpyDeviceToHost, s), "copy");
    HIP_OR_FAIL(ctx, hipStreamSynchronize(s), "sync");
    const uint64_t key = ctx->h_key[0];
    if (key == ~0ull) return ctx->fail(INPAINT_NO_CANDIDATE, "no valid centre in the rect");
    *source_index = (int64_t)(key & 0xffffffffu);
    *ssd = (uint32_t)(key >> 32);
    return INPAINT_OK;
}

static hipError_t ensure_events(inpaint_ctx *ctx, size_t n) {
    while (ctx->ev0.size() < n) {
        hipEvent_t a, b;
        hipError_t e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        if (e != hipSuccess) return e;
        ctx->ev0.push_back(a);
        ctx->ev1.push_back(b);
    }
    return hipSuccess;
}

// One fill iteration: exemplar search, then the commit kernel.  With timing
// on, event pair `slot` brackets the search.
static hipError_t enqueue_iteration(inpaint_ctx *ctx, hipStream_t s, int slot = -1) {
    const JobDev &d = ctx->d;
    hipError_t e = hipSuccess;
    hipEvent_t e0 = slot >= 0 ? ctx->ev0[slot] : nullptr, e1 = slot >= 0 ? ctx->ev1[slot] : nullptr;
    if (ctx->mfma)
        e = launch_search_mfma(d, false, d.r, d.rx0, d.ry0, d.rx1, d.ry1, d.ntx, d.nty, s, e0, e1);
    else if (ctx->direct)
        e = launch_search_direct(d, false, d.r, d.rx0, d.ry0, d.rx1, d.ry1, d.tile_rows, d.ntx, d.nty, s, e0, e1);
    else
        e = launch_search(d, false, d.r, d.rx0, d.ry0, d.rx1, d.ry1, d.tile_rows, d.ntx, d.nty, s, e0, e1);
    if (e == hipSuccess) e = launch_commit(d, s);
    return e;
}

// Adds the search times of the first `ran` event pairs (after a sync).
static void collect_times(inpaint_ctx *ctx, int64_t ran) {
    for (int64_t i = 0; i < ran && i < (int64_t)ctx->ev0.size(); ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ctx->ev0[i], ctx->ev1[i]) == hipSuccess) {
            ctx->prof_ms += ms;
            ctx->prof_n += 1;
        }
    }
}

static int32_t check_device_state(inpaint_ctx *ctx) {
    if (ctx->h_state->error) {
        ctx->sticky = INPAINT_DEVICE;
        ctx->err = std::string("device-side error: ") + status_name(ctx->h_state->error);
        return INPAINT_DEVICE;
    }
    return INPAINT_OK;
}

int32_t inpaint_step(inpaint_ctx *ctx, inpaint_step_info *info) {
    SharedDevice lock(g_device_mu);
    if (!ctx) return INPAINT_INVALID_ARGUMENT;
    if (ctx->sticky) return ctx->sticky;
    if (ctx->batch) return ctx->fail(INPAINT_INVALID_ARGUMENT, "context is attached to a batch");
    if (ctx->h_state->done) return INPAINT_DONE;
    hipStream_t s = ctx->stream;
    const int64_t before = ctx->h_state->iter;
    HIP_OR_FAIL(ctx, ctx->set_limit(before + 1), "limit");
    if (ctx->prof) HIP_OR_FAIL(ctx, ensure_events(ctx, 1), "events");
    HIP_OR_FAIL(ctx, enqueue_iteration(ctx, s, ctx->prof ? 0 : -1), "launch");
    HIP_OR_FAIL(ctx, ctx->pull_state(), "state");
    if (check_device_state(ctx) != INPAINT_OK) return INPAINT_DEVICE;
    if (ctx->prof) collect_times(ctx, ctx->h_state->iter - before);
    if (info) std::memcpy(info, &ctx->h_state->last, sizeof(*info));
    return INPAINT_OK;
}

static hipError_t ensure_graph(inpaint_ctx *ctx, int G) {
    if (ctx->graph && ctx->graph_n == G) return hipSuccess;
    if (ctx->graph) {
        hipGraphExecDestroy(ctx->graph);
        ctx->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
    for (int i = 0; i < G && e == hipSuccess; ++i) e = enqueue_iteration(ctx, ctx->cap_stream);
    hipError_t e2 = hipStreamEndCapture(ctx->cap_stream, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&ctx->graph, g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    if (e == hipSuccess) ctx->graph_n = G;
    return e;
}

int32_t inpaint_run(inpaint_ctx *ctx, int64_t max_iters, int64_t *iters_done, inpaint_step_info *log,
                    int64_t log_cap) {
    if (!ctx) return INPAINT_INVALID_ARGUMENT;
    // the persistent form's dispatches run alone on the device
    SharedDevice shared(g_device_mu, std::defer_lock);
    ExclusiveDevice excl(g_device_mu, std::defer_lock);
    if (ctx->run_form == INPAINT_FORM_PERSISTENT) excl.lock();
    else shared.lock();
    if (ctx->sticky) return ctx->sticky;
    if (ctx->batch) return ctx->fail(INPAINT_INVALID_ARGUMENT, "context is attached to a batch");
    const int64_t start = ctx->h_state->iter;
    if (ctx->h_state->done) {
        if (iters_done) *iters_done = 0;
        return INPAINT_DONE;
    }
    const int64_t limit = max_iters < 0 ? INT64_MAX : start + max_iters;
    hipStream_t s = ctx->stream;
    HIP_OR_FAIL(ctx, ctx->set_limit(limit), "limit");
    const int form = ctx->run_form;
    const int G = form == INPAINT_FORM_PLAIN ? 1 : ctx->p.iters_per_check;
    if (form == INPAINT_FORM_GRAPH) {
        if (ctx->prof) return ctx->fail(INPAINT_INVALID_ARGUMENT, "search timing is not available in the graph form");
        HIP_OR_FAIL(ctx, ensure_graph(ctx, G), "graph capture");
    } else if (ctx->prof) {
        // (a persistent dispatch is timed as a whole: one pair)
        HIP_OR_FAIL(ctx, ensure_events(ctx, form == INPAINT_FORM_PERSISTENT ? 1 : G), "events");
    }
    for (;;) {
        const int64_t before = ctx->h_state->iter;
        if (form == INPAINT_FORM_GRAPH) {
            HIP_OR_FAIL(ctx, hipGraphLaunch(ctx->graph, s), "graph launch");
        } else if (form == INPAINT_FORM_PERSISTENT) {
            const int n = (int)std::min<int64_t>(G, limit - before);
            const JobDev &d = ctx->d;
            if (ctx->prof) HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev0[0], s), "event");
            if (ctx->multi)
                HIP_OR_FAIL(ctx, launch_fill_multi(ctx->mplan, ctx->mfma, d.r, ctx->multi_grid, n, next_epoch(), s),
                            "persistent launch");
            else
                HIP_OR_FAIL(ctx, launch_fill(d, d.ntx * d.nty, n, next_epoch(), s), "persistent launch");
            if (ctx->prof) HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev1[0], s), "event");
        } else {
            // Stop enqueueing at the iteration limit; past the end of the
            // hole the kernels are no-ops.
            const int64_t n = std::min<int64_t>(G, limit - before);
            for (int64_t i = 0; i < n; ++i)
                HIP_OR_FAIL(ctx, enqueue_iteration(ctx, s, ctx->prof ? (int)i : -1), "launch");
        }
        HIP_OR_FAIL(ctx, ctx->pull_state(), "state");
        if (check_device_state(ctx) != INPAINT_OK) return INPAINT_DEVICE;
        if (ctx->prof) collect_times(ctx, form == INPAINT_FORM_PERSISTENT ? 1 : ctx->h_state->iter - before);
        if (ctx->h_state->done || ctx->h_state->iter >= limit) break;
    }
    const int64_t ran = ctx->h_state->iter - start;
    if (iters_done) *iters_done = ran;
    if (log && log_cap > 0) {
        const int64_t avail = std::max<int64_t>(0, std::min<int64_t>(ctx->d.log_cap, start + ran) - start);
        const int64_t cnt = std::min(avail, log_cap);
        if (cnt > 0) {
            HIP_OR_FAIL(ctx, hipMemcpyAsync(log, ctx->d.log + start, cnt * sizeof(StepRec), hipMemcpyDeviceToHost, s),
                        "log copy");
            HIP_OR_FAIL(ctx, hipStreamSynchronize(s), "sync");
        }
    }
    return ctx->h_state->done ? INPAINT_DONE : INPAINT_OK;
}

int32_t inpaint_read_log(inpaint_ctx *ctx, int64_t first, int64_t count, inpaint_step_info *out) {
    SharedDevice lock(g_device_mu);
    if (!ctx || !out || first < 0 || count < 0) return INPAINT_INVALID_ARGUMENT;
    if (ctx->sticky) return ctx->sticky;
    HIP_OR_FAIL(ctx, ctx->pull_state(), "state");
    const int64_t have = std::min<int64_t>(ctx->h_state->iter, ctx->d.log_cap);
    if (first + count > have) return ctx->fail(INPAINT_INVALID_ARGUMENT, "records not in the log");
    if (count == 0) return INPAINT_OK;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(out, ctx->d.log + first, count * sizeof(StepRec), hipMemcpyDeviceToHost,
                                    ctx->stream), "log copy");
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream), "sync");
    return INPAINT_OK;
}

int32_t inpaint_read_image(inpaint_ctx *ctx, uint8_t *rgb, int32_t stride) {
    SharedDevice lock(g_device_mu);
    if (!ctx || !rgb) return INPAINT_INVALID_ARGUMENT;
    if (ctx->sticky) return ctx->sticky;
    const int W = ctx->d.W, H = ctx->d.H;
    if (stride < 3 * W) return ctx->fail(INPAINT_INVALID_ARGUMENT, "stride smaller than a row");
    std::vector<uint32_t> tmp((size_t)W * H);
    HIP_OR_FAIL(ctx, hipMemcpyAsync(tmp.data(), ctx->d.img, tmp.size() * 4, hipMemcpyDeviceToHost, ctx->stream), "copy");
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream), "sync");
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const uint32_t v = tmp[(size_t)y * W + x];
            uint8_t *o = rgb + (size_t)y * stride + 3 * x;
            o[0] = v & 255;
            o[1] = (v >> 8) & 255;
            o[2] = (v >> 16) & 255;
        }
    return INPAINT_OK;
}

int32_t inpaint_read_state(inpaint_ctx *ctx, uint8_t *mask, double *conf) {
    SharedDevice lock(g_device_mu);
    if (!ctx) return INPAINT_INVALID_ARGUMENT;
    if (ctx->sticky) return ctx->sticky;
    const size_t n = (size_t)ctx->d.W * ctx->d.H;
    if (mask) HIP_OR_FAIL(ctx, hipMemcpyAsync(mask, ctx->d.hole, n, hipMemcpyDeviceToHost, ctx->stream), "copy");
    if (conf) HIP_OR_FAIL(ctx, hipMemcpyAsync(conf, ctx->d.conf, n * 8, hipMemcpyDeviceToHost, ctx->stream), "copy");
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream), "sync");
    return INPAINT_OK;
}

int32_t inpaint_remaining(inpaint_ctx *ctx, int64_t *remaining) {
    SharedDevice lock(g_device_mu);
    if (!ctx || !remaining) return INPAINT_INVALID_ARGUMENT;
    if (ctx->sticky) return ctx->sticky;
    HIP_OR_FAIL(ctx, ctx->pull_state(), "state");
    *remaining = ctx->h_state->remaining;
    return INPAINT_OK;
}

int32_t inpaint_progress(inpaint_ctx *ctx, int64_t *iterations, int64_t *remaining) {
    SharedDevice lock(g_device_mu);
    if (!ctx) return INPAINT_INVALID_ARGUMENT;
    if (ctx->sticky) return ctx->sticky;
    HIP_OR_FAIL(ctx, ctx->pull_state(), "state");
    if (iterations) *iterations = ctx->h_state->iter;
    if (remaining) *remaining = ctx->h_state->remaining;
    return INPAINT_OK;
}

int32_t inpaint_import_state(inpaint_ctx *ctx, const uint8_t *rgb, int32_t rgb_stride, int32_t channels,
                             const uint8_t *hole, int32_t hole_stride, const double *conf, int64_t iterations) {
    SharedDevice lock(g_device_mu);
    if (!ctx) return INPAINT_INVALID_ARGUMENT;
    if (ctx->sticky) return ctx->sticky;
    if (ctx->batch) return ctx->fail(INPAINT_INVALID_ARGUMENT, "context is attached to a batch");
    const JobDev &d = ctx->d;
    const int W = d.W, H = d.H;
    if (!rgb || !hole || !conf) return ctx->fail(INPAINT_INVALID_ARGUMENT, "NULL checkpoint array");
    if (channels != 3 && channels != 4) return ctx->fail(INPAINT_INVALID_ARGUMENT, "channels must be 3 or 4");
    if (rgb_stride < W * channels || hole_stride < W)
        return ctx->fail(INPAINT_INVALID_ARGUMENT, "row stride smaller than a row");
    if (iterations < 0) return ctx->fail(INPAINT_INVALID_ARGUMENT, "iterations must be >= 0");
    const MaskStats hm = mask_stats(hole, hole_stride, W, H);
    hipStream_t s = ctx->stream;
    // Staging in the priority-term plane (16 bytes per pixel, rebuilt below):
    // colours [0, 4n), hole [4n, 5n), row distances [5n, 6n), confidences [8n, 16n).
    const uint64_t n = (uint64_t)W * H;
    uint8_t *stage = (uint8_t *)d.pcd;
    uint8_t *s_rgb = stage, *s_hole = stage + 4 * n, *s_hdist = stage + 5 * n;
    double *s_conf = (double *)(stage + 8 * n);
    HIP_OR_FAIL(ctx, upload_rows(s_rgb, (size_t)W * channels, rgb, rgb_stride, H, s), "upload");
    HIP_OR_FAIL(ctx, upload_rows(s_hole, W, hole, hole_stride, H, s), "upload");
    HIP_OR_FAIL(ctx, hipMemcpyAsync(s_conf, conf, 8 * n, hipMemcpyHostToDevice, s), "upload");
    const uint32_t nonce = next_nonce();
    HIP_OR_FAIL(ctx, launch_import_check(d, s_hole, s_conf, nonce, s), "check");
    HIP_OR_FAIL(ctx, launch_seal(d, nonce, s), "check");
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->h_key, d.info, sizeof(InitInfo), hipMemcpyDeviceToHost, s), "check");
    HIP_OR_FAIL(ctx, hipStreamSynchronize(s), "check");
    InitInfo info;
    std::memcpy(&info, ctx->h_key, sizeof(info));
    if (!sealed(info, nonce, init_pixel_blocks(d)))
        return ctx->hip_fail(hipErrorUnknown, "checkpoint check kernels did not run to completion");
    if (info.bad != 0) {
        // nothing changed but the priority terms the staging overwrote
        HIP_OR_FAIL(ctx, launch_prio_init(d, s), "restore");
        HIP_OR_FAIL(ctx, hipStreamSynchronize(s), "restore");
        return ctx->fail(INPAINT_INVALID_ARGUMENT,
                         "checkpoint hole leaves the original hole, or a filled pixel's confidence is not in [0, 1]");
    }
    const uint32_t nonce2 = next_nonce();
    HIP_OR_FAIL(ctx, launch_import_apply(d, s_rgb, channels, s_hole, s_conf, d.hdist ? d.hdist : s_hdist, nonce2, s),
                "import");
    HIP_OR_FAIL(ctx, launch_seal(d, nonce2, s), "import");
    HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->h_key, d.info, sizeof(InitInfo), hipMemcpyDeviceToHost, s), "import");
    HIP_OR_FAIL(ctx, hipStreamSynchronize(s), "import");
    std::memcpy(&info, ctx->h_key, sizeof(info));
    if (!sealed(info, nonce2, init_pixel_blocks(d)))
        return ctx->hip_fail(hipErrorUnknown, "checkpoint import kernels did not run to completion");
    // (the check passed: every hole pixel of the checkpoint is in the
    // original hole, so the overlay counted all of them)
    if (info.hole_count != hm.count)
        return ctx->hip_fail(hipErrorUnknown, "the import read a hole map other than the caller's "
                                              "(its upload had not landed)");
    IterState &h = *ctx->h_state;
    std::memset(&h, 0, sizeof(h));
    h.remaining = info.hole_count;
    h.iter = iterations;
    h.iter_limit = INT64_MAX;
    h.done = info.hole_count == 0 ? 1 : 0;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(d.st, &h, sizeof(IterState), hipMemcpyHostToDevice, s), "state");
    HIP_OR_FAIL(ctx, launch_prio_init(d, s), "priorities");
    HIP_OR_FAIL(ctx, launch_commit(d, s), "select");   // selects and stages the next target
    HIP_OR_FAIL(ctx, ctx->pull_state(), "state");
    if (ctx->h_state->error) return ctx->hip_fail(hipErrorUnknown, "device error during the selection");
    return INPAINT_OK;
}

int32_t inpaint_profile_search(inpaint_ctx *ctx, int32_t enable) {
    if (!ctx) return INPAINT_INVALID_ARGUMENT;
    ctx->prof = enable != 0;
    ctx->prof_ms = 0.0;
    ctx->prof_n = 0;
    return INPAINT_OK;
}

int32_t inpaint_search_time(inpaint_ctx *ctx, double *total_ms, int64_t *searches) {
    if (!ctx) return INPAINT_INVALID_ARGUMENT;
    if (total_ms) *total_ms = ctx->prof_ms;
    if (searches) *searches = ctx->prof_n;
    return INPAINT_OK;
}

int32_t inpaint_run_form(const inpaint_ctx *ctx, int32_t *form) {
    if (!ctx || !form) return INPAINT_INVALID_ARGUMENT;
    *form = ctx->run_form;
    return INPAINT_OK;
}

}  // extern "C"

static int32_t batch_detach(inpaint_batch *b, inpaint_ctx *ctx);

extern "C" {

int32_t inpaint_destroy(inpaint_ctx *ctx) {
    SharedDevice lock(g_device_mu);
    if (!ctx) return INPAINT_INVALID_ARGUMENT;
    if (ctx->batch) batch_detach(ctx->batch, ctx);
    hipStreamSynchronize(ctx->stream);
    if (ctx->graph) hipGraphExecDestroy(ctx->graph);
    for (auto ev : ctx->ev0) hipEventDestroy(ev);
    for (auto ev : ctx->ev1) hipEventDestroy(ev);
    if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
    if (ctx->h_state) hipHostFree(ctx->h_state);
    if (ctx->h_key) hipHostFree(ctx->h_key);
    delete ctx;
    return INPAINT_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batch

namespace {

struct TuneChoice {
    int tile_rows = kDefaultTileRows;
    int grid = 0;     // 0 = one work-group per item
    int engine = 0;   // search engine: 0 SIMT (dot4), 1 int8 MFMA (contexts with the MFMA planes)
};

struct RadiusGroup {
    std::vector<WorkItem> items;     // (slot, tile) search work list
    std::vector<int32_t> ids;        // slots of this radius (commit list)
    WorkItem *d_items = nullptr;
    int32_t *d_n = nullptr;          // [0] = items, [1] = ids
    int32_t *d_ids = nullptr;        // capacity entries
    int32_t *h_n = nullptr;          // pinned staging of the two counts
    size_t cap = 0;
    TuneChoice tune;
    bool tuned = false;
};

std::string device_key() {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    return std::string(prop.gcnArchName) + "-cu" + std::to_string(prop.multiProcessorCount);
}

// Minimal flat JSON cache: {"key": [tile_rows, grid, engine], ...}
std::map<std::string, TuneChoice> read_cache(const char *path) {
    std::map<std::string, TuneChoice> m;
    if (!path) return m;
    FILE *f = std::fopen(path, "r");
    if (!f) return m;
    std::string s;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, k);
    std::fclose(f);
    size_t pos = 0;
    while ((pos = s.find('"', pos)) != std::string::npos) {
        const size_t end = s.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = s.substr(pos + 1, end - pos - 1);
        TuneChoice t;
        if (std::sscanf(s.c_str() + end + 1, " : [ %d , %d , %d ]", &t.tile_rows, &t.grid, &t.engine) == 3 &&
            tile_rows_ok(t.tile_rows) && (t.engine == 0 || t.engine == 1))
            m[key] = t;
        pos = end + 1;
    }
    return m;
}

void write_cache(const char *path, const std::map<std::string, TuneChoice> &m) {
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto &kv : m)
        std::fprintf(f, "  \"%s\": [%d, %d, %d]%s\n", kv.first.c_str(), kv.second.tile_rows, kv.second.grid,
                     kv.second.engine, ++i < m.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

}  // namespace

// Device work tables of the batched persistent dispatch of one (search
// form, radius) group, grown as needed.
struct MultiBuf {
    int32_t *commit = nullptr;
    WorkItem *items = nullptr;
    int32_t *first = nullptr;
    size_t cap_commit = 0, cap_items = 0, cap_first = 0;
    MultiPlan plan{};
    int grid = 0;
    bool mfma = false;
    int r = 0;
};

struct inpaint_batch {
    inpaint_batch_params bp{};
    std::string cache_path;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    int device = 0;           // device current at create (the workspace's)
    std::vector<inpaint_ctx *> slots;
    JobDev *d_slots = nullptr;
    JobDev *h_slots = nullptr;      // pinned staging of the slot table
    int64_t *d_active = nullptr;    // [0] = active count, then capacity int32 slot states
    int64_t *h_active = nullptr;    // pinned mirror of the same
    std::map<int, RadiusGroup> groups;
    bool dirty = true;
    hipGraphExec_t graph = nullptr;
    int graph_n = 0;
    std::string graph_sig;
    int cu_count = 256;
    // batched persistent form
    std::vector<MultiBuf> mbufs;   // one per dispatch group of running jobs (mixed MFMA radii, or form and radius)
    std::string multi_sig;         // running slots the uploaded plans were built for
    std::string nofit_sig;         // running slots that did not fit one dispatch
    std::map<std::pair<int, int>, int> mcap;   // co-resident groups per (form, radius)
    int desc_form = -1;            // form the slot table's tilings were built for
    int32_t last_form = INPAINT_FORM_GRAPH;
};

namespace {

hipError_t upload_slot(inpaint_batch *b, int i) {
    return hipMemcpyAsync(b->d_slots + i, b->h_slots + i, sizeof(JobDev), hipMemcpyHostToDevice, b->stream);
}

// Graph-form groups: the images of one radius searched by the same kernel,
// keyed r, or r + kMfmaGroup for contexts that carry the MFMA planes (their
// group may search on the matrix cores, if the autotuner finds it faster).
constexpr int kMfmaGroup = 16;
int group_key(const inpaint_ctx *c) { return c->d.r + (c->mfma && mfma_supported(c->d.r) ? kMfmaGroup : 0); }
bool key_mfma(int key) { return key >= kMfmaGroup; }
int key_r(int key) { return key % kMfmaGroup; }

JobDev slot_desc(const inpaint_ctx *c, const TuneChoice &t) {
    JobDev d = c->d;
    if (t.engine == 1) set_tiles(d, kMfmaTileRows, c->d.r);
    else set_tiles(d, t.tile_rows);
    return d;
}

hipError_t launch_group_search(const inpaint_batch *b, int key, const RadiusGroup &g, int grid, hipStream_t s) {
    if (g.tune.engine == 1) return launch_search_batched_mfma(b->d_slots, g.d_items, g.d_n, key_r(key), grid, s);
    return launch_search_batched(b->d_slots, g.d_items, g.d_n, key_r(key), g.tune.tile_rows, grid, s);
}

hipError_t upload_group(inpaint_batch *b, RadiusGroup &g) {
    const size_t n = g.items.size();
    hipError_t e = hipSuccess;
    if (!g.d_ids) {
        e = hipMalloc(&g.d_ids, sizeof(int32_t) * b->slots.size());
        if (e == hipSuccess) e = hipMalloc(&g.d_n, 2 * sizeof(int32_t));
        if (e == hipSuccess) e = hipHostMalloc((void **)&g.h_n, 2 * sizeof(int32_t), hipHostMallocDefault);
        if (e != hipSuccess) return e;
    }
    if (n > g.cap || !g.d_items) {
        if (g.d_items) hipFree(g.d_items);
        g.cap = std::max<size_t>(n, 1024) * 2;
        e = hipMalloc(&g.d_items, g.cap * sizeof(WorkItem));
        if (e != hipSuccess) return e;
        b->graph_sig.clear();  // pointer changed: recapture
    }
    if (n) e = hipMemcpyAsync(g.d_items, g.items.data(), n * sizeof(WorkItem), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !g.ids.empty())
        e = hipMemcpyAsync(g.d_ids, g.ids.data(), g.ids.size() * sizeof(int32_t), hipMemcpyHostToDevice, b->stream);
    g.h_n[0] = (int32_t)n;
    g.h_n[1] = (int32_t)g.ids.size();
    if (e == hipSuccess) e = hipMemcpyAsync(g.d_n, g.h_n, 2 * sizeof(int32_t), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // host vectors may change next
    return e;
}

// Rebuilds every radius group's (slot, tile) list for its tile shape.
hipError_t rebuild(inpaint_batch *b) {
    for (auto &kv : b->groups) {
        kv.second.items.clear();
        kv.second.ids.clear();
    }
    for (size_t i = 0; i < b->slots.size(); ++i) {
        inpaint_ctx *c = b->slots[i];
        if (!c) continue;
        RadiusGroup &g = b->groups[group_key(c)];
        g.ids.push_back((int32_t)i);
        b->h_slots[i] = slot_desc(c, g.tune);
        const int nt = b->h_slots[i].ntx * b->h_slots[i].nty;
        for (int t = 0; t < nt; ++t) g.items.push_back(WorkItem{(int32_t)i, t});
        hipError_t e = upload_slot(b, (int)i);
        if (e != hipSuccess) return e;
    }
    for (auto &kv : b->groups) {
        hipError_t e = upload_group(b, kv.second);
        if (e != hipSuccess) return e;
    }
    b->dirty = false;
    return hipSuccess;
}

// Persistent grid of the batched search: the tuned size, else 8 work-groups
// per CU.  It does not depend on the work-list length, so a captured graph
// survives attach / detach.
int grid_for(const inpaint_batch *b, const RadiusGroup &g) {
    if (g.tune.grid > 0) return g.tune.grid;
    return 8 * b->cu_count;
}

// One batch iteration: the persistent search of every radius group, then
// the commit work-groups of every group.  Work-list lengths are read on the
// device, so the captured graph stays valid while slots come and go.
hipError_t enqueue_batch_iteration(inpaint_batch *b, hipStream_t s) {
    for (auto &kv : b->groups) {
        hipError_t e = launch_group_search(b, kv.first, kv.second, grid_for(b, kv.second), s);
        if (e != hipSuccess) return e;
    }
    for (auto &kv : b->groups) {
        hipError_t e = launch_commit_batched(b->d_slots, kv.second.d_ids, kv.second.d_n + 1,
                                             (int)b->slots.size(), key_r(kv.first), s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Times the batched search of one radius group for each tile shape and
// persistent grid size, keeps the fastest.  The searches only rewrite the
// images' partial results, which every real search rewrites before use.
hipError_t autotune_group(inpaint_batch *b, int gkey, RadiusGroup &g, std::map<std::string, TuneChoice> &cache) {
    int64_t pixels = 0;
    for (auto *c : b->slots)
        if (c && group_key(c) == gkey) pixels += (int64_t)(c->d.rx1 - c->d.rx0) * (c->d.ry1 - c->d.ry0);
    int lg = 0;
    while ((1ll << (lg + 1)) <= pixels) ++lg;
    const std::string key = device_key() + "/r" + std::to_string(key_r(gkey)) + (key_mfma(gkey) ? "/mfma" : "") +
                            "/px2^" + std::to_string(lg);
    auto it = cache.find(key);
    if (it != cache.end()) {
        g.tune = it->second;
        g.tuned = true;
        return rebuild(b);
    }
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    float best_ms = 1e30f;
    TuneChoice best = g.tune;
    // (engine, tile rows): the SIMT tile shapes, and the MFMA tile (one
    // shape, only its grid is tuned) where the contexts carry its planes
    std::vector<std::pair<int, int>> shapes = {{0, 4}, {0, 8}, {0, 16}};
    if (key_mfma(gkey)) shapes.push_back({1, kMfmaTileRows});
    for (const auto &shape : shapes) {
        const int rows = shape.second;
        g.tune.engine = shape.first;
        g.tune.tile_rows = rows;
        g.tune.grid = 0;
        hipError_t e = rebuild(b);
        if (e != hipSuccess) return e;
        const int n = (int)g.items.size();
        for (int grid : {b->cu_count, 2 * b->cu_count, 4 * b->cu_count, 8 * b->cu_count, 16 * b->cu_count}) {
            if (grid > 2 * n + b->cu_count) continue;
            g.tune.grid = grid;
            float ms_min = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                hipEventRecord(e0, b->stream);
                e = launch_group_search(b, gkey, g, grid_for(b, g), b->stream);
                hipEventRecord(e1, b->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e != hipSuccess) return e;
                float ms = 0;
                hipEventElapsedTime(&ms, e0, e1);
                ms_min = std::min(ms_min, ms);
            }
            if (ms_min < best_ms) {
                best_ms = ms_min;
                best = g.tune;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    g.tune = best;
    g.tuned = true;
    cache[key] = best;
    return rebuild(b);
}

template <class T>
hipError_t grow(T **p, size_t *cap, size_t n) {
    if (*p && *cap >= n) return hipSuccess;
    if (*p) hipFree(*p);
    *p = nullptr;
    *cap = std::max<size_t>(n, 64) * 2;
    return hipMalloc((void **)p, *cap * sizeof(T));
}

bool multi_form(const inpaint_ctx *c) { return c->mfma && mfma_supported(c->d.r); }

// A job's JobDev with the tiling of the batched persistent search.
static JobDev multi_desc(const inpaint_ctx *c) {
    JobDev d = c->d;
    set_tiles(d, multi_form(c) ? kMfmaTileRows : kFillTileRows, multi_form(c) ? c->d.r : 0);
    return d;
}

// One batched persistent dispatch: its kernel (form, radius or kMultiMixed),
// search groups, jobs (batch slots) and (slot, tile) items with their radii.
struct MultiGroupPlan {
    bool mfma;
    int r, n_search;
    std::vector<int> jobs;
    std::vector<WorkItem> all;
    std::vector<int> radius;
};

// Splits jobs (slot, context) into batched persistent dispatches: the
// MFMA-form jobs of radius up to kMultiMixMaxR share one (the mixed-radius
// kernel) when they have several radii, the others go by (search form,
// radius).  Each dispatch has its committers first, then every remaining
// co-resident work-group searching, each with at most max_items items.
// Returns false when a dispatch does not fit.
static bool group_multi(inpaint_batch *b, const std::vector<std::pair<int, const inpaint_ctx *>> &jobs,
                        int max_items, std::vector<MultiGroupPlan> *plans) {
    std::set<int> mix_radii;
    for (const auto &j : jobs)
        if (multi_form(j.second) && j.second->d.r <= kMultiMixMaxR) mix_radii.insert(j.second->d.r);
    std::map<std::pair<int, int>, std::vector<std::pair<int, const inpaint_ctx *>>> groups;
    for (const auto &j : jobs) {
        const inpaint_ctx *c = j.second;
        const bool mixed = mix_radii.size() > 1 && multi_form(c) && c->d.r <= kMultiMixMaxR;
        groups[{multi_form(c) ? 1 : 0, mixed ? kMultiMixed : c->d.r}].push_back(j);
    }
    plans->clear();
    for (auto &kv : groups) {
        MultiGroupPlan pl{kv.first.first != 0, kv.first.second, 0, {}, {}, {}};
        auto it = b->mcap.find(kv.first);
        const int cap = it != b->mcap.end() ? it->second : (b->mcap[kv.first] = multi_capacity(pl.mfma, pl.r));
        const int n_commit = (int)kv.second.size();
        pl.n_search = cap - n_commit;
        for (const auto &j : kv.second) {
            const JobDev d = multi_desc(j.second);
            const int nt = d.ntx * d.nty;
            if (nt > 32 * kCommitThreads || (int64_t)d.W * d.H > (1ll << kSlotIndexBits)) return false;
            pl.jobs.push_back(j.first);
            for (int t = 0; t < nt; ++t) {
                pl.all.push_back(WorkItem{j.first, t});
                pl.radius.push_back(d.r);
            }
        }
        bool fit = n_commit <= cap / 2 && pl.n_search >= 1;
        if (fit && pl.r == kMultiMixed) {
            // each radius within its own share of the search groups
            std::vector<WorkItem> items;
            std::vector<int32_t> first;
            fit = spread_items_by_radius(pl.all, pl.radius, pl.n_search, &items, &first);
            for (int w = 0; fit && w < pl.n_search; ++w) fit = first[w + 1] - first[w] <= max_items;
        } else if (fit) {
            fit = (int64_t)pl.all.size() <= (int64_t)pl.n_search * max_items;
        }
        if (!fit) return false;
        plans->push_back(std::move(pl));
    }
    return true;
}

// The running jobs of the batch as (slot, context).
static std::vector<std::pair<int, const inpaint_ctx *>> running_jobs(const inpaint_batch *b) {
    const int32_t *state = (const int32_t *)(b->h_active + 1);
    std::vector<std::pair<int, const inpaint_ctx *>> jobs;
    for (size_t i = 0; i < b->slots.size(); ++i)
        if (b->slots[i] && state[i] == INPAINT_SLOT_RUNNING) jobs.push_back({(int)i, b->slots[i]});
    return jobs;
}

// AUTO steps the batched persistent form once every search work-group has at
// most this many (image, tile) items (a group with several restages a tile
// per item and iteration; the graph form restages every tile every
// iteration, so a few items per group are still the cheaper of the two).
constexpr int kAutoPersistentItems = 4;

// Plans the batched persistent dispatches of the running jobs (group_multi)
// and uploads the slot table with each job's persistent tiling.  *fits =
// false when a dispatch does not fit (the batch then steps in the graph
// form).  max_items: search items per search group allowed (1: every tile
// stays in LDS for the whole dispatch).
hipError_t plan_multi(inpaint_batch *b, int max_items, bool *fits) {
    *fits = false;
    const auto jobs = running_jobs(b);
    std::string sig = std::to_string(max_items) + "/";
    for (const auto &j : jobs) sig += std::to_string(j.first) + ":" + std::to_string((uintptr_t)j.second) + ",";
    if (!b->dirty && b->desc_form == INPAINT_FORM_PERSISTENT && sig == b->multi_sig) {
        *fits = true;
        return hipSuccess;
    }
    if (!b->dirty && sig == b->nofit_sig) return hipSuccess;
    std::vector<MultiGroupPlan> plans;
    if (!group_multi(b, jobs, max_items, &plans)) {
        b->nofit_sig = sig;
        return hipSuccess;
    }
    std::vector<JobDev> desc(b->slots.size());
    for (size_t i = 0; i < b->slots.size(); ++i)
        if (b->slots[i]) desc[i] = multi_desc(b->slots[i]);
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < b->slots.size() && e == hipSuccess; ++i) {
        if (!b->slots[i]) continue;
        b->h_slots[i] = desc[i];
        e = upload_slot(b, (int)i);
    }
    if (e != hipSuccess) return e;
    b->desc_form = INPAINT_FORM_PERSISTENT;
    b->graph_sig.clear();   // the graph form rebuilds its tilings
    b->mbufs.resize(plans.size());
    for (size_t gi = 0; gi < plans.size(); ++gi) {
        const MultiGroupPlan &pl = plans[gi];
        MultiBuf &m = b->mbufs[gi];
        m.mfma = pl.mfma;
        m.r = pl.r;
        std::vector<WorkItem> items;
        std::vector<int32_t> first;
        if (pl.r == kMultiMixed)
            spread_items_by_radius(pl.all, pl.radius, pl.n_search, &items, &first);   // fits: checked above
        else
            spread_items(pl.all, pl.n_search, &items, &first);
        e = grow(&m.commit, &m.cap_commit, pl.jobs.size());
        if (e == hipSuccess) e = grow(&m.items, &m.cap_items, items.size());
        if (e == hipSuccess) e = grow(&m.first, &m.cap_first, first.size());
        if (e == hipSuccess)
            e = hipMemcpyAsync(m.commit, pl.jobs.data(), 4 * pl.jobs.size(), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(m.items, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(m.first, first.data(), 4 * first.size(), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);   // host vectors go out of scope
        if (e != hipSuccess) return e;
        m.plan = MultiPlan{b->d_slots, m.commit, m.items, m.first, (int32_t)pl.jobs.size()};
        m.grid = (int)pl.jobs.size() + pl.n_search;
    }
    b->multi_sig = sig;
    *fits = true;
    return hipSuccess;
}

}  // namespace

extern "C" {

int32_t inpaint_batch_create(const inpaint_batch_params *bp, void *hip_stream, inpaint_batch **out) {
    if (!bp || !out || bp->capacity < 1 || bp->graph_iters < 1 || bp->graph_iters > kMaxDispatchIters)
        return INPAINT_INVALID_ARGUMENT;
    if (bp->form != 0 && bp->form != INPAINT_FORM_GRAPH && bp->form != INPAINT_FORM_PERSISTENT)
        return INPAINT_INVALID_ARGUMENT;
    inpaint_batch *b = new (std::nothrow) inpaint_batch();
    if (!b) return INPAINT_OUT_OF_MEMORY;
    b->bp = *bp;
    if (bp->tune_cache) b->cache_path = bp->tune_cache;
    b->stream = (hipStream_t)hip_stream;
    b->slots.assign(bp->capacity, nullptr);
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) b->cu_count = prop.multiProcessorCount;
    hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&b->d_slots, sizeof(JobDev) * bp->capacity);
    const size_t status_bytes = sizeof(int64_t) + sizeof(int32_t) * (size_t)bp->capacity;
    if (e == hipSuccess) e = hipMalloc(&b->d_active, status_bytes);
    if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_slots, sizeof(JobDev) * bp->capacity, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_active, status_bytes, hipHostMallocDefault);
    if (e == hipSuccess) std::memset(b->h_active, 0, status_bytes);
    if (e == hipSuccess) {
        std::memset(b->h_slots, 0, sizeof(JobDev) * bp->capacity);
        e = hipMemcpyAsync(b->d_slots, b->h_slots, sizeof(JobDev) * bp->capacity, hipMemcpyHostToDevice, b->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        inpaint_batch_destroy(b);
        return INPAINT_DEVICE;
    }
    *out = b;
    return INPAINT_OK;
}

int32_t inpaint_batch_attach(inpaint_batch *b, inpaint_ctx *ctx, int32_t *slot) {
    SharedDevice lock(g_device_mu);
    if (!b || !ctx || ctx->batch || ctx->sticky) return INPAINT_INVALID_ARGUMENT;
    if (ctx->d.policy != INPAINT_SOURCE_ORIGINAL || ctx->d.isect)
        return ctx->fail(INPAINT_INVALID_ARGUMENT, "a batch runs only the default candidate domain");
    int i = 0;
    while (i < (int)b->slots.size() && b->slots[i]) ++i;
    if (i == (int)b->slots.size()) return INPAINT_INVALID_ARGUMENT;
    // Make sure the context's own work has finished and its limit is open.
    if (ctx->set_limit(INT64_MAX) != hipSuccess || hipStreamSynchronize(ctx->stream) != hipSuccess)
        return ctx->hip_fail(hipErrorUnknown, "attach");
    b->slots[i] = ctx;
    ((int32_t *)(b->h_active + 1))[i] = ctx->h_state->done ? INPAINT_SLOT_FINISHED : INPAINT_SLOT_RUNNING;
    ctx->batch = b;
    if (b->groups.find(group_key(ctx)) == b->groups.end()) b->graph_sig.clear();
    b->groups[group_key(ctx)];
    b->dirty = true;
    if (slot) *slot = i;
    return INPAINT_OK;
}

int32_t inpaint_batch_detach(inpaint_batch *b, inpaint_ctx *ctx) {
    SharedDevice lock(g_device_mu);
    return batch_detach(b, ctx);
}

}  // extern "C"

static int32_t batch_detach(inpaint_batch *b, inpaint_ctx *ctx) {
    if (!b || !ctx || ctx->batch != b) return INPAINT_INVALID_ARGUMENT;
    for (size_t i = 0; i < b->slots.size(); ++i)
        if (b->slots[i] == ctx) {
            hipStreamSynchronize(b->stream);
            b->slots[i] = nullptr;
            std::memset(&b->h_slots[i], 0, sizeof(JobDev));
            upload_slot(b, (int)i);
            hipStreamSynchronize(b->stream);
        }
    ctx->batch = nullptr;
    ctx->pull_state();
    b->dirty = true;
    return INPAINT_OK;
}

extern "C" {

// One batch step in the batched persistent form: every planned group runs G
// iterations of its jobs in one persistent dispatch.
static hipError_t step_multi(inpaint_batch *b, int32_t G) {
    for (const MultiBuf &m : b->mbufs) {
        hipError_t e = launch_fill_multi(m.plan, m.mfma, m.r, m.grid, G, next_epoch(), b->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static int32_t finish_step(inpaint_batch *b, int64_t *active) {
    const int ns = (int)b->slots.size();
    hipError_t e = launch_count_active(b->d_slots, ns, b->d_active, (int32_t *)(b->d_active + 1), b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->h_active, b->d_active, sizeof(int64_t) + sizeof(int32_t) * ns, hipMemcpyDeviceToHost,
                           b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return INPAINT_DEVICE;
    if (active) *active = *b->h_active;
    return INPAINT_OK;
}

int32_t inpaint_batch_step(inpaint_batch *b, int32_t G, int64_t *active) {
    if (!b || G < 1) return INPAINT_INVALID_ARGUMENT;
    SharedDevice lock(g_device_mu);
    hipError_t e = hipSuccess;
    if (b->bp.form != INPAINT_FORM_GRAPH) {
        // AUTO takes the persistent form only while every search tile of
        // the running images can stay in LDS for the whole dispatch: with
        // more tiles than search groups the tiles are re-staged for every
        // target, and the graph form's many small search work-groups hide
        // that latency better.  So a large batch starts in the graph form
        // and its tail, when few images are left, runs persistent.
        bool fits = false;
        e = plan_multi(b, b->bp.form == INPAINT_FORM_PERSISTENT ? kMultiMaxItems : kAutoPersistentItems, &fits);
        if (e != hipSuccess) return INPAINT_DEVICE;
        if (fits) {
            b->dirty = false;
            b->last_form = INPAINT_FORM_PERSISTENT;
            // the dispatches run alone on the device
            lock.unlock();
            ExclusiveDevice excl(g_device_mu);
            e = step_multi(b, G);
            if (e != hipSuccess) return INPAINT_DEVICE;
            return finish_step(b, active);
        }
        if (b->bp.form == INPAINT_FORM_PERSISTENT)
            return INPAINT_INVALID_ARGUMENT;   // required, but the jobs do not fit one dispatch
    }
    b->last_form = INPAINT_FORM_GRAPH;
    if (b->desc_form != INPAINT_FORM_GRAPH) b->dirty = true;
    if (b->dirty) e = rebuild(b);
    if (e != hipSuccess) return INPAINT_DEVICE;
    b->desc_form = INPAINT_FORM_GRAPH;
    if (b->bp.autotune) {
        std::map<std::string, TuneChoice> cache;
        bool loaded = false, changed = false;
        for (auto &kv : b->groups) {
            if (kv.second.tuned || kv.second.items.empty()) continue;
            if (!loaded) {
                cache = read_cache(b->cache_path.empty() ? nullptr : b->cache_path.c_str());
                loaded = true;
            }
            e = autotune_group(b, kv.first, kv.second, cache);
            if (e != hipSuccess) return INPAINT_DEVICE;
            changed = true;
            b->graph_sig.clear();
        }
        if (changed && !b->cache_path.empty()) write_cache(b->cache_path.c_str(), cache);
    }
    std::string sig = std::to_string(G);
    for (auto &kv : b->groups)
        sig += "|" + std::to_string(kv.first) + ":" + std::to_string(kv.second.tune.engine) + ":" +
               std::to_string(kv.second.tune.tile_rows) + ":" +
               std::to_string(grid_for(b, kv.second));
    if (sig != b->graph_sig || !b->graph) {
        if (b->graph) hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
        hipGraph_t g = nullptr;
        e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
        for (int i = 0; i < G && e == hipSuccess; ++i) e = enqueue_batch_iteration(b, b->cap_stream);
        hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
        if (g) hipGraphDestroy(g);
        if (e != hipSuccess) return INPAINT_DEVICE;
        b->graph_sig = sig;
        b->graph_n = G;
    }
    e = hipGraphLaunch(b->graph, b->stream);
    if (e != hipSuccess) return INPAINT_DEVICE;
    return finish_step(b, active);
}

int32_t inpaint_batch_form(const inpaint_batch *b, int32_t *form) {
    if (!b || !form) return INPAINT_INVALID_ARGUMENT;
    *form = b->last_form;
    return INPAINT_OK;
}

int32_t inpaint_batch_room(inpaint_batch *b, const inpaint_ctx *ctx, int32_t tiles_per_group, int32_t *room) {
    SharedDevice lock(g_device_mu);
    if (!b || !ctx || !room || ctx->batch || tiles_per_group < 1 || tiles_per_group > kMultiMaxItems)
        return INPAINT_INVALID_ARGUMENT;
    auto jobs = running_jobs(b);
    jobs.push_back({(int)b->slots.size(), ctx});   // (a slot index no running job uses)
    std::vector<MultiGroupPlan> plans;
    *room = group_multi(b, jobs, tiles_per_group, &plans) ? 1 : 0;
    return INPAINT_OK;
}

int32_t inpaint_batch_status(const inpaint_batch *b, int32_t slot, int32_t *status) {
    if (!b || !status || slot < 0 || slot >= (int32_t)b->slots.size()) return INPAINT_INVALID_ARGUMENT;
    *status = b->slots[slot] ? ((const int32_t *)(b->h_active + 1))[slot] : INPAINT_SLOT_EMPTY;
    return INPAINT_OK;
}

int32_t inpaint_batch_destroy(inpaint_batch *b) {
    SharedDevice lock(g_device_mu);
    if (!b) return INPAINT_INVALID_ARGUMENT;
    for (auto *c : b->slots)
        if (c) c->batch = nullptr;
    if (b->stream) hipStreamSynchronize(b->stream);
    if (b->graph) hipGraphExecDestroy(b->graph);
    for (MultiBuf &m : b->mbufs) {
        if (m.commit) hipFree(m.commit);
        if (m.items) hipFree(m.items);
        if (m.first) hipFree(m.first);
    }
    for (auto &kv : b->groups) {
        if (kv.second.d_items) hipFree(kv.second.d_items);
        if (kv.second.d_n) hipFree(kv.second.d_n);
        if (kv.second.d_ids) hipFree(kv.second.d_ids);
        if (kv.second.h_n) hipHostFree(kv.second.h_n);
    }
    if (b->d_slots) hipFree(b->d_slots);
    if (b->d_active) hipFree(b->d_active);
    if (b->h_slots) hipHostFree(b->h_slots);
    if (b->h_active) hipHostFree(b->h_active);
    if (b->cap_stream) hipStreamDestroy(b->cap_stream);
    delete b;
    return INPAINT_OK;
}

}  // extern "C"
