// Device-side state of one removal job and the kernel entry points of
// libinpaint.so.  Included by the HIP kernel sources and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "inpaint.h"

namespace inpaint {

constexpr int kMaxRadius = 8;
constexpr int kMaxPatch = 2 * kMaxRadius + 1;          // 17
constexpr int kMaxOffsets = kMaxPatch * kMaxPatch;     // 289
constexpr int kMaskWords = (kMaxOffsets + 31) / 32;    // 10
constexpr int kBlock = 8;                              // priority block side (one wave)
constexpr int kTileW = 64;                             // search tile width (one wave)
constexpr int kSearchWaves = 4;                        // waves per search work-group
constexpr int kCommitThreads = 256;   // one work-group per image; 512 VGPRs per thread
constexpr int kMfmaMaxRadius = 6;     // int8-MFMA search: patches up to 13x13
constexpr int kMfmaTileRows = 16;     // MFMA search tile: 64 x 64 candidates
constexpr int kFillTileRows = 8;      // persistent fill: candidate rows per search thread

// Padding of the static search planes (srcp, vradp, srcw, srcq) around the
// image, in pixels: every staged search window -- a tile of up to 64 x 64
// candidates, its halo of up to kMaxRadius and the alignment of its start --
// lies inside the padded plane, so the search loads need no bounds checks.
// The pitch is a multiple of 8 pixels, so rows of every plane start on a
// 16-byte boundary.
constexpr int kPadL = 8, kPadT = 8, kPadR = 84, kPadB = 72;
__host__ __device__ inline int padded_pitch(int W) { return (kPadL + W + kPadR + 7) / 8 * 8; }
__host__ __device__ inline int padded_rows(int H) { return kPadT + H + kPadB; }
// First tile column of the MFMA search over a rect starting at rx0: moved
// left (by at most 7) so that every tile's staged window, which starts r
// columns left of the tile, starts on an 8-pixel boundary of the padded
// planes.  Columns left of rx0 are not candidates.
__host__ __device__ inline int mfma_tile_x0(int rx0, int r) { return rx0 - ((rx0 - r + kPadL) & 7); }

// Target patch as the search kernels read it.  Offset o = (dx, dy) has slot
// (dx + r) * P + (dy + r) (column-major, so one column's P values are
// contiguous).  tpix holds the target's RGBX word (X = 0) where the pixel is
// known and 0 elsewhere; bit `slot` of mbits is 1 where known.  sbits
// (ebits) mark the first (last) slot of each run of known slots in a column.
struct alignas(256) TargetStage {
    int32_t tx, ty, r, k;
    uint32_t t2;                 // sum over known pixels of R^2 + G^2 + B^2
    uint32_t pad0[3];
    uint32_t mbits[16];
    uint32_t sbits[16];
    uint32_t ebits[16];
    uint32_t tpix[kMaxOffsets + 15];
};

// One fill-iteration record, same layout as inpaint_step_info.
struct StepRec {
    int64_t target_index, source_index;
    uint32_t ssd;
    int32_t known_k, n_filled, reserved;
    double priority, confidence, data_term;
    int64_t remaining;
};
static_assert(sizeof(StepRec) == sizeof(inpaint_step_info), "record layout");

struct alignas(256) IterState {
    int64_t remaining;   // hole pixels left
    int64_t iter;        // iterations committed so far
    int64_t iter_limit;  // commits stop (without finishing) at this count
    int32_t done;        // 1 once the hole is empty
    int32_t error;       // INPAINT_* error seen on the device, 0 if none
    int32_t pending;     // 1 while a target is staged awaiting its search
    int32_t pad0;
    int64_t p_idx;       // staged target pixel
    double C, D, Pr;     // its confidence, data term and priority
    StepRec last;        // record of the last committed iteration
};

// Handshake of the persistent fill kernel (one per job).  The committer
// publishes each staged target in kGoCopies identical records, each with a
// go word: (epoch << 32) | (k + 1) once target k of the dispatch is staged,
// (epoch << 32) | 0xffffffff to stop.  Search work-group t polls and reads
// record t % kGoCopies, so a thousand work-groups do not all hit the same
// lines; each reports in its own slot word, so no address takes more than
// one writer.
constexpr int kGoCopies = 16;
struct alignas(256) FillRec {
    uint64_t go;
    uint32_t t2, k;
    uint32_t mbits[kMaskWords], sbits[kMaskWords], ebits[kMaskWords];
    uint32_t tpix[kMaxOffsets];
};
struct FillSync {
    FillRec rec[kGoCopies];
};
// Slot word of a search work-group: its minimum key for one iteration and
// the iteration's tag in one 64-bit word (so one plain device-scope store
// publishes both): bits 38..63 SSD, 8..37 raster index, 0..7 tag
// (k mod 255) + 1, 0 = not reported.  A tile with no valid candidate
// reports SSD and index all ones.  Needs SSD < 2^26 (true for P <= 17) and
// images below 2^30 pixels.
constexpr int kSlotIndexBits = 30;
// Per-block maximum of the priority keys: larger key wins, ties go to the
// lower raster index.  key = bit pattern of the (non-negative) priority
// P = C * D for front pixels, -1 elsewhere.
struct BlockBest {
    int64_t key;
    int64_t idx;
};

// Results of the init, count and import kernels, read back by the host.
// nonce is written by the first kernel of a sequence, seal by its last one,
// and blocks counts the work-groups of the pixel pass that ran to the end,
// so the host can tell "the kernels ran and found nothing" (a caller error)
// from "the kernels did not run" (a device error).
struct InitInfo {
    int64_t hole_count;
    int32_t bx0, by0, bx1, by1;  // bounding box of the hole, half-open
    int64_t valid_count;         // valid source centres in the search rect
    int64_t bad;                 // pixels of an imported checkpoint that fail its checks
    uint32_t nonce, seal;        // per-call value, from the first and the last kernel
    uint32_t blocks;             // work-groups of the pixel pass that completed
    uint32_t pad;
};

// Everything a kernel needs about one job.  Passed by value to the
// single-image kernels and stored in the slot table for batched ones.
struct JobDev {
    uint32_t *img;       // RGBX, W*H
    uint8_t *gray;       // W*H
    uint8_t *hole;       // W*H, 1 = still to fill
    uint8_t *hole0;      // W*H, 1 = in the original hole (fixed at create)
    uint8_t *vrad;       // W*H, largest r <= 8 with a valid patch at the centre
    double *conf;        // W*H
    double2 *pcd;        // W*H (C, D) of front pixels; C = -1 elsewhere
    BlockBest *blk;      // ceil(W/8)*ceil(H/8)
    uint64_t *partials;  // one (ssd << 32 | index) per search tile
    TargetStage *tgt;    // staged target of the fill loop
    TargetStage *qtgt;   // staged target of inpaint_find_exemplar
    uint32_t *srcw;      // MFMA: original RGBX ^ 0x80808080, padded plane (static)
    uint16_t *srcq;      // MFMA: (|s'|^2 low byte - 128, high byte - 128), padded plane (static)
    uint32_t *srcp;      // source RGBX in the padded plane, zero outside the image and in the hole;
                         // with INTERSECT scoring the 4th byte is 1 on source pixels.  Static,
                         // except under the CURRENT source policy (filled pixels are added)
    uint8_t *vradp;      // vrad in the padded plane, zero outside the image (static as srcp);
                         // with INTERSECT scoring 1 on source pixels, 0 elsewhere
    uint8_t *hdist;      // CURRENT policy with WHOLE scoring: per pixel, the horizontal distance
                         // (capped at 10) to the nearest hole or out-of-image pixel of its row
    IterState *st;
    FillSync *sync;
    uint64_t *fslot;     // one slot word per search tile
    StepRec *log;
    InitInfo *info;
    int32_t W, H, r, log_cap;
    int32_t rx0, ry0, rx1, ry1;   // search rect of centres (clipped)
    int32_t pbx0, pby0, pbx1, pby1;  // priority block range (block units)
    int32_t nbw;                  // blocks per image row
    int32_t tile_rows;            // candidate rows per thread in the search
    int32_t ntx, nty;             // search tiles over the rect
    int32_t mfma;                 // 1: the search runs on the matrix cores
    int32_t pitch;                // row pitch of srcp / vradp in pixels (multiple of 4)
    int32_t policy;               // INPAINT_SOURCE_*
    int32_t isect;                // 1: INTERSECT scoring
    double norm1, norm2;          // 255 * |n| for |n|^2 = 1 and 2
};

// (image slot, tile) work item of the batched persistent search.
struct WorkItem {
    int32_t slot;
    int32_t tile;
};

// Work of one batched persistent dispatch (k_fill_multi*): committer group
// c < n_commit commits the job in slot commit[c]; search group w (block
// n_commit + w) scores items [first[w], first[w + 1]) of `items`, at most
// kMultiMaxItems of them.  Each slot's JobDev carries the tiling of the
// dispatch's search form.
constexpr int kMultiMaxItems = 64;
// Iterations one persistent dispatch may run: its go words count them in
// 25 bits (k + 1 < 2^25 - 1).
constexpr int kMaxDispatchIters = (1 << 25) - 2;
struct MultiPlan {
    const JobDev *slots;
    const int32_t *commit;
    const WorkItem *items;
    const int32_t *first;
    int32_t n_commit;
};

// ---- launchers (defined in the .hip files) ----
hipError_t launch_init(const JobDev &d, const uint8_t *stage_rgb, int channels,
                       const uint8_t *stage_mask, uint8_t *hdist, uint32_t nonce, hipStream_t s);
// Work-groups of the pixel pass of launch_init / launch_import_*.
uint32_t init_pixel_blocks(const JobDev &d);
// Writes info->seal = nonce once every earlier kernel on the stream is done.
hipError_t launch_seal(const JobDev &d, uint32_t nonce, hipStream_t s);
hipError_t launch_count_valid(const JobDev &d, hipStream_t s);
// Checkpoint import: the checks (counted into info->bad, nothing written),
// then the overlay of the original-hole pixels (remaining hole counted into
// info->hole_count) and, under the CURRENT source policy, the rebuilt source
// and validity planes.
hipError_t launch_import_check(const JobDev &d, const uint8_t *hole, const double *conf, uint32_t nonce,
                               hipStream_t s);
hipError_t launch_import_apply(const JobDev &d, const uint8_t *rgb, int channels, const uint8_t *hole,
                               const double *conf, uint8_t *hdist, uint32_t nonce, hipStream_t s);
hipError_t launch_prio_init(const JobDev &d, hipStream_t s);
hipError_t launch_commit(const JobDev &d, hipStream_t s);
// SIMT search of one target; `d.isect` selects INTERSECT scoring.
hipError_t launch_search(const JobDev &d, bool query, int r, int rx0, int ry0, int rx1, int ry1,
                         int tile_rows, int ntx, int nty, hipStream_t s,
                         hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// The same search without LDS staging (source words read from the padded
// plane through the vector caches).
hipError_t launch_search_direct(const JobDev &d, bool query, int r, int rx0, int ry0, int rx1, int ry1,
                                int tile_rows, int ntx, int nty, hipStream_t s,
                                hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
bool mfma_supported(int r);
// int8-MFMA form of the search; same tiling as launch_search with tile_rows 16.
hipError_t launch_search_mfma(const JobDev &d, bool query, int r, int rx0, int ry0, int rx1, int ry1, int ntx, int nty,
                              hipStream_t s, hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
hipError_t launch_mfma_planes(const JobDev &d, hipStream_t s);
// The batch's search over a static (slot, tile) list on the matrix cores;
// each slot carries the MFMA tiling.
hipError_t launch_search_batched_mfma(const JobDev *slots, const WorkItem *items, const int32_t *nitems, int r,
                                      int grid, hipStream_t s);
hipError_t launch_stage_query(const JobDev &d, int tx, int ty, int r, hipStream_t s);
hipError_t launch_reduce_partials(const JobDev &d, int ntiles, uint64_t *out, hipStream_t s);
hipError_t launch_commit_batched(const JobDev *slots, const int32_t *ids, const int32_t *n, int grid, int r,
                                 hipStream_t s);
hipError_t launch_count_active(const JobDev *slots, int nslots, int64_t *out, int32_t *status, hipStream_t s);
hipError_t launch_search_batched(const JobDev *slots, const WorkItem *items, const int32_t *nitems,
                                 int r, int tile_rows, int grid, hipStream_t s);
// Persistent fill: runs up to n_iters iterations of the job in
// one dispatch; needs fill_grid(ntiles) co-resident work-groups.
hipError_t fill_blocks_per_cu(int r, bool mfma, int *blocks);
int fill_grid(int ntiles);
hipError_t launch_fill(const JobDev &d, int ntiles, int n_iters, uint32_t epoch, hipStream_t s);
// Batched persistent fill: up to n_iters iterations of every job of the plan
// (all of patch radius r) in one persistent dispatch of `grid` = n_commit +
// search groups.  MFMA: r <= 6, the int8-MFMA tiling; SIMT: the SIMT tiling
// of kFillTileRows.  MFMA with r = kMultiMixed: one dispatch for jobs of any
// radius up to kMultiMixMaxR, each committer and each served item taking
// its job's radius.
constexpr int kMultiMixed = 0;
constexpr int kMultiMixMaxR = 5;
hipError_t multi_blocks_per_cu(bool mfma, int r, int *blocks);
hipError_t launch_fill_multi(const MultiPlan &m, bool mfma, int r, int grid, int n_iters, uint32_t epoch,
                             hipStream_t s);

inline int search_tile_h(int tile_rows) { return kSearchWaves * tile_rows; }

// Allocation-free query (inpaint_find_exemplar_static): its target stage,
// per-tile partial minima and result key live in one static device array of
// kStaticScratchBytes per GPU instead of the workspace.
constexpr int kStaticMaxTiles = 32768;
constexpr uint64_t kStaticStageOff = 0;
constexpr uint64_t kStaticKeyOff = (sizeof(TargetStage) + 255) / 256 * 256;
constexpr uint64_t kStaticPartialsOff = kStaticKeyOff + 256;
constexpr uint64_t kStaticScratchBytes = kStaticPartialsOff + 8ull * kStaticMaxTiles;
// Takes the array's device address on `device`, which must be current
// (once per device; later calls return the first result).
hipError_t static_scratch_setup(int device);
// The address static_scratch_setup took on `device`, or NULL.
void *static_scratch(int device);

}  // namespace inpaint
