/*
 * CPU oracle for exemplar-based object removal (Criminisi-style best-first
 * patch filling), written from the paper's statement of the method.
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no code, header, table or constant with the HIP library: it is a
 * plain, single-threaded, slow and obviously correct restatement of what one
 * removal computes, so that the GPU path can be compared with it byte for byte.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared oracle.c -o liboracle.so -lm
 * (no fast-math; contraction off so every double operation rounds once, in the
 * order written here).
 *
 * What the method computes (paper, Section 3 and Section 5):
 *   - Source image S, hole (target region) Omega, known region Phi = S - Omega.
 *   - Fill front dOmega: the border of the hole.
 *   - Priority P(p) = C(p) * D(p) for p on the front (Eq. 1), with the
 *     confidence term C(p) = sum of C(q) over the known part of the patch
 *     divided by the patch area, and the data term D(p) = |isophote . normal|
 *     / 255 (Eq. 2).
 *   - The front pixel of maximum priority is filled next.
 *   - findBestPatch: the source patch minimising the sum of squared RGB
 *     differences over the target patch's known pixels (Eq. 3, Eq. 4).
 *   - Copy the chosen patch's pixels into the target's hole pixels, give them
 *     the target's confidence, and repeat until the hole is empty.
 *   - Optional search window: the hole's bounding box grown by alpha*w to the
 *     left and right and alpha*h up and down, clipped to the image (Eq. 6).
 *
 * Readings of points the paper leaves silent or prints garbled (each is also
 * listed in the design notes of the repository):
 *   R1  hole pixels are zeroed at create; no result may depend on them.
 *   R2  gray = (299 R + 587 G + 114 B + 500) div 1000 (integer BT.601).
 *   R3  alpha window: bbox [bx0,bx1)x[by0,by1) of the ORIGINAL hole, grown to
 *       round_half_up((1+2 alpha) w) wide (extra split floor-left/ceil-right),
 *       same in y, clipped; it bounds candidate centres.  (Eq. 6 prints o_x in
 *       the vertical bounds; the vertical bounds use the y centre and height.)
 *   R4  a candidate centre is valid iff its whole PxP window lies inside the
 *       image and inside the ORIGINAL known region Phi_0.
 *   R5  front = hole pixels with at least one in-image 4-neighbour known.
 *   R6  Eq. 2's confidence sum runs over the KNOWN pixels of the patch (the
 *       printed intersection with Omega would make every priority zero).
 *   R7  |Psi_p| is the constant P*P, also for patches clipped by the border.
 *   R8  the isophote is taken at the known pixel of the patch (all four
 *       4-neighbours in the image and known) with the largest central-
 *       difference gradient magnitude of the gray image, first in raster
 *       order on ties; isophote = (-gy, gx)/2.
 *   R9  the normal is the central difference of the hole indicator at p, with
 *       out-of-image pixels counted as hole, normalised by its length.
 *   R10 D takes the absolute value of the dot product.
 *   R12 ties: SSD ties go to the lowest raster index of the candidate centre;
 *       priority ties go to the lowest raster index of the front pixel.
 *   R13 SSD in exact integers over R, G, B only.
 *
 * Candidate-domain variants (selected at create; the defaults are the
 * readings above):
 *   source policy ORIGINAL (default): the source region Phi is the original
 *       known region Phi_0, so filled pixels never become sources (R4).
 *   source policy CURRENT: Phi is the current known region, so pixels become
 *       sources once they are filled (Section 3 defines Phi = S - Omega with
 *       Omega the region still to fill).
 *   scoring WHOLE (default): a candidate's whole window lies in the image and
 *       in Phi, and its SSD runs over the target's known pixels (R4).
 *   scoring INTERSECT: Eq. 4 read literally, as Section 5.4 describes for
 *       candidates that overlap the object.  Any centre in Phi is a candidate,
 *       whatever its window overlaps.  The SSD runs over the offsets where the
 *       target pixel is known AND the candidate pixel lies in the image and in
 *       Phi.  The copy fills only those hole pixels of the target whose source
 *       pixel lies in the image and in Phi (the rest stay in the hole for a
 *       later iteration); the centre is a source pixel, so the target pixel
 *       itself is always filled.  Which source pixels qualify is decided on the
 *       state before the copy.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_DONE 1
#define OR_INVALID_ARGUMENT (-1)
#define OR_NO_CANDIDATE (-2)
#define OR_OUT_OF_MEMORY (-3)

#define OR_SEARCH_FULL 0
#define OR_SEARCH_ALPHA 1
#define OR_SEARCH_RECT 2

#define OR_SOURCE_ORIGINAL 0
#define OR_SOURCE_CURRENT 1
#define OR_SCORE_WHOLE 0
#define OR_SCORE_INTERSECT 1

/* One record per fill iteration.  Field order and widths are fixed so Python
 * can read an array of them with a structured dtype. */
typedef struct {
    int64_t target_index;   /* raster index of the filled front pixel p^ */
    int64_t source_index;   /* raster index of the chosen source centre q^ */
    uint32_t ssd;           /* d(Psi_p^, Psi_q^) */
    int32_t known_k;        /* known pixels in the target patch */
    int32_t n_filled;       /* hole pixels filled this iteration */
    int32_t reserved;
    double priority;        /* P(p^) = C(p^) D(p^) */
    double confidence;      /* C(p^) */
    double data_term;       /* D(p^) */
    int64_t remaining;      /* hole pixels left after this iteration */
} oracle_step_info;

typedef struct {
    int32_t W, H, r, P;
    uint8_t *rgb;     /* current image I, H*W*3 */
    uint8_t *gray;    /* gray image, H*W */
    uint8_t *hole;    /* 1 where the pixel is in the current hole Omega */
    uint8_t *hole0;   /* 1 where the pixel is in the original hole Omega_0 */
    double *conf;     /* confidence C */
    int32_t rect[4];  /* candidate-centre search rectangle, half-open */
    int32_t policy;   /* OR_SOURCE_* */
    int32_t scoring;  /* OR_SCORE_* */
    int64_t remaining;
    int64_t iter;
    double norm[3];   /* 255 * |n| for |n|^2 = 1, 2 */
} oracle_state;

/* ---------------------------------------------------------------- helpers */

static int in_image(const oracle_state *s, int x, int y)
{
    return x >= 0 && y >= 0 && x < s->W && y < s->H;
}

/* Known = in the image and not in the current hole. */
static int known(const oracle_state *s, int x, int y)
{
    return in_image(s, x, y) && !s->hole[(int64_t)y * s->W + x];
}

/* The source region Phi: in the image and in the original known region, or
 * in the current known region under the CURRENT policy. */
static int in_source(const oracle_state *s, int x, int y)
{
    if (!in_image(s, x, y))
        return 0;
    int64_t i = (int64_t)y * s->W + x;
    return s->policy == OR_SOURCE_CURRENT ? !s->hole[i] : !s->hole0[i];
}

/* R4: the whole (2r+1)^2 window around (cx, cy) is inside the image and
 * inside the source region.  Under INTERSECT scoring only the centre has to
 * be a source pixel. */
static int valid_centre(const oracle_state *s, int cx, int cy, int r)
{
    if (s->scoring == OR_SCORE_INTERSECT)
        return in_source(s, cx, cy);
    if (cx - r < 0 || cy - r < 0 || cx + r >= s->W || cy + r >= s->H)
        return 0;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx)
            if (!in_source(s, cx + dx, cy + dy))
                return 0;
    return 1;
}

static int64_t round_half_up_div(int64_t num, int64_t den)
{
    /* floor(num/den + 1/2) for num >= 0, den > 0 */
    return (2 * num + den) / (2 * den);
}

/* R3 / Eq. 6: one axis of the alpha window.  The object spans [b0, b1) on
 * an axis of length n; the window is round_half_up((1 + 2 alpha) * w) wide,
 * the extra split floor to the low side and the rest to the high side. */
static void alpha_axis(int b0, int b1, int n, int an, int ad, int *lo, int *hi)
{
    int64_t w = b1 - b0;
    int64_t total = round_half_up_div(w * (ad + 2 * (int64_t)an), ad);
    int64_t extra = total - w;
    int64_t e_lo = extra / 2;
    int64_t e_hi = extra - e_lo;
    int64_t a = b0 - e_lo, b = b1 + e_hi;
    *lo = (int)(a < 0 ? 0 : a);
    *hi = (int)(b > n ? n : b);
}

/* ------------------------------------------------------------------ create */

int oracle_create(int32_t W, int32_t H, const uint8_t *rgb, int32_t rgb_stride,
                  int32_t channels, const uint8_t *mask, int32_t mask_stride,
                  int32_t r, int32_t search_mode, int32_t alpha_num,
                  int32_t alpha_den, const int32_t *rect, int32_t policy,
                  int32_t scoring, oracle_state **out)
{
    if (!rgb || !mask || !out || (channels != 3 && channels != 4))
        return OR_INVALID_ARGUMENT;
    if (r < 1 || r > 8)
        return OR_INVALID_ARGUMENT;
    int P = 2 * r + 1;
    if (W < P || H < P)
        return OR_INVALID_ARGUMENT;
    if (search_mode == OR_SEARCH_ALPHA && (alpha_num < 0 || alpha_den <= 0))
        return OR_INVALID_ARGUMENT;
    if (search_mode == OR_SEARCH_RECT && !rect)
        return OR_INVALID_ARGUMENT;
    if (search_mode < 0 || search_mode > 2)
        return OR_INVALID_ARGUMENT;
    if (policy < OR_SOURCE_ORIGINAL || policy > OR_SOURCE_CURRENT ||
        scoring < OR_SCORE_WHOLE || scoring > OR_SCORE_INTERSECT)
        return OR_INVALID_ARGUMENT;

    oracle_state *s = (oracle_state *)calloc(1, sizeof(oracle_state));
    if (!s)
        return OR_OUT_OF_MEMORY;
    int64_t n = (int64_t)W * H;
    s->W = W; s->H = H; s->r = r; s->P = P;
    s->policy = policy;
    s->scoring = scoring;
    s->rgb = (uint8_t *)malloc((size_t)n * 3);
    s->gray = (uint8_t *)malloc((size_t)n);
    s->hole = (uint8_t *)malloc((size_t)n);
    s->hole0 = (uint8_t *)malloc((size_t)n);
    s->conf = (double *)malloc((size_t)n * sizeof(double));
    if (!s->rgb || !s->gray || !s->hole || !s->hole0 || !s->conf) {
        free(s->rgb); free(s->gray); free(s->hole); free(s->hole0);
        free(s->conf); free(s);
        return OR_OUT_OF_MEMORY;
    }

    int64_t n_hole = 0;
    int bx0 = W, by0 = H, bx1 = 0, by1 = 0;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int64_t i = (int64_t)y * W + x;
            int h = mask[(int64_t)y * mask_stride + x] != 0;
            s->hole[i] = (uint8_t)h;
            s->hole0[i] = (uint8_t)h;
            const uint8_t *px = rgb + (int64_t)y * rgb_stride + (int64_t)x * channels;
            /* R1: hole pixels carry no information; zero them. */
            for (int c = 0; c < 3; ++c)
                s->rgb[i * 3 + c] = h ? 0 : px[c];
            /* R2: integer BT.601 luma, round half up. */
            int g = (299 * s->rgb[i * 3] + 587 * s->rgb[i * 3 + 1] +
                     114 * s->rgb[i * 3 + 2] + 500) / 1000;
            s->gray[i] = (uint8_t)g;
            /* Confidence starts at 1 on the known region, 0 in the hole. */
            s->conf[i] = h ? 0.0 : 1.0;
            if (h) {
                ++n_hole;
                if (x < bx0) bx0 = x;
                if (x + 1 > bx1) bx1 = x + 1;
                if (y < by0) by0 = y;
                if (y + 1 > by1) by1 = y + 1;
            }
        }
    }
    s->remaining = n_hole;
    s->iter = 0;
    s->norm[0] = 0.0;
    s->norm[1] = 255.0;
    s->norm[2] = sqrt(2.0) * 255.0;

    int bad = (n_hole == 0 || n_hole == n);
    if (!bad) {
        if (search_mode == OR_SEARCH_FULL) {
            s->rect[0] = 0; s->rect[1] = 0; s->rect[2] = W; s->rect[3] = H;
        } else if (search_mode == OR_SEARCH_ALPHA) {
            alpha_axis(bx0, bx1, W, alpha_num, alpha_den, &s->rect[0], &s->rect[2]);
            alpha_axis(by0, by1, H, alpha_num, alpha_den, &s->rect[1], &s->rect[3]);
        } else {
            if (rect[0] > rect[2] || rect[1] > rect[3])
                bad = 1;
            s->rect[0] = rect[0] < 0 ? 0 : rect[0];
            s->rect[1] = rect[1] < 0 ? 0 : rect[1];
            s->rect[2] = rect[2] > W ? W : rect[2];
            s->rect[3] = rect[3] > H ? H : rect[3];
        }
    }
    if (!bad) {
        /* At least one valid candidate centre must exist in the rectangle. */
        int any = 0;
        for (int y = s->rect[1]; y < s->rect[3] && !any; ++y)
            for (int x = s->rect[0]; x < s->rect[2] && !any; ++x)
                any = valid_centre(s, x, y, r);
        bad = !any;
    }
    if (bad) {
        free(s->rgb); free(s->gray); free(s->hole); free(s->hole0);
        free(s->conf); free(s);
        return OR_INVALID_ARGUMENT;
    }
    *out = s;
    return OR_OK;
}

void oracle_destroy(oracle_state *s)
{
    if (!s)
        return;
    free(s->rgb); free(s->gray); free(s->hole); free(s->hole0); free(s->conf);
    free(s);
}

/* ------------------------------------------------------------- fill front */

/* R5: hole pixel with at least one in-image 4-neighbour that is known. */
static int on_front(const oracle_state *s, int x, int y)
{
    if (!s->hole[(int64_t)y * s->W + x])
        return 0;
    return known(s, x + 1, y) || known(s, x - 1, y) ||
           known(s, x, y + 1) || known(s, x, y - 1);
}

/* Writes the front in raster order; returns its size (may exceed cap, in
 * which case only cap entries are written). */
int64_t oracle_front(const oracle_state *s, int32_t *out, int64_t cap)
{
    int64_t n = 0;
    for (int y = 0; y < s->H; ++y)
        for (int x = 0; x < s->W; ++x)
            if (on_front(s, x, y)) {
                if (out && n < cap)
                    out[n] = y * s->W + x;
                ++n;
            }
    return n;
}

/* -------------------------------------------------------------- priority */

/* Eq. 2, confidence term with R6 and R7. */
static double confidence_term(const oracle_state *s, int px, int py)
{
    int r = s->r;
    double sum = 0.0;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
            int x = px + dx, y = py + dy;
            if (known(s, x, y))
                sum = sum + s->conf[(int64_t)y * s->W + x];
        }
    return sum / (double)(s->P * s->P);
}

/* Hole indicator with out-of-image pixels counted as hole (R9). */
static int hole_or_outside(const oracle_state *s, int x, int y)
{
    return !in_image(s, x, y) || s->hole[(int64_t)y * s->W + x];
}

/* Eq. 2, data term with R8, R9 and R10. */
static double data_term(const oracle_state *s, int px, int py)
{
    int r = s->r, W = s->W;
    int gx = 0, gy = 0, best = -1;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
            int x = px + dx, y = py + dy;
            if (!known(s, x, y) || !known(s, x + 1, y) || !known(s, x - 1, y) ||
                !known(s, x, y + 1) || !known(s, x, y - 1))
                continue;
            int ax = (int)s->gray[(int64_t)y * W + x + 1] - (int)s->gray[(int64_t)y * W + x - 1];
            int ay = (int)s->gray[(int64_t)(y + 1) * W + x] - (int)s->gray[(int64_t)(y - 1) * W + x];
            int mag = ax * ax + ay * ay;
            if (mag > best) {
                best = mag;
                gx = ax;
                gy = ay;
            }
        }
    int nx = hole_or_outside(s, px + 1, py) - hole_or_outside(s, px - 1, py);
    int ny = hole_or_outside(s, px, py + 1) - hole_or_outside(s, px, py - 1);
    int kn = nx * nx + ny * ny;
    if (kn == 0)
        return 0.0;
    /* isophote (-gy, gx)/2 dotted with (nx, ny)/|n|, divided by 255 */
    int a = gx * ny - gy * nx;
    if (a < 0)
        a = -a;
    return (0.5 * (double)a) / s->norm[kn];
}

int oracle_priority(const oracle_state *s, int32_t x, int32_t y,
                    double *C, double *D, double *Pr)
{
    if (!in_image(s, x, y))
        return OR_INVALID_ARGUMENT;
    double c = confidence_term(s, x, y);
    double d = data_term(s, x, y);
    if (C) *C = c;
    if (D) *D = d;
    if (Pr) *Pr = c * d;   /* Eq. 1 */
    return OR_OK;
}

/* Front pixel of maximum priority; ties to the lowest raster index (R12). */
int oracle_select(const oracle_state *s, int64_t *idx, double *C, double *D, double *Pr)
{
    int64_t best_i = -1;
    double best_p = -1.0, best_c = 0.0, best_d = 0.0;
    for (int y = 0; y < s->H; ++y)
        for (int x = 0; x < s->W; ++x) {
            if (!on_front(s, x, y))
                continue;
            double c, d, p;
            oracle_priority(s, x, y, &c, &d, &p);
            if (p > best_p) {
                best_p = p; best_c = c; best_d = d;
                best_i = (int64_t)y * s->W + x;
            }
        }
    if (best_i < 0)
        return OR_DONE;
    *idx = best_i;
    if (C) *C = best_c;
    if (D) *D = best_d;
    if (Pr) *Pr = best_p;
    return OR_OK;
}

/* ---------------------------------------------------------- findBestPatch */

/* Eq. 3 / Eq. 4 over the candidate centres of `rect` (clipped to the image)
 * that satisfy R4: the (ssd, index)-lexicographic minimum of the masked SSD
 * between the target patch at (tx, ty) and the candidate's patch.  Offsets
 * with the target pixel outside the image or in the hole do not count; under
 * INTERSECT scoring neither do offsets whose candidate pixel is outside the
 * source region. */
int oracle_find_exemplar(const oracle_state *s, int32_t tx, int32_t ty, int32_t r,
                         const int32_t *rect, int64_t *idx, uint32_t *ssd,
                         int32_t *known_k)
{
    if (!in_image(s, tx, ty) || r < 1 || r > 8 || !rect)
        return OR_INVALID_ARGUMENT;
    if (rect[0] > rect[2] || rect[1] > rect[3])
        return OR_INVALID_ARGUMENT;
    int W = s->W;
    int x0 = rect[0] < 0 ? 0 : rect[0];
    int y0 = rect[1] < 0 ? 0 : rect[1];
    int x1 = rect[2] > s->W ? s->W : rect[2];
    int y1 = rect[3] > s->H ? s->H : rect[3];

    int k = 0;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx)
            k += known(s, tx + dx, ty + dy);

    int64_t best_d = -1, best_i = -1;
    for (int cy = y0; cy < y1; ++cy)
        for (int cx = x0; cx < x1; ++cx) {
            if (!valid_centre(s, cx, cy, r))
                continue;
            int64_t d = 0;
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    if (!known(s, tx + dx, ty + dy))
                        continue;
                    if (s->scoring == OR_SCORE_INTERSECT && !in_source(s, cx + dx, cy + dy))
                        continue;
                    const uint8_t *t = s->rgb + ((int64_t)(ty + dy) * W + (tx + dx)) * 3;
                    const uint8_t *q = s->rgb + ((int64_t)(cy + dy) * W + (cx + dx)) * 3;
                    for (int c = 0; c < 3; ++c) {
                        int64_t e = (int64_t)t[c] - (int64_t)q[c];
                        d += e * e;
                    }
                }
            if (best_i < 0 || d < best_d) {
                best_d = d;
                best_i = (int64_t)cy * W + cx;
            }
        }
    if (best_i < 0)
        return OR_NO_CANDIDATE;
    *idx = best_i;
    *ssd = (uint32_t)best_d;
    if (known_k)
        *known_k = k;
    return OR_OK;
}

/* ------------------------------------------------------------ fill loop */

/* One iteration: front, priority, select, search, copy (Section 3). */
int oracle_step(oracle_state *s, oracle_step_info *info)
{
    if (s->remaining == 0)
        return OR_DONE;
    int64_t p;
    double C, D, Pr;
    int st = oracle_select(s, &p, &C, &D, &Pr);
    if (st != OR_OK)
        return st;
    int W = s->W, r = s->r;
    int px = (int)(p % W), py = (int)(p / W);

    int64_t q;
    uint32_t d;
    int32_t k;
    st = oracle_find_exemplar(s, px, py, r, s->rect, &q, &d, &k);
    if (st != OR_OK)
        return st;
    int qx = (int)(q % W), qy = (int)(q / W);

    /* Copy the source patch into the target's hole pixels; they take the
     * target's confidence and leave the hole.  Under INTERSECT scoring only
     * the pixels whose source pixel is in the source region are copied, as
     * decided before the copy changes the hole. */
    uint8_t take[17 * 17];
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
            int x = px + dx, y = py + dy;
            int t = (dy + r) * s->P + (dx + r);
            take[t] = (uint8_t)(in_image(s, x, y) && s->hole[(int64_t)y * W + x] &&
                                (s->scoring != OR_SCORE_INTERSECT || in_source(s, qx + dx, qy + dy)));
        }
    int filled = 0;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
            int x = px + dx, y = py + dy;
            if (!take[(dy + r) * s->P + (dx + r)])
                continue;
            int64_t dst = (int64_t)y * W + x;
            int64_t src = (int64_t)(qy + dy) * W + (qx + dx);
            for (int c = 0; c < 3; ++c)
                s->rgb[dst * 3 + c] = s->rgb[src * 3 + c];
            s->gray[dst] = s->gray[src];
            s->conf[dst] = C;
            s->hole[dst] = 0;
            ++filled;
        }
    s->remaining -= filled;
    s->iter += 1;
    if (info) {
        memset(info, 0, sizeof(*info));
        info->target_index = p;
        info->source_index = q;
        info->ssd = d;
        info->known_k = k;
        info->n_filled = filled;
        info->priority = Pr;
        info->confidence = C;
        info->data_term = D;
        info->remaining = s->remaining;
    }
    return OR_OK;
}

int oracle_run(oracle_state *s, int64_t max_iters, int64_t *iters_done,
               oracle_step_info *log, int64_t log_cap)
{
    int64_t t = 0;
    int st = OR_OK;
    while (max_iters < 0 || t < max_iters) {
        oracle_step_info rec;
        st = oracle_step(s, &rec);
        if (st == OR_DONE) {
            st = OR_OK;
            break;
        }
        if (st != OR_OK)
            break;
        if (log && t < log_cap)
            log[t] = rec;
        ++t;
    }
    if (iters_done)
        *iters_done = t;
    if (st == OR_OK && s->remaining == 0)
        return OR_DONE;
    return st;
}

/* ------------------------------------------------------------- resume */

/* Iterative editing / resume (the paper's interactive workflow, Section 6):
 * replaces the fill state of a removal by a checkpoint of the same removal
 * -- the image, the hole still to fill, the confidence map and the number of
 * iterations done -- so that continuing from it gives what the uninterrupted
 * run gives.  The state is defined by the original hole (fixed at create),
 * so only pixels of the original hole change:
 *   - those still in the checkpoint's hole become hole again (zeroed, R1);
 *   - the others take the checkpoint's colour, its confidence and the gray
 *     value R2 gives for that colour.
 * Pixels outside the original hole keep the values given at create.  The
 * checkpoint's hole must lie inside the original hole, and its confidences
 * there must be in [0, 1]; otherwise nothing changes. */
int oracle_import_state(oracle_state *s, const uint8_t *rgb, int32_t rgb_stride,
                        int32_t channels, const uint8_t *hole, int32_t hole_stride,
                        const double *conf, int64_t iterations)
{
    if (!s || !rgb || !hole || !conf || iterations < 0 || (channels != 3 && channels != 4))
        return OR_INVALID_ARGUMENT;
    int W = s->W, H = s->H;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int64_t i = (int64_t)y * W + x;
            int h = hole[(int64_t)y * hole_stride + x] != 0;
            if (h && !s->hole0[i])
                return OR_INVALID_ARGUMENT;
            if (s->hole0[i] && !h && !(conf[i] >= 0.0 && conf[i] <= 1.0))
                return OR_INVALID_ARGUMENT;
        }
    int64_t remaining = 0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int64_t i = (int64_t)y * W + x;
            if (!s->hole0[i])
                continue;
            int h = hole[(int64_t)y * hole_stride + x] != 0;
            const uint8_t *px = rgb + (int64_t)y * rgb_stride + (int64_t)x * channels;
            for (int c = 0; c < 3; ++c)
                s->rgb[i * 3 + c] = h ? 0 : px[c];
            s->gray[i] = (uint8_t)((299 * s->rgb[i * 3] + 587 * s->rgb[i * 3 + 1] +
                                    114 * s->rgb[i * 3 + 2] + 500) / 1000);
            s->conf[i] = h ? 0.0 : conf[i];
            s->hole[i] = (uint8_t)h;
            remaining += h;
        }
    s->remaining = remaining;
    s->iter = iterations;
    return OR_OK;
}

int64_t oracle_iterations(const oracle_state *s)
{
    return s->iter;
}

/* -------------------------------------------------------------- accessors */

int oracle_read(const oracle_state *s, uint8_t *rgb, uint8_t *gray,
                uint8_t *hole, double *conf)
{
    int64_t n = (int64_t)s->W * s->H;
    if (rgb) memcpy(rgb, s->rgb, (size_t)n * 3);
    if (gray) memcpy(gray, s->gray, (size_t)n);
    if (hole) memcpy(hole, s->hole, (size_t)n);
    if (conf) memcpy(conf, s->conf, (size_t)n * sizeof(double));
    return OR_OK;
}

/* V_r as a 0/1 map (R4). */
int oracle_valid_map(const oracle_state *s, int32_t r, uint8_t *out)
{
    if (r < 1 || r > 8)
        return OR_INVALID_ARGUMENT;
    for (int y = 0; y < s->H; ++y)
        for (int x = 0; x < s->W; ++x)
            out[(int64_t)y * s->W + x] = (uint8_t)valid_centre(s, x, y, r);
    return OR_OK;
}

int oracle_get_rect(const oracle_state *s, int32_t *rect)
{
    memcpy(rect, s->rect, sizeof(s->rect));
    return OR_OK;
}

int64_t oracle_remaining(const oracle_state *s)
{
    return s->remaining;
}

int32_t oracle_step_info_size(void)
{
    return (int32_t)sizeof(oracle_step_info);
}
