/*
 * scpl_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of Seam Carving with
 * Parental Labeling (SCPL) video retargeting, written from the paper
 * "Fast Video Retargeting Based on Seam Carving with Parental Labeling"
 * (C. Zhu, arXiv 1903.03180).  It exists only so that tests, the smoke check
 * and the benchmark's CPU-baseline leg can check the HIP library against it.
 * The HIP library never links, loads or calls this file, and this file
 * includes nothing from the HIP library.
 *
 * Everything here is exact integer arithmetic.  Frames are physically carved
 * (copied and compacted) after every iteration, and every energy map is
 * recomputed in full from the carved frames, because that is the most direct
 * reading of the method.
 *
 * Readings of points the paper leaves open (each is also pinned by a test):
 *  - luma: Y = (77 R + 150 G + 29 B + 128) >> 8 (paper silent on colour).
 *  - gradient: 3x3 Sobel, L1 magnitude |Gx| + |Gy|, borders replicated
 *    (Sec. 3.3 names Sobel; border handling is not stated).
 *  - motion energy: the 0.6 / 0.4 weights of Sec. 3.3 are applied exactly
 *    after bringing the difference (0..255) to the gradient range (0..1530)
 *    by the factor 6:  e = 2 G + 18 |Y_t - Y_{t-1}|  (a common positive scale
 *    of 0.4 G + 0.6 * 6 D).  The first frame of the clip has no difference
 *    term.  After carving, the predecessor frame is carved with the same
 *    seams; a buffer's first frame uses a "ghost" copy of the original frame
 *    just before the buffer, carved along with the buffer.
 *  - cumulative energy, eq. (4): neighbours outside the image are ignored and
 *    ties go to the leftmost (smallest column) predecessor.
 *  - seams per iteration: eq. (6) takes every parent's least child; here the
 *    per-parent minima are ranked by (cumulative energy, column) and the first
 *    k_iter = min(k, number of parents, width - target) are removed.
 *  - ASDE, eqs. (7)-(8): population standard deviation over the T frames of
 *    the candidate buffer, per pixel floor(sqrt(T*S2 - S1^2)) = floor(T*Std),
 *    summed over all pixels.
 *  - threshold, eq. (9): phi(n) = alpha * maxval * sqrt(n - 1) / n, with n the
 *    buffer size including the candidate frame and maxval the largest value
 *    the energy function can take (1530 gradient, 7650 motion).  The
 *    candidate is rejected (buffer fixed, candidate starts the next buffer)
 *    when ASDE > phi(n), compared exactly in 128-bit integers.
 *  - uniform energy (Sec. 3.2): floor of the mean of the buffer's energy maps.
 *  - seam memorisation (named as future work in Sec. 5, not defined there):
 *    with a period m >= 2, buffer b is carved only when b mod m == 0; every
 *    other buffer removes from each of its frames the very pixels that buffer
 *    b - (b mod m) removed (same mask), keeping the rest of each row in
 *    order.
 */
#include "scpl_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Luma of interleaved 8-bit RGB (reading of the paper's unstated colour step). */
void oracle_luma(const uint8_t *rgb, int64_t npx, uint8_t *y)
{
    for (int64_t p = 0; p < npx; ++p) {
        int r = rgb[3 * p], g = rgb[3 * p + 1], b = rgb[3 * p + 2];
        y[p] = (uint8_t)((77 * r + 150 * g + 29 * b + 128) >> 8);
    }
}

/* Sobel L1 gradient magnitude at (i, j) of an H x W image, replicated borders
 * (Sec. 3.3, "Sobel gradient energy"). */
static int sobel_l1(const uint8_t *y, int H, int W, int i, int j)
{
    int im = clampi(i - 1, 0, H - 1), ip = clampi(i + 1, 0, H - 1);
    int jm = clampi(j - 1, 0, W - 1), jp = clampi(j + 1, 0, W - 1);
#define PX(r, c) ((int)y[(int64_t)(r) * W + (c)])
    int gx = (PX(im, jp) + 2 * PX(i, jp) + PX(ip, jp)) - (PX(im, jm) + 2 * PX(i, jm) + PX(ip, jm));
    int gy = (PX(ip, jm) + 2 * PX(ip, j) + PX(ip, jp)) - (PX(im, jm) + 2 * PX(im, j) + PX(im, jp));
#undef PX
    return abs(gx) + abs(gy);
}

/* Energy map of one frame (Sec. 3.3).  GRADIENT: e = G.  MOTION:
 * e = 2 G + 18 |y - yprev|, difference term 0 when yprev is NULL. */
void oracle_energy(const uint8_t *y, const uint8_t *yprev, int H, int W, int mode, int32_t *e)
{
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            int64_t p = (int64_t)i * W + j;
            int g = sobel_l1(y, H, W, i, j);
            if (mode == ORACLE_ENERGY_GRADIENT) {
                e[p] = g;
            } else {
                int d = yprev ? abs((int)y[p] - (int)yprev[p]) : 0;
                e[p] = 2 * g + 18 * d;
            }
        }
}

int32_t oracle_energy_max(int mode) { return mode == ORACLE_ENERGY_GRADIENT ? 1530 : 7650; }

/* Cumulative energy, eq. (4), with the indicator (back-pointer) array and the
 * parent label of every pixel (Sec. 3.1: the row-0 pixel a pixel traces back
 * to).  Ties go to the leftmost predecessor; out-of-range neighbours are
 * skipped.  ce, label and dir are H x W row-major. */
void oracle_dp(const int32_t *u, int H, int W, int32_t *ce, int32_t *label, int8_t *dir)
{
    for (int j = 0; j < W; ++j) {
        ce[j] = u[j];
        label[j] = j;
        dir[j] = 0;
    }
    for (int i = 1; i < H; ++i) {
        const int32_t *cu = ce + (int64_t)(i - 1) * W;
        const int32_t *lu = label + (int64_t)(i - 1) * W;
        for (int j = 0; j < W; ++j) {
            int best = -1;
            for (int p = j - 1; p <= j + 1; ++p) {
                if (p < 0 || p >= W) continue;
                if (best < 0 || cu[p] < cu[best]) best = p; /* strict: first minimum wins */
            }
            int64_t q = (int64_t)i * W + j;
            ce[q] = u[q] + cu[best];
            label[q] = lu[best];
            dir[q] = (int8_t)(best - j);
        }
    }
}

/* Per-parent least child, eq. (6), then the k_iter = min(k, P_eff, limit)
 * least of those by (cumulative energy, column).  Inputs are the last row of
 * the DP.  children[] receives k_iter columns in increasing column order.
 * Returns k_iter; *p_eff receives the number of distinct parents. */
typedef struct {
    int32_t ce, col;
} cand_t;

static int cand_cmp(const void *a, const void *b)
{
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    if (x->ce != y->ce) return x->ce < y->ce ? -1 : 1;
    return x->col < y->col ? -1 : (x->col > y->col);
}

static int int_cmp(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return x < y ? -1 : (x > y);
}

int oracle_select(const int32_t *ce_last, const int32_t *label_last, int W, int k, int limit,
                  int32_t *children, int32_t *p_eff)
{
    int32_t *best = (int32_t *)malloc(sizeof(int32_t) * (size_t)W);
    cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * (size_t)W);
    for (int j = 0; j < W; ++j) best[j] = -1;
    for (int j = 0; j < W; ++j) {
        int l = label_last[j];
        if (best[l] < 0 || ce_last[j] < ce_last[best[l]]) best[l] = j; /* leftmost least child */
    }
    int np = 0;
    for (int l = 0; l < W; ++l)
        if (best[l] >= 0) {
            cand[np].ce = ce_last[best[l]];
            cand[np].col = best[l];
            ++np;
        }
    qsort(cand, (size_t)np, sizeof(cand_t), cand_cmp);
    int kk = k;
    if (kk > np) kk = np;
    if (kk > limit) kk = limit;
    if (kk < 0) kk = 0;
    for (int s = 0; s < kk; ++s) children[s] = cand[s].col;
    qsort(children, (size_t)kk, sizeof(int32_t), int_cmp);
    if (p_eff) *p_eff = np;
    free(best);
    free(cand);
    return kk;
}

/* Trace each selected child back through the indicator array (Sec. 3.1).
 * seams is kk x H: seams[s*H + i] is the column of seam s in row i. */
void oracle_backtrack(const int8_t *dir, int H, int W, const int32_t *children, int kk, int32_t *seams)
{
    for (int s = 0; s < kk; ++s) {
        int x = children[s];
        seams[(int64_t)s * H + (H - 1)] = x;
        for (int i = H - 1; i >= 1; --i) {
            x += dir[(int64_t)i * W + x];
            seams[(int64_t)s * H + (i - 1)] = x;
        }
    }
}

/* floor(sqrt(q)) for 64-bit q, corrected in exact integer arithmetic. */
uint64_t oracle_isqrt(uint64_t q)
{
    uint64_t r = (uint64_t)sqrt((double)q);
    while ((u128)r * r > q) --r;
    while ((u128)(r + 1) * (r + 1) <= q) ++r;
    return r;
}

/* S = sum over pixels of floor(sqrt(n*S2 - S1^2)): n times the sum of the
 * per-pixel population standard deviations of eq. (8), floored per pixel. */
int64_t oracle_asde_sum(const uint64_t *s1, const uint64_t *s2, int64_t npx, int n)
{
    int64_t S = 0;
    for (int64_t p = 0; p < npx; ++p) {
        uint64_t q = (uint64_t)n * s2[p] - s1[p] * s1[p];
        S += (int64_t)oracle_isqrt(q);
    }
    return S;
}

/* Buffer-fix test, eqs. (7) and (9): ASDE = S / (n H W) > phi(n) =
 * alpha * maxval * sqrt(n - 1) / n, i.e. S * aden > anum * maxval * H W *
 * sqrt(n - 1), compared squared in 128-bit integers. */
int oracle_reject(int64_t S, int n, int64_t npx, int32_t emax, int32_t anum, int32_t aden)
{
    if (n <= 1) return 0;
    u128 lhs = (u128)(uint64_t)S * (uint64_t)aden;
    lhs = lhs * lhs;
    u128 b = (u128)(uint64_t)anum * (uint64_t)emax * (uint64_t)npx;
    u128 rhs = b * b * (u128)(uint64_t)(n - 1);
    return lhs > rhs;
}

/* Dynamic spatiotemporal buffer (Sec. 3.2): frames are appended one at a
 * time; the ASDE of the grown buffer is tested against phi(n); on rejection
 * the buffer is fixed without the new frame, which starts the next buffer.
 * Energies are those of the original frames.  buffer_id[t] receives the
 * buffer index of frame t; s_trace (nullable) receives S of each tested
 * candidate (-1 where no test was made).  Returns the number of buffers. */
int oracle_segment(const uint8_t *Y, int N, int H, int W, int mode, int use_buffer, int32_t anum,
                   int32_t aden, int max_buffer, int32_t *buffer_id, int64_t *s_trace)
{
    int64_t npx = (int64_t)H * W;
    int32_t emax = oracle_energy_max(mode);
    if (!use_buffer) {
        for (int t = 0; t < N; ++t) {
            buffer_id[t] = t;
            if (s_trace) s_trace[t] = -1;
        }
        return N;
    }
    uint64_t *s1 = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)npx);
    uint64_t *s2 = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)npx);
    uint64_t *c1 = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)npx);
    uint64_t *c2 = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)npx);
    int32_t *e = (int32_t *)malloc(sizeof(int32_t) * (size_t)npx);

    oracle_energy(Y, NULL, H, W, mode, e);
    for (int64_t p = 0; p < npx; ++p) {
        s1[p] = (uint64_t)e[p];
        s2[p] = (uint64_t)e[p] * (uint64_t)e[p];
    }
    int n = 1, nb = 0;
    buffer_id[0] = 0;
    if (s_trace) s_trace[0] = -1;
    for (int t = 1; t < N; ++t) {
        oracle_energy(Y + (int64_t)t * npx, Y + (int64_t)(t - 1) * npx, H, W, mode, e);
        int fix;
        if (max_buffer > 0 && n >= max_buffer) {
            fix = 1;
            if (s_trace) s_trace[t] = -1;
        } else {
            for (int64_t p = 0; p < npx; ++p) {
                c1[p] = s1[p] + (uint64_t)e[p];
                c2[p] = s2[p] + (uint64_t)e[p] * (uint64_t)e[p];
            }
            int64_t S = oracle_asde_sum(c1, c2, npx, n + 1);
            if (s_trace) s_trace[t] = S;
            fix = oracle_reject(S, n + 1, npx, emax, anum, aden);
            if (!fix) {
                memcpy(s1, c1, sizeof(uint64_t) * (size_t)npx);
                memcpy(s2, c2, sizeof(uint64_t) * (size_t)npx);
                ++n;
            }
        }
        if (fix) {
            ++nb;
            for (int64_t p = 0; p < npx; ++p) {
                s1[p] = (uint64_t)e[p];
                s2[p] = (uint64_t)e[p] * (uint64_t)e[p];
            }
            n = 1;
        }
        buffer_id[t] = nb;
    }
    free(s1);
    free(s2);
    free(c1);
    free(c2);
    free(e);
    return nb + 1;
}

/* Remove kk seams from an H x W x C image in place, giving H x (W-kk) x C.
 * seams[s*H + i] are the removed columns of row i; they must be distinct. */
static int remove_seams(uint8_t *img, int H, int W, int C, const int32_t *seams, int kk, uint8_t *mark)
{
    int Wn = W - kk;
    for (int i = 0; i < H; ++i) {
        memset(mark, 0, (size_t)W);
        for (int s = 0; s < kk; ++s) {
            int x = seams[(int64_t)s * H + i];
            if (x < 0 || x >= W || mark[x]) return -1;
            mark[x] = 1;
        }
        const uint8_t *src = img + (int64_t)i * W * C;
        uint8_t *dst = img + (int64_t)i * Wn * C; /* dst never overtakes src */
        int o = 0;
        for (int j = 0; j < W; ++j) {
            if (mark[j]) continue;
            for (int c = 0; c < C; ++c) dst[(int64_t)o * C + c] = src[(int64_t)j * C + c];
            ++o;
        }
    }
    return 0;
}

static void remove_seams_i32(int32_t *img, int H, int W, const int32_t *seams, int kk, uint8_t *mark)
{
    int Wn = W - kk;
    for (int i = 0; i < H; ++i) {
        memset(mark, 0, (size_t)W);
        for (int s = 0; s < kk; ++s) mark[seams[(int64_t)s * H + i]] = 1;
        const int32_t *src = img + (int64_t)i * W;
        int32_t *dst = img + (int64_t)i * Wn;
        int o = 0;
        for (int j = 0; j < W; ++j)
            if (!mark[j]) dst[o++] = src[j];
    }
}

/* Whole retarget (Secs. 3.1-3.3): segment the clip into buffers, then for
 * each buffer repeatedly compute the uniform energy of the carved frames,
 * run the labelled DP, pick seams and remove them from every frame of the
 * buffer, until the target width is reached.  frames: N x H x W x C u8.
 * out: N x H x Wt x C.  masks (nullable): N x H x W u16, 0 = kept, r+1 =
 * removed in iteration r of the frame's buffer.  buffer_id (nullable): N.
 * memo_period: 0 or 1 carves every buffer; m >= 2 carves buffer b only when
 * b mod m == 0 and gives every other buffer the removal of buffer
 * b - (b mod m) (seam memorisation, see the readings above).
 * log (nullable): per iteration of every carved buffer, in order, four int32:
 * (buffer, W_r, P_eff, k_iter); log_cap is its capacity in records and the
 * return value is the number of records (or a negative error). */
int64_t oracle_retarget(const uint8_t *frames, int N, int H, int W, int C, int Wt, int k, int mode,
                        int use_buffer, int32_t anum, int32_t aden, int max_buffer, int memo_period,
                        uint8_t *out, uint16_t *masks, int32_t *buffer_id, int32_t *log, int64_t log_cap)
{
    if (N < 1 || H < 1 || W < 1 || (C != 1 && C != 3) || Wt < 1 || Wt > W || k < 1 || memo_period < 0)
        return -1;
    int64_t npx = (int64_t)H * W;
    uint8_t *Y = (uint8_t *)malloc((size_t)(N * npx));
    if (C == 3)
        for (int t = 0; t < N; ++t) oracle_luma(frames + (int64_t)t * npx * 3, npx, Y + (int64_t)t * npx);
    else
        memcpy(Y, frames, (size_t)(N * npx));

    int32_t *bid = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int nbuf = oracle_segment(Y, N, H, W, mode, use_buffer, anum, aden, max_buffer, bid, NULL);
    if (buffer_id) memcpy(buffer_id, bid, sizeof(int32_t) * (size_t)N);

    int64_t nlog = 0;
    int t0 = 0;
    /* mask of the last carved buffer, for memorised buffers */
    uint16_t *memo_mask = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)npx);
    for (int b = 0; b < nbuf; ++b) {
        int T = 0;
        while (t0 + T < N && bid[t0 + T] == b) ++T;
        if (memo_period >= 2 && b % memo_period != 0) {
            for (int f = t0; f < t0 + T; ++f) {
                for (int i = 0; i < H; ++i) {
                    const uint8_t *src = frames + ((int64_t)f * H + i) * W * C;
                    uint8_t *dst = out + ((int64_t)f * H + i) * Wt * C;
                    int o = 0;
                    for (int j = 0; j < W; ++j) {
                        if (memo_mask[(int64_t)i * W + j] != 0) continue;
                        if (o >= Wt) return -3;
                        for (int c = 0; c < C; ++c) dst[o * C + c] = src[j * C + c];
                        ++o;
                    }
                    if (o != Wt) return -3;
                }
                if (masks) memcpy(masks + (int64_t)f * npx, memo_mask, sizeof(uint16_t) * (size_t)npx);
            }
            t0 += T;
            continue;
        }
        int ghost = (mode == ORACLE_ENERGY_MOTION && t0 > 0);
        int nwork = T + ghost; /* working luma frames: [ghost], t0 .. t0+T-1 */
        uint8_t *wy = (uint8_t *)malloc((size_t)(nwork * npx));
        uint8_t *wc = (uint8_t *)malloc((size_t)(T * npx * C));
        int32_t *colmap = (int32_t *)malloc(sizeof(int32_t) * (size_t)npx);
        for (int f = 0; f < nwork; ++f)
            memcpy(wy + f * npx, Y + (int64_t)(t0 - ghost + f) * npx, (size_t)npx);
        memcpy(wc, frames + (int64_t)t0 * npx * C, (size_t)(T * npx * C));
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j) colmap[(int64_t)i * W + j] = j;

        int32_t *u = (int32_t *)malloc(sizeof(int32_t) * (size_t)npx);
        int64_t *acc = (int64_t *)malloc(sizeof(int64_t) * (size_t)npx);
        int32_t *e = (int32_t *)malloc(sizeof(int32_t) * (size_t)npx);
        int32_t *ce = (int32_t *)malloc(sizeof(int32_t) * (size_t)npx);
        int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)npx);
        int8_t *dir = (int8_t *)malloc((size_t)npx);
        int32_t *children = (int32_t *)malloc(sizeof(int32_t) * (size_t)W);
        int32_t *seams = (int32_t *)malloc(sizeof(int32_t) * (size_t)W * (size_t)H);
        uint8_t *mark = (uint8_t *)malloc((size_t)W);
        uint16_t *bmask = (uint16_t *)calloc((size_t)npx, sizeof(uint16_t));

        int Wr = W, r = 0;
        while (Wr > Wt) {
            int64_t cpx = (int64_t)H * Wr;
            /* uniform energy: floor of the mean of the buffer's energy maps */
            memset(acc, 0, sizeof(int64_t) * (size_t)cpx);
            for (int f = ghost; f < nwork; ++f) {
                const uint8_t *prev = (f > 0) ? wy + (f - 1) * cpx : NULL;
                oracle_energy(wy + f * cpx, prev, H, Wr, mode, e);
                for (int64_t p = 0; p < cpx; ++p) acc[p] += e[p];
            }
            for (int64_t p = 0; p < cpx; ++p) u[p] = (int32_t)(acc[p] / T);

            oracle_dp(u, H, Wr, ce, lab, dir);
            int32_t peff = 0;
            int kk = oracle_select(ce + (int64_t)(H - 1) * Wr, lab + (int64_t)(H - 1) * Wr, Wr, k, Wr - Wt,
                                   children, &peff);
            oracle_backtrack(dir, H, Wr, children, kk, seams);
            if (log && nlog < log_cap) {
                log[4 * nlog + 0] = b;
                log[4 * nlog + 1] = Wr;
                log[4 * nlog + 2] = peff;
                log[4 * nlog + 3] = kk;
            }
            ++nlog;
            /* record the removal in original coordinates, then carve */
            for (int s = 0; s < kk; ++s)
                for (int i = 0; i < H; ++i) {
                    int x = seams[(int64_t)s * H + i];
                    bmask[(int64_t)i * W + colmap[(int64_t)i * Wr + x]] = (uint16_t)(r + 1);
                }
            for (int f = 0; f < nwork; ++f)
                if (remove_seams(wy + f * cpx, H, Wr, 1, seams, kk, mark)) return -2;
            /* compact the working frames to the new stride */
            for (int f = 1; f < nwork; ++f)
                memmove(wy + f * (int64_t)H * (Wr - kk), wy + f * cpx, (size_t)((int64_t)H * (Wr - kk)));
            for (int f = 0; f < T; ++f)
                if (remove_seams(wc + f * cpx * C, H, Wr, C, seams, kk, mark)) return -2;
            for (int f = 1; f < T; ++f)
                memmove(wc + f * (int64_t)H * (Wr - kk) * C, wc + f * cpx * C, (size_t)((int64_t)H * (Wr - kk) * C));
            remove_seams_i32(colmap, H, Wr, seams, kk, mark);
            Wr -= kk;
            ++r;
        }
        for (int f = 0; f < T; ++f) {
            memcpy(out + (int64_t)(t0 + f) * H * Wt * C, wc + (int64_t)f * H * Wt * C, (size_t)((int64_t)H * Wt * C));
            if (masks) memcpy(masks + (int64_t)(t0 + f) * npx, bmask, sizeof(uint16_t) * (size_t)npx);
        }
        memcpy(memo_mask, bmask, sizeof(uint16_t) * (size_t)npx);
        free(wy); free(wc); free(colmap); free(u); free(acc); free(e); free(ce); free(lab); free(dir);
        free(children); free(seams); free(mark); free(bmask);
        t0 += T;
    }
    free(Y);
    free(bid);
    free(memo_mask);
    return nlog;
}
