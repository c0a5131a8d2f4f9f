/*
 * Drives the CPU oracle (oracle/scpl_oracle.c) through every entry point on
 * seeded pseudo-random inputs, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  The inputs include
 * the degenerate shapes (one row, one column, one frame, W = Wt), tie-heavy
 * energies, RGB and luma clips, every energy mode, buffer options, seam
 * memorisation and k >= W.  Exit status 0 when every call returned; the
 * sanitizers abort on the first error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/scpl_oracle.h"

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;

static uint32_t next_u32(void)
{
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(rng_state >> 33);
}

/* a clip of smooth ramps plus a moving bright block and noise, so that the
 * energy has structure, ties and motion */
static void fill_clip(uint8_t *f, int N, int H, int W, int C, int coarse)
{
    for (int t = 0; t < N; ++t)
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j)
                for (int c = 0; c < C; ++c) {
                    int v = (i * 3 + j * 2 + c * 40) & 255;
                    if (coarse) v = (v / 64) * 64;
                    if (i >= (t * 2) % (H + 1) && i < (t * 2) % (H + 1) + H / 3 + 1 && j >= t % (W + 1) &&
                        j < t % (W + 1) + W / 4 + 1)
                        v = 230;
                    if (t >= N / 2 && N > 3) v = 255 - v;
                    v += (int)(next_u32() % 5) - 2;
                    f[(((size_t)t * H + i) * W + j) * C + c] = (uint8_t)(v < 0 ? 0 : v > 255 ? 255 : v);
                }
}

static int run_case(int N, int H, int W, int C, int Wt, int k, int mode, int use_buffer, int anum, int aden,
                    int max_buffer, int memo, int coarse)
{
    const size_t npx = (size_t)H * W;
    uint8_t *f = malloc((size_t)N * npx * C);
    uint8_t *out = malloc((size_t)N * H * Wt * C);
    uint16_t *masks = malloc((size_t)N * npx * sizeof(uint16_t));
    int32_t *bid = malloc((size_t)N * sizeof(int32_t));
    const int64_t cap = 4096;
    int32_t *log = malloc((size_t)cap * 4 * sizeof(int32_t));
    fill_clip(f, N, H, W, C, coarse);
    const int64_t n = oracle_retarget(f, N, H, W, C, Wt, k, mode, use_buffer, anum, aden, max_buffer, memo, out,
                                      masks, bid, log, cap);
    /* and without masks */
    const int64_t n2 = oracle_retarget(f, N, H, W, C, Wt, k, mode, use_buffer, anum, aden, max_buffer, memo, out,
                                       NULL, bid, log, cap);
    free(f);
    free(out);
    free(masks);
    free(bid);
    free(log);
    if (n < 0 || n2 != n) {
        fprintf(stderr, "case N=%d H=%d W=%d C=%d Wt=%d k=%d: %lld / %lld\n", N, H, W, C, Wt, k, (long long)n,
                (long long)n2);
        return 1;
    }
    return 0;
}

static int run_stages(int H, int W)
{
    const size_t npx = (size_t)H * W;
    uint8_t *y = malloc(npx), *yp = malloc(npx), *rgb = malloc(npx * 3);
    int32_t *e = malloc(npx * 4), *ce = malloc(npx * 4), *lab = malloc(npx * 4), *ch = malloc((size_t)W * 4);
    int32_t *seams = malloc(npx * 4), peff = 0;
    int8_t *dir = malloc(npx);
    uint64_t *s1 = malloc(npx * 8), *s2 = malloc(npx * 8);
    for (size_t p = 0; p < npx; ++p) {
        y[p] = (uint8_t)(next_u32() % 4);
        yp[p] = (uint8_t)(next_u32() & 255);
        rgb[3 * p] = rgb[3 * p + 1] = rgb[3 * p + 2] = y[p];
        s1[p] = next_u32() % 7651;
        s2[p] = s1[p] * s1[p];
    }
    oracle_luma(rgb, (int64_t)npx, y);
    for (int mode = 0; mode < 2; ++mode) {
        oracle_energy(y, mode ? yp : NULL, H, W, mode, e);
        oracle_dp(e, H, W, ce, lab, dir);
        for (int k = 1; k <= W + 1; k += (W > 8 ? W / 4 : 1)) {
            const int kk = oracle_select(ce + npx - W, lab + npx - W, W, k, W, ch, &peff);
            oracle_backtrack(dir, H, W, ch, kk, seams);
        }
    }
    int rc = 0;
    if (oracle_isqrt(0) != 0 || oracle_isqrt(UINT64_MAX) != 4294967295ull) rc = 1;
    const int64_t S = oracle_asde_sum(s1, s2, (int64_t)npx, 1);
    (void)oracle_reject(S, 2, (int64_t)npx, oracle_energy_max(1), 1, 5);
    free(y); free(yp); free(rgb); free(e); free(ce); free(lab); free(ch); free(seams); free(dir); free(s1); free(s2);
    return rc;
}

int main(void)
{
    int bad = 0;
    const int shapes[][2] = {{1, 1}, {1, 9}, {9, 1}, {2, 2}, {7, 8}, {31, 45}, {64, 33}};
    for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s) bad |= run_stages(shapes[s][0], shapes[s][1]);
    bad |= run_case(1, 1, 1, 1, 1, 1, 1, 1, 1, 5, 0, 0, 0);
    bad |= run_case(3, 1, 9, 3, 4, 2, 1, 1, 1, 5, 0, 0, 0);
    bad |= run_case(2, 9, 1, 1, 1, 3, 1, 1, 1, 5, 0, 0, 0);
    bad |= run_case(6, 20, 40, 3, 30, 4, 1, 1, 1, 5, 0, 0, 1);
    bad |= run_case(8, 24, 50, 1, 30, 50, 1, 1, 1, 5, 0, 0, 0);       /* k >= W: every parent's least child */
    bad |= run_case(10, 16, 30, 1, 20, 3, 0, 0, 1, 5, 0, 0, 1);       /* gradient, no buffer */
    bad |= run_case(12, 18, 36, 3, 25, 5, 1, 1, 3, 20, 4, 0, 0);      /* max_buffer */
    bad |= run_case(16, 20, 40, 1, 28, 4, 1, 1, 1, 1, 0, 2, 0);       /* memorisation, period 2 */
    bad |= run_case(5, 30, 30, 1, 30, 4, 1, 1, 1, 5, 0, 0, 0);        /* W == Wt */
    bad |= run_case(4, 12, 64, 3, 1, 1000, 1, 1, 0, 1, 0, 0, 1);      /* down to one column, alpha 0 */
    if (bad) return 1;
    printf("oracle sanitized run: ok\n");
    return 0;
}
