/*
 * scpl_oracle.h -- TEST INFRASTRUCTURE ONLY: declarations of the plain CPU
 * SCPL oracle (scpl_oracle.c).  Used by tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the HIP library.
 */
#ifndef SCPL_ORACLE_H
#define SCPL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_ENERGY_GRADIENT = 0, ORACLE_ENERGY_MOTION = 1 };

void oracle_luma(const uint8_t *rgb, int64_t npx, uint8_t *y);
void oracle_energy(const uint8_t *y, const uint8_t *yprev, int H, int W, int mode, int32_t *e);
int32_t oracle_energy_max(int mode);
void oracle_dp(const int32_t *u, int H, int W, int32_t *ce, int32_t *label, int8_t *dir);
int oracle_select(const int32_t *ce_last, const int32_t *label_last, int W, int k, int limit,
                  int32_t *children, int32_t *p_eff);
void oracle_backtrack(const int8_t *dir, int H, int W, const int32_t *children, int kk, int32_t *seams);
uint64_t oracle_isqrt(uint64_t q);
int64_t oracle_asde_sum(const uint64_t *s1, const uint64_t *s2, int64_t npx, int n);
int oracle_reject(int64_t S, int n, int64_t npx, int32_t emax, int32_t anum, int32_t aden);
int oracle_segment(const uint8_t *Y, int N, int H, int W, int mode, int use_buffer, int32_t anum,
                   int32_t aden, int max_buffer, int32_t *buffer_id, int64_t *s_trace);
int64_t oracle_retarget(const uint8_t *frames, int N, int H, int W, int C, int Wt, int k, int mode,
                        int use_buffer, int32_t anum, int32_t aden, int max_buffer, int memo_period,
                        uint8_t *out, uint16_t *masks, int32_t *buffer_id, int32_t *log, int64_t log_cap);

#ifdef __cplusplus
}
#endif
#endif
