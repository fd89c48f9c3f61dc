/*
 * CPU oracle for the partitioned reduction.  TEST INFRASTRUCTURE ONLY: the
 * GPU library neither includes this header nor links the oracle.
 * Definitions and citations are in oracle.c.
 */
#ifndef PCOLL_ORACLE_H
#define PCOLL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Partition plan: writes off[k], len[k] for k < nparts; returns the chunk
 * length psize, or -1 on bad arguments. */
int64_t orc_plan(int64_t count, int64_t nparts, int64_t align, int64_t *off,
                 int64_t *len);

void orc_sum_i32(int P, int64_t n, const int32_t *const *x, int32_t *y);
void orc_max_i32(int P, int64_t n, const int32_t *const *x, int32_t *y);

void orc_sum_f32_f64(int P, int64_t n, const float *const *x, double *y);
void orc_sum_f32_f64_omp(int P, int64_t n, const float *const *x, double *y);
int orc_omp_threads(void);
void orc_sum_f32_f32(int P, int64_t n, const float *const *x, int comp,
                     float *y);
void orc_max_f32(int P, int64_t n, const float *const *x, float *y);

double orc_bf16_decode(uint16_t h);
uint16_t orc_bf16_encode(double v);
void orc_sum_bf16_f64(int P, int64_t n, const uint16_t *const *x, double *y);
void orc_sum_bf16_f32(int P, int64_t n, const uint16_t *const *x, int comp,
                      uint16_t *y, float *y32);
void orc_sum_bf16_hilo(int P, int64_t n, const uint16_t *const *x, int comp,
                       uint16_t *hi, uint16_t *lo);
void orc_max_bf16(int P, int64_t n, const uint16_t *const *x, uint16_t *y);

double orc_e4m3_decode(uint8_t q);
uint8_t orc_e4m3_encode(double v);
void orc_e4m3_pack(int64_t n, const float *x, uint8_t *q, float *s);
void orc_sum_e4m3_f64(int P, int64_t n, const uint8_t *const *q,
                      const float *const *s, double *y);
void orc_sum_e4m3_f32(int P, int64_t n, const uint8_t *const *q,
                      const float *const *s, int comp, uint8_t *yq,
                      float *ys, float *y32);
double orc_e5m2_decode(uint8_t q);
uint8_t orc_e5m2_encode(double v);
void orc_e5m2_pack(int64_t n, const float *x, uint8_t *q, float *s);
void orc_sum_e5m2_f64(int P, int64_t n, const uint8_t *const *q,
                      const float *const *s, double *y);
void orc_sum_e5m2_f32(int P, int64_t n, const uint8_t *const *q,
                      const float *const *s, int comp, uint8_t *yq,
                      float *ys, float *y32);

double orc_e8m0_decode(uint8_t b);
int orc_mx_exponent(float amax);
void orc_mx_pack(int64_t n, const float *x, uint8_t *q, uint8_t *sb);
void orc_sum_mx_f64(int P, int64_t n, const uint8_t *const *q,
                    const uint8_t *const *sb, double *y);
void orc_sum_mx_f32(int P, int64_t n, const uint8_t *const *q,
                    const uint8_t *const *sb, int comp, uint8_t *yq,
                    uint8_t *ysb, float *y32);

#ifdef __cplusplus
}
#endif

#endif
