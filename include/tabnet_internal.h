/*
 * tabnet_internal.h -- host-only hooks for tests (no GPU needed).
 *
 * They expose the load-time arithmetic of tabnet_load (batch-norm folding, rounding,
 * header validation) and a serving runtime on a CPU stand-in device, so that they can be
 * checked on a machine without a GPU.  None of them touches the HIP runtime.  They are
 * exported by the test library libtabnet_test.so (the product library's code plus these
 * hooks), not by libtabnet.so.
 */
#ifndef TABNET_INTERNAL_H
#define TABNET_INTERNAL_H

#include <stddef.h>
#include <stdint.h>

#include "tabnet.h"

#ifdef __cplusplus
extern "C" {
#endif

/* bfloat16 bits of x, round to nearest even. */
uint16_t tabnet_hook_bf16_bits(double x);
/* float8 E4M3FN bits of x, round to nearest even, saturating at +-448. */
uint8_t tabnet_hook_e4m3_bits(double x);

/* FP4 E2M1 bits (sign in bit 3) of x, round to nearest even, saturating at +-6. */
uint8_t tabnet_hook_e2m1_bits(double x);
/* FP6 E2M3 bits (sign in bit 5) of x, round to nearest even, saturating at +-7.5. */
uint8_t tabnet_hook_e2m3_bits(double x);
/* float8 E5M2 bits of x, round to nearest even, saturating at +-57344. */
uint8_t tabnet_hook_e5m2_bits(double x);
/* FP6 E3M2 bits (sign in bit 5) of x, round to nearest even, saturating at +-28. */
uint8_t tabnet_hook_e3m2_bits(double x);
/* OCP MX shared exponent of a block with largest magnitude amax for an element format
 * with largest exponent emax: floor(log2 amax) - emax, clamped to [-126, 127]; 0 for 0. */
int tabnet_hook_mx_exponent(double amax, int emax);

/* The load-time INT8 coding of a weight matrix W [rows][cols] (row-major, caller-owned):
 * per row, scale = max_k |W_k| / 127 (1 for a zero row) into scales[row], and W_k
 * replaced in place by round(W_k / scale) (ties to even), as TABNET_INT8 packs it. */
void tabnet_hook_int8_rows(double* W, int rows, int cols, double* scales);

/* Parse and validate a TNW1 image held in memory (buffer of `len` bytes, caller-owned).
 * On success fills *cfg.  Returns the status tabnet_load would return for that file. */
tabnet_status tabnet_hook_parse(const void* buf, size_t len, tabnet_config* cfg);

/* Fold FC layer `layer` of the model in `buf` (index into the concatenation of shared
 * layers, step-specific layers pass by pass, then attentive layers) into W' and b'.
 * Wf receives rows x cols doubles, bf receives rows doubles; *rows / *cols are set.
 * Pass NULL Wf/bf to query the sizes. */
tabnet_status tabnet_hook_fold(const void* buf, size_t len, int layer, double* Wf, double* bf,
                               int* rows, int* cols);

/* Packed sizes of the model for a precision, in the chunk layout of the compiled kernel
 * for its shape: bytes of the packed GEMM units (fragments and shifts) and the number of
 * weight-stream chunks the kernel consumes per forward.  TABNET_E_UNSUPPORTED if no
 * kernel covers the shape. */
tabnet_status tabnet_hook_packed_sizes(const void* buf, size_t len, int precision,
                                       int64_t* wts_bytes, int64_t* n_chunks);

/* A server whose device side is a CPU stand-in (no GPU needed), for testing the
 * scheduling: admission, ordering, splitting across launches, scattering, cancellation
 * and failures.  Its "model" writes logits[r][o] = X[r][o % D] + o, masks_agg = 2 X and
 * masks_step[s] = X + s; each launch additionally sleeps delay_us microseconds.  Launch
 * number fail_launch (counted from 0 over the server's launches) fails to launch and
 * launch number fail_wait fails when its completion is waited on; -1 disables either.
 * Stop it with tabnet_serve_stop. */
/* The serving path's host copy (the scatter and gather of launches): n bytes from src to
 * dst; from 4 KiB up with non-temporal AVX2 stores where the CPU has them. */
void tabnet_hook_serve_copy(void* dst, const void* src, size_t n);

tabnet_status tabnet_hook_serve_start_fake(const tabnet_config* cfgs, int n_models,
                                           const tabnet_serve_opts* opts, int delay_us, int fail_launch,
                                           int fail_wait, tabnet_server** out);

#ifdef __cplusplus
}
#endif
#endif
