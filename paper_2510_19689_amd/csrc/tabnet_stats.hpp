// Library-internal entry points of the mask-statistics kernels (tabnet_stats.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tabnet {
// Workspace bytes for the statistics of up to `rows` rows of D columns.
size_t mask_stats_workspace_bytes(int64_t rows, int D);
// Column statistics of masks[rows][D] (FP32, row-major) on `stream`.  With rows_dev set
// the live row count is read from device memory (at most `rows`), so a captured graph
// can be replayed for any count.  Each output pointer may be null: mean[D], var[D]
// (population variance), q_out[D] (sum of squared deviations), n_out[1] (row count).
hipError_t enqueue_mask_stats(const float* masks, int64_t rows, const int64_t* rows_dev, int D, double* mean,
                              double* var, double* q_out, double* n_out, void* workspace, hipStream_t stream);
}  // namespace tabnet
