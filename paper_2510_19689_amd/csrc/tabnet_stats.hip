// Per-feature statistics of mask rows on the GPU: mean and population variance of every
// column of an [B, D] FP32 matrix (the aggregate mask, or one step's mask).
//
// The paper assesses the stability of TabNet's explanations under load by the variance of
// each feature's mask value over many served rows, next to each feature's importance
// (Sec. IV-C, Sec. V-C, Table IV).  These kernels compute both for any set of rows, as
// shifted sums: with K_d = m[0][d] (the column's first value, which every workgroup can
// read), S1_d = sum_r (m[r][d] - K_d) and S2_d = sum_r (m[r][d] - K_d)^2 in FP64 give
//     mean_d = K_d + S1_d / B,   M2_d = S2_d - S1_d^2 / B,   var_d = M2_d / B.
// The shift keeps the digits of a column whose spread is small next to its mean: the
// relative error of M2 is about eps * (var + (mean - K)^2) / var.
//
//   partial  one workgroup of 1024 threads per block of consecutive rows.  A thread owns
//            one column (or one column of a row lane when D < 1024, so that 1024 / D rows
//            are read side by side and every read of the block is one contiguous run),
//            keeps sixteen row loads in flight, and the row lanes of a column are added in
//            lane order.
//            Output: per block and column (S1, S2).  HBM-bound: each input byte is read
//            once.
//   merge    one workgroup per column adds the block sums: each thread a strided subset in
//            block order, then a fixed butterfly within each wavefront and the wavefronts
//            in order, so the result is the same on every run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "../../include/tabnet.h"
#include "tabnet_handle.hpp"
#include "tabnet_stats.hpp"

namespace tabnet {
namespace {

constexpr int kThreads = 1024;      // partial kernel: 16 waves per workgroup
constexpr int kMergeThreads = 256;
constexpr int kMaxBlocks = 1024;
constexpr int kRowsInFlight = 16;    // row loads a thread issues before it sums them

struct StatsPlan {
  int64_t rows_per_block;
  int blocks;
};

// Rows per block: a multiple of the rows one pass of the workgroup reads in flight
// (lanes x 16), and at least B / 1024 so that at most 1024 blocks write partial sums.
StatsPlan stats_plan(int64_t rows, int D) {
  const int width = D < kThreads ? D : kThreads;
  const int64_t pass = (int64_t)(kThreads / width) * kRowsInFlight;
  const int64_t want = (rows + kMaxBlocks - 1) / kMaxBlocks;
  StatsPlan p;
  p.rows_per_block = std::max<int64_t>(pass, (want + pass - 1) / pass * pass);
  p.blocks = (int)std::max<int64_t>(1, (rows + p.rows_per_block - 1) / p.rows_per_block);
  return p;
}

// Block sums.  Workspace layout: S1[D][G], S2[D][G] (doubles).
__global__ void __launch_bounds__(kThreads)
col_stats_partial(const float* __restrict__ m, int64_t B, const int64_t* __restrict__ B_dev, int D,
                  int64_t rows_per_block, int G, double* __restrict__ ps1, double* __restrict__ ps2) {
  __shared__ double s_1[kThreads], s_2[kThreads];
  if (B_dev != nullptr) B = *B_dev;
  const int g = (int)blockIdx.x;
  const int t = (int)threadIdx.x;
  const int64_t r0 = (int64_t)g * rows_per_block;
  const int64_t r1 = std::min<int64_t>(B, r0 + rows_per_block);
  const int width = D < kThreads ? D : kThreads;   // columns per column group
  const int lanes = kThreads / width;              // rows read side by side
  const int lane_row = t / width;
  for (int c0 = 0; c0 < D; c0 += width) {
    const int col = c0 + t % width;
    double s1 = 0.0, s2 = 0.0;
    if (lane_row < lanes && col < D && B > 0) {
      const float* p = m + col;
      const double K = (double)p[0];
      int64_t r = r0 + lane_row;
      // kRowsInFlight rows per trip: the loads are issued before the dependent FP64 sums
      for (; r + (kRowsInFlight - 1) * lanes < r1; r += kRowsInFlight * lanes) {
        float x[kRowsInFlight];
#pragma unroll
        for (int k = 0; k < kRowsInFlight; ++k) x[k] = p[(r + k * lanes) * D];
#pragma unroll
        for (int k = 0; k < kRowsInFlight; ++k) {
          const double d = (double)x[k] - K;
          s1 += d;
          s2 = __builtin_fma(d, d, s2);
        }
      }
      for (; r < r1; r += lanes) {
        const double d = (double)p[r * D] - K;
        s1 += d;
        s2 = __builtin_fma(d, d, s2);
      }
    }
    s_1[t] = s1;
    s_2[t] = s2;
    __syncthreads();
    if (t < width && col < D) {
      double a = s_1[t], b = s_2[t];
      for (int l = 1; l < lanes; ++l) {
        a += s_1[t + l * width];
        b += s_2[t + l * width];
      }
      ps1[(int64_t)col * G + g] = a;
      ps2[(int64_t)col * G + g] = b;
    }
    __syncthreads();
  }
}

// Sum of v over a wavefront, in a fixed butterfly order (every lane gets the total).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void __launch_bounds__(kMergeThreads)
col_stats_merge(const float* __restrict__ m, int64_t B, const int64_t* __restrict__ B_dev,
                const double* __restrict__ ps1, const double* __restrict__ ps2, int G, double* __restrict__ mean,
                double* __restrict__ var, double* __restrict__ q_out, double* __restrict__ n_out) {
  constexpr int kWaves = kMergeThreads / 64;
  __shared__ double s_1[kWaves], s_2[kWaves];
  if (B_dev != nullptr) B = *B_dev;
  const int col = (int)blockIdx.x;
  const int t = (int)threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int g = t; g < G; g += kMergeThreads) {
    a += ps1[(int64_t)col * G + g];
    b += ps2[(int64_t)col * G + g];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if ((t & 63) == 0) {
    s_1[t >> 6] = a;
    s_2[t >> 6] = b;
  }
  __syncthreads();
  if (t == 0) {
    double S1 = s_1[0], S2 = s_2[0];
    for (int w = 1; w < kWaves; ++w) {
      S1 += s_1[w];
      S2 += s_2[w];
    }
    const double n = (double)(B > 0 ? B : 0);
    double mu = 0.0, q = 0.0;
    if (n > 0.0) {
      mu = (double)m[col] + S1 / n;
      q = std::max(0.0, S2 - S1 * (S1 / n));
    }
    if (mean) mean[col] = mu;
    if (var) var[col] = n > 0.0 ? q / n : 0.0;
    if (q_out) q_out[col] = q;
    if (n_out && col == 0) *n_out = n;
  }
}

}  // namespace

size_t mask_stats_workspace_bytes(int64_t rows, int D) {
  const StatsPlan p = stats_plan(rows, D);
  return (size_t)p.blocks * 2 * (size_t)D * sizeof(double);
}

hipError_t enqueue_mask_stats(const float* masks, int64_t rows, const int64_t* rows_dev, int D, double* mean,
                              double* var, double* q_out, double* n_out, void* workspace, hipStream_t stream) {
  const StatsPlan p = stats_plan(rows, D);
  double* ps1 = static_cast<double*>(workspace);
  double* ps2 = ps1 + (size_t)D * p.blocks;
  hipLaunchKernelGGL(col_stats_partial, dim3((unsigned)p.blocks), dim3(kThreads), 0, stream, masks, rows, rows_dev,
                     D, p.rows_per_block, p.blocks, ps1, ps2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(col_stats_merge, dim3((unsigned)D), dim3(kMergeThreads), 0, stream, masks, rows, rows_dev, ps1, ps2,
                     p.blocks, mean, var, q_out, n_out);
  return hipGetLastError();
}

// Scratch of tabnet_mask_stats_noalloc: the partial sums of the statistics kernels, in a
// file-scope device array that each GPU holds for the life of the process.  In host code
// `scratch` is a stand-in symbol, not a device address: the address of a device's copy
// comes from hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (set up on the first call per device).
hipError_t scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

}  // namespace tabnet

extern "C" {

size_t tabnet_mask_stats_workspace_bytes(int64_t B, int32_t D) {
  if (B < 1 || D < 1) return 0;
  return tabnet::mask_stats_workspace_bytes(B, D);
}

tabnet_status tabnet_mask_stats(const float* masks, int64_t B, int32_t D, double* mean, double* var,
                                void* workspace, size_t workspace_bytes, void* stream) {
  if (!masks || !mean || !var || !workspace) {
    tabnet::set_error("tabnet_mask_stats: NULL pointer argument");
    return TABNET_E_INVALID;
  }
  if (B < 1 || D < 1 || D > (1 << 24) || B > (INT64_MAX / 4) / D) {
    tabnet::set_error("tabnet_mask_stats: B must be >= 1 and D in [1, 2^24] with B * D addressable");
    return TABNET_E_INVALID;
  }
  if (workspace_bytes < tabnet::mask_stats_workspace_bytes(B, D)) {
    tabnet::set_error("tabnet_mask_stats: workspace smaller than tabnet_mask_stats_workspace_bytes(B, D)");
    return TABNET_E_INVALID;
  }
  const hipError_t e = tabnet::enqueue_mask_stats(masks, B, nullptr, D, mean, var, nullptr, nullptr, workspace,
                                                  static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    tabnet::set_error(std::string("tabnet_mask_stats: ") + hipGetErrorString(e));
    return TABNET_E_HIP;
  }
  return TABNET_OK;
}

size_t tabnet_mask_stats_noalloc_max_bytes(void) { return tabnet::kNoAllocScratchBytes; }

tabnet_status tabnet_mask_stats_noalloc(const float* masks, int64_t B, int32_t D, double* mean, double* var,
                                        void* stream) {
  if (!masks || !mean || !var) {
    tabnet::set_error("tabnet_mask_stats_noalloc: NULL pointer argument");
    return TABNET_E_INVALID;
  }
  if (B < 1 || D < 1 || D > (1 << 24) || B > (INT64_MAX / 4) / D) {
    tabnet::set_error("tabnet_mask_stats_noalloc: B must be >= 1 and D in [1, 2^24] with B * D addressable");
    return TABNET_E_INVALID;
  }
  if (tabnet::mask_stats_workspace_bytes(B, D) > tabnet::kNoAllocScratchBytes) {
    tabnet::set_error("tabnet_mask_stats_noalloc: tabnet_mask_stats_workspace_bytes(B, D) exceeds the library's "
                      "scratch (tabnet_mask_stats_noalloc_max_bytes); use tabnet_mask_stats with a workspace");
    return TABNET_E_INVALID;
  }
  void* ws = nullptr;
  hipError_t e = tabnet::scratch_ptr(&ws);
  if (e == hipSuccess)
    e = tabnet::enqueue_mask_stats(masks, B, nullptr, D, mean, var, nullptr, nullptr, ws,
                                   static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    tabnet::set_error(std::string("tabnet_mask_stats_noalloc: ") + hipGetErrorString(e));
    return TABNET_E_HIP;
  }
  return TABNET_OK;
}

}  // extern "C"
