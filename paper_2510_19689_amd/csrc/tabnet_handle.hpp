// Library-internal view of a model handle, shared by the forward ABI and the server.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/tabnet.h"
#include "tabnet_kernel.hpp"
#include "tabnet_pack.hpp"

namespace tabnet {
struct KernelEntry;
const KernelEntry* find_kernel(int prec, int DT, int NT, int KA0, bool raw, int D, int n_out, int n_d,
                               const KernelEntry* twin = nullptr);
size_t kernel_lds_bytes(const KernelEntry* k, int D, int n_out, int n_d, int C, int tab_lds_len);
hipError_t prepare_kernel(const KernelEntry* k);
hipError_t launch_forward(const KernelEntry* k, const FwdArgs& a, hipStream_t stream);
const Plan* kernel_plan(const KernelEntry* k);
// (DT, NT, KA0) the kernel is compiled for: the model's own, or larger for a generic kernel
Shape kernel_shape(const KernelEntry* k);
}  // namespace tabnet

struct tabnet_handle {
  tabnet_config cfg;
  int precision;
  int device;
  tabnet::Shape shape;
  const tabnet::KernelEntry* kernel;
  unsigned char* d_wts = nullptr;
  tabnet::ChunkRec* d_chunks = nullptr;
  float* d_affine = nullptr;
  float* d_wfin = nullptr;
  int n_chunks = 0;
  bool failed = false;
  // categorical embedding of raw rows (tabnet_set_embeddings); C = 0 until set
  const tabnet::KernelEntry* kernel_raw = nullptr;
  int* d_emb_meta = nullptr;
  float* d_emb_tables = nullptr;
  int emb_C = 0;
  uint64_t* d_emb_colbits = nullptr;   // feature-to-column membership masks per lane
  int emb_tab_len = 0;           // floats in d_emb_tables
  bool emb_tab_lds = false;      // the tables fit in LDS beside everything else
};

namespace tabnet {
// Arguments of one forward over device buffers.  With B_dev set, the kernel reads the
// live row count from device memory (grid sized for B rows): a captured graph can then
// be replayed for any row count up to B.
FwdArgs forward_args(const tabnet_handle* h, const float* X, int64_t B, const int64_t* B_dev,
                     float* logits, float* masks_agg, float* masks_step);
hipError_t enqueue_forward(const tabnet_handle* h, const float* X, int64_t B, const int64_t* B_dev,
                           float* logits, float* masks_agg, float* masks_step, hipStream_t stream);
// The same over raw rows X_raw[B, C] (needs tabnet_set_embeddings): masks per raw column.
hipError_t enqueue_forward_raw(const tabnet_handle* h, const float* X_raw, int64_t B, const int64_t* B_dev,
                               float* logits, float* masks_agg, float* masks_step, hipStream_t stream);
// Sets the calling thread's tabnet_last_error message.
void set_error(const std::string& msg);
}  // namespace tabnet
