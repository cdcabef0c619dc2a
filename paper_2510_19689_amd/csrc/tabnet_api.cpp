// C ABI of libtabnet: handle life cycle, forward dispatch, error reporting.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tabnet.h"
#include "tabnet_kernel.hpp"
#include "tabnet_pack.hpp"

#include "tabnet_handle.hpp"

using namespace tabnet;

namespace {
thread_local std::string g_err;

tabnet_status fail(tabnet_status st, const std::string& msg) {
  g_err = msg;
  return st;
}
tabnet_status hip_fail(tabnet_handle* h, hipError_t e, const char* what) {
  if (h) h->failed = true;
  return fail(TABNET_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

void release(tabnet_handle* h) {
  if (h->d_emb_meta) (void)hipFree(h->d_emb_meta);
  if (h->d_emb_tables) (void)hipFree(h->d_emb_tables);
  if (h->d_emb_colbits) (void)hipFree(h->d_emb_colbits);
  h->d_emb_meta = nullptr;
  h->d_emb_tables = nullptr;
  h->d_emb_colbits = nullptr;
  if (h->d_wts) (void)hipFree(h->d_wts);
  if (h->d_chunks) (void)hipFree(h->d_chunks);
  if (h->d_affine) (void)hipFree(h->d_affine);
  if (h->d_wfin) (void)hipFree(h->d_wfin);
  h->d_wts = nullptr;
  h->d_chunks = nullptr;
  h->d_affine = h->d_wfin = nullptr;
}

template <class T>
tabnet_status upload(tabnet_handle* h, const std::vector<T>& src, T** dst, const char* what) {
  const size_t n = std::max<size_t>(src.size(), 1) * sizeof(T);
  hipError_t e = hipMalloc((void**)dst, n);
  if (e == hipErrorOutOfMemory) return fail(TABNET_E_OOM, std::string("out of device memory for ") + what);
  if (e != hipSuccess) return hip_fail(h, e, "hipMalloc");
  if (!src.empty()) {
    e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(h, e, "hipMemcpy (weights)");
  }
  return TABNET_OK;
}

tabnet_status ensure_device(tabnet_handle* h) {
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(h, e, "hipGetDevice");
  if (cur != h->device) {
    e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
  }
  return TABNET_OK;
}
}  // namespace

extern "C" {

int tabnet_abi_version(void) { return 100; }

const char* tabnet_last_error(void) { return g_err.c_str(); }

tabnet_status tabnet_load(const char* path, int precision, int device, tabnet_handle** out) {
  if (out == nullptr || path == nullptr) return fail(TABNET_E_INVALID, "tabnet_load: NULL argument");
  *out = nullptr;
  if (precision < TABNET_FP32 || precision > TABNET_FP8_WEIGHTS)
    return fail(TABNET_E_INVALID, "tabnet_load: unknown precision");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(TABNET_E_IO, std::string("tabnet_load: cannot open ") + path);
  std::vector<unsigned char> img;
  unsigned char buf[1 << 16];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) img.insert(img.end(), buf, buf + n);
  std::fclose(f);
  ModelRaw m;
  std::string err;
  tabnet_status st = parse_model(img.data(), img.size(), &m, &err);
  if (st != TABNET_OK) return fail(st, "tabnet_load: " + err);
  const Shape sh = shape_of(m.cfg);
  const KernelEntry* k = find_kernel(precision, sh.DT, sh.NT, sh.KA0, false, m.cfg.D, m.cfg.n_out,
                                     m.cfg.n_d);   // kernel prec = tabnet_precision
  if (!k) {
    char msg[256];
    std::snprintf(msg, sizeof msg,
                  "tabnet_load: no compiled kernel for D=%d (DT=%d), n_d+n_a=%d (NT=%d), n_d=%d (KA0=%d)",
                  m.cfg.D, sh.DT, m.cfg.n_d + m.cfg.n_a, sh.NT, m.cfg.n_d, sh.KA0);
    return fail(TABNET_E_UNSUPPORTED, msg);
  }
  // MX blocks are 32 consecutive channels of each GEMM input, the attention half's from its
  // own first channel.  The kernel forms them from 16-channel tile pairs, which holds when
  // the attention half starts a tile, or lies whole within the tile pair it starts in.
  if (precision >= TABNET_MXFP8 && precision <= TABNET_MXFP6_E3M2 && m.cfg.n_d % 16 != 0 && m.cfg.n_d % 16 + m.cfg.n_a > 32)
    return fail(TABNET_E_UNSUPPORTED,
                "tabnet_load: MX formats need n_d % 16 == 0 or n_d % 16 + n_a <= 32 (the attention half's "
                "32-channel blocks must fall on the kernel's tile pairs)");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return fail(TABNET_E_HIP, std::string("hipGetDeviceCount: ") + hipGetErrorString(e));
  if (device < 0 || device >= ndev) return fail(TABNET_E_INVALID, "tabnet_load: device ordinal out of range");
  e = hipSetDevice(device);
  if (e != hipSuccess) return fail(TABNET_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));

  if (kernel_lds_bytes(k, m.cfg.D, m.cfg.n_out, m.cfg.n_d, 0, 0) > (size_t)kMaxLdsBytes) {
    return fail(TABNET_E_UNSUPPORTED, "tabnet_load: the model needs more LDS than a workgroup has");
  }
  e = prepare_kernel(k);
  if (e != hipSuccess) return fail(TABNET_E_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));

  Packed pk;
  pack_model(m, precision, *kernel_plan(k), kernel_shape(k), &pk);
  tabnet_handle* h = new tabnet_handle();
  h->cfg = m.cfg;
  h->precision = precision;
  h->device = device;
  h->shape = sh;
  h->kernel = k;
  h->n_chunks = (int)pk.chunks.size();
  if ((st = upload(h, pk.wts, &h->d_wts, "weights")) != TABNET_OK ||
      (st = upload(h, pk.chunks, &h->d_chunks, "chunk table")) != TABNET_OK ||
      (st = upload(h, pk.in_affine, &h->d_affine, "input affine")) != TABNET_OK ||
      (st = upload(h, pk.wfin, &h->d_wfin, "final map")) != TABNET_OK) {
    release(h);
    delete h;
    return st;
  }
  *out = h;
  return TABNET_OK;
}

tabnet_status tabnet_get_config(const tabnet_handle* h, tabnet_config* out) {
  if (!h || !out) return fail(TABNET_E_INVALID, "tabnet_get_config: NULL argument");
  *out = h->cfg;
  return TABNET_OK;
}

int tabnet_get_precision(const tabnet_handle* h) { return h ? h->precision : -1; }

tabnet_status tabnet_forward(tabnet_handle* h, const float* X, int64_t B, float* logits,
                             float* masks_agg, float* masks_step, void* stream) {
  if (!h) return fail(TABNET_E_INVALID, "tabnet_forward: NULL handle");
  if (h->failed) return fail(TABNET_E_HIP, "tabnet_forward: handle failed earlier on a HIP error");
  if (B < 0 || B > 0x7fffffffLL) return fail(TABNET_E_INVALID, "tabnet_forward: B out of range");
  if (B == 0) return TABNET_OK;
  if (!X || !logits || !masks_agg) return fail(TABNET_E_INVALID, "tabnet_forward: NULL X, logits or masks_agg");
  tabnet_status st = ensure_device(h);
  if (st != TABNET_OK) return st;
  hipError_t e = tabnet::enqueue_forward(h, X, B, nullptr, logits, masks_agg, masks_step, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(h, e, "tabnet_forward: kernel launch");
  return TABNET_OK;
}

tabnet_status tabnet_set_embeddings(tabnet_handle* h, int32_t n_cols, const int32_t* cards, const int32_t* dims,
                                    const float* tables) {
  if (!h || !cards || !dims) return fail(TABNET_E_INVALID, "tabnet_set_embeddings: NULL argument");
  if (h->failed) return fail(TABNET_E_HIP, "tabnet_set_embeddings: handle failed earlier on a HIP error");
  const int D = h->cfg.D;
  if (n_cols < 1 || n_cols > D) return fail(TABNET_E_INVALID, "tabnet_set_embeddings: n_cols must be in [1, D]");
  // per model feature f: {raw column, levels (0: continuous), index of f's entry in level
  // 0's table row, table row width}
  std::vector<int> meta(4 * (size_t)D);
  int64_t at = 0, base = 0;
  for (int c = 0; c < n_cols; ++c) {
    if (cards[c] < 0 || dims[c] < 1 || (cards[c] == 0 && dims[c] != 1) || cards[c] > (1 << 24))
      return fail(TABNET_E_INVALID,
                  "tabnet_set_embeddings: need cards in [0, 2^24], dims >= 1, and dim 1 for a continuous column");
    if (at + dims[c] > D) return fail(TABNET_E_INVALID, "tabnet_set_embeddings: the widths add up to more than D");
    for (int k = 0; k < dims[c]; ++k) {
      int* d = &meta[4 * (size_t)(at + k)];
      d[0] = c;
      d[1] = cards[c];
      d[2] = (int)(base + k);
      d[3] = dims[c];
    }
    at += dims[c];
    base += (int64_t)cards[c] * dims[c];
    if (base > 0x7fffffffLL) return fail(TABNET_E_INVALID, "tabnet_set_embeddings: tables too large");
  }
  if (at != D) return fail(TABNET_E_INVALID, "tabnet_set_embeddings: the widths must add up to D");
  // membership masks of the per-column mask reduction: for column tile ct and lane l
  // (g = l / 16, r = l % 16), bit 4 t + i is set when feature 16 t + 4 g + i belongs to
  // raw column 16 ct + r
  const int DT = h->shape.DT;
  if (DT > 16) return fail(TABNET_E_UNSUPPORTED, "tabnet_set_embeddings: D above 256");
  const int n_ct = (n_cols + 15) / 16;
  std::vector<uint64_t> colbits((size_t)n_ct * 64, 0);
  for (int ct = 0; ct < n_ct; ++ct)
    for (int l = 0; l < 64; ++l)
      for (int t = 0; t < DT; ++t)
        for (int i = 0; i < 4; ++i) {
          const int f = 16 * t + 4 * (l / 16) + i;
          if (f < D && meta[4 * (size_t)f] == 16 * ct + l % 16) colbits[(size_t)ct * 64 + l] |= 1ull << (4 * t + i);
        }
  if (base > 0 && !tables) return fail(TABNET_E_INVALID, "tabnet_set_embeddings: NULL tables");
  const KernelEntry* k = find_kernel(h->precision, h->shape.DT, h->shape.NT, h->shape.KA0, true, D, h->cfg.n_out,
                                     h->cfg.n_d, h->kernel);
  if (!k) return fail(TABNET_E_UNSUPPORTED, "tabnet_set_embeddings: no compiled raw-row kernel for this shape");
  if (kernel_lds_bytes(k, D, h->cfg.n_out, h->cfg.n_d, n_cols, 0) > (size_t)kMaxLdsBytes)
    return fail(TABNET_E_UNSUPPORTED, "tabnet_set_embeddings: the raw-row kernel needs more LDS than a workgroup has");
  const bool tab_lds = kernel_lds_bytes(k, D, h->cfg.n_out, h->cfg.n_d, n_cols, (int)base) <= (size_t)kMaxLdsBytes;
  tabnet_status st = ensure_device(h);
  if (st != TABNET_OK) return st;
  hipError_t e = prepare_kernel(k);
  if (e != hipSuccess) return hip_fail(h, e, "hipFuncSetAttribute");
  // replace any earlier embedding; the device must be idle for the old buffers to go
  if (h->d_emb_meta || h->d_emb_tables) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(h, e, "hipDeviceSynchronize");
    if (h->d_emb_meta) (void)hipFree(h->d_emb_meta);
    if (h->d_emb_tables) (void)hipFree(h->d_emb_tables);
    if (h->d_emb_colbits) (void)hipFree(h->d_emb_colbits);
    h->d_emb_meta = nullptr;
    h->d_emb_tables = nullptr;
    h->d_emb_colbits = nullptr;
    h->emb_C = 0;
  }
  std::vector<float> tab(tables ? tables : nullptr, tables ? tables + base : nullptr);
  if ((st = upload(h, meta, &h->d_emb_meta, "embedding map")) != TABNET_OK ||
      (st = upload(h, tab, &h->d_emb_tables, "embedding tables")) != TABNET_OK ||
      (st = upload(h, colbits, &h->d_emb_colbits, "column masks")) != TABNET_OK)
    return st;
  h->kernel_raw = k;
  h->emb_C = n_cols;
  h->emb_tab_len = (int)base;
  h->emb_tab_lds = tab_lds;
  return TABNET_OK;
}

tabnet_status tabnet_forward_raw(tabnet_handle* h, const float* X_raw, int64_t B, float* logits,
                                 float* masks_agg_cols, float* masks_step_cols, void* stream) {
  if (!h) return fail(TABNET_E_INVALID, "tabnet_forward_raw: NULL handle");
  if (h->failed) return fail(TABNET_E_HIP, "tabnet_forward_raw: handle failed earlier on a HIP error");
  if (h->emb_C == 0) return fail(TABNET_E_INVALID, "tabnet_forward_raw: no embedding set (tabnet_set_embeddings)");
  if (B < 0 || B > 0x7fffffffLL) return fail(TABNET_E_INVALID, "tabnet_forward_raw: B out of range");
  if (B == 0) return TABNET_OK;
  if (!X_raw || !logits || !masks_agg_cols)
    return fail(TABNET_E_INVALID, "tabnet_forward_raw: NULL X_raw, logits or masks_agg_cols");
  tabnet_status st = ensure_device(h);
  if (st != TABNET_OK) return st;
  hipError_t e = tabnet::enqueue_forward_raw(h, X_raw, B, nullptr, logits, masks_agg_cols, masks_step_cols,
                                             (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(h, e, "tabnet_forward_raw: kernel launch");
  return TABNET_OK;
}

void tabnet_free(tabnet_handle* h) {
  if (!h) return;
  if (ensure_device(h) == TABNET_OK) (void)hipDeviceSynchronize();
  release(h);
  delete h;
}

}  // extern "C"

namespace tabnet {

FwdArgs forward_args(const tabnet_handle* h, const float* X, int64_t B, const int64_t* B_dev,
                     float* logits, float* masks_agg, float* masks_step) {
  FwdArgs a;
  a.X = X;
  a.logits = logits;
  a.masks_agg = masks_agg;
  a.masks_step = masks_step;
  a.wts = h->d_wts;
  a.chunks = h->d_chunks;
  a.n_chunks = h->n_chunks;
  a.in_affine = h->d_affine;
  a.wfin = h->d_wfin;
  a.B = B;
  a.B_dev = B_dev;
  a.D = h->cfg.D;
  a.n_d = h->cfg.n_d;
  a.n_a = h->cfg.n_a;
  a.n_steps = h->cfg.n_steps;
  a.n_sh = h->cfg.n_shared;
  a.n_ind = h->cfg.n_indep;
  a.n_out = h->cfg.n_out;
  a.gamma = (float)h->cfg.gamma;
  a.emb_meta = nullptr;
  a.emb_tables = nullptr;
  a.C = 0;
  a.tab_len = 0;
  a.tab_lds = 0;
  a.colbits = nullptr;
  return a;
}

hipError_t enqueue_forward(const tabnet_handle* h, const float* X, int64_t B, const int64_t* B_dev,
                           float* logits, float* masks_agg, float* masks_step, hipStream_t stream) {
  return launch_forward(h->kernel, forward_args(h, X, B, B_dev, logits, masks_agg, masks_step), stream);
}

hipError_t enqueue_forward_raw(const tabnet_handle* h, const float* X_raw, int64_t B, const int64_t* B_dev,
                               float* logits, float* masks_agg, float* masks_step, hipStream_t stream) {
  FwdArgs a = forward_args(h, X_raw, B, B_dev, logits, masks_agg, masks_step);
  a.emb_meta = h->d_emb_meta;
  a.emb_tables = h->d_emb_tables;
  a.C = h->emb_C;
  a.tab_len = h->emb_tab_len;
  a.tab_lds = h->emb_tab_lds ? 1 : 0;
  a.colbits = h->d_emb_colbits;
  return launch_forward(h->kernel_raw, a, stream);
}

void set_error(const std::string& msg) { g_err = msg; }

}  // namespace tabnet
