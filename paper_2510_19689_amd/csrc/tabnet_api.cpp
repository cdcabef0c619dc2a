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
  if (precision < TABNET_FP32 || precision > TABNET_FP8_E4M3)
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
  const int kprec = precision == TABNET_FP32 ? 0 : (precision == TABNET_BF16 ? 1 : 2);
  const KernelEntry* k = find_kernel(kprec, sh.DT, sh.NT, sh.KA0);
  if (!k) {
    char msg[256];
    std::snprintf(msg, sizeof msg,
                  "tabnet_load: no compiled kernel for D=%d (DT=%d), n_d+n_a=%d (NT=%d), n_d=%d (KA0=%d)",
                  m.cfg.D, sh.DT, m.cfg.n_d + m.cfg.n_a, sh.NT, m.cfg.n_d, sh.KA0);
    return fail(TABNET_E_UNSUPPORTED, msg);
  }
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return fail(TABNET_E_HIP, std::string("hipGetDeviceCount: ") + hipGetErrorString(e));
  if (device < 0 || device >= ndev) return fail(TABNET_E_INVALID, "tabnet_load: device ordinal out of range");
  e = hipSetDevice(device);
  if (e != hipSuccess) return fail(TABNET_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));

  if (kernel_lds_bytes(k, m.cfg.D, m.cfg.n_out, m.cfg.n_d) > 160 * 1024) {
    return fail(TABNET_E_UNSUPPORTED, "tabnet_load: the model needs more LDS than a workgroup has");
  }
  e = prepare_kernel(k, m.cfg.D, m.cfg.n_out, m.cfg.n_d);
  if (e != hipSuccess) return fail(TABNET_E_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));

  Packed pk;
  pack_model(m, precision, &pk);
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
  return a;
}

hipError_t enqueue_forward(const tabnet_handle* h, const float* X, int64_t B, const int64_t* B_dev,
                           float* logits, float* masks_agg, float* masks_step, hipStream_t stream) {
  return launch_forward(h->kernel, forward_args(h, X, B, B_dev, logits, masks_agg, masks_step), stream);
}

void set_error(const std::string& msg) { g_err = msg; }

}  // namespace tabnet
