// Host-only test hooks (include/tabnet_internal.h).
#include "../../include/tabnet_internal.h"

#include <string>
#include <vector>

#include "tabnet_handle.hpp"
#include "tabnet_pack.hpp"
#include "tabnet_serve.hpp"

using namespace tabnet;

extern "C" {

uint16_t tabnet_hook_bf16_bits(double x) { return bf16_bits_rne(x); }
uint8_t tabnet_hook_e4m3_bits(double x) { return e4m3_bits_rne(x); }
uint8_t tabnet_hook_e2m1_bits(double x) { return e2m1_bits_rne(x); }
uint8_t tabnet_hook_e2m3_bits(double x) { return e2m3_bits_rne(x); }
uint8_t tabnet_hook_e5m2_bits(double x) { return e5m2_bits_rne(x); }
uint8_t tabnet_hook_e3m2_bits(double x) { return e3m2_bits_rne(x); }
int tabnet_hook_mx_exponent(double amax, int emax) { return mx_exponent(amax, emax); }

void tabnet_hook_int8_rows(double* W, int rows, int cols, double* scales) {
  if (!W || !scales || rows < 1 || cols < 1) return;
  std::vector<double> w(W, W + (size_t)rows * cols), b(rows, 0.0), s;
  quantize_rows_int8(&w, &b, rows, cols, rows, &s);
  for (size_t i = 0; i < w.size(); ++i) W[i] = w[i];
  for (int r = 0; r < rows; ++r) scales[r] = s[r];
}

tabnet_status tabnet_hook_parse(const void* buf, size_t len, tabnet_config* cfg) {
  if (!buf || !cfg) return TABNET_E_INVALID;
  ModelRaw m;
  std::string err;
  tabnet_status st = parse_model((const unsigned char*)buf, len, &m, &err);
  if (st == TABNET_OK) *cfg = m.cfg;
  return st;
}

tabnet_status tabnet_hook_fold(const void* buf, size_t len, int layer, double* Wf, double* bf,
                               int* rows, int* cols) {
  if (!buf || !rows || !cols) return TABNET_E_INVALID;
  ModelRaw m;
  std::string err;
  tabnet_status st = parse_model((const unsigned char*)buf, len, &m, &err);
  if (st != TABNET_OK) return st;
  std::vector<const LayerRaw*> all;
  for (const auto& L : m.shared) all.push_back(&L);
  for (const auto& p : m.indep)
    for (const auto& L : p) all.push_back(&L);
  for (const auto& L : m.att) all.push_back(&L);
  if (layer < 0 || layer >= (int)all.size()) return TABNET_E_INVALID;
  *rows = all[layer]->rows;
  *cols = all[layer]->cols;
  if (!Wf || !bf) return TABNET_OK;
  std::vector<double> w, b;
  fold_layer(*all[layer], m.cfg.bn_eps, &w, &b);
  for (size_t i = 0; i < w.size(); ++i) Wf[i] = w[i];
  for (size_t i = 0; i < b.size(); ++i) bf[i] = b[i];
  return TABNET_OK;
}

tabnet_status tabnet_hook_packed_sizes(const void* buf, size_t len, int precision,
                                       int64_t* wts_bytes, int64_t* n_chunks) {
  if (!buf || !wts_bytes || !n_chunks) return TABNET_E_INVALID;
  ModelRaw m;
  std::string err;
  tabnet_status st = parse_model((const unsigned char*)buf, len, &m, &err);
  if (st != TABNET_OK) return st;
  if (precision < TABNET_FP32 || precision > TABNET_FP8_WEIGHTS) return TABNET_E_INVALID;
  const Shape sh = shape_of(m.cfg);
  const KernelEntry* k = find_kernel(precision, sh.DT, sh.NT, sh.KA0, false, m.cfg.D, m.cfg.n_out, m.cfg.n_d);
  if (!k) return TABNET_E_UNSUPPORTED;
  Packed pk;
  pack_model(m, precision, *kernel_plan(k), kernel_shape(k), &pk);
  *wts_bytes = (int64_t)pk.wts.size();
  *n_chunks = (int64_t)pk.chunks.size();
  return TABNET_OK;
}

}  // extern "C"

extern "C" tabnet_status tabnet_hook_serve_start_fake(const tabnet_config* cfgs, int n, const tabnet_serve_opts* opts,
                                                      int delay_us, int fail_launch, int fail_wait,
                                                      tabnet_server** out) {
  using namespace tabnet;
  if (!cfgs || n < 1 || !out) return TABNET_E_INVALID;
  tabnet_serve_opts o;
  tabnet_status st = fill_opts(opts, &o);
  if (st != TABNET_OK) return st;
  std::vector<ModelInfo> models;
  for (int i = 0; i < n; ++i) models.push_back(info_of(cfgs[i], o.with_step_masks != 0, nullptr));
  Executor* ex = make_fake_executor(models, o, delay_us, fail_launch, fail_wait);   // before models is moved
  return start_with(std::move(models), ex, o, out);
}

extern "C" void tabnet_hook_serve_copy(void* dst, const void* src, size_t n) { tabnet::serve_copy(dst, src, n); }
