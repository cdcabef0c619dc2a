// Load-time model preparation: parse TNW1, fold batch norms (FP64), round, pack.
#include "tabnet_pack.hpp"

#include <cmath>
#include <cstring>

namespace tabnet {

namespace {
constexpr char kMagic[4] = {'T', 'N', 'W', '1'};
constexpr uint32_t kVersion = 1;
constexpr size_t kHeader = 64;

template <class T>
T rd(const unsigned char* p) {
  T v;
  std::memcpy(&v, p, sizeof(T));
  return v;
}
size_t align256(size_t n) { return (n + 255) & ~size_t(255); }
}  // namespace

int64_t model_param_count(const tabnet_config& c) {
  const int64_t N = (int64_t)c.n_d + c.n_a, N2 = 2 * N;
  int64_t n = 4 * (int64_t)c.D;
  for (int l = 0; l < c.n_shared; ++l) n += N2 * (l == 0 ? c.D : N) + 4 * N2;
  for (int l = 0; l < c.n_indep; ++l)
    n += (int64_t)(c.n_steps + 1) * (N2 * ((c.n_shared == 0 && l == 0) ? c.D : N) + 4 * N2);
  n += (int64_t)c.n_steps * ((int64_t)c.D * c.n_a + 4 * (int64_t)c.D);
  n += (int64_t)c.n_out * c.n_d;
  return n;
}

tabnet_status validate_config(const tabnet_config& c, std::string* err) {
  auto bad = [&](const char* m) {
    *err = std::string("invalid model header: ") + m;
    return TABNET_E_INVALID;
  };
  if (c.D < 1 || c.D > 4096) return bad("D must be in [1, 4096]");
  if (c.n_d < 1 || c.n_a < 1) return bad("n_d and n_a must be >= 1");
  if (c.n_d + c.n_a > 1024) return bad("n_d + n_a must be <= 1024");
  if (c.n_steps < 1 || c.n_steps > 32) return bad("n_steps must be in [1, 32]");
  if (c.n_shared < 0 || c.n_indep < 0 || c.n_shared + c.n_indep < 1)
    return bad("need n_shared, n_indep >= 0 and at least one GLU layer");
  if ((int64_t)c.n_shared + (int64_t)(c.n_steps + 1) * c.n_indep > 96)
    return bad("too many feature-transformer layers (n_shared + (n_steps+1) n_indep > 96)");
  if (c.n_out < 1 || c.n_out > 64) return bad("n_out must be in [1, 64]");
  if (!(c.gamma >= 1.0) || !std::isfinite(c.gamma)) return bad("gamma must be finite and >= 1");
  if (!(c.bn_eps > 0.0) || !std::isfinite(c.bn_eps)) return bad("bn_eps must be > 0");
  return TABNET_OK;
}

tabnet_status parse_model(const unsigned char* data, size_t len, ModelRaw* m, std::string* err) {
  if (len < kHeader) {
    *err = "weight file truncated (shorter than the 64-byte header)";
    return TABNET_E_IO;
  }
  if (std::memcmp(data, kMagic, 4) != 0) {
    *err = "bad magic: not a TNW1 weight file";
    return TABNET_E_IO;
  }
  if (rd<uint32_t>(data + 4) != kVersion) {
    *err = "unsupported TNW1 version";
    return TABNET_E_IO;
  }
  tabnet_config& c = m->cfg;
  std::memset(&c, 0, sizeof(c));
  c.D = rd<int32_t>(data + 8);
  c.n_d = rd<int32_t>(data + 12);
  c.n_a = rd<int32_t>(data + 16);
  c.n_steps = rd<int32_t>(data + 20);
  c.n_shared = rd<int32_t>(data + 24);
  c.n_indep = rd<int32_t>(data + 28);
  c.n_out = rd<int32_t>(data + 32);
  c.gamma = rd<double>(data + 40);
  c.bn_eps = rd<double>(data + 48);
  const uint64_t nf = rd<uint64_t>(data + 56);
  tabnet_status st = validate_config(c, err);
  if (st != TABNET_OK) return st;
  if ((int64_t)nf != model_param_count(c)) {
    *err = "parameter count in header does not match the model shape";
    return TABNET_E_INVALID;
  }
  if (len < kHeader + nf * 4) {
    *err = "weight file truncated (payload shorter than the header announces)";
    return TABNET_E_IO;
  }
  m->storage.resize(nf);
  std::memcpy(m->storage.data(), data + kHeader, nf * 4);
  const float* p = m->storage.data();
  auto take = [&](int64_t n) {
    const float* q = p;
    p += n;
    return q;
  };
  auto take_bn = [&](int n) {
    BNRaw b;
    b.mean = take(n);
    b.var = take(n);
    b.gamma = take(n);
    b.beta = take(n);
    return b;
  };
  const int N = c.n_d + c.n_a, N2 = 2 * N;
  m->bn_in = take_bn(c.D);
  m->shared.clear();
  for (int l = 0; l < c.n_shared; ++l) {
    LayerRaw L;
    L.rows = N2;
    L.cols = l == 0 ? c.D : N;
    L.W = take((int64_t)L.rows * L.cols);
    L.bn = take_bn(N2);
    m->shared.push_back(L);
  }
  m->indep.assign(c.n_steps + 1, {});
  for (int s = 0; s <= c.n_steps; ++s)
    for (int l = 0; l < c.n_indep; ++l) {
      LayerRaw L;
      L.rows = N2;
      L.cols = (c.n_shared == 0 && l == 0) ? c.D : N;
      L.W = take((int64_t)L.rows * L.cols);
      L.bn = take_bn(N2);
      m->indep[s].push_back(L);
    }
  m->att.clear();
  for (int i = 0; i < c.n_steps; ++i) {
    LayerRaw L;
    L.rows = c.D;
    L.cols = c.n_a;
    L.W = take((int64_t)L.rows * L.cols);
    L.bn = take_bn(c.D);
    m->att.push_back(L);
  }
  m->w_fin = take((int64_t)c.n_out * c.n_d);
  if (p != m->storage.data() + nf) {
    *err = "internal: parameter walk mismatch";
    return TABNET_E_INVALID;
  }
  for (uint64_t i = 0; i < nf; ++i)
    if (!std::isfinite(m->storage[i])) {
      *err = "weight file holds a non-finite parameter";
      return TABNET_E_INVALID;
    }
  for (int j = 0; j < c.D; ++j)
    if (!(m->bn_in.var[j] + c.bn_eps > 0)) {
      *err = "input batch-norm variance + eps must be > 0";
      return TABNET_E_INVALID;
    }
  return TABNET_OK;
}

void fold_layer(const LayerRaw& L, double eps, std::vector<double>* Wf, std::vector<double>* bf) {
  Wf->assign((size_t)L.rows * L.cols, 0.0);
  bf->assign(L.rows, 0.0);
  for (int o = 0; o < L.rows; ++o) {
    const double s = (double)L.bn.gamma[o] / std::sqrt((double)L.bn.var[o] + eps);
    for (int k = 0; k < L.cols; ++k) (*Wf)[(size_t)o * L.cols + k] = s * (double)L.W[(size_t)o * L.cols + k];
    (*bf)[o] = (double)L.bn.beta[o] - s * (double)L.bn.mean[o];
  }
}

// ---------------------------------------------------------------- rounding
// bfloat16 keeps the float32 exponent and the top 7 stored mantissa bits.  From a double:
// the 52-bit mantissa is cut to 7 bits with round-to-nearest-even on the 45 dropped bits.
uint16_t bf16_bits_rne(double x) {
  uint64_t u;
  std::memcpy(&u, &x, 8);
  const uint16_t sign = (uint16_t)((u >> 63) << 15);
  const int e = (int)((u >> 52) & 0x7ff);
  uint64_t man = u & ((uint64_t(1) << 52) - 1);
  if (e == 0x7ff) return (uint16_t)(sign | 0x7f80 | (man ? 0x40 : 0));   // inf / nan
  if (e == 0) return sign;                                                // zero or tiny
  int eb = e - 1023 + 127;
  if (eb <= 0) {
    // below the bfloat16 normal range: round onto the subnormal grid 2^-133
    const double ax = std::fabs(x);
    const double q = std::nearbyint(std::ldexp(ax, 133));   // ties to even (default mode)
    return (uint16_t)(sign | (uint16_t)q);
  }
  uint64_t keep = man >> 45;
  const uint64_t rest = man & ((uint64_t(1) << 45) - 1);
  const uint64_t half = uint64_t(1) << 44;
  if (rest > half || (rest == half && (keep & 1))) {
    ++keep;
    if (keep == 128) {
      keep = 0;
      ++eb;
    }
  }
  if (eb >= 255) return (uint16_t)(sign | 0x7f80);
  return (uint16_t)(sign | (eb << 7) | keep);
}

double bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

// E4M3FN: bias 7, 3 stored mantissa bits, normals from 2^-6, subnormals k * 2^-9,
// largest finite 448 (S.1111.110); values beyond saturate to +-448.
uint8_t e4m3_bits_rne(double x) {
  const uint8_t sign = std::signbit(x) ? 0x80 : 0;
  double ax = std::fabs(x);
  if (std::isnan(x)) return 0x7f;
  if (ax >= 448.0) return sign | 0x7e;
  if (ax < std::ldexp(1.0, -6)) {
    const double q = std::nearbyint(std::ldexp(ax, 9));   // 0..8; 8 means 2^-6
    return sign | (uint8_t)q;                               // 8 encodes as exponent 1, man 0
  }
  int e;
  const double m = std::frexp(ax, &e);                     // ax = m 2^e, m in [0.5, 1)
  double q = std::nearbyint(std::ldexp(m, 4));              // 8..16
  if (q == 16.0) {
    q = 8.0;
    ++e;
  }
  const int eb = (e - 1) + 7;
  if (eb > 15 || (eb == 15 && q - 8.0 > 6.0)) return sign | 0x7e;
  return sign | (uint8_t)((eb << 3) | ((int)q - 8));
}

double e4m3_value(uint8_t b) {
  const int s = b >> 7, e = (b >> 3) & 15, m = b & 7;
  double v = e == 0 ? std::ldexp((double)m, -9) : std::ldexp(1.0 + m / 8.0, e - 7);
  if (e == 15 && m == 7) v = NAN;
  return s ? -v : v;
}

// ---------------------------------------------------------------- packing
Shape shape_of(const tabnet_config& c) {
  Shape s;
  s.DT = (c.D + 15) / 16;
  s.NT = (c.n_d + c.n_a + 15) / 16;
  s.KA0 = c.n_d / 16;
  return s;
}

namespace {

// A GEMM as the kernel sees it: MT output tiles x KT input tiles.  row_of(mt, i) gives
// the row of Wf feeding output slot 16 mt + i (or -1: zero row); col_of(kin) maps the
// kernel's K index (16 t + 4 g + j over the KT tiles) to a column of Wf (or -1).
struct GemmView {
  const std::vector<double>* Wf;
  int cols;
  int MT, KT;
  int (*row_of)(const void*, int, int);
  int (*col_of)(const void*, int);
  const void* ctx;
};

// Per-row quantisation scales for FP8 (one per Wf row); 1 for the other precisions.
void row_scales(const GemmView& g, int precision, int rows, std::vector<double>* sc) {
  sc->assign(rows, 1.0);
  if (precision != TABNET_FP8_E4M3) return;
  for (int r = 0; r < rows; ++r) {
    double amax = 0;
    for (int k = 0; k < g.cols; ++k) amax = std::fmax(amax, std::fabs((*g.Wf)[(size_t)r * g.cols + k]));
    (*sc)[r] = amax > 0 ? amax / 448.0 : 1.0;
  }
}

void emit(std::vector<unsigned char>* out, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  out->insert(out->end(), b, b + n);
}

// Appends the A-operand fragments of one GEMM to `wts` (aligned) and returns its offset.
int64_t pack_gemm(const GemmView& g, int precision, const std::vector<double>& sc,
                  std::vector<unsigned char>* wts) {
  wts->resize(align256(wts->size()), 0);
  const int64_t off = (int64_t)wts->size();
  auto wv = [&](int mt, int i, int kin) -> double {
    const int r = g.row_of(g.ctx, mt, i);
    const int c = g.col_of(g.ctx, kin);
    if (r < 0 || c < 0) return 0.0;
    return (*g.Wf)[(size_t)r * g.cols + c] / sc[r];
  };
  for (int mt = 0; mt < g.MT; ++mt) {
    if (precision == TABNET_FP32) {
      for (int kt = 0; kt < g.KT; ++kt)
        for (int lane = 0; lane < 64; ++lane) {
          const int i = lane & 15, q = lane >> 4;
          float v[4];
          for (int r = 0; r < 4; ++r) v[r] = (float)wv(mt, i, 16 * kt + 4 * q + r);
          emit(wts, v, sizeof v);
        }
    } else {
      const int KP = (g.KT + 1) / 2;   // an odd last tile is paired with a zero tile
      for (int kb = 0; kb < KP; ++kb)
        for (int lane = 0; lane < 64; ++lane) {
          const int i = lane & 15, q = lane >> 4;
          uint16_t v[8];
          for (int j = 0; j < 8; ++j) {
            const int t = 2 * kb + j / 4;
            const double x = t < g.KT ? wv(mt, i, 16 * t + 4 * q + (j & 3)) : 0.0;
            v[j] = precision == TABNET_BF16 ? bf16_bits_rne(x) : bf16_bits_rne(e4m3_value(e4m3_bits_rne(x)));
          }
          emit(wts, v, sizeof v);
        }
    }
  }
  return off;
}

struct GluCtx {
  int N, NT, K;
};
int glu_row(const void* c, int mt, int i) {
  const GluCtx* x = (const GluCtx*)c;
  const int half = mt / x->NT, ch = 16 * (mt % x->NT) + i;
  return ch < x->N ? half * x->N + ch : -1;
}
int plain_col(const void* c, int kin) {
  const GluCtx* x = (const GluCtx*)c;
  return kin < x->K ? kin : -1;
}
struct AttCtx {
  int D, n_d, N, KA0;
};
int att_row(const void* c, int mt, int i) {
  const AttCtx* x = (const AttCtx*)c;
  const int d = 16 * mt + i;
  return d < x->D ? d : -1;
}
int att_col(const void* c, int kin) {
  const AttCtx* x = (const AttCtx*)c;
  const int ch = 16 * x->KA0 + kin;   // channel of h
  return (ch >= x->n_d && ch < x->N) ? ch - x->n_d : -1;
}

}  // namespace

void pack_model(const ModelRaw& m, int precision, Packed* out) {
  const tabnet_config& c = m.cfg;
  const Shape sh = shape_of(c);
  const int N = c.n_d + c.n_a;
  *out = Packed();
  // input BN as a per-column affine map
  out->in_affine.assign(32 * sh.DT, 0.f);
  for (int j = 0; j < c.D; ++j) {
    const double s = (double)m.bn_in.gamma[j] / std::sqrt((double)m.bn_in.var[j] + c.bn_eps);
    out->in_affine[j] = (float)s;
    out->in_affine[16 * sh.DT + j] = (float)((double)m.bn_in.beta[j] - s * (double)m.bn_in.mean[j]);
  }
  // Bias block of one GEMM: for each output tile, 16 floats in C-layout order
  // (slot 4 q + i of tile mt is output feature 16 mt + 4 q + i).  FP8 appends the
  // per-output scales in the same order.
  auto add_bias = [&](const std::vector<double>& bf, const std::vector<double>& sc, int MT,
                      int (*row_of)(const void*, int, int), const void* ctx) {
    const int32_t off = (int32_t)out->bias.size();
    for (int mt = 0; mt < MT; ++mt)
      for (int i = 0; i < 16; ++i) {
        const int r = row_of(ctx, mt, i);
        out->bias.push_back(r < 0 ? 0.f : (float)bf[r]);
      }
    if (precision == TABNET_FP8_E4M3)
      for (int mt = 0; mt < MT; ++mt)
        for (int i = 0; i < 16; ++i) {
          const int r = row_of(ctx, mt, i);
          out->bias.push_back(r < 0 ? 0.f : (float)sc[r]);
        }
    return off;
  };
  std::vector<const LayerRaw*> ft;
  for (const auto& L : m.shared) ft.push_back(&L);
  for (const auto& pass : m.indep)
    for (const auto& L : pass) ft.push_back(&L);
  std::vector<double> Wf, bf, sc;
  for (const LayerRaw* L : ft) {
    fold_layer(*L, c.bn_eps, &Wf, &bf);
    GluCtx ctx{N, sh.NT, L->cols};
    // K tiles: the first layer of a pass reads the D features, the others the N channels
    GemmView g{&Wf, L->cols, 2 * sh.NT, (L->cols + 15) / 16, glu_row, plain_col, &ctx};
    row_scales(g, precision, L->rows, &sc);
    out->ft_w.push_back(pack_gemm(g, precision, sc, &out->wts));
    out->ft_b.push_back(add_bias(bf, sc, 2 * sh.NT, glu_row, &ctx));
  }
  for (const auto& L : m.att) {
    fold_layer(L, c.bn_eps, &Wf, &bf);
    AttCtx ctx{c.D, c.n_d, N, sh.KA0};
    GemmView g{&Wf, L.cols, sh.DT, sh.NT - sh.KA0, att_row, att_col, &ctx};
    row_scales(g, precision, L.rows, &sc);
    out->att_w.push_back(pack_gemm(g, precision, sc, &out->wts));
    out->att_b.push_back(add_bias(bf, sc, sh.DT, att_row, &ctx));
  }
  out->wts.resize(align256(out->wts.size()), 0);
  out->wfin.assign(m.w_fin, m.w_fin + (size_t)c.n_out * c.n_d);
}

}  // namespace tabnet
