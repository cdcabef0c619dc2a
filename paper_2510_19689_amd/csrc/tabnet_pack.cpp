// Load-time model preparation: parse TNW1, fold batch norms (FP64), round, pack.
#include "tabnet_pack.hpp"

#include <algorithm>
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

// Symmetric INT8 with one scale per output row: s_n = max_k |W'_nk| / 127 (1 for a zero
// row), Wf <- round(W' / s_n) (ties to even), the codes in [-127, 127].  The shift is kept
// as it is: the kernel adds it after dequantising the integer products.  Rows
// [neg_lo, rows) (the gate half of a GLU layer) get their shift and scale multiplied by
// -log2(e), the factor of the sigmoid's exponent.
void quantize_rows_int8(std::vector<double>* Wf, std::vector<double>* bf, int rows, int cols, int neg_lo,
                        std::vector<double>* scale) {
  const double kNegLog2e = -1.4426950408889634;
  scale->assign(rows, 1.0);
  for (int r = 0; r < rows; ++r) {
    double amax = 0;
    for (int k = 0; k < cols; ++k) amax = std::fmax(amax, std::fabs((*Wf)[(size_t)r * cols + k]));
    const double s = amax > 0 ? amax / 127.0 : 1.0;
    for (int k = 0; k < cols; ++k) {
      double& w = (*Wf)[(size_t)r * cols + k];
      w = std::nearbyint(w / s);
    }
    (*scale)[r] = r >= neg_lo ? s * kNegLog2e : s;
    if (r >= neg_lo) (*bf)[r] *= kNegLog2e;
  }
}

// FP4 E2M1 bits (sign in bit 3) of x, round to nearest even, saturating at +-6.  The grid
// is 0, 0.5, 1, 1.5 (step 0.5), 2, 3 (step 1), 4, 6 (step 2); within each step range the
// code is the rounded multiple plus an offset of the same parity, so ties to the even
// multiple are ties to the even code.
uint8_t e2m1_bits_rne(double x) {
  const uint8_t sign = std::signbit(x) ? 8 : 0;
  const double a = std::fabs(x);
  if (std::isnan(x)) return 7;
  int code;
  if (a < 2.0) code = (int)std::nearbyint(2.0 * a);             // 0 .. 4 (4 = 2.0)
  else if (a < 4.0) code = (int)std::nearbyint(a) + 2;          // 4 .. 6 (6 = 4.0)
  else code = std::min(7, (int)std::nearbyint(a / 2.0) + 4);    // 6, 7, saturating
  return sign | (uint8_t)code;
}

// FP6 E2M3 bits (sign in bit 5) of x, round to nearest even, saturating at +-7.5.  The grid
// has a step of 1/8 up to 2, 1/4 up to 4 and 1/2 up to 7.5; as for E2M1, each step range
// maps the rounded multiple to the code by an offset of the same parity.
uint8_t e2m3_bits_rne(double x) {
  const uint8_t sign = std::signbit(x) ? 32 : 0;
  const double a = std::fabs(x);
  if (std::isnan(x)) return 31;
  int code;
  if (a < 2.0) code = (int)std::nearbyint(8.0 * a);             // 0 .. 16 (16 = 2.0)
  else if (a < 4.0) code = (int)std::nearbyint(4.0 * a) + 8;    // 16 .. 24 (24 = 4.0)
  else code = std::min(31, (int)std::nearbyint(2.0 * a) + 16);  // 24 .. 31, saturating
  return sign | (uint8_t)code;
}

// FP8 E5M2: bias 15, 2 stored mantissa bits, normals from 2^-14, subnormals k * 2^-16,
// largest finite 57344 (S.11110.11); values beyond saturate to +-57344.
uint8_t e5m2_bits_rne(double x) {
  const uint8_t sign = std::signbit(x) ? 0x80 : 0;
  const double ax = std::fabs(x);
  if (std::isnan(x)) return 0x7f;
  if (ax >= 57344.0) return sign | 0x7b;
  if (ax < std::ldexp(1.0, -14)) return sign | (uint8_t)std::nearbyint(std::ldexp(ax, 16));   // 4 = 2^-14
  int e;
  const double m = std::frexp(ax, &e);                     // ax = m 2^e, m in [0.5, 1)
  double q = std::nearbyint(std::ldexp(m, 3));              // 4..8
  if (q == 8.0) {
    q = 4.0;
    ++e;
  }
  const int eb = (e - 1) + 15;
  if (eb > 30) return sign | 0x7b;
  return sign | (uint8_t)((eb << 2) | ((int)q - 4));
}

// FP6 E3M2 bits (sign in bit 5) of x, round to nearest even, saturating at +-28.  Below
// 1/2 the grid has a step of 1/16 (subnormals up to 3/16, then the binade [1/4, 1/2));
// each binade [2^k, 2^(k+1)) above has a step of 2^(k-2).  The code is the rounded
// multiple plus the even offset 4 k + 8, so ties to the even multiple are ties to the
// even code.
uint8_t e3m2_bits_rne(double x) {
  const uint8_t sign = std::signbit(x) ? 32 : 0;
  const double a = std::fabs(x);
  if (std::isnan(x)) return 31;
  if (a >= 28.0) return sign | 31;
  int e = 0;
  if (a >= 0.5) std::frexp(a, &e);                          // a = m 2^e, m in [0.5, 1)
  const int k = a >= 0.5 ? e - 1 : -2;
  const int code = (int)std::nearbyint(std::ldexp(a, 2 - k)) + 4 * k + 8;
  return sign | (uint8_t)std::min(31, code);
}

int mx_exponent(double amax, int emax) {
  if (!(amax > 0)) return 0;
  int e;
  std::frexp(amax, &e);   // amax = m 2^e, m in [0.5, 1): floor(log2 amax) = e - 1
  return std::max(-126, std::min(127, e - 1 - emax));
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

void emit(std::vector<unsigned char>* out, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  out->insert(out->end(), b, b + n);
}

// One A-operand fragment group: output tile rows row_of(i) (i = 0..15, -1 = zero row) of
// the folded weights Wf [rows][cols], K over KT tiles with col_of(kin) mapping the
// kernel's K index 16 t + 4 q + j to a column of Wf (-1 = zero).
// Only k-blocks [kb_lo, kb_hi) are emitted (a k-block is one K tile in FP32, a pair of
// K tiles in BF16, four K tiles in INT8); kb_hi < 0 means all of them.  In INT8, Wf holds
// the integer codes.
template <class RowOf, class ColOf>
void emit_fragments(const std::vector<double>& Wf, int cols, int KT, int precision, RowOf row_of,
                    ColOf col_of, std::vector<unsigned char>* wts, int kb_lo = 0, int kb_hi = -1) {
  auto wv = [&](int i, int kin) -> double {
    const int r = row_of(i);
    const int c = (kin < 16 * KT) ? col_of(kin) : -1;
    if (r < 0 || c < 0) return 0.0;
    return Wf[(size_t)r * cols + c];
  };
  if (precision == TABNET_FP32) {
    for (int kt = kb_lo; kt < (kb_hi < 0 ? KT : kb_hi); ++kt)
      for (int lane = 0; lane < 64; ++lane) {
        const int i = lane & 15, q = lane >> 4;
        float v[4];
        for (int r = 0; r < 4; ++r) v[r] = (float)wv(i, 16 * kt + 4 * q + r);
        emit(wts, v, sizeof v);
      }
  } else if (precision == TABNET_MXFP8 || precision == TABNET_MXFP8_E5M2 || precision == TABNET_MXFP4 ||
             precision == TABNET_MXFP6 || precision == TABNET_MXFP6_E3M2) {
    // Per k-block of eight K tiles: the E8M0 exponent of each of an output row's four
    // blocks (block b = K tiles 2 b and 2 b + 1, i.e. 32 consecutive K positions), then the
    // elements lane by lane in the order the kernel's B operand has them, then the scale
    // each lane supplies (the instruction takes block b's scale from lane group b).  The
    // two 8-bit element forms share one layout, and so do the 6- and 4-bit forms.
    const bool f8 = precision == TABNET_MXFP8 || precision == TABNET_MXFP8_E5M2;
    const bool f6 = precision == TABNET_MXFP6 || precision == TABNET_MXFP6_E3M2;
    const int emax = precision == TABNET_MXFP8        ? 8     // E4M3
                     : precision == TABNET_MXFP8_E5M2 ? 15    // E5M2
                     : precision == TABNET_MXFP6_E3M2 ? 4     // E3M2
                                                      : 2;    // E2M3, E2M1
    uint8_t (*const enc8)(double) = precision == TABNET_MXFP8 ? e4m3_bits_rne : e5m2_bits_rne;
    uint8_t (*const enc6)(double) = precision == TABNET_MXFP6 ? e2m3_bits_rne : e3m2_bits_rne;
    const int KB = (KT + 7) / 8;
    // Element e of lane group q holds tile tt (of the k-block) and feature 4 s + i of it:
    //   8-bit: e < 16 block q / 2, e >= 16 block 2 + q / 2, lane group s = q % 2 + 2 ((e % 16) / 8);
    //   6-, 4-bit: block q, lane group s = e / 8;
    // tile tt = 2 block + (e % 8) / 4, i = e % 4.
    struct Slot {
      int tt, k;   // tile within the k-block, offset 4 s + i within the tile
    };
    auto slot = [&](int q, int e) {
      const int blk = f8 ? (e < 16 ? q / 2 : 2 + q / 2) : q;
      const int sg = f8 ? q % 2 + 2 * ((e % 16) / 8) : e / 8;
      return Slot{2 * blk + (e % 8) / 4, 4 * sg + e % 4};
    };
    auto val = [&](int i, int kb, Slot sl) {
      const int t = 8 * kb + sl.tt;
      return t < KT ? wv(i, 16 * t + sl.k) : 0.0;
    };
    for (int kb = kb_lo; kb < (kb_hi < 0 ? KB : kb_hi); ++kb) {
      int X[16][4];
      for (int i = 0; i < 16; ++i)
        for (int b = 0; b < 4; ++b) {
          double amax = 0;
          for (int p = 0; p < 32; ++p) amax = std::fmax(amax, std::fabs(val(i, kb, Slot{2 * b + p / 16, p % 16})));
          X[i][b] = mx_exponent(amax, emax);
        }
      auto code = [&](int i, int kb, Slot sl, auto enc) { return enc(std::ldexp(val(i, kb, sl), -X[i][sl.tt / 2])); };
      if (f8) {
        for (int half = 0; half < 2; ++half)
          for (int lane = 0; lane < 64; ++lane) {
            const int i = lane & 15, q = lane >> 4;
            uint8_t v[16];
            for (int e = 16 * half; e < 16 * half + 16; ++e) v[e - 16 * half] = code(i, kb, slot(q, e), enc8);
            emit(wts, v, sizeof v);
          }
      } else if (f6) {
        // 32 six-bit elements per lane, element e in bits 6 e .. 6 e + 5 of 24 bytes:
        // bytes 0-15 of every lane, then bytes 16-23 of every lane
        uint8_t bytes[64][24];
        for (int lane = 0; lane < 64; ++lane) {
          const int i = lane & 15, q = lane >> 4;
          uint64_t w[3] = {0, 0, 0};
          for (int e = 0; e < 32; ++e) {
            const uint64_t c = code(i, kb, slot(q, e), enc6);
            const int bit = 6 * e;
            w[bit / 64] |= c << (bit % 64);
            if (bit % 64 > 58) w[bit / 64 + 1] |= c >> (64 - bit % 64);
          }
          std::memcpy(bytes[lane], w, 24);
        }
        for (int lane = 0; lane < 64; ++lane) emit(wts, bytes[lane], 16);
        for (int lane = 0; lane < 64; ++lane) emit(wts, bytes[lane] + 16, 8);
      } else {
        for (int lane = 0; lane < 64; ++lane) {
          const int i = lane & 15, q = lane >> 4;
          uint8_t v[16] = {};
          for (int e = 0; e < 32; ++e) v[e / 2] |= (uint8_t)(code(i, kb, slot(q, e), e2m1_bits_rne) << (4 * (e & 1)));
          emit(wts, v, sizeof v);
        }
      }
      for (int lane = 0; lane < 64; ++lane) {
        const uint32_t sc = (uint32_t)(X[lane & 15][lane >> 4] + 127);
        emit(wts, &sc, sizeof sc);
      }
    }
  } else if (precision == TABNET_FP8_E4M3 || precision == TABNET_FP8_WEIGHTS) {
    // Wf holds E4M3 values of W' / s_n; byte j of a lane is tile 4 kb + j / 4
    const int KQ = (KT + 3) / 4;   // missing tiles of the last block are zeros
    for (int kb = kb_lo; kb < (kb_hi < 0 ? KQ : kb_hi); ++kb)
      for (int lane = 0; lane < 64; ++lane) {
        const int i = lane & 15, q = lane >> 4;
        uint8_t v[16];
        for (int j = 0; j < 16; ++j) {
          const int t = 4 * kb + j / 4;
          v[j] = e4m3_bits_rne(t < KT ? wv(i, 16 * t + 4 * q + (j & 3)) : 0.0);
        }
        emit(wts, v, sizeof v);
      }
  } else if (precision == TABNET_INT8) {
    const int KQ = (KT + 3) / 4;   // missing tiles of the last block are zeros
    for (int kb = kb_lo; kb < (kb_hi < 0 ? KQ : kb_hi); ++kb)
      for (int lane = 0; lane < 64; ++lane) {
        const int i = lane & 15, q = lane >> 4;
        int8_t v[16];
        for (int j = 0; j < 16; ++j) {
          const int t = 4 * kb + j / 4;
          v[j] = (int8_t)std::lrint(t < KT ? wv(i, 16 * t + 4 * q + (j & 3)) : 0.0);
        }
        emit(wts, v, sizeof v);
      }
  } else {
    const int KP = (KT + 1) / 2;   // an odd last tile is paired with a zero tile
    for (int kb = kb_lo; kb < (kb_hi < 0 ? KP : kb_hi); ++kb)
      for (int lane = 0; lane < 64; ++lane) {
        const int i = lane & 15, q = lane >> 4;
        uint16_t v[8];
        for (int j = 0; j < 8; ++j) {
          const int t = 2 * kb + j / 4;
          const double x = t < KT ? wv(i, 16 * t + 4 * q + (j & 3)) : 0.0;
          v[j] = bf16_bits_rne(x);
        }
        emit(wts, v, sizeof v);
      }
  }
}

// 16 per-output values (shifts or scales) of one tile; rows past rows_valid get `pad`.
void emit_vals(const std::vector<double>& bf, int rows_valid, int first_row, float pad,
               std::vector<unsigned char>* wts) {
  float v[16];
  for (int i = 0; i < 16; ++i) v[i] = i < rows_valid ? (float)bf[first_row + i] : pad;
  emit(wts, v, sizeof v);
}

// E4M3 with one scale per output row: s_n = max_k |W'_nk| / 448 (1 for a zero row),
// Wf <- E4M3(W' / s_n) (round to nearest even).  The shift is kept as it is: the kernel adds
// it after dequantising the products.  Rows [neg_lo, rows) (the gate half of a GLU layer)
// get their shift and scale multiplied by -log2(e), the factor of the sigmoid's exponent.
void quantize_rows_e4m3(std::vector<double>* Wf, std::vector<double>* bf, int rows, int cols, int neg_lo,
                        std::vector<double>* scale) {
  const double kNegLog2e = -1.4426950408889634;
  scale->assign(rows, 1.0);
  for (int r = 0; r < rows; ++r) {
    double amax = 0;
    for (int k = 0; k < cols; ++k) amax = std::fmax(amax, std::fabs((*Wf)[(size_t)r * cols + k]));
    const double s = amax > 0 ? amax / 448.0 : 1.0;
    for (int k = 0; k < cols; ++k) {
      double& w = (*Wf)[(size_t)r * cols + k];
      w = e4m3_value(e4m3_bits_rne(w / s));
    }
    (*scale)[r] = r >= neg_lo ? s * kNegLog2e : s;
    if (r >= neg_lo) (*bf)[r] *= kNegLog2e;
  }
}

// Split-feature layout (see Plan): feature-transformer layers as K slices holding every
// output pair, attentive layers as chunks holding tpc feature tiles of every wave.
void pack_wide(const ModelRaw& m, int precision, const Plan& plan, const Shape& sh,
               const std::vector<const LayerRaw*>& ft, Packed* out) {
  const tabnet_config& c = m.cfg;
  const int N = c.n_d + c.n_a;
  std::vector<double> Wf, bf;
  auto align = [&]() { out->wts.resize(align256(out->wts.size()), 0); };
  // K tiles per k-block: FP32 one, BF16 two, E4M3 and INT8 four (E4M3 weights with BF16
  // inputs are widened in the kernel), MX eight
  const bool w8 = precision == TABNET_FP8_WEIGHTS || precision == TABNET_FP8_E4M3;   // E4M3 weight codes
  const bool i8 = precision == TABNET_INT8;
  const bool cs = w8 || i8;   // one scale per output channel
  const int kbn = ktiles_per_block(precision);
  std::vector<double> sc;
  std::vector<std::vector<ChunkRec>> ft_chunks, att_chunks;
  for (size_t li = 0; li < ft.size(); ++li) {
    const LayerRaw* L = ft[li];
    // the first layer of a pass reads the D features (over the kernel's feature tiles)
    const bool reads_d = c.n_shared > 0 ? li == 0 : (li - (size_t)c.n_shared) % (size_t)c.n_indep == 0;
    fold_layer(*L, c.bn_eps, &Wf, &bf);
    if (w8) quantize_rows_e4m3(&Wf, &bf, L->rows, L->cols, N, &sc);   // rows [N, 2N): the gates
    if (i8) quantize_rows_int8(&Wf, &bf, L->rows, L->cols, N, &sc);
    const int KT = reads_d ? sh.DT : sh.NT;
    const int K = L->cols;
    const int KB = (KT + kbn - 1) / kbn;
    align();
    out->ft_off.push_back((int64_t)out->wts.size());
    std::vector<ChunkRec> chunks;
    for (int kb0 = 0; kb0 < KB; kb0 += plan.sk) {
      const int kb1 = std::min(KB, kb0 + plan.sk);
      const int64_t at = (int64_t)out->wts.size();
      for (int pr = 0; pr < sh.NT; ++pr)
        for (int half = 0; half < 2; ++half)
          emit_fragments(
              Wf, L->cols, KT, precision,
              [&](int i) { const int ch = 16 * pr + i; return ch < N ? half * N + ch : -1; },
              [&](int kin) { return kin < K ? kin : -1; }, &out->wts, kb0, kb1);
      if (kb1 == KB)
        for (int pr = 0; pr < sh.NT; ++pr) {
          const int nv = std::min(16, N - 16 * pr);
          emit_vals(bf, nv, 16 * pr, 0.f, &out->wts);
          emit_vals(bf, nv, N + 16 * pr, 0.f, &out->wts);
        }
      if (kb1 == KB && cs)   // then the channel scales, in the same order
        for (int pr = 0; pr < sh.NT; ++pr) {
          const int nv = std::min(16, N - 16 * pr);
          emit_vals(sc, nv, 16 * pr, 1.f, &out->wts);
          emit_vals(sc, nv, N + 16 * pr, 1.f, &out->wts);
        }
      chunks.push_back(ChunkRec{at, (int32_t)((int64_t)out->wts.size() - at), 0});
    }
    ft_chunks.push_back(chunks);
  }
  const int KTA = sh.NT - sh.KA0;
  for (const auto& L : m.att) {
    fold_layer(L, c.bn_eps, &Wf, &bf);
    if (w8) quantize_rows_e4m3(&Wf, &bf, L.rows, L.cols, L.rows, &sc);
    if (i8) quantize_rows_int8(&Wf, &bf, L.rows, L.cols, L.rows, &sc);
    align();
    out->att_off.push_back((int64_t)out->wts.size());
    std::vector<ChunkRec> chunks;
    for (int j = 0; j < plan.tpw / plan.tpc; ++j) {
      const int64_t at = (int64_t)out->wts.size();
      for (int w = 0; w < plan.W; ++w)
        for (int q = 0; q < plan.tpc; ++q) {
          const int mt = w * plan.tpw + j * plan.tpc + q;   // feature tile (past DT: zeros)
          emit_fragments(
              Wf, L.cols, KTA, precision,
              [&](int i) { const int d = 16 * mt + i; return d < c.D ? d : -1; },
              [&](int kin) { const int ch = 16 * sh.KA0 + kin; return (ch >= c.n_d && ch < N) ? ch - c.n_d : -1; },
              &out->wts);
          emit_vals(bf, std::max(0, std::min(16, c.D - 16 * mt)), 16 * mt, 0.f, &out->wts);
          if (cs) emit_vals(sc, std::max(0, std::min(16, c.D - 16 * mt)), 16 * mt, 1.f, &out->wts);
        }
      chunks.push_back(ChunkRec{at, (int32_t)((int64_t)out->wts.size() - at), 0});
    }
    att_chunks.push_back(chunks);
  }
  align();
  out->wfin.assign(m.w_fin, m.w_fin + (size_t)c.n_out * c.n_d);
  const int L = c.n_shared + c.n_indep;
  auto lid = [&](int s, int l) { return l < c.n_shared ? l : c.n_shared + s * c.n_indep + (l - c.n_shared); };
  for (int s = 0; s <= c.n_steps; ++s) {
    if (s > 0)
      for (const ChunkRec& r : att_chunks[s - 1]) out->chunks.push_back(r);
    for (int l = 0; l < L; ++l)
      for (const ChunkRec& r : ft_chunks[lid(s, l)]) out->chunks.push_back(r);
  }
}

}  // namespace

void pack_model(const ModelRaw& m, int precision, const Plan& plan, const Shape& sh, Packed* out) {
  const tabnet_config& c = m.cfg;
  const int N = c.n_d + c.n_a;
  const bool fp8 = precision == TABNET_FP8_E4M3 || precision == TABNET_FP8_WEIGHTS;
  const bool i8 = precision == TABNET_INT8;
  *out = Packed();
  // input BN as a per-column affine map
  out->in_affine.assign(32 * sh.DT, 0.f);
  for (int j = 0; j < c.D; ++j) {
    const double s = (double)m.bn_in.gamma[j] / std::sqrt((double)m.bn_in.var[j] + c.bn_eps);
    out->in_affine[j] = (float)s;
    out->in_affine[16 * sh.DT + j] = (float)((double)m.bn_in.beta[j] - s * (double)m.bn_in.mean[j]);
  }
  std::vector<const LayerRaw*> ft;
  for (const auto& L : m.shared) ft.push_back(&L);
  for (const auto& pass : m.indep)
    for (const auto& L : pass) ft.push_back(&L);
  std::vector<double> Wf, bf, sc;
  auto align = [&]() { out->wts.resize(align256(out->wts.size()), 0); };
  if (plan.wide) {
    pack_wide(m, precision, plan, sh, ft, out);
    return;
  }
  // GLU layers: unit mt = [value tile fragments][gate tile fragments][value shifts][gate shifts]
  // over the kernel's tiles (a generic kernel's extra feature tiles and hidden channels are
  // zero weights and shifts)
  for (size_t li = 0; li < ft.size(); ++li) {
    const LayerRaw* L = ft[li];
    // the first layer of a pass reads the D features: the first shared layer, or without
    // shared layers the first step layer of each pass
    const bool reads_d = c.n_shared > 0 ? li == 0 : (li - (size_t)c.n_shared) % (size_t)c.n_indep == 0;
    fold_layer(*L, c.bn_eps, &Wf, &bf);
    if (fp8) quantize_rows_e4m3(&Wf, &bf, L->rows, L->cols, N, &sc);     // rows [N, 2N): the gates
    if (i8) quantize_rows_int8(&Wf, &bf, L->rows, L->cols, N, &sc);   // rows [N, 2N): the gates
    const int KT = reads_d ? sh.DT : sh.NT;
    const int K = L->cols;
    align();
    out->ft_off.push_back((int64_t)out->wts.size());
    for (int mt = 0; mt < sh.NT; ++mt) {
      const size_t unit0 = out->wts.size();
      for (int half = 0; half < 2; ++half)
        emit_fragments(
            Wf, L->cols, KT, precision,
            [&](int i) { const int ch = 16 * mt + i; return ch < N ? half * N + ch : -1; },
            [&](int kin) { return kin < K ? kin : -1; }, &out->wts);
      const int nv = std::max(0, std::min(16, N - 16 * mt));
      emit_vals(bf, nv, 16 * mt, 0.f, &out->wts);
      emit_vals(bf, nv, N + 16 * mt, 0.f, &out->wts);
      if (fp8 || i8) {
        emit_vals(sc, nv, 16 * mt, 1.f, &out->wts);
        emit_vals(sc, nv, N + 16 * mt, 1.f, &out->wts);
      }
      (void)unit0;
    }
  }
  // attentive layers: unit mt = [fragments over the attention half of h][shifts]
  for (const auto& L : m.att) {
    fold_layer(L, c.bn_eps, &Wf, &bf);
    if (fp8) quantize_rows_e4m3(&Wf, &bf, L.rows, L.cols, L.rows, &sc);
    if (i8) quantize_rows_int8(&Wf, &bf, L.rows, L.cols, L.rows, &sc);
    const int KTA = sh.NT - sh.KA0;
    align();
    out->att_off.push_back((int64_t)out->wts.size());
    for (int mt = 0; mt < sh.DT; ++mt) {
      emit_fragments(
          Wf, L.cols, KTA, precision,
          [&](int i) { const int d = 16 * mt + i; return d < c.D ? d : -1; },
          [&](int kin) { const int ch = 16 * sh.KA0 + kin; return (ch >= c.n_d && ch < N) ? ch - c.n_d : -1; },
          &out->wts);
      emit_vals(bf, std::max(0, std::min(16, c.D - 16 * mt)), 16 * mt, 0.f, &out->wts);
      if (fp8 || i8) emit_vals(sc, std::max(0, std::min(16, c.D - 16 * mt)), 16 * mt, 1.f, &out->wts);
    }
  }
  align();
  out->wfin.assign(m.w_fin, m.w_fin + (size_t)c.n_out * c.n_d);
  // The weight stream, in the order the kernel consumes it: pass 0's layers, then per
  // step the attentive GEMM and that pass's layers.
  auto add = [&](int64_t base, const GemmPlan& gp) {
    for (int ch = 0; ch < gp.nchunks; ++ch) {
      const int units = std::min(gp.upc, gp.nunits - ch * gp.upc);
      out->chunks.push_back(ChunkRec{base + (int64_t)ch * gp.upc * gp.unit, units * gp.unit, 0});
    }
  };
  const int L = c.n_shared + c.n_indep;
  auto lid = [&](int s, int l) { return l < c.n_shared ? l : c.n_shared + s * c.n_indep + (l - c.n_shared); };
  for (int s = 0; s <= c.n_steps; ++s) {
    if (s > 0) add(out->att_off[s - 1], plan.att);
    for (int l = 0; l < L; ++l) add(out->ft_off[lid(s, l)], l == 0 ? plan.first : plan.mid);
  }
}

}  // namespace tabnet
