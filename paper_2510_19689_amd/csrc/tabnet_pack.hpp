// Load-time model preparation (host only): batch-norm folding in FP64, rounding to the
// GEMM operand precision, and packing into the MFMA fragment order the kernel reads.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/tabnet.h"
#include "tabnet_kernel.hpp"

namespace tabnet {

// One inference batch norm: y -> gamma (y - mean) / sqrt(var + eps) + beta.
struct BNRaw {
  const float *mean, *var, *gamma, *beta;
};
struct LayerRaw {        // W [rows][cols] row-major, then the BN of its rows
  const float* W;
  int rows, cols;
  BNRaw bn;
};
struct ModelRaw {
  tabnet_config cfg;
  std::vector<float> storage;     // the file's float32 payload
  BNRaw bn_in;
  std::vector<LayerRaw> shared;              // n_shared
  std::vector<std::vector<LayerRaw>> indep;  // n_steps + 1 passes x n_indep
  std::vector<LayerRaw> att;                 // n_steps
  const float* w_fin;                        // [n_out][n_d]
};

// Parses a TNW1 image.  Returns TABNET_OK or an error with *err set.
tabnet_status parse_model(const unsigned char* data, size_t len, ModelRaw* m, std::string* err);
int64_t model_param_count(const tabnet_config& c);
tabnet_status validate_config(const tabnet_config& c, std::string* err);

// Folded affine map of one FC+BN layer, in FP64:  y = W' u + b'.
void fold_layer(const LayerRaw& L, double eps, std::vector<double>* Wf, std::vector<double>* bf);

// Round-to-nearest-even of a double onto bfloat16 / E4M3FN (saturating at 448), as bits.
uint16_t bf16_bits_rne(double x);
uint8_t e4m3_bits_rne(double x);
// FP4 E2M1 bits of a double (round to nearest even, saturating at +-6), and the OCP MX
// shared exponent floor(log2 amax) - emax clamped to [-126, 127] (0 for amax = 0).
uint8_t e2m1_bits_rne(double x);
// FP6 E2M3 bits of a double (round to nearest even, saturating at +-7.5).
uint8_t e2m3_bits_rne(double x);
// FP8 E5M2 and FP6 E3M2 bits of a double (round to nearest even, saturating at +-57344
// and +-28).
uint8_t e5m2_bits_rne(double x);
uint8_t e3m2_bits_rne(double x);
int mx_exponent(double amax, int emax);
double bf16_value(uint16_t bits);
double e4m3_value(uint8_t bits);

// Symmetric INT8 coding of each row of Wf [rows][cols] in place (codes as doubles), one
// scale per row into *scale; rows from neg_lo on (a GLU layer's gates) get their shift in
// *bf and their scale multiplied by -log2(e).
void quantize_rows_int8(std::vector<double>* Wf, std::vector<double>* bf, int rows, int cols, int neg_lo,
                        std::vector<double>* scale);

// Kernel shape: tiles of 16 features.
struct Shape {
  int DT, NT, KA0;
};
Shape shape_of(const tabnet_config& c);

// Packed image of a whole model for one precision.
struct Packed {
  std::vector<unsigned char> wts;   // GEMM units (fragments + shifts), 256-byte aligned per GEMM
  std::vector<ChunkRec> chunks;     // weight-stream chunks in the kernel's consumption order
  std::vector<float> in_affine;     // [2][16 DT]: input-BN scale, then shift
  std::vector<float> wfin;          // [n_out][n_d]
  std::vector<int64_t> ft_off;      // per unique feature-transformer layer
  std::vector<int64_t> att_off;     // per step
};
// Packs the model for `precision` in the chunk layout of `plan` (the kernel's plan) and
// the kernel's tiles `sh` (the model's own shape, or larger for a generic kernel).
void pack_model(const ModelRaw& m, int precision, const Plan& plan, const Shape& sh, Packed* out);

}  // namespace tabnet
