// Fused TabNet inference kernel for gfx950 (MI355X).
//
// One launch runs the whole forward for a batch.  Each wavefront owns R blocks of 16
// rows and carries them through every decision step without leaving registers:
//
//   input BN (per-column affine)           -> x, P = 1
//   feature-transformer pass 0             -> a
//   for each step i:
//     attentive FC (+folded BN) on MFMA    -> h_att;  z = P * h_att
//     sparsemax(z) per row                 -> M_i   (written to masks_step)
//     P <- P * (gamma - M_i);  u = M_i * x
//     feature-transformer pass i on MFMA   -> h = [d | a]
//     acc += ReLU(d);  eta = sum ReLU(d);  agg += eta * M_i
//   logits = acc W_fin^T;  masks_agg = agg / sum(agg)
//
// TabNet is the model the paper deploys and cites (Sec. I, Sec. II-B, with the step
// structure of Sec. IV-A); the masks are the audit output of Sec. III-B / Sec. V-C.
//
// Matrix-core mapping.  Every GEMM is computed transposed, out^T = W' * act^T, with the
// folded weights as the MFMA A operand and 16 batch rows as the B/C columns.  In the
// 16x16 C layout a lane holds batch row (lane % 16) and output features
// 16 t + 4 (lane / 16) + {0..3} of tile t.  The next GEMM's B operand wants, per lane,
// the same batch row and a run of K values; the host packs the A fragments with their
// K slots permuted to exactly the features the lane already holds, so a layer's output
// feeds the next layer (and the sparsemax, the prior, the masks) with no data movement
// between lanes.  A row's D features are spread over the 4 lanes {r, r+16, r+32, r+48};
// row reductions are in-lane sums plus two cross-lane exchanges.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tabnet {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef short s4 __attribute__((ext_vector_type(4)));

constexpr int kMaxFtLayers = 96;   // n_shared + (n_steps + 1) * n_indep
constexpr int kMaxSteps = 32;
constexpr int kWaves = 4;          // wavefronts per workgroup

// Byte offsets into the packed weight blob and float offsets into the bias blob.
struct LayerTable {
  int64_t w[kMaxFtLayers];
  int32_t b[kMaxFtLayers];
  int64_t aw[kMaxSteps];
  int32_t ab[kMaxSteps];
};

struct FwdArgs {
  const float* X;
  float* logits;
  float* masks_agg;
  float* masks_step;          // may be null
  const unsigned char* wts;   // packed GEMM weights
  const float* bias;          // folded shifts (and per-channel scales), C-layout order
  const float* in_affine;     // [2][16*DT]: input BN scale then shift, zero-padded
  const float* wfin;          // [n_out][n_d] float32
  int64_t B;
  int D, n_d, n_a, n_steps, n_sh, n_ind, n_out;
  float gamma;
  LayerTable lt;
};

}  // namespace tabnet
