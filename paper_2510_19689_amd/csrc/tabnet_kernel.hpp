// Fused TabNet inference kernel for gfx950 (MI355X): shared definitions of the kernel
// and of the host code that packs weights for it.
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
//
// Weight stream.  The weights are the same for every row, so a workgroup of W waves
// streams them through LDS once for all its rows: the packed GEMM weights are cut into
// chunks, listed on the host in the order the kernel consumes them, and a double buffer
// overlaps the global fetch of chunk c+1 with the MFMAs on chunk c.
//
// Packed layout of one GEMM (each starts 256-byte aligned), as a sequence of units:
//   GLU layer, unit mt = 0..NT-1:  [value-tile fragments][gate-tile fragments]
//                                  [16 value shifts][16 gate shifts]
//                                  (E4M3, INT8, E4M3 weights: then [16 value scales]
//                                  [16 gate scales])
//   attentive, unit mt = 0..DT-1:  [fragments][16 shifts] (with channel scales: then
//                                  [16 scales])
// A fragment is 64 lanes x 16 bytes: FP32 one per 16-wide K tile (a lane's float4 feeds
// four 16x16x4 MFMAs), BF16 one per pair of K tiles (8 bf16 per lane, one 16x16x32 MFMA;
// an odd last tile is paired with zeros), E4M3 and INT8 one per four K tiles (16 codes per
// lane: two 16x16x32 FP8 MFMAs, one 16x16x64 integer MFMA, or for E4M3 weights with BF16
// inputs two 16x16x32 BF16 MFMAs on codes widened to BF16; missing tiles are zeros).
// Shifts are in C-layout order: slot 4 q + i of tile mt is output feature 16 mt + 4 q + i.
// With channel scales the gate half's shifts and scales are stored multiplied by -log2(e),
// the factor of the sigmoid's exponent, and the shifts are not divided by the scales (the
// products of codes are dequantised before the shift is added).
// MX formats (OCP microscaling: blocks of 32 consecutive K positions share a power-of-two
// E8M0 scale) take eight K tiles per k-block, one 16x16x128 scaled MFMA; block b of a
// k-block is tiles 2 b and 2 b + 1.  MXFP8 (E4M3 or E5M2 elements) packs per k-block
// [64 lanes x 16 B: elements 0-15][64 x 16 B: elements 16-31][64 x 4 B: the E8M0 scale
// each lane supplies, in byte 0]; MXFP6 (E2M3 or E3M2) packs [64 x 16 B: bytes 0-15]
// [64 x 8 B: bytes 16-23 of 32 six-bit elements, element e in bits 6 e .. 6 e + 5]
// [64 x 4 B: scales]; MXFP4 packs [64 x 16 B: 32 E2M1 elements, element e in nibble e]
// [64 x 4 B: scales].  The instruction takes block b's scale from lane group b, and the
// kernel moves each block's elements to the lane groups the instruction reads them from
// (exchanges within a row's 4 lanes).  Element e of lane group q holds tile 2 blk + h of
// the k-block and feature 4 s + i of that tile, with i = e % 4, h = (e % 8) / 4 and
//   MXFP6, MXFP4: blk = q, s = e / 8 (lane group q holds instruction slots 32 q + e);
//   MXFP8: blk = q / 2 (e < 16) or 2 + q / 2 (e >= 16), s = q % 2 + 2 ((e % 16) / 8)
//          (lane group q holds slots 16 q + e for e < 16 and 64 + 16 q + e - 16).
// The scales are applied inside the instruction, so MX units carry shifts only.
#pragma once
#include <stdint.h>

namespace tabnet {

constexpr int kMaxFtLayers = 96;   // n_shared + (n_steps + 1) * n_indep
constexpr int kMaxSteps = 32;
constexpr int kFrag = 1024;        // bytes of one A fragment
constexpr int kMaxLdsBytes = 160 * 1024;   // LDS of one workgroup on gfx950
constexpr int kChunkTarget = 40960;

struct ChunkRec {
  int64_t off;     // byte offset into the packed weights
  int32_t bytes;   // multiple of 16
  int32_t pad;
};

struct GemmPlan {
  int unit;      // bytes per unit (one output tile, or value+gate tile pair)
  int nunits;
  int upc;       // units per chunk
  int nchunks;
};

// MX precisions by element width: 8-bit (E4M3, E5M2) and 6-bit (E2M3, E3M2) elements
constexpr bool is_mx8(int prec) { return prec == 4 || prec == 7; }
constexpr bool is_mx6(int prec) { return prec == 6 || prec == 8; }
// MX precisions (scaled matrix instruction)
constexpr bool is_mx(int prec) { return prec >= 4 && prec <= 8; }
// E4M3 weights with BF16 GEMM inputs (the codes are widened to BF16 for the BF16 MFMA)
constexpr bool is_fp8w(int prec) { return prec == 9; }
// K tiles per k-block: 1 (FP32), 2 (BF16), 4 (E4M3, INT8, E4M3 weights), 8 (every MX format)
constexpr int ktiles_per_block(int prec) { return prec == 0 ? 1 : (prec == 1 ? 2 : (is_mx(prec) ? 8 : 4)); }
constexpr int kblocks(int prec, int KT) {
  return (KT + ktiles_per_block(prec) - 1) / ktiles_per_block(prec);
}
// Bytes of one k-block of one output tile: a fragment, or the MX elements and scales.
constexpr int kMxScaleBytes = 256;
constexpr int kbytes(int prec) {
  return is_mx8(prec) ? 2 * kFrag + kMxScaleBytes
                      : (prec == 5 ? kFrag + kMxScaleBytes : (is_mx6(prec) ? kFrag + kFrag / 2 + kMxScaleBytes : kFrag));
}
// Per-output scales after the shifts (E4M3, INT8, E4M3 weights)
constexpr bool has_channel_scales(int prec) { return prec == 2 || prec == 3 || prec == 9; }
// GEMM inputs coded per row in the kernel (E4M3, INT8)
constexpr bool row_coded(int prec) { return prec == 2 || prec == 3; }
constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// Units per chunk: balanced chunks of at most `target` bytes (one unit if a single unit
// is larger).
constexpr GemmPlan gemm_plan(int unit, int nunits, int target) {
  const int nch0 = cdiv(unit * nunits, target);
  int upc = cdiv(nunits, nch0 < 1 ? 1 : nch0);
  const int cap = target / unit < 1 ? 1 : target / unit;
  if (upc > cap) upc = cap;
  return GemmPlan{unit, nunits, upc, cdiv(nunits, upc)};
}

// Bytes of one LDS weight buffer for a workgroup of W waves of R 16-row blocks: at most
// kChunkTarget, and small enough that the two buffers fit beside the per-wave mask
// staging areas (W * 16 R rows of up to 16 DT features) with 8 KiB left for the final
// map and the raw-row maps (4 D feature descriptors and an n_out x n_d map: 5.7 KiB at
// D = 208, n_d = 79 and 8 outputs).
constexpr int chunk_target(int DT, int R, int W) {
  const int room = (kMaxLdsBytes - W * 16 * R * 16 * DT * 4 - 8192) / 2 / 1024 * 1024;
  return room < kChunkTarget ? (room < 8192 ? 8192 : room) : kChunkTarget;
}

struct Plan {
  GemmPlan first, mid, att;
  int buf;       // bytes of one LDS weight buffer
  // Split-feature kernels (wide models): the features of one 16-row block are shared out
  // over the W waves of a workgroup.  A feature-transformer layer streams K slices of sk
  // k-blocks; a slice chunk holds, for every output tile pair, [value fragments][gate
  // fragments] of those k-blocks, and the layer's last slice adds the shifts of all pairs
  // ([pair][16 value | 16 gate] floats; with channel scales then the scales the same way).
  // An attentive chunk holds, for every wave, tpc of its feature tiles as [fragments][16
  // shifts] (with channel scales: then [16 scales]) units of att_unit bytes.
  int wide = 0;
  int W = 0, tpw = 0, sk = 0, tpc = 0, att_unit = 0;
};

constexpr int imax(int a, int b) { return a > b ? a : b; }

// prec: 0 FP32, 1 BF16, 2 E4M3 and 3 INT8 weights and activations (codes in the fragments,
// one FP32 scale per output channel after the shifts, one scale per input row formed in
// the kernel), 4 MXFP8, 5 MXFP4, 6 MXFP6, 7 MXFP8 with E5M2 elements and 8 MXFP6 with E3M2
// elements (weights and activations in OCP MX blocks), 9 E4M3 weights (one scale per
// output channel) with BF16 GEMM inputs.  DT = ceil(D/16), NT = ceil(N/16),
// KA0 = floor(n_d/16).
constexpr Plan make_plan(int prec, int DT, int NT, int KA0, int target) {
  const int sc = has_channel_scales(prec) ? 2 : 1;   // shifts, or shifts + scales
  const GemmPlan first = gemm_plan(2 * kblocks(prec, DT) * kbytes(prec) + 128 * sc, NT, target);
  const GemmPlan mid = gemm_plan(2 * kblocks(prec, NT) * kbytes(prec) + 128 * sc, NT, target);
  const GemmPlan att = gemm_plan(kblocks(prec, NT - KA0) * kbytes(prec) + 64 * sc, DT, target);
  const int buf = imax(first.upc * first.unit, imax(mid.upc * mid.unit, att.upc * att.unit));
  return Plan{first, mid, att, buf};
}

// Weight bytes of one K slice of the split-feature kernel, in KiB (plus the shifts).
constexpr int kWideSliceKib = 32;
// Split-feature plan: wave w owns feature tiles [w tpw, (w + 1) tpw) of the padded row
// (tpw even, so that BF16 tile pairs never straddle waves) and output tile pairs
// [w NT / W, (w + 1) NT / W) of every feature-transformer layer.
constexpr int wide_tpw(int DT, int W) { return (cdiv(DT, W) + 1) / 2 * 2; }
constexpr int wide_slice_bytes(int prec, int NT, int nkb, bool last) {
  return NT * 2 * nkb * kbytes(prec) + (last ? NT * 128 * (has_channel_scales(prec) ? 2 : 1) : 0);
}
constexpr Plan make_wide_plan(int prec, int DT, int NT, int KA0, int W) {
  Plan p{};
  p.wide = 1;
  p.W = W;
  p.tpw = wide_tpw(DT, W);
  constexpr int kib = kWideSliceKib;
  const int sk = kib * 1024 / (2 * NT * kbytes(prec));
  p.sk = sk < 1 ? 1 : sk;   // k-blocks per slice
  p.att_unit = kblocks(prec, NT - KA0) * kbytes(prec) + 64 * (has_channel_scales(prec) ? 2 : 1);
  int tpc = p.tpw;
  while (tpc > 1 && (W * tpc * p.att_unit > kib * 1024 + NT * 128 || p.tpw % tpc != 0)) --tpc;
  p.tpc = tpc;
  const int kbf = kblocks(prec, DT), kbm = kblocks(prec, NT);
  int buf = W * tpc * p.att_unit;
  buf = imax(buf, wide_slice_bytes(prec, NT, kbf < p.sk ? kbf : p.sk, true));
  buf = imax(buf, wide_slice_bytes(prec, NT, kbm < p.sk ? kbm : p.sk, true));
  p.buf = buf;
  // GemmPlan fields describe the chunk counts per GEMM (units are not used)
  p.first = GemmPlan{0, 0, 0, cdiv(kbf, p.sk)};
  p.mid = GemmPlan{0, 0, 0, cdiv(kbm, p.sk)};
  p.att = GemmPlan{0, 0, 0, p.tpw / tpc};
  return p;
}

struct FwdArgs {
  const float* X;
  float* logits;
  float* masks_agg;
  float* masks_step;          // may be null
  const unsigned char* wts;   // packed GEMM units
  const ChunkRec* chunks;     // consumption order
  const float* in_affine;     // [2][16*DT]: input BN scale then shift, zero-padded
  const float* wfin;          // [n_out][n_d] float32
  int64_t B;                  // rows (grid size); the live count if B_dev is null
  const int64_t* B_dev;       // if set: live row count in device memory, <= B
  int D, n_d, n_a, n_steps, n_sh, n_ind, n_out, n_chunks;
  float gamma;
  // Raw rows (the RAW kernels): X is [B, C] raw columns, embedded on the fly, and both
  // masks are written per raw column ([B, C] and [S, B, C]).
  const int* emb_meta;        // [D][4]: raw column, levels (0: continuous), table offset, width
  const float* emb_tables;    // the categorical columns' tables, concatenated
  int C;
  int tab_len;                // floats in emb_tables
  int tab_lds;                // 1: the kernel copies the tables into LDS
  const uint64_t* colbits;    // [ceil(C/16)][64]: per lane, its features' membership in column 16 ct + lane % 16
};

}  // namespace tabnet
