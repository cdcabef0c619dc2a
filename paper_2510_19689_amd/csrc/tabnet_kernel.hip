// Fused TabNet inference kernel for gfx950.  Layout and data flow: tabnet_kernel.hpp.
#include <hip/hip_runtime.h>

#include "tabnet_handle.hpp"
#include "tabnet_kernel.hpp"

namespace tabnet {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef int i4 __attribute__((ext_vector_type(4)));
typedef int i8v __attribute__((ext_vector_type(8)));

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kSqrtHalf = 0.70710678118654752f;
constexpr float kNegBig = -3.0e38f;   // score of a padded feature: never in the support

// Cross-lane pairs on the VALU: v_permlane16_swap exchanges rows (16 lanes) 0<->1 and
// 2<->3, v_permlane32_swap the two halves of the wave.  Called with the same value as
// both operands, the two results hold {own, partner} in an order that depends on the
// lane, so their sum (or max) is the pair's sum (max), formed in the same operand order
// in both lanes of the pair: the four lanes of a row end with bit-identical results.
__device__ __forceinline__ float pair16_sum(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float pair32_sum(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float pair16_max(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}
__device__ __forceinline__ float pair32_max(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}
__device__ __forceinline__ int pair16_sum(int v) {
  const auto r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
  return (int)(r[0] + r[1]);
}
__device__ __forceinline__ int pair32_sum(int v) {
  const auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
  return (int)(r[0] + r[1]);
}

// The value held by the partner lane (lane ^ 16, lane ^ 32).
__device__ __forceinline__ float partner16(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float((threadIdx.x & 16) ? r[0] : r[1]);
}
__device__ __forceinline__ float partner32(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float((threadIdx.x & 32) ? r[0] : r[1]);
}

// Sum / max over the 4 lanes {r, r+16, r+32, r+48} that hold one row.
__device__ __forceinline__ float row_sum(float v) { return pair32_sum(pair16_sum(v)); }
__device__ __forceinline__ int row_sum(int v) { return pair32_sum(pair16_sum(v)); }
__device__ __forceinline__ float row_max(float v) { return pair32_max(pair16_max(v)); }

// Two floats -> two bfloat16 (round to nearest even) packed low/high in one dword.
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
  typedef float fl2 __attribute__((ext_vector_type(2)));
  fl2 f = {lo, hi};
  bf2 b = __builtin_convertvector(f, bf2);
  return __builtin_bit_cast(uint32_t, b);
}

// Compare-exchange: a <- max, b <- min.
__device__ __forceinline__ void cex(float& a, float& b) {
  const float hi = fmaxf(a, b), lo = fminf(a, b);
  a = hi;
  b = lo;
}

// The 8 values {t1, t2} of the row's 4 lanes (t1 >= t2 in each), sorted descending into
// v[0..7], identically in all 4 lanes: merge pairs across lanes 16 apart into sorted
// quadruples, then quadruples across lanes 32 apart by a bitonic merge.
__device__ __forceinline__ void top8_sorted(float t1, float t2, float (&v)[8]) {
  const float u1 = partner16(t1), u2 = partner16(t2);
  float q[4];
  q[0] = fmaxf(t1, u1);
  q[3] = fminf(t2, u2);
  float m1 = fminf(t1, u1), m2 = fmaxf(t2, u2);
  q[1] = fmaxf(m1, m2);
  q[2] = fminf(m1, m2);
  // bitonic sequence: own quadruple descending, partner's ascending
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = q[k];
    v[7 - k] = partner32(q[k]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) cex(v[k], v[k + 4]);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    cex(v[k], v[k + 2]);
    cex(v[k + 4], v[k + 6]);
  }
#pragma unroll
  for (int k = 0; k < 8; k += 2) cex(v[k], v[k + 1]);
}

// logistic(g) = 1 / (1 + 2^(-g log2 e))
__device__ __forceinline__ float sigmoid_fast(float g) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-g * kLog2e));
}

// LDS writes by this wave are complete (cross-lane reuse inside the wave).
__device__ __forceinline__ void lds_wave_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }
// LDS writes of every wave are complete and every wave has arrived.  Global memory
// operations stay in flight (no vmcnt wait), so the weight prefetch keeps overlapping.
__device__ __forceinline__ void lds_block_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// ------------------------------------------------------------------------------------
// B operands: a lane's 4 consecutive features of each 16-feature tile, per row block.
template <int PREC, int KT, int R>
struct BOp;

template <int KT, int R>
struct BOp<0, KT, R> {        // FP32: the values themselves
  float v[R][KT][4];
  __device__ __forceinline__ void set(int rb, int t, const float (&x)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) v[rb][t][i] = x[i];
  }
};
template <int KT, int R>
struct BOp<1, KT, R> {        // BF16: two packed dwords per tile
  uint32_t v[R][KT][2];
  __device__ __forceinline__ void set(int rb, int t, const float (&x)[4]) {
    v[rb][t][0] = pack_bf16x2(x[0], x[1]);
    v[rb][t][1] = pack_bf16x2(x[2], x[3]);
  }
};

// E4M3 weights with BF16 inputs: the BF16 operand, and a row scale of 1 (the inputs are
// not scaled).
template <int KT, int R>
struct BOp<9, KT, R> : BOp<1, KT, R> {
  __device__ __forceinline__ float rscale(int) const { return 1.f; }
};

// E4M3 (the FP8 path): one scale per row, s = max_k |u_k| / 448, elements u_k / s rounded
// to nearest even in E4M3, four to a dword (feature 16 t + 4 g + i in byte i).  The
// largest element maps to 448 (|u * 448 / max| <= 448 (1 + 2^-23) rounds to 448), so no
// element leaves the E4M3 range.
template <int KT, int R>
struct BOp<2, KT, R> {
  uint32_t v[R][KT];
  float s[R];
  __device__ __forceinline__ float rscale(int rb) const { return s[rb]; }
  template <class F>
  __device__ __forceinline__ void build(F src) {
#pragma unroll
    for (int rb = 0; rb < R; ++rb) {
      float m0 = 0.f, m1 = 0.f;
#pragma unroll
      for (int t = 0; t < KT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (i & 1) m1 = fmaxf(m1, fabsf(src(rb, t, i)));
          else m0 = fmaxf(m0, fabsf(src(rb, t, i)));
        }
      const float amax = row_max(fmaxf(m0, m1));
      s[rb] = amax * (1.0f / 448.0f);
      const float inv = amax > 0.f ? 448.0f / amax : 0.f;
#pragma unroll
      for (int t = 0; t < KT; ++t) {
        int w = __builtin_amdgcn_cvt_pk_fp8_f32(src(rb, t, 0) * inv, src(rb, t, 1) * inv, 0, false);
        w = __builtin_amdgcn_cvt_pk_fp8_f32(src(rb, t, 2) * inv, src(rb, t, 3) * inv, w, true);
        v[rb][t] = (uint32_t)w;
      }
    }
  }
};

// INT8: symmetric codes with one step per row, s = max_k |u_k| / 127, c_k = round(u_k / s)
// (ties to even), four codes of a tile in one dword (feature 16 t + 4 g + i in byte i).
// The row maximum is the lane's own maximum and two cross-lane exchanges.  A code is
// formed by one FMA: u * (127 / max) + 1.5 * 2^23 rounds the exact product to an integer
// (ties to even) held in the low mantissa bits, whose low byte is the two's-complement
// code, since |u * 127 / max| <= 127.5 keeps the sum inside [2^23, 2^24).
template <int KT, int R>
struct BOp<3, KT, R> {
  uint32_t v[R][KT];
  float s[R];                 // the row's step (0 for an all-zero row)
  __device__ __forceinline__ float rscale(int rb) const { return s[rb]; }
  template <class F>
  __device__ __forceinline__ void build(F src) {
    constexpr float kRound = 12582912.0f;   // 1.5 * 2^23
#pragma unroll
    for (int rb = 0; rb < R; ++rb) {
      float m0 = 0.f, m1 = 0.f;
#pragma unroll
      for (int t = 0; t < KT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (i & 1) m1 = fmaxf(m1, fabsf(src(rb, t, i)));
          else m0 = fmaxf(m0, fabsf(src(rb, t, i)));
        }
      const float amax = row_max(fmaxf(m0, m1));
      s[rb] = amax * (1.0f / 127.0f);
      const float inv = amax > 0.f ? 127.0f / amax : 0.f;
#pragma unroll
      for (int t = 0; t < KT; ++t) {
        uint32_t c[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = __float_as_uint(__builtin_fmaf(src(rb, t, i), inv, kRound));
        // v_perm_b32: byte k of the result is byte sel_k of {src0 (bytes 4-7), src1 (bytes 0-3)}
        const uint32_t lo = __builtin_amdgcn_perm(c[1], c[0], 0x0c0c0400u);
        const uint32_t hi = __builtin_amdgcn_perm(c[3], c[2], 0x0c0c0400u);
        v[rb][t] = __builtin_amdgcn_perm(hi, lo, 0x05040100u);
      }
    }
  }
};

// OCP MX shared exponent of a block whose largest magnitude is amax: floor(log2 amax)
// minus the element format's emax, clamped to [-126, 127] (0 for a block of zeros).
template <int EMAX>
__device__ __forceinline__ int mx_exponent(float amax) {
  const int X = __builtin_amdgcn_frexp_expf(amax) - 1 - EMAX;   // amax = m 2^e, m in [0.5, 1)
  return amax > 0.f ? (X < -126 ? -126 : (X > 127 ? 127 : X)) : 0;
}

// MX blocks.  A k-block is eight K tiles (128 K positions, one scaled MFMA); its OCP MX
// blocks are the four runs of 32 consecutive K positions, block b = tiles 2 b and 2 b + 1.
// A lane holds 8 elements of every block (its features 4 g + i of both tiles), so a
// block's scale is the maximum over the row's 4 lanes, and the instruction's lane groups
// receive their blocks by exchanges within the row's 4 lanes (v_permlane16_swap,
// v_permlane32_swap; the order of the 8-element chunks inside a block is the one the host
// packs the weights with).
//
// Shared exponents of the four blocks of k-block kb.  Each lane takes the maxima of its
// 8 elements of every block; a reduce-scatter over the row's 4 lanes (one exchange with
// the lane 32 away, one with the lane 16 away) leaves lane group q the maximum of block q,
// whose exponent X_q it forms; an all-gather of the biased exponents X_q + 127 (bytes)
// gives every lane all four.  Returns the four biased exponents in bytes 0..3 and the
// lane's own (block q = its lane group) in *own.
template <int KT, int EMAX, class F>
__device__ __forceinline__ uint32_t mx_block_exponents(F src, int rb, int kb, uint32_t* own) {
  float m[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    float a0 = 0.f, a1 = 0.f;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = 8 * kb + 2 * b + h;
      if (t < KT)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (i & 1) a1 = fmaxf(a1, fabsf(src(rb, t, i)));
          else a0 = fmaxf(a0, fabsf(src(rb, t, i)));
        }
    }
    m[b] = fmaxf(a0, a1);
  }
  // lanes 0-31 reduce blocks 0, 1 and lanes 32-63 blocks 2, 3 over the pair 32 apart ...
  float p[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(m[k]), __float_as_uint(m[k + 2]), false, false);
    p[k] = fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
  }
  // ... then even lane groups block 2 j and odd ones block 2 j + 1 over the pair 16 apart
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(p[0]), __float_as_uint(p[1]), false, false);
  const uint32_t e = (uint32_t)(mx_exponent<EMAX>(fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]))) + 127);
  *own = e;
  // all-gather: a pair 16 apart returns blocks (2 j, 2 j + 1) in the order (even, odd)
  const auto a = __builtin_amdgcn_permlane16_swap(e, e, false, false);
  const uint32_t w = a[0] | (a[1] << 8);
  const auto c = __builtin_amdgcn_permlane32_swap(w, w, false, false);
  return c[0] | (c[1] << 16);
}

// 2^(X_b) from the biased exponent in byte b (an E8M0 scale is an FP32 exponent field).
__device__ __forceinline__ float mx_scale_of(uint32_t e4, int b) {
  return __uint_as_float(((e4 >> (8 * b)) & 0xffu) << 23);
}

// MXFP8 (E4M3 elements, E5M2 when E5M2 is set).  The instruction's lane group q holds
// instruction slots 16 q .. 16 q + 15 (dwords 0-3) and 64 + 16 q .. 64 + 16 q + 15 (dwords
// 4-7), and takes block b's scale from lane group b; slots 32 b' .. 32 b' + 31 share a
// scale.  So lane groups 0 and 1 carry halves of blocks 0 and 2, groups 2 and 3 halves of
// blocks 1 and 3: lane group q holds, in dwords 0-3, the elements of block q / 2 from lane
// groups q % 2 (dwords 0-1) and q % 2 + 2 (dwords 2-3), and in dwords 4-7 the same for
// block 2 + q / 2.  Each lane codes its 8 elements of every block (dword 2 h: tile 2 b + h,
// element i in byte i), keeps two blocks and swaps the other two with the lane 32 away.
// Elements are v / 2^X, clamped to the largest normal (+-448, E5M2 +-57344) and rounded
// to nearest even.
template <int KT, int R, bool E5M2>
struct MxF8Op {
  static constexpr int KB = kblocks(4, KT);
  uint32_t v[R][KB][8];
  uint32_t sc[R][KB];
  template <class F>
  __device__ __forceinline__ void build(F src) {
    constexpr int kEmax = E5M2 ? 15 : 8;
    constexpr float kMax = E5M2 ? 57344.0f : 448.0f;
#pragma unroll
    for (int rb = 0; rb < R; ++rb)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        uint32_t own;
        const uint32_t e4 = mx_block_exponents<KT, kEmax>(src, rb, kb, &own);
        uint32_t w[4][2];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const float scale = mx_scale_of(e4, b);
          const float lim = kMax * scale;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int t = 8 * kb + 2 * b + h;
            w[b][h] = 0u;
            if (t < KT) {
              float c[4];
#pragma unroll
              for (int i = 0; i < 4; ++i) c[i] = __builtin_amdgcn_fmed3f(src(rb, t, i), -lim, lim);
              typedef short sh2 __attribute__((ext_vector_type(2)));
              sh2 q = {0, 0};
              if constexpr (E5M2) {
                q = __builtin_amdgcn_cvt_scalef32_pk_bf8_f32(q, c[0], c[1], scale, false);
                q = __builtin_amdgcn_cvt_scalef32_pk_bf8_f32(q, c[2], c[3], scale, true);
              } else {
                q = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(q, c[0], c[1], scale, false);
                q = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(q, c[2], c[3], scale, true);
              }
              w[b][h] = __builtin_bit_cast(uint32_t, q);
            }
          }
        }
        // lanes 0-31 keep blocks 0 and 2 and receive them from the lane 32 away; lanes
        // 32-63 keep blocks 1 and 3 and receive those
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const auto r = __builtin_amdgcn_permlane32_swap(w[2 * p][h], w[2 * p + 1][h], false, false);
            v[rb][kb][4 * p + h] = r[0];
            v[rb][kb][4 * p + 2 + h] = r[1];
          }
        sc[rb][kb] = own;
      }
  }
};
template <int KT, int R>
struct BOp<4, KT, R> : MxF8Op<KT, R, false> {};
template <int KT, int R>
struct BOp<7, KT, R> : MxF8Op<KT, R, true> {};

// MXFP4 (E2M1 elements).  The instruction's lane group q holds slots 32 q .. 32 q + 31,
// block q, and supplies its scale.  Each lane codes its 8 elements of every block into
// one dword (nibble 4 h + i: tile 2 b + h, element i), and a 4 x 4 transpose over the
// row's 4 lanes (one exchange with the lane 32 away, one with the lane 16 away) gives lane
// group q dword s = lane group s's 8 elements of block q.  Elements are v / 2^X rounded
// to nearest even, saturating at +-6.
template <int KT, int R>
struct BOp<5, KT, R> {
  static constexpr int KB = kblocks(5, KT);
  uint32_t v[R][KB][4];
  uint32_t sc[R][KB];
  template <class F>
  __device__ __forceinline__ void build(F src) {
#pragma unroll
    for (int rb = 0; rb < R; ++rb)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        uint32_t own;
        const uint32_t e4 = mx_block_exponents<KT, 2>(src, rb, kb, &own);
        uint32_t w[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const float scale = mx_scale_of(e4, b);
          uint32_t q = 0u;
          const int t0 = 8 * kb + 2 * b, t1 = t0 + 1;
          if (t0 < KT) {
            q = __builtin_amdgcn_cvt_scalef32_pk_fp4_f32(q, src(rb, t0, 0), src(rb, t0, 1), scale, 0);
            q = __builtin_amdgcn_cvt_scalef32_pk_fp4_f32(q, src(rb, t0, 2), src(rb, t0, 3), scale, 1);
          }
          if (t1 < KT) {
            q = __builtin_amdgcn_cvt_scalef32_pk_fp4_f32(q, src(rb, t1, 0), src(rb, t1, 1), scale, 2);
            q = __builtin_amdgcn_cvt_scalef32_pk_fp4_f32(q, src(rb, t1, 2), src(rb, t1, 3), scale, 3);
          }
          w[b] = q;
        }
        // transpose: [w0 w1 w2 w3] of lane group s (block b in w_b) -> lane group q holds
        // [block q of groups 0, 1, 2, 3]
        uint32_t t4[4];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const auto r = __builtin_amdgcn_permlane32_swap(w[k], w[k + 2], false, false);
          t4[k] = r[0];
          t4[k + 2] = r[1];
        }
#pragma unroll
        for (int k = 0; k < 4; k += 2) {
          const auto r = __builtin_amdgcn_permlane16_swap(t4[k], t4[k + 1], false, false);
          v[rb][kb][k] = r[0];
          v[rb][kb][k + 1] = r[1];
        }
        sc[rb][kb] = own;
      }
  }
};

// MXFP6 (E2M3 elements, E3M2 when E3M2 is set).  The lane layout is MXFP4's: lane group q
// holds block q as its 32 elements, element 8 s + 4 h + i from lane group s (tile 2 q + h,
// feature 4 s + i).  The FP32 values are transposed over the row's 4 lanes first (16
// exchanges with the lane 32 away, 16 with the lane 16 away), so that each lane holds its
// whole block and takes its scale from its own 32 values.  The conversion takes two
// vectors of 16 values and interleaves them (element 2 j from the first, 2 j + 1 from the
// second), rounds v / 2^X to nearest even and saturates (+-7.5, E3M2 +-28).  It writes its
// result while it still reads its sources, so the result must not share registers with
// them: the instruction is issued with an early-clobber result operand (the builtin's
// register allocation allows the overlap).
template <int KT, int R, bool E3M2>
struct MxF6Op {
  static constexpr int KB = kblocks(6, KT);
  uint32_t v[R][KB][6];
  uint32_t sc[R][KB];
  template <class F>
  __device__ __forceinline__ void build(F src) {
    typedef float f16v __attribute__((ext_vector_type(16)));
#pragma unroll
    for (int rb = 0; rb < R; ++rb)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        uint32_t c[4][8];   // c[b][4 h + i]: this lane's elements of block b
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int t = 8 * kb + 2 * b + h;
              c[b][4 * h + i] = __float_as_uint(t < KT ? src(rb, t < KT ? t : 0, i) : 0.f);
            }
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const auto r = __builtin_amdgcn_permlane32_swap(c[k][e], c[k + 2][e], false, false);
            c[k][e] = r[0];
            c[k + 2][e] = r[1];
          }
#pragma unroll
        for (int k = 0; k < 4; k += 2)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const auto r = __builtin_amdgcn_permlane16_swap(c[k][e], c[k + 1][e], false, false);
            c[k][e] = r[0];
            c[k + 1][e] = r[1];
          }
        // now c[s][e'] is element 8 s + e' of this lane group's block
        f16v a, bv;
        float m0 = 0.f, m1 = 0.f;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int el = 8 * s + e;
            const float x = __uint_as_float(c[s][e]);
            if (el & 1) {
              bv[el >> 1] = x;
              m1 = fmaxf(m1, fabsf(x));
            } else {
              a[el >> 1] = x;
              m0 = fmaxf(m0, fabsf(x));
            }
          }
        const int X = mx_exponent<E3M2 ? 4 : 2>(fmaxf(m0, m1));
        const float scale = __builtin_amdgcn_ldexpf(1.0f, X);
        typedef unsigned u6v __attribute__((ext_vector_type(6)));
        u6v r;
        // early-clobber result: the destination registers may not overlap a, bv or scale
        if constexpr (E3M2)
          asm("v_cvt_scalef32_2xpk16_bf6_f32 %0, %1, %2, %3" : "=&v"(r) : "v"(a), "v"(bv), "v"(scale));
        else
          asm("v_cvt_scalef32_2xpk16_fp6_f32 %0, %1, %2, %3" : "=&v"(r) : "v"(a), "v"(bv), "v"(scale));
#pragma unroll
        for (int d = 0; d < 6; ++d) v[rb][kb][d] = r[d];
        sc[rb][kb] = (uint32_t)(X + 127);
      }
  }
};
template <int KT, int R>
struct BOp<6, KT, R> : MxF6Op<KT, R, false> {};
template <int KT, int R>
struct BOp<8, KT, R> : MxF6Op<KT, R, true> {};

// acc[rb] += W(one output tile, all K) * B[rb] with both operands in an MX format: one
// 16x16x128 scaled MFMA per k-block, the block scales applied inside the instruction.
template <int PREC, int KT, int R>
__device__ __forceinline__ void mma_tile_mx(const unsigned char* fr, const BOp<PREC, KT, R>& b, f4 (&acc)[R],
                                            int lane) {
  constexpr int KB = kblocks(PREC, KT);
  // element format code: E4M3 0, E5M2 1, E2M3 2, E3M2 3, E2M1 4
  constexpr int FMT = PREC == 4 ? 0 : (PREC == 7 ? 1 : (PREC == 6 ? 2 : (PREC == 8 ? 3 : 4)));
  constexpr int ND = is_mx8(PREC) ? 8 : (is_mx6(PREC) ? 6 : 4);   // operand dwords per lane
  constexpr int EL = kbytes(PREC) - kMxScaleBytes;            // element bytes per k-block
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    const unsigned char* f = fr + kb * kbytes(PREC);
    const i4 lo = *reinterpret_cast<const i4*>(f + lane * 16);
    i4 hi = {0, 0, 0, 0};
    if constexpr (is_mx8(PREC)) hi = *reinterpret_cast<const i4*>(f + kFrag + lane * 16);
    if constexpr (is_mx6(PREC)) {
      const uint2 m = *reinterpret_cast<const uint2*>(f + kFrag + lane * 8);
      hi = i4{(int)m.x, (int)m.y, 0, 0};
    }
    const i8v a = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    const int sa = *reinterpret_cast<const int*>(f + EL + lane * 4);
#pragma unroll
    for (int rb = 0; rb < R; ++rb) {
      i8v bb;
#pragma unroll
      for (int j = 0; j < 8; ++j) bb[j] = j < ND ? (int)b.v[rb][kb][j < ND ? j : 0] : 0;
      acc[rb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, bb, acc[rb], FMT, FMT, 0, sa, 0,
                                                                 (int)b.sc[rb][kb]);
    }
  }
}

// One k-block of an MX GEMM for one output tile: `f` points at the k-block's elements and
// scales (kbytes(PREC) bytes), `kb` selects the B operand's k-block.
template <int PREC, int KT>
__device__ __forceinline__ f4 mma_kblock_mx(const unsigned char* f, const BOp<PREC, KT, 1>& b, int kb, f4 acc,
                                            int lane) {
  constexpr int FMT = PREC == 4 ? 0 : (PREC == 7 ? 1 : (PREC == 6 ? 2 : (PREC == 8 ? 3 : 4)));
  constexpr int ND = is_mx8(PREC) ? 8 : (is_mx6(PREC) ? 6 : 4);
  constexpr int EL = kbytes(PREC) - kMxScaleBytes;
  const i4 lo = *reinterpret_cast<const i4*>(f + lane * 16);
  i4 hi = {0, 0, 0, 0};
  if constexpr (is_mx8(PREC)) hi = *reinterpret_cast<const i4*>(f + kFrag + lane * 16);
  if constexpr (is_mx6(PREC)) {
    const uint2 m = *reinterpret_cast<const uint2*>(f + kFrag + lane * 8);
    hi = i4{(int)m.x, (int)m.y, 0, 0};
  }
  const i8v a = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  const int sa = *reinterpret_cast<const int*>(f + EL + lane * 4);
  i8v bb;
#pragma unroll
  for (int j = 0; j < 8; ++j) bb[j] = j < ND ? (int)b.v[0][kb][j < ND ? j : 0] : 0;
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, bb, acc, FMT, FMT, 0, sa, 0, (int)b.sc[0][kb]);
}

// One k-block (four K tiles) of a GEMM with row-coded inputs for one output tile: `f`
// points at the k-block's 1 KiB fragment of weight codes, `kb` selects the B operand's
// tiles.  E4M3: two 16x16x32 FP8 MFMAs (bytes 0-7 and 8-15 of each lane).  INT8: one
// 16x16x64 MFMA whose INT32 sums are carried in the bits of `acc`.
template <int PREC, int KT>
__device__ __forceinline__ f4 mma_kblock_rc(const unsigned char* f, const BOp<PREC, KT, 1>& b, int kb, f4 acc,
                                            int lane) {
  const i4 a = *reinterpret_cast<const i4*>(f + lane * 16);
  if constexpr (PREC == 3) {
    uint32_t q[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = 4 * kb + j;
      q[j] = t < KT ? b.v[0][t < KT ? t : 0] : 0u;
    }
    return __builtin_bit_cast(f4, __builtin_amdgcn_mfma_i32_16x16x64_i8(a, __builtin_bit_cast(i4, q),
                                                                         __builtin_bit_cast(i4, acc), 0, 0, 0));
  } else {
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      const int t0 = 4 * kb + 2 * hf, t1 = t0 + 1;
      if (t0 < KT) {
        const long ah = (long)(((uint64_t)(uint32_t)a[2 * hf + 1] << 32) | (uint32_t)a[2 * hf]);
        const uint32_t lo = b.v[0][t0 < KT ? t0 : 0];
        const uint32_t hi = t1 < KT ? b.v[0][t1 < KT ? t1 : 0] : 0u;
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ah, (long)(((uint64_t)hi << 32) | lo), acc, 0, 0, 0);
      }
    }
    return acc;
  }
}

// INT32 sums held in the bits of an FP32 accumulator, as FP32 values.
__device__ __forceinline__ f4 i32_sums(f4 acc) {
  const i4 q = __builtin_bit_cast(i4, acc);
  return f4{(float)q[0], (float)q[1], (float)q[2], (float)q[3]};
}

// Fill a GEMM's B operand from src(rb, t, i), the input of row block rb at the lane's
// feature 16 t + 4 g + i.
template <int PREC, int KT, int R, class F>
__device__ __forceinline__ void build_b(BOp<PREC, KT, R>& b, F src) {
  if constexpr (PREC >= 2 && !is_fp8w(PREC)) {
    b.build(src);
  } else {
#pragma unroll
    for (int rb = 0; rb < R; ++rb)
#pragma unroll
      for (int t = 0; t < KT; ++t) {
        const float v[4] = {src(rb, t, 0), src(rb, t, 1), src(rb, t, 2), src(rb, t, 3)};
        b.set(rb, t, v);
      }
  }
}

// INT8: acc[rb] += Wq(one output tile, all K) * codes[rb], exactly in INT32 (K <= 2^14
// keeps |acc| < 127 * 127 * 2^14 < 2^31); four K tiles per 16x16x64 MFMA.
template <int KT, int R>
__device__ __forceinline__ void mma_tile_i8(const unsigned char* fr, const BOp<3, KT, R>& b, i4 (&acc)[R],
                                            int lane) {
  constexpr int KQ = kblocks(3, KT);
#pragma unroll
  for (int kb = 0; kb < KQ; ++kb) {
    const i4 a = *reinterpret_cast<const i4*>(fr + kb * kFrag + lane * 16);
#pragma unroll
    for (int rb = 0; rb < R; ++rb) {
      uint32_t q[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int t = 4 * kb + j;
        q[j] = t < KT ? b.v[rb][t < KT ? t : 0] : 0u;
      }
      acc[rb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, __builtin_bit_cast(i4, q), acc[rb], 0, 0, 0);
    }
  }
}

// acc[rb] += W'(one output tile, all K) * B[rb]; `fr` points at the tile's fragments
// in LDS (kblocks(PREC, KT) fragments of 1 KiB).
template <int PREC, int KT, int R>
__device__ __forceinline__ void mma_tile(const unsigned char* fr, const BOp<PREC, KT, R>& b,
                                         f4 (&acc)[R], int lane) {
  if constexpr (is_mx(PREC)) {
    mma_tile_mx<PREC, KT, R>(fr, b, acc, lane);
  } else if constexpr (PREC == 0) {
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      const f4 a = *reinterpret_cast<const f4*>(fr + kt * kFrag + lane * 16);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int rb = 0; rb < R; ++rb)
          acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r], b.v[rb][kt][r], acc[rb], 0, 0, 0);
    }
  } else {
    // Only the 16x16x32 BF16 MFMA is used, so every accumulator chain has one
    // instruction shape; an odd trailing K tile is paired with zeros.
    constexpr int KP = (KT + 1) / 2;
#pragma unroll
    for (int kb = 0; kb < KP; ++kb) {
      const s8 a = *reinterpret_cast<const s8*>(fr + kb * kFrag + lane * 16);
#pragma unroll
      for (int rb = 0; rb < R; ++rb) {
        constexpr int dummy = 0;
        const bool full = 2 * kb + 1 < KT;
        uint32_t q[4] = {b.v[rb][2 * kb][0], b.v[rb][2 * kb][1],
                         full ? b.v[rb][full ? 2 * kb + 1 : dummy][0] : 0u,
                         full ? b.v[rb][full ? 2 * kb + 1 : dummy][1] : 0u};
        const s8 bb = __builtin_bit_cast(s8, q);
        acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc[rb], 0, 0, 0);
      }
    }
  }
}

// E4M3: acc[rb] += Wq(one output tile, all K) * codes[rb] in FP32; a 1 KiB fragment holds
// four K tiles, as two 16x16x32 FP8 MFMAs (bytes 0-7 and 8-15 of each lane).
template <int KT, int R>
__device__ __forceinline__ void mma_tile_f8(const unsigned char* fr, const BOp<2, KT, R>& b, f4 (&acc)[R],
                                            int lane) {
  constexpr int KQ = kblocks(2, KT);
#pragma unroll
  for (int kb = 0; kb < KQ; ++kb) {
    const i4 a = *reinterpret_cast<const i4*>(fr + kb * kFrag + lane * 16);
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      if (4 * kb + 2 * hf < KT) {
        const long ah = (long)(((uint64_t)(uint32_t)a[2 * hf + 1] << 32) | (uint32_t)a[2 * hf]);
#pragma unroll
        for (int rb = 0; rb < R; ++rb) {
          const int t0 = 4 * kb + 2 * hf, t1 = t0 + 1;
          const uint32_t lo = b.v[rb][t0 < KT ? t0 : 0];
          const uint32_t hi = t1 < KT ? b.v[rb][t1 < KT ? t1 : 0] : 0u;
          const long bh = (long)(((uint64_t)hi << 32) | lo);
          acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ah, bh, acc[rb], 0, 0, 0);
        }
      }
    }
  }
}

// E4M3 weights, BF16 inputs: acc[rb] += Wq(one output tile, all K) * B[rb] in FP32.  A
// 1 KiB fragment holds four K tiles of codes (byte j of a lane: tile 4 kb + j / 4, feature
// 4 q + j % 4); each half (two tiles) is widened to eight BF16 values, exactly, and feeds
// one 16x16x32 BF16 MFMA with the matching tile pair of the BF16 operand.
__device__ __forceinline__ s8 widen_e4m3x8(uint32_t lo, uint32_t hi) {
  uint32_t w[4] = {__builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(lo, 1.0f, false)),
                   __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(lo, 1.0f, true)),
                   __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(hi, 1.0f, false)),
                   __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(hi, 1.0f, true))};
  return __builtin_bit_cast(s8, w);
}

template <int KT, int R>
__device__ __forceinline__ void mma_tile_w8(const unsigned char* fr, const BOp<9, KT, R>& b, f4 (&acc)[R],
                                            int lane) {
  constexpr int KQ = kblocks(9, KT);
#pragma unroll
  for (int kb = 0; kb < KQ; ++kb) {
    const i4 a = *reinterpret_cast<const i4*>(fr + kb * kFrag + lane * 16);
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      const int t0 = 4 * kb + 2 * hf, t1 = t0 + 1;
      if (t0 < KT) {
        const s8 aw = widen_e4m3x8(a[2 * hf], a[2 * hf + 1]);
#pragma unroll
        for (int rb = 0; rb < R; ++rb) {
          uint32_t q[4] = {b.v[rb][t0][0], b.v[rb][t0][1], t1 < KT ? b.v[rb][t1 < KT ? t1 : 0][0] : 0u,
                           t1 < KT ? b.v[rb][t1 < KT ? t1 : 0][1] : 0u};
          acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, __builtin_bit_cast(s8, q), acc[rb], 0, 0, 0);
        }
      }
    }
  }
}

// Formats with channel scales (E4M3, INT8, E4M3 weights): acc[rb] = Wq(one output tile) *
// input[rb] as FP32, before the dequantisation by (channel scale) x (row scale).
template <int PREC, int KT, int R>
__device__ __forceinline__ void mma_tile_coded(const unsigned char* fr, const BOp<PREC, KT, R>& b, f4 (&acc)[R],
                                               int lane) {
  if constexpr (is_fp8w(PREC)) {
#pragma unroll
    for (int rb = 0; rb < R; ++rb) acc[rb] = f4{0.f, 0.f, 0.f, 0.f};
    mma_tile_w8<KT, R>(fr, b, acc, lane);
  } else if constexpr (PREC == 3) {
    i4 q[R];
#pragma unroll
    for (int rb = 0; rb < R; ++rb) q[rb] = i4{0, 0, 0, 0};
    mma_tile_i8<KT, R>(fr, b, q, lane);
#pragma unroll
    for (int rb = 0; rb < R; ++rb) acc[rb] = f4{(float)q[rb][0], (float)q[rb][1], (float)q[rb][2], (float)q[rb][3]};
  } else {
#pragma unroll
    for (int rb = 0; rb < R; ++rb) acc[rb] = f4{0.f, 0.f, 0.f, 0.f};
    mma_tile_f8<KT, R>(fr, b, acc, lane);
  }
}

// ------------------------------------------------------------------------------------
// Double-buffered weight stream through LDS, shared by the W waves of a workgroup.  The
// chunk goes straight from global memory into LDS (global_load_lds_dwordx4: lane l of a
// wave writes base + 16 l).
template <int W, int BUF>
struct WeightStream {
  static constexpr int kW = W;
  static constexpr int T = 64 * W;
  static constexpr int NSTG = (BUF / 16 + T - 1) / T;
  unsigned char* lds;            // 2 * BUF bytes
  const unsigned char* wts;
  const ChunkRec* tab;
  int n, idx, cur, next_bytes;

  // Issue the global loads of the chunk after the current one.
  __device__ __forceinline__ void begin() {
    next_bytes = 0;
    if (idx + 1 < n) {
      const ChunkRec r = tab[idx + 1];
      next_bytes = r.bytes;
      const unsigned char* src = wts + r.off;
      unsigned char* dst = lds + (cur ^ 1) * BUF;
      const int wave = (int)threadIdx.x >> 6;
#pragma unroll
      for (int j = 0; j < NSTG; ++j) {
        const int p = (int)threadIdx.x + j * T;
        if (p * 16 < next_bytes)
          __builtin_amdgcn_global_load_lds(
              (const void __attribute__((address_space(1)))*)(src + (size_t)p * 16),
              (void __attribute__((address_space(3)))*)(dst + (j * T + wave * 64) * 16), 16, 0, 0);
      }
    }
  }
  // Complete them, wait for the whole workgroup, switch buffers.
  __device__ __forceinline__ void end() {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    lds_block_sync();
    cur ^= 1;
    ++idx;
  }
  __device__ __forceinline__ const unsigned char* ptr() const { return lds + cur * BUF; }
};

// One GLU layer: h <- GLU(u W'^T + b')  (first layer of a pass)
//            or  h <- (h + GLU(h W'^T + b')) * sqrt(1/2).
// Value tile mt and gate tile mt land in the same lanes and registers, so the GLU is
// lane-local.  The layer's units arrive chunk by chunk through the weight stream.
template <int PREC, int KT, int NT, int R, int UNIT, int UPC, int NCH, class WS>
__device__ __forceinline__ void glu_layer(WS& ws, const BOp<PREC, KT, R>& b,
                                          float (&h)[R][NT][4], bool first, int lane) {
  constexpr int KB = kblocks(PREC, KT);
  const int g = lane >> 4;
  // h is updated tile by tile in place: the B operand is a separate copy of the input.
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    ws.begin();
    const unsigned char* buf = ws.ptr();
#pragma unroll
    for (int u = 0; u < UPC; ++u) {
      const int mt = c * UPC + u;
      if (mt < NT) {
        const unsigned char* unit = buf + u * UNIT;
        const f4 bv = *reinterpret_cast<const f4*>(unit + 2 * KB * kbytes(PREC) + 16 * g);
        const f4 bg = *reinterpret_cast<const f4*>(unit + 2 * KB * kbytes(PREC) + 64 + 16 * g);
        if constexpr (has_channel_scales(PREC)) {
          // products of codes, dequantised by (channel scale) x (row scale); the gate's shift
          // and scale carry the factor -log2(e) of the sigmoid's exponent
          f4 qv[R], qg[R];
          mma_tile_coded<PREC, KT, R>(unit, b, qv, lane);
          mma_tile_coded<PREC, KT, R>(unit + KB * kbytes(PREC), b, qg, lane);
          const f4 sv = *reinterpret_cast<const f4*>(unit + 2 * KB * kbytes(PREC) + 128 + 16 * g);
          const f4 sgt = *reinterpret_cast<const f4*>(unit + 2 * KB * kbytes(PREC) + 192 + 16 * g);
#pragma unroll
          for (int rb = 0; rb < R; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float v = __builtin_fmaf(qv[rb][i], sv[i] * b.rscale(rb), bv[i]);
              const float e = __builtin_fmaf(qg[rb][i], sgt[i] * b.rscale(rb), bg[i]);
              const float sg = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(e));
              h[rb][mt][i] = first ? v * sg : __builtin_fmaf(v, sg, h[rb][mt][i]) * kSqrtHalf;
            }
        } else {
        f4 av[R], ag[R];
#pragma unroll
        for (int rb = 0; rb < R; ++rb) { av[rb] = bv; ag[rb] = bg; }
        mma_tile<PREC, KT, R>(unit, b, av, lane);
        mma_tile<PREC, KT, R>(unit + KB * kbytes(PREC), b, ag, lane);
#pragma unroll
        for (int rb = 0; rb < R; ++rb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float sg = sigmoid_fast(ag[rb][i]);
            h[rb][mt][i] = first ? av[rb][i] * sg : __builtin_fmaf(av[rb][i], sg, h[rb][mt][i]) * kSqrtHalf;
          }
        }
      }
    }
    ws.end();
  }
}

// Feature-transformer pass on input u (DT tiles); result h (NT tiles).  L = layers/pass.
template <int PREC, int DT, int NT, int KA0, int R, class WS>
__device__ __forceinline__ void ft_pass(WS& ws, int L, const BOp<PREC, DT, R>& u,
                                        float (&h)[R][NT][4], int lane) {
  constexpr Plan P = make_plan(PREC, DT, NT, KA0, chunk_target(DT, R, WS::kW));
  glu_layer<PREC, DT, NT, R, P.first.unit, P.first.upc, P.first.nchunks>(ws, u, h, true, lane);
  for (int l = 1; l < L; ++l) {
    BOp<PREC, NT, R> bh;
    build_b(bh, [&](int rb, int t, int i) { return h[rb][t][i]; });
    glu_layer<PREC, NT, NT, R, P.mid.unit, P.mid.upc, P.mid.nchunks>(ws, bh, h, false, lane);
  }
}

// Copy n consecutive floats from this wave's LDS staging area to global memory, with
// all 64 lanes writing consecutive 16-byte pieces (streaming stores).
__device__ __forceinline__ void stage_out(const float* st, float* dst, int n, int lane) {
  if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
    const int n4 = n & ~3;
    for (int e = 4 * lane; e < n4; e += 256)
      __builtin_nontemporal_store(*reinterpret_cast<const f4*>(st + e), reinterpret_cast<f4*>(dst + e));
    for (int e = n4 + lane; e < n; e += 64) __builtin_nontemporal_store(st[e], dst + e);
  } else {
    for (int e = lane; e < n; e += 64) __builtin_nontemporal_store(st[e], dst + e);
  }
}

// Raw-column view of a mask held in the lane layout (lane = row rl, features 16 t + 4 g + i):
// out[row][c] = sum of the row's mask over the features of raw column c, for all C
// columns, as FP32 MFMA products with the 0/1 membership matrix S[c][f] = (column of f == c).
// For 16 columns at a time the B operand of MFMA (t, i) is the lane's own value m[t][i]
// (k slot g holds feature 16 t + 4 g + i of row rl) and the A operand is the membership
// of that feature in column 16 ct + rl: bit 4 t + i of colbits[64 ct + lane], a table
// the host builds with the embedding.  The products are exact and the sums are FP32.
// The result lands as out[row rl][16 ct + 4 g + j] and is written to the wave's LDS
// staging area as [16][C] rows, ready for stage_out.
template <int DT>
__device__ __forceinline__ void reduce_columns(const float (&m)[DT][4], const uint64_t* colbits, int C, float* st,
                                               int lane) {
  static_assert(DT <= 16, "membership masks hold 64 features per lane");
  const int g = lane >> 4;
  const int rl = lane & 15;
  for (int ct = 0; 16 * ct < C; ++ct) {
    const uint64_t bits = colbits[64 * ct + lane];
    f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};   // two independent chains
#pragma unroll
    for (int t = 0; t < DT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float a = (bits >> (4 * t + i)) & 1 ? 1.f : 0.f;
        if ((i & 1) == 0)
          acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, m[t][i], acc0, 0, 0, 0);
        else
          acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, m[t][i], acc1, 0, 0, 0);
      }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = 16 * ct + 4 * g + j;
      if (c < C) st[rl * C + c] = acc0[j] + acc1[j];
    }
  }
}

// ------------------------------------------------------------------------------------
// The register-resident forward.  GEN: a kernel compiled for up to DT feature tiles and NT
// hidden tiles that serves smaller models too (the features past the model's D masked
// like those of a partial last tile, the hidden channels past n_d + n_a carried as zeros
// by zero weights and shifts); otherwise DT = ceil(D / 16) exactly.
template <int PREC, int DT, int NT, int KA0, int R, int W, bool RAW, bool GEN = false>
__global__ void __launch_bounds__(64 * W) tabnet_forward_kernel(FwdArgs A) {
  constexpr Plan PL = make_plan(PREC, DT, NT, KA0, chunk_target(DT, R, W));
  constexpr int KTA = NT - KA0;   // K tiles of the attentive GEMM (the attention half)
  // Where a 16-row block's resident state (x, P, the aggregate and M per feature; h and the
  // decision sums per hidden channel) passes the registers a wave has at W / 4 waves per
  // SIMD, less room for the GLU's operands, the aggregate mask lives in this wave's staging
  // area ([16 R rows][D], each lane reading and writing only its own features) and the step
  // masks leave straight from registers.  Elsewhere the aggregate stays in registers and
  // the step masks leave through the staging area as whole rows.
  constexpr bool AGG_LDS = !RAW && (16 * DT + 8 * NT) * R > 512 / (W < 4 ? 1 : W / 4) - 64;
  // There, FP32 and both FP8 forms also read x again from X before each pass instead of
  // keeping it (their spills shrink from 600-720 to 320-380 bytes per lane, and the 200-feature
  // forward gains 2-12%); BF16 and MXFP4, whose spills are smaller, lose 10% that way.
  constexpr bool X_AGAIN = AGG_LDS && (PREC == 0 || PREC == 2 || PREC == 9);
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  const int64_t B = A.B_dev != nullptr ? *A.B_dev : A.B;
  // A workgroup past the live rows leaves before its first barrier (all its waves alike).
  if ((int64_t)blockIdx.x * (16 * R * W) >= B) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4;
  const int rl = lane & 15;
  const int D = A.D, n_d = A.n_d;
  const int64_t wrow0 = ((int64_t)blockIdx.x * W + wave) * (16 * R);   // first row of this wave
  const int live_rows = (int)(B - wrow0 < 0 ? 0 : (B - wrow0 > 16 * R ? 16 * R : B - wrow0));
  float* stage = reinterpret_cast<float*>(smem + 2 * PL.buf) + (size_t)wave * 16 * R * D;
  // the final map, staged in LDS behind the mask staging areas (visible after the first barrier)
  float* wfin_s = reinterpret_cast<float*>(smem + 2 * PL.buf) + (size_t)W * 16 * R * D;
  for (int e = threadIdx.x; e < A.n_out * n_d; e += 64 * W) wfin_s[e] = A.wfin[e];
  // raw rows: the embedding map, staged behind the final map (the prologue needs it, so the
  // workgroup synchronises once more)
  int* meta_s = reinterpret_cast<int*>(wfin_s + ((A.n_out * n_d + 3) & ~3));   // 16-byte aligned
  // and the embedding tables after it when they fit (tab_lds), else they are read from L2
  float* tab_s = reinterpret_cast<float*>(meta_s + 4 * D);
  if constexpr (RAW) {
    // this wave's raw rows go straight into its LDS staging area (global_load_lds_dword:
    // lane l of an instruction writes base + 4 l), while the workgroup copies the maps
    {
      const float* src = A.X + wrow0 * A.C;
      const int n = live_rows * A.C;
      for (int j = 0; 64 * j < n; ++j)
        if (64 * j + lane < n)
          __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)(src + 64 * j + lane),
                                           (void __attribute__((address_space(3)))*)(stage + 64 * j), 4, 0, 0);
    }
    for (int e = threadIdx.x; e < 4 * D; e += 64 * W) meta_s[e] = A.emb_meta[e];
    if (A.tab_lds)
      for (int e = threadIdx.x; e < A.tab_len; e += 64 * W) tab_s[e] = A.emb_tables[e];
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  }
  bool live[R];
#pragma unroll
  for (int rb = 0; rb < R; ++rb) live[rb] = 16 * rb + rl < live_rows;
  // Is feature 16 t + 4 g + i a real column?  Only the model's last tile can be partial,
  // and (GEN) the tiles past it are padding.
  const int dlast = GEN ? (D - 1) >> 4 : DT - 1;
  bool last_ok[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) last_ok[i] = 16 * dlast + 4 * g + i < D;
  auto feat_ok = [&](int t, int i) { return GEN ? t < dlast || (t == dlast && last_ok[i]) : t < DT - 1 || last_ok[i]; };
  // this lane's features of tile t of row block rb in the staging area ([16 R rows][D])
  auto own_get = [&](int rb, int t, float (&m)[4]) {
    const float* sr = stage + (16 * rb + rl) * D + 16 * t + 4 * g;
#pragma unroll
    for (int i = 0; i < 4; ++i) m[i] = 0.f;
    if ((D & 3) == 0) {
      if (feat_ok(t, 0)) {
        const f4 q = *reinterpret_cast<const f4*>(sr);
        m[0] = q[0]; m[1] = q[1]; m[2] = q[2]; m[3] = q[3];
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (feat_ok(t, i)) m[i] = sr[i];
    }
  };
  auto own_put = [&](int rb, int t, const float (&m)[4]) {
    float* sr = stage + (16 * rb + rl) * D + 16 * t + 4 * g;
    if ((D & 3) == 0) {
      if (feat_ok(t, 0)) *reinterpret_cast<f4*>(sr) = f4{m[0], m[1], m[2], m[3]};
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (feat_ok(t, i)) sr[i] = m[i];
    }
  };

  WeightStream<W, PL.buf> ws;
  ws.lds = smem;
  ws.wts = A.wts;
  ws.tab = A.chunks;
  ws.n = A.n_chunks;
  ws.idx = -1;
  ws.cur = 1;
  ws.begin();     // first chunk -> buffer 0

  // ---- input batch norm (folded to a per-column affine map) ----
  // Raw rows are embedded first.  Model feature f is described by fdesc[f] = (raw column
  // c, its number of levels (0: continuous), index of the feature's entry in level 0's
  // table row, table row width): a continuous column passes through, a level l of a
  // categorical column contributes tables[z + l * w], and a value that is not a level in
  // [0, card) contributes 0.
  float x[R][DT][4];
  const bool vec4 = (D & 3) == 0;
  const int C = A.C;
  const int4* fdesc = reinterpret_cast<const int4*>(meta_s);
  float raw[RAW ? R : 1][RAW ? DT : 1][4];
  if constexpr (RAW) {
    // every feature is gathered from LDS: the raw rows (staged above), the maps, the tables
    const float* tab = A.tab_lds ? tab_s : A.emb_tables;
#pragma unroll
    for (int rb = 0; rb < R; ++rb)
#pragma unroll
      for (int t = 0; t < DT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int4 d = fdesc[feat_ok(t, i) ? 16 * t + 4 * g + i : 0];
          const float q = stage[(16 * rb + rl) * C + d.x];
          const bool level = q >= 0.f && q < (float)d.y && q == floorf(q);   // false for card 0
          const float tv = tab[level ? d.z + (int)q * d.w : 0];
          const float e = d.y == 0 ? q : (level ? tv : 0.f);
          raw[rb][t][i] = live[rb] && feat_ok(t, i) ? e : 0.f;
        }
  }
#pragma unroll
  for (int t = 0; t < DT; ++t) {
    const f4 sc = *reinterpret_cast<const f4*>(A.in_affine + 16 * t + 4 * g);
    const f4 sh = *reinterpret_cast<const f4*>(A.in_affine + 16 * DT + 16 * t + 4 * g);
#pragma unroll
    for (int rb = 0; rb < R; ++rb) {
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      const float* xr = A.X + (wrow0 + 16 * rb + rl) * D + 16 * t + 4 * g;
      if constexpr (RAW) {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = raw[rb][t][i];
      } else if (live[rb]) {
        if (vec4) {
          if (feat_ok(t, 0)) {
            const f4 q = *reinterpret_cast<const f4*>(xr);
            v[0] = q[0]; v[1] = q[1]; v[2] = q[2]; v[3] = q[3];
          }
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (feat_ok(t, i)) v[i] = xr[i];
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) x[rb][t][i] = v[i] * sc[i] + sh[i];
    }
  }
  ws.end();

  float P[R][DT][4], agg[AGG_LDS ? 1 : R][AGG_LDS ? 1 : DT][4], M[R][DT][4];
  // decision sums: only tiles [0, KA0] can hold decision channels (n_d < 16 (KA0 + 1))
  constexpr int KD = KA0 + 1 < NT ? KA0 + 1 : NT;
  float h[R][NT][4], acc[R][KD][4];
#pragma unroll
  for (int rb = 0; rb < R; ++rb) {
#pragma unroll
    for (int t = 0; t < DT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) { P[rb][t][i] = 1.f; if constexpr (!AGG_LDS) agg[rb][t][i] = 0.f; }
    if constexpr (AGG_LDS) {
      const float z[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < DT; ++t) own_put(rb, t, z);
    }
#pragma unroll
    for (int t = 0; t < KD; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[rb][t][i] = 0.f;
  }
  const int L = A.n_sh + A.n_ind;

  // ---- pass 0: only its attention half is used ----
  {
    BOp<PREC, DT, R> u;
    build_b(u, [&](int rb, int t, int i) { return x[rb][t][i]; });
    ft_pass<PREC, DT, NT, KA0, R>(ws, L, u, h, lane);
  }

  const int64_t step_stride = B * (int64_t)(RAW ? C : D);
  for (int s = 1; s <= A.n_steps; ++s) {
    // ---- attentive transformer: z = P * (a W_att'^T + b_att') ----
    {
      BOp<PREC, KTA, R> ba;
      // the attention half a = h[n_d, N): the scaled formats (E4M3, INT8, MX) take their
      // scales over those channels only (the weights of the other channels here are zero)
      const int n_att_end = n_d + A.n_a;
      build_b(ba, [&](int rb, int t, int i) {
        const int ch = 16 * (KA0 + t) + 4 * g + i;
        return !row_coded(PREC) && !is_mx(PREC) || (ch >= n_d && ch < n_att_end) ? h[rb][KA0 + t][i] : 0.f;
      });
      constexpr int KBA = kblocks(PREC, KTA);
#pragma unroll
      for (int c = 0; c < PL.att.nchunks; ++c) {
        ws.begin();
        const unsigned char* buf = ws.ptr();
#pragma unroll
        for (int u = 0; u < PL.att.upc; ++u) {
          const int mt = c * PL.att.upc + u;
          if (mt < DT) {
            const unsigned char* unit = buf + u * PL.att.unit;
            const f4 bv = *reinterpret_cast<const f4*>(unit + KBA * kbytes(PREC) + 16 * g);
            if constexpr (has_channel_scales(PREC)) {
              f4 qa[R];
              mma_tile_coded<PREC, KTA, R>(unit, ba, qa, lane);
              const f4 scl = *reinterpret_cast<const f4*>(unit + KBA * kbytes(PREC) + 64 + 16 * g);
#pragma unroll
              for (int rb = 0; rb < R; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const float hz = __builtin_fmaf(qa[rb][i], scl[i] * ba.rscale(rb), bv[i]);
                  M[rb][mt][i] = feat_ok(mt, i) ? P[rb][mt][i] * hz : kNegBig;
                }
            } else {
            f4 za[R];
#pragma unroll
            for (int rb = 0; rb < R; ++rb) za[rb] = bv;
            mma_tile<PREC, KTA, R>(unit, ba, za, lane);
#pragma unroll
            for (int rb = 0; rb < R; ++rb)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                M[rb][mt][i] = feat_ok(mt, i) ? P[rb][mt][i] * za[rb][i] : kNegBig;
              }
            }
          }
        }
        ws.end();
      }
    }
    // ---- sparsemax per row: Newton iteration on sum(max(z - tau, 0)) = 1 ----
    // For ANY set S of scores, (sum_S z - 1) / |S| is a lower bound of the threshold tau;
    // over the prefixes of a sorted list the best such bound is exact once the list holds
    // the support, and the largest score minus 1 is one too.  The start is the best
    // prefix bound of the row's top 8 candidates (the two largest scores of each of its
    // 4 lanes).  From a lower bound, each step tau <- (sum_{z > tau} z - 1) / |{z > tau}|
    // moves tau up monotonically and stops, exactly, once the support no longer shrinks.
    // If the first count equals the length kb of the best prefix and the prefix's smallest
    // value lies above the new tau, the counted set is that prefix, it is the support,
    // and the row is done after one pass.
    {
      float tau[R], vlast[R];
      int kprev[R], kbest[R];
      bool done[R];
#pragma unroll
      for (int rb = 0; rb < R; ++rb) {
        // this lane's two largest scores, in two independent chains merged at the end
        float a1 = kNegBig, a2 = kNegBig, b1 = kNegBig, b2 = kNegBig;
#pragma unroll
        for (int t = 0; t < DT; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float w = M[rb][t][i];
            if (i & 1) {
              b2 = __builtin_amdgcn_fmed3f(b1, b2, w);
              b1 = fmaxf(b1, w);
            } else {
              a2 = __builtin_amdgcn_fmed3f(a1, a2, w);
              a1 = fmaxf(a1, w);
            }
          }
        const float t1 = fmaxf(a1, b1);
        const float t2 = fmaxf(fminf(a1, b1), fmaxf(a2, b2));
        float v[8];
        top8_sorted(t1, t2, v);
        float c = 0.f, best = v[0] - 1.f, vl = v[0];
        int kb = 1;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          c += v[k];
          const float bnd = (c - 1.f) * (1.0f / (float)(k + 1));
          if (bnd > best) {
            best = bnd;
            kb = k + 1;
            vl = v[k];
          }
        }
        tau[rb] = best;
        kbest[rb] = kb;
        vlast[rb] = vl;
        kprev[rb] = 0x7fffffff;
        done[rb] = false;
      }
      for (int it = 0; it <= 16 * DT + 1; ++it) {
        bool any_open = false;
#pragma unroll
        for (int rb = 0; rb < R; ++rb) {
          // four independent partial sums (one per slot i), combined in a fixed order
          float sp[4] = {0.f, 0.f, 0.f, 0.f};
          int kp[4] = {0, 0, 0, 0};
#pragma unroll
          for (int t = 0; t < DT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const bool in = M[rb][t][i] > tau[rb];
              sp[i] += in ? M[rb][t][i] : 0.f;
              kp[i] += in ? 1 : 0;
            }
          float sm = row_sum((sp[0] + sp[1]) + (sp[2] + sp[3]));
          int k = row_sum((kp[0] + kp[1]) + (kp[2] + kp[3]));
          if (!done[rb]) {
            if (k >= kprev[rb]) {
              done[rb] = true;
            } else {
              tau[rb] = (sm - 1.f) / (float)k;
              kprev[rb] = k;
              if (it == 0 && k == kbest[rb] && vlast[rb] > tau[rb]) done[rb] = true;
            }
          }
          any_open |= !done[rb];
        }
        if (!__any(any_open)) break;
      }
#pragma unroll
      for (int rb = 0; rb < R; ++rb)
#pragma unroll
        for (int t = 0; t < DT; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) M[rb][t][i] = fmaxf(M[rb][t][i] - tau[rb], 0.f);
    }
    // ---- step mask out (through LDS, coalesced) first, so that the stores drain while
    // the prior update and the masked input are computed ----
    if (A.masks_step != nullptr) {
      if constexpr (RAW) {
#pragma unroll
        for (int rb = 0; rb < R; ++rb) reduce_columns<DT>(M[rb], A.colbits, C, stage + 16 * rb * C, lane);
        lds_wave_sync();
        stage_out(stage, A.masks_step + (int64_t)(s - 1) * step_stride + wrow0 * C, live_rows * C, lane);
      } else if constexpr (AGG_LDS) {
        // each lane stores its own 16-byte pieces (D % 4 == 0) or floats; ordinary stores, so
        // that L2 joins the pieces of a line before it writes the line back
#pragma unroll
        for (int rb = 0; rb < R; ++rb) {
          if (!live[rb]) continue;
          float* dr = A.masks_step + (int64_t)(s - 1) * step_stride + (wrow0 + 16 * rb + rl) * D + 4 * g;
#pragma unroll
          for (int t = 0; t < DT; ++t) {
            if (vec4) {
              if (feat_ok(t, 0))
                *reinterpret_cast<f4*>(dr + 16 * t) = f4{M[rb][t][0], M[rb][t][1], M[rb][t][2], M[rb][t][3]};
            } else {
#pragma unroll
              for (int i = 0; i < 4; ++i)
                if (feat_ok(t, i)) dr[16 * t + i] = M[rb][t][i];
            }
          }
        }
      } else {
#pragma unroll
        for (int rb = 0; rb < R; ++rb) {
          float* sr = stage + (16 * rb + rl) * D + 4 * g;
          if (vec4) {
            // D % 4 == 0: a lane's four features are 16-byte aligned and all real or all padding
#pragma unroll
            for (int t = 0; t < DT; ++t)
              if (feat_ok(t, 0))
                *reinterpret_cast<f4*>(sr + 16 * t) = f4{M[rb][t][0], M[rb][t][1], M[rb][t][2], M[rb][t][3]};
          } else {
#pragma unroll
            for (int t = 0; t < DT; ++t)
#pragma unroll
              for (int i = 0; i < 4; ++i)
                if (feat_ok(t, i)) sr[16 * t + i] = M[rb][t][i];
          }
        }
        lds_wave_sync();
        stage_out(stage, A.masks_step + (int64_t)(s - 1) * step_stride + wrow0 * D, live_rows * D, lane);
      }
    }
    BOp<PREC, DT, R> u;
#pragma unroll
    for (int rb = 0; rb < R; ++rb)
#pragma unroll
      for (int t = 0; t < DT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) P[rb][t][i] *= A.gamma - M[rb][t][i];
    if constexpr (X_AGAIN) {
      // x again from X and the input affine map (L2), so that it is not live across the
      // feature transformer: the same values as in the prologue
      float xs[R][DT][4];
#pragma unroll
      for (int t = 0; t < DT; ++t) {
        const f4 sc = *reinterpret_cast<const f4*>(A.in_affine + 16 * t + 4 * g);
        const f4 sh = *reinterpret_cast<const f4*>(A.in_affine + 16 * DT + 16 * t + 4 * g);
#pragma unroll
        for (int rb = 0; rb < R; ++rb) {
          float v[4] = {0.f, 0.f, 0.f, 0.f};
          const float* xr = A.X + (wrow0 + 16 * rb + rl) * D + 16 * t + 4 * g;
          if (live[rb]) {
            if (vec4) {
              if (feat_ok(t, 0)) {
                const f4 q = *reinterpret_cast<const f4*>(xr);
                v[0] = q[0]; v[1] = q[1]; v[2] = q[2]; v[3] = q[3];
              }
            } else {
#pragma unroll
              for (int i = 0; i < 4; ++i)
                if (feat_ok(t, i)) v[i] = xr[i];
            }
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) xs[rb][t][i] = v[i] * sc[i] + sh[i];
        }
      }
      build_b(u, [&](int rb, int t, int i) { return M[rb][t][i] * xs[rb][t][i]; });
    } else {
      build_b(u, [&](int rb, int t, int i) { return M[rb][t][i] * x[rb][t][i]; });
    }
    // ---- feature transformer pass s, decision aggregation ----
    ft_pass<PREC, DT, NT, KA0, R>(ws, L, u, h, lane);
#pragma unroll
    for (int rb = 0; rb < R; ++rb) {
      float ep[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < KD; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const bool dec = 16 * t + 4 * g + i < n_d;
          const float r = dec ? fmaxf(h[rb][t][i], 0.f) : 0.f;
          acc[rb][t][i] += r;
          ep[i] += r;
        }
      const float eta = row_sum((ep[0] + ep[1]) + (ep[2] + ep[3]));
      if constexpr (AGG_LDS) {
#pragma unroll
        for (int t = 0; t < DT; ++t) {
          float a[4];
          own_get(rb, t, a);
#pragma unroll
          for (int i = 0; i < 4; ++i) a[i] += eta * M[rb][t][i];
          own_put(rb, t, a);
        }
      } else {
#pragma unroll
        for (int t = 0; t < DT; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) agg[rb][t][i] += eta * M[rb][t][i];
      }
    }
  }

  // ---- outputs: logits = acc W_fin^T, masks_agg = agg / sum(agg) ----
#pragma unroll
  for (int rb = 0; rb < R; ++rb) {
    const int64_t row = wrow0 + 16 * rb + rl;
    for (int o = 0; o < A.n_out; ++o) {
      const float* wf = wfin_s + o * n_d;
      float part = 0.f;
#pragma unroll
      for (int t = 0; t < KD; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = 16 * t + 4 * g + i;
          if (c < n_d) part += acc[rb][t][i] * wf[c];
        }
      part = row_sum(part);
      if (live[rb] && g == (o & 3)) A.logits[row * A.n_out + o] = part;
    }
    float den = 0.f;
    if constexpr (AGG_LDS) {
#pragma unroll
      for (int t = 0; t < DT; ++t) {
        float a[4];
        own_get(rb, t, a);
#pragma unroll
        for (int i = 0; i < 4; ++i) den += a[i];
      }
    } else {
#pragma unroll
      for (int t = 0; t < DT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) den += agg[rb][t][i];
    }
    den = row_sum(den);
    const float inv = den > 0.f ? 1.0f / den : 0.f;
    if constexpr (RAW) {
#pragma unroll
      for (int t = 0; t < DT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) agg[rb][t][i] *= inv;
      reduce_columns<DT>(agg[rb], A.colbits, C, stage + 16 * rb * C, lane);
    } else if constexpr (AGG_LDS) {
#pragma unroll
      for (int t = 0; t < DT; ++t) {
        float a[4];
        own_get(rb, t, a);
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] *= inv;
        own_put(rb, t, a);
      }
    } else {
      float* sr = stage + (16 * rb + rl) * D + 4 * g;
      if (vec4) {
#pragma unroll
        for (int t = 0; t < DT; ++t)
          if (feat_ok(t, 0))
            *reinterpret_cast<f4*>(sr + 16 * t) =
                f4{agg[rb][t][0] * inv, agg[rb][t][1] * inv, agg[rb][t][2] * inv, agg[rb][t][3] * inv};
      } else {
#pragma unroll
        for (int t = 0; t < DT; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (feat_ok(t, i)) sr[16 * t + i] = agg[rb][t][i] * inv;
      }
    }
  }
  lds_wave_sync();
  stage_out(stage, (RAW ? A.masks_agg + wrow0 * C : A.masks_agg + wrow0 * D), live_rows * (RAW ? C : D), lane);
}

// ------------------------------------------------------------------------------------
// Split-feature kernel for wide models.  One workgroup of W waves carries one block of 16
// rows; wave w owns feature tiles [w TPW, (w + 1) TPW) (x, the prior, the aggregate and
// the mask of those features stay in its registers) and output tile pairs
// [w OPW, (w + 1) OPW) of every feature-transformer layer.  The waves meet in LDS:
//   u_s  the masked input u = M * x, in the B-operand layout of the first layer's GEMM
//        (each wave writes its tiles, every wave reads all of them);
//   h_s  the hidden state h of every layer (FP32), written by the owners of its tiles;
//   ex   per-row partial sums of the sparsemax passes and the aggregate's denominator;
//   st   per-row start bounds of the sparsemax.
// A layer's weights stream as K slices that hold every output pair, so all waves work on
// every chunk; the attentive weights stream as chunks holding TPC feature tiles of every
// wave.  Everything a row computes is in a fixed order, independent of the batch.
template <int PREC, int DT, int NT, int W>
struct WideGeom {
  static constexpr int TPW = wide_tpw(DT, W);     // feature tiles per wave
  static constexpr int DTP = TPW * W;             // padded feature tiles
  static constexpr int OPW = NT / W;              // output tile pairs per wave
  // u in LDS: FP32 tiles (FP32, and the MX and row-coded formats, whose waves code the whole
  // row themselves) or BF16 k-blocks
  static constexpr int UKB = PREC == 0 || is_mx(PREC) || row_coded(PREC) ? DTP : DTP / 2;
  static constexpr int UBYTES = UKB * kFrag;
};

// B operand of k-block kb.  The buffer holds [k-block][64 lanes][16 bytes] in the MFMA
// operand format, or (SRC_F32 with BF16 GEMMs) FP32 tiles [tile][64 lanes][4 floats] that
// are packed here, tile 2 kb and 2 kb + 1 (a tile at or past KT reads as zero).
template <int PREC, bool SRC_F32>
__device__ __forceinline__ void load_kblock(const unsigned char* src, int kb, int KT, int lane, f4& f, s8& b) {
  if constexpr (PREC == 0) {
    f = *reinterpret_cast<const f4*>(src + ((size_t)kb * 64 + lane) * 16);
  } else if constexpr (SRC_F32) {
    const f4 a = *reinterpret_cast<const f4*>(src + ((size_t)(2 * kb) * 64 + lane) * 16);
    f4 c = {0.f, 0.f, 0.f, 0.f};
    if (2 * kb + 1 < KT) c = *reinterpret_cast<const f4*>(src + ((size_t)(2 * kb + 1) * 64 + lane) * 16);
    uint32_t q[4] = {pack_bf16x2(a[0], a[1]), pack_bf16x2(a[2], a[3]), pack_bf16x2(c[0], c[1]),
                     pack_bf16x2(c[2], c[3])};
    b = __builtin_bit_cast(s8, q);
  } else {
    b = *reinterpret_cast<const s8*>(src + ((size_t)kb * 64 + lane) * 16);
  }
}

// One GLU layer of the split-feature kernel.  src: B operands of the layer input, KT
// tiles of K; h: this wave's OPW output tiles (updated in place after the first layer);
// the new h is published to h_s for all waves.
template <int PREC, int KT, int NT, int W, bool SRC_F32, class WS>
__device__ __forceinline__ void glu_layer_wide(WS& ws, const unsigned char* src, unsigned char* h_s, int sk,
                                               float (&h)[NT / W][4], bool first, int lane, int wave) {
  constexpr int OPW = NT / W;
  constexpr int KB = kblocks(PREC, KT);
  constexpr int FB = kbytes(PREC);   // weight bytes of one output tile's k-block
  const int g = lane >> 4;
  f4 av[OPW], ag[OPW];
#pragma unroll
  for (int p = 0; p < OPW; ++p) {
    av[p] = f4{0.f, 0.f, 0.f, 0.f};
    ag[p] = f4{0.f, 0.f, 0.f, 0.f};
  }
  // MX and the row-coded formats: every wave codes the whole layer input (FP32 tiles in
  // LDS) itself, into OCP blocks or with the row's scale (the maximum over all of K)
  BOp<PREC, KT, 1> bm;
  if constexpr (is_mx(PREC) || row_coded(PREC))
    build_b(bm, [&](int, int t, int i) { return reinterpret_cast<const float*>(src + ((size_t)t * 64 + lane) * 16)[i]; });
  for (int kb0 = 0; kb0 < KB; kb0 += sk) {
    const int nkb = KB - kb0 < sk ? KB - kb0 : sk;
    ws.begin();
    const unsigned char* buf = ws.ptr();
    for (int q = 0; q < nkb; ++q) {
      f4 bf = {0.f, 0.f, 0.f, 0.f};
      s8 bb = {}, bb2 = {};
      if constexpr (is_fp8w(PREC)) {
        // an E4M3 k-block spans two BF16 k-blocks of the input (one past the input's
        // last reads as zero)
        const int k2 = 2 * (kb0 + q);
        load_kblock<1, SRC_F32>(src, k2, KT, lane, bf, bb);
        if (k2 + 1 < kblocks(1, KT)) load_kblock<1, SRC_F32>(src, k2 + 1, KT, lane, bf, bb2);
      } else if constexpr (!is_mx(PREC) && !row_coded(PREC)) {
        load_kblock<PREC, SRC_F32>(src, kb0 + q, KT, lane, bf, bb);
      }
#pragma unroll
      for (int p = 0; p < OPW; ++p) {
        const int pr = wave * OPW + p;
        const unsigned char* fv = buf + ((size_t)(pr * 2 + 0) * nkb + q) * FB + lane * 16;
        const unsigned char* fg = buf + ((size_t)(pr * 2 + 1) * nkb + q) * FB + lane * 16;
        if constexpr (is_mx(PREC)) {
          av[p] = mma_kblock_mx<PREC, KT>(fv - lane * 16, bm, kb0 + q, av[p], lane);
          ag[p] = mma_kblock_mx<PREC, KT>(fg - lane * 16, bm, kb0 + q, ag[p], lane);
        } else if constexpr (row_coded(PREC)) {
          av[p] = mma_kblock_rc<PREC, KT>(fv - lane * 16, bm, kb0 + q, av[p], lane);
          ag[p] = mma_kblock_rc<PREC, KT>(fg - lane * 16, bm, kb0 + q, ag[p], lane);
        } else if constexpr (is_fp8w(PREC)) {
          const i4 a = *reinterpret_cast<const i4*>(fv);
          const i4 c = *reinterpret_cast<const i4*>(fg);
          av[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(widen_e4m3x8(a[0], a[1]), bb, av[p], 0, 0, 0);
          ag[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(widen_e4m3x8(c[0], c[1]), bb, ag[p], 0, 0, 0);
          av[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(widen_e4m3x8(a[2], a[3]), bb2, av[p], 0, 0, 0);
          ag[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(widen_e4m3x8(c[2], c[3]), bb2, ag[p], 0, 0, 0);
        } else if constexpr (PREC == 0) {
          const f4 a = *reinterpret_cast<const f4*>(fv);
          const f4 c = *reinterpret_cast<const f4*>(fg);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            av[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r], bf[r], av[p], 0, 0, 0);
            ag[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(c[r], bf[r], ag[p], 0, 0, 0);
          }
        } else {
          av[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const s8*>(fv), bb, av[p], 0, 0, 0);
          ag[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const s8*>(fg), bb, ag[p], 0, 0, 0);
        }
      }
    }
    if (kb0 + nkb == KB) {
      // shifts of every pair follow the fragments of the layer's last slice
      const float* sft = reinterpret_cast<const float*>(buf + (size_t)NT * 2 * nkb * FB);
#pragma unroll
      for (int p = 0; p < OPW; ++p) {
        const int pr = wave * OPW + p;
        const f4 sv = *reinterpret_cast<const f4*>(sft + pr * 32 + 4 * g);
        const f4 sg = *reinterpret_cast<const f4*>(sft + pr * 32 + 16 + 4 * g);
        if constexpr (has_channel_scales(PREC)) {
          // channel scales after all shifts; the gate's scale and shift carry -log2(e); the
          // row-coded formats scale by (channel scale) x (row scale)
          f4 cv = *reinterpret_cast<const f4*>(sft + NT * 32 + pr * 32 + 4 * g);
          f4 cg = *reinterpret_cast<const f4*>(sft + NT * 32 + pr * 32 + 16 + 4 * g);
          f4 qv = av[p], qg = ag[p];
          if constexpr (PREC == 3) {
            qv = i32_sums(qv);
            qg = i32_sums(qg);
          }
          if constexpr (row_coded(PREC)) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              cv[i] *= bm.rscale(0);
              cg[i] *= bm.rscale(0);
            }
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float v = __builtin_fmaf(qv[i], cv[i], sv[i]);
            const float sgm = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(__builtin_fmaf(qg[i], cg[i], sg[i])));
            h[p][i] = first ? v * sgm : __builtin_fmaf(v, sgm, h[p][i]) * kSqrtHalf;
          }
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float v = av[p][i] + sv[i];
            const float sgm = sigmoid_fast(ag[p][i] + sg[i]);
            h[p][i] = first ? v * sgm : __builtin_fmaf(v, sgm, h[p][i]) * kSqrtHalf;
          }
        }
      }
    }
    ws.end();
  }
  // publish this wave's tiles of h (the chunk barrier above ended every read of h_s)
#pragma unroll
  for (int p = 0; p < OPW; ++p)
    *reinterpret_cast<f4*>(h_s + ((size_t)(wave * OPW + p) * 64 + lane) * 16) = f4{h[p][0], h[p][1], h[p][2], h[p][3]};
  lds_block_sync();
}

// u = M * x of this wave's tiles into the B-operand layout of u_s.
template <int PREC, int TPW>
__device__ __forceinline__ void publish_u(unsigned char* u_s, const float (&m)[TPW][4], const float (&x)[TPW][4],
                                          int wave, int lane) {
  if constexpr (PREC == 0 || is_mx(PREC) || row_coded(PREC)) {
#pragma unroll
    for (int t = 0; t < TPW; ++t)
      *reinterpret_cast<f4*>(u_s + ((size_t)(wave * TPW + t) * 64 + lane) * 16) =
          f4{m[t][0] * x[t][0], m[t][1] * x[t][1], m[t][2] * x[t][2], m[t][3] * x[t][3]};
  } else {
#pragma unroll
    for (int t = 0; t < TPW; t += 2) {
      uint32_t q[4] = {pack_bf16x2(m[t][0] * x[t][0], m[t][1] * x[t][1]),
                       pack_bf16x2(m[t][2] * x[t][2], m[t][3] * x[t][3]),
                       pack_bf16x2(m[t + 1][0] * x[t + 1][0], m[t + 1][1] * x[t + 1][1]),
                       pack_bf16x2(m[t + 1][2] * x[t + 1][2], m[t + 1][3] * x[t + 1][3])};
      *reinterpret_cast<uint4*>(u_s + ((size_t)((wave * TPW + t) / 2) * 64 + lane) * 16) =
          uint4{q[0], q[1], q[2], q[3]};
    }
  }
}

// Store this wave's tiles [wave TPW, (wave + 1) TPW) of a 16-row mask block (each lane's
// row scaled by `scale`) to row r at dst_row0 + r D, through 2 KiB of LDS per wave: two
// tiles at a time are laid out as [16 rows][32 floats], and each store instruction then
// writes eight rows' 128 contiguous bytes, whole 128-byte lines when D % 32 == 0 (the
// lanes' own 16-byte pieces would leave every line half-written per instruction).
template <int TPW>
__device__ __forceinline__ void wide_store_rows(const float (&m)[TPW][4], float scale, float* stg, float* dst_row0,
                                                int D, int live_rows, int wave, int lane) {
  const int g = lane >> 4, rl = lane & 15;
#pragma unroll
  for (int t0 = 0; t0 < TPW; t0 += 2) {
    *reinterpret_cast<f4*>(stg + rl * 32 + 4 * g) =
        f4{m[t0][0] * scale, m[t0][1] * scale, m[t0][2] * scale, m[t0][3] * scale};
    *reinterpret_cast<f4*>(stg + rl * 32 + 16 + 4 * g) =
        f4{m[t0 + 1][0] * scale, m[t0 + 1][1] * scale, m[t0 + 1][2] * scale, m[t0 + 1][3] * scale};
    lds_wave_sync();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int r = 8 * k + (lane >> 3), c = (lane & 7) * 4;
      const int f = 16 * (wave * TPW + t0) + c;    // padded tiles past D are not stored
      const f4 v = *reinterpret_cast<const f4*>(stg + r * 32 + c);
      if (r < live_rows && f < D)
        __builtin_nontemporal_store(v, reinterpret_cast<f4*>(dst_row0 + (int64_t)r * D + f));
    }
    lds_wave_sync();
  }
}

// A workgroup holds RG such groups of W waves (RG blocks of 16 rows) that share every
// weight chunk, so the weights stream once per 16 RG rows.  Two waves per SIMD: the
// register budget is 256 per lane in all.
template <int PREC, int DT, int NT, int KA0, int W, int RG>
__global__ void __launch_bounds__(64 * W * RG) __attribute__((amdgpu_waves_per_eu(2)))
tabnet_wide_kernel(FwdArgs A) {
  using G = WideGeom<PREC, DT, NT, W>;
  constexpr int TPW = G::TPW, OPW = G::OPW;
  constexpr int KTA = NT - KA0;
  constexpr int KBA = kblocks(PREC, KTA);
  constexpr int KD = KA0 + 1 < NT ? KA0 + 1 : NT;   // tiles that can hold decision channels
  constexpr Plan PL = make_wide_plan(PREC, DT, NT, KA0, W);
  constexpr int GROUP_LDS = G::UBYTES + NT * kFrag + W * 16 * 8 * 4;
  static_assert(NT * kFrag >= W * 2048, "h_s doubles as 2 KiB of mask staging per wave");
  static_assert(TPW % 2 == 0, "mask staging takes tile pairs");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  const int64_t B = A.B_dev != nullptr ? *A.B_dev : A.B;
  if ((int64_t)blockIdx.x * 16 * RG >= B) return;  // every wave of the workgroup alike
  const int lane = threadIdx.x & 63;
  const int rg = (threadIdx.x >> 6) / W;           // row group
  const int wave = (threadIdx.x >> 6) % W;         // position in the feature split
  const int g = lane >> 4;
  const int rl = lane & 15;
  const int D = A.D, n_d = A.n_d;
  const int64_t row0 = ((int64_t)blockIdx.x * RG + rg) * 16;
  const int live_rows = (int)(B - row0 < 0 ? 0 : (B - row0 > 16 ? 16 : B - row0));
  const bool live = rl < live_rows;
  const int64_t row = row0 + rl;

  unsigned char* u_s = smem + 2 * PL.buf + (size_t)rg * GROUP_LDS;
  unsigned char* h_s = u_s + G::UBYTES;
  float* ex = reinterpret_cast<float*>(h_s + NT * kFrag);   // [2][W][16][2]
  float* st = ex + 2 * W * 16 * 2;                           // [W][16][4]
  float* wfin_s = reinterpret_cast<float*>(smem + 2 * PL.buf + (size_t)RG * GROUP_LDS);
  int* open_s = reinterpret_cast<int*>(wfin_s + A.n_out * n_d);   // [2][RG]: rows still open
  for (int e = threadIdx.x; e < A.n_out * n_d; e += 64 * W * RG) wfin_s[e] = A.wfin[e];

  WeightStream<W * RG, PL.buf> ws;
  ws.lds = smem;
  ws.wts = A.wts;
  ws.tab = A.chunks;
  ws.n = A.n_chunks;
  ws.idx = -1;
  ws.cur = 1;
  ws.begin();

  // ---- input batch norm of this wave's features ----
  float x[TPW][4];
  auto fok = [&](int t, int i) { return 16 * (wave * TPW + t) + 4 * g + i < D; };
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int T = wave * TPW + t;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float v = 0.f, sc = 0.f, sh = 0.f;
      if (T < DT) {
        sc = A.in_affine[16 * T + 4 * g + i];
        sh = A.in_affine[16 * DT + 16 * T + 4 * g + i];
        if (live && fok(t, i)) v = A.X[row * D + 16 * T + 4 * g + i];
      }
      x[t][i] = v * sc + sh;
    }
  }
  float P[TPW][4], agg[TPW][4], M[TPW][4], h[OPW][4], acc[KD][4];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      P[t][i] = 1.f;
      agg[t][i] = 0.f;
      M[t][i] = 1.f;                 // pass 0 reads u = x
    }
#pragma unroll
  for (int p = 0; p < OPW; ++p)
#pragma unroll
    for (int i = 0; i < 4; ++i) h[p][i] = 0.f;
#pragma unroll
  for (int t = 0; t < KD; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[t][i] = 0.f;
  publish_u<PREC, TPW>(u_s, M, x, wave, lane);
  ws.end();                          // first chunk in LDS, u_s visible to every wave
  const int L = A.n_sh + A.n_ind;
  auto ft_pass = [&]() {
    glu_layer_wide<PREC, DT, NT, W, false>(ws, u_s, h_s, PL.sk, h, true, lane, wave);
    for (int l = 1; l < L; ++l) glu_layer_wide<PREC, NT, NT, W, true>(ws, h_s, h_s, PL.sk, h, false, lane, wave);
  };
  ft_pass();

  const int64_t step_stride = B * (int64_t)D;
  for (int s = 1; s <= A.n_steps; ++s) {
    // ---- attentive transformer on this wave's feature tiles ----
    {
      constexpr int KB2 = kblocks(1, KTA);            // BF16 k-blocks of the input
      constexpr int FBA = kbytes(PREC);
      f4 bf[PREC == 0 ? KTA : 1];
      s8 bb[PREC == 0 || is_mx(PREC) || row_coded(PREC) ? 1 : KB2];
      // MX and the row-coded formats: the attention half a = h[n_d, n_d + n_a) in OCP
      // blocks, or coded with the scale of its own channels
      BOp<PREC, KTA, 1> bma;
      if constexpr (is_mx(PREC) || row_coded(PREC)) {
        const int n_att_end = n_d + A.n_a;
        build_b(bma, [&](int, int t, int i) {
          const int ch = 16 * (KA0 + t) + 4 * g + i;
          const float v = reinterpret_cast<const float*>(h_s + ((size_t)(KA0 + t) * 64 + lane) * 16)[i];
          return ch >= n_d && ch < n_att_end ? v : 0.f;
        });
      } else if constexpr (PREC == 0) {
#pragma unroll
        for (int t = 0; t < KTA; ++t) bf[t] = *reinterpret_cast<const f4*>(h_s + ((size_t)(KA0 + t) * 64 + lane) * 16);
      } else {
#pragma unroll
        for (int kb = 0; kb < KB2; ++kb) {
          const f4 a = *reinterpret_cast<const f4*>(h_s + ((size_t)(KA0 + 2 * kb) * 64 + lane) * 16);
          f4 c = {0.f, 0.f, 0.f, 0.f};
          if (2 * kb + 1 < KTA) c = *reinterpret_cast<const f4*>(h_s + ((size_t)(KA0 + 2 * kb + 1) * 64 + lane) * 16);
          uint32_t q[4] = {pack_bf16x2(a[0], a[1]), pack_bf16x2(a[2], a[3]), pack_bf16x2(c[0], c[1]),
                           pack_bf16x2(c[2], c[3])};
          if (2 * kb + 1 >= KTA) q[2] = q[3] = 0u;
          bb[kb] = __builtin_bit_cast(s8, q);
        }
      }
#pragma unroll
      for (int j = 0; j < TPW / PL.tpc; ++j) {
        ws.begin();
        const unsigned char* buf = ws.ptr();
#pragma unroll
        for (int q = 0; q < PL.tpc; ++q) {
          const int t = j * PL.tpc + q;      // compile-time after unrolling
          const unsigned char* unit = buf + (size_t)(wave * PL.tpc + q) * PL.att_unit;
          f4 z = *reinterpret_cast<const f4*>(unit + KBA * FBA + 16 * g);
          if constexpr (is_mx(PREC)) {
#pragma unroll
            for (int kb = 0; kb < KBA; ++kb) z = mma_kblock_mx<PREC, KTA>(unit + kb * FBA, bma, kb, z, lane);
          } else if constexpr (row_coded(PREC)) {
            f4 qa = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < KBA; ++kb) qa = mma_kblock_rc<PREC, KTA>(unit + kb * kFrag, bma, kb, qa, lane);
            if constexpr (PREC == 3) qa = i32_sums(qa);
            const f4 cs = *reinterpret_cast<const f4*>(unit + KBA * kFrag + 64 + 16 * g);
#pragma unroll
            for (int i = 0; i < 4; ++i) z[i] = __builtin_fmaf(qa[i], cs[i] * bma.rscale(0), z[i]);
          } else if constexpr (is_fp8w(PREC)) {
            f4 a8 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < KBA; ++kb) {
              const i4 a = *reinterpret_cast<const i4*>(unit + kb * kFrag + lane * 16);
              a8 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(widen_e4m3x8(a[0], a[1]), bb[2 * kb], a8, 0, 0, 0);
              if (2 * kb + 1 < KB2)
                a8 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(widen_e4m3x8(a[2], a[3]), bb[2 * kb + 1], a8, 0, 0, 0);
            }
            const f4 cs = *reinterpret_cast<const f4*>(unit + KBA * kFrag + 64 + 16 * g);
#pragma unroll
            for (int i = 0; i < 4; ++i) z[i] = __builtin_fmaf(a8[i], cs[i], z[i]);
          } else if constexpr (PREC == 0) {
#pragma unroll
            for (int kt = 0; kt < KTA; ++kt) {
              const f4 a = *reinterpret_cast<const f4*>(unit + kt * kFrag + lane * 16);
#pragma unroll
              for (int r = 0; r < 4; ++r) z = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r], bf[kt][r], z, 0, 0, 0);
            }
          } else {
#pragma unroll
            for (int kb = 0; kb < KBA; ++kb)
              z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const s8*>(unit + kb * kFrag + lane * 16),
                                                         bb[kb], z, 0, 0, 0);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) M[t][i] = fok(t, i) ? P[t][i] * z[i] : kNegBig;
        }
        ws.end();
      }
    }
    // ---- sparsemax over the row, whose features are spread over the W waves ----
    {
      float a1 = kNegBig, a2 = kNegBig, b1 = kNegBig, b2 = kNegBig;
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float w = M[t][i];
          if (i & 1) {
            b2 = __builtin_amdgcn_fmed3f(b1, b2, w);
            b1 = fmaxf(b1, w);
          } else {
            a2 = __builtin_amdgcn_fmed3f(a1, a2, w);
            a1 = fmaxf(a1, w);
          }
        }
      float v[8];
      top8_sorted(fmaxf(a1, b1), fmaxf(fminf(a1, b1), fmaxf(a2, b2)), v);
      // best prefix bound of this wave's candidates (a lower bound of the row's threshold)
      float c = 0.f, best = v[0] - 1.f, vl = v[0];
      int kb = 1;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        c += v[k];
        const float bnd = (c - 1.f) * (1.0f / (float)(k + 1));
        if (bnd > best) {
          best = bnd;
          kb = k + 1;
          vl = v[k];
        }
      }
      if (g == 0) {
        st[(wave * 16 + rl) * 4 + 0] = best;
        st[(wave * 16 + rl) * 4 + 1] = (float)kb;
        st[(wave * 16 + rl) * 4 + 2] = vl;
      }
      lds_block_sync();
      float tau = st[rl * 4 + 0];
      int kbest = (int)st[rl * 4 + 1];
      float vlast = st[rl * 4 + 2];
      for (int w = 1; w < W; ++w) {
        const float b = st[(w * 16 + rl) * 4 + 0];
        if (b > tau) {
          tau = b;
          kbest = (int)st[(w * 16 + rl) * 4 + 1];
          vlast = st[(w * 16 + rl) * 4 + 2];
        }
      }
      int kprev = 0x7fffffff;
      bool done = false;
      bool open = true;               // some row of this group is still open (wave-uniform)
      for (int it = 0; it <= 16 * G::DTP + 1; ++it) {
        float sp[4] = {0.f, 0.f, 0.f, 0.f};
        int kp[4] = {0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < TPW; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const bool in = M[t][i] > tau;
            sp[i] += in ? M[t][i] : 0.f;
            kp[i] += in ? 1 : 0;
          }
        const float smw = row_sum((sp[0] + sp[1]) + (sp[2] + sp[3]));
        const int kw = row_sum((kp[0] + kp[1]) + (kp[2] + kp[3]));
        float* e = ex + (size_t)(it & 1) * W * 16 * 2;
        if (g == 0) {
          e[(wave * 16 + rl) * 2 + 0] = smw;
          e[(wave * 16 + rl) * 2 + 1] = (float)kw;
        }
        if (wave == 0 && lane == 0) open_s[(it & 1) * RG + rg] = open ? 1 : 0;
        lds_block_sync();
        // leave together once no group had an open row after the previous pass
        int any_group = 0;
        for (int q = 0; q < RG; ++q) any_group |= open_s[(it & 1) * RG + q];
        if (!any_group) break;
        float sm = 0.f;
        int k = 0;
        for (int w = 0; w < W; ++w) {
          sm += e[(w * 16 + rl) * 2 + 0];
          k += (int)e[(w * 16 + rl) * 2 + 1];
        }
        if (!done) {
          if (k >= kprev) {
            done = true;
          } else {
            tau = (sm - 1.f) / (float)k;
            kprev = k;
            if (it == 0 && k == kbest && vlast > tau) done = true;
          }
        }
        open = __any(!done);
      }
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) M[t][i] = fmaxf(M[t][i] - tau, 0.f);
    }
    // ---- step mask out (h_s is free from the attentive GEMM until this pass's first layer
    // ends, so it serves as the staging area) ----
    if (A.masks_step != nullptr && (D & 31) == 0) {
      wide_store_rows<TPW>(M, 1.f, reinterpret_cast<float*>(h_s) + wave * 512,
                           A.masks_step + (int64_t)(s - 1) * step_stride + row0 * D, D, live_rows, wave, lane);
    } else if (A.masks_step != nullptr && live) {
      float* dst = A.masks_step + (int64_t)(s - 1) * step_stride + row * D;
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int f0 = 16 * (wave * TPW + t) + 4 * g;
        if (f0 + 3 < D && (D & 3) == 0) {
          __builtin_nontemporal_store(f4{M[t][0], M[t][1], M[t][2], M[t][3]}, reinterpret_cast<f4*>(dst + f0));
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (f0 + i < D) __builtin_nontemporal_store(M[t][i], dst + f0 + i);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) P[t][i] *= A.gamma - M[t][i];
    publish_u<PREC, TPW>(u_s, M, x, wave, lane);
    lds_block_sync();
    ft_pass();
    // ---- decision aggregation: every wave reads the decision half of h from h_s ----
    float ep[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < KD; ++t) {
      const f4 hv = *reinterpret_cast<const f4*>(h_s + ((size_t)t * 64 + lane) * 16);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float r = 16 * t + 4 * g + i < n_d ? fmaxf(hv[i], 0.f) : 0.f;
        acc[t][i] += r;
        ep[i] += r;
      }
    }
    const float eta = row_sum((ep[0] + ep[1]) + (ep[2] + ep[3]));
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) agg[t][i] += eta * M[t][i];
  }

  // ---- outputs ----
  if (wave == 0) {
    for (int o = 0; o < A.n_out; ++o) {
      const float* wf = wfin_s + o * n_d;
      float part = 0.f;
#pragma unroll
      for (int t = 0; t < KD; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = 16 * t + 4 * g + i;
          if (c < n_d) part += acc[t][i] * wf[c];
        }
      part = row_sum(part);
      if (live && g == (o & 3)) A.logits[row * A.n_out + o] = part;
    }
  }
  float dp = 0.f;
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) dp += agg[t][i];
  dp = row_sum(dp);
  if (g == 0) ex[wave * 16 + rl] = dp;
  lds_block_sync();
  float den = 0.f;
  for (int w = 0; w < W; ++w) den += ex[w * 16 + rl];
  const float inv = den > 0.f ? 1.0f / den : 0.f;
  if ((D & 31) == 0) {
    wide_store_rows<TPW>(agg, inv, reinterpret_cast<float*>(h_s) + wave * 512, A.masks_agg + row0 * D, D, live_rows,
                         wave, lane);
  } else if (live) {
    float* dst = A.masks_agg + row * D;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int f0 = 16 * (wave * TPW + t) + 4 * g;
      if (f0 + 3 < D && (D & 3) == 0) {
        __builtin_nontemporal_store(f4{agg[t][0] * inv, agg[t][1] * inv, agg[t][2] * inv, agg[t][3] * inv},
                                    reinterpret_cast<f4*>(dst + f0));
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (f0 + i < D) __builtin_nontemporal_store(agg[t][i] * inv, dst + f0 + i);
      }
    }
  }
}

// ------------------------------------------------------------------------------------
// Compiled shapes.  (DT, NT, KA0) = (ceil(D/16), ceil((n_d+n_a)/16), floor(n_d/16)); R is
// the number of 16-row blocks per wavefront and W the wavefronts per workgroup, both
// fixed per shape so that a row's arithmetic never depends on the batch size.
struct KernelEntry {
  int prec, DT, NT, KA0, R, W;
  bool raw;                  // embeds raw rows and writes masks per raw column
  void (*fn)(FwdArgs);
  Plan plan;                 // plan.wide: split-feature kernel, 16 rows per workgroup
  bool gen = false;          // generic: also serves models with fewer features or hidden channels
};

#define TABNET_SHAPE(P, DT, NT, KA0, R, W)                                                                 \
  {P, DT, NT, KA0, R, W, false, tabnet_forward_kernel<P, DT, NT, KA0, R, W, false>,                      \
   make_plan(P, DT, NT, KA0, chunk_target(DT, R, W))},                                                   \
      {P, DT, NT, KA0, R, W, true, tabnet_forward_kernel<P, DT, NT, KA0, R, W, true>,                    \
       make_plan(P, DT, NT, KA0, chunk_target(DT, R, W))},
// Split-feature kernels for models too wide for the register-resident layout.
// (W waves share out the features of 16 rows; RG such groups per workgroup: R = RG and
// the entry's W counts all W RG waves.)
#define TABNET_WIDE_SHAPE(P, DT, NT, KA0, W, RG)                                                         \
  {P, DT, NT, KA0, RG, W * RG, false, tabnet_wide_kernel<P, DT, NT, KA0, W, RG>,                         \
   make_wide_plan(P, DT, NT, KA0, W)},
#define TABNET_SHAPES(P)          \
  TABNET_SHAPE(P, 1, 1, 0, 1, 4)  \
  TABNET_SHAPE(P, 2, 1, 0, 1, 4)  \
  TABNET_SHAPE(P, 3, 1, 0, 1, 4)  \
  TABNET_SHAPE(P, 4, 1, 0, 1, 4)  \
  TABNET_SHAPE(P, 4, 2, 1, 1, 4)  \
  TABNET_SHAPE(P, 7, 4, 2, 1, 8)
// The 200-feature shape: eight waves per workgroup (two per SIMD, the register state
// partly spilled) beat four (one per SIMD, no spill) by 8-16% in FP32, BF16, both FP8
// forms and MXFP4 (paper_2510_19689_amd/tile_sweep.py), so those take eight, with four
// as the fallback for models whose final map leaves too little LDS (many outputs) or
// whose raw rows do not fit beside eight staging areas.  INT8 and the 8- and 6-bit MX
// forms, which spill far more at two waves per SIMD, take four.
#define TABNET_SHAPE_200(P) TABNET_SHAPE(P, 13, 8, 4, 1, 4)
// Generic entries (FP32, BF16, both FP8 forms, INT8; embedded rows): for a model outside
// the exact families, the smallest compiled DT >= ceil(D / 16) and NT >= ceil((n_d + n_a) / 16)
// with KA0 = floor(n_d / 16), for D <= 512 and n_d + n_a <= 128 (register-resident up to
// D = 208).  They are compiled in translation units of their own (tabnet_generic_*.hip) so
// that the build runs them in parallel.
#define TABNET_GENERIC(P, DT, NT, KA0, W)                                                             \
  {P, DT, NT, KA0, 1, W, false, tabnet_forward_kernel<P, DT, NT, KA0, 1, W, false, true>,            \
   make_plan(P, DT, NT, KA0, chunk_target(DT, 1, W)), true},
// raw-row twins (FP32 and BF16): the embedding gathered in the kernel, masks per raw column
#define TABNET_GENERIC_RAW(P, DT, NT, KA0, W)                                                         \
  {P, DT, NT, KA0, 1, W, true, tabnet_forward_kernel<P, DT, NT, KA0, 1, W, true, true>,              \
   make_plan(P, DT, NT, KA0, chunk_target(DT, 1, W)), true},
#define TABNET_GENERIC_NT_RAW(P, DT, W)                                                               \
  TABNET_GENERIC_RAW(P, DT, 1, 0, W) TABNET_GENERIC_RAW(P, DT, 2, 0, W) TABNET_GENERIC_RAW(P, DT, 2, 1, W)      \
  TABNET_GENERIC_RAW(P, DT, 4, 0, W) TABNET_GENERIC_RAW(P, DT, 4, 1, W) TABNET_GENERIC_RAW(P, DT, 4, 2, W)      \
  TABNET_GENERIC_RAW(P, DT, 4, 3, W) TABNET_GENERIC_RAW(P, DT, 8, 0, W) TABNET_GENERIC_RAW(P, DT, 8, 1, W)      \
  TABNET_GENERIC_RAW(P, DT, 8, 2, W) TABNET_GENERIC_RAW(P, DT, 8, 3, W) TABNET_GENERIC_RAW(P, DT, 8, 4, W)      \
  TABNET_GENERIC_RAW(P, DT, 8, 5, W) TABNET_GENERIC_RAW(P, DT, 8, 6, W) TABNET_GENERIC_RAW(P, DT, 8, 7, W)
#define TABNET_GENERIC_RAW_SET(P)                                                                     \
  TABNET_GENERIC_NT_RAW(P, 4, 8) TABNET_GENERIC_NT_RAW(P, 8, 8) TABNET_GENERIC_NT_RAW(P, 13, 8)                 \
  TABNET_GENERIC_NT_RAW(P, 13, 4)
#define TABNET_GENERIC_NT(P, DT, W)                                                                   \
  TABNET_GENERIC(P, DT, 1, 0, W) TABNET_GENERIC(P, DT, 2, 0, W) TABNET_GENERIC(P, DT, 2, 1, W)      \
  TABNET_GENERIC(P, DT, 4, 0, W) TABNET_GENERIC(P, DT, 4, 1, W) TABNET_GENERIC(P, DT, 4, 2, W)      \
  TABNET_GENERIC(P, DT, 4, 3, W) TABNET_GENERIC(P, DT, 8, 0, W) TABNET_GENERIC(P, DT, 8, 1, W)      \
  TABNET_GENERIC(P, DT, 8, 2, W) TABNET_GENERIC(P, DT, 8, 3, W) TABNET_GENERIC(P, DT, 8, 4, W)      \
  TABNET_GENERIC(P, DT, 8, 5, W) TABNET_GENERIC(P, DT, 8, 6, W) TABNET_GENERIC(P, DT, 8, 7, W)
// Wider models (D <= 512) on the split-feature kernel compiled for 32 feature tiles and 8
// hidden tiles, which masks its features by the runtime D already.
#define TABNET_GENERIC_WIDE(P, KA0)                                                                   \
  {P, 32, 8, KA0, 2, 8, false, tabnet_wide_kernel<P, 32, 8, KA0, 4, 2>, make_wide_plan(P, 32, 8, KA0, 4), true},
// eight waves per workgroup; at DT = 13 four where the LDS does not hold eight staging areas
#define TABNET_GENERIC_SET(P)                                                                         \
  TABNET_GENERIC_NT(P, 4, 8) TABNET_GENERIC_NT(P, 8, 8) TABNET_GENERIC_NT(P, 13, 8) TABNET_GENERIC_NT(P, 13, 4) \
  TABNET_GENERIC_WIDE(P, 0) TABNET_GENERIC_WIDE(P, 1) TABNET_GENERIC_WIDE(P, 2) TABNET_GENERIC_WIDE(P, 3)         \
  TABNET_GENERIC_WIDE(P, 4) TABNET_GENERIC_WIDE(P, 5) TABNET_GENERIC_WIDE(P, 6) TABNET_GENERIC_WIDE(P, 7)

#ifndef TABNET_GENERIC_TU
#define TABNET_SHAPE_200_W8(P) TABNET_SHAPE(P, 13, 8, 4, 1, 8) TABNET_SHAPE(P, 13, 8, 4, 1, 4)

#ifdef TABNET_TILE_SWEEP
// A tile-sweep build (paper_2510_19689_amd/tile_sweep.py) compiles only the candidate
// tiling it times, given as one TABNET_SHAPE or TABNET_WIDE_SHAPE entry, and no generic
// entries.
static const KernelEntry kKernels[] = {TABNET_TILE_SWEEP};
static const KernelEntry* const kGenericTables[] = {nullptr};
static const int* const kGenericCountPtrs[] = {nullptr};
#else
extern const KernelEntry kGenericFp32[], kGenericBf16[], kGenericFp8w[], kGenericFp8[], kGenericInt8[],
    kGenericFp32Raw[], kGenericBf16Raw[];
extern const int kGenericFp32Count, kGenericBf16Count, kGenericFp8wCount, kGenericFp8Count, kGenericInt8Count,
    kGenericFp32RawCount, kGenericBf16RawCount;
static const KernelEntry* const kGenericTables[] = {kGenericFp32, kGenericBf16,    kGenericFp8w,   kGenericFp8,
                                                    kGenericInt8, kGenericFp32Raw, kGenericBf16Raw};
static const int* const kGenericCountPtrs[] = {&kGenericFp32Count,    &kGenericBf16Count, &kGenericFp8wCount,
                                               &kGenericFp8Count,     &kGenericInt8Count, &kGenericFp32RawCount,
                                               &kGenericBf16RawCount};
static const KernelEntry kKernels[] = {TABNET_SHAPES(0) TABNET_SHAPE_200_W8(0) TABNET_SHAPES(1) TABNET_SHAPE_200_W8(1)
                                       TABNET_SHAPES(2) TABNET_SHAPE_200_W8(2) TABNET_SHAPES(3) TABNET_SHAPE_200(3)
                                       TABNET_SHAPES(4) TABNET_SHAPE_200(4) TABNET_SHAPES(5) TABNET_SHAPE_200_W8(5)
                                       TABNET_SHAPES(6) TABNET_SHAPE_200(6) TABNET_SHAPES(7) TABNET_SHAPE_200(7)
                                       TABNET_SHAPES(8) TABNET_SHAPE_200(8) TABNET_SHAPES(9) TABNET_SHAPE_200_W8(9)
                                       TABNET_WIDE_SHAPE(0, 32, 8, 4, 4, 2)
                                           TABNET_WIDE_SHAPE(1, 32, 8, 4, 4, 2)
                                               TABNET_WIDE_SHAPE(9, 32, 8, 4, 4, 2)
                                                   TABNET_WIDE_SHAPE(5, 32, 8, 4, 4, 2)
                                                       TABNET_WIDE_SHAPE(4, 32, 8, 4, 4, 2)
                                                           TABNET_WIDE_SHAPE(7, 32, 8, 4, 4, 2)
                                                               TABNET_WIDE_SHAPE(6, 32, 8, 4, 4, 2)
                                                                   TABNET_WIDE_SHAPE(8, 32, 8, 4, 4, 2)
                                                                       TABNET_WIDE_SHAPE(2, 32, 8, 4, 4, 2)
                                                                           TABNET_WIDE_SHAPE(3, 32, 8, 4, 4, 2)};
#endif

size_t kernel_lds_bytes(const KernelEntry* k, int D, int n_out, int n_d, int C, int tab_lds_len);

// The forward kernel of a model: the first compiled entry of its shape whose LDS holds the
// model (D, n_out, n_d) and whose raw-row twin (same tiling) holds it too without embedding
// tables; else the first that holds the model; else the first entry of the shape, whose
// LDS check then refuses the model.  A shape with no exact entry takes the first generic
// entry (FP32, BF16, both FP8 forms, INT8; embedded rows) with its KA0 and at least its DT
// and NT that holds the model, the smallest DT and then NT first.  With `twin`: the entry of
// the twin's tiling (R, W) and `raw`, so that a raw-row kernel shares the weight chunking of
// the handle's forward kernel (generic kernels have raw-row twins in FP32 and BF16, on the
// register-resident shapes).
const KernelEntry* find_kernel(int prec, int DT, int NT, int KA0, bool raw, int D, int n_out, int n_d,
                               const KernelEntry* twin) {
  auto shape_of = [&](const KernelEntry& e, bool r) {
    return e.prec == prec && e.DT == DT && e.NT == NT && e.KA0 == KA0 && e.raw == r;
  };
  auto fits = [&](const KernelEntry& e) { return kernel_lds_bytes(&e, D, n_out, n_d, 0, 0) <= (size_t)kMaxLdsBytes; };
  if (twin) {
    // the entry of the twin kernel's own shape and tiling (a generic twin's shape is larger
    // than the model's)
    auto same = [&](const KernelEntry& e) {
      return e.prec == prec && e.raw == raw && e.gen == twin->gen && e.DT == twin->DT && e.NT == twin->NT &&
             e.KA0 == twin->KA0 && e.R == twin->R && e.W == twin->W;
    };
    for (const auto& e : kKernels)
      if (same(e)) return &e;
    for (size_t ti = 0; ti < sizeof(kGenericTables) / sizeof(kGenericTables[0]); ++ti)
      if (kGenericTables[ti])
        for (int j = 0; j < *kGenericCountPtrs[ti]; ++j)
          if (same(kGenericTables[ti][j])) return &kGenericTables[ti][j];
    return nullptr;
  }
  const KernelEntry *first = nullptr, *first_fit = nullptr;
  for (const auto& e : kKernels) {
    if (!shape_of(e, raw)) continue;
    if (!first) first = &e;
    if (!fits(e)) continue;
    if (!first_fit) first_fit = &e;
    const KernelEntry* r = nullptr;
    for (const auto& e2 : kKernels)
      if (shape_of(e2, true) && e2.R == e.R && e2.W == e.W) r = &e2;
    if (raw || !r || fits(*r)) return &e;
  }
  if (!first && !raw) {
    const KernelEntry* gen_first = nullptr;
    for (size_t ti = 0; ti < sizeof(kGenericTables) / sizeof(kGenericTables[0]); ++ti) {
      if (!kGenericTables[ti]) continue;
      for (int j = 0; j < *kGenericCountPtrs[ti]; ++j) {
        const KernelEntry& e = kGenericTables[ti][j];
        if (e.raw || e.prec != prec || e.KA0 != KA0 || e.DT < DT || e.NT < NT) continue;
        if (!gen_first) gen_first = &e;
        if (fits(e)) return &e;
      }
    }
    return gen_first;
  }
  return first_fit ? first_fit : first;
}

// LDS of one workgroup: the two weight buffers, the per-wave mask staging areas, the
// final map and, for the raw-row kernels, the feature descriptors (4 D ints, 16-byte
// aligned) and the tables when they are staged.
size_t kernel_lds_bytes(const KernelEntry* k, int D, int n_out, int n_d, int C, int tab_lds_len) {
  (void)C;
  if (k->plan.wide) {
    // weight buffers; per row group u (B-operand layout), h (FP32), the sparsemax exchange
    // and start areas; the final map and the open-row flags
    const int wf = k->plan.W;
    const int dtp = wide_tpw(k->DT, wf) * wf;
    const size_t ub = (size_t)(k->prec == 0 || is_mx(k->prec) || row_coded(k->prec) ? dtp : dtp / 2) * kFrag;
    const size_t group = ub + (size_t)k->NT * kFrag + (size_t)wf * 16 * 8 * 4;
    return 2 * (size_t)k->plan.buf + (size_t)k->R * group + (size_t)n_out * n_d * 4 + 2 * (size_t)k->R * 4;
  }
  const size_t wf = k->raw ? ((size_t)n_out * n_d + 3) / 4 * 4 : (size_t)n_out * n_d;
  return 2 * (size_t)k->plan.buf + ((size_t)k->W * 16 * k->R * D + wf) * sizeof(float) +
         (k->raw ? 4 * (size_t)D * sizeof(int) + (size_t)tab_lds_len * sizeof(float) : 0);
}

// The attribute is a cap, not a reservation: it is set to the whole LDS of a workgroup so
// that models of different widths sharing a kernel never lower each other's cap.
hipError_t prepare_kernel(const KernelEntry* k) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k->fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kMaxLdsBytes);
}

hipError_t launch_forward(const KernelEntry* k, const FwdArgs& a, hipStream_t stream) {
  const int64_t rows_per_block = k->plan.wide ? 16LL * k->R : 16LL * k->R * k->W;
  const int64_t blocks = (a.B + rows_per_block - 1) / rows_per_block;
  hipLaunchKernelGGL(k->fn, dim3((unsigned)blocks), dim3(64 * k->W),
                     kernel_lds_bytes(k, a.D, a.n_out, a.n_d, a.C, a.tab_lds ? a.tab_len : 0), stream, a);
  return hipGetLastError();
}

const Plan* kernel_plan(const KernelEntry* k) { return &k->plan; }
Shape kernel_shape(const KernelEntry* k) { return Shape{k->DT, k->NT, k->KA0}; }
int kernel_waves(const KernelEntry* k) { return k->W; }
#endif  // TABNET_GENERIC_TU

}  // namespace tabnet
