// Fused TabNet inference kernel for gfx950.  Layout and data flow: tabnet_kernel.hpp.
#include "tabnet_kernel.hpp"

namespace tabnet {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kSqrtHalf = 0.70710678118654752f;
constexpr float kNegBig = -3.0e38f;   // score of a padded feature: never in the support

__device__ __forceinline__ float xor_shfl(float v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ int xor_shfl(int v, int m) { return __shfl_xor(v, m, 64); }

// Sum / max over the 4 lanes {r, r+16, r+32, r+48} that hold one row.  IEEE addition is
// commutative, so all four lanes obtain bit-identical results.
__device__ __forceinline__ float row_sum(float v) {
  v += xor_shfl(v, 16);
  v += xor_shfl(v, 32);
  return v;
}
__device__ __forceinline__ int row_sum(int v) {
  v += xor_shfl(v, 16);
  v += xor_shfl(v, 32);
  return v;
}
__device__ __forceinline__ float row_max(float v) {
  v = fmaxf(v, xor_shfl(v, 16));
  v = fmaxf(v, xor_shfl(v, 32));
  return v;
}

// Two floats -> two bfloat16 (round to nearest even) packed low/high in one dword.
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
  typedef float fl2 __attribute__((ext_vector_type(2)));
  fl2 f = {lo, hi};
  bf2 b = __builtin_convertvector(f, bf2);
  return __builtin_bit_cast(uint32_t, b);
}

// logistic(g) = 1 / (1 + 2^(-g log2 e))
__device__ __forceinline__ float sigmoid_fast(float g) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-g * kLog2e));
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

// acc[rb] += W'(tile mt, all K) * B[rb]  for one 16-row output tile.
//   FP32 fragments: per (mt, kt) 64 lanes x float4 (one float per 16x16x4 MFMA).
//   BF16 fragments: per (mt, kb) 64 lanes x 8 bf16 (pairs of K tiles, 16x16x32 MFMA);
//                   an odd trailing K tile is stored as a pair whose second tile is zero.
template <int PREC, int KT, int R>
__device__ __forceinline__ void mma_tile(const unsigned char* __restrict__ wl, int mt,
                                         const BOp<PREC, KT, R>& b, f4 (&acc)[R], int lane) {
  if constexpr (PREC == 0) {
    const f4* w = reinterpret_cast<const f4*>(wl) + (size_t)mt * KT * 64 + lane;
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      f4 a = w[kt * 64];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int rb = 0; rb < R; ++rb)
          acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r], b.v[rb][kt][r], acc[rb], 0, 0, 0);
    }
  } else {
    // K tiles are taken in pairs; an odd trailing tile is paired with zeros (its
    // fragment's upper half is zero on the weight side too).  Only the 16x16x32 BF16
    // MFMA is used on purpose: every accumulator chain has one instruction shape.
    constexpr int KP = (KT + 1) / 2;
    const unsigned char* base = wl + (size_t)mt * KP * 1024;
#pragma unroll
    for (int kb = 0; kb < KP; ++kb) {
      s8 a = *reinterpret_cast<const s8*>(base + (size_t)kb * 1024 + lane * 16);
#pragma unroll
      for (int rb = 0; rb < R; ++rb) {
        const bool full = 2 * kb + 1 < KT;
        uint32_t q[4] = {b.v[rb][2 * kb][0], b.v[rb][2 * kb][1],
                         full ? b.v[rb][full ? 2 * kb + 1 : 0][0] : 0u,
                         full ? b.v[rb][full ? 2 * kb + 1 : 0][1] : 0u};
        s8 bb = __builtin_bit_cast(s8, q);
        acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc[rb], 0, 0, 0);
      }
    }
  }
}

// One GLU layer: h <- GLU(u W'^T + b')  (first layer of a pass)
//            or  h <- (h + GLU(h W'^T + b')) * sqrt(1/2).
// Output tiles 0..NT-1 are the value half, NT..2NT-1 the gate half; value tile mt and
// gate tile mt land in the same lanes and registers, so the GLU is lane-local.
template <int PREC, int KT, int NT, int R>
__device__ __forceinline__ void glu_layer(const unsigned char* __restrict__ wl,
                                          const float* __restrict__ bl,
                                          const BOp<PREC, KT, R>& b, float (&h)[R][NT][4],
                                          bool first, int lane) {
  const int g = lane >> 4;
  float hn[R][NT][4];
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
    const f4 bv = *reinterpret_cast<const f4*>(bl + mt * 16 + 4 * g);
    const f4 bg = *reinterpret_cast<const f4*>(bl + (NT + mt) * 16 + 4 * g);
    f4 av[R], ag[R];
#pragma unroll
    for (int rb = 0; rb < R; ++rb) { av[rb] = bv; ag[rb] = bg; }
    mma_tile<PREC, KT, R>(wl, mt, b, av, lane);
    mma_tile<PREC, KT, R>(wl, NT + mt, b, ag, lane);
#pragma unroll
    for (int rb = 0; rb < R; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float gl = av[rb][i] * sigmoid_fast(ag[rb][i]);
        hn[rb][mt][i] = first ? gl : (h[rb][mt][i] + gl) * kSqrtHalf;
      }
  }
#pragma unroll
  for (int rb = 0; rb < R; ++rb)
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) h[rb][mt][i] = hn[rb][mt][i];
}

// Feature-transformer pass s on input u (DT tiles); result h (NT tiles).
template <int PREC, int DT, int NT, int R>
__device__ __forceinline__ void ft_pass(const FwdArgs& A, int s, const BOp<PREC, DT, R>& u,
                                        float (&h)[R][NT][4], int lane) {
  const int L = A.n_sh + A.n_ind;
  auto lid = [&](int l) { return l < A.n_sh ? l : A.n_sh + s * A.n_ind + (l - A.n_sh); };
  {
    const int id = lid(0);
    glu_layer<PREC, DT, NT, R>(A.wts + A.lt.w[id], A.bias + A.lt.b[id], u, h, true, lane);
  }
  for (int l = 1; l < L; ++l) {
    const int id = lid(l);
    BOp<PREC, NT, R> bh;
#pragma unroll
    for (int rb = 0; rb < R; ++rb)
#pragma unroll
      for (int t = 0; t < NT; ++t) bh.set(rb, t, h[rb][t]);
    glu_layer<PREC, NT, NT, R>(A.wts + A.lt.w[id], A.bias + A.lt.b[id], bh, h, false, lane);
  }
}

// ------------------------------------------------------------------------------------
template <int PREC, int DT, int NT, int KA0, int R>
__global__ void __launch_bounds__(64 * kWaves) tabnet_forward_kernel(FwdArgs A) {
  constexpr int KTA = NT - KA0;   // K tiles of the attentive GEMM (the attention half)
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4;
  const int D = A.D, n_d = A.n_d;
  const int64_t row0 = ((int64_t)blockIdx.x * kWaves + wave) * (16 * R) + (lane & 15);
  int64_t row[R];
  bool live[R];
#pragma unroll
  for (int rb = 0; rb < R; ++rb) {
    row[rb] = row0 + 16 * rb;
    live[rb] = row[rb] < A.B;
  }
  // Is feature 16 t + 4 g + i a real column?  Only the last tile can be partial.
  bool last_ok[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) last_ok[i] = 16 * (DT - 1) + 4 * g + i < D;
  auto feat_ok = [&](int t, int i) { return t < DT - 1 || last_ok[i]; };

  // ---- input batch norm (folded to a per-column affine map) ----
  float x[R][DT][4];
  const bool vec4 = (D & 3) == 0;
#pragma unroll
  for (int t = 0; t < DT; ++t) {
    const f4 sc = *reinterpret_cast<const f4*>(A.in_affine + 16 * t + 4 * g);
    const f4 sh = *reinterpret_cast<const f4*>(A.in_affine + 16 * DT + 16 * t + 4 * g);
#pragma unroll
    for (int rb = 0; rb < R; ++rb) {
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      const float* xr = A.X + row[rb] * D + 16 * t + 4 * g;
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
      for (int i = 0; i < 4; ++i) x[rb][t][i] = v[i] * sc[i] + sh[i];
    }
  }

  float P[R][DT][4], agg[R][DT][4], M[R][DT][4];
  float h[R][NT][4], acc[R][NT][4];
#pragma unroll
  for (int rb = 0; rb < R; ++rb) {
#pragma unroll
    for (int t = 0; t < DT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) { P[rb][t][i] = 1.f; agg[rb][t][i] = 0.f; }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[rb][t][i] = 0.f;
  }

  // ---- pass 0: only its attention half is used ----
  {
    BOp<PREC, DT, R> u;
#pragma unroll
    for (int rb = 0; rb < R; ++rb)
#pragma unroll
      for (int t = 0; t < DT; ++t) u.set(rb, t, x[rb][t]);
    ft_pass<PREC, DT, NT, R>(A, 0, u, h, lane);
  }

  const int64_t step_stride = A.B * (int64_t)D;
  for (int s = 1; s <= A.n_steps; ++s) {
    // ---- attentive transformer: z = P * (a W_att'^T + b_att') ----
    {
      BOp<PREC, KTA, R> ba;
#pragma unroll
      for (int rb = 0; rb < R; ++rb)
#pragma unroll
        for (int t = 0; t < KTA; ++t) ba.set(rb, t, h[rb][KA0 + t]);
      const unsigned char* wa = A.wts + A.lt.aw[s - 1];
      const float* baf = A.bias + A.lt.ab[s - 1];
#pragma unroll
      for (int mt = 0; mt < DT; ++mt) {
        const f4 bv = *reinterpret_cast<const f4*>(baf + mt * 16 + 4 * g);
        f4 za[R];
#pragma unroll
        for (int rb = 0; rb < R; ++rb) za[rb] = bv;
        mma_tile<PREC, KTA, R>(wa, mt, ba, za, lane);
#pragma unroll
        for (int rb = 0; rb < R; ++rb)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            M[rb][mt][i] = feat_ok(mt, i) ? P[rb][mt][i] * za[rb][i] : kNegBig;
      }
    }
    // ---- sparsemax per row: Newton iteration on sum(max(z - tau, 0)) = 1 ----
    // Scores are shifted by the row maximum (w = z - zmax <= 0), the support lies in
    // w > -1, and tau' = tau - zmax starts at its lower bound -1.  Each step sets
    // tau' = (sum_{w > tau'} w - 1) / |{w > tau'}|, which moves tau' up monotonically
    // and stops, exactly, once the support no longer shrinks.
    {
      float tau[R];
      int kprev[R];
      bool done[R];
#pragma unroll
      for (int rb = 0; rb < R; ++rb) {
        float m = kNegBig;
#pragma unroll
        for (int t = 0; t < DT; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) m = fmaxf(m, M[rb][t][i]);
        m = row_max(m);
#pragma unroll
        for (int t = 0; t < DT; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) M[rb][t][i] -= m;   // padded: stays hugely negative
        tau[rb] = -1.f;
        kprev[rb] = 0x7fffffff;
        done[rb] = false;
      }
      for (int it = 0; it <= 16 * DT + 1; ++it) {
        bool any_open = false;
#pragma unroll
        for (int rb = 0; rb < R; ++rb) {
          float sm = 0.f;
          int k = 0;
#pragma unroll
          for (int t = 0; t < DT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const bool in = M[rb][t][i] > tau[rb];
              sm += in ? M[rb][t][i] : 0.f;
              k += in ? 1 : 0;
            }
          sm = row_sum(sm);
          k = row_sum(k);
          if (!done[rb]) {
            if (k >= kprev[rb]) {
              done[rb] = true;
            } else {
              tau[rb] = (sm - 1.f) / (float)k;
              kprev[rb] = k;
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
    // ---- step mask out, prior update, masked input ----
    BOp<PREC, DT, R> u;
#pragma unroll
    for (int rb = 0; rb < R; ++rb) {
#pragma unroll
      for (int t = 0; t < DT; ++t) {
        float uu[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          P[rb][t][i] *= A.gamma - M[rb][t][i];
          uu[i] = M[rb][t][i] * x[rb][t][i];
        }
        u.set(rb, t, uu);
      }
      if (A.masks_step != nullptr && live[rb]) {
        float* mr = A.masks_step + (int64_t)(s - 1) * step_stride + row[rb] * D + 4 * g;
#pragma unroll
        for (int t = 0; t < DT; ++t) {
          if (vec4) {
            if (feat_ok(t, 0)) {
              f4 q = {M[rb][t][0], M[rb][t][1], M[rb][t][2], M[rb][t][3]};
              __builtin_nontemporal_store(q, reinterpret_cast<f4*>(mr + 16 * t));
            }
          } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if (feat_ok(t, i)) __builtin_nontemporal_store(M[rb][t][i], mr + 16 * t + i);
          }
        }
      }
    }
    // ---- feature transformer pass s, decision aggregation ----
    ft_pass<PREC, DT, NT, R>(A, s, u, h, lane);
#pragma unroll
    for (int rb = 0; rb < R; ++rb) {
      float eta = 0.f;
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const bool dec = 16 * t + 4 * g + i < n_d;
          const float r = dec ? fmaxf(h[rb][t][i], 0.f) : 0.f;
          acc[rb][t][i] += r;
          eta += r;
        }
      eta = row_sum(eta);
#pragma unroll
      for (int t = 0; t < DT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) agg[rb][t][i] += eta * M[rb][t][i];
    }
  }

  // ---- outputs: logits = acc W_fin^T, masks_agg = agg / sum(agg) ----
#pragma unroll
  for (int rb = 0; rb < R; ++rb) {
    for (int o = 0; o < A.n_out; ++o) {
      const float* wf = A.wfin + o * n_d;
      float part = 0.f;
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = 16 * t + 4 * g + i;
          if (c < n_d) part += acc[rb][t][i] * wf[c];
        }
      part = row_sum(part);
      if (live[rb] && g == (o & 3)) A.logits[row[rb] * A.n_out + o] = part;
    }
    float den = 0.f;
#pragma unroll
    for (int t = 0; t < DT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) den += agg[rb][t][i];
    den = row_sum(den);
    const float inv = den > 0.f ? 1.0f / den : 0.f;
    if (live[rb]) {
      float* ar = A.masks_agg + row[rb] * D + 4 * g;
#pragma unroll
      for (int t = 0; t < DT; ++t) {
        if (vec4) {
          if (feat_ok(t, 0)) {
            f4 q = {agg[rb][t][0] * inv, agg[rb][t][1] * inv, agg[rb][t][2] * inv,
                    agg[rb][t][3] * inv};
            __builtin_nontemporal_store(q, reinterpret_cast<f4*>(ar + 16 * t));
          }
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (feat_ok(t, i)) __builtin_nontemporal_store(agg[rb][t][i] * inv, ar + 16 * t + i);
        }
      }
    }
  }
}

}  // namespace tabnet

// ------------------------------------------------------------------------------------
// Compiled shapes.  (DT, NT, KA0) = (ceil(D/16), ceil((n_d+n_a)/16), floor(n_d/16)); R is
// the number of 16-row blocks per wavefront, fixed per shape so that a row's arithmetic
// never depends on the batch size.
namespace tabnet {

struct KernelEntry {
  int prec, DT, NT, KA0, R;
  void (*fn)(FwdArgs);
};

#define TABNET_SHAPE(P, DT, NT, KA0, R) {P, DT, NT, KA0, R, tabnet_forward_kernel<P, DT, NT, KA0, R>},
#define TABNET_SHAPES(P)        \
  TABNET_SHAPE(P, 1, 1, 0, 2)   \
  TABNET_SHAPE(P, 2, 1, 0, 2)   \
  TABNET_SHAPE(P, 3, 1, 0, 2)   \
  TABNET_SHAPE(P, 4, 1, 0, 2)   \
  TABNET_SHAPE(P, 4, 2, 1, 1)   \
  TABNET_SHAPE(P, 7, 4, 2, 1)   \
  TABNET_SHAPE(P, 13, 8, 4, 1)

static const KernelEntry kKernels[] = {TABNET_SHAPES(0) TABNET_SHAPES(1)};

const KernelEntry* find_kernel(int prec, int DT, int NT, int KA0) {
  for (const auto& e : kKernels)
    if (e.prec == prec && e.DT == DT && e.NT == NT && e.KA0 == KA0) return &e;
  return nullptr;
}

hipError_t launch_forward(const KernelEntry* k, const FwdArgs& a, hipStream_t stream) {
  const int64_t rows_per_block = 16LL * k->R * kWaves;
  const int64_t blocks = (a.B + rows_per_block - 1) / rows_per_block;
  hipLaunchKernelGGL(k->fn, dim3((unsigned)blocks), dim3(64 * kWaves), 0, stream, a);
  return hipGetLastError();
}

}  // namespace tabnet
