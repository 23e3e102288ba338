// Fused enumeration kernel for gfx950: synthon-row gather and FP32 combine, the
// decoder on MFMA, the per-query objective and bound mask, and a wave-level
// filter that appends only compounds better than the query's running threshold.
//
// Method (Section 4.2-4.3): the compound embedding is the sum of its per-slot
// rows (eq. "factorizer"); the first decoder layer is linear, so it is applied
// once per synthon row when the engine is built (P = U W1^T, the analogue of the
// cached contributions of eq. "apex") and the kernel only sums hoisted rows. The
// remaining layers run per compound: act -> GEMM (MFMA) -> act -> final layer.
//
// Work decomposition: a reaction's compounds form a grid a x b, with a over the
// first slot (or the first two slots of a three-slot reaction, a = i0 * n1 + i1)
// and b over the last slot, id = offset + a * nB + b. A tile is TA values of a
// by TB values of b; the A and B rows of a tile are staged in LDS once and every
// compound of the tile reads them from there. Each wave holds R blocks of 16
// compounds (one a, 16 consecutive b). Its layer-1 activations stay in registers
// in the MFMA B-operand layout for the whole GEMM; the GEMM weights stream
// through LDS in chunks of 16 output neurons, double-buffered and shared by the
// waves of the workgroup; the final layer accumulates chunk by chunk.
//
// MFMA 16x16 layouts used (D = A * B with A 16 x K, B K x 16, lane l, g = l / 16):
//   A: row l % 16, elements k = g * E .. g * E + E - 1 of the step
//   B: column l % 16, same k
//   D: column l % 16, rows 4 g + v for accumulator v = 0..3
// The contraction index may be permuted freely as long as both operands use the
// same order; the engine lays weights out in the order this kernel produces
// activations: lane group g owns k in [g H1/4, (g+1) H1/4), step s covers
// E consecutive values of it.
#pragma once
#include "apex_internal.h"

namespace apex {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(8 * sizeof(int)))) int i32x8;
typedef __attribute__((__vector_size__(2 * sizeof(short)))) short s16x2;

template <int PREC> struct MfmaT;
template <> struct MfmaT<APEX_PREC_FP32> {
  static constexpr int KS = 4, E = 1, EB = 4;
  using frag = float;
  __device__ static inline f32x4 mma(frag a, frag b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct MfmaT<APEX_PREC_BF16> {
  static constexpr int KS = 32, E = 8, EB = 2;
  using frag = bf16x8;
  __device__ static inline f32x4 mma(frag a, frag b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct MfmaT<APEX_PREC_FP8> {
  static constexpr int KS = 128, E = 32, EB = 1;
  using frag = i32x8;
  __device__ static inline f32x4 mma(frag a, frag b, f32x4 c) {
    // E4M3 x E4M3 (format selectors 0); unit scales select the unscaled form.
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
  }
};

// Activation on prescaled inputs. For SiLU the hoisted tables and GEMM biases
// carry a factor c = -log2(e): with h = c x, SiLU(x) * c = h / (1 + 2^h), one
// exp2 and one reciprocal; the factor 1/c is folded into the next layer.
template <int ACT>
__device__ __forceinline__ float act_pre(float h) {
  if constexpr (ACT == APEX_ACT_SILU) {
    float e = __builtin_amdgcn_exp2f(h);
    return h * __builtin_amdgcn_rcpf(1.0f + e);
  } else if constexpr (ACT == APEX_ACT_RELU) {
    return fmaxf(h, 0.0f);
  } else {
    return h;
  }
}

// Objective of one lane group's four heads, then combined across the groups in a
// fixed order; the scoring kernels use the same order, so a compound's objective
// is the same bits in every kernel.
__device__ __forceinline__ float obj_partial(const float* w4, const float* h4) {
  float p = w4[0] * h4[0];
  p = fmaf(w4[1], h4[1], p);
  p = fmaf(w4[2], h4[2], p);
  p = fmaf(w4[3], h4[3], p);
  return p;
}

__device__ __forceinline__ float canon_zero(float o) { return o == 0.0f ? 0.0f : o; }

// Order-preserving map of a float to uint32 (larger float -> larger key).
__device__ __forceinline__ uint32_t ord_f32(float o) {
  uint32_t u = __float_as_uint(o);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ bool key_passes(float o, uint64_t id, float tau_o, uint64_t tau_id) {
  return o > tau_o || (o == tau_o && id <= tau_id);
}

// Conversion of activations into MFMA operand fragments, four values at a time
// (element positions 4 q .. 4 q + 3 of the fragment).
template <int PREC> struct Pack;
template <> struct Pack<APEX_PREC_BF16> {
  __device__ static inline void put4(bf16x8& f, int q, float a, float b, float c, float d, float) {
    f[4 * q + 0] = (__bf16)a;
    f[4 * q + 1] = (__bf16)b;
    f[4 * q + 2] = (__bf16)c;
    f[4 * q + 3] = (__bf16)d;
  }
};
template <> struct Pack<APEX_PREC_FP8> {
  // xs: power-of-two scale; the hardware conversion divides by it and rounds to
  // nearest E4M3 (OCP, max 448). The engine picks xs from the library's exact
  // activation range, so no value overflows.
  __device__ static inline void put4(i32x8& f, int q, float a, float b, float c, float d, float xs) {
    s16x2 v = {0, 0};
    v = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(v, a, b, xs, false);
    v = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(v, c, d, xs, true);
    f[q] = __builtin_bit_cast(int, v);
  }
};

template <int PREC>
__device__ __forceinline__ typename MfmaT<PREC>::frag load_frag(const unsigned char* p) {
  using F = typename MfmaT<PREC>::frag;
  return *reinterpret_cast<const F*>(p);
}

// LDS bytes the fused kernel needs (host and device agree on this). The staged
// synthon rows (activation phase) and the double-buffered GEMM weight chunks
// (GEMM phase) share one region; the final-layer fragments and the GEMM start
// values stay resident.
__host__ __device__ constexpr int enum_lds_bytes(int prec, int h1, int nl, int h2, bool gather) {
  int eb = prec == APEX_PREC_FP32 ? 4 : (prec == APEX_PREC_BF16 ? 2 : 1);
  int ta = prec == APEX_PREC_FP32 ? 8 : (prec == APEX_PREC_BF16 ? 8 : 12);
  int rows = gather ? 0 : (ta + kTileB) * (h1 + kRowPad) * 4;
  int chunk = nl == 2 ? 2 * 16 * h1 * eb : 0;
  int region = rows > chunk ? rows : chunk;
  int wo = nl == 2 ? 16 * h2 * (prec == APEX_PREC_FP32 ? 4 : 2) : (nl == 1 ? 16 * h1 * eb : 0);
  int b2 = nl == 2 ? h2 * 4 : 0;
  return region + wo + b2;
}

__device__ __forceinline__ uint32_t find_reaction(const ReactDev* react, uint32_t n, uint64_t id) {
  uint32_t lo = 0, hi = n;  // last t with id_off <= id
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (react[mid].id_off <= id) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint32_t find_sel(const SelDev* sel, uint32_t n, uint64_t v) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (sel[mid].tile_start <= v) lo = mid; else hi = mid;
  }
  return lo;
}

template <int PREC, int H1, int NL, int ACT, bool GATHER>
__global__ __launch_bounds__(TileShape<PREC>::W * 64)
__attribute__((amdgpu_waves_per_eu(2, 2))) void k_enum(EnumArgs A) {
  using M = MfmaT<PREC>;
  using TS = TileShape<PREC>;
  using Frag = typename M::frag;
  constexpr int W = TS::W, T = W * 64;
  constexpr int R = TS::R, TA = TS::TA, TB = kTileB;
  constexpr int E = M::E;
  constexpr int NS = H1 / M::KS;  // k-steps over the first hidden width
  constexpr int KG = H1 / 4;      // activations per lane group
  constexpr int ROW = H1 + kRowPad;
  constexpr int CHUNK = 16 * H1 * M::EB;  // bytes of one 16-neuron GEMM weight chunk
  constexpr int NPRE = (CHUNK / 16 + T - 1) / T;
  constexpr bool FULL = (CHUNK / 16) % T == 0;  // every thread moves NPRE x 16 bytes
  constexpr int ROWS_BYTES = GATHER ? 0 : (TA + TB) * ROW * 4;
  constexpr int REGION = ROWS_BYTES > (NL == 2 ? 2 * CHUNK : 0) ? ROWS_BYTES : (NL == 2 ? 2 * CHUNK : 0);
  static_assert(NS * E == KG, "layout");
  static_assert(TA == W * R, "tile");

  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  float* sA = reinterpret_cast<float*>(smem);
  float* sB = sA + TA * ROW;
  unsigned char* sW = smem;  // GEMM weight chunks share the region with the staged rows
  unsigned char* sWo = smem + REGION;
  const uint32_t H2 = NL == 2 ? A.H2 : 0;
  float* sB2 = reinterpret_cast<float*>(
      sWo + (NL == 2 ? 16 * H2 * (PREC == APEX_PREC_FP32 ? 4 : 2) : (NL == 1 ? 16 * H1 * M::EB : 0)));

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, j = lane & 15;
  const int NC = NL == 2 ? (int)(H2 / 16) : 0;
  const float S2 = A.pd.scal[0], So = A.pd.scal[1], XS = A.pd.scal[2];

  // Work range of this workgroup. Tiles (or gathered compounds) are split into
  // contiguous runs; consecutive runs go to workgroups on the same XCD (blocks
  // are dispatched to XCDs round robin), so neighbouring tiles share that XCD's L2.
  uint64_t v, vend;
  {
    const uint32_t G = gridDim.x, bid = blockIdx.x;
    const uint32_t per_xcd = G / 8;
    const uint32_t wg = (G % 8 == 0) ? (bid % 8) * per_xcd + bid / 8 : bid;
    if (GATHER) {
      const uint64_t per_wg = W * R * 16;
      v = (uint64_t)wg * per_wg;
      vend = v + per_wg;
      if (v >= A.n_ids) return;
    } else {
      const uint64_t n = A.tile_end - A.tile_begin;
      const uint64_t per = (n + G - 1) / G;
      v = A.tile_begin + (uint64_t)wg * per;
      vend = v + per < A.tile_end ? v + per : A.tile_end;
      if (v >= vend) return;
    }
  }

  // Final-layer fragments and GEMM start values stay in LDS for the whole launch.
  {
    const int wo_bytes = NL == 2 ? 16 * (int)H2 * (PREC == APEX_PREC_FP32 ? 4 : 2) : (NL == 1 ? 16 * H1 * M::EB : 0);
    const uint4* src = reinterpret_cast<const uint4*>(A.pd.wo);
    uint4* dst = reinterpret_cast<uint4*>(sWo);
    for (int i = tid; i < wo_bytes / 16; i += T) dst[i] = src[i];
    if (NL == 2)
      for (int i = tid; i < (int)H2; i += T) sB2[i] = A.pd.b2[i];
    // gather mode stages no rows, so no later barrier precedes the first read
    __syncthreads();
  }
  const uint4* w2g = reinterpret_cast<const uint4*>(A.pd.w2);
  // the prefetched chunk is one SSA vector, so that it stays in registers
  typedef uint32_t PreV __attribute__((ext_vector_type(4 * NPRE)));
  auto pre_put = [](PreV& p, int q, uint4 w) {
    p[4 * q] = w.x; p[4 * q + 1] = w.y; p[4 * q + 2] = w.z; p[4 * q + 3] = w.w;
  };
  auto pre_get = [](const PreV& p, int q) { return make_uint4(p[4 * q], p[4 * q + 1], p[4 * q + 2], p[4 * q + 3]); };

  uint32_t si = 0;
  SelDev S{};
  ReactDev Rt{};
  uint64_t s_end = 0;
  if (!GATHER) {
    si = find_sel(A.sel, A.n_sel, v);
    S = A.sel[si];
    Rt = A.react[S.t];
    s_end = S.tile_start + (uint64_t)((Rt.nA + TA - 1) / TA) * S.tiles_b;
  }

  for (; v < vend; v += (GATHER ? vend : 1)) {
    PreV pre;
    // first GEMM weight chunk: loads issued now, stored after the activation phase
    if (NL == 2) {
#pragma unroll
      for (int q = 0; q < NPRE; ++q) {
        const int i = tid + q * T;
        if (FULL || i < CHUNK / 16) pre_put(pre, q, w2g[i]);
      }
    }
    // ---------------- locate the tile and stage its rows ----------------
    uint32_t a0 = 0, b0 = 0;
    if (!GATHER) {
      while (v >= s_end) {
        ++si;
        S = A.sel[si];
        Rt = A.react[S.t];
        s_end = S.tile_start + (uint64_t)((Rt.nA + TA - 1) / TA) * S.tiles_b;
      }
      const uint64_t lt = v - S.tile_start;
      const uint32_t ta = (uint32_t)(lt / S.tiles_b), tb = (uint32_t)(lt % S.tiles_b);
      a0 = ta * TA;
      b0 = tb * TB;
      constexpr int V4 = H1 / 4;
      for (int idx = tid; idx < (TA + TB) * V4; idx += T) {
        const int row = idx / V4, c4 = idx - row * V4;
        float4 val;
        if (row < TA) {
          uint32_t a = a0 + row;
          a = a < Rt.nA ? a : Rt.nA - 1;
          if (Rt.three) {
            const uint32_t i0 = a / Rt.n1, i1 = a - i0 * Rt.n1;
            const float4 p = reinterpret_cast<const float4*>(A.P + (uint64_t)(Rt.row0 + i0) * H1)[c4];
            const float4 q = reinterpret_cast<const float4*>(A.P + (uint64_t)(Rt.row1 + i1) * H1)[c4];
            val = make_float4(p.x + q.x, p.y + q.y, p.z + q.z, p.w + q.w);
          } else {
            val = reinterpret_cast<const float4*>(A.P + (uint64_t)(Rt.row0 + a) * H1)[c4];
          }
          *reinterpret_cast<float4*>(sA + row * ROW + 4 * c4) = val;
        } else {
          uint32_t b = b0 + (row - TA);
          b = b < Rt.nB ? b : Rt.nB - 1;
          val = reinterpret_cast<const float4*>(A.P + (uint64_t)(Rt.rowB + b) * H1)[c4];
          *reinterpret_cast<float4*>(sB + (row - TA) * ROW + 4 * c4) = val;
        }
      }
      __syncthreads();
    }

    // ---------------- layer-1 activations into registers ----------------
    // Row pointers first; then k-step outermost, rows innermost, so that a
    // B-row value shared by the R rows of a wave is consumed right after its load.
    Frag X[R][NS];
    const float* pa[R];
    const float* pa1[R];
    const float* pb[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      pa1[r] = nullptr;
      if (!GATHER) {
        const int aL = wave * R + r;
        pa[r] = sA + aL * ROW + g * KG;
        pb[r] = sB + j * ROW + g * KG;
      } else {
        uint64_t item = v + (uint64_t)(wave * R + r) * 16 + j;
        item = item < A.n_ids ? item : (uint64_t)A.n_ids - 1;
        const uint64_t id = A.ids[item];
        const uint32_t t = find_reaction(A.react, (uint32_t)A.n_reactions, id);
        const ReactDev rr = A.react[t];
        const uint64_t loc = id - rr.id_off;
        // ids past the library end are clamped to rows in bounds (reported as NaN)
        const uint64_t a64 = loc / rr.nB;
        const uint32_t a = a64 < rr.nA ? (uint32_t)a64 : rr.nA - 1;
        const uint32_t b = (uint32_t)(loc % rr.nB);
        if (rr.three) {
          const uint32_t i0 = a / rr.n1, i1 = a - i0 * rr.n1;
          pa[r] = A.P + (uint64_t)(rr.row0 + i0) * H1 + g * KG;
          pa1[r] = A.P + (uint64_t)(rr.row1 + i1) * H1 + g * KG;
        } else {
          pa[r] = A.P + (uint64_t)(rr.row0 + a) * H1 + g * KG;
        }
        pb[r] = A.P + (uint64_t)(rr.rowB + b) * H1 + g * KG;
      }
    }
    if constexpr (E == 1) {
      // fp32: one activation per step, four steps per 16-byte read
#pragma unroll
      for (int s4 = 0; s4 < NS / 4; ++s4) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          float4 xa = *reinterpret_cast<const float4*>(pa[r] + 4 * s4);
          if (GATHER && pa1[r]) {
            const float4 xq = *reinterpret_cast<const float4*>(pa1[r] + 4 * s4);
            xa = make_float4(xa.x + xq.x, xa.y + xq.y, xa.z + xq.z, xa.w + xq.w);
          }
          const float4 xb = *reinterpret_cast<const float4*>(pb[r] + 4 * s4);
          X[r][4 * s4 + 0] = act_pre<ACT>(xa.x + xb.x);
          X[r][4 * s4 + 1] = act_pre<ACT>(xa.y + xb.y);
          X[r][4 * s4 + 2] = act_pre<ACT>(xa.z + xb.z);
          X[r][4 * s4 + 3] = act_pre<ACT>(xa.w + xb.w);
          asm volatile("" : "+v"(X[r][4 * s4 + 0]), "+v"(X[r][4 * s4 + 1]), "+v"(X[r][4 * s4 + 2]),
                       "+v"(X[r][4 * s4 + 3])::"memory");
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          Frag f;
#pragma unroll
          for (int e4 = 0; e4 < E / 4; ++e4) {
            float4 xa = *reinterpret_cast<const float4*>(pa[r] + s * E + 4 * e4);
            if (GATHER && pa1[r]) {
              const float4 xq = *reinterpret_cast<const float4*>(pa1[r] + s * E + 4 * e4);
              xa = make_float4(xa.x + xq.x, xa.y + xq.y, xa.z + xq.z, xa.w + xq.w);
            }
            const float4 xb = *reinterpret_cast<const float4*>(pb[r] + s * E + 4 * e4);
            Pack<PREC>::put4(f, e4, act_pre<ACT>(xa.x + xb.x), act_pre<ACT>(xa.y + xb.y),
                             act_pre<ACT>(xa.z + xb.z), act_pre<ACT>(xa.w + xb.w), XS);
          }
          asm volatile("" : "+v"(f)::"memory");
          X[r][s] = f;
        }
      }
    }

    // ---------------- decoder layers on MFMA ----------------
    f32x4 hacc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) hacc[r] = f32x4{0.f, 0.f, 0.f, 0.f};

    if constexpr (NL == 0) {
      // One-layer decoder (the paper's linear probe, eq. "apex"): the hoisted rows
      // are the per-synthon head contributions (bias on slot 0), so their sum is
      // the heads; lane group g holds heads 4 g .. 4 g + 3.
      static_assert(PREC == APEX_PREC_FP32 && H1 == 16, "linear decoder: FP32, 16 padded heads");
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) hacc[r][q] = X[r][q];
    } else if constexpr (NL == 1) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const Frag wo = load_frag<PREC>(sWo + (size_t)(s * 64 + lane) * E * M::EB);
#pragma unroll
        for (int r = 0; r < R; ++r) hacc[r] = M::mma(wo, X[r][s], hacc[r]);
      }
    } else {
      // The staged rows are no longer needed: the region takes the weight chunks.
      __syncthreads();
      {
        uint4* dst = reinterpret_cast<uint4*>(sW);
#pragma unroll
        for (int q = 0; q < NPRE; ++q) {
          const int i = tid + q * T;
          if (FULL || i < CHUNK / 16) dst[i] = pre_get(pre, q);
        }
      }
      __syncthreads();

      // One chunk of 16 neurons: prefetch the next chunk, run the GEMM steps into
      // `acc`, and meanwhile finish the previous chunk (activation and its share
      // of the final layer) from `prev`; the two are independent, so the
      // activation's VALU work overlaps the MFMAs.
      uint32_t tprev[R][2];  // even chunk of a pair, packed bf16 (bf16/fp8 final layer)
      // pf: chunk c + 1 exists; a literal at every call, so the pipelined loop
      // body below has no branches and the scheduler can interleave its parts.
      auto gemm = [&](int c, f32x4 (&acc)[R], bool pf) {
        if (pf) {
#pragma unroll
          for (int q = 0; q < NPRE; ++q) {
            const int i = tid + q * T;
            if (FULL || i < CHUNK / 16) pre_put(pre, q, w2g[(size_t)(c + 1) * (CHUNK / 16) + i]);
          }
        }
        const f32x4 binit = *reinterpret_cast<const f32x4*>(sB2 + c * 16 + g * 4);
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = binit;
        const unsigned char* wc = sW + (c & 1) * CHUNK;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const Frag a = load_frag<PREC>(wc + (size_t)(s * 64 + lane) * E * M::EB);
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r] = M::mma(a, X[r][s], acc[r]);
        }
      };
      auto finish = [&](int c, const f32x4 (&acc)[R], bool odd) {  // odd: c & 1, a constant at each call
        float tv[R][4];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            float u = acc[r][q];
            if (PREC == APEX_PREC_FP8) u *= S2;
            tv[r][q] = act_pre<ACT>(u);
          }
        if constexpr (PREC == APEX_PREC_FP32) {
          const float* wof = reinterpret_cast<const float*>(sWo);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float wo = wof[(c * 4 + q) * 64 + lane];
#pragma unroll
            for (int r = 0; r < R; ++r)
              hacc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(wo, tv[r][q], hacc[r], 0, 0, 0);
          }
        } else {
          if (!odd) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
              tprev[r][0] = __builtin_bit_cast(uint32_t, bf16x2{(__bf16)tv[r][0], (__bf16)tv[r][1]});
              tprev[r][1] = __builtin_bit_cast(uint32_t, bf16x2{(__bf16)tv[r][2], (__bf16)tv[r][3]});
            }
          } else {
            const bf16x8 wo = *reinterpret_cast<const bf16x8*>(sWo + (size_t)((c >> 1) * 64 + lane) * 16);
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const bf16x2 p0 = __builtin_bit_cast(bf16x2, tprev[r][0]);
              const bf16x2 p1 = __builtin_bit_cast(bf16x2, tprev[r][1]);
              const bf16x8 xb = {p0[0], p0[1], p1[0], p1[1], (__bf16)tv[r][0], (__bf16)tv[r][1],
                                 (__bf16)tv[r][2], (__bf16)tv[r][3]};
              hacc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wo, xb, hacc[r], 0, 0, 0);
            }
          }
        }
      };
      auto publish = [&](int c, bool pf) {  // prefetched chunk c + 1 -> its LDS buffer
        if (pf) {
          uint4* dst = reinterpret_cast<uint4*>(sW + ((c + 1) & 1) * CHUNK);
#pragma unroll
          for (int q = 0; q < NPRE; ++q) {
            const int i = tid + q * T;
            if (FULL || i < CHUNK / 16) dst[i] = pre_get(pre, q);
          }
        }
        __syncthreads();
      };
      f32x4 accA[R], accB[R];
      gemm(0, accA, true);  // NC >= 2
      publish(0, true);
      int c = 1;
      for (; c + 1 < NC; c += 2) {  // chunks c + 1 and c + 2 <= NC - 1 exist
        gemm(c, accB, true);
        finish(c - 1, accA, false);
        publish(c, true);
        gemm(c + 1, accA, true);
        finish(c, accB, true);
        publish(c + 1, true);
      }
      gemm(c, accB, false);  // c == NC - 1 (NC is even)
      finish(c - 1, accA, false);
      finish(c, accB, true);
      __syncthreads();  // the region is restaged by the next tile
    }

    // ---------------- heads, objective, bounds, filter ----------------
    uint64_t cid[R];  // compound id (tile mode) or list position (gather mode)
    bool valid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!GATHER) {
        const uint32_t a = a0 + wave * R + r, b = b0 + j;
        valid[r] = a < Rt.nA && b < Rt.nB;
        cid[r] = Rt.id_off + (uint64_t)a * Rt.nB + b;
      } else {
        cid[r] = v + (uint64_t)(wave * R + r) * 16 + j;
        valid[r] = cid[r] < A.n_ids;
      }
    }
    float hb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) hb[q] = A.pd.bo[4 * g + q];
    float heads[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) heads[r][q] = fmaf(hacc[r][q], So, hb[q]);

    if constexpr (GATHER) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (valid[r]) {
          float4 o4 = make_float4(heads[r][0], heads[r][1], heads[r][2], heads[r][3]);
          if (A.ids[cid[r]] >= A.n_total) o4 = make_float4(NAN, NAN, NAN, NAN);
          *reinterpret_cast<float4*>(A.heads_out + cid[r] * 16 + 4 * g) = o4;
        }
    } else {
      for (uint32_t qi = 0; qi < A.n_queries; ++qi) {
        const QueryDev* Q = A.queries + qi;
        if (!Q->active) continue;
        if (Q->subset_bits && !((Q->subset_bits[S.t >> 5] >> (S.t & 31)) & 1u)) continue;
        const float tau_o = Q->st->tau_o;
        const uint64_t tau_id = Q->st->tau_id;
        float w4[4], lo4[4], hi4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          w4[q] = Q->w[4 * g + q];
          lo4[q] = Q->lo[4 * g + q];
          hi4[q] = Q->hi[4 * g + q];
        }
        uint32_t n_pass = 0;
        bool pass[R];
        float ov[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          float p = obj_partial(w4, heads[r]);
          int ok = 1;
#pragma unroll
          for (int q = 0; q < 4; ++q) ok &= (heads[r][q] >= lo4[q]) & (heads[r][q] <= hi4[q]);
          // combine the four lane groups: (g0 + g1) + (g2 + g3)
          p = p + __shfl_xor(p, 16);
          p = p + __shfl_xor(p, 32);
          ok &= __shfl_xor(ok, 16);
          ok &= __shfl_xor(ok, 32);
          const float o = canon_zero(p);
          ov[r] = o;
          pass[r] = g == 0 && valid[r] && ok && (o == o) && key_passes(o, cid[r], tau_o, tau_id);
        }
        uint64_t masks[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          masks[r] = __ballot(pass[r]);
          n_pass += (uint32_t)__popcll(masks[r]);
        }
        if (n_pass) {
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(&Q->st->count, n_pass);
          base = __shfl(base, 0);
          const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if (pass[r]) {
              const uint32_t idx = base + (uint32_t)__popcll(masks[r] & below);
              if (idx < Q->cap) {
                Q->cand_o[idx] = ov[r];
                Q->cand_id[idx] = cid[r];
              }
            }
            base += (uint32_t)__popcll(masks[r]);
          }
        }
      }
    }
    if (NL != 2 && !GATHER) __syncthreads();  // staged rows are reused by the next tile
  }
}

}  // namespace apex
