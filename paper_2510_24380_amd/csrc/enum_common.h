// Device helpers shared by the fused enumeration kernels (16x16 FP32 in
// enum_kernel.h, 32x32 BF16/FP8 in enum32_kernel.h) and the scoring, selection
// and lookup kernels: operand vector types, the prescaled activations, the
// objective's summation order, the (objective, id) key order of the threshold
// (eq. "apex_topk": larger objective first, smaller id on ties) and the
// reaction / tile-plan lookups.
#pragma once
#include "apex_internal.h"

namespace apex {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(8 * sizeof(int)))) int i32x8;
typedef __attribute__((__vector_size__(2 * sizeof(short)))) short s16x2;

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

// Objective of four heads, combined across groups of four in a fixed order by
// the callers; every kernel that scores a compound uses the same order, so its
// objective is the same bits in every kernel.
// Epilogue parameters of one query, copied to LDS once per tile launch: the
// threshold and the bounds do not change during a launch (the selections that
// move the threshold run between launches), so each tile reads them from LDS
// instead of through the query's pointers in global memory.
struct QLds {
  float w[kHeadsPad];
  float lo[kHeadsPad];
  float hi[kHeadsPad];
  float tau_o;
  uint32_t active;
  uint64_t tau_id;
  const uint32_t* subset_bits;
};
constexpr int kQLdsBytes = APEX_MAX_FUSED_QUERIES * (int)sizeof(QLds);

// Fills sQ[0, n_queries) (one wave per query, W waves): lanes 0..47 copy w, lo
// and hi, lanes 48..51 the rest. An inactive slot (a server slot without a
// query) may have no state: its threshold is not read.
__device__ __forceinline__ void copy_queries_lds(const EnumArgs& A, QLds* sQ, int wave, int W, int lane) {
  for (uint32_t qi = wave; qi < A.n_queries; qi += W) {
    const QueryDev* Q = A.queries + qi;
    QLds* L = sQ + qi;
    if (lane < 3 * kHeadsPad) {
      const float* src = lane < kHeadsPad ? Q->w : lane < 2 * kHeadsPad ? Q->lo : Q->hi;
      float* dst = lane < kHeadsPad ? L->w : lane < 2 * kHeadsPad ? L->lo : L->hi;
      dst[lane % kHeadsPad] = src[lane % kHeadsPad];
    } else if (lane == 48) {
      L->tau_o = Q->active ? Q->st->tau_o : 0.0f;
    } else if (lane == 49) {
      L->active = Q->active;
    } else if (lane == 50) {
      L->tau_id = Q->active ? Q->st->tau_id : 0ull;
    } else if (lane == 51) {
      L->subset_bits = Q->subset_bits;
    }
  }
}

__device__ __forceinline__ float obj_partial(const float* w4, const float* h4) {
  float p = w4[0] * h4[0];
  p = fmaf(w4[1], h4[1], p);
  p = fmaf(w4[2], h4[2], p);
  p = fmaf(w4[3], h4[3], p);
  return p;
}

__device__ __forceinline__ float canon_zero(float o) { return o == 0.0f ? 0.0f : o; }

// A compound is a candidate only when its objective is a finite number. The
// objective sums every head times its weight (zero weights included, and
// 0 * +-Inf is NaN), so it is finite exactly when every head is.
__device__ __forceinline__ bool finite_obj(float o) { return __builtin_fabsf(o) < __builtin_inff(); }

// Order-preserving map of a float to uint32 (larger float -> larger key).
__device__ __forceinline__ uint32_t ord_f32(float o) {
  uint32_t u = __float_as_uint(o);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ bool key_passes(float o, uint64_t id, float tau_o, uint64_t tau_id) {
  return o > tau_o || (o == tau_o && id <= tau_id);
}

// Conversion of activations into low-precision MFMA operand fragments, four
// values at a time (element positions 4 q .. 4 q + 3 of the fragment).
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

template <typename F>
__device__ __forceinline__ F load_frag(const unsigned char* p) {
  return *reinterpret_cast<const F*>(p);
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

// Dynamic tile sharing of the tile kernels (tile mode with work counters). A
// launch's tiles form eight contiguous regions, one per XCD (workgroups are
// dealt to the XCDs in turn); a workgroup takes kWorkRun tiles at a time from
// its own XCD's region through that region's counter, then from the others once
// that one is used up. XCDs and CUs run at different clocks, and equal static
// shares left the faster ones idle at the end of a launch.
constexpr int kWorkRun = 2;

__device__ __forceinline__ uint64_t uniform64(uint64_t x) {  // workgroup-uniform value into scalar registers
  return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(x >> 32)) << 32) |
         (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)x);
}

// Every thread of the workgroup calls it (it holds a barrier). Thread 0 takes
// the next run into s_run[0..1]; s_run[2] counts the regions found used up
// (zero before the first call). Returns the run as [v, vend), empty when no
// tile is left.
__device__ __forceinline__ void take_tile_run(const EnumArgs& A, uint64_t* s_run, uint64_t& v, uint64_t& vend) {
  if (threadIdx.x == 0) {
    const uint64_t n = A.tile_end - A.tile_begin, reg = (n + 7) / 8;
    const uint32_t home = blockIdx.x % 8;
    uint64_t r0 = 0, r1 = 0, tried = s_run[2];
    for (; tried < 8; ++tried) {
      const uint32_t r = (home + (uint32_t)tried) % 8;
      const uint64_t rb = r * reg, re = rb + reg < n ? rb + reg : n;
      if (rb >= re) continue;
      const uint64_t o = rb + atomicAdd(&A.work[r], (uint32_t)kWorkRun);
      if (o < re) {
        r0 = A.tile_begin + o;
        r1 = A.tile_begin + (o + kWorkRun < re ? o + kWorkRun : re);
        break;
      }
    }
    s_run[0] = r0;
    s_run[1] = r1;
    s_run[2] = tried;
  }
  __syncthreads();
  v = uniform64(s_run[0]);
  vend = uniform64(s_run[1]);
}

// Once per workgroup, after its last run: the last workgroup to finish (every
// other one has taken its last run) leaves the counters at zero for the next
// launch on the stream.
__device__ __forceinline__ void release_tile_counters(const EnumArgs& A) {
  if (threadIdx.x == 0 && atomicAdd(&A.work[8], 1u) == gridDim.x - 1) {
    for (int r = 0; r < 9; ++r) atomicExch(&A.work[r], 0u);
  }
}

}  // namespace apex
