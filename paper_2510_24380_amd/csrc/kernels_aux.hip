// Engine-build kernels (hoist, scales, weight layouts) and the selection kernels
// of the search: candidate scoring, radix select with compaction, rank sort,
// id sampling and id decoding.
#include "enum_common.h"
#include "launch.h"

namespace apex {

// ---------------------------------------------------------------------------
// Hoist (Section 4.3, eq. "apex"): the first decoder layer is linear in the
// compound embedding, so it distributes over the slot sum and is applied once
// per synthon row: P[r] = c * (W1 u_r + [r in slot 0] b1). Tiled FP32 GEMM,
// 64 x 64 outputs per workgroup, k in ascending order for every output.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_hoist(const float* __restrict__ U, uint32_t d, uint64_t rows,
                                               const float* __restrict__ W1, const float* __restrict__ b1,
                                               uint32_t n_w, uint32_t h1, const uint8_t* __restrict__ is_slot0,
                                               float c, float* __restrict__ P) {
  __shared__ float sU[16][65];
  __shared__ float sW[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const uint64_t r0 = (uint64_t)blockIdx.x * 64;
  const uint32_t n0 = blockIdx.y * 64;
  float acc[4][4] = {};
  for (uint32_t k0 = 0; k0 < d; k0 += 16) {
    for (int i = threadIdx.x; i < 16 * 64; i += 256) {
      const int kk = i & 15, rr = i >> 4;
      const uint64_t r = r0 + rr;
      const uint32_t k = k0 + kk;
      sU[kk][rr] = (r < rows && k < d) ? U[r * d + k] : 0.0f;
      const uint32_t n = n0 + rr;
      sW[kk][rr] = (n < n_w && k < d) ? W1[(uint64_t)n * d + k] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sU[kk][ty * 4 + i];
#pragma unroll
      for (int i = 0; i < 4; ++i) b[i] = sW[kk][tx * 4 + i];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[i][q] = fmaf(a[i], b[q], acc[i][q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint64_t r = r0 + ty * 4 + i;
    if (r >= rows) continue;
    const bool s0 = is_slot0[r] != 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t n = n0 + tx * 4 + q;
      if (n < h1) P[r * h1 + n] = c * (acc[i][q] + (s0 && n < n_w ? b1[n] : 0.0f));
    }
  }
}

// Per slot and column: extremes of P over the slot's rows.
__global__ void k_colext(const float* __restrict__ P, uint32_t h1, const uint64_t* __restrict__ slot_row0,
                         const uint32_t* __restrict__ slot_size, float* __restrict__ cmax, float* __restrict__ cmin) {
  const uint32_t slot = blockIdx.x;
  const uint32_t n = blockIdx.y * blockDim.x + threadIdx.x;
  if (n >= h1) return;
  float mx = -INFINITY, mn = INFINITY;
  const uint64_t r0 = slot_row0[slot];
  for (uint32_t i = 0; i < slot_size[slot]; ++i) {
    const float x = P[(r0 + i) * h1 + n];
    if (!(__builtin_fabsf(x) < __builtin_inff())) continue;  // non-finite rows never reach an answer
    mx = fmaxf(mx, x);
    mn = fminf(mn, x);
  }
  cmax[(uint64_t)slot * h1 + n] = mx;
  cmin[(uint64_t)slot * h1 + n] = mn;
}

__device__ inline void atomic_max_nonneg(float* addr, float v) {
  atomicMax(reinterpret_cast<unsigned int*>(addr), __float_as_uint(v));
}

// Largest |activation| any compound can produce in the first hidden layer, from
// the per-slot column extremes: h ranges over [sum of minima, sum of maxima].
__global__ void k_actmax(const float* __restrict__ cmax, const float* __restrict__ cmin, uint32_t h1,
                         const uint32_t* __restrict__ react_slot0, const uint32_t* __restrict__ react_nslots,
                         uint32_t n_react, int act, float c, float* __restrict__ out) {
  const uint32_t t = blockIdx.x;
  const uint32_t n = blockIdx.y * blockDim.x + threadIdx.x;
  if (t >= n_react || n >= h1) return;
  float hi = 0.0f, lo = 0.0f;
  for (uint32_t s = 0; s < react_nslots[t]; ++s) {
    hi += cmax[(uint64_t)(react_slot0[t] + s) * h1 + n];
    lo += cmin[(uint64_t)(react_slot0[t] + s) * h1 + n];
  }
  float m;
  if (act == APEX_ACT_SILU) {
    // tables carry c < 0; x = h / c ranges over [hi / c, lo / c]
    const float x1 = hi / c, x2 = lo / c;
    const float s1 = fabsf(x1 / (1.0f + expf(-x1))), s2 = fabsf(x2 / (1.0f + expf(-x2)));
    m = fabsf(c) * fmaxf(fmaxf(s1, s2), 0.2785f);
  } else if (act == APEX_ACT_RELU) {
    m = fmaxf(hi, 0.0f);
  } else {
    m = fmaxf(fabsf(hi), fabsf(lo));
  }
  if (m < __builtin_inff()) atomic_max_nonneg(out, m);  // a slot without finite rows has no range
}

__global__ void k_absmax(const float* __restrict__ x, uint64_t n, float* __restrict__ out) {
  float m = 0.0f;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(x[i]));
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomic_max_nonneg(out, m);
}

// Power-of-two scale 2^ceil(log2(m / 448)) that maps [0, m] into the E4M3
// range, clamped to [2^-60, 2^60] (1 for an empty or non-finite range).
__device__ inline float pow2_scale(float m) {
  if (!(m > 0.0f) || !(m < __builtin_inff())) return 1.0f;
  return exp2f(fminf(fmaxf(ceilf(log2f(m / 448.0f)), -60.0f), 60.0f));
}

// Scales of one precision. amax: [0] activation range, [1] |W2|, [2] |Wo|.
// scal: [0] S2, [1] So, [2] X conversion scale, [3] 1/s_w2, [4] 1/s_wo.
// The activation and W2 scales are powers of two, so S2 = s_w2 * xs is one
// too and the FP8 GEMM applies it as the MFMA's E8M0 scale of its weight
// operand (E4M3 rounding is relative, so a power-of-two scale loses nothing
// but the top of the range: the largest weight maps into (224, 448]).
__global__ void k_scales(const float* __restrict__ amax, int prec, int nl, float* __restrict__ scal) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float S2 = 1.0f, So = 1.0f, xs = 1.0f, iw2 = 1.0f, iwo = 1.0f;
  if (prec == APEX_PREC_FP8) {
    xs = pow2_scale(amax[0]);
    const float sw2 = pow2_scale(amax[1]);
    const float swo = amax[2] > 0.0f ? amax[2] / 448.0f : 1.0f;
    iw2 = 1.0f / sw2;
    iwo = 1.0f / swo;
    if (nl == 2) S2 = sw2 * xs;
    else So = swo * xs;
  }
  scal[0] = S2;
  scal[1] = So;
  scal[2] = xs;
  scal[3] = iw2;
  scal[4] = iwo;
}

// FP32 operand fragments of a weight matrix W [n_out x n_in] (row-major) for a
// layer whose input activations are in the 16x16 kernel's order: fragment
// (c, s, lane) holds W[16 c + lane % 16][g n_in/4 + s] * mul, g = lane / 16.
__global__ void k_frag_x(const float* __restrict__ W, uint32_t n_out, uint32_t n_in, uint32_t n_chunks, float mul,
                         float* __restrict__ out) {
  const uint32_t ns = n_in / 4;
  const uint64_t total = (uint64_t)n_chunks * ns * 64;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t lane = i % 64;
    const uint32_t s = (i / 64) % ns;
    const uint32_t c = (uint32_t)(i / (64ull * ns));
    const uint32_t row = 16 * c + lane % 16;
    const uint32_t k = (lane / 16) * (n_in / 4) + s;
    out[i] = row < n_out ? W[(uint64_t)row * n_in + k] * mul : 0.0f;
  }
}

// FP32 final-layer fragments when its input is the GEMM output in the 16x16 D
// layout (lane group g holds neurons 4 g + v of every 16-neuron chunk): index
// (c, v, lane) -> Wo[lane % 16][16 c + 4 g + v].
__global__ void k_frag_out_d(const float* __restrict__ Wo, uint32_t H, uint32_t h2, float mul,
                             float* __restrict__ out) {
  const uint32_t total = 16 * h2;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const uint32_t lane = i % 64, v = (i / 64) % 4, c = i / 256;
    const uint32_t head = lane % 16, neuron = 16 * c + 4 * (lane / 16) + v;
    out[i] = head < H ? Wo[(uint64_t)head * h2 + neuron] * mul : 0.0f;
  }
}

template <int PREC> __device__ inline void store_elem(void* base, uint64_t i, float v);
template <> __device__ inline void store_elem<APEX_PREC_BF16>(void* base, uint64_t i, float v) {
  reinterpret_cast<__bf16*>(base)[i] = (__bf16)v;
}
template <> __device__ inline void store_elem<APEX_PREC_FP8>(void* base, uint64_t i, float v) {
  v = fminf(fmaxf(v, -448.0f), 448.0f);
  s16x2 p = {0, 0};
  p = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(p, v, 0.0f, 1.0f, false);
  reinterpret_cast<uint8_t*>(base)[i] = (uint8_t)(__builtin_bit_cast(uint32_t, p) & 0xffu);
}

// Operand fragments for the 32x32 kernel (BF16, FP8): A fragment (c, s, lane, e)
// holds W[32 c + lane % 32][h n_in/2 + s E + e] * mul, h = lane / 32 (rows at or
// beyond n_out are zero). Each k-step of a chunk is 64 lanes x 16 bytes per
// 1 KB block: BF16 (E = 8) fills one block, lane-major; FP8 (E = 32 bytes per
// lane) fills two, elements 0..15 of every lane, then 16..31, so each of a
// lane's two 16-byte LDS reads covers 1 KB contiguously (no bank conflicts).
template <int PREC>
__global__ void k_frag_x32(const float* __restrict__ W, uint32_t n_out, uint32_t n_in, uint32_t n_chunks,
                           const float* __restrict__ mul_dev, float mul, void* __restrict__ out) {
  constexpr uint32_t E = PREC == APEX_PREC_BF16 ? 8 : 32;
  const uint32_t ns = n_in / (2 * E);
  const uint64_t total = (uint64_t)n_chunks * ns * 64 * E;
  const float m = mul * (mul_dev ? *mul_dev : 1.0f);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t e = PREC == APEX_PREC_BF16 ? i % E : (i % 16) + 16 * ((i / 1024) % 2);
    const uint32_t lane = PREC == APEX_PREC_BF16 ? (i / E) % 64 : (i / 16) % 64;
    const uint32_t s = (i / ((uint64_t)E * 64)) % ns;
    const uint32_t c = (uint32_t)(i / ((uint64_t)E * 64 * ns));
    const uint32_t row = 32 * c + lane % 32;
    const uint32_t k = (lane / 32) * (n_in / 2) + s * E + e;
    const float v = row < n_out ? W[(uint64_t)row * n_in + k] * m : 0.0f;
    store_elem<PREC>(out, i, v);
  }
}

// Final-layer fragments (BF16) of the 32x32 kernel, whose input is the GEMM
// output in the 32x32 D layout: fragment (c, st, lane, e) holds
// Wo[lane % 32][32 c + d32_row(8 st + e, lane / 32)] * mul (zero for padding heads).
__global__ void k_frag_out32(const float* __restrict__ Wo, uint32_t H, uint32_t h2, uint32_t h2k, float mul,
                             __bf16* __restrict__ out) {
  const uint32_t total = 32 * h2k;  // (h2k / 32) chunks x 2 steps x 64 lanes x 8; neurons >= h2 are zero
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const uint32_t e = i % 8, lane = (i / 8) % 64, st = (i / 512) % 2, c = i / 1024;
    const uint32_t head = lane % 32, hh = lane / 32;
    const uint32_t v = 8 * st + e;
    const uint32_t neuron = 32 * c + 8 * (v >> 2) + 4 * hh + (v & 3);
    out[i] = (__bf16)(head < H && neuron < h2 ? Wo[(uint64_t)head * h2 + neuron] * mul : 0.0f);
  }
}

// GEMM accumulator start values c * b2 (zero for padding neurons h2 .. h2k - 1;
// the GEMM's scale S2 multiplies only the product), and the padded final bias.
__global__ void k_bias(const float* __restrict__ b2, uint32_t h2, uint32_t h2k, float c, const float* __restrict__ scal,
                       const float* __restrict__ bo, uint32_t H, float* __restrict__ b2_out,
                       float* __restrict__ bo_out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (b2 && i < h2k) b2_out[i] = i < h2 ? c * b2[i] : 0.0f;
  if (i < kHeadsPad) bo_out[i] = i < H ? bo[i] : 0.0f;
}

// ---------------------------------------------------------------------------
// Scoring of gathered heads (objective in the fused kernel's order) and append.
// ---------------------------------------------------------------------------
__device__ inline float objective16(const float* w, const float* h) {
  float p[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) p[g] = obj_partial(w + 4 * g, h + 4 * g);
  return canon_zero((p[0] + p[1]) + (p[2] + p[3]));
}

// Scores listed compounds for each query (objective, bounds, the query's reaction
// subset, threshold) and appends the passing ones to its candidate buffer. The
// appends of a workgroup take one atomic on the query's counter (a wave prefix
// in LDS), so a sample in which most compounds pass does not serialise on it.
// n_src (optional): the list holds min(n, n_src->count) entries, a count known
// only on the device.
constexpr int kScoreThreads = 1024;
__global__ __launch_bounds__(kScoreThreads) void k_score(const float* __restrict__ heads,
                                                        const uint64_t* __restrict__ ids, uint32_t n_max,
                                                        const QState* __restrict__ n_src,
                                                        const QueryDev* __restrict__ qs, uint32_t nq,
                                                        const ReactDev* __restrict__ react, uint32_t n_react) {
  __shared__ uint32_t wave_count[kScoreThreads / 64];
  __shared__ uint32_t block_base;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t q = blockIdx.y;
  if (q >= nq) return;  // uniform per workgroup
  const QueryDev* Q = qs + q;
  if (!Q->active) return;
  const uint32_t n = n_src ? min(n_max, n_src->count) : n_max;
  bool pass = false;
  float o = 0.0f;
  uint64_t id = 0;
  if (i < n && Q->subset_bits) {
    const uint32_t t = find_reaction(react, n_react, ids[i]);
    if (!((Q->subset_bits[t >> 5] >> (t & 31)) & 1u)) id = ~0ull;  // outside the query's reactions
  }
  if (i < n && id != ~0ull) {
    float h[kHeadsPad];
    const float4* h4 = reinterpret_cast<const float4*>(heads + (uint64_t)i * kHeadsPad);
#pragma unroll
    for (int k4 = 0; k4 < kHeadsPad / 4; ++k4) {
      const float4 v = h4[k4];
      h[4 * k4] = v.x;
      h[4 * k4 + 1] = v.y;
      h[4 * k4 + 2] = v.z;
      h[4 * k4 + 3] = v.w;
    }
    o = objective16(Q->w, h);
    bool ok = finite_obj(o);
#pragma unroll
    for (int k = 0; k < kHeadsPad; ++k) ok = ok && h[k] >= Q->lo[k] && h[k] <= Q->hi[k];
    id = ids[i];
    pass = ok && key_passes(o, id, Q->st->tau_o, Q->st->tau_id);
  }
  const uint64_t m = __ballot(pass);
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wave_count[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int w = 0; w < kScoreThreads / 64; ++w) tot += wave_count[w];
    block_base = tot ? atomicAdd(&Q->st->count, tot) : 0u;
  }
  __syncthreads();
  if (pass) {
    uint32_t base = block_base;
    for (uint32_t w = 0; w < wave; ++w) base += wave_count[w];
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint32_t idx = base + (uint32_t)__popcll(m & below);
    if (idx < Q->cap) {
      Q->cand_o[idx] = o;
      Q->cand_id[idx] = id;
    }
  }
}

// Heads of the final answer of a low-precision search: every answer id is one of
// the rescored pool's ids, whose FP32 heads were already computed. One wave per
// answer id scans the pool's ids (pool ids are distinct) and copies the row.
// The pool holds min(pool_max, pool_src->count) entries and the answer
// min(want_max, want_src->count), counts known only on the device.
constexpr int kLookupThreads = 256;
__global__ __launch_bounds__(kLookupThreads) void k_pool_lookup(const uint64_t* __restrict__ pool_id,
                                                               const float* __restrict__ pool_heads,
                                                               uint32_t pool_max, const QState* __restrict__ pool_src,
                                                               const uint64_t* __restrict__ want, uint32_t want_max,
                                                               const QState* __restrict__ want_src,
                                                               float* __restrict__ out) {
  const uint32_t n_pool = min(pool_max, pool_src->count);
  const uint32_t n_want = min(want_max, want_src->count);
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t w = (blockIdx.x * kLookupThreads + threadIdx.x) >> 6;
  if (w >= n_want) return;  // uniform per wave
  const uint64_t id = want[w];
  uint32_t pos = UINT32_MAX;
  for (uint32_t t = lane; t < n_pool; t += 64)
    if (pool_id[t] == id) pos = t;
  const uint64_t hit = __ballot(pos != UINT32_MAX);
  if (!hit) return;
  const uint32_t src = (uint32_t)__shfl((int)pos, __ffsll((long long)hit) - 1);
  if (lane < kHeadsPad) out[(uint64_t)w * kHeadsPad + lane] = pool_heads[(uint64_t)src * kHeadsPad + lane];
}

// ---------------------------------------------------------------------------
// Selection over a query's candidate buffer: keep exactly the K best keys
// (objective desc, id asc) and raise the threshold to the K-th best key.
// After a pass over a chunk:
//  - more entries than the buffer holds: the chunk's appends are dropped, the
//    threshold is raised to the K-th best key among what was written (a valid
//    lower bound of the final K-th key) and the chunk is flagged for a re-run;
//  - more than the high-water mark (or `force`): compaction to the K best;
//  - otherwise: nothing but bookkeeping.
// Four launches, each deciding from the same state whether the select runs:
//  1. k_sel_plan (one workgroup): sorts a strided sample of the keys and places
//     kSelPivots pivots around the sample position of the K-th key;
//  2. k_sel_count (many workgroups): exact counts of keys above each pivot;
//  3. k_sel_compact (many workgroups): with the tightest pair of pivots that
//     encloses the K-th key, keys above the upper one go to the output
//     directly and keys between the two to the bracket buffer;
//  4. k_select (one workgroup): sorts the bracket in LDS, completes the K best
//     and updates the state. Small buffers, and brackets that do not fit, take
//     a one-workgroup radix select instead (exact for any key distribution).
// ---------------------------------------------------------------------------
__device__ inline float unord_f32(uint32_t k) {
  const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(u);
}

// (key desc, id asc): a ranks before b
__device__ __forceinline__ bool ranks_before(uint32_t ka, uint64_t ia, uint32_t kb, uint64_t ib) {
  return ka > kb || (ka == kb && ia < ib);
}

struct SelPlan {
  uint32_t n;   // valid entries
  bool run;     // a selection happens in this call
  bool over;    // the chunk overflowed the buffer
};

__device__ inline SelPlan sel_plan(const QueryDev& Q, int force) {
  const QState* st = Q.st;
  const uint32_t count = st->count;
  SelPlan p;
  p.over = count > Q.cap;
  p.n = p.over ? Q.cap : count;
  p.run = p.over || (force ? p.n > Q.K : count > Q.hwm);
  return p;
}

constexpr uint32_t kSelPivotMin = 12288;  // smaller buffers take the radix path
constexpr uint32_t kSelGrid = 128;        // workgroups per query of the counting passes
constexpr uint32_t kSelPassThreads = 256;

// The bracket: the lowest pivot u with fewer than K keys above it (keys above u
// are all kept; none: u = "infinity") and the highest pivot l with at least K
// keys at or above it (the K-th key is >= l; none: l = 0). Keys in [l, u]
// number cnt_ge(l) - cnt_gt(u).
struct Bracket {
  uint32_t u, l, above, total;  // total: keys >= l
  bool u_inf;
  bool fits;
};

__device__ inline Bracket sel_bracket(const SelScratch* S, uint32_t n, uint32_t K) {
  Bracket b;
  b.u = 0xffffffffu;
  b.u_inf = true;
  b.above = 0;
  for (int j = 0; j < kSelPivots; ++j)
    if (S->cnt_gt[j] < K) {
      b.u = S->piv[j];
      b.u_inf = false;
      b.above = S->cnt_gt[j];
    }
  b.l = 0;
  b.total = n;
  for (int j = kSelPivots - 1; j >= 0; --j)
    if (S->cnt_ge[j] >= K) {
      b.l = S->piv[j];
      b.total = S->cnt_ge[j];
    }
  b.fits = b.total - b.above <= kSelBracket;
  return b;
}

// Float4 range [b4, e4) of this workgroup's share of n entries (the n % 4
// tail goes to workgroup 0 as single entries).
__device__ inline void sel_share(uint32_t n, uint32_t& b4, uint32_t& e4) {
  const uint32_t n4 = n / 4;
  const uint32_t per = (n4 + gridDim.x - 1) / gridDim.x;
  b4 = min(n4, blockIdx.x * per);
  e4 = min(n4, b4 + per);
}

__global__ __launch_bounds__(kSelectThreads) void k_sel_plan(const QueryDev* __restrict__ qs, int force) {
  const QueryDev Q = qs[blockIdx.x];
  if (!Q.active) return;
  const SelPlan p = sel_plan(Q, force);
  if (!p.run) return;
  SelScratch* S = Q.sel;
  const uint32_t tid = threadIdx.x;
  if (p.n < kSelPivotMin) {
    if (tid == 0) S->mode = 1;
    return;
  }
  __shared__ uint32_t samp[kSelSample];
  for (uint32_t i = tid; i < kSelSample; i += kSelectThreads)
    samp[i] = ord_f32(Q.cand_o[((uint64_t)i * p.n) / kSelSample]);
  if (tid < kSelPivots) {
    S->cnt_gt[tid] = 0;
    S->cnt_ge[tid] = 0;
  }
  if (tid == 0) {
    S->pos_sure = 0;
    S->pos_br = 0;
    S->mode = 0;
  }
  __syncthreads();
  // bitonic sort, descending
  for (uint32_t size = 2; size <= kSelSample; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t t = tid; t < kSelSample / 2; t += kSelectThreads) {
        const uint32_t i = 2 * t - (t & (stride - 1)), j = i + stride;
        const bool desc = (i & size) == 0;
        const uint32_t a = samp[i], b = samp[j];
        if ((a < b) == desc) {
          samp[i] = b;
          samp[j] = a;
        }
      }
      __syncthreads();
    }
  }
  // pivots at sample positions r + d * 4 sd around the expected position r of
  // the K-th key (sd: binomial spread of that position)
  if (tid < kSelPivots) {
    const float d[kSelPivots] = {-4.0f, -2.0f, -1.0f, -0.25f, 0.25f, 1.0f, 2.0f, 4.0f};
    const float r = (float)Q.K * kSelSample / (float)p.n;
    const float sd = sqrtf(fmaxf(r * (1.0f - r / kSelSample), 0.0f)) + 1.0f;
    const float pos = fminf(fmaxf(r + d[tid] * 4.0f * sd, 0.0f), (float)(kSelSample - 1));
    S->piv[tid] = samp[(uint32_t)pos];
  }
}

__global__ __launch_bounds__(kSelPassThreads) void k_sel_count(const QueryDev* __restrict__ qs, int force) {
  const QueryDev Q = qs[blockIdx.y];
  if (!Q.active) return;
  const SelPlan p = sel_plan(Q, force);
  if (!p.run) return;
  SelScratch* S = Q.sel;
  if (S->mode) return;
  __shared__ uint32_t part[2 * kSelPivots];
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  if (tid < 2 * kSelPivots) part[tid] = 0;
  uint32_t pv[kSelPivots];
#pragma unroll
  for (int j = 0; j < kSelPivots; ++j) pv[j] = S->piv[j];
  __syncthreads();
  uint32_t gt[kSelPivots] = {}, ge[kSelPivots] = {};
  auto add = [&](float o) {
    const uint32_t kf = ord_f32(o);
#pragma unroll
    for (int j = 0; j < kSelPivots; ++j) {
      gt[j] += kf > pv[j];
      ge[j] += kf >= pv[j];
    }
  };
  uint32_t b4, e4;
  sel_share(p.n, b4, e4);
  const float4* o4 = reinterpret_cast<const float4*>(Q.cand_o);
  for (uint32_t i = b4 + tid; i < e4; i += kSelPassThreads) {
    const float4 v = o4[i];
    add(v.x);
    add(v.y);
    add(v.z);
    add(v.w);
  }
  if (blockIdx.x == 0 && tid < p.n % 4) add(Q.cand_o[4 * (p.n / 4) + tid]);
#pragma unroll
  for (int j = 0; j < kSelPivots; ++j) {
    uint32_t a = gt[j], b = ge[j];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      a += __shfl_xor(a, d);
      b += __shfl_xor(b, d);
    }
    if (lane == 0) {
      atomicAdd(&part[j], a);
      atomicAdd(&part[kSelPivots + j], b);
    }
  }
  __syncthreads();
  if (tid < kSelPivots) {
    atomicAdd(&S->cnt_gt[tid], part[tid]);
    atomicAdd(&S->cnt_ge[tid], part[kSelPivots + tid]);
  }
}

__global__ __launch_bounds__(kSelPassThreads) void k_sel_compact(const QueryDev* __restrict__ qs, int force) {
  const QueryDev Q = qs[blockIdx.y];
  if (!Q.active) return;
  const SelPlan p = sel_plan(Q, force);
  if (!p.run) return;
  SelScratch* S = Q.sel;
  if (S->mode) return;
  const Bracket br = sel_bracket(S, p.n, Q.K);
  if (!br.fits) return;
  constexpr uint32_t NW = kSelPassThreads / 64;
  __shared__ uint32_t w_sure[NW], w_br[NW], s_base[2];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  uint32_t b4, e4;
  sel_share(p.n, b4, e4);
  const float4* o4 = reinterpret_cast<const float4*>(Q.cand_o);
  // one extra round in workgroup 0 for the n % 4 tail; trip count uniform per
  // workgroup (barriers inside)
  const uint32_t rounds = (e4 - b4 + kSelPassThreads - 1) / kSelPassThreads + (blockIdx.x == 0 ? 1 : 0);
  for (uint32_t r = 0; r < rounds; ++r) {
    float o[4];
    uint32_t idx[4];
    bool ok[4];
    const bool tail = blockIdx.x == 0 && r + 1 == rounds;
    if (!tail) {
      const uint32_t i = b4 + r * kSelPassThreads + tid;
      const bool in = i < e4;
      const float4 v = in ? o4[i] : make_float4(0.f, 0.f, 0.f, 0.f);
      o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        idx[c] = 4 * i + c;
        ok[c] = in;
      }
    } else {
      const uint32_t i = 4 * (p.n / 4) + tid;
      const bool in = tid < p.n % 4;
      o[0] = in ? Q.cand_o[i] : 0.0f;
      idx[0] = i;
      ok[0] = in;
#pragma unroll
      for (int c = 1; c < 4; ++c) {
        o[c] = 0.0f;
        idx[c] = 0;
        ok[c] = false;
      }
    }
    uint64_t ms[4], mb[4];
    uint32_t ns = 0, nb = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t kf = ord_f32(o[c]);
      const bool sure = ok[c] && !br.u_inf && kf > br.u;
      const bool inb = ok[c] && kf >= br.l && (br.u_inf || kf <= br.u);
      ms[c] = __ballot(sure);
      mb[c] = __ballot(inb);
      ns += (uint32_t)__popcll(ms[c]);
      nb += (uint32_t)__popcll(mb[c]);
    }
    if (lane == 0) {
      w_sure[wave] = ns;
      w_br[wave] = nb;
    }
    __syncthreads();
    if (tid == 0) {
      uint32_t ts = 0, tb = 0;
      for (uint32_t w = 0; w < NW; ++w) {
        ts += w_sure[w];
        tb += w_br[w];
      }
      s_base[0] = ts ? atomicAdd(&S->pos_sure, ts) : 0u;
      s_base[1] = tb ? atomicAdd(&S->pos_br, tb) : 0u;
    }
    __syncthreads();
    uint32_t qs_ = s_base[0], qb = s_base[1];
    for (uint32_t w = 0; w < wave; ++w) {
      qs_ += w_sure[w];
      qb += w_br[w];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if ((ms[c] >> lane) & 1) {  // fewer than K of these in all
        const uint32_t q = qs_ + (uint32_t)__popcll(ms[c] & below);
        Q.tmp_o[q] = o[c];
        Q.tmp_id[q] = Q.cand_id[idx[c]];
      }
      if ((mb[c] >> lane) & 1) {  // at most kSelBracket of these in all
        const uint32_t q = qb + (uint32_t)__popcll(mb[c] & below);
        S->br_key[q] = ord_f32(o[c]);
        S->br_id[q] = Q.cand_id[idx[c]];
      }
      qs_ += (uint32_t)__popcll(ms[c]);
      qb += (uint32_t)__popcll(mb[c]);
    }
    __syncthreads();  // w_sure / w_br are rewritten by the next round
  }
}

// Adds one to hist[digit] for every active lane. Lanes of a wave that share a
// digit add together (candidate keys are nearly sorted by magnitude, so most of
// a wave falls into one or two bins and plain LDS atomics would serialise);
// the few lanes left after four rounds add individually. Every lane of the
// wave must call it.
__device__ inline void hist_add(uint32_t* hist, uint32_t digit, bool active) {
  const uint32_t lane = threadIdx.x & 63;
  bool pending = active;
  for (int it = 0; it < 4; ++it) {
    const uint64_t todo = __ballot(pending);
    if (!todo) return;
    const int leader = __ffsll((long long)todo) - 1;
    const uint32_t d = (uint32_t)__shfl((int)digit, leader);
    const bool mine = pending && digit == d;
    const uint64_t same = __ballot(mine);
    if ((int)lane == leader) atomicAdd(&hist[d], (uint32_t)__popcll(same));
    pending = pending && !mine;
  }
  if (pending) atomicAdd(&hist[digit], 1u);
}

// Calls f(value, index, valid) for every index in [0, n) of a candidate
// objective array, with all lanes of the workgroup in step (f may use ballots).
// Each thread keeps four 16-byte loads in flight, so that one workgroup moves
// enough bytes to stay off the memory latency.
template <class F>
__device__ inline void scan_objectives(const float* __restrict__ o, uint32_t n, F&& f) {
  constexpr uint32_t U = 4;
  const uint32_t nq = n / 4;
  const float4* o4 = reinterpret_cast<const float4*>(o);
  for (uint32_t base = 0; base < nq; base += U * kSelectThreads) {
    float4 v[U];
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      const uint32_t qi = base + u * kSelectThreads + threadIdx.x;
      v[u] = qi < nq ? o4[qi] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      const uint32_t qi = base + u * kSelectThreads + threadIdx.x;
      const bool ok = qi < nq;
      f(v[u].x, 4 * qi, ok);
      f(v[u].y, 4 * qi + 1, ok);
      f(v[u].z, 4 * qi + 2, ok);
      f(v[u].w, 4 * qi + 3, ok);
    }
  }
  const uint32_t i = 4 * nq + threadIdx.x;  // the last n % 4 entries
  const bool ok = i < n;
  f(ok ? o[i] : 0.f, i, ok);
}

// Digit search over 256 histogram bins by the first wave. Descending: the bin
// b with sum over bins above b < need <= the same sum including b; ascending:
// likewise from bin 0 up. Lane l holds four consecutive bins in visit order; a
// wave prefix sum finds the lane, the lane its bin.
template <bool DESC>
__device__ inline void digit_search(const uint32_t* hist, uint32_t need, uint32_t* s_digit, uint32_t* s_need,
                                    uint32_t* s_eq) {
  if (threadIdx.x >= 64) return;
  const uint32_t l = threadIdx.x;
  const uint32_t b0 = 4 * (DESC ? 63 - l : l);
  uint32_t h[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) h[e] = hist[DESC ? b0 + 3 - e : b0 + e];
  const uint32_t sl = h[0] + h[1] + h[2] + h[3];
  uint32_t inc = sl;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t v = __shfl_up(inc, d);
    if (l >= (uint32_t)d) inc += v;
  }
  const uint32_t exc = inc - sl;
  if (exc < need && need <= inc) {
    uint32_t cum = exc;
    int e = 0;
    for (; e < 3; ++e) {
      if (cum + h[e] >= need) break;
      cum += h[e];
    }
    *s_digit = DESC ? b0 + 3 - e : b0 + e;
    *s_need = need - cum;
    if (s_eq) *s_eq = h[e];
  }
}

// One-workgroup radix select: the K-th key T (8-bit digits of the order key)
// and, when keys equal to T must be split, the id cutoff I (ids ascending);
// then the K best go to tmp.
__device__ inline void radix_select(const QueryDev& Q, uint32_t n, uint32_t* T_out, uint64_t* I_out) {
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  __shared__ uint32_t hist[256];
  __shared__ uint32_t s_digit, s_need, s_eq, s_pos;
  const uint32_t K = Q.K;
  uint32_t prefix = 0, pmask = 0, need = K;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (uint32_t b = tid; b < 256; b += kSelectThreads) hist[b] = 0;
    __syncthreads();
    scan_objectives(Q.cand_o, n, [&](float o, uint32_t, bool ok) {
      const uint32_t kf = ord_f32(o);
      hist_add(hist, (kf >> shift) & 255u, ok && (kf & pmask) == prefix);
    });
    __syncthreads();
    digit_search<true>(hist, need, &s_digit, &s_need, &s_eq);
    __syncthreads();
    prefix |= s_digit << shift;
    pmask |= 255u << shift;
    need = s_need;
    __syncthreads();
  }
  const uint32_t T = prefix;
  const uint32_t eq = s_eq;  // entries whose key equals T
  // among ties on the objective: the `need` smallest ids
  uint64_t I = ~0ull;
  if (need < eq) {
    uint64_t ip = 0, im = 0;
    uint32_t want = need;
    for (int shift = 56; shift >= 0; shift -= 8) {
      for (uint32_t b = tid; b < 256; b += kSelectThreads) hist[b] = 0;
      __syncthreads();
      scan_objectives(Q.cand_o, n, [&](float o, uint32_t i, bool ok) {
        const bool tie = ok && ord_f32(o) == T;
        const uint64_t id = tie ? Q.cand_id[i] : 0ull;
        hist_add(hist, (uint32_t)(id >> shift) & 255u, tie && (id & im) == ip);
      });
      __syncthreads();
      digit_search<false>(hist, want, &s_digit, &s_need, nullptr);
      __syncthreads();
      ip |= (uint64_t)s_digit << shift;
      im |= 255ull << shift;
      want = s_need;
      __syncthreads();
    }
    I = ip;
  }
  // the K best to tmp (one LDS atomic per wave)
  if (tid == 0) s_pos = 0;
  __syncthreads();
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  scan_objectives(Q.cand_o, n, [&](float o, uint32_t i, bool ok) {
    const uint32_t kf = ord_f32(o);
    const bool cand = ok && kf >= T;
    const uint64_t id = cand ? Q.cand_id[i] : 0ull;
    const bool keep = cand && (kf > T || id <= I);
    const uint64_t m = __ballot(keep);
    uint32_t wbase = 0;
    if (lane == 0 && m) wbase = atomicAdd(&s_pos, (uint32_t)__popcll(m));
    wbase = (uint32_t)__shfl((int)wbase, 0);
    if (keep) {
      const uint32_t q = wbase + (uint32_t)__popcll(m & below);
      if (q < K) {
        Q.tmp_o[q] = o;
        Q.tmp_id[q] = id;
      }
    }
  });
  *T_out = T;
  *I_out = I;
}

// The bracket's `take` = K - above best entries, by a radix select over the
// bracket held in LDS (8-bit digits of the key, then of the id among ties), go
// after the `above` sure entries in tmp; returns the K-th key and id cutoff.
__device__ inline void bracket_finish(const QueryDev& Q, const SelScratch* S, uint32_t above, uint32_t* T_out,
                                      uint64_t* I_out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char sel_smem[];
  uint32_t* bk = reinterpret_cast<uint32_t*>(sel_smem);
  uint64_t* bi = reinterpret_cast<uint64_t*>(sel_smem + 4 * kSelBracket);
  __shared__ uint32_t hist[256];
  __shared__ uint32_t s_digit, s_need, s_eq, s_pos;
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t m = S->pos_br;
  for (uint32_t i = tid; i < m; i += kSelectThreads) {
    bk[i] = S->br_key[i];
    bi[i] = S->br_id[i];
  }
  __syncthreads();
  // calls f(key, index, valid) for every bracket entry, lanes of a wave in step
  auto each = [&](auto&& f) {
    for (uint32_t i0 = 0; i0 < m; i0 += kSelectThreads) {
      const uint32_t i = i0 + tid;
      const bool ok = i < m;
      f(ok ? bk[i] : 0u, i, ok);
    }
  };
  const uint32_t take = Q.K - above;  // 1 <= take <= m
  uint32_t prefix = 0, pmask = 0, need = take;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (uint32_t b = tid; b < 256; b += kSelectThreads) hist[b] = 0;
    __syncthreads();
    each([&](uint32_t kf, uint32_t, bool ok) { hist_add(hist, (kf >> shift) & 255u, ok && (kf & pmask) == prefix); });
    __syncthreads();
    digit_search<true>(hist, need, &s_digit, &s_need, &s_eq);
    __syncthreads();
    prefix |= s_digit << shift;
    pmask |= 255u << shift;
    need = s_need;
    __syncthreads();
  }
  const uint32_t T = prefix;
  uint64_t I = ~0ull;
  if (need < s_eq) {
    uint64_t ip = 0, im = 0;
    uint32_t want = need;
    for (int shift = 56; shift >= 0; shift -= 8) {
      for (uint32_t b = tid; b < 256; b += kSelectThreads) hist[b] = 0;
      __syncthreads();
      each([&](uint32_t kf, uint32_t i, bool ok) {
        const bool tie = ok && kf == T;
        const uint64_t id = tie ? bi[i] : 0ull;
        hist_add(hist, (uint32_t)(id >> shift) & 255u, tie && (id & im) == ip);
      });
      __syncthreads();
      digit_search<false>(hist, want, &s_digit, &s_need, nullptr);
      __syncthreads();
      ip |= (uint64_t)s_digit << shift;
      im |= 255ull << shift;
      want = s_need;
      __syncthreads();
    }
    I = ip;
  }
  if (tid == 0) s_pos = 0;
  __syncthreads();
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  each([&](uint32_t kf, uint32_t i, bool ok) {
    const bool keep = ok && (kf > T || (kf == T && bi[i] <= I));
    const uint64_t mk = __ballot(keep);
    uint32_t wbase = 0;
    if (lane == 0 && mk) wbase = atomicAdd(&s_pos, (uint32_t)__popcll(mk));
    wbase = (uint32_t)__shfl((int)wbase, 0);
    if (keep) {
      const uint32_t q = wbase + (uint32_t)__popcll(mk & below);
      Q.tmp_o[above + q] = unord_f32(kf);
      Q.tmp_id[above + q] = bi[i];
    }
  });
  *T_out = T;
  *I_out = I;
}

__global__ __launch_bounds__(kSelectThreads) void k_select(const QueryDev* __restrict__ qs, uint32_t chunk_id,
                                                          int force) {
  const QueryDev Q = qs[blockIdx.x];
  if (!Q.active) return;
  QState* st = Q.st;
  const uint32_t tid = threadIdx.x;
  const uint32_t count = st->count;
  const uint32_t base = st->chunk_base;
  const SelPlan p = sel_plan(Q, force);
  const uint32_t K = Q.K;
  __syncthreads();  // every thread has read the state before it changes
  if (!p.run) {
    if (tid == 0) {
      st->appended += count - base;
      st->chunk_base = count;
    }
    return;
  }
  const SelScratch* S = Q.sel;
  uint32_t T;
  uint64_t I;
  bool radix = S->mode != 0;
  uint32_t above = 0;
  if (!radix) {
    const Bracket br = sel_bracket(S, p.n, K);
    radix = !br.fits;
    above = br.above;
  }
  if (radix) radix_select(Q, p.n, &T, &I);
  else bracket_finish(Q, S, above, &T, &I);
  const float To = unord_f32(T);
  if (p.over) {
    if (tid == 0) {
      st->tau_o = To;
      st->tau_id = I;
      st->appended += count - base;
      st->count = base;
      st->overflow += 1;
      Q.rerun[chunk_id] = 1u;
    }
    return;
  }
  __syncthreads();
  for (uint32_t i = tid; i < K; i += kSelectThreads) {
    Q.cand_o[i] = Q.tmp_o[i];
    Q.cand_id[i] = Q.tmp_id[i];
  }
  __syncthreads();
  if (tid == 0) {
    st->appended += count - base;
    st->count = K;
    st->chunk_base = K;
    st->tau_o = To;
    st->tau_id = I;
  }
}

// Fresh threshold state: no threshold, nothing appended.
__global__ void k_state_reset(QState* st) {
  if (threadIdx.x == 0) {
    st->tau_o = -INFINITY;
    st->tau_id = ~0ull;
    st->count = 0;
    st->chunk_base = 0;
    st->overflow = 0;
    st->warm = 0;
    st->appended = 0;
  }
}

// Lowers each query's threshold slightly (tau - |tau| 2^-18 - 2^-100) and
// empties its buffer: used after the sampling pass, whose entries will be met
// again during the enumeration.
__global__ void k_tau_relax(const QueryDev* __restrict__ qs, uint32_t nq) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq || !qs[q].active) return;
  QState* st = qs[q].st;
  const float t = st->tau_o;
  if (st->count >= qs[q].K && t == t && t != -INFINITY) {
    st->tau_o = t - fabsf(t) * 3.814697265625e-06f - 7.888609052210118e-31f;
    st->tau_id = ~0ull;
    st->warm = 1;
  } else {
    st->tau_o = -INFINITY;
    st->tau_id = ~0ull;
    st->warm = 0;
  }
  st->count = 0;
  st->chunk_base = 0;
  st->appended = 0;
}

// Sort of up to kSelBracket entries (n = min(count, n_max)) by (objective desc,
// id asc), keeping the first min(n, n_out): each entry's rank is the number of
// entries ranked before it (keys are distinct), counted over a 2D grid - block
// x of entries against block y of entries staged in LDS, the block's count added
// to the entry's rank - then every entry with rank < n_out is written to its
// place. No barrier separates the comparisons, unlike a sorting network.
constexpr uint32_t kRankBlock = 256;
__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ __launch_bounds__(kRankBlock) void k_rank_count(const QueryDev* __restrict__ qs, uint32_t q,
                                                           uint32_t n_max, uint32_t* __restrict__ rank) {
  const QueryDev& Q = qs[q];
  const uint32_t n = min(Q.st->count, n_max);
  const uint32_t i0 = blockIdx.x * kRankBlock, j0 = blockIdx.y * kRankBlock;
  if (i0 >= n || j0 >= n) return;  // uniform per workgroup
  __shared__ uint32_t sk[kRankBlock];
  __shared__ uint64_t si[kRankBlock];
  const uint32_t t = threadIdx.x, m = min(kRankBlock, n - j0);
  sk[t] = t < m ? ord_f32(Q.cand_o[j0 + t]) : 0u;
  si[t] = t < m ? Q.cand_id[j0 + t] : ~0ull;
  __syncthreads();
  const uint32_t i = i0 + t;
  if (i >= n) return;
  const uint32_t ki = ord_f32(Q.cand_o[i]);
  const uint64_t ii = Q.cand_id[i];
  uint32_t c = 0;
  for (uint32_t k = 0; k < m; ++k) c += ranks_before(sk[k], si[k], ki, ii) ? 1u : 0u;
  if (c) atomicAdd(rank + i, c);
}

__global__ __launch_bounds__(kRankBlock) void k_rank_scatter(const QueryDev* __restrict__ qs, uint32_t q,
                                                             uint32_t n_max, uint32_t n_out,
                                                             const uint32_t* __restrict__ rank,
                                                             float* __restrict__ out_o, uint64_t* __restrict__ out_id) {
  const QueryDev& Q = qs[q];
  const uint32_t n = min(Q.st->count, n_max);
  const uint32_t i = blockIdx.x * kRankBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t r = rank[i];
  if (r < n_out) {
    out_o[r] = Q.cand_o[i];
    out_id[r] = Q.cand_id[i];
  }
}

// id -> (reaction, synthon per slot).
__global__ void k_decode(const ReactDev* __restrict__ react, uint32_t n_react, const uint64_t* __restrict__ ids,
                         const QState* __restrict__ st, uint32_t K, uint32_t* __restrict__ reaction,
                         uint32_t* __restrict__ synthon) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = min(st->count, K);
  if (i >= n) return;
  const uint64_t id = ids[i];
  const uint32_t t = find_reaction(react, n_react, id);
  const ReactDev r = react[t];
  const uint64_t loc = id - r.id_off;
  const uint32_t a = (uint32_t)(loc / r.nB), b = (uint32_t)(loc - (uint64_t)a * r.nB);
  reaction[i] = t;
  if (r.three) {
    synthon[3 * i + 0] = a / r.n1;
    synthon[3 * i + 1] = a % r.n1;
    synthon[3 * i + 2] = b;
  } else {
    synthon[3 * i + 0] = a;
    synthon[3 * i + 1] = b;
    synthon[3 * i + 2] = 0;
  }
}

// Stratified sample of n distinct compounds of a selection: draw i lies in the
// i-th of n equal parts of the selection's compound range (SplitMix64 offsets).
__global__ void k_sample_ids(const SelDev* __restrict__ sel, uint32_t n_sel, const ReactDev* __restrict__ react,
                             uint64_t total, uint32_t n, uint64_t seed, uint64_t* __restrict__ ids) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t lo = (uint64_t)(((unsigned __int128)total * i) / n);
  const uint64_t hi = (uint64_t)(((unsigned __int128)total * (i + 1)) / n);
  uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const uint64_t x = lo + (hi > lo ? z % (hi - lo) : 0);
  uint32_t a = 0, b = n_sel;
  while (b - a > 1) {
    const uint32_t m = (a + b) >> 1;
    if (sel[m].compound_start <= x) a = m; else b = m;
  }
  ids[i] = react[sel[a].t].id_off + (x - sel[a].compound_start);
}

// Sample for the threshold warm start: n compounds in groups of 32, group g
// taking two first-slot rows (a random even pair of a tile's eight) against the
// tile's 16 last-slot rows of one tile drawn from the g-th of equal parts of the
// selection's tile range. Tiles of different groups differ, so no compound is
// drawn twice (a repeated compound could push the sample's K-th key above the
// true K-th best). A group's compounds share rows, which the gather then reads
// once from the caches instead of once per compound. Positions outside the
// reaction get an id past the library's end (their heads come out NaN and
// they are not scored).
__global__ void k_sample_tiles(const SelDev* __restrict__ sel, uint32_t n_sel, const ReactDev* __restrict__ react,
                               uint64_t n_tiles, uint32_t n, uint64_t seed, uint64_t* __restrict__ ids) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t groups = (n + 31) / 32, g = i / 32, m = i % 32;
  const uint64_t lo = (uint64_t)(((unsigned __int128)n_tiles * g) / groups);
  const uint64_t hi = (uint64_t)(((unsigned __int128)n_tiles * (g + 1)) / groups);
  uint64_t z = seed + (uint64_t)(g + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const uint64_t v = lo + (hi > lo ? z % (hi - lo) : 0);
  uint32_t a = 0, b = n_sel;
  while (b - a > 1) {
    const uint32_t mid = (a + b) >> 1;
    if (sel[mid].tile_start <= v) a = mid; else b = mid;
  }
  const SelDev S = sel[a];
  const ReactDev R = react[S.t];
  const uint64_t lt = v - S.tile_start;
  const uint32_t ta = (uint32_t)(lt / S.tiles_b), tb = (uint32_t)(lt % S.tiles_b);
  const uint32_t r0 = 2 * (uint32_t)((z >> 40) % 4);  // rows r0, r0 + 1 of the tile's eight
  const uint32_t ra = ta * 8 + r0 + m / 16, rb = tb * kTileB + m % 16;
  ids[i] = (ra < R.nA && rb < R.nB) ? R.id_off + (uint64_t)ra * R.nB + rb : ~0ull;
}

// Largest |low-precision head - FP32 head| per head.
__global__ void k_head_err(const float* __restrict__ h_lp, const float* __restrict__ h_32, uint32_t n,
                           float* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * kHeadsPad) return;
  const float e = fabsf(h_lp[i] - h_32[i]);
  if (e < __builtin_inff()) atomic_max_nonneg(out + (i % kHeadsPad), e);  // compounds with non-finite heads never pass
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_hoist(const float* U, uint32_t d, uint64_t rows, const float* W1, const float* b1, uint32_t n_w,
                        uint32_t h1, const uint8_t* is_slot0, float c, float* P, hipStream_t s) {
  dim3 grid((unsigned)((rows + 63) / 64), (h1 + 63) / 64);
  hipLaunchKernelGGL(k_hoist, grid, dim3(256), 0, s, U, d, rows, W1, b1, n_w, h1, is_slot0, c, P);
  return hipGetLastError();
}

hipError_t launch_act_range(const float* P, uint32_t h1, const uint64_t* slot_row0, const uint32_t* slot_size,
                            uint32_t n_slots_total, const uint32_t* react_slot0, const uint32_t* react_nslots,
                            uint32_t n_react, int act, float c, float* cmax, float* cmin, float* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_colext, dim3(n_slots_total, (h1 + 127) / 128), dim3(128), 0, s, P, h1, slot_row0, slot_size,
                     cmax, cmin);
  hipLaunchKernelGGL(k_actmax, dim3(n_react, (h1 + 127) / 128), dim3(128), 0, s, cmax, cmin, h1, react_slot0,
                     react_nslots, n_react, act, c, out);
  return hipGetLastError();
}

hipError_t launch_absmax(const float* x, uint64_t n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_absmax, dim3(64), dim3(256), 0, s, x, n, out);
  return hipGetLastError();
}

hipError_t launch_scales(const float* amax, int prec, int nl, float* scal, hipStream_t s) {
  hipLaunchKernelGGL(k_scales, dim3(1), dim3(64), 0, s, amax, prec, nl, scal);
  return hipGetLastError();
}

hipError_t launch_frag_x(const float* W, uint32_t n_out, uint32_t n_in, uint32_t n_chunks, float mul, void* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_frag_x, dim3(256), dim3(256), 0, s, W, n_out, n_in, n_chunks, mul,
                     reinterpret_cast<float*>(out));
  return hipGetLastError();
}

hipError_t launch_frag_x32(int prec, const float* W, uint32_t n_out, uint32_t n_in, uint32_t n_chunks,
                           const float* mul_dev, float mul, void* out, hipStream_t s) {
  dim3 grid(256), block(256);
  if (prec == APEX_PREC_BF16)
    hipLaunchKernelGGL(k_frag_x32<APEX_PREC_BF16>, grid, block, 0, s, W, n_out, n_in, n_chunks, mul_dev, mul, out);
  else if (prec == APEX_PREC_FP8)
    hipLaunchKernelGGL(k_frag_x32<APEX_PREC_FP8>, grid, block, 0, s, W, n_out, n_in, n_chunks, mul_dev, mul, out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_frag_out32(const float* Wo, uint32_t H, uint32_t h2, uint32_t h2k, float mul, void* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_frag_out32, dim3(64), dim3(256), 0, s, Wo, H, h2, h2k, mul, reinterpret_cast<__bf16*>(out));
  return hipGetLastError();
}

hipError_t launch_frag_out_d(const float* Wo, uint32_t H, uint32_t h2, float mul, void* out, hipStream_t s) {
  hipLaunchKernelGGL(k_frag_out_d, dim3(64), dim3(256), 0, s, Wo, H, h2, mul, reinterpret_cast<float*>(out));
  return hipGetLastError();
}
hipError_t launch_bias(const float* b2, uint32_t h2, uint32_t h2k, float c, const float* scal, const float* bo,
                       uint32_t H, float* b2_out, float* bo_out, hipStream_t s) {
  if (h2k < h2) h2k = h2;
  const uint32_t n = h2k > kHeadsPad ? h2k : kHeadsPad;
  hipLaunchKernelGGL(k_bias, dim3((n + 255) / 256), dim3(256), 0, s, b2, h2, h2k, c, scal, bo, H, b2_out, bo_out);
  return hipGetLastError();
}

hipError_t launch_score(const float* heads, const uint64_t* ids, uint32_t n, const QState* n_src, const QueryDev* qs,
                        uint32_t nq, const ReactDev* react, uint32_t n_react, hipStream_t s) {
  if (n == 0 || nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_score, dim3((n + kScoreThreads - 1) / kScoreThreads, nq), dim3(kScoreThreads), 0, s, heads,
                     ids, n, n_src, qs, nq, react, n_react);
  return hipGetLastError();
}

hipError_t launch_pool_lookup(const uint64_t* pool_id, const float* pool_heads, uint32_t pool_max,
                              const QState* pool_src, const uint64_t* want, uint32_t want_max, const QState* want_src,
                              float* out, hipStream_t s) {
  if (want_max == 0 || pool_max == 0) return hipSuccess;
  if (!pool_src || !want_src) return hipErrorInvalidValue;
  constexpr uint32_t waves = kLookupThreads / 64;
  hipLaunchKernelGGL(k_pool_lookup, dim3((want_max + waves - 1) / waves), dim3(kLookupThreads), 0, s, pool_id,
                     pool_heads, pool_max, pool_src, want, want_max, want_src, out);
  return hipGetLastError();
}

hipError_t launch_select(const QueryDev* qs, uint32_t nq, uint32_t chunk_id, int force, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  constexpr size_t lds = 12 * kSelBracket;  // bracket keys and ids
  static hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_select),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(k_sel_plan, dim3(nq), dim3(kSelectThreads), 0, s, qs, force);
  hipLaunchKernelGGL(k_sel_count, dim3(kSelGrid, nq), dim3(kSelPassThreads), 0, s, qs, force);
  hipLaunchKernelGGL(k_sel_compact, dim3(kSelGrid, nq), dim3(kSelPassThreads), 0, s, qs, force);
  hipLaunchKernelGGL(k_select, dim3(nq), dim3(kSelectThreads), lds, s, qs, chunk_id, force);
  return hipGetLastError();
}

hipError_t launch_state_reset(QState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_tau_relax(const QueryDev* qs, uint32_t nq, hipStream_t s) {
  hipLaunchKernelGGL(k_tau_relax, dim3((nq + 63) / 64), dim3(64), 0, s, qs, nq);
  return hipGetLastError();
}

hipError_t launch_sort_small(const QueryDev* qs, uint32_t q, uint32_t n_max, uint32_t n_out, float* out_o,
                             uint64_t* out_id, uint32_t* rank, hipStream_t s) {
  if (n_max > kSelBracket) return hipErrorInvalidValue;
  if (n_max == 0) return hipSuccess;
  const uint32_t nb = (n_max + kRankBlock - 1) / kRankBlock;
  hipLaunchKernelGGL(k_zero_u32, dim3(nb), dim3(kRankBlock), 0, s, rank, n_max);
  hipLaunchKernelGGL(k_rank_count, dim3(nb, nb), dim3(kRankBlock), 0, s, qs, q, n_max, rank);
  hipLaunchKernelGGL(k_rank_scatter, dim3(nb), dim3(kRankBlock), 0, s, qs, q, n_max, n_out, rank, out_o, out_id);
  return hipGetLastError();
}

hipError_t launch_rank_sort(const QueryDev* qs, uint32_t q, uint32_t K, float* out_o, uint64_t* out_id,
                            uint32_t* rank, hipStream_t s) {
  if (K > kSelBracket) return hipErrorInvalidValue;  // longer answers are radix-sorted
  return launch_sort_small(qs, q, K, K, out_o, out_id, rank, s);
}

hipError_t launch_decode(const ReactDev* react, uint32_t n_react, const uint64_t* ids, const QState* st, uint32_t K,
                         uint32_t* reaction, uint32_t* synthon, hipStream_t s) {
  hipLaunchKernelGGL(k_decode, dim3((K + 255) / 256), dim3(256), 0, s, react, n_react, ids, st, K, reaction, synthon);
  return hipGetLastError();
}

hipError_t launch_sample_ids(const SelDev* sel, uint32_t n_sel, const ReactDev* react, uint64_t total, uint32_t n,
                             uint64_t seed, uint64_t* ids, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample_ids, dim3((n + 255) / 256), dim3(256), 0, s, sel, n_sel, react, total, n, seed, ids);
  return hipGetLastError();
}

hipError_t launch_sample_tiles(const SelDev* sel, uint32_t n_sel, const ReactDev* react, uint64_t n_tiles, uint32_t n,
                               uint64_t seed, uint64_t* ids, hipStream_t s) {
  if (tile_ta(false) != 8) return hipErrorInvalidValue;  // two of a tile's eight first-slot rows
  hipLaunchKernelGGL(k_sample_tiles, dim3((n + 255) / 256), dim3(256), 0, s, sel, n_sel, react, n_tiles, n, seed, ids);
  return hipGetLastError();
}

hipError_t launch_head_err(const float* h_lp, const float* h_32, uint32_t n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_head_err, dim3((n * kHeadsPad + 255) / 256), dim3(256), 0, s, h_lp, h_32, n, out);
  return hipGetLastError();
}

}  // namespace apex
