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
  atomic_max_nonneg(out, m);
}

__global__ void k_absmax(const float* __restrict__ x, uint64_t n, float* __restrict__ out) {
  float m = 0.0f;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(x[i]));
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomic_max_nonneg(out, m);
}

// Scales of one precision. amax: [0] activation range, [1] |W2|, [2] |Wo|.
// scal: [0] S2, [1] So, [2] X conversion scale, [3] 1/s_w2, [4] 1/s_wo.
__global__ void k_scales(const float* __restrict__ amax, int prec, int nl, float* __restrict__ scal) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float S2 = 1.0f, So = 1.0f, xs = 1.0f, iw2 = 1.0f, iwo = 1.0f;
  if (prec == APEX_PREC_FP8) {
    const float ax = amax[0] > 0.0f ? amax[0] : 1.0f;
    xs = exp2f(ceilf(log2f(ax / 448.0f)));
    const float sw2 = amax[1] > 0.0f ? amax[1] / 448.0f : 1.0f;
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
// beyond n_out are zero).
template <int PREC>
__global__ void k_frag_x32(const float* __restrict__ W, uint32_t n_out, uint32_t n_in, uint32_t n_chunks,
                           const float* __restrict__ mul_dev, float mul, void* __restrict__ out) {
  constexpr uint32_t E = PREC == APEX_PREC_BF16 ? 8 : 32;
  const uint32_t ns = n_in / (2 * E);
  const uint64_t total = (uint64_t)n_chunks * ns * 64 * E;
  const float m = mul * (mul_dev ? *mul_dev : 1.0f);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t e = i % E;
    const uint32_t lane = (i / E) % 64;
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

// GEMM accumulator start values c * b2 / S2 (zero for padding neurons h2 ..
// h2k - 1), and the padded final bias.
__global__ void k_bias(const float* __restrict__ b2, uint32_t h2, uint32_t h2k, float c, const float* __restrict__ scal,
                       const float* __restrict__ bo, uint32_t H, float* __restrict__ b2_out,
                       float* __restrict__ bo_out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (b2 && i < h2k) b2_out[i] = i < h2 ? c * b2[i] / scal[0] : 0.0f;
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
constexpr int kScoreThreads = 1024;
__global__ __launch_bounds__(kScoreThreads) void k_score(const float* __restrict__ heads,
                                                        const uint64_t* __restrict__ ids, uint32_t n,
                                                        const QueryDev* __restrict__ qs, uint32_t nq,
                                                        const ReactDev* __restrict__ react, uint32_t n_react) {
  __shared__ uint32_t wave_count[kScoreThreads / 64];
  __shared__ uint32_t block_base;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t q = blockIdx.y;
  if (q >= nq) return;  // uniform per workgroup
  const QueryDev* Q = qs + q;
  if (!Q->active) return;
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
    bool ok = o == o;
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
// the rescored pool's ids, whose FP32 heads were already computed; the row of
// each answer id is found in LDS tiles of the pool and copied.
constexpr int kLookupThreads = 256;
constexpr uint32_t kLookupTile = 2048;  // pool ids per workgroup
__global__ __launch_bounds__(kLookupThreads) void k_pool_lookup(const uint64_t* __restrict__ pool_id,
                                                               const float* __restrict__ pool_heads,
                                                               uint32_t n_pool, const uint64_t* __restrict__ want,
                                                               uint32_t n_want, float* __restrict__ out) {
  // grid: x over the wanted ids, y over tiles of the pool; the one workgroup
  // whose tile holds an id writes its row
  __shared__ uint64_t tile[kLookupTile];
  const uint32_t base = blockIdx.y * kLookupTile;
  const uint32_t lim = n_pool - base < kLookupTile ? n_pool - base : kLookupTile;
  for (uint32_t t = threadIdx.x; t < kLookupTile; t += kLookupThreads) tile[t] = t < lim ? pool_id[base + t] : ~0ull;
  __syncthreads();
  const uint32_t i = blockIdx.x * kLookupThreads + threadIdx.x;
  if (i >= n_want) return;
  const uint64_t id = want[i];
  uint32_t found = UINT32_MAX;
  for (uint32_t t = 0; t < lim; ++t)
    if (tile[t] == id) found = base + t;
  if (found != UINT32_MAX) {
    const float4* src = reinterpret_cast<const float4*>(pool_heads + (uint64_t)found * kHeadsPad);
    float4* dst = reinterpret_cast<float4*>(out + (uint64_t)i * kHeadsPad);
    for (int k4 = 0; k4 < kHeadsPad / 4; ++k4) dst[k4] = src[k4];
  }
}

// ---------------------------------------------------------------------------
// Radix select over a query's candidate buffer. After a pass over a chunk:
//  - more entries than the buffer holds: the chunk's appends are dropped, the
//    threshold is raised to the K-th best key among what was written (a valid
//    lower bound of the final K-th key) and the chunk is flagged for a re-run;
//  - more than the high-water mark (or `force`): keep exactly the K best keys
//    (objective desc, id asc), threshold = K-th best key;
//  - otherwise: nothing but bookkeeping.
// One workgroup per query.
// ---------------------------------------------------------------------------
__device__ inline float unord_f32(uint32_t k) {
  const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(u);
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

__global__ __launch_bounds__(kSelectThreads) void k_select(const QueryDev* __restrict__ qs, uint32_t chunk_id,
                                                          int force) {
  const QueryDev Q = qs[blockIdx.x];
  if (!Q.active) return;
  QState* st = Q.st;
  const uint32_t tid = threadIdx.x;
  __shared__ uint32_t hist[256];
  __shared__ uint32_t s_digit, s_need, s_eq, s_pos;
  const uint32_t count = st->count;
  const uint32_t base = st->chunk_base;
  const bool over = count > Q.cap;
  const uint32_t n = over ? Q.cap : count;
  const uint32_t K = Q.K;
  const bool run = over || (force ? n > K : count > Q.hwm);
  __syncthreads();
  if (!run) {
    if (tid == 0) {
      st->appended += count - base;
      st->chunk_base = count;
    }
    return;
  }
  // ---- K-th largest order key of the objective ----
  uint32_t prefix = 0, pmask = 0, need = K;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (uint32_t b = tid; b < 256; b += kSelectThreads) hist[b] = 0;
    __syncthreads();
    scan_objectives(Q.cand_o, n, [&](float o, uint32_t, bool ok) {
      const uint32_t kf = ord_f32(o);
      hist_add(hist, (kf >> shift) & 255u, ok && (kf & pmask) == prefix);
    });
    __syncthreads();
    if (tid == 0) {
      uint32_t cum = 0;
      int b = 255;
      for (; b > 0; --b) {
        if (cum + hist[b] >= need) break;
        cum += hist[b];
      }
      s_digit = (uint32_t)b;
      s_need = need - cum;
      s_eq = hist[b];
    }
    __syncthreads();
    prefix |= s_digit << shift;
    pmask |= 255u << shift;
    need = s_need;
    __syncthreads();
  }
  const uint32_t T = prefix;
  const uint32_t eq = s_eq;  // entries whose key equals T
  // ---- among ties on the objective: the `need` smallest ids ----
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
      if (tid == 0) {
        uint32_t cum = 0;
        int b = 0;
        for (; b < 255; ++b) {
          if (cum + hist[b] >= want) break;
          cum += hist[b];
        }
        s_digit = (uint32_t)b;
        s_need = want - cum;
      }
      __syncthreads();
      ip |= (uint64_t)s_digit << shift;
      im |= 255ull << shift;
      want = s_need;
      __syncthreads();
    }
    I = ip;
  }
  const float To = unord_f32(T);
  if (over) {
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
  // ---- compaction to exactly K entries (one LDS atomic per wave) ----
  if (tid == 0) s_pos = 0;
  __syncthreads();
  const uint32_t lane = tid & 63;
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
      const uint32_t p = wbase + (uint32_t)__popcll(m & below);
      if (p < K) {
        Q.tmp_o[p] = o;
        Q.tmp_id[p] = id;
      }
    }
  });
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
  } else {
    st->tau_o = -INFINITY;
    st->tau_id = ~0ull;
  }
  st->count = 0;
  st->chunk_base = 0;
  st->appended = 0;
}

// Sort n = min(count, K) entries by (objective desc, id asc): each entry's rank is
// the number of entries ranked before it (keys are distinct).
__global__ __launch_bounds__(256) void k_rank_sort(const QueryDev* __restrict__ qs, uint32_t q, float* __restrict__ out_o,
                                                   uint64_t* __restrict__ out_id) {
  const QueryDev& Q = qs[q];
  const uint32_t n = min(Q.st->count, Q.K);
  constexpr uint32_t TILE = 1024;
  __shared__ __attribute__((aligned(16))) float so[TILE];
  __shared__ __attribute__((aligned(16))) uint64_t sid[TILE];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool mine = i < n;
  const float o = mine ? Q.cand_o[i] : 0.0f;
  const uint64_t id = mine ? Q.cand_id[i] : 0;
  uint32_t rank = 0;
  for (uint32_t t0 = 0; t0 < n; t0 += TILE) {
    __syncthreads();
    // entries past n are (-inf, max id): they never rank before anything
    for (uint32_t k = threadIdx.x; k < TILE; k += blockDim.x) {
      const bool in = t0 + k < n;
      so[k] = in ? Q.cand_o[t0 + k] : -INFINITY;
      sid[k] = in ? Q.cand_id[t0 + k] : ~0ull;
    }
    __syncthreads();
    const uint32_t m = (min(TILE, n - t0) + 15u) & ~15u;
    if (mine) {
      const float4* so4 = reinterpret_cast<const float4*>(so);
      for (uint32_t k = 0; k < m; k += 16) {
        float4 a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = so4[k / 4 + u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float v[4] = {a[u].x, a[u].y, a[u].z, a[u].w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float x = v[e];
            rank += x > o;
            if (x == o) rank += sid[k + 4 * u + e] < id;
          }
        }
      }
    }
  }
  if (mine) {
    out_o[rank] = o;
    out_id[rank] = id;
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

// Largest |low-precision head - FP32 head| per head.
__global__ void k_head_err(const float* __restrict__ h_lp, const float* __restrict__ h_32, uint32_t n,
                           float* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * kHeadsPad) return;
  atomic_max_nonneg(out + (i % kHeadsPad), fabsf(h_lp[i] - h_32[i]));
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

hipError_t launch_score(const float* heads, const uint64_t* ids, uint32_t n, const QueryDev* qs, uint32_t nq,
                        const ReactDev* react, uint32_t n_react, hipStream_t s) {
  if (n == 0 || nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_score, dim3((n + kScoreThreads - 1) / kScoreThreads, nq), dim3(kScoreThreads), 0, s, heads,
                     ids, n, qs, nq, react, n_react);
  return hipGetLastError();
}

hipError_t launch_pool_lookup(const uint64_t* pool_id, const float* pool_heads, uint32_t n_pool, const uint64_t* want,
                              uint32_t n_want, float* out, hipStream_t s) {
  if (n_want == 0) return hipSuccess;
  if (n_pool == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pool_lookup,
                     dim3((n_want + kLookupThreads - 1) / kLookupThreads, (n_pool + kLookupTile - 1) / kLookupTile),
                     dim3(kLookupThreads), 0, s, pool_id, pool_heads, n_pool, want, n_want, out);
  return hipGetLastError();
}

hipError_t launch_select(const QueryDev* qs, uint32_t nq, uint32_t chunk_id, int force, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_select, dim3(nq), dim3(kSelectThreads), 0, s, qs, chunk_id, force);
  return hipGetLastError();
}

hipError_t launch_tau_relax(const QueryDev* qs, uint32_t nq, hipStream_t s) {
  hipLaunchKernelGGL(k_tau_relax, dim3((nq + 63) / 64), dim3(64), 0, s, qs, nq);
  return hipGetLastError();
}

hipError_t launch_rank_sort(const QueryDev* qs, uint32_t q, uint32_t K, float* out_o, uint64_t* out_id,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_rank_sort, dim3((K + 255) / 256), dim3(256), 0, s, qs, q, out_o, out_id);
  return hipGetLastError();
}

hipError_t launch_decode(const ReactDev* react, uint32_t n_react, const uint64_t* ids, const QState* st, uint32_t K,
                         uint32_t* reaction, uint32_t* synthon, hipStream_t s) {
  hipLaunchKernelGGL(k_decode, dim3((K + 255) / 256), dim3(256), 0, s, react, n_react, ids, st, K, reaction, synthon);
  return hipGetLastError();
}

hipError_t launch_sample_ids(const SelDev* sel, uint32_t n_sel, const ReactDev* react, uint64_t total, uint32_t n,
                             uint64_t seed, uint64_t* ids, hipStream_t s) {
  hipLaunchKernelGGL(k_sample_ids, dim3((n + 255) / 256), dim3(256), 0, s, sel, n_sel, react, total, n, seed, ids);
  return hipGetLastError();
}

hipError_t launch_head_err(const float* h_lp, const float* h_32, uint32_t n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_head_err, dim3((n * kHeadsPad + 255) / 256), dim3(256), 0, s, h_lp, h_32, n, out);
  return hipGetLastError();
}

}  // namespace apex
