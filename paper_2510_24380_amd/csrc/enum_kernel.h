// Fused FP32 enumeration kernel for gfx950 (16x16 MFMA, v_mfma_f32_16x16x4_f32):
// synthon-row gather and combine, the decoder on MFMA, the per-query objective
// and bound mask, and a wave-level filter that appends only compounds better
// than the query's running threshold. (BF16 and FP8 run the 32x32 kernel of
// enum32_kernel.h.)
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
//   A: row l % 16, element k = g of the step
//   B: column l % 16, same k
//   D: column l % 16, rows 4 g + v for accumulator v = 0..3
// The contraction index may be permuted freely as long as both operands use the
// same order; the engine lays weights out in the order this kernel produces
// activations: lane group g owns k in [g H1/4, (g+1) H1/4), step s covers
// value s of it.
#pragma once
#include "enum_common.h"

namespace apex {

__device__ __forceinline__ f32x4 mma16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// LDS bytes of the FP32 kernel (host and device agree on this). The staged
// synthon rows (activation phase) and the double-buffered GEMM weight chunks
// (GEMM phase) share one region; the final-layer fragments and the GEMM start
// values stay resident.
__host__ __device__ constexpr int enum_lds_bytes(int h1, int nl, int h2, bool gather) {
  int rows = gather ? 0 : (kTileA16 + kTileB) * (h1 + kRowPad) * 4;
  int chunk = nl == 2 ? 2 * 16 * h1 * 4 : 0;
  int region = rows > chunk ? rows : chunk;
  int wo = nl == 2 ? 16 * h2 * 4 : (nl == 1 ? 16 * h1 * 4 : 0);
  int b2 = nl == 2 ? h2 * 4 : 0;
  return region + wo + b2 + (gather ? 0 : kHeadsPad * 4 + kQLdsBytes);  // + final bias, query parameters
}

template <int H1, int NL, int ACT, bool GATHER>
__global__ __launch_bounds__(kWaves16 * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_enum(EnumArgs A) {
  constexpr int W = kWaves16, T = W * 64;
  constexpr int TA = kTileA16, TB = kTileB;
  constexpr int NS = H1 / 4;  // k-steps over the first hidden width (one activation each)
  constexpr int KG = H1 / 4;  // activations per lane group
  constexpr int ROW = H1 + kRowPad;
  constexpr int CHUNK = 16 * H1 * 4;  // bytes of one 16-neuron GEMM weight chunk
  constexpr int NPRE = (CHUNK / 16 + T - 1) / T;
  constexpr bool FULL = (CHUNK / 16) % T == 0;  // every thread moves NPRE x 16 bytes
  constexpr int ROWS_BYTES = GATHER ? 0 : (TA + TB) * ROW * 4;
  constexpr int REGION = ROWS_BYTES > (NL == 2 ? 2 * CHUNK : 0) ? ROWS_BYTES : (NL == 2 ? 2 * CHUNK : 0);
  static_assert(TA == W, "one A-row per wave");

  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  float* sA = reinterpret_cast<float*>(smem);
  float* sB = sA + TA * ROW;
  unsigned char* sW = smem;  // GEMM weight chunks share the region with the staged rows
  unsigned char* sWo = smem + REGION;
  const uint32_t H2 = NL == 2 ? A.H2 : 0;
  float* sB2 = reinterpret_cast<float*>(sWo + (NL == 2 ? 16 * H2 * 4 : (NL == 1 ? 16 * H1 * 4 : 0)));
  float* sBo = sB2 + (NL == 2 ? H2 : 0);                // tile mode: final bias
  QLds* sQ = reinterpret_cast<QLds*>(sBo + kHeadsPad);  // tile mode: one entry per query

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, j = lane & 15;
  const int NC = NL == 2 ? (int)(H2 / 16) : 0;
  const float So = A.pd.scal[1];

  // Work range of this workgroup. Tiles (or gathered compounds) are split into
  // contiguous runs; consecutive runs go to workgroups on the same XCD (blocks
  // are dispatched to XCDs round robin), so neighbouring tiles share that XCD's
  // L2. With work counters (tile mode), runs are taken at run time instead
  // (take_tile_run).
  const bool dyn = !GATHER && A.work != nullptr;
  uint64_t v, vend;
  {
    const uint32_t G = gridDim.x, bid = blockIdx.x;
    const uint32_t per_xcd = G / 8;
    const uint32_t wg = (G % 8 == 0) ? (bid % 8) * per_xcd + bid / 8 : bid;
    if (GATHER) {
      const uint64_t per_wg = W * 16;
      v = (uint64_t)wg * per_wg;
      vend = v + per_wg;
      if (v >= A.n_ids) return;
    } else if (dyn) {
      v = vend = 0;  // set by the first take below
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
    const int wo_bytes = NL == 2 ? 16 * (int)H2 * 4 : (NL == 1 ? 16 * H1 * 4 : 0);
    const uint4* src = reinterpret_cast<const uint4*>(A.pd.wo);
    uint4* dst = reinterpret_cast<uint4*>(sWo);
    for (int i = tid; i < wo_bytes / 16; i += T) dst[i] = src[i];
    if (NL == 2)
      for (int i = tid; i < (int)H2; i += T) sB2[i] = A.pd.b2[i];
    if (!GATHER) {
      if (tid < kHeadsPad) sBo[tid] = A.pd.bo[tid];
      copy_queries_lds(A, sQ, wave, W, lane);
    }
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

  __shared__ uint64_t s_run[3];  // dynamic work: the run taken, regions used up
  if (dyn && tid == 0) s_run[2] = 0;
  if (dyn) take_tile_run(A, s_run, v, vend);
  uint32_t si = 0;
  SelDev S{};
  ReactDev Rt{};
  uint64_t s_end = 0;
  if (!GATHER && v < vend) {
    si = find_sel(A.sel, A.n_sel, v);
    S = A.sel[si];
    Rt = A.react[S.t];
    s_end = S.tile_start + (uint64_t)((Rt.nA + TA - 1) / TA) * S.tiles_b;
  }

  for (; v < vend || (dyn && (take_tile_run(A, s_run, v, vend), v < vend)); v += (GATHER ? vend : 1)) {
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
      // the tile's selection entry: the next ones in turn, or (a run taken
      // elsewhere in the launch) a binary search
      for (int hop = 0; v < S.tile_start || v >= s_end; ++hop) {
        si = (dyn && (hop == 2 || v < S.tile_start)) ? find_sel(A.sel, A.n_sel, v) : si + 1;
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
    float X[NS];
    const float* pa;
    const float* pa1 = nullptr;
    const float* pb;
    if (!GATHER) {
      pa = sA + wave * ROW + g * KG;
      pb = sB + j * ROW + g * KG;
    } else {
      uint64_t item = v + (uint64_t)wave * 16 + j;
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
        pa = A.P + (uint64_t)(rr.row0 + i0) * H1 + g * KG;
        pa1 = A.P + (uint64_t)(rr.row1 + i1) * H1 + g * KG;
      } else {
        pa = A.P + (uint64_t)(rr.row0 + a) * H1 + g * KG;
      }
      pb = A.P + (uint64_t)(rr.rowB + b) * H1 + g * KG;
    }
    // four steps per 16-byte read
#pragma unroll
    for (int s4 = 0; s4 < NS / 4; ++s4) {
      float4 xa = *reinterpret_cast<const float4*>(pa + 4 * s4);
      if (GATHER && pa1) {
        const float4 xq = *reinterpret_cast<const float4*>(pa1 + 4 * s4);
        xa = make_float4(xa.x + xq.x, xa.y + xq.y, xa.z + xq.z, xa.w + xq.w);
      }
      const float4 xb = *reinterpret_cast<const float4*>(pb + 4 * s4);
      X[4 * s4 + 0] = act_pre<ACT>(xa.x + xb.x);
      X[4 * s4 + 1] = act_pre<ACT>(xa.y + xb.y);
      X[4 * s4 + 2] = act_pre<ACT>(xa.z + xb.z);
      X[4 * s4 + 3] = act_pre<ACT>(xa.w + xb.w);
      asm volatile("" : "+v"(X[4 * s4 + 0]), "+v"(X[4 * s4 + 1]), "+v"(X[4 * s4 + 2]), "+v"(X[4 * s4 + 3])::"memory");
    }

    // ---------------- decoder layers on MFMA ----------------
    f32x4 hacc = f32x4{0.f, 0.f, 0.f, 0.f};

    static_assert(NL >= 1, "the linear decoder runs in the scalar-contribution kernel");
    if constexpr (NL == 1) {
#pragma unroll
      for (int s = 0; s < NS; ++s) hacc = mma16x4(load_frag<float>(sWo + (size_t)(s * 64 + lane) * 4), X[s], hacc);
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
      // pf: chunk c + 1 exists; a literal at every call, so the pipelined loop
      // body below has no branches and the scheduler can interleave its parts.
      auto gemm = [&](int c, f32x4& acc, bool pf) {
        if (pf) {
#pragma unroll
          for (int q = 0; q < NPRE; ++q) {
            const int i = tid + q * T;
            if (FULL || i < CHUNK / 16) pre_put(pre, q, w2g[(size_t)(c + 1) * (CHUNK / 16) + i]);
          }
        }
        acc = *reinterpret_cast<const f32x4*>(sB2 + c * 16 + g * 4);
        const unsigned char* wc = sW + (c & 1) * CHUNK;
#pragma unroll
        for (int s = 0; s < NS; ++s) acc = mma16x4(load_frag<float>(wc + (size_t)(s * 64 + lane) * 4), X[s], acc);
      };
      auto finish = [&](int c, const f32x4& acc) {
        const float* wof = reinterpret_cast<const float*>(sWo);
#pragma unroll
        for (int q = 0; q < 4; ++q) hacc = mma16x4(wof[(c * 4 + q) * 64 + lane], act_pre<ACT>(acc[q]), hacc);
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
      f32x4 accA, accB;
      gemm(0, accA, true);  // NC >= 2
      publish(0, true);
      int c = 1;
      for (; c + 1 < NC; c += 2) {  // chunks c + 1 and c + 2 <= NC - 1 exist
        gemm(c, accB, true);
        finish(c - 1, accA);
        publish(c, true);
        gemm(c + 1, accA, true);
        finish(c, accB);
        publish(c + 1, true);
      }
      gemm(c, accB, false);  // c == NC - 1 (NC is even)
      finish(c - 1, accA);
      finish(c, accB);
      __syncthreads();  // the region is restaged by the next tile
    }

    // ---------------- heads, objective, bounds, filter ----------------
    uint64_t cid;  // compound id (tile mode) or list position (gather mode)
    bool valid;
    if (!GATHER) {
      const uint32_t a = a0 + wave, b = b0 + j;
      valid = a < Rt.nA && b < Rt.nB;
      cid = Rt.id_off + (uint64_t)a * Rt.nB + b;
    } else {
      cid = v + (uint64_t)wave * 16 + j;
      valid = cid < A.n_ids;
    }
    float heads[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) heads[q] = fmaf(hacc[q], So, GATHER ? A.pd.bo[4 * g + q] : sBo[4 * g + q]);

    if constexpr (GATHER) {
      if (valid) {
        float4 o4 = make_float4(heads[0], heads[1], heads[2], heads[3]);
        if (A.ids[cid] >= A.n_total) o4 = make_float4(NAN, NAN, NAN, NAN);
        *reinterpret_cast<float4*>(A.heads_out + cid * 16 + 4 * g) = o4;
      }
    } else {
      for (uint32_t qi = 0; qi < A.n_queries; ++qi) {
        const QLds* L = sQ + qi;
        if (!L->active) continue;
        if (L->subset_bits && !((L->subset_bits[S.t >> 5] >> (S.t & 31)) & 1u)) continue;
        const QueryDev* Q = A.queries + qi;  // appends only
        const float tau_o = L->tau_o;
        const uint64_t tau_id = L->tau_id;
        float w4[4];
        int ok = 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          w4[q] = L->w[4 * g + q];
          ok &= (heads[q] >= L->lo[4 * g + q]) & (heads[q] <= L->hi[4 * g + q]);
        }
        float p = obj_partial(w4, heads);
        // combine the four lane groups: (g0 + g1) + (g2 + g3)
        p = p + __shfl_xor(p, 16);
        p = p + __shfl_xor(p, 32);
        ok &= __shfl_xor(ok, 16);
        ok &= __shfl_xor(ok, 32);
        const float o = canon_zero(p);
        const bool pass = g == 0 && valid && ok && finite_obj(o) && key_passes(o, cid, tau_o, tau_id);
        const uint64_t mask = __ballot(pass);
        if (mask) {
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(&Q->st->count, (uint32_t)__popcll(mask));
          base = __shfl(base, 0);
          const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
          if (pass) {
            const uint32_t idx = base + (uint32_t)__popcll(mask & below);
            if (idx < Q->cap) {
              Q->cand_o[idx] = o;
              Q->cand_id[idx] = cid;
            }
          }
        }
      }
    }
    if (NL != 2 && !GATHER) __syncthreads();  // staged rows are reused by the next tile
  }
  if (dyn) release_tile_counters(A);
}

// Heads of listed compounds with a two-hidden-layer decoder, for short lists
// (FP32 rescoring of a pool, answer heads, warm-start samples). The tile
// kernel's gather mode gives each wave all H2/16 weight chunks in sequence,
// which leaves a short list with few, long-running workgroups. Here a workgroup
// takes 16 compounds, every wave computes their layer-1 activations, wave w
// takes chunks w, w + 8, ... (weights read from the caches) and leaves the
// chunks' second-layer activations in LDS; one wave then runs the final layer
// over the chunks in order 0, 1, ..., exactly as the tile kernel does, so the
// heads (and any objective formed from them) are the same bits as in the
// enumeration.
__host__ __device__ constexpr int gather_split_lds_bytes(int h2) { return 16 * h2 * 4 + h2 * 4 + h2 * 64; }

template <int H1, int ACT>
__global__ __launch_bounds__(kWaves16 * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gather_split(
    EnumArgs A) {
  constexpr int W = kWaves16, T = W * 64;
  constexpr int NS = H1 / 4, KG = H1 / 4;
  constexpr int B = 16;  // weight fragments per batch of loads
  static_assert(NS % B == 0, "layout");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const uint32_t H2 = A.H2;
  float* sWo = reinterpret_cast<float*>(smem);
  float* sB2 = sWo + 16 * H2;
  float* sAct = sB2 + H2;  // [H2 / 4 final-layer steps][64 lanes]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, j = lane & 15;
  const int NC = (int)(H2 / 16);
  const uint64_t v = (uint64_t)blockIdx.x * 16;
  if (v >= A.n_ids) return;  // uniform per workgroup
  {
    const uint4* src = reinterpret_cast<const uint4*>(A.pd.wo);
    uint4* dst = reinterpret_cast<uint4*>(sWo);
    for (int i = tid; i < (int)(16 * H2 / 4); i += T) dst[i] = src[i];
    for (int i = tid; i < (int)H2; i += T) sB2[i] = A.pd.b2[i];
  }
  // layer-1 activations of compound v + j
  uint64_t item = v + j;
  item = item < A.n_ids ? item : (uint64_t)A.n_ids - 1;
  const uint64_t id = A.ids[item];
  const ReactDev rr = A.react[find_reaction(A.react, (uint32_t)A.n_reactions, id)];
  const uint64_t loc = id - rr.id_off;
  // ids past the library end are clamped to rows in bounds (reported as NaN)
  const uint64_t a64 = loc / rr.nB;
  const uint32_t a = a64 < rr.nA ? (uint32_t)a64 : rr.nA - 1;
  const uint32_t b = (uint32_t)(loc % rr.nB);
  const float* pa;
  const float* pa1 = nullptr;
  if (rr.three) {
    const uint32_t i0 = a / rr.n1, i1 = a - i0 * rr.n1;
    pa = A.P + (uint64_t)(rr.row0 + i0) * H1 + g * KG;
    pa1 = A.P + (uint64_t)(rr.row1 + i1) * H1 + g * KG;
  } else {
    pa = A.P + (uint64_t)(rr.row0 + a) * H1 + g * KG;
  }
  const float* pb = A.P + (uint64_t)(rr.rowB + b) * H1 + g * KG;
  float X[NS];
#pragma unroll
  for (int s4 = 0; s4 < NS / 4; ++s4) {
    float4 xa = *reinterpret_cast<const float4*>(pa + 4 * s4);
    if (pa1) {
      const float4 xq = *reinterpret_cast<const float4*>(pa1 + 4 * s4);
      xa = make_float4(xa.x + xq.x, xa.y + xq.y, xa.z + xq.z, xa.w + xq.w);
    }
    const float4 xb = *reinterpret_cast<const float4*>(pb + 4 * s4);
    X[4 * s4 + 0] = act_pre<ACT>(xa.x + xb.x);
    X[4 * s4 + 1] = act_pre<ACT>(xa.y + xb.y);
    X[4 * s4 + 2] = act_pre<ACT>(xa.z + xb.z);
    X[4 * s4 + 3] = act_pre<ACT>(xa.w + xb.w);
    asm volatile("" : "+v"(X[4 * s4 + 0]), "+v"(X[4 * s4 + 1]), "+v"(X[4 * s4 + 2]), "+v"(X[4 * s4 + 3])::"memory");
  }
  __syncthreads();  // sWo, sB2
  // this wave's chunks: GEMM (weights in batches of B fragments, the next
  // batch in flight), then activation and the chunk's final-layer share
  const float* w2 = reinterpret_cast<const float*>(A.pd.w2);
  const float* wof = sWo;
  f32x4 hacc = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int c = wave; c < NC; c += W) {
    f32x4 acc = *reinterpret_cast<const f32x4*>(sB2 + c * 16 + g * 4);
    const float* wc = w2 + (size_t)c * NS * 64 + lane;
    float wb[B], wn[B];
#pragma unroll
    for (int e = 0; e < B; ++e) wb[e] = wc[(size_t)e * 64];
#pragma unroll
    for (int s0 = 0; s0 < NS; s0 += B) {
      asm volatile("" ::: "memory");  // at most two batches of loads in flight
      if (s0 + B < NS) {
#pragma unroll
        for (int e = 0; e < B; ++e) wn[e] = wc[(size_t)(s0 + B + e) * 64];
      }
#pragma unroll
      for (int e = 0; e < B; ++e) acc = mma16x4(wb[e], X[s0 + e], acc);
      if (s0 + B < NS) {
#pragma unroll
        for (int e = 0; e < B; ++e) wb[e] = wn[e];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) sAct[(c * 4 + q) * 64 + lane] = act_pre<ACT>(acc[q]);
  }
  __syncthreads();
  if (wave != 0) return;
  // final layer in chunk order, the tile kernel's accumulation sequence
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int q = 0; q < 4; ++q) hacc = mma16x4(wof[(c * 4 + q) * 64 + lane], sAct[(c * 4 + q) * 64 + lane], hacc);
  }
  const f32x4 h = hacc;
  const uint64_t cid = v + j;
  if (cid < A.n_ids) {
    const float So = A.pd.scal[1];
    float4 o4 = make_float4(fmaf(h[0], So, A.pd.bo[4 * g + 0]), fmaf(h[1], So, A.pd.bo[4 * g + 1]),
                            fmaf(h[2], So, A.pd.bo[4 * g + 2]), fmaf(h[3], So, A.pd.bo[4 * g + 3]));
    if (A.ids[cid] >= A.n_total) o4 = make_float4(NAN, NAN, NAN, NAN);
    *reinterpret_cast<float4*>(A.heads_out + cid * 16 + 4 * g) = o4;
  }
}

}  // namespace apex
