// Fused enumeration kernel for BF16 and FP8 on the 32x32 MFMA shapes of gfx950
// (v_mfma_f32_32x32x16_bf16, v_mfma_scale_f32_32x32x64_f8f6f4). Same method and
// tile decomposition as the 16x16 kernel in enum_kernel.h (Section 4.2-4.3: the
// summed, hoisted first layer, then act -> GEMM -> act -> final layer per
// compound, with the query's objective, bounds and threshold filter fused in);
// what differs is the operand geometry. The 32x32 shapes leave the vector ALU
// more issue slots next to the matrix core than the 16x16 ones, and the
// activations (two transcendentals each) are as much work as the MFMAs here.
//
// Geometry: 4 waves per workgroup, 32 compounds per wave, one per MFMA column
// (column j = lane % 32: A-row 2 w + j / 16 of the tile, B-row j % 16). A tile
// is 8 A-rows x 16 B-rows. Lane half h = lane / 32 owns first-layer neurons
// [h H1/2, (h+1) H1/2); k-step s covers E consecutive ones of them.
//
// MFMA 32x32 layouts (D = A * B, A 32 x K, B K x 32, lane l, h = l / 32):
//   A: row l % 32, elements k = h E .. h E + E - 1 of the step
//   B: column l % 32, same k
//   D: column l % 32, accumulator v at row 8 (v / 4) + 4 h + v % 4
// GEMM chunks are 32 output neurons; the final layer (heads as A rows, padded
// to 32) takes the chunk's 16 activations per lane directly as two k = 16 steps,
// so the contraction index is permuted on the host and no data moves between
// lanes. Lane halves hold heads {4h..4h+3} and {8+4h..8+4h+3} (accumulators
// 0..7); accumulators 8..15 are padding rows.
#pragma once
#include "enum_common.h"

namespace apex {

typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

template <int PREC> struct Mfma32;
// mma(a, b, c, sa): c + a b, times 2^(sa - 127) for FP8 (sa: E8M0 scale of
// the A operand; BF16 has no scale and ignores it).
// frag(base, s, lane): the lane's weight fragment of k-step s of a chunk in LDS
// (k-step blocks of 64 lanes x 16 bytes; FP8 keeps a lane's two halves in two
// consecutive blocks).
template <> struct Mfma32<APEX_PREC_BF16> {
  static constexpr int KS = 16, E = 8, EB = 2;
  using frag = bf16x8;
  __device__ static inline f32x16 mma(frag a, frag b, f32x16 c, int) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static inline frag frag_at(const unsigned char* base, int s, int lane) {
    return *reinterpret_cast<const frag*>(base + (size_t)(s * 64 + lane) * 16);
  }
};
template <> struct Mfma32<APEX_PREC_FP8> {
  static constexpr int KS = 64, E = 32, EB = 1;
  using frag = i32x8;
  __device__ static inline frag frag_at(const unsigned char* base, int s, int lane) {
    typedef __attribute__((__vector_size__(4 * sizeof(int)))) int i32x4;
    const i32x4 lo = *reinterpret_cast<const i32x4*>(base + (size_t)(s * 128 + lane) * 16);
    const i32x4 hi = *reinterpret_cast<const i32x4*>(base + (size_t)(s * 128 + 64 + lane) * 16);
    return frag{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  }
  __device__ static inline f32x16 mma(frag a, frag b, f32x16 c, int sa) {
    // E4M3 x E4M3 (format selectors 0); E8M0 scales sa on A, 127 (one) on B
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, sa, 0, 127);
  }
};
constexpr int kE8M0One = 127;

constexpr int kTileA32 = 8;  // A-rows per tile (2 per wave)
// Word 3 of a raw buffer resource on gfx9-family parts (32-bit data format;
// untyped loads use only the range and base).
constexpr int kBufferWord3 = 0x00020000;

// Row of accumulator v of lane half h in a 32x32 D tile.
__host__ __device__ constexpr int d32_row(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

// LDS bytes of the 32x32 kernel (host and device agree on this): staged rows
// and the double-buffered 32-neuron weight chunks share one region; GEMM start
// values stay resident; a one-hidden-layer decoder keeps its output weights in
// LDS, a two-hidden-layer one reads them from the caches.
__host__ __device__ constexpr int enum32_lds_bytes(int prec, int h1, int nl, int h2, bool gather) {
  int eb = prec == APEX_PREC_BF16 ? 2 : 1;
  int rows = gather ? 0 : (kTileA32 + kTileB) * (h1 + kRowPad) * 4;
  int chunk = nl == 2 ? 2 * 32 * h1 * eb : 0;
  int region = rows > chunk ? rows : chunk;
  int wo = nl == 1 ? 32 * h1 * eb : 0;
  int b2 = nl == 2 ? h2 * 4 : 0;
  return region + wo + b2 + kHeadsPad * 4 + (gather ? 0 : kQLdsBytes);  // + final bias, query parameters
}

template <int PREC, int H1, int NL, int ACT, bool GATHER>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_enum32(EnumArgs A) {
  using M = Mfma32<PREC>;
  using Frag = typename M::frag;
  constexpr int W = 4, T = 256;
  constexpr int TA = kTileA32, TB = kTileB;
  constexpr int E = M::E;
  constexpr int NS = H1 / M::KS;  // k-steps over the first hidden width
  constexpr int KH = H1 / 2;      // first-layer neurons per lane half
  constexpr int ROW = H1 + kRowPad;
  constexpr int CHUNK = 32 * H1 * M::EB;  // bytes of one 32-neuron GEMM weight chunk
  constexpr int NPRE = CHUNK / 16 / T;    // 16-byte pieces of a chunk per thread
  constexpr int ROWS_BYTES = GATHER ? 0 : (TA + TB) * ROW * 4;
  constexpr int REGION = ROWS_BYTES > (NL == 2 ? 2 * CHUNK : 0) ? ROWS_BYTES : (NL == 2 ? 2 * CHUNK : 0);
  static_assert(NS * E == KH, "layout");
  static_assert(CHUNK % (16 * T) == 0, "chunk split");
  static_assert(NL >= 1, "the linear decoder runs in the FP32 kernel");

  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  float* sA = reinterpret_cast<float*>(smem);
  float* sB = sA + TA * ROW;
  unsigned char* sW = smem;  // GEMM weight chunks share the region with the staged rows
  unsigned char* sWo = smem + REGION;  // one-hidden-layer output weights
  float* sB2 = reinterpret_cast<float*>(smem + REGION);  // two-hidden-layer GEMM start values
  // final bias, read from LDS in the epilogue (a global pointer to it would be
  // hoisted out of the tile loop and held in registers)
  float* sBo = reinterpret_cast<float*>(smem + REGION + (NL == 1 ? 32 * H1 * M::EB : 0)) + (NL == 2 ? A.H2 : 0);
  QLds* sQ = reinterpret_cast<QLds*>(sBo + kHeadsPad);  // tile mode: one entry per query

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, j = lane & 31;
  const uint32_t H2 = NL == 2 ? A.H2 : 0;
  const int NC = NL == 2 ? (int)(H2 / 32) : 0;
  const float So = A.pd.scal[1], XS = A.pd.scal[2];
  // the GEMM's power-of-two scale S2 as an E8M0 exponent (127 + log2 S2)
  const int s2e = (int)((__float_as_uint(A.pd.scal[0]) >> 23) & 0xffu);

  // Work range: XCD-aware contiguous runs, or (tile mode with work counters)
  // runs taken at run time (take_tile_run).
  const bool dyn = !GATHER && A.work != nullptr;
  uint64_t v, vend;
  {
    const uint32_t G = gridDim.x, bid = blockIdx.x;
    const uint32_t per_xcd = G / 8;
    const uint32_t wg = (G % 8 == 0) ? (bid % 8) * per_xcd + bid / 8 : bid;
    if (GATHER) {
      const uint64_t per_wg = W * 32;
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
  __shared__ uint64_t s_run[3];  // dynamic work: the run taken, regions used up
  if (dyn && tid == 0) s_run[2] = 0;
  auto take_run = [&]() { take_tile_run(A, s_run, v, vend); };

  // Resident LDS: GEMM start values, or the one-hidden-layer output weights.
  {
    if (NL == 2)
      for (int i = tid; i < (int)H2; i += T) sB2[i] = A.pd.b2[i];
    if (tid < kHeadsPad) sBo[tid] = A.pd.bo[tid];
    if (!GATHER) copy_queries_lds(A, sQ, wave, W, lane);
    if (NL == 1) {
      const uint4* src = reinterpret_cast<const uint4*>(A.pd.wo);
      uint4* dst = reinterpret_cast<uint4*>(sWo);
      for (int i = tid; i < 32 * H1 * M::EB / 16; i += T) dst[i] = src[i];
    }
    __syncthreads();  // gather mode stages no rows, so no later barrier precedes the first read
  }
  // Weight loads are buffer loads: the uniform part of the address lives in the
  // scalar resource and offset, the per-thread part is one 32-bit register, so
  // no 64-bit address per load is kept live across the loops (reads past the
  // resource's size return zeros instead of faulting).
  const __amdgpu_buffer_rsrc_t w2r = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(A.pd.w2), (short)0, NL == 2 ? NC * CHUNK : 0, kBufferWord3);
  const __amdgpu_buffer_rsrc_t wor =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(A.pd.wo), (short)0, NL == 2 ? NC * 2048 : 0, kBufferWord3);
  auto ldb16 = [](__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    return make_uint4(v[0], v[1], v[2], v[3]);
  };
  // GEMM weight chunk c -> LDS buffer buf, by loads that write LDS directly (no
  // registers held, no LDS stores issued): the q-th 1 KB block of wave w is
  // bytes q T 16 + 1024 w of the chunk, placed at the same offset of the buffer,
  // 16 bytes per lane. They are waited for right before the barrier that
  // publishes the buffer, a whole chunk later.
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);  // wave-uniform (scalar) offsets
  auto load_chunk = [&](int c, int buf) {
#pragma unroll
    for (int q = 0; q < NPRE; ++q) {
      const uint32_t off = (uint32_t)(q * T * 16 + wave_u * 1024);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          w2r, (__attribute__((address_space(3))) void*)(sW + buf * CHUNK + off), 16, 16u * (uint32_t)lane,
          (uint32_t)(c * CHUNK) + off, 0, 0);
    }
  };
  auto publish = [&]() {  // the chunk loads of this thread done, then all threads
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };

  if (dyn) take_run();
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

  for (; v < vend || (dyn && (take_run(), v < vend)); v += (GATHER ? vend : 1)) {
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
      // All loads of the tile's rows are issued before the first LDS store, so
      // one memory latency (not one per row piece) is exposed. Which of a
      // thread's pieces are A rows is the same for every thread.
      constexpr int V4 = H1 / 4;
      constexpr int NSTG = (TA + TB) * V4 / T;  // 16-byte pieces per thread
      constexpr int NSA = TA * V4 / T;          // of which A-row pieces
      constexpr int RPK = T / V4;               // rows advanced per piece
      static_assert(T % V4 == 0 && TA % RPK == 0, "staging split");
      // piece k of this thread: row k * RPK + r0, 16-byte column c4 (the same
      // for every k), so its LDS address is one register plus a constant
      const int r0 = tid / V4, c4 = tid % V4;
      float* const sdst = sA + r0 * ROW + 4 * c4;
      float4 stg[NSTG], stq[NSA];
#pragma unroll
      for (int k = 0; k < NSTG; ++k) {
        const int row = k * RPK + r0;
        if (k < NSA) {
          uint32_t a = a0 + row;
          a = a < Rt.nA ? a : Rt.nA - 1;
          if (Rt.three) {
            const uint32_t i0 = a / Rt.n1, i1 = a - i0 * Rt.n1;
            stg[k] = reinterpret_cast<const float4*>(A.P + (uint64_t)(Rt.row0 + i0) * H1)[c4];
            stq[k] = reinterpret_cast<const float4*>(A.P + (uint64_t)(Rt.row1 + i1) * H1)[c4];
          } else {
            stg[k] = reinterpret_cast<const float4*>(A.P + (uint64_t)(Rt.row0 + a) * H1)[c4];
          }
        } else {
          uint32_t b = b0 + (row - TA);
          b = b < Rt.nB ? b : Rt.nB - 1;
          stg[k] = reinterpret_cast<const float4*>(A.P + (uint64_t)(Rt.rowB + b) * H1)[c4];
        }
      }
#pragma unroll
      for (int k = 0; k < NSTG; ++k) {
        float4 val = stg[k];
        if (k < NSA && Rt.three) {
          const float4 q = stq[k];
          val = make_float4(val.x + q.x, val.y + q.y, val.z + q.z, val.w + q.w);
        }
        // sB follows sA, so rows from TA on land in sB
        *reinterpret_cast<float4*>(sdst + k * RPK * ROW) = val;
      }
      __syncthreads();
    }

    // ---------------- layer-1 activations into registers ----------------
    const float* pa;
    const float* pa1 = nullptr;
    const float* pb;
    if (!GATHER) {
      pa = sA + (2 * wave + (j >> 4)) * ROW + h * KH;
      pb = sB + (j & 15) * ROW + h * KH;
    } else {
      uint64_t item = v + (uint64_t)wave * 32 + j;
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
        pa = A.P + (uint64_t)(rr.row0 + i0) * H1 + h * KH;
        pa1 = A.P + (uint64_t)(rr.row1 + i1) * H1 + h * KH;
      } else {
        pa = A.P + (uint64_t)(rr.row0 + a) * H1 + h * KH;
      }
      pb = A.P + (uint64_t)(rr.rowB + b) * H1 + h * KH;
    }
    // Row values are read DU 16-byte units ahead of their use (a small software
    // pipeline), and a fence after each fragment keeps the compiler from
    // hoisting every read of the phase ahead of the activations.
    constexpr int DU = GATHER ? 4 : 2;  // LDS reads need less lead than global ones
    constexpr int NU = KH / 4;  // 16-byte units per lane and row
    float4 ra[DU], rb[DU], rq[DU];
#pragma unroll
    for (int u = 0; u < DU; ++u) {
      ra[u] = *reinterpret_cast<const float4*>(pa + 4 * u);
      rb[u] = *reinterpret_cast<const float4*>(pb + 4 * u);
      if (GATHER && pa1) rq[u] = *reinterpret_cast<const float4*>(pa1 + 4 * u);
    }
    Frag X[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      Frag f;
#pragma unroll
      for (int e4 = 0; e4 < E / 4; ++e4) {
        const int u = s * (E / 4) + e4;
        float4 xa = ra[u % DU];
        const float4 xb = rb[u % DU];
        if (GATHER && pa1) {
          const float4 xq = rq[u % DU];
          xa = make_float4(xa.x + xq.x, xa.y + xq.y, xa.z + xq.z, xa.w + xq.w);
        }
        if (u + DU < NU) {
          ra[u % DU] = *reinterpret_cast<const float4*>(pa + 4 * (u + DU));
          rb[u % DU] = *reinterpret_cast<const float4*>(pb + 4 * (u + DU));
          if (GATHER && pa1) rq[u % DU] = *reinterpret_cast<const float4*>(pa1 + 4 * (u + DU));
        }
        Pack<PREC>::put4(f, e4, act_pre<ACT>(xa.x + xb.x), act_pre<ACT>(xa.y + xb.y), act_pre<ACT>(xa.z + xb.z),
                         act_pre<ACT>(xa.w + xb.w), XS);
      }
      asm volatile("" : "+v"(f)::"memory");
      X[s] = f;
    }

    // ---------------- decoder layers on MFMA ----------------
    f32x16 hacc = {};
    if constexpr (NL == 1) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const Frag wo = M::frag_at(sWo, s, lane);
        hacc = M::mma(wo, X[s], hacc, kE8M0One);
      }
    } else {
      // The staged rows are no longer needed: the region takes the weight chunks.
      __syncthreads();
      // Waves in their GEMM phase issue before waves (of the other workgroup on
      // this CU) in their activation phase, so the matrix core is fed first and
      // the activation work fills the gaps (FP8 kernel time -7 %, BF16 -1.5 %).
      __builtin_amdgcn_s_setprio(1);
      load_chunk(0, 0);
      publish();

      // Static plan of the previous chunk's activation work over the k-steps
      // of a GEMM: activation v runs its four operations (exp2, add, rcp, mul)
      // DF steps apart, starting at step t0(v); pairs are converted to BF16 a
      // step after their last multiply; each final-layer MFMA follows its
      // eight conversions. Short GEMMs (under 8 steps) do all of it last.
      constexpr int DF = 1;
      auto fstep = [](int v, int op) {
        if (NS < 8) return NS - 1;
        const int t = v * (NS - 3 * DF) / 16 + op * DF;
        return t < NS ? t : NS - 1;
      };
      auto cstep = [&](int i) {  // BF16 conversion of activations 2i, 2i + 1
        const int t = fstep(2 * i + 1, 3) + 1;
        return t < NS ? t : NS - 1;
      };
      auto mstep = [&](int st) {  // final-layer MFMA of activations 8 st .. 8 st + 7
        int t = 0;
        for (int i = 4 * st; i < 4 * st + 4; ++i) t = cstep(i) > t ? cstep(i) : t;
        return t + 1 < NS ? t + 1 : NS - 1;
      };

      // One chunk of 32 neurons: start the loads of the next chunk (pf) into
      // the other buffer (last read in the chunk before this one, which every
      // wave has finished), run the GEMM steps into `acc`, and (fin)
      // interleave the activation and final layer of the previous chunk
      // (`old`, chunk c_old) with them. pf and fin are literals at every call.
      // Each step ends in a scheduling barrier, so the interleave is the one
      // written here: the weight read two steps ahead, the MFMA, then this
      // step's share of the activation work.
      auto gemm = [&](int c, f32x16& acc, bool pf, const f32x16& old, int c_old, bool fin) {
        // The start values and the final-layer weights are requested before the
        // next chunk's loads: the compiler cannot tell that those loads leave
        // the start values alone, and would otherwise wait for all of them here
        // (and, the counter being in order, for them again before the final layer).
        const float* b2c = sB2 + c * 32 + 4 * h;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 bq = *reinterpret_cast<const float4*>(b2c + 8 * q);
          acc[4 * q] = bq.x;
          acc[4 * q + 1] = bq.y;
          acc[4 * q + 2] = bq.z;
          acc[4 * q + 3] = bq.w;
        }
        bf16x8 wo[2];
        if (fin) {
#pragma unroll
          for (int st = 0; st < 2; ++st)
            wo[st] = __builtin_bit_cast(bf16x8, ldb16(wor, 16u * (uint32_t)lane, (uint32_t)(c_old * 2048 + st * 1024)));
        }
        if (pf) load_chunk(c + 1, (c + 1) & 1);
        const unsigned char* wc = sW + (c & 1) * CHUNK;
        Frag ring[3];
        ring[0] = M::frag_at(wc, 0, lane);
        if (NS > 1) ring[1] = M::frag_at(wc, 1, lane);
        float y[16], tq[16];
        bf16x8 xb[2];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          if (s + 2 < NS) ring[(s + 2) % 3] = M::frag_at(wc, s + 2, lane);
          acc = M::mma(ring[s % 3], X[s], acc, s2e);
          if (fin) {
            // the operations of act_pre, one at a time (same arithmetic)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              if (fstep(v, 0) == s) {
                float u = old[v];
                if constexpr (ACT == APEX_ACT_SILU) {
                  y[v] = u;
                  tq[v] = __builtin_amdgcn_exp2f(u);
                } else {
                  y[v] = act_pre<ACT>(u);
                }
              }
              if constexpr (ACT == APEX_ACT_SILU) {
                if (fstep(v, 1) == s) tq[v] = 1.0f + tq[v];
                if (fstep(v, 2) == s) tq[v] = __builtin_amdgcn_rcpf(tq[v]);
                if (fstep(v, 3) == s) y[v] = y[v] * tq[v];
              }
            }
#pragma unroll
            for (int i = 0; i < 8; ++i)
              if (cstep(i) == s) {
                xb[i >> 2][2 * (i & 3)] = (__bf16)y[2 * i];
                xb[i >> 2][2 * (i & 3) + 1] = (__bf16)y[2 * i + 1];
              }
#pragma unroll
            for (int st = 0; st < 2; ++st)
              if (mstep(st) == s) hacc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wo[st], xb[st], hacc, 0, 0, 0);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      };
      // the activation and final layer of one chunk on their own (last chunk)
      // (its final-layer weights wo are requested before the chunk's GEMM)
      auto finish = [&](const f32x16& acc, const bf16x8 (&wo_c)[2]) {
#pragma unroll
        for (int st = 0; st < 2; ++st) {
          const bf16x8 wo = wo_c[st];
          bf16x8 xb;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            float u = acc[8 * st + e];
            xb[e] = (__bf16)act_pre<ACT>(u);
          }
          hacc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wo, xb, hacc, 0, 0, 0);
        }
      };
      // NC is even (the host pads the width to a multiple of 64 neurons)
      f32x16 accA, accB;
      gemm(0, accA, true, accB, 0, false);
      publish();
      int c = 1;
      for (; c + 2 < NC; c += 2) {  // chunks c and c + 1 both have a successor
        gemm(c, accB, true, accA, c - 1, true);
        publish();
        gemm(c + 1, accA, true, accB, c, true);
        publish();
      }
      bf16x8 wo_last[2];
#pragma unroll
      for (int st = 0; st < 2; ++st)
        wo_last[st] = __builtin_bit_cast(bf16x8, ldb16(wor, 16u * (uint32_t)lane, (uint32_t)(c * 2048 + st * 1024)));
      gemm(c, accB, false, accA, c - 1, true);  // c == NC - 1
      finish(accB, wo_last);
      __syncthreads();  // the region is restaged by the next tile
    }

    __builtin_amdgcn_s_setprio(0);
    // ---------------- heads, objective, bounds, filter ----------------
    // The thread's tile coordinates are recomputed here from a copy of the
    // thread index the compiler cannot see through, so they are not kept live
    // (or spilled) across the whole tile loop.
    int tl = tid;
    asm volatile("" : "+v"(tl));
    const int jl = tl & 31;
    uint64_t cid;  // compound id (tile mode) or list position (gather mode)
    bool valid;
    if (!GATHER) {
      const uint32_t a = a0 + 2 * (tl >> 6) + (jl >> 4), b = b0 + (jl & 15);
      valid = a < Rt.nA && b < Rt.nB;
      cid = Rt.id_off + (uint64_t)a * Rt.nB + b;
    } else {
      cid = v + (uint64_t)(tl >> 6) * 32 + jl;
      valid = cid < A.n_ids;
    }
    // accumulators 0..3: heads 4h..4h+3; 4..7: heads 8+4h..8+4h+3
    float hd[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) hd[q] = fmaf(hacc[q], So, sBo[d32_row(q, h)]);

    if constexpr (GATHER) {
      if (valid) {
        float4 lo4 = make_float4(hd[0], hd[1], hd[2], hd[3]);
        float4 hi4 = make_float4(hd[4], hd[5], hd[6], hd[7]);
        if (A.ids[cid] >= A.n_total) lo4 = hi4 = make_float4(NAN, NAN, NAN, NAN);
        *reinterpret_cast<float4*>(A.heads_out + cid * 16 + 4 * h) = lo4;
        *reinterpret_cast<float4*>(A.heads_out + cid * 16 + 8 + 4 * h) = hi4;
      }
    } else {
      for (uint32_t qi = 0; qi < A.n_queries; ++qi) {
        const QLds* L = sQ + qi;
        if (!L->active) continue;
        if (L->subset_bits && !((L->subset_bits[S.t >> 5] >> (S.t & 31)) & 1u)) continue;
        const QueryDev* Q = A.queries + qi;  // appends only
        const float tau_o = L->tau_o;
        const uint64_t tau_id = L->tau_id;
        // objective in the order of the other kernels: groups of four heads,
        // (g0 + g1) + (g2 + g3); this lane half holds groups h and 2 + h
        float pA = obj_partial(L->w + 4 * h, hd);
        float pB = obj_partial(L->w + 8 + 4 * h, hd + 4);
        int ok = 1;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int hh = d32_row(q, h);
          ok &= (hd[q] >= L->lo[hh]) & (hd[q] <= L->hi[hh]);
        }
        const float oA = __shfl_xor(pA, 32), oB = __shfl_xor(pB, 32);
        ok &= __shfl_xor(ok, 32);
        const float o = canon_zero(h == 0 ? (pA + oA) + (pB + oB) : 0.0f);
        const bool pass = h == 0 && valid && ok && finite_obj(o) && key_passes(o, cid, tau_o, tau_id);
        const uint64_t m = __ballot(pass);
        if (m) {
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(&Q->st->count, (uint32_t)__popcll(m));
          base = __shfl(base, 0);
          if (pass) {
            const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
            const uint32_t idx = base + (uint32_t)__popcll(m & below);
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

}  // namespace apex
