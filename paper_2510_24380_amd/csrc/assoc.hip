// Associative embeddings (Section 4.2, eq. "assoc_embeds"): the table row of
// R-group r (a reaction's slot) and synthon s is u_{r,s} = K_r v_s, with K_r a
// d x dU key matrix per R-group and v_s a dU value vector per synthon. This is
// the step that produces the library tables the search consumes; per R-group
// it is the GEMM U_r = V_r K_r^T over the slot's synthon rows, run as a grouped
// GEMM on the FP32 matrix cores (16x16x4 MFMA, FP32 accumulation).
//
// One wave per 16 synthon rows of one slot: every 128 output columns take 8
// accumulator tiles, the value index advancing in steps of 4 (one value and
// eight key entries per lane and step). A 16x16x4 step has lane l supply
// A[l % 16][l / 16] (a value) and B[l / 16][l % 16] (a key entry, B = K_r^T) and
// return rows 4 (l / 16) + v, column l % 16 of the tile.
#include "enum_common.h"
#include "launch.h"

namespace apex {

constexpr int kAssocWaves = 4;
constexpr int kAssocMaxDU = 256;
constexpr int kAssocCols = 128;  // output columns per accumulator pass

__device__ __forceinline__ uint32_t find_assoc(const AssocSlot* s, uint32_t n, uint64_t v) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (s[mid].tile0 <= v) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kAssocWaves * 64) void k_assoc(const AssocSlot* __restrict__ slots, uint32_t n_slots,
                                                          uint64_t n_tiles, uint32_t d, uint32_t dU,
                                                          const float* __restrict__ keys,
                                                          const float* __restrict__ values, float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const uint64_t stride = (uint64_t)gridDim.x * kAssocWaves;
  const int r16 = lane & 15, k4 = lane >> 4;
  for (uint64_t v = (uint64_t)blockIdx.x * kAssocWaves + (threadIdx.x >> 6); v < n_tiles; v += stride) {
    const uint32_t si = find_assoc(slots, n_slots, v);
    const AssocSlot S = slots[si];
    const uint32_t i0 = (uint32_t)(v - S.tile0) * 16;
    const float* K = keys + (uint64_t)si * d * dU;
    const bool row_ok = i0 + r16 < S.n;
    const float* vrow = values + (S.row0 + i0 + r16) * (uint64_t)dU;
    for (uint32_t c0 = 0; c0 < d; c0 += kAssocCols) {
      f32x4 acc[kAssocCols / 16];
#pragma unroll
      for (int t = 0; t < kAssocCols / 16; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
      for (uint32_t k0 = 0; k0 < dU; k0 += 4) {
        const uint32_t kk = k0 + k4;
        const float a = (row_ok && kk < dU) ? vrow[kk] : 0.0f;  // A[r16][k4] = V[i0 + r16][kk]
#pragma unroll
        for (int t = 0; t < kAssocCols / 16; ++t) {
          const uint32_t j = c0 + 16 * t + r16;
          const float b = (j < d && kk < dU) ? K[(uint64_t)j * dU + kk] : 0.0f;  // B[k4][r16] = K[j][kk]
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
        }
      }
#pragma unroll
      for (int t = 0; t < kAssocCols / 16; ++t) {
        const uint32_t j = c0 + 16 * t + r16;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t i = i0 + 4 * k4 + q;
          if (i < S.n && j < d) out[(S.row0 + i) * (uint64_t)d + j] = acc[t][q];
        }
      }
    }
  }
}

hipError_t launch_assoc(const AssocSlot* slots, uint32_t n_slots, uint64_t n_tiles, uint32_t d, uint32_t dU,
                        const float* keys, const float* values, float* out, int n_cu, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  if (dU == 0 || dU > (uint32_t)kAssocMaxDU) return hipErrorInvalidValue;
  const uint64_t want = (n_tiles + kAssocWaves - 1) / kAssocWaves;
  const uint64_t cap = (uint64_t)std::max(1, n_cu) * 8;
  const uint32_t grid = (uint32_t)(want < cap ? want : cap);
  hipLaunchKernelGGL(k_assoc, dim3(grid), dim3(kAssocWaves * 64), 0, s, slots, n_slots, n_tiles, d, dU, keys, values,
                     out);
  return hipGetLastError();
}

}  // namespace apex
