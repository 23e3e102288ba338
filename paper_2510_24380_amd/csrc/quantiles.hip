// Head quantiles over a set of compounds: the percentile thresholds of
// counter-screening queries (Appendix A.11: bounds such as "every off-target
// docking score above its 50th percentile" are set from the library's own
// distribution of predicted heads). One workgroup per head sorts the listed
// compounds' FP32 heads in LDS (bitonic; non-finite values last and left out)
// and interpolates each requested level linearly between closest ranks:
// position p (n - 1) over the n finite values, as in the common "linear"
// quantile definition.
#include "enum_common.h"
#include "launch.h"

namespace apex {

constexpr uint32_t kQuantMax = 8192;  // compounds per call (LDS: 32 KB)
constexpr uint32_t kQuantThreads = 1024;

__global__ __launch_bounds__(kQuantThreads) void k_head_quantiles(const float* __restrict__ heads, uint32_t hs,
                                                                  uint32_t n, const float* __restrict__ levels,
                                                                  uint32_t n_levels, uint32_t H,
                                                                  float* __restrict__ out) {
  __shared__ float v[kQuantMax];
  __shared__ uint32_t n_fin;
  const uint32_t h = blockIdx.x;
  uint32_t m = 1;
  while (m < n) m <<= 1;
  if (threadIdx.x == 0) n_fin = 0;
  __syncthreads();
  uint32_t fin = 0;
  for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
    float x = i < n ? heads[(uint64_t)i * hs + h] : __builtin_inff();
    if (i < n && finite_obj(x)) {
      ++fin;
    } else {
      x = __builtin_inff();
    }
    v[i] = x;
  }
  if (fin) atomicAdd(&n_fin, fin);
  __syncthreads();
  for (uint32_t size = 2; size <= m; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
        const uint32_t j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const float a = v[i], b = v[j];
          if ((a > b) == up) {
            v[i] = b;
            v[j] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  const uint32_t nf = n_fin;
  for (uint32_t l = threadIdx.x; l < n_levels; l += blockDim.x) {
    float q = __builtin_nanf("");
    if (nf > 0) {
      const float p = fminf(fmaxf(levels[l], 0.0f), 1.0f);
      const float pos = p * (float)(nf - 1);
      const uint32_t lo = min((uint32_t)pos, nf - 1), hi = min(lo + 1, nf - 1);
      const float f = pos - (float)lo;
      q = v[lo] + f * (v[hi] - v[lo]);
    }
    out[(uint64_t)l * H + h] = q;
  }
}

hipError_t launch_head_quantiles(const float* heads, uint32_t hs, uint32_t n, const float* levels, uint32_t n_levels,
                                 uint32_t H, float* out, hipStream_t s) {
  if (n == 0 || n > kQuantMax || H == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_head_quantiles, dim3(H), dim3(kQuantThreads), 0, s, heads, hs, n, levels, n_levels, H, out);
  return hipGetLastError();
}

}  // namespace apex
