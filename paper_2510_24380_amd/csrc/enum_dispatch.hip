// Selection and launch of the fused enumeration kernel instantiations.
#include "enum_kernel.h"
#include "enum32_kernel.h"
#include "launch.h"

namespace apex {

const void* enum_kernel_fp32(int h1, int nl, int act, bool gather);
const void* enum_kernel_bf16(int h1, int nl, int act, bool gather);
const void* enum_kernel_fp8(int h1, int nl, int act, bool gather);
const void* gather_split_fp32(int h1, int act);

// FP32 gathers with two hidden layers use the split-chunk kernel
static bool split_gather(int prec, int nl, bool gather) { return prec == APEX_PREC_FP32 && nl == 2 && gather; }

static const void* enum_kernel(int prec, int h1, int nl, int act, bool gather) {
  if (split_gather(prec, nl, gather)) return gather_split_fp32(h1, act);
  if (prec == APEX_PREC_FP32) return enum_kernel_fp32(h1, nl, act, gather);
  if (prec == APEX_PREC_BF16) return enum_kernel_bf16(h1, nl, act, gather);
  if (prec == APEX_PREC_FP8) return enum_kernel_fp8(h1, nl, act, gather);
  return nullptr;
}

uint32_t gather_per_block(int prec, int nl) {
  return split_gather(prec, nl, true) ? 16u : (uint32_t)(enum_waves(prec) * enum_rows(prec) * 16);
}

static int lds_bytes(int prec, int h1, int nl, int h2, bool gather) {
  if (split_gather(prec, nl, gather)) return gather_split_lds_bytes(h2);
  return prec == APEX_PREC_FP32 ? enum_lds_bytes(h1, nl, h2, gather) : enum32_lds_bytes(prec, h1, nl, h2, gather);
}

hipError_t enum_prepare(int prec, int h1, int nl, int act, bool gather, uint32_t h2, int* max_wg_per_cu) {
  const void* k = enum_kernel(prec, h1, nl, act, gather);
  if (!k) return hipErrorInvalidValue;
  const int lds = lds_bytes(prec, h1, nl, (int)h2, gather);
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  if (max_wg_per_cu) {
    int n = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, enum_waves(prec) * 64, lds);
    if (e != hipSuccess) return e;
    *max_wg_per_cu = n;
  }
  return hipSuccess;
}

hipError_t launch_enum(int prec, int h1, int nl, int act, bool gather, const EnumArgs& a, uint32_t grid,
                       hipStream_t s) {
  const void* k = enum_kernel(prec, h1, nl, act, gather);
  if (!k) return hipErrorInvalidValue;
  const int lds = lds_bytes(prec, h1, nl, (int)a.H2, gather);
  void* args[] = {const_cast<EnumArgs*>(&a)};
  return hipLaunchKernel(k, dim3(grid), dim3(enum_waves(prec) * 64), args, (size_t)lds, s);
}

}  // namespace apex
