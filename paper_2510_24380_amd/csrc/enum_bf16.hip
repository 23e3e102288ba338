// Instantiations of the 32x32-MFMA fused enumeration kernel for APEX_PREC_BF16.
#include "enum32_kernel.h"

namespace apex {

#define APEX_K(H1, NL, ACT, G) reinterpret_cast<const void*>(&k_enum32<APEX_PREC_BF16, H1, NL, ACT, G>)
#define APEX_ACTS(H1, NL, G) \
  if (act == APEX_ACT_NONE) return APEX_K(H1, NL, APEX_ACT_NONE, G); \
  if (act == APEX_ACT_RELU) return APEX_K(H1, NL, APEX_ACT_RELU, G); \
  if (act == APEX_ACT_SILU) return APEX_K(H1, NL, APEX_ACT_SILU, G);
#define APEX_NLS(H1, G) \
  if (nl == 1) { APEX_ACTS(H1, 1, G) } \
  if (nl == 2) { APEX_ACTS(H1, 2, G) }
#define APEX_H1S(G) \
  if (h1 == 128) { APEX_NLS(128, G) } \
  if (h1 == 256) { APEX_NLS(256, G) } \
  if (h1 == 512) { APEX_NLS(512, G) }

const void* enum_kernel_bf16(int h1, int nl, int act, bool gather) {
  if (gather) { APEX_H1S(true) } else { APEX_H1S(false) }
  return nullptr;
}

}  // namespace apex
