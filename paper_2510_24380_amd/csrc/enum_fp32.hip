// Instantiations of the fused enumeration kernel for APEX_PREC_FP32.
#include "enum_kernel.h"

namespace apex {

#define APEX_K(H1, NL, ACT, G) reinterpret_cast<const void*>(&k_enum<H1, NL, ACT, G>)
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

#define APEX_H1S_GATHER \
  if (h1 == 128 && nl == 1) { APEX_ACTS(128, 1, true) } \
  if (h1 == 256 && nl == 1) { APEX_ACTS(256, 1, true) } \
  if (h1 == 512 && nl == 1) { APEX_ACTS(512, 1, true) }

// Gathers with two hidden layers use k_gather_split (below), not this kernel.
const void* enum_kernel_fp32(int h1, int nl, int act, bool gather) {
  if (gather) { APEX_H1S_GATHER } else { APEX_H1S(false) }
  return nullptr;
}

// Two-hidden-layer gathers of short lists (k_gather_split).
const void* gather_split_fp32(int h1, int act) {
#define APEX_G(H1) \
  if (h1 == H1) { \
    if (act == APEX_ACT_NONE) return reinterpret_cast<const void*>(&k_gather_split<H1, APEX_ACT_NONE>); \
    if (act == APEX_ACT_RELU) return reinterpret_cast<const void*>(&k_gather_split<H1, APEX_ACT_RELU>); \
    if (act == APEX_ACT_SILU) return reinterpret_cast<const void*>(&k_gather_split<H1, APEX_ACT_SILU>); \
  }
  APEX_G(128)
  APEX_G(256)
  APEX_G(512)
#undef APEX_G
  return nullptr;
}

}  // namespace apex
