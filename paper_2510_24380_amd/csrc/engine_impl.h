// Host-side handle types behind the opaque pointers of include/apex.h.
#pragma once
#include <atomic>
#include <mutex>
#include <utility>
#include <vector>

#include "apex_internal.h"

struct apex_library {
  uint32_t T = 0;
  uint32_t d = 0;
  const float* tables = nullptr;
  uint64_t rows = 0;
  uint64_t total = 0;
  std::vector<uint32_t> n_slots;     // [T]
  std::vector<uint32_t> slot_base;   // [T] index of the reaction's first slot
  std::vector<uint32_t> slot_sizes;  // [sum n_slots]
  std::vector<uint64_t> row_base;    // [sum n_slots] first table row of each slot
  std::vector<uint64_t> id_off;      // [T + 1]
};

struct apex_decoder {
  uint32_t L = 0;
  uint32_t act = 0;
  std::vector<uint32_t> dims;
  std::vector<const float*> W, b;
};

namespace apex {

struct PrecState {
  uint32_t h2k = 0;  // second hidden width as the kernel runs it (BF16/FP8: padded to 64, zero neurons)
  bool on = false;
  void* w2 = nullptr;
  void* wo = nullptr;
  float* b2 = nullptr;
  float* bo = nullptr;
  float* scal = nullptr;
  float* amax = nullptr;
  float* herr = nullptr;          // device: largest calibration error per head
  SelDev* plan = nullptr;         // device: whole-library tile plan
  uint64_t full_tiles = 0, full_compounds = 0;
  int wg_per_cu = 0;
  float delta[kHeadsPad] = {};    // host: per-head bound relaxation
  float scal_host[8] = {};
  PrecDev dev{};
};

}  // namespace apex

struct apex_engine {
  apex_library* lib = nullptr;
  uint32_t H1 = 0, H2 = 0, NL = 0, H = 0, act = 0;  // H2: the decoder's second hidden width
  // one-layer (linear-probe) decoder: FP32 searches run the scalar-contribution
  // kernel; HS is the row stride of every heads array (16, or 32 above 16 heads)
  bool scalar = false;
  uint32_t HS = apex::kHeadsPad;
  float c_act = 1.0f;
  std::vector<uint32_t> dims;
  uint32_t mask = 0, user_mask = 0;
  int device = 0, n_cu = 0;
  float* P = nullptr;
  apex::ReactDev* react = nullptr;
  uint8_t* is_slot0 = nullptr;
  uint64_t* slot_row0 = nullptr;
  uint32_t* slot_size = nullptr;
  uint32_t* react_slot0 = nullptr;
  uint32_t* react_nslots = nullptr;
  float* cmax = nullptr;
  float* cmin = nullptr;
  uint64_t* cal_ids = nullptr;
  float* cal_h32 = nullptr;
  float* cal_hlp = nullptr;
  // head quantiles (apex_engine_head_quantiles)
  uint64_t* qnt_ids = nullptr;
  float* qnt_heads = nullptr;
  float* qnt_levels = nullptr;
  float* qnt_out = nullptr;
  apex::PrecState prec[3];
  std::vector<apex::ReactDev> react_host;
  // optional timing of the fused enumeration kernel (HIP events on the search stream)
  bool profile = false;
  double prof_ms = 0.0;
  uint64_t prof_launches = 0, prof_compounds = 0;
  struct Timed {
    hipEvent_t a, b;
    uint64_t compounds;
  };
  std::vector<hipEvent_t> ev_free;
  std::vector<Timed> ev_pending;
  // pinned host buffers for the per-search result readback, reused across
  // searches (host memory; the library allocates no device memory)
  std::mutex pin_mu;
  std::vector<std::pair<void*, size_t>> pin_free;
  ~apex_engine() {
    for (auto e : ev_free) (void)hipEventDestroy(e);
    for (auto& t : ev_pending) {
      (void)hipEventDestroy(t.a);
      (void)hipEventDestroy(t.b);
    }
    for (auto& b : pin_free) (void)hipHostFree(b.first);
  }
};

namespace apex {
apex_status set_error(apex_status s, const char* fmt, ...);
void build_plan(const apex_library* L, bool scalar, const std::vector<uint32_t>& reactions, std::vector<SelDev>& plan,
                uint64_t* n_tiles, uint64_t* n_compounds);
// FP32/BF16/FP8 heads of listed compounds, rows of out_stride floats (0: the
// engine's heads stride; linear-probe engines may write exactly H columns).
apex_status engine_gather(apex_engine* E, int prec, const uint64_t* ids, uint32_t n, float* heads, hipStream_t s,
                          uint32_t out_stride = 0);
}  // namespace apex
