// Per-query pieces of the search driver, shared by apex_search / apex_search_batch
// and the serving loop (internal).
#pragma once
#include <utility>
#include <vector>

#include "engine_impl.h"

namespace apex {

struct Bump {
  char* base;
  size_t off = 0;
  explicit Bump(void* b) : base((char*)b) {}
  template <class T> T* take(size_t count) {
    const size_t o = off;
    off = (off + count * sizeof(T) + 255) & ~(size_t)255;
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
};

// Device buffers and sizes of one query.
struct QPlan {
  uint32_t k = 0, K = 0, cap = 0, hwm = 0, cap2 = 0, n_flags = 0;
  bool lowp = false;
  QState* st = nullptr;
  float* cand_o = nullptr;
  uint64_t* cand_id = nullptr;
  float* tmp_o = nullptr;
  uint64_t* tmp_id = nullptr;
  uint32_t* rerun = nullptr;      // [n_flags] per-chunk overflow flags
  uint32_t* subset_dev = nullptr; // [ceil(T/32)]
  float* pool_heads = nullptr;
  QState* st2 = nullptr;
  float* cand2_o = nullptr;
  uint64_t* cand2_id = nullptr;
  float* tmp2_o = nullptr;
  uint64_t* tmp2_id = nullptr;
  float* fin_o = nullptr;
  uint64_t* fin_id = nullptr;
  float* fin_heads = nullptr;
  uint32_t* fin_reaction = nullptr;
  uint32_t* fin_synthon = nullptr;
};

uint64_t env_u64(const char* name);
std::vector<std::pair<uint64_t, uint64_t>> chunk_schedule(uint64_t n_tiles, uint64_t tile_compounds);
uint32_t tile_compounds(int prec);
apex_status validate_query(const apex_engine* E, const apex_query* q);
void query_sizes(const apex_query* q, QPlan& P);
// Per-query buffers (n_flags overflow flags) from a bump allocator.
void query_layout(uint32_t n_reactions, uint32_t n_flags, Bump& b, QPlan& P);
QueryDev make_qdev(const apex_engine* E, const apex_query* q, const QPlan& p, bool relaxed, bool stage2);
std::vector<uint32_t> subset_bits(const apex_engine* E, const apex_query* q);
// Threshold state, subset bits and overflow flags of a fresh query (async).
apex_status query_device_init(const apex_engine* E, const apex_query* q, const QPlan& P, hipStream_t s);
apex_status fill_u32(uint32_t* p, uint32_t n, uint32_t v, hipStream_t s);
// One pass of the fused kernel over tiles [v0, v1) of a tile plan (async).
apex_status enum_pass(apex_engine* E, int prec, const SelDev* plan_dev, uint32_t n_sel, uint64_t v0, uint64_t v1,
                      const QueryDev* qd_dev, uint32_t nq, uint64_t compounds, hipStream_t s);
// Compounds of a host tile plan inside tiles [v0, v1).
uint64_t plan_compounds(const apex_engine* E, int prec, const std::vector<SelDev>& plan, uint64_t v0, uint64_t v1);
// Threshold warm start from a sample of compounds for the listed queries (async).
apex_status warm_start(apex_engine* E, int prec, const SelDev* plan_dev, uint32_t n_sel, uint64_t n_comp,
                       uint32_t n_sample, uint64_t* ids, float* heads, const QueryDev* qd_dev, uint32_t nq,
                       hipStream_t s);
// Answer of one query whose enumeration is complete (stage 3-4; synchronises s).
// st_known: the query's threshold state as already read back after its last
// select (saves a synchronisation), or nullptr.
apex_status finish_query(apex_engine* E, const apex_query* q, const QPlan& P, const QueryDev* qd_dev,
                         const QueryDev* qx_dev, hipStream_t s, apex_result* res,
                         const QState* st_known = nullptr);
// Resolves the engine's pending kernel timings (after a synchronisation).
apex_status profile_collect(apex_engine* E);

}  // namespace apex
