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

// Device buffers and sizes of one query. The threshold states, the overflow
// flags and the answer form one contiguous readback block [out, out + out_bytes)
// (out_layout), which the host reads in one copy once the search's device work
// is enqueued; the blocks of a batch's queries are adjacent.
struct QPlan {
  uint32_t k = 0, K = 0, cap = 0, hwm = 0, cap2 = 0, n_flags = 0;
  bool lowp = false;
  uint32_t hs = kHeadsPad;        // row stride of the answer's heads
  uint32_t n_cols = 0;            // linear-probe engines: per-row table columns (0 otherwise)
  uint64_t tab_rows = 0;
  ScalarQuery* sq = nullptr;      // linear-probe engines: the query's tables
  float* tab = nullptr;
  uint32_t* rs_hist = nullptr;    // radix-sort scratch (answers above kSortSmallMax entries)
  bool keep = false;              // APEX_QUERY_KEEP_VIOLATORS: layout fits the violation pass too
  bool viol = false;              // this run is the violation pass
  float* fin_c = nullptr;         // violation pass: the answer's violations
  char* out = nullptr;
  size_t out_bytes = 0;
  QState* st = nullptr;
  float* cand_o = nullptr;
  uint64_t* cand_id = nullptr;
  float* tmp_o = nullptr;
  uint64_t* tmp_id = nullptr;
  uint32_t* rerun = nullptr;      // [n_flags] per-chunk overflow flags
  uint32_t* subset_dev = nullptr; // [ceil(T/32)]
  SelScratch* sel = nullptr;      // selection scratch (both stages)
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
uint32_t spec_rank(uint32_t K, uint32_t n_sample, uint64_t n_comp);
uint64_t scalar_sample(uint32_t K, uint64_t total);
std::vector<std::pair<uint64_t, uint64_t>> chunk_schedule(uint64_t n_tiles, uint64_t tile_compounds, bool scalar);
uint32_t tile_compounds(bool scalar);
apex_status validate_query(const apex_engine* E, const apex_query* q);
void query_sizes(const apex_engine* E, const apex_query* q, QPlan& P);
// Per-query working buffers from a bump allocator (sets n_flags); then
// out_layout takes the query's readback block.
void query_layout(uint32_t n_reactions, uint32_t n_flags, Bump& b, QPlan& P);
void out_layout(Bump& b, QPlan& P);
QueryDev make_qdev(const apex_engine* E, const apex_query* q, const QPlan& p, bool relaxed, bool stage2);
std::vector<uint32_t> subset_bits(const apex_engine* E, const apex_query* q);
// Threshold state, subset bits and overflow flags of a fresh query (async).
apex_status query_device_init(const apex_engine* E, const apex_query* q, const QPlan& P, hipStream_t s);
apex_status fill_u32(uint32_t* p, uint32_t n, uint32_t v, hipStream_t s);
// One pass of the fused kernel over tiles [v0, v1) of a tile plan (async).
// work: kWorkCounters counters in device memory, zero before the first pass on
// the stream (each pass leaves them zero); the BF16/FP8 tile kernels share out
// their tiles through them.
constexpr uint32_t kWorkCounters = 9;
apex_status enum_pass(apex_engine* E, int prec, const SelDev* plan_dev, uint32_t n_sel, uint64_t v0, uint64_t v1,
                      const QueryDev* qd_dev, uint32_t nq, uint64_t compounds, uint32_t* work, hipStream_t s);
// Compounds of a host tile plan inside tiles [v0, v1).
uint64_t plan_compounds(const apex_engine* E, int prec, const std::vector<SelDev>& plan, uint64_t v0, uint64_t v1);
// Threshold warm start from a sample of compounds of a tile plan (n_tiles tiles,
// n_comp compounds) for the listed queries (async).
apex_status warm_start(apex_engine* E, int prec, const SelDev* plan_dev, uint32_t n_sel, uint64_t n_tiles,
                       uint64_t n_comp, uint32_t n_sample, uint64_t* ids, float* heads, const QueryDev* qd_dev,
                       uint32_t nq, hipStream_t s);
// Stage 3-4 device work of a query whose enumeration has been enqueued (async):
// FP32 rescoring of a low-precision pool, the ordered answer, its heads and
// decoding, all into the readback block. Every count it needs is read on the
// device, so it is enqueued without a synchronisation; if the host then finds
// an overflow flag set in the block, the chunk re-runs follow and this is
// enqueued again.
apex_status finish_launch(apex_engine* E, const QPlan& P, const QueryDev* qd_dev, const QueryDev* qx_dev,
                          hipStream_t s);
// Overflow flags of the query in a host copy of readback blocks that starts at
// block `base` (the first block of the copy).
const uint32_t* out_flags(const QPlan& P, const char* host, const char* base);
// Fills res (n_found, n_candidates and the requested arrays) from a host copy of
// readback blocks that starts at block `base`.
void finish_read(const apex_engine* E, const QPlan& P, const char* host, const char* base, apex_result* res);
// The same from the device: the counts from the host copy of the query's
// control words, the answer arrays (n_found entries) copied on stream s
// straight into the result arrays (a DMA when they are pinned host memory).
apex_status finish_read_direct(const apex_engine* E, const QPlan& P, const char* host, const char* base,
                               apex_result* res, hipStream_t s);
// Bytes of a query's output block before its answer arrays (states and re-run flags).
inline size_t out_control_bytes(const QPlan& P) { return (size_t)((const char*)P.fin_o - P.out); }

// A pinned host buffer from the engine's pool (ordinary host memory if pinning
// fails), returned to the pool on destruction. With pageable = true it is
// ordinary host memory and nothing is pinned.
class Readback {
 public:
  Readback(apex_engine* E, size_t bytes, bool pageable = false);
  ~Readback();
  Readback(const Readback&) = delete;
  Readback& operator=(const Readback&) = delete;
  char* data() { return p_; }

 private:
  apex_engine* E_;
  char* p_ = nullptr;
  size_t bytes_ = 0;
  bool pinned_ = false;
  std::vector<char> host_;
};
// Resolves the engine's pending kernel timings (after a synchronisation).
apex_status profile_collect(apex_engine* E);

}  // namespace apex
