// Host-side launchers of the HIP kernels (internal).
#pragma once
#include "apex_internal.h"

namespace apex {

hipError_t launch_enum(int prec, int h1, int nl, int act, bool gather, const EnumArgs& a, uint32_t grid,
                       hipStream_t s);
uint32_t gather_per_block(int prec, int nl);  // listed compounds per workgroup of a gather launch
hipError_t enum_prepare(int prec, int h1, int nl, int act, bool gather, uint32_t h2, int* max_wg_per_cu);

hipError_t launch_hoist(const float* U, uint32_t d, uint64_t rows, const float* W1, const float* b1, uint32_t n_w,
                        uint32_t h1, const uint8_t* is_slot0, float c, float* P, hipStream_t s);
hipError_t launch_act_range(const float* P, uint32_t h1, const uint64_t* slot_row0, const uint32_t* slot_size,
                            uint32_t n_slots_total, const uint32_t* react_slot0, const uint32_t* react_nslots,
                            uint32_t n_react, int act, float c, float* cmax, float* cmin, float* out,
                            hipStream_t s);
hipError_t launch_absmax(const float* x, uint64_t n, float* out, hipStream_t s);
hipError_t launch_scales(const float* amax, int prec, int nl, float* scal, hipStream_t s);
hipError_t launch_frag_x(const float* W, uint32_t n_out, uint32_t n_in, uint32_t n_chunks, float mul, void* out,
                         hipStream_t s);
hipError_t launch_frag_x32(int prec, const float* W, uint32_t n_out, uint32_t n_in, uint32_t n_chunks,
                           const float* mul_dev, float mul, void* out, hipStream_t s);
hipError_t launch_frag_out32(const float* Wo, uint32_t H, uint32_t h2, uint32_t h2k, float mul, void* out,
                             hipStream_t s);
hipError_t launch_frag_out_d(const float* Wo, uint32_t H, uint32_t h2, float mul, void* out, hipStream_t s);
hipError_t launch_bias(const float* b2, uint32_t h2, uint32_t h2k, float c, const float* scal, const float* bo,
                       uint32_t H, float* b2_out, float* bo_out, hipStream_t s);
// n_src (optional): score min(n, n_src->count) entries
hipError_t launch_score(const float* heads, const uint64_t* ids, uint32_t n, const QState* n_src, const QueryDev* qs,
                        uint32_t nq, const ReactDev* react, uint32_t n_react, hipStream_t s);
// pool of min(pool_max, pool_src->count) entries, answer of min(want_max, want_src->count)
hipError_t launch_pool_lookup(const uint64_t* pool_id, const float* pool_heads, uint32_t pool_max,
                              const QState* pool_src, const uint64_t* want, uint32_t want_max, const QState* want_src,
                              float* out, hipStream_t s);
hipError_t launch_select(const QueryDev* qs, uint32_t nq, uint32_t chunk_id, int force, hipStream_t s);
hipError_t launch_tau_relax(const QueryDev* qs, uint32_t nq, hipStream_t s);
hipError_t launch_state_reset(QState* st, hipStream_t s);
// Sorts min(count, K) entries of query q by (objective desc, id asc) into out,
// K <= 8192 (longer answers take the radix sort). rank: device scratch of K uint32.
hipError_t launch_rank_sort(const QueryDev* qs, uint32_t q, uint32_t K, float* out_o, uint64_t* out_id,
                            uint32_t* rank, hipStream_t s);
// Sorts min(count, n_max) <= 8192 entries of query q; the first min(that, n_out)
// go out. rank: device scratch of n_max uint32.
hipError_t launch_sort_small(const QueryDev* qs, uint32_t q, uint32_t n_max, uint32_t n_out, float* out_o,
                             uint64_t* out_id, uint32_t* rank, hipStream_t s);
constexpr uint32_t kSortSmallMax = 8192;
hipError_t launch_decode(const ReactDev* react, uint32_t n_react, const uint64_t* ids, const QState* st, uint32_t K,
                         uint32_t* reaction, uint32_t* synthon, hipStream_t s);
// Warm-start sample: groups of 32 compounds (2 x 16 of one tile) from disjoint tile strata.
hipError_t launch_sample_tiles(const SelDev* sel, uint32_t n_sel, const ReactDev* react, uint64_t n_tiles, uint32_t n,
                               uint64_t seed, uint64_t* ids, hipStream_t s);
hipError_t launch_sample_ids(const SelDev* sel, uint32_t n_sel, const ReactDev* react, uint64_t total, uint32_t n,
                             uint64_t seed, uint64_t* ids, hipStream_t s);
hipError_t launch_head_err(const float* h_lp, const float* h_32, uint32_t n, float* out, hipStream_t s);

// Linear-probe path (scalar.hip): per-query row tables, enumeration, scoring of
// listed compounds, FP32 heads of listed compounds (row stride hs).
hipError_t launch_qtab(const float* V, uint32_t hs, uint64_t rows, uint32_t H, const ScalarQuery* sq, hipStream_t s);
hipError_t scan_prepare(int* max_wg_per_cu);
hipError_t launch_scan(const EnumArgs& a, uint32_t grid_max, hipStream_t s);
hipError_t launch_scan_list(const uint64_t* ids, uint32_t n, const QueryDev* qs, uint32_t nq, const ReactDev* react,
                            uint32_t n_react, uint64_t n_total, hipStream_t s);
hipError_t launch_viol_answer(const ScalarQuery* sq, const ReactDev* react, uint32_t n_react, const uint64_t* ids,
                              const QState* st, uint32_t K, float* obj, float* viol, hipStream_t s);
hipError_t launch_head_quantiles(const float* heads, uint32_t hs, uint32_t n, const float* levels, uint32_t n_levels,
                                 uint32_t H, float* out, hipStream_t s);
hipError_t launch_assoc(const AssocSlot* slots, uint32_t n_slots, uint64_t n_tiles, uint32_t d, uint32_t dU,
                        const float* keys, const float* values, float* out, int n_cu, hipStream_t s);
hipError_t launch_lin_heads(const float* V, uint32_t hs, const ReactDev* react, uint32_t n_react, uint64_t n_total,
                            const uint64_t* ids, uint32_t n, float* heads, uint32_t ho, hipStream_t s);

// Radix sort (radix_sort.hip) of min(st->count, n_max) entries (src_o, src_id) by
// (objective desc, id asc); the first min(that, n_out) go to (out_o, out_id).
// a_*/b_*: two scratch pairs of n_max entries, distinct from the source and the
// output; hist: radix_hist_words(n_max) uint32; id_bytes: bytes of the largest id.
uint32_t radix_blocks(uint32_t n_max);
inline size_t radix_hist_words(uint32_t n_max) { return (size_t)256 * radix_blocks(n_max) + 256; }
hipError_t launch_radix_sort(const QState* st, uint32_t n_max, const float* src_o, const uint64_t* src_id,
                             uint32_t* a_k, uint64_t* a_id, uint32_t* b_k, uint64_t* b_id, float* out_o,
                             uint64_t* out_id, uint32_t n_out, uint32_t id_bytes, uint32_t* hist, hipStream_t s);

}  // namespace apex
