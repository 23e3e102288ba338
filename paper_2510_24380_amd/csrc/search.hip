// Search driver: one query or several fused queries over the library.
//
// Pipeline per call (all device work on the caller's stream):
//  1. threshold warm start: a stratified sample of compounds is scored and each
//     query's threshold set just below its K-th best sampled key (a valid lower
//     bound of the final K-th key); the sample entries are then dropped;
//  2. chunked enumeration: the fused kernel appends compounds whose key beats
//     the threshold; after each chunk the select kernel compacts the buffer to
//     the K best and raises the threshold (the chain-of-batches merge of
//     Appendix A.5, without materialising any score array); a chunk whose
//     appends overflow the buffer is dropped and re-run once the threshold is
//     higher;
//  3. FP32 precision: the K = k survivors are the answer. BF16/FP8: the K =
//     pool_factor * k survivors (enumerated with bounds relaxed by a per-head
//     margin) are rescored in FP32 with the exact bounds and the best k kept;
//  4. rank sort by (objective desc, id asc), FP32 heads of the answer, decode of
//     ids to (reaction, synthons) on the GPU (Appendix A.5), copy to the host.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <vector>

#include "launch.h"
#include "search_impl.h"

using namespace apex;

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return set_error(APEX_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

namespace apex {

// Rank in a sample of n_sample compounds (of n_comp) whose key is taken as the
// warm-start threshold of a query keeping K: the expected number m of the final
// K best in the sample plus four standard deviations and 8, at most K.
// APEX_TEST_SPEC_RANK forces the rank (tests of the verification).
uint32_t spec_rank(uint32_t K, uint32_t n_sample, uint64_t n_comp) {
  const uint64_t forced = env_u64("APEX_TEST_SPEC_RANK");
  if (forced) return (uint32_t)std::min<uint64_t>(forced, K);
  const double m = (double)K * (double)n_sample / (double)std::max<uint64_t>(n_comp, 1);
  const double r = std::ceil(m + 4.0 * std::sqrt(m) + 8.0);
  return r >= (double)K ? K : (uint32_t)r;
}

// Warm-start sample of the linear path: scoring a sampled compound costs about
// as much as a few hundred enumerated ones, so the sample grows with the library
// (1/64 of it, 2^16 .. 2^22 compounds, at least 64 K, at most an eighth of the
// library): each sampled compound
// then stands for fewer library compounds and the threshold starts closer to
// the final K-th key.
uint64_t scalar_sample(uint32_t K, uint64_t total) {
  uint64_t s = std::max<uint64_t>(std::max<uint64_t>(64ull * K, total / 64), 1ull << 16);
  s = std::min<uint64_t>(s, 1ull << 22);
  // at most an eighth of the library (the warm start's condition), not below 2^16
  return std::max<uint64_t>(std::min<uint64_t>(s, total / 8), 1ull << 16);
}

// compounds in the first chunk: small, so that the appends before the first
// select stay few even with the warm start's loose threshold
constexpr uint64_t kFirstChunk = 1ull << 20;
// answer arrays longer than this are copied from the device straight into the
// result arrays instead of through the readback of the whole output block
constexpr size_t kDirectReadback = 4u << 20;
constexpr uint64_t kMaxChunk = 1ull << 27;
// the scalar-contribution kernel spends ~1e-12 s per compound: its chunks may
// grow further before a launch and a select per chunk cost more than the chunk
constexpr uint64_t kMaxChunkScalar = 1ull << 31;

// Test knobs, read from the environment at every search: APEX_TEST_CHUNK fixes
// the chunk size (compounds) and APEX_TEST_CAP the candidate-buffer capacity
// (entries, at least 2K), so tests can force many chunks and buffer overflows.
uint64_t env_u64(const char* name) {
  const char* v = getenv(name);
  return v ? strtoull(v, nullptr, 10) : 0;
}

std::vector<std::pair<uint64_t, uint64_t>> chunk_schedule(uint64_t n_tiles, uint64_t tile_compounds, bool scalar) {
  std::vector<std::pair<uint64_t, uint64_t>> out;
  const uint64_t forced = env_u64("APEX_TEST_CHUNK");
  uint64_t per = std::max<uint64_t>(1, (forced ? forced : kFirstChunk) / tile_compounds);
  const uint64_t max_chunk = scalar ? kMaxChunkScalar : kMaxChunk;
  const uint64_t max_per = forced ? per : std::max<uint64_t>(1, max_chunk / tile_compounds);
  for (uint64_t v = 0; v < n_tiles;) {
    const uint64_t e = std::min(n_tiles, v + per);
    out.emplace_back(v, e);
    v = e;
    per = std::min(max_per, per * 2);
  }
  return out;
}

uint32_t tile_compounds(bool scalar) { return (uint32_t)(tile_ta(scalar) * tile_tb(scalar)); }

apex_status validate_query(const apex_engine* E, const apex_query* q) {
  if (!q) return set_error(APEX_E_INVALID, "null query");
  if (!q->objective_w) return set_error(APEX_E_INVALID, "null objective_w");
  if (q->k == 0) return set_error(APEX_E_INVALID, "k must be >= 1");
  if (q->k > (1u << 26)) return set_error(APEX_E_UNSUPPORTED, "k = %llu > 2^26", (unsigned long long)q->k);
  if (q->precision > APEX_PREC_FP8) return set_error(APEX_E_INVALID, "unknown precision %u", q->precision);
  if (q->precision != APEX_PREC_FP32 && !((E->user_mask >> q->precision) & 1u))
    return set_error(APEX_E_INVALID, "precision %u not enabled in this engine", q->precision);
  if (q->n_constraints > APEX_MAX_CONSTRAINTS)
    return set_error(APEX_E_INVALID, "%u constraints > %d", q->n_constraints, APEX_MAX_CONSTRAINTS);
  if (q->n_constraints && !q->constraints) return set_error(APEX_E_INVALID, "null constraints");
  for (uint32_t h = 0; h < E->H; ++h)
    if (!std::isfinite(q->objective_w[h])) return set_error(APEX_E_INVALID, "objective weight %u not finite", h);
  for (uint32_t c = 0; c < q->n_constraints; ++c) {
    const apex_constraint& k = q->constraints[c];
    if (k.head >= E->H) return set_error(APEX_E_INVALID, "constraint %u: head %u >= H = %u", c, k.head, E->H);
    if (std::isnan(k.lo) || std::isnan(k.hi)) return set_error(APEX_E_INVALID, "constraint %u: NaN bound", c);
    if (k.lo > k.hi) return set_error(APEX_E_INVALID, "constraint %u: lo > hi", c);
  }
  if (q->flags & ~APEX_QUERY_KEEP_VIOLATORS) return set_error(APEX_E_INVALID, "unknown query flags 0x%x", q->flags);
  if ((q->flags & APEX_QUERY_KEEP_VIOLATORS) && !E->scalar)
    return set_error(APEX_E_UNSUPPORTED, "the violation-ranked fallback needs a one-layer (linear-probe) engine");
  if (q->n_subset) {
    if (!q->subset) return set_error(APEX_E_INVALID, "null subset");
    std::vector<uint8_t> seen(E->lib->T, 0);
    for (uint32_t i = 0; i < q->n_subset; ++i) {
      if (q->subset[i] >= E->lib->T) return set_error(APEX_E_INVALID, "subset reaction %u out of range", q->subset[i]);
      if (seen[q->subset[i]]) return set_error(APEX_E_INVALID, "subset reaction %u repeated", q->subset[i]);
      seen[q->subset[i]] = 1;
    }
  }
  const uint32_t pf = q->pool_factor ? q->pool_factor : 4;
  if (q->precision != APEX_PREC_FP32 && (uint64_t)pf * q->k > (1u << 28))
    return set_error(APEX_E_UNSUPPORTED, "pool_factor * k too large");
  return APEX_OK;
}

// Distinct constrained heads of a query, with their intersected bounds.
static uint32_t constrained_heads(const apex_query* q, uint32_t* head, float* lo, float* hi) {
  uint32_t n = 0;
  for (uint32_t c = 0; c < q->n_constraints; ++c) {
    const apex_constraint& k = q->constraints[c];
    uint32_t j = 0;
    while (j < n && head[j] != k.head) ++j;
    if (j == n) {
      head[n] = k.head;
      lo[n] = -INFINITY;
      hi[n] = INFINITY;
      ++n;
    }
    lo[j] = std::max(lo[j], k.lo);
    hi[j] = std::min(hi[j], k.hi);
  }
  return n;
}

void query_sizes(const apex_engine* E, const apex_query* q, QPlan& P) {
  P.k = (uint32_t)q->k;
  P.lowp = q->precision != APEX_PREC_FP32;
  P.hs = E->scalar ? E->H : E->HS;  // linear-probe answers carry exactly H heads per row
  P.keep = (q->flags & APEX_QUERY_KEEP_VIOLATORS) != 0;
  if (E->scalar) {
    uint32_t head[APEX_MAX_CONSTRAINTS];
    float lo[APEX_MAX_CONSTRAINTS], hi[APEX_MAX_CONSTRAINTS];
    P.n_cols = 1 + constrained_heads(q, head, lo, hi);
    if (P.keep) P.n_cols = 1 + q->n_constraints;  // the violation pass's columns (one per constraint)
    P.tab_rows = E->lib->rows;
  }
  const uint32_t pf = q->pool_factor ? q->pool_factor : 4;
  P.K = P.lowp ? pf * P.k : P.k;
  uint64_t cap = std::min<uint64_t>(std::max<uint64_t>(64ull * P.K, 1ull << 18), 1ull << 22);
  cap = std::max<uint64_t>(cap, 2ull * P.K);
  if (E->scalar) cap = std::max<uint64_t>(cap, scalar_sample(P.K, E->lib->total));
  const uint64_t forced = env_u64("APEX_TEST_CAP");
  if (forced) cap = std::max<uint64_t>(forced, 2ull * P.K);
  P.cap = (uint32_t)cap;
  // select as soon as 8 K candidates (at least 2^15) have gathered: selects of
  // small buffers are cheap, and each one tightens the threshold for the rest
  P.hwm = (uint32_t)std::min<uint64_t>(P.cap / 2, std::max<uint64_t>(8ull * P.K, 1ull << 15));
  P.cap2 = P.K;
}

void query_layout(uint32_t T, uint32_t n_flags, Bump& b, QPlan& p) {
  p.n_flags = n_flags;
  p.cand_o = b.take<float>(p.cap);
  p.cand_id = b.take<uint64_t>(p.cap);
  p.tmp_o = b.take<float>(p.K);
  p.tmp_id = b.take<uint64_t>(p.K);
  p.subset_dev = b.take<uint32_t>((T + 31) / 32);
  p.sel = b.take<SelScratch>(1);
  if (p.n_cols) {
    p.sq = b.take<ScalarQuery>(1);
    p.tab = b.take<float>((size_t)p.n_cols * p.tab_rows);
  }
  // answers longer than one workgroup's sort are radix-sorted (the FP32 answer,
  // or the whole rescored pool of a low-precision search)
  const uint32_t sort_n = p.lowp ? p.cap2 : p.K;
  if (sort_n > kSortSmallMax) p.rs_hist = b.take<uint32_t>(radix_hist_words(sort_n));
  if (p.lowp) {
    p.pool_heads = b.take<float>((size_t)p.K * kHeadsPad);
    p.cand2_o = b.take<float>(p.cap2);
    p.cand2_id = b.take<uint64_t>(p.cap2);
    p.tmp2_o = b.take<float>(p.k);
    p.tmp2_id = b.take<uint64_t>(p.k);
  }
}

void out_layout(Bump& b, QPlan& p) {
  const size_t off0 = b.off;
  p.out = b.base ? b.base + off0 : nullptr;
  p.st = b.take<QState>(1);
  if (p.lowp) p.st2 = b.take<QState>(1);
  p.rerun = b.take<uint32_t>(p.n_flags);
  p.fin_o = b.take<float>(p.k);
  p.fin_id = b.take<uint64_t>(p.k);
  p.fin_heads = b.take<float>((size_t)p.k * p.hs);
  p.fin_reaction = b.take<uint32_t>(p.k);
  p.fin_synthon = b.take<uint32_t>((size_t)p.k * 3);
  if (p.keep) p.fin_c = b.take<float>(p.k);
  p.out_bytes = b.off - off0;
}

Readback::Readback(apex_engine* E, size_t bytes, bool pageable) : E_(E), bytes_(bytes) {
  if (pageable) {
    host_.resize(bytes);
    p_ = host_.data();
    return;
  }
  {
    std::lock_guard<std::mutex> lk(E->pin_mu);
    for (size_t i = 0; i < E->pin_free.size(); ++i)
      if (E->pin_free[i].second >= bytes) {
        p_ = (char*)E->pin_free[i].first;
        bytes_ = E->pin_free[i].second;
        E->pin_free.erase(E->pin_free.begin() + (long)i);
        pinned_ = true;
        return;
      }
  }
  const size_t want = std::max<size_t>(bytes, 1 << 20);
  void* p = nullptr;
  if (hipHostMalloc(&p, want, hipHostMallocDefault) == hipSuccess) {
    p_ = (char*)p;
    bytes_ = want;
    pinned_ = true;
  } else {
    (void)hipGetLastError();
    host_.resize(bytes);
    p_ = host_.data();
  }
}

Readback::~Readback() {
  if (!pinned_) return;
  std::lock_guard<std::mutex> lk(E_->pin_mu);
  E_->pin_free.emplace_back(p_, bytes_);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t n, uint32_t v) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

apex_status fill_u32(uint32_t* p, uint32_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return APEX_OK;
  hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  HIP_TRY(hipGetLastError());
  return APEX_OK;
}

QueryDev make_qdev(const apex_engine* E, const apex_query* q, const QPlan& p, bool relaxed, bool stage2) {
  QueryDev d{};
  for (int h = 0; h < kHeadsPad; ++h) {
    d.w[h] = h < (int)E->H ? q->objective_w[h] : 0.0f;
    d.lo[h] = -INFINITY;
    d.hi[h] = INFINITY;
  }
  // per-head bounds of the MLP kernels (at most 16 heads there; linear-probe
  // engines read their bounds from the query's ScalarQuery instead)
  for (uint32_t c = 0; c < q->n_constraints; ++c) {
    const apex_constraint& k = q->constraints[c];
    if (k.head >= (uint32_t)kHeadsPad) continue;
    d.lo[k.head] = std::max(d.lo[k.head], k.lo);
    d.hi[k.head] = std::min(d.hi[k.head], k.hi);
  }
  d.sq = p.sq;
  if (relaxed && p.lowp) {
    const float* dl = E->prec[q->precision].delta;
    for (int h = 0; h < kHeadsPad; ++h) {
      d.lo[h] -= dl[h];
      d.hi[h] += dl[h];
    }
  }
  if (!stage2) {
    d.st = p.st;
    d.cand_o = p.cand_o;
    d.cand_id = p.cand_id;
    d.tmp_o = p.tmp_o;
    d.tmp_id = p.tmp_id;
    d.rerun = p.rerun;
    d.cap = p.cap;
    d.K = p.K;
    d.hwm = p.hwm;
  } else {
    d.st = p.st2;
    d.cand_o = p.cand2_o;
    d.cand_id = p.cand2_id;
    d.tmp_o = p.tmp2_o;
    d.tmp_id = p.tmp2_id;
    d.rerun = p.rerun;  // never flagged: the rescoring buffer holds the whole pool
    d.cap = p.cap2;
    d.K = p.k;
    d.hwm = p.cap2;
  }
  d.subset_bits = q->n_subset ? p.subset_dev : nullptr;
  d.sel = p.sel;
  d.active = 1;
  return d;
}

std::vector<uint32_t> subset_bits(const apex_engine* E, const apex_query* q) {
  std::vector<uint32_t> bits;
  if (q->n_subset) {
    bits.assign((E->lib->T + 31) / 32, 0u);
    for (uint32_t j = 0; j < q->n_subset; ++j) bits[q->subset[j] >> 5] |= 1u << (q->subset[j] & 31);
  }
  return bits;
}

apex_status query_device_init(const apex_engine* E, const apex_query* q, const QPlan& P, hipStream_t s) {
  HIP_TRY(launch_state_reset(P.st, s));  // st2: reset by finish_launch
  const std::vector<uint32_t> bits = subset_bits(E, q);
  if (!bits.empty())
    HIP_TRY(hipMemcpyAsync(P.subset_dev, bits.data(), bits.size() * 4, hipMemcpyHostToDevice, s));
  if (P.sq) {
    // linear-probe engine: the query's per-row tables (Section 4.3: each
    // synthon's contribution to the objective, dotted once per query)
    ScalarQuery sq{};
    for (uint32_t h = 0; h < E->H; ++h) sq.w[h] = q->objective_w[h];
    if (P.viol) {
      sq.viol = 1;
      sq.n_ch = q->n_constraints;
      for (uint32_t c = 0; c < q->n_constraints; ++c) {
        sq.head[c] = q->constraints[c].head;
        sq.lo[c] = q->constraints[c].lo;
        sq.hi[c] = q->constraints[c].hi;
      }
    } else {
      sq.n_ch = constrained_heads(q, sq.head, sq.lo, sq.hi);
    }
    sq.tab = P.tab;
    sq.rows = P.tab_rows;
    HIP_TRY(hipMemcpyAsync(P.sq, &sq, sizeof(sq), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_qtab(E->P, E->HS, P.tab_rows, E->H, P.sq, s));
  }
  return fill_u32(P.rerun, P.n_flags, 0u, s);
}

uint64_t plan_compounds(const apex_engine* E, int prec, const std::vector<SelDev>& plan, uint64_t v0, uint64_t v1) {
  uint64_t c = 0;
  const uint64_t TA = tile_ta(E->scalar), TB = tile_tb(E->scalar);
  for (size_t r = 0; r < plan.size(); ++r) {
    const ReactDev& rd = E->react_host[plan[r].t];
    const uint64_t ta = (rd.nA + TA - 1) / TA;
    const uint64_t t0 = plan[r].tile_start, t1 = t0 + ta * plan[r].tiles_b;
    if (t1 <= v0 || t0 >= v1) continue;
    if (t0 >= v0 && t1 <= v1) {
      c += (uint64_t)rd.nA * rd.nB;
      continue;
    }
    // partially covered reaction: count tile by tile, ragged edges included
    for (uint64_t v = std::max(v0, t0); v < std::min(v1, t1); ++v) {
      const uint64_t lt = v - t0;
      const uint64_t ia = lt / plan[r].tiles_b, ib = lt % plan[r].tiles_b;
      c += std::min<uint64_t>(TA, rd.nA - ia * TA) * std::min<uint64_t>(TB, rd.nB - ib * TB);
    }
  }
  return c;
}

apex_status enum_pass(apex_engine* E, int prec, const SelDev* plan_dev, uint32_t n_sel, uint64_t v0, uint64_t v1,
                      const QueryDev* qd_dev, uint32_t nq, uint64_t compounds, uint32_t* work, hipStream_t s) {
  // the tile kernels keep every fused query's parameters in LDS
  if (nq == 0 || nq > APEX_MAX_FUSED_QUERIES) return set_error(APEX_E_INVALID, "internal: %u fused queries", nq);
  const PrecState& PS = E->prec[prec];
  EnumArgs a{};
  a.P = E->P;
  a.react = E->react;
  a.sel = plan_dev;
  a.n_sel = n_sel;
  a.pd = PS.dev;
  a.H2 = E->prec[prec].h2k;
  a.n_queries = nq;
  a.queries = qd_dev;
  a.n_reactions = E->lib->T;
  a.n_total = E->lib->total;
  a.tile_begin = v0;
  a.tile_end = v1;
  a.work = work;
  uint32_t grid_full = (uint32_t)(E->n_cu * PS.wg_per_cu);
  grid_full = std::max<uint32_t>(8, grid_full / 8 * 8);
  const uint64_t nt = v1 - v0;
  const uint32_t grid = nt < grid_full ? (uint32_t)nt : grid_full;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (E->profile) {
    for (hipEvent_t* e : {&e0, &e1}) {
      if (!E->ev_free.empty()) {
        *e = E->ev_free.back();
        E->ev_free.pop_back();
      } else {
        HIP_TRY(hipEventCreate(e));
      }
    }
    HIP_TRY(hipEventRecord(e0, s));
  }
  if (E->scalar)
    HIP_TRY(launch_scan(a, (uint32_t)std::max(1, E->n_cu * PS.wg_per_cu), s));
  else
    HIP_TRY(launch_enum(prec, E->H1, E->NL, E->act, false, a, grid, s));
  if (E->profile) {
    HIP_TRY(hipEventRecord(e1, s));
    E->ev_pending.push_back({e0, e1, compounds});
  }
  return APEX_OK;
}

apex_status profile_collect(apex_engine* E) {
  for (auto& t : E->ev_pending) {
    float ms = 0.0f;
    HIP_TRY(hipEventSynchronize(t.b));
    HIP_TRY(hipEventElapsedTime(&ms, t.a, t.b));
    E->prof_ms += ms;
    E->prof_launches += 1;
    E->prof_compounds += t.compounds;
    E->ev_free.push_back(t.a);
    E->ev_free.push_back(t.b);
  }
  E->ev_pending.clear();
  return APEX_OK;
}

apex_status warm_start(apex_engine* E, int prec, const SelDev* plan_dev, uint32_t n_sel, uint64_t n_tiles,
                       uint64_t n_comp, uint32_t n_sample, uint64_t* ids, float* heads, const QueryDev* qd_dev,
                       uint32_t nq, hipStream_t s) {
  if (E->scalar) {
    // distinct sampled compounds scored with the enumeration's own arithmetic
    HIP_TRY(launch_sample_ids(plan_dev, n_sel, E->react, n_comp, n_sample, 0xa5e7c0de1234ull, ids, s));
    HIP_TRY(launch_scan_list(ids, n_sample, qd_dev, nq, E->react, E->lib->T, E->lib->total, s));
  } else {
    HIP_TRY(launch_sample_tiles(plan_dev, n_sel, E->react, n_tiles, n_sample, 0xa5e7c0de1234ull, ids, s));
    apex_status st = engine_gather(E, prec, ids, n_sample, heads, s);
    if (st != APEX_OK) return st;
    HIP_TRY(launch_score(heads, ids, n_sample, nullptr, qd_dev, nq, E->react, E->lib->T, s));
  }
  HIP_TRY(launch_select(qd_dev, nq, 0, 1, s));
  HIP_TRY(launch_tau_relax(qd_dev, nq, s));
  return APEX_OK;
}

// The selection scratch's bracket keys (free once the selections are done)
// hold the ranks of the answer sort.
static uint32_t* rank_scratch(const QPlan& P) {
  return reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(P.sel) + offsetof(SelScratch, br_key));
}

// Bytes of the largest compound id (the id digits of the radix sort).
static uint32_t id_bytes(const apex_engine* E) {
  uint64_t m = E->lib->total ? E->lib->total - 1 : 0;
  uint32_t n = 1;
  while (m >>= 8) ++n;
  return n;
}

apex_status finish_launch(apex_engine* E, const QPlan& P, const QueryDev* qd_dev, const QueryDev* qx_dev,
                          hipStream_t s) {
  if (!P.lowp) {
    if (P.K > kSortSmallMax) {
      // scratch: the compaction buffer and the candidate buffer past its first
      // K entries (the K survivors stay intact for a re-run after an overflow)
      HIP_TRY(launch_radix_sort(P.st, P.K, P.cand_o, P.cand_id, reinterpret_cast<uint32_t*>(P.tmp_o), P.tmp_id,
                                reinterpret_cast<uint32_t*>(P.cand_o + P.K), P.cand_id + P.K, P.fin_o, P.fin_id, P.k,
                                id_bytes(E), P.rs_hist, s));
    } else {
      HIP_TRY(launch_rank_sort(qd_dev, 0, P.K, P.fin_o, P.fin_id, rank_scratch(P), s));
    }
    if (P.viol)  // the sorted keys are violations: move them, recompute the objectives
      HIP_TRY(launch_viol_answer(P.sq, E->react, E->lib->T, P.fin_id, P.st, P.K, P.fin_o, P.fin_c, s));
    // rows past the answer's length are computed from stale ids and never read
    apex_status st = engine_gather(E, APEX_PREC_FP32, P.fin_id, P.k, P.fin_heads, s, P.hs);
    if (st != APEX_OK) return st;
  } else {
    // the pool is the first min(count, K) entries; the scoring ignores the rest
    HIP_TRY(launch_state_reset(P.st2, s));  // this may be a second pass after re-runs
    apex_status st = engine_gather(E, APEX_PREC_FP32, P.cand_id, P.K, P.pool_heads, s);
    if (st != APEX_OK) return st;
    HIP_TRY(launch_score(P.pool_heads, P.cand_id, P.K, P.st, qx_dev, 1, E->react, E->lib->T, s));
    if (P.cap2 <= kSortSmallMax) {
      // the rescored pool fits one workgroup: sort all of it, keep the first k
      HIP_TRY(launch_sort_small(qx_dev, 0, P.cap2, P.k, P.fin_o, P.fin_id, rank_scratch(P), s));
    } else {
      // the whole rescored pool, radix-sorted; the first k are the answer
      HIP_TRY(launch_radix_sort(P.st2, P.cap2, P.cand2_o, P.cand2_id, reinterpret_cast<uint32_t*>(P.tmp_o),
                                P.tmp_id, reinterpret_cast<uint32_t*>(P.cand_o + P.K), P.cand_id + P.K, P.fin_o,
                                P.fin_id, P.k, id_bytes(E), P.rs_hist, s));
    }
    // the answer is part of the rescored pool
    HIP_TRY(launch_pool_lookup(P.cand_id, P.pool_heads, P.K, P.st, P.fin_id, P.k, P.st2, P.fin_heads, s));
  }
  HIP_TRY(launch_decode(E->react, E->lib->T, P.fin_id, P.lowp ? P.st2 : P.st, P.k, P.fin_reaction, P.fin_synthon,
                        s));
  return APEX_OK;
}

namespace {
template <class T>
const T* in_copy(const char* host, const char* base, const T* dev) {
  return reinterpret_cast<const T*>(host + ((const char*)dev - base));
}
}  // namespace

const uint32_t* out_flags(const QPlan& P, const char* host, const char* base) {
  return in_copy(host, base, P.rerun);
}

void finish_read(const apex_engine* E, const QPlan& P, const char* host, const char* base, apex_result* res) {
  const QState st1 = *in_copy(host, base, P.st);
  const uint32_t n1 = std::min(st1.count, P.K);
  const uint32_t n_found = P.lowp ? std::min(in_copy(host, base, P.st2)->count, P.k) : n1;
  res->n_found = n_found;
  res->n_candidates = st1.appended;
  if (n_found == 0) return;
  std::memcpy(res->ids, in_copy(host, base, P.fin_id), sizeof(uint64_t) * n_found);
  std::memcpy(res->objective, in_copy(host, base, P.fin_o), sizeof(float) * n_found);
  if (res->heads) {
    const float* h = in_copy(host, base, P.fin_heads);
    if (P.hs == E->H) {
      std::memcpy(res->heads, h, sizeof(float) * E->H * n_found);
    } else {
      for (uint32_t e = 0; e < n_found; ++e)
        std::memcpy(res->heads + (size_t)e * E->H, h + (size_t)e * P.hs, sizeof(float) * E->H);
    }
  }
  if (res->reaction) std::memcpy(res->reaction, in_copy(host, base, P.fin_reaction), sizeof(uint32_t) * n_found);
  if (res->violation && P.keep) {
    if (P.viol)
      std::memcpy(res->violation, in_copy(host, base, P.fin_c), sizeof(float) * n_found);
    else
      std::fill(res->violation, res->violation + n_found, 0.0f);
  }
  if (res->synthon) std::memcpy(res->synthon, in_copy(host, base, P.fin_synthon), sizeof(uint32_t) * 3 * n_found);
}

apex_status finish_read_direct(const apex_engine* E, const QPlan& P, const char* host, const char* base,
                               apex_result* res, hipStream_t s) {
  const QState st1 = *in_copy(host, base, P.st);
  const uint32_t n1 = std::min(st1.count, P.K);
  const uint32_t n_found = P.lowp ? std::min(in_copy(host, base, P.st2)->count, P.k) : n1;
  res->n_found = n_found;
  res->n_candidates = st1.appended;
  if (n_found == 0) return APEX_OK;
  const auto d2h = hipMemcpyDeviceToHost;
  HIP_TRY(hipMemcpyAsync(res->ids, P.fin_id, sizeof(uint64_t) * n_found, d2h, s));
  HIP_TRY(hipMemcpyAsync(res->objective, P.fin_o, sizeof(float) * n_found, d2h, s));
  if (res->heads) {
    if (P.hs == E->H)
      HIP_TRY(hipMemcpyAsync(res->heads, P.fin_heads, sizeof(float) * E->H * n_found, d2h, s));
    else
      HIP_TRY(hipMemcpy2DAsync(res->heads, sizeof(float) * E->H, P.fin_heads, sizeof(float) * P.hs,
                               sizeof(float) * E->H, n_found, d2h, s));
  }
  if (res->reaction) HIP_TRY(hipMemcpyAsync(res->reaction, P.fin_reaction, sizeof(uint32_t) * n_found, d2h, s));
  if (res->violation && P.keep) {
    if (P.viol)
      HIP_TRY(hipMemcpyAsync(res->violation, P.fin_c, sizeof(float) * n_found, d2h, s));
    else
      std::fill(res->violation, res->violation + n_found, 0.0f);
  }
  if (res->synthon) HIP_TRY(hipMemcpyAsync(res->synthon, P.fin_synthon, sizeof(uint32_t) * 3 * n_found, d2h, s));
  return APEX_OK;
}

}  // namespace apex

namespace {

struct Shared {
  QueryDev* qd = nullptr;   // enumeration-pass queries (relaxed bounds in low precision)
  QueryDev* qx = nullptr;   // exact-bound queries of the rescoring pass
  SelDev* plan = nullptr;
  uint64_t* sample_ids = nullptr;
  float* sample_heads = nullptr;
  uint32_t n_sample = 0;
  uint32_t n_flags = 0;
  uint32_t* work = nullptr;  // tile-sharing counters of the fused passes
};

uint32_t sample_count(const apex_engine* E, const std::vector<QPlan>& P) {
  uint32_t kmax = 0, capmin = UINT32_MAX;
  for (auto& p : P) {
    kmax = std::max(kmax, p.K);
    capmin = std::min(capmin, p.cap);
  }
  uint64_t s = E->scalar ? scalar_sample(kmax, E->lib->total)
                         : std::min<uint64_t>(std::max<uint64_t>(32ull * kmax, 1ull << 16), 1ull << 20);
  return (uint32_t)std::min<uint64_t>(s, capmin);
}

void batch_layout(const apex_engine* E, const apex_query* qs, uint32_t n, Bump& b, std::vector<QPlan>& P,
                  Shared& sh, bool viol = false) {
  P.assign(n, QPlan());
  for (uint32_t i = 0; i < n; ++i) {
    query_sizes(E, &qs[i], P[i]);
    P[i].viol = viol;
  }
  const int prec = (int)qs[0].precision;
  sh.n_flags = (uint32_t)chunk_schedule(E->prec[prec].full_tiles, tile_compounds(E->scalar), E->scalar).size() + 1;
  sh.n_sample = sample_count(E, P);
  const uint32_t T = E->lib->T;
  sh.qd = b.take<QueryDev>(n);
  sh.qx = b.take<QueryDev>(n);
  sh.plan = b.take<SelDev>(T);
  sh.sample_ids = b.take<uint64_t>(sh.n_sample);
  // the linear path scores its sample from the query tables, without heads
  sh.sample_heads = b.take<float>(E->scalar ? 1 : (size_t)sh.n_sample * kHeadsPad);
  sh.work = b.take<uint32_t>(kWorkCounters);
  for (uint32_t i = 0; i < n; ++i) query_layout(T, sh.n_flags, b, P[i]);
  for (uint32_t i = 0; i < n; ++i) out_layout(b, P[i]);  // adjacent readback blocks
}

}  // namespace

static apex_status run_search(apex_engine* E, const apex_query* qs, uint32_t nq, void* ws, size_t ws_bytes,
                              hipStream_t s, apex_result* res, bool pageable_readback = false, bool viol = false) {
  if (!E || !qs || !res || nq == 0) return set_error(APEX_E_INVALID, "null argument");
  if (nq > APEX_MAX_FUSED_QUERIES) return set_error(APEX_E_INVALID, "%u queries > %d", nq, APEX_MAX_FUSED_QUERIES);
  for (uint32_t i = 0; i < nq; ++i) {
    apex_status st = validate_query(E, &qs[i]);
    if (st != APEX_OK) return st;
    if (qs[i].precision != qs[0].precision)
      return set_error(APEX_E_INVALID, "fused queries must share one precision");
    if (nq > 1 && (qs[i].flags & APEX_QUERY_KEEP_VIOLATORS))
      return set_error(APEX_E_UNSUPPORTED, "the violation-ranked fallback runs one query at a time");
    if (res[i].capacity < qs[i].k || !res[i].ids || !res[i].objective)
      return set_error(APEX_E_INVALID, "result %u: capacity < k or null ids/objective", i);
  }
  if (!ws) return set_error(APEX_E_INVALID, "null workspace");
  if (((uintptr_t)ws) & 255) return set_error(APEX_E_INVALID, "workspace must be 256-byte aligned");
  const int prec = (int)qs[0].precision;
  const apex_library* L = E->lib;

  std::vector<QPlan> P;
  Shared sh;
  {
    Bump b(nullptr);
    batch_layout(E, qs, nq, b, P, sh, viol);
    if (b.off > ws_bytes)
      return set_error(APEX_E_NOMEM, "query workspace %zu bytes < %zu needed", ws_bytes, b.off);
  }
  Bump b(ws);
  batch_layout(E, qs, nq, b, P, sh, viol);

  // reactions searched by at least one query
  std::vector<uint8_t> want(L->T, 0);
  for (uint32_t i = 0; i < nq; ++i) {
    if (qs[i].n_subset == 0) std::fill(want.begin(), want.end(), 1);
    for (uint32_t j = 0; j < qs[i].n_subset; ++j) want[qs[i].subset[j]] = 1;
  }
  std::vector<uint32_t> reactions;
  for (uint32_t t = 0; t < L->T; ++t)
    if (want[t]) reactions.push_back(t);
  std::vector<SelDev> plan;
  uint64_t n_tiles = 0, n_comp = 0;
  build_plan(L, E->scalar, reactions, plan, &n_tiles, &n_comp);

  std::vector<QueryDev> qd(nq), qx(nq);
  for (uint32_t i = 0; i < nq; ++i) {
    apex_status st = query_device_init(E, &qs[i], P[i], s);
    if (st != APEX_OK) return st;
    qd[i] = make_qdev(E, &qs[i], P[i], true, false);
    qx[i] = make_qdev(E, &qs[i], P[i], false, P[i].lowp);
  }
  HIP_TRY(hipMemcpyAsync(sh.qd, qd.data(), sizeof(QueryDev) * nq, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(sh.qx, qx.data(), sizeof(QueryDev) * nq, hipMemcpyHostToDevice, s));
  {
    const apex_status st = fill_u32(sh.work, kWorkCounters, 0u, s);  // the passes leave them zero
    if (st != APEX_OK) return st;
  }
  if (!plan.empty())
    HIP_TRY(hipMemcpyAsync(sh.plan, plan.data(), sizeof(SelDev) * plan.size(), hipMemcpyHostToDevice, s));

  uint64_t scored = 0;
  // 1. threshold warm start from a stratified sample of the searched reactions:
  // each query's threshold is the key of rank r of the sample. r = K is a
  // guaranteed lower bound of the final K-th key; when the sample is much
  // smaller than the library, r is taken from the expected number of the final
  // K best in the sample plus a margin, which is speculative: a query left with
  // fewer than K survivors is enumerated again without the threshold (below).
  std::vector<uint8_t> spec(nq, 0);
  std::vector<QueryDev> qw(qd);
  if (n_comp >= 8ull * sh.n_sample) {
    bool any_spec = false;
    for (uint32_t i = 0; i < nq; ++i) {
      const uint32_t r = spec_rank(P[i].K, sh.n_sample, n_comp);
      if (r < P[i].K) {
        qw[i].K = r;
        spec[i] = 1;
        any_spec = true;
      }
    }
    if (any_spec) HIP_TRY(hipMemcpyAsync(sh.qd, qw.data(), sizeof(QueryDev) * nq, hipMemcpyHostToDevice, s));
    apex_status st = warm_start(E, prec, sh.plan, (uint32_t)plan.size(), n_tiles, n_comp, sh.n_sample,
                                sh.sample_ids, sh.sample_heads, sh.qd, nq, s);
    if (st != APEX_OK) return st;
    if (any_spec) HIP_TRY(hipMemcpyAsync(sh.qd, qd.data(), sizeof(QueryDev) * nq, hipMemcpyHostToDevice, s));
    scored += sh.n_sample;
  }

  // 2. chunked enumeration
  const auto chunks = chunk_schedule(n_tiles, tile_compounds(E->scalar), E->scalar);
  if (chunks.size() + 1 > sh.n_flags) return set_error(APEX_E_INVALID, "internal: chunk count");
  const uint32_t last_flag = sh.n_flags - 1;  // flag slot of the closing selections (never set)
  for (size_t c = 0; c < chunks.size(); ++c) {
    apex_status st = enum_pass(E, prec, sh.plan, (uint32_t)plan.size(), chunks[c].first, chunks[c].second, sh.qd,
                               nq, plan_compounds(E, prec, plan, chunks[c].first, chunks[c].second), sh.work, s);
    if (st != APEX_OK) return st;
    HIP_TRY(launch_select(sh.qd, nq, (uint32_t)c, 0, s));
  }
  scored += n_comp;
  HIP_TRY(launch_select(sh.qd, nq, last_flag, 1, s));

  // 3-4. answers, enqueued behind the enumeration; one readback of every
  // query's block then shows whether a chunk overflowed a candidate buffer, in
  // which case those chunks are re-run and the answers enqueued again
  const char* base = P[0].out;
  const size_t span = (size_t)((P[nq - 1].out + P[nq - 1].out_bytes) - base);
  // Long answers (over kDirectReadback bytes): each round reads back only the
  // queries' control words, and the answer arrays go from the device straight
  // into the result arrays once the rounds settle, n_found entries each.
  std::vector<size_t> ctl_off(nq);
  size_t ctl_total = 0;
  for (uint32_t i = 0; i < nq; ++i) {
    ctl_off[i] = ctl_total;
    ctl_total += out_control_bytes(P[i]);
  }
  const bool direct = span - ctl_total > kDirectReadback;
  Readback rb(E, direct ? ctl_total : span, pageable_readback);
  auto host_of = [&](uint32_t i) -> const char* {  // host copy of query i's block from P[i].out on
    return direct ? rb.data() + ctl_off[i] : rb.data() + (P[i].out - base);
  };
  uint32_t reruns = 0;
  for (int round = 0;; ++round) {
    for (uint32_t i = 0; i < nq; ++i) {
      apex_status st = finish_launch(E, P[i], sh.qd + i, sh.qx + i, s);
      if (st != APEX_OK) return st;
    }
    if (direct) {
      for (uint32_t i = 0; i < nq; ++i)
        HIP_TRY(hipMemcpyAsync(rb.data() + ctl_off[i], P[i].out, out_control_bytes(P[i]), hipMemcpyDeviceToHost, s));
    } else {
      HIP_TRY(hipMemcpyAsync(rb.data(), base, span, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<uint32_t> flags((size_t)nq * sh.n_flags);
    for (uint32_t i = 0; i < nq; ++i)
      std::memcpy(flags.data() + (size_t)i * sh.n_flags, out_flags(P[i], host_of(i), P[i].out), 4 * sh.n_flags);
    // a speculative threshold that left fewer than K survivors was above the
    // final K-th key: that query is enumerated again from scratch
    std::vector<uint8_t> redo(nq, 0);
    bool any_redo = false;
    for (uint32_t i = 0; i < nq; ++i) {
      if (!spec[i]) continue;
      spec[i] = 0;
      const QState* st = in_copy(host_of(i), P[i].out, P[i].st);
      if (st->warm && st->count < P[i].K) {
        redo[i] = 1;
        any_redo = true;
        std::fill(flags.begin() + (size_t)i * sh.n_flags, flags.begin() + (size_t)(i + 1) * sh.n_flags, 0u);
      }
    }
    bool any = false;
    for (uint32_t f : flags) any |= f != 0;
    if (!any && !any_redo) break;
    if (round > 64) return set_error(APEX_E_DEVICE, "candidate buffer overflow did not settle");
    for (uint32_t i = 0; i < nq; ++i) {
      apex_status st = fill_u32(P[i].rerun, sh.n_flags, 0u, s);
      if (st != APEX_OK) return st;
    }
    if (any_redo) {
      for (uint32_t i = 0; i < nq; ++i) {
        qd[i].active = redo[i];
        if (redo[i]) HIP_TRY(launch_state_reset(P[i].st, s));
      }
      HIP_TRY(hipMemcpyAsync(sh.qd, qd.data(), sizeof(QueryDev) * nq, hipMemcpyHostToDevice, s));
      for (size_t c = 0; c < chunks.size(); ++c) {
        const uint64_t cc = plan_compounds(E, prec, plan, chunks[c].first, chunks[c].second);
        apex_status st = enum_pass(E, prec, sh.plan, (uint32_t)plan.size(), chunks[c].first, chunks[c].second,
                                   sh.qd, nq, cc, sh.work, s);
        if (st != APEX_OK) return st;
        HIP_TRY(launch_select(sh.qd, nq, (uint32_t)c, 0, s));
        scored += cc;
        ++reruns;
      }
    }
    for (size_t c = 0; c < chunks.size(); ++c) {
      bool need = false;
      for (uint32_t i = 0; i < nq; ++i) {
        qd[i].active = flags[(size_t)i * sh.n_flags + c] ? 1u : 0u;
        need |= qd[i].active != 0;
      }
      if (!need) continue;
      HIP_TRY(hipMemcpyAsync(sh.qd, qd.data(), sizeof(QueryDev) * nq, hipMemcpyHostToDevice, s));
      const uint64_t cc = plan_compounds(E, prec, plan, chunks[c].first, chunks[c].second);
      apex_status st = enum_pass(E, prec, sh.plan, (uint32_t)plan.size(), chunks[c].first, chunks[c].second,
                                 sh.qd, nq, cc, sh.work, s);
      if (st != APEX_OK) return st;
      HIP_TRY(launch_select(sh.qd, nq, (uint32_t)c, 0, s));
      scored += cc;
      ++reruns;
    }
    for (uint32_t i = 0; i < nq; ++i) qd[i].active = 1;
    HIP_TRY(hipMemcpyAsync(sh.qd, qd.data(), sizeof(QueryDev) * nq, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_select(sh.qd, nq, last_flag, 1, s));
  }
  for (uint32_t i = 0; i < nq; ++i) {
    if (direct) {
      apex_status st = finish_read_direct(E, P[i], host_of(i), P[i].out, &res[i], s);
      if (st != APEX_OK) return st;
    } else {
      finish_read(E, P[i], host_of(i), P[i].out, &res[i]);
    }
    res[i].n_scored = scored;
    res[i].n_reruns = reruns;
  }
  if (direct) HIP_TRY(hipStreamSynchronize(s));
  return profile_collect(E);
}

extern "C" apex_status apex_query_workspace_size(const apex_engine* eng, const apex_query* q, size_t* bytes) {
  return apex_batch_workspace_size(eng, q, 1, bytes);
}

extern "C" apex_status apex_batch_workspace_size(const apex_engine* eng, const apex_query* qs, uint32_t n,
                                                 size_t* bytes) {
  if (!eng || !qs || !bytes || n == 0) return set_error(APEX_E_INVALID, "null argument");
  if (n > APEX_MAX_FUSED_QUERIES) return set_error(APEX_E_INVALID, "%u queries > %d", n, APEX_MAX_FUSED_QUERIES);
  for (uint32_t i = 0; i < n; ++i) {
    apex_status st = validate_query(eng, &qs[i]);
    if (st != APEX_OK) return st;
    if (qs[i].precision != qs[0].precision) return set_error(APEX_E_INVALID, "fused queries must share one precision");
  }
  std::vector<QPlan> P;
  Shared sh;
  Bump b(nullptr);
  batch_layout(eng, qs, n, b, P, sh);
  *bytes = b.off;
  return APEX_OK;
}

// One query; with APEX_QUERY_KEEP_VIOLATORS and fewer than k feasible
// compounds, a second pass ranks the violating compounds by their violation
// (the queue of Section 4.3 without its final removal) and fills the rest of
// the answer with the best of them.
static apex_status search_one(apex_engine* E, const apex_query* q, void* ws, size_t ws_bytes, hipStream_t s,
                              apex_result* res, bool pageable) {
  apex_status st = run_search(E, q, 1, ws, ws_bytes, s, res, pageable, false);
  if (st != APEX_OK || !(q->flags & APEX_QUERY_KEEP_VIOLATORS) || res->n_found >= q->k) return st;
  const uint64_t nf = res->n_found;
  apex_query q2 = *q;
  q2.k = q->k - nf;
  apex_result r2{};
  r2.capacity = q2.k;
  r2.ids = res->ids + nf;
  r2.objective = res->objective + nf;
  r2.heads = res->heads ? res->heads + nf * E->H : nullptr;
  r2.reaction = res->reaction ? res->reaction + nf : nullptr;
  r2.synthon = res->synthon ? res->synthon + nf * 3 : nullptr;
  r2.violation = res->violation ? res->violation + nf : nullptr;
  st = run_search(E, &q2, 1, ws, ws_bytes, s, &r2, pageable, true);
  if (st != APEX_OK) return st;
  res->n_found = nf + r2.n_found;
  res->n_scored += r2.n_scored;
  res->n_candidates += r2.n_candidates;
  res->n_reruns += r2.n_reruns;
  return APEX_OK;
}

extern "C" apex_status apex_search(apex_engine* eng, const apex_query* q, void* workspace, size_t workspace_bytes,
                                   void* stream, apex_result* result) {
  return search_one(eng, q, workspace, workspace_bytes, (hipStream_t)stream, result, false);
}

extern "C" apex_status apex_search_batch(apex_engine* eng, const apex_query* qs, uint32_t n, void* workspace,
                                         size_t workspace_bytes, void* stream, apex_result* results) {
  return run_search(eng, qs, n, workspace, workspace_bytes, (hipStream_t)stream, results);
}

extern "C" apex_status apex_engine_profile(apex_engine* eng, int enable, double* ms, uint64_t* launches,
                                           uint64_t* compounds) {
  if (!eng) return set_error(APEX_E_INVALID, "null engine");
  apex_status st = profile_collect(eng);
  if (st != APEX_OK) return st;
  if (ms) *ms = eng->prof_ms;
  if (launches) *launches = eng->prof_launches;
  if (compounds) *compounds = eng->prof_compounds;
  eng->profile = enable != 0;
  eng->prof_ms = 0.0;
  eng->prof_launches = 0;
  eng->prof_compounds = 0;
  return APEX_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free search: the query's scratch is a file-scope device array,
// one copy per GPU, held until the process ends. Host code never passes the
// array's name to a kernel or a copy (on the host it only names a stand-in);
// it uses the device address hipGetSymbolAddress reports for the current
// device, looked up once per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[APEX_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

apex_status static_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(APEX_E_UNSUPPORTED, "device %d >= %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(APEX_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return APEX_OK;
}
}  // namespace

extern "C" apex_status apex_search_noalloc(apex_engine* eng, const apex_query* q, void* stream, apex_result* result) {
  if (!eng || !q || !result) return set_error(APEX_E_INVALID, "null argument");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != eng->device)
    return set_error(APEX_E_INVALID, "current device %d is not the engine's device %d", dev, eng->device);
  size_t need = 0;
  apex_status st = apex_query_workspace_size(eng, q, &need);
  if (st != APEX_OK) return st;
  if (need > APEX_STATIC_SCRATCH_BYTES)
    return set_error(APEX_E_NOMEM, "query needs %zu bytes of scratch, more than the static %zu (use apex_search)",
                     need, (size_t)APEX_STATIC_SCRATCH_BYTES);
  void* ws = nullptr;
  st = static_scratch(dev, &ws);
  if (st != APEX_OK) return st;
  return search_one(eng, q, ws, APEX_STATIC_SCRATCH_BYTES, (hipStream_t)stream, result, true);
}
