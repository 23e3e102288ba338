// Search driver: one query or several fused queries over the library.
//
// Pipeline per call (all device work on the caller's stream):
//  1. threshold warm start: a stratified sample of compounds is scored and each
//     query's threshold set just below its K-th best sampled key (a valid lower
//     bound of the final K-th key); the sample entries are then dropped;
//  2. chunked enumeration: the fused kernel appends compounds whose key beats
//     the threshold; after each chunk the select kernel compacts the buffer to
//     the K best and raises the threshold (the chain-of-batches merge of
//     Appendix A.8, without materialising any score array); a chunk whose
//     appends overflow the buffer is dropped and re-run once the threshold is
//     higher;
//  3. FP32 precision: the K = k survivors are the answer. BF16/FP8: the K =
//     pool_factor * k survivors (enumerated with bounds relaxed by a per-head
//     margin) are rescored in FP32 with the exact bounds and the best k kept;
//  4. rank sort by (objective desc, id asc), FP32 heads of the answer, decode of
//     ids to (reaction, synthons) on the GPU (Appendix A.8), copy to the host.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>

#include "engine_impl.h"
#include "launch.h"

using namespace apex;

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return set_error(APEX_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

namespace {

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

struct QPlan {
  uint32_t k = 0, K = 0, cap = 0, hwm = 0, cap2 = 0;
  bool lowp = false;
  QState* st = nullptr;
  float* cand_o = nullptr;
  uint64_t* cand_id = nullptr;
  float* tmp_o = nullptr;
  uint64_t* tmp_id = nullptr;
  uint32_t* rerun = nullptr;
  uint32_t* subset_dev = nullptr;
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

struct Shared {
  QueryDev* qd = nullptr;   // enumeration-pass queries (relaxed bounds in low precision)
  QueryDev* qx = nullptr;   // exact-bound queries of the rescoring pass
  SelDev* plan = nullptr;
  uint64_t* sample_ids = nullptr;
  float* sample_heads = nullptr;
  uint32_t* fill_zero = nullptr;
  uint32_t n_sample = 0;
  uint32_t max_chunks = 0;
};

constexpr uint64_t kFirstChunk = 1ull << 22;  // compounds in the first chunk
constexpr uint64_t kMaxChunk = 1ull << 27;

// Test knobs, read from the environment at every search: APEX_TEST_CHUNK fixes
// the chunk size (compounds) and APEX_TEST_CAP the candidate-buffer capacity
// (entries, at least 2K), so tests can force many chunks and buffer overflows.
uint64_t env_u64(const char* name) {
  const char* v = getenv(name);
  return v ? strtoull(v, nullptr, 10) : 0;
}

std::vector<std::pair<uint64_t, uint64_t>> chunk_schedule(uint64_t n_tiles, uint64_t tile_compounds) {
  std::vector<std::pair<uint64_t, uint64_t>> out;
  const uint64_t forced = env_u64("APEX_TEST_CHUNK");
  uint64_t per = std::max<uint64_t>(1, (forced ? forced : kFirstChunk) / tile_compounds);
  const uint64_t max_per = forced ? per : std::max<uint64_t>(1, kMaxChunk / tile_compounds);
  for (uint64_t v = 0; v < n_tiles;) {
    const uint64_t e = std::min(n_tiles, v + per);
    out.emplace_back(v, e);
    v = e;
    per = std::min(max_per, per * 2);
  }
  return out;
}

uint32_t tile_compounds(int prec) { return (uint32_t)(tile_ta(prec) * tile_tb(prec)); }

apex_status validate(const apex_engine* E, const apex_query* q) {
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

uint32_t max_chunks(const apex_engine* E, int prec) {
  return (uint32_t)chunk_schedule(E->prec[prec].full_tiles, tile_compounds(prec)).size() + 1;
}

void query_sizes(const apex_query* q, QPlan& P) {
  P.k = (uint32_t)q->k;
  P.lowp = q->precision != APEX_PREC_FP32;
  const uint32_t pf = q->pool_factor ? q->pool_factor : 4;
  P.K = P.lowp ? pf * P.k : P.k;
  uint64_t cap = std::min<uint64_t>(std::max<uint64_t>(64ull * P.K, 1ull << 18), 1ull << 22);
  cap = std::max<uint64_t>(cap, 2ull * P.K);
  const uint64_t forced = env_u64("APEX_TEST_CAP");
  if (forced) cap = std::max<uint64_t>(forced, 2ull * P.K);
  P.cap = (uint32_t)cap;
  P.hwm = P.cap / 2;
  P.cap2 = P.K;
}

uint32_t sample_count(const std::vector<QPlan>& P) {
  uint32_t kmax = 0, capmin = UINT32_MAX;
  for (auto& p : P) {
    kmax = std::max(kmax, p.K);
    capmin = std::min(capmin, p.cap);
  }
  uint64_t s = std::min<uint64_t>(std::max<uint64_t>(32ull * kmax, 1ull << 16), 1ull << 20);
  return (uint32_t)std::min<uint64_t>(s, capmin);
}

void layout(const apex_engine* E, const apex_query* qs, uint32_t n, Bump& b, std::vector<QPlan>& P, Shared& sh) {
  P.assign(n, QPlan());
  for (uint32_t i = 0; i < n; ++i) query_sizes(&qs[i], P[i]);
  const int prec = (int)qs[0].precision;
  sh.max_chunks = max_chunks(E, prec);
  sh.n_sample = sample_count(P);
  const uint32_t T = E->lib->T;
  sh.qd = b.take<QueryDev>(n);
  sh.qx = b.take<QueryDev>(n);
  sh.plan = b.take<SelDev>(T);
  sh.sample_ids = b.take<uint64_t>(sh.n_sample);
  sh.sample_heads = b.take<float>((size_t)sh.n_sample * kHeadsPad);
  for (uint32_t i = 0; i < n; ++i) {
    QPlan& p = P[i];
    p.st = b.take<QState>(1);
    p.cand_o = b.take<float>(p.cap);
    p.cand_id = b.take<uint64_t>(p.cap);
    p.tmp_o = b.take<float>(p.K);
    p.tmp_id = b.take<uint64_t>(p.K);
    p.rerun = b.take<uint32_t>(sh.max_chunks + 1);
    p.subset_dev = b.take<uint32_t>((T + 31) / 32);
    if (p.lowp) {
      p.pool_heads = b.take<float>((size_t)p.K * kHeadsPad);
      p.st2 = b.take<QState>(1);
      p.cand2_o = b.take<float>(p.cap2);
      p.cand2_id = b.take<uint64_t>(p.cap2);
      p.tmp2_o = b.take<float>(p.k);
      p.tmp2_id = b.take<uint64_t>(p.k);
    }
    p.fin_o = b.take<float>(p.k);
    p.fin_id = b.take<uint64_t>(p.k);
    p.fin_heads = b.take<float>((size_t)p.k * kHeadsPad);
    p.fin_reaction = b.take<uint32_t>(p.k);
    p.fin_synthon = b.take<uint32_t>((size_t)p.k * 3);
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t n, uint32_t v) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

QueryDev make_qdev(const apex_engine* E, const apex_query* q, const QPlan& p, bool relaxed, bool stage2) {
  QueryDev d{};
  for (int h = 0; h < kHeadsPad; ++h) {
    d.w[h] = h < (int)E->H ? q->objective_w[h] : 0.0f;
    d.lo[h] = -INFINITY;
    d.hi[h] = INFINITY;
  }
  for (uint32_t c = 0; c < q->n_constraints; ++c) {
    const apex_constraint& k = q->constraints[c];
    d.lo[k.head] = std::max(d.lo[k.head], k.lo);
    d.hi[k.head] = std::min(d.hi[k.head], k.hi);
  }
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
    d.rerun = p.rerun;  // not used: stage 2 never overflows (cap2 >= pool)
    d.cap = p.cap2;
    d.K = p.k;
    d.hwm = p.cap2;
  }
  d.subset_bits = q->n_subset ? p.subset_dev : nullptr;
  d.active = 1;
  return d;
}

struct EventPool {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  hipEvent_t get() {
    if (used == ev.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev.push_back(e);
    }
    return ev[used++];
  }
  ~EventPool() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

}  // namespace

static apex_status run_search(apex_engine* E, const apex_query* qs, uint32_t nq, void* ws, size_t ws_bytes,
                              hipStream_t s, apex_result* res) {
  if (!E || !qs || !res || nq == 0) return set_error(APEX_E_INVALID, "null argument");
  if (nq > APEX_MAX_FUSED_QUERIES) return set_error(APEX_E_INVALID, "%u queries > %d", nq, APEX_MAX_FUSED_QUERIES);
  for (uint32_t i = 0; i < nq; ++i) {
    apex_status st = validate(E, &qs[i]);
    if (st != APEX_OK) return st;
    if (qs[i].precision != qs[0].precision)
      return set_error(APEX_E_INVALID, "fused queries must share one precision");
    if (res[i].capacity < qs[i].k || !res[i].ids || !res[i].objective)
      return set_error(APEX_E_INVALID, "result %u: capacity < k or null ids/objective", i);
  }
  if (!ws) return set_error(APEX_E_INVALID, "null workspace");
  if (((uintptr_t)ws) & 255) return set_error(APEX_E_INVALID, "workspace must be 256-byte aligned");
  const int prec = (int)qs[0].precision;
  const apex_library* L = E->lib;
  PrecState& PS = E->prec[prec];

  std::vector<QPlan> P;
  Shared sh;
  {
    Bump b(nullptr);
    layout(E, qs, nq, b, P, sh);
    if (b.off > ws_bytes)
      return set_error(APEX_E_NOMEM, "query workspace %zu bytes < %zu needed", ws_bytes, b.off);
  }
  Bump b(ws);
  layout(E, qs, nq, b, P, sh);

  // reactions searched by at least one query
  std::vector<uint8_t> want(L->T, 0);
  std::vector<std::vector<uint32_t>> bits(nq);
  for (uint32_t i = 0; i < nq; ++i) {
    if (qs[i].n_subset == 0) {
      std::fill(want.begin(), want.end(), 1);
    } else {
      bits[i].assign((L->T + 31) / 32, 0u);
      for (uint32_t j = 0; j < qs[i].n_subset; ++j) {
        const uint32_t t = qs[i].subset[j];
        want[t] = 1;
        bits[i][t >> 5] |= 1u << (t & 31);
      }
    }
  }
  std::vector<uint32_t> reactions;
  for (uint32_t t = 0; t < L->T; ++t)
    if (want[t]) reactions.push_back(t);
  std::vector<SelDev> plan;
  uint64_t n_tiles = 0, n_comp = 0;
  build_plan(L, prec, reactions, plan, &n_tiles, &n_comp);

  // device state
  std::vector<QueryDev> qd(nq), qx(nq);
  for (uint32_t i = 0; i < nq; ++i) {
    qd[i] = make_qdev(E, &qs[i], P[i], true, false);
    qx[i] = make_qdev(E, &qs[i], P[i], false, P[i].lowp);
  }
  QState init{};
  init.tau_o = -INFINITY;
  init.tau_id = ~0ull;
  for (uint32_t i = 0; i < nq; ++i) {
    HIP_TRY(hipMemcpyAsync(P[i].st, &init, sizeof(QState), hipMemcpyHostToDevice, s));
    if (P[i].lowp) HIP_TRY(hipMemcpyAsync(P[i].st2, &init, sizeof(QState), hipMemcpyHostToDevice, s));
    if (!bits[i].empty())
      HIP_TRY(hipMemcpyAsync(P[i].subset_dev, bits[i].data(), bits[i].size() * 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_fill_u32, dim3((sh.max_chunks + 1 + 255) / 256), dim3(256), 0, s, P[i].rerun,
                       sh.max_chunks + 1, 0u);
  }
  HIP_TRY(hipMemcpyAsync(sh.qd, qd.data(), sizeof(QueryDev) * nq, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(sh.qx, qx.data(), sizeof(QueryDev) * nq, hipMemcpyHostToDevice, s));
  if (!plan.empty()) HIP_TRY(hipMemcpyAsync(sh.plan, plan.data(), sizeof(SelDev) * plan.size(), hipMemcpyHostToDevice, s));

  EnumArgs a{};
  a.P = E->P;
  a.react = E->react;
  a.sel = sh.plan;
  a.n_sel = (uint32_t)plan.size();
  a.pd = PS.dev;
  a.H2 = E->H2;
  a.n_queries = nq;
  a.queries = sh.qd;
  a.n_reactions = L->T;

  uint64_t scored = 0;
  // 1. threshold warm start from a stratified sample
  if (n_comp >= 8ull * sh.n_sample) {
    HIP_TRY(launch_sample_ids(sh.plan, (uint32_t)plan.size(), E->react, n_comp, sh.n_sample, 0xa5e7c0de1234ull,
                              sh.sample_ids, s));
    apex_status st = engine_gather(E, prec, sh.sample_ids, sh.n_sample, sh.sample_heads, s);
    if (st != APEX_OK) return st;
    HIP_TRY(launch_score(sh.sample_heads, sh.sample_ids, sh.n_sample, sh.qd, nq, s));
    HIP_TRY(launch_select(sh.qd, nq, sh.max_chunks, 1, s));
    HIP_TRY(launch_tau_relax(sh.qd, nq, s));
    scored += sh.n_sample;
  }

  // 2. chunked enumeration
  const auto chunks = chunk_schedule(n_tiles, tile_compounds(prec));
  if (chunks.size() + 1 > sh.max_chunks + 1) return set_error(APEX_E_INVALID, "internal: chunk count");
  uint32_t grid_full = (uint32_t)(E->n_cu * PS.wg_per_cu);
  grid_full = std::max<uint32_t>(8, grid_full / 8 * 8);
  EventPool evp;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> timed;
  std::vector<uint64_t> timed_comp;
  auto chunk_compounds = [&](uint64_t v0, uint64_t v1) -> uint64_t {
    // compounds of the selection inside tiles [v0, v1) (ragged tiles counted exactly)
    uint64_t c = 0;
    for (size_t r = 0; r < plan.size(); ++r) {
      const ReactDev& rd = E->react_host[plan[r].t];
      const uint64_t ta = (rd.nA + tile_ta(prec) - 1) / tile_ta(prec);
      const uint64_t t0 = plan[r].tile_start, t1 = t0 + ta * plan[r].tiles_b;
      if (t1 <= v0 || t0 >= v1) continue;
      if (t0 >= v0 && t1 <= v1) {
        c += (uint64_t)rd.nA * rd.nB;
        continue;
      }
      for (uint64_t v = std::max(v0, t0); v < std::min(v1, t1); ++v) {
        const uint64_t lt = v - t0;
        const uint64_t ia = lt / plan[r].tiles_b, ib = lt % plan[r].tiles_b;
        const uint64_t na = std::min<uint64_t>(tile_ta(prec), rd.nA - ia * tile_ta(prec));
        const uint64_t nb = std::min<uint64_t>(tile_tb(prec), rd.nB - ib * tile_tb(prec));
        c += na * nb;
      }
    }
    return c;
  };
  auto enum_chunk = [&](uint64_t v0, uint64_t v1) -> apex_status {
    a.tile_begin = v0;
    a.tile_end = v1;
    const uint64_t nt = v1 - v0;
    const uint32_t grid = nt < grid_full ? (uint32_t)nt : grid_full;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (E->profile) {
      e0 = evp.get();
      e1 = evp.get();
      if (e0) HIP_TRY(hipEventRecord(e0, s));
    }
    HIP_TRY(launch_enum(prec, E->H1, E->NL, E->act, false, a, grid, s));
    if (E->profile && e0 && e1) {
      HIP_TRY(hipEventRecord(e1, s));
      timed.emplace_back(e0, e1);
      timed_comp.push_back(chunk_compounds(v0, v1));
    }
    return APEX_OK;
  };
  for (size_t c = 0; c < chunks.size(); ++c) {
    apex_status st = enum_chunk(chunks[c].first, chunks[c].second);
    if (st != APEX_OK) return st;
    HIP_TRY(launch_select(sh.qd, nq, (uint32_t)c, 0, s));
  }
  scored += n_comp;
  HIP_TRY(launch_select(sh.qd, nq, sh.max_chunks, 1, s));

  // re-runs of chunks whose appends overflowed a candidate buffer
  std::vector<uint32_t> flags((size_t)nq * (sh.max_chunks + 1));
  uint32_t reruns = 0;
  for (int round = 0;; ++round) {
    for (uint32_t i = 0; i < nq; ++i)
      HIP_TRY(hipMemcpyAsync(flags.data() + (size_t)i * (sh.max_chunks + 1), P[i].rerun,
                             sizeof(uint32_t) * (sh.max_chunks + 1), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    bool any = false;
    for (uint32_t f : flags) any |= f != 0;
    if (!any) break;
    if (round > 64) return set_error(APEX_E_DEVICE, "candidate buffer overflow did not settle");
    for (uint32_t i = 0; i < nq; ++i)
      hipLaunchKernelGGL(k_fill_u32, dim3((sh.max_chunks + 1 + 255) / 256), dim3(256), 0, s, P[i].rerun,
                         sh.max_chunks + 1, 0u);
    for (size_t c = 0; c < chunks.size(); ++c) {
      bool need = false;
      for (uint32_t i = 0; i < nq; ++i) {
        qd[i].active = flags[(size_t)i * (sh.max_chunks + 1) + c] ? 1u : 0u;
        need |= qd[i].active != 0;
      }
      if (!need) continue;
      HIP_TRY(hipMemcpyAsync(sh.qd, qd.data(), sizeof(QueryDev) * nq, hipMemcpyHostToDevice, s));
      apex_status st = enum_chunk(chunks[c].first, chunks[c].second);
      if (st != APEX_OK) return st;
      HIP_TRY(launch_select(sh.qd, nq, (uint32_t)c, 0, s));
      scored += chunk_compounds(chunks[c].first, chunks[c].second);
      ++reruns;
    }
    for (uint32_t i = 0; i < nq; ++i) qd[i].active = 1;
    HIP_TRY(hipMemcpyAsync(sh.qd, qd.data(), sizeof(QueryDev) * nq, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_select(sh.qd, nq, sh.max_chunks, 1, s));
  }

  // 3-4. answer of each query
  std::vector<QState> stv(nq), st2v(nq);
  for (uint32_t i = 0; i < nq; ++i)
    HIP_TRY(hipMemcpyAsync(&stv[i], P[i].st, sizeof(QState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<uint32_t> n_found(nq);
  for (uint32_t i = 0; i < nq; ++i) {
    const uint32_t n1 = std::min(stv[i].count, P[i].K);
    if (!P[i].lowp) {
      HIP_TRY(launch_rank_sort(sh.qd, i, P[i].K, P[i].fin_o, P[i].fin_id, s));
      n_found[i] = n1;
    } else if (n1 > 0) {
      apex_status st = engine_gather(E, APEX_PREC_FP32, P[i].cand_id, n1, P[i].pool_heads, s);
      if (st != APEX_OK) return st;
      HIP_TRY(launch_score(P[i].pool_heads, P[i].cand_id, n1, sh.qx + i, 1, s));
      HIP_TRY(launch_select(sh.qx + i, 1, 0, 1, s));
      HIP_TRY(launch_rank_sort(sh.qx, i, P[i].k, P[i].fin_o, P[i].fin_id, s));
      HIP_TRY(hipMemcpyAsync(&st2v[i], P[i].st2, sizeof(QState), hipMemcpyDeviceToHost, s));
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  for (uint32_t i = 0; i < nq; ++i) {
    if (P[i].lowp) n_found[i] = std::min(st2v[i].count, P[i].k);
    if (n_found[i] == 0) continue;
    apex_status st = engine_gather(E, APEX_PREC_FP32, P[i].fin_id, n_found[i], P[i].fin_heads, s);
    if (st != APEX_OK) return st;
    HIP_TRY(launch_decode(E->react, L->T, P[i].fin_id, P[i].lowp ? P[i].st2 : P[i].st, P[i].k, P[i].fin_reaction,
                          P[i].fin_synthon, s));
  }
  std::vector<std::vector<float>> heads(nq);
  for (uint32_t i = 0; i < nq; ++i) {
    const uint32_t n = n_found[i];
    apex_result& r = res[i];
    r.n_found = n;
    r.n_scored = scored;
    r.n_candidates = stv[i].appended;
    r.n_reruns = reruns;
    if (n == 0) continue;
    HIP_TRY(hipMemcpyAsync(r.ids, P[i].fin_id, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(r.objective, P[i].fin_o, sizeof(float) * n, hipMemcpyDeviceToHost, s));
    if (r.heads) {
      heads[i].resize((size_t)n * kHeadsPad);
      HIP_TRY(hipMemcpyAsync(heads[i].data(), P[i].fin_heads, sizeof(float) * n * kHeadsPad, hipMemcpyDeviceToHost, s));
    }
    if (r.reaction) HIP_TRY(hipMemcpyAsync(r.reaction, P[i].fin_reaction, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s));
    if (r.synthon) HIP_TRY(hipMemcpyAsync(r.synthon, P[i].fin_synthon, sizeof(uint32_t) * 3 * n, hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  for (uint32_t i = 0; i < nq; ++i)
    if (res[i].heads && n_found[i])
      for (uint32_t e = 0; e < n_found[i]; ++e)
        std::memcpy(res[i].heads + (size_t)e * E->H, heads[i].data() + (size_t)e * kHeadsPad, sizeof(float) * E->H);
  if (E->profile) {
    for (size_t t = 0; t < timed.size(); ++t) {
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, timed[t].first, timed[t].second));
      E->prof_ms += ms;
      E->prof_launches += 1;
      E->prof_compounds += timed_comp[t];
    }
  }
  return APEX_OK;
}

extern "C" apex_status apex_query_workspace_size(const apex_engine* eng, const apex_query* q, size_t* bytes) {
  return apex_batch_workspace_size(eng, q, 1, bytes);
}

extern "C" apex_status apex_batch_workspace_size(const apex_engine* eng, const apex_query* qs, uint32_t n,
                                                 size_t* bytes) {
  if (!eng || !qs || !bytes || n == 0) return set_error(APEX_E_INVALID, "null argument");
  if (n > APEX_MAX_FUSED_QUERIES) return set_error(APEX_E_INVALID, "%u queries > %d", n, APEX_MAX_FUSED_QUERIES);
  for (uint32_t i = 0; i < n; ++i) {
    apex_status st = validate(eng, &qs[i]);
    if (st != APEX_OK) return st;
    if (qs[i].precision != qs[0].precision) return set_error(APEX_E_INVALID, "fused queries must share one precision");
  }
  std::vector<QPlan> P;
  Shared sh;
  Bump b(nullptr);
  layout(eng, qs, n, b, P, sh);
  *bytes = b.off;
  return APEX_OK;
}

extern "C" apex_status apex_search(apex_engine* eng, const apex_query* q, void* workspace, size_t workspace_bytes,
                                   void* stream, apex_result* result) {
  return run_search(eng, q, 1, workspace, workspace_bytes, (hipStream_t)stream, result);
}

extern "C" apex_status apex_search_batch(apex_engine* eng, const apex_query* qs, uint32_t n, void* workspace,
                                         size_t workspace_bytes, void* stream, apex_result* results) {
  return run_search(eng, qs, n, workspace, workspace_bytes, (hipStream_t)stream, results);
}

extern "C" apex_status apex_engine_profile(apex_engine* eng, int enable, double* ms, uint64_t* launches,
                                           uint64_t* compounds) {
  if (!eng) return set_error(APEX_E_INVALID, "null engine");
  if (ms) *ms = eng->prof_ms;
  if (launches) *launches = eng->prof_launches;
  if (compounds) *compounds = eng->prof_compounds;
  eng->profile = enable != 0;
  eng->prof_ms = 0.0;
  eng->prof_launches = 0;
  eng->prof_compounds = 0;
  return APEX_OK;
}
