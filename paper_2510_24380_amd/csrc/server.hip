// Serving loop: continuous batching of queries over one engine.
//
// A host thread owns the device work. Submitted queries wait until their
// workspace fits in the caller's memory pool and an active slot is free; the
// smallest waiting query (compounds searched) is admitted first, except on every
// fourth admission, which takes the oldest.
// The library is cut into reaction-aligned chunks; every pass evaluates one chunk
// once for all active queries (of one precision) that still need it, so the
// combine and the decoder run once per compound for the whole group, and the
// objective, bounds and selection run per query (the fused kernel's query loop).
// A query joins at the next pass after admission and completes after it has
// seen every chunk holding its reactions, wrapping around the chunk cycle (the
// chunk of each pass is chosen for the active query with the fewest chunks
// left, or on every fourth pass for the oldest one); then
// its overflowed chunks are re-run, its pool rescored and its answer decoded and
// copied to the host. Per-compound arithmetic does not depend on which queries
// share a pass, so a query's result is the same alone and in any mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "launch.h"
#include "search_impl.h"

using namespace apex;

namespace {

using Clock = std::chrono::steady_clock;

double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }

enum { Q_PENDING = 0, Q_ACTIVE = 1, Q_DONE = 2, Q_CANCELLED = 3, Q_FAILED = 4 };

struct SQ {
  uint64_t ticket = 0;
  apex_query q{};
  std::vector<float> w;
  std::vector<apex_constraint> cons;
  std::vector<uint32_t> subset;
  QPlan P;
  size_t off = 0, bytes = 0;
  int slot = -1;
  std::vector<uint8_t> need;  // per chunk: still to be evaluated for this query
  uint32_t remaining = 0;
  uint64_t n_comp = 0;
  double t_submit = 0, t_done = 0;
  int state = Q_PENDING;
  bool cancel = false;
  apex_status err = APEX_OK;
  std::string err_text;
  std::vector<uint64_t> ids;
  std::vector<float> obj, heads;
  std::vector<uint32_t> reaction, synthon;
  uint64_t n_found = 0, n_scored = 0, n_candidates = 0;
  uint32_t n_reruns = 0;
};

// Reactions [r0, r1); a reaction larger than a chunk is split into chunks of
// consecutive tiles [tile0, tile1) of that one reaction (tiles are 8 x 16
// compounds in every precision), so that no pass runs much longer than a chunk.
struct Chunk {
  uint32_t r0, r1;
  uint64_t compounds;
  uint64_t tile0 = 0, tile1 = UINT64_MAX;
};

// First-fit allocator over [0, size) with 256-byte granularity.
struct Pool {
  std::map<size_t, size_t> free_;  // offset -> size
  void init(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, o = it->first + bytes;
        free_.erase(it);
        if (rest) free_[o] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

}  // namespace

struct apex_server {
  apex_engine* E = nullptr;
  apex_server_config cfg{};
  hipStream_t s = nullptr;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<std::shared_ptr<SQ>> pending;
  std::vector<std::shared_ptr<SQ>> slots;
  std::map<uint64_t, std::shared_ptr<SQ>> tickets;
  // device header of the pool
  QueryDev* qd_dev = nullptr;
  QueryDev* qx_dev = nullptr;
  SelDev* plan_dev = nullptr;
  uint32_t* work = nullptr;  // tile-sharing counters of the fused passes
  uint64_t* sample_ids = nullptr;
  float* sample_heads = nullptr;
  uint32_t n_sample = 0;
  char* arena = nullptr;
  Pool pool;
  std::vector<QueryDev> qd, qx;
  std::vector<Chunk> chunks;
  uint32_t cursor[3] = {0, 0, 0};
  int next_prec = 0;
  uint64_t passes = 0, admissions = 0;
  // statistics
  uint64_t submitted = 0, completed = 0, cancelled = 0, failed = 0;
  std::vector<double> latencies_ms;
  double busy_s = 0.0;
  uint64_t compounds = 0;
};

namespace {

size_t query_bytes(const apex_server* S, const apex_query* q, QPlan* P) {
  query_sizes(S->E, q, *P);
  Bump b(nullptr);
  query_layout(S->E->lib->T, (uint32_t)S->chunks.size() + 1, b, *P);
  out_layout(b, *P);
  return b.off;
}

// Reactions of a chunk that at least one of the listed queries searches.
void chunk_plan(apex_server* S, int prec, const Chunk& ch, const std::vector<SQ*>& qs, std::vector<SelDev>& plan,
                uint64_t* n_tiles, uint64_t* n_comp) {
  std::vector<uint32_t> rs;
  for (uint32_t t = ch.r0; t < ch.r1; ++t) {
    bool want = false;
    for (SQ* q : qs) {
      if (q->subset.empty() || std::binary_search(q->subset.begin(), q->subset.end(), t)) {
        want = true;
        break;
      }
    }
    if (want) rs.push_back(t);
  }
  build_plan(S->E->lib, S->E->scalar, rs, plan, n_tiles, n_comp);
}

bool chunk_wanted(const Chunk& ch, const SQ* q) {
  if (q->subset.empty()) return true;
  auto it = std::lower_bound(q->subset.begin(), q->subset.end(), ch.r0);
  return it != q->subset.end() && *it < ch.r1;
}

apex_status upload_active(apex_server* S, const std::vector<int>& on_slots) {
  for (auto& d : S->qd) d.active = 0;
  for (int sl : on_slots) S->qd[sl].active = 1;
  hipError_t e = hipMemcpyAsync(S->qd_dev, S->qd.data(), sizeof(QueryDev) * S->qd.size(), hipMemcpyHostToDevice, S->s);
  return e == hipSuccess ? APEX_OK : set_error(APEX_E_DEVICE, "upload: %s", hipGetErrorString(e));
}

// One fused pass: chunk c for the listed queries (all of precision prec).
apex_status run_pass(apex_server* S, int prec, uint32_t c, const std::vector<SQ*>& qs) {
  std::vector<SelDev> plan;
  uint64_t n_tiles = 0, n_comp = 0;
  chunk_plan(S, prec, S->chunks[c], qs, plan, &n_tiles, &n_comp);
  if (n_tiles == 0) return APEX_OK;
  std::vector<int> on;
  for (SQ* q : qs) on.push_back(q->slot);
  apex_status st = upload_active(S, on);
  if (st != APEX_OK) return st;
  hipError_t e = hipMemcpyAsync(S->plan_dev, plan.data(), sizeof(SelDev) * plan.size(), hipMemcpyHostToDevice, S->s);
  if (e != hipSuccess) return set_error(APEX_E_DEVICE, "upload: %s", hipGetErrorString(e));
  const Chunk& ch = S->chunks[c];
  const uint64_t v0 = std::min(ch.tile0, n_tiles), v1 = std::min(ch.tile1, n_tiles);
  if (v0 > 0 || v1 < n_tiles) n_comp = plan_compounds(S->E, prec, plan, v0, v1);
  const double t0 = now_s();
  st = enum_pass(S->E, prec, S->plan_dev, (uint32_t)plan.size(), v0, v1, S->qd_dev, (uint32_t)S->qd.size(), n_comp,
                 S->work, S->s);
  if (st != APEX_OK) return st;
  e = launch_select(S->qd_dev, (uint32_t)S->qd.size(), c, 0, S->s);
  if (e == hipSuccess) e = hipStreamSynchronize(S->s);
  if (e != hipSuccess) return set_error(APEX_E_DEVICE, "pass: %s", hipGetErrorString(e));
  S->busy_s += now_s() - t0;
  S->compounds += n_comp;
  for (SQ* q : qs) q->n_scored += n_comp;
  return profile_collect(S->E);
}

apex_status admit(apex_server* S, SQ* q) {
  apex_engine* E = S->E;
  Bump b(S->arena + q->off);
  query_layout(E->lib->T, (uint32_t)S->chunks.size() + 1, b, q->P);
  out_layout(b, q->P);
  apex_status st = query_device_init(E, &q->q, q->P, S->s);
  if (st != APEX_OK) return st;
  S->qd[q->slot] = make_qdev(E, &q->q, q->P, true, false);
  S->qd[q->slot].active = 0;
  S->qx[q->slot] = make_qdev(E, &q->q, q->P, false, q->P.lowp);
  hipError_t e = hipMemcpyAsync(S->qx_dev + q->slot, &S->qx[q->slot], sizeof(QueryDev), hipMemcpyHostToDevice, S->s);
  if (e != hipSuccess) return set_error(APEX_E_DEVICE, "upload: %s", hipGetErrorString(e));
  // compounds searched and chunks needed
  q->need.assign(S->chunks.size(), 0);
  q->remaining = 0;
  for (size_t c = 0; c < S->chunks.size(); ++c) {
    if (!chunk_wanted(S->chunks[c], q)) continue;
    q->need[c] = 1;
    q->remaining++;
  }
  // warm start: a sample of the whole library, scored with the query's subset;
  // no larger than the query's candidate buffer, which the sampled entries pass
  // through before the selection drops them
  const int prec = (int)q->q.precision;
  const uint32_t n_sample = std::min<uint32_t>(S->n_sample, q->P.cap);
  if (E->lib->total >= 8ull * n_sample && q->n_comp >= 8ull * n_sample) {
    st = upload_active(S, {q->slot});
    if (st != APEX_OK) return st;
    st = warm_start(E, prec, E->prec[prec].plan, E->lib->T, E->prec[prec].full_tiles, E->prec[prec].full_compounds,
                    n_sample, S->sample_ids, S->sample_heads, S->qd_dev, (uint32_t)S->qd.size(), S->s);
    if (st != APEX_OK) return st;
    q->n_scored += n_sample;
  }
  return APEX_OK;
}

apex_status finalize(apex_server* S, SQ* q) {
  apex_engine* E = S->E;
  const int prec = (int)q->q.precision;
  const uint32_t last_flag = (uint32_t)S->chunks.size();
  apex_status st = upload_active(S, {q->slot});
  if (st != APEX_OK) return st;
  hipError_t e = launch_select(S->qd_dev + q->slot, 1, last_flag, 1, S->s);
  if (e != hipSuccess) return set_error(APEX_E_DEVICE, "select: %s", hipGetErrorString(e));
  // the answer is enqueued behind the last select; one readback of the query's
  // block then shows whether any chunk overflowed and must be re-run first
  std::vector<uint32_t> flags(S->chunks.size() + 1);
  Readback rb(E, q->P.out_bytes);
  for (int round = 0;; ++round) {
    st = finish_launch(E, q->P, S->qd_dev + q->slot, S->qx_dev + q->slot, S->s);
    if (st != APEX_OK) return st;
    e = hipMemcpyAsync(rb.data(), q->P.out, q->P.out_bytes, hipMemcpyDeviceToHost, S->s);
    if (e == hipSuccess) e = hipStreamSynchronize(S->s);
    if (e != hipSuccess) return set_error(APEX_E_DEVICE, "readback: %s", hipGetErrorString(e));
    std::memcpy(flags.data(), out_flags(q->P, rb.data(), q->P.out), sizeof(uint32_t) * flags.size());
    bool any = false;
    for (uint32_t f : flags) any |= f != 0;
    if (!any) break;
    if (round > 64) return set_error(APEX_E_DEVICE, "candidate buffer overflow did not settle");
    st = fill_u32(q->P.rerun, (uint32_t)flags.size(), 0u, S->s);
    if (st != APEX_OK) return st;
    for (uint32_t c = 0; c < S->chunks.size(); ++c) {
      if (!flags[c]) continue;
      st = run_pass(S, prec, c, {q});
      if (st != APEX_OK) return st;
      q->n_reruns++;
    }
    st = upload_active(S, {q->slot});
    if (st != APEX_OK) return st;
    e = launch_select(S->qd_dev + q->slot, 1, last_flag, 1, S->s);
    if (e != hipSuccess) return set_error(APEX_E_DEVICE, "select: %s", hipGetErrorString(e));
  }
  const uint32_t k = (uint32_t)q->q.k;
  q->ids.resize(k);
  q->obj.resize(k);
  q->heads.resize((size_t)k * E->H);
  q->reaction.resize(k);
  q->synthon.resize((size_t)k * 3);
  apex_result r{};
  r.capacity = k;
  r.ids = q->ids.data();
  r.objective = q->obj.data();
  r.heads = q->heads.data();
  r.reaction = q->reaction.data();
  r.synthon = q->synthon.data();
  finish_read(E, q->P, rb.data(), q->P.out, &r);
  q->n_found = r.n_found;
  q->n_candidates = r.n_candidates;
  return APEX_OK;
}

void release_slot(apex_server* S, SQ* q) {
  if (q->slot >= 0) {
    S->slots[q->slot].reset();
    S->pool.release(q->off, q->bytes);
    q->slot = -1;
  }
}

void worker_loop(apex_server* S) {
  std::vector<std::shared_ptr<SQ>> admitted;
  for (;;) {
    admitted.clear();
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (;;) {
        if (S->stop) return;
        // cancelled active queries leave at a pass boundary
        for (auto& sp : S->slots)
          if (sp && sp->cancel) {
            sp->state = Q_CANCELLED;
            S->cancelled++;
            release_slot(S, sp.get());
            S->cv_done.notify_all();
          }
        for (auto it = S->pending.begin(); it != S->pending.end();) {
          if ((*it)->cancel) {
            (*it)->state = Q_CANCELLED;
            S->cancelled++;
            S->cv_done.notify_all();
            it = S->pending.erase(it);
          } else {
            ++it;
          }
        }
        while (!S->pending.empty()) {
          // the smallest waiting query first (compounds searched), except on
          // every fourth admission, which takes the oldest
          size_t pick = 0;
          if (S->admissions % 4 != 3)
            for (size_t i = 1; i < S->pending.size(); ++i)
              if (S->pending[i]->n_comp < S->pending[pick]->n_comp) pick = i;
          auto q = S->pending[pick];
          int slot = -1;
          for (size_t i = 0; i < S->slots.size(); ++i)
            if (!S->slots[i]) {
              slot = (int)i;
              break;
            }
          if (slot < 0) break;
          size_t off = 0;
          if (!S->pool.alloc(q->bytes, &off)) break;
          S->pending.erase(S->pending.begin() + (long)pick);
          S->admissions++;
          q->off = off;
          q->slot = slot;
          q->state = Q_ACTIVE;
          S->slots[slot] = q;
          admitted.push_back(q);
        }
        bool any_active = false;
        for (auto& sp : S->slots) any_active |= (bool)sp;
        if (any_active) break;
        S->cv_work.wait(lk);
      }
    }
    auto fail_all = [&](apex_status st) {
      std::lock_guard<std::mutex> lk(S->mu);
      const std::string text = apex_last_error();
      for (auto& sp : S->slots)
        if (sp) {
          sp->state = Q_FAILED;
          sp->err = st;
          sp->err_text = text;
          S->failed++;
          release_slot(S, sp.get());
        }
      S->cv_done.notify_all();
    };
    auto complete = [&](SQ* q) {
      std::lock_guard<std::mutex> lk(S->mu);
      q->state = Q_DONE;
      q->t_done = now_s();
      S->latencies_ms.push_back((q->t_done - q->t_submit) * 1e3);
      S->completed++;
      release_slot(S, q);
      S->cv_done.notify_all();
    };
    bool dead = false;
    for (auto& q : admitted) {
      apex_status st = admit(S, q.get());
      if (st == APEX_OK && q->remaining == 0) {
        st = finalize(S, q.get());
        if (st == APEX_OK) complete(q.get());
      }
      if (st != APEX_OK) {
        fail_all(st);
        dead = true;
        break;
      }
    }
    if (dead) continue;
    // choose a precision with work, round robin, then the next chunk it needs
    std::vector<SQ*> act[3];
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (auto& sp : S->slots)
        if (sp && sp->state == Q_ACTIVE && !sp->cancel && sp->remaining > 0) act[sp->q.precision].push_back(sp.get());
    }
    int prec = -1;
    for (int i = 0; i < 3; ++i) {
      const int p = (S->next_prec + i) % 3;
      if (!act[p].empty()) {
        prec = p;
        break;
      }
    }
    if (prec < 0) continue;
    S->next_prec = (prec + 1) % 3;
    // The pass takes the next chunk (from the cursor on) that a lead query
    // needs, and every active query of this precision that needs that chunk
    // joins it. The lead is the query with the fewest chunks left (short
    // queries are not held behind long ones), except on every fourth pass,
    // where it is the oldest query (long ones keep progressing under load).
    SQ* lead = nullptr;
    const bool oldest = (S->passes++ % 4) == 3;
    for (SQ* q : act[prec]) {
      const bool better = !lead || (oldest ? q->t_submit < lead->t_submit
                                           : (q->remaining < lead->remaining ||
                                              (q->remaining == lead->remaining && q->t_submit < lead->t_submit)));
      if (better) lead = q;
    }
    const uint32_t nch = (uint32_t)S->chunks.size();
    uint32_t c = S->cursor[prec];
    for (uint32_t step = 0; step < nch && !lead->need[c]; ++step) c = (c + 1) % nch;
    std::vector<SQ*> part;
    for (SQ* q : act[prec])
      if (q->need[c]) part.push_back(q);
    if (part.empty()) continue;
    apex_status st = run_pass(S, prec, c, part);
    if (st != APEX_OK) {
      fail_all(st);
      continue;
    }
    S->cursor[prec] = (c + 1) % nch;
    for (SQ* q : part) {
      q->need[c] = 0;
      if (--q->remaining == 0) {
        st = finalize(S, q);
        if (st != APEX_OK) {
          fail_all(st);
          break;
        }
        complete(q);
      }
    }
  }
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double x = p * (double)(v.size() - 1);
  const size_t i = (size_t)std::floor(x);
  const size_t j = std::min(v.size() - 1, i + 1);
  return v[i] + (x - (double)i) * (v[j] - v[i]);
}

}  // namespace

extern "C" apex_status apex_server_create(apex_engine* eng, const apex_server_config* cfg, apex_server** out) {
  if (!eng || !cfg || !out) return set_error(APEX_E_INVALID, "null argument");
  *out = nullptr;
  if (!cfg->pool) return set_error(APEX_E_INVALID, "null memory pool");
  if (((uintptr_t)cfg->pool) & 255) return set_error(APEX_E_INVALID, "pool must be 256-byte aligned");
  if (cfg->max_active == 0 || cfg->max_active > APEX_MAX_FUSED_QUERIES)
    return set_error(APEX_E_INVALID, "max_active must be in 1..%d", APEX_MAX_FUSED_QUERIES);
  auto S = std::make_unique<apex_server>();
  S->E = eng;
  S->cfg = *cfg;
  S->s = (hipStream_t)cfg->stream;
  // chunks of about chunk_compounds: runs of whole reactions, and tile ranges of
  // reactions larger than that
  const uint64_t target = cfg->chunk_compounds ? cfg->chunk_compounds : (1ull << 26);
  const apex_library* L = eng->lib;
  uint32_t r0 = 0;
  uint64_t acc = 0;
  for (uint32_t t = 0; t < L->T; ++t) {
    const uint64_t n_t = L->id_off[t + 1] - L->id_off[t];
    if (n_t > target) {
      if (acc > 0) S->chunks.push_back({r0, t, acc});
      const ReactDev& rd = eng->react_host[t];
      const uint64_t TA = tile_ta(eng->scalar), TB = tile_tb(eng->scalar);
      const uint64_t tiles = ((rd.nA + TA - 1) / TA) * ((rd.nB + TB - 1) / TB);
      const uint64_t pieces = (n_t + target - 1) / target;
      const uint64_t per = (tiles + pieces - 1) / pieces;
      for (uint64_t v = 0; v < tiles; v += per)
        S->chunks.push_back({t, t + 1, n_t * (std::min(tiles, v + per) - v) / tiles, v, std::min(tiles, v + per)});
      r0 = t + 1;
      acc = 0;
      continue;
    }
    acc += n_t;
    if (acc >= target || t + 1 == L->T) {
      S->chunks.push_back({r0, t + 1, acc});
      r0 = t + 1;
      acc = 0;
    }
  }
  if (acc > 0) S->chunks.push_back({r0, L->T, acc});
  S->n_sample = 1u << 16;
  Bump b(cfg->pool);
  S->qd_dev = b.take<QueryDev>(cfg->max_active);
  S->qx_dev = b.take<QueryDev>(cfg->max_active);
  S->plan_dev = b.take<SelDev>(L->T);
  S->work = b.take<uint32_t>(kWorkCounters);
  S->sample_ids = b.take<uint64_t>(S->n_sample);
  S->sample_heads = b.take<float>((size_t)S->n_sample * kHeadsPad);
  if (b.off >= cfg->pool_bytes)
    return set_error(APEX_E_NOMEM, "pool of %zu bytes < %zu bytes of server state", cfg->pool_bytes, b.off);
  S->arena = (char*)cfg->pool + b.off;
  S->pool.init(cfg->pool_bytes - b.off);
  S->slots.resize(cfg->max_active);
  S->qd.assign(cfg->max_active, QueryDev{});
  S->qx.assign(cfg->max_active, QueryDev{});
  hipError_t e = hipMemcpyAsync(S->qd_dev, S->qd.data(), sizeof(QueryDev) * cfg->max_active, hipMemcpyHostToDevice, S->s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(S->qx_dev, S->qx.data(), sizeof(QueryDev) * cfg->max_active, hipMemcpyHostToDevice, S->s);
  if (e == hipSuccess && fill_u32(S->work, kWorkCounters, 0u, S->s) != APEX_OK) e = hipErrorLaunchFailure;
  if (e == hipSuccess) e = hipStreamSynchronize(S->s);
  if (e != hipSuccess) return set_error(APEX_E_DEVICE, "server setup: %s", hipGetErrorString(e));
  int dev = 0;
  (void)hipGetDevice(&dev);
  apex_server* raw = S.get();
  raw->worker = std::thread([raw, dev]() {
    (void)hipSetDevice(dev);
    worker_loop(raw);
  });
  *out = S.release();
  return APEX_OK;
}

extern "C" apex_status apex_server_submit(apex_server* srv, const apex_query* q, uint64_t* ticket) {
  if (!srv || !q || !ticket) return set_error(APEX_E_INVALID, "null argument");
  apex_status st = validate_query(srv->E, q);
  if (st != APEX_OK) return st;
  if (q->flags & APEX_QUERY_KEEP_VIOLATORS)
    return set_error(APEX_E_UNSUPPORTED, "the violation-ranked fallback is not served; use apex_search");
  auto sq = std::make_shared<SQ>();
  sq->q = *q;
  sq->w.assign(q->objective_w, q->objective_w + srv->E->H);
  sq->cons.assign(q->constraints, q->constraints + q->n_constraints);
  sq->subset.assign(q->subset, q->subset + q->n_subset);
  std::sort(sq->subset.begin(), sq->subset.end());
  sq->q.objective_w = sq->w.data();
  sq->q.constraints = sq->cons.data();
  sq->q.subset = sq->subset.data();
  sq->bytes = query_bytes(srv, &sq->q, &sq->P);
  if (sq->subset.empty()) {
    sq->n_comp = srv->E->lib->total;
  } else {
    for (uint32_t t : sq->subset) sq->n_comp += srv->E->lib->id_off[t + 1] - srv->E->lib->id_off[t];
  }
  const size_t header = (size_t)(srv->arena - (char*)srv->cfg.pool);
  if (sq->bytes > srv->cfg.pool_bytes - header)
    return set_error(APEX_E_NOMEM, "query needs %zu bytes, more than the pool holds", sq->bytes);
  sq->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    sq->ticket = srv->next_ticket++;
    srv->pending.push_back(sq);
    srv->tickets[sq->ticket] = sq;
    srv->submitted++;
  }
  srv->cv_work.notify_one();
  *ticket = sq->ticket;
  return APEX_OK;
}

extern "C" apex_status apex_server_poll(apex_server* srv, uint64_t ticket, apex_result* result, int timeout_ms) {
  if (!srv) return set_error(APEX_E_INVALID, "null server");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return set_error(APEX_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  std::shared_ptr<SQ> q = it->second;
  auto finished = [&] { return q->state >= Q_DONE; };
  if (!finished()) {
    if (timeout_ms < 0) srv->cv_done.wait(lk, finished);
    else if (timeout_ms > 0) srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), finished);
  }
  if (!finished()) return APEX_E_PENDING;
  if (q->state == Q_CANCELLED) {
    srv->tickets.erase(it);
    return set_error(APEX_E_CANCELLED, "query %llu was cancelled", (unsigned long long)ticket);
  }
  if (q->state == Q_FAILED) {
    srv->tickets.erase(it);
    return set_error(q->err, "%s", q->err_text.c_str());
  }
  if (!result || !result->ids || !result->objective || result->capacity < q->n_found)
    return set_error(APEX_E_INVALID, "result needs capacity >= %llu and ids/objective arrays",
                     (unsigned long long)q->n_found);
  const uint64_t n = q->n_found;
  const uint32_t H = srv->E->H;
  std::memcpy(result->ids, q->ids.data(), n * sizeof(uint64_t));
  std::memcpy(result->objective, q->obj.data(), n * sizeof(float));
  if (result->heads) std::memcpy(result->heads, q->heads.data(), n * H * sizeof(float));
  if (result->reaction) std::memcpy(result->reaction, q->reaction.data(), n * sizeof(uint32_t));
  if (result->synthon) std::memcpy(result->synthon, q->synthon.data(), n * 3 * sizeof(uint32_t));
  result->n_found = n;
  result->n_scored = q->n_scored;
  result->n_candidates = q->n_candidates;
  result->n_reruns = q->n_reruns;
  srv->tickets.erase(it);
  return APEX_OK;
}

extern "C" apex_status apex_server_cancel(apex_server* srv, uint64_t ticket) {
  if (!srv) return set_error(APEX_E_INVALID, "null server");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return set_error(APEX_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    it->second->cancel = true;
  }
  srv->cv_work.notify_one();
  return APEX_OK;
}

extern "C" apex_status apex_server_stats_get(apex_server* srv, apex_server_stats* out) {
  if (!srv || !out) return set_error(APEX_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  out->submitted = srv->submitted;
  out->completed = srv->completed;
  out->cancelled = srv->cancelled;
  out->failed = srv->failed;
  uint64_t active = 0;
  for (auto& sp : srv->slots) active += sp ? 1 : 0;
  out->active = active;
  out->waiting = srv->pending.size();
  out->p50_latency_ms = percentile(srv->latencies_ms, 0.50);
  out->p99_latency_ms = percentile(srv->latencies_ms, 0.99);
  out->max_latency_ms = srv->latencies_ms.empty()
                            ? 0.0
                            : *std::max_element(srv->latencies_ms.begin(), srv->latencies_ms.end());
  out->compounds_per_s = srv->busy_s > 0 ? (double)srv->compounds / srv->busy_s : 0.0;
  out->compounds_scored = srv->compounds;
  return APEX_OK;
}

extern "C" apex_status apex_server_destroy(apex_server* srv) {
  if (!srv) return APEX_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  (void)hipStreamSynchronize(srv->s);
  delete srv;
  return APEX_OK;
}
