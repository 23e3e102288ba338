// Host side of the C ABI (include/apex.h): handles, validation, workspace
// layout, the engine build (hoist and weight layouts) and the search driver
// (threshold warm start, chunked enumeration with selection, re-runs of
// overflowed chunks, FP32 rescoring of the low-precision pool, decode).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "engine_impl.h"
#include "launch.h"

using namespace apex;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

apex_status apex::set_error(apex_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return set_error(APEX_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

extern "C" const char* apex_status_string(apex_status s) {
  switch (s) {
    case APEX_OK: return "APEX_OK";
    case APEX_E_INVALID: return "APEX_E_INVALID";
    case APEX_E_NOMEM: return "APEX_E_NOMEM";
    case APEX_E_DEVICE: return "APEX_E_DEVICE";
    case APEX_E_UNSUPPORTED: return "APEX_E_UNSUPPORTED";
    case APEX_E_PENDING: return "APEX_E_PENDING";
    case APEX_E_CANCELLED: return "APEX_E_CANCELLED";
  }
  return "unknown apex_status";
}

extern "C" const char* apex_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// library
// ---------------------------------------------------------------------------
extern "C" apex_status apex_library_create(const apex_library_desc* desc, apex_library** out) {
  if (!desc || !out) return set_error(APEX_E_INVALID, "null argument");
  *out = nullptr;
  if (desc->n_reactions == 0 || !desc->n_slots || !desc->slot_sizes || !desc->tables || desc->d == 0)
    return set_error(APEX_E_INVALID, "library needs reactions, slot arrays, d >= 1 and a table pointer");
  auto* L = new apex_library();
  L->T = desc->n_reactions;
  L->d = desc->d;
  L->tables = desc->tables;
  uint64_t rows = 0, total = 0;
  uint32_t sb = 0;
  for (uint32_t t = 0; t < L->T; ++t) {
    const uint32_t ns = desc->n_slots[t];
    if (ns != 2 && ns != 3) {
      delete L;
      return set_error(APEX_E_INVALID, "reaction %u has %u slots (2 or 3 supported)", t, ns);
    }
    L->n_slots.push_back(ns);
    L->slot_base.push_back(sb);
    unsigned __int128 cnt = 1;
    for (uint32_t s = 0; s < ns; ++s) {
      const uint32_t n = desc->slot_sizes[sb + s];
      if (n == 0) {
        delete L;
        return set_error(APEX_E_INVALID, "reaction %u slot %u is empty", t, s);
      }
      L->slot_sizes.push_back(n);
      L->row_base.push_back(rows);
      rows += n;
      cnt *= n;
    }
    const uint64_t nA = ns == 3 ? (uint64_t)desc->slot_sizes[sb] * desc->slot_sizes[sb + 1] : desc->slot_sizes[sb];
    if (nA > 0xffffffffull) {
      delete L;
      return set_error(APEX_E_INVALID, "reaction %u: first slots exceed 2^32 - 1 combinations", t);
    }
    L->id_off.push_back(total);
    if ((unsigned __int128)total + cnt > (unsigned __int128)UINT64_MAX) {
      delete L;
      return set_error(APEX_E_INVALID, "compound count overflows 64 bits");
    }
    total += (uint64_t)cnt;
    sb += ns;
  }
  if (rows > 0xffffffffull) {
    delete L;
    return set_error(APEX_E_INVALID, "more than 2^32 - 1 table rows");
  }
  L->id_off.push_back(total);
  L->rows = rows;
  L->total = total;
  *out = L;
  return APEX_OK;
}

extern "C" apex_status apex_library_destroy(apex_library* lib) {
  delete lib;
  return APEX_OK;
}

extern "C" apex_status apex_library_num_compounds(const apex_library* lib, uint64_t* out) {
  if (!lib || !out) return set_error(APEX_E_INVALID, "null argument");
  *out = lib->total;
  return APEX_OK;
}

extern "C" apex_status apex_decode_ids(const apex_library* lib, const uint64_t* ids, size_t n, uint32_t* reaction,
                                       uint32_t* synthon) {
  if (!lib || (n && (!ids || !reaction || !synthon))) return set_error(APEX_E_INVALID, "null argument");
  for (size_t q = 0; q < n; ++q) {
    const uint64_t id = ids[q];
    if (id >= lib->total) return set_error(APEX_E_INVALID, "id %llu out of range", (unsigned long long)id);
    const uint32_t t = (uint32_t)(std::upper_bound(lib->id_off.begin(), lib->id_off.end(), id) -
                                  lib->id_off.begin()) - 1;
    uint64_t r = id - lib->id_off[t];
    const uint32_t ns = lib->n_slots[t];
    uint32_t idx[3] = {0, 0, 0};
    for (int s = (int)ns - 1; s >= 0; --s) {
      const uint64_t m = lib->slot_sizes[lib->slot_base[t] + s];
      idx[s] = (uint32_t)(r % m);
      r /= m;
    }
    reaction[q] = t;
    for (int s = 0; s < 3; ++s) synthon[3 * q + s] = idx[s];
  }
  return APEX_OK;
}

// ---------------------------------------------------------------------------
// associative embeddings (Section 4.2, eq. "assoc_embeds")
// ---------------------------------------------------------------------------
extern "C" apex_status apex_assoc_workspace_size(const apex_library* lib, size_t* bytes) {
  if (!lib || !bytes) return set_error(APEX_E_INVALID, "null argument");
  *bytes = (sizeof(AssocSlot) * lib->slot_sizes.size() + 255) & ~(size_t)255;
  return APEX_OK;
}

extern "C" apex_status apex_assoc_embeddings(const apex_library* lib, uint32_t dU, const float* keys,
                                             const float* values, float* out, void* workspace, size_t workspace_bytes,
                                             void* stream) {
  if (!lib || !keys || !values || !out || !workspace) return set_error(APEX_E_INVALID, "null argument");
  if (dU == 0 || dU > APEX_MAX_ASSOC_DU) return set_error(APEX_E_UNSUPPORTED, "dU = %u (1..%d)", dU, APEX_MAX_ASSOC_DU);
  size_t need = 0;
  apex_assoc_workspace_size(lib, &need);
  if (workspace_bytes < need) return set_error(APEX_E_NOMEM, "workspace %zu bytes < %zu needed", workspace_bytes, need);
  if (((uintptr_t)workspace) & 255) return set_error(APEX_E_INVALID, "workspace must be 256-byte aligned");
  const size_t ns = lib->slot_sizes.size();
  std::vector<AssocSlot> slots(ns);
  uint64_t tiles = 0;
  for (size_t j = 0; j < ns; ++j) {
    slots[j].row0 = lib->row_base[j];
    slots[j].n = lib->slot_sizes[j];
    slots[j].tile0 = tiles;
    tiles += (lib->slot_sizes[j] + 15) / 16;
  }
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, n_cu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  auto* dslots = reinterpret_cast<AssocSlot*>(workspace);
  HIP_TRY(hipMemcpyAsync(dslots, slots.data(), sizeof(AssocSlot) * ns, hipMemcpyHostToDevice, s));
  HIP_TRY(launch_assoc(dslots, (uint32_t)ns, tiles, lib->d, dU, keys, values, out, n_cu, s));
  HIP_TRY(hipStreamSynchronize(s));
  return APEX_OK;
}

// ---------------------------------------------------------------------------
// decoder
// ---------------------------------------------------------------------------
extern "C" apex_status apex_decoder_create(const apex_decoder_desc* desc, apex_decoder** out) {
  if (!desc || !out || !desc->dims || !desc->W || !desc->b) return set_error(APEX_E_INVALID, "null argument");
  *out = nullptr;
  const uint32_t L = desc->n_layers;
  if (L < 1 || L > 3) return set_error(APEX_E_INVALID, "n_layers must be 1, 2 or 3");
  if (desc->act > APEX_ACT_SILU) return set_error(APEX_E_INVALID, "unknown activation %u", desc->act);
  for (uint32_t l = 0; l <= L; ++l)
    if (desc->dims[l] == 0) return set_error(APEX_E_INVALID, "dims[%u] is 0", l);
  for (uint32_t l = 0; l < L; ++l)
    if (!desc->W[l] || !desc->b[l]) return set_error(APEX_E_INVALID, "layer %u has a null pointer", l);
  const uint32_t H = desc->dims[L];
  if (H > APEX_MAX_HEADS) return set_error(APEX_E_UNSUPPORTED, "H = %u > %d heads", H, APEX_MAX_HEADS);
  if (L >= 2 && H > APEX_MAX_MLP_HEADS)
    return set_error(APEX_E_UNSUPPORTED, "H = %u > %d heads for a decoder with hidden layers", H, APEX_MAX_MLP_HEADS);
  const uint32_t h1 = desc->dims[1];
  if (L >= 2 && h1 != 128 && h1 != 256 && h1 != 512)
    return set_error(APEX_E_UNSUPPORTED, "first hidden width %u (128, 256 or 512 supported)", h1);
  if (L == 3 && (desc->dims[2] % 32 != 0 || desc->dims[2] > 512))
    return set_error(APEX_E_UNSUPPORTED, "second hidden width %u (multiple of 32, <= 512)", desc->dims[2]);
  auto* D = new apex_decoder();
  D->L = L;
  D->act = desc->act;
  D->dims.assign(desc->dims, desc->dims + L + 1);
  D->W.assign(desc->W, desc->W + L);
  D->b.assign(desc->b, desc->b + L);
  *out = D;
  return APEX_OK;
}

extern "C" apex_status apex_decoder_destroy(apex_decoder* dec) {
  delete dec;
  return APEX_OK;
}

// ---------------------------------------------------------------------------
// engine workspace layout
// ---------------------------------------------------------------------------
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

constexpr uint32_t kCalSamples = 8192;

float act_prescale(uint32_t act) { return act == APEX_ACT_SILU ? -1.4426950408889634f : 1.0f; }

int elem_bytes(int p) { return p == APEX_PREC_FP32 ? 4 : (p == APEX_PREC_BF16 ? 2 : 1); }

// Width of the hoisted rows: the first hidden layer, or, for a one-layer
// (linear-probe) decoder, the heads padded to 16 (32 above 16 heads).
uint32_t heads_stride(uint32_t H) { return H <= (uint32_t)kHeadsPad ? (uint32_t)kHeadsPad : (uint32_t)kScalarHeads; }
uint32_t hoist_width(const apex_decoder* D) { return D->L == 1 ? heads_stride(D->dims[1]) : D->dims[1]; }

void engine_layout(apex_engine* E, const apex_library* L, const apex_decoder* D, uint32_t mask, Bump& b) {
  const uint32_t H1 = hoist_width(D);
  const uint32_t H2 = D->L == 3 ? D->dims[2] : 0;
  const uint32_t nslots = (uint32_t)L->slot_sizes.size();
  E->P = b.take<float>((size_t)L->rows * H1);
  E->react = b.take<ReactDev>(L->T);
  E->is_slot0 = b.take<uint8_t>(L->rows);
  E->slot_row0 = b.take<uint64_t>(nslots);
  E->slot_size = b.take<uint32_t>(nslots);
  E->react_slot0 = b.take<uint32_t>(L->T);
  E->react_nslots = b.take<uint32_t>(L->T);
  E->cmax = b.take<float>((size_t)nslots * H1);
  E->cmin = b.take<float>((size_t)nslots * H1);
  E->cal_ids = b.take<uint64_t>(kCalSamples);
  E->cal_h32 = b.take<float>((size_t)kCalSamples * kHeadsPad);
  E->cal_hlp = b.take<float>((size_t)kCalSamples * kHeadsPad);
  E->qnt_ids = b.take<uint64_t>(APEX_MAX_QUANTILE_COMPOUNDS);
  E->qnt_heads = b.take<float>((size_t)APEX_MAX_QUANTILE_COMPOUNDS * kScalarHeads);
  E->qnt_levels = b.take<float>(APEX_MAX_QUANTILE_LEVELS);
  E->qnt_out = b.take<float>((size_t)APEX_MAX_QUANTILE_LEVELS * kScalarHeads);
  for (int p = 0; p < 3; ++p) {
    PrecState& S = E->prec[p];
    S.on = (mask >> p) & 1u;
    if (!S.on) continue;
    const int eb = elem_bytes(p);
    // FP32 runs the 16x16 kernel (16 padded heads), BF16/FP8 the 32x32 one (32)
    const size_t head_rows = p == APEX_PREC_FP32 ? 16 : 32;
    // the 32x32 kernel runs GEMM chunks in pairs: its width is padded to 64
    // with zero neurons (zero weights, zero start value, zero output weights)
    S.h2k = p == APEX_PREC_FP32 ? H2 : (H2 + 63) / 64 * 64;
    if (D->L == 3) {
      S.w2 = b.take<uint8_t>((size_t)S.h2k * H1 * eb);
      S.wo = b.take<uint8_t>(head_rows * S.h2k * (p == APEX_PREC_FP32 ? 4 : 2));
      S.b2 = b.take<float>(S.h2k);
    } else {
      S.w2 = nullptr;
      S.wo = b.take<uint8_t>(head_rows * H1 * eb);
      S.b2 = nullptr;
    }
    S.bo = b.take<float>(kHeadsPad);
    S.scal = b.take<float>(8);
    S.amax = b.take<float>(4);
    S.herr = b.take<float>(kHeadsPad);
    S.plan = b.take<SelDev>(L->T);
  }
}

}  // namespace

// Tile plan: the selected reactions in order, with their first tile and first
// compound in the pass.
void apex::build_plan(const apex_library* L, bool scalar, const std::vector<uint32_t>& reactions,
                      std::vector<SelDev>& plan, uint64_t* n_tiles, uint64_t* n_compounds) {
  const uint32_t TA = tile_ta(scalar), TB = tile_tb(scalar);
  plan.clear();
  uint64_t tiles = 0, comps = 0;
  for (uint32_t t : reactions) {
    const uint32_t sb = L->slot_base[t];
    const uint32_t ns = L->n_slots[t];
    const uint64_t nA = ns == 3 ? (uint64_t)L->slot_sizes[sb] * L->slot_sizes[sb + 1] : L->slot_sizes[sb];
    const uint64_t nB = L->slot_sizes[sb + ns - 1];
    SelDev s{};
    s.tile_start = tiles;
    s.compound_start = comps;
    s.t = t;
    s.tiles_b = (uint32_t)((nB + TB - 1) / TB);
    plan.push_back(s);
    tiles += ((nA + TA - 1) / TA) * s.tiles_b;
    comps += nA * nB;
  }
  *n_tiles = tiles;
  *n_compounds = comps;
}

extern "C" apex_status apex_engine_workspace_size(const apex_library* lib, const apex_decoder* dec,
                                                  uint32_t precisions, size_t* bytes) {
  if (!lib || !dec || !bytes) return set_error(APEX_E_INVALID, "null argument");
  if (precisions == 0 || (precisions & ~7u)) return set_error(APEX_E_INVALID, "precisions mask 0x%x", precisions);
  if (dec->dims[0] != lib->d) return set_error(APEX_E_INVALID, "decoder input %u != library d %u", dec->dims[0], lib->d);
  if (dec->L == 1 && (precisions & ~APEX_PREC_MASK(APEX_PREC_FP32)))
    return set_error(APEX_E_UNSUPPORTED, "a one-layer decoder has no matrix layer: FP32 only");
  apex_engine tmp;
  Bump b(nullptr);
  engine_layout(&tmp, lib, dec, precisions | APEX_PREC_MASK(APEX_PREC_FP32), b);
  *bytes = b.off;
  return APEX_OK;
}

apex_status apex::engine_gather(apex_engine* E, int prec, const uint64_t* ids, uint32_t n, float* heads,
                                hipStream_t s, uint32_t out_stride) {
  if (n == 0) return APEX_OK;
  if (E->scalar) {
    HIP_TRY(launch_lin_heads(E->P, E->HS, E->react, E->lib->T, E->lib->total, ids, n, heads,
                             out_stride ? out_stride : E->HS, s));
    return APEX_OK;
  }
  if (out_stride && out_stride != (uint32_t)kHeadsPad)
    return set_error(APEX_E_INVALID, "internal: heads stride %u", out_stride);
  const PrecState& S = E->prec[prec];
  EnumArgs a{};
  a.P = E->P;
  a.react = E->react;
  a.pd = S.dev;
  a.H2 = E->prec[prec].h2k;
  a.ids = ids;
  a.n_ids = n;
  a.n_reactions = E->lib->T;
  a.n_total = E->lib->total;
  a.heads_out = heads;
  const uint32_t per = gather_per_block(prec, (int)E->NL);
  const uint32_t grid = (n + per - 1) / per;
  HIP_TRY(launch_enum(prec, E->H1, E->NL, E->act, true, a, grid, s));
  return APEX_OK;
}

extern "C" apex_status apex_engine_create(apex_library* lib, apex_decoder* dec, uint32_t precisions, void* workspace,
                                          size_t workspace_bytes, void* stream, apex_engine** out) {
  if (!lib || !dec || !out || !workspace) return set_error(APEX_E_INVALID, "null argument");
  *out = nullptr;
  size_t need = 0;
  apex_status st = apex_engine_workspace_size(lib, dec, precisions, &need);
  if (st != APEX_OK) return st;
  if (workspace_bytes < need)
    return set_error(APEX_E_NOMEM, "engine workspace %zu bytes < %zu needed", workspace_bytes, need);
  if (((uintptr_t)workspace) & 255) return set_error(APEX_E_INVALID, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  auto* E = new apex_engine();
  E->lib = lib;
  E->scalar = dec->L == 1;
  E->HS = E->scalar ? heads_stride(dec->dims[1]) : (uint32_t)kHeadsPad;
  E->H1 = hoist_width(dec);
  E->H2 = dec->L == 3 ? dec->dims[2] : 0;
  E->NL = dec->L - 1;
  E->H = dec->dims[dec->L];
  E->act = dec->L == 1 ? (uint32_t)APEX_ACT_NONE : dec->act;  // no activation without a hidden layer
  E->c_act = act_prescale(E->act);
  E->dims = dec->dims;
  E->mask = precisions | APEX_PREC_MASK(APEX_PREC_FP32);
  E->user_mask = precisions;
  {
    Bump b(workspace);
    engine_layout(E, lib, dec, E->mask, b);
  }
  auto fail = [&](apex_status code) {
    delete E;
    return code;
  };
  hipError_t he = hipGetDevice(&E->device);
  if (he == hipSuccess) he = hipDeviceGetAttribute(&E->n_cu, hipDeviceAttributeMultiprocessorCount, E->device);
  if (he != hipSuccess) return fail(set_error(APEX_E_DEVICE, "device query: %s", hipGetErrorString(he)));

  // host-side descriptors
  const uint32_t T = lib->T, nslots = (uint32_t)lib->slot_sizes.size();
  std::vector<ReactDev> rd(T);
  std::vector<uint8_t> s0(lib->rows, 0);
  std::vector<uint64_t> srow(nslots);
  std::vector<uint32_t> ssz(nslots), rs0(T), rns(T);
  for (uint32_t j = 0; j < nslots; ++j) {
    srow[j] = lib->row_base[j];
    ssz[j] = lib->slot_sizes[j];
  }
  for (uint32_t t = 0; t < T; ++t) {
    const uint32_t sb = lib->slot_base[t], ns = lib->n_slots[t];
    ReactDev r{};
    r.id_off = lib->id_off[t];
    r.row0 = (uint32_t)lib->row_base[sb];
    r.row1 = (uint32_t)lib->row_base[sb + 1];
    r.rowB = (uint32_t)lib->row_base[sb + ns - 1];
    r.n1 = lib->slot_sizes[sb + 1];
    r.three = ns == 3;
    r.nA = ns == 3 ? lib->slot_sizes[sb] * lib->slot_sizes[sb + 1] : lib->slot_sizes[sb];
    r.nB = lib->slot_sizes[sb + ns - 1];
    rd[t] = r;
    rs0[t] = sb;
    rns[t] = ns;
    for (uint32_t i = 0; i < lib->slot_sizes[sb]; ++i) s0[lib->row_base[sb] + i] = 1;
  }
  E->react_host = rd;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  };
  he = up(E->react, rd.data(), sizeof(ReactDev) * T);
  if (he == hipSuccess) he = up(E->is_slot0, s0.data(), s0.size());
  if (he == hipSuccess) he = up(E->slot_row0, srow.data(), sizeof(uint64_t) * nslots);
  if (he == hipSuccess) he = up(E->slot_size, ssz.data(), sizeof(uint32_t) * nslots);
  if (he == hipSuccess) he = up(E->react_slot0, rs0.data(), sizeof(uint32_t) * T);
  if (he == hipSuccess) he = up(E->react_nslots, rns.data(), sizeof(uint32_t) * T);
  if (he != hipSuccess) return fail(set_error(APEX_E_DEVICE, "upload: %s", hipGetErrorString(he)));

  // hoist of the first layer (with its bias on slot-0 rows) and the activation prescale
  he = launch_hoist(lib->tables, lib->d, lib->rows, dec->W[0], dec->b[0], dec->dims[1], E->H1, E->is_slot0,
                    E->c_act, E->P, s);
  if (he != hipSuccess) return fail(set_error(APEX_E_DEVICE, "hoist: %s", hipGetErrorString(he)));

  const float* W2 = dec->L == 3 ? dec->W[1] : nullptr;
  const float* b2 = dec->L == 3 ? dec->b[1] : nullptr;
  const float* Wo = dec->W[dec->L - 1];
  const float* bo = dec->b[dec->L - 1];
  std::vector<uint32_t> all(T);
  for (uint32_t t = 0; t < T; ++t) all[t] = t;
  const bool need_range = (E->mask >> APEX_PREC_FP8) & 1u;
  for (int p = 0; p < 3; ++p) {
    PrecState& S = E->prec[p];
    if (!S.on) continue;
    std::vector<float> zero4(4, 0.0f);
    he = up(S.amax, zero4.data(), 4 * sizeof(float));
    if (he == hipSuccess && p == APEX_PREC_FP8 && need_range) {
      he = launch_act_range(E->P, E->H1, E->slot_row0, E->slot_size, nslots, E->react_slot0, E->react_nslots, T,
                            (int)E->act, E->c_act, E->cmax, E->cmin, S.amax + 0, s);
      if (he == hipSuccess && W2) he = launch_absmax(W2, (uint64_t)E->H2 * E->H1, S.amax + 1, s);
      if (he == hipSuccess) he = launch_absmax(Wo, (uint64_t)E->H * (E->NL == 2 ? E->H2 : E->H1), S.amax + 2, s);
    }
    if (he == hipSuccess) he = launch_scales(S.amax, p, E->NL, S.scal, s);
    if (he == hipSuccess) {
      if (E->NL == 2) {
        if (p == APEX_PREC_FP32) {
          he = launch_frag_x(W2, E->H2, E->H1, E->H2 / 16, 1.0f, S.w2, s);
          if (he == hipSuccess) he = launch_frag_out_d(Wo, E->H, E->H2, 1.0f / E->c_act, S.wo, s);
        } else {
          he = launch_frag_x32(p, W2, E->H2, E->H1, S.h2k / 32, p == APEX_PREC_FP8 ? S.scal + 3 : nullptr, 1.0f,
                               S.w2, s);
          if (he == hipSuccess) he = launch_frag_out32(Wo, E->H, E->H2, S.h2k, 1.0f / E->c_act, S.wo, s);
        }
        if (he == hipSuccess) he = launch_bias(b2, E->H2, S.h2k, E->c_act, S.scal, bo, E->H, S.b2, S.bo, s);
      } else if (E->NL == 1) {
        if (p == APEX_PREC_FP32)
          he = launch_frag_x(Wo, E->H, E->H1, 1, 1.0f / E->c_act, S.wo, s);
        else
          he = launch_frag_x32(p, Wo, E->H, E->H1, 1, p == APEX_PREC_FP8 ? S.scal + 4 : nullptr, 1.0f / E->c_act,
                               S.wo, s);
        if (he == hipSuccess) he = launch_bias(nullptr, 0, 0, E->c_act, S.scal, bo, E->H, nullptr, S.bo, s);
      } else {  // linear decoder: its bias is already in the slot-0 rows
        he = launch_bias(nullptr, 0, 0, 1.0f, S.scal, nullptr, 0, nullptr, S.bo, s);
      }
    }
    if (he != hipSuccess) return fail(set_error(APEX_E_DEVICE, "weight preparation: %s", hipGetErrorString(he)));
    S.dev.w2 = S.w2;
    S.dev.wo = S.wo;
    S.dev.b2 = S.b2;
    S.dev.bo = S.bo;
    S.dev.scal = S.scal;
    S.dev.delta = S.herr;
    std::vector<SelDev> plan;
    build_plan(lib, E->scalar, all, plan, &S.full_tiles, &S.full_compounds);
    he = up(S.plan, plan.data(), sizeof(SelDev) * plan.size());
    if (E->scalar) {
      if (he == hipSuccess) he = scan_prepare(&S.wg_per_cu);
    } else {
      if (he == hipSuccess) he = enum_prepare(p, E->H1, E->NL, (int)E->act, false, S.h2k, &S.wg_per_cu);
      if (he == hipSuccess) he = enum_prepare(p, E->H1, E->NL, (int)E->act, true, S.h2k, nullptr);
    }
    if (he != hipSuccess) return fail(set_error(APEX_E_DEVICE, "kernel setup: %s", hipGetErrorString(he)));
    if (S.wg_per_cu < 1) return fail(set_error(APEX_E_UNSUPPORTED, "fused kernel does not fit on a CU"));
  }

  // Low-precision relaxation: largest |head error| against FP32 over a
  // stratified sample of the library (linear-probe engines are FP32 only).
  const uint32_t ncal = E->scalar ? 0u : (uint32_t)std::min<uint64_t>(kCalSamples, lib->total);
  he = launch_sample_ids(E->prec[APEX_PREC_FP32].plan, T, E->react, lib->total, ncal, 0x5eed1234ull, E->cal_ids, s);
  if (he != hipSuccess) return fail(set_error(APEX_E_DEVICE, "calibration sample: %s", hipGetErrorString(he)));
  st = engine_gather(E, APEX_PREC_FP32, E->cal_ids, ncal, E->cal_h32, s);
  if (st != APEX_OK) return fail(st);
  for (int p = 1; p < 3; ++p) {
    PrecState& S = E->prec[p];
    if (!S.on) continue;
    std::vector<float> z(kHeadsPad, 0.0f);
    he = up(S.herr, z.data(), sizeof(float) * kHeadsPad);
    if (he != hipSuccess) return fail(set_error(APEX_E_DEVICE, "upload: %s", hipGetErrorString(he)));
    st = engine_gather(E, p, E->cal_ids, ncal, E->cal_hlp, s);
    if (st != APEX_OK) return fail(st);
    he = launch_head_err(E->cal_hlp, E->cal_h32, ncal, S.herr, s);
    if (he == hipSuccess)
      he = hipMemcpyAsync(S.delta, S.herr, sizeof(float) * kHeadsPad, hipMemcpyDeviceToHost, s);
    if (he != hipSuccess) return fail(set_error(APEX_E_DEVICE, "calibration: %s", hipGetErrorString(he)));
  }
  for (int p = 0; p < 3; ++p)
    if (E->prec[p].on) {
      he = hipMemcpyAsync(E->prec[p].scal_host, E->prec[p].scal, sizeof(float) * 8, hipMemcpyDeviceToHost, s);
      if (he != hipSuccess) return fail(set_error(APEX_E_DEVICE, "readback: %s", hipGetErrorString(he)));
    }
  he = hipStreamSynchronize(s);
  if (he != hipSuccess) return fail(set_error(APEX_E_DEVICE, "engine build: %s", hipGetErrorString(he)));
  // The margin is 1.25 x the largest error seen on the sample (about its
  // 99.99th percentile): a true answer is lost only if its own error exceeds it.
  for (int p = 1; p < 3; ++p)
    for (int h = 0; h < kHeadsPad; ++h) E->prec[p].delta[h] *= 1.25f;
  *out = E;
  return APEX_OK;
}

extern "C" apex_status apex_engine_destroy(apex_engine* eng) {
  delete eng;
  return APEX_OK;
}

extern "C" apex_status apex_engine_head_quantiles(apex_engine* eng, const uint64_t* ids, uint32_t n,
                                                  const float* levels, uint32_t n_levels, float* out, void* stream) {
  if (!eng || !levels || !out) return set_error(APEX_E_INVALID, "null argument");
  if (n == 0 || n > APEX_MAX_QUANTILE_COMPOUNDS)
    return set_error(APEX_E_INVALID, "n = %u compounds (1..%d)", n, APEX_MAX_QUANTILE_COMPOUNDS);
  if (n_levels == 0 || n_levels > APEX_MAX_QUANTILE_LEVELS)
    return set_error(APEX_E_INVALID, "n_levels = %u (1..%d)", n_levels, APEX_MAX_QUANTILE_LEVELS);
  for (uint32_t l = 0; l < n_levels; ++l)
    if (!(levels[l] >= 0.0f && levels[l] <= 1.0f)) return set_error(APEX_E_INVALID, "level %u outside [0, 1]", l);
  hipStream_t s = (hipStream_t)stream;
  apex_engine* E = eng;
  const uint64_t* dev_ids = ids;
  if (!ids) {
    HIP_TRY(launch_sample_ids(E->prec[APEX_PREC_FP32].plan, E->lib->T, E->react, E->lib->total, n, 0x9e3779b1ull,
                              E->qnt_ids, s));
    dev_ids = E->qnt_ids;
  }
  apex_status st = engine_gather(E, APEX_PREC_FP32, dev_ids, n, E->qnt_heads, s);
  if (st != APEX_OK) return st;
  HIP_TRY(hipMemcpyAsync(E->qnt_levels, levels, sizeof(float) * n_levels, hipMemcpyHostToDevice, s));
  HIP_TRY(launch_head_quantiles(E->qnt_heads, E->HS, n, E->qnt_levels, n_levels, E->H, E->qnt_out, s));
  HIP_TRY(hipMemcpyAsync(out, E->qnt_out, sizeof(float) * n_levels * E->H, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return APEX_OK;
}

extern "C" apex_status apex_engine_heads(apex_engine* eng, const uint64_t* ids, uint32_t n, uint32_t precision,
                                         float* heads, void* stream) {
  if (!eng || (n && (!ids || !heads))) return set_error(APEX_E_INVALID, "null argument");
  if (precision > APEX_PREC_FP8 || !eng->prec[precision].on)
    return set_error(APEX_E_INVALID, "precision %u not enabled in this engine", precision);
  return engine_gather(eng, (int)precision, ids, n, heads, (hipStream_t)stream);
}
