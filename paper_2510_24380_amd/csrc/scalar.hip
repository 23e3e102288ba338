// The paper's own search path for a linear probe (Section 4.3, eq. "apex";
// Appendix A.5): every head of a compound is the sum of its synthons' scalar
// contributions v_{i,r,s} (the hoisted rows of a one-layer decoder, bias on
// slot 0), so a query's objective and constrained heads are sums of per-row
// scalars. Per query, one pass over the synthon rows builds those scalars
// (k_qtab); the enumeration then spends one add and one compare per compound
// on the objective (k_scan), and evaluates the constrained heads only for
// compounds whose objective reaches the query's threshold.
//
// Arithmetic shared by every kernel here, so that a compound's objective and
// heads are the same bits wherever they are computed: a row's objective
// contribution is fma-accumulated over heads 0..H-1 in order; a compound's
// value is (slot 0 + slot 1) + slot 2 for three slots and slot 0 + slot 1 for
// two, in FP32.
#include "enum_common.h"
#include "launch.h"

namespace apex {

// ---------------------------------------------------------------------------
// Per-query row tables.
// ---------------------------------------------------------------------------
// One thread per row; the row is read as HS / 4 16-byte pieces and the
// weights come from LDS (the same fma order over heads 0..H-1).
template <int HS>
__global__ __launch_bounds__(256) void k_qtab(const float* __restrict__ V, uint64_t rows, uint32_t H,
                                              const ScalarQuery* __restrict__ sq) {
  __shared__ float w[HS];
  __shared__ uint32_t head[APEX_MAX_CONSTRAINTS];
  if (threadIdx.x < HS) w[threadIdx.x] = threadIdx.x < H ? sq->w[threadIdx.x] : 0.0f;
  if (threadIdx.x < APEX_MAX_CONSTRAINTS) head[threadIdx.x] = sq->head[threadIdx.x];
  __syncthreads();
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const float4* v4 = reinterpret_cast<const float4*>(V + r * HS);
  float o = 0.0f;
  bool fin = true;
#pragma unroll
  for (int q = 0; q < HS / 4; ++q) {
    const float4 x = v4[q];
    const float xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t h = 4 * q + e;
      if (h < H) {
        fin = fin && finite_obj(xs[e]);
        o = fmaf(w[h], xs[e], o);
      }
    }
  }
  float* tab = sq->tab;
  tab[r] = fin ? o : __builtin_nanf("");
  const uint32_t nch = sq->n_ch;
  const float* v = V + r * HS;
  for (uint32_t c = 0; c < nch; ++c) tab[(uint64_t)(c + 1) * rows + r] = v[head[c]];
}

// ---------------------------------------------------------------------------
// Helpers
// ---------------------------------------------------------------------------
// Table value of the A side (slot 0, or slots 0 and 1) of assignment a.
__device__ __forceinline__ float a_value(const float* __restrict__ col, const ReactDev& R, uint32_t a) {
  if (R.three) {
    const uint32_t i0 = a / R.n1, i1 = a - i0 * R.n1;
    return col[R.row0 + i0] + col[R.row1 + i1];
  }
  return col[R.row0 + a];
}

// Every constrained head of compound (a, b) within its bounds.
__device__ __forceinline__ bool scalar_feasible(const ScalarQuery* __restrict__ sq, const ReactDev& R, uint32_t a,
                                                uint32_t b) {
  const uint32_t nch = sq->n_ch;
  const uint64_t rows = sq->rows;
  bool ok = true;
  for (uint32_t c = 0; c < nch && ok; ++c) {
    const float* col = sq->tab + (uint64_t)(c + 1) * rows;
    const float h = a_value(col, R, a) + col[R.rowB + b];
    ok = h >= sq->lo[c] && h <= sq->hi[c];
  }
  return ok;
}

// Wave-uniform copies of values every lane holds alike (tile and query
// metadata), so the tile loop's control flow and addresses stay scalar.
__device__ __forceinline__ uint32_t uni32(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
  return ((uint64_t)uni32((uint32_t)(x >> 32)) << 32) | uni32((uint32_t)x);
}
__device__ __forceinline__ float unif(float x) { return __uint_as_float(uni32(__float_as_uint(x))); }
template <class T>
__device__ __forceinline__ T* uni_ptr(T* p) {
  return reinterpret_cast<T*>(uni64(reinterpret_cast<uint64_t>(p)));
}

// Violation of compound (a, b), c = -(sum over constraints of max(0, lo - f) +
// max(0, f - hi)), accumulated in constraint order (Section 4.3).
__device__ __forceinline__ float scalar_violation(const ScalarQuery* __restrict__ sq, const ReactDev& R, uint32_t a,
                                                  uint32_t b) {
  const uint32_t nch = sq->n_ch;
  const uint64_t rows = sq->rows;
  float acc = 0.0f;
  for (uint32_t c = 0; c < nch; ++c) {
    const float* col = sq->tab + (uint64_t)(c + 1) * rows;
    const float h = a_value(col, R, a) + col[R.rowB + b];
    acc = acc + fmaxf(0.0f, sq->lo[c] - h);
    acc = acc + fmaxf(0.0f, h - sq->hi[c]);
  }
  return -acc;
}

// Appends (o, id) of the lanes with pass set: one atomic per wave.
__device__ __forceinline__ void wave_append(const QueryDev& Q, bool pass, float o, uint64_t id, int lane) {
  const uint64_t m = __ballot(pass);
  if (!m) return;
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(&Q.st->count, (uint32_t)__popcll(m));
  base = __shfl(base, 0);
  if (pass) {
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint32_t idx = base + (uint32_t)__popcll(m & below);
    if (idx < Q.cap) {
      Q.cand_o[idx] = o;
      Q.cand_id[idx] = id;
    }
  }
}

// ---------------------------------------------------------------------------
// Enumeration. One wave per tile of kScalarTA A rows x 64 B rows; lane l holds
// B row b0 + l in a register and takes the tile's A values one at a time from a
// wave-private LDS row (a broadcast read). Per compound: one add and one max;
// a group of 16 A rows whose best sum reaches the threshold is re-run with the
// exact key order, the bounds and the append. Each wave takes a contiguous run
// of tiles, so the reaction lookup is a step forward, not a search, and a run
// of tiles sharing their A rows stages them once (one query per launch).
// The queries' parameters are copied to LDS once per launch (the threshold
// does not change during a launch; selections run between launches). In the
// exact pass the bounds of up to kScanLdsBounds constrained heads are checked
// from LDS: the tile's B-side values of those heads are staged once (on the
// tile's first group that reaches the threshold), the group's A-side values per
// group; queries with more constrained heads read the tables directly.
// ---------------------------------------------------------------------------
constexpr int kScanWaves = 4;
constexpr int kScanGroup = 16;
constexpr int kScanLdsBounds = 8;
constexpr uint32_t kScanOut = 128;  // per-wave append buffer (entries)

// Appends gathered in a wave-private LDS buffer and written to the query's
// candidate buffer with one atomic per flush: the hits of a large-k search are
// spread thinly over the whole library, and one atomic per hit on the query's
// single counter would serialise them.
struct WaveOut {
  float* o;
  uint64_t* id;
  uint32_t n;
  __device__ void flush(const QueryDev& Q, int lane) {
    if (n == 0) return;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(&Q.st->count, n);
    base = __shfl(base, 0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (uint32_t i = (uint32_t)lane; i < n; i += 64) {
      const uint32_t idx = base + i;
      if (idx < Q.cap) {
        Q.cand_o[idx] = o[i];
        Q.cand_id[idx] = id[i];
      }
    }
    __builtin_amdgcn_wave_barrier();
    n = 0;
  }
  __device__ void append(const QueryDev& Q, bool pass, float ov, uint64_t iv, int lane) {
    const uint64_t m = __ballot(pass);
    if (!m) return;
    const uint32_t c = (uint32_t)__popcll(m);
    if (n + c > kScanOut) flush(Q, lane);
    if (pass) {
      const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
      const uint32_t i = n + (uint32_t)__popcll(m & below);
      o[i] = ov;
      id[i] = iv;
    }
    n += c;
  }
};

struct ScanQ {
  const ScalarQuery* sq;
  const float* tab;
  const uint32_t* bits;
  float tau_o;
  uint32_t active;
  uint64_t tau_id;
  uint32_t viol;
  uint32_t n_ch;
  float lo[kScanLdsBounds];
  float hi[kScanLdsBounds];
};

__global__ __launch_bounds__(kScanWaves * 64) void k_scan(EnumArgs A) {
  __shared__ __attribute__((aligned(16))) float sA[kScanWaves][kScalarTA];
  __shared__ ScanQ sQ[APEX_MAX_FUSED_QUERIES];
  __shared__ float sBc[kScanWaves][kScanLdsBounds][64];          // B side of the bounded heads
  __shared__ float sAc[kScanWaves][kScanLdsBounds][kScanGroup];  // A side, one group
  __shared__ float sOutO[kScanWaves][kScanOut];
  __shared__ uint64_t sOutId[kScanWaves][kScanOut];
  const int lane = threadIdx.x & 63, wave = (int)uni32(threadIdx.x >> 6);
  const uint32_t nq = A.n_queries;
  if (threadIdx.x < nq) {
    const QueryDev& Q = A.queries[threadIdx.x];
    ScanQ L{};
    L.active = Q.active;
    if (L.active) {
      L.sq = Q.sq;
      L.tab = Q.sq->tab;
      L.bits = Q.subset_bits;
      L.tau_o = Q.st->tau_o;
      L.tau_id = Q.st->tau_id;
      L.viol = Q.sq->viol;
      L.n_ch = Q.sq->n_ch;
      for (int c = 0; c < kScanLdsBounds; ++c) {
        L.lo[c] = c < (int)L.n_ch ? Q.sq->lo[c] : 0.0f;
        L.hi[c] = c < (int)L.n_ch ? Q.sq->hi[c] : 0.0f;
      }
    }
    sQ[threadIdx.x] = L;
  }
  __syncthreads();
  // this wave's contiguous run of tiles
  const uint64_t n_waves = (uint64_t)gridDim.x * kScanWaves;
  const uint64_t n_tiles = A.tile_end - A.tile_begin;
  const uint64_t per = (n_tiles + n_waves - 1) / n_waves;
  uint64_t v = A.tile_begin + ((uint64_t)blockIdx.x * kScanWaves + wave) * per;
  const uint64_t vend = v + per < A.tile_end ? v + per : A.tile_end;
  if (v >= vend) return;
  float* row = sA[wave];
  WaveOut out{sOutO[wave], sOutId[wave], 0u};
  uint32_t out_q = 0;  // query whose hits the append buffer holds
  float (*bc)[64] = sBc[wave];
  float (*ac)[kScanGroup] = sAc[wave];
  uint32_t si = uni32(find_sel(A.sel, A.n_sel, v));
  SelDev S{};
  ReactDev R{};
  uint64_t s_end = 0;
  auto load_reaction = [&]() {
    S = A.sel[si];
    S.tile_start = uni64(S.tile_start);
    S.t = uni32(S.t);
    S.tiles_b = uni32(S.tiles_b);
    R = A.react[S.t];
    R.id_off = uni64(R.id_off);
    R.row0 = uni32(R.row0);
    R.row1 = uni32(R.row1);
    R.rowB = uni32(R.rowB);
    R.n1 = uni32(R.n1);
    R.nA = uni32(R.nA);
    R.nB = uni32(R.nB);
    R.three = uni32(R.three);
    s_end = S.tile_start + (uint64_t)((R.nA + kScalarTA - 1) / kScalarTA) * S.tiles_b;
  };
  load_reaction();
  uint64_t staged = ~0ull;  // (reaction, A block) whose A values sit in `row` (single query)
  for (; v < vend; ++v) {
    while (v >= s_end) {
      ++si;
      load_reaction();
    }
    const uint64_t lt = v - S.tile_start;
    const uint32_t ta = (uint32_t)(lt / S.tiles_b), tb = (uint32_t)(lt - (uint64_t)ta * S.tiles_b);
    const uint32_t a0 = ta * kScalarTA, b = tb * kScalarTB + (uint32_t)lane;
    const uint32_t na = min((uint32_t)kScalarTA, R.nA - a0);
    const bool b_ok = b < R.nB;
    const uint64_t key = ((uint64_t)si << 32) | ta;
    for (uint32_t qi = 0; qi < nq; ++qi) {
      const ScanQ& L = sQ[qi];
      if (!uni32(L.active)) continue;
      const uint32_t* bits = uni_ptr(L.bits);
      if (bits && !((uni32(bits[S.t >> 5]) >> (S.t & 31)) & 1u)) continue;
      const ScalarQuery* sq = uni_ptr(L.sq);
      const float* col0 = uni_ptr(L.tab);
      const float tau_o = unif(L.tau_o);
      const uint64_t tau_id = uni64(L.tau_id);
      const QueryDev& Q = A.queries[qi];
      if (out_q != qi) {  // the buffer holds one query's hits
        out.flush(A.queries[out_q], lane);
        out_q = qi;
      }
      const float bo = b_ok ? col0[R.rowB + b] : __builtin_nanf("");
      if (uni32(L.viol)) {
        // violation pass: every compound that violates a bound is ranked by its
        // violation (key) against the query's threshold; its objective only
        // needs to be finite
        for (uint32_t al = 0; al < na; ++al) {
          const uint32_t a = a0 + al;
          const float o = a_value(col0, R, a) + bo;
          bool pass = b_ok && finite_obj(o);
          float cv = 0.0f;
          if (pass) {
            cv = scalar_violation(sq, R, a, b);
            pass = cv < 0.0f;
          }
          const uint64_t id = R.id_off + (uint64_t)a * R.nB + b;
          pass = pass && key_passes(cv, id, tau_o, tau_id);
          wave_append(Q, pass, cv, id, lane);
        }
        continue;
      }
      // the row of A values (NaN past the reaction's edge: never passes)
      if (nq > 1 || staged != key) {
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int u = 0; u < kScalarTA / 64; ++u) {
          const uint32_t al = (uint32_t)(64 * u + lane);
          row[al] = al < na ? a_value(col0, R, a0 + al) : __builtin_nanf("");
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        staged = key;
      }
      const uint32_t nch = uni32(L.n_ch);
      const bool lds_bounds = nch <= (uint32_t)kScanLdsBounds;
      bool bc_staged = false;
      for (uint32_t g = 0; g < na; g += kScanGroup) {
        float mx = -__builtin_inff();
#pragma unroll
        for (int u = 0; u < kScanGroup; u += 4) {
          const float4 a4 = *reinterpret_cast<const float4*>(row + g + u);
          mx = fmaxf(mx, a4.x + bo);
          mx = fmaxf(mx, a4.y + bo);
          mx = fmaxf(mx, a4.z + bo);
          mx = fmaxf(mx, a4.w + bo);
        }
        if (__ballot(mx >= tau_o) == 0) continue;
        const uint32_t ge = min(g + kScanGroup, na);
        if (nch && lds_bounds) {
          // the bounded heads' values of this group's A rows (and, once per
          // tile, of the lane's B row) into LDS
          __builtin_amdgcn_wave_barrier();
          const uint64_t rows = sq->rows;
          if (!bc_staged) {
            for (uint32_t c = 0; c < nch; ++c)
              bc[c][lane] = b_ok ? col0[(uint64_t)(c + 1) * rows + R.rowB + b] : __builtin_nanf("");
            bc_staged = true;
          }
          for (uint32_t e = (uint32_t)lane; e < nch * kScanGroup; e += 64) {
            const uint32_t c = e / kScanGroup, u = e % kScanGroup;
            ac[c][u] = g + u < na ? a_value(col0 + (uint64_t)(c + 1) * rows, R, a0 + g + u) : __builtin_nanf("");
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
        }
        for (uint32_t al = g; al < ge; ++al) {
          const float o = canon_zero(row[al] + bo);
          bool pass = o >= tau_o;
          if (__ballot(pass) == 0) continue;
          const uint32_t a = a0 + al;
          const uint64_t id = R.id_off + (uint64_t)a * R.nB + b;
          pass = pass && finite_obj(o) && key_passes(o, id, tau_o, tau_id);
          if (lds_bounds) {
            for (uint32_t c = 0; c < nch; ++c) {
              const float hv = ac[c][al - g] + bc[c][lane];
              pass = pass && hv >= L.lo[c] && hv <= L.hi[c];
            }
          } else if (pass) {
            pass = scalar_feasible(sq, R, a, b);
          }
          out.append(Q, pass, o, id, lane);
        }
      }
    }
  }
  out.flush(A.queries[out_q], lane);
}

// Listed compounds (the threshold warm start's sample) scored for each query
// with the enumeration's arithmetic and appended if they pass; ids past the
// library's end are skipped.
// Append of a whole workgroup (every thread calls it once): one atomic on the
// query's counter per workgroup instead of one per wave. The warm-start sample
// is scored against an open threshold, so every listed compound appends, and
// per-wave atomics on the one counter serialise.
constexpr int kListThreads = 1024;
__device__ __forceinline__ void block_append(const QueryDev& Q, bool pass, float o, uint64_t id) {
  __shared__ uint32_t s_off[kListThreads / 64];
  __shared__ uint32_t s_base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t m = __ballot(pass);
  if (lane == 0) s_off[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t total = 0;
    for (int w = 0; w < kListThreads / 64; ++w) {
      const uint32_t c = s_off[w];
      s_off[w] = total;
      total += c;
    }
    s_base = total ? atomicAdd(&Q.st->count, total) : 0u;
  }
  __syncthreads();
  if (pass) {
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint32_t idx = s_base + s_off[wave] + (uint32_t)__popcll(m & below);
    if (idx < Q.cap) {
      Q.cand_o[idx] = o;
      Q.cand_id[idx] = id;
    }
  }
}

__global__ __launch_bounds__(kListThreads) void k_scan_list(const uint64_t* __restrict__ ids, uint32_t n,
                                                   const QueryDev* __restrict__ qs, uint32_t nq,
                                                   const ReactDev* __restrict__ react, uint32_t n_react,
                                                   uint64_t n_total) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t q = blockIdx.y;
  if (q >= nq) return;  // uniform per workgroup
  const QueryDev& Q = qs[q];
  if (!Q.active) return;
  bool pass = false;
  float o = 0.0f;
  uint64_t id = ~0ull;
  if (i < n) id = ids[i];
  if (id < n_total) {
    const uint32_t t = find_reaction(react, n_react, id);
    if (!Q.subset_bits || ((Q.subset_bits[t >> 5] >> (t & 31)) & 1u)) {
      const ReactDev R = react[t];
      const uint64_t loc = id - R.id_off;
      const uint32_t a = (uint32_t)(loc / R.nB), b = (uint32_t)(loc - (uint64_t)a * R.nB);
      const ScalarQuery* sq = Q.sq;
      o = canon_zero(a_value(sq->tab, R, a) + sq->tab[R.rowB + b]);
      if (sq->viol) {
        const bool fin = finite_obj(o);
        o = fin ? scalar_violation(sq, R, a, b) : 0.0f;  // the key of the violation pass
        pass = fin && o < 0.0f && key_passes(o, id, Q.st->tau_o, Q.st->tau_id);
      } else {
        pass = finite_obj(o) && key_passes(o, id, Q.st->tau_o, Q.st->tau_id) && scalar_feasible(sq, R, a, b);
      }
    }
  }
  block_append(Q, pass, o, id);  // every thread of the workgroup
}

// Answer of a violation pass: the sorted keys (violations) move to viol, and
// the objective of each listed compound is recomputed with the enumeration's
// arithmetic into obj. n = min(st->count, K) entries.
__global__ __launch_bounds__(256) void k_viol_answer(const ScalarQuery* __restrict__ sq,
                                                     const ReactDev* __restrict__ react, uint32_t n_react,
                                                     const uint64_t* __restrict__ ids, const QState* __restrict__ st,
                                                     uint32_t K, float* __restrict__ obj, float* __restrict__ viol) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= min(st->count, K)) return;
  const uint64_t id = ids[i];
  const uint32_t t = find_reaction(react, n_react, id);
  const ReactDev R = react[t];
  const uint64_t loc = id - R.id_off;
  const uint32_t a = (uint32_t)(loc / R.nB), b = (uint32_t)(loc - (uint64_t)a * R.nB);
  viol[i] = obj[i];
  obj[i] = canon_zero(a_value(sq->tab, R, a) + sq->tab[R.rowB + b]);
}

// FP32 heads of listed compounds, one thread per compound: heads[e * ho + h]
// for h < ho (columns past H are zero); an id past the library's end gives a
// row of NaN. V has hs >= ho columns.
__global__ __launch_bounds__(256) void k_lin_heads(const float* __restrict__ V, uint32_t hs,
                                                   const ReactDev* __restrict__ react, uint32_t n_react,
                                                   uint64_t n_total, const uint64_t* __restrict__ ids, uint32_t n,
                                                   float* __restrict__ heads, uint32_t ho) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const uint64_t id = ids[e];
  float* out = heads + (uint64_t)e * ho;
  if (id >= n_total) {
    for (uint32_t h = 0; h < ho; ++h) out[h] = __builtin_nanf("");
    return;
  }
  const uint32_t t = find_reaction(react, n_react, id);
  const ReactDev R = react[t];
  const uint64_t loc = id - R.id_off;
  const uint32_t a = (uint32_t)(loc / R.nB), b = (uint32_t)(loc - (uint64_t)a * R.nB);
  const float* vb = V + (uint64_t)(R.rowB + b) * hs;
  if (R.three) {
    const uint32_t i0 = a / R.n1, i1 = a - i0 * R.n1;
    const float* v0 = V + (uint64_t)(R.row0 + i0) * hs;
    const float* v1 = V + (uint64_t)(R.row1 + i1) * hs;
    for (uint32_t h = 0; h < ho; ++h) out[h] = (v0[h] + v1[h]) + vb[h];
  } else {
    const float* v0 = V + (uint64_t)(R.row0 + a) * hs;
    for (uint32_t h = 0; h < ho; ++h) out[h] = v0[h] + vb[h];
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_qtab(const float* V, uint32_t hs, uint64_t rows, uint32_t H, const ScalarQuery* sq,
                       hipStream_t s) {
  if (rows == 0) return hipSuccess;
  const dim3 grid((unsigned)((rows + 255) / 256)), block(256);
  if (hs == 16)
    hipLaunchKernelGGL(k_qtab<16>, grid, block, 0, s, V, rows, H, sq);
  else if (hs == 32)
    hipLaunchKernelGGL(k_qtab<32>, grid, block, 0, s, V, rows, H, sq);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t scan_prepare(int* max_wg_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(max_wg_per_cu, reinterpret_cast<const void*>(&k_scan),
                                                      kScanWaves * 64, 0);
}

hipError_t launch_scan(const EnumArgs& a, uint32_t grid_max, hipStream_t s) {
  const uint64_t nt = a.tile_end - a.tile_begin;
  if (nt == 0) return hipSuccess;
  const uint64_t want = (nt + kScanWaves - 1) / kScanWaves;
  const uint32_t grid = (uint32_t)(want < grid_max ? want : grid_max);
  hipLaunchKernelGGL(k_scan, dim3(grid), dim3(kScanWaves * 64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_scan_list(const uint64_t* ids, uint32_t n, const QueryDev* qs, uint32_t nq, const ReactDev* react,
                            uint32_t n_react, uint64_t n_total, hipStream_t s) {
  if (n == 0 || nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_list, dim3((n + kListThreads - 1) / kListThreads, nq), dim3(kListThreads), 0, s, ids, n,
                     qs, nq, react, n_react, n_total);
  return hipGetLastError();
}

hipError_t launch_viol_answer(const ScalarQuery* sq, const ReactDev* react, uint32_t n_react, const uint64_t* ids,
                              const QState* st, uint32_t K, float* obj, float* viol, hipStream_t s) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_viol_answer, dim3((K + 255) / 256), dim3(256), 0, s, sq, react, n_react, ids, st, K, obj, viol);
  return hipGetLastError();
}

hipError_t launch_lin_heads(const float* V, uint32_t hs, const ReactDev* react, uint32_t n_react, uint64_t n_total,
                            const uint64_t* ids, uint32_t n, float* heads, uint32_t ho, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (ho == 0 || ho > hs) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lin_heads, dim3((n + 255) / 256), dim3(256), 0, s, V, hs, react, n_react, n_total, ids, n,
                     heads, ho);
  return hipGetLastError();
}

}  // namespace apex
