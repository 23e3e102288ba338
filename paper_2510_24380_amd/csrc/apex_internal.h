// Internal types shared by the HIP kernels and the host engine (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/apex.h"

namespace apex {

constexpr int kRowPad = 4;             // LDS row padding (floats) for staged synthon rows
constexpr int kHeadsPad = 16;          // heads are padded to one 16-wide MFMA tile
constexpr uint32_t kSelectThreads = 1024;

// Workgroup and tile geometry of the fused kernels. A tile is TA "A" rows (slot
// 0, or slots 0 and 1 of a three-slot reaction) against 16 consecutive "B" rows
// (the last slot). FP32 (16x16 MFMA kernel): 8 waves of 16 compounds each (one
// A-row, 16 B-rows). BF16 and FP8 (32x32 MFMA kernel): 4 waves of 32 compounds
// each (two A-rows, 16 B-rows), small enough in LDS for two workgroups per CU.
constexpr int kWaves16 = 8, kTileA16 = 8;  // FP32 kernel: 8 waves, one A-row each
constexpr int kTileB = 16;
// Linear-probe engines (one decoder layer) run the scalar-contribution kernel
// instead: a tile is 64 "A" rows against 64 "B" rows, one wave, a lane per B
// row. Such engines have up to kScalarHeads heads.
constexpr int kScalarTA = 256, kScalarTB = 64;
constexpr int kScalarHeads = 32;

inline int tile_ta(bool scalar) { return scalar ? kScalarTA : 8; }
inline int tile_tb(bool scalar) { return scalar ? kScalarTB : kTileB; }
inline int enum_waves(int prec) { return prec == APEX_PREC_FP32 ? 8 : 4; }
// blocks of 16 compounds per wave
inline int enum_rows(int prec) { return prec == APEX_PREC_FP32 ? 1 : 2; }

// One reaction of the library as the kernels see it: every compound is a pair
// (a, b) with a over the first slot(s) and b over the last slot.
struct ReactDev {
  uint64_t id_off;  // id of the reaction's first compound
  uint32_t row0;    // table row of synthon 0 of slot 0
  uint32_t row1;    // table row of synthon 0 of slot 1 (three-slot reactions)
  uint32_t rowB;    // table row of synthon 0 of the last slot
  uint32_t n1;      // synthons in slot 1 (three-slot: a = i0 * n1 + i1)
  uint32_t nA;      // n0, or n0 * n1 for three slots
  uint32_t nB;      // synthons in the last slot
  uint32_t three;   // 1 for a three-slot reaction
  uint32_t pad;
};

// A reaction selected for a pass, with its place in the pass's tile sequence.
struct SelDev {
  uint64_t tile_start;      // first tile index of this reaction in the pass
  uint64_t compound_start;  // first compound (in selection order) of this reaction
  uint32_t t;               // reaction index
  uint32_t tiles_b;         // tiles along b
};

// Per-precision decoder state resident in the engine workspace.
struct PrecDev {
  const void* w2;      // GEMM2 fragments [chunks][H1/KS][64][E] (n_layers == 3)
  const void* wo;      // final-layer fragments
  const float* b2;     // GEMM2 accumulator initial values [H2]
  const float* bo;     // final bias [16]
  const float* scal;   // [0] GEMM2 scale S2, [1] final scale So, [2] X conversion scale
  const float* delta;  // [16] per-head relaxation used while enumerating in low precision
};

// Running state of one query's candidate buffer.
struct QState {
  float tau_o;        // threshold key: pass iff o > tau_o or (o == tau_o and id <= tau_id)
  uint32_t pad0;
  uint64_t tau_id;
  uint32_t count;     // entries appended (may exceed cap)
  uint32_t chunk_base;// count when the current chunk began
  uint32_t overflow;  // chunks re-run so far are flagged in the rerun list
  uint32_t warm;      // 1: the warm start set a finite threshold
  uint64_t appended;  // total appends over the search
};

// Selection scratch of one query (device): pivots placed from a sorted sample of
// the candidate keys, exact counts above them, and the "bracket" - the entries
// between the two pivots that enclose the K-th key - sorted in LDS.
constexpr uint32_t kSelSample = 2048;
constexpr uint32_t kSelBracket = 8192;
constexpr int kSelPivots = 8;
struct SelScratch {
  uint32_t piv[kSelPivots];     // order keys, non-increasing
  uint32_t cnt_gt[kSelPivots];  // entries with key > piv[j]
  uint32_t cnt_ge[kSelPivots];  // entries with key >= piv[j]
  uint32_t pos_sure, pos_br;    // compaction cursors
  uint32_t mode;                // 0: pivot path, 1: one-workgroup radix path
  uint32_t pad;
  uint32_t br_key[kSelBracket];
  uint64_t br_id[kSelBracket];
};

// Query of a linear-probe engine (Section 4.3, eq. "apex"): the objective and
// every constrained head are sums of per-synthon contributions, so the query is
// evaluated from per-row tables built once per query: column 0 holds each
// synthon row's objective contribution sum_h w[h] v[h] (NaN if a head of the
// row is not finite), column 1 + c the row's value of constrained head head[c].
// Ordinary passes list the distinct constrained heads with their intersected
// bounds; the violation pass (viol = 1) lists the query's constraints as given,
// since the violation sums over constraints.
struct ScalarQuery {
  float w[kScalarHeads];
  uint32_t head[APEX_MAX_CONSTRAINTS];  // constrained heads
  float lo[APEX_MAX_CONSTRAINTS];       // inclusive bounds
  float hi[APEX_MAX_CONSTRAINTS];
  uint32_t n_ch;                        // entries of head/lo/hi
  uint32_t viol;                        // 1: rank infeasible compounds by violation
  float* tab;                           // [1 + n_ch][rows]
  uint64_t rows;
};

// One R-group (slot) of the associative-embedding GEMM: its first table row,
// its synthon count and its first 16-row tile in the grouped launch.
struct AssocSlot {
  uint64_t row0;
  uint64_t tile0;
  uint32_t n;
  uint32_t pad;
};

// Query parameters for the fused kernel and the scoring kernels.
struct QueryDev {
  float w[kHeadsPad];
  float lo[kHeadsPad];   // per-head lower bound (intersection of the query's bounds)
  float hi[kHeadsPad];
  QState* st;
  float* cand_o;         // candidate buffer [cap]
  uint64_t* cand_id;
  float* tmp_o;          // compaction scratch [K]
  uint64_t* tmp_id;
  uint32_t* rerun;       // per-chunk overflow flags
  const uint32_t* subset_bits;  // [ceil(T/32)] or null (all reactions)
  uint32_t cap;
  uint32_t K;            // entries kept (k, or the low-precision pool size)
  uint32_t hwm;          // compaction trigger
  uint32_t active;       // 0: skip this query in a pass
  SelScratch* sel;       // selection scratch
  const ScalarQuery* sq; // linear-probe engines: the query's per-row tables
};

struct EnumArgs {
  const float* P;          // hoisted tables [rows][H1] FP32
  const ReactDev* react;
  const SelDev* sel;
  uint32_t n_sel;
  uint64_t tile_begin, tile_end;  // tiles of this launch
  PrecDev pd;
  uint32_t H2;             // second hidden width (n_layers == 3)
  uint32_t n_queries;
  const QueryDev* queries;
  // gather mode
  const uint64_t* ids;     // compound ids
  uint32_t n_ids;
  uint64_t n_reactions;
  uint64_t n_total;        // compounds in the library
  float* heads_out;        // [n_ids][16]
  // tile mode of the 32x32 kernels: eight region counters and an exit counter,
  // zero when a launch starts (the launch leaves them zero); null for static
  // work ranges
  uint32_t* work;
};

}  // namespace apex
