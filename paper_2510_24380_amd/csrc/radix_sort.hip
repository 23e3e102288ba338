// Ordering of long answers: a stable least-significant-digit radix sort of
// (objective, id) entries by objective descending, then id ascending (the
// answer order of eq. "apex_topk" with ties broken by the lower id). The
// composite key is (~ord(objective), id) sorted ascending: first the id's bytes
// (as many as the library's largest id needs), then the four bytes of the
// objective key, 8 bits per pass. Every pass is a per-block digit histogram, a
// scan of the histograms (digit-major, so equal digits keep block order) and a
// stable scatter: inside a block, items are ranked in index order, 256 at a
// time, with per-wave digit peer masks built from 8 ballots.
//
// The number of entries is read on the device (min(state->count, n_max)); the
// grid is sized for n_max.
#include "enum_common.h"
#include "launch.h"

namespace apex {

constexpr uint32_t kRsThreads = 256;
constexpr uint32_t kRsRounds = 16;
constexpr uint32_t kRsItems = kRsThreads * kRsRounds;  // per block

uint32_t radix_blocks(uint32_t n_max) { return (n_max + kRsItems - 1) / kRsItems; }

struct RsPass {
  const float* src_o;     // first pass: objectives (converted to keys on the fly)
  const uint32_t* src_k;  // later passes: keys
  const uint64_t* src_id;
  uint32_t* dst_k;        // intermediate passes
  uint64_t* dst_id;
  float* out_o;           // last pass: objectives, only entries ranked below n_out
  uint64_t* out_id;
  uint32_t n_out;
  uint32_t shift;         // bit position of the digit
  uint32_t on_id;         // 1: digit of the id, 0: digit of the key
  uint32_t n_max;
  const QState* st;       // n = min(st->count, n_max)
  uint32_t* hist;         // [256][blocks], offsets after the scan
  uint32_t* total;        // [256]
};

__device__ __forceinline__ uint32_t rs_key(const RsPass& p, uint32_t i) {
  if (p.src_o) return ~ord_f32(p.src_o[i]);  // descending objective
  return p.src_k[i];
}

__device__ __forceinline__ uint32_t rs_digit(const RsPass& p, uint32_t key, uint64_t id) {
  return p.on_id ? (uint32_t)(id >> p.shift) & 255u : (key >> p.shift) & 255u;
}

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(RsPass p) {
  __shared__ uint32_t h[256];
  const uint32_t n = min(p.st->count, p.n_max);
  const uint32_t blocks = gridDim.x;
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kRsItems;
  for (uint32_t r = 0; r < kRsRounds; ++r) {
    const uint32_t i = base + r * kRsThreads + threadIdx.x;
    if (i < n) {
      const uint64_t id = p.src_id[i];
      const uint32_t key = p.on_id ? 0u : rs_key(p, i);
      atomicAdd(&h[rs_digit(p, key, id)], 1u);
    }
  }
  __syncthreads();
  p.hist[(uint64_t)threadIdx.x * blocks + blockIdx.x] = h[threadIdx.x];
}

// One workgroup per digit: exclusive scan of that digit's block counts in
// place, and the digit's total.
__global__ __launch_bounds__(kRsThreads) void k_rs_scan_digit(uint32_t* __restrict__ hist, uint32_t blocks,
                                                             uint32_t* __restrict__ total) {
  __shared__ uint32_t part[kRsThreads];
  uint32_t* h = hist + (uint64_t)blockIdx.x * blocks;
  const uint32_t per = (blocks + kRsThreads - 1) / kRsThreads;
  const uint32_t b0 = threadIdx.x * per, b1 = min(blocks, b0 + per);
  uint32_t s = 0;
  for (uint32_t b = b0; b < b1; ++b) s += h[b];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (uint32_t t = 0; t < kRsThreads; ++t) {
      const uint32_t v = part[t];
      part[t] = acc;
      acc += v;
    }
    total[blockIdx.x] = acc;
  }
  __syncthreads();
  uint32_t acc = part[threadIdx.x];
  for (uint32_t b = b0; b < b1; ++b) {
    const uint32_t v = h[b];
    h[b] = acc;
    acc += v;
  }
}

__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(RsPass p) {
  __shared__ uint32_t dbase[256];                       // digit's first output position for this block
  __shared__ uint32_t wcnt[kRsThreads / 64][256];       // per-wave digit counts of the round
  const uint32_t n = min(p.st->count, p.n_max);
  const uint32_t blocks = gridDim.x;
  const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
  {
    uint32_t before = 0;  // entries of smaller digits over all blocks
    for (uint32_t d = 0; d < t; ++d) before += p.total[d];
    dbase[t] = before + p.hist[(uint64_t)t * blocks + blockIdx.x];
  }
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const uint32_t base = blockIdx.x * kRsItems;
  for (uint32_t r = 0; r < kRsRounds; ++r) {
    for (uint32_t w = 0; w < kRsThreads / 64; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const uint32_t i = base + r * kRsThreads + t;
    const bool in = i < n;
    uint64_t id = 0;
    uint32_t key = 0, dig = 0;
    if (in) {
      id = p.src_id[i];
      key = rs_key(p, i);
      dig = rs_digit(p, key, id);
    }
    uint64_t peers = __ballot(in);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t m = __ballot(in && ((dig >> bit) & 1u));
      peers &= ((dig >> bit) & 1u) ? m : ~m;
    }
    const uint32_t rank_w = (uint32_t)__popcll(peers & below);
    if (in && rank_w == 0) wcnt[wave][dig] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (in) {
      uint32_t pos = dbase[dig] + rank_w;
      for (uint32_t w = 0; w < wave; ++w) pos += wcnt[w][dig];
      if (p.dst_k) {
        p.dst_k[pos] = key;
        p.dst_id[pos] = id;
      } else if (pos < p.n_out) {
        const uint32_t ord = ~key;
        p.out_o[pos] = __uint_as_float((ord & 0x80000000u) ? (ord & 0x7fffffffu) : ~ord);
        p.out_id[pos] = id;
      }
    }
    __syncthreads();
    uint32_t add = 0;
    for (uint32_t w = 0; w < kRsThreads / 64; ++w) add += wcnt[w][t];
    dbase[t] += add;
  }
}

hipError_t launch_radix_sort(const QState* st, uint32_t n_max, const float* src_o, const uint64_t* src_id,
                             uint32_t* a_k, uint64_t* a_id, uint32_t* b_k, uint64_t* b_id, float* out_o,
                             uint64_t* out_id, uint32_t n_out, uint32_t id_bytes, uint32_t* hist, hipStream_t s) {
  if (n_max == 0) return hipSuccess;
  const uint32_t blocks = radix_blocks(n_max);
  uint32_t* total = hist + (uint64_t)256 * blocks;
  const uint32_t passes = id_bytes + 4;
  RsPass p{};
  p.st = st;
  p.n_max = n_max;
  p.hist = hist;
  p.total = total;
  p.n_out = n_out;
  const uint32_t* cur_k = nullptr;
  const uint64_t* cur_id = src_id;
  for (uint32_t j = 0; j < passes; ++j) {
    p.src_o = j == 0 ? src_o : nullptr;
    p.src_k = cur_k;
    p.src_id = cur_id;
    p.on_id = j < id_bytes ? 1u : 0u;
    p.shift = 8u * (j < id_bytes ? j : j - id_bytes);
    const bool last = j + 1 == passes;
    uint32_t* dk = (j & 1) ? b_k : a_k;
    uint64_t* did = (j & 1) ? b_id : a_id;
    p.dst_k = last ? nullptr : dk;
    p.dst_id = last ? nullptr : did;
    p.out_o = out_o;
    p.out_id = out_id;
    hipLaunchKernelGGL(k_rs_hist, dim3(blocks), dim3(kRsThreads), 0, s, p);
    hipLaunchKernelGGL(k_rs_scan_digit, dim3(256), dim3(kRsThreads), 0, s, hist, blocks, total);
    hipLaunchKernelGGL(k_rs_scatter, dim3(blocks), dim3(kRsThreads), 0, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur_k = dk;
    cur_id = did;
  }
  return hipSuccess;
}

}  // namespace apex
