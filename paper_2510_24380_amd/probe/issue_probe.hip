// Issue-rate probe of one wave on gfx950: a loop of 32x32 MFMAs spread over
// NCH independent accumulator chains (used in turn), with K independent vector
// operations (FMA or exp2) after each MFMA. The loop's shader-clock cycles
// (s_memtime) are written to cyc[0]; out[] only keeps the results alive.
// It measures how long a dependent MFMA waits for its predecessor and how much
// of a wave's own vector work overlaps its MFMAs, the two figures that set the
// fused kernel's per-chunk time. Not part of the engine.
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(8 * sizeof(int)))) int i32x8;

template <bool FP8, int NCH, int K, bool TRANS>
__global__ __launch_bounds__(64) void k_issue(float* out, unsigned long long* cyc, int iters) {
  const int t = threadIdx.x;
  bf16x8 a, b;
  i32x8 a8, b8;
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(0.001f * (t + e));
    b[e] = (__bf16)(0.002f * (t - e));
    a8[e] = 0x38383838 + t + e;  // E4M3 values near 0.6
    b8[e] = 0x30303030 + t - e;
  }
  f32x16 acc[NCH];
  for (int c = 0; c < NCH; ++c) acc[c] = f32x16{};
  float v[8];
  for (int j = 0; j < 8; ++j) v[j] = 0.1f * (t + j);
  const unsigned long long t0 = __builtin_amdgcn_s_memtime();
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      if (FP8)
        acc[c] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, acc[c], 0, 0, 0, 127, 0, 127);
      else
        acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (TRANS) v[k & 7] = __builtin_amdgcn_exp2f(v[k & 7]);
        else v[k & 7] = fmaf(v[k & 7], 0.999f, 0.001f);
      }
      // keep the written order: MFMA, then its K vector operations
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  const unsigned long long t1 = __builtin_amdgcn_s_memtime();
  float s = 0.f;
  for (int c = 0; c < NCH; ++c)
    for (int q = 0; q < 16; ++q) s += acc[c][q];
  for (int j = 0; j < 8; ++j) s += v[j];
  out[t] = s;
  if (t == 0) cyc[0] = t1 - t0;
}

template <bool FP8, int NCH, int K, bool TRANS>
static const void* kern() {
  return reinterpret_cast<const void*>(&k_issue<FP8, NCH, K, TRANS>);
}
template <bool FP8, int NCH>
static const void* by_k(int k, int trans) {
  if (k == 0) return kern<FP8, NCH, 0, false>();
  if (k == 2) return trans ? kern<FP8, NCH, 2, true>() : kern<FP8, NCH, 2, false>();
  if (k == 4) return trans ? kern<FP8, NCH, 4, true>() : kern<FP8, NCH, 4, false>();
  if (k == 8) return trans ? kern<FP8, NCH, 8, true>() : kern<FP8, NCH, 8, false>();
  return nullptr;
}
template <bool FP8>
static const void* by_chains(int nch, int k, int trans) {
  if (nch == 1) return by_k<FP8, 1>(k, trans);
  if (nch == 2) return by_k<FP8, 2>(k, trans);
  if (nch == 4) return by_k<FP8, 4>(k, trans);
  return nullptr;
}

// fp8: 0 = 32x32x16 BF16, 1 = 32x32x64 FP8 (E8M0 scales of one); nch in {1, 2, 4};
// k in {0, 2, 4, 8}; trans: exp2 instead of FMA. out: 64 floats, cyc: one
// 64-bit counter, both device memory. Returns 0, -1 for an unsupported shape,
// or the HIP error of the launch.
extern "C" int probe_issue(int fp8, int nch, int k, int trans, int iters, float* out, unsigned long long* cyc) {
  const void* f = fp8 ? by_chains<true>(nch, k, trans) : by_chains<false>(nch, k, trans);
  if (!f || iters <= 0) return -1;
  void* args[] = {&out, &cyc, &iters};
  hipError_t e = hipLaunchKernel(f, dim3(1), dim3(64), args, 0, 0);
  if (e != hipSuccess) return (int)e;
  return (int)hipDeviceSynchronize();
}
