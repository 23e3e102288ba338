// Lane-layout probe of the MFMA builtins and conversions the engine uses.
// Each kernel runs one wave: lane l reads its A and B operand registers from
// a[l], b[l] and writes its accumulator registers to d[NV l .. NV l + NV - 1]
// (NV = 4 for the 16x16 shapes, 16 for the 32x32 shapes).
// Used only by the layout test; not part of the engine.
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(8 * sizeof(int)))) int i32x8;
typedef __attribute__((__vector_size__(2 * sizeof(short)))) short s16x2;

__global__ void k_f32(const float* a, const float* b, float* d) {
  const int l = threadIdx.x;
  f32x4 c = {0, 0, 0, 0};
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[l], b[l], c, 0, 0, 0);
  for (int v = 0; v < 4; ++v) d[4 * l + v] = c[v];
}
__global__ void k_bf16(const bf16x8* a, const bf16x8* b, float* d) {
  const int l = threadIdx.x;
  f32x4 c = {0, 0, 0, 0};
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[l], b[l], c, 0, 0, 0);
  for (int v = 0; v < 4; ++v) d[4 * l + v] = c[v];
}
__global__ void k_fp8(const i32x8* a, const i32x8* b, float* d) {
  const int l = threadIdx.x;
  f32x4 c = {0, 0, 0, 0};
  c = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a[l], b[l], c, 0, 0, 0, 0, 0, 0);
  for (int v = 0; v < 4; ++v) d[4 * l + v] = c[v];
}
__global__ void k_bf16_32(const bf16x8* a, const bf16x8* b, float* d) {
  const int l = threadIdx.x;
  f32x16 c = {};
  c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[l], b[l], c, 0, 0, 0);
  for (int v = 0; v < 16; ++v) d[16 * l + v] = c[v];
}
__global__ void k_fp8_32(const i32x8* a, const i32x8* b, float* d) {
  const int l = threadIdx.x;
  f32x16 c = {};
  c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[l], b[l], c, 0, 0, 0, 0, 0, 0);
  for (int v = 0; v < 16; ++v) d[16 * l + v] = c[v];
}
// the same with E8M0 block scales sa, sb (2^(sa - 127), 2^(sb - 127)) on A and B
__global__ void k_fp8_32s(const i32x8* a, const i32x8* b, float* d, int sa, int sb) {
  const int l = threadIdx.x;
  f32x16 c = {};
  c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[l], b[l], c, 0, 0, 0, sa, 0, sb);
  for (int v = 0; v < 16; ++v) d[16 * l + v] = c[v];
}
// x[i] -> E4M3 byte with power-of-two scale xs (divides), and -> bf16 bits
__global__ void k_cvt(const float* x, int n, float xs, uint8_t* f8, uint16_t* bf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (2 * i + 1 >= n) return;
  s16x2 v = {0, 0};
  v = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(v, x[2 * i], x[2 * i + 1], xs, false);
  const uint32_t u = __builtin_bit_cast(uint32_t, v);
  f8[2 * i] = (uint8_t)(u & 0xff);
  f8[2 * i + 1] = (uint8_t)((u >> 8) & 0xff);
  bf[2 * i] = __builtin_bit_cast(uint16_t, (__bf16)x[2 * i]);
  bf[2 * i + 1] = __builtin_bit_cast(uint16_t, (__bf16)x[2 * i + 1]);
}

extern "C" int probe_mfma(int kind, const void* a, const void* b, float* d) {
  if (kind == 0) hipLaunchKernelGGL(k_f32, dim3(1), dim3(64), 0, 0, (const float*)a, (const float*)b, d);
  else if (kind == 1) hipLaunchKernelGGL(k_bf16, dim3(1), dim3(64), 0, 0, (const bf16x8*)a, (const bf16x8*)b, d);
  else if (kind == 2) hipLaunchKernelGGL(k_fp8, dim3(1), dim3(64), 0, 0, (const i32x8*)a, (const i32x8*)b, d);
  else if (kind == 3) hipLaunchKernelGGL(k_bf16_32, dim3(1), dim3(64), 0, 0, (const bf16x8*)a, (const bf16x8*)b, d);
  else if (kind == 4) hipLaunchKernelGGL(k_fp8_32, dim3(1), dim3(64), 0, 0, (const i32x8*)a, (const i32x8*)b, d);
  else return -1;
  return (int)hipDeviceSynchronize();
}
extern "C" int probe_mfma_fp8_scaled(const void* a, const void* b, float* d, int sa, int sb) {
  if (sa < 0 || sa > 254 || sb < 0 || sb > 254) return -1;
  hipLaunchKernelGGL(k_fp8_32s, dim3(1), dim3(64), 0, 0, (const i32x8*)a, (const i32x8*)b, d, sa, sb);
  return (int)hipDeviceSynchronize();
}
extern "C" int probe_cvt(const float* x, int n, float xs, uint8_t* f8, uint16_t* bf) {
  hipLaunchKernelGGL(k_cvt, dim3((n / 2 + 63) / 64), dim3(64), 0, 0, x, n, xs, f8, bf);
  return (int)hipDeviceSynchronize();
}
