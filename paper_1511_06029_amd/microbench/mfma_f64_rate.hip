// Register-only rate of the FP64 matrix instructions on gfx950: the ceiling
// the FP64 core-step kernels are compared with.
//
// Each wave keeps its operands in registers and issues ITER rounds of
// WR x WQ independent v_mfma_f64_4x4x4_4b (512 flops each) with the operand
// pattern of the fused-pair kernel (WQ input fragments, WR core fragments,
// WR x WQ accumulators), or of v_mfma_f64_16x16x4 (2048 flops each).  No
// memory traffic inside the loop; the accumulators are stored once so that
// nothing is optimised away.  Launch: `blocks` workgroups of 64 x waves
// threads (two waves per SIMD fill a CU at 8 waves per workgroup).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

typedef double v4d __attribute__((ext_vector_type(4)));

template <int WR, int WQ>
__global__ void __launch_bounds__(512) mfma4_kernel(double* out, int iter, double seed) {
  const int lane = threadIdx.x & 63;
  double a[WQ], b[WR];
  double acc[WR][WQ];   // one output per lane: four 4x4 blocks over 64 lanes
#pragma unroll
  for (int j = 0; j < WQ; ++j) a[j] = seed + 0.001 * (lane + j);
#pragma unroll
  for (int i = 0; i < WR; ++i) b[i] = seed - 0.002 * (lane + i);
#pragma unroll
  for (int i = 0; i < WR; ++i)
#pragma unroll
    for (int j = 0; j < WQ; ++j) acc[i][j] = 0.0;
  for (int t = 0; t < iter; ++t) {
#pragma unroll
    for (int i = 0; i < WR; ++i)
#pragma unroll
      for (int j = 0; j < WQ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[j], b[i], acc[i][j], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < WR; ++i)
#pragma unroll
    for (int j = 0; j < WQ; ++j) s += acc[i][j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int N>
__global__ void __launch_bounds__(512) mfma16_kernel(double* out, int iter, double seed) {
  const int lane = threadIdx.x & 63;
  const double a = seed + 0.001 * lane, b = seed - 0.002 * lane;
  v4d acc[N];
#pragma unroll
  for (int i = 0; i < N; ++i) acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int t = 0; t < iter; ++t) {
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

static double run(const void* fn, int blocks, int threads, int iter, double flops_per_wave_iter) {
  double* out = nullptr;
  if (hipMalloc(&out, (size_t)blocks * threads * sizeof(double)) != hipSuccess) return -1;
  double seed = 1.0;
  void* args[] = {&out, &iter, &seed};
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)hipLaunchKernel(fn, dim3(blocks), dim3(threads), args, 0, nullptr);   // warm-up
  (void)hipEventRecord(e0, nullptr);
  (void)hipLaunchKernel(fn, dim3(blocks), dim3(threads), args, 0, nullptr);
  (void)hipEventRecord(e1, nullptr);
  (void)hipEventSynchronize(e1);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipFree(out);
  const double waves = (double)blocks * threads / 64.0;
  return waves * iter * flops_per_wave_iter / (ms * 1e-3) / 1e12;
}

int main(int argc, char** argv) {
  int cus = 256;
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int iter = argc > 1 ? atoi(argv[1]) : 20000;
  printf("{\"compute_units\": %d, \"iterations\": %d, \"rates_tflops\": {", cus, iter);
  // the fused pair kernel's pattern: 4 core x 8 input fragments, 32 accumulators;
  // 8 waves per workgroup = 2 waves per SIMD, one workgroup per CU
  printf("\"4x4x4 pattern 4x8, 2 waves/SIMD\": %.2f, ",
         run((const void*)&mfma4_kernel<4, 8>, cus, 512, iter, 32 * 512.0));
  printf("\"4x4x4 pattern 4x8, 1 wave/SIMD\": %.2f, ",
         run((const void*)&mfma4_kernel<4, 8>, cus, 256, iter, 32 * 512.0));
  printf("\"4x4x4 pattern 4x4, 2 waves/SIMD\": %.2f, ",
         run((const void*)&mfma4_kernel<4, 4>, cus, 512, iter, 16 * 512.0));
  printf("\"4x4x4 pattern 8x4, 2 waves/SIMD\": %.2f, ",
         run((const void*)&mfma4_kernel<8, 4>, cus, 512, iter, 32 * 512.0));
  printf("\"4x4x4 pattern 2x8, 2 waves/SIMD\": %.2f, ",
         run((const void*)&mfma4_kernel<2, 8>, cus, 512, iter, 16 * 512.0));
  printf("\"4x4x4 pattern 8x8, 2 waves/SIMD\": %.2f, ",
         run((const void*)&mfma4_kernel<8, 8>, cus, 512, iter, 64 * 512.0));
  printf("\"4x4x4 pattern 1x1, 2 waves/SIMD\": %.2f, ",
         run((const void*)&mfma4_kernel<1, 1>, cus, 512, iter, 1 * 512.0));
  printf("\"16x16x4, 8 accumulators, 2 waves/SIMD\": %.2f",
         run((const void*)&mfma16_kernel<8>, cus, 512, iter, 8 * 2048.0));
  printf("}, \"peak_fp64_tflops\": 78.6}\n");
  return 0;
}
