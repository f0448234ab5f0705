// Measured ceilings of the device for the roofline: matrix-core throughput of
// the FP64 and FP32 16x16x4 instructions the transform uses, FP64 vector FMA
// throughput, and a streaming device copy.  Prints one JSON line.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

#define CHECK(x)                                                          \
  do {                                                                    \
    hipError_t e_ = (x);                                                  \
    if (e_ != hipSuccess) {                                               \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));             \
      exit(1);                                                            \
    }                                                                     \
  } while (0)

template <int CH>
__global__ __launch_bounds__(256) void mfma64(double* out, int iters) {
  d4 acc[CH];
  for (int c = 0; c < CH; c++) acc[c] = (d4){0, 0, 0, 0};
  const double a = threadIdx.x * 1e-3, b = blockIdx.x * 1e-3;
  for (int i = 0; i < iters; i++)
#pragma unroll
    for (int c = 0; c < CH; c++) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  double s = 0;
  for (int c = 0; c < CH; c++) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int CH>
__global__ __launch_bounds__(256) void mfma32(float* out, int iters) {
  f4 acc[CH];
  for (int c = 0; c < CH; c++) acc[c] = (f4){0, 0, 0, 0};
  const float a = threadIdx.x * 1e-3f, b = blockIdx.x * 1e-3f;
  for (int i = 0; i < iters; i++)
#pragma unroll
    for (int c = 0; c < CH; c++) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  float s = 0;
  for (int c = 0; c < CH; c++) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int CH>
__global__ __launch_bounds__(256) void vfma64(double* out, int iters) {
  double acc[CH];
  for (int c = 0; c < CH; c++) acc[c] = c;
  const double a = 1.0 + threadIdx.x * 1e-9, b = 1e-9 * blockIdx.x;
  for (int i = 0; i < iters; i++)
#pragma unroll
    for (int c = 0; c < CH; c++) acc[c] = __builtin_fma(acc[c], a, b);
  double s = 0;
  for (int c = 0; c < CH; c++) s += acc[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void copyk(const double2* __restrict__ x, double2* __restrict__ y, size_t n) {
  const size_t st = (size_t)gridDim.x * blockDim.x;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += st) y[i] = x[i];
}

template <typename K, typename P>
static float time_ms(K kern, int grid, P* out, int iters) {
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, 0, out, 8);
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, 0, out, iters);
  CHECK(hipEventRecord(e1));
  CHECK(hipEventSynchronize(e1));
  float ms = 0;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  return ms;
}

int main() {
  int dev = 0, ncu = 0;
  CHECK(hipGetDevice(&dev));
  CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int grid = ncu * 16, iters = 1000;
  const double waves = (double)grid * 4;
  double* o64;
  float* o32;
  CHECK(hipMalloc(&o64, (size_t)grid * 256 * sizeof(double)));
  CHECK(hipMalloc(&o32, (size_t)grid * 256 * sizeof(float)));
  const double mfma_flops = 2.0 * 16 * 16 * 4 * 4 * iters * waves;  // 4 chains
  const double t64 = time_ms(mfma64<4>, grid, o64, iters);
  const double t32 = time_ms(mfma32<4>, grid, o32, iters);
  const double tv = time_ms(vfma64<16>, grid, o64, iters);
  const double vflops = 2.0 * 16 * iters * waves * 64;
  const size_t bytes = (size_t)2 << 30;
  double2 *x, *y;
  CHECK(hipMalloc(&x, bytes));
  CHECK(hipMalloc(&y, bytes));
  CHECK(hipMemset(x, 0, bytes));
  CHECK(hipMemset(y, 0, bytes));
  const size_t n = bytes / sizeof(double2);
  hipLaunchKernelGGL(copyk, dim3(ncu * 16), dim3(256), 0, 0, x, y, n);
  CHECK(hipDeviceSynchronize());
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  CHECK(hipEventRecord(e0));
  for (int r = 0; r < 5; r++) hipLaunchKernelGGL(copyk, dim3(ncu * 16), dim3(256), 0, 0, x, y, n);
  CHECK(hipEventRecord(e1));
  CHECK(hipEventSynchronize(e1));
  float tc = 0;
  CHECK(hipEventElapsedTime(&tc, e0, e1));
  printf("{\"cus\": %d, \"mfma_f64_16x16x4_tflops\": %.1f, \"mfma_f32_16x16x4_tflops\": %.1f, "
         "\"vector_fma_f64_tflops\": %.1f, \"copy_gbs\": %.0f}\n",
         ncu, mfma_flops / t64 / 1e9, mfma_flops / t32 / 1e9, vflops / tv / 1e9,
         5.0 * 2 * bytes / tc / 1e6);
  CHECK(hipFree(x));
  CHECK(hipFree(y));
  CHECK(hipFree(o64));
  CHECK(hipFree(o32));
  return 0;
}
