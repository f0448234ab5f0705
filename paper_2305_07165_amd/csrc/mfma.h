// 16x16x4 matrix-core step for FP64 and FP32 on gfx950, with its lane layout.
//
// For a 64-lane wave with lr = lane % 16 and lk = lane / 16, one step computes
// C[16x16] += A[16x4] B[4x16].  Lane (lk, lr) supplies A[lr][k] and B[k][lr]
// and holds C[row(lk, t)][lr], t = 0..3, where row(lk, t) = 4t + lk for FP64
// and 4lk + t for FP32 (measured on the device).  The K index a lane supplies
// at step kk is free to choose as long as A and B agree; taking
// k = kidx(kk, lk) = row(lk, kk) makes result item kk of a finished tile
// exactly the B operand of step kk of the next product (rows of C become the
// K index), so chained contractions stay in registers.
#pragma once

#include <hip/hip_runtime.h>

namespace fgt {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4 acc;
  static __device__ __forceinline__ acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int t) { return 4 * t + lk; }
  static __device__ __forceinline__ int kidx(int kk, int lk) { return 4 * kk + lk; }
};
template <> struct Mfma<float> {
  typedef f4 acc;
  static __device__ __forceinline__ acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int t) { return 4 * lk + t; }
  static __device__ __forceinline__ int kidx(int kk, int lk) { return 4 * lk + kk; }
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2): workgroup b runs on XCD b % 8.  xcd_block maps b to a logical index so
// that every XCD owns one contiguous range of logical indices; with work laid
// out in Morton order, neighbors then share an L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
  const int per = nblocks / kXcds, rem = nblocks % kXcds;
  const int x = b % kXcds, local = b / kXcds;
  return x * per + (x < rem ? x : rem) + local;
}

// Masked load without a branch: the load always reads an in-bounds element
// (index 0 when masked off) and the value is selected afterwards, so the
// compiler can issue many such loads back to back instead of guarding each
// one with a branch and a wait.  base[0] must be valid.
template <typename T, typename S>
__device__ __forceinline__ T ld0(const S* __restrict__ base, int64_t idx, bool ok) {
  const S v = base[ok ? idx : 0];
  return ok ? (T)v : (T)0;
}

template <typename A> __device__ __forceinline__ void zero4(A& a) {
  a[0] = 0;
  a[1] = 0;
  a[2] = 0;
  a[3] = 0;
}

}  // namespace fgt
