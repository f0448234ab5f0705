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
  typedef double elem;
  typedef d4 acc;
  static __device__ __forceinline__ acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int t) { return 4 * t + lk; }
  static __device__ __forceinline__ int kidx(int kk, int lk) { return 4 * kk + lk; }
  // K index of step kk when neither operand is a chained result (both come
  // from memory or LDS): k = 4kk + lk, so ceil(K/4) steps cover K
  static __device__ __forceinline__ int kmem(int kk, int lk) { return 4 * kk + lk; }
  // N consecutive k-steps
  template <int N>
  static __device__ __forceinline__ acc steps(const double (&a)[N], const double (&b)[N], acc c) {
#pragma unroll
    for (int kk = 0; kk < N; kk++) c = step(a[kk], b[kk], c);
    return c;
  }
};
template <> struct Mfma<float> {
  typedef float elem;
  typedef f4 acc;
  static __device__ __forceinline__ acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int t) { return 4 * lk + t; }
  static __device__ __forceinline__ int kidx(int kk, int lk) { return 4 * lk + kk; }
  // as for FP64: with both operands from memory, K = 8 takes two steps, not four
  static __device__ __forceinline__ int kmem(int kk, int lk) { return 4 * kk + lk; }
  template <int N>
  static __device__ __forceinline__ acc steps(const float (&a)[N], const float (&b)[N], acc c) {
#pragma unroll
    for (int kk = 0; kk < N; kk++) c = step(a[kk], b[kk], c);
    return c;
  }
};

// Compute policy "BF16x3": FP32 operands and accumulators; a product of four
// k-steps is one 16x16x16 bf16 matrix-core product split three ways,
//   A B ~ A_lo B_hi + A_hi B_lo + A_hi B_hi,   X_hi = bf16(X), X_lo = bf16(X - X_hi),
// accumulated in FP32 (the A_lo B_lo term is dropped).  The 16x16x16 bf16 step
// takes A[lr][4lk+i] and B[4lk+i][lr], i = 0..3, from lane (lk, lr) and leaves
// C[4lk+t][lr] there (measured on the device): the FP32 layout of the four
// 16x16x4 steps it replaces (kidx(kk, lk) = 4lk + kk), so every kernel written
// for float runs unchanged in groups of four k-steps.
struct Bf16x3 {};
typedef short s4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint32_t bf16_rne_bits(float v) {
  const uint32_t u = __float_as_uint(v);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;  // round to nearest even (finite values)
}
template <> struct Mfma<Bf16x3> {
  typedef float elem;
  typedef f4 acc;
  static __device__ __forceinline__ int row(int lk, int t) { return 4 * lk + t; }
  static __device__ __forceinline__ int kidx(int kk, int lk) { return 4 * lk + kk; }
  // one bf16 product spans K = 16: memory operands keep the same layout
  static __device__ __forceinline__ int kmem(int kk, int lk) { return 4 * lk + kk; }
  template <int N>
  static __device__ __forceinline__ acc steps(const float (&a)[N], const float (&b)[N], acc c) {
    static_assert(N == 4, "BF16x3 products run four k-steps at a time");
    s4 ah, al, bh, bl;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const uint32_t ha = bf16_rne_bits(a[i]), hb = bf16_rne_bits(b[i]);
      ah[i] = (short)ha;
      bh[i] = (short)hb;
      al[i] = (short)bf16_rne_bits(a[i] - __uint_as_float(ha << 16));
      bl[i] = (short)bf16_rne_bits(b[i] - __uint_as_float(hb << 16));
    }
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
  }
};
template <typename C> using elem_t = typename Mfma<C>::elem;

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

// The two-element vector of a storage type: a stored (cos, sin) mode pair,
// which starts at an even index, is one aligned vector load or store.
template <typename T> struct Pair2;
template <> struct Pair2<double> { typedef double2 type; };
template <> struct Pair2<float> { typedef float2 type; };

template <typename A> __device__ __forceinline__ void zero4(A& a) {
  a[0] = 0;
  a[1] = 0;
  a[2] = 0;
  a[3] = 0;
}

}  // namespace fgt
