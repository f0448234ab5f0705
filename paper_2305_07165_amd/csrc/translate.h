// The out->in translation body shared by the per-stage kernels (kernels.hip)
// and the persistent batched kernels (kernels_fast.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "mfma.h"

namespace fgt {

// ---------------------------------------------------------------------------
// translate: psi_A = sum_{(B,dir) in P(A)} Rot(dir * L_c) phi_B.  One thread per
// mode multi-index (m_1..m_d); it owns the 2^d coefficients 2 m_a + v_a
// (v_a = 0: cos, 1: sin; for m_a = 0 the constant and the stored zero, which a
// shift leaves alone since rot of mode 0 is the identity).
// R2F: the tensors are stored [r3][r1][r2] (r2 fastest, the d = 3 layout of
// kernels_fast.hip) instead of [r3][r2][r1]; threads then run along m_2.  The
// pair along the fastest-stored axis is one aligned two-element vector.

template <typename T, int D, bool R2F>
__device__ __forceinline__ void translate_body(const T* __restrict__ phi,
                                               const int32_t* __restrict__ plist_start,
                                               const int32_t* __restrict__ plist_src,
                                               const int32_t* __restrict__ plist_dir,
                                               const T* __restrict__ rot, int M, int nr, int nA,
                                               T* __restrict__ psi, int bid) {
  typedef typename Pair2<T>::type T2;
  // Chunks of modes are dealt to the XCDs: XCD x sweeps every target box (in
  // Morton order) for chunks x, x + 8, ..., so each source slice of those
  // chunks is fetched into one L2 and reused by all its targets there; the
  // nchunk % 8 leftover chunks are split into eight contiguous box ranges, one
  // per XCD, so the XCDs get equal work.
  int nblk = 1;
  for (int a = 0; a < D; a++) nblk *= M;
  const int nch = (nblk + (int)blockDim.x - 1) / (int)blockDim.x;
  const int nbx = (nA + kXcds - 1) / kXcds;
  const int rounds = nch / kXcds;
  const int xcd = bid % kXcds, local = bid / kXcds;
  int A, chunk;
  if (local < rounds * nA) {
    const int r = local / nA;
    A = local - r * nA;
    chunk = kXcds * r + xcd;
  } else {
    const int j = local - rounds * nA;
    A = xcd * nbx + j % nbx;
    chunk = kXcds * rounds + j / nbx;
  }
  const int b = chunk * (int)blockDim.x + (int)threadIdx.x;
  if (A >= nA || chunk >= nch || b >= nblk) return;
  int m[3] = {0, 0, 0};
  {
    int q = b;
    if (R2F) {
      m[1] = q % M; q /= M;
      m[0] = q % M; q /= M;
      m[2] = q;
    } else {
      for (int a = 0; a < D; a++) { m[a] = q % M; q /= M; }
    }
  }
  constexpr int FA = R2F ? 1 : 0;  // the axis stored fastest
  constexpr int NV = 1 << D, NW = NV / 2;
  const int64_t stride[3] = {R2F ? nr : 1, R2F ? 1 : nr, (int64_t)nr * nr};
  // off[w]: the pair (v_FA = 0, 1) of coefficient v = spread(w), where w runs
  // over the cos/sin choices of the other axes
  int64_t off[NW];
#pragma unroll
  for (int w = 0; w < NW; w++) {
    int64_t o = stride[FA] * (2 * m[FA]);
    int bit = 0;
#pragma unroll
    for (int a = 0; a < D; a++) {
      if (a == FA) continue;
      o += stride[a] * (2 * m[a] + ((w >> bit) & 1));
      bit++;
    }
    off[w] = o;
  }
  auto vidx = [](int w, int vf) {  // coefficient v (bit a = sin member of axis a)
    int v = vf << FA, bit = 0;
    for (int a = 0; a < D; a++) {
      if (a == FA) continue;
      v |= ((w >> bit) & 1) << a;
      bit++;
    }
    return v;
  };
  T cs[3], sn[3];
  for (int a = 0; a < D; a++) { cs[a] = rot[2 * m[a]]; sn[a] = rot[2 * m[a] + 1]; }
  int64_t ncoef = nr;
  for (int a = 1; a < D; a++) ncoef *= nr;
  T acc[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) acc[v] = 0;
  const int q0 = plist_start[A], q1 = plist_start[A + 1];
  // two sources in flight: the loads of source q+1 are issued before the
  // rotations of source q (a q past the list reloads the last source)
  auto fetch = [&](int q, T (&x)[NV]) {
    const T* src = phi + (int64_t)plist_src[min(q, q1 - 1)] * ncoef;
#pragma unroll
    for (int w = 0; w < NW; w++) {
      const T2 v2 = *reinterpret_cast<const T2*>(src + off[w]);
      x[vidx(w, 0)] = v2.x;
      x[vidx(w, 1)] = v2.y;
    }
  };
  // rotations along every axis the source is displaced on; the last one adds
  // straight into the accumulators
  auto apply = [&](int q, T (&x)[NV]) {
    int code = plist_dir[q];
    int dir[3] = {0, 0, 0};
    int last = -1;
#pragma unroll
    for (int a = 0; a < D; a++) {
      dir[a] = code % 3 - 1;
      code /= 3;
      if (dir[a] != 0) last = a;
    }
#pragma unroll
    for (int a = 0; a < D; a++) {
      if (dir[a] == 0) continue;
      const T c = cs[a], s = dir[a] > 0 ? sn[a] : -sn[a];
      const int bit = 1 << a;
      if (a == last) {
#pragma unroll
        for (int v = 0; v < NV; v++) {
          if (v & bit) continue;
          const T xc = x[v], xs = x[v | bit];
          acc[v] = fma(c, xc, acc[v]);
          acc[v] = fma(-s, xs, acc[v]);
          acc[v | bit] = fma(s, xc, acc[v | bit]);
          acc[v | bit] = fma(c, xs, acc[v | bit]);
        }
      } else {
#pragma unroll
        for (int v = 0; v < NV; v++) {
          if (v & bit) continue;
          const T xc = x[v], xs = x[v | bit];
          x[v] = c * xc - s * xs;
          x[v | bit] = s * xc + c * xs;
        }
      }
    }
    if (last < 0) {
#pragma unroll
      for (int v = 0; v < NV; v++) acc[v] += x[v];
    }
  };
  T xa[NV], xb[NV];
  if (q0 < q1) {
    fetch(q0, xa);
    for (int q = q0; q < q1; q += 2) {
      fetch(q + 1, xb);
      apply(q, xa);
      if (q + 1 < q1) {
        fetch(q + 2, xa);
        apply(q + 1, xb);
      }
    }
  }
  T* dst = psi + (int64_t)A * ncoef;
#pragma unroll
  for (int w = 0; w < NW; w++) {
    T2 v2;
    v2.x = acc[vidx(w, 0)];
    v2.y = acc[vidx(w, 1)];
    *reinterpret_cast<T2*>(dst + off[w]) = v2;
  }
}

}  // namespace fgt
