// Device stages of the box Gauss transform (Algorithm 4) for gfx950.
//
// Every contraction is a dense small matrix product and runs on the matrix
// cores: v_mfma_f64_16x16x4f64 (FP64) or v_mfma_f32_16x16x4f32 (FP32).  For a
// 64-lane wave, with lr = lane % 16 and lk = lane / 16, one instruction computes
// C[16x16] += A[16x4] B[4x16] with lane operands A[lr][lk], B[lk][lr]; result t
// (t = 0..3) of a lane is C[row][lr] with row = 4*t + lk for FP64 and
// row = 4*lk + t for FP32 (Mfma<T>::row).
//
// Stages (d = 3 shown; the modes r of an axis are the nr = 2M-1 real plane
// waves, the nodes j/i its p Gauss-Legendre points):
//   form_leaf  Y_s[j3][r2][r1] = sum F2[r2][j2] F1[r1][j1] sigma_s[j3][j2][j1]
//   form_box   phi_A[r3][c]    = sum_{s in A} sum_j3 F3_s[r3][j3] Y_s[j3][c]
//              (formation at every leaf, merged into its cutoff-level box A)
//   translate  psi_A = sum_{B in P(A)} Rot(c_B - c_A) phi_B
//   eval_box   Z_s[i3][c]      = sum_r3 E3_s[i3][r3] psi_A[r3][c]
//   eval_leaf  u_s[i3][i2][i1] = sum E2[i2][r2] E1[i1][r1] Z_s[i3][r2][r1]
//   near       u_T (+)= sum_{S in D(T)} (V3 (x) V2 (x) V1) sigma_S
// All reductions are gathers with a fixed order: no atomics, deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "mfma.h"
#include "translate.h"

namespace fgt {

template <typename A> __device__ __forceinline__ void zero(A& a) {
  a[0] = 0; a[1] = 0; a[2] = 0; a[3] = 0;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

constexpr int kMaxRowTiles = kMaxModes / 16;  // 8

// ---------------------------------------------------------------------------
// form_leaf: contract axes 1..d-1 of a leaf's samples with its formation tables

template <typename T, int D>
__global__ __launch_bounds__(256) void k_form_leaf(const double* __restrict__ sigma,
                                                   const int32_t* __restrict__ leaf_id,
                                                   const int32_t* __restrict__ leaf_tab,
                                                   const T* __restrict__ F, int p, int nr,
                                                   T* __restrict__ Y) {
  typedef typename Mfma<T>::acc acc_t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int s = blockIdx.x;
  const int leaf = leaf_id[s];
  const int lane = lane_id(), w = wave_id();
  const int lr = lane & 15, lk = lane >> 4;
  const int nrp = (nr + 15) & ~15;
  const int ntile = nrp >> 4;
  const int ksteps = (p + 3) >> 2;
  if (D == 1) {
    for (int j = threadIdx.x; j < p; j += blockDim.x) Y[(int64_t)s * p + j] = (T)sigma[(int64_t)leaf * p + j];
    return;
  }
  const T* F1 = F + (int64_t)leaf_tab[s * D + 0] * nr * p;
  if (D == 2) {
    // Y[j2][r1] = sum_j1 sigma[j2][j1] F1[r1][j1]; waves split the r1 tiles
    const double* sg = sigma + (int64_t)leaf * p * p;
    for (int tj = w; tj < ntile; tj += 4) {
      acc_t acc;
      zero(acc);
      for (int kk = 0; kk < ksteps; kk++) {
        const int k = 4 * kk + lk;
        const int r1 = 16 * tj + lr;
        T a = (lr < p && k < p) ? (T)sg[lr * p + k] : (T)0;
        T b = (r1 < nr && k < p) ? F1[r1 * p + k] : (T)0;
        acc = Mfma<T>::step(a, b, acc);
      }
      const int r1 = 16 * tj + lr;
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const int j2 = Mfma<T>::row(lk, t);
        if (j2 < p && r1 < nr) Y[(int64_t)s * p * nr + j2 * nr + r1] = acc[t];
      }
    }
    return;
  }
  // D == 3
  const T* F2 = F + (int64_t)leaf_tab[s * D + 1] * nr * p;
  const int p3 = p * p * p;
  T* sS = smem;                         // [p^3]
  T* Xs = smem + p3 + w * 16 * nrp;     // per wave [16][nrp]
  const double* sg = sigma + (int64_t)leaf * p3;
  for (int idx = threadIdx.x; idx < p3; idx += blockDim.x) sS[idx] = (T)sg[idx];
  __syncthreads();
  const int nit = (p + 3) >> 2;
  const int64_t ybase = (int64_t)s * p * nr * nr;
  for (int it = 0; it < nit; it++) {
    const int j3 = w + 4 * it;
    const bool active = j3 < p;
    if (active) {
      // X[j2][r1] = sum_j1 sigma[j3][j2][j1] F1[r1][j1]
      for (int tj = 0; tj < ntile; tj++) {
        acc_t acc;
        zero(acc);
        const int r1 = 16 * tj + lr;
        for (int kk = 0; kk < ksteps; kk++) {
          const int k = 4 * kk + lk;
          T a = (lr < p && k < p) ? sS[(j3 * p + lr) * p + k] : (T)0;
          T b = (r1 < nr && k < p) ? F1[r1 * p + k] : (T)0;
          acc = Mfma<T>::step(a, b, acc);
        }
#pragma unroll
        for (int t = 0; t < 4; t++) Xs[(Mfma<T>::row(lk, t)) * nrp + r1] = acc[t];
      }
    }
    __syncthreads();
    if (active) {
      // Y[j3][r2][r1] = sum_j2 F2[r2][j2] X[j2][r1]
      for (int ti = 0; ti < ntile; ti++) {
        const int r2a = 16 * ti + lr;
        for (int tj = 0; tj < ntile; tj++) {
          acc_t acc;
          zero(acc);
          for (int kk = 0; kk < ksteps; kk++) {
            const int k = 4 * kk + lk;
            T a = (r2a < nr && k < p) ? F2[r2a * p + k] : (T)0;
            T b = (k < p) ? Xs[k * nrp + 16 * tj + lr] : (T)0;
            acc = Mfma<T>::step(a, b, acc);
          }
          const int r1 = 16 * tj + lr;
#pragma unroll
          for (int t = 0; t < 4; t++) {
            const int r2 = 16 * ti + Mfma<T>::row(lk, t);
            if (r2 < nr && r1 < nr) Y[ybase + ((int64_t)j3 * nr + r2) * nr + r1] = acc[t];
          }
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// form_box: phi_A[r][c] = sum_{s in A} sum_j F_s[r][j] Y_s[j][c]  (c < nr^(d-1))

template <typename T, int D>
__global__ __launch_bounds__(256) void k_form_box(const T* __restrict__ Y,
                                                  const int32_t* __restrict__ pw_start,
                                                  const int32_t* __restrict__ leaf_tab,
                                                  const T* __restrict__ F, int p, int nr,
                                                  int ncoltiles, T* __restrict__ phi) {
  typedef typename Mfma<T>::acc acc_t;
  const int A = blockIdx.x / ncoltiles;
  const int ct = blockIdx.x % ncoltiles;
  const int lane = lane_id(), w = wave_id();
  const int lr = lane & 15, lk = lane >> 4;
  int N2 = 1;
  for (int a = 1; a < D; a++) N2 *= nr;
  const int col = ct * 64 + w * 16 + lr;
  const int ntile = (nr + 15) >> 4;
  const int ksteps = (p + 3) >> 2;
  acc_t acc[kMaxRowTiles];
#pragma unroll
  for (int ti = 0; ti < kMaxRowTiles; ti++) zero(acc[ti]);
  const int s0 = pw_start[A], s1 = pw_start[A + 1];
  for (int s = s0; s < s1; s++) {
    const T* Fs = F + (int64_t)leaf_tab[s * D + (D - 1)] * nr * p;
    const T* Ys = Y + (int64_t)s * p * N2;
    for (int kk = 0; kk < ksteps; kk++) {
      const int k = 4 * kk + lk;
      T b = (k < p && col < N2) ? Ys[(int64_t)k * N2 + col] : (T)0;
#pragma unroll
      for (int ti = 0; ti < kMaxRowTiles; ti++) {
        if (ti < ntile) {
          const int r = 16 * ti + lr;
          T a = (r < nr && k < p) ? Fs[r * p + k] : (T)0;
          acc[ti] = Mfma<T>::step(a, b, acc[ti]);
        }
      }
    }
  }
  const int64_t base = (int64_t)A * nr * N2;
#pragma unroll
  for (int ti = 0; ti < kMaxRowTiles; ti++) {
    if (ti < ntile) {
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const int r = 16 * ti + Mfma<T>::row(lk, t);
        if (r < nr && col < N2) phi[base + (int64_t)r * N2 + col] = acc[ti][t];
      }
    }
  }
}

template <typename T, int D, bool R2F>
__global__ __launch_bounds__(256) void k_translate(const T* __restrict__ phi,
                                                   const int32_t* __restrict__ plist_start,
                                                   const int32_t* __restrict__ plist_src,
                                                   const int32_t* __restrict__ plist_dir,
                                                   const T* __restrict__ rot, int M, int nr,
                                                   int nA, T* __restrict__ psi) {
  translate_body<T, D, R2F>(phi, plist_start, plist_src, plist_dir, rot, M, nr, nA, psi, blockIdx.x);
}

// The same stage for many transforms in one launch.  Every transform's block
// range starts at a multiple of 8, so block b of a transform still runs on XCD
// b % 8 and the deal of chunks and box ranges above is kept.
template <typename T, int D, bool R2F>
__global__ __launch_bounds__(256) void k_translate_batched(const BatchJob* __restrict__ jobs,
                                                           const int32_t* __restrict__ start,
                                                           const int32_t* __restrict__ count,
                                                           int njobs) {
  const int j = batch_job_of(start, njobs, blockIdx.x);
  const int bid = blockIdx.x - start[j];
  if (bid >= count[j]) return;
  const DeviceArgs& a = jobs[j].a;
  translate_body<T, D, R2F>(static_cast<const T*>(a.phi), a.plist_start, a.plist_src, a.plist_dir,
                            static_cast<const T*>(a.rot), a.M, a.nr, (int)a.nA,
                            static_cast<T*>(const_cast<void*>(a.psi)), bid);
}

template <typename T>
void launch_translate_batched(int d, const BatchJob* jobs, const int32_t* start,
                              const int32_t* count, int njobs, int64_t grid, hipStream_t st) {
  if (d == 2)
    hipLaunchKernelGGL((k_translate_batched<T, 2, false>), dim3((unsigned)grid), dim3(256), 0, st, jobs,
                       start, count, njobs);
  else
    hipLaunchKernelGGL((k_translate_batched<T, 3, true>), dim3((unsigned)grid), dim3(256), 0, st, jobs,
                       start, count, njobs);
}
template void launch_translate_batched<double>(int, const BatchJob*, const int32_t*, const int32_t*,
                                               int, int64_t, hipStream_t);
template void launch_translate_batched<float>(int, const BatchJob*, const int32_t*, const int32_t*,
                                              int, int64_t, hipStream_t);

int64_t translate_blocks(const DeviceArgs& a) {
  int64_t nblk = 1;
  for (int i = 0; i < a.d; i++) nblk *= a.M;
  const int64_t nch = (nblk + 255) / 256, nbx = (a.nA + kXcds - 1) / kXcds;
  const int64_t rounds = nch / kXcds, rem = nch - rounds * kXcds;
  return kXcds * (rounds * a.nA + rem * nbx);
}

// ---------------------------------------------------------------------------
// eval_box: Z_s[i][c] = sum_r E_s[i][r] psi_A[r][c] for up to 64 stacked rows
// (count*p) of leaves of one box A.

template <typename T, int D>
__global__ __launch_bounds__(256) void k_eval_box(const T* __restrict__ psi,
                                                  const int32_t* __restrict__ echunk,
                                                  const int32_t* __restrict__ leaf_tab,
                                                  const T* __restrict__ E, int p, int nr,
                                                  int ncoltiles, T* __restrict__ Z) {
  typedef typename Mfma<T>::acc acc_t;
  const int item = blockIdx.x / ncoltiles;
  const int ct = blockIdx.x % ncoltiles;
  const int A = echunk[3 * item], s0 = echunk[3 * item + 1], cnt = echunk[3 * item + 2];
  const int lane = lane_id(), w = wave_id();
  const int lr = lane & 15, lk = lane >> 4;
  int N2 = 1;
  for (int a = 1; a < D; a++) N2 *= nr;
  const int col = ct * 64 + w * 16 + lr;
  const int ksteps = (nr + 3) >> 2;
  // the A-operand row of this lane in each of the 4 row tiles
  const T* erow[4];
  bool valid[4];
#pragma unroll
  for (int ti = 0; ti < 4; ti++) {
    const int row = 16 * ti + lr;
    const int ls = row / p, i = row % p;
    valid[ti] = ls < cnt;
    erow[ti] = valid[ti] ? E + ((int64_t)leaf_tab[(s0 + ls) * D + (D - 1)] * p + i) * nr : E;
  }
  acc_t acc[4];
#pragma unroll
  for (int ti = 0; ti < 4; ti++) zero(acc[ti]);
  const T* P = psi + (int64_t)A * nr * N2;
  for (int kk = 0; kk < ksteps; kk++) {
    const int k = 4 * kk + lk;
    T b = (k < nr && col < N2) ? P[(int64_t)k * N2 + col] : (T)0;
#pragma unroll
    for (int ti = 0; ti < 4; ti++) {
      T a = (valid[ti] && k < nr) ? erow[ti][k] : (T)0;
      acc[ti] = Mfma<T>::step(a, b, acc[ti]);
    }
  }
#pragma unroll
  for (int ti = 0; ti < 4; ti++) {
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int row = 16 * ti + Mfma<T>::row(lk, t);
      const int ls = row / p, i = row % p;
      if (ls < cnt && col < N2) Z[((int64_t)(s0 + ls) * p + i) * N2 + col] = acc[ti][t];
    }
  }
}

// ---------------------------------------------------------------------------
// eval_leaf: u_s = contraction of Z_s with the evaluation tables of axes d-1..1

template <typename T, int D>
__global__ __launch_bounds__(256) void k_eval_leaf(const T* __restrict__ Z,
                                                   const int32_t* __restrict__ leaf_id,
                                                   const int32_t* __restrict__ leaf_tab,
                                                   const T* __restrict__ E, int p, int nr,
                                                   double* __restrict__ u) {
  typedef typename Mfma<T>::acc acc_t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int s = blockIdx.x;
  const int leaf = leaf_id[s];
  const int lane = lane_id(), w = wave_id();
  const int lr = lane & 15, lk = lane >> 4;
  const int nrp = (nr + 15) & ~15;
  const int ntile = nrp >> 4;
  const int kr = (nr + 3) >> 2;
  if (D == 1) {
    for (int i = threadIdx.x; i < p; i += blockDim.x) u[(int64_t)leaf * p + i] = (double)Z[(int64_t)s * p + i];
    return;
  }
  const T* E1 = E + (int64_t)leaf_tab[s * D + 0] * p * nr;
  if (D == 2) {
    if (w != 0) return;
    // u[i2][i1] = sum_r1 Z[i2][r1] E1[i1][r1]
    const T* Zs = Z + (int64_t)s * p * nr;
    acc_t acc;
    zero(acc);
    for (int kk = 0; kk < kr; kk++) {
      const int k = 4 * kk + lk;
      T a = (lr < p && k < nr) ? Zs[lr * nr + k] : (T)0;
      T b = (lr < p && k < nr) ? E1[lr * nr + k] : (T)0;
      acc = Mfma<T>::step(a, b, acc);
    }
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int i2 = Mfma<T>::row(lk, t);
      if (i2 < p && lr < p) u[(int64_t)leaf * p * p + i2 * p + lr] = (double)acc[t];
    }
    return;
  }
  // D == 3
  const T* E2 = E + (int64_t)leaf_tab[s * D + 1] * p * nr;
  T* Ws = smem + w * nrp * 16;  // per wave [nrp][16]
  const int nit = (p + 3) >> 2;
  for (int it = 0; it < nit; it++) {
    const int i3 = w + 4 * it;
    const bool active = i3 < p;
    if (active) {
      // W[r2][i1] = sum_r1 Z[i3][r2][r1] E1[i1][r1]
      const T* Zs = Z + ((int64_t)s * p + i3) * nr * nr;
      for (int ti = 0; ti < ntile; ti++) {
        acc_t acc;
        zero(acc);
        const int r2a = 16 * ti + lr;
        for (int kk = 0; kk < kr; kk++) {
          const int k = 4 * kk + lk;
          T a = (r2a < nr && k < nr) ? Zs[r2a * nr + k] : (T)0;
          T b = (lr < p && k < nr) ? E1[lr * nr + k] : (T)0;
          acc = Mfma<T>::step(a, b, acc);
        }
#pragma unroll
        for (int t = 0; t < 4; t++) Ws[(16 * ti + Mfma<T>::row(lk, t)) * 16 + lr] = acc[t];
      }
    }
    __syncthreads();
    if (active) {
      // u[i3][i2][i1] = sum_r2 E2[i2][r2] W[r2][i1]
      acc_t acc;
      zero(acc);
      for (int kk = 0; kk < kr; kk++) {
        const int k = 4 * kk + lk;
        T a = (lr < p && k < nr) ? E2[lr * nr + k] : (T)0;
        T b = (k < nr) ? Ws[k * 16 + lr] : (T)0;
        acc = Mfma<T>::step(a, b, acc);
      }
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const int i2 = Mfma<T>::row(lk, t);
        if (i2 < p && lr < p) u[(int64_t)leaf * p * p * p + (i3 * p + i2) * p + lr] = (double)acc[t];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// near: u_T (+)= sum_{S in D(T)} (V_d (x) ... (x) V_1) sigma_S  (Lemma directbox)

template <typename T, int D>
__global__ __launch_bounds__(256) void k_near(const double* __restrict__ sigma,
                                              const int32_t* __restrict__ near_tgt,
                                              const int32_t* __restrict__ near_haspw,
                                              const int32_t* __restrict__ near_start,
                                              const int32_t* __restrict__ near_src,
                                              const int32_t* __restrict__ near_tab,
                                              const T* __restrict__ V, int p,
                                              double* __restrict__ u) {
  typedef typename Mfma<T>::acc acc_t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int t = blockIdx.x;
  const int T_leaf = near_tgt[t];
  const bool add = near_haspw[t] != 0;
  const int q0 = near_start[t], q1 = near_start[t + 1];
  const int lane = lane_id(), w = wave_id();
  const int lr = lane & 15, lk = lane >> 4;
  const int ks = (p + 3) >> 2;
  const int pp = p * p;
  if (D == 1) {
    if (threadIdx.x >= 64) return;
    double acc = 0.0;
    for (int q = q0; q < q1; q++) {
      const T* Vq = V + (int64_t)near_tab[q] * pp;
      const double* sg = sigma + (int64_t)near_src[q] * p;
      if (lane < p) {
        T s = 0;
        for (int j = 0; j < p; j++) s += Vq[lane * p + j] * (T)sg[j];
        acc += (double)s;
      }
    }
    if (lane < p) {
      double* ut = u + (int64_t)T_leaf * p;
      ut[lane] = add ? ut[lane] + acc : acc;
    }
    return;
  }
  if (D == 2) {
    // waves split the sources; partial results are summed in wave order
    T* t1 = smem + w * 256;        // per wave [16][16]
    T* red = smem + 4 * 256;       // [4][16][16]
    acc_t acc;
    zero(acc);
    const int nsrc = q1 - q0;
    const int nit = (nsrc + 3) >> 2;
    for (int it = 0; it < nit; it++) {
      const int q = q0 + w + 4 * it;
      const bool active = q < q1;
      const T* V1 = V;
      const T* V2 = V;
      if (active) {
        V1 = V + (int64_t)near_tab[q * 2 + 0] * pp;
        V2 = V + (int64_t)near_tab[q * 2 + 1] * pp;
        const double* sg = sigma + (int64_t)near_src[q] * pp;
        // t1[j2][i1] = sum_j1 sigma[j2][j1] V1[i1][j1]
        acc_t a1;
        zero(a1);
        for (int kk = 0; kk < ks; kk++) {
          const int k = 4 * kk + lk;
          T a = (lr < p && k < p) ? (T)sg[lr * p + k] : (T)0;
          T b = (lr < p && k < p) ? V1[lr * p + k] : (T)0;
          a1 = Mfma<T>::step(a, b, a1);
        }
#pragma unroll
        for (int tt = 0; tt < 4; tt++) t1[(Mfma<T>::row(lk, tt)) * 16 + lr] = a1[tt];
      }
      __syncthreads();
      if (active) {
        // acc[i2][i1] += sum_j2 V2[i2][j2] t1[j2][i1]
        for (int kk = 0; kk < ks; kk++) {
          const int k = 4 * kk + lk;
          T a = (lr < p && k < p) ? V2[lr * p + k] : (T)0;
          T b = (k < p) ? t1[k * 16 + lr] : (T)0;
          acc = Mfma<T>::step(a, b, acc);
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int tt = 0; tt < 4; tt++) red[w * 256 + (Mfma<T>::row(lk, tt)) * 16 + lr] = acc[tt];
    __syncthreads();
    if (w == 0) {
      double* ut = u + (int64_t)T_leaf * pp;
#pragma unroll
      for (int tt = 0; tt < 4; tt++) {
        const int i2 = Mfma<T>::row(lk, tt);
        const int o = i2 * 16 + lr;
        double v = (double)red[o];
        v += (double)red[256 + o];
        v += (double)red[512 + o];
        v += (double)red[768 + o];
        if (i2 < p && lr < p) ut[i2 * p + lr] = add ? ut[i2 * p + lr] + v : v;
      }
    }
    return;
  }
  // D == 3
  const int p3 = pp * p;
  T* sS = smem;             // [p^3] sigma_S, then t2[j3][i2*p+i1]
  T* t1 = smem + p3;        // [p^2][16]: t1[(j3,j2)][i1]
  const int nrt = (pp + 15) >> 4;  // row / column tiles of p^2
  const int nct_w = (nrt + 3) >> 2;  // step-3 column tiles per wave
  acc_t acc[4];
#pragma unroll
  for (int c = 0; c < 4; c++) zero(acc[c]);
  for (int q = q0; q < q1; q++) {
    const T* V1 = V + (int64_t)near_tab[q * 3 + 0] * pp;
    const T* V2 = V + (int64_t)near_tab[q * 3 + 1] * pp;
    const T* V3 = V + (int64_t)near_tab[q * 3 + 2] * pp;
    const double* sg = sigma + (int64_t)near_src[q] * p3;
    __syncthreads();
    for (int idx = threadIdx.x; idx < p3; idx += blockDim.x) sS[idx] = (T)sg[idx];
    __syncthreads();
    // step 1: t1[(j3,j2)][i1] = sum_j1 sigma[j3][j2][j1] V1[i1][j1]
    for (int rt = w; rt < nrt; rt += 4) {
      acc_t a1;
      zero(a1);
      const int row = 16 * rt + lr;
      for (int kk = 0; kk < ks; kk++) {
        const int k = 4 * kk + lk;
        T a = (row < pp && k < p) ? sS[row * p + k] : (T)0;
        T b = (lr < p && k < p) ? V1[lr * p + k] : (T)0;
        a1 = Mfma<T>::step(a, b, a1);
      }
#pragma unroll
      for (int tt = 0; tt < 4; tt++) {
        const int r = 16 * rt + Mfma<T>::row(lk, tt);
        if (r < pp) t1[r * 16 + lr] = a1[tt];
      }
    }
    __syncthreads();
    // step 2: t2[j3][i2][i1] = sum_j2 V2[i2][j2] t1[(j3,j2)][i1]  (into sS)
    for (int j3 = w; j3 < p; j3 += 4) {
      acc_t a2;
      zero(a2);
      for (int kk = 0; kk < ks; kk++) {
        const int k = 4 * kk + lk;
        T a = (lr < p && k < p) ? V2[lr * p + k] : (T)0;
        T b = (k < p) ? t1[(j3 * p + k) * 16 + lr] : (T)0;
        a2 = Mfma<T>::step(a, b, a2);
      }
#pragma unroll
      for (int tt = 0; tt < 4; tt++) {
        const int i2 = Mfma<T>::row(lk, tt);
        if (i2 < p && lr < p) sS[j3 * pp + i2 * p + lr] = a2[tt];
      }
    }
    __syncthreads();
    // step 3: acc[i3][c] += sum_j3 V3[i3][j3] t2[j3][c],  c = i2*p + i1
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const int ct = w + 4 * c;
      if (c < nct_w && ct < nrt) {
        const int colc = 16 * ct + lr;
        for (int kk = 0; kk < ks; kk++) {
          const int k = 4 * kk + lk;
          T a = (lr < p && k < p) ? V3[lr * p + k] : (T)0;
          T b = (k < p && colc < pp) ? sS[k * pp + colc] : (T)0;
          acc[c] = Mfma<T>::step(a, b, acc[c]);
        }
      }
    }
  }
  double* ut = u + (int64_t)T_leaf * p3;
#pragma unroll
  for (int c = 0; c < 4; c++) {
    const int ct = w + 4 * c;
    if (c < nct_w && ct < nrt) {
      const int colc = 16 * ct + lr;
#pragma unroll
      for (int tt = 0; tt < 4; tt++) {
        const int i3 = Mfma<T>::row(lk, tt);
        if (i3 < p && colc < pp) {
          const int64_t o = (int64_t)i3 * pp + colc;
          ut[o] = add ? ut[o] + (double)acc[c][tt] : (double)acc[c][tt];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// launchers

static inline int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; i++) r *= b;
  return r;
}

size_t lds_form_leaf(int d, int p, int nr, size_t tsize) {
  if (d < 3) return 0;
  const int nrp = (nr + 15) & ~15;
  return tsize * ((size_t)p * p * p + 4 * 16 * (size_t)nrp);
}
size_t lds_eval_leaf(int d, int p, int nr, size_t tsize) {
  (void)p;
  if (d < 3) return 0;
  const int nrp = (nr + 15) & ~15;
  return tsize * 4 * 16 * (size_t)nrp;
}
size_t lds_near(int d, int p, size_t tsize) {
  if (d == 2) return tsize * 8 * 256;
  if (d == 3) return tsize * ((size_t)p * p * p + (size_t)p * p * 16);
  return 0;
}

template <typename T, int D>
static hipError_t launch_all(const DeviceArgs& a, const double* sigma, double* u,
                             hipStream_t st, hipEvent_t* ev) {
  const int p = a.p, nr = a.nr;
  const T* F = static_cast<const T*>(a.F);
  const T* E = static_cast<const T*>(a.E);
  const T* V = static_cast<const T*>(a.V);
  const T* rot = static_cast<const T*>(a.rot);
  T* Y = static_cast<T*>(a.Y);
  T* phi = static_cast<T*>(a.phi);
  T* psi = static_cast<T*>(a.psi);
  const int N2 = ipow(nr, D - 1);
  const int ncol = (N2 + 63) / 64;
  auto rec = [&](int i) { if (ev) (void)hipEventRecord(ev[i], st); };
  rec(0);
  if (a.nL > 0) {
    hipLaunchKernelGGL((k_form_leaf<T, D>), dim3(a.nL), dim3(256),
                       lds_form_leaf(D, p, nr, sizeof(T)), st, sigma, a.pwleaf_id, a.pwleaf_tab,
                       F, p, nr, Y);
    rec(1);
    hipLaunchKernelGGL((k_form_box<T, D>), dim3((unsigned)(a.nA * ncol)), dim3(256), 0, st, Y,
                       a.pw_start, a.pwleaf_tab, F, p, nr, ncol, phi);
    rec(2);
    launch_translate<T>(a, st);
    rec(3);
    hipLaunchKernelGGL((k_eval_box<T, D>), dim3((unsigned)(a.nE * ncol)), dim3(256), 0, st, psi,
                       a.echunk, a.pwleaf_tab, E, p, nr, ncol, Y);
    rec(4);
    hipLaunchKernelGGL((k_eval_leaf<T, D>), dim3(a.nL), dim3(256),
                       lds_eval_leaf(D, p, nr, sizeof(T)), st, Y, a.pwleaf_id, a.pwleaf_tab, E,
                       p, nr, u);
    rec(5);
  } else {
    for (int i = 1; i <= 5; i++) rec(i);
  }
  if (a.nT > 0) {
    hipLaunchKernelGGL((k_near<T, D>), dim3(a.nT), dim3(256), lds_near(D, p, sizeof(T)), st,
                       sigma, a.near_tgt, a.near_haspw, a.near_start, a.near_src, a.near_tab, V,
                       p, u);
  }
  rec(6);
  return hipGetLastError();
}

template <typename T>
void launch_translate(const DeviceArgs& a, hipStream_t st) {
  const unsigned grid = (unsigned)translate_blocks(a);
  const T* phi = static_cast<const T*>(a.phi);
  const T* rot = static_cast<const T*>(a.rot);
  T* psi = static_cast<T*>(a.psi);
  const int nA = (int)a.nA;
  switch (a.d) {
    case 1:
      hipLaunchKernelGGL((k_translate<T, 1, false>), dim3(grid), dim3(256), 0, st, phi, a.plist_start,
                         a.plist_src, a.plist_dir, rot, a.M, a.nr, nA, psi);
      break;
    case 2:
      hipLaunchKernelGGL((k_translate<T, 2, false>), dim3(grid), dim3(256), 0, st, phi, a.plist_start,
                         a.plist_src, a.plist_dir, rot, a.M, a.nr, nA, psi);
      break;
    default:
      hipLaunchKernelGGL((k_translate<T, 3, true>), dim3(grid), dim3(256), 0, st, phi, a.plist_start,
                         a.plist_src, a.plist_dir, rot, a.M, a.nr, nA, psi);
      break;
  }
}
template void launch_translate<double>(const DeviceArgs&, hipStream_t);
template void launch_translate<float>(const DeviceArgs&, hipStream_t);

hipError_t launch_transform(const DeviceArgs& a, const double* sigma, double* u, hipStream_t st,
                            hipEvent_t* ev) {
  if (a.d >= 2) return launch_fast(a, sigma, u, st, ev);
  if (a.fp32) return launch_all<float, 1>(a, sigma, u, st, ev);
  return launch_all<double, 1>(a, sigma, u, st, ev);
}

}  // namespace fgt
