// Device bodies of the tuned stages of the box Gauss transform (d = 2, 3),
// shared by the per-stage kernels (kernels_fast.hip) and the persistent
// batched kernels (persist.hip).
//
// Tile counts are compile time: NT = ceil(nr/16) mode tiles per axis and
// KS = ceil(p/4) node steps (FP32 always runs 4 node steps, see mfma.h).
// Node axes are padded to 16 inside a tile.  Chained contractions pass result
// tiles from one matrix-core product to the next in registers (mfma.h); LDS is
// used only where a contraction runs across the tiles held by different waves.
//
// d = 3:
//   form3_plane Y_P[j3][r1][r2] = sum_{rows} F1_row[r1][j1] (sum_{s in row} sum_j2 sigma_s[j3][j2][j1] F2_s[r2][j2])
//   form_box    phi_A[r3][c]    = sum_{P in A} sum_j3 F3_P[r3][j3] Y_P[j3][c]
//   translate   psi_A = sum_{B in P(A)} Rot(c_B - c_A) phi_B        (kernels.hip)
//   eval_box    Z_P[i3][c]      = sum_r3 E3_P[i3][r3] psi_A[r3][c]
//   eval3_plane u_s[i3][i2][i1] = sum_r2 E2_s[i2][r2] (sum_r1 Z_P[i3][r1][r2] E1_row[i1][r1])
// (P: a plane of leaves sharing level and axis-3 table; row: leaves of a plane
// sharing the axis-1 table.  Grouping the sums this way is exact: each table
// factor is applied once to the sum of everything it multiplies.)
//   near3       u_T (+)= sum_S (V3 (x) V2 (x) V1) sigma_S, grouped by tables
// The mode tensors phi, psi, Y, Z of d = 3 are stored with the r2 index fastest
// ([r3][r1][r2]), so that every global operand load runs along a contiguous axis.
// d = 2 fuses formation and evaluation per box / per leaf (no intermediate).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "kernels.h"
#include "mfma.h"

namespace fgt {

__device__ __forceinline__ int lane_of() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_of() { return threadIdx.x >> 6; }

// r2 tiles per form3_plane work item: all of them while the y accumulators
// (NT x TG tiles) stay small, fewer for large NT.
__host__ __device__ constexpr int form3_tile_group(int nt) { return nt <= 4 ? nt : (nt == 5 ? 3 : 2); }

// k-steps of a node contraction (K = p <= 4 KS): chained operands need the
// register layout, which for FP32 and BF16x3 spreads K over all four steps;
// when both operands come from memory (MemSteps, k = Mfma::kmem) FP32 needs
// only KS.  BF16x3 products always span four steps.
template <typename C, int KS>
struct Steps {
  static constexpr int value = std::is_same<C, double>::value ? KS : 4;
};
template <typename C, int KS>
struct MemSteps {
  static constexpr int value = std::is_same<C, Bf16x3>::value ? 4 : KS;
};

// ---------------------------------------------------------------------------
// d = 3 formation, axes 2 and 1, per plane.  A plane is a run of leaves of one
// cutoff box with the same level and axis-3 position; its rows also share the
// axis-1 position (fgt_host.h).  By separability
//   Y_P[j3][r1][r2] = sum_rows F1_row[r1][j1] (sum_{s in row} sum_j2 sigma_s[j3][j2][j1] F2_s[r2][j2])
// and the last axis then runs once per plane instead of once per leaf.  A wave
// owns one item (j3 slice, group of TG r2 tiles); 4 items per workgroup, which
// share the plane's F2 and F1 tables through LDS:
//   X^T[j1][r2] += sigma_s[j3] x F2_s      over the leaves of a row (lanes along j1)
//   Y[r1][r2]   += F1_row x X^T            once per row (X^T chained as the B operand)

template <typename C, int NT, int KS>
__device__ __forceinline__ void form3_plane_body(const double* __restrict__ sigma,
                                                 const int32_t* __restrict__ leaf_id,
                                                 const int32_t* __restrict__ leaf_tab,
                                                 const int32_t* __restrict__ plane_order,
                                                 const int32_t* __restrict__ plane_row,
                                                 const int32_t* __restrict__ row_start,
                                                 const int32_t* __restrict__ row_tab,
                                                 const elem_t<C>* __restrict__ F, int p, int nr,
                                                 elem_t<C>* __restrict__ Y, int bid) {
  typedef elem_t<C> T;
  typedef Mfma<C> M;
  typedef typename M::acc acc_t;
  constexpr int S = Steps<C, KS>::value;      // chained (X^T as the B operand of Y)
  constexpr int SM = MemSteps<C, KS>::value;  // sigma x F2, both from memory
  constexpr int TG = form3_tile_group(NT), NG = (NT + TG - 1) / TG;
  // the plane's tables, shared by the four waves, staged in LDS: F2 of the
  // current and next leaf, F1 of the current row ([r][k], k stride 17)
  constexpr int KP = 17, TR = 16 * NT, TSZ = TR * KP;
  __shared__ T tabs[3 * TSZ];
  const int nitem = p * NG, nsplit = (nitem + 3) / 4;
  const int P = plane_order[bid / nsplit];  // planes with most work first
  const int lane = lane_of(), w = wave_of();
  const int item = (bid - (bid / nsplit) * nsplit) * 4 + w;
  const bool active = item < nitem;  // inactive waves still stage tables and meet the barriers
  const int j3 = active ? item / NG : 0, t0 = active ? (item - j3 * NG) * TG : 0;
  const int lr = lane & 15, lk = lane >> 4;
  const int rw0 = plane_row[P], rw1 = plane_row[P + 1];
  const int s_begin = row_start[rw0], s_end = row_start[rw1];
  const int64_t ppp = (int64_t)p * p * p;
  const int tid = threadIdx.x;
  // table t (nr x p) into LDS buffer buf, zero past nr / p
  auto stage = [&](const T* tab, int buf) {
    for (int e = tid; e < TR * 16; e += (int)blockDim.x) {
      const int r = e >> 4, k = e & 15;
      tabs[buf * TSZ + r * KP + k] = ld0<T>(tab, r * p + k, r < nr && k < p);
    }
  };
  auto load_av = [&](int s, T (&av)[SM]) {
    const bool ls = s < s_end;
    const int sc = ls ? s : s_begin;
    const double* sg = sigma + (int64_t)leaf_id[sc] * ppp;
#pragma unroll
    for (int kk = 0; kk < SM; kk++) {
      const int k = M::kmem(kk, lk);
      av[kk] = ld0<T>(sg, (j3 * p + k) * p + lr, ls && active && lr < p && k < p);  // A[j1][j2]
    }
  };
  acc_t y[NT][TG];
#pragma unroll
  for (int tj = 0; tj < NT; tj++)
#pragma unroll
    for (int g = 0; g < TG; g++) zero4(y[tj][g]);
  acc_t x[TG];
#pragma unroll
  for (int g = 0; g < TG; g++) zero4(x[g]);
  T av[SM];
  load_av(s_begin, av);
  stage(F + (int64_t)leaf_tab[s_begin * 3 + 1] * nr * p, 0);
  __syncthreads();
  int rw = rw0;
  int row_end = row_start[rw0 + 1];
  for (int s = s_begin; s < s_end; s++) {
    const int cur = (s - s_begin) & 1;
    T avn[SM];
    load_av(s + 1, avn);
    if (s + 1 < s_end) stage(F + (int64_t)leaf_tab[(s + 1) * 3 + 1] * nr * p, cur ^ 1);
    if (active) {
#pragma unroll
      for (int g = 0; g < TG; g++) {
        T b2[SM];
#pragma unroll
        for (int kk = 0; kk < SM; kk++) {
          const int k = M::kmem(kk, lk);
          b2[kk] = tabs[cur * TSZ + (16 * (t0 + g) + lr) * KP + k];  // B[j2][r2] = F2[r2][j2]
        }
        x[g] = M::template steps<SM>(av, b2, x[g]);
      }
    }
    if (s + 1 == row_end) {
      stage(F + (int64_t)row_tab[rw] * nr * p, 2);
      __syncthreads();
      if (active) {
#pragma unroll
        for (int tj = 0; tj < NT; tj++) {
          T a1[S];
#pragma unroll
          for (int kk = 0; kk < S; kk++) a1[kk] = tabs[2 * TSZ + (16 * tj + lr) * KP + M::kidx(kk, lk)];  // A[r1][j1]
#pragma unroll
          for (int g = 0; g < TG; g++) {
            T xb[S];
#pragma unroll
            for (int kk = 0; kk < S; kk++) xb[kk] = x[g][kk];
            y[tj][g] = M::template steps<S>(a1, xb, y[tj][g]);
          }
        }
      }
#pragma unroll
      for (int g = 0; g < TG; g++) zero4(x[g]);
      rw++;
      if (rw < rw1) row_end = row_start[rw + 1];
    }
    __syncthreads();  // the next leaf's table is staged; this leaf's and row's are read
#pragma unroll
    for (int kk = 0; kk < SM; kk++) av[kk] = avn[kk];
  }
  if (!active) return;
  T* Yp = Y + (int64_t)P * p * nr * nr;
#pragma unroll
  for (int g = 0; g < TG; g++) {
    const int r2 = 16 * (t0 + g) + lr;
#pragma unroll
    for (int tj = 0; tj < NT; tj++)
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const int r1 = 16 * tj + M::row(lk, t);
        if (r1 < nr && r2 < nr) Yp[((int64_t)j3 * nr + r1) * nr + r2] = y[tj][g][t];
      }
  }
}

// ---------------------------------------------------------------------------
// last-axis formation merged over the leaves of a cutoff box (a grouped GEMM)

// Tile shape of form_box: 16-column slabs per wave (H); a workgroup covers
// 64 H columns.  fgt_execute uses kFormBoxSlabs = 2: with the table operand
// shared through LDS, 2 slabs (more waves per SIMD) beat 4 on the 3D benchmark
// tree; with the table loaded by every wave, 4 had beaten 2, 3 and 8.  The
// other shape, kFormBoxSlabsAlt, is kept for batched launches; the columns and
// the order of every sum are the same, so results are identical.
constexpr int kFormBoxSlabs = kFormBoxTileSlabs[0];
constexpr int kFormBoxSlabsAlt = kFormBoxTileSlabs[1];
__host__ __device__ constexpr int form_box_cols_of(int slabs) { return 64 * slabs; }

template <typename C, int D, int NT, int KS, int H>
__device__ __forceinline__ void form_box_body(const elem_t<C>* __restrict__ Y,
                                                const int32_t* __restrict__ fitem,
                                                const int32_t* __restrict__ leaf_tab,
                                                const elem_t<C>* __restrict__ F, int p, int nr,
                                                int ncoltiles, int nmodes, int tp, int64_t ncoef_phi,
                                                elem_t<C>* __restrict__ phi,
                                                elem_t<C>* __restrict__ partial, int bid) {
  typedef elem_t<C> T;
  // one work item (<= kFormLeaves units of a box) x 64 H columns per
  // workgroup; every wave owns H 16-column slabs, sharing the table operand
  // (staged in LDS)
  typedef Mfma<C> M;
  typedef typename M::acc acc_t;
  constexpr int S = MemSteps<C, KS>::value;  // Y and F3 both come from memory
  const int item = bid / ncoltiles;
  const int ct = bid % ncoltiles;
  const int A = fitem[4 * item], slot = fitem[4 * item + 3];
  const int lane = lane_of(), w = wave_of();
  const int lr = lane & 15, lk = lane >> 4;
  const int N2 = D == 3 ? nr * nr : nr;
  int col[H];
  bool colok[H];
#pragma unroll
  for (int h = 0; h < H; h++) {
    col[h] = ct * form_box_cols_of(H) + w * (16 * H) + 16 * h + lr;
    colok[h] = col[h] < N2;
  }
  acc_t acc[NT][H];
#pragma unroll
  for (int ti = 0; ti < NT; ti++)
#pragma unroll
    for (int h = 0; h < H; h++) zero4(acc[ti][h]);
  const int s0 = fitem[4 * item + 1], s1 = fitem[4 * item + 2];
  // the units' last-axis tables, shared by the four waves, staged in LDS ([r][k],
  // k stride 17), two buffers: the next unit's is written during the products
  constexpr int KP = 17, TSZ = 16 * NT * KP;
  __shared__ T tabs[2 * TSZ];
  const int tid = threadIdx.x;
  auto stage = [&](int s, int buf) {
    const T* Fs = F + (int64_t)leaf_tab[s * D + (D - 1)] * nr * p;
    for (int e = tid; e < 16 * NT * 16; e += (int)blockDim.x) {
      const int r = e >> 4, k = e & 15;
      tabs[buf * TSZ + r * KP + k] = ld0<T>(Fs, r * p + k, r < nr && k < p);
    }
  };
  // Y operands of unit s; loads are masked, not branched, so that no
  // control-flow join forces a wait for the prefetched unit before the products
  auto load = [&](int s, T (&bb)[S][H]) {
    const bool ls = s < s1;
    const int sc = ls ? s : s0;
    const T* Ys = Y + (int64_t)sc * p * N2;
#pragma unroll
    for (int kk = 0; kk < S; kk++) {
      const int k = M::kmem(kk, lk);
#pragma unroll
      for (int h = 0; h < H; h++) bb[kk][h] = ld0<T>(Ys, (int64_t)k * N2 + col[h], ls && k < p && colok[h]);
    }
  };
  T b[S][H];
  load(s0, b);
  stage(s0, 0);
  __syncthreads();
  for (int s = s0; s < s1; s++) {
    const int cur = (s - s0) & 1;
    T bn[S][H];
    load(s + 1, bn);
    if (s + 1 < s1) stage(s + 1, cur ^ 1);
    T a[NT][S];
#pragma unroll
    for (int ti = 0; ti < NT; ti++)
#pragma unroll
      for (int kk = 0; kk < S; kk++) a[ti][kk] = tabs[cur * TSZ + (16 * ti + lr) * KP + M::kmem(kk, lk)];
#pragma unroll
    for (int h = 0; h < H; h++) {
      T bh[S];
#pragma unroll
      for (int kk = 0; kk < S; kk++) bh[kk] = b[kk][h];
#pragma unroll
      for (int ti = 0; ti < NT; ti++) acc[ti][h] = M::template steps<S>(a[ti], bh, acc[ti][h]);
    }
    __syncthreads();  // the next unit's table is staged; this one's is read
#pragma unroll
    for (int kk = 0; kk < S; kk++)
#pragma unroll
      for (int h = 0; h < H; h++) b[kk][h] = bn[kk][h];
  }
  // a box's only item writes phi; items of a split box write partial sums,
  // tile-major with tp pairs per tile when tp > 0 (d = 3, kernels.h)
  T* out = slot < 0 ? phi + (int64_t)A * ncoef_phi : partial + (int64_t)slot * ncoef_phi;
  const bool tiled = D == 3 && tp > 0;
  const int64_t rstride = tiled ? 4 * tp : N2;
  int64_t coff[H];
#pragma unroll
  for (int h = 0; h < H; h++)
    coff[h] = tiled && colok[h] ? phi_tiled_col(nmodes, tp, nr, col[h] / nr, col[h] - (col[h] / nr) * nr) : col[h];
#pragma unroll
  for (int ti = 0; ti < NT; ti++)
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int r = 16 * ti + M::row(lk, t);
#pragma unroll
      for (int h = 0; h < H; h++)
        if (r < nr && colok[h]) out[(int64_t)r * rstride + coff[h]] = acc[ti][h][t];
    }
}

// phi_A = sum of the partial sums of a split box, in item order (deterministic)
template <typename T>
__device__ __forceinline__ void reduce_partials_body(const T* __restrict__ partial,
                                                       const int32_t* __restrict__ fred,
                                                       int64_t ncoef, int nchunk,
                                                       T* __restrict__ phi, int bid) {
  const int r = bid / nchunk;
  const int64_t i = (int64_t)(bid % nchunk) * blockDim.x + threadIdx.x;
  if (i >= ncoef) return;
  const int A = fred[3 * r], slot0 = fred[3 * r + 1], n = fred[3 * r + 2];
  T s = 0;
  for (int k = 0; k < n; k++) s += partial[(int64_t)(slot0 + k) * ncoef + i];
  phi[(int64_t)A * ncoef + i] = s;
}

// ---------------------------------------------------------------------------
// d = 3 out->in translation fused with the first evaluation contraction.
// A workgroup owns one target group (up to kTeGroup neighboring cutoff boxes,
// with the union of their P-lists: fgt_host.h te_*) and one tile of mode-column
// pairs (m1, m2).  Phase 1: a thread owns one unit (m3, pair), the 2 x 2 x 2
// coefficients of the cos/sin members of m1, m2, m3 (four aligned pairs along
// r2, loaded as vectors); each source box of the group is loaded once and
// rotated into the accumulators of every member that takes it,
// psi_A = sum_{B in P(A)} Rot(c_B - c_A) phi_B.  The members' psi tiles are
// staged in LDS kTeSlots at a time; phase 2 contracts each with the axis-3
// evaluation table of every plane of its box, Z_P[i3][c] = sum_r3 E3_P[i3][r3]
// psi_A[r3][c], the (member, plane, 16-column group) items split evenly over
// the waves.  psi never goes to HBM.
constexpr int kTeSlots = 2;  // member tiles held in LDS at once

// LDS of the psi tiles: kTeSlots tiles of nr rows of 4 tp + 1 columns (odd,
// to spread the banks)
inline size_t transeval_lds(int tp, int nr, size_t ts) { return (size_t)kTeSlots * nr * (4 * tp + 1) * ts; }
// the most any plan of NT 16-row mode tiles needs: nr 4 tp <= 2048 (the tiles'
// 256 units of 8 coefficients) and nr <= 16 NT
inline size_t transeval_lds_max(int NT, size_t ts) { return (size_t)kTeSlots * (2048 + 16 * NT) * ts; }

// Translation of one unit's 8 coefficients (v = v1 + 2 v2 + 4 v3, bit a the
// sin member along axis a + 1) by one box along axis AX + 1 in direction DD:
// each (cos, sin) pair of that axis turns by the angle of its mode, the
// real form of the diagonal translation T_{out->in} of Eq. (diagonaltranslation)
// (c, s: cosine and sine of that angle for the unit's mode on the axis).  In
// place:
template <int AX, int DD, typename T>
__device__ __forceinline__ void te_rotate(T c, T sn, T (&y)[8]) {
  const T s = DD > 0 ? sn : -sn;
  constexpr int bit = 1 << AX;
#pragma unroll
  for (int v = 0; v < 8; v++) {
    if (v & bit) continue;
    const T xc = y[v], xs = y[v | bit];
    y[v] = c * xc - s * xs;
    y[v | bit] = s * xc + c * xs;
  }
}
// ... and accumulated: a += R y
template <int AX, int DD, typename T>
__device__ __forceinline__ void te_rotate_acc(T c, T sn, const T (&y)[8], T (&a)[8]) {
  const T s = DD > 0 ? sn : -sn;
  constexpr int bit = 1 << AX;
#pragma unroll
  for (int v = 0; v < 8; v++) {
    if (v & bit) continue;
    const T xc = y[v], xs = y[v | bit];
    a[v] = fma(c, xc, a[v]);
    a[v] = fma(-s, xs, a[v]);
    a[v | bit] = fma(s, xc, a[v | bit]);
    a[v | bit] = fma(c, xs, a[v | bit]);
  }
}
// a member's share of a source already turned along axis 3: a += R2 R1 y
template <int D1, int D2, typename T>
__device__ __forceinline__ void te_member(const T (&cs)[3], const T (&sn)[3], const T (&y)[8], T (&a)[8]) {
  if constexpr (D1 != 0 && D2 != 0) {
    T z[8];
#pragma unroll
    for (int v = 0; v < 8; v++) z[v] = y[v];
    te_rotate<0, D1>(cs[0], sn[0], z);
    te_rotate_acc<1, D2>(cs[1], sn[1], z, a);
  } else if constexpr (D1 != 0) {
    te_rotate_acc<0, D1>(cs[0], sn[0], y, a);
  } else if constexpr (D2 != 0) {
    te_rotate_acc<1, D2>(cs[1], sn[1], y, a);
  } else {
#pragma unroll
    for (int v = 0; v < 8; v++) a[v] += y[v];
  }
}

template <typename C, int NT>
__device__ __forceinline__ void transeval3_body(const elem_t<C>* __restrict__ phi,
                                                const int32_t* __restrict__ te_start,
                                                const int32_t* __restrict__ te_mem,
                                                const int32_t* __restrict__ te_src,
                                                const int32_t* __restrict__ te_dir,
                                                const int32_t* __restrict__ te_wg,
                                                const elem_t<C>* __restrict__ rot,
                                                const int32_t* __restrict__ plane_start,
                                                const int32_t* __restrict__ plane_tab,
                                                const elem_t<C>* __restrict__ E, int p, int M,
                                                int nr, int TP, elem_t<C>* __restrict__ Z,
                                                elem_t<C>* __restrict__ ps, int bid) {
  typedef elem_t<C> T;
  typedef typename Pair2<T>::type T2;
  typedef Mfma<C> M_;
  typedef typename M_::acc acc_t;
  constexpr int G = kTeGroup, S = kTeSlots, Q = 4 * NT;
  const int LDW = 4 * TP + 1;
  const int npair = M * M;
  const int ntile = (npair + TP - 1) / TP;
  // the plan's workgroup table: group and tile, longest first per XCD
  const int g = te_wg[2 * bid], tile = te_wg[2 * bid + 1];
  if (g < 0) return;  // whole workgroup
  const int j0 = tile * TP;
  const int tph = min(TP, npair - j0);  // pairs of this tile
  const int ncol = 4 * tph;             // column c = v1 (2 tph) + 2 jj + v2
  const int64_t nr2 = (int64_t)nr * nr;
  const int64_t ncoef = (int64_t)ntile * nr * 4 * TP;  // tile-major phi (kernels.h)
  const int tid = threadIdx.x;
  const bool active = tid < M * tph;
  const int m3 = active ? tid / tph : 0;
  const int jj = active ? tid - m3 * tph : 0;
  const int m1 = (j0 + jj) / M, m2 = (j0 + jj) - m1 * M;

  // ---- phase 1: translations of every member into registers
  T acc[G][8];
#pragma unroll
  for (int t = 0; t < G; t++)
#pragma unroll
    for (int v = 0; v < 8; v++) acc[t][v] = 0;
  const int e0 = te_start[g], e1 = te_start[g + 1];
  if (active && e0 < e1) {
    const T cs[3] = {rot[2 * m1], rot[2 * m2], rot[2 * m3]};
    const T sn[3] = {rot[2 * m1 + 1], rot[2 * m2 + 1], rot[2 * m3 + 1]};
    // coefficient v = v1 + 2 v2 + 4 v3 (bit a: sin member of the axis-(a+1)
    // pair); pair w = v1 + 2 v3 holds v2 = 0, 1 at off[w], off[w] + 1 of the
    // tile's block, whose rows are 4 TP apart
    int off[4];
#pragma unroll
    for (int w = 0; w < 4; w++) {
      const int v1 = w & 1, v3 = w >> 1;
      off[w] = (2 * m3 + v3) * 4 * TP + v1 * 2 * TP + 2 * jj;
    }
    const int64_t tile_off = (int64_t)tile * nr * 4 * TP;
    auto fetch = [&](int e, T (&x)[8]) {
      const T* src = phi + (int64_t)te_src[min(e, e1 - 1)] * ncoef + tile_off;
#pragma unroll
      for (int w = 0; w < 4; w++) {
        const T2 v2 = *reinterpret_cast<const T2*>(src + off[w]);
        const int v = (w & 1) | ((w >> 1) << 2);
        x[v] = v2.x;
        x[v | 2] = v2.y;
      }
    };
    // Members share the axis-3 offset of an entry's source (fgt_host.h), so
    // the source is rotated along axis 3 once, in place, and every member
    // then applies only its own axis-1 and axis-2 rotations, the last of them
    // straight into its accumulators; the offsets are compile-time constants
    // of te_member, selected by one uniform branch per member.
    auto members = [&](int e, T (&x)[8]) {
      constexpr int W = (G + 3) / 4;  // direction words per entry
      uint32_t wd[W];
#pragma unroll
      for (int i = 0; i < W; i++) wd[i] = (uint32_t)te_dir[W * e + i];
      uint32_t cmin = 0xFFu;  // any present member's code
#pragma unroll
      for (int t = 0; t < G; t++) cmin = min(cmin, (wd[t >> 2] >> (8 * (t & 3))) & 0xFFu);
      const int d3 = (int)(cmin / 9) - 1;
      if (d3 > 0) te_rotate<2, 1>(cs[2], sn[2], x);
      if (d3 < 0) te_rotate<2, -1>(cs[2], sn[2], x);
#pragma unroll
      for (int t = 0; t < G; t++) {
        const int code = (int)((wd[t >> 2] >> (8 * (t & 3))) & 0xFFu);
        if (code == kTeNoDir) continue;
        switch (code % 9) {  // (d1 + 1) + 3 (d2 + 1)
          case 0: te_member<-1, -1>(cs, sn, x, acc[t]); break;
          case 1: te_member<0, -1>(cs, sn, x, acc[t]); break;
          case 2: te_member<1, -1>(cs, sn, x, acc[t]); break;
          case 3: te_member<-1, 0>(cs, sn, x, acc[t]); break;
          case 4: te_member<0, 0>(cs, sn, x, acc[t]); break;
          case 5: te_member<1, 0>(cs, sn, x, acc[t]); break;
          case 6: te_member<-1, 1>(cs, sn, x, acc[t]); break;
          case 7: te_member<0, 1>(cs, sn, x, acc[t]); break;
          default: te_member<1, 1>(cs, sn, x, acc[t]); break;
        }
      }
    };
    // two sources in flight: the loads of entry e+1 are issued before the
    // rotations of entry e (an e past the list reloads the last source)
    T xa[8], xb[8];
    fetch(e0, xa);
    for (int e = e0; e < e1; e += 2) {
      fetch(e + 1, xb);
      members(e, xa);
      fetch(e + 2, xa);
      if (e + 1 < e1) members(e + 1, xb);
    }
  }

  // ---- phase 2, kTeSlots members at a time: Z_P[i3][c] = sum_r3 E3_P[i3][r3]
  // psi_A[r3][c].  A wave takes a contiguous run of (slot, plane, column
  // group) items and loads a plane's axis-3 table once for its column groups.
  // The K index of (group g, step kk) is 16 g + 4 lk + kk: a lane's four table
  // entries are two aligned pairs of its row, loaded as vectors.
  const int lane = lane_of(), w = wave_of();
  const int nw = (int)blockDim.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int ncg = (ncol + 15) / 16;
#pragma unroll
  for (int pass = 0; pass < G / S; pass++) {
    int memA[S], P0[S], np[S];
    bool any = false;
#pragma unroll
    for (int s = 0; s < S; s++) {
      memA[s] = te_mem[(int64_t)g * G + pass * S + s];
      any = any || memA[s] >= 0;
      P0[s] = memA[s] >= 0 ? plane_start[memA[s]] : 0;
      np[s] = memA[s] >= 0 ? plane_start[memA[s] + 1] - P0[s] : 0;
    }
    if (!any) continue;  // uniform over the workgroup
    if (pass > 0) __syncthreads();  // the previous pass has read its tiles
    if (active) {
#pragma unroll
      for (int s = 0; s < S; s++) {
        if (memA[s] < 0) continue;
        T* pt = ps + s * nr * LDW;
#pragma unroll
        for (int v = 0; v < 8; v++) {
          const int v1 = v & 1, v2 = (v >> 1) & 1, v3 = v >> 2;
          pt[(2 * m3 + v3) * LDW + v1 * 2 * tph + 2 * jj + v2] = acc[pass * S + s][v];
        }
      }
    }
    __syncthreads();
    int total = 0;
#pragma unroll
    for (int s = 0; s < S; s++) total += np[s] * ncg;
    const int it0 = (int)((int64_t)total * w / nw), it1 = (int)((int64_t)total * (w + 1) / nw);
    int lastP = -1;
    T aq[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) aq[i] = 0;
    for (int it = it0; it < it1; it++) {
      int slot = -1, r = it, P = 0;
#pragma unroll
      for (int s = 0; s < S; s++) {
        const int n = np[s] * ncg;
        if (slot < 0) {
          if (r < n) {
            slot = s;
            P = P0[s];
          } else {
            r -= n;
          }
        }
      }
      const int pq = r / ncg;
      const int cg = r - pq * ncg;
      P += pq;
      if (P != lastP) {
        lastP = P;
        const T* E3 = E + (int64_t)plane_tab[P * 3 + 2] * p * nr;
#pragma unroll
        for (int gk = 0; gk < NT; gk++)
#pragma unroll
          for (int h = 0; h < 2; h++) {
            const int k = 16 * gk + 4 * lk + 2 * h;  // even: the pair (k, k+1) is inside the row or past it
            const bool ok = lr < p && k < nr;
            const T2 v2 = *reinterpret_cast<const T2*>(E3 + (ok ? lr * nr + k : 0));
            aq[4 * gk + 2 * h] = ok ? v2.x : (T)0;
            aq[4 * gk + 2 * h + 1] = ok ? v2.y : (T)0;
          }
      }
      const T* pt = ps + slot * nr * LDW;
      const int col = 16 * cg + lr;
      const bool colok = col < ncol;
      acc_t d;
      zero4(d);
#pragma unroll
      for (int gk = 0; gk < NT; gk++) {
        T aqg[4], bq[4];
#pragma unroll
        for (int kk = 0; kk < 4; kk++) {
          const int k = 16 * gk + 4 * lk + kk;
          const T v = pt[(k < nr && colok ? k * LDW + col : 0)];  // LDS: select, no branch
          bq[kk] = k < nr && colok ? v : (T)0;
          aqg[kk] = aq[4 * gk + kk];
        }
        d = M_::template steps<4>(aqg, bq, d);
      }
      const int v1 = col >= 2 * tph ? 1 : 0;
      const int rem = col - v1 * 2 * tph;
      const int jc = j0 + (rem >> 1);
      const int mc1 = jc / M, mc2 = jc - mc1 * M;
      const int64_t cglob = (int64_t)(2 * mc1 + v1) * nr + 2 * mc2 + (rem & 1);
      T* Zp = Z + (int64_t)P * p * nr2;
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const int i3 = M_::row(lk, t);
        if (i3 < p && colok) Zp[(int64_t)i3 * nr2 + cglob] = d[t];
      }
    }
  }
}

inline int64_t transeval3_blocks(const DeviceArgs& a) { return a.nTW; }

// ---------------------------------------------------------------------------
// first evaluation contraction: Z rows of every leaf of one box for one tile of
// 64 columns.  The box's psi columns stay in registers while the workgroup
// walks the stacked leaf rows (s*p + i) two 16-row tiles at a time.  Boxes are
// visited in the order box_order (most leaves first).

template <typename C, int D, int NT>
__device__ __forceinline__ void eval_box_body(const elem_t<C>* __restrict__ psi,
                                                const int32_t* __restrict__ box_order,
                                                const int32_t* __restrict__ pw_start,
                                                const int32_t* __restrict__ leaf_tab,
                                                const elem_t<C>* __restrict__ E, int p, int nr,
                                                int ncoltiles, uint32_t pmagic,
                                                elem_t<C>* __restrict__ Z, int bid) {
  typedef elem_t<C> T;
  typedef Mfma<C> M;
  typedef typename M::acc acc_t;
  constexpr int Q = 4 * NT;
  const int A = box_order[bid / ncoltiles];
  const int ct = bid % ncoltiles;
  const int lane = lane_of(), w = wave_of();
  const int lr = lane & 15, lk = lane >> 4;
  const int N2 = D == 3 ? nr * nr : nr;
  const int col = ct * 64 + w * 16 + lr;
  const bool colok = col < N2;
  const T* P = psi + (int64_t)A * nr * N2;
  T b[Q];
#pragma unroll
  for (int q = 0; q < Q; q++) {
    const int k = 16 * (q >> 2) + M::kidx(q & 3, lk);
    b[q] = ld0<T>(P, (int64_t)k * N2 + col, k < nr && colok);
  }
  const int s0 = pw_start[A];
  const int rows = (pw_start[A + 1] - s0) * p;
  T* Zb = Z + (int64_t)s0 * p * N2;
  auto tab_of = [&](int row) {
    const int ls = (int)__umulhi((uint32_t)row, pmagic);  // row / p
    return ld0<int32_t>(leaf_tab, (int64_t)(s0 + ls) * D + (D - 1), row < rows);
  };
  int tnext[2] = {tab_of(lr), tab_of(16 + lr)};
  for (int rt = 0; rt < rows; rt += 32) {
    acc_t acc[2];
    int eoff[2];
    bool ok[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
      zero4(acc[h]);
      const int row = rt + 16 * h + lr;
      const int ls = (int)__umulhi((uint32_t)row, pmagic);
      ok[h] = row < rows;
      eoff[h] = ok[h] ? (tnext[h] * p + (row - ls * p)) * nr : 0;
    }
    tnext[0] = tab_of(rt + 32 + lr);
    tnext[1] = tab_of(rt + 48 + lr);
#pragma unroll
    for (int g = 0; g < NT; g++) {
      T bq[4];
#pragma unroll
      for (int kk = 0; kk < 4; kk++) bq[kk] = b[4 * g + kk];
#pragma unroll
      for (int h = 0; h < 2; h++) {
        T aq[4];
#pragma unroll
        for (int kk = 0; kk < 4; kk++) {
          const int k = 16 * g + M::kidx(kk, lk);
          aq[kk] = ld0<T>(E, eoff[h] + k, ok[h] && k < nr);
        }
        acc[h] = M::template steps<4>(aq, bq, acc[h]);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; h++)
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const int r = rt + 16 * h + M::row(lk, t);
        if (r < rows && colok) Zb[(int64_t)r * N2 + col] = acc[h][t];
      }
  }
}

// ---------------------------------------------------------------------------
// d = 3 evaluation, axes 1 and 2, one i3 slice of one plane per wave (a plane
// spans ceil(p/4) workgroups).  Z_P is stored [i3][r1][r2] (r2 fastest).  Per
// slice and row:
//   W^T[r2][i1] = sum_r1 Z_P[r1][r2] E1_row[i1][r1]       (lanes along r2: coalesced)
// and per leaf s of the row:
//   u_s[i2][i1] = sum_r2 E2_s[i2][r2] W^T[r2][i1]         (B operand chained from W^T)

template <typename C, int NT>
__device__ __forceinline__ void eval3_plane_body(const elem_t<C>* __restrict__ Z,
                                                 const int32_t* __restrict__ leaf_id,
                                                 const int32_t* __restrict__ leaf_tab,
                                                 const int32_t* __restrict__ plane_order,
                                                 const int32_t* __restrict__ plane_row,
                                                 const int32_t* __restrict__ row_start,
                                                 const int32_t* __restrict__ row_tab,
                                                 const elem_t<C>* __restrict__ E, int p, int nr,
                                                 double* __restrict__ u, int bid) {
  typedef elem_t<C> T;
  typedef Mfma<C> M;
  typedef typename M::acc acc_t;
  constexpr int Q = 4 * NT;
  const int nsplit = (p + 3) / 4;
  const int P = plane_order[bid / nsplit];  // planes with most work first
  const int lane = lane_of(), w = wave_of();
  const int i3 = (bid - (bid / nsplit) * nsplit) * 4 + w;
  if (i3 >= p) return;
  const int lr = lane & 15, lk = lane >> 4;
  const int rw0 = plane_row[P], rw1 = plane_row[P + 1];
  const int64_t ppp = (int64_t)p * p * p;
  const T* Zs = Z + ((int64_t)P * p + i3) * nr * nr;
  for (int rw = rw0; rw < rw1; rw++) {
    const T* E1 = E + (int64_t)row_tab[rw] * p * nr;
    T b1[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) {
      const int k = 16 * (q >> 2) + M::kidx(q & 3, lk);
      b1[q] = ld0<T>(E1, lr * nr + k, lr < p && k < nr);  // B[r1][i1] = E1[i1][r1]
    }
    const int s0 = row_start[rw], s1 = row_start[rw + 1];
    {
      acc_t wt[NT];  // W^T, rows r2 (tile ti), columns i1
#pragma unroll
      for (int ti = 0; ti < NT; ti++) {
        zero4(wt[ti]);
        const int r2 = 16 * ti + lr;
#pragma unroll
        for (int g = 0; g < NT; g++) {
          T aq[4], bq[4];
#pragma unroll
          for (int kk = 0; kk < 4; kk++) {
            const int k = 16 * g + M::kidx(kk, lk);  // r1
            aq[kk] = ld0<T>(Zs, k * nr + r2, r2 < nr && k < nr);
            bq[kk] = b1[4 * g + kk];
          }
          wt[ti] = M::template steps<4>(aq, bq, wt[ti]);
        }
      }
      for (int s = s0; s < s1; s++) {
        const T* E2 = E + (int64_t)leaf_tab[s * 3 + 1] * p * nr;
        T a2[Q];
#pragma unroll
        for (int q = 0; q < Q; q++) {
          const int k = 16 * (q >> 2) + M::kidx(q & 3, lk);
          a2[q] = ld0<T>(E2, lr * nr + k, lr < p && k < nr);  // A[i2][r2]
        }
        acc_t u0, u1;  // two accumulation chains, summed at the end
        zero4(u0);
        zero4(u1);
#pragma unroll
        for (int ti = 0; ti < NT; ti++) {
          T aq[4], bq[4];
#pragma unroll
          for (int kk = 0; kk < 4; kk++) {
            aq[kk] = a2[4 * ti + kk];
            bq[kk] = wt[ti][kk];
          }
          if (ti & 1) u1 = M::template steps<4>(aq, bq, u1);
          else u0 = M::template steps<4>(aq, bq, u0);
        }
        const acc_t uu = u0 + u1;
        double* ul = u + (int64_t)leaf_id[s] * ppp;
#pragma unroll
        for (int t = 0; t < 4; t++) {
          const int i2 = M::row(lk, t);
          if (i2 < p && lr < p) ul[((int64_t)i3 * p + i2) * p + lr] = (double)uu[t];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// d = 3 near field, one target leaf per workgroup.  A target's sources are
// sorted by (V3, V1, V2): axis 2 is contracted per source, axis 1 once per
// (V3, V1) run and axis 3 once per V3 run (separability, Remark dircost).
//   level A  T^T[j3][j1][i2] += sum_j2 sigma[j3][j2][j1] V2[i2][j2]  (lanes along j1)
//   level B  U[j3][i1][i2]   += sum_j1 V1[i1][j1] T^T[j3][j1][i2]    (chained)
//   level C  u[i3][i2][i1]   += sum_j3 V3[i3][j3] U[j3][i1][i2]      (j3 spans waves: LDS)

template <typename C, int KS>
__device__ __forceinline__ void near3_body(const double* __restrict__ sigma,
                                             const int32_t* __restrict__ near_tgt,
                                             const int32_t* __restrict__ near_haspw,
                                             const int32_t* __restrict__ near_start,
                                             const int32_t* __restrict__ near_src,
                                             const int32_t* __restrict__ near_tab,
                                             const elem_t<C>* __restrict__ V, int p,
                                             double* __restrict__ u, int bid) {
  typedef elem_t<C> T;
  typedef Mfma<C> M;
  typedef typename M::acc acc_t;
  constexpr int S = Steps<C, KS>::value;      // level B: the chained T^T as B operand
  constexpr int SM = MemSteps<C, KS>::value;  // levels A and C: operands from memory / LDS
  constexpr int RS = 17;            // padded i2 stride of the LDS tile
  constexpr int US = 16 * RS + 4;   // padded j3 stride
  __shared__ T Us[16 * US];         // U[j3][i2][i1]
  const int t = bid;
  const int Tleaf = near_tgt[t];
  const bool add = near_haspw[t] != 0;
  const int q0 = near_start[t], q1 = near_start[t + 1];
  const int lane = lane_of(), w = wave_of();
  const int lr = lane & 15, lk = lane >> 4;
  const int pp = p * p;
  acc_t tacc[KS], uacc[KS], oacc[KS];  // tile c <-> j3 (or i2) = w + 4c
#pragma unroll
  for (int c = 0; c < KS; c++) {
    zero4(tacc[c]);
    zero4(uacc[c]);
    zero4(oacc[c]);
  }
  for (int q = q0; q < q1; q++) {
    const int t1 = near_tab[q * 3 + 0], t2 = near_tab[q * 3 + 1], t3 = near_tab[q * 3 + 2];
    const double* sg = sigma + (int64_t)near_src[q] * pp * p;
    const T* V2 = V + (int64_t)t2 * pp;
    T b2[SM];
#pragma unroll
    for (int kk = 0; kk < SM; kk++) {
      const int k = M::kmem(kk, lk);
      b2[kk] = ld0<T>(V2, lr * p + k, lr < p && k < p);  // B[j2][i2] = V2[i2][j2]
    }
    T av[KS][SM];
#pragma unroll
    for (int c = 0; c < KS; c++) {
      const int j3 = w + 4 * c;
#pragma unroll
      for (int kk = 0; kk < SM; kk++) {
        const int k = M::kmem(kk, lk);
        av[c][kk] = ld0<T>(sg, (j3 * p + k) * p + lr, j3 < p && lr < p && k < p);  // A[j1][j2]
      }
    }
#pragma unroll
    for (int c = 0; c < KS; c++)
      tacc[c] = M::template steps<SM>(av[c], b2, tacc[c]);
    const bool last = q + 1 == q1;
    const bool end1 = last || near_tab[q * 3 + 5] != t3 || near_tab[q * 3 + 3] != t1;
    const bool end3 = last || near_tab[q * 3 + 5] != t3;
    if (end1) {
      const T* V1 = V + (int64_t)t1 * pp;
      T a1[S];
#pragma unroll
      for (int kk = 0; kk < S; kk++) {
        const int k = M::kidx(kk, lk);
        a1[kk] = ld0<T>(V1, lr * p + k, lr < p && k < p);  // A[i1][j1]
      }
#pragma unroll
      for (int c = 0; c < KS; c++) {
        {
          T tb[S];
#pragma unroll
          for (int kk = 0; kk < S; kk++) tb[kk] = tacc[c][kk];
          uacc[c] = M::template steps<S>(a1, tb, uacc[c]);
        }
        zero4(tacc[c]);
      }
    }
    if (end3) {
      __syncthreads();  // previous readers of Us are done
#pragma unroll
      for (int c = 0; c < KS; c++) {
        const int j3 = w + 4 * c;
        if (j3 < p) {
#pragma unroll
          for (int tt = 0; tt < 4; tt++) Us[j3 * US + lr * RS + M::row(lk, tt)] = uacc[c][tt];
        }
        zero4(uacc[c]);
      }
      __syncthreads();
      const T* V3 = V + (int64_t)t3 * pp;
      T a3[SM];
#pragma unroll
      for (int kk = 0; kk < SM; kk++) {
        const int k = M::kmem(kk, lk);
        a3[kk] = ld0<T>(V3, lr * p + k, lr < p && k < p);  // A[i3][j3]
      }
#pragma unroll
      for (int c = 0; c < KS; c++) {
        const int i2 = w + 4 * c;  // column tile (i2, i1 = lr); rows i2 >= p are never stored
        T bq[SM];
#pragma unroll
        for (int kk = 0; kk < SM; kk++) {
          const int j3 = M::kmem(kk, lk);
          const T uv = Us[j3 < p && i2 < p ? j3 * US + i2 * RS + lr : 0];  // LDS: select, no branch
          bq[kk] = j3 < p ? uv : (T)0;
        }
        oacc[c] = M::template steps<SM>(a3, bq, oacc[c]);
      }
    }
  }
  double* ut = u + (int64_t)Tleaf * pp * p;
  double prev[KS][4];
#pragma unroll
  for (int c = 0; c < KS; c++)
#pragma unroll
    for (int tt = 0; tt < 4; tt++) {
      const int i2 = w + 4 * c, i3 = M::row(lk, tt);
      const bool ok = add && i2 < p && lr < p && i3 < p;
      prev[c][tt] = ld0<double>(ut, ((int64_t)i3 * p + i2) * p + lr, ok);
    }
#pragma unroll
  for (int c = 0; c < KS; c++) {
    const int i2 = w + 4 * c;
    if (i2 < p && lr < p) {
#pragma unroll
      for (int tt = 0; tt < 4; tt++) {
        const int i3 = M::row(lk, tt);
        if (i3 < p) ut[((int64_t)i3 * p + i2) * p + lr] = prev[c][tt] + (double)oacc[c][tt];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// d = 2: formation of a whole cutoff box, both axes, leaves in sequence.
// Waves split the r1 tiles; every wave keeps all r2 tiles of its columns.

template <typename C, int NT, int KS>
__device__ __forceinline__ void form2_box_body(const double* __restrict__ sigma,
                                                 const int32_t* __restrict__ fitem,
                                                 const int32_t* __restrict__ leaf_id,
                                                 const int32_t* __restrict__ leaf_tab,
                                                 const elem_t<C>* __restrict__ F, int p, int nr,
                                                 elem_t<C>* __restrict__ phi, elem_t<C>* __restrict__ partial, int bid) {
  typedef elem_t<C> T;
  typedef Mfma<C> M;
  typedef typename M::acc acc_t;
  constexpr int S = Steps<C, KS>::value;      // F2 x X (X chained as the B operand)
  constexpr int SM = MemSteps<C, KS>::value;  // sigma x F1, both from memory
  constexpr int TW = (NT + 3) / 4;  // r1 tiles per wave
  const int item = bid;
  const int A = fitem[4 * item], slot = fitem[4 * item + 3];
  const int lane = lane_of(), w = wave_of();
  const int lr = lane & 15, lk = lane >> 4;
  acc_t acc[NT][TW];
#pragma unroll
  for (int ti = 0; ti < NT; ti++)
#pragma unroll
    for (int c = 0; c < TW; c++) zero4(acc[ti][c]);
  const int s0 = fitem[4 * item + 1], s1 = fitem[4 * item + 2];
  for (int s = s0; s < s1; s++) {
    const T* F1 = F + (int64_t)leaf_tab[s * 2 + 0] * nr * p;
    const T* F2 = F + (int64_t)leaf_tab[s * 2 + 1] * nr * p;
    const double* sg = sigma + (int64_t)leaf_id[s] * p * p;
    T av[SM], a2[NT][S];
#pragma unroll
    for (int kk = 0; kk < SM; kk++) {
      const int k = M::kmem(kk, lk);
      av[kk] = ld0<T>(sg, lr * p + k, lr < p && k < p);
    }
#pragma unroll
    for (int kk = 0; kk < S; kk++) {
      const int k = M::kidx(kk, lk);
#pragma unroll
      for (int ti = 0; ti < NT; ti++) {
        const int r = 16 * ti + lr;
        a2[ti][kk] = ld0<T>(F2, r * p + k, r < nr && k < p);
      }
    }
#pragma unroll
    for (int c = 0; c < TW; c++) {
      const int tj = w + 4 * c;
      if (tj < NT) {
        // X[j2][r1] = sum_j1 sigma[j2][j1] F1[r1][j1]
        acc_t x;
        zero4(x);
        T bq[SM];
#pragma unroll
        for (int kk = 0; kk < SM; kk++) {
          const int k = M::kmem(kk, lk), r = 16 * tj + lr;
          bq[kk] = ld0<T>(F1, r * p + k, r < nr && k < p);
        }
        x = M::template steps<SM>(av, bq, x);
        // phi[r2][r1] += sum_j2 F2[r2][j2] X[j2][r1]
        T xb[S];
#pragma unroll
        for (int kk = 0; kk < S; kk++) xb[kk] = x[kk];
#pragma unroll
        for (int ti = 0; ti < NT; ti++) acc[ti][c] = M::template steps<S>(a2[ti], xb, acc[ti][c]);
      }
    }
  }
  T* out = slot < 0 ? phi + (int64_t)A * nr * nr : partial + (int64_t)slot * nr * nr;
#pragma unroll
  for (int c = 0; c < TW; c++) {
    const int tj = w + 4 * c;
    const int r1 = 16 * tj + lr;
    if (tj < NT && r1 < nr) {
#pragma unroll
      for (int ti = 0; ti < NT; ti++)
#pragma unroll
        for (int t = 0; t < 4; t++) {
          const int r2 = 16 * ti + M::row(lk, t);
          if (r2 < nr) out[r2 * nr + r1] = acc[ti][c][t];
        }
    }
  }
}

// d = 2: evaluation of one leaf per wave from its box's incoming expansion.
template <typename C, int NT>
__device__ __forceinline__ void eval2_leaf_body(const elem_t<C>* __restrict__ psi,
                                                  const int32_t* __restrict__ leaf_box,
                                                  const int32_t* __restrict__ leaf_id,
                                                  const int32_t* __restrict__ leaf_tab,
                                                  const elem_t<C>* __restrict__ E, int p, int nr,
                                                  int nleaf, double* __restrict__ u, int bid) {
  typedef elem_t<C> T;
  typedef Mfma<C> M;
  typedef typename M::acc acc_t;
  constexpr int Q = 4 * NT;
  const int lane = lane_of(), w = wave_of();
  const int s = bid * 4 + w;
  if (s >= nleaf) return;
  const int lr = lane & 15, lk = lane >> 4;
  const T* E1 = E + (int64_t)leaf_tab[s * 2 + 0] * p * nr;
  const T* E2 = E + (int64_t)leaf_tab[s * 2 + 1] * p * nr;
  const T* P = psi + (int64_t)leaf_box[s] * nr * nr;
  // W[r2][i1] = sum_r1 psi[r2][r1] E1[i1][r1]
  acc_t wt[NT];
#pragma unroll
  for (int ti = 0; ti < NT; ti++) zero4(wt[ti]);
#pragma unroll
  for (int g = 0; g < NT; g++) {
    T bq[4];
#pragma unroll
    for (int kk = 0; kk < 4; kk++) {
      const int k = 16 * g + M::kidx(kk, lk);
      bq[kk] = ld0<T>(E1, lr * nr + k, lr < p && k < nr);
    }
#pragma unroll
    for (int ti = 0; ti < NT; ti++) {
      const int r2 = 16 * ti + lr;
      T aq[4];
#pragma unroll
      for (int kk = 0; kk < 4; kk++) {
        const int k = 16 * g + M::kidx(kk, lk);
        aq[kk] = ld0<T>(P, r2 * nr + k, r2 < nr && k < nr);
      }
      wt[ti] = M::template steps<4>(aq, bq, wt[ti]);
    }
  }
  // u[i2][i1] = sum_r2 E2[i2][r2] W[r2][i1]
  acc_t uu;
  zero4(uu);
#pragma unroll
  for (int ti = 0; ti < NT; ti++) {
    T aq[4], bq[4];
#pragma unroll
    for (int kk = 0; kk < 4; kk++) {
      const int k = 16 * ti + M::kidx(kk, lk);
      aq[kk] = ld0<T>(E2, lr * nr + k, lr < p && k < nr);
      bq[kk] = wt[ti][kk];
    }
    uu = M::template steps<4>(aq, bq, uu);
  }
  double* ul = u + (int64_t)leaf_id[s] * p * p;
#pragma unroll
  for (int t = 0; t < 4; t++) {
    const int i2 = M::row(lk, t);
    if (i2 < p && lr < p) ul[i2 * p + lr] = (double)uu[t];
  }
}

// d = 2 near field: one target per wave; sources sorted by (V2, V1): axis 1
// per source, axis 2 once per V2 group.
template <typename C, int KS>
__device__ __forceinline__ void near2_body(const double* __restrict__ sigma,
                                             const int32_t* __restrict__ near_tgt,
                                             const int32_t* __restrict__ near_haspw,
                                             const int32_t* __restrict__ near_start,
                                             const int32_t* __restrict__ near_src,
                                             const int32_t* __restrict__ near_tab,
                                             const elem_t<C>* __restrict__ V, int p, int ntgt,
                                             double* __restrict__ u, int bid) {
  typedef elem_t<C> T;
  typedef Mfma<C> M;
  typedef typename M::acc acc_t;
  constexpr int S = Steps<C, KS>::value;      // V2 x T (T chained as the B operand)
  constexpr int SM = MemSteps<C, KS>::value;  // sigma x V1, both from memory
  const int lane = lane_of(), w = wave_of();
  const int t = bid * 4 + w;
  if (t >= ntgt) return;
  const int lr = lane & 15, lk = lane >> 4;
  const int pp = p * p;
  const int q0 = near_start[t], q1 = near_start[t + 1];
  acc_t tacc, oacc;
  zero4(tacc);
  zero4(oacc);
  for (int q = q0; q < q1; q++) {
    const int t1 = near_tab[q * 2 + 0], t2 = near_tab[q * 2 + 1];
    const double* sg = sigma + (int64_t)near_src[q] * pp;
    const T* V1 = V + (int64_t)t1 * pp;
    {
      T aq[SM], bq[SM];
#pragma unroll
      for (int kk = 0; kk < SM; kk++) {
        const int k = M::kmem(kk, lk);
        aq[kk] = ld0<T>(sg, lr * p + k, lr < p && k < p);
        bq[kk] = ld0<T>(V1, lr * p + k, lr < p && k < p);
      }
      tacc = M::template steps<SM>(aq, bq, tacc);  // T[j2][i1]
    }
    if (q + 1 == q1 || near_tab[q * 2 + 3] != t2) {
      const T* V2 = V + (int64_t)t2 * pp;
      T aq[S], bq[S];
#pragma unroll
      for (int kk = 0; kk < S; kk++) {
        const int k = M::kidx(kk, lk);
        aq[kk] = ld0<T>(V2, lr * p + k, lr < p && k < p);
        bq[kk] = tacc[kk];
      }
      oacc = M::template steps<S>(aq, bq, oacc);  // u[i2][i1] += V2[i2][j2] T[j2][i1]
      zero4(tacc);
    }
  }
  double* ut = u + (int64_t)near_tgt[t] * pp;
  const bool add = near_haspw[t] != 0;
#pragma unroll
  for (int tt = 0; tt < 4; tt++) {
    const int i2 = M::row(lk, tt);
    if (i2 < p && lr < p) ut[i2 * p + lr] = add ? ut[i2 * p + lr] + (double)oacc[tt] : (double)oacc[tt];
  }
}

// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ const T* cptr(const void* p) { return static_cast<const T*>(p); }
template <typename T> __device__ __forceinline__ T* mptr(void* p) { return static_cast<T*>(p); }
__device__ __forceinline__ int n2_of(int d, int nr) { return d == 3 ? nr * nr : nr; }
__device__ __forceinline__ uint32_t pmagic_of(int p) { return (uint32_t)((0x100000000ull + p - 1) / p); }

}  // namespace fgt
