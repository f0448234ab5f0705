// The point Gauss transform with proxy grids (declared in fgt_point.h): the
// device side.  Per execution:
//   1. k_anterp   charges -> proxy charges on the grids of the dense boxes
//   2. the box transform's plane-wave stages over the proxy grids (formation
//      with point-evaluation tables, translation, evaluation on the grids)
//   3. k_interp   grid potentials -> the targets of every plane-wave box
//   4. k_direct   the D-lists summed directly, plus the plane-wave part, into u
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fgt.h"
#include "../../include/fgt_point.h"
#include "mfma.h"
#include "plan_internal.h"
#include "point_host.h"

namespace fgt {
namespace {

constexpr int kPT = 256;  // threads per workgroup
constexpr int kPMax = 16;

// Lagrange weights of the p Gauss-Legendre nodes at t in [-1, 1], by the
// barycentric formula; a node hit exactly gets the unit weight.
__device__ __forceinline__ void lagrange(int p, double t, const double* __restrict__ eta,
                                         const double* __restrict__ lam, double (&w)[kPMax]) {
  double den = 0.0;
  int hit = -1;
#pragma unroll
  for (int k = 0; k < kPMax; k++) {
    const double dt = k < p ? t - eta[k] : 1.0;
    if (k < p && dt == 0.0) hit = k;
    // 1/dt: the hardware estimate refined by two Newton steps (each doubles the
    // correct bits), instead of a full division per node
    double r = __builtin_amdgcn_rcp(dt);
    r = fma(r, fma(-dt, r, 1.0), r);
    r = fma(r, fma(-dt, r, 1.0), r);
    w[k] = (k < p && dt != 0.0) ? lam[k] * r : 0.0;
    den += w[k];
  }
  const double inv = hit >= 0 ? 0.0 : 1.0 / den;
#pragma unroll
  for (int k = 0; k < kPMax; k++) w[k] = hit >= 0 ? (k == hit ? 1.0 : 0.0) : w[k] * inv;
}

// Local coordinate in [-1, 1] of x on axis a of the box (level l, coord c).
__device__ __forceinline__ double local_coord(double x, int l, int32_t c) {
  const double L = ldexp(1.0, -l);
  const double lo = -0.5 + (double)c * L;
  double t = 2.0 * (x - lo) / L - 1.0;
  return t < -1.0 ? -1.0 : (t > 1.0 ? 1.0 : t);
}

// 1. Proxy charges of one grid: Q[k] = sum over its sources of
// prod_a l_{k_a}(t_a) q, node k = k_1 + p k_2 (+ p^2 k_3).  Thread (k_1, k_2) =
// (tid % 16, tid / 16) owns the nodes k_3 = 0..15 of its column; sources come
// in chunks whose per-axis weights are computed once into LDS, and per source
// a thread forms l_{k_1} l_{k_2} q once and scales the broadcast axis-3
// weights by it.
// Work item (grid, first source, end source, partial slot): a grid's sources
// are split into parts of at most kAnterpPart, each summed by one workgroup
// into its slot of `partial` (or straight into Q when the grid has one part);
// k_anterp_reduce then adds a grid's parts in order.
template <int D>
__global__ __launch_bounds__(kPT) void k_anterp(const double* __restrict__ q, const int32_t* __restrict__ src_perm,
                                                const double* __restrict__ src_xyz,
                                                const int32_t* __restrict__ items,
                                                const int32_t* __restrict__ px_coord, int lp, int p,
                                                const double* __restrict__ eta, const double* __restrict__ lam,
                                                double* __restrict__ Q, double* __restrict__ partial) {
  constexpr int CH = 64;
  constexpr int NE = D == 3 ? kPMax : 1;
  __shared__ __align__(16) double W[CH][D][kPMax];
  __shared__ double qs[CH];
  const int b = items[4 * blockIdx.x], slot = items[4 * blockIdx.x + 3], tid = threadIdx.x;
  const int k1 = tid & 15, k2 = tid >> 4;
  const int s0 = items[4 * blockIdx.x + 1], s1 = items[4 * blockIdx.x + 2];
  double acc[NE];
#pragma unroll
  for (int j = 0; j < NE; j++) acc[j] = 0.0;
  for (int c0 = s0; c0 < s1; c0 += CH) {
    const int nc = min(CH, s1 - c0);
    if (tid < nc * D) {
      const int s = tid / D, a = tid - (tid / D) * D;
      const double t = local_coord(src_xyz[(int64_t)(c0 + s) * D + a], lp, px_coord[(int64_t)b * D + a]);
      double w[kPMax];
      lagrange(p, t, eta, lam, w);
#pragma unroll
      for (int k = 0; k < kPMax; k++) W[s][a][k] = w[k];
    }
    if (tid < nc) qs[tid] = q[src_perm[c0 + tid]];
    __syncthreads();
    for (int s = 0; s < nc; s++) {
      const double w12 = W[s][0][k1] * W[s][1][k2] * qs[s];
      if (D == 3) {
        const double2* w3 = reinterpret_cast<const double2*>(&W[s][D - 1][0]);
#pragma unroll
        for (int j = 0; j < kPMax / 2; j++) {
          const double2 v = w3[j];  // the same words in every lane: a broadcast
          acc[2 * j] += w12 * v.x;
          acc[2 * j + 1] += w12 * v.y;
        }
      } else {
        acc[0] += w12;
      }
    }
    __syncthreads();
  }
  if (k1 < p && k2 < p) {
    int64_t pd = (int64_t)p * p;
    if (D == 3) pd *= p;
    double* out = slot >= 0 ? partial + (int64_t)slot * pd : Q + (int64_t)b * pd;
#pragma unroll
    for (int j = 0; j < NE; j++)
      if (j < (D == 3 ? p : 1)) out[k1 + p * k2 + (int64_t)p * p * j] = acc[j];
  }
}

// 1 (d = 3). The same proxy charges on the matrix cores: per item,
//   Q[k1][(k2, k3)] = sum_s l_{k1}(s) G[s][(k2, k3)],  G[s][(k2, k3)] = q_s l_{k2}(s) l_{k3}(s),
// a 16 x K x 256 product over the item's sources (K = its source count).  Wave
// w owns the columns k3 = 4w..4w+3 (four 16 x 16 result tiles, k2 along the
// lanes); a k-step takes four sources of the chunk, whose weights sit in LDS.
// Rows, columns and sources past p or past the item read zero weights.
__global__ __launch_bounds__(kPT) void k_anterp3(const double* __restrict__ q, const int32_t* __restrict__ src_perm,
                                                 const double* __restrict__ src_xyz,
                                                 const int32_t* __restrict__ items,
                                                 const int32_t* __restrict__ px_coord, int lp, int p,
                                                 const double* __restrict__ eta, const double* __restrict__ lam,
                                                 double* __restrict__ Q, double* __restrict__ partial) {
  typedef Mfma<double> MF;
  constexpr int CH = 64;
  __shared__ __align__(16) double W[CH][3][kPMax];
  __shared__ double qs[CH];
  const int b = items[4 * blockIdx.x], slot = items[4 * blockIdx.x + 3], tid = threadIdx.x;
  const int s0 = items[4 * blockIdx.x + 1], s1 = items[4 * blockIdx.x + 2];
  const int lane = tid & 63, w = tid >> 6, lr = lane & 15, lk = lane >> 4;
  MF::acc acc[4];
#pragma unroll
  for (int j = 0; j < 4; j++) acc[j] = MF::acc{0.0, 0.0, 0.0, 0.0};
  for (int c0 = s0; c0 < s1; c0 += CH) {
    const int nc = min(CH, s1 - c0);
    if (tid < CH * 3) {
      const int s = tid / 3, a = tid - (tid / 3) * 3;
      double wv[kPMax];
      if (s < nc) {
        lagrange(p, local_coord(src_xyz[(int64_t)(c0 + s) * 3 + a], lp, px_coord[(int64_t)b * 3 + a]), eta, lam, wv);
      } else {
#pragma unroll
        for (int k = 0; k < kPMax; k++) wv[k] = 0.0;
      }
#pragma unroll
      for (int k = 0; k < kPMax; k++) W[s][a][k] = wv[k];
    }
    if (tid < CH) qs[tid] = tid < nc ? q[src_perm[c0 + tid]] : 0.0;
    __syncthreads();
    const int nk = (nc + 3) / 4;
#pragma unroll 4
    for (int kk = 0; kk < nk; kk++) {
      const int s = 4 * kk + lk;
      const double a1 = W[s][0][lr];
      const double wq = qs[s] * W[s][1][lr];
#pragma unroll
      for (int j = 0; j < 4; j++) acc[j] = MF::step(a1, wq * W[s][2][4 * w + j], acc[j]);
    }
    __syncthreads();
  }
  // lane (lk, lr) holds rows k1 = 4t + lk of column k2 = lr in tile k3 = 4w + j
  const int64_t pd = (int64_t)p * p * p;
  double* out = slot >= 0 ? partial + (int64_t)slot * pd : Q + (int64_t)b * pd;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const int k3 = 4 * w + j;
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int k1 = MF::row(lk, t);
      if (k1 < p && lr < p && k3 < p) out[k1 + (int64_t)p * lr + (int64_t)p * p * k3] = acc[j][t];
    }
  }
}

// Q of a grid split into parts: the parts' sums added in part order.  Item =
// (grid, first slot, parts); a workgroup takes kPT nodes of one item.
__global__ __launch_bounds__(kPT) void k_anterp_reduce(const int32_t* __restrict__ items,
                                                       const double* __restrict__ partial, int pd,
                                                       double* __restrict__ Q) {
  const int nchunk = (pd + kPT - 1) / kPT;
  const int r = blockIdx.x / nchunk;
  const int e = (blockIdx.x - r * nchunk) * kPT + threadIdx.x;
  if (e >= pd) return;
  const int b = items[3 * r], slot0 = items[3 * r + 1], n = items[3 * r + 2];
  double sum = 0.0;
  for (int i = 0; i < n; i++) sum += partial[(int64_t)(slot0 + i) * pd + e];
  Q[(int64_t)b * pd + e] = sum;
}

// 3. The grid potential of one plane-wave box's grid at one chunk of its
// targets (written at their sorted positions): work item = (grid, chunk of
// kPT targets).  The grid sits in LDS; every lane reads the same node at the
// same time.
template <int D>
__global__ __launch_bounds__(kPT) void k_interp(const double* __restrict__ U, const int32_t* __restrict__ items,
                                                const int32_t* __restrict__ px_tgt,
                                                const int32_t* __restrict__ px_coord, int lp, int p,
                                                const double* __restrict__ eta, const double* __restrict__ lam,
                                                const double* __restrict__ tgt_xyz, double* __restrict__ uw) {
  __shared__ __align__(16) double Us[kPMax * kPMax * (D == 3 ? kPMax : 1)];
  const int b = items[2 * blockIdx.x], tb = items[2 * blockIdx.x + 1], tid = threadIdx.x;
  int pd = p * p;
  if (D == 3) pd *= p;
  // node (k1, k2, k3) at k1 + 16 k2 + 256 k3 in LDS (rows 16-aligned), zero
  // past p
  for (int e = tid; e < kPMax * kPMax * (D == 3 ? kPMax : 1); e += kPT) {
    const int k1 = e % kPMax, k2 = (e / kPMax) % kPMax, k3 = e / (kPMax * kPMax);
    const bool in = k1 < p && k2 < p && k3 < (D == 3 ? p : 1);
    Us[e] = in ? U[(int64_t)b * pd + k1 + p * k2 + p * p * k3] : 0.0;
  }
  __syncthreads();
  const int t1 = px_tgt[2 * b + 1];
  const int pos = tb + tid;
  if (pos >= t1) return;
  double w1[kPMax], w2[kPMax], w3[kPMax];
  lagrange(p, local_coord(tgt_xyz[(int64_t)pos * D + 0], lp, px_coord[(int64_t)b * D + 0]), eta, lam, w1);
  lagrange(p, local_coord(tgt_xyz[(int64_t)pos * D + 1], lp, px_coord[(int64_t)b * D + 1]), eta, lam, w2);
  if (D == 3)
    lagrange(p, local_coord(tgt_xyz[(int64_t)pos * D + 2], lp, px_coord[(int64_t)b * D + 2]), eta, lam, w3);
  double u = 0.0;
  for (int k3 = 0; k3 < (D == 3 ? p : 1); k3++) {
    double s3 = 0.0;
    for (int k2 = 0; k2 < p; k2++) {
      const double2* row = reinterpret_cast<const double2*>(Us + kPMax * k2 + kPMax * kPMax * k3);
      double s2 = 0.0;
#pragma unroll
      for (int h = 0; h < kPMax / 2; h++) {
        const double2 v = row[h];  // weights past p are zero
        s2 += w1[2 * h] * v.x + w1[2 * h + 1] * v.y;
      }
      double wk2 = 0.0;
#pragma unroll
      for (int k = 0; k < kPMax; k++) wk2 = k == k2 ? w2[k] : wk2;
      s3 += wk2 * s2;
    }
    double wk3 = 1.0;
    if (D == 3) {
#pragma unroll
      for (int k = 0; k < kPMax; k++) wk3 = k == k3 ? w3[k] : wk3;
    }
    u += wk3 * s3;
  }
  uw[pos] = u;
}

// 3 (d = 3). The same grid potentials on the matrix cores, per tile of 16
// targets t:
//   V[t][(k2, k3)] = sum_k1 l_{k1}(t) U[k1][k2][k3]      (16 x 16 x 256, k1 the K axis)
//   u_t = sum_{k2, k3} V[t][(k2, k3)] l_{k2}(t) l_{k3}(t)  (in the lanes, then across them)
// Work item = (grid, chunk of kPT targets): wave w takes the tiles of targets
// 64w + 16i, i = 0..3, all waves in step (the tile's weights are written to
// LDS between barriers).  The grid sits in LDS with the k2 stride padded to 17
// so that the 16 lanes reading one k1 row hit distinct banks.
__global__ __launch_bounds__(kPT) void k_interp3(const double* __restrict__ U, const int32_t* __restrict__ items,
                                                 const int32_t* __restrict__ px_tgt,
                                                 const int32_t* __restrict__ px_coord, int lp, int p,
                                                 const double* __restrict__ eta, const double* __restrict__ lam,
                                                 const double* __restrict__ tgt_xyz, double* __restrict__ uw) {
  typedef Mfma<double> MF;
  constexpr int S2 = kPMax + 1, S3 = kPMax * S2;  // LDS strides of k2 and k3
  __shared__ __align__(16) double Us[kPMax * S3];
  __shared__ double Wt[4][16][3][kPMax + 1];
  const int b = items[2 * blockIdx.x], tb = items[2 * blockIdx.x + 1], tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, lr = lane & 15, lk = lane >> 4;
  const int64_t pd = (int64_t)p * p * p;
  for (int e = tid; e < kPMax * kPMax * kPMax; e += kPT) {
    const int k1 = e % kPMax, k2 = (e / kPMax) % kPMax, k3 = e / (kPMax * kPMax);
    const bool in = k1 < p && k2 < p && k3 < p;
    Us[k1 + S2 * k2 + S3 * k3] = in ? U[(int64_t)b * pd + k1 + p * k2 + p * p * k3] : 0.0;
  }
  const int t1 = px_tgt[2 * b + 1];
  for (int i = 0; i < 4; i++) {
    const int base = tb + 64 * w + 16 * i;
    if (lane < 48) {
      const int tt = lane & 15, a = lane >> 4;
      const int pos = base + tt;
      double wv[kPMax];
      if (pos < t1) {
        lagrange(p, local_coord(tgt_xyz[(int64_t)pos * 3 + a], lp, px_coord[(int64_t)b * 3 + a]), eta, lam, wv);
      } else {
#pragma unroll
        for (int k = 0; k < kPMax; k++) wv[k] = 0.0;
      }
#pragma unroll
      for (int k = 0; k < kPMax; k++) Wt[w][tt][a][k] = wv[k];
    }
    __syncthreads();  // the grid (first pass) and this tile's weights are in LDS
    if (base < t1) {  // uniform over the wave
      double a1[4], w2[4], part[4];
#pragma unroll
      for (int kk = 0; kk < 4; kk++) a1[kk] = Wt[w][lr][0][4 * kk + lk];  // A[t = lr][k1 = 4kk + lk]
#pragma unroll
      for (int j = 0; j < 4; j++) {
        w2[j] = Wt[w][MF::row(lk, j)][1][lr];  // l_{k2 = lr} of target 4j + lk
        part[j] = 0.0;
      }
#pragma unroll 4
      for (int k3 = 0; k3 < p; k3++) {
        MF::acc v = MF::acc{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; kk++) v = MF::step(a1[kk], Us[(4 * kk + lk) + S2 * lr + S3 * k3], v);
#pragma unroll
        for (int j = 0; j < 4; j++) part[j] += v[j] * w2[j] * Wt[w][MF::row(lk, j)][2][k3];
      }
      // sum over k2: the 16 lanes lr of each row
#pragma unroll
      for (int off = 1; off < 16; off <<= 1)
#pragma unroll
        for (int j = 0; j < 4; j++) part[j] += __shfl_xor(part[j], off);
      if (lr == 0) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int pos = base + MF::row(lk, j);
          if (pos < t1) uw[pos] = part[j];
        }
      }
    }
    __syncthreads();  // the tile's weights have been read
  }
}

// 4. One chunk of kPT targets of a leaf (work item = (leaf, first target)):
// the sum over the sources of its D-list, in a fixed order, plus the
// plane-wave part when the leaf has one; u in the caller's order.
template <int D>
__global__ __launch_bounds__(kPT) void k_direct(const double* __restrict__ q, const int32_t* __restrict__ src_perm,
                                                const double* __restrict__ src_xyz,
                                                const double* __restrict__ tgt_xyz,
                                                const int32_t* __restrict__ tgt_perm,
                                                const int32_t* __restrict__ leaf_src_start,
                                                const int32_t* __restrict__ leaf_tgt_start,
                                                const int32_t* __restrict__ dl_tgt,
                                                const int32_t* __restrict__ dl_haspw,
                                                const int32_t* __restrict__ dl_start,
                                                const int32_t* __restrict__ dl_src,
                                                const int32_t* __restrict__ items, double inv_delta,
                                                const double* __restrict__ uw, double* __restrict__ u) {
  __shared__ double ys[kPT][D + 1];
  const int k = items[2 * blockIdx.x], tid = threadIdx.x;
  const int T = dl_tgt[k];
  const bool haspw = dl_haspw[k] != 0;
  const int t1 = leaf_tgt_start[T + 1];
  const int e0 = dl_start[k], e1 = dl_start[k + 1];
  {
    const int tb = items[2 * blockIdx.x + 1];
    const int pos = tb + tid;
    const bool mine = pos < t1;
    double x[3] = {0.0, 0.0, 0.0};
    if (mine && e0 < e1)  // coordinates only where there is a direct part
      for (int a = 0; a < D; a++) x[a] = tgt_xyz[(int64_t)pos * D + a];
    double acc = 0.0;
    for (int e = e0; e < e1; e++) {
      const int S = dl_src[e];
      const int s0 = leaf_src_start[S], s1 = leaf_src_start[S + 1];
      for (int sb = s0; sb < s1; sb += kPT) {
        const int n = min(kPT, s1 - sb);
        if (tid < n) {
          for (int a = 0; a < D; a++) ys[tid][a] = src_xyz[(int64_t)(sb + tid) * D + a];
          ys[tid][D] = q[src_perm[sb + tid]];
        }
        __syncthreads();
        if (mine) {
          for (int j = 0; j < n; j++) {
            double r2 = 0.0;
            for (int a = 0; a < D; a++) {
              const double dx = x[a] - ys[j][a];
              r2 += dx * dx;
            }
            acc += exp(-r2 * inv_delta) * ys[j][D];
          }
        }
        __syncthreads();
      }
    }
    if (mine) u[tgt_perm[pos]] = acc + (haspw ? uw[pos] : 0.0);
  }
}

}  // namespace
}  // namespace fgt

struct fgt_point_plan {
  fgt::PointHost ph;
  fgt_plan_t* pw = nullptr;  // the plane-wave stages over the proxy grids
  bool host_only = true;
  int device = -1;
  hipStream_t stream = nullptr;
  std::vector<void*> allocs;
  int64_t device_bytes = 0;
  // device arrays
  int32_t *src_perm = nullptr, *tgt_perm = nullptr, *leaf_src_start = nullptr, *leaf_tgt_start = nullptr;
  int32_t *dl_tgt = nullptr, *dl_haspw = nullptr, *dl_start = nullptr, *dl_src = nullptr;
  int32_t *px_src = nullptr, *px_tgt = nullptr, *px_coord = nullptr;
  int32_t *interp_items = nullptr, *direct_items = nullptr, *anterp_items = nullptr, *reduce_items = nullptr;
  double* partial = nullptr;
  double *src_xyz = nullptr, *tgt_xyz = nullptr, *eta = nullptr, *lam = nullptr;
  double *Q = nullptr, *U = nullptr, *uw = nullptr;
};

namespace {

int hip_fail(hipError_t e, const char* what) {
  return fgt::set_error(FGT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename X>
int upload(fgt_point_plan_t* pp, const std::vector<X>& v, X** out) {
  *out = nullptr;
  if (v.empty()) return FGT_OK;
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, v.size() * sizeof(X));
  if (e != hipSuccess) return fgt::set_error(FGT_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  pp->allocs.push_back(d);
  pp->device_bytes += (int64_t)(v.size() * sizeof(X));
  if ((e = hipMemcpy(d, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy");
  *out = static_cast<X*>(d);
  return FGT_OK;
}

int alloc_doubles(fgt_point_plan_t* pp, size_t n, double** out) {
  *out = nullptr;
  if (n == 0) return FGT_OK;
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, n * sizeof(double));
  if (e != hipSuccess) return fgt::set_error(FGT_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  pp->allocs.push_back(d);
  pp->device_bytes += (int64_t)(n * sizeof(double));
  *out = static_cast<double*>(d);
  return FGT_OK;
}

void release(fgt_point_plan_t* pp) {
  if (!pp) return;
  if (!pp->host_only) {
    (void)hipSetDevice(pp->device);
    (void)hipStreamSynchronize(pp->stream);
  }
  for (void* x : pp->allocs) (void)hipFree(x);
  if (pp->pw) fgt_destroy(pp->pw);
  delete pp;
}

int setup(fgt_point_plan_t* pp, hipStream_t stream) {
  fgt::PointHost& ph = pp->ph;
  hipError_t e = hipGetDevice(&pp->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  pp->stream = stream;
  int rc;
  std::vector<double> eta, lam;
  fgt::gl_barycentric(ph.p, eta, lam);
  if ((rc = upload(pp, ph.src_perm, &pp->src_perm)) || (rc = upload(pp, ph.tgt_perm, &pp->tgt_perm)) ||
      (rc = upload(pp, ph.leaf_src_start, &pp->leaf_src_start)) ||
      (rc = upload(pp, ph.leaf_tgt_start, &pp->leaf_tgt_start)) || (rc = upload(pp, ph.dl_tgt, &pp->dl_tgt)) ||
      (rc = upload(pp, ph.dl_haspw, &pp->dl_haspw)) || (rc = upload(pp, ph.dl_start, &pp->dl_start)) ||
      (rc = upload(pp, ph.dl_src, &pp->dl_src)) || (rc = upload(pp, ph.px_src_start, &pp->px_src)) ||
      (rc = upload(pp, ph.px_tgt_start, &pp->px_tgt)) || (rc = upload(pp, ph.px_coord, &pp->px_coord)) ||
      (rc = upload(pp, ph.interp_items, &pp->interp_items)) ||
      (rc = upload(pp, ph.anterp_items, &pp->anterp_items)) || (rc = upload(pp, ph.reduce_items, &pp->reduce_items)) ||
      (rc = upload(pp, ph.direct_items, &pp->direct_items)) || (rc = upload(pp, ph.src_xyz, &pp->src_xyz)) ||
      (rc = upload(pp, ph.tgt_xyz, &pp->tgt_xyz)) || (rc = upload(pp, eta, &pp->eta)) ||
      (rc = upload(pp, lam, &pp->lam)))
    return rc;
  const int64_t npx = (int64_t)ph.px_level.size();
  int64_t pd = (int64_t)ph.p * ph.p;
  if (ph.d == 3) pd *= ph.p;
  if ((rc = alloc_doubles(pp, (size_t)(npx * pd), &pp->Q)) || (rc = alloc_doubles(pp, (size_t)(npx * pd), &pp->U)) ||
      (rc = alloc_doubles(pp, (size_t)(ph.n_anterp_slots * pd), &pp->partial)) ||
      (rc = alloc_doubles(pp, (size_t)ph.ntgt, &pp->uw)))
    return rc;
  if (ph.n_pwbox > 0) {
    fgt_plan_t* pw = new (std::nothrow) fgt_plan_t();
    if (!pw) return fgt::set_error(FGT_ERR_OOM, "host allocation");
    pw->hp = ph.hp;
    pw->host_only = true;
    if ((rc = fgt::plan_upload(pw, stream)) != FGT_OK) {
      fgt_destroy(pw);
      return rc;
    }
    pp->pw = pw;
    pp->device_bytes += pw->device_bytes;
  }
  pp->host_only = false;
  return FGT_OK;
}

}  // namespace

extern "C" {

int fgt_point_plan(int dim, int64_t nsrc, const double* src, int64_t ntgt, const double* tgt, double delta,
                   double tol, const fgt_point_opts_t* opts, fgt_point_plan_t** out) {
  if (!out) return fgt::set_error(FGT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  fgt_point_opts_t o{};
  if (opts) o = *opts;
  const int p = o.p == 0 ? 16 : o.p, ns = o.ns == 0 ? 64 : o.ns;
  fgt_point_plan_t* pp = new (std::nothrow) fgt_point_plan_t();
  if (!pp) return fgt::set_error(FGT_ERR_OOM, "host allocation");
  std::string err;
  int rc;
  try {
    rc = fgt::build_point_plan(dim, nsrc, src, ntgt, tgt, delta, tol, p, ns, pp->ph, err);
  } catch (const std::bad_alloc&) {
    rc = FGT_ERR_OOM;
    err = "host allocation";
  } catch (...) {
    rc = FGT_ERR_INVALID_ARG;
    err = "unexpected exception while planning";
  }
  if (rc != FGT_OK) {
    delete pp;
    return fgt::set_error(rc, err);
  }
  if (!o.host_only) {
    rc = setup(pp, static_cast<hipStream_t>(o.stream));
    if (rc != FGT_OK) {
      const std::string keep = fgt_last_error();
      release(pp);
      return fgt::set_error(rc, keep);
    }
  }
  *out = pp;
  return FGT_OK;
}

int fgt_point_execute(fgt_point_plan_t* pp, const double* q, double* u) {
  if (!pp) return fgt::set_error(FGT_ERR_INVALID_ARG, "plan is NULL");
  if (pp->host_only) return fgt::set_error(FGT_ERR_INVALID_ARG, "host-only plan cannot execute");
  const fgt::PointHost& ph = pp->ph;
  if ((ph.nsrc > 0 && !q) || (ph.ntgt > 0 && !u)) return fgt::set_error(FGT_ERR_INVALID_ARG, "q/u is NULL");
  hipError_t e = hipSetDevice(pp->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if (ph.ntgt == 0) return FGT_OK;
  hipStream_t st = pp->stream;
  const int d = ph.d;
  const int64_t npx = (int64_t)ph.px_level.size();
  if (pp->pw && npx > 0) {
    const unsigned na = (unsigned)(ph.anterp_items.size() / 4), nred = (unsigned)(ph.reduce_items.size() / 3);
    if (d == 3)
      hipLaunchKernelGGL(fgt::k_anterp3, dim3(na), dim3(fgt::kPT), 0, st, q, pp->src_perm, pp->src_xyz,
                         pp->anterp_items, pp->px_coord, ph.lp, ph.p, pp->eta, pp->lam, pp->Q, pp->partial);
    else
      hipLaunchKernelGGL(fgt::k_anterp<2>, dim3(na), dim3(fgt::kPT), 0, st, q, pp->src_perm, pp->src_xyz,
                         pp->anterp_items, pp->px_coord, ph.lp, ph.p, pp->eta, pp->lam, pp->Q, pp->partial);
    if (nred > 0) {
      const int pd = d == 3 ? ph.p * ph.p * ph.p : ph.p * ph.p;
      const unsigned nchunk = (unsigned)((pd + fgt::kPT - 1) / fgt::kPT);
      hipLaunchKernelGGL(fgt::k_anterp_reduce, dim3(nred * nchunk), dim3(fgt::kPT), 0, st, pp->reduce_items,
                         pp->partial, pd, pp->Q);
    }
    int rc = fgt::execute_args(pp->pw->args, pp->Q, pp->U, st);
    if (rc != FGT_OK) return rc;
    const unsigned nb = (unsigned)(ph.interp_items.size() / 2);
    if (nb > 0) {
      if (d == 3)
        hipLaunchKernelGGL(fgt::k_interp3, dim3(nb), dim3(fgt::kPT), 0, st, pp->U, pp->interp_items, pp->px_tgt,
                           pp->px_coord, ph.lp, ph.p, pp->eta, pp->lam, pp->tgt_xyz, pp->uw);
      else
        hipLaunchKernelGGL(fgt::k_interp<2>, dim3(nb), dim3(fgt::kPT), 0, st, pp->U, pp->interp_items, pp->px_tgt,
                           pp->px_coord, ph.lp, ph.p, pp->eta, pp->lam, pp->tgt_xyz, pp->uw);
    }
  }
  const unsigned ndl = (unsigned)(ph.direct_items.size() / 2);
  if (ndl > 0) {
    const double inv_delta = 1.0 / ph.delta;
    if (d == 3)
      hipLaunchKernelGGL(fgt::k_direct<3>, dim3(ndl), dim3(fgt::kPT), 0, st, q, pp->src_perm, pp->src_xyz,
                         pp->tgt_xyz, pp->tgt_perm, pp->leaf_src_start, pp->leaf_tgt_start, pp->dl_tgt, pp->dl_haspw,
                         pp->dl_start, pp->dl_src, pp->direct_items, inv_delta, pp->uw, u);
    else
      hipLaunchKernelGGL(fgt::k_direct<2>, dim3(ndl), dim3(fgt::kPT), 0, st, q, pp->src_perm, pp->src_xyz,
                         pp->tgt_xyz, pp->tgt_perm, pp->leaf_src_start, pp->leaf_tgt_start, pp->dl_tgt, pp->dl_haspw,
                         pp->dl_start, pp->dl_src, pp->direct_items, inv_delta, pp->uw, u);
  }
  e = hipGetLastError();
  return e == hipSuccess ? FGT_OK : hip_fail(e, "kernel launch");
}

int fgt_point_info(const fgt_point_plan_t* pp, fgt_point_info_t* info) {
  if (!pp || !info) return fgt::set_error(FGT_ERR_INVALID_ARG, "plan or info is NULL");
  const fgt::PointHost& ph = pp->ph;
  *info = fgt_point_info_t{};
  info->dim = ph.d;
  info->p = ph.p;
  info->ns = ph.ns;
  info->lc = ph.lc;
  info->lp = ph.lp;
  info->nr = ph.hp.nr;
  info->nsrc = ph.nsrc;
  info->ntgt = ph.ntgt;
  info->nleaves = (int64_t)ph.leaf_level.size();
  info->ndense = ph.n_dense;
  info->npwbox = ph.n_pwbox;
  info->nproxy = (int64_t)ph.px_level.size();
  info->nplist = (int64_t)ph.hp.plist_src.size();
  info->ndirect_terms = ph.n_direct_terms;
  info->delta = ph.delta;
  info->tol = ph.tol;
  info->proxy_err = ph.proxy_err;
  info->device_bytes = pp->device_bytes;
  return FGT_OK;
}

int64_t fgt_point_array(const fgt_point_plan_t* pp, const char* name, void* dst, int64_t cap) {
  if (!pp || !name) return fgt::set_error(FGT_ERR_INVALID_ARG, "plan or name is NULL");
  const fgt::PointHost& ph = pp->ph;
  const std::vector<int32_t>* v = nullptr;
  const std::string n(name);
  if (n == "leaf_level") v = &ph.leaf_level;
  else if (n == "leaf_coord") v = &ph.leaf_coord;
  else if (n == "leaf_dense") v = &ph.leaf_dense;
  else if (n == "src_perm") v = &ph.src_perm;
  else if (n == "tgt_perm") v = &ph.tgt_perm;
  else if (n == "leaf_src_start") v = &ph.leaf_src_start;
  else if (n == "leaf_tgt_start") v = &ph.leaf_tgt_start;
  else if (n == "dl_tgt") v = &ph.dl_tgt;
  else if (n == "dl_haspw") v = &ph.dl_haspw;
  else if (n == "dl_start") v = &ph.dl_start;
  else if (n == "dl_src") v = &ph.dl_src;
  else if (n == "px_coord") v = &ph.px_coord;
  else if (n == "px_src_start") v = &ph.px_src_start;
  else if (n == "px_tgt_start") v = &ph.px_tgt_start;
  else if (n == "plist_start") v = &ph.hp.plist_start;
  else if (n == "plist_src") v = &ph.hp.plist_src;
  else if (n == "plist_dir") v = &ph.hp.plist_dir;
  else if (n == "pw_start") v = &ph.hp.pw_start;
  else if (n == "pwleaf_id") v = &ph.hp.pwleaf_id;
  else return fgt::set_error(FGT_ERR_INVALID_ARG, "unknown array " + n);
  const int64_t len = (int64_t)v->size();
  if (dst && cap > 0) std::memcpy(dst, v->data(), sizeof(int32_t) * (size_t)std::min<int64_t>(cap, len));
  return len;
}

void fgt_point_destroy(fgt_point_plan_t* pp) { release(pp); }

}  // extern "C"
