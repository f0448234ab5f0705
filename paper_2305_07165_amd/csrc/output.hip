// Adaptive trees on the device: resolving a Gaussian-sum density (Algorithm
// 3), output-tree refinement and coarsening of the box Gauss transform
// (Section 4.2, Algorithms 5 and 6), and point evaluation of a tree's
// piecewise polynomial (the leaf model of Eq. (papprox)).
//
// Device work: the coefficient-tail error estimate of Eq. (funerr) per box,
// polynomial prolongation of leaf values to descendants, restriction of four
// (or eight) children's interpolants to their parent's nodes, and point
// evaluation.  The tree edits (which leaves split or merge, rebalancing) are
// host logic in output_host.cpp; every transform runs through fgt_execute.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/fgt.h"
#include "../../include/fgt_density.h"
#include "../../include/fgt_output.h"
#include "fgt_host.h"
#include "output_host.h"
#include "plan_internal.h"

struct fgt_output {
  fgt::LeafTree tree;
  int p = 0;
  int device = 0;
  double* u = nullptr;
  fgt_output_info_t info{};
};

struct fgt_density {
  fgt::LeafTree tree;
  int p = 0;
  double* sigma = nullptr;
  fgt_density_info_t info{};
};

namespace {

constexpr int kThreads = 256;

int hip_err(hipError_t e, const char* what) {
  return fgt::set_error(FGT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

__host__ __device__ inline int ipow_i(int p, int d) {
  int r = 1;
  for (int a = 0; a < d; a++) r *= p;
  return r;
}

// out = M applied along axis a of `in`, whose extents are e[0..2] (axis 0
// fastest, e[a] = p): out[.. i ..] = sum_k M[row(i)][k] in[.. k ..] for i < m,
// row(i) = rows ? rows[i] : i.  M is [p][p] row-major in global memory.
__device__ void contract_axis(const double* __restrict__ in, double* __restrict__ out,
                              const double* __restrict__ M, const int32_t* __restrict__ rows, int m,
                              int p, int a, const int e[3]) {
  int eo[3] = {e[0], e[1], e[2]};
  eo[a] = m;
  const int total = eo[0] * eo[1] * eo[2];
  const int stride = a == 0 ? 1 : (a == 1 ? e[0] : e[0] * e[1]);
  for (int o = threadIdx.x; o < total; o += blockDim.x) {
    const int i0 = o % eo[0];
    const int r = o / eo[0];
    const int i1 = r % eo[1];
    const int i2 = r / eo[1];
    const int ia = a == 0 ? i0 : (a == 1 ? i1 : i2);
    const int row = rows ? rows[ia] : ia;
    const int b0 = a == 0 ? 0 : i0, b1 = a == 1 ? 0 : i1, b2 = a == 2 ? 0 : i2;
    const double* src = in + b0 + e[0] * (b1 + e[1] * b2);
    const double* mr = M + (size_t)row * p;
    double s = 0.0;
    for (int k = 0; k < p; k++) s += mr[k] * src[k * stride];
    out[o] = s;
  }
}

// Sum over the block in a fixed order (wave shuffles, then the waves in
// order); the result is valid in thread 0.  scr holds >= blockDim/64 doubles.
__device__ double block_sum(double v, double* scr) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scr[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) s += scr[w];
  return s;
}

// Per box b: e[b] = sqrt(mean of c_alpha^2 over the tail mask) (Eq. (funerr))
// and l2[b] = int_box u^2 (Gauss-Legendre), from the node values at
// vals[slot[b]] (slot NULL: b) of a box at level[b].
__global__ __launch_bounds__(kThreads) void k_tail(const double* __restrict__ vals,
                                                   const int32_t* __restrict__ slot,
                                                   const int32_t* __restrict__ level, int64_t n, int p,
                                                   int d, const double* __restrict__ V2P,
                                                   const double* __restrict__ wgl,
                                                   const uint8_t* __restrict__ mask, double inv_ntail,
                                                   double* __restrict__ e_out,
                                                   double* __restrict__ l2_out) {
  extern __shared__ double lds[];
  const int np = ipow_i(p, d);
  const int64_t b = blockIdx.x;
  if (b >= n) return;
  double* A = lds;
  double* B = lds + np;
  const double* src = vals + (int64_t)(slot ? slot[b] : b) * np;
  double l2 = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const double v = src[i];
    A[i] = v;
    int r = i;
    double w = 1.0;
    for (int a = 0; a < d; a++) {
      w *= wgl[r % p];
      r /= p;
    }
    l2 += w * v * v;
  }
  __syncthreads();
  const int e[3] = {p, d > 1 ? p : 1, d > 2 ? p : 1};
  double* in = A;
  double* out = B;
  for (int a = 0; a < d; a++) {
    contract_axis(in, out, V2P, nullptr, p, p, a, e);
    __syncthreads();
    double* t = in;
    in = out;
    out = t;
  }
  double tail = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x)
    if (mask[i]) tail += in[i] * in[i];
  const double s_l2 = block_sum(l2, out);
  const double s_tail = block_sum(tail, out + 8);
  if (threadIdx.x == 0) {
    const double half = ldexp(1.0, -level[b] - 1);  // L/2, the Jacobian per axis
    double jac = 1.0;
    for (int a = 0; a < d; a++) jac *= half;
    e_out[b] = sqrt(s_tail * inv_ntail);
    l2_out[b] = s_l2 * jac;
  }
}

// dst[b] = (P_{tab[b,1]} x ... x P_{tab[b,d]}) src[src_slot[b]]: values at the
// nodes of box b from those of the box containing it (tab < 0: same extent on
// that axis, identity).
__global__ __launch_bounds__(kThreads) void k_prolong(const double* __restrict__ src,
                                                      const int32_t* __restrict__ src_slot,
                                                      const int32_t* __restrict__ tab,
                                                      const double* __restrict__ P,
                                                      double* __restrict__ dst, int64_t n, int p,
                                                      int d) {
  extern __shared__ double lds[];
  const int np = ipow_i(p, d);
  const int64_t b = blockIdx.x;
  if (b >= n) return;
  double* A = lds;
  double* B = lds + np;
  const double* s = src + (int64_t)src_slot[b] * np;
  for (int i = threadIdx.x; i < np; i += blockDim.x) A[i] = s[i];
  __syncthreads();
  const int e[3] = {p, d > 1 ? p : 1, d > 2 ? p : 1};
  double* in = A;
  double* out = B;
  for (int a = 0; a < d; a++) {
    const int t = tab[b * d + a];
    if (t < 0) continue;
    contract_axis(in, out, P + (size_t)t * p * p, nullptr, p, p, a, e);
    __syncthreads();
    double* x = in;
    in = out;
    out = x;
  }
  double* o = dst + b * np;
  for (int i = threadIdx.x; i < np; i += blockDim.x) o[i] = in[i];
}

// For candidate parent b: u at the parent's nodes from its 2^d children's
// interpolants (Algorithm 6).  A parent node on axis a lies in child half
// h = (eta >= 0); rows[h][0..m_h) lists those nodes and R[h] holds the child's
// Lagrange basis at them.  Child c has offset bit a = (c >> a) & 1 on axis a.
__global__ __launch_bounds__(kThreads) void k_restrict(double* __restrict__ pool,
                                                       const int32_t* __restrict__ child_slot,
                                                       const int32_t* __restrict__ parent_slot,
                                                       const double* __restrict__ R,
                                                       const int32_t* __restrict__ rows, int m0,
                                                       int m1, int64_t n, int p, int d) {
  extern __shared__ double lds[];
  const int np = ipow_i(p, d);
  const int nd = 1 << d;
  const int64_t b = blockIdx.x;
  if (b >= n) return;
  double* A = lds;
  double* B = lds + np;
  double* dst = pool + (int64_t)parent_slot[b] * np;
  for (int c = 0; c < nd; c++) {
    const double* s = pool + (int64_t)child_slot[b * nd + c] * np;
    for (int i = threadIdx.x; i < np; i += blockDim.x) A[i] = s[i];
    __syncthreads();
    int e[3] = {p, d > 1 ? p : 1, d > 2 ? p : 1};
    double* in = A;
    double* out = B;
    for (int a = 0; a < d; a++) {
      const int h = (c >> a) & 1;
      const int m = h ? m1 : m0;
      contract_axis(in, out, R + (size_t)h * p * p, rows + h * p, m, p, a, e);
      e[a] = m;
      __syncthreads();
      double* x = in;
      in = out;
      out = x;
    }
    const int total = e[0] * e[1] * e[2];
    const int32_t* r0 = rows + (c & 1) * p;
    const int32_t* r1 = rows + ((c >> 1) & 1) * p;
    const int32_t* r2 = rows + ((c >> 2) & 1) * p;
    for (int o = threadIdx.x; o < total; o += blockDim.x) {
      const int i0 = o % e[0];
      const int r = o / e[0];
      const int i1 = r % e[1];
      const int i2 = r / e[1];
      const int q0 = r0[i0], q1 = d > 1 ? r1[i1] : 0, q2 = d > 2 ? r2[i2] : 0;
      dst[q0 + p * (q1 + p * q2)] = in[o];
    }
    __syncthreads();
  }
}

// sigma(x) = sum_i a_i exp(-|x - c_i - s|^2 / w_i^2) at node j of box b, one
// node per thread; the shifts s are {-1,0,1}^d when periodic, else 0.
__global__ __launch_bounds__(kThreads) void k_sample_gauss(const int32_t* __restrict__ level,
                                                           const int32_t* __restrict__ coord, int64_t nbox,
                                                           int p, int d, const double* __restrict__ eta,
                                                           const double* __restrict__ gc,
                                                           const double* __restrict__ gw,
                                                           const double* __restrict__ ga, int64_t ng,
                                                           int periodic, double* __restrict__ out) {
  const int np = ipow_i(p, d);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbox * np) return;
  const int64_t b = t / np;
  int j = (int)(t - b * np);
  const double L = ldexp(1.0, -level[b]);
  double x[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < d; a++) {
    x[a] = -0.5 + ((double)coord[b * d + a] + 0.5) * L + 0.5 * L * eta[j % p];
    j /= p;
  }
  const int nimg = periodic ? (d == 1 ? 3 : (d == 2 ? 9 : 27)) : 1;
  double s = 0.0;
  for (int64_t i = 0; i < ng; i++) {
    const double w2 = gw[i] * gw[i];
    for (int im = 0; im < nimg; im++) {
      int code = im;
      double r2 = 0.0;
      for (int a = 0; a < d; a++) {
        const double sh = periodic ? (double)(code % 3 - 1) : 0.0;
        code /= 3;
        const double dx = x[a] - (gc[i * d + a] + sh);
        r2 += dx * dx;
      }
      s += ga[i] * exp(-r2 / w2);
    }
  }
  out[t] = s;
}

// One point per thread: locate the leaf (last Morton start <= the point's
// key), then sum the tensor Lagrange interpolant of its node values.
template <int P, int D>
__global__ __launch_bounds__(kThreads) void k_interp(const double* __restrict__ u,
                                                     const uint64_t* __restrict__ mkey,
                                                     const int32_t* __restrict__ mleaf,
                                                     const int32_t* __restrict__ level,
                                                     const int32_t* __restrict__ coord, int64_t n,
                                                     int lmax, const double* __restrict__ V2P,
                                                     const double* __restrict__ x, int64_t npts,
                                                     double* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= npts) return;
  const int64_t nb = (int64_t)1 << lmax;
  double xa[D];
  uint64_t key = 0;
  {
    int64_t cell[D];
#pragma unroll
    for (int a = 0; a < D; a++) {
      double v = x[q * D + a];
      v = v < -0.5 ? -0.5 : (v > 0.5 ? 0.5 : v);
      if (!(v == v)) v = -0.5;
      xa[a] = v;
      int64_t c = (int64_t)floor((v + 0.5) * (double)nb);
      cell[a] = c < 0 ? 0 : (c >= nb ? nb - 1 : c);
    }
    for (int bit = 0; bit < lmax; bit++)
#pragma unroll
      for (int a = 0; a < D; a++) key |= (((uint64_t)cell[a] >> bit) & 1ull) << (bit * D + a);
  }
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (mkey[mid] <= key) lo = mid;
    else hi = mid - 1;
  }
  const int32_t leaf = mleaf[lo];
  const double L = ldexp(1.0, -level[leaf]);
  // Legendre values per axis; the Lagrange basis l_j = sum_n V2P[n][j] P_n
  double Pn[D][P];
#pragma unroll
  for (int a = 0; a < D; a++) {
    const double t = 2.0 * (xa[a] - (-0.5 + coord[(int64_t)leaf * D + a] * L)) / L - 1.0;
    Pn[a][0] = 1.0;
    if (P > 1) Pn[a][1] = t;
#pragma unroll
    for (int k = 2; k < P; k++) Pn[a][k] = ((2 * k - 1) * t * Pn[a][k - 1] - (k - 1) * Pn[a][k - 2]) / k;
  }
  double ell0[P];
#pragma unroll
  for (int j = 0; j < P; j++) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < P; k++) s += V2P[k * P + j] * Pn[0][k];
    ell0[j] = s;
  }
  constexpr int NP = D == 1 ? P : (D == 2 ? P * P : P * P * P);
  const double* ul = u + (int64_t)leaf * NP;
  double s = 0.0;
  if constexpr (D == 1) {
#pragma unroll
    for (int j = 0; j < P; j++) s += ell0[j] * ul[j];
  } else if constexpr (D == 2) {
    for (int j2 = 0; j2 < P; j2++) {
      double l2 = 0.0, r = 0.0;
#pragma unroll
      for (int k = 0; k < P; k++) l2 += V2P[k * P + j2] * Pn[1][k];
#pragma unroll
      for (int j = 0; j < P; j++) r += ell0[j] * ul[j + P * j2];
      s += l2 * r;
    }
  } else {
    for (int j3 = 0; j3 < P; j3++) {
      double l3 = 0.0, r3 = 0.0;
#pragma unroll
      for (int k = 0; k < P; k++) l3 += V2P[k * P + j3] * Pn[2][k];
      for (int j2 = 0; j2 < P; j2++) {
        double l2 = 0.0, r = 0.0;
#pragma unroll
        for (int k = 0; k < P; k++) l2 += V2P[k * P + j2] * Pn[1][k];
#pragma unroll
        for (int j = 0; j < P; j++) r += ell0[j] * ul[j + P * (j2 + P * j3)];
        r3 += l2 * r;
      }
      s += l3 * r3;
    }
  }
  out[q] = s;
}

template <int P>
hipError_t launch_interp_p(int d, dim3 g, hipStream_t st, const double* u, const uint64_t* mk,
                           const int32_t* ml, const int32_t* lv, const int32_t* cs, int64_t n,
                           int lmax, const double* V2P, const double* x, int64_t npts, double* out) {
  if (d == 1)
    hipLaunchKernelGGL((k_interp<P, 1>), g, dim3(kThreads), 0, st, u, mk, ml, lv, cs, n, lmax, V2P, x,
                       npts, out);
  else if (d == 2)
    hipLaunchKernelGGL((k_interp<P, 2>), g, dim3(kThreads), 0, st, u, mk, ml, lv, cs, n, lmax, V2P, x,
                       npts, out);
  else
    hipLaunchKernelGGL((k_interp<P, 3>), g, dim3(kThreads), 0, st, u, mk, ml, lv, cs, n, lmax, V2P, x,
                       npts, out);
  return hipGetLastError();
}

hipError_t launch_interp(int p, int d, dim3 g, hipStream_t st, const double* u, const uint64_t* mk,
                         const int32_t* ml, const int32_t* lv, const int32_t* cs, int64_t n, int lmax,
                         const double* V2P, const double* x, int64_t npts, double* out) {
  switch (p) {
#define FGT_INTERP_CASE(PP) \
  case PP: return launch_interp_p<PP>(d, g, st, u, mk, ml, lv, cs, n, lmax, V2P, x, npts, out);
    FGT_INTERP_CASE(1) FGT_INTERP_CASE(2) FGT_INTERP_CASE(3) FGT_INTERP_CASE(4)
    FGT_INTERP_CASE(5) FGT_INTERP_CASE(6) FGT_INTERP_CASE(7) FGT_INTERP_CASE(8)
    FGT_INTERP_CASE(9) FGT_INTERP_CASE(10) FGT_INTERP_CASE(11) FGT_INTERP_CASE(12)
    FGT_INTERP_CASE(13) FGT_INTERP_CASE(14) FGT_INTERP_CASE(15) FGT_INTERP_CASE(16)
#undef FGT_INTERP_CASE
    default: return hipErrorInvalidValue;
  }
}

// Device allocations of one call, released together (after the stream has
// been synchronized).
struct DevArena {
  hipStream_t st = nullptr;
  std::vector<void*> ptrs;
  explicit DevArena(hipStream_t s) : st(s) {}
  ~DevArena() {
    if (!ptrs.empty()) (void)hipStreamSynchronize(st);
    for (void* q : ptrs) (void)hipFree(q);
  }
  int alloc(size_t bytes, void** out) {
    *out = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) {
      *out = nullptr;
      return fgt::set_error(FGT_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    ptrs.push_back(*out);
    return FGT_OK;
  }
  template <typename T>
  int upload(const std::vector<T>& v, T** out, hipStream_t st) {
    void* q;
    int rc = alloc(v.size() * sizeof(T), &q);
    if (rc) return rc;
    *out = static_cast<T*>(q);
    if (v.empty()) return FGT_OK;
    hipError_t e = hipMemcpyAsync(q, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_err(e, "hipMemcpyAsync");
    return FGT_OK;
  }
  void release(void* q) {
    auto it = std::find(ptrs.begin(), ptrs.end(), q);
    if (it != ptrs.end()) {
      (void)hipFree(q);
      ptrs.erase(it);
    }
  }
  // hands ownership of q to the caller
  void keep(void* q) {
    auto it = std::find(ptrs.begin(), ptrs.end(), q);
    if (it != ptrs.end()) ptrs.erase(it);
  }
};

// Tables and scratch of the error estimate, shared by every pass.
struct TailCtx {
  int p = 0, d = 0, np = 0;
  double inv_ntail = 0.0;
  double* V2P = nullptr;
  double* w = nullptr;
  uint8_t* mask = nullptr;
  size_t lds = 0;
};

int tail_setup(DevArena& ar, int p, int d, hipStream_t st, TailCtx& t) {
  std::vector<double> V2P, eta, w;
  fgt::value_to_legendre(p, V2P, eta, w);
  std::vector<uint8_t> mask = fgt::tail_mask(p, d);
  int64_t nt = 0;
  for (uint8_t m : mask) nt += m;
  t.p = p;
  t.d = d;
  t.np = ipow_i(p, d);
  t.inv_ntail = nt > 0 ? 1.0 / (double)nt : 0.0;
  // two buffers of p^d values; at least 16 each, for the block sums of k_tail
  t.lds = 2 * sizeof(double) * (size_t)std::max(t.np, 16);
  int rc;
  if ((rc = ar.upload(V2P, &t.V2P, st)) || (rc = ar.upload(w, &t.w, st)) ||
      (rc = ar.upload(mask, &t.mask, st)))
    return rc;
  return FGT_OK;
}

// e and int u^2 of n boxes whose values sit at vals[slot[b]] (slot NULL: b);
// waits for the stream and returns them on the host.
int tail_run(DevArena& ar, const TailCtx& t, const double* vals, const std::vector<int32_t>* slot,
             const std::vector<int32_t>& level, hipStream_t st, std::vector<double>& e,
             std::vector<double>& l2) {
  const int64_t n = (int64_t)level.size();
  e.assign(n, 0.0);
  l2.assign(n, 0.0);
  if (n == 0) return FGT_OK;
  int32_t* d_lv = nullptr;
  int32_t* d_slot = nullptr;
  void* d_e = nullptr;
  void* d_l2 = nullptr;
  int rc;
  if ((rc = ar.upload(level, &d_lv, st)) || (slot && (rc = ar.upload(*slot, &d_slot, st))) ||
      (rc = ar.alloc(n * sizeof(double), &d_e)) || (rc = ar.alloc(n * sizeof(double), &d_l2)))
    return rc;
  hipLaunchKernelGGL(k_tail, dim3((unsigned)n), dim3(kThreads), t.lds, st, vals, d_slot, d_lv, n, t.p,
                     t.d, t.V2P, t.w, t.mask, t.inv_ntail, static_cast<double*>(d_e),
                     static_cast<double*>(d_l2));
  hipError_t er = hipGetLastError();
  if (er != hipSuccess) return hip_err(er, "k_tail launch");
  if ((er = hipMemcpyAsync(e.data(), d_e, n * sizeof(double), hipMemcpyDeviceToHost, st)) ||
      (er = hipMemcpyAsync(l2.data(), d_l2, n * sizeof(double), hipMemcpyDeviceToHost, st)) ||
      (er = hipStreamSynchronize(st)))
    return hip_err(er, "tail results");
  ar.release(d_lv);
  if (d_slot) ar.release(d_slot);
  ar.release(d_e);
  ar.release(d_l2);
  return FGT_OK;
}

// Values on the leaves of `to` from values on the leaves of `from` (every leaf
// of `to` lies in leaf src[j] of `from`, whose values sit at slot
// from_slot[src[j]]): polynomial prolongation, one table per (depth, offset).
int prolong_run(DevArena& ar, int p, const fgt::LeafTree& from, const std::vector<int32_t>& from_slot,
                const fgt::LeafTree& to, const std::vector<int32_t>& src, const double* vals,
                double* dst, size_t lds, hipStream_t st) {
  const int d = to.d;
  const int64_t n = to.size();
  if (n == 0) return FGT_OK;
  std::map<std::pair<int, int64_t>, int32_t> ids;
  std::vector<double> tabs, Pm;
  std::vector<int32_t> tab((size_t)n * d), slot(n);
  for (int64_t j = 0; j < n; j++) {
    const int32_t s = src[j];
    slot[j] = from_slot[s];
    const int r = to.level[j] - from.level[s];
    for (int a = 0; a < d; a++) {
      if (r == 0) {
        tab[j * d + a] = -1;
        continue;
      }
      const int64_t o = (int64_t)to.coord[j * d + a] - ((int64_t)from.coord[(int64_t)s * d + a] << r);
      auto key = std::make_pair(r, o);
      auto it = ids.find(key);
      if (it == ids.end()) {
        fgt::prolong_matrix(p, r, o, Pm);
        it = ids.emplace(key, (int32_t)ids.size()).first;
        tabs.insert(tabs.end(), Pm.begin(), Pm.end());
      }
      tab[j * d + a] = it->second;
    }
  }
  if (tabs.empty()) tabs.assign(1, 0.0);
  int32_t* d_tab;
  int32_t* d_slot;
  double* d_P;
  int rc;
  if ((rc = ar.upload(tab, &d_tab, st)) || (rc = ar.upload(slot, &d_slot, st)) ||
      (rc = ar.upload(tabs, &d_P, st)))
    return rc;
  hipLaunchKernelGGL(k_prolong, dim3((unsigned)n), dim3(kThreads), lds, st, vals, d_slot, d_tab, d_P,
                     dst, n, p, d);
  hipError_t er = hipGetLastError();
  if (er != hipSuccess) return hip_err(er, "k_prolong launch");
  if ((er = hipStreamSynchronize(st))) return hip_err(er, "prolong");
  ar.release(d_tab);
  ar.release(d_slot);
  ar.release(d_P);
  return FGT_OK;
}

int check_tree(const fgt_tree_t* tree) {
  if (!tree || tree->dim < 1 || tree->dim > 3 || tree->nleaves < 1 || !tree->level || !tree->coord)
    return fgt::set_error(FGT_ERR_INVALID_ARG, "tree is NULL, empty or of dim outside 1..3");
  const int d = tree->dim;
  const int maxlev = d == 3 ? 19 : (d == 2 ? 28 : 30);
  for (int64_t i = 0; i < tree->nleaves; i++) {
    const int l = tree->level[i];
    if (l < 0 || l > maxlev) return fgt::set_error(FGT_ERR_INVALID_ARG, "leaf level out of range");
    for (int a = 0; a < d; a++) {
      const int32_t c = tree->coord[i * d + a];
      if (c < 0 || (int64_t)c >= ((int64_t)1 << l))
        return fgt::set_error(FGT_ERR_NOT_TILING, "leaf coordinate outside [0, 2^level)");
    }
  }
  return FGT_OK;
}

int lds_check(size_t need) {
  int dev = 0, lds_max = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return hip_err(e, "hipDeviceGetAttribute");
  if (need > (size_t)lds_max)
    return fgt::set_error(FGT_ERR_UNSUPPORTED, "output kernels need " + std::to_string(need) +
                                                   " bytes of LDS, device allows " + std::to_string(lds_max));
  return FGT_OK;
}

int resolve(const fgt_tree_t* tree, int p, double delta, double tol, int bc, const fgt_opts_t* opts,
            const fgt_output_opts_t& oo, const double* sigma, fgt_output* res) {
  const int d = tree->dim;
  const int nd = 1 << d;
  const bool periodic = bc == FGT_PERIODIC;
  const double eps = oo.eps > 0 ? oo.eps : tol;
  fgt_opts_t po{};
  po.force_lc = -1;
  if (opts) po = *opts;
  po.host_only = 0;
  po.own_stream = 0;
  po.profile = 0;
  hipStream_t st = static_cast<hipStream_t>(po.stream);
  fgt_output_info_t& info = res->info;
  info = fgt_output_info_t{};
  info.dim = d;
  info.p = p;

  fgt::LeafTree T;
  T.d = d;
  T.level.assign(tree->level, tree->level + tree->nleaves);
  T.coord.assign(tree->coord, tree->coord + tree->nleaves * d);
  int lmax0 = 0;
  for (int32_t l : T.level) lmax0 = std::max(lmax0, (int)l);
  info.nleaves_in = T.size();
  info.nboxes_in = fgt::count_boxes(T);

  DevArena ar(st);
  TailCtx tc;
  int rc = tail_setup(ar, p, d, st, tc);
  if (rc) return rc;
  if ((rc = lds_check(tc.lds))) return rc;
  const int np = tc.np;
  const size_t vbytes = sizeof(double) * (size_t)np;

  const double* cur_sigma = sigma;
  void* own_sigma = nullptr;
  void* u = nullptr;
  std::vector<double> e, l2;
  double thr = 0.0;
  std::vector<int32_t> ident;
  for (int pass = 0;; pass++) {
    if (T.size() >= ((int64_t)1 << 31)) return fgt::set_error(FGT_ERR_UNSUPPORTED, "too many leaves");
    fgt_tree_t tt{d, T.size(), T.level.data(), T.coord.data()};
    fgt_plan_t* pl = nullptr;
    if ((rc = fgt_plan(&tt, p, delta, tol, bc, &po, &pl))) return rc;
    if ((rc = ar.alloc(vbytes * T.size(), &u))) {
      fgt_destroy(pl);
      return rc;
    }
    rc = fgt_execute(pl, cur_sigma, static_cast<double*>(u));
    if (!rc) rc = tail_run(ar, tc, static_cast<double*>(u), nullptr, T.level, st, e, l2);
    fgt_destroy(pl);
    if (rc) return rc;
    info.passes = pass + 1;
    double s = 0.0;
    for (double v : l2) s += v;
    info.u_l2 = std::sqrt(s);
    thr = eps * info.u_l2;
    if (!oo.refine || (oo.max_passes > 0 && pass >= oo.max_passes)) break;
    std::vector<uint8_t> flag(T.size(), 0);
    int64_t nflag = 0;
    for (int64_t i = 0; i < T.size(); i++)
      if (e[i] > thr && T.level[i] < lmax0) {
        flag[i] = 1;
        nflag++;
      }
    if (nflag == 0) break;
    fgt::LeafTree T2;
    std::vector<int32_t> src;
    int64_t ns = 0, nb = 0;
    fgt::split_and_balance(T, flag, periodic, T2, src, &ns, &nb);
    info.added_refine += ns * nd;
    info.added_refine_balance += nb * nd;
    void* ns_sigma = nullptr;
    if ((rc = ar.alloc(vbytes * T2.size(), &ns_sigma))) return rc;
    ident.resize(T.size());
    for (int64_t i = 0; i < T.size(); i++) ident[i] = (int32_t)i;
    if ((rc = prolong_run(ar, p, T, ident, T2, src, cur_sigma, static_cast<double*>(ns_sigma), tc.lds, st)))
      return rc;
    ar.release(u);
    u = nullptr;
    if (own_sigma) ar.release(own_sigma);
    own_sigma = ns_sigma;
    cur_sigma = static_cast<const double*>(ns_sigma);
    T = std::move(T2);
  }
  if (own_sigma) {
    ar.release(own_sigma);
    own_sigma = nullptr;
  }

  if (oo.coarsen) {
    // Algorithm 6 on a pool of values: the refined leaves, then one slot per
    // candidate parent (at most one per internal box of the refined tree)
    const int64_t n = T.size();
    const int64_t cap = fgt::count_boxes(T);
    void* pool = nullptr;
    if ((rc = ar.alloc(vbytes * cap, &pool))) return rc;
    double* P = static_cast<double*>(pool);
    hipError_t er = hipMemcpyAsync(P, u, vbytes * n, hipMemcpyDeviceToDevice, st);
    if (er != hipSuccess) return hip_err(er, "hipMemcpyAsync");
    // restriction tables: parent nodes of each half and the child's basis there
    std::vector<double> eta(p), wq(p), tR[2];
    fgt::gauss_legendre(p, eta.data(), wq.data());
    std::vector<int32_t> rows(2 * p, 0);
    int m[2] = {0, 0};
    std::vector<double> R(2 * (size_t)p * p, 0.0);
    for (int h = 0; h < 2; h++) {
      std::vector<double> t(p), Lm;
      for (int i = 0; i < p; i++) t[i] = h ? 2.0 * eta[i] - 1.0 : 2.0 * eta[i] + 1.0;
      fgt::lagrange_matrix(p, t.data(), p, Lm);
      std::copy(Lm.begin(), Lm.end(), R.begin() + (size_t)h * p * p);
      for (int i = 0; i < p; i++)
        if ((eta[i] >= 0.0) == (h == 1)) rows[h * p + m[h]++] = i;
    }
    double* d_R;
    int32_t* d_rows;
    if ((rc = ar.upload(R, &d_R, st)) || (rc = ar.upload(rows, &d_rows, st))) return rc;
    er = hipStreamSynchronize(st);
    if (er != hipSuccess) return hip_err(er, "coarsen setup");
    ar.release(u);
    u = nullptr;

    const int bits = 58 / d;
    auto key = [&](int l, const int32_t* c) {
      uint64_t k = (uint64_t)l << 58;
      for (int a = 0; a < d; a++) k |= (uint64_t)(uint32_t)c[a] << (a * bits);
      return k;
    };
    struct Box { int32_t c[3]; };
    std::unordered_map<uint64_t, int32_t> slot_of;  // current leaves -> pool slot
    std::vector<std::vector<Box>> bylevel(lmax0 + 2);
    int lmax = 0;
    for (int64_t i = 0; i < n; i++) {
      Box b{{0, 0, 0}};
      for (int a = 0; a < d; a++) b.c[a] = T.coord[i * d + a];
      slot_of[key(T.level[i], b.c)] = (int32_t)i;
      bylevel[T.level[i]].push_back(b);
      lmax = std::max(lmax, (int)T.level[i]);
    }
    int64_t next = n;
    for (int l = lmax - 1; l >= 0; l--) {
      // parents at level l whose 2^d children are all leaves
      std::map<uint64_t, Box> cand;  // ordered: deterministic slots
      std::unordered_map<uint64_t, int> cnt;
      for (const Box& b : bylevel[l + 1]) {
        if (!slot_of.count(key(l + 1, b.c))) continue;
        Box par{{0, 0, 0}};
        for (int a = 0; a < d; a++) par.c[a] = b.c[a] >> 1;
        const uint64_t pk = key(l, par.c);
        if (++cnt[pk] == nd) cand.emplace(pk, par);
      }
      if (cand.empty()) continue;
      const int64_t nc = (int64_t)cand.size();
      if (next + nc > cap) return fgt::set_error(FGT_ERR_INVALID_ARG, "internal: coarsening pool overflow");
      std::vector<int32_t> cs((size_t)nc * nd), ps(nc), lv(nc, l);
      std::vector<Box> order;
      order.reserve(nc);
      int64_t k = 0;
      for (auto& kv : cand) {
        const Box& par = kv.second;
        for (int c = 0; c < nd; c++) {
          int32_t ch[3] = {0, 0, 0};
          for (int a = 0; a < d; a++) ch[a] = 2 * par.c[a] + ((c >> a) & 1);
          cs[k * nd + c] = slot_of.at(key(l + 1, ch));
        }
        ps[k] = (int32_t)(next + k);
        order.push_back(par);
        k++;
      }
      int32_t* d_cs;
      int32_t* d_ps;
      if ((rc = ar.upload(cs, &d_cs, st)) || (rc = ar.upload(ps, &d_ps, st))) return rc;
      hipLaunchKernelGGL(k_restrict, dim3((unsigned)nc), dim3(kThreads), tc.lds, st, P, d_cs, d_ps, d_R,
                         d_rows, m[0], m[1], nc, p, d);
      er = hipGetLastError();
      if (er != hipSuccess) return hip_err(er, "k_restrict launch");
      if ((rc = tail_run(ar, tc, P, &ps, lv, st, e, l2))) return rc;
      ar.release(d_cs);
      ar.release(d_ps);
      next += nc;
      for (int64_t j = 0; j < nc; j++) {
        if (!(e[j] <= thr)) continue;
        const Box& par = order[j];
        for (int c = 0; c < nd; c++) {
          int32_t ch[3] = {0, 0, 0};
          for (int a = 0; a < d; a++) ch[a] = 2 * par.c[a] + ((c >> a) & 1);
          slot_of.erase(key(l + 1, ch));
        }
        slot_of[key(l, par.c)] = ps[j];
        bylevel[l].push_back(par);
        info.deleted_coarsen += nd;
      }
    }
    // the coarsened tree, Morton order, and its slots
    fgt::LeafTree Tc;
    Tc.d = d;
    std::vector<int32_t> slots0;
    for (int l = 0; l <= lmax; l++)
      for (const Box& b : bylevel[l]) {
        auto it = slot_of.find(key(l, b.c));
        if (it == slot_of.end()) continue;
        Tc.level.push_back(l);
        for (int a = 0; a < d; a++) Tc.coord.push_back(b.c[a]);
        slots0.push_back(it->second);
        slot_of.erase(it);  // a box listed twice is taken once
      }
    std::vector<int32_t> perm;
    fgt::morton_sort(Tc, &perm);
    std::vector<int32_t> slots(perm.size());
    for (size_t j = 0; j < perm.size(); j++) slots[j] = slots0[perm[j]];
    // rebalance; new leaves interpolate the leaf they split
    fgt::LeafTree Tf;
    std::vector<int32_t> src;
    int64_t ns = 0, nb = 0;
    fgt::split_and_balance(Tc, {}, periodic, Tf, src, &ns, &nb);
    info.added_balance = nb * nd;
    if ((rc = ar.alloc(vbytes * Tf.size(), &u))) return rc;
    if ((rc = prolong_run(ar, p, Tc, slots, Tf, src, P, static_cast<double*>(u), tc.lds, st))) return rc;
    ar.release(pool);
    T = std::move(Tf);
  }

  if ((rc = tail_run(ar, tc, static_cast<double*>(u), nullptr, T.level, st, e, l2))) return rc;
  info.max_leaf_error = 0.0;
  for (double v : e) info.max_leaf_error = std::max(info.max_leaf_error, v);
  info.threshold = thr;
  info.nleaves = T.size();
  info.nboxes = fgt::count_boxes(T);
  res->tree = std::move(T);
  res->p = p;
  res->u = static_cast<double*>(u);
  ar.keep(u);
  return FGT_OK;
}

// Device copies of a Gaussian sum and of the node positions.
struct GaussDev {
  int d = 0, periodic = 0;
  int64_t n = 0;
  double *c = nullptr, *w = nullptr, *a = nullptr, *eta = nullptr;
};

int check_gaussians(const fgt_gaussians_t* g) {
  if (!g || g->dim < 1 || g->dim > 3 || g->n < 1 || !g->centers || !g->widths || !g->amps)
    return fgt::set_error(FGT_ERR_INVALID_ARG, "gaussians NULL, empty or of dim outside 1..3");
  for (int64_t i = 0; i < g->n; i++)
    if (!(g->widths[i] > 0) || !std::isfinite(g->widths[i]) || !std::isfinite(g->amps[i]))
      return fgt::set_error(FGT_ERR_INVALID_ARG, "gaussian widths must be > 0 and amplitudes finite");
  for (int64_t i = 0; i < g->n * g->dim; i++)
    if (!std::isfinite(g->centers[i])) return fgt::set_error(FGT_ERR_INVALID_ARG, "non-finite center");
  return FGT_OK;
}

int gauss_upload(DevArena& ar, const fgt_gaussians_t* g, int p, hipStream_t st, GaussDev& gd) {
  std::vector<double> eta(p), w(p);
  fgt::gauss_legendre(p, eta.data(), w.data());
  std::vector<double> c(g->centers, g->centers + g->n * g->dim), wd(g->widths, g->widths + g->n),
      a(g->amps, g->amps + g->n);
  gd.d = g->dim;
  gd.n = g->n;
  gd.periodic = g->periodic ? 1 : 0;
  int rc;
  if ((rc = ar.upload(c, &gd.c, st)) || (rc = ar.upload(wd, &gd.w, st)) || (rc = ar.upload(a, &gd.a, st)) ||
      (rc = ar.upload(eta, &gd.eta, st)))
    return rc;
  // the host vectors are about to go out of scope
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_err(e, "gaussian upload");
  return FGT_OK;
}

// sigma at the nodes of boxes (level[i], coord[i*d..]) into out[nbox][p^d]
int sample_run(DevArena& ar, const GaussDev& gd, int p, const std::vector<int32_t>& level,
               const std::vector<int32_t>& coord, double* out, hipStream_t st) {
  const int64_t nbox = (int64_t)level.size();
  if (nbox == 0) return FGT_OK;
  int32_t *d_l, *d_c;
  int rc;
  if ((rc = ar.upload(level, &d_l, st)) || (rc = ar.upload(coord, &d_c, st))) return rc;
  const int64_t nt = nbox * ipow_i(p, gd.d);
  const int64_t nblk = (nt + kThreads - 1) / kThreads;
  if (nblk >= ((int64_t)1 << 31)) return fgt::set_error(FGT_ERR_UNSUPPORTED, "too many nodes in one launch");
  hipLaunchKernelGGL(k_sample_gauss, dim3((unsigned)nblk), dim3(kThreads), 0, st, d_l, d_c, nbox, p, gd.d, gd.eta,
                     gd.c, gd.w, gd.a, gd.n, gd.periodic, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "k_sample_gauss launch");
  if ((e = hipStreamSynchronize(st))) return hip_err(e, "sample");
  ar.release(d_l);
  ar.release(d_c);
  return FGT_OK;
}

// (int_{R^d} sigma^2)^(1/2) of the non-periodized sum, in closed form
double gaussian_l2(const fgt_gaussians_t* g) {
  const int d = g->dim;
  double s = 0.0;
  for (int64_t i = 0; i < g->n; i++)
    for (int64_t j = 0; j < g->n; j++) {
      const double wi2 = g->widths[i] * g->widths[i], wj2 = g->widths[j] * g->widths[j];
      double r2 = 0.0;
      for (int a = 0; a < d; a++) {
        const double dx = g->centers[i * d + a] - g->centers[j * d + a];
        r2 += dx * dx;
      }
      s += g->amps[i] * g->amps[j] * std::pow(M_PI * wi2 * wj2 / (wi2 + wj2), 0.5 * d) *
           std::exp(-r2 / (wi2 + wj2));
    }
  return std::sqrt(std::max(s, 1e-300));
}

int resolve_density(const fgt_gaussians_t* g, int p, double eps, const fgt_resolve_opts_t& o,
                    fgt_density* res) {
  const int d = g->dim;
  const int nd = 1 << d;
  hipStream_t st = static_cast<hipStream_t>(o.stream);
  DevArena ar(st);
  TailCtx tc;
  int rc = tail_setup(ar, p, d, st, tc);
  if (rc) return rc;
  if ((rc = lds_check(tc.lds))) return rc;
  GaussDev gd;
  if ((rc = gauss_upload(ar, g, p, st, gd))) return rc;
  const int np = tc.np;
  fgt_density_info_t& info = res->info;
  info = fgt_density_info_t{};
  info.dim = d;
  info.p = p;
  info.norm = o.norm > 0 ? o.norm : gaussian_l2(g);
  info.threshold = eps * info.norm;

  // level min_level: every box
  std::vector<int32_t> bc;  // coords of the boxes of the current level
  {
    const int64_t nb = (int64_t)1 << o.min_level;
    int64_t total = 1;
    for (int a = 0; a < d; a++) total *= nb;
    bc.resize(total * d);
    for (int64_t i = 0; i < total; i++) {
      int64_t r = i;
      for (int a = 0; a < d; a++) {
        bc[i * d + a] = (int32_t)(r % nb);
        r /= nb;
      }
    }
  }
  fgt::LeafTree T;
  T.d = d;
  const int64_t chunk = std::max<int64_t>(1, ((int64_t)1 << 27) / np);  // <= 1 GiB of samples per launch
  void* vals = nullptr;
  int64_t vals_cap = 0;  // boxes the sample buffer holds
  for (int l = o.min_level; !bc.empty(); l++) {
    const int64_t nb = (int64_t)bc.size() / d;
    std::vector<int32_t> next;
    for (int64_t s0 = 0; s0 < nb; s0 += chunk) {
      const int64_t m = std::min(chunk, nb - s0);
      std::vector<uint8_t> split(m, 0);
      if (l < o.max_level) {
        if (m > vals_cap) {
          if (vals) ar.release(vals);
          vals = nullptr;
          vals_cap = std::min(chunk, std::max(m, 2 * vals_cap));
          if ((rc = ar.alloc(sizeof(double) * (size_t)np * vals_cap, &vals))) return rc;
        }
        std::vector<int32_t> lv(m, l), cs(bc.begin() + s0 * d, bc.begin() + (s0 + m) * d);
        if ((rc = sample_run(ar, gd, p, lv, cs, static_cast<double*>(vals), st))) return rc;
        std::vector<double> e, l2;
        if ((rc = tail_run(ar, tc, static_cast<double*>(vals), nullptr, lv, st, e, l2))) return rc;
        for (int64_t i = 0; i < m; i++) split[i] = e[i] > info.threshold;
        info.boxes_sampled += m;
      }
      for (int64_t i = 0; i < m; i++) {
        const int32_t* c = &bc[(s0 + i) * d];
        if (!split[i]) {
          T.level.push_back(l);
          for (int a = 0; a < d; a++) T.coord.push_back(c[a]);
          continue;
        }
        for (int k = 0; k < nd; k++)
          for (int a = 0; a < d; a++) next.push_back(2 * c[a] + ((k >> a) & 1));
      }
    }
    if (o.max_leaves > 0 && T.size() + (int64_t)next.size() / d > o.max_leaves)
      return fgt::set_error(FGT_ERR_UNSUPPORTED, "the tree would exceed max_leaves");
    bc.swap(next);
  }
  if (vals) ar.release(vals);
  info.nleaves_unbalanced = T.size();
  fgt::LeafTree B;
  std::vector<int32_t> src;
  fgt::split_and_balance(T, {}, g->periodic != 0, B, src, nullptr, nullptr);
  void* sig = nullptr;
  if ((rc = ar.alloc(sizeof(double) * (size_t)np * B.size(), &sig))) return rc;
  for (int64_t s0 = 0; s0 < B.size(); s0 += chunk) {
    const int64_t m = std::min(chunk, B.size() - s0);
    std::vector<int32_t> lv(B.level.begin() + s0, B.level.begin() + s0 + m),
        cs(B.coord.begin() + s0 * d, B.coord.begin() + (s0 + m) * d);
    if ((rc = sample_run(ar, gd, p, lv, cs, static_cast<double*>(sig) + s0 * np, st))) return rc;
  }
  info.nleaves = B.size();
  info.lmin = 1 << 30;
  info.lmax = 0;
  for (int32_t l : B.level) {
    info.lmin = std::min(info.lmin, (int32_t)l);
    info.lmax = std::max(info.lmax, (int32_t)l);
  }
  res->tree = std::move(B);
  res->p = p;
  res->sigma = static_cast<double*>(sig);
  ar.keep(sig);
  return FGT_OK;
}

}  // namespace

extern "C" {

int fgt_output_resolve(const fgt_tree_t* tree, int p, double delta, double tol, int bc,
                       const fgt_opts_t* opts, const fgt_output_opts_t* oopts, const double* sigma_dev,
                       fgt_output_t** out) {
  if (!out) return fgt::set_error(FGT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int rc = check_tree(tree);
  if (rc) return rc;
  if (!sigma_dev) return fgt::set_error(FGT_ERR_INVALID_ARG, "sigma is NULL");
  if (p < 1 || p > fgt::kMaxP) return fgt::set_error(FGT_ERR_INVALID_ARG, "p must be in [1,16]");
  fgt_output_opts_t oo{0.0, 1, 1, 0};
  if (oopts) oo = *oopts;
  if (oo.eps < 0 || oo.eps >= 1 || oo.max_passes < 0)
    return fgt::set_error(FGT_ERR_INVALID_ARG, "eps must be in [0, 1) and max_passes >= 0");
  fgt_output* res = new (std::nothrow) fgt_output();
  if (!res) return fgt::set_error(FGT_ERR_OOM, "host allocation");
  try {
    rc = resolve(tree, p, delta, tol, bc, opts, oo, sigma_dev, res);
  } catch (const std::bad_alloc&) {
    rc = fgt::set_error(FGT_ERR_OOM, "host allocation");
  } catch (...) {
    rc = fgt::set_error(FGT_ERR_INVALID_ARG, "unexpected exception while resolving the output");
  }
  if (rc) {
    delete res;
    return rc;
  }
  (void)hipGetDevice(&res->device);
  *out = res;
  return FGT_OK;
}

int fgt_output_info(const fgt_output_t* o, fgt_output_info_t* info) {
  if (!o || !info) return fgt::set_error(FGT_ERR_INVALID_ARG, "NULL argument");
  *info = o->info;
  return FGT_OK;
}

int fgt_output_tree(const fgt_output_t* o, int32_t* level, int32_t* coord) {
  if (!o || !level || !coord) return fgt::set_error(FGT_ERR_INVALID_ARG, "NULL argument");
  std::copy(o->tree.level.begin(), o->tree.level.end(), level);
  std::copy(o->tree.coord.begin(), o->tree.coord.end(), coord);
  return FGT_OK;
}

int fgt_output_values(const fgt_output_t* o, double* u_dev) {
  if (!o || !u_dev) return fgt::set_error(FGT_ERR_INVALID_ARG, "NULL argument");
  const size_t bytes = sizeof(double) * (size_t)o->tree.size() * ipow_i(o->p, o->tree.d);
  hipError_t e = hipMemcpy(u_dev, o->u, bytes, hipMemcpyDeviceToDevice);
  if (e != hipSuccess) return hip_err(e, "hipMemcpy");
  return FGT_OK;
}

void fgt_output_destroy(fgt_output_t* o) {
  if (!o) return;
  if (o->u) (void)hipFree(o->u);
  delete o;
}

int fgt_interp(const fgt_tree_t* tree, int p, const double* u_dev, int64_t npts, const double* x_dev,
               double* out_dev, void* stream) {
  int rc = check_tree(tree);
  if (rc) return rc;
  if (p < 1 || p > fgt::kMaxP) return fgt::set_error(FGT_ERR_INVALID_ARG, "p must be in [1,16]");
  if (npts < 0 || (npts > 0 && (!u_dev || !x_dev || !out_dev)))
    return fgt::set_error(FGT_ERR_INVALID_ARG, "npts < 0 or a NULL array");
  if (npts == 0) return FGT_OK;
  if (npts > ((int64_t)1 << 40)) return fgt::set_error(FGT_ERR_UNSUPPORTED, "too many points");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int d = tree->dim;
  const int64_t n = tree->nleaves;
  int lmax = 0;
  for (int64_t i = 0; i < n; i++) lmax = std::max(lmax, (int)tree->level[i]);
  try {
    std::vector<std::pair<uint64_t, int32_t>> k(n);
    for (int64_t i = 0; i < n; i++)
      k[i] = {fgt::morton_key(d, tree->level[i], &tree->coord[i * d], lmax), (int32_t)i};
    std::sort(k.begin(), k.end());
    std::vector<uint64_t> mkey(n);
    std::vector<int32_t> mleaf(n), lv(tree->level, tree->level + n), cs(tree->coord, tree->coord + n * d);
    for (int64_t j = 0; j < n; j++) {
      mkey[j] = k[j].first;
      mleaf[j] = k[j].second;
    }
    std::vector<double> V2P, eta, w;
    fgt::value_to_legendre(p, V2P, eta, w);
    DevArena ar(st);
    uint64_t* d_k;
    int32_t *d_l, *d_lv, *d_cs;
    double* d_V;
    if ((rc = ar.upload(mkey, &d_k, st)) || (rc = ar.upload(mleaf, &d_l, st)) ||
        (rc = ar.upload(lv, &d_lv, st)) || (rc = ar.upload(cs, &d_cs, st)) || (rc = ar.upload(V2P, &d_V, st)))
      return rc;
    const int64_t nblk = (npts + kThreads - 1) / kThreads;
    if (nblk >= ((int64_t)1 << 31)) return fgt::set_error(FGT_ERR_UNSUPPORTED, "too many points");
    hipError_t e = launch_interp(p, d, dim3((unsigned)nblk), st, u_dev, d_k, d_l, d_lv, d_cs, n, lmax, d_V,
                                 x_dev, npts, out_dev);
    if (e != hipSuccess) return hip_err(e, "k_interp launch");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(e, "fgt_interp");
  } catch (const std::bad_alloc&) {
    return fgt::set_error(FGT_ERR_OOM, "host allocation");
  }
  return FGT_OK;
}

int64_t fgt_tree_balance(const fgt_tree_t* tree, int bc, int32_t* level_out, int32_t* coord_out,
                         int64_t cap) {
  int rc = check_tree(tree);
  if (rc) return rc;
  if (bc != FGT_FREE && bc != FGT_PERIODIC) return fgt::set_error(FGT_ERR_INVALID_ARG, "bad bc");
  try {
    fgt::LeafTree T, B;
    T.d = tree->dim;
    T.level.assign(tree->level, tree->level + tree->nleaves);
    T.coord.assign(tree->coord, tree->coord + tree->nleaves * tree->dim);
    std::vector<int32_t> src;
    fgt::split_and_balance(T, {}, bc == FGT_PERIODIC, B, src, nullptr, nullptr);
    const int64_t n = B.size();
    if (level_out && coord_out) {
      const int64_t m = std::min(n, cap);
      std::copy(B.level.begin(), B.level.begin() + m, level_out);
      std::copy(B.coord.begin(), B.coord.begin() + m * T.d, coord_out);
    }
    return n;
  } catch (const std::bad_alloc&) {
    return fgt::set_error(FGT_ERR_OOM, "host allocation");
  }
}

int fgt_resolve_gaussians(const fgt_gaussians_t* g, int p, double eps, const fgt_resolve_opts_t* opts,
                          fgt_density_t** out) {
  if (!out) return fgt::set_error(FGT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int rc = check_gaussians(g);
  if (rc) return rc;
  if (p < 1 || p > fgt::kMaxP) return fgt::set_error(FGT_ERR_INVALID_ARG, "p must be in [1,16]");
  if (!(eps > 0 && eps < 1)) return fgt::set_error(FGT_ERR_INVALID_ARG, "eps must be in (0, 1)");
  fgt_resolve_opts_t o{0, 12, 0, 0.0, nullptr};
  if (opts) o = *opts;
  const int maxlev = g->dim == 3 ? 19 : (g->dim == 2 ? 28 : 30);
  if (o.min_level < 0 || o.max_level < o.min_level || o.max_level > maxlev || o.max_leaves < 0 || o.norm < 0)
    return fgt::set_error(FGT_ERR_INVALID_ARG, "need 0 <= min_level <= max_level <= the dimension's limit");
  if ((int64_t)g->dim * o.min_level > 24)
    return fgt::set_error(FGT_ERR_UNSUPPORTED, "min_level gives more than 2^24 boxes");
  fgt_density* res = new (std::nothrow) fgt_density();
  if (!res) return fgt::set_error(FGT_ERR_OOM, "host allocation");
  try {
    rc = resolve_density(g, p, eps, o, res);
  } catch (const std::bad_alloc&) {
    rc = fgt::set_error(FGT_ERR_OOM, "host allocation");
  }
  if (rc) {
    delete res;
    return rc;
  }
  *out = res;
  return FGT_OK;
}

int fgt_density_info(const fgt_density_t* r, fgt_density_info_t* info) {
  if (!r || !info) return fgt::set_error(FGT_ERR_INVALID_ARG, "NULL argument");
  *info = r->info;
  return FGT_OK;
}

int fgt_density_tree(const fgt_density_t* r, int32_t* level, int32_t* coord) {
  if (!r || !level || !coord) return fgt::set_error(FGT_ERR_INVALID_ARG, "NULL argument");
  std::copy(r->tree.level.begin(), r->tree.level.end(), level);
  std::copy(r->tree.coord.begin(), r->tree.coord.end(), coord);
  return FGT_OK;
}

int fgt_density_values(const fgt_density_t* r, double* sigma_dev) {
  if (!r || !sigma_dev) return fgt::set_error(FGT_ERR_INVALID_ARG, "NULL argument");
  const size_t bytes = sizeof(double) * (size_t)r->tree.size() * ipow_i(r->p, r->tree.d);
  hipError_t e = hipMemcpy(sigma_dev, r->sigma, bytes, hipMemcpyDeviceToDevice);
  if (e != hipSuccess) return hip_err(e, "hipMemcpy");
  return FGT_OK;
}

void fgt_density_destroy(fgt_density_t* r) {
  if (!r) return;
  if (r->sigma) (void)hipFree(r->sigma);
  delete r;
}

int fgt_sample_gaussians(const fgt_gaussians_t* g, const fgt_tree_t* tree, int p, double* sigma_dev,
                         void* stream) {
  int rc = check_gaussians(g);
  if (rc || (rc = check_tree(tree))) return rc;
  if (tree->dim != g->dim) return fgt::set_error(FGT_ERR_INVALID_ARG, "tree and gaussians differ in dim");
  if (p < 1 || p > fgt::kMaxP) return fgt::set_error(FGT_ERR_INVALID_ARG, "p must be in [1,16]");
  if (!sigma_dev) return fgt::set_error(FGT_ERR_INVALID_ARG, "sigma is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  try {
    DevArena ar(st);
    GaussDev gd;
    if ((rc = gauss_upload(ar, g, p, st, gd))) return rc;
    const int d = tree->dim;
    const int64_t np = ipow_i(p, d);
    const int64_t chunk = std::max<int64_t>(1, ((int64_t)1 << 27) / np);
    for (int64_t s0 = 0; s0 < tree->nleaves; s0 += chunk) {
      const int64_t m = std::min(chunk, tree->nleaves - s0);
      std::vector<int32_t> lv(tree->level + s0, tree->level + s0 + m),
          cs(tree->coord + s0 * d, tree->coord + (s0 + m) * d);
      if ((rc = sample_run(ar, gd, p, lv, cs, sigma_dev + s0 * np, st))) return rc;
    }
  } catch (const std::bad_alloc&) {
    return fgt::set_error(FGT_ERR_OOM, "host allocation");
  }
  return FGT_OK;
}

}  // extern "C"
