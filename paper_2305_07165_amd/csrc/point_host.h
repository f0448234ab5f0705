// Host plan of the point Gauss transform with proxy grids (the paper's closing
// remark: the sources of a leaf replaced by an equivalent tensor grid of
// proxy points, so that the plane-wave stages run in tensor form).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "fgt_host.h"

namespace fgt {

struct PointHost {
  int d = 0, p = 0, ns = 0;
  double delta = 0, tol = 0;
  int64_t nsrc = 0, ntgt = 0;
  int lc = 0;      // cutoff level (box side >= D0 sqrt(delta))
  int lp = 0;      // proxy level: the proxy grids sit on the boxes of level lp inside
                   // the plane-wave boxes (lp - lc chosen from p and tol)
  double proxy_err = 0;  // worst interpolation error of a plane wave on a proxy box

  // Algorithm 1's leaves (levels <= lc), Morton order
  std::vector<int32_t> leaf_level, leaf_coord;  // coord[i*d+a]
  std::vector<int32_t> leaf_dense;              // more than ns sources or targets, at lc
  // points sorted by (leaf, proxy box): caller index of each sorted position
  std::vector<int32_t> src_perm, tgt_perm;
  std::vector<double> src_xyz, tgt_xyz;         // sorted coordinates [n][d]
  std::vector<int32_t> leaf_src_start, leaf_tgt_start;  // [nleaf+1]

  // direct part (Algorithm 2, last loop, read from the target side): for each
  // leaf with targets, the leaves with sources in its D-list
  std::vector<int32_t> dl_tgt;     // [nDT] target leaf
  std::vector<int32_t> dl_haspw;   // [nDT] 1: its targets also receive plane waves
  std::vector<int32_t> dl_start;   // [nDT+1]
  std::vector<int32_t> dl_src;     // source leaf

  // proxy boxes (the plane-wave "leaves"): level lp, global coords
  std::vector<int32_t> px_level, px_coord;
  std::vector<int32_t> px_src_start, px_tgt_start;  // [2 npx]: [start, end) of the sorted
                                                    // points of each proxy box (sources: dense
                                                    // boxes only)
  std::vector<int32_t> px_tgt_list;                 // proxy boxes holding targets
  // work items of 256 targets: (proxy box, first sorted target) for the
  // interpolation, (D-list entry, first sorted target) for the direct sums
  std::vector<int32_t> interp_items, direct_items;
  // anterpolation items (proxy box, first source, end source, partial slot or
  // -1) with at most kAnterpPart sources each; grids of several parts are
  // summed by the reduce items (proxy box, first slot, parts)
  std::vector<int32_t> anterp_items, reduce_items;
  int64_t n_anterp_slots = 0;

  // the plane-wave stages over the proxy boxes (box Gauss transform kernels)
  HostPlan hp;
  int64_t n_dense = 0, n_pwbox = 0, n_direct_terms = 0;
};

// Builds the whole host plan.  src/tgt: [n][d] points of [-1/2, 1/2]^d.
int build_point_plan(int d, int64_t nsrc, const double* src, int64_t ntgt, const double* tgt,
                     double delta, double tol, int p, int ns, PointHost& ph, std::string& err);

// Barycentric weights of the p Gauss-Legendre nodes (Lagrange interpolation).
void gl_barycentric(int p, std::vector<double>& eta, std::vector<double>& lam);

}  // namespace fgt
