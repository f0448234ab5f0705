// Host side of the output-tree refinement and coarsening (Section 4.2,
// Algorithms 5 and 6): tree edits with 2:1 rebalancing, the interpolation
// tables that move leaf values between a box and its descendants, the
// coefficient-tail mask of Eq. (funerr), and the point locator.
#pragma once

#include <cstdint>
#include <vector>

namespace fgt {

struct LeafTree {
  int d = 0;
  std::vector<int32_t> level, coord;  // coord[i*d+a]
  int64_t size() const { return (int64_t)level.size(); }
};

// Splits the leaves with split[i] != 0 into their 2^d children, then splits
// coarse leaves until every two leaves that share a boundary point (corner
// adjacency, wrapped when periodic) differ by at most one level.  out lists
// the resulting leaves in Morton order of their lower corners; src[j] is the
// leaf of `in` that contains out leaf j.  *n_split and *n_balance receive the
// number of requested and of balancing splits.
void split_and_balance(const LeafTree& in, const std::vector<uint8_t>& split, bool periodic,
                       LeafTree& out, std::vector<int32_t>& src, int64_t* n_split,
                       int64_t* n_balance);

// Number of boxes of the tree: its leaves and all their ancestors.
int64_t count_boxes(const LeafTree& t);

// Leaves in Morton order of their lower corners (at the finest level).
void morton_sort(LeafTree& t, std::vector<int32_t>* perm);

// Lower-corner Morton key of a box at resolution lmax (d * lmax <= 60 bits).
uint64_t morton_key(int d, int level, const int32_t* coord, int lmax);

// Legendre coefficients from node values on [-1,1]: c_n = sum_j V2P[n][j] v_j
// (Eq. (val2poleq)); and the Gauss-Legendre weights.
void value_to_legendre(int p, std::vector<double>& V2P, std::vector<double>& eta,
                       std::vector<double>& w);

// Lagrange matrix L[i][j] = l_j(t_i) of the p Gauss-Legendre nodes at m points.
void lagrange_matrix(int p, const double* t, int m, std::vector<double>& L);

// Values at the nodes of a descendant r levels below, at offset o (0 <= o <
// 2^r) along one axis, from the values at the box's own nodes: [p][p].
void prolong_matrix(int p, int r, int64_t o, std::vector<double>& P);

// The tail of Eq. (funerr): multi-indices alpha (axis 1 fastest) with
// ||alpha||_2 >= p; for d = 1, where that set is empty, the last two orders.
std::vector<uint8_t> tail_mask(int p, int d);

}  // namespace fgt
