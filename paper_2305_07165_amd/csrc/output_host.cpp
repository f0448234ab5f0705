// Host side of the output-tree refinement and coarsening (Section 4.2).
#include "output_host.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <unordered_map>
#include <unordered_set>

#include "fgt_host.h"

namespace fgt {

namespace {

int max_level_of(int d) { return d == 3 ? 19 : (d == 2 ? 28 : 30); }

// Unique key of a box (level, coords): level in the top 6 bits, then 58/d bits
// per axis.
struct BoxKey {
  int d, bits;
  explicit BoxKey(int dim) : d(dim), bits(58 / dim) {}
  uint64_t operator()(int l, const int32_t* c) const {
    uint64_t k = (uint64_t)l << 58;
    for (int a = 0; a < d; a++) k |= (uint64_t)(uint32_t)c[a] << (a * bits);
    return k;
  }
};

void legendre_row(int p, double t, double* P) {
  P[0] = 1.0;
  if (p > 1) P[1] = t;
  for (int n = 2; n < p; n++) P[n] = ((2 * n - 1) * t * P[n - 1] - (n - 1) * P[n - 2]) / n;
}

}  // namespace

void split_and_balance(const LeafTree& in, const std::vector<uint8_t>& split, bool periodic,
                       LeafTree& out, std::vector<int32_t>& src, int64_t* n_split,
                       int64_t* n_balance) {
  const int d = in.d, nd = 1 << d, n3 = d == 1 ? 3 : (d == 2 ? 9 : 27);
  const int maxlev = max_level_of(d);
  BoxKey key(d);
  using Entry = std::array<int32_t, 4>;  // coords (3), source leaf
  std::unordered_map<uint64_t, int32_t> leaf;  // key -> source leaf
  std::vector<std::vector<Entry>> bylevel(maxlev + 2);
  leaf.reserve((size_t)in.size() * 2);
  auto add = [&](int l, const int32_t* c, int32_t s) {
    leaf[key(l, c)] = s;
    bylevel[l].push_back({c[0], d > 1 ? c[1] : 0, d > 2 ? c[2] : 0, s});
  };
  auto split_box = [&](int l, const int32_t* c, int32_t s) {
    leaf.erase(key(l, c));
    for (int b = 0; b < nd; b++) {
      int32_t ch[3] = {0, 0, 0};
      for (int a = 0; a < d; a++) ch[a] = 2 * c[a] + ((b >> a) & 1);
      add(l + 1, ch, s);
    }
  };
  int64_t ns = 0, nb = 0;
  for (int64_t i = 0; i < in.size(); i++) {
    const int32_t* c = &in.coord[i * d];
    if (!split.empty() && split[i] && in.level[i] < maxlev) {
      // the parent is never recorded as a leaf
      for (int b = 0; b < nd; b++) {
        int32_t ch[3] = {0, 0, 0};
        for (int a = 0; a < d; a++) ch[a] = 2 * c[a] + ((b >> a) & 1);
        add(in.level[i] + 1, ch, (int32_t)i);
      }
      ns++;
    } else {
      add(in.level[i], c, (int32_t)i);
    }
  }
  int lmax = 0;
  for (int l = 0; l <= maxlev + 1; l++)
    if (!bylevel[l].empty()) lmax = l;
  // finest level first: a split only creates leaves at coarser levels than
  // the one being checked, which are checked later
  for (int l = lmax; l >= 2; l--) {
    const int64_t nbox = (int64_t)1 << l;
    for (size_t k = 0; k < bylevel[l].size(); k++) {
      const Entry e = bylevel[l][k];
      if (!leaf.count(key(l, e.data()))) continue;
      for (int code = 0; code < n3; code++) {
        int32_t q[3] = {0, 0, 0};
        bool zero = true, inside = true;
        int cc = code;
        for (int a = 0; a < d; a++) {
          const int dir = cc % 3 - 1;
          cc /= 3;
          zero = zero && dir == 0;
          int64_t v = (int64_t)e[a] + dir;
          if (v < 0 || v >= nbox) {
            if (!periodic) inside = false;
            v = (v + nbox) % nbox;
          }
          q[a] = (int32_t)v;
        }
        if (zero || !inside) continue;
        // the leaf covering box (l, q), if it is coarser than l - 1
        for (int ll = l - 2; ll >= 0; ll--) {
          int32_t c[3] = {0, 0, 0};
          for (int a = 0; a < d; a++) c[a] = q[a] >> (l - ll);
          auto it = leaf.find(key(ll, c));
          if (it == leaf.end()) continue;
          const int32_t s = it->second;
          for (int m = ll; m < l - 1; m++) {
            for (int a = 0; a < d; a++) c[a] = q[a] >> (l - m);
            split_box(m, c, s);
            nb++;
          }
          break;
        }
      }
    }
  }
  out = LeafTree();
  out.d = d;
  std::vector<int32_t> s0;
  for (int l = 0; l <= maxlev + 1; l++)
    for (const Entry& e : bylevel[l]) {
      auto it = leaf.find(key(l, e.data()));
      if (it == leaf.end()) continue;
      out.level.push_back(l);
      for (int a = 0; a < d; a++) out.coord.push_back(e[a]);
      s0.push_back(it->second);
    }
  std::vector<int32_t> perm;
  morton_sort(out, &perm);
  src.resize(perm.size());
  for (size_t j = 0; j < perm.size(); j++) src[j] = s0[perm[j]];
  if (n_split) *n_split = ns;
  if (n_balance) *n_balance = nb;
}

int64_t count_boxes(const LeafTree& t) {
  const int d = t.d;
  BoxKey key(d);
  std::unordered_set<uint64_t> seen;
  seen.reserve((size_t)t.size() * 2);
  for (int64_t i = 0; i < t.size(); i++) {
    int32_t c[3] = {0, 0, 0};
    for (int a = 0; a < d; a++) c[a] = t.coord[i * d + a];
    for (int l = t.level[i]; l >= 0; l--) {
      if (!seen.insert(key(l, c)).second) break;
      for (int a = 0; a < d; a++) c[a] >>= 1;
    }
  }
  return (int64_t)seen.size();
}

uint64_t morton_key(int d, int level, const int32_t* coord, int lmax) {
  uint64_t v[3] = {0, 0, 0};
  for (int a = 0; a < d; a++) v[a] = (uint64_t)(uint32_t)coord[a] << (lmax - level);
  uint64_t m = 0;
  for (int b = 0; b < lmax; b++)
    for (int a = 0; a < d; a++) m |= ((v[a] >> b) & 1ull) << (b * d + a);
  return m;
}

void morton_sort(LeafTree& t, std::vector<int32_t>* perm_out) {
  const int d = t.d;
  const int64_t n = t.size();
  int lmax = 0;
  for (int32_t l : t.level) lmax = std::max(lmax, (int)l);
  std::vector<std::pair<uint64_t, int32_t>> k(n);
  for (int64_t i = 0; i < n; i++) k[i] = {morton_key(d, t.level[i], &t.coord[i * d], lmax), (int32_t)i};
  std::sort(k.begin(), k.end());
  LeafTree s;
  s.d = d;
  s.level.resize(n);
  s.coord.resize(n * d);
  std::vector<int32_t> perm(n);
  for (int64_t j = 0; j < n; j++) {
    const int32_t i = k[j].second;
    perm[j] = i;
    s.level[j] = t.level[i];
    for (int a = 0; a < d; a++) s.coord[j * d + a] = t.coord[i * d + a];
  }
  t = std::move(s);
  if (perm_out) *perm_out = std::move(perm);
}

void value_to_legendre(int p, std::vector<double>& V2P, std::vector<double>& eta,
                       std::vector<double>& w) {
  eta.assign(p, 0.0);
  w.assign(p, 0.0);
  gauss_legendre(p, eta.data(), w.data());
  V2P.assign((size_t)p * p, 0.0);
  std::vector<double> P(p);
  for (int j = 0; j < p; j++) {
    legendre_row(p, eta[j], P.data());
    for (int n = 0; n < p; n++) V2P[(size_t)n * p + j] = 0.5 * (2 * n + 1) * w[j] * P[n];
  }
}

void lagrange_matrix(int p, const double* t, int m, std::vector<double>& L) {
  std::vector<double> V2P, eta, w, P(p);
  value_to_legendre(p, V2P, eta, w);
  L.assign((size_t)m * p, 0.0);
  for (int i = 0; i < m; i++) {
    legendre_row(p, t[i], P.data());
    for (int j = 0; j < p; j++) {
      double s = 0.0;
      for (int n = 0; n < p; n++) s += V2P[(size_t)n * p + j] * P[n];
      L[(size_t)i * p + j] = s;
    }
  }
}

void prolong_matrix(int p, int r, int64_t o, std::vector<double>& Pm) {
  std::vector<double> eta(p), w(p), t(p);
  gauss_legendre(p, eta.data(), w.data());
  const double scale = std::ldexp(1.0, -r);
  for (int i = 0; i < p; i++) t[i] = -1.0 + (2.0 * (double)o + 1.0 + eta[i]) * scale;
  lagrange_matrix(p, t.data(), p, Pm);
}

std::vector<uint8_t> tail_mask(int p, int d) {
  int64_t np = 1;
  for (int a = 0; a < d; a++) np *= p;
  std::vector<uint8_t> m(np, 0);
  for (int64_t i = 0; i < np; i++) {
    int64_t r = i, s2 = 0, a1 = 0;
    for (int a = 0; a < d; a++) {
      const int64_t al = r % p;
      r /= p;
      s2 += al * al;
      if (a == 0) a1 = al;
    }
    m[i] = d == 1 ? (a1 >= p - 2) : (s2 >= (int64_t)p * p);
  }
  return m;
}

}  // namespace fgt
