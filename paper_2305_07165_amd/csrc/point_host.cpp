// Host plan of the point Gauss transform with proxy grids.
//
// The tree is Algorithm 1's: boxes with more than n_s sources or targets are
// split down to the cutoff level l_c (side >= D0 sqrt(delta)), the tree is
// level-restricted, and a leaf at l_c holding more than n_s points (dense)
// gets no coarse neighbor.  Interactions follow Eq. (pgt2) and the P- and
// D-lists defined after Algorithm 1: a target in a leaf T at l_c takes every
// dense colleague (T itself included) by plane waves and the rest of its
// neighbor list directly; targets in leaves above l_c take their whole
// neighbor list directly.
//
// Plane waves run through proxy grids, as the paper's closing remark
// proposes: inside every plane-wave box the points are binned into the boxes
// of a finer level l_p, and each occupied one carries the tensor grid of p
// Gauss-Legendre nodes per axis.  Charges are spread to the grid by Lagrange
// interpolation weights (anterpolation), so that the grid's outgoing plane-wave
// expansion (Eq. (multipoleexpansion)) is that of the points; the incoming
// expansion is evaluated on the grid (Eq. (localexpansion)) and interpolated to
// the targets.  l_p is the coarsest level at which p nodes interpolate every
// plane wave of the expansion to tol / (10 d) on a proxy box.  The grids are
// then exactly the leaves of a box transform, and its kernels run unchanged
// with the formation tables evaluated at the proxy nodes instead of
// integrated.
#include "point_host.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <unordered_map>

#include "../../include/fgt.h"
#include "output_host.h"

namespace fgt {

namespace {

struct BoxKey {
  int d, bits;
  explicit BoxKey(int dim) : d(dim), bits(58 / dim) {}
  uint64_t operator()(int l, const int32_t* c) const {
    uint64_t k = (uint64_t)l << 58;
    for (int a = 0; a < d; a++) k |= (uint64_t)(uint32_t)c[a] << (a * bits);
    return k;
  }
};

int32_t cell_of(double x, int l) {
  const int64_t n = (int64_t)1 << l;
  int64_t k = (int64_t)std::floor((x + 0.5) * (double)n);
  if (k < 0) k = 0;
  if (k >= n) k = n - 1;
  return (int32_t)k;
}

uint64_t interleave(const int32_t* c, int d) {
  uint64_t m = 0;
  for (int b = 0; b < 21; b++)
    for (int a = 0; a < d; a++) m |= (((uint64_t)(uint32_t)c[a] >> b) & 1ull) << (b * d + a);
  return m;
}

// Largest error of the degree p-1 Lagrange interpolant at the Gauss-Legendre
// nodes of exp(i theta t) over t in [-1, 1] (sampled on a fine grid).
double interp_error(int p, double theta, const std::vector<double>& eta, const std::vector<double>& lam) {
  double worst = 0;
  const int m = 401;
  for (int s = 0; s < m; s++) {
    const double t = -1.0 + 2.0 * s / (m - 1);
    std::complex<double> num = 0;
    double den = 0;
    int hit = -1;
    for (int k = 0; k < p; k++) {
      if (t == eta[k]) { hit = k; break; }
      const double c = lam[k] / (t - eta[k]);
      num += c * std::exp(std::complex<double>(0.0, theta * eta[k]));
      den += c;
    }
    const std::complex<double> v = hit >= 0 ? std::exp(std::complex<double>(0.0, theta * eta[hit])) : num / den;
    worst = std::max(worst, std::abs(v - std::exp(std::complex<double>(0.0, theta * t))));
  }
  return worst;
}

}  // namespace

void gl_barycentric(int p, std::vector<double>& eta, std::vector<double>& lam) {
  std::vector<double> w(p);
  eta.assign(p, 0.0);
  lam.assign(p, 0.0);
  gauss_legendre(p, eta.data(), w.data());
  // lambda_k proportional to (-1)^k sqrt((1 - eta_k^2) w_k) for Gauss-Legendre nodes
  for (int k = 0; k < p; k++) lam[k] = ((k & 1) ? -1.0 : 1.0) * std::sqrt((1.0 - eta[k] * eta[k]) * w[k]);
}

int build_point_plan(int d, int64_t nsrc, const double* src, int64_t ntgt, const double* tgt,
                     double delta, double tol, int p, int ns, PointHost& ph, std::string& err) {
  if (d != 2 && d != 3) { err = "dim must be 2 or 3"; return FGT_ERR_INVALID_ARG; }
  if (nsrc < 0 || ntgt < 0 || (nsrc > 0 && !src) || (ntgt > 0 && !tgt)) {
    err = "point arrays";
    return FGT_ERR_INVALID_ARG;
  }
  if (nsrc >= ((int64_t)1 << 31) || ntgt >= ((int64_t)1 << 31)) { err = "at most 2^31 - 1 points"; return FGT_ERR_UNSUPPORTED; }
  if (p < 4 || p > kMaxP) { err = "p must be in [4, 16]"; return FGT_ERR_INVALID_ARG; }
  if (ns < 1) { err = "n_s must be >= 1"; return FGT_ERR_INVALID_ARG; }
  if (!(delta > 0) || !std::isfinite(delta)) { err = "delta must be > 0"; return FGT_ERR_INVALID_ARG; }
  if (!(tol >= 1e-12 && tol < 0.1)) { err = "tol must be in [1e-12, 0.1)"; return FGT_ERR_INVALID_ARG; }
  for (int64_t i = 0; i < nsrc * d; i++)
    if (!(std::fabs(src[i]) <= 0.5)) { err = "a source lies outside [-1/2, 1/2]^d"; return FGT_ERR_INVALID_ARG; }
  for (int64_t i = 0; i < ntgt * d; i++)
    if (!(std::fabs(tgt[i]) <= 0.5)) { err = "a target lies outside [-1/2, 1/2]^d"; return FGT_ERR_INVALID_ARG; }

  ph = PointHost();
  ph.d = d; ph.p = p; ph.ns = ns; ph.delta = delta; ph.tol = tol; ph.nsrc = nsrc; ph.ntgt = ntgt;
  HostPlan& hp = ph.hp;
  hp.d = d; hp.p = p; hp.bc = FGT_FREE; hp.precision = FGT_FP64; hp.delta = delta; hp.tol = tol;
  hp.sqrt_delta = std::sqrt(delta);
  hp.point_tables = true;

  // ---- cutoff level and plane waves (Theorem 1), as for the box transform
  const double D0 = std::sqrt(std::log(3.0 / tol));
  const double cut = D0 * hp.sqrt_delta;
  int lc = cut >= 1.0 ? 0 : (int)std::floor(std::log2(1.0 / cut));
  while (lc > 0 && std::ldexp(1.0, -lc) < cut) lc--;
  while (std::ldexp(1.0, -(lc + 1)) >= cut) lc++;
  const int maxlev = d == 3 ? 14 : 20;
  if (lc > maxlev - 4) { err = "delta too small for this build (cutoff level too fine)"; return FGT_ERR_UNSUPPORTED; }
  hp.lc = lc;
  hp.Llc = std::ldexp(1.0, -lc);
  double R = (lc == 0 ? 1.0 : 2.0 * hp.Llc) / hp.sqrt_delta;
  if (R < D0) R = D0;
  hp.pw = pw_params(tol, R);
  hp.nr = 2 * hp.pw.M - 1;
  hp.nrs = 2 * hp.pw.M;
  if (hp.nrs > kMaxModes) { err = "too many plane-wave modes for this build (2M > 128)"; return FGT_ERR_UNSUPPORTED; }
  ph.lc = lc;

  // ---- proxy level: p nodes interpolate every plane wave on a proxy box
  std::vector<double> eta, lam;
  gl_barycentric(p, eta, lam);
  const double kmax = (hp.pw.M - 1) * hp.pw.h / hp.sqrt_delta;
  int s = 0;
  for (;; s++) {
    if (lc + s > maxlev) { err = "p too small for tol: the proxy boxes would be too fine"; return FGT_ERR_UNSUPPORTED; }
    const double theta = kmax * std::ldexp(hp.Llc, -s) * 0.5;
    ph.proxy_err = interp_error(p, theta, eta, lam);
    if (ph.proxy_err <= tol / (10.0 * d)) break;
  }
  ph.lp = lc + s;
  const int lp = ph.lp;

  // ---- Algorithm 1: split boxes with more than ns sources or targets, down to lc
  BoxKey key(d);
  std::vector<int32_t> sc((size_t)nsrc * d), tc((size_t)ntgt * d);  // cells at level lp
  for (int64_t i = 0; i < nsrc * d; i++) sc[i] = cell_of(src[i], lp);
  for (int64_t i = 0; i < ntgt * d; i++) tc[i] = cell_of(tgt[i], lp);
  LeafTree t0;
  t0.d = d;
  {
    std::unordered_map<uint64_t, std::pair<int64_t, int64_t>> cnt;
    std::vector<std::array<int32_t, 3>> active{{0, 0, 0}};
    for (int l = 0; l <= lc; l++) {
      cnt.clear();
      int32_t c[3] = {0, 0, 0};
      for (int64_t i = 0; i < nsrc; i++) {
        for (int a = 0; a < d; a++) c[a] = sc[i * d + a] >> (lp - l);
        cnt[key(l, c)].first++;
      }
      for (int64_t i = 0; i < ntgt; i++) {
        for (int a = 0; a < d; a++) c[a] = tc[i * d + a] >> (lp - l);
        cnt[key(l, c)].second++;
      }
      std::vector<std::array<int32_t, 3>> next;
      for (const auto& b : active) {
        auto it = cnt.find(key(l, b.data()));
        const bool split = l < lc && it != cnt.end() && (it->second.first > ns || it->second.second > ns);
        if (!split) {
          t0.level.push_back(l);
          for (int a = 0; a < d; a++) t0.coord.push_back(b[a]);
          continue;
        }
        for (int o = 0; o < (1 << d); o++) {
          std::array<int32_t, 3> ch{0, 0, 0};
          for (int a = 0; a < d; a++) ch[a] = 2 * b[a] + ((o >> a) & 1);
          next.push_back(ch);
        }
      }
      active.swap(next);
    }
  }
  // level restriction, then no coarse neighbor for a dense leaf at lc
  LeafTree t1, t2;
  std::vector<int32_t> srcmap;
  int64_t nsplit = 0, nbal = 0;
  split_and_balance(t0, {}, false, t1, srcmap, &nsplit, &nbal);
  auto leaf_index = [&](const LeafTree& t) {
    std::unordered_map<uint64_t, int32_t> m;
    m.reserve((size_t)t.size() * 2);
    for (int64_t i = 0; i < t.size(); i++) m[key(t.level[i], &t.coord[i * d])] = (int32_t)i;
    return m;
  };
  auto locate = [&](const std::unordered_map<uint64_t, int32_t>& m, const int32_t* cell_lp) -> int32_t {
    int32_t c[3] = {0, 0, 0};
    for (int l = lc; l >= 0; l--) {
      for (int a = 0; a < d; a++) c[a] = cell_lp[a] >> (lp - l);
      auto it = m.find(key(l, c));
      if (it != m.end()) return it->second;
    }
    return -1;
  };
  auto dense_flags = [&](const LeafTree& t, const std::unordered_map<uint64_t, int32_t>& m) {
    std::vector<int64_t> cs(t.size(), 0), ct(t.size(), 0);
    for (int64_t i = 0; i < nsrc; i++) cs[locate(m, &sc[i * d])]++;
    for (int64_t i = 0; i < ntgt; i++) ct[locate(m, &tc[i * d])]++;
    std::vector<int32_t> f(t.size(), 0);
    for (int64_t i = 0; i < t.size(); i++) f[i] = t.level[i] == lc && (cs[i] > ns || ct[i] > ns);
    return f;
  };
  const int n3 = d == 2 ? 9 : 27;
  auto dir_of = [&](int code, int* dir) {
    for (int a = 0; a < d; a++) { dir[a] = code % 3 - 1; code /= 3; }
  };
  {
    auto m1 = leaf_index(t1);
    std::vector<int32_t> f1 = dense_flags(t1, m1);
    std::vector<uint8_t> split(t1.size(), 0);
    const int64_t nb = (int64_t)1 << lc;
    for (int64_t i = 0; i < t1.size(); i++) {
      if (!f1[i]) continue;
      for (int code = 0; code < n3; code++) {
        int dir[3];
        dir_of(code, dir);
        int32_t q[3] = {0, 0, 0};
        bool inside = true;
        for (int a = 0; a < d; a++) {
          const int64_t v = (int64_t)t1.coord[i * d + a] + dir[a];
          if (v < 0 || v >= nb) inside = false;
          q[a] = (int32_t)v;
        }
        if (!inside || lc == 0) continue;
        int32_t par[3] = {0, 0, 0};
        for (int a = 0; a < d; a++) par[a] = q[a] >> 1;
        auto it = m1.find(key(lc - 1, par));
        if (it != m1.end()) split[it->second] = 1;
      }
    }
    split_and_balance(t1, split, false, t2, srcmap, &nsplit, &nbal);
  }
  const int64_t nleaf = t2.size();
  auto m2 = leaf_index(t2);
  ph.leaf_level = t2.level;
  ph.leaf_coord = t2.coord;
  ph.leaf_dense = dense_flags(t2, m2);

  // ---- points by leaf; the plane-wave boxes and their colleagues
  std::vector<int32_t> sleaf(nsrc), tleaf(ntgt);
  std::vector<int64_t> lsrc(nleaf, 0), ltgt(nleaf, 0);
  for (int64_t i = 0; i < nsrc; i++) lsrc[sleaf[i] = locate(m2, &sc[i * d])]++;
  for (int64_t i = 0; i < ntgt; i++) ltgt[tleaf[i] = locate(m2, &tc[i * d])]++;
  auto colleague = [&](int64_t i, int code, int32_t* q) -> int32_t {  // leaf at the same level, or -1
    int dir[3];
    dir_of(code, dir);
    const int l = t2.level[i];
    const int64_t nb = (int64_t)1 << l;
    for (int a = 0; a < d; a++) {
      const int64_t v = (int64_t)t2.coord[i * d + a] + dir[a];
      if (v < 0 || v >= nb) return -1;
      q[a] = (int32_t)v;
    }
    auto it = m2.find(key(l, q));
    return it == m2.end() ? -1 : it->second;
  };
  std::vector<int32_t> pwidx(nleaf, -1);
  std::vector<int32_t> pwbox;  // leaf of each plane-wave box (Morton order: leaves are)
  for (int64_t i = 0; i < nleaf; i++) {
    if (t2.level[i] != lc) continue;
    bool pw = ph.leaf_dense[i] != 0;
    if (!pw && ltgt[i] > 0) {
      for (int code = 0; code < n3 && !pw; code++) {
        int32_t q[3];
        const int32_t j = colleague(i, code, q);
        pw = j >= 0 && ph.leaf_dense[j];
      }
    }
    if (pw) {
      pwidx[i] = (int32_t)pwbox.size();
      pwbox.push_back((int32_t)i);
    }
  }
  const int32_t nA = (int32_t)pwbox.size();
  ph.n_pwbox = nA;
  for (int64_t i = 0; i < nleaf; i++) ph.n_dense += ph.leaf_dense[i];

  // ---- sort the points by (leaf, proxy box), leaves in Morton order
  auto sort_points = [&](int64_t n, const std::vector<int32_t>& cell, const std::vector<int32_t>& leaf,
                         const double* xyz, std::vector<int32_t>& perm, std::vector<double>& sorted) {
    std::vector<std::pair<uint64_t, int32_t>> k((size_t)n);
    for (int64_t i = 0; i < n; i++) {
      const int32_t L = leaf[i];
      uint64_t sub = 0;
      if (pwidx[L] >= 0) {
        int32_t rel[3] = {0, 0, 0};
        for (int a = 0; a < d; a++) rel[a] = cell[i * d + a] - (t2.coord[(int64_t)L * d + a] << (lp - lc));
        sub = interleave(rel, d);
      }
      k[i] = {((uint64_t)L << 40) | sub, (int32_t)i};
    }
    std::stable_sort(k.begin(), k.end());
    perm.resize(n);
    sorted.resize((size_t)n * d);
    for (int64_t s2 = 0; s2 < n; s2++) {
      perm[s2] = k[s2].second;
      for (int a = 0; a < d; a++) sorted[s2 * d + a] = xyz[(int64_t)k[s2].second * d + a];
    }
  };
  if (lp - lc > 13) { err = "internal: proxy level too deep"; return FGT_ERR_UNSUPPORTED; }
  sort_points(nsrc, sc, sleaf, src, ph.src_perm, ph.src_xyz);
  sort_points(ntgt, tc, tleaf, tgt, ph.tgt_perm, ph.tgt_xyz);
  ph.leaf_src_start.assign(nleaf + 1, 0);
  ph.leaf_tgt_start.assign(nleaf + 1, 0);
  for (int64_t i = 0; i < nleaf; i++) {
    ph.leaf_src_start[i + 1] = ph.leaf_src_start[i] + (int32_t)lsrc[i];
    ph.leaf_tgt_start[i + 1] = ph.leaf_tgt_start[i] + (int32_t)ltgt[i];
  }

  // ---- proxy boxes: in each plane-wave box, the level-lp boxes holding its
  // sources (dense boxes only: a sparse box's sources go direct) or targets
  std::vector<PwLeafRef> pl;
  for (int32_t a = 0; a < nA; a++) {
    const int32_t L = pwbox[a];
    const bool dense = ph.leaf_dense[L] != 0;
    // distinct proxy boxes in this leaf, from both sorted point lists
    std::vector<std::pair<uint64_t, std::array<int32_t, 3>>> subs;
    auto collect = [&](int32_t s0, int32_t s1, const std::vector<int32_t>& perm, const std::vector<int32_t>& cell) {
      for (int32_t s2 = s0; s2 < s1; s2++) {
        std::array<int32_t, 3> c{0, 0, 0}, rel{0, 0, 0};
        for (int b = 0; b < d; b++) {
          c[b] = cell[(int64_t)perm[s2] * d + b];
          rel[b] = c[b] - (t2.coord[(int64_t)L * d + b] << (lp - lc));
        }
        const uint64_t k = interleave(rel.data(), d);
        if (subs.empty() || subs.back().first != k) subs.push_back({k, c});
      }
    };
    if (dense) collect(ph.leaf_src_start[L], ph.leaf_src_start[L + 1], ph.src_perm, sc);
    collect(ph.leaf_tgt_start[L], ph.leaf_tgt_start[L + 1], ph.tgt_perm, tc);
    std::sort(subs.begin(), subs.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    subs.erase(std::unique(subs.begin(), subs.end(), [](const auto& x, const auto& y) { return x.first == y.first; }),
               subs.end());
    for (const auto& sb : subs) {
      const int32_t id = (int32_t)ph.px_level.size();
      ph.px_level.push_back(lp);
      for (int b = 0; b < d; b++) ph.px_coord.push_back(sb.second[b]);
      const int sh = lp - lc;
      auto rel = [&](int b) { return (uint64_t)(sb.second[b] - ((sb.second[b] >> sh) << sh)); };
      const uint64_t m = d == 3 ? ((rel(2) << 42) | (rel(0) << 21) | rel(1)) : ((rel(1) << 21) | rel(0));
      pl.push_back({a, m, id, d == 3 ? lp : 0});
    }
  }
  const int64_t npx = (int64_t)ph.px_level.size();
  // point ranges of every proxy box (points of a leaf are sorted by proxy box)
  ph.px_src_start.assign(npx + 1, 0);
  ph.px_tgt_start.assign(npx + 1, 0);
  {
    std::unordered_map<uint64_t, int32_t> pxmap;
    for (int64_t i = 0; i < npx; i++) pxmap[key(lp, &ph.px_coord[i * d])] = (int32_t)i;
    std::vector<int32_t> c0(npx, 0), c1(npx, 0), t0v(npx, 0), t1v(npx, 0);
    std::vector<uint8_t> sseen(npx, 0), tseen(npx, 0);
    for (int64_t s2 = 0; s2 < nsrc; s2++) {
      const int32_t L = sleaf[ph.src_perm[s2]];
      if (pwidx[L] < 0 || !ph.leaf_dense[L]) continue;
      const int32_t x = pxmap.at(key(lp, &sc[(int64_t)ph.src_perm[s2] * d]));
      if (!sseen[x]) { sseen[x] = 1; c0[x] = (int32_t)s2; }
      c1[x] = (int32_t)s2 + 1;
    }
    for (int64_t s2 = 0; s2 < ntgt; s2++) {
      const int32_t L = tleaf[ph.tgt_perm[s2]];
      if (pwidx[L] < 0) continue;
      const int32_t x = pxmap.at(key(lp, &tc[(int64_t)ph.tgt_perm[s2] * d]));
      if (!tseen[x]) { tseen[x] = 1; t0v[x] = (int32_t)s2; }
      t1v[x] = (int32_t)s2 + 1;
    }
    // stored as [start, end) pairs packed into start arrays of 2 npx entries
    ph.px_src_start.assign(2 * npx, 0);
    ph.px_tgt_start.assign(2 * npx, 0);
    for (int64_t i = 0; i < npx; i++) {
      ph.px_src_start[2 * i] = c0[i];
      ph.px_src_start[2 * i + 1] = c1[i];
      ph.px_tgt_start[2 * i] = t0v[i];
      ph.px_tgt_start[2 * i + 1] = t1v[i];
      if (t1v[i] > t0v[i]) ph.px_tgt_list.push_back((int32_t)i);
    }
  }

  // ---- the box transform's plane-wave lists over the proxy boxes
  hp.nleaves = npx;
  hp.level = ph.px_level;
  hp.coord = ph.px_coord;
  hp.lmin = hp.lmax = lp;
  hp.pwbox_isleaf.assign(nA, 0);
  finish_pw_lists(hp, pl, nA, ph.px_level.data(), ph.px_coord.data(), true);
  // P-lists: the dense colleagues of every plane-wave box, itself included
  // (each list sorted by source box, then code: see build_te_groups)
  hp.plist_start.assign(nA + 1, 0);
  for (int32_t a = 0; a < nA; a++) {
    std::vector<std::pair<int32_t, int32_t>> ents;
    for (int code = 0; code < n3; code++) {
      int32_t q[3];
      const int32_t j = colleague(pwbox[a], code, q);
      if (j < 0 || !ph.leaf_dense[j]) continue;
      ents.push_back({pwidx[j], code});  // dir = source - target per axis
    }
    std::sort(ents.begin(), ents.end());
    for (auto& e : ents) {
      hp.plist_src.push_back(e.first);
      hp.plist_dir.push_back(e.second);
    }
    hp.plist_start[a + 1] = (int32_t)hp.plist_src.size();
  }
  if (d == 3 && hp.fuse_te) {
    std::vector<int32_t> bc((size_t)nA * 3);
    for (int32_t a = 0; a < nA; a++)
      for (int ax = 0; ax < 3; ax++) bc[(size_t)a * 3 + ax] = t2.coord[(size_t)pwbox[a] * 3 + ax];
    build_te_groups(hp, bc);
  }
  hp.nvtab = 0;
  build_tables(hp);

  // ---- direct part: every leaf with targets gathers from the leaves of its
  // neighbor list that hold sources, except (at lc) its dense colleagues
  for (int64_t T = 0; T < nleaf; T++) {
    if (ltgt[T] == 0) continue;
    const int l = t2.level[T];
    const int64_t nb = (int64_t)1 << l;
    std::vector<int32_t> ents;
    for (int code = 0; code < n3; code++) {
      int dir[3];
      dir_of(code, dir);
      int32_t q[3] = {0, 0, 0};
      bool inside = true;
      for (int a = 0; a < d; a++) {
        const int64_t v = (int64_t)t2.coord[T * d + a] + dir[a];
        if (v < 0 || v >= nb) inside = false;
        q[a] = (int32_t)v;
      }
      if (!inside) continue;
      auto it = m2.find(key(l, q));
      if (it != m2.end()) { ents.push_back(it->second); continue; }
      if (l >= 1) {
        int32_t par[3] = {0, 0, 0};
        for (int a = 0; a < d; a++) par[a] = q[a] >> 1;
        auto ip = m2.find(key(l - 1, par));
        if (ip != m2.end()) { ents.push_back(ip->second); continue; }
      }
      // finer leaves: children of the neighbor box that touch T
      for (int o = 0; o < (1 << d); o++) {
        int32_t ch[3] = {0, 0, 0};
        bool ok = true;
        for (int a = 0; a < d; a++) {
          const int bit = (o >> a) & 1;
          if ((dir[a] == -1 && bit == 0) || (dir[a] == 1 && bit == 1)) ok = false;
          ch[a] = 2 * q[a] + bit;
        }
        if (!ok) continue;
        auto ic = m2.find(key(l + 1, ch));
        if (ic != m2.end()) ents.push_back(ic->second);
      }
    }
    std::sort(ents.begin(), ents.end());
    ents.erase(std::unique(ents.begin(), ents.end()), ents.end());
    int64_t terms = 0;
    const size_t before = ph.dl_src.size();
    for (int32_t S : ents) {
      if (lsrc[S] == 0) continue;
      if (l == lc && t2.level[S] == lc && ph.leaf_dense[S]) continue;  // by plane waves
      ph.dl_src.push_back(S);
      terms += lsrc[S];
    }
    ph.dl_tgt.push_back((int32_t)T);
    ph.dl_haspw.push_back(pwidx[T] >= 0 ? 1 : 0);
    ph.dl_start.push_back((int32_t)before);
    ph.n_direct_terms += terms * ltgt[T];
  }
  ph.dl_start.push_back((int32_t)ph.dl_src.size());
  constexpr int32_t kChunk = 256;  // threads per workgroup of the device kernels
  constexpr int32_t kAnterpPart = 1024;
  for (int64_t x = 0; x < npx; x++) {
    const int32_t a0 = ph.px_src_start[2 * x], a1 = ph.px_src_start[2 * x + 1];
    const int32_t parts = std::max<int32_t>(1, (a1 - a0 + kAnterpPart - 1) / kAnterpPart);
    if (parts == 1) {
      ph.anterp_items.insert(ph.anterp_items.end(), {(int32_t)x, a0, a1, -1});
      continue;
    }
    const int32_t slot0 = (int32_t)ph.n_anterp_slots;
    for (int32_t i = 0; i < parts; i++)
      ph.anterp_items.insert(ph.anterp_items.end(),
                             {(int32_t)x, a0 + i * kAnterpPart, std::min(a1, a0 + (i + 1) * kAnterpPart),
                              slot0 + i});
    ph.reduce_items.insert(ph.reduce_items.end(), {(int32_t)x, slot0, parts});
    ph.n_anterp_slots += parts;
  }
  for (int32_t x : ph.px_tgt_list)
    for (int32_t tb = ph.px_tgt_start[2 * x]; tb < ph.px_tgt_start[2 * x + 1]; tb += kChunk)
      ph.interp_items.insert(ph.interp_items.end(), {x, tb});
  for (size_t k = 0; k < ph.dl_tgt.size(); k++) {
    const int32_t T = ph.dl_tgt[k];
    for (int32_t tb = ph.leaf_tgt_start[T]; tb < ph.leaf_tgt_start[T + 1]; tb += kChunk)
      ph.direct_items.insert(ph.direct_items.end(), {(int32_t)k, tb});
  }
  return FGT_OK;
}

}  // namespace fgt
