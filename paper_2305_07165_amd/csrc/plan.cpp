// Host plan of the box Gauss transform: tree validation, the cutoff level and
// plane-wave parameters (Theorem 1), and the flat lists that drive the device
// stages of Algorithm 4 (f-flags, P-lists, D-lists; Section 4.2).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "fgt_host.h"
#include "../../include/fgt.h"

namespace fgt {

int periodic_terms(double eps, double delta) {
  return (int)std::ceil(std::sqrt(std::log(1.0 / eps)) / (M_PI * std::sqrt(delta)));
}

PwParams pw_params(double eps, double R) {
  PwParams q;
  q.eps = eps;
  q.D0 = std::sqrt(std::log(3.0 / eps));
  q.R = R;
  q.h = 2.0 * M_PI / (R + q.D0);
  q.M = (int)std::ceil(q.D0 * (R + q.D0) / M_PI);
  return q;
}

namespace {

int max_level_for_dim(int d) { return d == 3 ? 19 : (d == 2 ? 28 : 30); }

// Unique 64-bit key of a box (level, coords).
struct KeyMaker {
  int d, bits;
  explicit KeyMaker(int dim) : d(dim), bits(58 / dim) {}
  uint64_t operator()(int l, const int32_t* c) const {
    uint64_t k = (uint64_t)l << 58;
    for (int a = 0; a < d; a++) k |= (uint64_t)(uint32_t)c[a] << (a * bits);
    return k;
  }
};

uint64_t morton(const int32_t* c, int d, int shift) {
  // interleave the bits of coords scaled by 2^shift (up to 21 bits per axis)
  uint64_t m = 0;
  uint64_t v[3] = {0, 0, 0};
  for (int a = 0; a < d; a++) v[a] = (uint64_t)(uint32_t)c[a] << shift;
  for (int b = 0; b < 21; b++)
    for (int a = 0; a < d; a++) m |= ((v[a] >> b) & 1ull) << (b * d + a);
  return m;
}

int ipow3(int d) { return d == 1 ? 3 : (d == 2 ? 9 : 27); }

void dir_of(int code, int d, int* dir) {
  for (int a = 0; a < d; a++) {
    dir[a] = code % 3 - 1;
    code /= 3;
  }
}

}  // namespace

// Orders the plane-wave leaves by (box, level, key) and fills the lists the
// box-level stages run over: pw_start, pwleaf_id/tab/box, the form/eval table
// ids (one table per level and position along an axis inside the cutoff box),
// for d = 3 the planes and rows, the fused-translation choice, the dispatch
// order of boxes, the formation items and the evaluation chunks.
void finish_pw_lists(HostPlan& hp, std::vector<PwLeafRef>& pl, int32_t nA, const int32_t* level,
                     const int32_t* coord, bool allow_fuse) {
  const int d = hp.d, p = hp.p, lc = hp.lc;
  std::sort(pl.begin(), pl.end(), [](const PwLeafRef& x, const PwLeafRef& y) {
    if (x.box != y.box) return x.box < y.box;
    if (x.lv != y.lv) return x.lv < y.lv;
    return x.m < y.m;
  });
  std::unordered_map<uint64_t, int32_t> ftab;  // (level, pos) -> id
  std::vector<int32_t> ftab_lv, ftab_pos;
  hp.pw_start.assign(nA + 1, 0);
  hp.pwleaf_id.resize(pl.size());
  hp.pwleaf_tab.resize(pl.size() * d);
  hp.pwleaf_box.resize(pl.size());
  for (size_t s = 0; s < pl.size(); s++) {
    int32_t i = pl[s].id;
    int l = level[i];
    hp.pwleaf_id[s] = i;
    hp.pwleaf_box[s] = pl[s].box;
    hp.pw_start[pl[s].box + 1]++;
    for (int a = 0; a < d; a++) {
      int32_t pos = coord[i * d + a] - ((coord[i * d + a] >> (l - lc)) << (l - lc));
      uint64_t k = ((uint64_t)l << 32) | (uint32_t)pos;
      auto it = ftab.find(k);
      int32_t id;
      if (it == ftab.end()) {
        id = (int32_t)ftab_lv.size();
        ftab.emplace(k, id);
        ftab_lv.push_back(l);
        ftab_pos.push_back(pos);
      } else {
        id = it->second;
      }
      hp.pwleaf_tab[s * d + a] = id;
    }
  }
  for (int32_t a = 0; a < nA; a++) hp.pw_start[a + 1] += hp.pw_start[a];
  hp.nftab = (int)ftab_lv.size();
  hp.ftab_meta = ftab_lv;
  hp.ftab_meta.insert(hp.ftab_meta.end(), ftab_pos.begin(), ftab_pos.end());

  // d = 3 planes and rows (see the leaf order above)
  if (d == 3) {
    hp.plane_start.assign(nA + 1, 0);
    for (int32_t a = 0; a < nA; a++) {
      for (int32_t s = hp.pw_start[a]; s < hp.pw_start[a + 1]; s++) {
        const int32_t t3 = hp.pwleaf_tab[s * 3 + 2], t1 = hp.pwleaf_tab[s * 3 + 0];
        const bool new_plane = s == hp.pw_start[a] || hp.pwleaf_tab[(s - 1) * 3 + 2] != t3;
        const bool new_row = new_plane || hp.pwleaf_tab[(s - 1) * 3 + 0] != t1;
        if (new_plane) {
          hp.plane_row.push_back((int32_t)hp.row_tab.size());
          hp.plane_tab.insert(hp.plane_tab.end(), {0, 0, t3});
        }
        if (new_row) {
          hp.row_start.push_back(s);
          hp.row_tab.push_back(t1);
        }
      }
      hp.plane_start[a + 1] = (int32_t)hp.plane_row.size();
    }
    hp.plane_row.push_back((int32_t)hp.row_tab.size());
    hp.row_start.push_back((int32_t)pl.size());
    // planes dispatched longest first: leaves (one axis-2 product each) and
    // rows (three times the products each, the axis-1 step) of the plane
    const int32_t npl = (int32_t)hp.plane_row.size() - 1;
    std::vector<int32_t> work(npl);
    for (int32_t P = 0; P < npl; P++) {
      const int32_t r0 = hp.plane_row[P], r1 = hp.plane_row[P + 1];
      work[P] = (hp.row_start[r1] - hp.row_start[r0]) + 3 * (r1 - r0);
    }
    hp.plane_order.resize(npl);
    for (int32_t P = 0; P < npl; P++) hp.plane_order[P] = P;
    std::stable_sort(hp.plane_order.begin(), hp.plane_order.end(),
                     [&](int32_t x, int32_t y) { return work[x] > work[y]; });
  }
  if (d == 3) {
    // measured: the fused kernel wins while psi is large and n_r <= 64 (up to
    // four mode tiles); with wider tiles its tile shape reads phi less
    // contiguously than the plain translation and the pair of kernels is faster
    const double ts = hp.precision == FGT_FP64 ? 8.0 : 4.0;
    hp.fuse_te = allow_fuse && hp.nrs <= 64 && ts * nA * (double)hp.nrs * hp.nrs * hp.nrs > kFuseBytes;
  }
  // the units the box-level stages run over: planes for d = 3, leaves otherwise
  const std::vector<int32_t>& unit_start = d == 3 ? hp.plane_start : hp.pw_start;

  // dispatch order of per-box work: most units first (longest work first)
  hp.box_order.resize(nA);
  for (int32_t a = 0; a < nA; a++) hp.box_order[a] = a;
  std::stable_sort(hp.box_order.begin(), hp.box_order.end(), [&](int32_t x, int32_t y) {
    return unit_start[x + 1] - unit_start[x] > unit_start[y + 1] - unit_start[y];
  });

  // formation work items: at most kFormLeaves units each
  for (int32_t a = 0; a < nA; a++) {
    const int32_t s0 = unit_start[a], s1 = unit_start[a + 1];
    if (s1 - s0 <= kFormLeaves) {
      hp.fitem.insert(hp.fitem.end(), {a, s0, s1, -1});
      continue;
    }
    const int32_t first = hp.nslots;
    for (int32_t s = s0; s < s1; s += kFormLeaves)
      hp.fitem.insert(hp.fitem.end(), {a, s, std::min(s + kFormLeaves, s1), hp.nslots++});
    hp.fred.insert(hp.fred.end(), {a, first, hp.nslots - first});
  }

  {
    const size_t ni = hp.fitem.size() / 4;
    std::vector<int32_t> ord(ni);
    for (size_t i = 0; i < ni; i++) ord[i] = (int32_t)i;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
      return hp.fitem[4 * x + 2] - hp.fitem[4 * x + 1] > hp.fitem[4 * y + 2] - hp.fitem[4 * y + 1];
    });
    std::vector<int32_t> f2;
    f2.reserve(hp.fitem.size());
    for (int32_t i : ord) f2.insert(f2.end(), hp.fitem.begin() + 4 * i, hp.fitem.begin() + 4 * i + 4);
    hp.fitem.swap(f2);
  }

  // evaluation chunks: up to 64 stacked rows (count*p) of one box
  const int per = std::max(1, 64 / p);
  for (int32_t a = 0; a < nA; a++)
    for (int32_t s = hp.pw_start[a]; s < hp.pw_start[a + 1]; s += per) {
      hp.echunk.push_back(a);
      hp.echunk.push_back(s);
      hp.echunk.push_back(std::min(per, hp.pw_start[a + 1] - s));
    }

}

// Fused-translation target groups: the plane-wave boxes that share a parent at
// level lc - 1 and their position along axis 3 (at most four, contiguous in
// Morton order).  The entries of a group are the distinct (source box, rank)
// pairs of its members' P-lists, rank counting repeats of one source in one
// list (a box that is its own neighbor through two periodic images), sorted by
// source box then rank.  Since every P-list is sorted by (source box, code), a
// member meets its sources in its own list's order, so its sum is formed in
// the same order as on its own.
void build_te_groups(HostPlan& hp, const std::vector<int32_t>& box_coord) {
  hp.te_start.assign(1, 0);
  hp.te_mem.clear();
  hp.te_src.clear();
  hp.te_dir.clear();
  hp.te_wg.clear();
  const int32_t nA = (int32_t)hp.n_pwbox();
  std::unordered_map<uint64_t, int32_t> gmap;
  std::vector<std::vector<int32_t>> groups;
  for (int32_t a = 0; a < nA; a++) {
    const int32_t* c = &box_coord[(size_t)a * 3];
    const uint64_t k = ((uint64_t)(uint32_t)(c[0] >> 1) << 42) | ((uint64_t)(uint32_t)(c[1] >> 1) << 21) |
                       (uint64_t)(uint32_t)c[2];
    auto it = gmap.find(k);
    if (it == gmap.end()) {
      gmap.emplace(k, (int32_t)groups.size());
      groups.push_back({a});
    } else {
      groups[it->second].push_back(a);
    }
  }
  struct Ent {
    int32_t src, rank, d3;
    uint8_t dir[kTeGroup];
  };
  // the entries of a member set, sorted.  An entry also keys on the axis-3
  // part of the code, so that its members share it (the kernel rotates the
  // source along axis 3 once per entry); members at one axis-3 position meet
  // a source box at one axis-3 offset anyway, so this splits nothing unless a
  // box repeats in a list
  auto entries_of = [&](const std::vector<int32_t>& mem) {
    std::vector<Ent> ents;
    std::unordered_map<uint64_t, size_t> at;  // (src, rank, d3) -> entry
    for (size_t t = 0; t < mem.size(); t++) {
      const int32_t A = mem[t];
      int32_t prev = -1, rank = 0;
      for (int32_t q = hp.plist_start[A]; q < hp.plist_start[A + 1]; q++) {
        const int32_t B = hp.plist_src[q];
        rank = B == prev ? rank + 1 : 0;
        prev = B;
        const int32_t d3 = hp.plist_dir[q] / 9;
        const uint64_t k = ((uint64_t)(uint32_t)B << 32) | ((uint64_t)(uint32_t)rank << 2) | (uint32_t)d3;
        auto it = at.find(k);
        size_t e;
        if (it == at.end()) {
          e = ents.size();
          at.emplace(k, e);
          Ent n{B, rank, d3, {}};
          for (int s = 0; s < kTeGroup; s++) n.dir[s] = (uint8_t)kTeNoDir;
          ents.push_back(n);
        } else {
          e = it->second;
        }
        ents[e].dir[t] = (uint8_t)hp.plist_dir[q];
      }
    }
    std::sort(ents.begin(), ents.end(), [](const Ent& x, const Ent& y) {
      return x.src != y.src ? x.src < y.src : (x.rank != y.rank ? x.rank < y.rank : x.d3 < y.d3);
    });
    return ents;
  };
  const int32_t ng = (int32_t)groups.size();
  std::vector<double> work(ng);
  for (int32_t g = 0; g < ng; g++) {
    const auto& mem = groups[g];
    const std::vector<Ent> ents = entries_of(mem);
    for (const Ent& e : ents) {
      hp.te_src.push_back(e.src);
      for (int w = 0; w < (kTeGroup + 3) / 4; w++) {  // as many words as the kernel reads
        uint32_t word = 0;
        for (int b = 0; b < 4; b++)
          word |= (uint32_t)(4 * w + b < kTeGroup ? e.dir[4 * w + b] : (uint8_t)kTeNoDir) << (8 * b);
        hp.te_dir.push_back((int32_t)word);
      }
    }
    for (int s = 0; s < kTeGroup; s++) hp.te_mem.push_back(s < (int)mem.size() ? mem[s] : -1);
    hp.te_start.push_back((int32_t)hp.te_src.size());
    // workgroup cost model (units of one source rotation of a tile): one load
    // per entry, the rotations, and the plane contractions
    double w = (double)ents.size();
    for (int32_t A : mem)
      w += (hp.plist_start[A + 1] - hp.plist_start[A]) + 4.0 * (hp.plane_start[A + 1] - hp.plane_start[A]);
    work[g] = w;
  }

  // tiles: a multiple of 4 pairs (16 columns) with M pairs * M units <= 256
  // threads, at most all M^2 pairs
  const int M = hp.pw.M;
  hp.te_tp = std::min(std::max(1, 4 * (256 / (4 * M))), M * M);
  const int ntile = (M * M + hp.te_tp - 1) / hp.te_tp;
  // Workgroup order.  Tile t of every group runs on XCD t % 8, so that a
  // source tile is read into one L2, and each XCD sweeps its tiles one after
  // the other with the groups in Morton order, so that the groups resident
  // at one time share most of their sources in that L2.  The tiles past the
  // last multiple of 8 are one such sweep cut into eight runs of equal work,
  // one per XCD.  The last kTeTail workgroups of every XCD run longest first,
  // so that no long group starts late.
  auto spread = [](uint32_t v) {  // bit i of v to bit 3 i
    uint64_t r = 0;
    for (int i = 0; i < 21; i++) r |= (uint64_t)((v >> i) & 1u) << (3 * i);
    return r;
  };
  std::vector<uint64_t> mkey(ng);
  for (int32_t g = 0; g < ng; g++) {
    const int32_t* c = &box_coord[(size_t)groups[g][0] * 3];
    mkey[g] = spread((uint32_t)(c[0] >> 1)) | spread((uint32_t)(c[1] >> 1)) << 1 | spread((uint32_t)c[2]) << 2;
  }
  std::vector<int32_t> order(ng);
  for (int32_t g = 0; g < ng; g++) order[g] = g;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return mkey[x] < mkey[y]; });
  const int fixed = ntile / kXcdCount * kXcdCount;
  std::vector<std::vector<std::pair<int32_t, int32_t>>> q(kXcdCount);
  for (int t = 0; t < fixed; t++)
    for (int32_t g : order) q[t % kXcdCount].push_back({g, t});
  double rest = 0;
  for (int t = fixed; t < ntile; t++)
    for (int32_t g : order) rest += work[g];
  double done = 0;
  for (int t = fixed; t < ntile; t++)
    for (int32_t g : order) {
      const int x = std::min(kXcdCount - 1, (int)(kXcdCount * (done + 0.5 * work[g]) / rest));
      q[x].push_back({g, t});
      done += work[g];
    }
  for (auto& v : q) {
    const size_t k0 = v.size() > (size_t)kTeTail ? v.size() - kTeTail : 0;
    std::stable_sort(v.begin() + k0, v.end(), [&](const std::pair<int32_t, int32_t>& x,
                                                  const std::pair<int32_t, int32_t>& y) {
      return work[x.first] > work[y.first];
    });
  }
  size_t len = 0;
  for (auto& v : q) len = std::max(len, v.size());
  hp.te_wg.assign(2 * len * kXcdCount, -1);
  for (int x = 0; x < kXcdCount; x++)
    for (size_t k = 0; k < q[x].size(); k++) {
      hp.te_wg[2 * (k * kXcdCount + x)] = q[x][k].first;
      hp.te_wg[2 * (k * kXcdCount + x) + 1] = q[x][k].second;
    }
}

int build_host_plan(int d, int64_t n, const int32_t* level, const int32_t* coord, int p,
                    double delta, double tol, int bc, int precision, double eps_internal,
                    int force_lc, bool allow_fuse, HostPlan& hp, std::string& err) {
  if (d < 1 || d > kMaxDim) { err = "dim must be 1, 2 or 3"; return FGT_ERR_INVALID_ARG; }
  if (n < 1 || !level || !coord) { err = "empty tree"; return FGT_ERR_INVALID_ARG; }
  if (p < 1 || p > kMaxP) { err = "p must be in [1,16]"; return FGT_ERR_INVALID_ARG; }
  if (!(delta > 0) || !std::isfinite(delta)) { err = "delta must be > 0"; return FGT_ERR_INVALID_ARG; }
  if (!(tol > 0 && tol < 0.1)) { err = "tol must be in (0, 0.1) (Theorem 1 needs eps < 0.1)"; return FGT_ERR_INVALID_ARG; }
  if (bc != FGT_FREE && bc != FGT_PERIODIC) { err = "bc must be FGT_FREE or FGT_PERIODIC"; return FGT_ERR_INVALID_ARG; }
  if (precision != FGT_FP64 && precision != FGT_FP32 && precision != FGT_BF16X3) {
    err = "precision must be FGT_FP64, FGT_FP32 or FGT_BF16X3";
    return FGT_ERR_INVALID_ARG;
  }
  if (precision == FGT_BF16X3 && d == 1) { err = "FGT_BF16X3 needs d = 2 or 3"; return FGT_ERR_UNSUPPORTED; }
  // reduced precision is offered only where its rounding stays below tol
  // (measured against the FP64 oracle over whole trees): FP32 products and
  // expansions add a relative l2 error of about 2e-7, split bf16 products
  // about 3e-6
  if (precision == FGT_FP32 && tol < kMinTolFp32) {
    err = "FGT_FP32 needs tol >= 1e-6 (FP64 below)";
    return FGT_ERR_UNSUPPORTED;
  }
  if (precision == FGT_BF16X3 && tol < kMinTolBf16x3) {
    err = "FGT_BF16X3 needs tol >= 1e-4 (FGT_FP32 or FGT_FP64 below)";
    return FGT_ERR_UNSUPPORTED;
  }
  if (eps_internal < 0 || eps_internal >= 0.1) { err = "eps_internal must be 0 or in (0, 0.1)"; return FGT_ERR_INVALID_ARG; }
  const bool periodic = bc == FGT_PERIODIC;

  hp = HostPlan();
  hp.d = d; hp.p = p; hp.bc = bc; hp.precision = precision;
  hp.delta = delta; hp.tol = tol; hp.nleaves = n;
  hp.level.assign(level, level + n);
  hp.coord.assign(coord, coord + n * d);
  hp.sqrt_delta = std::sqrt(delta);

  // ---- tree validation: ranges, tiling, 2:1 balance
  const int maxlev = max_level_for_dim(d);
  int lmin = 1 << 30, lmax = 0;
  for (int64_t i = 0; i < n; i++) {
    int l = level[i];
    if (l < 0 || l > maxlev) { err = "leaf level out of range for this dimension"; return FGT_ERR_INVALID_ARG; }
    for (int a = 0; a < d; a++) {
      int32_t c = coord[i * d + a];
      if (c < 0 || (int64_t)c >= ((int64_t)1 << l)) { err = "leaf coordinate outside [0, 2^level)"; return FGT_ERR_NOT_TILING; }
    }
    lmin = std::min(lmin, l);
    lmax = std::max(lmax, l);
  }
  hp.lmin = lmin; hp.lmax = lmax;
  KeyMaker key(d);
  std::unordered_map<uint64_t, int32_t> leafmap;
  leafmap.reserve((size_t)n * 2);
  unsigned __int128 vol = 0;
  for (int64_t i = 0; i < n; i++) {
    if (!leafmap.emplace(key(level[i], &coord[i * d]), (int32_t)i).second) {
      err = "duplicate leaf"; return FGT_ERR_NOT_TILING;
    }
    vol += (unsigned __int128)1 << (d * (lmax - level[i]));
  }
  if (vol != ((unsigned __int128)1 << (d * lmax))) { err = "leaves do not cover the unit box exactly"; return FGT_ERR_NOT_TILING; }
  for (int64_t i = 0; i < n; i++) {
    int32_t c[3];
    for (int l = level[i] - 1; l >= 0; l--) {
      for (int a = 0; a < d; a++) c[a] = coord[i * d + a] >> (level[i] - l);
      if (leafmap.count(key(l, c))) { err = "a leaf contains another leaf"; return FGT_ERR_NOT_TILING; }
    }
  }
  // covering leaf of box (l, q): the leaf at level <= l that contains it, or -1
  auto covering = [&](int l, const int32_t* q, int* lev_out) -> int32_t {
    int32_t c[3];
    for (int ll = l; ll >= 0; ll--) {
      for (int a = 0; a < d; a++) c[a] = q[a] >> (l - ll);
      auto it = leafmap.find(key(ll, c));
      if (it != leafmap.end()) { *lev_out = ll; return it->second; }
    }
    return -1;
  };
  // wrap (periodic) or reject (free) a neighbor coordinate at level l
  auto neighbor = [&](int l, const int32_t* c, const int* dir, int32_t* q, int* shift) -> bool {
    int64_t nb = (int64_t)1 << l;
    for (int a = 0; a < d; a++) {
      int64_t v = (int64_t)c[a] + dir[a];
      int s = 0;
      if (v < 0) { v += nb; s = -1; }
      else if (v >= nb) { v -= nb; s = 1; }
      if (s != 0 && !periodic) return false;
      q[a] = (int32_t)v;
      if (shift) shift[a] = s;
    }
    return true;
  };
  const int n3 = ipow3(d);
  for (int64_t i = 0; i < n; i++) {
    int l = level[i];
    if (l < 2) continue;
    for (int code = 0; code < n3; code++) {
      int dir[3];
      dir_of(code, d, dir);
      bool zero = true;
      for (int a = 0; a < d; a++) zero = zero && dir[a] == 0;
      if (zero) continue;
      int32_t q[3];
      if (!neighbor(l, &coord[i * d], dir, q, nullptr)) continue;
      int lv;
      if (covering(l, q, &lv) >= 0 && lv < l - 1) {
        err = "tree is not level-restricted (2:1 balance with corner adjacency)";
        return FGT_ERR_NOT_BALANCED;
      }
    }
  }

  // ---- method parameters: eps, cutoff level, range R, modes (Theorem 1)
  const double eps = eps_internal > 0 ? eps_internal : tol;
  const double D0 = std::sqrt(std::log(3.0 / eps));
  const double cut = D0 * hp.sqrt_delta;  // cutoff length D0 sqrt(delta)
  int lc_auto = cut >= 1.0 ? 0 : (int)std::floor(std::log2(1.0 / cut));
  // guard the floor against rounding: the box side must not be below the cutoff length
  while (lc_auto > 0 && std::ldexp(1.0, -lc_auto) < cut) lc_auto--;
  while (std::ldexp(1.0, -(lc_auto + 1)) >= cut) lc_auto++;
  int lc = lc_auto;
  if (force_lc >= 0) {
    if (force_lc > lc_auto) { err = "force_lc finer than the automatic cutoff level would drop interactions"; return FGT_ERR_INVALID_ARG; }
    lc = force_lc;
  }
  if (lc > maxlev) lc = maxlev;
  // Periodic with l_c <= 1 (Section 5): the periodic kernel's truncated Fourier
  // series (Section 2.2) on the root replaces the image layer.  Its terms
  // sqrt(pi delta) exp(-pi^2 delta n^2) exp(2 pi i n x), |n| <= n_p, are the
  // plane waves of Theorem 1 with h = 2 pi sqrt(delta) (k_n = 2 pi n, weight
  // h/(2 sqrt(pi)) exp(-n^2 h^2/4)) and M = n_p + 1: the same tables, one box,
  // its only translation the identity, and no near field.
  const bool fourier = periodic && lc <= 1;
  hp.fourier = fourier;
  if (fourier) lc = 0;
  hp.lc = lc;
  hp.Llc = std::ldexp(1.0, -lc);
  if (fourier) {
    hp.pw.eps = eps;
    hp.pw.D0 = D0;
    hp.pw.R = 0.0;
    hp.pw.h = 2.0 * M_PI * hp.sqrt_delta;
    hp.pw.M = periodic_terms(eps, delta) + 1;
  } else {
    // largest per-axis separation between a target in a cutoff box and a source
    // in one of its colleagues (or the box itself when the root is the only box)
    double R = (lc == 0 ? 1.0 : 2.0 * hp.Llc) / hp.sqrt_delta;
    if (R < D0) R = D0;
    hp.pw = pw_params(eps, R);
  }
  hp.nr = 2 * hp.pw.M - 1;
  hp.nrs = 2 * hp.pw.M;
  if (hp.nrs > kMaxModes) { err = "too many plane-wave modes for this build (2M > 128)"; return FGT_ERR_UNSUPPORTED; }

  // ---- cutoff-level boxes and f-flags (Definition fflagdef)
  struct LcBox { int32_t c[3]; int isleaf; int f; int32_t idx; };
  std::unordered_map<uint64_t, int32_t> lcmap;
  std::vector<LcBox> lcbox;
  for (int64_t i = 0; i < n; i++) {
    int l = level[i];
    if (l < lc) continue;
    LcBox b{};
    for (int a = 0; a < d; a++) b.c[a] = coord[i * d + a] >> (l - lc);
    uint64_t k = key(lc, b.c);
    auto it = lcmap.find(k);
    if (it == lcmap.end()) {
      b.isleaf = (l == lc);
      b.f = 0;
      b.idx = -1;
      lcmap.emplace(k, (int32_t)lcbox.size());
      lcbox.push_back(b);
    }
  }
  for (auto& b : lcbox) {
    if (!b.isleaf || fourier) { b.f = 1; continue; }
    for (int code = 0; code < n3 && !b.f; code++) {
      int dir[3];
      dir_of(code, d, dir);
      int32_t q[3];
      if (!neighbor(lc, b.c, dir, q, nullptr)) continue;
      auto it = lcmap.find(key(lc, q));
      if (it != lcmap.end() && !lcbox[it->second].isleaf) b.f = 1;
    }
  }
  std::vector<int32_t> pwb;
  for (int32_t i = 0; i < (int32_t)lcbox.size(); i++)
    if (lcbox[i].f) pwb.push_back(i);
  std::sort(pwb.begin(), pwb.end(), [&](int32_t x, int32_t y) {
    return morton(lcbox[x].c, d, 0) < morton(lcbox[y].c, d, 0);
  });
  for (int32_t a = 0; a < (int32_t)pwb.size(); a++) lcbox[pwb[a]].idx = a;
  const int32_t nA = (int32_t)pwb.size();
  hp.pwbox_isleaf.resize(nA);
  for (int32_t a = 0; a < nA; a++) hp.pwbox_isleaf[a] = lcbox[pwb[a]].isleaf;

  // ---- plane-wave leaves grouped by their cutoff box; form/eval table ids
  // d = 3: within a box, leaves are ordered by (level, position on axis 3,
  // position on axis 1, position on axis 2), so that a plane (leaves of one
  // level sharing the axis-3 position, hence the axis-3 table) and a row of a
  // plane (also sharing the axis-1 position and table) are contiguous ranges.
  std::vector<PwLeafRef> pl;
  for (int64_t i = 0; i < n; i++) {
    int l = level[i];
    if (l < lc) continue;
    int32_t c[3];
    for (int a = 0; a < d; a++) c[a] = coord[i * d + a] >> (l - lc);
    const LcBox& b = lcbox[lcmap[key(lc, c)]];
    if (!b.f) continue;
    uint64_t m = morton(&coord[i * d], d, lmax - l);
    int32_t lv = 0;
    if (d == 3) {
      const int sh = l - lc;  // < 21: positions take 21 bits each
      auto rel = [&](int a) { return (uint64_t)(coord[i * d + a] - ((coord[i * d + a] >> sh) << sh)); };
      m = (rel(2) << 42) | (rel(0) << 21) | rel(1);
      lv = l;
    }
    pl.push_back({b.idx, m, (int32_t)i, lv});
  }
  finish_pw_lists(hp, pl, nA, level, coord, allow_fuse);

  // ---- P-lists (Definition before Algorithm 4, read for every box with f = 1):
  // colleagues with f = 1 (images included when periodic), excluding pairs of
  // two leaves, which the near field handles.
  // Each list is sorted by (source box, code), the order the fused translation's
  // target groups keep for every member.
  hp.plist_start.assign(nA + 1, 0);
  for (int32_t a = 0; a < nA; a++) {
    const LcBox& A = lcbox[pwb[a]];
    std::vector<std::pair<int32_t, int32_t>> ents;  // (source box, code)
    for (int code = 0; code < n3; code++) {
      int dir[3];
      dir_of(code, d, dir);
      int32_t q[3];
      if (fourier) {
        // the root's expansion already holds every image: itself, unshifted
        bool zero = true;
        for (int a = 0; a < d; a++) zero = zero && dir[a] == 0;
        if (!zero) continue;
        ents.push_back({A.idx, code});
        continue;
      }
      if (!neighbor(lc, A.c, dir, q, nullptr)) continue;
      auto it = lcmap.find(key(lc, q));
      if (it == lcmap.end()) continue;
      const LcBox& B = lcbox[it->second];
      if (!B.f || (A.isleaf && B.isleaf)) continue;
      ents.push_back({B.idx, code});  // dir = B - A per axis
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
      for (int ax = 0; ax < 3; ax++) bc[(size_t)a * 3 + ax] = lcbox[pwb[a]].c[ax];
    build_te_groups(hp, bc);
  }

  // ---- D-lists: every leaf at level <= lc gathers from its leaf neighbors at
  // levels <= lc (colleagues, coarse and fine neighbors; images if periodic).
  std::unordered_map<uint64_t, int32_t> vtab;  // (source level, type) -> id
  std::vector<int32_t> vtab_lv, vtab_ty;
  std::vector<std::pair<int64_t, int32_t>> tgt;  // (morton, leaf)
  for (int64_t i = 0; i < n && !fourier; i++)
    if (level[i] <= lc) tgt.push_back({(int64_t)morton(&coord[i * d], d, lmax - level[i]), (int32_t)i});
  std::sort(tgt.begin(), tgt.end());
  hp.near_start.push_back(0);
  for (auto& tt : tgt) {
    const int32_t T = tt.second;
    const int l = level[T];
    const int32_t* cT = &coord[T * d];
    struct Ent { int32_t S; int shift[3]; };
    std::vector<Ent> ents;
    auto add = [&](int32_t S, const int* shift) {
      for (auto& e : ents) {
        bool same = e.S == S;
        for (int a = 0; a < d && same; a++) same = e.shift[a] == shift[a];
        if (same) return;
      }
      Ent e{S, {0, 0, 0}};
      for (int a = 0; a < d; a++) e.shift[a] = shift[a];
      ents.push_back(e);
    };
    for (int code = 0; code < n3; code++) {
      int dir[3];
      dir_of(code, d, dir);
      int32_t q[3];
      int shift[3] = {0, 0, 0};
      if (!neighbor(l, cT, dir, q, shift)) continue;
      // same level
      auto it = leafmap.find(key(l, q));
      if (it != leafmap.end()) { add(it->second, shift); continue; }
      // coarser leaf containing the neighbor box
      if (l >= 1) {
        int32_t par[3];
        for (int a = 0; a < d; a++) par[a] = q[a] >> 1;
        auto ip = leafmap.find(key(l - 1, par));
        if (ip != leafmap.end()) { add(ip->second, shift); continue; }
      }
      // finer leaves (children of the neighbor box that touch T)
      if (l + 1 <= lc) {
        int nb = 1 << d;
        for (int b = 0; b < nb; b++) {
          int32_t ch[3];
          bool ok = true;
          for (int a = 0; a < d; a++) {
            int bit = (b >> a) & 1;
            if (dir[a] == -1 && bit == 0) ok = false;
            if (dir[a] == 1 && bit == 1) ok = false;
            ch[a] = 2 * q[a] + bit;
          }
          if (!ok) continue;
          auto ic = leafmap.find(key(l + 1, ch));
          if (ic != leafmap.end()) add(ic->second, shift);
        }
      }
    }
    std::sort(ents.begin(), ents.end(), [&](const Ent& x, const Ent& y) {
      if (x.S != y.S) return x.S < y.S;
      for (int a = 0; a < d; a++) if (x.shift[a] != y.shift[a]) return x.shift[a] < y.shift[a];
      return false;
    });
    // one row per source: d table ids (axis 1..d) then the source leaf
    std::vector<std::array<int32_t, kMaxDim + 1>> rows;
    for (auto& e : ents) {
      const int lS = level[e.S];
      if (lS > lc) continue;
      const int lF = std::max(l, lS);
      std::array<int32_t, kMaxDim + 1> row{};
      row[kMaxDim] = e.S;
      for (int a = 0; a < d; a++) {
        // centers in units of 2^-(lF+1); S shifted by its image
        int64_t cTu = (2 * (int64_t)cT[a] + 1) << (lF - l);
        int64_t cSu = ((2 * (int64_t)coord[e.S * d + a] + 1) << (lF - lS)) + ((int64_t)e.shift[a] << (lF + 1));
        int64_t diff = cTu - cSu;
        int64_t LS = (int64_t)1 << (lF + 1 - lS);
        int64_t rel4 = 4 * diff / LS;  // 4 (c_T - c_S)/L_S
        int type = -1;
        if (l == lS) type = rel4 == -4 ? 0 : rel4 == 0 ? 1 : rel4 == 4 ? 2 : -1;
        else if (l == lS + 1) type = rel4 == -3 ? 3 : rel4 == -1 ? 4 : rel4 == 1 ? 5 : rel4 == 3 ? 6 : -1;
        else if (l == lS - 1) type = rel4 == -6 ? 7 : rel4 == -2 ? 8 : rel4 == 2 ? 9 : rel4 == 6 ? 10 : -1;
        if (type < 0 || 4 * diff % LS != 0) { err = "internal: unexpected neighbor geometry"; return FGT_ERR_INVALID_ARG; }
        uint64_t k = ((uint64_t)lS << 32) | (uint32_t)type;
        auto iv = vtab.find(k);
        int32_t id;
        if (iv == vtab.end()) {
          id = (int32_t)vtab_lv.size();
          vtab.emplace(k, id);
          vtab_lv.push_back(lS);
          vtab_ty.push_back(type);
        } else {
          id = iv->second;
        }
        row[a] = id;
      }
      rows.push_back(row);
    }
    // sort so that runs of equal tables are contiguous: d = 3 by (axis 3,
    // axis 1, axis 2) -- the kernel contracts axis 2 per source, axis 1 per
    // run of (axis 3, axis 1) and axis 3 per run of axis 3; d = 2 by (axis 2,
    // axis 1) -- axis 1 per source, axis 2 per run
    static const int order3[3] = {2, 0, 1}, order2[2] = {1, 0}, order1[1] = {0};
    const int* order = d == 3 ? order3 : (d == 2 ? order2 : order1);
    std::sort(rows.begin(), rows.end(), [&](const std::array<int32_t, kMaxDim + 1>& x,
                                            const std::array<int32_t, kMaxDim + 1>& y) {
      for (int i = 0; i < d; i++) if (x[order[i]] != y[order[i]]) return x[order[i]] < y[order[i]];
      return x[kMaxDim] < y[kMaxDim];
    });
    for (auto& row : rows) {
      hp.near_src.push_back(row[kMaxDim]);
      for (int a = 0; a < d; a++) hp.near_tab.push_back(row[a]);
    }
    hp.near_tgt.push_back(T);
    int haspw = 0;
    if (l == lc) {
      auto it = lcmap.find(key(lc, cT));
      haspw = (it != lcmap.end() && lcbox[it->second].f) ? 1 : 0;
    }
    hp.near_haspw.push_back(haspw);
    hp.near_start.push_back((int32_t)hp.near_src.size());
  }
  {
    // dispatch order of the near targets (workgroup b runs on XCD b % 8): the
    // targets in Morton order are cut into eight runs of equal count, run x on
    // XCD x, so that the targets resident on an XCD at one time are neighbors
    // and find most of their sources' sigma in its L2; the last kNearTail of
    // a run go most sources first, so that no long target starts late
    const int64_t nt = (int64_t)hp.near_tgt.size();
    int lmax = 0;
    for (int64_t i = 0; i < n; i++) lmax = std::max(lmax, (int)level[i]);
    std::vector<uint64_t> mk(nt, 0);
    for (int64_t i = 0; i < nt; i++) {
      const int32_t T = hp.near_tgt[i];
      for (int a = 0; a < d; a++) {
        const uint32_t c = (uint32_t)coord[(int64_t)T * d + a] << (lmax - level[T]);
        for (int b = 0; b < 32 && d * b + a < 64; b++) mk[i] |= (uint64_t)((c >> b) & 1u) << (d * b + a);
      }
    }
    std::vector<int32_t> mo(nt);
    for (int64_t i = 0; i < nt; i++) mo[i] = (int32_t)i;
    std::stable_sort(mo.begin(), mo.end(), [&](int32_t x, int32_t y) { return mk[x] < mk[y]; });
    auto nsrc = [&](int32_t i) { return hp.near_start[i + 1] - hp.near_start[i]; };
    std::vector<std::vector<int32_t>> run(kXcdCount);
    {
      const int64_t base = nt / kXcdCount, extra = nt % kXcdCount;
      int64_t at = 0;
      for (int x = 0; x < kXcdCount; x++) {
        const int64_t len = base + (x < extra ? 1 : 0);
        run[x].assign(mo.begin() + at, mo.begin() + at + len);
        at += len;
        const size_t k0 = run[x].size() > (size_t)kNearTail ? run[x].size() - kNearTail : 0;
        std::stable_sort(run[x].begin() + k0, run[x].end(),
                         [&](int32_t u, int32_t v) { return nsrc(u) > nsrc(v); });
      }
    }
    std::vector<int32_t> ord;
    ord.reserve(nt);
    for (size_t k = 0; k < run[0].size(); k++)  // run 0 is a longest one
      for (int x = 0; x < kXcdCount; x++)
        if (k < run[x].size()) ord.push_back(run[x][k]);
    std::vector<int32_t> tg, hpw, st{0}, src, tab;
    for (int32_t i : ord) {
      tg.push_back(hp.near_tgt[i]);
      hpw.push_back(hp.near_haspw[i]);
      for (int32_t q = hp.near_start[i]; q < hp.near_start[i + 1]; q++) {
        src.push_back(hp.near_src[q]);
        for (int a = 0; a < d; a++) tab.push_back(hp.near_tab[(int64_t)q * d + a]);
      }
      st.push_back((int32_t)src.size());
    }
    hp.near_tgt.swap(tg);
    hp.near_haspw.swap(hpw);
    hp.near_start.swap(st);
    hp.near_src.swap(src);
    hp.near_tab.swap(tab);
  }
  hp.nvtab = (int)vtab_lv.size();
  hp.vtab_meta = vtab_lv;
  hp.vtab_meta.insert(hp.vtab_meta.end(), vtab_ty.begin(), vtab_ty.end());

  build_tables(hp);
  return FGT_OK;
}

}  // namespace fgt
