// Host-side plan of the box Gauss transform: parameters, flat tree lists and
// the FP64 one-dimensional tables.  Built once by fgt_plan(), then uploaded.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace fgt {

constexpr int kMaxDim = 3;
constexpr int kMaxP = 16;      // nodes per axis handled by the kernels
// smallest tol a reduced-precision plan accepts (FGT_ERR_UNSUPPORTED below)
constexpr double kMinTolFp32 = 1e-6 * (1 - 1e-9);
constexpr double kMinTolBf16x3 = 1e-4 * (1 - 1e-9);
constexpr int kMaxModes = 128; // stored plane-wave modes per axis (2M)
constexpr int kFormLeaves = 8; // leaves per formation work item
constexpr double kFuseBytes = 128e6;  // psi bytes above which the 3D translation is fused
constexpr int kTeGroup = 4;    // target boxes per fused-translation group (siblings)
constexpr int kTeNoDir = 0xFF; // group entry: the member does not take this source
constexpr int kTeTail = 288;   // fused translation: workgroups per XCD run longest first at the end
                               // (three rounds of 32 CUs x 3 resident workgroups)
constexpr int kNearTail = 64;  // near field: targets per XCD run most sources first at the end
                               // (one round of 32 CUs x 2 resident workgroups)
constexpr int kXcdCount = 8;   // XCDs (separate L2s) of the device; workgroup b runs on b % 8

// Plane-wave parameters of Theorem 1 for tolerance eps and range R (units of
// sqrt(delta)): D0 = sqrt(log(3/eps)), h = 2 pi/(R + D0), M = ceil(D0 (R+D0)/pi).
struct PwParams {
  double eps = 0, D0 = 0, R = 0, h = 0;
  int M = 0;
};
PwParams pw_params(double eps, double R);

// n_p = ceil(sqrt(log(1/eps))/(pi sqrt(delta))): Fourier terms per side of the
// periodic Gaussian on the unit interval (Section 2.2, Table 2).
int periodic_terms(double eps, double delta);

struct HostPlan {
  // problem
  int d = 0, p = 0, bc = 0, precision = 0;
  double delta = 0, tol = 0;
  int64_t nleaves = 0;
  std::vector<int32_t> level, coord;  // caller order, coord[i*d+a]
  int lmin = 0, lmax = 0;

  // method parameters
  int lc = 0;          // cutoff level
  double Llc = 1;      // side of a cutoff-level box
  PwParams pw;         // eps, D0, R, h, M
  int nr = 0;          // real modes per axis, 2M-1
  int nrs = 0;         // stored modes per axis, 2M: every expansion, table and
                       // intermediate stores mode m's (cos, sin) pair at 2m, 2m+1,
                       // the constant mode at 0 and a zero at 1 (the sin of m = 0)
  double sqrt_delta = 0;
  // periodic with l_c <= 1: the root's Fourier series (lc = 0, h = 2 pi
  // sqrt(delta), M = n_p + 1, identity translation, no near field)
  bool fourier = false;

  // formation tables evaluated at the leaf nodes instead of integrated over the
  // leaf: the leaves are proxy grids of a point transform (point_host.h)
  bool point_tables = false;

  // d = 3: fuse the translations with the first evaluation step when the
  // incoming expansions would not stay in the caches (more than kFuseBytes)
  bool fuse_te = false;

  // plane-wave boxes (cutoff level, f = 1), Morton order
  std::vector<int32_t> pwbox_isleaf;  // [nA]
  std::vector<int32_t> pw_start;      // [nA+1] ranges of pw leaves per box
  std::vector<int32_t> pwleaf_id;     // [nL] caller leaf index
  std::vector<int32_t> pwleaf_tab;    // [nL*d] form/eval table id per axis
  std::vector<int32_t> pwleaf_box;    // [nL] cutoff box of each pw leaf
  std::vector<int32_t> box_order;     // [nA] pw boxes by decreasing leaf count (dispatch order)
  std::vector<int32_t> plist_start;   // [nA+1]
  std::vector<int32_t> plist_src;     // [nP] plane-wave box index
  std::vector<int32_t> plist_dir;     // [nP] sum_a (dir_a+1) 3^a, dir = src - dst
                                      // (each box's list sorted by source box, then code)
  // d = 3 fused translation: groups of up to kTeGroup target boxes, the
  // children of one parent at level lc - 1 that share their position along
  // axis 3, each with the union of its members' P-lists.
  // Entry e of group g is a source box te_src[e] and, per member slot t, its
  // direction code in the member's P-list (byte t % 4 of te_dir[W e + t / 4],
  // W = (kTeGroup + 3) / 4 words per entry; kTeNoDir: not in it).  A member
  // meets its own P-list in its own order, and the members of an entry share
  // the axis-3 part of their codes (code / 9).
  std::vector<int32_t> te_start;      // [nG+1] ranges of entries per group
  std::vector<int32_t> te_mem;        // [nG*kTeGroup] member box per slot, -1 = empty
  std::vector<int32_t> te_src;        // [nTE]
  std::vector<int32_t> te_dir;        // [nTE*W] packed direction codes
  // tiles of the fused translation: te_tp (m1, m2) mode pairs each (kernels.h
  // keeps phi tile-major with the same tiles); workgroup b of the launch runs
  // group te_wg[2b] on tile te_wg[2b+1] (-1: nothing).  Tile t of every group
  // runs on XCD t % 8 (b % 8 is the XCD of workgroup b) so that a source tile
  // is read into one L2; each XCD sweeps its tiles in turn, the groups of a
  // sweep in Morton order; the tiles past the last multiple of 8 are one sweep
  // cut into eight runs of equal work; the last kTeTail workgroups of an XCD
  // run longest first.
  int te_tp = 0;
  std::vector<int32_t> te_wg;         // [nWG*2]
  // d = 3 only: a plane is a run of pw leaves of one box with the same level and
  // axis-3 position (one axis-3 table); a row is a run of a plane's leaves that
  // also share the axis-1 position (one axis-1 table)
  std::vector<int32_t> plane_start;   // [nA+1] ranges of planes per box
  std::vector<int32_t> plane_tab;     // [nPl*3] entry 2: the plane's axis-3 table (0, 0, t3)
  std::vector<int32_t> plane_row;     // [nPl+1] ranges of rows per plane
  std::vector<int32_t> row_start;     // [nR+1] ranges of pw leaves per row
  std::vector<int32_t> row_tab;       // [nR] the row's axis-1 table
  std::vector<int32_t> plane_order;   // [nPl] dispatch order of the per-plane stages: most work first
  // evaluation work items: (box, first pw leaf, count) with count*p <= 64 rows
  std::vector<int32_t> echunk;        // [nE*3]
  // formation work items: (box, first unit, end unit, partial slot or -1), a unit
  // being a plane for d = 3 and a pw leaf otherwise;
  // boxes with more than kFormLeaves units are split, their partial sums
  // reduced in item order by (box, first slot, slot count) records
  std::vector<int32_t> fitem;         // [nFI*4]
  std::vector<int32_t> fred;          // [nFR*3]
  int32_t nslots = 0;

  // near field: targets at level <= lc, gather lists
  std::vector<int32_t> near_tgt;      // [nT] caller leaf index
  std::vector<int32_t> near_haspw;    // [nT] 1 if the leaf also receives a pw evaluation
  std::vector<int32_t> near_start;    // [nT+1]
  std::vector<int32_t> near_src;      // [nN] caller leaf index
  std::vector<int32_t> near_tab;      // [nN*d] near table id per axis; a target's sources
                                      // are sorted by tables: (axis 3, axis 1, axis 2) for
                                      // d = 3, (axis 2, axis 1) for d = 2

  // tables (FP64; rounded once to the compute precision on upload)
  int nftab = 0, nvtab = 0;
  std::vector<int32_t> ftab_meta;     // [2*nftab] level of each form/eval table, then its position
  std::vector<int32_t> vtab_meta;     // [2*nvtab] source level of each near table, then its type (0..10)
  std::vector<double> F;              // [nftab][nrs][p]  leaf values -> cutoff-box pw moments
  std::vector<double> E;              // [nftab][p][nrs]  cutoff-box pw moments -> leaf values
  std::vector<double> V;              // [nvtab][p][p]   source values -> target values
  std::vector<double> rot;            // [M][2]  cos, sin of k_m * Llc

  // counts for reporting
  int64_t n_pwbox() const { return (int64_t)pwbox_isleaf.size(); }
  int64_t n_pwleaf() const { return (int64_t)pwleaf_id.size(); }
  int64_t n_plist() const { return (int64_t)plist_src.size(); }
  int64_t n_te_group() const { return te_start.empty() ? 0 : (int64_t)te_start.size() - 1; }
  int64_t n_near_tgt() const { return (int64_t)near_tgt.size(); }
  int64_t n_near_pair() const { return (int64_t)near_src.size(); }
  int64_t n_plane() const { return row_start.empty() ? 0 : (int64_t)plane_row.size() - 1; }
  int64_t n_row() const { return row_start.empty() ? 0 : (int64_t)row_start.size() - 1; }
};

// A plane-wave leaf of cutoff box `box`: `id` its row in sigma / u, `lv` its
// level, `m` its order key inside the box.
struct PwLeafRef { int32_t box; uint64_t m; int32_t id; int32_t lv; };
// Sorts the plane-wave leaves by (box, level, key) and fills pw_start,
// pwleaf_id/tab/box, the form/eval table ids (nftab, ftab_meta), for d = 3 the
// planes and rows, fuse_te, box_order, the formation items (fitem, fred,
// nslots) and the evaluation chunks.  level/coord are indexed by id.
void finish_pw_lists(HostPlan& hp, std::vector<PwLeafRef>& pl, int32_t nA, const int32_t* level,
                     const int32_t* coord, bool allow_fuse);

// Groups the plane-wave boxes of a fused d = 3 plan (te_*) from the P-lists
// and box_coord [nA*3], the boxes' coordinates at the cutoff level.
void build_te_groups(HostPlan& hp, const std::vector<int32_t>& box_coord);

// Validates the tree and fills every field above.  Returns an FGT_* code.
int build_host_plan(int dim, int64_t nleaves, const int32_t* level, const int32_t* coord,
                    int p, double delta, double tol, int bc, int precision,
                    double eps_internal, int force_lc, bool allow_fuse, HostPlan& hp,
                    std::string& err);

// Tables (tables.cpp)
void gauss_legendre(int n, double* x, double* w);
void build_tables(HostPlan& hp);

}  // namespace fgt
