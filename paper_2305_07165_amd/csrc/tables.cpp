// FP64 one-dimensional tables of the box Gauss transform (Section 4.1).
//
// Real plane-wave basis.  Theorem 1 approximates G(x) by
//   sum_{m=-M}^{M-1} w_m exp(i k_m x),  k_m = m h / sqrt(delta),
//   w_m = h/(2 sqrt(pi)) exp(-m^2 h^2/4).
// Its proof bounds the truncation error by the two-sided tail |m| >= M, so the
// symmetric sum over |m| <= M-1 (which the paper notes could be used instead)
// keeps the same bound.  For real x that sum is real:
//   G(x - y) ~ sum_r wh_r b_r(x - c) b_r(y - c)      (any center c)
// with b_0 = 1, b_{2m-1} = cos(k_m .), b_{2m} = sin(k_m .), m = 1..M-1 and
// weights wh_0 = w_0, wh_{2m-1} = wh_{2m} = 2 w_m: nr = 2M-1 real modes per axis,
// the same information as the complex expansion of a real density (whose
// coefficients satisfy v(-m) = conj(v(m))) at half the storage.  A shift of the
// expansion center is a 2x2 rotation of each (cos, sin) pair, the real form of
// the diagonal translations T_{c->p}, T_{out->in}, T_{p->c}.
//
// Storage order of the modes (nrs = 2M per axis): b_0 at 0, a zero at 1, and
// the pair (cos, sin) of mode m at (2m, 2m+1).  The zero row of F and column
// of E make the stored slot 1 an exact zero mode, so every mode index m owns
// an aligned pair and a shift rotates every pair alike (m = 0 by the identity).
//
// Tables (per axis, all FP64):
//  F[l,pos][r][j]  leaf values (level l, position pos inside its cutoff box
//                  along the axis) -> moments about the cutoff-box center:
//                  wh_r int_S b_r(y - c_A) l_j(y) dy  =  T_{pol->pw} T_{val->pol}
//                  with the center shift folded in (Definitions val2poldef,
//                  pol2pwdef; the integrals I[P_n] = 2 i^n j_n of Eq. (pwintegrals2)).
//  E[l,pos][i][r]  b_r(x_i - c_A): moments about the cutoff-box center -> leaf
//                  node values (Definition pw2pot with the shift folded in).
//  V[l,type][i][j] int_S exp(-(x_i - y)^2/delta) l_j(y) dy for the 11 neighbor
//                  offsets of Definitions pol2potdef-pol2potdef3 (T_{val->pot}).
//  rot[m]          cos, sin of k_m L_c (colleague shift at the cutoff level).
// l_j is the Lagrange polynomial of the leaf's Gauss-Legendre node j, written
// through the Legendre coefficients of Eq. (val2poleq): l_j = sum_n V2P[n][j] P_n.
#include <cmath>
#include <cstring>
#include <vector>

#include "fgt_host.h"

namespace fgt {

void gauss_legendre(int n, double* x, double* w) {
  // Newton iteration on P_n from the Chebyshev-like first guess; ascending nodes
  const int half = (n + 1) / 2;
  for (int k = 0; k < half; k++) {
    double z = std::cos(M_PI * (4.0 * k + 3.0) / (4.0 * n + 2.0));
    double dpn = 1.0;
    for (int iter = 0; iter < 64; iter++) {
      double pm1 = 1.0, pn = z;  // P_0, P_1
      for (int j = 2; j <= n; j++) {
        double pnew = ((2 * j - 1) * z * pn - (j - 1) * pm1) / j;
        pm1 = pn;
        pn = pnew;
      }
      if (n == 1) { pn = z; pm1 = 1.0; }
      dpn = n * (pm1 - z * pn) / (1.0 - z * z);
      double step = pn / dpn;
      z -= step;
      if (std::fabs(step) <= 1e-16 * std::fabs(z) + 1e-300) {
        // one more evaluation of the derivative at the final root
        pm1 = 1.0; pn = z;
        for (int j = 2; j <= n; j++) {
          double pnew = ((2 * j - 1) * z * pn - (j - 1) * pm1) / j;
          pm1 = pn;
          pn = pnew;
        }
        if (n == 1) { pn = z; pm1 = 1.0; }
        dpn = n * (pm1 - z * pn) / (1.0 - z * z);
        break;
      }
    }
    x[n - 1 - k] = z;
    x[k] = -z;
    w[k] = w[n - 1 - k] = 2.0 / ((1.0 - z * z) * dpn * dpn);
  }
  if (n % 2) x[n / 2] = 0.0;
}

namespace {

void legendre_values(int n, double t, double* P) {
  P[0] = 1.0;
  if (n > 1) P[1] = t;
  for (int k = 2; k < n; k++) P[k] = ((2 * k - 1) * t * P[k - 1] - (k - 1) * P[k - 2]) / k;
}

// Spherical Bessel j_0..j_{n-1} at x >= 0: power series for small x, otherwise
// Miller's downward recurrence normalized by sum_k (2k+1) j_k^2 = 1.
void spherical_bessel(int n, double x, double* j) {
  if (x < 0.25) {
    double pw = 1.0, dfac = 1.0;  // x^k, (2k+1)!!
    for (int k = 0; k < n; k++) {
      if (k > 0) { pw *= x; dfac *= (2 * k + 1); }
      double term = 1.0, sum = 1.0, y = -0.5 * x * x;
      for (int s = 1; s < 30; s++) {
        term *= y / (s * (2.0 * k + 2.0 * s + 1.0));
        sum += term;
        if (std::fabs(term) < 1e-18 * std::fabs(sum)) break;
      }
      j[k] = pw / dfac * sum;
    }
    return;
  }
  const int K = n + (int)std::ceil(x) + 40;
  std::vector<double> f(K + 2, 0.0);
  f[K + 1] = 0.0;
  f[K] = 1e-30;
  for (int k = K; k >= 1; k--) {
    f[k - 1] = (2.0 * k + 1.0) / x * f[k] - f[k + 1];
    if (std::fabs(f[k - 1]) > 1e100) {  // keep sum (2k+1) f_k^2 finite
      for (int q = k - 1; q <= K; q++) f[q] *= 1e-100;
    }
  }
  double s = 0.0;
  for (int k = 0; k <= K; k++) s += (2.0 * k + 1.0) * f[k] * f[k];
  double scale = 1.0 / std::sqrt(s);
  // fix the sign with j_0 = sin x / x (or j_1 when j_0 is near a zero)
  double j0 = std::sin(x) / x;
  double j1 = std::sin(x) / (x * x) - std::cos(x) / x;
  double ref = std::fabs(j0) > std::fabs(j1) ? j0 : j1;
  double got = std::fabs(j0) > std::fabs(j1) ? f[0] : f[1];
  if ((ref < 0) != (got < 0)) scale = -scale;
  for (int k = 0; k < n; k++) j[k] = f[k] * scale;
}

// int_{-1}^{1} cos(a t) P_n(t) dt and int sin(a t) P_n(t) dt: real and imaginary
// parts of I[P_n](a) = 2 i^n j_n(a), Eq. (pwintegrals2).
void cos_sin_moments(int p, double a, double* C, double* S) {
  double j[64];
  spherical_bessel(p, a, j);
  for (int n = 0; n < p; n++) {
    switch (n & 3) {
      case 0: C[n] = 2 * j[n]; S[n] = 0; break;
      case 1: C[n] = 0; S[n] = 2 * j[n]; break;
      case 2: C[n] = -2 * j[n]; S[n] = 0; break;
      default: C[n] = 0; S[n] = -2 * j[n]; break;
    }
  }
}

// int_{-1}^{1} exp(-(t - s)^2/lam^2) P_n(s) ds, n < p, by composite 24-point
// Gauss-Legendre over the part of [-1,1] within 6.5 lam of t (the rest is
// below 1e-18), panels no wider than min(lam/2, 1/4).
void gauss_legendre_moments(int p, double t, double lam, const double* xq, const double* wq,
                            int nq, double* out) {
  for (int n = 0; n < p; n++) out[n] = 0.0;
  double lo = std::fmax(-1.0, t - 6.5 * lam), hi = std::fmin(1.0, t + 6.5 * lam);
  if (!(hi > lo)) return;
  double width = std::fmin(0.5 * lam, 0.25);
  int np = (int)std::ceil((hi - lo) / width);
  if (np < 1) np = 1;
  double hw = (hi - lo) / np;
  double P[64];
  for (int k = 0; k < np; k++) {
    double a = lo + k * hw, mid = a + 0.5 * hw, r = 0.5 * hw;
    for (int q = 0; q < nq; q++) {
      double s = mid + r * xq[q];
      double e = (t - s) / lam;
      double g = std::exp(-e * e) * r * wq[q];
      legendre_values(p, s, P);
      for (int n = 0; n < p; n++) out[n] += g * P[n];
    }
  }
}

}  // namespace

void build_tables(HostPlan& hp) {
  const int p = hp.p, nr = hp.nrs, M = hp.pw.M;
  const double h = hp.pw.h, sd = hp.sqrt_delta;
  std::vector<double> eta(p), wgl(p), V2P(p * p), P(p);
  gauss_legendre(p, eta.data(), wgl.data());
  for (int j = 0; j < p; j++) {
    legendre_values(p, eta[j], P.data());
    for (int n = 0; n < p; n++) V2P[n * p + j] = 0.5 * (2 * n + 1) * wgl[j] * P[n];
  }
  // weights wh_r (Theorem 1, folded into the formation tables)
  std::vector<double> km(M), wm(M);
  for (int m = 0; m < M; m++) {
    km[m] = m * h / sd;
    wm[m] = (m == 0 ? 0.5 : 1.0) * h / std::sqrt(M_PI) * std::exp(-0.25 * m * m * h * h);
  }

  // ---- formation / evaluation tables
  hp.F.assign((size_t)hp.nftab * nr * p, 0.0);
  hp.E.assign((size_t)hp.nftab * p * nr, 0.0);
  std::vector<double> Tpw(nr * p), C(p), S(p);
  for (int id = 0; id < hp.nftab; id++) {
    const int l = hp.ftab_meta[id], pos = hp.ftab_meta[hp.nftab + id];
    const double L = std::ldexp(1.0, -l);
    const double shift = L * (pos + 0.5) - 0.5 * hp.Llc;  // c_S - c_A
    if (hp.point_tables) {
      // point transform: the leaf's p^d values are charges at its nodes (a proxy
      // grid), so F holds wh_r b_r(z_j - c_A) at the nodes z_j (Eq.
      // (multipoleexpansion) for one charge) instead of integrals
      double* Fo = &hp.F[(size_t)id * nr * p];
      for (int j = 0; j < p; j++) {
        const double z = shift + 0.5 * L * eta[j];
        Fo[0 * p + j] = wm[0];
        Fo[1 * p + j] = 0.0;  // the zero slot
        for (int m = 1; m < M; m++) {
          Fo[(2 * m) * p + j] = wm[m] * std::cos(km[m] * z);
          Fo[(2 * m + 1) * p + j] = wm[m] * std::sin(km[m] * z);
        }
      }
    }
    for (int m = 0; m < M && !hp.point_tables; m++) {
      cos_sin_moments(p, km[m] * 0.5 * L, C.data(), S.data());
      const double cs = std::cos(km[m] * shift), sn = std::sin(km[m] * shift);
      const double sc = wm[m] * 0.5 * L;
      if (m == 0) {
        for (int n = 0; n < p; n++) {
          Tpw[n] = sc * C[n];
          Tpw[p + n] = 0.0;  // the zero slot
        }
      } else {
        for (int n = 0; n < p; n++) {
          Tpw[(2 * m) * p + n] = sc * (cs * C[n] - sn * S[n]);
          Tpw[(2 * m + 1) * p + n] = sc * (sn * C[n] + cs * S[n]);
        }
      }
    }
    double* Fo = &hp.F[(size_t)id * nr * p];
    for (int r = 0; r < nr && !hp.point_tables; r++)
      for (int j = 0; j < p; j++) {
        double s = 0.0;
        for (int n = 0; n < p; n++) s += Tpw[r * p + n] * V2P[n * p + j];
        Fo[r * p + j] = s;
      }
    double* Eo = &hp.E[(size_t)id * p * nr];
    for (int i = 0; i < p; i++) {
      const double x = shift + 0.5 * L * eta[i];  // x_i - c_A
      Eo[i * nr + 0] = 1.0;
      Eo[i * nr + 1] = 0.0;  // the zero slot
      for (int m = 1; m < M; m++) {
        Eo[i * nr + 2 * m] = std::cos(km[m] * x);
        Eo[i * nr + 2 * m + 1] = std::sin(km[m] * x);
      }
    }
  }

  // ---- near-field tables
  static const double rel_of_type[11] = {-1.0, 0.0, 1.0, -0.75, -0.25, 0.25, 0.75,
                                         -1.5, -0.5, 0.5, 1.5};
  const int nq = 24;
  std::vector<double> xq(nq), wq(nq), Tpot(p * p), mom(p);
  gauss_legendre(nq, xq.data(), wq.data());
  hp.V.assign((size_t)hp.nvtab * p * p, 0.0);
  for (int id = 0; id < hp.nvtab; id++) {
    const int l = hp.vtab_meta[id], type = hp.vtab_meta[hp.nvtab + id];
    const double LS = std::ldexp(1.0, -l);
    const double LT = type < 3 ? LS : (type < 7 ? 0.5 * LS : 2.0 * LS);
    const double lam = 2.0 * sd / LS;
    for (int i = 0; i < p; i++) {
      const double xi = rel_of_type[type] * LS + 0.5 * LT * eta[i];  // x_i - c_S
      gauss_legendre_moments(p, 2.0 * xi / LS, lam, xq.data(), wq.data(), nq, mom.data());
      for (int n = 0; n < p; n++) Tpot[i * p + n] = 0.5 * LS * mom[n];
    }
    double* Vo = &hp.V[(size_t)id * p * p];
    for (int i = 0; i < p; i++)
      for (int j = 0; j < p; j++) {
        double s = 0.0;
        for (int n = 0; n < p; n++) s += Tpot[i * p + n] * V2P[n * p + j];
        Vo[i * p + j] = s;
      }
  }

  hp.rot.assign(2 * M, 0.0);
  for (int m = 0; m < M; m++) {
    hp.rot[2 * m] = std::cos(km[m] * hp.Llc);
    hp.rot[2 * m + 1] = std::sin(km[m] * hp.Llc);
  }
}

}  // namespace fgt
