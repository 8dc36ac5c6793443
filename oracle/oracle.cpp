// Test infrastructure, not product code.
//
// A plain, slow CPU evaluation of the helicity- and colour-summed tree-level
// squared matrix element |M|^2 for
//   e+ e- -> mu+ mu-  (photon + Z),  g g -> t tbar + n g  (n = 0..3),
//   u ubar -> e+ e- + n g  (photon + Z, n = 0..3: the Drell-Yan family),  g g -> g g.
//
// It follows the paper's section "Parallel scattering amplitudes": external
// wavefunctions, propagators and vertices are evaluated explicitly, every
// non-vanishing spin configuration is evaluated and summed, and the colour
// inner product is taken at the end.  The paper gives no Feynman rules, so they
// are the textbook ones (Peskin & Schroeder conventions, Feynman gauge for
// gluons, unitary gauge with a fixed width for the Z, metric (+,-,-,-)).
//
// Two evaluations of the QCD amplitudes are provided:
//  * "dressed": colour-dressed Berends-Giele recursion with explicit SU(3)
//    generators and structure constants, summed over every external colour
//    assignment.  This is the plain definition: the sum over all tree Feynman
//    diagrams, squared and summed over colours.  Slow; small cases only.
//  * "ordered": colour-ordered partial amplitudes A(sigma) for every ordering
//    of the gluons along the quark line (colour-ordered Berends-Giele
//    recursion), contracted with the colour matrix
//    C(sigma, tau) = sum over colours of (T..T)_ij conj((T..T)_ij), which is
//    computed numerically from explicit Gell-Mann matrices.  This is the
//    colour-flow decomposition that the paper's colour algebra uses (section
//    "Numerical stability": colour-ordered amplitudes and an integer colour
//    matrix).
//
// Conventions chosen here (free choices; the summed result does not depend on
// them): Dirac representation of the gamma matrices, helicity spinors, linear
// (real) gluon polarisation vectors.  Everything is templated on the real type
// so that an extended-precision (long double) build can arbitrate rounding.
//
// Nothing here is shared with the GPU path.

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <numeric>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

template <class R> using cx = std::complex<R>;
template <class R> using V4 = std::array<cx<R>, 4>;      // complex four-vector, upper index
template <class R> using Spinor = std::array<cx<R>, 4>;  // Dirac spinor (column or row)
template <class R> using Mat = std::array<std::array<cx<R>, 4>, 4>;

// ---------------------------------------------------------------- Dirac algebra

template <class R> struct Dirac {
  Mat<R> g[4];  // gamma^mu, Dirac representation
  Mat<R> g5;
  Dirac() {
    const cx<R> I(0, 1);
    cx<R> sig[4][2][2] = {};
    sig[0][0][0] = 1; sig[0][1][1] = 1;
    sig[1][0][1] = 1; sig[1][1][0] = 1;
    sig[2][0][1] = -I; sig[2][1][0] = I;
    sig[3][0][0] = 1; sig[3][1][1] = -1;
    for (auto& m : g) for (auto& r : m) for (auto& e : r) e = 0;
    for (auto& r : g5) for (auto& e : r) e = 0;
    // gamma^0 = diag(1, 1, -1, -1); gamma^k = [[0, sigma^k], [-sigma^k, 0]]
    for (int a = 0; a < 2; ++a) {
      g[0][a][a] = 1;
      g[0][a + 2][a + 2] = -1;
      g5[a][a + 2] = 1;  // gamma5 = [[0, 1], [1, 0]]
      g5[a + 2][a] = 1;
    }
    for (int k = 1; k <= 3; ++k)
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          g[k][a][b + 2] = sig[k][a][b];
          g[k][a + 2][b] = -sig[k][a][b];
        }
  }
};

template <class R> const Dirac<R>& dirac() {
  static const Dirac<R> d;
  return d;
}

template <class R, class A, class B> cx<R> mdot(const A& a, const B& b) {
  return cx<R>(a[0]) * cx<R>(b[0]) - cx<R>(a[1]) * cx<R>(b[1]) - cx<R>(a[2]) * cx<R>(b[2]) -
         cx<R>(a[3]) * cx<R>(b[3]);
}

// a-slash = gamma^mu a_mu = gamma^0 a^0 - gamma^k a^k
template <class R> Mat<R> slash(const V4<R>& a) {
  const Dirac<R>& d = dirac<R>();
  Mat<R> m;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      m[i][j] = d.g[0][i][j] * a[0] - d.g[1][i][j] * a[1] - d.g[2][i][j] * a[2] - d.g[3][i][j] * a[3];
  return m;
}

template <class R> Spinor<R> mat_vec(const Mat<R>& m, const Spinor<R>& v) {
  Spinor<R> r;
  for (int i = 0; i < 4; ++i) {
    r[i] = 0;
    for (int j = 0; j < 4; ++j) r[i] += m[i][j] * v[j];
  }
  return r;
}

template <class R> Spinor<R> vec_mat(const Spinor<R>& v, const Mat<R>& m) {
  Spinor<R> r;
  for (int j = 0; j < 4; ++j) {
    r[j] = 0;
    for (int i = 0; i < 4; ++i) r[j] += v[i] * m[i][j];
  }
  return r;
}

template <class R> cx<R> row_col(const Spinor<R>& a, const Spinor<R>& b) {
  cx<R> s = 0;
  for (int i = 0; i < 4; ++i) s += a[i] * b[i];
  return s;
}

// bar(psi) = psi^dagger gamma^0
template <class R> Spinor<R> dirac_bar(const Spinor<R>& s) {
  const Dirac<R>& d = dirac<R>();
  Spinor<R> c;
  for (int i = 0; i < 4; ++i) c[i] = std::conj(s[i]);
  return vec_mat(c, d.g[0]);
}

template <class R> V4<R> real4(const R* p) { return V4<R>{cx<R>(p[0]), cx<R>(p[1]), cx<R>(p[2]), cx<R>(p[3])}; }

// --------------------------------------------------------------- external states

// Two-component helicity eigenstates chi_lambda(p-hat) with (sigma . p-hat) chi = lambda chi:
// chi_+ = (cos(theta/2), e^{i phi} sin(theta/2)),  chi_- = (-e^{-i phi} sin(theta/2), cos(theta/2)).
// For p-hat exactly along -z the azimuth is taken as phi = 0.
template <class R> void helicity_chi(const R* p, int lam, cx<R> chi[2]) {
  R P = std::sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
  R ct = P > 0 ? p[3] / P : R(1);
  R c2 = std::sqrt(std::max(R(0), (1 + ct) / 2));
  R s2 = std::sqrt(std::max(R(0), (1 - ct) / 2));
  R pt = std::sqrt(p[1] * p[1] + p[2] * p[2]);
  cx<R> eph = pt > 0 ? cx<R>(p[1] / pt, p[2] / pt) : cx<R>(1, 0);
  if (lam > 0) {
    chi[0] = c2;
    chi[1] = eph * s2;
  } else {
    chi[0] = -std::conj(eph) * s2;
    chi[1] = c2;
  }
}

// Dirac-representation particle spinor u(p, lambda) = (sqrt(E+m) chi, lambda |p| / sqrt(E+m) chi).
template <class R> Spinor<R> spinor_u(const R* p, R m, int lam) {
  cx<R> chi[2];
  helicity_chi(p, lam, chi);
  R P = std::sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
  R a = std::sqrt(p[0] + m);
  R b = lam * P / a;
  return Spinor<R>{a * chi[0], a * chi[1], b * chi[0], b * chi[1]};
}

// Antiparticle spinor v(p, lambda) = gamma5 u(p, -lambda): it solves (p-slash + m) v = 0
// and sum_lambda v vbar = p-slash - m.
template <class R> Spinor<R> spinor_v(const R* p, R m, int lam) {
  return mat_vec(dirac<R>().g5, spinor_u(p, m, -lam));
}

// Linear polarisation vectors of a massless vector boson with momentum k:
// e1 = (0, cos(th) cos(ph), cos(th) sin(ph), -sin(th)), e2 = (0, -sin(ph), cos(ph), 0).
template <class R> V4<R> lin_pol(const R* k, int s) {
  R P = std::sqrt(k[1] * k[1] + k[2] * k[2] + k[3] * k[3]);
  R pt = std::sqrt(k[1] * k[1] + k[2] * k[2]);
  R ct = k[3] / P, st = pt / P;
  R cp = pt > 0 ? k[1] / pt : R(1), sp = pt > 0 ? k[2] / pt : R(0);
  if (s == 0) return V4<R>{cx<R>(0), cx<R>(ct * cp), cx<R>(ct * sp), cx<R>(-st)};
  return V4<R>{cx<R>(0), cx<R>(-sp), cx<R>(cp), cx<R>(0)};
}

// Helicity polarisation of a massless vector boson with momentum k, physical helicity lam:
// (e1 + i lam e2) / sqrt(2) up to a phase (e1, e2, k-hat right-handed), conjugated for an
// outgoing boson.  |M_h|^2 of one helicity configuration does not depend on the phases.
template <class R> V4<R> hel_pol(const R* k, int lam, bool outgoing) {
  const V4<R> e1 = lin_pol(k, 0), e2 = lin_pol(k, 1);
  const cx<R> c(0, outgoing ? -R(lam) : R(lam));
  const R r = 1 / std::sqrt(R(2));
  V4<R> e;
  for (int mu = 0; mu < 4; ++mu) e[mu] = (e1[mu] + c * e2[mu]) * r;
  return e;
}

// -------------------------------------------------------------------- SU(3)

template <class R> struct SU3 {
  cx<R> T[8][3][3];  // T^a = lambda^a / 2, Gell-Mann matrices
  R f[8][8][8];      // structure constants, [T^a, T^b] = i f^{abc} T^c
  SU3() {
    const cx<R> I(0, 1);
    cx<R> l[8][3][3] = {};
    l[0][0][1] = 1; l[0][1][0] = 1;
    l[1][0][1] = -I; l[1][1][0] = I;
    l[2][0][0] = 1; l[2][1][1] = -1;
    l[3][0][2] = 1; l[3][2][0] = 1;
    l[4][0][2] = -I; l[4][2][0] = I;
    l[5][1][2] = 1; l[5][2][1] = 1;
    l[6][1][2] = -I; l[6][2][1] = I;
    R r3 = 1 / std::sqrt(R(3));
    l[7][0][0] = r3; l[7][1][1] = r3; l[7][2][2] = -2 * r3;
    for (int a = 0; a < 8; ++a)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) T[a][i][j] = l[a][i][j] / R(2);
    // f^{abc} = -2 i Tr([T^a, T^b] T^c)
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b)
        for (int c = 0; c < 8; ++c) {
          cx<R> tr = 0;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
              for (int k = 0; k < 3; ++k)
                tr += (T[a][i][j] * T[b][j][k] - T[b][i][j] * T[a][j][k]) * T[c][k][i];
          R v = (cx<R>(0, -2) * tr).real();
          f[a][b][c] = std::abs(v) < R(1e-12) ? R(0) : v;
        }
  }
};

template <class R> const SU3<R>& su3() {
  static const SU3<R> s;
  return s;
}

// ------------------------------------------------------------------ the card

template <class R> struct Couplings {
  R mZ, wZ, e, sw2, cw2, mT;
};

// Electroweak inputs (mZ, alpha, G_F): mW^2 = mZ^2/2 + sqrt(mZ^4/4 - pi alpha mZ^2 / (sqrt(2) G_F)),
// sin^2(theta_W) = 1 - mW^2 / mZ^2, e = sqrt(4 pi alpha).
template <class R> Couplings<R> make_couplings(const double* card) {
  Couplings<R> c;
  c.mZ = card[0];
  c.wZ = card[1];
  R alpha = R(1) / R(card[2]);
  R Gf = card[3];
  R pi = std::acos(R(-1));
  R mZ2 = c.mZ * c.mZ;
  R mW2 = mZ2 / 2 + std::sqrt(mZ2 * mZ2 / 4 - pi * alpha * mZ2 / (std::sqrt(R(2)) * Gf));
  c.cw2 = mW2 / mZ2;
  c.sw2 = 1 - c.cw2;
  c.e = std::sqrt(4 * pi * alpha);
  c.mT = card[4];
  return c;
}

// --------------------------------------------------- e+ e- -> mu+ mu- (2 diagrams)

// Particles: 1 e+ (incoming), 2 e- (incoming), 3 mu+ (outgoing), 4 mu- (outgoing).
// Vertices from L = -e Q psibar A-slash psi - e/(sw cw) psibar Z-slash (T3 P_L - Q sw^2) psi, Q = -1.
// per_hel (optional): |M_h|^2 / 4 of each helicity configuration, index sum_k [h_k = +1] 2^(3 - k).
template <class R> R me2_eemumu(const R* mom, const Couplings<R>& cp, R* per_hel = nullptr) {
  const Dirac<R>& d = dirac<R>();
  const cx<R> I(0, 1);
  const R* p1 = mom;
  const R* p2 = mom + 4;
  const R* p3 = mom + 8;
  const R* p4 = mom + 12;
  R gL = R(-0.5) + cp.sw2, gR = cp.sw2;
  R gz = cp.e / std::sqrt(cp.sw2 * cp.cw2);
  Mat<R> PL, PR;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cx<R> id = (i == j) ? cx<R>(1) : cx<R>(0);
      PL[i][j] = (id - d.g5[i][j]) / R(2);
      PR[i][j] = (id + d.g5[i][j]) / R(2);
    }
  // vertex matrices Gamma^mu for the photon and the Z
  Mat<R> Vg[4], Vz[4];
  for (int mu = 0; mu < 4; ++mu)
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        Vg[mu][i][j] = I * cp.e * d.g[mu][i][j];  // -i e Q gamma^mu with Q = -1
        cx<R> gLR = 0;
        for (int k = 0; k < 4; ++k) gLR += d.g[mu][i][k] * (gL * PL[k][j] + gR * PR[k][j]);
        Vz[mu][i][j] = -I * gz * gLR;
      }
  R q[4];
  for (int mu = 0; mu < 4; ++mu) q[mu] = p1[mu] + p2[mu];
  R s = q[0] * q[0] - q[1] * q[1] - q[2] * q[2] - q[3] * q[3];
  cx<R> dz = cx<R>(s - cp.mZ * cp.mZ, cp.mZ * cp.wZ);
  const R metric[4] = {1, -1, -1, -1};
  R sum = 0;
  for (int h1 = -1; h1 <= 1; h1 += 2)
    for (int h2 = -1; h2 <= 1; h2 += 2)
      for (int h3 = -1; h3 <= 1; h3 += 2)
        for (int h4 = -1; h4 <= 1; h4 += 2) {
          Spinor<R> vb1 = dirac_bar(spinor_v(p1, R(0), h1));  // incoming e+
          Spinor<R> u2 = spinor_u(p2, R(0), h2);             // incoming e-
          Spinor<R> v3 = spinor_v(p3, R(0), h3);             // outgoing mu+
          Spinor<R> ub4 = dirac_bar(spinor_u(p4, R(0), h4));  // outgoing mu-
          // currents with an upper Lorentz index
          cx<R> jeg[4], jez[4], jmg[4], jmz[4];
          for (int mu = 0; mu < 4; ++mu) {
            jeg[mu] = row_col(vb1, mat_vec(Vg[mu], u2));
            jez[mu] = row_col(vb1, mat_vec(Vz[mu], u2));
            jmg[mu] = row_col(ub4, mat_vec(Vg[mu], v3));
            jmz[mu] = row_col(ub4, mat_vec(Vz[mu], v3));
          }
          // photon propagator -i g_{mu nu} / s
          cx<R> amp = 0;
          for (int mu = 0; mu < 4; ++mu) amp += -I * jmg[mu] * metric[mu] * jeg[mu] / s;
          // Z propagator -i (g_{mu nu} - q_mu q_nu / mZ^2) / (s - mZ^2 + i mZ wZ)
          cx<R> gg = 0, qm = 0, qe = 0;
          for (int mu = 0; mu < 4; ++mu) {
            gg += jmz[mu] * metric[mu] * jez[mu];
            qm += jmz[mu] * metric[mu] * q[mu];
            qe += jez[mu] * metric[mu] * q[mu];
          }
          amp += -I * (gg - qm * qe / (cp.mZ * cp.mZ)) / dz;
          sum += std::norm(amp);
          if (per_hel) per_hel[((h1 > 0) << 3) | ((h2 > 0) << 2) | ((h3 > 0) << 1) | (h4 > 0)] = std::norm(amp) / 4;
        }
  return sum / 4;  // average over the 2 x 2 initial helicities
}

// ------------------------------------------- QCD building blocks (shared by both evaluations)

// Three-gluon vertex with all momenta incoming, legs (mu, k), (nu, p), (rho, q):
// V^{mu nu rho} = g^{mu nu} (k - p)^rho + g^{nu rho} (p - q)^mu + g^{rho mu} (q - k)^nu.
// Contracted with the two vectors a (leg mu) and b (leg nu); returns the open upper index rho.
template <class R> V4<R> vertex3(const V4<R>& a, const R* k, const V4<R>& b, const R* p) {
  R q[4];
  for (int i = 0; i < 4; ++i) q[i] = -(k[i] + p[i]);
  R kmp[4], pmq[4], qmk[4];
  for (int i = 0; i < 4; ++i) {
    kmp[i] = k[i] - p[i];
    pmq[i] = p[i] - q[i];
    qmk[i] = q[i] - k[i];
  }
  cx<R> ab = mdot<R>(a, b), pa = mdot<R>(pmq, a), qb = mdot<R>(qmk, b);
  V4<R> r;
  for (int i = 0; i < 4; ++i) r[i] = ab * kmp[i] + b[i] * pa + a[i] * qb;
  return r;
}

// The three Lorentz structures of the four-gluon vertex with legs (mu, nu, rho, sigma) = (a, b, c, open):
// L1 = g^{mu rho} g^{nu sigma} - g^{mu sigma} g^{nu rho}
// L2 = g^{mu nu} g^{rho sigma} - g^{mu sigma} g^{nu rho}
// L3 = g^{mu nu} g^{rho sigma} - g^{mu rho} g^{nu sigma}
template <class R> void vertex4(const V4<R>& a, const V4<R>& b, const V4<R>& c, V4<R> L[3]) {
  cx<R> ab = mdot<R>(a, b), ac = mdot<R>(a, c), bc = mdot<R>(b, c);
  for (int i = 0; i < 4; ++i) {
    L[0][i] = ac * b[i] - bc * a[i];
    L[1][i] = ab * c[i] - bc * a[i];
    L[2][i] = ab * c[i] - ac * b[i];
  }
}

// External data of one QCD configuration: gluons 0..n-1 with incoming momenta q and
// polarisation vectors eps; quark line ubar(p3) ... v(p4).
template <class R> struct QcdLegs {
  int n;
  R q[8][4];     // incoming momenta of the gluons
  V4<R> eps[8];  // gluon polarisations (conjugated for outgoing gluons)
  R q3[4], q4[4];
  Spinor<R> ubar3, v4;
  R mT;
};

// ------------------------------------------- colour-ordered evaluation

// Colour-ordered rules: the ordered product (T^{s1} ... T^{sn})_{i j} multiplies
// A(s); reading f^{abc} T^c = -i [T^a, T^b] off the full Feynman rules gives
//   quark-gluon vertex: i gamma^mu; three-gluon vertex for the ordered pair (X, Y): -i V(Q_X, Q_Y, -Q_X-Q_Y);
//   four-gluon vertex for the ordered triple (X, Y, Z): i (2 g^{mu rho} g^{nu sigma} - g^{mu sigma} g^{nu rho} - g^{mu nu} g^{rho sigma});
//   gluon propagator -i g_{mu nu}/Q^2; quark propagator i (K-slash + m)/(K^2 - m^2),
// with the strong coupling set to 1 (every amplitude carries g_s^n).
// Returns A(perm) for the ordering `perm` of the n gluons, read from the ubar(p3) end.
template <class R> cx<R> ordered_amp(const QcdLegs<R>& L, const int* perm) {
  const int n = L.n;
  const cx<R> I(0, 1);
  // gluon currents J[a][b] for consecutive ranges a..b of the ordering
  static thread_local std::vector<V4<R>> J;
  static thread_local std::vector<std::array<R, 4>> Q;
  J.assign(n * n, V4<R>{});
  Q.assign(n * n, std::array<R, 4>{});
  auto idx = [n](int a, int b) { return a * n + b; };
  for (int a = 0; a < n; ++a) {
    J[idx(a, a)] = L.eps[perm[a]];
    for (int i = 0; i < 4; ++i) Q[idx(a, a)][i] = L.q[perm[a]][i];
  }
  for (int len = 2; len <= n; ++len)
    for (int a = 0; a + len - 1 < n; ++a) {
      int b = a + len - 1;
      auto& Qab = Q[idx(a, b)];
      for (int i = 0; i < 4; ++i) Qab[i] = Q[idx(a, a)][i] + Q[idx(a + 1, b)][i];
      V4<R> acc{};
      for (int k = a; k < b; ++k) {
        V4<R> v = vertex3(J[idx(a, k)], Q[idx(a, k)].data(), J[idx(k + 1, b)], Q[idx(k + 1, b)].data());
        for (int i = 0; i < 4; ++i) acc[i] += -I * v[i];
      }
      for (int k = a; k < b; ++k)
        for (int l = k + 1; l < b; ++l) {
          V4<R> Ls[3];
          vertex4(J[idx(a, k)], J[idx(k + 1, l)], J[idx(l + 1, b)], Ls);
          // 2 g^{mu rho} g^{nu sigma} - g^{mu sigma} g^{nu rho} - g^{mu nu} g^{rho sigma} = L1 - L3
          for (int i = 0; i < 4; ++i) acc[i] += I * (Ls[0][i] - Ls[2][i]);
        }
      R Q2 = Qab[0] * Qab[0] - Qab[1] * Qab[1] - Qab[2] * Qab[2] - Qab[3] * Qab[3];
      for (int i = 0; i < 4; ++i) J[idx(a, b)][i] = -I * acc[i] / Q2;
    }
  // quark currents psi[k] carry gluons perm[k..n-1] attached to v(p4)
  static thread_local std::vector<Spinor<R>> psi;
  psi.assign(n + 1, Spinor<R>{});
  psi[n] = L.v4;
  for (int k = n - 1; k >= 1; --k) {
    R K[4];
    for (int i = 0; i < 4; ++i) K[i] = L.q4[i] + Q[idx(k, n - 1)][i];
    Spinor<R> acc{};
    for (int j = k; j < n; ++j) {
      Spinor<R> t = mat_vec(slash(J[idx(k, j)]), psi[j + 1]);
      for (int i = 0; i < 4; ++i) acc[i] += I * t[i];
    }
    V4<R> Kc = real4<R>(K);
    Mat<R> prop = slash(Kc);
    for (int i = 0; i < 4; ++i) prop[i][i] += L.mT;
    R den = K[0] * K[0] - K[1] * K[1] - K[2] * K[2] - K[3] * K[3] - L.mT * L.mT;
    Spinor<R> t = mat_vec(prop, acc);
    for (int i = 0; i < 4; ++i) psi[k][i] = I * t[i] / den;
  }
  cx<R> amp = 0;
  for (int j = 0; j < n; ++j) amp += I * row_col(L.ubar3, mat_vec(slash(J[idx(0, j)]), psi[j + 1]));
  return amp;
}

// Colour matrix C(s, t) = sum over a_1..a_n, i, j of (T^{a_s1} .. T^{a_sn})_{ij} conj((T^{a_t1} .. T^{a_tn})_{ij})
// for all orderings s, t of n gluons (lexicographic order), by explicit summation.
template <class R> std::vector<R> colour_matrix_numeric(int n) {
  const SU3<R>& S = su3<R>();
  std::vector<std::vector<int>> perms;
  std::vector<int> p(n);
  std::iota(p.begin(), p.end(), 0);
  do perms.push_back(p); while (std::next_permutation(p.begin(), p.end()));
  const int np = (int)perms.size();
  long ntup = 1;
  for (int i = 0; i < n; ++i) ntup *= 8;
  // X[s][tuple] = 3x3 matrix product
  std::vector<cx<R>> X((size_t)np * ntup * 9);
#pragma omp parallel for schedule(static)
  for (long t = 0; t < ntup; ++t) {
    int a[8];
    long r = t;
    for (int i = 0; i < n; ++i) { a[i] = r % 8; r /= 8; }
    for (int s = 0; s < np; ++s) {
      cx<R> m[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) m[i][j] = S.T[a[perms[s][0]]][i][j];
      for (int k = 1; k < n; ++k) {
        cx<R> nm[3][3];
        const auto& Tk = S.T[a[perms[s][k]]];
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            nm[i][j] = 0;
            for (int l = 0; l < 3; ++l) nm[i][j] += m[i][l] * Tk[l][j];
          }
        std::memcpy(m, nm, sizeof m);
      }
      cx<R>* dst = &X[((size_t)s * ntup + t) * 9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) dst[i * 3 + j] = m[i][j];
    }
  }
  std::vector<R> C((size_t)np * np);
#pragma omp parallel for schedule(dynamic)
  for (int s = 0; s < np; ++s)
    for (int t = 0; t < np; ++t) {
      cx<R> acc = 0;
      const cx<R>* xs = &X[(size_t)s * ntup * 9];
      const cx<R>* xt = &X[(size_t)t * ntup * 9];
      for (long k = 0; k < ntup * 9; ++k) acc += xs[k] * std::conj(xt[k]);
      C[(size_t)s * np + t] = acc.real();
    }
  return C;
}

// The sums above run over 8^n terms with cancellations, so they are always
// accumulated in long double and then rounded to the requested type.
template <class R> const std::vector<R>& colour_matrix_cached(int n) {
  static std::mutex mu;
  static std::vector<R> cache[8];
  std::lock_guard<std::mutex> lock(mu);
  if (cache[n].empty()) {
    std::vector<long double> c = colour_matrix_numeric<long double>(n);
    cache[n].assign(c.begin(), c.end());
  }
  return cache[n];
}

// ------------------------------------------- colour-dressed evaluation

// Colour-dressed Berends-Giele recursion with explicit colour indices.  Gluon
// currents J^a(S) for subsets S of the gluons, quark currents psi_i(S) attached
// to v(p4).  Full Feynman rules (strong coupling set to 1):
//   q-qbar-g: i gamma^mu T^a_{ij};  ggg: f^{abc} V^{mu nu rho}(k, p, q);
//   gggg: -i [f^{abe} f^{cde} L1 + f^{ace} f^{bde} L2 + f^{ade} f^{bce} L3];
//   gluon propagator -i delta^{ab} g_{mu nu}/Q^2; quark propagator i (K-slash + m)/(K^2 - m^2).
// Every Feynman diagram appears once: gluon subsets are split into unordered
// parts, and the quark line is closed at the vertex next to ubar(p3).
template <class R> struct Dressed {
  int n;
  std::vector<std::array<V4<R>, 8>> J;  // [mask][colour]
  std::vector<std::array<bool, 8>> Jnz;
  std::vector<std::array<R, 4>> Q;

  // vertex sums at subset `mask` (before the propagator), result acc[colour of the open leg]
  void vertex_sum(int mask, std::array<V4<R>, 8>& acc) const {
    const SU3<R>& S = su3<R>();
    const cx<R> I(0, 1);
    for (auto& v : acc) v = V4<R>{};
    const int low = mask & -mask;
    // three-gluon vertex, unordered splits {S1, S2} with S1 holding the lowest gluon
    for (int s1 = (mask - 1) & mask; s1 > 0; s1 = (s1 - 1) & mask) {
      if (!(s1 & low)) continue;
      int s2 = mask ^ s1;
      for (int b = 0; b < 8; ++b) {
        if (!Jnz[s1][b]) continue;
        for (int c = 0; c < 8; ++c) {
          if (!Jnz[s2][c]) continue;
          V4<R> v = vertex3(J[s1][b], Q[s1].data(), J[s2][c], Q[s2].data());
          for (int e = 0; e < 8; ++e) {
            R f = S.f[b][c][e];
            if (f == 0) continue;
            for (int i = 0; i < 4; ++i) acc[e][i] += f * v[i];
          }
        }
      }
    }
    // four-gluon vertex, unordered triples {S1, S2, S3}
    for (int s1 = (mask - 1) & mask; s1 > 0; s1 = (s1 - 1) & mask) {
      if (!(s1 & low)) continue;
      int rest = mask ^ s1;
      int low2 = rest & -rest;
      for (int s2 = (rest - 1) & rest; s2 > 0; s2 = (s2 - 1) & rest) {
        if (!(s2 & low2)) continue;
        int s3 = rest ^ s2;
        for (int b = 0; b < 8; ++b) {
          if (!Jnz[s1][b]) continue;
          for (int c = 0; c < 8; ++c) {
            if (!Jnz[s2][c]) continue;
            for (int d = 0; d < 8; ++d) {
              if (!Jnz[s3][d]) continue;
              V4<R> Ls[3];
              vertex4(J[s1][b], J[s2][c], J[s3][d], Ls);
              for (int r = 0; r < 8; ++r) {
                R c1 = 0, c2 = 0, c3 = 0;
                for (int e = 0; e < 8; ++e) {
                  c1 += S.f[b][c][e] * S.f[d][r][e];
                  c2 += S.f[b][d][e] * S.f[c][r][e];
                  c3 += S.f[b][r][e] * S.f[c][d][e];
                }
                if (c1 == 0 && c2 == 0 && c3 == 0) continue;
                for (int i = 0; i < 4; ++i) acc[r][i] += -I * (c1 * Ls[0][i] + c2 * Ls[1][i] + c3 * Ls[2][i]);
              }
            }
          }
        }
      }
    }
  }

  // fill gluon currents for every subset of `upto` (a bitmask) given external colours
  void gluon_currents(const QcdLegs<R>& L, const int* col, int upto) {
    n = L.n;
    const cx<R> I(0, 1);
    J.assign(1 << n, {});
    Jnz.assign(1 << n, {});
    Q.assign(1 << n, {});
    for (int k = 0; k < n; ++k) {
      int m = 1 << k;
      J[m][col[k]] = L.eps[k];
      Jnz[m][col[k]] = true;
      for (int i = 0; i < 4; ++i) Q[m][i] = L.q[k][i];
    }
    std::vector<int> masks;
    for (int m = 1; m < (1 << n); ++m)
      if ((m & upto) == m && __builtin_popcount(m) >= 2) masks.push_back(m);
    std::stable_sort(masks.begin(), masks.end(),
                     [](int a, int b) { return __builtin_popcount(a) < __builtin_popcount(b); });
    for (int m : masks) {
      int low = m & -m;
      for (int i = 0; i < 4; ++i) Q[m][i] = Q[low][i] + Q[m ^ low][i];
      std::array<V4<R>, 8> acc;
      vertex_sum(m, acc);
      R Q2 = Q[m][0] * Q[m][0] - Q[m][1] * Q[m][1] - Q[m][2] * Q[m][2] - Q[m][3] * Q[m][3];
      for (int a = 0; a < 8; ++a) {
        bool nz = false;
        for (int i = 0; i < 4; ++i) {
          J[m][a][i] = -I * acc[a][i] / Q2;
          nz = nz || acc[a][i] != cx<R>(0);
        }
        Jnz[m][a] = nz;
      }
    }
  }
};

// Full amplitude of g...g -> t tbar for given gluon colours col[], returns A[i3] for the
// three colours of the top, with the antitop colour j4 fixed.
template <class R> void dressed_amp_tt(const QcdLegs<R>& L, const int* col, int j4, cx<R> out[3],
                                       Dressed<R>& D) {
  const SU3<R>& S = su3<R>();
  const cx<R> I(0, 1);
  const int n = L.n, all = (1 << n) - 1;
  D.gluon_currents(L, col, all);
  // quark currents for every proper subset
  std::vector<std::array<Spinor<R>, 3>> psi(1 << n);
  std::vector<std::array<bool, 3>> pnz(1 << n);
  for (int i = 0; i < 3; ++i) {
    psi[0][i] = (i == j4) ? L.v4 : Spinor<R>{};
    pnz[0][i] = (i == j4);
  }
  std::vector<int> masks;
  for (int m = 1; m < all; ++m) masks.push_back(m);
  std::stable_sort(masks.begin(), masks.end(),
                   [](int a, int b) { return __builtin_popcount(a) < __builtin_popcount(b); });
  // vertex i gamma^mu T^a_{ij} J^a_mu psi_j(rest), summed over the gluon subset S1 at the vertex
  auto attach = [&](int mask, std::array<Spinor<R>, 3>& acc, std::array<bool, 3>& nz) {
    for (auto& s : acc) s = Spinor<R>{};
    nz = {false, false, false};
    for (int s1 = mask; s1 > 0; s1 = (s1 - 1) & mask) {
      int s2 = mask ^ s1;
      for (int a = 0; a < 8; ++a) {
        if (!D.Jnz[s1][a]) continue;
        Mat<R> js = slash(D.J[s1][a]);
        for (int j = 0; j < 3; ++j) {
          if (!pnz[s2][j]) continue;
          Spinor<R> t = mat_vec(js, psi[s2][j]);
          for (int i = 0; i < 3; ++i) {
            cx<R> tij = S.T[a][i][j];
            if (tij == cx<R>(0)) continue;
            for (int k = 0; k < 4; ++k) acc[i][k] += I * tij * t[k];
            nz[i] = true;
          }
        }
      }
    }
  };
  for (int m : masks) {
    R K[4] = {L.q4[0], L.q4[1], L.q4[2], L.q4[3]};
    for (int k = 0; k < n; ++k)
      if (m >> k & 1)
        for (int i = 0; i < 4; ++i) K[i] += L.q[k][i];
    std::array<Spinor<R>, 3> acc;
    std::array<bool, 3> nz;
    attach(m, acc, nz);
    V4<R> Kc = real4<R>(K);
    Mat<R> prop = slash(Kc);
    for (int i = 0; i < 4; ++i) prop[i][i] += L.mT;
    R den = K[0] * K[0] - K[1] * K[1] - K[2] * K[2] - K[3] * K[3] - L.mT * L.mT;
    for (int i = 0; i < 3; ++i) {
      pnz[m][i] = nz[i];
      if (!nz[i]) { psi[m][i] = Spinor<R>{}; continue; }
      Spinor<R> t = mat_vec(prop, acc[i]);
      for (int k = 0; k < 4; ++k) psi[m][i][k] = I * t[k] / den;
    }
  }
  // close at the vertex next to ubar(p3)
  std::array<Spinor<R>, 3> acc;
  std::array<bool, 3> nz;
  attach(all, acc, nz);
  for (int i = 0; i < 3; ++i) out[i] = nz[i] ? row_col(L.ubar3, acc[i]) : cx<R>(0);
}

// Pure-gluon amplitude: close the recursion on the last gluon.
template <class R> cx<R> dressed_amp_gluons(const QcdLegs<R>& L, const int* col, Dressed<R>& D) {
  const int n = L.n, last = n - 1, rest = (1 << last) - 1;
  D.gluon_currents(L, col, rest);
  std::array<V4<R>, 8> acc;
  D.vertex_sum(rest, acc);
  return mdot<R>(acc[col[last]], L.eps[last]);
}

// ------------------------------------------- u ubar -> e+ e- + n g (Drell-Yan family)

// Particles: 0 u (incoming), 1 ubar (incoming), 2 e+ (outgoing), 3 e- (outgoing), 4.. gluons
// (outgoing).  The quark line runs from vbar(p_ubar) to u(p_u); the gluons and one electroweak
// boson (photon or Z, s-channel, decaying to the lepton pair) attach to it.  Feynman rules with
// the strong coupling set to 1 (every amplitude carries g_s^n):
//   photon: vertex -i e Q gamma^mu (Q_u = 2/3, Q_e = -1), propagator -i g_{mu nu} / q^2;
//   Z: vertex -i (e / (sw cw)) gamma^mu (gL P_L + gR P_R), gL = T3 - Q sw^2, gR = -Q sw^2
//      (u: T3 = 1/2; e: T3 = -1/2), propagator -i (g_{mu nu} - q_mu q_nu / mZ^2) / (q^2 - mZ^2 + i mZ wZ);
//   quark-gluon vertex and gluon interactions as in the colour-ordered and colour-dressed
//   evaluations above; massless quark propagator i K-slash / K^2.
template <class R> struct DyLegs {
  int n;
  R q[8][4];     // incoming momenta of the gluons (outgoing ones negated)
  V4<R> eps[8];  // gluon polarisations (real linear ones, or conjugated circular ones)
  R p1[4];       // u momentum (incoming)
  R qv[4];       // momentum of the electroweak boson, p_e+ + p_e- (outgoing)
  Spinor<R> u1, vbar2;
  Mat<R> ew;  // the boson insertion as a matrix on the quark line: quark vertex x propagator x lepton current
};

// The electroweak insertion for given lepton spinors: sum over photon and Z of
// Gamma_q^nu P_{nu mu} L^mu with the lepton current L^mu = ubar(e-) Gamma_e^mu v(e+).
template <class R> Mat<R> dy_insertion(const Couplings<R>& cp, const Spinor<R>& v_ep, const Spinor<R>& ubar_em,
                                       const R* qv) {
  const Dirac<R>& d = dirac<R>();
  const cx<R> I(0, 1);
  const R metric[4] = {1, -1, -1, -1};
  const R Qu = R(2) / R(3), Qe = -1;
  const R gLu = R(0.5) - Qu * cp.sw2, gRu = -Qu * cp.sw2;
  const R gLe = R(-0.5) - Qe * cp.sw2, gRe = -Qe * cp.sw2;
  const R gz = cp.e / std::sqrt(cp.sw2 * cp.cw2);
  Mat<R> PL, PR;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      const cx<R> id = (i == j) ? cx<R>(1) : cx<R>(0);
      PL[i][j] = (id - d.g5[i][j]) / R(2);
      PR[i][j] = (id + d.g5[i][j]) / R(2);
    }
  // vertex matrices Gamma^mu of the photon and the Z for a fermion of the given couplings
  auto vertex = [&](int mu, bool z, R Q, R gL, R gR) {
    Mat<R> m;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        if (!z) {
          m[i][j] = -I * cp.e * Q * d.g[mu][i][j];
        } else {
          cx<R> t = 0;
          for (int k = 0; k < 4; ++k) t += d.g[mu][i][k] * (gL * PL[k][j] + gR * PR[k][j]);
          m[i][j] = -I * gz * t;
        }
      }
    return m;
  };
  const R s = qv[0] * qv[0] - qv[1] * qv[1] - qv[2] * qv[2] - qv[3] * qv[3];
  const cx<R> dz(s - cp.mZ * cp.mZ, cp.mZ * cp.wZ);
  Mat<R> out;
  for (auto& r : out)
    for (auto& e : r) e = 0;
  for (int z = 0; z < 2; ++z) {
    // lepton current with an upper index
    cx<R> L[4];
    for (int mu = 0; mu < 4; ++mu)
      L[mu] = row_col(ubar_em, mat_vec(vertex(mu, z, Qe, gLe, gRe), v_ep));
    // propagator times current, lower index: P_{nu mu} L^mu
    cx<R> PLow[4];
    cx<R> qL = 0;
    for (int mu = 0; mu < 4; ++mu) qL += metric[mu] * qv[mu] * L[mu];
    for (int nu = 0; nu < 4; ++nu) {
      if (!z) {
        PLow[nu] = -I * metric[nu] * L[nu] / s;
      } else {
        PLow[nu] = -I * (metric[nu] * L[nu] - metric[nu] * qv[nu] * qL / (cp.mZ * cp.mZ)) / dz;
      }
    }
    for (int nu = 0; nu < 4; ++nu) {
      const Mat<R> G = vertex(nu, z, Qu, gLu, gRu);
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) out[i][j] += G[i][j] * PLow[nu];
    }
  }
  return out;
}

// External states of one spin configuration: spins[k] in {0, 1} is the helicity -1 / +1 of the
// quarks and leptons, and of the gluons the linear polarisation e1 / e2 (helicity_basis false)
// or the helicity -1 / +1 (true).  gauge_leg >= 0 replaces that gluon's polarisation by its momentum.
template <class R> DyLegs<R> dy_legs(const R* mom, int npar, const Couplings<R>& cp, const int* spins, int gauge_leg,
                                     bool helicity_basis = false) {
  DyLegs<R> L;
  L.n = npar - 4;
  for (int g = 0; g < L.n; ++g) {
    const R* p = mom + 4 * (4 + g);
    for (int i = 0; i < 4; ++i) L.q[g][i] = -p[i];
    if (g == gauge_leg) L.eps[g] = real4<R>(p);
    else if (helicity_basis) L.eps[g] = hel_pol(p, 2 * spins[4 + g] - 1, true);
    else L.eps[g] = lin_pol(p, spins[4 + g]);
  }
  for (int i = 0; i < 4; ++i) {
    L.p1[i] = mom[i];
    L.qv[i] = mom[8 + i] + mom[12 + i];
  }
  L.u1 = spinor_u(mom, R(0), 2 * spins[0] - 1);
  L.vbar2 = dirac_bar(spinor_v(mom + 4, R(0), 2 * spins[1] - 1));
  const Spinor<R> v_ep = spinor_v(mom + 8, R(0), 2 * spins[2] - 1);
  const Spinor<R> ubar_em = dirac_bar(spinor_u(mom + 12, R(0), 2 * spins[3] - 1));
  L.ew = dy_insertion(cp, v_ep, ubar_em, L.qv);
  return L;
}

// i K-slash / K^2 applied to a spinor (massless quark propagator)
template <class R> Spinor<R> massless_prop(const R* K, const Spinor<R>& x) {
  const cx<R> I(0, 1);
  const Spinor<R> t = mat_vec(slash(real4<R>(K)), x);
  const R den = K[0] * K[0] - K[1] * K[1] - K[2] * K[2] - K[3] * K[3];
  Spinor<R> r;
  for (int i = 0; i < 4; ++i) r[i] = I * t[i] / den;
  return r;
}

// Colour-ordered amplitude A(perm) of u ubar -> e+ e- + n g for the gluon ordering `perm`,
// read from the vbar(p_ubar) end: the ordered product (T^{s1} .. T^{sn})_{j i} (j the ubar
// colour, i the u colour) multiplies it.  The boson attaches anywhere between the gluon
// currents of consecutive ranges of the ordering.
template <class R> cx<R> ordered_amp_dy(const DyLegs<R>& L, const int* perm) {
  const int n = L.n;
  const cx<R> I(0, 1);
  std::vector<V4<R>> J(n * n > 0 ? n * n : 1);
  std::vector<std::array<R, 4>> Q(n * n > 0 ? n * n : 1);
  auto idx = [n](int a, int b) { return a * n + b; };
  for (int a = 0; a < n; ++a) {
    J[idx(a, a)] = L.eps[perm[a]];
    for (int i = 0; i < 4; ++i) Q[idx(a, a)][i] = L.q[perm[a]][i];
  }
  for (int len = 2; len <= n; ++len)
    for (int a = 0; a + len - 1 < n; ++a) {
      const int b = a + len - 1;
      auto& Qab = Q[idx(a, b)];
      for (int i = 0; i < 4; ++i) Qab[i] = Q[idx(a, a)][i] + Q[idx(a + 1, b)][i];
      V4<R> acc{};
      for (int k = a; k < b; ++k) {
        V4<R> v = vertex3(J[idx(a, k)], Q[idx(a, k)].data(), J[idx(k + 1, b)], Q[idx(k + 1, b)].data());
        for (int i = 0; i < 4; ++i) acc[i] += -I * v[i];
      }
      for (int k = a; k < b; ++k)
        for (int l = k + 1; l < b; ++l) {
          V4<R> Ls[3];
          vertex4(J[idx(a, k)], J[idx(k + 1, l)], J[idx(l + 1, b)], Ls);
          for (int i = 0; i < 4; ++i) acc[i] += I * (Ls[0][i] - Ls[2][i]);
        }
      const R Q2 = Qab[0] * Qab[0] - Qab[1] * Qab[1] - Qab[2] * Qab[2] - Qab[3] * Qab[3];
      for (int i = 0; i < 4; ++i) J[idx(a, b)][i] = -I * acc[i] / Q2;
    }
  // psi[k][e]: u(p_u) with the gluons perm[k..n-1] attached (and the boson if e = 1), the
  // propagator of the last attachment included (psi[n][0] is the external spinor)
  std::vector<std::array<Spinor<R>, 2>> psi(n + 1);
  for (int k = n; k >= 0; --k) {
    R K[4];
    for (int i = 0; i < 4; ++i) {
      K[i] = L.p1[i];
      for (int m = k; m < n; ++m) K[i] += L.q[perm[m]][i];
    }
    for (int e = 0; e < 2; ++e) {
      if (k == n && e == 0) {
        psi[n][0] = L.u1;
        continue;
      }
      Spinor<R> acc{};
      for (int j = k; j < n; ++j) {
        const Spinor<R> t = mat_vec(slash(J[idx(k, j)]), psi[j + 1][e]);
        for (int i = 0; i < 4; ++i) acc[i] += I * t[i];
      }
      if (e == 1) {
        const Spinor<R> t = mat_vec(L.ew, psi[k][0]);
        for (int i = 0; i < 4; ++i) acc[i] += t[i];
      }
      R Ke[4];
      for (int i = 0; i < 4; ++i) Ke[i] = K[i] - (e ? L.qv[i] : R(0));
      psi[k][e] = massless_prop(Ke, acc);
    }
  }
  // close at the vbar(p_ubar) end
  Spinor<R> acc{};
  for (int j = 0; j < n; ++j) {
    const Spinor<R> t = mat_vec(slash(J[idx(0, j)]), psi[j + 1][1]);
    for (int i = 0; i < 4; ++i) acc[i] += I * t[i];
  }
  const Spinor<R> t = mat_vec(L.ew, psi[0][0]);
  for (int i = 0; i < 4; ++i) acc[i] += t[i];
  return row_col(L.vbar2, acc);
}

// Colour-dressed amplitude of u ubar -> e+ e- + n g for gluon colours col[], u colour i1;
// out[j] for the three ubar colours j.  Every Feynman diagram with explicit generators and
// structure constants (the plain definition).
template <class R> void dressed_amp_dy(const DyLegs<R>& L, const int* col, int i1, cx<R> out[3], Dressed<R>& D) {
  const SU3<R>& S = su3<R>();
  const cx<R> I(0, 1);
  const int n = L.n, all = (1 << n) - 1;
  QcdLegs<R> G;
  G.n = n;
  for (int g = 0; g < n; ++g) {
    G.eps[g] = L.eps[g];
    for (int i = 0; i < 4; ++i) G.q[g][i] = L.q[g][i];
  }
  if (n > 0) D.gluon_currents(G, col, all);
  // psi[mask][e][colour], as in ordered_amp_dy but for subsets of the gluons
  std::vector<std::array<std::array<Spinor<R>, 3>, 2>> psi(1 << n);
  std::vector<std::array<std::array<bool, 3>, 2>> pnz(1 << n);
  std::vector<int> masks;
  for (int m = 0; m <= all; ++m) masks.push_back(m);
  std::stable_sort(masks.begin(), masks.end(),
                   [](int a, int b) { return __builtin_popcount(a) < __builtin_popcount(b); });
  // vertex i gamma^mu T^a_{jk} J^a_mu psi_k(rest) summed over the gluon subset S1 at the vertex,
  // then (e = 1) the boson insertion on psi(mask, e = 0)
  auto attach = [&](int mask, int e, std::array<Spinor<R>, 3>& acc, std::array<bool, 3>& nz) {
    for (auto& x : acc) x = Spinor<R>{};
    nz = {false, false, false};
    for (int s1 = mask; s1 > 0; s1 = (s1 - 1) & mask) {
      const int s2 = mask ^ s1;
      for (int a = 0; a < 8; ++a) {
        if (!D.Jnz[s1][a]) continue;
        const Mat<R> js = slash(D.J[s1][a]);
        for (int k = 0; k < 3; ++k) {
          if (!pnz[s2][e][k]) continue;
          const Spinor<R> t = mat_vec(js, psi[s2][e][k]);
          for (int j = 0; j < 3; ++j) {
            const cx<R> tjk = S.T[a][j][k];
            if (tjk == cx<R>(0)) continue;
            for (int c = 0; c < 4; ++c) acc[j][c] += I * tjk * t[c];
            nz[j] = true;
          }
        }
      }
    }
    if (e == 1)
      for (int j = 0; j < 3; ++j) {
        if (!pnz[mask][0][j]) continue;
        const Spinor<R> t = mat_vec(L.ew, psi[mask][0][j]);
        for (int c = 0; c < 4; ++c) acc[j][c] += t[c];
        nz[j] = true;
      }
  };
  for (int m : masks) {
    if (m == all) break;  // the full set is closed below, not propagated
    R K[4] = {L.p1[0], L.p1[1], L.p1[2], L.p1[3]};
    for (int g = 0; g < n; ++g)
      if (m >> g & 1)
        for (int i = 0; i < 4; ++i) K[i] += L.q[g][i];
    for (int e = 0; e < 2; ++e) {
      if (m == 0 && e == 0) {
        for (int j = 0; j < 3; ++j) {
          psi[0][0][j] = (j == i1) ? L.u1 : Spinor<R>{};
          pnz[0][0][j] = (j == i1);
        }
        continue;
      }
      std::array<Spinor<R>, 3> acc;
      std::array<bool, 3> nz;
      attach(m, e, acc, nz);
      R Ke[4];
      for (int i = 0; i < 4; ++i) Ke[i] = K[i] - (e ? L.qv[i] : R(0));
      for (int j = 0; j < 3; ++j) {
        pnz[m][e][j] = nz[j];
        psi[m][e][j] = nz[j] ? massless_prop(Ke, acc[j]) : Spinor<R>{};
      }
    }
  }
  if (all == 0) {
    // no gluons: the boson insertion alone between the two spinors
    for (int j = 0; j < 3; ++j) out[j] = (j == i1) ? row_col(L.vbar2, mat_vec(L.ew, L.u1)) : cx<R>(0);
    return;
  }
  // psi(all, e = 0) is needed by the closing insertion: propagate it too
  {
    R K[4] = {L.p1[0], L.p1[1], L.p1[2], L.p1[3]};
    for (int g = 0; g < n; ++g)
      for (int i = 0; i < 4; ++i) K[i] += L.q[g][i];
    std::array<Spinor<R>, 3> acc;
    std::array<bool, 3> nz;
    attach(all, 0, acc, nz);
    for (int j = 0; j < 3; ++j) {
      pnz[all][0][j] = nz[j];
      psi[all][0][j] = nz[j] ? massless_prop(K, acc[j]) : Spinor<R>{};
    }
  }
  std::array<Spinor<R>, 3> acc;
  std::array<bool, 3> nz;
  attach(all, 1, acc, nz);
  for (int j = 0; j < 3; ++j) out[j] = nz[j] ? row_col(L.vbar2, acc[j]) : cx<R>(0);
}

// sum over spins of sum over colours of |A|^2 for u ubar -> e+ e- + n g (g_s = 1):
// colour-ordered amplitudes with the colour matrix (dressed = false) or every colour
// assignment of the dressed amplitude (dressed = true)
template <class R> R spin_colour_sum_dy(const R* mom, int npar, const Couplings<R>& cp, bool dressed) {
  const int n = npar - 4;
  int spins[8];
  R total = 0;
  if (!dressed) {
    std::vector<std::vector<int>> perms;
    std::vector<int> p(n);
    std::iota(p.begin(), p.end(), 0);
    do perms.push_back(p); while (std::next_permutation(p.begin(), p.end()));
    const int np = (int)perms.size();
    // colour matrix of the quark line with n gluons (the same traces as for a top pair);
    // with no gluon the colour sum is delta_ij delta_ij = 3
    std::vector<R> C(1, R(3));
    if (n > 0) C = colour_matrix_cached<R>(n);
    std::vector<cx<R>> A(np);
    for (int cfg = 0; cfg < (1 << npar); ++cfg) {
      for (int k = 0; k < npar; ++k) spins[k] = (cfg >> k) & 1;
      const DyLegs<R> L = dy_legs(mom, npar, cp, spins, -1);
      for (int s = 0; s < np; ++s) A[s] = ordered_amp_dy(L, perms[s].data());
      for (int s = 0; s < np; ++s) {
        cx<R> row = 0;
        for (int t = 0; t < np; ++t) row += C[(size_t)s * np + t] * std::conj(A[t]);
        total += (A[s] * row).real();
      }
    }
    return total;
  }
  long ncol = 1;
  for (int i = 0; i < n; ++i) ncol *= 8;
  Dressed<R> D;
  int col[8];
  for (int cfg = 0; cfg < (1 << npar); ++cfg) {
    for (int k = 0; k < npar; ++k) spins[k] = (cfg >> k) & 1;
    const DyLegs<R> L = dy_legs(mom, npar, cp, spins, -1);
    for (long c = 0; c < ncol; ++c) {
      long r = c;
      for (int k = 0; k < n; ++k) { col[k] = r % 8; r /= 8; }
      for (int i1 = 0; i1 < 3; ++i1) {
        cx<R> a[3];
        dressed_amp_dy(L, col, i1, a, D);
        for (int j = 0; j < 3; ++j) total += std::norm(a[j]);
      }
    }
  }
  return total;
}

// ------------------------------------------- process set-up and spin sums

enum { P_EEMUMU = 0, P_GGTT = 1, P_GGTTG = 2, P_GGTTGG = 3, P_GGTTGGG = 4,
       P_UUEE = 5, P_UUEEG = 6, P_UUEEGG = 7, P_UUEEGGG = 8, P_GGGG = 9 };

bool is_dy(int proc) { return proc >= P_UUEE && proc <= P_UUEEGGG; }

int npar_of(int proc) {
  switch (proc) {
    case P_EEMUMU: return 4;
    case P_GGTT: return 4;
    case P_GGTTG: return 5;
    case P_GGTTGG: return 6;
    case P_GGTTGGG: return 7;
    case P_UUEE: return 4;
    case P_UUEEG: return 5;
    case P_UUEEGG: return 6;
    case P_UUEEGGG: return 7;
    case P_GGGG: return 4;
  }
  return -1;
}

// Averaging and symmetry factor: initial spins x initial colours x (identical final-state gluons)!
double iden_of(int proc) {
  switch (proc) {
    case P_EEMUMU: return 4;
    case P_GGTT: return 256;
    case P_GGTTG: return 256;
    case P_GGTTGG: return 512;
    case P_GGTTGGG: return 1536;
    // quark-antiquark initial state: 4 spins x 9 colours x (identical final-state gluons)!
    case P_UUEE: return 36;
    case P_UUEEG: return 36;
    case P_UUEEGG: return 72;
    case P_UUEEGGG: return 216;
    case P_GGGG: return 512;
  }
  return 0;
}

// Build the external states of g g -> t tbar + gluons for one spin configuration.
// Particles: 0, 1 incoming gluons; 2 top; 3 antitop; 4.. outgoing gluons.
// spins[k] in {0, 1}: linear polarisation index for gluons, helicity (2 s - 1) for quarks.
// spins[k] in {0, 1}: linear polarisation e1 / e2 for gluons (helicity_basis false) or helicity
// -1 / +1 (true); helicity -1 / +1 for the top and antitop.
template <class R> QcdLegs<R> qcd_legs(const R* mom, int npar, R mT, const int* spins, int gauge_leg,
                                       bool helicity_basis = false) {
  QcdLegs<R> L;
  L.mT = mT;
  L.n = npar - 2;
  int g = 0;
  for (int k = 0; k < npar; ++k) {
    if (k == 2 || k == 3) continue;
    const R* p = mom + 4 * k;
    R sgn = (k < 2) ? R(1) : R(-1);
    for (int i = 0; i < 4; ++i) L.q[g][i] = sgn * p[i];
    if (g == gauge_leg) {
      // Ward-identity check: polarisation replaced by the gluon momentum
      L.eps[g] = real4<R>(p);
    } else if (helicity_basis) {
      L.eps[g] = hel_pol(p, 2 * spins[k] - 1, k >= 2);
    } else {
      L.eps[g] = lin_pol(p, spins[k]);  // real, so conjugation for outgoing gluons is trivial
    }
    ++g;
  }
  const R* p3 = mom + 8;
  const R* p4 = mom + 12;
  for (int i = 0; i < 4; ++i) {
    L.q3[i] = -p3[i];
    L.q4[i] = -p4[i];
  }
  L.ubar3 = dirac_bar(spinor_u(p3, mT, 2 * spins[2] - 1));
  L.v4 = spinor_v(p4, mT, 2 * spins[3] - 1);
  return L;
}

template <class R> QcdLegs<R> gluon_legs(const R* mom, int npar, const int* spins) {
  QcdLegs<R> L;
  L.mT = 0;
  L.n = npar;
  for (int k = 0; k < npar; ++k) {
    const R* p = mom + 4 * k;
    R sgn = (k < 2) ? R(1) : R(-1);
    for (int i = 0; i < 4; ++i) L.q[k][i] = sgn * p[i];
    L.eps[k] = lin_pol(p, spins[k]);
  }
  return L;
}

// sum over spins of sum over colours of |A|^2, colour-ordered evaluation, g_s = 1
template <class R> R spin_colour_sum_ordered(const R* mom, int npar, R mT) {
  const int n = npar - 2;
  const std::vector<R>& C = colour_matrix_cached<R>(n);
  std::vector<std::vector<int>> perms;
  std::vector<int> p(n);
  std::iota(p.begin(), p.end(), 0);
  do perms.push_back(p); while (std::next_permutation(p.begin(), p.end()));
  const int np = (int)perms.size();
  std::vector<cx<R>> A(np);
  R total = 0;
  int spins[8];
  for (int cfg = 0; cfg < (1 << npar); ++cfg) {
    for (int k = 0; k < npar; ++k) spins[k] = (cfg >> k) & 1;
    QcdLegs<R> L = qcd_legs(mom, npar, mT, spins, -1);
    for (int s = 0; s < np; ++s) A[s] = ordered_amp(L, perms[s].data());
    R m2 = 0;
    for (int s = 0; s < np; ++s) {
      cx<R> row = 0;
      for (int t = 0; t < np; ++t) row += C[(size_t)s * np + t] * std::conj(A[t]);
      m2 += (A[s] * row).real();
    }
    total += m2;
  }
  return total;
}

// sum over spins and over every external colour assignment of |A|^2, dressed evaluation, g_s = 1
template <class R> R spin_colour_sum_dressed(const R* mom, int npar, R mT, bool pure_gluon, int nthreads) {
  const int n = pure_gluon ? npar : npar - 2;
  long ncol = 1;
  for (int i = 0; i < n; ++i) ncol *= 8;
  R total = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : total)
  {
    Dressed<R> D;
    int spins[8], col[8];
#pragma omp for schedule(dynamic, 16) collapse(2)
    for (int cfg = 0; cfg < (1 << npar); ++cfg)
      for (long c = 0; c < ncol; ++c) {
        for (int k = 0; k < npar; ++k) spins[k] = (cfg >> k) & 1;
        long r = c;
        for (int k = 0; k < n; ++k) { col[k] = r % 8; r /= 8; }
        if (pure_gluon) {
          QcdLegs<R> L = gluon_legs(mom, npar, spins);
          total += std::norm(dressed_amp_gluons(L, col, D));
        } else {
          QcdLegs<R> L = qcd_legs(mom, npar, mT, spins, -1);
          for (int j4 = 0; j4 < 3; ++j4) {
            cx<R> a[3];
            dressed_amp_tt(L, col, j4, a, D);
            for (int i = 0; i < 3; ++i) total += std::norm(a[i]);
          }
        }
      }
  }
  return total;
}

template <class R> int me2_batch(int proc, const double* card, double alpha_s, int64_t nevt, const double* mom,
                                 double* out, int mode, int nthreads) {
  int npar = npar_of(proc);
  if (npar < 0 || nevt < 0 || (nevt > 0 && (!mom || !out)) || !card) return -1;
  if (proc == P_GGGG && mode != 1) return -2;  // pure gluons: dressed evaluation only
  if (nthreads <= 0) nthreads = 1;
  Couplings<R> cp = make_couplings<R>(card);
  R pi = std::acos(R(-1));
  R gs2 = 4 * pi * R(alpha_s);
  // a tree amplitude with a quark pair and n gluons carries g_s^n; with n gluons only, g_s^(n-2)
  int ngl = (proc == P_GGGG) ? 4 : npar - 2;
  int power = (proc == P_GGGG) ? ngl - 2 : ngl;
  R coup = 1;
  for (int i = 0; i < power; ++i) coup *= gs2;
  R iden = iden_of(proc);
  if (proc == P_EEMUMU) {
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 64)
    for (int64_t e = 0; e < nevt; ++e) {
      R m[16];
      for (int i = 0; i < 16; ++i) m[i] = mom[e * 16 + i];
      out[e] = (double)me2_eemumu(m, cp);
    }
    return 0;
  }
  if (is_dy(proc)) {
    // n gluons: g_s^(2n); colour-ordered (mode 0) or every colour assignment (mode 1)
    R cdy = 1;
    for (int i = 0; i < npar - 4; ++i) cdy *= gs2;
    if (mode == 0 && npar > 4) colour_matrix_cached<R>(npar - 4);
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int64_t e = 0; e < nevt; ++e) {
      R m[32];
      for (int i = 0; i < 4 * npar; ++i) m[i] = mom[e * 4 * npar + i];
      out[e] = (double)(cdy * spin_colour_sum_dy(m, npar, cp, mode == 1) / iden);
    }
    return 0;
  }
  if (mode == 0) {
    colour_matrix_cached<R>(ngl);
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int64_t e = 0; e < nevt; ++e) {
      R m[32];
      for (int i = 0; i < 4 * npar; ++i) m[i] = mom[e * 4 * npar + i];
      out[e] = (double)(coup * spin_colour_sum_ordered(m, npar, cp.mT) / iden);
    }
    return 0;
  }
  for (int64_t e = 0; e < nevt; ++e) {
    R m[32];
    for (int i = 0; i < 4 * npar; ++i) m[i] = mom[e * 4 * npar + i];
    out[e] = (double)(coup * spin_colour_sum_dressed(m, npar, cp.mT, proc == P_GGGG, nthreads) / iden);
  }
  return 0;
}

}  // namespace

// ------------------------------------------- Feynman diagrams one by one (channel weights)
//
// Every tree diagram of g g -> t tbar + n g and of u ubar -> e+ e- + n g is enumerated
// explicitly and evaluated on its own, with the colour factors stripped from the Feynman rules
// (strong coupling 1): quark-gluon vertex i gamma^mu (T^a stripped); three-gluon vertex
// V^{mu nu rho} (f^{abc} stripped); four-gluon vertex -i L_s for each of its three colour
// structures f^{abe} f^{cde}, f^{ace} f^{bde}, f^{ade} f^{bce} (so a diagram with m four-gluon
// vertices is 3^m terms); gluon propagator -i g / Q^2; quark propagator i (K-slash + m) /
// (K^2 - m^2); for Drell-Yan the electroweak insertion of the recursion above (photon and Z
// exchange together).  The colour factor of each term, from explicit generators and structure
// constants, is kept beside it, so that the sum over terms of colour x value is the amplitude
// for given colours (checked against the colour-dressed recursion).
//
// A diagram is a sequence of gluon trees along the quark line, read from the barred spinor (the
// top, or the ubar), with the electroweak boson at one position for Drell-Yan; a tree is a
// gluon, a three-gluon vertex joining two trees or a four-gluon vertex joining three (children
// unordered).  Keys name diagrams independently of the enumeration order: a gluon is g<particle
// index>, a three-gluon vertex (x,y), a four-gluon vertex [x,y,z] (children's keys sorted), the
// boson W, and a diagram its elements joined by ';' from the barred end.

struct Tree {
  int kind;  // 1 gluon, 3 or 4: vertex joining the children c
  int leaf;  // gluon index (kind 1)
  int c[3];
};

struct DiagramList {
  std::vector<Tree> pool;
  std::vector<std::vector<int>> seq;  // tree indices from the barred end; -1 is the electroweak boson
  std::vector<std::string> key;
};

const std::vector<int>& trees_over(int mask, std::vector<Tree>& pool, std::map<int, std::vector<int>>& memo) {
  auto it = memo.find(mask);
  if (it != memo.end()) return it->second;
  std::vector<int> out;
  const int low = mask & -mask;
  if (mask == low) {
    pool.push_back(Tree{1, __builtin_ctz(mask), {-1, -1, -1}});
    out.push_back((int)pool.size() - 1);
  } else {
    // unordered splits into two parts (the first holds the lowest gluon), then into three
    for (int a = (mask - 1) & mask; a > 0; a = (a - 1) & mask) {
      if (!(a & low)) continue;
      const int b = mask ^ a;
      const std::vector<int> ta = trees_over(a, pool, memo), tb = trees_over(b, pool, memo);
      for (int x : ta)
        for (int y : tb) {
          pool.push_back(Tree{3, -1, {x, y, -1}});
          out.push_back((int)pool.size() - 1);
        }
    }
    for (int a = (mask - 1) & mask; a > 0; a = (a - 1) & mask) {
      if (!(a & low)) continue;
      const int rest = mask ^ a, low2 = rest & -rest;
      for (int b = (rest - 1) & rest; b > 0; b = (b - 1) & rest) {
        if (!(b & low2)) continue;
        const int c = rest ^ b;
        const std::vector<int> ta = trees_over(a, pool, memo), tb = trees_over(b, pool, memo),
                               tc = trees_over(c, pool, memo);
        for (int x : ta)
          for (int y : tb)
            for (int z : tc) {
              pool.push_back(Tree{4, -1, {x, y, z}});
              out.push_back((int)pool.size() - 1);
            }
      }
    }
  }
  return memo[mask] = out;
}

std::string tree_key(const std::vector<Tree>& pool, int t, const int* particle) {
  const Tree& x = pool[t];
  if (x.kind == 1) return "g" + std::to_string(particle[x.leaf]);
  std::vector<std::string> k;
  for (int i = 0; i < x.kind - 1; ++i) k.push_back(tree_key(pool, x.c[i], particle));
  std::sort(k.begin(), k.end());
  std::string s = x.kind == 3 ? "(" : "[";
  for (size_t i = 0; i < k.size(); ++i) s += (i ? "," : "") + k[i];
  return s + (x.kind == 3 ? ")" : "]");
}

void ordered_partitions(int rem, std::vector<int>& cur, std::vector<std::vector<int>>& out) {
  if (!rem) {
    out.push_back(cur);
    return;
  }
  for (int s = rem; s > 0; s = (s - 1) & rem) {
    cur.push_back(s);
    ordered_partitions(rem ^ s, cur, out);
    cur.pop_back();
  }
}

// n gluons; dy: Drell-Yan (boson inserted at every position).  particle[g]: particle index of gluon g.
DiagramList enumerate_diagrams(int n, bool dy, const int* particle) {
  DiagramList D;
  std::map<int, std::vector<int>> memo;
  std::vector<std::vector<int>> parts;
  std::vector<int> cur;
  ordered_partitions((1 << n) - 1, cur, parts);
  for (const auto& blocks : parts) {
    std::vector<std::vector<int>> choice(blocks.size());
    for (size_t i = 0; i < blocks.size(); ++i) choice[i] = trees_over(blocks[i], D.pool, memo);
    std::vector<size_t> idx(blocks.size(), 0);
    while (true) {
      std::vector<int> s;
      for (size_t i = 0; i < blocks.size(); ++i) s.push_back(choice[i][idx[i]]);
      for (size_t pos = 0; pos <= (dy ? s.size() : 0); ++pos) {
        std::vector<int> q = s;
        if (dy) q.insert(q.begin() + pos, -1);
        std::string k;
        for (size_t i = 0; i < q.size(); ++i) k += (i ? ";" : "") + (q[i] < 0 ? std::string("W") : tree_key(D.pool, q[i], particle));
        D.seq.push_back(q);
        D.key.push_back(k);
      }
      size_t i = 0;
      while (i < idx.size() && ++idx[i] == choice[i].size()) idx[i++] = 0;
      if (i == idx.size()) break;
    }
  }
  return D;
}

// one term of a gluon tree: its current (propagator included; the polarisation for a gluon),
// colour vector, incoming momentum
template <class R> struct TreeTerm {
  V4<R> J;
  std::array<R, 8> C;
  std::array<R, 4> Q;
};

template <class R>
std::vector<TreeTerm<R>> tree_terms(const std::vector<Tree>& pool, int t, const V4<R>* eps, const R (*q)[4],
                                    const int* col) {
  const Tree& x = pool[t];
  const SU3<R>& S = su3<R>();
  const cx<R> I(0, 1);
  std::vector<TreeTerm<R>> out;
  if (x.kind == 1) {
    TreeTerm<R> w;
    w.J = eps[x.leaf];
    w.C.fill(0);
    w.C[col ? col[x.leaf] : 0] = 1;
    for (int i = 0; i < 4; ++i) w.Q[i] = q[x.leaf][i];
    out.push_back(w);
    return out;
  }
  std::vector<std::vector<TreeTerm<R>>> ch;
  for (int i = 0; i < x.kind - 1; ++i) ch.push_back(tree_terms(pool, x.c[i], eps, q, col));
  if (x.kind == 3) {
    for (const auto& a : ch[0])
      for (const auto& b : ch[1]) {
        TreeTerm<R> w;
        for (int i = 0; i < 4; ++i) w.Q[i] = a.Q[i] + b.Q[i];
        const R Q2 = w.Q[0] * w.Q[0] - w.Q[1] * w.Q[1] - w.Q[2] * w.Q[2] - w.Q[3] * w.Q[3];
        const V4<R> v = vertex3(a.J, a.Q.data(), b.J, b.Q.data());
        for (int i = 0; i < 4; ++i) w.J[i] = -I * v[i] / Q2;
        for (int e = 0; e < 8; ++e) {
          R c = 0;
          for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 8; ++j) c += S.f[i][j][e] * a.C[i] * b.C[j];
          w.C[e] = c;
        }
        out.push_back(w);
      }
    return out;
  }
  for (const auto& a : ch[0])
    for (const auto& b : ch[1])
      for (const auto& c : ch[2]) {
        V4<R> L[3];
        vertex4(a.J, b.J, c.J, L);
        std::array<R, 4> Qs;
        for (int i = 0; i < 4; ++i) Qs[i] = a.Q[i] + b.Q[i] + c.Q[i];
        const R Q2 = Qs[0] * Qs[0] - Qs[1] * Qs[1] - Qs[2] * Qs[2] - Qs[3] * Qs[3];
        for (int s = 0; s < 3; ++s) {
          TreeTerm<R> w;
          w.Q = Qs;
          // vertex -i L_s, propagator -i / Q^2
          for (int i = 0; i < 4; ++i) w.J[i] = -L[s][i] / Q2;
          for (int r = 0; r < 8; ++r) {
            R acc = 0;
            for (int i = 0; i < 8; ++i) {
              if (a.C[i] == 0) continue;
              for (int j = 0; j < 8; ++j) {
                if (b.C[j] == 0) continue;
                for (int k = 0; k < 8; ++k) {
                  if (c.C[k] == 0) continue;
                  R ff = 0;
                  for (int e = 0; e < 8; ++e)
                    ff += s == 0 ? S.f[i][j][e] * S.f[k][r][e]
                                 : s == 1 ? S.f[i][k][e] * S.f[j][r][e] : S.f[i][r][e] * S.f[j][k][e];
                  acc += ff * a.C[i] * b.C[j] * c.C[k];
                }
              }
            }
            w.C[r] = acc;
          }
          out.push_back(w);
        }
      }
  return out;
}

// The terms of one diagram for one spin configuration: calls f(value, colour) for every term,
// colour the 3 x 3 matrix of the quark line (rows: the barred end's colour).  tt: legs of
// g g -> t tbar + n g; dy: legs of u ubar -> e+ e- + n g (exactly one of them non-null).
template <class R, class F>
void diagram_terms(const DiagramList& D, int d, const QcdLegs<R>* tt, const DyLegs<R>* dy, const int* col, F&& f) {
  const SU3<R>& S = su3<R>();
  const cx<R> I(0, 1);
  const auto& s = D.seq[d];
  const int k = (int)s.size();
  std::vector<std::vector<TreeTerm<R>>> el(k);
  for (int i = 0; i < k; ++i)
    if (s[i] >= 0) el[i] = tt ? tree_terms(D.pool, s[i], tt->eps, tt->q, col) : tree_terms(D.pool, s[i], dy->eps, dy->q, col);
  std::vector<size_t> idx(k, 0);
  while (true) {
    // from the unbarred end: spinor, then for each element from the last to the first its
    // vertex, with a propagator between consecutive elements
    Spinor<R> psi = tt ? tt->v4 : dy->u1;
    std::array<R, 4> K;
    for (int i = 0; i < 4; ++i) K[i] = tt ? tt->q4[i] : dy->p1[i];
    std::array<std::array<cx<R>, 3>, 3> M{};  // colour of the elements to the right
    for (int a = 0; a < 3; ++a) M[a][a] = 1;
    for (int i = k - 1; i >= 0; --i) {
      if (i < k - 1) {
        // propagator with the momentum of the side toward the unbarred end
        if (tt) {
          V4<R> Kc = real4<R>(K.data());
          Mat<R> prop = slash(Kc);
          for (int a = 0; a < 4; ++a) prop[a][a] += tt->mT;
          const R den = K[0] * K[0] - K[1] * K[1] - K[2] * K[2] - K[3] * K[3] - tt->mT * tt->mT;
          const Spinor<R> t = mat_vec(prop, psi);
          for (int a = 0; a < 4; ++a) psi[a] = I * t[a] / den;
        } else {
          psi = massless_prop(K.data(), psi);
        }
      }
      if (s[i] < 0) {
        psi = mat_vec(dy->ew, psi);
        for (int a = 0; a < 4; ++a) K[a] -= dy->qv[a];
      } else {
        const TreeTerm<R>& w = el[i][idx[i]];
        const Spinor<R> t = mat_vec(slash(w.J), psi);
        for (int a = 0; a < 4; ++a) psi[a] = I * t[a];
        for (int a = 0; a < 4; ++a) K[a] += w.Q[a];
        std::array<std::array<cx<R>, 3>, 3> TM{};
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            cx<R> acc = 0;
            for (int c = 0; c < 3; ++c) {
              cx<R> tc = 0;
              for (int g = 0; g < 8; ++g) tc += w.C[g] * S.T[g][a][c];
              acc += tc * M[c][b];
            }
            TM[a][b] = acc;
          }
        M = TM;
      }
    }
    const cx<R> value = row_col(tt ? tt->ubar3 : dy->vbar2, psi);
    f(value, M);
    int i = 0;
    while (i < k && (s[i] < 0 || ++idx[i] == el[i].size())) {
      idx[i] = 0;
      ++i;
    }
    if (i == k) break;
  }
}

int diagram_setup(int proc, int& npar, bool& dy, DiagramList& D) {
  npar = npar_of(proc);
  dy = proc == P_UUEE || proc == P_UUEEG || proc == P_UUEEGG || proc == P_UUEEGGG;
  const bool tt = proc == P_GGTT || proc == P_GGTTG || proc == P_GGTTGG || proc == P_GGTTGGG;
  if (!(dy || tt)) return -1;
  const int n = dy ? npar - 4 : npar - 2;
  int particle[8];
  for (int g = 0; g < n; ++g) particle[g] = dy ? g + 4 : (g < 2 ? g : g + 2);
  D = enumerate_diagrams(n, dy, particle);
  return 0;
}

extern "C" {

// |M|^2 for nevt events, momenta [nevt][npar][4] (E, px, py, pz) in GeV.
// card = {mZ, wZ, 1/alpha, G_F, m_top, w_top}.  mode 0: colour-ordered, 1: colour-dressed.
// Returns 0 on success, negative on bad arguments.
int oracle_me2(int proc, const double* card, double alpha_s, int64_t nevt, const double* mom, double* out,
               int mode, int nthreads) {
  return me2_batch<double>(proc, card, alpha_s, nevt, mom, out, mode, nthreads);
}

// Same, evaluated in long double (x87 extended precision) and rounded to double at the end.
int oracle_me2_ld(int proc, const double* card, double alpha_s, int64_t nevt, const double* mom, double* out,
                  int mode, int nthreads) {
  return me2_batch<long double>(proc, card, alpha_s, nevt, mom, out, mode, nthreads);
}

// |M_h|^2 of each helicity configuration of one event, normalised as oracle_me2 (they sum to it):
// physical helicities (circular gluon polarisations), out[h] for h = sum_k [h_k = +1] 2^(npar-1-k),
// k = 0 .. npar-1 in particle order.  out has 2^npar entries.
int oracle_me2_hel(int proc, const double* card, double alpha_s, const double* mom, double* out) {
  const int npar = npar_of(proc);
  if (npar < 0 || proc == P_GGGG || !card || !mom || !out) return -1;
  Couplings<double> cp = make_couplings<double>(card);
  if (proc == P_EEMUMU) {
    me2_eemumu(mom, cp, out);
    return 0;
  }
  if (is_dy(proc)) {
    const double pi = std::acos(-1.0);
    const int n = npar - 4;
    double coup = 1;
    for (int i = 0; i < n; ++i) coup *= 4 * pi * alpha_s;
    std::vector<double> C(1, 3.0);
    if (n > 0) C = colour_matrix_cached<double>(n);
    std::vector<std::vector<int>> perms;
    std::vector<int> p(n);
    std::iota(p.begin(), p.end(), 0);
    do perms.push_back(p); while (std::next_permutation(p.begin(), p.end()));
    const int np = (int)perms.size();
    std::vector<cx<double>> A(np);
    int spins[8];
    for (int h = 0; h < (1 << npar); ++h) {
      for (int k = 0; k < npar; ++k) spins[k] = (h >> (npar - 1 - k)) & 1;
      const DyLegs<double> L = dy_legs(mom, npar, cp, spins, -1, true);
      for (int s = 0; s < np; ++s) A[s] = ordered_amp_dy(L, perms[s].data());
      double m2 = 0;
      for (int s = 0; s < np; ++s) {
        cx<double> row = 0;
        for (int t = 0; t < np; ++t) row += C[(size_t)s * np + t] * std::conj(A[t]);
        m2 += (A[s] * row).real();
      }
      out[h] = coup * m2 / iden_of(proc);
    }
    return 0;
  }
  const double pi = std::acos(-1.0);
  const int n = npar - 2;
  double coup = 1;
  for (int i = 0; i < n; ++i) coup *= 4 * pi * alpha_s;
  const double iden = iden_of(proc);
  const std::vector<double>& C = colour_matrix_cached<double>(n);
  std::vector<std::vector<int>> perms;
  std::vector<int> p(n);
  std::iota(p.begin(), p.end(), 0);
  do perms.push_back(p); while (std::next_permutation(p.begin(), p.end()));
  const int np = (int)perms.size();
  std::vector<cx<double>> A(np);
  int spins[8];
  for (int h = 0; h < (1 << npar); ++h) {
    for (int k = 0; k < npar; ++k) spins[k] = (h >> (npar - 1 - k)) & 1;
    QcdLegs<double> L = qcd_legs(mom, npar, cp.mT, spins, -1, true);
    for (int s = 0; s < np; ++s) A[s] = ordered_amp(L, perms[s].data());
    double m2 = 0;
    for (int s = 0; s < np; ++s) {
      cx<double> row = 0;
      for (int t = 0; t < np; ++t) row += C[(size_t)s * np + t] * std::conj(A[t]);
      m2 += (A[s] * row).real();
    }
    out[h] = coup * m2 / iden;
  }
  return 0;
}

// Colour-ordered partial amplitudes in the helicity basis (as oracle_partial_amps with circular
// gluon polarisations), spins[k] in {0, 1} for helicity -1 / +1.
int oracle_partial_amps_hel(int npar, const double* card, const double* mom, const int* spins, double* out) {
  if (npar < 4 || npar > 7 || !mom || !spins || !out) return -1;
  Couplings<double> cp = make_couplings<double>(card);
  QcdLegs<double> L = qcd_legs(mom, npar, cp.mT, spins, -1, true);
  const int n = npar - 2;
  std::vector<int> p(n);
  std::iota(p.begin(), p.end(), 0);
  int s = 0;
  do {
    cx<double> a = ordered_amp(L, p.data());
    out[2 * s] = a.real();
    out[2 * s + 1] = a.imag();
    ++s;
  } while (std::next_permutation(p.begin(), p.end()));
  return 0;
}

// Colour matrix for n gluons on a quark line, orderings in lexicographic order; out is (n!)^2.
int oracle_colour_matrix(int n, double* out) {
  if (n < 1 || n > 6 || !out) return -1;
  const std::vector<double>& C = colour_matrix_cached<double>(n);
  std::copy(C.begin(), C.end(), out);  // rounded from a long double accumulation
  return 0;
}

// Colour-ordered partial amplitudes (g_s = 1) of g g -> t tbar + gluons for one event and one spin
// configuration, orderings in lexicographic order; out = [n!][2] (re, im).  gauge_leg >= 0 replaces
// that gluon's polarisation by its momentum (Ward identity check).
int oracle_partial_amps(int npar, const double* card, const double* mom, const int* spins, int gauge_leg,
                        double* out) {
  if (npar < 4 || npar > 7 || !mom || !spins || !out) return -1;
  Couplings<double> cp = make_couplings<double>(card);
  QcdLegs<double> L = qcd_legs(mom, npar, cp.mT, spins, gauge_leg);
  const int n = npar - 2;
  std::vector<int> p(n);
  std::iota(p.begin(), p.end(), 0);
  int s = 0;
  do {
    cx<double> a = ordered_amp(L, p.data());
    out[2 * s] = a.real();
    out[2 * s + 1] = a.imag();
    ++s;
  } while (std::next_permutation(p.begin(), p.end()));
  return 0;
}

// Colour-dressed amplitude for explicit colours (g_s = 1): gluon colours col[0..n-1] in 0..7,
// top colour i3 and antitop colour j4 in 0..2.  gauge_leg as above.  Pure-gluon processes
// (pure_gluon = 1) ignore i3 and j4.
int oracle_dressed_amp(int npar, const double* card, const double* mom, const int* spins, const int* col, int i3,
                       int j4, int gauge_leg, int pure_gluon, double* out) {
  if (npar < 4 || npar > 7 || !mom || !spins || !col || !out) return -1;
  Couplings<double> cp = make_couplings<double>(card);
  Dressed<double> D;
  cx<double> a;
  if (pure_gluon) {
    QcdLegs<double> L = gluon_legs(mom, npar, spins);
    if (gauge_leg >= 0) L.eps[gauge_leg] = real4<double>(mom + 4 * gauge_leg);
    a = dressed_amp_gluons(L, col, D);
  } else {
    QcdLegs<double> L = qcd_legs(mom, npar, cp.mT, spins, gauge_leg);
    cx<double> v[3];
    dressed_amp_tt(L, col, j4, v, D);
    a = v[i3];
  }
  out[0] = a.real();
  out[1] = a.imag();
  return 0;
}

// Colour-ordered partial amplitudes (g_s = 1) of u ubar -> e+ e- + n g (npar = 4 + n) for one
// event and one spin configuration (spins[k] in {0, 1}; gluons linear e1 / e2, or helicity -1 / +1
// with helicity_basis = 1), orderings in lexicographic order; out = [n!][2].  gauge_leg >= 0
// replaces that gluon's polarisation by its momentum.
int oracle_partial_amps_dy(int npar, const double* card, const double* mom, const int* spins, int gauge_leg,
                           int helicity_basis, double* out) {
  if (npar < 4 || npar > 7 || !card || !mom || !spins || !out) return -1;
  Couplings<double> cp = make_couplings<double>(card);
  const DyLegs<double> L = dy_legs(mom, npar, cp, spins, gauge_leg, helicity_basis != 0);
  const int n = npar - 4;
  std::vector<int> p(n);
  std::iota(p.begin(), p.end(), 0);
  int s = 0;
  do {
    const cx<double> a = ordered_amp_dy(L, p.data());
    out[2 * s] = a.real();
    out[2 * s + 1] = a.imag();
    ++s;
  } while (std::next_permutation(p.begin(), p.end()));
  return 0;
}

// Colour-dressed amplitude (g_s = 1) of u ubar -> e+ e- + n g for gluon colours col[] (0..7),
// u colour i1 and ubar colour j2 (0..2), linear gluon polarisations; gauge_leg as above.
int oracle_dressed_amp_dy(int npar, const double* card, const double* mom, const int* spins, const int* col, int i1,
                          int j2, int gauge_leg, double* out) {
  if (npar < 4 || npar > 7 || !card || !mom || !spins || (!col && npar > 4) || !out || i1 < 0 || i1 > 2 || j2 < 0 ||
      j2 > 2)
    return -1;
  Couplings<double> cp = make_couplings<double>(card);
  const DyLegs<double> L = dy_legs(mom, npar, cp, spins, gauge_leg);
  Dressed<double> D;
  cx<double> a[3];
  const int none[1] = {0};
  dressed_amp_dy(L, col ? col : none, i1, a, D);
  out[0] = a[j2].real();
  out[1] = a[j2].imag();
  return 0;
}

// Diagram keys of a process (see "Feynman diagrams one by one"), joined by newlines into buf
// (cap bytes, NUL-terminated); returns the number of diagrams, or -(bytes needed) if cap is too
// small, or -1 for a process without a quark line.
int oracle_diagram_keys(int proc, char* buf, int cap) {
  int npar;
  bool dy;
  DiagramList D;
  if (diagram_setup(proc, npar, dy, D) != 0) return -1;
  std::string all;
  for (size_t d = 0; d < D.key.size(); ++d) all += (d ? "\n" : "") + D.key[d];
  if ((int)all.size() + 1 > cap) return -(int)(all.size() + 1);
  std::memcpy(buf, all.c_str(), all.size() + 1);
  return (int)D.key.size();
}

// Channel weights: out[e][d] = sum over every spin configuration and over the terms of diagram d
// of |value|^2 (colour stripped, g_s = 1, no normalisation), diagrams in the order of
// oracle_diagram_keys.  Returns 0, or -1 for a process without a quark line.
int oracle_channel_weights(int proc, const double* card, int64_t nevt, const double* mom, double* out,
                           int nthreads) {
  int npar;
  bool dy;
  DiagramList D;
  if (!card || !mom || !out || nevt < 0 || diagram_setup(proc, npar, dy, D) != 0) return -1;
  const Couplings<double> cp = make_couplings<double>(card);
  const int nd = (int)D.seq.size();
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic) num_threads(nthreads > 0 ? nthreads : 1)
#endif
  for (int64_t e = 0; e < nevt; ++e) {
    const double* p = mom + e * npar * 4;
    double* w = out + e * nd;
    for (int d = 0; d < nd; ++d) w[d] = 0;
    int spins[8];
    for (int h = 0; h < (1 << npar); ++h) {
      for (int k = 0; k < npar; ++k) spins[k] = h >> (npar - 1 - k) & 1;
      if (dy) {
        const DyLegs<double> L = dy_legs(p, npar, cp, spins, -1);
        for (int d = 0; d < nd; ++d)
          diagram_terms<double>(D, d, nullptr, &L, nullptr, [&](cx<double> v, const auto&) { w[d] += std::norm(v); });
      } else {
        const QcdLegs<double> L = qcd_legs(p, npar, cp.mT, spins, -1);
        for (int d = 0; d < nd; ++d)
          diagram_terms<double>(D, d, &L, nullptr, nullptr, [&](cx<double> v, const auto&) { w[d] += std::norm(v); });
      }
    }
  }
  return 0;
}

// Sum over every diagram and term of colour factor x value for explicit colours: gluon colours
// col[] (0..7), row colour (the top, or the ubar) and column colour (the antitop, or the u),
// spins as oracle_dressed_amp / oracle_dressed_amp_dy; out = (re, im).  Equals the colour-dressed
// amplitude.
int oracle_diagram_sum(int proc, const double* card, const double* mom, const int* spins, const int* col, int row,
                       int column, double* out) {
  int npar;
  bool dy;
  DiagramList D;
  if (!card || !mom || !spins || !out || row < 0 || row > 2 || column < 0 || column > 2 ||
      diagram_setup(proc, npar, dy, D) != 0)
    return -1;
  const Couplings<double> cp = make_couplings<double>(card);
  const int none[1] = {0};
  const int* c = col ? col : none;
  cx<double> acc = 0;
  auto add = [&](cx<double> v, const std::array<std::array<cx<double>, 3>, 3>& M) { acc += M[row][column] * v; };
  if (dy) {
    const DyLegs<double> L = dy_legs(mom, npar, cp, spins, -1);
    for (size_t d = 0; d < D.seq.size(); ++d) diagram_terms<double>(D, (int)d, nullptr, &L, c, add);
  } else {
    const QcdLegs<double> L = qcd_legs(mom, npar, cp.mT, spins, -1);
    for (size_t d = 0; d < D.seq.size(); ++d) diagram_terms<double>(D, (int)d, &L, nullptr, c, add);
  }
  out[0] = acc.real();
  out[1] = acc.imag();
  return 0;
}

// External states, for identity tests.  kind 0: u(p, lam); 1: v(p, lam); 2: ubar; 3: vbar
// (out = 4 complex); kind 4: linear polarisation vector s = lam (out = 4 complex).
int oracle_external(int kind, const double* p, double m, int lam, double* out) {
  std::array<cx<double>, 4> r;
  switch (kind) {
    case 0: r = spinor_u(p, m, lam); break;
    case 1: r = spinor_v(p, m, lam); break;
    case 2: r = dirac_bar(spinor_u(p, m, lam)); break;
    case 3: r = dirac_bar(spinor_v(p, m, lam)); break;
    case 4: r = lin_pol(p, lam); break;
    default: return -1;
  }
  for (int i = 0; i < 4; ++i) {
    out[2 * i] = r[i].real();
    out[2 * i + 1] = r[i].imag();
  }
  return 0;
}

// Gamma matrices: mu = 0..3 gives gamma^mu, mu = 5 gives gamma5; out = [4][4][2].
int oracle_gamma(int mu, double* out) {
  const Dirac<double>& d = dirac<double>();
  const Mat<double>* m = (mu >= 0 && mu < 4) ? &d.g[mu] : (mu == 5 ? &d.g5 : nullptr);
  if (!m) return -1;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      out[(i * 4 + j) * 2] = (*m)[i][j].real();
      out[(i * 4 + j) * 2 + 1] = (*m)[i][j].imag();
    }
  return 0;
}

// SU(3): T = [8][3][3][2] generators, f = [8][8][8] structure constants.
int oracle_su3(double* T, double* f) {
  const SU3<double>& S = su3<double>();
  for (int a = 0; a < 8; ++a)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T[((a * 3 + i) * 3 + j) * 2] = S.T[a][i][j].real();
        T[((a * 3 + i) * 3 + j) * 2 + 1] = S.T[a][i][j].imag();
      }
  for (int a = 0; a < 512; ++a) f[a] = (&S.f[0][0][0])[a];
  return 0;
}

// Derived electroweak parameters from the card: out = {sin^2 thetaW, cos^2 thetaW, e}.
int oracle_ew(const double* card, double* out) {
  Couplings<double> c = make_couplings<double>(card);
  out[0] = c.sw2;
  out[1] = c.cw2;
  out[2] = c.e;
  return 0;
}

int oracle_iden(int proc, double* out) {
  double v = iden_of(proc);
  if (v == 0) return -1;
  *out = v;
  return 0;
}

}  // extern "C"
