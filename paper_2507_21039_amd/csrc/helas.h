// HELAS-style wavefunction and vertex routines for gfx950, one event and one
// helicity per lane.
//
// These are the building blocks that the paper's section "Parallel scattering
// amplitudes" describes: external wavefunctions (ixxxxx / oxxxxx / vxxxxx),
// off-shell currents that merge wavefunctions through a vertex and a propagator,
// and amplitude routines that close a diagram at a final vertex.  The naming
// follows the ALOHA scheme in spirit (amplitude = "_amp" where ALOHA writes
// "_0", off-shell current = "_psi" / "_psibar" / "_vec"), but the formulas below
// are this project's own, written in the chiral (Weyl) representation
//   gamma^mu = [[0, sigma^mu], [sigmabar^mu, 0]], psi = (psi_L, psi_R),
// metric (+,-,-,-), with couplings and factors of i left to the generated code.
//
// Every function is __host__ __device__ so the generated call sequences can
// also be evaluated on the CPU in tests; the product path runs them on the GPU.
#pragma once

#include <hip/hip_runtime.h>

#define HME_FN __host__ __device__ __forceinline__

// The per-event table lives in LDS on the GPU; its pointer carries the LDS address
// space there so that reads become ds_read (on the host, for tests, it is a plain pointer).
#if defined(__HIP_DEVICE_COMPILE__)
#define HME_LDS __attribute__((address_space(3)))
#else
#define HME_LDS
#endif

namespace hme {

template <class T> struct cx {
  T r, i;
};

template <class T> HME_FN cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <class T> HME_FN cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <class T> HME_FN cx<T> operator-(cx<T> a) { return {-a.r, -a.i}; }
template <class T> HME_FN cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <class T> HME_FN cx<T> operator*(T s, cx<T> a) { return {s * a.r, s * a.i}; }
template <class T> HME_FN cx<T> mul_i(cx<T> a) { return {-a.i, a.r}; }  // i * a

// Fused multiply-adds: sums of products are written as chains of these so that each term
// after the first costs FMAs only (the vertex routines are bound by instruction issue).
HME_FN double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
HME_FN float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// acc + a b
template <class T> HME_FN cx<T> cfma(cx<T> a, cx<T> b, cx<T> acc) {
  return {fmadd(a.r, b.r, fmadd(-a.i, b.i, acc.r)), fmadd(a.r, b.i, fmadd(a.i, b.r, acc.i))};
}
// acc - a b
template <class T> HME_FN cx<T> cfms(cx<T> a, cx<T> b, cx<T> acc) {
  return {fmadd(-a.r, b.r, fmadd(a.i, b.i, acc.r)), fmadd(-a.r, b.i, fmadd(-a.i, b.r, acc.i))};
}
// acc + s a, s real
template <class T> HME_FN cx<T> rfma(T s, cx<T> a, cx<T> acc) { return {fmadd(s, a.r, acc.r), fmadd(s, a.i, acc.i)}; }
template <class T> HME_FN cx<T> conj(cx<T> a) { return {a.r, -a.i}; }
template <class T, class U> HME_FN cx<T> cast(cx<U> a) { return {T(a.r), T(a.i)}; }

// Dirac spinor (column for "_in" states, row for barred states) and vector wavefunction
// (contravariant components).
template <class T> struct sp4 {
  cx<T> c[4];
};
template <class T> struct vw4 {
  cx<T> c[4];
};

template <class T, class U> HME_FN sp4<T> cast(const sp4<U>& a) {
  return {{cast<T>(a.c[0]), cast<T>(a.c[1]), cast<T>(a.c[2]), cast<T>(a.c[3])}};
}
template <class T, class U> HME_FN vw4<T> cast(const vw4<U>& a) {
  return {{cast<T>(a.c[0]), cast<T>(a.c[1]), cast<T>(a.c[2]), cast<T>(a.c[3])}};
}

// Minkowski product of two complex vectors (bilinear, no conjugation)
template <class T> HME_FN cx<T> mdot(const vw4<T>& a, const vw4<T>& b) {
  return cfms(a.c[3], b.c[3], cfms(a.c[2], b.c[2], cfms(a.c[1], b.c[1], a.c[0] * b.c[0])));
}
// Minkowski product of a real vector with a complex vector
template <class T> HME_FN cx<T> mdot(const T* q, const vw4<T>& a) {
  return rfma(-q[3], a.c[3], rfma(-q[2], a.c[2], rfma(-q[1], a.c[1], q[0] * a.c[0])));
}

// ------------------------------------------------------------------ external states
// Momenta p = (E, px, py, pz).  lam = +1 / -1 is the helicity.

// Two-component helicity states (sigma . p-hat) chi = lam chi, normalised to 1:
// chi_+ ~ (|p| + pz, px + i py), chi_- ~ (-px + i py, |p| + pz); for p-hat = -z
// exactly, chi_+ = (0, 1) and chi_- = (-1, 0).  |p| + pz is formed without
// cancellation.
HME_FN void helicity_chi(const double* p, int lam, cx<double> chi[2]) {
  const double pt2 = p[1] * p[1] + p[2] * p[2];
  const double P = sqrt(pt2 + p[3] * p[3]);
  const double ppz = p[3] >= 0 ? P + p[3] : pt2 / (P - p[3]);
  const bool axis = ppz == 0.0;
  const double nrm = axis ? 0.0 : 1.0 / sqrt(2.0 * P * ppz);
  if (lam > 0) {
    chi[0] = {axis ? 0.0 : ppz * nrm, 0.0};
    chi[1] = {axis ? 1.0 : p[1] * nrm, axis ? 0.0 : p[2] * nrm};
  } else {
    chi[0] = {axis ? -1.0 : -p[1] * nrm, axis ? 0.0 : p[2] * nrm};
    chi[1] = {axis ? 0.0 : ppz * nrm, 0.0};
  }
}

// sqrt(E + |p|) and sqrt(E - |p|) = m / sqrt(E + |p|)
HME_FN void spinor_weights(const double* p, double m, double& wp, double& wm) {
  const double P = sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
  wp = sqrt(p[0] + P);
  wm = m == 0.0 ? 0.0 : m / wp;
}

// Flowing-in fermion: nsf = +1 gives u(p, lam) (incoming fermion),
// nsf = -1 gives v(p, lam) (outgoing antifermion).  Chiral basis:
// u = (sqrt(E - lam P) chi_lam, sqrt(E + lam P) chi_lam),
// v = (sqrt(E + lam P) chi_-lam, -sqrt(E - lam P) chi_-lam).
HME_FN sp4<double> ixxxxx(const double* p, double m, int lam, int nsf) {
  double wp, wm;
  spinor_weights(p, m, wp, wm);
  cx<double> chi[2];
  sp4<double> w;
  if (nsf > 0) {
    helicity_chi(p, lam, chi);
    const double a = lam > 0 ? wm : wp, b = lam > 0 ? wp : wm;
    w.c[0] = a * chi[0];
    w.c[1] = a * chi[1];
    w.c[2] = b * chi[0];
    w.c[3] = b * chi[1];
  } else {
    helicity_chi(p, -lam, chi);
    const double a = lam > 0 ? wp : wm, b = lam > 0 ? wm : wp;
    w.c[0] = a * chi[0];
    w.c[1] = a * chi[1];
    w.c[2] = -b * chi[0];
    w.c[3] = -b * chi[1];
  }
  return w;
}

// Flowing-out fermion (row spinor): nsf = +1 gives ubar(p, lam) (outgoing fermion),
// nsf = -1 gives vbar(p, lam) (incoming antifermion); bar(psi) = psi^dagger gamma^0,
// which swaps the chiral halves and conjugates.
HME_FN sp4<double> oxxxxx(const double* p, double m, int lam, int nsf) {
  double wp, wm;
  spinor_weights(p, m, wp, wm);
  cx<double> chi[2];
  sp4<double> w;
  if (nsf > 0) {
    helicity_chi(p, lam, chi);
    const double a = lam > 0 ? wp : wm, b = lam > 0 ? wm : wp;  // (sqrt(E+lam P), sqrt(E-lam P))
    w.c[0] = a * conj(chi[0]);
    w.c[1] = a * conj(chi[1]);
    w.c[2] = b * conj(chi[0]);
    w.c[3] = b * conj(chi[1]);
  } else {
    helicity_chi(p, -lam, chi);
    const double a = lam > 0 ? wm : wp, b = lam > 0 ? wp : wm;  // (-sqrt(E-lam P), sqrt(E+lam P))
    w.c[0] = -a * conj(chi[0]);
    w.c[1] = -a * conj(chi[1]);
    w.c[2] = b * conj(chi[0]);
    w.c[3] = b * conj(chi[1]);
  }
  return w;
}

// Massless vector boson: eps(k, lam) = (-lam e1 - i e2) / sqrt(2) with
// e1 = (0, cos(th) cos(ph), cos(th) sin(ph), -sin(th)), e2 = (0, -sin(ph), cos(ph), 0);
// nsv = -1 (incoming) returns eps, nsv = +1 (outgoing) returns conj(eps).
HME_FN vw4<double> vxxxxx(const double* k, int lam, int nsv) {
  const double pt2 = k[1] * k[1] + k[2] * k[2];
  const double pt = sqrt(pt2);
  const double P = sqrt(pt2 + k[3] * k[3]);
  const double ct = k[3] / P, st = pt / P;
  const double cp = pt > 0 ? k[1] / pt : 1.0, sp = pt > 0 ? k[2] / pt : 0.0;
  const double r = 0.70710678118654752440;  // 1/sqrt(2)
  const double a = -lam * r;
  const double b = nsv < 0 ? -r : r;  // imaginary part sign: -i e2 (incoming), +i e2 (outgoing)
  vw4<double> w;
  w.c[0] = {0.0, 0.0};
  w.c[1] = {a * ct * cp, -b * sp};
  w.c[2] = {a * ct * sp, b * cp};
  w.c[3] = {-a * st, 0.0};
  return w;
}

// ------------------------------------------------------------------ fermion-vector vertices
// Light-cone components of a vector V: vp = V0 + V3, vm = V0 - V3, vt = V1 + i V2,
// vtb = V1 - i V2, so that sigma.V = [[vm, -vtb], [-vt, vp]] and sigmabar.V = [[vp, vtb], [vt, vm]].
// The fermion vertices use V only through these.  A vector built in the kernel is converted at
// each use (vlc_of); the external gluons and the recycled currents also keep their light-cone
// form in the per-event table, so that their uses in fermion vertices start from it.  An
// external massless gluon has V0 = Im V3 = 0, so its vp = -vm is real (vlcx).
template <class T> struct vlc {
  cx<T> p, m, t, tb;
};
template <class T> struct vlcx {
  T p;
  cx<T> t, tb;
};
template <class T> HME_FN vlc<T> vlc_of(const vw4<T>& V) {
  return {V.c[0] + V.c[3], V.c[0] - V.c[3], V.c[1] + mul_i(V.c[2]), V.c[1] - mul_i(V.c[2])};
}

// Amplitude fbar V-slash f (ALOHA-style "FFV1_0").
// Grouped by the vector's components: vm (fb0 f2 + fb3 f1) + vp (fb1 f3 + fb2 f0)
// + vtb (fb2 f1 - fb0 f3) + vt (fb3 f0 - fb1 f2).
template <class T> struct ffv_bilinears {
  cx<T> p1, p2, p3, p4;
};
template <class T> HME_FN ffv_bilinears<T> ffv_amp_bilinears(const sp4<T>& fb, const sp4<T>& f) {
  return {cfma(fb.c[3], f.c[1], fb.c[0] * f.c[2]), cfma(fb.c[2], f.c[0], fb.c[1] * f.c[3]),
          cfms(fb.c[0], f.c[3], fb.c[2] * f.c[1]), cfms(fb.c[1], f.c[2], fb.c[3] * f.c[0])};
}
template <class T> HME_FN cx<T> ffv_amp(const sp4<T>& fb, const sp4<T>& f, const vlc<T>& v) {
  const ffv_bilinears<T> b = ffv_amp_bilinears(fb, f);
  return cfma(v.t, b.p4, cfma(v.tb, b.p3, cfma(v.p, b.p2, v.m * b.p1)));
}
template <class T> HME_FN cx<T> ffv_amp(const sp4<T>& fb, const sp4<T>& f, const vlcx<T>& v) {
  const ffv_bilinears<T> b = ffv_amp_bilinears(fb, f);
  return cfma(v.t, b.p4, cfma(v.tb, b.p3, rfma(v.p, b.p2, (-v.p) * b.p1)));
}
template <class T> HME_FN cx<T> ffv_amp(const sp4<T>& fb, const sp4<T>& f, const vw4<T>& V) {
  return ffv_amp(fb, f, vlc_of(V));
}

// Same with chiral couplings gamma^mu (gL P_L + gR P_R).
template <class T> HME_FN cx<T> ffvlr_amp(const sp4<T>& fb, const sp4<T>& f, const vw4<T>& V, T gL, T gR) {
  const cx<T> vp = V.c[0] + V.c[3], vm = V.c[0] - V.c[3];
  const cx<T> vt = V.c[1] + mul_i(V.c[2]), vtb = V.c[1] - mul_i(V.c[2]);
  return gR * (fb.c[0] * (vm * f.c[2] - vtb * f.c[3]) + fb.c[1] * (vp * f.c[3] - vt * f.c[2])) +
         gL * (fb.c[2] * (vp * f.c[0] + vtb * f.c[1]) + fb.c[3] * (vt * f.c[0] + vm * f.c[1]));
}

// Off-shell spinor: (K-slash + m) V-slash f * den, with K the momentum along the
// fermion arrow after the vertex and den = 1 / (K^2 - m^2).
template <class T> HME_FN sp4<T> ffv_psi(const sp4<T>& f, const vw4<T>& V, const T* K, T m, T den) {
  const cx<T> vp = V.c[0] + V.c[3], vm = V.c[0] - V.c[3];
  const cx<T> vt = V.c[1] + mul_i(V.c[2]), vtb = V.c[1] - mul_i(V.c[2]);
  const cx<T> g0 = cfms(vtb, f.c[3], vm * f.c[2]);
  const cx<T> g1 = cfms(vt, f.c[2], vp * f.c[3]);
  const cx<T> g2 = cfma(vtb, f.c[1], vp * f.c[0]);
  const cx<T> g3 = cfma(vm, f.c[1], vt * f.c[0]);
  // the propagator factor is folded into K and m
  const T kp = den * (K[0] + K[3]), km = den * (K[0] - K[3]), md = den * m;
  const cx<T> kt = {den * K[1], den * K[2]}, ktb = {kt.r, -kt.i};
  sp4<T> o;
  o.c[0] = cfms(ktb, g3, rfma(md, g0, km * g2));
  o.c[1] = cfms(kt, g2, rfma(md, g1, kp * g3));
  o.c[2] = cfma(ktb, g1, rfma(md, g2, kp * g0));
  o.c[3] = cfma(kt, g0, rfma(md, g3, km * g1));
  return o;
}

// Off-shell barred spinor: fb V-slash (K-slash + m) * den, K along the fermion arrow
// before the vertex, den = 1 / (K^2 - m^2).
template <class T> HME_FN sp4<T> ffv_psibar(const sp4<T>& fb, const vw4<T>& V, const T* K, T m, T den) {
  const cx<T> vp = V.c[0] + V.c[3], vm = V.c[0] - V.c[3];
  const cx<T> vt = V.c[1] + mul_i(V.c[2]), vtb = V.c[1] - mul_i(V.c[2]);
  const cx<T> h0 = cfma(fb.c[3], vt, fb.c[2] * vp);
  const cx<T> h1 = cfma(fb.c[3], vm, fb.c[2] * vtb);
  const cx<T> h2 = cfms(fb.c[1], vt, fb.c[0] * vm);
  const cx<T> h3 = cfms(fb.c[0], vtb, fb.c[1] * vp);
  const T kp = den * (K[0] + K[3]), km = den * (K[0] - K[3]), md = den * m;
  const cx<T> kt = {den * K[1], den * K[2]}, ktb = {kt.r, -kt.i};
  sp4<T> o;
  o.c[0] = cfma(kt, h3, rfma(md, h0, kp * h2));
  o.c[1] = cfma(ktb, h2, rfma(md, h1, km * h3));
  o.c[2] = cfms(kt, h1, rfma(md, h2, km * h0));
  o.c[3] = cfms(ktb, h0, rfma(md, h3, kp * h1));
  return o;
}

// Off-shell vector from a fermion pair through a massless propagator: J^mu = fb gamma^mu f * den.
template <class T> HME_FN vw4<T> ffv_vec(const sp4<T>& fb, const sp4<T>& f, T den) {
  vw4<T> J;
  J.c[0] = den * cfma(fb.c[3], f.c[1], cfma(fb.c[2], f.c[0], cfma(fb.c[1], f.c[3], fb.c[0] * f.c[2])));
  J.c[1] = den * cfms(fb.c[3], f.c[0], cfms(fb.c[2], f.c[1], cfma(fb.c[1], f.c[2], fb.c[0] * f.c[3])));
  J.c[2] = den * mul_i(cfms(fb.c[3], f.c[0], cfma(fb.c[2], f.c[1], cfms(fb.c[0], f.c[3], fb.c[1] * f.c[2]))));
  J.c[3] = den * cfma(fb.c[3], f.c[1], cfms(fb.c[2], f.c[0], cfms(fb.c[1], f.c[3], fb.c[0] * f.c[2])));
  return J;
}

// Off-shell massive vector (unitary gauge, fixed width) from a fermion pair with chiral couplings:
// J^mu = (j^mu - Q^mu (Q.j) / M^2) * den, j^mu = fb gamma^mu (gL P_L + gR P_R) f,
// den = 1 / (Q^2 - M^2 + i M W) (complex).
template <class T>
HME_FN vw4<T> ffvlr_vec_massive(const sp4<T>& fb, const sp4<T>& f, T gL, T gR, const T* Q, T M, cx<T> den) {
  vw4<T> j;
  j.c[0] = gR * (fb.c[0] * f.c[2] + fb.c[1] * f.c[3]) + gL * (fb.c[2] * f.c[0] + fb.c[3] * f.c[1]);
  j.c[1] = gR * (fb.c[0] * f.c[3] + fb.c[1] * f.c[2]) - gL * (fb.c[2] * f.c[1] + fb.c[3] * f.c[0]);
  j.c[2] = mul_i(gR * (fb.c[1] * f.c[2] - fb.c[0] * f.c[3]) + gL * (fb.c[2] * f.c[1] - fb.c[3] * f.c[0]));
  j.c[3] = gR * (fb.c[0] * f.c[2] - fb.c[1] * f.c[3]) - gL * (fb.c[2] * f.c[0] - fb.c[3] * f.c[1]);
  const cx<T> qj = (T(1) / (M * M)) * mdot(Q, j);
  vw4<T> J;
  for (int mu = 0; mu < 4; ++mu) J.c[mu] = den * (j.c[mu] - Q[mu] * qj);
  return J;
}

// ------------------------------------------------------------------ gluon self-couplings
// Three-vector vertex V^{mu nu rho}(k, p, q) = g^{mu nu}(k - p)^rho + g^{nu rho}(p - q)^mu + g^{rho mu}(q - k)^nu
// with all momenta incoming.

// Amplitude a_mu b_nu c_rho V^{mu nu rho}(Qa, Qb, Qc) (ALOHA-style "VVV1_0").
template <class T>
HME_FN cx<T> vvv_amp(const vw4<T>& a, const T* Qa, const vw4<T>& b, const T* Qb, const vw4<T>& c, const T* Qc) {
  T d1[4], d2[4], d3[4];
  for (int mu = 0; mu < 4; ++mu) {
    d1[mu] = Qa[mu] - Qb[mu];
    d2[mu] = Qb[mu] - Qc[mu];
    d3[mu] = Qc[mu] - Qa[mu];
  }
  return cfma(mdot(c, a), mdot(d3, b), cfma(mdot(b, c), mdot(d2, a), mdot(a, b) * mdot(d1, c)));
}

// Off-shell vector through a massless propagator (ALOHA-style "VVV1P0_1"):
// J^rho = V^{mu nu rho}(Qa, Qb, -Qa-Qb) a_mu b_nu * den
//       = [(a.b)(Qa - Qb)^rho + b^rho (Qa + 2 Qb).a - a^rho (2 Qa + Qb).b] * den.
template <class T> HME_FN vw4<T> vvv_vec(const vw4<T>& a, const T* Qa, const vw4<T>& b, const T* Qb, T den) {
  T u[4], v[4], w[4];
  for (int mu = 0; mu < 4; ++mu) {
    u[mu] = Qa[mu] - Qb[mu];
    v[mu] = Qa[mu] + 2 * Qb[mu];
    w[mu] = 2 * Qa[mu] + Qb[mu];
  }
  const cx<T> ab = den * mdot(a, b), va = den * mdot(v, a), wb = den * mdot(w, b);
  vw4<T> J;
  for (int mu = 0; mu < 4; ++mu) J.c[mu] = cfms(wb, a.c[mu], cfma(va, b.c[mu], u[mu] * ab));
  return J;
}

// Four-vector vertex structures with legs (a: mu, b: nu, c: rho, d: sigma):
//   S = 1: g^{mu rho} g^{nu sigma} - g^{mu sigma} g^{nu rho}
//   S = 2: g^{mu nu} g^{rho sigma} - g^{mu sigma} g^{nu rho}
//   S = 3: g^{mu nu} g^{rho sigma} - g^{mu rho} g^{nu sigma}
template <int S, class T> HME_FN cx<T> vvvv_amp(const vw4<T>& a, const vw4<T>& b, const vw4<T>& c, const vw4<T>& d) {
  if (S == 1) return cfms(mdot(a, d), mdot(b, c), mdot(a, c) * mdot(b, d));
  if (S == 2) return cfms(mdot(a, d), mdot(b, c), mdot(a, b) * mdot(c, d));
  return cfms(mdot(a, c), mdot(b, d), mdot(a, b) * mdot(c, d));
}

// Off-shell leg d through a massless propagator.
template <int S, class T> HME_FN vw4<T> vvvv_vec(const vw4<T>& a, const vw4<T>& b, const vw4<T>& c, T den) {
  vw4<T> J;
  if (S == 1) {
    const cx<T> x = den * mdot(a, c), y = den * mdot(b, c);
    for (int mu = 0; mu < 4; ++mu) J.c[mu] = cfms(y, a.c[mu], x * b.c[mu]);
  } else if (S == 2) {
    const cx<T> x = den * mdot(a, b), y = den * mdot(b, c);
    for (int mu = 0; mu < 4; ++mu) J.c[mu] = cfms(y, a.c[mu], x * c.c[mu]);
  } else {
    const cx<T> x = den * mdot(a, b), y = den * mdot(a, c);
    for (int mu = 0; mu < 4; ++mu) J.c[mu] = cfms(y, b.c[mu], x * c.c[mu]);
  }
  return J;
}

}  // namespace hme

namespace hme {

// Momentum sums and propagator denominators are read from the per-event table
// that the kernel keeps in LDS.  The reads are volatile so that every use loads
// the value again instead of the compiler keeping it in a register across the
// whole diagram sequence (register pressure, not LDS traffic, is the limit).
// The table holds the arithmetic type of the kernel that reads it (values are computed in
// double and rounded once when stored).
template <class S> using tab_of = const volatile HME_LDS S*;
typedef tab_of<double> tab_ptr;

template <class T> struct m4 {
  T v[4];
  HME_FN const T& operator[](int i) const { return v[i]; }
  HME_FN operator const T*() const { return v; }
};

template <class T, class S> HME_FN m4<T> qv(const volatile HME_LDS S* tab, int i) {
  return m4<T>{{T(tab[4 * i]), T(tab[4 * i + 1]), T(tab[4 * i + 2]), T(tab[4 * i + 3])}};
}

template <class T, class S> HME_FN T dv(const volatile HME_LDS S* tab, int i) { return T(tab[i]); }

}  // namespace hme

namespace hme {

// ------------------------------------------------------------------ per-event kits
// The external states of both helicities, computed once per event into the LDS table;
// each lane reads the half of its own helicity at every use (no arithmetic per use).

// Massless vector with nsv = -1 (incoming: eps) or +1 (outgoing: conj(eps)): for lam = +1
// then lam = -1 the nonzero parts (Re eps1, Re eps2, Re eps3, Im eps1, Im eps2), with
// eps(k, lam) = (-lam e1 - i e2) / sqrt(2) and e1, e2 as in vxxxxx (eps0 = Im eps3 = 0).
template <class S> HME_FN void vector_kit(const double* k, int nsv, S* kit) {
  const double pt2 = k[1] * k[1] + k[2] * k[2];
  const double pt = sqrt(pt2);
  const double P = sqrt(pt2 + k[3] * k[3]);
  const double ct = k[3] / P, st = pt / P;
  const double cp = pt > 0 ? k[1] / pt : 1.0, sp = pt > 0 ? k[2] / pt : 0.0;
  const double r = 0.70710678118654752440;
  const double e1[3] = {r * ct * cp, r * ct * sp, -r * st}, e2[2] = {-r * sp, r * cp};
  const double b = nsv < 0 ? -1.0 : 1.0;  // imaginary part: -i e2 (incoming), +i e2 (outgoing)
  for (int h = 0; h < 2; ++h) {
    const double a = h == 0 ? -1.0 : 1.0;  // -lam
    S* o = kit + 5 * h;
    o[0] = S(a * e1[0]);
    o[1] = S(a * e1[1]);
    o[2] = S(a * e1[2]);
    o[3] = S(b * e2[0]);
    o[4] = S(b * e2[1]);
  }
}

// The same states in light-cone form for the fermion vertices: for lam = +1 then lam = -1,
// (vp, Re vt, Im vt, Re vtb, Im vtb) with vp = Re eps3 = -vm (eps0 = Im eps3 = 0), formed in
// double from the kit above and rounded once.
template <class S> HME_FN void vector_lc_kit(const double* k, int nsv, S* kit) {
  double c[10];
  vector_kit(k, nsv, c);
  for (int h = 0; h < 2; ++h) {
    const double* e = c + 5 * h;  // Re eps1, Re eps2, Re eps3, Im eps1, Im eps2
    S* o = kit + 5 * h;
    o[0] = S(e[2]);
    o[1] = S(e[0] - e[4]);  // vt = eps1 + i eps2
    o[2] = S(e[3] + e[1]);
    o[3] = S(e[0] + e[4]);  // vtb = eps1 - i eps2
    o[4] = S(e[3] - e[1]);
  }
}

// Fermion states for lam = +1 then lam = -1, each 4 complex components as (re, im) pairs:
// kind 1, ubar(p, lam) of an outgoing fermion (oxxxxx with nsf = +1); kind 2, v(p, lam) of an
// outgoing antifermion (ixxxxx with nsf = -1); kind 3, vbar(p, lam) of an incoming antifermion
// (oxxxxx with nsf = -1); kind 4, u(p, lam) of an incoming fermion (ixxxxx with nsf = +1).
template <class S> HME_FN void fermion_kit(const double* p, double m, int kind, S* kit) {
  if (kind >= 3) {
    for (int h = 0; h < 2; ++h) {
      const int lam = h == 0 ? 1 : -1;
      const sp4<double> w = kind == 3 ? oxxxxx(p, m, lam, -1) : ixxxxx(p, m, lam, +1);
      for (int c = 0; c < 4; ++c) {
        kit[8 * h + 2 * c] = S(w.c[c].r);
        kit[8 * h + 2 * c + 1] = S(w.c[c].i);
      }
    }
    return;
  }
  double wp, wm;
  spinor_weights(p, m, wp, wm);
  for (int h = 0; h < 2; ++h) {
    const int lam = h == 0 ? 1 : -1;
    cx<double> chi[2];
    sp4<double> w;
    const double a = lam > 0 ? wp : wm, b = lam > 0 ? wm : wp;
    if (kind == 1) {
      helicity_chi(p, lam, chi);
      w = {{a * conj(chi[0]), a * conj(chi[1]), b * conj(chi[0]), b * conj(chi[1])}};
    } else {
      helicity_chi(p, -lam, chi);
      w = {{a * chi[0], a * chi[1], -b * chi[0], -b * chi[1]}};
    }
    for (int c = 0; c < 4; ++c) {
      kit[8 * h + 2 * c] = S(w.c[c].r);
      kit[8 * h + 2 * c + 1] = S(w.c[c].i);
    }
  }
}

// A kit read out of the table (N values, already in the arithmetic type).
template <class T, int N> struct kitv {
  T v[N];
};
template <class T, int N, class S> HME_FN kitv<T, N> load_kit(const volatile HME_LDS S* kit) {
  kitv<T, N> r;
#pragma unroll
  for (int i = 0; i < N; ++i) r.v[i] = T(kit[i]);
  return r;
}

// The state from the half of a kit that belongs to the lane's helicity (lam and nsv are
// already folded into the kit; the arguments keep the call shape of the builders above).
template <class T> HME_FN vw4<T> vxxxxx_from(const kitv<T, 5>& k, int, int) {
  vw4<T> w;
  w.c[0] = {T(0), T(0)};
  w.c[1] = {k.v[0], k.v[3]};
  w.c[2] = {k.v[1], k.v[4]};
  w.c[3] = {k.v[2], T(0)};
  return w;
}
template <class T> HME_FN sp4<T> spinor_from(const kitv<T, 8>& k) {
  return {{{k.v[0], k.v[1]}, {k.v[2], k.v[3]}, {k.v[4], k.v[5]}, {k.v[6], k.v[7]}}};
}
template <class T> HME_FN sp4<T> oxxxxx_from(const kitv<T, 8>& k, int) { return spinor_from<T>(k); }
template <class T> HME_FN sp4<T> ixxxxx_from(const kitv<T, 8>& k, int) { return spinor_from<T>(k); }

template <class T, class S> HME_FN vw4<T> vxxxxx_kit(const volatile HME_LDS S* kit, int lam, int nsv) {
  return vxxxxx_from<T>(load_kit<T, 5>(kit + (lam > 0 ? 0 : 5)), lam, nsv);
}
template <class T, class S> HME_FN sp4<T> oxxxxx_kit(const volatile HME_LDS S* kit, int lam) {
  return spinor_from<T>(load_kit<T, 8>(kit + (lam > 0 ? 0 : 8)));
}
template <class T, class S> HME_FN sp4<T> ixxxxx_kit(const volatile HME_LDS S* kit, int lam) {
  return spinor_from<T>(load_kit<T, 8>(kit + (lam > 0 ? 0 : 8)));
}

template <class T, class S> HME_FN vlcx<T> vxxxxx_lc_kit(const volatile HME_LDS S* kit, int lam) {
  const kitv<T, 5> k = load_kit<T, 5>(kit + (lam > 0 ? 0 : 5));
  return {k.v[0], {k.v[1], k.v[2]}, {k.v[3], k.v[4]}};
}

// Observer of the amplitude terms in the generated code: term(d, a) for each term a of diagram
// d.  The default does nothing (and costs nothing).
struct NoObserver {
  template <class C> HME_FN void term(int, const C&) const {}
};

// Recycled wavefunctions (helicity recycling): a wavefunction built from two external states
// is computed once per event for each of its 4 helicity pairs and stored in the table as its
// 4 complex components; a lane reads the pair of its helicity.
template <class W, class S> HME_FN void store_wf(const W& x, S* o) {
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    o[2 * mu] = x.c[mu].r;
    o[2 * mu + 1] = x.c[mu].i;
  }
}
template <class T, class S> HME_FN vw4<T> recycled_vw4(const volatile HME_LDS S* p, int off) {
  const kitv<T, 8> k = load_kit<T, 8>(p + off);
  vw4<T> w;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) w.c[mu] = {k.v[2 * mu], k.v[2 * mu + 1]};
  return w;
}
template <class T, class S> HME_FN void store_lc(const vlc<T>& x, S* o) {
  o[0] = x.p.r;
  o[1] = x.p.i;
  o[2] = x.m.r;
  o[3] = x.m.i;
  o[4] = x.t.r;
  o[5] = x.t.i;
  o[6] = x.tb.r;
  o[7] = x.tb.i;
}
template <class T, class S> HME_FN vlc<T> recycled_vlc(const volatile HME_LDS S* p, int off) {
  const kitv<T, 8> k = load_kit<T, 8>(p + off);
  return {{k.v[0], k.v[1]}, {k.v[2], k.v[3]}, {k.v[4], k.v[5]}, {k.v[6], k.v[7]}};
}
template <class T, class S> HME_FN sp4<T> recycled_sp4(const volatile HME_LDS S* p, int off) {
  const kitv<T, 8> k = load_kit<T, 8>(p + off);
  sp4<T> w;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) w.c[mu] = {k.v[2 * mu], k.v[2 * mu + 1]};
  return w;
}

// ------------------------------------------------------------------ vertices with per-event kits
// The helicity-independent parts of a vertex (momentum combinations, propagator factor) are
// computed once per event into the table; these variants read them instead of forming them
// at every use.

// vvv_vec with k = (den (Qa - Qb), den (Qa + 2 Qb), den (2 Qa + Qb)).
template <class T> HME_FN vw4<T> vvv_vec_k(const vw4<T>& a, const vw4<T>& b, const kitv<T, 12>& k) {
  const cx<T> ab = mdot(a, b), va = mdot(k.v + 4, a), wb = mdot(k.v + 8, b);
  vw4<T> J;
  for (int mu = 0; mu < 4; ++mu) J.c[mu] = cfms(wb, a.c[mu], cfma(va, b.c[mu], k.v[mu] * ab));
  return J;
}

// Feynman-diagram gauge propagator of an internal gluon (Hagiwara, Kanzaki, Li, Mawatari and
// Nakamura, Eur. Phys. J. C 80 (2020) 584): i/Q^2 [-g + (n Q + Q n)/(n.Q)] applied to the vertex,
// i.e. the Feynman-gauge current J (propagator included) becomes J - nt (Q.J) - Q (nt.J) with
// k = (nt, Q), nt = n / (n.Q), n = (sign Q0, -Q3vec / |Q3vec|).
template <class T> HME_FN vw4<T> fd_project(const vw4<T>& J, const kitv<T, 8>& k) {
  const cx<T> qj = mdot(k.v + 4, J), nj = mdot(k.v, J);
  vw4<T> r;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) r.c[mu] = rfma(-k.v[4 + mu], nj, rfma(-k.v[mu], qj, J.c[mu]));
  return r;
}

// vvv_amp with k = (Qa - Qb, Qb - Qc, Qc - Qa).
template <class T>
HME_FN cx<T> vvv_amp_k(const vw4<T>& a, const vw4<T>& b, const vw4<T>& c, const kitv<T, 12>& k) {
  return cfma(mdot(c, a), mdot(k.v + 8, b), cfma(mdot(b, c), mdot(k.v + 4, a), mdot(a, b) * mdot(k.v, c)));
}

// ffv_psi / ffv_psibar with k = den (K0 + K3, K0 - K3, K1, K2, m), from the products g / h of
// V-slash and the spinor.
template <class T> HME_FN sp4<T> psi_out(const cx<T>& g0, const cx<T>& g1, const cx<T>& g2, const cx<T>& g3,
                                        const kitv<T, 5>& k) {
  const T kp = k.v[0], km = k.v[1], md = k.v[4];
  const cx<T> kt = {k.v[2], k.v[3]}, ktb = {k.v[2], -k.v[3]};
  sp4<T> o;
  o.c[0] = cfms(ktb, g3, rfma(md, g0, km * g2));
  o.c[1] = cfms(kt, g2, rfma(md, g1, kp * g3));
  o.c[2] = cfma(ktb, g1, rfma(md, g2, kp * g0));
  o.c[3] = cfma(kt, g0, rfma(md, g3, km * g1));
  return o;
}
template <class T> HME_FN sp4<T> ffv_psi_k(const sp4<T>& f, const vlc<T>& v, const kitv<T, 5>& k) {
  return psi_out(cfms(v.tb, f.c[3], v.m * f.c[2]), cfms(v.t, f.c[2], v.p * f.c[3]),
                 cfma(v.tb, f.c[1], v.p * f.c[0]), cfma(v.m, f.c[1], v.t * f.c[0]), k);
}
template <class T> HME_FN sp4<T> ffv_psi_k(const sp4<T>& f, const vlcx<T>& v, const kitv<T, 5>& k) {
  return psi_out(cfms(v.tb, f.c[3], (-v.p) * f.c[2]), cfms(v.t, f.c[2], v.p * f.c[3]),
                 cfma(v.tb, f.c[1], v.p * f.c[0]), rfma(-v.p, f.c[1], v.t * f.c[0]), k);
}
template <class T> HME_FN sp4<T> ffv_psi_k(const sp4<T>& f, const vw4<T>& V, const kitv<T, 5>& k) {
  return ffv_psi_k(f, vlc_of(V), k);
}

template <class T> HME_FN sp4<T> psibar_out(const cx<T>& h0, const cx<T>& h1, const cx<T>& h2, const cx<T>& h3,
                                           const kitv<T, 5>& k) {
  const T kp = k.v[0], km = k.v[1], md = k.v[4];
  const cx<T> kt = {k.v[2], k.v[3]}, ktb = {k.v[2], -k.v[3]};
  sp4<T> o;
  o.c[0] = cfma(kt, h3, rfma(md, h0, kp * h2));
  o.c[1] = cfma(ktb, h2, rfma(md, h1, km * h3));
  o.c[2] = cfms(kt, h1, rfma(md, h2, km * h0));
  o.c[3] = cfms(ktb, h0, rfma(md, h3, kp * h1));
  return o;
}
template <class T> HME_FN sp4<T> ffv_psibar_k(const sp4<T>& fb, const vlc<T>& v, const kitv<T, 5>& k) {
  return psibar_out(cfma(fb.c[3], v.t, fb.c[2] * v.p), cfma(fb.c[3], v.m, fb.c[2] * v.tb),
                    cfms(fb.c[1], v.t, fb.c[0] * v.m), cfms(fb.c[0], v.tb, fb.c[1] * v.p), k);
}
template <class T> HME_FN sp4<T> ffv_psibar_k(const sp4<T>& fb, const vlcx<T>& v, const kitv<T, 5>& k) {
  return psibar_out(cfma(fb.c[3], v.t, v.p * fb.c[2]), rfma(-v.p, fb.c[3], fb.c[2] * v.tb),
                    cfms(fb.c[1], v.t, (-v.p) * fb.c[0]), cfms(fb.c[0], v.tb, v.p * fb.c[1]), k);
}
template <class T> HME_FN sp4<T> ffv_psibar_k(const sp4<T>& fb, const vw4<T>& V, const kitv<T, 5>& k) {
  return ffv_psibar_k(fb, vlc_of(V), k);
}

// ------------------------------------------------------------------ compensated per-event arithmetic
// A propagator denominator Q^2 - m^2 of an almost on-shell line is a small difference of large
// numbers (soft or collinear emissions), so the rounding of the momentum sum Q and of Q^2 is
// amplified by Q0^2 / |Q^2 - m^2|.  The per-event table therefore forms momentum sums, their
// differences and Q^2 - m^2 as unevaluated sums hi + lo of two doubles (error-free
// transformations: Knuth's two-sum, and the exact product a b = p + fma(a, b, -p)), and rounds
// once at the end.  This runs once per event, not per helicity.  Contraction is switched off in
// these functions: the device compiler would otherwise fuse a product into a later sum (for
// example round(a^2) + b into fma(a, a, b)), which breaks the error-free transformations.
struct dd {
  double hi, lo;
};
HME_FN dd two_sum(double a, double b) {
  _Pragma("clang fp contract(off)")
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
HME_FN dd quick_two_sum(double a, double b) {  // |a| >= |b|
  _Pragma("clang fp contract(off)")
  const double s = a + b;
  return {s, b - (s - a)};
}
HME_FN dd dd_add(dd a, dd b) {
  _Pragma("clang fp contract(off)")
  const dd s = two_sum(a.hi, b.hi);
  return quick_two_sum(s.hi, s.lo + (a.lo + b.lo));
}
HME_FN dd dd_scale(double k, dd a) {  // k a for a small integer k (exact)
  _Pragma("clang fp contract(off)")
  return {k * a.hi, k * a.lo};
}
HME_FN dd dd_neg(dd a) {
  _Pragma("clang fp contract(off)")
  return {-a.hi, -a.lo};
}
HME_FN dd two_prod(double a, double b) {
  _Pragma("clang fp contract(off)")
  const double p = a * b;
  return {p, __builtin_fma(a, b, -p)};
}
HME_FN dd dd_sq(dd a) {
  _Pragma("clang fp contract(off)")
  const dd p = two_prod(a.hi, a.hi);
  return quick_two_sum(p.hi, __builtin_fma(2.0 * a.hi, a.lo, p.lo));
}
HME_FN double dd_val(dd a) {
  _Pragma("clang fp contract(off)")
  return a.hi + a.lo;
}
// Minkowski square minus m^2 of a compensated four-vector, rounded once
HME_FN double dd_minkowski_sq(const dd* Q, double m) {
  _Pragma("clang fp contract(off)")
  dd s = dd_sq(Q[0]);
  s = dd_add(s, dd_neg(dd_sq(Q[1])));
  s = dd_add(s, dd_neg(dd_sq(Q[2])));
  s = dd_add(s, dd_neg(dd_sq(Q[3])));
  if (m != 0.0) s = dd_add(s, dd_neg(two_prod(m, m)));
  return dd_val(s);
}

// ------------------------------------------------------------------ electroweak current (Drell-Yan)
// The lepton pair of q qbar -> e+ e- (+ gluons) as one vector wavefunction attached to the quark
// line with a plain gamma^mu: W^mu = A_gamma L^mu + A_Z (L^mu - q^mu (q.L) / mZ^2), with the lepton
// current L^mu = ubar(e-) gamma^mu v(e+), q = p(e+) + p(e-), s = q^2,
//   A_gamma = e^2 Qq Qe / s,  A_Z = e^2 / (sw^2 cw^2) gq ge / (s - mZ^2 + i mZ wZ).
// For massless fermions the chirality of each line is its helicity (u(p, +) and ubar(p, +) are
// right-handed), so the Z couplings gL P_L + gR P_R reduce to the number gq = gR or gL of the
// quark's helicity and ge = gR or gL of the electron's.  The vertex factors -i, the photon and Z
// propagators' -i, common to every diagram, are left out.  q^2 and q^2 - mZ^2 are formed in
// compensated arithmetic.  Item c of the kit (8 doubles: the 4 complex components) holds the
// current for helicities (quark, e+, e-) = bits (4, 2, 1) of c set for +1.
struct EwCouplings {
  double cA, cZ;    // e^2 Qq Qe and e^2 / (sw^2 cw^2)
  double gLq, gRq;  // quark Z couplings T3 - Qq sw^2, -Qq sw^2
  double gLe, gRe;  // electron Z couplings -1/2 + sw^2, sw^2
  double mZ, wZ;
};

template <class S>
HME_FN void ew_kit(const double* pep, const double* pem, const EwCouplings& c, int item, S* kit) {
  const int hq = (item >> 2 & 1) ? 1 : -1, hep = (item >> 1 & 1) ? 1 : -1, hem = (item & 1) ? 1 : -1;
  const vw4<double> L = ffv_vec<double>(oxxxxx(pem, 0.0, hem, +1), ixxxxx(pep, 0.0, hep, -1), 1.0);
  dd Q[4];
  double q[4];
  for (int mu = 0; mu < 4; ++mu) {
    Q[mu] = two_sum(pep[mu], pem[mu]);
    q[mu] = dd_val(Q[mu]);
  }
  const double s = dd_minkowski_sq(Q, 0.0);
  const double dr = dd_minkowski_sq(Q, c.mZ), di = c.mZ * c.wZ, dn = 1.0 / (dr * dr + di * di);
  const double gz = c.cZ * (hq > 0 ? c.gRq : c.gLq) * (hem > 0 ? c.gRe : c.gLe);
  const cx<double> az = {gz * dr * dn, -gz * di * dn};  // gz / (s - mZ^2 + i mZ wZ)
  const double aa = c.cA / s;
  const cx<double> ql = (1.0 / (c.mZ * c.mZ)) * mdot(q, L);
  for (int mu = 0; mu < 4; ++mu) {
    const cx<double> w = aa * L.c[mu] + az * (L.c[mu] - q[mu] * ql);
    kit[2 * mu] = S(w.r);
    kit[2 * mu + 1] = S(w.i);
  }
}

template <class T, class S> HME_FN vw4<T> ew_from_kit(const volatile HME_LDS S* kit, int hq, int hep, int hem) {
  const int item = (hq > 0 ? 4 : 0) + (hep > 0 ? 2 : 0) + (hem > 0 ? 1 : 0);
  const kitv<T, 8> k = load_kit<T, 8>(kit + 8 * item);
  vw4<T> w;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) w.c[mu] = {k.v[2 * mu], k.v[2 * mu + 1]};
  return w;
}

// Scheduling fence for the generated code: table reads issued before it are not moved
// past it, so their LDS latency overlaps the arithmetic that follows.
#if defined(__HIP_DEVICE_COMPILE__)
#define HME_FENCE() __builtin_amdgcn_sched_barrier(0)
#else
#define HME_FENCE() ((void)0)
#endif

}  // namespace hme
