// Device routines for tree-level QCD helicity amplitudes on CDNA4 (gfx950).
//
// Wavefunctions and vertex functions of the HELAS family for massless quarks
// and gluons: the paper's section 4 (Table 4) and its appendix give the
// gluon self-coupling routines vvvxxx, jvvxx0, ggggxx and jgggx0; the quark
// routines (external spinors, qqg vertex and currents) are written here from
// the Dirac algebra.
//
// Design differences from the paper's cmplx[6] wavefunctions:
//  * a wavefunction holds only its components; the flowing-out momentum of
//    every current is a subset sum of external momenta formed once in FP64
//    by the generated code, together with 1/P^2;
//  * massless quark wavefunctions are two-component Weyl spinors: a fermion
//    line has a fixed chirality h = +1 (right-handed) or -1, known at compile
//    time, so gamma-matrix products reduce to 2x2 sigma products
//    S_h(v) = v^0 - h (v . sigma);
//  * all couplings are 1 here; the common factor g_s^(n-2) of every diagram is
//    applied to |M|^2 at the end.
//
// Conventions (metric +,-,-,-):
//   external gluon   eps(p, lam)   incoming,  eps(p, lam)^*  outgoing,
//                    eps = (0, -lam*theta_hat - i*phi_hat)/sqrt2, slot momentum -p / +p
//   flowing-in quark  phi = sqrt(2E) xi_h(p): u(p,lam) of an incoming quark
//                     (h = lam) or v(p,lam) of an outgoing antiquark (h = -lam)
//   flowing-out quark chi = conj(sqrt(2E) xi_h(p)): u-bar of an outgoing quark
//                     (h = lam) or v-bar of an incoming antiquark (h = -lam)
//   sqrt(2E) xi_+ = (sqrt(E+pz), (px + i py)/sqrt(E+pz)),
//   sqrt(2E) xi_- = ((-px + i py)/sqrt(E+pz), sqrt(E+pz)),
//   with the p parallel to -z branch xi_+ = (0, 1), xi_- = (-1, 0).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace heget {

template <class R> struct cx { R re, im; };
template <class R> struct vec4 { cx<R> c0, c1, c2, c3; };   // complex 4-vector, upper index
template <class R> struct mom4 { R e, x, y, z; };          // real 4-vector, upper index
template <class R> struct wsp { cx<R> s0, s1; };           // Weyl 2-spinor

#define HD __device__ __forceinline__

template <class R> HD cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R> HD cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R> HD cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <class R> HD cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R> HD cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <class R> HD cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
template <class R> HD cx<R> times_i(cx<R> a) { return {-a.im, a.re}; }

template <class R> HD vec4<R> operator+(const vec4<R>& a, const vec4<R>& b) {
  return {a.c0 + b.c0, a.c1 + b.c1, a.c2 + b.c2, a.c3 + b.c3};
}
template <class R> HD vec4<R> operator-(const vec4<R>& a, const vec4<R>& b) {
  return {a.c0 - b.c0, a.c1 - b.c1, a.c2 - b.c2, a.c3 - b.c3};
}
template <class R> HD wsp<R> operator+(const wsp<R>& a, const wsp<R>& b) { return {a.s0 + b.s0, a.s1 + b.s1}; }
template <class R> HD wsp<R> operator-(const wsp<R>& a, const wsp<R>& b) { return {a.s0 - b.s0, a.s1 - b.s1}; }
// a + s b for a real factor s (operand sums of a closing vertex)
template <class R> HD vec4<R> lin(const vec4<R>& a, R s, const vec4<R>& b) {
  return {a.c0 + s * b.c0, a.c1 + s * b.c1, a.c2 + s * b.c2, a.c3 + s * b.c3};
}
template <class R> HD wsp<R> lin(const wsp<R>& a, R s, const wsp<R>& b) { return {a.s0 + s * b.s0, a.s1 + s * b.s1}; }
template <class R> HD vec4<R> scale(cx<R> s, const vec4<R>& a) {
  return {s * a.c0, s * a.c1, s * a.c2, s * a.c3};
}

// Minkowski bilinear of two complex vectors (no conjugation)
template <class R> HD cx<R> mdot(const vec4<R>& a, const vec4<R>& b) {
  return a.c0 * b.c0 - a.c1 * b.c1 - a.c2 * b.c2 - a.c3 * b.c3;
}
// real momentum . complex vector
template <class R> HD cx<R> pdot(const mom4<R>& p, const vec4<R>& a) {
  return cx<R>{p.e * a.c0.re - p.x * a.c1.re - p.y * a.c2.re - p.z * a.c3.re,
               p.e * a.c0.im - p.x * a.c1.im - p.y * a.c2.im - p.z * a.c3.im};
}

HD double msq(const mom4<double>& p) { return p.e * p.e - p.x * p.x - p.y * p.y - p.z * p.z; }
HD mom4<double> add(const mom4<double>& a, const mom4<double>& b) {
  return {a.e + b.e, a.x + b.x, a.y + b.y, a.z + b.z};
}
template <class R> HD mom4<R> to(const mom4<double>& p) { return {(R)p.e, (R)p.x, (R)p.y, (R)p.z}; }

// 1/P^2 of a propagator from its float64 invariant.  float: the hardware reciprocal of the rounded
// invariant (1 ulp of float).  double: the hardware reciprocal estimate refined by two Newton-Raphson
// steps r <- r + r (1 - x r), each of which squares the relative error, to about 1 ulp of double.
template <class R> HD R inv_msq(const mom4<double>& p);
template <> HD float inv_msq<float>(const mom4<double>& p) { return __builtin_amdgcn_rcpf((float)msq(p)); }
template <> HD double inv_msq<double>(const mom4<double>& p) {
  const double x = msq(p);
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
  r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
  return r;
}

// ------------------------------------------------------------ external states

// 1/sqrt(x) for x > 0: the hardware estimate, in float64 refined by two Newton-Raphson steps
// y <- y (3 - x y^2) / 2 (each squares the relative error).
HD float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
HD double rsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * __builtin_fma(-h * y, y, 1.5);
  y = y * __builtin_fma(-h * y, y, 1.5);
  return y;
}

// Polarisation of a massless gluon with physical momentum p and helicity lam, computed in the
// precision of the result (R).  outgoing = true returns the complex conjugate.
template <class R> HD vec4<R> vxxxx0(const mom4<double>& p, int lam, bool outgoing) {
  const R px = R(p.x), py = R(p.y), pz = R(p.z);
  const R pt2 = px * px + py * py;
  const R ipa = rsq(pt2 + pz * pz);
  const bool side = pt2 > R(0);
  const R ipt = side ? rsq(pt2) : R(0);
  const R ct = pz * ipa, st = pt2 * ipt * ipa;
  const R cf = side ? px * ipt : R(1);
  const R sf = side ? py * ipt : R(0);
  const R r2 = R(0.70710678118654752440);
  const R l = lam > 0 ? r2 : -r2;
  const R im_sign = outgoing ? -r2 : r2;
  vec4<R> e;
  e.c0 = {R(0), R(0)};
  e.c1 = {-l * ct * cf, im_sign * sf};
  e.c2 = {-l * ct * sf, -im_sign * cf};
  e.c3 = {l * st, R(0)};
  return e;
}

// Test-hook form of vxxxx0: with gauge set the polarisation is replaced by the gluon's momentum
// over its energy, the substitution under which every amplitude must vanish (current
// conservation, section 4: eq. vvv-amplitude and the qqg vertex); otherwise vxxxx0.
template <class R> HD vec4<R> vxxxx0g(const mom4<double>& p, int lam, bool outgoing, bool gauge) {
  if (gauge) {
    const double ie = 1.0 / p.e;
    vec4<R> k;
    k.c0 = {R(1), R(0)};
    k.c1 = {R(p.x * ie), R(0)};
    k.c2 = {R(p.y * ie), R(0)};
    k.c3 = {R(p.z * ie), R(0)};
    return k;
  }
  return vxxxx0<R>(p, lam, outgoing);
}

// sqrt(2E) xi_h(p) for a massless momentum (float64 inputs, result in R)
template <class R, int H> HD wsp<R> weyl_xi(const mom4<double>& p) {
  double rho = p.e + p.z;
  wsp<R> w;
  if (rho > 1e-10 * p.e) {
    const double isr = rsq(rho), sr = rho * isr;
    if (H > 0) {
      w.s0 = {R(sr), R(0)};
      w.s1 = {R(p.x * isr), R(p.y * isr)};
    } else {
      w.s0 = {R(-p.x * isr), R(p.y * isr)};
      w.s1 = {R(sr), R(0)};
    }
  } else {
    const double s2e = 2.0 * p.e * rsq(2.0 * p.e);
    if (H > 0) {
      w.s0 = {R(0), R(0)};
      w.s1 = {R(s2e), R(0)};
    } else {
      w.s0 = {R(-s2e), R(0)};
      w.s1 = {R(0), R(0)};
    }
  }
  return w;
}
template <class R, int H> HD wsp<R> ixxxx0(const mom4<double>& p) { return weyl_xi<R, H>(p); }
template <class R, int H> HD wsp<R> oxxxx0(const mom4<double>& p) {
  wsp<R> w = weyl_xi<R, H>(p);
  return {conj(w.s0), conj(w.s1)};
}

// ------------------------------------------------------------ gluon routines

// Amplitude of the three-gluon vertex (paper: vvvxxx, coupling 1).
template <class R>
HD cx<R> vvvxxx(const vec4<R>& a, const mom4<R>& pa, const vec4<R>& b, const mom4<R>& pb,
                const vec4<R>& c, const mom4<R>& pc) {
  cx<R> vab = mdot(a, b), vbc = mdot(b, c), vca = mdot(c, a);
  mom4<R> dab{pa.e - pb.e, pa.x - pb.x, pa.y - pb.y, pa.z - pb.z};
  mom4<R> dbc{pb.e - pc.e, pb.x - pc.x, pb.y - pc.y, pb.z - pc.z};
  mom4<R> dca{pc.e - pa.e, pc.x - pa.x, pc.y - pa.y, pc.z - pa.z};
  return -(vab * pdot(dab, c) + vbc * pdot(dbc, a) + vca * pdot(dca, b));
}

// Off-shell gluon from two gluons (paper: jvvxx0), Feynman gauge, times 1/P^2.
template <class R>
HD vec4<R> jvvxx0(const vec4<R>& a, const mom4<R>& pa, const vec4<R>& b, const mom4<R>& pb, R inv_s) {
  cx<R> gab = mdot(a, b);
  mom4<R> sa{pa.e + 2 * pb.e, pa.x + 2 * pb.x, pa.y + 2 * pb.y, pa.z + 2 * pb.z};
  mom4<R> sb{2 * pa.e + pb.e, 2 * pa.x + pb.x, 2 * pa.y + pb.y, 2 * pa.z + pb.z};
  cx<R> sga = inv_s * pdot(sa, a);
  cx<R> sgb = inv_s * pdot(sb, b);
  cx<R> g = inv_s * gab;
  // -[(pa - pb)(a.b) + (sa.a) b - (sb.b) a] / s
  vec4<R> j;
  j.c0 = cx<R>{-(pa.e - pb.e) * g.re, -(pa.e - pb.e) * g.im} - sga * b.c0 + sgb * a.c0;
  j.c1 = cx<R>{-(pa.x - pb.x) * g.re, -(pa.x - pb.x) * g.im} - sga * b.c1 + sgb * a.c1;
  j.c2 = cx<R>{-(pa.y - pb.y) * g.re, -(pa.y - pb.y) * g.im} - sga * b.c2 + sgb * a.c2;
  j.c3 = cx<R>{-(pa.z - pb.z) * g.re, -(pa.z - pb.z) * g.im} - sga * b.c3 + sgb * a.c3;
  return j;
}

// One colour piece of the four-gluon vertex amplitude (paper: ggggxx).
template <class R>
HD cx<R> ggggxx(const vec4<R>& a, const vec4<R>& b, const vec4<R>& c, const vec4<R>& d) {
  return mdot(a, d) * mdot(b, c) - mdot(a, c) * mdot(b, d);
}

// One colour piece of the off-shell gluon from three gluons (paper: jgggx0), times 1/P^2.
template <class R>
HD vec4<R> jgggx0(const vec4<R>& a, const vec4<R>& b, const vec4<R>& c, R inv_s) {
  cx<R> cb = inv_s * mdot(c, b);
  cx<R> ac = inv_s * mdot(a, c);
  return {cb * a.c0 - ac * b.c0, cb * a.c1 - ac * b.c1, cb * a.c2 - ac * b.c2, cb * a.c3 - ac * b.c3};
}

// ------------------------------------------------------------ quark routines

// S_h(v) psi with S_h(v) = v^0 - h (v . sigma), v complex
template <class R, int H> HD wsp<R> smul(const vec4<R>& v, const wsp<R>& f) {
  const R h = R(H);
  cx<R> m00 = v.c0 - h * v.c3, m11 = v.c0 + h * v.c3;
  cx<R> v12m = v.c1 - times_i(v.c2);   // v1 - i v2
  cx<R> v12p = v.c1 + times_i(v.c2);   // v1 + i v2
  return {m00 * f.s0 - h * (v12m * f.s1), -h * (v12p * f.s0) + m11 * f.s1};
}
template <class R, int H> HD wsp<R> smulp(const mom4<R>& p, const wsp<R>& f) {
  const R h = R(H);
  R m00 = p.e - h * p.z, m11 = p.e + h * p.z;
  cx<R> v12m{p.x, -p.y}, v12p{p.x, p.y};
  return {m00 * f.s0 - h * (v12m * f.s1), -h * (v12p * f.s0) + m11 * f.s1};
}
// row spinor times S_h(v)
template <class R, int H> HD wsp<R> rmul(const wsp<R>& g, const vec4<R>& v) {
  const R h = R(H);
  cx<R> m00 = v.c0 - h * v.c3, m11 = v.c0 + h * v.c3;
  cx<R> v12m = v.c1 - times_i(v.c2);
  cx<R> v12p = v.c1 + times_i(v.c2);
  return {g.s0 * m00 - h * (g.s1 * v12p), -h * (g.s0 * v12m) + g.s1 * m11};
}
template <class R, int H> HD wsp<R> rmulp(const wsp<R>& g, const mom4<R>& p) {
  const R h = R(H);
  R m00 = p.e - h * p.z, m11 = p.e + h * p.z;
  cx<R> v12m{p.x, -p.y}, v12p{p.x, p.y};
  return {m00 * g.s0 - h * (g.s1 * v12p), -h * (g.s0 * v12m) + m11 * g.s1};
}

// qqg vertex amplitude  chi^T S_h(v) phi   (colour factor -T^a applied by the generator)
template <class R, int H> HD cx<R> iovxx0(const wsp<R>& fi, const wsp<R>& fo, const vec4<R>& v) {
  wsp<R> t = smul<R, H>(v, fi);
  return fo.s0 * t.s0 + fo.s1 * t.s1;
}
// off-shell flowing-in quark  S_{-h}(P) S_h(v) phi / P^2
template <class R, int H>
HD wsp<R> fvixx0(const wsp<R>& fi, const vec4<R>& v, const mom4<R>& p, R inv_s) {
  wsp<R> t = smulp<R, -H>(p, smul<R, H>(v, fi));
  return {inv_s * t.s0, inv_s * t.s1};
}
// off-shell flowing-out quark  -chi^T S_h(v) S_{-h}(P) / P^2
template <class R, int H>
HD wsp<R> fvoxx0(const wsp<R>& fo, const vec4<R>& v, const mom4<R>& p, R inv_s) {
  wsp<R> t = rmulp<R, -H>(rmul<R, H>(fo, v), p);
  return {(-inv_s) * t.s0, (-inv_s) * t.s1};
}
// off-shell gluon from a quark pair  J^0 = chi.phi, J^k = h chi sigma^k phi, times 1/P^2
template <class R, int H> HD vec4<R> jioxx0(const wsp<R>& fi, const wsp<R>& fo, R inv_s) {
  const R h = R(H) * inv_s;
  vec4<R> j;
  j.c0 = inv_s * (fo.s0 * fi.s0 + fo.s1 * fi.s1);
  j.c1 = h * (fo.s0 * fi.s1 + fo.s1 * fi.s0);
  j.c2 = h * times_i(fo.s1 * fi.s0 - fo.s0 * fi.s1);
  j.c3 = h * (fo.s0 * fi.s0 - fo.s1 * fi.s1);
  return j;
}

#undef HD
}  // namespace heget
