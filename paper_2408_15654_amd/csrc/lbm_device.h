// Device-side per-site arithmetic of the coupled three-field lattice
// Boltzmann step (Zhan, Liang, Chai, Shi, arXiv:2408.15654), templated on
// the arithmetic type R (float or double).
//
// Lattice: D2Q9, c_0..c_8 = (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1)
// (-1,-1) (1,-1) (the order of the rows of M in Eq. (34)), weights 4/9,
// 1/9, 1/36, c_s^2 = 1/3, lattice units.
//
// The collisions are done in raw-moment space (Sec. 4): the nine moments of
// Eq. (34) are formed with shared partial sums, the equilibrium and source
// moments are their closed forms, and the inverse transform is applied
// explicitly.  h_0 is never formed: column 0 of M is e_0 and rows 1-8 of
// M^-1 have a zero first entry, so h_0 feeds nothing.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

// Parameters of the physics, pre-combined on the host.
template <class R>
struct Phys {
  R phiA, phiB, phiAB;     // phiA, phiB, phiA + phiB
  R c4W;                   // 4 / (W dphi): delta = c4W (phiA-phi)(phi-phiB)
  R cbulk;                 // 24 / (W dphi^4): bulk part of mu_phi
  R cW;                    // 3 W / (2 dphi^2): gradient part and Marangoni
  R rhoB, drho;            // rho = rhoB + drho (phi - phiB)
  R muB, dmu;              // mu  = muB  + dmu  (phi - phiB)
  R Mdrho;                 // M drho: S = Mdrho (grad phi - delta n)
  R gx, gy;                // body force per unit mass
  R sigma0, beta;          // equation of state
  R r, rm1;                // r and r - 1
  R s1f, s2f, s3f, s4f;    // rates of the phase-field LB
  R s1g, s2g, s3g, s4g;    // rates of the surfactant LB
  R s3h, s4h;              // free rates of the flow LB (s2 is per site)
  R uwb, uwt;              // wall speeds (bottom, top)
  R psi_max;               // Langmuir clamp 1 - 1e-9
  R eps_n;                 // n = grad phi / (|grad phi| + eps_n)
  int eos;                 // 0 linear, 1 Langmuir
};

// x/3 and x/9.  In float32 the rounded reciprocals are biased (1/3 by
// +3.0e-8 relative), and the third-order equilibrium moments rho u/3 and
// X u/3 of the collisions are large terms whose differences make the
// viscous stress and the diffusive flux: the bias changes the effective
// viscosity by parts per million and the error of a decaying flow then
// grows step after step (to 2.6e-5 of u over 5000 steps of the 2048x2048
// field).  Adding the product with the reciprocal's remainder in one fused
// multiply-add leaves only the product's unbiased rounding.  float64 keeps
// the plain product (bias 2e-17).
template <class R>
__device__ __forceinline__ R third_of(R x) {
  return x * (R(1) / R(3));
}
template <>
__device__ __forceinline__ float third_of<float>(float x) {
  return __builtin_fmaf(x, 0x1.555556p-2f, x * -0x1.555556p-27f);
}
// 1/x.  float32: the hardware reciprocal (within 1 ulp) refined by one
// Newton step in fused multiply-adds, 3 instructions instead of the ~10 of
// a correctly rounded division, and within an ulp of it (on the parity
// problems it gave the rounded quotient wherever it is used: their results
// are bitwise those of the division).  Where many sites share one x (a
// uniform phase) they would share an error too, as they share the rounding
// of a division: a relative 1e-7 in u or in a relaxation rate, with no
// large term to amplify it (unlike the 1/3 of third_of).  float64 keeps the
// division.
template <class R>
__device__ __forceinline__ R recip(R x) {
  return R(1) / x;
}
template <>
__device__ __forceinline__ float recip<float>(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(__builtin_fmaf(-x, r, 1.0f), r, r);
}
template <class R>
__device__ __forceinline__ R ninth_of(R x) {
  return x * (R(1) / R(9));
}
template <>
__device__ __forceinline__ float ninth_of<float>(float x) {
  return __builtin_fmaf(x, 0x1.c71c72p-4f, x * -0x1.c71c72p-31f);
}

template <class R>
__device__ __forceinline__ R rho_of(const Phys<R>& p, R phi) {
  return p.rhoB + p.drho * (phi - p.phiB);
}

// Eq. (20) (linear) or Eq. (19) (Langmuir).
template <class R>
__device__ __forceinline__ R sigma_of(const Phys<R>& p, R psi) {
  if (p.eos == 1) {
    R q = psi < p.psi_max ? psi : p.psi_max;
    return p.sigma0 * (R(1) + p.beta * log(R(1) - q));
  }
  return p.sigma0 - p.sigma0 * p.beta * psi;
}

// Isotropic D2Q9 stencil values of one scalar around a site: m = row y-1,
// c = row y, n = row y+1; L = column x-1, R = column x+1.
template <class R>
struct Nine {
  R mL, m, mR, cL, c, cR, nL, n, nR;
};

// grad X = sum_i w_i c_i X(x + c_i) / c_s^2.
template <class R>
__device__ __forceinline__ void grad9(const Nine<R>& v, R& gx, R& gy) {
  const R third = R(1) / R(3), twelfth = R(1) / R(12);
  gx = third * (v.cR - v.cL) + twelfth * ((v.nR - v.nL) + (v.mR - v.mL));
  gy = third * (v.n - v.m) + twelfth * ((v.nR + v.nL) - (v.mR + v.mL));
}

// lap X = sum_i 2 w_i (X(x + c_i) - X(x)) / c_s^2, summed as differences
// from the centre value (exact for close values) to limit cancellation.
template <class R>
__device__ __forceinline__ R lap9(const Nine<R>& v) {
  const R a = R(2) / R(3), b = R(1) / R(6);
  const R c = v.c;
  return a * (((v.cR - c) + (v.cL - c)) + ((v.n - c) + (v.m - c))) +
         b * (((v.nR - c) + (v.nL - c)) + ((v.mR - c) + (v.mL - c)));
}

// Everything the closures and the sources need at one site.
template <class R>
struct Front {
  R phi, psi, rho;
  R ux, uy, jx, jy;       // u and rho u
  R Sx, Sy;               // mass flux, Eq. (16)
  R Fx, Fy;               // total force
  R grx, gry;             // grad rho
  R nx, ny, delta, a;     // normal, Eq. (8) delta and a = d delta/d phi
  R gpx, gpy;             // grad psi (general r)
  R P;                    // pressure, Eq. (32b)
  R dpux, dpuy;           // d_t(phi u)
  R dqux, dquy;           // d_t(psi u)
  R dTxx, dTxy, dTyy;     // d_t(rho uu - (Su + uS)/2)
  R s2h;                  // viscous rate, Eq. (33)
};

// Interface normal n = grad phi / (|grad phi| + eps) and delta(phi) of
// Eq. (8), from phi and its gradient.
template <class R>
__device__ __forceinline__ void normal_delta(const Phys<R>& p, R phi, R gfx, R gfy, R& nx,
                                             R& ny, R& delta) {
  const R gn = sqrt(gfx * gfx + gfy * gfy);
  const R inv = recip(gn + p.eps_n);
  nx = gfx * inv;
  ny = gfy * inv;
  delta = p.c4W * ((p.phiA - phi) * (phi - p.phiB));
}

// Mass flux of Eq. (16), S = M (rhoA - rhoB)/(phiA - phiB) (grad phi -
// delta n), from phi and its gradient.  The step recomputes the previous
// level's S this way from the stored previous phi (the stencil over the
// rest values it reads anyway) instead of storing it: the same arithmetic
// on the same values as the step that produced that level.
template <class R>
__device__ __forceinline__ void mass_flux(const Phys<R>& p, R phi, R gfx, R gfy, R& Sx, R& Sy) {
  R nx, ny, delta;
  normal_delta(p, phi, gfx, gfy, nx, ny, delta);
  Sx = p.Mdrho * (gfx - delta * nx);
  Sy = p.Mdrho * (gfy - delta * ny);
}

// Forces, closures and time differences at one site, from the stencils
// (grad phi, lap phi, grad sigma, grad psi), sigma, the post-stream h_1..h_8
// and the previous level (phi, psi, u, S).  Eqs. (8), (15), (16), (18),
// (32a) read as rho u = sum c_i h_i + F/2, (32b) with K = 2/3.
template <class R, bool HAS_S>
__device__ __forceinline__ void site_front(const Phys<R>& p, Front<R>& s, R phi,
                                           R psi, R sig, R gfx, R gfy, R lphi,
                                           R gsx, R gsy, const R* h, R php,
                                           R psp, R uxp, R uyp, R Sxp, R Syp) {
  s.phi = phi;
  s.psi = psi;
  const R gn2 = gfx * gfx + gfy * gfy;
  normal_delta(p, phi, gfx, gfy, s.nx, s.ny, s.delta);
  const R qa = p.phiA - phi, qb = phi - p.phiB, qab = p.phiAB - phi - phi;
  s.a = p.c4W * qab;
  // capillary force sigma mu_phi grad phi plus Marangoni force, Eq. (18)
  const R muphi = p.cbulk * (qa * qb * qab) - p.cW * lphi;
  const R sdp = gsx * gfx + gsy * gfy;
  const R rho = rho_of(p, phi);
  s.rho = rho;
  s.Fx = sig * muphi * gfx + p.cW * (gn2 * gsx - sdp * gfx) + rho * p.gx;
  s.Fy = sig * muphi * gfy + p.cW * (gn2 * gsy - sdp * gfy) + rho * p.gy;
  if (HAS_S) {
    mass_flux(p, phi, gfx, gfy, s.Sx, s.Sy);
    s.grx = p.drho * gfx;
    s.gry = p.drho * gfy;
  } else {
    s.Sx = s.Sy = s.grx = s.gry = R(0);
  }
  // first moment and sum of h_1..h_8 (h[k] holds h_{k+1}).  The sum pairs
  // opposite directions first: each h_i carries 3 w_i c_i . rho u (Eq.
  // (30)), far larger than the pressure the sum leaves, and the pair sums
  // cancel those parts exactly (nearly equal magnitudes), so P keeps the
  // precision of its own size rather than that of rho u.
  const R d57 = h[4] - h[6], d68 = h[5] - h[7];
  const R jx0 = (h[0] - h[2]) + (d57 - d68);
  const R jy0 = (h[1] - h[3]) + (d57 + d68);
  const R sumh = ((h[0] + h[2]) + (h[1] + h[3])) + ((h[4] + h[6]) + (h[5] + h[7]));
  s.jx = jx0 + R(0.5) * s.Fx;
  s.jy = jy0 + R(0.5) * s.Fy;
  const R irho = recip(rho);
  s.ux = s.jx * irho;
  s.uy = s.jy * irho;
  const R ux = s.ux, uy = s.uy;
  // backward time differences against the previous level
  s.dpux = phi * ux - php * uxp;
  s.dpuy = phi * uy - php * uyp;
  s.dqux = psi * ux - psp * uxp;
  s.dquy = psi * uy - psp * uyp;
  const R rhop = rho_of(p, php);
  R Txx = rho * ux * ux, Txy = rho * ux * uy, Tyy = rho * uy * uy;
  R Txxp = rhop * uxp * uxp, Txyp = rhop * uxp * uyp, Tyyp = rhop * uyp * uyp;
  if (HAS_S) {
    Txx -= s.Sx * ux;
    Tyy -= s.Sy * uy;
    Txy -= R(0.5) * (s.Sx * uy + ux * s.Sy);
    Txxp -= Sxp * uxp;
    Tyyp -= Syp * uyp;
    Txyp -= R(0.5) * (Sxp * uyp + uxp * Syp);
  }
  s.dTxx = Txx - Txxp;
  s.dTxy = Txy - Txyp;
  s.dTyy = Tyy - Tyyp;
  // Eq. (32b): P = c_s^2/(1-w0) [sum_{i!=0} h_i + u.grad rho/2
  //            - w0 (rho u - S).u/(2 c_s^2) + K/2 d_t(rho u.u - S.u)]
  const R udr = ux * s.grx + uy * s.gry;
  const R Au = (s.jx - s.Sx) * ux + (s.jy - s.Sy) * uy;
  s.P = R(0.6) * (sumh + R(0.5) * udr - R(2) / R(3) * Au +
                  R(1) / R(3) * (s.dTxx + s.dTyy));
  // Eq. (33): 1/s2 = 3 mu/rho + 1/2
  const R mu = p.muB + p.dmu * (phi - p.phiB);
  s.s2h = recip(R(3) * mu * irho + R(0.5));
}

// MRT collision of a convection-diffusion LB (Eqs. (21), (25)) in raw-moment
// space, on DEVIATIONS d_i = f_i - w_i X from the rest equilibrium of the
// site's value X (the zeroth moment rounded to the arithmetic type; the
// deviations carry the rounding remainder as their zeroth moment m0, so
// X + m0 = sum f_i).  The rest part w_i X has moments
// (X, 0, 0, X/3, X/3, 0, 0, 0, X/9), all of which the collision keeps, so
// only the deviations are relaxed:
//   m_eq - m_rest = (0, X ux, X uy, 0, 0, 0, X ux/3, X uy/3, 0),
//   m_F           = (0, Vx/3, Vy/3, 0, 0, 0, Vx/9, Vy/9, 0),
// with the source w_i c_i.V, V = 3 d_t(X u) + (flux term).  Rates s1 (first
// moments), s2 (second), s3 (third), s4 (fourth).  The zeroth moment is
// conserved, remainder m0 included, so no rounding of X is ever lost from
// the sum of X (a change of X far below its last bit accumulates in m0
// until it shows).  In place on d[0..8].  Working on deviations keeps every
// intermediate small, so low-precision arithmetic and storage lose little
// absolute accuracy.
template <class R>
__device__ __forceinline__ void collide_cde(R* d, R X, R ux, R uy, R Vx, R Vy,
                                            R s1, R s2, R s3, R s4) {
  const R a57 = d[5] + d[7], a68 = d[6] + d[8];
  const R d57 = d[5] - d[7], d68 = d[6] - d[8];
  R m5 = a57 - a68, m8 = a57 + a68;
  R m6 = d57 - d68, m7 = d57 + d68;
  R m1 = (d[1] - d[3]) + m6, m2 = (d[2] - d[4]) + m7;
  R m3 = (d[1] + d[3]) + m8, m4 = (d[2] + d[4]) + m8;
  const R m0 = (d[0] + (m3 + m4)) - m8;  // sum of the incoming d_i
  const R Xux = X * ux, Xuy = X * uy;
  const R h1 = R(1) - R(0.5) * s1, h3 = R(1) - R(0.5) * s3;
  m1 = m1 - s1 * (m1 - Xux) + h1 * third_of(Vx);
  m2 = m2 - s1 * (m2 - Xuy) + h1 * third_of(Vy);
  m3 = m3 - s2 * m3;
  m4 = m4 - s2 * m4;
  m5 = m5 - s2 * m5;
  m6 = m6 - s3 * (m6 - third_of(Xux)) + h3 * ninth_of(Vx);
  m7 = m7 - s3 * (m7 - third_of(Xuy)) + h3 * ninth_of(Vy);
  m8 = m8 - s4 * m8;
  // d = M^-1 m
  d[0] = m0 - m3 - m4 + m8;
  d[1] = R(0.5) * (m1 + m3 - m6 - m8);
  d[2] = R(0.5) * (m2 + m4 - m7 - m8);
  d[3] = R(0.5) * (-m1 + m3 + m6 - m8);
  d[4] = R(0.5) * (-m2 + m4 + m7 - m8);
  d[5] = R(0.25) * (m5 + m6 + m7 + m8);
  d[6] = R(0.25) * (-m5 - m6 + m7 + m8);
  d[7] = R(0.25) * (m5 - m6 - m7 + m8);
  d[8] = R(0.25) * (-m5 + m6 - m7 + m8);
}

// Streaming in deviation form.  Population i arriving at a site comes from
// source site s_i with stored deviation dsrc_i (relative to w_i X(s_i)); e_i
// = X(s_i) - Xc is the source's rest value relative to the site's own old
// value Xc.  The new zeroth moment is
//   X' = sum_i (w_i X(s_i) + dsrc_i) = Xc + sum_i w_i e_i + sum_i dsrc_i,
// formed from small differences as Xc + dX and rounded.  The deviations are
// taken relative to w_i times that ROUNDED value, dsrc_i + w_i (e_i - dR),
// dR = round(Xc + dX) - Xc (exact for nearby values), so they sum to the
// rounding remainder dX - dR instead of dropping it: the stored state keeps
// the sum of X exactly, whatever the precision of X.
template <class R>
__device__ __forceinline__ R restream(R* d, const R* e, R Xc) {
  const R w0 = R(4) / R(9), w1 = R(1) / R(9), w5 = R(1) / R(36);
  const R se = w0 * e[0] + w1 * ((e[1] + e[2]) + (e[3] + e[4])) +
               w5 * ((e[5] + e[6]) + (e[7] + e[8]));
  const R sd = ((d[0] + (d[1] + d[2])) + (d[3] + d[4])) + ((d[5] + d[6]) + (d[7] + d[8]));
  const R dX = se + sd;
  const R Xn = Xc + dX;
  const R dR = Xn - Xc;
  d[0] += w0 * (e[0] - dR);
#pragma unroll
  for (int i = 1; i < 5; ++i) d[i] += w1 * (e[i] - dR);
#pragma unroll
  for (int i = 5; i < 9; ++i) d[i] += w5 * (e[i] - dR);
  return Xn;
}

// MRT collision of the flow LB (Eq. (29)) on h_1..h_8 (h[k] = h_{k+1}),
// with the equilibrium (30) and source (30)-(31) in moment form:
//   m_eq = (., rho ux, rho uy, P + Ax ux, P + Ay uy, (Ax uy + Ay ux)/2,
//           rho ux/3, rho uy/3, P/3 + A.u/3),  A = rho u - S,
//   m_H  = (B, Fx, Fy, B/3 + m2xx, B/3 + m2yy, m2xy, Fx/3, Fy/3,
//           B/9 + tr m2/3),  B = u.grad rho,
//   m2 = d_t(rho uu - (Su+uS)/2) + c_s^2 (u grad rho + grad rho u).
// The first moments become m1 + F whatever s1 is, since rho u = m1 + F/2.
template <class R>
__device__ __forceinline__ void collide_flow(R* h, const Front<R>& s, R s3, R s4) {
  const R a57 = h[4] + h[6], a68 = h[5] + h[7];
  const R d57 = h[4] - h[6], d68 = h[5] - h[7];
  R m5 = a57 - a68, m8 = a57 + a68;
  R m6 = d57 - d68, m7 = d57 + d68;
  R m1 = (h[0] - h[2]) + m6, m2 = (h[1] - h[3]) + m7;
  R m3 = (h[0] + h[2]) + m8, m4 = (h[1] + h[3]) + m8;
  const R ux = s.ux, uy = s.uy;
  const R Ax = s.jx - s.Sx, Ay = s.jy - s.Sy;
  const R Au = Ax * ux + Ay * uy;
  const R B = ux * s.grx + uy * s.gry;
  const R mxx = s.dTxx + third_of(R(2) * ux * s.grx);
  const R myy = s.dTyy + third_of(R(2) * uy * s.gry);
  const R mxy = s.dTxy + third_of(ux * s.gry + uy * s.grx);
  const R s2 = s.s2h, h2 = R(1) - R(0.5) * s2;
  const R h3 = R(1) - R(0.5) * s3, h4 = R(1) - R(0.5) * s4;
  m1 = m1 + s.Fx;
  m2 = m2 + s.Fy;
  m3 = m3 - s2 * (m3 - (s.P + Ax * ux)) + h2 * (third_of(B) + mxx);
  m4 = m4 - s2 * (m4 - (s.P + Ay * uy)) + h2 * (third_of(B) + myy);
  m5 = m5 - s2 * (m5 - R(0.5) * (Ax * uy + Ay * ux)) + h2 * mxy;
  m6 = m6 - s3 * (m6 - third_of(s.jx)) + h3 * third_of(s.Fx);
  m7 = m7 - s3 * (m7 - third_of(s.jy)) + h3 * third_of(s.Fy);
  m8 = m8 - s4 * (m8 - third_of(s.P + Au)) + h4 * (ninth_of(B) + third_of(mxx + myy));
  h[0] = R(0.5) * (m1 + m3 - m6 - m8);
  h[1] = R(0.5) * (m2 + m4 - m7 - m8);
  h[2] = R(0.5) * (-m1 + m3 + m6 - m8);
  h[3] = R(0.5) * (-m2 + m4 + m7 - m8);
  h[4] = R(0.25) * (m5 + m6 + m7 + m8);
  h[5] = R(0.25) * (-m5 - m6 + m7 + m8);
  h[6] = R(0.25) * (m5 - m6 - m7 + m8);
  h[7] = R(0.25) * (-m5 + m6 - m7 + m8);
}

// Front of one site under a prescribed velocity (Sec. 4.2): u is given, so
// only what the phase-field and surfactant collisions use is formed; the
// previous level's velocity is the same u.
template <class R>
__device__ __forceinline__ void site_front_prescribed(const Phys<R>& p, Front<R>& s, R phi,
                                                      R psi, R gfx, R gfy, R ux, R uy,
                                                      R php, R psp) {
  s.phi = phi;
  s.psi = psi;
  normal_delta(p, phi, gfx, gfy, s.nx, s.ny, s.delta);
  s.a = p.c4W * (p.phiAB - phi - phi);
  s.ux = ux;
  s.uy = uy;
  s.dpux = phi * ux - php * ux;
  s.dpuy = phi * uy - php * uy;
  s.dqux = psi * ux - psp * ux;
  s.dquy = psi * uy - psp * uy;
  s.rho = R(1);
  s.jx = s.jy = s.Sx = s.Sy = s.Fx = s.Fy = s.grx = s.gry = s.P = R(0);
  s.dTxx = s.dTxy = s.dTyy = s.s2h = R(0);
}

// The phase-field and surfactant collisions of one site (9 populations each).
template <class R, bool GENR>
__device__ __forceinline__ void collide_fg(const Phys<R>& p, const Front<R>& s, R* f, R* g) {
  // phase field: V = 3 d_t(phi u) + delta n  (Eq. (22))
  collide_cde(f, s.phi, s.ux, s.uy, R(3) * s.dpux + s.delta * s.nx,
              R(3) * s.dpuy + s.delta * s.ny, p.s1f, p.s2f, p.s3f, p.s4f);
  // surfactant: V = 3 d_t(psi u) + j, j = r a psi n - (r-1)(n.grad psi) n;
  // at r = 1, j = a psi n exactly as in Eq. (26)
  R jx, jy;
  if (GENR) {
    const R ndg = s.nx * s.gpx + s.ny * s.gpy;
    const R k = p.r * s.a * s.psi - p.rm1 * ndg;
    jx = k * s.nx;
    jy = k * s.ny;
  } else {
    const R k = s.a * s.psi;
    jx = k * s.nx;
    jy = k * s.ny;
  }
  collide_cde(g, s.psi, s.ux, s.uy, R(3) * s.dqux + jx, R(3) * s.dquy + jy,
              p.s1g, p.s2g, p.s3g, p.s4g);
}

// The three collisions of one site.  f, g: 9 populations; h: h_1..h_8.
template <class R, bool GENR>
__device__ __forceinline__ void collide_site(const Phys<R>& p, const Front<R>& s,
                                             R* f, R* g, R* h) {
  collide_fg<R, GENR>(p, s, f, g);
  collide_flow(h, s, p.s3h, p.s4h);
}

}  // namespace lbm
