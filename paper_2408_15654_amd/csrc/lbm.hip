// HIP kernels and C ABI of the coupled three-field lattice Boltzmann library
// (phase field f, surfactant g, flow h; arXiv:2408.15654), for gfx950.
//
// State on the device (structure of arrays, x fastest, one plane per
// quantity, planes padded to 64 elements), two copies (ping-pong):
//   populations  planes 0-8: deviations d_i = f_i - w_i phi of the
//                post-collision phase-field populations from the rest
//                equilibrium of their own site; 9-17: the same for g with
//                psi; 18-25: h_1..h_8 (h_0 is never read: column 0 of M is
//                e_0 and rows 1-8 of M^-1 start with 0);
//   rest         planes phi, psi of the same (previous) time level.
// plus, updated in place (each site reads and writes only its own entries):
//   aux          planes ux, uy, Sx, Sy of the previous time level (the
//                first-order time differences need them; phi, psi come from
//                the rest planes);
//   scratch      float64 planes for host transfers and read-back.
// Storage type: float64, float32, or float16 with per-field power-of-two
// scales (deviations and h are small numbers; phi, psi stay float32).
//
// One time step is ONE launch of lbm_step_kernel.  Each wavefront owns a
// strip of 62 columns (plus one halo column on each side, lanes 0 and
// w+1) and walks down a tile of rows.  For each row it pulls the f and g
// deviations of the NEXT row, rebuilds that row's phi, psi (and sigma(psi))
// from them and the rest values of their source sites, keeps a three-row
// window of phi, psi, sigma in registers and takes x-neighbours from
// adjacent lanes with cross-lane moves, so the 9-point stencils need no LDS
// and no barrier.  The h populations and the previous level are read for
// the current row only, and every population is written once.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "lbm.h"
#include "lbm_device.h"

using namespace lbm;

namespace {

constexpr int kWave = 64;
constexpr int kStrip = kWave - 2;  // interior columns per wavefront
constexpr int kWavesPerBlock = 4;
constexpr int kPlanes = 26;
constexpr int kRest = 2;
constexpr int kAux = 4;
constexpr int kScratch = 8;
constexpr int kReduceBlocks = 1024;
constexpr int kReduceVals = 8;

// Storage precisions: S population type, A type of phi/psi/u/S planes,
// R arithmetic type, SCALED: populations carry power-of-two scales.
struct F64 {
  using S = double;
  using A = double;
  using R = double;
  static constexpr bool SCALED = false;
};
struct F32 {
  using S = float;
  using A = float;
  using R = float;
  static constexpr bool SCALED = false;
};
struct F16 {
  using S = _Float16;
  using A = float;
  using R = float;
  static constexpr bool SCALED = true;
};

template <class P>
struct Scales {
  typename P::R f, g, h;     // multiply before storing
  typename P::R fi, gi, hi;  // multiply after loading
};

template <class P>
__device__ __forceinline__ typename P::R ld(const typename P::S *p, long long i,
                                            typename P::R inv) {
  using R = typename P::R;
  if constexpr (P::SCALED)
    return R(p[i]) * inv;
  else
    return R(p[i]);
}
template <class P>
__device__ __forceinline__ void st(typename P::S *p, long long i, typename P::R v,
                                   typename P::R scale) {
  using S = typename P::S;
  if constexpr (P::SCALED)
    p[i] = S(v * scale);
  else
    p[i] = S(v);
}

template <class P>
struct StepArgs {
  Phys<typename P::R> p;
  Scales<P> sc;
  const typename P::S *src;
  const typename P::A *src_rest;
  typename P::S *dst;
  typename P::A *dst_rest;
  typename P::A *aux;
  int *flag;
  long long plane;
  int nx, ny, walls;
  int nstrips, ntiles, rows;
};

// Row offsets and wall flags for pulling row y.
struct RowIdx {
  long long rc, rm, rp;  // offsets of rows y, y-1, y+1 (valid even at walls)
  bool bot, top;         // row y touches the bottom / top wall
};

__device__ __forceinline__ RowIdx row_index(int y, int nx, int ny, int walls) {
  RowIdx r;
  int ym = y - 1, yp = y + 1;
  r.bot = walls && y == 0;
  r.top = walls && y == ny - 1;
  if (ym < 0) ym = walls ? y : ym + ny;
  if (yp >= ny) yp = walls ? y : yp - ny;
  r.rc = (long long)y * nx;
  r.rm = (long long)ym * nx;
  r.rp = (long long)yp * nx;
  return r;
}

// Row y of the lattice for a row index that may lie one or two rows
// outside: periodic wrap, or clamped between walls (clamped rows are only
// read where the bounce-back makes their value irrelevant).
__device__ __forceinline__ int wrap_row(int y, int ny, int walls) {
  if (walls) return y < 0 ? 0 : (y >= ny ? ny - 1 : y);
  return y < 0 ? y + ny : (y >= ny ? y - ny : y);
}

// Pull streaming of one 9-population field to site (x, row): population i
// comes from x - c_i; across a wall it is the opposite population of the
// site itself (half-way bounce-back, no flux).
template <class P>
__device__ __forceinline__ void pull9(const typename P::S *__restrict__ s, long long pl,
                                      const RowIdx &r, int x, int xm, int xp,
                                      typename P::R inv, typename P::R *f) {
  f[0] = ld<P>(s, r.rc + x, inv);
  f[1] = ld<P>(s, pl + r.rc + xm, inv);
  f[2] = r.bot ? ld<P>(s, 4 * pl + r.rc + x, inv) : ld<P>(s, 2 * pl + r.rm + x, inv);
  f[3] = ld<P>(s, 3 * pl + r.rc + xp, inv);
  f[4] = r.top ? ld<P>(s, 2 * pl + r.rc + x, inv) : ld<P>(s, 4 * pl + r.rp + x, inv);
  f[5] = r.bot ? ld<P>(s, 7 * pl + r.rc + x, inv) : ld<P>(s, 5 * pl + r.rm + xm, inv);
  f[6] = r.bot ? ld<P>(s, 8 * pl + r.rc + x, inv) : ld<P>(s, 6 * pl + r.rm + xp, inv);
  f[7] = r.top ? ld<P>(s, 5 * pl + r.rc + x, inv) : ld<P>(s, 7 * pl + r.rp + xp, inv);
  f[8] = r.top ? ld<P>(s, 6 * pl + r.rc + x, inv) : ld<P>(s, 8 * pl + r.rp + xm, inv);
}

// Pull of h_1..h_8 (planes 18-25); across a wall, bounce-back with Ladd's
// moving-wall term 2 w_i rho_w (c_i.u_w)/c_s^2 = rho_w c_ix u_w / 6 for the
// diagonal populations (rho_w = rho at the site at collision time).
template <class P>
__device__ __forceinline__ void pull_h(const typename P::S *__restrict__ s0, long long pl,
                                       const RowIdx &r, int x, int xm, int xp,
                                       typename P::R inv, typename P::R rho_w,
                                       typename P::R uwb, typename P::R uwt,
                                       typename P::R *h) {
  using R = typename P::R;
  const typename P::S *s = s0 + 18 * pl;  // s[(i-1) pl] is h_i
  const R kb = rho_w * uwb * R(1.0 / 6.0), kt = rho_w * uwt * R(1.0 / 6.0);
  h[0] = ld<P>(s, r.rc + xm, inv);
  h[1] = r.bot ? ld<P>(s, 3 * pl + r.rc + x, inv) : ld<P>(s, pl + r.rm + x, inv);
  h[2] = ld<P>(s, 2 * pl + r.rc + xp, inv);
  h[3] = r.top ? ld<P>(s, pl + r.rc + x, inv) : ld<P>(s, 3 * pl + r.rp + x, inv);
  h[4] = r.bot ? ld<P>(s, 6 * pl + r.rc + x, inv) + kb : ld<P>(s, 4 * pl + r.rm + xm, inv);
  h[5] = r.bot ? ld<P>(s, 7 * pl + r.rc + x, inv) - kb : ld<P>(s, 5 * pl + r.rm + xp, inv);
  h[6] = r.top ? ld<P>(s, 4 * pl + r.rc + x, inv) - kt : ld<P>(s, 6 * pl + r.rp + xp, inv);
  h[7] = r.top ? ld<P>(s, 5 * pl + r.rc + x, inv) + kt : ld<P>(s, 7 * pl + r.rp + xm, inv);
}

// Rest values of the nine source sites of a row r relative to the site's
// own value: e_i = X(x - c_i) - X(x); bounced populations come from the
// site itself (e_i = 0).  v holds X at rows r-1 (m), r (c), r+1 (n) of
// columns x-1 (L), x, x+1 (R).
template <class R>
__device__ __forceinline__ void source_offsets(const Nine<R> &v, bool bot, bool top, R *e) {
  const R c = v.c;
  e[0] = R(0);
  e[1] = v.cL - c;
  e[3] = v.cR - c;
  e[2] = bot ? R(0) : v.m - c;
  e[5] = bot ? R(0) : v.mL - c;
  e[6] = bot ? R(0) : v.mR - c;
  e[4] = top ? R(0) : v.n - c;
  e[7] = top ? R(0) : v.nR - c;
  e[8] = top ? R(0) : v.nL - c;
}

// Value of lane-1 / lane+1 of the wavefront.
template <class R>
__device__ __forceinline__ R from_left(R v) {
  return __shfl_up(v, 1, kWave);
}
template <class R>
__device__ __forceinline__ R from_right(R v) {
  return __shfl_down(v, 1, kWave);
}

template <class R>
__device__ __forceinline__ Nine<R> window(R m, R c, R n) {
  Nine<R> v;
  v.m = m;
  v.c = c;
  v.n = n;
  v.mL = from_left(m);
  v.mR = from_right(m);
  v.cL = from_left(c);
  v.cR = from_right(c);
  v.nL = from_left(n);
  v.nR = from_right(n);
  return v;
}

// One column of an old rest field with its two x-neighbours.  The halo
// lanes (0 and w+1) have no lane beyond them and read that neighbour.
template <class R>
struct Col3 {
  R L, C, Rt;
};

template <class A, class R>
__device__ __forceinline__ Col3<R> load_col3(const A *__restrict__ a, long long row,
                                             int x, int xm, int xp, int lane, int w) {
  Col3<R> c;
  c.C = R(a[row + x]);
  c.L = from_left(c.C);
  c.Rt = from_right(c.C);
  if (lane == 0) c.L = R(a[row + xm]);
  if (lane == w + 1) c.Rt = R(a[row + xp]);
  return c;
}

template <class R>
__device__ __forceinline__ Nine<R> nine_of(const Col3<R> &m, const Col3<R> &c,
                                           const Col3<R> &n) {
  Nine<R> v;
  v.mL = m.L;
  v.m = m.C;
  v.mR = m.Rt;
  v.cL = c.L;
  v.c = c.C;
  v.cR = c.Rt;
  v.nL = n.L;
  v.n = n.C;
  v.nR = n.Rt;
  return v;
}

// The fused step: pull-stream + boundaries, phi/psi/sigma, stencils, forces,
// closures, three MRT collisions, store.  See the file header.
template <class P, bool GENR, bool HAS_S>
__global__ void __launch_bounds__(256)
lbm_step_kernel(const StepArgs<P> a) {
  using R = typename P::R;
  using S = typename P::S;
  using A = typename P::A;
  const int lane = threadIdx.x & (kWave - 1);
  const int tile = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (tile >= a.ntiles) return;  // whole wavefronts only
  const int nx = a.nx, ny = a.ny, walls = a.walls;
  const int strip = tile % a.nstrips;
  const int chunk = tile / a.nstrips;
  const int x0 = strip * kStrip;
  const int w = min(kStrip, nx - x0);
  const bool interior = lane >= 1 && lane <= w;
  int xl = x0 - 1 + min(lane, w + 1);
  const int x = xl < 0 ? xl + nx : (xl >= nx ? xl - nx : xl);
  const int xm = x == 0 ? nx - 1 : x - 1;
  const int xp = x == nx - 1 ? 0 : x + 1;
  const int y0 = chunk * a.rows;
  const int y1 = min(y0 + a.rows, ny);
  const long long pl = a.plane;
  const S *__restrict__ src = a.src;
  const A *__restrict__ rX = a.src_rest;       // old phi
  const A *__restrict__ rY = a.src_rest + pl;  // old psi
  S *__restrict__ dst = a.dst;
  A *__restrict__ aux = a.aux;
  const Phys<R> &p = a.p;
  const Scales<P> &sc = a.sc;

  // old rest field at row y (wrapped or clamped) with x-neighbours
  auto col = [&](const A *f, int y) {
    return load_col3<A, R>(f, (long long)wrap_row(y, ny, walls) * nx, x, xm, xp, lane, w);
  };
  // new phi, psi, sigma of row r and its deviations (relative to them),
  // given the old rest fields at rows r-1, r, r+1
  auto advance = [&](int r, const Col3<R> &Xm, const Col3<R> &Xc, const Col3<R> &Xn,
                     const Col3<R> &Ym, const Col3<R> &Yc, const Col3<R> &Yn, R *d,
                     R *q, R &ph, R &ps, R &sg) {
    const RowIdx ri = row_index(r, nx, ny, walls);
    pull9<P>(src, pl, ri, x, xm, xp, sc.fi, d);
    pull9<P>(src + 9 * pl, pl, ri, x, xm, xp, sc.gi, q);
    R e[9];
    source_offsets(nine_of(Xm, Xc, Xn), ri.bot, ri.top, e);
    ph = restream(d, e, Xc.C);
    source_offsets(nine_of(Ym, Yc, Yn), ri.bot, ri.top, e);
    ps = restream(q, e, Yc.C);
    sg = sigma_of(p, ps);
  };

  Col3<R> X0 = col(rX, y0 - 1), X1 = col(rX, y0), X2 = col(rX, y0 + 1);
  Col3<R> Y0 = col(rY, y0 - 1), Y1 = col(rY, y0), Y2 = col(rY, y0 + 1);
  R dc[9], qc[9];
  R phc, psc, sgc, phm, psm, sgm;
  advance(y0, X0, X1, X2, Y0, Y1, Y2, dc, qc, phc, psc, sgc);
  if (walls && y0 == 0) {  // mirror ghost row below the bottom wall
    phm = phc;
    psm = psc;
    sgm = sgc;
  } else {
    R dt[9], qt[9];
    const Col3<R> Xa = col(rX, y0 - 2), Ya = col(rY, y0 - 2);
    advance(y0 == 0 ? ny - 1 : y0 - 1, Xa, X0, X1, Ya, Y0, Y1, dt, qt, phm, psm, sgm);
  }
  // window of old rest values: rows y-1 (X0), y (X1), y+1 (X2)

  for (int y = y0; y < y1; ++y) {
    const Col3<R> X3 = col(rX, y + 2), Y3 = col(rY, y + 2);
    // next row: its deviations are kept for the next iteration
    R dn[9], qn[9];
    R phn, psn, sgn;
    const bool ghost = walls && y + 1 == ny;
    if (!ghost) {
      advance(y + 1 == ny ? 0 : y + 1, X1, X2, X3, Y1, Y2, Y3, dn, qn, phn, psn, sgn);
    } else {  // mirror ghost row above the top wall
#pragma unroll
      for (int i = 0; i < 9; ++i) dn[i] = qn[i] = R(0);
      phn = phc;
      psn = psc;
      sgn = sgc;
    }

    // current row: h populations and the previous level
    const RowIdx r = row_index(y, nx, ny, walls);
    const long long k = r.rc + x;
    const R php = X1.C, psp = Y1.C;
    const R uxp = R(aux[k]), uyp = R(aux[pl + k]);
    R Sxp = R(0), Syp = R(0);
    if (HAS_S) {
      Sxp = R(aux[2 * pl + k]);
      Syp = R(aux[3 * pl + k]);
    }
    R h[8];
    pull_h<P>(src, pl, r, x, xm, xp, sc.hi, rho_of(p, php), p.uwb, p.uwt, h);

    // stencils from the register window
    const Nine<R> vphi = window(phm, phc, phn);
    const Nine<R> vsig = window(sgm, sgc, sgn);
    R gfx, gfy, gsx, gsy;
    grad9(vphi, gfx, gfy);
    grad9(vsig, gsx, gsy);
    const R lphi = lap9(vphi);

    Front<R> s;
    site_front<R, HAS_S>(p, s, phc, psc, sgc, gfx, gfy, lphi, gsx, gsy, h, php, psp, uxp,
                         uyp, Sxp, Syp);
    if (GENR) {
      const Nine<R> vpsi = window(psm, psc, psn);
      grad9(vpsi, s.gpx, s.gpy);
    } else {
      s.gpx = s.gpy = R(0);
    }
    collide_site<R, GENR>(p, s, dc, qc, h);

    if (interior) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        st<P>(dst, i * pl + k, dc[i], sc.f);
        st<P>(dst, (9 + i) * pl + k, qc[i], sc.g);
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) st<P>(dst, (18 + i) * pl + k, h[i], sc.h);
      a.dst_rest[k] = A(phc);
      a.dst_rest[pl + k] = A(psc);
      aux[k] = A(s.ux);
      aux[pl + k] = A(s.uy);
      if (HAS_S) {
        aux[2 * pl + k] = A(s.Sx);
        aux[3 * pl + k] = A(s.Sy);
      }
      if (!isfinite(phc + psc + s.ux + s.uy)) *a.flag = 1;
    }

    // slide the windows
    phm = phc;
    psm = psc;
    sgm = sgc;
    phc = phn;
    psc = psn;
    sgc = sgn;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      dc[i] = dn[i];
      qc[i] = qn[i];
    }
    X0 = X1;
    X1 = X2;
    X2 = X3;
    Y0 = Y1;
    Y1 = Y2;
    Y2 = Y3;
  }
}

// ------------------------------------------------------------ site kernels

// Neighbour of site (x, y) at offset (dx, dy) in {-1,0,1}^2: periodic in x;
// periodic in y or, between walls, the wall row itself (mirror ghost).
__device__ __forceinline__ long long nbr_index(int x, int y, int dx, int dy, int nx,
                                               int ny, int walls) {
  int xx = x + dx, yy = y + dy;
  xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
  if (walls) {
    yy = yy < 0 ? 0 : (yy >= ny ? ny - 1 : yy);
  } else {
    yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
  }
  return (long long)yy * nx + xx;
}

template <class T, class R>
__device__ __forceinline__ Nine<R> gather9(const T *a, int x, int y, int nx, int ny,
                                           int walls) {
  Nine<R> v;
  v.mL = R(a[nbr_index(x, y, -1, -1, nx, ny, walls)]);
  v.m = R(a[nbr_index(x, y, 0, -1, nx, ny, walls)]);
  v.mR = R(a[nbr_index(x, y, 1, -1, nx, ny, walls)]);
  v.cL = R(a[nbr_index(x, y, -1, 0, nx, ny, walls)]);
  v.c = R(a[nbr_index(x, y, 0, 0, nx, ny, walls)]);
  v.cR = R(a[nbr_index(x, y, 1, 0, nx, ny, walls)]);
  v.nL = R(a[nbr_index(x, y, -1, 1, nx, ny, walls)]);
  v.n = R(a[nbr_index(x, y, 0, 1, nx, ny, walls)]);
  v.nR = R(a[nbr_index(x, y, 1, 1, nx, ny, walls)]);
  return v;
}

template <class P>
struct SiteArgs {
  const typename P::S *src;
  const typename P::A *src_rest;
  typename P::S *dst;
  typename P::A *dst_rest;
  typename P::A *aux;
  double *scratch;  // kScratch float64 planes
  Scales<P> sc;
  long long plane;
  int nx, ny, walls;
};

// Initial state in float64: post-collision populations := equilibria of
// Eqs. (22), (26), (30) with P = 0 and S of Eq. (16) from the gradient of
// the initial phi; previous level := the initial fields.  Inputs are
// scratch planes 0-3 (phi, psi, ux, uy).  f and g are stored as deviations
// from w_i times the STORED rest value, so storing phi, psi in a narrower
// type leaves the populations themselves exact up to their own rounding.
template <class P>
__global__ void __launch_bounds__(256)
lbm_init_kernel(const SiteArgs<P> a, const Phys<double> p) {
  using A = typename P::A;
  using R = typename P::R;
  const long long n = (long long)a.nx * a.ny;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int x = int(k % a.nx), y = int(k / a.nx);
  const long long pl = a.plane;
  const double *phi0 = a.scratch, *psi0 = a.scratch + pl;
  const double *ux0 = a.scratch + 2 * pl, *uy0 = a.scratch + 3 * pl;
  const Nine<double> v = gather9<double, double>(phi0, x, y, a.nx, a.ny, a.walls);
  double gx, gy;
  grad9(v, gx, gy);
  const double phi = phi0[k], psi = psi0[k], ux = ux0[k], uy = uy0[k];
  const double gn = sqrt(gx * gx + gy * gy);
  const double inv = 1.0 / (gn + p.eps_n);
  const double delta = p.c4W * ((p.phiA - phi) * (phi - p.phiB));
  const double Sx = p.Mdrho * (gx - delta * gx * inv);
  const double Sy = p.Mdrho * (gy - delta * gy * inv);
  const double rho = rho_of(p, phi);
  const double jx = rho * ux, jy = rho * uy;
  const double Ax = jx - Sx, Ay = jy - Sy, Au = Ax * ux + Ay * uy;
  const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                       1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  const double phis = double(A(phi)), psis = double(A(psi));
  for (int i = 0; i < 9; ++i) {
    const double cu = cx[i] * ux + cy[i] * uy;
    st<P>(a.dst, i * pl + k, R(w[i] * (phi - phis) + w[i] * phi * 3.0 * cu), a.sc.f);
    st<P>(a.dst, (9 + i) * pl + k, R(w[i] * (psi - psis) + w[i] * psi * 3.0 * cu), a.sc.g);
    if (i > 0) {
      const double cj = cx[i] * jx + cy[i] * jy;
      const double cA = cx[i] * Ax + cy[i] * Ay;
      st<P>(a.dst, (17 + i) * pl + k, R(w[i] * (3.0 * cj + 4.5 * cA * cu - 1.5 * Au)),
            a.sc.h);
    }
  }
  a.dst_rest[k] = A(phi);
  a.dst_rest[pl + k] = A(psi);
  a.aux[k] = A(ux);
  a.aux[pl + k] = A(uy);
  a.aux[2 * pl + k] = A(Sx);
  a.aux[3 * pl + k] = A(Sy);
}

// Read-back, pass 1: phi, psi, sigma of the current level into scratch
// planes 5-7 (arithmetic type R), by the same streaming as the step.
template <class P>
__global__ void __launch_bounds__(256)
lbm_macro_scalars_kernel(const SiteArgs<P> a, const Phys<typename P::R> p) {
  using R = typename P::R;
  const long long n = (long long)a.nx * a.ny;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int x = int(k % a.nx), y = int(k / a.nx);
  const int xm = x == 0 ? a.nx - 1 : x - 1, xp = x == a.nx - 1 ? 0 : x + 1;
  const long long pl = a.plane;
  const RowIdx r = row_index(y, a.nx, a.ny, a.walls);
  R d[9], q[9], e[9];
  pull9<P>(a.src, pl, r, x, xm, xp, a.sc.fi, d);
  pull9<P>(a.src + 9 * pl, pl, r, x, xm, xp, a.sc.gi, q);
  const Nine<R> vx = gather9<typename P::A, R>(a.src_rest, x, y, a.nx, a.ny, a.walls);
  source_offsets(vx, r.bot, r.top, e);
  const R phi = restream(d, e, vx.c);
  const Nine<R> vy = gather9<typename P::A, R>(a.src_rest + pl, x, y, a.nx, a.ny, a.walls);
  source_offsets(vy, r.bot, r.top, e);
  const R psi = restream(q, e, vy.c);
  R *out = reinterpret_cast<R *>(a.scratch + 5 * pl);
  out[k] = phi;
  out[pl + k] = psi;
  out[2 * pl + k] = sigma_of(p, psi);
}

// Read-back, pass 2: u and P by the same closures as the step, float64
// phi, psi, ux, uy, P into scratch planes 0-4.
template <class P, bool HAS_S>
__global__ void __launch_bounds__(256)
lbm_macro_fields_kernel(const SiteArgs<P> a, const Phys<typename P::R> p) {
  using R = typename P::R;
  const long long n = (long long)a.nx * a.ny;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int x = int(k % a.nx), y = int(k / a.nx);
  const int xm = x == 0 ? a.nx - 1 : x - 1, xp = x == a.nx - 1 ? 0 : x + 1;
  const long long pl = a.plane;
  const R *sc = reinterpret_cast<const R *>(a.scratch + 5 * pl);
  const Nine<R> vphi = gather9<R, R>(sc, x, y, a.nx, a.ny, a.walls);
  const Nine<R> vsig = gather9<R, R>(sc + 2 * pl, x, y, a.nx, a.ny, a.walls);
  R gfx, gfy, gsx, gsy;
  grad9(vphi, gfx, gfy);
  grad9(vsig, gsx, gsy);
  const R lphi = lap9(vphi);
  const R php = R(a.src_rest[k]), psp = R(a.src_rest[pl + k]);
  const R uxp = R(a.aux[k]), uyp = R(a.aux[pl + k]);
  const R Sxp = HAS_S ? R(a.aux[2 * pl + k]) : R(0);
  const R Syp = HAS_S ? R(a.aux[3 * pl + k]) : R(0);
  const RowIdx r = row_index(y, a.nx, a.ny, a.walls);
  R h[8];
  pull_h<P>(a.src, pl, r, x, xm, xp, a.sc.hi, rho_of(p, php), p.uwb, p.uwt, h);
  Front<R> s;
  site_front<R, HAS_S>(p, s, vphi.c, sc[pl + k], vsig.c, gfx, gfy, lphi, gsx, gsy, h, php,
                       psp, uxp, uyp, Sxp, Syp);
  a.scratch[k] = double(s.phi);
  a.scratch[pl + k] = double(s.psi);
  a.scratch[2 * pl + k] = double(s.ux);
  a.scratch[3 * pl + k] = double(s.uy);
  a.scratch[4 * pl + k] = double(s.P);
}

// Float64 reductions over scratch planes 0-3 (phi, psi, ux, uy): per-block
// partial sums in a fixed order (wavefront shuffles, then LDS), then one
// block adds the partials in a fixed order.  Deterministic.
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, kWave));
  return v;
}

__global__ void __launch_bounds__(256)
lbm_reduce_kernel(const double *scratch, long long plane, long long n,
                  const Phys<double> p, double *partials) {
  double acc[kReduceVals] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const double phi = scratch[k], psi = scratch[plane + k];
    const double ux = scratch[2 * plane + k], uy = scratch[3 * plane + k];
    const double rho = rho_of(p, phi);
    const double u2 = ux * ux + uy * uy;
    acc[0] += phi;
    acc[1] += psi;
    acc[2] += rho * ux;
    acc[3] += rho * uy;
    acc[4] += 0.5 * rho * u2;
    acc[5] = fmax(acc[5], sqrt(u2));
    if (!isfinite(phi + psi + ux + uy)) acc[6] = 1.0;
  }
  __shared__ double lds[kReduceVals][256 / kWave];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
  for (int j = 0; j < 7; ++j) {
    const double v = (j == 5 || j == 6) ? wave_max(acc[j]) : wave_sum(acc[j]);
    if (lane == 0) lds[j][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const int j = threadIdx.x;
    double v = lds[j][0];
    for (int q = 1; q < 256 / kWave; ++q)
      v = (j == 5 || j == 6) ? fmax(v, lds[j][q]) : v + lds[j][q];
    partials[blockIdx.x * kReduceVals + j] = v;
  }
}

__global__ void __launch_bounds__(64)
lbm_reduce_final_kernel(const double *partials, int nblocks, double *out) {
  if (threadIdx.x >= 7) return;
  const int j = threadIdx.x;
  double v = partials[j];
  for (int b = 1; b < nblocks; ++b) {
    const double q = partials[b * kReduceVals + j];
    v = (j == 5 || j == 6) ? fmax(v, q) : v + q;
  }
  out[j] = v;
}

// ------------------------------------------------------------------ host

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t storage_size(int prec) {
  return prec == LBM_FP64 ? 8 : (prec == LBM_FP32 ? 4 : 2);
}
size_t field_size(int prec) { return prec == LBM_FP64 ? 8 : 4; }

struct Layout {
  long long plane;  // elements per plane
  size_t pop_bytes, rest_bytes, aux_bytes, scratch_bytes, partial_bytes;
  size_t off_pop[2], off_rest[2], off_aux, off_scratch, off_partial, off_flag, total;
};

Layout make_layout(const lbm_params &p) {
  Layout L;
  const long long n = (long long)p.nx * p.ny;
  L.plane = (long long)align_up((size_t)n, 64);
  L.pop_bytes = align_up((size_t)kPlanes * L.plane * storage_size(p.precision), 256);
  L.rest_bytes = align_up((size_t)kRest * L.plane * field_size(p.precision), 256);
  L.aux_bytes = align_up((size_t)kAux * L.plane * field_size(p.precision), 256);
  L.scratch_bytes = align_up((size_t)kScratch * L.plane * 8, 256);
  L.partial_bytes = align_up((size_t)(kReduceBlocks + 1) * kReduceVals * 8, 256);
  size_t o = 0;
  for (int c = 0; c < 2; ++c) {
    L.off_pop[c] = o;
    o += L.pop_bytes;
    L.off_rest[c] = o;
    o += L.rest_bytes;
  }
  L.off_aux = o;
  o += L.aux_bytes;
  L.off_scratch = o;
  o += L.scratch_bytes;
  L.off_partial = o;
  o += L.partial_bytes;
  L.off_flag = o;
  o += 256;
  L.total = o;
  return L;
}

std::string g_create_error;

const char *validate(const lbm_params *p) {
  if (!p) return "params is NULL";
  if (p->nx < 3 || p->ny < 3) return "nx and ny must be >= 3";
  if ((long long)p->nx * p->ny > (1LL << 31)) return "grid too large";
  if (p->walls_y != 0 && p->walls_y != 1) return "walls_y must be 0 or 1";
  if (p->eos != LBM_EOS_LINEAR && p->eos != LBM_EOS_LANGMUIR) return "unknown eos";
  if (p->precision != LBM_FP64 && p->precision != LBM_FP32 && p->precision != LBM_FP16DEV)
    return "unknown precision";
  if (p->reserved != 0) return "reserved must be 0";
  if (!(p->phiA > p->phiB)) return "phiA must exceed phiB";
  if (!(p->W > 0)) return "W must be > 0";
  if (!(p->M > 0) || !(p->D > 0)) return "M and D must be > 0 (tau > 1/2)";
  if (!(p->rhoA > 0) || !(p->rhoB > 0)) return "densities must be > 0";
  if (!(p->muA > 0) || !(p->muB > 0)) return "viscosities must be > 0";
  if (!(p->r >= 0)) return "r must be >= 0";
  if (!(p->sigma0 >= 0)) return "sigma0 must be >= 0";
  const double fin[] = {p->u_wall_bot, p->u_wall_top, p->beta, p->gx, p->gy};
  for (double v : fin)
    if (!std::isfinite(v)) return "non-finite parameter";
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      if (!(p->s_free[a][b] > 0 && p->s_free[a][b] < 2)) return "free rates must lie in (0, 2)";
  for (int a = 0; a < 3; ++a) {
    const double s = p->fp16_scale[a];
    if (s == 0) continue;
    int e;
    if (!(s > 0) || std::frexp(s, &e) != 0.5 || e < -30 || e > 31)
      return "fp16_scale entries must be 0 or powers of two in [2^-30, 2^30]";
  }
  return nullptr;
}

template <class R>
Phys<R> make_phys(const lbm_params &q) {
  Phys<R> p;
  const double dphi = q.phiA - q.phiB;
  const double drho = (q.rhoA - q.rhoB) / dphi;
  p.phiA = R(q.phiA);
  p.phiB = R(q.phiB);
  p.phiAB = R(q.phiA + q.phiB);
  p.c4W = R(4.0 / (q.W * dphi));
  p.cbulk = R(24.0 / (q.W * dphi * dphi * dphi * dphi));
  p.cW = R(1.5 * q.W / (dphi * dphi));
  p.rhoB = R(q.rhoB);
  p.drho = R(drho);
  p.muB = R(q.muB);
  p.dmu = R((q.muA - q.muB) / dphi);
  p.Mdrho = R(q.M * drho);
  p.gx = R(q.gx);
  p.gy = R(q.gy);
  p.sigma0 = R(q.sigma0);
  p.beta = R(q.beta);
  p.r = R(q.r);
  p.rm1 = R(q.r - 1.0);
  p.s1f = R(1.0 / (3.0 * q.M + 0.5));
  p.s2f = R(q.s_free[0][0]);
  p.s3f = R(q.s_free[0][1]);
  p.s4f = R(q.s_free[0][2]);
  p.s1g = R(1.0 / (3.0 * q.D + 0.5));
  p.s2g = R(q.s_free[1][0]);
  p.s3g = R(q.s_free[1][1]);
  p.s4g = R(q.s_free[1][2]);
  p.s3h = R(q.s_free[2][1]);
  p.s4h = R(q.s_free[2][2]);
  p.uwb = R(q.u_wall_bot);
  p.uwt = R(q.u_wall_top);
  p.psi_max = R(1.0 - 1e-9);
  // 1e-4 of the largest gradient of the equilibrium profile: inside drops,
  // where |grad phi| can fall below delta(phi), the sharpening flux must not
  // become anti-diffusive (it would amplify rounding differences)
  p.eps_n = R(1e-4 * dphi / q.W);
  p.eos = q.eos;
  return p;
}

// Default float16 scales: deviations of f and g are at most a few 1e-2 of
// their field, h_i are O(w_i (3P + 3 c.rho u)); the scales put the expected
// magnitudes near 2^4..2^8, well inside float16's normal range.
void fp16_scales(const lbm_params &q, double out[3]) {
  const double dflt[3] = {4096.0, 4096.0, 16384.0};
  for (int a = 0; a < 3; ++a) out[a] = q.fp16_scale[a] > 0 ? q.fp16_scale[a] : dflt[a];
}

template <class P>
Scales<P> make_scales(const lbm_params &q) {
  using R = typename P::R;
  Scales<P> s;
  double v[3] = {1.0, 1.0, 1.0};
  if (P::SCALED) fp16_scales(q, v);
  s.f = R(v[0]);
  s.g = R(v[1]);
  s.h = R(v[2]);
  s.fi = R(1.0 / v[0]);
  s.gi = R(1.0 / v[1]);
  s.hi = R(1.0 / v[2]);
  return s;
}

}  // namespace

struct lbm_handle {
  lbm_params p;
  Layout L;
  hipStream_t stream;
  char *ws;
  int cur;
  int64_t step;
  bool valid;
  int rows;
  bool genr, has_s;
  std::string err;
};

namespace {

lbm_status fail(lbm_handle *h, lbm_status s, const std::string &msg) {
  if (h)
    h->err = msg;
  else
    g_create_error = msg;
  return s;
}

lbm_status hip_check(lbm_handle *h, hipError_t e, const char *what) {
  if (e == hipSuccess) return LBM_OK;
  return fail(h, LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void *pops(lbm_handle *h, int which) { return h->ws + h->L.off_pop[which]; }
void *rest(lbm_handle *h, int which) { return h->ws + h->L.off_rest[which]; }
void *auxp(lbm_handle *h) { return h->ws + h->L.off_aux; }
double *scratch(lbm_handle *h) { return reinterpret_cast<double *>(h->ws + h->L.off_scratch); }
double *partials(lbm_handle *h) { return reinterpret_cast<double *>(h->ws + h->L.off_partial); }
int *flagp(lbm_handle *h) { return reinterpret_cast<int *>(h->ws + h->L.off_flag); }

template <class P>
SiteArgs<P> site_args(lbm_handle *h) {
  SiteArgs<P> a;
  a.src = static_cast<const typename P::S *>(pops(h, h->cur));
  a.src_rest = static_cast<const typename P::A *>(rest(h, h->cur));
  a.dst = static_cast<typename P::S *>(pops(h, h->cur));
  a.dst_rest = static_cast<typename P::A *>(rest(h, h->cur));
  a.aux = static_cast<typename P::A *>(auxp(h));
  a.scratch = scratch(h);
  a.sc = make_scales<P>(h->p);
  a.plane = h->L.plane;
  a.nx = h->p.nx;
  a.ny = h->p.ny;
  a.walls = h->p.walls_y;
  return a;
}

int default_rows(const lbm_params &p) {
  const long long strips = (p.nx + kStrip - 1) / kStrip;
  // aim for at least ~8192 wavefronts on large grids, but keep tiles tall
  // enough that the two extra halo rows stay a small overhead
  long long rows = strips * p.ny / 8192;
  if (rows < 8) rows = 8;
  if (rows > 64) rows = 64;
  return int(rows);
}

template <class P, bool GENR, bool HAS_S>
hipError_t launch_step(lbm_handle *h) {
  StepArgs<P> a;
  a.p = make_phys<typename P::R>(h->p);
  a.sc = make_scales<P>(h->p);
  a.src = static_cast<const typename P::S *>(pops(h, h->cur));
  a.src_rest = static_cast<const typename P::A *>(rest(h, h->cur));
  a.dst = static_cast<typename P::S *>(pops(h, h->cur ^ 1));
  a.dst_rest = static_cast<typename P::A *>(rest(h, h->cur ^ 1));
  a.aux = static_cast<typename P::A *>(auxp(h));
  a.flag = flagp(h);
  a.plane = h->L.plane;
  a.nx = h->p.nx;
  a.ny = h->p.ny;
  a.walls = h->p.walls_y;
  a.nstrips = (h->p.nx + kStrip - 1) / kStrip;
  a.rows = h->rows;
  a.ntiles = a.nstrips * ((h->p.ny + a.rows - 1) / a.rows);
  const int blocks = (a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL((lbm_step_kernel<P, GENR, HAS_S>), dim3(blocks),
                     dim3(kWave * kWavesPerBlock), 0, h->stream, a);
  return hipGetLastError();
}

template <class P>
hipError_t launch_step_prec(lbm_handle *h) {
  if (h->genr)
    return h->has_s ? launch_step<P, true, true>(h) : launch_step<P, true, false>(h);
  return h->has_s ? launch_step<P, false, true>(h) : launch_step<P, false, false>(h);
}

hipError_t run_step(lbm_handle *h) {
  switch (h->p.precision) {
    case LBM_FP64: return launch_step_prec<F64>(h);
    case LBM_FP32: return launch_step_prec<F32>(h);
    default: return launch_step_prec<F16>(h);
  }
}

template <class P>
hipError_t launch_macros(lbm_handle *h) {
  SiteArgs<P> a = site_args<P>(h);
  const long long n = (long long)h->p.nx * h->p.ny;
  const int blocks = int((n + 255) / 256);
  const Phys<typename P::R> p = make_phys<typename P::R>(h->p);
  hipLaunchKernelGGL((lbm_macro_scalars_kernel<P>), dim3(blocks), dim3(256), 0, h->stream,
                     a, p);
  if (h->has_s)
    hipLaunchKernelGGL((lbm_macro_fields_kernel<P, true>), dim3(blocks), dim3(256), 0,
                       h->stream, a, p);
  else
    hipLaunchKernelGGL((lbm_macro_fields_kernel<P, false>), dim3(blocks), dim3(256), 0,
                       h->stream, a, p);
  return hipGetLastError();
}

hipError_t run_macros(lbm_handle *h) {
  switch (h->p.precision) {
    case LBM_FP64: return launch_macros<F64>(h);
    case LBM_FP32: return launch_macros<F32>(h);
    default: return launch_macros<F16>(h);
  }
}

template <class P>
hipError_t launch_init(lbm_handle *h) {
  SiteArgs<P> a = site_args<P>(h);
  const long long n = (long long)h->p.nx * h->p.ny;
  const Phys<double> p = make_phys<double>(h->p);
  hipLaunchKernelGGL((lbm_init_kernel<P>), dim3(int((n + 255) / 256)), dim3(256), 0,
                     h->stream, a, p);
  return hipGetLastError();
}

hipError_t run_init(lbm_handle *h) {
  switch (h->p.precision) {
    case LBM_FP64: return launch_init<F64>(h);
    case LBM_FP32: return launch_init<F32>(h);
    default: return launch_init<F16>(h);
  }
}

// Reads the sticky device flag (synchronising); marks the state invalid.
lbm_status check_flag(lbm_handle *h) {
  int flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, flagp(h), sizeof(int), hipMemcpyDeviceToHost,
                                h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_check(h, e, "reading the non-finite flag");
  if (flag) {
    h->valid = false;
    return fail(h, LBM_ENONFINITE, "the device produced a non-finite value");
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(const lbm_params *params) {
  if (validate(params)) return 0;
  return make_layout(*params).total;
}

lbm_status lbm_create(const lbm_params *params, void *dev_ws, size_t ws_bytes,
                      void *hip_stream, lbm_handle **out) {
  if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (const char *m = validate(params)) return fail(nullptr, LBM_EINVAL, m);
  const Layout L = make_layout(*params);
  if (!dev_ws) return fail(nullptr, LBM_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(dev_ws) % 256)
    return fail(nullptr, LBM_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total) return fail(nullptr, LBM_ENOMEM, "workspace too small");
  lbm_handle *h = new (std::nothrow) lbm_handle();
  if (!h) return fail(nullptr, LBM_ENOMEM, "out of host memory");
  h->p = *params;
  h->L = L;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->ws = static_cast<char *>(dev_ws);
  h->cur = 0;
  h->step = 0;
  h->valid = false;
  h->rows = default_rows(*params);
  h->genr = params->r != 1.0;
  h->has_s = params->rhoA != params->rhoB;
  *out = h;
  return LBM_OK;
}

lbm_status lbm_init_fields(lbm_handle *h, const double *phi, const double *psi,
                           const double *ux, const double *uy) {
  if (!h) return LBM_EINVAL;
  if (!phi || !psi || !ux || !uy) return fail(h, LBM_EINVAL, "NULL field");
  const long long n = (long long)h->p.nx * h->p.ny;
  for (long long k = 0; k < n; ++k) {
    if (!std::isfinite(phi[k]) || !std::isfinite(psi[k]) || !std::isfinite(ux[k]) ||
        !std::isfinite(uy[k]))
      return fail(h, LBM_EINVAL, "non-finite initial value");
    if (h->p.eos == LBM_EOS_LANGMUIR && psi[k] >= 1.0)
      return fail(h, LBM_EINVAL, "Langmuir EOS needs psi < 1");
  }
  double *sc = scratch(h);
  const long long pl = h->L.plane;
  const double *src[4] = {phi, psi, ux, uy};
  for (int j = 0; j < 4; ++j) {
    hipError_t e = hipMemcpyAsync(sc + j * pl, src[j], n * sizeof(double),
                                  hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_check(h, e, "copying initial fields");
  }
  h->cur = 0;
  hipError_t e = run_init(h);
  if (e == hipSuccess) e = hipMemsetAsync(flagp(h), 0, sizeof(int), h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_check(h, e, "initialising");
  h->step = 0;
  h->valid = true;
  return LBM_OK;
}

lbm_status lbm_step(lbm_handle *h, int64_t nsteps) {
  if (!h) return LBM_EINVAL;
  if (nsteps < 0) return fail(h, LBM_EINVAL, "nsteps < 0");
  if (!h->valid) return fail(h, LBM_ESTATE, "no valid state");
  for (int64_t t = 0; t < nsteps; ++t) {
    hipError_t e = run_step(h);
    if (e != hipSuccess) return hip_check(h, e, "launching the step kernel");
    h->cur ^= 1;
    h->step += 1;
  }
  return LBM_OK;
}

lbm_status lbm_read_fields(lbm_handle *h, double *phi, double *psi, double *ux,
                           double *uy, double *P) {
  if (!h) return LBM_EINVAL;
  if (!h->valid) return fail(h, LBM_ESTATE, "no valid state");
  lbm_status st = check_flag(h);
  if (st != LBM_OK) return st;
  hipError_t e = run_macros(h);
  if (e != hipSuccess) return hip_check(h, e, "launching read-back kernels");
  const long long n = (long long)h->p.nx * h->p.ny;
  double *dst[5] = {phi, psi, ux, uy, P};
  for (int j = 0; j < 5; ++j) {
    if (!dst[j]) continue;
    e = hipMemcpyAsync(dst[j], scratch(h) + j * h->L.plane, n * sizeof(double),
                       hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_check(h, e, "copying fields");
  }
  e = hipStreamSynchronize(h->stream);
  return hip_check(h, e, "reading fields");
}

lbm_status lbm_moments(lbm_handle *h, lbm_moments_t *out) {
  if (!h) return LBM_EINVAL;
  if (!out) return fail(h, LBM_EINVAL, "out is NULL");
  if (!h->valid) return fail(h, LBM_ESTATE, "no valid state");
  lbm_status st = check_flag(h);
  if (st != LBM_OK) return st;
  hipError_t e = run_macros(h);
  if (e != hipSuccess) return hip_check(h, e, "launching read-back kernels");
  const Phys<double> p = make_phys<double>(h->p);
  double *part = partials(h);
  const long long n = (long long)h->p.nx * h->p.ny;
  hipLaunchKernelGGL(lbm_reduce_kernel, dim3(kReduceBlocks), dim3(256), 0, h->stream,
                     (const double *)scratch(h), h->L.plane, n, p, part);
  hipLaunchKernelGGL(lbm_reduce_final_kernel, dim3(1), dim3(64), 0, h->stream,
                     (const double *)part, kReduceBlocks, part + kReduceBlocks * kReduceVals);
  e = hipGetLastError();
  double v[kReduceVals];
  if (e == hipSuccess)
    e = hipMemcpyAsync(v, part + kReduceBlocks * kReduceVals, sizeof v,
                       hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_check(h, e, "reducing");
  out->step = h->step;
  out->sum_phi = v[0];
  out->sum_psi = v[1];
  out->mom_x = v[2];
  out->mom_y = v[3];
  out->kinetic = v[4];
  out->max_u = v[5];
  out->nonfinite = v[6] != 0.0;
  out->pad = 0;
  if (out->nonfinite) {
    h->valid = false;
    return fail(h, LBM_ENONFINITE, "non-finite macroscopic field");
  }
  return LBM_OK;
}

size_t lbm_state_bytes(const lbm_handle *h) {
  if (!h) return 0;
  return sizeof(int64_t) + h->L.pop_bytes + h->L.rest_bytes + h->L.aux_bytes;
}

lbm_status lbm_get_state(lbm_handle *h, void *host_buf, size_t bytes) {
  if (!h) return LBM_EINVAL;
  if (!host_buf || bytes != lbm_state_bytes(h)) return fail(h, LBM_EINVAL, "bad buffer");
  if (!h->valid) return fail(h, LBM_ESTATE, "no valid state");
  lbm_status st = check_flag(h);
  if (st != LBM_OK) return st;
  char *b = static_cast<char *>(host_buf);
  std::memcpy(b, &h->step, sizeof(int64_t));
  b += sizeof(int64_t);
  const void *parts[3] = {pops(h, h->cur), rest(h, h->cur), auxp(h)};
  const size_t sizes[3] = {h->L.pop_bytes, h->L.rest_bytes, h->L.aux_bytes};
  hipError_t e = hipSuccess;
  for (int j = 0; j < 3 && e == hipSuccess; ++j) {
    e = hipMemcpyAsync(b, parts[j], sizes[j], hipMemcpyDeviceToHost, h->stream);
    b += sizes[j];
  }
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return hip_check(h, e, "saving state");
}

lbm_status lbm_set_state(lbm_handle *h, const void *host_buf, size_t bytes) {
  if (!h) return LBM_EINVAL;
  if (!host_buf || bytes != lbm_state_bytes(h)) return fail(h, LBM_EINVAL, "bad buffer");
  const char *b = static_cast<const char *>(host_buf);
  int64_t step;
  std::memcpy(&step, b, sizeof(int64_t));
  b += sizeof(int64_t);
  h->cur = 0;
  void *parts[3] = {pops(h, 0), rest(h, 0), auxp(h)};
  const size_t sizes[3] = {h->L.pop_bytes, h->L.rest_bytes, h->L.aux_bytes};
  hipError_t e = hipSuccess;
  for (int j = 0; j < 3 && e == hipSuccess; ++j) {
    e = hipMemcpyAsync(parts[j], b, sizes[j], hipMemcpyHostToDevice, h->stream);
    b += sizes[j];
  }
  if (e == hipSuccess) e = hipMemsetAsync(flagp(h), 0, sizeof(int), h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_check(h, e, "restoring state");
  h->step = step;
  h->valid = true;
  return LBM_OK;
}

void lbm_destroy(lbm_handle *h) { delete h; }

const char *lbm_last_error(const lbm_handle *h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

lbm_status lbm_set_tile_rows(lbm_handle *h, int32_t rows) {
  if (!h) return LBM_EINVAL;
  if (rows < 0 || rows > 4096) return fail(h, LBM_EINVAL, "rows out of range");
  h->rows = rows == 0 ? default_rows(h->p) : rows;
  return LBM_OK;
}

const char *lbm_step_kernel_name(const lbm_handle *h) {
  (void)h;
  return "lbm_step_kernel";
}

}  // extern "C"
