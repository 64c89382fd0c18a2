/*
 * FP64 CPU oracle of the phase-field lattice Boltzmann method for insoluble
 * surfactant transport in two-phase flows (Zhan, Liang, Chai, Shi,
 * arXiv:2408.15654).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  It shares no
 * code, header, table or constant with the HIP library.
 *
 * Everything is double precision, lattice units (dx = dt = c = 1), D2Q9.
 * Collisions are literal 9x9 matrix products m = M f, f* = M^-1 m*.
 *
 * The state kept between steps is the POST-COLLISION populations f*, g*, h*
 * of the previous step plus the previous time level's (phi, psi, u, S), which
 * the first-order time differences need.  One step is:
 *   stream (pull, half-way bounce-back at walls)   Sec. 4 intro
 *   phi = sum f, psi = sum g                       Eqs. (24), (27)
 *   rho, mu, sigma                                 Eqs. (15), (19)/(20)
 *   gradient / Laplacian stencils                  (not given by the paper)
 *   delta, n, S, F_s                               Eqs. (8), (16), (18)
 *   rho u, time differences, P                     Eqs. (32a), (32b)
 *   equilibria and sources                         Eqs. (22), (26), (30), (31)
 *   MRT collision in moment space                  Eqs. (21), (25), (29), (34)
 *
 * Readings where the paper is silent or garbled (each is listed with its
 * reason in the design notes of the repository):
 *   - phi_A, phi_B are parameters (tests use 1, 0).
 *   - The bulk term of the capillary force carries 1/(phi_A-phi_B)^2 twice,
 *     as differentiating the first line of Eq. (18) on the profile (7) gives.
 *   - Eq. (32a) is read as  rho u = sum c_i h_i + F/2  (sum c_i h_i^eq = rho u).
 *   - Stencils: isotropic D2Q9 differences, grad X = sum w_i c_i X(x+c_i)/cs2,
 *     lap X = sum 2 w_i (X(x+c_i)-X(x))/cs2; next to a wall the missing
 *     neighbour row is the wall row itself (mirror ghost).
 *   - Time derivatives: backward difference X(t) - X(t-1).
 *   - n = grad phi / (|grad phi| + eps), eps = 1e-4 (phiA - phiB) / W, i.e.
 *     1e-4 of the largest gradient of the profile (7).  Inside a drop,
 *     far from its rim, |grad phi| can fall below delta(phi) (at the centre
 *     it cancels to rounding level); there the sharpening flux with a unit
 *     normal would be anti-diffusive and the step would amplify rounding
 *     differences without bound.  With this eps the bulk stays diffusive,
 *     while at the interface (|grad phi| ~ 1/W) n is a unit vector to 1e-4.
 *   - General r: the source of the psi-LB carries
 *       j = r a psi n - (r-1) (n . grad psi) n,  a = 4(phiA+phiB-2phi)/(W dphi),
 *     from Eqs. (3)-(4) with psi = delta psi_hat and grad delta / delta = a n;
 *     at r = 1 this is exactly the source of Eq. (26).
 *   - Free relaxation rates (s2,s3,s4 of f and g; s1,s3,s4 of h; all s0) are
 *     parameters; s1 of h and every s0 provably do not affect the result.
 *   - Bounce-back: f and g plain (no flux); h with the moving-wall term
 *     2 w_i rho_w c_i.u_w / cs2, rho_w = rho(phi) of the boundary site at the
 *     time of the collision.
 *   - Initial state: post-collision populations are the equilibria of the
 *     initial fields (P = 0); the stored previous level is the initial fields,
 *     so the first time differences are taken against them.
 *   - Langmuir EOS: sigma uses min(psi, 1 - 1e-9) inside the logarithm.
 *   - Prescribed velocity (flow = 1, the setting of Sec. 4.2): u is the
 *     given initial field at every level, P = 0, only f and g evolve; the
 *     time differences become (phi - phi_prev) u and (psi - psi_prev) u.
 *
 * Every part is pinned by a test against a fact outside this file
 * (conservation, closed forms, moment conditions, symmetries, Laplace's
 * law, uniform acceleration, layered Couette flow).  In particular the
 * factor K = w0/(c^2 - c_s^2) of Eq. (32b) is fixed by the pressure of a
 * uniformly accelerated fluid staying constant, the Langmuir law (19) by
 * the Laplace jump of a drop with uniform surfactant, and the wall density
 * of the moving-wall term by no-slip Couette flow of a dense layer.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 9

/* D2Q9 velocities in the order fixed by rows 2-3 of M in Eq. (34). */
static const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double WT[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

/* Natural (raw-moment) transformation matrix, Eq. (34). */
static const double MM[Q][Q] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1}, {0, 1, 0, 1, 0, 1, 1, 1, 1},
    {0, 0, 1, 0, 1, 1, 1, 1, 1},    {0, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 1, -1, -1, 1},  {0, 0, 0, 0, 0, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, 1, 1, 1, 1}};

/* Its inverse, worked out by hand; the tests check MM * MINV = I exactly. */
static const double MINV[Q][Q] = {
    {1, 0, 0, -1, -1, 0, 0, 0, 1},
    {0, 0.5, 0, 0.5, 0, 0, -0.5, 0, -0.5},
    {0, 0, 0.5, 0, 0.5, 0, 0, -0.5, -0.5},
    {0, -0.5, 0, 0.5, 0, 0, 0.5, 0, -0.5},
    {0, 0, -0.5, 0, 0.5, 0, 0, 0.5, -0.5},
    {0, 0, 0, 0, 0, 0.25, 0.25, 0.25, 0.25},
    {0, 0, 0, 0, 0, -0.25, -0.25, 0.25, 0.25},
    {0, 0, 0, 0, 0, 0.25, -0.25, -0.25, 0.25},
    {0, 0, 0, 0, 0, -0.25, 0.25, -0.25, 0.25}};

/* Problem parameters (Sec. 2 and Sec. 3).  Field order is part of the ctypes
 * shim in oracle.py. */
typedef struct {
  int32_t nx, ny;
  int32_t walls_y; /* 0: periodic in y; 1: half-way bounce-back walls */
  int32_t eos;     /* 0: linear Eq. (20); 1: Langmuir Eq. (19) */
  int32_t flow;    /* 0: flow from the Navier-Stokes LB; 1: prescribed u */
  int32_t pad;
  double u_wall_bot, u_wall_top; /* tangential wall speeds */
  double phiA, phiB, W, M, D, r;
  double rhoA, rhoB, muA, muB;
  double sigma0, beta; /* beta is E_0 of Eqs. (19)-(20) */
  double gx, gy;       /* body force per unit mass, F_b = rho g */
  double s_free[3][3]; /* f: s2,s3,s4; g: s2,s3,s4; h: s1,s3,s4 */
  double s0;           /* s0 of all three fields */
  double rho0;         /* rho_0 of lambda_0, Eq. (30) */
} or_params;

/* Per-site macroscopic inputs of the equilibria and sources. */
typedef struct {
  double phi, psi, rho;
  double ux, uy;                 /* velocity u */
  double Sx, Sy;                 /* mass flux S, Eq. (16) */
  double P;                      /* pressure */
  double delta;                  /* Eq. (8) */
  double nx, ny;                 /* interface normal */
  double a;                      /* 4(phiA+phiB-2phi)/(W dphi) */
  double gpsix, gpsiy;           /* grad psi (general r only) */
  double dphiux, dphiuy;         /* d_t(phi u) */
  double dpsiux, dpsiuy;         /* d_t(psi u) */
  double dTxx, dTxy, dTyy;       /* d_t(rho uu - (Su+uS)/2) */
  double grhox, grhoy;           /* grad rho */
  double Fx, Fy;                 /* total force F = F_s + F_b */
} or_site;

static inline int site_index(int y, int x, int nx) { return y * nx + x; }

static int check_params(const or_params *p) {
  if (p->nx < 3 || p->ny < 3) return -1;
  if (!(p->phiA > p->phiB)) return -1;
  if (!(p->W > 0) || !(p->M > 0) || !(p->D > 0)) return -1;
  if (!(p->rhoA > 0) || !(p->rhoB > 0) || !(p->muA > 0) || !(p->muB > 0))
    return -1;
  if (!(p->r >= 0)) return -1;
  if (p->flow != 0 && p->flow != 1) return -1;
  return 0;
}

/* ---------------------------------------------------------------- EOS etc. */

/* Regularisation of the unit normal n = grad phi / (|grad phi| + eps). */
static double normal_eps(const or_params *p) {
  return 1e-4 * (p->phiA - p->phiB) / p->W;
}

/* Eq. (15). */
static double rho_of(const or_params *p, double phi) {
  return (phi - p->phiB) / (p->phiA - p->phiB) * (p->rhoA - p->rhoB) + p->rhoB;
}
static double mu_of(const or_params *p, double phi) {
  return (phi - p->phiB) / (p->phiA - p->phiB) * (p->muA - p->muB) + p->muB;
}

/* Eq. (20) (linear) or Eq. (19) (Langmuir). */
static double sigma_of(const or_params *p, double psi) {
  if (p->eos == 1) {
    double q = psi < 1.0 - 1e-9 ? psi : 1.0 - 1e-9;
    return p->sigma0 * (1.0 + p->beta * log(1.0 - q));
  }
  return p->sigma0 * (1.0 - p->beta * psi);
}

/* ------------------------------------------------------------ stencils */

/* Value of a site field at (x+dx, y+dy): periodic in x; periodic in y or,
 * between walls, the nearest row inside the domain (mirror ghost). */
static double nbr(const or_params *p, const double *a, int x, int y, int dx,
                  int dy) {
  int xx = ((x + dx) % p->nx + p->nx) % p->nx;
  int yy = y + dy;
  if (p->walls_y) {
    if (yy < 0) yy = 0;
    if (yy >= p->ny) yy = p->ny - 1;
  } else {
    yy = (yy % p->ny + p->ny) % p->ny;
  }
  return a[site_index(yy, xx, p->nx)];
}

static void grad(const or_params *p, const double *a, int x, int y, double *gx,
                 double *gy) {
  double sx = 0, sy = 0;
  for (int i = 1; i < Q; i++) {
    double v = nbr(p, a, x, y, CX[i], CY[i]);
    sx += WT[i] * CX[i] * v;
    sy += WT[i] * CY[i] * v;
  }
  *gx = sx / CS2;
  *gy = sy / CS2;
}

static double lap(const or_params *p, const double *a, int x, int y) {
  double c = a[site_index(y, x, p->nx)], s = 0;
  for (int i = 1; i < Q; i++) s += 2.0 * WT[i] * (nbr(p, a, x, y, CX[i], CY[i]) - c);
  return s / CS2;
}

/* Exported for the stencil tests. */
void or_stencils(const or_params *p, const double *a, double *gx, double *gy,
                 double *lp) {
  int nx = p->nx, ny = p->ny;
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      int k = site_index(y, x, nx);
      grad(p, a, x, y, &gx[k], &gy[k]);
      lp[k] = lap(p, a, x, y);
    }
}

/* ------------------------------------------------- equilibria and sources */

/* Eqs. (22), (26), (30) with (31); j for general r as stated at the top. */
void or_site_distributions(const or_params *p, const or_site *s,
                           double feq[Q], double Fsrc[Q], double geq[Q],
                           double Gsrc[Q], double heq[Q], double Hsrc[Q]) {
  const double dphi = p->phiA - p->phiB;
  (void)dphi;
  /* vector carried by the psi source besides d_t(psi u) */
  double ndg = s->nx * s->gpsix + s->ny * s->gpsiy;
  double jx = p->r * s->a * s->psi * s->nx - (p->r - 1.0) * ndg * s->nx;
  double jy = p->r * s->a * s->psi * s->ny - (p->r - 1.0) * ndg * s->ny;
  /* momentum and the tensor (rho u - S) u */
  double mx = s->rho * s->ux, my = s->rho * s->uy;
  double Ax = mx - s->Sx, Ay = my - s->Sy;
  double AU[2][2] = {{Ax * s->ux, Ax * s->uy}, {Ay * s->ux, Ay * s->uy}};
  /* m_2H of Eq. (31) */
  double m2[2][2];
  m2[0][0] = s->dTxx + CS2 * (s->ux * s->grhox + s->grhox * s->ux);
  m2[0][1] = s->dTxy + CS2 * (s->ux * s->grhoy + s->grhox * s->uy);
  m2[1][0] = s->dTxy + CS2 * (s->uy * s->grhox + s->grhoy * s->ux);
  m2[1][1] = s->dTyy + CS2 * (s->uy * s->grhoy + s->grhoy * s->uy);
  double udr = s->ux * s->grhox + s->uy * s->grhoy;

  for (int i = 0; i < Q; i++) {
    double cu = CX[i] * s->ux + CY[i] * s->uy;
    feq[i] = WT[i] * s->phi * (1.0 + cu / CS2);
    geq[i] = WT[i] * s->psi * (1.0 + cu / CS2);
    Fsrc[i] = WT[i] * (CX[i] * s->dphiux + CY[i] * s->dphiuy) / CS2 +
              WT[i] * s->delta * (CX[i] * s->nx + CY[i] * s->ny);
    Gsrc[i] = WT[i] * (CX[i] * s->dpsiux + CY[i] * s->dpsiuy) / CS2 +
              WT[i] * (CX[i] * jx + CY[i] * jy);

    double c[2] = {(double)CX[i], (double)CY[i]};
    /* Q_i = c_i c_i - cs2 I */
    double Qi[2][2] = {{c[0] * c[0] - CS2, c[0] * c[1]},
                       {c[1] * c[0], c[1] * c[1] - CS2}};
    double AUQ = 0, M2Q = 0;
    for (int a = 0; a < 2; a++)
      for (int b = 0; b < 2; b++) {
        AUQ += AU[a][b] * Qi[a][b];
        M2Q += m2[a][b] * Qi[a][b];
      }
    double lam = (i == 0) ? p->rho0 + (WT[0] - 1.0) * s->P / CS2
                          : WT[i] * s->P / CS2;
    heq[i] = lam + WT[i] * ((c[0] * mx + c[1] * my) / CS2 +
                            AUQ / (2.0 * CS2 * CS2));
    Hsrc[i] = WT[i] * (udr + (c[0] * s->Fx + c[1] * s->Fy) / CS2 +
                       M2Q / (2.0 * CS2 * CS2));
  }
}

/* Collision of Eqs. (21)/(25)/(29) done in moment space (Sec. 4 intro):
 *   m = M f,  m* = m - S (m - m_eq) + (I - S/2) M F,  f* = M^-1 m*. */
void or_collide(const double f[Q], const double feq[Q], const double F[Q],
                const double S[Q], double out[Q]) {
  double m[Q], me[Q], mf[Q], ms[Q];
  for (int k = 0; k < Q; k++) {
    m[k] = me[k] = mf[k] = 0;
    for (int j = 0; j < Q; j++) {
      m[k] += MM[k][j] * f[j];
      me[k] += MM[k][j] * feq[j];
      mf[k] += MM[k][j] * F[j];
    }
    ms[k] = m[k] - S[k] * (m[k] - me[k]) + (1.0 - S[k] / 2.0) * mf[k];
  }
  for (int i = 0; i < Q; i++) {
    out[i] = 0;
    for (int k = 0; k < Q; k++) out[i] += MINV[i][k] * ms[k];
  }
}

void or_matrices(double *M81, double *Minv81) {
  for (int i = 0; i < Q; i++)
    for (int j = 0; j < Q; j++) {
      M81[i * Q + j] = MM[i][j];
      Minv81[i * Q + j] = MINV[i][j];
    }
}

/* Relaxation vectors S^k = diag(s0,s1,s1,s2,s2,s2,s3,s3,s4), Eq. (34), with
 * s1^f from Eq. (23), s1^g from Eq. (28) and s2^h from Eq. (33). */
static void rates_f(const or_params *p, double S[Q]) {
  double s1 = 1.0 / (p->M / CS2 + 0.5);
  double v[Q] = {p->s0, s1, s1, p->s_free[0][0], p->s_free[0][0],
                 p->s_free[0][0], p->s_free[0][1], p->s_free[0][1],
                 p->s_free[0][2]};
  memcpy(S, v, sizeof v);
}
static void rates_g(const or_params *p, double S[Q]) {
  double s1 = 1.0 / (p->D / CS2 + 0.5);
  double v[Q] = {p->s0, s1, s1, p->s_free[1][0], p->s_free[1][0],
                 p->s_free[1][0], p->s_free[1][1], p->s_free[1][1],
                 p->s_free[1][2]};
  memcpy(S, v, sizeof v);
}
static void rates_h(const or_params *p, double rho, double mu, double S[Q]) {
  double s2 = 1.0 / (mu / (rho * CS2) + 0.5);
  double v[Q] = {p->s0,          p->s_free[2][0], p->s_free[2][0],
                 s2,             s2,              s2,
                 p->s_free[2][1], p->s_free[2][1], p->s_free[2][2]};
  memcpy(S, v, sizeof v);
}

/* --------------------------------------------------------- whole grid */

/* Per-site macroscopic fields of one time level. */
typedef struct {
  double *phi, *psi, *sig, *ux, *uy, *P;
  double *fpre, *gpre, *hpre; /* [Q][N] post-stream populations */
  double *site;               /* N or_site records, as doubles */
} front_t;

/* Pull streaming with half-way bounce-back (Sec. 4 intro). */
static void stream(const or_params *p, const double *fs, const double *gs,
                   const double *hs, const double *aux_phi, double *f,
                   double *g, double *h) {
  const int nx = p->nx, ny = p->ny;
  const size_t N = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      size_t k = site_index(y, x, nx);
      for (int i = 0; i < Q; i++) {
        int sx = x - CX[i], sy = y - CY[i];
        if (p->walls_y && (sy < 0 || sy >= ny)) {
          double uw = sy < 0 ? p->u_wall_bot : p->u_wall_top;
          double rw = rho_of(p, aux_phi[k]);
          f[i * N + k] = fs[OPP[i] * N + k];
          g[i * N + k] = gs[OPP[i] * N + k];
          h[i * N + k] = hs[OPP[i] * N + k] + 2.0 * WT[i] * rw * (CX[i] * uw) / CS2;
        } else {
          sx = (sx % nx + nx) % nx;
          sy = (sy % ny + ny) % ny;
          size_t ks = site_index(sy, sx, nx);
          f[i * N + k] = fs[i * N + ks];
          g[i * N + k] = gs[i * N + ks];
          h[i * N + k] = hs[i * N + ks];
        }
      }
    }
}

/* Stream, then everything up to (and including) the pressure, Eqs. (8),
 * (15)-(20), (24), (27), (32a), (32b).  aux holds the previous level's
 * (phi, psi, ux, uy, Sx, Sy). */
static void front_half(const or_params *p, const double *fs, const double *gs,
                       const double *hs, const double *aux, front_t *fr) {
  const int nx = p->nx, ny = p->ny;
  const size_t N = (size_t)nx * ny;
  const double dphi = p->phiA - p->phiB;
  const double drho = (p->rhoA - p->rhoB) / dphi;
  const double w0 = WT[0];
  const double K = w0 / (1.0 - CS2); /* K = w0 / (c^2 - cs^2), c = 1 */

  stream(p, fs, gs, hs, aux, fr->fpre, fr->gpre, fr->hpre);

#pragma omp parallel for schedule(static)
  for (size_t k = 0; k < N; k++) {
    double sf = 0, sg = 0;
    for (int i = 0; i < Q; i++) {
      sf += fr->fpre[i * N + k];
      sg += fr->gpre[i * N + k];
    }
    fr->phi[k] = sf;
    fr->psi[k] = sg;
    fr->sig[k] = sigma_of(p, sg);
  }

#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      size_t k = site_index(y, x, nx);
      or_site *s = (or_site *)(fr->site) + k;
      double phi = fr->phi[k], psi = fr->psi[k], sig = fr->sig[k];
      double gpx, gpy, gsx, gsy, gqx = 0, gqy = 0;
      grad(p, fr->phi, x, y, &gpx, &gpy);
      grad(p, fr->sig, x, y, &gsx, &gsy);
      grad(p, fr->psi, x, y, &gqx, &gqy);
      double lp = lap(p, fr->phi, x, y);
      double gn = sqrt(gpx * gpx + gpy * gpy);
      double eps = normal_eps(p);
      double nx_ = gpx / (gn + eps), ny_ = gpy / (gn + eps);
      double delta = 4.0 * (p->phiA - phi) * (phi - p->phiB) / (p->W * dphi);
      double a = 4.0 * (p->phiA + p->phiB - 2.0 * phi) / (p->W * dphi);
      double rho = rho_of(p, phi);
      /* Eq. (18): capillary part sigma mu_phi grad phi, Marangoni part */
      double muphi = 1.5 / (dphi * dphi) *
                     (16.0 * (p->phiA - phi) * (phi - p->phiB) *
                          (p->phiA + p->phiB - 2.0 * phi) / (p->W * dphi * dphi) -
                      p->W * lp);
      double cm = 1.5 * p->W / (dphi * dphi);
      double sdp = gsx * gpx + gsy * gpy;
      double Fx = sig * muphi * gpx + cm * (gn * gn * gsx - sdp * gpx) + rho * p->gx;
      double Fy = sig * muphi * gpy + cm * (gn * gn * gsy - sdp * gpy) + rho * p->gy;
      /* Eq. (16) */
      double Sx = p->M * drho * (gpx - delta * nx_);
      double Sy = p->M * drho * (gpy - delta * ny_);
      double grx = drho * gpx, gry = drho * gpy;
      /* Eq. (32a), read as rho u = sum c_i h_i + F/2 */
      double jx = 0, jy = 0, sum_h = 0;
      for (int i = 0; i < Q; i++) {
        double hi = fr->hpre[i * N + k];
        jx += CX[i] * hi;
        jy += CY[i] * hi;
        if (i != 0) sum_h += hi;
      }
      double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho;
      if (p->flow == 1) {
        /* prescribed velocity (Sec. 4.2): u is the given field, held in the
         * previous-level record and never replaced; no flow LB */
        ux = aux[2 * N + k];
        uy = aux[3 * N + k];
      }
      /* previous level */
      double php = aux[0 * N + k], psp = aux[1 * N + k];
      double uxp = aux[2 * N + k], uyp = aux[3 * N + k];
      double Sxp = aux[4 * N + k], Syp = aux[5 * N + k];
      double rhop = rho_of(p, php);
      double Txx = rho * ux * ux - Sx * ux;
      double Txy = rho * ux * uy - 0.5 * (Sx * uy + ux * Sy);
      double Tyy = rho * uy * uy - Sy * uy;
      double Txxp = rhop * uxp * uxp - Sxp * uxp;
      double Txyp = rhop * uxp * uyp - 0.5 * (Sxp * uyp + uxp * Syp);
      double Tyyp = rhop * uyp * uyp - Syp * uyp;
      double dTxx = Txx - Txxp, dTxy = Txy - Txyp, dTyy = Tyy - Tyyp;
      /* Eq. (32b), K = w0/(c^2-cs^2), d_t(rho u.u - S.u) = tr dT */
      double udr = ux * grx + uy * gry;
      double AU = (rho * ux - Sx) * ux + (rho * uy - Sy) * uy;
      double P = CS2 / (1.0 - w0) *
                 (sum_h + 0.5 * udr - w0 * AU / (2.0 * CS2) +
                  K * 0.5 * (dTxx + dTyy));
      if (p->flow == 1) P = 0.0;
      fr->ux[k] = ux;
      fr->uy[k] = uy;
      fr->P[k] = P;

      s->phi = phi; s->psi = psi; s->rho = rho;
      s->ux = ux; s->uy = uy; s->Sx = Sx; s->Sy = Sy; s->P = P;
      s->delta = delta; s->nx = nx_; s->ny = ny_; s->a = a;
      s->gpsix = gqx; s->gpsiy = gqy;
      s->dphiux = phi * ux - php * uxp; s->dphiuy = phi * uy - php * uyp;
      s->dpsiux = psi * ux - psp * uxp; s->dpsiuy = psi * uy - psp * uyp;
      s->dTxx = dTxx; s->dTxy = dTxy; s->dTyy = dTyy;
      s->grhox = grx; s->grhoy = gry;
      s->Fx = Fx; s->Fy = Fy;
    }
}

static int front_alloc(front_t *fr, size_t N) {
  memset(fr, 0, sizeof *fr);
  fr->phi = malloc(6 * N * sizeof(double));
  fr->fpre = malloc(3 * Q * N * sizeof(double));
  fr->site = malloc(N * sizeof(or_site));
  if (!fr->phi || !fr->fpre || !fr->site) {
    free(fr->phi); free(fr->fpre); free(fr->site);
    return -2;
  }
  fr->psi = fr->phi + N; fr->sig = fr->phi + 2 * N;
  fr->ux = fr->phi + 3 * N; fr->uy = fr->phi + 4 * N; fr->P = fr->phi + 5 * N;
  fr->gpre = fr->fpre + Q * N; fr->hpre = fr->fpre + 2 * Q * N;
  return 0;
}
static void front_free(front_t *fr) {
  free(fr->phi); free(fr->fpre); free(fr->site);
}

/* Initial state: post-collision populations = equilibria of the initial
 * fields with P = 0; S from Eq. (16) on the initial phi; previous level =
 * the initial fields. */
int or_init(const or_params *p, const double *phi0, const double *psi0,
            const double *ux0, const double *uy0, double *f, double *g,
            double *h, double *aux) {
  if (check_params(p)) return -1;
  const int nx = p->nx, ny = p->ny;
  const size_t N = (size_t)nx * ny;
  const double dphi = p->phiA - p->phiB;
  const double drho = (p->rhoA - p->rhoB) / dphi;
  for (size_t k = 0; k < N; k++)
    if (!isfinite(phi0[k]) || !isfinite(psi0[k]) || !isfinite(ux0[k]) ||
        !isfinite(uy0[k]))
      return -1;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      size_t k = site_index(y, x, nx);
      double phi = phi0[k];
      double gpx, gpy;
      grad(p, phi0, x, y, &gpx, &gpy);
      double gn = sqrt(gpx * gpx + gpy * gpy);
      double eps = normal_eps(p);
      double nx_ = gpx / (gn + eps), ny_ = gpy / (gn + eps);
      double delta = 4.0 * (p->phiA - phi) * (phi - p->phiB) / (p->W * dphi);
      or_site s;
      memset(&s, 0, sizeof s);
      s.phi = phi; s.psi = psi0[k]; s.rho = rho_of(p, phi);
      s.ux = ux0[k]; s.uy = uy0[k];
      s.Sx = p->M * drho * (gpx - delta * nx_);
      s.Sy = p->M * drho * (gpy - delta * ny_);
      s.P = 0.0;
      double feq[Q], F[Q], geq[Q], G[Q], heq[Q], H[Q];
      or_site_distributions(p, &s, feq, F, geq, G, heq, H);
      for (int i = 0; i < Q; i++) {
        f[i * N + k] = feq[i];
        g[i * N + k] = geq[i];
        h[i * N + k] = heq[i];
      }
      aux[0 * N + k] = phi; aux[1 * N + k] = psi0[k];
      aux[2 * N + k] = ux0[k]; aux[3 * N + k] = uy0[k];
      aux[4 * N + k] = s.Sx; aux[5 * N + k] = s.Sy;
    }
  return 0;
}

/* nsteps full time steps, in place on (f, g, h, aux). */
int or_step(const or_params *p, double *f, double *g, double *h, double *aux,
            int64_t nsteps) {
  if (check_params(p)) return -1;
  const size_t N = (size_t)p->nx * p->ny;
  front_t fr;
  if (front_alloc(&fr, N)) return -2;
  double Sf[Q], Sg[Q];
  rates_f(p, Sf);
  rates_g(p, Sg);
  for (int64_t t = 0; t < nsteps; t++) {
    front_half(p, f, g, h, aux, &fr);
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < N; k++) {
      const or_site *s = (const or_site *)(fr.site) + k;
      double feq[Q], F[Q], geq[Q], G[Q], heq[Q], H[Q], Sh[Q];
      double fi[Q], gi[Q], hi[Q], fo[Q], go[Q], ho[Q];
      or_site_distributions(p, s, feq, F, geq, G, heq, H);
      rates_h(p, s->rho, mu_of(p, s->phi), Sh);
      for (int i = 0; i < Q; i++) {
        fi[i] = fr.fpre[i * N + k];
        gi[i] = fr.gpre[i * N + k];
        hi[i] = fr.hpre[i * N + k];
      }
      or_collide(fi, feq, F, Sf, fo);
      or_collide(gi, geq, G, Sg, go);
      for (int i = 0; i < Q; i++) {
        f[i * N + k] = fo[i];
        g[i * N + k] = go[i];
      }
      aux[0 * N + k] = s->phi; aux[1 * N + k] = s->psi;
      if (p->flow == 1) continue; /* prescribed u: h and u are not evolved */
      or_collide(hi, heq, H, Sh, ho);
      for (int i = 0; i < Q; i++) h[i * N + k] = ho[i];
      aux[2 * N + k] = s->ux; aux[3 * N + k] = s->uy;
      aux[4 * N + k] = s->Sx; aux[5 * N + k] = s->Sy;
    }
  }
  front_free(&fr);
  return 0;
}

/* Macroscopic fields of the current time level (no collision). */
int or_macros(const or_params *p, const double *f, const double *g,
              const double *h, const double *aux, double *phi, double *psi,
              double *ux, double *uy, double *P) {
  if (check_params(p)) return -1;
  const size_t N = (size_t)p->nx * p->ny;
  front_t fr;
  if (front_alloc(&fr, N)) return -2;
  front_half(p, f, g, h, aux, &fr);
  for (size_t k = 0; k < N; k++) {
    if (phi) phi[k] = fr.phi[k];
    if (psi) psi[k] = fr.psi[k];
    if (ux) ux[k] = fr.ux[k];
    if (uy) uy[k] = fr.uy[k];
    if (P) P[k] = fr.P[k];
  }
  front_free(&fr);
  return 0;
}

/* Per-site equilibria/sources of the current time level, for tests that
 * check the moment conditions (Appendix A) on a running state. */
int or_site_fields(const or_params *p, const double *f, const double *g,
                   const double *h, const double *aux, or_site *out) {
  if (check_params(p)) return -1;
  const size_t N = (size_t)p->nx * p->ny;
  front_t fr;
  if (front_alloc(&fr, N)) return -2;
  front_half(p, f, g, h, aux, &fr);
  memcpy(out, fr.site, N * sizeof(or_site));
  front_free(&fr);
  return 0;
}

int or_sizeof_site(void) { return (int)sizeof(or_site); }
int or_sizeof_params(void) { return (int)sizeof(or_params); }

/* Thread count of the OpenMP loops (the results do not depend on it). */
void or_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int or_get_threads(void) { return omp_get_max_threads(); }
