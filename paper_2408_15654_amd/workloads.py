"""Seeded synthetic problems shaped like the paper's workloads.

This module only builds INPUTS: a plain parameter dictionary and the initial
macroscopic fields (phi, psi, ux, uy) as float64 arrays of shape (ny, nx),
x fastest.  It contains none of the lattice Boltzmann arithmetic; the library
and the CPU oracle each turn these inputs into populations on their own.

Initial interface profiles follow the one-dimensional equilibria of the paper:
phi = (phiA+phiB)/2 + (phiA-phiB)/2 tanh(2 d / W) with d the signed distance to
the drop boundary (Sec. 2.1, Eq. (7)), and interface-confined surfactant
psi = psi_0 * 4 (phiA-phi)(phi-phiB)/(phiA-phiB)^2, the unit-peak form of
Eq. (13).

Parameter dictionary keys (all lattice units, dx = dt = 1):
  nx, ny            grid size; x is always periodic
  walls_y           0 periodic in y, 1 half-way bounce-back walls
  u_wall_bot/top    tangential wall speeds
  phiA, phiB        order-parameter values of fluids A and B
  W, M, D, r        interface width, mobility, surfactant diffusivity,
                    normal-diffusion ratio (Eqs. (3), (6), (9))
  rhoA, rhoB, muA, muB   densities and dynamic viscosities (Eq. (15))
  sigma0, beta, eos surface tension, elasticity E_0, 'linear' or 'langmuir'
  gx, gy            body force per unit mass
  s_free            3x3 free relaxation rates (f: s2,s3,s4; g: s2,s3,s4;
                    h: s1,s3,s4), default all 1.0
  flow              'ns' (velocity from the Navier-Stokes LB, default) or
                    'prescribed' (u held at the initial field, Sec. 4.2)
  precision         'fp64', 'fp32' or 'fp16dev' (library only)
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 240815654


@dataclasses.dataclass
class Problem:
    name: str
    params: dict
    phi0: np.ndarray
    psi0: np.ndarray
    ux0: np.ndarray
    uy0: np.ndarray
    steps: int

    @property
    def fields0(self):
        return self.phi0, self.psi0, self.ux0, self.uy0

    @property
    def sites(self) -> int:
        return int(self.params["nx"]) * int(self.params["ny"])


def base_params(nx: int, ny: int, **kw) -> dict:
    p = dict(nx=nx, ny=ny, walls_y=0, u_wall_bot=0.0, u_wall_top=0.0, phiA=1.0,
             phiB=0.0, W=4.0, M=0.02, D=0.01, r=1.0, rhoA=1.0, rhoB=1.0,
             muA=0.1, muB=0.1, sigma0=1e-3, beta=0.0, eos="linear", gx=0.0,
             gy=0.0, s_free=[[1.0] * 3 for _ in range(3)], precision="fp64")
    p.update(kw)
    return p


def tanh_profile(d: np.ndarray, W: float, phiA=1.0, phiB=0.0) -> np.ndarray:
    """phi as a function of signed distance d (positive inside fluid A)."""
    return 0.5 * (phiA + phiB) + 0.5 * (phiA - phiB) * np.tanh(2.0 * d / W)


def unit_peak(phi: np.ndarray, phiA=1.0, phiB=0.0) -> np.ndarray:
    return 4.0 * (phiA - phi) * (phi - phiB) / (phiA - phiB) ** 2


def _grid(nx, ny):
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    return x, y


def _periodic_delta(a, c, n):
    d = a - c
    return d - n * np.round(d / n)


def single_drop(nx, ny, R, cx=None, cy=None, W=4.0, periodic_y=True):
    x, y = _grid(nx, ny)
    cx = nx / 2.0 if cx is None else cx
    cy = ny / 2.0 if cy is None else cy
    dx = _periodic_delta(x, cx, nx)
    dy = _periodic_delta(y, cy, ny) if periodic_y else y - cy
    rr = np.hypot(dx, dy)
    theta = np.arctan2(dy, dx)
    phi = tanh_profile(R - rr, W)
    return phi, theta


# ----------------------------------------------------------------- configs

def c1_stationary_drop(beta=0.3, r=0.0, psi_mode=0.5, steps=2000, **kw) -> Problem:
    """64x64 periodic, drop R=16 at the centre, W=4, equal density/viscosity,
    tau_f = 0.8, M=0.02, D=0.01, r=0, sigma0=1e-3, linear EOS beta=0.3,
    psi = (1 + 0.5 cos theta) * unit-peak profile, u = 0, 2000 steps."""
    nx = ny = 64
    p = base_params(nx, ny, W=4.0, M=0.02, D=0.01, r=r, rhoA=1.0, rhoB=1.0,
                    muA=0.1, muB=0.1, sigma0=1e-3, beta=beta)
    p.update(kw)
    phi, th = single_drop(nx, ny, 16.0, W=p["W"])
    psi = (1.0 + psi_mode * np.cos(th)) * unit_peak(phi)
    z = np.zeros_like(phi)
    return Problem("c1_drop64", p, phi, psi, z, z.copy(), steps)


def c2_shear_drop(beta=0.5, steps=20000, nx=256, ny=128, R=32.0, U=0.01,
                  Re=0.1, Ca=0.2, **kw) -> Problem:
    """Drop in simple shear between moving walls: 256x128, R=32, W=4, rho=1,
    walls at -U (bottom) and +U (top), Re = rho gdot R^2/mu, Ca = mu gdot R/sigma0,
    D=0.005, M=0.02, r=1, psi_0 = 1, linear EOS, initial linear shear profile."""
    H = float(ny)
    gdot = 2.0 * U / H
    mu = gdot * R * R / Re
    sigma0 = mu * gdot * R / Ca
    p = base_params(nx, ny, walls_y=1, u_wall_bot=-U, u_wall_top=U, W=4.0,
                    M=0.02, D=0.005, r=1.0, rhoA=1.0, rhoB=1.0, muA=mu, muB=mu,
                    sigma0=sigma0, beta=beta)
    p.update(kw)
    phi, _ = single_drop(nx, ny, R, cx=nx / 2.0, cy=(ny - 1) / 2.0, W=p["W"],
                         periodic_y=False)
    psi = unit_peak(phi)
    x, y = _grid(nx, ny)
    ux = U * (2.0 * (y + 0.5) / H - 1.0)
    return Problem("c2_shear256x128", p, phi, psi, ux, np.zeros_like(ux), steps)


def _random_streamfunction_velocity(nx, ny, rng, kmax=8, umax=1e-3):
    """Divergence-free u = curl(psi_s), psi_s a sum of Fourier modes with
    1 <= |k|_inf <= kmax, amplitudes N(0,1)/|k|^2, normalised to max|u|."""
    xs = 2 * math.pi * np.arange(nx) / nx
    ys = 2 * math.pi * np.arange(ny) / ny
    # psi_s = a cos(ph) + b sin(ph), ph = kx x + ky y, so
    # u = (ky', -kx') (-a sin(ph) + b cos(ph)) with k' = 2 pi k / n; the
    # separable forms sin(ph) = sy cx + cy sx, cos(ph) = cy cx - sy sx turn
    # the sum over modes into one matrix product per component.
    ycols, xcols, cu, cv = [], [], [], []
    for kx in range(-kmax, kmax + 1):
        for ky in range(0, kmax + 1):
            if ky == 0 and kx <= 0:
                continue
            k2 = kx * kx + ky * ky
            a, b = rng.standard_normal(2) / k2
            sx, cx = np.sin(kx * xs), np.cos(kx * xs)
            sy, cy = np.sin(ky * ys), np.cos(ky * ys)
            # -a sin(ph) + b cos(ph) = (-a) sy cx + (-a) cy sx + b cy cx - b sy sx
            for yv, xv, c in ((sy, cx, -a), (cy, sx, -a), (cy, cx, b), (sy, sx, -b)):
                ycols.append(yv)
                xcols.append(xv)
                cu.append(c * 2 * math.pi * ky / ny)
                cv.append(-c * 2 * math.pi * kx / nx)
    Y = np.stack(ycols, axis=1)
    X = np.stack(xcols, axis=1)
    ux = (Y * np.array(cu)) @ X.T
    uy = (Y * np.array(cv)) @ X.T
    s = umax / np.hypot(ux, uy).max()
    return ux * s, uy * s


def many_drops(nx, ny, ndrops, rmin, rmax, gap, rng, W=4.0):
    """Non-overlapping circles (periodic), rejection sampled with an interface
    gap >= gap.  Returns phi, index of the nearest drop per site, centres, radii.
    Each drop's signed distance is evaluated in a window reaching 12 W past
    its rim, beyond which the profile equals its bulk value to 1e-20."""
    cs, rs = [], []
    tries = 0
    while len(cs) < ndrops:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place drops")
        R = rng.uniform(rmin, rmax)
        c = rng.uniform(0, [nx, ny])
        ok = True
        for c2, r2 in zip(cs, rs):
            d = np.abs(c - c2)
            d = np.minimum(d, [nx, ny] - d)
            if math.hypot(*d) < R + r2 + gap:
                ok = False
                break
        if ok:
            cs.append(c)
            rs.append(R)
    best = np.full((ny, nx), -np.inf)
    idx = np.zeros((ny, nx), dtype=np.int64)
    for j, (c, R) in enumerate(zip(cs, rs)):
        h = int(math.ceil(R + 12 * W))
        xi = np.arange(int(c[0]) - h, int(c[0]) + h + 1)
        yi = np.arange(int(c[1]) - h, int(c[1]) + h + 1)
        dx = _periodic_delta(xi.astype(float), c[0], nx)
        dy = _periodic_delta(yi.astype(float), c[1], ny)
        d = R - np.hypot(dx[None, :], dy[:, None])
        ix = np.ix_(yi % ny, xi % nx)
        sub = best[ix]
        m = d > sub
        sub[m] = d[m]
        best[ix] = sub
        isub = idx[ix]
        isub[m] = j
        idx[ix] = isub
    return tanh_profile(best, W), idx, np.array(cs), np.array(rs)


def c3_many_drops(precision="fp32", steps=5000, nx=2048, ny=2048, ndrops=400,
                  seed=None, **kw) -> Problem:
    """2048x2048 periodic, 400 drops R~U[8,24] with interface gap >= 3W,
    rhoA/rhoB = muA/muB = 10 (tau_f = 0.8 in both phases), sigma0=1e-3,
    beta=0.5, D=0.01, M=0.02, W=4, r=1, per-drop psi_0 ~ U[0.5,1.5],
    random divergence-free initial velocity with max|u| = 1e-3."""
    rng = np.random.default_rng(SEED_BASE + 3 if seed is None else seed)
    W = 4.0
    phi, idx, cs, rs = many_drops(nx, ny, ndrops, 8.0, 24.0, 3 * W, rng, W)
    psi0 = rng.uniform(0.5, 1.5, size=len(rs))
    psi = psi0[idx] * unit_peak(phi)
    ux, uy = _random_streamfunction_velocity(nx, ny, rng)
    p = base_params(nx, ny, W=W, M=0.02, D=0.01, r=1.0, rhoA=10.0, rhoB=1.0,
                    muA=1.0, muB=0.1, sigma0=1e-3, beta=0.5, precision=precision)
    p.update(kw)
    return Problem(f"c3_drops{nx}x{ny}", p, phi, psi, ux, uy, steps)


def shear_instance(rng, H, precision="fp32", steps=10000) -> Problem:
    """Drop in simple shear in a 2H x H channel with walls at -U/+U: R = H/4,
    Re = 0.1, nu = min(1.6, 0.0125 H), U = 8 Re nu / H, Ca ~ U[0.05,0.4]
    (sigma0 = nu U / (2 Ca)), beta ~ U[0,0.8], r in {0,1}, D=0.005, M=0.02."""
    H = int(H)
    L = 2 * H
    nu = min(1.6, 0.0125 * H)
    Re = 0.1
    U = 8 * Re * nu / H
    Ca = rng.uniform(0.05, 0.4)
    beta = rng.uniform(0.0, 0.8)
    r = float(rng.integers(0, 2))
    R = H / 4.0
    sigma0 = nu * U / (2 * Ca)
    p = base_params(L, H, walls_y=1, u_wall_bot=-U, u_wall_top=U, W=4.0, M=0.02,
                    D=0.005, r=r, rhoA=1.0, rhoB=1.0, muA=nu, muB=nu,
                    sigma0=sigma0, beta=beta, precision=precision)
    phi, _ = single_drop(L, H, R, cx=L / 2.0, cy=(H - 1) / 2.0, W=4.0,
                         periodic_y=False)
    psi = unit_peak(phi)
    x, y = _grid(L, H)
    ux = U * (2.0 * (y + 0.5) / H - 1.0)
    return Problem(f"shear{L}x{H}", p, phi, psi, ux, np.zeros_like(ux), steps)


def c4_instance(rng, precision="fp32", steps=10000) -> Problem:
    """One drop-in-shear instance of the batched sweep: site count log-uniform
    in [64^2, 512^2], aspect 2:1 (H = round(sqrt(N/2)), at least 16), then
    shear_instance."""
    N = math.exp(rng.uniform(math.log(64 ** 2), math.log(512 ** 2)))
    H = max(16, int(round(math.sqrt(N / 2))))
    return shear_instance(rng, H, precision=precision, steps=steps)


def c4_batch(n=256, seed=None, precision="fp32", steps=10000):
    rng = np.random.default_rng(SEED_BASE + 4 if seed is None else seed)
    return [c4_instance(rng, precision, steps) for _ in range(n)]


def migration_instance(rng, N, precision="fp32", steps=1000) -> Problem:
    """Marangoni migration: square periodic grid of N sites, drop R = sqrt(N)/4,
    psi = (1 + 0.5 cos theta) * unit-peak profile, nu = 0.1,
    sigma0 = mu 1e-3 / Ca, Ca ~ U[0.05,0.4], beta ~ U[0,0.8]."""
    n = max(32, int(round(math.sqrt(N))))
    R = n / 4.0
    Ca = rng.uniform(0.05, 0.4)
    beta = rng.uniform(0.0, 0.8)
    mu = 0.1
    p = base_params(n, n, W=4.0, M=0.02, D=0.01, r=1.0, muA=mu, muB=mu,
                    sigma0=mu * 1e-3 / Ca, beta=beta, precision=precision)
    phi, th = single_drop(n, n, R, W=4.0)
    psi = (1.0 + 0.5 * np.cos(th)) * unit_peak(phi)
    z = np.zeros_like(phi)
    return Problem(f"migration{n}", p, phi, psi, z, z.copy(), steps)


def e2_convection(nx=100, R=20.0, u=(0.05, 0.0), steps=2000, r=1.0, precision="fp64",
                  **kw) -> Problem:
    """Sec. 4.2 in lattice units: domain [-0.5,0.5]^2 with dx = 0.01,
    dt = 0.001 -> 100x100 periodic, R = 0.2 -> 20, W = 4, M_phi = 0.1 ->
    M = M_phi dt/dx^2 = 1.0, D = 0.2 -> 2.0, prescribed uniform u = (0.5, 0)
    -> 0.05, psi = phi initially; t = 2 -> 2000 steps (one crossing of the
    periodic domain)."""
    p = base_params(nx, nx, W=4.0, M=1.0, D=2.0, r=r, sigma0=0.0, beta=0.0,
                    flow="prescribed", precision=precision)
    p.update(kw)
    phi, _ = single_drop(nx, nx, R, W=4.0)
    ux = np.full_like(phi, u[0])
    uy = np.full_like(phi, u[1])
    return Problem("e2_convection", p, phi, phi.copy(), ux, uy, steps)


def e3_rising_bubble(beta=0.0, nx=240, precision="fp32", steps=None, M=0.02, g=None,
                     **kw) -> Problem:
    """Sec. 4.3 in lattice units: domain [-2R,2R] x [0,8R], R = 0.25,
    dx = 1/240, dt = dx^2 -> nx x 2nx with walls at the bottom and the top
    (no slip) and periodic x; bubble R = nx/4 centred at (nx/2, nx/2).  The
    bubble is fluid A here (phi = 1 inside), so the shape diagnostics give its
    centre of mass Y_c.  Re = 2 rho R sqrt(2gR)/mu = 35, Bo = 4 rho g R^2 /
    sigma0 = 10, Pe = 2R sqrt(2gR)/D = 10 with the heavy fluid's rho = 1,
    density and viscosity ratios 10, sqrt(2gR) = 0.7 in units of the domain
    width: nu = 0.01, g = 0.98 dx^3, D = 0.035.  psi from the unit-peak
    profile with psi_0 = 1; linear EOS with E_0 = beta.  t = 3 -> 3 nx^2
    steps.  M is not given in the paper (0.02 here)."""
    dx = 1.0 / nx
    R = nx / 4.0
    nu = 0.01
    g = 0.98 * dx ** 3 if g is None else g
    rho_h, rho_b = 1.0, 0.1
    mu_h, mu_b = nu * rho_h, nu * rho_b
    sigma0 = 4 * rho_h * g * R * R / 10.0
    D = 0.035
    p = base_params(nx, 2 * nx, walls_y=1, W=4.0, M=M, D=D, r=1.0, rhoA=rho_b, rhoB=rho_h,
                    muA=mu_b, muB=mu_h, sigma0=sigma0, beta=beta, gy=-g,
                    precision=precision)
    p.update(kw)
    phi, _ = single_drop(nx, 2 * nx, R, cx=nx / 2.0, cy=nx / 2.0, W=4.0, periodic_y=False)
    psi = unit_peak(phi)
    z = np.zeros_like(phi)
    return Problem(f"e3_bubble{nx}", p, phi, psi, z, z.copy(),
                   3 * nx * nx if steps is None else steps)


# ------------------------------------------------------- pin problems

def e1_surface_diffusion(nx=100, R=25.0, steps=200) -> Problem:
    """Sec. 4.1 in lattice units: domain [-2,2]^2 with dx=0.04, dt=0.005 ->
    100x100, R=25, W=4, M=0.1*dt/dx^2=0.3125, D=1*dt/dx^2=3.125, t=1 -> 200
    steps; psi_hat(theta,0) = (1 - cos theta)/2 carried by the unit-integral
    delta profile 4 phi (1-phi)/W.  sigma0 = 0 keeps u = 0 exactly."""
    p = base_params(nx, nx, W=4.0, M=0.3125, D=3.125, r=1.0, sigma0=0.0,
                    beta=0.0)
    phi, th = single_drop(nx, nx, R, W=4.0)
    psi = 0.5 * (1.0 - np.cos(th)) * unit_peak(phi) / p["W"]
    z = np.zeros_like(phi)
    return Problem("e1_surface_diffusion", p, phi, psi, z, z.copy(), steps)


def random_small(seed: int, nx=None, ny=None, walls=None, r=None, eos=None,
                 precision="fp64", steps=20, wall_drop=False) -> Problem:
    """Random small problem for parity tests: odd sizes, walls or periodic,
    r in {0,1,2}, linear or Langmuir EOS, density/viscosity ratios, random
    drop and velocity field.  wall_drop (with walls): the drop is centred on
    the bottom wall and fluid A is 3 or 10 times denser than fluid B, so
    the dense fluid lies against a moving wall."""
    rng = np.random.default_rng(SEED_BASE + 1000 + seed)
    nx = int(rng.integers(40, 130)) if nx is None else nx
    ny = int(rng.integers(20, 70)) if ny is None else ny
    walls = bool(rng.integers(0, 2)) if walls is None else walls
    r = float(rng.choice([0.0, 1.0, 2.0])) if r is None else r
    eos = str(rng.choice(["linear", "langmuir"])) if eos is None else eos
    rhoA = float(rng.choice([1.0, 3.0, 10.0]))
    if wall_drop:
        rhoA = float(rng.choice([3.0, 10.0]))
    muA = float(rng.uniform(0.05, 0.3))
    U = 0.02 if walls else 0.0
    p = base_params(nx, ny, walls_y=int(walls), u_wall_bot=-U * rng.uniform(0, 1),
                    u_wall_top=U * rng.uniform(0, 1), W=4.0,
                    M=float(rng.uniform(0.01, 0.1)), D=float(rng.uniform(0.005, 0.1)),
                    r=r, rhoA=rhoA, rhoB=1.0, muA=muA, muB=0.1,
                    sigma0=float(rng.uniform(1e-3, 1e-2)),
                    beta=float(rng.uniform(0.1, 0.6)), eos=eos,
                    gx=float(rng.uniform(-1e-6, 1e-6)), gy=float(rng.uniform(-1e-6, 1e-6)),
                    s_free=rng.uniform(0.8, 1.6, size=(3, 3)).tolist(),
                    precision=precision)
    R = min(nx, ny) * float(rng.uniform(0.2, 0.3))
    cy = (ny - 1) * rng.uniform(0.45, 0.55)
    if wall_drop:
        if not walls:
            raise ValueError("wall_drop needs walls")
        R = min(nx, 2 * ny) * 0.3
        cy = 0.0
    phi, th = single_drop(nx, ny, R, cx=nx * rng.uniform(0.4, 0.6), cy=cy, W=4.0,
                          periodic_y=not walls)
    psi = float(rng.uniform(0.3, 0.6)) * (1 + 0.4 * np.cos(th + rng.uniform(0, 6))) * unit_peak(phi)
    x, y = _grid(nx, ny)
    ux = 1e-3 * np.sin(2 * np.pi * y / ny + rng.uniform(0, 6)) * rng.uniform(0.5, 1)
    uy = 1e-3 * np.sin(2 * np.pi * x / nx + rng.uniform(0, 6)) * rng.uniform(0.5, 1)
    if walls:
        uy = uy * np.sin(np.pi * (y + 0.5) / ny)
    return Problem(f"random{seed}_{nx}x{ny}", p, phi, psi, ux, uy, steps)
