"""Parity of the HIP library (through the C ABI) with the FP64 CPU oracle.

Relative L-infinity error per field: e(X) = max|X_gpu - X_oracle| /
max|X_oracle| for phi, psi and P; for the velocity the vector form
e(u) = max|u_gpu - u_oracle| / max|u_oracle| (|.| the Euclidean norm), so a
small cross-flow component is measured against the flow speed.  Bars: 1e-12
for float64 storage, 1e-5 for float32 storage on phi, psi and u, 1e-3 for
float16-deviation storage.  Inputs are the seeded synthetic problems of
workloads.py.
"""
import numpy as np
import pytest

import oracle as O
from paper_2408_15654_amd import lbm, workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp16dev": 1e-3}
FIELDS = ("phi", "psi", "u")


def rel_linf(a, b):
    s = np.abs(b).max()
    return float(np.abs(a - b).max() / (s if s > 0 else 1.0))


def errors(got, want, fields):
    out = {}
    for k in fields:
        if k == "u":
            d = np.hypot(got["ux"] - want["ux"], got["uy"] - want["uy"])
            s = np.hypot(want["ux"], want["uy"]).max()
            out[k] = float(d.max() / (s if s > 0 else 1.0))
        else:
            out[k] = rel_linf(got[k], want[k])
    return out


def run_gpu(pr, precision, steps, rows=None):
    sim = lbm.Simulation(dict(pr.params, precision=precision))
    if rows is not None:
        sim.set_tile_rows(rows)
    sim.init_fields(*pr.fields0)
    sim.step(steps)
    out = sim.read_fields()
    return sim, out


_ORACLE_CACHE = {}


def run_oracle(pr, steps, cache=False):
    """The oracle's state and fields after `steps`.  cache=True keeps the
    result for the other storage precisions of the same problem (the input
    recipe is deterministic, so its name and parameters identify it)."""
    key = (pr.name, repr(sorted((k, repr(v)) for k, v in pr.params.items()
                                if k != "precision")), steps)
    if cache and key in _ORACLE_CACHE:
        return _ORACLE_CACHE[key]
    ref = O.OracleSim(pr.params, *pr.fields0)
    ref.step(steps)
    out = (ref, ref.fields())
    if cache:
        _ORACLE_CACHE.clear()  # one large problem at a time
        _ORACLE_CACHE[key] = out
    return out


def check_moments(sim, ref, steps):
    """Float64 device reductions (lbm_moments) against the oracle's sums of
    the same level: phi and psi to 1e-12 relative; momentum to 1e-12 of the
    sum of rho|u| (it may cancel to rounding level); kinetic energy and the
    largest speed to 1e-12 relative."""
    m, mo = sim.moments(), ref.moments()
    assert m["step"] == steps
    for k in ("sum_phi", "sum_psi", "kinetic", "max_u"):
        assert abs(m[k] - mo[k]) <= 1e-12 * abs(mo[k]), (k, m[k], mo[k])
    fl = ref.fields()
    p = ref.params
    phiA, phiB = p.get("phiA", 1.0), p.get("phiB", 0.0)
    rho = (fl["phi"] - phiB) / (phiA - phiB) * (p["rhoA"] - p["rhoB"]) + p["rhoB"]
    scale = float((rho * np.hypot(fl["ux"], fl["uy"])).sum())
    for k in ("mom_x", "mom_y"):
        assert abs(m[k] - mo[k]) <= 1e-12 * scale, (k, m[k], mo[k], scale)


def check(got, want, tol, label, fields=FIELDS):
    errs = errors(got, want, fields)
    print(label, " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    for k, e in errs.items():
        assert e <= tol, (label, k, e)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
def test_initial_level_matches_oracle(precision):
    pr = W.c1_stationary_drop()
    _, got = run_gpu(pr, precision, 0)
    _, want = run_oracle(pr, 0)
    check(got, want, TOL[precision], f"init {precision}", FIELDS + ("P",))




@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
def test_drop64_full_run(precision):
    """64x64 drop, 2000 steps (the full run of the small configuration)."""
    pr = W.c1_stationary_drop()
    sim, got = run_gpu(pr, precision, pr.steps)
    ref, want = run_oracle(pr, pr.steps)
    check(got, want, TOL[precision], f"drop64 {precision}")
    if precision == "fp64":
        check(got, want, TOL[precision], "drop64 fp64 P", ("P",))
        check_moments(sim, ref, pr.steps)


def test_drop64_fp16dev_conserves_mass():
    """float16 storage rounds stochastically, with each site's rounding
    errors of f_1..f_8 and g_1..g_8 carried into its rest populations: the
    sums of phi and psi stay within 1e-6 of the oracle's over 2000 steps."""
    pr = W.c1_stationary_drop()
    sim, _ = run_gpu(pr, "fp16dev", pr.steps)
    ref, _ = run_oracle(pr, pr.steps)
    m, mo = sim.moments(), ref.moments()
    for k in ("sum_phi", "sum_psi"):
        assert abs(m[k] - mo[k]) <= 1e-6 * abs(mo[k]), (k, m[k], mo[k])


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
def test_surface_diffusion_run(precision):
    """Surfactant diffusing along a circle at rest (Sec. 4.1 set-up in
    lattice units: 100x100, R = 25, tau_psi = 9.875), its full 200 steps."""
    pr = W.e1_surface_diffusion()
    sim, got = run_gpu(pr, precision, pr.steps)
    _, want = run_oracle(pr, pr.steps)
    check(got, want, TOL[precision], f"e1 {precision}", ("phi", "psi"))
    assert np.abs(got["ux"]).max() == 0.0 and np.abs(got["uy"]).max() == 0.0
    sim.close()


@pytest.mark.parametrize("seed", range(8))
def test_random_small_fp64(seed):
    """Odd sizes, walls or periodic, r in {0,1,2}, linear or Langmuir EOS,
    density and viscosity ratios, body force, random free rates."""
    pr = W.random_small(seed, steps=60)
    _, got = run_gpu(pr, "fp64", pr.steps)
    _, want = run_oracle(pr, pr.steps)
    check(got, want, 1e-12, f"random{seed} {pr.params['nx']}x{pr.params['ny']} "
          f"walls={pr.params['walls_y']} r={pr.params['r']} eos={pr.params['eos']}",
          FIELDS + ("P",))


@pytest.mark.parametrize("seed", range(8))
def test_random_small_fp32(seed):
    pr = W.random_small(seed, steps=60)
    _, got = run_gpu(pr, "fp32", pr.steps)
    _, want = run_oracle(pr, pr.steps)
    check(got, want, 1e-5, f"random{seed} fp32")


@pytest.mark.parametrize("seed", range(8))
def test_random_small_fp16dev(seed):
    """Float16-deviation storage on the random problems (walls or periodic,
    r in {0, 1, 2}, linear or Langmuir EOS, density ratios, body force, odd
    and even widths): within the float16 bar after 60 steps."""
    pr = W.random_small(seed, steps=60)
    _, got = run_gpu(pr, "fp16dev", pr.steps)
    _, want = run_oracle(pr, pr.steps)
    check(got, want, TOL["fp16dev"], f"random{seed} fp16dev")


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
@pytest.mark.parametrize("seed", range(3))
def test_dense_drop_on_moving_wall(seed, precision):
    """A drop of the denser fluid A (density ratio 3 or 10) centred on the
    bottom wall, so fluid A lies against the moving bottom wall: its
    bounce-back term carries rho_w = rho(phi) of the boundary site, far from
    1 there.  Odd and even widths."""
    pr = W.random_small(300 + seed, walls=True, wall_drop=True, steps=60)
    sim, got = run_gpu(pr, precision, pr.steps)
    _, want = run_oracle(pr, pr.steps)
    fields = FIELDS + ("P",) if precision == "fp64" else FIELDS
    check(got, want, TOL[precision], f"wall drop{seed} {precision} "
          f"{pr.params['nx']}x{pr.params['ny']} rhoA={pr.params['rhoA']}", fields)
    sim.close()


@pytest.mark.parametrize("nx,ny", [(3, 3), (5, 4), (61, 7), (62, 9), (63, 5), (64, 3),
                                   (125, 11), (186, 6)])
def test_ragged_and_tiny_grids(nx, ny):
    """Strip widths that are 62 +- 1, grids narrower than a wavefront and
    the minimum size, with walls (odd) and periodic (even) widths."""
    pr = W.random_small(100 + nx, nx=nx, ny=ny, walls=bool(nx % 2), steps=12)
    _, got = run_gpu(pr, "fp64", pr.steps)
    _, want = run_oracle(pr, pr.steps)
    check(got, want, 1e-12, f"grid {nx}x{ny}")


@pytest.mark.parametrize("precision", ["fp32", "fp16dev"])
@pytest.mark.parametrize("nx,ny,walls", [(4, 5, True), (6, 3, False), (122, 7, True),
                                         (124, 9, False), (126, 5, True), (250, 6, False),
                                         (248, 4, True)])
def test_two_column_lanes(nx, ny, walls, precision):
    """float32 and float16 storage with an even nx run two columns per lane
    (124 interior columns per wavefront): widths at and around one and two
    strips, narrower than a wavefront, and the seam of the periodic wrap
    falling inside a lane pair of the halo."""
    pr = W.random_small(200 + nx, nx=nx, ny=ny, walls=walls, steps=20)
    _, got = run_gpu(pr, precision, pr.steps)
    _, want = run_oracle(pr, pr.steps)
    check(got, want, TOL[precision], f"{precision} pairs {nx}x{ny} walls={walls}",
          FIELDS + ("P",))


@pytest.mark.parametrize("precision,nx", [("fp32", 250), ("fp16dev", 250), ("fp32", 251),
                                         ("fp16dev", 251)])
def test_tile_height_does_not_change_results_reduced(precision, nx):
    """float32 and float16 storage, two columns per lane (even nx) and one
    (odd nx): every tile height gives the same bits."""
    pr = W.random_small(5, nx=nx, ny=40, walls=True, steps=15)
    outs = []
    for rows in (1, 3, 7, 40, 0):  # 0: the default (small grid: the shortest fitting tiles)
        _, got = run_gpu(pr, precision, pr.steps, rows=rows)
        outs.append(got)
    for o in outs[1:]:
        for k in ("phi", "psi", "ux", "uy", "P"):
            assert np.array_equal(o[k], outs[0][k]), k


@pytest.mark.parametrize("precision,beta", [("fp64", 0.5), ("fp32", 0.5), ("fp16dev", 0.5),
                                            ("fp64", 0.0), ("fp32", 0.0), ("fp16dev", 0.0)])
def test_shear_drop(precision, beta):
    """256x128 channel between moving walls, drop R=32, 2000 steps (Sec.
    4.4 geometry with the full coupled scheme)."""
    pr = W.c2_shear_drop(beta=beta)
    sim, got = run_gpu(pr, precision, 2000)
    ref, want = run_oracle(pr, 2000, cache=True)
    check(got, want, TOL[precision], f"shear {precision} beta={beta}")
    if precision == "fp64":
        # P is recovered from sum_{i!=0} h_i (Eq. (32b)), and each h_i holds
        # 3 w_i (P + c_i . rho u) (Eq. (30)): its rounding scales with
        # |P| + |rho u|.  Here the walls drive rho|u| = 1e-2 while |P| stays
        # near 1e-4, so P is held to 1e-12 of that scale.
        rho = want["phi"] * (pr.params["rhoA"] - pr.params["rhoB"]) + pr.params["rhoB"]
        scale = (np.abs(want["P"]) + rho * np.hypot(want["ux"], want["uy"])).max()
        eP = np.abs(got["P"] - want["P"]).max() / scale
        print(f"shear fp64 beta={beta} P (population scale) {eP:.2e}", flush=True)
        assert eP <= TOL[precision], eP
        check_moments(sim, ref, 2000)
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
def test_many_drops_full_size(precision):
    """2048x2048, 400 drops, density ratio 10, in the launch configuration
    the benchmark times: every site compared after 200 steps (the oracle
    runs once, about half a minute on 16 host cores, and serves all three
    storage precisions)."""
    pr = W.c3_many_drops(precision=precision)
    sim, got = run_gpu(pr, precision, 200)
    ref, want = run_oracle(pr, 200, cache=True)
    check(got, want, TOL[precision], f"drops2048 {precision}")
    if precision == "fp64":
        check(got, want, TOL[precision], "drops2048 fp64 P", ("P",))
        check_moments(sim, ref, 200)
    sim.close()


# Largest square grid each storage precision accepts (the 26 population
# planes of one copy are addressed with 32-bit byte offsets, so they must fit
# in 4 GiB), and a tile side that divides it.
MAX_GRID = {"fp64": (4544, 142), "fp32": (6426, 126), "fp16dev": (9088, 142)}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
def test_largest_grid_equals_its_tiled_small_copy(precision):
    """The largest grid the library accepts, filled with copies of a small
    periodic field: every site has the neighbourhood it has in the small
    run, so after a few steps the large fields are the small ones tiled.
    Bitwise for float64 and float32 storage; float16 storage draws its
    rounding bits per site, so there phi, psi and u are held to the float16
    bar (P, a diagnostic near 1e-8 here, is not under it).  Any offset that
    overflows at the largest sizes breaks the copy.  The large fields are
    also held, at the storage's bar, to the oracle's run of the small field,
    tiled (the problem is translation invariant)."""
    n, p = MAX_GRID[precision]
    steps = 3
    pr = W.c3_many_drops(precision=precision, nx=p, ny=p, ndrops=2)
    _, small = run_gpu(pr, precision, steps)
    reps = (n // p, n // p)
    sim = lbm.Simulation(dict(pr.params, nx=n, ny=n, precision=precision))
    sim.init_fields(*[np.tile(a, reps) for a in pr.fields0])
    sim.step(steps)
    got = sim.read_fields()
    sim.close()
    del sim
    _, ref = run_oracle(pr, steps)
    check(got, {k: np.tile(ref[k], reps) for k in ("phi", "psi", "ux", "uy")}, TOL[precision],
          f"largest grid {precision} {n}^2 against the oracle")
    want = {k: np.tile(small[k], reps) for k in ("phi", "psi", "ux", "uy", "P")}
    if precision == "fp16dev":
        err = errors(got, want, FIELDS)
        assert max(err.values()) <= TOL[precision], err
    else:
        for k in want:
            assert np.array_equal(got[k], want[k]), k


@pytest.mark.parametrize("precision,walls", [("fp32", False), ("fp16dev", False),
                                             ("fp32", True), ("fp16dev", True)])
def test_default_tile_plan_gives_the_bits_of_one_row_tiles(precision, walls):
    """2048x1024: the default plan cuts each XCD's 128-row band into tall
    tiles followed by 1-row tiles (float32 storage: 2-row tiles and 15 rows
    of 1-row tiles; float16 storage: one tile per wavefront slot, 15 tiles
    of 8 rows, then 8 rows of 1-row tiles, on a 256-CU device).  Bitwise the
    same fields as 1-row tiles everywhere: periodic drops, and a dense drop
    on the moving bottom wall (the top wall row is then walked by a 1-row
    tile at the end of the last band)."""
    if walls:
        pr = W.random_small(7, nx=2048, ny=1024, walls=True, wall_drop=True,
                            precision=precision)
    else:
        pr = W.c3_many_drops(precision=precision, nx=2048, ny=1024, ndrops=200)
    sim = lbm.Simulation(dict(pr.params, precision=precision))
    plan = sim.tile_plan()
    print(f"{precision} 2048x1024 tile plan {plan}", flush=True)
    assert plan[0] > 1 and plan[1] > 0 and plan[2] == 1, plan
    sim.init_fields(*pr.fields0)
    sim.step(12)
    got = sim.read_fields()
    sim.close()
    _, want = run_gpu(pr, precision, 12, rows=1)
    for k in ("phi", "psi", "ux", "uy", "P"):
        assert np.array_equal(got[k], want[k]), k


@pytest.mark.parametrize("ny", [5, 9, 43, 130])
@pytest.mark.parametrize("walls", [False, True])
def test_band_edges_cover_every_row(ny, walls):
    """Grids whose height leaves some XCD bands empty (5 rows), uneven (9,
    43, 130 rows over 8 bands) or partly in 1-row tail tiles: every tile
    height gives the bits of 1-row tiles, so no row is skipped or walked
    twice at a band's edges."""
    pr = W.random_small(11, nx=64, ny=ny, walls=walls, steps=8)
    _, want = run_gpu(pr, "fp32", pr.steps, rows=1)
    for rows in (2, 3, 7, 0):
        _, got = run_gpu(pr, "fp32", pr.steps, rows=rows)
        for k in ("phi", "psi", "ux", "uy", "P"):
            assert np.array_equal(got[k], want[k]), (rows, k)


@pytest.mark.parametrize("precision", ["fp32", "fp16dev"])
def test_odd_grid_equals_its_tiled_small_copy(precision):
    """2047x2047 (odd, so one column per lane) filled with 23x23 copies of
    an 89x89 periodic field: after a few steps the large fields are the
    small ones tiled, bitwise for float32 storage and at the float16 bar
    for float16 storage (its rounding bits depend on the site), and at the
    storage's bar against the oracle's run of the small field.  The large
    grid runs the large-grid tile plan of the one-column kernels."""
    n, p = 2047, 89
    steps = 3
    pr = W.c3_many_drops(precision=precision, nx=p, ny=p, ndrops=2)
    _, small = run_gpu(pr, precision, steps)
    reps = (n // p, n // p)
    sim = lbm.Simulation(dict(pr.params, nx=n, ny=n, precision=precision))
    assert sim.step_kernel_name().split(", ")[1] == "1", sim.step_kernel_name()
    sim.init_fields(*[np.tile(a, reps) for a in pr.fields0])
    sim.step(steps)
    got = sim.read_fields()
    sim.close()
    del sim
    _, ref = run_oracle(pr, steps)
    check(got, {k: np.tile(ref[k], reps) for k in ("phi", "psi", "ux", "uy")}, TOL[precision],
          f"odd grid {precision} {n}^2 against the oracle")
    want = {k: np.tile(small[k], reps) for k in ("phi", "psi", "ux", "uy", "P")}
    if precision == "fp16dev":
        err = errors(got, want, FIELDS)
        assert max(err.values()) <= TOL[precision], err
    else:
        for k in want:
            assert np.array_equal(got[k], want[k]), k


def test_tile_height_does_not_change_results():
    """Each site's arithmetic is independent of the tiling: bitwise equal."""
    pr = W.random_small(3, nx=150, ny=70, steps=25)
    outs = []
    for rows in (1, 3, 8, 70, 200, 0):
        _, got = run_gpu(pr, "fp64", pr.steps, rows=rows)
        outs.append(got)
    for o in outs[1:]:
        for k in ("phi", "psi", "ux", "uy", "P"):
            assert np.array_equal(o[k], outs[0][k]), k


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
def test_checkpoint_restore_is_bitwise(precision):
    pr = W.random_small(4, steps=30)
    sim = lbm.Simulation(dict(pr.params, precision=precision))
    sim.init_fields(*pr.fields0)
    sim.step(10)
    state = sim.get_state()
    sim.step(20)
    a = sim.read_fields()
    sim.step(5)
    sim.set_state(state)
    assert sim.moments()["step"] == 10
    sim.step(20)
    b = sim.read_fields()
    sim.close()
    # the state is self-contained: a fresh handle continues the same way
    fresh = lbm.Simulation(dict(pr.params, precision=precision))
    fresh.set_state(state)
    fresh.step(20)
    c = fresh.read_fields()
    fresh.close()
    for k in ("phi", "psi", "ux", "uy", "P"):
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k


def test_nonfinite_is_reported_and_blocks_stepping():
    """A NaN forced into the state from the host surfaces as LBM_ENONFINITE
    at the next synchronising call; stepping is refused until re-init."""
    pr = W.random_small(5, steps=5)
    sim = lbm.Simulation(dict(pr.params, precision="fp64"))
    sim.init_fields(*pr.fields0)
    state = bytearray(sim.get_state())
    nan = np.array([np.nan], dtype=np.float64).tobytes()
    off = 8 + 8 * (3 * pr.params["nx"] + 5)  # a population of some site
    state[off:off + 8] = nan
    sim.set_state(bytes(state))
    sim.step(3)
    with pytest.raises(lbm.NonFiniteError):
        sim.moments()
    with pytest.raises(lbm.LbmError) as e:
        sim.step(1)
    assert e.value.status == lbm.LBM_ESTATE
    sim.init_fields(*pr.fields0)
    sim.step(2)
    assert np.isfinite(sim.moments()["sum_phi"])


def test_close_waits_for_the_work_on_a_side_stream():
    """A simulation on a stream of its own (default priority): lbm_step only
    enqueues, and lbm_destroy waits for that stream, so once close() returns
    the workspace is no longer written and may be released or reused."""
    import torch

    pr = W.c3_many_drops(precision="fp32", nx=512, ny=512, ndrops=10)
    side = torch.cuda.Stream()
    sim = lbm.Simulation(pr.params, stream=side)
    sim.init_fields(*pr.fields0)
    sim.step(400)
    sim.close()
    assert side.query()
    del sim
    torch.cuda.synchronize()


def test_float16_saturation_is_reported():
    """float16-deviation storage with a scale far too large for the
    deviations (2^30 on f): the conversion would store them saturated at
    65504, and the step reports that as a lost state (LBM_ENONFINITE),
    after which stepping is refused.  The default scales stay clean."""
    pr = W.c1_stationary_drop()
    sim = lbm.Simulation(dict(pr.params, precision="fp16dev", fp16_scale=(2.0 ** 30, 0, 0)))
    sim.init_fields(*pr.fields0)
    sim.step(2)
    with pytest.raises(lbm.NonFiniteError):
        sim.moments()
    with pytest.raises(lbm.LbmError) as e:
        sim.step(1)
    assert e.value.status == lbm.LBM_ESTATE
    sim.close()
    ok = lbm.Simulation(dict(pr.params, precision="fp16dev"))
    ok.init_fields(*pr.fields0)
    ok.step(50)
    assert ok.moments()["nonfinite"] == 0
    ok.close()


def test_invalid_arguments():
    pr = W.c1_stationary_drop()
    with pytest.raises(lbm.LbmError):
        lbm.Simulation(dict(pr.params, M=0.0))
    sim = lbm.Simulation(pr.params)
    with pytest.raises(lbm.LbmError) as e:
        sim.step(1)  # not initialised
    assert e.value.status == lbm.LBM_ESTATE
    bad = pr.phi0.copy()
    bad[3, 3] = np.inf
    with pytest.raises(lbm.LbmError) as e:
        sim.init_fields(bad, pr.psi0, pr.ux0, pr.uy0)
    assert e.value.status == lbm.LBM_EINVAL
    lang = lbm.Simulation(dict(pr.params, eos="langmuir"))
    with pytest.raises(lbm.LbmError):
        lang.init_fields(pr.phi0, pr.psi0 + 1.0, pr.ux0, pr.uy0)
    sim.init_fields(*pr.fields0)
    with pytest.raises(lbm.LbmError):
        sim.step(-1)


# ------------------------------------------------ prescribed velocity (Sec. 4.2)



@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
def test_prescribed_convection_full_run(precision):
    """Drop in a uniform prescribed flow (Sec. 4.2): 100x100, 2000 steps."""
    pr = W.e2_convection()
    _, got = run_gpu(pr, precision, pr.steps)
    _, want = run_oracle(pr, pr.steps)
    check(got, want, TOL[precision], f"e2 {precision}")
    assert np.abs(got["P"]).max() == 0.0


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
@pytest.mark.parametrize("seed", range(4))
def test_prescribed_random_small(seed, precision):
    """Random sizes, walls, r, EOS, with a smooth prescribed velocity field,
    in every storage precision.  (A velocity drawn independently per site
    makes some of these problems amplify a 1e-15 perturbation to 1e-10 in
    the oracle alone.)"""
    pr = W.random_small(200 + seed, steps=40)
    ny, nx = pr.phi0.shape
    y, x = np.mgrid[0:ny, 0:nx]
    ux = 0.04 * np.sin(2 * np.pi * y / ny + seed)
    uy = 0.03 * np.cos(2 * np.pi * x / nx + 2 * seed)
    params = dict(pr.params, flow="prescribed")
    sim = lbm.Simulation(dict(params, precision=precision))
    sim.init_fields(pr.phi0, pr.psi0, ux, uy)
    sim.step(pr.steps)
    got = sim.read_fields()
    sim.close()
    ref = O.OracleSim(params, pr.phi0, pr.psi0, ux, uy)
    ref.step(pr.steps)
    want = ref.fields()
    check(got, want, TOL[precision], f"prescribed random{seed} {precision} "
          f"{params['nx']}x{params['ny']} walls={params['walls_y']} r={params['r']}")


# ------------------------------------------------ shape diagnostics

# shape quantities against the oracle's: the step's own bar carried over
# (relative, or absolute below 1), loosened for the derived quantities
SHAPE_TOL = {"fp64": 1e-10, "fp32": 1e-4, "fp16dev": 1e-2}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
def test_shape_diagnostics_match_the_oracle(precision):
    """lbm_shape (device float64 reductions) against the plain numpy
    diagnostics: on the library's own read-back phi (same input: the
    reductions alone, to 1e-12 in every precision) and on the oracle's phi
    of the same run."""
    import shape as SH

    pr = W.c2_shear_drop(beta=0.5)
    sim = lbm.Simulation(dict(pr.params, precision=precision))
    sim.init_fields(*pr.fields0)
    sim.step(300)
    got = sim.shape()
    mine = SH.shape(sim.read_fields()["phi"], pr.params)
    _, want_f = run_oracle(pr, 300)
    want = SH.shape(want_f["phi"], pr.params)
    for k in mine:
        scale = max(abs(mine[k]), 1.0)
        assert abs(got[k] - mine[k]) <= 1e-12 * scale, (k, got[k], mine[k])
        assert abs(got[k] - want[k]) <= SHAPE_TOL[precision] * scale, (k, got[k], want[k])
    assert 0.0 < got["taylor_D"] < 0.5 and got["length"] > 2 * np.pi * 32 * 0.95
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
def test_rising_bubble_small(precision):
    """Buoyant bubble between walls (Sec. 4.3 geometry, 40x80), 400 steps,
    with surfactant (beta 0.5).  g = 5e-6: at g = 2e-5 this small problem
    amplifies a 1e-15 perturbation to 1e-4 in the oracle alone."""
    pr = W.e3_rising_bubble(nx=40, g=5e-6, steps=400, beta=0.5)
    _, got = run_gpu(pr, precision, pr.steps)
    _, want = run_oracle(pr, pr.steps)
    check(got, want, TOL[precision], f"bubble40 {precision}")


def test_step_kernel_name_names_the_variant():
    """lbm_step_kernel_name gives the template arguments of the kernel
    lbm_step launches: storage (the cache-resident variants for 64-320 MB of
    step traffic), columns per lane, r != 1, rho_A != rho_B, Navier-Stokes."""
    cases = [
        (W.c3_many_drops(precision="fp32"), "fp32", "lbm_step_kernel<F32, 2, false, true, true>"),
        (W.c3_many_drops(precision="fp32", nx=724, ny=362, ndrops=12), "fp32",
         "lbm_step_kernel<F32C, 2, false, true, true>"),
        (W.c1_stationary_drop(), "fp64", "lbm_step_kernel<F64, 1, true, false, true>"),
        (W.c1_stationary_drop(), "fp16dev", "lbm_step_kernel<F16, 2, true, false, true>"),
        (W.e2_convection(nx=101), "fp32", "lbm_step_kernel<F32, 1, false, false, false>"),
    ]
    for pr, prec, want in cases:
        sim = lbm.Simulation(dict(pr.params, precision=prec))
        assert sim.step_kernel_name() == want, (prec, pr.params["nx"], sim.step_kernel_name())
        sim.close()


@pytest.mark.parametrize("precision,nx,ny", [("fp64", 301, 123), ("fp32", 500, 130),
                                             ("fp32", 251, 97)])
def test_integer_translation_is_bitwise(precision, nx, ny):
    """Periodic grid: the initial fields shifted by an odd offset give the
    unshifted result shifted by the same offset, bit for bit (every site
    computes the same thing wherever its strip, tile or the periodic seam
    falls).  Float16 storage draws rounding bits per site and is not
    translation invariant bitwise."""
    pr = W.c3_many_drops(precision=precision, nx=nx, ny=ny, ndrops=max(2, nx * ny // 12000))
    dx, dy = 37, 11
    _, a = run_gpu(pr, precision, 25)
    shifted = [np.roll(f, (dy, dx), axis=(0, 1)) for f in pr.fields0]
    sim = lbm.Simulation(dict(pr.params, precision=precision))
    sim.init_fields(*shifted)
    sim.step(25)
    b = sim.read_fields()
    sim.close()
    for k in ("phi", "psi", "ux", "uy", "P"):
        assert np.array_equal(np.roll(a[k], (dy, dx), axis=(0, 1)), b[k]), k

