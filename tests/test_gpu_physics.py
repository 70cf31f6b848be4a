"""The GPU path against the physics the paper fixes (P10, P11 and the
resolution study of Sec. "Far-field Results", Fig. "resolution").

  - Squirmer: the free squirmer's time-averaged swim speed <v>/v0 for
    R in {4, 6, 8, 10, 12, 16} and L in {10R, 15R, 20R}, against the values
    the paper plots for the same method (fixture under tests/golden).  The
    tolerance is 1%, and 1.5% at R = 4, where the paper's own series scatter
    by 0.9%.
  - P11: the finite-size extrapolation v(L) = v_inf + a (R/L)^3 over
    L in {64, 96, 128, 160, 192} at R = 8, with |v_inf / v0 - 1| <= 1.5%.
    Here v0 = 2 B1 / 3 (eq. squirmer-speed).
  - P10, passive sphere: the steady drag of a no-slip sphere in a periodic
    box, as the normalised speed K = 6 pi eta R U / F.  It is compared with
    the paper's passive-sphere series (fixture; within 1%) and with the drag
    factor of a simple cubic array (Hasimoto; within 3%: the staircase sphere's
    hydrodynamic radius differs from R by a fraction of a cell).
  - P10, rotating sphere: T = -8 pi eta R^3 omega (1 + c phi).  The fitted
    infinite-box factor tends to 1 as R grows, and c to the mean-field
    value 1.

<v> is the mean of v.e over the second half of a 12,000-step run, sampled
every 50 steps.
"""
import math
import sys
from pathlib import Path

import numpy as np
import pytest

from tests import stokes

pytestmark = pytest.mark.gpu

B1 = 1e-3
V0 = 2.0 * B1 / 3.0
NU = 1.0 / 6.0
STEPS = 12000
GOLDEN = Path(__file__).resolve().parent / "golden"
_cache = {}


def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_04799_amd import lbsq
    return lbsq


def note(msg):
    print("[gpu-physics] " + msg, flush=True)
    sys.stdout.flush()


def swim_speed(R, L, beta=0.0):
    key = (R, L, beta)
    if key in _cache:
        return _cache[key]
    lbsq = gpu()
    note("free squirmer R=%g in %d^3, beta=%g, %d steps" % (R, L, beta, STEPS))
    s = lbsq.Sim((L, L, L))
    s.add_squirmer((L / 2.0, L / 2.0, L / 2.0), (1.0, 0.0, 0.0), R, B1=B1, beta=beta)
    v = []
    for _ in range(STEPS // 50):
        s.step(50)
        b = s.body(0)
        v.append(float(np.dot(b["v"], b["e"])) / V0)
    s.close()
    _cache[key] = float(np.mean(v[len(v) // 2:]))
    return _cache[key]


def paper(name, R_, L_over_R):
    for line in (GOLDEN / name).read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            r, l, v = line.split()
            if int(r) == R_ and int(l) == L_over_R:
                return float(v)
    raise KeyError((R_, L_over_R))


SWEEP = [(R, lr) for R in (4, 6, 8, 10, 12, 16) for lr in (10, 15, 20)]


@pytest.mark.parametrize("R,L_over_R", SWEEP)
def test_swim_speed_matches_paper(R, L_over_R):
    got = swim_speed(float(R), R * L_over_R)
    ref = paper("fig_resolution_swim_speed.txt", R, L_over_R)
    note("R=%d L=%dR: <v>/v0 = %.5f, paper %.5f" % (R, L_over_R, got, ref))
    assert abs(got / ref - 1.0) < (0.015 if R == 4 else 0.01)


@pytest.mark.parametrize("beta", [-5.0, 0.0, 5.0])
def test_P11_finite_size_extrapolation(beta):
    """v(L) = v_inf + a (R/L)^3 over L in {64, ..., 192} at R = 8.  The
    Stokes swimming speed 2 B1 / 3 does not depend on beta (eq.
    squirmer-speed).  The neutral squirmer's v_inf is within 1.5% of it.
    Pushers and pullers carry the inertial correction of a squirmer at
    small but finite Reynolds number Re = v0 R / nu (0.032 here): the pusher
    swims faster and the puller slower, by about 0.1 |beta| Re (2% here);
    test_pusher_puller_shift_scales_with_reynolds shows it is linear in Re."""
    R = 8.0
    Ls = [64, 96, 128, 160, 192]
    v = np.array([swim_speed(R, L, beta) for L in Ls])
    x = (R / np.array(Ls, dtype=float)) ** 3
    A = np.stack([np.ones_like(x), x], axis=1)
    (v_inf, a), *_ = np.linalg.lstsq(A, v, rcond=None)
    note("beta=%g: v(L)/v0 = %s -> v_inf/v0 = %.5f (slope %.3g)" % (beta, np.round(v, 5).tolist(), v_inf, a))
    if beta == 0.0:
        assert abs(v_inf - 1.0) <= 0.015
        # periodic images slow the swimmer: the speed rises with the box
        assert a < 0.0
    else:
        assert abs(v_inf - 1.0) <= 0.03
        assert (v_inf - 1.0) * beta < 0.0  # pusher (beta < 0) faster, puller slower


def test_pusher_puller_shift_scales_with_reynolds():
    """The pusher/puller speed shift is inertial: half the difference of the
    speeds at beta = -5 and +5 (R = 8, L = 15R) falls in proportion to B1,
    i.e. to the Reynolds number, from B1 = 1e-3 to 2.5e-4 (ratio 4 within
    25%), and at B1 = 2.5e-4 both speeds are within 1% of 2 B1 / 3."""
    lbsq = gpu()
    R, L = 8.0, 120
    shift = {}
    for b1 in (1e-3, 2.5e-4):
        v = {}
        for beta in (-5.0, 5.0):
            s = lbsq.Sim((L, L, L))
            s.add_squirmer((L / 2.0, L / 2.0, L / 2.0), (1.0, 0.0, 0.0), R, B1=b1, beta=beta)
            sp = []
            for _ in range(STEPS // 50):
                s.step(50)
                b = s.body(0)
                sp.append(float(np.dot(b["v"], b["e"])) / (2.0 * b1 / 3.0))
            s.close()
            v[beta] = float(np.mean(sp[len(sp) // 2:]))
        shift[b1] = 0.5 * (v[-5.0] - v[5.0])
        note("B1=%g: <v>/v0 pusher %.5f, puller %.5f, half difference %.5f" % (b1, v[-5.0], v[5.0], shift[b1]))
        if b1 < 1e-3:
            assert abs(v[-5.0] - 1.0) < 0.01 and abs(v[5.0] - 1.0) < 0.01
    ratio = shift[1e-3] / shift[2.5e-4]
    note("ratio of the shifts %.3f (4 if linear in Re)" % ratio)
    assert shift[1e-3] > 0.0 and 3.0 < ratio < 5.0


PASSIVE = [(R, lr) for lr in (10, 15, 20) for R in (4, 6, 8, 10, 12) if not (lr == 20 and R == 12)]


@pytest.mark.parametrize("R,L_over_R", PASSIVE)
def test_P10_passive_sphere_drag(R, L_over_R):
    lbsq = gpu()
    L = R * L_over_R
    Kh = stokes.k_hasimoto(stokes.volume_fraction(R, L))
    # superficial speed near 1e-3 nu / R: particle Reynolds number 1e-3
    g = (1e-3 * NU / R) * 6.0 * math.pi * NU * R / (Kh * L ** 3)
    note("fixed sphere R=%d in %d^3 pushed by g=%.3g" % (R, L, g))
    s = lbsq.Sim((L, L, L), g=(g, 0.0, 0.0))
    s.add_squirmer((L / 2.0, L / 2.0, L / 2.0), (1.0, 0.0, 0.0), R, mode="fixed")
    K, balance = stokes.steady_drag(s.step, s.populations, s.set_populations, s.fields,
                                    lambda: s.force_torque(0)[0][0], R, L, g, NU)
    s.close()
    ref = paper("fig_resolution_passive_speed.txt", R, L_over_R)
    note("R=%d L=%dR: K = %.5f, paper %.5f, Hasimoto %.5f, F/(g N_f) = %.5f" % (R, L_over_R, K, ref, Kh, balance))
    assert abs(balance - 1.0) < 2e-3
    assert abs(K / ref - 1.0) < 0.01
    assert abs(K / Kh - 1.0) < 0.03


def test_P10_rotating_sphere_torque():
    lbsq = gpu()
    A = {}
    for R in (4, 8, 12):
        w = 1e-2 * NU / R ** 2  # rotational Reynolds number 1e-2
        ratio, phi = [], []
        for L in (6 * R, 8 * R):
            s = lbsq.Sim((L, L, L))
            s.add_squirmer((L / 2.0, L / 2.0, L / 2.0), (1.0, 0.0, 0.0), R, mode="prescribed", w=(0.0, 0.0, w))
            s.step(6 * stokes.box_relaxation_steps(L, NU))
            T = s.force_torque(0)[1]
            s.close()
            ratio.append(T[2] / (-8.0 * math.pi * NU * R ** 3 * w))
            phi.append(stokes.volume_fraction(R, L))
            assert abs(T[0]) < 1e-6 * abs(T[2]) and abs(T[1]) < 1e-6 * abs(T[2])
        # ratio = A (1 + c phi), two boxes
        c = (ratio[0] - ratio[1]) / (ratio[1] * phi[0] - ratio[0] * phi[1])
        A[R] = ratio[1] / (1.0 + c * phi[1])
        note("R=%d: T/T_Stokes = %s at phi = %s -> A = %.5f, c = %.3f"
             % (R, np.round(ratio, 5).tolist(), np.round(phi, 5).tolist(), A[R], c))
        assert 0.6 < c < 1.5
        assert abs(A[R] - 1.0) < 0.06
    assert abs(A[12] - 1.0) < abs(A[4] - 1.0)


def test_E4_head_on_pair_is_point_symmetric():
    """Two pullers (beta = 5) facing each other, 12R apart along their axes
    and offset laterally by d = 2 y0 (Sec. "Interaction between Two
    Squirmers").  The paper's comparison trajectories are only plotted, so
    this checks what the set-up fixes.
    - The half-turn about the z axis through the box centre maps the lattice,
      the D3Q19 set and the pair onto themselves, so the trajectories stay
      point images of each other.
    - Total momentum, fluid plus bodies, is conserved (force-free swimmers,
      no walls).
    - The bodies never overlap.

    At the paper's size: R = 9 in a periodic 250^3 box, 12R apart, through
    closest approach (160,000 steps)."""
    lbsq = gpu()
    R, shape, steps = 9.0, (250, 250, 250), 160000
    y0 = 1.5 * R
    c = np.array(shape, dtype=float) / 2.0
    s = lbsq.Sim(shape)
    s.add_squirmer(c + (-6.0 * R, -y0, 0.0), (1.0, 0.0, 0.0), R, B1=B1, beta=5.0)
    s.add_squirmer(c + (6.0 * R, y0, 0.0), (-1.0, 0.0, 0.0), R, B1=B1, beta=5.0)
    m = 4.0 / 3.0 * math.pi * R ** 3  # neutrally buoyant
    note("head-on pair R=%g in %s, d=%g, %d steps" % (R, shape, 2 * y0, steps))
    gap_min, sym_max, P_drift = np.inf, 0.0, 0.0
    P0 = None
    for k in range(steps // 1000):
        s.step(1000)
        b0, b1 = s.body(0), s.body(1)
        d = b1["pos"] - b0["pos"]
        d -= np.array(shape) * np.round(d / np.array(shape))
        gap_min = min(gap_min, float(np.linalg.norm(d)) - 2.0 * R)
        sym = np.concatenate([b0["pos"] + b1["pos"] - 2.0 * c, b0["e"] + b1["e"]])
        sym_max = max(sym_max, float(np.abs(sym).max()))
        _, P = s.audit()
        Ptot = P + m * (b0["v"] + b1["v"])
        if P0 is None:
            P0 = Ptot
        P_drift = max(P_drift, float(np.abs(Ptot - P0).max()))
    s.close()
    lateral = float(abs(b0["pos"][1] - c[1]))
    note("closest surface gap %.3f, lateral offset %.3f -> %.3f, symmetry error %.2e, momentum drift %.2e (m v0 = %.2e)"
         % (gap_min, y0, lateral, sym_max, P_drift, m * V0))
    assert gap_min > 0.0
    assert sym_max < 1e-4
    assert P_drift < 1e-6 * m * V0 * shape[0]


@pytest.mark.parametrize("beta", [-5.0, 0.0, 5.0])
def test_E1_bulk_field_matches_periodic_analytic(beta):
    """The flow field of a free squirmer at R = 8 in a periodic box L = 10R
    against eq. (squirmerflow) summed over the periodic images (Sec.
    "Squirmers in Bulk"; the paper reports a mean error of about 8% there).
    - The image sum runs over a spherical shell of images.
    - The uniform strain that the spherical order leaves (a periodic field has
      zero mean gradient) is removed.
    - The mean velocity of each field is removed.
    - The comparison is over every second cell in each direction, for fluid
      cells at least one cell outside the surface.
    Relative L2 error and the mean relative error where the analytic flow is
    above a tenth of its RMS: both within 8% (observed 3-4%)."""
    lbsq = gpu()
    R, L = 8.0, 80
    note("bulk field R=%g L=%d beta=%g" % (R, L, beta))
    s = lbsq.Sim((L, L, L))
    s.add_squirmer((L / 2.0, L / 2.0, L / 2.0), (1.0, 0.0, 0.0), R, B1=B1, beta=beta)
    s.step(5000)
    _, u, own = s.fields()
    b = s.body(0)
    s.close()
    pos, e = b["pos"], b["e"]
    sl = (slice(0, None, 2),) * 3
    zz, yy, xx = np.meshgrid(*(np.arange(0, L, 2) + 0.5,) * 3, indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()])
    d = pts - pos[:, None]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(0))
    keep = (own[sl] == 0).ravel() & (r >= R + 1.0)
    u_lb = np.stack([u[k][sl].ravel() for k in range(3)])[:, keep]
    G = stokes.image_sum_mean_gradient(pos, e, R, B1, beta * B1, L, 4)
    u_an = stokes.periodic_squirmer_field(pos[:, None] + d, pos, e, R, B1, beta * B1, L, 4) - G @ d
    u_an = u_an[:, keep]
    u_lb = u_lb - u_lb.mean(axis=1, keepdims=True)
    u_an = u_an - u_an.mean(axis=1, keepdims=True)
    na = np.sqrt((u_an ** 2).sum(0))
    nd = np.sqrt(((u_lb - u_an) ** 2).sum(0))
    rel_l2 = float(np.sqrt((nd ** 2).sum() / (na ** 2).sum()))
    big = na > 0.1 * np.sqrt((na ** 2).mean())
    mean_rel = float((nd[big] / na[big]).mean())
    note("beta=%g: relative L2 %.4f, mean relative error %.4f" % (beta, rel_l2, mean_rel))
    assert rel_l2 < 0.08 and mean_rel < 0.08


def test_E5_neutral_squirmer_oscillates_in_a_tube():
    """A neutral squirmer (beta = 0) started off the axis of a round tube,
    parallel to it, with D = 20R/3 and R = 9, periodic along the axis (Sec.
    "Squirmer in a Round Tube").  The paper compares the trajectories with
    published boundary-element results, which it only plots.  This checks
    what the set-up fixes.
    - The swimmer turns away from the near wall, crosses the axis and swings
      out to the mirror-image offset: the orbit of a reversible, mirror-
      symmetric system, so the amplitude is kept (within 2%).
    - The orientation tilt changes sign at the turning point.
    The tube length is 85 cells (the paper's 3 pi R is not an integer)."""
    from tests import scenes
    lbsq = gpu()
    R = 9.0
    nx = ny = 64
    nz = 85
    y0 = -2.1 * R
    note("neutral squirmer in a tube D=%g, R=%g, y0=%g" % (20 * R / 3, R, y0))
    s = lbsq.Sim((nx, ny, nz))
    s.set_static_mask(scenes.tube_mask(nx, ny, nz, 10.0 * R / 3.0))
    s.add_squirmer((nx / 2.0 + y0, ny / 2.0, nz / 2.0), (0.0, 0.0, 1.0), R, B1=B1, beta=0.0)
    travel, zprev = 0.0, nz / 2.0
    xmax, z_at_xmax, ex_at_start = -1e9, 0.0, None
    for _ in range(150):
        s.step(2000)
        b = s.body(0)
        dz = b["pos"][2] - zprev
        travel += dz - nz * round(dz / nz)
        zprev = b["pos"][2]
        x = b["pos"][0] - nx / 2.0
        if ex_at_start is None:
            ex_at_start = b["e"][0]
        if x > xmax:
            xmax, z_at_xmax, ex_at_max = x, travel, b["e"][0]
    ex_end = b["e"][0]
    s.close()
    note("amplitude %.3f R (started at %.3f R), turning point after %.2f R of travel, tilt %+.3f -> %+.3f"
         % (xmax / R, y0 / R, z_at_xmax / R, ex_at_start, ex_end))
    assert abs(xmax / abs(y0) - 1.0) < 0.02
    assert ex_at_start > 0.0 and ex_end < 0.0
    assert 0.2 * travel < z_at_xmax < 0.8 * travel


@pytest.mark.parametrize("beta", [-3.0, 0.0, 3.0])
def test_near_field_scene_long_run(beta):
    """The near-field scene at its real size over its full run: a 256^3
    periodic box, a fixed no-slip sphere A = 32 at the centre, and a squirmer
    (R = 16) heading at it with an impact parameter drawn from the seed, 16
    cells from its surface, for beta in {-3, 0, 3}, 50,000 steps (the
    library's default layout, the pull layout at this size):
    - the swimmer closes in on the obstacle at a speed of order v0, and the
      two never overlap (WCA holds them apart at contact);
    - every body state stays finite and the swimmer stays slow (|v| < 10 v0);
    - the mean fluid density moves by under 5e-5 relative, while the fluid
      cell count changes as the swimmer crosses the lattice.  Mass is not
      conserved exactly with moving boundaries: besides the conversions
      (which the paper's Sec. 3 notes conserve it only on average), each
      moving-wall link adds mass 2 w_i rho_w c_i.u_b / c_s^2, and over the
      staircase surface the slip's link sum does not vanish (the oracle's
      mass bookkeeping pin checks that these are the only sources).  Held
      still, a squirmer would drift the mass steadily; one that swims samples
      many surface offsets, and 50,000 steps here change it by 1e-6 to
      2.3e-5 depending on beta."""
    from tests import scenes
    lbsq = gpu()
    sc = scenes.obstacle_scene(0)
    steps = 50000
    note("near-field scene 256^3, b=%.3f, beta=%g, %d steps" % (sc["b"], beta, steps))
    s = lbsq.Sim((256, 256, 256))
    s.add_squirmer(sc["obstacle"], (1.0, 0.0, 0.0), sc["A"], mode="fixed")
    s.add_squirmer(sc["squirmer"], (1.0, 0.0, 0.0), sc["R"], B1=B1, beta=beta)
    centre = np.array(sc["obstacle"])

    def gap():
        return float(np.linalg.norm(s.body(1)["pos"] - centre)) - sc["A"] - sc["R"]

    m0, _ = s.audit()
    n0 = s.info()["n_fluid"]
    g0, x0 = gap(), float(s.body(1)["pos"][0])
    gaps = []
    for _ in range(steps // 2500):
        s.step(2500)
        b = s.body(1)
        assert all(np.isfinite(b[k]).all() for k in ("pos", "v", "e", "w"))
        assert np.linalg.norm(b["v"]) < 10.0 * V0
        gaps.append(gap())
    m1, _ = s.audit()
    n1 = s.info()["n_fluid"]
    x1 = float(s.body(1)["pos"][0])
    s.close()
    drho = (m1 / n1) / (m0 / n0) - 1.0
    note("  gap %.2f -> %.2f (min %.2f), x advanced %.2f cells, fluid cells %+d, mean density %+.2e"
         % (g0, gaps[-1], min(gaps), x1 - x0, n1 - n0, drho))
    assert min(gaps) > 0.0
    assert min(gaps) < g0 and x1 - x0 > 0.3 * V0 * 20000
    assert abs(drho) < 5e-5


@pytest.mark.parametrize("beta", [-3.0, 0.0, 3.0])
def test_tube_scene_on_axis(beta):
    """The confined scene at its real size over its full run: a squirmer
    R = 12 on the axis of a no-slip tube of radius 24 (96 x 96 x 512, a
    static wall mask), beta in {-3, 0, 3}, 50,000 steps.  The tube is
    symmetric about its axis, so the swimmer stays on it and keeps its
    heading; the wall slows it below its free speed 2 B1 / 3 (the
    confinement R / r = 0.5).  The mean fluid density moves by under 5e-5
    (the moving-wall link mass of the slip, as in the near-field scene,
    odd in beta here: -2.0e-5, +6e-7 and +2.3e-5 for beta = -3, 0, 3)."""
    from tests import scenes
    lbsq = gpu()
    shape, steps = (96, 96, 512), 50000
    note("tube scene 96x96x512 r=24, R=12, beta=%g, %d steps" % (beta, steps))
    s = lbsq.Sim(shape)
    s.set_static_mask(scenes.tube_mask(*shape, 24.0))
    s.add_squirmer((48.0, 48.0, 256.0), (0.0, 0.0, 1.0), 12.0, B1=B1, beta=beta)
    m0, _ = s.audit()
    n0 = s.info()["n_fluid"]
    v = []
    for _ in range(steps // 500):
        s.step(500)
        b = s.body(0)
        assert all(np.isfinite(b[k]).all() for k in ("pos", "v", "e", "w"))
        v.append(float(b["v"][2]))
    b = s.body(0)
    m1, _ = s.audit()
    n1 = s.info()["n_fluid"]
    s.close()
    vm = float(np.mean(v[len(v) // 2:])) / V0
    off_axis = float(np.hypot(b["pos"][0] - 48.0, b["pos"][1] - 48.0))
    drho = (m1 / n1) / (m0 / n0) - 1.0
    note("  <v>/v0 = %.4f over the second half, off axis %.2e cells, heading e_z = %.9f, mean density %+.2e"
         % (vm, off_axis, b["e"][2], drho))
    assert 0.1 < vm < 1.05
    # FP32 round-off breaks the mirror symmetry only at the 1e-7 level
    assert off_axis < 1e-3 and b["e"][2] > 1.0 - 1e-6
    assert abs(drho) < 5e-5


def test_E6_orbit_and_scatter_either_side_of_the_boundary():
    """The orbit/scatter study at the paper's smallest obstacle, A/R = 6.25
    (A = 50, R = 8): the paper places the critical -beta between 32 and 34,
    and the bisection here between 29 and 30 (320^3, B1 = 2e-3, start 5
    cells off at 30 degrees, contact range sigma = 3).  Well on either side:
    beta = -45 orbits, sweeping past half a revolution at a steady gap
    within the contact range; beta = -20 touches and leaves.  Each run stops
    as soon as it is decided (about 70,000-80,000 steps)."""
    gpu()
    from paper_1903_04799_amd import orbit
    out = {}
    for beta in (-45.0, -20.0):
        note("E6: A = 50, R = 8, 320^3, sigma = 3, beta = %g" % beta)
        r = orbit.orbit_run(beta, A=50.0, R=8.0, n=320, B1=2e-3, gap0=5.0, angle_deg=30.0, max_steps=200000,
                            wca_sigma=3.0)
        note("  %s at step %d, min gap %.2f, swept %.1f deg" % (r["outcome"], r["decided_at"], r["min_gap"],
                                                                r["max_swept_deg"]))
        out[beta] = r
    orb, sca = out[-45.0], out[-20.0]
    assert orb["outcome"] == "orbit" and orb["max_swept_deg"] > 180.0
    # it circles at the contact distance, never overlapping
    assert 2.0 < orb["min_gap"] < 2.0 ** (1.0 / 6.0) * 3.0 + 0.4
    assert sca["outcome"] == "scatter" and sca["max_swept_deg"] < 180.0 and sca["min_gap"] > 2.0
