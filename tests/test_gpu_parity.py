"""GPU parity: the gfx950 library against the FP64 oracle, through the C ABI.

Tolerances (FP32 arithmetic on stored FP32 deviations):
  - velocity: max_x |u_gpu - u_ref| / max_x |u_ref| <= 1e-5;
  - density deviations: max |rho_gpu - rho_ref| <= 1e-9;
  - force: |F_gpu - F_ref| <= 1e-5 of the Stokes drag scale 6 pi eta R U
    (U the larger of the swim speed 2 B1 / 3 and the body speed).  The net
    force on a swimmer tends to zero (self-propulsion is force-free), so the
    net force itself is no scale for its error; torque likewise against
    R times that scale;
  - body positions: 1e-5 of the displacement;
  - owners, link sets and conversion geometry: bit-exact.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from tests import scenes

pytestmark = pytest.mark.gpu

U_TOL = 1e-5
F_TOL = 1e-5
# BF16 keeps 8 significand bits and misses the 1e-3 field bound of the
# reduced-precision form by a little; its tests assert twice the error it
# measures on the same scene
BF16_L2_32 = 2.2e-3


def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_04799_amd import lbsq
    return lbsq


def note(msg):
    print("[gpu-parity] " + msg, flush=True)
    sys.stdout.flush()


# the two population layouts: one buffer updated in place, or two buffers
# with pull streaming
LAYOUTS = ["inplace", "ab"]


def make_pair(shape, bodies=(), mask=None, g=(0.0, 0.0, 0.0), storage="f32", f0=None, audit_every=0,
              layout="inplace"):
    lbsq = gpu()
    o = O.OracleSim(*shape, g=g)
    s = lbsq.Sim(shape, storage=storage, g=g, audit_every=audit_every, layout=layout)
    if mask is not None:
        o.set_static_mask(mask)
        s.set_static_mask(mask)
    modes = {"free": O.FREE, "fixed": O.FIXED, "prescribed": O.PRESCRIBED}
    for b in bodies:
        b = dict(b)
        mode = b.pop("mode", "free")
        o.add_body(b["pos"], b.get("e", (1, 0, 0)), b["R"], B1=b.get("B1", 0.0), beta=b.get("beta", 0.0),
                   mode=modes[mode], v=b.get("v", (0, 0, 0)), w=b.get("w", (0, 0, 0)))
        s.add_squirmer(b["pos"], b.get("e", (1, 0, 0)), b["R"], B1=b.get("B1", 0.0), beta=b.get("beta", 0.0),
                       mode=mode, v=b.get("v", (0, 0, 0)), w=b.get("w", (0, 0, 0)))
    if f0 is not None:
        o.set_populations(f0)
        s.set_populations(f0)
    return o, s


def rel_u_err(s, o):
    rho, u, own = s.fields()
    rho_o, u_o, own_o = o.fields()
    assert np.array_equal(own, own_o), "owner fields differ"
    fl = own_o == 0
    du = np.linalg.norm(u - u_o, axis=0)[fl].max()
    ref = np.linalg.norm(u_o, axis=0)[fl].max()
    drho = np.abs(rho - rho_o)[fl].max()
    return du / ref, drho


def drag_scale(specs, nu=1 / 6):
    """6 pi eta R U of the largest body (eta = rho0 nu, rho0 = 1)."""
    U = max(max(2 / 3 * abs(b.get("B1", 0.0)), np.linalg.norm(b.get("v", (0, 0, 0)))) for b in specs)
    R = max(b["R"] for b in specs)
    return 6 * np.pi * nu * R * max(U, 1e-4), R


def check_bodies(s, o, specs, f_tol=F_TOL, pos_tol=1e-5, exact_pos=False):
    fs, R = drag_scale(specs)
    for i, spec in enumerate(specs):
        b = o.body(i)
        F, T = s.force_torque(i)
        Fo = b["Fbb"] + b["Fc"]
        To = b["Tbb"] + b["Tc"]
        assert np.abs(F - Fo).max() <= f_tol * fs, (i, F, Fo)
        assert np.abs(T - To).max() <= f_tol * fs * R, (i, T, To)
        st = s.body(i)
        if exact_pos:
            assert np.array_equal(st["pos"], b["pos"])
        else:
            disp = np.abs(b["pos"] - np.asarray(spec["pos"])).max()
            assert np.abs(st["pos"] - b["pos"]).max() <= pos_tol * max(disp, 1e-3), (i, st["pos"], b["pos"])


def random_state(shape, seed, amp=1e-3):
    _, w = O.lattice()
    nx, ny, nz = shape
    return w[:, None, None, None] * (1.0 + scenes.noise(seed, (19, nz, ny, nx), amp))


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("shape", [(23, 19, 17), (64, 8, 6)])
def test_periodic_fluid_random_state(shape, layout):
    note("periodic fluid %s, %s" % (shape, layout))
    f0 = random_state(shape, 3)
    o, s = make_pair(shape, f0=f0, layout=layout)
    for _ in range(3):
        o.step(10)
        s.step(10)
        err, drho = rel_u_err(s, o)
        assert err <= U_TOL and drho <= 1e-9, (err, drho)
    fg, fo = s.populations(), o.populations()
    assert np.abs(fg - fo).max() <= 1e-8


@pytest.mark.parametrize("layout", LAYOUTS)
def test_rest_state_is_bitwise_fixed_point(layout):
    note("rest state with a fixed no-slip sphere, %s" % layout)
    lbsq = gpu()
    s = lbsq.Sim((24, 24, 24), layout=layout)
    s.add_squirmer((12, 12, 12), (1, 0, 0), 5.0, B1=0.0, mode="fixed")
    f0 = s.populations()
    s.step(50)
    f1 = s.populations()
    assert np.array_equal(f0, f1)
    # the force is a sum of O(1e3) link terms of size ~0.1 whose pressure
    # parts cancel; what is left is FP64 round-off
    F, T = s.force_torque(0)
    assert np.abs(F).max() < 1e-13 and np.abs(T).max() < 1e-12


@pytest.mark.parametrize("layout", LAYOUTS)
def test_config_small_free_squirmer(layout):
    """32^3 box, R=4 neutral squirmer at the centre swimming along +x,
    B1 = 1e-3, 200 steps (the oracle-size configuration)."""
    note("32^3 R=4 beta=0 free, 200 steps, %s" % layout)
    shape = (32, 32, 32)
    body = dict(pos=(16.0, 16.0, 16.0), e=(1, 0, 0), R=4.0, B1=1e-3, beta=0.0)
    o, s = make_pair(shape, [body], layout=layout)
    for _ in range(4):
        o.step(50)
        s.step(50)
        err, drho = rel_u_err(s, o)
        assert err <= U_TOL, err
        check_bodies(s, o, [body])
    m_g, P_g = s.audit()
    m_o, P_o = o.audit()
    assert abs(m_g - m_o) <= 1e-9 * m_o
    assert np.abs(P_g - P_o).max() <= 1e-5 * np.abs(P_o).max()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("beta", [-5.0, 5.0])
def test_free_squirmer_tilted(beta, layout):
    note("tilted free squirmer beta=%g, %s" % (beta, layout))
    shape = (30, 26, 22)
    e = scenes.unit_vector(np.random.default_rng(11))
    body = dict(pos=(14.3, 12.9, 10.6), e=tuple(e), R=4.5, B1=2e-3, beta=beta)
    o, s = make_pair(shape, [body], layout=layout)
    o.step(120)
    s.step(120)
    err, _ = rel_u_err(s, o)
    assert err <= U_TOL, err
    check_bodies(s, o, [body])
    assert np.abs(s.body(0)["e"] - o.body(0)["e"]).max() < 1e-7


@pytest.mark.parametrize("layout", LAYOUTS)
def test_prescribed_motion_geometry_bit_exact(layout):
    """A prescribed body crosses many cells: owners and the full link set
    equal the oracle's bit for bit at every step; fields stay in tolerance."""
    note("prescribed moving body, per-step link sets, %s" % layout)
    shape = (28, 24, 20)
    body = dict(pos=(9.2, 11.7, 10.1), e=(0, 1, 0), R=3.7, B1=5e-3, beta=2.0, mode="prescribed",
                v=(0.23, 0.07, -0.05), w=(0.0, 0.01, 0.02))
    o, s = make_pair(shape, [body], layout=layout)
    for t in range(25):
        o.step(1)
        s.step(1)
        cg, dg, og = s.links()
        co, do, oo = o.links()
        assert np.array_equal(cg, co) and np.array_equal(dg, do) and np.array_equal(og, oo), t
        assert np.array_equal(s.body(0)["pos"], o.body(0)["pos"])
    err, _ = rel_u_err(s, o)
    assert err <= U_TOL, err
    check_bodies(s, o, [body], exact_pos=True)


def test_prescribed_motion_across_periodic_boundary():
    """Bodies whose boxes wrap around the periodic box: one starts astride a
    corner and crosses two faces, the other crosses one.  Owners, links and
    positions equal the oracle's bit for bit at every step."""
    note("prescribed bodies across the periodic faces, per-step link sets")
    shape = (28, 24, 20)
    bodies = [dict(pos=(0.3, 23.6, 0.4), e=(0, 0, 1), R=3.2, B1=4e-3, beta=-1.5, mode="prescribed",
                   v=(-0.11, 0.09, 0.13), w=(0.01, 0.0, -0.02)),
              dict(pos=(22.4, 12.3, 9.7), e=(1, 0, 0), R=3.6, B1=5e-3, beta=2.5, mode="prescribed",
                   v=(0.27, 0.21, 0.0), w=(0.0, 0.02, 0.0))]
    o, s = make_pair(shape, bodies)
    for t in range(30):
        o.step(1)
        s.step(1)
        cg, dg, og = s.links()
        co, do, oo = o.links()
        assert np.array_equal(cg, co) and np.array_equal(dg, do) and np.array_equal(og, oo), t
        for i in range(2):
            assert np.array_equal(s.body(i)["pos"], o.body(i)["pos"]), (t, i)
    # the first body has wrapped across the x and y faces, the second across x
    p0, p1 = s.body(0)["pos"], s.body(1)["pos"]
    assert p0[0] > 20.0 and p0[1] < 5.0 and p1[0] < 5.0
    err, _ = rel_u_err(s, o)
    assert err <= U_TOL, err
    check_bodies(s, o, bodies, exact_pos=True)


@pytest.mark.parametrize("nbody", [8, 9, 10])
def test_many_bodies_fused_and_separate_update(nbody):
    """Free, fixed and prescribed bodies at the limit of the body update in
    the fluid launch's last boundary block (8, its LDS tables full) and just
    past it (9, 10: the one-block body kernel runs instead).  Fields,
    owners, forces and positions against the oracle."""
    note("%d bodies, %s body update" % (nbody, "fused" if nbody <= 8 else "separate"))
    shape = (40, 40, 24)
    rng = np.random.default_rng(11)
    bodies = []
    for k in range(nbody):
        e = rng.standard_normal(3)
        mode = "fixed" if k % 4 == 3 else ("prescribed" if k == 5 else "free")
        b = dict(pos=(6.5 + 9.0 * (k % 4) + 0.3 * rng.random(), 7.0 + 13.0 * (k // 4) + 0.3 * rng.random(),
                      12.0 + 0.4 * rng.random()),
                 e=tuple(e / np.linalg.norm(e)), R=2.6 + 0.6 * rng.random(), B1=0.01, beta=float(rng.uniform(-3, 3)),
                 mode=mode)
        if mode == "prescribed":
            b.update(v=(0.0, 0.03, 0.05), w=(0.0, 0.0, 0.01))
        bodies.append(b)
    o, s = make_pair(shape, bodies)
    for _ in range(4):
        o.step(15)
        s.step(15)
        err, _ = rel_u_err(s, o)
        assert err <= U_TOL, err
        check_bodies(s, o, bodies)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_two_squirmers_with_contact(layout):
    """Two free squirmers swimming at each other reach WCA contact."""
    note("two squirmers, WCA, %s" % layout)
    shape = (40, 24, 24)
    bodies = [dict(pos=(13.0, 12.0, 12.0), e=(1, 0, 0), R=4.0, B1=0.03, beta=1.0),
              dict(pos=(23.5, 12.3, 12.1), e=(-1, 0.1, 0), R=4.0, B1=0.03, beta=-1.0)]
    lbsq = gpu()
    o = O.OracleSim(*shape, wca_sigma=1.0, wca_eps=0.01)
    s = lbsq.Sim(shape, wca_sigma=1.0, wca_eps=0.01, layout=layout)
    for b in bodies:
        o.add_body(b["pos"], b["e"], b["R"], B1=b["B1"], beta=b["beta"])
        s.add_squirmer(b["pos"], b["e"], b["R"], B1=b["B1"], beta=b["beta"])
    wca_seen = False
    for _ in range(6):
        o.step(25)
        s.step(25)
        wca_seen |= np.abs(o.body(0)["Fwca"]).max() > 0
        err, _ = rel_u_err(s, o)
        assert err <= U_TOL, err
        check_bodies(s, o, bodies)
    assert wca_seen


@pytest.mark.parametrize("layout", LAYOUTS)
def test_tube_with_static_walls(layout):
    note("squirmer in a tube, %s" % layout)
    shape = (24, 24, 40)
    mask = scenes.tube_mask(*shape, radius=9.0)
    body = dict(pos=(12.0, 12.0, 20.0), e=(0, 0, 1), R=4.0, B1=2e-3, beta=3.0)
    o, s = make_pair(shape, [body], mask=mask, layout=layout)
    o.step(150)
    s.step(150)
    err, _ = rel_u_err(s, o)
    assert err <= U_TOL, err
    check_bodies(s, o, [body])
    cg, dg, og = s.links()
    co, do, oo = o.links()
    assert np.array_equal(cg, co) and np.array_equal(dg, do) and np.array_equal(og, oo)


def test_fixed_obstacle_and_squirmer():
    note("fixed obstacle + squirmer")
    shape = (40, 32, 32)
    bodies = [dict(pos=(26.0, 16.0, 16.0), R=6.0, mode="fixed"),
              dict(pos=(12.0, 18.5, 16.0), e=(1, 0, 0), R=4.0, B1=5e-3, beta=-3.0)]
    o, s = make_pair(shape, bodies)
    o.step(100)
    s.step(100)
    err, _ = rel_u_err(s, o)
    assert err <= U_TOL, err
    check_bodies(s, o, bodies)


def test_symmetric_placement_no_lateral_force():
    note("symmetry")
    lbsq = gpu()
    s = lbsq.Sim((24, 24, 24))
    s.add_squirmer((12, 12, 12), (1, 0, 0), 4.0, B1=1e-3, beta=5.0)
    s.step(6)
    F, T = s.force_torque(0)
    assert abs(F[0]) > 0
    # FP32 round-off only: 1e-6 of the axial force (torque: times R)
    assert abs(F[1]) < 1e-6 * abs(F[0]) and abs(F[2]) < 1e-6 * abs(F[0])
    assert np.abs(T).max() < 1e-6 * 4.0 * abs(F[0])


@pytest.mark.parametrize("layout", LAYOUTS)
def test_poiseuille_body_force_hook(layout):
    note("Poiseuille (test body force), %s" % layout)
    H, g = 8, 1e-4
    shape = (4, H + 2, 4)
    mask = np.zeros((4, H + 2, 4), np.uint8)
    mask[:, 0, :] = 1
    mask[:, H + 1, :] = 1
    o, s = make_pair(shape, mask=mask, g=(g, 0.0, 0.0), layout=layout)
    n = int(40 / ((1 / 6) * (np.pi / H) ** 2))
    o.step(n)
    s.step(n)
    err, _ = rel_u_err(s, o)
    assert err <= U_TOL, err
    _, u, _ = s.fields()
    yp = np.arange(1, H + 1) - 0.5
    exact = g / (2 / 6) * yp * (H - yp)
    assert np.abs(u[0, 0, 1:H + 1, 0] - exact).max() <= 1e-5 * exact.max()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("storage,saved_at", [("f32", 60), ("f32", 61), ("f16", 61)])
def test_determinism_and_checkpoint_resume(storage, saved_at, layout):
    """Runs repeat bit for bit, and a state saved after an even or an odd
    number of steps (the two layouts of the in-place buffer) resumes to the
    same bits."""
    note("determinism + checkpoint (%s, saved after %d steps, %s)" % (storage, saved_at, layout))
    lbsq = gpu()
    shape = (32, 28, 24)
    specs = [((15.2, 13.9, 12.3), (0.6, 0.8, 0.0), 4.2, -2.0), ((4.1, 5.3, 6.2), (0.0, -0.6, 0.8), 3.1, 1.5)]

    def fresh():
        s = lbsq.Sim(shape, storage=storage, layout=layout)
        for pos, e, R, beta in specs:
            s.add_squirmer(pos, e, R, B1=0.01, beta=beta)
        return s

    a = fresh()
    a.step(saved_at)
    blob = a.save_state()
    a.step(60)
    b = fresh()
    b.step(saved_at + 60)
    assert np.array_equal(a.populations(), b.populations())
    c = fresh()
    c.load_state(blob)
    c.step(60)
    assert np.array_equal(a.populations(), c.populations())
    for i in range(len(specs)):
        for k in ("pos", "e", "v", "w"):
            assert np.array_equal(a.body(i)[k], c.body(i)[k])


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("saved_at", [40, 41])
def test_checkpoint_with_static_walls(saved_at, layout):
    """A state with static walls (a tube) saved after an even or odd step
    resumes bit for bit in a fresh handle that was never given the wall
    mask: the walls travel with the saved owners, and the streaming path's
    per-cell wall masks and its list of non-wall cell groups are rebuilt
    from them.  A state without walls loaded into a handle with walls
    resumes as its original did."""
    note("checkpoint with static walls (saved after %d steps, %s)" % (saved_at, layout))
    lbsq = gpu()
    shape = (30, 26, 28)
    mask = scenes.tube_mask(*shape, radius=11.0)

    def fresh(walls=True):
        s = lbsq.Sim(shape, layout=layout)
        if walls:
            s.set_static_mask(mask)
        s.add_squirmer((14.3, 12.9, 10.6), (0.3, 0.2, 0.93), 3.5, B1=0.02, beta=-2.0)
        return s

    a = fresh()
    a.step(saved_at)
    blob = a.save_state()
    a.step(50)
    c = fresh(walls=False)
    c.load_state(blob)
    c.step(50)
    assert np.array_equal(a.populations(), c.populations())
    for k in ("pos", "e", "v", "w"):
        assert np.array_equal(a.body(0)[k], c.body(0)[k])
    _, _, own_a = a.fields()
    _, _, own_c = c.fields()
    assert np.array_equal(own_a, own_c) and (own_a == 255).sum() == mask.sum()
    a.close()
    c.close()
    # and the other way: a state without walls loaded into a handle that was
    # given walls drops them (every group of cells streams again)
    b = fresh(walls=False)
    b.step(saved_at)
    blob = b.save_state()
    b.step(50)
    d = fresh(walls=True)
    d.load_state(blob)
    d.step(50)
    assert np.array_equal(b.populations(), d.populations())
    for k in ("pos", "e", "v", "w"):
        assert np.array_equal(b.body(0)[k], d.body(0)[k])
    _, _, own_b = b.fields()
    _, _, own_d = d.fields()
    assert np.array_equal(own_b, own_d) and not (own_d == 255).any()
    b.close()
    d.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_fused_audit_runs_and_flags_nothing(layout):
    note("fused audit, %s" % layout)
    shape = (20, 20, 20)
    o, s = make_pair(shape, [dict(pos=(10, 10, 10), R=4.0, B1=1e-3)], audit_every=5, layout=layout)
    s.step(40)
    o.step(40)
    s.sync()
    m_g, P_g = s.audit()
    m_o, P_o = o.audit()
    assert abs(m_g - m_o) <= 1e-9 * m_o and np.abs(P_g - P_o).max() <= 1e-5 * np.abs(P_o).max()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_audit_changes_no_result(storage, layout):
    """The fused audit (every 100 steps by default in the binding) only
    reads: a run audited every 7 steps ends bit for bit where an unaudited
    one does, populations, owners and bodies."""
    note("audit changes no result (%s, %s)" % (storage, layout))
    lbsq = gpu()
    out = []
    for every in (0, 7):
        s = lbsq.Sim((30, 26, 22), storage=storage, layout=layout, audit_every=every)
        s.add_squirmer((14.3, 12.9, 10.6), (0.6, 0.8, 0.0), 4.5, B1=5e-3, beta=-3.0)
        s.step(100)
        out.append((s.populations(), s.fields()[2], s.body(0)))
        s.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    for k in ("pos", "e", "v", "w"):
        assert np.array_equal(out[0][2][k], out[1][2][k])


def test_nan_is_reported():
    note("NaN detection via the fused audit")
    lbsq = gpu()
    s = lbsq.Sim((16, 16, 16), audit_every=1)
    f = s.populations()
    f[3, 4, 5, 6] = np.nan
    s.set_populations(f)
    s.step(2)
    with pytest.raises(lbsq.LBError) as ei:
        s.sync()
    assert ei.value.code == lbsq.LB_ENAN


def test_error_paths():
    note("error paths")
    lbsq = gpu()
    s = lbsq.Sim((24, 24, 24))
    s.add_squirmer((8, 12, 12), (1, 0, 0), 4.0)
    with pytest.raises(lbsq.LBError) as ei:
        s.add_squirmer((12, 12, 12), (1, 0, 0), 4.0)  # overlaps
    assert ei.value.code == lbsq.LB_EGEOM
    with pytest.raises(lbsq.LBError) as ei:
        s.add_squirmer((18, 12, 12), (0, 0, 0), 2.0)  # zero orientation
    assert ei.value.code == lbsq.LB_EINVAL
    with pytest.raises(lbsq.LBError) as ei:
        s.set_static_mask(np.zeros(24 ** 3))  # after a body
    assert ei.value.code == lbsq.LB_ESTATE
    with pytest.raises(lbsq.LBError) as ei:
        lbsq.Sim((16, 16, 16)).add_squirmer((8, 8, 8), (1, 0, 0), 6.0)  # box too small
    assert ei.value.code == lbsq.LB_EGEOM
    s.step(1)
    with pytest.raises(lbsq.LBError) as ei:
        s.add_squirmer((20, 20, 20), (1, 0, 0), 1.0)
    assert ei.value.code == lbsq.LB_ESTATE


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("storage,l2_tol", [("f16", 1e-3), ("bf16", BF16_L2_32)])
def test_reduced_precision_storage(storage, l2_tol, layout):
    """FP16 (scale 2^14) and BF16 deviation storage: velocity-field L2 error
    and swim velocity against the FP64 oracle."""
    note("storage %s, %s" % (storage, layout))
    shape = (32, 32, 32)
    body = dict(pos=(16.0, 16.0, 16.0), e=(1, 0, 0), R=4.0, B1=1e-3, beta=-3.0)
    o, s = make_pair(shape, [body], storage=storage, layout=layout)
    o.step(200)
    s.step(200)
    _, u, own = s.fields()
    _, u_o, own_o = o.fields()
    assert np.array_equal(own, own_o)
    fl = own_o == 0
    l2 = np.linalg.norm((u - u_o)[:, fl]) / np.linalg.norm(u_o[:, fl])
    note("  %s velocity L2 error %.3e" % (storage, l2))
    assert l2 <= l2_tol
    vg, vo = s.body(0)["v"][0], o.body(0)["v"][0]
    assert abs(vg - vo) <= 5e-3 * abs(vo)


@pytest.mark.slow
def test_full_size_box_128_few_steps():
    """128^3, R=8 pusher at the box centre (the FP32 benchmark workload),
    a few steps compared field by field with the oracle."""
    note("128^3 R=8 beta=-5, 4 steps")
    shape = (128, 128, 128)
    body = dict(pos=(64.0, 64.0, 64.0), e=(1, 0, 0), R=8.0, B1=1e-3, beta=-5.0)
    o, s = make_pair(shape, [body])
    o.step(4)
    s.step(4)
    err, _ = rel_u_err(s, o)
    assert err <= U_TOL, err
    check_bodies(s, o, [body])


@pytest.mark.slow
def test_reduced_precision_tube():
    """The precision form on the tube scene: FP16 (scale 2^14) and BF16
    deviation storage, FP32 collision, FP64 forces and integration, against
    the FP64 oracle after 20 steps: velocity-field L2 error (FP16 <= 1e-3;
    BF16, which misses that bound at 1.1e-3, <= twice that) and the
    swimmer's velocity (0.5%)."""
    lbsq = gpu()
    note("tube 96x96x512, FP16 and BF16 storage, 20 steps")
    shape = (96, 96, 512)
    mask = scenes.tube_mask(*shape, 24.0)
    body = dict(pos=(48.0, 48.0, 256.0), e=(0, 0, 1), R=12.0, B1=1e-3, beta=0.0)
    o = O.OracleSim(*shape)
    o.set_static_mask(mask)
    o.add_body(body["pos"], body["e"], body["R"], B1=body["B1"], beta=body["beta"])
    o.step(20)
    _, u_o, own_o = o.fields()
    fl = own_o == 0
    vo = o.body(0)["v"][2]
    for storage, l2_tol, v_tol in (("f16", 1e-3, 5e-3), ("bf16", 2.2e-3, 5e-3)):
        s = lbsq.Sim(shape, storage=storage)
        s.set_static_mask(mask)
        s.add_squirmer(body["pos"], body["e"], body["R"], B1=body["B1"], beta=body["beta"])
        s.step(20)
        _, u, own = s.fields()
        assert np.array_equal(own, own_o)
        l2 = np.linalg.norm((u - u_o)[:, fl]) / np.linalg.norm(u_o[:, fl])
        vg = s.body(0)["v"][2]
        s.close()
        note("  %s L2 %.2e, swim velocity %.6e vs %.6e" % (storage, l2, vg, vo))
        assert l2 <= l2_tol
        assert abs(vg - vo) <= v_tol * abs(vo)


@pytest.mark.slow
def test_reduced_precision_256():
    """The precision form on the 256^3 scene: a free squirmer R = 16 (beta =
    -3) in a periodic 256^3 box, FP16 and BF16 deviation storage against the
    FP64 oracle after 6 steps: identical owners, velocity-field L2 error
    (FP16 <= 1e-3; BF16, which misses that bound at 1.0e-3, <= twice that)
    and the swimmer's velocity (0.5%)."""
    lbsq = gpu()
    note("256^3 R=16, FP16 and BF16 storage, 6 steps")
    shape = (256, 256, 256)
    body = dict(pos=(127.3, 128.6, 128.2), e=(0.8, 0.6, 0.0), R=16.0, B1=1e-3, beta=-3.0)
    o = O.OracleSim(*shape)
    o.add_body(body["pos"], body["e"], body["R"], B1=body["B1"], beta=body["beta"])
    o.step(6)
    _, u_o, own_o = o.fields()
    fl = own_o == 0
    vo = o.body(0)["v"]
    del o
    for storage, l2_tol, v_tol in (("f16", 1e-3, 5e-3), ("bf16", 2.0e-3, 5e-3)):
        s = lbsq.Sim(shape, storage=storage)
        s.add_squirmer(body["pos"], body["e"], body["R"], B1=body["B1"], beta=body["beta"])
        s.step(6)
        _, u, own = s.fields()
        assert np.array_equal(own, own_o)
        l2 = np.linalg.norm((u - u_o)[:, fl]) / np.linalg.norm(u_o[:, fl])
        vg = s.body(0)["v"]
        s.close()
        note("  %s L2 %.2e, velocity %s vs %s" % (storage, l2, vg, vo))
        assert l2 <= l2_tol
        assert np.linalg.norm(vg - vo) <= v_tol * np.linalg.norm(vo)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_storage_rounds_to_nearest_even(storage):
    """Populations written through the ABI are stored as deviations
    f - w_i rho0, scaled by 2^14 (FP16) or 1 (BF16), rounded to nearest even;
    reading them back must give exactly that rounding (numpy's float16 cast
    is round-to-nearest-even; BF16 is rounded here on the float32 bits)."""
    lbsq = gpu()
    shape = (16, 12, 10)
    _, w = O.lattice()
    rng = np.random.default_rng(11)
    dev = rng.uniform(-2e-3, 2e-3, size=(19,) + shape[::-1]) * 10.0 ** rng.integers(-3, 1, size=(19,) + shape[::-1])
    f = w[:, None, None, None] + dev
    s = lbsq.Sim(shape, storage=storage)
    s.set_populations(f)
    got = s.populations()
    d32 = (f - w[:, None, None, None]).astype(np.float32)
    if storage == "f16":
        q = (d32 * np.float32(2.0 ** 14)).astype(np.float16).astype(np.float64) / 2.0 ** 14
    else:
        u = d32.view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
        q = (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    want = w[:, None, None, None] + q
    assert np.array_equal(got, want), np.abs(got - want).max()


def test_kernel_timing_changes_no_result():
    """Per-launch timing events (stamped by the fluid launch itself) return
    one positive duration per step and leave every population, owner and body
    state bit-identical to an untimed run of the same steps."""
    L = gpu()
    note("kernel timing: 48^3, R = 6 free squirmer, 12 steps timed and untimed")
    out = []
    for timed in (False, True):
        s = L.Sim((48, 48, 48))
        s.add_squirmer((24.3, 23.8, 24.1), (1.0, 0.2, -0.1), 6.0, B1=1e-3, beta=2.0)
        s.step(3)
        if timed:
            s.kernel_timing(True)
        s.step(12)
        if timed:
            ms, launches = s.kernel_time()
            s.kernel_timing(False)
            assert launches == 12
            assert ms > 0.0 and ms / launches < 50.0
        f = s.populations()
        _, _, own = s.fields()
        b = s.body(0)
        s.close()
        out.append((f, own, b))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    for k in ("pos", "e", "v", "w"):
        assert np.array_equal(out[0][2][k], out[1][2][k])


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("storage,n", [("f32", 1023), ("f16", 1290), ("f32", 383), ("f16", 483)])
def test_largest_box_translation_invariance(storage, n, layout):
    """The largest cubic boxes of each population form: 1023^3 in FP32 and
    1290^3 in FP16 (92-103 GB on the device), the largest the 32-bit offsets
    of population planes allow; 383^3 in FP32 and 483^3 in FP16, the
    largest whose tiled populations (19 directions per group of 256 cells)
    fit 32-bit offsets. A prescribed squirmer
    straddling the periodic z boundary, so that it touches the highest
    offsets, must see exactly the forces of the same squirmer shifted by an
    integer number of cells to the low planes. Positions, velocities and
    lever arms are dyadic, so both runs do the same arithmetic; the force
    sums are integer. Owners, forces, torques and the conversion parts must
    agree bit for bit after every step."""
    import torch
    lbsq = gpu()
    note("largest box %d^3 %s %s: translation invariance at the highest offsets" % (n, storage, layout))
    z_top, z_low = n - 1.625, 20.375  # the first straddles the periodic z boundary
    shift = n - 22  # = z_top - z_low, whole cells
    v, w = (2.0 ** -10, 0.0, 2.0 ** -11), (0.0, 0.0, 2.0 ** -12)
    runs = []
    for z in (z_top, z_low):
        s = lbsq.Sim((n, n, n), storage=storage, layout=layout)
        s.add_squirmer((n / 2 + 0.25, n / 2 - 0.125, z), (0.6, 0.8, 0.0), 6.0, B1=1e-3, beta=2.0,
                       mode="prescribed", v=v, w=w)
        out = []
        for _ in range(6):
            s.step(2)
            F, T = s.force_torque(0)
            fp = s.force_parts(0)
            Fbb, Tbb, Fc, Tc = fp["Fbb"], fp["Tbb"], fp["Fc"], fp["Tc"]
            b = s.body(0)
            out.append((F, T, Fbb, Tbb, Fc, Tc, b["pos"], b["e"]))
        assert s.info()["steps"] == 12
        s.close()
        runs.append(out)
        torch.cuda.empty_cache()
    for k, (a, b) in enumerate(zip(runs[0], runs[1])):
        for q in range(6):
            assert np.array_equal(a[q], b[q]), "step %d, quantity %d: %s vs %s" % (2 * k + 2, q, a[q], b[q])
        d = np.mod(a[6] - b[6], n)
        assert np.array_equal(d, np.array([0.0, 0.0, float(shift)])), d
        assert np.array_equal(a[7], b[7])


def test_checkpoint_rejects_the_other_layout():
    """A saved state records its population layout: restoring it into a
    handle of the other layout is refused (the raw population bytes mean
    different slots), into one of the same layout it resumes."""
    lbsq = gpu()
    note("checkpoint across layouts")
    shape = (20, 18, 16)
    a = lbsq.Sim(shape, layout="ab")
    a.add_squirmer((9.3, 8.8, 7.9), (1, 0, 0), 3.5, B1=5e-3)
    a.step(7)
    blob = a.save_state()
    b = lbsq.Sim(shape)
    b.add_squirmer((9.3, 8.8, 7.9), (1, 0, 0), 3.5, B1=5e-3)
    with pytest.raises(lbsq.LBError) as ei:
        b.load_state(blob)
    assert ei.value.code == lbsq.LB_EINVAL
    c = lbsq.Sim(shape, layout="ab")
    c.add_squirmer((9.3, 8.8, 7.9), (1, 0, 0), 3.5, B1=5e-3)
    c.load_state(blob)
    a.step(5)
    c.step(5)
    assert np.array_equal(a.populations(), c.populations())
    for s in (a, b, c):
        s.close()


def test_layouts_agree_bit_for_bit():
    """Both population layouts do the same arithmetic on the same values
    (only the slots differ), so a scene with walls, a free squirmer and a
    prescribed body converting cells gives bit-identical populations, body
    states and forces in both."""
    lbsq = gpu()
    note("in-place and pull layouts, bit for bit")
    shape = (30, 26, 28)
    mask = scenes.tube_mask(*shape, radius=12.0)
    out = []
    for layout in LAYOUTS:
        s = lbsq.Sim(shape, layout=layout)
        s.set_static_mask(mask)
        s.add_squirmer((14.3, 12.9, 10.6), (0.3, 0.2, 0.93), 3.5, B1=0.02, beta=-2.0)
        s.add_squirmer((15.1, 13.4, 20.2), (0, 0, 1), 3.0, B1=5e-3, mode="prescribed", v=(0.0, 0.04, 0.17))
        s.step(33)
        st = [s.body(i) for i in range(2)]
        ft = [s.force_torque(i) for i in range(2)]
        out.append((s.populations(), st, ft))
        s.close()
    assert np.array_equal(out[0][0], out[1][0])
    for i in range(2):
        for k in ("pos", "e", "v", "w"):
            assert np.array_equal(out[0][1][i][k], out[1][1][i][k])
        assert np.array_equal(out[0][2][i][0], out[1][2][i][0]) and np.array_equal(out[0][2][i][1], out[1][2][i][1])


def test_automatic_layout_follows_the_box_size():
    """LB_LAYOUT_AUTO resolves to in place for a small box and to the pull
    layout above 5,500,000 cells; a saved state shows which (it restores
    only into a handle of the same layout)."""
    lbsq = gpu()
    note("automatic layout: 24^3 and 180^3")
    for n, resolved, other in ((24, "inplace", "ab"), (180, "ab", "inplace")):
        a = lbsq.Sim((n, n, n), layout="auto")
        a.step(3)
        blob = a.save_state()
        same = lbsq.Sim((n, n, n), layout=resolved)
        same.load_state(blob)
        diff = lbsq.Sim((n, n, n), layout=other)
        with pytest.raises(lbsq.LBError) as ei:
            diff.load_state(blob)
        assert ei.value.code == lbsq.LB_EINVAL
        for s in (a, same, diff):
            s.close()
