"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: each checks a closed
form, an exact invariant, a linear-algebra eigenvalue, a brute-force set
computed independently in exact integer arithmetic, or a symmetry.  A plausible
slip anywhere in the oracle (a dropped term, a wrong sign or index, a
transposed operand) breaks at least one of them.

Labels P1..P15 name the pins; each test states what it fixes and where the
paper (or the mathematics) fixes it.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from tests import stokes

pytestmark = pytest.mark.filterwarnings("ignore")


# --------------------------------------------------------------------------
# an independent statement of the D3Q19 lattice (all c in {-1,0,1}^3 with
# |c|^2 <= 2; weights 1/3, 1/18, 1/36)
def d3q19_independent():
    vel = [c for c in itertools.product((-1, 0, 1), repeat=3) if sum(x * x for x in c) <= 2]
    wt = {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}
    return np.array(vel), np.array([wt[sum(x * x for x in c)] for c in vel])


def test_lattice_is_d3q19_with_adjacent_opposites():
    c, w = O.lattice()
    ci, wi = d3q19_independent()
    assert sorted(map(tuple, c)) == sorted(map(tuple, ci))
    for vec, wt in zip(c, w):
        k = [tuple(x) for x in ci].index(tuple(vec))
        assert wt == wi[k]
    assert tuple(c[0]) == (0, 0, 0)
    for i in range(1, 19, 2):
        assert np.array_equal(c[i + 1], -c[i])
    # isotropy of the weights: second and fourth moments
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(3) / 3, atol=1e-15)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(m4, iso, atol=1e-15)


# --------------------------------------------------------------------------
# P1: equilibrium moments (the garbled 1/6 coefficients would fail these)
@pytest.mark.parametrize("seed", range(5))
def test_P1_equilibrium_moments(seed):
    rng = np.random.default_rng(seed)
    rho = 1 + 0.1 * rng.standard_normal()
    u = 0.05 * rng.standard_normal(3)
    c, _ = O.lattice()
    f = O.feq(rho, u)
    assert abs(f.sum() - rho) < 1e-15
    assert np.allclose(c.T @ f, rho * u, atol=1e-16)
    pi = np.einsum("i,ia,ib->ab", f, c, c)
    assert np.allclose(pi, rho / 3 * np.eye(3) + rho * np.outer(u, u), atol=1e-15)


# --------------------------------------------------------------------------
# P2: mass and momentum conservation to round-off in a periodic box
def test_P2_periodic_conservation():
    rng = np.random.default_rng(1)
    n = 12
    s = O.OracleSim(n, n, n)
    _, w = O.lattice()
    f = w[:, None, None, None] * (1 + 0.02 * rng.standard_normal((19, n, n, n)))
    s.set_populations(f)
    m0, p0 = s.audit()
    s.step(1000)
    m1, p1 = s.audit()
    assert abs(m1 - m0) <= 1e-13 * m0
    assert np.max(np.abs(p1 - p0)) <= 1e-13 * m0


# --------------------------------------------------------------------------
# P3: the slip of eq. (squirmer) equals the analytic flow eq. (squirmerflow)
# at r = R minus the swim velocity of eq. (squirmer-speed)
def squirmer_flow(r_vec, e, R, B1, B2):
    """eq. (squirmerflow), typed from the paper independently of the oracle."""
    r = np.linalg.norm(r_vec)
    n = r_vec / r
    en = e @ n
    u = B1 * R ** 3 / r ** 3 * (en * n - e / 3)
    u = u + B2 * (R ** 4 / r ** 4 - R ** 2 / r ** 2) * (1.5 * en ** 2 - 0.5) * n
    u = u + B2 * R ** 4 / r ** 4 * en * (en * n - e)
    return u


@pytest.mark.parametrize("beta", [-5.0, 0.0, 3.0])
def test_P3_slip_matches_analytic_field(beta):
    rng = np.random.default_rng(7)
    B1, R = 1e-3, 8.0
    e = rng.standard_normal(3)
    e /= np.linalg.norm(e)
    for _ in range(20):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        lhs = squirmer_flow(R * n, e, R, B1, beta * B1)
        rhs = O.slip(n * rng.uniform(0.5, 9.0), e, B1, beta) + 2.0 / 3.0 * B1 * e
        assert np.allclose(lhs, rhs, rtol=0, atol=1e-17)
        # tangential, magnitude B1 |sin t| |1 + beta cos t|
        sl = O.slip(n, e, B1, beta)
        cos_t = e @ n
        assert abs(sl @ n) < 1e-18
        assert abs(np.linalg.norm(sl) - B1 * math.sqrt(1 - cos_t ** 2) * abs(1 + beta * cos_t)) < 1e-17


def test_P3_analytic_field_is_divergence_free():
    # guards the typed analytic field itself
    e = np.array([0.3, -0.4, 0.866])
    e /= np.linalg.norm(e)
    h = 1e-4
    for p in ([11.0, 2.0, -3.0], [-4.0, 9.0, 1.5]):
        p = np.array(p)
        div = 0.0
        for k in range(3):
            dp = np.zeros(3)
            dp[k] = h
            div += (squirmer_flow(p + dp, e, 8, 1e-3, 5e-3)[k]
                    - squirmer_flow(p - dp, e, 8, 1e-3, 5e-3)[k]) / (2 * h)
        assert abs(div) < 1e-11


# --------------------------------------------------------------------------
# P4a: shear-wave decay equals the eigenvalue of the linearised one-step
# TRT operator built here from the definition of the scheme
def trt_step_matrix(kvec, lam_e, lam_o):
    c, w = O.lattice()
    opp = np.array([0] + [i + 1 if i % 2 == 1 else i - 1 for i in range(1, 19)])
    P = np.eye(19)[opp]
    E = w[:, None] * (1 + 3 * c @ c.T)  # linearised equilibrium about rest
    I = np.eye(19)
    Cop = I - lam_e * (I + P) / 2 @ (I - E) - lam_o * (I - P) / 2 @ (I - E)
    S = np.diag(np.exp(-1j * (c @ kvec)))  # pull streaming of mode e^{i k.x}
    return Cop @ S


def shear_eigenvalue(N, nu, magic):
    lam_e = 1 / (3 * nu + 0.5)
    lam_o = 1 / (magic / (1 / lam_e - 0.5) + 0.5)
    k = 2 * np.pi / N
    M = trt_step_matrix(np.array([0.0, k, 0.0]), lam_e, lam_o)
    ev, V = np.linalg.eig(M)
    c, _ = O.lattice()
    # the eigenvector carrying x-momentum
    ov = np.abs(c[:, 0] @ V)
    best = np.argmax(ov * (np.abs(ev) > 0.5))
    return ev[best]


@pytest.mark.parametrize("nu", [1 / 6, 0.05])
def test_P4_shear_wave_eigenvalue(nu):
    N, U = 32, 1e-6
    lam = shear_eigenvalue(N, nu, 3 / 16)
    assert abs(lam.imag) < 1e-14
    s = O.OracleSim(1, N, 1, nu=nu)
    y = np.arange(N) + 0.5
    prof = np.sin(2 * np.pi * y / N)
    f = np.stack([O.feq(1.0, [U * p, 0, 0]) for p in prof], axis=1).reshape(19, 1, N, 1)
    s.set_populations(f)

    def amp():
        _, u, _ = s.fields()
        return (u[0, 0, :, 0] @ prof) / (prof @ prof)

    s.step(40)
    a0 = amp()
    s.step(60)
    a1 = amp()
    lam_meas = (a1 / a0) ** (1 / 60)
    assert abs(lam_meas - lam.real) < 1e-10


def test_P4_shear_eigenvalue_tends_to_viscous_decay():
    # |lambda - exp(-nu k^2)| = O(k^4): ratio ~16 per halving of k
    nu = 1 / 6
    errs = [abs(shear_eigenvalue(N, nu, 3 / 16).real - math.exp(-nu * (2 * math.pi / N) ** 2))
            for N in (16, 32, 64)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20


# P4b: body-force Poiseuille between halfway bounce-back walls is exactly
# parabolic when Lambda = 3/16, for any viscosity
def poiseuille_error(nu, magic, H=8, g=1e-4):
    ny = H + 2
    s = O.OracleSim(2, ny, 2, nu=nu, magic=magic, g=(g, 0, 0))
    solid = np.zeros((2, ny, 2), np.uint8)
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    s.set_static_mask(solid)
    s.step(int(40 / (nu * (np.pi / H) ** 2)))
    _, u, _ = s.fields()
    ux = u[0, 0, 1:ny - 1, 0]
    yp = np.arange(1, ny - 1) - 0.5
    exact = g / (2 * nu) * yp * (H - yp)
    return np.max(np.abs(ux - exact)) / exact.max()


@pytest.mark.parametrize("nu", [1 / 6, 0.05, 0.4])
def test_P4_poiseuille_exact_at_magic(nu):
    assert poiseuille_error(nu, 3 / 16) < 1e-12


def test_P4_poiseuille_not_exact_off_magic():
    # the wall-slip error depends on Lambda only: that is what fixes the
    # reading of the printed magic product
    e1 = poiseuille_error(1 / 6, 1 / 4)
    e2 = poiseuille_error(0.05, 1 / 4)
    assert e1 > 1e-3 and abs(e1 - e2) < 1e-9


# --------------------------------------------------------------------------
# P5: Couette flow with one moving wall (moving bounce-back) is linear
def test_P5_couette_exact():
    H, U = 8, 1e-3
    ny = H + 2
    s = O.OracleSim(2, ny, 2)
    solid = np.zeros((2, ny, 2), np.uint8)
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    wu = np.zeros((3, 2, ny, 2))
    wu[0, :, ny - 1, :] = U
    s.set_static_mask(solid, wu)
    s.step(int(40 / ((1 / 6) * (np.pi / H) ** 2)))
    rho, u, _ = s.fields()
    yp = np.arange(1, ny - 1) - 0.5
    assert np.max(np.abs(u[0, 0, 1:ny - 1, 0] - U * yp / H)) < 1e-12 * U * 1e3
    assert np.max(np.abs(u[1:, 0, 1:ny - 1, 0])) < 1e-15


# --------------------------------------------------------------------------
# P6: a FREE swimmer exchanges momentum with the fluid and nothing else
def test_P6_total_momentum_conserved_with_conversions():
    s = O.OracleSim(20, 20, 20)
    s.add_body((10.3, 9.8, 10.1), (1, 0.2, -0.1), 3.5, B1=0.03, beta=-2.0)
    m = s.body(0)["m"]
    _, P0 = s.audit()
    total0 = P0.copy()
    nconv = 0
    scale = 0.0
    for _ in range(150):
        s.step(1)
        st = s.step_stats()
        nconv += st["ncovered"] + st["nuncovered"]
        b = s.body(0)
        scale = max(scale, np.abs(b["Fbb"]).max() + np.abs(b["Fc"]).max())
        _, P = s.audit()
        # the conversion at the end of the step has moved momentum out of or
        # into the fluid; the body receives it in the next integration
        total = P + m * b["v"] + b["Fc_next"]
        assert np.max(np.abs(total - total0)) < 1e-13 * max(1.0, m * np.abs(b["v"]).max())
    assert nconv > 20  # conversions did happen
    assert s.body(0)["pos"][0] > 11.0


# P7: exact mass bookkeeping of links, covered and uncovered cells
def test_P7_mass_bookkeeping():
    s = O.OracleSim(20, 18, 16)
    s.add_body((8.2, 9.1, 7.7), (0, 1, 0), 3.2, B1=0.01, beta=2.0, mode=O.PRESCRIBED,
               v=(0.31, -0.07, 0.05), w=(0.0, 0.02, 0.01))
    M, _ = s.audit()
    seen = 0
    for _ in range(40):
        s.step(1)
        st = s.step_stats()
        M1, _ = s.audit()
        pred = st["link_mass"] - st["covered_mass"] + st["uncovered_mass"]
        assert abs((M1 - M) - pred) < 1e-13 * M
        seen += st["ncovered"] + st["nuncovered"]
        M = M1
    assert seen > 50


# --------------------------------------------------------------------------
# P8: geometry and link set against brute force in exact integer arithmetic
ONE = 1 << 20


def exact_owner(shape, bodies):
    """Owner per cell from the tie-inclusive inside test written with explicit
    periodic images and Python integers (positions and radii rounded
    half-to-even onto the 2^-20 grid)."""
    nx, ny, nz = shape
    own = np.zeros((nz, ny, nx), np.uint8)
    for b, (pos, R) in enumerate(bodies):
        P = [round(Fraction(p) * ONE) for p in pos]
        Rq = round(Fraction(R) * ONE)
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    tot = 0
                    for c, p, L in ((x, P[0], nx), (y, P[1], ny), (z, P[2], nz)):
                        X = (2 * c + 1) * (ONE // 2)
                        tot += min((X - p - s * L * ONE) ** 2 for s in (-1, 0, 1))
                    if tot <= Rq * Rq:
                        own[z, y, x] = b + 1
    return own


def brute_links(own):
    c, _ = O.lattice()
    out = set()
    fluid = own == 0
    for i in range(1, 19):
        # source s = x - c_i, i.e. value at x of own shifted by +c_i
        src = np.roll(own, shift=(c[i][2], c[i][1], c[i][0]), axis=(0, 1, 2))
        for z, y, x in zip(*np.nonzero(fluid & (src != 0))):
            nx_, ny_ = own.shape[2], own.shape[1]
            out.add((int(x + nx_ * (y + ny_ * z)), i, int(src[z, y, x])))
    return out


P8_CASES = [
    ((16, 16, 16), [((8.0, 8.0, 8.0), 4.0)]),                        # lattice-symmetric
    ((16, 14, 12), [((0.3, 13.9, 6.2), 3.7)]),                        # wraps in x and y
    ((18, 18, 18), [((13.5, 14.5, 10.5), 5.0)]),                      # exact ties at |d| = R
    ((18, 18, 18), [((13.5 + 2 ** -21, 14.5, 10.5 - 3 * 2 ** -21), 5.0)]),  # half-quantum rounding
    ((20, 16, 16), [((5.1, 8.2, 7.9), 3.1), ((14.6, 8.0, 8.4), 2.6)]),  # two bodies
]


@pytest.mark.parametrize("shape,bodies", P8_CASES)
def test_P8_owner_and_links_exact(shape, bodies):
    s = O.OracleSim(*shape)
    for pos, R in bodies:
        s.add_body(pos, (1, 0, 0), R, mode=O.FIXED)
    _, _, own = s.fields()
    ref = exact_owner(shape, bodies)
    assert np.array_equal(own, ref)
    cell, d, b = s.links()
    got = list(zip(cell.tolist(), d.tolist(), b.tolist()))
    assert got == sorted(got)
    assert set(got) == brute_links(ref)


def test_P8_conversion_sets_exact():
    shape = (14, 14, 14)
    s = O.OracleSim(*shape)
    s.add_body((5.3, 7.1, 6.9), (1, 0, 0), 3.3, mode=O.PRESCRIBED, v=(0.37, 0.11, -0.05))
    prev = exact_owner(shape, [(s.body(0)["pos"], 3.3)])
    total = 0
    for _ in range(12):
        s.step(1)
        # cells convert right after the body moves: geometry at the new position
        cur = exact_owner(shape, [(s.body(0)["pos"], 3.3)])
        cov, covb, unc, uncb = s.conversions()
        flat_prev, flat_cur = prev.reshape(-1), cur.reshape(-1)
        exp_cov = np.nonzero((flat_prev == 0) & (flat_cur != 0))[0]
        exp_unc = np.nonzero((flat_prev != 0) & (flat_cur == 0))[0]
        assert np.array_equal(np.sort(cov), exp_cov) and np.all(covb == 1)
        assert np.array_equal(np.sort(unc), exp_unc) and np.all(uncb == 1)
        total += len(exp_cov) + len(exp_unc)
        prev = cur
    assert total > 20


# --------------------------------------------------------------------------
# P9: lattice-symmetric placement gives no lateral force and no torque;
# permuting the axes permutes the results
@pytest.mark.parametrize("beta", [-5.0, 5.0])
def test_P9_symmetry(beta):
    def run(e):
        s = O.OracleSim(24, 24, 24)
        s.add_body((12, 12, 12), e, 4.0, B1=1e-3, beta=beta)
        s.step(6)
        return s.body(0)
    bx = run((1, 0, 0))
    Fx = abs(bx["F"][0])
    assert Fx > 0
    # the force is a sum of ~5e3 link terms of size ~0.1, so round-off is
    # ~1e-15 absolute; a broken index or sign gives O(0.1 Fx)
    assert abs(bx["F"][1]) < 1e-9 * Fx and abs(bx["F"][2]) < 1e-9 * Fx
    assert np.abs(bx["T"]).max() < 1e-9 * Fx
    by = run((0, 1, 0))
    assert abs(by["F"][1] - bx["F"][0]) < 1e-9 * Fx
    assert abs(by["v"][1] - bx["v"][0]) < 1e-9 * abs(bx["v"][0])
    assert abs(by["F"][0]) < 1e-9 * Fx and abs(by["F"][2]) < 1e-9 * Fx


# --------------------------------------------------------------------------
# P9 (pair): two squirmers facing each other, offset laterally, placed
# point-symmetrically about the box centre.  The half-turn about the z axis
# through the centre maps the lattice, the D3Q19 set and the pair onto
# themselves: positions stay point images, forces and torques map as
# (x, y, z) -> (-x, -y, z).  B1 is large enough that both bodies convert
# cells within the run.  A body-dependent slip in the link set, the
# conversion or the force bookkeeping breaks this.
def test_P9_head_on_pair_point_symmetry():
    R, B1 = 4.0, 1e-2
    shape = (48, 32, 32)
    c = np.array(shape, dtype=float) / 2.0
    o = O.OracleSim(*shape)
    o.add_body(c + (-9.0, -3.0, 0.0), (1.0, 0.0, 0.0), R, B1=B1, beta=5.0)
    o.add_body(c + (9.0, 3.0, 0.0), (-1.0, 0.0, 0.0), R, B1=B1, beta=5.0)
    converted = 0
    for _ in range(150):
        o.step(1)
        converted += o.step_stats()["ncovered"]
        b0, b1 = o.body(0), o.body(1)
        scale = np.abs(b0["F"]).max() + 1e-30
        assert np.abs(b0["pos"] + b1["pos"] - 2.0 * c).max() < 1e-12
        assert np.abs(b0["e"] + b1["e"]).max() < 1e-12
        turn = np.array([-1.0, -1.0, 1.0])
        assert np.abs(b1["F"] - turn * b0["F"]).max() < 1e-9 * scale
        assert np.abs(b1["T"] - turn * b0["T"]).max() < 1e-9 * scale * R
    assert converted > 0
    o.close()


# --------------------------------------------------------------------------
# P10: the moving-wall term and the momentum exchange against textbook Stokes
# flow.  A staircase sphere's hydrodynamic radius differs from R by a
# fraction of a cell, so these hold to a few per cent at R = 4.  A dropped
# rigid-body term, a wrong lever arm or sign, or a factor in the momentum
# exchange misses by far more.  The references and the steady-state driver
# are in tests/stokes.py.
@pytest.mark.slow
def test_P10_rotating_sphere_torque():
    R, nu = 4.0, 1.0 / 6.0
    w = 1e-2 * nu / R ** 2  # rotational Reynolds number 1e-2
    ratio, phi = [], []
    for L in (24, 32):
        o = O.OracleSim(L, L, L, nu=nu)
        o.add_body((L / 2, L / 2, L / 2), (1.0, 0.0, 0.0), R, mode=O.PRESCRIBED, w=(0.0, 0.0, w))
        o.step(5 * stokes.box_relaxation_steps(L, nu))
        T = o.body(0)["T"]
        o.close()
        assert abs(T[0]) < 1e-9 * abs(T[2]) and abs(T[1]) < 1e-9 * abs(T[2])
        ratio.append(T[2] / (-8.0 * math.pi * nu * R ** 3 * w))
        phi.append(stokes.volume_fraction(R, L))
    # ratio = A (1 + c phi): A is the infinite-box torque factor, c = 1 to
    # leading order (zero mean vorticity of a periodic field)
    c = (ratio[0] - ratio[1]) / (ratio[1] * phi[0] - ratio[0] * phi[1])
    A = ratio[1] / (1.0 + c * phi[1])
    assert 0.6 < c < 1.5, (ratio, c)
    assert abs(A - 1.0) < 0.06, (ratio, A)


@pytest.mark.slow
def test_P10_fixed_sphere_drag_against_hasimoto():
    R, L, nu = 4.0, 24, 1.0 / 6.0
    Kh = stokes.k_hasimoto(stokes.volume_fraction(R, L))
    # superficial speed near 1e-3 nu / R: particle Reynolds number 1e-3
    g = (1e-3 * nu / R) * 6.0 * math.pi * nu * R / (Kh * L ** 3)
    o = O.OracleSim(L, L, L, nu=nu, g=(g, 0.0, 0.0))
    o.add_body((L / 2, L / 2, L / 2), (1.0, 0.0, 0.0), R, mode=O.FIXED)
    o.step(1)
    K, balance = stokes.steady_drag(o.step, o.populations, o.set_populations, o.fields,
                                    lambda: o.body(0)["F"][0], R, L, g, nu)
    o.close()
    assert abs(balance - 1.0) < 1e-3
    assert abs(K / Kh - 1.0) < 0.03, (K, Kh)


# --------------------------------------------------------------------------
# P12: integrator closed forms
def test_P12_constant_force_closed_form():
    m, I = 3.0, 0.7
    F = np.array([2e-4, -1e-4, 5e-5])
    pos = np.array([10.0, 10.0, 10.0])
    v0 = np.array([1e-3, 0.0, -2e-3])
    st = (pos.copy(), np.array([1.0, 0, 0]), v0.copy(), np.zeros(3))
    n = 200
    for _ in range(n):
        st = O.integrate(*st, F, np.zeros(3), m, I, O.FREE, (1000, 1000, 1000))
    assert np.allclose(st[2], v0 + n * F / m, rtol=1e-13, atol=1e-17)
    assert np.allclose(st[0], pos + n * v0 + F / m * n * (n + 1) / 2, rtol=1e-13, atol=1e-12)


def test_P12_constant_rotation_closed_form():
    w = np.array([0.003, -0.001, 0.002])
    e0 = np.array([0.0, 0.6, 0.8])
    st = (np.zeros(3) + 5, e0.copy(), np.zeros(3), w.copy())
    n = 300
    for _ in range(n):
        st = O.integrate(*st, np.zeros(3), np.zeros(3), 1.0, 1.0, O.PRESCRIBED, (50, 50, 50))
    th = np.linalg.norm(w) * n
    k = w / np.linalg.norm(w)
    exp = e0 * math.cos(th) + np.cross(k, e0) * math.sin(th) + k * (k @ e0) * (1 - math.cos(th))
    assert np.allclose(st[1], exp, atol=1e-13)
    assert np.array_equal(st[0], np.zeros(3) + 5)


def test_P12_fixed_body_does_not_move():
    st = O.integrate([3.0, 4.0, 5.0], [1, 0, 0], [0.1, 0, 0], [0, 0.1, 0], [1.0, 1, 1], [1.0, 1, 1],
                     1.0, 1.0, O.FIXED, (10, 10, 10))
    assert list(st[0]) == [3, 4, 5] and list(st[1]) == [1, 0, 0]


def test_P12_periodic_wrap():
    st = O.integrate([9.9, 0.05, 5.0], [1, 0, 0], [0.2, -0.1, 0], [0, 0, 0], [0, 0, 0], [0, 0, 0],
                     1.0, 1.0, O.PRESCRIBED, (10, 10, 10))
    assert np.allclose(st[0], [0.1, 9.95, 5.0], atol=1e-14)


# --------------------------------------------------------------------------
# P13: WCA as the derivative of the shifted Lennard-Jones potential
def test_P13_wca_closed_forms():
    sig, eps = 1.3, 0.02
    assert abs(O.wca(sig, sig, eps) - 24 * eps / sig) < 1e-15
    rc = 2 ** (1 / 6) * sig
    assert O.wca(rc, sig, eps) == 0.0 and O.wca(rc * 1.5, sig, eps) == 0.0
    assert abs(O.wca(rc * (1 - 1e-9), sig, eps)) < 1e-8

    def U(r):
        return 4 * eps * ((sig / r) ** 12 - (sig / r) ** 6) + eps

    for r in (0.9 * sig, sig, 1.05 * sig, 1.1 * sig):
        h = 1e-6 * r
        assert abs(O.wca(r, sig, eps) - (-(U(r + h) - U(r - h)) / (2 * h))) < 1e-6 * 24 * eps / sig
    assert O.wca(0.01 * sig, sig, eps) == O.wca(0.05 * sig, sig, eps)


# --------------------------------------------------------------------------
# P14: the rest state is a fixed point
def test_P14_rest_state_fixed_point():
    s = O.OracleSim(16, 16, 16)
    s.add_body((8, 8, 8), (1, 0, 0), 4.0, B1=0.0, mode=O.FIXED)
    f0 = s.populations().copy()
    s.step(200)
    f1 = s.populations()
    # FP64 round-off of sum(w_i) only; no drift
    assert np.max(np.abs(f1 - f0)) < 1e-15
    b = s.body(0)
    assert np.abs(b["F"]).max() < 1e-14 and np.abs(b["T"]).max() < 1e-13


def test_rates_follow_viscosity_and_magic():
    s = O.OracleSim(4, 4, 4, nu=1 / 6, magic=3 / 16)
    le, lo = s.rates()
    # nu = (1/lam_e - 1/2)/3 and (1/lam_e - 1/2)(1/lam_o - 1/2) = Lambda
    assert abs((1 / le - 0.5) / 3 - 1 / 6) < 1e-15
    assert abs((1 / le - 0.5) * (1 / lo - 0.5) - 3 / 16) < 1e-15


# --------------------------------------------------------------------------
# P11 (oracle part): the free squirmer's swim speed against the speeds the
# paper plots for the same method in its resolution study (fixture with
# citation under tests/golden).  This pins the evaluation point of the wall
# velocity: at the link midpoint the oracle lands within a few per cent of
# the paper; at the solid node centre it swims 13% fast, at the fluid node
# 13% slow (R = 4).
GOLDEN = __import__("pathlib").Path(__file__).resolve().parent / "golden" / "fig_resolution_swim_speed.txt"


def paper_swim_speed(R, L_over_R):
    for line in GOLDEN.read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            r, l, v = line.split()
            if int(r) == R and int(l) == L_over_R:
                return float(v)
    raise KeyError((R, L_over_R))


@pytest.mark.slow
def test_P11_swim_speed_matches_paper_R4():
    R, L, B1 = 4.0, 40, 1e-3
    v0 = 2.0 * B1 / 3.0  # eq. (squirmer-speed)
    o = O.OracleSim(L, L, L)
    o.add_body((L / 2, L / 2, L / 2), (1.0, 0.0, 0.0), R, B1=B1, beta=0.0)
    speeds = []
    for t in range(1000):
        o.step(1)
        b = o.body(0)
        speeds.append(float(np.dot(b["v"], b["e"])) / v0)
    mean = float(np.mean(speeds[300:]))
    ref = paper_swim_speed(4, 10)
    # the paper's own series at R = 4 differ by 0.9% between box sizes and
    # the instantaneous speed fluctuates by about 1%: 3% separates the
    # readings by a factor of four
    assert abs(mean / ref - 1.0) < 0.03, (mean, ref)


# --------------------------------------------------------------------------
# P15: cell conversion alone (Sec. "Numerical Method", the refill and
# zeroing of converted cells and eq. (consforce)), recomputed here from the
# text with no oracle arithmetic.  A prescribed body that translates and
# rotates is moved by a fraction of a cell on a random fluid state, and one
# conversion is run.  Expected, cell by cell:
#   - covered cells (fluid before, body now) hand the momentum sum_i c_i f_i
#     to the body, F_c += p and T_c += d x p, with d the lever arm from the
#     body centre to the cell centre; their populations become zero;
#   - uncovered cells (body before, fluid now) are refilled with the
#     equilibrium at the mean density of their D3Q19 neighbours that are fluid
#     at both time levels (rho0 if there are none) and at the rigid-body
#     velocity v + w x d without the squirmer slip, and the body gives up that
#     momentum: F_c -= rho u, T_c -= d x rho u;
#   - every other fluid cell keeps its populations.
# A sign of either torque term, the order of either cross product, the
# neighbour set or the refill velocity, taken otherwise, misses by orders of
# magnitude more than the tolerance.
def _feq_text(c, w, rho, u):
    cu = c @ u
    return w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * float(u @ u))


def _lever_to(shape, pos, x, y, z):
    d = np.array([x + 0.5, y + 0.5, z + 0.5]) - np.asarray(pos, dtype=float)
    L = np.asarray(shape, dtype=float)
    return d - L * np.round(d / L)


@pytest.mark.parametrize("case", range(3))
def test_P15_conversion_force_torque_and_refill(case):
    shape = [(14, 13, 12), (16, 14, 15), (13, 15, 14)][case]
    rng = np.random.default_rng(1500 + case)
    nx, ny, nz = shape
    R = [3.6, 4.2, 3.3][case]
    pos0 = np.array(shape, dtype=float) / 2.0 + rng.uniform(-0.5, 0.5, 3)
    e = rng.standard_normal(3)
    e /= np.linalg.norm(e)
    v = rng.uniform(-0.05, 0.05, 3)
    w = rng.uniform(-0.04, 0.04, 3)
    step = rng.uniform(0.35, 0.6, 3) * rng.choice([-1.0, 1.0], 3)
    pos1 = pos0 + step
    B1, beta = 0.02, -3.0

    o = O.OracleSim(*shape)
    o.add_body(pos0, e, R, B1=B1, beta=beta, mode=O.PRESCRIBED, v=v, w=w)
    c, wt = O.lattice()
    # random fluid state: density 1 +- 5%, velocity up to 0.05, plus noise
    rho_f = 1.0 + 0.05 * rng.standard_normal((nz, ny, nx))
    u_f = 0.05 * rng.standard_normal((3, nz, ny, nx))
    cu = np.einsum("ia,azyx->izyx", c.astype(float), u_f)
    f = wt[:, None, None, None] * rho_f * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * (u_f ** 2).sum(0))
    f += 1e-3 * rng.standard_normal(f.shape)
    o.set_populations(f)
    f_before = o.populations().copy()  # zero inside the body at pos0

    o.set_body(0, pos1, e, v, w)
    o.convert_only()
    b = o.body(0)
    f_after = o.populations()

    own0 = exact_owner(shape, [(pos0, R)])
    own1 = exact_owner(shape, [(pos1, R)])
    covered = (own0 == 0) & (own1 != 0)
    uncovered = (own0 != 0) & (own1 == 0)
    stay = (own0 == 0) & (own1 == 0)
    assert covered.sum() >= 10 and uncovered.sum() >= 10

    Fc = np.zeros(3)
    Tc = np.zeros(3)
    expect = np.zeros_like(f_before)
    expect[:, stay] = f_before[:, stay]
    for z, y, x in zip(*np.nonzero(covered)):
        p = np.array([sum(c[i][a] * f_before[i, z, y, x] for i in range(19)) for a in range(3)])
        d = _lever_to(shape, pos1, x, y, z)
        Fc += p
        Tc += np.array([d[1] * p[2] - d[2] * p[1], d[2] * p[0] - d[0] * p[2],
                        d[0] * p[1] - d[1] * p[0]])
    for z, y, x in zip(*np.nonzero(uncovered)):
        dens = []
        for i in range(1, 19):
            xx, yy, zz = (x + c[i][0]) % nx, (y + c[i][1]) % ny, (z + c[i][2]) % nz
            if stay[zz, yy, xx]:
                dens.append(f_before[:, zz, yy, xx].sum())
        rho_bar = sum(dens) / len(dens) if dens else 1.0
        d = _lever_to(shape, pos1, x, y, z)
        u = v + np.array([w[1] * d[2] - w[2] * d[1], w[2] * d[0] - w[0] * d[2],
                          w[0] * d[1] - w[1] * d[0]])
        expect[:, z, y, x] = _feq_text(c.astype(float), wt, rho_bar, u)
        p = rho_bar * u
        Fc -= p
        Tc -= np.array([d[1] * p[2] - d[2] * p[1], d[2] * p[0] - d[0] * p[2],
                        d[0] * p[1] - d[1] * p[0]])

    # covered and uncovered momenta are each ~0.05 per cell; their sums and
    # lever-arm products are O(1), so FP64 reordering gives ~1e-15
    assert np.abs(b["Fc_next"] - Fc).max() < 1e-14 * max(1.0, np.abs(Fc).max())
    assert np.abs(b["Tc_next"] - Tc).max() < 1e-14 * max(1.0, np.abs(Tc).max() * R)
    assert np.abs(f_after - expect).max() < 1e-15
    # the torque is not degenerate: a flipped sign or swapped product moves
    # it by far more than the tolerance
    assert np.abs(Tc).max() > 1e-3
    o.close()
