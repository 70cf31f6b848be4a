"""Steady Stokes flow past one sphere in a periodic box: reference values
and a driver that reaches the steady state, for the P10 tests.

The drag reference is the drag factor of a simple cubic array of spheres,
F = 6 pi eta R U / K(phi), with U the superficial velocity: the fluid's
velocity averaged over the whole cell, relative to the spheres.  The series
is Hasimoto (J. Fluid Mech. 5, 1959) for the leading terms and Sangani &
Acrivos (Int. J. Multiphase Flow 8, 1982) for the rest.  It gives
K = 0.720 / 0.812 / 0.859 at L = 10R / 15R / 20R.

The torque reference is Stokes' -8 pi eta R^3 omega.  In a periodic box the
velocity field has zero mean vorticity.  The fluid therefore turns against
the sphere at about phi * omega, which raises the torque by the factor
1 / (1 - phi) to leading order.
"""
import math

import numpy as np

# D3Q19 weights in the canonical order: rest, 6 axis links, 12 edge links
W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)


def k_hasimoto(phi):
    c = phi ** (1.0 / 3.0)
    return (1.0 - 1.7601 * c + phi - 1.5593 * phi ** 2 + 3.9799 * phi ** (8.0 / 3.0)
            - 3.0734 * phi ** (10.0 / 3.0))


def volume_fraction(R, L):
    return 4.0 / 3.0 * math.pi * R ** 3 / float(L) ** 3


def box_relaxation_steps(L, nu):
    """e-folding time of the box's slowest viscous mode, k = 2 pi / L."""
    return int(math.ceil(L * L / (4.0 * math.pi ** 2 * nu)))


def steady_drag(step, get_f, set_f, fields, force_x, R, L, g, nu, rho0=1.0, iterations=5):
    """Drive a fixed sphere in fluid pushed by the body-force density g along
    x to its steady state.  Return (K, F / (g N_fluid)).

    The mean flow of a periodic box relaxes slowly, with time constant
    N_fluid K / (6 pi eta R).  That is thousands of box-relaxation times at
    L = 20R.  Stokes flow is linear in the forcing, however, so the steady
    state is a fixed point of this map:
    1. let the flow shape relax for two box-relaxation times;
    2. scale every fluid population's deviation from rest so that the drag
       equals the total body force.
    The drag then stays at g N_fluid (momentum balance), which the second
    return value shows.

    The callables take and return the canonical FP64 population array
    f[19][nz][ny][nx] (solid cells 0), the fields (rho, u, owner) and the
    body's hydrodynamic force along x.
    """
    _, _, own = fields()
    fluid = own == 0
    n_fluid = int(fluid.sum())
    tp = box_relaxation_steps(L, nu)
    rest = (rho0 * W)[:, None, None, None]
    for _ in range(iterations):
        step(2 * tp)
        F = force_x()
        f = get_f()
        f = np.where(fluid[None], rest + (g * n_fluid / F) * (f - rest), 0.0)
        set_f(f)
        del f
    step(2 * tp)
    F = force_x()
    _, u, _ = fields()
    u_sup = float(u[0][fluid].sum()) / float(L) ** 3
    eta = rho0 * nu
    return 6.0 * math.pi * eta * R * u_sup / F, F / (g * n_fluid)


def squirmer_field(d, e, R, B1, B2):
    """Flow of a squirmer in unbounded fluid (Blake 1971; Ishikawa et al.
    2006), the paper's eq. (squirmerflow): lab-frame velocity at the offsets
    d[3][M] from the centre, for orientation e.  It vanishes at infinity and
    equals slip + (2/3) B1 e on r = R."""
    r = np.sqrt((d * d).sum(axis=0))
    n = d / r
    en = (e[:, None] * n).sum(axis=0)
    q3, q2, q4 = (R / r) ** 3, (R / r) ** 2, (R / r) ** 4
    u = B1 * q3 * (en * n - e[:, None] / 3.0)
    u += B2 * (q4 - q2) * (1.5 * en * en - 0.5) * n
    u += B2 * q4 * en * (en * n - e[:, None])
    return u


def periodic_squirmer_field(x, centre, e, R, B1, B2, L, shells):
    """eq. (squirmerflow) summed over the periodic images n L with |n| <= shells
    (a spherical shell of images).  The sums of the r^-2 and r^-3 terms
    converge only conditionally: the spherical order fixes them up to a
    uniform velocity, which a comparison removes."""
    x = np.asarray(x, dtype=float)
    c = np.asarray(centre, dtype=float)[:, None]
    e = np.asarray(e, dtype=float)
    u = np.zeros_like(x)
    rng = range(-shells, shells + 1)
    for i in rng:
        for j in rng:
            for k in rng:
                if i * i + j * j + k * k > shells * shells:
                    continue
                shift = np.array([i, j, k], dtype=float)[:, None] * L
                u += squirmer_field(x - c - shift, e, R, B1, B2)
    return u


def image_sum_mean_gradient(centre, e, R, B1, B2, L, shells, m=40):
    """Box average of the velocity gradient of periodic_squirmer_field over
    the cube of side L centred on the body: (1/V) times the surface integral
    of u n over its faces, with an m x m midpoint rule per face.

    A periodic field has zero mean gradient.  The spherical order of the image
    sum leaves a uniform strain, proportional to the stresslet density B2 / L^3;
    subtracting G . (x - centre) turns the sum into the periodic solution.
    """
    c = np.asarray(centre, dtype=float)
    G = np.zeros((3, 3))
    g = (np.arange(m) + 0.5) * L / m - L / 2.0
    A, B = np.meshgrid(g, g, indexing="ij")
    for k in range(3):
        o = [j for j in range(3) if j != k]
        for sign in (1.0, -1.0):
            pts = np.zeros((3, m * m))
            pts[o[0]] = c[o[0]] + A.ravel()
            pts[o[1]] = c[o[1]] + B.ravel()
            pts[k] = c[k] + sign * L / 2.0
            u = periodic_squirmer_field(pts, c, e, R, B1, B2, L, shells)
            G[:, k] += sign * u.mean(axis=1) / L
    return G
