"""Scattering off, or orbiting around, a fixed spherical obstacle (Sec.
"Scattering off and Orbiting around a Stationary Spherical Obstacle").

A squirmer of radius R starts a surface gap g0 away from a fixed no-slip
sphere of radius A and swims toward its centre along a heading turned by a
small angle off the radial direction (the symmetry breaking the paper
describes).  The run is classified as

  - ``orbit``: the swimmer revolves more than halfway around the obstacle
    (the swept angle of its position about the obstacle's centre exceeds
    180 degrees), the paper's criterion;
  - ``scatter``: after contact (surface gap below ``contact_gap``) it
    leaves again, the gap rising above ``release_gap``;
  - ``no contact``: the run ends without contact (the swimmer is held off
    or turned away before it reaches the obstacle);
  - ``undecided``: contact, but neither of the above within the run.

The motion stays in the plane spanned by the start position and the
heading (the z = centre plane), so the swept angle is measured there.
`bisect` brackets the critical beta between an orbiting and a scattering
value, as the paper does once one of each is known.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import lbsq


def classify(gaps, angles, contact_gap=1.5, release_gap=16.0):
    """Outcome of a run from its sampled surface gaps and unwrapped swept
    angles (radians, from the start).  Returns (outcome, index) with the
    sample index at which it was decided (or the last one)."""
    touched = None
    for k, (g, a) in enumerate(zip(gaps, angles)):
        if abs(a) > math.pi:
            return "orbit", k
        if touched is None and g < contact_gap:
            touched = k
        if touched is not None and g > release_gap:
            return "scatter", k
    if touched is None:
        return "no contact", len(gaps) - 1
    return "undecided", len(gaps) - 1


def start_geometry(A, R, n, gap0, angle_deg=0.0, y0=0.0):
    """Obstacle centre, swimmer start and heading.  The obstacle sits at the
    box centre; the swimmer starts on the -x side with its surface gap0 from
    the obstacle's (measured along x), displaced by y0 along +y, heading
    along +x turned by angle_deg towards +y.  The paper breaks the symmetry
    of the radial approach either way: by a small angle (its text) or by a
    small offset y0 (its figure's inset)."""
    c = np.array([n / 2.0, n / 2.0, n / 2.0])
    d0 = A + R + gap0
    start = c + np.array([-d0, float(y0), 0.0])
    th = math.radians(angle_deg)
    return c, start, (math.cos(th), math.sin(th), 0.0)


def orbit_run(beta, A=50.0, R=8.0, n=384, B1=1e-3, gap0=16.0, angle_deg=5.0, y0=0.0, max_steps=600000,
              every=2000, storage="f16", layout="auto", wca_sigma=1.0, wca_eps=0.01, contact_gap=None,
              release_gap=16.0, log=None):
    """One run; stops as soon as the outcome is decided.  Returns a dict with
    the outcome, the step it was decided at, and the sampled trajectory
    (step, surface gap, swept angle in degrees, heading angle to the
    obstacle centre in degrees).  The contact repulsion (WCA, surface to
    surface) has range 2^(1/6) wca_sigma; contact is a gap below that range
    plus 0.4 cells unless contact_gap is given."""
    if contact_gap is None:
        contact_gap = 2.0 ** (1.0 / 6.0) * wca_sigma + 0.4
    c, start, e = start_geometry(A, R, n, gap0, angle_deg, y0)
    s = lbsq.Sim((n, n, n), storage=storage, layout=layout, wca_sigma=wca_sigma, wca_eps=wca_eps)
    s.add_squirmer(tuple(c), (1.0, 0.0, 0.0), A, B1=0.0, mode="fixed")
    s.add_squirmer(tuple(start), e, R, B1=B1, beta=beta)
    phi0 = math.atan2(start[1] - c[1], start[0] - c[0])
    prev, unwrap = phi0, 0.0
    rows, gaps, angles = [], [], []
    t0 = time.time()
    outcome, k = "undecided", 0
    steps = 0
    try:
        while steps < max_steps:
            s.step(every)
            steps += every
            b = s.body(1)
            r = b["pos"] - c
            r -= n * np.round(r / n)
            dist = float(np.linalg.norm(r))
            phi = math.atan2(r[1], r[0])
            dphi = phi - prev
            dphi -= 2.0 * math.pi * round(dphi / (2.0 * math.pi))
            unwrap += dphi
            prev = phi
            heading = math.degrees(math.acos(max(-1.0, min(1.0, float(-np.dot(r, b["e"]) / dist)))))
            gap = dist - A - R
            gaps.append(gap)
            angles.append(unwrap)
            rows.append((steps, gap, math.degrees(unwrap), heading))
            if log is not None and (steps // every) % 25 == 0:
                log("  beta %g step %d: gap %.2f, swept %.1f deg, heading %.1f deg off the centre (%.0f s)"
                    % (beta, steps, gap, math.degrees(unwrap), heading, time.time() - t0))
            outcome, k = classify(gaps, angles, contact_gap, release_gap)
            if outcome in ("orbit", "scatter"):
                break
    finally:
        s.close()
    return {"beta": beta, "outcome": outcome, "decided_at": rows[k][0] if rows else 0, "steps": steps,
            "min_gap": float(min(gaps)) if gaps else None,
            "max_swept_deg": float(max(abs(a) for a in angles) * 180.0 / math.pi) if angles else 0.0,
            "trajectory": rows, "A": A, "R": R, "n": n, "B1": B1, "gap0": gap0, "angle_deg": angle_deg, "y0": y0,
            "wca_sigma": wca_sigma, "wca_eps": wca_eps,
            "storage": storage, "seconds": time.time() - t0}


def bisect(beta_orbit, beta_scatter, tol=1.0, run=orbit_run, **kw):
    """Bracket the critical beta between a value known to orbit and one known
    to scatter (or not to orbit), halving the bracket until it is narrower
    than tol.  Returns the bracket and every run made."""
    lo, hi = float(beta_orbit), float(beta_scatter)
    runs = []
    while abs(hi - lo) > tol:
        mid = 0.5 * (lo + hi)
        r = run(mid, **kw)
        runs.append(r)
        if r["outcome"] == "orbit":
            lo = mid
        else:
            hi = mid
    return (lo, hi), runs


def main(argv=None):
    """Bracket the critical beta at one obstacle size: check that the first
    beta orbits and the second does not (unless --known), then bisect until
    the bracket is narrower than --tol or --budget seconds have passed.
    Prints one line per run and the bracket; --out writes every run."""
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--A", type=float, default=50.0, help="obstacle radius")
    ap.add_argument("--R", type=float, default=8.0, help="squirmer radius")
    ap.add_argument("--n", type=int, default=320, help="cubic box edge")
    ap.add_argument("--B1", type=float, default=2e-3)
    ap.add_argument("--sigma", type=float, default=3.0, help="WCA range parameter")
    ap.add_argument("--eps", type=float, default=0.01, help="WCA strength")
    ap.add_argument("--angle", type=float, default=30.0, help="heading off radial, degrees")
    ap.add_argument("--gap0", type=float, default=5.0, help="start surface gap")
    ap.add_argument("--max-steps", type=int, default=450000)
    ap.add_argument("--storage", default="f16")
    ap.add_argument("--orbit", type=float, default=-45.0, help="a beta expected to orbit")
    ap.add_argument("--scatter", type=float, default=-20.0, help="a beta expected not to")
    ap.add_argument("--known", action="store_true", help="the two ends are known; do not rerun them")
    ap.add_argument("--tol", type=float, default=1.5)
    ap.add_argument("--budget", type=float, default=1e9, help="start no run after this many seconds")
    ap.add_argument("--out", default=None, help="JSON file for every run")
    a = ap.parse_args(argv)
    t0 = time.time()
    runs = []

    def one(beta):
        r = orbit_run(beta, A=a.A, R=a.R, n=a.n, B1=a.B1, gap0=a.gap0, angle_deg=a.angle, max_steps=a.max_steps,
                      storage=a.storage, wca_sigma=a.sigma, wca_eps=a.eps, log=lambda m: print(m, flush=True))
        runs.append(r)
        print("beta %g: %s at step %d (min gap %.2f, swept %.1f deg, %.0f s)"
              % (beta, r["outcome"], r["decided_at"], r["min_gap"], r["max_swept_deg"], r["seconds"]), flush=True)
        if a.out:
            with open(a.out, "w") as f:
                json.dump(runs, f)
        return r

    lo, hi = a.orbit, a.scatter
    if not a.known:
        if one(lo)["outcome"] != "orbit":
            print("no bracket: beta %g does not orbit" % lo)
            return 1
        if one(hi)["outcome"] == "orbit":
            print("no bracket: beta %g orbits too" % hi)
            return 1

    while abs(hi - lo) > a.tol and time.time() - t0 < a.budget:
        mid = round(0.5 * (lo + hi))
        if mid in (lo, hi):
            break
        if one(mid)["outcome"] == "orbit":
            lo = mid
        else:
            hi = mid
    ran = {r["beta"] for r in runs}
    note = "" if lo in ran and hi in ran else " (an end taken as known, not run)"
    print("bracket: beta %g orbits, beta %g does not (A/R = %g)%s" % (lo, hi, a.A / a.R, note))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
