"""The orbit/scatter driver's bookkeeping (CPU): the classification of a
sampled trajectory by the paper's criterion (Sec. "Scattering off and
Orbiting around a Stationary Spherical Obstacle": an orbit revolves more
than halfway around the obstacle) and the bisection over beta, on
synthetic trajectories and a fake run.  A GPU run of the driver on each
side of the boundary is in test_gpu_physics.py (E6)."""
import math

import numpy as np

from paper_1903_04799_amd import orbit


def test_orbit_needs_more_than_half_a_revolution():
    gaps = [10.0, 3.0, 1.0, 1.1, 1.0, 1.2]
    angles = [0.0, 0.2, 1.0, 2.0, 3.0, 3.0]
    assert orbit.classify(gaps, angles)[0] == "undecided"
    angles[-1] = math.pi + 0.01
    assert orbit.classify(gaps, angles) == ("orbit", 5)
    # either sense of revolution counts
    assert orbit.classify(gaps, [-a for a in angles]) == ("orbit", 5)


def test_scatter_needs_contact_then_release():
    # leaving without ever touching is not a scattering off the obstacle
    assert orbit.classify([10.0, 12.0, 30.0], [0.0, 0.1, 0.2])[0] == "no contact"
    out = orbit.classify([10.0, 1.0, 5.0, 17.0], [0.0, 0.3, 0.5, 0.6])
    assert out == ("scatter", 3)
    # a release before contact does not count
    assert orbit.classify([20.0, 1.2, 1.0], [0.0, 0.1, 0.2])[0] == "undecided"


def test_bisection_brackets_the_critical_beta():
    critical = -33.3

    def fake(beta, **kw):
        return {"beta": beta, "outcome": "orbit" if beta < critical else "scatter"}

    (lo, hi), runs = orbit.bisect(-50.0, -20.0, tol=1.0, run=fake)
    assert lo <= critical <= hi and hi - lo <= 1.0
    assert all(r["outcome"] == ("orbit" if r["beta"] < critical else "scatter") for r in runs)


def test_start_geometry_angle_or_offset():
    A, R, n, gap0 = 96.0, 8.0, 320, 4.0
    # an angled start: the surface gap is gap0, the heading turned by the angle
    c, start, e = orbit.start_geometry(A, R, n, gap0, angle_deg=30.0)
    assert abs(np.linalg.norm(start - c) - A - R - gap0) < 1e-12
    assert abs(math.degrees(math.atan2(e[1], e[0])) - 30.0) < 1e-12
    # an offset start along +x: the heading line passes the obstacle centre
    # at distance y0 (the impact parameter of the paper's inset)
    c, start, e = orbit.start_geometry(A, R, n, gap0, y0=2.5)
    rel = c - start
    miss = abs(rel[0] * e[1] - rel[1] * e[0])
    assert e == (1.0, 0.0, 0.0) and abs(miss - 2.5) < 1e-12
    # both stay in the z = n/2 plane, where the swept angle is measured
    assert start[2] == c[2] == n / 2.0


def test_command_line_brackets_and_checks_its_ends(monkeypatch, capsys, tmp_path):
    critical = -29.5
    calls = []

    def fake(beta, **kw):
        calls.append(beta)
        return {"beta": beta, "outcome": "orbit" if beta <= critical else "scatter", "decided_at": 1000,
                "min_gap": 2.7, "max_swept_deg": 100.0, "seconds": 0.0}

    monkeypatch.setattr(orbit, "orbit_run", fake)
    out = tmp_path / "runs.json"
    assert orbit.main(["--orbit", "-45", "--scatter", "-20", "--tol", "1.5", "--out", str(out)]) == 0
    assert calls[:2] == [-45.0, -20.0]
    line = capsys.readouterr().out.strip().splitlines()[-1]
    assert line == "bracket: beta -30 orbits, beta -29 does not (A/R = 6.25)"
    import json
    assert [r["beta"] for r in json.loads(out.read_text())] == calls
    # with known ends only the midpoints run, and the bracket says when an
    # end of it was not run
    calls.clear()
    assert orbit.main(["--orbit", "-30", "--scatter", "-6", "--known", "--A", "96"]) == 0
    assert -30.0 not in calls and -6.0 not in calls and calls[0] == -18.0
    # every midpoint scattered, so the orbiting end is the unrun -30
    line = capsys.readouterr().out.strip().splitlines()[-1]
    assert line == "bracket: beta -30 orbits, beta -29 does not (A/R = 12) (an end taken as known, not run)"
    calls.clear()
    assert orbit.main(["--orbit", "-40", "--scatter", "-20", "--known"]) == 0
    line = capsys.readouterr().out.strip().splitlines()[-1]
    assert line == "bracket: beta -30 orbits, beta -29 does not (A/R = 6.25)" and -40.0 not in calls
    # ends on the wrong side: no bracket
    assert orbit.main(["--orbit", "-20", "--scatter", "-10"]) == 1
    assert orbit.main(["--orbit", "-45", "--scatter", "-40"]) == 1
