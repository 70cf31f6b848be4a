"""Seeded synthetic inputs shared by the oracle and the GPU tests.

Only geometry and random numbers live here (box sizes, body placements,
orientations, noise); none of the lattice Boltzmann arithmetic does.
"""
import numpy as np


def unit_vector(rng):
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def noise(seed, shape, amplitude):
    """Gaussian noise of the given shape (population perturbations)."""
    return amplitude * np.random.default_rng(seed).standard_normal(shape)


def tube_mask(nx, ny, nz, radius, centre=None, axis="z"):
    """Static wall mask [z, y, x]: cells whose centre lies at or beyond
    `radius` from the tube axis (parallel to z, or to x with axis="x";
    centre gives the axis' position in the other two coordinates)."""
    if axis == "x":
        cy, cz = centre if centre is not None else (ny / 2.0, nz / 2.0)
        y = np.arange(ny) + 0.5
        z = np.arange(nz) + 0.5
        r2 = (y[None, :] - cy) ** 2 + (z[:, None] - cz) ** 2
        return np.broadcast_to((r2 >= radius ** 2)[:, :, None], (nz, ny, nx)).astype(np.uint8)
    cx, cy = centre if centre is not None else (nx / 2.0, ny / 2.0)
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    r2 = (x[None, :] - cx) ** 2 + (y[:, None] - cy) ** 2
    return np.broadcast_to((r2 >= radius ** 2)[None, :, :], (nz, ny, nx)).astype(np.uint8)


def obstacle_scene(seed, n=256, A=32.0, R=16.0):
    """Squirmer approaching a fixed sphere: impact parameter b ~ U[0, 2R]."""
    rng = np.random.default_rng(seed)
    b = rng.uniform(0.0, 2.0 * R)
    c = n / 2.0
    return {"obstacle": (c, c, c), "A": A, "squirmer": (c - A - 2 * R, c + b, c), "R": R, "b": b}
