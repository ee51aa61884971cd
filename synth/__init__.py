"""Seeded synthetic inputs for the MPC-SRD step.

This module only draws inputs.  It holds none of the method's arithmetic, and
it is the one module that both the GPU tests and the oracle tests use.

Recipe (the paper's workloads are synthetic fluid boxes; no dataset is
involved):
  * positions i.i.d. uniform in the box [0, L_x) x [0, L_y) x [0, L_z)
    (with walls z is drawn in [0, H));
  * velocities i.i.d. normal with standard deviation sqrt(kT/m) per
    component, then the FP64 mean is subtracted;
  * N = round(density * number of fluid cells).
Lengths are in units of the cell size a.
"""
from __future__ import annotations

import math

import numpy as np

DEG = math.pi / 180.0


def n_particles(L, density: float) -> int:
    return int(round(density * L[0] * L[1] * L[2]))


def box_state(L, density: float = 10.0, kT: float = 1.0, mass: float = 1.0,
              seed: int = 1, n: int | None = None, velocity: str = "normal"):
    """Return (x, v), each float64 of shape (3, n).

    velocity = "normal" (Maxwellian) or "uniform" (a non-Gaussian start:
    uniform in [-b, b] with b = sqrt(3 kT/m), the same variance).
    """
    rng = np.random.default_rng(seed)
    if n is None:
        n = n_particles(L, density)
    x = np.empty((3, n), dtype=np.float64)
    for k in range(3):
        xk = rng.random(n) * float(L[k])
        # random() < 1, but the product can round up to L for non-powers of 2
        x[k] = np.minimum(xk, np.nextafter(float(L[k]), 0.0))
    sd = math.sqrt(kT / mass)
    if velocity == "normal":
        v = rng.normal(0.0, sd, size=(3, n))
    elif velocity == "uniform":
        b = math.sqrt(3.0) * sd
        v = rng.uniform(-b, b, size=(3, n))
    else:
        raise ValueError(velocity)
    if n > 0:
        v -= v.mean(axis=1, keepdims=True)
    return np.ascontiguousarray(x), np.ascontiguousarray(v)


# --- the five workloads --------------------------------------------------
def config(name: str) -> dict:
    """Parameters of the five benchmark workloads (angles in radians)."""
    common = dict(h=0.1, alpha=130.0 * DEG, kT=1.0, mass=1.0, density=10.0, seed=1,
                  mbs=False, walls=False, g=(0.0, 0.0, 0.0))
    if name == "C1":   # plain SRD FP64, 16^3, 100 steps
        return dict(common, L=(16, 16, 16), form="fp64", steps=100, reorder_every=0)
    if name == "C2":   # MBS thermostat, 256^3, reorder every 20 steps, 200 steps
        return dict(common, L=(256, 256, 256), mbs=True, form="fp64", steps=200,
                    reorder_every=20)
    if name == "C3":   # precision form vs plain, 512^3, 100 steps
        return dict(common, L=(512, 512, 512), form="split", steps=100, reorder_every=0)
    if name == "C5":   # Poiseuille flow between no-slip walls, 256x256x64
        return dict(common, L=(256, 256, 64), walls=True, mbs=True, g=(1e-3, 0.0, 0.0),
                    form="split", steps=20000, reorder_every=0)
    raise ValueError(name)


def batch_boxes(nbox: int = 64, seed: int = 4, lmin: int = 16, lmax: int = 96) -> list:
    """Box parameters of the batched ensemble: each edge uniform in {lmin..lmax},
    density uniform in {5, 10, 20}, angle uniform in [90, 150] degrees, kT
    uniform in [0.5, 2], h = 0.1, seed of box b = 1000 + b."""
    rng = np.random.default_rng(seed)
    boxes = []
    for b in range(nbox):
        L = tuple(int(v) for v in rng.integers(lmin, lmax + 1, size=3))
        dens = float(rng.choice([5.0, 10.0, 20.0]))
        alpha = float(rng.uniform(90.0, 150.0)) * DEG
        kT = float(rng.uniform(0.5, 2.0))
        boxes.append(dict(L=L, density=dens, alpha=alpha, kT=kT, h=0.1, mass=1.0,
                          seed=1000 + b, mbs=False, walls=False, g=(0.0, 0.0, 0.0)))
    return boxes
