"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module generates initial density fields only; it holds none of the
method's arithmetic (no operator, scheme or solver code) and imports neither
the GPU library nor the oracle.  Every generator is deterministic in its seed
(numpy PCG64 via ``default_rng``).

Arrays are float64, shape (n, m), x (index i) fastest; the cell (i, j) centre
is ((i + 1/2) h, (j + 1/2) h) (App. A, cell-centred grid with p_r = (r - 1/2) h
for 1-based r).

Workloads (each named by what it is):

* ``noise``: phi0 = mean + U[-amp, amp] per cell, the random-perturbation
  initial data of the effective-time-step study (Sec. 4.4) with the amplitude
  of the first workload below.
* ``crystallites``: a 0.07 liquid background with three circular crystallites
  of the one-mode hexagonal profile of Sec. 4.6 (eq. single_mode_density),
  each at a random centre and a random orientation.
* ``paper_initial_data``: the smooth initial field of the convergence tests
  (Sec. 4.1, eq. initial-data) on Omega = (0, 32)^2.
* ``batch``: 64 independent simulations with sizes, eps, mean density and
  beta drawn per simulation.
* ``noise3``: the three-dimensional workload, 0.07 + U[-0.05, 0.05] on an
  m x n x l grid.
* ``strained_crystal``: the sheared-crystal set-up of Sec. 4.6 on its 512 x 400
  grid: a band of 20 atomic layers of the one-mode profile (solid density
  phi_s, amplitude A(phi_s, eps)) in a liquid of density phi_l, a pinning
  weight of 2 in strips of height pi around the bottom and top rows of atoms,
  and a prescribed configuration equal to the crystal with its bottom row
  shifted left by 4 % of 2 pi.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def cell_centres(m: int, n: int, h: float):
    x = (np.arange(m) + 0.5) * h
    y = (np.arange(n) + 0.5) * h
    return np.meshgrid(x, y, indexing="xy")  # shapes (n, m)


def noise(m: int, n: int, mean: float = 0.07, amp: float = 0.05, seed: int = 1) -> np.ndarray:
    """mean + uniform noise in [-amp, amp] on every cell."""
    rng = np.random.default_rng(seed)
    return mean + rng.uniform(-amp, amp, size=(n, m))


def noise3(m: int, n: int, l: int, mean: float = 0.07, amp: float = 0.05,
           seed: int = 7) -> np.ndarray:
    """Three-dimensional grid (shape (l, n, m), x fastest): mean + U[-amp, amp]."""
    rng = np.random.default_rng(seed)
    return mean + rng.uniform(-amp, amp, size=(l, n, m))


def crystallites(m: int, n: int, h: float, count: int = 3, radius_cells: float = 20.0,
                 background: float = 0.07, amplitude: float = 0.3, seed: int = 2,
                 max_tries: int = 10000) -> np.ndarray:
    """Background density with `count` circular one-mode crystallites.

    Inside a disc of radius `radius_cells * h` around a centre (xc, yc), in
    coordinates rotated by theta about the centre (minimum periodic image),
    phi = background + amplitude*(cos x' cos(y'/sqrt3) - cos(2 y'/sqrt3)/2).
    Centres are uniform on the domain and kept more than two radii apart
    (periodic distance); theta is uniform in [0, pi/3) since the profile is
    invariant under rotations by pi/3.
    """
    rng = np.random.default_rng(seed)
    Lx, Ly = m * h, n * h
    R = radius_cells * h
    centres = []
    tries = 0
    while len(centres) < count:
        tries += 1
        if tries > max_tries:
            raise ValueError("could not place non-overlapping crystallites")
        c = (rng.uniform(0, Lx), rng.uniform(0, Ly))
        ok = True
        for (a, b) in centres:
            dx = (c[0] - a + Lx / 2) % Lx - Lx / 2
            dy = (c[1] - b + Ly / 2) % Ly - Ly / 2
            if math.hypot(dx, dy) <= 2 * R:
                ok = False
                break
        if ok:
            centres.append(c)
    thetas = rng.uniform(0, math.pi / 3, size=count)
    X, Y = cell_centres(m, n, h)
    phi = np.full((n, m), background, dtype=np.float64)
    for (xc, yc), th in zip(centres, thetas):
        dx = (X - xc + Lx / 2) % Lx - Lx / 2
        dy = (Y - yc + Ly / 2) % Ly - Ly / 2
        inside = dx * dx + dy * dy <= R * R
        xr = math.cos(th) * dx + math.sin(th) * dy
        yr = -math.sin(th) * dx + math.cos(th) * dy
        prof = np.cos(xr) * np.cos(yr / math.sqrt(3)) - 0.5 * np.cos(2 * yr / math.sqrt(3))
        phi = np.where(inside, background + amplitude * prof, phi)
    return phi


def paper_initial_data(m: int, n: int, L: float = 32.0) -> np.ndarray:
    """Smooth initial field of the convergence tests on (0, L)^2 (Sec. 4.1)."""
    h = L / m
    X, Y = cell_centres(m, n, h)
    p = math.pi
    return (0.07 - 0.02 * np.cos(2 * p * (X - 12) / 32) * np.sin(2 * p * (Y - 1) / 32)
            + 0.02 * np.cos(p * (X + 10) / 32) ** 2 * np.cos(p * (Y + 3) / 32) ** 2
            - 0.01 * np.sin(4 * p * X / 32) ** 2 * np.sin(4 * p * (Y - 6) / 32) ** 2)


def strained_crystal(m: int = 512, n: int = 400, h: float = 4 * math.pi / (16 * math.sqrt(3)),
                     eps: float = 0.6, phi_s: float = 0.395, phi_l: float = 0.57,
                     layers: int = 20, weight: float = 2.0, shear: float = 0.04,
                     seed: int = 6, amp: float = 1e-3):
    """(phi0, W, phi_hat) of the sheared-crystal test (Sec. 4.6).

    The crystal is phi_s + A (cos(q x) cos(q y / sqrt3) - cos(2 q y / sqrt3) / 2)
    with q = sqrt(3)/2 and A = 4 phi_s / 5 + (4/15) sqrt(15 eps - 36 phi_s^2)
    (eq. single_mode_density); its rows of atoms are 2 pi apart in y, and a
    band of `layers` rows centred in the domain holds it, the rest is liquid
    phi_l.  A seeded perturbation of size `amp` breaks the symmetry.  W =
    `weight` within pi / 2 of the bottom and top rows, else 0; phi_hat is the
    crystal there, its bottom strip shifted left by `shear` * 2 pi.
    """
    q = math.sqrt(3.0) / 2.0
    A = 0.8 * phi_s + (4.0 / 15.0) * math.sqrt(15.0 * eps - 36.0 * phi_s ** 2)
    X, Y = cell_centres(m, n, h)
    Ly = n * h
    y0 = Ly / 2 - (layers - 1) * math.pi       # bottom row of atoms
    y1 = y0 + 2 * math.pi * (layers - 1)       # top row

    def crystal(x, y):
        return phi_s + A * (np.cos(q * x) * np.cos(q * y / math.sqrt(3.0))
                            - 0.5 * np.cos(2 * q * y / math.sqrt(3.0)))

    band = np.abs(Y - 0.5 * (y0 + y1)) <= 0.5 * (y1 - y0) + math.pi
    phi = np.where(band, crystal(X, Y - y0), phi_l)
    rng = np.random.default_rng(seed)
    phi = phi + amp * rng.uniform(-1.0, 1.0, size=phi.shape)
    bottom = np.abs(Y - y0) < 0.5 * math.pi
    top = np.abs(Y - y1) < 0.5 * math.pi
    W = np.where(bottom | top, weight, 0.0)
    hat = np.where(bottom, crystal(X + shear * 2 * math.pi, Y - y0), crystal(X, Y - y0))
    hat = np.where(bottom | top, hat, phi)
    return phi, W, hat


@dataclass
class SimSpec:
    """One independent simulation of the batched workload."""
    N: int
    eps: float
    mean: float
    beta: float
    seed: int
    h: float = math.pi / 4
    dt: float = 0.05
    M: float = 1.0
    scheme: int = 2
    phi0: np.ndarray = field(default=None, repr=False)


def batch(nsim: int = 64, seed: int = 4, sizes=(128, 256, 512, 1024), amp: float = 0.05,
          make_fields: bool = True):
    """Specifications of `nsim` independent simulations: N uniform over `sizes`,
    eps ~ U[0.02, 0.3], mean phi ~ U[0.05, 0.3], beta ~ U[0.5, 2], phi0 = mean
    + U[-amp, amp] from a per-simulation seed."""
    rng = np.random.default_rng(seed)
    sims = []
    for k in range(nsim):
        N = int(rng.choice(sizes))
        eps = float(rng.uniform(0.02, 0.3))
        mean = float(rng.uniform(0.05, 0.3))
        beta = float(rng.uniform(0.5, 2.0))
        sub = int(rng.integers(0, 2**31 - 1))
        sp = SimSpec(N=N, eps=eps, mean=mean, beta=beta, seed=sub)
        if make_fields:
            sp.phi0 = noise(N, N, mean=mean, amp=amp, seed=sub)
        sims.append(sp)
    return sims


# Named workloads: (description, parameters).  Sizes are the real ones; tests
# scale them down where the oracle must finish in seconds.
WORKLOADS = {
    "scheme1_64": dict(scheme=1, N=64, h=0.5, eps=0.025, beta=0.9, M=1.0, dt=0.1, steps=10,
                       init="noise", seed=1),
    "scheme2_1024": dict(scheme=2, N=1024, h=math.pi / 4, eps=0.025, beta=0.9, M=1.0, dt=0.05,
                         steps=200, init="crystallites", seed=2),
    "scheme2_2048_mixed": dict(scheme=2, N=2048, h=math.pi / 4, eps=0.025, beta=0.9, M=1.0,
                               dt=0.05, steps=200, init="crystallites", seed=3),
}


def initial_field(name: str, N: int | None = None) -> np.ndarray:
    w = WORKLOADS[name]
    N = N or w["N"]
    if w["init"] == "noise":
        return noise(N, N, mean=0.07, amp=0.05, seed=w["seed"])
    return crystallites(N, N, w["h"], seed=w["seed"])
