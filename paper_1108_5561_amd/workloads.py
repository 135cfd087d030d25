"""Seeded synthetic workloads: grid geometry and initial-condition shapes.

This module holds no arithmetic of the method: it draws random numbers and
builds dimensionless profiles; the energy scales (e.g. the energy density at
a given temperature) are supplied by the caller.  Both the GPU path and the
CPU reference consume the same arrays.

Workloads (transverse grids of boost-invariant Milne runs):
  small   32 x 32, dx 0.2 fm, Gaussian of width 2 fm, tau 0.5 -> 2.0 fm/c in 150 steps
  prec    256 x 256, dx 0.025 fm, Gaussian x (1 + 0.05 N(0,1)) white noise
          (default_rng(2), row-major), tau 0.5 -> 8 fm/c in 1000 steps
  spots   512 x 512, dx 0.03 fm, background + 40 Gaussian hot spots of width
          0.4 fm, centres uniform in a 6 fm disk, amplitudes exponential with
          mean 20 GeV/fm^3 (default_rng(3); per spot U1, U2, A), 2000 steps
  batch   64 events: side n_e uniform on {64..256} and eta/s uniform on
          [0.05, 0.3] (default_rng(4), per event n_e then eta/s), box
          15.36 fm (dx = 15.36 / n_e), hot spots as `spots` with
          default_rng(4000 + e); tau 0.5 -> 8 fm/c, dtau = 0.00375 fm/c
  adjoint 128 x 128, dx 0.12 fm, hot spots as `spots` with default_rng(5),
          eta/s 0.16, 600 steps of 0.00375 fm/c, checkpoints every 50 steps
The hot-spot workloads sit on a background floor the caller adds (the
benchmark uses eps_EoS(0.25 GeV)).
"""
from __future__ import annotations

import numpy as np

WORKLOADS = {
    "small": dict(nx=32, ny=32, dx=0.2, tau0=0.5, tau1=2.0, steps=150, eta_over_s=0.08),
    "prec": dict(nx=256, ny=256, dx=0.025, tau0=0.5, tau1=8.0, steps=1000, eta_over_s=0.08),
    "spots": dict(nx=512, ny=512, dx=0.03, tau0=0.5, tau1=8.0, steps=2000, eta_over_s=0.16),
    "batch": dict(n_events=64, n_min=64, n_max=256, box=15.36, tau0=0.5, tau1=8.0, steps=2000),
    "adjoint": dict(nx=128, ny=128, dx=0.12, tau0=0.5, steps=600, dtau=0.00375, eta_over_s=0.16,
                    checkpoint_every=50, seed=5),
}


def cell_centres(n, dx):
    """Cell-centre coordinates of a periodic box [-n dx/2, n dx/2)."""
    return (np.arange(n) - (n - 1) / 2.0) * dx


def gaussian_shape(nx, ny, dx, width):
    """exp(-r^2 / (2 width^2)) on cell centres, shape (ny, nx)."""
    x = cell_centres(nx, dx)
    y = cell_centres(ny, dx)
    X, Y = np.meshgrid(x, y)
    return np.exp(-(X ** 2 + Y ** 2) / (2 * width ** 2))


def white_noise_factor(nx, ny, amplitude=0.05, seed=2):
    """1 + amplitude * N(0, 1), row-major draws from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return 1.0 + amplitude * rng.standard_normal((ny, nx))


def hot_spots(nx, ny, dx, n_spots=40, width=0.4, disk_radius=6.0, mean_amplitude=20.0, seed=3):
    """sum_i A_i exp(-|x - c_i|^2 / (2 width^2)) in GeV/fm^3 (no background).

    Per spot, in order: U1, U2 ~ U[0, 1) and A ~ Exp(mean_amplitude);
    c_i = disk_radius sqrt(U1) (cos 2 pi U2, sin 2 pi U2).
    """
    rng = np.random.default_rng(seed)
    x = cell_centres(nx, dx)
    y = cell_centres(ny, dx)
    X, Y = np.meshgrid(x, y)
    out = np.zeros((ny, nx))
    for _ in range(n_spots):
        u1, u2 = rng.random(), rng.random()
        amp = rng.exponential(mean_amplitude)
        r = disk_radius * np.sqrt(u1)
        cx, cy = r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)
        out += amp * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * width ** 2))
    return out


def random_flow(nx, ny, amplitude, seed):
    """Small random transverse flow fields (u^x, u^y) for tests."""
    rng = np.random.default_rng(seed)
    return amplitude * rng.standard_normal((ny, nx)), amplitude * rng.standard_normal((ny, nx))


def batch_events(n_events=64, n_min=64, n_max=256, box=15.36, eta_lo=0.05, eta_hi=0.3, seed=4):
    """Per event (n, n, dx, eta/s): n uniform on {n_min..n_max}, then eta/s
    uniform on [eta_lo, eta_hi), both from default_rng(seed) in that order
    per event; dx = box / n."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_events):
        n = int(rng.integers(n_min, n_max + 1))
        eta = float(rng.uniform(eta_lo, eta_hi))
        out.append((n, n, box / n, eta))
    return out


def batch_hot_spots(events, seed0=4000):
    """Hot-spot profiles (GeV/fm^3, no background) of the events of
    batch_events, event e drawn from default_rng(seed0 + e)."""
    return [hot_spots(nx, ny, dx, seed=seed0 + e) for e, (nx, ny, dx, _) in enumerate(events)]

