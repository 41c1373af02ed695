"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds only random draws and the analytic description of the obstacle
curves: a radius function r(t) given as a cosine series, the curve
z(t) = r(t) (cos t, sin t) and its first two parameter derivatives, plus the
incident-angle sets of the workloads.  It contains none of the solver's
arithmetic: no quadrature nodes or weights, no kernels, no linear algebra.  Both
the CPU oracle and the GPU path sample the curve themselves.

Workloads (the obstacle families are the paper's: a smooth star, Sec. 6.1, and a
random-Fourier "rough" obstacle, Sec. 6.2; sizes are this project's):

* ``star``     r(t) = 1 + 0.3 cos 5t, N = 800, omega = 10, d = 2 pi, theta = -pi/5.
* ``wavy20``   r(t) = 1 + sum_{k<=20} a_k cos(k t + phi_k), a_k ~ U(0, 0.3/k),
               N = 1e4, omega = 40, 100 angles theta ~ U(-pi/2, 0).
* ``wavy40``   40 harmonics, a_k ~ U(0, 0.2/k), N = 1e5, omega = 60,
               200 angles on 4 shared Bloch phases.
* ``star_d1``  the scaling test of Sec. 6.1: r(t) = 0.35 + 0.105 cos 3t, period d = 1 (the
               neighbour images come within 0.25 of the obstacle), omega = 10, theta = -pi/5;
               N = 2^17 there, smaller here by default.
* ``star_d1_tr`` the same grating as a transmission problem (Sec. 5, the second case of
               Sec. 6.1): refractive index n = 1.5 inside the obstacle, N = 2^17 nodes
               (2^18 unknowns), leaf boxes of 128 unknowns.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass
class Curve:
    """Radial curve z(t) = r(t) (cos t, sin t), r(t) = r0 + sum_k a_k cos(k t + phi_k).

    The parameterization is counter-clockwise on t in [0, 2 pi).
    """

    r0: float
    a: np.ndarray = field(default_factory=lambda: np.zeros(0))
    k: np.ndarray = field(default_factory=lambda: np.zeros(0))
    phi: np.ndarray = field(default_factory=lambda: np.zeros(0))

    def radius(self, t):
        """r(t), r'(t), r''(t) at the parameter values t (any shape)."""
        t = np.asarray(t, dtype=np.float64)
        r = np.full(t.shape, float(self.r0))
        dr = np.zeros(t.shape)
        d2r = np.zeros(t.shape)
        for ak, kk, pk in zip(self.a, self.k, self.phi):
            arg = kk * t + pk
            c, s = np.cos(arg), np.sin(arg)
            r += ak * c
            dr -= ak * kk * s
            d2r -= ak * kk * kk * c
        return r, dr, d2r

    def sample(self, t):
        """Curve point z(t), velocity z'(t) and acceleration z''(t), each shape (len(t), 2)."""
        t = np.asarray(t, dtype=np.float64)
        r, dr, d2r = self.radius(t)
        c, s = np.cos(t), np.sin(t)
        z = np.stack([r * c, r * s], axis=-1)
        dz = np.stack([dr * c - r * s, dr * s + r * c], axis=-1)
        d2z = np.stack([d2r * c - 2 * dr * s - r * c, d2r * s + 2 * dr * c - r * s], axis=-1)
        return z, dz, d2z

    def max_abs_x(self, n=65536):
        z, _, _ = self.sample(np.arange(n) * (TWO_PI / n))
        return float(np.max(np.abs(z[:, 0])))

    def max_abs_y(self, n=65536):
        z, _, _ = self.sample(np.arange(n) * (TWO_PI / n))
        return float(np.max(np.abs(z[:, 1])))


def circle(R=1.0) -> Curve:
    return Curve(r0=float(R))


def star(r0=1.0, amp=0.3, k=5) -> Curve:
    return Curve(r0=r0, a=np.array([amp]), k=np.array([float(k)]), phi=np.array([0.0]))


def wavy(seed: int, K: int, cmax: float, period: float = TWO_PI) -> Curve:
    """Seeded rough obstacle r(t) = 1 + sum_{k<=K} a_k cos(k t + phi_k).

    Draw order: a = U(0,1,K) * (cmax / k), then phi = U(0, 2 pi, K), from
    ``numpy.random.default_rng(seed)``.  A draw is rejected (seed += 1000) when
    min r < 0.2 on a 65536-point grid or when the gap to the unit-cell walls
    (period/2 - max |x|) is below 0.5.
    """
    s = int(seed)
    for _ in range(64):
        rng = np.random.default_rng(s)
        ks = np.arange(1, K + 1, dtype=np.float64)
        a = rng.uniform(0.0, 1.0, K) * (cmax / ks)
        phi = rng.uniform(0.0, TWO_PI, K)
        c = Curve(r0=1.0, a=a, k=ks, phi=phi)
        tt = np.arange(65536) * (TWO_PI / 65536)
        r, _, _ = c.radius(tt)
        if r.min() >= 0.2 and period / 2 - c.max_abs_x() >= 0.5:
            return c
        s += 1000
    raise RuntimeError("wavy: no admissible draw")


def random_angles(seed: int, n: int, omega: float, period: float, wood_min: float = 0.75):
    """n angles theta ~ U(-pi/2, 0) from rng(seed), skipping draws within ``wood_min``
    of a Wood's anomaly (min over Bragg orders of |k_n| below ``wood_min``)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        th = float(rng.uniform(-math.pi / 2, 0.0))
        kap = omega * math.cos(th)
        nmin = math.floor((-omega - kap) * period / TWO_PI) - 1
        nmax = math.ceil((omega - kap) * period / TWO_PI) + 1
        kn = [abs(omega ** 2 - (kap + TWO_PI * j / period) ** 2) ** 0.5 for j in range(nmin, nmax + 1)]
        if min(kn) >= wood_min:
            out.append(th)
    return np.array(out)


def shared_phase_angles(omega: float, period: float, n_phase: int = 4, per_phase: int = 50):
    """Angles whose cos(theta) form n_phase interleaved arithmetic series with spacing
    2 pi/(omega d), so each series shares one Bloch phase alpha_j = exp(i pi (j+1/2)/2)
    (for n_phase = 4).  Returned grouped by phase: theta[j*per_phase + m]."""
    out = []
    for j in range(n_phase):
        for m in range(per_phase):
            c = (m - per_phase // 2 + (j + 0.5) / n_phase) * TWO_PI / (omega * period)
            out.append(-math.acos(c))
    return np.array(out)


def wood_sweep_angles(omega: float, period: float, n: int = 200, groups: int = 21):
    """The angle sweep of Sec. 6.2: cos(theta) in steps of 2 pi / (groups omega d) from grazing
    (theta -> -pi), so the Bloch phases repeat with period `groups`.  When omega d / (2 pi) is an
    integer, every angle of the phase alpha = 1 sits exactly on a Wood's anomaly (some k_n = 0) and
    its neighbours come close to one."""
    c = -1.0 + np.arange(1, n + 1) * TWO_PI / (groups * omega * period)
    c = c[c < 1.0]
    return -np.arccos(c)


def rank_training_set(n: int = 64, seed: int = 4242):
    """Seeded obstacles for fitting and checking the rank predictor (64 by default).

    Per obstacle, drawn in this order from ``numpy.random.default_rng(seed)``: K ~ U{4..40}
    harmonics, roughness cmax ~ U(0.05, 0.3), N log-uniform in [2e3, 5e4] (rounded to a multiple
    of 64), omega ~ U(10, 80), tol from {1e-10, 1e-12, 1e-13}, a shape seed; the far-field circle
    is requested for every other obstacle.  Returns a list of dicts (curve, N, omega, tol, far).
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        K = int(rng.integers(4, 41))
        cmax = float(rng.uniform(0.05, 0.3))
        N = int(round(math.exp(rng.uniform(math.log(2e3), math.log(5e4))) / 64.0)) * 64
        omega = float(rng.uniform(10.0, 80.0))
        tol = float([1e-10, 1e-12, 1e-13][int(rng.integers(0, 3))])
        shape_seed = int(rng.integers(0, 2 ** 31))
        out.append({"curve": wavy(shape_seed, K, cmax), "N": N, "omega": omega, "tol": tol, "far": i % 2 == 1})
    return out


def c5_batch(n: int = 64, seed0: int = 1301500):
    """The 64-obstacle batch of the learned-rank workload.  Obstacle i, from
    ``numpy.random.default_rng(seed0 + i)`` in this order: N = integers(2000, 50001) rounded down to
    even, omega = uniform(10, 80); the shape is ``wavy(seed0 + i, 20, 0.3)`` for even i (the
    20-harmonic family) and ``wavy(seed0 + i, 40, 0.2)`` for odd i (the 40-harmonic family); 50
    angles from ``random_angles(seed0 + i + 1, 50, omega, 2 pi)``; ID tolerance 1e-12.
    Returns a list of dicts (curve, N, omega, period, thetas, tol)."""
    out = []
    for i in range(n):
        s = seed0 + i
        rng = np.random.default_rng(s)
        N = int(rng.integers(2000, 50001)) // 2 * 2
        omega = float(rng.uniform(10.0, 80.0))
        K, cmax = (20, 0.3) if i % 2 == 0 else (40, 0.2)
        out.append({"curve": wavy(s, K, cmax), "N": N, "omega": omega, "period": TWO_PI,
                    "thetas": random_angles(s + 1, 50, omega, TWO_PI), "tol": 1e-12})
    return out


@dataclass
class Workload:
    name: str
    curve: Curve
    N: int
    omega: float
    period: float
    thetas: np.ndarray
    tol: float
    leaf_size: int
    quad: str  # "kr6" or "kress"
    index: float = 0.0  # > 0: transmission problem with this refractive index inside the obstacle


def workload(name: str) -> Workload:
    if name == "star":
        return Workload("star", star(), 800, 10.0, TWO_PI, np.array([-math.pi / 5]), 1e-10, 50, "kress")
    if name == "wavy20":
        c = wavy(130102, 20, 0.3)
        th = random_angles(130102 + 1, 100, 40.0, TWO_PI)
        return Workload("wavy20", c, 10000, 40.0, TWO_PI, th, 1e-10, 64, "kr6")
    if name == "star_d1":
        return Workload("star_d1", star(0.35, 0.105, 3), 131072, 10.0, 1.0, np.array([-math.pi / 5]), 1e-10, 64,
                        "kr6")
    if name == "star_d1_tr":
        return Workload("star_d1_tr", star(0.35, 0.105, 3), 131072, 10.0, 1.0, np.array([-math.pi / 5]), 1e-10, 128,
                        "kr6", 1.5)
    if name == "wavy40":
        c = wavy(130103, 40, 0.2)
        th = shared_phase_angles(60.0, TWO_PI)
        return Workload("wavy40", c, 100000, 60.0, TWO_PI, th, 1e-10, 64, "kr6")
    raise KeyError(name)
