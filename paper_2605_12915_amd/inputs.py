"""Seeded, synthetic initial data for the Active Flux step (host, FP64).

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
only the *problem statement*: analytic initial conditions, the ideal-gas map
from primitive to conservative variables (Sec. 2, closure for E), Gauss-Legendre
cell averages and direct point sampling (Sec. 6, opening paragraph: averages by
quadrature, point values sampled from the primitive data).  None of the scheme's
arithmetic (centre recovery, acoustic operator, feet, fluxes) lives here.

State layout (shared with the C ABI): an array of shape (16, ny, nx), float64,
x index fastest.  Planes 0..3 are the conservative cell averages
(rho, rho*u, rho*v, E) of cell C_ij = [x_i, x_{i+1}] x [y_j, y_{j+1}];
planes 4..7 the primitive (rho, u, v, p) at the vertex (x_i, y_j); planes 8..11
at the vertical-edge midpoint (x_i, y_{j+1/2}); planes 12..15 at the
horizontal-edge midpoint (x_{i+1/2}, y_j)  (Sec. 2, list of degrees of freedom).
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Callable, Tuple

import numpy as np

AVG, V, EV, EH = 0, 4, 8, 12
NPLANES = 16

PrimFn = Callable[[np.ndarray, np.ndarray], Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]]


@dataclasses.dataclass
class Problem:
    """A periodic problem on [x0, x0 + nx*h] x [y0, y0 + ny*h]."""
    name: str
    nx: int
    ny: int
    x0: float
    y0: float
    h: float
    gamma: float
    prim: PrimFn            # tensor-grid evaluator: prim(xv, yv) -> 4 arrays (len(yv), len(xv))
    bg: Tuple[float, float, float, float] = (1.0, 0.0, 0.0, 1.0)   # (rho, u, v, p) background

    def state(self, ngl: int = 5) -> np.ndarray:
        return make_state(self.prim, self.nx, self.ny, self.x0, self.y0, self.h, self.gamma, ngl)

    def max_signal_speed(self) -> float:
        return max_signal_speed(self.prim, self.nx, self.ny, self.x0, self.y0, self.h, self.gamma)

    def dt_for_cfl(self, cfl: float) -> float:
        """dt from the paper's CFL definition (dt/dx) * max(|u| + c) (Sec. 6, opening
        paragraph), the maximum taken over the sampled initial data at the vertex,
        edge-midpoint and cell-centre locations."""
        return cfl * self.h / self.max_signal_speed()


def cons_from_prim(rho, u, v, p, gamma):
    """Ideal-gas closure of Sec. 2: U = (rho, rho u, rho v, E), E = p/(g-1) + rho|u|^2/2."""
    return rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)


def _gl(n: int):
    g, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (g + 1.0), 0.5 * w          # nodes in [0,1], weights sum to 1


def _workers() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(16, os.cpu_count() or 1))


def make_state(prim: PrimFn, nx: int, ny: int, x0: float, y0: float, h: float,
               gamma: float, ngl: int = 5, chunk_rows: int = 64) -> np.ndarray:
    """Cell averages by ngl x ngl Gauss-Legendre quadrature of U(W(x,y)); point
    values sampled from W(x,y).  Row chunks are independent and evaluated by a
    thread pool (numpy releases the GIL); the result does not depend on it."""
    s = np.empty((NPLANES, ny, nx), dtype=np.float64)
    gx, gw = _gl(ngl)
    xi = x0 + h * np.arange(nx, dtype=np.float64)
    yj = y0 + h * np.arange(ny, dtype=np.float64)
    xq = (xi[:, None] + h * gx[None, :]).reshape(-1)

    def averages(j0):
        j1 = min(ny, j0 + chunk_rows)
        yq = (yj[j0:j1, None] + h * gx[None, :]).reshape(-1)
        W = prim(xq, yq)
        U = cons_from_prim(*W, gamma)
        for k in range(4):
            a = U[k].reshape(j1 - j0, ngl, nx, ngl)
            s[AVG + k, j0:j1] = np.einsum("ajbk,j,k->ab", a, gw, gw, optimize=True)

    def points(j0):
        j1 = min(ny, j0 + chunk_rows)
        for base, dx, dy in ((V, 0.0, 0.0), (EV, 0.0, 0.5), (EH, 0.5, 0.0)):
            W = prim(xi + dx * h, yj[j0:j1] + dy * h)
            for k in range(4):
                s[base + k, j0:j1] = W[k]

    starts = list(range(0, ny, chunk_rows))
    nw = _workers()
    if nw > 1 and len(starts) > 1:
        with ThreadPoolExecutor(max_workers=nw) as ex:
            list(ex.map(averages, starts))
            list(ex.map(points, starts))
    else:
        for j0 in starts:
            averages(j0)
            points(j0)
    return s


def max_signal_speed(prim: PrimFn, nx, ny, x0, y0, h, gamma, chunk_rows: int = 512) -> float:
    xi = x0 + h * np.arange(nx, dtype=np.float64)
    yj = y0 + h * np.arange(ny, dtype=np.float64)
    m = 0.0
    for dx, dy in ((0.0, 0.0), (0.0, 0.5), (0.5, 0.0), (0.5, 0.5)):
        for j0 in range(0, ny, chunk_rows):
            j1 = min(ny, j0 + chunk_rows)
            rho, u, v, p = prim(xi + dx * h, yj[j0:j1] + dy * h)
            m = max(m, float(np.max(np.sqrt(u * u + v * v) + np.sqrt(gamma * p / rho))))
    return m


# ----------------------------------------------------------------------------------
# Analytic initial conditions
# ----------------------------------------------------------------------------------

def isentropic_vortex(n: int, L: float = 10.0, center=(5.0, 5.0), uinf=(1.0, 1.0),
                      beta: float = 5.0, gamma: float = 1.4, y0: float = 0.0,
                      ny: int | None = None) -> Problem:
    """Isentropic vortex of Sec. 6.2 (rho_inf = p_inf = 1), on the periodic square
    [0, L] x [y0, y0 + L].  The perturbation is evaluated from the single unwrapped
    centre, so a tiny periodic seam remains (about beta/(2 pi) e^{-12} * 5)."""
    xc, yc = center
    ny = n if ny is None else ny
    h = L / n

    def prim(xv, yv):
        X, Y = np.meshgrid(xv, yv)
        dx, dy = X - xc, Y - yc
        r2 = dx * dx + dy * dy
        e = np.exp(0.5 * (1.0 - r2))
        du = -beta / (2.0 * math.pi) * e * dy
        dv = beta / (2.0 * math.pi) * e * dx
        T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi ** 2) * e * e
        rho = T ** (1.0 / (gamma - 1.0))
        return rho, uinf[0] + du, uinf[1] + dv, rho ** gamma

    return Problem("isentropic_vortex", n, ny, 0.0, y0, h, gamma, prim,
                   bg=(1.0, uinf[0], uinf[1], 1.0))


def fourier_modes(n: int, seed: int = 2, nmodes: int = 16, kmax: int = 8, amp: float = 1e-3,
                  rho0: float = 1.0, p0: float = 1.0 / 1.4, vel=(0.5, 0.3),
                  gamma: float = 1.4) -> Problem:
    """Uniform background plus `nmodes` seeded random Fourier modes per primitive field,
    integer wavenumbers in [-kmax, kmax]^2 minus the origin, uniform phases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    modes = []
    for _f in range(4):
        ks = []
        while len(ks) < nmodes:
            kx, ky = rng.integers(-kmax, kmax + 1, size=2)
            if kx == 0 and ky == 0:
                continue
            ks.append((int(kx), int(ky)))
        ph = rng.uniform(0.0, 2.0 * math.pi, size=nmodes)
        modes.append((np.array(ks, dtype=np.float64), ph))
    base = (rho0, vel[0], vel[1], p0)

    def prim(xv, yv):
        out = []
        for f in range(4):
            ks, ph = modes[f]
            ex = np.exp(2j * math.pi * np.outer(ks[:, 0], xv))            # (M, nx)
            ey = np.exp(2j * math.pi * np.outer(yv, ks[:, 1])) * np.exp(1j * ph)[None, :]
            out.append(base[f] + amp * (ey @ ex).real)
        return tuple(out)

    return Problem("fourier_modes", n, n, 0.0, 0.0, 1.0 / n, gamma, prim, bg=base)


def gaussian_pulse(n: int, L: float = 1.0, amp: float = 0.1, width: float = 0.05,
                   center=None, gamma: float = 1.4, rho0: float = 1.0,
                   vel=(0.0, 0.0), x0: float = 0.0) -> Problem:
    """Isentropic Gaussian density pulse at rest, p = p0 (rho/rho0)^gamma with
    p0 = 1/gamma (the form of Sec. 6.3: rho = 1 + A exp(-alpha r^2), p = rho^gamma/gamma)."""
    c = (x0 + 0.5 * L, x0 + 0.5 * L) if center is None else center

    def prim(xv, yv):
        X, Y = np.meshgrid(xv, yv)
        r2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2
        rho = rho0 * (1.0 + amp * np.exp(-r2 / (width * width)))
        p = (rho / rho0) ** gamma / gamma
        return rho, np.full_like(rho, vel[0]), np.full_like(rho, vel[1]), p

    return Problem("gaussian_pulse", n, n, x0, x0, L / n, gamma, prim,
                   bg=(rho0, vel[0], vel[1], 1.0 / gamma))


def paper_pulse(n: int, L: float = 8.0, A: float = 0.25, alpha: float = 20.0,
                gamma: float = 1.4) -> Problem:
    """Sec. 6.3: [-4,4]^2, rho = 1 + A exp(-alpha r^2), u = v = 0, p = rho^gamma / gamma."""
    def prim(xv, yv):
        X, Y = np.meshgrid(xv, yv)
        rho = 1.0 + A * np.exp(-alpha * (X * X + Y * Y))
        return rho, np.zeros_like(rho), np.zeros_like(rho), rho ** gamma / gamma

    return Problem("paper_pulse", n, n, -0.5 * L, -0.5 * L, L / n, gamma, prim,
                   bg=(1.0, 0.0, 0.0, 1.0 / gamma))


def acoustic_pulse_adjoint(n: int, seed: int = 4, amp: float = 0.05, width: float = 0.05,
                           gamma: float = 1.4) -> Problem:
    """Gaussian acoustic pulse on [0,1]^2 at rest with a seeded centre jitter of up
    to one cell: rho = 1 + amp g, p = 1/gamma + amp g, g = exp(-(|x - xc|/width)^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / n
    xc = 0.5 + rng.uniform(-h, h)
    yc = 0.5 + rng.uniform(-h, h)

    def prim(xv, yv):
        X, Y = np.meshgrid(xv, yv)
        g = np.exp(-((X - xc) ** 2 + (Y - yc) ** 2) / (width * width))
        rho = 1.0 + amp * g
        return rho, np.zeros_like(rho), np.zeros_like(rho), 1.0 / gamma + amp * g

    return Problem("acoustic_pulse", n, n, 0.0, 0.0, h, gamma, prim,
                   bg=(1.0, 0.0, 0.0, 1.0 / gamma))


def double_shear_layer(n: int, U0: float = 1.0, mach: float = 0.1, width: float = 1.0 / 30.0,
                       pert: float = 0.05, gamma: float = 1.4) -> Problem:
    """Low-Mach double shear layer on the periodic unit square: u = U0 tanh((y-1/4)/w)
    for y <= 1/2 and U0 tanh((3/4-y)/w) above, v = pert U0 sin(2 pi x), rho = 1,
    p = 1/(gamma M^2)."""
    p0 = 1.0 / (gamma * mach * mach)

    def prim(xv, yv):
        X, Y = np.meshgrid(xv, yv)
        Yw = np.mod(Y, 1.0)
        u = np.where(Yw <= 0.5, U0 * np.tanh((Yw - 0.25) / width), U0 * np.tanh((0.75 - Yw) / width))
        v = pert * U0 * np.sin(2.0 * math.pi * X)
        rho = np.ones_like(u)
        return rho, u, v, np.full_like(u, p0)

    return Problem("double_shear_layer", n, n, 0.0, 0.0, 1.0 / n, gamma, prim,
                   bg=(1.0, 0.0, 0.0, p0))


def uniform(n: int, W=(1.0, 0.3, -0.2, 0.8), gamma: float = 1.4, ny: int | None = None) -> Problem:
    ny = n if ny is None else ny

    def prim(xv, yv):
        shp = (len(yv), len(xv))
        return tuple(np.full(shp, float(w)) for w in W)

    return Problem("uniform", n, ny, 0.0, 0.0, 1.0 / n, gamma, prim, bg=tuple(W))


def random_smooth(nx: int, ny: int | None = None, seed: int = 0, amp: float = 0.05,
                  vel=(0.3, -0.2), gamma: float = 1.4, kmax: int = 3) -> Problem:
    """Smooth random periodic data (a few low Fourier modes per field) around a
    moving background; used for parity cases on small non-square grids."""
    ny = nx if ny is None else ny
    rng = np.random.Generator(np.random.PCG64(seed))
    nm = 6
    coef = []
    for _f in range(4):
        kx = rng.integers(-kmax, kmax + 1, size=nm)
        ky = rng.integers(-kmax, kmax + 1, size=nm)
        ph = rng.uniform(0, 2 * math.pi, size=nm)
        a = rng.uniform(0.3, 1.0, size=nm)
        coef.append((kx, ky, ph, a))
    base = (1.0, vel[0], vel[1], 1.0)

    def prim(xv, yv):
        X, Y = np.meshgrid(xv, yv)
        out = []
        for f in range(4):
            kx, ky, ph, a = coef[f]
            acc = np.zeros_like(X)
            for m in range(nm):
                acc += a[m] * np.cos(2 * math.pi * (kx[m] * X + ky[m] * Y) + ph[m])
            out.append(base[f] + amp * acc / nm)
        return tuple(out)

    return Problem("random_smooth", nx, ny, 0.0, 0.0, 1.0 / nx, gamma, prim, bg=base)


def mixed_packet(n: int, eps: float = 1e-6, M: float = 0.2, phi_deg: float = 25.0,
                 gamma: float = 1.4):
    """Linearized mixed wave packet of Sec. 4.2 on the periodic unit square: entropy
    k1 = 2pi(1,2), shear k2 = 2pi(2,1), acoustic+ k3 = 2pi(3,2), acoustic- k4 = 2pi(2,3),
    all amplitudes eps, background rho0 = p0 = 1, |u0| = M at angle phi.
    Returns (problem, exact(t) -> prim tensor-grid evaluator)."""
    rho0, p0 = 1.0, 1.0
    c0 = math.sqrt(gamma * p0 / rho0)
    u0 = M * math.cos(math.radians(phi_deg))
    v0 = M * math.sin(math.radians(phi_deg))
    k1 = 2 * math.pi * np.array([1.0, 2.0])
    k2 = 2 * math.pi * np.array([2.0, 1.0])
    k3 = 2 * math.pi * np.array([3.0, 2.0])
    k4 = 2 * math.pi * np.array([2.0, 3.0])

    def at(t):
        def prim(xv, yv):
            X, Y = np.meshgrid(xv, yv)
            rho = np.full_like(X, rho0)
            u = np.full_like(X, u0)
            v = np.full_like(X, v0)
            p = np.full_like(X, p0)
            om = lambda k: u0 * k[0] + v0 * k[1]
            # entropy
            ph = k1[0] * X + k1[1] * Y - om(k1) * t
            rho = rho + eps * np.cos(ph)
            # shear
            K = np.hypot(*k2)
            ph = k2[0] * X + k2[1] * Y - om(k2) * t
            u = u - eps * (k2[1] / K) * np.cos(ph)
            v = v + eps * (k2[0] / K) * np.cos(ph)
            for k, s in ((k3, 1.0), (k4, -1.0)):
                K = np.hypot(*k)
                ph = k[0] * X + k[1] * Y - (om(k) + s * c0 * K) * t
                cc = np.cos(ph)
                p = p + eps * cc
                rho = rho + eps / c0 ** 2 * cc
                u = u + s * eps / (rho0 * c0) * (k[0] / K) * cc
                v = v + s * eps / (rho0 * c0) * (k[1] / K) * cc
            return rho, u, v, p
        return prim

    prob = Problem("mixed_packet", n, n, 0.0, 0.0, 1.0 / n, gamma, at(0.0),
                   bg=(rho0, u0, v0, p0))
    return prob, at


def low_mach_shear(nx: int = 64, ny: int | None = None, R: float = 1e-3, M: float = 1e-2, delta: float = 0.1,
                   gamma: float = 1.4) -> Problem:
    """Sec. 6, low Mach number shear: [0, 2] x [-0.5, 0.5], rho = gamma + R (1 - 2a(y)),
    u = M (1 - 2a(y)), v = delta M sin(2 pi x), p = 1, with the smoothed indicator a(y)
    of the band |y| < 1/4 (sine ramps of width 1/16)."""
    ny = nx // 2 if ny is None else ny

    def a_of(y):
        a = np.zeros_like(y)
        a = np.where((y >= -9 / 32) & (y < -7 / 32), 0.5 * (1.0 + np.sin(16 * math.pi * (y + 0.25))), a)
        a = np.where((y >= -7 / 32) & (y < 7 / 32), 1.0, a)
        a = np.where((y >= 7 / 32) & (y < 9 / 32), 0.5 * (1.0 - np.sin(16 * math.pi * (y - 0.25))), a)
        return a

    def prim(xv, yv):
        X, Y = np.meshgrid(xv, yv)
        a = a_of(Y)
        return gamma + R * (1.0 - 2.0 * a), M * (1.0 - 2.0 * a), delta * M * np.sin(2 * math.pi * X), np.ones_like(X)

    assert 2 * ny == nx, "the domain is 2 x 1 with square cells"
    return Problem("low_mach_shear", nx, ny, 0.0, -0.5, 2.0 / nx, gamma, prim, bg=(gamma, 0.0, 0.0, 1.0))


def kelvin_helmholtz(n: int = 64, gamma: float = 1.4) -> Problem:
    """Sec. 6, robustness test: [-1, 1]^2, B(y) = tanh(15y + 7.5) - tanh(15y - 7.5),
    rho = 1/2 + 3/4 B, u = (B - 1)/2, v = sin(2 pi x)/10, p = 1."""
    def prim(xv, yv):
        X, Y = np.meshgrid(xv, yv)
        B = np.tanh(15 * Y + 7.5) - np.tanh(15 * Y - 7.5)
        return 0.5 + 0.75 * B, 0.5 * (B - 1.0), 0.1 * np.sin(2 * math.pi * X), np.ones_like(X)

    return Problem("kelvin_helmholtz", n, n, -1.0, -1.0, 2.0 / n, gamma, prim, bg=(1.0, 0.0, 0.0, 1.0))


def batch_sizes(count: int = 64, lo: int = 32, hi: int = 1024, seed: int = 5):
    """Log-uniform instance sizes N_k = round(exp U[ln lo, ln hi])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [int(round(math.exp(x))) for x in rng.uniform(math.log(lo), math.log(hi), size=count)]
