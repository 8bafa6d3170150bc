"""Fourier analysis of the implemented step (Sec. 5), measured on the GPU.

About a uniform state W0 the step is, to first order, a 16x16 amplification matrix
G(xi, eta) acting on a Fourier mode's amplitudes over the four families (cell average,
V, Ev, Eh; every family as primitive perturbations).  `SymbolMeter.measure` obtains it
from the library's FP64 step itself: for each of the 16 amplitudes, one periodic mode
e^{i(xi i + eta j)} on an nx x ny grid with xi = 2 pi mx / nx, eta = 2 pi my / ny, four
steps (real and imaginary part, +-eps) and central differences; the response of every
cell is projected back onto the mode.  The averages are stored conservatively, so the
perturbation enters through dU/dW at W0 and the response leaves through its inverse.

On G, the accuracy measures of Sec. 5:
  * the exact modes q_j (entropy, shear, acoustic +, acoustic -) sampled on the four
    families (exact cell average; V, Ev, Eh at (0, 0), (0, 1/2), (1/2, 0) cells) and
    their exact one-step gains g_j = e^{-i omega_j dt};
  * the one-step residual ||G q - g q|| / ||q|| and the repeated-step error
    ||G^n q - g^n q|| / ||q|| (eq. repeated-error), which the refinement study holds at
    fixed K and T as kappa = K h -> 0;
  * the directional modal amplitude and phase errors (eq. modal-amplitude-phase-errors)
    of the numerical eigenvalues matched one-to-one to the q_j by largest normalized
    right-eigenvector overlap;
  * the one-step pressure gain of the acoustic mode at the Ev nodes and its error
    (Sec. 5.3).

Only the step runs on the GPU; the differences, projections and eigen-decompositions are
host post-processing of its outputs (numpy).
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

BRANCHES = ("entropy", "shear", "acoustic+", "acoustic-")

# Sec. 5 background: rho0 = p0 = 1, |u0| = 0.2 at 25 degrees
PAPER_BACKGROUND = (1.0, 0.2 * math.cos(math.radians(25.0)), 0.2 * math.sin(math.radians(25.0)), 1.0)


def sound_speed(W0: Sequence[float], gamma: float) -> float:
    return math.sqrt(gamma * W0[3] / W0[0])


def dU_dW(W0: Sequence[float], gamma: float) -> np.ndarray:
    """Jacobian of (rho, rho u, rho v, E) with respect to (rho, u, v, p) at W0."""
    r, u, v, _ = W0
    return np.array([[1.0, 0.0, 0.0, 0.0],
                     [u, r, 0.0, 0.0],
                     [v, 0.0, r, 0.0],
                     [0.5 * (u * u + v * v), r * u, r * v, 1.0 / (gamma - 1.0)]])


def uniform_state(W0: Sequence[float], gamma: float, nx: int, ny: int) -> np.ndarray:
    r, u, v, p = W0
    U = (r, r * u, r * v, p / (gamma - 1.0) + 0.5 * r * (u * u + v * v))
    s = np.empty((16, ny, nx))
    for k in range(4):
        s[k] = U[k]
        s[4 + k] = s[8 + k] = s[12 + k] = W0[k]
    return s


def lattice_wavevector(nx: int, ny: int, mx: int, my: int) -> Tuple[float, float]:
    return 2.0 * math.pi * mx / nx, 2.0 * math.pi * my / ny


class SymbolMeter:
    """Measures G(xi, eta) of the FP64 GPU step on an nx x ny periodic grid."""

    def __init__(self, nx: int, ny: int, scheme: str = "tai", W0: Sequence[float] = PAPER_BACKGROUND,
                 gamma: float = 1.4, eps: float = 1e-6, device=None):
        import torch

        from .stepper import Stepper
        self.torch = torch
        self.nx, self.ny, self.W0, self.gamma, self.eps = nx, ny, tuple(map(float, W0)), gamma, eps
        self.h = 1.0 / max(nx, ny)
        self.c0 = sound_speed(self.W0, gamma)
        self.st = Stepper(nx, ny, self.h, gamma, scheme=scheme, device=device)
        self.device = self.st.device
        self.M = dU_dW(self.W0, gamma)
        self.Minv = np.linalg.inv(self.M)
        self.s0 = uniform_state(self.W0, gamma, nx, ny)
        self._x = torch.empty((16, ny, nx), dtype=torch.float64, device=self.device)
        self._y = torch.empty_like(self._x)

    def _run(self, planes: np.ndarray, dt: float) -> np.ndarray:
        self._x.copy_(self.torch.from_numpy(planes))
        self.st.step_out(self._x, dt, self._y)
        return self._y.cpu().numpy()

    def measure(self, mx: int, my: int, nu: float) -> np.ndarray:
        """G at xi = 2 pi mx / nx, eta = 2 pi my / ny for nu = c0 dt / h."""
        xi, eta = lattice_wavevector(self.nx, self.ny, mx, my)
        dt = nu * self.h / self.c0
        i = np.arange(self.nx)
        j = np.arange(self.ny)
        ph = np.exp(1j * (xi * i[None, :] + eta * j[:, None]))       # [j][i]
        G = np.zeros((16, 16), complex)
        for col in range(16):
            f, v = divmod(col, 4)
            z = np.zeros((16, self.ny, self.nx), complex)
            if f == 0:
                for k in range(4):
                    z[k] = self.M[k, v] * ph
            else:
                z[col] = ph
            resp = []
            for part in (z.real, z.imag):
                up = self._run(self.s0 + self.eps * part, dt)
                dn = self._run(self.s0 - self.eps * part, dt)
                resp.append((up - dn) / (2.0 * self.eps))
            R = resp[0] + 1j * resp[1]
            R[0:4] = np.einsum("kl,lji->kji", self.Minv, R[0:4])
            G[:, col] = (R * np.conj(ph)[None]).mean(axis=(1, 2))
        return G


def exact_modes(xi: float, eta: float, W0: Sequence[float] = PAPER_BACKGROUND, gamma: float = 1.4) -> np.ndarray:
    """Rows: the four exact modes of the linearized Euler equations about W0, each as a
    16-vector over the families."""
    rho0, _, _, p0 = W0
    c0 = sound_speed(W0, gamma)
    Z0 = rho0 * c0
    kap = math.hypot(xi, eta)
    kx, ky = xi / kap, eta / kap
    amps = [np.array([1.0, 0.0, 0.0, 0.0]),                 # entropy: density alone
            np.array([0.0, -ky, kx, 0.0]),                  # shear: velocity normal to k
            np.array([1.0 / c0 ** 2, kx / Z0, ky / Z0, 1.0]),   # acoustic, along k
            np.array([1.0 / c0 ** 2, -kx / Z0, -ky / Z0, 1.0])]

    def cell_average(k):
        return 1.0 if abs(k) < 1e-14 else (np.exp(1j * k) - 1.0) / (1j * k)

    av = cell_average(xi) * cell_average(eta)
    rows = []
    for a in amps:
        a = a.astype(complex)
        rows.append(np.concatenate([av * a, a, np.exp(0.5j * eta) * a, np.exp(0.5j * xi) * a]))
    return np.array(rows)


def exact_gains(xi: float, eta: float, nu: float, W0: Sequence[float] = PAPER_BACKGROUND,
                gamma: float = 1.4) -> np.ndarray:
    """e^{-i omega_j dt} of the four modes; with lambda = dt / h = nu / c0 the advective
    phase is lambda (u0 xi + v0 eta) and the acoustic one nu |(xi, eta)|."""
    c0 = sound_speed(W0, gamma)
    adv = (nu / c0) * (W0[1] * xi + W0[2] * eta)
    ac = nu * math.hypot(xi, eta)
    return np.exp(-1j * np.array([adv, adv, adv + ac, adv - ac]))


def one_step_residuals(G: np.ndarray, Q: np.ndarray, g: np.ndarray) -> np.ndarray:
    return np.array([np.linalg.norm(G @ q - gj * q) / np.linalg.norm(q) for q, gj in zip(Q, g)])


def repeated_step_errors(G: np.ndarray, Q: np.ndarray, g: np.ndarray, n: int) -> np.ndarray:
    Gn = np.linalg.matrix_power(G, n)
    return np.array([np.linalg.norm(Gn @ q - gj ** n * q) / np.linalg.norm(q) for q, gj in zip(Q, g)])


def match_eigenvalues(G: np.ndarray, Q: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Eigenvalues of G assigned one-to-one to the rows of Q, pairs taken in order of
    decreasing normalized overlap |q^H v| / (|q| |v|).  Returns (eigenvalues, overlaps)."""
    w, V = np.linalg.eig(G)
    Vn = V / np.linalg.norm(V, axis=0, keepdims=True)
    Qn = Q / np.linalg.norm(Q, axis=1, keepdims=True)
    O = np.abs(Qn.conj() @ Vn)
    order = np.dstack(np.unravel_index(np.argsort(-O, axis=None), O.shape))[0]
    taken_j, taken_m = set(), set()
    lam = np.zeros(Q.shape[0], complex)
    ov = np.zeros(Q.shape[0])
    for j, m in order:
        if j in taken_j or m in taken_m:
            continue
        lam[j], ov[j] = w[m], O[j, m]
        taken_j.add(j)
        taken_m.add(m)
        if len(taken_j) == Q.shape[0]:
            break
    return lam, ov


def modal_errors(G: np.ndarray, Q: np.ndarray, g: np.ndarray) -> Dict[str, np.ndarray]:
    """eps_A = ||g~| - 1|, eps_phi = |arg(g~ / g)| per branch, and the overlaps."""
    lam, ov = match_eigenvalues(G, Q)
    return {"amplitude": np.abs(np.abs(lam) - 1.0), "phase": np.abs(np.angle(lam / g)), "overlap": ov,
            "eigenvalue": lam}


def pressure_gain(G: np.ndarray, xi: float, eta: float, nu: float, W0: Sequence[float] = PAPER_BACKGROUND,
                  gamma: float = 1.4) -> Tuple[complex, float]:
    """Sec. 5.3: one-step gain of the Ev-node pressure for the exact acoustic mode
    (branch +), and its distance from the exact gain."""
    q = exact_modes(xi, eta, W0, gamma)[2]
    k = 8 + 3                                       # Ev family, pressure
    g = complex((G @ q)[k] / q[k])
    return g, abs(g - exact_gains(xi, eta, nu, W0, gamma)[2])


def polar_grid(kappa: float, theta: float, nmax: int = 512) -> Tuple[int, int, int, int]:
    """A periodic grid and lattice mode close to the wave vector kappa (cos, sin)(theta):
    one period per grid length along each axis with a component, n = round(2 pi / |k|)
    (at least 4 and at most nmax; beyond nmax that component is taken as zero)."""
    out = []
    for comp in (kappa * math.cos(theta), kappa * math.sin(theta)):
        n = int(round(2.0 * math.pi / abs(comp))) if abs(comp) > 1e-12 else nmax + 1
        if n > nmax:
            out += [8, 0]
        else:
            out += [max(n, 4), 1 if comp > 0 else -1]
    nx, mx, ny, my = out
    return nx, ny, mx, my


def polar_modal_errors(kappa: float, nu: float, ndir: int, scheme: str = "tai",
                       W0: Sequence[float] = PAPER_BACKGROUND, gamma: float = 1.4,
                       device=None) -> List[dict]:
    """Directional modal errors of the GPU step near |(xi, eta)| = kappa over ndir
    directions; each entry holds the lattice wave vector actually used."""
    rows = []
    meters: Dict[Tuple[int, int], SymbolMeter] = {}
    for d in range(ndir):
        th = 2.0 * math.pi * d / ndir
        nx, ny, mx, my = polar_grid(kappa, th)
        if (nx, ny) not in meters:
            meters[(nx, ny)] = SymbolMeter(nx, ny, scheme, W0, gamma, device=device)
        G = meters[(nx, ny)].measure(mx, my, nu)
        xi, eta = lattice_wavevector(nx, ny, mx, my)
        e = modal_errors(G, exact_modes(xi, eta, W0, gamma), exact_gains(xi, eta, nu, W0, gamma))
        rows.append({"theta": math.atan2(eta, xi), "kappa": math.hypot(xi, eta), "xi": xi, "eta": eta,
                     "nx": nx, "ny": ny, "G": G, **e})
    return rows


def refinement_errors(n: int, mx: int, my: int, nu: float, scheme: str = "tai", T: float = 1.0,
                      W0: Sequence[float] = PAPER_BACKGROUND, gamma: float = 1.4,
                      device=None) -> dict:
    """One level of the refinement study on an n x n grid with the lattice mode (mx, my):
    K = 1, so h = kappa; N = round(c0 T / (nu kappa)) steps, with nu adjusted so that
    N dt = T exactly.  Returns the one-step residuals and repeated-step errors."""
    xi, eta = lattice_wavevector(n, n, mx, my)
    kap = math.hypot(xi, eta)
    c0 = sound_speed(W0, gamma)
    N = max(1, int(round(c0 * T / (nu * kap))))
    nu_eff = c0 * T / (kap * N)
    G = SymbolMeter(n, n, scheme, W0, gamma, device=device).measure(mx, my, nu_eff)
    Q, g = exact_modes(xi, eta, W0, gamma), exact_gains(xi, eta, nu_eff, W0, gamma)
    return {"kappa": kap, "steps": N, "nu": nu_eff, "G": G, "one_step": one_step_residuals(G, Q, g),
            "repeated": repeated_step_errors(G, Q, g, N)}
