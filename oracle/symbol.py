"""Fourier (von Neumann) symbol of the linearized fully discrete scheme.

TEST INFRASTRUCTURE ONLY (an oracle of the linearized step).  Independent numpy
implementation of Sec. 5 and App. D: the 16x16 amplification matrix
G_m(xi, eta; nu, W0) for m in {RB, TAI} (eq. full-symbol), built from
  * the centre row C(z_x, z_y) (eq. center-row),
  * the nodal rows of a cell and the reconstruction row R(x, y)
    (eq. nodal-row-matrix, eq. reconstruction-row),
  * the exact acoustic map A_K^sigma through the compact monomial block
    (eq. compact-monomial-block),
  * the advection map D_K^sigma = R(X_K - d^sigma) (eq. advection-map),
  * the RB point map A + D - S (eq. rb-point-map) or the TAI map
    D + (I_h Delta)(X_K - d) with Delta_K = A_K - S_K (eq. tai-increments,
    eq. tai-point-map),
  * the space-time Simpson edge rows and the average row (eq. space-time-edge,
    eq. average-row).

Readings (the paper is garbled or silent here):
  * eq. nodal-row-matrix: the entry in row m, column n is the node at
    x = n/2, y = m/2 of the cell (geometry of Sec. 2); the reconstruction row pairs
    the Lagrange weight in x with the column index and the one in y with the row.
  * q^ex of eq. pressure-response: the cell-average family is the exact cell
    average of the mode, the V, Ev, Eh families are the mode sampled at (0,0),
    (0,1/2), (1/2,0) in cell units.
  * the exact pressure gain includes the advective phase,
    g_ex = exp(-i [lambda (u0 xi + v0 eta) + s nu kappa]).
  * the "exact one-step residual" of the refinement study is ||G q - g q|| / ||q|| for
    the exact mode q, unscaled; the refinement holds K = 1 and T = 1, so h = kappa and
    N = T / dt = c0 / (nu kappa) steps.

State ordering of q: [avg(rho,u,v,p), V(rho,u,v,p), Ev(...), Eh(...)], every family
as primitive perturbations.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from scipy.special import gamma as Gamma

FAM_AVG, FAM_V, FAM_EV, FAM_EH = 0, 1, 2, 3


# ---------------------------------------------------------------------------
# App. D geometry
# ---------------------------------------------------------------------------

@lru_cache(maxsize=None)
def _mu(theta0: float, theta1: float, m: int, n: int) -> float:
    """int_{theta0}^{theta1} cos^m sin^n, by Gauss-Legendre (trig polynomial of
    degree <= 6: 24 nodes per quadrant are exact to round-off)."""
    g, w = np.polynomial.legendre.leggauss(24)
    tot = 0.0
    k0 = int(round(theta0 / (0.5 * math.pi)))
    k1 = int(round(theta1 / (0.5 * math.pi)))
    for k in range(k0, k1):
        a, b = k * 0.5 * math.pi, (k + 1) * 0.5 * math.pi
        t = 0.5 * (b - a) * g + 0.5 * (a + b)
        tot += 0.5 * (b - a) * np.sum(w * np.cos(t) ** m * np.sin(t) ** n)
    return float(tot)


def _zeta(j: int) -> float:
    return math.sqrt(math.pi) * Gamma((j + 1) / 2) / Gamma(j / 2 + 1)


@lru_cache(maxsize=None)
def block(a: int, b: int, theta0: float, theta1: float) -> np.ndarray:
    """C_ab^Theta, input/output ordered (pi, u, v)."""
    q = a + b
    chi = 1.0 if q == 0 else 1.0 + 1.0 / q
    g = q + 1 + 3 * chi
    mu = lambda m, n: _mu(theta0, theta1, m, n)
    M = mu(a, b) * _zeta(q + 1)
    X = mu(a + 2, b) * _zeta(q + 3)
    Y = mu(a + 1, b + 1) * _zeta(q + 3)
    Zz = mu(a, b + 2) * _zeta(q + 3)
    Px = (q + 2) * mu(a + 1, b) * _zeta(q + 2)
    Py = (q + 2) * mu(a, b + 1) * _zeta(q + 2)
    C = np.array([[(q + 1) * M, -Px, -Py],
                  [-Px, g * X - chi * M, g * Y],
                  [-Py, g * Y, g * Zz - chi * M]]) / (4 * math.pi)
    if q == 0:
        om = (theta1 - theta0) / (2 * math.pi)
        C = C + (2 * om / 3) * np.diag([0.0, 1.0, 1.0])
    return C


# node families for the acoustic map: position in cells from (x_i, y_j), wedges
# (angle range, owning cell offset)
HALF = 0.5 * math.pi
NODES = {
    "V": ((0.0, 0.0), [((0.0, HALF), (0, 0)), ((HALF, 2 * HALF), (-1, 0)),
                       ((2 * HALF, 3 * HALF), (-1, -1)), ((3 * HALF, 4 * HALF), (0, -1))]),
    "Ev": ((0.0, 0.5), [((-HALF, HALF), (0, 0)), ((HALF, 3 * HALF), (-1, 0))]),
    "Eh": ((0.5, 0.0), [((0.0, 2 * HALF), (0, 0)), ((2 * HALF, 4 * HALF), (0, -1))]),
    "C": ((0.5, 0.5), [((0.0, 4 * HALF), (0, 0))]),
}


def lagrange_monomials(X0):
    xs = [X0, X0 + 0.5, X0 + 1.0]
    L = np.zeros((3, 3))
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        den = (xs[a] - xs[b]) * (xs[a] - xs[c])
        L[a] = [xs[b] * xs[c] / den, -(xs[b] + xs[c]) / den, 1.0 / den]
    return L


def lag(s):
    return np.array([0.5 * s * (s - 1), 1 - s * s, 0.5 * s * (s + 1)])


class Symbol:
    """Linearized scheme about a uniform background W0 = (rho0, u0, v0, p0)."""

    def __init__(self, W0=(1.0, 0.2 * math.cos(math.radians(25)), 0.2 * math.sin(math.radians(25)), 1.0),
                 gamma=1.4):
        self.rho0, self.u0, self.v0, self.p0 = map(float, W0)
        self.gamma = gamma
        self.c0 = math.sqrt(gamma * self.p0 / self.rho0)
        self.Z0 = self.rho0 * self.c0

    # ---- scalar rows (length 4 over families avg, V, Ev, Eh) -----------------
    @staticmethod
    def e(f):
        r = np.zeros(4, complex)
        r[f] = 1.0
        return r

    def centre_row(self, zx, zy):
        return np.array([9 / 4, -(1 + zx) * (1 + zy) / 16, -(1 + zx) / 4, -(1 + zy) / 4], complex)

    def node_row(self, a, b, zx, zy):
        """Scalar row of the Q2 node at x = a/2, y = b/2 of cell C_ij."""
        e = self.e
        tab = {(0, 0): e(FAM_V), (1, 0): e(FAM_EH), (2, 0): zx * e(FAM_V),
               (0, 1): e(FAM_EV), (1, 1): self.centre_row(zx, zy), (2, 1): zx * e(FAM_EV),
               (0, 2): zy * e(FAM_V), (1, 2): zy * e(FAM_EH), (2, 2): zx * zy * e(FAM_V)}
        return tab[(a, b)]

    @staticmethod
    def expand(row, var):
        """Scalar family row -> 16-vector acting on variable var."""
        out = np.zeros(16, complex)
        out[var::4] = row
        return out

    def recon_row(self, x, y, zx, zy):
        """Scalar reconstruction row R(x, y), (x, y) in cells from (x_i, y_j)."""
        r, s = math.floor(x), math.floor(y)
        lx, ly = lag(2 * (x - r) - 1), lag(2 * (y - s) - 1)
        acc = np.zeros(4, complex)
        for a in range(3):
            for b in range(3):
                acc += lx[a] * ly[b] * self.node_row(a, b, zx, zy)
        return zx ** r * zy ** s * acc

    def select(self, K, zx, zy):
        """S_K: 4x16 selection of the time-n value at node K."""
        if K == "C":
            row = self.centre_row(zx, zy)
        else:
            row = self.e({"V": FAM_V, "Ev": FAM_EV, "Eh": FAM_EH}[K])
        return np.stack([self.expand(row, k) for k in range(4)])

    def acoustic(self, K, r, zx, zy):
        """A_K: 4x16 rows of the frozen exact acoustic update at node K, radius r."""
        (Kx, Ky), wedges = NODES[K]
        out = np.zeros((3, 16), complex)      # (pi, u, v) rows
        for (t0, t1), (ci, cj) in wedges:
            Lx = lagrange_monomials(ci - Kx)
            Ly = lagrange_monomials(cj - Ky)
            ph = zx ** ci * zy ** cj
            for al in range(3):
                for be in range(3):
                    srow = np.zeros(4, complex)
                    for a in range(3):
                        for b in range(3):
                            srow += Lx[a, al] * Ly[b, be] * self.node_row(a, b, zx, zy)
                    srow *= ph
                    data = np.stack([self.expand(srow, 3) / self.Z0, self.expand(srow, 1), self.expand(srow, 2)])
                    C = self._block(al, be, t0, t1)
                    out += r ** (al + be) * (C @ data)
        S = self.select(K, zx, zy)
        p_ac = self.Z0 * out[0]
        rho_ac = S[0] + (p_ac - S[3]) / self.c0 ** 2
        return np.stack([rho_ac, out[1], out[2], p_ac])

    @staticmethod
    def _block(a, b, t0, t1):
        if t0 < 0:     # Ev right half-plane [-pi/2, pi/2] = [3pi/2, 2pi] + [0, pi/2]
            return block(a, b, t0 + 2 * math.pi, 2 * math.pi) + block(a, b, 0.0, t1)
        return block(a, b, t0, t1)

    def increment_interp(self, Delta, x, y, zx, zy):
        """(I_h Delta)(x, y): 4x16, Delta = dict K -> 4x16 node increment rows."""
        r, s = math.floor(x), math.floor(y)
        lx, ly = lag(2 * (x - r) - 1), lag(2 * (y - s) - 1)
        tab = {(0, 0): Delta["V"], (1, 0): Delta["Eh"], (2, 0): zx * Delta["V"],
               (0, 1): Delta["Ev"], (1, 1): Delta["C"], (2, 1): zx * Delta["Ev"],
               (0, 2): zy * Delta["V"], (1, 2): zy * Delta["Eh"], (2, 2): zx * zy * Delta["V"]}
        acc = np.zeros((4, 16), complex)
        for a in range(3):
            for b in range(3):
                acc += lx[a] * ly[b] * tab[(a, b)]
        return zx ** r * zy ** s * acc

    def point_maps(self, method, sigma, nu, xi, eta):
        zx, zy = np.exp(1j * xi), np.exp(1j * eta)
        lam = nu / self.c0
        r = sigma * nu
        dx, dy = sigma * lam * self.u0, sigma * lam * self.v0
        out = {}
        if method == "TAI":
            Delta = {K: self.acoustic(K, r, zx, zy) - self.select(K, zx, zy) for K in NODES}
        for K in ("V", "Ev", "Eh"):
            (Kx, Ky), _ = NODES[K]
            D = np.stack([self.expand(self.recon_row(Kx - dx, Ky - dy, zx, zy), k) for k in range(4)])
            if method == "RB":
                out[K] = self.acoustic(K, r, zx, zy) + D - self.select(K, zx, zy)
            elif method == "TAI":
                out[K] = D + self.increment_interp(Delta, Kx - dx, Ky - dy, zx, zy)
            else:
                raise ValueError(method)
        return out

    def jac_x(self):
        r0, u0, v0, p0, g = self.rho0, self.u0, self.v0, self.p0, self.gamma
        return np.array([[u0, r0, 0, 0], [0, u0, 0, 1 / r0], [0, 0, u0, 0], [0, g * p0, 0, u0]], float)

    def jac_y(self):
        r0, u0, v0, p0, g = self.rho0, self.u0, self.v0, self.p0, self.gamma
        return np.array([[v0, 0, r0, 0], [0, v0, 0, 0], [0, 0, v0, 1 / r0], [0, 0, g * p0, v0]], float)

    def G(self, method, nu, xi, eta):
        zx, zy = np.exp(1j * xi), np.exp(1j * eta)
        lam = nu / self.c0
        Ex = np.zeros((4, 16), complex)
        Ey = np.zeros((4, 16), complex)
        half = None
        for sigma, w in ((0.0, 1 / 6), (0.5, 4 / 6), (1.0, 1 / 6)):
            P = self.point_maps(method, sigma, nu, xi, eta)
            if sigma == 1.0:
                half = P
            Ex += w * ((1 + zy) * P["V"] + 4 * P["Ev"]) / 6
            Ey += w * ((1 + zx) * P["V"] + 4 * P["Eh"]) / 6
        B = np.zeros((4, 16), complex)
        B[:, 0:4] = np.eye(4)
        Gav = B - lam * (zx - 1) * (self.jac_x() @ Ex) - lam * (zy - 1) * (self.jac_y() @ Ey)
        return np.vstack([Gav, half["V"], half["Ev"], half["Eh"]])

    # ---- exact modes --------------------------------------------------------
    @staticmethod
    def sample_families(rvec, xi, eta):
        """16-vector of the mode rvec e^{i k.x}: exact cell average, then the values at
        V (0, 0), Ev (0, 1/2) and Eh (1/2, 0) in cell units."""
        avg = _cellavg(xi) * _cellavg(eta)
        return np.concatenate([avg * rvec, rvec, np.exp(0.5j * eta) * rvec, np.exp(0.5j * xi) * rvec])

    def acoustic_mode(self, xi, eta, s=+1):
        """q^ex for the acoustic branch s (mode r_s(k) e^{i k.x})."""
        kap = math.hypot(xi, eta)
        kx, ky = xi / kap, eta / kap
        rvec = np.array([1 / self.c0 ** 2, s * kx / self.Z0, s * ky / self.Z0, 1.0], complex)
        return self.sample_families(rvec, xi, eta)

    BRANCHES = ("entropy", "shear", "acoustic+", "acoustic-")

    def exact_modes(self, xi, eta):
        """The four exact modes q_j of the linearized Euler equations about W0 (rows, in
        BRANCHES order): entropy (density only), shear (velocity normal to k), and the two
        acoustic branches (pressure with the density p/c0^2 and velocity +-k p/Z0)."""
        kap = math.hypot(xi, eta)
        kx, ky = xi / kap, eta / kap
        shear = np.array([0.0, -ky, kx, 0.0], complex)
        return np.stack([self.sample_families(np.array([1.0, 0, 0, 0], complex), xi, eta),
                         self.sample_families(shear, xi, eta),
                         self.acoustic_mode(xi, eta, +1), self.acoustic_mode(xi, eta, -1)])

    def exact_gains(self, xi, eta, nu):
        """g_j = e^{-i omega_j dt}: advection alone for entropy and shear, advection plus
        or minus the sound speed for the acoustic branches."""
        return np.array([self.exact_gain(xi, eta, nu, 0), self.exact_gain(xi, eta, nu, 0),
                         self.exact_gain(xi, eta, nu, +1), self.exact_gain(xi, eta, nu, -1)])

    def exact_gain(self, xi, eta, nu, s=+1):
        lam = nu / self.c0
        kap = math.hypot(xi, eta)
        return np.exp(-1j * (lam * (self.u0 * xi + self.v0 * eta) + s * nu * kap))

    def pressure_gain(self, method, kappa, theta, nu):
        xi, eta = kappa * math.cos(theta), kappa * math.sin(theta)
        q = self.acoustic_mode(xi, eta, +1)
        Gq = self.G(method, nu, xi, eta) @ q
        idx = 8 + 3      # Ev family, pressure
        return Gq[idx] / q[idx]


def _cellavg(k):
    return 1.0 if abs(k) < 1e-14 else (np.exp(1j * k) - 1) / (1j * k)


# ---------------------------------------------------------------------------
# Sec. 5: one-step residual, repeated-step error, modal errors
# ---------------------------------------------------------------------------

def one_step_residual(G, q, g):
    """||G q - g q|| / ||q|| for the exact mode q with exact gain g."""
    return float(np.linalg.norm(G @ q - g * q) / np.linalg.norm(q))


def repeated_step_error(G, q, g, n):
    """eq. repeated-error: ||G^n q - g^n q|| / ||q||."""
    v = q.copy()
    for _ in range(n):
        v = G @ v
    return float(np.linalg.norm(v - g ** n * q) / np.linalg.norm(q))


def match_modes(G, Q):
    """Numerical eigenvalues of G assigned one-to-one to the exact modes (rows of Q) by
    largest normalized right-eigenvector overlap |q^H v| / (|q| |v|): the largest
    overlap over unassigned pairs is taken first.  Returns (eigenvalues, overlaps,
    eigenvector indices)."""
    w, V = np.linalg.eig(G)
    O = np.abs(Q.conj() @ V)
    O /= np.linalg.norm(Q, axis=1)[:, None] * np.linalg.norm(V, axis=0)[None, :]
    rows, cols = list(range(Q.shape[0])), list(range(V.shape[1]))
    gt = np.zeros(Q.shape[0], complex)
    ov = np.zeros(Q.shape[0])
    idx = np.zeros(Q.shape[0], int)
    while rows:
        j, m = max(((j, m) for j in rows for m in cols), key=lambda jm: O[jm])
        gt[j], ov[j], idx[j] = w[m], O[j, m], m
        rows.remove(j)
        cols.remove(m)
    return gt, ov, idx


def modal_errors(sym: Symbol, method: str, nu: float, xi: float, eta: float):
    """eq. modal-amplitude-phase-errors for the four branches: (eps_A, eps_phi, overlaps)
    with eps_A = ||g~| - 1| and eps_phi = |arg(g~ / g)|."""
    gt, ov, _ = match_modes(sym.G(method, nu, xi, eta), sym.exact_modes(xi, eta))
    g = sym.exact_gains(xi, eta, nu)
    return np.abs(np.abs(gt) - 1.0), np.abs(np.angle(gt / g)), ov


def spectral_radius(sym: Symbol, method: str, nu: float, n: int = 24, kmin=None):
    """max |eig G(xi, eta)| over an n x n sample of (-pi, pi]^2 (origin excluded)."""
    ks = np.linspace(-math.pi, math.pi, n, endpoint=False) + math.pi / n
    best = 0.0
    for xi in ks:
        for eta in ks:
            ev = np.linalg.eigvals(sym.G(method, nu, xi, eta))
            best = max(best, float(np.max(np.abs(ev))))
    return best


def max_power_norm(sym: Symbol, method: str, nu: float, n: int = 24, nmax: int = 1000):
    """max over the sample and over 1 <= k <= nmax of ||G^k||_2."""
    ks = np.linspace(-math.pi, math.pi, n, endpoint=False) + math.pi / n
    best = 0.0
    for xi in ks:
        for eta in ks:
            G = sym.G(method, nu, xi, eta)
            P = np.eye(16, dtype=complex)
            for _ in range(nmax):
                P = G @ P
                best = max(best, float(np.linalg.norm(P, 2)))
    return best


class FastSymbol:
    """G(xi, eta) for one (method, nu) as a trigonometric polynomial
    sum_{a,b} G_ab e^{i(a xi + b eta)}: its coefficients are read off by a 2-D DFT of
    G at N x N roots of unity (exact when every exponent lies in (-N/2, N/2])."""

    def __init__(self, sym: Symbol, method: str, nu: float, N: int = 12):
        self.N = N
        ks = 2 * math.pi * np.arange(N) / N
        vals = np.zeros((N, N, 16, 16), complex)
        for a, xi in enumerate(ks):
            for b, eta in enumerate(ks):
                vals[a, b] = sym.G(method, nu, xi, eta)
        self.coef = np.fft.fft2(vals, axes=(0, 1)) / (N * N)   # coef[m, n] multiplies e^{i(m xi + n eta)}
        self.m = np.fft.fftfreq(N, 1.0 / N)                     # exponent of e^{i xi}

    def G(self, xi, eta):
        xi = np.atleast_1d(np.asarray(xi, float))
        eta = np.atleast_1d(np.asarray(eta, float))
        ex = np.exp(1j * np.outer(xi, self.m))                  # (B, N)
        ey = np.exp(1j * np.outer(eta, self.m))
        return np.einsum("pa,pb,abij->pij", ex, ey, self.coef, optimize=True)

    def max_exponent_mass(self, k):
        """Norm of the coefficients with |exponent| >= k (0 means N was large enough)."""
        sel = (np.abs(self.m)[:, None] >= k) | (np.abs(self.m)[None, :] >= k)
        return float(np.abs(self.coef[sel]).max())
