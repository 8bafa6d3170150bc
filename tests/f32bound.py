"""Stated accuracy of the FP32 precision form, per plane of the state.

An FP32 perturbation state holds each perturbation W' = W - W_bg to about one ulp of
its own size, and the acoustic increments carry pressure perturbations into
velocities through the impedance Z0 = rho0 c0 (and velocities into pressure), so the
attainable absolute accuracy of a plane is a few ulps of the perturbation magnitude
expressed in that plane's units:
  density planes      A = max(|rho'|, |p'| / c0^2)
  velocity planes     A = max(|u'|, |v'|, |p'| / Z0)      (momenta: rho0 times that)
  pressure planes     A = max(|p'|, Z0 |u'|, Z0 |v'|)     (energy: A / (gamma - 1))
The bound per plane after n steps is
  2e-5 range  +  16 ulps(A)  +  2 ulps(max |W|) sqrt(n).
The first term is the relative accuracy on developed flows; the second covers fields
that start at rest, whose range after a few steps is far below the pressure that
drives them; the third is the rounding of the absolute fluxes (O(M) mass flux against
an O(M^2) density perturbation in low-Mach flow), accumulated over the steps as a
random walk.
"""
import math

import numpy as np

EPS32 = float(np.finfo(np.float32).eps)


def f32_tolerance(want: np.ndarray, start: np.ndarray, bg, gamma: float, nsteps: int) -> np.ndarray:
    """Per-plane absolute tolerance for an FP32 result `want` (FP64 reference, absolute
    variables) reached from `start` (absolute FP64 state) in nsteps steps."""
    r0, u0, v0, p0 = (float(x) for x in bg)
    c0 = math.sqrt(gamma * p0 / r0)
    Z0 = r0 * c0

    def pmax(s, planes, off):
        return max(float(np.abs(s[k] - off).max()) for k in planes)

    amp = {}
    for s in (start, want):
        rho = pmax(s, (4, 8, 12), r0)
        uu = max(pmax(s, (5, 9, 13), u0), pmax(s, (6, 10, 14), v0))
        pp = pmax(s, (7, 11, 15), p0)
        amp["rho"] = max(amp.get("rho", 0.0), rho, pp / (c0 * c0))
        amp["vel"] = max(amp.get("vel", 0.0), uu, pp / Z0)
        amp["p"] = max(amp.get("p", 0.0), pp, Z0 * uu)
    A = np.empty(16)
    A[0] = amp["rho"]
    A[1] = A[2] = r0 * amp["vel"] + amp["rho"] * max(abs(u0), abs(v0))
    A[3] = amp["p"] / (gamma - 1.0) + r0 * (abs(u0) + abs(v0)) * amp["vel"]
    for f in (4, 8, 12):
        A[f], A[f + 1], A[f + 2], A[f + 3] = amp["rho"], amp["vel"], amp["vel"], amp["p"]
    rng = want.max(axis=(1, 2)) - want.min(axis=(1, 2))
    wmax = np.abs(want).max(axis=(1, 2))
    return 2e-5 * rng + 16 * EPS32 * A + 2 * EPS32 * wmax * math.sqrt(nsteps)
