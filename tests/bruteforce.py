"""Brute-force TDI synthesis in the time domain (numpy), for tiny inputs.

This is the plain definition the fast heterodyned waveform approximates: the
exact Estabrook-Wahlquist single-link response of a rigid, equal-arm,
circularly orbiting LISA, combined into first-generation Michelson X, Y, Z with
the delays evaluated analytically (no interpolation), transformed to A, E, T
(Sec. 2) and Fourier transformed with the convention
x~(f_k) = dt * sum_n x(n dt) exp(-2 pi i k n / M).

It is written independently of the oracle's C code, from the same physical
definitions, and is used only to pin the oracle.  The carrier phase is formed
in numpy long double because 2 pi f0 t reaches ~1e6 rad over a year.
"""
from __future__ import annotations

import numpy as np

C_LIGHT = 299792458.0
AU = 1.495978707e11
YEAR = 31557600.0
LPI = np.longdouble("3.14159265358979323846264338327950288")


def positions(t: np.ndarray, L: float) -> np.ndarray:
    """Spacecraft positions [3 craft][3 xyz][len(t)] of the rigid orbit."""
    e = L / (2.0 * np.sqrt(3.0) * AU)
    a = 2.0 * np.pi * t / YEAR
    out = np.empty((3, 3, t.size))
    for i in range(3):
        b = 2.0 * np.pi * i / 3.0
        out[i, 0] = AU * np.cos(a) + 0.5 * e * AU * (np.cos(2 * a - b) - 3 * np.cos(b))
        out[i, 1] = AU * np.sin(a) + 0.5 * e * AU * (np.sin(2 * a - b) - 3 * np.sin(b))
        out[i, 2] = -np.sqrt(3.0) * e * AU * np.cos(a - b)
    return out


def source(p):
    """Propagation direction and the plus/cross amplitudes on the tensor basis."""
    A, f0, fd, phi0, iota, psi, lam, beta = [float(v) for v in p]
    omega = np.array([np.cos(beta) * np.cos(lam), np.cos(beta) * np.sin(lam), np.sin(beta)])
    P = np.array([np.sin(lam), -np.cos(lam), 0.0])
    Q = np.array([-np.sin(beta) * np.cos(lam), -np.sin(beta) * np.sin(lam), np.cos(beta)])
    ep = np.outer(P, P) - np.outer(Q, Q)
    ex = np.outer(P, Q) + np.outer(Q, P)
    # h(xi) = h_plus(xi) eps_plus + h_cross(xi) eps_cross with the polarisation
    # angle rotating the basis by 2 psi
    eps_p = np.cos(2 * psi) * ep + np.sin(2 * psi) * ex
    eps_x = -np.sin(2 * psi) * ep + np.cos(2 * psi) * ex
    return -omega, eps_p, eps_x


def strain_pc(p, xi):
    """h_plus and h_cross at retarded time xi (long double phase)."""
    A, f0, fd, phi0, iota = [float(v) for v in p[:5]]
    xi = np.asarray(xi, dtype=np.longdouble)
    ph = np.longdouble(phi0) + 2 * LPI * np.longdouble(f0) * xi + LPI * np.longdouble(fd) * xi * xi
    ci = np.cos(iota)
    hp = A * (1 + ci * ci) * np.cos(ph)
    hx = -2.0 * A * ci * np.sin(ph)
    return hp.astype(np.float64), hx.astype(np.float64)


def link(p, s: int, r: int, t: np.ndarray, L: float) -> np.ndarray:
    """Fractional-frequency response y_{s->r}(t), geometry frozen at t."""
    khat, eps_p, eps_x = source(p)
    x = positions(t, L)
    xs, xr = x[s], x[r]
    n = (xr - xs) / L
    kn = khat @ n
    Fp = np.einsum("it,ij,jt->t", n, eps_p, n)
    Fx = np.einsum("it,ij,jt->t", n, eps_x, n)
    tl = np.asarray(t, dtype=np.longdouble)
    xi_r = tl - (khat @ xr / C_LIGHT).astype(np.longdouble)
    xi_s = tl - np.longdouble(L / C_LIGHT) - (khat @ xs / C_LIGHT).astype(np.longdouble)
    hp_s, hx_s = strain_pc(p, xi_s)
    hp_r, hx_r = strain_pc(p, xi_r)
    return (Fp * (hp_s - hp_r) + Fx * (hx_s - hx_r)) / (2.0 * (1.0 - kn))


def michelson_xyz(p, t: np.ndarray, L: float):
    """First-generation equal-arm Michelson X, Y, Z at times t.

    R_ab(t) = y_{b->a}(t) + y_{a->b}(t - L/c)   (round trip a -> b -> a)
    X = R_12(t) - R_13(t) - R_12(t - 2L/c) + R_13(t - 2L/c), cyclic for Y, Z.
    """
    tau = L / C_LIGHT

    def R(a, b, tt):
        return link(p, b, a, tt, L) + link(p, a, b, tt - tau, L)

    out = []
    for v, (b1, b2) in ((0, (1, 2)), (1, (2, 0)), (2, (0, 1))):
        out.append(R(v, b1, t) - R(v, b2, t) - R(v, b1, t - 2 * tau) + R(v, b2, t - 2 * tau))
    return out


def aet_spectrum(p, T: float, M: int, L: float = 2.5e9):
    """A, E, T spectra (all M bins) from the sampled time series."""
    dt = T / M
    t = np.arange(M, dtype=np.float64) * dt
    X, Y, Z = michelson_xyz(p, t, L)
    A = (Z - X) / np.sqrt(2.0)
    E = (X - 2.0 * Y + Z) / np.sqrt(6.0)
    Tc = (X + Y + Z) / np.sqrt(3.0)
    return [np.fft.fft(s) * dt for s in (A, E, Tc)]


def long_wavelength_michelson(p, t: np.ndarray, L: float, vertex: int = 0) -> np.ndarray:
    """Closed-form Michelson response at `vertex` for f L/c << 1 and fdot = 0.

    Expanding y_{s->r} to first order in the light travel time gives
    y ~ -(L/2c) n^T dh/dt n; the round trip doubles it and (1 - D^2) ~ 2(L/c) d/dt,
    so X ~ -2 (L/c)^2 d^2/dt^2 [n12^T h n12 - n13^T h n13] at spacecraft 1
    (Y, Z cyclically), and for a monochromatic source d^2/dt^2 -> -(2 pi f0)^2.
    Neglected: the yearly change of the arm directions (relative size
    f_orbit/f0) and higher orders in f L/c.
    """
    khat, eps_p, eps_x = source(p)
    x = positions(t, L)
    f0 = float(p[1])
    v = vertex
    xi = t - khat @ x[v] / C_LIGHT
    hp, hx = strain_pc(p, xi)
    out = np.zeros_like(t)
    for sgn, j in ((1.0, (v + 1) % 3), (-1.0, (v + 2) % 3)):
        n = (x[j] - x[v]) / L
        Fp = np.einsum("it,ij,jt->t", n, eps_p, n)
        Fx = np.einsum("it,ij,jt->t", n, eps_x, n)
        out += sgn * (Fp * hp + Fx * hx)
    return 2.0 * (L / C_LIGHT) ** 2 * (2 * np.pi * f0) ** 2 * out
