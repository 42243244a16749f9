"""Seeded synthetic inputs for the HPS workloads.

This module only evaluates the problem data -- coefficient fields, manufactured
solutions and loads -- at points the caller supplies.  It holds none of the
solver's arithmetic (no grids, no differentiation matrices, no tree); the
library and the oracle each compute their own node coordinates and pass them
here.  Loads g = A u of manufactured solutions use the analytic derivatives of
u and the operator A of the problem statement (paper, eq. defA).

All random draws use ``numpy.random.default_rng(seed)`` in the order listed.
"""

import numpy as np

TWO_PI = 2.0 * np.pi


def apply_A(c, u, ux, uy, uxx, uxy, uyy):
    """[Au] = -c11 u_xx - 2 c12 u_xy - c22 u_yy + c1 u_x + c2 u_y + c u."""
    c11, c12, c22, c1, c2, c0 = c
    return (-c11 * uxx - 2.0 * c12 * uxy - c22 * uyy + c1 * ux + c2 * uy
            + c0 * u)


# -- workload 1: Poisson, u = exp(x) cos(y) + x^2 y --------------------------
def poisson_coeffs(x, y):
    z = np.zeros_like(x)
    o = np.ones_like(x)
    return np.stack([o, z, o, z, z, z])


def poisson_u(x, y):
    return np.exp(x) * np.cos(y) + x * x * y


def poisson_g(x, y):
    # exp(x) cos(y) is harmonic, so -Lap u = -2 y
    return -2.0 * y


# -- workload 2 family: full variable-coefficient operator -------------------
def varcoeff(x, y, phases=None):
    """c11 = 1 + .5 sin(2 pi x) cos(2 pi y), c22 = 1 + .3 cos(2 pi x),
    c12 = .1 sin(pi x) sin(pi y), c1 = c2 = .5 sin(2 pi y), c = 1 + x^2;
    optional phases (6 values) shift every sine/cosine argument."""
    f = np.zeros(6) if phases is None else np.asarray(phases, dtype=float)
    c11 = 1.0 + 0.5 * np.sin(TWO_PI * x + f[0]) * np.cos(TWO_PI * y + f[1])
    c22 = 1.0 + 0.3 * np.cos(TWO_PI * x + f[2])
    c12 = 0.1 * np.sin(np.pi * x + f[3]) * np.sin(np.pi * y + f[4])
    c1 = 0.5 * np.sin(TWO_PI * y + f[5])
    c0 = 1.0 + x * x
    return np.stack([c11, c12, c22, c1, c1.copy(), c0])


class FourierSolution:
    """u = sum_k a_k cos(2 pi (m_k x + n_k y) + phi_k), a ~ N(0,1),
    m, n ~ U{1..4}, phi ~ U[0, 2 pi).  Draw order: a, m, n, phi."""

    def __init__(self, seed, n_modes=8):
        rng = np.random.default_rng(seed)
        self.a = rng.standard_normal(n_modes)
        self.m = rng.integers(1, 5, n_modes)
        self.n = rng.integers(1, 5, n_modes)
        self.phi = rng.uniform(0.0, TWO_PI, n_modes)

    def derivs(self, x, y):
        u = np.zeros_like(x)
        ux = np.zeros_like(x)
        uy = np.zeros_like(x)
        uxx = np.zeros_like(x)
        uxy = np.zeros_like(x)
        uyy = np.zeros_like(x)
        for a, m, n, ph in zip(self.a, self.m, self.n, self.phi):
            th = TWO_PI * (m * x + n * y) + ph
            cs, sn = np.cos(th), np.sin(th)
            km, kn = TWO_PI * m, TWO_PI * n
            u += a * cs
            ux -= a * km * sn
            uy -= a * kn * sn
            uxx -= a * km * km * cs
            uxy -= a * km * kn * cs
            uyy -= a * kn * kn * cs
        return u, ux, uy, uxx, uxy, uyy

    def u(self, x, y):
        return self.derivs(x, y)[0]

    def g(self, x, y, coeffs):
        return apply_A(coeffs, *self.derivs(x, y))


class PolySolution:
    """u = sum_{i,j <= deg} a_ij x^i y^j with a ~ N(0,1) (seeded)."""

    def __init__(self, seed, deg):
        rng = np.random.default_rng(seed)
        self.a = rng.standard_normal((deg + 1, deg + 1))
        self.deg = deg

    def derivs(self, x, y):
        d = self.deg
        out = [np.zeros_like(x) for _ in range(6)]
        for i in range(d + 1):
            for j in range(d + 1):
                a = self.a[i, j]
                xi = x ** i
                yj = y ** j
                dxi = i * x ** (i - 1) if i >= 1 else 0.0 * x
                dyj = j * y ** (j - 1) if j >= 1 else 0.0 * y
                ddxi = i * (i - 1) * x ** (i - 2) if i >= 2 else 0.0 * x
                ddyj = j * (j - 1) * y ** (j - 2) if j >= 2 else 0.0 * y
                out[0] += a * xi * yj
                out[1] += a * dxi * yj
                out[2] += a * xi * dyj
                out[3] += a * ddxi * yj
                out[4] += a * dxi * dyj
                out[5] += a * xi * ddyj
        return tuple(out)

    def u(self, x, y):
        return self.derivs(x, y)[0]

    def g(self, x, y, coeffs):
        return apply_A(coeffs, *self.derivs(x, y))


# -- workload 3: backward-Euler heat step (I - dt Lap) u = u_prev -----------
HEAT_DT = 1e-3


def heat_coeffs(x, y, dt=HEAT_DT):
    z = np.zeros_like(x)
    d = np.full_like(x, dt)
    return np.stack([d, z, d.copy(), z, z.copy(), np.ones_like(x)])


def gaussian_bumps(x, y, seed, n_bumps=16, width=0.05):
    """u0 = sum_k exp(-|x - x_k|^2 / w^2), x_k ~ U[0.15, 0.85]^2."""
    rng = np.random.default_rng(seed)
    ctr = rng.uniform(0.15, 0.85, (n_bumps, 2))
    u = np.zeros_like(x)
    for (cx, cy) in ctr:
        u += np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / width ** 2)
    return u


# -- workload 4: refined trees, concentrated load ---------------------------
def refined_problem(seed):
    """Per-problem draws: 6 phases ~ U[0, 2pi), then x_hat ~ U[0.1, 0.9]^2."""
    rng = np.random.default_rng(seed)
    phases = rng.uniform(0.0, TWO_PI, 6)
    xhat = rng.uniform(0.1, 0.9, 2)
    return phases, xhat


def gaussian_load(x, y, xhat, width=1e-3):
    return np.exp(-((x - xhat[0]) ** 2 + (y - xhat[1]) ** 2) / width ** 2)


# -- workload 5: coefficient perturbation for the gradient problem ----------
def problem_phases(seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, TWO_PI, 6)


class Perturbation:
    """delta = sum of 4 Fourier modes (a ~ N(0,1), m, n ~ U{1..3},
    phi ~ U[0, 2pi)), scaled so that max |delta| = 1 over a 513 x 513 grid."""

    def __init__(self, seed, n_modes=4):
        rng = np.random.default_rng(seed)
        self.a = rng.standard_normal(n_modes)
        self.m = rng.integers(1, 4, n_modes)
        self.n = rng.integers(1, 4, n_modes)
        self.phi = rng.uniform(0.0, TWO_PI, n_modes)
        t = np.linspace(0.0, 1.0, 513)
        X, Y = np.meshgrid(t, t)
        self.scale = 1.0 / np.max(np.abs(self._raw(X, Y)))

    def _raw(self, x, y):
        d = np.zeros_like(x)
        for a, m, n, ph in zip(self.a, self.m, self.n, self.phi):
            d += a * np.cos(TWO_PI * (m * x + n * y) + ph)
        return d

    def __call__(self, x, y):
        return self.scale * self._raw(x, y)


# -- accuracy experiments against an over-resolved self-reference ------------
# Variable-coefficient Helmholtz (paper Sec. 7.2): -Lap u - kappa^2 (1 - c) u = g
# on the unit square, c a sum of two Gaussians (the scattering potential), g a
# Gaussian, kappa = 40; Dirichlet data 0 (the paper does not state it).
HELM_KAPPA = 40.0


def scattering_potential(x, y):
    return (0.5 * np.exp(-200.0 * ((x - 0.35) ** 2 + (y - 0.6) ** 2))
            + 0.5 * np.exp(-200.0 * ((x - 0.6) ** 2 + (y - 0.45) ** 2)))


def helmholtz_coeffs(x, y, kappa=HELM_KAPPA):
    z = np.zeros_like(x)
    o = np.ones_like(x)
    return np.stack([o, z, o.copy(), z, z.copy(),
                     -kappa * kappa * (1.0 - scattering_potential(x, y))])


def helmholtz_load(x, y):
    return np.exp(-300.0 * ((x - 0.25) ** 2 + (y - 0.75) ** 2))


# Poisson with an indicator load (paper Sec. 7.4): g = 1 on [1/4, 1/2]^2, else
# 0, Dirichlet data 0 (not stated in the paper); the jumps lie on leaf edges
# when the number of leaves per side is a multiple of 4.
def indicator_load(x, y):
    return ((x >= 0.25) & (x <= 0.5) & (y >= 0.25) & (y <= 0.5)).astype(float)


# -- workload 7: Crank-Nicolson step of convection-diffusion (Sec. 7.6) -------
# u_t = eps Lap u - u_x on [0,1]^2, periodic in x, zero Neumann data in y,
# initial value exp(-alpha |x - xhat|^2).  One step with time step k solves
# (I/k - A/2) u_new = (I/k + A/2) u_old with A = eps Lap - d/dx; in the form
# of the problem statement the left operator has c11 = c22 = eps/2, c1 = 1/2,
# c = 1/k.
CD_EPS = 1.0 / 200.0
CD_ALPHA = 50.0
CD_XHAT = (0.25, 0.25)


def convdiff_coeffs(x, y, k, eps=CD_EPS):
    z = np.zeros_like(x)
    e = np.full_like(x, 0.5 * eps)
    return np.stack([e, z, e.copy(), np.full_like(x, 0.5), z.copy(), np.full_like(x, 1.0 / k)])


def convdiff_initial(x, y, alpha=CD_ALPHA, xhat=CD_XHAT):
    return np.exp(-alpha * ((x - xhat[0]) ** 2 + (y - xhat[1]) ** 2))


class PolyYSolution:
    """u = sum_{j <= deg} a_j y^j with a ~ N(0,1) (seeded): constant in x, so
    periodic in x for any period."""

    def __init__(self, seed, deg):
        self.a = np.random.default_rng(seed).standard_normal(deg + 1)

    def derivs(self, x, y):
        z = np.zeros_like(x)
        u, uy, uyy = z.copy(), z.copy(), z.copy()
        for j, a in enumerate(self.a):
            u += a * y ** j
            if j >= 1:
                uy += a * j * y ** (j - 1)
            if j >= 2:
                uyy += a * j * (j - 1) * y ** (j - 2)
        return u, z.copy(), uy, z.copy(), z.copy(), uyy

    def u(self, x, y):
        return self.derivs(x, y)[0]

    def g(self, x, y, coeffs):
        return apply_A(coeffs, *self.derivs(x, y))


def side_data(sol, xy, kinds, rect):
    """Boundary data at boundary nodes xy [n, 2] with side conditions kinds
    ('D', 'N' or 'P' per node) on the rectangle (X0, X1, Y0, Y1): u on
    Dirichlet sides, the flux +u_x (vertical sides) or +u_y (horizontal
    sides) on Neumann sides, 0 on periodic sides."""
    x, y = xy[:, 0], xy[:, 1]
    u, ux, uy = sol.derivs(x, y)[:3]
    X0, X1, Y0, Y1 = rect
    tol = 1e-12 * max(X1 - X0, Y1 - Y0)
    horiz = (np.abs(y - Y0) <= tol) | (np.abs(y - Y1) <= tol)
    flux = np.where(horiz, uy, ux)
    kinds = np.asarray(kinds)
    return np.where(kinds == "D", u, np.where(kinds == "N", flux, 0.0))


def convdiff_smooth_initial(x, y, beta=12.0, xhat=CD_XHAT):
    """A bump near xhat that fits the side conditions of the Sec. 7.6
    problem: periodic in x, and even about y = 0 and y = 1 (so every odd
    y-derivative, the Neumann data included, vanishes there)."""
    bx = np.exp(beta * (np.cos(TWO_PI * (x - xhat[0])) - 1.0))
    by = (np.exp(beta * (np.cos(np.pi * (y - xhat[1])) - 1.0)) +
          np.exp(beta * (np.cos(np.pi * (y + xhat[1])) - 1.0)))
    return bx * by


# -- Sec. 7.3: concentrated load, kappa = 20, refinement toward the load -----
CONC_KAPPA = 20.0
CONC_ALPHA = 3000.0
CONC_XHAT = (0.25, 0.75)      # a vertex of the 4 x 4 grid (one level of refinement: 28 leaves)


def concentrated_coeffs(x, y, kappa=CONC_KAPPA):
    """-Lap u - kappa^2 u."""
    z = np.zeros_like(x)
    o = np.ones_like(x)
    return np.stack([o, z, o.copy(), z, z.copy(), np.full_like(x, -kappa * kappa)])


def concentrated_load(x, y, alpha=CONC_ALPHA, xhat=CONC_XHAT):
    return np.exp(-alpha * ((x - xhat[0]) ** 2 + (y - xhat[1]) ** 2))
