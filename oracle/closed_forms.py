"""Closed-form results for the two-fluid (Maxwell + London) model, in FP64.

TEST INFRASTRUCTURE ONLY.  This module, like everything under ``oracle/``, is
imported by ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py``; the product library never imports it.

Contents (each function cites the passage it follows):

* continuum wavenumber, skin depth and normal-incidence reflection
  (Sec. 4.1 Eqs. nk, ngamma, nkappa, skin; Sec. 4.2 Eqs. beta, Ref, beta_cases);
* the same quantities for the discrete leap-frog scheme of Algorithm 1
  (derived from the update equations of Algorithm 1; see ``discrete_*``);
* the exact single-mode amplification matrix of one time step (Algorithm 1);
* the stability bound of that step.

Units are SI throughout.  ``ell`` denotes 1/lambda_L^2 (m^-2); ``ell = 0`` is a
non-superconducting material (Sec. 3).
"""
import numpy as np

EPS0 = 8.8541878128e-12  # F/m (CODATA 2018)
MU0 = 1.25663706212e-6   # H/m (CODATA 2018)
C0 = 1.0 / np.sqrt(EPS0 * MU0)
ETA0 = np.sqrt(MU0 / EPS0)


# ----------------------------------------------------------------------------
# Continuum model, Sec. 4.1 and Sec. 4.2
# ----------------------------------------------------------------------------
def wavenumber(omega, eps_r=1.0, sigma=0.0, ell=0.0, mu_r=1.0):
    """Complex k of a plane wave in a homogeneous two-fluid medium (Eq. nk).

    k^2 = (mu eps omega^2 - 1/lambda^2) + i mu sigma omega, root with Im k >= 0.
    """
    mu = MU0 * mu_r
    eps = EPS0 * eps_r
    k2 = (mu * eps * omega**2 - ell) + 1j * mu * sigma * omega
    k = np.sqrt(np.asarray(k2, dtype=complex))
    return np.where(np.imag(k) < 0, -k, k)


def gamma_kappa(omega, eps_r=1.0, sigma=0.0, ell=0.0, mu_r=1.0):
    """Real and imaginary parts of k written out as in Eqs. ngamma and nkappa."""
    mu = MU0 * mu_r
    eps = EPS0 * eps_r
    a = mu * eps * omega**2 - ell
    m = np.sqrt(a**2 + (mu * sigma * omega) ** 2)
    gamma = np.sqrt((m + a) / 2.0)
    kappa = np.sqrt(np.maximum(m - a, 0.0) / 2.0)
    return gamma, kappa


def skin_depth(freq, eps_r=1.0, sigma=0.0, ell=0.0):
    """delta = 1/kappa (Eq. skin); inf where kappa = 0 (a lossless propagating medium)."""
    _, kappa = gamma_kappa(2 * np.pi * np.asarray(freq, dtype=float), eps_r, sigma, ell)
    with np.errstate(divide="ignore"):
        return np.where(kappa > 0, 1.0 / np.where(kappa > 0, kappa, 1.0), np.inf)


def reflection(freq, eps_r1=1.0, eps_r2=1.0, sigma2=0.0, ell2=0.0):
    """Normal-incidence power reflection R = |(1-beta)/(1+beta)|^2 (Eqs. beta, Ref).

    beta = sqrt(mu1/eps1) k2 / (mu2 omega); medium 1 is lossless (vacuum in the paper).
    """
    omega = 2 * np.pi * np.asarray(freq, dtype=float)
    k2 = wavenumber(omega, eps_r2, sigma2, ell2)
    beta = np.sqrt(MU0 / (EPS0 * eps_r1)) * k2 / (MU0 * omega)
    r = (1 - beta) / (1 + beta)
    return np.abs(r) ** 2


def cutoff_frequency(ell, eps_r=1.0):
    """sigma = 0 cutoff f_c = 1/(2 pi lambda sqrt(mu eps)) (Eq. beta_cases)."""
    return np.sqrt(ell) / (2 * np.pi * np.sqrt(MU0 * EPS0 * eps_r))


# ----------------------------------------------------------------------------
# The discrete scheme of Algorithm 1 (plane waves and single modes)
# ----------------------------------------------------------------------------
def step_coefficients(dt, theta, eps_r, sigma, ell):
    """Per-edge coefficients of one step of Algorithm 1 in the form x' = a x + b (...).

    Step 3 of Algorithm 1: E' = (1 + theta s)^-1 (E + dt/eps curlH - (1-theta) s E - dt/eps Js),
    s = sigma dt / eps.  Hence a = (1 - (1-theta) s)/(1 + theta s), b = (dt/eps)/(1 + theta s).
    Steps 2 and 4 together advance Js by j E with j = dt/(lambda^2 mu0) = dt ell / mu0.
    """
    eps = EPS0 * eps_r
    s = sigma * dt / eps
    a = (1 - (1 - theta) * s) / (1 + theta * s)
    b = (dt / eps) / (1 + theta * s)
    j = dt * ell / MU0
    return a, b, j


def discrete_K(k, d):
    """Discrete wavenumber of a centred difference on spacing d: K = (2/d) sin(k d / 2)."""
    return 2.0 / d * np.sin(k * d / 2.0)


def levi_civita(i, j, k):
    return int(np.sign((j - i) * (k - i) * (k - j)))


def amplification_matrix(kwave, d, dt, theta, eps_r, sigma, ell, axis=2, pol=0):
    """Exact 3x3 map of one fused leap-frog step for one grid Fourier mode.

    Mode: E_pol = X cos(k x_axis) on E nodes, H_h = Y sin(k x_axis) on H nodes
    (shifted by half a cell), Js_pol = Z cos(k x_axis), with h the third axis.
    State (X, Y, Z) = (E^n, H^{n-1/2}, Js^{n-1/2}).  Derived from Algorithm 1
    with B = mu0 H: the H update is H' = H - (dt/mu0) curl E, the Js update
    is Js' = Js + j E and the E update is E' = a E + b (curl H' - Js').
    """
    h_ax = 3 - axis - pol
    s = levi_civita(h_ax, axis, pol)
    K = discrete_K(kwave, d)
    a, b, j = step_coefficients(dt, theta, eps_r, sigma, ell)
    hh = dt / MU0
    return np.array(
        [
            [a - b * hh * K * K - b * j, -b * s * K, -b],
            [hh * s * K, 1.0, 0.0],
            [j, 0.0, 1.0],
        ]
    )


def half_kick_matrix(kwave, d, dt, eps_r, sigma, ell, axis=2, pol=0, sign=+1.0):
    """Map (E^n, H^{n-1/2}, Js^{n-1/2}) -> (E^n, H^n, Js^n) for one mode (sign=+1).

    Integer-time values follow from the half updates of Algorithm 1 (steps 1, 2
    read backwards): H^n = H^{n-1/2} - (dt/2 mu0) curl E^n, Js^n = Js^{n-1/2} + (j/2) E^n.
    """
    h_ax = 3 - axis - pol
    s = levi_civita(h_ax, axis, pol)
    K = discrete_K(kwave, d)
    _, _, j = step_coefficients(dt, 1.0, eps_r, sigma, ell)
    hh = dt / MU0
    T = np.eye(3)
    T[1, 0] = sign * 0.5 * hh * s * K
    T[2, 0] = sign * 0.5 * j
    return T


def discrete_K2(omega, dt, theta, eps_r, sigma, ell):
    """Squared discrete wavenumber of a time-harmonic wave exp(-i omega t) under Algorithm 1.

    With Omega = (2/dt) sin(omega dt/2) and Theta = cos(omega dt/2) + i (1 - 2 theta) sin(omega dt/2),
    the leap-frog gives K^2 = mu0 eps Omega^2 + i mu0 sigma Omega Theta - ell.
    """
    Om = 2.0 / dt * np.sin(omega * dt / 2.0)
    Th = np.cos(omega * dt / 2.0) + 1j * (1 - 2 * theta) * np.sin(omega * dt / 2.0)
    return MU0 * EPS0 * eps_r * Om**2 + 1j * MU0 * sigma * Om * Th - ell


def discrete_k(omega, d, dt, theta, eps_r, sigma, ell):
    """Grid wavenumber k with (2/d) sin(k d/2) = K; the root with Im k >= 0, Re k >= 0."""
    K2 = discrete_K2(omega, dt, theta, eps_r, sigma, ell)
    # 2 cos(k d) = 2 - K^2 d^2
    kd = np.arccos(1.0 - K2 * d * d / 2.0 + 0j)
    k = kd / d
    if np.imag(k) < 0 or (np.imag(k) == 0 and np.real(k) < 0):
        k = -k
    return k


def discrete_skin_depth(freq, d, dt, theta, eps_r, sigma, ell):
    return 1.0 / np.imag(discrete_k(2 * np.pi * freq, d, dt, theta, eps_r, sigma, ell))


def discrete_reflection(freq, d, dt, theta, m1, m2, m0=None):
    """Discrete normal-incidence amplitude reflection at a node-aligned interface.

    Frequency-domain recurrence of the 1-D scheme: (E_{i+1} - 2E_i + E_{i-1})/d^2 + q_i E_i = 0
    with q = mu0 eps Omega^2 + i mu0 sigma Omega Theta - ell, i.e. q is the K^2 of
    ``discrete_K2`` for that node's material.  Medium 1 fills nodes i < 0, medium 2 nodes i > 0, and node 0 has
    q0 (by default the mean of q1 and q2).  Each medium is a tuple (eps_r, sigma, ell).
    Returns the complex r.
    """
    omega = 2 * np.pi * freq
    q1 = discrete_K2(omega, dt, theta, *m1)
    q2 = discrete_K2(omega, dt, theta, *m2)
    q0 = 0.5 * (q1 + q2) if m0 is None else discrete_K2(omega, dt, theta, *m0)
    k1 = discrete_k(omega, d, dt, theta, *m1)
    k2 = discrete_k(omega, d, dt, theta, *m2)
    dq = d * d * (q0 - q2)
    num = np.exp(-1j * k2 * d) - np.exp(-1j * k1 * d) - dq
    den = np.exp(1j * k1 * d) - np.exp(-1j * k2 * d) + dq
    return num / den


def stable_dt(spacings, ell_max, eps_r_min=1.0):
    """Largest stable dt of the leap-frog with a London term (theta >= 1/2, sigma >= 0).

    From the amplification matrix: with w^2 = (c dt)^2 ell / eps_r and v^2 = (c dt)^2 sum 4/d^2 / eps_r
    the step is stable iff w^2 + v^2 < 4, so dt < 2 / (c sqrt(sum 4/d_i^2 + ell_max)) for eps_r = 1.
    """
    c = C0 / np.sqrt(eps_r_min)
    s = sum(4.0 / (d * d) for d in spacings)
    return 2.0 / (c * np.sqrt(s + ell_max))
