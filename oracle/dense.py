"""Dense-grid FP64 finite-difference solver (oracle O1).

The same scheme the MPS method discretises, evaluated on the full grid:

* Vlasov equation without collisions, one electron species (Problem
  Statement, eq. 1 with C = 0):  df/dt = -v df/dx - (q/m) E df/dv.
* Poisson + E = -dphi/dx (Problem Statement, eqs. 2-3) with an immobile
  neutralising background: the periodic 3-point Laplacian is singular, so
  phi = L^+ n (pseudo-inverse; the constant background drops out because
  L^+ 1 = 0) and E = -Dx phi with the same periodic central difference.
* Periodic second-order central difference in x (SI, "First Derivative,
  Centered, Periodic Boundary Conditions"), or the upwind alternative (SI,
  "Upwind time evolution"): the second-order backward difference where
  v > 0 and the forward one where v < 0 (SI, "First Derivative, Forward /
  Backward, Periodic Boundary Conditions").  Reading: the paper's sentence
  (backward for positive velocities) is followed; its displayed formula
  pairs forward with H(v), which would be the downwind choice.
* Central difference in v with zero-gradient boundaries by a mirrored ghost
  point, which makes the derivative vanish at the first and last node (SI,
  "First Derivative, Centered, Zero Gradient Boundary Conditions").
* Left Riemann sum for integrals (SI, "Integration").
* Collisions (Methods, "Collision Operator"): the Dougherty operator
  nu d/dv [(v - v0) f + vth^2 df/dv] with v0 the species' average velocity
  and vth its thermal velocity.  Reading: both are the local moments of f at
  each x (left Riemann sums like the density): n = dv sum_j f, v0 = dv sum_j
  v_j f / n, vth^2 = dv sum_j v_j^2 f / n - v0^2, recomputed from every RK
  stage's state, so the operator conserves density, momentum and energy up
  to the discretisation; where n = 0 the drift and temperature are taken as
  0.  A second model (coll_model = 1) keeps v0 and vth as fixed parameters
  of the species (a linearisation about one Maxwellian).  Both derivatives
  are the zero-gradient central difference in v.
* Several species (Methods, the Landau / Buneman / shock set-ups): each
  species s has its own v grid and q_s/m_s and all share x and E; Poisson
  reads Laplacian(phi) = -sum_s q_s n_s (normalised units; the
  pseudo-inverse again drops the mean, i.e. any neutralising background).
  One species with q = -1 is the single-electron case above.
* Classic RK4 with a fixed step (SI, "Compressed time evolution algorithm"),
  or an adaptive one (Methods, "Time Evolution Procedure", eq. CFL): a
  fraction cfl of dt_max = (|v|_max / dx + |q/m| |E|_max / dv)^-1 for one
  collisionless species, |E|_max measured on the state at the start of the
  step.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__``.
"""
from __future__ import annotations

import numpy as np


def density(F: np.ndarray, dv: float) -> np.ndarray:
    """n_i = dv * sum_j F_ij  (SI, Integration: left Riemann sum)."""
    return dv * F.sum(axis=1)


def poisson_field(n: np.ndarray, dx: float) -> np.ndarray:
    """E = -Dx L^+ n on the periodic grid (Problem Statement eqs. 2-3).

    L (periodic 3-point Laplacian) and Dx (periodic central difference) are
    circulant, so the discrete Fourier transform diagonalises both: mode
    theta = 2 pi q / N has L -> -4 sin^2(theta/2)/dx^2 and Dx -> i sin(theta)/dx.
    The pseudo-inverse maps the q = 0 mode (the neutralising background) to 0.
    """
    N = n.size
    nh = np.fft.fft(n)
    theta = 2.0 * np.pi * np.arange(N) / N
    lam_L = -4.0 * np.sin(theta / 2.0) ** 2 / dx ** 2
    lam_D = 1j * np.sin(theta) / dx
    Eh = np.zeros_like(nh)
    nz = np.arange(N) != 0
    Eh[nz] = -lam_D[nz] * nh[nz] / lam_L[nz]
    return np.real(np.fft.ifft(Eh))


def poisson_field_dense(n: np.ndarray, dx: float) -> np.ndarray:
    """Same field with explicit matrices: E = -Dx pinv(L) n (small N only).
    The paper's own route for the inverse Laplacian: build the matrix, invert
    it (SI, "Inverse Laplacian")."""
    N = n.size
    L = np.zeros((N, N))
    Dx = np.zeros((N, N))
    for i in range(N):
        L[i, i] = -2.0
        L[i, (i + 1) % N] += 1.0
        L[i, (i - 1) % N] += 1.0
        Dx[i, (i + 1) % N] += 0.5
        Dx[i, (i - 1) % N] -= 0.5
    L /= dx ** 2
    Dx /= dx
    return -Dx @ np.linalg.pinv(L) @ n


def ddx(F: np.ndarray, dx: float) -> np.ndarray:
    """(F_{i+1,j} - F_{i-1,j}) / (2 dx), i periodic."""
    return (np.roll(F, -1, axis=0) - np.roll(F, 1, axis=0)) / (2.0 * dx)


def ddx_backward(F: np.ndarray, dx: float) -> np.ndarray:
    """(3 F_i - 4 F_{i-1} + F_{i-2}) / (2 dx), i periodic."""
    return (3.0 * F - 4.0 * np.roll(F, 1, axis=0) + np.roll(F, 2, axis=0)) / (2.0 * dx)


def ddx_forward(F: np.ndarray, dx: float) -> np.ndarray:
    """(-3 F_i + 4 F_{i+1} - F_{i+2}) / (2 dx), i periodic."""
    return (-3.0 * F + 4.0 * np.roll(F, -1, axis=0) - np.roll(F, -2, axis=0)) / (2.0 * dx)


def advection(F: np.ndarray, p) -> np.ndarray:
    """v df/dx on the grid: central, or upwind (backward where v > 0,
    forward where v < 0; v = 0 contributes nothing either way)."""
    v = p.v()
    if getattr(p, "x_scheme", 0) == 1:
        return (np.maximum(v, 0.0)[None, :] * ddx_backward(F, p.dx)
                + np.minimum(v, 0.0)[None, :] * ddx_forward(F, p.dx))
    return v[None, :] * ddx(F, p.dx)


def ddv(F: np.ndarray, dv: float) -> np.ndarray:
    """(F_{i,j+1} - F_{i,j-1}) / (2 dv) inside, 0 at j = 0 and j = Nv-1."""
    out = np.zeros_like(F)
    out[:, 1:-1] = (F[:, 2:] - F[:, :-2]) / (2.0 * dv)
    return out


def field(F: np.ndarray, p) -> np.ndarray:
    return poisson_field(density(F, p.dv), p.dx)


def collision_moments(F: np.ndarray, p):
    """Local drift v0(x) and thermal speed squared vth^2(x) of F: n = dv sum
    F, v0 = dv sum v F / n, vth^2 = dv sum v^2 F / n - v0^2 (0 where n = 0)."""
    v = p.v()
    n = p.dv * F.sum(axis=1)
    P = p.dv * (F * v[None, :]).sum(axis=1)
    W = p.dv * (F * (v * v)[None, :]).sum(axis=1)
    ok = n != 0.0
    v0 = np.zeros_like(n)
    v0[ok] = P[ok] / n[ok]
    T = np.zeros_like(n)
    T[ok] = W[ok] / n[ok] - v0[ok] ** 2
    return v0, T


def collision(F: np.ndarray, p) -> np.ndarray:
    """nu Dv[(v - v0) F + vth^2 Dv F] (Dougherty): v0, vth^2 the local
    moments of F (coll_model 0), or the species' fixed parameters
    (coll_model 1)."""
    v = p.v()
    if getattr(p, "coll_model", 0) == 1:
        G = (v - p.nu_v0)[None, :] * F + p.nu_vth ** 2 * ddv(F, p.dv)
    else:
        v0, T = collision_moments(F, p)
        G = (v[None, :] - v0[:, None]) * F + T[:, None] * ddv(F, p.dv)
    return p.nu * ddv(G, p.dv)


def rhs(F: np.ndarray, p, E: np.ndarray | None = None) -> np.ndarray:
    """R(F) = -v Dx F - (q/m) E Dv F + C[F]  (eq. 1); E from F alone (one
    electron species on a neutralising background) unless given."""
    if E is None:
        E = field(F, p)
    out = -advection(F, p) - p.qm * E[:, None] * ddv(F, p.dv)
    if getattr(p, "nu", 0.0) != 0.0:
        out = out + collision(F, p)
    return out


def field_species(Fs, ps, charges) -> np.ndarray:
    """E of several species: Laplacian(phi) = -sum_s q_s n_s."""
    rho = sum(-q * density(F, p.dv) for F, p, q in zip(Fs, ps, charges))
    return poisson_field(rho, ps[0].dx)


def rk4_step_species(Fs, ps, charges, dt: float):
    """One RK4 step of all species together; E of each stage from all of
    them."""
    def R(Gs):
        E = field_species(Gs, ps, charges)
        return [rhs(G, p, E) for G, p in zip(Gs, ps)]
    k1 = R(Fs)
    k2 = R([F + 0.5 * dt * k for F, k in zip(Fs, k1)])
    k3 = R([F + 0.5 * dt * k for F, k in zip(Fs, k2)])
    k4 = R([F + dt * k for F, k in zip(Fs, k3)])
    return [F + (dt / 6.0) * (a + 2.0 * b + 2.0 * c + d)
            for F, a, b, c, d in zip(Fs, k1, k2, k3, k4)]


def cfl_dt(F: np.ndarray, p) -> float:
    """cfl * (|v|_max / dx + |q/m| |E|_max / dv)^-1 (eq. CFL, one species,
    no collisions)."""
    vmax = max(abs(p.v_min), abs(p.v_max))
    emax = float(np.abs(field(F, p)).max())
    inv = vmax / p.dx + abs(p.qm) * emax / p.dv
    nu = getattr(p, "nu", 0.0)
    if nu != 0.0:
        # the collision terms of eq. CFL
        inv += nu * vmax / p.dv + 2.0 * nu * p.nu_vth ** 2 / p.dv ** 2
    return p.cfl / inv


def rk4_step(F: np.ndarray, p, dt: float | None = None) -> np.ndarray:
    """f_{n+1} = f_n + dt/6 (k1 + 2 k2 + 2 k3 + k4)  (SI, RK4); dt is the
    fixed p.dt, or the adaptive CFL step when p.cfl > 0."""
    if dt is not None:
        h = dt
    elif getattr(p, "cfl", 0.0) > 0.0:
        h = cfl_dt(F, p)
    else:
        h = p.dt
    k1 = rhs(F, p)
    k2 = rhs(F + 0.5 * h * k1, p)
    k3 = rhs(F + 0.5 * h * k2, p)
    k4 = rhs(F + h * k3, p)
    return F + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def initial(ax: np.ndarray, bv: np.ndarray) -> np.ndarray:
    """f0(x_i, v_j) = sum_r ax[r, i] bv[r, j]."""
    return np.einsum("ri,rj->ij", ax, bv)


def diagnostics(F: np.ndarray, p) -> dict:
    """Mass, momentum, kinetic energy (left Riemann sums) and field energy
    W_E = 1/2 dx sum_i E_i^2."""
    v = p.v()
    w = p.dx * p.dv
    E = field(F, p)
    return {
        "mass": w * F.sum(),
        "momentum": w * (F * v[None, :]).sum(),
        "kinetic": 0.5 * w * (F * (v ** 2)[None, :]).sum(),
        "field_energy": 0.5 * p.dx * float(np.sum(E ** 2)),
    }
