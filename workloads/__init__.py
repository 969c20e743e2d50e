"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *describes* workloads and draws their inputs: grid bounds,
the separable initial profiles ``f0(x, v) = sum_r ax[r](x) * bv[r](v)`` sampled
on the grid, and i.i.d. Gaussian tensor cores used as a seeded perturbation.
It holds none of the method's arithmetic (no MPS/MPO algebra, no
factorisation, no time stepping) and imports nothing from ``oracle`` or from
the HIP package, so both sides can take their inputs from here.

Grid convention (the paper's uniform finite-difference grid, periodic in x,
closed zero-gradient interval in v):
  x_i = x_min + i*dx, dx = (x_max - x_min) / Nx, i in [0, Nx)
  v_j = v_min + j*dv, dv = (v_max - v_min) / (Nv - 1), j in [0, Nv)
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

ORDER_SEQ = 0          # sequential: x bits (coarse->fine) then v bits
ORDER_INTERLEAVED = 1  # interleaved: x1, v1, x2, v2, ... (coarse->fine)
ORDER_S2 = 2           # sequential: x bits fine->coarse, then v coarse->fine
ORDER_S3 = 3           # sequential: x bits coarse->fine, then v fine->coarse
ORDER_IG = 4           # interleaved, each (x_k, v_k) pair one site of dimension 4

PREC_FP64 = 0
PREC_FP32_CONTRACT = 1
PREC_BF16_CONTRACT = 2


@dataclasses.dataclass
class Problem:
    """Parameters of one 1D1V Vlasov-Poisson solve (single electron species)."""
    Lx: int
    Lv: int
    order: int
    x_min: float
    x_max: float
    v_min: float
    v_max: float
    qm: float = -1.0
    dt: float = 0.05
    chi_max: int = 16
    level: int = 1          # compression level C1..C5 (which points are capped)
    df_max: int = 0         # cap on the field bond, 0 = uncapped
    tol: float = 1e-10      # per-bond relative discarded weight
    precision: int = PREC_FP64
    x_scheme: int = 0       # x advection: 0 central, 1 upwind (second order)
    cfl: float = 0.0        # > 0: adaptive dt, this fraction of the CFL limit
    compression: int = 0    # 0 sweep, 1 centre-first (sequential orderings)
    nu: float = 0.0         # Dougherty collision rate (0: collisionless)
    nu_v0: float = 0.0      # its drift velocity
    nu_vth: float = 1.0     # its thermal speed
    coll_model: int = 0     # 0: drift and thermal speed from the moments of f; 1: fixed
    tall_apply: int = 0     # library only: 0 one reflector at a time, 1 compact WY (tall blocks)

    @property
    def Nx(self) -> int:
        return 1 << self.Lx

    @property
    def Nv(self) -> int:
        return 1 << self.Lv

    @property
    def dx(self) -> float:
        return (self.x_max - self.x_min) / self.Nx

    @property
    def dv(self) -> float:
        return (self.v_max - self.v_min) / (self.Nv - 1)

    def x(self) -> np.ndarray:
        return self.x_min + self.dx * np.arange(self.Nx)

    def v(self) -> np.ndarray:
        return self.v_min + self.dv * np.arange(self.Nv)

    @property
    def n_sites(self) -> int:
        return self.Lx + self.Lv


@dataclasses.dataclass
class Workload:
    name: str
    problem: Problem
    ax: np.ndarray          # (rank, Nx)
    bv: np.ndarray          # (rank, Nv)
    steps: int


def landau_profiles(p: Problem, k: float, alpha: float):
    """f0 = (1 + alpha cos(k x)) exp(-v^2/2)/sqrt(2 pi) as one separable term."""
    ax = (1.0 + alpha * np.cos(k * p.x()))[None, :]
    bv = (np.exp(-0.5 * p.v() ** 2) / math.sqrt(2.0 * math.pi))[None, :]
    return ax, bv


def two_stream_profiles(p: Problem, k: float, alpha: float, v0: float = 2.4):
    """f0 = (1 + alpha cos(k x)) [e^{-(v-v0)^2/2} + e^{-(v+v0)^2/2}] / (2 sqrt(2 pi))."""
    v = p.v()
    ax = (1.0 + alpha * np.cos(k * p.x()))[None, :]
    bv = ((np.exp(-0.5 * (v - v0) ** 2) + np.exp(-0.5 * (v + v0) ** 2))
          / (2.0 * math.sqrt(2.0 * math.pi)))[None, :]
    return ax, bv


def stable_dt(p: Problem, dt_cfg: Optional[float]) -> float:
    """Fixed RK4 step: keep the stated dt when the x-advection Courant number
    v_max*dt/dx stays <= 2 (inside the RK4 imaginary-axis limit 2*sqrt(2)),
    else use 1.3*dx/v_max."""
    vmax = max(abs(p.v_min), abs(p.v_max))
    if dt_cfg is not None and vmax * dt_cfg / p.dx <= 2.0:
        return dt_cfg
    lim = 1.3 * p.dx / vmax
    return lim if dt_cfg is None else min(dt_cfg, lim)


def buneman(L: int = 9, Lv: Optional[int] = None, chi: int = 64, tol: float = 0.0,
            level: int = 5, df_max: int = 0, order: int = ORDER_SEQ, k: float = 0.1,
            A: float = 1e-3, mass_ratio: float = 25.0, dt_cfg: Optional[float] = None,
            nu: float = 0.0):
    """Buneman instability (Methods): electrons drifting at v0 = omega_pe / k
    (= 1/k in these units) with unit thermal speed and a (1 + A cos kx)
    perturbation, ions at rest with T_i = T_e (vth_i^2 = m_e / m_i); x in
    [-pi/k, pi/k) periodic; v in +-6/k (electrons) and +-50 vth_i (ions).
    Returns ([electron workload, ion workload], [q_e, q_i] = [-1, +1]); both
    share Lx = L and dt (the electron CFL limit)."""
    Lv = L if Lv is None else Lv
    x0, x1 = -math.pi / k, math.pi / k
    vth_i = math.sqrt(1.0 / mass_ratio)
    pe = Problem(Lx=L, Lv=Lv, order=order, x_min=x0, x_max=x1, v_min=-6.0 / k,
                 v_max=6.0 / k, qm=-1.0, chi_max=chi, level=level, df_max=df_max, tol=tol,
                 nu=nu, nu_v0=1.0 / k, nu_vth=1.0)
    pe.dt = stable_dt(pe, dt_cfg)
    pi_ = Problem(Lx=L, Lv=Lv, order=order, x_min=x0, x_max=x1, v_min=-50.0 * vth_i,
                  v_max=50.0 * vth_i, qm=1.0 / mass_ratio, dt=pe.dt, chi_max=chi,
                  level=level, df_max=df_max, tol=tol, nu=nu, nu_v0=0.0, nu_vth=vth_i)
    ve, vi = pe.v(), pi_.v()
    ax_e = (1.0 + A * np.cos(k * pe.x()))[None, :]
    bv_e = (np.exp(-0.5 * (ve - 1.0 / k) ** 2) / math.sqrt(2.0 * math.pi))[None, :]
    ax_i = np.ones((1, pe.Nx))
    bv_i = (np.exp(-0.5 * (vi / vth_i) ** 2) / math.sqrt(2.0 * math.pi * vth_i ** 2))[None, :]
    tag = "2^%dx2^%d_chi%d" % (L, Lv, chi)
    return ([Workload("buneman_electrons_" + tag, pe, ax_e, bv_e, 2000),
             Workload("buneman_ions_" + tag, pi_, ax_i, bv_i, 2000)], [-1.0, 1.0])


def landau_two_species(L: int = 6, Lv: Optional[int] = None, chi: int = 24, tol: float = 0.0,
                       level: int = 5, df_max: int = 0, order: int = ORDER_SEQ,
                       k: float = 0.75, A: float = 0.5, mass_ratio: float = 1836.0,
                       periods: int = 1, dt_cfg: Optional[float] = None, nu: float = 0.0):
    """Nonlinear Landau damping with mobile ions (Methods): Maxwellian ions
    and electrons of equal temperature (v_th,i^2 = m_e / m_i), the electrons
    modulated by (1 + A cos kx); x in [-a pi/k, a pi/k) with a = periods;
    v in +-6 v_th,s for each species.  Returns ([electrons, ions], [q_e, q_i]
    = [-1, +1]); both share Lx and dt (the electron CFL limit)."""
    Lv = L if Lv is None else Lv
    x0, x1 = -periods * math.pi / k, periods * math.pi / k
    vth_i = math.sqrt(1.0 / mass_ratio)
    pe = Problem(Lx=L, Lv=Lv, order=order, x_min=x0, x_max=x1, v_min=-6.0, v_max=6.0,
                 qm=-1.0, chi_max=chi, level=level, df_max=df_max, tol=tol, nu=nu)
    pe.dt = stable_dt(pe, dt_cfg)
    pi_ = Problem(Lx=L, Lv=Lv, order=order, x_min=x0, x_max=x1, v_min=-6.0 * vth_i,
                  v_max=6.0 * vth_i, qm=1.0 / mass_ratio, dt=pe.dt, chi_max=chi,
                  level=level, df_max=df_max, tol=tol, nu=nu, nu_vth=vth_i)
    ax_e = (1.0 + A * np.cos(k * pe.x()))[None, :]
    bv_e = (np.exp(-0.5 * pe.v() ** 2) / math.sqrt(2.0 * math.pi))[None, :]
    ax_i = np.ones((1, pe.Nx))
    bv_i = (np.exp(-0.5 * (pi_.v() / vth_i) ** 2) / math.sqrt(2.0 * math.pi * vth_i ** 2))[None, :]
    tag = "2^%dx2^%d_chi%d" % (L, Lv, chi)
    return ([Workload("landau_electrons_" + tag, pe, ax_e, bv_e, 1000),
             Workload("landau_ions_" + tag, pi_, ax_i, bv_i, 1000)], [-1.0, 1.0])


def landau_small(chi: int = 16, tol: float = 1e-10, level: int = 1,
                 L: int = 6, Lv: Optional[int] = None) -> Workload:
    """Landau damping, x in [0, 4 pi) periodic, v in [-6, 6], k=0.5,
    alpha=0.01, sequential ordering, dt=0.05, 100 steps."""
    Lv = L if Lv is None else Lv
    p = Problem(Lx=L, Lv=Lv, order=ORDER_SEQ, x_min=0.0, x_max=4.0 * math.pi,
                v_min=-6.0, v_max=6.0, dt=0.05, chi_max=chi, level=level,
                tol=tol)
    ax, bv = landau_profiles(p, 0.5, 0.01)
    return Workload("landau_2^%dx2^%d_seq_chi%d" % (L, Lv, chi), p, ax, bv, 100)


def two_stream(L: int = 10, chi: int = 64, tol: float = 1e-10, level: int = 1,
               df_max: int = 0, dt_cfg: Optional[float] = 0.02,
               order: int = ORDER_INTERLEAVED, steps: int = 2000) -> Workload:
    """Two-stream instability, x in [0, 10 pi) periodic (k=0.2), v in [-8, 8],
    beams at +-2.4 with unit thermal speed, interleaved ordering."""
    p = Problem(Lx=L, Lv=L, order=order, x_min=0.0, x_max=10.0 * math.pi,
                v_min=-8.0, v_max=8.0, chi_max=chi, level=level, df_max=df_max,
                tol=tol)
    p.dt = stable_dt(p, dt_cfg)
    ax, bv = two_stream_profiles(p, 0.2, 1e-3)
    return Workload("two_stream_2^%dx2^%d_%s_chi%d" % (
        L, L, "if" if order == ORDER_INTERLEAVED else "seq", chi), p, ax, bv, steps)


def landau_sweep(count: int = 64, seed: int = 2205) -> List[Workload]:
    """Parameter sweep of Landau instances: k ~ U[0.3, 0.6],
    alpha = 10^U[-3,-1], L ~ U{8..11}, chi ~ U{16,32,48,64}; drawn per
    instance in that order from one seeded generator."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        k = rng.uniform(0.3, 0.6)
        alpha = 10.0 ** rng.uniform(-3.0, -1.0)
        L = int(rng.integers(8, 12))
        chi = int(rng.choice([16, 32, 48, 64]))
        p = Problem(Lx=L, Lv=L, order=ORDER_SEQ, x_min=0.0,
                    x_max=2.0 * math.pi / k, v_min=-6.0, v_max=6.0,
                    chi_max=chi, level=1, tol=1e-10)
        p.dt = stable_dt(p, 0.05)
        ax, bv = landau_profiles(p, k, alpha)
        out.append(Workload("landau_sweep_%d" % i, p, ax, bv, 500))
    return out


def random_mps_cores(n_sites: int, chi: int, seed: int = 2205) -> List[np.ndarray]:
    """i.i.d. N(0, 1/(2*r_right)) cores A_j[a, s, b] with bonds
    r_j = min(chi, 2^j, 2^(n-j)); the variance choice makes the expected
    squared norm of the represented vector equal to one."""
    rng = np.random.default_rng(seed)
    bonds = [1] + [min(chi, 2 ** j, 2 ** (n_sites - j)) for j in range(1, n_sites)] + [1]
    cores = []
    for j in range(n_sites):
        a, b = bonds[j], bonds[j + 1]
        cores.append(rng.standard_normal((a, 2, b)) / math.sqrt(2.0 * b))
    return cores


def random_matrix(m: int, n: int, seed: int, decay: float = 0.0) -> np.ndarray:
    """Seeded Gaussian m x n matrix; with decay > 0 its columns are scaled by
    10^(-decay * j / n) so that the spectrum spans `decay` decades."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    if decay > 0:
        A = A * (10.0 ** (-decay * np.arange(n) / max(n, 1)))[None, :]
    return A
