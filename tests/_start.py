"""Start states for parity tests, built on the host by the oracle.

A parity test runs the GPU and the oracle from the same state.  That state
is made here with the oracle's own arithmetic from the seeded inputs of
``workloads`` (the separable profile as a product MPS, plus an optional
seeded random-MPS perturbation, compressed as the problem says), and the
GPU receives it through ``mps_set_cores``.  Nothing the GPU computes is
ever an input of the oracle.
"""
import numpy as np

import workloads as wl
from oracle import mps as omps


def oracle_start(w, pert_chi=0, amp=0.0, seed=2205, pert=None):
    """The problem's initial state f0 (the profile's product MPS compressed
    to the problem's cap and tolerance), plus amp times the seeded random
    MPS of bond pert_chi (or the given cores), compressed again.  In the
    IG ordering the cores are the oracle's fused sites of dimension 4."""
    p = w.problem
    assert w.ax.shape[0] == 1 and w.bv.shape[0] == 1
    binary = 1 if p.order == 4 else p.order
    f = omps.chain_product_mps(omps.vector_mps(w.ax[0]), omps.vector_mps(w.bv[0]),
                               p.Lx, p.Lv, binary)
    if p.order == 4:
        f = omps.fuse_pairs(f)
    f = omps.compress_state(f, p.chi_max, p)
    if pert is None and pert_chi:
        pert = wl.random_mps_cores(p.n_sites, pert_chi, seed=seed)
    if pert is not None:
        if p.order == 4:
            pert = omps.fuse_pairs(pert)
        f = omps.compress_state(omps.add([(1.0, f), (amp, pert)]), p.chi_max, p)
    return f


def binary_cores(f, p):
    """The cores the library holds: binary sites; a fused IG site of
    dimension 4 is split exactly into its x and v sites (SVD of the site,
    every value kept)."""
    if p.order != 4:
        return [np.ascontiguousarray(c) for c in f]
    out = []
    for c in f:
        l, _, r = c.shape
        M = c.reshape(l * 2, 2 * r)
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        out.append(np.ascontiguousarray(U.reshape(l, 2, -1)))
        out.append(np.ascontiguousarray((S[:, None] * Vt).reshape(-1, 2, r)))
    return out


def gpu_state(B, w, f):
    """A library state of w's problem holding the cores f."""
    st = B.MpsState(w.problem, w.ax, w.bv)
    st.set_cores(binary_cores(f, w.problem))
    return st
