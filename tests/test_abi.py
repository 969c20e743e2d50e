"""CPU checks of the C-ABI library: it loads, exports every symbol the
headers declare, and its host-built operator MPOs decode to the paper's
stencils and agree with the oracle's independently built MPOs."""
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2205_11990_amd", "libmpsvlasov.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB),
                                reason="HIP library not built (run __graft_entry__.build())")


def _declared():
    names = set()
    for h in ("mps_vlasov.h", "mps_blocks.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"\b(mpsb?_[a-z_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    declared = _declared()
    assert declared, "no declarations parsed"
    missing = declared - exported
    assert not missing, missing


def test_binding_signatures_cover_the_headers():
    from paper_2205_11990_amd import binding
    assert set(binding.EXPORTED) == _declared()
    binding.lib()  # loads without a GPU


def _dense(W):
    from oracle import mps
    return mps.mpo_to_matrix(W)


@pytest.mark.parametrize("L", [2, 3, 5, 7])
def test_library_operators_decode_to_stencils(L):
    from paper_2205_11990_amd import binding
    from oracle import mps
    N = 2 ** L
    h = 0.37
    Dx = _dense(binding.operator(0, L, 0.0, h))
    Dv = _dense(binding.operator(1, L, 0.0, h))
    G = _dense(binding.operator(2, L, 0.0, h))
    V = _dense(binding.operator(3, L, -2.0, h))
    ref = np.zeros((N, N))
    for o in range(N):
        ref[o, (o + 1) % N] += 0.5 / h
        ref[o, (o - 1) % N] -= 0.5 / h
    assert np.abs(Dx - ref).max() < 1e-13
    refv = np.zeros((N, N))
    for o in range(1, N - 1):
        refv[o, o + 1] += 0.5 / h
        refv[o, o - 1] -= 0.5 / h
    assert np.abs(Dv - refv).max() < 1e-13
    assert np.abs(V - np.diag(-2.0 + h * np.arange(N))).max() < 1e-13
    # G = Dx pinv(Laplacian) built from the oracle's printed MPOs
    Lap = mps.mpo_to_matrix(mps.mpo_d2_periodic(L, h))
    Dxo = mps.mpo_to_matrix(mps.mpo_d1_periodic(L, h))
    assert np.abs(G - Dxo @ np.linalg.pinv(Lap)).max() < 1e-12
    assert np.abs(G - _dense(mps.poisson_mpo(L, h))).max() < 1e-13


@pytest.mark.parametrize("L", [2, 3, 5, 7])
def test_library_upwind_operators_match_the_oracle(L):
    """The library's one-sided derivatives (exact carry automata, bond 3)
    equal the oracle's (printed stencils through TT-SVD), and its velocity
    split diag(max(v,0)), diag(min(v,0)) equals the grid values, for grids
    symmetric about 0 and not."""
    from paper_2205_11990_amd import binding
    from oracle import mps
    N = 2 ** L
    h = 0.37
    Db = _dense(binding.operator(4, L, 0.0, h))
    Df = _dense(binding.operator(5, L, 0.0, h))
    assert np.abs(Db - _dense(mps.mpo_d1_backward(L, h))).max() < 1e-12 / h
    assert np.abs(Df - _dense(mps.mpo_d1_forward(L, h))).max() < 1e-12 / h
    assert max(w.shape[3] for w in binding.operator(4, L, 0.0, h)) <= 3
    for v0, dv in ((-1.0, 2.0 / (N - 1)), (-0.3, 0.21), (0.5, 0.1), (-9.0, 0.1)):
        v = v0 + dv * np.arange(N)
        P = _dense(binding.operator(6, L, v0, dv))
        M = _dense(binding.operator(7, L, v0, dv))
        assert np.abs(P - np.diag(np.maximum(v, 0.0))).max() < 1e-12 * max(1.0, np.abs(v).max())
        assert np.abs(M - np.diag(np.minimum(v, 0.0))).max() < 1e-12 * max(1.0, np.abs(v).max())


def test_library_operator_bonds():
    from paper_2205_11990_amd import binding
    assert [w.shape[3] for w in binding.operator(0, 6, 0, 1.0)[:-1]] == [3] * 5
    assert [w.shape[3] for w in binding.operator(1, 6, 0, 1.0)[:-1]] == [5] * 5
    assert [w.shape[3] for w in binding.operator(3, 6, 0, 1.0)[:-1]] == [2] * 5


def test_qr_mode_and_batch_graph_arguments_are_rejected_without_a_gpu():
    """mpsb_qr_tall refuses a reflector-application mode other than 0 or 1
    and mpsb_batch_step_graph a NULL batch, before any device work."""
    import ctypes
    from paper_2205_11990_amd import binding
    L = binding.lib()
    fake = ctypes.c_void_p(8)  # never dereferenced: the checks come first
    assert L.mpsb_qr_tall(4, 4, fake, None, 2, None) == binding.MPS_EINVAL
    assert L.mpsb_qr_tall(4, 4, fake, None, -1, None) == binding.MPS_EINVAL
    assert L.mpsb_qr_tall(0, 4, fake, None, 0, None) == binding.MPS_EINVAL
    c, r = ctypes.c_int64(), ctypes.c_int64()
    assert L.mpsb_batch_step_graph(None, 1, ctypes.byref(c), ctypes.byref(r)) == binding.MPS_EINVAL
    assert "NULL" in L.mps_last_error().decode()


def test_invalid_arguments_are_rejected_without_a_gpu():
    from paper_2205_11990_amd import binding
    with pytest.raises(binding.MpsError) as e:
        binding.operator(9, 4, 0.0, 1.0)
    assert e.value.status == binding.MPS_EINVAL
    with pytest.raises(binding.MpsError):
        binding.operator(0, 1, 0.0, 1.0)
    import workloads as wl
    p = wl.landau_small().problem
    p.Lx = 20
    with pytest.raises(binding.MpsError):
        binding.workspace_bound(p)
    p = wl.two_stream().problem
    assert binding.workspace_bound(p) > 0


def test_workspace_bound_grows_with_the_problem():
    """The admission bound (host arithmetic only) grows with the grid and
    the bond cap, is larger for the interleaved ordering with an uncapped
    field bond, and leaves the per-request budget far below one GPU's HBM
    at the benchmarked size."""
    from paper_2205_11990_amd import binding
    import workloads as wl
    b = {}
    for L in (6, 8, 10, 12):
        for chi in (16, 64, 128):
            b[L, chi] = binding.workspace_bound(wl.two_stream(L=L, chi=chi, df_max=4).problem)
    for L in (6, 8, 10):
        for chi in (16, 64):
            assert b[L, chi] <= b[L + 2, chi]
            assert b[L, chi] <= b[L, 128]
    seq = wl.two_stream(L=10, chi=64, df_max=4, order=wl.ORDER_SEQ).problem
    full_df = wl.two_stream(L=10, chi=64, df_max=0).problem
    assert binding.workspace_bound(full_df) >= b[10, 64] >= binding.workspace_bound(seq)
    assert b[10, 64] < (4 << 30)


_BAD = [
    ("Lx", 1), ("Lv", 1), ("Lx", 15), ("Lv", 0), ("order", 5), ("order", -1),
    ("dt", 0.0), ("dt", -0.1), ("dt", float("nan")), ("chi_max", 0),
    ("level", 0), ("level", 6), ("df_max", -1), ("tol", -1e-12),
    ("tol", float("nan")), ("precision", 3), ("x_scheme", 2), ("cfl", -0.5),
    ("qm", float("inf")), ("nu", -0.01), ("nu", float("nan")),
    ("nu_vth", float("nan")), ("compression", 2),
]


@pytest.mark.parametrize("field,value", _BAD)
def test_every_parameter_check_rejects_without_a_gpu(field, value):
    """The admission bound runs the same parameter checks as state creation
    (host only), so each invalid field gives MPS_EINVAL here."""
    from paper_2205_11990_amd import binding
    import workloads as wl
    p = wl.landau_small().problem
    setattr(p, field, value)
    with pytest.raises(binding.MpsError) as e:
        binding.workspace_bound(p)
    assert e.value.status == binding.MPS_EINVAL


def test_parameter_checks_that_couple_fields():
    from paper_2205_11990_amd import binding
    import workloads as wl

    def rejected(p):
        with pytest.raises(binding.MpsError) as e:
            binding.workspace_bound(p)
        return e.value.status == binding.MPS_EINVAL

    p = wl.landau_small(L=4, Lv=5).problem
    for order in (1, 4):                   # interleaved orderings need Lx == Lv
        p.order = order
        assert rejected(p)
    p = wl.landau_small().problem
    p.x_max = p.x_min                      # empty intervals
    assert rejected(p)
    p = wl.landau_small().problem
    p.v_min = p.v_max + 1.0
    assert rejected(p)
    p = wl.landau_small().problem
    p.compression = 1                      # centre-first needs a sequential order
    for order in (1, 4):
        p.order = order
        assert rejected(p)
    p = wl.landau_small().problem
    p.dt = 0.0                             # no fixed dt needed with adaptive dt
    p.cfl = 0.5
    assert binding.workspace_bound(p) > 0
    # the smallest and largest grids of every ordering are accepted
    for L in (2, 14):
        for order in range(5):
            p = wl.landau_small().problem
            p.Lx = p.Lv = L
            p.order = order
            assert binding.workspace_bound(p) > 0
