"""The allocation-free truncated SVD (mpsb_svd_truncate_noalloc: every
workspace in a fixed device array) against the allocating entry point
(mpsb_svd_truncate) on the same inputs: two calls in a row, the second
smaller, then a rejected oversize shape."""
import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2205_11990_amd import binding
    binding.lib()
    return binding


def _both(B, X, cap, tol):
    import torch
    m, c = X.shape
    kmax = min(m, c, cap) if cap > 0 else min(m, c)
    Vt0, US0, sig0, disc0 = B.svd_truncate(X, cap=cap, tol=tol)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Vt = torch.empty(kmax * c, dtype=torch.float64, device="cuda")
    US = torch.empty(m * kmax, dtype=torch.float64, device="cuda")
    sig = torch.empty(min(m, c), dtype=torch.float64, device="cuda")
    D, disc = B.svd_truncate_noalloc(Xd, Vt, US, sig, cap=cap, tol=tol)
    return (Vt0.cpu().numpy(), US0.cpu().numpy(), sig0.cpu().numpy(), disc0,
            Vt[:D * c].view(D, c).cpu().numpy(), US[:m * D].view(m, D).cpu().numpy(),
            sig.cpu().numpy(), disc, D)


@pytest.mark.parametrize("shapes", [[(1024, 128, 64, 0.0), (300, 96, 0, 1e-10)],
                                    [(200, 256, 128, 0.0), (96, 700, 0, 1e-8)]])
def test_noalloc_svd_equals_allocating_entry_point(B, shapes):
    for m, c, cap, tol in shapes:
        _say("noalloc svd %d x %d cap %d tol %g" % (m, c, cap, tol))
        X = wl.random_matrix(m, c, seed=7 * m + c, decay=10)
        Vt0, US0, s0, d0, Vt, US, s, d, D = _both(B, X, cap, tol)
        assert Vt.shape == Vt0.shape and US.shape == US0.shape and D == Vt0.shape[0]
        scale = s0[0]
        assert np.abs(s - s0).max() <= 1e-13 * scale
        assert np.abs(Vt - Vt0).max() <= 1e-12
        assert np.abs(US - US0).max() <= 1e-12 * scale
        assert abs(d - d0) <= 1e-14 + 1e-12 * d0
        # and the factorisation itself: the best rank-D approximation
        U, S, W = np.linalg.svd(X, full_matrices=False)
        best = (U[:, :D] * S[:D]) @ W[:D]
        assert np.abs(US @ Vt - best).max() <= 1e-12 * S[0] * np.sqrt(max(m, c))


def test_noalloc_svd_rejects_shapes_beyond_its_scratch(B):
    import torch
    _say("noalloc svd oversize")
    X = torch.zeros((3000, 64), dtype=torch.float64, device="cuda")
    Vt = torch.empty(64 * 64, dtype=torch.float64, device="cuda")
    US = torch.empty(3000 * 64, dtype=torch.float64, device="cuda")
    sig = torch.empty(64, dtype=torch.float64, device="cuda")
    with pytest.raises(B.MpsError) as e:
        B.svd_truncate_noalloc(X, Vt, US, sig)
    assert e.value.status == B.MPS_EINVAL
