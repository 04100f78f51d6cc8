"""Admission rule of the solve server (CPU: pure function of the library)."""
import os

import pytest

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1811_11558_amd", "libfvim.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def test_first_request_that_fits_is_admitted():
    from paper_1811_11558_amd import admit_index
    assert admit_index([10, 5, 3], budget=12, in_use=8) == 2     # small ones pass a waiting large one
    assert admit_index([3, 5, 10], budget=12, in_use=8) == 0     # submission order otherwise
    assert admit_index([10, 20], budget=12, in_use=0) == 0
    assert admit_index([10, 20], budget=12, in_use=3) == -1      # nothing fits until memory frees
    assert admit_index([], budget=12, in_use=0) == -1
    assert admit_index([12], budget=12, in_use=0) == 0           # exactly the budget


def test_footprint_grows_with_grid():
    from paper_1811_11558_amd import request_bytes
    g = lambda n, nz: dict(nx=n, ny=n, nz=nz, lx=1.0, ly=1.0, lz=0.25)
    sizes = [request_bytes(g(n, nz)) for n, nz in ((64, 32), (128, 64), (256, 64), (512, 96))]
    assert all(a < b for a, b in zip(sizes, sizes[1:]))
    # the state and work arrays of a solve: at least 56 float64 tensors-worth per voxel
    assert sizes[-1] >= 56 * 8 * 512 * 512 * 96


def test_newton_krylov_footprint_counts_its_basis():
    """Solver 2 keeps krylov_dim + 2 strain fields (6 float64 per voxel each)
    beyond what the other solvers need; the others ignore krylov_dim."""
    from paper_1811_11558_amd import EPOptions, request_bytes
    g = dict(nx=128, ny=128, nz=64, lx=1.0, ly=1.0, lz=0.25)
    V = 128 * 128 * 64
    base = request_bytes(g, opts=EPOptions(solver=0))
    assert request_bytes(g, opts=EPOptions(solver=0, krylov_dim=30)) == base
    for m, md in ((0, 20), (5, 5), (30, 30)):
        extra = request_bytes(g, opts=EPOptions(solver=2, krylov_dim=m)) - base
        basis = 8 * 6 * V * (md + 2)
        assert basis <= extra < basis + (1 << 20), (m, extra, basis)


def test_friction_footprint_counts_its_workspace():
    """mu_f > 0 adds the tangential contact workspace (9 surface fields and
    two 2-plane spectra) to a request's footprint."""
    from paper_1811_11558_amd import EPOptions, request_bytes
    g = dict(nx=256, ny=256, nz=32, lx=1.0, ly=1.0, lz=0.25)
    base = request_bytes(g, opts=EPOptions())
    extra = request_bytes(g, opts=EPOptions(mu_f=0.3, q_ratio=(0.5, 0.0))) - base
    assert 9 * 8 * 256 * 256 <= extra < 9 * 8 * 256 * 256 + 16 * 129 * 256 * 16 + (1 << 20)
