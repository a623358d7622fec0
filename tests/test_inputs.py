"""Seeded input generators: determinism and the structure the workloads need (no GPU)."""
import numpy as np

import la_inputs


def test_seeded_and_deterministic():
    a = la_inputs.gaussian((17, 9), 5)
    b = la_inputs.gaussian((17, 9), 5)
    assert a.dtype == np.float32 and np.array_equal(a, b)
    assert not np.array_equal(a, la_inputs.gaussian((17, 9), 6))


def test_haar_and_column_orthonormal():
    q = la_inputs.haar(50, 7)
    assert np.abs(q.T @ q - np.eye(50)).max() < 1e-13
    c = la_inputs.column_orthonormal(120, 30, 8)
    assert np.abs(c.T @ c - np.eye(30)).max() < 1e-13
    # sign convention: R of the QR of the same Gaussian has a positive diagonal
    g = la_inputs.rng(8).standard_normal(size=(120, 30))
    r = c.T @ g
    assert np.all(np.diag(r) > 0)


def test_singular_values_pinned_endpoints():
    s = la_inputs.singular_values(64, 1e-6, 9)
    assert s[0] == 1.0 and s[-1] == 1e-6
    assert np.all(np.diff(s) <= 0) and s.min() >= 1e-6


def test_polar_case_construction():
    case = la_inputs.polar_case(40, 24, 1e-3, seeds=(1, 2, 3))
    sv = np.linalg.svd(case.A64, compute_uv=False)
    assert abs(sv.max() - 1.0) < 1e-13 and abs(sv.min() - 1e-3) < 1e-15
    assert case.A32.dtype == np.float32 and case.A32.shape == (40, 24)
    U = case.U_exact
    assert np.abs(U.T @ U - np.eye(24)).max() < 1e-13


def test_serve_stream_and_sizes():
    n = la_inputs.serve_sizes(2000, 4)
    assert n.min() >= 128 and n.max() <= 4096 and np.all(n % 64 == 0)
    st = la_inputs.serve_stream(100.0, 10.0, 5, pool_size=8)
    assert 800 < len(st) < 1200
    assert all(0 <= i < 8 for _, i in st)
    ts = [t for t, _ in st]
    assert ts == sorted(ts)
