"""la_polar_noalloc (the allocation-free polar) against la_polar through the C
ABI: bitwise the same U, H and info on two calls in a row, the second with a
smaller input (the static workspace keeps the first call's contents), a tall
input whose Gram takes split-K slices, and the rejection of an input whose
workspace exceeds the static buffer (U untouched)."""
import ctypes

import numpy as np
import pytest
import torch

import la_inputs

pytestmark = pytest.mark.gpu

NOALLOC_BYTES = 64 << 20    # LA_POLAR_NOALLOC_BYTES in include/la.h


@pytest.fixture(scope="module")
def la():
    import paper_2112_09017_amd as la
    la.lib()
    return la


def both(la, A32, **opts):
    Ad = torch.from_numpy(np.ascontiguousarray(A32)).to("cuda")
    U1, H1, i1 = la.polar(Ad, **opts)
    U2, H2, i2 = la.polar_noalloc(Ad, **opts)
    torch.cuda.synchronize()
    return (U1.cpu().numpy(), H1.cpu().numpy(), i1), (U2.cpu().numpy(), H2.cpu().numpy(), i2)


@pytest.mark.parametrize("opts", [{}, dict(prec_precond=1, prec_ns=1, prec_h=1)],
                         ids=["auto", "fp32"])
def test_noalloc_equals_polar_twice_then_smaller(la, opts):
    for shape, seeds in (((700, 300), (61, 62, 63)), ((256, 130), (64, 65, 66)),
                         ((5000, 96), (67, 68, 69))):
        case = la_inputs.polar_case(shape[0], shape[1], 1e-3, seeds=seeds)
        (U1, H1, i1), (U2, H2, i2) = both(la, case.A32, **opts)
        assert np.array_equal(U1, U2) and np.array_equal(H1, H2), shape
        assert i1 == i2, shape
        assert np.isfinite(U2).all()


def test_noalloc_rejects_inputs_beyond_the_static_buffer(la):
    n = 2304
    assert la.polar_workspace_size(n, n) > NOALLOC_BYTES
    Ad = torch.zeros((n, n), device="cuda")
    Ad.diagonal().fill_(1.0)
    U = torch.full((n, n), 7.0, device="cuda")
    with pytest.raises(la.LAError) as ei:
        la.polar_noalloc(Ad, U=U)
    assert ei.value.status == la.Status.TOO_LARGE
    torch.cuda.synchronize()
    assert bool((U == 7.0).all())
    # a size that fits still runs afterwards
    case = la_inputs.polar_case(128, 128, 1e-2, seeds=(70, 71, 72))
    (U1, H1, _), (U2, H2, _) = both(la, case.A32)
    assert np.array_equal(U1, U2) and np.array_equal(H1, H2)
