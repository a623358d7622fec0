"""Continuous-batching server (la_serve_*) on the GPU.

* a request's factors are bitwise identical alone and in a mix of sizes and
  phases (every tile is computed the same way whatever shares the launch);
* requests overlap on the device (shared ticks) and are admitted by HBM
  footprint (a tight arena forces waiting, never overflow); the two size
  bands give the same bits as one band for all sizes;
* every result meets the polar tolerances and matches the FP64 oracle's H;
* many small requests in flight at once give the same bits for the same input;
* error paths: non-finite input fails alone, too-large and queue-full are
  rejected at submit, unknown and twice-polled ids are reported.
"""
import math
import time

import numpy as np
import pytest

import la_inputs
import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def la():
    import paper_2112_09017_amd as la
    la.lib()
    return la


def wait_all(srv, ids, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(ids):
        for i in ids:
            if i in out:
                continue
            r = srv.poll(i)
            if r is not None:
                out[i] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(ids) - len(out)} requests pending")
        time.sleep(0.001)
    return out


SIZES = [(128, 128, 1e-2), (192, 192, 1e-3), (320, 320, 1e-4), (640, 256, 1e-3),
         (512, 512, 1e-5), (256, 128, 1e-2)]


def cases():
    return [la_inputs.polar_case(m, n, lo, seeds=(900 + i, 910 + i, 920 + i))
            for i, (m, n, lo) in enumerate(SIZES)]


def test_mix_equals_alone_and_meets_tolerance(la):
    cs = cases()
    with la.Server(1 << 30, max_slots=16) as srv:
        ids = [srv.submit(c.A32) for c in cs]
        mix = wait_all(srv, ids)
        st = srv.stats()
    total_iters = sum(mix[i][3]["iters_precond"] + mix[i][3]["iters_ns"] for i in ids)
    print("stats", st, "total iterations", total_iters)
    assert st["completed"] == len(cs)
    assert st["ticks"] < total_iters          # requests shared ticks (overlap)
    for c, i in zip(cs, ids):
        status, U, H, info = mix[i]
        assert status == la.Status.OK
        with la.Server(1 << 30) as alone:
            j = alone.submit(c.A32)
            s2, U2, H2, info2 = wait_all(alone, [j])[j]
        assert np.array_equal(U, U2) and np.array_equal(H, H2), c.A32.shape
        assert info == info2
        A = c.A32.astype(np.float64)
        U64, H64 = U.astype(np.float64), H.astype(np.float64)
        n = U.shape[1]
        orth = np.linalg.norm(U64.T @ U64 - np.eye(n)) / math.sqrt(n)
        resid = np.linalg.norm(A - U64 @ H64) / np.linalg.norm(A)
        _, Ho, _ = oracle.polar(A)
        dh = np.linalg.norm(H64 - Ho) / np.linalg.norm(A)
        print(c.A32.shape, info, orth, resid, dh)
        assert orth <= TOL and resid <= TOL and dh <= TOL


def fp64_checks(A32, U, H, V, s):
    """Exact FP64 orthogonality, residual and ||H - V diag(s) V^T||_F / ||A||_F
    by torch products on the GPU (test tooling)."""
    import torch
    n = U.shape[1]
    Ad = torch.from_numpy(A32).to("cuda").double()
    Ud = torch.from_numpy(U).to("cuda").double()
    Hd = torch.from_numpy(H).to("cuda").double()
    G = Ud.t().contiguous() @ Ud
    G.diagonal().sub_(1.0)
    orth = torch.linalg.norm(G).item() / math.sqrt(n)
    nA = torch.linalg.norm(Ad).item()
    resid = torch.linalg.norm(Ad - Ud @ Hd).item() / nA
    sd = torch.from_numpy(s).to("cuda")
    dh = torch.linalg.norm(Hd - (V * sd[None, :]) @ V.t().contiguous()).item() / nA
    return orth, resid, dh


def test_large_tile_requests_mix_equals_alone(la):
    """N = 3072 and N = 4096 requests (cond 1e6 and 1e5) take the grouped
    kernels' 256 x 256 tiles (updates of both, the 4096 Grams too, at 6xBF16
    and 3xBF16); served among small requests they are bitwise the same as
    served alone, and meet the tolerances by exact FP64 checks."""
    import torch
    big = []
    for n, lo, seeds in ((3072, 1e-6, (990, 991, 992)), (4096, 1e-5, (993, 994, 995))):
        A, Q, s, V = la_inputs.polar_case_torch(n, n, lo, seeds)
        del Q
        big.append((A, s, V))
    torch.cuda.empty_cache()
    small = cases()[:4]
    with la.Server(8 << 30, max_slots=16) as srv:
        ids = [srv.submit(small[0].A32), srv.submit(big[0][0]), srv.submit(small[1].A32),
               srv.submit(big[1][0]), srv.submit(small[2].A32), srv.submit(small[3].A32)]
        mix = wait_all(srv, ids, timeout=300)
        st = srv.stats()
    assert st["completed"] == len(ids)
    # the big requests tick in the large band, the small ones in the small
    # band; one band for all of them gives the same bits
    inputs = [small[0].A32, big[0][0], small[1].A32, big[1][0], small[2].A32, small[3].A32]
    with la.Server(8 << 30, max_slots=16, bands=1) as one:
        ids1 = [one.submit(A) for A in inputs]
        mix1 = wait_all(one, ids1, timeout=300)
    for i, i1 in zip(ids, ids1):
        assert mix[i][0] == mix1[i1][0] == la.Status.OK
        assert np.array_equal(mix[i][1], mix1[i1][1]) and np.array_equal(mix[i][2], mix1[i1][2])
        assert mix[i][3] == mix1[i1][3]
    for (A, s, V), i in zip(big, (ids[1], ids[3])):
        status, U, H, info = mix[i]
        assert status == la.Status.OK
        with la.Server(8 << 30) as alone:
            j = alone.submit(A)
            s2, U2, H2, info2 = wait_all(alone, [j], timeout=300)[j]
        assert np.array_equal(U, U2) and np.array_equal(H, H2), A.shape
        assert info == info2
        assert np.array_equal(H, H.T)
        orth, resid, dh = fp64_checks(A, U, H, V, s)
        print(A.shape, info, f"orth={orth:.2e} resid={resid:.2e} dH={dh:.2e}")
        assert orth <= TOL and resid <= TOL and dh <= TOL


def test_busy_tick_large_tiles_equal_alone(la):
    """Seven 2304 x 2304 requests in flight need 7 x 81 = 567 large tiles, more
    than twice the CUs, so their ticks run every product on 256 x 256 tiles; one
    of them served alone takes 128 x 128 tiles (81 large ones would leave most
    CUs idle).  The tile class must not change a bit."""
    import torch
    cs = [la_inputs.polar_case_torch(2304, 2304, 10.0 ** -(2 + i % 4), (1000 + 3 * i, 1001 + 3 * i,
                                                                       1002 + 3 * i))
          for i in range(7)]
    torch.cuda.empty_cache()
    with la.Server(4 << 30, max_slots=16) as srv:
        ids = [srv.submit(c[0]) for c in cs]
        mix = wait_all(srv, ids, timeout=300)
    for k in (0, 6):
        A, _, s, V = cs[k]
        with la.Server(4 << 30) as alone:
            j = alone.submit(A)
            s2, U2, H2, info2 = wait_all(alone, [j], timeout=300)[j]
        status, U, H, info = mix[ids[k]]
        assert status == s2 == la.Status.OK
        assert np.array_equal(U, U2) and np.array_equal(H, H2)
        assert info == info2
        orth, resid, dh = fp64_checks(A, U, H, V, s)
        print(k, info, f"orth={orth:.2e} resid={resid:.2e} dH={dh:.2e}")
        assert orth <= TOL and resid <= TOL and dh <= TOL


def test_tight_arena_admission(la):
    """An arena that holds two 512 x 512 requests at a time still serves six."""
    cs = [la_inputs.polar_case(512, 512, 1e-3, seeds=(930 + i, 940 + i, 950 + i))
          for i in range(6)]
    reserve = 8 << 20                                   # server descriptors
    per = 4 * (3 * 512 * 512 + 512 * 512) + (1 << 16)   # one 512 x 512 request
    per_big = 4 * (3 * 2048 * 2048 + 2048 * 2048) + (1 << 16)
    # the 2048 request takes most of the arena, so the small ones wait for it
    arena = reserve + per_big + per + (1 << 20)
    with la.Server(arena, max_slots=8) as srv:
        big = la_inputs.polar_case(2048, 2048, 1e-2, seeds=(960, 961, 962))
        ids = [srv.submit(big.A32)] + [srv.submit(c.A32) for c in cs]
        out = wait_all(srv, ids, timeout=300)
        st = srv.stats()
    print(st, "arena", arena, "2048 footprint", per_big)
    assert st["completed"] == 7
    assert st["arena_high_water"] <= arena
    for i in ids:
        assert out[i][0] == la.Status.OK


def test_many_small_requests_in_flight(la):
    """1200 requests of 64 x 64 submitted back to back on 4096 slots, so that
    each grouped launch holds dozens of problems laid out over the XCDs (with
    empty padding items).  Every request completes, 30 copies of each of 40
    inputs give the same bits wherever and whenever they ran, and each
    distinct result meets the polar tolerances."""
    distinct = [la_inputs.polar_case(64, 64, 10.0 ** -(1 + i % 4),
                                     seeds=(970 + i, 1070 + i, 1170 + i)) for i in range(40)]
    reps = 30
    peak_active = 0
    with la.Server(512 << 20, max_slots=4096) as srv:
        ids = [srv.submit(distinct[k % 40].A32) for k in range(40 * reps)]
        out = {}
        t0 = time.time()
        while len(out) < len(ids):
            peak_active = max(peak_active, srv.stats()["active"])
            for i in ids:
                if i not in out:
                    r = srv.poll(i)
                    if r is not None:
                        out[i] = r
            assert time.time() - t0 < 100, f"{len(ids) - len(out)} requests pending"
            time.sleep(0.001)
        st = srv.stats()
    print(st, "peak active", peak_active)
    assert st["completed"] == len(ids) and st["failed"] == 0
    for k, i in enumerate(ids):
        status, U, H, info = out[i]
        assert status == la.Status.OK
        j = ids[k % 40]
        assert np.array_equal(U, out[j][1]) and np.array_equal(H, out[j][2]), k
    for c, i in zip(distinct, ids[:40]):
        A = c.A32.astype(np.float64)
        U64, H64 = out[i][1].astype(np.float64), out[i][2].astype(np.float64)
        orth = np.linalg.norm(U64.T @ U64 - np.eye(64)) / 8.0
        resid = np.linalg.norm(A - U64 @ H64) / np.linalg.norm(A)
        assert orth <= TOL and resid <= TOL, (orth, resid)


def test_error_paths(la):
    good = la_inputs.polar_case(128, 128, 1e-2, seeds=(970, 971, 972))
    for bands in (-1, 3):
        with pytest.raises(la.LAError) as e:
            la.Server(256 << 20, bands=bands)
        assert e.value.status == la.Status.INVALID_ARG
    with la.Server(256 << 20, max_slots=4, max_queue=3) as srv:
        with pytest.raises(la.LAError) as e:
            srv.submit(np.ones((8192, 8192), np.float32))
        assert e.value.status == la.Status.TOO_LARGE
        with pytest.raises(la.LAError) as e:
            srv.submit(np.ones((3, 5), np.float32))
        assert e.value.status == la.Status.SHAPE
        bad = srv.submit(np.full((64, 64), np.nan, np.float32))
        ok = srv.submit(good.A32)
        out = wait_all(srv, [bad, ok])
        assert out[bad][0] == la.Status.NONFINITE
        assert out[ok][0] == la.Status.OK
        with pytest.raises(la.LAError) as e:
            srv.poll(ok)                      # already collected
        assert e.value.status == la.Status.UNKNOWN_REQUEST
        capped = srv.submit(good.A32, max_iter=1)
        r = wait_all(srv, [capped])[capped]
        assert r[0] == la.Status.NOT_CONVERGED and r[3]["iters_ns"] == 1
    with la.Server(256 << 20, max_slots=1, max_queue=2) as srv:
        big = la_inputs.polar_case(1024, 1024, 1e-2, seeds=(973, 974, 975))
        ids = []
        with pytest.raises(la.LAError) as e:
            for _ in range(64):
                ids.append(srv.submit(big.A32))
        assert e.value.status == la.Status.QUEUE_FULL
        assert srv.poll(ids[-1]) is None      # still pending (NOT_READY)
    # leaving the with-block destroyed the server with requests pending


def test_matches_la_polar_tolerances_for_tall(la):
    c = la_inputs.polar_case(1500, 300, 1e-4, seeds=(980, 981, 982))
    with la.Server(1 << 30) as srv:
        i = srv.submit(c.A32)
        st, U, H, info = wait_all(srv, [i])[i]
    A = c.A32.astype(np.float64)
    U, H = U.astype(np.float64), H.astype(np.float64)
    orth = np.linalg.norm(U.T @ U - np.eye(300)) / math.sqrt(300)
    resid = np.linalg.norm(A - U @ H) / np.linalg.norm(A)
    print(info, orth, resid)
    assert st == la.Status.OK and orth <= TOL and resid <= TOL
