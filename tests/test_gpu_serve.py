"""Continuous-batching server: results are the same alone and in the mix; work overlaps on the device;
admission, failure isolation and cancellation behave."""
import numpy as np
import pytest

import oracle
import paper_1105_5481_amd as kpm
from paper_1105_5481_amd import workloads as wl
from paper_1105_5481_amd.serve import KPMRequest, Server, latency_stats
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _requests():
    """Mixed sizes (all larger than one workgroup's LDS, so they run through the batch), kinds and
    arrival times in chunks; request k arrives while earlier ones are still in flight."""
    reqs = []
    specs = [
        (wl.square_lattice(96, W=1.0, seed=1), 256, 8, wl.VEC_RADEMACHER, 0),
        (wl.spin_cubic_lattice(16, seed=2), 128, 4, wl.VEC_PHASE, 0),
        (wl.cubic_lattice(20, W=2.0, seed=3), 200, 5, wl.VEC_RADEMACHER, 1),
        (wl.square_lattice(80, W=2.0, seed=4), 64, 9, wl.VEC_PHASE, 2),
        (wl.spin_cubic_lattice(14, seed=5), 300, 6, wl.VEC_PHASE, 3),
        (wl.lattice_to_csr(wl.square_lattice(70, W=1.0, seed=6)), 96, 7, wl.VEC_RADEMACHER, 4),
        (wl.Lattice(dim=2, L=(50, 60, 1), t=1.0, hop=wl.HOP_SPIN,
                    spinor=wl.spinor_of(*wl.spins_uniform(3000, 7))), 150, 5, wl.VEC_PHASE, 6),
        (wl.square_lattice(128, W=0.5, seed=8), 512, 4, wl.VEC_RADEMACHER, 9),
        # temporally blocked 2D solves (4-step and 3-step passes, chunk remainders)
        (wl.Lattice(dim=2, L=(300, 40, 1), t=1.0, onsite=wl.anderson_onsite(12000, 2.0, 9)), 270, 8,
         wl.VEC_RADEMACHER, 1),
        (wl.Lattice(dim=2, L=(200, 30, 1), t=1.0, hop=wl.HOP_SPIN,
                    spinor=wl.spinor_of(*wl.spins_uniform(6000, 10))), 180, 6, wl.VEC_PHASE, 2),
        (wl.Lattice(dim=2, L=(260, 20, 1), t=1.0, onsite=wl.anderson_onsite(5200, 1.0, 11)), 77, 36,
         wl.VEC_RADEMACHER, 5),
    ]
    for k, (op, M, R, vec, arr) in enumerate(specs):
        reqs.append(KPMRequest(op=op, M=M, R=R, vec=vec, seed=100 + k, instance=k, arrival=arr, rid=k))
    return reqs


def _solo(req, prec, a, b):
    h = kpm.Hamiltonian(req.op, a, b, prec)
    mu = kpm.moments(h, req.M, req.R, req.vec, req.seed, req.instance).cpu().numpy()
    h.free()
    return mu


def test_served_equals_solo_and_overlaps():
    reqs = _requests()
    srv = Server(prec=kpm.F32, max_active=8, chunk=16)
    res = srv.run(reqs, clock="chunks")
    srv.close()
    assert [r.status for r in res] == ["ok"] * len(reqs)
    # the last three run temporally blocked passes inside the shared launches
    for req in reqs[-3:]:
        h = kpm.Hamiltonian(req.op, 4.5, 0.0, kpm.F32)
        s = kpm.Solve(h, req.M, req.R, req.vec, 1, 0)
        assert kpm.lib().kpm_solve_mode(s._s) == 3
        s.close()
        h.free()
    for req, r in zip(reqs, res):
        solo = _solo(req, kpm.F32, r.a, r.b)
        assert np.array_equal(r.mu, solo), req.rid
        assert np.all(np.isfinite(r.rho))
    # FP32 against the oracle for two of them
    for k in (0, 4):
        ref = gu.oracle_moments(reqs[k].op, res[k].a, res[k].b, reqs[k].M, reqs[k].R, reqs[k].vec, reqs[k].seed,
                                reqs[k].instance)
        gu.assert_fp32(res[k].mu, ref, f"served request {k}")
    # work of different requests shared launches, and requests were admitted while others ran
    assert srv.max_concurrent >= 3
    assert any(len(rids) >= 2 for _, rids in srv.chunk_log)
    late = [r for r in res if any(o.t_admit < r.t_admit < o.t_done for o in res if o.rid != r.rid)]
    assert late, "no request was admitted while another was in flight"


def test_fp64_fcfs_matches_oracle():
    reqs = _requests()[:3]
    srv = Server(prec=kpm.F64, max_active=1, chunk=64)
    res = srv.run(reqs, clock="chunks")
    srv.close()
    for req, r in zip(reqs, res):
        assert r.status == "ok"
        ref = gu.oracle_moments(req.op, r.a, r.b, req.M, req.R, req.vec, req.seed, req.instance)
        gu.assert_fp64(r.mu, ref, f"fcfs fp64 request {req.rid}")
    assert srv.max_concurrent == 1


def test_admission_rejects_oversize_and_isolates_failures():
    reqs = _requests()[:4]
    big = KPMRequest(op=wl.square_lattice(2048, W=1.0, seed=9), M=64, R=64, arrival=0, rid=10)
    lo, hi = oracle.gershgorin_lattice(2, (96, 96), 1.0, 0, reqs[0].op.onsite, None)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    bad = KPMRequest(op=reqs[0].op, M=256, R=8, seed=5, scale=(0.45 * a, b), arrival=1, rid=11)
    # a CSR whose last column index is out of range: the device structure check rejects it
    csr = wl.lattice_to_csr(wl.square_lattice(10, W=1.0, seed=3))
    col = csr.col.copy()
    col[-1] = csr.n
    broken = KPMRequest(op=wl.CSR(n=csr.n, row_ptr=csr.row_ptr, col=col, val_re=csr.val_re), M=32, R=4, arrival=1,
                        rid=12)
    srv = Server(prec=kpm.F32, max_active=8, chunk=16, hbm_budget=256 << 20)
    res = srv.run(reqs + [big, bad, broken], clock="chunks")
    srv.close()
    st = {r.rid: r.status for r in res}
    assert st[10] == "oom"
    assert st[11] == "bounds"
    assert st[12] == "error"
    for req in reqs:
        r = [x for x in res if x.rid == req.rid][0]
        assert r.status == "ok"
        assert np.array_equal(r.mu, _solo(req, kpm.F32, r.a, r.b))


def test_cancel():
    reqs = _requests()[:3]
    srv = Server(prec=kpm.F32, max_active=4, chunk=4)
    for r in reqs:
        srv.submit(r)
    srv.step()
    srv.cancel(1)
    while srv.busy():
        srv.step()
    import torch
    torch.cuda.synchronize()
    srv._retire()
    srv.close()
    assert srv.results[1].status == "cancelled"
    assert srv.results[0].status == "ok" and srv.results[2].status == "ok"


def test_many_retire_together():
    """Several solves finishing in the same chunk retire together."""
    reqs = [KPMRequest(op=wl.square_lattice(90, W=1.0, seed=k), M=64, R=8, seed=k, arrival=0, rid=k) for k in range(6)]
    srv = Server(prec=kpm.F32, max_active=8, chunk=64)
    res = srv.run(reqs, clock="chunks")
    srv.close()
    assert [r.status for r in res] == ["ok"] * 6
    for req, r in zip(reqs, res):
        assert np.array_equal(r.mu, _solo(req, kpm.F32, r.a, r.b))


def test_wall_clock_trace_latency():
    reqs = _requests()
    for k, r in enumerate(reqs):
        r.arrival = 0.002 * k
    srv = Server(prec=kpm.F32, max_active=8, chunk=16)
    res = srv.run(reqs, clock="wall")
    srv.close()
    st = latency_stats(res)
    print("  latency", st)
    assert st["n"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] > 0


def test_lanczos_scaled_requests():
    """Requests that ask for the Lanczos interval get a tighter scale than Gershgorin and the same
    moments as a solo solve on that scale."""
    reqs = [KPMRequest(op=wl.spin_cubic_lattice(18, seed=90 + k), M=128, R=4, vec=wl.VEC_PHASE, seed=k, arrival=0,
                       rid=k, bounds="lanczos", lanczos_k=80) for k in range(3)]
    srv = Server(prec=kpm.F32, max_active=4, chunk=32)
    res = srv.run(reqs, clock="chunks")
    srv.close()
    for req, r in zip(reqs, res):
        assert r.status == "ok"
        lo, hi = oracle.gershgorin_lattice(3, (18, 18, 18), 1.0, 1, None, req.op.spinor)
        assert r.a < oracle.scale_from_bounds(lo, hi, 0.01)[0]
        assert np.array_equal(r.mu, _solo(req, kpm.F32, r.a, r.b))
