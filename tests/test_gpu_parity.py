"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle, element by element.

Sizes are chosen so the oracle finishes in seconds while the GPU launch still spans several
tiles with a ragged tail (sites x 16-byte chunks not a multiple of the tile).
"""
import numpy as np
import pytest

import oracle
import paper_1105_5481_amd as kpm
from paper_1105_5481_amd import workloads as wl
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available()
    kpm.lib()
    oracle.build()
    yield


def _cases():
    c = []
    c.append(("paper_cube_10", wl.cubic_lattice(10), 128, 4, wl.VEC_RADEMACHER))
    c.append(("square_37x19_phase_oddM", wl.Lattice(dim=2, L=(37, 19, 1), t=1.0,
                                                    onsite=wl.anderson_onsite(37 * 19, 2.0, 3)), 97, 5, wl.VEC_PHASE))
    c.append(("spin3d_12x10x6_phase", wl.spin_cubic_lattice(6, seed=4), 64, 3, wl.VEC_PHASE))
    lat = wl.spin_cubic_lattice(7, seed=5)
    lat.onsite = wl.anderson_onsite(7 ** 3, 1.0, 5)
    c.append(("spin3d_7_onsite_pm1", lat, 80, 6, wl.VEC_RADEMACHER))
    th, ph = wl.spins_uniform(16 * 9, 6)
    c.append(("spin2d_16x9_pm1", wl.Lattice(dim=2, L=(16, 9, 1), t=0.8, hop=wl.HOP_SPIN, spinor=wl.spinor_of(th, ph),
                                            theta=th, phi=ph), 70, 7, wl.VEC_RADEMACHER))
    c.append(("square_extent1_self_loop", wl.Lattice(dim=2, L=(5, 1, 1), t=1.0, onsite=wl.anderson_onsite(5, 1.0, 7)),
              40, 3, wl.VEC_RADEMACHER))
    c.append(("cube_2x3x4_extent2", wl.Lattice(dim=3, L=(2, 3, 4), t=1.1, onsite=wl.anderson_onsite(24, 1.0, 8)),
              33, 2, wl.VEC_PHASE))
    c.append(("csr_from_lattice", wl.lattice_to_csr(wl.square_lattice(24, W=1.5, seed=9)), 60, 4, wl.VEC_RADEMACHER))
    c.append(("csr_random_complex", wl.random_hermitian_csr(300, 8, seed=10), 50, 3, wl.VEC_PHASE))
    c.append(("csr_random_real_phase", wl.random_hermitian_csr(257, 6, seed=11, complex_values=False), 41, 5,
              wl.VEC_PHASE))
    c.append(("unit_trace_6x6", wl.square_lattice(6, W=2.0, seed=12), 50, 36, wl.VEC_UNIT))
    for M in (1, 2, 3):
        c.append((f"tiny_M{M}", wl.square_lattice(9, W=1.0, seed=13), M, 3, wl.VEC_RADEMACHER))
    c.append(("square_1x1_all_self", wl.Lattice(dim=2, L=(1, 1, 1), t=1.0, onsite=np.array([0.3])), 20, 2,
              wl.VEC_RADEMACHER))
    c.append(("spin3d_5_R1_phase", wl.spin_cubic_lattice(5, seed=14), 30, 1, wl.VEC_PHASE))
    c.append(("csr_empty_rows", _csr_with_empty_rows(), 40, 3, wl.VEC_PHASE))
    return c


def _csr_with_empty_rows():
    """A 64 x 64 complex Hermitian matrix acting on 50 of the indices; the other 14 rows (and
    columns) hold no entries at all."""
    g = np.random.default_rng(15)
    n, live = 64, np.sort(g.choice(64, size=50, replace=False))
    A = np.zeros((n, n), complex)
    for i in live:
        for j in g.choice(live, size=4, replace=False):
            v = complex(g.normal(), g.normal() if i != j else 0.0)
            A[i, j] += v
            A[j, i] += np.conj(v)
    rows, cols = np.nonzero(A)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    row_ptr = np.zeros(n + 1, np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    vals = A[rows, cols]
    return wl.CSR(n=n, row_ptr=row_ptr, col=cols.astype(np.int32), val_re=np.ascontiguousarray(vals.real),
                  val_im=np.ascontiguousarray(vals.imag))


CASES = _cases()


# execution paths: one workgroup with the vectors in LDS (small), one-step march kernels, several
# steps per pass (temporal blocking: 2D and 3D lattices), flat kernels
PATHS = {"small": dict(small=1), "march": dict(small=0, march=1, tblock=0),
         "blocked": dict(small=0, march=1, tblock=-1, tb3=1), "flat": dict(small=0, march=0)}


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fp64_and_fp32_match_oracle(case, path):
    name, op, M, R, vec = case
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    ref = gu.oracle_moments(op, a, b, M, R, vec, seed=777, instance=1)
    with kpm.launch_settings(**PATHS[path]):
        g64 = gu.gpu_moments(op, a, b, kpm.F64, M, R, vec, seed=777, instance=1)
        gu.assert_fp64(g64, ref, f"{name} [{path}]")
        g32 = gu.gpu_moments(op, a, b, kpm.F32, M, R, vec, seed=777, instance=1)
        gu.assert_fp32(g32, ref, f"{name} [{path}]")


@pytest.mark.parametrize("path", list(PATHS))
def test_config1_full_fp64(path):
    """2D 32x32, t=1, on-site uniform[-0.5, 0.5], Gershgorin bounds, M=256, R=8 +-1 vectors, and its
    Jackson DoS on 1024 Chebyshev points."""
    import torch
    cfg = wl.config1()
    op = cfg["lattice"]
    lo, hi = gu.oracle_bounds(op)
    glo, ghi = kpm.gershgorin(op)
    assert (glo, ghi) == (lo, hi)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    ref = gu.oracle_moments(op, a, b, cfg["M"], cfg["R"], cfg["vec"], cfg["seed"])
    with kpm.launch_settings(**PATHS[path]):
        g = gu.gpu_moments(op, a, b, kpm.F64, cfg["M"], cfg["R"], cfg["vec"], cfg["seed"])
        g32 = gu.gpu_moments(op, a, b, kpm.F32, cfg["M"], cfg["R"], cfg["vec"], cfg["seed"])
    gu.assert_fp64(g, ref, f"config1 [{path}]")
    gu.assert_fp32(g32, ref, f"config1 f32 [{path}]")
    assert g[0] == 1.0
    om_ref, rho_ref = oracle.dos(ref, cfg["K"], a, b)
    om, rho = kpm.dos(torch.from_numpy(g).cuda(), cfg["K"], a, b)
    assert np.abs(rho.cpu().numpy() - rho_ref).max() <= 1e-12 * np.abs(rho_ref).max()


@pytest.mark.parametrize("vec", [0, 1, 2])
def test_start_vectors_match_oracle(vec):
    N, R, seed, inst = 1000, 13, 4242, 5
    ref = oracle.start_vectors(vec, seed, inst, N, R).T              # (N, R) complex
    g = kpm.start_vectors(vec, True, seed, inst, N, R).cpu().numpy()
    gz = g[..., 0] + 1j * g[..., 1]
    assert np.array_equal(gz, ref)


def test_gershgorin_matches_oracle():
    ops = [wl.square_lattice(33, W=1.0, seed=1), wl.cubic_lattice(9, W=0.5, seed=2),
           wl.spin_cubic_lattice(11, seed=3), wl.random_hermitian_csr(200, 6, seed=4)]
    for op in ops:
        lo, hi = gu.oracle_bounds(op)
        glo, ghi = kpm.gershgorin(op)
        if getattr(op, "hop", 0) == wl.HOP_REAL and not isinstance(op, wl.CSR):
            assert (glo, ghi) == (lo, hi)
        else:
            assert abs(glo - lo) <= 4e-16 * abs(lo) and abs(ghi - hi) <= 4e-16 * abs(hi)


def test_launch_shape_does_not_change_fp64_result():
    op = wl.spin_cubic_lattice(9, seed=21)
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    outs = []
    for kw in [dict(max_blocks=2048), dict(max_blocks=8), dict(march_items=1), dict(march_items=100000),
               dict(march=0, elems_per_thread=4), dict(march=0, elems_per_thread=4, max_blocks=8),
               dict(march=0, elems_per_thread=1), dict(alternate=0), dict(xcd_split=1), dict(xcd_split=3),
               dict(march_items=100000, xcd_split=2, alternate=1), dict(streaming=0), dict(streaming=1)]:
        with kpm.launch_settings(**kw):
            outs.append(gu.gpu_moments(op, a, b, kpm.F64, 60, 5, wl.VEC_PHASE, seed=3))
    assert np.array_equal(outs[0], outs[1])              # same work items, different grid: bitwise
    assert np.array_equal(outs[4], outs[5])
    ref = gu.oracle_moments(op, a, b, 60, 5, wl.VEC_PHASE, seed=3)
    for o in outs:
        gu.assert_fp64(o, ref, "launch shape")


def test_chunked_solve_is_bitwise_equal():
    op = wl.square_lattice(40, W=1.0, seed=22)
    lo, hi = gu.oracle_bounds(op)
    a, b = oracle.scale_from_bounds(lo, hi, 0.01)
    h = kpm.Hamiltonian(op, a, b, kpm.F32)
    whole = kpm.moments(h, 301, 6, wl.VEC_RADEMACHER, seed=5).cpu().numpy()
    for chunk in (1, 7, 64, 1000):
        s = kpm.Solve(h, 301, 6, wl.VEC_RADEMACHER, seed=5)
        rem = 1
        while rem > 0:
            rem = s.advance(chunk)
        mu = s.finish().cpu().numpy()
        s.close()
        assert np.array_equal(mu, whole), chunk
    h.free()


@pytest.mark.parametrize("prec", [kpm.F64, kpm.F32])
def test_batched_equals_solo_bitwise(prec):
    ops = [wl.spin_cubic_lattice(L, seed=30 + L) for L in (5, 9, 6, 11)]
    hs, ab = [], []
    for op in ops:
        lo, hi = gu.oracle_bounds(op)
        a, b = oracle.scale_from_bounds(lo, hi, 0.01)
        hs.append(kpm.Hamiltonian(op, a, b, prec))
        ab.append((a, b))
    Ms = [64, 31, 128, 2]
    Rs = [4, 3, 5, 2]
    seeds = [11, 12, 13, 14]
    batched = [m.cpu().numpy() for m in kpm.moments_batched(hs, Ms, Rs, wl.VEC_PHASE, seeds, [0, 1, 2, 3])]
    for k, h in enumerate(hs):
        solo = kpm.moments(h, Ms[k], Rs[k], wl.VEC_PHASE, seeds[k], k).cpu().numpy()
        assert np.array_equal(batched[k], solo), k
        if prec == kpm.F64:
            ref = gu.oracle_moments(ops[k], ab[k][0], ab[k][1], Ms[k], Rs[k], wl.VEC_PHASE, seeds[k], k)
            gu.assert_fp64(batched[k], ref, f"batched[{k}]")
    for h in hs:
        h.free()


@pytest.mark.parametrize("prec", [kpm.F64, kpm.F32])
def test_batched_waves_bitwise(prec):
    """Batched solves split into cache-sized waves (1 MiB forces several waves, 0 one wave) give
    the solo moments bit for bit, with single-workgroup, march and CSR instances mixed."""
    ops = [wl.spin_cubic_lattice(5, seed=70), wl.spin_cubic_lattice(12, seed=71), wl.spin_cubic_lattice(17, seed=72),
           wl.square_lattice(70, W=1.0, seed=73), wl.lattice_to_csr(wl.square_lattice(30, W=1.0, seed=74)),
           wl.cubic_lattice(16, W=2.0, seed=75)]
    hs = []
    for op in ops:
        lo, hi = gu.oracle_bounds(op)
        a, b = oracle.scale_from_bounds(lo, hi, 0.01)
        hs.append(kpm.Hamiltonian(op, a, b, prec))
    Ms, Rs = [40, 64, 90, 50, 33, 128], [3, 4, 3, 5, 2, 4]
    seeds, insts = [5, 6, 7, 8, 9, 10], [1, 2, 3, 4, 5, 6]
    # static batches take one step per pass, so their solo reference does too (a blocked solo solve
    # forms the same vectors but sums its dot partials over other work items)
    with kpm.launch_settings(tblock=0):
        solo = [kpm.moments(h, Ms[k], Rs[k], wl.VEC_PHASE, seeds[k], insts[k]).cpu().numpy()
                for k, h in enumerate(hs)]
    for wave in (1, 0, 192):
        with kpm.launch_settings(wave_mib=wave):
            got = [m.cpu().numpy() for m in kpm.moments_batched(hs, Ms, Rs, wl.VEC_PHASE, seeds, insts)]
        for k in range(len(hs)):
            assert np.array_equal(got[k], solo[k]), (wave, k)
    for h in hs:
        h.free()


@pytest.mark.parametrize("prec", [kpm.F64, kpm.F32])
def test_batched_wave_placement_bitwise(prec):
    """Ten spin cubes of one kernel class in one wave, the largest big enough for a plan of their
    own that splits them over the XCDs: the wave balances them whole over the XCDs by load, which
    changes only which block runs a work item, so every result equals the solo solve bit for bit
    (and the FP64 ones the oracle)."""
    sizes = [6, 9, 12, 16, 20, 24, 30, 36, 46, 48]
    ops = [wl.spin_cubic_lattice(L, seed=90 + L) for L in sizes]
    hs, ab = [], []
    for op in ops:
        lo, hi = gu.oracle_bounds(op)
        a, b = oracle.scale_from_bounds(lo, hi, 0.01)
        hs.append(kpm.Hamiltonian(op, a, b, prec))
        ab.append((a, b))
    M, R = 24, 16
    seeds, insts = list(range(60, 70)), list(range(10))
    got = [m.cpu().numpy() for m in kpm.moments_batched(hs, M, R, wl.VEC_PHASE, seeds, insts)]
    for k, h in enumerate(hs):
        solo = kpm.moments(h, M, R, wl.VEC_PHASE, seeds[k], insts[k]).cpu().numpy()
        assert np.array_equal(got[k], solo), (sizes[k], k)
    if prec == kpm.F64:
        for k in (1, 8):
            ref = gu.oracle_moments(ops[k], ab[k][0], ab[k][1], M, R, wl.VEC_PHASE, seeds[k], insts[k])
            gu.assert_fp64(got[k], ref, f"wave placement L={sizes[k]}")
    for h in hs:
        h.free()


def test_batched_wave_mixed_kinds_bitwise():
    """A wave with single-workgroup, CSR, 2D march and at least eight 3D spin march instances (each
    kernel class placed on its own, the spin cubes whole per XCD): every result equals its solo
    solve bit for bit, also when the wave budget cuts the batch into several waves."""
    ops = ([wl.spin_cubic_lattice(L, seed=400 + L) for L in (5, 13, 15, 17, 19, 21, 23, 26, 29, 31)] +
           [wl.lattice_to_csr(wl.square_lattice(25, W=1.0, seed=420)), wl.square_lattice(90, W=2.0, seed=421)])
    hs = []
    for op in ops:
        lo, hi = gu.oracle_bounds(op)
        a, b = oracle.scale_from_bounds(lo, hi, 0.01)
        hs.append(kpm.Hamiltonian(op, a, b, kpm.F32))
    n = len(hs)
    Ms = [20 + 3 * k for k in range(n)]
    Rs = [8 + (k % 5) for k in range(n)]      # >= 4 chunks per site: every cube from L = 13 up marches
    seeds, insts = [70 + k for k in range(n)], list(range(n))
    with kpm.launch_settings(tblock=0):
        solo = [kpm.moments(h, Ms[k], Rs[k], wl.VEC_PHASE, seeds[k], insts[k]).cpu().numpy()
                for k, h in enumerate(hs)]
    for wave in (0, 2):
        with kpm.launch_settings(wave_mib=wave):
            got = [m.cpu().numpy() for m in kpm.moments_batched(hs, Ms, Rs, wl.VEC_PHASE, seeds, insts)]
        for k in range(n):
            assert np.array_equal(got[k], solo[k]), (wave, k)
    for h in hs:
        h.free()


def test_mixed_operator_batch():
    ops = [wl.square_lattice(20, W=1.0, seed=40), wl.spin_cubic_lattice(6, seed=41), wl.cubic_lattice(7, W=1.0, seed=42)]
    hs = []
    for op in ops:
        lo, hi = gu.oracle_bounds(op)
        a, b = oracle.scale_from_bounds(lo, hi, 0.01)
        hs.append(kpm.Hamiltonian(op, a, b, kpm.F64))
    batched = [m.cpu().numpy() for m in kpm.moments_batched(hs, 40, 3, wl.VEC_PHASE, [1, 2, 3], [0, 0, 0])]
    for k, h in enumerate(hs):
        solo = kpm.moments(h, 40, 3, wl.VEC_PHASE, k + 1, 0).cpu().numpy()
        assert np.array_equal(batched[k], solo), k


def test_repeat_is_deterministic():
    op = wl.spin_cubic_lattice(10, seed=50)
    a, b = 6.0 / 0.99, 0.0
    x = gu.gpu_moments(op, a, b, kpm.F32, 100, 8, wl.VEC_PHASE, seed=1)
    y = gu.gpu_moments(op, a, b, kpm.F32, 100, 8, wl.VEC_PHASE, seed=1)
    assert np.array_equal(x, y)


@pytest.mark.parametrize("jackson", [True, False])
@pytest.mark.parametrize("K,M", [(1024, 256), (300, 77), (16, 40)])
def test_dos_matches_oracle(K, M, jackson):
    import torch
    g = np.random.default_rng(K + M)
    mu = np.r_[1.0, g.uniform(-0.5, 0.5, M - 1) / np.sqrt(np.arange(1, M))]
    a, b = 4.2, -0.3
    om_ref, rho_ref = oracle.dos(mu, K, a, b, use_jackson=jackson)
    om, rho = kpm.dos(torch.from_numpy(mu).cuda(), K, a, b, jackson=jackson)
    om, rho = om.cpu().numpy(), rho.cpu().numpy()
    assert np.abs(om - om_ref).max() <= 1e-14 * max(abs(a), abs(b))
    scale = np.abs(rho_ref).max()
    print(f"  dos K={K} M={M}: max rel {np.abs(rho - rho_ref).max() / scale:.3e}")
    assert np.abs(rho - rho_ref).max() <= 1e-12 * scale


def test_workspace_too_small_is_rejected():
    import torch
    op = wl.square_lattice(8)
    h = kpm.Hamiltonian(op, 4.1, 0.0, kpm.F64)
    need = h.workspace_bytes(20, 2, 0)
    ws = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    mu = torch.empty(20, dtype=torch.float64, device="cuda")
    st = kpm.lib().kpm_moments(h.handle, 20, 2, 0, 1, 0, ws.data_ptr(), need - 256, mu.data_ptr(), None)
    assert st == 6
    h.free()
