"""Host logic of the launch autotuner: shape keys and the keys tuned per operator class."""
from types import SimpleNamespace

from paper_1105_5481_amd import tune
from paper_1105_5481_amd import workloads as wl


def _h(op, prec=1):
    return SimpleNamespace(op=op, prec=prec)


def test_shape_key_distinguishes_shapes():
    a = _h(wl.spin_cubic_lattice(8, seed=1))
    b = _h(wl.spin_cubic_lattice(9, seed=1))
    c = _h(wl.lattice_to_csr(wl.square_lattice(6, seed=2)))
    assert tune.shape_key([a], 16, wl.VEC_PHASE) != tune.shape_key([b], 16, wl.VEC_PHASE)
    assert tune.shape_key([a], 16, wl.VEC_PHASE) != tune.shape_key([a], 8, wl.VEC_PHASE)
    assert tune.shape_key([a], 16, wl.VEC_PHASE) != tune.shape_key([a], 16, wl.VEC_RADEMACHER)
    assert tune.shape_key([a], 16, wl.VEC_PHASE) != tune.shape_key([_h(a.op, 0)], 16, wl.VEC_PHASE)
    # same spins, other values: same class; batch order does not matter
    a2 = _h(wl.spin_cubic_lattice(8, seed=5))
    assert tune.shape_key([a], 4, 1) == tune.shape_key([a2], 4, 1)
    assert tune.shape_key([a, c], [4, 2], 1) == tune.shape_key([c, a], [2, 4], 1)
    assert "csr36x" in tune.shape_key([c], 2, 0)
    assert tune.shape_key([a, a2, c], 4, 1).endswith("d3s8x8x8R4*2")
    many = [_h(wl.spin_cubic_lattice(L, seed=L)) for L in range(4, 40)]
    k = tune.shape_key(many, 4, 1)
    assert len(k) < 200 and k == tune.shape_key(many[::-1], 4, 1)


def test_keys_per_operator_class():
    lat = _h(wl.square_lattice(6, seed=3))
    csr = _h(wl.lattice_to_csr(wl.square_lattice(6, seed=3)))
    assert tune._keys_for([lat]) == tune.LATTICE_KEYS
    assert tune._keys_for([csr]) == tune.FLAT_KEYS
    ks = tune._keys_for([lat, csr])
    assert "march_items" in ks and "elems_per_thread" in ks and "wave_mib" in ks
    for k in ks:
        assert tune.CANDIDATES[k]
