"""Every binding call that takes a `stream` gives the same results on a side stream (a torch stream
or its raw handle) as on the current stream: the library work, the tensors the binding allocates and
the torch operations it issues all run on that stream."""
import numpy as np
import pytest

import paper_1105_5481_amd as kpm
from paper_1105_5481_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _run(stream):
    import torch
    lat = wl.spin_cubic_lattice(12, seed=4)
    a, b = kpm.lanczos_scale(lat, k=40, stream=stream)
    lo, hi = kpm.gershgorin(lat, stream=stream)
    h = kpm.Hamiltonian(lat, a, b, kpm.F32, stream=stream)
    mu = kpm.moments(h, 64, 8, kpm.VEC_PHASE, 3, 0, stream=stream)
    om, rho = kpm.dos(mu, 128, a, b, stream=stream)
    omg, G = kpm.green(mu, 96, a, b, stream=stream)
    mus = kpm.moments_batched([h, h], [32, 48], [4, 2], kpm.VEC_PHASE, [1, 2], [0, 1], stream=stream)
    s = kpm.Solve(h, 40, 4, kpm.VEC_PHASE, 5, 0, stream=stream)
    while s.advance(7, stream=stream) > 0:
        pass
    mu_s = s.finish(stream=stream)
    om_l, rho_l = kpm.ldos(h, [0, 5], 32, stream=stream)
    H = torch.tensor(wl.dense_symmetric(96, 2), device="cuda")
    mu_d = kpm.dense_moments(H, 3.2, 0.0, 40, 16, kpm.VEC_RADEMACHER, 1, 0, stream=stream)
    sv = kpm.start_vectors(kpm.VEC_PHASE, True, 3, 0, 50, 4, stream=stream)
    torch.cuda.synchronize()
    out = [np.array([a, b, lo, hi]), mu, om, rho, omg, G, *mus, mu_s, om_l, rho_l, mu_d, sv]
    s.close()
    h.free()
    return [x if isinstance(x, np.ndarray) else x.cpu().numpy() for x in out]


@pytest.mark.parametrize("kind", ["torch", "raw"])
def test_side_stream_matches_current_stream(kind):
    import torch
    ref = _run(None)
    side = torch.cuda.Stream()
    got = _run(side if kind == "torch" else side.cuda_stream)
    assert len(got) == len(ref)
    for k, (x, y) in enumerate(zip(got, ref)):
        assert x.shape == y.shape and np.array_equal(x, y), k
