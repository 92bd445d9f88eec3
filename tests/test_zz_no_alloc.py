"""The no-allocation energy entry point against fracture_energy.

fracture_energy_noalloc evaluates the energies of a caller-given state from
a static device scratch array, with no handle and no allocation; on the same
state it must return what a handle's fracture_energy returns (the same
kernels in the same reduction order: equal bit for bit).  Each case calls it
twice in a row, the second time on a smaller mesh, so the second call reuses
scratch the first one left behind.
"""

import numpy as np
import pytest

from paper_1511_08463_amd import fracture, workloads

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _state(p, seed):
    n_nodes, ndof = fracture.fracture_sizes(fracture.make_params(**p))
    rng = np.random.default_rng(seed)
    u = 0.01 * rng.standard_normal(ndof)
    alpha = rng.uniform(0.0, 1.0, n_nodes)
    return u, alpha


def _both(p, load, seed):
    """(handle energies, no-allocation energies) of one seeded state."""
    torch = _torch()
    params = fracture.make_params(**p)
    u, alpha = _state(p, seed)
    s = fracture.Fracture(params, None, device="cuda:0")
    s.set_state(u=u, alpha=alpha, alpha_prev=np.zeros_like(alpha))
    s.set_load(load)
    # set_load lifts the boundary values into u: evaluate both on that u
    u_l = s.state()[0]
    want = s.energy()
    stream = s.stream
    du = torch.as_tensor(u_l, device="cuda:0")
    da = torch.as_tensor(alpha, device="cuda:0")
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    fracture.fracture_energy_noalloc(params, load, du.data_ptr(), da.data_ptr(),
                                     stream.cuda_stream, out.data_ptr())
    stream.synchronize()
    got = tuple(out.cpu().numpy())
    s.close()
    return want, got


CASES = [
    ("tension AT1", [(workloads.tension(96, 0.05, nx=96, ny=80), 0.3),
                     (workloads.tension(40, 0.05, nx=40, ny=24), 0.1)]),
    ("tension AT2", [(workloads.tension(128, 0.03, "AT2", nx=128, ny=64), 0.2),
                     (workloads.tension(8, 0.2, "AT2", nx=8, ny=8), 0.05)]),
    ("thermal shock 2D", [(workloads.tshock(64, 16, ratio=4.0), 1.2),
                          (workloads.tshock(16, 4, ratio=2.0), 0.5)]),
    ("thermal 3D", [(workloads.thermal(16, 12, 6), 1.3),
                    (workloads.thermal(4, 4, 2), 0.7)]),
]


@pytest.mark.parametrize("name,calls", CASES, ids=[c[0] for c in CASES])
def test_noalloc_energy_equals_handle_energy(name, calls):
    for k, (p, load) in enumerate(calls):
        print(f"[noalloc] {name} call {k + 1}: {p['nx']}x{p['ny']}"
              + (f"x{p['nz']}" if p.get("dim") == 3 else "") + f" load {load}", flush=True)
        want, got = _both(p, load, seed=17 + k)
        assert np.all(np.isfinite(got))
        assert got == want, (name, k, got, want)


def test_noalloc_energy_repeated_calls_agree():
    """The same state twice after a larger one: identical results (nothing
    in the scratch carries over between calls)."""
    big = workloads.tension(256, 0.02, nx=256, ny=192)
    small = workloads.tension(24, 0.1, nx=24, ny=16)
    first = _both(small, 0.1, seed=5)[1]
    _both(big, 0.4, seed=6)
    again = _both(small, 0.1, seed=5)[1]
    assert first == again
