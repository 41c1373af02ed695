"""hbs_apply_noalloc (workspaces in a static per-device scratch, no device allocation) against
hbs_apply, through the C ABI: the same kernels on the same data, so the results agree to the
relative 1e-12 bar of two applications of one factorization (in practice bit for bit)."""
import numpy as np
import pytest

import qpinputs
from paper_1301_1247_amd.geometry import discretize

pytestmark = pytest.mark.gpu


def _rand(torch, r, N, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    re = torch.randn((r, N), generator=g, dtype=torch.float64)
    im = torch.randn((r, N), generator=g, dtype=torch.float64)
    return torch.complex(re, im).to("cuda")


def _close(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    return np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


@pytest.mark.parametrize("name,N,omega,tol", [("wavy20", 2000, 40.0, 1e-12), ("wavy40", 100000, 60.0, 1e-13)])
def test_noalloc_apply_matches_apply(gpu_lib, name, N, omega, tol):
    import torch
    c = qpinputs.workload(name).curve
    nodes, w, nrm, _ = discretize(c, N)
    t = lambda a: torch.from_numpy(a).to("cuda")
    h = gpu_lib.Handle(t(nodes), t(w), t(nrm), omega, tol, device=True)
    # two calls in a row, the second with fewer columns, and one with refinement steps
    for r, refine, seed in ((4, 0, 1), (1, 0, 2), (2, 2, 3)):
        b = _rand(torch, r, N, seed)
        cached = gpu_lib.pool_cached_bytes()
        peak = h.stats().device_bytes_peak
        x_na = h.apply_noalloc(b, refine=refine)
        assert gpu_lib.pool_cached_bytes() == cached        # nothing drawn from or returned to the pool
        assert h.stats().device_bytes_peak == peak
        x_ref = h.apply(b, refine=refine)
        assert _close(x_na, x_ref), (r, refine)
    # the handle's own workspaces are intact after the no-alloc calls
    b = _rand(torch, 3, N, 4)
    assert _close(h.apply(b), h.apply_noalloc(b))


def test_noalloc_rejects_too_many_columns(gpu_lib):
    import torch
    c = qpinputs.workload("wavy20").curve
    N = 2000
    nodes, w, nrm, _ = discretize(c, N)
    t = lambda a: torch.from_numpy(a).to("cuda")
    h = gpu_lib.Handle(t(nodes), t(w), t(nrm), 40.0, 1e-12, device=True)
    r = 2048  # about 0.2 GB of level and ping-pong buffers
    b = torch.zeros((r, N), dtype=torch.complex128, device="cuda")
    with pytest.raises(gpu_lib.HBSError) as e:
        h.apply_noalloc(b)
    assert e.value.code == -3 and "scratch" in str(e.value)
    # a host-pointer handle is refused
    h2 = gpu_lib.Handle(nodes, w, nrm, 40.0, 1e-12)
    with pytest.raises(ValueError):
        h2.apply_noalloc(b[:1])
