"""The library's device buffers through a caller's allocator (nm_set_allocator):
torch's caching allocator serves every buffer of an assembly and a solve, the
result matches the hipMalloc run, and every buffer is returned."""
import gc

import numpy as np
import pytest

from conftest import planet as make_planet

pytestmark = pytest.mark.gpu


def test_torch_caching_allocator_serves_library_buffers():
    import torch
    import paper_1906_11082_amd as nm
    d = make_planet("homogeneous_ball", n_half=3, order=1)
    print("\n[case] allocator: ball n_half=3", flush=True)
    G0 = nm.Pencil(d)
    r0 = G0.filtered_eig(0.5, 40.0, 12, 1e-10, degree=40, block=8)
    dev = torch.cuda.current_device()
    live, counts = {}, {"alloc": 0, "free": 0}

    def alloc(nbytes):
        p = torch.cuda.caching_allocator_alloc(nbytes, device=dev)
        counts["alloc"] += 1
        live[p] = nbytes
        return p

    def free(p):
        counts["free"] += 1
        live.pop(p)
        torch.cuda.caching_allocator_delete(p)

    nm.set_allocator(alloc, free)
    try:
        G = nm.Pencil(d)
        r = G.filtered_eig(0.5, 40.0, 12, 1e-10, degree=40, block=8)
        lam, resid, count = r.lam.copy(), r.resid.copy(), r.count
        peak = counts["alloc"]
        del r, G
        gc.collect()
    finally:
        nm.set_allocator(None, None)
    print("allocator: %d buffers allocated and %d freed" % (counts["alloc"], counts["free"]), flush=True)
    assert peak > 10
    assert counts["free"] == counts["alloc"] and not live
    assert count == r0.count == 12
    assert np.abs(lam - r0.lam).max() <= 1e-12 * r0.lam.max()
    assert resid.max() <= 1e-10
