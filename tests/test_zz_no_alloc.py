"""nm_pencil_apply_noalloc (operators with the library's static scratch array,
for callers that cannot allocate) against nm_pencil_apply."""
import numpy as np
import pytest

from conftest import planet as make_planet

pytestmark = pytest.mark.gpu


def test_noalloc_equals_allocating_entry_point():
    """Every operator through the no-allocation entry point equals the
    allocating one bit for bit (same kernels), on two calls in a row with the
    second on fewer columns, with no device allocation by the library during
    the calls; sizes beyond the scratch array and mass_passes are rejected."""
    import torch
    import paper_1906_11082_amd as nm
    print("\n[case] no-alloc entry point, three-layer planet n_half=4", flush=True)
    nm.load_library()
    d = make_planet("three_layer_planet", n_half=4, order=2, pres_order=1)
    G = nm.Pencil(d)
    n, n_p = G.n, G.n_p
    count = {"alloc": 0}
    dev = torch.cuda.current_device()

    def alloc(nbytes):
        count["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(nbytes, device=dev)

    nm.set_allocator(alloc, torch.cuda.caching_allocator_delete)
    try:
        g = torch.Generator(device="cpu").manual_seed(11)
        cases = [(nm.OP_M, 0, n, n), (nm.OP_AG, 0, n, n), (nm.OP_R, 0, n, n), (nm.OP_A, 0, n, n),
                 (nm.OP_MINV, 0, n, n), (nm.OP_B, 0, n, n), (nm.OP_EGT, 0, n, n_p), (nm.OP_EG, 0, n_p, n),
                 (nm.OP_KP, 0, n_p, n_p), (nm.OP_KPINV, 0, n_p, n_p), (nm.OP_MINV, 1, n, n), (nm.OP_B, 1, n, n)]
        for ncols in (16, 5):
            for op, prec, rin, rout in cases:
                dt = torch.float32 if prec else torch.float64
                X = torch.randn(rin, ncols, generator=g, dtype=torch.float64).to(dt).cuda()
                kw = dict(precision=prec, kM=14, kP=9)
                ref = G.apply(op, X, out_rows=rout, **kw)
                Y = torch.full((rout, ncols), float("nan"), dtype=dt, device="cuda")
                torch.cuda.synchronize()
                before = count["alloc"]
                G.apply_noalloc(op, X, Y, **kw)
                torch.cuda.synchronize()
                assert count["alloc"] == before, (op, prec, ncols)
                assert torch.equal(Y, ref), (op, prec, ncols)
        print("library allocations outside the no-alloc calls: %d" % count["alloc"], flush=True)
        assert count["alloc"] > 0  # the hooks do see the allocating entry point's buffers
        # beyond the scratch array: rejected before any launch
        wide = 2 * (256 << 20) // (8 * n) + 8
        X = torch.zeros(n, wide, dtype=torch.float64, device="cuda")
        Y = torch.zeros_like(X)
        with pytest.raises(nm.NMError) as e:
            G.apply_noalloc(nm.OP_B, X, Y)
        assert e.value.status == -1 and "scratch" in str(e.value)
        with pytest.raises(nm.NMError) as e:
            G.apply_noalloc(nm.OP_MINV, X[:, :8].contiguous(), Y[:, :8].contiguous(), mass_passes=2)
        assert e.value.status == -1
    finally:
        nm.set_allocator(None, None)
