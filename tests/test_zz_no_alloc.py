"""gwg_loss_noalloc (the loss with its work buffer in fixed library device
memory, for callers that cannot allocate) against gwg_loss, through the C
ABI: identical loss and dL/dI on two calls in a row, the second with a
smaller input, and a clear error beyond the fixed size."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2601_04370_amd as gwg

pytestmark = pytest.mark.gpu


def _call(ctx, fn, irr, kind, w_f, w_e):
    D, nl, F = irr.shape[:3]
    B = int(np.prod(irr.shape[3:]))
    loss = torch.full((1,), np.nan, dtype=torch.float64, device="cuda:0")
    g = torch.full_like(irr, np.nan)
    rc = fn(ctx.h, irr.data_ptr(), D, nl, F, B, kind, w_f, w_e, loss.data_ptr(), g.data_ptr(),
            torch.cuda.current_stream().cuda_stream)
    return rc, loss, g


@pytest.mark.parametrize("kind,w_f,w_e", [(0, 1.0, 1.0), (1, 10.0, 3.0)])
def test_noalloc_loss_matches_loss(kind, w_f, w_e):
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ctx = gwg.Context(0)
    lib = gwg.load_library()
    rng = np.random.default_rng(7 + kind)
    # first a large shape (diff_1200: 3 wavelengths, 441 FoV points, 32 x 32
    # bins, two designs), then a smaller one that reuses the scratch
    for shape in ((2, 3, 441, 32, 32), (1, 2, 9, 8, 8)):
        print(f"noalloc loss kind {kind} shape {shape}", flush=True)
        irr = torch.tensor(rng.uniform(0.0, 1e-3, size=shape), device="cuda:0")
        rc0, L0, g0 = _call(ctx, lib.gwg_loss, irr, kind, w_f, w_e)
        rc1, L1, g1 = _call(ctx, lib.gwg_loss_noalloc, irr, kind, w_f, w_e)
        torch.cuda.synchronize()
        assert rc0 == gwg.gwg.GWG_OK and rc1 == gwg.gwg.GWG_OK, lib.gwg_last_error(ctx.h)
        assert torch.equal(L0, L1) and torch.equal(g0, g1)
        assert torch.isfinite(L1).all() and torch.isfinite(g1).all()
    # beyond the fixed scratch: rejected before any launch
    D, nl, F, B = 64, 31, 121, 256     # 264704 doubles: fits
    big = torch.zeros((D, nl, F, B), dtype=torch.float64, device="cuda:0")
    rc, _, _ = _call(ctx, lib.gwg_loss_noalloc, big, kind, w_f, w_e)
    assert rc == gwg.gwg.GWG_OK
    big = torch.zeros((128, nl, F, B), dtype=torch.float64, device="cuda:0")   # 529408 > 524288
    rc, L, _ = _call(ctx, lib.gwg_loss_noalloc, big, kind, w_f, w_e)
    torch.cuda.synchronize()
    assert rc == gwg.gwg.GWG_E_INVAL
    assert b"scratch" in lib.gwg_last_error(ctx.h)
    assert torch.isnan(L).all()
    ctx.close()
