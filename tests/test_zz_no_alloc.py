"""The allocation-free diagnostics entry point (wmb_diagnostics_noalloc),
through the C ABI, against wmb_diagnostics: the same twelve numbers, bitwise,
on two calls in a row (the second on a smaller batch, so the static records
hold the first call's contents when it starts), and the size limit of its
static records."""
import numpy as np
import pytest

from paper_1701_07452_amd import inputs as I
from tests.test_gpu_parity import CASES, gpu_sim, wmb  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def _reference(sim):
    tot, dn, dr, nfl = sim.diagnostics()
    return np.array(list(tot) + [dn, dr, float(nfl), float(sim.protected_faces())])


def test_noalloc_diagnostics_equal_the_allocating_ones(wmb):
    import torch

    runs = [
        # first: the uneven tiling in FP64 after 3 steps (records 0..19 written)
        (CASES["uneven"], 0, dict(limiter_beta=1.5)),
        # second, smaller: 8 patches of 8^3 in FP32 (records 0..7 rewritten)
        (CASES["uniform8"], 1, {}),
    ]
    for k, (case, prec, kw) in enumerate(runs):
        G, (q, b) = case()
        N = G.shape
        sim = gpu_sim(wmb, G, q, b, prec, dx=(1.0 / N[2], 1.0 / N[1], 1.0 / N[0]), **kw)
        sim.run_steps(3)
        sim.synchronize()
        ref = _reference(sim)
        out = torch.full((12,), float("nan"), dtype=torch.float64, device="cuda")
        sim.diagnostics_noalloc(out)
        sim.synchronize()
        got = out.cpu().numpy()
        print("call %d (%d patches): %s" % (k, G.npatch, got))
        assert np.array_equal(got, ref), (k, got, ref)
        assert got[10] == 0 and np.isfinite(got).all()
        sim.close()


def test_noalloc_diagnostics_reject_batches_beyond_the_records(wmb):
    """32769 patches of 4^3 (one record each) exceed the 32768 static
    records: WMB_ESIZE with a message, nothing launched."""
    import torch

    G = I.uniform_grid((4 * 32769, 4, 4), 4)
    sim = wmb.Sim(wmb.make_params(dx=(1.0, 1.0, 1.0), ghost=4, precision=wmb.WMB_FP32), G.descs)
    out = torch.zeros(12, dtype=torch.float64, device="cuda")
    with pytest.raises(wmb.WmbError) as e:
        sim.diagnostics_noalloc(out)
    assert e.value.code == wmb.WMB_ESIZE and "32768" in str(e.value)
    sim.close()
    del sim
    torch.cuda.empty_cache()
