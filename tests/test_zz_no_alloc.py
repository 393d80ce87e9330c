"""The allocation-free variant of tcm_moments through the C ABI.

tcm_moments_noalloc takes device inputs and outputs and keeps every scratch byte in the
library's static per-device array.  Checked here: its moments, radius and centre equal those of
tcm_moments on the same molecule bit for bit (the same tiling and kernels), on two calls in a
row (the second with a smaller molecule, so stale scratch from the first would show), at both
precisions; it changes nothing in the context's accounted device memory; a molecule whose scratch
would not fit the static array is refused with TCM_ENOMEM before anything is launched."""
import numpy as np
import pytest

from paper_0704_1672_amd import tcm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tcm.Context(0)
    yield c.h
    c.close()


def device_soa(xyz, q):
    import torch
    t = torch.tensor(np.vstack([xyz.T, q[None, :]]), dtype=torch.float64, device="cuda").contiguous()
    return t


def noalloc(ctx, xyz, q, L, prec, centre):
    import torch
    t = device_soa(xyz, q)
    Q = torch.full(((L + 1) ** 2,), float("nan"), dtype=torch.float64, device="cuda")
    meta = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    used0, _ = tcm.tcm_mem_info(ctx)
    tcm.tcm_moments_noalloc(ctx, t[0], t[1], t[2], t[3], len(q), centre, L, prec, Q, meta)
    torch.cuda.synchronize()                       # the call is asynchronous on the context's stream
    used1, _ = tcm.tcm_mem_info(ctx)
    m = meta.cpu().numpy()
    return Q.cpu().numpy(), m[3], m[:3], used1 - used0


@pytest.mark.parametrize("prec", [tcm.TCM_F64, tcm.TCM_F32C])
def test_noalloc_equals_tcm_moments_twice(ctx, synth, prec):
    L = 16
    cases = [(300_000, np.array([1.0, -2.0, 0.5])), (5_000, None)]    # the second smaller
    for k, (n, centre) in enumerate(cases):
        print(f"noalloc case prec={prec} n={n} L={L}", flush=True)
        xyz, q = synth.ball(70 + k, L, n, 40.0, np.array([3.0, 1.0, -2.0]))
        Qr, rr, cr = tcm.tcm_moments(ctx, xyz, q, L, prec, centre=centre)
        Qn, rn, cn, grew = noalloc(ctx, xyz, q, L, prec, centre)
        assert grew == 0
        assert np.array_equal(Qn, Qr), (n, np.max(np.abs(Qn - Qr)))
        assert rn == rr and np.array_equal(cn, cr)


def test_noalloc_small_orders_and_empty(ctx, synth):
    for L, n in [(0, 700), (3, 2049), (8, 0)]:
        print(f"noalloc case L={L} n={n}", flush=True)
        xyz, q = synth.ball(90 + L, max(L, 1), max(n, 1), 5.0, np.zeros(3))
        xyz, q = xyz[:n], q[:n]
        centre = np.array([0.5, 0.0, 0.0]) if n == 0 else None
        if n == 0:
            xyz, q = np.zeros((1, 3)), np.zeros(1)        # buffers to point at; n = 0 is passed
        Qr, rr, cr = tcm.tcm_moments(ctx, xyz[:n], q[:n], L, tcm.TCM_F64, centre=centre)
        import torch
        t = device_soa(xyz, q)
        Q = torch.full(((L + 1) ** 2,), float("nan"), dtype=torch.float64, device="cuda")
        meta = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        tcm.tcm_moments_noalloc(ctx, t[0], t[1], t[2], t[3], n, centre, L, tcm.TCM_F64, Q, meta)
        torch.cuda.synchronize()
        assert np.array_equal(Q.cpu().numpy(), Qr)
        m = meta.cpu().numpy()
        assert m[3] == rr and np.array_equal(m[:3], cr)


def test_noalloc_refuses_what_does_not_fit(ctx, synth):
    import torch
    t = torch.zeros((4, 16), dtype=torch.float64, device="cuda")
    Q = torch.zeros(((tcm.TCM_LMAX + 1) ** 2,), dtype=torch.float64, device="cuda")
    meta = torch.zeros((8,), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    n = 10 ** 9                                    # its tile partials alone: ~4 GB at order 32
    with pytest.raises(tcm.TCMError) as e:
        tcm.tcm_moments_noalloc(ctx, t[0], t[1], t[2], t[3], n, None, tcm.TCM_LMAX, tcm.TCM_F64, Q, meta)
    assert e.value.code == tcm.TCM_ENOMEM
    with pytest.raises(tcm.TCMError) as e:
        tcm.tcm_moments_noalloc(ctx, t[0], t[1], t[2], t[3], 16, None, tcm.TCM_LMAX + 1, tcm.TCM_F64, Q, meta)
    assert e.value.code == tcm.TCM_EINVAL
