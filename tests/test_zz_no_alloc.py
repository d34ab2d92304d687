"""frg_rhs_noalloc (the rhs from the library's static scratch) against frg_rhs,
through the C ABI: the same kernels on the same inputs, so the results agree bit
for bit.  Calls follow each other on one device and share its scratch: the
benchmark size in symmetric-vertex mode first, then smaller contexts (every
column computed), so a later call finds the previous call's contents in the
scratch.  A context whose workspace exceeds the scratch is refused."""
import numpy as np
import pytest

from paper_1510_07799_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1510_07799_amd import frg  # noqa: E402

N32 = dict(t=1.0, tp=-0.25, mu=-0.9, U=2.5, N=32, n_rad=6, n_ang=4)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def check(g, V, T, prec, vsym):
    g.set_vsym(vsym)
    try:
        ref = g.rhs(T, V, prec).clone()
        F = torch.full_like(V, float("nan"))
        g.rhs_noalloc(T, V, F, prec)
        torch.cuda.synchronize()
        same = torch.equal(F, ref)
        d = (F - ref).abs().max().item() / ref.abs().max().item()
        print(f"[noalloc] N={g.N} prec={prec} vsym={vsym} T={T}: equal {same}, normwise {d:.2e}", flush=True)
        assert same
    finally:
        g.set_vsym(False)


def test_noalloc_matches_rhs_on_calls_in_a_row():
    cases = []
    p3 = I.model_params("C3")
    g3 = frg.Context(**p3)
    V3 = dev(I.random_vertex(96, p3["U"], seed=101, amp=0.3, symmetrise=True))
    cases.append((g3, V3, True))
    g32 = frg.Context(**N32)
    cases.append((g32, dev(I.random_vertex(32, N32["U"], seed=102, amp=0.3, symmetrise=False)), False))
    p1 = I.model_params("C1")
    g16 = frg.Context(**p1)
    cases.append((g16, dev(I.random_vertex(16, p1["U"], seed=103, amp=0.3, symmetrise=False)), False))
    for prec in (frg.PREC_SPLIT_BF16, frg.PREC_FP64):
        for g, V, vs in cases:            # decreasing sizes: each call after a larger one
            check(g, V, 0.05, prec, vs)
    # and a second round at other temperatures, smallest first
    for g, V, vs in reversed(cases):
        check(g, V, 1e-3, frg.PREC_SPLIT_BF16, vs)
    for g, _, _ in cases:
        g.close()


def test_noalloc_refuses_a_workspace_beyond_the_scratch():
    p3 = I.model_params("C3")
    g = frg.Context(**p3)
    V = torch.zeros(96 ** 3, dtype=torch.float64, device="cuda")
    F = torch.zeros_like(V)
    with pytest.raises(frg.FRGError) as e:
        g.rhs_noalloc(0.05, V, F, frg.PREC_FP64)   # every column in FP64: beyond 256 MiB
    assert e.value.status == frg.ENOTSUP
    assert "static scratch" in str(e.value)
    g.close()
