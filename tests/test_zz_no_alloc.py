"""The allocation-free residual norm (mg_residual_norm_noalloc, for callers
that cannot allocate) against mg_residual_norm, both through the C ABI.

Two calls in a row share the library's static scratch array; the second
runs on a smaller hierarchy, so partial sums left over from the first call
would show in its result.  The bar is the FP64 one of the solver: the two
entry points run the same kernels, and differ only in where the final
square root is taken (host or device), at most one rounding apart.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1104_1703_amd import mg as M
    M.load_library()
    return M


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_noalloc_residual_norm_matches_allocating_entry_point(mg):
    from paper_1104_1703_amd import gen
    cases = [gen.holes_problem(n=64, seed=2),
             gen.random_small_problem((24, 40, 56), 3, active_frac=0.7, blur=1.5)]
    assert cases[1].mask.size < cases[0].mask.size
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(11)
    for p in cases:
        print(f"[case] {p.name} shape={p.shape} active={p.n_active}", flush=True)
        H = mg.Hierarchy(_dev(p.mask), p.h)
        rho = _dev(p.rho)
        phi = _dev(rng.standard_normal(p.shape))          # junk on inactive cells too
        B = None if p.dirichlet is None else _dev(p.dirichlet)
        ref = H.residual_norm(rho, phi, B)
        torch.cuda.synchronize()
        before = torch.cuda.memory_stats()["allocation.all.allocated"]
        H.residual_norm_noalloc(rho, phi, B, out=out)
        torch.cuda.synchronize()
        assert torch.cuda.memory_stats()["allocation.all.allocated"] == before
        got = float(out.item())
        print(f"  noalloc {got!r} allocating {ref!r}", flush=True)
        assert ref > 0 and abs(got - ref) <= 1e-15 * ref
        H.close()


def test_noalloc_rejects_a_foreign_device_or_null(mg):
    import ctypes as C
    lib = mg.load_library()
    assert lib.mg_residual_norm_noalloc(None, None, None, None, None) == mg.MG_ERR_ARG
