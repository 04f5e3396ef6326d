"""Work-item shapes of the smoother (default, given, or picked by the
autotuner at hierarchy creation): z marches of 8/16/32 planes on the finest
level and 2/4/8 planes or whole 8^3 cubes on coarse levels.  Every shape
runs the same arithmetic on every cell, so iterates are bit for bit those
of the default shapes; only the grouping of the residual norm's partial
sums (one per finest work item) changes, so norms agree to rounding."""
import os
import tempfile

import numpy as np
import pytest

from paper_1104_1703_amd import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1104_1703_amd import mg as M
    M.load_library()
    return M


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


PROBLEMS = {
    "holes64": lambda: gen.holes_problem(n=64, seed=2),
    "rand_ragged": lambda: gen.random_small_problem((24, 40, 56), 3, active_frac=0.7, blur=1.5),
    "rand_dirichlet": lambda: gen.random_small_problem((32, 32, 32), 5, active_frac=0.8, blur=1.0),
    "porous64": lambda: gen.porous_problem(n=64, seed=4),
    "deep_6144": lambda: gen.random_small_problem((24, 128, 128), 9, active_frac=0.75, blur=2.0),
}
VARIANTS = [dict(item_depth_fine=8), dict(item_depth_fine=32), dict(item_depth_l1=2), dict(item_depth_l1=8),
            dict(item_depth_coarse=4), dict(item_depth_coarse=8),
            dict(item_depth_fine=32, item_depth_l1=8, item_depth_coarse=8),
            dict(item_depth_l1=1), dict(item_depth_coarse=1), dict(item_depth_fine=8, item_depth_l1=1, item_depth_coarse=1)]


def _same_solve(a, ia, b, ib, what):
    assert (ia["status"], ia["cycles"], ia["switched_at"], ia["order_used"]) == \
        (ib["status"], ib["cycles"], ib["switched_at"], ib["order_used"]), what
    assert np.array_equal(a, b), what
    ha, hb = np.array(ia["history"]), np.array(ib["history"])
    assert np.all(np.abs(ha - hb) <= 1e-13 * np.abs(hb) + 1e-16 * ia["r_ref"]), what


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_item_depths_give_the_default_iterates(mg, name, precision):
    p = PROBLEMS[name]()
    print(f"[case] {name} {precision} shape={p.shape}", flush=True)
    rho = dev(p.rho)
    d = None if p.dirichlet is None else dev(p.dirichlet)
    H0 = mg.Hierarchy(dev(p.mask), p.h, precision=precision)
    f = H0.fold(rho, d)
    ref_v = {}
    for order in (1, 2):
        x = torch.zeros(p.shape, dtype=torch.float64, device="cuda")
        for _ in range(2):
            x = H0.vcycle(x, f, order=order)
        ref_v[order] = host(x)
    ref, rinfo = H0.solve(rho, None, d, tol=1e-10)
    ref = host(ref)
    for opts in VARIANTS:
        H = mg.Hierarchy(dev(p.mask), p.h, precision=precision, **opts)
        depths = H.item_depths()
        print(f"  {opts}: depths {depths}", flush=True)
        if "item_depth_fine" in opts:
            assert depths[2][0] == opts["item_depth_fine"]
        for order in (1, 2):
            x = torch.zeros(p.shape, dtype=torch.float64, device="cuda")
            for _ in range(2):
                x = H.vcycle(x, f, order=order)
            assert np.array_equal(host(x), ref_v[order]), (name, opts, order)
        got, info = H.solve(rho, None, d, tol=1e-10)
        _same_solve(host(got), info, ref, rinfo, (name, opts))
        H.close()
    H0.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tuned_hierarchy_solves_as_the_default_and_caches_its_choice(mg, precision):
    """The autotuner times each candidate depth on the hierarchy itself; the
    tuned hierarchy gives the default iterates, and a second creation with
    the same cache file takes the recorded depths without timing."""
    p = gen.holes_problem(n=128, seed=2)
    rho = dev(p.rho)
    with tempfile.TemporaryDirectory() as tmp:
        cache = os.path.join(tmp, "tune.txt")
        old = os.environ.get("MG_TUNE_CACHE")
        os.environ["MG_TUNE_CACHE"] = cache
        try:
            H0 = mg.Hierarchy(dev(p.mask), p.h, precision=precision)
            Ht = mg.Hierarchy(dev(p.mask), p.h, precision=precision, tune=1)
            depths = Ht.item_depths()
            print(f"[case] holes128 {precision}: tuned depths {depths}", flush=True)
            lines = open(cache).read().split("\n")
            assert sum(1 for ln in lines if ln.strip()) >= 2
            for o in (1, 2):
                for l, dz in enumerate(depths[o]):
                    assert dz in ((8, 16, 32) if l == 0 else (1, 2, 4, 8))
            ref, rinfo = H0.solve(rho, tol=1e-10)
            got, info = Ht.solve(rho, tol=1e-10)
            _same_solve(host(got), info, host(ref), rinfo, "tuned")
            H2 = mg.Hierarchy(dev(p.mask), p.h, precision=precision, tune=1)
            assert H2.item_depths() == depths
            assert open(cache).read().split("\n") == lines      # cache hit: nothing appended
            H2.close()
            Ht.close()
            H0.close()
        finally:
            if old is None:
                os.environ.pop("MG_TUNE_CACHE", None)
            else:
                os.environ["MG_TUNE_CACHE"] = old


def test_invalid_depths_are_rejected(mg):
    p = gen.sphere_problem(16)
    for opts in (dict(item_depth_fine=12), dict(item_depth_l1=16), dict(tune=2), dict(item_depth_fine=1),
                 dict(fuse_passes=1, item_depth_fine=8), dict(fuse_passes=1, item_depth_coarse=1),
                 dict(fuse_restrict=2), dict(fuse_restrict=-1)):
        with pytest.raises(mg.MGError) as e:
            mg.Hierarchy(dev(p.mask), p.h, **opts)
        assert e.value.status == mg.MG_ERR_ARG
    with pytest.raises(mg.MGError):
        mg.Batch([dev(p.mask)], [p.h], tune=1)
