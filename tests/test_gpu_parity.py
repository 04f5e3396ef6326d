"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Bar (FP64): max |gpu - oracle| / max |oracle| <= 1e-11 per field after the
same number of operations; integer hierarchy data bit-exact; same cycle
count, status and switch cycle for solves; residual histories within 1e-6
relative.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import oracle as O
from paper_1104_1703_amd import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
TOL = 1e-11


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


def relerr(a, b, where=None):
    if where is not None:
        a, b = a[where], b[where]
    scale = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / scale)


PROBLEMS = {
    "sphere32": lambda: gen.sphere_problem(32),
    "holes64": lambda: gen.holes_problem(n=64, seed=2),
    "rand_ragged": lambda: gen.random_small_problem((24, 40, 56), 3, active_frac=0.7, blur=1.5),
    "rand_dirichlet": lambda: gen.random_small_problem((32, 32, 32), 5, active_frac=0.8, blur=1.0),
    "porous64": lambda: gen.porous_problem(n=64, seed=4),
    "patch_odd": lambda: gen.patch_problems(count=3, seed=3)[2],
    # 24 halves only to 6: the deepest level (6 x 32 x 32 = 6144 cells) is above the
    # 4096-cell small-level size and runs alone in the one-workgroup kernel
    "deep_6144": lambda: gen.random_small_problem((24, 128, 128), 9, active_frac=0.75, blur=2.0),
}


def _print_case(name, p):
    print(f"[case] {name} shape={p.shape} active={p.n_active}", flush=True)


def _pair(name, mg, **opts):
    p = PROBLEMS[name]()
    _print_case(name, p)
    H = mg.Hierarchy(dev(p.mask), p.h, **opts)
    orc = O.Oracle(p.mask, p.h, min_coarse_dim=opts.get("min_coarse_dim", 4))
    return p, H, orc


# ---------------------------------------------------------------- hierarchy
@pytest.mark.parametrize("name", list(PROBLEMS))
def test_hierarchy_counts_and_active_sets(mg, name):
    p, H, orc = _pair(name, mg)
    assert H.nlevels(0) == orc.nlevels(0)
    for order in (1, 2):
        assert H.nlevels(order) == orc.nlevels(order)
    for l in range(orc.nlevels(0)):
        assert np.array_equal(host(H.counts(l)), orc.counts(l).astype(np.int32))
        for order in (1, 2):
            assert H.n_active(l, order) == int(orc.active(l, order).sum())
    for order in (1, 2):
        for l in range(orc.nlevels(order)):
            assert relerr(host(H.diag(l, order)), orc.diag(l, order)) <= 1e-15
    H.close()


# ---------------------------------------------------------------- operators
@pytest.mark.parametrize("name", ["sphere32", "rand_ragged", "rand_dirichlet", "patch_odd"])
def test_fold_equals_minus_residual_of_zero(mg, name):
    p, H, orc = _pair(name, mg)
    f = host(H.fold(dev(p.rho), None if p.dirichlet is None else dev(p.dirichlet)))
    ref = -orc.residual(0, np.zeros(p.shape), p.rho, p.dirichlet)
    assert relerr(f, ref) <= 1e-13
    H.close()


def _rand_on(act, seed):
    rng = np.random.default_rng(seed)
    return np.where(act, rng.standard_normal(act.shape), 0.0)


@pytest.mark.parametrize("name", ["sphere32", "holes64", "rand_ragged", "rand_dirichlet", "patch_odd"])
@pytest.mark.parametrize("order", [1, 2])
def test_smoother_residual_restrict_prolong_each_level(mg, name, order):
    p, H, orc = _pair(name, mg)
    for l in range(orc.nlevels(order)):
        act = orc.active(l, order).astype(bool)
        x = _rand_on(act, 10 + l)
        if l == 0:
            f_or = p.rho
            B = p.dirichlet
            f_gpu = H.fold(dev(p.rho), None if B is None else dev(B))
        else:
            f_or = _rand_on(act, 20 + l)
            B = None
            f_gpu = dev(f_or)
        for passes in (1, 2):
            got = host(H.smooth(l, dev(x), f_gpu, passes=passes, order=order))
            ref = orc.smooth(l, x, f_or, B, passes=passes, order=order)
            assert relerr(got, ref) <= TOL, (l, passes)
        got = host(H.residual(l, dev(x), f_gpu, order=order))
        ref = orc.residual(l, x, f_or, B, order=order)
        assert relerr(got, ref) <= TOL, l
        if l + 1 < orc.nlevels(order):
            got = host(H.restrict_residual(l, dev(x), f_gpu, order=order))
            refc = orc.restrict(l, ref, order=order)
            assert relerr(got, refc) <= TOL, l
            cact = orc.active(l + 1, order).astype(bool)
            xc = _rand_on(cact, 30 + l)
            got = host(H.prolong(l, dev(xc), dev(x), order=order))
            refp = orc.prolong(l, xc, x, order=order)
            assert relerr(got, refp, act) <= TOL, l
    H.close()


@pytest.mark.parametrize("name", ["sphere32", "holes64", "rand_dirichlet"])
@pytest.mark.parametrize("order", [1, 2])
def test_vcycle_matches_oracle_per_cycle(mg, name, order):
    p, H, orc = _pair(name, mg)
    B = p.dirichlet
    f = H.fold(dev(p.rho), None if B is None else dev(B))
    x_g = torch.zeros(p.shape, dtype=torch.float64, device="cuda")
    x_o = np.zeros(p.shape)
    act = p.mask == 1
    for c in range(3):
        x_g = H.vcycle(x_g, f, order=order)
        x_o = orc.vcycle(x_o, p.rho, B, order=order)
        assert relerr(host(x_g), x_o, act) <= TOL, c
    H.close()


# ---------------------------------------------------------------- solves
def _solve_pair(mg, name, tol=1e-10, **opts):
    p, H, orc = _pair(name, mg, **{k: v for k, v in opts.items() if k in ("min_coarse_dim",)})
    H.close()
    H = mg.Hierarchy(dev(p.mask), p.h, **opts)
    B = None if p.dirichlet is None else dev(p.dirichlet)
    phi, info = H.solve(dev(p.rho), None, B, tol=tol)
    oo = {k: v for k, v in opts.items() if k in ("n_pre", "n_post", "n_cycles", "max_cycles", "bc_order", "eta")}
    if "n_coarse_sweeps" in opts:
        oo["n_coarse"] = opts["n_coarse_sweeps"]
    ref, rinfo = orc.solve(p.rho, None, p.dirichlet, tol=tol, **oo)
    return p, H, host(phi), info, ref, rinfo


@pytest.mark.parametrize("name", ["sphere32", "holes64", "rand_ragged", "rand_dirichlet", "patch_odd", "deep_6144"])
def test_solve_matches_oracle(mg, name):
    p, H, got, info, ref, rinfo = _solve_pair(mg, name)
    act = p.mask == 1
    assert info["status"] == rinfo["status"] == 0
    assert info["cycles"] == rinfo["cycles"]
    assert info["switched_at"] == rinfo["switched_at"]
    assert relerr(got, ref, act) <= TOL
    # residual norms agree to 1e-6 relative down to the cancellation floor:
    # evaluating h^-2 (sum x_j - d x_i) - f loses about eps * ||f|| absolutely
    h1, h2 = np.array(info["history"]), np.array(rinfo["history"])
    assert np.all(np.abs(h1 - h2) <= 1e-6 * h2 + 1e-13 * info["r_ref"])
    assert info["r_final"] <= 1e-10 * info["r_ref"]
    H.close()


def test_solve_auto_switch_islands(mg):
    p, H, got, info, ref, rinfo = _solve_pair(mg, "porous64", tol=1e-10)
    assert rinfo["switched_at"] >= 1
    assert info["switched_at"] == rinfo["switched_at"] and info["order_used"] == 1
    assert info["cycles"] == rinfo["cycles"]
    assert relerr(got, ref, p.mask == 1) <= TOL
    # the next solve starts in first order (hold of 10 solves)
    B = None
    phi2, info2 = H.solve(dev(p.rho), None, B, tol=1e-10)
    assert info2["order_used"] == 1 and info2["switched_at"] == -1
    H.close()


@pytest.mark.parametrize("opts", [dict(bc_order="first"), dict(n_cycles=2), dict(n_pre=1, n_post=2),
                                  dict(use_graph=1), dict(n_pre=3, n_post=1, n_coarse_sweeps=7)])
def test_solve_options_match_oracle(mg, opts):
    p, H, got, info, ref, rinfo = _solve_pair(mg, "holes64", **opts)
    assert info["status"] == rinfo["status"]
    assert info["cycles"] == rinfo["cycles"]
    assert relerr(got, ref, p.mask == 1) <= TOL
    H.close()


def test_graph_replays_match_direct_launches(mg):
    """Each cycle replayed from a captured graph gives bit for bit what the
    directly launched kernels give, on every replay (38 replays per solve,
    host work between them) and across solves on one hierarchy."""
    p = gen.holes_problem(64, 2)
    rho = dev(p.rho)
    Hd = mg.Hierarchy(dev(p.mask), p.h, use_graph=0)
    Hg = mg.Hierarchy(dev(p.mask), p.h, use_graph=1)
    for _ in range(3):  # the first solve switches order; the next start in first order (hold)
        ref, rinfo = Hd.solve(rho, None, None, tol=1e-10)
        got, info = Hg.solve(rho, None, None, tol=1e-10)
        assert info["cycles"] == rinfo["cycles"] and info["order_used"] == rinfo["order_used"]
        assert info["history"] == rinfo["history"]
        assert np.array_equal(host(got), host(ref))
    Hd.close()
    Hg.close()


@pytest.mark.parametrize("name", ["sphere32", "holes64", "porous64", "rand_dirichlet"])
@pytest.mark.parametrize("opts", [dict(), dict(max_cycles=5), dict(bc_order="second"), dict(bc_order="first"),
                                  dict(n_pre=1, n_post=2), dict(n_cycles=2), dict(max_cycles=1)])
def test_input_norm_loop_equals_trailing_norm_loop(mg, name, opts):
    """FP64 solves with direct launches take each cycle's norm from the next
    cycle's first finest pass (deciding while that cycle runs); with captured
    graphs each cycle ends with the residual-norm march.  Both give the same
    norms bit for bit, so the same cycles, switch, histories and solution,
    through stops, order switches, the cycle cap and repeated solves."""
    p = PROBLEMS[name]()
    _print_case(name, p)
    rho = dev(p.rho)
    d = None if p.dirichlet is None else dev(p.dirichlet)
    Hd = mg.Hierarchy(dev(p.mask), p.h, use_graph=0, **opts)
    Hg = mg.Hierarchy(dev(p.mask), p.h, use_graph=1, **opts)
    for _ in range(2):
        ref, rinfo = Hg.solve(rho, None, d, tol=1e-10, check=False)
        got, info = Hd.solve(rho, None, d, tol=1e-10, check=False)
        assert (info["status"], info["cycles"], info["switched_at"], info["order_used"]) == \
            (rinfo["status"], rinfo["cycles"], rinfo["switched_at"], rinfo["order_used"]), (name, opts)
        assert info["history"] == rinfo["history"]
        assert np.array_equal(host(got), host(ref))
    # the halt flag is clear after the solve: an entry point still works
    x = Hd.smooth(0, got, Hd.fold(rho, d), passes=1)
    assert np.isfinite(host(x)).all()
    Hd.close()
    Hg.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_entry_points_after_a_solve(mg, precision):
    """A solve keeps one cycle in flight and lets the device stop it; the
    flag that does so must be clear afterwards: the residual norm of the
    returned solution equals the solve's final norm, and a second solve from
    that solution stops at once."""
    p = gen.holes_problem(64, 2)
    H = mg.Hierarchy(dev(p.mask), p.h, precision=precision)
    phi, info = H.solve(dev(p.rho), None, None, tol=1e-9)
    assert info["status"] == 0
    rn = H.residual_norm(dev(p.rho), phi, None)
    assert abs(rn - info["r_final"]) <= 1e-12 * info["r_final"]
    phi2, info2 = H.solve(dev(p.rho), phi.clone(), None, tol=1e-9)
    assert info2["status"] == 0 and info2["cycles"] == 0
    assert np.array_equal(host(phi2)[p.mask == 1], host(phi)[p.mask == 1])
    H.close()


def test_solve_from_guess_and_residual_norm(mg):
    p = gen.random_small_problem((32, 32, 32), 8, active_frac=0.8, blur=1.0)
    H = mg.Hierarchy(dev(p.mask), p.h)
    orc = O.Oracle(p.mask, p.h)
    rng = np.random.default_rng(0)
    guess = rng.standard_normal(p.shape)           # inactive cells carry junk: never read
    phi = dev(guess.copy())
    B = dev(p.dirichlet)
    rn = H.residual_norm(dev(p.rho), phi, B)
    assert abs(rn - orc.residual_norm(p.rho, np.where(p.mask == 1, guess, 0.0), p.dirichlet)) <= 1e-12 * rn
    phi, info = H.solve(dev(p.rho), phi, B, tol=1e-9)
    ref, rinfo = orc.solve(p.rho, np.where(p.mask == 1, guess, 0.0), p.dirichlet, tol=1e-9)
    got = host(phi)
    act = p.mask == 1
    assert info["cycles"] == rinfo["cycles"]
    assert relerr(got, ref, act) <= TOL
    assert np.array_equal(got[~act], guess[~act])   # inactive cells untouched
    H.close()


# ---------------------------------------------------------------- edge cases
def test_invalid_masks_are_rejected(mg):
    m = np.ones((16, 16, 16), np.int8)
    with pytest.raises(mg.MGError) as e:
        mg.Hierarchy(dev(m), 1 / 16)                 # active frame
    assert e.value.status == mg.MG_ERR_ARG
    m2 = gen.sphere_problem(16).mask.copy()
    m2[8, 8, 8] = 0
    with pytest.raises(mg.MGError) as e:
        mg.Hierarchy(dev(m2), 1 / 16)                # value other than +-1
    assert e.value.status == mg.MG_ERR_ARG
    with pytest.raises(mg.MGError) as e:
        mg.Hierarchy(dev(-np.ones((8, 8, 8), np.int8)), 1 / 8)
    assert e.value.status == mg.MG_ERR_NO_ACTIVE


def test_single_active_cell_and_odd_dims(mg):
    m = -np.ones((5, 7, 9), np.int8)                 # odd dims: one level only
    m[2, 3, 4] = 1
    rho = np.zeros(m.shape)
    rho[2, 3, 4] = 2.0
    H = mg.Hierarchy(dev(m), 0.5)
    assert H.nlevels(2) == 1
    phi, info = H.solve(dev(rho), tol=1e-12)
    orc = O.Oracle(m, 0.5)
    ref, rinfo = orc.solve(rho, tol=1e-12)
    assert info["cycles"] == rinfo["cycles"] == 1
    assert abs(host(phi)[2, 3, 4] - ref[2, 3, 4]) <= 1e-15 * abs(ref[2, 3, 4])
    assert ref[2, 3, 4] == pytest.approx(2.0 * 0.25 / -12.0)   # 12 phi/h^2 = -rho: exact
    H.close()


def test_zero_rhs_returns_at_once(mg):
    p = gen.sphere_problem(16)
    H = mg.Hierarchy(dev(p.mask), p.h)
    phi, info = H.solve(torch.zeros(p.shape, dtype=torch.float64, device="cuda"), tol=1e-10)
    assert info["status"] == 0 and info["cycles"] == 0
    assert not host(phi).any()
    H.close()


def test_max_cycles_status(mg):
    p = gen.holes_problem(n=64, seed=2)
    H = mg.Hierarchy(dev(p.mask), p.h, max_cycles=2)
    phi, info = H.solve(dev(p.rho), tol=1e-12)
    assert info["status"] == mg.MG_NOT_CONVERGED and info["cycles"] == 2
    H.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_kernel_timing_leaves_the_solve_unchanged(mg, precision):
    """Event pairs around one kind of finest-level launch inside a solve (the
    benchmark's in-solve kernel timing) leave every solve bit for bit as it
    was.  With n_pre = n_post = 2 a cycle has one pass that also forms the
    residual and its restriction, one that applies the prolongation and two
    others: in FP64 the first pass of every cycle after the first forms the
    input norm, except right after an order switch, so the plain ones are
    one per cycle plus those; in the mixed inner cycle both are plain.  A
    halted speculative cycle leaves no record."""
    p = gen.holes_problem(n=64, seed=2)
    kinds = ["plain", "residual", "prolong", "norm"]
    ref_H = mg.Hierarchy(dev(p.mask), p.h, precision=precision)
    refs = [ref_H.solve(dev(p.rho), tol=1e-10) for _ in kinds]
    H = mg.Hierarchy(dev(p.mask), p.h, precision=precision)
    for kind, (ref, rinfo) in zip(kinds, refs):
        H.kernel_timing(True, kind)
        got, info = H.solve(dev(p.rho), tol=1e-10)
        ms, n = H.kernel_timing_read()
        print(f"[case] holes64 {precision} {kind}: {n} launches, {ms / max(n, 1) * 1e3:.2f} us each", flush=True)
        assert info["cycles"] == rinfo["cycles"] and info["switched_at"] == rinfo["switched_at"]
        assert np.array_equal(host(got), host(ref)), kind
        cyc, sw = info["cycles"], int(info["switched_at"] >= 0)
        if precision == "fp64":
            expect = {"plain": cyc + 1 + sw, "residual": cyc, "prolong": cyc, "norm": cyc - 1 - sw}[kind]
        else:
            expect = {"plain": 2 * cyc, "residual": cyc, "prolong": cyc, "norm": 0}[kind]
        assert n == expect, (kind, n, expect)
        assert (ms > 0) == (n > 0)
    H.kernel_timing(False)
    H.solve(dev(p.rho), tol=1e-10)
    assert H.kernel_timing_read()[1] == n          # stopped: the record is kept
    H.kernel_timing(True)
    assert H.kernel_timing_read() == (0.0, 0)      # restarted: cleared
    G = mg.Hierarchy(dev(p.mask), p.h, use_graph=1)
    with pytest.raises(RuntimeError):
        G.kernel_timing(True)
    for X in (ref_H, H, G):
        X.close()


# ---------------------------------------------------------------- full size
def _check_solve_pair(info, rinfo, got, ref, act, what):
    assert info["status"] == rinfo["status"] == 0, what
    assert (info["cycles"], info["switched_at"], info["order_used"]) == \
        (rinfo["cycles"], rinfo["switched_at"], rinfo["order_used"]), (what, info["cycles"], rinfo["cycles"])
    err = relerr(got, ref, act)
    print(f"  {what}: cycles {info['cycles']} switched at {info['switched_at']} order {info['order_used']} "
          f"max rel diff {err:.2e}", flush=True)
    assert err <= TOL, what
    h1, h2 = np.array(info["history"]), np.array(rinfo["history"])
    assert np.all(np.abs(h1 - h2) <= 1e-6 * h2 + 1e-13 * info["r_ref"]), what


def test_full_size_holes256_bench_path_two_solves(mg):
    """The 256^3 masked workload solved exactly as the benchmark times it
    (default options: automatic boundary order, direct launches, each
    cycle's norm formed by the next cycle's first finest pass) twice on one
    fresh hierarchy: the first solve starts in second order and switches,
    the second starts held in first order.  The oracle solves the same
    sequence on one oracle hierarchy (which keeps the same hold); each
    solution is compared element by element after the same cycles."""
    p = gen.holes_problem(n=256, seed=2)
    _print_case("holes256", p)
    O.set_threads(min(16, os.cpu_count() or 1))
    H = mg.Hierarchy(dev(p.mask), p.h)
    orc = O.Oracle(p.mask, p.h)
    act = p.mask == 1
    rho = dev(p.rho)
    infos = []
    for k in range(2):
        phi, info = H.solve(rho, tol=1e-10)
        got = host(phi)
        ref, rinfo = orc.solve(p.rho, tol=1e-10)
        _check_solve_pair(info, rinfo, got, ref, act, f"solve {k}")
        infos.append(info)
    assert infos[0]["switched_at"] >= 1 and infos[0]["order_used"] == 1
    assert infos[1]["switched_at"] == -1 and infos[1]["order_used"] == 1
    H.close()


def test_full_size_holes256_second_order_two_cycles(mg):
    """Forced second order for two cycles (before the switch would fire):
    the coarse levels' second-order operators at full size, element by
    element."""
    p = gen.holes_problem(n=256, seed=2)
    H = mg.Hierarchy(dev(p.mask), p.h, bc_order="second", max_cycles=2)
    orc = O.Oracle(p.mask, p.h)
    phi, info = H.solve(dev(p.rho), tol=1e-12, check=False)
    ref, rinfo = orc.solve(p.rho, tol=1e-12, bc_order="second", max_cycles=2)
    assert info["cycles"] == rinfo["cycles"] == 2
    assert relerr(host(phi), ref, p.mask == 1) <= TOL
    H.close()


def test_full_size_holes256_variants_against_converged_oracle(mg):
    """Each solution the benchmark reports for the 256^3 workload (FP64,
    mixed precision, learned guess at stride 4, learned + mixed; all to
    1e-10 from their own starts) against the oracle run to its FP64 floor
    (1e-13), per result: max |phi - phi_oracle| / max |phi_oracle| <= 1e-9
    over the active cells (plain FP64 additionally matches the oracle's
    same-cycle iterate to 1e-11 in the bench-path test above)."""
    from paper_1104_1703_amd import guess
    p = gen.holes_problem(n=256, seed=2)
    _print_case("holes256", p)
    O.set_threads(min(16, os.cpu_count() or 1))
    ref, rinfo = O.Oracle(p.mask, p.h).solve(p.rho, tol=1e-13, max_cycles=120)
    assert rinfo["status"] == 0
    act = p.mask == 1
    mask, rho = dev(p.mask), dev(p.rho)
    net = guess.load_network()
    for name, prec, learned in (("fp64", "fp64", False), ("mixed", "mixed", False), ("learned", "fp64", True),
                                ("learned_mixed", "mixed", True)):
        H = mg.Hierarchy(mask, p.h, precision=prec, tune=1)
        phi0 = net.infer(rho, mask, stride=4) if learned else None
        phi, info = H.solve(rho, phi0, None, tol=1e-10)
        err = relerr(host(phi), ref, act)
        print(f"  {name}: cycles {info['cycles']} max rel error vs converged oracle {err:.2e}", flush=True)
        assert info["status"] == 0 and err <= 1e-9, name
        H.close()


def test_full_size_porous512_mixed_and_fp64(mg):
    """The 512^3 porous workload (4096 holes, most below the coarse cell size;
    k^-2 random-field rho) solved to 1e-10 in mixed precision and in FP64:
    both converged solutions pass the oracle's own FP64 residual test, and
    the mixed solution agrees with the FP64 one to 1e-9."""
    p = gen.porous_problem(512, seed=4)
    _print_case("porous512", p)
    act = p.mask == 1
    orc = O.Oracle(p.mask, p.h)
    out = {}
    for prec in ("mixed", "fp64"):
        H = mg.Hierarchy(dev(p.mask), p.h, precision=prec)
        phi, info = H.solve(dev(p.rho), tol=1e-10)
        print(f"[porous512] {prec}: status {info['status']} cycles {info['cycles']} "
              f"switched at {info['switched_at']} ms {info['ms']:.1f}", flush=True)
        assert info["status"] == 0
        got = host(phi)
        H.close()
        rr = orc.residual_norm(p.rho, np.where(act, got, 0.0))
        assert rr <= 1e-10 * info["r_ref"] * (1 + 1e-6), (prec, rr / info["r_ref"])
        out[prec] = got
    assert relerr(out["mixed"], out["fp64"], act) <= 1e-9


# ---------------------------------------------------------------- mixed precision
@pytest.mark.parametrize("name", ["sphere32", "holes64", "porous64", "rand_dirichlet"])
def test_mixed_precision_matches_converged_oracle(mg, name):
    """FP32 inner cycles inside FP64 iterative refinement: the FP64 residual
    reaches the same 1e-10 target and the solution matches the oracle's
    converged FP64 solution to 1e-9 (the exact-solution error of a 1e-10
    residual is below that for these operators)."""
    p = PROBLEMS[name]()
    _print_case(name, p)
    B = None if p.dirichlet is None else dev(p.dirichlet)
    H = mg.Hierarchy(dev(p.mask), p.h, precision="mixed")
    phi, info = H.solve(dev(p.rho), None, B, tol=1e-10)
    assert info["status"] == 0 and info["r_final"] <= 1e-10 * info["r_ref"]
    H2 = mg.Hierarchy(dev(p.mask), p.h)
    phi64, info64 = H2.solve(dev(p.rho), None, B, tol=1e-10)
    orc = O.Oracle(p.mask, p.h)
    ref, _ = orc.solve(p.rho, None, p.dirichlet, tol=1e-13, max_cycles=400)
    act = p.mask == 1
    err_mixed = relerr(host(phi), ref, act)
    err_fp64 = relerr(host(phi64), ref, act)
    print(f"[mixed] {name}: cycles mixed={info['cycles']} fp64={info64['cycles']} "
          f"err mixed={err_mixed:.2e} fp64={err_fp64:.2e}", flush=True)
    assert err_mixed <= 1e-9
    assert info["cycles"] <= info64["cycles"] + 3
    # the GPU's own residual of the mixed solution agrees with the oracle's
    rr = orc.residual_norm(p.rho, np.where(act, host(phi), 0.0), p.dirichlet)
    assert rr <= 1e-10 * info["r_ref"] * (1 + 1e-6)
    H.close()
    H2.close()


# ---------------------------------------------------------------- batched solver
def _batch_case(mg, probs, engine=None, **opts):
    B = mg.Batch([dev(p.mask) for p in probs], [p.h for p in probs], **opts)
    if engine is not None:
        B.set_engine(engine)
    rhos = [dev(p.rho) for p in probs]
    dirs = [None if p.dirichlet is None else dev(p.dirichlet) for p in probs]
    phis, infos, ms = B.solve(rhos, None, dirs, tol=1e-10, check=False)
    return B, [host(x) for x in phis], infos, ms


@pytest.mark.parametrize("opts", [dict(), dict(bc_order="second"), dict(n_cycles=2), dict(engine="persistent"),
                                  dict(engine="persistent", bc_order="second")])
def test_batch_matches_oracle_per_patch(mg, opts):
    """Uneven patches in one batch on the phase programs: every patch takes
    the same cycles, switch and solution as the oracle's own solve of it.  In
    forced second order the porous patch diverges (features below the coarse
    cell size, Sec. 4), in the oracle as in the batch."""
    probs = gen.patch_problems(count=6, seed=3) + [gen.sphere_problem(32), gen.holes_problem(n=64, seed=2),
                                                   gen.porous_problem(n=64, seed=4)]
    for p in probs:
        _print_case(p.name, p)
    B, got, infos, ms = _batch_case(mg, probs, **opts)
    assert B.phases(1) > 0 and B.phases(2) > 0 and B.grid > 0   # phase engine in use
    assert B.validate() == (0, "")
    oo = {k: v for k, v in opts.items() if k in ("bc_order", "n_cycles")}
    for p, x, info in zip(probs, got, infos):
        orc = O.Oracle(p.mask, p.h)
        ref, rinfo = orc.solve(p.rho, None, p.dirichlet, tol=1e-10, **oo)
        act = p.mask == 1
        assert info["status"] == rinfo["status"], (p.name, info["status"], rinfo["status"])
        if opts.get("bc_order") == "second" and p.name.startswith("porous"):
            assert info["status"] == mg.MG_ERR_DIVERGED
            continue
        assert info["status"] == 0, p.name
        assert info["cycles"] == rinfo["cycles"], (p.name, info["cycles"], rinfo["cycles"])
        assert info["switched_at"] == rinfo["switched_at"], p.name
        assert relerr(x, ref, act) <= TOL, p.name
    B.close()


def _oracle_solves(probs, **opts):
    """Oracle solves of many patches on the host cores, one patch per thread."""
    def one(p):
        O.set_threads(1)
        return O.Oracle(p.mask, p.h).solve(p.rho, None, p.dirichlet, tol=1e-10, **opts)
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(one, probs))


def test_batch_patches512_matches_oracle_per_patch(mg):
    """The batched workload itself: 512 patches (seed 3; edges log-uniform
    in 16..128, multiples of 8; blob masks; trilinear Dirichlet data;
    lognormal rho) in one batch with the default options, as the benchmark
    times it.  Every patch takes the oracle's status, cycles and switch, and
    its solution matches the oracle's element by element."""
    probs = gen.patch_problems(count=512, seed=3)
    print(f"[case] patches512: {sum(p.mask.size for p in probs)} cells, "
          f"{sum(p.n_active for p in probs)} active", flush=True)
    B, got, infos, ms = _batch_case(mg, probs)
    assert B.phases(2) > 0
    # the host-side check of every work item, descriptor, offset and LDS size
    # the phase kernels read (run at creation too, before any phase kernel)
    assert B.validate() == (0, "")
    B.close()
    # the same programs as one persistent launch per V-cycle, bit for bit.  A
    # fresh batch: a patch that switched order above starts its next solve on
    # the same hierarchy in first order (the hold of Sec. 4).
    B2, got_p, infos_p, ms_p = _batch_case(mg, probs, engine="persistent")
    print(f"  phase programs {ms:.1f} ms, persistent {ms_p:.1f} ms", flush=True)
    for p, x, xp, info, ip in zip(probs, got, got_p, infos, infos_p):
        assert (ip["status"], ip["cycles"], ip["switched_at"], ip["r_final"]) == \
            (info["status"], info["cycles"], info["switched_at"], info["r_final"]), p.name
        assert np.array_equal(xp, x), p.name
    B2.close()
    refs = _oracle_solves(probs)
    worst = 0.0
    for p, x, info, (ref, rinfo) in zip(probs, got, infos, refs):
        assert info["status"] == rinfo["status"] == 0, p.name
        assert (info["cycles"], info["switched_at"], info["order_used"]) == \
            (rinfo["cycles"], rinfo["switched_at"], rinfo["order_used"]), p.name
        err = relerr(x, ref, p.mask == 1)
        worst = max(worst, err)
        assert err <= TOL, (p.name, err)
    print(f"  worst patch max rel diff {worst:.2e}; cycles "
          f"{min(i['cycles'] for i in infos)}..{max(i['cycles'] for i in infos)}", flush=True)


@pytest.mark.parametrize("engine", ["phased", "phased_graph", "lockstep", "persistent"])
def test_batch_equals_single_solves_and_repeats(mg, engine):
    """24 patches solved twice (the second solve starts in first order where
    the first switched): on either engine every patch equals its own
    single-grid solve bit for bit, with the same cycles and switch."""
    probs = gen.patch_problems(count=22, seed=12) + [gen.porous_problem(n=64, seed=4), gen.sphere_problem(32)]
    B = mg.Batch([dev(p.mask) for p in probs], [p.h for p in probs], use_graph=int(engine == "phased_graph"))
    B.set_engine("persistent" if engine == "persistent" else engine != "lockstep")
    singles = [mg.Hierarchy(dev(p.mask), p.h) for p in probs]
    rhos = [dev(p.rho) for p in probs]
    dirs = [None if p.dirichlet is None else dev(p.dirichlet) for p in probs]
    for rep in range(2):
        print(f"[case] {engine} batch of {len(probs)}, solve {rep}", flush=True)
        got, infos, ms = B.solve(rhos, dirichlets=dirs, tol=1e-10)
        assert ms > 0
        for p, H, x, info, r, d in zip(probs, singles, got, infos, rhos, dirs):
            ref, rinfo = H.solve(r, None, d, tol=1e-10)
            assert info["status"] == rinfo["status"] == 0, p.name
            assert (info["cycles"], info["switched_at"], info["order_used"]) == \
                (rinfo["cycles"], rinfo["switched_at"], rinfo["order_used"]), p.name
            assert info["r0"] == rinfo["r0"] and info["r_ref"] == rinfo["r_ref"], p.name
            assert info["r_final"] == rinfo["r_final"], p.name
            assert np.array_equal(host(x), host(ref)), p.name
        if rep == 0:
            assert any(i["switched_at"] > 0 for i in infos)
    assert any(i["order_used"] == 1 for i in infos)
    for H in singles:
        H.close()
    B.close()


@pytest.mark.parametrize("graph", [0, 1, "persistent"])
def test_batch_mixes_whole_workgroup_patches(mg, graph):
    """Patches whose whole hierarchy runs in one workgroup (sphere 16^3) or
    that have a single level (6 x 10 x 10) get the residual-norm march in the
    pre program while the others' first pass forms the norm: every patch
    still equals its single-grid solve bit for bit."""
    probs = gen.patch_problems(count=4, seed=12) + [gen.sphere_problem(16), gen.sphere_problem(32),
                                                    gen.random_small_problem((6, 10, 10), 7, active_frac=0.8)]
    for p in probs:
        _print_case(p.name, p)
    B = mg.Batch([dev(p.mask) for p in probs], [p.h for p in probs], use_graph=int(graph == 1))
    if graph == "persistent":
        B.set_engine("persistent")
    assert B.phases(1) > 0 and B.phases(2) > 0
    rhos = [dev(p.rho) for p in probs]
    dirs = [None if p.dirichlet is None else dev(p.dirichlet) for p in probs]
    got, infos, _ = B.solve(rhos, dirichlets=dirs, tol=1e-10, check=False)
    for p, x, info, r, d in zip(probs, got, infos, rhos, dirs):
        H = mg.Hierarchy(dev(p.mask), p.h)
        ref, rinfo = H.solve(r, None, d, tol=1e-10, check=False)
        assert info["status"] == rinfo["status"], p.name
        assert (info["cycles"], info["switched_at"], info["r_final"]) == \
            (rinfo["cycles"], rinfo["switched_at"], rinfo["r_final"]), p.name
        assert np.array_equal(host(x), host(ref)), p.name
        H.close()
    B.close()


@pytest.mark.parametrize("engine", ["phased", "persistent"])
def test_batch_guess_and_max_cycles(mg, engine):
    """Phase engines with a non-zero guess (junk in inactive cells must not
    leak) and a cycle cap: the same iterate as single solves, MG_NOT_CONVERGED
    reported per patch."""
    probs = gen.patch_problems(count=5, seed=21)
    B = mg.Batch([dev(p.mask) for p in probs], [p.h for p in probs], max_cycles=3)
    B.set_engine(engine)
    assert B.phases(2) > 0
    rng = np.random.default_rng(5)
    guesses = [rng.standard_normal(p.mask.shape) for p in probs]
    rhos = [dev(p.rho) for p in probs]
    dirs = [None if p.dirichlet is None else dev(p.dirichlet) for p in probs]
    got, infos, _ = B.solve(rhos, [dev(g) for g in guesses], dirs, tol=1e-10)
    for p, g, x, info, r, d in zip(probs, guesses, got, infos, rhos, dirs):
        H = mg.Hierarchy(dev(p.mask), p.h, max_cycles=3)
        ref, rinfo = H.solve(r, dev(g), d, tol=1e-10, check=False)
        assert info["cycles"] == rinfo["cycles"] == 3 and info["status"] == rinfo["status"] == mg.MG_NOT_CONVERGED
        assert np.array_equal(host(x), host(ref)), p.name
        H.close()
    B.close()


def test_batch_odd_pass_count_runs_per_patch(mg):
    """1 + 2 passes leave the finest iterate in the other buffer after each
    cycle: no phase programs, the per-patch engine solves, oracle parity."""
    probs = gen.patch_problems(count=3, seed=5) + [gen.sphere_problem(16)]
    B, got, infos, ms = _batch_case(mg, probs, n_pre=1, n_post=2)
    assert B.grid == 0 and B.phases(2) == 0
    with pytest.raises(mg.MGError) as e:
        B.set_engine(True)
    assert e.value.status == mg.MG_ERR_ARG
    for p, x, info in zip(probs, got, infos):
        ref, rinfo = O.Oracle(p.mask, p.h).solve(p.rho, None, p.dirichlet, tol=1e-10, n_pre=1, n_post=2)
        assert info["status"] == rinfo["status"] == 0, p.name
        assert info["cycles"] == rinfo["cycles"] and info["switched_at"] == rinfo["switched_at"], p.name
        assert relerr(x, ref, p.mask == 1) <= TOL, p.name
    B.close()


@pytest.mark.parametrize("opts", [dict(), dict(n_cycles=2)])
def test_batch_per_patch_engine_matches_oracle(mg, opts):
    probs = gen.patch_problems(count=5, seed=11) + [gen.sphere_problem(32), gen.porous_problem(n=64, seed=4)]
    for p in probs:
        _print_case(p.name, p)
    B = mg.Batch([dev(p.mask) for p in probs], [p.h for p in probs], **opts)
    B.set_engine(False)
    got, infos, ms = B.solve([dev(p.rho) for p in probs], None,
                             [None if p.dirichlet is None else dev(p.dirichlet) for p in probs], tol=1e-10)
    for p, x, info in zip(probs, got, infos):
        orc = O.Oracle(p.mask, p.h)
        oo = {k: v for k, v in opts.items() if k in ("n_cycles",)}
        ref, rinfo = orc.solve(p.rho, None, p.dirichlet, tol=1e-10, **oo)
        assert info["status"] == rinfo["status"] == 0, p.name
        assert info["cycles"] == rinfo["cycles"] and info["switched_at"] == rinfo["switched_at"], p.name
        assert relerr(host(x), ref, p.mask == 1) <= TOL, p.name
    B.close()


# ---------------------------------------------------------------- finest pass with the residual
@pytest.mark.parametrize("name", ["sphere32", "holes64", "rand_ragged", "rand_dirichlet", "porous64", "patch_odd"])
@pytest.mark.parametrize("opts", [dict(), dict(precision="mixed"), dict(item_depth_fine=8), dict(item_depth_fine=32),
                                  dict(n_pre=3, n_post=3), dict(n_pre=1, n_post=2),
                                  dict(precision="mixed", n_pre=1, n_post=2), dict(n_cycles=2),
                                  dict(use_graph=1), dict(bc_order="first")])
def test_residual_pass_solve_equals_residual_march(mg, name, opts):
    """The last finest pre-smoothing pass that also forms the residual and its
    R1 restriction (3-cell halo, residual one plane behind the black
    half-sweep) gives the same solves as a plain pass followed by the residual
    march, bit for bit: cycles, switch, norm history and solution, on a fresh
    hierarchy's first solve and on the held second one (also from a zero
    input in the mixed inner cycle with one pre-smoothing pass)."""
    p = PROBLEMS[name]()
    _print_case(name, p)
    rho = dev(p.rho)
    d = None if p.dirichlet is None else dev(p.dirichlet)
    out = []
    for fr in (0, 1):
        H = mg.Hierarchy(dev(p.mask), p.h, fuse_restrict=fr, **opts)
        for _ in range(2):
            phi, info = H.solve(rho, None, d, tol=1e-10)
            out.append((host(phi), info))
        H.close()
    for (a, ia), (b, ib) in zip(out[:2], out[2:]):
        assert ia["status"] == ib["status"] == 0, (name, opts)
        assert (ia["cycles"], ia["switched_at"], ia["order_used"]) == \
            (ib["cycles"], ib["switched_at"], ib["order_used"]), (name, opts)
        assert ia["history"] == ib["history"], (name, opts)
        assert np.array_equal(a, b), (name, opts)


# ---------------------------------------------------------------- fused pairs of passes
@pytest.mark.parametrize("name", ["sphere32", "holes64", "rand_ragged", "rand_dirichlet", "patch_odd"])
def test_fused_passes_equal_single_passes_each_level(mg, name):
    """Two passes in one march (4-cell halo, four half-sweeps one plane apart)
    give what two single passes give, bit for bit, on every level and order,
    for 2, 3 and 4 passes (the odd one left as a single pass)."""
    p, H1, orc = _pair(name, mg)
    H2 = mg.Hierarchy(dev(p.mask), p.h, fuse_passes=1)
    for order in (1, 2):
        for l in range(orc.nlevels(order)):
            act = orc.active(l, order).astype(bool)
            x = dev(_rand_on(act, 30 + l))
            f = dev(_rand_on(act, 40 + l) * (1.0 + l))
            for passes in (2, 3, 4):
                a = host(H1.smooth(l, x, f, passes=passes, order=order))
                b = host(H2.smooth(l, x, f, passes=passes, order=order))
                assert np.array_equal(a, b), (name, order, l, passes)
    H1.close()
    H2.close()


@pytest.mark.parametrize("name", ["sphere32", "holes64", "rand_dirichlet", "porous64", "patch_odd"])
@pytest.mark.parametrize("opts", [dict(), dict(precision="mixed"), dict(n_pre=3, n_post=3), dict(n_pre=1, n_post=2),
                                  dict(n_cycles=2), dict(n_post=0), dict(use_graph=1),
                                  dict(use_graph=1, n_pre=3, n_post=3), dict(use_graph=1, n_pre=1, n_post=2)])
def test_fused_solve_equals_unfused_solve(mg, name, opts):
    """Whole solves with fused pairs of passes (the finest prolongation pass
    fused with the pass after it) equal the unfused solves bit for bit:
    cycles, switch, norm history and solution; with captured graphs the
    replays track the finest buffer across cycles by the fused launch count."""
    p = PROBLEMS[name]()
    _print_case(name, p)
    rho = dev(p.rho)
    d = None if p.dirichlet is None else dev(p.dirichlet)
    out = []
    for fuse in (0, 1):
        H = mg.Hierarchy(dev(p.mask), p.h, fuse_passes=fuse, **opts)
        phi, info = H.solve(rho, None, d, tol=1e-10)
        out.append((host(phi), info))
        H.close()
    (a, ia), (b, ib) = out
    assert ia["status"] == ib["status"] == 0, (name, opts)
    assert (ia["cycles"], ia["switched_at"], ia["order_used"]) == (ib["cycles"], ib["switched_at"], ib["order_used"])
    assert ia["history"] == ib["history"]
    assert np.array_equal(a, b)
