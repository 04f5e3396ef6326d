"""GPU one-way nested levels (csrc/amr.hip, paper_1104_1703_amd/amr.py)
against the oracle (oracle/amr.py): interface Dirichlet values, the 5-point
gradient, the whole nested solve and its accuracy orders (Sec. 5.1)."""
import numpy as np
import pytest
import torch

from oracle import amr as OA
from oracle import oracle as O
from paper_1104_1703_amd import gen

pytestmark = pytest.mark.gpu


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


COARSE = ((12, 10, 14), 0.1, (0.05, -0.02, 0.1))
PATCH = ((10, 8, 12), 0.05, (0.35, 0.3, 0.45))


def test_amr_dirichlet_matches_oracle(mg):
    """Interior centres, face centres, the 2 g - B_i rule and the zero edges:
    the same trilinear weights and sums, contraction off on the GPU."""
    rng = np.random.default_rng(1)
    (cs, hc, oc), (fs, hf, of) = COARSE, PATCH
    pc = rng.standard_normal(cs)
    ref = OA.patch_dirichlet(pc, hc, oc, fs, hf, of)
    got = host(mg.amr_dirichlet(dev(pc), hc, oc, fs, hf, of))
    assert np.abs(got - ref).max() <= 1e-15 * np.abs(ref).max()


@pytest.mark.parametrize("with_coarse", [True, False])
def test_amr_grad5_matches_oracle(mg, with_coarse):
    rng = np.random.default_rng(2)
    (cs, hc, oc), (fs, hf, of) = ((16, 14, 18), 0.1, (0.0, -0.1, 0.05)), PATCH
    phi = rng.standard_normal(fs)
    mask = (rng.random(fs) < 0.8).astype(np.int8) * 2 - 1
    mask[0], mask[-1], mask[:, 0], mask[:, -1], mask[:, :, 0], mask[:, :, -1] = -1, -1, -1, -1, -1, -1
    if with_coarse:
        pc = rng.standard_normal(cs)
        ref = OA.grad5(phi, mask == 1, hf, of, coarse=(pc, hc, oc))
        got = host(mg.amr_grad5(dev(phi), dev(mask), hf, of, coarse=(dev(pc), hc, oc)))
    else:
        bnd = rng.standard_normal(fs)
        ref = OA.grad5(phi, mask == 1, hf, of, bnd=bnd)
        got = host(mg.amr_grad5(dev(phi), dev(mask), hf, of, bnd=dev(bnd)))
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.abs(got[ok] - ref[ok]).max() <= 1e-13 * np.abs(ref[ok]).max()


def test_amr_rejects_uncovered_patch(mg):
    (cs, hc, oc), (fs, hf, _) = COARSE, PATCH
    pc = dev(np.zeros(cs))
    with pytest.raises(mg.MGError) as e:
        mg.amr_dirichlet(pc, hc, oc, fs, hf, (0.0, 0.0, 0.0))  # patch face below the first coarse centre
    assert e.value.status == mg.MG_ERR_ARG
    with pytest.raises(mg.MGError) as e:
        mg.amr_grad5(dev(np.zeros(fs)), dev(gen.frame_mask(fs)), hf, (0.35, 0.3, 1.0), coarse=(pc, hc, oc))
    assert e.value.status == mg.MG_ERR_ARG


def _oracle_solve(mask, h, rho, B):
    phi, info = O.Oracle(mask, h).solve(rho, None, B, tol=1e-12, max_cycles=400)
    assert info["status"] == 0
    return phi


def test_nested_solve_matches_oracle(mg):
    """Three levels at 16^3 solved one way on the GPU and by the oracle:
    every level's potential and gradient agree (both to 1e-12), and so do the
    composite-grid errors."""
    from paper_1104_1703_amd import amr
    levels, ms = amr.solve_nested(16, 2, r0=0.1, tol=1e-12)
    ref = OA.solve_nested(16, 2, 0.1, _oracle_solve)
    gref = OA.nested_grads(ref)
    for L, R, G in zip(levels, ref, gref):
        assert L.info["status"] == 0
        act = gen.frame_mask(L.shape) == 1
        phi = host(L.phi)
        assert np.abs(phi - R[0])[act].max() <= 1e-10 * np.abs(R[0][act]).max()
        assert np.abs(host(L.B) - R[2])[act].max() <= 1e-10 * np.abs(R[2]).max()
        g = host(L.grad)
        assert np.array_equal(np.isnan(g), np.isnan(G))  # level-0 stencils leaving the array
        ok = ~np.isnan(G)
        assert np.abs(g - G)[ok].max() <= 1e-8 * np.abs(G[ok]).max()
    got = [(host(L.phi), None, host(L.B), L.shape, L.h, L.origin) for L in levels]
    e_gpu = OA.composite_errors(got, [host(L.grad) for L in levels], 0.1)
    e_ref = OA.composite_errors(ref, gref, 0.1)
    for k in e_ref:
        assert abs(e_gpu[k] - e_ref[k]) <= 1e-6 * e_ref[k], k


def test_nested_accuracy_orders_on_gpu(mg):
    """The accuracy study on the GPU path with three refined levels at 32^3,
    64^3 and 128^3 (finest cell 1/1024): potential second order, gradient
    maximum first order at the interfaces, gradient L2 near second order."""
    from paper_1104_1703_amd import amr
    errs = []
    for n in (32, 64, 128):
        levels, ms = amr.solve_nested(n, 3, r0=0.1, tol=1e-12)
        got = [(host(L.phi), None, host(L.B), L.shape, L.h, L.origin) for L in levels]
        errs.append(OA.composite_errors(got, [host(L.grad) for L in levels], 0.1))
        print(f"[amr] n={n} ms={ms:.1f} " + " ".join(f"{k}={v:.3e}" for k, v in errs[-1].items()), flush=True)
    for a, b in zip(errs, errs[1:]):
        order = {k: np.log2(a[k] / b[k]) for k in a}
        assert order["phi_linf"] > 1.8 and order["phi_l2"] > 1.8, order
        assert 0.5 < order["grad_linf"] < 1.3, order
        assert order["grad_l2"] > 1.4, order
