"""Pins of the one-way nested-level oracle (oracle/amr.py; Sec. 3 one-way
interface, Sec. 5.1 accuracy tests), CPU only."""
import numpy as np
import pytest

from oracle import amr
from oracle import oracle as O
from paper_1104_1703_amd import gen


def _lin(coef):
    return lambda P: coef[0] + coef[1] * P[..., 0] + coef[2] * P[..., 1] + coef[3] * P[..., 2]


def test_interpolation_and_interface_values_reproduce_linear_fields():
    """Trilinear interpolation is exact on linear fields, so are the patch's
    interior B and its face values (B_i + B_j)/2 (the values the solver
    reads): no term is dropped and no face misplaced."""
    rng = np.random.default_rng(0)
    f = _lin(rng.standard_normal(4))
    shape_c, hc, oc = (12, 10, 14), 0.1, (0.05, -0.02, 0.1)
    pc = f(gen.level_centres(shape_c, hc, oc))
    pts = np.array(oc) + 0.3 + rng.random((200, 3)) * 0.6
    assert np.abs(amr.interp(pc, hc, oc, pts) - f(pts)).max() < 1e-14
    shape, hf, of = (10, 8, 12), 0.05, (0.35, 0.3, 0.45)
    B = amr.patch_dirichlet(pc, hc, oc, shape, hf, of)
    ctr = gen.level_centres(shape, hf, of)
    assert np.abs(B[1:-1, 1:-1, 1:-1] - f(ctr[1:-1, 1:-1, 1:-1])).max() < 1e-14
    inner = (slice(1, -1), slice(1, -1))
    for ax in range(3):
        for fr, ac in ((0, 1), (-1, -2)):
            sf = [slice(1, -1)] * 3
            sa = [slice(1, -1)] * 3
            sf[2 - ax], sa[2 - ax] = fr, ac
            face = 0.5 * (B[tuple(sf)] + B[tuple(sa)])
            pts = 0.5 * (ctr[tuple(sf)] + ctr[tuple(sa)])
            assert np.abs(face - f(pts)).max() < 1e-14, (ax, fr)
    with pytest.raises(ValueError):
        amr.interp(pc, hc, oc, np.array([[0.0, 0.0, 0.0]]))


def test_five_point_gradient_is_exact_on_quartics_and_linear_coarse_data():
    """The 5-point difference is exact for polynomials up to degree 4 along
    the differentiated axis; beyond the level, a linear coarser field gives
    exact values, so a linear potential's gradient is exact everywhere."""
    shape, h, o = (14, 13, 15), 0.07, (0.1, 0.0, -0.05)
    c = gen.level_centres(shape, h, o)
    X, Y, Z = c[..., 0], c[..., 1], c[..., 2]
    q = X ** 4 + 2 * Y ** 3 - Z ** 4 + X * Y - 3 * Y * Z
    ge = np.stack([4 * X ** 3 + Y, 6 * Y ** 2 + X - 3 * Z, -4 * Z ** 3 - 3 * Y])
    act = gen.frame_mask(shape) == 1
    g = amr.grad5(q, act, h, o, bnd=q)
    inner = (slice(None), slice(2, -2), slice(2, -2), slice(2, -2))
    assert np.abs(g[inner] - ge[inner]).max() < 1e-11
    assert np.isnan(g[0][1, 1, 1])  # needs x index -1 with no coarser level
    f = _lin([0.3, 1.5, -2.0, 0.7])
    shape_c, hc, oc = (12, 12, 12), 2 * h, (o[0] - 0.3, o[1] - 0.3, o[2] - 0.3)
    pc = f(gen.level_centres(shape_c, hc, oc))
    g = amr.grad5(f(c), act, h, o, coarse=(pc, hc, oc))
    for ax, v in enumerate((1.5, -2.0, 0.7)):
        assert np.abs(g[ax][act] - v).max() < 1e-11


def _solve(mask, h, rho, B):
    phi, info = O.Oracle(mask, h).solve(rho, None, B, tol=1e-12, max_cycles=400)
    assert info["status"] == 0
    return phi


def _errors(n, depth, exact_interface=False, r0=0.1):
    lev = amr.solve_nested(n, depth, r0, _solve, exact_interface=exact_interface)
    return amr.composite_errors(lev, amr.nested_grads(lev, r0, exact_interface), r0)


def test_accuracy_orders_of_the_one_way_interface():
    """Sec. 5.1 on the 3D ln profile with two refined levels: the potential
    converges at second order; the gradient's maximum error is degraded to
    first order by the interpolated interface values (its L2 error stays
    close to second order); with exact values at the interfaces (the paper's
    control run) the gradient's maximum error is second order again."""
    e = [_errors(n, 2) for n in (16, 32)]
    order = {k: np.log2(e[0][k] / e[1][k]) for k in e[0]}
    assert order["phi_linf"] > 1.8 and order["phi_l2"] > 1.8, order
    assert 0.5 < order["grad_linf"] < 1.3, order
    assert order["grad_l2"] > 1.5, order
    x = [_errors(n, 2, exact_interface=True) for n in (16, 32)]
    xo = {k: np.log2(x[0][k] / x[1][k]) for k in x[0]}
    assert xo["grad_linf"] > 1.7 and xo["phi_linf"] > 1.8, xo
    assert x[1]["grad_linf"] < 0.5 * e[1]["grad_linf"]
