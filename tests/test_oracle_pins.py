"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics, independent of the oracle's own code.

Each pin is chosen so that a plausible slip in the oracle (a dropped
neighbour, a wrong h scaling, a transposed transfer, a wrong colour order, a
missing coarse-level reset) fails at least one test:

* closed-form discrete solutions for sine right-hand sides (operator scale,
  boundary, convergence to the discrete solution);
* the paper's printed FFT error columns (Sec. 5.4, Tables 12 and 14);
* exact solves by dense LU (own assembly of A by Kronecker sums) and by
  DST-I diagonalisation for random right-hand sides;
* Fourier symbols of A, of full weighting, of linear interpolation and of
  the weighted-Jacobi sweep on sine modes;
* the red-black invariant (zero residual on the colour just relaxed);
* exactness of the 1-DOF coarsest level;
* symmetry and affinity of the V-cycle map;
* the asymptotic convergence factor against local Fourier analysis.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.fft

import lfa
from paper_1208_4247_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def lam_h(ks, h):
    """Discrete Laplacian eigenvalue of prod sin(k_i pi x_i): the symbol of
    the 5-/7-point scheme, sum_i (4/h^2) sin^2(k_i pi h / 2)."""
    return sum(4.0 / h ** 2 * math.sin(k * math.pi * h / 2) ** 2 for k in ks)


def dense_A(d, m):
    """A assembled from scratch as a Kronecker sum of 1D second differences
    (h^-2 tridiag(-1, 2, -1)); C-order flattening puts x last (fastest)."""
    h = 1.0 / (m + 1)
    T = (np.diag(2.0 * np.ones(m)) - np.diag(np.ones(m - 1), 1) - np.diag(np.ones(m - 1), -1)) / h ** 2
    I = np.eye(m)
    if d == 2:
        return np.kron(I, T) + np.kron(T, I)
    return np.kron(I, np.kron(I, T)) + np.kron(I, np.kron(T, I)) + np.kron(T, np.kron(I, I))


def dst_solve(f):
    """Exact solution of A u = f by the sine transform (DST-I diagonalises A
    with eigenvalues lam_h)."""
    d, m = f.ndim, f.shape[0]
    h = 1.0 / (m + 1)
    lam1 = 4.0 / h ** 2 * np.sin(np.arange(1, m + 1) * np.pi * h / 2) ** 2
    if d == 2:
        lam = lam1[:, None] + lam1[None, :]
    else:
        lam = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]
    fh = scipy.fft.dstn(f, type=1)
    return scipy.fft.idstn(fh / lam, type=1)


def node_colour(d, m):
    """0 where the node-index sum is even (red), 1 where odd (black)."""
    idx = np.indices((m,) * d).sum(axis=0) + d  # node indices are storage + 1
    return idx % 2


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


# ----------------------------------------------------------------- operator


@pytest.mark.parametrize("d,m,ks", [(2, 15, (1, 1)), (2, 31, (3, 7)), (3, 15, (1, 2, 5)), (3, 7, (7, 1, 3))])
def test_operator_symbol(orc, d, m, ks):
    h = 1.0 / (m + 1)
    phi = wl.sine_product(d, m, ks)
    Aphi = orc.apply_A(phi)
    assert np.max(np.abs(Aphi - lam_h(ks, h) * phi)) <= 1e-12 * lam_h(ks, h)


@pytest.mark.parametrize("d,m", [(2, 7), (3, 3), (3, 7)])
def test_operator_matches_dense_assembly(orc, d, m):
    v = wl.rhs_uniform(d, m, seed=11)
    A = dense_A(d, m)
    np.testing.assert_allclose(orc.apply_A(v).ravel(), A @ v.ravel(), rtol=1e-13, atol=1e-9)
    f = wl.rhs_uniform(d, m, seed=12)
    r = orc.residual(v, f)
    np.testing.assert_allclose(r.ravel(), f.ravel() - A @ v.ravel(), rtol=1e-13, atol=1e-9)


def test_norm_is_euclidean(orc):
    r = wl.rhs_uniform(3, 15, seed=5)
    assert orc.norm2(r) == pytest.approx(float(np.sqrt(np.sum(r * r))), rel=1e-14)


# ----------------------------------------------------------------- transfers


@pytest.mark.parametrize("d,mc,ks", [(2, 15, (1, 1)), (2, 15, (5, 11)), (3, 7, (1, 3, 6)), (3, 15, (9, 2, 4))])
def test_full_weighting_symbol(orc, d, mc, ks):
    """FW of a fine sine mode = prod cos^2(k_i pi h_f / 2) times the mode at
    the coarse nodes."""
    mf = 2 * mc + 1
    hf = 1.0 / (mf + 1)
    fine = wl.sine_product(d, mf, ks)
    coarse = wl.sine_product(d, mc, ks)
    fac = np.prod([math.cos(k * math.pi * hf / 2) ** 2 for k in ks])
    np.testing.assert_allclose(orc.restrict_fw(fine), fac * coarse, atol=1e-14)


@pytest.mark.parametrize("d,mc,ks", [(2, 15, (1, 1)), (2, 7, (3, 5)), (3, 7, (1, 3, 6)), (3, 3, (2, 1, 3))])
def test_linear_interpolation_symbol(orc, d, mc, ks):
    """Interpolating a coarse sine mode: exact at fine nodes that coincide
    with coarse ones along an axis; at odd fine nodes along an axis the mode
    picks up a factor cos(k pi h_f)."""
    mf = 2 * mc + 1
    hf = 1.0 / (mf + 1)
    coarse = wl.sine_product(d, mc, ks)
    got = orc.prolong_add(coarse, np.zeros((mf,) * d))
    want = wl.sine_product(d, mf, ks)
    for ax in range(d):
        k = ks[ax]
        odd = (np.arange(1, mf + 1) % 2 == 1)  # odd fine node index along axis
        fac = np.where(odd, math.cos(k * math.pi * hf), 1.0)
        shape = [1] * d
        shape[d - 1 - ax] = mf  # axis 0 (x) is the last numpy axis
        want = want * fac.reshape(shape)
    np.testing.assert_allclose(got, want, atol=1e-14)


@pytest.mark.parametrize("d,mc", [(2, 7), (3, 3)])
def test_restriction_is_scaled_interpolation_transpose(orc, d, mc):
    """FW = 2^-d P^T: <R r, e> = 2^-d <r, P e> for random r, e."""
    mf = 2 * mc + 1
    r = wl.rhs_uniform(d, mf, seed=21)
    e = wl.rhs_uniform(d, mc, seed=22)
    lhs = float(np.sum(orc.restrict_fw(r) * e))
    rhs = float(np.sum(r * orc.prolong_add(e, np.zeros((mf,) * d)))) / 2 ** d
    assert lhs == pytest.approx(rhs, rel=1e-13)


# ----------------------------------------------------------------- smoothers


@pytest.mark.parametrize("d,m", [(2, 15), (2, 31), (3, 7), (3, 15)])
def test_rb_invariant(orc, d, m):
    """After a forward sweep (red, black) the residual vanishes on black
    nodes; after a backward sweep (black, red) on red nodes."""
    f = wl.rhs_uniform(d, m, seed=31)
    u0 = wl.rhs_uniform(d, m, seed=32)
    col = node_colour(d, m)
    scale = np.max(np.abs(orc.apply_A(u0))) + np.max(np.abs(f))
    uf = orc.rbgs(u0, f, 1, backward=False)
    rf = orc.residual(uf, f)
    assert np.max(np.abs(rf[col == 1])) <= 1e-13 * scale
    assert np.max(np.abs(rf[col == 0])) > 1e-3 * scale
    ub = orc.rbgs(u0, f, 1, backward=True)
    rb = orc.residual(ub, f)
    assert np.max(np.abs(rb[col == 0])) <= 1e-13 * scale
    assert np.max(np.abs(rb[col == 1])) > 1e-3 * scale


def test_rb_red_is_even_node_sum(orc):
    """The first half-sweep of a forward sweep touches exactly the nodes with
    an even node-index sum (node (1,1) in 2D is red; node (1,1,1) in 3D is
    black)."""
    for d, m in [(2, 7), (3, 7)]:
        f = wl.rhs_uniform(d, m, seed=33)
        u0 = np.zeros((m,) * d)
        u1 = orc.rbgs_color(u0, f, 0)
        col = node_colour(d, m)
        assert np.all(u1[col == 1] == 0.0)
        assert np.all(u1[col == 0] != 0.0)
    assert node_colour(2, 3)[0, 0] == 0 and node_colour(3, 3)[0, 0, 0] == 1


@pytest.mark.parametrize("d,m,ks,omega", [(2, 31, (3, 5), 0.8), (3, 15, (2, 7, 1), 6 / 7), (2, 15, (1, 1), 2 / 3)])
def test_weighted_jacobi_symbol(orc, d, m, ks, omega):
    """With f = 0 a Jacobi sweep scales a sine mode by
    1 - omega h^2 lam_h / (2d)."""
    h = 1.0 / (m + 1)
    phi = wl.sine_product(d, m, ks)
    got = orc.wj(phi, np.zeros_like(phi), omega, 1)
    fac = 1.0 - omega * h * h * lam_h(ks, h) / (2 * d)
    np.testing.assert_allclose(got, fac * phi, atol=1e-14)


def test_coarsest_level_exact(orc):
    """On the 1-DOF level the cycle is the exact solve (u = h^2 f / 2d)."""
    for d in (2, 3):
        f = np.full((1,) * d, 3.7)
        u = orc.vcycle(np.zeros((1,) * d), f)
        assert abs(orc.residual(u, f).item()) <= 1e-14 * 3.7
        u, it, relres, st, _ = orc.solve(f)
        assert it == 1 and st == 0 and relres <= 1e-15


# ----------------------------------------------------------------- exact solves


@pytest.mark.parametrize("d,m", [(2, 3), (2, 7), (2, 15), (3, 3), (3, 7)])
def test_solve_matches_dense_lu(orc, d, m):
    f = wl.rhs_uniform(d, m, seed=40 + m)
    u_lu = np.linalg.solve(dense_A(d, m), f.ravel()).reshape(f.shape)
    u, it, relres, st, _ = orc.solve(f, rtol=1e-14, maxit=60)
    assert st == 0
    assert rel(u, u_lu) <= 1e-12


@pytest.mark.parametrize("d,m", [(2, 127), (3, 31), (3, 63)])
def test_solve_matches_dst(orc, d, m):
    f = wl.rhs_uniform(d, m, seed=50 + m)
    u, it, relres, st, _ = orc.solve(f, rtol=1e-13, maxit=60)
    assert st == 0
    assert rel(u, dst_solve(f)) <= 1e-10


@pytest.mark.parametrize("d,m", [(2, 63), (3, 31)])
def test_closed_form_sine_modes(orc, d, m):
    """f = sum a_m prod sin(k pi x): the discrete solution is
    sum a_m / lam_h(k_m) prod sin(k pi x) exactly."""
    amps, ks = wl.sine_modes(seed=7, d=d, nmodes=4, kmax=min(32, m))
    f = np.zeros((m,) * d)
    uh = np.zeros((m,) * d)
    h = 1.0 / (m + 1)
    for a, k in zip(amps, ks):
        phi = wl.sine_product(d, m, k)
        f += a * phi
        uh += a / lam_h(k, h) * phi
    u, it, relres, st, _ = orc.solve(f, rtol=1e-13, maxit=60)
    assert st == 0 and relres <= 1e-13
    assert rel(u, uh) <= 1e-10


def _l2h_error(d, m, u):
    h = 1.0 / (m + 1)
    e = u - wl.sine_product(d, m)
    return math.sqrt(h ** d * float(np.sum(e * e)))


@pytest.mark.parametrize("d,L", [(3, 5), (3, 6), (3, 7), (3, 8), (2, 9), (2, 10), (2, 11), (2, 12)])
def test_paper_fft_error_column(orc, d, L):
    """The converged discrete solution reproduces the paper's FFT error
    columns (Sec. 5.4, Tables 12 and 14): every printed digit in 3D (within
    one unit of the 4th digit), within 0.5% in 2D (the printed 2D values sit
    0.04-0.36% below the exact discrete error, by the closed form
    |pi^2 h^2 / (4 sin^2(pi h / 2)) - 1| 2^(-d/2))."""
    with open(os.path.join(GOLDEN, "paper_fft_error.json")) as fh:
        gold = json.load(fh)
    printed = gold["%dd" % d][str(L)]
    m = 2 ** L - 1
    f = wl.rhs_sine(d, m)
    # At 4095^2 the FP64 residual itself has a rounding floor near
    # eps * 8|u| / h^2 ~ 5e-10 relative, so 1e-10 is unreachable there; the
    # iterate keeps converging, so run a fixed budget and accept 1e-9.
    u, it, relres, st, _ = orc.solve(f, rtol=1e-10, maxit=30)
    assert relres <= 1e-9
    err = _l2h_error(d, m, u)
    if d == 3:
        ulp = 10.0 ** (math.floor(math.log10(printed)) - 3)
        assert abs(err - printed) <= 1.0 * ulp, (err, printed)
    else:
        assert abs(err - printed) <= 5e-3 * printed, (err, printed)


def test_second_order_discretisation(orc):
    """Error ratio ~4 per halving of h (O(h^2), as the paper observes)."""
    errs = []
    for m in (31, 63, 127):
        u, *_ = orc.solve(wl.rhs_sine(2, m), rtol=1e-12)
        errs.append(_l2h_error(2, m, u))
    for a, b in zip(errs, errs[1:]):
        assert 3.9 < a / b < 4.1


# ----------------------------------------------------------------- V-cycle structure


@pytest.mark.parametrize("d,m,nu", [(2, 31, 2), (3, 15, 2), (2, 15, 1), (3, 7, 3)])
def test_vcycle_symmetric(orc, d, m, nu):
    """With nu1 = nu2, forward pre- and backward post-smoothing and
    FW = 2^-d P^T, the map B: f -> V(0; f) is symmetric."""
    f1 = wl.rhs_uniform(d, m, seed=61)
    f2 = wl.rhs_uniform(d, m, seed=62)
    z = np.zeros_like(f1)
    b1 = orc.vcycle(z, f1, nu, nu)
    b2 = orc.vcycle(z, f2, nu, nu)
    a, b = float(np.sum(b1 * f2)), float(np.sum(f1 * b2))
    assert abs(a - b) <= 1e-13 * max(abs(a), abs(b))


def test_vcycle_symmetry_detects_wrong_post_order(orc):
    """Plant a slip (post-smoothing in forward order, built from the
    oracle's own pieces) and check that the symmetry pin catches it."""
    d, m = 2, 15
    f1 = wl.rhs_uniform(d, m, seed=61)
    f2 = wl.rhs_uniform(d, m, seed=62)

    def two_grid(f, post_backward):
        u = orc.rbgs(np.zeros_like(f), f, 1, backward=False)
        fc = orc.restrict_fw(orc.residual(u, f))
        ec = dst_solve(fc)
        u = orc.prolong_add(ec, u)
        return orc.rbgs(u, f, 1, backward=post_backward)

    def asym(post_backward):
        b1, b2 = two_grid(f1, post_backward), two_grid(f2, post_backward)
        a, b = float(np.sum(b1 * f2)), float(np.sum(f1 * b2))
        return abs(a - b) / abs(a)

    assert asym(True) <= 1e-12
    assert asym(False) > 1e-6


@pytest.mark.parametrize("d,m", [(2, 31), (3, 15)])
def test_vcycle_affine(orc, d, m):
    u = wl.rhs_uniform(d, m, seed=71)
    f1 = wl.rhs_uniform(d, m, seed=72)
    f2 = wl.rhs_uniform(d, m, seed=73)
    z = np.zeros_like(u)
    assert np.all(orc.vcycle(z, z) == 0.0)
    lhs = orc.vcycle(u, f1 + f2) - orc.vcycle(u, f1)
    rhs = orc.vcycle(z, f2)
    assert rel(lhs, rhs) <= 1e-12
    # no state carried between cycles: the same call twice gives the same bits
    assert np.array_equal(orc.vcycle(u, f1), orc.vcycle(u, f1))


def _asymptotic_factor(orc, d, m, nu1, nu2, cycles=20, **kw):
    """Power iteration on the error: f = 0, random start, renormalised."""
    u = wl.rhs_uniform(d, m, seed=81)
    z = np.zeros_like(u)
    ratio = 0.0
    for _ in range(cycles):
        n0 = np.linalg.norm(u)
        u = orc.vcycle(u, z, nu1, nu2, **kw)
        n1 = np.linalg.norm(u)
        ratio = n1 / n0
        u = u / n1
    return ratio


def _two_grid(orc, u, f, nu1, nu2):
    """Two-grid cycle from the oracle's own pieces with an exact (DST) coarse
    solve."""
    u = orc.rbgs(u, f, nu1, backward=False)
    fc = orc.restrict_fw(orc.residual(u, f))
    u = orc.prolong_add(dst_solve(fc), u)
    return orc.rbgs(u, f, nu2, backward=True)


@pytest.mark.parametrize("d,m,nu1,nu2", [(2, 127, 2, 2), (2, 127, 1, 1), (2, 127, 2, 0), (3, 31, 2, 2), (3, 31, 1, 1)])
def test_two_grid_factor_vs_lfa(orc, d, m, nu1, nu2):
    """The oracle's smoother, residual, FW and interpolation, closed by an
    exact coarse solve, converge at the LFA two-grid rate of the same
    smoother order (forward pre, backward post) within 0.01."""
    rho_lfa = lfa.two_grid_factor(d, nu1, nu2, n=48 if d == 2 else 14)
    u = wl.rhs_uniform(d, m, seed=81)
    z = np.zeros_like(u)
    for _ in range(40):
        n0 = np.linalg.norm(u)
        u = _two_grid(orc, u, z, nu1, nu2)
        n1 = np.linalg.norm(u)
        rho = n1 / n0
        u = u / n1
    assert abs(rho - rho_lfa) <= 0.01, (rho, rho_lfa)


@pytest.mark.parametrize("d,ms,nu1,nu2", [(2, (63, 127, 255), 2, 2), (2, (63, 127), 1, 1), (3, (15, 31, 63), 2, 2), (3, (15, 31), 1, 1)])
def test_vcycle_factor_near_two_grid_and_h_independent(orc, d, ms, nu1, nu2):
    """The V-cycle replaces the exact coarse solve by recursion, so its
    asymptotic factor sits near the two-grid factor (-0.03 .. +0.05; small
    grids converge a little faster because of the boundary)
    and does not grow with the grid size."""
    rho_lfa = lfa.two_grid_factor(d, nu1, nu2, n=48 if d == 2 else 14)
    rhos = [_asymptotic_factor(orc, d, m, nu1, nu2) for m in ms]
    for rho in rhos:
        assert rho_lfa - 0.03 <= rho <= rho_lfa + 0.05, (rhos, rho_lfa)
    assert max(rhos) - min(rhos) <= 0.02, rhos


def test_lfa_reproduces_textbook_two_grid_factors():
    """Sanity of the LFA code itself: the classical 2D values for GS-RB with
    FW and bilinear interpolation (nu pre-sweeps): 0.250, 0.074, 0.053."""
    for nu, want in [(1, 0.250), (2, 0.074), (3, 0.053)]:
        assert lfa.two_grid_factor(2, nu, 0, n=48) == pytest.approx(want, abs=1.5e-3)


def test_h_independent_iteration_count(orc):
    """Iterations to a fixed tolerance do not grow with the grid size (the
    paper's observation in Table 5)."""
    its = [orc.solve(wl.rhs_sine(2, m), rtol=1e-10)[1] for m in (63, 127, 255, 511)]
    assert max(its) - min(its) <= 1, its


def test_solve_loop_bookkeeping(orc):
    """Stop at the first residual <= rtol * res0; maxit caps the count and
    reports not-converged; a zero RHS with a zero guess needs no cycle;
    resuming with the original res0 continues the same sequence."""
    f = wl.rhs_sine(2, 63)
    u, it, relres, st, hist = orc.solve(f, rtol=1e-10)
    assert st == 0 and relres <= 1e-10
    assert np.all(hist[:-1] > 1e-10 * hist[0]) and hist[-1] <= 1e-10 * hist[0]
    u3, it3, rel3, st3, _ = orc.solve(f, rtol=1e-10, maxit=3)
    assert it3 == 3 and st3 == 1 and rel3 > 1e-10
    ur, itr, relr, str_, _ = orc.solve(f, u0=u3, rtol=1e-10, res0=hist[0])
    assert itr == it - 3
    assert np.array_equal(ur, u)
    z = np.zeros_like(f)
    _, it0, rel0, st0, _ = orc.solve(z)
    assert it0 == 0 and st0 == 0 and rel0 == 0.0


@pytest.mark.parametrize("d,m,omega", [(2, 127, 0.8), (2, 127, 2 / 3), (3, 31, 6 / 7)])
def test_weighted_jacobi_two_grid_vs_lfa(orc, d, m, omega):
    """Weighted Jacobi V(1,1) pieces with an exact coarse solve converge at
    the LFA two-grid rate within 0.01 (the smoother of Table 5)."""
    rho_lfa = lfa.two_grid_factor(d, 1, 1, n=48 if d == 2 else 14, smoother="wj", omega=omega)
    u = wl.rhs_uniform(d, m, seed=82)
    z = np.zeros_like(u)
    for _ in range(40):
        n0 = np.linalg.norm(u)
        v = orc.wj(u, z, omega, 1)
        fc = orc.restrict_fw(orc.residual(v, z))
        v = orc.prolong_add(dst_solve(fc), v)
        u = orc.wj(v, z, omega, 1)
        n1 = np.linalg.norm(u)
        rho = n1 / n0
        u = u / n1
    assert abs(rho - rho_lfa) <= 0.01, (rho, rho_lfa)


def test_fmg_reaches_discretisation_accuracy(orc):
    """Full multigrid (Algorithm 2) lands within a small factor of the
    discrete solution's error, as the FMG columns of Tables 12 and 14 do
    (there FMG(3,3) stays within 1.9-2.6x of the FFT error in 3D and FMG(1,2)
    within 0.8x in 2D; this library's transfers differ from the paper's, so
    the bounds are loose): 2D FMG(2,2) within 1.5x, 3D FMG(3,3) within 3x,
    and more sweeps never hurt much."""
    for d, m, nu, bound in [(2, 255, 2, 1.5), (2, 511, 2, 1.5), (3, 31, 3, 3.0), (3, 63, 3, 3.0)]:
        u = orc.fmg(wl.rhs_sine(d, m), nu, nu)
        uex, *_ = orc.solve(wl.rhs_sine(d, m), rtol=1e-11)
        e_fmg, e_disc = _l2h_error(d, m, u), _l2h_error(d, m, uex)
        assert e_fmg <= bound * e_disc, (e_fmg, e_disc)
        e1 = _l2h_error(d, m, orc.fmg(wl.rhs_sine(d, m), 1, 1))
        assert e1 > e_fmg
