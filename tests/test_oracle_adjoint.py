"""Pins of the oracle's adjoint (dJ/drho by reverse passes) against finite
differences of the oracle's forward run.

Loss of the gradient workload: J = sum over cells and wavelengths of
(ln U - ln U*)^2, U* the energy density of a perturbed density field.
"""

import numpy as np
import pytest

from paper_1709_03802_amd import workloads as W


def loss_and_ubar(U, Ustar):
    d = np.log(U) - np.log(Ustar)
    return float(np.sum(d * d)), 2.0 * d / U


def forward(orc, grid, pol):
    m = orc.Model(grid)
    return m, orc.run(m, pol)


def J_of(orc, grid, pol, rho, Ustar):
    g = grid.copy()
    g.rho = rho
    _, r = forward(orc, g, pol)
    return loss_and_ubar(r.U, Ustar)[0]


def setup(n, nside, lambdas, n_scatter, seed):
    wl = W.plain16(n=n, nside=nside, lambdas=np.asarray(lambdas), n_scatter=n_scatter)
    grid = wl.grid.copy()
    rng = np.random.default_rng(seed)
    grid.rho = grid.rho * np.exp(0.3 * rng.standard_normal(grid.n))
    return grid, wl.policy


@pytest.mark.parametrize("n,nside,n_scatter", [(3, 2, 1), (4, 1, 2)])
def test_adjoint_matches_central_differences_on_every_cell(orc, n, nside, n_scatter):
    grid, pol = setup(n, nside, [0.3, 1.0], n_scatter, seed=1)
    target = grid.copy()
    target.rho = W.perturbed_rho(grid.rho, 0.3, seed=3802)
    _, rt = forward(orc, target, pol)
    m, r = forward(orc, grid, pol)
    J, Ubar = loss_and_ubar(r.U, rt.U)
    g = orc.adjoint(m, pol, r, Ubar)
    fd = np.zeros(grid.n)
    for c in range(grid.n):
        h = 1e-5 * grid.rho[c]
        rp = grid.rho.copy()
        rp[c] += h
        rm = grid.rho.copy()
        rm[c] -= h
        fd[c] = (J_of(orc, grid, pol, rp, rt.U) - J_of(orc, grid, pol, rm, rt.U)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=2e-5, atol=2e-6 * np.abs(fd).max())


def test_adjoint_dot_product(orc):
    grid, pol = setup(6, 4, [0.2, 0.55, 2.0], 2, seed=2)
    target = grid.copy()
    target.rho = W.perturbed_rho(grid.rho, 0.3, seed=3802)
    _, rt = forward(orc, target, pol)
    m, r = forward(orc, grid, pol)
    J, Ubar = loss_and_ubar(r.U, rt.U)
    g = orc.adjoint(m, pol, r, Ubar)
    rng = np.random.default_rng(9)
    for _ in range(2):
        drho = rng.standard_normal(grid.n) * grid.rho
        eps = 1e-6
        jp = J_of(orc, grid, pol, grid.rho + eps * drho, rt.U)
        jm = J_of(orc, grid, pol, grid.rho - eps * drho, rt.U)
        dd = (jp - jm) / (2 * eps)
        assert float(g @ drho) == pytest.approx(dd, rel=1e-6)


def test_adjoint_zero_at_target(orc):
    grid, pol = setup(3, 2, [0.55], 1, seed=4)
    m, r = forward(orc, grid, pol)
    J, Ubar = loss_and_ubar(r.U, r.U)
    assert J == 0.0
    assert np.all(orc.adjoint(m, pol, r, Ubar) == 0.0)


def escape_loss(run, Fstar):
    d = np.log(run.escape) - np.log(Fstar)
    return float(np.sum(d * d)), 2.0 * d / run.escape


@pytest.mark.parametrize("n,nside,n_scatter", [(3, 2, 1), (4, 1, 2)])
def test_escape_loss_adjoint_matches_central_differences(orc, n, nside, n_scatter):
    """A loss on the escaping luminosity by direction, alone and together with
    the energy-density loss, against central differences on every cell."""
    grid, pol = setup(n, nside, [0.3, 1.0], n_scatter, seed=3)
    target = grid.copy()
    target.rho = W.perturbed_rho(grid.rho, 0.3, seed=3802)
    _, rt = forward(orc, target, pol)
    m, r = forward(orc, grid, pol)
    _, Ebar = escape_loss(r, rt.escape)
    _, Ubar = loss_and_ubar(r.U, rt.U)
    g_e = orc.adjoint(m, pol, r, None, Ebar=Ebar)
    g_both = orc.adjoint(m, pol, r, Ubar, Ebar=Ebar)
    g_u = orc.adjoint(m, pol, r, Ubar)
    np.testing.assert_allclose(g_both, g_e + g_u, rtol=1e-12, atol=1e-15 * np.abs(g_both).max())

    def J(rho):
        g = grid.copy()
        g.rho = rho
        _, rr = forward(orc, g, pol)
        return escape_loss(rr, rt.escape)[0]

    fd = np.zeros(grid.n)
    for c in range(grid.n):
        h = 1e-5 * grid.rho[c]
        rp = grid.rho.copy()
        rp[c] += h
        rm = grid.rho.copy()
        rm[c] -= h
        fd[c] = (J(rp) - J(rm)) / (2 * h)
    np.testing.assert_allclose(g_e, fd, rtol=2e-5, atol=2e-6 * np.abs(fd).max())


def test_scattered_light_loss_adjoint_matches_central_differences(orc):
    """A loss on S_total = S_1 + ... + S_{K+1} (hence on j_sca): every order
    receives dJ/dS_total; the adjoint matches central differences on every
    cell of a small grid."""
    grid, pol = setup(3, 2, [0.3, 1.0], 2, seed=4)
    m, r = forward(orc, grid, pol)
    rng = np.random.default_rng(8)
    w = rng.random(m.s_size)

    def J(rho):
        g = grid.copy()
        g.rho = rho
        return float(w @ forward(orc, g, pol)[1].S_total)

    gad = orc.adjoint(m, pol, r, Ubar=np.zeros((m.nl, m.n)), Sbar_total=w)
    fd = np.zeros(grid.n)
    for c in range(grid.n):
        h = 1e-5 * grid.rho[c]
        rp = grid.rho.copy()
        rp[c] += h
        rm = grid.rho.copy()
        rm[c] -= h
        fd[c] = (J(rp) - J(rm)) / (2 * h)
    np.testing.assert_allclose(gad, fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())
