"""The fluid step (paper sections 2.2-2.4): drift-diffusion-reaction update of the
electron and ion densities with Koren-limited advective fluxes, central
diffusive fluxes, the ionisation source, refinement-boundary ghosts and flux
fix-up, the explicit trapezoidal time step and its time-step limits.

CPU tests pin the oracle to what the paper and the mathematics fix:
* the Koren limiter's values at points where each branch is active;
* the lookup table: exact at the entries, linear between them, the last
  entry beyond emax;
* a uniform density in a uniform field stays uniform on a refined tree
  (every ghost rule and the flux fix-up reproduce a constant);
* mass conservation across a refinement boundary without sources (the
  coarse flux is the mean of the fine fluxes);
* a whole time step on a uniform neutral plasma in a uniform field equals
  Heun's method for n' = k n in closed form, and the time-step limit equals
  its closed form;
* along x, a stage on a uniform tree equals a one-dimensional evaluation of
  the paper's flux formulas written out below with numpy, for both signs of
  the velocity.
GPU tests compare the HIP path with the oracle stage by stage and step by
step, on the small streamer tree and on the full benchmark tree."""
import numpy as np
import pytest

import oracle as O
from workloads import (constant_table, synthetic_n2_table, EMAX, uniform_boxes,
                       refine_boxes_explicit, streamer_small)
from tests import _geom as G

E_CHARGE = 1.602176634e-19
EPS0 = 8.8541878128e-12


def psi(x):
    return O.lib().oracle_koren_psi(float(x))


def test_koren_limiter_values():
    # psi = 0 for x <= 0, x up to 0.4, (2 + x) / 6 up to 4, then 1
    for x, want in [(-3.0, 0.0), (0.0, 0.0), (0.1, 0.1), (0.4, 0.4), (1.0, 0.5),
                    (2.0, 4.0 / 6.0), (4.0, 1.0), (50.0, 1.0)]:
        assert abs(psi(x) - want) < 1e-15, (x, psi(x), want)


def coeffs(tab, emax, E):
    out = np.zeros(3)
    T = np.ascontiguousarray(tab, dtype=np.float64)
    O.lib().oracle_fluid_coeffs(O._ptr(T), len(T), float(emax), float(E), O._ptr(out))
    return out


def test_lookup_table_interpolation():
    tab = synthetic_n2_table(11, 10.0)               # entries at E = 0, 1, ..., 10
    for k in range(11):
        np.testing.assert_allclose(coeffs(tab, 10.0, k), tab[k], rtol=1e-15)
    np.testing.assert_allclose(coeffs(tab, 10.0, 2.25), 0.75 * tab[2] + 0.25 * tab[3], rtol=1e-14)
    np.testing.assert_allclose(coeffs(tab, 10.0, 13.0), tab[10], rtol=0)


def linear_phi_tree(bl, axis, volts, length, nmax=None):
    """Oracle tree with phi exactly linear along `axis` (Dirichlet 0 and
    `volts` on that axis' faces, Neumann elsewhere) and no charge."""
    bct = [1] * 6
    bcv = [0.0] * 6
    bct[2 * axis] = bct[2 * axis + 1] = 0
    bcv[2 * axis + 1] = volts
    o = O.OracleTree(bl.level, bl.ijk, bl.tree, length=length, bc_type=bct, bc_val=bcv)
    lv, ij = o.index(O.IDX_LEVEL), o.index(O.IDX_IJK)
    x = G.cell_centres(lv, ij, length)[axis]
    o.set_field(O.PHI, volts * x / length)
    o.set_field(O.RHS, np.zeros_like(x))
    return o


def test_uniform_density_stays_uniform_on_a_refined_tree():
    bl = refine_boxes_explicit(2, [(2, 0, 0, 0), (3, 1, 1, 1), (3, 0, 1, 0)])
    o = linear_phi_tree(bl, 2, 8e3, 0.01)
    ef, en = o.efield()
    n = np.full((o.n, 8, 8, 8), 3e18)
    tab = constant_table(0.04, 0.12, 0.0)
    oe, oi, lim = o.fluid_stage(n, n, n, n, ef, en, tab, EMAX, 1e-12)
    leaf = o.leaf_mask()
    np.testing.assert_allclose(oe[leaf], 3e18, rtol=1e-13)
    np.testing.assert_allclose(oi[leaf], 3e18, rtol=0)


def blob_setup():
    """A refined tree, a charged blob (so the field is not uniform) and an
    electron blob that straddles the refinement boundary at x = 0.5 and
    vanishes well inside the domain."""
    bl = refine_boxes_explicit(2, [(2, 1, 0, 0), (2, 1, 1, 0), (2, 1, 0, 1), (2, 1, 1, 1),
                                   (3, 2, 1, 1), (3, 2, 2, 1)])
    L = 0.01
    o = O.OracleTree(bl.level, bl.ijk, bl.tree, length=L, bc_type=[1, 1, 1, 1, 0, 0],
                     bc_val=[0, 0, 0, 0, 0, 2e4])
    lv, ij = o.index(O.IDX_LEVEL), o.index(O.IDX_IJK)
    x, y, z, _ = G.cell_centres(lv, ij, L)
    r2 = ((x - 0.5 * L) ** 2 + (y - 0.4 * L) ** 2 + (z - 0.45 * L) ** 2) / (0.08 * L) ** 2
    ne = 1e19 * np.exp(-r2) + 1e-300
    ni = 0.5 * ne
    o.set_field(O.RHS, -E_CHARGE * (ni - ne) / EPS0)
    o.fmg_solve(tol=1e-10)
    return o, lv, ne, ni


def test_mass_is_conserved_across_a_refinement_boundary():
    o, lv, ne, ni = blob_setup()
    ef, en = o.efield()
    tab = synthetic_n2_table()
    tab[:, 2] = 0.0                                  # no ionisation
    oe, oi, lim = o.fluid_stage(ne, ni, ne, ni, ef, en, tab, EMAX, 2e-11)
    leaf = o.leaf_mask()
    vol = (0.01 / (8.0 * 2.0 ** (lv - 1))) ** 3
    m0 = np.sum(ne[leaf].sum(axis=(1, 2, 3)) * vol[leaf])
    m1 = np.sum(oe[leaf].sum(axis=(1, 2, 3)) * vol[leaf])
    moved = np.sum(np.abs(oe - ne)[leaf].sum(axis=(1, 2, 3)) * vol[leaf])
    assert moved > 1e-3 * m0                         # the stage moved charge
    assert abs(m1 - m0) <= 1e-13 * m0, (m1 - m0) / m0


def test_time_step_equals_heun_in_a_uniform_field():
    """Uniform neutral plasma, uniform field E0 along z: fluxes are
    divergence-free and the charge stays zero, so n_e' = k n_e, n_i' = k n_e
    with k = alpha mu E0, and the trapezoidal step is Heun's method."""
    L, V = 0.004, 8e3                                # E0 = 2 MV/m
    o = linear_phi_tree(uniform_boxes(3), 2, V, L)
    mu, D, al = 0.04, 0.12, 2e4
    tab = constant_table(mu, D, al)
    n0 = 1e17
    ne = np.full((o.n, 8, 8, 8), n0)
    dt = 3e-11
    oe, oi, dt_next = o.fluid_step(ne, ne.copy(), dt, tab, EMAX)
    E0 = V / L
    hk = dt * al * mu * E0
    leaf = o.leaf_mask()
    np.testing.assert_allclose(oe[leaf], n0 * (1 + hk + hk * hk / 2), rtol=1e-12)
    np.testing.assert_allclose(oi[leaf], n0 + n0 * (hk + hk * hk / 2), rtol=1e-12)
    h = L / 32
    n1 = n0 * (1 + hk)                               # the limit is taken in the second stage
    want = min(0.5 * h / (mu * E0), 1.0 / (mu * E0 / h + 6 * D / h ** 2), EPS0 / (E_CHARGE * mu * n1))
    assert abs(dt_next - 0.9 * want) <= 1e-12 * want


def psi_np(x):
    return max(0.0, min(1.0, (2.0 + x) / 6.0, x))


def koren_1d(n, v, D, h, dt):
    """One forward Euler step of the paper's 1-D scheme on cells 0..N-1 with
    mirrored ghosts; v[f], f = 0..N the face velocities."""
    N = len(n)
    g = np.concatenate([[n[1], n[0]], n, [n[-1], n[-2]]])   # g[c + 2] = n[c]
    F = np.zeros(N + 1)
    for f in range(N + 1):
        nm1, ni, ni1, ni2 = g[f], g[f + 1], g[f + 2], g[f + 3]   # cells f-2 .. f+1
        b = ni1 - ni
        if v[f] < 0:
            lim = 0.0 if b == 0 else psi_np((ni2 - ni1) / b) * b
            nf = ni1 - lim
        else:
            lim = 0.0 if b == 0 else psi_np((ni - nm1) / b) * b
            nf = ni + lim
        F[f] = v[f] * nf - D * b / h
    return n - dt * (F[1:] - F[:-1]) / h


@pytest.mark.parametrize("volts", [5e3, -5e3])
def test_stage_along_x_equals_the_one_dimensional_scheme(volts):
    L = 0.004
    o = linear_phi_tree(uniform_boxes(3), 0, volts, L)
    lv, ij = o.index(O.IDX_LEVEL), o.index(O.IDX_IJK)
    x = G.cell_centres(lv, ij, L)[0]
    rng = np.random.default_rng(7)
    prof = 1e18 * (1.0 + rng.random(32)) * (np.arange(32) > 9) + 1e16 * np.arange(32)
    cell = np.floor(x / (L / 32)).astype(int)
    ne = prof[np.clip(cell, 0, 31)]
    ef, en = o.efield()
    mu, D = 0.04, 0.12
    dt = 2e-12
    oe, _, _ = o.fluid_stage(ne, ne, ne, ne, ef, en, constant_table(mu, D, 0.0), EMAX, dt)
    h = L / 32
    v = np.full(33, -mu * (-volts / L))              # E_x = -dphi/dx
    want = koren_1d(prof, v, D, h, dt)
    leaf = o.leaf_mask()
    got = oe[leaf]
    gx = cell[leaf]
    for c in range(32):
        vals = got[gx == c]
        np.testing.assert_allclose(vals, want[c], rtol=1e-12, err_msg=f"cell {c}")


# --------------------------------------------------------------------- GPU

def small_si_tree():
    """The small streamer tree (649 boxes, refined around the channel) in a
    (1 cm)^3 domain: 20 kV on top, grounded bottom, Neumann sides."""
    w = streamer_small()
    b = w.boxes
    return b, 0.01, (1, 1, 1, 1, 0, 0), (0.0, 0.0, 0.0, 0.0, 0.0, 2e4)


def densities(lv, ij, L, seed, head=(0.5, 0.5, 0.62), width=0.05):
    """Background 1e15 m^-3 plus a seeded, perturbed 1e19 m^-3 blob at the
    streamer head (it crosses the refinement boundaries); ions 0.8 of it."""
    x, y, z, _ = G.cell_centres(lv, ij, L)
    rng = np.random.default_rng(seed)
    r2 = ((x - head[0] * L) ** 2 + (y - head[1] * L) ** 2 + (z - head[2] * L) ** 2) / (width * L) ** 2
    blob = 1e19 * np.exp(-r2)
    ne = 1e15 + blob * (1.0 + 0.3 * rng.random(x.shape))
    ni = 1e15 + 0.8 * blob
    return ne, ni


def pair(bl, L, bct, bcv):
    from paper_1708_08434_amd import mg as M
    g = M.Tree(bl.level, bl.ijk, bl.tree, (0.0, 0.0, 0.0), L, bct, bcv)
    o = O.OracleTree(bl.level, bl.ijk, bl.tree, length=L, bc_type=bct, bc_val=bcv)
    assert np.array_equal(g.index(M.MG_IDX_ORDER), o.index(O.IDX_ORDER))
    return g, o


def dev(g, a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(g.device)


def leaf_close(got, want, leaf, rtol, what):
    err = np.abs(got - want)[leaf].max() / np.abs(want[leaf]).max()
    print(f"{what}: max difference {err:.2e} of the largest value", flush=True)
    assert err <= rtol, (what, err)


@pytest.mark.gpu
def test_gpu_stage_matches_the_oracle():
    """Same densities and the same field (the oracle's) on both sides: the
    outputs of a stage, the solver's right-hand side and the time-step bound."""
    import torch
    from paper_1708_08434_amd import mg as M
    bl, L, bct, bcv = small_si_tree()
    g, o = pair(bl, L, bct, bcv)
    lv, ij = o.index(O.IDX_LEVEL), o.index(O.IDX_IJK)
    ne, ni = densities(lv, ij, L, 11)
    o.set_field(O.RHS, -E_CHARGE * (ni - ne) / EPS0)
    o.fmg_solve(tol=1e-10)
    ef, en = o.efield()
    tab = synthetic_n2_table()
    g.fluid_bind(tab, EMAX)
    Ef, En, Ne, Ni, N0e, N0i = (dev(g, a) for a in (ef, en, ne, ni, 0.9 * ne, 1.1 * ni))
    Oe, Oi = torch.zeros_like(Ne), torch.zeros_like(Ni)
    dt = 5e-12
    lim_g = M.mg_fluid_stage(g.h, Ef.data_ptr(), En.data_ptr(), Ne.data_ptr(), Ni.data_ptr(),
                             N0e.data_ptr(), N0i.data_ptr(), dt, 0.5, 0.5, Oe.data_ptr(), Oi.data_ptr())
    oe, oi, lim_o = o.fluid_stage(ne, ni, 0.9 * ne, 1.1 * ni, ef, en, tab, EMAX, dt, 0.5, 0.5)
    leaf = o.leaf_mask()
    torch.cuda.synchronize()
    leaf_close(Oe.cpu().numpy(), oe, leaf, 1e-12, "n_e")
    leaf_close(Oi.cpu().numpy(), oi, leaf, 1e-12, "n_i")
    leaf_close(g.get_field(M.MG_FIELD_RHS), o.get_field(O.RHS), leaf, 1e-12, "right-hand side")
    assert abs(lim_g - lim_o) <= 1e-12 * lim_o, (lim_g, lim_o)
    assert np.abs(Oe.cpu().numpy() - ne)[leaf].max() > 1e-3 * ne.max()   # the stage did something


@pytest.mark.gpu
def test_gpu_stage_conserves_mass_at_refinement_boundaries():
    import torch
    from paper_1708_08434_amd import mg as M
    bl, L, bct, bcv = small_si_tree()
    g, o = pair(bl, L, bct, bcv)
    lv, ij = o.index(O.IDX_LEVEL), o.index(O.IDX_IJK)
    # a blob around the streamer head, which crosses refinement boundaries;
    # at the domain faces (>= 6.7 widths away) it is ~1e-19 of its peak, so
    # no mass flows out there
    ne, ni = densities(lv, ij, L, 12, head=(0.5, 0.5, 0.6), width=0.06)
    ne -= 1e15
    g.set_field(M.MG_FIELD_RHS, -E_CHARGE * (ni - ne) / EPS0)
    g.fmg_solve()
    tab = synthetic_n2_table()
    tab[:, 2] = 0.0                                  # no ionisation
    g.fluid_bind(tab, EMAX)
    face, norm = g.efield(to_numpy=False)
    Ne, Ni = dev(g, ne), dev(g, ni)
    Oe, Oi = torch.zeros_like(Ne), torch.zeros_like(Ni)
    M.mg_fluid_stage(g.h, face.data_ptr(), norm.data_ptr(), Ne.data_ptr(), Ni.data_ptr(), Ne.data_ptr(),
                     Ni.data_ptr(), 2e-11, 0.0, 1.0, Oe.data_ptr(), Oi.data_ptr())
    leaf = o.leaf_mask()
    vol = (L / (8.0 * 2.0 ** (lv - 1))) ** 3
    out = Oe.cpu().numpy()
    m0 = np.sum(ne[leaf].sum(axis=(1, 2, 3)) * vol[leaf])
    m1 = np.sum(out[leaf].sum(axis=(1, 2, 3)) * vol[leaf])
    assert np.abs(out - ne)[leaf].max() > 1e-3 * ne.max()
    assert abs(m1 - m0) <= 1e-13 * m0, (m1 - m0) / m0


def step_parity(bl, L, bct, bcv, ne, ni, dt, rtol):
    from paper_1708_08434_amd import mg as M
    g, o = pair(bl, L, bct, bcv)
    b = -E_CHARGE * (ni - ne) / EPS0
    g.set_field(M.MG_FIELD_RHS, b)
    o.set_field(O.RHS, b)
    g.fmg_solve(rel_tol=1e-10)
    o.fmg_solve(tol=1e-10)
    tab = synthetic_n2_table()
    g.fluid_bind(tab, EMAX)
    Ne, Ni = dev(g, ne), dev(g, ni)
    nxt_g = M.mg_fluid_step(g.h, Ne.data_ptr(), Ni.data_ptr(), dt, 2)
    oe, oi, nxt_o = o.fluid_step(ne, ni, dt, tab, EMAX, 2)
    leaf = o.leaf_mask()
    leaf_close(Ne.cpu().numpy(), oe, leaf, rtol, "n_e after the step")
    leaf_close(Ni.cpu().numpy(), oi, leaf, rtol, "n_i after the step")
    leaf_close(g.get_field(M.MG_FIELD_PHI), o.get_field(O.PHI), leaf, rtol, "phi after the step")
    assert abs(nxt_g - nxt_o) <= rtol * nxt_o, (nxt_g, nxt_o)
    return nxt_g


@pytest.mark.gpu
def test_gpu_time_step_matches_the_oracle():
    bl, L, bct, bcv = small_si_tree()
    o = O.OracleTree(bl.level, bl.ijk, bl.tree, length=L)
    ne, ni = densities(o.index(O.IDX_LEVEL), o.index(O.IDX_IJK), L, 13)
    step_parity(bl, L, bct, bcv, ne, ni, 5e-12, 1e-10)


@pytest.mark.gpu
def test_gpu_time_step_full_size_matches_the_oracle():
    """The paper's setup ((40 mm)^3, 80 kV, the benchmark tree) with a
    perturbed electron blob at the streamer head, one whole step."""
    from workloads import paper_setup
    w = paper_setup()
    bl = w.boxes
    o = O.OracleTree(bl.level, bl.ijk, bl.tree, length=w.length)
    ne, ni = densities(o.index(O.IDX_LEVEL), o.index(O.IDX_IJK), w.length, 14, width=0.03)
    nxt = step_parity(bl, w.length, w.bc_type, w.bc_val, ne, ni, 2e-12, 1e-9)
    print("next dt", nxt, flush=True)


@pytest.mark.gpu
def test_gpu_step_reports_a_non_finite_density():
    """A NaN density (a diverged step) is not silently carried on: the stage's
    time-step bound is NaN and the step returns MG_ENOCONV."""
    import torch
    from paper_1708_08434_amd import mg as M
    bl, L, bct, bcv = small_si_tree()
    g, o = pair(bl, L, bct, bcv)
    lv, ij = o.index(O.IDX_LEVEL), o.index(O.IDX_IJK)
    ne, ni = densities(lv, ij, L, 15)
    g.set_field(M.MG_FIELD_RHS, -E_CHARGE * (ni - ne) / EPS0)
    g.fmg_solve()
    g.fluid_bind(synthetic_n2_table(), EMAX)
    leaf = o.leaf_mask()
    q = int(np.nonzero(leaf)[0][len(np.nonzero(leaf)[0]) // 2])
    bad = ne.copy()
    bad[q, 3, 4, 5] = np.nan
    face, norm = g.efield(to_numpy=False)
    Ne, Ni = dev(g, bad), dev(g, ni)
    Oe, Oi = torch.zeros_like(Ne), torch.zeros_like(Ni)
    lim = M.mg_fluid_stage(g.h, face.data_ptr(), norm.data_ptr(), Ne.data_ptr(), Ni.data_ptr(),
                           Ne.data_ptr(), Ni.data_ptr(), 1e-12, 0.0, 1.0, Oe.data_ptr(), Oi.data_ptr())
    assert np.isnan(lim), lim
    with pytest.raises(M.MGError) as e:
        M.mg_fluid_step(g.h, Ne.data_ptr(), Ni.data_ptr(), 1e-12, 2)
    assert e.value.code == M.MG_ENOCONV
    # finite densities still step normally afterwards
    g.set_field(M.MG_FIELD_RHS, -E_CHARGE * (ni - ne) / EPS0)
    g.fmg_solve()
    Ne, Ni = dev(g, ne), dev(g, ni)  # the failed step left NaN in both (updated in place)
    dt = M.mg_fluid_step(g.h, Ne.data_ptr(), Ni.data_ptr(), 1e-12, 2)
    assert np.isfinite(dt) and dt > 0
