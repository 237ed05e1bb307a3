"""The oracle's pins have teeth: each test plants one plausible mistake in the
oracle (on the CPU, through monkeypatch) and checks that at least one pin
then fails.  Nothing here touches the GPU path."""
import math

import numpy as np
import pytest

from oracle import adjoint, coupling, fem, multigrid as mg
from paper_2101_08453_amd import inputs
from tests import test_oracle_adjoint as t_adj
from tests import test_oracle_coupling as t_cpl
from tests import test_oracle_fem as t_fem
from tests import test_oracle_krylov as t_kry
from tests import test_oracle_line as t_line
from tests import test_oracle_multigrid as t_mg


def _hier_krylov():
    p = inputs.hills_problem(12, 10, 6, 2, 71, a=(1.0, 1.0, 4.0), noise=0.2)
    return p, mg.build_hierarchy(p.X, p.Y, p.Z, p.a, p.gamma, coarse_max=40)


def _hier_line():
    p = inputs.hills_problem(10, 9, 6, 2, 81, a=(1.0, 1.0, 0.5), noise=0.2)
    return p, mg.build_hierarchy(p.X, p.Y, p.Z, p.a, p.gamma, coarse_max=60)


def _some_pin_fails(checks):
    """Run the pins; True as soon as one of them fails an assertion (or the
    mistake makes a system singular).  Any other error propagates."""
    for fn, args in checks:
        try:
            fn(*args)
        except (AssertionError, np.linalg.LinAlgError):
            return True
    return False


# ---------------------------------------------------------------- mutations

def _gauss_at_half(mp):
    mp.setattr(fem, "GAUSS_POINTS", fem.GAUSS_POINTS * (0.5 / fem.G))


def _stiffness_without_detj(mp):
    def bad(xe, c):
        Ke = np.zeros((xe.shape[0], 8, 8))
        for xi in fem.GAUSS_POINTS:
            B, _ = fem.physical_gradients(xe, xi)
            Ke += np.einsum("eda,d,edb->eab", B, c, B)
        return Ke
    mp.setattr(fem, "element_stiffness", bad)


def _a_instead_of_inverse(mp):
    mp.setattr(fem, "penalty_coefficients", lambda a: np.asarray(a, dtype=np.float64) ** 2)


def _transposed_jacobian(mp):
    mp.setattr(fem, "jacobian", lambda xe, xi: np.einsum("ead,am->emd", xe, fem.shape_grad_ref(xi)))


def _rhs_weight_one(mp):
    def bad(xe, u0e):
        B, det = fem.physical_gradients(xe, fem.CENTRE)
        return -1.0 * det[:, None] * np.einsum("eda,ed->ea", B, u0e)
    mp.setattr(fem, "element_rhs", bad)


def _rhs_wrong_sign(mp):
    good = fem.element_rhs
    mp.setattr(fem, "element_rhs", lambda xe, u0e: -good(xe, u0e))


def _recover_wrong_sign(mp):
    mp.setattr(fem, "recover", lambda X, Y, Z, u0, a, lam:
               u0 - fem.penalty_coefficients(a)[:, None, None, None] * fem.centre_gradient(X, Y, Z, lam))


def _top_face_free(mp):
    good = fem.free_mask
    mp.setattr(fem, "free_mask", lambda nx, ny, nz, gamma: good(nx, ny, nz, gamma | 2))


def _interp_weight_third(mp):
    good = mg.interpolation_1d

    def bad(n, keep):
        P = good(n, keep).tolil()
        P[P == 0.5] = 1.0 / 3.0
        return P.tocsr()
    mp.setattr(mg, "interpolation_1d", bad)


def _gs_upper_triangle(mp):
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    def bad(K_full, mask, dims, x, f, order=None, reverse=False):
        nx, ny, nz = dims
        order = mg.colour_order(nx, ny, nz, mask) if order is None else order
        x = np.array(x, dtype=np.float64)
        Kp = K_full[order][:, order].tocsr()
        r = f[order] - (K_full @ x)[order]
        x[order] += spla.spsolve_triangular(sp.triu(Kp).tocsr(), r, lower=False)
        return x
    mp.setattr(mg, "gs_sweep_full", bad)


def _centre_height_from_top(mp):
    def bad(X, Y, Z, k, j, i):
        sl = (slice(k, k + 2), slice(j, j + 2), slice(i, i + 2))
        c = np.array([X[sl].mean(), Y[sl].mean(), Z[k + 1, j:j + 2, i:i + 2].mean()])
        return c, Z[0, j:j + 2, i:i + 2].mean()
    mp.setattr(coupling, "element_centre", bad)
    good = coupling.element_centres

    def bad_all(X, Y, Z):
        c = good(X, Y, Z)
        c[2] = 0.25 * (Z[1:, :-1, :-1] + Z[1:, :-1, 1:] + Z[1:, 1:, :-1] + Z[1:, 1:, 1:])
        return c
    mp.setattr(coupling, "element_centres", bad_all)


def _colours_transposed(mp):
    mp.setattr(mg, "COLOURS", ((0, 0), (0, 1), (1, 0), (1, 1)))


def _ratio_inverted(mp):
    good = mg.coupling_ratio
    mp.setattr(mg, "coupling_ratio", lambda h3, hh, a, rule: 1.0 / good(h3, hh, a, rule))


def _log_law_without_z0(mp):
    good = coupling.column_profile

    def bad(h, v, zeta, z0):
        h = np.asarray(h, dtype=np.float64)
        if z0 < zeta < h[0]:
            return np.asarray(v, dtype=np.float64)[..., 0] * (math.log(zeta) / math.log(h[0]))
        return good(h, v, zeta, z0)
    mp.setattr(coupling, "column_profile", bad)


def _bilinear_weight_flipped(mp):
    good = coupling.bilinear_cell

    def bad(pos, origin, spacing, n):
        i, w = good(pos, origin, spacing, n)
        return i, 1.0 - w
    mp.setattr(coupling, "bilinear_cell", bad)


def _loss_gradient_halved(mp):
    good = adjoint.surface_loss

    def bad(u, mask):
        L, g = good(u, mask)
        return L, 0.5 * g
    mp.setattr(adjoint, "surface_loss", bad)


def _reverse_sweep_not_reversed(mp):
    good = mg.line_sweep_full
    mp.setattr(mg, "line_sweep_full", lambda K, mask, dims, x, f, reverse=False: good(K, mask, dims, x, f))


def _cg_beta_inverted(mp):
    def bad(self, f, steps=None, rtol=1e-12, maxiter=500):
        K = self.levels[0].K
        x = np.zeros_like(f)
        r = f.copy()
        z = self.precondition(r)
        p = z.copy()
        rz = r @ z
        hist = []
        for _ in range(steps if steps is not None else maxiter):
            q = K @ p
            alpha = rz / (p @ q)
            x = x + alpha * p
            r = r - alpha * q
            hist.append(np.linalg.norm(r) / np.linalg.norm(f))
            if steps is None and hist[-1] <= rtol:
                break
            z = self.precondition(r)
            rz_new = r @ z
            p = z + (rz / rz_new) * p
            rz = rz_new
        return x, hist
    mp.setattr(mg.Multigrid, "pcg", bad)


def _geometry_at_centre_only(mp):
    def bad(X, Y, Z):
        nx, ny, nz = fem.dims_of(X)
        xe = fem.element_coords(X, Y, Z, fem.element_node_ids(nx, ny, nz))
        return np.linalg.det(fem.jacobian(xe, fem.CENTRE))
    mp.setattr(fem, "min_detJ", bad)


def _geometry_without_last_gauss_point(mp):
    def bad(X, Y, Z):
        nx, ny, nz = fem.dims_of(X)
        xe = fem.element_coords(X, Y, Z, fem.element_node_ids(nx, ny, nz))
        pts = list(fem.GAUSS_POINTS[:-1]) + [fem.CENTRE]
        return np.min(np.stack([np.linalg.det(fem.jacobian(xe, xi)) for xi in pts], 1), 1)
    mp.setattr(fem, "min_detJ", bad)


def _pushed_corners():
    return [(t_fem.test_min_detJ_of_a_box_with_one_corner_pushed_in, (c, t))
            for c in range(8) for t in (0.3, 0.8)]


MUTATIONS = {
    "geometry checked at the centre only": (_geometry_at_centre_only, _pushed_corners),
    "geometry check skips a Gauss point": (_geometry_without_last_gauss_point, _pushed_corners),
    "Gauss points at +-1/2": (_gauss_at_half, lambda: [
        (t_fem.test_box_element_is_tensor_product, ((30.0, 25.0, 5.0), (1.0, 1.0, 1.0))),
        (t_fem.test_cube_interior_stencil, ())]),
    "stiffness without det J": (_stiffness_without_detj, lambda: [
        (t_fem.test_box_element_is_tensor_product, ((30.0, 25.0, 5.0), (1.0, 1.0, 1.0))),
        (t_fem.test_coordinate_scaling, ())]),
    "A instead of A^-1": (_a_instead_of_inverse, lambda: [
        (t_fem.test_box_element_is_tensor_product, ((30.0, 30.0, 7.2), (1.0, 2.0, 10.0))),
        (t_fem.test_penalty_scaling_and_z_translation, ())]),
    "transposed Jacobian": (_transposed_jacobian, lambda: [
        (t_fem.test_linear_lambda_gradient_exact_on_distorted_mesh, ()),
        (t_fem.test_matrix_free_apply_equals_assembled, ())]),
    "right-hand side weight 1 for 8": (_rhs_weight_one, lambda: [
        (t_fem.test_box_rhs_closed_form, ()),
        (t_fem.test_weak_divergence_identity_and_zero_at_solution, ())]),
    "right-hand side sign": (_rhs_wrong_sign, lambda: [
        (t_fem.test_box_rhs_closed_form, ()),
        (t_fem.test_mass_conservation_through_a_box_grid_column, ())]),
    "recovery sign": (_recover_wrong_sign, lambda: [
        (t_fem.test_recovery_of_a_linear_multiplier, ())]),
    "top face free": (_top_face_free, lambda: [(t_fem.test_free_mask_counts, ())]),
    "interpolation weight 1/3": (_interp_weight_third, lambda: [
        (t_mg.test_interpolation_reproduces_linear_functions_and_odd_counts, ())]),
    "colours (0,0),(0,1),(1,0),(1,1)": (_colours_transposed, lambda: [
        (t_mg.test_gauss_seidel_sweep_equals_pointwise_loop, ())]),
    "Gauss-Seidel with the upper triangle": (_gs_upper_triangle, lambda: [
        (t_mg.test_gauss_seidel_sweep_equals_pointwise_loop, ())]),
    "centre height from the top nodes": (_centre_height_from_top, lambda: [
        (t_cpl.test_centres_and_heights_on_a_flat_box, ())]),
    "coupling ratio inverted": (_ratio_inverted, lambda: [
        (t_mg.test_decision_stretched_grid_unit_penalties, ()),
        (t_mg.test_decision_vertical_anisotropy_operator_rule, ())]),
    "log law without z0": (_log_law_without_z0, lambda: [
        (t_cpl.test_log_law_below_the_lowest_level_and_constant_above_the_top, ())]),
    "bilinear weight flipped": (_bilinear_weight_flipped, lambda: [
        (t_cpl.test_interpolation_is_exact_for_fields_linear_in_position_and_height, ())]),
    "loss gradient halved": (_loss_gradient_halved, lambda: [
        (t_adj.test_u0_gradient_matches_central_differences, ())]),
    "reverse line sweep not reversed": (_reverse_sweep_not_reversed, lambda: [
        (t_line.test_reverse_line_sweep_is_the_energy_adjoint, (_hier_line(),))]),
    "CG beta inverted": (_cg_beta_inverted, lambda: [
        (t_kry.test_cg_energy_error_never_exceeds_the_stationary_iteration, (_hier_krylov(),))]),
}


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_fails_a_pin(name, monkeypatch):
    plant, checks = MUTATIONS[name]
    plant(monkeypatch)
    assert _some_pin_fails(checks()), f"no pin caught: {name}"


def test_pins_pass_without_a_mistake():
    checks = [c for _, make in MUTATIONS.values() for c in make()]
    assert not _some_pin_fails(checks)
