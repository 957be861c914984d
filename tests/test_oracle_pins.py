"""The FP64 oracle against facts the paper and mathematics fix (CPU only)."""

import pytest

import oracle_pins as P  # noqa: E402


@pytest.mark.parametrize("R", [2, 4, 32, 128])
def test_cell_rule_matches_exact_box_membership(R):
    P.check_cell_rule(R)


def test_intermediate_tails_zeroed_is_textbook_mlp():
    P.check_textbook_mlp()


def test_multiplicative_tail_is_appendix_quadratic_form():
    P.check_quadratic_form()


def test_exit_at_k_equals_truncated_network():
    P.check_truncation()


def test_output_accumulates_tails():
    P.check_accumulation()


def test_matches_scalar_twin_on_tiny_grid():
    P.check_scalar_twin()


def test_matches_mpmath_50_digits():
    P.check_mpmath()


def test_lod_clamp_far_field_and_full_map():
    P.check_lod_and_far()


def test_gradient_matches_torch_autograd():
    P.check_gradient_autograd()


def test_gradient_matches_central_differences():
    P.check_gradient_fd()


# network-depth map construction (Sec. 3.2, Eq. 5-7)

def test_required_depth_is_eq5_written_out():
    P.check_required_depth_definition()


def test_required_depth_hand_cases():
    P.check_required_depth_extremes()


def test_required_depth_range_and_monotone_in_r():
    P.check_required_depth_monotone()


def test_vanishing_tails_cap_the_depth():
    P.check_vanishing_tails()


def test_samples_are_the_512_grid_cell_centres():
    P.check_sample_lattice()


def test_map_matches_brute_force_scalar_twin():
    P.check_construct_brute_force()


# map-free dynamic early exit (Sec. 4.4 ablation)

def test_dynamic_exit_is_the_rule_written_out():
    P.check_dynamic_definition()


def test_dynamic_exit_hand_cases():
    P.check_dynamic_hand_cases()


def test_dynamic_monotone_and_tails_sum_to_outputs():
    P.check_dynamic_monotone_and_tails()


def test_dynamic_exit_after_last_live_tail():
    P.check_dynamic_vanishing_tails()


def test_dynamic_matches_scalar_twin():
    P.check_dynamic_scalar_twin()


# sparse network-depth octree (Sec. 3.2, Eq. 5-7)

def test_octree_matches_recursive_scalar_twin():
    P.check_octree_brute_force()


def test_octree_closed_form_constant_models():
    P.check_octree_constant_models()


def test_octree_invariants():
    P.check_octree_invariants()


def test_octree_lookup_lands_in_containing_leaf():
    P.check_octree_lookup()


# FINER backbone (SAND-FINER, Sec. 4.1; the activation is FINER's own)

def test_finer_zeros_extrema_and_odd_symmetry():
    P.check_finer_roots()


def test_activation_slopes_match_central_differences():
    P.check_finer_slope()


@pytest.mark.parametrize("check", ["scalar_twin", "mpmath", "truncation", "gradient_autograd",
                                   "gradient_fd"])
def test_finer_network(check):
    getattr(P, "check_" + check)(activation="finer")
