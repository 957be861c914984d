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
