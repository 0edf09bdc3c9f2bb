"""The pins must catch plausible mistakes in the oracle.

Each mutant replaces one oracle function with a plausibly wrong version (on
the CPU, inside the test only) and runs the pins of test_oracle_pins; at
least one pin has to fail for every mutant.
"""
import contextlib

import numpy as np
import pytest

from oracle import nmf64
from tests import test_oracle_pins as pins


def _ratio(num, den):
    return nmf64.ratio(num, den)


def h_weight_squared(Vh, M, W, H, eps=nmf64.EPS_FLOOR):
    Y = W @ H
    return np.maximum(H * _ratio(W.T @ (M * M * Vh), W.T @ (M * M * Y)), eps)


def h_den_unweighted(Vh, M, W, H, eps=nmf64.EPS_FLOOR):
    Y = W @ H
    return np.maximum(H * _ratio(W.T @ (M * Vh), W.T @ Y), eps)


def h_swapped(Vh, M, W, H, eps=nmf64.EPS_FLOOR):
    Y = W @ H
    return np.maximum(H * _ratio(W.T @ (M * Y), W.T @ (M * Vh)), eps)


def w_num_unweighted(Vh, M, W, H, eps=nmf64.EPS_FLOOR):
    Y = W @ H
    return np.maximum(W * _ratio(Vh @ H.T, (M * Y) @ H.T), eps)


def w_square_exponent(Vh, M, W, H, eps=nmf64.EPS_FLOOR):
    Y = W @ H
    return np.maximum(W * _ratio((M * Vh) @ H.T, (M * Y) @ H.T) ** 2, eps)


def objective_weight_squared(Vh, M, W, H):
    R = np.asarray(Vh, float) - np.asarray(W, float) @ np.asarray(H, float)
    return float(np.sum(np.asarray(M, float) ** 2 * R * R))


def ratio_zero_den_zero(num, den):
    num = np.asarray(num, float)
    den = np.asarray(den, float)
    out = np.zeros_like(num)
    nz = den > 0
    out[nz] = num[nz] / den[nz]
    return out


def prep_keeps_masked(V, M):
    V = np.asarray(V, float)
    M = np.asarray(M, float)
    return V.copy(), M, 0


_orig_build = nmf64.build_basis


def build_jacobi(V, M, W0, H0, iters, eps=nmf64.EPS_FLOOR, normalize=False, history=True):
    Vh, Mw, _ = nmf64.prep(V, M)
    W, H = np.asarray(W0, float).copy(), np.asarray(H0, float).copy()
    J = []
    for _ in range(iters):
        J.append(nmf64.objective(Vh, Mw, W, H))
        Hn = nmf64.update_H(Vh, Mw, W, H, eps)
        W = nmf64.update_W(Vh, Mw, W, H, eps)  # old H
        H = Hn
    J.append(nmf64.objective(Vh, Mw, W, H))
    return W, H, np.array(J)


def project_num_unmasked(T, MT, H, C0, iters, eps=nmf64.EPS_FLOOR):
    Th, MTw, _ = nmf64.prep(T, MT)
    H = np.asarray(H, float)
    C = np.asarray(C0, float).copy()
    num = Th @ H.T
    for _ in range(iters):
        den = (MTw * (C @ H)) @ H.T
        C = np.maximum(C * nmf64.ratio(num, den), eps)
    return C


def frame_objective_weight_squared(T, MT, H, C):
    Th, MTw, _ = nmf64.prep(T, MT)
    R = Th - np.asarray(C, float) @ np.asarray(H, float)
    return np.sum(MTw * MTw * R * R, axis=1)


def frame_objective_no_prep(T, MT, H, C):
    R = np.asarray(T, float) - np.asarray(C, float) @ np.asarray(H, float)
    return np.sum(np.asarray(MT, float) * R * R, axis=1)


def frame_objective_transposed_sum(T, MT, H, C):
    Th, MTw, _ = nmf64.prep(T, MT)
    R = Th - np.asarray(C, float) @ np.asarray(H, float)
    return np.sum(MTw * R * R, axis=0)[: Th.shape[0]]


def subtract_ignores_scale(T, MT, H, C, scale=None):
    return _orig_subtract(T, MT, H, C, None)


def subtract_scales_data(T, MT, H, C, scale=None):
    T, MT = np.asarray(T, float), np.asarray(MT, float)
    model = np.asarray(C, float) @ np.asarray(H, float)
    s = np.ones(T.shape[0]) if scale is None else np.asarray(scale, float)
    resid = s[:, None] * T - model
    resid[MT == 0] = np.nan
    return model, resid


def subtract_no_nan(T, MT, H, C, scale=None):
    T = np.asarray(T, float)
    model = np.asarray(C, float) @ np.asarray(H, float)
    s = np.ones(T.shape[0]) if scale is None else np.asarray(scale, float)
    return model, T - s[:, None] * model


def stop_test_absolute(J, t, check_every, tol):
    c = int(check_every)
    return c > 0 and t >= c and t % c == 0 and (J[t - c] - J[t]) < tol


def stop_test_off_by_one(J, t, check_every, tol):
    c = int(check_every)
    return c > 0 and t > c and (t - 1) % c == 0 and (J[t - 1 - c] - J[t - 1]) / J[t - 1 - c] < tol


_orig_subtract = nmf64.subtract

MUTANTS = {
    "frame objective with squared weights": ("frame_objective", frame_objective_weight_squared),
    "frame objective keeps masked data": ("frame_objective", frame_objective_no_prep),
    "frame objective summed over the wrong axis": ("frame_objective",
                                                   frame_objective_transposed_sum),
    "subtraction ignores the scale": ("subtract", subtract_ignores_scale),
    "subtraction scales the data instead of the model": ("subtract", subtract_scales_data),
    "subtraction keeps masked residuals": ("subtract", subtract_no_nan),
    "stop test on the absolute decrease": ("stop_test", stop_test_absolute),
    "stop test one iteration late": ("stop_test", stop_test_off_by_one),
    "H-rule with squared weights": ("update_H", h_weight_squared),
    "H-rule denominator without weights": ("update_H", h_den_unweighted),
    "H-rule numerator/denominator swapped": ("update_H", h_swapped),
    "W-rule numerator without weights": ("update_W", w_num_unweighted),
    "W-rule ratio squared": ("update_W", w_square_exponent),
    "objective with squared weights": ("objective", objective_weight_squared),
    "zero denominator zeroes the factor": ("ratio", ratio_zero_den_zero),
    "masked data not removed": ("prep", prep_keeps_masked),
    "W-rule uses the old H (Jacobi order)": ("build_basis", build_jacobi),
    "projection numerator ignores weights": ("project", project_num_unmasked),
}


def _pin_suite():
    """Pins run against the (possibly mutated) oracle, as (name, thunk)."""
    yield "hand-worked objective", pins.test_objective_hand_worked_value
    for s in range(8):
        yield f"monotone {s}", lambda s=s: pins.test_monotone_each_half_step(s)
    yield "planted recovery", lambda: pins.test_planted_exact_low_rank_recovered(0)
    yield "fixed point", pins.test_planted_fixed_point
    yield "rank-1 SVD", pins.test_rank1_unweighted_reaches_svd
    for s in range(2):
        yield f"H-rule NNLS {s}", lambda s=s: pins.test_H_rule_alone_reaches_columnwise_nnls(s)
        yield f"W-rule NNLS {s}", lambda s=s: pins.test_W_rule_alone_reaches_rowwise_nnls(s)
    for s in range(3):
        yield f"projection NNLS {s}", lambda s=s: pins.test_projection_limit_is_bruteforce_nnls(s)
    yield "projection K=1", pins.test_projection_k1_one_step_closed_form
    yield "masked garbage", pins.test_masked_garbage_is_ignored
    yield "fully masked", pins.test_fully_masked_row_and_column_keep_factors
    yield "prep flags", pins.test_prep_flags_bad_data_under_weight
    yield "frame objective by hand", pins.test_frame_objective_hand_worked
    yield "frame objective = NNLS cost", pins.test_frame_objective_equals_nnls_cost
    yield "subtraction by hand", pins.test_subtract_hand_worked
    yield "stop test by hand", pins.test_stop_test_hand_worked
    yield "tolerant build", pins.test_build_basis_tol_stops_at_the_rule


@contextlib.contextmanager
def _patched(name, fn):
    orig = getattr(nmf64, name)
    setattr(nmf64, name, fn)
    try:
        yield
    finally:
        setattr(nmf64, name, orig)


def test_pins_pass_on_the_real_oracle():
    for name, thunk in _pin_suite():
        thunk()


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_each_mutant_is_caught(mutant):
    attr, fn = MUTANTS[mutant]
    caught = []
    with _patched(attr, fn):
        for name, thunk in _pin_suite():
            try:
                with np.errstate(all="ignore"):
                    thunk()
            except (AssertionError, ValueError, FloatingPointError, np.linalg.LinAlgError):
                caught.append(name)
    assert caught, f"no pin catches: {mutant}"
