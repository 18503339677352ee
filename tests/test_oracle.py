"""The FP64 oracle checked against the paper's Eq. (1) and mathematics (CPU)."""
import pytest

import oracle
import oracle_pins as P


def test_golden_worked_examples_naive():
    P.pin_golden(oracle.dft3d_naive)


def test_golden_worked_examples_fft():
    P.pin_golden(oracle.fft3d)


def test_closed_forms_naive():
    P.pin_closed_forms(oracle.dft3d_naive)


def test_closed_forms_fft():
    P.pin_closed_forms(oracle.fft3d, shapes=((4, 4, 4), (3, 5, 2), (6, 2, 5), (16, 9, 10)))


def test_naive_matches_numpy_witness():
    P.pin_naive_vs_numpy()


def test_fft_matches_bruteforce():
    P.pin_fft_vs_naive()


def test_fft_matches_numpy_witness():
    P.pin_fft_vs_numpy()


def test_invariants():
    P.pin_invariants()


def test_fp16_rounding():
    P.pin_fp16_rounding()


def test_bf16_rounding():
    P.pin_bf16_rounding()


def test_scaled16_rule():
    P.pin_q16_rule()


def test_energy_and_gradient():
    P.pin_energy()


def test_rejects_bad_arguments():
    import numpy as np
    with pytest.raises(RuntimeError):
        oracle.fft3d(np.zeros((2, 2, 2), complex), sign=0)
    with pytest.raises(RuntimeError):
        oracle.fft3d(np.zeros((2, 2, 2), complex), order=(0, 0, 1))


def test_real_transforms():
    P.pin_real()


def test_apply_potential():
    P.pin_apply_potential()


def test_density():
    P.pin_density()
