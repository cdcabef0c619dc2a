"""Pins for the oracle's bfloat16 / E4M3FN rounding against torch's CPU casts."""
import numpy as np
import torch

from oracle.rounding import round_bf16, round_e4m3


def test_bf16_matches_torch_cast():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-3, 2000), rng.normal(0, 1e4, 2000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, -3.0e-5])]).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_bf16(x.astype(np.float64)), ref)


def test_e4m3_matches_torch_cast_in_range():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-448, 448, 20000), rng.normal(0, 0.01, 5000), rng.normal(0, 1, 5000),
                        np.array([0.0, 448.0, -448.0, 2 ** -6, 2 ** -9, 1.5 * 2 ** -9, 0.0625 * 17])])
    x = x.astype(np.float32)
    ref = torch.tensor(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_e4m3(x.astype(np.float64)), ref)


def test_e4m3_saturates():
    np.testing.assert_array_equal(round_e4m3(np.array([500.0, -1e6, 449.0])), [448.0, -448.0, 448.0])


def test_grids():
    # bf16 keeps 8 significant bits: 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8 -> 1 + 2^-6
    assert round_bf16(np.array([1 + 2 ** -8]))[0] == 1.0
    assert round_bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6
    # e4m3 keeps 4 significant bits: 1 + 2^-4 ties to 1.0, 1 + 3*2^-4 ties to 1.25
    assert round_e4m3(np.array([1 + 2 ** -4]))[0] == 1.0
    assert round_e4m3(np.array([1 + 3 * 2 ** -4]))[0] == 1.25
