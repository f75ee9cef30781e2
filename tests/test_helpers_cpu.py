"""The parity gate itself (tests/helpers.rel_err): a wrong tile inside a
large output fails it even where the whole-array relative Frobenius error
stays under the BF16 bound, while rounding-sized noise passes."""
import numpy as np

from helpers import TOL, rel_err, rel_fro, row_rel


def _core(seed=0, shape=(512, 16, 256)):
    return np.random.RandomState(seed).standard_normal(shape)


def test_wrong_tile_fails_row_gate():
    want = _core()
    got = want.copy()
    # one 16 x 16 tile of one mode slice replaced by values of the same size
    got[32:48, 5, 64:80] = np.random.RandomState(1).standard_normal((16, 16))
    assert rel_fro(got, want) < TOL["bf16"]        # invisible to the norm
    assert rel_err(got, want) > 5 * TOL["bf16"]    # caught by the rows


def test_single_wrong_entry_fails_fp32_gate():
    want = _core(2, (64, 4096))
    got = want.copy()
    got[17, 1234] += 0.01
    assert rel_fro(got, want) < TOL["f32"] * 100
    assert rel_err(got, want) > TOL["f32"]


def test_rounding_noise_passes():
    want = _core(3)
    got = want * (1 + 2.0 ** -9 * np.random.RandomState(4).uniform(-1, 1, want.shape))
    assert rel_err(got, want) < TOL["bf16"] / 4
    got32 = want.astype(np.float32).astype(np.float64)
    assert rel_err(got32, want) < TOL["f32"] / 10


def test_small_rows_and_zero_rows():
    want = _core(5, (128, 64))
    want[7] = 0.0
    want[9] *= 1e-6
    got = want.copy()
    assert row_rel(got, want) == 0.0
    # a small row measured against the RMS row norm: noise of that size passes
    got[9] += 1e-6 * np.random.RandomState(6).standard_normal(64)
    assert row_rel(got, want) < 1e-5
    # a wrong zero row fails
    got[7, 3] = 0.5
    assert row_rel(got, want) > TOL["bf16"]


def test_rows_merge_trailing_axes():
    # rows hold at least 64 entries: (8, 4, 4) merges into rows of 128
    want = _core(7, (8, 8, 4, 4))
    got = want.copy()
    got[3, 2, 1, 1] += 1.0
    assert row_rel(got, want) > 0.05
    assert rel_err(want, want) == 0.0
