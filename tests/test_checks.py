"""The amplitude comparison of the GPU parity tests, on CPU data.

Reference amplitudes come from the oracle's state vector of a small circuit;
the mistakes are planted in copies of them here, on the CPU.
"""

import numpy as np

from checks import K_MAX, assert_close, errors
from oracle import circuit as OC, statevector as SV
from workloads import circuits as W


def _ref():
    return SV.simulate(OC.parse(W.random_grid_circuit(4, 4, 10, 0)))


def test_rounding_noise_passes():
    ref = _ref()
    rng = np.random.default_rng(0)
    rms = np.linalg.norm(ref) / np.sqrt(ref.size)
    noise = (rng.standard_normal(ref.size) + 1j * rng.standard_normal(ref.size)) * (2e-6 * rms / np.sqrt(2))
    e = assert_close(ref + noise, ref, 1e-5)
    assert e["norm"] < 1e-5 and e["max_over_rms"] < K_MAX * 1e-5


def test_one_wrong_amplitude_fails_the_element_bound_only():
    ref = _ref()
    bad = ref.copy()
    rms = np.linalg.norm(ref) / np.sqrt(ref.size)
    bad[12345] += 1e-3 * rms  # one amplitude off by 0.1 % of rms over 2^16 values
    e = errors(bad, ref)
    assert e["norm"] < 1e-5  # the norm-wise bound alone would pass it
    try:
        assert_close(bad, ref, 1e-5)
    except AssertionError as ex:
        assert "max |a - ref|" in str(ex)
    else:
        raise AssertionError("a single wrong amplitude passed")


def test_swapped_index_bit_fails():
    ref = _ref()
    idx = np.arange(ref.size)
    swapped = ref[idx ^ (1 << 15)]  # top index bit flipped
    try:
        assert_close(swapped, ref, 1e-4)
    except AssertionError:
        pass
    else:
        raise AssertionError("a flipped index bit passed")
