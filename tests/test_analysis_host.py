"""Host-side logic of the analysis module against the oracle (no GPU).

The chaotic optimum of App. B: the library's closed form must equal the
oracle's eps_opt (itself pinned against the Porter-Thomas truncation in
test_oracle_pins.py) everywhere it is used, including the exact regime where
4 chi >= 2^(N/2) and the error is 0.
"""
import pytest

from paper_2207_05612_amd import analysis
from oracle import chaotic


@pytest.mark.parametrize("chi", [1, 4, 16, 64, 256, 1024])
@pytest.mark.parametrize("n_qubits", [12, 20, 28, 32, 54])
@pytest.mark.parametrize("depth", [1, 4, 8, 20])
def test_chaotic_optimum_matches_the_oracle(chi, n_qubits, depth):
    want = max(chaotic.eps_opt(chi, n_qubits, depth), 0.0)
    got = analysis.chaotic_optimum_error(chi, n_qubits, depth)
    assert abs(got - want) <= 1e-12 * max(1.0, abs(want))


def test_printed_closed_form_is_not_used():
    # 28 qubits, chi 64, depth 4: the derivation gives 7.16 %, the printed form 14.85 %
    assert abs(analysis.chaotic_optimum_error(64, 28, 4) - 0.0715750858) < 1e-9


def test_error_rate_definition():
    assert analysis.error_rate(1.0, 10) == 0.0
    assert analysis.error_rate(0.5, 0) == 0.0
    assert abs(analysis.error_rate(0.25, 2) - 0.5) < 1e-15
