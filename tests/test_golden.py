"""Numbers printed in the paper, stored under tests/golden with citations."""
import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def test_untruncated_count_is_central_binomial():
    g = json.load(open(os.path.join(HERE, "golden", "paper_numbers.json")))
    v = g["untruncated_strings_N12_open_J1_h0.5_dtau0.04_tau20"]["value"]
    # the saturated TFIM support has C(2n, n) strings (checked for small n
    # against the oracle in test_oracle_pins); the paper's N=12 count is C(24,12)
    assert v == math.comb(24, 12)
