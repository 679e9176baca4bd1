"""The C-ABI library loads here (no GPU needed), exports every symbol that
include/bse.h declares, and its host-only sign generator matches the input
generator's SplitMix64 bit for bit."""
import os
import re

import numpy as np
import pytest

from paper_2205_06690_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "bse.h")).read()
    return sorted(set(re.findall(r"\b(bse_[a-z_A-Z]+)\s*\(", txt)))


def test_header_symbols_exported():
    from paper_2205_06690_amd import bse
    decl = _declared()
    assert len(decl) >= 14
    for name in decl:
        assert hasattr(bse.LIB, name), name
    assert set(decl) == set(bse.EXPORTS)


def test_generate_signs_matches_inputs():
    from paper_2205_06690_amd import bse
    for seed, L, n in [(0, 10, 8), (1, 10, 120), (2**63 + 12345, 7, 33)]:
        assert np.array_equal(bse.generate_signs(seed, L, n), inputs.stochastic_signs(seed, L, n))


def test_argument_errors_without_device():
    from paper_2205_06690_amd import bse
    with pytest.raises(bse.BseError) as e:
        bse.generate_signs(0, 0, 5)
    assert e.value.code == bse.BSE_ERR_ARG
