"""Host-side arithmetic of the solver comparison (no GPU): the shift-averaged LLR
term against the oracle's blocked LLR value at every shift."""

import numpy as np

from oracle import t2s as O
from paper_1809_04195_amd.solver_compare import llr_mean_over_shifts


def test_llr_mean_over_shifts_matches_oracle():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 16, 24)) + 1j * rng.standard_normal((3, 16, 24))
    b = 4
    want = np.mean([O.llr_value(x, (sy, sz), b) for sy in range(b) for sz in range(b)])
    assert abs(llr_mean_over_shifts(x, b) - want) < 1e-10 * want
