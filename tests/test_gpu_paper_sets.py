"""TH-BSGS and plain BSGS with resident plaintexts at the paper's Set-B and
Set-C parameters (Table V: N = 2^15 and 2^16, L + 1 = 16 and 32 primes of 54
bits, alpha = 8 and 12): every limb on the integer path, basis conversions
from 8, 12 and 13 source limbs, the fused middle layer over 24 and 44 limbs.
A banded matrix of 16 diagonals at the top level, split (2, 2, 4) and
(4, 4): the GPU's ciphertext equals the oracle's bit for bit."""
import numpy as np
import pytest

import workload as W
from gpu_common import LTCase, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["B", "C"])
def test_paper_set_banded_bit_exact(name):
    log("paper set", name)
    prm = W.params_paper_set(name)
    level = prm.max_level
    w = W.LTWorkload("set" + name, prm, level, W.banded_diagonals(51, prm.slots, range(16)),
                     W.input_vector(51, prm.slots), (2, 2, 4), (4, 4), 51)
    case = LTCase(w)
    for algo in ("th", "bsgs"):
        got, lvl, _ = case.gpu_out(algo)
        assert lvl == level - 1
        assert np.array_equal(got, case.oracle_out(algo)), algo
