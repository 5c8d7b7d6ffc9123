"""The CPU oracle against what the paper and the mathematics fix (no GPU)."""
import numpy as np
import pytest

import oracle
from paper_2507_10424_amd import workloads as wl
from oracle_pins import ALL_PINS, codebook, read_tanner_golden


@pytest.mark.parametrize("pin", ALL_PINS, ids=[p.__name__ for p in ALL_PINS])
def test_pin(pin, orc):
    pin(orc)


def test_paper_tanner_fixture():
    """Sec. II-A example: the index sets give a (3,6)-regular H of GF(2)
    rank 5 (32 codewords, minimum distance 4); the printed indicator vectors
    agree with the index sets except check 3, which repeats check 1."""
    sets, vecs = read_tanner_golden()
    H = wl.paper_tanner_example()
    for i, s in enumerate(sets):
        assert sorted(np.nonzero(H[i])[0] + 1) == s
        if i != 2:
            assert list(H[i]) == vecs[i]
    assert vecs[2] == vecs[0] and list(H[2]) != vecs[2]
    assert np.all(H.sum(0) == 3) and np.all(H.sum(1) == 6)
    book = codebook(H)
    assert book.shape[0] == 32
    assert int(book[1:].sum(1).min()) == 4
    enc = wl.gf2_encoder(H)
    assert enc.rank == 5


# Planted mistakes in copies of the oracle (compiled with -DORACLE_MUTANT=k):
# 1 channel term dropped from the bit update, 2 no extrinsic subtraction,
# 3 own sign kept in the sign product, 4 own magnitude kept in the minimum,
# 5 slicer polarity flipped, 6 no pre-loop codeword test, 7 operands of the
# extrinsic subtraction swapped.
MUTANTS = [1, 2, 3, 4, 5, 6, 7]


@pytest.mark.parametrize("mutant", MUTANTS)
def test_pins_catch_planted_mistake(mutant, tmp_path):
    path = oracle.build_oracle(mutant=mutant, out=str(tmp_path / f"liboracle_m{mutant}.so"))
    bad = oracle.Oracle(path)
    failed = []
    for pin in ALL_PINS:
        try:
            pin(bad)
        except (AssertionError, ValueError):
            failed.append(pin.__name__)
    assert failed, f"no pin catches mutant {mutant}"
