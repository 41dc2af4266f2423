"""Golden fixture (tests/golden/edt_7x6x5.txt, written by make_golden.py
from the oracle only): the stored values are re-derived by exhaustive search
over the sites, and the oracle must still produce them."""
import os

import numpy as np
import pytest

from oracle.brute import brute_edt
from tests.golden import make_golden

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load():
    rows = [l.split() for l in open(os.path.join(HERE, "edt_7x6x5.txt")) if not l.startswith("#")]
    a = np.array(rows, dtype=np.int64)
    return a[:, 1].reshape(make_golden.SHAPE), a[:, 2].reshape(make_golden.SHAPE)


def test_fixture_matches_definition():
    d2, site = load()
    bd, bs = brute_edt(make_golden.build())
    assert np.array_equal(d2, bd) and np.array_equal(site, bs)


def test_oracle_reproduces_fixture(oracle_lib):
    d2, site = load()
    od, os_ = oracle_lib.edt(make_golden.build())
    assert np.array_equal(od, d2) and np.array_equal(os_, site)


@pytest.mark.gpu
def test_device_reproduces_fixture():
    from tests.gpu_util import gpu_edt
    d2, site = load()
    gd, gs = gpu_edt(make_golden.build())
    assert np.array_equal(gd, d2) and np.array_equal(gs, site)
